// PBD-R solver substep on gfx950 (MI355X).
//
// One substep of Alg. 1 of "Physically Accurate Rigid-Body Dynamics in
// Particle-Based Simulation" (arXiv 2603.14634) as a chain of kernels on one
// stream:
//
//   predict_keys   integration step (Alg. 1, first loop) and hash-grid key of
//                  every particle; from the second substep of a call on, it
//                  first folds the previous substep's result into the state
//                  (x += dX, v = V)
//   radix_hist     counts of every 8-bit digit of the keys
//   radix x P      stable LSD radix sort of (key, id), one digit per pass:
//                  tile counts, a scan per digit over the tiles, then each
//                  tile ranks its keys by ballots and writes them in place;
//                  the last pass also writes sorted copies of the FP32
//                  predicted positions and body ids
//   cells          per-key table from the sorted keys, written for occupied
//                  keys only and tagged with the substep: first and end slot,
//                  body signature (the key's single body, or "mixed")
//   neighbours     walks particles in key order: 27-cell stencil (skipping
//                  keys that hold only the particle's own body), FP32
//                  predicate, ascending lists
//   iterate x K    bodies packed into workgroups, whole waves per body, one
//                  particle per lane: particle contacts, shape matching
//                  (Sec. III-C, Mueller et al. 2005), incremental velocity update
//                  (Sec. III-B) and momentum conservation constraint (Sec.
//                  III-C, Eqs. (4)-(5))
//   finalize       x = X_init + (X_K - X_init), v = V_K; non-finite check
//
// Numerics.  Inside a substep positions are carried as the displacement
// delta = X_i - X_init (small magnitude), so FP32 resolves corrections far
// below the ulp of world coordinates: pair separations are formed as
// (X_init,p - X_init,q) + (delta_p - delta_q) (the first difference is exact
// for nearby particles), and body-relative coordinates are formed against an
// anchor particle of the body.  Velocities follow the paper's incremental
// update V_{i+1} = V_i + dX / dt.  Per-body sums are fixed-order reductions
// (lane swaps and DPP within a wave, then the wave partials in wave order), so results are
// bitwise reproducible.
//
// The neighbour-search decisions (key, predicate) are taken in FP32 with no
// contraction, op by op, so they are reproducible by any IEEE FP32 evaluation
// of the same sequence.
#include "pbdr_device.h"
#include "pbdr_math.h"

#include <hip/hip_ext.h>

#include <math.h>

namespace pbdr {
namespace {

using namespace dev;

constexpr int kWaves = kBlock / 64;

// Workgroup i of a launch runs on XCD i % 8 (each XCD has its own L2).  This
// gives XCD x the contiguous range of logical workgroups x*q + min(x, r) ..
// (q + [x < r] of them, q = n / 8, r = n % 8), a bijection of [0, n): work that
// is adjacent in the logical order (neighbouring bodies, which share cache
// lines at their ends and read each other's positions; neighbouring keys)
// then meets in one L2.
__device__ inline int xcd_block()
{
    const uint32_t nb = gridDim.x, q = nb / 8u, r = nb % 8u, x = blockIdx.x % 8u;
    return (int)(x * q + (x < r ? x : r) + blockIdx.x / 8u);
}

// The same renumbering of workgroups first .. gridDim.x - 1 among themselves
// (the XCD of their residue class is rotated by `first`, each class still on
// one XCD).
__device__ inline int xcd_block_from(int first)
{
    const uint32_t hb = blockIdx.x - (uint32_t)first, nb = gridDim.x - (uint32_t)first, q = nb / 8u, r = nb % 8u,
                   x = hb % 8u;
    return first + (int)(x * q + (x < r ? x : r) + hb / 8u);
}

// ---------------------------------------------------------------------------
// integration step + keys
// ---------------------------------------------------------------------------

// MULTI: multi-scene mode (Scene::pscene set); a separate instance, so that
// the single-scene kernels carry none of its checks.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_predict_keys(Scene s, StepConsts c, int fold_src)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    // the key sort of this substep starts from zero digit counts
    if (i < kMaxRadixPasses * kRadixBins) s.hist[i] = 0u;
    // a new substep: fresh tags for the key table and one-launch iterations
    // (no other thread of this launch reads the epoch)
    if (i == 0) s.counters->epoch += 1u;
    if (i >= s.n_sort) return;
    const size_t n = (size_t)s.n;
    const MultiScene* ms = nullptr;
    if (MULTI) {                       // this particle's scene, if stepped
        const int32_t sc = s.pscene[i];
        if (sc < 0 || !s.mscene[sc].active) {
            s.key[i] = s.T;            // sorts after every stepped particle
            return;
        }
        ms = &s.mscene[sc];
    }
    const float* g = ms ? ms->g : c.g;
    float xt[3];
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
        const size_t j = k * n + i;
        float x, v;
        if (fold_src >= 0) {           // end of the previous substep of this frame
            x = s.x0[j] + s.dl[fold_src][j];
            v = s.vel[fold_src][j];
            finite = finite && isfinite(x) && isfinite(v);
        } else {                       // first substep of a frame: the committed state
            x = s.x[j];
            v = s.v[j];
        }
        s.x0[j] = x;                   // X_init of this substep
        const float a = g[k] + (s.accel ? s.accel[j] : 0.0f);
        const float dv = c.h * a;
        const float vt = v + dv;
        const float dx = c.h * vt;
        xt[k] = x + dx;
        s.xt[j] = xt[k];
        s.dl[0][j] = dx;      // delta_0 = X~ - X_init
        s.vel[0][j] = vt;     // V_0 = V~
    }
    if (!finite) atomicOr(&s.counters->err, kErrNonFinite);
    s.key[i] = (ms ? ms->key_base : 0u) + morton(cell_axis(xt[0], c.origin[0], c.inv_cell),
                                                 cell_axis(xt[1], c.origin[1], c.inv_cell),
                                                 cell_axis(xt[2], c.origin[2], c.inv_cell),
                                                 ms ? ms->key_mask : c.key_mask);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (key, id), 8-bit digits.  One histogram of all
// digits of all passes first; then per pass three launches: each tile counts
// its digits, one scan per digit over the tiles turns the counts into output
// positions, and each tile ranks its keys and writes them there.  No
// workgroup waits for another.
// ---------------------------------------------------------------------------

// Inclusive prefix sum over the lanes of a wave: shifts by 1, 2, 4, 8 within
// each 16-lane row (DPP, lanes without a source add 0), then each row adds the
// last lane of the rows before it (row broadcasts).
__device__ inline uint32_t wave_inclusive_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

// Exclusive prefix sum of one value per thread over the workgroup (kBlock
// threads); `tmp` holds kWaves words of LDS.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t incl = wave_inclusive_scan(v);
    if (lane == 63) tmp[wave] = incl;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < kWaves; ++w)
        if (w < wave) before += tmp[w];
    __syncthreads();                  // tmp may be reused at once
    return before + incl - v;
}


// Digit counts of every pass over all keys: each workgroup of THREADS threads
// counts a chunk of 16 THREADS keys in LDS (16 consecutive keys per thread,
// equal digits of a run counted once) and adds its non-zero counts to the
// global table.  It also writes the first pass's per-tile counts (the tiles
// of a chunk, in the keys' input order), so that pass needs no counting
// launch of its own.
template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_radix_hist(Scene s)
{
    constexpr int kHistChunk = 16 * THREADS;
    constexpr int kMaxChunkTiles = kHistChunk / (kBlock * 4);
    __shared__ uint32_t h[kMaxRadixPasses * kRadixBins];
    __shared__ uint32_t ht[kMaxChunkTiles * kRadixBins];
    const int P = s.radix_passes;
    const int tile_keys = kBlock * (int)s.radix_items;
    const int chunk_tiles = kHistChunk / tile_keys;
    for (int t = threadIdx.x; t < P * kRadixBins; t += THREADS) h[t] = 0u;
    for (int t = threadIdx.x; t < chunk_tiles * kRadixBins; t += THREADS) ht[t] = 0u;
    __syncthreads();
    const size_t n = (size_t)s.n_sort;
    const size_t i0 = (size_t)blockIdx.x * kHistChunk + 16 * (size_t)threadIdx.x;
    uint32_t k[16];
    if (i0 + 16 <= n) {
        const uint4* src = reinterpret_cast<const uint4*>(s.key + i0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint4 q = src[u];
            k[4 * u] = q.x; k[4 * u + 1] = q.y; k[4 * u + 2] = q.z; k[4 * u + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) k[u] = i0 + u < n ? s.key[i0 + u] : 0u;
    }
    const int cnt = i0 >= n ? 0 : (int)min((size_t)16, n - i0);
    // the thread's 16 keys lie in one tile (16 divides the tile size)
    uint32_t* hp0 = &ht[(16 * (int)threadIdx.x / tile_keys) * kRadixBins];
    for (int p = 0; p < P; ++p) {
        const uint32_t sh = kRadixBits * p;
        uint32_t run_d = 0, run_n = 0;
        for (int u = 0; u < cnt; ++u) {
            const uint32_t d = (k[u] >> sh) & (kRadixBins - 1);
            if (run_n && d != run_d) {
                atomicAdd(&h[p * kRadixBins + run_d], run_n);
                if (p == 0) atomicAdd(&hp0[run_d], run_n);
                run_n = 0;
            }
            run_d = d;
            ++run_n;
        }
        if (run_n) {
            atomicAdd(&h[p * kRadixBins + run_d], run_n);
            if (p == 0) atomicAdd(&hp0[run_d], run_n);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P * kRadixBins; t += THREADS)
        if (h[t]) atomicAdd(&s.hist[t], h[t]);
    // the chunk's tiles: [digit][tile] like k_radix_count
    const uint32_t T = s.n_radix_tiles;
    for (int t = threadIdx.x; t < chunk_tiles * kRadixBins; t += THREADS) {
        const uint32_t tile = (uint32_t)blockIdx.x * (uint32_t)chunk_tiles + (uint32_t)(t / kRadixBins);
        if (tile < T) s.tile_off[(size_t)(t % kRadixBins) * T + tile] = ht[t];
    }
}

// Pass p, step 1: the digit counts of one tile (kBlock threads of ITEMS
// keys; thread t counts keys ITEMS t .. ITEMS t + ITEMS - 1 of the tile, equal
// digits of a run once) to tile_off[d][tile].
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_radix_count(Scene s, int p, const uint32_t* kin)
{
    static_assert(kBlock == kRadixBins, "one thread per digit");
    __shared__ uint32_t h[kRadixBins];
    const int tid = threadIdx.x;
    h[tid] = 0u;
    __syncthreads();
    const size_t n = (size_t)s.n_sort;
    const uint32_t tile = blockIdx.x;
    const size_t i0 = (size_t)tile * (kBlock * ITEMS) + (size_t)tid * ITEMS;
    uint32_t k[ITEMS];
    if (i0 + ITEMS <= n) {
        const uint4* src = reinterpret_cast<const uint4*>(kin + i0);
#pragma unroll
        for (int u = 0; u < ITEMS / 4; ++u) {
            const uint4 q = src[u];
            k[4 * u] = q.x; k[4 * u + 1] = q.y; k[4 * u + 2] = q.z; k[4 * u + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) k[u] = i0 + u < n ? kin[i0 + u] : 0u;
    }
    const int cnt = i0 >= n ? 0 : (int)min((size_t)ITEMS, n - i0);
    const uint32_t sh = kRadixBits * p;
    uint32_t run_d = 0, run_n = 0;
#pragma unroll
    for (int u = 0; u < ITEMS; ++u) {
        if (u >= cnt) break;
        const uint32_t d = (k[u] >> sh) & (kRadixBins - 1);
        if (run_n && d != run_d) {
            atomicAdd(&h[run_d], run_n);
            run_n = 0;
        }
        run_d = d;
        ++run_n;
    }
    if (run_n) atomicAdd(&h[run_d], run_n);
    __syncthreads();
    s.tile_off[(size_t)tid * s.n_radix_tiles + tile] = h[tid];
}

// Pass p, step 2: workgroup d turns digit d's tile counts into the first
// output position of the digit in each tile: the count of smaller digits over
// all keys plus the counts of d in earlier tiles.
__global__ void __launch_bounds__(kBlock) k_radix_scan(Scene s, int p)
{
    __shared__ uint32_t tmp[kWaves];
    __shared__ uint32_t s_base, s_total;
    const int tid = threadIdx.x;
    const uint32_t d = blockIdx.x;
    const uint32_t below = block_exclusive_scan(s.hist[p * kRadixBins + tid], tmp);
    if ((uint32_t)tid == d) s_base = below;
    __syncthreads();
    uint32_t carry = s_base;
    const uint32_t T = s.n_radix_tiles;
    uint32_t* row = s.tile_off + (size_t)d * T;
    for (uint32_t t0 = 0; t0 < T; t0 += kBlock) {
        const uint32_t t = t0 + (uint32_t)tid;
        const uint32_t c = t < T ? row[t] : 0u;
        const uint32_t ex = block_exclusive_scan(c, tmp);
        if (t < T) row[t] = carry + ex;
        if (tid == kBlock - 1) s_total = ex + c;
        __syncthreads();
        carry += s_total;
        __syncthreads();
    }
}

// Pass p, step 3: keys kin (ids iin, or the key's index when iin is null) ->
// kout, iout, stable.  Item t of lane l of wave w is key w * 64 ITEMS + 64 t
// + l of the tile: each wave ranks its items in that order by matching equal
// digits across lanes with ballots, so ranks follow key order within the
// tile.  The tile's keys go through LDS in (digit, key order), so the slots
// of one digit are written to consecutive positions.  The last pass also
// writes each particle's predicted position and body to its sorted slot (sxt4).
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(Scene s, int p, const uint32_t* kin, const uint32_t* iin,
                                                          uint32_t* kout, uint32_t* iout)
{
    constexpr int TILE = kBlock * ITEMS;
    __shared__ uint32_t s_key[TILE], s_id[TILE];
    __shared__ uint32_t wcnt[kWaves][kRadixBins];   // per-wave digit counters, then wave offsets
    __shared__ uint32_t lstart[kRadixBins];         // first LDS slot of each digit in the tile
    __shared__ int32_t gshift[kRadixBins];          // output position - LDS slot, per digit
    __shared__ uint32_t tmp[kWaves];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = tid; t < kWaves * kRadixBins; t += kBlock) (&wcnt[0][0])[t] = 0u;
    __syncthreads();
    const uint32_t tile = blockIdx.x;
    const uint32_t n = (uint32_t)s.n_sort;
    const uint32_t sh = kRadixBits * p;
    const uint32_t first = tile * TILE + (uint32_t)wave * 64u * ITEMS + (uint32_t)lane;

    uint32_t k[ITEMS], id[ITEMS], r[ITEMS];
#pragma unroll
    for (int t = 0; t < ITEMS; ++t) {
        const uint32_t e = first + 64u * t;
        k[t] = e < n ? kin[e] : 0u;
        id[t] = e < n ? (iin ? iin[e] : e) : 0u;
    }
    // rank within the wave, item by item (each lane's items in key order)
#pragma unroll
    for (int t = 0; t < ITEMS; ++t) {
        const bool valid = first + 64u * t < n;
        const uint32_t d = (k[t] >> sh) & (kRadixBins - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        const uint32_t prior = valid ? wcnt[wave][d] : 0u;
        r[t] = prior + below;
        if (valid && lane == __ffsll((long long)peers) - 1) wcnt[wave][d] = prior + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // thread d: wave offsets and the tile's count of digit d
    const uint32_t d = (uint32_t)tid;
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t c = wcnt[w][d];
        wcnt[w][d] = total;
        total += c;
    }
    const uint32_t local = block_exclusive_scan(total, tmp);          // first slot of digit d in the tile
    lstart[d] = local;
    gshift[d] = (int32_t)s.tile_off[(size_t)d * s.n_radix_tiles + tile] - (int32_t)local;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < ITEMS; ++t) {
        if (first + 64u * t >= n) continue;
        const uint32_t dd = (k[t] >> sh) & (kRadixBins - 1);
        const uint32_t slot = lstart[dd] + wcnt[wave][dd] + r[t];
        s_key[slot] = k[t];
        s_id[slot] = id[t];
    }
    __syncthreads();
    const uint32_t in_tile = min((uint32_t)TILE, n - tile * TILE);
    const bool last = p == s.radix_passes - 1;
    const size_t ns = (size_t)s.n;
    for (uint32_t j = (uint32_t)tid; j < in_tile; j += kBlock) {
        const uint32_t kk = s_key[j], ii = s_id[j];
        const uint32_t pos = (uint32_t)((int32_t)j + gshift[(kk >> sh) & (kRadixBins - 1)]);
        if (pos >= n) {                // (counts and keys disagree: cannot happen)
            atomicOr(&s.counters->err, kErrInternal);
            continue;
        }
        kout[pos] = kk;
        iout[pos] = ii;
        if (last && kk < s.T)          // stepped particles (in multi-scene mode the others take key T)
            s.sxt4[pos] = make_float4(s.xt[ii], s.xt[ns + ii], s.xt[2 * ns + ii], __int_as_float(s.body[ii]));
    }
}

// Per-key table from the sorted keys: the first particle of each key writes
// the key's entry (first slot, end slot, body signature, substep).
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_cells(Scene s)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const int ng = MULTI ? s.n_active : s.n;     // sorted particles that are stepped
    if (j >= ng) return;
    const uint32_t key = s.skey[j];
    // (only after a sort that gave up can a key be out of range; the frame is
    // then discarded)
    if (key >= s.T || (j > 0 && s.skey[j - 1] == key)) return;
    const int32_t b = __float_as_int(s.sxt4[j].w);
    int e = j + 1;
    int32_t sig = b;                 // the one body of all the key's particles, or -2
    while (e < ng && s.skey[e] == key) {
        if (__float_as_int(s.sxt4[e].w) != b) sig = -2;
        ++e;
    }
    s.cells[key] = make_uint4((uint32_t)j, (uint32_t)e, (uint32_t)sig, s.counters->epoch);
}

// ---------------------------------------------------------------------------
// neighbour lists, one thread per particle in key order
// ---------------------------------------------------------------------------

// One candidate of particle i (list `lst`, slot k at lst[k * stride]): same
// body (which also excludes i) and the FP32 predicate, then an insertion that
// keeps the `cap` smallest ids in ascending order.  Lists are short (most
// particles have none), so they are kept in place in the output array.
__device__ __forceinline__ void nbr_consider(uint32_t* lst, size_t stride, int cap, uint32_t& count, int32_t pb,
                                             float px, float py, float pz, float r2, const float4 o,
                                             const uint32_t* sorted, uint32_t q)
{
    if (__float_as_int(o.w) == pb) return;
    if (!within(px, py, pz, o.x, o.y, o.z, r2)) return;
    const uint32_t id = sorted[q];        // (loaded only for a neighbour)
    const int m = (int)(count < (uint32_t)cap ? count : (uint32_t)cap);
    ++count;
    if (m == cap && id > lst[(size_t)(cap - 1) * stride]) return;
    int pos = (m == cap) ? cap - 1 : m;
    while (pos > 0 && lst[(size_t)(pos - 1) * stride] > id) {
        lst[(size_t)pos * stride] = lst[(size_t)(pos - 1) * stride];
        --pos;
    }
    lst[(size_t)pos * stride] = id;
}

// One thread per particle in key order.  The 27 keys are walked one z-layer
// of 9 at a time: the layer's table entries are loaded together, then the
// first candidate of each of its keys, so the loads of a layer are in flight
// together; further candidates of a key (rare with >= 8 keys per particle)
// follow.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_neighbours(Scene s, StepConsts c)
{
    const int blk = xcd_block();
    const int j = blk * kBlock + threadIdx.x;  // position in key order
    // multi-scene mode: the stepped particles come first in key order
    bool live = j < (MULTI ? s.n_active : s.n);
    const size_t n = (size_t)s.n;
    const int cap = c.nbr_cap;
    const uint32_t epoch = s.counters->epoch;
    uint32_t count = 0;
    const uint32_t i = live ? s.sorted[j] : 0u;
    uint32_t key_base = 0u, key_mask = c.key_mask;
    if (MULTI && live) {                // multi-scene mode: the particle's own scene table
        const int32_t sc = s.pscene[i];
        live = sc >= 0;                 // (false only after a sort that gave up)
        if (live) {
            key_base = s.mscene[sc].key_base;
            key_mask = s.mscene[sc].key_mask;
        }
    }
    if (live) {
        const float4 me = s.sxt4[j];
        const float px = me.x, py = me.y, pz = me.z;
        const int32_t pb = __float_as_int(me.w);
        const uint32_t cx = cell_axis(px, c.origin[0], c.inv_cell);
        const uint32_t cy = cell_axis(py, c.origin[1], c.inv_cell);
        const uint32_t cz = cell_axis(pz, c.origin[2], c.inv_cell);
        uint32_t* lst = s.nbr + i;
        // the spread (Morton) bits of the three cells along each axis, so
        // that each stencil key is two ORs
        uint32_t sx[3], sy[3], sz[3];
        for (int d = 0; d < 3; ++d) {
            sx[d] = spread3(cx + (uint32_t)(d - 1));
            sy[d] = spread3(cy + (uint32_t)(d - 1)) << 1;
            sz[d] = spread3(cz + (uint32_t)(d - 1)) << 2;
        }
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            uint32_t lo[9], hi[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                const uint32_t k = key_base + ((sx[u % 3] | sy[u / 3] | sz[dz]) & key_mask);
                const uint4 e = s.cells[k];
                lo[u] = e.x;
                // an entry of an earlier substep is an empty key, and a key
                // holding only this particle's body has no candidates
                hi[u] = (e.w != epoch || (int32_t)e.z == pb) ? e.x : e.y;
            }
            float4 o[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) o[u] = hi[u] > lo[u] ? s.sxt4[lo[u]] : me;
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                if (hi[u] > lo[u]) {
                    nbr_consider(lst, n, cap, count, pb, px, py, pz, c.search_r2, o[u], s.sorted, lo[u]);
                    for (uint32_t q = lo[u] + 1; q < hi[u]; ++q)
                        nbr_consider(lst, n, cap, count, pb, px, py, pz, c.search_r2, s.sxt4[q], s.sorted, q);
                }
            }
        }
        s.nbr_n[i] = count;
    }
    // statistics: this workgroup's own slot (no contention); the capacity
    // error is latched only when it happens
    __shared__ uint32_t st_max[kWaves];
    __shared__ unsigned long long st_sum[kWaves];
    uint32_t mx = count;
    unsigned long long sum = count;
    for (int off = 32; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off, 64));
        sum += __shfl_xor(sum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        st_max[threadIdx.x >> 6] = mx;
        st_sum[threadIdx.x >> 6] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t bm = 0;
        unsigned long long bs = 0;
        for (int w = 0; w < kWaves; ++w) {
            bm = max(bm, st_max[w]);
            bs += st_sum[w];
        }
        const int rows = min(kBlock, s.n - blk * kBlock);
        NbrStats& slot = s.nbr_stats[blk];
        slot.max_nbr = max(slot.max_nbr, bm);
        slot.sum += bs;
        slot.rows += (unsigned long long)rows;
        if (bm > (uint32_t)cap) atomicOr(&s.counters->err, kErrCapacity);
    }
}

// ---------------------------------------------------------------------------
// one Jacobi iteration (Alg. 1 loop body)
// ---------------------------------------------------------------------------

// Signed distance n . X_i - d of a particle from plane pl, in FP64 (the
// penetration r - e is formed from it before any rounding).
// Whether X_i = x0 + del lies clearly outside plane pl's contact range: the
// signed distance evaluated in FP32 exceeds r by more than 2^-20 of the
// magnitudes involved (several times the bound of that evaluation's
// rounding), so the FP64 distance below exceeds r as well and its test can
// be skipped without changing any result.  mag: |x0|_1 + |del|_1.
__device__ __forceinline__ bool plane_far(const StepConsts& c, int pl, const float* x0, const float* del, float mag)
{
    const float e = c.plane_n[pl][0] * (x0[0] + del[0]) + c.plane_n[pl][1] * (x0[1] + del[1]) +
                    c.plane_n[pl][2] * (x0[2] + del[2]) - c.plane_d[pl];
    return e > c.radius + 0x1p-20f * (mag + fabsf(c.plane_d[pl]));
}

__device__ __forceinline__ double plane_gap(const StepConsts& c, int pl, const float* x0, const float* del)
{
    double e = -c.plane_d_d[pl];
    for (int j = 0; j < 3; ++j) e += (double)c.plane_n[pl][j] * ((double)x0[j] + (double)del[j]);
    return e;
}

// Contact with a particle of another body (constraint (2)) from X_i: the
// mass-weighted split of the penetration, Coulomb friction from the relative
// displacement since X_init, and the pair weight of the averaging mode.  xq,
// dq: the partner's X_init and X_i - X_init; mq, nq: its mass and list length.
// The correction is sc * t (false: no contact).  Shared by all iteration
// kernels, with contraction limited to single expressions, so that they
// round alike.
__device__ __forceinline__ bool pair_terms(const StepConsts& c, uint32_t avg, float mu, const float* x0,
                                           const float* del, float m, uint32_t ni, const float* xq, const float* dq,
                                           float mq, uint32_t nq, float& sc, float* t)
{
#pragma clang fp contract(on)
    // separation, distance, penetration and normal in FP64: the separation
    // of two FP32 positions and the penetration 2r - l are exact or nearly so
    // there, and only the correction is rounded
    double d[3];
    float u[3];
    for (int j = 0; j < 3; ++j) {
        d[j] = ((double)x0[j] - (double)xq[j]) + ((double)del[j] - (double)dq[j]);
        u[j] = del[j] - dq[j];
    }
    const double l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(l2 > 0.0) || !(l2 < c.two_r_d * c.two_r_d)) return false;
    const double il = rsqrt64(l2);
    const double l = l2 * il;
    const float nx = (float)(d[0] * il), ny = (float)(d[1] * il), nz = (float)(d[2] * il);
    const float pen = (float)(c.two_r_d - l);
    const float alpha = mq * frcp(m + mq);          // w_p / (w_p + w_q)
    const float un = u[0] * nx + u[1] * ny + u[2] * nz;
    const float ux = u[0] - un * nx, uy = u[1] - un * ny, uz = u[2] - un * nz;
    const float ut2 = ux * ux + uy * uy + uz * uz;
    const float f = ut2 > 0.0f ? fminf(1.0f, mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
    float wgt = 1.0f;
    if (avg == 0u)
        wgt = frcp((float)(ni > nq ? ni : nq));
    else if (avg == 1u)
        wgt = frcp((float)ni);
    sc = alpha * wgt;
    t[0] = pen * nx - f * ux;
    t[1] = pen * ny - f * uy;
    t[2] = pen * nz - f * uz;
    return true;
}

__device__ __forceinline__ void pair_correction(const StepConsts& c, uint32_t avg, float mu, const float* x0,
                                                const float* del, float m, uint32_t ni, const float* xq,
                                                const float* dq, float mq, uint32_t nq, float* Cd)
{
#pragma clang fp contract(on)
    float sc, t[3];
    if (!pair_terms(c, avg, mu, x0, del, m, ni, xq, dq, mq, nq, sc, t)) return;
    for (int j = 0; j < 3; ++j) Cd[j] += sc * t[j];
}

// Sum of the per-wave partials (NV float4 per wave) of a body's waves w0 ..
// w0 + nw - 1, in wave order; the LDS reads of U waves are issued together.
template <int NV, int U>
__device__ inline void sum_wave_partials(const float4* red, int w0, int nw, float* T)
{
    for (int j = 0; j < 4 * NV; ++j) T[j] = 0.0f;
    for (int w = 0; w < nw; w += U) {
        float4 p[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int wu = w + u < nw ? w + u : nw - 1;
#pragma unroll
            for (int j = 0; j < NV; ++j) p[u][j] = red[(w0 + wu) * NV + j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (w + u >= nw) break;
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                T[4 * j] += p[u][j].x;
                T[4 * j + 1] += p[u][j].y;
                T[4 * j + 2] += p[u][j].z;
                T[4 * j + 3] += p[u][j].w;
            }
        }
    }
}

// The rotation of shape matching (FP32, orthogonal to a few 1e-7) made
// orthogonal to FP64 precision by one Newton step X <- (X + X^-T) / 2 (the
// iteration that converges to the orthogonal polar factor, quadratically);
// applied in FP64, so that it moves a body's goal rigidly: a rotation that is
// orthogonal only to 1e-7 would stretch a decimetre-sized body's goal shape
// by 1e-8 m.
// Each cofactor is formed where it is used (few FP64 values live at once).
__device__ __forceinline__ double cofactor64(const float* X, int a, int b, int c, int d)
{
    return (double)X[a] * (double)X[b] - (double)X[c] * (double)X[d];
}

__device__ inline void orthonormalise64(const float* X, double* Rd)
{
    // cofactor k of X (row-major): the (1, 1) minor pattern of cof3
    constexpr int kIdx[9][4] = {{4, 8, 5, 7}, {5, 6, 3, 8}, {3, 7, 4, 6}, {2, 7, 1, 8}, {0, 8, 2, 6},
                                {1, 6, 0, 7}, {1, 5, 2, 4}, {2, 3, 0, 5}, {0, 4, 1, 3}};
    double det = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) det += (double)X[k] * cofactor64(X, kIdx[k][0], kIdx[k][1], kIdx[k][2], kIdx[k][3]);
    // 1 / det (about 1): the FP32 reciprocal refined by two Newton steps,
    // each doubling its correct bits, to FP64 precision
    double id = (double)frcp((float)det);
#pragma unroll
    for (int k = 0; k < 2; ++k) id = __builtin_fma(id, __builtin_fma(-det, id, 1.0), id);
#pragma unroll
    for (int k = 0; k < 9; ++k)
        Rd[k] = 0.5 * ((double)X[k] + cofactor64(X, kIdx[k][0], kIdx[k][1], kIdx[k][2], kIdx[k][3]) * id);
}

// Shape matching's goal offset D = R q - (y - c) of one particle, y its
// position relative to the body's anchor (x0 - anchor + del).  The terms are
// body-sized (up to decimetres) while D is of the order of the contact
// corrections (micrometres), so it is formed in FP64: the products of FP32
// values and the anchor difference are exact there, and only the result is
// rounded.  In FP32 every particle's goal would carry a rounding of ~ulp(0.1 m)
// = 7e-9 m that no rigid motion absorbs, and resting contacts amplify such
// particle-level differences over the iterations.
// Rc: the body's R (row-major) and centre relative to the anchor, in FP64.
__device__ __forceinline__ void goal_offset(const double* Rc, const float* q, const float* x0, const float* anchor,
                                            const float* del, float* D)
{
    for (int a = 0; a < 3; ++a) {
        const double rq = Rc[3 * a] * (double)q[0] + Rc[3 * a + 1] * (double)q[1] + Rc[3 * a + 2] * (double)q[2];
        const double ya = ((double)x0[a] - (double)anchor[a]) + (double)del[a];
        D[a] = (float)(rq - (ya - Rc[9 + a]));
    }
}

// This wave's partial sums of shape matching, sum m y and sum m y q^T (12
// values), to LDS: in FP32 (red32), or in FP64 (red64) when `wide`.
// y: the particle's position relative to the body's anchor, (x0 - anchor) +
// del, in FP32; a wide body's sums take it in FP64 (exact there).
template <bool WIDE_OK>
__device__ __forceinline__ void sm_wave_partials(bool wide, float m, const float* x0, const float* anchor,
                                                 const float* del, const float* q, int wave, int lane, float4* red32,
                                                 double* red64)
{
    if (WIDE_OK && wide) {
        // three groups of four sums (fewer FP64 values live at once); after
        // the reduction row j of group g holds sum 4 g + j
        const double md = m;
        auto y = [&](int j) { return ((double)x0[j] - (double)anchor[j]) + (double)del[j]; };
#pragma unroll
        for (int g = 0; g < 3; ++g) {
            double S[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = 4 * g + u;          // 0-2: m y, 3-11: m y_a q_b
                S[u] = k < 3 ? md * y(k) : md * y((k - 3) / 3) * (double)q[(k - 3) % 3];
            }
            wave_sums_by_row64<4>(S);
            if ((lane & 15) == 15) red64[wave * 12 + 4 * g + (lane >> 4)] = S[0];
        }
    } else {
        float y[3];
        for (int j = 0; j < 3; ++j) y[j] = (x0[j] - anchor[j]) + del[j];
        float S[12];
        for (int j = 0; j < 3; ++j) S[j] = m * y[j];
        for (int a = 0; a < 3; ++a)
            for (int k2 = 0; k2 < 3; ++k2) S[3 + 3 * a + k2] = m * y[a] * q[k2];
        wave_sums_by_row<12>(S);
        if ((lane & 15) == 15) {
            float* dst = (float*)red32 + wave * 12 + (lane >> 4) * 3;
            for (int j = 0; j < 3; ++j) dst[j] = S[j];
        }
    }
}

// Centre (relative to the body's anchor) and covariance A = sum m (y - c) q^T
// of a body from its waves' partials, on the body's lane:
// A = sum m y q^T - c (sum m q)^T.  M: the body mass in FP32; M64 the same in
// FP64 (a wide body's centre divides by it).
template <bool WIDE_OK, int UNROLL>
__device__ __forceinline__ void sm_body_sums(int w0, int nw, float M, double M64, const float* mq3,
                                             const float4* red32, const double* red64, float* cc, double* cd,
                                             float* A)
{
    if (WIDE_OK && nw > kWideBodyWaves) {
        // centre, then the covariance row by row (few FP64 values live at once)
        const double im = 1.0 / M64;
        double c[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < nw; ++w)
            for (int j = 0; j < 3; ++j) c[j] += red64[(w0 + w) * 12 + j];
        for (int j = 0; j < 3; ++j) {
            c[j] *= im;
            cc[j] = (float)c[j];
            cd[j] = c[j];
        }
        for (int a = 0; a < 3; ++a) {
            double t[3] = {0.0, 0.0, 0.0};
            for (int w = 0; w < nw; ++w)
                for (int k2 = 0; k2 < 3; ++k2) t[k2] += red64[(w0 + w) * 12 + 3 + 3 * a + k2];
            for (int k2 = 0; k2 < 3; ++k2) A[3 * a + k2] = (float)(t[k2] - c[a] * (double)mq3[k2]);
        }
    } else {
        float T[12];
        sum_wave_partials<3, UNROLL>(red32, w0, nw, T);
        const float im = frcp(M);
        for (int j = 0; j < 3; ++j) {
            cc[j] = T[j] * im;
            cd[j] = (double)cc[j];
        }
        for (int a = 0; a < 3; ++a)
            for (int k2 = 0; k2 < 3; ++k2) A[3 * a + k2] = T[3 + 3 * a + k2] - cc[a] * mq3[k2];
    }
}

constexpr int kNSm = 12, kNMom = 24;       // per-wave partial sums (float4 aligned; 21 momentum sums used)

// Contact corrections of particle i from X_i (Jacobi): planes (constraint
// (1)) and particles of other bodies (constraint (2)), friction from the
// displacement since X_init; accumulated into Cd, the planes first, then the
// partners in list order.
__device__ __forceinline__ void plane_contacts(const StepConsts& c, float mu, const float* x0, const float* del,
                                               float* Cd)
{
    const float mag = fabsf(x0[0]) + fabsf(x0[1]) + fabsf(x0[2]) + fabsf(del[0]) + fabsf(del[1]) + fabsf(del[2]);
    // the FP32 pre-filter over all planes first, so that the FP64 work below
    // is skipped by waves with no particle near a plane
    uint32_t near = 0u;
    for (int pl = 0; pl < c.n_planes; ++pl)
        if (!plane_far(c, pl, x0, del, mag)) near |= 1u << pl;
    if (near != 0u) {
        for (int pl = 0; pl < c.n_planes; ++pl) {
            if (!(near & (1u << pl))) continue;
            const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
            const float un = nx * del[0] + ny * del[1] + nz * del[2];
            const double e = plane_gap(c, pl, x0, del);
            if (!(e < c.radius_d)) continue;
            const float pen = (float)(c.radius_d - e);
            const float ux = del[0] - un * nx, uy = del[1] - un * ny, uz = del[2] - un * nz;
            const float ut2 = ux * ux + uy * uy + uz * uz;
            const float f = ut2 > 0.0f ? fminf(1.0f, mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
            Cd[0] += pen * nx - f * ux;
            Cd[1] += pen * ny - f * uy;
            Cd[2] += pen * nz - f * uz;
        }
    }
}

template <bool MULTI>
__device__ __forceinline__ void contact_correction(const Scene& s, const StepConsts& c, const float* dl, uint32_t avg,
                                                   size_t n, int i, const float* x0, const float* del, float m,
                                                   float* Cd)
{
    const float mu = MULTI ? s.mscene[s.pscene[i]].mu : c.mu;   // multi-scene mode: per scene
    plane_contacts(c, mu, x0, del, Cd);
    const uint32_t ni = s.nbr_n[i];
    const uint32_t cnt = ni < (uint32_t)c.nbr_cap ? ni : (uint32_t)c.nbr_cap;
    for (uint32_t sl = 0; sl < cnt; ++sl) {
        const uint32_t jq = s.nbr[sl * n + i];
        float xq[3], dq[3];
        for (int j = 0; j < 3; ++j) {
            xq[j] = s.x0[j * n + jq];
            dq[j] = dl[j * n + jq];
        }
        pair_correction(c, avg, mu, x0, del, m, ni, xq, dq, s.mass[jq], avg == 0u ? s.nbr_n[jq] : 0u, Cd);
    }
}

// The partner contacts of one wave's particles (one body's, single-scene
// mode), spread over its lanes.  A wave that loops over each particle's list
// makes as many passes as its longest list (about two in a settled pile,
// where most particles have none); here the wave's (particle, slot) pairs are
// numbered in particle order, then slot order (a scan of the list lengths),
// lane l computes pair base + l of each window of 64, and every particle then
// adds the corrections of its own pairs in slot order, as the loop does.
// Called by all 64 lanes (lane swaps).  ni, j0: the lane's list length and
// first partner id, loaded with its particle's data (0 for a lane without a
// particle), so that a pair of slot 0 takes its partner's id from that lane.
__device__ __forceinline__ void pair_contacts_spread(const Scene& s, const StepConsts& c, const float* dl,
                                                     uint32_t avg, size_t n, int i, int lane, uint32_t ni,
                                                     uint32_t j0, const float* x0, const float* del, float m,
                                                     float* Cd)
{
#pragma clang fp contract(on)
    const uint32_t cnt = ni < (uint32_t)c.nbr_cap ? ni : (uint32_t)c.nbr_cap;
    const uint32_t incl = wave_inclusive_scan(cnt);
    const uint32_t off = incl - cnt;
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
    for (uint32_t base = 0; base < total; base += 64u) {
        const uint32_t p = base + (uint32_t)lane;
        // the particle (lane) of pair p: the first lane whose inclusive count exceeds p
        int o = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1)
            if ((uint32_t)__shfl((int)incl, o + step - 1, 64) <= p) o += step;
        o = o < 63 ? o : 63;
        float ox[3], od[3];
        for (int j = 0; j < 3; ++j) {
            ox[j] = __shfl(x0[j], o, 64);
            od[j] = __shfl(del[j], o, 64);
        }
        const float om = __shfl(m, o, 64);
        const uint32_t oni = (uint32_t)__shfl((int)ni, o, 64), ooff = (uint32_t)__shfl((int)off, o, 64);
        const uint32_t oj0 = (uint32_t)__shfl((int)j0, o, 64);
        float sc = 0.0f, t[3] = {0.0f, 0.0f, 0.0f};
        if (p < total) {
            const int io = i - lane + o;             // the wave's particles are consecutive
            const uint32_t jq = p == ooff ? oj0 : s.nbr[(size_t)(p - ooff) * n + io];
            float xq[3], dq[3];
            for (int j = 0; j < 3; ++j) {
                xq[j] = s.x0[j * n + jq];
                dq[j] = dl[j * n + jq];
            }
            if (!pair_terms(c, avg, c.mu, ox, od, om, oni, xq, dq, s.mass[jq], avg == 0u ? s.nbr_n[jq] : 0u, sc, t))
                sc = 0.0f;                           // (a contact has sc > 0)
        }
        // this particle's pairs in the window: lanes lo - base .. hi - base - 1
        const uint32_t lo = off > base ? off : base, hi = incl < base + 64u ? incl : base + 64u;
        const uint32_t mine = hi > lo ? hi - lo : 0u;
        for (uint32_t k = 0; __any(k < mine); ++k) {
            const int src = (int)(lo - base + k);
            const float a = __shfl(sc, src, 64);
            float b[3];
            for (int j = 0; j < 3; ++j) b[j] = __shfl(t[j], src, 64);
            if (k < mine && a != 0.0f)
                for (int j = 0; j < 3; ++j) Cd[j] += a * b[j];
        }
    }
}

// Shape matching of one body, on its lane: centre and covariance from the
// partials of its waves w0 .. w0 + nw - 1, the rotation (from the second
// iteration on refined from the previous iteration's, Rprev, by Newton steps
// on SO(3)), made orthogonal in FP64; then R and the centre to `rd` (FP64)
// and to `sm` (FP32, 12 values), and R's FP32 rounding kept for the next
// iteration.
template <bool WIDE_OK, int UNROLL>
__device__ __forceinline__ void body_shape_match(const Scene& s, int it, int bb, int w0, int nw, float M, double M64,
                                                 const float* mq3, const float* Rprev, const float4* red32,
                                                 const double* red64, float* sm, double* rd)
{
    float cc[3], A[9], Rb[9];
    sm_body_sums<WIDE_OK, UNROLL>(w0, nw, M, M64, mq3, red32, red64, cc, &rd[9], A);
    if (!(it > 0 && polar_refine_steps(A, Rprev, Rb))) polar_rotation(A, Rb);
    orthonormalise64(Rb, rd);
    for (int j = 0; j < 9; ++j) Rb[j] = (float)rd[j];
    for (int j = 0; j < 9; ++j) sm[j] = Rb[j];
    for (int j = 0; j < 3; ++j) sm[9 + j] = cc[j];
    if (s.body_rot)
        for (int j = 0; j < 9; ++j) s.body_rot[9 * (size_t)bb + j] = Rb[j];
}

// This wave's partial sums of the momentum constraint to LDS slot `slot`, in
// the frame centred on c_i: z_b = r + C (before shape matching), z_a = z_b + D,
// with r = x - c_i, C the contact correction and D the goal offset.
__device__ __forceinline__ void mom_wave_partials(const StepConsts& c, float m, const float* r, const float* Cd,
                                                  const float* Dd, const float* V, int slot, int lane,
                                                  float4* red_mom)
{
    float S[kNMom];
    float zb[3], za[3], vb[3], t[3];
    for (int j = 0; j < 3; ++j) {
        zb[j] = r[j] + Cd[j];
        za[j] = zb[j] + Dd[j];
        vb[j] = V[j] + Cd[j] * c.inv_h;
        S[j] = m * Cd[j];               // S1 = sum m C
        S[3 + j] = m * Dd[j];           // S2 = sum m D
        S[6 + j] = m * vb[j];           // S3 = P_bsm
    }
    cross(zb, Dd, t);
    for (int j = 0; j < 3; ++j) S[9 + j] = m * t[j];          // S4 = sum m z_b x D
    cross(Dd, vb, t);
    for (int j = 0; j < 3; ++j) S[12 + j] = m * t[j];         // S5 = sum m D x v_b
    S[15] = m * (za[1] * za[1] + za[2] * za[2]);              // S6: inertia about c_i
    S[16] = m * (za[0] * za[0] + za[2] * za[2]);
    S[17] = m * (za[0] * za[0] + za[1] * za[1]);
    S[18] = -m * za[0] * za[1];
    S[19] = -m * za[0] * za[2];
    S[20] = -m * za[1] * za[2];
    S[21] = S[22] = S[23] = 0.0f;
    wave_sums_by_row<kNMom>(S);
    if ((lane & 15) == 15) {
        float* dst = (float*)red_mom + slot * kNMom + (lane >> 4) * (kNMom / 4);
        for (int j = 0; j < kNMom / 4; ++j) dst[j] = S[j];
    }
}

// The momentum conservation constraint of one body, on its lane, from the
// partials of its waves w0 .. w0 + nw - 1: dv (3), omega (3) and c_asm - c_i
// (3) to `out`.
template <int UNROLL>
__device__ __forceinline__ void body_momentum(const StepConsts& c, int w0, int nw, float Mb, const float4* red_mom,
                                              float* out)
{
    float T[kNMom];
    sum_wave_partials<kNMom / 4, UNROLL>(red_mom, w0, nw, T);
    const float im = frcp(Mb);
    float cb[3], Db[3], cab[3], dvb[3] = {0.0f, 0.0f, 0.0f}, wb[3] = {0.0f, 0.0f, 0.0f};
    for (int j = 0; j < 3; ++j) {
        cb[j] = T[j] * im;                   // c_bsm - c_i
        Db[j] = T[3 + j] * im;               // mean shape-matching shift
        cab[j] = cb[j] + Db[j];              // c_asm - c_i
    }
    // Eq. (4): dv = (P_bsm - P_asm) / M,  P_asm - P_bsm = sum m D / dt
    if (!(c.flags & kFlagNoLinMom))
        for (int j = 0; j < 3; ++j) dvb[j] = -T[3 + j] * c.inv_h * im;
    // Eq. (5): omega = I^-1 (L_asm - L_bsm); the difference is formed from
    // the small quantities: (sum m r_b x D)/dt + sum m D x v_b - Db x P_bsm
    if (!(c.flags & kFlagNoAngMom)) {
        float cbxD[3], DbxP[3], dL[3], I6[6];
        cross(cb, &T[3], cbxD);
        cross(Db, &T[6], DbxP);
        for (int j = 0; j < 3; ++j) dL[j] = (T[9 + j] - cbxD[j]) * c.inv_h + T[12 + j] - DbxP[j];
        // parallel-axis shift of the inertia from c_i to c_asm
        I6[0] = T[15] - Mb * (cab[1] * cab[1] + cab[2] * cab[2]);
        I6[1] = T[16] - Mb * (cab[0] * cab[0] + cab[2] * cab[2]);
        I6[2] = T[17] - Mb * (cab[0] * cab[0] + cab[1] * cab[1]);
        I6[3] = T[18] + Mb * cab[0] * cab[1];
        I6[4] = T[19] + Mb * cab[0] * cab[2];
        I6[5] = T[20] + Mb * cab[1] * cab[2];
        const float scale = fmaxf(I6[0] + I6[1] + I6[2], Mb * c.two_r * c.two_r);
        solve_inertia(I6, dL, scale, wb);
    }
    for (int j = 0; j < 3; ++j) {
        out[j] = dvb[j];
        out[3 + j] = wb[j];
        out[6 + j] = cab[j];
    }
}

// X_{i+1} - X_init and V_{i+1} of particle i (Sec. III-B velocity update with
// the momentum terms of Sec. III-C): mom = the body's dv, omega, c_asm - c_i.
__device__ __forceinline__ void particle_update(const StepConsts& c, const float* mom, const float* x0,
                                                const float* del, const float* V, const float* r, const float* Cd,
                                                const float* Dd, size_t n, int i, float* dn, float* vn)
{
    float dv[3], w[3], ca[3];
    for (int j = 0; j < 3; ++j) {
        dv[j] = mom[j];
        w[j] = mom[3 + j];
        ca[j] = mom[6 + j];
    }
    float ra[3], wr[3];
    for (int j = 0; j < 3; ++j) ra[j] = r[j] + Cd[j] + Dd[j] - ca[j];
    cross(w, ra, wr);
    for (int j = 0; j < 3; ++j) {
        const float step = Cd[j] + Dd[j];
        const float dvi = dv[j] - wr[j];
        const float dnew = (del[j] + step) + c.h * dvi;
        dn[j * n + i] = dnew;
        if (c.flags & kFlagStdVelocity) {
            // standard PBD: V = (X_{i+1} - X_init) / dt in world FP32 coordinates
            const float xw = x0[j] + dnew;
            vn[j * n + i] = (xw - x0[j]) * c.inv_h;
        } else {
            vn[j * n + i] = (V[j] + step * c.inv_h) + dvi;
        }
    }
}

// Bodies are packed into workgroups of W waves; each body owns ceil(n/64)
// consecutive waves, one particle per lane.  Per-body sums are wave sums (lane swaps, DPP)
// combined over the body's waves; the per-body 3x3 algebra runs on lane j of
// wave 0 for the j-th body of the workgroup.  `it` is the iteration index in
// the substep: from the second iteration on, the rotation is refined from the
// previous iteration's.  blk: the workgroup's index in the packing.
// SM_UNROLL / MOM_UNROLL: waves whose partial sums the per-body lane reads
// from LDS at once.
template <bool MULTI, bool WIDE_OK, int SM_UNROLL, int MOM_UNROLL, bool SPREAD = false>
__device__ __forceinline__ void iterate_body(const Scene& s, const StepConsts& c, int src, int it, int blk)
{
    __shared__ float4 red_sm[kMaxWaves * kNSm / 4];
    __shared__ double red_sm64[WIDE_OK ? kMaxWaves * kNSm : 1];
    __shared__ float4 red_mom[kMaxWaves * kNMom / 4];
    __shared__ float body_sm[kMaxWaves * 12];    // per body of the workgroup: R (9), centre (3)
    __shared__ float body_mom[kMaxWaves * 9];    // dv (3), omega (3), c_asm - c_i (3)
    __shared__ double body_rd[kMaxWaves * 12];   // R and centre in FP64 (goal offsets)

    // the wave index as a wave-uniform (scalar) value: the per-wave table and
    // body entries below then come through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int g = blk * s.waves_per_block + wave;
    const int b = s.wave_body[g];                 // -1: idle wave
    const int blk_b0 = s.block_body[2 * blk], blk_nb = s.block_body[2 * blk + 1];
    int s0 = 0, e0 = 0, lw0 = wave;
    if (b >= 0) {
        s0 = s.body_start[b];
        e0 = s.body_start[b + 1];
        lw0 = s.body_wave0[b] - blk * s.waves_per_block;
    }
    const int lb = b >= blk_b0 ? b - blk_b0 : 0;  // body slot within the workgroup
    const int i = s0 + (wave - lw0) * 64 + lane;  // this lane's particle
    const bool act = b >= 0 && i < e0;
    const bool wide = e0 - s0 > 64 * kWideBodyWaves;
    const size_t n = (size_t)s.n;
    const float* dl = s.dl[src];
    const float* vl = s.vel[src];
    float* dn = s.dl[src ^ 1];
    float* vn = s.vel[src ^ 1];
    const float ax = s.x0[s0], ay = s.x0[n + s0], az = s.x0[2 * n + s0];   // body anchor
    const float anc[3] = {ax, ay, az};
    const uint32_t avg = (c.flags >> kAvgShift) & 3u;

    float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, V[3] = {0.0f, 0.0f, 0.0f};
    float q[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f, Cd[3] = {0.0f, 0.0f, 0.0f};
    uint32_t ni = 0u, j0 = 0u;
    if (act) {
        for (int j = 0; j < 3; ++j) {
            x0[j] = s.x0[j * n + i];
            del[j] = dl[j * n + i];
            V[j] = vl[j * n + i];
            q[j] = s.q[j * n + i];
        }
        m = s.mass[i];
        if (SPREAD) {           // list length and first partner: no load waits on another
            ni = s.nbr_n[i];
            j0 = s.nbr[i];
        }
    }
    if (SPREAD) {               // single-scene mode: partner contacts spread over the wave's lanes
        if (act) plane_contacts(c, c.mu, x0, del, Cd);
        pair_contacts_spread(s, c, dl, avg, n, i, lane, ni, j0, x0, del, m, Cd);
    } else if (act) {
        contact_correction<MULTI>(s, c, dl, avg, n, i, x0, del, m, Cd);
    }

    // shape matching on X_i: centre and covariance in one reduction,
    // A = sum m (x - c) q^T = sum m y q^T - c (sum m q)^T, y = x - anchor
    sm_wave_partials<WIDE_OK>(wide, m, x0, anc, del, q, wave, lane, red_sm, red_sm64);

    // per-body lane of wave 0: body slot `lane` of this workgroup (its data
    // is loaded here, so that it holds no registers through the contacts)
    const bool body_lane = wave == 0 && lane < blk_nb;
    const int bb = blk_b0 + (body_lane ? lane : 0);
    int bl_w0 = 0, bl_nw = 0;
    float bl_M = 1.0f, Rprev[9], mq3[3];
    double bl_M64 = 1.0;
    if (body_lane) {
        bl_w0 = s.body_wave0[bb] - blk * s.waves_per_block;
        bl_nw = (s.body_start[bb + 1] - s.body_start[bb] + 63) >> 6;
        bl_M = s.body_mass[bb];
        if (WIDE_OK) bl_M64 = s.body_mass64[bb];
        for (int j = 0; j < 3; ++j) mq3[j] = s.body_mq[3 * (size_t)bb + j];
        if (it > 0)
            for (int j = 0; j < 9; ++j) Rprev[j] = s.body_rot[9 * (size_t)bb + j];
    }
    __syncthreads();
    if (body_lane)              // one lane per body: centre, covariance, rotation
        body_shape_match<WIDE_OK, SM_UNROLL>(s, it, bb, bl_w0, bl_nw, bl_M, bl_M64, mq3, Rprev, red_sm, red_sm64,
                                             &body_sm[lane * 12], &body_rd[lane * 12]);
    __syncthreads();
    float cyv[3];
    for (int j = 0; j < 3; ++j) cyv[j] = body_sm[lb * 12 + 9 + j];

    // goal offsets D = R q - (x - c) and the momentum sums, in the frame
    // centred on c_i
    float r[3], Dd[3] = {0.0f, 0.0f, 0.0f};
    for (int j = 0; j < 3; ++j) r[j] = ((x0[j] - anc[j]) + del[j]) - cyv[j];
    if (act) goal_offset(&body_rd[lb * 12], q, x0, anc, del, Dd);
    mom_wave_partials(c, m, r, Cd, Dd, V, wave, lane, red_mom);
    __syncthreads();

    // momentum conservation constraint, one lane per body
    if (body_lane) body_momentum<MOM_UNROLL>(c, bl_w0, bl_nw, bl_M, red_mom, &body_mom[lane * 9]);
    __syncthreads();
    if (!act) return;
    particle_update(c, &body_mom[lb * 9], x0, del, V, r, Cd, Dd, n, i, dn, vn);
}

// A body of more than 4 and at most kMaxWaves waves in a workgroup of 4
// waves.  Such workgroups come first in the launch, so they start first and
// their longer run overlaps the other workgroups'.  Wave w takes the body's
// chunks of 64 particles w, w + 4, w + 8, w + 12, and for each does what one
// wave of iterate_body does for its particles, with the chunk's partial sums
// in the LDS slots of the wave it stands for: the body's sums and arithmetic
// are those of a workgroup of kMaxWaves waves.  Between the phases a
// particle's contact correction and goal offset wait in its own slots of the
// output arrays (X_{i+1} - X_init and V_{i+1}), which its last phase
// overwrites; its other data is read again.
template <int SM_UNROLL, int MOM_UNROLL>
__device__ __forceinline__ void iterate_chunked(const Scene& s, const StepConsts& c, int src, int it)
{
    __shared__ float4 red_sm[kMaxWaves * kNSm / 4];
    __shared__ double red_sm64[kMaxWaves * kNSm];
    __shared__ float4 red_mom[kMaxWaves * kNMom / 4];
    __shared__ float body_sm[12];
    __shared__ float body_mom[9];
    __shared__ double body_rd[12];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int waves = (int)(blockDim.x >> 6);
    const int b = s.block_body[2 * blockIdx.x];
    const int s0 = s.body_start[b], e0 = s.body_start[b + 1];
    const int nw = (e0 - s0 + 63) >> 6;
    const bool wide = e0 - s0 > 64 * kWideBodyWaves;
    const size_t n = (size_t)s.n;
    const float* dl = s.dl[src];
    const float* vl = s.vel[src];
    float* dn = s.dl[src ^ 1];
    float* vn = s.vel[src ^ 1];
    const float anc[3] = {s.x0[s0], s.x0[n + s0], s.x0[2 * n + s0]};   // body anchor
    const uint32_t avg = (c.flags >> kAvgShift) & 3u;

    const bool body_lane = threadIdx.x == 0;
    float bl_M = 1.0f, Rprev[9], mq3[3];
    double bl_M64 = 1.0;
    if (body_lane) {
        bl_M = s.body_mass[b];
        bl_M64 = s.body_mass64[b];
        for (int j = 0; j < 3; ++j) mq3[j] = s.body_mq[3 * (size_t)b + j];
        if (it > 0)
            for (int j = 0; j < 9; ++j) Rprev[j] = s.body_rot[9 * (size_t)b + j];
    }

    // contacts, then the chunk's shape-matching partials
    for (int k = wave; k < nw; k += waves) {
        const int i = s0 + 64 * k + lane;
        const bool act = i < e0;
        float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, q[3] = {0.0f, 0.0f, 0.0f};
        float m = 0.0f, Cd[3] = {0.0f, 0.0f, 0.0f};
        if (act) {
            for (int j = 0; j < 3; ++j) {
                x0[j] = s.x0[j * n + i];
                del[j] = dl[j * n + i];
                q[j] = s.q[j * n + i];
            }
            m = s.mass[i];
            contact_correction<false>(s, c, dl, avg, n, i, x0, del, m, Cd);
            for (int j = 0; j < 3; ++j) dn[j * n + i] = Cd[j];
        }
        sm_wave_partials<true>(wide, m, x0, anc, del, q, k, lane, red_sm, red_sm64);
    }
    __syncthreads();
    if (body_lane)
        body_shape_match<true, SM_UNROLL>(s, it, b, 0, nw, bl_M, bl_M64, mq3, Rprev, red_sm, red_sm64, body_sm,
                                          body_rd);
    __syncthreads();
    float cyv[3];
    for (int j = 0; j < 3; ++j) cyv[j] = body_sm[9 + j];

    // goal offsets and the chunk's momentum partials
    for (int k = wave; k < nw; k += waves) {
        const int i = s0 + 64 * k + lane;
        const bool act = i < e0;
        float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, V[3] = {0.0f, 0.0f, 0.0f};
        float q[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f, Cd[3] = {0.0f, 0.0f, 0.0f};
        if (act) {
            for (int j = 0; j < 3; ++j) {
                x0[j] = s.x0[j * n + i];
                del[j] = dl[j * n + i];
                V[j] = vl[j * n + i];
                q[j] = s.q[j * n + i];
                Cd[j] = dn[j * n + i];
            }
            m = s.mass[i];
        }
        float r[3], Dd[3] = {0.0f, 0.0f, 0.0f};
        for (int j = 0; j < 3; ++j) r[j] = ((x0[j] - anc[j]) + del[j]) - cyv[j];
        if (act) {
            goal_offset(body_rd, q, x0, anc, del, Dd);
            for (int j = 0; j < 3; ++j) vn[j * n + i] = Dd[j];
        }
        mom_wave_partials(c, m, r, Cd, Dd, V, k, lane, red_mom);
    }
    __syncthreads();
    if (body_lane) body_momentum<MOM_UNROLL>(c, 0, nw, bl_M, red_mom, body_mom);
    __syncthreads();

    for (int k = wave; k < nw; k += waves) {
        const int i = s0 + 64 * k + lane;
        if (i >= e0) continue;
        float x0[3], del[3], V[3], Cd[3], Dd[3], r[3];
        for (int j = 0; j < 3; ++j) {
            x0[j] = s.x0[j * n + i];
            del[j] = dl[j * n + i];
            V[j] = vl[j * n + i];
            Cd[j] = dn[j * n + i];
            Dd[j] = vn[j * n + i];
        }
        for (int j = 0; j < 3; ++j) r[j] = ((x0[j] - anc[j]) + del[j]) - cyv[j];
        particle_update(c, body_mom, x0, del, V, r, Cd, Dd, n, i, dn, vn);
    }
}

// The iteration kernel in two register budgets: the compiler's choice (about
// 78 VGPRs, fastest when the grid fits the GPU at once), and at most 80 VGPRs
// (6 waves per SIMD, a few values spilled) for grids that oversubscribe it,
// where more workgroups per CU hide each other's per-body phases, and whose
// partner contacts are spread over each wave's lanes.
// WIDE: some body of the launch spans more than kWideBodyWaves waves (FP64
// sums for those bodies; the other bodies' arithmetic is the same in both
// instances)
template <bool MULTI, bool WIDE>
__global__ void __launch_bounds__(64 * kMaxWaves) k_iterate(Scene s, StepConsts c, int src, int it)
{
    iterate_body<MULTI, WIDE, 4, 4>(s, c, src, it, xcd_block());
}

// 4-wave workgroups: the first s.n_chunked take one body of more than 4
// waves each, in chunks; the others bodies of up to 4 waves (never wide),
// with the partner contacts spread over each wave's lanes
__global__ void __launch_bounds__(64 * kMaxWaves) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_iterate_dense(Scene s, StepConsts c, int src, int it)
{
    if ((int)blockIdx.x < s.n_chunked) {
        iterate_chunked<4, 4>(s, c, src, it);
        return;
    }
    iterate_body<false, false, 2, 2, true>(s, c, src, it, xcd_block_from(s.n_chunked));
}

// ---------------------------------------------------------------------------
// all K iterations of a substep in one launch
// ---------------------------------------------------------------------------

// For a scene whose iteration grid the GPU holds at once (checked on the host
// from the kernel's occupancy), the K Jacobi iterations of a substep run in
// one launch.  A workgroup keeps its particles' state in registers across the
// iterations.  A particle with contact partners publishes each component of
// its X_{it+1} - X_init as one 64-bit word, the value's bits under a tag that
// names the substep and the iteration, with an agent-scope (XCD-coherent)
// atomic store; a partner reading X_it polls the word with agent-scope
// atomic loads until the tag is that of iteration it.  Value and readiness
// travel together, so a read costs one memory round trip once the value is
// there.  Waiting for a partner's X_it also orders the reuse of the double
// buffer: the partner wrote X_it after it had read this particle's X_{it-1},
// so X_{it+1} can replace X_{it-1}.  Particles without partners in other
// bodies never wait.  Every wait is bounded: one that gives up latches
// kErrWait instead of hanging, and the frame is then discarded.  The
// arithmetic is that of iterate_body, in the same order.
constexpr uint32_t kWaitLimit = 1u << 20;

// tag of X_it in substep `epoch` (K < 64 iterations; tags repeat after 2^26 substeps)
__device__ inline uint32_t iter_tag(uint32_t epoch, int it) { return (epoch << 6) | (uint32_t)it; }

// Called once per unsuccessful poll of a partner wait: true (and nowait set)
// once this wait has polled kWaitLimit times, which latches kErrWait, or, checked
// every 256 polls, once some other wait of the launch has given up.
__device__ inline bool stop_waiting(const Scene& s, uint32_t spins, bool& nowait)
{
    if (spins > kWaitLimit) {
        atomicOr(&s.counters->err, kErrWait);
        nowait = true;
    } else if ((spins & 255u) == 0u &&
               (__hip_atomic_load(&s.counters->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrWait)) {
        nowait = true;
    }
    return nowait;
}

__global__ void __launch_bounds__(64 * kMaxWaves) k_iterate_resident(Scene s, StepConsts c, int K)
{
    constexpr int PG = 2;                // contact partners whose positions are loaded together
    constexpr int NSM = 12, NMOM = 24;
    __shared__ float4 red_sm[kMaxWaves * NSM / 4];
    __shared__ double red_sm64[kMaxWaves * NSM];
    __shared__ float4 red_mom[kMaxWaves * NMOM / 4];
    __shared__ float body_sm[kMaxWaves * 12];
    __shared__ float body_mom[kMaxWaves * 9];
    __shared__ double body_rd[kMaxWaves * 12];

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int blk = xcd_block();
    const int W = s.waves_per_block;
    const int g = blk * W + wave;
    const int b = s.wave_body[g];                 // -1: idle wave
    const int blk_b0 = s.block_body[2 * blk], blk_nb = s.block_body[2 * blk + 1];
    int s0 = 0, e0 = 0, lw0 = wave;
    if (b >= 0) {
        s0 = s.body_start[b];
        e0 = s.body_start[b + 1];
        lw0 = s.body_wave0[b] - blk * W;
    }
    const int lb = b >= blk_b0 ? b - blk_b0 : 0;
    const int i = s0 + (wave - lw0) * 64 + lane;
    const bool act = b >= 0 && i < e0;
    const bool wide = e0 - s0 > 64 * kWideBodyWaves;
    const size_t n = (size_t)s.n;
    const float ax = s.x0[s0], ay = s.x0[n + s0], az = s.x0[2 * n + s0];   // body anchor
    const float anc[3] = {ax, ay, az};
    const uint32_t avg = (c.flags >> kAvgShift) & 3u;

    // per-body constants in LDS rather than in registers of every lane; the
    // previous iteration's rotation is read from the body's LDS slot
    __shared__ float body_mq_s[kMaxWaves * 3];
    __shared__ int body_waves_s[kMaxWaves * 2];   // first wave in the workgroup, wave count
    __shared__ float body_M_s[kMaxWaves];
    __shared__ double body_M64_s[kMaxWaves];
    const bool body_lane = wave == 0 && lane < blk_nb;
    if (body_lane) {
        const int bb = blk_b0 + lane;
        body_waves_s[2 * lane] = s.body_wave0[bb] - blk * W;
        body_waves_s[2 * lane + 1] = (s.body_start[bb + 1] - s.body_start[bb] + 63) >> 6;
        body_M_s[lane] = s.body_mass[bb];
        body_M64_s[lane] = s.body_mass64[bb];
        for (int j = 0; j < 3; ++j) body_mq_s[lane * 3 + j] = s.body_mq[3 * (size_t)bb + j];
    }

    // X_0 - X_init and V_0 from the integration step stay in registers; the
    // constants X_init, q and m of the lane's particle wait in LDS and are
    // read in each phase that uses them, so that they do not hold registers
    // through the per-body algebra
    __shared__ float p_const[7][64 * kMaxWaves];
    const int tid = threadIdx.x;
    float del[3] = {0.0f, 0.0f, 0.0f}, V[3] = {0.0f, 0.0f, 0.0f};
    uint32_t ni = 0u;
    {
        float cv[7] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (act) {
            for (int j = 0; j < 3; ++j) {
                cv[j] = s.x0[j * n + i];
                del[j] = s.dl[0][j * n + i];
                V[j] = s.vel[0][j * n + i];
                cv[3 + j] = s.q[j * n + i];
            }
            cv[6] = s.mass[i];
            ni = s.nbr_n[i];
        }
        for (int j = 0; j < 7; ++j) p_const[j][tid] = cv[j];
    }
    float x0[3], q[3], m;
    auto load_consts = [&]() {
        for (int j = 0; j < 3; ++j) {
            x0[j] = p_const[j][tid];
            q[j] = p_const[3 + j][tid];
        }
        m = p_const[6][tid];
    };
    const uint32_t cnt = ni < (uint32_t)c.nbr_cap ? ni : (uint32_t)c.nbr_cap;
    const float mu = c.mu;
    const uint32_t epoch = s.counters->epoch;
    // No waiting once a list has overflowed (partners then need not list each
    // other both ways) or a wait has given up anywhere: the frame is discarded
    // in either case, and the launch only has to end.
    bool nowait = (__hip_atomic_load(&s.counters->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                   (kErrCapacity | kErrWait)) != 0u;

    for (int it = 0; it < K; ++it) {
        const unsigned long long* tg = s.tagged + (size_t)(it & 1) * 3 * n;   // partners' X_it, tagged
        load_consts();
        sm_wave_partials<true>(wide, m, x0, anc, del, q, wave, lane, red_sm, red_sm64);
        // the first PE partners' words are loaded during the per-body phase,
        // which does not need them, and checked after it
        constexpr int PE = 1;
        const uint32_t want = iter_tag(epoch, it);
        uint32_t je[PE];
        unsigned long long we[PE][3];
        for (int g = 0; g < PE; ++g) {
            je[g] = 0u;
            for (int j = 0; j < 3; ++j) we[g][j] = 0ull;
        }
        if (act && cnt > 0u) {
            for (int g = 0; g < PE; ++g) je[g] = s.nbr[((uint32_t)g < cnt ? g : 0) * n + i];
            if (it > 0)
                for (int g = 0; g < PE; ++g)
                    for (int j = 0; j < 3; ++j)
                        we[g][j] = __hip_atomic_load(&tg[j * n + je[g]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (body_lane) {
            float cc[3], A[9], Rb[9];
            float mq3[3], Rprev[9];
            for (int j = 0; j < 3; ++j) mq3[j] = body_mq_s[lane * 3 + j];
            sm_body_sums<true, 4>(body_waves_s[2 * lane], body_waves_s[2 * lane + 1], body_M_s[lane],
                                  body_M64_s[lane], mq3, red_sm, red_sm64, cc, &body_rd[lane * 12 + 9], A);
            for (int j = 0; j < 9; ++j) Rprev[j] = body_sm[lane * 12 + j];   // (it > 0) the last iteration's
            if (!(it > 0 && polar_refine_steps(A, Rprev, Rb))) polar_rotation(A, Rb);
            orthonormalise64(Rb, &body_rd[lane * 12]);
            for (int j = 0; j < 9; ++j) body_sm[lane * 12 + j] = (float)body_rd[lane * 12 + j];
            for (int j = 0; j < 3; ++j) body_sm[lane * 12 + 9 + j] = cc[j];
        }
        __syncthreads();
        // goal offsets (shape matching), formed before the contacts so that
        // the body's rotation and centre need not stay in registers through them
        load_consts();
        float r[3], Dd[3] = {0.0f, 0.0f, 0.0f};
        {
            float cyv[3];
            for (int j = 0; j < 3; ++j) cyv[j] = body_sm[lb * 12 + 9 + j];
            for (int j = 0; j < 3; ++j) r[j] = ((x0[j] - anc[j]) + del[j]) - cyv[j];
            if (act) goal_offset(&body_rd[lb * 12], q, x0, anc, del, Dd);
        }

        // contacts from X_i (planes, then partners in list order)
        float Cd[3] = {0.0f, 0.0f, 0.0f};
        if (act) {
            const float mag =
                fabsf(x0[0]) + fabsf(x0[1]) + fabsf(x0[2]) + fabsf(del[0]) + fabsf(del[1]) + fabsf(del[2]);
            for (int pl = 0; pl < c.n_planes; ++pl) {
                if (plane_far(c, pl, x0, del, mag)) continue;
                const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
                const float un = nx * del[0] + ny * del[1] + nz * del[2];
                const double e = plane_gap(c, pl, x0, del);
                if (!(e < c.radius_d)) continue;
                const float pen = (float)(c.radius_d - e);
                const float ux = del[0] - un * nx, uy = del[1] - un * ny, uz = del[2] - un * nz;
                const float ut2 = ux * ux + uy * uy + uz * uz;
                const float f = ut2 > 0.0f ? fminf(1.0f, mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
                Cd[0] += pen * nx - f * ux;
                Cd[1] += pen * ny - f * uy;
                Cd[2] += pen * nz - f * uz;
            }
            // the early group: its words are usually ready by now
            if (cnt > 0u) {
                float xe[PE][3], de[PE][3];
                for (int g = 0; g < PE; ++g)
                    for (int j = 0; j < 3; ++j) xe[g][j] = s.x0[j * n + je[g]];
                if (it == 0) {                        // X_0 from the integration step
                    for (int g = 0; g < PE; ++g)
                        for (int j = 0; j < 3; ++j) de[g][j] = s.dl[0][j * n + je[g]];
                } else {
                    uint32_t spins = 0;
                    while (!nowait) {
                        bool ready = true;
                        for (int g = 0; g < PE; ++g)
                            for (int j = 0; j < 3; ++j) ready = ready && (uint32_t)(we[g][j] >> 32) == want;
                        if (ready || stop_waiting(s, ++spins, nowait)) break;
                        __builtin_amdgcn_s_sleep(1);
                        for (int g = 0; g < PE; ++g)
                            for (int j = 0; j < 3; ++j)
                                we[g][j] = __hip_atomic_load(&tg[j * n + je[g]], __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                    }
                    for (int g = 0; g < PE; ++g)
                        for (int j = 0; j < 3; ++j) de[g][j] = __uint_as_float((uint32_t)we[g][j]);
                }
                for (int g = 0; g < PE; ++g)
                    if ((uint32_t)g < cnt)
                        pair_correction(c, avg, mu, x0, del, m, ni, xe[g], de[g], s.mass[je[g]],
                                        avg == 0u ? s.nbr_n[je[g]] : 0u, Cd);
            }
            // further partners PG at a time: their tagged words are loaded
            // together and polled again only while a tag is not yet X_it's
            for (uint32_t sl = PE; sl < cnt; sl += PG) {
                uint32_t jq[PG];
                float xq[PG][3], dq[PG][3];
                for (int g = 0; g < PG; ++g) {
                    jq[g] = sl + g < cnt ? s.nbr[(sl + g) * n + i] : s.nbr[sl * n + i];
                    for (int j = 0; j < 3; ++j) xq[g][j] = s.x0[j * n + jq[g]];
                }
                if (it == 0) {                        // X_0 from the integration step
                    for (int g = 0; g < PG; ++g)
                        for (int j = 0; j < 3; ++j) dq[g][j] = s.dl[0][j * n + jq[g]];
                } else {
                    unsigned long long w[PG][3];
                    uint32_t spins = 0;
                    while (true) {
                        for (int g = 0; g < PG; ++g)
                            for (int j = 0; j < 3; ++j)
                                w[g][j] = __hip_atomic_load(&tg[j * n + jq[g]], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                        bool ready = true;
                        for (int g = 0; g < PG; ++g)
                            for (int j = 0; j < 3; ++j) ready = ready && (uint32_t)(w[g][j] >> 32) == want;
                        if (ready || nowait || stop_waiting(s, ++spins, nowait)) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    for (int g = 0; g < PG; ++g)
                        for (int j = 0; j < 3; ++j) dq[g][j] = __uint_as_float((uint32_t)w[g][j]);
                }
                for (int g = 0; g < PG; ++g)
                    if (sl + g < cnt)
                        pair_correction(c, avg, mu, x0, del, m, ni, xq[g], dq[g], s.mass[jq[g]],
                                        avg == 0u ? s.nbr_n[jq[g]] : 0u, Cd);
            }
        }


        // r + C + D and C + D: all the velocity update needs of this phase
        float za[3], step[3];
        {
            float S[NMOM];
            float zb[3], vb[3], t[3];
            for (int j = 0; j < 3; ++j) {
                zb[j] = r[j] + Cd[j];
                za[j] = zb[j] + Dd[j];
                step[j] = Cd[j] + Dd[j];
                vb[j] = V[j] + Cd[j] * c.inv_h;
                S[j] = m * Cd[j];
                S[3 + j] = m * Dd[j];
                S[6 + j] = m * vb[j];
            }
            cross(zb, Dd, t);
            for (int j = 0; j < 3; ++j) S[9 + j] = m * t[j];
            cross(Dd, vb, t);
            for (int j = 0; j < 3; ++j) S[12 + j] = m * t[j];
            S[15] = m * (za[1] * za[1] + za[2] * za[2]);
            S[16] = m * (za[0] * za[0] + za[2] * za[2]);
            S[17] = m * (za[0] * za[0] + za[1] * za[1]);
            S[18] = -m * za[0] * za[1];
            S[19] = -m * za[0] * za[2];
            S[20] = -m * za[1] * za[2];
            S[21] = S[22] = S[23] = 0.0f;
            wave_sums_by_row<NMOM>(S);
            if ((lane & 15) == 15) {
                float* dst = (float*)red_mom + wave * NMOM + (lane >> 4) * (NMOM / 4);
                for (int j = 0; j < NMOM / 4; ++j) dst[j] = S[j];
            }
        }
        __syncthreads();
        if (body_lane) {
            float T[NMOM];
            sum_wave_partials<NMOM / 4, 4>(red_mom, body_waves_s[2 * lane], body_waves_s[2 * lane + 1], T);
            const float Mb = body_M_s[lane], im = frcp(Mb);
            float cb[3], Db[3], cab[3], dvb[3] = {0.0f, 0.0f, 0.0f}, wb[3] = {0.0f, 0.0f, 0.0f};
            for (int j = 0; j < 3; ++j) {
                cb[j] = T[j] * im;
                Db[j] = T[3 + j] * im;
                cab[j] = cb[j] + Db[j];
            }
            if (!(c.flags & kFlagNoLinMom))
                for (int j = 0; j < 3; ++j) dvb[j] = -T[3 + j] * c.inv_h * im;
            if (!(c.flags & kFlagNoAngMom)) {
                float cbxD[3], DbxP[3], dL[3], I6[6];
                cross(cb, &T[3], cbxD);
                cross(Db, &T[6], DbxP);
                for (int j = 0; j < 3; ++j) dL[j] = (T[9 + j] - cbxD[j]) * c.inv_h + T[12 + j] - DbxP[j];
                I6[0] = T[15] - Mb * (cab[1] * cab[1] + cab[2] * cab[2]);
                I6[1] = T[16] - Mb * (cab[0] * cab[0] + cab[2] * cab[2]);
                I6[2] = T[17] - Mb * (cab[0] * cab[0] + cab[1] * cab[1]);
                I6[3] = T[18] + Mb * cab[0] * cab[1];
                I6[4] = T[19] + Mb * cab[0] * cab[2];
                I6[5] = T[20] + Mb * cab[1] * cab[2];
                const float scale = fmaxf(I6[0] + I6[1] + I6[2], Mb * c.two_r * c.two_r);
                solve_inertia(I6, dL, scale, wb);
            }
            for (int j = 0; j < 3; ++j) {
                body_mom[lane * 9 + j] = dvb[j];
                body_mom[lane * 9 + 3 + j] = wb[j];
                body_mom[lane * 9 + 6 + j] = cab[j];
            }
        }
        __syncthreads();
        if (act) {
            float dv[3], w[3], ca[3], ra[3], wr[3];
            for (int j = 0; j < 3; ++j) {
                dv[j] = body_mom[lb * 9 + j];
                w[j] = body_mom[lb * 9 + 3 + j];
                ca[j] = body_mom[lb * 9 + 6 + j];
            }
            for (int j = 0; j < 3; ++j) ra[j] = za[j] - ca[j];
            cross(w, ra, wr);
            for (int j = 0; j < 3; ++j) {
                const float dvi = dv[j] - wr[j];
                const float dnew = (del[j] + step[j]) + c.h * dvi;
                if (c.flags & kFlagStdVelocity) {
                    const float x0j = p_const[j][tid];
                    const float xw = x0j + dnew;
                    V[j] = (xw - x0j) * c.inv_h;
                } else {
                    V[j] = (V[j] + step[j] * c.inv_h) + dvi;
                }
                del[j] = dnew;
            }
        }
        if (it + 1 < K && act && cnt > 0u) {   // publish X_{it+1} for the partners
            unsigned long long* tn = s.tagged + (size_t)((it + 1) & 1) * 3 * n;
            const unsigned long long tag = (unsigned long long)iter_tag(epoch, it + 1) << 32;
            for (int j = 0; j < 3; ++j)
                __hip_atomic_store(&tn[j * n + i], tag | __float_as_uint(del[j]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // X_K - X_init and V_K where the finalize step reads them
    if (act) {
        float* dn = s.dl[K & 1];
        float* vn = s.vel[K & 1];
        for (int j = 0; j < 3; ++j) {
            dn[j * n + i] = del[j];
            vn[j * n + i] = V[j];
        }
    }
    if (body_lane && s.body_rot)
        for (int j = 0; j < 9; ++j) s.body_rot[9 * (size_t)(blk_b0 + lane) + j] = body_sm[lane * 12 + j];
}

// End of a frame, in two launches so that a frame is committed whole or not
// at all: k_check latches a non-finite X_K or V_K; k_commit then writes
// x = X_init + (X_K - X_init), v = V_K as the new state only if no error has
// been latched (in this frame or before), so after an error the state stays
// at the last frame completed without one.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_check(Scene s, int src)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    if (MULTI) {
        const int32_t sc = s.pscene[i];
        if (sc < 0 || !s.mscene[sc].active) return;
    }
    const size_t n = (size_t)s.n;
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
        const size_t j = k * n + i;
        finite = finite && isfinite(s.x0[j] + s.dl[src][j]) && isfinite(s.vel[src][j]);
    }
    if (!finite) atomicOr(&s.counters->err, kErrNonFinite);
}

template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_commit(Scene s, int src)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    if (__hip_atomic_load(&s.counters->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrDiscard) return;
    if (MULTI) {
        const int32_t sc = s.pscene[i];
        if (sc < 0 || !s.mscene[sc].active) return;
    }
    const size_t n = (size_t)s.n;
    for (int k = 0; k < 3; ++k) {
        const size_t j = k * n + i;
        s.x[j] = s.x0[j] + s.dl[src][j];
        s.v[j] = s.vel[src][j];
    }
}

__global__ void __launch_bounds__(kBlock) k_clear_counters(Counters* c, NbrStats* st, uint32_t n_slots)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) c->err = 0u;
    if (i < n_slots) {
        st[i].max_nbr = 0u;
        st[i].sum = 0ull;
        st[i].rows = 0ull;
    }
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* p, size_t words)
{
    const size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x;
    if (i < words) p[i] = 0u;
}

__global__ void __launch_bounds__(64) k_next_epoch(Counters* c)
{
    if (threadIdx.x == 0) c->epoch += 1u;
}

__global__ void __launch_bounds__(kBlock) k_init_tables(Scene s, size_t table)
{
    const size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x;
    if (i < table) s.cells[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i < (size_t)(kMaxRadixPasses * kRadixBins)) s.hist[i] = 0u;
    if (i == 0) s.counters->epoch = 0u;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_iterate(const Scene& s, const StepConsts& c, int src, int it, hipStream_t stream)
{
    const dim3 grid(s.n_iter_blocks), block(64 * s.waves_per_block);
    if (s.pscene) {         // multi-scene mode: a body's arithmetic does not depend on the mix
        if (s.wide_bodies)
            hipLaunchKernelGGL((k_iterate<true, true>), grid, block, 0, stream, s, c, src, it);
        else
            hipLaunchKernelGGL((k_iterate<true, false>), grid, block, 0, stream, s, c, src, it);
    } else if (s.dense_iterate) {
        hipLaunchKernelGGL(k_iterate_dense, grid, block, 0, stream, s, c, src, it);
    } else if (s.wide_bodies) {
        hipLaunchKernelGGL((k_iterate<false, true>), grid, block, 0, stream, s, c, src, it);
    } else {
        hipLaunchKernelGGL((k_iterate<false, false>), grid, block, 0, stream, s, c, src, it);
    }
}

// The same launch with a pair of events bound to the dispatch itself: their
// timestamps are the kernel's own begin and end, with no marker packets between.
void launch_iterate_timed(const Scene& s, const StepConsts& c, int src, int it, hipStream_t stream, hipEvent_t t0,
                          hipEvent_t t1)
{
    const dim3 grid(s.n_iter_blocks), block(64 * s.waves_per_block);
    if (s.dense_iterate)
        hipExtLaunchKernelGGL(k_iterate_dense, grid, block, 0, stream, t0, t1, 0, s, c, src, it);
    else if (s.wide_bodies)
        hipExtLaunchKernelGGL((k_iterate<false, true>), grid, block, 0, stream, t0, t1, 0, s, c, src, it);
    else
        hipExtLaunchKernelGGL((k_iterate<false, false>), grid, block, 0, stream, t0, t1, 0, s, c, src, it);
}

}  // namespace

hipError_t enqueue_zero(void* p, size_t bytes, hipStream_t stream)
{
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words)), dim3(kBlock), 0, stream, (uint32_t*)p, words);
    return hipGetLastError();
}

hipError_t enqueue_clear_counters(const Scene& s, hipStream_t stream)
{
    const uint32_t slots = (uint32_t)blocks_for((size_t)s.n);
    hipLaunchKernelGGL(k_clear_counters, dim3(blocks_for(slots > 0 ? slots : 1)), dim3(kBlock), 0, stream, s.counters,
                       s.nbr_stats, slots);
    return hipGetLastError();
}

hipError_t enqueue_init_tables(const Scene& s, size_t table, hipStream_t stream)
{
    size_t items = table;
    items = items > (size_t)(kMaxRadixPasses * kRadixBins) ? items : (size_t)(kMaxRadixPasses * kRadixBins);
    hipLaunchKernelGGL(k_init_tables, dim3(blocks_for(items)), dim3(kBlock), 0, stream, s, table);
    return hipGetLastError();
}

hipError_t enqueue_iterations(const Scene& s, const StepConsts& c, int iterations, int count, hipStream_t stream)
{
    if (s.n <= 0 || count <= 0) return hipSuccess;
    if (s.resident_iterate) {       // each launch: all K iterations
        for (int k = 0; k < count; ++k) {
            hipLaunchKernelGGL(k_next_epoch, dim3(1), dim3(64), 0, stream, s.counters);
            hipLaunchKernelGGL(k_iterate_resident, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s,
                               c, iterations);
        }
        return hipGetLastError();
    }
    int src = 0;
    for (int it = 0; it < count; ++it) {
        launch_iterate(s, c, src, it, stream);
        src ^= 1;
    }
    return hipGetLastError();
}

hipError_t enqueue_iterations_timed(const Scene& s, const StepConsts& c, int iterations, int count,
                                    hipStream_t stream, const hipEvent_t* t0, const hipEvent_t* t1)
{
    if (s.n <= 0 || count <= 0) return hipSuccess;
    if (s.resident_iterate) {       // each launch: all K iterations; the new epoch is set outside the events
        for (int k = 0; k < count; ++k) {
            hipLaunchKernelGGL(k_next_epoch, dim3(1), dim3(64), 0, stream, s.counters);
            hipExtLaunchKernelGGL(k_iterate_resident, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream,
                                  t0[k], t1[k], 0, s, c, iterations);
        }
        return hipGetLastError();
    }
    int src = 0;
    for (int it = 0; it < count; ++it) {
        launch_iterate_timed(s, c, src, it, stream, t0[it], t1[it]);
        src ^= 1;
    }
    return hipGetLastError();
}

int resident_iterate_capacity(int waves_per_block)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_iterate_resident, 64 * waves_per_block, 0) !=
        hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t enqueue_substeps(const Scene& s, const StepConsts& c, int iterations, int count, hipStream_t stream)
{
    if (s.n <= 0 || count <= 0) return hipSuccess;
    const bool multi = s.pscene != nullptr;
    if (multi && s.n_active <= 0) return hipSuccess;
    // multi-scene mode: the particle kernels cover the arena up to its last
    // scene, the neighbour kernel the stepped particles only (its workgroups
    // are renumbered across XCDs, so the grid must hold no idle tail)
    const size_t extent = multi ? (size_t)s.n_extent : (size_t)s.n;
    const unsigned nb = blocks_for(extent);
    const unsigned nb_nbr = multi ? blocks_for((size_t)s.n_active) : nb;
    const size_t pred_items = (size_t)(kMaxRadixPasses * kRadixBins);
    const unsigned nb_pred = blocks_for(extent > pred_items ? extent : pred_items);
    const int hist_threads = radix_hist_threads_for((size_t)s.n_sort);
    const size_t hist_chunk = 16 * (size_t)hist_threads;
    const unsigned nb_hist = (unsigned)(((size_t)s.n_sort + hist_chunk - 1) / hist_chunk);
    const int last = iterations % 2;      // buffer holding X_K - X_init and V_K
    for (int sub = 0; sub < count; ++sub) {
        if (multi)
            hipLaunchKernelGGL(k_predict_keys<true>, dim3(nb_pred), dim3(kBlock), 0, stream, s, c, sub == 0 ? -1 : last);
        else
            hipLaunchKernelGGL(k_predict_keys<false>, dim3(nb_pred), dim3(kBlock), 0, stream, s, c,
                               sub == 0 ? -1 : last);
        // (key, id) sorted by key, stable: digit counts, then one pass per digit
        if (hist_threads == 1024)
            hipLaunchKernelGGL(k_radix_hist<1024>, dim3(nb_hist), dim3(1024), 0, stream, s);
        else
            hipLaunchKernelGGL(k_radix_hist<256>, dim3(nb_hist), dim3(256), 0, stream, s);
        for (int p = 0; p < s.radix_passes; ++p) {
            const uint32_t* kin = p == 0 ? s.key : s.kbuf[(p - 1) & 1];
            const uint32_t* iin = p == 0 ? nullptr : s.ibuf[(p - 1) & 1];
            const dim3 tiles(s.n_radix_tiles);
            // (the first pass's tile counts come from the histogram launch)
            if (s.radix_items == 16) {
                if (p > 0) hipLaunchKernelGGL(k_radix_count<16>, tiles, dim3(kBlock), 0, stream, s, p, kin);
                hipLaunchKernelGGL(k_radix_scan, dim3(kRadixBins), dim3(kBlock), 0, stream, s, p);
                hipLaunchKernelGGL(k_radix_scatter<16>, tiles, dim3(kBlock), 0, stream, s, p, kin, iin,
                                   s.kbuf[p & 1], s.ibuf[p & 1]);
            } else {
                if (p > 0) hipLaunchKernelGGL(k_radix_count<4>, tiles, dim3(kBlock), 0, stream, s, p, kin);
                hipLaunchKernelGGL(k_radix_scan, dim3(kRadixBins), dim3(kBlock), 0, stream, s, p);
                hipLaunchKernelGGL(k_radix_scatter<4>, tiles, dim3(kBlock), 0, stream, s, p, kin, iin,
                                   s.kbuf[p & 1], s.ibuf[p & 1]);
            }
        }
        if (multi) {
            hipLaunchKernelGGL(k_cells<true>, dim3(nb_nbr), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_neighbours<true>, dim3(nb_nbr), dim3(kBlock), 0, stream, s, c);
        } else {
            hipLaunchKernelGGL(k_cells<false>, dim3(nb), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_neighbours<false>, dim3(nb), dim3(kBlock), 0, stream, s, c);
        }
        if (!multi && s.resident_iterate) {
            hipLaunchKernelGGL(k_iterate_resident, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s,
                               c, iterations);
            continue;
        }
        int src = 0;
        for (int it = 0; it < iterations; ++it) {
            launch_iterate(s, c, src, it, stream);
            src ^= 1;
        }
    }
    if (multi) {
        hipLaunchKernelGGL(k_check<true>, dim3(nb), dim3(kBlock), 0, stream, s, last);
        hipLaunchKernelGGL(k_commit<true>, dim3(nb), dim3(kBlock), 0, stream, s, last);
    } else {
        hipLaunchKernelGGL(k_check<false>, dim3(nb), dim3(kBlock), 0, stream, s, last);
        hipLaunchKernelGGL(k_commit<false>, dim3(nb), dim3(kBlock), 0, stream, s, last);
    }
    return hipGetLastError();
}

}  // namespace pbdr
