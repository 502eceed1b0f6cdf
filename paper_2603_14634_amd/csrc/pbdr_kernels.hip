// PBD-R solver substep on gfx950 (MI355X).
//
// One substep of Alg. 1 of "Physically Accurate Rigid-Body Dynamics in
// Particle-Based Simulation" (arXiv 2603.14634) as a chain of kernels on one
// stream:
//
//   predict_keys   integration step (Alg. 1, first loop), hash-grid key and
//                  per-key slot of every particle (atomic counting pass); from
//                  the second substep of a call on, it first folds the previous
//                  substep's result into the state (x += dX, v = V)
//   scan           exclusive prefix sum of the per-key counts in one launch
//                  (decoupled look-back) -> per-key first slot and count;
//                  re-zeroes the counts
//   scatter        particles grouped by key, with sorted copies of the FP32
//                  predicted positions and body ids, and each key's body
//                  signature (its single body, or "mixed")
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

// ---------------------------------------------------------------------------
// integration step + keys + counting pass
// ---------------------------------------------------------------------------

// MULTI: multi-scene mode (Scene::pscene set); a separate instance, so that
// the single-scene kernels carry none of its checks.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_predict_keys(Scene s, StepConsts c, int fold_src)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < (int)s.n_scan_tiles) s.tile_state[i] = 0ull;   // scan look-back state of this substep
    if (!MULTI && i == 0) s.counters->epoch += 1u;      // a new substep: fresh tags for one-launch iterations
    if (i >= s.n) return;
    const size_t n = (size_t)s.n;
    const MultiScene* ms = nullptr;
    if (MULTI) {                       // this particle's scene, if stepped
        const int32_t sc = s.pscene[i];
        if (sc < 0 || !s.mscene[sc].active) return;
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
    const uint32_t key = (ms ? ms->key_base : 0u) + morton(cell_axis(xt[0], c.origin[0], c.inv_cell),
                                                           cell_axis(xt[1], c.origin[1], c.inv_cell),
                                                           cell_axis(xt[2], c.origin[2], c.inv_cell),
                                                           ms ? ms->key_mask : c.key_mask);
    s.key[i] = key;
    s.rank[i] = atomicAdd(&s.cell_count[key], 1u);
}

// ---------------------------------------------------------------------------
// exclusive scan of the cell counts in one launch (decoupled look-back: each
// tile publishes its total at once and its inclusive prefix as soon as it is
// known; a wave inspects 64 predecessors per step)
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

// Sum over the 64 lanes of a wave, returned to every lane: row sums by DPP,
// the four row sums gathered in lane 63 by row broadcasts, then read out.
__device__ inline uint32_t wave_total(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false);  // row_half_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false);  // row_mirror
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Exclusive prefix sums of N values per thread over the workgroup, each value
// scanned on its own (the N scans share one barrier).  tot[k] receives the
// workgroup total of value k.
template <int N>
__device__ inline void block_exclusive_scans(const uint32_t* v, uint32_t (*wave_tot)[kWaves], uint32_t* excl,
                                             uint32_t* tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl[N];
#pragma unroll
    for (int k = 0; k < N; ++k) incl[k] = wave_inclusive_scan(v[k]);
    if (lane == 63)
#pragma unroll
        for (int k = 0; k < N; ++k) wave_tot[k][wave] = incl[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        uint32_t before = 0, all = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) before += wave_tot[k][w];
            all += wave_tot[k][w];
        }
        excl[k] = before + incl[k] - v[k];
        tot[k] = all;
    }
}

constexpr unsigned long long kTileAggregate = 1ull << 32, kTileInclusive = 2ull << 32;
constexpr uint32_t kSpinLimit = 1u << 22;   // bounded wait: flag an error, never hang

// A tile is kScanTile keys in kChunks chunks of 4 keys per thread, so every
// count load and entry store of a chunk is one contiguous, coalesced access.
constexpr int kChunks = kScanTile / (4 * kBlock);

__global__ void __launch_bounds__(kBlock) k_scan(Scene s)
{
    __shared__ uint32_t wave_tot[kChunks][kWaves];
    __shared__ uint32_t s_prefix;
    // workgroups are dispatched in index order, so a tile only waits on tiles
    // that already run; the wait is bounded all the same
    const uint32_t tile = blockIdx.x;
    const size_t tbase = (size_t)tile * kScanTile;
    uint32_t vals[kChunks][4], csum[kChunks], excl[kChunks], chunk_tot[kChunks];
    // all chunks are loaded before any is scanned, so their loads overlap
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
        const size_t base = tbase + (size_t)ch * 4 * kBlock + 4 * (size_t)threadIdx.x;
        if (base + 3 < s.T) {
            const uint4 v = *(const uint4*)&s.cell_count[base];
            vals[ch][0] = v.x; vals[ch][1] = v.y; vals[ch][2] = v.z; vals[ch][3] = v.w;
        } else {
            for (int k = 0; k < 4; ++k) vals[ch][k] = base + k < s.T ? s.cell_count[base + k] : 0u;
        }
    }
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {       // counts ready for the next substep
        const size_t base = tbase + (size_t)ch * 4 * kBlock + 4 * (size_t)threadIdx.x;
        if (base + 3 < s.T) {
            *(uint4*)&s.cell_count[base] = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (int k = 0; k < 4; ++k)
                if (base + k < s.T) s.cell_count[base + k] = 0u;
        }
        csum[ch] = vals[ch][0] + vals[ch][1] + vals[ch][2] + vals[ch][3];
    }
    block_exclusive_scans<kChunks>(csum, wave_tot, excl, chunk_tot);
    uint32_t total = 0;
    for (int ch = 0; ch < kChunks; ++ch) total += chunk_tot[ch];
    if (threadIdx.x < 64) {                       // wave 0: publish and look back
        const int lane = threadIdx.x;
        uint32_t prefix = 0;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&s.tile_state[0], kTileInclusive | total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&s.tile_state[tile], kTileAggregate | total, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int top = (int)tile - 1;               // newest predecessor not yet summed
            uint32_t spins = 0;
            while (true) {
                const int t = top - lane;
                const unsigned long long st =
                    t >= 0 ? __hip_atomic_load(&s.tile_state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : kTileInclusive;
                const uint32_t status = (uint32_t)(st >> 32);
                const unsigned long long incl = __ballot(status == 2u);
                const unsigned long long empty = __ballot(status == 0u);
                const int stop = incl ? __ffsll((long long)incl) - 1 : 63;   // lanes 0..stop matter
                const unsigned long long mask = stop == 63 ? ~0ull : ((1ull << (stop + 1)) - 1ull);
                if (empty & mask) {               // a predecessor has not published yet
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(&s.counters->err, kErrInternal);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint32_t v = lane <= stop ? (uint32_t)st : 0u;
                prefix += wave_total(v);
                if (incl) break;
                top -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&s.tile_state[tile], kTileInclusive | (prefix + total), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    uint32_t run_chunk = s_prefix;
    for (int ch = 0; ch < kChunks; ++ch) {
        const size_t base = tbase + (size_t)ch * 4 * kBlock + 4 * (size_t)threadIdx.x;
        uint32_t run = run_chunk + excl[ch];
        for (int k = 0; k < 4; ++k) {
            if (base + k < s.T) s.cells[base + k] = make_uint2(run, 0xffffffffu);   // signature: empty
            run += vals[ch][k];
        }
        run_chunk += chunk_tot[ch];
    }
    // end sentinel: the number of particles grouped (all of them, or in
    // multi-scene mode those stepped)
    if (tile == gridDim.x - 1 && threadIdx.x == 0) s.cells[s.T] = make_uint2(s_prefix + total, 0xffffffffu);
}

template <bool MULTI>
__global__ void __launch_bounds__(kBlock) k_scatter(Scene s)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    if (MULTI) {                       // stepped particles only
        const int32_t sc = s.pscene[i];
        if (sc < 0 || !s.mscene[sc].active) return;
    }
    const size_t n = (size_t)s.n;
    const uint32_t key = s.key[i];
    const uint32_t slot = s.cells[key].x + s.rank[i];
    const int32_t b = s.body[i];
    s.sorted_raw[slot] = (uint32_t)i;
    s.sxt4[slot] = make_float4(s.xt[i], s.xt[n + i], s.xt[2 * n + i], __int_as_float(b));
    // body signature of the key: the one body of all its particles, or -2
    int* sig = (int*)&s.cells[key].y;
    const int32_t old = atomicCAS(sig, -1, b);
    if (old != -1 && old != b && old != -2) atomicExch(sig, -2);
}

// ---------------------------------------------------------------------------
// neighbour lists, one thread per particle in key order
// ---------------------------------------------------------------------------

// At most 128 VGPRs (4 waves per SIMD, no spill): the 27 key ranges and 9
// candidates in flight otherwise take ~156 and leave 3 waves per SIMD.
template <bool MULTI>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_neighbours(Scene s, StepConsts c)
{
    extern __shared__ uint32_t lst[];          // [cap][kBlock], slot-major
    const int blk = xcd_block();
    const int j = blk * kBlock + threadIdx.x;  // position in key order
    // multi-scene mode: the key order holds the stepped particles only
    bool live = j < (MULTI ? (int)s.cells[s.T].x : s.n);
    const size_t n = (size_t)s.n;
    const int cap = c.nbr_cap;
    const int tid = threadIdx.x;
    uint32_t count = 0;
    uint32_t i = live ? s.sorted_raw[j] : 0u;
    uint32_t key_base = 0u, key_mask = c.key_mask;
    if (MULTI && live) {                // multi-scene mode: the particle's own scene table
        const int32_t sc = s.pscene[i];
        key_base = s.mscene[sc].key_base;
        key_mask = s.mscene[sc].key_mask;
    }
    if (live) {
        const float4 me = s.sxt4[j];
        const float px = me.x, py = me.y, pz = me.z;
        const int32_t pb = __float_as_int(me.w);
        const uint32_t cx = cell_axis(px, c.origin[0], c.inv_cell);
        const uint32_t cy = cell_axis(py, c.origin[1], c.inv_cell);
        const uint32_t cz = cell_axis(pz, c.origin[2], c.inv_cell);
        uint32_t lo[27], hi[27];
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const uint32_t k = key_base + morton(cx + (uint32_t)(t % 3 - 1), cy + (uint32_t)((t / 3) % 3 - 1),
                                                 cz + (uint32_t)(t / 9 - 1), key_mask);
            const uint2 e = s.cells[k];
            const uint32_t end = s.cells[k + 1].x;
            lo[t] = e.x;
            // a key holding only this particle's body has no candidates
            hi[t] = (int32_t)e.y == pb ? e.x : end;
        }
        auto consider = [&](uint32_t q, const float4 o) {
            if (__float_as_int(o.w) == pb) return;            // same body (also excludes i)
            if (!within(px, py, pz, o.x, o.y, o.z, c.search_r2)) return;
            const uint32_t id = s.sorted_raw[q];
            // insert keeping the `cap` smallest ids in ascending order
            const int m = (int)(count < (uint32_t)cap ? count : (uint32_t)cap);
            ++count;
            if (m == cap && id > lst[(cap - 1) * kBlock + tid]) return;
            int pos = (m == cap) ? cap - 1 : m;
            while (pos > 0 && lst[(pos - 1) * kBlock + tid] > id) {
                lst[pos * kBlock + tid] = lst[(pos - 1) * kBlock + tid];
                --pos;
            }
            lst[pos * kBlock + tid] = id;
        };
        // one z-layer of 9 keys at a time: the first candidate of every key is
        // loaded before any is examined, so the loads are in flight together;
        // further candidates of a key (rare with >= 8 keys per particle) follow
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            float4 o[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                const int t = 9 * dz + u;
                o[u] = hi[t] > lo[t] ? s.sxt4[lo[t]] : me;
            }
#pragma unroll
            for (int u = 0; u < 9; ++u) {
                const int t = 9 * dz + u;
                if (hi[t] > lo[t]) {
                    consider(lo[t], o[u]);
                    for (uint32_t q = lo[t] + 1; q < hi[t]; ++q) consider(q, s.sxt4[q]);
                }
            }
        }
        s.nbr_n[i] = count;
        const uint32_t stored = count < (uint32_t)cap ? count : (uint32_t)cap;
        for (uint32_t k = 0; k < stored; ++k) s.nbr[k * n + i] = lst[k * kBlock + tid];
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

// Contact with a particle of another body (constraint (2)) from X_i: the
// mass-weighted split of the penetration, Coulomb friction from the relative
// displacement since X_init, and the pair weight of the averaging mode.  xq,
// dq: the partner's X_init and X_i - X_init; mq, nq: its mass and list length.
// Shared by both iteration kernels, with contraction limited to single
// expressions, so that both round alike.
__device__ __forceinline__ void pair_correction(const StepConsts& c, uint32_t avg, float mu, const float* x0,
                                                const float* del, float m, uint32_t ni, const float* xq,
                                                const float* dq, float mq, uint32_t nq, float* Cd)
{
#pragma clang fp contract(on)
    float d[3], u[3];
    for (int j = 0; j < 3; ++j) {
        d[j] = (x0[j] - xq[j]) + (del[j] - dq[j]);
        u[j] = del[j] - dq[j];
    }
    const float l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const float l = __builtin_amdgcn_sqrtf(l2);
    if (!(l > 0.0f) || !(l < c.two_r)) return;
    const float il = frcp(l);
    const float nx = d[0] * il, ny = d[1] * il, nz = d[2] * il;
    const float pen = c.two_r - l;
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
    const float sc = alpha * wgt;
    Cd[0] += sc * (pen * nx - f * ux);
    Cd[1] += sc * (pen * ny - f * uy);
    Cd[2] += sc * (pen * nz - f * uz);
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

// Bodies are packed into workgroups of W waves; each body owns ceil(n/64)
// consecutive waves, one particle per lane.  Per-body sums are wave sums (lane swaps, DPP)
// combined over the body's waves; the per-body 3x3 algebra runs on lane j of
// wave 0 for the j-th body of the workgroup.  `it` is the iteration index in
// the substep: from the second iteration on, the rotation is refined from the
// previous iteration's.  SM_UNROLL / MOM_UNROLL: waves whose partial sums the
// per-body lane reads from LDS at once.
template <bool MULTI, int SM_UNROLL, int MOM_UNROLL>
__device__ __forceinline__ void iterate_body(const Scene& s, const StepConsts& c, int src, int it)
{
    constexpr int NSM = 12, NMOM = 24;          // per-wave partial sums (float4 aligned; 21 used)
    __shared__ float4 red_sm[kMaxWaves * NSM / 4];
    __shared__ float4 red_mom[kMaxWaves * NMOM / 4];
    __shared__ float body_sm[kMaxWaves * 12];    // per body of the workgroup: R (9), centre (3)
    __shared__ float body_mom[kMaxWaves * 9];    // dv (3), omega (3), c_asm - c_i (3)

    // the wave index as a wave-uniform (scalar) value: the per-wave table and
    // body entries below then come through scalar loads
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int blk = xcd_block();
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
    const size_t n = (size_t)s.n;
    const float* dl = s.dl[src];
    const float* vl = s.vel[src];
    float* dn = s.dl[src ^ 1];
    float* vn = s.vel[src ^ 1];
    const float ax = s.x0[s0], ay = s.x0[n + s0], az = s.x0[2 * n + s0];   // body anchor
    const uint32_t avg = (c.flags >> kAvgShift) & 3u;

    // per-body lane of wave 0: body slot `lane` of this workgroup
    const bool body_lane = wave == 0 && lane < blk_nb;
    const int bb = blk_b0 + (body_lane ? lane : 0);
    int bl_w0 = 0, bl_nw = 0;
    float bl_M = 1.0f, Rprev[9], mq3[3];
    if (body_lane) {
        bl_w0 = s.body_wave0[bb] - blk * s.waves_per_block;
        bl_nw = (s.body_start[bb + 1] - s.body_start[bb] + 63) >> 6;
        bl_M = s.body_mass[bb];
        for (int j = 0; j < 3; ++j) mq3[j] = s.body_mq[3 * (size_t)bb + j];
        if (it > 0)
            for (int j = 0; j < 9; ++j) Rprev[j] = s.body_rot[9 * (size_t)bb + j];
    }

    float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, V[3] = {0.0f, 0.0f, 0.0f};
    float q[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f, Cd[3] = {0.0f, 0.0f, 0.0f};
    if (act) {
        for (int j = 0; j < 3; ++j) {
            x0[j] = s.x0[j * n + i];
            del[j] = dl[j * n + i];
            V[j] = vl[j * n + i];
            q[j] = s.q[j * n + i];
        }
        m = s.mass[i];
    }

    // contacts, from X_i (Jacobi): planes (constraint (1)) and particles of
    // other bodies (constraint (2)); friction from the displacement since X_init
    if (act) {
        const float mu = MULTI ? s.mscene[s.pscene[i]].mu : c.mu;   // multi-scene mode: per scene
        for (int pl = 0; pl < c.n_planes; ++pl) {
            const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
            const float un = nx * del[0] + ny * del[1] + nz * del[2];
            const float e = ((nx * x0[0] + ny * x0[1] + nz * x0[2]) - c.plane_d[pl]) + un;
            if (!(e < c.radius)) continue;
            const float pen = c.radius - e;
            const float ux = del[0] - un * nx, uy = del[1] - un * ny, uz = del[2] - un * nz;
            const float ut2 = ux * ux + uy * uy + uz * uz;
            const float f = ut2 > 0.0f ? fminf(1.0f, mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
            Cd[0] += pen * nx - f * ux;
            Cd[1] += pen * ny - f * uy;
            Cd[2] += pen * nz - f * uz;
        }
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

    // shape matching on X_i: centre and covariance in one reduction,
    // A = sum m (x - c) q^T = sum m y q^T - c (sum m q)^T, y = x - anchor
    float y[3];
    y[0] = (x0[0] - ax) + del[0];
    y[1] = (x0[1] - ay) + del[1];
    y[2] = (x0[2] - az) + del[2];
    {
        float S[NSM];
        for (int j = 0; j < 3; ++j) S[j] = m * y[j];
        for (int a = 0; a < 3; ++a)
            for (int k2 = 0; k2 < 3; ++k2) S[3 + 3 * a + k2] = m * y[a] * q[k2];
        wave_sums_by_row<NSM>(S);
        if ((lane & 15) == 15) {      // row j holds sums j NSM/4 .. j NSM/4 + NSM/4 - 1
            float* dst = (float*)red_sm + wave * NSM + (lane >> 4) * (NSM / 4);
            for (int j = 0; j < NSM / 4; ++j) dst[j] = S[j];
        }
    }
    __syncthreads();
    if (body_lane) {            // one lane per body: centre, covariance, rotation
        float T[NSM];
        sum_wave_partials<NSM / 4, SM_UNROLL>(red_sm, bl_w0, bl_nw, T);
        const float im = frcp(bl_M);
        float cc[3], A[9], Rb[9];
        for (int j = 0; j < 3; ++j) cc[j] = T[j] * im;
        for (int a = 0; a < 3; ++a)
            for (int k2 = 0; k2 < 3; ++k2) A[3 * a + k2] = T[3 + 3 * a + k2] - cc[a] * mq3[k2];
        if (!(it > 0 && polar_refine(A, Rprev, Rb))) polar_rotation(A, Rb);
        for (int j = 0; j < 9; ++j) body_sm[lane * 12 + j] = Rb[j];
        for (int j = 0; j < 3; ++j) body_sm[lane * 12 + 9 + j] = cc[j];
        if (s.body_rot)
            for (int j = 0; j < 9; ++j) s.body_rot[9 * (size_t)bb + j] = Rb[j];
    }
    __syncthreads();
    float R[9], cyv[3];
    for (int j = 0; j < 9; ++j) R[j] = body_sm[lb * 12 + j];
    for (int j = 0; j < 3; ++j) cyv[j] = body_sm[lb * 12 + 9 + j];

    // goal offsets D = R q - (x - c) and the momentum sums, in the frame
    // centred on c_i: z_b = r + C (before shape matching), z_a = z_b + D
    float r[3], Dd[3];
    for (int j = 0; j < 3; ++j) r[j] = y[j] - cyv[j];
    for (int a = 0; a < 3; ++a)
        Dd[a] = act ? (R[3 * a] * q[0] + R[3 * a + 1] * q[1] + R[3 * a + 2] * q[2]) - r[a] : 0.0f;
    {
        float S[NMOM];
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
        wave_sums_by_row<NMOM>(S);
        if ((lane & 15) == 15) {
            float* dst = (float*)red_mom + wave * NMOM + (lane >> 4) * (NMOM / 4);
            for (int j = 0; j < NMOM / 4; ++j) dst[j] = S[j];
        }
    }
    __syncthreads();

    // momentum conservation constraint, one lane per body
    if (body_lane) {
        float T[NMOM];
        sum_wave_partials<NMOM / 4, MOM_UNROLL>(red_mom, bl_w0, bl_nw, T);
        const float Mb = bl_M, im = frcp(Mb);
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
            body_mom[lane * 9 + j] = dvb[j];
            body_mom[lane * 9 + 3 + j] = wb[j];
            body_mom[lane * 9 + 6 + j] = cab[j];
        }
    }
    __syncthreads();
    if (!act) return;
    float dv[3], w[3], ca[3];
    for (int j = 0; j < 3; ++j) {
        dv[j] = body_mom[lb * 9 + j];
        w[j] = body_mom[lb * 9 + 3 + j];
        ca[j] = body_mom[lb * 9 + 6 + j];
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

// The iteration kernel in two register budgets: the compiler's choice (about
// 85 VGPRs, fastest when the grid fits the GPU at once), and at most 80 VGPRs
// (6 waves per SIMD, a few values spilled) for grids that oversubscribe it,
// where more workgroups per CU hide each other's per-body phases.
template <bool MULTI>
__global__ void __launch_bounds__(64 * kMaxWaves) k_iterate(Scene s, StepConsts c, int src, int it)
{
    iterate_body<MULTI, 4, 4>(s, c, src, it);
}

__global__ void __launch_bounds__(64 * kMaxWaves) __attribute__((amdgpu_waves_per_eu(6, 6)))
k_iterate_dense(Scene s, StepConsts c, int src, int it)
{
    iterate_body<false, 2, 2>(s, c, src, it);
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
    __shared__ float4 red_mom[kMaxWaves * NMOM / 4];
    __shared__ float body_sm[kMaxWaves * 12];
    __shared__ float body_mom[kMaxWaves * 9];

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
    const size_t n = (size_t)s.n;
    const float ax = s.x0[s0], ay = s.x0[n + s0], az = s.x0[2 * n + s0];   // body anchor
    const uint32_t avg = (c.flags >> kAvgShift) & 3u;

    const bool body_lane = wave == 0 && lane < blk_nb;
    const int bb = blk_b0 + (body_lane ? lane : 0);
    int bl_w0 = 0, bl_nw = 0;
    float bl_M = 1.0f, Rprev[9], mq3[3];
    if (body_lane) {
        bl_w0 = s.body_wave0[bb] - blk * W;
        bl_nw = (s.body_start[bb + 1] - s.body_start[bb] + 63) >> 6;
        bl_M = s.body_mass[bb];
        for (int j = 0; j < 3; ++j) mq3[j] = s.body_mq[3 * (size_t)bb + j];
    }

    // X_0 - X_init and V_0 from the integration step; the rest is constant
    float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, V[3] = {0.0f, 0.0f, 0.0f};
    float q[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f;
    uint32_t ni = 0u;
    if (act) {
        for (int j = 0; j < 3; ++j) {
            x0[j] = s.x0[j * n + i];
            del[j] = s.dl[0][j * n + i];
            V[j] = s.vel[0][j * n + i];
            q[j] = s.q[j * n + i];
        }
        m = s.mass[i];
        ni = s.nbr_n[i];
    }
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
        // the first PE partners' words are loaded before the shape-matching
        // phase, which does not need them, and checked after it
        constexpr int PE = 3;
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

        float y[3];
        y[0] = (x0[0] - ax) + del[0];
        y[1] = (x0[1] - ay) + del[1];
        y[2] = (x0[2] - az) + del[2];
        {
            float S[NSM];
            for (int j = 0; j < 3; ++j) S[j] = m * y[j];
            for (int a = 0; a < 3; ++a)
                for (int k2 = 0; k2 < 3; ++k2) S[3 + 3 * a + k2] = m * y[a] * q[k2];
            wave_sums_by_row<NSM>(S);
            if ((lane & 15) == 15) {
                float* dst = (float*)red_sm + wave * NSM + (lane >> 4) * (NSM / 4);
                for (int j = 0; j < NSM / 4; ++j) dst[j] = S[j];
            }
        }
        __syncthreads();
        if (body_lane) {
            float T[NSM];
            sum_wave_partials<NSM / 4, 4>(red_sm, bl_w0, bl_nw, T);
            const float im = frcp(bl_M);
            float cc[3], A[9], Rb[9];
            for (int j = 0; j < 3; ++j) cc[j] = T[j] * im;
            for (int a = 0; a < 3; ++a)
                for (int k2 = 0; k2 < 3; ++k2) A[3 * a + k2] = T[3 + 3 * a + k2] - cc[a] * mq3[k2];
            if (!(it > 0 && polar_refine(A, Rprev, Rb))) polar_rotation(A, Rb);
            for (int j = 0; j < 9; ++j) body_sm[lane * 12 + j] = Rprev[j] = Rb[j];
            for (int j = 0; j < 3; ++j) body_sm[lane * 12 + 9 + j] = cc[j];
        }
        __syncthreads();
        float R[9], cyv[3];
        for (int j = 0; j < 9; ++j) R[j] = body_sm[lb * 12 + j];
        for (int j = 0; j < 3; ++j) cyv[j] = body_sm[lb * 12 + 9 + j];

        // contacts from X_i (planes, then partners in list order)
        float Cd[3] = {0.0f, 0.0f, 0.0f};
        if (act) {
            for (int pl = 0; pl < c.n_planes; ++pl) {
                const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
                const float un = nx * del[0] + ny * del[1] + nz * del[2];
                const float e = ((nx * x0[0] + ny * x0[1] + nz * x0[2]) - c.plane_d[pl]) + un;
                if (!(e < c.radius)) continue;
                const float pen = c.radius - e;
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


        float r[3], Dd[3];
        for (int j = 0; j < 3; ++j) r[j] = y[j] - cyv[j];
        for (int a = 0; a < 3; ++a)
            Dd[a] = act ? (R[3 * a] * q[0] + R[3 * a + 1] * q[1] + R[3 * a + 2] * q[2]) - r[a] : 0.0f;
        {
            float S[NMOM];
            float zb[3], za[3], vb[3], t[3];
            for (int j = 0; j < 3; ++j) {
                zb[j] = r[j] + Cd[j];
                za[j] = zb[j] + Dd[j];
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
            sum_wave_partials<NMOM / 4, 4>(red_mom, bl_w0, bl_nw, T);
            const float Mb = bl_M, im = frcp(Mb);
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
            for (int j = 0; j < 3; ++j) ra[j] = r[j] + Cd[j] + Dd[j] - ca[j];
            cross(w, ra, wr);
            for (int j = 0; j < 3; ++j) {
                const float step = Cd[j] + Dd[j];
                const float dvi = dv[j] - wr[j];
                const float dnew = (del[j] + step) + c.h * dvi;
                if (c.flags & kFlagStdVelocity) {
                    const float xw = x0[j] + dnew;
                    V[j] = (xw - x0[j]) * c.inv_h;
                } else {
                    V[j] = (V[j] + step * c.inv_h) + dvi;
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
        for (int j = 0; j < 9; ++j) s.body_rot[9 * (size_t)bb + j] = Rprev[j];
}

// Canonical (key, id) order from the key grouping of the last substep: the
// grouping keeps an arbitrary order inside a key (slots from atomic ranks);
// particle i goes to its key's first slot plus the number of smaller ids
// sharing its key.  Run on demand, outside the substep.
__global__ void __launch_bounds__(kBlock) k_canonical(Scene s)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= s.n) return;
    const uint32_t i = s.sorted_raw[j];
    const uint32_t k = s.key[i];
    const uint32_t b0 = s.cells[k].x, b1 = s.cells[k + 1].x;
    uint32_t below = 0;
    for (uint32_t q = b0; q < b1; ++q) below += (s.sorted_raw[q] < i) ? 1u : 0u;
    s.sorted[b0 + below] = i;
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

__global__ void __launch_bounds__(64) k_next_epoch(Counters* c)
{
    if (threadIdx.x == 0) c->epoch += 1u;
}

__global__ void __launch_bounds__(kBlock) k_init_tables(Scene s)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < s.T) s.cell_count[i] = 0u;
    if (i == 0) s.cells[s.T] = make_uint2((uint32_t)s.n, 0xffffffffu);
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_iterate(const Scene& s, const StepConsts& c, int src, int it, hipStream_t stream)
{
    if (s.pscene)           // multi-scene mode: one variant for every mix
        hipLaunchKernelGGL(k_iterate<true>, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s, c, src,
                           it);
    else if (s.dense_iterate)
        hipLaunchKernelGGL(k_iterate_dense, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s, c, src,
                           it);
    else
        hipLaunchKernelGGL(k_iterate<false>, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s, c,
                           src, it);
}

// The same launch with a pair of events bound to the dispatch itself: their
// timestamps are the kernel's own begin and end, with no marker packets between.
void launch_iterate_timed(const Scene& s, const StepConsts& c, int src, int it, hipStream_t stream, hipEvent_t t0,
                          hipEvent_t t1)
{
    if (s.dense_iterate)
        hipExtLaunchKernelGGL(k_iterate_dense, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, t0, t1,
                              0, s, c, src, it);
    else
        hipExtLaunchKernelGGL(k_iterate<false>, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, t0, t1, 0,
                              s, c, src, it);
}

}  // namespace

hipError_t enqueue_clear_counters(const Scene& s, hipStream_t stream)
{
    const uint32_t slots = (uint32_t)blocks_for((size_t)s.n);
    hipLaunchKernelGGL(k_clear_counters, dim3(blocks_for(slots > 0 ? slots : 1)), dim3(kBlock), 0, stream, s.counters,
                       s.nbr_stats, slots);
    return hipGetLastError();
}

hipError_t enqueue_init_tables(const Scene& s, hipStream_t stream)
{
    hipLaunchKernelGGL(k_init_tables, dim3(blocks_for((size_t)s.T)), dim3(kBlock), 0, stream, s);
    return hipGetLastError();
}

hipError_t enqueue_canonical_order(const Scene& s, hipStream_t stream)
{
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_canonical, dim3(blocks_for((size_t)s.n)), dim3(kBlock), 0, stream, s);
    return hipGetLastError();
}

hipError_t enqueue_iterations(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
                              hipStream_t stream)
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
        if (s2) launch_iterate(*s2, c, src, it, stream);
        src ^= 1;
    }
    return hipGetLastError();
}

hipError_t enqueue_iterations_timed(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
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
        if (s2) {       // one iteration = both launches: begin of the first, end of the second
            launch_iterate_timed(s, c, src, it, stream, t0[it], nullptr);
            launch_iterate_timed(*s2, c, src, it, stream, nullptr, t1[it]);
        } else {
            launch_iterate_timed(s, c, src, it, stream, t0[it], t1[it]);
        }
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

hipError_t enqueue_substeps(const Scene& s, const Scene* s2, const StepConsts& c, int iterations, int count,
                            hipStream_t stream)
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
    const unsigned nb_pred = blocks_for(extent > (size_t)s.n_scan_tiles ? extent : (size_t)s.n_scan_tiles);
    const size_t nbr_lds = (size_t)c.nbr_cap * kBlock * sizeof(uint32_t);
    const int last = iterations % 2;      // buffer holding X_K - X_init and V_K
    for (int sub = 0; sub < count; ++sub) {
        if (multi) {
            hipLaunchKernelGGL(k_predict_keys<true>, dim3(nb_pred), dim3(kBlock), 0, stream, s, c, sub == 0 ? -1 : last);
            hipLaunchKernelGGL(k_scan, dim3(s.n_scan_tiles), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_scatter<true>, dim3(nb), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_neighbours<true>, dim3(nb_nbr), dim3(kBlock), nbr_lds, stream, s, c);
        } else {
            hipLaunchKernelGGL(k_predict_keys<false>, dim3(nb_pred), dim3(kBlock), 0, stream, s, c,
                               sub == 0 ? -1 : last);
            hipLaunchKernelGGL(k_scan, dim3(s.n_scan_tiles), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_scatter<false>, dim3(nb), dim3(kBlock), 0, stream, s);
            hipLaunchKernelGGL(k_neighbours<false>, dim3(nb), dim3(kBlock), nbr_lds, stream, s, c);
        }
        if (!multi && s.resident_iterate) {
            hipLaunchKernelGGL(k_iterate_resident, dim3(s.n_iter_blocks), dim3(64 * s.waves_per_block), 0, stream, s,
                               c, iterations);
            continue;
        }
        int src = 0;
        for (int it = 0; it < iterations; ++it) {
            launch_iterate(s, c, src, it, stream);
            if (s2) launch_iterate(*s2, c, src, it, stream);
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
