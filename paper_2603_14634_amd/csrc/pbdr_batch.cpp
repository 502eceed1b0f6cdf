// Scene batches: many independent scenes stepped together by the
// multi-workgroup kernels of the single-scene path (every substep of Alg. 1
// spread over the whole GPU), for scenes too large for one workgroup each.
//
// All resident scenes share one workspace: particle arrays of capacity P in
// the single-scene layout ([3][P] SoA), a body arena (each scene takes its
// bodies plus one terminating entry, so body_start[b + 1] is always the end of
// body b), and a key arena in which each scene owns a hash table of its own
// (so the neighbour walk of one scene never meets another scene's particles).
// A launch steps the scenes whose `active` flag is set; the others' particles
// take no key and are left untouched.  Per call the host packs the stepped
// bodies into iteration workgroups and uploads the tables with the per-scene
// constants (gravity, friction coefficient, table range).
#include "pbdr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "pbdr_device.h"
#include "pbdr_host.h"

using pbdr::host::fail;
using pbdr::host::RangeAlloc;
using pbdr::host::Resolved;

namespace {

constexpr int kMinTableBits = 10, kMaxTableBits = 24;
constexpr int32_t kBatchMaxParticles = 1 << 24;   // keeps the key arena within 32-bit ranges

// Table bits of a scene of n particles: about four keys per particle.
int table_bits(int32_t n)
{
    int k = kMinTableBits;
    while (k < kMaxTableBits && ((size_t)1 << k) < 4 * (size_t)n) ++k;
    return k;
}

struct BLayout {
    size_t x, v, x0, mass, body, q, body_start, body_mass, body_mass64, dl0, dl1, vel0, vel1, xt, sxt4, key, kbuf0, kbuf1, ibuf0,
        ibuf1, nbr_n, nbr, hist, tile_off, cells, body_rot, counters, nbr_stats, body_mq, pscene, plan,
        total;
    size_t plan_bytes, mscene_off, wave_off, block_off, wave0_off;   // within the plan region
    size_t max_waves, max_blocks;
};

// Upper bound on the padded waves of one packing: bodies need ceil(n_b / 64)
// <= n_b / 64 + 1 waves, greedy packing wastes less than half of each
// workgroup it closes for lack of room, and a workgroup is also closed at the
// end of every scene (<= W - 1 waves).
size_t batch_max_waves(int32_t P, int32_t B, int32_t S)
{
    return 2 * ((size_t)P / 64 + (size_t)B + 1) + (size_t)(S + 1) * pbdr::kMaxWaves;
}

BLayout make_blayout(int32_t P, int32_t BC, int32_t S, size_t K, int cap)
{
    const size_t N = (size_t)P, B = (size_t)BC;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255u) & ~(size_t)255u;
        return o;
    };
    BLayout L;
    L.x = take(12 * N);
    L.v = take(12 * N);
    L.x0 = take(12 * N);
    L.mass = take(4 * N);
    L.body = take(4 * N);
    L.q = take(12 * N);
    L.body_start = take(4 * (B + 1));
    L.body_mass = take(4 * B);
    L.body_mass64 = take(8 * B);
    L.dl0 = take(12 * N);
    L.dl1 = take(12 * N);
    L.vel0 = take(12 * N);
    L.vel1 = take(12 * N);
    L.xt = take(12 * N);
    L.sxt4 = take(16 * N);
    L.key = take(4 * N);
    L.kbuf0 = take(4 * N);
    L.kbuf1 = take(4 * N);
    L.ibuf0 = take(4 * N);
    L.ibuf1 = take(4 * N);
    L.nbr_n = take(4 * N);
    L.nbr = take(4 * N * (size_t)cap);
    L.hist = take(4 * pbdr::kMaxRadixPasses * pbdr::kRadixBins);
    L.tile_off = take(4 * pbdr::kRadixBins * pbdr::radix_tiles_capacity(N));
    L.cells = take(16 * K);
    L.body_rot = take(36 * B);
    L.counters = take(sizeof(pbdr::Counters));
    L.nbr_stats = take(sizeof(pbdr::NbrStats) * ((N + pbdr::kBlock - 1) / pbdr::kBlock));
    L.body_mq = take(12 * B);
    L.pscene = take(4 * N);
    // per-call plan: scene constants, wave table, workgroup table, first wave of each body
    L.max_waves = batch_max_waves(P, BC, S);
    L.max_blocks = L.max_waves / 4 + 1;
    size_t po = 0;
    auto ptake = [&](size_t bytes) {
        const size_t o = po;
        po += (bytes + 255u) & ~(size_t)255u;
        return o;
    };
    L.mscene_off = ptake(sizeof(pbdr::MultiScene) * (size_t)S);
    L.wave_off = ptake(4 * L.max_waves);
    L.block_off = ptake(8 * L.max_blocks);
    L.wave0_off = ptake(4 * B);
    L.plan_bytes = po;
    L.plan = take(po);
    L.total = off;
    return L;
}

struct BSlot {
    bool used = false;
    int32_t p0 = 0, n = 0, b0 = 0, nb = 0, k0 = 0, kbits = 0, max_need = 0;
    float g[3] = {0.0f, 0.0f, 0.0f};
    float mu = 0.0f;
};

}  // namespace

struct pbdr_batch {
    Resolved res;
    BLayout lay;
    pbdr::Scene dev;
    pbdr::StepConsts consts;
    hipStream_t stream = nullptr;
    hipStream_t upload = nullptr;         // scene uploads, so that adding never waits for running frames
    hipEvent_t uploaded = nullptr;        // the last upload; the next launch waits for it
    bool upload_pending = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int32_t S = 0, P = 0, B = 0, BC = 0;
    size_t K = 0;
    RangeAlloc parts, bodies, keys;
    std::vector<BSlot> slots;
    int32_t used_particles = 0, used_bodies = 0, used_scenes = 0;
    std::vector<int32_t> body_need;       // waves of each body id (0: terminator or free)
    // two pinned plan buffers, alternated; each is reused only after its upload ran
    char* h_plan[2] = {nullptr, nullptr};
    hipEvent_t plan_done[2] = {nullptr, nullptr};
    int plan_buf = 0;
};

namespace {

pbdr_status bcheck_slot(const pbdr_batch* b, int32_t slot)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    if (slot < 0 || slot >= b->S || !b->slots[(size_t)slot].used)
        return fail(PBDR_ERR_INVALID_ARG, "slot %d is not a resident scene", slot);
    return PBDR_OK;
}

void release_batch(pbdr_batch* b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->h_plan[k]) (void)hipHostFree(b->h_plan[k]);
        if (b->plan_done[k]) (void)hipEventDestroy(b->plan_done[k]);
    }
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->upload) (void)hipStreamDestroy(b->upload);
}

pbdr_status blatched(pbdr_batch* b, int32_t* max_nbr)
{
    pbdr::Counters c;
    const size_t nslots = ((size_t)b->P + pbdr::kBlock - 1) / pbdr::kBlock;
    std::vector<pbdr::NbrStats> st(nslots);
    HIP_TRY(hipMemcpyAsync(&c, b->ws + b->lay.counters, sizeof(c), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipMemcpyAsync(st.data(), b->ws + b->lay.nbr_stats, nslots * sizeof(pbdr::NbrStats),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    uint32_t mx = 0;
    for (const auto& e : st) mx = std::max(mx, e.max_nbr);
    if (max_nbr) *max_nbr = (int32_t)mx;
    return pbdr::host::latched_status(c.err, mx, b->res.cap);
}

// Plans and enqueues `frames` frames of the scenes flagged in `active`.
pbdr_status enqueue_segment(pbdr_batch* b, const std::vector<char>& active, int32_t frames)
{
    const BLayout& L = b->lay;
    // pack the stepped bodies (in id order, workgroups closed at scene ends)
    int max_need = 0;
    for (int32_t s = 0; s < b->S; ++s)
        if (active[(size_t)s]) max_need = std::max(max_need, b->slots[(size_t)s].max_need);
    if (max_need == 0) return PBDR_OK;
    const int W = std::max(4, max_need);
    const int k = b->plan_buf;
    b->plan_buf ^= 1;
    HIP_TRY(hipEventSynchronize(b->plan_done[k]));      // its previous upload has run
    char* hp = b->h_plan[k];
    auto* ms = (pbdr::MultiScene*)(hp + L.mscene_off);
    auto* waves = (int32_t*)(hp + L.wave_off);
    auto* blocks = (int32_t*)(hp + L.block_off);
    auto* wave0 = (int32_t*)(hp + L.wave0_off);
    size_t nw = 0;
    int32_t b_lo = b->BC, b_hi = 0;       // body ids with a first wave in this plan
    auto close_block = [&]() {           // pad the open workgroup with idle waves
        while (nw % (size_t)W) waves[nw++] = -1;
    };
    for (int32_t s = 0; s < b->S; ++s) {
        const BSlot& sl = b->slots[(size_t)s];
        pbdr::MultiScene& m = ms[s];
        std::memset(&m, 0, sizeof(m));
        if (!sl.used) continue;
        for (int j = 0; j < 3; ++j) m.g[j] = sl.g[j];
        m.mu = sl.mu;
        m.key_base = (uint32_t)sl.k0;
        m.key_mask = (uint32_t)((1u << sl.kbits) - 1u);
        m.active = active[(size_t)s] ? 1u : 0u;
        if (!m.active) continue;
        close_block();                     // a workgroup holds bodies of one scene (consecutive ids)
        b_lo = std::min(b_lo, sl.b0);
        b_hi = std::max(b_hi, sl.b0 + sl.nb);
        for (int32_t bb = sl.b0; bb < sl.b0 + sl.nb; ++bb) {
            const int need = b->body_need[(size_t)bb];
            if (nw + 2 * (size_t)W > L.max_waves) return fail(PBDR_ERR_INVALID_ARG, "internal: packing bound");
            if (nw % (size_t)W + (size_t)need > (size_t)W) close_block();
            wave0[bb] = (int32_t)nw;
            for (int w = 0; w < need; ++w) waves[nw++] = bb;
        }
    }
    close_block();
    const size_t nblk = nw / (size_t)W;
    if (nblk > L.max_blocks) return fail(PBDR_ERR_INVALID_ARG, "internal: block table bound");
    for (size_t blk = 0; blk < nblk; ++blk) {
        int32_t first = -1, last = -1;
        for (int w = 0; w < W; ++w) {
            const int32_t bb = waves[blk * (size_t)W + (size_t)w];
            if (bb < 0) continue;
            if (first < 0) first = bb;
            last = bb;
        }
        blocks[2 * blk] = first < 0 ? 0 : first;
        blocks[2 * blk + 1] = first < 0 ? 0 : last - first + 1;
    }
    // one upload of the plan (waits for scenes added since the last launch)
    if (b->upload_pending) {
        HIP_TRY(hipStreamWaitEvent(b->stream, b->uploaded, 0));
        b->upload_pending = false;
    }
    // only the parts in use: scene constants, the waves and workgroups of
    // this plan, and the first waves of the bodies it packs
    auto up = [&](size_t off, size_t bytes) {
        return hipMemcpyAsync(b->ws + L.plan + off, hp + off, bytes, hipMemcpyHostToDevice, b->stream);
    };
    HIP_TRY(up(L.mscene_off, sizeof(pbdr::MultiScene) * (size_t)b->S));
    HIP_TRY(up(L.wave_off, 4 * nw));
    HIP_TRY(up(L.block_off, 8 * nblk));
    HIP_TRY(up(L.wave0_off + 4 * (size_t)b_lo, 4 * (size_t)(b_hi - b_lo)));
    HIP_TRY(hipEventRecord(b->plan_done[k], b->stream));
    pbdr::Scene d = b->dev;
    const uint32_t khi = (uint32_t)b->keys.high_water((int32_t)b->K);
    d.T = khi > 0 ? khi : 1u;
    // keys of the sort: the scenes' keys (< T) and T for particles not stepped
    int bits = 1;
    while (bits < 32 && (d.T >> bits) != 0u) ++bits;
    d.radix_passes = (bits + pbdr::kRadixBits - 1) / pbdr::kRadixBits;
    d.skey = d.kbuf[(d.radix_passes - 1) & 1];
    d.sorted = d.ibuf[(d.radix_passes - 1) & 1];
    d.waves_per_block = W;
    d.n_iter_blocks = (int32_t)nblk;
    d.n_extent = b->parts.high_water(b->P);
    d.n_sort = d.n_extent;
    d.radix_items = pbdr::radix_items_for((size_t)d.n_sort);
    d.n_radix_tiles = (uint32_t)pbdr::radix_tiles_for((size_t)d.n_sort);
    d.n_active = 0;
    for (int32_t s = 0; s < b->S; ++s)
        if (b->slots[(size_t)s].used && active[(size_t)s]) d.n_active += b->slots[(size_t)s].n;
    d.dense_iterate = 0;      // a scene's result depends on the scene only, not on the mix
    d.wide_bodies = max_need > pbdr::kWideBodyWaves ? 1 : 0;
    const long long total = (long long)frames * b->res.p.substeps;
    if (total > 0x7fffffffll) return fail(PBDR_ERR_INVALID_ARG, "too many substeps in one call");
    hipError_t e = pbdr::enqueue_substeps(d, b->consts, b->res.p.iterations, (int)total, b->stream);
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return PBDR_OK;
}

}  // namespace

extern "C" {

size_t pbdr_batch_bytes(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies)
{
    if (max_scenes < 1 || max_scenes > (1 << 16) || max_particles < 1 || max_bodies < 1 ||
        max_particles > kBatchMaxParticles || max_bodies > max_particles)
        return 0;
    Resolved r;
    if (pbdr::host::resolve(params, max_particles, &r) != PBDR_OK) return 0;
    const size_t K = 4 * (size_t)max_particles + ((size_t)1 << kMinTableBits) * (size_t)max_scenes;
    return make_blayout(max_particles, max_bodies + max_scenes, max_scenes, K * 2, r.cap).total;
}

pbdr_status pbdr_batch_create(const pbdr_params* params, int32_t max_scenes, int32_t max_particles,
                              int32_t max_bodies, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                              pbdr_batch** out)
{
    pbdr::host::clear_error();
    if (!out) return fail(PBDR_ERR_INVALID_ARG, "out must not be NULL");
    *out = nullptr;
    if (max_scenes < 1 || max_scenes > (1 << 16) || max_particles < 1 || max_bodies < 1 ||
        max_particles > kBatchMaxParticles || max_bodies > max_particles)
        return fail(PBDR_ERR_INVALID_ARG, "need 1 <= max_bodies <= max_particles <= %d and 1 <= max_scenes <= 65536",
                    kBatchMaxParticles);
    Resolved r;
    pbdr_status st = pbdr::host::resolve(params, max_particles, &r);
    if (st != PBDR_OK) return st;
    // keys: each scene's table has fewer than 8 keys per particle, or 2^10
    const size_t K = 2 * (4 * (size_t)max_particles + ((size_t)1 << kMinTableBits) * (size_t)max_scenes);
    const BLayout L = make_blayout(max_particles, max_bodies + max_scenes, max_scenes, K, r.cap);
    if (!dev_workspace || ((uintptr_t)dev_workspace & 255u) != 0)
        return fail(PBDR_ERR_WORKSPACE, "workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < L.total) return fail(PBDR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    pbdr_batch* b = new (std::nothrow) pbdr_batch();
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "out of host memory");
    b->res = r;
    b->lay = L;
    b->stream = (hipStream_t)hip_stream;
    b->ws = (char*)dev_workspace;
    b->ws_bytes = ws_bytes;
    b->S = max_scenes;
    b->P = max_particles;
    b->B = max_bodies;
    b->BC = max_bodies + max_scenes;
    b->K = K;
    b->parts.init(max_particles);
    b->bodies.init(b->BC);
    b->keys.init((int32_t)K);
    b->slots.assign((size_t)max_scenes, BSlot());
    b->body_need.assign((size_t)b->BC, 0);
    pbdr::host::fill_step_consts(r, &b->consts);
    char* w = b->ws;
    pbdr::Scene& d = b->dev;
    std::memset(&d, 0, sizeof(d));
    d.n = max_particles;
    d.nb = b->BC;
    d.T = (uint32_t)K;
    d.n_sort = max_particles;
    d.radix_passes = 1;
    d.radix_items = pbdr::radix_items_for((size_t)max_particles);
    d.n_radix_tiles = (uint32_t)pbdr::radix_tiles_for((size_t)max_particles);
    d.x = (float*)(w + L.x);
    d.v = (float*)(w + L.v);
    d.x0 = (float*)(w + L.x0);
    d.mass = (const float*)(w + L.mass);
    d.body = (const int32_t*)(w + L.body);
    d.q = (const float*)(w + L.q);
    d.body_start = (const int32_t*)(w + L.body_start);
    d.body_mass = (const float*)(w + L.body_mass);
    d.body_mass64 = (const double*)(w + L.body_mass64);
    d.wave_body = (const int32_t*)(w + L.plan + L.wave_off);
    d.body_wave0 = (const int32_t*)(w + L.plan + L.wave0_off);
    d.block_body = (const int32_t*)(w + L.plan + L.block_off);
    d.body_mq = (const float*)(w + L.body_mq);
    d.dl[0] = (float*)(w + L.dl0);
    d.dl[1] = (float*)(w + L.dl1);
    d.vel[0] = (float*)(w + L.vel0);
    d.vel[1] = (float*)(w + L.vel1);
    d.xt = (float*)(w + L.xt);
    d.sxt4 = (float4*)(w + L.sxt4);
    d.key = (uint32_t*)(w + L.key);
    d.kbuf[0] = (uint32_t*)(w + L.kbuf0);
    d.kbuf[1] = (uint32_t*)(w + L.kbuf1);
    d.ibuf[0] = (uint32_t*)(w + L.ibuf0);
    d.ibuf[1] = (uint32_t*)(w + L.ibuf1);
    d.skey = d.kbuf[0];
    d.sorted = d.ibuf[0];
    d.nbr_n = (uint32_t*)(w + L.nbr_n);
    d.nbr = (uint32_t*)(w + L.nbr);
    d.hist = (uint32_t*)(w + L.hist);
    d.tile_off = (uint32_t*)(w + L.tile_off);
    d.cells = (uint4*)(w + L.cells);
    d.body_rot = (float*)(w + L.body_rot);
    d.counters = (pbdr::Counters*)(w + L.counters);
    d.nbr_stats = (pbdr::NbrStats*)(w + L.nbr_stats);
    d.accel = nullptr;
    d.pscene = (const int32_t*)(w + L.pscene);
    d.mscene = (const pbdr::MultiScene*)(w + L.plan + L.mscene_off);
    hipError_t e = hipStreamCreateWithFlags(&b->upload, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc((void**)&b->h_plan[k], L.plan_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->plan_done[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b->plan_done[k], b->stream);
    }
    // no particle belongs to a scene yet; tables empty, counters clear
    if (e == hipSuccess) e = hipMemsetAsync(w + L.pscene, 0xff, 4 * (size_t)max_particles, b->stream);
    if (e == hipSuccess) e = pbdr::enqueue_clear_counters(d, b->stream);
    if (e == hipSuccess) e = pbdr::enqueue_init_tables(d, K, b->stream);
    // the sort's buffers hold valid ids and keys from the start
    if (e == hipSuccess) e = hipMemsetAsync(w + L.kbuf0, 0, L.nbr_n - L.kbuf0, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        release_batch(b);
        delete b;
        return fail(PBDR_ERR_DEVICE, "batch set-up failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return PBDR_OK;
}

pbdr_status pbdr_batch_add(pbdr_batch* b, const pbdr_pool_scene_desc* desc, int32_t* slot_out)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    if (!desc || !slot_out) return fail(PBDR_ERR_INVALID_ARG, "desc and slot must not be NULL");
    *slot_out = -1;
    const int32_t n = desc->n_particles, nb = desc->n_bodies;
    if (n < 1 || nb < 1 || nb > n) return fail(PBDR_ERR_INVALID_ARG, "a scene needs n_particles >= n_bodies >= 1");
    if (!desc->x || !desc->v || !desc->mass || !desc->body_start)
        return fail(PBDR_ERR_INVALID_ARG, "desc arrays must not be NULL");
    if (desc->body_start[0] != 0 || desc->body_start[nb] != n)
        return fail(PBDR_ERR_INVALID_ARG, "body_start must begin at 0 and end at n_particles");
    int max_need = 0;
    for (int32_t bb = 0; bb < nb; ++bb) {
        const int32_t len = desc->body_start[bb + 1] - desc->body_start[bb];
        if (len < 1) return fail(PBDR_ERR_INVALID_ARG, "body %d is empty or body_start decreases", bb);
        if (len > 64 * pbdr::kMaxWaves)
            return fail(PBDR_ERR_INVALID_ARG, "body %d has %d particles, more than %d", bb, len, 64 * pbdr::kMaxWaves);
        max_need = std::max(max_need, (len + 63) / 64);
    }
    for (int32_t i = 0; i < n; ++i)
        if (!(std::isfinite(desc->mass[i]) && desc->mass[i] > 0.0f))
            return fail(PBDR_ERR_INVALID_ARG, "mass[%d] must be finite and > 0", i);
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(desc->x[i]) || !std::isfinite(desc->v[i]))
            return fail(PBDR_ERR_INVALID_ARG, "x and v must be finite");
    if (!pbdr::host::finite3(desc->gravity)) return fail(PBDR_ERR_INVALID_ARG, "gravity must be finite");
    if (!(std::isfinite(desc->friction_mu) && desc->friction_mu >= 0.0))
        return fail(PBDR_ERR_INVALID_ARG, "friction_mu must be finite and >= 0");
    int32_t slot = -1;
    for (int32_t s = 0; s < b->S; ++s)
        if (!b->slots[(size_t)s].used) {
            slot = s;
            break;
        }
    if (slot < 0) return fail(PBDR_ERR_CAPACITY, "all %d scene slots are in use", b->S);
    const int kbits = table_bits(n);
    const int32_t p0 = b->parts.alloc(n);
    const int32_t b0 = p0 < 0 ? -1 : b->bodies.alloc(nb + 1);
    const int32_t k0 = b0 < 0 ? -1 : b->keys.alloc(1 << kbits);
    if (k0 < 0) {
        if (b0 >= 0) b->bodies.release(b0, nb + 1);
        if (p0 >= 0) b->parts.release(p0, n);
        return fail(PBDR_ERR_CAPACITY, "no free range for %d particles, %d bodies and %d keys", n, nb + 1, 1 << kbits);
    }
    // rest pose (FP64): body mass, centre, q = x - c (Sec. III-C, shape matching)
    std::vector<int32_t> body((size_t)n), pscene((size_t)n, slot), bstart((size_t)nb + 1);
    std::vector<float> bmass((size_t)nb + 1, 0.0f), q(3 * (size_t)n), bmq(3 * ((size_t)nb + 1), 0.0f);
    std::vector<double> bmass64((size_t)nb + 1, 0.0);
    for (int32_t bb = 0; bb < nb; ++bb) {
        double M = 0.0, cm[3] = {0.0, 0.0, 0.0};
        for (int32_t i = desc->body_start[bb]; i < desc->body_start[bb + 1]; ++i) {
            body[(size_t)i] = b0 + bb;
            M += desc->mass[i];
            for (int k = 0; k < 3; ++k) cm[k] += (double)desc->mass[i] * (double)desc->x[(size_t)k * n + i];
        }
        bmass[(size_t)bb] = (float)M;
        bmass64[(size_t)bb] = M;
        for (int k = 0; k < 3; ++k) cm[k] /= M;
        double mq[3] = {0.0, 0.0, 0.0};
        for (int32_t i = desc->body_start[bb]; i < desc->body_start[bb + 1]; ++i)
            for (int k = 0; k < 3; ++k) {
                const size_t j = (size_t)k * n + i;
                q[j] = (float)((double)desc->x[j] - cm[k]);
                mq[k] += (double)desc->mass[i] * (double)q[j];
            }
        for (int k = 0; k < 3; ++k) bmq[3 * (size_t)bb + k] = (float)mq[k];
    }
    for (int32_t bb = 0; bb <= nb; ++bb) bstart[(size_t)bb] = p0 + desc->body_start[bb];
    const BLayout& L = b->lay;
    const size_t P = (size_t)b->P;
    auto h2d = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpyAsync(b->ws + off, src, bytes, hipMemcpyHostToDevice, b->upload);
    };
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        const size_t dst = (size_t)k * P + (size_t)p0, src = (size_t)k * n;
        e = h2d(L.x + 4 * dst, desc->x + src, 4 * (size_t)n);
        if (e == hipSuccess) e = h2d(L.v + 4 * dst, desc->v + src, 4 * (size_t)n);
        if (e == hipSuccess) e = h2d(L.q + 4 * dst, q.data() + src, 4 * (size_t)n);
    }
    if (e == hipSuccess) e = h2d(L.mass + 4 * (size_t)p0, desc->mass, 4 * (size_t)n);
    if (e == hipSuccess) e = h2d(L.body + 4 * (size_t)p0, body.data(), 4 * (size_t)n);
    if (e == hipSuccess) e = h2d(L.pscene + 4 * (size_t)p0, pscene.data(), 4 * (size_t)n);
    if (e == hipSuccess) e = h2d(L.body_start + 4 * (size_t)b0, bstart.data(), 4 * ((size_t)nb + 1));
    if (e == hipSuccess) e = h2d(L.body_mass + 4 * (size_t)b0, bmass.data(), 4 * ((size_t)nb + 1));
    if (e == hipSuccess) e = h2d(L.body_mass64 + 8 * (size_t)b0, bmass64.data(), 8 * ((size_t)nb + 1));
    if (e == hipSuccess) e = h2d(L.body_mq + 12 * (size_t)b0, bmq.data(), 12 * ((size_t)nb + 1));
    if (e == hipSuccess) e = hipStreamSynchronize(b->upload);      // host arrays are freed on return
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, b->upload);
    if (e != hipSuccess) {
        b->keys.release(k0, 1 << kbits);
        b->bodies.release(b0, nb + 1);
        b->parts.release(p0, n);
        return fail(PBDR_ERR_DEVICE, "scene upload failed: %s", hipGetErrorString(e));
    }
    b->upload_pending = true;
    BSlot& sl = b->slots[(size_t)slot];
    sl.used = true;
    sl.p0 = p0;
    sl.n = n;
    sl.b0 = b0;
    sl.nb = nb;
    sl.k0 = k0;
    sl.kbits = kbits;
    sl.max_need = max_need;
    for (int k = 0; k < 3; ++k) sl.g[k] = (float)desc->gravity[k];
    sl.mu = (float)desc->friction_mu;
    for (int32_t bb = 0; bb < nb; ++bb)
        b->body_need[(size_t)(b0 + bb)] = (desc->body_start[bb + 1] - desc->body_start[bb] + 63) / 64;
    b->body_need[(size_t)(b0 + nb)] = 0;
    b->used_particles += n;
    b->used_bodies += nb;
    b->used_scenes += 1;
    *slot_out = slot;
    return PBDR_OK;
}

pbdr_status pbdr_batch_remove(pbdr_batch* b, int32_t slot)
{
    pbdr_status st = bcheck_slot(b, slot);
    if (st != PBDR_OK) return st;
    BSlot& sl = b->slots[(size_t)slot];
    // its particles belong to no scene from the next launch on; cleared on the
    // upload stream, so that a scene added into the same range later is
    // uploaded after the clear (the next launch waits for both)
    HIP_TRY(hipMemsetAsync(b->ws + b->lay.pscene + 4 * (size_t)sl.p0, 0xff, 4 * (size_t)sl.n, b->upload));
    HIP_TRY(hipEventRecord(b->uploaded, b->upload));
    b->upload_pending = true;
    for (int32_t bb = sl.b0; bb <= sl.b0 + sl.nb; ++bb) b->body_need[(size_t)bb] = 0;
    b->keys.release(sl.k0, 1 << sl.kbits);
    b->bodies.release(sl.b0, sl.nb + 1);
    b->parts.release(sl.p0, sl.n);
    b->used_particles -= sl.n;
    b->used_bodies -= sl.nb;
    b->used_scenes -= 1;
    sl = BSlot();
    return PBDR_OK;
}

pbdr_status pbdr_batch_step_slots(pbdr_batch* b, int32_t count, const int32_t* slots, const int32_t* frames)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    if (count < 0 || (count > 0 && (!slots || !frames)))
        return fail(PBDR_ERR_INVALID_ARG, "slots and frames must hold count entries");
    std::vector<int32_t> want((size_t)b->S, 0);
    for (int32_t j = 0; j < count; ++j) {
        pbdr_status st = bcheck_slot(b, slots[j]);
        if (st != PBDR_OK) return st;
        if (frames[j] < 0) return fail(PBDR_ERR_INVALID_ARG, "frames must be >= 0");
        if (want[(size_t)slots[j]] != 0) return fail(PBDR_ERR_INVALID_ARG, "slot %d is listed twice", slots[j]);
        want[(size_t)slots[j]] = frames[j];
    }
    // segments of equal membership: every listed scene up to the fewest
    // frames still wanted, then those that want more, and so on
    int32_t done = 0;
    while (true) {
        int32_t next = 0;
        for (int32_t s = 0; s < b->S; ++s)
            if (want[(size_t)s] > done && (next == 0 || want[(size_t)s] < next)) next = want[(size_t)s];
        if (next == 0) break;
        std::vector<char> active((size_t)b->S, 0);
        for (int32_t s = 0; s < b->S; ++s) active[(size_t)s] = want[(size_t)s] > done ? 1 : 0;
        pbdr_status st = enqueue_segment(b, active, next - done);
        if (st != PBDR_OK) return st;
        done = next;
    }
    return PBDR_OK;
}

pbdr_status pbdr_batch_step(pbdr_batch* b, int32_t n_frames)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    if (n_frames < 0) return fail(PBDR_ERR_INVALID_ARG, "n_frames must be >= 0");
    if (n_frames == 0) return PBDR_OK;
    std::vector<char> active((size_t)b->S, 0);
    for (int32_t s = 0; s < b->S; ++s) active[(size_t)s] = b->slots[(size_t)s].used ? 1 : 0;
    return enqueue_segment(b, active, n_frames);
}

pbdr_status pbdr_batch_substep(pbdr_batch* b, int32_t n_substeps)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    if (n_substeps < 0) return fail(PBDR_ERR_INVALID_ARG, "n_substeps must be >= 0");
    if (n_substeps == 0) return PBDR_OK;
    // as one frame of n_substeps substeps
    const int32_t keep = b->res.p.substeps;
    b->res.p.substeps = n_substeps;
    std::vector<char> active((size_t)b->S, 0);
    for (int32_t s = 0; s < b->S; ++s) active[(size_t)s] = b->slots[(size_t)s].used ? 1 : 0;
    pbdr_status st = enqueue_segment(b, active, 1);
    b->res.p.substeps = keep;
    return st;
}

pbdr_status pbdr_batch_read_state(pbdr_batch* b, int32_t slot, float* x, float* v, int32_t on_device)
{
    pbdr_status st = bcheck_slot(b, slot);
    if (st != PBDR_OK) return st;
    const BSlot& sl = b->slots[(size_t)slot];
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t P = (size_t)b->P;
    for (int k = 0; k < 3; ++k) {
        const size_t src = 4 * ((size_t)k * P + (size_t)sl.p0), dst = (size_t)k * sl.n;
        if (x) HIP_TRY(hipMemcpyAsync(x + dst, b->ws + b->lay.x + src, 4 * (size_t)sl.n, kind, b->stream));
        if (v) HIP_TRY(hipMemcpyAsync(v + dst, b->ws + b->lay.v + src, 4 * (size_t)sl.n, kind, b->stream));
    }
    return blatched(b, nullptr);
}

pbdr_status pbdr_batch_read_debug(pbdr_batch* b, int32_t slot, int32_t what, void* dst)
{
    pbdr_status st = bcheck_slot(b, slot);
    if (st != PBDR_OK) return st;
    if (!dst) return fail(PBDR_ERR_INVALID_ARG, "dst must not be NULL");
    const BSlot& sl = b->slots[(size_t)slot];
    const size_t P = (size_t)b->P, n = (size_t)sl.n, p0 = (size_t)sl.p0;
    switch (what) {
    case PBDR_DEBUG_XT:
    case PBDR_DEBUG_DELTA: {
        const size_t base = what == PBDR_DEBUG_XT ? b->lay.xt
                                                  : ((b->res.p.iterations % 2 == 0) ? b->lay.dl0 : b->lay.dl1);
        for (int k = 0; k < 3; ++k)
            HIP_TRY(hipMemcpyAsync((float*)dst + (size_t)k * n, b->ws + base + 4 * ((size_t)k * P + p0), 4 * n,
                                   hipMemcpyDeviceToHost, b->stream));
        break;
    }
    case PBDR_DEBUG_NBR_COUNT:
        HIP_TRY(hipMemcpyAsync(dst, b->ws + b->lay.nbr_n + 4 * p0, 4 * n, hipMemcpyDeviceToHost, b->stream));
        break;
    case PBDR_DEBUG_NBR: {
        const size_t cap = (size_t)b->res.cap;
        for (size_t k = 0; k < cap; ++k)
            HIP_TRY(hipMemcpyAsync((uint32_t*)dst + k * n, b->ws + b->lay.nbr + 4 * (k * P + p0), 4 * n,
                                   hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        // scene-local ids (entries past each list's length are left as stored)
        std::vector<uint32_t> cnt(n);
        HIP_TRY(hipMemcpy(cnt.data(), b->ws + b->lay.nbr_n + 4 * p0, 4 * n, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < cap; ++k)
            for (size_t i = 0; i < n; ++i)
                if (k < cnt[i]) ((uint32_t*)dst)[k * n + i] -= (uint32_t)p0;
        return PBDR_OK;
    }
    default: return fail(PBDR_ERR_INVALID_ARG, "unknown or unsupported debug buffer %d", what);
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    return PBDR_OK;
}

pbdr_status pbdr_batch_check(pbdr_batch* b, int32_t* max_neighbours)
{
    if (!b) return fail(PBDR_ERR_INVALID_ARG, "batch is NULL");
    return blatched(b, max_neighbours);
}

pbdr_status pbdr_batch_info_get(const pbdr_batch* b, pbdr_batch_info* out)
{
    if (!b || !out) return fail(PBDR_ERR_INVALID_ARG, "batch and out must not be NULL");
    out->max_scenes = b->S;
    out->scenes_used = b->used_scenes;
    out->max_particles = b->P;
    out->particles_used = b->used_particles;
    out->largest_free_particles = b->parts.largest();
    out->max_bodies = b->B;
    out->bodies_used = b->used_bodies;
    out->max_keys = (int32_t)b->K;
    out->largest_free_keys = b->keys.largest();
    out->workspace_bytes = b->lay.total;
    return PBDR_OK;
}

void pbdr_batch_destroy(pbdr_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    release_batch(b);
    delete b;
}

}  // extern "C"
