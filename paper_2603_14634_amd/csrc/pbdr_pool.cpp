// Host side of scene pools: arena allocation (admission), scene upload with the
// FP64 rest pose, launch plans grouped by size class (one launch per class, the
// classes on parallel streams), the launch-shape tuner, and read-back.  See
// include/pbdr.h for the contract.
#include "pbdr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "pbdr_host.h"
#include "pbdr_pool_device.h"

using pbdr::host::fail;
using pbdr::host::RangeAlloc;
using pbdr::host::Resolved;

namespace {

constexpr int kClasses = pbdr::kPoolClasses;          // tunable (register-resident) classes
constexpr int kLaunchClasses = kClasses + 1;           // ... and the large scenes
constexpr int kBig = pbdr::kPoolBigClass;
constexpr int kLanes = PBDR_POOL_LANES;                // independent launch streams
static_assert(kClasses == PBDR_POOL_CLASSES, "class count");
static_assert(pbdr::kPoolBigMaxParticles == PBDR_POOL_MAX_PARTICLES, "pool scene size");
static_assert(pbdr::kPoolBigMaxBodies == PBDR_POOL_MAX_BODIES, "pool body count");

struct PoolLayout {
    size_t x, v, x0, mass, q, pbody, dl, xt, sxt4, nbr_n, nbr, save_x, save_v, body_first, body_mass, body_mq, scenes,
        stats, save_stats, order, part, sid, rank, vel, cd, total;
};

// Slot-sum arena of the large scenes: every scene needs at most
// n / 64 + 1 + n_bodies slots.
size_t slot_arena(int32_t S, int32_t P, int32_t Bc) { return (size_t)P / 64 + (size_t)Bc + (size_t)S; }

PoolLayout pool_layout(int32_t S, int32_t P, int32_t Bc, int cap)
{
    const size_t s = (size_t)S, p = (size_t)P, b = (size_t)Bc;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255u) & ~(size_t)255u;
        return o;
    };
    PoolLayout L;
    L.x = take(12 * p);
    L.v = take(12 * p);
    L.x0 = take(12 * p);
    L.mass = take(4 * p);
    L.q = take(12 * p);
    L.pbody = take(2 * p);
    L.dl = take(12 * p);
    L.xt = take(12 * p);
    L.sxt4 = take(16 * p);
    L.nbr_n = take(4 * p);
    L.nbr = take(4 * p * (size_t)cap);
    L.save_x = take(12 * p);
    L.save_v = take(12 * p);
    L.body_first = take(4 * b);
    L.body_mass = take(4 * b);
    L.body_mq = take(12 * b);
    L.scenes = take(sizeof(pbdr::PoolScene) * s);
    L.stats = take(sizeof(pbdr::PoolStat) * s);
    L.save_stats = take(sizeof(pbdr::PoolStat) * s);
    L.order = take(8 * s * (kLanes + 1));    // one launch list per lane, and the captured graph's
    L.part = take(4 * 24 * slot_arena(S, P, Bc));
    L.sid = take(4 * p);
    L.rank = take(4 * p);
    L.vel = take(12 * p);
    L.cd = take(12 * p);
    L.total = off;
    return L;
}

// First-fit allocator of index ranges in [0, capacity), coalescing on release.
struct SlotInfo {
    bool used = false;
    int32_t p0 = 0, n = 0, b0 = 0, nb = 0, cls = 0;
    int32_t lanes_slots = 0;        // 64-lane slots of the wave-aligned bodies
    int32_t s_base = -1;            // large scenes: range in the slot-sum arena
    float g[3] = {0.0f, 0.0f, 0.0f};
    float mu = 0.0f;
    pbdr::PoolScene rec = {};     // its device record, uploaded when added
    std::vector<char> staging;    // host copy of the upload, kept until the slot is freed
    hipEvent_t uploaded = nullptr;  // recorded after the upload
};

// Launch class of a scene: register-resident by size, or the large-scene kernel.
int class_of(int32_t n, int32_t nb, int32_t lanes_slots, int max_cls)
{
    if (n > pbdr::pool_class_bound(max_cls) || nb > pbdr::kPoolMaxBodies || lanes_slots > pbdr::kPoolMaxSlots)
        return kBig;
    int c = 0;
    while (c < kClasses - 1 && n > pbdr::pool_class_bound(c)) ++c;
    return c;
}

// Fewest supported register sets per lane covering `slots` 64-lane slots with `waves` waves.
int sets_for(int32_t slots, int waves)
{
    int s = (int)((slots + waves - 1) / waves);
    if (s < 1) s = 1;
    while (s <= 8 && !pbdr::pool_slots_supported(s)) ++s;
    return s;
}

// The set width, widened until at most 8 register sets cover the slots.
int width_for(int32_t slots, int waves)
{
    while (waves < 16 && sets_for(slots, waves) > 8) waves *= 2;
    return waves;
}

bool valid_waves(int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 16; }

}  // namespace

struct pbdr_pool {
    Resolved res;
    pbdr::PoolConsts consts;
    pbdr::PoolDev dev;
    PoolLayout lay;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t aux[kLanes][kLaunchClasses] = {};
    hipEvent_t fork[kLanes] = {};
    hipEvent_t join[kLanes][kLaunchClasses] = {};
    hipEvent_t added = nullptr;          // recorded after the latest upload of an added scene
    int32_t S = 0, P = 0, Bc = 0;
    int max_cls = 0;
    bool big_ok = false;                 // the device holds the large-scene kernel's LDS
    std::vector<SlotInfo> slots;
    std::vector<int32_t> free_slots;
    RangeAlloc parts, bodies, slot_sums;
    int32_t used_particles = 0, used_bodies = 0, used_scenes = 0;
    int waves[kClasses];
    // per lane, double-buffered pinned launch lists of (slot, units)
    int2* h_order[kLanes][2] = {};
    hipEvent_t uploaded[kLanes][2] = {};
    hipEvent_t done[kLanes] = {};        // recorded after each lane's latest launch
    int plan_buf[kLanes] = {};
    // pbdr_pool_step replays a captured graph of lane 0's class launches (its
    // fork and join included) while the resident scenes, the tuning and the
    // frame count stay the same; a change of any of them captures it again
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    uint64_t generation = 1;             // bumped by every change of the resident set or tuning
    uint64_t graph_generation = 0;
    int32_t graph_frames = 0;
};

namespace {

void drop_graph(pbdr_pool* p)
{
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->graph_generation = 0;
}

void release_host(pbdr_pool* p)
{
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    for (SlotInfo& si : p->slots)
        if (si.uploaded) (void)hipEventDestroy(si.uploaded);
    for (int l = 0; l < kLanes; ++l) {
        for (int c = 0; c < kLaunchClasses; ++c) {
            if (p->aux[l][c]) (void)hipStreamDestroy(p->aux[l][c]);
            if (p->join[l][c]) (void)hipEventDestroy(p->join[l][c]);
        }
        if (p->fork[l]) (void)hipEventDestroy(p->fork[l]);
        if (p->done[l]) (void)hipEventDestroy(p->done[l]);
        for (int b = 0; b < 2; ++b) {
            if (p->uploaded[l][b]) (void)hipEventDestroy(p->uploaded[l][b]);
            if (p->h_order[l][b]) (void)hipHostFree(p->h_order[l][b]);
        }
    }
    if (p->added) (void)hipEventDestroy(p->added);
}

pbdr_status check_slot(const pbdr_pool* p, int32_t slot)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (slot < 0 || slot >= p->S || !p->slots[(size_t)slot].used)
        return fail(PBDR_ERR_INVALID_ARG, "slot %d is not a resident scene", slot);
    return PBDR_OK;
}

// Launches, on `stream` and the aux streams of `lane`, every size class with
// work: slot j advances units[j] units (0 = stays).  The launch list is
// uploaded from the lane's pinned buffers, so launches on different lanes may
// be in flight together.
// The launch list: slots with work grouped by class (largest scenes first),
// written to ho; first/count/nmax per class.  Returns the list length.
int build_list(const pbdr_pool* p, const std::vector<int32_t>& units, int only_class, int2* ho,
               int* first, int* count, int32_t* nmax)
{
    std::vector<int32_t> by_class[kLaunchClasses];
    for (int c = 0; c < kLaunchClasses; ++c) nmax[c] = 0;      // largest slot count per class
    for (int32_t j = 0; j < p->S; ++j) {
        const SlotInfo& si = p->slots[(size_t)j];
        if (!si.used || units[(size_t)j] <= 0 || (only_class >= 0 && si.cls != only_class)) continue;
        by_class[si.cls].push_back(j);
        nmax[si.cls] = std::max(nmax[si.cls], si.lanes_slots);
    }
    int at = 0;
    for (int c = 0; c < kLaunchClasses; ++c) {
        auto& v = by_class[c];
        // largest scenes first: they finish last, so they start first
        std::stable_sort(v.begin(), v.end(),
                         [&](int32_t a, int32_t bb) { return p->slots[(size_t)a].n > p->slots[(size_t)bb].n; });
        first[c] = at;
        count[c] = (int)v.size();
        for (int32_t j : v) ho[at++] = make_int2(j, units[(size_t)j]);
    }
    return at;
}

// Enqueues the class launches of a list already on the device (dev_order),
// on `stream`, or side by side on the lane's aux streams (fork and join by
// events, which a stream capture records as graph dependencies).
pbdr_status enqueue_classes(pbdr_pool* p, int lane, hipStream_t stream, const char* dev_order, const int* first,
                            const int* count, const int32_t* nmax, int subs_per_unit)
{
    pbdr::PoolDev d = p->dev;
    d.order = (const int2*)dev_order;
    int active = 0;
    for (int c = 0; c < kLaunchClasses; ++c) active += count[c] > 0;
    // Lane 0 runs several classes side by side on its aux streams; the other
    // lanes run their classes one after another on their own stream (every
    // stream shares a few hardware queues, so fewer streams keep the lanes apart).
    if (lane != 0) active = 1;
    if (active > 1) HIP_TRY(hipEventRecord(p->fork[lane], stream));
    for (int c = 0; c < kLaunchClasses; ++c) {
        if (!count[c]) continue;
        hipStream_t s = stream;
        if (active > 1) {       // classes run side by side on the lane's aux streams
            s = p->aux[lane][c];
            HIP_TRY(hipStreamWaitEvent(s, p->fork[lane], 0));
        }
        const int w = c == kBig ? 16 : width_for(nmax[c], p->waves[c]);
        hipError_t e = pbdr::enqueue_pool_class(d, p->consts, c, w, c == kBig ? 1 : sets_for(nmax[c], w), first[c],
                                                count[c], subs_per_unit, s);
        if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "pool launch failed: %s", hipGetErrorString(e));
        if (active > 1) HIP_TRY(hipEventRecord(p->join[lane][c], s));
    }
    if (active > 1)
        for (int c = 0; c < kLaunchClasses; ++c)
            if (count[c]) HIP_TRY(hipStreamWaitEvent(stream, p->join[lane][c], 0));
    return PBDR_OK;
}

pbdr_status launch(pbdr_pool* p, int lane, hipStream_t stream, const std::vector<int32_t>& units, int subs_per_unit,
                   int only_class = -1, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr)
{
    const int b = p->plan_buf[lane];
    p->plan_buf[lane] ^= 1;
    HIP_TRY(hipEventSynchronize(p->uploaded[lane][b]));       // the buffer's previous upload is done
    int2* ho = p->h_order[lane][b];
    int first[kLaunchClasses], count[kLaunchClasses];
    int32_t nmax[kLaunchClasses];
    const int at = build_list(p, units, only_class, ho, first, count, nmax);
    if (at == 0) return PBDR_OK;
    HIP_TRY(hipStreamWaitEvent(stream, p->added, 0));          // scenes added on the pool's stream are in place
    char* dev_order = p->ws + p->lay.order + 8 * (size_t)p->S * lane;
    HIP_TRY(hipMemcpyAsync(dev_order, ho, 8 * (size_t)at, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(p->uploaded[lane][b], stream));
    if (t0) HIP_TRY(hipEventRecord(t0, stream));
    pbdr_status st = enqueue_classes(p, lane, stream, dev_order, first, count, nmax, subs_per_unit);
    if (st != PBDR_OK) return st;
    if (t1) HIP_TRY(hipEventRecord(t1, stream));
    HIP_TRY(hipEventRecord(p->done[lane], stream));
    return PBDR_OK;
}

// pbdr_pool_step: every resident scene advances n_frames frames, by replaying
// the captured graph of lane 0's class launches (captured again when the
// resident set, the tuning or n_frames changed since).
pbdr_status launch_graph(pbdr_pool* p, int32_t n_frames)
{
    if (!p->gexec || p->graph_generation != p->generation || p->graph_frames != n_frames) {
        drop_graph(p);
        std::vector<int32_t> units((size_t)p->S, n_frames);
        std::vector<int2> ho((size_t)p->S);
        int first[kLaunchClasses], count[kLaunchClasses];
        int32_t nmax[kLaunchClasses];
        const int at = build_list(p, units, -1, ho.data(), first, count, nmax);
        if (at == 0) return PBDR_OK;
        // the graph's own launch list, read by every replay
        char* dev_order = p->ws + p->lay.order + 8 * (size_t)p->S * kLanes;
        HIP_TRY(hipStreamWaitEvent(p->stream, p->added, 0));
        HIP_TRY(hipMemcpyAsync(dev_order, ho.data(), 8 * (size_t)at, hipMemcpyHostToDevice, p->stream));
        HIP_TRY(hipStreamSynchronize(p->stream));
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
        pbdr_status st = enqueue_classes(p, 0, p->cap_stream, dev_order, first, count, nmax, p->res.p.substeps);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
        if (st != PBDR_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != PBDR_OK ? st : fail(PBDR_ERR_DEVICE, "pool graph capture failed: %s", hipGetErrorString(e));
        }
        p->graph = g;
        HIP_TRY(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
        p->graph_generation = p->generation;
        p->graph_frames = n_frames;
    }
    HIP_TRY(hipStreamWaitEvent(p->stream, p->added, 0));
    HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
    HIP_TRY(hipEventRecord(p->done[0], p->stream));
    return PBDR_OK;
}

pbdr_status scene_status(pbdr_pool* p, int32_t slot, uint32_t* max_nbr)
{
    pbdr::PoolStat st;
    HIP_TRY(hipMemcpyAsync(&st, p->ws + p->lay.stats + sizeof(pbdr::PoolStat) * (size_t)slot, sizeof(st),
                           hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
    if (max_nbr) *max_nbr = st.max_nbr;
    // after any of these the slot keeps the state of its last clean frame and is no longer stepped
    if (st.err & pbdr::kErrCapacity)
        return fail(PBDR_ERR_CAPACITY, "a neighbour list of slot %d reached %u entries, above nbr_cap %d", slot, st.max_nbr,
                    p->res.cap);
    if (st.err & pbdr::kErrNonFinite) return fail(PBDR_ERR_NONFINITE, "a position or velocity of slot %d became non-finite", slot);
    if (st.err & pbdr::kErrInternal) return fail(PBDR_ERR_DEVICE, "slot %d did not fit its launch shape", slot);
    return PBDR_OK;
}

pbdr_status copy_components(pbdr_pool* p, size_t arena_off, const SlotInfo& si, float* dst, hipMemcpyKind kind)
{
    for (int k = 0; k < 3; ++k)
        HIP_TRY(hipMemcpyAsync(dst + (size_t)k * si.n,
                               p->ws + arena_off + 4 * ((size_t)k * p->P + (size_t)si.p0), 4 * (size_t)si.n, kind,
                               p->stream));
    return PBDR_OK;
}

}  // namespace

extern "C" {

size_t pbdr_pool_bytes(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies)
{
    Resolved r;
    if (pbdr::host::resolve(params, max_particles, &r) != PBDR_OK) return 0;
    if (max_scenes < 1 || max_particles < 1 || max_bodies < 1) {
        fail(PBDR_ERR_INVALID_ARG, "pool capacities must be >= 1");
        return 0;
    }
    return pool_layout(max_scenes, max_particles, max_bodies, r.cap).total;
}

pbdr_status pbdr_pool_create(const pbdr_params* params, int32_t max_scenes, int32_t max_particles, int32_t max_bodies,
                             void* dev_workspace, size_t ws_bytes, void* hip_stream, pbdr_pool** out)
{
    pbdr::host::clear_error();
    if (!out) return fail(PBDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Resolved r;
    pbdr_status st = pbdr::host::resolve(params, max_particles, &r);
    if (st != PBDR_OK) return st;
    if (max_scenes < 1 || max_particles < 1 || max_bodies < 1)
        return fail(PBDR_ERR_INVALID_ARG, "pool capacities must be >= 1");
    const PoolLayout lay = pool_layout(max_scenes, max_particles, max_bodies, r.cap);
    if (!dev_workspace) return fail(PBDR_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)dev_workspace & 255u) != 0) return fail(PBDR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < lay.total) return fail(PBDR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);

    int dev = 0, lds_max = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    int max_cls = -1;
    for (int c = 0; c < kClasses; ++c)
        if (pbdr::pool_lds_bytes(c) <= (size_t)lds_max) max_cls = c;
    if (max_cls < 0) return fail(PBDR_ERR_DEVICE, "the device offers %d bytes of LDS per workgroup, too few for pools", lds_max);
    const bool big_ok = pbdr::pool_lds_bytes(kBig) <= (size_t)lds_max;
    {
        const size_t need = std::max(pbdr::pool_lds_bytes(max_cls), big_ok ? pbdr::pool_lds_bytes(kBig) : (size_t)0);
        hipError_t e = pbdr::pool_prepare(need);
        if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "pool kernel set-up failed: %s", hipGetErrorString(e));
    }

    pbdr_pool* p = new (std::nothrow) pbdr_pool();
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "out of host memory");
    p->res = r;
    p->lay = lay;
    p->ws = (char*)dev_workspace;
    p->ws_bytes = ws_bytes;
    p->stream = (hipStream_t)hip_stream;
    p->S = max_scenes;
    p->P = max_particles;
    p->Bc = max_bodies;
    p->max_cls = max_cls;
    p->big_ok = big_ok;
    p->slots.resize((size_t)max_scenes);
    for (int32_t j = max_scenes - 1; j >= 0; --j) p->free_slots.push_back(j);
    p->parts.init(max_particles);
    p->bodies.init(max_bodies);
    p->slot_sums.init((int32_t)slot_arena(max_scenes, max_particles, max_bodies));
    for (int c = 0; c < kClasses; ++c) p->waves[c] = std::min(16, std::max(1, pbdr::pool_class_bound(c) / 64));   // one set

    pbdr::PoolConsts& c = p->consts;
    std::memset(&c, 0, sizeof(c));
    c.h = (float)r.h;
    c.inv_h = (float)(1.0 / r.h);
    c.radius = (float)r.p.radius;
    c.two_r = (float)(2.0 * r.p.radius);
    c.search_r2 = (float)(r.rs * r.rs);
    c.search_r = (float)r.rs;
    c.box_margin = (float)(2.0 * r.rs);
    c.inv_cell = (float)(1.0 / r.a);
    for (int k = 0; k < 3; ++k) c.origin[k] = (float)r.p.grid_origin[k];
    c.nbr_cap = r.cap;
    c.flags = r.p.flags & ~PBDR_FLAG_NO_GRAPH;
    c.n_planes = r.p.n_planes;
    for (int j = 0; j < r.p.n_planes; ++j) {
        for (int k = 0; k < 3; ++k) c.plane_n[j][k] = (float)r.p.planes[j][k];
        c.plane_d[j] = (float)r.p.planes[j][3];
        c.plane_d_d[j] = r.p.planes[j][3];
    }
    c.radius_d = r.p.radius;
    c.two_r_d = 2.0 * r.p.radius;
    c.iterations = r.p.iterations;

    char* w = p->ws;
    pbdr::PoolDev& d = p->dev;
    d.P = max_particles;
    d.x = (float*)(w + lay.x);
    d.v = (float*)(w + lay.v);
    d.x0 = (float*)(w + lay.x0);
    d.mass = (const float*)(w + lay.mass);
    d.q = (const float*)(w + lay.q);
    d.pbody = (const uint16_t*)(w + lay.pbody);
    d.dl = (float*)(w + lay.dl);
    d.xt = (float*)(w + lay.xt);
    d.sxt4 = (float4*)(w + lay.sxt4);
    d.nbr_n = (uint32_t*)(w + lay.nbr_n);
    d.nbr = (uint32_t*)(w + lay.nbr);
    d.body_first = (const int32_t*)(w + lay.body_first);
    d.body_mass = (const float*)(w + lay.body_mass);
    d.body_mq = (const float*)(w + lay.body_mq);
    d.scenes = (const pbdr::PoolScene*)(w + lay.scenes);
    d.stats = (pbdr::PoolStat*)(w + lay.stats);
    d.order = (const int2*)(w + lay.order);
    d.part = (float*)(w + lay.part);
    d.sid = (uint32_t*)(w + lay.sid);
    d.rank = (uint32_t*)(w + lay.rank);
    d.vel = (float*)(w + lay.vel);
    d.cd = (float*)(w + lay.cd);

    hipError_t e = hipSuccess;
    for (int l = 0; l < kLanes && e == hipSuccess; ++l) {
        for (int k = 0; k < kLaunchClasses && e == hipSuccess && l == 0; ++k) {
            e = hipStreamCreateWithFlags(&p->aux[l][k], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[l][k], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork[l], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done[l], hipEventDisableTiming);
        for (int b = 0; b < 2 && e == hipSuccess; ++b) {
            e = hipEventCreateWithFlags(&p->uploaded[l][b], hipEventDisableTiming);
            if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_order[l][b], 8 * (size_t)max_scenes, 0);
        }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->added, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemsetAsync(p->ws + lay.scenes, 0, sizeof(pbdr::PoolScene) * (size_t)max_scenes, p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->ws + lay.stats, 0, sizeof(pbdr::PoolStat) * (size_t)max_scenes, p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->added, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        release_host(p);
        delete p;
        return fail(PBDR_ERR_DEVICE, "pool set-up failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return PBDR_OK;
}

pbdr_status pbdr_pool_add(pbdr_pool* p, const pbdr_pool_scene_desc* desc, int32_t* slot_out)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (!desc || !slot_out) return fail(PBDR_ERR_INVALID_ARG, "desc and slot must not be NULL");
    *slot_out = -1;
    const int32_t n = desc->n_particles, nb = desc->n_bodies;
    const int32_t nmax = p->big_ok ? pbdr::kPoolBigMaxParticles : pbdr::pool_class_bound(p->max_cls);
    const int32_t bmax = p->big_ok ? pbdr::kPoolBigMaxBodies : pbdr::kPoolMaxBodies;
    if (n < 1 || n > nmax) return fail(PBDR_ERR_INVALID_ARG, "a pooled scene needs 1..%d particles, got %d", nmax, n);
    if (nb < 1 || nb > bmax || nb > n)
        return fail(PBDR_ERR_INVALID_ARG, "a pooled scene needs 1..%d bodies, got %d", bmax, nb);
    if (!desc->x || !desc->v || !desc->mass || !desc->body_start)
        return fail(PBDR_ERR_INVALID_ARG, "desc arrays must not be NULL");
    if (desc->body_start[0] != 0 || desc->body_start[nb] != n)
        return fail(PBDR_ERR_INVALID_ARG, "body_start must begin at 0 and end at n_particles");
    int32_t lanes_slots = 0;
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t len = desc->body_start[b + 1] - desc->body_start[b];
        if (len < 1) return fail(PBDR_ERR_INVALID_ARG, "body %d is empty or body_start decreases", b);
        lanes_slots += (len + 63) / 64;
    }
    const int cls = class_of(n, nb, lanes_slots, p->max_cls);
    if (cls == kBig && !p->big_ok)
        return fail(PBDR_ERR_INVALID_ARG, "a pooled scene's bodies may fill at most %d slots of 64 lanes (one body per "
                    "slot) on this device, this one needs %d", pbdr::kPoolMaxSlots, lanes_slots);
    for (int32_t i = 0; i < n; ++i)
        if (!(std::isfinite(desc->mass[i]) && desc->mass[i] > 0.0f))
            return fail(PBDR_ERR_INVALID_ARG, "mass[%d] must be finite and > 0", i);
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
        if (!std::isfinite(desc->x[i]) || !std::isfinite(desc->v[i]))
            return fail(PBDR_ERR_INVALID_ARG, "x and v must be finite");
    if (!pbdr::host::finite3(desc->gravity)) return fail(PBDR_ERR_INVALID_ARG, "gravity must be finite");
    if (!(std::isfinite(desc->friction_mu) && desc->friction_mu >= 0.0))
        return fail(PBDR_ERR_INVALID_ARG, "friction_mu must be finite and >= 0");
    if (p->free_slots.empty()) return fail(PBDR_ERR_CAPACITY, "all %d slots are in use", p->S);
    const int32_t p0 = p->parts.alloc(n);
    if (p0 < 0) return fail(PBDR_ERR_CAPACITY, "no free range of %d particles", n);
    const int32_t b0 = p->bodies.alloc(nb);
    if (b0 < 0) {
        p->parts.release(p0, n);
        return fail(PBDR_ERR_CAPACITY, "no free range of %d bodies", nb);
    }
    const int32_t sb = cls == kBig ? p->slot_sums.alloc(lanes_slots) : -1;
    if (cls == kBig && sb < 0) {          // cannot happen: the arena covers every admissible set of scenes
        p->parts.release(p0, n);
        p->bodies.release(b0, nb);
        return fail(PBDR_ERR_CAPACITY, "no free range of %d slot sums", lanes_slots);
    }
    const int32_t slot = p->free_slots.back();
    p->free_slots.pop_back();
    SlotInfo& si = p->slots[(size_t)slot];
    si.used = true;
    p->generation += 1;
    si.p0 = p0;
    si.n = n;
    si.b0 = b0;
    si.nb = nb;
    si.cls = cls;
    si.lanes_slots = lanes_slots;
    si.s_base = sb;
    for (int k = 0; k < 3; ++k) si.g[k] = (float)desc->gravity[k];
    si.mu = (float)desc->friction_mu;

    // rest pose in FP64: body mass, centre, q = x - c (Sec. III-C, shape matching)
    const size_t N = (size_t)n, B = (size_t)nb;
    const size_t o_x = 0, o_v = o_x + 12 * N, o_m = o_v + 12 * N, o_q = o_m + 4 * N, o_pb = o_q + 12 * N,
                 o_bf = o_pb + ((2 * N + 3) & ~(size_t)3), o_bm = o_bf + 4 * B, o_mq = o_bm + 4 * B,
                 o_end = o_mq + 12 * B;
    si.staging.assign(o_end, 0);
    float* xs = (float*)(si.staging.data() + o_x);
    float* vs = (float*)(si.staging.data() + o_v);
    float* ms = (float*)(si.staging.data() + o_m);
    std::memcpy(xs, desc->x, 12 * N);
    std::memcpy(vs, desc->v, 12 * N);
    std::memcpy(ms, desc->mass, 4 * N);
    float* q = (float*)(si.staging.data() + o_q);
    uint16_t* pb = (uint16_t*)(si.staging.data() + o_pb);
    int32_t* bf = (int32_t*)(si.staging.data() + o_bf);
    float* bm = (float*)(si.staging.data() + o_bm);
    float* mq = (float*)(si.staging.data() + o_mq);
    for (int32_t b = 0; b < nb; ++b) {
        double M = 0.0, cm[3] = {0.0, 0.0, 0.0};
        bf[b] = desc->body_start[b];
        for (int32_t i = desc->body_start[b]; i < desc->body_start[b + 1]; ++i) {
            pb[i] = (uint16_t)b;
            const double m = desc->mass[i];
            M += m;
            for (int k = 0; k < 3; ++k) cm[k] += m * (double)desc->x[(size_t)k * N + i];
        }
        bm[b] = (float)M;
        for (int k = 0; k < 3; ++k) cm[k] /= M;
        double s[3] = {0.0, 0.0, 0.0};
        for (int32_t i = desc->body_start[b]; i < desc->body_start[b + 1]; ++i)
            for (int k = 0; k < 3; ++k) {
                const size_t j = (size_t)k * N + i;
                q[j] = (float)((double)desc->x[j] - cm[k]);
                s[k] += (double)desc->mass[i] * (double)q[j];
            }
        for (int k = 0; k < 3; ++k) mq[3 * b + k] = (float)s[k];
    }
    auto h2d = [&](size_t off, const void* src, size_t bytes) {
        return hipMemcpyAsync(p->ws + off, src, bytes, hipMemcpyHostToDevice, p->stream);
    };
    const size_t P = (size_t)p->P;
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        e = h2d(p->lay.x + 4 * ((size_t)k * P + p0), xs + (size_t)k * N, 4 * N);
        if (e == hipSuccess) e = h2d(p->lay.v + 4 * ((size_t)k * P + p0), vs + (size_t)k * N, 4 * N);
        if (e == hipSuccess) e = h2d(p->lay.q + 4 * ((size_t)k * P + p0), q + (size_t)k * N, 4 * N);
    }
    if (e == hipSuccess) e = h2d(p->lay.mass + 4 * (size_t)p0, ms, 4 * N);
    if (e == hipSuccess) e = h2d(p->lay.pbody + 2 * (size_t)p0, pb, 2 * N);
    if (e == hipSuccess) e = h2d(p->lay.body_first + 4 * (size_t)b0, bf, 4 * B);
    if (e == hipSuccess) e = h2d(p->lay.body_mass + 4 * (size_t)b0, bm, 4 * B);
    if (e == hipSuccess) e = h2d(p->lay.body_mq + 12 * (size_t)b0, mq, 12 * B);
    if (e == hipSuccess)
        e = hipMemsetAsync(p->ws + p->lay.stats + sizeof(pbdr::PoolStat) * (size_t)slot, 0, sizeof(pbdr::PoolStat),
                           p->stream);
    si.rec = pbdr::PoolScene{};
    si.rec.p0 = p0;
    si.rec.n = n;
    si.rec.b0 = b0;
    si.rec.nb = nb;
    si.rec.s_base = sb;
    for (int k = 0; k < 3; ++k) si.rec.g[k] = si.g[k];
    si.rec.mu = si.mu;
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->ws + p->lay.scenes + sizeof(pbdr::PoolScene) * (size_t)slot, &si.rec,
                           sizeof(pbdr::PoolScene), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess && !si.uploaded) e = hipEventCreateWithFlags(&si.uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(si.uploaded, p->stream);
    if (e == hipSuccess) e = hipEventRecord(p->added, p->stream);
    p->used_particles += n;
    p->used_bodies += nb;
    p->used_scenes += 1;
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(p->stream);
        pbdr_pool_remove(p, slot);
        return fail(PBDR_ERR_DEVICE, "scene upload failed: %s", hipGetErrorString(e));
    }
    *slot_out = slot;
    return PBDR_OK;
}

pbdr_status pbdr_pool_remove(pbdr_pool* p, int32_t slot)
{
    pbdr_status st = check_slot(p, slot);
    if (st != PBDR_OK) return st;
    SlotInfo& si = p->slots[(size_t)slot];
    p->parts.release(si.p0, si.n);
    p->bodies.release(si.b0, si.nb);
    if (si.s_base >= 0) p->slot_sums.release(si.s_base, si.lanes_slots);
    si.s_base = -1;
    p->used_particles -= si.n;
    p->used_bodies -= si.nb;
    p->used_scenes -= 1;
    si.used = false;
    p->generation += 1;
    if (si.uploaded) HIP_TRY(hipEventSynchronize(si.uploaded));   // the upload has read the staging copy
    si.staging.clear();
    si.staging.shrink_to_fit();
    p->free_slots.push_back(slot);
    return PBDR_OK;
}

pbdr_status pbdr_pool_step(pbdr_pool* p, int32_t n_frames)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (n_frames < 0) return fail(PBDR_ERR_INVALID_ARG, "n_frames must be >= 0");
    if ((long long)n_frames * p->res.p.substeps > INT_MAX) return fail(PBDR_ERR_INVALID_ARG, "too many substeps in one call");
    if (n_frames == 0) return PBDR_OK;
    if (p->res.p.flags & PBDR_FLAG_NO_GRAPH) {
        std::vector<int32_t> units((size_t)p->S, n_frames);
        return launch(p, 0, p->stream, units, p->res.p.substeps);
    }
    return launch_graph(p, n_frames);
}

pbdr_status pbdr_pool_step_slots(pbdr_pool* p, int32_t count, const int32_t* slots, const int32_t* frames)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (count < 0 || (count > 0 && (!slots || !frames))) return fail(PBDR_ERR_INVALID_ARG, "bad slot list");
    std::vector<int32_t> units((size_t)p->S, 0);
    for (int32_t j = 0; j < count; ++j) {
        pbdr_status st = check_slot(p, slots[j]);
        if (st != PBDR_OK) return st;
        if (frames[j] < 0 || (long long)frames[j] * p->res.p.substeps > INT_MAX)
            return fail(PBDR_ERR_INVALID_ARG, "frames[%d] out of range", j);
        units[(size_t)slots[j]] = frames[j];
    }
    return launch(p, 0, p->stream, units, p->res.p.substeps);
}

pbdr_status pbdr_pool_step_slots_on(pbdr_pool* p, int32_t lane, void* hip_stream, int32_t count, const int32_t* slots,
                                    const int32_t* frames)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (lane < 0 || lane >= kLanes) return fail(PBDR_ERR_INVALID_ARG, "lane must be in [0, %d)", kLanes);
    if (count < 0 || (count > 0 && (!slots || !frames))) return fail(PBDR_ERR_INVALID_ARG, "bad slot list");
    std::vector<int32_t> units((size_t)p->S, 0);
    for (int32_t j = 0; j < count; ++j) {
        pbdr_status st = check_slot(p, slots[j]);
        if (st != PBDR_OK) return st;
        if (frames[j] < 0 || (long long)frames[j] * p->res.p.substeps > INT_MAX)
            return fail(PBDR_ERR_INVALID_ARG, "frames[%d] out of range", j);
        units[(size_t)slots[j]] = frames[j];
    }
    return launch(p, lane, (hipStream_t)hip_stream, units, p->res.p.substeps);
}

pbdr_status pbdr_pool_slot_class(const pbdr_pool* p, int32_t slot, int32_t* cls)
{
    pbdr_status st = check_slot(p, slot);
    if (st != PBDR_OK) return st;
    if (!cls) return fail(PBDR_ERR_INVALID_ARG, "cls is NULL");
    *cls = p->slots[(size_t)slot].cls;
    return PBDR_OK;
}

pbdr_status pbdr_pool_class_for(const pbdr_pool* p, int32_t n_particles, int32_t n_bodies, const int32_t* body_start,
                                int32_t* cls)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (!body_start || !cls) return fail(PBDR_ERR_INVALID_ARG, "body_start and cls must not be NULL");
    *cls = -1;
    if (n_particles < 1 || n_bodies < 1 || n_bodies > n_particles)
        return fail(PBDR_ERR_INVALID_ARG, "a scene needs n_particles >= n_bodies >= 1, got %d and %d", n_particles,
                    n_bodies);
    if (body_start[0] != 0 || body_start[n_bodies] != n_particles)
        return fail(PBDR_ERR_INVALID_ARG, "body_start must begin at 0 and end at n_particles");
    int64_t lanes_slots = 0;
    for (int32_t b = 0; b < n_bodies; ++b) {
        const int32_t len = body_start[b + 1] - body_start[b];
        if (len < 1) return fail(PBDR_ERR_INVALID_ARG, "body %d is empty or body_start decreases", b);
        lanes_slots += (len + 63) / 64;
    }
    const int c = class_of(n_particles, n_bodies, (int32_t)std::min<int64_t>(lanes_slots, INT32_MAX), p->max_cls);
    const int32_t nmax = p->big_ok ? pbdr::kPoolBigMaxParticles : pbdr::pool_class_bound(p->max_cls);
    const int32_t bmax = p->big_ok ? pbdr::kPoolBigMaxBodies : pbdr::kPoolMaxBodies;
    if ((c == kBig && !p->big_ok) || n_particles > nmax || n_bodies > bmax)
        return fail(PBDR_ERR_INVALID_ARG, "a scene of %d particles and %d bodies does not fit this pool", n_particles,
                    n_bodies);
    *cls = c;
    return PBDR_OK;
}

pbdr_status pbdr_pool_substep(pbdr_pool* p, int32_t n_substeps)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (n_substeps < 0) return fail(PBDR_ERR_INVALID_ARG, "n_substeps must be >= 0");
    if (n_substeps == 0) return PBDR_OK;
    std::vector<int32_t> units((size_t)p->S, n_substeps);
    return launch(p, 0, p->stream, units, 1);
}

pbdr_status pbdr_pool_read_state(pbdr_pool* p, int32_t slot, float* x, float* v, int32_t on_device)
{
    pbdr_status st = check_slot(p, slot);
    if (st != PBDR_OK) return st;
    const SlotInfo& si = p->slots[(size_t)slot];
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (x && (st = copy_components(p, p->lay.x, si, x, kind)) != PBDR_OK) return st;
    if (v && (st = copy_components(p, p->lay.v, si, v, kind)) != PBDR_OK) return st;
    return scene_status(p, slot, nullptr);
}

pbdr_status pbdr_pool_read_debug(pbdr_pool* p, int32_t slot, int32_t what, void* dst)
{
    pbdr_status st = check_slot(p, slot);
    if (st != PBDR_OK) return st;
    if (!dst) return fail(PBDR_ERR_INVALID_ARG, "dst is NULL");
    const SlotInfo& si = p->slots[(size_t)slot];
    const size_t N = (size_t)si.n;
    switch (what) {
    case PBDR_DEBUG_XT: st = copy_components(p, p->lay.xt, si, (float*)dst, hipMemcpyDeviceToHost); break;
    case PBDR_DEBUG_DELTA: st = copy_components(p, p->lay.dl, si, (float*)dst, hipMemcpyDeviceToHost); break;
    case PBDR_DEBUG_NBR_COUNT:
        HIP_TRY(hipMemcpyAsync(dst, p->ws + p->lay.nbr_n + 4 * (size_t)si.p0, 4 * N, hipMemcpyDeviceToHost, p->stream));
        break;
    case PBDR_DEBUG_NBR:
        HIP_TRY(hipMemcpyAsync(dst, p->ws + p->lay.nbr + 4 * (size_t)p->res.cap * si.p0, 4 * (size_t)p->res.cap * N,
                               hipMemcpyDeviceToHost, p->stream));
        break;
    default: return fail(PBDR_ERR_INVALID_ARG, "debug buffer %d is not kept by pools", what);
    }
    if (st != PBDR_OK) return st;
    HIP_TRY(hipStreamSynchronize(p->stream));
    return PBDR_OK;
}

pbdr_status pbdr_pool_check(pbdr_pool* p, int32_t slot, int32_t* max_neighbours)
{
    pbdr_status st = check_slot(p, slot);
    if (st != PBDR_OK) return st;
    uint32_t mx = 0;
    st = scene_status(p, slot, &mx);
    if (max_neighbours) *max_neighbours = (int32_t)mx;
    return st;
}

pbdr_status pbdr_pool_get_tuning(const pbdr_pool* p, int32_t* waves)
{
    if (!p || !waves) return fail(PBDR_ERR_INVALID_ARG, "pool and waves must not be NULL");
    for (int c = 0; c < kClasses; ++c) waves[c] = p->waves[c];
    return PBDR_OK;
}

pbdr_status pbdr_pool_set_tuning(pbdr_pool* p, const int32_t* waves)
{
    if (!p || !waves) return fail(PBDR_ERR_INVALID_ARG, "pool and waves must not be NULL");
    for (int c = 0; c < kClasses; ++c)
        if (!valid_waves(waves[c])) return fail(PBDR_ERR_INVALID_ARG, "waves[%d] = %d is not 1, 2, 4, 8 or 16", c, waves[c]);
    for (int c = 0; c < kClasses; ++c) p->waves[c] = waves[c];
    p->generation += 1;
    return PBDR_OK;
}

pbdr_status pbdr_pool_autotune(pbdr_pool* p, int32_t n_frames, int32_t repeats, double* ms_out)
{
    if (!p) return fail(PBDR_ERR_INVALID_ARG, "pool is NULL");
    if (n_frames < 1 || repeats < 1) return fail(PBDR_ERR_INVALID_ARG, "n_frames and repeats must be >= 1");
    if ((long long)n_frames * p->res.p.substeps > INT_MAX) return fail(PBDR_ERR_INVALID_ARG, "too many substeps");
    const size_t P = (size_t)p->P;
    const size_t stats_bytes = sizeof(pbdr::PoolStat) * (size_t)p->S;
    HIP_TRY(hipMemcpyAsync(p->ws + p->lay.save_x, p->ws + p->lay.x, 12 * P, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->ws + p->lay.save_v, p->ws + p->lay.v, 12 * P, hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(hipMemcpyAsync(p->ws + p->lay.save_stats, p->ws + p->lay.stats, stats_bytes, hipMemcpyDeviceToDevice, p->stream));
    auto restore = [&]() -> pbdr_status {
        HIP_TRY(hipMemcpyAsync(p->ws + p->lay.x, p->ws + p->lay.save_x, 12 * P, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->ws + p->lay.v, p->ws + p->lay.save_v, 12 * P, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(p->ws + p->lay.stats, p->ws + p->lay.save_stats, stats_bytes, hipMemcpyDeviceToDevice,
                               p->stream));
        return PBDR_OK;
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    std::vector<int32_t> units((size_t)p->S, n_frames);
    pbdr_status st = PBDR_OK;
    for (int c = 0; c < kClasses && st == PBDR_OK; ++c) {
        int32_t nmax = 0;
        for (const SlotInfo& si : p->slots)
            if (si.used && si.cls == c) nmax = std::max(nmax, si.lanes_slots);
        if (ms_out) ms_out[c] = 0.0;
        if (nmax == 0) continue;
        double best = 1e300;
        int best_w = p->waves[c];
        for (int w = 1; w <= 16 && st == PBDR_OK; w *= 2) {
            if (sets_for(nmax, w) > 8) continue;
            const int saved = p->waves[c];
            p->waves[c] = w;
            double t_best = 1e300;
            for (int r = 0; r < repeats && st == PBDR_OK; ++r) {
                if ((st = restore()) != PBDR_OK) break;
                if ((st = launch(p, 0, p->stream, units, p->res.p.substeps, c, t0, t1)) != PBDR_OK) break;
                hipError_t e = hipEventSynchronize(t1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
                if (e != hipSuccess) st = fail(PBDR_ERR_DEVICE, "tuner timing failed: %s", hipGetErrorString(e));
                t_best = std::min(t_best, (double)ms);
            }
            p->waves[c] = saved;
            if (t_best < best) {
                best = t_best;
                best_w = w;
            }
        }
        p->waves[c] = best_w;
        if (ms_out) ms_out[c] = best;
    }
    p->generation += 1;
    pbdr_status st2 = restore();
    hipError_t e = hipStreamSynchronize(p->stream);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != PBDR_OK) return st;
    if (st2 != PBDR_OK) return st2;
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "tuner: %s", hipGetErrorString(e));
    return PBDR_OK;
}

pbdr_status pbdr_pool_info_get(const pbdr_pool* p, pbdr_pool_info* out)
{
    if (!p || !out) return fail(PBDR_ERR_INVALID_ARG, "pool and out must not be NULL");
    out->max_scenes = p->S;
    out->scenes_used = p->used_scenes;
    out->max_particles = p->P;
    out->particles_used = p->used_particles;
    out->largest_free_particles = p->parts.largest();
    out->max_bodies = p->Bc;
    out->bodies_used = p->used_bodies;
    out->largest_free_bodies = p->bodies.largest();
    out->max_scene_particles = p->big_ok ? pbdr::kPoolBigMaxParticles : pbdr::pool_class_bound(p->max_cls);
    out->workspace_bytes = p->lay.total;
    return PBDR_OK;
}

void pbdr_pool_destroy(pbdr_pool* p)
{
    if (!p) return;
    // every lane's work ends before the caller may free the workspace
    for (int l = 0; l < kLanes; ++l)
        if (p->done[l]) (void)hipEventSynchronize(p->done[l]);
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    release_host(p);
    delete p;
}

}  // extern "C"
