// Host side of libpbdr: argument validation, workspace layout, scene
// creation, stepping (direct launches or a captured per-frame HIP graph),
// and result / debug read-back.  See include/pbdr.h for the contract.
#include "pbdr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "pbdr_device.h"
#include "pbdr_host.h"
#include "pbdr_state.h"

namespace pbdr {
namespace host {

thread_local char g_err[512] = "";

pbdr_status fail(pbdr_status st, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

void clear_error() { g_err[0] = 0; }

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

static_assert(pbdr::kErrCapacity == PBDR_COND_CAPACITY && pbdr::kErrNonFinite == PBDR_COND_NONFINITE &&
                  pbdr::kErrInternal == PBDR_COND_INTERNAL && pbdr::kErrWait == PBDR_COND_PARTNER_WAIT,
              "latched condition bits");

pbdr_status latched_status(uint32_t err, uint32_t max_nbr, int cap)
{
    // a list over capacity first: it can make one-launch waits give up as well
    if ((err & pbdr::kErrCapacity) && cap > 0)
        return fail(PBDR_ERR_CAPACITY,
                    "a neighbour list reached %u entries, above nbr_cap %d; the state is that of the last frame "
                    "completed before it",
                    max_nbr, cap);
    if (err & pbdr::kErrCapacity)
        return fail(PBDR_ERR_CAPACITY,
                    "a neighbour list exceeded nbr_cap; the state is that of the last frame completed before it");
    if (err & pbdr::kErrNonFinite)
        return fail(PBDR_ERR_NONFINITE,
                    "a position or velocity became non-finite; the state is that of the last frame completed before it");
    if (err & pbdr::kErrWait)
        return fail(PBDR_ERR_DEVICE,
                    "a one-launch iteration gave up waiting for a contact partner (workgroups not resident together; "
                    "PBDR_FLAG_ITERATION_LAUNCHES avoids the form); the frame was discarded");
    if (err & pbdr::kErrInternal)
        return fail(PBDR_ERR_DEVICE, "an internal consistency check failed on the device; the frame was discarded");
    return PBDR_OK;
}

pbdr_status resolve(const pbdr_params* in, int32_t n, Resolved* out)
{
    if (!in) return fail(PBDR_ERR_INVALID_ARG, "params is NULL");
    const pbdr_params& p = *in;
    if (!(std::isfinite(p.dt_frame) && p.dt_frame > 0.0)) return fail(PBDR_ERR_INVALID_ARG, "dt_frame must be finite and > 0");
    if (p.substeps < 1 || p.substeps > 100000) return fail(PBDR_ERR_INVALID_ARG, "substeps must be in [1, 100000]");
    if (p.iterations < 0 || p.iterations > 100000) return fail(PBDR_ERR_INVALID_ARG, "iterations must be in [0, 100000]");
    if (!finite3(p.gravity)) return fail(PBDR_ERR_INVALID_ARG, "gravity must be finite");
    if (!(std::isfinite(p.friction_mu) && p.friction_mu >= 0.0)) return fail(PBDR_ERR_INVALID_ARG, "friction_mu must be finite and >= 0");
    if (!(std::isfinite(p.radius) && p.radius > 0.0)) return fail(PBDR_ERR_INVALID_ARG, "radius must be finite and > 0");
    if (!(std::isfinite(p.search_radius) && p.search_radius >= 0.0)) return fail(PBDR_ERR_INVALID_ARG, "search_radius must be finite and >= 0");
    if (!(std::isfinite(p.cell_size) && p.cell_size >= 0.0)) return fail(PBDR_ERR_INVALID_ARG, "cell_size must be finite and >= 0");
    if (!finite3(p.grid_origin)) return fail(PBDR_ERR_INVALID_ARG, "grid_origin must be finite");
    if (p.n_planes < 0 || p.n_planes > PBDR_MAX_PLANES) return fail(PBDR_ERR_INVALID_ARG, "n_planes must be in [0, %d]", PBDR_MAX_PLANES);
    for (int j = 0; j < p.n_planes; ++j) {
        const double* pl = p.planes[j];
        if (!(finite3(pl) && std::isfinite(pl[3]))) return fail(PBDR_ERR_INVALID_ARG, "plane %d is not finite", j);
        const double len = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        if (std::fabs(len - 1.0) > 1e-6) return fail(PBDR_ERR_INVALID_ARG, "plane %d normal is not unit length", j);
    }
    if (p.flags & ~kKnownFlags) return fail(PBDR_ERR_INVALID_ARG, "unknown flag bits 0x%x", p.flags & ~kKnownFlags);
    if ((p.flags & PBDR_PP_AVG_MASK) == (3u << 8)) return fail(PBDR_ERR_INVALID_ARG, "invalid pair averaging mode");
    if (p.nbr_cap < 0 || p.nbr_cap > pbdr::kMaxCap) return fail(PBDR_ERR_INVALID_ARG, "nbr_cap must be in [0, %d]", pbdr::kMaxCap);
    if (p.hash_bits != 0 && (p.hash_bits < kMinHashBits || p.hash_bits > kMaxHashBits))
        return fail(PBDR_ERR_INVALID_ARG, "hash_bits must be 0 or in [%d, %d]", kMinHashBits, kMaxHashBits);
    if (n < 0 || n > kMaxParticles) return fail(PBDR_ERR_INVALID_ARG, "particle count %d out of range", n);
    Resolved r;
    r.p = p;
    r.h = p.dt_frame / (double)p.substeps;
    r.rs = p.search_radius > 0.0 ? p.search_radius : 2.0 * p.radius;
    r.a = p.cell_size > 0.0 ? p.cell_size : r.rs * (1.0 + 1.0 / 1024.0);
    if (r.a < r.rs) return fail(PBDR_ERR_INVALID_ARG, "cell_size %g is below the search radius %g", r.a, r.rs);
    if (p.hash_bits) {
        r.k = p.hash_bits;
    } else {
        int k = 10;
        while (k < kMaxHashBits && (1ll << k) < 8ll * (long long)n) ++k;
        r.k = k;
    }
    r.cap = p.nbr_cap ? p.nbr_cap : 32;
    *out = r;
    return PBDR_OK;
}

}  // namespace host
}  // namespace pbdr

namespace {

using pbdr::host::fail;
using pbdr::host::Resolved;
using pbdr::host::resolve;
using pbdr::host::g_err;

struct Layout {
    size_t x, v, x0, mass, body, q, body_start, body_mass, body_mass64, dl0, dl1, vel0, vel1, xt, sxt4, key, kbuf0, kbuf1,
        ibuf0, ibuf1, nbr_n, nbr, hist, tile_off, cells, body_rot, counters, nbr_stats, wave_body,
        body_wave0, block_body, tagged, body_mq, body_out, total;
};

// Passes of the key sort (8-bit digits) for keys of `bits` bits.
int radix_passes(int bits) { return std::max(1, (bits + pbdr::kRadixBits - 1) / pbdr::kRadixBits); }

// Upper bound on the padded wave count of the iteration kernel's body packing:
// each body needs ceil(n_b / 64) <= n_b / 64 + 1 waves.  Greedy packing into
// workgroups of W waves wastes less than half of every workgroup it closes
// for lack of room.  In the 4-wave packing of the 80-VGPR kernel a body of
// more than 4 waves takes one workgroup of 4 waves, fewer than it needs.  The
// last workgroup is padded by at most W - 1 waves.
size_t max_iteration_waves(int32_t n, int32_t nb)
{
    return 4 * ((size_t)n / 64 + (size_t)nb + 2) + 2 * pbdr::kMaxWaves;
}

Layout make_layout(int32_t n, int32_t nb, int k, int cap)
{
    const size_t N = (size_t)n, B = (size_t)nb, T = (size_t)1 << k;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255u) & ~(size_t)255u;
        return o;
    };
    Layout L;
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
    L.cells = take(16 * T);
    L.body_rot = take(36 * B);
    L.counters = take(sizeof(pbdr::Counters));
    L.nbr_stats = take(sizeof(pbdr::NbrStats) * ((N + pbdr::kBlock - 1) / pbdr::kBlock));
    L.wave_body = take(4 * max_iteration_waves(n, nb));
    L.body_wave0 = take(4 * B);
    L.block_body = take(8 * (max_iteration_waves(n, nb) / 4 + 2));
    L.tagged = take(48 * N);
    L.body_mq = take(12 * B);
    L.body_out = take(18 * sizeof(double) * B);
    L.total = off;
    return L;
}

}  // namespace

struct pbdr_scene {
    Resolved res;
    Layout lay;
    pbdr::Scene dev;
    pbdr::StepConsts consts;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;          // one frame
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_n = nullptr;        // kGraphFrames frames
    hipGraphExec_t exec_n = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int max_body = 0;
    bool stepped = false;
    bool fixed_record = false;           // a reused host record (not freed by destroy)
    // the one-launch iteration form: possible for this scene (its grid alone
    // is resident at once), and the number of its workgroups the device holds
    bool one_launch_ok = false;
    int one_launch_capacity = 0;
    int device = 0;
};

namespace {

// Frames per graph for long step() calls: replaying one graph per frame
// leaves the GPU waiting on the host between graphs.
constexpr int kGraphFrames = 8;

// Scenes that can run their iterations as one launch, per process.  The
// one-launch kernel's workgroups wait for each other, so they must all be
// resident at once: a scene takes that form only while its grid and the
// grids of every such scene on another stream of its device fit on the device
// together (scenes on one stream run one after another).  Otherwise the call
// uses one launch per iteration (the same arithmetic, no waits).
std::mutex g_one_launch_mu;
std::vector<pbdr_scene*> g_one_launch;

void drop_graph(pbdr_scene* s);

void one_launch_register(pbdr_scene* s)
{
    if (!s->one_launch_ok) return;
    std::lock_guard<std::mutex> lock(g_one_launch_mu);
    g_one_launch.push_back(s);
}

void one_launch_unregister(pbdr_scene* s)
{
    std::lock_guard<std::mutex> lock(g_one_launch_mu);
    g_one_launch.erase(std::remove(g_one_launch.begin(), g_one_launch.end(), s), g_one_launch.end());
}

// Chooses the iteration form of the next enqueued work (drops graphs
// captured with the other form).
void choose_iteration_form(pbdr_scene* s)
{
    int want = 0;
    if (s->one_launch_ok) {
        std::lock_guard<std::mutex> lock(g_one_launch_mu);
        long long blocks = s->dev.n_iter_blocks;
        for (const pbdr_scene* o : g_one_launch)
            if (o != s && o->device == s->device && o->stream != s->stream) blocks += o->dev.n_iter_blocks;
        want = blocks <= (long long)s->one_launch_capacity ? 1 : 0;
    }
    if (want != s->dev.resident_iterate) {
        drop_graph(s);
        s->dev.resident_iterate = want;
    }
}

void drop_graph(pbdr_scene* s)
{
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->exec_n) (void)hipGraphExecDestroy(s->exec_n);
    if (s->graph_n) (void)hipGraphDestroy(s->graph_n);
    s->exec = nullptr;
    s->graph = nullptr;
    s->exec_n = nullptr;
    s->graph_n = nullptr;
}

pbdr_status read_counters(pbdr_scene* s, pbdr::Counters* c)
{
    HIP_TRY(hipMemcpyAsync(c, s->ws + s->lay.counters, sizeof(*c), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PBDR_OK;
}

// Reduces the per-workgroup neighbour statistics (synchronises).
pbdr_status read_nbr_stats(pbdr_scene* s, uint32_t* max_nbr, double* mean)
{
    const size_t slots = ((size_t)s->dev.n + pbdr::kBlock - 1) / pbdr::kBlock;
    std::vector<pbdr::NbrStats> st(slots);
    if (slots) HIP_TRY(hipMemcpyAsync(st.data(), s->ws + s->lay.nbr_stats, slots * sizeof(pbdr::NbrStats),
                                      hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    uint32_t mx = 0;
    unsigned long long sum = 0, rows = 0;
    for (const auto& e : st) {
        mx = std::max(mx, e.max_nbr);
        sum += e.sum;
        rows += e.rows;
    }
    if (max_nbr) *max_nbr = mx;
    if (mean) *mean = rows ? (double)sum / (double)rows : 0.0;
    return PBDR_OK;
}

pbdr_status latched(pbdr_scene* s)
{
    pbdr::Counters c;
    pbdr_status st = read_counters(s, &c);
    if (st != PBDR_OK) return st;
    uint32_t mx = 0;
    if (c.err & pbdr::kErrCapacity) read_nbr_stats(s, &mx, nullptr);
    return pbdr::host::latched_status(c.err, mx, s->res.cap);
}

void fill_consts(pbdr_scene* s) { pbdr::host::fill_step_consts(s->res, &s->consts); }

}  // namespace

void pbdr::host::fill_step_consts(const Resolved& r, pbdr::StepConsts* out)
{
    pbdr::StepConsts& c = *out;
    std::memset(&c, 0, sizeof(c));
    c.h = (float)r.h;
    c.inv_h = (float)(1.0 / r.h);
    for (int k = 0; k < 3; ++k) {
        c.g[k] = (float)r.p.gravity[k];
        c.origin[k] = (float)r.p.grid_origin[k];
    }
    c.mu = (float)r.p.friction_mu;
    c.radius = (float)r.p.radius;
    c.two_r = (float)(2.0 * r.p.radius);
    c.search_r2 = (float)(r.rs * r.rs);
    c.inv_cell = (float)(1.0 / r.a);
    c.key_mask = (uint32_t)((1ull << r.k) - 1ull);
    c.nbr_cap = r.cap;
    c.flags = r.p.flags;
    c.n_planes = r.p.n_planes;
    for (int j = 0; j < r.p.n_planes; ++j) {
        for (int k = 0; k < 3; ++k) c.plane_n[j][k] = (float)r.p.planes[j][k];
        c.plane_d[j] = (float)r.p.planes[j][3];
        c.plane_d_d[j] = r.p.planes[j][3];
    }
    c.radius_d = r.p.radius;
    c.two_r_d = 2.0 * r.p.radius;
}

namespace {

void fill_device(pbdr_scene* s, int32_t n, int32_t nb)
{
    char* w = s->ws;
    const Layout& L = s->lay;
    pbdr::Scene& d = s->dev;
    d.n = n;
    d.nb = nb;
    d.T = (uint32_t)(1ull << s->res.k);
    d.n_sort = n;
    d.radix_passes = radix_passes(s->res.k);
    d.radix_items = pbdr::radix_items_for((size_t)n);
    d.n_radix_tiles = (uint32_t)pbdr::radix_tiles_for((size_t)n);
    d.x = (float*)(w + L.x);
    d.v = (float*)(w + L.v);
    d.x0 = (float*)(w + L.x0);
    d.mass = (const float*)(w + L.mass);
    d.body = (const int32_t*)(w + L.body);
    d.q = (const float*)(w + L.q);
    d.body_start = (const int32_t*)(w + L.body_start);
    d.body_mass = (const float*)(w + L.body_mass);
    d.body_mass64 = (const double*)(w + L.body_mass64);
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
    d.skey = d.kbuf[(d.radix_passes - 1) & 1];
    d.sorted = d.ibuf[(d.radix_passes - 1) & 1];
    d.nbr_n = (uint32_t*)(w + L.nbr_n);
    d.nbr = (uint32_t*)(w + L.nbr);
    d.hist = (uint32_t*)(w + L.hist);
    d.tile_off = (uint32_t*)(w + L.tile_off);
    d.cells = (uint4*)(w + L.cells);
    d.body_rot = (float*)(w + L.body_rot);
    d.counters = (pbdr::Counters*)(w + L.counters);
    d.nbr_stats = (pbdr::NbrStats*)(w + L.nbr_stats);
    d.wave_body = (const int32_t*)(w + L.wave_body);
    d.body_wave0 = (const int32_t*)(w + L.body_wave0);
    d.block_body = (const int32_t*)(w + L.block_body);
    d.tagged = (unsigned long long*)(w + L.tagged);
    d.resident_iterate = 0;
    d.body_mq = (const float*)(w + L.body_mq);
    d.pscene = nullptr;                   // one scene
    d.mscene = nullptr;
    d.n_extent = n;
    d.n_active = n;
    d.accel = nullptr;
}

pbdr_status check_host_finite(const float* a, size_t count, const char* what)
{
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(a[i])) return fail(PBDR_ERR_INVALID_ARG, "%s[%zu] is not finite", what, i);
    return PBDR_OK;
}

pbdr_status enqueue(pbdr_scene* s, int32_t substeps_total)
{
    choose_iteration_form(s);
    hipError_t e = pbdr::enqueue_substeps(s->dev, s->consts, s->res.p.iterations, substeps_total,
                                          s->stream);
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    s->stepped = true;
    return PBDR_OK;
}

// Captures `frames` frames (each ending with the state written back) into a
// graph, instantiated once and replayed on the scene's stream.
pbdr_status capture(pbdr_scene* s, int frames, hipGraph_t* graph, hipGraphExec_t* exec)
{
    if (*exec) return PBDR_OK;
    if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int f = 0; f < frames && e == hipSuccess; ++f)
        e = pbdr::enqueue_substeps(s->dev, s->consts, s->res.p.iterations, s->res.p.substeps,
                                   s->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(PBDR_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    *graph = g;
    HIP_TRY(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0));
    return PBDR_OK;
}

}  // namespace

extern "C" {

int32_t pbdr_abi_version(void) { return PBDR_ABI_VERSION; }

pbdr_status pbdr_condition_status(uint32_t conditions)
{
    g_err[0] = 0;
    return pbdr::host::latched_status(conditions, 0u, 0);
}

const char* pbdr_last_error(void) { return g_err; }

size_t pbdr_scene_bytes(const pbdr_params* params, int32_t n_particles, int32_t n_bodies)
{
    Resolved r;
    if (resolve(params, n_particles, &r) != PBDR_OK) return 0;
    if (n_bodies < 0 || (n_particles > 0 && n_bodies < 1) || n_bodies > n_particles) {
        fail(PBDR_ERR_INVALID_ARG, "body count %d invalid for %d particles", n_bodies, n_particles);
        return 0;
    }
    return make_layout(n_particles, n_bodies, r.k, r.cap).total;
}

}  // extern "C"

namespace {

// pbdr_scene_create into `dev_workspace`; `fixed` (or NULL) is the host
// record to fill instead of a new one (the static scene of a device).
pbdr_status create_scene(const pbdr_params* params, const pbdr_scene_desc* desc, void* dev_workspace,
                         size_t ws_bytes, void* hip_stream, pbdr_scene* fixed, pbdr_scene** out)
{
    g_err[0] = 0;
    if (!out) return fail(PBDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(PBDR_ERR_INVALID_ARG, "desc is NULL");
    const int32_t n = desc->n_particles, nb = desc->n_bodies;
    Resolved r;
    pbdr_status st = resolve(params, n, &r);
    if (st != PBDR_OK) return st;
    if (nb < 0 || nb > n || (n > 0 && nb < 1)) return fail(PBDR_ERR_INVALID_ARG, "body count %d invalid for %d particles", nb, n);
    if (n > 0 && (!desc->x || !desc->v || !desc->mass || !desc->body_start))
        return fail(PBDR_ERR_INVALID_ARG, "desc arrays must not be NULL");
    int max_body = 0;
    if (n > 0) {
        if (desc->body_start[0] != 0 || desc->body_start[nb] != n)
            return fail(PBDR_ERR_INVALID_ARG, "body_start must begin at 0 and end at n_particles");
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t len = desc->body_start[b + 1] - desc->body_start[b];
            if (len < 1) return fail(PBDR_ERR_INVALID_ARG, "body %d is empty or body_start decreases", b);
            if (len > PBDR_MAX_BODY_PARTICLES)
                return fail(PBDR_ERR_INVALID_ARG, "body %d has %d particles (max %d)", b, len, PBDR_MAX_BODY_PARTICLES);
            if (len > max_body) max_body = len;
        }
        for (int32_t i = 0; i < n; ++i)
            if (!(std::isfinite(desc->mass[i]) && desc->mass[i] > 0.0f))
                return fail(PBDR_ERR_INVALID_ARG, "mass[%d] must be finite and > 0", i);
        if ((st = check_host_finite(desc->x, 3 * (size_t)n, "x")) != PBDR_OK) return st;
        if ((st = check_host_finite(desc->v, 3 * (size_t)n, "v")) != PBDR_OK) return st;
        if (desc->rest_q && (st = check_host_finite(desc->rest_q, 3 * (size_t)n, "rest_q")) != PBDR_OK) return st;
    }
    const Layout lay = make_layout(n, nb, r.k, r.cap);
    if (!dev_workspace) return fail(PBDR_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)dev_workspace & 255u) != 0) return fail(PBDR_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < lay.total) return fail(PBDR_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, lay.total);

    pbdr_scene* s = fixed;
    if (s) {
        *s = pbdr_scene();
        s->fixed_record = true;
        r.p.flags |= PBDR_FLAG_NO_GRAPH;       // direct launches: capturing a graph would allocate
    } else {
        s = new (std::nothrow) pbdr_scene();
        if (!s) return fail(PBDR_ERR_INVALID_ARG, "out of host memory");
    }
    auto discard = [&]() {
        if (!fixed) delete s;
    };
    s->res = r;
    s->lay = lay;
    s->stream = (hipStream_t)hip_stream;
    s->ws = (char*)dev_workspace;
    s->ws_bytes = ws_bytes;
    s->max_body = max_body;
    fill_device(s, n, nb);
    fill_consts(s);

    // iteration-kernel packing: each body takes ceil(n_b / 64) consecutive
    // waves; bodies are packed greedily, in order, into workgroups of W waves,
    // and a workgroup holds consecutive bodies only (its body-lane slots are
    // body ids from its first).  Returns the padded wave table and fills the
    // first wave of every packed body and each workgroup's (first body, count).
    auto pack = [&](int W, int min_need, int max_need, std::vector<int32_t>& waves, std::vector<int32_t>& blocks,
                    std::vector<int32_t>& body_wave0) {
        int32_t prev = -2;
        for (int32_t b = 0; b < nb; ++b) {
            const int need = (desc->body_start[b + 1] - desc->body_start[b] + 63) / 64;
            if (need < min_need || need > max_need) continue;
            const int used = (int)(waves.size() % (size_t)W);
            if (used > 0 && (used + need > W || b != prev + 1))
                waves.resize(waves.size() + (size_t)(W - used), -1);
            body_wave0[(size_t)b] = (int32_t)waves.size();
            waves.resize(waves.size() + (size_t)need, b);
            prev = b;
        }
        if (waves.size() % (size_t)W) waves.resize(waves.size() + (size_t)W - waves.size() % (size_t)W, -1);
        const size_t nblk = waves.size() / (size_t)W;
        blocks.assign(2 * nblk, 0);
        for (size_t blk = 0; blk < nblk; ++blk) {
            int32_t first = -1, last = -1;
            for (int w = 0; w < W; ++w) {
                const int32_t bb = waves[blk * W + w];
                if (bb < 0) continue;
                if (first < 0) first = bb;
                last = bb;
            }
            blocks[2 * blk] = first < 0 ? 0 : first;
            blocks[2 * blk + 1] = first < 0 ? 0 : last - first + 1;
        }
    };
    int cus = 256;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    }
    const int W = std::max(4, (max_body + 63) / 64);
    std::vector<int32_t> wave_body, block_body, body_wave0((size_t)nb);
    pack(W, 0, W, wave_body, block_body, body_wave0);
    s->dev.waves_per_block = W;
    s->dev.n_iter_blocks = (int32_t)(wave_body.size() / (size_t)W);
    // More workgroups than the GPU holds at once with 4 waves per SIMD (16 per
    // CU, the ~100-VGPR kernel): take the 80-VGPR kernel (6 waves per SIMD)
    // with workgroups of 4 waves, so that more of them share a CU.  Bodies of
    // more than 4 waves then take one such workgroup each, at the front of the
    // launch, which goes over their particles in chunks of 4 waves.
    s->dev.dense_iterate = s->dev.n_iter_blocks > cus * (16 / W) ? 1 : 0;
    s->dev.wide_bodies = W > pbdr::kWideBodyWaves ? 1 : 0;
    s->dev.n_chunked = 0;
    constexpr int kDenseWaves = 4;      // workgroup of the 80-VGPR kernel
    if (s->dev.dense_iterate && W > kDenseWaves) {
        wave_body.clear();
        for (int32_t b = 0; b < nb; ++b) {
            if ((desc->body_start[b + 1] - desc->body_start[b] + 63) / 64 <= kDenseWaves) continue;
            body_wave0[(size_t)b] = (int32_t)wave_body.size();
            wave_body.resize(wave_body.size() + kDenseWaves, b);
            s->dev.n_chunked += 1;
        }
        pack(kDenseWaves, 0, kDenseWaves, wave_body, block_body, body_wave0);   // (block_body of all)
        s->dev.waves_per_block = kDenseWaves;
        s->dev.n_iter_blocks = (int32_t)(wave_body.size() / kDenseWaves);
        s->dev.dense_iterate = 1;
        s->dev.wide_bodies = 0;
    }
    if (wave_body.size() > max_iteration_waves(n, nb) || block_body.size() / 2 > max_iteration_waves(n, nb) / 4 + 2) {
        discard();
        return fail(PBDR_ERR_INVALID_ARG, "internal: body packing exceeds its bound");
    }
    // all iterations of a substep in one launch when every workgroup of the
    // single iteration launch is resident at once (and K fits the 6-bit
    // iteration field of the tags)
    (void)hipGetDevice(&s->device);
    if (!s->dev.dense_iterate && !(s->res.p.flags & PBDR_FLAG_ITERATION_LAUNCHES) &&
        s->dev.n_iter_blocks > 0 && s->res.p.iterations < 64) {
        s->one_launch_capacity = pbdr::resident_iterate_capacity(s->dev.waves_per_block);
        s->one_launch_ok = s->dev.n_iter_blocks <= s->one_launch_capacity;
    }
    s->dev.resident_iterate = s->one_launch_ok ? 1 : 0;

    // rest pose (FP64): body mass, centre, q = x - c  (Sec. III-C, shape matching)
    std::vector<int32_t> body((size_t)n);
    std::vector<float> bmass((size_t)nb), q(3 * (size_t)n), bmq(3 * (size_t)nb);
    std::vector<double> bmass64((size_t)nb);
    for (int32_t b = 0; b < nb; ++b) {
        double M = 0.0, cm[3] = {0.0, 0.0, 0.0};
        for (int32_t i = desc->body_start[b]; i < desc->body_start[b + 1]; ++i) {
            body[(size_t)i] = b;
            const double m = desc->mass[i];
            M += m;
            for (int k = 0; k < 3; ++k) cm[k] += m * (double)desc->x[(size_t)k * n + i];
        }
        bmass[(size_t)b] = (float)M;
        bmass64[(size_t)b] = M;
        for (int k = 0; k < 3; ++k) cm[k] /= M;
        double mq[3] = {0.0, 0.0, 0.0};
        for (int32_t i = desc->body_start[b]; i < desc->body_start[b + 1]; ++i)
            for (int k = 0; k < 3; ++k) {
                const size_t j = (size_t)k * n + i;
                q[j] = desc->rest_q ? desc->rest_q[j] : (float)((double)desc->x[j] - cm[k]);
                mq[k] += (double)desc->mass[i] * (double)q[j];   // of the stored FP32 offsets
            }
        for (int k = 0; k < 3; ++k) bmq[3 * (size_t)b + k] = (float)mq[k];
    }
    auto h2d = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(s->ws + off, src, bytes, hipMemcpyHostToDevice, s->stream);
    };
    hipError_t e = hipSuccess;
    if (n > 0) {
        if (e == hipSuccess) e = h2d(lay.x, desc->x, 12 * (size_t)n);
        if (e == hipSuccess) e = h2d(lay.v, desc->v, 12 * (size_t)n);
        if (e == hipSuccess) e = h2d(lay.mass, desc->mass, 4 * (size_t)n);
        if (e == hipSuccess) e = h2d(lay.body, body.data(), 4 * (size_t)n);
        if (e == hipSuccess) e = h2d(lay.q, q.data(), 12 * (size_t)n);
        if (e == hipSuccess) e = h2d(lay.body_start, desc->body_start, 4 * ((size_t)nb + 1));
        if (e == hipSuccess) e = h2d(lay.body_mass, bmass.data(), 4 * (size_t)nb);
        if (e == hipSuccess) e = h2d(lay.body_mass64, bmass64.data(), 8 * (size_t)nb);
        if (e == hipSuccess) e = h2d(lay.wave_body, wave_body.data(), 4 * wave_body.size());
        if (e == hipSuccess) e = h2d(lay.body_wave0, body_wave0.data(), 4 * (size_t)nb);
        if (e == hipSuccess) e = h2d(lay.block_body, block_body.data(), 4 * block_body.size());
        if (e == hipSuccess) e = h2d(lay.body_mq, bmq.data(), 12 * (size_t)nb);
    }
    if (e == hipSuccess) e = pbdr::enqueue_clear_counters(s->dev, s->stream);
    if (e == hipSuccess) e = pbdr::enqueue_init_tables(s->dev, (size_t)s->dev.T, s->stream);
    // one-launch iterations: no tag may match before it is written
    if (e == hipSuccess) e = pbdr::enqueue_zero(s->dev.tagged, 48 * (size_t)n, s->stream);
    // the sort's buffers hold valid ids and keys from the start
    if (e == hipSuccess) e = pbdr::enqueue_zero(s->ws + lay.kbuf0, lay.nbr_n - lay.kbuf0, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        discard();
        return fail(PBDR_ERR_DEVICE, "scene upload failed: %s", hipGetErrorString(e));
    }
    one_launch_register(s);
    *out = s;
    return PBDR_OK;
}

constexpr int kFixedRecords = 64;
pbdr_scene g_fixed_scene[kFixedRecords];     // host records that are reused, not allocated

}  // namespace

pbdr_scene* pbdr::host::fixed_scene_record(int index)
{
    return index >= 0 && index < kFixedRecords ? &g_fixed_scene[index] : nullptr;
}

void pbdr::host::release_fixed_record(pbdr_scene* record)
{
    if (record && record->ws) {
        (void)hipStreamSynchronize(record->stream);
        one_launch_unregister(record);
        record->ws = nullptr;
    }
}

pbdr_status pbdr::host::create_scene_in(const pbdr_params* params, const pbdr_scene_desc* desc,
                                        void* dev_workspace, size_t ws_bytes, void* hip_stream,
                                        pbdr_scene* record, pbdr_scene** out)
{
    return create_scene(params, desc, dev_workspace, ws_bytes, hip_stream, record, out);
}

extern "C" {

pbdr_status pbdr_scene_create(const pbdr_params* params, const pbdr_scene_desc* desc, void* dev_workspace,
                              size_t ws_bytes, void* hip_stream, pbdr_scene** out)
{
    return create_scene(params, desc, dev_workspace, ws_bytes, hip_stream, nullptr, out);
}

pbdr_status pbdr_scene_set_accel(pbdr_scene* s, const float* accel_dev)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (s->dev.accel != accel_dev) drop_graph(s);
    s->dev.accel = accel_dev;
    return PBDR_OK;
}

pbdr_status pbdr_scene_set_stream(pbdr_scene* s, void* hip_stream)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::lock_guard<std::mutex> lock(g_one_launch_mu);
    s->stream = (hipStream_t)hip_stream;
    return PBDR_OK;
}

pbdr_status pbdr_scene_step(pbdr_scene* s, int32_t n_frames)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (n_frames < 0) return fail(PBDR_ERR_INVALID_ARG, "n_frames must be >= 0");
    if (n_frames == 0 || s->dev.n == 0) return PBDR_OK;
    if (s->res.p.flags & PBDR_FLAG_NO_GRAPH) {
        const long long total = (long long)n_frames * s->res.p.substeps;
        if (total > 0x7fffffffll) return fail(PBDR_ERR_INVALID_ARG, "too many substeps in one call");
        return enqueue(s, (int32_t)total);
    }
    choose_iteration_form(s);
    int32_t left = n_frames;
    if (left >= kGraphFrames) {
        pbdr_status st = capture(s, kGraphFrames, &s->graph_n, &s->exec_n);
        if (st != PBDR_OK) return st;
        for (; left >= kGraphFrames; left -= kGraphFrames) HIP_TRY(hipGraphLaunch(s->exec_n, s->stream));
    }
    if (left > 0) {
        pbdr_status st = capture(s, 1, &s->graph, &s->exec);
        if (st != PBDR_OK) return st;
        for (; left > 0; --left) HIP_TRY(hipGraphLaunch(s->exec, s->stream));
    }
    s->stepped = true;
    return PBDR_OK;
}

pbdr_status pbdr_scene_launch_iterations(pbdr_scene* s, int32_t n_launches)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (n_launches < 0) return fail(PBDR_ERR_INVALID_ARG, "n_launches must be >= 0");
    if (!s->stepped) return fail(PBDR_ERR_STATE, "no substep has run yet");
    choose_iteration_form(s);
    hipError_t e = pbdr::enqueue_iterations(s->dev, s->consts, s->res.p.iterations, n_launches,
                                            s->stream);
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return PBDR_OK;
}

pbdr_status pbdr_scene_time_iterations(pbdr_scene* s, int32_t n_launches, float* out_us)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (n_launches < 1 || n_launches > PBDR_MAX_TIMED_LAUNCHES)
        return fail(PBDR_ERR_INVALID_ARG, "n_launches must be in [1, %d]", PBDR_MAX_TIMED_LAUNCHES);
    if (!out_us) return fail(PBDR_ERR_INVALID_ARG, "out_us must not be NULL");
    if (!s->stepped) return fail(PBDR_ERR_STATE, "no substep has run yet");
    if (s->dev.n == 0) {
        for (int32_t i = 0; i < n_launches; ++i) out_us[i] = 0.0f;
        return PBDR_OK;
    }
    choose_iteration_form(s);
    std::vector<hipEvent_t> ev(2 * (size_t)n_launches, nullptr);
    auto release = [&]() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    };
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    if (e == hipSuccess)
        e = pbdr::enqueue_iterations_timed(s->dev, s->consts, s->res.p.iterations, n_launches,
                                           s->stream, ev.data(), ev.data() + n_launches);
    if (e == hipSuccess) e = hipEventSynchronize(ev.back());
    for (int32_t i = 0; i < n_launches && e == hipSuccess; ++i) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, ev[(size_t)i], ev[(size_t)n_launches + i]);
        out_us[i] = 1e3f * ms;
    }
    release();
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "timed iteration launches failed: %s", hipGetErrorString(e));
    return PBDR_OK;
}

pbdr_status pbdr_scene_substep(pbdr_scene* s, int32_t n_substeps)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (n_substeps < 0) return fail(PBDR_ERR_INVALID_ARG, "n_substeps must be >= 0");
    if (n_substeps == 0 || s->dev.n == 0) return PBDR_OK;
    return enqueue(s, n_substeps);
}

pbdr_status pbdr_scene_set_state(pbdr_scene* s, const float* x, const float* v, int32_t on_device)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    const size_t bytes = 12 * (size_t)s->dev.n;
    if (bytes == 0) return PBDR_OK;
    if (!x || !v) return fail(PBDR_ERR_INVALID_ARG, "x and v must not be NULL");
    if (!on_device) {
        pbdr_status st = check_host_finite(x, 3 * (size_t)s->dev.n, "x");
        if (st == PBDR_OK) st = check_host_finite(v, 3 * (size_t)s->dev.n, "v");
        if (st != PBDR_OK) return st;
    }
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(s->ws + s->lay.x, x, bytes, kind, s->stream));
    HIP_TRY(hipMemcpyAsync(s->ws + s->lay.v, v, bytes, kind, s->stream));
    HIP_TRY(pbdr::enqueue_clear_counters(s->dev, s->stream));
    if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));
    return PBDR_OK;
}

pbdr_status pbdr_scene_read_state(pbdr_scene* s, float* x, float* v, int32_t on_device)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    const size_t bytes = 12 * (size_t)s->dev.n;
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (bytes && x) HIP_TRY(hipMemcpyAsync(x, s->ws + s->lay.x, bytes, kind, s->stream));
    if (bytes && v) HIP_TRY(hipMemcpyAsync(v, s->ws + s->lay.v, bytes, kind, s->stream));
    return latched(s);
}

pbdr_status pbdr_scene_read_bodies(pbdr_scene* s, double* com, double* rot9, double* P, double* L)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    const size_t B = (size_t)s->dev.nb;
    if (B == 0) return latched(s);
    double* dev_out = reinterpret_cast<double*>(s->ws + s->lay.body_out);
    hipError_t e = pbdr::enqueue_body_state(s->dev, dev_out, s->stream);
    if (e != hipSuccess) return fail(PBDR_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    std::vector<double> h(18 * B);
    HIP_TRY(hipMemcpyAsync(h.data(), dev_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (size_t b = 0; b < B; ++b) {
        const double* o = h.data() + 18 * b;
        for (int k = 0; k < 3; ++k) {
            if (com) com[3 * b + k] = o[k];
            if (P) P[3 * b + k] = o[12 + k];
            if (L) L[3 * b + k] = o[15 + k];
        }
        if (rot9)
            for (int k = 0; k < 9; ++k) rot9[9 * b + k] = o[3 + k];
    }
    return latched(s);
}

pbdr_status pbdr_scene_read_rest(pbdr_scene* s, float* rest_q)
{
    if (!s || !rest_q) return fail(PBDR_ERR_INVALID_ARG, "scene and rest_q must not be NULL");
    const size_t bytes = 12 * (size_t)s->dev.n;
    if (bytes) HIP_TRY(hipMemcpyAsync(rest_q, s->ws + s->lay.q, bytes, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PBDR_OK;
}

pbdr_status pbdr_scene_check(pbdr_scene* s, int32_t* max_neighbours)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    if (max_neighbours) {
        uint32_t mx = 0;
        pbdr_status st = read_nbr_stats(s, &mx, nullptr);
        if (st != PBDR_OK) return st;
        *max_neighbours = (int32_t)mx;
    }
    return latched(s);
}

pbdr_status pbdr_scene_neighbour_stats(pbdr_scene* s, int32_t* max_neighbours, double* mean_neighbours)
{
    if (!s) return fail(PBDR_ERR_INVALID_ARG, "scene is NULL");
    uint32_t mx = 0;
    pbdr_status st = read_nbr_stats(s, &mx, mean_neighbours);
    if (st != PBDR_OK) return st;
    if (max_neighbours) *max_neighbours = (int32_t)mx;
    return PBDR_OK;
}

pbdr_status pbdr_scene_read_debug(pbdr_scene* s, int32_t what, void* dst)
{
    if (!s || !dst) return fail(PBDR_ERR_INVALID_ARG, "scene and dst must not be NULL");
    const size_t N = (size_t)s->dev.n, T = (size_t)s->dev.T;
    size_t off = 0, bytes = 0;
    switch (what) {
    case PBDR_DEBUG_XT: off = s->lay.xt; bytes = 12 * N; break;
    case PBDR_DEBUG_KEYS: off = s->lay.key; bytes = 4 * N; break;
    case PBDR_DEBUG_SORTED:
        if (!s->stepped) return fail(PBDR_ERR_STATE, "no substep has run yet");
        off = (size_t)((const char*)s->dev.sorted - s->ws);
        bytes = 4 * N;
        break;
    case PBDR_DEBUG_CELL_START:
    case PBDR_DEBUG_CELL_COUNT: {   // the per-key entries of the last substep
        if (!s->stepped) return fail(PBDR_ERR_STATE, "no substep has run yet");
        std::vector<uint32_t> e(4 * T);
        pbdr::Counters c;
        HIP_TRY(hipMemcpyAsync(e.data(), s->ws + s->lay.cells, 16 * T, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipMemcpyAsync(&c, s->ws + s->lay.counters, sizeof(c), hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
        uint32_t* out = (uint32_t*)dst;
        // an entry of an earlier substep is an empty key, whose first slot is
        // that of the next occupied key (or N)
        uint32_t next = (uint32_t)N;
        for (size_t k = T; k-- > 0;) {
            const uint32_t* ek = e.data() + 4 * k;
            const bool occ = ek[3] == c.epoch;
            if (occ) next = ek[0];
            out[k] = what == PBDR_DEBUG_CELL_START ? next : (occ ? ek[1] - ek[0] : 0u);
        }
        return PBDR_OK;
    }
    case PBDR_DEBUG_NBR_COUNT: off = s->lay.nbr_n; bytes = 4 * N; break;
    case PBDR_DEBUG_NBR: off = s->lay.nbr; bytes = 4 * N * (size_t)s->res.cap; break;
    case PBDR_DEBUG_DELTA:
        off = (s->res.p.iterations % 2 == 0) ? s->lay.dl0 : s->lay.dl1;
        bytes = 12 * N;
        break;
    default: return fail(PBDR_ERR_INVALID_ARG, "unknown debug buffer %d", what);
    }
    if (bytes) HIP_TRY(hipMemcpyAsync(dst, s->ws + off, bytes, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PBDR_OK;
}

pbdr_status pbdr_scene_info_get(const pbdr_scene* s, pbdr_scene_info* out)
{
    if (!s || !out) return fail(PBDR_ERR_INVALID_ARG, "scene and out must not be NULL");
    out->n_particles = s->dev.n;
    out->n_bodies = s->dev.nb;
    out->hash_bits = s->res.k;
    out->nbr_cap = s->res.cap;
    out->substep_h = s->res.h;
    out->search_radius = s->res.rs;
    out->cell_size = s->res.a;
    out->waves_per_block = s->dev.waves_per_block;
    out->iteration_blocks = s->dev.n_iter_blocks;
    out->max_body_particles = s->max_body;
    out->iteration_kernel = s->dev.resident_iterate ? 2 : s->dev.dense_iterate;
    out->workspace_bytes = s->lay.total;
    return PBDR_OK;
}

void pbdr_scene_destroy(pbdr_scene* s)
{
    if (!s) return;
    // the scene's work ends before the caller may free the workspace
    (void)hipStreamSynchronize(s->stream);
    one_launch_unregister(s);
    drop_graph(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->fixed_record) {         // a reused host record: released, not freed
        s->ws = nullptr;
        return;
    }
    delete s;
}

}  // extern "C"
