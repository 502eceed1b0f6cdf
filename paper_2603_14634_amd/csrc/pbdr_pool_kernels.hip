// Scene pools on gfx950: many independent scenes, one workgroup each.
//
// A workgroup runs every substep of its scene for the whole call (units x
// substeps), with workgroup barriers only: scenes never interact, so no grid
// synchronisation or relaunch is needed between substeps or iterations.  The
// substep is the same as the single-scene path (Alg. 1 with the velocity update
// of Sec. III-B and the momentum constraint of Sec. III-C, Eqs. (4)-(5)):
//
//   predict      integration step; X_init is published for neighbours
//   index        cell keys counted into a workgroup-local hash table in LDS,
//                scanned, particles grouped by key
//   broad phase  boxes of every body's predicted positions; a particle more
//                than 2 R_s from every other body's box has no neighbours
//   neighbours   27-cell walk, same-body candidates skipped before any position
//                is loaded, FP32 predicate, ascending lists
//   iterate x K  contacts, shape matching and momentum constraint; per-body
//                sums are fixed-order wave reductions (DPP) over the body's
//                64-lane slots, combined in slot order by one lane per body
//
// Bodies are wave-aligned: body b owns ceil(n_b / 64) consecutive slots of 64
// lanes, one particle per lane, so a slot never mixes bodies.
//
// Two kernels share this arithmetic:
//   k_pool      scenes of up to 8192 particles and 64 bodies (128 slots); the
//               particle state stays in registers for the whole call, slot s in
//               register set s / W of wave s % W, and the key-grouped ids live
//               in LDS
//   k_pool_big  scenes of up to 65535 particles and 256 bodies; 16 waves walk
//               the slots in every phase and the state, ids and slot sums stay
//               in global memory (L2)
// Every sum and every list is independent of W, of the register sets per lane
// and of the hash-table size, so a scene's result does not depend on the
// launch shape or on the other scenes of the pool.
#include "pbdr_math.h"
#include "pbdr_pool_device.h"

namespace pbdr {
namespace {

using namespace dev;

constexpr int kSums = 24;             // per-slot partial sums (12 shape matching, 21 momentum)

// Fixed-pattern DPP move; lanes the pattern does not feed keep v.
template <int CTRL, int ROWS>
__device__ inline float dpp_keep(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v),
                                                                 CTRL, ROWS, 0xf, false));
}

// Minimum and maximum over the 64 lanes (valid in lane 63), same tree as the sums.
__device__ inline float wave_min_to_63(float v)
{
    v = fminf(v, dpp_keep<0xb1, 0xf>(v));
    v = fminf(v, dpp_keep<0x4e, 0xf>(v));
    v = fminf(v, dpp_keep<0x141, 0xf>(v));
    v = fminf(v, dpp_keep<0x140, 0xf>(v));
    v = fminf(v, dpp_keep<0x142, 0xa>(v));
    v = fminf(v, dpp_keep<0x143, 0xc>(v));
    return v;
}

__device__ inline float wave_max_to_63(float v)
{
    v = fmaxf(v, dpp_keep<0xb1, 0xf>(v));
    v = fmaxf(v, dpp_keep<0x4e, 0xf>(v));
    v = fmaxf(v, dpp_keep<0x141, 0xf>(v));
    v = fmaxf(v, dpp_keep<0x140, 0xf>(v));
    v = fmaxf(v, dpp_keep<0x142, 0xa>(v));
    v = fmaxf(v, dpp_keep<0x143, 0xc>(v));
    return v;
}

// Exclusive scan of one value per thread over the workgroup; `tot` gets the total.
__device__ inline uint32_t wg_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, W = blockDim.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_tot[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < W; ++w) {
        const uint32_t t = wave_tot[w];
        if (w < wave) before += t;
        all += t;
    }
    *tot = all;
    __syncthreads();          // wave_tot may be reused right after
    return before + x - v;
}

// Exclusive scan of the Tc key counts in tab (in place); tab[Tc] = n.
__device__ inline void scan_keys(uint32_t* tab, uint32_t Tc, int n, uint32_t* wave_tot)
{
    const int T = blockDim.x, tid = threadIdx.x;
    const uint32_t per = Tc > (uint32_t)T ? Tc / (uint32_t)T : 1u;
    const uint32_t k0 = (uint32_t)tid * per;
    uint32_t run = 0;
    if (k0 < Tc)
        for (uint32_t j = 0; j < per; ++j) run += tab[k0 + j];
    uint32_t tot;
    uint32_t ex = wg_exclusive_scan(run, wave_tot, &tot);
    if (k0 < Tc)
        for (uint32_t j = 0; j < per; ++j) {
            const uint32_t cnt = tab[k0 + j];
            tab[k0 + j] = ex;
            ex += cnt;
        }
    if (tid == 0) tab[Tc] = (uint32_t)n;
}

// Per-body LDS record (floats).
enum : int {
    kBM = 0,          // body mass
    kBMq = 1,         // sum m q (3)
    kBAnchor = 4,     // X_init of the body's first particle (3)
    kBR = 7,          // rotation (9)
    kBC = 16,         // centre relative to the anchor (3)
    kBDv = 19,        // linear correction (3)
    kBW = 22,         // angular velocity correction (3)
    kBCa = 25,        // c_asm - c_i (3)
    kBRprev = 28,     // previous iteration's rotation (9)
    kBFirst = 37,     // first particle (int bits)
    kBSlot0 = 38,     // first slot (int bits)
    kBSlots = 39,     // slot count (int bits)
    kBLo = 40,        // box of the predicted positions: lower corner (3)
    kBHi = 43,        // upper corner (3)
    kBFar = 46,       // 1: coordinates too large for the box test (int bits)
};

// Per-scene values every phase needs.
struct Ctx {
    const PoolDev* d;
    const PoolConsts* c;
    int n, p0;
    size_t P;
    float g[3], mu;
    uint32_t avg, mask;
    int cap;
    uint32_t* lists;
};

// Integration step (Alg. 1, first loop) in the FP32 recipe of the hash grid.
__device__ inline void predict_one(const Ctx& x, const float* x0, float* V, float* del, float* xt)
{
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) {
        const float dv = x.c->h * x.g[k];
        const float vt = V[k] + dv;
        const float dx = x.c->h * vt;
        xt[k] = x0[k] + dx;
        del[k] = dx;        // delta_0 = X~ - X_init
        V[k] = vt;          // V_0 = V~
    }
}

__device__ inline uint32_t cell_key(const Ctx& x, const float* xt)
{
    const PoolConsts& c = *x.c;
    return morton(cell_axis(xt[0], c.origin[0], c.inv_cell), cell_axis(xt[1], c.origin[1], c.inv_cell),
                  cell_axis(xt[2], c.origin[2], c.inv_cell), x.mask);
}

// Box of a body from its slots' boxes (slot s at boxes + s * stride).
__device__ inline void body_box(const Ctx& x, float* br, const float* boxes, int stride)
{
    const int s0 = __float_as_int(br[kBSlot0]), ns = __float_as_int(br[kBSlots]);
    float bx[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int sl = s0; sl < s0 + ns; ++sl)
        for (int k = 0; k < 3; ++k) {
            bx[k] = fminf(bx[k], boxes[sl * stride + k]);
            bx[3 + k] = fmaxf(bx[3 + k], boxes[sl * stride + 3 + k]);
        }
    const float lim = 1048576.0f * x.c->search_r;     // beyond 2^20 R_s the margin may not cover rounding
    bool far = false;
    for (int k = 0; k < 3; ++k) {
        br[kBLo + k] = bx[k];
        br[kBHi + k] = bx[3 + k];
        far = far || !(fabsf(bx[k]) < lim) || !(fabsf(bx[3 + k]) < lim);
    }
    br[kBFar] = __int_as_float(far ? 1 : 0);
}

__device__ inline bool boxes_near(const Ctx& x, const float* ba, const float* bb)
{
    if (__float_as_int(ba[kBFar]) || __float_as_int(bb[kBFar])) return true;
    const float e = x.c->box_margin;
    bool near = true;
    for (int k = 0; k < 3; ++k) near = near && ba[kBLo + k] - e <= bb[kBHi + k] && bb[kBLo + k] - e <= ba[kBHi + k];
    return near;
}

// A particle farther than 2 R_s (on some axis) from a body's box has no
// neighbour in it: every FP32 predicate with that body's particles is false.
__device__ inline bool point_near(const Ctx& x, const float* xt, const float* bo)
{
    if (__float_as_int(bo[kBFar])) return true;
    const float e = x.c->box_margin;
    bool in = true;
    for (int k = 0; k < 3; ++k) in = in && xt[k] >= bo[kBLo + k] - e && xt[k] <= bo[kBHi + k] + e;
    return in;
}

// 27-cell walk of particle i (body bdy): tab holds the key starts, sid the
// key-grouped (id | body << 16) entries, sxt the key-grouped predicted
// positions.  Writes the ascending list (the cap smallest ids) and returns
// the true count.
__device__ inline uint32_t walk(const Ctx& x, const uint32_t* tab, const uint32_t* sid, const float4* sxt, int i,
                                int bdy, const float* xt)
{
    const PoolConsts& c = *x.c;
    const int cap = x.cap, n = x.n;
    uint32_t* lists = x.lists;
    const uint32_t cx = cell_axis(xt[0], c.origin[0], c.inv_cell);
    const uint32_t cy = cell_axis(xt[1], c.origin[1], c.inv_cell);
    const uint32_t cz = cell_axis(xt[2], c.origin[2], c.inv_cell);
    uint32_t cnt = 0;
    for (int t = 0; t < 27; ++t) {
        const uint32_t k = morton(cx + (uint32_t)(t % 3 - 1), cy + (uint32_t)((t / 3) % 3 - 1), cz + (uint32_t)(t / 9 - 1),
                                  x.mask);
        const uint32_t a = tab[k], e = tab[k + 1];
        for (uint32_t qq = a; qq < e; ++qq) {
            const uint32_t en = sid[qq];
            if ((int)(en >> 16) == bdy) continue;              // same body (also i itself)
            const float4 o = sxt[qq];
            if (!within(xt[0], xt[1], xt[2], o.x, o.y, o.z, c.search_r2)) continue;
            const uint32_t id = en & 0xffffu;
            // insert keeping the `cap` smallest ids in ascending order
            const int mm = (int)(cnt < (uint32_t)cap ? cnt : (uint32_t)cap);
            ++cnt;
            if (mm == cap && id > lists[(size_t)(cap - 1) * n + i]) continue;
            int pos = mm == cap ? cap - 1 : mm;
            while (pos > 0) {
                const uint32_t prev = lists[(size_t)(pos - 1) * n + i];
                if (prev < id) break;
                lists[(size_t)pos * n + i] = prev;
                --pos;
            }
            lists[(size_t)pos * n + i] = id;
        }
    }
    return cnt;
}

// Contact displacement of particle i from X_i (Jacobi): planes (constraint
// (1)) and particles of other bodies (constraint (2)); friction from the
// displacement since X_init.
__device__ inline void contacts(const Ctx& x, int i, const float* x0, const float* del, float m, uint32_t ni, float* Cd)
{
    const PoolConsts& c = *x.c;
    const PoolDev& d = *x.d;
    const size_t P = x.P;
    for (int k = 0; k < 3; ++k) Cd[k] = 0.0f;
    // planes clearly out of contact range in FP32 (by 2^-20 of the magnitudes
    // involved, several times that evaluation's rounding bound) skip the FP64 test
    const float mag = fabsf(x0[0]) + fabsf(x0[1]) + fabsf(x0[2]) + fabsf(del[0]) + fabsf(del[1]) + fabsf(del[2]);
    for (int pl = 0; pl < c.n_planes; ++pl) {
        const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
        const float e32 = nx * (x0[0] + del[0]) + ny * (x0[1] + del[1]) + nz * (x0[2] + del[2]) - c.plane_d[pl];
        if (e32 > c.radius + 0x1p-20f * (mag + fabsf(c.plane_d[pl]))) continue;
        const float un = nx * del[0] + ny * del[1] + nz * del[2];
        // signed distance and penetration in FP64, rounded only as a correction
        double e = -c.plane_d_d[pl];
        for (int k = 0; k < 3; ++k) e += (double)c.plane_n[pl][k] * ((double)x0[k] + (double)del[k]);
        if (!(e < c.radius_d)) continue;
        const float pen = (float)(c.radius_d - e);
        const float ux = del[0] - un * nx, uy = del[1] - un * ny, uz = del[2] - un * nz;
        const float ut2 = ux * ux + uy * uy + uz * uz;
        const float f = ut2 > 0.0f ? fminf(1.0f, x.mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
        Cd[0] += pen * nx - f * ux;
        Cd[1] += pen * ny - f * uy;
        Cd[2] += pen * nz - f * uz;
    }
    const uint32_t stored = ni < (uint32_t)x.cap ? ni : (uint32_t)x.cap;
    for (uint32_t sl = 0; sl < stored; ++sl) {
        const uint32_t jq = x.lists[(size_t)sl * x.n + i];
        const size_t gq = (size_t)x.p0 + jq;
        // separation, distance, penetration and normal in FP64
        double dd[3];
        float u[3];
        for (int k = 0; k < 3; ++k) {
            const float dj = d.dl[k * P + gq];
            dd[k] = ((double)x0[k] - (double)d.x0[k * P + gq]) + ((double)del[k] - (double)dj);
            u[k] = del[k] - dj;
        }
        const double l2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
        if (!(l2 > 0.0) || !(l2 < c.two_r_d * c.two_r_d)) continue;
        const double il = rsqrt64(l2);
        const double l = l2 * il;
        const float nx = (float)(dd[0] * il), ny = (float)(dd[1] * il), nz = (float)(dd[2] * il);
        const float pen = (float)(c.two_r_d - l);
        const float mq = d.mass[gq];
        const float alpha = mq * frcp(m + mq);           // w_p / (w_p + w_q)
        const float un = u[0] * nx + u[1] * ny + u[2] * nz;
        const float ux = u[0] - un * nx, uy = u[1] - un * ny, uz = u[2] - un * nz;
        const float ut2 = ux * ux + uy * uy + uz * uz;
        const float f = ut2 > 0.0f ? fminf(1.0f, x.mu * pen * __builtin_amdgcn_rsqf(ut2)) : 0.0f;
        float wgt = 1.0f;
        if (x.avg == 0u) {
            const uint32_t nq = d.nbr_n[gq];
            wgt = frcp((float)(ni > nq ? ni : nq));
        } else if (x.avg == 1u) {
            wgt = frcp((float)ni);
        }
        const float scl = alpha * wgt;
        Cd[0] += scl * (pen * nx - f * ux);
        Cd[1] += scl * (pen * ny - f * uy);
        Cd[2] += scl * (pen * nz - f * uz);
    }
}

// Shape-matching terms of one particle: m y and m y q^T, y = X_i - anchor.
__device__ inline void sm_terms(bool act, const float* br, const float* x0, const float* del, const float* q, float m,
                                float* Sv)
{
    float y[3];
    for (int k = 0; k < 3; ++k) y[k] = act ? (x0[k] - br[kBAnchor + k]) + del[k] : 0.0f;
    for (int k = 0; k < 3; ++k) Sv[k] = m * y[k];
    for (int a = 0; a < 3; ++a)
        for (int k2 = 0; k2 < 3; ++k2) Sv[3 + 3 * a + k2] = m * y[a] * q[k2];
}

// Offsets of a particle in the frame centred on the body's current centre:
// r = (X_i - anchor) - c and the shape-matching goal offset D = R q - r.  D's
// terms are body-sized while D is of the order of the contact corrections, so
// it is formed in FP64 (products of FP32 values and the anchor difference are
// exact there; only the result is rounded): in FP32 each particle's goal
// would carry a rounding of ~ulp(0.1 m) that no rigid motion absorbs.
__device__ inline void goal_offsets(bool act, const float* br, const float* x0, const float* del, const float* q,
                                    float* rr, float* Dd)
{
    for (int k = 0; k < 3; ++k) rr[k] = ((x0[k] - br[kBAnchor + k]) + del[k]) - br[kBC + k];
    for (int a = 0; a < 3; ++a) {
        const double rq = (double)br[kBR + 3 * a] * (double)q[0] + (double)br[kBR + 3 * a + 1] * (double)q[1] +
                          (double)br[kBR + 3 * a + 2] * (double)q[2];
        const double ya = ((double)x0[a] - (double)br[kBAnchor + a]) + (double)del[a];
        Dd[a] = act ? (float)(rq - (ya - (double)br[kBC + a])) : 0.0f;
    }
}

// Momentum terms of one particle (Eqs. (4)-(5) in the frame centred on c_i):
// m C, m D, m v_b, m z_b x D, m D x v_b, and the inertia terms of z_a.
__device__ inline void mom_terms(const Ctx& x, bool act, const float* br, const float* x0, const float* del,
                                 const float* q, const float* V, const float* Cd, float m, float* Sv)
{
    float rr[3], Dd[3], zb[3], za[3], vb[3], t3[3];
    goal_offsets(act, br, x0, del, q, rr, Dd);
    for (int k = 0; k < 3; ++k) {
        zb[k] = rr[k] + Cd[k];
        za[k] = zb[k] + Dd[k];
        vb[k] = V[k] + Cd[k] * x.c->inv_h;
        Sv[k] = m * Cd[k];
        Sv[3 + k] = m * Dd[k];
        Sv[6 + k] = m * vb[k];
    }
    cross(zb, Dd, t3);
    for (int k = 0; k < 3; ++k) Sv[9 + k] = m * t3[k];
    cross(Dd, vb, t3);
    for (int k = 0; k < 3; ++k) Sv[12 + k] = m * t3[k];
    Sv[15] = m * (za[1] * za[1] + za[2] * za[2]);
    Sv[16] = m * (za[0] * za[0] + za[2] * za[2]);
    Sv[17] = m * (za[0] * za[0] + za[1] * za[1]);
    Sv[18] = -m * za[0] * za[1];
    Sv[19] = -m * za[0] * za[2];
    Sv[20] = -m * za[1] * za[2];
    Sv[21] = Sv[22] = Sv[23] = 0.0f;
}

// Sums a wave's 4 NV terms over its lanes and stores them at dst[0 .. 4 NV):
// after the reduction row j of the wave holds terms j NV .. j NV + NV - 1, and
// one lane per row stores them.
template <int NV>
__device__ inline void wave_store(float* Sv, float* dst, int lane)
{
    wave_sums_by_row<4 * NV>(Sv);
    if ((lane & 15) == 15) {
        float* d = dst + (lane >> 4) * NV;
        for (int j = 0; j < NV; ++j) d[j] = Sv[j];
    }
}

// Body lane: centre, covariance and rotation from the slot sums (Sec. III-C).
__device__ inline void body_rotation(float* br, const float* part, int it)
{
    const int s0 = __float_as_int(br[kBSlot0]), ns = __float_as_int(br[kBSlots]);
    float Tt[12];
    for (int j = 0; j < 12; ++j) Tt[j] = 0.0f;
    for (int s = s0; s < s0 + ns; ++s) {
        const float* pp = part + s * kSums;
        for (int j = 0; j < 12; ++j) Tt[j] += pp[j];
    }
    const float im = frcp(br[kBM]);
    float cc[3], A[9], Rb[9];
    for (int k = 0; k < 3; ++k) cc[k] = Tt[k] * im;
    for (int a = 0; a < 3; ++a)
        for (int k2 = 0; k2 < 3; ++k2) A[3 * a + k2] = Tt[3 + 3 * a + k2] - cc[a] * br[kBMq + k2];
    if (!(it > 0 && polar_refine(A, br + kBRprev, Rb))) polar_rotation(A, Rb);
    for (int j = 0; j < 9; ++j) br[kBR + j] = br[kBRprev + j] = Rb[j];
    for (int k = 0; k < 3; ++k) br[kBC + k] = cc[k];
}

// Body lane: momentum conservation constraint, Eqs. (4)-(5).
__device__ inline void body_momentum(const PoolConsts& c, float* br, const float* part)
{
    const int s0 = __float_as_int(br[kBSlot0]), ns = __float_as_int(br[kBSlots]);
    float Tt[21];
    for (int j = 0; j < 21; ++j) Tt[j] = 0.0f;
    for (int s = s0; s < s0 + ns; ++s) {
        const float* pp = part + s * kSums;
        for (int j = 0; j < 21; ++j) Tt[j] += pp[j];
    }
    const float Mb = br[kBM], im = frcp(Mb);
    float cb[3], Db[3], cab[3], dvb[3] = {0.0f, 0.0f, 0.0f}, wb[3] = {0.0f, 0.0f, 0.0f};
    for (int k = 0; k < 3; ++k) {
        cb[k] = Tt[k] * im;          // c_bsm - c_i
        Db[k] = Tt[3 + k] * im;      // mean shape-matching shift
        cab[k] = cb[k] + Db[k];      // c_asm - c_i
    }
    // Eq. (4): dv = (P_bsm - P_asm) / M, P_asm - P_bsm = sum m D / dt
    if (!(c.flags & kFlagNoLinMom))
        for (int k = 0; k < 3; ++k) dvb[k] = -Tt[3 + k] * c.inv_h * im;
    // Eq. (5): omega = I^-1 (L_asm - L_bsm), the difference formed from the
    // small quantities; inertia moved from c_i to c_asm (parallel axes)
    if (!(c.flags & kFlagNoAngMom)) {
        float cbxD[3], DbxP[3], dL[3], I6[6];
        cross(cb, &Tt[3], cbxD);
        cross(Db, &Tt[6], DbxP);
        for (int k = 0; k < 3; ++k) dL[k] = (Tt[9 + k] - cbxD[k]) * c.inv_h + Tt[12 + k] - DbxP[k];
        I6[0] = Tt[15] - Mb * (cab[1] * cab[1] + cab[2] * cab[2]);
        I6[1] = Tt[16] - Mb * (cab[0] * cab[0] + cab[2] * cab[2]);
        I6[2] = Tt[17] - Mb * (cab[0] * cab[0] + cab[1] * cab[1]);
        I6[3] = Tt[18] + Mb * cab[0] * cab[1];
        I6[4] = Tt[19] + Mb * cab[0] * cab[2];
        I6[5] = Tt[20] + Mb * cab[1] * cab[2];
        const float scale = fmaxf(I6[0] + I6[1] + I6[2], Mb * c.two_r * c.two_r);
        solve_inertia(I6, dL, scale, wb);
    }
    for (int k = 0; k < 3; ++k) {
        br[kBDv + k] = dvb[k];
        br[kBW + k] = wb[k];
        br[kBCa + k] = cab[k];
    }
}

// Particle update X_{i+1}, V_{i+1} (incremental velocity, Sec. III-B) with
// the momentum correction of its body.
__device__ inline void update_one(const PoolConsts& c, const float* br, const float* x0, const float* q,
                                  const float* Cd, float* del, float* V)
{
    float rr[3], Dd[3], ra[3], wr[3], w3[3];
    goal_offsets(true, br, x0, del, q, rr, Dd);
    for (int k = 0; k < 3; ++k) {
        ra[k] = rr[k] + Cd[k] + Dd[k] - br[kBCa + k];
        w3[k] = br[kBW + k];
    }
    cross(w3, ra, wr);
    for (int k = 0; k < 3; ++k) {
        const float step = Cd[k] + Dd[k];
        const float dvi = br[kBDv + k] - wr[k];
        const float dnew = (del[k] + step) + c.h * dvi;
        if (c.flags & kFlagStdVelocity) {
            // standard PBD: V = (X_{i+1} - X_init) / dt in world FP32 coordinates
            const float xw = x0[k] + dnew;
            V[k] = (xw - x0[k]) * c.inv_h;
        } else {
            V[k] = (V[k] + step * c.inv_h) + dvi;
        }
        del[k] = dnew;
    }
}

// Body records and the wave-aligned slot table; returns the slot count (the
// table holds at most max_slots).  Synchronises the workgroup.
__device__ inline int setup_bodies(const PoolDev& d, int b0, int nb, int n, float* bod, int2* slot_tab, int max_slots,
                                   uint32_t* misc)
{
    const int T = blockDim.x, tid = threadIdx.x;
    for (int b = tid; b < nb; b += T) {
        float* r = bod + b * kPoolBodyFloats;
        r[kBM] = d.body_mass[b0 + b];
        for (int k = 0; k < 3; ++k) r[kBMq + k] = d.body_mq[3 * (size_t)(b0 + b) + k];
        r[kBFirst] = __int_as_float(d.body_first[b0 + b]);
    }
    if (tid == 0) {
        misc[16] = 0u;   // error bits
        misc[17] = 0u;   // largest list
        int s0 = 0;
        for (int b = 0; b < nb; ++b) {
            const int f = d.body_first[b0 + b];
            const int e = b + 1 < nb ? d.body_first[b0 + b + 1] : n;
            const int ns = (e - f + 63) >> 6;
            float* r = bod + b * kPoolBodyFloats;
            r[kBSlot0] = __int_as_float(s0);
            r[kBSlots] = __int_as_float(ns);
            for (int j = 0; j < ns && s0 + j < max_slots; ++j)
                slot_tab[s0 + j] = make_int2(b | ((e - f - 64 * j < 64 ? e - f - 64 * j : 64) << 16), f + 64 * j);
            s0 += ns;
        }
        misc[18] = (uint32_t)s0;   // slots in use
    }
    __syncthreads();
    return (int)misc[18];
}

// Largest list length of the wave; latched with the capacity error.
__device__ inline void note_lengths(uint32_t my_max, int cap, uint32_t* misc)
{
    for (int off = 32; off > 0; off >>= 1) my_max = max(my_max, (uint32_t)__shfl_xor(my_max, off, 64));
    if ((threadIdx.x & 63) == 0 && my_max) {
        atomicMax(&misc[17], my_max);
        if (my_max > (uint32_t)cap) atomicOr(&misc[16], kErrCapacity);
    }
}

__device__ inline Ctx make_ctx(const PoolDev& d, const PoolConsts& c, const PoolScene& sc, uint32_t mask)
{
    Ctx x;
    x.d = &d;
    x.c = &c;
    x.n = sc.n;
    x.p0 = sc.p0;
    x.P = (size_t)d.P;
    for (int k = 0; k < 3; ++k) x.g[k] = sc.g[k];
    x.mu = sc.mu;
    x.avg = (c.flags >> kAvgShift) & 3u;
    x.mask = mask;
    x.cap = c.nbr_cap;
    x.lists = d.nbr + (size_t)c.nbr_cap * sc.p0;
    return x;
}

__device__ inline void latch(const PoolDev& d, int slot, const uint32_t* misc)
{
    PoolStat& st = d.stats[slot];
    if (misc[16]) st.err |= misc[16];
    if (misc[17] > st.max_nbr) st.max_nbr = misc[17];
}

// ---------------------------------------------------------------------------
// register-resident scenes
// ---------------------------------------------------------------------------

template <int S, int LB>
__global__ void __launch_bounds__(LB) k_pool(PoolDev d, PoolConsts c, int first, int subs_per_unit,
                                                              int kb, int bound)
{
    extern __shared__ float4 lds4[];
    uint32_t* lds = (uint32_t*)lds4;
    const uint32_t Tc = 1u << kb;
    uint32_t* tab = lds;                                          // [Tc + 1] key counts -> first slots
    uint32_t* sid = tab + ((Tc + 1 + 3) & ~3u);                   // [bound] id | body << 16, key-grouped
    float* part = (float*)(sid + bound);                          // [kPoolMaxSlots * kSums]
    float* bod = part + kPoolMaxSlots * kSums;                    // [64 * kPoolBodyFloats]
    int2* slot_tab = (int2*)(bod + kPoolMaxBodies * kPoolBodyFloats);   // [kPoolMaxSlots] (body, first particle)
    uint8_t* ovl = (uint8_t*)(slot_tab + kPoolMaxSlots);          // [64][64] bodies whose boxes come near
    uint32_t* ovl_n = (uint32_t*)(ovl + kPoolMaxBodies * kPoolMaxBodies);   // [64]
    uint32_t* misc = ovl_n + kPoolMaxBodies;                      // wave totals [16], flags

    const int2 job = d.order[first + blockIdx.x];                  // (slot, frames or substeps)
    const int slot = job.x;
    const PoolScene& sc = d.scenes[slot];
    const int n = sc.n, nb = sc.nb, p0 = sc.p0, b0 = sc.b0;
    const int units = job.y;
    if (units <= 0 || n <= 0) return;                              // uniform over the workgroup
    if (d.stats[slot].err & kErrDiscard) return;                   // stays at its last clean frame
    const int total_subs = units * subs_per_unit;
    const int T = blockDim.x, W = T >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    const size_t P = (size_t)d.P;
    const Ctx x = make_ctx(d, c, sc, Tc - 1u);

    const int n_slots = setup_bodies(d, b0, nb, n, bod, slot_tab, kPoolMaxSlots, misc);
    if (n_slots > W * S || n_slots > kPoolMaxSlots) {   // launch shape too small: never expected
        if (tid == 0) atomicOr(&d.stats[slot].err, kErrInternal);
        return;
    }

    // per-lane particles: register set r holds lane `lane` of slot r * W + wave
    float x0[S][3], V[S][3], del[S][3], q[S][3], m[S], Cd[S][3];
    int bdy[S], pid[S];
    uint32_t nn[S];
    bool act[S], live[S];
#pragma unroll
    for (int r = 0; r < S; ++r) {
        const int sl = r * W + wave;
        live[r] = sl < n_slots;                                   // uniform over the wave
        const int2 st = live[r] ? slot_tab[sl] : make_int2(0, 0);
        const int i = st.y + lane;
        act[r] = live[r] && lane < (st.x >> 16);
        pid[r] = act[r] ? i : 0;
        m[r] = 0.0f;
        bdy[r] = st.x & 0xffff;
        nn[r] = 0u;
        for (int k = 0; k < 3; ++k) x0[r][k] = V[r][k] = del[r][k] = q[r][k] = Cd[r][k] = 0.0f;
        if (act[r]) {
            const size_t g = (size_t)p0 + i;
            for (int k = 0; k < 3; ++k) {
                x0[r][k] = d.x[k * P + g];
                V[r][k] = d.v[k * P + g];
                q[r][k] = d.q[k * P + g];
            }
            m[r] = d.mass[g];
        }
    }

    for (int sub = 0; sub < total_subs; ++sub) {
        const bool last_sub = sub + 1 == total_subs;
        // ---- predict + key counts -------------------------------------------
        for (uint32_t k = tid; k <= Tc; k += T) tab[k] = 0u;
        if (tid < kPoolMaxBodies) ovl_n[tid] = 0u;
        __syncthreads();
        uint32_t key[S], rank[S];
        float xt[S][3];
#pragma unroll
        for (int r = 0; r < S; ++r) {
            key[r] = 0u;
            rank[r] = 0u;
            for (int k = 0; k < 3; ++k) xt[r][k] = 0.0f;
            if (!act[r]) continue;
            const int i = pid[r];
            const size_t g = (size_t)p0 + i;
            predict_one(x, x0[r], V[r], del[r], xt[r]);
            for (int k = 0; k < 3; ++k) {
                d.x0[k * P + g] = x0[r][k];      // X_init, read by neighbours
                d.dl[k * P + g] = del[r][k];
                if (last_sub) d.xt[k * P + g] = xt[r][k];
            }
            key[r] = cell_key(x, xt[r]);
            rank[r] = atomicAdd(&tab[key[r]], 1u);
            if (i == __float_as_int(bod[bdy[r] * kPoolBodyFloats + kBFirst]))   // anchor: X_init of the body's first particle
                for (int k = 0; k < 3; ++k) bod[bdy[r] * kPoolBodyFloats + kBAnchor + k] = x0[r][k];
        }
        // box of each slot's predicted positions (broad phase of the neighbour search)
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (!live[r]) continue;                                       // uniform over the wave
            float bx[6];
            for (int k = 0; k < 3; ++k) {
                bx[k] = wave_min_to_63(act[r] ? xt[r][k] : INFINITY);
                bx[3 + k] = wave_max_to_63(act[r] ? xt[r][k] : -INFINITY);
            }
            if (lane == 63)
                for (int k = 0; k < 6; ++k) part[(r * W + wave) * kSums + k] = bx[k];
        }
        __syncthreads();
        for (int b = tid; b < nb; b += T) body_box(x, bod + b * kPoolBodyFloats, part, kSums);
        scan_keys(tab, Tc, n, misc);
        __syncthreads();
        // ---- group by key, body pairs whose grown boxes overlap ----------------
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (!act[r]) continue;
            const uint32_t at = tab[key[r]] + rank[r];
            sid[at] = (uint32_t)pid[r] | ((uint32_t)bdy[r] << 16);
            d.sxt4[(size_t)p0 + at] = make_float4(xt[r][0], xt[r][1], xt[r][2], 0.0f);
        }
        for (int t = tid; t < nb * nb; t += T) {
            const int a = t / nb, b = t - a * nb;
            if (a != b && boxes_near(x, bod + a * kPoolBodyFloats, bod + b * kPoolBodyFloats))
                ovl[a * kPoolMaxBodies + atomicAdd(&ovl_n[a], 1u)] = (uint8_t)b;
        }
        __syncthreads();
        // ---- neighbour lists ---------------------------------------------------
        uint32_t my_max = 0;
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (!act[r]) continue;
            bool near = false;
            const uint32_t no = ovl_n[bdy[r]];
            for (uint32_t j = 0; j < no && !near; ++j)
                near = point_near(x, xt[r], bod + ovl[bdy[r] * kPoolMaxBodies + j] * kPoolBodyFloats);
            const uint32_t cnt = near ? walk(x, tab, sid, d.sxt4 + p0, pid[r], bdy[r], xt[r]) : 0u;
            nn[r] = cnt;
            d.nbr_n[(size_t)p0 + pid[r]] = cnt;
            my_max = cnt > my_max ? cnt : my_max;
        }
        note_lengths(my_max, x.cap, misc);
        __syncthreads();   // lists, counts, X_init and delta_0 visible to the workgroup

        // ---- K Jacobi iterations ---------------------------------------------
        for (int it = 0; it < c.iterations; ++it) {
            // contacts from X_i and the shape-matching sums
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (act[r]) {
                    contacts(x, pid[r], x0[r], del[r], m[r], nn[r], Cd[r]);
                } else {
                    for (int k = 0; k < 3; ++k) Cd[r][k] = 0.0f;
                }
                if (live[r]) {
                    float Sv[12];
                    sm_terms(act[r], bod + bdy[r] * kPoolBodyFloats, x0[r], del[r], q[r], m[r], Sv);
                    wave_store<3>(Sv, part + (r * W + wave) * kSums, lane);
                }
            }
            __syncthreads();
            for (int b = tid; b < nb; b += T) body_rotation(bod + b * kPoolBodyFloats, part, it);
            __syncthreads();
            // goal offsets and the momentum sums
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (!live[r]) continue;
                float Sv[24];
                mom_terms(x, act[r], bod + bdy[r] * kPoolBodyFloats, x0[r], del[r], q[r], V[r], Cd[r], m[r], Sv);
                wave_store<6>(Sv, part + (r * W + wave) * kSums, lane);
            }
            __syncthreads();
            for (int b = tid; b < nb; b += T) body_momentum(c, bod + b * kPoolBodyFloats, part);
            __syncthreads();
            // particle update: X_{i+1}, V_{i+1}
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (!act[r]) continue;
                update_one(c, bod + bdy[r] * kPoolBodyFloats, x0[r], q[r], Cd[r], del[r], V[r]);
                for (int k = 0; k < 3; ++k) d.dl[k * P + (size_t)p0 + pid[r]] = del[r][k];
            }
            __syncthreads();   // X_{i+1} visible to neighbours before the next iteration
        }
        // ---- end of substep: X_K, V_K become the state ---------------------------
        bool finite = true;
#pragma unroll
        for (int r = 0; r < S; ++r) {
            if (!act[r]) continue;
            for (int k = 0; k < 3; ++k) {
                x0[r][k] = x0[r][k] + del[r][k];
                finite = finite && isfinite(x0[r][k]) && isfinite(V[r][k]);
            }
        }
        if (!finite) atomicOr(&misc[16], kErrNonFinite);
        // ---- end of a unit (a frame, or a substep of pbdr_pool_substep): the
        // state is committed only if the scene has latched no error, so after
        // one it keeps the last unit completed without it
        if ((sub + 1) % subs_per_unit == 0) {
            __syncthreads();
            if (misc[16]) break;                                   // uniform: read after the barrier
#pragma unroll
            for (int r = 0; r < S; ++r) {
                if (!act[r]) continue;
                const size_t g = (size_t)p0 + pid[r];
                for (int k = 0; k < 3; ++k) {
                    d.x[k * P + g] = x0[r][k];
                    d.v[k * P + g] = V[r][k];
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) latch(d, slot, misc);
}

// ---------------------------------------------------------------------------
// large scenes: state in global memory, 16 waves walking the slots
// ---------------------------------------------------------------------------

constexpr int kBigWaves = 16;
constexpr int kBigWords = kPoolBigMaxBodies / 32;

__device__ inline void load3(const float* a, size_t P, size_t g, float* o)
{
    for (int k = 0; k < 3; ++k) o[k] = a[k * P + g];
}

__device__ inline void store3(float* a, size_t P, size_t g, const float* o)
{
    for (int k = 0; k < 3; ++k) a[k * P + g] = o[k];
}

__global__ void __launch_bounds__(64 * kBigWaves) k_pool_big(PoolDev d, PoolConsts c, int first, int subs_per_unit)
{
    extern __shared__ float4 lds4[];
    uint32_t* lds = (uint32_t*)lds4;
    constexpr uint32_t Tc = 1u << kPoolBigKeyBits;
    uint32_t* tab = lds;                                               // [Tc + 1]
    float* bod = (float*)(tab + ((Tc + 1 + 3) & ~3u));                 // [256 * kPoolBodyFloats]
    int2* slot_tab = (int2*)(bod + kPoolBigMaxBodies * kPoolBodyFloats);   // [kPoolBigMaxSlots]
    uint32_t* ovl = (uint32_t*)(slot_tab + kPoolBigMaxSlots);          // [256][8] bit sets of near bodies
    uint32_t* misc = ovl + kPoolBigMaxBodies * kBigWords;              // wave totals [16], flags

    const int2 job = d.order[first + blockIdx.x];                       // (slot, frames or substeps)
    const int slot = job.x;
    const PoolScene& sc = d.scenes[slot];
    const int n = sc.n, nb = sc.nb, p0 = sc.p0, b0 = sc.b0;
    const int units = job.y;
    if (units <= 0 || n <= 0) return;                                   // uniform over the workgroup
    if (d.stats[slot].err & kErrDiscard) return;                        // stays at its last clean frame
    const int total_subs = units * subs_per_unit;
    const int T = blockDim.x, W = T >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    const size_t P = (size_t)d.P;
    const Ctx x = make_ctx(d, c, sc, Tc - 1u);
    float* part = d.part + (size_t)sc.s_base * kSums;                  // [n_slots * kSums] slot sums and boxes
    uint32_t* sidg = d.sid + p0;                                       // [n] key-grouped entries
    uint32_t* rankg = d.rank + p0;                                     // [n] slot within the key
    float* velg = d.vel;                                               // [3][P] V_i during a substep
    float* cdg = d.cd;                                                 // [3][P] contact displacement of the iteration

    const int n_slots = setup_bodies(d, b0, nb, n, bod, slot_tab, kPoolBigMaxSlots, misc);
    if (n_slots > kPoolBigMaxSlots || nb > kPoolBigMaxBodies) {        // rejected by the host: never expected
        if (tid == 0) atomicOr(&d.stats[slot].err, kErrInternal);
        return;
    }

    for (int sub = 0; sub < total_subs; ++sub) {
        for (uint32_t k = tid; k <= Tc; k += T) tab[k] = 0u;
        for (int k = tid; k < nb * kBigWords; k += T) ovl[k] = 0u;
        __syncthreads();
        // ---- predict + key counts + slot boxes --------------------------------
        for (int s = wave; s < n_slots; s += W) {
            const int2 st = slot_tab[s];
            const int i = st.y + lane, b = st.x & 0xffff;
            const bool act = lane < (st.x >> 16);
            float xt[3] = {0.0f, 0.0f, 0.0f};
            if (act) {
                const size_t g = (size_t)p0 + i;
                float x0[3], V[3], del[3];
                if (sub % subs_per_unit == 0) {        // first substep of a unit: the committed state
                    load3(d.x, P, g, x0);
                    load3(d.v, P, g, V);
                } else {                               // X_K, V_K of the previous substep
                    load3(d.x0, P, g, x0);
                    load3(velg, P, g, V);
                }
                predict_one(x, x0, V, del, xt);
                store3(d.x0, P, g, x0);
                store3(d.dl, P, g, del);
                store3(velg, P, g, V);
                store3(d.xt, P, g, xt);
                rankg[i] = atomicAdd(&tab[cell_key(x, xt)], 1u);
                if (i == __float_as_int(bod[b * kPoolBodyFloats + kBFirst]))
                    for (int k = 0; k < 3; ++k) bod[b * kPoolBodyFloats + kBAnchor + k] = x0[k];
            }
            float bx[6];
            for (int k = 0; k < 3; ++k) {
                bx[k] = wave_min_to_63(act ? xt[k] : INFINITY);
                bx[3 + k] = wave_max_to_63(act ? xt[k] : -INFINITY);
            }
            if (lane == 63)
                for (int k = 0; k < 6; ++k) part[s * kSums + k] = bx[k];
        }
        __syncthreads();
        for (int b = tid; b < nb; b += T) body_box(x, bod + b * kPoolBodyFloats, part, kSums);
        scan_keys(tab, Tc, n, misc);
        __syncthreads();
        // ---- group by key, body pairs whose grown boxes overlap ----------------
        for (int s = wave; s < n_slots; s += W) {
            const int2 st = slot_tab[s];
            const int i = st.y + lane, b = st.x & 0xffff;
            if (lane >= (st.x >> 16)) continue;
            const size_t g = (size_t)p0 + i;
            float xt[3];
            load3(d.xt, P, g, xt);
            const uint32_t at = tab[cell_key(x, xt)] + rankg[i];
            sidg[at] = (uint32_t)i | ((uint32_t)b << 16);
            d.sxt4[(size_t)p0 + at] = make_float4(xt[0], xt[1], xt[2], 0.0f);
        }
        for (int t = tid; t < nb * nb; t += T) {
            const int a = t / nb, b = t - a * nb;
            if (a != b && boxes_near(x, bod + a * kPoolBodyFloats, bod + b * kPoolBodyFloats))
                atomicOr(&ovl[a * kBigWords + (b >> 5)], 1u << (b & 31));
        }
        __syncthreads();
        // ---- neighbour lists ---------------------------------------------------
        uint32_t my_max = 0;
        for (int s = wave; s < n_slots; s += W) {
            const int2 st = slot_tab[s];
            const int i = st.y + lane, b = st.x & 0xffff;
            if (lane >= (st.x >> 16)) continue;
            const size_t g = (size_t)p0 + i;
            float xt[3];
            load3(d.xt, P, g, xt);
            bool near = false;
            for (int w = 0; w < kBigWords && !near; ++w) {
                uint32_t bits = ovl[b * kBigWords + w];
                while (bits && !near) {
                    const int j = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    near = point_near(x, xt, bod + (32 * w + j) * kPoolBodyFloats);
                }
            }
            const uint32_t cnt = near ? walk(x, tab, sidg, d.sxt4 + p0, i, b, xt) : 0u;
            d.nbr_n[g] = cnt;
            my_max = cnt > my_max ? cnt : my_max;
        }
        note_lengths(my_max, x.cap, misc);
        __syncthreads();

        // ---- K Jacobi iterations ---------------------------------------------
        for (int it = 0; it < c.iterations; ++it) {
            for (int s = wave; s < n_slots; s += W) {
                const int2 st = slot_tab[s];
                const int i = st.y + lane, b = st.x & 0xffff;
                const bool act = lane < (st.x >> 16);
                float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, q[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f;
                if (act) {
                    const size_t g = (size_t)p0 + i;
                    float Cd[3];
                    load3(d.x0, P, g, x0);
                    load3(d.dl, P, g, del);
                    load3(d.q, P, g, q);
                    m = d.mass[g];
                    contacts(x, i, x0, del, m, d.nbr_n[g], Cd);
                    store3(cdg, P, g, Cd);
                }
                float Sv[12];
                sm_terms(act, bod + b * kPoolBodyFloats, x0, del, q, m, Sv);
                wave_store<3>(Sv, part + s * kSums, lane);
            }
            __syncthreads();
            for (int b = tid; b < nb; b += T) body_rotation(bod + b * kPoolBodyFloats, part, it);
            __syncthreads();
            for (int s = wave; s < n_slots; s += W) {
                const int2 st = slot_tab[s];
                const int i = st.y + lane, b = st.x & 0xffff;
                const bool act = lane < (st.x >> 16);
                float x0[3] = {0.0f, 0.0f, 0.0f}, del[3] = {0.0f, 0.0f, 0.0f}, q[3] = {0.0f, 0.0f, 0.0f},
                      V[3] = {0.0f, 0.0f, 0.0f}, Cd[3] = {0.0f, 0.0f, 0.0f}, m = 0.0f;
                if (act) {
                    const size_t g = (size_t)p0 + i;
                    load3(d.x0, P, g, x0);
                    load3(d.dl, P, g, del);
                    load3(d.q, P, g, q);
                    load3(velg, P, g, V);
                    load3(cdg, P, g, Cd);
                    m = d.mass[g];
                }
                float Sv[24];
                mom_terms(x, act, bod + b * kPoolBodyFloats, x0, del, q, V, Cd, m, Sv);
                wave_store<6>(Sv, part + s * kSums, lane);
            }
            __syncthreads();
            for (int b = tid; b < nb; b += T) body_momentum(c, bod + b * kPoolBodyFloats, part);
            __syncthreads();
            for (int s = wave; s < n_slots; s += W) {
                const int2 st = slot_tab[s];
                const int i = st.y + lane, b = st.x & 0xffff;
                if (lane >= (st.x >> 16)) continue;
                const size_t g = (size_t)p0 + i;
                float x0[3], del[3], q[3], V[3], Cd[3];
                load3(d.x0, P, g, x0);
                load3(d.dl, P, g, del);
                load3(d.q, P, g, q);
                load3(velg, P, g, V);
                load3(cdg, P, g, Cd);
                update_one(c, bod + b * kPoolBodyFloats, x0, q, Cd, del, V);
                store3(d.dl, P, g, del);
                store3(velg, P, g, V);
            }
            __syncthreads();
        }
        // ---- end of substep: X_K (into the X_init buffer) and V_K ---------------
        bool finite = true;
        for (int s = wave; s < n_slots; s += W) {
            const int2 st = slot_tab[s];
            const int i = st.y + lane;
            if (lane >= (st.x >> 16)) continue;
            const size_t g = (size_t)p0 + i;
            float x0[3], del[3], V[3];
            load3(d.x0, P, g, x0);
            load3(d.dl, P, g, del);
            load3(velg, P, g, V);
            for (int k = 0; k < 3; ++k) {
                x0[k] = x0[k] + del[k];
                finite = finite && isfinite(x0[k]) && isfinite(V[k]);
            }
            store3(d.x0, P, g, x0);
        }
        if (!finite) atomicOr(&misc[16], kErrNonFinite);
        __syncthreads();
        // ---- end of a unit: committed only without a latched error ---------------
        if ((sub + 1) % subs_per_unit == 0) {
            if (misc[16]) break;                                   // uniform: read after the barrier
            for (int s = wave; s < n_slots; s += W) {
                const int2 st = slot_tab[s];
                if (lane >= (st.x >> 16)) continue;
                const size_t g = (size_t)p0 + st.y + lane;
                float x0[3], V[3];
                load3(d.x0, P, g, x0);
                load3(velg, P, g, V);
                store3(d.x, P, g, x0);
                store3(d.v, P, g, V);
            }
        }
    }
    if (tid == 0) latch(d, slot, misc);
}

}  // namespace

size_t pool_lds_bytes(int cls)
{
    if (cls == kPoolBigClass) {
        const size_t Tc = (size_t)1 << kPoolBigKeyBits;
        return 4 * ((Tc + 1 + 3) & ~(size_t)3) + 4 * kPoolBigMaxBodies * kPoolBodyFloats + 8 * kPoolBigMaxSlots +
               4 * kPoolBigMaxBodies * kBigWords + 4 * 32;
    }
    const size_t bound = (size_t)pool_class_bound(cls);
    const size_t Tc = (size_t)1 << pool_class_key_bits(cls);
    return 4 * ((Tc + 1 + 3) & ~(size_t)3) + 4 * bound + 4 * kPoolMaxSlots * kSums +
           4 * kPoolMaxBodies * kPoolBodyFloats + 8 * kPoolMaxSlots + kPoolMaxBodies * kPoolMaxBodies +
           4 * kPoolMaxBodies + 4 * 32;
}

hipError_t pool_prepare(size_t max_lds)
{
    hipError_t e = hipSuccess;
#define PBDR_POOL_ATTR(S_, LB_)                                                                              \
    if (e == hipSuccess)                                                                                     \
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pool<S_, LB_>),                             \
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
#define PBDR_POOL_ATTRS(S_) PBDR_POOL_ATTR(S_, 256) PBDR_POOL_ATTR(S_, 512) PBDR_POOL_ATTR(S_, 1024)
    PBDR_POOL_ATTRS(1)
    PBDR_POOL_ATTRS(2)
    PBDR_POOL_ATTRS(3)
    PBDR_POOL_ATTRS(4)
    PBDR_POOL_ATTRS(5)
    PBDR_POOL_ATTRS(6)
    PBDR_POOL_ATTRS(8)
#undef PBDR_POOL_ATTRS
#undef PBDR_POOL_ATTR
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pool_big), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)max_lds);
    return e;
}

hipError_t enqueue_pool_class(const PoolDev& d, const PoolConsts& c, int cls, int waves, int slots, int first,
                              int count, int subs_per_unit, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    const size_t lds = pool_lds_bytes(cls);
    const dim3 grid((unsigned)count);
    if (cls == kPoolBigClass) {
        hipLaunchKernelGGL(k_pool_big, grid, dim3(64 * kBigWaves), lds, stream, d, c, first, subs_per_unit);
        return hipGetLastError();
    }
    const int kb = pool_class_key_bits(cls), bound = pool_class_bound(cls);
    const dim3 block((unsigned)(64 * waves));
    const int lb = waves <= 4 ? 256 : (waves <= 8 ? 512 : 1024);
#define PBDR_POOL_CASE(S_, LB_)                                                                                  \
    if (slots == S_ && lb == LB_) {                                                                              \
        hipLaunchKernelGGL((k_pool<S_, LB_>), grid, block, lds, stream, d, c, first, subs_per_unit, kb, bound); \
        return hipGetLastError();                                                                                \
    }
#define PBDR_POOL_SLOTS(S_) PBDR_POOL_CASE(S_, 256) PBDR_POOL_CASE(S_, 512) PBDR_POOL_CASE(S_, 1024)
    PBDR_POOL_SLOTS(1)
    PBDR_POOL_SLOTS(2)
    PBDR_POOL_SLOTS(3)
    PBDR_POOL_SLOTS(4)
    PBDR_POOL_SLOTS(5)
    PBDR_POOL_SLOTS(6)
    PBDR_POOL_SLOTS(8)
#undef PBDR_POOL_SLOTS
#undef PBDR_POOL_CASE
    return hipErrorInvalidValue;
}

}  // namespace pbdr
