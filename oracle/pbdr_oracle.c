/*
 * FP64 CPU reference ("oracle") for the PBD-R solver substep of
 * "Physically Accurate Rigid-Body Dynamics in Particle-Based Simulation"
 * (arXiv 2603.14634).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the GPU library.
 *
 * It is written to be read against the paper: plain loops, FP64, no blocking
 * or fusion, per-body sums in ascending particle order.  Each function names
 * the passage it follows.  Where the paper is silent, the reading taken is
 * stated at the function.  Build with -O2 -ffp-contract=off (no FMA
 * contraction anywhere, so the FP32 indexing recipe is evaluated op by op).
 */
#include "pbdr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define X_(a, n, i) ((a)[(i)])
#define Y_(a, n, i) ((a)[(size_t)(n) + (i)])
#define Z_(a, n, i) ((a)[2 * (size_t)(n) + (i)])

static int threads_of(const orc_params* p) { return p->n_threads > 1 ? p->n_threads : 1; }

/* ------------------------------------------------------------------------ */
/* small 3-vector / 3x3 helpers                                              */
/* ------------------------------------------------------------------------ */

static void cross3(const double* a, const double* b, double* out)
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------------ */
/* Rest pose: shape matching needs, per body, the rest configuration measured */
/* from the rest centre of mass (Sec. III-C; Mueller et al. 2005).  Reading:  */
/* the rest pose is the configuration at creation; masses weight the centre. */
/* ------------------------------------------------------------------------ */
void orc_rest_pose(int32_t n, int32_t nb, const int32_t* body_start, const double* mass,
                   const double* x0, double* q_out, double* body_mass_out)
{
    for (int32_t b = 0; b < nb; ++b) {
        double M = 0.0, c[3] = {0.0, 0.0, 0.0};
        for (int32_t i = body_start[b]; i < body_start[b + 1]; ++i) {
            M += mass[i];
            c[0] += mass[i] * X_(x0, n, i);
            c[1] += mass[i] * Y_(x0, n, i);
            c[2] += mass[i] * Z_(x0, n, i);
        }
        c[0] /= M; c[1] /= M; c[2] /= M;
        body_mass_out[b] = M;
        for (int32_t i = body_start[b]; i < body_start[b + 1]; ++i) {
            X_(q_out, n, i) = X_(x0, n, i) - c[0];
            Y_(q_out, n, i) = Y_(x0, n, i) - c[1];
            Z_(q_out, n, i) = Z_(x0, n, i) - c[2];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour search.  The paper's particle-particle contact (Sec. III-A,      */
/* constraint (2); Alg. 1 ParticleParticleContact) acts between particles of  */
/* different object groups but gives no search method.  Reading: a uniform   */
/* hash grid over FP32 predicted positions, whose every decision is taken in  */
/* FP32 (the paper's machine precision, Sec. IV-B "Implementation details"):  */
/*                                                                            */
/*   predicted position   a = g + accel;  vt = v + h*a;  xt = x + h*vt        */
/*   cell coordinate      c = floor((xt - o) * inv_a), clamped to +-2^24,     */
/*                        wrapped to 10 bits                                  */
/*   key                  3D Morton interleave of the wrapped coordinates,    */
/*                        low k bits                                          */
/*   predicate            q != p, body(q) != body(p),                         */
/*                        ((dx*dx + dy*dy) + dz*dz) < fl32(R_s^2),            */
/*                        dx = xt_q - xt_p                                    */
/*                                                                            */
/* Every line above is one rounded FP32 operation.  The neighbour list of p  */
/* is the ascending list of all q satisfying the predicate; the grid only     */
/* finds them (cell edge a >= R_s, 27-cell stencil).                          */
/* ------------------------------------------------------------------------ */
void orc_predict32(int32_t n, const orc_params* p, const float* x, const float* v,
                   const float* accel, float* xt_out)
{
    const float h32 = (float)p->h;
    for (int32_t k = 0; k < 3; ++k) {
        const float g32 = (float)p->gravity[k];
        for (int32_t i = 0; i < n; ++i) {
            const size_t j = (size_t)k * (size_t)n + (size_t)i;
            const float a = g32 + (accel ? accel[j] : 0.0f);
            const float dv = h32 * a;
            const float vt = v[j] + dv;
            const float dx = h32 * vt;
            xt_out[j] = x[j] + dx;
        }
    }
}

static uint32_t cell_axis(float xt, float o, float inv_a)
{
    const float t = xt - o;
    const float u = t * inv_a;
    float f = floorf(u);
    if (!(f >= -16777216.0f)) f = -16777216.0f;
    if (!(f <= 16777216.0f)) f = 16777216.0f;
    return ((uint32_t)(int32_t)f) & 1023u;
}

static uint32_t spread_bits(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

static uint32_t morton_key(uint32_t cx, uint32_t cy, uint32_t cz, uint32_t mask)
{
    return (spread_bits(cx & 1023u) | (spread_bits(cy & 1023u) << 1) | (spread_bits(cz & 1023u) << 2)) & mask;
}

typedef struct { float o[3]; float inv_a; float r2; uint32_t mask; } grid32;

static grid32 grid_of(const orc_params* p)
{
    grid32 g;
    for (int k = 0; k < 3; ++k) g.o[k] = (float)p->grid_origin[k];
    g.inv_a = (float)(1.0 / p->cell_size);
    g.r2 = (float)(p->search_radius * p->search_radius);
    g.mask = (p->hash_bits >= 32) ? 0xffffffffu : ((1u << p->hash_bits) - 1u);
    return g;
}

void orc_cell_keys(int32_t n, const orc_params* p, const float* xt, uint32_t* key_out)
{
    const grid32 g = grid_of(p);
    for (int32_t i = 0; i < n; ++i) {
        uint32_t cx = cell_axis(X_(xt, n, i), g.o[0], g.inv_a);
        uint32_t cy = cell_axis(Y_(xt, n, i), g.o[1], g.inv_a);
        uint32_t cz = cell_axis(Z_(xt, n, i), g.o[2], g.inv_a);
        key_out[i] = morton_key(cx, cy, cz, g.mask);
    }
}

static int pair_in_range(const float* xt, int32_t n, int32_t i, int32_t j, float r2)
{
    const float dx = X_(xt, n, j) - X_(xt, n, i);
    const float dy = Y_(xt, n, j) - Y_(xt, n, i);
    const float dz = Z_(xt, n, j) - Z_(xt, n, i);
    const float sx = dx * dx;
    const float sy = dy * dy;
    const float sz = dz * dz;
    const float s = (sx + sy) + sz;
    return s < r2;
}

static int cmp_u32(const void* a, const void* b)
{
    const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

/* Builds the sorted order, cell tables and CSR neighbour lists (no cap). */
static int32_t build_index(int32_t n, const orc_params* p, const int32_t* body, const float* xt,
                           uint32_t* key, uint32_t* sorted_id, uint32_t* cell_start,
                           uint32_t* cell_count, uint32_t** nbr_off_out, uint32_t** nbr_flat_out)
{
    const grid32 g = grid_of(p);
    const size_t T = (size_t)g.mask + 1u;
    orc_cell_keys(n, p, xt, key);
    /* stable counting sort by key: ties keep ascending particle id */
    memset(cell_count, 0, T * sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) cell_count[key[i]] += 1u;
    uint32_t run = 0;
    for (size_t t = 0; t < T; ++t) { cell_start[t] = run; run += cell_count[t]; }
    uint32_t* fill = (uint32_t*)calloc(T, sizeof(uint32_t));
    for (int32_t i = 0; i < n; ++i) {
        sorted_id[cell_start[key[i]] + fill[key[i]]] = (uint32_t)i;
        fill[key[i]] += 1u;
    }
    free(fill);
    /* neighbour lists: 27-cell stencil, predicate, ascending order */
    uint32_t* cnt = (uint32_t*)calloc((size_t)n + 1u, sizeof(uint32_t));
    int nthr = threads_of(p);
    (void)nthr;
    for (int pass = 0; pass < 2; ++pass) {
        uint32_t* off = (pass == 1) ? *nbr_off_out : NULL;
        uint32_t* flat = (pass == 1) ? *nbr_flat_out : NULL;
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthr)
        for (int32_t i = 0; i < n; ++i) {
            const uint32_t cx = cell_axis(X_(xt, n, i), g.o[0], g.inv_a);
            const uint32_t cy = cell_axis(Y_(xt, n, i), g.o[1], g.inv_a);
            const uint32_t cz = cell_axis(Z_(xt, n, i), g.o[2], g.inv_a);
            uint32_t c = 0;
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const uint32_t k = morton_key(cx + (uint32_t)dx, cy + (uint32_t)dy,
                                                      cz + (uint32_t)dz, g.mask);
                        for (uint32_t s = cell_start[k]; s < cell_start[k] + cell_count[k]; ++s) {
                            const int32_t j = (int32_t)sorted_id[s];
                            if (j == i || body[j] == body[i]) continue;
                            if (!pair_in_range(xt, n, i, j, g.r2)) continue;
                            if (pass == 1) flat[off[i] + c] = (uint32_t)j;
                            ++c;
                        }
                    }
            if (pass == 0) cnt[i] = c;
            else qsort(flat + off[i], c, sizeof(uint32_t), cmp_u32);
        }
        if (pass == 0) {
            uint32_t* o = (uint32_t*)malloc(((size_t)n + 1u) * sizeof(uint32_t));
            o[0] = 0;
            for (int32_t i = 0; i < n; ++i) o[i + 1] = o[i] + cnt[i];
            *nbr_off_out = o;
            *nbr_flat_out = (uint32_t*)malloc(((size_t)o[n] + 1u) * sizeof(uint32_t));
        }
    }
    int32_t mx = 0;
    for (int32_t i = 0; i < n; ++i) if ((int32_t)cnt[i] > mx) mx = (int32_t)cnt[i];
    free(cnt);
    return mx;
}

int32_t orc_index(int32_t n, const orc_params* p, const int32_t* body, const float* xt,
                  uint32_t* key, uint32_t* sorted_id, uint32_t* cell_start,
                  uint32_t* cell_count, uint32_t* nbr_count, uint32_t* nbr)
{
    uint32_t *off = NULL, *flat = NULL;
    int32_t mx = build_index(n, p, body, xt, key, sorted_id, cell_start, cell_count, &off, &flat);
    for (int32_t i = 0; i < n; ++i) {
        const uint32_t c = off[i + 1] - off[i];
        nbr_count[i] = c;
        for (uint32_t s = 0; s < c && (int32_t)s < p->nbr_cap; ++s)
            nbr[(size_t)i * (size_t)p->nbr_cap + s] = flat[off[i] + s];
    }
    free(off);
    free(flat);
    return mx;
}

/* ------------------------------------------------------------------------ */
/* Polar decomposition for shape matching (Sec. III-C; Mueller et al. 2005): */
/* the goal positions use the rotation of the least-squares optimal rigid    */
/* transform from the rest pose.  Its plain definition: the R in SO(3) that  */
/* maximises tr(R^T A).  Computed from an SVD A = U S V^T obtained by        */
/* one-sided (Hestenes) Jacobi rotations: with singular values sorted        */
/* descending and U, V made proper (det +1) by completing u3 = u1 x u2 and   */
/* flipping v3 when needed, R = U V^T (the sign of the smallest singular     */
/* value absorbs any reflection).                                            */
/* ------------------------------------------------------------------------ */
void orc_polar(const double* A, double* R)
{
    double B[3][3], V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[r][c] = A[3 * r + c];
    static const int PI[3] = {0, 0, 1}, PJ[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 100; ++sweep) {
        double worst = 0.0;
        for (int pr = 0; pr < 3; ++pr) {
            const int i = PI[pr], j = PJ[pr];
            double al = 0.0, be = 0.0, ga = 0.0;
            for (int k = 0; k < 3; ++k) {
                al += B[k][i] * B[k][i];
                be += B[k][j] * B[k][j];
                ga += B[k][i] * B[k][j];
            }
            if (ga == 0.0) continue;
            const double rel = fabs(ga) / sqrt(al * be);
            if (rel > worst) worst = rel;
            if (rel < 1e-16) continue;
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int k = 0; k < 3; ++k) {
                const double bi = B[k][i], bj = B[k][j];
                B[k][i] = c * bi - s * bj;
                B[k][j] = s * bi + c * bj;
                const double vi = V[k][i], vj = V[k][j];
                V[k][i] = c * vi - s * vj;
                V[k][j] = s * vi + c * vj;
            }
        }
        if (worst < 1e-15) break;
    }
    double sig[3];
    int ord[3] = {0, 1, 2};
    for (int j = 0; j < 3; ++j) sig[j] = sqrt(B[0][j] * B[0][j] + B[1][j] * B[1][j] + B[2][j] * B[2][j]);
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (sig[ord[b]] > sig[ord[a]]) { int t = ord[a]; ord[a] = ord[b]; ord[b] = t; }
    double u1[3], u2[3], u3[3], v1[3], v2[3], v3[3];
    for (int k = 0; k < 3; ++k) {
        v1[k] = V[k][ord[0]];
        v2[k] = V[k][ord[1]];
        v3[k] = V[k][ord[2]];
    }
    if (sig[ord[0]] == 0.0) {  /* A = 0: every rotation is optimal; take I */
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    for (int k = 0; k < 3; ++k) u1[k] = B[k][ord[0]] / sig[ord[0]];
    if (sig[ord[1]] > 1e-12 * sig[ord[0]]) {
        for (int k = 0; k < 3; ++k) u2[k] = B[k][ord[1]] / sig[ord[1]];
    } else {  /* rank 1: any unit vector orthogonal to u1 */
        const double e[3] = {fabs(u1[0]) < 0.9 ? 1.0 : 0.0, fabs(u1[0]) < 0.9 ? 0.0 : 1.0, 0.0};
        cross3(u1, e, u2);
    }
    const double d12 = dot3(u1, u2);
    for (int k = 0; k < 3; ++k) u2[k] -= d12 * u1[k];
    const double n2 = norm3(u2);
    for (int k = 0; k < 3; ++k) u2[k] /= n2;
    cross3(u1, u2, u3);
    double vc[3];
    cross3(v1, v2, vc);
    if (dot3(vc, v3) < 0.0)
        for (int k = 0; k < 3; ++k) v3[k] = -v3[k];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[3 * r + c] = u1[r] * v1[c] + u2[r] * v2[c] + u3[r] * v3[c];
}

/* ------------------------------------------------------------------------ */
/* Symmetric 3x3 pseudo-inverse by the cyclic Jacobi eigenvalue method.      */
/* Used for omega = I^-1 dL (Sec. III-C, angular momentum correction).       */
/* Reading: a body whose inertia tensor is singular (one particle, or all    */
/* particles on a line) gets the pseudo-inverse: eigenvalues at or below     */
/* `cutoff` are dropped.  The caller takes the cutoff relative to the body's */
/* own scale (see momentum_body), because the inertia tensor of a            */
/* one-particle body is rounding noise, not zero.                            */
/* ------------------------------------------------------------------------ */
void orc_pinv_sym3(const double* S, double cutoff, double* out)
{
    double a[3][3], Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) a[r][c] = 0.5 * (S[3 * r + c] + S[3 * c + r]);
    const double tr = a[0][0] + a[1][1] + a[2][2];
    for (int k = 0; k < 9; ++k) out[k] = 0.0;
    if (!(tr > 0.0)) return;
    static const int PI[3] = {0, 0, 1}, PJ[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off <= 1e-300 || off <= 1e-17 * tr) break;
        for (int pr = 0; pr < 3; ++pr) {
            const int p = PI[pr], q = PJ[pr];
            if (a[p][q] == 0.0) continue;
            const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
            J[p][p] = c; J[q][q] = c; J[p][q] = s; J[q][p] = -s;
            double T1[3][3], T2[3][3], Qn[3][3];
            for (int r = 0; r < 3; ++r)          /* T1 = A J */
                for (int cc = 0; cc < 3; ++cc) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += a[r][k] * J[k][cc];
                    T1[r][cc] = acc;
                }
            for (int r = 0; r < 3; ++r)          /* T2 = J^T A J */
                for (int cc = 0; cc < 3; ++cc) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += J[k][r] * T1[k][cc];
                    T2[r][cc] = acc;
                }
            for (int r = 0; r < 3; ++r)          /* Q = Q J */
                for (int cc = 0; cc < 3; ++cc) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += Q[r][k] * J[k][cc];
                    Qn[r][cc] = acc;
                }
            memcpy(a, T2, sizeof(a));
            memcpy(Q, Qn, sizeof(Q));
            a[p][q] = a[q][p] = 0.0;
        }
    }
    for (int k = 0; k < 3; ++k) {
        const double lam = a[k][k];
        if (!(lam > cutoff)) continue;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) out[3 * r + c] += Q[r][k] * Q[c][k] / lam;
    }
}

/* ------------------------------------------------------------------------ */
/* Momentum conservation constraint (Sec. III-C, Eqs. (4)-(5)).              */
/* For one body: P = sum m v, L = sum (x - x_com) x m v, x_com = sum m x / M, */
/* each state about its own centre of mass.  dv = (P_bsm - P_asm)/M;         */
/* omega = I^-1 (L_asm - L_bsm) with I = sum m (|r|^2 I3 - r r^T),           */
/* r = x_asm - x_com(asm).  Both corrections are applied together:           */
/*   v = v_asm + dv - omega x r,   x = x_asm + (dv - omega x r) dt.          */
/* Arrays are SoA with stride `stride`, particles s .. e-1.                  */
/* ------------------------------------------------------------------------ */
static void momentum_body(int32_t s, int32_t e, int32_t stride, const double* mass,
                          const double* xb, const double* vb, const double* xa, const double* va,
                          double h, double radius, uint32_t flags, double* xo, double* vo)
{
    const size_t n = (size_t)stride;
    double M = 0.0, cb[3] = {0, 0, 0}, ca[3] = {0, 0, 0}, Pb[3] = {0, 0, 0}, Pa[3] = {0, 0, 0};
    for (int32_t i = s; i < e; ++i) {
        const double m = mass[i];
        M += m;
        for (int k = 0; k < 3; ++k) {
            cb[k] += m * xb[k * n + i];
            ca[k] += m * xa[k * n + i];
            Pb[k] += m * vb[k * n + i];
            Pa[k] += m * va[k * n + i];
        }
    }
    for (int k = 0; k < 3; ++k) { cb[k] /= M; ca[k] /= M; }
    double Lb[3] = {0, 0, 0}, La[3] = {0, 0, 0}, I[9] = {0};
    for (int32_t i = s; i < e; ++i) {
        const double m = mass[i];
        double rb[3], ra[3], vbi[3], vai[3], t[3];
        for (int k = 0; k < 3; ++k) {
            rb[k] = xb[k * n + i] - cb[k];
            ra[k] = xa[k * n + i] - ca[k];
            vbi[k] = vb[k * n + i];
            vai[k] = va[k * n + i];
        }
        cross3(rb, vbi, t);
        for (int k = 0; k < 3; ++k) Lb[k] += m * t[k];
        cross3(ra, vai, t);
        for (int k = 0; k < 3; ++k) La[k] += m * t[k];
        const double rr = dot3(ra, ra);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) I[3 * r + c] += m * ((r == c ? rr : 0.0) - ra[r] * ra[c]);
    }
    double dv[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    if (!(flags & ORC_NO_LIN_MOM))
        for (int k = 0; k < 3; ++k) dv[k] = (Pb[k] - Pa[k]) / M;
    if (!(flags & ORC_NO_ANG_MOM)) {
        /* pseudo-inverse cutoff: 1e-12 of max(trace I, M (2r)^2), so that a
           one-particle body (inertia = rounding noise) gets no angular step */
        double Ip[9], dL[3];
        for (int k = 0; k < 3; ++k) dL[k] = La[k] - Lb[k];
        const double scale = fmax(I[0] + I[4] + I[8], M * 4.0 * radius * radius);
        orc_pinv_sym3(I, 1e-12 * scale, Ip);
        for (int r = 0; r < 3; ++r) w[r] = Ip[3 * r] * dL[0] + Ip[3 * r + 1] * dL[1] + Ip[3 * r + 2] * dL[2];
    }
    for (int32_t i = s; i < e; ++i) {
        double ra[3], wr[3];
        for (int k = 0; k < 3; ++k) ra[k] = xa[k * n + i] - ca[k];
        cross3(w, ra, wr);
        for (int k = 0; k < 3; ++k) {
            const double dvi = dv[k] - wr[k];
            vo[k * n + i] = va[k * n + i] + dvi;
            xo[k * n + i] = xa[k * n + i] + dvi * h;
        }
    }
}

void orc_enforce_momentum(int32_t n, const double* mass, const double* xb, const double* vb,
                          const double* xa, const double* va, double h, double radius, uint32_t flags,
                          double* x_out, double* v_out)
{
    if (n <= 0) return;
    const size_t n3 = 3u * (size_t)n;
    double* buf = (double*)calloc(6u * n3, sizeof(double));
    if (!buf) return;
    double *sxb = buf, *svb = buf + n3, *sxa = buf + 2 * n3, *sva = buf + 3 * n3;
    double *sxo = buf + 4 * n3, *svo = buf + 5 * n3;
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            sxb[(size_t)k * n + i] = xb[3 * i + k];
            svb[(size_t)k * n + i] = vb[3 * i + k];
            sxa[(size_t)k * n + i] = xa[3 * i + k];
            sva[(size_t)k * n + i] = va[3 * i + k];
        }
    momentum_body(0, n, n, mass, sxb, svb, sxa, sva, h, radius, flags, sxo, svo);
    for (int32_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            x_out[3 * i + k] = sxo[(size_t)k * n + i];
            v_out[3 * i + k] = svo[(size_t)k * n + i];
        }
    free(buf);
}

/* ------------------------------------------------------------------------ */
/* Contact projections (Sec. III-A constraints (1) and (2); Alg. 1           */
/* ParticleGroundContact / ParticleParticleContact).  The paper names the    */
/* constraints and a friction coefficient but not their formulas.  Readings: */
/*  * a plane (n, d) keeps the sphere surface on the plane: n.x >= d + r;    */
/*    penetration pi = r - (n.x - d) moves the particle by pi n;             */
/*  * two spheres of different bodies touch at distance 2r; penetration      */
/*    pi = 2r - |x_p - x_q| is split by inverse mass, w_p / (w_p + w_q);     */
/*  * Coulomb friction in position form, static and kinetic coefficient mu:  */
/*    the tangential displacement u_t since the substep start (relative, for */
/*    a pair) is removed up to mu * pi:  -u_t * min(1, mu pi / |u_t|);       */
/*    planes act as infinite mass;                                           */
/*  * a pair's correction is divided by max(n_p, n_q), the two neighbour-list */
/*    lengths (symmetric, so each pair exchanges equal and opposite momentum).*/
/* All corrections are computed from X_i (Jacobi).                           */
/* ------------------------------------------------------------------------ */
static void plane_delta(const orc_params* p, const double* xi, const double* x0, double* out)
{
    out[0] = out[1] = out[2] = 0.0;
    const double r = p->radius;
    for (int j = 0; j < p->n_planes; ++j) {
        const double* nrm = p->planes[j];
        const double e = dot3(nrm, xi) - nrm[3];
        if (!(e < r)) continue;
        const double pen = r - e;
        double u[3] = {xi[0] - x0[0], xi[1] - x0[1], xi[2] - x0[2]};
        const double un = dot3(u, nrm);
        for (int k = 0; k < 3; ++k) u[k] -= un * nrm[k];
        const double ut = norm3(u);
        double f = 0.0;
        if (ut > 0.0) f = fmin(1.0, p->mu * pen / ut);
        for (int k = 0; k < 3; ++k) out[k] += pen * nrm[k] - f * u[k];
    }
}

static void pair_delta(const orc_params* p, const double* xi, const double* x0i, double mi,
                       const double* xj, const double* x0j, double mj, double* out)
{
    out[0] = out[1] = out[2] = 0.0;
    const double d[3] = {xi[0] - xj[0], xi[1] - xj[1], xi[2] - xj[2]};
    const double l = norm3(d);
    const double two_r = 2.0 * p->radius;
    if (!(l > 0.0) || !(l < two_r)) return;
    const double nrm[3] = {d[0] / l, d[1] / l, d[2] / l};
    const double pen = two_r - l;
    const double wi = 1.0 / mi, wj = 1.0 / mj;
    const double alpha = wi / (wi + wj);
    double u[3];
    for (int k = 0; k < 3; ++k) u[k] = (xi[k] - x0i[k]) - (xj[k] - x0j[k]);
    const double un = dot3(u, nrm);
    for (int k = 0; k < 3; ++k) u[k] -= un * nrm[k];
    const double ut = norm3(u);
    double f = 0.0;
    if (ut > 0.0) f = fmin(1.0, p->mu * pen / ut);
    for (int k = 0; k < 3; ++k) out[k] = alpha * (pen * nrm[k] - f * u[k]);
}

/* ------------------------------------------------------------------------ */
/* One substep: Alg. 1 (integration step, then K Jacobi iterations of        */
/* contacts + shape matching, velocity update, momentum constraint).         */
/* Readings:                                                                 */
/*  * f_ext covers gravity (w m g = g) plus an optional per-particle         */
/*    acceleration;                                                          */
/*  * velocity update (Sec. III-B, Eqs. (1)-(3)) is incremental across       */
/*    iterations: V_{i+1} = V_i + dX_i / dt, which equals (X_{i+1}-X_init)/dt */
/*    in exact arithmetic for every i (the paper's V~ + dX/dt is its i = 0   */
/*    case); ORC_STD_VELOCITY gives standard PBD's (X_{i+1} - X_init)/dt;    */
/*  * "before shape matching" is X_i + dX_PG + dX_PP with matching velocity,  */
/*    "after" is X_{i+1}, V_{i+1} (Sec. III-C); the constraint runs every     */
/*    iteration, inside the solver loop of Alg. 1.                           */
/* ------------------------------------------------------------------------ */
int32_t orc_substep(const orc_params* p, int32_t n, int32_t nb, const int32_t* body_start,
                    const double* mass, const double* body_mass, const double* q,
                    const double* accel, double* x, double* v)
{
    if (n <= 0) return 0;
    const size_t n3 = 3u * (size_t)n;
    const double h = p->h;
    const int nthr = threads_of(p);
    double* buf = (double*)malloc(9u * n3 * sizeof(double));
    double *x0 = buf, *X = buf + n3, *V = buf + 2 * n3, *Cd = buf + 3 * n3, *Dd = buf + 4 * n3;
    double *Xb = buf + 5 * n3, *Vb = buf + 6 * n3, *Xa = buf + 7 * n3, *Va = buf + 8 * n3;
    int32_t* body = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    for (int32_t b = 0; b < nb; ++b)
        for (int32_t i = body_start[b]; i < body_start[b + 1]; ++i) body[i] = b;

    /* integration step (Alg. 1, first loop) */
    for (int k = 0; k < 3; ++k)
        for (int32_t i = 0; i < n; ++i) {
            const size_t j = (size_t)k * n + i;
            const double a = p->gravity[k] + (accel ? accel[j] : 0.0);
            x0[j] = x[j];
            V[j] = v[j] + h * a;
            X[j] = x[j] + h * V[j];
        }

    /* neighbour lists from the FP32 recipe */
    float* f32 = (float*)malloc(3u * n3 * sizeof(float));
    float *x32 = f32, *v32 = f32 + n3, *xt32 = f32 + 2 * n3;
    float* a32 = NULL;
    for (size_t j = 0; j < n3; ++j) { x32[j] = (float)x[j]; v32[j] = (float)v[j]; }
    if (accel) {
        a32 = (float*)malloc(n3 * sizeof(float));
        for (size_t j = 0; j < n3; ++j) a32[j] = (float)accel[j];
    }
    orc_predict32(n, p, x32, v32, a32, xt32);
    const size_t T = (size_t)1u << p->hash_bits;
    uint32_t* ib = (uint32_t*)malloc((2u * (size_t)n + 2u * T) * sizeof(uint32_t));
    uint32_t *key = ib, *sid = ib + n, *cs = ib + 2 * (size_t)n, *cc = cs + T;
    uint32_t *off = NULL, *flat = NULL;
    const int32_t max_nbr = build_index(n, p, body, xt32, key, sid, cs, cc, &off, &flat);
    free(ib);
    free(f32);
    free(a32);

    const uint32_t avg = (p->flags >> ORC_PP_AVG_SHIFT) & 3u;
    for (int32_t it = 0; it < p->iterations; ++it) {
        /* contacts: planes and pairs, from X_i */
#pragma omp parallel for schedule(static) num_threads(nthr)
        for (int32_t i = 0; i < n; ++i) {
            const double xi[3] = {X_(X, n, i), Y_(X, n, i), Z_(X, n, i)};
            const double x0i[3] = {X_(x0, n, i), Y_(x0, n, i), Z_(x0, n, i)};
            double acc[3], d[3];
            plane_delta(p, xi, x0i, acc);
            const uint32_t ni = off[i + 1] - off[i];
            for (uint32_t s = off[i]; s < off[i + 1]; ++s) {
                const int32_t j = (int32_t)flat[s];
                const uint32_t nj = off[j + 1] - off[j];
                const double xj[3] = {X_(X, n, j), Y_(X, n, j), Z_(X, n, j)};
                const double x0j[3] = {X_(x0, n, j), Y_(x0, n, j), Z_(x0, n, j)};
                pair_delta(p, xi, x0i, mass[i], xj, x0j, mass[j], d);
                double wgt = 1.0;
                if (avg == ORC_PP_AVG_MAX) wgt = 1.0 / (double)(ni > nj ? ni : nj);
                else if (avg == ORC_PP_AVG_OWN) wgt = 1.0 / (double)ni;
                for (int k = 0; k < 3; ++k) acc[k] += wgt * d[k];
            }
            X_(Cd, n, i) = acc[0]; Y_(Cd, n, i) = acc[1]; Z_(Cd, n, i) = acc[2];
        }
        /* shape matching per body (Mueller et al. 2005), from X_i */
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthr)
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t s = body_start[b], e = body_start[b + 1];
            double c[3] = {0, 0, 0}, A[9] = {0}, R[9];
            for (int32_t i = s; i < e; ++i) {
                c[0] += mass[i] * X_(X, n, i);
                c[1] += mass[i] * Y_(X, n, i);
                c[2] += mass[i] * Z_(X, n, i);
            }
            for (int k = 0; k < 3; ++k) c[k] /= body_mass[b];
            for (int32_t i = s; i < e; ++i) {
                const double r[3] = {X_(X, n, i) - c[0], Y_(X, n, i) - c[1], Z_(X, n, i) - c[2]};
                const double qi[3] = {X_(q, n, i), Y_(q, n, i), Z_(q, n, i)};
                for (int a = 0; a < 3; ++a)
                    for (int bb = 0; bb < 3; ++bb) A[3 * a + bb] += mass[i] * r[a] * qi[bb];
            }
            orc_polar(A, R);
            for (int32_t i = s; i < e; ++i) {
                const double qi[3] = {X_(q, n, i), Y_(q, n, i), Z_(q, n, i)};
                for (int a = 0; a < 3; ++a) {
                    const double goal = R[3 * a] * qi[0] + R[3 * a + 1] * qi[1] + R[3 * a + 2] * qi[2] + c[a];
                    Dd[(size_t)a * n + i] = goal - X[(size_t)a * n + i];
                }
            }
        }
        /* position and velocity update (Alg. 1; Sec. III-B) */
        for (size_t j = 0; j < n3; ++j) {
            Xb[j] = X[j] + Cd[j];
            Xa[j] = Xb[j] + Dd[j];
            if (p->flags & ORC_STD_VELOCITY) {
                Vb[j] = (Xb[j] - x0[j]) / h;
                Va[j] = (Xa[j] - x0[j]) / h;
            } else {
                Vb[j] = V[j] + Cd[j] / h;
                Va[j] = Vb[j] + Dd[j] / h;
            }
        }
        /* momentum conservation constraint, per body (Sec. III-C) */
        if ((p->flags & (ORC_NO_LIN_MOM | ORC_NO_ANG_MOM)) == (ORC_NO_LIN_MOM | ORC_NO_ANG_MOM)) {
            memcpy(X, Xa, n3 * sizeof(double));
            memcpy(V, Va, n3 * sizeof(double));
        } else {
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthr)
            for (int32_t b = 0; b < nb; ++b)
                momentum_body(body_start[b], body_start[b + 1], n, mass, Xb, Vb, Xa, Va, h,
                              p->radius, p->flags, X, V);
        }
    }
    memcpy(x, X, n3 * sizeof(double));
    memcpy(v, V, n3 * sizeof(double));
    free(off);
    free(flat);
    free(body);
    free(buf);
    return max_nbr;
}

int32_t orc_run(const orc_params* p, int32_t n, int32_t nb, const int32_t* body_start,
                const double* mass, const double* body_mass, const double* q,
                const double* accel, double* x, double* v, int32_t n_substeps)
{
    int32_t mx = 0;
    for (int32_t s = 0; s < n_substeps; ++s) {
        const int32_t m = orc_substep(p, n, nb, body_start, mass, body_mass, q, accel, x, v);
        if (m > mx) mx = m;
    }
    return mx;
}

/* Per-body state of (x, v): centre of mass, the rotation of shape matching for
 * this pose (Sec. III-C: the least-squares rotation from the rest offsets q,
 * i.e. the polar rotation of A = sum m (x - c) q^T), linear momentum and
 * angular momentum about the centre (the quantities of Sec. III-C, Eqs.
 * (4)-(5)).  Plain definitions, FP64, ascending particle order. */
void orc_body_state(int32_t n, int32_t nb, const int32_t* body_start, const double* mass, const double* q,
                    const double* x, const double* v, double* com, double* rot9, double* P, double* L)
{
    for (int32_t b = 0; b < nb; ++b) {
        double M = 0.0, c[3] = {0.0, 0.0, 0.0};
        for (int32_t i = body_start[b]; i < body_start[b + 1]; ++i) {
            M += mass[i];
            c[0] += mass[i] * X_(x, n, i);
            c[1] += mass[i] * Y_(x, n, i);
            c[2] += mass[i] * Z_(x, n, i);
        }
        for (int a = 0; a < 3; ++a) c[a] /= M;
        double A[9] = {0}, Pb[3] = {0}, Lb[3] = {0};
        for (int32_t i = body_start[b]; i < body_start[b + 1]; ++i) {
            const double r[3] = {X_(x, n, i) - c[0], Y_(x, n, i) - c[1], Z_(x, n, i) - c[2]};
            const double qi[3] = {X_(q, n, i), Y_(q, n, i), Z_(q, n, i)};
            const double vi[3] = {X_(v, n, i), Y_(v, n, i), Z_(v, n, i)};
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) A[3 * a + k] += mass[i] * r[a] * qi[k];
            for (int a = 0; a < 3; ++a) Pb[a] += mass[i] * vi[a];
            Lb[0] += mass[i] * (r[1] * vi[2] - r[2] * vi[1]);
            Lb[1] += mass[i] * (r[2] * vi[0] - r[0] * vi[2]);
            Lb[2] += mass[i] * (r[0] * vi[1] - r[1] * vi[0]);
        }
        for (int a = 0; a < 3; ++a) {
            com[3 * (size_t)b + a] = c[a];
            P[3 * (size_t)b + a] = Pb[a];
            L[3 * (size_t)b + a] = Lb[a];
        }
        orc_polar(A, rot9 + 9 * (size_t)b);
    }
}
