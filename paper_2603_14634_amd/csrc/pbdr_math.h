// Device-side arithmetic shared by the PBD-R kernels of libpbdr: the FP32
// hash-grid key and neighbour predicate, fixed-order wave reductions, and
// the small 3x3 algebra of shape matching and of the momentum constraint.
// Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace pbdr {
namespace dev {

// ---------------------------------------------------------------------------
// hash grid (FP32, contraction off)
// ---------------------------------------------------------------------------

__device__ inline uint32_t cell_axis(float xt, float o, float inv_a)
{
#pragma clang fp contract(off)
    const float t = xt - o;
    const float u = t * inv_a;
    float f = floorf(u);
    if (!(f >= -16777216.0f)) f = -16777216.0f;
    if (!(f <= 16777216.0f)) f = 16777216.0f;
    return ((uint32_t)(int32_t)f) & 1023u;
}

// spreads the 10 low bits of v to bit positions 0, 3, 6, ..., 27
__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline uint32_t morton(uint32_t cx, uint32_t cy, uint32_t cz, uint32_t mask)
{
    return (spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2)) & mask;
}

__device__ inline bool within(float ax, float ay, float az, float bx, float by, float bz, float r2)
{
#pragma clang fp contract(off)
    const float dx = bx - ax;
    const float dy = by - ay;
    const float dz = bz - az;
    const float sx = dx * dx;
    const float sy = dy * dy;
    const float sz = dz * dz;
    const float s = (sx + sy) + sz;
    return s < r2;
}

// ---------------------------------------------------------------------------
// wave / workgroup reductions
// ---------------------------------------------------------------------------

template <int CTRL, int ROWS>
__device__ inline float dpp_add(float v)
{
    return v + __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS,
                                                                      0xf, false));
}

// Sum over the 64 lanes, exact same order every time; valid in lane 63.
__device__ inline float wave_sum_to_63(float v)
{
    v = dpp_add<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v = dpp_add<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]   -> quad sums
    v = dpp_add<0x141, 0xf>(v);   // row_half_mirror       -> 8-lane sums
    v = dpp_add<0x140, 0xf>(v);   // row_mirror            -> 16-lane row sums
    v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    return v;
}

// Sums over the 64 lanes of K values at once (K a multiple of 4), in a fixed
// order.  The gfx950 lane swaps pair up values: v_permlane32_swap exchanges
// the upper half of one register with the lower half of another, so one swap
// and one add fold two values from 64 lanes to 32; v_permlane16_swap does the
// same for rows (16 lanes) within each half; DPP then sums each row.  That is
// about 2.5 K instructions where K separate wave sums take 6 K or more.  On
// return, every lane of row j (lanes 16 j .. 16 j + 15) of v[p] holds the sum
// of value j K/4 + p, for p < K/4.
template <int K>
__device__ inline void wave_sums_by_row(float* v)
{
    static_assert(K % 4 == 0, "K must be a multiple of 4");
    constexpr int H = K / 2, Q = K / 4;
    // value p in lanes 0-31, value p + H in lanes 32-63
#pragma unroll
    for (int p = 0; p < H; ++p) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[p]), __float_as_uint(v[p + H]), false,
                                                        false);
        const unsigned lo = r[0], hi = r[1];   // (element-wise __builtin_bit_cast of r drops r[1])
        v[p] = __uint_as_float(lo) + __uint_as_float(hi);
    }
    // value p in row 0, p + Q in row 1, p + H in row 2, p + H + Q in row 3
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[p]), __float_as_uint(v[p + Q]), false,
                                                        false);
        const unsigned lo = r[0], hi = r[1];
        v[p] = __uint_as_float(lo) + __uint_as_float(hi);
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        float t = v[p];
        t = dpp_add<0xb1, 0xf>(t);    // quad_perm [1,0,3,2]
        t = dpp_add<0x4e, 0xf>(t);    // quad_perm [2,3,0,1]
        t = dpp_add<0x141, 0xf>(t);   // row_half_mirror
        t = dpp_add<0x140, 0xf>(t);   // row_mirror: the row sum in all 16 lanes
        v[p] = t;
    }
}

// FP64 form of wave_sums_by_row: the same lane swaps and DPP steps applied to
// both 32-bit halves of each value, with FP64 adds.  On return, every lane of
// row j of v[p] holds the sum of value j K/4 + p, for p < K/4.
template <int CTRL>
__device__ inline double dpp_add64(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xf, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xf, 0xf, false);
    return v + __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <int K>
__device__ inline void wave_sums_by_row64(double* v)
{
    static_assert(K % 4 == 0, "K must be a multiple of 4");
    constexpr int H = K / 2, Q = K / 4;
#pragma unroll
    for (int p = 0; p < H; ++p) {
        const unsigned long long a = __builtin_bit_cast(unsigned long long, v[p]);
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v[p + H]);
        const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
        const unsigned l0 = lo[0], l1 = lo[1], h0 = hi[0], h1 = hi[1];
        v[p] = __builtin_bit_cast(double, ((unsigned long long)h0 << 32) | l0) +
               __builtin_bit_cast(double, ((unsigned long long)h1 << 32) | l1);
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const unsigned long long a = __builtin_bit_cast(unsigned long long, v[p]);
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v[p + Q]);
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
        const unsigned l0 = lo[0], l1 = lo[1], h0 = hi[0], h1 = hi[1];
        v[p] = __builtin_bit_cast(double, ((unsigned long long)h0 << 32) | l0) +
               __builtin_bit_cast(double, ((unsigned long long)h1 << 32) | l1);
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        double t = v[p];
        t = dpp_add64<0xb1>(t);    // quad_perm [1,0,3,2]
        t = dpp_add64<0x4e>(t);    // quad_perm [2,3,0,1]
        t = dpp_add64<0x141>(t);   // row_half_mirror
        t = dpp_add64<0x140>(t);   // row_mirror: the row sum in all 16 lanes
        v[p] = t;
    }
}

// ---------------------------------------------------------------------------
// small 3x3 algebra (FP32)
// ---------------------------------------------------------------------------

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// 1 / sqrt(a) for a positive normal FP64 a: the hardware estimate (about 22
// correct bits) refined by two Newton steps y <- y + y (1 - a y^2) / 2, each
// of which doubles the correct bits, so the result is within a few ulps of
// the exact value.  Nine instructions where sqrt and a correctly rounded
// division take about thirty.
__device__ inline double rsqrt64(double a)
{
    const double h = 0.5 * a;
    double y = __builtin_amdgcn_rsq(a);
#pragma unroll
    for (int k = 0; k < 2; ++k) y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
    return y;
}

__device__ inline void cross(const float* a, const float* b, float* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// cofactor matrix: inverse transpose = cof / det
__device__ inline void cof3(const float* m, float* c)
{
    c[0] = m[4] * m[8] - m[5] * m[7];
    c[1] = m[5] * m[6] - m[3] * m[8];
    c[2] = m[3] * m[7] - m[4] * m[6];
    c[3] = m[2] * m[7] - m[1] * m[8];
    c[4] = m[0] * m[8] - m[2] * m[6];
    c[5] = m[1] * m[6] - m[0] * m[7];
    c[6] = m[1] * m[5] - m[2] * m[4];
    c[7] = m[2] * m[3] - m[0] * m[5];
    c[8] = m[0] * m[4] - m[1] * m[3];
}

// One Jacobi rotation zeroing a[p][q] of a symmetric 3x3 matrix (r is the
// remaining index); Q accumulates the rotations (columns = eigenvectors).
template <int p, int q, int r>
__device__ inline void jacobi_rotate(float* a, float* Q)
{
    const float apq = a[3 * p + q];
    if (apq == 0.0f) return;
    const float theta = (a[3 * q + q] - a[3 * p + p]) / (2.0f * apq);
    const float t = copysignf(1.0f, theta) / (fabsf(theta) + sqrtf(theta * theta + 1.0f));
    const float cs = 1.0f / sqrtf(t * t + 1.0f), sn = t * cs;
    a[3 * p + p] -= t * apq;
    a[3 * q + q] += t * apq;
    a[3 * p + q] = a[3 * q + p] = 0.0f;
    const float arp = a[3 * r + p], arq = a[3 * r + q];
    a[3 * r + p] = a[3 * p + r] = cs * arp - sn * arq;
    a[3 * r + q] = a[3 * q + r] = sn * arp + cs * arq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float qp = Q[3 * k + p], qq = Q[3 * k + q];
        Q[3 * k + p] = cs * qp - sn * qq;
        Q[3 * k + q] = sn * qp + cs * qq;
    }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix a (row-major,
// overwritten by a near-diagonal matrix); columns of Q are the eigenvectors.
__device__ inline void sym_eig3(float* a, float* Q)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) Q[k] = (k % 4 == 0) ? 1.0f : 0.0f;
    for (int sweep = 0; sweep < 10; ++sweep) {
        const float off = fabsf(a[1]) + fabsf(a[2]) + fabsf(a[5]);
        const float diag = fabsf(a[0]) + fabsf(a[4]) + fabsf(a[8]);
        if (!(off > 1e-9f * diag)) break;
        jacobi_rotate<0, 1, 2>(a, Q);
        jacobi_rotate<0, 2, 1>(a, Q);
        jacobi_rotate<1, 2, 0>(a, Q);
    }
}

// Swaps eigenpairs (lam_i, column i of V) and (lam_j, column j) if lam_j > lam_i.
template <int i, int j>
__device__ inline void order_pair(float* lam, float* V)
{
    const bool sw = lam[j] > lam[i];
    const float li = lam[i], lj = lam[j];
    lam[i] = sw ? lj : li;
    lam[j] = sw ? li : lj;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float vi = V[3 * k + i], vj = V[3 * k + j];
        V[3 * k + i] = sw ? vj : vi;
        V[3 * k + j] = sw ? vi : vj;
    }
}

// Rotation from the eigenvectors of A^T A, completing a proper frame; used when
// A is (near) singular, where the Newton iteration below cannot run.
__device__ inline void rotation_from_normal_eq(const float* A, float* R)
{
    float S[9], V[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            S[3 * r + cc] = A[r] * A[cc] + A[3 + r] * A[3 + cc] + A[6 + r] * A[6 + cc];
    sym_eig3(S, V);
    float lam[3] = {S[0], S[4], S[8]};
    order_pair<0, 1>(lam, V);
    order_pair<0, 2>(lam, V);
    order_pair<1, 2>(lam, V);            // descending
    float v0[3], v1[3], u0[3], u1[3], u2[3], v2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        v0[j] = V[3 * j];
        v1[j] = V[3 * j + 1];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        u0[j] = A[3 * j] * v0[0] + A[3 * j + 1] * v0[1] + A[3 * j + 2] * v0[2];
        u1[j] = A[3 * j] * v1[0] + A[3 * j + 1] * v1[1] + A[3 * j + 2] * v1[2];
    }
    const float n0 = sqrtf(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
    if (!(n0 > 0.0f)) {
#pragma unroll
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0f : 0.0f;
        return;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) u0[j] /= n0;
    const float d = u0[0] * u1[0] + u0[1] * u1[1] + u0[2] * u1[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) u1[j] -= d * u0[j];
    float n1 = sqrtf(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    if (!(n1 > 1e-6f * n0)) {
        // rank one: any unit vector orthogonal to u0
        const float e[3] = {fabsf(u0[0]) < 0.9f ? 1.0f : 0.0f, fabsf(u0[0]) < 0.9f ? 0.0f : 1.0f, 0.0f};
        cross(u0, e, u1);
        n1 = sqrtf(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) u1[j] /= n1;
    cross(u0, u1, u2);
    cross(v0, v1, v2);                   // proper right frame
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) R[3 * r + cc] = u0[r] * v0[cc] + u1[r] * v1[cc] + u2[r] * v2[cc];
}

// Rotation maximising tr(R^T A): Higham's determinant-scaled Newton iteration
// X <- (g X + X^-T / g) / 2, g = |det X|^(-1/3), for the orthogonal polar
// factor; a reflection (det A < 0) is turned into the nearest rotation by
// flipping the direction of the smallest eigenvalue of the symmetric factor.
// The scaling only speeds convergence, so it uses hardware log2 / exp2; the
// last step is unscaled.
__device__ inline void polar_rotation(const float* A, float* R)
{
    float nrm2 = 0.0f;
    for (int k = 0; k < 9; ++k) nrm2 += A[k] * A[k];
    float Ca[9];
    cof3(A, Ca);
    const float dA = A[0] * Ca[0] + A[1] * Ca[1] + A[2] * Ca[2];
    if (!(nrm2 > 0.0f)) {
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0f : 0.0f;
        return;
    }
    if (!(fabsf(dA) > 1e-5f * nrm2 * sqrtf(nrm2))) {
        rotation_from_normal_eq(A, R);
        return;
    }
    float X[9], C[9];
    for (int k = 0; k < 9; ++k) {
        X[k] = A[k];
        C[k] = Ca[k];
    }
    float det = dA;
    for (int it = 0; it < 24; ++it) {
        const float g = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(fabsf(det)) * (1.0f / 3.0f));
        const float a = 0.5f * frcp(g), b = 0.5f * g * frcp(det);
        float diff = 0.0f;
        for (int k = 0; k < 9; ++k) {
            const float xn = a * X[k] + b * C[k];
            diff += (xn - X[k]) * (xn - X[k]);
            X[k] = xn;
        }
        cof3(X, C);
        det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
        if (diff < 1e-10f) break;
    }
    {   // final unscaled step
        const float id = frcp(det);
        for (int k = 0; k < 9; ++k) X[k] = 0.5f * (X[k] + C[k] * id);
    }
    if (dA < 0.0f) {
        float H[9], Q[9];
        for (int r = 0; r < 3; ++r)          // H = X^T A (symmetric factor)
            for (int cc = 0; cc < 3; ++cc)
                H[3 * r + cc] = X[r] * A[cc] + X[3 + r] * A[3 + cc] + X[6 + r] * A[6 + cc];
        for (int r = 0; r < 3; ++r)
            for (int cc = r + 1; cc < 3; ++cc) H[3 * r + cc] = H[3 * cc + r] = 0.5f * (H[3 * r + cc] + H[3 * cc + r]);
        sym_eig3(H, Q);
        float lam[3] = {H[0], H[4], H[8]};
        order_pair<0, 1>(lam, Q);
        order_pair<0, 2>(lam, Q);
        order_pair<1, 2>(lam, Q);        // smallest eigenvalue last
        const float w[3] = {Q[2], Q[5], Q[8]};
        const float Xw[3] = {X[0] * w[0] + X[1] * w[1] + X[2] * w[2], X[3] * w[0] + X[4] * w[1] + X[5] * w[2],
                             X[6] * w[0] + X[7] * w[1] + X[8] * w[2]};
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) X[3 * r + cc] -= 2.0f * Xw[r] * w[cc];
    }
    for (int k = 0; k < 9; ++k) R[k] = X[k];
}

// Rotation maximising tr(R^T A), refined from a nearby rotation R0 (the
// previous solver iteration's): Newton steps on SO(3).  With B = R^T A the
// gradient of tr(Q^T B) at Q = I is -g, g = (B12 - B21, B20 - B02, B01 - B10),
// and the Hessian is sym(B) - tr(B) I, so the step is omega = -(tr(B) I -
// sym(B))^-1 g, applied through the Cayley map; one unscaled Newton polar step
// then restores orthogonality.  Returns false when the start is too far (the
// step does not shrink below 3e-5 rad within two steps) or the Hessian is not
// definite; the caller then uses polar_rotation.
// polar_refine_steps: the Newton steps alone, leaving X orthogonal to about
// 1e-7 (for callers that make it orthogonal themselves).
__device__ inline bool polar_refine_steps(const float* A, const float* R0, float* X)
{
    for (int k = 0; k < 9; ++k) X[k] = R0[k];
    bool done = false;
    for (int step = 0; step < 2 && !done; ++step) {
        float B[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) B[3 * a + b] = X[a] * A[b] + X[3 + a] * A[3 + b] + X[6 + a] * A[6 + b];
        const float g[3] = {B[5] - B[7], B[6] - B[2], B[1] - B[3]};
        const float tr = B[0] + B[4] + B[8];
        const float H[9] = {tr - B[0], -0.5f * (B[1] + B[3]), -0.5f * (B[2] + B[6]),
                            -0.5f * (B[1] + B[3]), tr - B[4], -0.5f * (B[5] + B[7]),
                            -0.5f * (B[2] + B[6]), -0.5f * (B[5] + B[7]), tr - B[8]};
        float C[9];
        cof3(H, C);
        const float det = H[0] * C[0] + H[1] * C[1] + H[2] * C[2];
        const float t3 = tr * (1.0f / 3.0f);
        if (!(tr > 0.0f) || !(det > 1e-4f * t3 * t3 * t3)) return false;
        const float id = frcp(det);
        float w[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) w[r] = -0.5f * (C[3 * r] * g[0] + C[3 * r + 1] * g[1] + C[3 * r + 2] * g[2]) * id;
        const float w2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];   // |omega / 2|^2
        done = w2 < 2.25e-10f;                                        // |omega| < 3e-5
        // Cayley: Q = I + 2 / (1 + |w|^2) ([w]x + [w]x^2)
        const float f = 2.0f * frcp(1.0f + w2);
        const float Q[9] = {1.0f + f * (w[0] * w[0] - w2), f * (w[0] * w[1] - w[2]), f * (w[0] * w[2] + w[1]),
                            f * (w[0] * w[1] + w[2]), 1.0f + f * (w[1] * w[1] - w2), f * (w[1] * w[2] - w[0]),
                            f * (w[0] * w[2] - w[1]), f * (w[1] * w[2] + w[0]), 1.0f + f * (w[2] * w[2] - w2)};
        float Y[9];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) Y[3 * a + b] = X[3 * a] * Q[b] + X[3 * a + 1] * Q[3 + b] + X[3 * a + 2] * Q[6 + b];
        for (int k = 0; k < 9; ++k) X[k] = Y[k];
    }
    return done;
}

__device__ inline bool polar_refine(const float* A, const float* R0, float* R)
{
    float X[9];
    if (!polar_refine_steps(A, R0, X)) return false;
    float C[9];
    cof3(X, C);
    const float id = frcp(X[0] * C[0] + X[1] * C[1] + X[2] * C[2]);
    for (int k = 0; k < 9; ++k) R[k] = 0.5f * (X[k] + C[k] * id);
    return true;
}

// omega = I^+ L for a symmetric positive semi-definite inertia tensor
// (xx, yy, zz, xy, xz, yz).  `scale` = max(trace I, M (2r)^2) sets what counts
// as zero: the inertia of a one-particle body is rounding noise, and a body
// whose particles lie on a line has one vanishing eigenvalue.  Well
// conditioned tensors use the closed-form inverse; otherwise an
// eigen-decomposition drops eigenvalues at or below 1e-6 * scale.
__device__ inline void solve_inertia(const float* I6, const float* L, float scale, float* w)
{
    const float I[9] = {I6[0], I6[3], I6[4], I6[3], I6[1], I6[5], I6[4], I6[5], I6[2]};
    w[0] = w[1] = w[2] = 0.0f;
    if (!(scale > 0.0f)) return;
    float C[9];
    cof3(I, C);
    const float det = I[0] * C[0] + I[1] * C[1] + I[2] * C[2];
    const float t3 = scale * (1.0f / 3.0f);
    if (det > 1e-3f * t3 * t3 * t3) {
        const float id = frcp(det);    // I^-1 = cof^T / det, cof symmetric here
        for (int r = 0; r < 3; ++r) w[r] = (C[3 * r] * L[0] + C[3 * r + 1] * L[1] + C[3 * r + 2] * L[2]) * id;
        return;
    }
    float a[9], Q[9];
    for (int k = 0; k < 9; ++k) a[k] = I[k];
    sym_eig3(a, Q);
    for (int k = 0; k < 3; ++k) {
        const float lam = a[4 * k];
        if (!(lam > 1e-6f * scale)) continue;
        const float proj = (Q[k] * L[0] + Q[3 + k] * L[1] + Q[6 + k] * L[2]) / lam;
        for (int r = 0; r < 3; ++r) w[r] += proj * Q[3 * r + k];
    }
}

}  // namespace dev
}  // namespace pbdr
