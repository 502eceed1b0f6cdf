// PBD-R solver substep on gfx950 (MI355X).
//
// One substep of Alg. 1 of "Physically Accurate Rigid-Body Dynamics in
// Particle-Based Simulation" (arXiv 2603.14634) as a chain of kernels on one
// stream:
//
//   predict_keys      integration step (Alg. 1, first loop) + hash-grid key and
//                     per-key slot of every particle (atomic counting pass)
//   scan (3 kernels)  exclusive prefix sum of the per-key counts -> cell starts
//   scatter           particles grouped by key; sorted copies of the FP32
//                     predicted positions and body ids for the neighbour pass
//   neighbours        27-cell stencil, FP32 predicate, ascending lists; also
//                     writes the canonical (key, id) order
//   iterate x K       one workgroup per body: shape matching (Sec. III-C,
//                     Mueller et al. 2005), ground and particle contacts,
//                     incremental velocity update (Sec. III-B), momentum
//                     conservation constraint (Sec. III-C, Eqs. (4)-(5))
//   finalize          x = X_init + (X_K - X_init), v = V_K; non-finite check
//
// Numerics.  Inside a substep positions are carried as the displacement
// delta = X_i - X_init (small magnitude), so FP32 resolves corrections far
// below the ulp of world coordinates: pair separations are formed as
// (X_init,p - X_init,q) + (delta_p - delta_q) (the first difference is exact
// for nearby particles), and body-relative coordinates are formed against an
// anchor particle of the body.  Velocities follow the paper's incremental
// update V_{i+1} = V_i + dX / dt.  All per-body sums are fixed-order tree
// reductions (wave shuffles, then LDS), so results are bitwise reproducible.
//
// The neighbour-search decisions (key, predicate) are taken in FP32 with no
// contraction, op by op, so they are reproducible by any IEEE FP32 evaluation
// of the same sequence.
#include "pbdr_device.h"

#include <math.h>

namespace pbdr {
namespace {

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
// integration step + keys + counting pass
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t* p, uint32_t n, uint32_t value)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void __launch_bounds__(kBlock) k_predict_keys(Scene s, StepConsts c)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const size_t n = (size_t)s.n;
    float xt[3];
    for (int k = 0; k < 3; ++k) {
        const size_t j = k * n + i;
        const float a = c.g[k] + (s.accel ? s.accel[j] : 0.0f);
        const float dv = c.h * a;
        const float vt = s.v[j] + dv;
        const float dx = c.h * vt;
        xt[k] = s.x[j] + dx;
        s.xt[j] = xt[k];
        s.dl[0][j] = dx;      // delta_0 = X~ - X_init
        s.vel[0][j] = vt;     // V_0 = V~
    }
    const uint32_t key = morton(cell_axis(xt[0], c.origin[0], c.inv_cell),
                                cell_axis(xt[1], c.origin[1], c.inv_cell),
                                cell_axis(xt[2], c.origin[2], c.inv_cell), c.key_mask);
    s.key[i] = key;
    s.rank[i] = atomicAdd(&s.cell_count[key], 1u);
}

// ---------------------------------------------------------------------------
// exclusive scan of the cell counts
// ---------------------------------------------------------------------------

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_tot[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wave) before += wave_tot[w];
        all += wave_tot[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_tiles(const uint32_t* counts, uint32_t T, uint32_t* tile_sums)
{
    __shared__ uint32_t wave_tot[kBlock / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < T) sum += counts[base + k];
    uint32_t total;
    (void)block_exclusive_scan(sum, wave_tot, &total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// single workgroup: tile sums -> exclusive tile offsets (in place)
__global__ void __launch_bounds__(kBlock) k_scan_tile_sums(uint32_t* tile_sums, uint32_t n_tiles)
{
    __shared__ uint32_t wave_tot[kBlock / 64];
    const uint32_t per = (n_tiles + kBlock - 1) / kBlock;
    const uint32_t lo = threadIdx.x * per;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; ++k)
        if (lo + k < n_tiles) sum += tile_sums[lo + k];
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, wave_tot, &total);
    for (uint32_t k = 0; k < per; ++k)
        if (lo + k < n_tiles) {
            const uint32_t c = tile_sums[lo + k];
            tile_sums[lo + k] = run;
            run += c;
        }
}

__global__ void __launch_bounds__(kBlock) k_scan_write(const uint32_t* counts, uint32_t T,
                                                       const uint32_t* tile_offsets, uint32_t* starts)
{
    __shared__ uint32_t wave_tot[kBlock / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t sum = 0;
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (base + k < T) ? counts[base + k] : 0u;
        sum += vals[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, wave_tot, &total) + tile_offsets[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < T) starts[base + k] = run;
        run += vals[k];
    }
}

__global__ void __launch_bounds__(kBlock) k_scatter(Scene s)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const size_t n = (size_t)s.n;
    const uint32_t slot = s.cell_start[s.key[i]] + s.rank[i];
    s.sorted_raw[slot] = (uint32_t)i;
    s.sxt[slot] = s.xt[i];
    s.sxt[n + slot] = s.xt[n + i];
    s.sxt[2 * n + slot] = s.xt[2 * n + i];
    s.sbody[slot] = s.body[i];
}

// ---------------------------------------------------------------------------
// neighbour lists
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_neighbours(Scene s, StepConsts c)
{
    extern __shared__ uint32_t lst[];          // [cap][kBlock], slot-major
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool live = i < s.n;
    const size_t n = (size_t)s.n;
    const int cap = c.nbr_cap;
    uint32_t count = 0;
    if (live) {
        const float px = s.xt[i], py = s.xt[n + i], pz = s.xt[2 * n + i];
        const int32_t pb = s.body[i];
        const uint32_t cx = cell_axis(px, c.origin[0], c.inv_cell);
        const uint32_t cy = cell_axis(py, c.origin[1], c.inv_cell);
        const uint32_t cz = cell_axis(pz, c.origin[2], c.inv_cell);
        // canonical slot of i inside its own key: ids below i sharing the key
        {
            const uint32_t k = s.key[i];
            const uint32_t b = s.cell_start[k], e = b + s.cell_count[k];
            uint32_t below = 0;
            for (uint32_t j = b; j < e; ++j) below += (s.sorted_raw[j] < (uint32_t)i) ? 1u : 0u;
            s.sorted[b + below] = (uint32_t)i;
        }
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const uint32_t k = morton(cx + (uint32_t)dx, cy + (uint32_t)dy, cz + (uint32_t)dz,
                                              c.key_mask);
                    const uint32_t b = s.cell_start[k], e = b + s.cell_count[k];
                    for (uint32_t j = b; j < e; ++j) {
                        if (s.sbody[j] == pb) continue;      // same body (also excludes i)
                        if (!within(px, py, pz, s.sxt[j], s.sxt[n + j], s.sxt[2 * n + j], c.search_r2))
                            continue;
                        const uint32_t q = s.sorted_raw[j];
                        // insert q keeping the `cap` smallest ids in ascending order
                        int m = (int)(count < (uint32_t)cap ? count : (uint32_t)cap);
                        if (m == cap && q > lst[(cap - 1) * kBlock + threadIdx.x]) {
                            ++count;
                            continue;
                        }
                        int pos = (m == cap) ? cap - 1 : m;
                        while (pos > 0 && lst[(pos - 1) * kBlock + threadIdx.x] > q) {
                            lst[pos * kBlock + threadIdx.x] = lst[(pos - 1) * kBlock + threadIdx.x];
                            --pos;
                        }
                        lst[pos * kBlock + threadIdx.x] = q;
                        ++count;
                    }
                }
        s.nbr_n[i] = count;
        const uint32_t stored = count < (uint32_t)cap ? count : (uint32_t)cap;
        for (uint32_t k = 0; k < stored; ++k) s.nbr[k * n + i] = lst[k * kBlock + threadIdx.x];
    }
    // statistics and capacity check, one atomic per wave
    uint32_t mx = count;
    unsigned long long sum = count;
    for (int off = 32; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off, 64));
        sum += __shfl_xor(sum, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        const int lo = blockIdx.x * kBlock + (threadIdx.x & ~63);
        const int rows = min(64, s.n - lo);
        if (rows > 0) {
            atomicMax(&s.counters->max_nbr, mx);
            atomicAdd(&s.counters->nbr_sum, sum);
            atomicAdd(&s.counters->nbr_rows, (unsigned long long)rows);
            if (mx > (uint32_t)cap) atomicOr(&s.counters->err, kErrCapacity);
        }
    }
}

// ---------------------------------------------------------------------------
// small 3x3 algebra (FP32)
// ---------------------------------------------------------------------------

__device__ inline float det3(const float* m)
{
    return m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
           m[2] * (m[3] * m[7] - m[4] * m[6]);
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

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix a (row-major,
// overwritten by a near-diagonal matrix); columns of Q are the eigenvectors.
__device__ void sym_eig3(float* a, float* Q)
{
    for (int k = 0; k < 9; ++k) Q[k] = (k % 4 == 0) ? 1.0f : 0.0f;
    for (int sweep = 0; sweep < 10; ++sweep) {
        const float off = fabsf(a[1]) + fabsf(a[2]) + fabsf(a[5]);
        const float diag = fabsf(a[0]) + fabsf(a[4]) + fabsf(a[8]);
        if (!(off > 1e-9f * diag)) break;
        for (int pr = 0; pr < 3; ++pr) {
            const int p = pr == 2 ? 1 : 0, q = pr == 0 ? 1 : 2, r = 3 - p - q;
            const float apq = a[3 * p + q];
            if (apq == 0.0f) continue;
            const float theta = (a[3 * q + q] - a[3 * p + p]) / (2.0f * apq);
            const float t = copysignf(1.0f, theta) / (fabsf(theta) + sqrtf(theta * theta + 1.0f));
            const float cs = 1.0f / sqrtf(t * t + 1.0f), sn = t * cs;
            a[3 * p + p] -= t * apq;
            a[3 * q + q] += t * apq;
            a[3 * p + q] = a[3 * q + p] = 0.0f;
            const float arp = a[3 * r + p], arq = a[3 * r + q];
            a[3 * r + p] = a[3 * p + r] = cs * arp - sn * arq;
            a[3 * r + q] = a[3 * q + r] = sn * arp + cs * arq;
            for (int k = 0; k < 3; ++k) {
                const float qp = Q[3 * k + p], qq = Q[3 * k + q];
                Q[3 * k + p] = cs * qp - sn * qq;
                Q[3 * k + q] = sn * qp + cs * qq;
            }
        }
    }
}

// Rotation from the eigenvectors of A^T A, completing a proper frame; used when
// A is (near) singular, where the Newton iteration below cannot run.
__device__ void rotation_from_normal_eq(const float* A, float* R)
{
    float S[9], V[9];
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc)
            S[3 * r + cc] = A[r] * A[cc] + A[3 + r] * A[3 + cc] + A[6 + r] * A[6 + cc];
    sym_eig3(S, V);
    int o[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (S[4 * o[b]] > S[4 * o[a]]) { const int t = o[a]; o[a] = o[b]; o[b] = t; }
    float v[3][3], u[3][3];
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) v[k][j] = V[3 * j + o[k]];   // v[k] = k-th eigenvector
    for (int k = 0; k < 2; ++k)
        for (int j = 0; j < 3; ++j) u[k][j] = A[3 * j] * v[k][0] + A[3 * j + 1] * v[k][1] + A[3 * j + 2] * v[k][2];
    float n0 = sqrtf(u[0][0] * u[0][0] + u[0][1] * u[0][1] + u[0][2] * u[0][2]);
    if (!(n0 > 0.0f)) {
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0f : 0.0f;
        return;
    }
    for (int j = 0; j < 3; ++j) u[0][j] /= n0;
    float d = u[0][0] * u[1][0] + u[0][1] * u[1][1] + u[0][2] * u[1][2];
    for (int j = 0; j < 3; ++j) u[1][j] -= d * u[0][j];
    float n1 = sqrtf(u[1][0] * u[1][0] + u[1][1] * u[1][1] + u[1][2] * u[1][2]);
    if (!(n1 > 1e-6f * n0)) {
        // rank one: any unit vector orthogonal to u0
        const float e[3] = {fabsf(u[0][0]) < 0.9f ? 1.0f : 0.0f, fabsf(u[0][0]) < 0.9f ? 0.0f : 1.0f, 0.0f};
        u[1][0] = u[0][1] * e[2] - u[0][2] * e[1];
        u[1][1] = u[0][2] * e[0] - u[0][0] * e[2];
        u[1][2] = u[0][0] * e[1] - u[0][1] * e[0];
        n1 = sqrtf(u[1][0] * u[1][0] + u[1][1] * u[1][1] + u[1][2] * u[1][2]);
    }
    for (int j = 0; j < 3; ++j) u[1][j] /= n1;
    u[2][0] = u[0][1] * u[1][2] - u[0][2] * u[1][1];
    u[2][1] = u[0][2] * u[1][0] - u[0][0] * u[1][2];
    u[2][2] = u[0][0] * u[1][1] - u[0][1] * u[1][0];
    const float vc[3] = {v[0][1] * v[1][2] - v[0][2] * v[1][1], v[0][2] * v[1][0] - v[0][0] * v[1][2],
                         v[0][0] * v[1][1] - v[0][1] * v[1][0]};
    for (int j = 0; j < 3; ++j) v[2][j] = vc[j];    // proper right frame
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) R[3 * r + cc] = u[0][r] * v[0][cc] + u[1][r] * v[1][cc] + u[2][r] * v[2][cc];
}

// Rotation maximising tr(R^T A): Higham's determinant-scaled Newton iteration
// X <- (g X + X^-T / g) / 2, g = |det X|^(-1/3), for the orthogonal polar
// factor; a reflection (det A < 0) is turned into the nearest rotation by
// flipping the direction of the smallest eigenvalue of the symmetric factor.
__device__ void polar_rotation(const float* A, float* R)
{
    float nrm2 = 0.0f;
    for (int k = 0; k < 9; ++k) nrm2 += A[k] * A[k];
    const float dA = det3(A);
    if (!(nrm2 > 0.0f)) {
        for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0f : 0.0f;
        return;
    }
    if (!(fabsf(dA) > 1e-5f * nrm2 * sqrtf(nrm2))) {
        rotation_from_normal_eq(A, R);
        return;
    }
    float X[9], C[9];
    for (int k = 0; k < 9; ++k) X[k] = A[k];
    for (int it = 0; it < 24; ++it) {
        cof3(X, C);
        const float det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
        const float g = cbrtf(fabsf(det));           // 1 / gamma
        const float a = 0.5f / g, b = 0.5f * g / det;
        float diff = 0.0f;
        for (int k = 0; k < 9; ++k) {
            const float xn = a * X[k] + b * C[k];
            diff += (xn - X[k]) * (xn - X[k]);
            X[k] = xn;
        }
        if (diff < 1e-12f) break;
    }
    {   // final unscaled step
        cof3(X, C);
        const float det = X[0] * C[0] + X[1] * C[1] + X[2] * C[2];
        for (int k = 0; k < 9; ++k) X[k] = 0.5f * (X[k] + C[k] / det);
    }
    if (dA < 0.0f) {
        float H[9], Q[9];
        for (int r = 0; r < 3; ++r)          // H = X^T A (symmetric factor)
            for (int cc = 0; cc < 3; ++cc)
                H[3 * r + cc] = X[r] * A[cc] + X[3 + r] * A[3 + cc] + X[6 + r] * A[6 + cc];
        for (int r = 0; r < 3; ++r)
            for (int cc = r + 1; cc < 3; ++cc) H[3 * r + cc] = H[3 * cc + r] = 0.5f * (H[3 * r + cc] + H[3 * cc + r]);
        sym_eig3(H, Q);
        int m = 0;
        if (H[4] < H[4 * m]) m = 1;
        if (H[8] < H[4 * m]) m = 2;
        const float w[3] = {Q[m], Q[3 + m], Q[6 + m]};
        const float Xw[3] = {X[0] * w[0] + X[1] * w[1] + X[2] * w[2], X[3] * w[0] + X[4] * w[1] + X[5] * w[2],
                             X[6] * w[0] + X[7] * w[1] + X[8] * w[2]};
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc) X[3 * r + cc] -= 2.0f * Xw[r] * w[cc];
    }
    for (int k = 0; k < 9; ++k) R[k] = X[k];
}

// omega = I^+ L for a symmetric positive semi-definite inertia tensor
// (xx, yy, zz, xy, xz, yz).  `scale` = max(trace I, M (2r)^2) sets what counts
// as zero: the inertia of a one-particle body is rounding noise, and a body
// whose particles lie on a line has one vanishing eigenvalue.  Well
// conditioned tensors use the closed-form inverse; otherwise an
// eigen-decomposition drops eigenvalues at or below 1e-6 * scale.
__device__ void solve_inertia(const float* I6, const float* L, float scale, float* w)
{
    const float I[9] = {I6[0], I6[3], I6[4], I6[3], I6[1], I6[5], I6[4], I6[5], I6[2]};
    w[0] = w[1] = w[2] = 0.0f;
    if (!(scale > 0.0f)) return;
    float C[9];
    cof3(I, C);
    const float det = I[0] * C[0] + I[1] * C[1] + I[2] * C[2];
    const float t3 = scale * (1.0f / 3.0f);
    if (det > 1e-3f * t3 * t3 * t3) {
        const float id = 1.0f / det;    // I^-1 = cof^T / det, cof symmetric here
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

// ---------------------------------------------------------------------------
// per-body reductions: wave butterfly, then a fixed-order sum over waves
// ---------------------------------------------------------------------------

template <int NV>
__device__ inline void block_sum(float (&v)[NV], float* red /* >= 5 * NV */)
{
    for (int j = 0; j < NV; ++j)
        for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        for (int j = 0; j < NV; ++j) red[wave * NV + j] = v[j];
    __syncthreads();
    if (threadIdx.x < NV) {
        const int j = threadIdx.x;
        red[4 * NV + j] = ((red[j] + red[NV + j]) + red[2 * NV + j]) + red[3 * NV + j];
    }
    __syncthreads();
    for (int j = 0; j < NV; ++j) v[j] = red[4 * NV + j];
    __syncthreads();
}

__device__ inline void cross(const float* a, const float* b, float* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// one Jacobi iteration (Alg. 1 loop body); one workgroup per body
// ---------------------------------------------------------------------------

template <int PPT>
__global__ void __launch_bounds__(kBlock) k_iterate(Scene s, StepConsts c, int src)
{
    __shared__ float red[5 * 24];
    __shared__ float bc[16];

    const int b = blockIdx.x;
    const int s0 = s.body_start[b], e0 = s.body_start[b + 1];
    const float M = s.body_mass[b];
    const float invM = 1.0f / M;
    const size_t n = (size_t)s.n;
    const float* dl = s.dl[src];
    const float* vl = s.vel[src];
    float* dn = s.dl[src ^ 1];
    float* vn = s.vel[src ^ 1];
    const float ax = s.x[s0], ay = s.x[n + s0], az = s.x[2 * n + s0];   // body anchor

    float y[PPT][3], del[PPT][3], V[PPT][3], q[PPT][3], m[PPT], x0[PPT][3];
    int idx[PPT];
    float acc[24];
    for (int j = 0; j < 3; ++j) acc[j] = 0.0f;
    for (int k = 0; k < PPT; ++k) {
        const int i = s0 + threadIdx.x + k * kBlock;
        idx[k] = i;
        if (i < e0) {
            for (int j = 0; j < 3; ++j) {
                x0[k][j] = s.x[j * n + i];
                del[k][j] = dl[j * n + i];
                V[k][j] = vl[j * n + i];
                q[k][j] = s.q[j * n + i];
            }
            m[k] = s.mass[i];
            y[k][0] = (x0[k][0] - ax) + del[k][0];
            y[k][1] = (x0[k][1] - ay) + del[k][1];
            y[k][2] = (x0[k][2] - az) + del[k][2];
        } else {
            for (int j = 0; j < 3; ++j) x0[k][j] = del[k][j] = V[k][j] = q[k][j] = y[k][j] = 0.0f;
            m[k] = 0.0f;
        }
        for (int j = 0; j < 3; ++j) acc[j] += m[k] * y[k][j];
    }
    // centre of mass of X_i (anchor frame)
    {
        float t3[3] = {acc[0], acc[1], acc[2]};
        block_sum<3>(t3, red);
        for (int j = 0; j < 3; ++j) acc[j] = t3[j] * invM;
    }
    const float cy[3] = {acc[0], acc[1], acc[2]};
    // covariance A = sum m (x - c) q^T
    float r[PPT][3];
    {
        float A[9];
        for (int j = 0; j < 9; ++j) A[j] = 0.0f;
        for (int k = 0; k < PPT; ++k) {
            for (int j = 0; j < 3; ++j) r[k][j] = y[k][j] - cy[j];
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) A[3 * a + bb] += m[k] * r[k][a] * q[k][bb];
        }
        block_sum<9>(A, red);
        if (threadIdx.x == 0) {
            float R[9];
            polar_rotation(A, R);
            for (int j = 0; j < 9; ++j) bc[j] = R[j];
        }
        __syncthreads();
    }
    float R[9];
    for (int j = 0; j < 9; ++j) R[j] = bc[j];

    // contacts, shape matching goal, and momentum partial sums
    float Cd[PPT][3], Dd[PPT][3];
    for (int j = 0; j < 24; ++j) acc[j] = 0.0f;
    for (int k = 0; k < PPT; ++k) {
        const int i = idx[k];
        for (int j = 0; j < 3; ++j) Cd[k][j] = Dd[k][j] = 0.0f;
        if (i >= e0) continue;
        // ground / planes (constraint (1)), friction from the displacement since X_init
        for (int pl = 0; pl < c.n_planes; ++pl) {
            const float nx = c.plane_n[pl][0], ny = c.plane_n[pl][1], nz = c.plane_n[pl][2];
            const float e = ((nx * x0[k][0] + ny * x0[k][1] + nz * x0[k][2]) - c.plane_d[pl]) +
                            (nx * del[k][0] + ny * del[k][1] + nz * del[k][2]);
            if (!(e < c.radius)) continue;
            const float pen = c.radius - e;
            const float un = nx * del[k][0] + ny * del[k][1] + nz * del[k][2];
            const float ux = del[k][0] - un * nx, uy = del[k][1] - un * ny, uz = del[k][2] - un * nz;
            const float ut = sqrtf(ux * ux + uy * uy + uz * uz);
            const float f = ut > 0.0f ? fminf(1.0f, c.mu * pen / ut) : 0.0f;
            Cd[k][0] += pen * nx - f * ux;
            Cd[k][1] += pen * ny - f * uy;
            Cd[k][2] += pen * nz - f * uz;
        }
        // particle-particle contacts (constraint (2)), symmetric averaging
        const uint32_t ni = s.nbr_n[i];
        const uint32_t cnt = ni < (uint32_t)c.nbr_cap ? ni : (uint32_t)c.nbr_cap;
        for (uint32_t sl = 0; sl < cnt; ++sl) {
            const uint32_t jq = s.nbr[sl * n + i];
            float d[3], u[3];
            for (int j = 0; j < 3; ++j) {
                const float dj = dl[j * n + jq];
                d[j] = (x0[k][j] - s.x[j * n + jq]) + (del[k][j] - dj);
                u[j] = del[k][j] - dj;
            }
            const float l2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const float l = sqrtf(l2);
            if (!(l > 0.0f) || !(l < c.two_r)) continue;
            const float il = 1.0f / l;
            const float nx = d[0] * il, ny = d[1] * il, nz = d[2] * il;
            const float pen = c.two_r - l;
            const float mq = s.mass[jq];
            const float alpha = mq / (m[k] + mq);          // w_p / (w_p + w_q)
            const float un = u[0] * nx + u[1] * ny + u[2] * nz;
            const float ux = u[0] - un * nx, uy = u[1] - un * ny, uz = u[2] - un * nz;
            const float ut = sqrtf(ux * ux + uy * uy + uz * uz);
            const float f = ut > 0.0f ? fminf(1.0f, c.mu * pen / ut) : 0.0f;
            float wgt = 1.0f;
            const uint32_t avg = (c.flags >> kAvgShift) & 3u;
            if (avg == 0u) {
                const uint32_t nq = s.nbr_n[jq];
                wgt = 1.0f / (float)(ni > nq ? ni : nq);
            } else if (avg == 1u) {
                wgt = 1.0f / (float)ni;
            }
            const float sc = alpha * wgt;
            Cd[k][0] += sc * (pen * nx - f * ux);
            Cd[k][1] += sc * (pen * ny - f * uy);
            Cd[k][2] += sc * (pen * nz - f * uz);
        }
        // shape matching: goal R q + c, i.e. D = R q - (x - c)
        for (int a = 0; a < 3; ++a)
            Dd[k][a] = (R[3 * a] * q[k][0] + R[3 * a + 1] * q[k][1] + R[3 * a + 2] * q[k][2]) - r[k][a];
        // momentum sums in the frame centred on c_i: z_b = r + C, z_a = z_b + D
        const float mk = m[k];
        float zb[3], za[3], vb[3], t[3];
        for (int j = 0; j < 3; ++j) {
            zb[j] = r[k][j] + Cd[k][j];
            za[j] = zb[j] + Dd[k][j];
            vb[j] = V[k][j] + Cd[k][j] * c.inv_h;
            acc[j] += mk * r[k][j];           // S0 = sum m r (rounding residual of c)
            acc[3 + j] += mk * Cd[k][j];      // S1 = sum m C
            acc[6 + j] += mk * Dd[k][j];      // S2 = sum m D
            acc[9 + j] += mk * vb[j];         // S3 = P_bsm
        }
        cross(zb, Dd[k], t);
        for (int j = 0; j < 3; ++j) acc[12 + j] += mk * t[j];     // S4 = sum m z_b x D
        cross(Dd[k], vb, t);
        for (int j = 0; j < 3; ++j) acc[15 + j] += mk * t[j];     // S5 = sum m D x v_b
        acc[18] += mk * (za[1] * za[1] + za[2] * za[2]);          // S6: inertia about c_i
        acc[19] += mk * (za[0] * za[0] + za[2] * za[2]);
        acc[20] += mk * (za[0] * za[0] + za[1] * za[1]);
        acc[21] -= mk * za[0] * za[1];
        acc[22] -= mk * za[0] * za[2];
        acc[23] -= mk * za[1] * za[2];
    }
    {
        float S[24];
        for (int j = 0; j < 24; ++j) S[j] = acc[j];
        block_sum<24>(S, red);
        if (threadIdx.x == 0) {
            float cb[3], Db[3], ca[3], dv[3] = {0.0f, 0.0f, 0.0f}, w[3] = {0.0f, 0.0f, 0.0f};
            for (int j = 0; j < 3; ++j) {
                cb[j] = (S[j] + S[3 + j]) * invM;    // c_bsm - c_i
                Db[j] = S[6 + j] * invM;             // mean shape-matching shift
                ca[j] = cb[j] + Db[j];               // c_asm - c_i
            }
            // Eq. (4): dv = (P_bsm - P_asm) / M,  P_asm - P_bsm = sum m D / dt
            if (!(c.flags & kFlagNoLinMom))
                for (int j = 0; j < 3; ++j) dv[j] = -S[6 + j] * c.inv_h * invM;
            // Eq. (5): omega = I^-1 (L_asm - L_bsm); the difference is formed from
            // the small quantities: (sum m r_b x D)/dt + sum m D x v_b - Db x P_bsm
            if (!(c.flags & kFlagNoAngMom)) {
                float cbxD[3], DbxP[3], dL[3], I6[6];
                cross(cb, &S[6], cbxD);
                cross(Db, &S[9], DbxP);
                for (int j = 0; j < 3; ++j) dL[j] = (S[12 + j] - cbxD[j]) * c.inv_h + S[15 + j] - DbxP[j];
                // parallel-axis shift of the inertia from c_i to c_asm
                I6[0] = S[18] - M * (ca[1] * ca[1] + ca[2] * ca[2]);
                I6[1] = S[19] - M * (ca[0] * ca[0] + ca[2] * ca[2]);
                I6[2] = S[20] - M * (ca[0] * ca[0] + ca[1] * ca[1]);
                I6[3] = S[21] + M * ca[0] * ca[1];
                I6[4] = S[22] + M * ca[0] * ca[2];
                I6[5] = S[23] + M * ca[1] * ca[2];
                const float scale = fmaxf(I6[0] + I6[1] + I6[2], M * c.two_r * c.two_r);
                solve_inertia(I6, dL, scale, w);
            }
            for (int j = 0; j < 3; ++j) {
                bc[j] = dv[j];
                bc[3 + j] = w[j];
                bc[6 + j] = ca[j];
            }
        }
        __syncthreads();
    }
    const float dv[3] = {bc[0], bc[1], bc[2]}, w[3] = {bc[3], bc[4], bc[5]}, ca[3] = {bc[6], bc[7], bc[8]};
    if (threadIdx.x == 0 && s.body_rot)
        for (int j = 0; j < 9; ++j) s.body_rot[9 * (size_t)b + j] = R[j];
    for (int k = 0; k < PPT; ++k) {
        const int i = idx[k];
        if (i >= e0) continue;
        float ra[3], wr[3];
        for (int j = 0; j < 3; ++j) ra[j] = r[k][j] + Cd[k][j] + Dd[k][j] - ca[j];
        cross(w, ra, wr);
        for (int j = 0; j < 3; ++j) {
            const float step = Cd[k][j] + Dd[k][j];
            const float dvi = dv[j] - wr[j];
            dn[j * n + i] = (del[k][j] + step) + c.h * dvi;
            if (c.flags & kFlagStdVelocity) {
                // standard PBD: V = (X_{i+1} - X_init) / dt in world FP32 coordinates
                const float xw = x0[k][j] + ((del[k][j] + step) + c.h * dvi);
                vn[j * n + i] = (xw - x0[k][j]) * c.inv_h;
            } else {
                vn[j * n + i] = (V[k][j] + step * c.inv_h) + dvi;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_finalize(Scene s, int src)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= s.n) return;
    const size_t n = (size_t)s.n;
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
        const size_t j = k * n + i;
        const float x = s.x[j] + s.dl[src][j];
        const float v = s.vel[src][j];
        finite = finite && isfinite(x) && isfinite(v);
        s.x[j] = x;
        s.v[j] = v;
    }
    if (!finite) atomicOr(&s.counters->err, kErrNonFinite);
}

__global__ void k_clear_counters(Counters* c)
{
    c->err = 0u;
    c->max_nbr = 0u;
    c->nbr_sum = 0ull;
    c->nbr_rows = 0ull;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t enqueue_clear_counters(const Scene& s, hipStream_t stream)
{
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(1), 0, stream, s.counters);
    return hipGetLastError();
}

namespace {
void launch_iterate(const Scene& s, const StepConsts& c, int ppt, int src, hipStream_t stream)
{
    switch (ppt) {
    case 1: hipLaunchKernelGGL(k_iterate<1>, dim3(s.nb), dim3(kBlock), 0, stream, s, c, src); break;
    case 2: hipLaunchKernelGGL(k_iterate<2>, dim3(s.nb), dim3(kBlock), 0, stream, s, c, src); break;
    default: hipLaunchKernelGGL(k_iterate<4>, dim3(s.nb), dim3(kBlock), 0, stream, s, c, src); break;
    }
}
}  // namespace

hipError_t enqueue_iterations(const Scene& s, const StepConsts& c, int ppt, int count, hipStream_t stream)
{
    if (s.n <= 0 || count <= 0) return hipSuccess;
    int src = 0;
    for (int it = 0; it < count; ++it) {
        launch_iterate(s, c, ppt, src, stream);
        src ^= 1;
    }
    return hipGetLastError();
}

hipError_t enqueue_substeps(const Scene& s, const StepConsts& c, int iterations, int ppt, int count,
                            hipStream_t stream)
{
    if (s.n <= 0 || count <= 0) return hipSuccess;
    const unsigned nb = blocks_for((size_t)s.n);
    const size_t nbr_lds = (size_t)c.nbr_cap * kBlock * sizeof(uint32_t);
    for (int sub = 0; sub < count; ++sub) {
        hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(s.T)), dim3(kBlock), 0, stream, s.cell_count, s.T, 0u);
        hipLaunchKernelGGL(k_predict_keys, dim3(nb), dim3(kBlock), 0, stream, s, c);
        hipLaunchKernelGGL(k_scan_tiles, dim3(s.n_scan_tiles), dim3(kBlock), 0, stream, s.cell_count, s.T,
                           s.tile_sums);
        hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kBlock), 0, stream, s.tile_sums, s.n_scan_tiles);
        hipLaunchKernelGGL(k_scan_write, dim3(s.n_scan_tiles), dim3(kBlock), 0, stream, s.cell_count, s.T,
                           s.tile_sums, s.cell_start);
        hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, stream, s);
        hipLaunchKernelGGL(k_neighbours, dim3(nb), dim3(kBlock), nbr_lds, stream, s, c);
        int src = 0;
        for (int it = 0; it < iterations; ++it) {
            launch_iterate(s, c, ppt, src, stream);
            src ^= 1;
        }
        hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(kBlock), 0, stream, s, src);
    }
    return hipGetLastError();
}

}  // namespace pbdr
