// Per-body state of a single scene for pbdr_scene_read_bodies: centre of
// mass, the rotation of shape matching for the current pose (Sec. III-C),
// and linear and angular momentum about the centre (the quantities of the
// momentum constraint, Eqs. (4)-(5)).  One workgroup per body, FP64 sums in
// a fixed order.
#include "pbdr_math.h"
#include "pbdr_state.h"

namespace pbdr {
namespace {

using namespace dev;

// Sum of `cnt` FP64 values over the workgroup in a fixed order (butterfly
// within each wave, then waves in order); every thread receives the sums.
template <int cnt>
__device__ inline void block_sum_f64(double* a, double (*red)[cnt])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < cnt; ++k)
        for (int off = 32; off > 0; off >>= 1) a[k] += __shfl_xor(a[k], off, 64);
    if (lane == 0)
        for (int k = 0; k < cnt; ++k) red[wave][k] = a[k];
    __syncthreads();
    for (int k = 0; k < cnt; ++k) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) t += red[w][k];
        a[k] = t;
    }
    __syncthreads();
}

// Per-body state of the current (x, v), one workgroup per body, FP64 sums:
// centre of mass, the rotation of shape matching for this pose (the proper
// rotation maximising tr(R^T A), A = sum m (x - c) q^T against the rest
// offsets q, Sec. III-C), linear momentum and angular momentum about the
// centre.  out[18 b ..]: c (3), R row-major (9), P (3), L (3).
__global__ void __launch_bounds__(kBlock) k_body_state(Scene s, double* out)
{
    __shared__ double red[kBlock / 64][16];
    const int b = blockIdx.x;
    const int p0 = s.body_start[b], p1 = s.body_start[b + 1];
    const size_t N = (size_t)s.n;
    double m1[4] = {0.0, 0.0, 0.0, 0.0};
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kBlock) {
        const double m = s.mass[p];
        m1[0] += m;
        for (int a = 0; a < 3; ++a) m1[1 + a] += m * (double)s.x[a * N + p];
    }
    block_sum_f64<4>(m1, reinterpret_cast<double (*)[4]>(&red[0][0]));
    const double c[3] = {m1[1] / m1[0], m1[2] / m1[0], m1[3] / m1[0]};
    double t[15];
    for (int k = 0; k < 15; ++k) t[k] = 0.0;
    for (int p = p0 + (int)threadIdx.x; p < p1; p += kBlock) {
        const double m = s.mass[p];
        double r[3], q[3], v[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = (double)s.x[a * N + p] - c[a];
            q[a] = s.q[a * N + p];
            v[a] = s.v[a * N + p];
        }
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 3; ++j) t[3 * a + j] += m * r[a] * q[j];
        for (int a = 0; a < 3; ++a) t[9 + a] += m * v[a];
        t[12] += m * (r[1] * v[2] - r[2] * v[1]);
        t[13] += m * (r[2] * v[0] - r[0] * v[2]);
        t[14] += m * (r[0] * v[1] - r[1] * v[0]);
    }
    block_sum_f64<15>(t, reinterpret_cast<double (*)[15]>(&red[0][0]));
    if (threadIdx.x == 0) {
        double scale = 0.0;
        for (int k = 0; k < 9; ++k) scale = fmax(scale, fabs(t[k]));
        float A[9], R[9];
        for (int k = 0; k < 9; ++k) A[k] = scale > 0.0 ? (float)(t[k] / scale) : 0.0f;
        polar_rotation(A, R);
        double* o = out + 18 * (size_t)b;
        for (int a = 0; a < 3; ++a) o[a] = c[a];
        for (int k = 0; k < 9; ++k) o[3 + k] = R[k];
        for (int a = 0; a < 6; ++a) o[12 + a] = t[9 + a];
    }
}

}  // namespace

hipError_t enqueue_body_state(const Scene& s, double* out, hipStream_t stream)
{
    if (s.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_body_state, dim3(s.nb), dim3(kBlock), 0, stream, s, out);
    return hipGetLastError();
}

}  // namespace pbdr
