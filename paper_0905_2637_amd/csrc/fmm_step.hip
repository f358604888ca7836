// fmm_step.hip -- the particle update of the vortex-method time stepping
// (Section 3, eq. 6: in ideal 2D flow the particles move with the local
// velocity and keep their circulation).  The explicit midpoint rule
//   x_mid = x_n + dt/2 u(x_n),   x_n+1 = x_n + dt u(x_mid)
// needs one update of the form (xo, yo) = (x, y) + c (u, v) per stage; the
// velocities come from full FMM evaluations (fmm_api.cpp enqueues them).
#include "fmm_device.h"

namespace fmm {
namespace {

constexpr int kStepThreads = 256;
constexpr int kStepPer = 4;        // elements per thread

// HBM-bound: 32 B read and 16 B written per particle.
__global__ void __launch_bounds__(kStepThreads)
k_advance(int64_t n, const double* x, const double* y, const double* __restrict__ u,
          const double* __restrict__ v, double c, double* xo, double* yo)
{
    const int64_t base = int64_t(blockIdx.x) * (kStepThreads * kStepPer) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < kStepPer; ++r) {
        const int64_t i = base + int64_t(r) * kStepThreads;
        if (i < n) {
            const double xn = x[i] + c * u[i];
            const double yn = y[i] + c * v[i];
            xo[i] = xn;          // xo may alias x (in-place update): read before write per element
            yo[i] = yn;
        }
    }
}

}  // namespace

// a = b = 0 over n entries (a fill kernel rather than a memset node, so that
// a caller may capture it into a graph)
__global__ void __launch_bounds__(kStepThreads) k_zero2(int64_t n, double* a, double* b)
{
    const int64_t base = int64_t(blockIdx.x) * (kStepThreads * kStepPer) + threadIdx.x;
#pragma unroll
    for (int r = 0; r < kStepPer; ++r) {
        const int64_t i = base + int64_t(r) * kStepThreads;
        if (i < n) {
            a[i] = 0.0;
            b[i] = 0.0;
        }
    }
}

hipError_t launch_zero2(int64_t n, double* a, double* b, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t per_block = int64_t(kStepThreads) * kStepPer;
    hipLaunchKernelGGL(k_zero2, dim3(unsigned((n + per_block - 1) / per_block)), dim3(kStepThreads), 0, st, n, a, b);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t n, const double* x, const double* y, const double* u, const double* v, double c,
                          double* xo, double* yo, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t per_block = int64_t(kStepThreads) * kStepPer;
    hipLaunchKernelGGL(k_advance, dim3(unsigned((n + per_block - 1) / per_block)), dim3(kStepThreads), 0, st, n, x,
                       y, u, v, c, xo, yo);
    return hipGetLastError();
}

}  // namespace fmm
