// fmm_upward.hip -- upward sweep (Section 2.2, Fig. 2): P2M at the leaves and
// M2M from every level to its parent level.
//
// Coefficients are scaled by the box width w_l so that the shift operators do
// not depend on the level: for a box of centre c,
//   ahat_k = sum_j gamma_j ((z_j - c) / w_l)^k,        k = 0 .. p-1,
// which is the textbook multipole expansion of 1/z, phi(z) = sum_k a_k /
// (z - c)^(k+1), with a_k = ahat_k w_l^k.  The M2M shift from a child in
// position c (delta = (c_child - c_parent) / w_parent = (+-1 +- i)/4) reads
//   ahat^P_k = sum_{m<=k} C(k,m) 2^-m delta^(k-m) ahat^child_m,
// one of four fixed lower-triangular matrices built on the host.
#include "fmm_device.h"

namespace fmm {
namespace {

// One thread per leaf: sum over the leaf's particles with incremental powers.
template <int P>
__global__ void __launch_bounds__(256)
k_p2m(int L, int p, const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
      const double* __restrict__ ys, const double* __restrict__ gs, const Domain* __restrict__ dom,
      cd* __restrict__ me_leaf)
{
    const int64_t nleaf = int64_t(1) << (2 * L);
    const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m >= nleaf) return;
    const Domain d = *dom;
    const double w = ldexp(d.W, -L);
    const double cx = d.x0 + (double(morton_x(uint32_t(m))) + 0.5) * w;
    const double cy = d.y0 + (double(morton_y(uint32_t(m))) + 0.5) * w;
    double ax[P], ay[P];
#pragma unroll
    for (int k = 0; k < P; ++k) { ax[k] = 0.0; ay[k] = 0.0; }
    const int s0 = leaf_start[m], s1 = leaf_start[m + 1];
    for (int q = s0; q < s1; ++q) {
        const double zx = (xs[q] - cx) * d.s, zy = (ys[q] - cy) * d.s;
        double px = gs[q], py = 0.0;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            ax[k] += px;
            ay[k] += py;
            const double t = px * zx - py * zy;
            py = px * zy + py * zx;
            px = t;
        }
    }
    cd* out = me_leaf + m * p;
#pragma unroll
    for (int k = 0; k < P; ++k)
        if (k < p) out[k] = cd{ax[k], ay[k]};
}

// One thread per parent box at level l: four children at level l+1.
template <int P>
__global__ void __launch_bounds__(256)
k_m2m(int64_t nparent, int p, const cd* __restrict__ child, cd* __restrict__ parent, const cd* __restrict__ M)
{
    const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (m >= nparent) return;
    double bx[P], by[P];
#pragma unroll
    for (int k = 0; k < P; ++k) { bx[k] = 0.0; by[k] = 0.0; }
    for (int c = 0; c < 4; ++c) {
        const cd* src = child + (4 * m + c) * p;
        double ax[P], ay[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k < p) { const cd t = src[k]; ax[k] = t.x; ay[k] = t.y; }
            else { ax[k] = 0.0; ay[k] = 0.0; }
        }
        const cd* Mc = M + c * P * P;
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int j = 0; j <= k; ++j) {
                const cd t = Mc[k * P + j];
                cmac(bx[k], by[k], t.x, t.y, ax[j], ay[j]);
            }
        }
    }
    cd* dst = parent + m * p;
#pragma unroll
    for (int k = 0; k < P; ++k)
        if (k < p) dst[k] = cd{bx[k], by[k]};
}

template <int P>
hipError_t p2m_impl(const Buffers& b, int p, int L, hipStream_t st)
{
    const int64_t nleaf = int64_t(1) << (2 * L);
    hipLaunchKernelGGL(k_p2m<P>, dim3(unsigned((nleaf + 255) / 256)), dim3(256), 0, st, L, p, b.leaf_start,
                       b.xs, b.ys, b.gs, b.dom, b.me + level_offset(L) * p);
    return hipGetLastError();
}

template <int P>
hipError_t m2m_impl(const Buffers& b, int p, int l, hipStream_t st)
{
    const int64_t np = int64_t(1) << (2 * l);
    hipLaunchKernelGGL(k_m2m<P>, dim3(unsigned((np + 255) / 256)), dim3(256), 0, st, np, p,
                       b.me + level_offset(l + 1) * p, b.me + level_offset(l) * p, b.t_m2m);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_p2m(const Buffers& b, int P, int p, int L, hipStream_t st)
{
#define CALL_P2M(PP) p2m_impl<PP>(b, p, L, st)
    switch (P) {
        case 8: return CALL_P2M(8);
        case 12: return CALL_P2M(12);
        case 16: return CALL_P2M(16);
        case 17: return CALL_P2M(17);
        case 20: return CALL_P2M(20);
        case 24: return CALL_P2M(24);
        case 32: return CALL_P2M(32);
        default: return hipErrorInvalidValue;
    }
#undef CALL_P2M
}

hipError_t launch_m2m(const Buffers& b, int P, int p, int l, hipStream_t st)
{
#define CALL_M2M(PP) m2m_impl<PP>(b, p, l, st)
    switch (P) {
        case 8: return CALL_M2M(8);
        case 12: return CALL_M2M(12);
        case 16: return CALL_M2M(16);
        case 17: return CALL_M2M(17);
        case 20: return CALL_M2M(20);
        case 24: return CALL_M2M(24);
        case 32: return CALL_M2M(32);
        default: return hipErrorInvalidValue;
    }
#undef CALL_M2M
}

}  // namespace fmm
