// fmm_near.hip -- evaluation step (Section 2.2): for every particle the far
// field from its leaf's local expansion (L2P) plus the near field summed
// directly over the leaf and its touching leaves (P2P) with the Gaussian
// regularised kernel of eq. 8, written out as the velocity of eq. 9 in the
// caller's order.
//
// Complex form: phi(z_i) = sum_j gamma_j (1 - exp(-|z_i - z_j|^2 / 2 sigma^2))
// / (z_i - z_j) over near pairs, plus L2P; u = Im(phi)/(2 pi), v = Re(phi)/(2 pi).
// Zero-distance pairs contribute nothing.
//
// One wavefront per target leaf.  The sources of the 3 x 3 neighbourhood are
// staged through LDS in chunks with coalesced loads (each leaf's particles are
// contiguous in the sorted arrays); each lane owns one target and one of S
// interleaved slices of the staged sources, S = 64 / (targets rounded up to a
// power of two), and the S partial sums are combined with cross-lane
// shuffles.  Leaves with more than 64 particles are walked in target chunks.
//
// FP64: 1 - exp(-t) and the reciprocal are evaluated inline (polynomial and
// Newton-refined hardware estimate) instead of library calls.
//
// Mixed precision: sources and targets are FP32 offsets from their own leaf
// centre in leaf-width units; a source's leaf offset (-1, 0 or +1 per axis)
// is added when it is staged, so every difference is taken between numbers
// of magnitude <= 1.5 and keeps ~1e-7 relative accuracy (absolute FP32
// coordinates in the unit square would lose three more digits).  The
// exponential is 2^x on the hardware transcendental unit and the reciprocal
// the hardware reciprocal; accumulation is FP32 per lane.  The far field (L2P)
// stays FP64.
#include "fmm_device.h"

namespace fmm {
namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251;
constexpr int kStage = 256;   // sources staged per chunk

struct Src64 { double x, y, g; };

// ln 2 split into its nearest double and the remainder (for the reduction
// t = k ln2 - r done with fused multiply-adds).
constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;
constexpr double kLog2E = 1.4426950408889634;

// 1 - exp(-t) for t >= 0 in FP64, within a few ulp for every t.  Reduce
// t = k ln2 - r with |r| <= ln2/2 (Cody and Waite), take expm1(r) from its
// Taylor series to r^14 (remainder below 1e-18 relative), and use
//   1 - e^-t = (1 - 2^-k) - 2^-k expm1(r),
// which is -expm1(-t) itself for k = 0 and free of cancellation for k >= 1.
// Beyond t = 37 the result rounds to 1, so t is clamped at 40.
__device__ __forceinline__ double one_minus_exp_neg(double t)
{
    t = fmin(t, 40.0);
    const double k = rint(t * kLog2E);
    double r = fma(k, kLn2Hi, -t);
    r = fma(k, kLn2Lo, r);
    double q = 1.1470745597729725e-11;      // 1/14!
    q = fma(q, r, 1.6059043836821613e-10);  // 1/13!
    q = fma(q, r, 2.08767569878681e-09);
    q = fma(q, r, 2.505210838544172e-08);
    q = fma(q, r, 2.755731922398589e-07);
    q = fma(q, r, 2.7557319223985893e-06);
    q = fma(q, r, 2.48015873015873e-05);
    q = fma(q, r, 0.0001984126984126984);
    q = fma(q, r, 0.001388888888888889);
    q = fma(q, r, 0.008333333333333333);
    q = fma(q, r, 0.041666666666666664);
    q = fma(q, r, 0.16666666666666666);
    q = fma(q, r, 0.5);
    q = fma(q, r, 1.0);
    const double em = q * r;                // expm1(r)
    const double s = ldexp(1.0, -int(k));   // 2^-k, exact
    return fma(-s, em, 1.0 - s);
}

// 1/x for a positive normal x: hardware estimate and two Newton steps.
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

template <int P, bool MIXED>
__global__ void __launch_bounds__(64)
k_p2p_l2p(int L, int p, int has_far, const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
          const double* __restrict__ ys, const double* __restrict__ gs, const float4* __restrict__ pk,
          const uint32_t* __restrict__ perm, const cd* __restrict__ le_leaf, const Domain* __restrict__ dom,
          double inv2s2, double* __restrict__ u, double* __restrict__ v)
{
    const uint32_t m = blockIdx.x;
    const int s0 = leaf_start[m];
    const int nt = leaf_start[m + 1] - s0;
    if (nt == 0) return;
    const int a = int(morton_x(m)), b = int(morton_y(m)), side = 1 << L;
    const int lane = threadIdx.x;

    // the 3 x 3 neighbourhood, row by row; clipped leaves are empty
    int nbeg[9], npre[10];
    npre[0] = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int na = a + (q % 3) - 1, nb = b + (q / 3) - 1;
        int cnt = 0, beg = 0;
        if (na >= 0 && nb >= 0 && na < side && nb < side) {
            const uint32_t sm = morton(uint32_t(na), uint32_t(nb));
            beg = leaf_start[sm];
            cnt = leaf_start[sm + 1] - beg;
        }
        nbeg[q] = beg;
        npre[q + 1] = npre[q] + cnt;
    }
    const int tot = npre[9];

    const int lgT = nt >= 64 ? 6 : (nt <= 1 ? 0 : 32 - __clz(nt - 1));
    const int T = 1 << lgT;
    const int S = 64 >> lgT;
    const int ti = lane & (T - 1);
    const int si = lane >> lgT;

    const Domain d = *dom;
    const double w = ldexp(d.W, -L);
    const double cx = d.x0 + (double(a) + 0.5) * w;
    const double cy = d.y0 + (double(b) + 0.5) * w;
    // leaf-width units: |z|^2 / (2 sigma^2) = |zhat|^2 w^2 / (2 sigma^2), and
    // exp(-t) = 2^(-t log2(e)); w = 1/s
    const float c2 = float(inv2s2 * 1.4426950408889634074 / (d.s * d.s));

    using Stage = typename std::conditional<MIXED, float4, Src64>::type;
    __shared__ Stage src[kStage];

    for (int c0 = 0; c0 < nt; c0 += T) {
        const int i = c0 + ti;
        const bool act = i < nt;
        const int ip = s0 + (act ? i : 0);
        double xi = 0.0, yi = 0.0;
        float oxi = 0.f, oyi = 0.f;
        if constexpr (MIXED) {
            const float4 t = pk[ip];
            oxi = t.x; oyi = t.y;
        } else {
            xi = xs[ip]; yi = ys[ip];
        }
        double acc_x = 0.0, acc_y = 0.0;
        float facc_x = 0.f, facc_y = 0.f;

        for (int base = 0; base < tot; base += kStage) {
            const int cnt = min(kStage, tot - base);
            __syncthreads();
            for (int k = lane; k < cnt; k += 64) {
                const int idx = base + k;
                int q = 0;
#pragma unroll
                for (int r = 1; r < 9; ++r) q += (idx >= npre[r]) ? 1 : 0;
                const int j = nbeg[q] + (idx - npre[q]);
                if constexpr (MIXED) {
                    float4 t = pk[j];
                    t.x += float((q % 3) - 1);   // source position relative to the target leaf centre
                    t.y += float((q / 3) - 1);
                    src[k] = t;
                } else {
                    src[k] = Src64{xs[j], ys[j], gs[j]};
                }
            }
            __syncthreads();
            if constexpr (MIXED) {
                for (int jj = si; jj < cnt; jj += S) {
                    const float4 t = src[jj];
                    const float dx = oxi - t.x, dy = oyi - t.y;
                    const float r2 = fmaf(dx, dx, dy * dy);
                    const float e = __builtin_amdgcn_exp2f(-r2 * c2);
                    const float q = t.z * (1.0f - e) * __builtin_amdgcn_rcpf(fmaxf(r2, 1e-30f));
                    facc_x = fmaf(q, dx, facc_x);
                    facc_y = fmaf(-q, dy, facc_y);
                }
            } else {
                for (int jj = si; jj < cnt; jj += S) {
                    const Src64 t = src[jj];
                    const double dx = xi - t.x, dy = yi - t.y;
                    const double r2 = fma(dx, dx, dy * dy);
                    const double f = one_minus_exp_neg(r2 * inv2s2);
                    const double q = r2 > 0.0 ? t.g * f * recip(r2) : 0.0;
                    acc_x = fma(q, dx, acc_x);
                    acc_y = fma(-q, dy, acc_y);
                }
            }
        }

        if constexpr (MIXED) {
            for (int off = T; off < 64; off <<= 1) {
                facc_x += __shfl_xor(facc_x, off, 64);
                facc_y += __shfl_xor(facc_y, off, 64);
            }
            acc_x = double(facc_x) * d.s;   // leaf units -> physical: 1/(w z) = s/z
            acc_y = double(facc_y) * d.s;
        } else {
            for (int off = T; off < 64; off <<= 1) {
                acc_x += __shfl_xor(acc_x, off, 64);
                acc_y += __shfl_xor(acc_y, off, 64);
            }
        }

        if (si == 0 && act) {
            if (has_far) {
                if constexpr (MIXED) { xi = xs[ip]; yi = ys[ip]; }
                const double zx = (xi - cx) * d.s, zy = (yi - cy) * d.s;
                const cd* bl = le_leaf + int64_t(m) * p;
                double fx = 0.0, fy = 0.0;
#pragma unroll
                for (int k = P - 1; k >= 0; --k) {
                    if (k < p) {
                        const cd t = bl[k];
                        const double nx = fx * zx - fy * zy + t.x;
                        fy = fx * zy + fy * zx + t.y;
                        fx = nx;
                    }
                }
                acc_x += fx * d.s;
                acc_y += fy * d.s;
            }
            const uint32_t o = perm[ip];
            u[o] = acc_y * kInv2Pi;
            v[o] = acc_x * kInv2Pi;
        }
    }
}

template <int P>
hipError_t p2p_impl(const Buffers& b, int p, int L, bool has_far, bool mixed, double sigma, double* u,
                    double* v, hipStream_t st)
{
    const int64_t nleaf = int64_t(1) << (2 * L);
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    const cd* le_leaf = b.le + level_offset(L) * p;
    if (mixed) {
        hipLaunchKernelGGL((k_p2p_l2p<P, true>), dim3(unsigned(nleaf)), dim3(64), 0, st, L, p, has_far ? 1 : 0,
                           b.leaf_start, b.xs, b.ys, b.gs, b.pk, b.perm, le_leaf, b.dom, inv2s2, u, v);
    } else {
        hipLaunchKernelGGL((k_p2p_l2p<P, false>), dim3(unsigned(nleaf)), dim3(64), 0, st, L, p, has_far ? 1 : 0,
                           b.leaf_start, b.xs, b.ys, b.gs, b.pk, b.perm, le_leaf, b.dom, inv2s2, u, v);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_p2p(const Buffers& b, int P, int p, int L, bool has_far, bool mixed, double sigma,
                      double* u, double* v, hipStream_t st)
{
    switch (P) {
        case 8: return p2p_impl<8>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 12: return p2p_impl<12>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 16: return p2p_impl<16>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 17: return p2p_impl<17>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 20: return p2p_impl<20>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 24: return p2p_impl<24>(b, p, L, has_far, mixed, sigma, u, v, st);
        case 32: return p2p_impl<32>(b, p, L, has_far, mixed, sigma, u, v, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fmm
