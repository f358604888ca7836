// fmm_fgt.hip -- the fast Gauss transform on the quadtree's leaf boxes
// (Section 8 names the fast Gauss transform among the transforms the library
// should take next):
//   G(y_i) = sum_j q_j exp(-|y_i - x_j|^2 / delta),   delta = 2 sigma^2,
// at the particles (the term j = i included), by the published algorithm of
// Greengard and Strain (SIAM J. Sci. Stat. Comput. 12, 1991):
//   P2H  every leaf box B: A_a = sum_j q_j s1^a1 s2^a2 / (a1! a2!),
//        s = (x_j - c_B) / sqrt(delta), a1, a2 < p (its Hermite expansion);
//   H2T  every leaf box C, from every box B within Chebyshev box distance nc:
//        B_b += sum_a A_a h_{a1+b1}(tau1) h_{a2+b2}(tau2),
//        tau = (c_C - c_B) / sqrt(delta), h_n the Hermite functions;
//   T2P  G(y) = sum_b B_b (-1)^(b1+b2) u1^b1 u2^b2 / (b1! b2!),
//        u = (y - c_C) / sqrt(delta) (the Taylor expansion about c_C).
// The box offsets are integers, so tau takes the values d w / sqrt(delta),
// |d| <= nc, and the h_n(tau) form one small table (built on the host).
// H2T is the matrix product Hx^T A Hy per box pair, done as two passes of
// fused multiply-adds: a lane owns one or two output rows b1, forms C_b1,a2 =
// sum_a1 h_{a1+b1}(tau1) A_a1a2, then adds sum_a2 C_b1,a2 h_{a2+b2}(tau2)
// to B_b1b2.  With few
// boxes the rows of the range are split over up to 8 workgroup rows, each
// writing a partial expansion; a fixed-order sum joins them.
#include "fmm_device.h"

namespace fmm {
namespace {

constexpr int kFgtThreads = 256;

// Lanes of a wavefront in groups of P, one group per box; the 64 / P groups of
// a wavefront take consecutive boxes.
template <int P>
struct Groups {
    static constexpr int kPerWave = 64 / P;
    static constexpr int kPerBlock = kPerWave * (kFgtThreads / 64);
};

__device__ __forceinline__ double box_centre(uint32_t k, double o, double w)
{
    return o + (double(k) + 0.5) * w;
}

// P2H: lane (box, a1) accumulates A_{a1, a2} for every a2, then scales by
// 1/(a1! a2!) (zero for terms >= p, which the table fk holds).
template <int P>
__global__ void __launch_bounds__(kFgtThreads)
k_p2h(int L, const Inst* __restrict__ inst, const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
      const double* __restrict__ ys, const double* __restrict__ gs, const double* __restrict__ fk, double rsd,
      double* __restrict__ A)
{
    using G = Groups<P>;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / P, a1 = lane % P;
    if (grp >= G::kPerWave) return;
    const int64_t m = int64_t(blockIdx.x) * G::kPerBlock + wv * G::kPerWave + grp;
    if (m >= (int64_t(1) << (2 * L))) return;
    const Domain d = inst[0].dom;
    const double w = ldexp(d.W, -L);
    const double cx = box_centre(morton_x(uint32_t(m)), d.x0, w);
    const double cy = box_centre(morton_y(uint32_t(m)), d.y0, w);
    double acc[P];
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = 0.0;
    const int j0 = leaf_start[m], j1 = leaf_start[m + 1];
    for (int j = j0; j < j1; ++j) {
        const double s1 = (xs[j] - cx) * rsd, s2 = (ys[j] - cy) * rsd;
        double t = gs[j];
        for (int k = 0; k < a1; ++k) t *= s1;       // q s1^a1
#pragma unroll
        for (int k = 0; k < P; ++k) {
            acc[k] += t;
            t *= s2;
        }
    }
    double* dst = A + m * (P * P) + a1 * P;
    const double f1 = fk[a1];
#pragma unroll
    for (int k = 0; k < P; ++k) dst[k] = acc[k] * f1 * fk[k];
}

// H2T lanes: R output rows b1 per lane (each coefficient of A a lane loads
// then feeds R multiply-adds), P / R lanes per box.
template <int P>
struct H2TGroups {
    static constexpr int kRows = P <= 12 ? 2 : 1;
    static constexpr int kLanes = P / kRows;
    static constexpr int kPerWave = 64 / kLanes;
    static constexpr int kPerBlock = kPerWave * (kFgtThreads / 64);
};

// H2T: lane (box, rows b1 = q, q + P/R, ...).  The table ht holds h_n(d w /
// sqrt(delta)) at [(d + nc) (2P - 1) + n]: the lane-dependent Hx values come
// from an LDS copy, the Hy values (the same for the whole workgroup: they
// depend on the row offset db only) straight from memory through scalar
// loads.  Stage 1 forms C_b1,a2 = sum_a1 h_{a1+b1}(tau1) A_a1a2, stage 2 adds
// sum_a2 C_b1,a2 h_{a2+b2}(tau2) to B_b1b2.
template <int P>
__global__ void __launch_bounds__(kFgtThreads)
k_h2t(int L, int nc, const double* __restrict__ A, const double* __restrict__ ht, const double* __restrict__ fk,
      double* __restrict__ B)
{
    using G = H2TGroups<P>;
    constexpr int R = G::kRows, NH = 2 * P - 1;
    // this workgroup row's share of the range's rows db
    const int rows = 2 * nc + 1, per = (rows + int(gridDim.y) - 1) / int(gridDim.y);
    const int db0 = -nc + int(blockIdx.y) * per, db1 = min(nc, db0 + per - 1);
    extern __shared__ double sht[];
    const int nt = rows * NH;
    for (int e = threadIdx.x; e < nt; e += kFgtThreads) sht[e] = ht[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / G::kLanes, q = lane % G::kLanes;
    const int side = 1 << L;
    const int64_t m = int64_t(blockIdx.x) * G::kPerBlock + wv * G::kPerWave + grp;
    if (grp >= G::kPerWave || m >= int64_t(side) * side) return;
    const int ca = int(morton_x(uint32_t(m))), cb = int(morton_y(uint32_t(m)));
    double acc[R][P];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k = 0; k < P; ++k) acc[r][k] = 0.0;
    for (int db = db0; db <= db1; ++db) {
        const int sb = cb - db;
        if (sb < 0 || sb >= side) continue;
        const double* hy = ht + (db + nc) * NH;
        for (int da = -nc; da <= nc; ++da) {
            const int sa = ca - da;
            if (sa < 0 || sa >= side) continue;
            const double* hx = sht + (da + nc) * NH + q;
            const double* As = A + int64_t(morton(uint32_t(sa), uint32_t(sb))) * (P * P);
            double c[R][P];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < P; ++k) c[r][k] = 0.0;
#pragma unroll
            for (int a1 = 0; a1 < P; ++a1) {
                double h[R];
#pragma unroll
                for (int r = 0; r < R; ++r) h[r] = hx[a1 + r * G::kLanes];
#pragma unroll
                for (int a2 = 0; a2 < P; ++a2) {
                    const double av = As[a1 * P + a2];
#pragma unroll
                    for (int r = 0; r < R; ++r) c[r][a2] = fma(av, h[r], c[r][a2]);
                }
            }
#pragma unroll
            for (int b2 = 0; b2 < P; ++b2) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double s = acc[r][b2];
#pragma unroll
                    for (int a2 = 0; a2 < P; ++a2) s = fma(c[r][a2], hy[a2 + b2], s);
                    acc[r][b2] = s;
                }
            }
        }
    }
    // (-1)^(b1+b2) / (b1! b2!), zero for terms >= p; partial expansion blockIdx.y
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int b1 = q + r * G::kLanes;
        double* dst = B + (int64_t(blockIdx.y) * side * side + m) * (P * P) + b1 * P;
        const double f1 = (b1 & 1) ? -fk[b1] : fk[b1];
#pragma unroll
        for (int b2 = 0; b2 < P; ++b2) dst[b2] = acc[r][b2] * ((b2 & 1) ? -f1 : f1) * fk[b2];
    }
}

// Partial expansions 1 .. parts-1 added to partial 0, in that order.
__global__ void __launch_bounds__(kFgtThreads) k_fgt_join(int64_t len, int parts, double* __restrict__ B)
{
    const int64_t e = int64_t(blockIdx.x) * kFgtThreads + threadIdx.x;
    if (e >= len) return;
    double s = B[e];
    for (int g = 1; g < parts; ++g) s += B[int64_t(g) * len + e];
    B[e] = s;
}

// T2P: one particle (or target point) per thread in sorted order, G to its
// input position; v is cleared.
template <int P>
__global__ void __launch_bounds__(kFgtThreads)
k_t2p(int n, int L, const Inst* __restrict__ inst, const uint32_t* __restrict__ ksorted,
      const double* __restrict__ xs, const double* __restrict__ ys, const uint32_t* __restrict__ perm,
      const double* __restrict__ Bc, double rsd, double* __restrict__ u, double* __restrict__ v)
{
    const int i = blockIdx.x * kFgtThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t m = ksorted[i];                 // single instance: the key is the leaf
    const Domain d = inst[0].dom;
    const double w = ldexp(d.W, -L);
    const double u1 = (xs[i] - box_centre(morton_x(m), d.x0, w)) * rsd;
    const double u2 = (ys[i] - box_centre(morton_y(m), d.y0, w)) * rsd;
    const double* b = Bc + int64_t(m) * (P * P);
    double acc = 0.0;
#pragma unroll
    for (int b1 = P - 1; b1 >= 0; --b1) {
        double r = 0.0;
#pragma unroll
        for (int b2 = P - 1; b2 >= 0; --b2) r = fma(r, u2, b[b1 * P + b2]);
        acc = fma(acc, u1, r);
    }
    const uint32_t o = perm[i];
    u[o] = acc;
    v[o] = 0.0;
}

template <int P>
hipError_t fgt_impl(const Buffers& b, int n, int L, double sigma, int nc, int parts, int m, double* u, double* v,
                    hipStream_t st)
{
    using G = Groups<P>;
    using H = H2TGroups<P>;
    const int64_t nbox = int64_t(1) << (2 * L);
    const double rsd = 1.0 / std::sqrt(2.0 * sigma * sigma);
    const unsigned gx = unsigned((nbox + G::kPerBlock - 1) / G::kPerBlock);
    hipLaunchKernelGGL(k_p2h<P>, dim3(gx), dim3(kFgtThreads), 0, st, L, b.inst, b.leaf_start, b.xs, b.ys, b.gs,
                       b.t_sout, rsd, b.fgt_a);
    const size_t lds = sizeof(double) * size_t(2 * nc + 1) * (2 * P - 1);
    const unsigned hx = unsigned((nbox + H::kPerBlock - 1) / H::kPerBlock);
    hipLaunchKernelGGL(k_h2t<P>, dim3(hx, unsigned(parts)), dim3(kFgtThreads), lds, st, L, nc, b.fgt_a, b.fgt_h,
                       b.t_sout, b.fgt_b);
    if (parts > 1) {
        const int64_t len = nbox * P * P;
        hipLaunchKernelGGL(k_fgt_join, dim3(unsigned((len + kFgtThreads - 1) / kFgtThreads)), dim3(kFgtThreads), 0,
                           st, len, parts, b.fgt_b);
    }
    if (m > 0)   // at the sorted target points
        hipLaunchKernelGGL(k_t2p<P>, dim3(unsigned((m + kFgtThreads - 1) / kFgtThreads)), dim3(kFgtThreads), 0, st,
                           m, L, b.inst, b.tks, b.txs, b.tys, b.tperm, b.fgt_b, rsd, u, v);
    else
        hipLaunchKernelGGL(k_t2p<P>, dim3(unsigned((n + kFgtThreads - 1) / kFgtThreads)), dim3(kFgtThreads), 0, st,
                           n, L, b.inst, b.ksorted, b.xs, b.ys, b.perm, b.fgt_b, rsd, u, v);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fgt(const Buffers& b, int P, int n, int L, double sigma, int nc, int parts, int m, double* u,
                      double* v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (parts < 1 || parts > 2 * nc + 1) return hipErrorInvalidValue;
    switch (P) {
        case 8: return fgt_impl<8>(b, n, L, sigma, nc, parts, m, u, v, st);
        case 12: return fgt_impl<12>(b, n, L, sigma, nc, parts, m, u, v, st);
        case 16: return fgt_impl<16>(b, n, L, sigma, nc, parts, m, u, v, st);
        default: return hipErrorInvalidValue;
    }
}

int fgt_parts(int P, int L, int nc)
{
    // enough workgroup rows for about 4096 wavefronts, at most 8 and at most
    // one per row of the range
    const int per_wave = P == 8 ? H2TGroups<8>::kPerWave : P == 12 ? H2TGroups<12>::kPerWave : H2TGroups<16>::kPerWave;
    const int64_t waves = ((int64_t(1) << (2 * L)) + per_wave - 1) / per_wave;
    const int64_t want = (4096 + waves - 1) / waves;
    return int(std::max<int64_t>(1, std::min<int64_t>({want, 8, 2 * nc + 1})));
}

void fgt_hermite_table(int P, int nc, double w_over_sd, double* out)
{
    const int NH = 2 * P - 1;
    for (int d = -nc; d <= nc; ++d) {
        const double t = double(d) * w_over_sd;
        double* h = out + (d + nc) * NH;
        h[0] = std::exp(-t * t);
        if (NH > 1) h[1] = 2.0 * t * h[0];
        for (int k = 1; k + 1 < NH; ++k) h[k + 1] = 2.0 * t * h[k] - 2.0 * double(k) * h[k - 1];
    }
}

}  // namespace fmm
