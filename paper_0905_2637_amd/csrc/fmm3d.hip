// fmm3d.hip -- the 3D form of the method on the GPU: the same tree and
// sweeps on a uniform octree (Section 8: the method carries over to 3D with
// a new kernel, its series expansions and translation operators), for the
// Laplace kernel 1/r with Cartesian Taylor expansions of total degree <= p.
//
// Per particle: potential phi(x) = sum_j q_j / |x - y_j| and its gradient,
// pairs at zero distance left out.  With w the box width of a level, c a
// box centre and everything scaled to unit boxes:
//   moments  Ms_k = sum_j q_j prod_i ((c_i - y_ji) / w)^k_i / k_i!
//   M2M      Ms_k(parent) = sum_{m <= k} Ms_m(child) 2^-|m| prod_i (s_i / 4)^(k_i - m_i) / (k_i - m_i)!,
//            s_i = +1 / -1 as the parent centre lies above / below the child's
//   M2L      Ls_n(t) = sum_k Ms_k(s) D_(k+n)((t - s) / w),   D_m = d^m (1/r)
//   L2L      Ls_n(child) += 2^-(1+|n|) sum_{m >= n} Ls_m(parent) 4^-(|m|-|n|) prod_i t_i^(m_i-n_i) / (m_i-n_i)!,
//            t_i = +1 / -1 as the child centre lies above / below the parent's
//   L2P      phi(x) = (1/w) sum_n Ls_n u^n / n!,  d phi / dx_i = (1/w^2) sum_n Ls_n u^(n-e_i) / (n-e_i)!,
//            u = (x - c) / w
// The scaling makes the M2L data level-independent: one table of D_m at the
// 316 integer offsets of the interaction lists.
//
// Layout: octree boxes in Morton order per level (children of box k at
// 8k .. 8k+7), levels one after another; coefficients of a box contiguous in
// the graded order of fmm3d_internal.h.  Tree build: keys, the library's
// stable radix sort (records carry x, y, q; z is gathered after), leaf
// ranges by binary search.
#include "fmm3d_internal.h"

namespace fmm3 {
namespace {

constexpr int kTpb = 256;
constexpr int kEvalTpb = 64;

__device__ inline uint32_t morton3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t k = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i)
        k |= (((a >> i) & 1u) << (3 * i)) | (((b >> i) & 1u) << (3 * i + 1)) | (((c >> i) & 1u) << (3 * i + 2));
    return k;
}

__device__ inline void unmorton3(uint32_t k, int& a, int& b, int& c)
{
    a = b = c = 0;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        a |= int((k >> (3 * i)) & 1u) << i;
        b |= int((k >> (3 * i + 1)) & 1u) << i;
        c |= int((k >> (3 * i + 2)) & 1u) << i;
    }
}

// multi-index (a, b, c) of graded position t
__device__ inline void decode3(int t, int& a, int& b, int& c)
{
    int d = 0;
    while (tet3(d + 1) <= t) ++d;
    int r = t - tet3(d), s = 0;
    while (tri3(s + 1) <= r) ++s;
    c = r - tri3(s);
    b = s - c;
    a = d - s;
}

// 1 / j! and 4^-j / j! for j <= kP3Max (the shift coefficients of M2M and L2L)
__constant__ double kInvFact3[kP3Max + 1] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720,
                                             1.0 / 5040, 1.0 / 40320, 1.0 / 362880};
__constant__ double kQuarterFact3[kP3Max + 1] = {1.0, 0.25, 1.0 / 32, 1.0 / 384, 1.0 / 6144, 1.0 / 122880,
                                                 1.0 / 2949120, 1.0 / 82575360, 1.0 / 2642411520.0,
                                                 1.0 / 95126814720.0};

// u^a (a <= kP3Max)
__device__ inline double ipow3(double u, int a)
{
    double r = 1.0;
    for (int i = 0; i < a; ++i) r *= u;
    return r;
}

__device__ inline double quarter_f(int j) { return kQuarterFact3[j]; }

// ---- tree -------------------------------------------------------------------

__global__ void __launch_bounds__(kTpb)
k3_keys(int n, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z, Geo3 g,
        uint32_t* __restrict__ key, unsigned long long* __restrict__ nbad)
{
    const int i = int(blockIdx.x) * kTpb + int(threadIdx.x);
    bool bad = false;
    if (i < n) {
        const double side = ldexp(1.0, g.L);
        const double u[3] = {(x[i] - g.x0) / g.W * side, (y[i] - g.y0) / g.W * side, (z[i] - g.z0) / g.W * side};
        uint32_t cc[3] = {0u, 0u, 0u};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!(u[d] >= 0.0 && u[d] < side)) bad = true;
            else cc[d] = uint32_t(floor(u[d]));
        }
        key[i] = bad ? (1u << (3 * g.L)) : morton3(cc[0], cc[1], cc[2]);
    }
    const uint64_t m = __ballot(bad);
    if (__lane_id() == 0 && m) atomicAdd(nbad, (unsigned long long)__popcll(m));
}

__global__ void __launch_bounds__(kTpb)
k3_gather(int n, const uint32_t* __restrict__ perm, const double* __restrict__ z, double* __restrict__ zs)
{
    const int i = int(blockIdx.x) * kTpb + int(threadIdx.x);
    if (i < n) zs[i] = z[perm[i]];
}

// leaf_start[b] = first sorted position with key >= b, b = 0 .. 8^L
__global__ void __launch_bounds__(kTpb)
k3_leaf_start(int64_t nleaf, int n, const uint32_t* __restrict__ ks, int32_t* __restrict__ leaf_start)
{
    const int64_t b = int64_t(blockIdx.x) * kTpb + threadIdx.x;
    if (b > nleaf) return;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (int64_t(ks[mid]) < b) lo = mid + 1;
        else hi = mid;
    }
    leaf_start[b] = lo;
}

__global__ void k3_clear(unsigned long long* nbad) { *nbad = 0ull; }

__global__ void __launch_bounds__(kTpb)
k3_zero4(int n, double* __restrict__ a, double* __restrict__ b, double* __restrict__ c, double* __restrict__ d)
{
    const int i = int(blockIdx.x) * kTpb + int(threadIdx.x);
    if (i < n) a[i] = b[i] = c[i] = d[i] = 0.0;
}

// ---- upward sweep -------------------------------------------------------------

// one workgroup per leaf, one thread per coefficient
__global__ void __launch_bounds__(kTpb)
k3_p2m(Geo3 g, const int32_t* __restrict__ ls, const double* __restrict__ xs, const double* __restrict__ ys,
       const double* __restrict__ zs, const double* __restrict__ qs, double* __restrict__ me)
{
    const uint32_t leaf = blockIdx.x;
    const int t = int(threadIdx.x);
    if (t >= g.T) return;
    int la, lb, lc;
    unmorton3(leaf, la, lb, lc);
    const double w = ldexp(g.W, -g.L);
    const double cx = g.x0 + (la + 0.5) * w, cy = g.y0 + (lb + 0.5) * w, cz = g.z0 + (lc + 0.5) * w;
    int a, b, c;
    decode3(t, a, b, c);
    const double inv_w = 1.0 / w;
    double acc = 0.0;
    for (int j = ls[leaf]; j < ls[leaf + 1]; ++j)
        acc += qs[j] * ipow3((cx - xs[j]) * inv_w, a) * ipow3((cy - ys[j]) * inv_w, b) *
               ipow3((cz - zs[j]) * inv_w, c);
    me[(lvl_off3(g.L) + leaf) * g.T + t] = acc * (kInvFact3[a] * kInvFact3[b] * kInvFact3[c]);
}

// parents at level l from their eight children; one workgroup per parent
__global__ void __launch_bounds__(kTpb)
k3_m2m(Geo3 g, int l, double* __restrict__ me)
{
    __shared__ double sm[8 * kT3Max];
    const uint32_t par = blockIdx.x;
    const int t = int(threadIdx.x), T = g.T;
    const double* src = me + (lvl_off3(l + 1) + int64_t(8) * par) * T;
    for (int e = t; e < 8 * T; e += int(blockDim.x)) sm[e] = src[e];
    __syncthreads();
    // A child's sign in the shift depends only on the parities of k - m: for
    // every term m replace the eight children's moments by their signed sums
    // H_pi(m) = sum_ch (-1)^popcount(ch & pi) Ms_m(ch) (a Walsh-Hadamard
    // transform over the children, one column per thread), so that each
    // output sums over m once instead of eight times.
    for (int m = t; m < T; m += int(blockDim.x)) {
        double v[8];
#pragma unroll
        for (int ch = 0; ch < 8; ++ch) v[ch] = sm[ch * T + m];
#pragma unroll
        for (int h = 1; h < 8; h <<= 1)
#pragma unroll
            for (int ch = 0; ch < 8; ++ch)
                if (!(ch & h)) {
                    const double u = v[ch], w = v[ch | h];
                    v[ch] = u + w;
                    v[ch | h] = u - w;
                }
#pragma unroll
        for (int pi = 0; pi < 8; ++pi) sm[pi * T + m] = v[pi];
    }
    __syncthreads();
    if (t >= T) return;
    int a, b, c;
    decode3(t, a, b, c);
    double acc = 0.0;
    for (int i = 0; i <= a; ++i)
        for (int j = 0; j <= b; ++j)
            for (int k = 0; k <= c; ++k) {
                const int pi = ((a - i) & 1) | (((b - j) & 1) << 1) | (((c - k) & 1) << 2);
                const double coef = ldexp(1.0, -(i + j + k)) * quarter_f(a - i) * quarter_f(b - j) * quarter_f(c - k);
                acc += sm[pi * T + pos3(i, j, k)] * coef;
            }
    me[(lvl_off3(l) + par) * T + t] = acc;
}

// ---- downward sweep -------------------------------------------------------------

// M2L of level l: one workgroup per target box, one thread per local
// coefficient; each interaction-list member's moments and derivative row are
// staged in LDS and read back as broadcasts (moments) and contiguous runs
// (derivatives)
__global__ void __launch_bounds__(kTpb)
k3_m2l(Geo3 g, int l, const double* __restrict__ me, double* __restrict__ le, const double* __restrict__ dtab)
{
    __shared__ double sM[kT3Max];
    __shared__ double sD[kT3Max2];
    const uint32_t box = blockIdx.x;
    const int t = int(threadIdx.x), T = g.T, T2 = g.T2, p = g.p;
    const int side = 1 << l;
    int ta, tb, tc;
    unmorton3(box, ta, tb, tc);
    int an = 0, bn = 0, cn = 0;
    if (t < T) decode3(t, an, bn, cn);
    const int dn = an + bn + cn, sn = bn + cn;
    const double* me_l = me + lvl_off3(l) * T;
    double acc = 0.0;
    for (int sc = 2 * (tc >> 1) - 2; sc <= 2 * (tc >> 1) + 3; ++sc)
        for (int sb = 2 * (tb >> 1) - 2; sb <= 2 * (tb >> 1) + 3; ++sb)
            for (int sa = 2 * (ta >> 1) - 2; sa <= 2 * (ta >> 1) + 3; ++sa) {
                if (sa < 0 || sb < 0 || sc < 0 || sa >= side || sb >= side || sc >= side) continue;
                if (abs(sa - ta) <= 1 && abs(sb - tb) <= 1 && abs(sc - tc) <= 1) continue;
                const double* src = me_l + int64_t(morton3(uint32_t(sa), uint32_t(sb), uint32_t(sc))) * T;
                const double* drow = dtab + int64_t(off3_index(ta - sa, tb - sb, tc - sc)) * T2;
                __syncthreads();
                for (int e = t; e < T; e += kTpb) sM[e] = src[e];
                for (int e = t; e < T2; e += kTpb) sD[e] = drow[e];
                __syncthreads();
                if (t < T)
                    for (int dk = 0; dk <= p; ++dk)
                        for (int sk = 0; sk <= dk; ++sk) {
                            const int base = tet3(dk + dn) + tri3(sk + sn) + cn;
                            const int kb = tet3(dk) + tri3(sk);
                            for (int ck = 0; ck <= sk; ++ck) acc = fma(sM[kb + ck], sD[base + ck], acc);
                        }
            }
    if (t < T) le[(lvl_off3(l) + box) * T + t] = acc;
}

// M2L for 1 <= p <= kLaneMaxP3 (9), all levels in one launch.  One lane per target box:
// a workgroup takes the 64 boxes of one parity class (child position in the
// parent) under a 4 x 4 x 4 block of parents, so all its lanes walk the same
// 189 offsets, and each wavefront computes a quarter of the output terms.
// The derivative row of the current offset is the same for every lane: it is
// staged in LDS as a dense (2p+1)^3 cube and read back as broadcasts.  In the
// cube the entry of k + n sits at cube(k) + cube(n): cube(n) is a
// compile-time constant of the unrolled output loop, cube(k) one LDS read per
// source term.
// wavefronts per workgroup (each takes 1/waves of the output terms): eight
// from p = 7 on keeps the accumulators of a lane within about 60 registers
template <int P>
__host__ __device__ constexpr int lane_waves() { return P >= 7 ? 8 : 4; }
template <int P>
__host__ __device__ constexpr int lane_terms() { return (tet3(P + 1) + lane_waves<P>() - 1) / lane_waves<P>(); }

template <int P>
__host__ __device__ constexpr int cube_of(int t)
{
    int d = 0;
    while (tet3(d + 1) <= t) ++d;
    int r = t - tet3(d), s = 0;
    while (tri3(s + 1) <= r) ++s;
    const int c = r - tri3(s), b = s - c, a = d - s;
    return (a * (2 * P + 1) + b) * (2 * P + 1) + c;
}

struct LaneLevels {
    int n_levels;
    int first_level;
    int blk_begin[kDepth3Max + 1];   // first workgroup of each level, then the total
};

// FMA block of one wavefront for one interaction offset: outputs
// [W Q, W Q + Q) of its lane's target, all terms of the lane's source
template <int P, int W>
__device__ __forceinline__ void m2l_lanes_fma(double (&acc)[lane_terms<P>()], const double* __restrict__ sD,
                                              const double* __restrict__ src, bool vs, const int* __restrict__ sK)
{
    constexpr int T = tet3(P + 1), Q = lane_terms<P>(), N0 = W * Q, N1 = N0 + Q < T ? N0 + Q : T;
    // two source terms per step, the step loop kept rolled: unrolled, the
    // scheduler hoists the LDS reads of many terms and spills
#pragma unroll 1
    for (int k0 = 0; k0 < T; k0 += 2) {
        double m[2];
        int ik[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int k = k0 + j;
            const bool in = k < T;
            m[j] = (vs && in) ? src[k] : 0.0;
            ik[j] = in ? sK[k] : 0;
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const double* d = sD + ik[j];
#pragma unroll
            for (int n = N0; n < N1; ++n) acc[n - N0] = fma(d[cube_of<P>(n)], m[j], acc[n - N0]);
        }
    }
}

template <int P>
__global__ void __launch_bounds__(64 * lane_waves<P>())
k3_m2l_lanes(Geo3 g, LaneLevels lv, const double* __restrict__ me, double* __restrict__ le,
             const double* __restrict__ dcube, const int* __restrict__ kcube)
{
    constexpr int T = tet3(P + 1), Q = lane_terms<P>(), NT = 64 * lane_waves<P>();
    constexpr int S = 2 * P + 1, S3 = S * S * S;
    __shared__ double sD[S3];
    __shared__ int sK[T];
    int li = 0;
    while (li + 1 < lv.n_levels && int(blockIdx.x) >= lv.blk_begin[li + 1]) ++li;
    const int l = lv.first_level + li;
    const int blk = int(blockIdx.x) - lv.blk_begin[li];
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int lane = int(threadIdx.x) & 63;
    const int cls = int(blockIdx.y);
    const int cx = cls & 1, cy = (cls >> 1) & 1, cz = cls >> 2;
    const int h = 1 << (l - 1), nb = h >= 4 ? h / 4 : 1, side = 2 * h;
    const int bx = blk % nb, by = (blk / nb) % nb, bz = blk / (nb * nb);
    const int px = 4 * bx + (lane & 3), py = 4 * by + ((lane >> 2) & 3), pz = 4 * bz + (lane >> 4);
    const bool vt = px < h && py < h && pz < h;
    const int ta = 2 * px + cx, tb = 2 * py + cy, tc = 2 * pz + cz;
    const double* me_l = me + lvl_off3(l) * T;
    for (int e = int(threadIdx.x); e < T; e += NT) sK[e] = kcube[e];
    double acc[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[i] = 0.0;
    for (int oz = cz - 3; oz <= cz + 2; ++oz)
        for (int oy = cy - 3; oy <= cy + 2; ++oy)
            for (int ox = cx - 3; ox <= cx + 2; ++ox) {
                if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
                const double* drow = dcube + int64_t(off3_index(ox, oy, oz)) * S3;
                __syncthreads();
                for (int e = int(threadIdx.x); e < S3; e += NT) sD[e] = drow[e];
                __syncthreads();
                const int sa = ta - ox, sb = tb - oy, sc = tc - oz;
                const bool vs = vt && sa >= 0 && sb >= 0 && sc >= 0 && sa < side && sb < side && sc < side;
                const double* src = me_l + (vs ? int64_t(morton3(uint32_t(sa), uint32_t(sb), uint32_t(sc))) * T : 0);
                switch (wave) {
                    case 0: m2l_lanes_fma<P, 0>(acc, sD, src, vs, sK); break;
                    case 1: m2l_lanes_fma<P, 1>(acc, sD, src, vs, sK); break;
                    case 2: m2l_lanes_fma<P, 2>(acc, sD, src, vs, sK); break;
                    case 3: m2l_lanes_fma<P, 3>(acc, sD, src, vs, sK); break;
                    case 4: if constexpr (lane_waves<P>() > 4) m2l_lanes_fma<P, 4>(acc, sD, src, vs, sK); break;
                    case 5: if constexpr (lane_waves<P>() > 4) m2l_lanes_fma<P, 5>(acc, sD, src, vs, sK); break;
                    case 6: if constexpr (lane_waves<P>() > 4) m2l_lanes_fma<P, 6>(acc, sD, src, vs, sK); break;
                    default: if constexpr (lane_waves<P>() > 4) m2l_lanes_fma<P, 7>(acc, sD, src, vs, sK); break;
                }
            }
    if (vt) {
        double* dst = le + (lvl_off3(l) + int64_t(morton3(uint32_t(ta), uint32_t(tb), uint32_t(tc)))) * T + wave * Q;
        const int cnt = wave * Q + Q < T ? Q : T - wave * Q;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i < cnt) dst[i] = acc[i];
    }
}

// L2L into level l (>= 3): one workgroup per child box
__global__ void __launch_bounds__(kTpb)
k3_l2l(Geo3 g, int l, double* __restrict__ le)
{
    __shared__ double sL[kT3Max];
    const uint32_t box = blockIdx.x;
    const int t = int(threadIdx.x), T = g.T, p = g.p;
    const double* par = le + (lvl_off3(l - 1) + (box >> 3)) * T;
    for (int e = t; e < T; e += int(blockDim.x)) sL[e] = par[e];
    __syncthreads();
    if (t >= T) return;
    const int bx = box & 1, by = (box >> 1) & 1, bz = (box >> 2) & 1;
    int a, b, c;
    decode3(t, a, b, c);
    double acc = 0.0;
    for (int i = a; i <= p; ++i)
        for (int j = b; i + j <= p; ++j)
            for (int k = c; i + j + k <= p; ++k) {
                const bool neg = (((1 - bx) & (i - a)) ^ ((1 - by) & (j - b)) ^ ((1 - bz) & (k - c))) & 1;
                const double v = sL[pos3(i, j, k)] * quarter_f(i - a) * quarter_f(j - b) * quarter_f(k - c);
                acc += neg ? -v : v;
            }
    double* dst = le + (lvl_off3(l) + box) * T + t;
    *dst += acc * ldexp(1.0, -(1 + a + b + c));
}

// ---- evaluation: L2P and the near field -----------------------------------------

// one wavefront per leaf (leaves hold tens of particles); targets in chunks of
// 64, the sources of each of the 27 near leaves staged in LDS in chunks of 64
template <int P>
__global__ void __launch_bounds__(kEvalTpb)
k3_eval(Geo3 g, int far, const int32_t* __restrict__ ls, const double* __restrict__ xs,
        const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ qs,
        const uint32_t* __restrict__ perm, const double* __restrict__ le, double* __restrict__ phi,
        double* __restrict__ gx, double* __restrict__ gy, double* __restrict__ gz)
{
    constexpr int T = tet3(P + 1);
    __shared__ double sL[T];
    __shared__ double sx[kEvalTpb], sy[kEvalTpb], sz[kEvalTpb], sq[kEvalTpb];
    const uint32_t leaf = blockIdx.x;
    const int t0 = ls[leaf], t1 = ls[leaf + 1];
    if (t0 == t1) return;
    const int side = 1 << g.L;
    int la, lb, lc;
    unmorton3(leaf, la, lb, lc);
    const double w = ldexp(g.W, -g.L);
    const double cx = g.x0 + (la + 0.5) * w, cy = g.y0 + (lb + 0.5) * w, cz = g.z0 + (lc + 0.5) * w;
    if (far)
        for (int e = int(threadIdx.x); e < T; e += kEvalTpb) sL[e] = le[(lvl_off3(g.L) + leaf) * T + e];
    for (int base = t0; base < t1; base += kEvalTpb) {
        const int i = base + int(threadIdx.x);
        const bool act = i < t1;
        const double xi = act ? xs[i] : 0.0, yi = act ? ys[i] : 0.0, zi = act ? zs[i] : 0.0;
        double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
        __syncthreads();
        if (far && act) {
            double px[P + 1], py[P + 1], pz[P + 1];
            const double ux = (xi - cx) / w, uy = (yi - cy) / w, uz = (zi - cz) / w;
            px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
            for (int k = 1; k <= P; ++k) {
                const double rk = 1.0 / double(k);     // a compile-time constant once unrolled
                px[k] = px[k - 1] * ux * rk;
                py[k] = py[k - 1] * uy * rk;
                pz[k] = pz[k - 1] * uz * rk;
            }
#pragma unroll
            for (int d = 0; d <= P; ++d)
#pragma unroll
                for (int s = 0; s <= d; ++s)
#pragma unroll
                    for (int c = 0; c <= s; ++c) {
                        const int a = d - s, b = s - c;
                        const double l = sL[pos3(a, b, c)];
                        f += l * px[a] * py[b] * pz[c];
                        if (a > 0) fx += l * px[a - 1] * py[b] * pz[c];
                        if (b > 0) fy += l * px[a] * py[b - 1] * pz[c];
                        if (c > 0) fz += l * px[a] * py[b] * pz[c - 1];
                    }
            f /= w;
            const double w2 = w * w;
            fx /= w2;
            fy /= w2;
            fz /= w2;
        }
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int na = la + dx, nb = lb + dy, nc = lc + dz;
                    if (na < 0 || nb < 0 || nc < 0 || na >= side || nb >= side || nc >= side) continue;
                    const uint32_t nl = morton3(uint32_t(na), uint32_t(nb), uint32_t(nc));
                    const int s0 = ls[nl], s1 = ls[nl + 1];
                    for (int cb = s0; cb < s1; cb += kEvalTpb) {
                        __syncthreads();
                        const int j = cb + int(threadIdx.x);
                        if (j < s1) {
                            sx[threadIdx.x] = xs[j];
                            sy[threadIdx.x] = ys[j];
                            sz[threadIdx.x] = zs[j];
                            sq[threadIdx.x] = qs[j];
                        }
                        __syncthreads();
                        const int cnt = min(kEvalTpb, s1 - cb);
                        if (act)
#pragma unroll 4
                            for (int jj = 0; jj < cnt; ++jj) {
                                const double ddx = xi - sx[jj], ddy = yi - sy[jj], ddz = zi - sz[jj];
                                const double r2 = ddx * ddx + ddy * ddy + ddz * ddz;
                                if (r2 == 0.0) continue;
                                const double ir = 1.0 / sqrt(r2);
                                const double qr = sq[jj] * ir;
                                f += qr;
                                const double cc = qr * ir * ir;
                                fx -= cc * ddx;
                                fy -= cc * ddy;
                                fz -= cc * ddz;
                            }
                    }
                }
        if (act) {
            const uint32_t o = perm[i];
            phi[o] = f;
            gx[o] = fx;
            gy[o] = fy;
            gz[o] = fz;
        }
    }
}

int blocks(int64_t n) { return int((n + kTpb - 1) / kTpb); }

}  // namespace

hipError_t launch3_clear(const Bufs3& b, hipStream_t st)
{
    hipLaunchKernelGGL(k3_clear, dim3(1), dim3(1), 0, st, b.nbad);
    return hipGetLastError();
}

hipError_t launch3_tree(const Bufs3& b, const Geo3& g, int n, const double* x, const double* y, const double* z,
                        const double* q, hipStream_t st)
{
    hipLaunchKernelGGL(k3_keys, dim3(blocks(n)), dim3(kTpb), 0, st, n, x, y, z, g, b.key, b.nbad);
    const hipError_t e = fmm::launch_sort_keys(b.sort, n, b.key, x, y, q, b.ks, b.perm, b.xs, b.ys, b.qs,
                                               3 * g.L + 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k3_gather, dim3(blocks(n)), dim3(kTpb), 0, st, n, b.perm, z, b.zs);
    const int64_t nleaf = int64_t(1) << (3 * g.L);
    hipLaunchKernelGGL(k3_leaf_start, dim3(blocks(nleaf + 1)), dim3(kTpb), 0, st, nleaf, n, b.ks, b.leaf_start);
    return hipGetLastError();
}

// the coefficient kernels take one thread per term: T rounded up to wavefronts
static unsigned coef_threads(const Geo3& g) { return unsigned((g.T + 63) / 64 * 64); }

hipError_t launch3_upward(const Bufs3& b, const Geo3& g, hipStream_t st)
{
    const unsigned nleaf = 1u << (3 * g.L);
    hipLaunchKernelGGL(k3_p2m, dim3(nleaf), dim3(coef_threads(g)), 0, st, g, b.leaf_start, b.xs, b.ys, b.zs, b.qs,
                       b.me);
    for (int l = g.L - 1; l >= 2; --l)
        hipLaunchKernelGGL(k3_m2m, dim3(1u << (3 * l)), dim3(coef_threads(g)), 0, st, g, l, b.me);
    return hipGetLastError();
}

namespace {
template <int P>
void m2l_lanes(const Bufs3& b, const Geo3& g, hipStream_t st)
{
    LaneLevels lv{};
    lv.first_level = 2;
    lv.n_levels = g.L - 1;
    int total = 0;
    for (int l = 2; l <= g.L; ++l) {
        lv.blk_begin[l - 2] = total;
        const int h = 1 << (l - 1), nb = h >= 4 ? h / 4 : 1;
        total += nb * nb * nb;
    }
    lv.blk_begin[g.L - 1] = total;
    hipLaunchKernelGGL((k3_m2l_lanes<P>), dim3(unsigned(total), 8u), dim3(64 * lane_waves<P>()), 0, st, g, lv, b.me, b.le, b.dcube,
                       b.kcube);
}
}  // namespace

hipError_t launch3_m2l(const Bufs3& b, const Geo3& g, hipStream_t st)
{
    // the lane kernel reads the derivative cubes, which the plan holds only
    // for 1 <= p <= kLaneMaxP3
    static_assert(kLaneMaxP3 <= 9, "lane M2L instantiated for p <= 9 only");
    if (g.p >= 1 && g.p <= kLaneMaxP3) {
        switch (g.p) {
            case 1: m2l_lanes<1>(b, g, st); return hipGetLastError();
            case 2: m2l_lanes<2>(b, g, st); return hipGetLastError();
            case 3: m2l_lanes<3>(b, g, st); return hipGetLastError();
            case 4: m2l_lanes<4>(b, g, st); return hipGetLastError();
            case 5: m2l_lanes<5>(b, g, st); return hipGetLastError();
            case 6: m2l_lanes<6>(b, g, st); return hipGetLastError();
            case 7: m2l_lanes<7>(b, g, st); return hipGetLastError();
            case 8: m2l_lanes<8>(b, g, st); return hipGetLastError();
            case 9: m2l_lanes<9>(b, g, st); return hipGetLastError();
            default: break;
        }
    }
    for (int l = 2; l <= g.L; ++l)
        hipLaunchKernelGGL(k3_m2l, dim3(1u << (3 * l)), dim3(kTpb), 0, st, g, l, b.me, b.le, b.dtab);
    return hipGetLastError();
}

hipError_t launch3_l2l(const Bufs3& b, const Geo3& g, hipStream_t st)
{
    for (int l = 3; l <= g.L; ++l)
        hipLaunchKernelGGL(k3_l2l, dim3(1u << (3 * l)), dim3(coef_threads(g)), 0, st, g, l, b.le);
    return hipGetLastError();
}

namespace {
template <int P>
void eval_p(const Bufs3& b, const Geo3& g, hipStream_t st, double* phi, double* gx, double* gy, double* gz)
{
    const unsigned nleaf = 1u << (3 * g.L);
    hipLaunchKernelGGL((k3_eval<P>), dim3(nleaf), dim3(kEvalTpb), 0, st, g, g.L >= 2 ? 1 : 0, b.leaf_start, b.xs,
                       b.ys, b.zs, b.qs, b.perm, b.le, phi, gx, gy, gz);
}
}  // namespace

hipError_t launch3_eval(const Bufs3& b, const Geo3& g, int n, double* phi, double* gx, double* gy, double* gz,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k3_zero4, dim3(blocks(n)), dim3(kTpb), 0, st, n, phi, gx, gy, gz);
    switch (g.p) {
        case 0: eval_p<0>(b, g, st, phi, gx, gy, gz); break;
        case 1: eval_p<1>(b, g, st, phi, gx, gy, gz); break;
        case 2: eval_p<2>(b, g, st, phi, gx, gy, gz); break;
        case 3: eval_p<3>(b, g, st, phi, gx, gy, gz); break;
        case 4: eval_p<4>(b, g, st, phi, gx, gy, gz); break;
        case 5: eval_p<5>(b, g, st, phi, gx, gy, gz); break;
        case 6: eval_p<6>(b, g, st, phi, gx, gy, gz); break;
        case 7: eval_p<7>(b, g, st, phi, gx, gy, gz); break;
        case 8: eval_p<8>(b, g, st, phi, gx, gy, gz); break;
        case 9: eval_p<9>(b, g, st, phi, gx, gy, gz); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fmm3
