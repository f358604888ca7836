// fmm_downward.hip -- downward sweep (Section 2.2, Fig. 2): M2L over every
// box's interaction list, then L2L from each level to the next.
//
// Scaled coefficients make the translation operators level-independent.
// With ahat_k = a_k / w^k (multipole) and bhat_l = b_l w^(l+1) (local), the
// textbook M2L of the 1/z expansions, tau = (c_source - c_target) / w an
// integer offset with max(|dx|, |dy|) in {2, 3}, reads
//   bhat_l = sum_k (-1)^(k+1) C(k+l, k) tau^-(k+l+1) ahat_k .
// Writing C(k+l, k) = (k+l)! / (k! l!) factors it into a Hankel matrix
// between two diagonal scalings:
//   bhat_l = (1/l!) sum_k h_{k+l}(tau) abar_k,
//   h_n(tau) = n! tau^-(n+1),   abar_k = (-1)^(k+1) ahat_k / k!,
// so each of the 40 offsets is described by 2p-1 numbers instead of p^2 and
// the whole table (49 slots of a 7 x 7 grid, FP64 and FP32 copies) stays in
// the scalar/L1 caches.  The multipole arrays already hold abar (the upward
// sweep stores them that way), so only the output scaling 1/l! remains.  The
// product is dense: every (k, l) pair is one complex multiply-add, 8 p^2
// flops per interaction-list pair; on the vector units (FP64, and FP32 in
// the mixed form) the members are taken two at a time where the square's
// symmetries relate their data, which halves that (see the work items
// below).
//
// Lane mapping: a workgroup of 4 wavefronts covers 16 x 16 target boxes of
// one level; wavefront c holds the 64 boxes in child position c of their
// parents, so the 27 interaction-list offsets, and with them the translation
// data, are uniform across the wavefront.  Each lane owns one target box and
// keeps all p local coefficients in registers.  Every level from 2 to L is
// handled by one launch (M2L of different levels are independent); L2L then
// runs down the tree, adding the parent's shifted expansion.
#include "fmm_device.h"

#include <type_traits>
#include <utility>

namespace fmm {
namespace {

// Workgroups of one level: 16 x 16 target boxes each (one for levels < 4).
__host__ __device__ inline int level_blocks(int l)
{
    const int side = 1 << l;
    const int bpr = side >= 16 ? side / 16 : 1;
    return bpr * bpr;
}

// Runs of consecutive M2L workgroups kept on one XCD (xcd_runs): neighbouring
// tiles read overlapping source halos.  Measured 1-2 % faster than the plain
// round-robin placement on 1M-64M particle trees.
constexpr int kM2LXcdRun = 8;

// M2L by symmetric pairs.  The Hankel data of two offsets related by a
// symmetry of the square differ only by conjugation and the sign
// (-1)^(n+1): h_n(conj tau) = conj h_n(tau), h_n(-tau) = (-1)^(n+1) h_n(tau).
// For such a pair (tau, tau') with sources A and B, and S = A + B, D = A - B,
//   tau' = conj tau:   h A + h' B = u S + i v D                  (h = u + i v)
//   tau' = -conj tau:  the same for n odd, u D + i v S for n even
//   tau' = -tau, real: u S for n odd, u D for n even
// so one complex multiply-add (four FMAs, two for a real tau) serves two
// list members.  On an axis or a diagonal the data of one offset have a zero
// component (tau real: all real; tau = i y: imaginary for n even, real for n
// odd; tau = a (1 + i s), s = +-1: real or imaginary for n odd, and for n
// even u and v of equal size, v = s u for n = 2 mod 4 and -s u for n = 0 mod
// 4), so a single member costs two FMAs per term there: with p = ax - s ay
// and q = ax + s ay, b += u p + i v q (n = 2 mod 4) or u q + i v p (n = 0 mod
// 4).  The 27 offsets of child (0, 0), dx, dy in [-2, 3] and not both in
// [-1, 1], make 15 work items: 9 conjugate pairs, 2 negated-conjugate pairs,
// the real pair (-2, 0), (2, 0), and (3, 0), (0, 3), (3, 3) alone; the
// other children mirror them (dx -> -dx for child x = 1, dy -> -dy for
// y = 1), which keeps every relation.  Against 27 general members (4 FMAs
// per term each) the items take 52 / 108 of the FMAs.
enum : int { kItemConj = 0, kItemNegConj = 1, kItemNegReal = 2, kItemOneReal = 3, kItemOneImag = 4, kItemOneDiag = 5 };
constexpr int kM2LItems = 15;
__constant__ int8_t kM2LItemTab[kM2LItems][3] = {
    {-2, 1, kItemConj}, {2, 1, kItemConj}, {3, 1, kItemConj}, {-2, 2, kItemConj}, {2, 2, kItemConj},
    {3, 2, kItemConj}, {-1, 2, kItemConj}, {0, 2, kItemConj}, {1, 2, kItemConj},
    {-2, 3, kItemNegConj}, {-1, 3, kItemNegConj},
    {-2, 0, kItemNegReal}, {3, 0, kItemOneReal},
    {0, 3, kItemOneImag}, {3, 3, kItemOneDiag},
};

// Work items run in blocks of kM2LK consecutive source terms k, with the
// next block's loads in flight while the current block's products run: two
// blocks of both members and the 2P accumulators fit the registers of three
// wavefronts per SIMD.  (Carrying the next item's first block across the
// item loop as well made the compiler spill.)
constexpr int kM2LK = 4;
template <typename T>
struct M2LBlock {
    cplx<T> a[kM2LK], b[kM2LK];
};

// The products of one block (terms k0 .. k0 + kM2LK - 1) of a work item of
// kind KIND with Hankel data h; s = dy / dx for a diagonal.
template <typename T, int P, int KIND>
__device__ __forceinline__ void m2l_block(T* bx, T* by, const cplx<T>* __restrict__ h, const M2LBlock<T>& r,
                                          int k0, T s)
{
    constexpr int K = kM2LK;
    const int nk = k0 + K <= P ? K : P - k0;
    if constexpr (KIND <= kItemNegReal) {
        T Sx[K], Sy[K], Dx[K], Dy[K];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            if (kk < nk) {
                Sx[kk] = r.a[kk].x + r.b[kk].x;
                Sy[kk] = r.a[kk].y + r.b[kk].y;
                Dx[kk] = r.a[kk].x - r.b[kk].x;
                Dy[kk] = r.a[kk].y - r.b[kk].y;
            }
        }
#pragma unroll
        for (int nn = 0; nn < 2 * P - 1; ++nn) {
            if (nn < k0 || nn > k0 + nk + P - 2) continue;
            const cplx<T> hn = h[nn];
            const T u = hn.x, v = hn.y;
#pragma unroll
            for (int kk = 0; kk < K; ++kk) {
                const int j = nn - k0 - kk;
                if (kk >= nk || j < 0 || j >= P) continue;
                if (KIND == kItemNegReal) {
                    const T X = (nn & 1) ? Sx[kk] : Dx[kk], Y = (nn & 1) ? Sy[kk] : Dy[kk];
                    bx[j] = fma(u, X, bx[j]);
                    by[j] = fma(u, Y, by[j]);
                } else if (KIND == kItemConj || (nn & 1)) {
                    bx[j] = fma(u, Sx[kk], fma(-v, Dy[kk], bx[j]));
                    by[j] = fma(u, Sy[kk], fma(v, Dx[kk], by[j]));
                } else {
                    bx[j] = fma(u, Dx[kk], fma(-v, Sy[kk], bx[j]));
                    by[j] = fma(u, Dy[kk], fma(v, Sx[kk], by[j]));
                }
            }
        }
    } else {
        // a single member: n odd first with the source as it is, then n even
        // with (p, q) = (ax - s ay, ax + s ay) in its place (diagonal)
        T ax[K], ay[K];
#pragma unroll
        for (int kk = 0; kk < K; ++kk) {
            if (kk < nk) {
                ax[kk] = r.a[kk].x;
                ay[kk] = r.a[kk].y;
            }
        }
#pragma unroll
        for (int par = 1; par >= 0; --par) {
            if (KIND == kItemOneDiag && par == 0) {
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    if (kk < nk) {
                        const T pk = fma(-s, ay[kk], ax[kk]), qk = fma(s, ay[kk], ax[kk]);
                        ax[kk] = pk;
                        ay[kk] = qk;
                    }
                }
            }
#pragma unroll
            for (int nn = par; nn < 2 * P - 1; nn += 2) {
                if (nn < k0 || nn > k0 + nk + P - 2) continue;
                const cplx<T> hn = h[nn];
                const T u = hn.x, v = hn.y;
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int j = nn - k0 - kk;
                    if (kk >= nk || j < 0 || j >= P) continue;
                    if (KIND == kItemOneImag ? par == 1 : (nn & 3) == 3) {        // real data
                        bx[j] = fma(u, ax[kk], bx[j]);
                        by[j] = fma(u, ay[kk], by[j]);
                    } else if (KIND == kItemOneImag || (nn & 3) == 1) {          // imaginary data
                        bx[j] = fma(-v, ay[kk], bx[j]);
                        by[j] = fma(v, ax[kk], by[j]);
                    } else if ((nn & 3) == 2) {                                  // diagonal, v = s u
                        bx[j] = fma(u, ax[kk], bx[j]);
                        by[j] = fma(v, ay[kk], by[j]);
                    } else {                                                     // diagonal, v = -s u
                        bx[j] = fma(u, ay[kk], bx[j]);
                        by[j] = fma(v, ax[kk], by[j]);
                    }
                }
            }
        }
    }
}

// Block k0 .. k0 + kM2LK - 1 of the work items it0 <= it < it1 (all of kind
// KIND, or kItemNegReal with the single (3, 0) among them) that workgroup row
// g of G takes, for child (cx, cy): slot(dx, dy) names the source box at
// offset (dx, dy), term(slot, k) reads its term k, and zero_slot is a box of
// zeros (the partner of the item that has none).  K0 is a template argument:
// the accumulators are indexed by it and must stay in registers.
template <typename T, int P, int KIND, int K0, typename Slot, typename Term>
__device__ __forceinline__ void m2l_kind_block(T* bx, T* by, const cplx<T>* __restrict__ H, int cx, int cy, int g,
                                               int G, int it0, int it1, int zero_slot, Slot slot, Term term)
{
    constexpr int NH = 2 * P - 1;
    for (int it = it0 + (g - it0 % G + G) % G; it < it1; it += G) {
        int dx = kM2LItemTab[it][0], dy = kM2LItemTab[it][1];
        const bool pair = kM2LItemTab[it][2] != kItemOneReal;
        if (cx) dx = -dx;
        if (cy) dy = -dy;
        const cplx<T>* h = H + ((dy + 3) * kHankelGrid + (dx + 3)) * NH;
        const int ia = slot(dx, dy);
        const int ib = KIND <= kItemNegReal && pair
                           ? slot(KIND == kItemConj ? dx : -dx, KIND == kItemNegConj ? dy : -dy)
                           : zero_slot;
        M2LBlock<T> r;
#pragma unroll
        for (int kk = 0; kk < kM2LK; ++kk) {
            if (K0 + kk < P) {                  // abar_k, zero for k >= p
                const auto ta = term(ia, K0 + kk);
                r.a[kk] = cplx<T>{T(ta.x), T(ta.y)};
                if (KIND <= kItemNegReal) {
                    const auto tb = term(ib, K0 + kk);
                    r.b[kk] = cplx<T>{T(tb.x), T(tb.y)};
                }
            }
        }
        m2l_block<T, P, KIND>(bx, by, h, r, K0, dx == dy ? T(1) : T(-1));
    }
}

// Block K0 of all 15 work items of row g of G (the table's kinds in order).
template <typename T, int P, int K0, typename Slot, typename Term>
__device__ __forceinline__ void m2l_items_block(T* bx, T* by, const cplx<T>* __restrict__ H, int cx, int cy, int g,
                                                int G, int zero_slot, Slot slot, Term term)
{
    m2l_kind_block<T, P, kItemConj, K0>(bx, by, H, cx, cy, g, G, 0, 9, zero_slot, slot, term);
    m2l_kind_block<T, P, kItemNegConj, K0>(bx, by, H, cx, cy, g, G, 9, 11, zero_slot, slot, term);
    m2l_kind_block<T, P, kItemNegReal, K0>(bx, by, H, cx, cy, g, G, 11, 13, zero_slot, slot, term);
    m2l_kind_block<T, P, kItemOneImag, K0>(bx, by, H, cx, cy, g, G, 13, 14, zero_slot, slot, term);
    m2l_kind_block<T, P, kItemOneDiag, K0>(bx, by, H, cx, cy, g, G, 14, 15, zero_slot, slot, term);
}

// f(std::integral_constant<int, c>) for c = 0 .. sizeof...(C) - 1, in order.
template <typename F, int... C>
__device__ __forceinline__ void m2l_for_chunks(F f, std::integer_sequence<int, C...>)
{
    (f(std::integral_constant<int, C>{}), ...);
}

// gridDim.y = G in {1, 2, 3}: workgroup row g takes every G-th work item
// (the matrix-core kernel: every G-th member of the interaction list) and
// writes its partial sum to out[g] (out[0] = le).
struct M2LOut {
    cd* out[3];
};

// FP64 M2L with the sources of the workgroup's tile staged in LDS once: the
// 16 x 16 target boxes of a workgroup (four child classes of an 8 x 8 parent
// block) draw their interaction lists from the 20 x 20 boxes around them;
// boxes outside the grid are staged as zeros.  Same work items and block
// order as k_m2l_chunks, so the two give the same bits.  The stage takes
// 6.4 KB per expansion term (109 KB at p = 17), which leaves room for one
// workgroup per CU: on grids of a few tens of workgroups it is the faster
// (the whole stage loaded once); on larger ones the chunked stage, whose
// smaller footprint lets more wavefronts hide the loads.
constexpr int kHalo = 20;
constexpr int kM2LStageMaxWg = 32;
template <int P>
__global__ void __launch_bounds__(256)
k_m2l64_lds(Work wk, int n_inst, const Inst* __restrict__ inst, const cd* __restrict__ me_all, M2LOut dst_,
            const cplx<double>* __restrict__ H, const double* __restrict__ sout_)
{
    __shared__ cd sA[(kHalo * kHalo + 1) * P];        // + a box of zeros
    const int lin = xcd_runs(int(blockIdx.x + gridDim.x * blockIdx.y), int(gridDim.x * gridDim.y), kM2LXcdRun);
    const int g = lin / int(gridDim.x), blk = lin % int(gridDim.x);
    if (blk >= wk.wg_begin[n_inst]) return;                // past the launch's work (batched plans)
    const int pos = find_inst(wk.wg_begin, n_inst, blk);
    const int q = wk.order[pos];
    const int G = min(int(gridDim.y), inst[q].g64);
    if (g >= G) return;
    int bl = blk - wk.wg_begin[pos];
    int l = wk.arg[2 * pos];
    while (bl >= level_blocks(l)) { bl -= level_blocks(l); ++l; }
    const cd* me = me_all + inst[q].box_off * P;
    cd* __restrict__ le = g == 0 ? dst_.out[0] + inst[q].box_off * P : dst_.out[g] + inst[q].split_off * P;
    const int side = 1 << l;
    const int bpr = side >= 16 ? side / 16 : 1;
    const int bx = bl % bpr, by = bl / bpr;
    const cd* me_l = me + level_offset(l) * P;
    const int x_lo = 16 * bx - 2, y_lo = 16 * by - 2;
    // eight loads in flight per thread before their LDS writes
    for (int e0 = threadIdx.x; e0 < kHalo * kHalo * P; e0 += 256 * 8) {
        cd v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u, hb = e / P, k = e - hb * P;
            const int sa = x_lo + hb % kHalo, sb = y_lo + hb / kHalo;
            const bool in = e < kHalo * kHalo * P && sa >= 0 && sb >= 0 && sa < side && sb < side;
            v[u] = me_l[in ? int64_t(morton(uint32_t(sa), uint32_t(sb))) * P + k : 0];
            if (!in) v[u] = cd{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + 256 * u < kHalo * kHalo * P) sA[e0 + 256 * u] = v[u];
    }
    for (int k = threadIdx.x; k < P; k += 256) sA[kHalo * kHalo * P + k] = cd{0.0, 0.0};
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int cx = wave & 1, cy = wave >> 1;
    const int ta = 2 * (bx * 8 + (lane & 7)) + cx;
    const int tb = 2 * (by * 8 + (lane >> 3)) + cy;
    const bool active = ta < side && tb < side;
    double bx_[P], by_[P];
#pragma unroll
    for (int k = 0; k < P; ++k) { bx_[k] = 0.0; by_[k] = 0.0; }
    // the work items block by block, in the order of k_m2l_chunks
    auto slot = [&](int dx, int dy) { return (tb + dy - y_lo) * kHalo + (ta + dx - x_lo); };
    auto term = [&](int sl, int k) { return sA[sl * P + k]; };
    m2l_for_chunks([&](auto c) {
        m2l_items_block<double, P, decltype(c)::value * kM2LK>(bx_, by_, H, cx, cy, g, G, kHalo * kHalo, slot, term);
    }, std::make_integer_sequence<int, (P + kM2LK - 1) / kM2LK>{});
    if (active) {
        cd* dst = le + (level_offset(l) + int64_t(morton(uint32_t(ta), uint32_t(tb)))) * P;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double sc = sout_[k];
            dst[k] = cd{bx_[k] * sc, by_[k] * sc};
        }
    }
}

// M2L by symmetric pairs (T = double: every FP64 level but the smallest
// launches; T = float: the FP32 levels of the mixed form on the vector
// units) with the workgroup's sources staged in LDS kM2LK terms at a time:
// the 16 x 16 targets of a workgroup draw every source from the 20 x 20
// boxes around them, so chunk c holds terms 4c .. 4c + 3 of those 400 boxes
// (25.6 KB in FP64, k-major, zeros outside the level and past p, one zero
// box at the end for the item without a partner) and every wavefront runs
// block c of all its work items from it.  The loads of a chunk are
// coalesced and shared by the workgroup's 256 targets instead of issued per
// lane and member; in FP64 the same items and block order as k_m2l64_lds,
// so the two give the same bits.
template <int P, typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P > 24 ? 2 : 3)))
k_m2l_chunks(Work wk, int n_inst, const Inst* __restrict__ inst, const cd* __restrict__ me_all, M2LOut dst_,
             const cplx<T>* __restrict__ H, const double* __restrict__ sout_)
{
    constexpr int NB = (P + kM2LK - 1) / kM2LK;
    constexpr int NBOX = kHalo * kHalo;
    __shared__ cplx<T> sA[kM2LK][NBOX + 1];
    const int lin = xcd_runs(int(blockIdx.x + gridDim.x * blockIdx.y), int(gridDim.x * gridDim.y), kM2LXcdRun);
    const int g = lin / int(gridDim.x), blk = lin % int(gridDim.x);
    if (blk >= wk.wg_begin[n_inst]) return;                // past the launch's work (batched plans)
    const int pos = find_inst(wk.wg_begin, n_inst, blk);
    const int q = wk.order[pos];
    // split lists: FP32 levels always over the launch's three rows, FP64
    // levels over the instance's g64 (the rows past it have nothing to do)
    const int G = std::is_same<T, float>::value ? int(gridDim.y) : min(int(gridDim.y), inst[q].g64);
    if (g >= G) return;
    int bl = blk - wk.wg_begin[pos];
    int l = wk.arg[2 * pos];
    while (bl >= level_blocks(l)) { bl -= level_blocks(l); ++l; }
    const cd* me = me_all + inst[q].box_off * P;
    cd* __restrict__ le = g == 0 ? dst_.out[0] + inst[q].box_off * P : dst_.out[g] + inst[q].split_off * P;
    const int side = 1 << l;
    const int bpr = side >= 16 ? side / 16 : 1;
    const int bx = bl % bpr, by = bl / bpr;
    const cd* me_l = me + level_offset(l) * P;
    const int x_lo = 16 * bx - 2, y_lo = 16 * by - 2;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int cx = wave & 1, cy = wave >> 1;
    const int ta = 2 * (bx * 8 + (lane & 7)) + cx;
    const int tb = 2 * (by * 8 + (lane >> 3)) + cy;
    const bool active = ta < side && tb < side;
    T bx_[P], by_[P];
#pragma unroll
    for (int k = 0; k < P; ++k) { bx_[k] = T(0); by_[k] = T(0); }
    // halo slot of the source at offset (dx, dy) from this lane's target
    auto slot = [&](int dx, int dy) { return (tb + dy - y_lo) * kHalo + (ta + dx - x_lo); };
    m2l_for_chunks([&](auto c) {
        constexpr int k0 = decltype(c)::value * kM2LK;
        if (k0 > 0) __syncthreads();                        // every wavefront is done with the last chunk
        // every load issued before the first LDS write (one memory round
        // trip); outside the level, past p and past the stage: the level's
        // first term is read and replaced by zero
        constexpr int NE = NBOX * kM2LK, NIT = (NE + 255) / 256;
        cplx<T> v[NIT];
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = int(threadIdx.x) + 256 * i;
            const int hb = e / kM2LK, kk = e - hb * kM2LK;  // a box's terms from consecutive threads
            const int sa = x_lo + hb % kHalo, sb = y_lo + hb / kHalo;
            const bool in = e < NE && sa >= 0 && sb >= 0 && sa < side && sb < side && k0 + kk < P;
            const cd t = me_l[in ? int64_t(morton(uint32_t(sa), uint32_t(sb))) * P + k0 + kk : 0];
            v[i] = cplx<T>{T(t.x), T(t.y)};
            if (!in) v[i] = cplx<T>{T(0), T(0)};
        }
#pragma unroll
        for (int i = 0; i < NIT; ++i) {
            const int e = int(threadIdx.x) + 256 * i;
            if (e < NE) sA[e % kM2LK][e / kM2LK] = v[i];
        }
        if (threadIdx.x < kM2LK) sA[threadIdx.x][NBOX] = cplx<T>{T(0), T(0)};
        __syncthreads();
        // block c of every work item of this row
        m2l_items_block<T, P, k0>(bx_, by_, H, cx, cy, g, G, NBOX, slot, [&](int sl, int k) { return sA[k - k0][sl]; });
    }, std::make_integer_sequence<int, NB>{});
    if (active) {
        cd* dst = le + (level_offset(l) + int64_t(morton(uint32_t(ta), uint32_t(tb)))) * P;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const double sc = sout_[k];
            dst[k] = cd{double(bx_[k]) * sc, double(by_[k]) * sc};
        }
    }
}

// FP32 M2L on the matrix cores.  Written real-valued, the factored M2L of
// one interaction-list member is a dense product
//   [Re b; Im b] = [[Hr, -Hi], [Hi, Hr]] [Re abar; Im abar],  H[l][k] = h_{k+l}(tau),
// a (2P x 2P) matrix times the 2P terms of the source: for all targets of
// one offset tau together, a GEMM.  A wavefront holds the 64 targets of one
// child class (the same 27 offsets for all of them) as four column tiles of
// 16, and accumulates 16 x 16 output tiles over all its members with
// v_mfma_f32_16x16x4f32 (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
// D[i][j] in lane j + 16 (i/4), element i % 4).
//   Operands.  The workgroup's 16 x 16 targets draw every source from the
// 20 x 20 boxes around them; those boxes' multipole terms are staged once per
// workgroup in LDS, converted to FP32 and laid out real-valued (2P terms per
// box, one word of padding against bank conflicts; boxes outside the level
// are zeros), so a B fragment is one LDS word per lane.  The operator
// fragments are formed from the workgroup's LDS copy of the h_n of the 40
// offsets (rows and columns past 2P are zero), once per member and k-step,
// and serve all four column tiles.  78 KB of LDS per workgroup: two per CU.
// Same outputs as k_m2l_chunks; a list split over G rows takes every G-th
// interaction-list member.
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaHalo = 20;
// compact slot of offset (dx, dy), max(|dx|, |dy|) in {2, 3}: the 49 slots of
// the 7 x 7 grid without its inner 3 x 3
__device__ __forceinline__ int far_slot(int dx, int dy)
{
    const int s = (dy + 3) * kHankelGrid + (dx + 3);
    const int inner_before = dy < -1 ? 0 : (dy > 1 ? 9 : 3 * (dy + 1) + (dx < -1 ? 0 : (dx > 1 ? 3 : dx + 1)));
    return s - inner_before;
}

template <int P>
__global__ void __launch_bounds__(256, 2)
k_m2l_mfma(Work wk, int n_inst, const Inst* __restrict__ inst, const cd* __restrict__ me_all, M2LOut dst_,
           const cplx<float>* __restrict__ H, const double* __restrict__ sout_, int GG)
{
    constexpr int NH = 2 * P - 1;
    constexpr int R2 = 2 * P;                  // real-valued size
    constexpr int MT = (R2 + 15) / 16;         // output row tiles
    constexpr int KS = (R2 + 3) / 4;           // steps of 4 input terms
    constexpr int HS = R2 + 1;                 // words per staged box
    constexpr int NSLOT = kHankelGrid * kHankelGrid - 9;
    __shared__ cplx<float> sH[NSLOT * NH];
    __shared__ float hal[kMfmaHalo * kMfmaHalo * HS];
    const int G = GG;
    const int total = wk.wg_begin[n_inst];
    const int items = total * GG;
    if (int(blockIdx.x) >= items) return;                  // past the launch's work (batched plans)
    for (int e = threadIdx.x; e < kHankelGrid * kHankelGrid * NH; e += 256) {
        const int slot = e / NH, dx = slot % kHankelGrid - 3, dy = slot / kHankelGrid - 3;
        if (dx < -1 || dx > 1 || dy < -1 || dy > 1) sH[far_slot(dx, dy) * NH + e % NH] = H[e];
    }

    auto item = [&](const int g, const int blk) {
    const int pos = find_inst(wk.wg_begin, n_inst, blk);   // place in the launch order
    const int q = wk.order[pos];
    int bl = blk - wk.wg_begin[pos];
    int l = wk.arg[2 * pos];
    while (bl >= level_blocks(l)) { bl -= level_blocks(l); ++l; }
    const cd* me = me_all + inst[q].box_off * P;
    cd* __restrict__ le = g == 0 ? dst_.out[0] + inst[q].box_off * P : dst_.out[g] + inst[q].split_off * P;
    const int side = 1 << l;
    const int bpr = side >= 16 ? side / 16 : 1;
    const int bx = bl % bpr, by = bl / bpr;
    const int tid = threadIdx.x;
    const cd* me_l = me + level_offset(l) * P;

    // stage the 20 x 20 source boxes from (16 bx - 2, 16 by - 2) on
    const int ox = 16 * bx - 2, oy = 16 * by - 2;
    // eight loads in flight per thread before their LDS writes
    constexpr int NHAL = kMfmaHalo * kMfmaHalo * P;
    constexpr int NU = 8;
    for (int e0 = tid; e0 < NHAL; e0 += 256 * NU) {
        cd v[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = e0 + 256 * u, box = e / P, k = e % P;
            const int sa = ox + box % kMfmaHalo, sb = oy + box / kMfmaHalo;
            const bool in = e < NHAL && sa >= 0 && sb >= 0 && sa < side && sb < side;
            v[u] = me_l[in ? int64_t(morton(uint32_t(sa), uint32_t(sb))) * P + k : 0];
            if (!in) v[u] = cd{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = e0 + 256 * u, box = e / P, k = e % P;
            if (e < NHAL) {
                hal[box * HS + k] = float(v[u].x);
                hal[box * HS + P + k] = float(v[u].y);
            }
        }
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int cx = wave & 1, cy = wave >> 1;
    const int li = lane & 15, lq = lane >> 4;  // fragment row / column, and k quarter

    // the lane's target in each column tile: t = 16 n + li, laid out 8 x 8,
    // and its place in the staged halo
    int ta[4], tb[4], hx[4], hy[4];
    bool act[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int t = 16 * n + li;
        ta[n] = 2 * (bx * 8 + (t & 7)) + cx;
        tb[n] = 2 * (by * 8 + (t >> 3)) + cy;
        hx[n] = ta[n] - ox;
        hy[n] = tb[n] - oy;
        act[n] = ta[n] < side && tb[n] < side;
    }

    mfma_f4 acc[MT][4];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = mfma_f4{0.f, 0.f, 0.f, 0.f};

    int member = 0;
    for (int o = 0; o < 36; ++o) {
        int dx, dy;
        if (!il_offset(cx, cy, o, dx, dy)) continue;
        if ((member++) % G != g) continue;
        // source terms (B fragments): column li of tile n, rows 4 ks + lq,
        // from the staged halo (zeros past 2P and outside the level)
        const float* src[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) src[n] = hal + ((hy[n] + dy) * kMfmaHalo + hx[n] + dx) * HS;
        const cplx<float>* h = sH + far_slot(dx, dy) * NH;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int c = 4 * ks + lq;
            float bv[4];
#pragma unroll
            for (int n = 0; n < 4; ++n) bv[n] = c < R2 ? src[n][c] : 0.f;
            // operator fragments: row 16 m + li, column c
            float av[MT];
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int r = 16 * m + li;
                float val = 0.f;
                if (r < R2 && c < R2) {
                    const bool rim = r >= P, cim = c >= P;
                    const cplx<float> hn = h[(rim ? r - P : r) + (cim ? c - P : c)];
                    val = rim == cim ? hn.x : (rim ? hn.y : -hn.y);
                }
                av[m] = val;
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int n = 0; n < 4; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m], bv[n], acc[m][n], 0, 0, 0);
        }
    }

    // rows r < P are Re b_r, rows P <= r < 2P are Im b_(r-P); scaled by 1/l!
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        if (!act[n]) continue;
        double* dst = reinterpret_cast<double*>(le + (level_offset(l) + int64_t(morton(uint32_t(ta[n]), uint32_t(tb[n])))) * P);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * m + 4 * lq + v;
                if (r < R2) {
                    const int k = r < P ? r : r - P;
                    dst[2 * k + (r < P ? 0 : 1)] = double(acc[m][n][v]) * sout_[k];   // zero for k >= p
                }
            }
    }
    };
    // items in turn; the staged halo is reused by the next item
    for (int it = int(blockIdx.x); it < items;) {
        const int lin = xcd_runs(it, items, kM2LXcdRun);
        item(lin / total, lin % total);
        it += int(gridDim.x);
        if (it < items) __syncthreads();
    }
}

// L2L, subtree-fused like the upward sweep: a workgroup owns one box at level
// lt (whose local expansion is final) and walks up to three levels down its
// z-order-contiguous subtree in LDS.  Each child adds the parent's shifted
// expansion to what M2L wrote for it:
//   bhat^c_m += sum_{j>=m} C(j,m) delta^(j-m) 2^-(m+1) bhat^P_j ,
// the parent's Taylor series translated by delta (shift_taylor, in the
// registers of the thread that owns the child), then scaled by the exact
// 2^-(m+1).  (P = 32, whose P complex registers would not fit beside the
// rest, keeps the operator matrix Lt[c][m][j] in LDS.)
constexpr int kDownThreads = 256;

// part[0], part[1]: partial M2L sums of levels <= split_level (M2L ran with
// its interaction list split over two or three wavefronts there; part[1]
// only on the levels of Inst::part1); they are added to le when a level's M2L
// result is first read.
// All of the subtree's M2L results are loaded before the first wait: the
// levels above the last into LDS, the last level (at most 64 boxes) into the
// registers of the threads that finish it, which also keeps the LDS small
// enough for several workgroups per CU.
// Work table arg: lt, d.
template <int P>
__global__ void __launch_bounds__(kDownThreads)
k_downward(Work wk, int n_inst, const Inst* __restrict__ inst, cd* __restrict__ le_all,
           const cd* __restrict__ Lt, const cd* __restrict__ part0_all, const cd* __restrict__ part1_all)
{
    constexpr int kUp = (21 * P + kDownThreads - 1) / kDownThreads;     // levels lt .. lt+d-1 per thread
    constexpr int kLast = (64 * P + kDownThreads - 1) / kDownThreads;   // last level per thread
    constexpr bool kMatrix = P > 24;     // operator matrix in LDS instead of register shifts
    // levels lt, lt+1, lt+2 (1 + 4 + 16 boxes; with register shifts also the
    // last level, 64 more) at P (4^t - 1) / 3
    __shared__ cd sh[kMatrix ? 21 * P : 85 * P];
    __shared__ cd sL[kMatrix ? 4 * P * P : 1];
    const int tid = threadIdx.x;
    if (int(blockIdx.x) >= wk.wg_begin[n_inst]) return;           // past the launch's work (batched plans)
    const int pos = find_inst(wk.wg_begin, n_inst, blockIdx.x);   // place in the launch order
    const int q = wk.order[pos];
    const int64_t root = blockIdx.x - wk.wg_begin[pos];
    const int lt = wk.arg[2 * pos], d = wk.arg[2 * pos + 1];
    const int last = lt + d;
    const int split_level = inst[q].split;
    cd* le = le_all + inst[q].box_off * P;
    const cd* part0 = part0_all + inst[q].split_off * P;
    const cd* part1 = part1_all + inst[q].split_off * P;
    const int part1_levels = inst[q].part1;
    // What M2L left for each coefficient of the subtree, with the partial
    // sums added; the root (level lt) is final unless lt = 2, which gets no
    // L2L and finishes its M2L sum here.  Every thread issues the same loads
    // (indices clamped past the subtree's end; a partial-sum array only when
    // some level of the workgroup has one), all before the first wait, and
    // combines them afterwards.  The launches are grouped so that the large
    // ones cover three full levels.
    const int lo = lt == 2 ? lt : lt + 1;             // first level that takes partial sums
    const bool any0 = lo <= min(split_level, last);
    const bool any1 = any0 && ((part1_levels >> lo) & ((2 << (min(split_level, last) - lo)) - 1)) != 0;
    const int n_up = P * ((1 << (2 * d)) - 1) / 3;     // coefficients of levels lt .. last-1
    const int n_last = P << (2 * d);
    // slot i < kUp: coefficient tid + 256 i of levels lt .. last-1; slot
    // kUp + i: coefficient tid + 256 i of the last level
    constexpr int kSlots = kUp + kLast;
    int64_t gi[kSlots];
    bool a0[kSlots], a1[kSlots];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        int j, e;
        if (i < kUp) {
            const int e0 = tid + kDownThreads * i;
            const int ec = e0 < n_up ? e0 : 0;
            const int t = ec < P ? 0 : (ec < 5 * P ? 1 : 2);   // level lt + t
            j = lt + t;
            e = ec - P * ((1 << (2 * t)) - 1) / 3;
        } else {
            const int e0 = tid + kDownThreads * (i - kUp);
            j = last;
            e = e0 < n_last ? e0 : 0;
        }
        gi[i] = (level_offset(j) + (root << (2 * (j - lt)))) * P + e;
        a0[i] = j >= lo && j <= split_level;
        a1[i] = a0[i] && ((part1_levels >> j) & 1);
    }
    cd rv[kSlots], r0[kSlots], r1[kSlots];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) rv[i] = le[gi[i]];
    if (any0) {
#pragma unroll
        for (int i = 0; i < kSlots; ++i) r0[i] = part0[a0[i] ? gi[i] : 0];   // entry 0 always exists
    }
    if (any1) {
#pragma unroll
        for (int i = 0; i < kSlots; ++i) r1[i] = part1[a1[i] ? gi[i] : 0];
    }
    cd up[kUp], lastv[kLast];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        double x = rv[i].x, y = rv[i].y;
        if (any0) {
            x = a0[i] ? x + r0[i].x : x;
            y = a0[i] ? y + r0[i].y : y;
        }
        if (any1) {
            x = a1[i] ? x + r1[i].x : x;
            y = a1[i] ? y + r1[i].y : y;
        }
        if (i < kUp) up[i] = cd{x, y};
        else lastv[i - kUp] = cd{x, y};
    }
    if constexpr (kMatrix)
        for (int e = tid; e < 4 * P * P; e += kDownThreads) sL[e] = Lt[e];
#pragma unroll
    for (int i = 0; i < kUp; ++i) {
        const int e = tid + kDownThreads * i;
        if (e < n_up) {
            sh[e] = up[i];
            if (e < P && lt == 2 && lt <= split_level) le[level_offset(lt) * P + root * P + e] = up[i];
        }
    }
    if constexpr (!kMatrix) {
#pragma unroll
        for (int i = 0; i < kLast; ++i) {
            const int e = tid + kDownThreads * i;
            if (e < n_last) sh[n_up + e] = lastv[i];
        }
        __syncthreads();
        // level by level: thread t < 4^(j - lt) finishes child t in LDS (all
        // in the first wavefront: a wavefront's instruction stream costs the
        // same however few lanes are live), then the level goes out in whole
        // rows
        for (int j = lt + 1; j <= last; ++j) {
            const int n_out = 1 << (2 * (j - lt));
            const int in_off = P * ((n_out >> 2) - 1) / 3, out_off = P * (n_out - 1) / 3;
            const int t = tid;
            if (t < n_out) {
                cd b[P];
                const cd* par = sh + in_off + (t >> 2) * P;
#pragma unroll
                for (int k = 0; k < P; ++k) b[k] = par[k];
                double dx, dy;
                child_delta(t & 3, dx, dy);
                shift_taylor<P>(b, dx, dy);
                cd* mine = sh + out_off + t * P;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    const double f = ldexp(1.0, -(k + 1));
                    const cd c = mine[k];
                    mine[k] = cd{fma(b[k].x, f, c.x), fma(b[k].y, f, c.y)};
                }
            }
            __syncthreads();
            cd* g = le + (level_offset(j) + (root << (2 * (j - lt)))) * P;
            for (int e = tid; e < n_out * P; e += kDownThreads) g[e] = sh[out_off + e];
        }
        return;
    }
    __syncthreads();
    int n_in = 1;
    for (int j = lt + 1; j <= last; ++j) {
        const int n_out = n_in << 2;
        const int in_off = P * (n_in - 1) / 3, out_off = P * (n_out - 1) / 3;
        const int64_t gfirst = root << (2 * (j - lt));
        cd* g = le + (level_offset(j) + gfirst) * P;
#pragma unroll
        for (int i = 0; i < kLast; ++i) {
            const int e = tid + kDownThreads * i;
            if (e >= n_out * P) continue;
            const int o = e / P, k = e % P;
            const cd cur = j == last ? lastv[i] : sh[out_off + e];
            double bx = cur.x, by = cur.y;
            const cd* par = sh + in_off + (o >> 2) * P;
            const cd* Lr = sL + ((o & 3) * P + k) * P;     // rows k >= p are zero
            // the full row (entries m < k are zero): a fixed trip count lets
            // the LDS loads be issued together
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const cd t = Lr[m];
                const cd s = par[m];
                cmac(bx, by, t.x, t.y, s.x, s.y);
            }
            g[e] = cd{bx, by};
            if (j < last) sh[out_off + e] = cd{bx, by};
        }
        if (j == last) break;
        __syncthreads();
        n_in = n_out;
    }
}

// Debug: the interaction list of boxes [b0, b0 + cnt) in the order of the
// list offsets (il_offset), as global box ids, -1 padded to 27 entries, box
// b0 first.
__global__ void __launch_bounds__(256) k_ilist(int L, int64_t b0, int64_t cnt, int32_t* __restrict__ out)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const int64_t g = b0 + i;
    if (g >= level_offset(L + 1)) return;
    int l = 0;
    while (level_offset(l + 1) <= g) ++l;
    const uint32_t k = uint32_t(g - level_offset(l));
    const int ta = int(morton_x(k)), tb = int(morton_y(k)), side = 1 << l;
    int32_t* dst = out + i * 27;
    int n = 0;
    if (l >= 2) {
        const int cx = ta & 1, cy = tb & 1;
        for (int o = 0; o < 36; ++o) {
            int dx, dy;
            if (!il_offset(cx, cy, o, dx, dy)) continue;
            const int sa = ta + dx, sb = tb + dy;
            if (sa < 0 || sb < 0 || sa >= side || sb >= side) continue;
            dst[n++] = int32_t(level_offset(l) + morton(uint32_t(sa), uint32_t(sb)));
        }
    }
    for (; n < 27; ++n) dst[n] = -1;
}

template <int P>
hipError_t m2l_impl(const Buffers& b, const Work& w, int nwg, bool fp32, bool mfma, int groups, hipStream_t st)
{
    if (nwg <= 0) return hipSuccess;
    const dim3 grid{unsigned(nwg), unsigned(groups), 1u};
    const M2LOut out{{b.le, b.le_part[0], b.le_part[1]}};
    if constexpr (P <= 24) {
        if (fp32 && mfma) {   // one-dimensional: work items (tile, list share), one per workgroup
            hipLaunchKernelGGL((k_m2l_mfma<P>), dim3(unsigned(int64_t(nwg) * groups)), dim3(256), 0, st, w, b.n_inst,
                               b.inst, b.me, out, reinterpret_cast<const cplx<float>*>(b.t_h32), b.t_sout, groups);
            return hipGetLastError();
        }
        if (fp32) {
            hipLaunchKernelGGL((k_m2l_chunks<P, float>), grid, dim3(256), 0, st, w, b.n_inst, b.inst, b.me, out,
                               reinterpret_cast<const cplx<float>*>(b.t_h32), b.t_sout);
            return hipGetLastError();
        }
    }
    if constexpr (P <= 20) {       // beyond, the staged form spills registers
        if (int64_t(nwg) * groups <= kM2LStageMaxWg) {
            hipLaunchKernelGGL((k_m2l64_lds<P>), grid, dim3(256), 0, st, w, b.n_inst, b.inst, b.me, out,
                               reinterpret_cast<const cplx<double>*>(b.t_h64), b.t_sout);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_m2l_chunks<P, double>), grid, dim3(256), 0, st, w, b.n_inst, b.inst, b.me, out,
                       reinterpret_cast<const cplx<double>*>(b.t_h64), b.t_sout);
    return hipGetLastError();
}

template <int P>
hipError_t downward_impl(const Buffers& b, const Work& w, int nwg, hipStream_t st)
{
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_downward<P>, dim3(unsigned(nwg)), dim3(kDownThreads), 0, st, w, b.n_inst, b.inst, b.le,
                       b.t_l2l, b.le_part[0], b.le_part[1]);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_m2l(const Buffers& b, int P, const Work& w, int nwg, bool fp32, bool mfma, int groups,
                      hipStream_t st)
{
    switch (P) {
        case 8: return m2l_impl<8>(b, w, nwg, fp32, mfma, groups, st);
        case 12: return m2l_impl<12>(b, w, nwg, fp32, mfma, groups, st);
        case 16: return m2l_impl<16>(b, w, nwg, fp32, mfma, groups, st);
        case 17: return m2l_impl<17>(b, w, nwg, fp32, mfma, groups, st);
        case 20: return m2l_impl<20>(b, w, nwg, fp32, mfma, groups, st);
        case 24: return m2l_impl<24>(b, w, nwg, fp32, mfma, groups, st);
        case 32:   // FP32 translation data would overflow: mixed mode stops at p = 22
            return fp32 ? hipErrorInvalidValue : m2l_impl<32>(b, w, nwg, false, false, groups, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_downward(const Buffers& b, int P, const Work& w, int nwg, hipStream_t st)
{
    switch (P) {
        case 8: return downward_impl<8>(b, w, nwg, st);
        case 12: return downward_impl<12>(b, w, nwg, st);
        case 16: return downward_impl<16>(b, w, nwg, st);
        case 17: return downward_impl<17>(b, w, nwg, st);
        case 20: return downward_impl<20>(b, w, nwg, st);
        case 24: return downward_impl<24>(b, w, nwg, st);
        case 32: return downward_impl<32>(b, w, nwg, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ilist(int L, int64_t b0, int64_t cnt, int32_t* out, hipStream_t st)
{
    if (cnt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ilist, dim3(unsigned((cnt + 255) / 256)), dim3(256), 0, st, L, b0, cnt, out);
    return hipGetLastError();
}

}  // namespace fmm
