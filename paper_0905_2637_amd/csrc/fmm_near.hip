// fmm_near.hip -- evaluation step (Section 2.2): for every particle the far
// field from its leaf's local expansion (L2P) plus the near field summed
// directly over the leaf and its touching leaves (P2P) with the Gaussian
// regularised kernel of eq. 8, written out as the velocity of eq. 9 in the
// caller's order.  A plan may select the singular kernel of eq. 7 (point
// vortices) instead: the Gaussian factor below is then 1, and the kernels
// are compiled without it.  Or the Lennard-Jones force of molecular dynamics
// (a short-range kernel, cut off within a leaf width): then the pair term is
// 24 eps (2 (s/r)^12 - (s/r)^6) / r^2 times the separation, the output the
// force itself, and there is no far field.
//
// Complex form: phi(z_i) = sum_j gamma_j (1 - exp(-|z_i - z_j|^2 / 2 sigma^2))
// / (z_i - z_j) over near pairs, plus L2P; u = Im(phi)/(2 pi), v = Re(phi)/(2 pi).
// Zero-distance pairs contribute nothing.
//
// Work decomposition: one wavefront per target leaf, four independent
// wavefronts (four z-order-consecutive leaves) per workgroup so that a CU
// holds more wavefronts than its workgroup slots would allow with one-wave
// groups; each wavefront stages into its own LDS region and synchronises only
// with itself.  The particles of the
// 3 x 3 neighbourhood are staged through LDS in chunks with coalesced loads
// (each leaf's particles are contiguous in the sorted arrays), padded with
// inert sources (zero circulation; at the leaf centre for the FP64 Gaussian
// kernel, far away otherwise) to a multiple of the slice count so every lane
// runs the same, unrollable trip count.  Register
// blocking: a lane owns R targets and one of S interleaved slices of the
// staged sources, so each LDS read feeds R pair interactions; the S partial
// sums meet through LDS.  Leaves with more than 64
// particles are walked in target chunks of 64.
//
// FP64: the Gaussian factor, as 1 - 2^(r^2 (-log2 e / 2 sigma^2)), and the
// reciprocal are evaluated inline (polynomial and Newton-refined hardware
// estimate) instead of library calls; a lane's R targets share one
// reciprocal per source (that of the product of their r^2).  Differences are taken between
// physical positions, exact for nearby points, so a pair's term keeps its
// relative accuracy however close the pair is.
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

struct Src64 { double x, y, g; };

// Constants of the pair kernel (uniform over a launch).
struct PairK {
    double nl2;              // Gaussian core: -log2(e) / (2 sigma^2), so exp(-r^2/2s^2) = 2^(nl2 r^2)
    double s2, rc2, e24;     // Lennard-Jones: s^2, cutoff^2, 24 eps
};

// g (1 - 2^x) for x <= 0 in FP64, within 1.5e-15 relative of the exact
// value for every x (a CPU check of this operation sequence against a
// long-double reference on 2e7 points, x from -1e-18 to -70).  Split x = k +
// f with k = rint(x) and f = x - k, both exact, |f| <= 1/2; take 2^f - 1 =
// f q(f) with q a degree-9 near-minimax fit of (2^f - 1)/f on [-1/2, 1/2]
// (fit error 1.25e-15 relative), and use
//   g (1 - 2^x) = g (1 - 2^k) - g 2^k (2^f - 1),
// which is -g (2^f - 1) for k = 0 and free of cancellation for k <= -1; g 2^k
// is one ldexp, so the circulation costs no extra multiply.  No clamp is
// needed: f stays in [-1/2, 1/2] for every x (x - rint(x) is exact, and 0
// once |x| >= 2^52), and the hardware conversion of k to an integer
// saturates, so for k below -2^31 the ldexp gives 0 and the result is g.
__device__ __forceinline__ double g_one_minus_exp2(double x, double g)
{
    const double k = __builtin_rint(x);
    const double f = x - k;
    int ki;
    // the instruction's own saturation (a C++ conversion would be undefined
    // out of range)
    asm("v_cvt_i32_f64 %0, %1" : "=v"(ki) : "v"(k));
    double q = 7.054911498517923e-09;
    q = fma(q, f, 1.0205975487818139e-07);
    q = fma(q, f, 1.3215542376478124e-06);
    q = fma(q, f, 1.5252672644100859e-05);
    q = fma(q, f, 0.00015403530253982429);
    q = fma(q, f, 0.0013333558201124075);
    q = fma(q, f, 0.009618129107737676);
    q = fma(q, f, 0.055504108664650574);
    q = fma(q, f, 0.24022650695909853);
    q = fma(q, f, 0.6931471805599462);
    const double em = q * f;                // 2^f - 1
    const double gs = ldexp(g, ki);         // g 2^k, exact unless it underflows
    return fma(-gs, em, g - gs);
}

// 1/x for a positive normal x: hardware estimate (about 2^-26 relative)
// and one Newton step, which squares the relative error.
__device__ __forceinline__ double recip(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// 1/a[r] for R positive values with one hardware reciprocal (about four
// times the cost of an FMA): that of their product, refined by one Newton
// step, times the other factors; a few ulp.  The product must stay normal:
// every a[r] within [1e-76, 1e75] keeps it so.
template <int R>
__device__ __forceinline__ void recip_n(const double* a, double* ia)
{
    if constexpr (R == 1) {
        ia[0] = recip(a[0]);
    } else if constexpr (R == 2) {
        const double y = recip(a[0] * a[1]);
        ia[0] = y * a[1];
        ia[1] = y * a[0];
    } else {
        static_assert(R == 4, "one, two or four values");
        const double p01 = a[0] * a[1], p23 = a[2] * a[3];
        const double y = recip(p01 * p23);
        const double y01 = y * p23, y23 = y * p01;
        ia[0] = y01 * a[1];
        ia[1] = y01 * a[0];
        ia[2] = y23 * a[3];
        ia[3] = y23 * a[2];
    }
}

// Floor of the Gaussian pair term's r^2: positive for coincident points,
// whose term then vanishes through 1 - 2^0 = 0 and dx = dy = 0.  It changes
// the term by a relative 1e-76 / sigma^2 at most (below an ulp for sigma >=
// 1e-30) and keeps four r^2 of separations up to 1e37 within recip_n's range.
constexpr double kGaussR2Floor = 1e-76;

// L2P: h = sum_k le[k] z^k by Horner from the top term (terms >= p are zero),
// each step h = h z + le[k] as four fused multiply-adds.
template <int P>
__device__ __forceinline__ void l2p_horner(const cd* le, double zx, double zy, double& hx, double& hy)
{
    hx = le[P - 1].x;
    hy = le[P - 1].y;
#pragma unroll
    for (int k = P - 2; k >= 0; --k) {
        const cd t = le[k];
        const double nx = fma(hx, zx, fma(-hy, zy, t.x));
        hy = fma(hx, zy, fma(hy, zx, t.y));
        hx = nx;
    }
}

constexpr int kNearStage = 256;    // staged sources per chunk and wavefront

// Orders one wavefront's LDS writes before its later LDS reads (the lanes of
// a wavefront run in lockstep, so this is all the synchronisation needed).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int kR = 4;              // most targets per lane

// Sum over staged sources jb + si, jb = 0, S, 2S, ... < cnt for the R
// targets a lane owns.  FP32 leaf-relative form: coordinates in leaf widths,
// exp(-t) = 2^(-t log2 e) with c2 = w^2 log2(e) / (2 sigma^2).  The singular
// kernel of eq. 7 has no Gaussian factor.  (No Lennard-Jones form in FP32.)
template <int R, int KER>
__device__ __forceinline__ void p2p_f32(const float4* __restrict__ src, int cnt, int S, int si, float c2,
                                        const float* ox, const float* oy, float* fx, float* fy)
{
#pragma unroll 2
    for (int jb = 0; jb < cnt; jb += S) {
        const float4 t = src[jb + si];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const float dx = ox[r] - t.x, dy = oy[r] - t.y;
            float q2;
            if constexpr (KER == kNearSingular) {
                // a select, not a guard term: gamma / guard would overflow
                // for large circulations and the product with dx = 0 give NaN
                const float r2 = fmaf(dx, dx, dy * dy);
                q2 = r2 > 0.0f ? t.z * __builtin_amdgcn_rcpf(r2) : 0.0f;
            } else {
                // > 0 for coincident points, whose term is then 0 through 1 - e = 0
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, 1e-30f));
                const float e = __builtin_amdgcn_exp2f(-r2 * c2);
                q2 = fmaf(-t.z, e, t.z) * __builtin_amdgcn_rcpf(r2);
            }
            fx[r] = fmaf(q2, dx, fx[r]);
            fy[r] = fmaf(-q2, dy, fy[r]);
        }
    }
}

// Lennard-Jones pair term -V'(r) / r = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2 for
// 0 < r < rc, else 0 (a select, so the infinities of r = 0 never reach the
// sums).
__device__ __forceinline__ double lj_term(double r2, const PairK& k)
{
    const double ir2 = recip(r2);
    const double s2 = k.s2 * ir2;
    const double s6 = s2 * s2 * s2;
    const double f = k.e24 * s6 * fma(2.0, s6, -1.0) * ir2;
    return (r2 > 0.0 && r2 < k.rc2) ? f : 0.0;
}

template <int R, int KER>
__device__ __forceinline__ void p2p_f64(const Src64* __restrict__ src, int cnt, int S, int si, const PairK& k,
                                        const double* x, const double* y, double* ax, double* ay)
{
    if constexpr (KER == kNearGauss) {
        // the R targets' 1 / r^2 share one hardware reciprocal
        for (int jb = 0; jb < cnt; jb += S) {
            const Src64 t = src[jb + si];
            double dx[R], dy[R], r2[R], ir[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                dx[r] = x[r] - t.x;
                dy[r] = y[r] - t.y;
                r2[r] = fma(dx[r], dx[r], fma(dy[r], dy[r], kGaussR2Floor));
            }
            recip_n<R>(r2, ir);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double q2 = g_one_minus_exp2(r2[r] * k.nl2, t.g) * ir[r];
                ax[r] = fma(q2, dx[r], ax[r]);
                ay[r] = fma(-q2, dy[r], ay[r]);
            }
        }
        return;
    }
    for (int jb = 0; jb < cnt; jb += S) {
        const Src64 t = src[jb + si];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double dx = x[r] - t.x, dy = y[r] - t.y;
            double q2;
            if constexpr (KER == kNearLJ) {
                q2 = lj_term(fma(dx, dx, dy * dy), k);   // gamma takes no part
            } else {
                // coincident points by a select: a guard term in r2 would
                // let gamma / guard overflow for large circulations
                const double r2 = fma(dx, dx, dy * dy);
                q2 = r2 > 0.0 ? t.g * recip(r2) : 0.0;
            }
            ax[r] = fma(q2, dx, ax[r]);
            ay[r] = fma(-q2, dy, ay[r]);
        }
    }
}

// What one wavefront needs to know about its target leaf.
struct LeafCtx {
    uint32_t m;                 // z-order index of the target leaf
    int s0, nt;                 // its sorted particle range
    int nbeg[9], npre[10];      // the 3 x 3 neighbourhood: starts and running counts
    int R, TG, S;               // targets per lane, target groups, source slices (TG S <= 64)
    int chunk;                  // staged sources per chunk: a multiple of S, at most kNearStage
    double cx, cy, s;           // leaf centre, 1/leaf width
    float c2;                   // w^2 log2(e) / (2 sigma^2)
    PairK k;                    // the pair kernel's constants
};

constexpr int kStageSlots = kNearStage / 64;   // staged sources per lane and chunk

// All targets of one leaf, in chunks of T = R TG: lane (slice si, group tg)
// owns targets tg + TG r (r < R) of the chunk and sums them over the staged
// sources si, si + S, ...; lanes past TG S repeat slice 0's work and are
// left out of the sums.
// le_sh: this wavefront's LDS copy of the leaf's local expansion (P terms).
// sink != nullptr: the near-field sums (physical units, before the 1 / 2 pi)
// go to sink[i] for target i of the leaf instead of being finished here.
// tx, ty: the targets' sorted positions (the particles' own for the particle
// sum), perm: their sorted position -> output index.
template <int P, bool MIXED, int R, int KER>
__device__ __forceinline__ void leaf_near_far(const LeafCtx& c, int lane, void* stage_raw, cd* le_sh, int has_far,
                                              const double* __restrict__ tx, const double* __restrict__ ty,
                                              const double* __restrict__ xs, const double* __restrict__ ys,
                                              const double* __restrict__ gs, const float4* __restrict__ pk,
                                              const uint32_t* __restrict__ perm, const cd* __restrict__ le_leaf,
                                              cd* sink, double* __restrict__ u, double* __restrict__ v)
{
    using Stage = typename std::conditional<MIXED, float4, Src64>::type;
    Stage* src = static_cast<Stage*>(stage_raw);
    const int TG = c.TG;             // target groups
    const int S = c.S;               // source slices
    const int T = R * TG;            // targets per chunk
    // lane / TG without an integer division: the float quotient is within
    // 2e-5 of lane / TG (lane < 64, TG <= 64), and a non-multiple lies at
    // least 1/64 above an integer
    const int si0 = int(float(lane) * __builtin_amdgcn_rcpf(float(TG)) + 1e-3f);
    const int tg = lane - si0 * TG;
    const int si = si0 < S ? si0 : 0;   // idle lanes shadow slice 0
    // staged chunks of whole slices' worth of sources (a multiple of S)
    const int chunk = c.chunk;
    const int tot = c.npre[9];

    // the leaf's local expansion goes through LDS (read back as broadcasts),
    // keeping P complex values out of the scalar registers
    if (has_far)
        for (int k = lane; k < P; k += 64) le_sh[k] = le_leaf[int64_t(c.m) * P + k];

    for (int c0 = 0; c0 < c.nt; c0 += T) {
        double xi[R], yi[R], ax[R], ay[R];
        float oxi[R], oyi[R], fx[R], fy[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = c0 + tg + TG * r;
            // a target past the leaf's count sits at the leaf centre, so that
            // its distances stay on the leaf's scale (its sums are dropped)
            xi[r] = c.cx; yi[r] = c.cy; oxi[r] = 0.f; oyi[r] = 0.f;
            ax[r] = 0.0; ay[r] = 0.0; fx[r] = 0.f; fy[r] = 0.f;
            if (i < c.nt) {
                if constexpr (MIXED) {
                    const float4 t = pk[c.s0 + i];
                    oxi[r] = t.x; oyi[r] = t.y;
                } else {
                    xi[r] = tx[c.s0 + i]; yi[r] = ty[c.s0 + i];
                }
            }
        }
        // slice lane si < R finishes target c0 + tg + TG si; its output slot
        // (and, in mixed mode, its FP64 position for L2P) is fetched up front
        const int il = c0 + tg + TG * si0;
        const bool own = si0 < R && il < c.nt;
        uint32_t o = 0;
        double px = 0.0, py = 0.0;
        if (own && !sink) {
            o = perm[c.s0 + il];
            if constexpr (MIXED) { px = tx[c.s0 + il]; py = ty[c.s0 + il]; }
        }

        for (int base = 0; base < tot; base += chunk) {
            const int cnt = min(chunk, tot - base);
            // every lane finds the neighbour leaf of each of its slots, then all
            // loads are issued before the first wait (one memory round trip)
            Stage val[kStageSlots];
#pragma unroll
            for (int sl = 0; sl < kStageSlots; ++sl) {
                const int k = lane + 64 * sl;
                // inert slots: no circulation; for the Gaussian kernel at the
                // leaf centre (distances on the leaf's scale), else far away
                if constexpr (MIXED) val[sl] = make_float4(1.0e4f, 1.0e4f, 0.0f, 0.0f);
                else if constexpr (KER == kNearGauss) val[sl] = Src64{c.cx, c.cy, 0.0};
                else val[sl] = Src64{1.0e10, 1.0e10, 0.0};
                if (k < cnt) {
                    const int j = base + k;             // position in the neighbourhood run
                    int delta = c.nbeg[0], q = 0;       // npre[0] = 0
#pragma unroll
                    for (int qq = 1; qq < 9; ++qq) {
                        const bool ge = j >= c.npre[qq];
                        delta = ge ? c.nbeg[qq] - c.npre[qq] : delta;
                        q = ge ? qq : q;
                    }
                    const int gi = j + delta;
                    if constexpr (MIXED) {
                        float4 t = pk[gi];
                        const int qy = (q * 11) >> 5;   // q / 3 for q < 9
                        t.x += float(q - 3 * qy - 1);   // source relative to the target leaf centre
                        t.y += float(qy - 1);
                        val[sl] = t;
                    } else {
                        val[sl] = Src64{xs[gi], ys[gi], gs[gi]};
                    }
                }
            }
            wave_sync();
#pragma unroll
            for (int sl = 0; sl < kStageSlots; ++sl) {
                const int k = lane + 64 * sl;
                src[k] = val[sl];   // inert past cnt: a slice's last step reads them
            }
            wave_sync();
            if constexpr (MIXED) p2p_f32<R, KER>(src, cnt, S, si, c.c2, oxi, oyi, fx, fy);
            else p2p_f64<R, KER>(src, cnt, S, si, c.k, xi, yi, ax, ay);
        }

        // combine the S slices through the staging area: every slice lane
        // writes its partial sums, and the lane that finishes target r of a
        // group adds the S partial sums in slice order.  (Cross-lane xor
        // shuffles, log2(S) rounds per target and component, measured slower
        // for every layout of the C2, C3 and C5 workloads.)
        double sx[R], sy[R];
        {
            using Part = typename std::conditional<MIXED, float2, cd>::type;
            Part* red = static_cast<Part*>(stage_raw);   // S TG R partial sums: within the staging area
            wave_sync();                                 // every lane is done with the staged sources
            if (si0 < S) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (MIXED) red[(si0 * TG + tg) * R + r] = make_float2(fx[r], fy[r]);
                    else red[(si0 * TG + tg) * R + r] = cd{ax[r], ay[r]};
                }
            }
            wave_sync();
            const int rr = si0 < R ? si0 : 0;            // the target this lane may finish
            double vx = 0.0, vy = 0.0;
            if constexpr (MIXED) {
                float fxs = 0.f, fys = 0.f;
                for (int k = 0; k < S; ++k) {
                    const float2 t = red[(k * TG + tg) * R + rr];
                    fxs += t.x;
                    fys += t.y;
                }
                vx = double(fxs) * c.s;
                vy = double(fys) * c.s;
            } else {
                for (int k = 0; k < S; ++k) {
                    const cd t = red[(k * TG + tg) * R + rr];
                    vx += t.x;
                    vy += t.y;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                sx[r] = vx;
                sy[r] = vy;
            }
            wave_sync();                                 // before the area is staged again
        }
        if (own) {
            double accx = sx[0], accy = sy[0];
            if constexpr (!MIXED) { px = xi[0]; py = yi[0]; }
#pragma unroll
            for (int r = 1; r < R; ++r)
                if (si0 == r) {
                    accx = sx[r];
                    accy = sy[r];
                    if constexpr (!MIXED) { px = xi[r]; py = yi[r]; }
                }
            if (sink) {
                sink[il] = cd{accx, accy};
                continue;
            }
            if (has_far) {
                const double zx = (px - c.cx) * c.s, zy = (py - c.cy) * c.s;
                double hx, hy;
                l2p_horner<P>(le_sh, zx, zy, hx, hy);
                accx = fma(hx, c.s, accx);
                accy = fma(hy, c.s, accy);
            }
            if constexpr (KER == kNearLJ) {    // the force (Fx, Fy) = (sum q dx, sum q dy)
                u[o] = accx;
                v[o] = -accy;
            } else {
                u[o] = accy * kInv2Pi;
                v[o] = accx * kInv2Pi;
            }
        }
    }
}

// The blocking of a leaf of nt targets: ceil(nt / 64) chunks of equal size
// t <= 64, blocked as the plan's table says for t (bt: R, TG, S, each 65
// bytes, indexed by t).
__device__ __forceinline__ void set_blocking(LeafCtx& c, const uint8_t* __restrict__ bt)
{
    int t = c.nt > 0 ? c.nt : 1;
    if (t > 64) {
        const int chunks = (t + 63) >> 6;
        t = (t + chunks - 1) / chunks;
    }
    c.R = bt[t];
    c.TG = bt[65 + t];
    c.S = bt[130 + t];
    c.chunk = (kNearStage / c.S) * c.S;
}

// Context of leaf m of an instance: its range and its 3 x 3 neighbourhood,
// row by row (clipped leaves are empty; with no_siblings, so are the other
// three leaves of its quad).
__device__ __forceinline__ void make_ctx(LeafCtx& c, uint32_t m, int L, const int32_t* __restrict__ leaf_start,
                                         const Domain& d, const PairK& k, bool no_siblings,
                                         const uint8_t* __restrict__ bt)
{
    c.k = k;
    c.m = m;
    c.s0 = leaf_start[m];
    c.nt = leaf_start[m + 1] - c.s0;
    const int a = int(morton_x(m)), b = int(morton_y(m)), side = 1 << L;
    c.npre[0] = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int na = a + (q % 3) - 1, nb = b + (q / 3) - 1;
        int cnt = 0, beg = 0;
        const bool sib = no_siblings && (na >> 1) == (a >> 1) && (nb >> 1) == (b >> 1);
        if (na >= 0 && nb >= 0 && na < side && nb < side && !sib) {
            const uint32_t sm = morton(uint32_t(na), uint32_t(nb));
            beg = leaf_start[sm];
            cnt = leaf_start[sm + 1] - beg;
        }
        c.nbeg[q] = beg;
        c.npre[q + 1] = c.npre[q] + cnt;
    }
    set_blocking(c, bt);
    const double w = ldexp(d.W, -L);
    c.cx = d.x0 + (double(a) + 0.5) * w;
    c.cy = d.y0 + (double(b) + 0.5) * w;
    c.s = d.s;
    // leaf-width units: |z|^2 / (2 sigma^2) = |zhat|^2 w^2 / (2 sigma^2), and
    // exp(-t) = 2^(-t log2(e)); w = 1/s
    c.c2 = float(-k.nl2 / (d.s * d.s));
}

// register blocking pays once a chunk is full; sparse leaves keep one target
// per lane (fewer slices to combine)
template <int P, bool MIXED, int KER>
__device__ __forceinline__ void leaf_dispatch(const LeafCtx& c, int lane, void* st, cd* lsh, int has_far,
                                              const double* __restrict__ tx, const double* __restrict__ ty,
                                              const double* __restrict__ xs, const double* __restrict__ ys,
                                              const double* __restrict__ gs, const float4* __restrict__ pk,
                                              const uint32_t* __restrict__ perm, const cd* __restrict__ le_leaf,
                                              cd* sink, double* __restrict__ u, double* __restrict__ v)
{
    if (c.R == 4)
        leaf_near_far<P, MIXED, 4, KER>(c, lane, st, lsh, has_far, tx, ty, xs, ys, gs, pk, perm, le_leaf, sink, u, v);
    else if (c.R == 2)
        leaf_near_far<P, MIXED, 2, KER>(c, lane, st, lsh, has_far, tx, ty, xs, ys, gs, pk, perm, le_leaf, sink, u, v);
    else
        leaf_near_far<P, MIXED, 1, KER>(c, lane, st, lsh, has_far, tx, ty, xs, ys, gs, pk, perm, le_leaf, sink, u, v);
}

// Quads of sibling leaves: the four leaves of a 2 x 2 block touch each other,
// so every pair of particles inside a quad is a near pair of both of its
// particles, and the kernel is odd (K(-z) = -K(z)).  A workgroup of four
// wavefronts owns one quad of at most kQuadMax particles, staged with one
// particle per lane; wavefront w takes the rotations s = 8w + 1 .. 8w + 8
// (s = 32 on the lower half of the lanes only), lane i meeting particle
// (i + s) mod 64 once and handing the reverse term to that lane by a
// cross-lane shuffle.  Each unordered pair is evaluated once; the five
// neighbours outside the quad are summed per leaf as before.  All partial
// sums meet in LDS and are added in a fixed order, so the result does not
// depend on scheduling.  FP64 only: in the mixed form a pair costs a third as
// much, and the staging, barriers and shuffles measured slower than the work
// they save.
constexpr int kQuadMax = 64;

template <int KER>
__device__ __forceinline__ void quad_pairs(const Src64* qsh, int lane, int w, const PairK& k, double& sx, double& sy)
{
    const Src64 me = qsh[lane];
    double ax = 0.0, ay = 0.0;
    auto step = [&](int s, bool act) {
        const Src64 t = qsh[(lane + s) & 63];
        const double dx = me.x - t.x, dy = me.y - t.y;
        double qi, qj;
        if constexpr (KER == kNearLJ) {       // no circulation; the padding lies out of range
            const double q = lj_term(fma(dx, dx, dy * dy), k);
            qi = act ? q : 0.0;
            qj = qi;
        } else {
            const double r2 = fma(dx, dx, dy * dy);
            const double q = r2 > 0.0 ? recip(r2) : 0.0;
            qi = act ? t.g * q : 0.0;
            qj = act ? me.g * q : 0.0;
        }
        ax = fma(qi, dx, ax);
        ay = fma(-qi, dy, ay);
        const int from = (lane - s) & 63;
        ax += __shfl(-qj * dx, from, 64);
        ay += __shfl(qj * dy, from, 64);
    };
    if constexpr (KER == kNearGauss) {
        // rotations s0 and s0 + 1 together: their 1 / r^2 share one reciprocal
        auto step2 = [&](int s0, bool act1) {
            const Src64 t0 = qsh[(lane + s0) & 63], t1 = qsh[(lane + s0 + 1) & 63];
            const double dx0 = me.x - t0.x, dy0 = me.y - t0.y;
            const double dx1 = me.x - t1.x, dy1 = me.y - t1.y;
            double r2[2], ir[2];
            r2[0] = fma(dx0, dx0, fma(dy0, dy0, kGaussR2Floor));
            r2[1] = fma(dx1, dx1, fma(dy1, dy1, kGaussR2Floor));
            recip_n<2>(r2, ir);
            const double q0 = g_one_minus_exp2(r2[0] * k.nl2, 1.0) * ir[0];
            const double q1 = g_one_minus_exp2(r2[1] * k.nl2, 1.0) * ir[1];
            const double qi0 = t0.g * q0, qj0 = me.g * q0;
            const double qi1 = act1 ? t1.g * q1 : 0.0, qj1 = act1 ? me.g * q1 : 0.0;
            ax = fma(qi0, dx0, ax);
            ay = fma(-qi0, dy0, ay);
            ax += __shfl(-qj0 * dx0, (lane - s0) & 63, 64);
            ay += __shfl(qj0 * dy0, (lane - s0) & 63, 64);
            ax = fma(qi1, dx1, ax);
            ay = fma(-qi1, dy1, ay);
            ax += __shfl(-qj1 * dx1, (lane - s0 - 1) & 63, 64);
            ay += __shfl(qj1 * dy1, (lane - s0 - 1) & 63, 64);
        };
        for (int k = 0; k < 4; ++k) step2(8 * w + 1 + 2 * k, w != 3 || k != 3 || lane < 32);
    } else {
        for (int k = 0; k < (w == 3 ? 7 : 8); ++k) step(8 * w + 1 + k, true);
        if (w == 3) step(32, lane < 32);
    }
    sx = ax;
    sy = ay;
}

// WAVES wavefronts per workgroup, one leaf each (four: one quad); the work
// table gives every instance ceil(4^L / WAVES) workgroups.
template <int P, bool MIXED, int WAVES, int KER>
__global__ void __launch_bounds__(64 * WAVES)
k_p2p_l2p(Work wk, int n_inst, const Inst* __restrict__ inst, const int32_t* __restrict__ leaf_start_all,
          const double* __restrict__ xs, const double* __restrict__ ys, const double* __restrict__ gs,
          const float4* __restrict__ pk, const uint32_t* __restrict__ perm, const cd* __restrict__ le_all,
          PairK kp, const uint8_t* __restrict__ bt, double* __restrict__ u, double* __restrict__ v)
{
    using Stage = typename std::conditional<MIXED, float4, Src64>::type;
    constexpr bool kQuads = WAVES == 4 && !MIXED;
    __shared__ Stage stage_all[WAVES][kNearStage];
    __shared__ cd le_all_sh[WAVES][P];
    __shared__ Src64 qsh[kQuads ? kQuadMax : 1];
    __shared__ cd part_sh[kQuads ? 5 : 1][kQuads ? kQuadMax : 1];   // outside, then the 4 rotation groups

    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t blk = flat_block();
    if (blk >= wk.wg_begin[n_inst]) return;                        // past the last row's end
    const int pos = find_inst(wk.wg_begin, n_inst, int(blk));      // place in the launch order
    const int qi = wk.order[pos];
    const int L = inst[qi].L;
    const int has_far = KER != kNearLJ && L >= 2 ? 1 : 0;   // Lennard-Jones: no far field
    const int32_t* leaf_start = leaf_start_all + inst[qi].leaf_off;
    const cd* le_leaf = le_all + (inst[qi].box_off + level_offset(L)) * P;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const int64_t mm = (blk - wk.wg_begin[pos]) * WAVES + wv;
    const Domain d = inst[qi].dom;
    void* st = stage_all[wv];
    cd* lsh = le_all_sh[wv];

    // quad path: a whole quad (L >= 1) of 2 .. kQuadMax particles; the same
    // decision in every wavefront of the workgroup
    int sq = 0, nq = 0;
    if constexpr (kQuads) {
        if (L >= 1) {
            const int64_t m0 = mm - wv;
            sq = leaf_start[m0];
            nq = leaf_start[m0 + 4] - sq;
        }
    }
    if (!(kQuads && nq > 1 && nq <= kQuadMax)) {
        if (mm >= nleaf) return;
        LeafCtx c;
        make_ctx(c, uint32_t(mm), L, leaf_start, d, kp, false, bt);
        if (c.nt == 0) return;
        leaf_dispatch<P, MIXED, KER>(c, lane, st, lsh, has_far, xs, ys, xs, ys, gs, pk, perm, le_leaf, nullptr, u, v);
        return;
    }

    LeafCtx c;
    make_ctx(c, uint32_t(mm), L, leaf_start, d, kp, true, bt);
    // stage the quad, one particle per lane; past nq inert padding without
    // circulation: for the Gaussian kernel on the last particle (distances
    // stay on the quad's scale), else far away
    if (wv == 0) {
        const int i = sq + min(lane, nq - 1);
        const Src64 pad = KER == kNearGauss ? Src64{xs[i], ys[i], 0.0} : Src64{1.0e10, 1.0e10, 0.0};
        qsh[lane] = lane < nq ? Src64{xs[i], ys[i], gs[i]} : pad;
    }
    __syncthreads();
    // the leaf's targets against the neighbours outside the quad
    if (c.nt > 0)
        leaf_dispatch<P, MIXED, KER>(c, lane, st, lsh, 0, xs, ys, xs, ys, gs, pk, perm, le_leaf,
                                     part_sh[0] + (c.s0 - sq), u, v);
    // this wavefront's share of the pairs inside the quad
    double ix, iy;
    quad_pairs<KER>(qsh, lane, wv, kp, ix, iy);
    part_sh[1 + wv][lane] = cd{ix, iy};
    __syncthreads();
    if (c.nt == 0) return;
    if (has_far)
        for (int k = lane; k < P; k += 64) lsh[k] = le_leaf[int64_t(c.m) * P + k];
    wave_sync();
    if (lane < c.nt) {
        const int j = c.s0 - sq + lane;
        double accx = part_sh[0][j].x, accy = part_sh[0][j].y;
#pragma unroll
        for (int g = 1; g < 5; ++g) {
            accx += part_sh[g][j].x;
            accy += part_sh[g][j].y;
        }
        const int i = c.s0 + lane;
        if (has_far) {
            const double zx = (xs[i] - c.cx) * c.s, zy = (ys[i] - c.cy) * c.s;
            double hx, hy;
            l2p_horner<P>(lsh, zx, zy, hx, hy);
            accx = fma(hx, c.s, accx);
            accy = fma(hy, c.s, accy);
        }
        const uint32_t o = perm[i];
        if constexpr (KER == kNearLJ) {
            u[o] = accx;
            v[o] = -accy;
        } else {
            u[o] = accy * kInv2Pi;
            v[o] = accx * kInv2Pi;
        }
    }
}

// Target points (eq. 1 with targets distinct from the sources): one
// wavefront per leaf of the points' tree, its points against the particles
// of the 3 x 3 neighbourhood, plus L2P from the leaf's local expansion.
// Single instance, FP64.
template <int P, int KER>
__global__ void __launch_bounds__(256)
k_p2p_at(int L, const Inst* __restrict__ inst, const int32_t* __restrict__ leaf_start,
         const int32_t* __restrict__ tleaf_start, const double* __restrict__ xs, const double* __restrict__ ys,
         const double* __restrict__ gs, const double* __restrict__ txs, const double* __restrict__ tys,
         const uint32_t* __restrict__ tperm, const cd* __restrict__ le_all, PairK kp, const uint8_t* __restrict__ bt,
         double* __restrict__ u, double* __restrict__ v)
{
    __shared__ Src64 stage_all[4][kNearStage];
    __shared__ cd le_all_sh[4][P];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t mm = flat_block() * 4 + wv;
    if (mm >= (int64_t(1) << (2 * L))) return;
    LeafCtx c;
    make_ctx(c, uint32_t(mm), L, leaf_start, inst[0].dom, kp, false, bt);   // the particles around the leaf
    c.s0 = tleaf_start[mm];                                                    // and the leaf's points
    c.nt = tleaf_start[mm + 1] - c.s0;
    if (c.nt == 0) return;
    set_blocking(c, bt);
    const cd* le_leaf = le_all + (inst[0].box_off + level_offset(L)) * P;
    leaf_dispatch<P, false, KER>(c, lane, stage_all[wv], le_all_sh[wv], L >= 2 ? 1 : 0, txs, tys, xs, ys, gs,
                                 nullptr, tperm, le_leaf, nullptr, u, v);
}

// The pair kernel's constants from the plan's choice.
PairK pair_constants(const NearKernel& nk)
{
    PairK k{};
    if (nk.kind == kNearGauss) {
        const double l2 = 1.4426950408889634074 / (2.0 * nk.sigma * nk.sigma);
        k.nl2 = -l2;
    }
    if (nk.kind == kNearLJ) {
        k.s2 = nk.sigma * nk.sigma;
        k.rc2 = nk.cutoff * nk.cutoff;
        k.e24 = 24.0 * nk.eps;
    }
    return k;
}

template <int P, int WAVES, int KER>
void p2p_launch(const Buffers& b, const Work& w, int nwg, bool mixed, const PairK& k, const uint8_t* bt, double* u,
                double* v, hipStream_t st)
{
    if constexpr (KER != kNearLJ) {
        if (mixed) {
            hipLaunchKernelGGL((k_p2p_l2p<P, true, WAVES, KER>), row_grid(nwg), dim3(64 * WAVES), 0, st, w,
                               b.n_inst, b.inst, b.leaf_start, b.xs, b.ys, b.gs, b.pk, b.perm, b.le, k, bt, u, v);
            return;
        }
    }
    hipLaunchKernelGGL((k_p2p_l2p<P, false, WAVES, KER>), row_grid(nwg), dim3(64 * WAVES), 0, st, w, b.n_inst,
                       b.inst, b.leaf_start, b.xs, b.ys, b.gs, b.pk, b.perm, b.le, k, bt, u, v);
}

template <int P, int WAVES>
void p2p_kernel(const Buffers& b, const Work& w, int nwg, bool mixed, const NearKernel& nk, const uint8_t* bt,
                double* u, double* v, hipStream_t st)
{
    const PairK k = pair_constants(nk);
    if (nk.kind == kNearSingular) p2p_launch<P, WAVES, kNearSingular>(b, w, nwg, mixed, k, bt, u, v, st);
    else if (nk.kind == kNearLJ) p2p_launch<P, WAVES, kNearLJ>(b, w, nwg, mixed, k, bt, u, v, st);
    else p2p_launch<P, WAVES, kNearGauss>(b, w, nwg, mixed, k, bt, u, v, st);
}

template <int P>
hipError_t p2p_waves(const Buffers& b, const Work& w, int nwg, int waves, bool mixed, const NearKernel& nk,
                     const uint8_t* bt, double* u, double* v, hipStream_t st)
{
    if (nwg <= 0) return hipSuccess;
    if (waves != 2 && waves != 4) return hipErrorInvalidValue;
    if (nk.kind != kNearGauss && nk.kind != kNearSingular && nk.kind != kNearLJ) return hipErrorInvalidValue;
    if (mixed && nk.kind == kNearLJ) return hipErrorInvalidValue;
    if (waves == 2) p2p_kernel<P, 2>(b, w, nwg, mixed, nk, bt, u, v, st);
    else p2p_kernel<P, 4>(b, w, nwg, mixed, nk, bt, u, v, st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_p2p_at(const Buffers& b, int P, int L, const NearKernel& nk, int block, double* u, double* v,
                         hipStream_t st)
{
    const uint8_t* bt = b.blk_tab + block * kBlockTabBytes;
    if (nk.kind != kNearGauss && nk.kind != kNearSingular) return hipErrorInvalidValue;
    const bool singular = nk.kind == kNearSingular;
    const PairK kp = pair_constants(nk);
    const dim3 grid = row_grid(((int64_t(1) << (2 * L)) + 3) / 4);
#define FMM_AT_CASE(PP)                                                                                            \
    case PP:                                                                                                       \
        if (singular)                                                                                              \
            hipLaunchKernelGGL((k_p2p_at<PP, kNearSingular>), grid, dim3(256), 0, st, L, b.inst, b.leaf_start,    \
                               b.tleaf_start, b.xs, b.ys, b.gs, b.txs, b.tys, b.tperm, b.le, kp, bt, u, v);        \
        else                                                                                                       \
            hipLaunchKernelGGL((k_p2p_at<PP, kNearGauss>), grid, dim3(256), 0, st, L, b.inst, b.leaf_start,       \
                               b.tleaf_start, b.xs, b.ys, b.gs, b.txs, b.tys, b.tperm, b.le, kp, bt, u, v);        \
        return hipGetLastError();
    switch (P) {
        FMM_AT_CASE(8)
        FMM_AT_CASE(12)
        FMM_AT_CASE(16)
        FMM_AT_CASE(17)
        FMM_AT_CASE(20)
        FMM_AT_CASE(24)
        FMM_AT_CASE(32)
        default: return hipErrorInvalidValue;
    }
#undef FMM_AT_CASE
}

// Blocking table of a policy: 0 pads a chunk's targets to a power of two T
// (R = 4 at T = 64, 2 at T = 32, 1 below; TG = T / R, S = 64 / TG); 1 keeps
// the most lanes on real pairs, t S / (64 R) with TG = ceil(t / R) and S =
// floor(64 / TG), the larger R on a tie.
void block_table(int policy, uint8_t* out)
{
    for (int t = 0; t <= 64; ++t) {
        int R = 1, TG = 1, S = 64;
        if (t > 0 && policy == 0) {
            int T = 1;
            while (T < t) T <<= 1;
            R = T >= 64 ? 4 : (T == 32 ? 2 : 1);
            TG = T / R;
            S = 64 / TG;
        } else if (t > 0) {
            int bR = 1, bTG = t, bS = 64 / t;
            for (int r = 2; r <= 4; r <<= 1) {
                const int tg = (t + r - 1) / r, sl = 64 / tg;
                if (t * sl * bR >= t * bS * r) {
                    bR = r;
                    bTG = tg;
                    bS = sl;
                }
            }
            R = bR;
            TG = bTG;
            S = bS;
        }
        out[t] = uint8_t(R);
        out[65 + t] = uint8_t(TG);
        out[130 + t] = uint8_t(S);
    }
}

hipError_t launch_p2p(const Buffers& b, int P, const Work& w, int nwg, int waves, bool mixed, const NearKernel& nk,
                      int block, double* u, double* v, hipStream_t st)
{
    const uint8_t* bt = b.blk_tab + block * kBlockTabBytes;
    switch (P) {
        case 8: return p2p_waves<8>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 12: return p2p_waves<12>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 16: return p2p_waves<16>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 17: return p2p_waves<17>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 20: return p2p_waves<20>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 24: return p2p_waves<24>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        case 32: return p2p_waves<32>(b, w, nwg, waves, mixed, nk, bt, u, v, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fmm
