// fmm_upward.hip -- upward sweep (Section 2.2, Fig. 2): P2M at the leaves and
// M2M from every level to its parent level, down to level 2.
//
// Coefficients are scaled by the box width w_l so that the shift operators do
// not depend on the level: for a box of centre c,
//   ahat_k = sum_j gamma_j ((z_j - c) / w_l)^k,        k = 0 .. p-1,
// which is the textbook multipole expansion of 1/z, phi(z) = sum_k a_k /
// (z - c)^(k+1), with a_k = ahat_k w_l^k.  The M2M shift from a child in
// position c (delta = (c_child - c_parent) / w_parent = (+-1 +- i)/4) reads
//   ahat^P_k = sum_{m<=k} C(k,m) 2^-m delta^(k-m) ahat^child_m,
// the moments 2^-m ahat^child_m translated by delta (the same for every
// level).
//
// What is stored is abar_k = s_k ahat_k, s_k = (-1)^(k+1) / k! (the input
// scaling of the factored M2L, which then reads the coefficients as they
// are): P2M multiplies by s_k once.  M2M undoes the scaling and multiplies
// by the exact 2^-m and by delta^-m (one table entry per m and child
// position), forms the binomial sums sum_{m<=k} C(k,m) u_m in registers
// (additions only, no matrix), multiplies term k by delta^k (exact), and
// scales the sum of the four children by s_k again.  (P = 32, whose P complex registers would not fit beside
// the rest, keeps the operator matrices, built for abar: S M S^-1, entries
// (-1)^(k-m) 2^-m delta^(k-m) / (k-m)!, read from LDS.)
//
// Storage: every box holds P >= p coefficients (P the compiled expansion
// size), terms k >= p zero; the operator rows k >= p are zero as well, so
// the padding stays zero and no loop needs the runtime p.
//
// Subtree fusion: z-order makes the descendants of a box at any level one
// contiguous run of boxes, so a workgroup that owns a box at level lt can
// build up to three levels below it (64 + 16 + 4 + 1 boxes) in LDS and write
// every level out for M2L.  The sweep is a handful of launches (levels
// L -> L-3 -> ... -> 2) instead of one per level, and no level waits for a
// grid-wide barrier inside a launch.
#include "fmm_device.h"

namespace fmm {
namespace {

constexpr int kUpThreads = 256;
constexpr int kP2MLanes = 4;            // threads per leaf in P2M

// z^N (N >= 1, a constant) by repeated squaring
template <int N>
__device__ __forceinline__ void cpow(double zx, double zy, double& rx, double& ry)
{
    double bx = zx, by = zy;
    bool first = true;
#pragma unroll
    for (int n = N; n > 0; n >>= 1) {
        if (n & 1) {
            if (first) {
                rx = bx;
                ry = by;
                first = false;
            } else {
                const double tx = rx * bx - ry * by;
                ry = rx * by + ry * bx;
                rx = tx;
            }
        }
        if (n > 1) {
            const double tx = bx * bx - by * by;
            by = 2.0 * bx * by;
            bx = tx;
        }
    }
}

constexpr int kP2MTerms = 12;           // expansion terms per P2M pass (a multiple of kP2MLanes)

// v from the lane whose index differs in bit log2(M) (M = 1, 2), within
// aligned groups of four lanes, by two 32-bit quad permutes
template <int M>
__device__ __forceinline__ double quad_xor(double v)
{
    constexpr int kCtrl = M == 1 ? 0xB1 : 0x4E;     // quad_perm [1,0,3,2] or [2,3,0,1]
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), kCtrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// P2M terms k0 .. k0 + NT - 1 of one leaf: this thread sums particles j0,
// j0 + 4, ... < s1 (the four threads of the leaf start at its first four),
// the quad adds the four sums, and thread r writes the terms k = r mod 4,
// scaled by s_k, to LDS (shrow) and to the leaf's expansion (dst).
template <int P, int K0>
__device__ __forceinline__ void p2m_block(const double* __restrict__ xs, const double* __restrict__ ys,
                                          const double* __restrict__ gs, int j0, int s1, int r, double cx,
                                          double cy, double s, const double* __restrict__ sk, cd* shrow,
                                          cd* __restrict__ dst)
{
    constexpr int NT = P - K0 < kP2MTerms ? P - K0 : kP2MTerms;
    static_assert(K0 % kP2MLanes == 0, "blocks start at a multiple of the quad");
    double ax[NT], ay[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) { ax[k] = 0.0; ay[k] = 0.0; }
    constexpr int kBatch = 2;               // particles of one thread whose loads are issued together
    for (; j0 < s1; j0 += kBatch * kP2MLanes) {
        double bxp[kBatch], byp[kBatch], bgp[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            // past the end: reload the last particle with zero circulation
            const int j = min(j0 + kP2MLanes * u, s1 - 1);
            bxp[u] = xs[j];
            byp[u] = ys[j];
            bgp[u] = j0 + kP2MLanes * u < s1 ? gs[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const double zx = (bxp[u] - cx) * s, zy = (byp[u] - cy) * s;
            double px = bgp[u], py = 0.0;
            if constexpr (K0 > 0) {
                double kx, ky;
                cpow<K0>(zx, zy, kx, ky);
                px = bgp[u] * kx;
                py = bgp[u] * ky;
            }
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                ax[k] += px;
                ay[k] += py;
                const double nx = px * zx - py * zy;
                py = px * zy + py * zx;
                px = nx;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        ax[k] += quad_xor<1>(ax[k]);
        ay[k] += quad_xor<1>(ay[k]);
        ax[k] += quad_xor<2>(ax[k]);
        ay[k] += quad_xor<2>(ay[k]);
    }
    // thread r writes k = k0 + r, k0 + r + 4, ... (picked by selects, not branches)
#pragma unroll
    for (int q = 0; q < (NT + kP2MLanes - 1) / kP2MLanes; ++q) {
        double vx = ax[kP2MLanes * q], vy = ay[kP2MLanes * q];
#pragma unroll
        for (int c = 1; c < kP2MLanes; ++c) {
            if (kP2MLanes * q + c < NT) {
                vx = r == c ? ax[kP2MLanes * q + c] : vx;
                vy = r == c ? ay[kP2MLanes * q + c] : vy;
            }
        }
        const int k = K0 + kP2MLanes * q + r;
        if (kP2MLanes * q + r < NT) {
            const double sc = sk[k];                // s_k; zero for k >= p
            const cd val = cd{vx * sc, vy * sc};
            shrow[k] = val;
            dst[k] = val;
        }
    }
}

// Workgroup = one box at level lt = lb - d (d <= 3) of one instance (work
// table arg: lt, d).  from_particles: the 4^d boxes of level lb are leaves
// and get their expansion from P2M; otherwise they are read from global
// memory, all loads issued before the first wait.  LDS holds one level at a
// time: thread t shifts child t in place, then the threads of the parents'
// coefficients add the four children (in child order) and, after a barrier,
// write the parents over their input.  The kernel is held to 128 VGPRs:
// four workgroups fit on a CU, so a launch of 4 x 256 workgroups runs in
// one round.
template <int P>
__global__ void __launch_bounds__(kUpThreads, 4)
k_upward(Work wk, int n_inst, const Inst* __restrict__ inst, int p, int from_particles,
         const int32_t* __restrict__ leaf_start_all, const double* __restrict__ xs, const double* __restrict__ ys,
         const double* __restrict__ gs, cd* __restrict__ me_all, const cd* __restrict__ M,
         const double* __restrict__ sk)
{
    constexpr bool kMatrix = P > 24;     // operator matrices in LDS instead of register shifts
    __shared__ cd sh[64 * P + 1];        // the current level of the subtree (<= 64 boxes) + a junk slot
    __shared__ cd sM[kMatrix ? 4 * P * P : 1];   // the four M2M matrices
    // the scaled shift (P <= 24): sT[c][m] = (2^-m / s_m) delta_c^-m (zero for m >= p) takes abar to
    // the moments 2^-m ahat divided by delta_c^m, whose binomial sums times sD[c][l] = delta_c^l are
    // the shifted moments
    __shared__ cd sT[kMatrix ? 1 : 4 * P], sD[kMatrix ? 1 : 4 * P];
    const int tid = threadIdx.x;
    if (int(blockIdx.x) >= wk.wg_begin[n_inst]) return;           // past the launch's work (batched plans)
    const int pos = find_inst(wk.wg_begin, n_inst, blockIdx.x);   // place in the launch order
    const int q = wk.order[pos];
    const int64_t root = blockIdx.x - wk.wg_begin[pos];     // z-order index at level lt
    const int lt = wk.arg[2 * pos], d = wk.arg[2 * pos + 1];
    const int L = inst[q].L;
    const int32_t* leaf_start = leaf_start_all + inst[q].leaf_off;
    cd* me = me_all + inst[q].box_off * P;
    if (kMatrix && d > 0)
        for (int e = tid; e < 4 * P * P; e += kUpThreads) sM[e] = M[e];
    if (!kMatrix && tid < 4 * P) {
        const int c = tid / P, m = tid % P;
        double dx, dy;
        child_delta(c, dx, dy);
        // delta^m and delta^-m = (8 conj delta)^m by repeated products: Gaussian
        // integers times powers of two, exact
        const double ix = 8.0 * dx, iy = -8.0 * dy;
        double tx = 1.0, ty = 0.0, ex = 1.0, ey = 0.0;
        for (int n = 0; n < m; ++n) {
            const double t2 = tx * ix - ty * iy;
            ty = tx * iy + ty * ix;
            tx = t2;
            const double e2 = ex * dx - ey * dy;
            ey = ex * dy + ey * dx;
            ex = e2;
        }
        const double f = sk[m] != 0.0 ? ldexp(1.0 / sk[m], -m) : 0.0;
        sT[tid] = cd{tx * f, ty * f};
        sD[tid] = cd{ex, ey};
    }
    const int lb = lt + d;
    const int nb = 1 << (2 * d);         // boxes at level lb under this root
    const int64_t first = root << (2 * d);

    // ---- level lb into sh[0 .. nb*P) ----
    if (from_particles) {
        const Domain dm = inst[q].dom;
        const double w = ldexp(dm.W, -L);
        if constexpr (P <= 24) {
            // four threads per leaf take every fourth particle each, with all
            // terms of a block of kP2MTerms (g z^k by repeated products from
            // z^k0); the four partial sums meet by quad permutes, added in the
            // same order in every thread
            for (int slot = tid; slot < nb * kP2MLanes; slot += kUpThreads) {
                const int i = slot / kP2MLanes;
                const int r = slot % kP2MLanes;
                const uint32_t leaf = uint32_t(first + i);
                const double cx = dm.x0 + (double(morton_x(leaf)) + 0.5) * w;
                const double cy = dm.y0 + (double(morton_y(leaf)) + 0.5) * w;
                const int s0 = leaf_start[leaf], s1 = leaf_start[leaf + 1];
                cd* dst = me + (level_offset(L) + int64_t(leaf)) * P;
                p2m_block<P, 0>(xs, ys, gs, s0 + r, s1, r, cx, cy, dm.s, sk, sh + i * P, dst);
                if constexpr (P > kP2MTerms)
                    p2m_block<P, kP2MTerms>(xs, ys, gs, s0 + r, s1, r, cx, cy, dm.s, sk, sh + i * P, dst);
            }
        } else {
            constexpr int KR = (P + kP2MLanes - 1) / kP2MLanes;
            for (int slot = tid; slot < nb * kP2MLanes; slot += kUpThreads) {
                const int i = slot / kP2MLanes;
                const int r = slot % kP2MLanes;           // this thread owns k = r, r+4, r+8, ...
                const uint32_t leaf = uint32_t(first + i);
                const double cx = dm.x0 + (double(morton_x(leaf)) + 0.5) * w;
                const double cy = dm.y0 + (double(morton_y(leaf)) + 0.5) * w;
                double ax[KR], ay[KR];
#pragma unroll
                for (int q = 0; q < KR; ++q) { ax[q] = 0.0; ay[q] = 0.0; }
                const int s0 = leaf_start[leaf], s1 = leaf_start[leaf + 1];
                constexpr int kBatch = 8;       // particles whose loads are issued together
                for (int j0 = s0; j0 < s1; j0 += kBatch) {
                    double bxp[kBatch], byp[kBatch], bgp[kBatch];
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        // past the end: reload the last particle with zero circulation
                        const int j = min(j0 + u, s1 - 1);
                        bxp[u] = xs[j];
                        byp[u] = ys[j];
                        bgp[u] = j0 + u < s1 ? gs[j] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < kBatch; ++u) {
                        const double zx = (bxp[u] - cx) * dm.s, zy = (byp[u] - cy) * dm.s;
                        // z^2, z^3, z^4 and gamma z^r (r = this thread's first term)
                        const double z2x = zx * zx - zy * zy, z2y = 2.0 * zx * zy;
                        const double z3x = z2x * zx - z2y * zy, z3y = z2x * zy + z2y * zx;
                        const double z4x = z2x * z2x - z2y * z2y, z4y = 2.0 * z2x * z2y;
                        const double rx = r == 0 ? 1.0 : (r == 1 ? zx : (r == 2 ? z2x : z3x));
                        const double ry = r == 0 ? 0.0 : (r == 1 ? zy : (r == 2 ? z2y : z3y));
                        double px = bgp[u] * rx, py = bgp[u] * ry;
#pragma unroll
                        for (int q = 0; q < KR; ++q) {
                            ax[q] += px;
                            ay[q] += py;
                            const double nx = px * z4x - py * z4y;
                            py = px * z4y + py * z4x;
                            px = nx;
                        }
                    }
                }
                cd* dst = me + (level_offset(L) + int64_t(leaf)) * P;
#pragma unroll
                for (int q = 0; q < KR; ++q) {
                    const int k = r + kP2MLanes * q;
                    if (k < P) {
                        const double sc = sk[k];                  // s_k; zero for k >= p
                        const cd val = cd{ax[q] * sc, ay[q] * sc};
                        sh[i * P + k] = val;
                        dst[k] = val;
                    }
                }
            }
        }
    } else {
        constexpr int kIn = (64 * P + kUpThreads - 1) / kUpThreads;
        const cd* src = me + (level_offset(lb) + first) * P;
        cd in[kIn];
#pragma unroll
        for (int i = 0; i < kIn; ++i) {      // unconditional (clamped) loads, all in flight
            const int e = tid + kUpThreads * i;
            in[i] = src[e < nb * P ? e : 0];
        }
        // unconditional stores (out-of-range ones to the junk slot), so that
        // no load is sunk into a branch behind the previous one's wait
#pragma unroll
        for (int i = 0; i < kIn; ++i) {
            const int e = tid + kUpThreads * i;
            sh[e < nb * P ? e : 64 * P] = in[i];
        }
    }
    __syncthreads();

    // ---- M2M from level j+1 to level j, j = lb-1 .. lt ----
    // (at most 16 P outputs per level: kOut per thread)
    constexpr int kOut = (16 * P + kUpThreads - 1) / kUpThreads;
    int n_in = nb;
    for (int j = lb - 1; j >= lt; --j) {
        const int n_out = n_in >> 2;
        const int64_t gfirst = root << (2 * (j - lt));
        cd* gdst = me + (level_offset(j) + gfirst) * P;
        if constexpr (!kMatrix) {
            // child t: abar -> 2^-m ahat / delta^m, binomial sums (the shift
            // by delta = 1, additions only), times delta^l: the moments
            // shifted to the parent centre (all children in the first
            // wavefront: a wavefront's instruction stream costs the same
            // however few lanes are live)
            const int t = tid;
            if (t < n_in) {
                const cd* tr = sT + (t & 3) * P;
                const cd* dr = sD + (t & 3) * P;
                cd u[P];
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const cd a = sh[t * P + m];
                    const cd f = tr[m];
                    u[m] = cd{a.x * f.x - a.y * f.y, a.x * f.y + a.y * f.x};
                }
                binomial_sums<P>(u);
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const cd f = dr[m];
                    sh[t * P + m] = cd{u[m].x * f.x - u[m].y * f.y, u[m].x * f.y + u[m].y * f.x};
                }
            }
            __syncthreads();
        }
        cd res[kOut];
#pragma unroll
        for (int i = 0; i < kOut; ++i) {
            const int e = tid + kUpThreads * i;
            res[i] = cd{0.0, 0.0};
            if (e >= n_out * P) continue;
            const int o = e / P, k = e % P;
            double bx = 0.0, by = 0.0;
            if constexpr (!kMatrix) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const cd t = sh[(4 * o + c) * P + k];
                    bx += t.x;
                    by += t.y;
                }
                const double sc = sk[k];                 // zero for k >= p
                bx *= sc;
                by *= sc;
            } else {
                // the full row (entries m > k are zero): a fixed trip count
                // lets the LDS loads be issued together
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const cd* a = sh + (4 * o + c) * P;
                    const cd* Mr = sM + (c * P + k) * P;     // rows k >= p are zero
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const cd t = Mr[m];
                        const cd s = a[m];
                        cmac(bx, by, t.x, t.y, s.x, s.y);
                    }
                }
            }
            res[i] = cd{bx, by};
            gdst[e] = res[i];
        }
        if (j == lt) break;
        __syncthreads();                 // every thread has read level j+1
#pragma unroll
        for (int i = 0; i < kOut; ++i) {
            const int e = tid + kUpThreads * i;
            if (e < n_out * P) sh[e] = res[i];
        }
        __syncthreads();
        n_in = n_out;
    }
}

template <int P>
hipError_t upward_impl(const Buffers& b, int p, const Work& w, int nwg, bool leaves, hipStream_t st)
{
    if (nwg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_upward<P>, dim3(unsigned(nwg)), dim3(kUpThreads), 0, st, w, b.n_inst, b.inst, p,
                       leaves ? 1 : 0, b.leaf_start, b.xs, b.ys, b.gs, b.me, b.t_m2m, b.t_sin);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_upward(const Buffers& b, int P, int p, const Work& w, int nwg, bool from_particles,
                         hipStream_t st)
{
    switch (P) {
        case 8: return upward_impl<8>(b, p, w, nwg, from_particles, st);
        case 12: return upward_impl<12>(b, p, w, nwg, from_particles, st);
        case 16: return upward_impl<16>(b, p, w, nwg, from_particles, st);
        case 17: return upward_impl<17>(b, p, w, nwg, from_particles, st);
        case 20: return upward_impl<20>(b, p, w, nwg, from_particles, st);
        case 24: return upward_impl<24>(b, p, w, nwg, from_particles, st);
        case 32: return upward_impl<32>(b, p, w, nwg, from_particles, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fmm
