// fmm_schedule.h -- the launch schedule of one evaluation, per instance.
//
// An evaluation after the tree build is a fixed list of launches: upward
// groups (P2M, then M2M, up to three levels per launch), four M2L launches
// (FP64 / FP32 levels x levels with the interaction list split over several
// wavefronts / unsplit), downward groups (L2L, up to three levels per
// launch) and the near field.  What an instance contributes to each launch
// (its workgroup count and two launch-specific arguments) depends only on
// its depth and the plan's settings, so the same functions build the work
// tables on the host (single plans, where every size is known when the plan
// is made) and on the device (batched plans, whose instance sizes and
// depths arrive in device memory with every call).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace fmm {

enum LaunchKind { L_UP = 0, L_M2L = 1, L_DOWN = 2, L_P2P = 3 };

// One launch of the fixed list: its kind and, for a group or M2L launch,
// which one (upward / downward group index; M2L precision and part).
struct LaunchDesc {
    int kind;
    int group;      // L_UP, L_DOWN: group index from the leaves / from level 2
    int fp32;       // L_M2L: 1 for the FP32 levels of the mixed form
    int part;       // L_M2L: 0 = split levels (list over 2-3 wavefronts), 1 = unsplit
};

// Settings the schedule depends on (uniform over a plan).
struct SchedCfg {
    int mixed;           // FP32 M2L on the finest `fine` levels
    int fine;
    int split_max;       // M2L levels <= min(L, split_max) split their lists; < 2: never
    int p2p_waves;       // leaves per near-field workgroup
};

// Most launches in the fixed list: 4 upward groups, 4 M2L, 4 downward, P2P.
constexpr int kMaxLaunches = 16;
// Interaction-list wavefront split: FP64 levels of an instance with fewer
// than this many split-level tiles use three wavefronts per list, else two.
constexpr int kM2LFewTiles = 256;

__host__ __device__ inline int sched_split_level(int L, int split_max)
{
    return (L <= 2 || split_max < 2) ? 1 : (L < split_max ? L : split_max);
}

// Workgroups of one M2L level: 16 x 16 target boxes each (one below level 4).
__host__ __device__ inline int sched_level_blocks(int l)
{
    const int side = 1 << l;
    const int bpr = side >= 16 ? side / 16 : 1;
    return bpr * bpr;
}

// Upward groups of a tree of depth L: group 0 holds the leaves (P2M) and up
// to three M2M levels, the next ones three levels each, down to level 2.
__host__ __device__ inline int sched_up_groups(int L)
{
    if (L < 2) return 0;
    return L == 2 ? 1 : (L - 2 + 2) / 3;
}

// Downward groups: L2L from level 2 in groups of up to three levels, the
// remainder of (L - 2) / 3 first, so the large launches near the leaves
// cover three full levels.
__host__ __device__ inline int sched_down_groups(int L) { return L < 3 ? 0 : (L - 2 + 2) / 3; }

// Workgroups and arguments of an instance of depth L in launch d (0
// workgroups: it takes no part).
__host__ __device__ inline void sched_inst(const SchedCfg& c, const LaunchDesc& d, int L, int& wg, int& a0, int& a1)
{
    wg = 0;
    a0 = 0;
    a1 = 0;
    if (d.kind == L_UP) {
        if (L < 2) return;
        int lb = L, lt = L - 3 > 2 ? L - 3 : 2, k = 0;
        while (k < d.group && lt > 2) {
            lb = lt;
            lt = lb - 3 > 2 ? lb - 3 : 2;
            ++k;
        }
        if (k < d.group) return;
        wg = 1 << (2 * lt);
        a0 = lt;
        a1 = lb - lt;
    } else if (d.kind == L_M2L) {
        if (L < 2) return;
        const int fine = c.mixed ? c.fine : 0;
        const int f32 = L - fine + 1 > 2 ? L - fine + 1 : 2;
        const int lo = d.fp32 ? f32 : 2, hi = d.fp32 ? L : f32 - 1;
        const int sl = sched_split_level(L, c.split_max);
        const int a = d.part == 0 ? lo : (lo > sl + 1 ? lo : sl + 1);
        const int b = d.part == 0 ? (hi < sl ? hi : sl) : hi;
        if (b < a) return;
        int cnt = 0;
        for (int l = a; l <= b; ++l) cnt += sched_level_blocks(l);
        wg = cnt;
        a0 = a;
        a1 = b;
    } else if (d.kind == L_DOWN) {
        if (L < 3) return;
        const int r = (L - 2) % 3;
        const int lt = d.group == 0 ? 2 : 2 + (r ? r : 3) + 3 * (d.group - 1);
        if (lt >= L) return;
        wg = 1 << (2 * lt);
        a0 = lt;
        a1 = d.group == 0 && r ? r : 3;
    } else {
        const int64_t nleaf = int64_t(1) << (2 * L);
        wg = int((nleaf + c.p2p_waves - 1) / c.p2p_waves);
    }
}

// Wavefronts an instance's split M2L levels divide each list over (FP32
// levels always three; FP64 levels three when they have few tiles), and the
// levels that therefore have a second partial sum (bit l).
__host__ __device__ inline void sched_m2l_groups(const SchedCfg& c, int L, int& g64, int& part1)
{
    g64 = 2;
    part1 = 0;
    for (int fp32 = 0; fp32 < 2; ++fp32) {
        const LaunchDesc d{L_M2L, 0, fp32, 0};
        int wg, a, b;
        sched_inst(c, d, L, wg, a, b);
        if (wg == 0) continue;
        const int gi = (fp32 || wg < kM2LFewTiles) ? 3 : 2;
        if (!fp32) g64 = gi;
        if (gi == 3)
            for (int l = a; l <= b; ++l) part1 |= 1 << l;
    }
}

// The paper's work model (Section 5.2): a non-leaf box costs p^2 (2 n_c +
// n_IL) (eq. 13), a leaf 2 N_i p + p^2 n_IL + n_nd N_i^2 (eq. 14), and a tree
// the sum over its boxes (eq. 15, read for the whole tree of depth L: levels
// 0 .. L-1 non-leaf, 4^L leaves).  N_i is the mean occupancy N / 4^L; n_c =
// 4, n_IL = 27 (Table 1), n_nd = 9 (the leaf and its 8 neighbours).
__host__ __device__ inline double sched_work(int64_t n, int L, int p)
{
    const double pp = double(p) * p;
    const double nc = 4.0, nil = 27.0, nnd = 9.0;
    const double nonleaf = (double((int64_t(1) << (2 * L))) - 1.0) / 3.0 * pp * (2.0 * nc + nil);
    const double leaves = double(int64_t(1) << (2 * L));
    const double ni = double(n) / leaves;
    return nonleaf + leaves * (2.0 * ni * p + pp * nil + nnd * ni * ni);
}

}  // namespace fmm
