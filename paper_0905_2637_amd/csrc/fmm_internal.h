// fmm_internal.h -- types and launcher declarations shared by the library's
// translation units.  Not part of the public ABI (see include/fmm.h).
//
// A plan holds one or more FMM instances (a single evaluation is a batch of
// one).  Every instance has its own uniform quadtree of depth L_i over its own
// square; the instances' particles are concatenated, and their leaf ranges,
// multipole and local expansions live in per-instance segments of shared
// arrays.  Each stage is one launch over the work of all instances: the
// workgroups of a launch are numbered instance after instance, and a
// workgroup finds its instance in a prefix table built on the host at plan
// time.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fmm.h"
#include "fmm_schedule.h"

namespace fmm {

// Square domain of one instance: [x0, x0 + W]^2 and s = 2^L / W, the
// reciprocal of the leaf width, computed as one correctly rounded division.
struct Domain {
    double x0, y0, W, s;
};

struct cd { double x, y; };   // complex FP64
struct cf { float x, y; };    // complex FP32

constexpr int kMaxDepth = 13;
constexpr int kMaxP = 32;
constexpr int kMaxPMixed = 22;      // FP32 translation data overflows beyond this
constexpr int kHankelGrid = 7;      // integer M2L offsets (dx, dy) with |dx|, |dy| <= 3
constexpr int kBBoxBlocks = 256;
constexpr int kMaxInstances = 1 << 16;
// Widest domain and narrowest Gaussian core: the FP64 near field takes four
// squared separations, each floored at 1e-76, through one reciprocal of their
// product, which stays normal for separations below about 1e37; the floor
// changes a pair term by less than an ulp for sigma >= 1e-30.
constexpr double kMaxWidth = 1e36;
constexpr double kMinGaussSigma = 1e-30;

// Number of boxes in levels 0 .. l-1, i.e. the global id of the first box of
// level l (Section 5.3 counts (4^(L+1) - 1)/3 boxes in a full quadtree).
__host__ __device__ inline int64_t level_offset(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }

// Expansion sizes the kernels are compiled for; a plan uses the smallest
// one >= p and zero-pads coefficients k >= p, which leaves the p-term result
// unchanged (every operator maps terms < p only from terms < p).
inline int instantiated_terms(int p)
{
    static const int sizes[] = {8, 12, 16, 17, 20, 24, 32};
    for (int s : sizes)
        if (p <= s) return s;
    return -1;
}

// M2L on levels up to an instance's split level runs with the interaction
// list split over several wavefronts (more parallelism where levels have few
// boxes), two or three.  The partial sums beyond the first go to extra
// buffers sized for levels up to kM2LSplitMaxLevel and are added by the
// downward sweep.
constexpr int kM2LSplitMaxLevel = 8;

// One instance of a plan (device table, built on the host).
struct Inst {
    int64_t part_off;    // first particle in the concatenated arrays
    int64_t leaf_off;    // first entry of its leaf_start segment (4^L + 1 entries)
    int64_t box_off;     // first box of its expansion segments (Lambda(L) boxes)
    int64_t split_off;   // first box of its partial-M2L segments
    int32_t L;           // depth
    int32_t split;       // M2L split level (levels 2 .. split have partial sums)
    int32_t part1;       // bit l set: M2L level l has a second partial sum
    int32_t g64;         // wavefronts its split FP64 M2L levels divide a list over
    Domain dom;          // its square; s = 2^L / W
};

// Per-launch work table, in launch order: workgroups [wg_begin[k],
// wg_begin[k+1]) belong to instance order[k]; arg[2k], arg[2k+1] carry
// launch-specific values for it.  The order puts the instances with the most
// estimated work first (the paper's work model, eqs. 13-15), so the heaviest
// workgroups are dispatched first and the lightest fill the tail.
struct Work {
    const int32_t* wg_begin;
    const int32_t* arg;
    const int32_t* order;
};

// Place in the launch order of workgroup `wg` (uniform binary search over the
// prefix table).
__device__ __forceinline__ int find_inst(const int32_t* __restrict__ wg_begin, int n_inst, int wg)
{
    int lo = 0, hi = n_inst;      // wg_begin[lo] <= wg < wg_begin[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wg_begin[mid] <= wg) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroups are handed to the chip's 8 XCDs in turn (workgroup b to XCD
// b mod 8), and each XCD has an L2 of its own.  xcd_runs renumbers them so
// that every XCD takes runs of `run` consecutive logical workgroups, the runs
// dealt out in turn: neighbouring workgroups, which read much of the same
// data, then share an L2, and the order in which work starts is kept at the
// granularity of 8 runs.  A bijection on [0, G); the last G mod (8 run)
// workgroups keep their numbers.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_runs(int b, int G, int run)
{
    const int span = kXcds * run;
    if (run <= 1 || b >= G - G % span) return b;
    const int x = b % kXcds, k = b / kXcds;
    return ((k / run) * kXcds + x) * run + k % run;
}

// A launch counts its work-items in 32 bits per grid dimension, so a launch
// of one wavefront per leaf at depth 13 (2^26 leaves x 64 lanes) does not fit
// in one row.  Such launches take rows of at most kGridRow workgroups in y;
// flat_block() is the workgroup's place in the flattened grid.
constexpr int64_t kGridRow = int64_t(1) << 20;
inline dim3 row_grid(int64_t nwg)
{
    return dim3(unsigned(nwg < kGridRow ? nwg : kGridRow), unsigned((nwg + kGridRow - 1) / kGridRow));
}
__device__ __forceinline__ int64_t flat_block() { return blockIdx.x + int64_t(gridDim.x) * blockIdx.y; }

// Near-field pair kernel of a plan.  The far field, where there is one,
// always uses the expansions of the singular kernel; the Lennard-Jones force
// is cut off within a leaf width and has none.
enum NearKind : int { kNearGauss = 0, kNearSingular = 1, kNearLJ = 2 };
struct NearKernel {
    int kind;
    double sigma;     // Gaussian core size, or the Lennard-Jones length s
    double eps;       // Lennard-Jones energy
    double cutoff;    // Lennard-Jones cutoff
};

// Device pointers of one plan, all inside the caller's workspace.
struct Buffers {
    Inst* inst;            // [n_inst]
    int n_inst;
    int key_shift;         // 2 * (deepest depth): the instance id sits above it
    int32_t* bad_blk;      // [radix blocks] particles outside the domain / NaN, per tile
    double* bbox;          // [8 * kBBoxBlocks] partial bounding boxes (particles, then target points)
    int32_t* leaf_start;   // [sum (4^L_i + 1)] sorted ranges of every leaf of every instance
    int32_t* hist;         // [256 * radix blocks] digit-major tile histograms
    int32_t* hist_scan;    // [256 * radix blocks + 1] exclusive scan of hist, then the total
    int32_t* scan_part;    // [scan chunks + 1]
    uint32_t* key;         // [n_max] instance and leaf key per input particle
    uint32_t* ksorted;     // [n_max] sorted keys
    uint32_t* perm;        // [n_max] sorted position -> input index
    double* xs;            // [n_max] sorted positions and circulations
    double* ys;
    double* gs;
    uint32_t* ktmp;        // [n_max] radix ping-pong partners of the five arrays above
    uint32_t* itmp;
    double* xt;
    double* yt;
    double* gt;
    float4* pk;            // [n_max] mixed: leaf-relative FP32 (ox, oy, gamma, 0)
    uint8_t* blk_tab;      // [kBlockPolicies][kBlockTabBytes] near-field register-blocking tables
    // target points (fmm_evaluate_at), sorted like the particles; null when
    // the plan has no target capacity
    uint32_t* tkey;        // [m_max] leaf key per input point
    uint32_t* tks;         // [m_max] sorted keys
    uint32_t* tperm;       // [m_max] sorted position -> input index
    double* txs;           // [m_max] sorted positions
    double* tys;
    int32_t* tleaf_start;  // [4^L + 1] sorted ranges of the points of every leaf
    int32_t* tbad;         // [radix blocks of m_max] points outside the domain / NaN, per tile
    cd* me;                // [sum Lambda_i * P] scaled multipole coefficients, zero-padded to P
    cd* le;                // [sum Lambda_i * P] scaled local coefficients
    cd* le_part[2];        // [sum Lambda(split)_i * P] partial M2L sums of the split levels
    cd* t_m2m;             // [4][P][P]
    cd* t_l2l;             // [4][P][P]
    cd* t_h64;             // [49][2P-1] M2L translation data, FP64
    cf* t_h32;             // [49][2P-1] M2L translation data, FP32
    double* t_sin;         // [P] (-1)^(k+1) / k!
    double* t_sout;        // [P] 1 / l!
    // Gauss transform plans: Hermite and Taylor coefficients of every leaf
    // box, and the Hermite functions at the box offsets
    double* fgt_a;         // [4^L][P][P]
    double* fgt_b;         // [parts][4^L][P][P] (partial Taylor expansions, joined into part 0)
    double* fgt_h;         // [2 nc + 1][2P - 1]
};

// Chunk of the histogram scan handled by one workgroup.
constexpr int kScanChunk = 2048;

// Radix sort geometry (fmm_tree.hip): passes of 8-bit digits over the key
// bits, and workgroup tiles of 4096 keys.
int radix_passes(int key_bits);
int64_t radix_blocks(int64_t n);

// ---- launchers (each enqueues on `st` and returns the launch status) -------

// auto domain (single instance): bounding square of the particles and the m
// target points into inst[0].dom
hipError_t launch_domain(const Buffers& b, int n, const double* x, const double* y, int L, hipStream_t st,
                         int m = 0, const double* tx = nullptr, const double* ty = nullptr);
// n_dev (batched plans): the call's particle count and leaf entries on the
// device; n and leaf_entries are then the capacities the grids are sized for
hipError_t launch_tree(const Buffers& b, int n, const double* x, const double* y, const double* g,
                       int key_bits, int64_t leaf_entries, bool mixed, hipStream_t st,
                       const int32_t* n_dev = nullptr);
// the target points' keys, sort and leaf ranges (single instance)
hipError_t launch_tree_points(const Buffers& b, int m, const double* tx, const double* ty, int key_bits,
                              int64_t leaf_entries, hipStream_t st);
// P2M + M2M of up to three levels per launch; `from_particles` for the first
hipError_t launch_upward(const Buffers& b, int P, int p, const Work& w, int nwg, bool from_particles,
                         hipStream_t st);
// fp32 levels on the matrix cores when mfma is set
hipError_t launch_m2l(const Buffers& b, int P, const Work& w, int nwg, bool fp32, bool mfma, int groups,
                      hipStream_t st);
hipError_t launch_downward(const Buffers& b, int P, const Work& w, int nwg, hipStream_t st);   // L2L
// near field (+ L2P where there is a far field) with the plan's pair kernel
// block: the near-field register-blocking policy (block_table)
hipError_t launch_p2p(const Buffers& b, int P, const Work& w, int nwg, int waves, bool mixed, const NearKernel& nk,
                      int block, double* u, double* v, hipStream_t st);
// Near-field register-blocking tables: per policy, R, TG and S by chunk size
// t = 0 .. 64 (65 bytes each)
constexpr int kBlockPolicies = 2;
constexpr int kBlockTabBytes = 3 * 65;
void block_table(int policy, uint8_t* out);
// near field + L2P at the sorted target points of a single-instance FP64 plan
// (Gaussian or singular kernel)
hipError_t launch_p2p_at(const Buffers& b, int P, int L, const NearKernel& nk, int block, double* u, double* v,
                         hipStream_t st);
// interaction lists of boxes [b0, b0 + cnt) of a depth-L tree into out[cnt][27]
hipError_t launch_ilist(int L, int64_t b0, int64_t cnt, int32_t* out, hipStream_t st);
// the fast Gauss transform of a single-instance plan (after the tree): P
// Hermite terms per axis (8, 12 or 16), boxes within Chebyshev distance nc,
// the range's rows split over `parts` partial expansions; evaluated at the
// particles, or at the m sorted target points when m > 0
hipError_t launch_fgt(const Buffers& b, int P, int n, int L, double sigma, int nc, int parts, int m, double* u,
                      double* v, hipStream_t st);
int fgt_parts(int P, int L, int nc);
// h_n(d w / sqrt(delta)), |d| <= nc, n < 2P - 1, into out[(d + nc) (2P - 1) + n]
void fgt_hermite_table(int P, int nc, double w_over_sd, double* out);
// a[0..n) = b[0..n) = 0
hipError_t launch_zero2(int64_t n, double* a, double* b, hipStream_t st);
// time stepping: (xo, yo) = (x, y) + c (u, v); xo, yo may alias x, y
hipError_t launch_advance(int64_t n, const double* x, const double* y, const double* u, const double* v, double c,
                          double* xo, double* yo, hipStream_t st);

// The instance table of a batched call, turned into the plan's work tables
// on the device (fmm_batch.hip).
struct BatchSched {
    // the call
    int n_inst;
    const int64_t* offsets;       // [n_inst + 1]
    const int32_t* depths;        // [n_inst]
    // the plan
    int max_inst;
    int64_t n_max, leaf_cap, box_cap, split_cap;
    int depth_max, p, work_order;
    Domain dom;                   // the shared explicit square (s is set per depth)
    SchedCfg cfg;
    int n_launch;
    LaunchDesc launch[kMaxLaunches];
    // outputs
    Inst* inst;                   // [max_inst]
    int32_t* tables;              // [n_launch][4 max_inst + 1]
    int32_t* counts;              // [2]: particles of the call, leaf entries (0 when rejected)
    int32_t* status;              // FMM_OK or the rejection's status code
    double* work;                 // [max_inst] work estimates, input order
    int32_t* order;               // [max_inst] launch order
};
hipError_t launch_batch_schedule(const BatchSched& s, hipStream_t st);

// ---- plans over a library-provided buffer ----------------------------------
// a single-instance plan whose workspace is d_buffer (bytes, 256-byte aligned)
// and which records no stage-timing events
fmm_status plan_in_buffer(const fmm_params* prm, void* d_buffer, size_t bytes, void* stream, fmm_plan_t* out);

// ---- host-side operator tables (FP64, built once per plan) -----------------
void build_tables(int P, int p, cd* m2m, cd* l2l, cd* h64, cf* h32, double* sin_, double* sout_);

}  // namespace fmm
