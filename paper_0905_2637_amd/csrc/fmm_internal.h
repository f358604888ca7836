// fmm_internal.h -- types and launcher declarations shared by the library's
// translation units.  Not part of the public ABI (see include/fmm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fmm {

// Square domain of one evaluation: [x0, x0 + W]^2 and s = 2^L / W, the
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

// Device pointers of one plan, all inside the caller's workspace.
struct Buffers {
    int32_t* bad_blk;      // [radix blocks] particles outside the explicit domain / NaN, per tile
    Domain* dom;
    double* bbox;          // [4 * kBBoxBlocks] partial bounding boxes
    int32_t* leaf_start;   // [nleaf + 1]
    int32_t* hist;         // [256 * radix blocks] digit-major tile histograms
    int32_t* hist_scan;    // [256 * radix blocks + 1] exclusive scan of hist, then the total
    int32_t* scan_part;    // [scan chunks + 1]
    uint32_t* key;         // [n_max] leaf z-order key per input particle
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
    cd* me;                // [Lambda * p] scaled multipole coefficients
    cd* le;                // [Lambda * p] scaled local coefficients
    cd* le_part[2];        // [Lambda(split level) * p] partial M2L sums of the split levels
    int32_t* ilist;        // [Lambda * 27] debug: interaction lists
    cd* t_m2m;             // [4][P][P]
    cd* t_l2l;             // [4][P][P]
    cd* t_h64;             // [49][2P-1] M2L translation data, FP64
    cf* t_h32;             // [49][2P-1] M2L translation data, FP32
    double* t_sin;         // [P] (-1)^(k+1) / k!
    double* t_sout;        // [P] 1 / l!
};

struct Layout {
    size_t bad_blk, dom, bbox, leaf_start, hist, hist_scan, scan_part, key, ksorted, perm, xs, ys, gs;
    size_t ktmp, itmp, xt, yt, gt, pk, me, le, le_part[2], t_m2m, t_l2l, t_h64, t_h32, t_sin, t_sout;
    size_t total;
};

// Radix sort geometry (fmm_tree.hip): passes of 8-bit digits over 2L key
// bits, and workgroup tiles of 4096 keys.
int radix_passes(int L);
int64_t radix_blocks(int64_t n);

// Chunk of the histogram scan handled by one workgroup.
constexpr int kScanChunk = 2048;

// ---- launchers (each enqueues on `st` and returns the launch status) -------

hipError_t launch_domain(const Buffers& b, int n, const double* x, const double* y, int L, hipStream_t st);
hipError_t launch_tree(const Buffers& b, int n, int L, const double* x, const double* y, const double* g,
                       bool explicit_dom, Domain hdom, bool mixed, hipStream_t st);
hipError_t launch_upward(const Buffers& b, int P, int p, int L, hipStream_t st);     // P2M + M2M
hipError_t launch_m2l(const Buffers& b, int P, int p, int lmin, int lmax, bool fp32, int groups, hipStream_t st);
hipError_t launch_downward(const Buffers& b, int P, int p, int L, int split_level, hipStream_t st);   // L2L

// Levels up to this one run M2L with the interaction list split over three
// wavefronts (more parallelism where a level has few boxes); deeper levels
// have enough boxes to fill the GPU with one wavefront per 64 boxes.
constexpr int kM2LSplitMaxLevel = 8;
inline int m2l_split_level(int L) { return L <= 2 ? 1 : (L < kM2LSplitMaxLevel ? L : kM2LSplitMaxLevel); }
hipError_t launch_p2p(const Buffers& b, int P, int p, int L, bool has_far, bool mixed, double sigma,
                      double* u, double* v, hipStream_t st);
hipError_t launch_ilist(const Buffers& b, int L, hipStream_t st);

// ---- host-side operator tables (FP64, built once per plan) -----------------
void build_tables(int P, int p, cd* m2m, cd* l2l, cd* h64, cf* h32, double* sin_, double* sout_);

}  // namespace fmm
