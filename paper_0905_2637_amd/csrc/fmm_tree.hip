// fmm_tree.hip -- tree build on the GPU: domain, z-order leaf keys, stable
// LSD radix sort of the particles by key, leaf ranges, sorted particle arrays.
//
// The uniform quadtree of Section 2.1 needs no pointer structure: box (a, b)
// at level l covers [x0 + a w_l, x0 + (a+1) w_l) x [...], its z-order number
// (Section 5.1) is the bit interleave of (a, b), and the particles of any box
// at any level form one contiguous range of the key-sorted particle array.
//
// Sort: least-significant-digit radix sort with 8-bit digits, ceil(2L/8)
// passes.  Each pass is a per-tile digit histogram, an exclusive scan of the
// digit-major histogram table, and a stable scatter in which every wavefront
// ranks its 64 keys by digit with 8 ballots (lanes sharing a digit are found
// by intersecting the ballots of the digit's bits).  Every pass is stable, so
// the final permutation is the unique one with ties in input order, and no
// global atomics are involved: the result is bit-for-bit reproducible.
//
// Several instances sort together: the key of a particle of instance i is
// (i << 2 L_max) | (leaf key at depth L_i << 2 (L_max - L_i)), which orders
// instances first and leaves within each instance, so every instance's
// particles end up contiguous and in their own leaf order.
//
// The particle record (key, input index, x, y, gamma) travels with the sort,
// so every pass reads and writes whole streams (the scatter writes runs of
// ~16 records per digit and tile) and no random gather follows: the last pass
// writes the sorted arrays the later stages read, plus the mixed-precision
// FP32 leaf-relative record.  The first histogram pass computes the keys.
#include "fmm_device.h"

namespace fmm {
namespace {

// ---------------------------------------------------------------------------
// Domain
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_bbox_partial(int n, const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ part)
{
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double xv = x[i], yv = y[i];
        // fmin/fmax ignore a NaN operand: NaNs never move the box
        xmin = fmin(xmin, xv); xmax = fmax(xmax, xv);
        ymin = fmin(ymin, yv); ymax = fmax(ymax, yv);
    }
    __shared__ double sh[4][256];
    sh[0][threadIdx.x] = xmin; sh[1][threadIdx.x] = xmax;
    sh[2][threadIdx.x] = ymin; sh[3][threadIdx.x] = ymax;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + s]);
            sh[1][threadIdx.x] = fmax(sh[1][threadIdx.x], sh[1][threadIdx.x + s]);
            sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + s]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = sh[0][0];
        part[4 * blockIdx.x + 1] = sh[1][0];
        part[4 * blockIdx.x + 2] = sh[2][0];
        part[4 * blockIdx.x + 3] = sh[3][0];
    }
}

// Bounding square: x0 = min x, y0 = min y, W = the larger extent, 1 if the
// particles span nothing or the extent is not finite.
__global__ void k_bbox_final(int nblk, const double* __restrict__ part, int L, Domain* dom)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        xmin = fmin(xmin, part[4 * b + 0]); xmax = fmax(xmax, part[4 * b + 1]);
        ymin = fmin(ymin, part[4 * b + 2]); ymax = fmax(ymax, part[4 * b + 3]);
    }
    double w = xmax - xmin;
    if (ymax - ymin > w) w = ymax - ymin;
    if (!(w > 0.0) || !isfinite(w)) w = 1.0;
    if (!isfinite(xmin)) xmin = 0.0;
    if (!isfinite(ymin)) ymin = 0.0;
    Domain d;
    d.x0 = xmin; d.y0 = ymin; d.W = w;
    d.s = ldexp(1.0, L) / w;
    *dom = d;
}

// ---------------------------------------------------------------------------
// Keys
// ---------------------------------------------------------------------------

// Box index along one axis: t = (v - o) * s, two correctly rounded FP64
// operations (an FMA cannot fuse a product of a difference).  Inside when
// 0 <= t <= 2^L; the far edge belongs to the last box; outside or NaN is
// clamped and flagged.
__device__ __forceinline__ int axis_box(double v, double o, double s, int side, bool& bad)
{
    const double t = (v - o) * s;
    if (!(t >= 0.0 && t <= double(side))) {
        bad = true;
        return t > double(side) ? side - 1 : 0;
    }
    const int b = int(floor(t));
    return b > side - 1 ? side - 1 : b;
}

// ---------------------------------------------------------------------------
// Exclusive scan (of the radix histogram table)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan over a 256-thread block; *total gets the block sum.
__device__ __forceinline__ int block_excl_scan(int v, int* total)
{
    __shared__ int wsum[5];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int k = 0; k < 4; ++k) { const int t = wsum[k]; wsum[k] = run; run += t; }
        wsum[4] = run;
    }
    __syncthreads();
    const int r = inc - v + wsum[w];
    *total = wsum[4];
    __syncthreads();
    return r;
}

constexpr int kScanPerThread = kScanChunk / 256;

__global__ void __launch_bounds__(256)
k_scan_reduce(int64_t m, const int32_t* __restrict__ in, int32_t* __restrict__ part)
{
    const int64_t base = int64_t(blockIdx.x) * kScanChunk + int64_t(threadIdx.x) * kScanPerThread;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) s += (base + k < m) ? in[base + k] : 0;
    int total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Second level: every workgroup adds up the chunk sums before its own (there
// are few: n / 4096 tiles x 256 digits / 2048 per chunk), scans its chunk
// and the last one writes the grand total to out[m].
__global__ void __launch_bounds__(256)
k_scan_down(int64_t m, int nb, const int32_t* __restrict__ in, const int32_t* __restrict__ part,
            int32_t* __restrict__ out)
{
    int pre = 0;
    for (int i = threadIdx.x; i < int(blockIdx.x); i += 256) pre += part[i];
    int before;
    block_excl_scan(pre, &before);          // the block sum of pre: every chunk before this one
    const int64_t base = int64_t(blockIdx.x) * kScanChunk + int64_t(threadIdx.x) * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) { v[k] = (base + k < m) ? in[base + k] : 0; s += v[k]; }
    int total;
    int run = block_excl_scan(s, &total) + before;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[m] = before + total;
}

// ---------------------------------------------------------------------------
// Radix passes
// ---------------------------------------------------------------------------

constexpr int kRadixBins = 256;
constexpr int kRadixTile = 4096;   // keys per workgroup

// Instance owning input particle i (its particles are [part_off, next part_off)).
__device__ __forceinline__ int particle_inst(const Inst* __restrict__ inst, int n_inst, int64_t i)
{
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (inst[mid].part_off <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// The histogram kernels and the scatter take the same 4096-key tiles with
// TPB-thread workgroups, 4096 / TPB keys per thread.  Few tiles (small n)
// run with 1024 threads, so that every CU still holds many wavefronts to hide
// the memory latency of these passes; many tiles run with 256 threads and 16
// keys per thread, which measured faster there.

// First pass: the sort key of every particle (kept in input order for
// inspection), the out-of-domain count of the tile (every particle counts
// when the domain is wider than kMaxWidth), and the tile's histogram of the
// lowest digit.
template <int TPB>
__global__ void __launch_bounds__(TPB)
k_rhist_keys(int n, const double* __restrict__ x, const double* __restrict__ y, const Inst* __restrict__ inst,
             int n_inst, int key_shift, int nblk, uint32_t* __restrict__ key, int32_t* __restrict__ hist,
             int32_t* __restrict__ bad_blk, const int32_t* __restrict__ n_dev)
{
    if (n_dev) n = *n_dev;       // batched plans: the call's particle count, from the device
    constexpr int kTileRounds = kRadixTile / TPB;
    __shared__ int h[kRadixBins];
    __shared__ int nbad;
    const int64_t base = int64_t(blockIdx.x) * kRadixTile;
    if (base >= n) {             // a tile past the call's particles: empty (no input read)
        if (threadIdx.x < kRadixBins) hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = 0;
        if (threadIdx.x == 0) bad_blk[blockIdx.x] = 0;
        return;
    }
    if (threadIdx.x == 0) nbad = 0;
    if (threadIdx.x < kRadixBins) h[threadIdx.x] = 0;
    int mybad = 0;
    // all coordinate loads first, then keys and counting
    double xv[kTileRounds], yv[kTileRounds];
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const int64_t i = base + r * TPB + threadIdx.x;
        const int64_t ic = i < n ? i : base;
        xv[r] = x[ic];
        yv[r] = y[ic];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const int64_t i = base + r * TPB + threadIdx.x;
        if (i < n) {
            const int q = n_inst == 1 ? 0 : particle_inst(inst, n_inst, i);
            const int L = inst[q].L;
            const Domain d = inst[q].dom;
            const int side = 1 << L;
            bool bad = !(d.W <= kMaxWidth);    // a bounding square wider than the limit
            const int a = axis_box(xv[r], d.x0, d.s, side, bad);
            const int b = axis_box(yv[r], d.y0, d.s, side, bad);
            const uint32_t k = (uint32_t(q) << key_shift) | (morton(uint32_t(a), uint32_t(b)) << (key_shift - 2 * L));
            key[i] = k;
            atomicAdd(&h[k & (kRadixBins - 1)], 1);
            mybad += bad ? 1 : 0;
        }
    }
    if (mybad) atomicAdd(&nbad, mybad);
    __syncthreads();
    if (threadIdx.x < kRadixBins) hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
    if (threadIdx.x == 0) bad_blk[blockIdx.x] = nbad;
}

// Leaf (a, b), depth and domain of a sort key.
struct KeyLeaf {
    int q, L;
    uint32_t local;      // leaf key at depth L
};

__device__ __forceinline__ KeyLeaf key_leaf(uint32_t k, const Inst* __restrict__ inst, int key_shift)
{
    KeyLeaf r;
    r.q = key_shift >= 32 ? 0 : int(k >> key_shift);
    r.L = inst[r.q].L;
    const uint32_t mask = key_shift >= 32 ? 0xFFFFFFFFu : ((1u << key_shift) - 1u);
    r.local = (k & mask) >> (key_shift - 2 * r.L);
    return r;
}

// Digit histogram of one tile, written digit-major: hist[d * nblk + block].
template <int TPB>
__global__ void __launch_bounds__(TPB)
k_rhist(int n, const uint32_t* __restrict__ kin, int shift, int nblk, int32_t* __restrict__ hist,
        const int32_t* __restrict__ n_dev)
{
    if (n_dev) n = *n_dev;
    constexpr int kTileRounds = kRadixTile / TPB;
    __shared__ int h[kRadixBins];
    const int64_t base = int64_t(blockIdx.x) * kRadixTile;
    if (base >= n) {             // a tile past the call's particles: empty
        if (threadIdx.x < kRadixBins) hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = 0;
        return;
    }
    if (threadIdx.x < kRadixBins) h[threadIdx.x] = 0;
    uint32_t kv[kTileRounds];
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const int64_t i = base + r * TPB + threadIdx.x;
        kv[r] = kin[i < n ? i : base];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kTileRounds; ++r) {
        const int64_t i = base + r * TPB + threadIdx.x;
        if (i < n) atomicAdd(&h[(kv[r] >> shift) & (kRadixBins - 1)], 1);
    }
    __syncthreads();
    if (threadIdx.x < kRadixBins) hist[int64_t(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// Scatter tiles go to the XCDs in runs of this many from this many tiles on
// (below it the remapping measured no gain).
constexpr int kScatterXcdRun = 16;
constexpr int kScatterXcdMinTiles = 512;

// Where a sorted record goes, and what it carries.
struct Records {
    uint32_t* k;
    uint32_t* idx;
    double* x;
    double* y;
    double* g;
};

// Stable scatter of one tile, in two phases.
// Phase A ranks the tile: wavefront w owns input positions
// [4096 w / W, 4096 (w + 1) / W) of the W = TPB / 64 wavefronts and takes
// them 64 per round, in input order (loaded up front for 4 rounds, round by
// round for 16, which measured faster for each); it ranks
// its lanes by digit with 8 ballots, and the per-wavefront digit counts order
// the wavefronts, giving every record its position in the digit-sorted tile.
// Phase B stages each array through LDS in that order, so that consecutive
// threads write consecutive addresses of each digit's run (offs[d * nblk +
// block] is where the tile's run of digit d starts): whole cache lines
// instead of scattered 8-byte writes.
// iin == nullptr means the identity (first pass).  pk != nullptr (last pass,
// mixed precision) also writes the FP32 leaf-relative record
// (x - c, y - c) / w_L, gamma of the leaf centre c.
template <int TPB>
__global__ void __launch_bounds__(TPB)
k_rscatter(int n, const uint32_t* __restrict__ kin, const uint32_t* __restrict__ iin,
           const double* __restrict__ xin, const double* __restrict__ yin, const double* __restrict__ gin,
           int shift, int nblk, const int32_t* __restrict__ hist, const int32_t* __restrict__ offs, Records out,
           float4* __restrict__ pk, const Inst* __restrict__ inst, int key_shift, const int32_t* __restrict__ n_dev)
{
    if (n_dev) n = *n_dev;
    constexpr int kScatterThreads = TPB;
    constexpr int kScatterWaves = TPB / 64;
    constexpr int kPerThread = kRadixTile / TPB;
    constexpr bool kUpFront = kPerThread <= 4;
    __shared__ int gbase[kRadixBins];      // global start of this tile's run of digit d
    __shared__ int tstart[kRadixBins];     // start of digit d in the sorted tile
    __shared__ int wsum[4];
    __shared__ int whist[kScatterWaves][kRadixBins];   // per wavefront: records of digit d so far
    __shared__ uint32_t sk[kRadixTile];
    __shared__ double sv[kRadixTile];
    const int tid = threadIdx.x, lane = int(__lane_id()), w = tid >> 6;
    // large sorts: runs of kScatterXcdRun consecutive tiles per XCD, so that
    // the runs of one digit that neighbouring tiles write side by side meet
    // in one L2 (whole lines go out) instead of leaving partial lines in two
    const int blk = nblk >= kScatterXcdMinTiles ? xcd_runs(int(blockIdx.x), nblk, kScatterXcdRun) : int(blockIdx.x);
    const int64_t tile = int64_t(blk) * kRadixTile;
    if (tile >= n) return;       // a tile past the call's particles: nothing to move
    const int tile_n = int(min(int64_t(kRadixTile), int64_t(n) - tile));
    constexpr int kWaveKeys = kRadixTile / kScatterWaves;

    // the tile's histogram (one digit per thread of the first 256) scanned
    // into tstart; the first four wavefronts hold it
    int hv = 0, hinc = 0;
    if (tid < kRadixBins) {
        hv = hist[int64_t(tid) * nblk + blk];
        gbase[tid] = offs[int64_t(tid) * nblk + blk];
        hinc = wave_incl_scan(hv);
        if (lane == 63) wsum[w] = hinc;
    }
#pragma unroll
    for (int e = tid; e < kScatterWaves * kRadixBins; e += kScatterThreads) (&whist[0][0])[e] = 0;

    uint32_t kr[kPerThread], vr[kPerThread];
    double xr[kPerThread], yr[kPerThread], gr[kPerThread];
    bool valid[kPerThread];
    auto load = [&](int r) {
        const int li = w * kWaveKeys + r * 64 + lane;
        valid[r] = li < tile_n;
        const int64_t i = tile + (valid[r] ? li : 0);
        kr[r] = valid[r] ? kin[i] : 0u;
        vr[r] = iin ? iin[i] : uint32_t(i);
        xr[r] = xin[i];
        yr[r] = yin[i];
        gr[r] = gin ? gin[i] : 0.0;
    };
    if constexpr (kUpFront) {
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) load(r);
    }
    __syncthreads();
    if (tid < kRadixBins) {
        int before = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) before += q < w ? wsum[q] : 0;
        tstart[tid] = before + hinc - hv;
    }

    // rank within the wavefront, round after round (input order): equal
    // digits of one round are told apart by 8 ballots, earlier rounds by the
    // wavefront's running count of the digit
    const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
    int lpos[kPerThread], dig[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        if constexpr (!kUpFront) load(r);
        const int d = int((kr[r] >> shift) & (kRadixBins - 1));
        uint64_t same = __ballot(valid[r]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const int rank = __popcll(same & lt_mask);
        const int before = whist[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid[r] && rank == 0) whist[w][d] = before + __popcll(same);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        lpos[r] = valid[r] ? before + rank : -1;
        dig[r] = d;
    }
    __syncthreads();
    // exclusive prefix over the wavefronts, per digit
    if (tid < kRadixBins) {
        int acc = 0;
#pragma unroll
        for (int q = 0; q < kScatterWaves; ++q) {
            const int t = whist[q][tid];
            whist[q][tid] = acc;
            acc += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) lpos[r] += tstart[dig[r]] + whist[w][dig[r]];

    // ---- phase B: stage each array in sorted order, write whole runs ----
    int dst[kPerThread];
    uint32_t ks_[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) sk[lpos[r]] = kr[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int j = r * kScatterThreads + tid;
        dst[r] = -1;
        if (j < tile_n) {
            const uint32_t k = sk[j];
            const int d = int((k >> shift) & (kRadixBins - 1));
            ks_[r] = k;
            dst[r] = gbase[d] + (j - tstart[d]);
            out.k[dst[r]] = k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) sk[lpos[r]] = vr[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (dst[r] >= 0) out.idx[dst[r]] = sk[r * kScatterThreads + tid];

    double xs_[kPerThread], ys_[kPerThread];
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) sv[lpos[r]] = xr[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        xs_[r] = sv[r * kScatterThreads + tid];
        if (dst[r] >= 0) out.x[dst[r]] = xs_[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) sv[lpos[r]] = yr[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        ys_[r] = sv[r * kScatterThreads + tid];
        if (dst[r] >= 0) out.y[dst[r]] = ys_[r];
    }
    if (!out.g) return;                    // point records (target points) carry no circulation
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r)
        if (lpos[r] >= 0) sv[lpos[r]] = gr[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        if (dst[r] < 0) continue;
        const double gv = sv[r * kScatterThreads + tid];
        out.g[dst[r]] = gv;
        if (pk) {
            const KeyLeaf kl = key_leaf(ks_[r], inst, key_shift);
            const Domain dm = inst[kl.q].dom;
            const double wl = ldexp(dm.W, -kl.L);
            const double cx = dm.x0 + (double(morton_x(kl.local)) + 0.5) * wl;
            const double cy = dm.y0 + (double(morton_y(kl.local)) + 0.5) * wl;
            pk[dst[r]] = make_float4(float((xs_[r] - cx) * dm.s), float((ys_[r] - cy) * dm.s), float(gv), 0.0f);
        }
    }
}

// Depth 0: one leaf, nothing to sort.
__global__ void __launch_bounds__(256)
k_copy_one_leaf(int n, const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ g,
                Records out, float4* __restrict__ pk, const Inst* __restrict__ inst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xv = x[i], yv = y[i], gv = g ? g[i] : 0.0;
    out.k[i] = 0u;
    out.idx[i] = uint32_t(i);
    out.x[i] = xv;
    out.y[i] = yv;
    if (out.g) out.g[i] = gv;
    if (pk) {
        const Domain dm = inst[0].dom;
        const double cx = dm.x0 + 0.5 * dm.W, cy = dm.y0 + 0.5 * dm.W;
        pk[i] = make_float4(float((xv - cx) * dm.s), float((yv - cy) * dm.s), float(gv), 0.0f);
    }
}

// Sorted position -> global leaf_start entry (instance segment + leaf).
__device__ __forceinline__ int64_t leaf_entry(uint32_t k, const Inst* __restrict__ inst, int key_shift)
{
    const KeyLeaf kl = key_leaf(k, inst, key_shift);
    return inst[kl.q].leaf_off + int64_t(kl.local);
}

// leaf_start[e] = first sorted position whose leaf entry is >= e, for every
// entry e < entries: position i owns the entries in (entry(i-1), entry(i)].
// Each instance's segment ends with one extra entry, which thereby receives
// the first position of the next instance (its particle count end).
// A workgroup takes kBoundsRounds x 256 consecutive positions, 256 per round
// (coalesced); all its key loads are issued before any range is written,
// and a single-instance plan reads its instance record once.
constexpr int kBoundsRounds = 16;

__global__ void __launch_bounds__(256)
k_bounds(int n, int64_t entries, const uint32_t* __restrict__ ks, const Inst* __restrict__ inst, int n_inst,
         int key_shift, int32_t* __restrict__ leaf_start, const int32_t* __restrict__ n_dev)
{
    if (n_dev) {                 // batched plans: particles and leaf entries of the call
        n = n_dev[0];
        entries = n_dev[1];
    }
    const int64_t base = int64_t(blockIdx.x) * (256 * kBoundsRounds) + threadIdx.x;
    uint32_t kp[kBoundsRounds], kc[kBoundsRounds];      // keys of i - 1 and i
#pragma unroll
    for (int r = 0; r < kBoundsRounds; ++r) {
        const int64_t i = base + int64_t(r) * 256;
        const int64_t ip = i - 1 < 0 ? 0 : (i - 1 < n ? i - 1 : (n > 0 ? n - 1 : 0));
        const int64_t ic = i < n ? i : (n > 0 ? n - 1 : 0);
        kp[r] = ks[ip];
        kc[r] = ks[ic];
    }
    const int L0 = inst[0].L;
    const int64_t off0 = inst[0].leaf_off;
    auto entry = [&](uint32_t k) -> int64_t {
        if (n_inst == 1) return off0 + int64_t(k >> (key_shift - 2 * L0));
        return leaf_entry(k, inst, key_shift);
    };
#pragma unroll
    for (int r = 0; r < kBoundsRounds; ++r) {
        const int64_t i = base + int64_t(r) * 256;
        if (i > n) break;
        const int64_t lo = i == 0 ? 0 : entry(kp[r]) + 1;
        const int64_t hi = i == n ? entries - 1 : entry(kc[r]);
        for (int64_t e = lo; e <= hi; ++e) leaf_start[e] = int32_t(i);
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_domain(const Buffers& b, int n, const double* x, const double* y, int L, hipStream_t st,
                         int m, const double* tx, const double* ty)
{
    hipLaunchKernelGGL(k_bbox_partial, dim3(kBBoxBlocks), dim3(256), 0, st, n, x, y, b.bbox);
    if (m > 0)   // target points: their partial boxes follow the particles'
        hipLaunchKernelGGL(k_bbox_partial, dim3(kBBoxBlocks), dim3(256), 0, st, m, tx, ty, b.bbox + 4 * kBBoxBlocks);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, m > 0 ? 2 * kBBoxBlocks : kBBoxBlocks, b.bbox, L,
                       &b.inst[0].dom);
    return hipGetLastError();
}

int radix_passes(int key_bits) { return (key_bits + 7) / 8; }

int64_t radix_blocks(int64_t n) { return (n + kRadixTile - 1) / kRadixTile; }

namespace {

// Radix passes of at most this many tiles use the 1024-thread kernels.
#ifndef FMM_TREE_TPB
#define FMM_TREE_TPB 0
#endif
constexpr int kWideTilesMax = 2048;

// Exclusive scan of hist[0..m) into out[0..m], out[m] = total.
void scan_table(const Buffers& b, int64_t m, hipStream_t st)
{
    const int nsb = int((m + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nsb), dim3(256), 0, st, m, b.hist, b.scan_part);
    hipLaunchKernelGGL(k_scan_down, dim3(nsb), dim3(256), 0, st, m, nsb, b.hist, b.scan_part, b.hist_scan);
}

}  // namespace

namespace {

// Keys, sort and leaf ranges of one point set: records (key, index, x, y and,
// when g != nullptr, gamma), final arrays in fin, leaf ranges in leaf_start.
void sort_points(const Buffers& b, int n, const double* x, const double* y, const double* g, uint32_t* key,
                 int32_t* bad_blk, const Records& fin, float4* pk, int32_t* leaf_start, int key_bits,
                 int64_t leaf_entries, hipStream_t st, const int32_t* n_dev = nullptr)
{
    const int nblk = int(radix_blocks(n));
    const int64_t m = int64_t(kRadixBins) * nblk;
    const Records tmp{b.ktmp, b.itmp, b.xt, b.yt, g ? b.gt : nullptr};
    const bool wide = FMM_TREE_TPB == 1024 || (FMM_TREE_TPB == 0 && nblk <= kWideTilesMax);
    if (wide)
        hipLaunchKernelGGL(k_rhist_keys<1024>, dim3(nblk), dim3(1024), 0, st, n, x, y, b.inst, b.n_inst,
                           b.key_shift, nblk, key, b.hist, bad_blk, n_dev);
    else
        hipLaunchKernelGGL(k_rhist_keys<256>, dim3(nblk), dim3(256), 0, st, n, x, y, b.inst, b.n_inst,
                           b.key_shift, nblk, key, b.hist, bad_blk, n_dev);
    const int npass = radix_passes(key_bits);
    if (npass == 0) {
        hipLaunchKernelGGL(k_copy_one_leaf, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, x, y, g, fin, pk, b.inst);
    } else {
        // the last pass writes the final arrays, the others alternate with tmp
        const uint32_t* kin = key;
        const uint32_t* iin = nullptr;
        const double *xin = x, *yin = y, *gin = g;
        for (int pass = 0; pass < npass; ++pass) {
            const Records& out = ((npass - 1 - pass) & 1) ? tmp : fin;
            const int shift = 8 * pass;
            if (pass > 0 && wide)
                hipLaunchKernelGGL(k_rhist<1024>, dim3(nblk), dim3(1024), 0, st, n, kin, shift, nblk, b.hist, n_dev);
            else if (pass > 0)
                hipLaunchKernelGGL(k_rhist<256>, dim3(nblk), dim3(256), 0, st, n, kin, shift, nblk, b.hist, n_dev);
            scan_table(b, m, st);
            const bool last = pass == npass - 1;
            if (wide)
                hipLaunchKernelGGL(k_rscatter<1024>, dim3(nblk), dim3(1024), 0, st, n, kin, iin, xin, yin, gin,
                                   shift, nblk, b.hist, b.hist_scan, out, last ? pk : nullptr, b.inst, b.key_shift,
                                   n_dev);
            else
                hipLaunchKernelGGL(k_rscatter<256>, dim3(nblk), dim3(256), 0, st, n, kin, iin, xin, yin, gin,
                                   shift, nblk, b.hist, b.hist_scan, out, last ? pk : nullptr, b.inst, b.key_shift,
                                   n_dev);
            kin = out.k;
            iin = out.idx;
            xin = out.x;
            yin = out.y;
            gin = out.g;
        }
    }
    hipLaunchKernelGGL(k_bounds, dim3(blocks_for(int64_t(n) + 1, 256 * kBoundsRounds)), dim3(256), 0, st, n,
                       leaf_entries, fin.k, b.inst, b.n_inst, b.key_shift, leaf_start, n_dev);
}

}  // namespace

hipError_t launch_tree(const Buffers& b, int n, const double* x, const double* y, const double* g,
                       int key_bits, int64_t leaf_entries, bool mixed, hipStream_t st, const int32_t* n_dev)
{
    const Records fin{b.ksorted, b.perm, b.xs, b.ys, b.gs};
    sort_points(b, n, x, y, g, b.key, b.bad_blk, fin, mixed ? b.pk : nullptr, b.leaf_start, key_bits,
                leaf_entries, st, n_dev);
    return hipGetLastError();
}

hipError_t launch_tree_points(const Buffers& b, int m, const double* tx, const double* ty, int key_bits,
                              int64_t leaf_entries, hipStream_t st)
{
    const Records fin{b.tks, b.tperm, b.txs, b.tys, nullptr};
    sort_points(b, m, tx, ty, nullptr, b.tkey, b.tbad, fin, nullptr, b.tleaf_start, key_bits, leaf_entries, st);
    return hipGetLastError();
}

hipError_t launch_sort_keys(const Buffers& b, int n, const uint32_t* key, const double* x, const double* y,
                            const double* g, uint32_t* ks, uint32_t* perm, double* xs, double* ys, double* gs,
                            int key_bits, hipStream_t st)
{
    const int npass = radix_passes(key_bits);
    if (n <= 0 || npass <= 0) return hipErrorInvalidValue;
    const int nblk = int(radix_blocks(n));
    const int64_t m = int64_t(kRadixBins) * nblk;
    const Records fin{ks, perm, xs, ys, gs};
    const Records tmp{b.ktmp, b.itmp, b.xt, b.yt, b.gt};
    const bool wide = nblk <= kWideTilesMax;
    const uint32_t* kin = key;
    const uint32_t* iin = nullptr;
    const double *xin = x, *yin = y, *gin = g;
    for (int pass = 0; pass < npass; ++pass) {
        const Records& out = ((npass - 1 - pass) & 1) ? tmp : fin;
        const int shift = 8 * pass;
        if (wide)
            hipLaunchKernelGGL(k_rhist<1024>, dim3(nblk), dim3(1024), 0, st, n, kin, shift, nblk, b.hist, nullptr);
        else
            hipLaunchKernelGGL(k_rhist<256>, dim3(nblk), dim3(256), 0, st, n, kin, shift, nblk, b.hist, nullptr);
        scan_table(b, m, st);
        if (wide)
            hipLaunchKernelGGL(k_rscatter<1024>, dim3(nblk), dim3(1024), 0, st, n, kin, iin, xin, yin, gin, shift,
                               nblk, b.hist, b.hist_scan, out, nullptr, nullptr, 0, nullptr);
        else
            hipLaunchKernelGGL(k_rscatter<256>, dim3(nblk), dim3(256), 0, st, n, kin, iin, xin, yin, gin, shift,
                               nblk, b.hist, b.hist_scan, out, nullptr, nullptr, 0, nullptr);
        kin = out.k;
        iin = out.idx;
        xin = out.x;
        yin = out.y;
        gin = out.g;
    }
    return hipGetLastError();
}

}  // namespace fmm
