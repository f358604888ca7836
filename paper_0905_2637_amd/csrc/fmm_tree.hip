// fmm_tree.hip -- tree build on the GPU: domain, z-order leaf keys, counting
// sort of the particles by leaf, leaf ranges, sorted particle arrays.
//
// The uniform quadtree of Section 2.1 needs no pointer structure: box (a, b)
// at level l covers [x0 + a w_l, x0 + (a+1) w_l) x [...], its z-order number
// (Section 5.1) is the bit interleave of (a, b), and the particles of any box
// at any level form one contiguous range of the leaf-sorted particle array.
// Sorting by leaf key is a counting sort with 4^L buckets (a radix sort whose
// single digit is the whole key): one pass counts, a scan turns counts into
// leaf starts, one pass scatters.  The atomics of the counting pass fix each
// particle's slot inside its leaf in arrival order; a final pass re-ranks
// every leaf's members by input index, so the permutation is the unique stable
// one (ties in input order) and runs are bit-for-bit reproducible.
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

// Zero the leaf counters and the status word; in explicit-domain mode also
// store the domain.
__global__ void __launch_bounds__(256)
k_reset(int32_t* __restrict__ cnt, int64_t nleaf, int64_t* status, Domain* dom, Domain d, int write_dom)
{
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nleaf; i += stride) cnt[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        status[0] = 0;
        if (write_dom) *dom = d;
    }
}

// ---------------------------------------------------------------------------
// Keys and counting
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

__global__ void __launch_bounds__(256)
k_keys(int n, const double* __restrict__ x, const double* __restrict__ y, const Domain* __restrict__ dom,
       int L, uint32_t* __restrict__ key, uint32_t* __restrict__ slot, int32_t* __restrict__ cnt,
       int64_t* __restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const Domain d = *dom;
        const int side = 1 << L;
        const int a = axis_box(x[i], d.x0, d.s, side, bad);
        const int b = axis_box(y[i], d.y0, d.s, side, bad);
        const uint32_t k = morton(uint32_t(a), uint32_t(b));
        key[i] = k;
        slot[i] = uint32_t(atomicAdd(&cnt[k], 1));
    }
    const uint64_t m = __ballot(bad);
    if (m != 0 && __lane_id() == uint32_t(__ffsll((unsigned long long)m) - 1))
        atomicAdd((unsigned long long*)status, (unsigned long long)__popcll(m));
}

// ---------------------------------------------------------------------------
// Exclusive scan of the leaf counts -> leaf_start[0 .. nleaf]
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

// Single workgroup: exclusive scan of the chunk sums, part[nb] = grand total.
__global__ void __launch_bounds__(256) k_scan_top(int nb, int32_t* __restrict__ part)
{
    int carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int i = base + threadIdx.x;
        const int v = i < nb ? part[i] : 0;
        int total;
        const int e = block_excl_scan(v, &total);
        if (i < nb) part[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ void __launch_bounds__(256)
k_scan_down(int64_t m, int nb, const int32_t* __restrict__ in, const int32_t* __restrict__ part,
            int32_t* __restrict__ out)
{
    const int64_t base = int64_t(blockIdx.x) * kScanChunk + int64_t(threadIdx.x) * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) { v[k] = (base + k < m) ? in[base + k] : 0; s += v[k]; }
    int total;
    int run = block_excl_scan(s, &total) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[m] = part[nb];
}

// ---------------------------------------------------------------------------
// Scatter, stable re-rank, gather
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_scatter(int n, const uint32_t* __restrict__ key, const uint32_t* __restrict__ slot,
          const int32_t* __restrict__ leaf_start, uint32_t* __restrict__ perm_tmp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm_tmp[leaf_start[key[i]] + slot[i]] = uint32_t(i);
}

// One thread per leaf-sorted position: its final place inside the leaf is the
// number of the leaf's members with a smaller input index.  Writes the
// permutation and the sorted SoA copies; in mixed mode also the FP32
// leaf-relative record (x - c, y - c) / w_L, gamma, where c is the leaf centre.
__global__ void __launch_bounds__(256)
k_gather(int n, int L, const uint32_t* __restrict__ key, const uint32_t* __restrict__ perm_tmp,
         const int32_t* __restrict__ leaf_start, const double* __restrict__ x, const double* __restrict__ y,
         const double* __restrict__ g, const Domain* __restrict__ dom, uint32_t* __restrict__ perm,
         double* __restrict__ xs, double* __restrict__ ys, double* __restrict__ gs, float4* __restrict__ pk)
{
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    const uint32_t j = perm_tmp[pos];
    const uint32_t k = key[j];
    const int s0 = leaf_start[k], s1 = leaf_start[k + 1];
    int rank = 0;
    for (int q = s0; q < s1; ++q) rank += perm_tmp[q] < j ? 1 : 0;
    const int d = s0 + rank;
    const double xv = x[j], yv = y[j], gv = g[j];
    perm[d] = j;
    xs[d] = xv;
    ys[d] = yv;
    gs[d] = gv;
    if (pk) {
        const Domain dm = *dom;
        const double w = ldexp(dm.W, -L);
        const double cx = dm.x0 + (double(morton_x(k)) + 0.5) * w;
        const double cy = dm.y0 + (double(morton_y(k)) + 0.5) * w;
        pk[d] = make_float4(float((xv - cx) * dm.s), float((yv - cy) * dm.s), float(gv), 0.0f);
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_domain(const Buffers& b, int64_t nleaf, int n, const double* x, const double* y,
                         int L, bool auto_domain, Domain explicit_dom, hipStream_t st)
{
    if (auto_domain) {
        hipLaunchKernelGGL(k_bbox_partial, dim3(kBBoxBlocks), dim3(256), 0, st, n, x, y, b.bbox);
        hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, st, kBBoxBlocks, b.bbox, L, b.dom);
    }
    const unsigned nb = unsigned(std::min<int64_t>(4096, std::max<int64_t>(1, (nleaf + 255) / 256)));
    hipLaunchKernelGGL(k_reset, dim3(nb), dim3(256), 0, st, b.cnt, nleaf, b.status, b.dom, explicit_dom,
                       auto_domain ? 0 : 1);
    return hipGetLastError();
}

hipError_t launch_tree(const Buffers& b, int n, int L, const double* x, const double* y, const double* g,
                       bool mixed, hipStream_t st)
{
    const int64_t nleaf = int64_t(1) << (2 * L);
    if (n > 0)
        hipLaunchKernelGGL(k_keys, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, x, y, b.dom, L, b.key,
                           b.slot, b.cnt, b.status);
    const int nb = int((nleaf + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(256), 0, st, nleaf, b.cnt, b.scan_part);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, st, nb, b.scan_part);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(256), 0, st, nleaf, nb, b.cnt, b.scan_part, b.leaf_start);
    if (n > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, b.key, b.slot,
                           b.leaf_start, b.perm_tmp);
        hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, L, b.key, b.perm_tmp,
                           b.leaf_start, x, y, g, b.dom, b.perm, b.xs, b.ys, b.gs, mixed ? b.pk : nullptr);
    }
    return hipGetLastError();
}

}  // namespace fmm
