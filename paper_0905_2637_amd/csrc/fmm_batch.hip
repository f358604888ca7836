// fmm_batch.hip -- the work tables of a batched evaluation, built on the
// device from the instance sizes and depths of the call.
//
// A batched plan fixes capacities only (particles, instances, leaves, the
// deepest tree).  Every fmm_evaluate_batch call hands over its instance CSR
// offsets and depths in device memory; one workgroup then validates them
// against the capacities, lays the instances' segments out (leaf ranges,
// expansions, partial M2L sums), orders the instances by the paper's work
// estimate (Section 5.2, eqs. 13-15; heaviest first) and writes, for every
// launch of the plan's fixed launch list, the table the stage kernels read:
// the workgroup prefix over the instances in launch order, two arguments per
// instance and the order itself.  Tables are padded to the plan's instance
// capacity (unused slots own no workgroups), so the stage kernels, launched
// with grids sized for the capacities and captured once into a graph, serve
// any instance set that fits: a workgroup past its launch's total returns at
// once.  An instance set that does not fit (or is malformed) gets empty
// tables and a zero particle count, so nothing runs, and a status code that
// fmm_get_status reports.
#include "fmm_device.h"
#include "fmm_schedule.h"

namespace fmm {
namespace {

constexpr int kSchedThreads = 1024;
constexpr int kSchedWaves = kSchedThreads / 64;
constexpr int kOrderBins = 256;          // work-estimate buckets (quarter octaves)

// Exclusive prefix of v over the workgroup (every thread calls it); *total
// gets the sum.  sh: kSchedWaves + 1 int64 of LDS.
__device__ int64_t block_scan64(int64_t v, int64_t* sh, int64_t* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    __syncthreads();                      // sh free from any previous use
    if (lane == 63) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < kSchedWaves; ++i) {
            const int64_t t = sh[i];
            sh[i] = run;
            run += t;
        }
        sh[kSchedWaves] = run;
    }
    __syncthreads();
    const int64_t ex = sh[w] + x - v;
    *total = sh[kSchedWaves];
    return ex;
}

__device__ __forceinline__ int64_t lambda_boxes(int L) { return level_offset(L + 1); }

}  // namespace

__global__ void __launch_bounds__(kSchedThreads) k_batch_schedule(BatchSched s)
{
    __shared__ int64_t sh[kSchedWaves + 1];
    __shared__ int bad;
    __shared__ int hist[kOrderBins];
    __shared__ int bin_run[kOrderBins];
    const int tid = threadIdx.x;
    const int n = s.n_inst, M = s.max_inst;
    // contiguous share of the instances (input order, then launch order)
    const int per = (M + kSchedThreads - 1) / kSchedThreads;
    const int i0 = min(M, tid * per), i1 = min(M, i0 + per);
    if (tid == 0) bad = 0;
    __syncthreads();

    // ---- validation and segment sizes (input order) ----
    int64_t leaves = 0, boxes = 0, splits = 0;
    int flag = 0;
    for (int i = i0; i < i1 && i < n; ++i) {
        const int L = s.depths[i];
        const int64_t a = s.offsets[i], b = s.offsets[i + 1];
        if (L < 0 || L > s.depth_max) flag |= 1;
        if (b < a || a < 0) flag |= 1;
        if (i == 0 && a != 0) flag |= 1;
        if (flag) continue;
        leaves += (int64_t(1) << (2 * L)) + 1;
        boxes += lambda_boxes(L);
        splits += lambda_boxes(L < kM2LSplitMaxLevel ? L : kM2LSplitMaxLevel);
    }
    if (tid == 0 && (s.offsets[n] > s.n_max || s.offsets[n] < 0)) flag |= 2;
    if (flag) atomicOr(&bad, flag);
    int64_t t_leaves, t_boxes, t_splits;
    const int64_t x_leaves = block_scan64(leaves, sh, &t_leaves);
    const int64_t x_boxes = block_scan64(boxes, sh, &t_boxes);
    const int64_t x_splits = block_scan64(splits, sh, &t_splits);
    __syncthreads();
    int code = bad;
    if (!code && (t_leaves > s.leaf_cap || t_boxes > s.box_cap || t_splits > s.split_cap)) code = 2;
    const int64_t n_total = code ? 0 : s.offsets[n];
    if (tid == 0) {
        *s.status = code == 0 ? 0 : ((code & 1) ? -1 : -2);     // FMM_OK, FMM_E_ARG, FMM_E_CAPACITY
        s.counts[0] = int32_t(n_total);
        s.counts[1] = code ? 0 : int32_t(t_leaves);
    }

    // ---- instance records ----
    {
        int64_t lo = x_leaves, bo = x_boxes, so = x_splits;
        for (int i = i0; i < i1; ++i) {
            Inst I{};
            if (!code && i < n) {
                const int L = s.depths[i];
                I.part_off = s.offsets[i];
                I.leaf_off = lo;
                I.box_off = bo;
                I.split_off = so;
                I.L = L;
                I.split = sched_split_level(L, s.cfg.split_max);
                sched_m2l_groups(s.cfg, L, I.g64, I.part1);
                I.dom = s.dom;
                I.dom.s = ldexp(1.0, L) / s.dom.W;
                lo += (int64_t(1) << (2 * L)) + 1;
                bo += lambda_boxes(L);
                so += lambda_boxes(L < kM2LSplitMaxLevel ? L : kM2LSplitMaxLevel);
                s.work[i] = sched_work(s.offsets[i + 1] - s.offsets[i], L, s.p);
            } else {
                // unused slot: owns no particles, leaves or boxes
                I.part_off = n_total;
                I.leaf_off = code ? 0 : t_leaves;
                I.box_off = code ? 0 : t_boxes;
                I.split_off = code ? 0 : t_splits;
                I.L = 0;
                I.split = 1;
                I.g64 = 2;
                I.dom = s.dom;
                I.dom.s = 1.0 / s.dom.W;
                s.work[i] = 0.0;
            }
            s.inst[i] = I;
        }
    }

    // ---- launch order: heaviest estimate first, stable among equals ----
    // (a counting sort on quarter-octave buckets of the estimate)
    for (int b = tid; b < kOrderBins; b += kSchedThreads) hist[b] = 0;
    __syncthreads();
    auto bin_of = [&](int i) -> int {
        if (!s.work_order || code) return kOrderBins - 1;
        const double w = s.work[i];
        const int e = w > 1.0 ? int(4.0 * log2(w)) : 0;       // 0 .. 4 * 1023
        return kOrderBins - 1 - (e < kOrderBins - 1 ? e : kOrderBins - 1);   // heavier: smaller bin
    };
    __threadfence_block();
    for (int i = i0; i < i1 && i < n; ++i) atomicAdd(&hist[bin_of(i)], 1);
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int b = 0; b < kOrderBins; ++b) {
            const int c = hist[b];
            bin_run[b] = run;
            run += c;
        }
    }
    __syncthreads();
    // stable placement: the instances go through in input order, one wave
    // chunk of 64 at a time; lanes of a chunk that share a bucket are ranked
    // by lane (ballots over the bucket's bits), and the bucket's running
    // position advances by the chunk's count
    for (int c0 = 0; c0 < n; c0 += kSchedThreads) {
        for (int w = 0; w < kSchedWaves; ++w) {
            if ((tid >> 6) == w) {
                const int lane = tid & 63;
                const int i = c0 + tid;
                const bool live = i < n;
                const int bin = live ? bin_of(i) : 0;
                uint64_t same = __ballot(live);
                for (int bit = 0; bit < 8; ++bit) {
                    const uint64_t ones = __ballot(live && ((bin >> bit) & 1));
                    same &= ((bin >> bit) & 1) ? ones : ~ones;
                }
                const uint64_t below = same & ((uint64_t(1) << lane) - 1);
                const int rank = __popcll(below);
                const int cnt = __popcll(same);
                const int base = live ? bin_run[bin] : 0;
                if (live) s.order[base + rank] = i;
                // the lowest lane of each bucket advances it (after every lane read it)
                __builtin_amdgcn_wave_barrier();
                if (live && rank == 0) bin_run[bin] = base + cnt;
            }
            __syncthreads();
        }
    }
    for (int k = n + tid; k < M; k += kSchedThreads) s.order[k] = 0;
    __syncthreads();

    // ---- work tables, in launch order ----
    const int T = 4 * M + 1;
    for (int t = 0; t < s.n_launch; ++t) {
        int32_t* wg_begin = s.tables + int64_t(t) * T;
        int32_t* arg = wg_begin + M + 1;
        int32_t* ord = wg_begin + 3 * M + 1;
        int64_t sum = 0;
        for (int k = i0; k < i1 && k < n && !code; ++k) {
            int wg, a0, a1;
            sched_inst(s.cfg, s.launch[t], s.depths[s.order[k]], wg, a0, a1);
            sum += wg;
        }
        int64_t total;
        int64_t run = block_scan64(sum, sh, &total);
        for (int k = i0; k < i1; ++k) {
            int wg = 0, a0 = 0, a1 = 0, q = 0;
            if (k < n && !code) {
                q = s.order[k];
                sched_inst(s.cfg, s.launch[t], s.depths[q], wg, a0, a1);
            }
            wg_begin[k] = int32_t(run);
            arg[2 * k] = a0;
            arg[2 * k + 1] = a1;
            ord[k] = q;
            run += wg;
        }
        if (tid == 0) wg_begin[M] = int32_t(total);
    }
}

hipError_t launch_batch_schedule(const BatchSched& s, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_schedule, dim3(1), dim3(kSchedThreads), 0, st, s);
    return hipGetLastError();
}

}  // namespace fmm
