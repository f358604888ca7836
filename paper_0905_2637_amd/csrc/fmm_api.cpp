// fmm_api.cpp -- the C ABI of include/fmm.h: argument validation, workspace
// layout, the launch schedule of one evaluation (single or batched), hipGraph
// replay of the batched form, stage timing, the autotuner and inspection.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"

using namespace fmm;

namespace {

enum Stage { ST_TREE = 0, ST_UP, ST_M2L, ST_DOWN, ST_P2P, ST_COUNT };
const char* const kStageNames[ST_COUNT] = {"tree", "p2m_m2m", "m2l", "l2l", "p2p_l2p"};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Launch shapes the autotuner chooses among.
struct Tuning {
    int p2p_waves = 4;                   // leaves (wavefronts) per P2P workgroup: 2 or 4
    int split_max = kM2LSplitMaxLevel;   // M2L list split on levels <= this; < 2: never
    int m2l_mfma = 0;                    // unsplit FP32 M2L levels on the matrix cores (else paired, vector units)
    int work_order = 1;                  // launch order: most estimated work first (else input order)
    int p2p_block = 0;                   // near-field register-blocking policy (block_table)
};

// Host description of the instances of a plan.
struct Shape {
    int n_inst = 1;
    std::vector<int32_t> depth;
    std::vector<int64_t> part_off;       // first particle of every instance
    int64_t n_cap = 0;                   // particle capacity (the total count if batched)
    int64_t m_cap = 0;                   // target point capacity (single plans; 0: none)
    int fgt_nc = -1;                     // Gauss transform: box range (-1: not a Gauss transform plan)
    int Lmax = 0;
    int key_bits = 0;
    int64_t leaf_entries = 0;            // sum (4^L_i + 1)
    int64_t boxes = 0;                   // sum Lambda(L_i)
    int64_t split_boxes = 0;             // sum Lambda(min(L_i, kM2LSplitMaxLevel))
    std::vector<int64_t> leaf_off, box_off, split_off;
    std::vector<double> work;            // eq. 13-15 estimate per instance
    std::vector<int32_t> by_work;        // instances by decreasing estimate (stable)
    // batched plans: the instance set arrives with every call, so the plan
    // holds capacities (n_inst above is the instance capacity, leaf_entries,
    // boxes and split_boxes the segment capacities) and no per-instance data
    bool batched = false;
};

// Gauss transform plans: at most 16 Hermite terms per axis and a box range of
// at most 63 (the Hermite table of the range fits in a workgroup's LDS).
constexpr int kFgtMaxP = 16;
constexpr int kFgtMaxRange = 63;

struct Launch {
    LaunchDesc desc;
    int nwg;         // workgroups (batched plans: the capacity bound)
    int table;       // its work table
    int groups;      // M2L: 3 or 2 with the list split, else 1
};

int ceil_log2(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

int table_ints(int n_inst) { return 4 * n_inst + 1; }   // wg_begin [n+1], arg [2n], order [n]

fmm_status validate_common(const fmm_params* prm)
{
    if (!prm) return FMM_E_ARG;
    if (prm->kernel != FMM_KERNEL_GAUSSIAN && prm->kernel != FMM_KERNEL_SINGULAR &&
        prm->kernel != FMM_KERNEL_LENNARD_JONES && prm->kernel != FMM_KERNEL_GAUSS_TRANSFORM)
        return FMM_E_ARG;
    if (prm->kernel != FMM_KERNEL_SINGULAR && (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma)))
        return FMM_E_ARG;
    if (prm->kernel == FMM_KERNEL_GAUSSIAN && !(prm->sigma >= kMinGaussSigma)) return FMM_E_ARG;
    if (prm->kernel == FMM_KERNEL_LENNARD_JONES) {
        if (!(prm->lj_epsilon > 0.0) || !std::isfinite(prm->lj_epsilon)) return FMM_E_ARG;
        if (!(prm->cutoff > 0.0) || !std::isfinite(prm->cutoff)) return FMM_E_ARG;
        // the 3 x 3 leaves around a particle must hold every partner within the cutoff
        if (!(prm->width > 0.0)) return FMM_E_UNSUPPORTED;
        if (prm->precision != FMM_PREC_FP64) return FMM_E_UNSUPPORTED;
    }
    if (prm->kernel == FMM_KERNEL_GAUSS_TRANSFORM) {
        // the box range follows from sigma and the leaf width
        if (!(prm->width > 0.0)) return FMM_E_UNSUPPORTED;
        if (prm->precision != FMM_PREC_FP64 || prm->p > kFgtMaxP) return FMM_E_UNSUPPORTED;
    }
    if (prm->p < 1 || prm->p > kMaxP) return FMM_E_ARG;
    if (prm->precision != FMM_PREC_FP64 && prm->precision != FMM_PREC_MIXED) return FMM_E_ARG;
    if (prm->m_max < 0 || prm->m_max > int64_t(0x7fffffff)) return FMM_E_ARG;
    if (prm->width > 0.0) {
        if (!std::isfinite(prm->width) || !std::isfinite(prm->x0) || !std::isfinite(prm->y0)) return FMM_E_ARG;
        if (prm->width > kMaxWidth) return FMM_E_ARG;
    }
    if (prm->precision == FMM_PREC_MIXED) {
        if (prm->fp32_fine_levels < 0 || prm->fp32_fine_levels > kMaxDepth) return FMM_E_ARG;
        if (prm->p > kMaxPMixed) return FMM_E_UNSUPPORTED;
    }
    if (prm->max_instances < 0) return FMM_E_ARG;
    return FMM_OK;
}

fmm_status finish_shape(Shape& sh)
{
    sh.Lmax = 0;
    for (int L : sh.depth) sh.Lmax = std::max(sh.Lmax, L);
    sh.key_bits = (sh.n_inst > 1 ? ceil_log2(sh.n_inst) : 0) + 2 * sh.Lmax;
    if (sh.key_bits > 32) return FMM_E_UNSUPPORTED;
    sh.leaf_off.resize(sh.n_inst);
    sh.box_off.resize(sh.n_inst);
    sh.split_off.resize(sh.n_inst);
    sh.leaf_entries = sh.boxes = sh.split_boxes = 0;
    for (int i = 0; i < sh.n_inst; ++i) {
        const int L = sh.depth[i];
        sh.leaf_off[i] = sh.leaf_entries;
        sh.box_off[i] = sh.boxes;
        sh.split_off[i] = sh.split_boxes;
        sh.leaf_entries += (int64_t(1) << (2 * L)) + 1;
        sh.boxes += level_offset(L + 1);
        sh.split_boxes += level_offset(std::min(L, kM2LSplitMaxLevel) + 1);
    }
    // workgroup numbers of a launch are int32
    if (sh.boxes > int64_t(0x3fffffff) || sh.leaf_entries > int64_t(0x7fffffff)) return FMM_E_UNSUPPORTED;
    return FMM_OK;
}

// Gauss transform: boxes farther than nc apart are left out.  Their particles
// lie at least nc w apart, so exp(-(nc w)^2 / delta) <= 1e-16 (delta =
// 2 sigma^2) bounds a left-out term: nc = ceil(sqrt(ln 1e16) sqrt(delta) / w),
// at most the grid's extent.
int fgt_range(double sigma, double w, int L)
{
    const double nc = std::ceil(std::sqrt(std::log(1e16)) * std::sqrt(2.0) * sigma / w);
    const double side = std::ldexp(1.0, L);
    return int(std::min(nc, side - 1.0 > 0.0 ? side - 1.0 : 0.0) + 0.5);
}

// Lennard-Jones: every partner within the cutoff must lie in the 3 x 3 leaves
// around a particle, so the cutoff may not exceed the deepest leaf width.
bool cutoff_fits(const fmm_params* prm, int deepest)
{
    return prm->kernel != FMM_KERNEL_LENNARD_JONES || prm->cutoff <= std::ldexp(prm->width, -deepest);
}

fmm_status single_shape(const fmm_params* prm, Shape& sh)
{
    if (prm->n_max < 0 || prm->n_max > int64_t(0x7fffffff)) return FMM_E_ARG;
    if (prm->depth < 0 || prm->depth > kMaxDepth) return FMM_E_ARG;
    if (prm->precision == FMM_PREC_MIXED && prm->fp32_fine_levels > std::max(0, prm->depth - 1)) return FMM_E_ARG;
    sh.n_inst = 1;
    sh.depth = {prm->depth};
    sh.part_off = {0};
    sh.n_cap = prm->n_max;
    sh.m_cap = prm->m_max;
    if (!cutoff_fits(prm, prm->depth)) return FMM_E_UNSUPPORTED;
    if (prm->kernel == FMM_KERNEL_GAUSS_TRANSFORM) {
        sh.fgt_nc = fgt_range(prm->sigma, std::ldexp(prm->width, -prm->depth), prm->depth);
        if (sh.fgt_nc > kFgtMaxRange) return FMM_E_UNSUPPORTED;
    }
    return finish_shape(sh);
}

// A batched plan: capacities only (the instance set arrives with every call).
fmm_status batch_shape(const fmm_params* prm, Shape& sh, int64_t& max_leaves)
{
    const int M = prm->max_instances;
    if (M < 2 || M > kMaxInstances) return FMM_E_ARG;
    if (prm->n_max < 0 || prm->n_max > int64_t(0x7fffffff)) return FMM_E_ARG;
    if (prm->depth < 0 || prm->depth > kMaxDepth || prm->max_leaves < 0) return FMM_E_ARG;
    if (!(prm->width > 0.0)) return FMM_E_UNSUPPORTED;   // batched instances need the explicit square
    if (prm->m_max != 0) return FMM_E_ARG;                 // target points: single plans only
    if (prm->kernel == FMM_KERNEL_GAUSS_TRANSFORM) return FMM_E_UNSUPPORTED;
    if (!cutoff_fits(prm, prm->depth)) return FMM_E_UNSUPPORTED;
    max_leaves = prm->max_leaves > 0 ? prm->max_leaves : int64_t(M) << (2 * prm->depth);
    sh.batched = true;
    sh.n_inst = M;
    sh.n_cap = prm->n_max;
    sh.Lmax = prm->depth;
    sh.key_bits = ceil_log2(M) + 2 * sh.Lmax;
    if (sh.key_bits > 32) return FMM_E_UNSUPPORTED;
    // sum over instances of (4^L + 1) leaf entries, and of Lambda(L) = (4 4^L - 1) / 3 boxes
    sh.leaf_entries = max_leaves + M;
    sh.boxes = (4 * max_leaves + 2) / 3;
    sh.split_boxes = sh.boxes;
    // workgroup numbers of a launch are int32
    if (sh.boxes > int64_t(0x3fffffff) || sh.leaf_entries > int64_t(0x7fffffff)) return FMM_E_UNSUPPORTED;
    return FMM_OK;
}

struct Layout {
    size_t inst, tables, bad_blk, bbox, leaf_start, hist, hist_scan, scan_part;
    size_t key, ksorted, perm, xs, ys, gs, ktmp, itmp, xt, yt, gt, pk, blk_tab, me, le, le_part[2];
    size_t tkey, tks, tperm, txs, tys, tleaf_start, tbad;
    size_t fgt_a, fgt_b, fgt_h;
    size_t t_m2m, t_l2l, t_h64, t_h32, t_sin, t_sout;
    size_t counts, status, work, order;
    size_t total;
};

Layout make_layout(const Shape& sh, int P, bool mixed)
{
    const size_t n = size_t(std::max<int64_t>(sh.n_cap, 1));
    const size_t m = size_t(sh.m_cap);
    const size_t nm = std::max(n, m);   // the radix temporaries serve both point sets
    const size_t nblk = size_t(radix_blocks(int64_t(nm)));
    const size_t nhist = size_t(256) * nblk;
    const size_t nscan = (nhist + kScanChunk - 1) / kScanChunk;
    Layout ly{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    ly.inst = take(sizeof(Inst) * size_t(sh.n_inst));
    ly.tables = take(sizeof(int32_t) * size_t(kMaxLaunches) * size_t(table_ints(sh.n_inst)));
    ly.bad_blk = take(sizeof(int32_t) * nblk);
    ly.bbox = take(sizeof(double) * 8 * kBBoxBlocks);
    ly.leaf_start = take(sizeof(int32_t) * size_t(sh.leaf_entries));
    ly.hist = take(sizeof(int32_t) * nhist);
    ly.hist_scan = take(sizeof(int32_t) * (nhist + 1));   // + the grand total
    ly.scan_part = take(sizeof(int32_t) * (nscan + 1));
    ly.key = take(sizeof(uint32_t) * n);
    ly.ksorted = take(sizeof(uint32_t) * n);
    ly.perm = take(sizeof(uint32_t) * n);
    ly.xs = take(sizeof(double) * n);
    ly.ys = take(sizeof(double) * n);
    ly.gs = take(sizeof(double) * n);
    ly.ktmp = take(sizeof(uint32_t) * nm);
    ly.itmp = take(sizeof(uint32_t) * nm);
    ly.xt = take(sizeof(double) * nm);
    ly.yt = take(sizeof(double) * nm);
    ly.gt = take(sizeof(double) * n);
    ly.tkey = take(sizeof(uint32_t) * m);
    ly.tks = take(sizeof(uint32_t) * m);
    ly.tperm = take(sizeof(uint32_t) * m);
    ly.txs = take(sizeof(double) * m);
    ly.tys = take(sizeof(double) * m);
    ly.tleaf_start = take(m ? sizeof(int32_t) * size_t(sh.leaf_entries) : 0);
    ly.tbad = take(sizeof(int32_t) * size_t(radix_blocks(int64_t(m))));
    ly.pk = take(mixed ? sizeof(float4) * n : 0);
    ly.blk_tab = take(size_t(kBlockPolicies) * kBlockTabBytes);
    // expansions: P >= p coefficients per box (the compiled size), zero-padded
    ly.me = take(sizeof(cd) * size_t(sh.boxes) * P);
    ly.le = take(sizeof(cd) * size_t(sh.boxes) * P);
    ly.le_part[0] = take(sizeof(cd) * size_t(sh.split_boxes) * P);
    ly.le_part[1] = take(sizeof(cd) * size_t(sh.split_boxes) * P);
    ly.t_m2m = take(sizeof(cd) * 4 * P * P);
    ly.t_l2l = take(sizeof(cd) * 4 * P * P);
    ly.t_h64 = take(sizeof(cd) * kHankelGrid * kHankelGrid * (2 * P - 1));
    ly.t_h32 = take(sizeof(cf) * kHankelGrid * kHankelGrid * (2 * P - 1));
    ly.t_sin = take(sizeof(double) * P);
    ly.t_sout = take(sizeof(double) * P);
    const bool fgt = sh.fgt_nc >= 0;
    const size_t fgt_boxes = fgt ? size_t(1) << (2 * sh.depth[0]) : 0;
    ly.fgt_a = take(sizeof(double) * fgt_boxes * P * P);
    const size_t parts = fgt ? size_t(fgt_parts(P, sh.depth[0], sh.fgt_nc)) : 0;
    ly.fgt_b = take(sizeof(double) * parts * fgt_boxes * P * P);
    ly.fgt_h = take(fgt ? sizeof(double) * size_t(2 * sh.fgt_nc + 1) * (2 * P - 1) : 0);
    // batched plans: what the table kernel reports of a call
    ly.counts = take(sizeof(int32_t) * 2);
    ly.status = take(sizeof(int32_t));
    ly.work = take(sh.batched ? sizeof(double) * size_t(sh.n_inst) : 0);
    ly.order = take(sh.batched ? sizeof(int32_t) * size_t(sh.n_inst) : 0);
    ly.total = off;
    return ly;
}

}  // namespace

// Stage timing: every timed evaluation records ST_COUNT + 1 events into one
// slot of a ring; a slot is harvested (its stage times added to the totals)
// before it is reused and when fmm_stats is called, so a run of timed
// evaluations never waits on the device.
constexpr int kTimingRing = 32;

struct fmm_plan_s {
    fmm_params prm;
    int P;
    bool auto_domain;
    bool mixed;
    bool batch;
    Shape shape;
    Tuning tune;
    std::vector<Launch> launches;
    std::vector<int32_t> host_tables;    // kMaxLaunches work tables of table_ints(n_inst)
    std::vector<int32_t> part1_levels;   // per instance: bit l set if M2L level l has a second partial sum
    std::vector<int32_t> g64;            // per instance: wavefronts per list on its split FP64 M2L levels
    int32_t* d_tables;
    Buffers buf;
    // batched plans: capacities and the device outputs of the table kernel
    int64_t max_leaves;
    int32_t* d_counts;                   // [2] particles and leaf entries of the last call
    int32_t* d_status;                   // the last call's instance set: FMM_OK or why it was rejected
    double* d_work;                      // [max_inst] work estimates of the last call's instances
    int32_t* d_order;                    // [max_inst] their launch order
    int32_t last_inst;                   // instance set of the last call (autotuning re-times it)
    int32_t tune_timed;                  // the last autotuning: candidates timed
    double tune_near_share;              // and the work model's near-field share that ordered them
    const int64_t* last_offsets;
    const int32_t* last_depths;
    int64_t last_n;
    int64_t last_m;                      // target points of the last evaluation (0: none)
    hipStream_t last_stream;             // stream of the last evaluation (inspection waits on it)
    // the radix sort's ping-pong arrays, dead outside the tree build: the
    // interaction-list dump stages its chunks there
    char* dump_scratch;
    size_t dump_scratch_bytes;
    // stage timing
    bool timing;
    bool have_events;
    hipEvent_t ev[kTimingRing][ST_COUNT + 1];
    bool pending[kTimingRing];
    int64_t next_slot;
    int64_t n_timed;
    double total_ms[ST_COUNT];
    // batched form: the evaluation captured once per set of arrays, replayed
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    const void* gptr[5];
    // time stepping: one step captured once per set of arrays, n and dt
    hipGraph_t sgraph;
    hipGraphExec_t sgexec;
    const void* sptr[4];
    int64_t sn;
    double sdt;
};

namespace {

hipError_t harvest(fmm_plan_s* pl, int slot)
{
    if (!pl->pending[slot]) return hipSuccess;
    hipError_t e = hipEventSynchronize(pl->ev[slot][ST_COUNT]);
    if (e != hipSuccess) return e;
    for (int i = 0; i < ST_COUNT; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, pl->ev[slot][i], pl->ev[slot][i + 1]);
        if (e != hipSuccess) return e;
        pl->total_ms[i] += ms;
    }
    pl->pending[slot] = false;
    pl->n_timed += 1;
    return hipSuccess;
}

void destroy_events(fmm_plan_s* pl, int upto_slot)
{
    for (int r = 0; r < upto_slot; ++r)
        for (int i = 0; i <= ST_COUNT; ++i) hipEventDestroy(pl->ev[r][i]);
}

void drop_graph(fmm_plan_s* pl)
{
    if (pl->gexec) hipGraphExecDestroy(pl->gexec);
    if (pl->graph) hipGraphDestroy(pl->graph);
    pl->gexec = nullptr;
    pl->graph = nullptr;
    for (auto& q : pl->gptr) q = nullptr;
    if (pl->sgexec) hipGraphExecDestroy(pl->sgexec);
    if (pl->sgraph) hipGraphDestroy(pl->sgraph);
    pl->sgexec = nullptr;
    pl->sgraph = nullptr;
    for (auto& q : pl->sptr) q = nullptr;
    pl->sn = -1;
}

// Capture the enqueue callback into a graph on the plan's private stream.
template <typename F>
hipError_t capture(fmm_plan_s* pl, F&& enqueue, hipGraph_t* graph, hipGraphExec_t* exec)
{
    *graph = nullptr;
    *exec = nullptr;
    if (!pl->cap_stream) {
        const hipError_t e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            pl->cap_stream = nullptr;
            return e;
        }
    }
    hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t ce = enqueue(pl->cap_stream);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(pl->cap_stream, &gr);
    if (ce != hipSuccess || e != hipSuccess || !gr) {
        if (gr) hipGraphDestroy(gr);
        return ce != hipSuccess ? ce : (e != hipSuccess ? e : hipErrorUnknown);
    }
    e = hipGraphInstantiate(exec, gr, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(gr);
        *exec = nullptr;
        return e;
    }
    *graph = gr;
    return hipSuccess;
}

SchedCfg sched_cfg(const fmm_plan_s* pl)
{
    return SchedCfg{pl->mixed ? 1 : 0, pl->prm.fp32_fine_levels, pl->tune.split_max, pl->tune.p2p_waves};
}

// The fixed launch list for trees no deeper than Lmax: upward groups, the
// four M2L launches (FP64 / FP32 levels x split / unsplit), downward groups,
// the near field.
std::vector<LaunchDesc> launch_list(int Lmax, bool mixed)
{
    std::vector<LaunchDesc> v;
    for (int g = 0; g < sched_up_groups(Lmax); ++g) v.push_back(LaunchDesc{L_UP, g, 0, 0});
    for (int fp32 = 0; fp32 < (mixed ? 2 : 1); ++fp32)
        for (int part = 0; part < 2; ++part) v.push_back(LaunchDesc{L_M2L, 0, fp32, part});
    for (int g = 0; g < sched_down_groups(Lmax); ++g) v.push_back(LaunchDesc{L_DOWN, g, 0, 0});
    v.push_back(LaunchDesc{L_P2P, 0, 0, 0});
    return v;
}

// Workgroups a launch can need over any instance set that fits a batched
// plan: with c = max over depths L <= Lmax of (wg(L) - b 4^L), b = wg(Lmax) /
// 4^Lmax, every instance needs at most c + b 4^L, so a set needs at most
// n_inst c + b sum 4^L <= max_inst c + b max_leaves.
int64_t capacity_bound(const SchedCfg& cfg, const LaunchDesc& d, int Lmax, int max_inst, int64_t max_leaves)
{
    int wg, a0, a1;
    sched_inst(cfg, d, Lmax, wg, a0, a1);
    const double b = double(wg) / std::ldexp(1.0, 2 * Lmax);
    double c = 0.0;
    for (int L = 0; L <= Lmax; ++L) {
        sched_inst(cfg, d, L, wg, a0, a1);
        c = std::max(c, double(wg) - b * std::ldexp(1.0, 2 * L));
    }
    return int64_t(std::ceil(double(max_inst) * c + b * double(max_leaves)));
}

// Launch list and, for single plans, the work tables for the current
// tuning.  Workgroups of a launch are numbered instance after instance (in
// the launch order); an instance without work in a launch gets an empty
// range.  Single plans keep only the launches with work and size them
// exactly; batched plans keep the whole list, sized for their capacities,
// and get their tables from the device at every call.
void build_schedule(fmm_plan_s* pl)
{
    const Shape& sh = pl->shape;
    const int n = sh.n_inst;
    const int ti = table_ints(n);
    const SchedCfg cfg = sched_cfg(pl);
    pl->launches.clear();
    pl->host_tables.assign(size_t(kMaxLaunches) * ti, 0);
    const std::vector<LaunchDesc> list = launch_list(sh.Lmax, pl->mixed);
    if (sh.batched) {
        // one workgroup per work item of the largest instance set that fits
        // (a workgroup past the call's work returns at once); launches no
        // instance that fits can use are left out
        for (const LaunchDesc& d : list) {
            const int64_t bound = capacity_bound(cfg, d, sh.Lmax, n, pl->max_leaves);
            if (bound <= 0) continue;
            const int groups = d.kind == L_M2L && d.part == 0 ? 3 : 1;
            pl->launches.push_back(Launch{d, int(bound), int(pl->launches.size()), groups});
        }
        return;
    }
    // launch order of the instances: by decreasing estimated work, or as given
    std::vector<int32_t> ord(n);
    for (int k = 0; k < n; ++k) ord[k] = pl->tune.work_order ? sh.by_work[k] : k;
    pl->part1_levels.assign(n, 0);
    pl->g64.assign(n, 2);
    for (int i = 0; i < n; ++i) sched_m2l_groups(cfg, sh.depth[i], pl->g64[i], pl->part1_levels[i]);
    for (const LaunchDesc& d : list) {
        const int t = int(pl->launches.size());
        int32_t* tb = pl->host_tables.data() + size_t(t) * ti;
        tb[0] = 0;
        int groups = 1;
        for (int k = 0; k < n; ++k) {
            const int i = ord[k];
            int wg, a0, a1;
            sched_inst(cfg, d, sh.depth[i], wg, a0, a1);
            tb[k + 1] = tb[k] + wg;
            tb[n + 1 + 2 * k] = a0;
            tb[n + 2 + 2 * k] = a1;
            tb[3 * n + 1 + k] = i;
            if (d.kind == L_M2L && d.part == 0 && wg > 0)
                groups = std::max(groups, d.fp32 ? 3 : pl->g64[i]);
        }
        if (tb[n] > 0) pl->launches.push_back(Launch{d, tb[n], t, groups});
    }
}

std::vector<Inst> build_inst(const fmm_plan_s* pl)
{
    const Shape& sh = pl->shape;
    std::vector<Inst> v(sh.n_inst);
    for (int i = 0; i < sh.n_inst; ++i) {
        Inst& I = v[i];
        I.part_off = sh.part_off[i];
        I.leaf_off = sh.leaf_off[i];
        I.box_off = sh.box_off[i];
        I.split_off = sh.split_off[i];
        I.L = sh.depth[i];
        I.split = sched_split_level(I.L, pl->tune.split_max);
        I.part1 = pl->part1_levels[i];
        I.g64 = pl->g64[i];
        if (pl->auto_domain)   // the bounding square is written on the device by every evaluation
            I.dom = Domain{0.0, 0.0, 1.0, std::ldexp(1.0, I.L)};
        else
            I.dom = Domain{pl->prm.x0, pl->prm.y0, pl->prm.width, std::ldexp(1.0, I.L) / pl->prm.width};
    }
    return v;
}

hipError_t upload_schedule(fmm_plan_s* pl, hipStream_t st)
{
    build_schedule(pl);
    drop_graph(pl);
    if (pl->shape.batched) return hipSuccess;   // tables come from the device at every call
    std::vector<Inst> iv = build_inst(pl);
    hipError_t e = hipSuccess;
    if (pl->auto_domain && pl->last_n > 0) {
        // keep the last evaluation's bounding square for inspection
        e = hipMemcpyAsync(&iv[0].dom, &pl->buf.inst[0].dom, sizeof(Domain), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->buf.inst, iv.data(), iv.size() * sizeof(Inst), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pl->d_tables, pl->host_tables.data(), pl->host_tables.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the host vectors go out of scope
    return e;
}

Work work_of(const fmm_plan_s* pl, const Launch& ln)
{
    const int n = pl->shape.n_inst;
    const int32_t* tb = pl->d_tables + size_t(ln.table) * table_ints(n);
    return Work{tb, tb + n + 1, tb + 3 * n + 1};
}

// Enqueue one whole evaluation on st: velocities at the particles, or, when
// m > 0, at the m target points (tx, ty), sorted into the same tree.
hipError_t enqueue_all(fmm_plan_s* pl, int64_t n, const double* x, const double* y, const double* g, double* u,
                       double* v, hipStream_t st, bool timing, int slot, int64_t m = 0, const double* tx = nullptr,
                       const double* ty = nullptr)
{
    const Buffers& b = pl->buf;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    auto mark = [&](int i) { if (timing) chk(hipEventRecord(pl->ev[slot][i], st)); };
    const int P = pl->P, p = pl->prm.p;
    const NearKernel nk{pl->prm.kernel, pl->prm.sigma, pl->prm.lj_epsilon, pl->prm.cutoff};
    const bool far = pl->prm.kernel != FMM_KERNEL_LENNARD_JONES;   // short range: near field only

    mark(ST_TREE);
    if (pl->auto_domain) chk(launch_domain(b, int(n), x, y, pl->shape.depth[0], st, int(m), tx, ty));
    // batched plans: n and the leaf entries are capacities; the call's counts are on the device
    chk(launch_tree(b, int(n), x, y, g, pl->shape.key_bits, pl->shape.leaf_entries, pl->mixed, st,
                    pl->shape.batched ? pl->d_counts : nullptr));
    if (m > 0) chk(launch_tree_points(b, int(m), tx, ty, pl->shape.key_bits, pl->shape.leaf_entries, st));
    if (pl->shape.fgt_nc >= 0) {   // Gauss transform: Hermite, Hermite to Taylor, Taylor evaluation
        mark(ST_UP);
        const int L = pl->shape.depth[0], nc = pl->shape.fgt_nc;
        chk(launch_fgt(b, P, int(n), L, pl->prm.sigma, nc, fgt_parts(P, L, nc), int(m), u, v, st));
        for (int s2 = ST_M2L; s2 <= ST_COUNT; ++s2) mark(s2);
        return e;
    }
    int stage = ST_TREE;
    for (const Launch& ln : pl->launches) {
        const int kind = ln.desc.kind;
        const int want = kind == L_UP ? ST_UP : kind == L_M2L ? ST_M2L : kind == L_DOWN ? ST_DOWN : ST_P2P;
        while (stage < want) mark(++stage);
        const Work w = work_of(pl, ln);
        if (!far && kind != L_P2P) continue;
        switch (kind) {
            case L_UP: chk(launch_upward(b, P, p, w, ln.nwg, ln.desc.group == 0, st)); break;
            case L_M2L:   // the matrix cores take the unsplit FP32 levels (split ones stage too much per item)
                chk(launch_m2l(b, P, w, ln.nwg, ln.desc.fp32 != 0, pl->tune.m2l_mfma != 0 && ln.desc.part == 1,
                               ln.groups, st));
                break;
            case L_DOWN: chk(launch_downward(b, P, w, ln.nwg, st)); break;
            case L_P2P:
                if (m > 0)
                    chk(launch_p2p_at(b, P, pl->shape.depth[0], nk, pl->tune.p2p_block, u, v, st));
                else
                    chk(launch_p2p(b, P, w, ln.nwg, pl->tune.p2p_waves, pl->mixed, nk, pl->tune.p2p_block, u, v, st));
                break;
        }
    }
    while (stage < ST_COUNT) mark(++stage);
    return e;
}

void rank_by_work(Shape& sh, int p)
{
    sh.work.resize(sh.n_inst);
    for (int i = 0; i < sh.n_inst; ++i) {
        const int64_t end = i + 1 < sh.n_inst ? sh.part_off[i + 1] : sh.n_cap;
        sh.work[i] = sched_work(end - sh.part_off[i], sh.depth[i], p);
    }
    sh.by_work.resize(sh.n_inst);
    for (int i = 0; i < sh.n_inst; ++i) sh.by_work[i] = i;
    std::stable_sort(sh.by_work.begin(), sh.by_work.end(),
                     [&](int32_t a, int32_t b) { return sh.work[a] > sh.work[b]; });
}

fmm_status make_plan(const fmm_params* prm, Shape&& sh, bool batch, void* d_workspace, size_t bytes, void* stream,
                     fmm_plan_t* out, bool events = true, int64_t max_leaves = 0)
{
    if (!sh.batched) rank_by_work(sh, prm->p);
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) return FMM_E_ARG;
    const int P = instantiated_terms(prm->p);
    const bool mixed = prm->precision == FMM_PREC_MIXED;
    const Layout ly = make_layout(sh, P, mixed);
    if (bytes < ly.total) return FMM_E_CAPACITY;

    fmm_plan_s* pl = new (std::nothrow) fmm_plan_s();
    if (!pl) return FMM_E_NOMEM;
    pl->prm = *prm;
    pl->P = P;
    pl->auto_domain = !(prm->width > 0.0);
    pl->mixed = mixed;
    pl->batch = batch;
    // measured defaults: in FP64 the utilisation-first blocking is faster on
    // every workload, in the mixed form the power-of-two one on uniform
    // particles; the FP32 M2L levels run paired on the vector units (faster
    // than the matrix cores on C2 and C5)
    pl->tune.p2p_block = mixed ? 0 : 1;
    pl->tune.m2l_mfma = 0;
    pl->shape = std::move(sh);
    pl->last_n = -1;
    pl->last_m = 0;
    pl->last_stream = static_cast<hipStream_t>(stream);
    pl->sn = -1;
    char* base = static_cast<char*>(d_workspace);
    Buffers& b = pl->buf;
    b.inst = reinterpret_cast<Inst*>(base + ly.inst);
    b.n_inst = pl->shape.n_inst;
    b.key_shift = 2 * pl->shape.Lmax;
    pl->d_tables = reinterpret_cast<int32_t*>(base + ly.tables);
    b.bad_blk = reinterpret_cast<int32_t*>(base + ly.bad_blk);
    b.bbox = reinterpret_cast<double*>(base + ly.bbox);
    b.leaf_start = reinterpret_cast<int32_t*>(base + ly.leaf_start);
    b.hist = reinterpret_cast<int32_t*>(base + ly.hist);
    b.hist_scan = reinterpret_cast<int32_t*>(base + ly.hist_scan);
    b.scan_part = reinterpret_cast<int32_t*>(base + ly.scan_part);
    b.key = reinterpret_cast<uint32_t*>(base + ly.key);
    b.ksorted = reinterpret_cast<uint32_t*>(base + ly.ksorted);
    b.perm = reinterpret_cast<uint32_t*>(base + ly.perm);
    b.xs = reinterpret_cast<double*>(base + ly.xs);
    b.ys = reinterpret_cast<double*>(base + ly.ys);
    b.gs = reinterpret_cast<double*>(base + ly.gs);
    b.ktmp = reinterpret_cast<uint32_t*>(base + ly.ktmp);
    b.itmp = reinterpret_cast<uint32_t*>(base + ly.itmp);
    b.xt = reinterpret_cast<double*>(base + ly.xt);
    b.yt = reinterpret_cast<double*>(base + ly.yt);
    b.gt = reinterpret_cast<double*>(base + ly.gt);
    b.pk = mixed ? reinterpret_cast<float4*>(base + ly.pk) : nullptr;
    b.blk_tab = reinterpret_cast<uint8_t*>(base + ly.blk_tab);
    const bool targets = pl->shape.m_cap > 0;
    b.tkey = targets ? reinterpret_cast<uint32_t*>(base + ly.tkey) : nullptr;
    b.tks = targets ? reinterpret_cast<uint32_t*>(base + ly.tks) : nullptr;
    b.tperm = targets ? reinterpret_cast<uint32_t*>(base + ly.tperm) : nullptr;
    b.txs = targets ? reinterpret_cast<double*>(base + ly.txs) : nullptr;
    b.tys = targets ? reinterpret_cast<double*>(base + ly.tys) : nullptr;
    b.tleaf_start = targets ? reinterpret_cast<int32_t*>(base + ly.tleaf_start) : nullptr;
    b.tbad = targets ? reinterpret_cast<int32_t*>(base + ly.tbad) : nullptr;
    b.me = reinterpret_cast<cd*>(base + ly.me);
    b.le = reinterpret_cast<cd*>(base + ly.le);
    b.le_part[0] = reinterpret_cast<cd*>(base + ly.le_part[0]);
    b.le_part[1] = reinterpret_cast<cd*>(base + ly.le_part[1]);
    pl->dump_scratch = base + ly.ktmp;
    pl->dump_scratch_bytes = ly.tkey - ly.ktmp;
    pl->max_leaves = max_leaves;
    pl->d_counts = reinterpret_cast<int32_t*>(base + ly.counts);
    pl->d_status = reinterpret_cast<int32_t*>(base + ly.status);
    pl->d_work = reinterpret_cast<double*>(base + ly.work);
    pl->d_order = reinterpret_cast<int32_t*>(base + ly.order);
    pl->last_inst = 0;
    b.t_m2m = reinterpret_cast<cd*>(base + ly.t_m2m);
    b.t_l2l = reinterpret_cast<cd*>(base + ly.t_l2l);
    b.t_h64 = reinterpret_cast<cd*>(base + ly.t_h64);
    b.t_h32 = reinterpret_cast<cf*>(base + ly.t_h32);
    b.t_sin = reinterpret_cast<double*>(base + ly.t_sin);
    b.t_sout = reinterpret_cast<double*>(base + ly.t_sout);
    const bool fgt = pl->shape.fgt_nc >= 0;
    b.fgt_a = fgt ? reinterpret_cast<double*>(base + ly.fgt_a) : nullptr;
    b.fgt_b = fgt ? reinterpret_cast<double*>(base + ly.fgt_b) : nullptr;
    b.fgt_h = fgt ? reinterpret_cast<double*>(base + ly.fgt_h) : nullptr;

    const size_t nh = size_t(kHankelGrid) * kHankelGrid * (2 * P - 1);
    std::vector<cd> m2m(size_t(4) * P * P), l2l(size_t(4) * P * P), h64(nh);
    std::vector<cf> h32(nh);
    std::vector<double> sin_(P), sout_(P);
    build_tables(P, prm->p, m2m.data(), l2l.data(), h64.data(), h32.data(), sin_.data(), sout_.data());

    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    auto cp = [&](void* dst, const void* src, size_t nbytes) {
        if (e == hipSuccess) e = hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, st);
    };
    cp(b.t_m2m, m2m.data(), m2m.size() * sizeof(cd));
    cp(b.t_l2l, l2l.data(), l2l.size() * sizeof(cd));
    cp(b.t_h64, h64.data(), h64.size() * sizeof(cd));
    cp(b.t_h32, h32.data(), h32.size() * sizeof(cf));
    cp(b.t_sin, sin_.data(), sin_.size() * sizeof(double));
    cp(b.t_sout, sout_.data(), sout_.size() * sizeof(double));
    std::vector<uint8_t> blk(size_t(kBlockPolicies) * kBlockTabBytes);
    for (int k = 0; k < kBlockPolicies; ++k) block_table(k, blk.data() + size_t(k) * kBlockTabBytes);
    cp(b.blk_tab, blk.data(), blk.size());
    std::vector<double> fgt_h;
    if (fgt) {
        const int nc = pl->shape.fgt_nc;
        fgt_h.resize(size_t(2 * nc + 1) * (2 * P - 1));
        const double w = std::ldexp(prm->width, -pl->shape.depth[0]);
        fgt_hermite_table(P, nc, w / (std::sqrt(2.0) * prm->sigma), fgt_h.data());
        cp(b.fgt_h, fgt_h.data(), fgt_h.size() * sizeof(double));
    }
    if (e == hipSuccess) e = upload_schedule(pl, st);      // synchronises st
    if (e != hipSuccess) {
        delete pl;
        return FMM_E_DEVICE;
    }
    pl->have_events = events;
    for (int r = 0; r < kTimingRing && pl->have_events; ++r)
        for (int i = 0; i <= ST_COUNT; ++i)
            if (hipEventCreate(&pl->ev[r][i]) != hipSuccess) {
                for (int j = 0; j < i; ++j) hipEventDestroy(pl->ev[r][j]);
                destroy_events(pl, r);
                pl->have_events = false;
                break;
            }
    *out = pl;
    return FMM_OK;
}

fmm_status run_once(fmm_plan_s* pl, int64_t n, const double* x, const double* y, const double* g, double* u,
                    double* v, void* stream)
{
    if (pl->batch)   // the instance set of the plan's last call
        return fmm_evaluate_batch(pl, pl->last_inst, pl->last_offsets, pl->last_depths, x, y, g, u, v, stream);
    return fmm_evaluate(pl, n, x, y, g, u, v, stream);
}

}  // namespace

namespace fmm {

// A single-instance plan over a device buffer the library itself provides
// (no stage-timing events, so building it creates no HIP objects beyond the
// uploads it enqueues).
fmm_status plan_in_buffer(const fmm_params* prm, void* d_buffer, size_t bytes, void* stream, fmm_plan_t* out)
{
    if (!out || !d_buffer) return FMM_E_ARG;
    *out = nullptr;
    fmm_status s = validate_common(prm);
    if (s != FMM_OK) return s;
    Shape sh;
    s = single_shape(prm, sh);
    if (s != FMM_OK) return s;
    return make_plan(prm, std::move(sh), false, d_buffer, bytes, stream, out, false);
}

}  // namespace fmm

extern "C" {

const char* fmm_status_string(fmm_status s)
{
    switch (s) {
        case FMM_OK: return "ok";
        case FMM_E_ARG: return "invalid argument";
        case FMM_E_CAPACITY: return "capacity exceeded";
        case FMM_E_DOMAIN: return "particles outside the domain";
        case FMM_E_NOMEM: return "host allocation failed";
        case FMM_E_DEVICE: return "HIP runtime error";
        case FMM_E_UNSUPPORTED: return "unsupported parameter combination";
    }
    return "unknown status";
}

const char* fmm_stage_name(int32_t stage)
{
    if (stage < 0 || stage >= ST_COUNT) return nullptr;
    return kStageNames[stage];
}

fmm_status fmm_workspace_size(const fmm_params* prm, size_t* bytes)
{
    if (!bytes) return FMM_E_ARG;
    fmm_status s = validate_common(prm);
    if (s != FMM_OK) return s;
    Shape sh;
    int64_t max_leaves = 0;
    s = prm->max_instances > 1 ? batch_shape(prm, sh, max_leaves) : single_shape(prm, sh);
    if (s != FMM_OK) return s;
    *bytes = make_layout(sh, instantiated_terms(prm->p), prm->precision == FMM_PREC_MIXED).total;
    return FMM_OK;
}

fmm_status fmm_plan(const fmm_params* prm, void* d_workspace, size_t bytes, void* stream, fmm_plan_t* out)
{
    if (!out || !d_workspace) return FMM_E_ARG;
    *out = nullptr;
    fmm_status s = validate_common(prm);
    if (s != FMM_OK) return s;
    Shape sh;
    if (prm->max_instances > 1) {
        int64_t max_leaves = 0;
        s = batch_shape(prm, sh, max_leaves);
        if (s != FMM_OK) return s;
        return make_plan(prm, std::move(sh), true, d_workspace, bytes, stream, out, true, max_leaves);
    }
    s = single_shape(prm, sh);
    if (s != FMM_OK) return s;
    return make_plan(prm, std::move(sh), false, d_workspace, bytes, stream, out);
}

fmm_status fmm_set_timing(fmm_plan_t plan, int32_t on)
{
    if (!plan) return FMM_E_ARG;
    if (on && !plan->have_events) return FMM_E_DEVICE;
    if (plan->have_events)
        for (int r = 0; r < kTimingRing; ++r)
            if (harvest(plan, r) != hipSuccess) return FMM_E_DEVICE;
    plan->timing = on != 0;
    plan->n_timed = 0;
    for (int i = 0; i < ST_COUNT; ++i) plan->total_ms[i] = 0.0;
    return FMM_OK;
}

fmm_status fmm_evaluate(fmm_plan_t plan, int64_t n, const double* d_x, const double* d_y,
                        const double* d_gamma, double* d_u, double* d_v, void* stream)
{
    if (!plan || plan->batch) return FMM_E_ARG;
    if (n < 0) return FMM_E_ARG;
    if (n > plan->shape.n_cap) return FMM_E_CAPACITY;
    if (n > 0 && (!d_x || !d_y || !d_gamma || !d_u || !d_v)) return FMM_E_ARG;
    plan->last_n = n;
    plan->last_m = 0;
    plan->last_stream = static_cast<hipStream_t>(stream);
    if (n == 0) return FMM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    const int slot = int(plan->next_slot % kTimingRing);
    if (plan->timing) {
        e = harvest(plan, slot);
        plan->next_slot += 1;
    }
    if (e == hipSuccess) e = enqueue_all(plan, n, d_x, d_y, d_gamma, d_u, d_v, st, plan->timing, slot);
    if (plan->timing && e == hipSuccess) plan->pending[slot] = true;
    return e == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_evaluate_at(fmm_plan_t plan, int64_t n, const double* d_x, const double* d_y,
                           const double* d_gamma, int64_t m, const double* d_tx, const double* d_ty, double* d_u,
                           double* d_v, void* stream)
{
    if (!plan || plan->batch) return FMM_E_ARG;
    if (n < 0 || m < 0) return FMM_E_ARG;
    if (plan->mixed || plan->prm.kernel == FMM_KERNEL_LENNARD_JONES) return FMM_E_UNSUPPORTED;
    if (n > plan->shape.n_cap || m > plan->shape.m_cap) return FMM_E_CAPACITY;
    if (n > 0 && (!d_x || !d_y || !d_gamma)) return FMM_E_ARG;
    if (m > 0 && (!d_tx || !d_ty || !d_u || !d_v)) return FMM_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    plan->last_n = 0;
    plan->last_m = 0;
    plan->last_stream = static_cast<hipStream_t>(stream);
    if (m == 0) return FMM_OK;
    if (n == 0) {   // no sources: the velocity vanishes everywhere
        return launch_zero2(m, d_u, d_v, st) == hipSuccess ? FMM_OK : FMM_E_DEVICE;
    }
    plan->last_n = n;
    plan->last_m = m;
    hipError_t e = hipSuccess;
    const int slot = int(plan->next_slot % kTimingRing);
    if (plan->timing) {
        e = harvest(plan, slot);
        plan->next_slot += 1;
    }
    if (e == hipSuccess)
        e = enqueue_all(plan, n, d_x, d_y, d_gamma, d_u, d_v, st, plan->timing, slot, m, d_tx, d_ty);
    if (plan->timing && e == hipSuccess) plan->pending[slot] = true;
    return e == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_evaluate_batch(fmm_plan_t plan, int32_t n_inst, const int64_t* d_offsets, const int32_t* d_depths,
                              const double* d_x, const double* d_y, const double* d_gamma, double* d_u, double* d_v,
                              void* stream)
{
    if (!plan || !plan->batch) return FMM_E_ARG;
    if (n_inst < 1 || n_inst > plan->shape.n_inst) return FMM_E_ARG;
    if (!d_offsets || !d_depths || !d_x || !d_y || !d_gamma || !d_u || !d_v) return FMM_E_ARG;
    const int64_t n = plan->shape.n_cap;   // capacity: the grids are sized for it
    hipStream_t st = static_cast<hipStream_t>(stream);
    plan->last_n = n;
    plan->last_m = 0;
    plan->last_stream = st;
    plan->last_inst = n_inst;
    plan->last_offsets = d_offsets;
    plan->last_depths = d_depths;
    // the call's instance table -> the plan's work tables, on the device
    BatchSched bs{};
    bs.n_inst = n_inst;
    bs.offsets = d_offsets;
    bs.depths = d_depths;
    bs.max_inst = plan->shape.n_inst;
    bs.n_max = n;
    bs.leaf_cap = plan->shape.leaf_entries;
    bs.box_cap = plan->shape.boxes;
    bs.split_cap = plan->shape.split_boxes;
    bs.depth_max = plan->shape.Lmax;
    bs.p = plan->prm.p;
    bs.work_order = plan->tune.work_order;
    bs.dom = Domain{plan->prm.x0, plan->prm.y0, plan->prm.width, 0.0};
    bs.cfg = sched_cfg(plan);
    bs.n_launch = int(plan->launches.size());
    for (int t = 0; t < bs.n_launch; ++t) bs.launch[t] = plan->launches[size_t(t)].desc;
    bs.inst = plan->buf.inst;
    bs.tables = plan->d_tables;
    bs.counts = plan->d_counts;
    bs.status = plan->d_status;
    bs.work = plan->d_work;
    bs.order = plan->d_order;
    if (launch_batch_schedule(bs, st) != hipSuccess) return FMM_E_DEVICE;
    if (plan->timing) {
        // timed: enqueued eagerly with stage events, no graph
        const int slot = int(plan->next_slot % kTimingRing);
        hipError_t e = harvest(plan, slot);
        plan->next_slot += 1;
        if (e == hipSuccess) e = enqueue_all(plan, n, d_x, d_y, d_gamma, d_u, d_v, st, true, slot);
        if (e == hipSuccess) plan->pending[slot] = true;
        return e == hipSuccess ? FMM_OK : FMM_E_DEVICE;
    }
    const void* ptrs[5] = {d_x, d_y, d_gamma, d_u, d_v};
    bool same = plan->gexec != nullptr;
    for (int i = 0; i < 5 && same; ++i) same = plan->gptr[i] == ptrs[i];
    if (!same) {
        // capture the stage launches for these arrays on the plan's own stream
        if (plan->gexec) hipGraphExecDestroy(plan->gexec);
        if (plan->graph) hipGraphDestroy(plan->graph);
        plan->gexec = nullptr;
        plan->graph = nullptr;
        const hipError_t e = capture(
            plan, [&](hipStream_t cs) { return enqueue_all(plan, n, d_x, d_y, d_gamma, d_u, d_v, cs, false, 0); },
            &plan->graph, &plan->gexec);
        if (e != hipSuccess) return FMM_E_DEVICE;
        for (int i = 0; i < 5; ++i) plan->gptr[i] = ptrs[i];
    }
    return hipGraphLaunch(plan->gexec, st) == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_advance_rk2(fmm_plan_t plan, int64_t n, double* d_x, double* d_y, const double* d_gamma, double dt,
                           int32_t n_steps, double* d_scratch, void* stream)
{
    if (!plan || plan->batch) return FMM_E_ARG;
    if (n < 0 || n_steps < 0 || !std::isfinite(dt)) return FMM_E_ARG;
    if (plan->prm.kernel == FMM_KERNEL_LENNARD_JONES || plan->prm.kernel == FMM_KERNEL_GAUSS_TRANSFORM)
        return FMM_E_UNSUPPORTED;   // forces or a transform, not velocities
    if (n > plan->shape.n_cap) return FMM_E_CAPACITY;
    if (n == 0 || n_steps == 0) return FMM_OK;
    if (!d_x || !d_y || !d_gamma || !d_scratch) return FMM_E_ARG;
    plan->last_n = n;
    plan->last_m = 0;
    plan->last_stream = static_cast<hipStream_t>(stream);
    double* u = d_scratch;
    double* v = d_scratch + n;
    double* xm = d_scratch + 2 * n;
    double* ym = d_scratch + 3 * n;
    const void* ptrs[4] = {d_x, d_y, d_gamma, d_scratch};
    bool same = plan->sgexec != nullptr && plan->sn == n && plan->sdt == dt;
    for (int i = 0; i < 4 && same; ++i) same = plan->sptr[i] == ptrs[i];
    if (!same) {
        if (plan->sgexec) hipGraphExecDestroy(plan->sgexec);
        if (plan->sgraph) hipGraphDestroy(plan->sgraph);
        plan->sgexec = nullptr;
        plan->sgraph = nullptr;
        // one explicit-midpoint step: two evaluations and two particle updates
        auto step = [&](hipStream_t cs) -> hipError_t {
            hipError_t e = enqueue_all(plan, n, d_x, d_y, d_gamma, u, v, cs, false, 0);
            if (e == hipSuccess) e = launch_advance(n, d_x, d_y, u, v, 0.5 * dt, xm, ym, cs);
            if (e == hipSuccess) e = enqueue_all(plan, n, xm, ym, d_gamma, u, v, cs, false, 0);
            if (e == hipSuccess) e = launch_advance(n, d_x, d_y, u, v, dt, d_x, d_y, cs);
            return e;
        };
        if (capture(plan, step, &plan->sgraph, &plan->sgexec) != hipSuccess) return FMM_E_DEVICE;
        for (int i = 0; i < 4; ++i) plan->sptr[i] = ptrs[i];
        plan->sn = n;
        plan->sdt = dt;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int32_t s = 0; s < n_steps; ++s)
        if (hipGraphLaunch(plan->sgexec, st) != hipSuccess) return FMM_E_DEVICE;
    return FMM_OK;
}

fmm_status fmm_get_status(fmm_plan_t plan, void* stream, int64_t* n_bad)
{
    if (!plan || !n_bad) return FMM_E_ARG;
    *n_bad = 0;
    if (plan->last_n <= 0) return FMM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nblk = size_t(radix_blocks(plan->last_n));
    const size_t tblk = size_t(radix_blocks(plan->last_m));
    std::vector<int32_t> per(nblk + tblk);
    if (hipMemcpyAsync(per.data(), plan->buf.bad_blk, nblk * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
        return FMM_E_DEVICE;
    if (tblk > 0 && hipMemcpyAsync(per.data() + nblk, plan->buf.tbad, tblk * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, st) != hipSuccess)
        return FMM_E_DEVICE;
    int32_t rejected = 0;
    if (plan->batch &&
        hipMemcpyAsync(&rejected, plan->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return FMM_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return FMM_E_DEVICE;
    if (rejected != 0) return fmm_status(rejected);   // the call's instance set computed nothing
    int64_t v = 0;
    for (int32_t c : per) v += c;
    *n_bad = v;
    return v == 0 ? FMM_OK : FMM_E_DOMAIN;
}

fmm_status fmm_stats(fmm_plan_t plan, double* stage_ms, int32_t n_stages, int32_t* n_written,
                     int64_t* n_evaluations)
{
    if (!plan || (n_stages > 0 && !stage_ms)) return FMM_E_ARG;
    if (n_written) *n_written = 0;
    if (n_evaluations) *n_evaluations = 0;
    if (!plan->have_events) return FMM_E_DEVICE;
    for (int r = 0; r < kTimingRing; ++r)
        if (harvest(plan, r) != hipSuccess) return FMM_E_DEVICE;
    if (plan->n_timed == 0) return FMM_E_ARG;
    const int m = std::min<int>(n_stages, ST_COUNT);
    for (int i = 0; i < m; ++i) stage_ms[i] = plan->total_ms[i] / double(plan->n_timed);
    if (n_written) *n_written = m;
    if (n_evaluations) *n_evaluations = plan->n_timed;
    return FMM_OK;
}

fmm_status fmm_get_tuning(fmm_plan_t plan, int32_t* p2p_waves, int32_t* m2l_split_max, int32_t* m2l_mfma,
                          int32_t* work_order, int32_t* p2p_block)
{
    if (!plan || !p2p_waves || !m2l_split_max || !m2l_mfma || !work_order || !p2p_block) return FMM_E_ARG;
    *p2p_waves = plan->tune.p2p_waves;
    *m2l_split_max = plan->tune.split_max;
    *m2l_mfma = plan->tune.m2l_mfma;
    *work_order = plan->tune.work_order;
    *p2p_block = plan->tune.p2p_block;
    return FMM_OK;
}

fmm_status fmm_set_tuning(fmm_plan_t plan, int32_t p2p_waves, int32_t m2l_split_max, int32_t m2l_mfma,
                          int32_t work_order, int32_t p2p_block, void* stream)
{
    if (!plan) return FMM_E_ARG;
    if (p2p_waves != 2 && p2p_waves != 4) return FMM_E_ARG;
    if (m2l_split_max < 0 || m2l_split_max > kM2LSplitMaxLevel) return FMM_E_ARG;
    if ((m2l_mfma != 0 && m2l_mfma != 1) || (work_order != 0 && work_order != 1)) return FMM_E_ARG;
    if (p2p_block < 0 || p2p_block >= kBlockPolicies) return FMM_E_ARG;
    plan->tune.p2p_waves = p2p_waves;
    plan->tune.split_max = m2l_split_max;
    plan->tune.m2l_mfma = m2l_mfma;
    plan->tune.work_order = work_order;
    plan->tune.p2p_block = p2p_block;
    return upload_schedule(plan, static_cast<hipStream_t>(stream)) == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_work_estimate(fmm_plan_t plan, double* work, int32_t n_out, int32_t* n_written)
{
    if (!plan || (n_out > 0 && !work)) return FMM_E_ARG;
    if (plan->batch) {   // computed on the device for the last call's instances
        const int m = std::max(0, std::min<int>(n_out, plan->last_inst));
        if (m > 0) {
            if (hipMemcpyAsync(work, plan->d_work, size_t(m) * sizeof(double), hipMemcpyDeviceToHost,
                               plan->last_stream) != hipSuccess ||
                hipStreamSynchronize(plan->last_stream) != hipSuccess)
                return FMM_E_DEVICE;
        }
        if (n_written) *n_written = m;
        return FMM_OK;
    }
    const int m = std::min<int>(n_out, plan->shape.n_inst);
    for (int i = 0; i < m; ++i) work[i] = plan->shape.work[i];
    if (n_written) *n_written = m;
    return FMM_OK;
}

fmm_status fmm_autotune(fmm_plan_t plan, int64_t n, const double* d_x, const double* d_y, const double* d_gamma,
                        double* d_u, double* d_v, void* stream, int32_t reps)
{
    if (!plan) return FMM_E_ARG;
    if (!d_x || !d_y || !d_gamma || !d_u || !d_v) return FMM_E_ARG;
    if (reps < 1) reps = 3;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<int32_t> depths = plan->shape.depth;
    std::vector<int64_t> offs = {0, n};
    if (plan->batch) {
        // the instance set of the last call: its particle count, offsets and depths
        if (plan->last_inst < 1) return FMM_E_ARG;
        int32_t cnt[2] = {0, 0};
        depths.resize(size_t(plan->last_inst));
        offs.resize(size_t(plan->last_inst) + 1);
        if (hipStreamSynchronize(plan->last_stream) != hipSuccess ||
            hipMemcpy(cnt, plan->d_counts, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(depths.data(), plan->last_depths, depths.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(offs.data(), plan->last_offsets, offs.size() * sizeof(int64_t), hipMemcpyDeviceToHost) !=
                hipSuccess)
            return FMM_E_DEVICE;
        n = cnt[0];
        if (n <= 0) return FMM_E_ARG;   // rejected or empty instance set
    }
    if (n <= 0 || n > plan->shape.n_cap) return FMM_E_ARG;

    // signature of the problem: compiled size, precision, n and the depth mix
    char sig[512];
    {
        int64_t hist[kMaxDepth + 1] = {0};
        for (int L : depths) hist[std::min(std::max(L, 0), kMaxDepth)]++;
        std::string d;
        for (int L = 0; L <= kMaxDepth; ++L)
            if (hist[L]) d += std::to_string(L) + "x" + std::to_string(hist[L]) + ",";
        std::snprintf(sig, sizeof(sig), "P%d-%s-f%d-n%lld-%s", plan->P, plan->mixed ? "mixed" : "fp64",
                      plan->mixed ? plan->prm.fp32_fine_levels : 0, (long long)n, d.c_str());
    }
    const char* cache = std::getenv("FMM_AUTOTUNE_CACHE");
    if (cache && *cache) {
        if (FILE* f = std::fopen(cache, "r")) {
            char key[512];
            int w = 0, sm = 0, mf = 0, bk = 0, fw = 0, fsm = 0, fmf = 0, fbk = 0;
            bool found = false;
            while (std::fscanf(f, "%511s %d %d %d %d", key, &w, &sm, &mf, &bk) == 5)
                if (std::strcmp(key, sig) == 0) {   // the last entry wins
                    found = true;
                    fw = w;
                    fsm = sm;
                    fmf = mf;
                    fbk = bk;
                }
            std::fclose(f);
            if (found) {
                plan->tune_timed = 0;
                return fmm_set_tuning(plan, fw, fsm, fmf, plan->tune.work_order, fbk, stream);
            }
        }
    }

    const Tuning saved = plan->tune;
    const bool was_timing = plan->timing;
    plan->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return FMM_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return FMM_E_DEVICE;
    }
    const int waves[2] = {2, 4};
    const int splits[3] = {0, 5, kM2LSplitMaxLevel};
    // the matrix-core choice matters only where some M2L level runs in FP32
    const int n_mfma = (plan->mixed && plan->P <= 24) ? 2 : 1;
    float best = 1e30f;
    Tuning best_t = saved;
    fmm_status rs = FMM_OK;
    int timed = 0;
    auto time_one = [&](int w, int sm, int mf, int bk) {
        if (rs != FMM_OK) return;
        rs = fmm_set_tuning(plan, w, sm, mf, saved.work_order, bk, stream);
        if (rs == FMM_OK) rs = run_once(plan, n, d_x, d_y, d_gamma, d_u, d_v, stream);   // warm-up, capture
        float tmin = 1e30f;
        for (int r = 0; r < reps && rs == FMM_OK; ++r) {
            if (hipEventRecord(e0, st) != hipSuccess) { rs = FMM_E_DEVICE; break; }
            rs = run_once(plan, n, d_x, d_y, d_gamma, d_u, d_v, stream);
            if (rs != FMM_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rs = FMM_E_DEVICE;
                break;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rs = FMM_E_DEVICE; break; }
            tmin = std::min(tmin, ms);
        }
        ++timed;
        if (rs == FMM_OK && tmin < best) {
            best = tmin;
            best_t = plan->tune;
        }
    };
    // The paper's work model (Section 5.2) splits each instance's estimate
    // into the near field (n_nd N_i^2 per leaf, eq. 14, with 2 N_i p for
    // P2M/L2P) and the far field (p^2 (2 n_c + n_IL) per non-leaf box, eq.
    // 13, and p^2 n_IL per leaf): the launch shapes of the larger part are
    // searched first, those of the other part only if it holds at least
    // kTuneMinShare of the estimate.  FMM_AUTOTUNE_EXHAUSTIVE=1 times the
    // whole grid instead.
    double near = 0.0, far = 0.0;
    for (size_t i = 0; i < depths.size(); ++i) {
        const int L = std::min(std::max(int(depths[i]), 0), kMaxDepth);
        const double leaves = std::ldexp(1.0, 2 * L), pp = double(plan->prm.p) * plan->prm.p;
        const double ni = double(offs[i + 1] - offs[i]) / leaves;
        near += leaves * (9.0 * ni * ni + 2.0 * ni * plan->prm.p);
        far += (leaves - 1.0) / 3.0 * pp * 35.0 + (L >= 2 ? leaves * pp * 27.0 : 0.0);
    }
    const double near_share = near + far > 0.0 ? near / (near + far) : 1.0;
    const char* ex = std::getenv("FMM_AUTOTUNE_EXHAUSTIVE");
    if (ex && std::atoi(ex) == 1) {
        for (int mi = 0; mi < n_mfma; ++mi)
            for (int wi = 0; wi < 2; ++wi)
                for (int bk = 0; bk < kBlockPolicies; ++bk)
                    for (int si = 0; si < 3; ++si)
                        time_one(waves[wi], splits[si], n_mfma == 2 ? mi : saved.m2l_mfma, bk);
    } else {
        constexpr double kTuneMinShare = 0.1;
        time_one(saved.p2p_waves, saved.split_max, saved.m2l_mfma, saved.p2p_block);   // the current shape
        auto near_group = [&]() {
            const Tuning b = best_t;
            for (int w : waves)
                for (int bk = 0; bk < kBlockPolicies; ++bk)
                    if (w != b.p2p_waves || bk != b.p2p_block) time_one(w, b.split_max, b.m2l_mfma, bk);
        };
        auto far_group = [&]() {
            const Tuning b = best_t;
            for (int mi = 0; mi < n_mfma; ++mi)
                for (int sm : splits) {
                    const int mf = n_mfma == 2 ? mi : b.m2l_mfma;
                    if (sm != b.split_max || mf != b.m2l_mfma) time_one(b.p2p_waves, sm, mf, b.p2p_block);
                }
        };
        if (near_share >= 0.5) {
            near_group();
            if (1.0 - near_share >= kTuneMinShare) far_group();
        } else {
            far_group();
            if (near_share >= kTuneMinShare) near_group();
        }
    }
    plan->tune_timed = timed;
    plan->tune_near_share = near_share;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    plan->timing = was_timing;
    if (rs != FMM_OK) {
        plan->tune = saved;
        upload_schedule(plan, st);
        return rs;
    }
    rs = fmm_set_tuning(plan, best_t.p2p_waves, best_t.split_max, best_t.m2l_mfma, best_t.work_order,
                        best_t.p2p_block, stream);
    if (rs == FMM_OK && cache && *cache) {
        if (FILE* f = std::fopen(cache, "a")) {
            std::fprintf(f, "%s %d %d %d %d\n", sig, best_t.p2p_waves, best_t.split_max, best_t.m2l_mfma,
                         best_t.p2p_block);
            std::fclose(f);
        }
    }
    return rs;
}

fmm_status fmm_autotune_report(fmm_plan_t plan, int32_t* candidates_timed, double* near_share)
{
    if (!plan || !candidates_timed || !near_share) return FMM_E_ARG;
    *candidates_timed = plan->tune_timed;
    *near_share = plan->tune_near_share;
    return FMM_OK;
}

fmm_status fmm_debug_dump(fmm_plan_t plan, int32_t what, void* host_buf, size_t bytes, size_t* needed)
{
    if (!plan || !needed) return FMM_E_ARG;
    const fmm_params& prm = plan->prm;
    const size_t n = size_t(std::max<int64_t>(plan->last_n, 0));
    const size_t nbox = size_t(plan->shape.boxes);
    const void* src = nullptr;
    size_t sz = 0;
    switch (what) {
        case FMM_DUMP_KEYS: src = plan->buf.key; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_PERM: src = plan->buf.perm; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_LEAF_START:
            src = plan->buf.leaf_start;
            sz = size_t(plan->shape.leaf_entries) * sizeof(int32_t);
            break;
        case FMM_DUMP_ME: src = plan->buf.me; sz = nbox * prm.p * sizeof(cd); break;   // device rows: stride P
        case FMM_DUMP_LE: src = plan->buf.le; sz = nbox * prm.p * sizeof(cd); break;
        case FMM_DUMP_DOMAIN: src = &plan->buf.inst[0].dom; sz = sizeof(Domain); break;
        case FMM_DUMP_TKEYS: src = plan->buf.tkey; sz = size_t(plan->last_m) * sizeof(uint32_t); break;
        case FMM_DUMP_TPERM: src = plan->buf.tperm; sz = size_t(plan->last_m) * sizeof(uint32_t); break;
        case FMM_DUMP_TLEAF_START:
            src = plan->buf.tleaf_start;
            sz = plan->last_m > 0 ? size_t(plan->shape.leaf_entries) * sizeof(int32_t) : 0;
            break;
        case FMM_DUMP_ILIST:
            if (plan->shape.n_inst != 1) return FMM_E_UNSUPPORTED;
            sz = nbox * 27 * sizeof(int32_t);
            break;
        default: return FMM_E_ARG;
    }
    *needed = sz;
    if (!host_buf || bytes < sz) return FMM_E_CAPACITY;
    if (sz == 0) return FMM_OK;
    hipStream_t st = plan->last_stream;
    if (hipStreamSynchronize(st) != hipSuccess) return FMM_E_DEVICE;
    auto fetch = [&](void* dst, const void* from, size_t nbytes) {
        if (hipMemcpyAsync(dst, from, nbytes, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    if (what == FMM_DUMP_ILIST) {
        // inspection only: the lists are written in chunks into the sort's
        // ping-pong arrays (rewritten by every tree build) and copied out
        const int64_t per = int64_t(plan->dump_scratch_bytes / (27 * sizeof(int32_t)));
        int32_t* d = reinterpret_cast<int32_t*>(plan->dump_scratch);
        int32_t* h = static_cast<int32_t*>(host_buf);
        for (int64_t b0 = 0; b0 < int64_t(nbox); b0 += per) {
            const int64_t cnt = std::min<int64_t>(per, int64_t(nbox) - b0);
            if (launch_ilist(plan->shape.depth[0], b0, cnt, d, st) != hipSuccess) return FMM_E_DEVICE;
            if (!fetch(h + b0 * 27, d, size_t(cnt) * 27 * sizeof(int32_t))) return FMM_E_DEVICE;
        }
        return FMM_OK;
    }
    if (what == FMM_DUMP_ME || what == FMM_DUMP_LE) {
        // device rows hold P coefficients; hand out the first p of each.
        // Multipole rows hold abar_k = (-1)^(k+1) ahat_k / k!: undo that.
        const int P = plan->P, p = prm.p;
        std::vector<cd> tmp(nbox * size_t(P));
        if (!fetch(tmp.data(), src, tmp.size() * sizeof(cd))) return FMM_E_DEVICE;
        std::vector<double> unscale(p, 1.0);
        if (what == FMM_DUMP_ME) {
            long double f = 1.0L;
            for (int k = 0; k < p; ++k) {
                if (k > 0) f *= (long double)k;
                unscale[k] = double((k % 2) ? f : -f);
            }
        }
        cd* out = static_cast<cd*>(host_buf);
        for (size_t bx = 0; bx < nbox; ++bx)
            for (int k = 0; k < p; ++k)
                out[bx * p + k] = cd{tmp[bx * P + k].x * unscale[k], tmp[bx * P + k].y * unscale[k]};
        return FMM_OK;
    }
    return fetch(host_buf, src, sz) ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_destroy(fmm_plan_t plan)
{
    if (!plan) return FMM_OK;
    if (plan->have_events) {
        for (int r = 0; r < kTimingRing; ++r) harvest(plan, r);
        destroy_events(plan, kTimingRing);
    }
    drop_graph(plan);
    if (plan->cap_stream) hipStreamDestroy(plan->cap_stream);
    delete plan;
    return FMM_OK;
}

}  // extern "C"
