// fmm_api.cpp -- the C ABI of include/fmm.h: argument validation, workspace
// layout, plan construction and the stage sequence of one evaluation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_internal.h"

using namespace fmm;

namespace {

enum Stage { ST_TREE = 0, ST_UP, ST_M2L, ST_DOWN, ST_P2P, ST_COUNT };
const char* const kStageNames[ST_COUNT] = {"tree", "p2m_m2m", "m2l", "l2l", "p2p_l2p"};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

fmm_status validate(const fmm_params* prm)
{
    if (!prm) return FMM_E_ARG;
    if (prm->n_max < 0 || prm->n_max > int64_t(0x7fffffff)) return FMM_E_ARG;
    if (!(prm->sigma > 0.0) || !std::isfinite(prm->sigma)) return FMM_E_ARG;
    if (prm->p < 1 || prm->p > kMaxP) return FMM_E_ARG;
    if (prm->depth < 0 || prm->depth > kMaxDepth) return FMM_E_ARG;
    if (prm->precision != FMM_PREC_FP64 && prm->precision != FMM_PREC_MIXED) return FMM_E_ARG;
    if (prm->width > 0.0) {
        if (!std::isfinite(prm->width) || !std::isfinite(prm->x0) || !std::isfinite(prm->y0)) return FMM_E_ARG;
    }
    if (prm->precision == FMM_PREC_MIXED) {
        if (prm->fp32_fine_levels < 0 || prm->fp32_fine_levels > std::max(0, prm->depth - 1)) return FMM_E_ARG;
        if (prm->p > kMaxPMixed) return FMM_E_UNSUPPORTED;
    }
    return FMM_OK;
}

Layout make_layout(const fmm_params& prm)
{
    const int P = instantiated_terms(prm.p);
    const int L = prm.depth;
    const size_t n = size_t(std::max<int64_t>(prm.n_max, 1));
    const size_t nleaf = size_t(1) << (2 * L);
    const size_t nbox = size_t(level_offset(L + 1));
    const size_t nhist = size_t(256) * size_t(radix_blocks(int64_t(n)));
    const size_t nscan = (nhist + kScanChunk - 1) / kScanChunk;
    const bool mixed = prm.precision == FMM_PREC_MIXED;
    Layout ly{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
    ly.bad_blk = take(sizeof(int32_t) * size_t(radix_blocks(int64_t(n))));
    ly.dom = take(sizeof(Domain));
    ly.bbox = take(sizeof(double) * 4 * kBBoxBlocks);
    ly.leaf_start = take(sizeof(int32_t) * (nleaf + 1));
    ly.hist = take(sizeof(int32_t) * nhist);
    ly.hist_scan = take(sizeof(int32_t) * (nhist + 1));   // + the grand total
    ly.scan_part = take(sizeof(int32_t) * (nscan + 1));
    ly.key = take(sizeof(uint32_t) * n);
    ly.ksorted = take(sizeof(uint32_t) * n);
    ly.perm = take(sizeof(uint32_t) * n);
    ly.xs = take(sizeof(double) * n);
    ly.ys = take(sizeof(double) * n);
    ly.gs = take(sizeof(double) * n);
    ly.ktmp = take(sizeof(uint32_t) * n);
    ly.itmp = take(sizeof(uint32_t) * n);
    ly.xt = take(sizeof(double) * n);
    ly.yt = take(sizeof(double) * n);
    ly.gt = take(sizeof(double) * n);
    ly.pk = take(mixed ? sizeof(float4) * n : 0);
    // expansions: P >= p coefficients per box (the compiled size), zero-padded
    ly.me = take(sizeof(cd) * nbox * P);
    ly.le = take(sizeof(cd) * nbox * P);
    {
        const size_t nsplit = size_t(level_offset(m2l_split_level(L) + 1));
        ly.le_part[0] = take(sizeof(cd) * nsplit * P);
        ly.le_part[1] = take(sizeof(cd) * nsplit * P);
    }
    ly.t_m2m = take(sizeof(cd) * 4 * P * P);
    ly.t_l2l = take(sizeof(cd) * 4 * P * P);
    ly.t_h64 = take(sizeof(cd) * kHankelGrid * kHankelGrid * (2 * P - 1));
    ly.t_h32 = take(sizeof(cf) * kHankelGrid * kHankelGrid * (2 * P - 1));
    ly.t_sin = take(sizeof(double) * P);
    ly.t_sout = take(sizeof(double) * P);
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
    Buffers buf;
    int64_t last_n;
    bool timing;
    bool have_events;
    hipEvent_t ev[kTimingRing][ST_COUNT + 1];
    bool pending[kTimingRing];
    int64_t next_slot;
    int64_t n_timed;
    double total_ms[ST_COUNT];
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

}  // namespace

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
    const fmm_status s = validate(prm);
    if (s != FMM_OK) return s;
    *bytes = make_layout(*prm).total;
    return FMM_OK;
}

fmm_status fmm_plan(const fmm_params* prm, void* d_workspace, size_t bytes, void* stream, fmm_plan_t* out)
{
    if (!out || !d_workspace) return FMM_E_ARG;
    *out = nullptr;
    fmm_status s = validate(prm);
    if (s != FMM_OK) return s;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) != 0) return FMM_E_ARG;
    const Layout ly = make_layout(*prm);
    if (bytes < ly.total) return FMM_E_CAPACITY;

    fmm_plan_s* pl = new (std::nothrow) fmm_plan_s();
    if (!pl) return FMM_E_NOMEM;
    pl->prm = *prm;
    pl->P = instantiated_terms(prm->p);
    pl->auto_domain = !(prm->width > 0.0);
    pl->mixed = prm->precision == FMM_PREC_MIXED;
    pl->last_n = -1;
    char* base = static_cast<char*>(d_workspace);
    Buffers& b = pl->buf;
    b.bad_blk = reinterpret_cast<int32_t*>(base + ly.bad_blk);
    b.dom = reinterpret_cast<Domain*>(base + ly.dom);
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
    b.pk = pl->mixed ? reinterpret_cast<float4*>(base + ly.pk) : nullptr;
    b.me = reinterpret_cast<cd*>(base + ly.me);
    b.le = reinterpret_cast<cd*>(base + ly.le);
    b.le_part[0] = reinterpret_cast<cd*>(base + ly.le_part[0]);
    b.le_part[1] = reinterpret_cast<cd*>(base + ly.le_part[1]);
    b.ilist = nullptr;
    b.t_m2m = reinterpret_cast<cd*>(base + ly.t_m2m);
    b.t_l2l = reinterpret_cast<cd*>(base + ly.t_l2l);
    b.t_h64 = reinterpret_cast<cd*>(base + ly.t_h64);
    b.t_h32 = reinterpret_cast<cf*>(base + ly.t_h32);
    b.t_sin = reinterpret_cast<double*>(base + ly.t_sin);
    b.t_sout = reinterpret_cast<double*>(base + ly.t_sout);

    const int P = pl->P;
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
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables go out of scope
    if (e != hipSuccess) {
        delete pl;
        return FMM_E_DEVICE;
    }
    pl->have_events = true;
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
    if (!plan) return FMM_E_ARG;
    if (n < 0) return FMM_E_ARG;
    if (n > plan->prm.n_max) return FMM_E_CAPACITY;
    if (n > 0 && (!d_x || !d_y || !d_gamma || !d_u || !d_v)) return FMM_E_ARG;
    plan->last_n = n;
    if (n == 0) return FMM_OK;

    hipStream_t st = static_cast<hipStream_t>(stream);
    const fmm_params& prm = plan->prm;
    const Buffers& b = plan->buf;
    const int L = prm.depth, p = prm.p, P = plan->P;
    const bool timing = plan->timing;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    const int slot = int(plan->next_slot % kTimingRing);
    if (timing) {
        chk(harvest(plan, slot));
        plan->next_slot += 1;
    }
    auto mark = [&](int i) { if (timing) chk(hipEventRecord(plan->ev[slot][i], st)); };

    Domain dom{};
    if (!plan->auto_domain) {
        dom.x0 = prm.x0;
        dom.y0 = prm.y0;
        dom.W = prm.width;
        dom.s = std::ldexp(1.0, L) / prm.width;
    }
    const bool far = L >= 2;

    mark(ST_TREE);
    if (plan->auto_domain) chk(launch_domain(b, int(n), d_x, d_y, L, st));
    chk(launch_tree(b, int(n), L, d_x, d_y, d_gamma, !plan->auto_domain, dom, plan->mixed, st));
    mark(ST_UP);
    if (far) chk(launch_upward(b, P, p, L, st));
    mark(ST_M2L);
    const int sl = m2l_split_level(L);
    if (far) {
        // levels [2, f32) in FP64, [f32, L] in FP32; levels <= sl with the
        // interaction list split over three wavefronts
        const int fine = plan->mixed ? prm.fp32_fine_levels : 0;
        const int f32 = std::max(2, L - fine + 1);
        auto run = [&](int lo, int hi, bool fp32) {
            if (hi < lo) return;
            const int mid = std::min(hi, sl);
            if (lo <= mid) chk(launch_m2l(b, P, p, lo, mid, fp32, 3, st));
            if (std::max(lo, mid + 1) <= hi) chk(launch_m2l(b, P, p, std::max(lo, mid + 1), hi, fp32, 1, st));
        };
        run(2, f32 - 1, false);
        run(f32, L, true);
    }
    mark(ST_DOWN);
    if (far) chk(launch_downward(b, P, p, L, sl, st));
    mark(ST_P2P);
    chk(launch_p2p(b, P, p, L, far, plan->mixed, prm.sigma, d_u, d_v, st));
    mark(ST_COUNT);
    if (timing && e == hipSuccess) plan->pending[slot] = true;
    return e == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm_get_status(fmm_plan_t plan, void* stream, int64_t* n_bad)
{
    if (!plan || !n_bad) return FMM_E_ARG;
    *n_bad = 0;
    if (plan->last_n <= 0) return FMM_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t nblk = size_t(radix_blocks(plan->last_n));
    std::vector<int32_t> per(nblk);
    if (hipMemcpyAsync(per.data(), plan->buf.bad_blk, nblk * sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return FMM_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return FMM_E_DEVICE;
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

fmm_status fmm_debug_dump(fmm_plan_t plan, int32_t what, void* host_buf, size_t bytes, size_t* needed)
{
    if (!plan || !needed) return FMM_E_ARG;
    const fmm_params& prm = plan->prm;
    const int L = prm.depth;
    const size_t n = size_t(std::max<int64_t>(plan->last_n, 0));
    const size_t nleaf = size_t(1) << (2 * L);
    const size_t nbox = size_t(level_offset(L + 1));
    const void* src = nullptr;
    size_t sz = 0;
    switch (what) {
        case FMM_DUMP_KEYS: src = plan->buf.key; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_PERM: src = plan->buf.perm; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_LEAF_START: src = plan->buf.leaf_start; sz = (nleaf + 1) * sizeof(int32_t); break;
        case FMM_DUMP_ME: src = plan->buf.me; sz = nbox * prm.p * sizeof(cd); break;   // stored with stride P
        case FMM_DUMP_LE: src = plan->buf.le; sz = nbox * prm.p * sizeof(cd); break;
        case FMM_DUMP_DOMAIN: src = plan->buf.dom; sz = sizeof(Domain); break;
        case FMM_DUMP_ILIST: sz = nbox * 27 * sizeof(int32_t); break;
        default: return FMM_E_ARG;
    }
    *needed = sz;
    if (!host_buf || bytes < sz) return FMM_E_CAPACITY;
    if (sz == 0) return FMM_OK;
    if (hipDeviceSynchronize() != hipSuccess) return FMM_E_DEVICE;
    if (what == FMM_DUMP_ILIST) {
        // debug only: a temporary device buffer for the lists
        int32_t* d = nullptr;
        if (hipMalloc(&d, sz) != hipSuccess) return FMM_E_DEVICE;
        Buffers b = plan->buf;
        b.ilist = d;
        hipError_t e = launch_ilist(b, L, nullptr);
        if (e == hipSuccess) e = hipMemcpy(host_buf, d, sz, hipMemcpyDeviceToHost);
        hipFree(d);
        return e == hipSuccess ? FMM_OK : FMM_E_DEVICE;
    }
    if (what == FMM_DUMP_ME || what == FMM_DUMP_LE) {
        // device rows hold P coefficients; hand out the first p of each
        const int P = plan->P, p = prm.p;
        std::vector<cd> tmp(nbox * size_t(P));
        if (hipMemcpy(tmp.data(), src, tmp.size() * sizeof(cd), hipMemcpyDeviceToHost) != hipSuccess)
            return FMM_E_DEVICE;
        cd* out = static_cast<cd*>(host_buf);
        for (size_t bx = 0; bx < nbox; ++bx)
            for (int k = 0; k < p; ++k) out[bx * p + k] = tmp[bx * P + k];
        return FMM_OK;
    }
    if (hipMemcpy(host_buf, src, sz, hipMemcpyDeviceToHost) != hipSuccess) return FMM_E_DEVICE;
    return FMM_OK;
}

fmm_status fmm_destroy(fmm_plan_t plan)
{
    if (!plan) return FMM_OK;
    if (plan->have_events) {
        for (int r = 0; r < kTimingRing; ++r) harvest(plan, r);
        destroy_events(plan, kTimingRing);
    }
    delete plan;
    return FMM_OK;
}

}  // extern "C"
