// fmm3d_api.cpp -- C ABI of the 3D form: parameter checks, workspace layout,
// the derivative table of the M2L and the launch sequence of one evaluation.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/fmm.h"
#include "fmm3d_internal.h"

using namespace fmm3;

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout3 {
    size_t hist, hist_scan, scan_part, ktmp, itmp, xt, yt, gt;
    size_t key, ks, perm, xs, ys, zs, qs, leaf_start, me, le, dtab, dcube, kcube, nbad;
    size_t total;
};

fmm_status validate3(const fmm3d_params* prm)
{
    if (!prm) return FMM_E_ARG;
    if (prm->n_max < 0 || prm->n_max > int64_t(0x7fffffff)) return FMM_E_ARG;
    if (prm->p < 0 || prm->depth < 0) return FMM_E_ARG;
    if (prm->p > kP3Max || prm->depth > kDepth3Max) return FMM_E_UNSUPPORTED;
    if (!std::isfinite(prm->x0) || !std::isfinite(prm->y0) || !std::isfinite(prm->z0)) return FMM_E_ARG;
    if (!(prm->width > 0.0) || !std::isfinite(prm->width)) return FMM_E_ARG;
    return FMM_OK;
}

Layout3 layout3(const fmm3d_params* prm)
{
    const size_t n = size_t(prm->n_max > 0 ? prm->n_max : 1);
    const size_t nblk = size_t(fmm::radix_blocks(int64_t(n)));
    const size_t nhist = size_t(256) * nblk;
    const size_t nscan = (nhist + fmm::kScanChunk - 1) / fmm::kScanChunk;
    const int L = prm->depth, T = tet3(prm->p + 1), T2 = tet3(2 * prm->p + 1);
    const size_t nbox = size_t(lvl_off3(L + 1));
    Layout3 ly{};
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    ly.hist = take(sizeof(int32_t) * nhist);
    ly.hist_scan = take(sizeof(int32_t) * (nhist + 1));
    ly.scan_part = take(sizeof(int32_t) * (nscan + 1));
    ly.ktmp = take(sizeof(uint32_t) * n);
    ly.itmp = take(sizeof(uint32_t) * n);
    ly.xt = take(sizeof(double) * n);
    ly.yt = take(sizeof(double) * n);
    ly.gt = take(sizeof(double) * n);
    ly.key = take(sizeof(uint32_t) * n);
    ly.ks = take(sizeof(uint32_t) * n);
    ly.perm = take(sizeof(uint32_t) * n);
    ly.xs = take(sizeof(double) * n);
    ly.ys = take(sizeof(double) * n);
    ly.zs = take(sizeof(double) * n);
    ly.qs = take(sizeof(double) * n);
    ly.leaf_start = take(sizeof(int32_t) * ((size_t(1) << (3 * L)) + 1));
    ly.me = take(sizeof(double) * nbox * size_t(T));
    ly.le = take(sizeof(double) * nbox * size_t(T));
    ly.dtab = take(sizeof(double) * size_t(kOffsets3) * size_t(T2));
    const size_t S = size_t(2 * prm->p + 1);
    const bool lanes = prm->p >= 1 && prm->p <= kLaneMaxP3;
    ly.dcube = take(lanes ? sizeof(double) * size_t(kOffsets3) * S * S * S : 0);
    ly.kcube = take(lanes ? sizeof(int32_t) * size_t(T) : 0);
    ly.nbad = take(sizeof(unsigned long long));
    ly.total = off;
    return ly;
}

// D_m(o) = d^m (1/|R|) at R = o for every offset o in [-3, 3]^3 outside the
// near block [-1, 1]^3 and |m| <= 2p, graded order.  b_m = D_m / m! are the
// Taylor coefficients of 1/|R + h| in h.  With r = |R| and
//   u(h) = (2 R.h + |h|^2) / r^2,   1/|R + h| = (1/r) (1 + u)^(-1/2)
//        = (1/r) sum_n C(-1/2, n) u^n,
// they follow from powers of u in truncated three-variable polynomials: u
// has no constant term, so u^n starts at degree n and the sum up to degree
// q = 2p is finite and exact.  The sum cancels heavily at high degree, so it
// runs in extended precision (long double: within 2e-16 of each degree's
// largest entry up to p = 6 and 6e-14 at p = 9, against 5e-11 at p = 9 in
// double).  (A
// binomial-series composition; the oracle takes the three-term recurrence
// of the same coefficients, so the two tables share no arithmetic.)
std::vector<double> derivative_table(int p)
{
    const int q = 2 * p, T2 = tet3(q + 1);
    std::vector<double> tab(size_t(kOffsets3) * size_t(T2), 0.0);
    std::vector<double> fact(q + 1, 1.0);
    for (int i = 1; i <= q; ++i) fact[i] = fact[i - 1] * i;
    // the six terms of u: h_i with coefficient 2 R_i / r^2, h_i^2 with 1 / r^2
    const int ue[6][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
    std::vector<long double> un(T2), nx(T2), bm(T2);
    for (int oz = -3; oz <= 3; ++oz)
        for (int oy = -3; oy <= 3; ++oy)
            for (int ox = -3; ox <= 3; ++ox) {
                if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
                const double R[3] = {double(ox), double(oy), double(oz)};
                const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
                const long double lr2 = r2;
                const long double uc[6] = {2.0L * R[0] / lr2, 2.0L * R[1] / lr2, 2.0L * R[2] / lr2, 1.0L / lr2,
                                           1.0L / lr2, 1.0L / lr2};
                std::fill(un.begin(), un.end(), 0.0L);
                std::fill(bm.begin(), bm.end(), 0.0L);
                un[0] = 1.0L;                                  // u^0
                long double binom = 1.0L;                      // C(-1/2, n)
                for (int n = 0; n <= q; ++n) {
                    for (int k = tet3(n); k < T2; ++k) bm[size_t(k)] += binom * un[size_t(k)];
                    if (n == q) break;
                    binom *= (-0.5L - n) / (long double)(n + 1);
                    // u^(n+1) = u^n u, truncated at degree q; u^n has degrees n .. q
                    std::fill(nx.begin(), nx.end(), 0.0L);
                    for (int d = n; d < q; ++d)
                        for (int s = 0; s <= d; ++s)
                            for (int c = 0; c <= s; ++c) {
                                const int a = d - s, b = s - c;
                                const long double v = un[size_t(pos3(a, b, c))];
                                if (v == 0.0L) continue;
                                for (int t = 0; t < 6; ++t) {
                                    const int e = t < 3 ? 1 : 2;
                                    if (d + e > q) continue;
                                    const int* x = ue[t];
                                    nx[size_t(pos3(a + x[0], b + x[1], c + x[2]))] += v * uc[t];
                                }
                            }
                    un.swap(nx);
                }
                const long double ir = 1.0L / sqrtl(lr2);
                double* row = tab.data() + size_t(off3_index(ox, oy, oz)) * size_t(T2);
                for (int d = 0; d <= q; ++d)
                    for (int s = 0; s <= d; ++s)
                        for (int c = 0; c <= s; ++c) {
                            const int a = d - s, b = s - c;
                            const int k = pos3(a, b, c);
                            row[k] = double(ir * bm[size_t(k)] * fact[a] * fact[b] * fact[c]);
                        }
            }
    return tab;
}

}  // namespace

struct fmm3d_plan_s {
    fmm3d_params prm;
    Bufs3 buf;
    Geo3 geo;
    std::vector<double> dtab_host;   // source of the table upload, kept until the plan ends
    std::vector<double> dcube_host;
    std::vector<int32_t> kcube_host;
    int64_t last_n = 0;
};

extern "C" {

fmm_status fmm3d_workspace_size(const fmm3d_params* prm, size_t* bytes)
{
    if (!bytes) return FMM_E_ARG;
    *bytes = 0;
    const fmm_status s = validate3(prm);
    if (s != FMM_OK) return s;
    *bytes = layout3(prm).total;
    return FMM_OK;
}

fmm_status fmm3d_plan(const fmm3d_params* prm, void* d_workspace, size_t bytes, void* stream, fmm3d_plan_t* out)
{
    if (!out || !d_workspace) return FMM_E_ARG;
    *out = nullptr;
    fmm_status s = validate3(prm);
    if (s != FMM_OK) return s;
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return FMM_E_ARG;
    const Layout3 ly = layout3(prm);
    if (bytes < ly.total) return FMM_E_CAPACITY;
    fmm3d_plan_s* pl = new (std::nothrow) fmm3d_plan_s;
    if (!pl) return FMM_E_NOMEM;
    pl->prm = *prm;
    char* base = static_cast<char*>(d_workspace);
    auto at = [&](size_t o) { return static_cast<void*>(base + o); };
    Bufs3& b = pl->buf;
    b.sort = fmm::Buffers{};
    b.sort.hist = static_cast<int32_t*>(at(ly.hist));
    b.sort.hist_scan = static_cast<int32_t*>(at(ly.hist_scan));
    b.sort.scan_part = static_cast<int32_t*>(at(ly.scan_part));
    b.sort.ktmp = static_cast<uint32_t*>(at(ly.ktmp));
    b.sort.itmp = static_cast<uint32_t*>(at(ly.itmp));
    b.sort.xt = static_cast<double*>(at(ly.xt));
    b.sort.yt = static_cast<double*>(at(ly.yt));
    b.sort.gt = static_cast<double*>(at(ly.gt));
    b.key = static_cast<uint32_t*>(at(ly.key));
    b.ks = static_cast<uint32_t*>(at(ly.ks));
    b.perm = static_cast<uint32_t*>(at(ly.perm));
    b.xs = static_cast<double*>(at(ly.xs));
    b.ys = static_cast<double*>(at(ly.ys));
    b.zs = static_cast<double*>(at(ly.zs));
    b.qs = static_cast<double*>(at(ly.qs));
    b.leaf_start = static_cast<int32_t*>(at(ly.leaf_start));
    b.me = static_cast<double*>(at(ly.me));
    b.le = static_cast<double*>(at(ly.le));
    b.dtab = static_cast<double*>(at(ly.dtab));
    b.dcube = static_cast<double*>(at(ly.dcube));
    b.kcube = static_cast<int32_t*>(at(ly.kcube));
    b.nbad = static_cast<unsigned long long*>(at(ly.nbad));
    Geo3& g = pl->geo;
    g.x0 = prm->x0;
    g.y0 = prm->y0;
    g.z0 = prm->z0;
    g.W = prm->width;
    g.L = prm->depth;
    g.p = prm->p;
    g.T = tet3(prm->p + 1);
    g.T2 = tet3(2 * prm->p + 1);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool lanes = prm->p >= 1 && prm->p <= kLaneMaxP3;
    try {
        pl->dtab_host = derivative_table(prm->p);
        if (lanes) {
            // the graded rows rearranged as dense (2p+1)^3 cubes (entries of degree > 2p stay 0)
            const int S = 2 * prm->p + 1, T2 = g.T2;
            pl->dcube_host.assign(size_t(kOffsets3) * size_t(S * S * S), 0.0);
            for (int o = 0; o < kOffsets3; ++o)
                for (int d = 0; d <= 2 * prm->p; ++d)
                    for (int s2 = 0; s2 <= d; ++s2)
                        for (int c = 0; c <= s2; ++c) {
                            const int a = d - s2, bb = s2 - c;
                            pl->dcube_host[size_t(o) * size_t(S * S * S) + size_t((a * S + bb) * S + c)] =
                                pl->dtab_host[size_t(o) * size_t(T2) + size_t(pos3(a, bb, c))];
                        }
            pl->kcube_host.assign(size_t(g.T), 0);
            for (int d = 0; d <= prm->p; ++d)
                for (int s2 = 0; s2 <= d; ++s2)
                    for (int c = 0; c <= s2; ++c) {
                        const int a = d - s2, bb = s2 - c;
                        pl->kcube_host[size_t(pos3(a, bb, c))] = (a * S + bb) * S + c;
                    }
        }
    } catch (...) {
        delete pl;
        return FMM_E_NOMEM;
    }
    if (lanes && (hipMemcpyAsync(b.dcube, pl->dcube_host.data(), pl->dcube_host.size() * sizeof(double),
                                 hipMemcpyHostToDevice, st) != hipSuccess ||
                  hipMemcpyAsync(b.kcube, pl->kcube_host.data(), pl->kcube_host.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st) != hipSuccess)) {
        delete pl;
        return FMM_E_DEVICE;
    }
    if (hipMemcpyAsync(b.dtab, pl->dtab_host.data(), pl->dtab_host.size() * sizeof(double), hipMemcpyHostToDevice,
                       st) != hipSuccess ||
        launch3_clear(b, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        delete pl;
        return FMM_E_DEVICE;
    }
    *out = pl;
    return FMM_OK;
}

fmm_status fmm3d_evaluate(fmm3d_plan_t plan, int64_t n, const double* d_x, const double* d_y, const double* d_z,
                          const double* d_q, double* d_phi, double* d_gx, double* d_gy, double* d_gz, void* stream)
{
    if (!plan) return FMM_E_ARG;
    if (n < 0) return FMM_E_ARG;
    if (n > plan->prm.n_max) return FMM_E_CAPACITY;
    if (n > 0 && (!d_x || !d_y || !d_z || !d_q || !d_phi || !d_gx || !d_gy || !d_gz)) return FMM_E_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    plan->last_n = n;
    const Bufs3& b = plan->buf;
    const Geo3& g = plan->geo;
    if (launch3_clear(b, st) != hipSuccess) return FMM_E_DEVICE;
    if (n == 0) return FMM_OK;
    const int ni = int(n);
    if (launch3_tree(b, g, ni, d_x, d_y, d_z, d_q, st) != hipSuccess) return FMM_E_DEVICE;
    if (g.L >= 2) {
        if (launch3_upward(b, g, st) != hipSuccess) return FMM_E_DEVICE;
        if (launch3_m2l(b, g, st) != hipSuccess) return FMM_E_DEVICE;
        if (launch3_l2l(b, g, st) != hipSuccess) return FMM_E_DEVICE;
    }
    if (launch3_eval(b, g, ni, d_phi, d_gx, d_gy, d_gz, st) != hipSuccess) return FMM_E_DEVICE;
    return FMM_OK;
}

fmm_status fmm3d_get_status(fmm3d_plan_t plan, void* stream, int64_t* n_outside)
{
    if (!plan || !n_outside) return FMM_E_ARG;
    *n_outside = 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned long long v = 0;
    if (hipMemcpyAsync(&v, plan->buf.nbad, sizeof v, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return FMM_E_DEVICE;
    *n_outside = int64_t(v);
    return v == 0 ? FMM_OK : FMM_E_DOMAIN;
}

fmm_status fmm3d_debug_dump(fmm3d_plan_t plan, int32_t what, void* host_buf, size_t bytes, size_t* needed)
{
    if (!plan || !needed) return FMM_E_ARG;
    const size_t n = size_t(plan->last_n > 0 ? plan->last_n : 0);
    const void* src = nullptr;
    size_t sz = 0;
    switch (what) {
        case FMM_DUMP_KEYS: src = plan->buf.key; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_PERM: src = plan->buf.perm; sz = n * sizeof(uint32_t); break;
        case FMM_DUMP_LEAF_START:
            src = plan->buf.leaf_start;
            sz = n > 0 ? ((size_t(1) << (3 * plan->geo.L)) + 1) * sizeof(int32_t) : 0;
            break;
        default: return FMM_E_ARG;
    }
    *needed = sz;
    if (!host_buf || bytes < sz) return FMM_E_CAPACITY;
    if (sz == 0) return FMM_OK;
    if (hipDeviceSynchronize() != hipSuccess) return FMM_E_DEVICE;
    return hipMemcpy(host_buf, src, sz, hipMemcpyDeviceToHost) == hipSuccess ? FMM_OK : FMM_E_DEVICE;
}

fmm_status fmm3d_destroy(fmm3d_plan_t plan)
{
    delete plan;
    return FMM_OK;
}

}  // extern "C"
