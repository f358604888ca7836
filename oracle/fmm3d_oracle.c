/*
 * fmm3d_oracle.c -- plain FP64 CPU reference for the 3D form of the FMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite and the benchmark's CPU
 * checks load this library.  The GPU library never links, loads or calls it,
 * and the two share no source, header or table.
 *
 * The paper's method carries over to three dimensions unchanged in its tree
 * and sweeps (uniform octree, near field = the box and the 26 boxes touching
 * it, interaction list = same-level boxes whose parents touch the parent but
 * which do not touch the box itself: up to 189); what changes is the kernel
 * with its series expansions and translation operators (Section 8).  The
 * kernel here is the 3D Laplace kernel 1/r, with Cartesian Taylor expansions
 * of total degree <= p, written with plain multi-index definitions:
 *
 *   potential      phi(x)    = sum_j q_j / |x - y_j|           (pairs at r = 0 left out)
 *   gradient       grad phi(x) = sum_j -q_j (x - y_j) / |x - y_j|^3
 *   derivatives    D_m(R)    = d^m (1/|R|) / dR^m,  m = (m1, m2, m3)
 *   P2M            M_k(c)    = sum_j q_j (y_j - c)^k / k!
 *   multipole eval phi(x)   ~= sum_k (-1)^|k| M_k(c) D_k(x - c)
 *   M2M            M_k(c')   = sum_{m <= k} M_m(c) (c - c')^(k-m) / (k-m)!
 *   M2L            L_n(t)    = sum_k (-1)^|k| M_k(s) D_(k+n)(t - s) / n!
 *   local eval     phi(x)   ~= sum_n L_n(t) (x - t)^n
 *   L2L            L_n(t')   = sum_{m >= n} L_m(t) C(m, n) (t' - t)^(m-n),  C = prod binom(m_i, n_i)
 * with k! = k1! k2! k3!, |k| = k1 + k2 + k3 and all sums over |k|, |n| <= p.
 * The derivatives come from the recurrence satisfied by b_m = D_m / m!
 * (from differentiating |R|^2 (1/|R|)^2 = 1 and the harmonicity of 1/r):
 *   |m| |R|^2 b_m + (2|m| - 1) sum_i R_i b_(m-e_i) + (|m| - 1) sum_i b_(m-2e_i) = 0,
 * pinned by the tests against closed forms, finite differences and the
 * Laplace equation.
 *
 * Coefficient layout of the single-operator entry points: a dense cube
 * c[(a (p+1) + b) (p+1) + c3] for multi-index (a, b, c3) with a + b + c3 <= p,
 * the other entries unused (written as 0).  The whole FMM numbers box (a, b, c)
 * of level l as (c 2^l + b) 2^l + a after the level's offset (8^l - 1) / 7.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define P3MAX 12

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

static double binom(int m, int n)
{
    double b = 1.0;
    for (int i = 1; i <= n; ++i) b = b * (m - n + i) / i;
    return b;
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

static int cube(int a, int b, int c, int q) { return (a * (q + 1) + b) * (q + 1) + c; }

/* D[cube(a, b, c, q)] = d^(a,b,c) (1/|R|) for a + b + c <= q. */
void oracle3_deriv(int q, double rx, double ry, double rz, double* D)
{
    const int s = q + 1;
    double* bm = calloc((size_t)s * s * s, sizeof(double));
    memset(D, 0, sizeof(double) * s * s * s);
    const double r2 = rx * rx + ry * ry + rz * rz;
    bm[cube(0, 0, 0, q)] = 1.0 / sqrt(r2);
    for (int d = 1; d <= q; ++d)
        for (int a = 0; a <= d; ++a)
            for (int b = 0; a + b <= d; ++b) {
                const int c = d - a - b;
                double first = 0.0, second = 0.0;
                if (a >= 1) first += rx * bm[cube(a - 1, b, c, q)];
                if (b >= 1) first += ry * bm[cube(a, b - 1, c, q)];
                if (c >= 1) first += rz * bm[cube(a, b, c - 1, q)];
                if (a >= 2) second += bm[cube(a - 2, b, c, q)];
                if (b >= 2) second += bm[cube(a, b - 2, c, q)];
                if (c >= 2) second += bm[cube(a, b, c - 2, q)];
                bm[cube(a, b, c, q)] = -((2 * d - 1) * first + (d - 1) * second) / (d * r2);
            }
    for (int a = 0; a <= q; ++a)
        for (int b = 0; a + b <= q; ++b)
            for (int c = 0; a + b + c <= q; ++c)
                D[cube(a, b, c, q)] = bm[cube(a, b, c, q)] * fact(a) * fact(b) * fact(c);
    free(bm);
}

/* Plain sums at the n particles (or at nt of them, listed in t). */
void oracle3_direct(int64_t n, const double* x, const double* y, const double* z, const double* q,
                    int64_t nt, const int64_t* t, double* phi, double* gx, double* gy, double* gz)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t ii = 0; ii < nt; ++ii) {
        const int64_t i = t ? t[ii] : ii;
        double f = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            f += q[j] / r;
            const double c = q[j] / (r2 * r);
            ax -= c * dx;
            ay -= c * dy;
            az -= c * dz;
        }
        phi[ii] = f;
        gx[ii] = ax;
        gy[ii] = ay;
        gz[ii] = az;
    }
}

/* ---- single operators (dense-cube coefficients of degree <= p) ---------- */

void oracle3_p2m(int64_t n, const double* x, const double* y, const double* z, const double* q, double cx,
                 double cy, double cz, int p, double* M)
{
    const int s = p + 1;
    memset(M, 0, sizeof(double) * s * s * s);
    for (int64_t j = 0; j < n; ++j)
        for (int a = 0; a <= p; ++a)
            for (int b = 0; a + b <= p; ++b)
                for (int c = 0; a + b + c <= p; ++c)
                    M[cube(a, b, c, p)] += q[j] * ipow(x[j] - cx, a) * ipow(y[j] - cy, b) * ipow(z[j] - cz, c) /
                                           (fact(a) * fact(b) * fact(c));
}

/* phi at R = x - c from the multipole expansion about c */
double oracle3_me_eval(int p, const double* M, double rx, double ry, double rz)
{
    double* D = malloc(sizeof(double) * (p + 1) * (p + 1) * (p + 1));
    oracle3_deriv(p, rx, ry, rz, D);
    double f = 0.0;
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; ++c)
                f += (((a + b + c) & 1) ? -1.0 : 1.0) * M[cube(a, b, c, p)] * D[cube(a, b, c, p)];
    free(D);
    return f;
}

/* M about c' from M about c; (dx, dy, dz) = c' - c */
void oracle3_m2m(int p, const double* M, double dx, double dy, double dz, double* Mo)
{
    const int s = p + 1;
    memset(Mo, 0, sizeof(double) * s * s * s);
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; ++c) {
                double acc = 0.0;
                for (int i = 0; i <= a; ++i)
                    for (int j = 0; j <= b; ++j)
                        for (int k = 0; k <= c; ++k)
                            acc += M[cube(i, j, k, p)] * ipow(-dx, a - i) * ipow(-dy, b - j) * ipow(-dz, c - k) /
                                   (fact(a - i) * fact(b - j) * fact(c - k));
                Mo[cube(a, b, c, p)] = acc;
            }
}

/* L about t from M about s; (rx, ry, rz) = t - s */
void oracle3_m2l(int p, const double* M, double rx, double ry, double rz, double* L)
{
    const int s = p + 1, q = 2 * p;
    double* D = malloc(sizeof(double) * (q + 1) * (q + 1) * (q + 1));
    oracle3_deriv(q, rx, ry, rz, D);
    memset(L, 0, sizeof(double) * s * s * s);
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; ++c) {
                double acc = 0.0;
                for (int i = 0; i <= p; ++i)
                    for (int j = 0; i + j <= p; ++j)
                        for (int k = 0; i + j + k <= p; ++k)
                            acc += (((i + j + k) & 1) ? -1.0 : 1.0) * M[cube(i, j, k, p)] *
                                   D[cube(a + i, b + j, c + k, q)];
                L[cube(a, b, c, p)] = acc / (fact(a) * fact(b) * fact(c));
            }
    free(D);
}

/* L about t' from L about t; (dx, dy, dz) = t' - t */
void oracle3_l2l(int p, const double* L, double dx, double dy, double dz, double* Lo)
{
    const int s = p + 1;
    memset(Lo, 0, sizeof(double) * s * s * s);
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; ++c) {
                double acc = 0.0;
                for (int i = a; i <= p; ++i)
                    for (int j = b; i + j <= p; ++j)
                        for (int k = c; i + j + k <= p; ++k)
                            acc += L[cube(i, j, k, p)] * binom(i, a) * binom(j, b) * binom(k, c) *
                                   ipow(dx, i - a) * ipow(dy, j - b) * ipow(dz, k - c);
                Lo[cube(a, b, c, p)] = acc;
            }
}

/* phi and grad phi at e = x - t from the local expansion about t: out[4] */
void oracle3_l2p(int p, const double* L, double ex, double ey, double ez, double* out)
{
    double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int a = 0; a <= p; ++a)
        for (int b = 0; a + b <= p; ++b)
            for (int c = 0; a + b + c <= p; ++c) {
                const double l = L[cube(a, b, c, p)];
                f += l * ipow(ex, a) * ipow(ey, b) * ipow(ez, c);
                if (a > 0) fx += l * a * ipow(ex, a - 1) * ipow(ey, b) * ipow(ez, c);
                if (b > 0) fy += l * b * ipow(ex, a) * ipow(ey, b - 1) * ipow(ez, c);
                if (c > 0) fz += l * c * ipow(ex, a) * ipow(ey, b) * ipow(ez, c - 1);
            }
    out[0] = f;
    out[1] = fx;
    out[2] = fy;
    out[3] = fz;
}

/* ---- whole FMM ------------------------------------------------------------ */

static int64_t lvl_off(int l) { return (((int64_t)1 << (3 * l)) - 1) / 7; }

/* Leaf coordinates of each particle; -1 for a particle outside the cube
 * [x0, x0 + W)^3 or with a NaN coordinate.  Returns the number of those. */
int64_t oracle3_leaf_coords(int64_t n, const double* x, const double* y, const double* z, int L, double x0,
                            double y0, double z0, double W, int32_t* ia, int32_t* ib, int32_t* ic)
{
    const double side = ldexp(1.0, L);
    int64_t bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double u[3] = {(x[i] - x0) / W * side, (y[i] - y0) / W * side, (z[i] - z0) / W * side};
        int ok = 1, v[3];
        for (int d = 0; d < 3; ++d) {
            if (!(u[d] >= 0.0 && u[d] < side)) ok = 0;
            else v[d] = (int)floor(u[d]);
        }
        if (!ok) {
            ia[i] = ib[i] = ic[i] = -1;
            ++bad;
        } else {
            ia[i] = v[0];
            ib[i] = v[1];
            ic[i] = v[2];
        }
    }
    return bad;
}

/* Morton number of leaf (a, b, c): bit i of a, b, c goes to bit 3i, 3i+1, 3i+2. */
uint32_t oracle3_morton(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t k = 0;
    for (int i = 0; i < 10; ++i)
        k |= (((a >> i) & 1u) << (3 * i)) | (((b >> i) & 1u) << (3 * i + 1)) | (((c >> i) & 1u) << (3 * i + 2));
    return k;
}

/* One FMM evaluation at the particles.  Returns the number of particles
 * outside the cube (their outputs are 0 and they act on nothing). */
int64_t oracle3_fmm(int64_t n, const double* x, const double* y, const double* z, const double* q, int p, int L,
                    double x0, double y0, double z0, double W, double* phi, double* gx, double* gy, double* gz)
{
    const int s = p + 1, cs = s * s * s;
    const int side = 1 << L;
    const int64_t nleaf = (int64_t)side * side * side;
    int32_t* ia = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t* ib = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int32_t* ic = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    const int64_t bad = oracle3_leaf_coords(n, x, y, z, L, x0, y0, z0, W, ia, ib, ic);
    /* particles per leaf (row-major leaf index), in input order */
    int64_t* start = calloc(nleaf + 1, sizeof(int64_t));
    int64_t* list = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        if (ia[i] >= 0) ++start[((int64_t)ic[i] * side + ib[i]) * side + ia[i] + 1];
    for (int64_t b = 0; b < nleaf; ++b) start[b + 1] += start[b];
    int64_t* fill = malloc(sizeof(int64_t) * (nleaf + 1));
    memcpy(fill, start, sizeof(int64_t) * (nleaf + 1));
    for (int64_t i = 0; i < n; ++i)
        if (ia[i] >= 0) list[fill[((int64_t)ic[i] * side + ib[i]) * side + ia[i]]++] = i;
    free(fill);

    const int64_t nbox = lvl_off(L + 1);
    double* M = calloc((size_t)nbox * cs, sizeof(double));
    double* Lc = calloc((size_t)nbox * cs, sizeof(double));
    for (int64_t i = 0; i < n; ++i) phi[i] = gx[i] = gy[i] = gz[i] = 0.0;

    /* box centre at level l */
#define CEN(l, a) (((a) + 0.5) * (W / (double)(1 << (l))))
    if (L >= 2) {
        /* P2M at the leaves */
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t b = 0; b < nleaf; ++b) {
            const int a0 = (int)(b % side), b0 = (int)((b / side) % side), c0 = (int)(b / ((int64_t)side * side));
            double* m = M + (lvl_off(L) + b) * cs;
            for (int64_t e = start[b]; e < start[b + 1]; ++e) {
                double t[P3MAX + 1][P3MAX + 1][P3MAX + 1];
                const int64_t j = list[e];
                oracle3_p2m(1, x + j, y + j, z + j, q + j, x0 + CEN(L, a0), y0 + CEN(L, b0), z0 + CEN(L, c0), p,
                            &t[0][0][0]);
                for (int k = 0; k < cs; ++k) m[k] += (&t[0][0][0])[k];
            }
        }
        /* M2M up to level 2 */
        for (int l = L - 1; l >= 2; --l) {
            const int sd = 1 << l;
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < (int64_t)sd * sd * sd; ++b) {
                const int a0 = (int)(b % sd), b0 = (int)((b / sd) % sd), c0 = (int)(b / ((int64_t)sd * sd));
                double* m = M + (lvl_off(l) + b) * cs;
                double t[P3MAX + 1][P3MAX + 1][P3MAX + 1];
                for (int ch = 0; ch < 8; ++ch) {
                    const int ca = 2 * a0 + (ch & 1), cb = 2 * b0 + ((ch >> 1) & 1), cc = 2 * c0 + (ch >> 2);
                    const double* mc = M + (lvl_off(l + 1) + ((int64_t)cc * 2 * sd + cb) * 2 * sd + ca) * cs;
                    oracle3_m2m(p, mc, CEN(l, a0) - CEN(l + 1, ca), CEN(l, b0) - CEN(l + 1, cb),
                                CEN(l, c0) - CEN(l + 1, cc), &t[0][0][0]);
                    for (int k = 0; k < cs; ++k) m[k] += (&t[0][0][0])[k];
                }
            }
        }
        /* M2L over the interaction lists, levels 2..L */
        for (int l = 2; l <= L; ++l) {
            const int sd = 1 << l;
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t b = 0; b < (int64_t)sd * sd * sd; ++b) {
                const int a0 = (int)(b % sd), b0 = (int)((b / sd) % sd), c0 = (int)(b / ((int64_t)sd * sd));
                double* lo = Lc + (lvl_off(l) + b) * cs;
                double t[P3MAX + 1][P3MAX + 1][P3MAX + 1];
                /* candidates: the children of the parent's 27 neighbours */
                for (int sc = 2 * (c0 / 2) - 2; sc <= 2 * (c0 / 2) + 3; ++sc)
                    for (int sb = 2 * (b0 / 2) - 2; sb <= 2 * (b0 / 2) + 3; ++sb)
                        for (int sa = 2 * (a0 / 2) - 2; sa <= 2 * (a0 / 2) + 3; ++sa) {
                            if (sa < 0 || sb < 0 || sc < 0 || sa >= sd || sb >= sd || sc >= sd) continue;
                            const int parents_touch = abs(sa / 2 - a0 / 2) <= 1 && abs(sb / 2 - b0 / 2) <= 1 &&
                                                      abs(sc / 2 - c0 / 2) <= 1;
                            const int touch = abs(sa - a0) <= 1 && abs(sb - b0) <= 1 && abs(sc - c0) <= 1;
                            if (!parents_touch || touch) continue;
                            const double* ms = M + (lvl_off(l) + ((int64_t)sc * sd + sb) * sd + sa) * cs;
                            oracle3_m2l(p, ms, CEN(l, a0) - CEN(l, sa), CEN(l, b0) - CEN(l, sb),
                                        CEN(l, c0) - CEN(l, sc), &t[0][0][0]);
                            for (int k = 0; k < cs; ++k) lo[k] += (&t[0][0][0])[k];
                        }
            }
        }
        /* L2L down to the leaves */
        for (int l = 3; l <= L; ++l) {
            const int sd = 1 << l;
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < (int64_t)sd * sd * sd; ++b) {
                const int a0 = (int)(b % sd), b0 = (int)((b / sd) % sd), c0 = (int)(b / ((int64_t)sd * sd));
                const int pa = a0 / 2, pb = b0 / 2, pc = c0 / 2, ps = sd / 2;
                const double* lp = Lc + (lvl_off(l - 1) + ((int64_t)pc * ps + pb) * ps + pa) * cs;
                double t[P3MAX + 1][P3MAX + 1][P3MAX + 1];
                oracle3_l2l(p, lp, CEN(l, a0) - CEN(l - 1, pa), CEN(l, b0) - CEN(l - 1, pb),
                            CEN(l, c0) - CEN(l - 1, pc), &t[0][0][0]);
                double* lo = Lc + (lvl_off(l) + b) * cs;
                for (int k = 0; k < cs; ++k) lo[k] += (&t[0][0][0])[k];
            }
        }
    }
    /* L2P and the near field */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t b = 0; b < nleaf; ++b) {
        const int a0 = (int)(b % side), b0 = (int)((b / side) % side), c0 = (int)(b / ((int64_t)side * side));
        for (int64_t e = start[b]; e < start[b + 1]; ++e) {
            const int64_t i = list[e];
            double o[4] = {0.0, 0.0, 0.0, 0.0};
            if (L >= 2)
                oracle3_l2p(p, Lc + (lvl_off(L) + b) * cs, x[i] - (x0 + CEN(L, a0)), y[i] - (y0 + CEN(L, b0)),
                            z[i] - (z0 + CEN(L, c0)), o);
            for (int dc = -1; dc <= 1; ++dc)
                for (int db = -1; db <= 1; ++db)
                    for (int da = -1; da <= 1; ++da) {
                        const int na = a0 + da, nb = b0 + db, nc = c0 + dc;
                        if (na < 0 || nb < 0 || nc < 0 || na >= side || nb >= side || nc >= side) continue;
                        const int64_t nbx = ((int64_t)nc * side + nb) * side + na;
                        for (int64_t f = start[nbx]; f < start[nbx + 1]; ++f) {
                            const int64_t j = list[f];
                            const double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            if (r2 == 0.0) continue;
                            const double r = sqrt(r2);
                            o[0] += q[j] / r;
                            const double c = q[j] / (r2 * r);
                            o[1] -= c * dx;
                            o[2] -= c * dy;
                            o[3] -= c * dz;
                        }
                    }
            phi[i] = o[0];
            gx[i] = o[1];
            gy[i] = o[2];
            gz[i] = o[3];
        }
    }
#undef CEN
    free(M);
    free(Lc);
    free(start);
    free(list);
    free(ia);
    free(ib);
    free(ic);
    return bad;
}
