/*
 * fmm_oracle.c -- plain FP64 CPU reference for the 2D vortex-particle FMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library never
 * links, loads or calls it, and the two share no source, header or table.
 *
 * What it computes, and the passage of Cruz, Knepley & Barba (PetFMM) each
 * part follows:
 *   - regularised Biot-Savart direct sum ............ Section 3, eqs. 8-9
 *   - split-kernel direct sum (what the FMM approximates: the near field
 *     uses the Gaussian-regularised kernel, the far field the singular
 *     kernel whose expansions are used) ............. Section 3, text after eq. 9
 *   - uniform quadtree, near field = the box and the boxes touching it,
 *     interaction list = same-level far boxes whose parents touch
 *     ............................................... Section 2.1, Fig. 1; Section 2.2
 *   - z-order (Morton) box numbering .................. Section 5.1
 *   - upward sweep (P2M, M2M), downward sweep (M2L over the interaction
 *     list, L2L), evaluation (L2P + near-field direct) .. Section 2.2, Fig. 2
 *   - Lennard-Jones forces and energy with a cutoff (a further kernel the
 *     paper names for molecular dynamics) ............ Section 8
 *   - Gauss transform, plain and fast (Greengard and Strain's Hermite /
 *     Taylor algorithm on the leaf boxes; a transform the paper names) .. Section 8
 * The paper leaves out the expansion mathematics and points to Greengard and
 * Rokhlin; the expansions below are the textbook complex-variable ones for the
 * Cauchy kernel 1/z, kept unscaled (coefficients about geometric box centres).
 *
 * Complex form used throughout: z = x + i y and
 *     phi(z_i) = sum_j gamma_j c_ij / (z_i - z_j),
 *     c_ij = 1 - exp(-|z_i - z_j|^2 / (2 sigma^2))   (regularised pair)
 *     c_ij = 1                                       (singular, far pair)
 * so that the velocity of eq. 9 is u = Im(phi) / (2 pi), v = Re(phi) / (2 pi).
 * A pair at zero distance contributes nothing (the kernel of eq. 8 tends to 0).
 *
 * sigma = 0 selects the singular kernel of eq. 7 (point vortices) for every
 * pair, near ones included: c_ij = 1, the sigma -> 0 limit of the Gaussian
 * core.  A pair at zero distance still contributes nothing (the singular
 * kernel has no value there; the sums leave such pairs out).
 *
 * Parity status: every function here is pinned by the CPU tests (closed
 * forms, invariants, operator identities, brute force); none is unpinned.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared -lm.
 * -ffp-contract=off keeps the quantisation (x - x0) * s as two correctly
 * rounded operations, which fixes the box of every particle exactly.
 */
#include <complex.h>
#include <pthread.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define TWO_PI 6.283185307179586476925286766559

/* ---------------------------------------------------------------------- */
/* Domain and quantisation (Section 2.1: uniform subdivision of a square). */
/* ---------------------------------------------------------------------- */

/* Bounding square of the points: x0 = min x, y0 = min y, W = the larger
 * extent (1 if the points span nothing).  NaNs are ignored here and counted
 * as out-of-domain by the quantiser. */
void oracle_bounding_square(int64_t n, const double* x, const double* y, double* dom)
{
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] == x[i]) { if (x[i] < xmin) xmin = x[i]; if (x[i] > xmax) xmax = x[i]; }
        if (y[i] == y[i]) { if (y[i] < ymin) ymin = y[i]; if (y[i] > ymax) ymax = y[i]; }
    }
    double w = xmax - xmin;
    if (ymax - ymin > w) w = ymax - ymin;
    if (!(w > 0.0) || !isfinite(w)) { w = 1.0; }
    if (!isfinite(xmin)) xmin = 0.0;
    if (!isfinite(ymin)) ymin = 0.0;
    dom[0] = xmin; dom[1] = ymin; dom[2] = w;
}

/* Box index along one axis at level L: t = (v - o) * s with s = 2^L / W, one
 * correctly rounded division done by the caller.  A point is inside when
 * 0 <= t <= 2^L; t == 2^L (the far edge) goes to the last box.  Points
 * outside (or NaN) are clamped and reported through *bad. */
static int64_t axis_box(double v, double o, double s, int64_t side, int* bad)
{
    double t = (v - o) * s;
    if (!(t >= 0.0 && t <= (double)side)) {
        *bad = 1;
        if (t > (double)side) return side - 1;
        return 0;                       /* below the domain, or NaN */
    }
    int64_t b = (int64_t)floor(t);
    if (b > side - 1) b = side - 1;
    return b;
}

/* Level-L box coordinates of every particle; returns the number of
 * particles outside the square [x0, x0+W]^2. */
int64_t oracle_quantize(int64_t n, const double* x, const double* y, int L,
                        double x0, double y0, double W, int32_t* ia, int32_t* ib)
{
    const int64_t side = (int64_t)1 << L;
    const double s = ldexp(1.0, L) / W;
    int64_t nbad = 0;
    for (int64_t i = 0; i < n; ++i) {
        int bad = 0;
        ia[i] = (int32_t)axis_box(x[i], x0, s, side, &bad);
        ib[i] = (int32_t)axis_box(y[i], y0, s, side, &bad);
        nbad += bad;
    }
    return nbad;
}

/* z-order number of box (a, b): bit k of a goes to bit 2k, bit k of b to
 * bit 2k+1 (Section 5.1 uses the z-order numbering of quadtree nodes). */
uint32_t oracle_morton(uint32_t a, uint32_t b)
{
    uint32_t key = 0;
    for (int k = 0; k < 16; ++k) {
        key |= ((a >> k) & 1u) << (2 * k);
        key |= ((b >> k) & 1u) << (2 * k + 1);
    }
    return key;
}

typedef struct { uint32_t key; uint32_t idx; } key_idx;

static int cmp_key_idx(const void* pa, const void* pb)
{
    const key_idx* a = (const key_idx*)pa;
    const key_idx* b = (const key_idx*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->idx != b->idx) return a->idx < b->idx ? -1 : 1;
    return 0;
}

/* Tree build: leaf key of every particle (input order), the permutation that
 * sorts particles by (key, input index), and leaf_start[4^L + 1] giving the
 * sorted range of every leaf in z-order.  Returns the out-of-domain count. */
int64_t oracle_tree(int64_t n, const double* x, const double* y, int L,
                    double x0, double y0, double W,
                    uint32_t* key, uint32_t* perm, int64_t* leaf_start)
{
    int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t nbad = oracle_quantize(n, x, y, L, x0, y0, W, ia, ib);
    key_idx* ki = (key_idx*)malloc(sizeof(key_idx) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        key[i] = oracle_morton((uint32_t)ia[i], (uint32_t)ib[i]);
        ki[i].key = key[i];
        ki[i].idx = (uint32_t)i;
    }
    qsort(ki, (size_t)n, sizeof(key_idx), cmp_key_idx);
    const int64_t nleaf = (int64_t)1 << (2 * L);
    memset(leaf_start, 0, sizeof(int64_t) * (size_t)(nleaf + 1));
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = ki[i].idx;
        leaf_start[ki[i].key + 1] += 1;
    }
    for (int64_t m = 0; m < nleaf; ++m) leaf_start[m + 1] += leaf_start[m];
    free(ki); free(ia); free(ib);
    return nbad;
}

/* ---------------------------------------------------------------------- */
/* Kernels and direct sums (Section 3, eqs. 7-9).                          */
/* ---------------------------------------------------------------------- */

/* Contribution gamma * c / (z_i - z_j) of source j at target i, added to
 * (*re, *im).  regularised != 0 uses the Gaussian core of eq. 8, otherwise the
 * singular kernel of eq. 7.  Zero distance contributes nothing. */
static void pair_phi(double xi, double yi, double xj, double yj, double gj,
                     double inv_2s2, int regularised, double* re, double* im)
{
    double dx = xi - xj, dy = yi - yj;
    double r2 = dx * dx + dy * dy;
    if (r2 == 0.0) return;
    double c = regularised ? -expm1(-r2 * inv_2s2) : 1.0;
    /* 1 / (dx + i dy) = (dx - i dy) / r2 */
    double q = gj * c / r2;
    *re += q * dx;
    *im -= q * dy;
}

/* 1/(2 sigma^2) of the Gaussian core; 0 (unused) for the singular kernel. */
static double core_factor(double sigma) { return sigma > 0.0 ? 1.0 / (2.0 * sigma * sigma) : 0.0; }

/* Regularised direct sum, eq. 9: u_i = sum_{j != i} gamma_j K_sigma(x_i - x_j)
 * (sigma = 0: the singular sum of eq. 7 over every pair j != i at nonzero
 * distance).  tgt == NULL evaluates every particle (nt must equal n). */
void oracle_direct(int64_t n, const double* x, const double* y, const double* g,
                   double sigma, int64_t nt, const int64_t* tgt, double* u, double* v)
{
    const double inv_2s2 = core_factor(sigma);
    const int reg = sigma > 0.0;   /* 0: singular kernel everywhere */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            pair_phi(x[i], y[i], x[j], y[j], g[j], inv_2s2, reg, &re, &im);
        }
        u[t] = im / TWO_PI;
        v[t] = re / TWO_PI;
    }
}

/* Split-kernel direct sum: the regularised kernel for pairs whose level-L
 * leaves touch (Chebyshev leaf distance <= 1), the singular kernel for every
 * other pair.  This is exactly the sum the FMM approximates, since the far
 * field is represented by expansions of the singular kernel (Section 3). */
void oracle_direct_split(int64_t n, const double* x, const double* y, const double* g,
                         double sigma, int L, double x0, double y0, double W,
                         int64_t nt, const int64_t* tgt, double* u, double* v)
{
    const double inv_2s2 = core_factor(sigma);
    const int reg = sigma > 0.0;   /* 0: singular kernel everywhere */
    int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    oracle_quantize(n, x, y, L, x0, y0, W, ia, ib);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t i = tgt ? tgt[t] : t;
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            int near = abs(ia[i] - ia[j]) <= 1 && abs(ib[i] - ib[j]) <= 1;
            pair_phi(x[i], y[i], x[j], y[j], g[j], inv_2s2, reg && near, &re, &im);
        }
        u[t] = im / TWO_PI;
        v[t] = re / TWO_PI;
    }
    free(ia); free(ib);
}

/* The regularised sum of eq. 1 at m target points (tx, ty) distinct from
 * the sources: no pair is excluded, and a target on top of a source gets
 * nothing from it (the regularised kernel vanishes at zero distance). */
void oracle_direct_at(int64_t n, const double* x, const double* y, const double* g, double sigma,
                      int64_t m, const double* tx, const double* ty, double* u, double* v)
{
    const double inv_2s2 = core_factor(sigma);
    const int reg = sigma > 0.0;   /* 0: singular kernel everywhere */
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j)
            pair_phi(tx[t], ty[t], x[j], y[j], g[j], inv_2s2, reg, &re, &im);
        u[t] = im / TWO_PI;
        v[t] = re / TWO_PI;
    }
}

/* The split-kernel sum at target points: the regularised kernel for sources
 * whose leaf touches the target's leaf, the singular kernel otherwise. */
void oracle_direct_split_at(int64_t n, const double* x, const double* y, const double* g, double sigma,
                            int L, double x0, double y0, double W, int64_t m, const double* tx,
                            const double* ty, double* u, double* v)
{
    const double inv_2s2 = core_factor(sigma);
    const int reg = sigma > 0.0;   /* 0: singular kernel everywhere */
    int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ta = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* tb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    oracle_quantize(n, x, y, L, x0, y0, W, ia, ib);
    oracle_quantize(m, tx, ty, L, x0, y0, W, ta, tb);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int near = abs(ta[t] - ia[j]) <= 1 && abs(tb[t] - ib[j]) <= 1;
            pair_phi(tx[t], ty[t], x[j], y[j], g[j], inv_2s2, reg && near, &re, &im);
        }
        u[t] = im / TWO_PI;
        v[t] = re / TWO_PI;
    }
    free(ia); free(ib); free(ta); free(tb);
}

/* ---------------------------------------------------------------------- */
/* Expansion operators: textbook complex expansions of 1/z, p terms        */
/* (k = 0 .. p-1), unscaled.  Section 2 defines the ME and LE; the          */
/* mathematics is Greengard and Rokhlin's.                                  */
/* ---------------------------------------------------------------------- */

/* Largest supported number of expansion terms. */
#define ORACLE_PMAX 64

/* Binomial coefficients C(n, k), n < 2 * ORACLE_PMAX, from Pascal's rule
 * (exact while below 2^53, i.e. for every n <= 53). */
static double BINOM[2 * ORACLE_PMAX][2 * ORACLE_PMAX];
static pthread_once_t binom_once = PTHREAD_ONCE_INIT;

static void binom_fill(void)
{
    for (int nn = 0; nn < 2 * ORACLE_PMAX; ++nn) {
        BINOM[nn][0] = 1.0;
        for (int k = 1; k <= nn; ++k)
            BINOM[nn][k] = BINOM[nn - 1][k - 1] + (k < nn ? BINOM[nn - 1][k] : 0.0);
    }
}

static double binom(int nn, int k)
{
    if (k < 0 || k > nn) return 0.0;
    return BINOM[nn][k];
}

/* Integer powers d^0 .. d^(q-1) by repeated multiplication. */
static void powers(cplx d, int q, cplx* out)
{
    cplx pw = 1.0;
    for (int i = 0; i < q; ++i) { out[i] = pw; pw *= d; }
}

/* Number of OpenMP threads the parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Must be called (single-threaded) before any operator below is used. */
int oracle_init(void)
{
    pthread_once(&binom_once, binom_fill);
    return ORACLE_PMAX;
}

/* P2M: a_k = sum_j gamma_j (z_j - c)^k, so that far from the cluster
 * phi(z) = sum_k a_k / (z - c)^(k+1). */
void oracle_p2m(int64_t n, const double* x, const double* y, const double* g,
                double cx, double cy, int p, double* a_out)
{
    cplx* a = (cplx*)a_out;
    const cplx c = cx + I * cy;
    for (int k = 0; k < p; ++k) a[k] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        cplx d = (x[j] + I * y[j]) - c;
        cplx pw = 1.0;
        for (int k = 0; k < p; ++k) { a[k] += g[j] * pw; pw *= d; }
    }
}

/* Evaluate a multipole expansion about c at z: sum_k a_k / (z - c)^(k+1). */
void oracle_me_eval(int p, const double* a_in, double cx, double cy,
                    double zx, double zy, double* phi)
{
    const cplx* a = (const cplx*)a_in;
    cplx w = 1.0 / ((zx + I * zy) - (cx + I * cy));
    cplx pw = w, s = 0.0;
    for (int k = 0; k < p; ++k) { s += a[k] * pw; pw *= w; }
    phi[0] = creal(s); phi[1] = cimag(s);
}

/* M2M: shift a child ME to its parent centre, d = c_child - c_parent:
 * a^P_k = sum_{m<=k} C(k,m) a^c_m d^(k-m).  Accumulates into aP. */
void oracle_m2m(int p, const double* ac_in, double dx, double dy, double* aP_out)
{
    const cplx* ac = (const cplx*)ac_in;
    cplx* aP = (cplx*)aP_out;
    cplx dp[ORACLE_PMAX];
    powers(dx + I * dy, p, dp);
    for (int k = 0; k < p; ++k) {
        cplx s = 0.0;
        for (int m = 0; m <= k; ++m) s += binom(k, m) * ac[m] * dp[k - m];
        aP[k] += s;
    }
}

/* M2L: turn a source ME into a local expansion about the target centre,
 * tau = c_source - c_target:
 * b_l = sum_k (-1)^(k+1) C(k+l, k) a_k tau^-(k+l+1).  Accumulates into b. */
void oracle_m2l(int p, const double* a_in, double tx, double ty, double* b_out)
{
    const cplx* a = (const cplx*)a_in;
    cplx* b = (cplx*)b_out;
    cplx ip[2 * ORACLE_PMAX + 1];                                   /* tau^-q */
    powers(1.0 / (tx + I * ty), 2 * p + 1, ip);
    for (int l = 0; l < p; ++l) {
        cplx s = 0.0;
        for (int k = 0; k < p; ++k) {
            double sign = (k % 2 == 0) ? -1.0 : 1.0;                 /* (-1)^(k+1) */
            s += sign * binom(k + l, k) * a[k] * ip[k + l + 1];
        }
        b[l] += s;
    }
}

/* L2L: re-centre a local expansion (a polynomial) from the parent centre to
 * the child centre, d = c_child - c_parent:
 * b^c_m = sum_{l>=m} C(l,m) b^P_l d^(l-m).  Accumulates into bc. */
void oracle_l2l(int p, const double* bP_in, double dx, double dy, double* bc_out)
{
    const cplx* bP = (const cplx*)bP_in;
    cplx* bc = (cplx*)bc_out;
    cplx dp[ORACLE_PMAX];
    powers(dx + I * dy, p, dp);
    for (int m = 0; m < p; ++m) {
        cplx s = 0.0;
        for (int l = m; l < p; ++l) s += binom(l, m) * bP[l] * dp[l - m];
        bc[m] += s;
    }
}

/* L2P: evaluate a local expansion about c at z: sum_l b_l (z - c)^l. */
void oracle_l2p(int p, const double* b_in, double cx, double cy,
                double zx, double zy, double* phi)
{
    const cplx* b = (const cplx*)b_in;
    cplx d = (zx + I * zy) - (cx + I * cy);
    cplx pw = 1.0, s = 0.0;
    for (int l = 0; l < p; ++l) { s += b[l] * pw; pw *= d; }
    phi[0] = creal(s); phi[1] = cimag(s);
}

/* ---------------------------------------------------------------------- */
/* Lists (Section 2.1, Fig. 1b; Section 2.2; Table 1: at most 27 IL boxes,  */
/* 8 neighbours).                                                           */
/* ---------------------------------------------------------------------- */

static int cheb(int a0, int b0, int a1, int b1)
{
    int da = abs(a0 - a1), db = abs(b0 - b1);
    return da > db ? da : db;
}

/* Near list of leaf (a, b) at level L: itself and every touching leaf. */
int oracle_near_list(int L, int a, int b, int32_t* sa, int32_t* sb)
{
    const int side = 1 << L;
    int cnt = 0;
    for (int j = b - 1; j <= b + 1; ++j)
        for (int i = a - 1; i <= a + 1; ++i) {
            if (i < 0 || j < 0 || i >= side || j >= side) continue;
            sa[cnt] = i; sb[cnt] = j; ++cnt;
        }
    return cnt;
}

/* Interaction list of box (a, b) at level l >= 2: the children of the
 * parent's neighbours (parent included) that do not touch (a, b). */
int oracle_interaction_list(int l, int a, int b, int32_t* sa, int32_t* sb)
{
    if (l < 2) return 0;
    const int pside = 1 << (l - 1);
    const int pa = a >> 1, pb = b >> 1;
    int cnt = 0;
    for (int qb = pb - 1; qb <= pb + 1; ++qb)
        for (int qa = pa - 1; qa <= pa + 1; ++qa) {
            if (qa < 0 || qb < 0 || qa >= pside || qb >= pside) continue;
            for (int cb = 0; cb < 2; ++cb)
                for (int ca = 0; ca < 2; ++ca) {
                    int sa_ = 2 * qa + ca, sb_ = 2 * qb + cb;
                    if (cheb(sa_, sb_, a, b) >= 2) { sa[cnt] = sa_; sb[cnt] = sb_; ++cnt; }
                }
        }
    return cnt;
}

/* ---------------------------------------------------------------------- */
/* The FMM (Section 2.2, Fig. 2).                                           */
/* ---------------------------------------------------------------------- */

static int64_t level_offset(int l) { return (((int64_t)1 << (2 * l)) - 1) / 3; }

static void box_centre(int l, int a, int b, double x0, double y0, double W,
                       double* cx, double* cy)
{
    double w = ldexp(W, -l);
    *cx = x0 + ((double)a + 0.5) * w;
    *cy = y0 + ((double)b + 0.5) * w;
}

/* One FMM evaluation.  Boxes are stored per level in row-major order
 * (index b * 2^l + a) starting at level_offset(l); coefficients are p complex
 * values per box.  tgt == NULL evaluates all particles (nt == n); otherwise
 * only the listed particles, with the downward sweep restricted to their
 * leaves and ancestors.  me_dump / le_dump, if not NULL, receive the
 * multipole and local coefficients of every box (Lambda * p complex values).
 * Returns the out-of-domain particle count. */
static int64_t fmm_core(int64_t n, const double* x, const double* y, const double* g,
                        double sigma, int p, int L, double x0, double y0, double W,
                        int64_t nt, const int64_t* tgt, const double* ptx, const double* pty,
                        double* u, double* v, double* me_dump, double* le_dump)
{
    oracle_init();
    const int64_t side = (int64_t)1 << L;
    const int64_t nleaf = side * side;
    const int64_t nbox = level_offset(L + 1);
    const double inv_2s2 = core_factor(sigma);
    const int reg = sigma > 0.0;   /* 0: singular kernel everywhere */

    int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t nbad = oracle_quantize(n, x, y, L, x0, y0, W, ia, ib);

    /* leaf membership (row-major leaf order, particles in input order) */
    int64_t* start = (int64_t*)calloc((size_t)(nleaf + 1), sizeof(int64_t));
    int64_t* member = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) start[(int64_t)ib[i] * side + ia[i] + 1] += 1;
    for (int64_t m = 0; m < nleaf; ++m) start[m + 1] += start[m];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)nleaf);
        memcpy(fill, start, sizeof(int64_t) * (size_t)nleaf);
        for (int64_t i = 0; i < n; ++i) member[fill[(int64_t)ib[i] * side + ia[i]]++] = i;
        free(fill);
    }

    cplx* me = (cplx*)calloc((size_t)(nbox * p), sizeof(cplx));
    cplx* le = (cplx*)calloc((size_t)(nbox * p), sizeof(cplx));

    /* target points (ptx != NULL): their leaves */
    int32_t* pa = NULL;
    int32_t* pb = NULL;
    if (ptx) {
        pa = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
        pb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
        nbad += oracle_quantize(nt, ptx, pty, L, x0, y0, W, pa, pb);
    }

    /* which boxes need a local expansion: all, or the targets' leaves and
     * their ancestors */
    char* need = (char*)calloc((size_t)nbox, 1);
    if (!tgt && !ptx) {
        memset(need, 1, (size_t)nbox);
    } else {
        for (int64_t t = 0; t < nt; ++t) {
            int a = ptx ? pa[t] : ia[tgt[t]], b = ptx ? pb[t] : ib[tgt[t]];
            for (int l = L; l >= 0; --l) {
                need[level_offset(l) + ((int64_t)b << l) + a] = 1;
                a >>= 1; b >>= 1;
            }
        }
    }

    /* Upward sweep: P2M at the leaves. */
    #pragma omp parallel
    {
        double* xs = (double*)malloc(sizeof(double) * 3 * 4096);
        size_t cap = 4096;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t m = 0; m < nleaf; ++m) {
            int64_t cnt = start[m + 1] - start[m];
            if (cnt == 0) continue;
            if ((size_t)cnt > cap) { cap = (size_t)cnt; xs = (double*)realloc(xs, sizeof(double) * 3 * cap); }
            for (int64_t q = 0; q < cnt; ++q) {
                int64_t i = member[start[m] + q];
                xs[q] = x[i]; xs[cap + q] = y[i]; xs[2 * cap + q] = g[i];
            }
            double cx, cy;
            box_centre(L, (int)(m % side), (int)(m / side), x0, y0, W, &cx, &cy);
            oracle_p2m(cnt, xs, xs + cap, xs + 2 * cap, cx, cy, p,
                       (double*)(me + (level_offset(L) + m) * p));
        }
        free(xs);
    }

    /* Upward sweep: M2M from level l+1 to level l, l = L-1 .. 2. */
    for (int l = L - 1; l >= 2; --l) {
        const int ls = 1 << l;
        #pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < (int64_t)ls * ls; ++m) {
            int a = (int)(m % ls), b = (int)(m / ls);
            double px, py;
            box_centre(l, a, b, x0, y0, W, &px, &py);
            cplx* aP = me + (level_offset(l) + m) * p;
            for (int cb = 0; cb < 2; ++cb)
                for (int ca = 0; ca < 2; ++ca) {
                    int c_a = 2 * a + ca, c_b = 2 * b + cb;
                    double cx, cy;
                    box_centre(l + 1, c_a, c_b, x0, y0, W, &cx, &cy);
                    const cplx* ac = me + (level_offset(l + 1) + ((int64_t)c_b << (l + 1)) + c_a) * p;
                    oracle_m2m(p, (const double*)ac, cx - px, cy - py, (double*)aP);
                }
        }
    }

    /* Downward sweep: for l = 2 .. L, L2L from the parent (nothing at
     * level 2: at level 1 every box touches every other) plus M2L from
     * every member of the interaction list. */
    for (int l = 2; l <= L; ++l) {
        const int ls = 1 << l;
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t m = 0; m < (int64_t)ls * ls; ++m) {
            if (!need[level_offset(l) + m]) continue;
            int a = (int)(m % ls), b = (int)(m / ls);
            double tx, ty;
            box_centre(l, a, b, x0, y0, W, &tx, &ty);
            cplx* bt = le + (level_offset(l) + m) * p;
            if (l > 2) {
                int pa = a >> 1, pb = b >> 1;
                double px, py;
                box_centre(l - 1, pa, pb, x0, y0, W, &px, &py);
                const cplx* bP = le + (level_offset(l - 1) + ((int64_t)pb << (l - 1)) + pa) * p;
                oracle_l2l(p, (const double*)bP, tx - px, ty - py, (double*)bt);
            }
            int32_t sa[27], sb[27];
            int cnt = oracle_interaction_list(l, a, b, sa, sb);
            for (int s = 0; s < cnt; ++s) {
                double sx, sy;
                box_centre(l, sa[s], sb[s], x0, y0, W, &sx, &sy);
                const cplx* as = me + (level_offset(l) + ((int64_t)sb[s] << l) + sa[s]) * p;
                oracle_m2l(p, (const double*)as, sx - tx, sy - ty, (double*)bt);
            }
        }
    }

    /* Evaluation: L2P plus the near field with the regularised kernel, at
     * particles (a particle skips itself) or at target points (which skip
     * nothing: a coincident source contributes zero). */
    const int64_t count = (tgt || ptx) ? nt : n;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = ptx ? -1 : (tgt ? tgt[t] : t);
        const int a = ptx ? pa[t] : ia[i], b = ptx ? pb[t] : ib[i];
        const double px = ptx ? ptx[t] : x[i], py = ptx ? pty[t] : y[i];
        double phi[2] = {0.0, 0.0};
        if (L >= 2) {
            double cx, cy;
            box_centre(L, a, b, x0, y0, W, &cx, &cy);
            oracle_l2p(p, (const double*)(le + (level_offset(L) + (int64_t)b * side + a) * p),
                       cx, cy, px, py, phi);
        }
        int32_t na[9], nb[9];
        int nn = oracle_near_list(L, a, b, na, nb);
        for (int s = 0; s < nn; ++s) {
            int64_t leaf = (int64_t)nb[s] * side + na[s];
            for (int64_t q = start[leaf]; q < start[leaf + 1]; ++q) {
                int64_t j = member[q];
                if (j == i) continue;
                pair_phi(px, py, x[j], y[j], g[j], inv_2s2, reg, &phi[0], &phi[1]);
            }
        }
        u[t] = phi[1] / TWO_PI;
        v[t] = phi[0] / TWO_PI;
    }

    if (me_dump) memcpy(me_dump, me, sizeof(cplx) * (size_t)(nbox * p));
    if (le_dump) memcpy(le_dump, le, sizeof(cplx) * (size_t)(nbox * p));
    free(need); free(le); free(me); free(member); free(start); free(ia); free(ib); free(pa); free(pb);
    return nbad;
}

int64_t oracle_fmm(int64_t n, const double* x, const double* y, const double* g,
                   double sigma, int p, int L, double x0, double y0, double W,
                   int64_t nt, const int64_t* tgt, double* u, double* v,
                   double* me_dump, double* le_dump)
{
    return fmm_core(n, x, y, g, sigma, p, L, x0, y0, W, nt, tgt, NULL, NULL, u, v, me_dump, le_dump);
}

/* The FMM of the particles evaluated at m target points (tx, ty) (eq. 1 with
 * targets distinct from the sources): each point takes L2P from its leaf and
 * the regularised near field from the sources of the touching leaves.
 * Returns the number of sources and targets outside the domain. */
int64_t oracle_fmm_at(int64_t n, const double* x, const double* y, const double* g,
                      double sigma, int p, int L, double x0, double y0, double W,
                      int64_t m, const double* tx, const double* ty, double* u, double* v)
{
    return fmm_core(n, x, y, g, sigma, p, L, x0, y0, W, m, NULL, tx, ty, u, v, NULL, NULL);
}

/* ---------------------------------------------------------------------- */
/* Lennard-Jones particles (Section 8 names the Lennard-Jones potential of   */
/* molecular dynamics as a further kernel): the pair potential              */
/*   V(r) = 4 eps ((s/r)^12 - (s/r)^6)  for 0 < r < rc, 0 otherwise         */
/* (truncated at the cutoff rc, not shifted), and the force on i,           */
/*   F_i = sum_{j != i} -V'(r_ij) (x_i - x_j) / r_ij,                         */
/*   -V'(r) / r = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2.                        */
/* A pair at zero distance contributes nothing.  Plain O(N^2) sums.          */
/* ---------------------------------------------------------------------- */
static int lj_pair(double dx, double dy, double eps, double sig, double rc, double* fr, double* v)
{
    const double r2 = dx * dx + dy * dy;
    if (r2 == 0.0 || r2 >= rc * rc) return 0;
    const double sr2 = sig * sig / r2;
    const double sr6 = sr2 * sr2 * sr2;
    *fr = 24.0 * eps * (2.0 * sr6 * sr6 - sr6) / r2;   /* -V'(r) / r */
    *v = 4.0 * eps * (sr6 * sr6 - sr6);
    return 1;
}

/* Force (fx, fy) on every particle, or on the particles tgt[0..nt) when tgt
 * != NULL (nt == n otherwise). */
void oracle_lj_forces(int64_t n, const double* x, const double* y, double eps, double sig, double rc,
                      int64_t nt, const int64_t* tgt, double* fx, double* fy)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = tgt ? tgt[t] : t;
        double ax = 0.0, ay = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double fr, v;
            if (j == i) continue;
            const double dx = x[i] - x[j], dy = y[i] - y[j];
            if (lj_pair(dx, dy, eps, sig, rc, &fr, &v)) {
                ax += fr * dx;
                ay += fr * dy;
            }
        }
        fx[t] = ax;
        fy[t] = ay;
    }
}

/* Total potential energy, each pair counted once. */
double oracle_lj_energy(int64_t n, const double* x, const double* y, double eps, double sig, double rc)
{
    double e = 0.0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : e)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double fr, v;
            if (lj_pair(x[i] - x[j], y[i] - y[j], eps, sig, rc, &fr, &v)) e += v;
        }
    }
    return e;
}

/* ---------------------------------------------------------------------- */
/* Gauss transform (Section 8 names the fast Gauss transform among the      */
/* transforms the library should take next):                                */
/*   G(y_i) = sum_j q_j exp(-|y_i - x_j|^2 / delta),  delta = 2 sigma^2,    */
/* at the particles themselves (the term j = i included).  The fast form is */
/* the published algorithm of Greengard and Strain (SIAM J. Sci. Stat.      */
/* Comput. 12, 1991) on the quadtree's leaf boxes:                          */
/*   - Hermite expansion of every box B about its centre c_B, with          */
/*     s = (x - c_B) / sqrt(delta):                                          */
/*       A_a = sum_{j in B} q_j s1^a1 s2^a2 / (a1! a2!),   a1, a2 < p;       */
/*     it represents B's field as sum_a A_a h_a1(t1) h_a2(t2),              */
/*     t = (y - c_B) / sqrt(delta), h_n(t) = (-1)^n d^n/dt^n exp(-t^2)      */
/*     (e^{-(t-s)^2} = sum_n s^n / n! h_n(t));                               */
/*   - Hermite to Taylor: for every box C and every box B whose Chebyshev    */
/*     box distance is at most nc, with tau = (c_C - c_B) / sqrt(delta),     */
/*       B_b += (-1)^(b1+b2) / (b1! b2!) sum_a A_a h_{a1+b1}(tau1)          */
/*              h_{a2+b2}(tau2),   b1, b2 < p;                               */
/*   - evaluation: G(y) = sum_b B_b u1^b1 u2^b2, u = (y - c_C) / sqrt(delta). */
/* Boxes farther apart than nc contribute less than exp(-(nc w)^2 / delta)  */
/* per unit of source strength and are left out.                           */
/* ---------------------------------------------------------------------- */

/* h_0 .. h_{m-1} at t by the three-term recurrence
 * h_{n+1}(t) = 2 t h_n(t) - 2 n h_{n-1}(t), h_0 = exp(-t^2), h_1 = 2 t h_0. */
void oracle_hermite(int m, double t, double* h)
{
    if (m <= 0) return;
    h[0] = exp(-t * t);
    if (m > 1) h[1] = 2.0 * t * h[0];
    for (int k = 1; k + 1 < m; ++k) h[k + 1] = 2.0 * t * h[k] - 2.0 * (double)k * h[k - 1];
}

/* The plain sum at the particles tgt[0..nt) (all of them if tgt == NULL). */
void oracle_gauss_direct(int64_t n, const double* x, const double* y, const double* q, double sigma,
                         int64_t nt, const int64_t* tgt, double* G)
{
    const double inv_delta = 1.0 / (2.0 * sigma * sigma);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t i = tgt ? tgt[t] : t;
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = x[i] - x[j], dy = y[i] - y[j];
            acc += q[j] * exp(-(dx * dx + dy * dy) * inv_delta);
        }
        G[t] = acc;
    }
}

/* The plain sum at m points (tx, ty) apart from the particles. */
void oracle_gauss_direct_at(int64_t n, const double* x, const double* y, const double* q, double sigma,
                            int64_t m, const double* tx, const double* ty, double* G)
{
    const double inv_delta = 1.0 / (2.0 * sigma * sigma);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        double acc = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double dx = tx[t] - x[j], dy = ty[t] - y[j];
            acc += q[j] * exp(-(dx * dx + dy * dy) * inv_delta);
        }
        G[t] = acc;
    }
}

/* The fast form on the 4^L leaf boxes of [x0, x0+W]^2, p Hermite terms per
 * axis (1 <= p <= 32), boxes within Chebyshev distance nc, evaluated at the
 * particles (tx == NULL) or at the m points (tx, ty), each in its own leaf
 * box.  Returns the number of particles and points outside the square. */
static int64_t fgt_core(int64_t n, const double* x, const double* y, const double* q, double sigma, int p, int L,
                        double x0, double y0, double W, int nc, int64_t m, const double* tx, const double* ty,
                        double* G)
{
    const int64_t side = (int64_t)1 << L;
    const int64_t nbox = side * side;
    const double sd = sqrt(2.0 * sigma * sigma);        /* sqrt(delta) */
    const int pp = p * p;
    int32_t* ia = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* ib = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    const int64_t nbad = oracle_quantize(n, x, y, L, x0, y0, W, ia, ib);
    double* A = (double*)calloc((size_t)(nbox * pp), sizeof(double));
    double* B = (double*)calloc((size_t)(nbox * pp), sizeof(double));
    double fact[64];
    fact[0] = 1.0;
    for (int k = 1; k < 64; ++k) fact[k] = fact[k - 1] * (double)k;

    /* Hermite expansions (row-major boxes, a = a1 * p + a2) */
    for (int64_t j = 0; j < n; ++j) {
        double cx, cy;
        box_centre(L, ia[j], ib[j], x0, y0, W, &cx, &cy);
        const double s1 = (x[j] - cx) / sd, s2 = (y[j] - cy) / sd;
        double* Ab = A + ((int64_t)ib[j] * side + ia[j]) * pp;
        for (int a1 = 0; a1 < p; ++a1)
            for (int a2 = 0; a2 < p; ++a2)
                Ab[a1 * p + a2] += q[j] * pow(s1, a1) * pow(s2, a2) / (fact[a1] * fact[a2]);
    }
    /* Hermite to Taylor */
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < nbox; ++c) {
        const int ca = (int)(c % side), cb = (int)(c / side);
        double h1[64], h2[64];
        for (int db = -nc; db <= nc; ++db) {
            for (int da = -nc; da <= nc; ++da) {
                const int sa = ca - da, sb = cb - db;          /* source box, tau = (da, db) w / sd */
                if (sa < 0 || sb < 0 || sa >= side || sb >= side) continue;
                const double* As = A + ((int64_t)sb * side + sa) * pp;
                const double w = ldexp(W, -L);
                oracle_hermite(2 * p - 1, (double)da * w / sd, h1);
                oracle_hermite(2 * p - 1, (double)db * w / sd, h2);
                for (int b1 = 0; b1 < p; ++b1)
                    for (int b2 = 0; b2 < p; ++b2) {
                        double acc = 0.0;
                        for (int a1 = 0; a1 < p; ++a1)
                            for (int a2 = 0; a2 < p; ++a2) acc += As[a1 * p + a2] * h1[a1 + b1] * h2[a2 + b2];
                        const double sgn = ((b1 + b2) & 1) ? -1.0 : 1.0;
                        B[c * pp + b1 * p + b2] += sgn * acc / (fact[b1] * fact[b2]);
                    }
            }
        }
    }
    /* evaluation */
    const int64_t ne = tx ? m : n;
    int32_t* ea = ia;
    int32_t* eb = ib;
    int64_t ebad = 0;
    if (tx) {
        ea = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
        eb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
        ebad = oracle_quantize(m, tx, ty, L, x0, y0, W, ea, eb);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ne; ++i) {
        double cx, cy;
        box_centre(L, ea[i], eb[i], x0, y0, W, &cx, &cy);
        const double px = tx ? tx[i] : x[i], py = tx ? ty[i] : y[i];
        const double u1 = (px - cx) / sd, u2 = (py - cy) / sd;
        const double* Bc = B + ((int64_t)eb[i] * side + ea[i]) * pp;
        double acc = 0.0;
        for (int b1 = 0; b1 < p; ++b1)
            for (int b2 = 0; b2 < p; ++b2) acc += Bc[b1 * p + b2] * pow(u1, b1) * pow(u2, b2);
        G[i] = acc;
    }
    if (tx) { free(ea); free(eb); }
    free(A); free(B); free(ia); free(ib);
    return nbad + ebad;
}

int64_t oracle_fgt(int64_t n, const double* x, const double* y, const double* q, double sigma, int p, int L,
                   double x0, double y0, double W, int nc, double* G)
{
    return fgt_core(n, x, y, q, sigma, p, L, x0, y0, W, nc, 0, NULL, NULL, G);
}

/* The fast form evaluated at m points (tx, ty) apart from the particles. */
int64_t oracle_fgt_at(int64_t n, const double* x, const double* y, const double* q, double sigma, int p, int L,
                      double x0, double y0, double W, int nc, int64_t m, const double* tx, const double* ty,
                      double* G)
{
    return fgt_core(n, x, y, q, sigma, p, L, x0, y0, W, nc, m, tx, ty, G);
}

/* ---------------------------------------------------------------------- */
/* Vortex-method time stepping (Section 3, eq. 6): in ideal 2D flow every  */
/* particle moves with the local velocity and keeps its circulation.  The  */
/* paper names no integrator; this is the explicit midpoint rule (second-  */
/* order Runge-Kutta):                                                     */
/*   k1 = u(x_n),  x_mid = x_n + dt/2 k1,  k2 = u(x_mid),  x_n+1 = x_n + dt k2 */
/* with the velocity from the FMM above (use_fmm != 0; the particles'      */
/* bounding square recomputed at every stage) or from the regularised      */
/* direct sum.  x, y are advanced in place.                                */
/* ---------------------------------------------------------------------- */
void oracle_advance_rk2(int64_t n, double* x, double* y, const double* g, double sigma, int p, int L,
                        int use_fmm, double dt, int steps)
{
    double* u = malloc(sizeof(double) * (size_t)n);
    double* v = malloc(sizeof(double) * (size_t)n);
    double* xm = malloc(sizeof(double) * (size_t)n);
    double* ym = malloc(sizeof(double) * (size_t)n);
    double dom[3];
    for (int s = 0; s < steps; ++s) {
        if (use_fmm) {
            oracle_bounding_square(n, x, y, dom);
            oracle_fmm(n, x, y, g, sigma, p, L, dom[0], dom[1], dom[2], n, NULL, u, v, NULL, NULL);
        } else {
            oracle_direct(n, x, y, g, sigma, n, NULL, u, v);
        }
        for (int64_t i = 0; i < n; ++i) {
            xm[i] = x[i] + 0.5 * dt * u[i];
            ym[i] = y[i] + 0.5 * dt * v[i];
        }
        if (use_fmm) {
            oracle_bounding_square(n, xm, ym, dom);
            oracle_fmm(n, xm, ym, g, sigma, p, L, dom[0], dom[1], dom[2], n, NULL, u, v, NULL, NULL);
        } else {
            oracle_direct(n, xm, ym, g, sigma, n, NULL, u, v);
        }
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + dt * u[i];
            y[i] = y[i] + dt * v[i];
        }
    }
    free(u); free(v); free(xm); free(ym);
}
