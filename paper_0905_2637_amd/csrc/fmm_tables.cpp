// fmm_tables.cpp -- host construction of the level-independent translation
// operators of the scaled 1/z expansions (built once per plan, FP64, with the
// powers and factorials accumulated in long double before rounding).
//
// Multipole coefficients are stored as abar_k = s_k ahat_k with
// s_k = (-1)^(k+1) / k!, the input scaling of the factored M2L, so that M2L
// reads them as they are.
//   M2M  (child position c, delta = (+-1 +- i)/4, see fmm_upward.hip) on
//        ahat: M[k][j] = C(k,j) 2^-j delta^(k-j), j <= k < p; on abar the same
//        map is S M S^-1:
//        M'[c][k][j] = (-1)^(k-j) 2^-j delta^(k-j) / (k-j)!
//   L2L  Lt[c][k][j] = C(j,k) delta^(j-k) 2^-(k+1),       p > k, j >= k
//        (rows k >= p of both are zero, so zero-padded terms stay zero)
//   M2L  Hankel data h_n(tau) = n! tau^-(n+1) for the integer offsets
//        tau = dx + i dy, |dx|, |dy| <= 3 (7 x 7 grid, the 9 touching offsets
//        unused), n = 0 .. 2p-2; zero for n > 2p-2 so that zero-padded terms
//        never meet an overflowed FP32 entry.
//        sin[k] = s_k = (-1)^(k+1) / k!,  sout[l] = 1 / l!   (see fmm_downward.hip)
#include <complex>
#include <vector>

#include "fmm_internal.h"

namespace fmm {

namespace {
using cld = std::complex<long double>;

long double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0L;
    long double c = 1.0L;
    for (int i = 1; i <= k; ++i) c = c * (long double)(n - k + i) / (long double)i;
    return c;
}

cld child_delta(int c)
{
    return cld((c & 1) ? 0.25L : -0.25L, (c & 2) ? 0.25L : -0.25L);
}

cd to_cd(cld z) { return cd{double(z.real()), double(z.imag())}; }
}  // namespace

void build_tables(int P, int p, cd* m2m, cd* l2l, cd* h64, cf* h32, double* sin_, double* sout_)
{
    for (int c = 0; c < 4; ++c) {
        const cld dl = child_delta(c);
        std::vector<cld> pw(P);
        pw[0] = 1.0L;
        for (int i = 1; i < P; ++i) pw[i] = pw[i - 1] * dl;
        for (int k = 0; k < P; ++k)
            for (int j = 0; j < P; ++j) {
                cld mv = 0.0L, lv = 0.0L;
                // rows k >= p stay zero: the padded terms never fill up
                if (k < p && j <= k) {
                    long double f = 1.0L;                       // (k - j)!
                    for (int i = 2; i <= k - j; ++i) f *= (long double)i;
                    const long double sg = ((k - j) % 2) ? -1.0L : 1.0L;
                    mv = sg * std::pow(0.5L, (long double)j) * pw[k - j] / f;
                }
                if (k < p && j >= k) lv = binom(j, k) * pw[j - k] * std::pow(0.5L, (long double)(k + 1));
                m2m[(c * P + k) * P + j] = to_cd(mv);
                l2l[(c * P + k) * P + j] = to_cd(lv);
            }
    }
    const int nh = 2 * P - 1;
    for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            const int slot = (dy + 3) * kHankelGrid + (dx + 3);
            const bool used = !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1);
            const cld inv = used ? 1.0L / cld((long double)dx, (long double)dy) : cld(0.0L, 0.0L);
            cld t = inv;                 // tau^-(n+1)
            long double fact = 1.0L;     // n!
            for (int n = 0; n < nh; ++n) {
                cld h = (used && n <= 2 * p - 2) ? fact * t : cld(0.0L, 0.0L);
                h64[slot * nh + n] = to_cd(h);
                h32[slot * nh + n] = cf{float(h.real()), float(h.imag())};
                t *= inv;
                fact *= (long double)(n + 1);
            }
        }
    long double f = 1.0L;
    for (int k = 0; k < P; ++k) {
        if (k > 0) f *= (long double)k;
        sin_[k] = k < p ? double(((k % 2) ? 1.0L : -1.0L) / f) : 0.0;
        sout_[k] = k < p ? double(1.0L / f) : 0.0;
    }
}

}  // namespace fmm
