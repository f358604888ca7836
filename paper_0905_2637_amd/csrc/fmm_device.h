// fmm_device.h -- small device helpers shared by the kernels.
#pragma once

#include "fmm_internal.h"

namespace fmm {

// Spread the low 16 bits of v to the even bit positions.
__device__ __forceinline__ uint32_t spread_bits(uint32_t v)
{
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Inverse of spread_bits: gather the even bits of v.
__device__ __forceinline__ uint32_t compact_bits(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}

// z-order number of box (a, b): x bits in even positions, y bits in odd ones.
__device__ __forceinline__ uint32_t morton(uint32_t a, uint32_t b) { return spread_bits(a) | (spread_bits(b) << 1); }
__device__ __forceinline__ uint32_t morton_x(uint32_t k) { return compact_bits(k); }
__device__ __forceinline__ uint32_t morton_y(uint32_t k) { return compact_bits(k >> 1); }

// Offset number o (0 .. 35) of the interaction list of a box in child
// position (cx, cy) of its parent: the 6 x 6 children of the parent's 3 x 3
// neighbourhood, relative to the box; false for the 9 that touch the box.
__device__ __forceinline__ bool il_offset(int cx, int cy, int o, int& dx, int& dy)
{
    dx = (o % 6) - 2 - cx;
    dy = (o / 6) - 2 - cy;
    return !(dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1);
}

template <typename T> struct cplx { T x, y; };

template <typename T>
__device__ __forceinline__ void cmac(T& ax, T& ay, T bx, T by, T cx, T cy)
{   // a += b * c
    ax = fma(bx, cx, ax);
    ax = fma(-by, cy, ax);
    ay = fma(bx, cy, ay);
    ay = fma(by, cx, ay);
}

// The child-centre offset of child position c (bit 0: x, bit 1: y) in
// units of the parent width, (+-1 +- i) / 4: exact in binary.
__device__ __forceinline__ void child_delta(int c, double& dx, double& dy)
{
    dx = (c & 1) ? 0.25 : -0.25;
    dy = (c & 2) ? 0.25 : -0.25;
}

// Translation of a truncated series, in registers (repeated synthetic
// division, P (P - 1) / 2 steps; no operator matrix).
//
// Moments (multipole side) by d = 1: u_k <- sum_{m <= k} C(k, m) u_m, the
// coefficients of sum_j g_j (z_j - c + 1)^k from those of (z_j - c)^k, by
// additions only (a shift by any d is this between the scalings u_m d^-m
// and u_k d^k).
template <int P>
__device__ __forceinline__ void binomial_sums(cd* u)
{
#pragma unroll
    for (int i = 0; i < P - 1; ++i) {
#pragma unroll
        for (int l = P - 1; l > i; --l) {       // u_l += u_(l-1), the old u_(l-1)
            u[l].x += u[l - 1].x;
            u[l].y += u[l - 1].y;
        }
    }
}

// Taylor series (local side): b_k <- sum_{j >= k} C(j, k) d^(j-k) b_j, the
// coefficients of p(x + d) from those of p(x) = sum_j b_j x^j.
template <int P>
__device__ __forceinline__ void shift_taylor(cd* b, double dx, double dy)
{
#pragma unroll
    for (int i = 0; i < P - 1; ++i) {
#pragma unroll
        for (int j = P - 2; j >= i; --j) {      // b_j += d b_(j+1), the new b_(j+1)
            const cd a = b[j + 1];
            b[j].x = fma(dx, a.x, fma(-dy, a.y, b[j].x));
            b[j].y = fma(dx, a.y, fma(dy, a.x, b[j].y));
        }
    }
}

}  // namespace fmm
