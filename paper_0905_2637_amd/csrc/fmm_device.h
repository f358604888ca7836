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

}  // namespace fmm
