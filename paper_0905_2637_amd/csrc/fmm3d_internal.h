// fmm3d_internal.h -- device buffers, geometry and launchers of the 3D form
// (fmm3d.hip, fmm3d_api.cpp).
//
// Coefficients of total degree <= p are stored in graded order: degree d,
// then s = b + c ascending, then c ascending, so multi-index (a, b, c) sits
// at tet(a + b + c) + tri(b + c) + c with tet(d) = d (d+1) (d+2) / 6 (the
// number of multi-indices of degree < d) and tri(s) = s (s+1) / 2.  With this
// order the multi-indices k + n for fixed n, fixed degree of k and fixed
// b + c of k are contiguous in c, which the M2L loop uses.
#pragma once

#include "fmm_internal.h"

namespace fmm {
// Stable LSD radix sort of n precomputed 32-bit keys (key_bits of them
// significant) carrying (input index, x, y, g); final arrays in (ks, perm,
// xs, ys, gs).  Uses the radix temporaries of b.  n >= 1.
hipError_t launch_sort_keys(const Buffers& b, int n, const uint32_t* key, const double* x, const double* y,
                            const double* g, uint32_t* ks, uint32_t* perm, double* xs, double* ys, double* gs,
                            int key_bits, hipStream_t st);
}  // namespace fmm

namespace fmm3 {

constexpr int kP3Max = 9;          // expansion degree
constexpr int kT3Max = 220;        // terms of degree <= 9
constexpr int kT3Max2 = 1330;      // terms of degree <= 18 (derivatives for the M2L)
constexpr int kDepth3Max = 7;      // 21 key bits plus the outside flag
constexpr int kOffsets3 = 343;     // offsets in [-3, 3]^3
constexpr int kLaneMaxP3 = 9;      // degrees whose M2L takes one lane per target box (1 .. this);
                                   // the derivative cubes are allocated and the lane kernel
                                   // dispatched for exactly these

__host__ __device__ constexpr int tet3(int d) { return d * (d + 1) * (d + 2) / 6; }
__host__ __device__ constexpr int tri3(int s) { return s * (s + 1) / 2; }
__host__ __device__ constexpr int pos3(int a, int b, int c) { return tet3(a + b + c) + tri3(b + c) + c; }
__host__ __device__ constexpr int64_t lvl_off3(int l) { return ((int64_t(1) << (3 * l)) - 1) / 7; }
__host__ __device__ constexpr int off3_index(int ox, int oy, int oz) { return ((oz + 3) * 7 + (oy + 3)) * 7 + (ox + 3); }

// Cube [x0, x0 + W)^3, depth L, degree p with T = tet3(p + 1) terms and
// T2 = tet3(2 p + 1) derivative terms.
struct Geo3 {
    double x0, y0, z0, W;
    int L, p, T, T2;
};

struct Bufs3 {
    fmm::Buffers sort;          // radix temporaries only (hist, hist_scan, scan_part, ktmp, itmp, xt, yt, gt)
    uint32_t* key;              // [n_max] leaf key per input particle (2^(3L) outside the cube)
    uint32_t* ks;               // [n_max] sorted keys
    uint32_t* perm;             // [n_max] sorted position -> input index
    double *xs, *ys, *zs, *qs;  // [n_max] sorted particles
    int32_t* leaf_start;        // [8^L + 1] sorted range of every leaf; the last entry counts the inside ones
    double* me;                 // [boxes of levels 0..L][T] scaled moments
    double* le;                 // [boxes of levels 0..L][T] scaled local coefficients
    double* dtab;               // [343][T2] derivatives of 1/r at the integer offsets, graded order
    double* dcube;              // p <= kLaneMaxP3: [343][(2p+1)^3] the same derivatives as dense cubes
    int32_t* kcube;             // p <= kLaneMaxP3: [T] cube index of each graded multi-index
    unsigned long long* nbad;   // particles outside the cube or NaN
};

hipError_t launch3_tree(const Bufs3& b, const Geo3& g, int n, const double* x, const double* y, const double* z,
                        const double* q, hipStream_t st);
hipError_t launch3_upward(const Bufs3& b, const Geo3& g, hipStream_t st);
hipError_t launch3_m2l(const Bufs3& b, const Geo3& g, hipStream_t st);
hipError_t launch3_l2l(const Bufs3& b, const Geo3& g, hipStream_t st);
hipError_t launch3_eval(const Bufs3& b, const Geo3& g, int n, double* phi, double* gx, double* gy, double* gz,
                        hipStream_t st);
hipError_t launch3_clear(const Bufs3& b, hipStream_t st);

}  // namespace fmm3
