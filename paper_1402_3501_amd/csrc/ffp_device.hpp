// Device-side exact modular arithmetic shared by the gfx950 kernels.
//
// Integers are carried in FP64 registers whenever they stay below 2^53 in
// magnitude: sums and products of such integers are then exact, which is the
// delayed-reduction argument of Section 3.1 of the paper (k products of
// residues are summed exactly while k (p-1)^2 < 2^53).  A reduction is the
// floor division by p done with one multiplication by 1/p and a correction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffp {

// canonical residue of an integer-valued double |x| < 2^53
__device__ __forceinline__ double mod_canon(double x, double p, double pinv) {
    const double q = floor(x * pinv);
    double r = fma(-q, p, x);  // exact: the true value is a small integer
    // q is off by at most one: two selects (no branches) fix it
    r = r < 0.0 ? r + p : r;
    r = r >= p ? r - p : r;
    return r;
}

// residue of x in (-p, p) (balanced enough to bound later sums); |x| < 2^53
__device__ __forceinline__ double mod_near(double x, double p, double pinv) {
    double q = rint(x * pinv);
    return fma(-q, p, x);
}

// centred representative of a canonical residue v in [0, p)
__device__ __forceinline__ double centre(int32_t v, double p, int32_t half) {
    return v > half ? (double)v - p : (double)v;
}

// inverse of a in [1, p) modulo p (p < 2^31), extended Euclid; quotients by
// correctly rounded FP64 division, whose floor is exact for operands < 2^53
__device__ __forceinline__ int32_t inv_mod(int32_t a, int32_t p) {
    int32_t r0 = p, r1 = a, s0 = 0, s1 = 1;
    while (r1 != 0) {
        int32_t q = (int32_t)floor((double)r0 / (double)r1);
        int32_t t = r0 - q * r1;
        r0 = r1;
        r1 = t;
        t = s0 - q * s1;
        s0 = s1;
        s1 = t;
    }
    return s0 < 0 ? s0 + p : s0;
}

// same for p < 2^24: all remainders are exact in FP32, the quotient comes from
// the hardware reciprocal and is corrected by at most a few steps
__device__ __forceinline__ int32_t inv_mod_small(int32_t a, int32_t p) {
    int32_t r0 = p, r1 = a, s0 = 0, s1 = 1;
    while (r1 != 0) {
        int32_t q = (int32_t)((float)r0 * __builtin_amdgcn_rcpf((float)r1));
        int32_t t = r0 - q * r1;
        while (t < 0) { --q; t += r1; }
        while (t >= r1) { ++q; t -= r1; }
        r0 = r1;
        r1 = t;
        t = s0 - q * s1;
        s0 = s1;
        s1 = t;
    }
    return s0 < 0 ? s0 + p : s0;
}

// inverse for a wave-uniform operand, on the scalar unit: quotients by
// repeated subtraction (most Euclid quotients are 1..3), the hardware
// reciprocal only for the rare large ones
__device__ __forceinline__ int32_t inv_mod_uniform(int32_t a, int32_t p) {
    int32_t r0 = p, r1 = a, s0 = 0, s1 = 1;
    while (r1 != 0) {
        int32_t q, t;
        if (r0 >= (r1 << 3)) {
            q = (int32_t)((float)r0 * __builtin_amdgcn_rcpf((float)r1));
            t = r0 - q * r1;
            while (t < 0) { --q; t += r1; }
            while (t >= r1) { ++q; t -= r1; }
        } else {
            q = 0;
            t = r0;
            while (t >= r1) { t -= r1; ++q; }
        }
        r0 = r1;
        r1 = t;
        t = s0 - q * s1;
        s0 = s1;
        s1 = t;
    }
    return s0 < 0 ? s0 + p : s0;
}

// Tile order (one-dimensional grid of ntx x nty tiles): workgroup b runs on
// XCD b % 8 (the dispatcher deals workgroups round robin over the eight
// XCDs, each with its own L2), so when nty is a multiple of 8 each XCD gets
// a band of nty / 8 tile rows, walked four tile rows at a time: the tiles an
// XCD runs together share A row panels and B column panels in its L2.
__device__ __forceinline__ void xcd_tile(int b, int ntx, int nty, int &ty, int &tx) {
    if (nty % 8 != 0) {
        ty = b / ntx;
        tx = b % ntx;
        return;
    }
    constexpr int GM = 4;
    const int xcd = b & 7, loc = b >> 3, band = nty / 8;
    const int g = loc / (GM * ntx), in = loc % (GM * ntx);
    const int rows = band - g * GM < GM ? band - g * GM : GM;
    ty = xcd * band + g * GM + in % rows;
    tx = in / rows;
}

}  // namespace ffp
