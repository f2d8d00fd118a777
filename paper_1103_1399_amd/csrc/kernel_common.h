// kernel_common.h -- device helpers shared by the pass kernels
// (pass_kernels.hip) and the other kernels (kernels.hip): complex types, the
// LDS swizzle, the per-qubit rotation in shear form, and the per-step
// schedule coefficients evaluated on the device.  Internal to libqaa.
//
// Arithmetic conventions (see include/qaa.h for the physics):
//  - A step's driver factor exp(-i theta H_B) is applied qubit by qubit as
//    [[c, i s], [i s, c]] with c = cos(theta/2), s = sin(theta/2); its global
//    phase exp(-i n theta/2) is folded into the next diagonal phase.
//  - Each 2x2 block is two real plane rotations by theta/2, applied in place
//    as three shears with t = tan(theta/4) and s (three FMAs per component
//    pair; the sheared product stays area-preserving under FP32 rounding of
//    t and s, so no systematic norm drift comes from the coefficients).
//  - Diagonal phases exp(-i a E) come from a lookup table over E evaluated
//    in FP64 and rounded once.
#pragma once

#include "qaa_internal.h"

#include <cmath>
#include <cstdint>

namespace qaa {
namespace {

template <typename F> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

// XOR swizzle of an LDS element index.  It is linear over XOR
// (swz(a ^ b) == swz(a) ^ swz(b)), so a thread part and a register part of
// an index can be swizzled separately.  It spreads indices that differ only
// in high bits over distinct LDS banks (64 banks x 4 B).
template <typename F>
__device__ __forceinline__ uint32_t swz(uint32_t l)
{
    if constexpr (sizeof(F) == 4)
        return l ^ (((l >> 5) ^ (l >> 10)) & 31u);
    else
        return l ^ (((l >> 4) ^ (l >> 8) ^ (l >> 12)) & 15u);
}

template <typename F2, typename F>
__device__ __forceinline__ F2 cmul(F2 a, F2 b)
{
    F2 r;
    r.x = fma(a.x, b.x, -(a.y * b.y));
    r.y = fma(a.x, b.y, a.y * b.x);
    return r;
}

// Coefficients of one rotation angle theta: t = tan(theta/4),
// s = sin(theta/2).
template <typename F>
struct Rot {
    F t, s;
};

// Rotate register bit b of every pair in v: (x0, x1) <- (c x0 + i s x1,
// c x1 + i s x0), c = cos(theta/2), s = sin(theta/2).  In real components
// this is the plane rotation by theta/2 of (Re x0, Im x1) and of
// (Re x1, Im x0).  Each is applied in place as three shears,
// u -= t w; w += s u; u -= t w (t = tan(theta/4)): three FMAs per pair of
// components, no temporaries, and with FP32-rounded t and s the product
// stays area-preserving, so rounding adds no systematic norm drift.
template <int RB, typename F2, typename F>
__device__ __forceinline__ void rotate_bit(F2 (&v)[1 << RB], int b, const Rot<F> &k)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << b)) continue;
        const int m = j | (1 << b);
        F &u0 = v[j].x, &w0 = v[m].y;     // (Re x0, Im x1)
        F &u1 = v[m].x, &w1 = v[j].y;     // (Re x1, Im x0)
        u0 = fma(-k.t, w0, u0);
        u1 = fma(-k.t, w1, u1);
        w0 = fma(k.s, u0, w0);
        w1 = fma(k.s, u1, w1);
        u0 = fma(-k.t, w0, u0);
        u1 = fma(-k.t, w1, u1);
    }
}

// Rotate every register bit in mask (uniform over the workgroup).
template <int RB, typename F2, typename F>
__device__ __forceinline__ void rotate_mask(F2 (&v)[1 << RB], uint32_t mask, const Rot<F> &k)
{
#pragma unroll
    for (int b = 0; b < RB; ++b)
        if ((mask >> b) & 1u) rotate_bit<RB>(v, b, k);
}

template <typename F>
__host__ __device__ inline Rot<F> make_rot(double t, double s)
{
    Rot<F> k;
    k.t = (F)t;
    k.s = (F)s;
    return k;
}

template <typename ET> constexpr int lut_cap() { return sizeof(ET) == 1 ? kLutMaxU8 : kLutMax; }

struct DevCoef {
    double s, theta, t, sn;
    bool flip;
};

// Shear coefficients of the rotation by phi = theta/2 reduced to
// [-pi/2, pi/2] (flip: reduced by pi, the block changes sign), and the
// step's global phase n theta/2 (+ pi for odd n when flipped) mod 2 pi.
__host__ __device__ inline void rot_params(double theta, double &t, double &sn, bool &flip)
{
    double phi = fmod(0.5 * theta, 2.0 * M_PI);
    if (phi > M_PI) phi -= 2.0 * M_PI;
    flip = false;
    if (phi > 0.5 * M_PI) {
        phi -= M_PI;
        flip = true;
    } else if (phi < -0.5 * M_PI) {
        phi += M_PI;
        flip = true;
    }
    t = tan(0.5 * phi);
    sn = sin(phi);
}

__device__ __forceinline__ double step_gphase(int n, double theta, bool flip)
{
    return fmod(0.5 * (double)n * theta + (flip ? M_PI * (double)(n & 1) : 0.0), 2.0 * M_PI);
}

// Step k of N over total time T: schedule value s_k at the step midpoint
// (knots v[0..count), count 0 = linear) and the rotation coefficients of
// theta_k = dt (1 - s_k) (same formulas as the host).
__device__ __forceinline__ DevCoef dev_step_coef(double T, int64_t N, int64_t k, const double *v, int count)
{
    DevCoef c;
    const double dt = T / (double)N;
    c.s = sched_mid(v, count, k, N);
    c.theta = dt * (1.0 - c.s);
    rot_params(c.theta, c.t, c.sn, c.flip);
    return c;
}

}  // namespace
}  // namespace qaa
