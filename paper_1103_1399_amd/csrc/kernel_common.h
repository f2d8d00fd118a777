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

// ---------------------------------------------------------------------------
// Bit-sliced clause counting (the energy function of Sec. 4.3), shared by
// the energy-table kernel and the kernels that recompute E(z) from the
// clause records instead of reading a table.  A thread scores the 32
// basis states z = 32t .. 32t+31 at once: per clause one 32-bit word of
// outcomes, summed into counter planes by carry-save adders.
// ---------------------------------------------------------------------------
// Carry-save adder on bit planes: a + b + c = lo + 2 hi, bit by bit.
__host__ __device__ inline void csa(uint32_t &hi, uint32_t &lo, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t u = a ^ b;
    hi = (a & b) | (u & c);
    lo = u ^ c;
}

template <int K>
struct BitCounter {
    uint32_t p[K];       // counter planes: bit i of p[b] is bit b of the count of z = 32t + i
    uint32_t ovf;        // lanes whose count passed 2^K - 1

    __host__ __device__ void clear()
    {
#pragma unroll
        for (int b = 0; b < K; ++b) p[b] = 0u;
        ovf = 0u;
    }
    // add `carry` at plane `from` and ripple upwards
    __host__ __device__ void ripple(uint32_t carry, int from)
    {
#pragma unroll
        for (int b = 0; b < K; ++b) {
            if (b < from) continue;
            const uint32_t nc = p[b] & carry;
            p[b] ^= carry;
            carry = nc;
        }
        ovf |= carry;
    }
    __host__ __device__ void add8(const uint32_t (&w)[8])
    {
        uint32_t twos_a, twos_b, fours_a, fours_b, eights;
        csa(twos_a, p[0], p[0], w[0], w[1]);
        csa(twos_b, p[0], p[0], w[2], w[3]);
        csa(fours_a, p[1], p[1], twos_a, twos_b);
        csa(twos_a, p[0], p[0], w[4], w[5]);
        csa(twos_b, p[0], p[0], w[6], w[7]);
        csa(fours_b, p[1], p[1], twos_a, twos_b);
        csa(eights, p[2], p[2], fours_a, fours_b);
        ripple(eights, 3);
    }
    __host__ __device__ void counts(uint32_t (&e)[32]) const
    {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            uint32_t v = 0u;
#pragma unroll
            for (int b = 0; b < K; ++b) v |= ((p[b] >> i) & 1u) << b;
            e[i] = v;
        }
    }
};

// Add clauses cl[0..m) for the block of thread t (z = 32t .. 32t+31).
template <int K>
__host__ __device__ inline void score_clauses(BitCounter<K> &bc, const ClauseRec *__restrict__ cl, int m, uint32_t t)
{
    auto word = [&](const ClauseRec &r) { return (t & r.mhi) == r.phi ? r.low : 0u; };
    int c = 0;
    for (; c + 8 <= m; c += 8) {
        uint32_t w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) w[j] = word(cl[c + j]);
        bc.add8(w);
    }
    for (; c < m; ++c) bc.ripple(word(cl[c]), 0);
}

// Count of z = 32t + lane from the planes.
template <int K>
__host__ __device__ inline uint32_t count_of(const BitCounter<K> &bc, uint32_t lane)
{
    uint32_t v = 0u;
#pragma unroll
    for (int b = 0; b < K; ++b) v |= ((bc.p[b] >> lane) & 1u) << b;
    return v;
}

}  // namespace
}  // namespace qaa
