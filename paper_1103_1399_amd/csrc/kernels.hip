// kernels.hip -- gfx950 kernels of libqaa: energy table, state
// initialisation, the fused split-step passes, the LDS-resident small-state
// evolution, and the FP64 observables reduction.
//
// Arithmetic conventions (see include/qaa.h for the physics):
//  - A step's driver factor exp(-i theta H_B) is applied qubit by qubit as
//    [[c, i s], [i s, c]] with c = cos(theta/2), s = sin(theta/2); its global
//    phase exp(-i n theta/2) is folded into the next diagonal phase.
//  - Each 2x2 block is two real plane rotations by theta/2, applied in place
//    as three shears with t = tan(theta/4) and s (three FMAs per component
//    pair; the sheared product stays area-preserving under FP32 rounding of
//    t and s, so no systematic norm drift comes from the coefficients).
//  - Diagonal phases exp(-i a E) come from a per-launch lookup table over E
//    evaluated in FP64 and rounded once.
#include "qaa_internal.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>

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

// ---------------------------------------------------------------------------
// Energy table, bit-sliced.  Thread t scores z = 32t .. 32t+31 at once: for
// each clause the 32 outcomes form one word (bit i: z = 32t + i violates
// it), and the words are summed bit-parallel into counter planes (plane p
// holds bit p of the 32 counts).  Eight clauses at a time go through a
// carry-save tree (planes 0..2 are running sums; the eights it produces
// ripple into the planes above), about 9 word operations per clause for 32
// basis states.  K = 8 planes count to 255; a carry out of the top plane is
// recorded (ovf), and the host then recomputes with K = 16 (m <= 65535).
// Clause records are staged through LDS in chunks, so every wave reads
// them with low-latency broadcast loads instead of scalar-cache round trips.
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

constexpr int kClauseChunk = 1024;     // clause records staged in LDS at a time (16 KiB)

// stats: [0] ~E_min (maximum of complements), [1] E_max, [2] some E > 255
// with a uint8 table, [3] some count passed the K planes (recompute wider)
template <typename ET, int K>
__global__ void __launch_bounds__(256) energy_kernel(const ClauseRec *__restrict__ cl, int m, int n,
                                                     ET *__restrict__ table, uint32_t *__restrict__ stats)
{
    __shared__ ClauseRec cl_s[kClauseChunk];
    const uint64_t dim = 1ull << n;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;     // n <= 34: t < 2^29
    const uint64_t zb = (uint64_t)t * 32ull;
    const bool active = zb < dim;
    BitCounter<K> bc;
    bc.clear();
    for (int c0 = 0; c0 < m; c0 += kClauseChunk) {
        const int cm = min(kClauseChunk, m - c0);
        __syncthreads();         // the previous chunk is read
        for (int i = (int)threadIdx.x; i < cm; i += (int)blockDim.x) cl_s[i] = cl[c0 + i];
        __syncthreads();
        if (active) score_clauses<K>(bc, cl_s, cm, t);
    }
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, over = 0u, wide = 0u;
    if (active) {
        uint32_t e[32];
        bc.counts(e);
        const int cnt = dim < 32 ? (int)dim : 32;
        const uint32_t valid = cnt == 32 ? 0xFFFFFFFFu : ((1u << cnt) - 1u);
        wide = (bc.ovf & valid) ? 1u : 0u;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i < cnt) {
                lo = min(lo, e[i]);
                hi = max(hi, e[i]);
            }
        }
        if (cnt == 32) {
            if constexpr (sizeof(ET) == 1) {
                over = hi > 255u ? 1u : 0u;
                uint4 q[2];
                uint32_t *qw = reinterpret_cast<uint32_t *>(q);
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    qw[d] = (e[4 * d] & 0xFFu) | ((e[4 * d + 1] & 0xFFu) << 8) | ((e[4 * d + 2] & 0xFFu) << 16) |
                            ((e[4 * d + 3] & 0xFFu) << 24);
                uint4 *dst = reinterpret_cast<uint4 *>(table + zb);
                dst[0] = q[0];
                dst[1] = q[1];
            } else {
                uint4 q[4];
                uint32_t *qw = reinterpret_cast<uint32_t *>(q);
#pragma unroll
                for (int d = 0; d < 16; ++d) qw[d] = (e[2 * d] & 0xFFFFu) | ((e[2 * d + 1] & 0xFFFFu) << 16);
                uint4 *dst = reinterpret_cast<uint4 *>(table + zb);
#pragma unroll
                for (int d = 0; d < 4; ++d) dst[d] = q[d];
            }
        } else {
            if (sizeof(ET) == 1) over = hi > 255u ? 1u : 0u;
            for (int i = 0; i < cnt; ++i) table[zb + i] = (ET)e[i];
        }
    }
    // Reduction of min / max / flags: waves, then the workgroup, then one
    // thread updates the global words -- and only where it would change
    // them.  All workgroups target the same four words, so unconditional
    // atomics from every wave serialise at one address (that alone took
    // 3 ms at n = 28); a possibly stale plain read is safe to test against,
    // since the words only grow.
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
        over |= (uint32_t)__shfl_xor((int)over, off, 64);
        wide |= (uint32_t)__shfl_xor((int)wide, off, 64);
    }
    __shared__ uint32_t red[4][4];
    const int wave = (int)(threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = ~lo;      // stats[0] holds ~E_min (the maximum of the
        red[wave][1] = hi;       // complements), so that a zero-filled block
        red[wave][2] = over;     // is the neutral start for all of them
        red[wave][3] = wide;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = (int)threadIdx.x;
        uint32_t v = red[0][k];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = k < 2 ? max(v, red[w][k]) : (v | red[w][k]);
        const uint32_t seen = __atomic_load_n(&stats[k], __ATOMIC_RELAXED);
        if (k < 2 ? v > seen : (v & ~seen) != 0u) {
            if (k < 2)
                atomicMax(&stats[k], v);
            else
                atomicOr(&stats[k], v);
        }
    }
}

template <typename ET>
__global__ void __launch_bounds__(256) count_equal_kernel(const ET *__restrict__ table, uint64_t dim, uint32_t value,
                                                          unsigned long long *__restrict__ count)
{
    unsigned long long c = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride)
        c += (uint32_t)table[z] == value ? 1ull : 0ull;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// ---------------------------------------------------------------------------
// Initial states.
// ---------------------------------------------------------------------------
template <typename F>
__global__ void __launch_bounds__(256) init_uniform_kernel(typename V2<F>::T *__restrict__ amp, uint64_t dim, F a)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        typename V2<F>::T v;
        v.x = a;
        v.y = F(0);
        amp[z] = v;
    }
}

template <typename F>
__global__ void __launch_bounds__(256) init_basis_kernel(typename V2<F>::T *__restrict__ amp, uint64_t dim, uint64_t z0)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        typename V2<F>::T v;
        v.x = z == z0 ? F(1) : F(0);
        v.y = F(0);
        amp[z] = v;
    }
}

// ---------------------------------------------------------------------------
// One fused pass over 2^TB-amplitude tiles (see PassDesc).
//
// The grid is persistent: workgroup b handles tiles b, b + G, b + 2G, ...
// and keeps two register sets, so the HBM loads of its next tile are in
// flight while the current tile is rotated, phased and stored.
// ---------------------------------------------------------------------------

// Add every lane's fixed-point norm share into *acc (one atomic per wave).
__device__ __forceinline__ void norm_accumulate(unsigned long long *acc, unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(acc, v);
}

// Workgroup barrier that orders LDS traffic only: HBM loads issued before it
// stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename F, typename ET, int TB, int RB>
struct PassTraits {
    using F2 = typename V2<F>::T;
    static constexpr int WB = TB - RB;
    static constexpr uint32_t WG = 1u << WB;
    static constexpr int R = 1 << RB;
    static constexpr uint32_t TS = 1u << TB;
    static constexpr int DT = sizeof(F) == 4 ? 0 : 1;
    static constexpr uint32_t TSP = TS + kPadN[DT] * (TS >> kPadS[DT]);
    static constexpr int VW = 16 / sizeof(F2);     // amplitudes per 16-byte access
    static constexpr int EPV = 16 / sizeof(ET);    // energies per 16-byte access
    static constexpr int EB = sizeof(ET) == 1 ? 4 : 3;
    static constexpr int NE = (int)(TS / EPV / WG) > 0 ? (int)(TS / EPV / WG) : 1;
};

// Registers holding one tile in flight: residency-0 amplitudes and energies.
template <typename F, typename ET, int TB, int RB>
struct TileRegs {
    typename V2<F>::T v[1 << RB];
    uint4 ev[PassTraits<F, ET, TB, RB>::NE];
};

// Physical base index of tile w: bit j of w goes to the j-th set bit of
// rest_mask (scalar bit scans, no memory access).
template <typename F, typename ET, int TB, int RB>
__device__ __forceinline__ uint64_t tile_base(const PassDesc &d, uint64_t w)
{
    uint64_t base = 0, m = d.rest_mask;
    while (w) {
        const uint64_t low = m & (~m + 1ull);     // lowest remaining position
        if (w & 1ull) base |= low;
        m ^= low;
        w >>= 1;
    }
    return base;
}

// 32-bit word at a byte offset inside the pass descriptor.
__device__ __forceinline__ uint32_t desc_word(const PassDesc &d, uint32_t byte_off)
{
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(&d) + byte_off);
}
__device__ __forceinline__ uint32_t desc_u8(const PassDesc &d, uint32_t byte_off)
{
    return (desc_word(d, byte_off & ~3u) >> (8 * (byte_off & 3u))) & 0xFFu;
}
__device__ __forceinline__ uint32_t desc_u16(const PassDesc &d, uint32_t byte_off)
{
    return (desc_word(d, byte_off & ~3u) >> (8 * (byte_off & 2u))) & 0xFFFFu;
}

// Issue the HBM loads of one tile: residency-0 registers and, for a phase
// pass, the tile's energies (16 consecutive bytes per access; tile bits 0..3
// are physical bits 0..3 in every plan).
template <typename F, typename ET, int TB, int RB, bool PHASE>
__device__ __forceinline__ void pass_load(TileRegs<F, ET, TB, RB> &tr, const typename V2<F>::T *__restrict__ amp,
                                          const ET *__restrict__ table, const PassDesc &d, uint64_t base, uint64_t tg,
                                          uint32_t tid)
{
    using P = PassTraits<F, ET, TB, RB>;
    using F2 = typename P::F2;
    auto &v = tr.v;
    auto &ev = tr.ev;
    const F2 *p = amp + (base | tg);
#pragma unroll
    for (int j = 0; j < P::R; j += P::VW) {
        if constexpr (P::VW == 2 && PHASE) {
            typedef float f32x4 __attribute__((ext_vector_type(4)));
            const f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p + d.goff_first[j]));
            v[j].x = q.x;
            v[j].y = q.y;
            v[j + 1].x = q.z;
            v[j + 1].y = q.w;
        } else if constexpr (P::VW == 2) {
            const float4 q = *reinterpret_cast<const float4 *>(p + d.goff_first[j]);
            v[j].x = q.x;
            v[j].y = q.y;
            v[j + 1].x = q.z;
            v[j + 1].y = q.w;
        } else {
            v[j] = p[d.goff_first[j]];
        }
    }
    if constexpr (PHASE) {
#pragma unroll
        for (int i = 0; i < P::NE; ++i) {
            const uint32_t c = tid + (uint32_t)i * P::WG;
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < TB - P::EB; ++j) off |= (uint64_t)((c >> j) & 1u) << d.tile_pos[P::EB + j];
            ev[i] = *reinterpret_cast<const uint4 *>(table + (base | off));
        }
    }
}

// Residencies of one tile, ending with the store to HBM.
template <typename F, typename ET, int TB, int RB, bool PHASE>
__device__ __forceinline__ void pass_compute(TileRegs<F, ET, TB, RB> &tr, typename V2<F>::T *__restrict__ amp,
                                             const PassDesc &d, uint64_t base,
                                             uint64_t tg_last, uint32_t tid,
                                             typename V2<F>::T *tile, const typename V2<F>::T *lut, ET *etile,
                                             const Rot<F> &kA, const Rot<F> &kB, bool meas,
                                             unsigned long long &ssq)
{
    using P = PassTraits<F, ET, TB, RB>;
    using F2 = typename P::F2;
    constexpr int DT = P::DT;
    constexpr int R = P::R;
    constexpr int VW = P::VW;
    auto &v = tr.v;
    const auto &ev = tr.ev;
    // the previous tile's LDS reads are finished before this tile writes
    lds_barrier();
    if constexpr (PHASE) {
#pragma unroll
        for (int i = 0; i < P::NE; ++i)
            *reinterpret_cast<uint4 *>(etile + (size_t)(tid + (uint32_t)i * P::WG) * P::EPV) = ev[i];
        lds_barrier();
    }
    const int last = d.n_res - 1;
    // thread part of the tile-local index in residency r
    auto thread_part = [&](int r) {
        const uint32_t o_tpos = (uint32_t)offsetof(PassDesc, tpos) + 16u * (uint32_t)r;
        uint32_t lt = 0;
#pragma unroll
        for (int k = 0; k < P::WB; ++k) lt |= ((tid >> k) & 1u) << desc_u8(d, o_tpos + k);
        return lt;
    };
    // rotations and phase of residency r on the registers
    auto apply = [&](int r, uint32_t lt) {
        const uint32_t o_lj = (uint32_t)offsetof(PassDesc, lj) + 2u * kMaxRegs * (uint32_t)r;
        const uint32_t masks = desc_word(d, (uint32_t)offsetof(PassDesc, masks) + 4u * (uint32_t)r);
        rotate_mask<RB, F2, F>(v, masks & 0xFFu, kA);
        if (PHASE && r == d.phase_at) {
            // four amplitudes at a time keeps the table reads' registers few
#pragma unroll
            for (int j0 = 0; j0 < R; j0 += 4) {
#pragma unroll
                for (int j = j0; j < j0 + 4; ++j) {
                    const uint32_t e = (uint32_t)etile[lt + desc_u16(d, o_lj + 2 * j)];
                    v[j] = cmul<F2, F>(v[j], lut[e]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        rotate_mask<RB, F2, F>(v, (masks >> 8) & 0xFFu, kB);
    };
    auto to_lds = [&](int r, uint32_t ltp) {
        const uint32_t o_ljp = (uint32_t)offsetof(PassDesc, ljp) + 2u * kMaxRegs * (uint32_t)r;
#pragma unroll
        for (int j = 0; j < R; j += VW) {
            F2 *q = tile + ltp + desc_u16(d, o_ljp + 2 * j);
            if constexpr (VW == 2) {
                float4 t4;
                t4.x = v[j].x;
                t4.y = v[j].y;
                t4.z = v[j + 1].x;
                t4.w = v[j + 1].y;
                *reinterpret_cast<float4 *>(q) = t4;
            } else {
                *q = v[j];
            }
        }
    };
    auto from_lds = [&](int r, uint32_t ltp) {
        const uint32_t o_ljp = (uint32_t)offsetof(PassDesc, ljp) + 2u * kMaxRegs * (uint32_t)r;
#pragma unroll
        for (int j = 0; j < R; j += VW) {
            const F2 *q = tile + ltp + desc_u16(d, o_ljp + 2 * j);
            if constexpr (VW == 2) {
                const float4 t4 = *reinterpret_cast<const float4 *>(q);
                v[j].x = t4.x;
                v[j].y = t4.y;
                v[j + 1].x = t4.z;
                v[j + 1].y = t4.w;
            } else {
                v[j] = *q;
            }
        }
    };
    // residency 0 works on the registers loaded from HBM; it is kept out of
    // the loop below so that the loop never waits on HBM loads
    {
        const uint32_t lt = thread_part(0);
        apply(0, lt);
        if (last > 0) {
            to_lds(0, lt + kPadN[DT] * (lt >> kPadS[DT]));
            lds_barrier();
        }
    }
    for (int r = 1; r <= last; ++r) {
        const uint32_t lt = thread_part(r);
        const uint32_t ltp = lt + kPadN[DT] * (lt >> kPadS[DT]);
        from_lds(r, ltp);
        apply(r, lt);
        if (r < last) {
            to_lds(r, ltp);
            lds_barrier();
        }
    }
    F2 *p = amp + (base | tg_last);
    if (meas) {
        // this thread's share of |psi|^2 over the tile, as a fixed-point
        // integer: the total does not depend on which workgroup handled
        // which tile, nor on the order of the additions
        F st = F(0);
#pragma unroll
        for (int j = 0; j < R; ++j) st = fma(v[j].x, v[j].x, fma(v[j].y, v[j].y, st));
        ssq += (unsigned long long)((double)st * kNormFixedScale + 0.5);
    }
    // Passes without a phase store with non-temporal (streaming) hints:
    // measured 5 % faster.  With a phase the hint's register constraints
    // push the kernel past 256 VGPRs, so those keep plain stores.
#pragma unroll
    for (int j = 0; j < R; j += VW) {
        if constexpr (VW == 2) {
            if constexpr (!PHASE) {
                typedef float f32x4 __attribute__((ext_vector_type(4)));
                f32x4 q = {v[j].x, v[j].y, v[j + 1].x, v[j + 1].y};
                __builtin_nontemporal_store(q, reinterpret_cast<f32x4 *>(p + d.goff_last[j]));
            } else {
                float4 q;
                q.x = v[j].x;
                q.y = v[j].y;
                q.z = v[j + 1].x;
                q.w = v[j + 1].y;
                *reinterpret_cast<float4 *>(p + d.goff_last[j]) = q;
            }
        } else {
            if constexpr (!PHASE) {
                typedef double f64x2 __attribute__((ext_vector_type(2)));
                f64x2 q = {v[j].x, v[j].y};
                __builtin_nontemporal_store(q, reinterpret_cast<f64x2 *>(p + d.goff_last[j]));
            } else {
                p[d.goff_last[j]] = v[j];
            }
        }
    }
}

// The tiles first, first + stride, ... (< end) of one pass, pipelined: the
// HBM loads of the next tile are in flight while the current one is
// computed (PIPE), else only tile `first`.  The phase table (a pass with a
// phase) is built in LDS from phi, gphase and the norm correction *acc_in.
// Returns this thread's fixed-point share of sum |psi|^2 when meas is set.
template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE>
__device__ __forceinline__ unsigned long long tile_loop(typename V2<F>::T *__restrict__ amp,
                                                        const ET *__restrict__ table, const PassDesc &d,
                                                        uint64_t first, uint64_t stride, uint64_t end, double phi,
                                                        double gphase, int emax,
                                                        const unsigned long long *acc_in, const Rot<F> &kA,
                                                        const Rot<F> &kB, bool meas)
{
    using P = PassTraits<F, ET, TB, RB>;
    using F2 = typename P::F2;
    static_assert(P::R <= kMaxRegs, "register count");
    extern __shared__ __align__(16) unsigned char smem[];
    F2 *tile = reinterpret_cast<F2 *>(smem);
    F2 *lut = tile + P::TSP;
    ET *etile = reinterpret_cast<ET *>(lut + lut_cap<ET>());

    const uint32_t tid = threadIdx.x;
    uint64_t tg_first = 0, tg_last = 0;
#pragma unroll
    for (int k = 0; k < P::WB; ++k) {
        tg_first |= (uint64_t)((tid >> k) & 1u) << d.gpos_first[k];
        tg_last |= (uint64_t)((tid >> k) & 1u) << d.gpos_last[k];
    }

    // The loads of the next tile are issued unconditionally (past the end,
    // the last tile is read again and not used) so that the number of
    // memory operations in flight is the same on every path; otherwise the
    // compiler's wait counts assume the worst path and stall on the prefetch.
    TileRegs<F, ET, TB, RB> ta, tb;
    // d.reverse: slot w holds tile (tile_begin + tile_count - 1) - (w - tile_begin)
    const uint64_t mirror = d.reverse ? 2 * d.tile_begin + d.tile_count - 1 : 0;
    auto tile_at = [&](uint64_t x) { return tile_base<F, ET, TB, RB>(d, d.reverse ? mirror - x : x); };
    uint64_t w = first;             // callers pass first < end
    pass_load<F, ET, TB, RB, PHASE>(ta, amp, table, d, tile_at(w), tg_first, tid);

    if constexpr (PHASE) {
        const double scale = acc_in ? rsqrt((double)(*acc_in) * (1.0 / kNormFixedScale)) : 1.0;
        for (int e = (int)tid; e <= emax; e += (int)P::WG) {
            double sn, cs;
            sincos(fma(phi, (double)e, gphase), &sn, &cs);
            F2 L;
            L.x = (F)(scale * cs);
            L.y = (F)(-scale * sn);
            lut[e] = L;
        }
    }

    unsigned long long ss = 0ull;
    if constexpr (!PIPE) {
        pass_compute<F, ET, TB, RB, PHASE>(ta, amp, d, tile_at(w), tg_last, tid, tile, lut, etile,
                                           kA, kB, meas, ss);
    }
    while (PIPE) {
        const uint64_t w1 = w + stride;
        pass_load<F, ET, TB, RB, PHASE>(tb, amp, table, d, tile_at(w1 < end ? w1 : w), tg_first,
                                        tid);
        pass_compute<F, ET, TB, RB, PHASE>(ta, amp, d, tile_at(w), tg_last, tid, tile, lut, etile,
                                           kA, kB, meas, ss);
        if (w1 >= end) break;
        const uint64_t w2 = w1 + stride;
        pass_load<F, ET, TB, RB, PHASE>(ta, amp, table, d, tile_at(w2 < end ? w2 : w1), tg_first,
                                        tid);
        pass_compute<F, ET, TB, RB, PHASE>(tb, amp, d, tile_at(w1), tg_last, tid, tile, lut,
                                           etile, kA, kB, meas, ss);
        if (w2 >= end) break;
        w = w2;
    }
    return ss;
}

// Two workgroups of 256 threads per CU (2^13-amplitude tiles, LDS-bound),
// or one of 512 (2^14-amplitude tiles), means two waves per SIMD: the
// register budget is held to that occupancy.
// PIPE: persistent grid (workgroup b takes tiles b, b + grid, ...) with the
// next tile's loads in flight; otherwise one workgroup per tile.
template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE>
__global__ void __launch_bounds__(1 << (TB - RB), (TB - RB) >= 9 ? 1 : 2)
pass_kernel(typename V2<F>::T *__restrict__ amp, const ET *__restrict__ table, const PassDesc d)
{
    if (d.acc_zero && blockIdx.x == 0 && threadIdx.x == 0) *d.acc_zero = 0ull;
    const uint64_t first = d.tile_begin + blockIdx.x;     // grid size <= tile_count
    const unsigned long long ss = tile_loop<F, ET, TB, RB, PHASE, PIPE>(
        amp, table, d, first, gridDim.x, d.tile_begin + d.tile_count, d.phi, d.gphase, d.emax, d.acc_in,
        make_rot<F>(d.tA, d.sA), make_rot<F>(d.tB, d.sB), d.acc_out != nullptr);
    if (d.acc_out) norm_accumulate(d.acc_out, ss);
}

// ---------------------------------------------------------------------------
// Batched passes (see BatchInst).
// ---------------------------------------------------------------------------
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

// Workgroup b takes a chunk of up to chunk_tiles consecutive tiles of state
// chunk_inst[b] (pipelined like pass_kernel); the pass kind, the rotation
// and phase coefficients follow from the global step s, the pass index j
// and the state's own schedule.
template <typename F, typename ET, int TB, int RB>
__global__ void __launch_bounds__(1 << (TB - RB), 2)
batch_pass_kernel(const BatchInst *__restrict__ insts, const uint32_t *__restrict__ chunk_inst,
                  const PassDesc *__restrict__ structs, int64_t s, int j, int chunk_tiles)
{
    const uint64_t g = blockIdx.x;
    const BatchInst &I = insts[chunk_inst[g]];
    if (s >= I.N) return;
    const int r = I.r;
    const int idx = s == 0 ? j : j + 1;       // position in this step's set order
    if (idx >= r) return;
    const bool fwd = (s & 1) == 0;
    const bool last = idx == r - 1;
    const int set = fwd ? idx : r - 1 - idx;
    int kind;
    if (s == 0 && idx == 0)
        kind = 0;
    else if (!last)
        kind = set;
    else if (s + 1 < I.N)
        kind = set == r - 1 ? r - 1 : r;
    else
        kind = set == r - 1 ? r + 1 : r + 2;
    const PassDesc &d = structs[I.struct_base + kind];
    const uint64_t ntiles = 1ull << (I.n - TB);
    const uint64_t w0 = (g - I.chunk_offset) * (uint64_t)chunk_tiles;
    const uint64_t w1 = w0 + (uint64_t)chunk_tiles < ntiles ? w0 + (uint64_t)chunk_tiles : ntiles;

    const double dt = I.T / (double)I.N;
    const DevCoef ck = dev_step_coef(I.T, I.N, s, I.sched.v, I.sched.count);
    Rot<F> kA = make_rot<F>(ck.t, ck.sn), kB = make_rot<F>(0.0, 0.0);
    double phi = 0.0, gph = 0.0;
    if (kind == 0) {
        kB = kA;
        phi = 0.5 * dt * ck.s;
    } else if (kind == r - 1 || kind == r) {
        const DevCoef cn = dev_step_coef(I.T, I.N, s + 1, I.sched.v, I.sched.count);
        kB = make_rot<F>(cn.t, cn.sn);
        phi = 0.5 * dt * (ck.s + cn.s);
        gph = step_gphase(I.n, ck.theta, ck.flip);
    } else if (kind >= r + 1) {
        phi = 0.5 * dt * ck.s;
        gph = step_gphase(I.n, ck.theta, ck.flip);
    }
    // norm control rides on the passes over the top set (every other step)
    unsigned long long *acc_in = nullptr, *acc_out = nullptr;
    if (I.acc && set == r - 1 && last) {
        const int64_t gj = s >> 1;
        acc_out = I.acc + gj % 3;
        acc_in = gj > 0 ? I.acc + (gj + 2) % 3 : nullptr;
        if (w0 == 0 && threadIdx.x == 0) I.acc[(gj + 1) % 3] = 0ull;
    }
    auto *amp = reinterpret_cast<typename V2<F>::T *>(I.amp);
    const ET *table = reinterpret_cast<const ET *>(I.table);
    unsigned long long ss;
    if (d.phase_at >= 0)
        ss = tile_loop<F, ET, TB, RB, true, true>(amp, table, d, w0, 1, w1, phi, gph, I.emax, acc_in, kA, kB,
                                                  acc_out != nullptr);
    else
        ss = tile_loop<F, ET, TB, RB, false, true>(amp, table, d, w0, 1, w1, phi, gph, I.emax, acc_in, kA, kB,
                                                   acc_out != nullptr);
    if (acc_out) norm_accumulate(acc_out, ss);
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup: all steps k0..k1-1 in LDS.  Workgroup b
// evolves state descs[b] (so one launch serves a batch of small states).
//
// The steps run in chunks of up to 32.  At the start of a chunk every
// thread helps build the chunk's coefficients in LDS -- per step the
// rotation (t, s) and the phase row L[e] = exp(-i (phi e + gphase)),
// e = 0..emax, evaluated in FP64 and rounded once -- so that inside the
// chunk a step is only table lookups, rotations and LDS exchanges, with no
// FP64 transcendental on its critical path.  The state is renormalised
// exactly (FP64 norm) once per chunk, folded into the chunk's first row; in
// between the rotations are area-preserving and each phase factor is unit
// to FP32 rounding, so a chunk drifts by at most a few 1e-7.
// RING: LDS entries for the chunk's phase rows (rows of emax + 1 entries).
// ---------------------------------------------------------------------------
constexpr int kResChunk = 32;

template <typename F, typename ET, int RB, int WB, int RING>
__device__ __forceinline__ void resident_body(const ResidentDesc &d)
{
    using F2 = typename V2<F>::T;
    constexpr int R = 1 << RB;
    constexpr uint32_t TS = 1u << (RB + WB);
    extern __shared__ __align__(16) unsigned char smem[];
    F2 *tile = reinterpret_cast<F2 *>(smem);
    F2 *ring = tile + TS;
    ET *etile = reinterpret_cast<ET *>(ring + RING);

    F2 *__restrict__ amp = reinterpret_cast<F2 *>(d.amp);
    const ET *__restrict__ table = reinterpret_cast<const ET *>(d.table);
    const int n = d.n;
    const uint32_t dim = 1u << n;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = 1u << d.thr_bits;
    const bool active = tid < nthr;
    const uint32_t used = (1u << d.reg_bits) - 1u;   // register-index bits in use

    // Per-group index maps, computed once: thread part lt (per thread) and
    // register offsets lj (uniform) of every group; reading them from the
    // descriptor inside the step loop would put a chain of memory loads on
    // every step.
    __shared__ uint32_t lt_s[8][1 << WB];
    __shared__ uint32_t lj_s[8][R];
    __shared__ uint32_t gm_s[8];
    for (int g = 0; g < d.n_groups; ++g) {
        uint32_t lt = 0;
        for (int k = 0; k < d.thr_bits; ++k) lt |= ((tid >> k) & 1u) << d.tpos[g][k];
        lt_s[g][tid] = lt;
    }
    for (uint32_t x = tid; x < 8u * R; x += blockDim.x) {
        const int g = (int)(x / R), j = (int)(x % R);
        uint32_t o = 0;
        if (g < d.n_groups)
            for (int i = 0; i < RB && i < d.reg_bits; ++i)
                if ((j >> i) & 1) o |= 1u << d.gbits[g][i];
        lj_s[g][j] = o;
    }
    if (tid < 8) gm_s[tid] = d.gmask[tid];
    __shared__ double knots_s[kMaxKnots];
    const int kcount = d.sched.count;
    for (int x = (int)tid; x < kcount; x += (int)blockDim.x) knots_s[x] = d.sched.v[x];

    for (uint32_t z = tid; z < dim; z += blockDim.x) {
        tile[swz<F>(z)] = amp[z];
        etile[z] = table[z];
    }

    const double dt = d.T / (double)d.N;
    const int width = d.emax + 1;                       // entries of a phase row
    const int chunk = min(kResChunk, RING / width);     // >= 1: width <= the LUT limit <= RING
    __shared__ double red[(1 << WB) / 64];
    __shared__ double phi_s[kResChunk], gph_s[kResChunk];
    __shared__ Rot<F> rot_s[kResChunk];
    double part = 0.0;     // this thread's share of |psi|^2 after the last residency
    // Norm of the state from the per-thread partials: butterfly sums inside
    // each wave, then the wave sums in order (a fixed order: deterministic).
    auto measure = [&]() {
        double t = part;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((tid & 63) == 0) red[tid >> 6] = t;
        __syncthreads();
        double total = 0.0;
#pragma unroll
        for (int w = 0; w < (1 << WB) / 64; ++w) total += red[w];
        __syncthreads();      // red is rewritten by the next measure
        return total;
    };
    // phase angle phi_k, global phase and rotation of step k: the half phase
    // that opens the range (k == k0), else the merged halves of k-1 and k
    // with step k-1's driver global phase
    auto step_terms = [&](int64_t k, double &phi, double &gph, double &rt, double &rs) {
        const double sk = sched_mid(knots_s, kcount, k, d.N);
        bool flip;
        rot_params(dt * (1.0 - sk), rt, rs, flip);
        if (k == d.k0) {
            phi = 0.5 * dt * sk;
            gph = 0.0;
        } else {
            const double sp = sched_mid(knots_s, kcount, k - 1, d.N);
            const double thp = dt * (1.0 - sp);
            double tp, sq;
            bool fp;
            rot_params(thp, tp, sq, fp);
            phi = 0.5 * dt * (sp + sk);
            gph = step_gphase(n, thp, fp);
        }
    };
    // rows [0, rows) of the chunk's phase table from phi_s / gph_s; row 0
    // carries the norm correction
    auto build_rows = [&](int rows, double scale0) {
        for (int x = (int)tid; x < rows * width; x += (int)blockDim.x) {
            const int j = x / width, e = x - j * width;
            double sn, cs;
            sincos(fma(phi_s[j], (double)e, gph_s[j]), &sn, &cs);
            const double sc = j == 0 ? scale0 : 1.0;
            F2 L;
            L.x = (F)(sc * cs);
            L.y = (F)(-sc * sn);
            ring[x] = L;
        }
    };
    auto residency = [&](int g, const F2 *lut, uint32_t rmask, const Rot<F> &k, bool meas) {
        if (active) {
            const uint32_t lt = lt_s[g][tid];
            const uint32_t slt = swz<F>(lt);
            uint32_t lj[R];
#pragma unroll
            for (int j = 0; j < R; ++j) lj[j] = lj_s[g][j];
            F2 v[R];
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (((uint32_t)j & ~used) == 0) v[j] = tile[slt ^ swz<F>(lj[j])];
            if (lut) {
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if (((uint32_t)j & ~used) == 0) v[j] = cmul<F2, F>(v[j], lut[(uint32_t)etile[lt | lj[j]]]);
            }
            rotate_mask<RB>(v, rmask, k);
            F ss = F(0);
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (((uint32_t)j & ~used) == 0) {
                    tile[slt ^ swz<F>(lj[j])] = v[j];
                    ss = fma(v[j].x, v[j].x, fma(v[j].y, v[j].y, ss));
                }
            if (meas) part = (double)ss;
        }
        __syncthreads();
    };

    double scale = 1.0;          // norm correction for the next phase row
    for (int64_t kc = d.k0; kc < d.k1; kc += chunk) {
        const int cs = (int)min<int64_t>((int64_t)chunk, d.k1 - kc);
        __syncthreads();         // knots loaded / the previous chunk's rows read
        if ((int)tid < cs) {
            double phi, gph, rt, rs;
            step_terms(kc + (int)tid, phi, gph, rt, rs);
            phi_s[tid] = phi;
            gph_s[tid] = gph;
            rot_s[tid] = make_rot<F>(rt, rs);
        }
        __syncthreads();
        build_rows(cs, scale);
        __syncthreads();
        for (int j = 0; j < cs; ++j) {
            const Rot<F> rk = rot_s[j];
            for (int g = 0; g < d.n_groups; ++g)
                residency(g, g == 0 ? ring + j * width : nullptr, gm_s[g], rk, j == cs - 1 && g == d.n_groups - 1);
        }
        scale = rsqrt(measure());
    }
    if (d.k1 > d.k0) {
        // closing half phase of the last step, with its driver global phase
        __syncthreads();
        if (tid == 0) {
            const double sl = sched_mid(knots_s, kcount, d.k1 - 1, d.N);
            const double thl = dt * (1.0 - sl);
            double tl, sl2;
            bool fl;
            rot_params(thl, tl, sl2, fl);
            phi_s[0] = 0.5 * dt * sl;
            gph_s[0] = step_gphase(n, thl, fl);
        }
        __syncthreads();
        build_rows(1, scale);
        __syncthreads();
        residency(0, ring, 0u, make_rot<F>(0.0, 0.0), false);
    }
    for (uint32_t z = tid; z < dim; z += blockDim.x) amp[z] = tile[swz<F>(z)];
}

// Coefficient rows in LDS: a single state has the device to itself, a
// batch keeps its workgroups small enough for two per CU.
constexpr int kResRingOne = 2048;
constexpr int kResRingBatch = 1024;

// One state, descriptor passed by value.
template <typename F, typename ET, int RB, int WB>
__global__ void __launch_bounds__(1 << WB) resident_one_kernel(const ResidentDesc d)
{
    resident_body<F, ET, RB, WB, kResRingOne>(d);
}

// A batch of states, workgroup b takes descs[b].
template <typename F, typename ET, int RB, int WB>
__global__ void __launch_bounds__(1 << WB) resident_batch_kernel(const ResidentDesc *__restrict__ descs)
{
    resident_body<F, ET, RB, WB, kResRingBatch>(descs[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Observables: per-block FP64 partials, then one block sums them in a fixed
// order (deterministic for a given grid size).
// ---------------------------------------------------------------------------
template <typename F, typename ET>
__global__ void __launch_bounds__(256) obs_partial_kernel(const typename V2<F>::T *__restrict__ amp,
                                                          const ET *__restrict__ table, uint64_t dim, uint32_t emin,
                                                          double *__restrict__ partials)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < dim; z += stride) {
        const typename V2<F>::T v = amp[z];
        const double p = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        const uint32_t e = (uint32_t)table[z];
        a0 += p;
        a1 += (double)e * p;
        a2 += e == emin ? p : 0.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off, 64);
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
    }
    __shared__ double red[4][3];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = a0;
        red[wave][1] = a1;
        red[wave][2] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w][threadIdx.x];
        partials[(uint64_t)blockIdx.x * 3 + threadIdx.x] = t;
    }
}

__global__ void __launch_bounds__(256) obs_final_kernel(const double *__restrict__ partials, int nblocks,
                                                        double *__restrict__ out)
{
    __shared__ double red[256][3];
    double a[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int c = 0; c < 3; ++c) a[c] += partials[(uint64_t)b * 3 + c];
    for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = a[c];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int c = 0; c < 3; ++c) red[threadIdx.x][c] += red[threadIdx.x + h][c];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[0][threadIdx.x];
}

__global__ void zero_u64_kernel(unsigned long long *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap)
{
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE>
hipError_t launch_pass_p(void *amp, const void *table, const PassDesc &d, hipStream_t s)
{
    using F2 = typename V2<F>::T;
    constexpr int DT = sizeof(F) == 4 ? 0 : 1;
    constexpr size_t TS = size_t(1) << TB;
    const size_t lds = sizeof(F2) * (TS + kPadN[DT] * (TS >> kPadS[DT]) + lut_cap<ET>()) + sizeof(ET) * TS;
    const void *fn = reinterpret_cast<const void *>(&pass_kernel<F, ET, TB, RB, PHASE, PIPE>);
    // persistent grid: as many workgroups as fit on the device at once
    // (set up once per instantiation; static initialisation is thread-safe)
    struct Setup {
        hipError_t err;
        unsigned resident;
    };
    static const Setup setup = [&] {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int dev = 0, cus = 0, per_cu = 0;
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 1 << (TB - RB), lds);
        return Setup{e, (unsigned)std::max(1, cus * std::max(1, per_cu))};
    }();
    if (setup.err != hipSuccess) return setup.err;
    const unsigned grid = PIPE ? (unsigned)std::min<uint64_t>(d.tile_count, setup.resident) : (unsigned)d.tile_count;
    hipLaunchKernelGGL((pass_kernel<F, ET, TB, RB, PHASE, PIPE>), dim3(grid), dim3(1u << (TB - RB)), lds, s,
                       reinterpret_cast<F2 *>(amp), reinterpret_cast<const ET *>(table), d);
    return hipGetLastError();
}

// Kernel variant: the persistent grid with the next tile's loads in
// flight, or one workgroup per tile, as the planner chose for the pass
// (PassDesc::persist).  Tuning switch QAA_PASS_VARIANT: 2 forces the
// persistent grid everywhere, 0 one workgroup per tile everywhere.
inline int pass_variant()
{
    static const int v = [] {
        const char *e = std::getenv("QAA_PASS_VARIANT");
        return e ? (std::atoi(e) & 2) : -1;
    }();
    return v;
}

template <typename F, typename ET, int TB, int RB, bool PHASE>
hipError_t launch_pass_v(void *amp, const void *table, const PassDesc &d, hipStream_t s)
{
    const int v = pass_variant();
    if (v == 0 || (v < 0 && !d.persist)) return launch_pass_p<F, ET, TB, RB, PHASE, false>(amp, table, d, s);
    return launch_pass_p<F, ET, TB, RB, PHASE, true>(amp, table, d, s);
}

template <typename F, typename ET, int TB, int RB>
hipError_t launch_pass_t(void *amp, const void *table, const PassDesc &d, hipStream_t s)
{
    if (d.phase_at >= 0) return launch_pass_v<F, ET, TB, RB, true>(amp, table, d, s);
    return launch_pass_v<F, ET, TB, RB, false>(amp, table, d, s);
}

template <typename F, typename ET, int RB, int WB, bool ONE>
hipError_t launch_resident_t(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, hipStream_t s)
{
    using F2 = typename V2<F>::T;
    const size_t ring = ONE ? kResRingOne : kResRingBatch;
    const size_t lds = sizeof(F2) * ((size_t(1) << (RB + WB)) + ring) + sizeof(ET) * (size_t(1) << (RB + WB));
    const void *fn;
    if constexpr (ONE)
        fn = reinterpret_cast<const void *>(&resident_one_kernel<F, ET, RB, WB>);
    else
        fn = reinterpret_cast<const void *>(&resident_batch_kernel<F, ET, RB, WB>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    if constexpr (ONE)
        hipLaunchKernelGGL((resident_one_kernel<F, ET, RB, WB>), dim3(1), dim3(1u << WB), lds, s, *one);
    else
        hipLaunchKernelGGL((resident_batch_kernel<F, ET, RB, WB>), dim3(count), dim3(1u << WB), lds, s, descs_dev);
    return hipGetLastError();
}

}  // namespace

// Tile shapes compiled into the library (planner picks among them).
//   complex64 : tile 2^13 = 8192 amps, 32 per thread, 256 threads;
//               tile 2^14 = 16384 amps, 32 per thread, 512 threads (uint8 table)
//   complex128: tile 2^12 = 4096 amps, 16 per thread, 256 threads
hipError_t launch_pass(void *amp, int dtype, const void *table, int etype, int tile_bits, int reg_bits,
                       const PassDesc &d, hipStream_t s)
{
    // 2^14-amplitude tiles: complex64 with a uint8 table only (LDS)
    if (dtype == 0 && tile_bits == kWideTileBits && reg_bits == 5 && etype == 0)
        return launch_pass_t<float, uint8_t, kWideTileBits, 5>(amp, table, d, s);
    if (dtype == 0 && tile_bits == 13 && reg_bits == 5) {
        if (etype == 0) return launch_pass_t<float, uint8_t, 13, 5>(amp, table, d, s);
        return launch_pass_t<float, uint16_t, 13, 5>(amp, table, d, s);
    }
    if (dtype == 1 && tile_bits == 12 && reg_bits == 4) {
        if (etype == 0) return launch_pass_t<double, uint8_t, 12, 4>(amp, table, d, s);
        return launch_pass_t<double, uint16_t, 12, 4>(amp, table, d, s);
    }
    return hipErrorInvalidValue;
}

template <typename F, typename ET, int TB, int RB>
hipError_t launch_batch_t(const BatchInst *insts, const uint32_t *chunk_inst, uint64_t chunks, const PassDesc *structs,
                          int64_t s, int j, int chunk_tiles, hipStream_t st)
{
    using F2 = typename V2<F>::T;
    constexpr int DT = sizeof(F) == 4 ? 0 : 1;
    constexpr size_t TS = size_t(1) << TB;
    const size_t lds = sizeof(F2) * (TS + kPadN[DT] * (TS >> kPadS[DT]) + lut_cap<ET>()) + sizeof(ET) * TS;
    const void *fn = reinterpret_cast<const void *>(&batch_pass_kernel<F, ET, TB, RB>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((batch_pass_kernel<F, ET, TB, RB>), dim3((unsigned)chunks), dim3(1u << (TB - RB)), lds, st,
                       insts, chunk_inst, structs, s, j, chunk_tiles);
    return hipGetLastError();
}

hipError_t launch_batch_pass(const BatchInst *insts, const uint32_t *chunk_inst, uint64_t chunks,
                             const PassDesc *structs, int64_t s, int j, int chunk_tiles, int dtype, int etype,
                             int tile_bits, int reg_bits, hipStream_t st)
{
    if (chunks == 0) return hipSuccess;
    if (dtype == 0 && tile_bits == 13 && reg_bits == 5) {
        if (etype == 0)
            return launch_batch_t<float, uint8_t, 13, 5>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
        return launch_batch_t<float, uint16_t, 13, 5>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
    }
    if (dtype == 1 && tile_bits == 12 && reg_bits == 4) {
        if (etype == 0)
            return launch_batch_t<double, uint8_t, 12, 4>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
        return launch_batch_t<double, uint16_t, 12, 4>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
    }
    return hipErrorInvalidValue;
}

// Single-state shapes (see resident_shape): 2^(rb + wb) amplitudes.
template <typename F, typename ET>
hipError_t launch_resident_one(const ResidentDesc *one, int rb, int wb, hipStream_t s)
{
    if (rb == 2 && wb == 8) return launch_resident_t<F, ET, 2, 8, true>(nullptr, one, 1, s);
    if (rb == 2 && wb == 9) return launch_resident_t<F, ET, 2, 9, true>(nullptr, one, 1, s);
    if (rb == 2 && wb == 10) return launch_resident_t<F, ET, 2, 10, true>(nullptr, one, 1, s);
    if constexpr (sizeof(F) == 4)
        if (rb == 3 && wb == 10) return launch_resident_t<F, ET, 3, 10, true>(nullptr, one, 1, s);
    return hipErrorInvalidValue;
}

hipError_t launch_resident(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, int dtype, int etype,
                           int rb, int wb, hipStream_t s)
{
    if (one) {
        if (dtype == 0)
            return etype == 0 ? launch_resident_one<float, uint8_t>(one, rb, wb, s)
                              : launch_resident_one<float, uint16_t>(one, rb, wb, s);
        return etype == 0 ? launch_resident_one<double, uint8_t>(one, rb, wb, s)
                          : launch_resident_one<double, uint16_t>(one, rb, wb, s);
    }
    if (rb != kResRegBits[dtype] || wb != kResThrBits) return hipErrorInvalidValue;
    if (dtype == 0) {
        if (etype == 0) return launch_resident_t<float, uint8_t, 5, 8, false>(descs_dev, nullptr, count, s);
        return launch_resident_t<float, uint16_t, 5, 8, false>(descs_dev, nullptr, count, s);
    }
    if (etype == 0) return launch_resident_t<double, uint8_t, 4, 8, false>(descs_dev, nullptr, count, s);
    return launch_resident_t<double, uint16_t, 4, 8, false>(descs_dev, nullptr, count, s);
}

hipError_t launch_energy(const ClauseRec *cl, int m, int n, void *table, int etype, bool wide, uint32_t *stats,
                         hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const uint64_t threads = (dim + 31) / 32;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    if (etype == 0) {
        if (!wide)
            hipLaunchKernelGGL((energy_kernel<uint8_t, 8>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint8_t *>(table), stats);
        else
            hipLaunchKernelGGL((energy_kernel<uint8_t, 16>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint8_t *>(table), stats);
    } else {
        if (!wide)
            hipLaunchKernelGGL((energy_kernel<uint16_t, 8>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint16_t *>(table), stats);
        else
            hipLaunchKernelGGL((energy_kernel<uint16_t, 16>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint16_t *>(table), stats);
    }
    return hipGetLastError();
}

void energy_block_host(const ClauseRec *cl, int m, uint32_t t, uint32_t *out32)
{
    // as on the device: 8 planes, 16 when some count passes 255
    uint32_t e[32];
    BitCounter<8> narrow;
    narrow.clear();
    score_clauses<8>(narrow, cl, m, t);
    if (!narrow.ovf) {
        narrow.counts(e);
    } else {
        BitCounter<16> wide;
        wide.clear();
        score_clauses<16>(wide, cl, m, t);
        wide.counts(e);
    }
    for (int i = 0; i < 32; ++i) out32[i] = e[i];
}

hipError_t launch_count_equal(const void *table, int etype, int n, int value, unsigned long long *count,
                              hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const unsigned grid = grid_for(dim, 256 * 16, 4096);
    if (etype == 0)
        hipLaunchKernelGGL((count_equal_kernel<uint8_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint8_t *>(table), dim, (uint32_t)value, count);
    else
        hipLaunchKernelGGL((count_equal_kernel<uint16_t>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<const uint16_t *>(table), dim, (uint32_t)value, count);
    return hipGetLastError();
}

hipError_t launch_init_uniform(void *amp, int dtype, int n, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const unsigned grid = grid_for(dim, 256 * 8, 8192);
    const double a = std::ldexp(1.0, -(n / 2)) * ((n & 1) ? std::sqrt(0.5) : 1.0);
    if (dtype == 0)
        hipLaunchKernelGGL((init_uniform_kernel<float>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<float2 *>(amp), dim, (float)a);
    else
        hipLaunchKernelGGL((init_uniform_kernel<double>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<double2 *>(amp), dim, a);
    return hipGetLastError();
}

hipError_t launch_init_basis(void *amp, int dtype, int n, uint64_t z0, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const unsigned grid = grid_for(dim, 256 * 8, 8192);
    if (dtype == 0)
        hipLaunchKernelGGL((init_basis_kernel<float>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<float2 *>(amp), dim, z0);
    else
        hipLaunchKernelGGL((init_basis_kernel<double>), dim3(grid), dim3(256), 0, s,
                           reinterpret_cast<double2 *>(amp), dim, z0);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3((count + 63) / 64), dim3(64), 0, s, p, count);
    return hipGetLastError();
}

int observables_blocks(int n)
{
    const uint64_t dim = 1ull << n;
    return (int)grid_for(dim, 256 * 16, 2048);
}

hipError_t launch_observables(const void *amp, int dtype, const void *table, int etype, int n, int emin,
                              double *partials, int nblocks, double *out, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    if (dtype == 0) {
        if (etype == 0)
            hipLaunchKernelGGL((obs_partial_kernel<float, uint8_t>), dim3(nblocks), dim3(256), 0, s,
                               reinterpret_cast<const float2 *>(amp), reinterpret_cast<const uint8_t *>(table), dim,
                               (uint32_t)emin, partials);
        else
            hipLaunchKernelGGL((obs_partial_kernel<float, uint16_t>), dim3(nblocks), dim3(256), 0, s,
                               reinterpret_cast<const float2 *>(amp), reinterpret_cast<const uint16_t *>(table), dim,
                               (uint32_t)emin, partials);
    } else {
        if (etype == 0)
            hipLaunchKernelGGL((obs_partial_kernel<double, uint8_t>), dim3(nblocks), dim3(256), 0, s,
                               reinterpret_cast<const double2 *>(amp), reinterpret_cast<const uint8_t *>(table), dim,
                               (uint32_t)emin, partials);
        else
            hipLaunchKernelGGL((obs_partial_kernel<double, uint16_t>), dim3(nblocks), dim3(256), 0, s,
                               reinterpret_cast<const double2 *>(amp), reinterpret_cast<const uint16_t *>(table), dim,
                               (uint32_t)emin, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace qaa
