// kernels.hip -- gfx950 kernels of libqaa: energy table, state
// initialisation, the fused split-step passes, the LDS-resident small-state
// evolution, and the FP64 observables reduction.
//
// Arithmetic conventions (see include/qaa.h for the physics):
//  - A step's driver factor exp(-i theta H_B) is applied qubit by qubit as
//    [[c, i s], [i s, c]] with c = cos(theta/2), s = sin(theta/2); its global
//    phase exp(-i n theta/2) is folded into the next diagonal phase.
//  - c is carried as cm1 = c - 1 so that the update x + cm1 x keeps the
//    small correction exact to FP32 relative precision ("delta form").
//  - Diagonal phases exp(-i a E) come from a per-launch lookup table over E
//    evaluated in FP64 and rounded once.
#include "qaa_internal.h"

#include <cmath>

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

// Rotate register bit b of every pair in v: (x0, x1) <- (c x0 + i s x1,
// c x1 + i s x0) with c = 1 + cm1.
template <int RB, typename F2, typename F>
__device__ __forceinline__ void rotate_bit(F2 (&v)[1 << RB], int b, F cm1, F s)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        if (j & (1 << b)) continue;
        const int k = j | (1 << b);
        const F2 x0 = v[j], x1 = v[k];
        v[j].x = fma(-s, x1.y, fma(cm1, x0.x, x0.x));
        v[j].y = fma(s, x1.x, fma(cm1, x0.y, x0.y));
        v[k].x = fma(-s, x0.y, fma(cm1, x1.x, x1.x));
        v[k].y = fma(s, x0.x, fma(cm1, x1.y, x1.y));
    }
}

template <int RB, typename F2, typename F>
__device__ __forceinline__ void rotate_mask(F2 (&v)[1 << RB], uint32_t mask, F cm1, F s)
{
#pragma unroll
    for (int b = 0; b < RB; ++b)
        if ((mask >> b) & 1u) rotate_bit<RB>(v, b, cm1, s);
}

template <typename ET> constexpr int lut_cap() { return sizeof(ET) == 1 ? kLutMaxU8 : kLutMax; }

// ---------------------------------------------------------------------------
// Energy table.  Thread t scores z = 8t .. 8t+7 against every clause with
// 16-bit packed counters (no overflow: m <= 65535).
// ---------------------------------------------------------------------------
template <typename ET>
__global__ void __launch_bounds__(256) energy_kernel(const ClauseRec *__restrict__ cl, int m, int n,
                                                     ET *__restrict__ table, uint32_t *__restrict__ stats)
{
    const uint64_t dim = 1ull << n;
    const uint64_t zb = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8ull;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, over = 0u;
    if (zb < dim) {
        uint64_t acc_a = 0, acc_b = 0;
        for (int c = 0; c < m; ++c) {
            const ClauseRec r = cl[c];
            const bool hit = (zb & r.mhi) == r.phi;
            acc_a += hit ? r.lo_a : 0ull;
            acc_b += hit ? r.lo_b : 0ull;
        }
        const int cnt = dim < 8 ? (int)dim : 8;
        uint32_t e[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            e[j] = (uint32_t)((acc_a >> (16 * j)) & 0xFFFFu);
            e[j + 4] = (uint32_t)((acc_b >> (16 * j)) & 0xFFFFu);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j < cnt) {
                lo = min(lo, e[j]);
                hi = max(hi, e[j]);
            }
        }
        if (sizeof(ET) == 1) {
            over = hi > 255u ? 1u : 0u;
            if (cnt == 8) {
                uint64_t packed = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) packed |= (uint64_t)(e[j] & 0xFFu) << (8 * j);
                *reinterpret_cast<uint64_t *>(table + zb) = packed;
            } else {
                for (int j = 0; j < cnt; ++j) table[zb + j] = (ET)e[j];
            }
        } else {
            if (cnt == 8) {
                uint4 packed;
                packed.x = e[0] | (e[1] << 16);
                packed.y = e[2] | (e[3] << 16);
                packed.z = e[4] | (e[5] << 16);
                packed.w = e[6] | (e[7] << 16);
                *reinterpret_cast<uint4 *>(table + zb) = packed;
            } else {
                for (int j = 0; j < cnt; ++j) table[zb + j] = (ET)e[j];
            }
        }
    }
    // wave reduction of min / max / overflow, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
        over |= (uint32_t)__shfl_xor((int)over, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&stats[0], lo);
        atomicMax(&stats[1], hi);
        if (over) atomicOr(&stats[2], over);
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
// ---------------------------------------------------------------------------
template <typename F, typename ET, int TB, int RB>
__global__ void __launch_bounds__(1 << (TB - RB))
pass_kernel(typename V2<F>::T *__restrict__ amp, const ET *__restrict__ table, const PassDesc d)
{
    using F2 = typename V2<F>::T;
    constexpr int WB = TB - RB;
    constexpr uint32_t WG = 1u << WB;
    constexpr int R = 1 << RB;
    constexpr uint32_t TS = 1u << TB;
    extern __shared__ __align__(16) unsigned char smem[];
    F2 *tile = reinterpret_cast<F2 *>(smem);
    F2 *lut = tile + TS;
    ET *etile = reinterpret_cast<ET *>(lut + lut_cap<ET>());

    const uint32_t tid = threadIdx.x;
    const bool has_phase = d.phase_at >= 0;

    uint64_t base = 0;
    {
        const uint64_t w = blockIdx.x;
        for (int j = 0; j < d.n_rest; ++j) base |= ((w >> j) & 1ull) << d.rest_pos[j];
    }
    if (has_phase) {
        const double scale = d.acc_in ? rsqrt((double)(*d.acc_in) * (1.0 / kNormFixedScale)) : 1.0;
        for (int e = (int)tid; e <= d.emax; e += (int)WG) {
            double sn, cs;
            sincos(fma(d.phi, (double)e, d.gphase), &sn, &cs);
            F2 L;
            L.x = (F)(scale * cs);
            L.y = (F)(-scale * sn);
            lut[e] = L;
        }
    }
    if (d.acc_zero && blockIdx.x == 0 && tid == 0) *d.acc_zero = 0ull;

    // global -> registers -> LDS.  Each access moves 16 bytes: VW
    // consecutive amplitudes (tile bit 0 is physical bit 0, so pairs are
    // adjacent in memory).  Vector v = tid + i * WG covers tile-local
    // indices VW*v .. VW*v + VW-1.  All loads are issued before the first
    // LDS store so that every thread has R loads in flight.
    constexpr int VW = 16 / sizeof(F2);          // amplitudes per 16-byte access
    constexpr int NV = R / VW;                   // vector accesses per thread
    constexpr int VB = VW == 2 ? 1 : 0;          // log2(VW)
    uint64_t off_t = 0;
#pragma unroll
    for (int j = 0; j < WB; ++j) off_t |= (uint64_t)((tid >> j) & 1u) << d.tile_pos[VB + j];
    uint64_t goff[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        uint64_t off_i = 0;
#pragma unroll
        for (int j = 0; j < RB - VB; ++j)
            if ((i >> j) & 1) off_i |= 1ull << d.tile_pos[VB + WB + j];
        goff[i] = base | off_t | off_i;
    }
    {
        F2 v[R];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if constexpr (VW == 2) {
                const float4 q = *reinterpret_cast<const float4 *>(amp + goff[i]);
                v[2 * i].x = q.x;
                v[2 * i].y = q.y;
                v[2 * i + 1].x = q.z;
                v[2 * i + 1].y = q.w;
            } else {
                v[i] = amp[goff[i]];
            }
        }
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int k = 0; k < VW; ++k) tile[swz<F>((uint32_t)(VW * (tid + i * WG) + k))] = v[VW * i + k];
    }
    if (has_phase) {
        // energies: 16 consecutive bytes (tile bits 0..3 are physical bits
        // 0..3 in every plan) per access
        constexpr int EPV = 16 / sizeof(ET);                  // entries per 16-byte access
        constexpr int EB = sizeof(ET) == 1 ? 4 : 3;           // log2(EPV)
        constexpr int NE = (int)(TS / EPV / WG) > 0 ? (int)(TS / EPV / WG) : 1;
        uint4 ev[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const uint32_t c = tid + (uint32_t)i * WG;          // chunk index
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < TB - EB; ++j) off |= (uint64_t)((c >> j) & 1u) << d.tile_pos[EB + j];
            ev[i] = *reinterpret_cast<const uint4 *>(table + (base | off));
        }
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const uint32_t c = tid + (uint32_t)i * WG;
            *reinterpret_cast<uint4 *>(etile + (size_t)c * EPV) = ev[i];
        }
    }
    __syncthreads();

    const F cm1A = (F)d.cm1A, sA = (F)d.sA, cm1B = (F)d.cm1B, sB = (F)d.sB;
    for (int r = 0; r < d.n_res; ++r) {
        uint32_t lt = 0;
#pragma unroll
        for (int k = 0; k < WB; ++k) lt |= ((tid >> k) & 1u) << d.tpos[r][k];
        const uint32_t slt = swz<F>(lt);
        uint32_t lj[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            uint32_t x = 0;
#pragma unroll
            for (int i = 0; i < RB; ++i)
                if ((j >> i) & 1) x |= 1u << d.gbits[r][i];
            lj[j] = x;
        }
        F2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = tile[slt ^ swz<F>(lj[j])];
        rotate_mask<RB>(v, d.maskA[r], cm1A, sA);
        if (r == d.phase_at) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const uint32_t e = (uint32_t)etile[lt | lj[j]];
                v[j] = cmul<F2, F>(v[j], lut[e]);
            }
        }
        rotate_mask<RB>(v, d.maskB[r], cm1B, sB);
#pragma unroll
        for (int j = 0; j < R; ++j) tile[slt ^ swz<F>(lj[j])] = v[j];
        __syncthreads();
    }

    F ss = F(0);
    {
        F2 v[R];
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int k = 0; k < VW; ++k) v[VW * i + k] = tile[swz<F>((uint32_t)(VW * (tid + i * WG) + k))];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
#pragma unroll
            for (int k = 0; k < VW; ++k) ss = fma(v[VW * i + k].x, v[VW * i + k].x, fma(v[VW * i + k].y, v[VW * i + k].y, ss));
            if constexpr (VW == 2) {
                float4 q;
                q.x = v[2 * i].x;
                q.y = v[2 * i].y;
                q.z = v[2 * i + 1].x;
                q.w = v[2 * i + 1].y;
                *reinterpret_cast<float4 *>(amp + goff[i]) = q;
            } else {
                amp[goff[i]] = v[i];
            }
        }
    }
    if (d.acc_out) {
        double t = (double)ss;
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        __shared__ double wsum[WG / 64];
        if ((tid & 63) == 0) wsum[tid >> 6] = t;
        __syncthreads();
        if (tid == 0) {
            double b = 0.0;
            for (int w = 0; w < (int)(WG / 64); ++w) b += wsum[w];
            atomicAdd(d.acc_out, (unsigned long long)(b * kNormFixedScale + 0.5));
        }
    }
}

// ---------------------------------------------------------------------------
// Whole state in one workgroup: all steps k0..k1-1 in LDS.  Workgroup b
// evolves state descs[b] (so one launch serves a batch of small states).
// ---------------------------------------------------------------------------
template <typename F, typename ET, int RB, int WB>
__device__ __forceinline__ void resident_body(const ResidentDesc &d)
{
    using F2 = typename V2<F>::T;
    constexpr int R = 1 << RB;
    constexpr uint32_t TS = 1u << (RB + WB);
    extern __shared__ __align__(16) unsigned char smem[];
    F2 *tile = reinterpret_cast<F2 *>(smem);
    F2 *lut = tile + TS;
    ET *etile = reinterpret_cast<ET *>(lut + lut_cap<ET>());

    F2 *__restrict__ amp = reinterpret_cast<F2 *>(d.amp);
    const ET *__restrict__ table = reinterpret_cast<const ET *>(d.table);
    const int n = d.n;
    const uint32_t dim = 1u << n;
    const uint32_t tid = threadIdx.x;
    const uint32_t nthr = 1u << d.thr_bits;
    const bool active = tid < nthr;
    const uint32_t used = (1u << d.reg_bits) - 1u;   // register-index bits in use

    for (uint32_t z = tid; z < dim; z += blockDim.x) {
        tile[swz<F>(z)] = amp[z];
        etile[z] = table[z];
    }

    const double T = d.T;
    const double Nd = (double)d.N;
    const double dt = T / Nd;
    __shared__ double red[1 << WB];
    __shared__ double norm_sh;
    double part = 0.0;     // this thread's share of |psi|^2 after the last residency
    // Norm of the state from the per-thread partials (fixed order).
    auto measure = [&]() {
        red[tid] = part;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (uint32_t k = 0; k < blockDim.x; ++k) t += red[k];
            norm_sh = t;
        }
        __syncthreads();
        return norm_sh;
    };
    auto build_lut = [&](double phi, double gph, double scale) {
        __syncthreads();
        for (int e = (int)tid; e <= d.emax; e += (int)blockDim.x) {
            double sn, cs;
            sincos(fma(phi, (double)e, gph), &sn, &cs);
            F2 L;
            L.x = (F)(scale * cs);
            L.y = (F)(-scale * sn);
            lut[e] = L;
        }
        __syncthreads();
    };
    auto residency = [&](int g, bool phase, uint32_t rmask, F cm1, F s, bool meas) {
        if (active) {
            uint32_t lt = 0;
            for (int k = 0; k < d.thr_bits; ++k) lt |= ((tid >> k) & 1u) << d.tpos[g][k];
            const uint32_t slt = swz<F>(lt);
            uint32_t lj[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                uint32_t x = 0;
#pragma unroll
                for (int i = 0; i < RB; ++i)
                    if (((j >> i) & 1) && i < d.reg_bits) x |= 1u << d.gbits[g][i];
                lj[j] = x;
            }
            F2 v[R];
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (((uint32_t)j & ~used) == 0) v[j] = tile[slt ^ swz<F>(lj[j])];
            if (phase) {
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if (((uint32_t)j & ~used) == 0) v[j] = cmul<F2, F>(v[j], lut[(uint32_t)etile[lt | lj[j]]]);
            }
            rotate_mask<RB>(v, rmask, cm1, s);
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

    double theta_prev = 0.0, s_prev = 0.0;
    for (int64_t k = d.k0; k < d.k1; ++k) {
        const double sk = ((double)k + 0.5) / Nd;
        const double theta = dt * (1.0 - sk);
        double phi, gph;
        if (k == d.k0) {
            phi = 0.5 * dt * sk;
            gph = 0.0;
        } else {
            phi = 0.5 * dt * (s_prev + sk);
            gph = fmod(0.5 * (double)n * theta_prev, 2.0 * M_PI);
        }
        const double scale = k == d.k0 ? 1.0 : rsqrt(measure());
        build_lut(phi, gph, scale);
        const double q = sin(0.25 * theta);
        const F cm1 = (F)(-2.0 * q * q);
        const F s = (F)sin(0.5 * theta);
        for (int g = 0; g < d.n_groups; ++g) residency(g, g == 0, d.gmask[g], cm1, s, g == d.n_groups - 1);
        theta_prev = theta;
        s_prev = sk;
    }
    if (d.k1 > d.k0) {
        const double scale = rsqrt(measure());
        build_lut(0.5 * dt * s_prev, fmod(0.5 * (double)n * theta_prev, 2.0 * M_PI), scale);
        residency(0, true, 0u, F(0), F(0), false);
    }
    for (uint32_t z = tid; z < dim; z += blockDim.x) amp[z] = tile[swz<F>(z)];
}

// One state, descriptor passed by value.
template <typename F, typename ET, int RB, int WB>
__global__ void __launch_bounds__(1 << WB) resident_one_kernel(const ResidentDesc d)
{
    resident_body<F, ET, RB, WB>(d);
}

// A batch of states, workgroup b takes descs[b].
template <typename F, typename ET, int RB, int WB>
__global__ void __launch_bounds__(1 << WB) resident_batch_kernel(const ResidentDesc *__restrict__ descs)
{
    resident_body<F, ET, RB, WB>(descs[blockIdx.x]);
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

template <typename F, typename ET, int TB, int RB>
hipError_t launch_pass_t(void *amp, const void *table, const PassDesc &d, hipStream_t s)
{
    using F2 = typename V2<F>::T;
    const size_t lds = sizeof(F2) * ((size_t(1) << TB) + lut_cap<ET>()) + sizeof(ET) * (size_t(1) << TB);
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&pass_kernel<F, ET, TB, RB>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    const unsigned grid = 1u << (d.n - TB);
    hipLaunchKernelGGL((pass_kernel<F, ET, TB, RB>), dim3(grid), dim3(1u << (TB - RB)), lds, s,
                       reinterpret_cast<F2 *>(amp), reinterpret_cast<const ET *>(table), d);
    return hipGetLastError();
}

template <typename F, typename ET, int RB, int WB>
hipError_t launch_resident_t(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, hipStream_t s)
{
    using F2 = typename V2<F>::T;
    const size_t lds = sizeof(F2) * ((size_t(1) << (RB + WB)) + lut_cap<ET>()) + sizeof(ET) * (size_t(1) << (RB + WB));
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&resident_one_kernel<F, ET, RB, WB>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&resident_batch_kernel<F, ET, RB, WB>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    if (one)
        hipLaunchKernelGGL((resident_one_kernel<F, ET, RB, WB>), dim3(1), dim3(1u << WB), lds, s, *one);
    else
        hipLaunchKernelGGL((resident_batch_kernel<F, ET, RB, WB>), dim3(count), dim3(1u << WB), lds, s, descs_dev);
    return hipGetLastError();
}

}  // namespace

// Tile shapes compiled into the library (planner picks among them).
//   complex64 : tile 2^13 = 8192 amps, 32 per thread, 256 threads
//   complex128: tile 2^12 = 4096 amps, 16 per thread, 256 threads
hipError_t launch_pass(void *amp, int dtype, const void *table, int etype, int tile_bits, int reg_bits,
                       const PassDesc &d, hipStream_t s)
{
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

hipError_t launch_resident(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, int dtype, int etype,
                           hipStream_t s)
{
    if (dtype == 0) {
        if (etype == 0) return launch_resident_t<float, uint8_t, 5, 8>(descs_dev, one, count, s);
        return launch_resident_t<float, uint16_t, 5, 8>(descs_dev, one, count, s);
    }
    if (etype == 0) return launch_resident_t<double, uint8_t, 4, 8>(descs_dev, one, count, s);
    return launch_resident_t<double, uint16_t, 4, 8>(descs_dev, one, count, s);
}

hipError_t launch_energy(const ClauseRec *cl, int m, int n, void *table, int etype, uint32_t *stats, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const uint64_t threads = (dim + 7) / 8;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    if (etype == 0)
        hipLaunchKernelGGL((energy_kernel<uint8_t>), dim3(grid), dim3(256), 0, s, cl, m, n,
                           reinterpret_cast<uint8_t *>(table), stats);
    else
        hipLaunchKernelGGL((energy_kernel<uint16_t>), dim3(grid), dim3(256), 0, s, cl, m, n,
                           reinterpret_cast<uint16_t *>(table), stats);
    return hipGetLastError();
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
