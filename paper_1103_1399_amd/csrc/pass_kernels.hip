// pass_kernels.hip -- the fused split-step passes of libqaa on gfx950: one
// HBM pass over 2^TB-amplitude tiles (pass_kernel, one state) and its
// lock-step batched form (batch_pass_kernel, many states), and their
// launchers.  See PassDesc (qaa_internal.h) for the tile and residency
// layout and kernel_common.h for the rotation arithmetic.
#include "qaa_internal.h"
#include <hip/hip_ext.h>
#include "kernel_common.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>

namespace qaa {
namespace {

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

// Add each wave's fixed-point norm share into its partial slot (wave g of
// the grid into slot g mod kNormPartials): no barrier, and a slot takes
// only the few shares of waves kNormPartials apart in the grid.
__device__ __forceinline__ void norm_accumulate_partials(unsigned long long *slots, unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const uint32_t waves = (blockDim.x + 63) >> 6;
    const uint32_t g = blockIdx.x * waves + (threadIdx.x >> 6);
    if ((threadIdx.x & 63) == 0) atomicAdd(slots + (g & (kNormPartials - 1)), v);
}

// Workgroup b < min(kNormReducers, grid) sums its share of the partial
// slots of the previous measuring pass, clears them for the next one, and
// adds the sum into *dst (the total the next phase pass reads).  Its first
// wave does it alone: no LDS (the pass kernels' LDS budget is exact) and
// no barrier.
__device__ __noinline__ void norm_reduce_partials(unsigned long long *src, unsigned long long *dst)
{
    if (threadIdx.x >= 64) return;
    const uint32_t nred = gridDim.x < (uint32_t)kNormReducers ? gridDim.x : (uint32_t)kNormReducers;
    const uint32_t chunk = ((uint32_t)kNormPartials + nred - 1) / nred;
    const uint32_t lo = blockIdx.x * chunk;
    const uint32_t hi = lo + chunk < (uint32_t)kNormPartials ? lo + chunk : (uint32_t)kNormPartials;
    unsigned long long v = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 64) {
        v += src[i];
        src[i] = 0ull;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (threadIdx.x == 0) atomicAdd(dst, v);
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
template <typename F, typename ET, int TB, int RB, bool PHASE, bool RECOMP>
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
    if constexpr (PHASE && !RECOMP) {
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

// LDS a recompute-mode workgroup gives its clause records: kPassClauses
// 16-byte slots, the last one holding the survivor counter.
constexpr int kPassClauses = 128;

// The energies of the tile at `base` into etile, recomputed from the clause
// records: thread tid scores the RUN consecutive tile-local indices
// tid*RUN .. tid*RUN + RUN - 1 (RUN = 32 for complex64, 16 for complex128:
// the tile's passenger bits), which are consecutive basis states z because
// the low tile bits are the low physical bits in every plan.
//
// Only clauses that some z of the tile violates are scored: the qubits
// outside the tile are fixed for the whole tile (its base), so a clause
// whose literal on such a qubit is satisfied there adds nothing to any
// count of the tile.  The records are read from the instance's list,
// kPassClauses - 1 at a time; the survivors of each batch go to cls (in
// whatever order the LDS atomic gives them: the counts do not depend on
// it) and are scored.  With 13 of 28 qubits in a tile, a random clause
// survives with probability (1 - 15/56)^3 = 0.39.
template <typename F, typename ET, int TB, int RB>
__device__ __forceinline__ void tile_energies(const PassDesc &d, uint64_t base, uint32_t tid, ET *etile,
                                              ClauseRec *cls)
{
    using P = PassTraits<F, ET, TB, RB>;
    constexpr int RUN = (int)(P::TS / P::WG);
    constexpr int LRUN = RUN == 32 ? 5 : 4;
    static_assert(RUN == (1 << LRUN), "one run of consecutive z per thread");
    static_assert((int)P::WG >= kPassClauses - 1, "one clause record per thread and batch");
    constexpr int K = sizeof(ET) == 1 ? 8 : 16;      // E <= 255 with a uint8 width, else <= 1023
    constexpr int kBatch = kPassClauses - 1;
    const uint32_t l0 = tid * (uint32_t)RUN;
    uint64_t off = 0;
#pragma unroll
    for (int j = LRUN; j < TB; ++j) off |= (uint64_t)((l0 >> j) & 1u) << d.tile_pos[j];
    const uint64_t z0 = base | off;
    const uint32_t t = (uint32_t)(z0 >> 5), lane0 = (uint32_t)(z0 & 31u);
    // index bits 5.. of z that stay fixed over the tile, and their values
    const uint32_t out_t = (uint32_t)(d.rest_mask >> 5), base_t = (uint32_t)(base >> 5);
    unsigned int *count = reinterpret_cast<unsigned int *>(cls + kBatch);
    BitCounter<K> bc;
    bc.clear();
    const int m = d.m;
    for (int c0 = 0; c0 < m; c0 += kBatch) {
        lds_barrier();                       // the previous batch is scored
        if (tid == 0) *count = 0u;
        lds_barrier();
        const int c = c0 + (int)tid;
        if ((int)tid < kBatch && c < m) {
            const ClauseRec r = d.clauses[c];
            if (((base_t ^ r.phi) & r.mhi & out_t) == 0u) cls[atomicAdd(count, 1u)] = r;
        }
        lds_barrier();
        score_clauses<K>(bc, cls, (int)*count, t);
    }
#pragma unroll
    for (int i = 0; i < RUN; ++i) etile[l0 + i] = (ET)count_of<K>(bc, lane0 + (uint32_t)i);
}

// Residencies of one tile, ending with the store to HBM.
template <typename F, typename ET, int TB, int RB, bool PHASE, bool RECOMP>
__device__ __forceinline__ void pass_compute(TileRegs<F, ET, TB, RB> &tr, typename V2<F>::T *__restrict__ amp,
                                             const PassDesc &d, uint64_t base,
                                             uint64_t tg_last, uint32_t tid,
                                             typename V2<F>::T *tile, const typename V2<F>::T *lut, ET *etile,
                                             ClauseRec *cls, const Rot<F> &kA, const Rot<F> &kB, bool meas,
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
    if constexpr (PHASE && RECOMP) {
        tile_energies<F, ET, TB, RB>(d, base, tid, etile, cls);
        lds_barrier();
    } else if constexpr (PHASE) {
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
    // measured 5 % faster.  Passes with a phase keep plain stores: in the
    // persistent kernel the hint's register constraints push it past 256
    // VGPRs, and in the other the streaming stores made the n = 28 set-0
    // passes 7 % slower (what they write is what the next pass, running in
    // the opposite direction, reads first from the last-level cache).
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
template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE, bool RECOMP = false>
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
    ClauseRec *cls = reinterpret_cast<ClauseRec *>(etile + P::TS);     // recompute mode only

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
    pass_load<F, ET, TB, RB, PHASE, RECOMP>(ta, amp, table, d, tile_at(w), tg_first, tid);

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
        pass_compute<F, ET, TB, RB, PHASE, RECOMP>(ta, amp, d, tile_at(w), tg_last, tid, tile, lut, etile,
                                                   cls, kA, kB, meas, ss);
    }
    while (PIPE) {
        const uint64_t w1 = w + stride;
        pass_load<F, ET, TB, RB, PHASE, RECOMP>(tb, amp, table, d, tile_at(w1 < end ? w1 : w), tg_first,
                                        tid);
        pass_compute<F, ET, TB, RB, PHASE, RECOMP>(ta, amp, d, tile_at(w), tg_last, tid, tile, lut, etile,
                                                   cls, kA, kB, meas, ss);
        if (w1 >= end) break;
        const uint64_t w2 = w1 + stride;
        pass_load<F, ET, TB, RB, PHASE, RECOMP>(ta, amp, table, d, tile_at(w2 < end ? w2 : w1), tg_first,
                                        tid);
        pass_compute<F, ET, TB, RB, PHASE, RECOMP>(tb, amp, d, tile_at(w1), tg_last, tid, tile, lut,
                                                   etile, cls, kA, kB, meas, ss);
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
// The hardware deals workgroups to the 8 XCDs round-robin (workgroup b
// runs on XCD b % 8).  xk >= 0 (the grid a power of two, at least
// 2^(xk + 3)): workgroup b takes the slot whose index bits xk .. xk + 2 are
// b % 8 and whose other bits are b / 8 in order, so that bits xk .. xk + 2
// of every tile number it handles name its XCD.  The planner picks xk so
// that those tile bits are the amplitude-index bits of byte-address bits
// 10..12: each XCD then works on its own eighth of memory, interleaved at
// 1 KiB, which streams fastest on MI355X (n = 28, 256-byte runs: 5.78
// against 5.31 TB/s for the plain order).
template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE, bool RECOMP>
__global__ void __launch_bounds__(1 << (TB - RB), (TB - RB) >= 9 ? 1 : 2)
pass_kernel(typename V2<F>::T *__restrict__ amp, const ET *__restrict__ table, const PassDesc d, int32_t xk)
{
    if (d.acc_zero && blockIdx.x == 0 && threadIdx.x == 0) *d.acc_zero = 0ull;
    if (d.red_dst && blockIdx.x < (uint32_t)kNormReducers) norm_reduce_partials(d.red_src, d.red_dst);
    uint32_t slot = blockIdx.x;
    if (xk >= 0) {
        const uint32_t r = slot >> 3;
        slot = (r & ((1u << xk) - 1u)) | ((slot & 7u) << xk) | ((r >> xk) << (xk + 3));
    }
    const uint64_t first = d.tile_begin + slot;           // grid size <= tile_count
    const unsigned long long ss = tile_loop<F, ET, TB, RB, PHASE, PIPE, RECOMP>(
        amp, table, d, first, gridDim.x, d.tile_begin + d.tile_count, d.phi, d.gphase, d.emax, d.acc_in,
        make_rot<F>(d.tA, d.sA), make_rot<F>(d.tB, d.sB), d.acc_out != nullptr);
    if (d.acc_out) norm_accumulate_partials(d.acc_out, ss);
}

// ---------------------------------------------------------------------------
// Batched passes (see BatchInst).
// ---------------------------------------------------------------------------
// Workgroup b takes a chunk of up to chunk_tiles consecutive tiles of state
// chunk_inst[b] (pipelined like pass_kernel); the pass kind, the rotation
// and phase coefficients follow from the global step s, the pass index j
// and the state's own schedule.
template <typename F, typename ET, int TB, int RB>
__global__ void __launch_bounds__(1 << (TB - RB), (TB - RB) >= 9 ? 1 : 2)
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
    const uint64_t w0 = (g - I.chunk_offset[TB == kWideTileBits ? 1 : 0]) * (uint64_t)chunk_tiles;
    if (w0 >= ntiles) return;       // (the host's chunk tables never ask for this)
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

// Slot arrangement of a pass grid (see pass_kernel): PassDesc::xcd_map 0
// leaves the plain order, 1 puts the XCD on the grid's top three bits (one
// contiguous range of tiles per XCD), 2 + k on tile-number bits k .. k + 2.
// QAA_XCD_MAP=0 keeps the plain order everywhere (a tuning switch; results
// do not depend on it).
inline int xcd_bit(const PassDesc &d, unsigned grid)
{
    static const bool off = [] {
        const char *e = std::getenv("QAA_XCD_MAP");
        return e && std::atoi(e) == 0;
    }();
    if (off || d.xcd_map <= 0 || grid < 8 || (grid & (grid - 1))) return -1;
    int lg = 0;
    while ((1u << lg) < grid) ++lg;
    const int k = d.xcd_map == 1 ? lg - 3 : d.xcd_map - 2;
    return k + 3 <= lg ? k : lg - 3;
}

template <typename F, typename ET, int TB, int RB, bool PHASE, bool PIPE, bool RECOMP>
hipError_t launch_pass_p(void *amp, const void *table, const PassDesc &d, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1)
{
    using F2 = typename V2<F>::T;
    constexpr int DT = sizeof(F) == 4 ? 0 : 1;
    constexpr size_t TS = size_t(1) << TB;
    const size_t lds = sizeof(F2) * (TS + kPadN[DT] * (TS >> kPadS[DT]) + lut_cap<ET>()) + sizeof(ET) * TS +
                       (RECOMP ? sizeof(ClauseRec) * kPassClauses : 0);
    const void *fn = reinterpret_cast<const void *>(&pass_kernel<F, ET, TB, RB, PHASE, PIPE, RECOMP>);
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
    // profiling: the start and stop events ride on the dispatch itself
    // (no separate event-record commands between the passes)
    if (ev0)
        hipExtLaunchKernelGGL((pass_kernel<F, ET, TB, RB, PHASE, PIPE, RECOMP>), dim3(grid), dim3(1u << (TB - RB)),
                              (std::uint32_t)lds, s, ev0, ev1, 0u, reinterpret_cast<F2 *>(amp),
                              reinterpret_cast<const ET *>(table), d, xcd_bit(d, grid));
    else
        hipLaunchKernelGGL((pass_kernel<F, ET, TB, RB, PHASE, PIPE, RECOMP>), dim3(grid), dim3(1u << (TB - RB)), lds,
                           s, reinterpret_cast<F2 *>(amp), reinterpret_cast<const ET *>(table), d, xcd_bit(d, grid));
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
hipError_t launch_pass_v(void *amp, const void *table, const PassDesc &d, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1)
{
    // recompute mode (no table): passes with a phase score their tiles'
    // energies from the clause records
    if (PHASE && !table) {
        if constexpr (PHASE) {
            // (the persistent form would spill registers with 16-bit energies)
            const int v = pass_variant();
            if (sizeof(ET) == 2 || v == 0 || (v < 0 && !d.persist))
                return launch_pass_p<F, ET, TB, RB, true, false, true>(amp, table, d, s, ev0, ev1);
            if constexpr (sizeof(ET) == 1) return launch_pass_p<F, ET, TB, RB, true, true, true>(amp, table, d, s, ev0, ev1);
        }
    }
    const int v = pass_variant();
    if (v == 0 || (v < 0 && !d.persist)) return launch_pass_p<F, ET, TB, RB, PHASE, false, false>(amp, table, d, s, ev0, ev1);
    return launch_pass_p<F, ET, TB, RB, PHASE, true, false>(amp, table, d, s, ev0, ev1);
}

template <typename F, typename ET, int TB, int RB>
hipError_t launch_pass_t(void *amp, const void *table, const PassDesc &d, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1)
{
    if (d.phase_at >= 0) return launch_pass_v<F, ET, TB, RB, true>(amp, table, d, s, ev0, ev1);
    return launch_pass_v<F, ET, TB, RB, false>(amp, table, d, s, ev0, ev1);
}

}  // namespace

// Tile shapes compiled into the library (planner picks among them).
//   complex64 : tile 2^13 = 8192 amps, 32 per thread, 256 threads;
//               tile 2^14 = 16384 amps, 32 per thread, 512 threads (uint8 table)
//   complex128: tile 2^12 = 4096 amps, 16 per thread, 256 threads
hipError_t launch_pass(void *amp, int dtype, const void *table, int etype, int tile_bits, int reg_bits,
                       const PassDesc &d, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    // 2^14-amplitude tiles: complex64 with a uint8 table only (LDS)
    if (dtype == 0 && tile_bits == kWideTileBits && reg_bits == 5 && etype == 0)
        return launch_pass_t<float, uint8_t, kWideTileBits, 5>(amp, table, d, s, ev0, ev1);
    if (dtype == 0 && tile_bits == 13 && reg_bits == 5) {
        if (etype == 0) return launch_pass_t<float, uint8_t, 13, 5>(amp, table, d, s, ev0, ev1);
        return launch_pass_t<float, uint16_t, 13, 5>(amp, table, d, s, ev0, ev1);
    }
    if (dtype == 0 && tile_bits == 13 && reg_bits == kSmallPlanRegBits) {
        if (etype == 0) return launch_pass_t<float, uint8_t, 13, kSmallPlanRegBits>(amp, table, d, s, ev0, ev1);
        return launch_pass_t<float, uint16_t, 13, kSmallPlanRegBits>(amp, table, d, s, ev0, ev1);
    }
    if (dtype == 1 && tile_bits == 12 && reg_bits == 4) {
        if (etype == 0) return launch_pass_t<double, uint8_t, 12, 4>(amp, table, d, s, ev0, ev1);
        return launch_pass_t<double, uint16_t, 12, 4>(amp, table, d, s, ev0, ev1);
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
    if (dtype == 0 && tile_bits == kWideTileBits && reg_bits == 5 && etype == 0)
        return launch_batch_t<float, uint8_t, kWideTileBits, 5>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles,
                                                                 st);
    if (dtype == 0 && tile_bits == 13 && reg_bits == 5) {
        if (etype == 0)
            return launch_batch_t<float, uint8_t, 13, 5>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
        return launch_batch_t<float, uint16_t, 13, 5>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
    }
    if (dtype == 0 && tile_bits == 13 && reg_bits == kSmallPlanRegBits) {
        if (etype == 0)
            return launch_batch_t<float, uint8_t, 13, kSmallPlanRegBits>(insts, chunk_inst, chunks, structs, s, j,
                                                                          chunk_tiles, st);
        return launch_batch_t<float, uint16_t, 13, kSmallPlanRegBits>(insts, chunk_inst, chunks, structs, s, j,
                                                                       chunk_tiles, st);
    }
    if (dtype == 1 && tile_bits == 12 && reg_bits == 4) {
        if (etype == 0)
            return launch_batch_t<double, uint8_t, 12, 4>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
        return launch_batch_t<double, uint16_t, 12, 4>(insts, chunk_inst, chunks, structs, s, j, chunk_tiles, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace qaa
