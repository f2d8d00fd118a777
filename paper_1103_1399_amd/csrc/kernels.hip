// kernels.hip -- gfx950 kernels of libqaa other than the fused passes
// (pass_kernels.hip): the energy table, state initialisation, the
// LDS-resident small-state evolution, and the FP64 observables reduction.
// Rotation arithmetic and schedule coefficients: kernel_common.h.
#include "qaa_internal.h"
#include "kernel_common.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>

namespace qaa {
namespace {

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

constexpr int kClauseChunk = 1024;     // clause records staged in LDS at a time (16 KiB)

// stats: [0] ~E_min (maximum of complements), [1] E_max, [2] some E > 255
// with a uint8 table, [3] some count passed the K planes (recompute wider).
// table == nullptr: statistics only (no table is written).  count != nullptr:
// also add the number of z with E(z) == count_value into *count.
template <typename ET, int K>
__global__ void __launch_bounds__(256) energy_kernel(const ClauseRec *__restrict__ cl, int m, int n,
                                                     ET *__restrict__ table, uint32_t *__restrict__ stats,
                                                     uint32_t count_value, unsigned long long *__restrict__ count)
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
    uint32_t lo = 0xFFFFFFFFu, hi = 0u, over = 0u, wide = 0u, hits = 0u;
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
                hits += e[i] == count_value ? 1u : 0u;
            }
        }
        if (!table) {
            if (sizeof(ET) == 1) over = hi > 255u ? 1u : 0u;
        } else if (cnt == 32) {
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
    __shared__ unsigned long long red_hits[4];
    const int wave = (int)(threadIdx.x >> 6);
    unsigned long long h = hits;
    for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = ~lo;      // stats[0] holds ~E_min (the maximum of the
        red[wave][1] = hi;       // complements), so that a zero-filled block
        red[wave][2] = over;     // is the neutral start for all of them
        red[wave][3] = wide;
        red_hits[wave] = h;
    }
    __syncthreads();
    if (count && threadIdx.x == 4) {
        unsigned long long c = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) c += red_hits[w];
        if (c) atomicAdd(count, c);
    }
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

// Phase angle phi_k, global phase and rotation coefficients (rt, rs) of
// step k of a range that opens at k0: the half phase that opens the range
// (k == k0), else the merged halves of k-1 and k with step k-1's driver
// global phase.
__device__ __forceinline__ void res_step_terms(const double *knots, int kcount, int64_t k, int64_t k0, int64_t N,
                                               double dt, int n, double &phi, double &gph, double &rt, double &rs)
{
    const double sk = sched_mid(knots, kcount, k, N);
    bool flip;
    rot_params(dt * (1.0 - sk), rt, rs, flip);
    if (k == k0) {
        phi = 0.5 * dt * sk;
        gph = 0.0;
    } else {
        const double sp = sched_mid(knots, kcount, k - 1, N);
        const double thp = dt * (1.0 - sp);
        double tp, sq;
        bool fp;
        rot_params(thp, tp, sq, fp);
        phi = 0.5 * dt * (sp + sk);
        gph = step_gphase(n, thp, fp);
    }
}

// Rows [0, rows) of a chunk's phase table, row j entry e =
// exp(-i (phi_j e + gph_j)) in FP64 rounded once; row 0 carries the norm
// correction scale0.  Threads tid = 0..nthr-1 share the entries.
template <typename F2, typename F>
__device__ __forceinline__ void res_build_rows(F2 *ring, const double *phi_s, const double *gph_s, int rows,
                                               int width, double scale0, int tid, int nthr)
{
    for (int x = tid; x < rows * width; x += nthr) {
        const int j = x / width, e = x - j * width;
        double sn, cs;
        sincos(fma(phi_s[j], (double)e, gph_s[j]), &sn, &cs);
        const double sc = j == 0 ? scale0 : 1.0;
        F2 L;
        L.x = (F)(sc * cs);
        L.y = (F)(-sc * sn);
        ring[x] = L;
    }
}

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
        if (table) etile[z] = table[z];
    }
    if (!table) {
        // recompute mode: score the state's energies once, 32 z per thread
        constexpr int K = sizeof(ET) == 1 ? 8 : 16;
        const uint32_t blocks = (dim + 31u) / 32u;
        for (uint32_t b = tid; b < blocks; b += blockDim.x) {
            BitCounter<K> bc;
            bc.clear();
            score_clauses<K>(bc, d.clauses, d.m, b);
            const uint32_t cnt = dim < 32u ? dim : 32u;
            for (uint32_t i = 0; i < cnt; ++i) etile[32u * b + i] = (ET)count_of<K>(bc, i);
        }
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
    auto step_terms = [&](int64_t k, double &phi, double &gph, double &rt, double &rs) {
        res_step_terms(knots_s, kcount, k, d.k0, d.N, dt, n, phi, gph, rt, rs);
    };
    auto build_rows = [&](int rows, double scale0) {
        res_build_rows<F2, F>(ring, phi_s, gph_s, rows, width, scale0, (int)tid, (int)blockDim.x);
    };
    // Few registers per thread (a single state of up to 2^11 amplitudes: 4
    // per thread, at most 512 threads): every group's LDS offsets and the
    // phase group's energies are kept in registers for the whole run, so a
    // residency starts with its tile loads instead of a chain of index
    // loads.  (With 1024 threads the register budget is 128 and these maps
    // would spill; batches hold 16 or 32 amplitudes per thread.  Both read
    // the offsets from LDS.)
    constexpr bool kRegMaps = R <= 4 && WB <= 9;
    constexpr int kG = kRegMaps ? 8 : 1;
    uint32_t slt_r[kG], off_r[kG][kRegMaps ? R : 1];
    uint32_t e0_r[kRegMaps ? R : 1];
    if constexpr (kRegMaps) {
        __syncthreads();          // lt_s / lj_s written
#pragma unroll
        for (int g = 0; g < kG; ++g) {
            const uint32_t lt = g < d.n_groups ? lt_s[g][tid] : 0u;
            slt_r[g] = swz<F>(lt);
#pragma unroll
            for (int j = 0; j < R; ++j) off_r[g][j] = g < d.n_groups ? swz<F>(lj_s[g][j]) : 0u;
        }
        const uint32_t lt0 = lt_s[0][tid];
#pragma unroll
        for (int j = 0; j < R; ++j) e0_r[j] = ((uint32_t)j & ~used) == 0 && active ? (uint32_t)etile[lt0 | lj_s[0][j]] : 0u;
    }
    auto residency = [&](int g, const F2 *lut, uint32_t rmask, const Rot<F> &k, bool meas) {
        if (active) {
            F2 v[R];
            if constexpr (kRegMaps) {
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if (((uint32_t)j & ~used) == 0) v[j] = tile[slt_r[g] ^ off_r[g][j]];
                if (lut) {     // the phase is applied in group 0 only
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        if (((uint32_t)j & ~used) == 0) v[j] = cmul<F2, F>(v[j], lut[e0_r[j]]);
                }
                rotate_mask<RB>(v, rmask, k);
                F ss = F(0);
#pragma unroll
                for (int j = 0; j < R; ++j)
                    if (((uint32_t)j & ~used) == 0) {
                        tile[slt_r[g] ^ off_r[g][j]] = v[j];
                        ss = fma(v[j].x, v[j].x, fma(v[j].y, v[j].y, ss));
                    }
                if (meas) part = (double)ss;
            } else {
                const uint32_t lt = lt_s[g][tid];
                const uint32_t slt = swz<F>(lt);
                uint32_t lj[R];
#pragma unroll
                for (int j = 0; j < R; ++j) lj[j] = lj_s[g][j];
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
        }
        __syncthreads();
    };
    // every group of one step (unrolled, so register-held maps stay in
    // registers)
    auto step_groups = [&](const F2 *lut, const Rot<F> &rk, bool meas_last) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            if (g < d.n_groups)
                residency(g, g == 0 ? lut : nullptr, gm_s[g], rk, meas_last && g == d.n_groups - 1);
        }
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
        for (int j = 0; j < cs; ++j) step_groups(ring + j * width, rot_s[j], j == cs - 1);
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
// One complex64 state of n = RB + 6 + WV qubits (n = 8..12) held in
// registers: 2^RB amplitudes per thread, 64 << WV threads.  Layout A puts
// qubits 0..RB-1 in the register index, qubits RB..RB+5 in the lane index
// and the top WV qubits in the wave index; layout B swaps the lowest WV
// register bits with the wave bits.  A step applies its phase row and then
// rotates every qubit: those in register bits inside the thread, those in
// lane bits with the partner lane's value (cross-lane shuffles; each lane
// keeps its own half of the pair, with the same three-shear arithmetic as
// rotate_bit), and the wave qubits after one exchange through LDS into the
// other layout.  Steps alternate the layout they start in, so a step costs
// one exchange (none at n = 8) and one barrier, instead of an LDS
// residency with a barrier per pair of qubits.  Coefficients, phase rows
// and the once-per-chunk renormalisation are as in resident_body.
// ---------------------------------------------------------------------------
// The value of lane l ^ (1 << B) of the wave.  Within a row of 16 lanes the
// exchange is a DPP move (no trip through the LDS crossbar): quad_perm
// [1,0,3,2] and [2,3,0,1] swap lanes 1 and 2 apart; a half-row mirror
// (l ^ 7 within 8) followed by a quad reversal (l ^ 3) gives l ^ 4; a row
// mirror (l ^ 15 within 16) followed by a half-row mirror gives l ^ 8.
// Lanes 16 and 32 apart go through ds_bpermute.
template <int B>
__device__ __forceinline__ float lane_xor(float x)
{
    const int v = __float_as_int(x);
    if constexpr (B == 0) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true));
    } else if constexpr (B == 1) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true));
    } else if constexpr (B == 2) {
        const int t = __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);
        return __int_as_float(__builtin_amdgcn_update_dpp(0, t, 0x1B, 0xF, 0xF, true));
    } else if constexpr (B == 3) {
        const int t = __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);
        return __int_as_float(__builtin_amdgcn_update_dpp(0, t, 0x141, 0xF, 0xF, true));
    } else {
        return __shfl_xor(x, 1 << B, 64);
    }
}

template <int B, int RB, typename F>
__device__ __forceinline__ void rotate_lane_bit(float2 (&v)[1 << RB], const Rot<F> &k)
{
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        const float px = lane_xor<B>(v[j].x);
        const float py = lane_xor<B>(v[j].y);
        // (Re mine, Im partner) and (Re partner, Im mine) are the two
        // sheared planes; this lane keeps Re mine and Im mine
        const float a = fma(-k.t, py, v[j].x);
        const float w = fma(k.s, a, py);
        const float c = fma(-k.t, v[j].y, px);
        v[j].x = fma(-k.t, w, a);
        v[j].y = fma(k.s, c, v[j].y);
    }
}

template <int RB, typename F>
__device__ __forceinline__ void rotate_lanes(float2 (&v)[1 << RB], const Rot<F> &k)
{
    rotate_lane_bit<0, RB>(v, k);
    rotate_lane_bit<1, RB>(v, k);
    rotate_lane_bit<2, RB>(v, k);
    rotate_lane_bit<3, RB>(v, k);
    rotate_lane_bit<4, RB>(v, k);
    rotate_lane_bit<5, RB>(v, k);
}

template <typename ET, int RB, int WV>
__global__ void __launch_bounds__(64 << WV) resident_lane_kernel(const ResidentDesc d)
{
    using F = float;
    using F2 = float2;
    constexpr int R = 1 << RB;
    constexpr uint32_t NT = 64u << WV;
    constexpr uint32_t DIM = (uint32_t)R * NT;
    constexpr uint32_t LO = (1u << WV) - 1u;
    static_assert(WV <= RB, "the wave bits swap with register bits");
    extern __shared__ __align__(16) unsigned char smem[];
    F2 *xbuf = reinterpret_cast<F2 *>(smem);             // two exchange buffers of DIM entries
    F2 *ring = xbuf + 2 * DIM;                           // phase rows
    ET *etile = reinterpret_cast<ET *>(ring + kResRingOne);   // recompute mode: energies

    F2 *__restrict__ amp = reinterpret_cast<F2 *>(d.amp);
    const ET *__restrict__ table = reinterpret_cast<const ET *>(d.table);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    auto zA = [&](uint32_t j) { return j | (lane << RB) | (wave << (RB + 6)); };
    auto zB = [&](uint32_t j) { return wave | (j & ~LO) | (lane << RB) | ((j & LO) << (RB + 6)); };

    __shared__ double knots_s[kMaxKnots];
    const int kcount = d.sched.count;
    for (int x = (int)tid; x < kcount; x += (int)NT) knots_s[x] = d.sched.v[x];
    if (!table) {
        // recompute mode: score the state's energies once, 32 z per thread
        constexpr int K = sizeof(ET) == 1 ? 8 : 16;
        for (uint32_t b = tid; b < DIM / 32u; b += NT) {
            BitCounter<K> bc;
            bc.clear();
            score_clauses<K>(bc, d.clauses, d.m, b);
            for (uint32_t i = 0; i < 32u; ++i) etile[32u * b + i] = (ET)count_of<K>(bc, i);
        }
        __syncthreads();
    }
    F2 v[R];
    uint32_t eA[R], eB[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        v[j] = amp[zA(j)];
        eA[j] = table ? (uint32_t)table[zA(j)] : (uint32_t)etile[zA(j)];
        eB[j] = table ? (uint32_t)table[zB(j)] : (uint32_t)etile[zB(j)];
    }

    const double dt = d.T / (double)d.N;
    const int width = d.emax + 1;
    const int chunk = min(kResChunk, kResRingOne / width);
    __shared__ double red[NT / 64];
    __shared__ double phi_s[kResChunk], gph_s[kResChunk];
    __shared__ Rot<F> rot_s[kResChunk];
    bool inA = true;          // layout the state is in
    int buf = 0;              // exchange buffer written next
    auto phase = [&](const F2 *lut) {
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = cmul<F2, F>(v[j], lut[inA ? eA[j] : eB[j]]);
    };
    auto rotA = [&](const Rot<F> &k) {
        rotate_mask<RB>(v, (1u << RB) - 1u, k);
        rotate_lanes<RB>(v, k);
    };
    auto rotB = [&](const Rot<F> &k) {
#pragma unroll
        for (int b = 0; b < WV; ++b) rotate_bit<RB>(v, b, k);
    };
    // to the other layout through LDS; two buffers in turn, so one barrier
    // per exchange (a buffer is rewritten only after every thread has
    // passed the next exchange's barrier, i.e. finished reading it)
    auto exchange = [&]() {
        F2 *x = xbuf + buf * DIM;
#pragma unroll
        for (int j = 0; j < R; ++j) x[swz<F>(inA ? zA(j) : zB(j))] = v[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = x[swz<F>(inA ? zB(j) : zA(j))];
        inA = !inA;
        buf ^= 1;
    };
    auto step = [&](const F2 *lut, const Rot<F> &k) {
        phase(lut);
        if constexpr (WV == 0) {
            rotA(k);
        } else if (inA) {
            rotA(k);
            exchange();
            rotB(k);
        } else {
            rotB(k);
            exchange();
            rotA(k);
        }
    };
    auto measure = [&]() {
        F ss = F(0);
#pragma unroll
        for (int j = 0; j < R; ++j) ss = fma(v[j].x, v[j].x, fma(v[j].y, v[j].y, ss));
        double t = (double)ss;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if (lane == 0) red[wave] = t;
        __syncthreads();
        double total = 0.0;
#pragma unroll
        for (int w = 0; w < (int)(NT / 64); ++w) total += red[w];
        return total;
    };

    double scale = 1.0;
    for (int64_t kc = d.k0; kc < d.k1; kc += chunk) {
        const int cs = (int)min<int64_t>((int64_t)chunk, d.k1 - kc);
        __syncthreads();         // knots loaded / the previous chunk's rows and norm read
        if ((int)tid < cs) {
            double phi, gph, rt, rs;
            res_step_terms(knots_s, kcount, kc + (int)tid, d.k0, d.N, dt, d.n, phi, gph, rt, rs);
            phi_s[tid] = phi;
            gph_s[tid] = gph;
            rot_s[tid] = make_rot<F>(rt, rs);
        }
        __syncthreads();
        res_build_rows<F2, F>(ring, phi_s, gph_s, cs, width, scale, (int)tid, (int)NT);
        __syncthreads();
        for (int j = 0; j < cs; ++j) step(ring + j * width, rot_s[j]);
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
            gph_s[0] = step_gphase(d.n, thl, fl);
        }
        __syncthreads();
        res_build_rows<F2, F>(ring, phi_s, gph_s, 1, width, scale, (int)tid, (int)NT);
        __syncthreads();
        phase(ring);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) amp[inA ? zA(j) : zB(j)] = v[j];
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

// Recompute mode (no table): thread blocks of 32 consecutive z, each scored
// against the clause records (staged in LDS when they fit), then summed as
// obs_partial_kernel does.
template <typename F, int K>
__global__ void __launch_bounds__(256) obs_recompute_kernel(const typename V2<F>::T *__restrict__ amp, int n,
                                                            const ClauseRec *__restrict__ cl, int m, uint32_t emin,
                                                            double *__restrict__ partials)
{
    __shared__ ClauseRec cl_s[kClauseChunk];
    const bool staged = m <= kClauseChunk;
    if (staged)
        for (int i = (int)threadIdx.x; i < m; i += (int)blockDim.x) cl_s[i] = cl[i];
    __syncthreads();
    const ClauseRec *src = staged ? cl_s : cl;
    const uint64_t dim = 1ull << n;
    const uint64_t blocks = (dim + 31) / 32;
    const uint32_t cnt = dim < 32 ? (uint32_t)dim : 32u;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < blocks; b += stride) {
        BitCounter<K> bc;
        bc.clear();
        score_clauses<K>(bc, src, m, (uint32_t)b);
        for (uint32_t i = 0; i < cnt; ++i) {
            const typename V2<F>::T v = amp[32 * b + i];
            const double p = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            const uint32_t e = count_of<K>(bc, i);
            a0 += p;
            a1 += (double)e * p;
            a2 += e == emin ? p : 0.0;
        }
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

// A single complex64 state of n = 8..12 runs resident_lane_kernel instead
// of the LDS-resident kernel (QAA_RESIDENT_LANES=0 turns it off; results
// differ by rounding only).
constexpr int kResLaneMinN = 8;
constexpr int kResLaneMaxN = 12;

static bool resident_lanes_enabled()
{
    static const bool on = [] {
        const char *e = std::getenv("QAA_RESIDENT_LANES");
        return !(e && std::atoi(e) == 0);
    }();
    return on;
}

template <typename ET, int RB, int WV>
hipError_t launch_resident_lane_t(const ResidentDesc &one, hipStream_t s)
{
    constexpr size_t DIM = size_t(1) << (RB + 6 + WV);
    const size_t lds = sizeof(float2) * (2 * DIM + kResRingOne) + sizeof(ET) * DIM;
    const void *fn = reinterpret_cast<const void *>(&resident_lane_kernel<ET, RB, WV>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((resident_lane_kernel<ET, RB, WV>), dim3(1), dim3(64u << WV), lds, s, one);
    return hipGetLastError();
}

template <typename ET>
hipError_t launch_resident_lane(const ResidentDesc &one, hipStream_t s)
{
    switch (one.n) {
    case 8: return launch_resident_lane_t<ET, 2, 0>(one, s);
    case 9: return launch_resident_lane_t<ET, 2, 1>(one, s);
    case 10: return launch_resident_lane_t<ET, 2, 2>(one, s);
    case 11: return launch_resident_lane_t<ET, 3, 2>(one, s);
    case 12: return launch_resident_lane_t<ET, 3, 3>(one, s);
    default: return hipErrorInvalidValue;
    }
}

// Single-state shapes (see resident_shape): 2^(rb + wb) amplitudes.
template <typename F, typename ET>
hipError_t launch_resident_one(const ResidentDesc *one, int rb, int wb, hipStream_t s)
{
    if constexpr (sizeof(F) == 4)
        if (resident_lanes_enabled() && one->n >= kResLaneMinN && one->n <= kResLaneMaxN)
            return launch_resident_lane<ET>(*one, s);
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
                         int count_value, unsigned long long *count, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    const uint64_t threads = (dim + 31) / 32;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    const uint32_t cv = (uint32_t)count_value;
    if (etype == 0) {
        if (!wide)
            hipLaunchKernelGGL((energy_kernel<uint8_t, 8>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint8_t *>(table), stats, cv, count);
        else
            hipLaunchKernelGGL((energy_kernel<uint8_t, 16>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint8_t *>(table), stats, cv, count);
    } else {
        if (!wide)
            hipLaunchKernelGGL((energy_kernel<uint16_t, 8>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint16_t *>(table), stats, cv, count);
        else
            hipLaunchKernelGGL((energy_kernel<uint16_t, 16>), dim3(grid), dim3(256), 0, s, cl, m, n,
                               reinterpret_cast<uint16_t *>(table), stats, cv, count);
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

hipError_t launch_observables(const void *amp, int dtype, const void *table, int etype, const ClauseRec *clauses,
                              int m, int n, int emin, double *partials, int nblocks, double *out, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    if (!table) {
        const bool narrow = etype == 0;      // counts fit 8 planes when E_max <= 255
        if (dtype == 0) {
            if (narrow)
                hipLaunchKernelGGL((obs_recompute_kernel<float, 8>), dim3(nblocks), dim3(256), 0, s,
                                   reinterpret_cast<const float2 *>(amp), n, clauses, m, (uint32_t)emin, partials);
            else
                hipLaunchKernelGGL((obs_recompute_kernel<float, 16>), dim3(nblocks), dim3(256), 0, s,
                                   reinterpret_cast<const float2 *>(amp), n, clauses, m, (uint32_t)emin, partials);
        } else {
            if (narrow)
                hipLaunchKernelGGL((obs_recompute_kernel<double, 8>), dim3(nblocks), dim3(256), 0, s,
                                   reinterpret_cast<const double2 *>(amp), n, clauses, m, (uint32_t)emin, partials);
            else
                hipLaunchKernelGGL((obs_recompute_kernel<double, 16>), dim3(nblocks), dim3(256), 0, s,
                                   reinterpret_cast<const double2 *>(amp), n, clauses, m, (uint32_t)emin, partials);
        }
    } else if (dtype == 0) {
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
