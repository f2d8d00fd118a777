// qaa_internal.h -- structures shared by the host runtime and the gfx950
// kernels of libqaa.  Not part of the public ABI (include/qaa.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "qaa.h"

namespace qaa {

// Largest number of register-group residencies in one pass (see PassDesc).
constexpr int kMaxRes = 12;
// Phase lookup table capacity: E in [0, kLutMax).
constexpr int kLutMax = 1024;
constexpr int kLutMaxU8 = 256;

// Interpolation schedule as the kernels and the host planner consume it:
// count == 0 is the linear s(u) = u; otherwise v[0..count) are the knots of
// a piecewise-linear s(u) at u_j = j/(count - 1) (see qaa_schedule).
constexpr int kMaxKnots = QAA_SCHED_MAX_KNOTS;
struct SchedKnots {
    int32_t count;
    int32_t pad_;
    double v[kMaxKnots];
};

// s at the midpoint u_k = (k + 1/2)/N of step k.  Host and device evaluate
// this same expression (the product and the quotient are correctly rounded
// and the interpolation is one explicit fma), so a state gets the same s_k
// whether its coefficients are made on the host or on the device.  With
// the knots {0, 1} it returns exactly (k + 1/2)/N, the linear schedule.
__host__ __device__ inline double sched_mid(const double *v, int count, int64_t k, int64_t N)
{
    if (count < 2) return ((double)k + 0.5) / (double)N;
    const double x = ((double)k + 0.5) * (double)(count - 1) / (double)N;
    int j = (int)x;                      // x >= 0: truncation is floor
    if (j > count - 2) j = count - 2;
    return fma(x - (double)j, v[j + 1] - v[j], v[j]);
}

// One clause in the form the energy kernel consumes.  A clause over three
// distinct variables is violated by z iff (z & mask) == pat, where mask has
// the clause's three variable bits and pat has the bits of the negated
// literals.  The kernel scores 32 consecutive z at once, so the test splits
// at bit 5: the high part ((z >> 5) & mhi) == phi is one compare for all 32,
// and bit i of `low` is the outcome of the low part for z & 31 == i.
struct ClauseRec {
    uint32_t mhi, phi;     // mask / pattern bits >= 5, shifted down by 5
    uint32_t low;          // bit i: (i & mask) == (pat & mask & 31), i = 0..31
    uint32_t pad_;
};

// One HBM pass of the split-step evolution over tiles of 2^TB amplitudes.
//
// A tile is the set of basis states that agree on all bits outside
// tile_pos[0..TB): tile-local index l (TB bits) maps to the physical index
// by placing bit j of l at bit tile_pos[j]; the workgroup id is spread over
// rest_pos[0..n_rest) the same way.  The tile is processed in a sequence of
// "residencies".  In residency r every thread holds 2^RB amplitudes in
// registers: register index j and thread index t address tile-local index
//     l = lt_r(t) | lj_r(j),   lt_r(t) = sum_k bit_k(t) << tpos[r][k],
// where lj_r(j) places the register bits on the residency's register group.
// Residency 0 loads its registers from HBM and the last residency stores
// them to HBM (goff_*/gpos_* give those global offsets); in between, the
// tile passes through LDS (padded index, ljp = padded lj).  Each residency:
//   1. rotations on the register bits in maskA (masks[r] & 0xff) with
//      coefficient set A,
//   2. if r == phase_at: the diagonal phase exp(-i (phi E + gphase)),
//   3. rotations on the register bits in maskB (masks[r] >> 8) with
//      coefficient set B.
// A rotation is the single-qubit factor of exp(-i theta H_B) without its
// global phase: [[c, i s], [i s, c]], c = cos(theta/2), s = sin(theta/2),
// applied in place as three shears, given as t = tan(theta/4) and s (the
// host reduces theta/2 to [-pi/2, pi/2]; the sign flip of the reduction
// goes into the global phase).
// The global phase exp(-i n theta / 2) of each step is folded into gphase.
// The kernel reads the per-residency tables as whole 32-bit words so that
// they come through the scalar cache (a sub-word load at a run-time index
// would be a vector memory load, and waiting for it would also wait for the
// HBM prefetch of the next tile).
// For complex64, register bit 0 is always tile bit 0 (= physical bit 0), so
// register pairs (j, j+1) are adjacent in memory and move as 16 bytes.
//
// Energies: a pass with a phase reads its tile's E(z) from the table, or,
// when there is no table (recompute mode), scores the tile's basis states
// against the clause records (32 consecutive z per thread, bit-sliced).
//
// Norm control: rounding in FP32 does not keep |psi|^2 = 1, and on the
// nearly uniform states of the early sweep all amplitudes round alike, so
// the error would add up coherently.  Every pass adds its output's
// sum |psi|^2 into acc_out as a 2^-60 fixed-point integer (integer atomics:
// order-independent, hence deterministic), clears acc_zero for the pass
// after it, and a pass with a phase divides its LUT by sqrt(*acc_in), the
// norm measured by the pass before it (acc_in == nullptr: no rescale).
// A measuring pass adds each wave's share into one of kNormPartials slots
// (acc_out, wave g of the grid into slot g mod kNormPartials), so that no
// address takes more than a few of the tens of thousands of shares (one
// address taking them all serialises them: about 3 ms per n = 28 pass).
// The pass after it reduces the slots (red_src, clearing them) into the
// single total red_dst with one atomic per reducing workgroup.
constexpr int kNormPartials = 8192;
constexpr int kNormReducers = 64;           // workgroups that reduce the slots
constexpr int kNormTotalsWords = 16;        // the ring of three totals, padded to a line
constexpr int kNormWords = kNormTotalsWords + kNormPartials;
constexpr int kMaxRegs = 32;
struct PassDesc {
    int32_t n;
    int32_t n_rest;
    int32_t n_res;
    int32_t phase_at;          // -1: no phase in this pass
    int32_t emax;              // largest E value the LUT must cover
    int32_t set_id;            // qubit set of this pass (host bookkeeping)
    int32_t reverse;           // visit the tiles in descending order
    int32_t persist;           // 1: persistent pipelined grid, 0: one workgroup per tile
    double tA, sA, tB, sB;     // tan(theta/4), sin(theta/2) of the rotations before (A) / after (B) the phase
    double phi, gphase;
    uint64_t tile_begin;       // this launch handles tiles [tile_begin, tile_begin + tile_count)
    uint64_t tile_count;
    unsigned long long *acc_in;        // norm total the phase is scaled by (nullptr: none)
    unsigned long long *acc_out;       // norm partial slots this pass adds its shares into
    unsigned long long *acc_zero;      // norm total to clear for a later pass
    unsigned long long *red_src;       // norm partial slots to reduce (and clear) ...
    unsigned long long *red_dst;       //   into this total (nullptr: no reduction)
    const ClauseRec *clauses;          // recompute mode (no energy table): the clause records
    int32_t m;                         //   and their number
    int32_t xcd_map;                   // grid slots by XCD: 0 plain, 1 top bits, 2 + k tile bit k
    int32_t reg_bits;                  // register bits per thread the pass was planned for
    int32_t pad_;
    uint64_t goff_first[kMaxRegs];     // residency 0: global offset of register j
    uint64_t goff_last[kMaxRegs];      // last residency: global offset of register j
    uint16_t ljp[kMaxRes][kMaxRegs];   // residency r: padded LDS offset of register j
    uint16_t lj[kMaxRes][kMaxRegs];    // residency r: tile-local offset of register j
    uint64_t rest_mask;                // physical bits outside the tile (= rest_pos as a mask)
    uint8_t tile_pos[16];
    uint8_t rest_pos[40];
    uint8_t tpos[kMaxRes][16];         // residency r: tile bit of thread-index bit k
    uint8_t gpos_first[16];            // residency 0: physical bit of thread-index bit k
    uint8_t gpos_last[16];             // last residency: physical bit of thread-index bit k
    uint32_t masks[kMaxRes];           // residency r: maskA | maskB << 8 (register-bit masks)
};

// LDS padding of the tile: element index l is stored at
// l + kPadN[dtype] * (l >> kPadS[dtype]) (additive over disjoint bits).
constexpr int kPadN[2] = {2, 1};
constexpr int kPadS[2] = {5, 4};

// Whole-state-in-one-workgroup evolution (n <= tile bits): the workgroup
// runs all steps k0..k1-1 of one state without leaving LDS, and rescales by
// the exact FP64 norm once per step (folded into the next phase table).
constexpr double kNormFixedScale = 1152921504606846976.0;   // 2^60
struct ResidentDesc {
    void *amp;
    const void *table;
    int32_t n;
    int32_t emax;
    int32_t n_groups;
    int32_t pad_;
    double T;
    int64_t N;
    int64_t k0, k1;
    int32_t reg_bits;          // register bits in use (min(RB, n))
    int32_t thr_bits;          // thread-index bits in use (n - reg_bits)
    uint8_t gbits[8][8];       // group g: state bit of register bit i
    uint8_t tpos[8][16];       // group g: state bit of thread-index bit k
    uint8_t gmask[8];          // register bits of group g that rotate
    const ClauseRec *clauses;  // table == nullptr: energies recomputed from these clause records
    int32_t m;
    int32_t pad2_;
    SchedKnots sched;
};

// One state of a batched evolution run pass by pass (n above the resident
// size).  Every launch applies one pass of step s to every state that is
// still running; a workgroup finds its state from its global tile number.
// The pass structure comes from structs[struct_base + kind] with
//   kind 0: first pass (half phase, then set 0),
//   kind m (1 <= m <= r-2): middle pass over set m,
//   kind r-1 / r: turn pass over set r-1 / set 0,
//   kind r+1 / r+2: last pass over set r-1 / set 0,
// and the rotation and phase coefficients are computed on the device from
// (T, N, schedule, s) exactly as the host computes them for a single state.
struct BatchInst {
    void *amp;
    const void *table;
    unsigned long long *acc;   // 3 norm-control slots of this state
    double T;
    int64_t N;
    uint64_t chunk_offset[2];  // first workgroup chunk of this state in its launch group, for passes
                               // in base tiles [0] and in wide tiles [1]
    int32_t n, emax, r, struct_base;
    SchedKnots sched;
};

// Kernel launch helpers (defined in the .hip files).
// wide: 16 counter planes instead of 8 (needed only when some count > 255);
// stats[4] as documented at the kernel, zero-filled by the caller; table may
// be null (statistics only); count (may be null) receives the number of z
// with E(z) == count_value.
hipError_t launch_energy(const ClauseRec *cl, int m, int n, void *table, int etype, bool wide,
                         uint32_t *stats, int count_value, unsigned long long *count, hipStream_t s);
// Host evaluation of the energy kernel's per-thread arithmetic: the counts
// of z = 32t .. 32t+31 into out32[0..32) (for host-side checks).
void energy_block_host(const ClauseRec *cl, int m, uint32_t t, uint32_t *out32);
hipError_t launch_count_equal(const void *table, int etype, int n, int value,
                              unsigned long long *count, hipStream_t s);
hipError_t launch_init_uniform(void *amp, int dtype, int n, hipStream_t s);
hipError_t launch_init_basis(void *amp, int dtype, int n, uint64_t z0, hipStream_t s);
// ev0, ev1: when set, start and stop events of the pass's dispatch (profiling)
hipError_t launch_pass(void *amp, int dtype, const void *table, int etype, int tile_bits,
                       int reg_bits, const PassDesc &d, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
hipError_t launch_zero_u64(unsigned long long *p, int count, hipStream_t s);
// One lock-step pass (step s, sub-pass j) over a group of states with the
// same number of qubit sets: workgroup b takes up to chunk_tiles tiles of
// state chunk_inst[b]; chunks = workgroups launched (the chunks of the
// states still running, which come first).
hipError_t launch_batch_pass(const BatchInst *insts, const uint32_t *chunk_inst, uint64_t chunks,
                             const PassDesc *structs, int64_t s, int j, int chunk_tiles, int dtype, int etype,
                             int tile_bits, int reg_bits, hipStream_t st);
// Resident evolution: one state (one != nullptr, descriptor by value) or a
// batch of `count` states whose descriptors are in device memory.  rb / wb
// are the kernel's register bits and thread-index bits: resident_shape()
// for one state, kResRegBits[dtype] / kResThrBits for a batch.
hipError_t launch_resident(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, int dtype,
                           int etype, int rb, int wb, hipStream_t s);
// Register/thread split of the batched resident kernel: complex64 5+8,
// complex128 4+8 bits (2^13 / 2^12 amplitudes in one 256-thread workgroup).
constexpr int kResRegBits[2] = {5, 4};
constexpr int kResThrBits = 8;
// A single state runs in one workgroup whose threads hold few amplitudes
// each: 256 threads up to n = 10, then 512 (n = 11) and 1024 (n = 12, 13),
// with 2 register bits (3 at n = 13).  Each step's serial chain per
// thread (loads, rotations, phase) then stays short; a state of 2^10
// amplitudes runs as 256 threads x 4 instead of 32 threads x 32.  Batches
// keep the 256-thread split: many workgroups fill the device anyway.
inline void resident_shape(int n, int *rb, int *wb)
{
    *wb = n <= 10 ? 8 : (n == 11 ? 9 : 10);
    *rb = n <= 12 ? 2 : 3;
}
// Pass tile shapes: complex64 2^13 (5 register bits), complex128 2^12 (4).
constexpr int kPassTileBits[2] = {13, 12};
// Wide tile (complex64 with a uint8 table only): 2^14 amplitudes, 512
// threads x 32 registers, one workgroup per CU (154 KiB of LDS).
constexpr int kWideTileBits = 14;
constexpr int kPassRegBits[2] = {5, 4};
// Complex64 plans of two sets in 2^13-amplitude tiles (n = 14..21) use 4
// register bits: 512 threads per tile of 16 amplitudes each, so that the
// few workgroups of a small state (8..256) finish their tiles sooner.
constexpr int kSmallPlanRegBits = 4;
// Low physical bits every high-qubit tile carries so that each global access
// is a contiguous 256-byte run (32 complex64 / 16 complex128).
constexpr int kPassengerBits[2] = {5, 4};
// table == nullptr: energies scored from clauses[0..m) instead.
hipError_t launch_observables(const void *amp, int dtype, const void *table, int etype, const ClauseRec *clauses,
                              int m, int n, int emin, double *partials, int nblocks, double *out,
                              hipStream_t s);
int observables_blocks(int n);

// y = H(s) x for real FP64 vectors of 2^n entries (spectrum.hip).
hipError_t launch_hmv_product(const double *x, const void *table, int etype, double *y, int n, double s,
                              hipStream_t st);
// The k lowest levels of H(s) after `iters` Lanczos steps from v0
// (device) for each of the count values s_values[i], into the host array
// evals[i * k ..] (NaN where fewer were found), and their residual norms
// into bounds[i * k ..] when bounds is not null.  Synchronous on st.
qaa_status lanczos_lowest(int n, const void *table, int etype, int count, const double *s_values, const double *v0,
                          int iters, int k, double *evals, double *bounds, hipStream_t st);

// Checks a caller's schedule (NULL: linear) and copies it into *out; sets
// the thread's error message on failure.
qaa_status to_knots(const qaa_schedule *sched, SchedKnots *out, const char *who);

// Sets the calling thread's qaa_last_error() message (cleared for QAA_OK)
// and returns st.
qaa_status set_error(qaa_status st, const char *msg);

}  // namespace qaa
