// qaa_internal.h -- structures shared by the host runtime and the gfx950
// kernels of libqaa.  Not part of the public ABI (include/qaa.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qaa {

// Largest number of register-group residencies in one pass (see PassDesc).
constexpr int kMaxRes = 12;
// Phase lookup table capacity: E in [0, kLutMax).
constexpr int kLutMax = 1024;
constexpr int kLutMaxU8 = 256;

// One clause in the form the energy kernel consumes.  A clause over three
// distinct variables is violated by z iff (z & mask) == pat, where mask has
// the clause's three variable bits and pat has the bits of the negated
// literals.  The kernel scores 8 consecutive z at once: the part of the test
// on bits >= 3 (mhi/phi) is one compare for all 8, and lo_a/lo_b hold the
// 0/1 outcome of the bits-0..2 part for z mod 8 = 0..3 / 4..7 as four 16-bit
// lanes each, ready to be added to packed counters.
struct ClauseRec {
    uint64_t mhi, phi;
    uint64_t lo_a, lo_b;
};

// One HBM pass of the split-step evolution over tiles of 2^TB amplitudes.
//
// A tile is the set of basis states that agree on all bits outside
// tile_pos[0..TB): tile-local index l (TB bits) maps to the physical index
// by placing bit j of l at bit tile_pos[j]; the workgroup id is spread over
// rest_pos[0..n_rest) the same way.  Inside the workgroup the tile sits in
// LDS; a "residency" loads it into registers so that register bit i of
// every thread is tile-local bit gbits[r][i] (the other tile bits index the
// threads), applies the operations of that residency, and stores it back:
//   1. rotations on the register bits in maskA[r] with coefficient set A,
//   2. if r == phase_at: the diagonal phase exp(-i (phi E + gphase)),
//   3. rotations on the register bits in maskB[r] with coefficient set B.
// A rotation is the single-qubit factor of exp(-i theta H_B) without its
// global phase: [[c, i s], [i s, c]], c = cos(theta/2), s = sin(theta/2),
// given as cm1 = c - 1 = -2 sin^2(theta/4) (accurate for small theta) and s.
// The global phase exp(-i n theta / 2) of each step is folded into gphase.
//
// Norm control: rounding in FP32 does not keep |psi|^2 = 1, and on the
// nearly uniform states of the early sweep all amplitudes round alike, so
// the error would add up coherently.  Every pass adds its output's
// sum |psi|^2 into acc_out as a 2^-60 fixed-point integer (integer atomics:
// order-independent, hence deterministic), clears acc_zero for the pass
// after it, and a pass with a phase divides its LUT by sqrt(*acc_in), the
// norm measured by the pass before it (acc_in == nullptr: no rescale).
struct PassDesc {
    int32_t n;
    int32_t n_rest;
    int32_t n_res;
    int32_t phase_at;          // -1: no phase in this pass
    int32_t emax;              // largest E value the LUT must cover
    int32_t pad_;
    double cm1A, sA, cm1B, sB;
    double phi, gphase;
    unsigned long long *acc_in;
    unsigned long long *acc_out;
    unsigned long long *acc_zero;
    uint8_t tile_pos[16];
    uint8_t rest_pos[40];
    uint8_t gbits[kMaxRes][8];     // residency r: tile bit of register bit i
    uint8_t tpos[kMaxRes][16];     // residency r: tile bit of thread-index bit k
    uint8_t maskA[kMaxRes];
    uint8_t maskB[kMaxRes];
};

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
};

// Kernel launch helpers (defined in the .hip files).
hipError_t launch_energy(const ClauseRec *cl, int m, int n, void *table, int etype,
                         uint32_t *stats, hipStream_t s);
hipError_t launch_count_equal(const void *table, int etype, int n, int value,
                              unsigned long long *count, hipStream_t s);
hipError_t launch_init_uniform(void *amp, int dtype, int n, hipStream_t s);
hipError_t launch_init_basis(void *amp, int dtype, int n, uint64_t z0, hipStream_t s);
hipError_t launch_pass(void *amp, int dtype, const void *table, int etype, int tile_bits,
                       int reg_bits, const PassDesc &d, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int count, hipStream_t s);
// Resident evolution: one state (one != nullptr, descriptor by value) or a
// batch of `count` states whose descriptors are in device memory.
hipError_t launch_resident(const ResidentDesc *descs_dev, const ResidentDesc *one, int count, int dtype,
                           int etype, hipStream_t s);
// Register/thread split of the resident kernels: complex64 5+8, complex128 4+8.
constexpr int kResRegBits[2] = {5, 4};
constexpr int kResThrBits = 8;
// Pass tile shapes: complex64 2^13 (5 register bits), complex128 2^12 (4).
constexpr int kPassTileBits[2] = {13, 12};
constexpr int kPassRegBits[2] = {5, 4};
// Low physical bits every high-qubit tile carries so that each global access
// is a contiguous 256-byte run (32 complex64 / 16 complex128).
constexpr int kPassengerBits[2] = {5, 4};
hipError_t launch_observables(const void *amp, int dtype, const void *table, int etype, int n,
                              int emin, double *partials, int nblocks, double *out,
                              hipStream_t s);
int observables_blocks(int n);

}  // namespace qaa
