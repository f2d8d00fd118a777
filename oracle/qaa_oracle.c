/*
 * qaa_oracle.c -- plain CPU oracle for the adiabatic 3-SAT state-vector
 * evolution.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the product library never does.
 * It shares no code, header or table with the HIP path.
 *
 * Everything is complex128 / FP64 and written for obviousness, not speed
 * (the only concession is an OpenMP "parallel for" over basis states).
 *
 * Conventions, each from the paper:
 *  - Basis (Sec. 2.1): computational basis |q_n ... q_2 q_1>, sigma_z
 *    eigenvectors.  Variable x_i is carried by qubit q_i, which is bit (i-1)
 *    of the basis-state index z (q_1 is the least significant bit).
 *  - Clauses (Sec. 2.2, K-SAT definition): each clause is the disjunction of
 *    k = 3 literals from {e_i, not e_i}.  A literal is given DIMACS style:
 *    +v means x_v, -v means "not x_v", v in 1..n.
 *  - Final Hamiltonian (Sec. 4.3): H_P is diagonal; its value on |z> is the
 *    number of clauses that the assignment z leaves unsatisfied (the
 *    proportionality constant is taken as 1; duplicated clauses count once
 *    per copy).
 *  - Interpolation (Sec. 2.1, eq. 1): H(s) = (1-s) H_B + s H_P, s = t/T.
 *    The paper asks only that s go from 0 to 1 slowly enough; besides its
 *    linear s(u) = u (u = t/T) the oracle takes a schedule table: s(u)
 *    piecewise linear through the points (j/(count-1), knots[j]).
 *  - Initial Hamiltonian: H_B = sum_i (1 - sigma^x_i)/2, whose ground state is
 *    the uniform superposition of Sec. 2.1 (eigenvalue 0).
 *
 * Integrator (the paper does not state one): N second-order (Strang) steps
 * of size dt = T/N.  Step k (k = 0..N-1) evaluates the schedule at the step
 * midpoint, s_k = s(u_k) with u_k = (k + 1/2)/N, and applies, in time order,
 *      exp(-i (dt/2) s_k H_P)  exp(-i dt (1-s_k) H_B)  exp(-i (dt/2) s_k H_P).
 * exp(-i theta H_B) factorises over qubits into 2x2 blocks
 *      exp(-i theta (1 - sigma^x)/2) = [[alpha, beta], [beta, alpha]],
 *      alpha = (1 + e^{-i theta})/2,  beta = (1 - e^{-i theta})/2,
 * with the global phase kept.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Truth value of one literal under assignment z (Sec. 2.2). */
static int literal_true(int32_t lit, uint64_t z)
{
    int32_t v = lit > 0 ? lit : -lit;
    int x_v = (int)((z >> (v - 1)) & 1u);
    return lit > 0 ? x_v : !x_v;
}

/* Clause C = (a_1 or a_2 or a_3) is satisfied iff some literal is true. */
static int clause_satisfied(const int32_t *c, uint64_t z)
{
    return literal_true(c[0], z) || literal_true(c[1], z) || literal_true(c[2], z);
}

/*
 * Energy function of Sec. 4.3: E(z) = number of unsatisfied clauses.
 * lits: 3*m signed 1-based literals.  E: 2^n outputs.
 * Returns 0, or -1 when a literal is out of range.
 */
int oracle_energy(int n, int m, const int32_t *lits, int32_t *E)
{
    for (int i = 0; i < 3 * m; ++i) {
        int32_t v = lits[i] > 0 ? lits[i] : -lits[i];
        if (v < 1 || v > n) return -1;
    }
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < dim; ++z) {
        int32_t e = 0;
        for (int c = 0; c < m; ++c)
            if (!clause_satisfied(lits + 3 * c, (uint64_t)z)) e += 1;
        E[z] = e;
    }
    return 0;
}

/* E(z) for a list of basis states only (same definition, one z at a time):
 * lets tests check a large table on a sample without 2^n work. */
int oracle_energy_at(int n, int m, const int32_t *lits, const uint64_t *zs, int64_t count, int32_t *E)
{
    for (int i = 0; i < 3 * m; ++i) {
        int32_t v = lits[i] > 0 ? lits[i] : -lits[i];
        if (v < 1 || v > n) return -1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        int32_t e = 0;
        for (int c = 0; c < m; ++c)
            if (!clause_satisfied(lits + 3 * c, zs[i])) e += 1;
        E[i] = e;
    }
    return 0;
}

/* psi(z) <- exp(-i a E(z)) psi(z): the diagonal factor exp(-i a H_P). */
static void apply_problem_phase(cplx *psi, const int32_t *E, int64_t dim, double a)
{
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < dim; ++z)
        psi[z] *= cexp(-I * a * (double)E[z]);
}

/* exp(-i theta H_B) = product over qubits q of the 2x2 block acting on the
 * pair (z, z + 2^q) with bit q of z clear. */
static void apply_driver(cplx *psi, int n, double theta)
{
    const int64_t dim = (int64_t)1 << n;
    const cplx e = cexp(-I * theta);
    const cplx alpha = (1.0 + e) / 2.0;
    const cplx beta = (1.0 - e) / 2.0;
    for (int q = 0; q < n; ++q) {
        const int64_t bit = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < dim; ++z) {
            if (z & bit) continue;
            cplx x0 = psi[z], x1 = psi[z | bit];
            psi[z] = alpha * x0 + beta * x1;
            psi[z | bit] = beta * x0 + alpha * x1;
        }
    }
}

/* Uniform superposition of Sec. 2.1: psi(z) = 2^{-n/2}. */
void oracle_init_uniform(int n, double *psi_ri)
{
    cplx *psi = (cplx *)psi_ri;
    const int64_t dim = (int64_t)1 << n;
    const double a = 1.0 / sqrt((double)dim);
    for (int64_t z = 0; z < dim; ++z) psi[z] = a;
}

/*
 * The schedule s(u), u = t/T in [0, 1]: u itself when count == 0, else the
 * straight line between the two knots whose abscissae j h, (j+1) h
 * (h = 1/(count-1)) enclose u.
 */
static double schedule_value(double u, const double *knots, int count)
{
    if (count == 0) return u;
    const double h = 1.0 / (double)(count - 1);
    int j = (int)floor(u / h);
    if (j > count - 2) j = count - 2;
    if (j < 0) j = 0;
    const double w = (u - (double)j * h) / h;     /* 0 <= w <= 1 inside the segment */
    return (1.0 - w) * knots[j] + w * knots[j + 1];
}

/*
 * Steps k0 .. k1-1 of the N-step second-order evolution over total time T.
 * psi_ri: 2^n complex128 amplitudes, interleaved (re, im), updated in place.
 * knots/count: the schedule table (count == 0: linear schedule; else
 * 2 <= count and knots[0..count) in [0, 1]).
 * Returns 0, or -1 on bad arguments.
 */
int oracle_evolve(int n, int m, const int32_t *lits, double *psi_ri,
                  double T, int64_t N, int64_t k0, int64_t k1, const double *knots, int count)
{
    if (n < 1 || n > 34 || m < 0 || N < 0 || k0 < 0 || k1 < k0 || k1 > N) return -1;
    if (count != 0 && (count < 2 || !knots)) return -1;
    for (int j = 0; j < count; ++j)
        if (!(knots[j] >= 0.0 && knots[j] <= 1.0)) return -1;
    if (N == 0 || k0 == k1) return 0;
    const int64_t dim = (int64_t)1 << n;
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * (size_t)dim);
    if (!E) return -1;
    if (oracle_energy(n, m, lits, E) != 0) { free(E); return -1; }
    cplx *psi = (cplx *)psi_ri;
    const double dt = T / (double)N;
    for (int64_t k = k0; k < k1; ++k) {
        const double s = schedule_value(((double)k + 0.5) / (double)N, knots, count);
        apply_problem_phase(psi, E, dim, 0.5 * dt * s);
        apply_driver(psi, n, dt * (1.0 - s));
        apply_problem_phase(psi, E, dim, 0.5 * dt * s);
    }
    free(E);
    return 0;
}

/*
 * Observables of the final state (Sec. 2.1: the answer is read from the
 * ground manifold of H_P, whose degeneracy is the number of basis states at
 * the minimum energy):
 *   out[0] = norm          = sum_z |psi(z)|^2
 *   out[1] = <H_P>         = sum_z E(z) |psi(z)|^2
 *   out[2] = P_success     = sum over z with E(z) = E_min of |psi(z)|^2
 * e_min / degeneracy: minimum of E and how many z attain it.
 */
int oracle_observables(int n, int m, const int32_t *lits, const double *psi_ri,
                       double *out, int32_t *e_min, int64_t *degeneracy)
{
    const int64_t dim = (int64_t)1 << n;
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * (size_t)dim);
    if (!E) return -1;
    if (oracle_energy(n, m, lits, E) != 0) { free(E); return -1; }
    int32_t emin = E[0];
    for (int64_t z = 1; z < dim; ++z)
        if (E[z] < emin) emin = E[z];
    int64_t deg = 0;
    for (int64_t z = 0; z < dim; ++z)
        if (E[z] == emin) ++deg;
    const cplx *psi = (const cplx *)psi_ri;
    double norm = 0.0, energy = 0.0, psucc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : norm, energy, psucc)
    for (int64_t z = 0; z < dim; ++z) {
        double p = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
        norm += p;
        energy += (double)E[z] * p;
        if (E[z] == emin) psucc += p;
    }
    free(E);
    out[0] = norm;
    out[1] = energy;
    out[2] = psucc;
    *e_min = emin;
    *degeneracy = deg;
    return 0;
}

/* Thread count OpenMP will use (reported beside CPU timings), and a way to
 * change it for timing runs (it does not change any result). */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int t) { if (t > 0) omp_set_num_threads(t); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_num_threads(int t) { (void)t; }
#endif
