// spectrum.hip -- lowest eigenvalues of H(s) = (1 - s) H_B + s H_P
// (Sec. 2.1, eq. 1) by Lanczos with full reorthogonalisation, FP64.
//
// H(s) is real and symmetric in the computational basis:
//     (H x)(z) = ((1 - s) n/2 + s E(z)) x(z) - (1 - s)/2 sum_q x(z xor 2^q),
// since H_B = sum_q (1 - sigma^x_q)/2 and sigma^x_q flips bit q of z.
// The device runs the whole Lanczos recurrence (matrix-vector product,
// three-term recurrence, one classical Gram-Schmidt sweep against every
// earlier Lanczos vector, normalisation) without a host round trip; the
// host reads the tridiagonal coefficients once at the end and finds the
// lowest Ritz values by Sturm-sequence bisection (Barth, Martin and
// Wilkinson, 1967).
#include "qaa_internal.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <string>
#include <vector>

namespace qaa {
namespace {

// Tile of the matrix-vector product: 2^kHmvTile consecutive z per
// workgroup, staged in LDS so the flips of the low qubits read LDS; the
// flips of the high qubits read the partner tile from memory, which for a
// fixed qubit is itself contiguous (coalesced).
constexpr int kHmvTile = 10;
constexpr int kThreads = 256;
// Partial sums per vector in the dot products: fixed, so the order of
// every FP64 sum is fixed (deterministic results).
constexpr int kDotBlocks = 2048;
constexpr int kDotWaves = kThreads / 64;
constexpr int kDotGroup = 8;      // vectors per sweep over w

template <typename ET>
__global__ void __launch_bounds__(kThreads)
hmv_kernel(const double *__restrict__ x, const ET *__restrict__ E, double *__restrict__ y, int n, int tb,
           double diag_b, double off, double s)
{
    __shared__ double xs[1 << kHmvTile];
    const uint32_t tsize = 1u << tb;
    const uint64_t base = (uint64_t)blockIdx.x << tb;
    for (uint32_t l = threadIdx.x; l < tsize; l += blockDim.x) xs[l] = x[base + l];
    __syncthreads();
    for (uint32_t l = threadIdx.x; l < tsize; l += blockDim.x) {
        const uint64_t z = base + l;
        double acc = 0.0;
        for (int q = 0; q < tb; ++q) acc += xs[l ^ (1u << q)];
        for (int q = tb; q < n; ++q) acc += x[z ^ (1ull << q)];
        y[z] = fma(fma(s, (double)E[z], diag_b), xs[l], off * acc);
    }
}

// This workgroup's part of V_j . w for the G vectors j0 .. j0+G-1, into
// partials[j * gridDim.x + block] (lanes summed by butterflies, then the
// four waves in order through LDS).  G is a compile-time
// count so that the G loads of an element are issued back to back (a
// run-time guard per load would make each one wait for the previous).
template <int G>
__device__ __forceinline__ void dots_group(const double *__restrict__ V, int j0, const double *__restrict__ w,
                                           uint64_t dim, double *__restrict__ partials)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t e0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    double p[G];
#pragma unroll
    for (int i = 0; i < G; ++i) p[i] = 0.0;
    for (uint64_t e = e0; e < dim; e += stride) {
        const double we = w[e];
        double v[G];
#pragma unroll
        for (int i = 0; i < G; ++i) v[i] = V[(uint64_t)(j0 + i) * dim + e];
#pragma unroll
        for (int i = 0; i < G; ++i) p[i] = fma(v[i], we, p[i]);
    }
    __shared__ double red[kDotGroup][kDotWaves];
#pragma unroll
    for (int i = 0; i < G; ++i) {
        double t = p[i];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) red[i][wave] = t;
    }
    __syncthreads();
    if ((int)threadIdx.x < G) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kDotWaves; ++q) t += red[threadIdx.x][q];
        partials[(uint64_t)(j0 + (int)threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();      // red is rewritten by the next group
}

// Partial dot products V_j . w for j < k (V_j = V + j * dim): groups of
// kDotGroup vectors per sweep over w, then the remaining ones one by one.
__global__ void __launch_bounds__(kThreads)
dots_kernel(const double *__restrict__ V, int k, const double *__restrict__ w, uint64_t dim,
            double *__restrict__ partials)
{
    int j0 = 0;
    for (; j0 + kDotGroup <= k; j0 += kDotGroup) dots_group<kDotGroup>(V, j0, w, dim, partials);
    for (; j0 < k; ++j0) dots_group<1>(V, j0, w, dim, partials);
}

// out[j] = sum of the np partials of vector j, in a fixed order (block j).
__global__ void __launch_bounds__(kThreads)
sum_partials_kernel(const double *__restrict__ partials, int np, double *__restrict__ out)
{
    const int j = (int)blockIdx.x;
    double t = 0.0;
    for (int p = (int)threadIdx.x; p < np; p += (int)blockDim.x) t += partials[(uint64_t)j * np + p];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    __shared__ double red[kThreads / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double total = 0.0;
        for (int i = 0; i < kThreads / 64; ++i) total += red[i];
        out[j] = total;
    }
}

// w -= sum_{j < k} c[j] V_j.
__global__ void __launch_bounds__(kThreads)
update_kernel(double *__restrict__ w, const double *__restrict__ V, int k, const double *__restrict__ c,
              uint64_t dim)
{
    extern __shared__ double cs[];
    for (int j = (int)threadIdx.x; j < k; j += (int)blockDim.x) cs[j] = c[j];
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < dim; e += stride) {
        double acc = 0.0;
        for (int j = 0; j < k; ++j) acc = fma(cs[j], V[(uint64_t)j * dim + e], acc);
        w[e] -= acc;
    }
}

// v = w / sqrt(*nrm2) (v = 0 if the norm is exactly 0).  Block 0 also
// records alpha[j] = ca[j] + cb[j] (the recurrence's coefficient of the
// newest vector and its correction from the sweep; ca == nullptr: none)
// and beta[j] = sqrt(*nrm2).
__global__ void __launch_bounds__(kThreads)
normalize_kernel(const double *__restrict__ w, double *__restrict__ v, const double *__restrict__ nrm2,
                 uint64_t dim, const double *__restrict__ ca, const double *__restrict__ cb, int j,
                 double *__restrict__ alpha, double *__restrict__ beta)
{
    const double b = sqrt(*nrm2);
    const double inv = b > 0.0 ? 1.0 / b : 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < dim; e += stride) v[e] = w[e] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (ca) alpha[j] = ca[j] + cb[j];
        if (beta) beta[j] = b;
    }
}

unsigned grid_for(uint64_t dim)
{
    const uint64_t b = (dim + kThreads - 1) / kThreads;
    return (unsigned)std::min<uint64_t>(b, 4096);
}

// The number of eigenvalues of the symmetric tridiagonal matrix
// (diagonal a[0..m), off-diagonal b[0..m-1)) that are smaller than x:
// the count of negative pivots of the LDL^T factorisation of T - x I.
int sturm_count(const std::vector<double> &a, const std::vector<double> &b, int m, double x, double pivmin)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
        q = (a[i] - x) - (i > 0 ? b[i - 1] * b[i - 1] / q : 0.0);
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// The i-th smallest eigenvalue (i = 0, 1, ...) of the tridiagonal matrix,
// by bisection inside the Gershgorin interval.
double tridiag_eig(const std::vector<double> &a, const std::vector<double> &b, int m, int i)
{
    double lo = a[0], hi = a[0], scale = 0.0;
    for (int r = 0; r < m; ++r) {
        const double rad = (r > 0 ? std::fabs(b[r - 1]) : 0.0) + (r + 1 < m ? std::fabs(b[r]) : 0.0);
        lo = std::min(lo, a[r] - rad);
        hi = std::max(hi, a[r] + rad);
        scale = std::max(scale, std::fabs(a[r]) + rad);
    }
    const double pivmin = DBL_MIN * std::max(1.0, scale * scale);
    lo -= DBL_EPSILON * scale + pivmin;
    hi += DBL_EPSILON * scale + pivmin;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, m, mid, pivmin) > i)
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

template <typename ET>
hipError_t launch_hmv(const double *x, const void *table, double *y, int n, double s, hipStream_t st)
{
    const int tb = std::min(n, kHmvTile);
    const unsigned blocks = (unsigned)(1ull << (n - tb));
    hipLaunchKernelGGL((hmv_kernel<ET>), dim3(blocks), dim3(kThreads), 0, st, x, reinterpret_cast<const ET *>(table),
                       y, n, tb, (1.0 - s) * 0.5 * (double)n, -0.5 * (1.0 - s), s);
    return hipGetLastError();
}

// c[0..k) = V[0..k)^T w, through `partials` (k * kDotBlocks).
hipError_t project(const double *V, int k, const double *w, uint64_t dim, double *partials, double *c,
                   hipStream_t st)
{
    const unsigned nb = (unsigned)std::min<uint64_t>(kDotBlocks, (dim + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(dots_kernel, dim3(nb), dim3(kThreads), 0, st, V, k, w, dim, partials);
    hipLaunchKernelGGL(sum_partials_kernel, dim3((unsigned)k), dim3(kThreads), 0, st, partials, (int)nb, c);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_hmv_product(const double *x, const void *table, int etype, double *y, int n, double s,
                              hipStream_t st)
{
    return etype == 0 ? launch_hmv<uint8_t>(x, table, y, n, s, st) : launch_hmv<uint16_t>(x, table, y, n, s, st);
}

namespace {

// Residual norm of the Ritz pair at theta: |beta_m| |y[m-1]|, with y the
// unit eigenvector of the leading m x m block of T at theta.  Since H is
// symmetric, some eigenvalue of H lies within this distance of theta.  y
// comes from inverse iteration with (T - theta I), factored by Gaussian
// elimination with partial pivoting for tridiagonal matrices (the scheme
// of LAPACK's dgttrf / dgtts2).
double ritz_residual(const std::vector<double> &a, const std::vector<double> &b, int m, double theta,
                     double beta_m, double pivmin)
{
    std::vector<double> dl(m), d(m), du(m), du2(m, 0.0), x(m, 1.0);
    std::vector<char> swap(m, 0);
    for (int i = 0; i < m; ++i) {
        d[i] = a[i] - theta;
        if (i + 1 < m) dl[i] = du[i] = b[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            if (std::fabs(d[i]) < pivmin) d[i] = pivmin;
            const double f = dl[i] / d[i];
            dl[i] = f;
            d[i + 1] -= f * du[i];
        } else {                              // interchange rows i and i + 1
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - f * d[i + 1];
            if (i + 2 < m) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
            swap[i] = 1;
        }
    }
    if (std::fabs(d[m - 1]) < pivmin) d[m - 1] = pivmin;
    for (int it = 0; it < 3; ++it) {
        for (int i = 0; i + 1 < m; ++i) {     // L z = P x
            if (swap[i]) {
                const double t = x[i];
                x[i] = x[i + 1];
                x[i + 1] = t - dl[i] * x[i];
            } else {
                x[i + 1] -= dl[i] * x[i];
            }
        }
        x[m - 1] /= d[m - 1];                 // U x = z
        if (m > 1) x[m - 2] = (x[m - 2] - du[m - 2] * x[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i) x[i] = (x[i] - du[i] * x[i + 1] - du2[i] * x[i + 2]) / d[i];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm = std::max(nrm, std::fabs(x[i]));
        for (int i = 0; i < m; ++i) x[i] /= nrm;
    }
    double nrm2 = 0.0;
    for (int i = 0; i < m; ++i) nrm2 += x[i] * x[i];
    return std::fabs(beta_m) * std::fabs(x[m - 1]) / std::sqrt(nrm2);
}

// The lowest k levels of the tridiagonal matrix (alpha a, beta b) that a
// Lanczos run produced, into evals (NaN where fewer were found), and, if
// bounds is not null, the residual norm of each (a distance within which
// H has an eigenvalue).
void levels_from_tridiag(const std::vector<double> &a, const std::vector<double> &b, int iters, int k,
                         double *evals, double *bounds)
{
    // The Krylov space closes at the first negligible beta: T splits there
    // and only its leading block belongs to the start vector's space.
    double scale = 0.0;
    for (int j = 0; j < iters; ++j) scale = std::max(scale, std::fabs(a[j]) + 2.0 * b[j]);
    int m = iters;
    for (int j = 0; j + 1 < iters; ++j)
        if (!(b[j] > 1e-12 * std::max(scale, 1.0))) {
            m = j + 1;
            break;
        }
    // Levels, not Ritz values: once the start vector's Krylov space is used
    // up, rounding feeds in directions outside it and a degenerate level can
    // show up again (a genuine second eigenvector); values closer than
    // 1e-10 of the matrix scale count as one level.
    const double merge = 1e-10 * std::max(scale, 1.0);
    const double pivmin = DBL_MIN * std::max(1.0, scale * scale);
    int got = 0;
    for (int i = 0; i < m && got < k; ++i) {
        const double x = tridiag_eig(a, b, m, i);
        if (got == 0 || x - evals[got - 1] > merge) {
            if (bounds) bounds[got] = ritz_residual(a, b, m, x, b[m - 1], pivmin);
            evals[got++] = x;
        }
    }
    for (int i = got; i < k; ++i) {
        evals[i] = NAN;
        if (bounds) bounds[i] = NAN;
    }
}

}  // namespace

extern "C" qaa_status qaa_debug_tridiag_levels(const double *alpha, const double *beta, int32_t m, int32_t k,
                                               double *evals, double *bounds)
{
    if (!alpha || !beta || !evals || m < 1 || k < 1)
        return set_error(QAA_ERR_INVALID_ARG, "qaa_debug_tridiag_levels: bad arguments");
    const std::vector<double> a(alpha, alpha + m), b(beta, beta + m);
    levels_from_tridiag(a, b, m, k, evals, bounds);
    return set_error(QAA_OK, nullptr);
}

qaa_status lanczos_lowest(int n, const void *table, int etype, int count, const double *s_values, const double *v0,
                          int iters, int k, double *evals, double *bounds, hipStream_t st)
{
    const uint64_t dim = 1ull << n;
    iters = (int)std::min<uint64_t>((uint64_t)iters, dim);
    // device memory, taken once for all values of s: V (iters + 1 vectors),
    // w, the dot partials and the small coefficient arrays
    const size_t vec = sizeof(double) * dim;
    const size_t nparts = (size_t)(iters + 1) * kDotBlocks;
    const size_t small = sizeof(double) * (4 * (size_t)(iters + 1) + 2);
    char *mem = nullptr;
    const size_t bytes = vec * (size_t)(iters + 2) + sizeof(double) * nparts + small;
    if (hipMallocAsync(reinterpret_cast<void **>(&mem), bytes, st) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QAA_ERR_OUT_OF_MEMORY, "qaa_spectrum: Lanczos workspace allocation failed");
    }
    double *V = reinterpret_cast<double *>(mem);
    double *w = V + dim * (uint64_t)(iters + 1);
    double *partials = w + dim;
    double *ca = partials + nparts;            // alpha_j of the three-term recurrence (iters + 1)
    double *cb = ca + (iters + 1);             // coefficients of the reorthogonalisation sweep (iters + 1)
    double *alpha = cb + (iters + 1);
    double *beta = alpha + (iters + 1);
    double *nrm2 = beta + (iters + 1);
    double *n0 = nrm2 + 1;                     // |v0|^2
    const unsigned g = grid_for(dim);
    hipError_t e = hipSuccess;
    auto ok = [&]() { return (e = hipGetLastError()) == hipSuccess; };
    std::vector<double> a((size_t)iters), b((size_t)iters);
    double v0_norm2 = 0.0;
    for (int si = 0; si < count && e == hipSuccess; ++si) {
        const double s = s_values[si];
        // v_0 = v0 / |v0|
        e = project(v0, 1, v0, dim, partials, n0, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(normalize_kernel, dim3(g), dim3(kThreads), 0, st, v0, V, (const double *)n0, dim,
                               (const double *)nullptr, (const double *)nullptr, 0, (double *)nullptr,
                               (double *)nullptr);
            ok();
        }
        for (int j = 0; j < iters && e == hipSuccess; ++j) {
            double *vj = V + dim * (uint64_t)j;
            e = launch_hmv_product(vj, table, etype, w, n, s, st);
            // three-term recurrence: w -= beta_{j-1} v_{j-1}; alpha_j = v_j . w; w -= alpha_j v_j
            if (e == hipSuccess && j > 0) {
                hipLaunchKernelGGL(update_kernel, dim3(g), dim3(kThreads), sizeof(double), st, w,
                                   (const double *)(vj - dim), 1, (const double *)(beta + (j - 1)), dim);
                ok();
            }
            if (e == hipSuccess) e = project(vj, 1, w, dim, partials, ca + j, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(update_kernel, dim3(g), dim3(kThreads), sizeof(double), st, w, (const double *)vj,
                                   1, (const double *)(ca + j), dim);
                ok();
            }
            // then one classical Gram-Schmidt sweep against v_0 .. v_j: the
            // recurrence already removed the large components, so the sweep
            // only takes out what rounding left (full reorthogonalisation)
            if (e == hipSuccess) e = project(V, j + 1, w, dim, partials, cb, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(update_kernel, dim3(g), dim3(kThreads), sizeof(double) * (j + 1), st, w,
                                   (const double *)V, j + 1, (const double *)cb, dim);
                ok();
            }
            if (e == hipSuccess) e = project(w, 1, w, dim, partials, nrm2, st);
            if (e == hipSuccess) {
                hipLaunchKernelGGL(normalize_kernel, dim3(g), dim3(kThreads), 0, st, (const double *)w,
                                   V + dim * (uint64_t)(j + 1), (const double *)nrm2, dim, (const double *)ca,
                                   (const double *)cb, j, alpha, beta);
                ok();
            }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&v0_norm2, n0, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(a.data(), alpha, sizeof(double) * iters, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(b.data(), beta, sizeof(double) * iters, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) break;
        if (!(v0_norm2 > 0.0) || !std::isfinite(v0_norm2)) {
            (void)hipFreeAsync(mem, st);
            return set_error(QAA_ERR_INVALID_ARG, "qaa_spectrum: the start vector v0 is zero or not finite");
        }
        levels_from_tridiag(a, b, iters, k, evals + (size_t)si * k, bounds ? bounds + (size_t)si * k : nullptr);
    }
    (void)hipFreeAsync(mem, st);
    if (e != hipSuccess)
        return set_error(QAA_ERR_DEVICE, (std::string("qaa_spectrum: ") + hipGetErrorString(e)).c_str());
    return QAA_OK;
}

}  // namespace qaa
