// Sturm bisection of tridiagonal matrices, smoothed IDoS and level sums.
#include <algorithm>

#include "device_common.hpp"

namespace mlmc {

// ---------------------------------------------------------------------------
// Bisection: one workgroup per tridiagonal (d, e) at a time, or per part of
// its eigenvalues when the batch is too small to fill the chip; d and e are
// staged in LDS (e squared there), so the serial Sturm recurrences read
// broadcast LDS.  A grid smaller than the batch walks it with a stride
// (a bisection running beside other kernels keeps to a few workgroups per CU).
// ---------------------------------------------------------------------------
constexpr int kBisectThreads = 256;
// Largest matrix side whose d and e^2 are staged in LDS (16 bytes per row);
// larger tridiagonals are read from device memory where they lie (e is
// squared in place there).
constexpr int64_t kBisectLdsMaxLd = 8192;

template <bool GLOBAL>
__global__ __launch_bounds__(kBisectThreads) void bisect_kernel(const double *__restrict__ dall,
                                                                double *__restrict__ eall, int64_t lde,
                                                                const int32_t *__restrict__ n_in, int64_t batch,
                                                                int64_t ld_max, double *__restrict__ w, int64_t ldw,
                                                                int parts) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *red = reinterpret_cast<double *>(smem);
    int *cnt = reinterpret_cast<int *>(red + 32);
    double *dl = reinterpret_cast<double *>(cnt + kBisectThreads + 8);
    double *el = dl + ld_max;
    for (int64_t job = blockIdx.x; job < batch * parts; job += gridDim.x) {
        const int64_t u = job / parts;
        const int part = (int)(job % parts);
        const int n = n_in[u];
        double *wu = w + u * ldw;
        if (n < 0 || n > ld_max) {
            for (int64_t i = threadIdx.x; i < ldw && i < ld_max; i += blockDim.x) wu[i] = NAN;
            continue;
        }
        const double *d = dl;
        double *e = el;
        if constexpr (GLOBAL) {
            d = dall + u * lde;
            e = eall + u * lde;
        } else {
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                dl[i] = dall[u * lde + i];
                el[i] = (i + 1 < n) ? eall[u * lde + i] : 0.0;
            }
        }
        __syncthreads();
        bisect_block(d, e, n, wu, red, cnt, part, parts);
        __syncthreads();  // d, e are read to the end before the next matrix replaces them
    }
}

hipError_t launch_bisect(const double *d, double *e, int64_t lde, const int32_t *n_in, int64_t batch,
                         int64_t ld_max, double *w, int64_t ldw, hipStream_t s, int64_t max_blocks) {
    if (batch == 0) return hipSuccess;
    const bool global = ld_max > kBisectLdsMaxLd;
    const size_t lds = 32 * sizeof(double) + (kBisectThreads + 8) * sizeof(int) +
                       (global ? 0 : 2 * sizeof(double) * (size_t)ld_max);
    const void *fn = global ? reinterpret_cast<const void *>(bisect_kernel<true>)
                            : reinterpret_cast<const void *>(bisect_kernel<false>);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    // A batch of fewer than 512 matrices (with no cap on the grid) splits each
    // matrix's eigenvalues over up to ld_max / 256 workgroups, so that about
    // 512 run; the global-memory variant squares e in place and keeps one.
    int parts = 1;
    if (!global && max_blocks <= 0 && batch < 512)
        parts = (int)std::max<int64_t>(1, std::min<int64_t>(512 / batch, (ld_max + kBisectThreads - 1) / kBisectThreads));
    const int64_t jobs = batch * parts;
    const int64_t blocks = (max_blocks > 0 && max_blocks < jobs) ? max_blocks : jobs;
    if (global)
        hipLaunchKernelGGL(bisect_kernel<true>, dim3((unsigned)blocks), dim3(kBisectThreads), lds, s, d, e, lde, n_in,
                           batch, ld_max, w, ldw, parts);
    else
        hipLaunchKernelGGL(bisect_kernel<false>, dim3((unsigned)blocks), dim3(kBisectThreads), lds, s, d, e, lde, n_in,
                           batch, ld_max, w, ldw, parts);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Smoothed IDoS (eq. (IDoS), nearest-point rule, eq. (MLMC_smoothing)).
// Thread = (outcome, energy).  For each k-point the ascending eigenvalues are
// split by binary search into those with g = 1 exactly (counted), a window
// where g is evaluated, and those with g = 0; k-points are summed in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int count_le(const double *E, int n, double x) {  // #{E_i <= x}
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (E[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ int count_lt(const double *E, int n, double x) {  // #{E_i < x}
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (E[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double smooth_step(int smoother, double x) {
    if (smoother == MLMC_SMOOTH_GAUSS) return 0.5 * erfc(x * 0.70710678118654752440);
    if (x <= -1.0) return 1.0;
    if (x >= 1.0) return 0.0;
    return 0.5 - 1.125 * x + 0.625 * x * x * x;
}

__global__ __launch_bounds__(256) void idos_kernel(const double *__restrict__ w, int64_t ldw,
                                                   const int32_t *__restrict__ n, int n_k,
                                                   const double *__restrict__ kweight, double inv_area,
                                                   const double *__restrict__ eps, int n_eps, double delta,
                                                   int smoother, double *__restrict__ out) {
    const int64_t s = blockIdx.x;
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= n_eps) return;
    const double ej = eps[j];
    const double cut = (smoother == MLMC_SMOOTH_GAUSS) ? kGaussCut : 1.0;
    const double lo_e = ej - cut * delta, hi_e = ej + cut * delta;
    const double inv_delta = 1.0 / delta;
    double acc = 0.0;
    for (int k = 0; k < n_k; ++k) {
        const int64_t unit = s * n_k + k;
        const int nu = max(0, min(n[unit], (int)ldw));
        const double *E = w + unit * ldw;
        const int below = count_le(E, nu, lo_e);
        const int upto = count_lt(E, nu, hi_e);
        double sum = (double)below;
        for (int i = below; i < upto; ++i) sum += smooth_step(smoother, (E[i] - ej) * inv_delta);
        acc += kweight[k] * sum;
    }
    out[s * n_eps + j] = acc * inv_area;
}

hipError_t launch_idos(const double *w, int64_t ldw, const int32_t *n, int64_t n_samples, int n_k,
                       const double *kweight, double inv_area, const double *eps, int n_eps, double delta,
                       int smoother, double *out, hipStream_t s) {
    if (n_samples == 0 || n_eps == 0) return hipSuccess;
    const int threads = 256;
    dim3 grid((unsigned)n_samples, (unsigned)((n_eps + threads - 1) / threads));
    hipLaunchKernelGGL(idos_kernel, grid, dim3(threads), 0, s, w, ldw, n, n_k, kweight, inv_area, eps, n_eps, delta,
                       smoother, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Level sums of eq. (MLMC): thread = energy, samples accumulated in order.
// Optionally the per-sample values Y_s and Q_s themselves (rows of y_out,
// q_out); stats may be null when only those are wanted.
// ---------------------------------------------------------------------------
__global__ void level_stats_kernel(const double *__restrict__ fine, const double *__restrict__ quarters,
                                   int64_t n_samples, int n_eps, double *__restrict__ stats,
                                   double *__restrict__ y_out, double *__restrict__ q_out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_eps) return;
    double sy = 0.0, syy = 0.0, sq = 0.0, sqq = 0.0;
    for (int64_t s = 0; s < n_samples; ++s) {
        const double qf = fine[s * n_eps + j];
        double y = qf;
        if (quarters) {
            const double *q = quarters + s * 4 * (int64_t)n_eps;
            y = qf - 0.25 * (q[j] + q[n_eps + j] + q[2 * n_eps + j] + q[3 * n_eps + j]);
        }
        if (y_out) y_out[s * n_eps + j] = y;
        if (q_out) q_out[s * n_eps + j] = qf;
        sy += y;
        syy += y * y;
        sq += qf;
        sqq += qf * qf;
    }
    if (!stats) return;
    stats[j] += sy;
    stats[n_eps + j] += syy;
    stats[2 * n_eps + j] += sq;
    stats[3 * n_eps + j] += sqq;
}

hipError_t launch_level_stats(const double *fine, const double *quarters, int64_t n_samples, int n_eps,
                              double *stats, hipStream_t s, double *y_out, double *q_out) {
    if (n_eps == 0 || n_samples == 0) return hipSuccess;
    const int threads = 128;
    hipLaunchKernelGGL(level_stats_kernel, dim3((n_eps + threads - 1) / threads), dim3(threads), 0, s, fine, quarters,
                       n_samples, n_eps, stats, y_out, q_out);
    return hipGetLastError();
}

}  // namespace mlmc
