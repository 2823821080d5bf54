// Internal declarations of the gfx950 library behind include/mlmc.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "mlmc.h"

namespace mlmc {

// ---------------------------------------------------------------------------
// Complex arithmetic on interleaved (re, im) pairs.
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> c_add(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_sub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_mul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> c_mulc(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cpx<T> c_cmul(cpx<T> a, cpx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> c_conj(cpx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> c_scale(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ T c_abs2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// Device copy of a lattice (built once by mlmc_lattice_create).
// hop_i[h] = (R1, R2, from, to); hop_f[h] = (re, im, d1, d2) with
// d = R + frac(to) - frac(from) the unwrapped displacement in units of a1, a2.
// ---------------------------------------------------------------------------
struct DevLattice {
    const int4 *hop_i;
    const double4 *hop_f;
    const int32_t *orb_group;
    const uint8_t *removable;
    int n_orb;
    int n_groups;
    int n_hops;
    uint32_t lattice_id;
    double cell_area;
    // overlap table of a non-orthogonal basis (n_ovl == 0: orthogonal)
    const int4 *ovl_i;
    const double4 *ovl_f;
    int n_ovl;
};

// Largest pristine matrix side handled by the LDS-resident fused kernel.
constexpr int kSmallMaxF64 = 128;
constexpr int kSmallMaxF32 = 180;
// Largest matrix side of the device-memory reduction (the largest pristine
// supercell the assembly accepts).
constexpr int kLargeMaxF64 = 16384;
constexpr int kLargeMaxF32 = 16384;
// Gaussian smoothing is evaluated for |x| < kGaussCut and is exactly 0 / 1 beyond.
constexpr double kGaussCut = 10.0;

__host__ __device__ constexpr int64_t packed_size(int64_t n) { return n * (n + 1) / 2; }

// ---------------------------------------------------------------------------
// Launchers (each returns hipGetLastError() of its launch).
// ---------------------------------------------------------------------------
hipError_t launch_sample_vacancies(const DevLattice &lat, int N, uint64_t threshold, uint64_t seed, uint64_t tag,
                                   int64_t first, int64_t n_samples, uint8_t *mask, hipStream_t s,
                                   const int64_t *first_dev = nullptr);
// *counter += delta on the device.
hipError_t launch_advance_counter(int64_t *counter, int64_t delta, hipStream_t s);
hipError_t launch_partition(int N, int G, const uint8_t *mask, int64_t n_samples, uint8_t *quarters, hipStream_t s);
hipError_t launch_kgrid(int kind, int K, double *kred, double *kweight, hipStream_t s);
// Number of points of a grid kind (K^2, or 3 K^2 for the three-rhombus lattice).
int kgrid_count(int kind, int K);

template <typename T>
hipError_t launch_assemble(const DevLattice &lat, int N, const uint8_t *masks, int64_t n_samples, const double *kred,
                           int n_k, cpx<T> *H, int64_t ld, int32_t *n_out, hipStream_t s, bool overlap = false,
                           bool lower = false);

// Fused LDS kernel: (assemble or load) -> Householder -> bisection -> eigenvalues.
template <typename T>
hipError_t launch_small_from_lattice(const DevLattice &lat, int N, const uint8_t *masks, int64_t n_samples,
                                     const double *kred, int n_k, double *w, int64_t ldw, int32_t *n_out,
                                     hipStream_t s);
template <typename T>
hipError_t launch_small_from_matrix(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *w,
                                    int64_t ldw, hipStream_t s, const int64_t *offs = nullptr);

// Eigenvalues and eigenvectors of LDS-resident matrices (ld <= the small
// path's bound): one workgroup per matrix, the reflectors kept in LDS,
// inverse iteration on the tridiagonal, V = Q D Z.  work: eigh_work_bytes.
template <typename T>
hipError_t launch_eigh_small(const cpx<T> *H, int64_t ld, const int64_t *offs, const int32_t *n_in, int64_t batch,
                             double *w, int64_t ldw, cpx<T> *V, int64_t ldv, double *work, hipStream_t s);
inline size_t eigh_work_bytes(int64_t ld, int64_t batch) {
    return sizeof(double) * (size_t)((((ld * ld + 1) & ~int64_t(1)) + 6 * ld * ld) * batch);
}

// Per-kernel timing inside launchers that issue several kernels: when the
// calling thread enqueues work for a context whose launch timer is on, an
// event pair brackets `launch` on stream s under `name`; otherwise `launch`
// just runs.  `launch` enqueues one kernel and returns its launch status.
hipError_t timed_sub(const char *name, hipStream_t s, hipError_t (*launch)(void *), void *arg);
template <typename F>
inline hipError_t timed_call(const char *name, hipStream_t s, F &&f) {
    using Fn = typename std::remove_reference<F>::type;
    return timed_sub(name, s, [](void *p) { return (*static_cast<Fn *>(p))(); }, static_cast<void *>(&f));
}

// Two-stage reduction to tridiagonal form.  Stage 1 (launch_band_reduce):
// dense -> band of half-width 16, in place in H (lower triangle).  Stage 2
// (launch_band_chase): band -> tridiagonal (d, e) by bulge chasing.  Both use
// the per-matrix workspace of tridiag_twostage_work_elems complex elements,
// in disjoint parts (stage 1: V, X, W, T and the Hermitian product's
// partials; the chase: the band), so that the chase of one batch may run
// beside stage 1 of another batch on the same workspace.  The chase runs on
// at most max_blocks workgroups (one per CU; 0: one per matrix).  offs:
// element offset of each matrix in H (NULL: u ld^2).  stride:
// elements between consecutive matrices' workspaces (0: the two-stage
// layout's own size; a caller whose other kernels use a larger per-matrix
// workspace passes that, so that their parts stay disjoint).
// upd_rows: row height of the rank-2k update's tiles, 32 (32 x 64 tiles with
// 16 KiB of LDS, small enough to share a CU with a chase workgroup) or 64
// (64 x 64 tiles, 64 KiB).
template <typename T>
hipError_t launch_band_reduce(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                              hipStream_t s, int64_t stride = 0, const int64_t *offs = nullptr, int upd_rows = 32);
template <typename T>
hipError_t launch_band_chase(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                             int64_t lde, cpx<T> *work, hipStream_t s, int64_t max_blocks = 0, int64_t stride = 0,
                             const int64_t *offs = nullptr);
template <typename T>
size_t tridiag_twostage_work_elems(int64_t ld);
// Rank-2k update A22 -= V W^H + W V^H below panel p (see band_reduce.hip).
template <typename T>
hipError_t launch_rank2k_update(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                int64_t stride, int p, int min_m, hipStream_t s);

// Generalised problem H c = E S c (generalized.hip): S = L L^H in place in S
// (lower), H <- L^{-1} H L^{-H} in place (lower triangle).  Workspace per
// matrix: generalized_work_elems complex elements.  Supported for
// ld <= kGenMax.
constexpr int kGenMax = 2048;
template <typename T>
size_t generalized_work_elems(int64_t ld);
template <typename T>
hipError_t launch_cholesky_reduce(cpx<T> *H, cpx<T> *S, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                  hipStream_t s);

// Sturm-count bisection of (d, e) -> ascending eigenvalues; at most
// max_blocks workgroups (0: one per matrix).  e is overwritten when ld_max
// exceeds the LDS staging limit (it is squared in place).
hipError_t launch_bisect(const double *d, double *e, int64_t lde, const int32_t *n_in, int64_t batch,
                         int64_t ld_max, double *w, int64_t ldw, hipStream_t s, int64_t max_blocks = 0);

hipError_t launch_idos(const double *w, int64_t ldw, const int32_t *n, int64_t n_samples, int n_k,
                       const double *kweight, double inv_area, const double *eps, int n_eps, double delta,
                       int smoother, double *out, hipStream_t s);
hipError_t launch_level_stats(const double *fine, const double *quarters, int64_t n_samples, int n_eps,
                              double *stats, hipStream_t s, double *y_out = nullptr, double *q_out = nullptr);

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed butterfly order within a wave, then
// waves summed in index order).  `scratch` holds >= 16 doubles in LDS.
// All threads of the block must call them; every thread gets the result.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += scratch[i];
    return r;
}
__device__ __forceinline__ double block_min(double v, double *scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_min(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double r = scratch[0];
    for (int i = 1; i < nw; ++i) r = fmin(r, scratch[i]);
    return r;
}
__device__ __forceinline__ double block_max(double v, double *scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double r = scratch[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, scratch[i]);
    return r;
}

}  // namespace mlmc
