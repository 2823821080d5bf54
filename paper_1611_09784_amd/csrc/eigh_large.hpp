// Eigenvectors of matrices above the LDS-resident size: stage 1
// keeps each panel's block reflector (V_p, T_p), inverse iteration runs on
// the band matrix of half-width kB that stage 1 leaves in the lower triangle
// of H, and the band's eigenvectors go back through the kept reflectors.
#pragma once
#include <algorithm>

#include "twostage_common.hpp"

namespace mlmc {

// Largest side of the banded eigenvector path.
constexpr int kEighLargeMax = 4096;

// Elements of one matrix's reflector store: per panel V_p [kB][ld] (rows
// below the panel's band; the rest untouched) and T_p [kB][kB] row-major.
inline int64_t eigh_keep_elems(int64_t ld) { return ((ld + kB - 1) / kB) * (kB * ld + kB * kB); }

// Stage 1 as launch_band_reduce (32-row update tiles) that also copies every
// panel's V_p, T_p into keep + u * keep_stride (keep_stride >= eigh_keep_elems(ld)).
template <typename T>
hipError_t launch_band_reduce_keep(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                   hipStream_t s, int64_t stride, const int64_t *offs, cpx<T> *keep, int64_t keep_stride);

// Inverse iteration: one wavefront per cluster, its LU factors in a slice of
// device scratch of band_ii_wave_bytes(ld).
// Scratch: U rows of 2 kB + 1 entries, kB multipliers and a pivot index per
// elimination step, for ld + kIIStep steps (whole blocks of kIIStep), and the
// iterated vector.  LDS: the (kB + 1) x (2 kB + 1) elimination window,
// kIIStep steps of incoming band rows and of outgoing factors, a ring of
// kIIYRing entries of the iterated vector.
constexpr int kIIStep = 4;
constexpr int kIIYRing = 64;
inline int64_t band_ii_wave_bytes(int64_t ld) {
    return ((ld + kIIStep) * ((3 * kB + 1) * 16 + 4) + ld * 16 + 255) / 256 * 256;
}
inline int64_t band_ii_lds_bytes(int64_t) {
    return 16 * ((kB + 1) * (2 * kB + 1) + kIIStep * (2 * (2 * kB + 1) + kB) + kIIYRing) + 4 * kIIStep;
}
// Wavefronts (scratch slices) of one launch: what the CUs' LDS holds at once
// (at most four per SIMD), and no more than the eigenvalues of the batch; the
// launch takes fewer when registers allow fewer per CU.
inline int64_t band_ii_waves(int64_t ld, int64_t batch) {
    const int64_t per_cu = std::min<int64_t>(16, (160 * 1024) / band_ii_lds_bytes(ld));
    return std::max<int64_t>(1, std::min<int64_t>(256 * per_cu, batch * ld));
}
inline size_t band_ii_scratch_bytes(int64_t ld, int64_t batch) {
    return (size_t)band_ii_waves(ld, batch) * (size_t)band_ii_wave_bytes(ld);
}

// Matrix u's leading ld x n_u block (offs: element offsets, NULL: u ld^2) to
// dst + u ld^2.
template <typename T>
hipError_t launch_gather_matrices(const cpx<T> *H, int64_t ld, const int64_t *offs, const int32_t *n_in,
                                  int64_t batch, cpx<T> *dst, hipStream_t s);

// Columns 0..n_u-1 of V_u (complex128, column-major, ldv, matrix u at u ldv^2):
// unit eigenvectors of the band matrix in H (matrix u at u ld^2, complex128 or
// complex64, widened) for the ascending eigenvalues w_in[u ld + i];
// w_out[u ldw + i]: their Rayleigh quotients, ascending (NaN for i < ld when
// n_u is outside [0, ld]).
template <typename T>
hipError_t launch_band_inverse_iteration(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch,
                                         const double *w_in, double *w_out, int64_t ldw, cpx<double> *V, int64_t ldv,
                                         void *scratch, hipStream_t s);

// Panels stage 1 runs for side bound ld (p = 0, 16, ... while p + kB + 1 < ld),
// and groups of four of them.
inline int eigh_panels(int64_t ld) { return ld > kB + 1 ? (int)((ld - kB - 2) / kB + 1) : 0; }
inline int eigh_panel_groups(int64_t ld) { return (eigh_panels(ld) + 3) / 4; }
// Complex128 elements of one matrix's compound T factors (64 x 64 per group).
inline int64_t eigh_group_t_elems(int64_t ld) { return (int64_t)eigh_panel_groups(ld) * 64 * 64; }

// V_u <- Q_u V_u, Q_u = (I - V_0 T_0 V_0^H) ... (I - V_P T_P V_P^H) from the
// reflector store (complex128 or complex64, widened), four panels at a time
// (tg: batch * eigh_group_t_elems(ld) complex128 elements of scratch).
template <typename T>
hipError_t launch_panel_backtransform(const cpx<T> *keep, int64_t keep_stride, int64_t ld, const int32_t *n_in,
                                      int64_t batch, cpx<double> *V, int64_t ldv, cpx<double> *tg, hipStream_t s);

// X_u <- L_u^{-H} X_u for the columns and rows 0..n_u-1 (L_u lower
// triangular with a real positive diagonal, column-major, ld; X_u
// column-major, ldx), computed in double.
template <typename T>
hipError_t launch_trsm_lh(const cpx<T> *L, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *X, int64_t ldx,
                          hipStream_t s);

// The leading n_u x n_u block of each complex128 matrix of src (ld apart),
// rounded to complex64, into dst (ldv apart).
hipError_t launch_narrow_vectors(const cpx<double> *src, int64_t ld, const int32_t *n_in, int64_t batch,
                                 cpx<float> *dst, int64_t ldv, hipStream_t s);

}  // namespace mlmc
