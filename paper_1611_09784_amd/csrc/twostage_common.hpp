// Shared pieces of the two-stage Householder tridiagonalisation (dense ->
// band of half-width kB in band_reduce.hip, band -> tridiagonal in
// band_chase.hip): band geometry, the per-matrix workspace, cross-lane
// reductions and the Householder reflector.
#pragma once

#include <utility>

#include "device_common.hpp"

namespace mlmc {

constexpr int kB = 16;                 // band half-width = panel width
constexpr int kBandLd = 2 * kB + 1;    // stored sub-diagonals per column (incl. diagonal)

// Per-matrix workspace (complex elements): V [kB][ld], X [kB][ld], W [kB][ld],
// T [kB][kB], band [ld + 1][kBandLd], then the Hermitian product's
// per-row-block partial products [ceil(ld / 16)][kB][kB] (row blocks of 16,
// 32 or 64 rows).  The band's last
// column is a discard slot: lanes with nothing to store write there, so that
// every store of a block is issued unconditionally.  Stage 1 never touches
// the band and the chase touches nothing else.
template <typename T>
size_t tridiag_twostage_work_elems(int64_t ld) {
    return (size_t)(3 * kB) * (size_t)ld + (size_t)kB * kB + (size_t)kBandLd * (size_t)(ld + 1) +
           (size_t)((ld + 15) / 16) * kB * kB;
}
// Offset of the partial products within a matrix's workspace.
inline int64_t hemm_partials_offset(int64_t ld) { return 3 * kB * ld + kB * kB + kBandLd * (ld + 1); }

template <typename T>
struct TwoView {
    cpx<T> *V, *X, *W, *Tm, *band, *zp;
    __device__ TwoView(cpx<T> *wall, int64_t stride, int64_t ld, int64_t u) {
        cpx<T> *b = wall + u * stride;
        V = b;
        X = V + (int64_t)kB * ld;
        W = X + (int64_t)kB * ld;
        Tm = W + (int64_t)kB * ld;
        band = Tm + kB * kB;
        zp = band + kBandLd * (ld + 1);
    }
};

template <typename T>
__device__ __forceinline__ cpx<T> *hemm_partials(const TwoView<T> &w, int64_t) {
    return w.zp;
}

// Element offset of matrix u of a batch: offs[u] in a ragged layout, else
// u ld^2 (matrices ld x ld apart).
__device__ __forceinline__ int64_t mat_offset(const int64_t *offs, int64_t u, int64_t ld) {
    return offs ? offs[u] : u * ld * ld;
}

// Componentwise select (a select of whole structs can become a select of
// their addresses, which forces register arrays into scratch memory).
template <typename T>
__device__ __forceinline__ cpx<T> csel(bool c, cpx<T> a, cpx<T> b) {
    return {c ? a.re : b.re, c ? a.im : b.im};
}

template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> a, int src) {
    return {__shfl(a.re, src, 64), __shfl(a.im, src, 64)};
}

// Cross-lane moves without the LDS crossbar.  A wavefront is four rows of 16
// lanes.  Within a row: DPP quad permutations and the half-row / row mirrors.
// Across rows: the permlane swaps, which exchange odd with even 16-lane rows
// (16) or the upper with the lower 32 lanes (32) of two registers; swapping a
// register with itself leaves each lane with its own word and its partner's.
// Each op is applied to the 32-bit words of a float or double.
template <int CTRL>
__device__ __forceinline__ int dpp_word(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(dpp_word<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_word<CTRL>((int)b), hi = dpp_word<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// Returns (own, partner) ordered as the swap leaves them in its two registers.
template <bool ROWS32>
__device__ __forceinline__ void swap_word(int v, int &a, int &b) {
    if constexpr (ROWS32) {
        const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        a = (int)q[0];
        b = (int)q[1];
    } else {
        const auto q = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        a = (int)q[0];
        b = (int)q[1];
    }
}
template <bool ROWS32>
__device__ __forceinline__ void swap_pair(float x, float &a, float &b) {
    int ia, ib;
    swap_word<ROWS32>(__float_as_int(x), ia, ib);
    a = __int_as_float(ia);
    b = __int_as_float(ib);
}
template <bool ROWS32>
__device__ __forceinline__ void swap_pair(double x, double &a, double &b) {
    const long long w = __double_as_longlong(x);
    int alo, blo, ahi, bhi;
    swap_word<ROWS32>((int)w, alo, blo);
    swap_word<ROWS32>((int)(w >> 32), ahi, bhi);
    a = __longlong_as_double(((long long)ahi << 32) | (unsigned)alo);
    b = __longlong_as_double(((long long)bhi << 32) | (unsigned)blo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- 7 - i within each 8
constexpr int kDppMirror = 0x140;     // lane i <- 15 - i within each 16

// Sum over the 16 lanes of each row; every lane of the row gets the same bits
// (each step adds a lane's value and its partner's, which are equal pairwise).
template <typename T>
__device__ __forceinline__ T row_sum(T x) {
    x += dpp<kDppXor1>(x);
    x += dpp<kDppXor2>(x);
    x += dpp<kDppHalfMirror>(x);
    return x + dpp<kDppMirror>(x);
}
// Sum over the four rows at each lane position.
template <typename T>
__device__ __forceinline__ T col_sum(T x) {
    T a, b;
    swap_pair<false>(x, a, b);
    x = a + b;
    swap_pair<true>(x, a, b);
    return a + b;
}
// Row 0's value at each lane position, in every row.
template <typename T>
__device__ __forceinline__ T from_row0(T x) {
    T a, b;
    swap_pair<false>(x, a, b);  // a: rows (0, 0, 2, 2)
    swap_pair<true>(a, x, b);   // x: rows (0, 0, 0, 0)
    return x;
}
template <typename T>
__device__ __forceinline__ T lane0(T x);
template <>
__device__ __forceinline__ float lane0(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
}
template <>
__device__ __forceinline__ double lane0(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, 0), hi = __builtin_amdgcn_readlane((int)(b >> 32), 0);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1/x and 1/sqrt(x) for x >= kRefinedMin: the hardware estimates refined by
// two Newton steps each (quadratic convergence to within about an ulp).
constexpr double kRefinedMin = 1e-290;
__device__ __forceinline__ double rcp_refined(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double h = fma(-x, r, 1.0);
    r = fma(r, h, r);
    h = fma(-x, r, 1.0);
    return fma(r, h, r);
}
__device__ __forceinline__ double rsq_refined(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = fma(-x * y, y, 1.0);  // 1 - x y^2
        y = fma(0.5 * y, h, y);
    }
    return y;
}

// Reflector of x (norm^2 nrm2, first entry x0): v0 = x0 - alpha with
// alpha = -e^{i arg x0} |x|, tau = 2 / |v|^2 = 1 / (|x| (|x| + |x0|)) (0 when
// x = 0).  Square roots and quotients come from the refined reciprocal
// estimates; inputs below kRefinedMin take the exact operations.
template <typename T>
__device__ __forceinline__ void make_reflector(double nrm2, cpx<T> x0, T &tau, cpx<T> &v0, cpx<T> &alpha) {
    tau = T(0);
    v0 = x0;
    alpha = x0;
    if (nrm2 > 0.0) {
        const double xr = (double)x0.re, xi = (double)x0.im, ax2 = xr * xr + xi * xi;
        const double xnorm = nrm2 >= kRefinedMin ? nrm2 * rsq_refined(nrm2) : sqrt(nrm2);
        double pr = 1.0, pi = 0.0, ax0 = 0.0;
        if (ax2 >= kRefinedMin) {
            const double inv = rsq_refined(ax2);
            ax0 = ax2 * inv;
            pr = xr * inv;
            pi = xi * inv;
        } else if (ax2 > 0.0) {
            ax0 = sqrt(ax2);
            pr = xr / ax0;
            pi = xi / ax0;
        }
        const double vh = xnorm * (xnorm + ax0);  // |v|^2 / 2
        tau = (T)(vh >= kRefinedMin ? rcp_refined(vh) : 1.0 / vh);
        v0 = {(T)(xr + pr * xnorm), (T)(xi + pi * xnorm)};
        alpha = {(T)(-pr * xnorm), (T)(-pi * xnorm)};
    }
}

}  // namespace mlmc
