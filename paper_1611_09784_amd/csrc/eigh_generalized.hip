// Eigenvectors of the generalised problem H c = E S c (the non-orthogonal
// basis of Section 3.1): with S = L L^H and C = L^{-1} H L^{-H} (the
// Cholesky reduction of the generalised eigenvalue path), C y = E y gives
// c = L^{-H} y, S-orthonormal when the y are orthonormal.  This file holds
// the back-substitution X <- L^{-H} X.
#include "eigh_large.hpp"

namespace mlmc {

namespace {

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cpx<double> ldw(const cpx<double> *p) {
    const d2v v = *reinterpret_cast<const d2v *>(p);
    return {v.x, v.y};
}
__device__ __forceinline__ cpx<double> ldw(const cpx<float> *p) {
    const f2v v = *reinterpret_cast<const f2v *>(p);
    return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stn(cpx<double> *p, cpx<double> x) { *reinterpret_cast<d2v *>(p) = d2v{x.re, x.im}; }
__device__ __forceinline__ void stn(cpx<float> *p, cpx<double> x) {
    *reinterpret_cast<f2v *>(p) = f2v{(float)x.re, (float)x.im};
}

// One workgroup per (matrix, 16 columns of X): L^H X = Y solved from the last
// block of 16 rows up.  For block b (rows r0 .. r1 - 1) thread (rr, j) sums
// conj(L[q][r0 + i]) X[q][j] over the solved rows q = r1 + rr + 16 s (the
// columns of L below the block are contiguous), the 16 lanes rr add up, and
// the 16 threads rr = 0 then solve the block's upper triangle L_bb^H in LDS,
// one column each, in double.
template <typename T>
__global__ __launch_bounds__(256) void trsm_lh_kernel(const cpx<T> *__restrict__ Lall, int64_t ld,
                                                      const int32_t *__restrict__ n_in, int64_t batch,
                                                      cpx<T> *__restrict__ Xall, int64_t ldx, int64_t tiles) {
    __shared__ cpx<double> Lbb[kB][kB + 1], Yb[kB][kB], Db[kB][kB];
    const int64_t u = blockIdx.x / tiles;
    const int tile = (int)(blockIdx.x % tiles);
    if (u >= batch) return;
    const int n = n_in[u];
    if (n < 1 || n > ld) return;
    const int col0 = tile * kB;
    if (col0 >= n) return;
    const cpx<T> *L = Lall + u * ld * ld;
    cpx<T> *X = Xall + u * ldx * ldx;
    const int t = threadIdx.x, rr = t & (kB - 1), j = t >> 4;
    const bool live = col0 + j < n;
    const int col = live ? col0 + j : col0;
    cpx<T> *xc = X + (int64_t)col * ldx;
    for (int r0 = (n - 1) / kB * kB; r0 >= 0; r0 -= kB) {
        const int r1 = min(r0 + kB, n), h = r1 - r0;
#pragma unroll
        for (int half = 0; half < kB; half += kB / 2) {
            cpx<double> acc[kB / 2];
#pragma unroll
            for (int i = 0; i < kB / 2; ++i) acc[i] = {0.0, 0.0};
            if (live) {
                for (int q = r1 + rr; q < n; q += kB) {
                    const cpx<double> x = ldw(xc + q);
#pragma unroll
                    for (int i = 0; i < kB / 2; ++i) {
                        const int c = min(r0 + half + i, n - 1);
                        acc[i] = c_add(acc[i], c_cmul(ldw(L + (int64_t)c * ld + q), x));
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < kB / 2; ++i) {
#pragma unroll
                for (int o = 1; o < kB; o <<= 1) {
                    acc[i].re += __shfl_xor(acc[i].re, o, 64);
                    acc[i].im += __shfl_xor(acc[i].im, o, 64);
                }
                if (rr == 0) Db[half + i][j] = acc[i];
            }
        }
        // the diagonal block (lower triangle) and the right-hand sides
        Lbb[rr][j] = (rr < h && j <= rr) ? ldw(L + (int64_t)(r0 + j) * ld + r0 + rr) : cpx<double>{0.0, 0.0};
        Yb[rr][j] = (rr < h && live) ? ldw(xc + r0 + rr) : cpx<double>{0.0, 0.0};
        __syncthreads();
        if (rr == 0 && live) {
            for (int i = h - 1; i >= 0; --i) {
                cpx<double> y = c_sub(Yb[i][j], Db[i][j]);
                for (int k = i + 1; k < h; ++k) y = c_sub(y, c_cmul(Lbb[k][i], Yb[k][j]));
                const double dii = Lbb[i][i].re;  // the Cholesky factor's diagonal is real and positive
                Yb[i][j] = {y.re / dii, y.im / dii};
            }
        }
        __syncthreads();
        if (rr < h && live) stn(xc + r0 + rr, Yb[rr][j]);
        __syncthreads();  // the block's rows are read by the next block's sums
    }
}

}  // namespace

template <typename T>
hipError_t launch_trsm_lh(const cpx<T> *L, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *X, int64_t ldx,
                          hipStream_t s) {
    if (batch == 0 || ld == 0) return hipSuccess;
    const int64_t tiles = (ld + kB - 1) / kB;
    hipLaunchKernelGGL(trsm_lh_kernel<T>, dim3((unsigned)(batch * tiles)), dim3(256), 0, s, L, ld, n_in, batch, X, ldx,
                       tiles);
    return hipGetLastError();
}

template hipError_t launch_trsm_lh<double>(const cpx<double> *, int64_t, const int32_t *, int64_t, cpx<double> *,
                                           int64_t, hipStream_t);
template hipError_t launch_trsm_lh<float>(const cpx<float> *, int64_t, const int32_t *, int64_t, cpx<float> *, int64_t,
                                          hipStream_t);

}  // namespace mlmc
