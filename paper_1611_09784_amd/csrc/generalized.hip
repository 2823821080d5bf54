// Generalised Hermitian-definite eigenproblem H c = E S c of a non-orthogonal
// basis (Section 3.1, with the overlap matrix S), reduced to a standard one
// on the GPU for a batch of matrices in device memory:
//   1. Cholesky S = L L^H, blocked by 16-column panels (Golub & Van Loan,
//      Alg. 4.2.1 on the diagonal block, then L21 = A21 L11^{-H} and the
//      rank-16 update S22 -= L21 L21^H on the matrix cores);
//   2. C = L^{-1} H L^{-H} by the blocked two-sided algorithm (Golub & Van
//      Loan Sec. 8.7.2, the LAPACK hegst ordering): per panel
//        C11 = L11^{-1} A11 L11^{-H},  A21 <- A21 L11^{-H} - 1/2 L21 C11,
//        A22 -= A21 L21^H + L21 A21^H,  A21 <- A21 - 1/2 L21 C11,
//        C21 = L22^{-1} A21 (forward substitution by 16-row blocks).
// Only lower triangles are read and written; C then goes through the
// standard eigensolver.  The inverses of the 16 x 16 diagonal blocks of L are
// kept in the workspace after the band array of the two-stage layout.
#include "twostage_common.hpp"

namespace mlmc {

constexpr int kGenThreads = 256;
constexpr int kTrsmThreads = 512;

template <typename T>
size_t generalized_work_elems(int64_t ld) {
    return tridiag_twostage_work_elems<T>(ld) + (size_t)((ld + kB - 1) / kB) * kB * kB;
}

template <typename T>
__device__ __forceinline__ cpx<T> *linv_blocks(const TwoView<T> &w, int64_t) {
    // The Hermitian product's partial products start here too; they are
    // written only by the standard reduction of C, after the last use of L^-1.
    return w.zp;
}

// Panel p of the Cholesky factorisation; S22 -= L21 L21^H follows as a
// rank-2k update with V = L21, W = L21 / 2.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void chol_panel_kernel(cpx<T> *__restrict__ Sall, int64_t ld,
                                                                  const int32_t *__restrict__ n_in,
                                                                  cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ cpx<T> A[kB][kB + 1];
    __shared__ cpx<T> Li[kB][kB + 1];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    if (n < 0 || n > ld || p >= n) return;
    const int nb = min(kB, n - p);
    const int t = threadIdx.x, r0 = t % kB, c0 = t / kB;
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> *S = Sall + u * ld * ld;
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *Linv = linv_blocks(w, ld) + (int64_t)(p / kB) * kB * kB;
    A[r0][c0] = (r0 < nb && c0 <= r0) ? S[(p + r0) + (int64_t)(p + c0) * ld] : zero;
    __syncthreads();
    for (int j = 0; j < nb; ++j) {  // diagonal block: column j, then the trailing outer product
        if (t == 0) A[j][j] = {(T)sqrt((double)A[j][j].re), T(0)};  // not positive: NaN propagates
        __syncthreads();
        if (t > j && t < nb) A[t][j] = c_scale((T)(1.0 / (double)A[j][j].re), A[t][j]);
        __syncthreads();
        if (r0 > j && c0 > j && c0 <= r0 && r0 < nb) A[r0][c0] = c_sub(A[r0][c0], c_mulc(A[r0][j], A[c0][j]));
        __syncthreads();
    }
    if (t < kB) {  // column t of L11^{-1} by forward substitution (identity beyond nb)
        cpx<T> x[kB];
#pragma unroll
        for (int i = 0; i < kB; ++i) {
            cpx<T> v = (i == t) ? cpx<T>{T(1), T(0)} : zero;
#pragma unroll
            for (int k = 0; k < i; ++k) v = c_sub(v, c_mul(A[i][k], x[k]));
            x[i] = (i < nb) ? c_scale((T)(1.0 / (double)A[i][i].re), v) : ((i == t) ? cpx<T>{T(1), T(0)} : zero);
        }
#pragma unroll
        for (int i = 0; i < kB; ++i) Li[i][t] = x[i];
    }
    __syncthreads();
    if (r0 < nb && c0 <= r0) S[(p + r0) + (int64_t)(p + c0) * ld] = A[r0][c0];
    Linv[r0 * kB + c0] = Li[r0][c0];
    // panel below the diagonal block: L21 = A21 L11^{-H}
    for (int r = p + kB + t; r < n; r += kGenThreads) {
        cpx<T> a[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) a[k] = S[r + (int64_t)(p + k) * ld];
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            cpx<T> l = zero;
#pragma unroll
            for (int k = 0; k <= j; ++k) l = c_add(l, c_mulc(a[k], Li[j][k]));
            S[r + (int64_t)(p + j) * ld] = l;
            w.V[(int64_t)j * ld + r] = l;
            w.W[(int64_t)j * ld + r] = c_scale(T(0.5), l);
        }
    }
}

// First half of panel p of the two-sided reduction: C11 = L11^{-1} A11
// L11^{-H} in place, A21 <- A21 L11^{-H} - 1/2 L21 C11; V = L21, W = A21 for
// the rank-2k update of A22 that follows.
template <typename T>
__global__ __launch_bounds__(kGenThreads) void hegst_a_kernel(cpx<T> *__restrict__ Hall,
                                                               const cpx<T> *__restrict__ Sall, int64_t ld,
                                                               const int32_t *__restrict__ n_in,
                                                               cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ cpx<T> A11[kB][kB + 1], Li[kB][kB + 1], Tm[kB][kB + 1];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    if (n < 0 || n > ld || p >= n) return;
    const int nb = min(kB, n - p);
    const int t = threadIdx.x, r0 = t % kB, c0 = t / kB;
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> *H = Hall + u * ld * ld;
    const cpx<T> *S = Sall + u * ld * ld;
    const TwoView<T> w(wall, stride, ld, u);
    const cpx<T> *Linv = linv_blocks(w, ld) + (int64_t)(p / kB) * kB * kB;
    Li[r0][c0] = Linv[r0 * kB + c0];
    {
        cpx<T> a = zero;
        if (r0 < nb && c0 < nb)
            a = (r0 >= c0) ? H[(p + r0) + (int64_t)(p + c0) * ld] : c_conj(H[(p + c0) + (int64_t)(p + r0) * ld]);
        A11[r0][c0] = a;
    }
    __syncthreads();
    {
        cpx<T> acc = zero;
#pragma unroll
        for (int k = 0; k < kB; ++k) acc = c_add(acc, c_mul(Li[r0][k], A11[k][c0]));
        Tm[r0][c0] = acc;
    }
    __syncthreads();
    {
        cpx<T> acc = zero;
#pragma unroll
        for (int k = 0; k < kB; ++k) acc = c_add(acc, c_mulc(Tm[r0][k], Li[c0][k]));
        if (r0 == c0) acc.im = T(0);
        A11[r0][c0] = acc;
    }
    __syncthreads();
    if (r0 < nb && c0 <= r0) H[(p + r0) + (int64_t)(p + c0) * ld] = A11[r0][c0];
    for (int r = p + kB + t; r < n; r += kGenThreads) {
        cpx<T> a[kB], l[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            a[k] = H[r + (int64_t)(p + k) * ld];
            l[k] = S[r + (int64_t)(p + k) * ld];
        }
#pragma unroll
        for (int j = 0; j < kB; ++j) {
            cpx<T> b = zero, q = zero;
#pragma unroll
            for (int k = 0; k <= j; ++k) b = c_add(b, c_mulc(a[k], Li[j][k]));
#pragma unroll
            for (int k = 0; k < kB; ++k) q = c_add(q, c_mul(l[k], A11[k][j]));
            b = c_sub(b, c_scale(T(0.5), q));
            H[r + (int64_t)(p + j) * ld] = b;
            w.V[(int64_t)j * ld + r] = l[j];
            w.W[(int64_t)j * ld + r] = b;
        }
    }
}

// Second half of panel p: A21 <- A21 - 1/2 L21 C11, then C21 = L22^{-1} A21.
// The rows below the panel are taken in segments of RPT * kTrsmThreads rows:
// thread t holds rows g + t + kTrsmThreads i (i < RPT) of segment g in
// registers.  The substitution runs over 16-row blocks q of L22: rows of
// earlier segments are already solved and stored in H, so their block of the
// solution is read back from H; a block inside the segment is first
// multiplied by the inverse of its diagonal block; then every row of the
// segment below the block subtracts L[r, q..q+15] times the block's solution.
template <typename T, int RPT>
__global__ __launch_bounds__(kTrsmThreads) void hegst_b_kernel(cpx<T> *__restrict__ Hall,
                                                                const cpx<T> *__restrict__ Sall, int64_t ld,
                                                                const int32_t *__restrict__ n_in,
                                                                cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ cpx<T> C11[kB][kB + 1], LiB[kB][kB + 1], X[kB][kB + 1];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB;
    if (n < 0 || n > ld || s >= n) return;
    const int t = threadIdx.x;
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> *H = Hall + u * ld * ld;
    const cpx<T> *S = Sall + u * ld * ld;
    const TwoView<T> w(wall, stride, ld, u);
    const cpx<T> *Lblk = linv_blocks(w, ld);
    if (t < kB * kB) {
        const int r0 = t % kB, c0 = t / kB;
        C11[r0][c0] = (r0 >= c0) ? H[(p + r0) + (int64_t)(p + c0) * ld] : c_conj(H[(p + c0) + (int64_t)(p + r0) * ld]);
        X[r0][c0] = zero;
    }
    __syncthreads();
    constexpr int kSeg = RPT * kTrsmThreads;
    for (int g = s; g < n; g += kSeg) {
        cpx<T> a[RPT][kB];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = g + t + kTrsmThreads * i;
            const bool own = r < n;
            cpx<T> l[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                a[i][k] = own ? H[r + (int64_t)(p + k) * ld] : zero;
                l[k] = own ? S[r + (int64_t)(p + k) * ld] : zero;
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                cpx<T> q = zero;
#pragma unroll
                for (int k = 0; k < kB; ++k) q = c_add(q, c_mul(l[k], C11[k][j]));
                a[i][j] = c_sub(a[i][j], c_scale(T(0.5), q));
            }
        }
        for (int q0 = s; q0 < n; q0 += kB) {
            const int qb = min(kB, n - q0);
            if (q0 < g) {
                // a block solved in an earlier segment: its solution is in H
                if (t < kB * kB) {
                    const int r0 = t % kB, c0 = t / kB;
                    X[r0][c0] = (r0 < qb) ? H[(q0 + r0) + (int64_t)(p + c0) * ld] : zero;
                }
                __syncthreads();
            } else {
                if (t < kB * kB) LiB[t % kB][t / kB] = Lblk[(int64_t)(q0 / kB) * kB * kB + (t % kB) * kB + t / kB];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = g + t + kTrsmThreads * i;
                    if (r >= q0 && r < q0 + qb) {
#pragma unroll
                        for (int j = 0; j < kB; ++j) X[r - q0][j] = a[i][j];
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = g + t + kTrsmThreads * i;
                    if (r >= q0 && r < q0 + qb) {
#pragma unroll
                        for (int j = 0; j < kB; ++j) {
                            cpx<T> x = zero;
#pragma unroll
                            for (int k = 0; k < kB; ++k) x = c_add(x, c_mul(LiB[r - q0][k], X[k][j]));
                            a[i][j] = x;
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const int r = g + t + kTrsmThreads * i;
                    if (r >= q0 && r < q0 + qb) {
#pragma unroll
                        for (int j = 0; j < kB; ++j) X[r - q0][j] = a[i][j];
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int r = g + t + kTrsmThreads * i;
                if (r >= q0 + qb && r < n) {
                    for (int k = 0; k < qb; ++k) {
                        const cpx<T> lk = S[r + (int64_t)(q0 + k) * ld];
#pragma unroll
                        for (int j = 0; j < kB; ++j) a[i][j] = c_sub(a[i][j], c_mul(lk, X[k][j]));
                    }
                }
            }
            __syncthreads();
            if (q0 + qb >= g + kSeg) break;  // the rest of the rows belong to later segments
        }
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
            const int r = g + t + kTrsmThreads * i;
            if (r < n) {
#pragma unroll
                for (int j = 0; j < kB; ++j) H[r + (int64_t)(p + j) * ld] = a[i][j];
            }
        }
        __syncthreads();  // this segment's solution is in H before the next segment reads it
    }
}

template <typename T>
hipError_t launch_cholesky_reduce(cpx<T> *H, cpx<T> *S, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                  hipStream_t s) {
    if (batch == 0 || ld == 0) return hipSuccess;
    if (ld > kGenMax) return hipErrorInvalidValue;
    const int64_t stride = (int64_t)generalized_work_elems<T>(ld);
    const unsigned B = (unsigned)batch;
    for (int p = 0; p < ld; p += kB) {
        hipLaunchKernelGGL(chol_panel_kernel<T>, dim3(B), dim3(kGenThreads), 0, s, S, ld, n_in, work, stride, p);
        if (p + kB < ld) {
            const hipError_t err = launch_rank2k_update<T>(S, ld, n_in, batch, work, stride, p, 1, s);
            if (err != hipSuccess) return err;
        }
    }
    for (int p = 0; p < ld; p += kB) {
        hipLaunchKernelGGL(hegst_a_kernel<T>, dim3(B), dim3(kGenThreads), 0, s, H, S, ld, n_in, work, stride, p);
        if (p + kB < ld) {
            hipError_t err = launch_rank2k_update<T>(H, ld, n_in, batch, work, stride, p, 1, s);
            if (err != hipSuccess) return err;
            if (ld - p - kB <= kTrsmThreads)
                hipLaunchKernelGGL((hegst_b_kernel<T, 1>), dim3(B), dim3(kTrsmThreads), 0, s, H, S, ld, n_in, work,
                                   stride, p);
            else
                hipLaunchKernelGGL((hegst_b_kernel<T, 2>), dim3(B), dim3(kTrsmThreads), 0, s, H, S, ld, n_in, work,
                                   stride, p);
        }
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

template size_t generalized_work_elems<double>(int64_t);
template size_t generalized_work_elems<float>(int64_t);
template hipError_t launch_cholesky_reduce<double>(cpx<double> *, cpx<double> *, int64_t, const int32_t *, int64_t,
                                                   cpx<double> *, hipStream_t);
template hipError_t launch_cholesky_reduce<float>(cpx<float> *, cpx<float> *, int64_t, const int32_t *, int64_t,
                                                  cpx<float> *, hipStream_t);

}  // namespace mlmc
