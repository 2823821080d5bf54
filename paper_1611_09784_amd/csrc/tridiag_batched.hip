// Batched blocked Householder tridiagonalisation of Hermitian matrices held
// in device memory (lower triangle read and written only).
//
// All matrices of a batch advance through the columns in lockstep, one
// column per pair of launches, so that the bandwidth-bound part of every
// column (a Hermitian matrix-vector product over the trailing lower
// triangle) runs with the whole GPU's parallelism, while the short serial
// part of a column (finishing reflector j, bringing column j+1 up to date and
// forming reflector j+1) is paid once per column for the whole batch.
//
// Columns are grouped in panels of kPanel.  Inside a panel the trailing
// matrix A is not modified: the current matrix is A - V W^H - W V^H with the
// panel's reflector vectors v (columns of V) and w (columns of W), so
//   p = tau (A v - V (W^H v) - W (V^H v)),   w = p - (tau/2)(v^H p) v,
// and after the panel the trailing lower triangle receives the rank-2*kPanel
// update once (the blocked form of the two-sided Householder reduction).
//
// Kernels (per column j = j0 + i of panel j0):
//   start_kernel   column j0 (i = 0) up to date -> reflector j0
//   matvec_kernel  A v over the lower triangle; one wavefront per 16-column
//                  strip walks the strip in 64-row tiles, keeps the column
//                  sums in registers and writes one row partial per tile
//   finish_kernel  sums the partials in a fixed order, applies the panel
//                  corrections, stores v_j and w_j; then brings column j+1 up
//                  to date and forms reflector j+1 (if it is in the panel)
//   update_kernel  rank-2*kPanel update of the trailing lower triangle
//   tail_kernel    the last 2x2 block
// All sums have a fixed order, so the result does not depend on the batch.
#include "device_common.hpp"

namespace mlmc {

constexpr int kPanel = 16;
constexpr int kTileRows = 64;
constexpr int kStripCols = 16;
constexpr int kMvWaves = 4;
constexpr int kSerThreads = 256;
constexpr int kUpdCols = 16;

__host__ __device__ inline int64_t strips_of(int64_t m) { return (m + kStripCols - 1) / kStripCols; }

// Per-matrix workspace, in complex elements:
//   V [kPanel][ld], W [kPanel][ld], vcur [ld], ycol [ld], rowpart [strips(ld)][ld], tau (1 element)
template <typename T>
size_t tridiag_batched_work_elems(int64_t ld) {
    return (size_t)(2 * kPanel + 2 + strips_of(ld)) * (size_t)ld + 1;
}

template <typename T>
struct BatchedView {
    cpx<T> *V, *W, *vcur, *ycol, *rowpart, *tau;
    __device__ BatchedView(cpx<T> *wall, int64_t stride, int64_t ld, int64_t u) {
        cpx<T> *b = wall + u * stride;
        V = b;
        W = b + (int64_t)kPanel * ld;
        vcur = W + (int64_t)kPanel * ld;
        ycol = vcur + ld;
        rowpart = ycol + ld;
        tau = rowpart + strips_of(ld) * ld;
    }
};

template <typename T>
__device__ __forceinline__ cpx<T> shfl_xor_c(cpx<T> a, int m) {
    return {__shfl_xor(a.re, m, 64), __shfl_xor(a.im, m, 64)};
}

// Bring column j (rows j..n-1) up to date with the first `ip` reflectors of
// the panel, record d_j and e_j, and form reflector j: vcur[r] for r > j and
// tau.  `corr` holds >= 2*kPanel complex values of LDS, `red` 32 doubles.
template <typename T>
__device__ void start_column(const cpx<T> *__restrict__ H, int64_t ld, int n, int j, int ip, const BatchedView<T> &w,
                             double *d, double *e, cpx<T> *corr, double *red) {
    const int t = threadIdx.x;
    if (t < 2 * ip) corr[t] = (t < ip) ? w.V[(int64_t)t * ld + j] : w.W[(int64_t)(t - ip) * ld + j];
    __syncthreads();
    double np = 0.0;
    cpx<T> x0 = {T(0), T(0)};
    for (int r = j + t; r < n; r += kSerThreads) {
        cpx<T> a = H[r + (int64_t)j * ld];
#pragma unroll 4
        for (int k = 0; k < ip; ++k) {
            const cpx<T> vk = w.V[(int64_t)k * ld + r], wk = w.W[(int64_t)k * ld + r];
            a = c_sub(a, c_add(c_mulc(vk, corr[ip + k]), c_mulc(wk, corr[k])));
        }
        if (r == j) {
            d[j] = (double)a.re;
        } else {
            w.vcur[r] = a;
            np += (double)c_abs2(a);
            if (r == j + 1) corr[2 * kPanel - 1] = a;
        }
    }
    const double nrm2 = block_sum(np, red);
    x0 = corr[2 * kPanel - 1];
    const double xnorm = sqrt(nrm2);
    T tau = T(0);
    cpx<T> v0 = x0;
    if (xnorm > 0.0) {
        const double ax0 = sqrt((double)c_abs2(x0));
        const double pr = ax0 > 0.0 ? (double)x0.re / ax0 : 1.0;
        const double pi = ax0 > 0.0 ? (double)x0.im / ax0 : 0.0;
        const double v0r = (double)x0.re + pr * xnorm, v0i = (double)x0.im + pi * xnorm;
        const double vn2 = nrm2 - ax0 * ax0 + v0r * v0r + v0i * v0i;
        tau = (T)(2.0 / vn2);
        v0 = {(T)v0r, (T)v0i};
    }
    if (t == 0) {
        e[j] = xnorm;
        w.vcur[j + 1] = v0;
        w.tau[0] = {tau, T(0)};
    }
}

template <typename T>
__global__ __launch_bounds__(kSerThreads) void start_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                            const int32_t *__restrict__ n_in, double *__restrict__ dall,
                                                            double *__restrict__ eall, int64_t lde,
                                                            cpx<T> *__restrict__ wall, int64_t stride, int j) {
    __shared__ cpx<T> corr[2 * kPanel];
    __shared__ double red[32];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    if (n < 0 || n > ld || j + 2 >= n) return;
    const BatchedView<T> w(wall, stride, ld, u);
    start_column<T>(Hall + u * ld * ld, ld, n, j, 0, w, dall + u * lde, eall + u * lde, corr, red);
}

// y = A v partials for column j: wavefront (blockIdx.y * kMvWaves + wid) owns
// strip S of kStripCols columns [b0 + S*kStripCols, ...) and walks its tiles
// from the diagonal down.  Lanes: 16 row lanes x 4 column lanes.
template <typename T>
__global__ __launch_bounds__(kMvWaves * 64) void matvec_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                               const int32_t *__restrict__ n_in,
                                                               cpx<T> *__restrict__ wall, int64_t stride, int j) {
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    if (n < 0 || n > ld || j + 2 >= n) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int b0 = j + 1, m = n - b0;
    const int S = blockIdx.y * kMvWaves + wid;
    if (S >= strips_of(m)) return;
    const BatchedView<T> w(wall, stride, ld, u);
    const cpx<T> *H = Hall + u * ld * ld;
    const cpx<T> *v = w.vcur;
    const int lr = lane & 15, lc = lane >> 4;
    const int nI = (m + kTileRows - 1) / kTileRows;
    const int cbase = b0 + S * kStripCols;
    cpx<T> vc[4], colacc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = cbase + lc + 4 * t;
        vc[t] = c < n ? v[c] : cpx<T>{T(0), T(0)};
        colacc[t] = {T(0), T(0)};
    }
    cpx<T> *rp = w.rowpart + (int64_t)S * ld;
    // Tiles are software-pipelined: the loads of tile I+1 are issued before
    // tile I is reduced, so every wavefront keeps a tile in flight.
    auto load_tile = [&](int I, cpx<T> (&a)[4][4], cpx<T> (&vr)[4]) {
        const int rbase = b0 + I * kTileRows;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = cbase + lc + 4 * t;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rbase + lr + 16 * q;
                a[t][q] = (r < n && c < n && r >= c) ? H[r + (int64_t)c * ld] : cpx<T>{T(0), T(0)};
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rbase + lr + 16 * q;
            vr[q] = r < n ? v[r] : cpx<T>{T(0), T(0)};
        }
    };
    int I = (S * kStripCols) / kTileRows;
    cpx<T> a[4][4], vr[4];
    load_tile(I, a, vr);
    for (; I < nI; ++I) {
        cpx<T> an[4][4], vrn[4];
        if (I + 1 < nI) load_tile(I + 1, an, vrn);
        const int rbase = b0 + I * kTileRows;
        cpx<T> rowacc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) rowacc[q] = {T(0), T(0)};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = cbase + lc + 4 * t;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rbase + lr + 16 * q;
                cpx<T> x = a[t][q];
                if (r == c) x.im = T(0);
                rowacc[q] = c_add(rowacc[q], c_mul(x, vc[t]));
                if (r > c) colacc[t] = c_add(colacc[t], c_cmul(x, vr[q]));
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            rowacc[q] = c_add(rowacc[q], shfl_xor_c(rowacc[q], 16));
            rowacc[q] = c_add(rowacc[q], shfl_xor_c(rowacc[q], 32));
        }
        if (lc == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rbase + lr + 16 * q;
                if (r < n) rp[r] = rowacc[q];
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            vr[t] = vrn[t];
#pragma unroll
            for (int q = 0; q < 4; ++q) a[t][q] = an[t][q];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) colacc[t] = c_add(colacc[t], shfl_xor_c(colacc[t], off));
    }
    if (lr == 0) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int c = cbase + lc + 4 * t;
            if (c < n) w.ycol[c] = colacc[t];
        }
    }
}

// Finish reflector j = j0 + i (store v_j, w_j) and start column j + 1 when it
// belongs to the same panel.
template <typename T>
__global__ __launch_bounds__(kSerThreads) void finish_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                             const int32_t *__restrict__ n_in,
                                                             double *__restrict__ dall, double *__restrict__ eall,
                                                             int64_t lde, cpx<T> *__restrict__ wall, int64_t stride,
                                                             int j0, int i) {
    __shared__ cpx<T> dots[2 * kPanel];
    __shared__ cpx<T> corr[2 * kPanel];
    __shared__ double red[32];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int j = j0 + i;
    if (n < 0 || n > ld || j + 2 >= n) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const BatchedView<T> w(wall, stride, ld, u);
    const int b0 = j + 1;
    const cpx<T> *v = w.vcur;
    // panel dot products W[k]^H v and V[k]^H v (k < i), one wavefront per product
    for (int q = wid; q < 2 * i; q += kSerThreads / 64) {
        const cpx<T> *col = (q < i) ? w.W + (int64_t)q * ld : w.V + (int64_t)(q - i) * ld;
        cpx<T> s = {T(0), T(0)};
#pragma unroll 4
        for (int r = b0 + lane; r < n; r += 64) s = c_add(s, c_cmul(col[r], v[r]));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s = c_add(s, shfl_xor_c(s, off));
        if (lane == 0) dots[q] = s;
    }
    __syncthreads();
    const T tau = w.tau[0].re;
    double kp = 0.0;
    for (int r = b0 + t; r < n; r += kSerThreads) {
        cpx<T> s = w.ycol[r];
        const int smax = (r - b0) / kStripCols;
#pragma unroll 8
        for (int S = 0; S <= smax; ++S) s = c_add(s, w.rowpart[(int64_t)S * ld + r]);
#pragma unroll 4
        for (int k = 0; k < i; ++k)
            s = c_sub(s, c_add(c_mul(w.V[(int64_t)k * ld + r], dots[k]), c_mul(w.W[(int64_t)k * ld + r], dots[i + k])));
        const cpx<T> p = c_scale(tau, s);
        w.ycol[r] = p;
        kp += (double)v[r].re * (double)p.re + (double)v[r].im * (double)p.im;
    }
    const double vhp = block_sum(kp, red);
    const T K = (T)(0.5 * (double)tau * vhp);
    for (int r = b0 + t; r < n; r += kSerThreads) {
        w.V[(int64_t)i * ld + r] = v[r];
        w.W[(int64_t)i * ld + r] = c_sub(w.ycol[r], c_scale(K, v[r]));
    }
    __syncthreads();
    if (i + 1 < kPanel && j + 3 < n)
        start_column<T>(Hall + u * ld * ld, ld, n, j + 1, i + 1, w, dall + u * lde, eall + u * lde, corr, red);
}

// Trailing update after panel j0:
//   A[r, c] -= sum_k V[k][r] conj(W[k][c]) + W[k][r] conj(V[k][c])
// for c0 <= c <= r < n, c0 = j0 + (reflectors of the panel).  A workgroup
// owns a 64 x 64 block of the lower triangle; it stages the panel's V and W
// values of its 64 rows and 64 columns in LDS, and each lane accumulates a
// 4 x 4 micro-tile (rows lr + 16q, columns lc + 4t of its wavefront's
// 16-column strip), i.e. two complex multiply-adds per LDS value.
constexpr int kUpdBlock = 64;

template <typename T>
__global__ __launch_bounds__(256) void update_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                     const int32_t *__restrict__ n_in, cpx<T> *__restrict__ wall,
                                                     int64_t stride, int j0) {
    __shared__ cpx<T> sVr[kPanel][kUpdBlock], sWr[kPanel][kUpdBlock], sVc[kPanel][kUpdBlock], sWc[kPanel][kUpdBlock];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    if (n < 0 || n > ld || j0 + 2 >= n) return;
    const int nbp = min(kPanel, n - 2 - j0);
    const int c0 = j0 + nbp;
    const int rb = c0 + blockIdx.y * kUpdBlock, cb = c0 + blockIdx.z * kUpdBlock;
    if (rb >= n || cb > rb + kUpdBlock - 1) return;  // outside the lower triangle (uniform per block)
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const BatchedView<T> w(wall, stride, ld, u);
    for (int idx = t; idx < nbp * kUpdBlock; idx += 256) {
        const int k = idx / kUpdBlock, l = idx % kUpdBlock;
        const int r = rb + l, c = cb + l;
        const cpx<T> zero = {T(0), T(0)};
        sVr[k][l] = r < n ? w.V[(int64_t)k * ld + r] : zero;
        sWr[k][l] = r < n ? w.W[(int64_t)k * ld + r] : zero;
        sVc[k][l] = c < n ? w.V[(int64_t)k * ld + c] : zero;
        sWc[k][l] = c < n ? w.W[(int64_t)k * ld + c] : zero;
    }
    __syncthreads();
    const int cs = cb + wid * kUpdCols;  // this wavefront's 16-column strip
    if (cs >= n || cs > rb + kUpdBlock - 1) return;
    const int lr = lane & 15, lc = lane >> 4;
    cpx<T> acc[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[tt][q] = {T(0), T(0)};
    for (int k = 0; k < nbp; ++k) {
        cpx<T> vr[4], wr[4], vc[4], wc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            vr[q] = sVr[k][lr + 16 * q];
            wr[q] = sWr[k][lr + 16 * q];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            vc[tt] = sVc[k][wid * kUpdCols + lc + 4 * tt];
            wc[tt] = sWc[k][wid * kUpdCols + lc + 4 * tt];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[tt][q] = c_add(acc[tt][q], c_add(c_mulc(vr[q], wc[tt]), c_mulc(wr[q], vc[tt])));
    }
    cpx<T> *H = Hall + u * ld * ld;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = cs + lc + 4 * tt;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rb + lr + 16 * q;
            if (r < n && c < n && r >= c) {
                cpx<T> &a = H[r + (int64_t)c * ld];
                a = c_sub(a, acc[tt][q]);
            }
        }
    }
}

template <typename T>
__global__ void tail_kernel(const cpx<T> *__restrict__ Hall, int64_t ld, const int32_t *__restrict__ n_in,
                            int64_t batch, double *__restrict__ dall, double *__restrict__ eall, int64_t lde) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= batch) return;
    const int n = n_in[u];
    double *d = dall + u * lde;
    double *e = eall + u * lde;
    const cpx<T> *H = Hall + u * ld * ld;
    if (n < 0 || n > ld) {
        for (int64_t i = 0; i < lde; ++i) d[i] = NAN;
        return;
    }
    if (n >= 2) {
        d[n - 2] = (double)H[(n - 2) + (int64_t)(n - 2) * ld].re;
        e[n - 2] = sqrt((double)c_abs2(H[(n - 1) + (int64_t)(n - 2) * ld]));
        d[n - 1] = (double)H[(n - 1) + (int64_t)(n - 1) * ld].re;
    } else if (n == 1) {
        d[0] = (double)H[0].re;
    }
}

template <typename T>
hipError_t launch_tridiag_batched(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                                  int64_t lde, cpx<T> *work, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int64_t stride = (int64_t)tridiag_batched_work_elems<T>(ld);
    const unsigned B = (unsigned)batch;
    for (int j0 = 0; j0 + 2 < ld; j0 += kPanel) {
        hipLaunchKernelGGL(start_kernel<T>, dim3(B), dim3(kSerThreads), 0, s, H, ld, n_in, d, e, lde, work, stride, j0);
        for (int i = 0; i < kPanel && j0 + i + 2 < ld; ++i) {
            const int j = j0 + i;
            const int64_t nS = strips_of(ld - j - 1);
            hipLaunchKernelGGL(matvec_kernel<T>, dim3(B, (unsigned)((nS + kMvWaves - 1) / kMvWaves)),
                               dim3(kMvWaves * 64), 0, s, H, ld, n_in, work, stride, j);
            hipLaunchKernelGGL(finish_kernel<T>, dim3(B), dim3(kSerThreads), 0, s, H, ld, n_in, d, e, lde, work,
                               stride, j0, i);
        }
        const int64_t mt = ld - j0 - 1;
        const unsigned nblk = (unsigned)((mt + kUpdBlock - 1) / kUpdBlock);
        hipLaunchKernelGGL(update_kernel<T>, dim3(B, nblk, nblk), dim3(256), 0, s, H, ld, n_in, work, stride, j0);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(tail_kernel<T>, dim3((B + 127) / 128), dim3(128), 0, s, H, ld, n_in, batch, d, e, lde);
    return hipGetLastError();
}

template size_t tridiag_batched_work_elems<double>(int64_t);
template size_t tridiag_batched_work_elems<float>(int64_t);
template hipError_t launch_tridiag_batched<double>(cpx<double> *, int64_t, const int32_t *, int64_t, double *,
                                                   double *, int64_t, cpx<double> *, hipStream_t);
template hipError_t launch_tridiag_batched<float>(cpx<float> *, int64_t, const int32_t *, int64_t, double *, double *,
                                                  int64_t, cpx<float> *, hipStream_t);

}  // namespace mlmc
