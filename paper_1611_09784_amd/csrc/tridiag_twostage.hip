// Two-stage Householder tridiagonalisation of a batch of Hermitian matrices
// held in device memory (only the lower triangle is read and written).
//
// Stage 1 (dense -> band of half-bandwidth kB), one panel of kB columns at a
// time for the whole batch:
//   qr_panel_kernel  Householder QR of the kB-column panel below the band,
//                    A[s:n, p:p+kB] = Q R (s = p + kB), Q = I - V T V^H
//                    (compact WY; reflectors of unit phase alpha = -e^{i arg x0}|x|)
//   hemm_kernel      X = A22 V with A22 = A[s:n, s:n] read from its stored
//                    lower triangle (each output row reads its row left of the
//                    diagonal and its column below it), one wavefront per 64
//                    output rows, no partial sums
//   wfactor_kernel   W = X T - 1/2 V (T^H V^H X T)
//   update_kernel    A22 <- Q^H A22 Q = A22 - V W^H - W V^H (lower triangle)
// Per panel the trailing matrix is read about three times, instead of once
// per column as in a one-stage reduction.
//
// Stage 2 (band -> tridiagonal), chase_kernel: one wavefront per matrix.  The
// band is copied to a compact column-major band array with room for the
// bulge (2*kB sub-diagonals).  Sweep j annihilates column j below the
// sub-diagonal with a reflector on rows j+1..j+kB, applied two-sidedly to the
// kB x kB diagonal block and from the right to the block below, which fills
// it; the fill's first column is then annihilated by the next reflector, and
// so on down the band (bulge chasing).  Each 16 x 16 block lives in registers
// (16 row lanes x 4 column lanes, 4 columns per lane); the next step's blocks
// are prefetched while the current one is processed.
#include "device_common.hpp"

namespace mlmc {

constexpr int kB = 16;                 // band half-width = panel width
constexpr int kBandLd = 2 * kB + 1;    // stored sub-diagonals per column (incl. diagonal)
constexpr int kQrThreads = 256;
constexpr int kHemmRows = 64;
constexpr int kHemmChunk = 64;
constexpr int kWThreads = 256;
constexpr int kUpdBlk = 64;

// Per-matrix workspace (complex elements): V [kB][ld], X [kB][ld], W [kB][ld],
// T [kB][kB], band [ld][kBandLd].
template <typename T>
size_t tridiag_twostage_work_elems(int64_t ld) {
    return (size_t)(3 * kB) * (size_t)ld + (size_t)kB * kB + (size_t)kBandLd * (size_t)ld;
}

template <typename T>
struct TwoView {
    cpx<T> *V, *X, *W, *Tm, *band;
    __device__ TwoView(cpx<T> *wall, int64_t stride, int64_t ld, int64_t u) {
        cpx<T> *b = wall + u * stride;
        V = b;
        X = V + (int64_t)kB * ld;
        W = X + (int64_t)kB * ld;
        Tm = W + (int64_t)kB * ld;
        band = Tm + kB * kB;
    }
};

template <typename T>
__device__ __forceinline__ cpx<T> shfl_c(cpx<T> a, int src) {
    return {__shfl(a.re, src, 64), __shfl(a.im, src, 64)};
}
template <typename T>
__device__ __forceinline__ cpx<T> shfl_xor2(cpx<T> a, int m) {
    return {__shfl_xor(a.re, m, 64), __shfl_xor(a.im, m, 64)};
}

// Reflector of x (norm^2 nrm2, first entry x0): v0 = x0 - alpha with
// alpha = -e^{i arg x0} |x|, tau = 2 / |v|^2 (0 when x = 0).
template <typename T>
__device__ __forceinline__ void make_reflector(double nrm2, cpx<T> x0, T &tau, cpx<T> &v0, cpx<T> &alpha) {
    const double xnorm = sqrt(nrm2);
    tau = T(0);
    v0 = x0;
    alpha = x0;
    if (xnorm > 0.0) {
        const double ax0 = sqrt((double)c_abs2(x0));
        const double pr = ax0 > 0.0 ? (double)x0.re / ax0 : 1.0;
        const double pi = ax0 > 0.0 ? (double)x0.im / ax0 : 0.0;
        const double v0r = (double)x0.re + pr * xnorm, v0i = (double)x0.im + pi * xnorm;
        const double vn2 = nrm2 - ax0 * ax0 + v0r * v0r + v0i * v0i;
        tau = (T)(2.0 / vn2);
        v0 = {(T)v0r, (T)v0i};
        alpha = {(T)(-pr * xnorm), (T)(-pi * xnorm)};
    }
}

// ---------------------------------------------------------------------------
// Stage 1: panel QR.  One workgroup per matrix.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kQrThreads) void qr_panel_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                              const int32_t *__restrict__ n_in,
                                                              cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ cpx<T> part[kQrThreads / 64][kB];
    __shared__ cpx<T> dots[kB];
    __shared__ cpx<T> Ts[kB][kB];
    __shared__ double red[32];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *A = Hall + u * ld * ld;
    const int nr = min(m - 1, kB);
    for (int idx = t; idx < kB * kB; idx += kQrThreads) Ts[idx / kB][idx % kB] = {T(0), T(0)};
    for (int i = 0; i < kB; ++i) {
        cpx<T> *Vi = w.V + (int64_t)i * ld;
        if (i >= nr) {  // no reflector: V column is zero
            for (int r = s + t; r < n; r += kQrThreads) Vi[r] = {T(0), T(0)};
            continue;
        }
        const int r0 = s + i;
        cpx<T> *colA = A + (int64_t)(p + i) * ld;
        double np = 0.0;
        for (int r = r0 + t; r < n; r += kQrThreads) np += (double)c_abs2(colA[r]);
        const double nrm2 = block_sum(np, red);
        const cpx<T> x0 = colA[r0];
        T tau;
        cpx<T> v0, alpha;
        make_reflector<T>(nrm2, x0, tau, v0, alpha);
        // v into V[i] (zero above r0), the panel column becomes (alpha, 0, ..., 0)
        for (int r = s + t; r < n; r += kQrThreads) {
            cpx<T> vr = {T(0), T(0)};
            if (r == r0) vr = v0;
            else if (r > r0) vr = colA[r];
            Vi[r] = vr;
        }
        __syncthreads();
        for (int r = r0 + t; r < n; r += kQrThreads) colA[r] = (r == r0) ? alpha : cpx<T>{T(0), T(0)};
        // products with the remaining panel columns (c > i) and with earlier reflectors (k < i)
        cpx<T> acc[kB];
#pragma unroll
        for (int c = 0; c < kB; ++c) acc[c] = {T(0), T(0)};
        for (int r = r0 + t; r < n; r += kQrThreads) {
            const cpx<T> vr = Vi[r];
#pragma unroll
            for (int c = 0; c < kB; ++c) {
                if (c > i) acc[c] = c_add(acc[c], c_cmul(vr, A[r + (int64_t)(p + c) * ld]));
                else if (c < i) acc[c] = c_add(acc[c], c_cmul(w.V[(int64_t)c * ld + r], vr));
            }
        }
#pragma unroll
        for (int c = 0; c < kB; ++c) {
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) acc[c] = c_add(acc[c], shfl_xor2(acc[c], off));
            if (lane == 0) part[wid][c] = acc[c];
        }
        __syncthreads();
        if (t < kB) {
            cpx<T> sum = part[0][t];
            for (int q = 1; q < kQrThreads / 64; ++q) sum = c_add(sum, part[q][t]);
            dots[t] = sum;
        }
        __syncthreads();
        // apply the reflector to the remaining panel columns
        for (int r = r0 + t; r < n; r += kQrThreads) {
            const cpx<T> vr = Vi[r];
#pragma unroll
            for (int c = 0; c < kB; ++c) {
                if (c > i) {
                    cpx<T> &a = A[r + (int64_t)(p + c) * ld];
                    a = c_sub(a, c_scale(tau, c_mul(vr, dots[c])));
                }
            }
        }
        // T[:i, i] = -tau T[:i, :i] (V^H v_i)[:i], T[i, i] = tau
        if (t == 0) {
            for (int k = 0; k < i; ++k) {
                cpx<T> sum = {T(0), T(0)};
                for (int q = k; q < i; ++q) sum = c_add(sum, c_mul(Ts[k][q], dots[q]));
                Ts[k][i] = c_scale(-tau, sum);
            }
            Ts[i][i] = {tau, T(0)};
        }
        __syncthreads();
    }
    for (int idx = t; idx < kB * kB; idx += kQrThreads) w.Tm[idx] = Ts[idx / kB][idx % kB];
}

// ---------------------------------------------------------------------------
// Stage 1: X = A22 V.  One wavefront per 64 output rows; lane = row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(64) void hemm_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                  const int32_t *__restrict__ n_in, cpx<T> *__restrict__ wall,
                                                  int64_t stride, int p) {
    __shared__ cpx<T> sV[kHemmChunk][kB];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    const int rb = s + blockIdx.y * kHemmRows;
    if (rb >= n) return;
    const int lane = threadIdx.x;
    const TwoView<T> w(wall, stride, ld, u);
    const cpx<T> *A = Hall + u * ld * ld;
    const int r = rb + lane;
    const bool rowok = r < n;
    cpx<T> acc[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) acc[k] = {T(0), T(0)};
    for (int cb = s; cb < n; cb += kHemmChunk) {
        const int cn = min(kHemmChunk, n - cb);
        __syncthreads();
        for (int idx = lane; idx < kHemmChunk * kB; idx += 64) {
            const int c = idx % kHemmChunk, k = idx / kHemmChunk;
            sV[c][k] = c < cn ? w.V[(int64_t)k * ld + cb + c] : cpx<T>{T(0), T(0)};
        }
        __syncthreads();
        if (!rowok) continue;
        for (int cc = 0; cc < cn; ++cc) {
            const int c = cb + cc;
            cpx<T> a;
            if (c < r) a = A[r + (int64_t)c * ld];            // stored lower part of row r
            else if (c > r) a = c_conj(A[c + (int64_t)r * ld]);  // column r below the diagonal
            else a = {A[r + (int64_t)r * ld].re, T(0)};
#pragma unroll
            for (int k = 0; k < kB; ++k) acc[k] = c_add(acc[k], c_mul(a, sV[cc][k]));
        }
    }
    if (rowok) {
#pragma unroll
        for (int k = 0; k < kB; ++k) w.X[(int64_t)k * ld + r] = acc[k];
    }
}

// ---------------------------------------------------------------------------
// Stage 1: W = X T - 1/2 V Y, Y = T^H (V^H X T).  One workgroup per matrix.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWThreads) void wfactor_kernel(const int32_t *__restrict__ n_in, int64_t ld,
                                                            cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ cpx<T> Ts[kB][kB];
    constexpr int kZGroups = 8;
    __shared__ cpx<T> Zp[kZGroups][kB][kB];  // [row group][k][l]
    __shared__ cpx<T> Y[kB][kB];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    const int t = threadIdx.x;
    const TwoView<T> w(wall, stride, ld, u);
    for (int idx = t; idx < kB * kB; idx += kWThreads) Ts[idx / kB][idx % kB] = w.Tm[idx];
    __syncthreads();
    // X <- X T (per row)
#pragma unroll 1
    for (int r = s + t; r < n; r += kWThreads) {
        cpx<T> x[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) x[q] = w.X[(int64_t)q * ld + r];
        // `zr` is 0 but depends on r, so the 16 x 16 table stays in LDS instead
        // of being hoisted out of the row loop into (spilled) registers.
        const int zr = r >> 30;
        for (int l = 0; l < kB; ++l) {  // T is upper triangular: column l uses rows q <= l
            cpx<T> sum = {T(0), T(0)};
#pragma unroll
            for (int q = 0; q < kB; ++q)
                if (q <= l) sum = c_add(sum, c_mul(x[q], Ts[q + zr][l]));
            w.X[(int64_t)l * ld + r] = sum;
        }
    }
    __syncthreads();
    // Z = V^H (X T): thread (row group g, k) accumulates Z[k][:] over rows r = s + g, s + g + G, ...
    if (t < kZGroups * kB) {
        const int k = t % kB, g = t / kB;
        constexpr int G = kZGroups;
        cpx<T> z[kB];
#pragma unroll
        for (int l = 0; l < kB; ++l) z[l] = {T(0), T(0)};
#pragma unroll 1
        for (int r = s + g; r < n; r += G) {
            const cpx<T> vk = w.V[(int64_t)k * ld + r];
#pragma unroll
            for (int l = 0; l < kB; ++l) z[l] = c_add(z[l], c_cmul(vk, w.X[(int64_t)l * ld + r]));
        }
#pragma unroll
        for (int l = 0; l < kB; ++l) Zp[g][k][l] = z[l];
    }
    __syncthreads();
    {
        const int k = t / kB, l = t % kB;  // Y = T^H Z, T upper triangular
        cpx<T> y = {T(0), T(0)};
        for (int q = 0; q <= k; ++q) {
            cpx<T> zql = {T(0), T(0)};
            for (int g = 0; g < kZGroups; ++g) zql = c_add(zql, Zp[g][q][l]);
            y = c_add(y, c_cmul(Ts[q][k], zql));
        }
        Y[k][l] = y;
    }
    __syncthreads();
#pragma unroll 1
    for (int r = s + t; r < n; r += kWThreads) {
        cpx<T> v[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) v[k] = w.V[(int64_t)k * ld + r];
        const int zr = r >> 30;  // see above
        for (int l = 0; l < kB; ++l) {
            cpx<T> sum = {T(0), T(0)};
#pragma unroll
            for (int k = 0; k < kB; ++k) sum = c_add(sum, c_mul(v[k], Y[k + zr][l]));
            w.W[(int64_t)l * ld + r] = c_sub(w.X[(int64_t)l * ld + r], c_scale(T(0.5), sum));
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 1: A22 -= V W^H + W V^H on the lower triangle.  A workgroup owns a
// 64 x 64 block and stages its rows' and columns' V, W in LDS; each lane
// accumulates a 4 x 4 micro-tile.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void band_update_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                          const int32_t *__restrict__ n_in, cpx<T> *__restrict__ wall,
                                                          int64_t stride, int p) {
    __shared__ cpx<T> sVr[kB][kUpdBlk], sWr[kB][kUpdBlk], sVc[kB][kUpdBlk], sWc[kB][kUpdBlk];
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB;
    if (n < 0 || n > ld || n - s < 2) return;
    const int rb = s + blockIdx.y * kUpdBlk, cb = s + blockIdx.z * kUpdBlk;
    if (rb >= n || cb > rb + kUpdBlk - 1) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const TwoView<T> w(wall, stride, ld, u);
    for (int idx = t; idx < kB * kUpdBlk; idx += 256) {
        const int k = idx / kUpdBlk, l = idx % kUpdBlk;
        const int r = rb + l, c = cb + l;
        const cpx<T> zero = {T(0), T(0)};
        sVr[k][l] = r < n ? w.V[(int64_t)k * ld + r] : zero;
        sWr[k][l] = r < n ? w.W[(int64_t)k * ld + r] : zero;
        sVc[k][l] = c < n ? w.V[(int64_t)k * ld + c] : zero;
        sWc[k][l] = c < n ? w.W[(int64_t)k * ld + c] : zero;
    }
    __syncthreads();
    const int cs = cb + wid * 16;
    if (cs >= n || cs > rb + kUpdBlk - 1) return;
    const int lr = lane & 15, lc = lane >> 4;
    cpx<T> acc[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[tt][q] = {T(0), T(0)};
    for (int k = 0; k < kB; ++k) {
        cpx<T> vr[4], wr[4], vc[4], wc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            vr[q] = sVr[k][lr + 16 * q];
            wr[q] = sWr[k][lr + 16 * q];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            vc[tt] = sVc[k][wid * 16 + lc + 4 * tt];
            wc[tt] = sWc[k][wid * 16 + lc + 4 * tt];
        }
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[tt][q] = c_add(acc[tt][q], c_add(c_mulc(vr[q], wc[tt]), c_mulc(wr[q], vc[tt])));
    }
    cpx<T> *A = Hall + u * ld * ld;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = cs + lc + 4 * tt;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rb + lr + 16 * q;
            if (r < n && c < n && r >= c) {
                cpx<T> &a = A[r + (int64_t)c * ld];
                a = c_sub(a, acc[tt][q]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 2: bulge chasing band -> tridiagonal, one wavefront per matrix.
// band[c * kBandLd + o] = A[c + o, c], o = 0..2kB.
// ---------------------------------------------------------------------------
template <typename T>
struct Blk {  // 16 x 16 block: lane (r = lane & 15, g = lane >> 4) holds columns g + 4t
    cpx<T> e[4];
};

template <typename T>
__device__ __forceinline__ cpx<T> band_get(const cpx<T> *band, int row, int col) {
    return band[(int64_t)col * kBandLd + (row - col)];
}

// Load A[r0 + r, c0 + c] (r < nrow, c < ncol) where every such element lies
// on or below the diagonal and within the stored band.
template <typename T>
__device__ __forceinline__ void load_blk(const cpx<T> *band, int r0, int c0, int nrow, int ncol, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        b.e[tt] = (r < nrow && c < ncol) ? band_get(band, r0 + r, c0 + c) : cpx<T>{T(0), T(0)};
    }
}
// Hermitian diagonal block A[r0.., r0..] of size L from its lower part.
template <typename T>
__device__ __forceinline__ void load_diag(const cpx<T> *band, int r0, int L, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        cpx<T> x = {T(0), T(0)};
        if (r < L && c < L) {
            if (r > c) x = band_get(band, r0 + r, r0 + c);
            else if (r < c) x = c_conj(band_get(band, r0 + c, r0 + r));
            else x = {band_get(band, r0 + r, r0 + r).re, T(0)};
        }
        b.e[tt] = x;
    }
}

template <typename T>
__device__ __forceinline__ cpx<T> sum16(cpx<T> x) {  // over the 16 row lanes of a column group
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) x = c_add(x, shfl_xor2(x, off));
    return x;
}
template <typename T>
__device__ __forceinline__ cpx<T> sum4g(cpx<T> x) {  // over the 4 column groups of a row
    x = c_add(x, shfl_xor2(x, 16));
    return c_add(x, shfl_xor2(x, 32));
}

template <typename T>
__global__ __launch_bounds__(64) void chase_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                   const int32_t *__restrict__ n_in, double *__restrict__ dall,
                                                   double *__restrict__ eall, int64_t lde, cpx<T> *__restrict__ wall,
                                                   int64_t stride) {
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    double *d = dall + u * lde;
    double *e = eall + u * lde;
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    if (n < 0 || n > ld) {
        for (int64_t i = lane; i < lde; i += 64) d[i] = NAN;
        return;
    }
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *band = w.band;
    const cpx<T> *A = Hall + u * ld * ld;
    for (int64_t q = lane; q < (int64_t)n * kBandLd; q += 64) {
        const int c = (int)(q / kBandLd), o = (int)(q % kBandLd);
        band[q] = (o <= kB && c + o < n) ? A[(c + o) + (int64_t)c * ld] : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    for (int j = 0; j + 2 < n; ++j) {
        int lo = j + 1, hi = min(j + kB, n - 1);
        int L = hi - lo + 1;
        if (L < 2) continue;
        // Step 0: the "previous block" is column j itself: B = A[lo..hi, j].
        Blk<T> B, D, E;
        load_blk(band, lo, j, L, 1, B);
        int col0 = j;  // first column of the block B
        int Lprev = 1;
        D = {};
        E = {};
        load_diag(band, lo, L, D);
        int lo1 = hi + 1, hi1 = min(hi + kB, n - 1), L1 = hi1 - lo1 + 1;
        if (L1 > 0) load_blk(band, lo1, lo, L1, L, E);
        while (true) {
            // reflector from the first column of B (held by column group 0, tt = 0)
            const cpx<T> xr = (g == 0 && r < L) ? B.e[0] : cpx<T>{T(0), T(0)};
            const double nrm2 = (double)sum16(cpx<T>{c_abs2(xr), T(0)}).re;
            const double nrm2_all = __shfl((double)nrm2, 0, 64);
            const cpx<T> x0 = shfl_c(B.e[0], 0);
            T tau;
            cpx<T> v0, alpha;
            make_reflector<T>(nrm2_all, x0, tau, v0, alpha);
            const cpx<T> xsrc = shfl_c(B.e[0], r);  // every lane takes row r of B's first column
            const cpx<T> vr = (r == 0) ? v0 : ((r < L) ? xsrc : cpx<T>{T(0), T(0)});
            cpx<T> vcol[4];
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) vcol[tt] = shfl_c(vr, g + 4 * tt);  // v at this lane's columns
            // prefetch the next step's diagonal block and block below (disjoint from this step's writes)
            const int lo2 = hi1 + 1, hi2 = min(hi1 + kB, n - 1), L2 = hi2 - lo2 + 1;
            Blk<T> Dn = {}, En = {};
            if (L1 > 0) load_diag(band, lo1, L1, Dn);
            if (L1 > 0 && L2 > 0) load_blk(band, lo2, lo1, L2, L1, En);
            // B <- H B
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const cpx<T> sc = sum16(c_cmul(vr, B.e[tt]));
                B.e[tt] = c_sub(B.e[tt], c_scale(tau, c_mul(vr, sc)));
            }
            // the annihilated column is exactly (alpha, 0, ..., 0)
            if (g == 0 && r < L) B.e[0] = (r == 0) ? alpha : cpx<T>{T(0), T(0)};
            // D <- H D H
            cpx<T> pr = {T(0), T(0)};
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) pr = c_add(pr, c_mul(D.e[tt], vcol[tt]));
            pr = c_scale(tau, sum4g(pr));
            const cpx<T> vhp = sum16(c_cmul(vr, pr));
            const T K = (T)0.5 * tau * vhp.re;
            const cpx<T> wr = c_sub(pr, c_scale(K, vr));
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const cpx<T> wc = shfl_c(wr, g + 4 * tt);
                D.e[tt] = c_sub(D.e[tt], c_add(c_mulc(vr, wc), c_mulc(wr, vcol[tt])));
            }
            // E <- E H
            if (L1 > 0) {
                cpx<T> q = {T(0), T(0)};
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) q = c_add(q, c_mul(E.e[tt], vcol[tt]));
                q = sum4g(q);
#pragma unroll
                for (int tt = 0; tt < 4; ++tt) E.e[tt] = c_sub(E.e[tt], c_scale(tau, c_mulc(q, vcol[tt])));
            }
            // store B (final for this sweep) and the lower part of D
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const int c = g + 4 * tt;
                if (r < L && c < Lprev) band[(int64_t)(col0 + c) * kBandLd + (lo + r - col0 - c)] = B.e[tt];
                if (r < L && c < L && r >= c) band[(int64_t)(lo + c) * kBandLd + (r - c)] = D.e[tt];
            }
            if (L1 < 2) {  // nothing left to chase (a 1-row block needs no annihilation)
                if (L1 == 1) {
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        const int c = g + 4 * tt;
                        if (r < 1 && c < L) band[(int64_t)(lo + c) * kBandLd + (lo1 + r - lo - c)] = E.e[tt];
                    }
                }
                break;
            }
            // advance: the filled block below becomes the next B
            B = E;
            D = Dn;
            E = En;
            col0 = lo;
            Lprev = L;
            lo = lo1;
            hi = hi1;
            L = L1;
            lo1 = lo2;
            hi1 = hi2;
            L1 = L2;
        }
        __syncthreads();
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        d[i] = (double)band[(int64_t)i * kBandLd].re;
        if (i + 1 < n) e[i] = sqrt((double)c_abs2(band[(int64_t)i * kBandLd + 1]));
    }
}

template <typename T>
hipError_t launch_tridiag_twostage(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                                   int64_t lde, cpx<T> *work, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int64_t stride = (int64_t)tridiag_twostage_work_elems<T>(ld);
    const unsigned B = (unsigned)batch;
    for (int p = 0; p + kB + 1 < ld; p += kB) {
        const int64_t mmax = ld - p - kB;
        hipLaunchKernelGGL(qr_panel_kernel<T>, dim3(B), dim3(kQrThreads), 0, s, H, ld, n_in, work, stride, p);
        hipLaunchKernelGGL(hemm_kernel<T>, dim3(B, (unsigned)((mmax + kHemmRows - 1) / kHemmRows)), dim3(64), 0, s, H,
                           ld, n_in, work, stride, p);
        hipLaunchKernelGGL(wfactor_kernel<T>, dim3(B), dim3(kWThreads), 0, s, n_in, ld, work, stride, p);
        const unsigned nblk = (unsigned)((mmax + kUpdBlk - 1) / kUpdBlk);
        hipLaunchKernelGGL(band_update_kernel<T>, dim3(B, nblk, nblk), dim3(256), 0, s, H, ld, n_in, work, stride, p);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    hipLaunchKernelGGL(chase_kernel<T>, dim3(B), dim3(64), 0, s, H, ld, n_in, d, e, lde, work, stride);
    return hipGetLastError();
}

template size_t tridiag_twostage_work_elems<double>(int64_t);
template size_t tridiag_twostage_work_elems<float>(int64_t);
template hipError_t launch_tridiag_twostage<double>(cpx<double> *, int64_t, const int32_t *, int64_t, double *,
                                                    double *, int64_t, cpx<double> *, hipStream_t);
template hipError_t launch_tridiag_twostage<float>(cpx<float> *, int64_t, const int32_t *, int64_t, double *,
                                                   double *, int64_t, cpx<float> *, hipStream_t);

}  // namespace mlmc
