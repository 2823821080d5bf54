// Stage 1 of the two-stage Householder tridiagonalisation of a batch of
// Hermitian matrices held in device memory (only the lower triangle is read
// and written): dense -> band of half-bandwidth kB, one panel of kB columns at
// a time for the whole batch:
//   qr_panel_reg_kernel / qr_panel_kernel
//                    Householder QR of the kB-column panel below the band,
//                    A[s:n, p:p+kB] = Q R (s = p + kB), Q = I - V T V^H
//                    (compact WY; reflectors of unit phase alpha = -e^{i arg x0}|x|)
//                    (and V T, the Hermitian product's operand)
//   hemm_kernel      X T = A22 (V T) with A22 = A[s:n, s:n] read from its
//                    stored lower triangle, one wavefront per 64 output rows,
//                    on the matrix cores; each wavefront also forms
//                    V_rows^H (X T)_rows for its rows
//   wfactor_kernel   W = X T - 1/2 V Y, Y = T^H sum over row blocks of those
//   band_update32_kernel  A22 <- Q^H A22 Q = A22 - V W^H - W V^H (lower
//                    triangle, 32 x 64 tiles; band_update_kernel, 64 x 64
//                    tiles, serves the generalised path's Cholesky updates)
// Complex products on the matrix cores take three real products each.  Per
// panel the trailing matrix is read about three times, instead of once per
// column as in a one-stage reduction.
#include <algorithm>

#include "eigh_large.hpp"
#include "twostage_common.hpp"

namespace mlmc {

constexpr int kQrThreads = 256;
constexpr int kHemmDepth = 2;  // Hermitian product: register sets of its load pipeline
constexpr int kWThreads = 256;
constexpr int kUpdBlk = 64;

// Workgroups are dispatched round-robin over the chip's 8 XCDs (each with its
// own L2).  Kernels with several workgroups per matrix take their (matrix,
// tile) from the linear workgroup id so that all tiles of a matrix run on one
// XCD back to back and share its V / W panels in that L2:
// XCD x = w % 8 processes matrices x, x + 8, ... tile by tile.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_tile(int64_t w, int64_t tiles, int64_t &u, int64_t &tile) {
    const int64_t x = w % kXcds, k = w / kXcds;
    u = x + kXcds * (k / tiles);
    tile = k % tiles;
}
inline unsigned xcd_grid(int64_t batch, int64_t tiles) {
    return (unsigned)(kXcds * ((batch + kXcds - 1) / kXcds) * tiles);
}

// Two-register permlane swap: returns (vdst, src0) after the swap of a
// (as vdst) and b (as src0); their sum leaves a reduced over the lane pair in
// the even rows (lower half) and b in the odd rows (upper half).
template <bool ROWS32>
__device__ __forceinline__ void swap2_word(int a, int b, int &oa, int &ob) {
    if constexpr (ROWS32) {
        const auto q = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        oa = (int)q[0];
        ob = (int)q[1];
    } else {
        const auto q = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        oa = (int)q[0];
        ob = (int)q[1];
    }
}
template <bool ROWS32>
__device__ __forceinline__ float swap_sum(float a, float b) {
    int oa, ob;
    swap2_word<ROWS32>(__float_as_int(a), __float_as_int(b), oa, ob);
    return __int_as_float(oa) + __int_as_float(ob);
}
template <bool ROWS32>
__device__ __forceinline__ double swap_sum(double a, double b) {
    const long long wa = __double_as_longlong(a), wb = __double_as_longlong(b);
    int alo, blo, ahi, bhi;
    swap2_word<ROWS32>((int)wa, (int)wb, alo, blo);
    swap2_word<ROWS32>((int)(wa >> 32), (int)(wb >> 32), ahi, bhi);
    return __longlong_as_double(((long long)ahi << 32) | (unsigned)alo) +
           __longlong_as_double(((long long)bhi << 32) | (unsigned)blo);
}
// One halving step of a reduce-scatter within rows: lanes with bit B clear
// keep element j, the others element j + H; each adds its partner's copy
// (the partner lane is given by the DPP pattern, whose pairs differ in bit B).
template <int CTRL, int B, typename T>
__device__ __forceinline__ T keep_send_sum(T lo, T hi) {
    const bool upper = (threadIdx.x >> B) & 1;
    const T keep = upper ? hi : lo, send = upper ? lo : hi;
    return keep + dpp<CTRL>(send);
}
// Reduce-scatter of 32 values over the 64 lanes of a wavefront: afterwards
// lane l holds the sum over all lanes of element
// e(l) = 16 b5 + 8 b4 + 4 b3 + 2 b2 + b1 (b_k = bit k of l).  The pairing of
// each step is fixed, so every run and both lanes holding an element get the
// same bits.
__device__ __forceinline__ int scatter_elem(int lane) {
    return 16 * ((lane >> 5) & 1) + 8 * ((lane >> 4) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) +
           ((lane >> 1) & 1);
}
template <typename T>
__device__ __forceinline__ T wave_reduce_scatter32(const T (&x)[32]) {
    T y[16], z[8], q[4], h[2];
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = swap_sum<true>(x[j], x[j + 16]);
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = swap_sum<false>(y[j], y[j + 8]);
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = keep_send_sum<kDppMirror, 3>(z[j], z[j + 4]);
#pragma unroll
    for (int j = 0; j < 2; ++j) h[j] = keep_send_sum<kDppHalfMirror, 2>(q[j], q[j + 2]);
    const T o = keep_send_sum<kDppXor2, 1>(h[0], h[1]);
    return o + dpp<kDppXor1>(o);
}

// Matrix-core 16x16x4 products (D += A B, A 16x4, B 4x16).  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; slot v of lane l receives D[row][l % 16]
// with row = 4v + l/16 for the f64 instruction and 4(l/16) + v for the f32 one.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Complex accumulate D += a b on real matrix cores (four real products).
template <typename T>
__device__ __forceinline__ void cmma(cpx<T> a, cpx<T> b, typename Mfma<T>::v4 &dre, typename Mfma<T>::v4 &dim) {
    dre = Mfma<T>::mma(a.re, b.re, dre);
    dre = Mfma<T>::mma(-a.im, b.im, dre);
    dim = Mfma<T>::mma(a.re, b.im, dim);
    dim = Mfma<T>::mma(a.im, b.re, dim);
}

// Complex accumulate with three real products per complex one (Gauss's
// form): P += Re a Re b, Q += Im a Im b, R += (Re a + Im a)(Re b + Im b), so
// that the complex sum is (P - Q) + i (R - P - Q).  as, bs: Re + Im of a, b.
// The error of the imaginary part stays within a small multiple of the
// product of the operands' norms, as for the four-product form.
template <typename T>
struct CAcc3 {
    typename Mfma<T>::v4 p, q, r;
    __device__ __forceinline__ void zero() {
        p = q = r = typename Mfma<T>::v4{T(0), T(0), T(0), T(0)};
    }
    __device__ __forceinline__ void mma(cpx<T> a, T as, cpx<T> b, T bs) {
        p = Mfma<T>::mma(a.re, b.re, p);
        q = Mfma<T>::mma(a.im, b.im, q);
        r = Mfma<T>::mma(as, bs, r);
    }
    __device__ __forceinline__ typename Mfma<T>::v4 re() const { return p - q; }
    __device__ __forceinline__ typename Mfma<T>::v4 im() const { return r - p - q; }
};

// V T (rows s..n-1, T upper triangular in LDS) into the W slot, where the
// Hermitian product takes it as its operand (the W factor overwrites it).
template <typename T>
__device__ __forceinline__ void vt_row(const cpx<T> (&v)[kB], const cpx<T> (&Ts)[kB][kB], cpx<T> (&out)[kB]) {
#pragma unroll
    for (int l = 0; l < kB; ++l) {
        cpx<T> sum = {T(0), T(0)};
#pragma unroll
        for (int q = 0; q <= l; ++q) sum = c_add(sum, c_mul(v[q], Ts[q][l]));
        out[l] = sum;
    }
}
template <typename T>
__device__ __noinline__ void store_vt(const TwoView<T> &w, int64_t ld, int s, int n, int t, int nt,
                                      const cpx<T> (&Ts)[kB][kB]) {
#pragma unroll 1
    for (int r = s + t; r < n; r += nt) {
        cpx<T> v[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) v[q] = w.V[(int64_t)q * ld + r];
#pragma unroll
        for (int l = 0; l < kB; ++l) {
            cpx<T> sum = {T(0), T(0)};
#pragma unroll
            for (int q = 0; q <= l; ++q) sum = c_add(sum, c_mul(v[q], Ts[q][l]));
            w.W[(int64_t)l * ld + r] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 1: panel QR.  One workgroup per matrix.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kQrThreads) void qr_panel_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                              const int64_t *__restrict__ offs,
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
    cpx<T> *A = Hall + mat_offset(offs, u, ld);
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
            acc[c] = {col_sum(row_sum(acc[c].re)), col_sum(row_sum(acc[c].im))};
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
    store_vt<T>(w, ld, s, n, t, kQrThreads, Ts);
}

// ---------------------------------------------------------------------------
// Stage 1: X = A22 V.  One wavefront per 64 output rows; lane = row.
// ---------------------------------------------------------------------------

// Panel QR with the panel in registers: one workgroup of NT >= m threads per
// matrix, thread t holds row s + t of the 16 panel columns.  Per reflector two
// workgroup reductions (column norm with the pivot, then the 16 products with
// the other columns, reduce-scattered within each wavefront); the panel is
// read and written once.  Column i keeps its reflector v below the band
// (v0 at the pivot row) until the write-back.  The reflector index is a
// template parameter so that every register index is static.
template <typename T, int NT>
struct QrShared {
    double part[NT / 64][32];
    double dotw[NT / 64][2 * kB];  // each wavefront's copy of the summed products
    double nred[NT / 64];
    cpx<T> x0s;
    cpx<T> Ts[kB][kB];
    cpx<T> alphas[kB];
};

template <typename T, int NT, int I>
__device__ __forceinline__ void qr_reflect(QrShared<T, NT> &sh, cpx<T> (&P)[kB], int s, int n, int nr) {
    constexpr int NW = NT / 64;
    if (I >= nr) return;  // uniform over the workgroup
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int r = s + t, r0 = s + I;
    const bool own = r < n;
    const cpx<T> zero = {T(0), T(0)};
    // norm of column I from the pivot row down, and the pivot
    double ws = (own && r >= r0) ? (double)c_abs2(P[I]) : 0.0;
    ws = col_sum(row_sum(ws));
    if (lane == 0) sh.nred[wid] = ws;
    if (r == r0) {
        sh.x0s.re = P[I].re;
        sh.x0s.im = P[I].im;
    }
    __syncthreads();
    double nrm2 = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) nrm2 += sh.nred[q];
    T tau;
    cpx<T> v0, alpha;
    make_reflector<T>(nrm2, cpx<T>{sh.x0s.re, sh.x0s.im}, tau, v0, alpha);
    const cpx<T> v = csel(r == r0, v0, csel(own && r > r0, P[I], zero));
    // v^H P[:, c] for c > I and V[:, c]^H v for c < I
    T x[32];
#pragma unroll
    for (int c = 0; c < kB; ++c) {
        const cpx<T> term = c > I ? c_cmul(v, P[c]) : (c < I ? c_cmul(P[c], v) : zero);  // c is static
        x[2 * c] = term.re;
        x[2 * c + 1] = term.im;
    }
    const T red = wave_reduce_scatter32(x);
    if ((lane & 1) == 0) sh.part[wid][scatter_elem(lane)] = (double)red;
    __syncthreads();
    // Every wavefront sums the parts into its own copy and reads it back: a
    // wavefront's LDS operations complete in order, so no second barrier.
    if (lane < 2 * kB) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) sum += sh.part[q][lane];
        sh.dotw[wid][lane] = sum;
    }
    __builtin_amdgcn_wave_barrier();
    const double *dotf = sh.dotw[wid];
    // apply the reflector to the columns right of I
#pragma unroll
    for (int c = I + 1; c < kB; ++c) {
        const cpx<T> dc = {(T)dotf[2 * c], (T)dotf[2 * c + 1]};
        P[c] = c_sub(P[c], c_scale(tau, c_mul(v, dc)));
    }
    P[I] = csel(r == r0, v0, P[I]);
    // T[:I, I] = -tau T[:I, :I] (V^H v_I)[:I], T[I, I] = tau
    if (t < I) {
        cpx<T> sum = zero;
        for (int q = t; q < I; ++q)
            sum = c_add(sum, c_mul(sh.Ts[t][q], cpx<T>{(T)dotf[2 * q], (T)dotf[2 * q + 1]}));
        sh.Ts[t][I] = c_scale(-tau, sum);
    }
    if (t == I) {
        sh.Ts[I][I] = {tau, T(0)};
        sh.alphas[I].re = alpha.re;
        sh.alphas[I].im = alpha.im;
    }
}
template <typename T, int NT, int... Is>
__device__ __forceinline__ void qr_reflect_all(QrShared<T, NT> &sh, cpx<T> (&P)[kB], int s, int n, int nr,
                                               std::integer_sequence<int, Is...>) {
    (qr_reflect<T, NT, Is>(sh, P, s, n, nr), ...);
}

template <typename T, int NT>
__global__ __launch_bounds__(NT) void qr_panel_reg_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                          const int64_t *__restrict__ offs,
                                                          const int32_t *__restrict__ n_in,
                                                          cpx<T> *__restrict__ wall, int64_t stride, int p) {
    __shared__ QrShared<T, NT> sh;
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2 || m > NT) return;
    const int t = threadIdx.x;
    const int r = s + t;
    const bool own = r < n;
    const int ldi = (int)ld;
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *A = Hall + mat_offset(offs, u, ld);
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> P[kB];
#pragma unroll
    for (int c = 0; c < kB; ++c) {
        const cpx<T> a = A[own ? r + (p + c) * ldi : 0];
        P[c] = csel(own, a, zero);
    }
    for (int idx = t; idx < kB * kB; idx += NT) sh.Ts[idx / kB][idx % kB] = zero;
    const int nr = min(m - 1, kB);
    qr_reflect_all<T, NT>(sh, P, s, n, nr, std::make_integer_sequence<int, kB>{});
    __syncthreads();
    if (own) {
        cpx<T> v[kB], vt[kB];
#pragma unroll
        for (int c = 0; c < kB; ++c) {
            const int r0c = s + c;
            const bool refl = c < nr;
            const cpx<T> al = {sh.alphas[c].re, sh.alphas[c].im};
            v[c] = csel(refl && r >= r0c, P[c], zero);
            w.V[c * ldi + r] = v[c];
            // Rows s .. s + c of column p + c are the band's (R above the
            // pivot, alpha at it); the zeros below lie outside the band and
            // are never read again.
            if (t <= c) A[r + (p + c) * ldi] = csel(!refl || r < r0c, P[c], csel(r == r0c, al, zero));
        }
        vt_row<T>(v, sh.Ts, vt);
#pragma unroll
        for (int l = 0; l < kB; ++l) w.W[l * ldi + r] = vt[l];
    }
    for (int idx = t; idx < kB * kB; idx += NT) w.Tm[idx] = sh.Ts[idx / kB][idx % kB];
}

// Panel QR for panels taller than a workgroup: thread t holds rows
// s + t + NT k (k < R) of W of the panel's columns at a time (R W complex
// values per thread).  The W-column sub-panels are factored left to right.
// Each is first brought up to date by the reflectors of the sub-panels before
// it in compact WY form, A_g <- (I - V T V^H)^H A_g = A_g - V T^H (V^H A_g),
// and after it the triangular factor grows by a block column,
// T = [[T0, -T0 (V0^H V1) T1], [0, T1]] (V1 the new reflectors, T1 their own
// factor).  A thread needs V only on its own rows, which it wrote itself, so
// V is read back without synchronisation.  Per reflector two workgroup
// reductions as in the one-row-per-thread kernel; per later sub-panel two
// more (V^H A_g and V0^H V1).  The panel is read and written once.
// Sub-panel width for R rows per thread: 256 bytes of panel per thread
// (64 registers).
template <typename T>
constexpr int kBlkW(int R) {
    return (int)(256 / (2 * sizeof(T))) / R;
}

// 32 rows per thread for complex64 (16, a variant launched above, for complex128).
template <typename T>
constexpr int kBlkR32 = sizeof(T) == 4 ? 32 : 16;

template <typename T, int NT, int SL>
struct QrBlkShared {
    double part[2][NT / 64][SL];  // per-wavefront reduce-scattered sums, two buffers in turn
    double dotw[NT / 64][SL];     // each wavefront's copy of the summed products
    double nred[2][NT / 64];  // column norms and pivots of consecutive reflectors alternate, so
    cpx<T> x0s[2];            // that no barrier is needed between a read and the next write
    cpx<T> Ts[kB][kB];
    cpx<T> Zs[kB][kB];  // T^H (V^H A_g), then (V0^H V1) T1
    cpx<T> alphas[kB];
};

// One chunk of 32 values of a workgroup sum: this wavefront's reduce-scatter
// into slots 32 chunk .. 32 chunk + 31 of `part`.
template <typename T, int NT, int SL>
__device__ __forceinline__ void blk_red_chunk(double (&part)[NT / 64][SL], int chunk, const T (&x)[32]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T r = wave_reduce_scatter32(x);
    if ((lane & 1) == 0) part[wid][32 * chunk + scatter_elem(lane)] = (double)r;
}
// After the chunks: one barrier, then every wavefront sums the NV values
// into its own copy and reads it back (a wavefront's LDS operations complete
// in order).  Consecutive sums alternate between the two buffers of `part`,
// so that a sum's writes never meet a slower wavefront's reads of the sum
// before the previous one (a barrier separates them).
template <int NT, int SL, int NV>
__device__ __forceinline__ const double *blk_red_finish(double (&part)[NT / 64][SL], double (&dotw)[NT / 64][SL]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
#pragma unroll
    for (int e = lane; e < NV; e += 64) {
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < NT / 64; ++q) sum += part[q][e];
        dotw[wid][e] = sum;
    }
    __builtin_amdgcn_wave_barrier();
    return dotw[wid];
}

template <typename T, int NT, int R>
__device__ __forceinline__ void blk_load_v(const TwoView<T> &w, int ldi, int s, int n, int q, cpx<T> (&vq)[R]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = s + t + NT * k;
        const cpx<T> a = w.V[r < n ? q * ldi + r : 0];
        vq[k] = csel(r < n, a, cpx<T>{T(0), T(0)});
    }
}

// X[q][c] = sum over the thread's rows of conj(V[q][r]) B[r][c] for the
// reflectors q < Q of earlier sub-panels (16 products per chunk), summed over
// the workgroup: X at 2 (q W + c) (re, im) of the returned copy.
// Reflectors per chunk of a V^H product: 16 products, or fewer when R rows of
// them would not stay in registers (at most 32 complex values of V per chunk).
template <int R, int W>
constexpr int kBlkQB = (16 / W) < (32 / R) ? (16 / W) : (32 / R);
// LDS slots of a workgroup sum: the largest V^H product (reflectors of all
// sub-panels but the last) in chunks of 32, at least one chunk.
template <int R, int W>
constexpr int kBlkSlots = 32 * ((kB - W + kBlkQB<R, W> - 1) / kBlkQB<R, W> > 1
                                    ? (kB - W + kBlkQB<R, W> - 1) / kBlkQB<R, W> : 1);
// Slot of X[q][c] (re; im at +1) in the summed copy: chunk q / QB holds
// 32 slots, of which it fills 2 QB W.
template <int R, int W>
__device__ __forceinline__ int blk_slot(int q, int c) {
    constexpr int QB = kBlkQB<R, W>;
    return 32 * (q / QB) + 2 * ((q % QB) * W + c);
}

template <typename T, int NT, int R, int W, int Q>
__device__ __forceinline__ const double *blk_vh_times(QrBlkShared<T, NT, kBlkSlots<R, W>> &sh, const TwoView<T> &w, int ldi, int s,
                                                      int n, const cpx<T> (&Bm)[R][W], int &pb) {
    constexpr int QB = kBlkQB<R, W>, NCH = (Q + QB - 1) / QB;
    static_assert(QB >= 1 && NCH * 32 <= kBlkSlots<R, W>, "chunks within the LDS slots");
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
        T x[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) x[j] = T(0);
#pragma unroll
        for (int qq = 0; qq < QB; ++qq) {
            if (ch * QB + qq >= Q) break;  // static: the last chunk's padding stays zero
            cpx<T> vq[R];
            blk_load_v<T, NT, R>(w, ldi, s, n, ch * QB + qq, vq);
#pragma unroll
            for (int c = 0; c < W; ++c) {
                cpx<T> acc = {T(0), T(0)};
#pragma unroll
                for (int k = 0; k < R; ++k) acc = c_add(acc, c_cmul(vq[k], Bm[k][c]));
                x[2 * (qq * W + c)] = acc.re;
                x[2 * (qq * W + c) + 1] = acc.im;
            }
        }
        blk_red_chunk<T, NT, kBlkSlots<R, W>>(sh.part[pb], ch, x);
    }
    const double *out = blk_red_finish<NT, kBlkSlots<R, W>, 32 * NCH>(sh.part[pb], sh.dotw);
    pb ^= 1;
    return out;
}

// Reflector I = c0 + C of the panel (column C of the sub-panel in P).
template <typename T, int NT, int R, int W, int C>
__device__ __forceinline__ void qr_blk_reflect(QrBlkShared<T, NT, kBlkSlots<R, W>> &sh, cpx<T> (&P)[R][W], int c0, int s, int n,
                                               int nr, int &pb) {
    constexpr int NW = NT / 64;
    const int I = c0 + C;
    if (I >= nr) return;  // uniform over the workgroup
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int r0 = s + I;
    const cpx<T> zero = {T(0), T(0)};
    // norm of column I from the pivot row down; the pivot is row s + I, which
    // thread I holds first
    double ws = 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = s + t + NT * k;
        ws += (r < n && r >= r0) ? (double)c_abs2(P[k][C]) : 0.0;
    }
    ws = col_sum(row_sum(ws));
    const int nb = I & 1;
    if (lane == 0) sh.nred[nb][wid] = ws;
    if (t == I) sh.x0s[nb] = P[0][C];
    __syncthreads();
    double nrm2 = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) nrm2 += sh.nred[nb][q];
    T tau;
    cpx<T> v0, alpha;
    make_reflector<T>(nrm2, sh.x0s[nb], tau, v0, alpha);
    cpx<T> v[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = s + t + NT * k;
        v[k] = csel(r == r0, v0, csel(r < n && r > r0, P[k][C], zero));
    }
    // (a one-column sub-panel has no other columns: no second reduction)
    if constexpr (W > 1) {
        // v^H P[:, c] for the sub-panel's columns c > C, V[:, c]^H v for c < C
        T x[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) x[j] = T(0);
#pragma unroll
        for (int c = 0; c < W; ++c) {
            cpx<T> acc = zero;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (c > C) acc = c_add(acc, c_cmul(v[k], P[k][c]));
                else if (c < C) acc = c_add(acc, c_cmul(P[k][c], v[k]));
            }
            x[2 * c] = acc.re;
            x[2 * c + 1] = acc.im;
        }
        blk_red_chunk<T, NT, kBlkSlots<R, W>>(sh.part[pb], 0, x);
        const double *d = blk_red_finish<NT, kBlkSlots<R, W>, 2 * W>(sh.part[pb], sh.dotw);
        pb ^= 1;
#pragma unroll
        for (int c = C + 1; c < W; ++c) {
            const cpx<T> dc = {(T)d[2 * c], (T)d[2 * c + 1]};
#pragma unroll
            for (int k = 0; k < R; ++k) P[k][c] = c_sub(P[k][c], c_scale(tau, c_mul(v[k], dc)));
        }
        // T[c0:I, I] = -tau T[c0:I, c0:I] (V^H v_I)[c0:I], T[I, I] = tau
        if (t >= c0 && t < I) {
            cpx<T> sum = zero;
            for (int q = t; q < I; ++q)
                sum = c_add(sum, c_mul(sh.Ts[t][q], cpx<T>{(T)d[2 * (q - c0)], (T)d[2 * (q - c0) + 1]}));
            sh.Ts[t][I] = c_scale(-tau, sum);
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) P[k][C] = csel(s + t + NT * k == r0, v0, P[k][C]);
    if (t == I) {
        sh.Ts[I][I] = {tau, T(0)};
        sh.alphas[I] = alpha;
    }
}
template <typename T, int NT, int R, int W, int... Cs>
__device__ __forceinline__ void qr_blk_reflect_all(QrBlkShared<T, NT, kBlkSlots<R, W>> &sh, cpx<T> (&P)[R][W], int c0, int s, int n,
                                                   int nr, int &pb, std::integer_sequence<int, Cs...>) {
    (qr_blk_reflect<T, NT, R, W, Cs>(sh, P, c0, s, n, nr, pb), ...);
}

// Sub-panel G (panel columns G W .. G W + W - 1).
template <typename T, int NT, int R, int W, int G>
__device__ __forceinline__ void qr_blk_subpanel(QrBlkShared<T, NT, kBlkSlots<R, W>> &sh, cpx<T> *A, const TwoView<T> &w, int ldi,
                                                int p, int s, int n, int nr, int &pb) {
    constexpr int c0 = G * W;
    const int t = threadIdx.x;
    const cpx<T> zero = {T(0), T(0)};
    cpx<T> P[R][W];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = s + t + NT * k;
#pragma unroll
        for (int c = 0; c < W; ++c) {
            const cpx<T> a = A[r < n ? r + (p + c0 + c) * ldi : 0];
            P[k][c] = csel(r < n, a, zero);
        }
    }
    if constexpr (G > 0) {
        // A_g <- A_g - V Z, Z = T^H (V^H A_g), over the reflectors q < c0
        const double *Y = blk_vh_times<T, NT, R, W, c0>(sh, w, ldi, s, n, P, pb);
        if (t < c0 * W) {
            const int q = t / W, c = t % W;
            cpx<T> z = zero;
            for (int q2 = 0; q2 <= q; ++q2)
                z = c_add(z, c_cmul(sh.Ts[q2][q], cpx<T>{(T)Y[blk_slot<R, W>(q2, c)], (T)Y[blk_slot<R, W>(q2, c) + 1]}));
            sh.Zs[q][c] = z;
        }
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < c0; ++q) {
            cpx<T> vq[R];
            blk_load_v<T, NT, R>(w, ldi, s, n, q, vq);
#pragma unroll
            for (int c = 0; c < W; ++c) {
                const cpx<T> zc = sh.Zs[q][c];
#pragma unroll
                for (int k = 0; k < R; ++k) P[k][c] = c_sub(P[k][c], c_mul(vq[k], zc));
            }
        }
    }
    qr_blk_reflect_all<T, NT, R, W>(sh, P, c0, s, n, nr, pb, std::make_integer_sequence<int, W>{});
    // V columns (zero above each pivot) and the band part of the panel
    // columns: rows s .. s + I of column p + I (R above the pivot, alpha at
    // it); the zeros below lie outside the band and are never read again.
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const int I = c0 + c, r0c = s + I;
        const bool refl = I < nr;
        const cpx<T> al = sh.alphas[I];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = s + t + NT * k;
            const cpx<T> vk = csel(refl && r >= r0c, P[k][c], zero);
            if (r < n) w.V[I * ldi + r] = vk;
            if (k == 0 && t <= I) A[r + (p + I) * ldi] = csel(!refl || r < r0c, P[k][c], csel(r == r0c, al, zero));
            P[k][c] = vk;
        }
    }
    if constexpr (G > 0) {
        // T[0:c0, c0:c0+W] = -T[0:c0, 0:c0] (V0^H V1) T[c0:c0+W, c0:c0+W]
        const double *X = blk_vh_times<T, NT, R, W, c0>(sh, w, ldi, s, n, P, pb);
        if (t < c0 * W) {
            const int q = t / W, c = t % W;
            cpx<T> m1 = zero;
            for (int c2 = 0; c2 <= c; ++c2)
                m1 = c_add(m1, c_mul(cpx<T>{(T)X[blk_slot<R, W>(q, c2)], (T)X[blk_slot<R, W>(q, c2) + 1]},
                                     sh.Ts[c0 + c2][c0 + c]));
            sh.Zs[q][c] = m1;
        }
        __syncthreads();
        if (t < c0 * W) {
            const int q = t / W, c = t % W;
            cpx<T> tq = zero;
            for (int q2 = q; q2 < c0; ++q2) tq = c_add(tq, c_mul(sh.Ts[q][q2], sh.Zs[q2][c]));
            sh.Ts[q][c0 + c] = {-tq.re, -tq.im};
        }
    }
}
template <typename T, int NT, int R, int W, int... Gs>
__device__ __forceinline__ void qr_blk_all(QrBlkShared<T, NT, kBlkSlots<R, W>> &sh, cpx<T> *A, const TwoView<T> &w, int ldi, int p,
                                           int s, int n, int nr, int &pb, std::integer_sequence<int, Gs...>) {
    (qr_blk_subpanel<T, NT, R, W, Gs>(sh, A, w, ldi, p, s, n, nr, pb), ...);
}

template <typename T, int NT, int R, int W>
__global__ __launch_bounds__(NT) void qr_panel_blk_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                          const int64_t *__restrict__ offs,
                                                          const int32_t *__restrict__ n_in,
                                                          cpx<T> *__restrict__ wall, int64_t stride, int p) {
    static_assert(kB % W == 0 && W * R * 2 * sizeof(T) == 256, "sub-panel of 256 bytes per thread");
    __shared__ QrBlkShared<T, NT, kBlkSlots<R, W>> sh;
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2 || m > NT * R) return;
    const int t = threadIdx.x;
    const int ldi = (int)ld;
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *A = Hall + mat_offset(offs, u, ld);
    const cpx<T> zero = {T(0), T(0)};
    for (int idx = t; idx < kB * kB; idx += NT) sh.Ts[idx / kB][idx % kB] = zero;
    const int nr = min(m - 1, kB);
    int pb = 0;
    // (the first reduction's barrier orders the zeroing of T before its writes)
    qr_blk_all<T, NT, R, W>(sh, A, w, ldi, p, s, n, nr, pb, std::make_integer_sequence<int, kB / W>{});
    __syncthreads();
    store_vt<T>(w, ld, s, n, t, NT, sh.Ts);  // V T for the Hermitian product (own rows of V)
    for (int idx = t; idx < kB * kB; idx += NT) w.Tm[idx] = sh.Ts[idx / kB][idx % kB];
}

// Raw operand loads of one hemm step (columns c0 .. c0 + 3) and their fix-up.
// Offsets are 32-bit (ld * ld fits) and selects are per real component, so
// that the loads are straight-line code.
template <typename T, int NTL>
__device__ __forceinline__ void hemm_fetch(const cpx<T> *A, const cpx<T> *V, int ld, int n, int rb, int c0,
                                           cpx<T> (&a)[NTL], cpx<T> &vb) {
    const int lane = threadIdx.x, ii = lane & 15, c = c0 + (lane >> 4);
    vb = V[c < n ? ii * ld + c : 0];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        const int r = rb + 16 * t + ii;
        const int hi = r > c ? r : c, lo = r > c ? c : r;
        a[t] = A[(r < n && c < n) ? hi + lo * ld : 0];
    }
}
template <typename T, int NTL>
__device__ __forceinline__ void hemm_fix(int n, int rb, int c0, cpx<T> (&a)[NTL], cpx<T> &vb) {
    const int lane = threadIdx.x, ii = lane & 15, c = c0 + (lane >> 4);
    vb.re = c < n ? vb.re : T(0);
    vb.im = c < n ? vb.im : T(0);
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        const int r = rb + 16 * t + ii;
        const bool ok = r < n && c < n;
        const T re = a[t].re, im = a[t].im;
        a[t].re = ok ? re : T(0);
        a[t].im = (ok && c != r) ? (c > r ? -im : im) : T(0);
    }
}

// After the Hermitian product of a wavefront's row block (rows rb ..,
// NTL tiles of 16): its rows of X T, and Z_b = V_rows^H (X T)_rows for each
// 16-row tile b, on the matrix cores (the accumulators are already laid out
// as the B operand of a 4-row step), into Zall[b][16][16] for the W factor.
template <typename T, int NTL, typename Acc>
__device__ __forceinline__ void hemm_finish(const Acc (&acc)[NTL], const cpx<T> *Vo, cpx<T> *X, cpx<T> *Z,
                                            int ldi, int n, int rb) {
    using v4 = typename Mfma<T>::v4;
    const int lane = (int)threadIdx.x & 63, ii = lane & 15;
    cpx<T> vz[NTL][4];
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb + 16 * t + Mfma<T>::row(lane, v);
            vz[t][v] = Vo[r < n ? ii * ldi + r : 0];
        }
    v4 dre[NTL], dim[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        dre[t] = acc[t].re();
        dim[t] = acc[t].im();
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb + 16 * t + Mfma<T>::row(lane, v);
            if (r < n) X[ii * ldi + r] = {dre[t][v], dim[t][v]};
        }
    // Z_b[i][l] = sum_r conj(V[r][i]) (X T)[r][l]: step (t, v) takes the rows
    // rb + 16 t + row(lane, v), lane supplying A[ii][kk] = conj(V[r][ii]) and
    // B[kk][ii] = (X T)[r][ii] (its own accumulator entry).
    // One partial per 16-row tile, so that the sums do not depend on how
    // many tiles a wavefront takes.
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
        v4 zre = v4{T(0), T(0), T(0), T(0)}, zim = v4{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = rb + 16 * t + Mfma<T>::row(lane, v);
            const cpx<T> vr = vz[t][v];
            const cpx<T> a = {r < n ? vr.re : T(0), r < n ? -vr.im : T(0)};
            cmma<T>(a, cpx<T>{dre[t][v], dim[t][v]}, zre, zim);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Z[t * kB * kB + Mfma<T>::row(lane, v) * kB + ii] = {zre[v], zim[v]};
    }
}

// X T = A22 (V T) on the matrix cores: one wavefront per 16 NTL output rows
// (NTL 16-row tiles: four, or fewer when the batch is too small to give
// every SIMD two wavefronts) x 16 columns; each step consumes 4 columns of
// A22.
template <typename T, int NTL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void hemm_kernel(
    const cpx<T> *__restrict__ Hall, int64_t ld, const int64_t *__restrict__ offs, const int32_t *__restrict__ n_in,
    const cpx<T> *__restrict__ VTall,
    const cpx<T> *__restrict__ Vall, cpx<T> *__restrict__ Xall, cpx<T> *__restrict__ Zall, int64_t stride, int p,
    int64_t batch, int64_t tiles) {
    int64_t u, tile;
    xcd_tile(blockIdx.x, tiles, u, tile);
    if (u >= batch) return;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    constexpr int kRows = 16 * NTL;
    const int rb = s + (int)tile * kRows;
    if (rb >= n) return;
    const cpx<T> *A = Hall + mat_offset(offs, u, ld);
    const cpx<T> *V = VTall + u * stride;
    CAcc3<T> acc[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t].zero();
    // Raw loads (every lane loads from a valid address: the stored lower
    // element of its position, element 0 when outside the matrix) are issued
    // kHemmDepth - 1 steps ahead into a ring of register sets; the fix-up
    // (mask, conjugation of mirrored elements, real diagonal) happens at
    // use, so no load is waited for early.  The empty asm with a memory
    // clobber after each prefetch keeps the compiler from turning the
    // loop-carried loaded values into loop-carried addresses (which would
    // move the loads down to their use).
    //
    // Column order: the wavefront of 64-row block I starts at column offset
    // -64 I (mod m, in steps of 4 columns) and wraps around, so that the
    // wavefronts of a matrix do not all stream the same columns at the same
    // time (about 9 % faster than all starting at column s).  Steps past
    // the last one (the step count is padded to a multiple of kHemmDepth)
    // read column n, which is masked to zero.
    constexpr int D = kHemmDepth;
    cpx<T> a[D][NTL], b[D];
    int cs[D];
    const int ldi = (int)ld;
    const int m4 = (m + 3) & ~3, nst = m4 / 4;
    // (the offset follows the 64-row block, so that every row sums its
    // columns in the same order whatever NTL is)
    int of = (m4 - ((kRows * (int)tile) & ~63) % m4) % m4, fetched = 0;
    auto fetch_next = [&](int slot) {
        cs[slot] = fetched < nst ? s + of : n;
        hemm_fetch<T, NTL>(A, V, ldi, n, rb, cs[slot], a[slot], b[slot]);
        of = of + 4 >= m4 ? 0 : of + 4;
        ++fetched;
    };
#pragma unroll
    for (int i = 0; i < D - 1; ++i) fetch_next(i);
    for (int q = 0; q < nst; q += D) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            fetch_next((i + D - 1) % D);
            asm volatile("" ::: "memory");
            hemm_fix<T, NTL>(n, rb, cs[i], a[i], b[i]);
#pragma unroll
            for (int t = 0; t < NTL; ++t) acc[t].mma(a[i][t], a[i][t].re + a[i][t].im, b[i], b[i].re + b[i].im);
        }
    }
    hemm_finish<T, NTL>(acc, Vall + u * stride, Xall + u * stride, Zall + u * stride + (int64_t)tile * NTL * kB * kB,
                        ldi, n, rb);
}

// ---------------------------------------------------------------------------
// Stage 1: W = X T - 1/2 V Y, Y = T^H Z, Z = sum over the Hermitian product's
// 16-row tiles of V_rows^H (X T)_rows.  `rblocks` workgroups per matrix, each
// forming Y and taking every rblocks-th block of 256 rows (several when the
// batch is too small to fill the chip).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kWThreads) void wfactor_kernel(const int32_t *__restrict__ n_in, int64_t ld,
                                                            cpx<T> *__restrict__ wall, int64_t stride, int p,
                                                            int rblocks) {
    __shared__ cpx<T> Ts[kB][kB], Zs[kB][kB], Y[kB][kB];
    static_assert(kWThreads == kB * kB, "one thread per entry of the 16 x 16 factors");
    const int64_t u = blockIdx.x / rblocks;
    const int rb = (int)(blockIdx.x % rblocks);
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    const int t = threadIdx.x, k = t / kB, l = t % kB;
    const TwoView<T> w(wall, stride, ld, u);
    const cpx<T> *Zp = hemm_partials(w, ld);
    const int blocks = (m + 15) / 16;  // the Hermitian product's 16-row tiles
    Ts[k][l] = w.Tm[t];
    // four partial sums over the tiles b = i (mod 4), then their sum in
    // order: a fixed order, with four independent chains of loads and adds
    cpx<T> z4[4] = {{T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}, {T(0), T(0)}};
    int b = 0;
    for (; b + 4 <= blocks; b += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z4[i] = c_add(z4[i], Zp[(int64_t)(b + i) * kB * kB + t]);
    }
    for (int i = 0; b + i < blocks; ++i) z4[i] = c_add(z4[i], Zp[(int64_t)(b + i) * kB * kB + t]);
    Zs[k][l] = c_add(c_add(z4[0], z4[1]), c_add(z4[2], z4[3]));
    __syncthreads();
    cpx<T> y = {T(0), T(0)};  // Y = T^H Z, T upper triangular
    for (int q = 0; q <= k; ++q) y = c_add(y, c_cmul(Ts[q][k], Zs[q][l]));
    Y[k][l] = y;
    __syncthreads();
#pragma unroll 1
    for (int r = s + kWThreads * rb + t; r < n; r += kWThreads * rblocks) {
        cpx<T> v[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) v[q] = w.V[(int64_t)q * ld + r];
        const int zr = r >> 30;  // 0, but keeps the 16 x 16 table in LDS rather than in (spilled) registers
        for (int c = 0; c < kB; ++c) {
            cpx<T> sum = {T(0), T(0)};
#pragma unroll
            for (int q = 0; q < kB; ++q) sum = c_add(sum, c_mul(v[q], Y[q + zr][c]));
            w.W[(int64_t)c * ld + r] = c_sub(w.X[(int64_t)c * ld + r], c_scale(T(0.5), sum));
        }
    }
}

// ---------------------------------------------------------------------------
// Stage 1: A22 -= V W^H + W V^H on the lower triangle.  A workgroup owns a
// 64 x 64 block and stages its rows' and columns' V, W in LDS; each lane
// accumulates a 4 x 4 micro-tile.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void band_update_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                          const int64_t *__restrict__ offs,
                                                          const int32_t *__restrict__ n_in, cpx<T> *__restrict__ wall,
                                                          int64_t stride, int p, int64_t batch, int64_t tiles,
                                                          int min_m) {
    __shared__ cpx<T> sVr[kB][kUpdBlk], sWr[kB][kUpdBlk], sVc[kB][kUpdBlk], sWc[kB][kUpdBlk];
    int64_t u, tile;
    xcd_tile(blockIdx.x, tiles, u, tile);
    if (u >= batch) return;
    const int n = n_in[u];
    const int s = p + kB;
    if (n < 0 || n > ld || n - s < min_m) return;
    // lower-triangle tile (bi, bj), bj <= bi, from tile = bi (bi + 1) / 2 + bj
    int bi = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((int64_t)bi * (bi + 1) / 2 > tile) --bi;
    while ((int64_t)(bi + 1) * (bi + 2) / 2 <= tile) ++bi;
    const int bj = (int)(tile - (int64_t)bi * (bi + 1) / 2);
    const int rb = s + bi * kUpdBlk, cb = s + bj * kUpdBlk;
    if (rb >= n || cb > rb + kUpdBlk - 1) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int ii = lane & 15, kk = lane >> 4;
    const TwoView<T> w(wall, stride, ld, u);
    const int ldi = (int)ld;
    // Stage the V, W strips of the tile's rows and columns (straight-line
    // loads, out-of-range entries read element 0 and are zeroed at the store).
    constexpr int kFill = kB * kUpdBlk / 256;
    cpx<T> fv[kFill][4];
#pragma unroll
    for (int q = 0; q < kFill; ++q) {
        const int idx = t + 256 * q, k = idx / kUpdBlk, l = idx % kUpdBlk;
        const int r = rb + l, c = cb + l;
        fv[q][0] = w.V[r < n ? k * ldi + r : 0];
        fv[q][1] = w.W[r < n ? k * ldi + r : 0];
        fv[q][2] = w.V[c < n ? k * ldi + c : 0];
        fv[q][3] = w.W[c < n ? k * ldi + c : 0];
    }
    // This wave's part of the tile: rows rb + 16 tt + ii, columns cs + row(lane, v),
    // loaded now so that the loads are in flight during the products.
    const int cs = cb + wid * 16;
    cpx<T> *A = Hall + mat_offset(offs, u, ld);
    cpx<T> x[4][4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int r = rb + 16 * tt + ii;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = cs + Mfma<T>::row(lane, v);
            x[tt][v] = A[(r < n && c < n && r >= c) ? r + c * ldi : 0];
        }
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = 0; q < kFill; ++q) {
        const int idx = t + 256 * q, k = idx / kUpdBlk, l = idx % kUpdBlk;
        const bool okr = rb + l < n, okc = cb + l < n;
        sVr[k][l] = {okr ? fv[q][0].re : T(0), okr ? fv[q][0].im : T(0)};
        sWr[k][l] = {okr ? fv[q][1].re : T(0), okr ? fv[q][1].im : T(0)};
        sVc[k][l] = {okc ? fv[q][2].re : T(0), okc ? fv[q][2].im : T(0)};
        sWc[k][l] = {okc ? fv[q][3].re : T(0), okc ? fv[q][3].im : T(0)};
    }
    __syncthreads();
    if (cs >= n || cs > rb + kUpdBlk - 1) return;
    // (V W^H + W V^H)[r, c] = sum_k P[r, k] conj(Q[c, k]) with P = [V W], Q = [W V]
    // (k < 2 kB).  The matrix cores compute the transposed tile
    // D[c][r] = sum_k conj(Q[c, k]) P[r, k] so that the lane-fast index of the
    // result is the row r of A (coalesced column-major read-modify-write).
    CAcc3<T> acc[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) acc[tt].zero();
    // In a diagonal tile, row blocks above this wavefront's 16 columns lie in
    // the upper triangle (never stored): in FP64 their products are skipped
    // (in FP32 the branches cost the kernel a wavefront per SIMD, more than
    // the skipped products save).
    constexpr bool kSkipUpper = sizeof(T) == 8;
    const int tt0 = (kSkipUpper && rb == cb) ? __builtin_amdgcn_readfirstlane(wid) : 0;
#pragma unroll 2
    for (int k0 = 0; k0 < 2 * kB; k0 += 4) {
        const int k = k0 + kk;
        const cpx<T> a = c_conj((k < kB) ? sWc[k][wid * 16 + ii] : sVc[k - kB][wid * 16 + ii]);
        const T as = a.re + a.im;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            if (tt < tt0) continue;
            const cpx<T> b = (k < kB) ? sVr[k][16 * tt + ii] : sWr[k - kB][16 * tt + ii];
            acc[tt].mma(a, as, b, b.re + b.im);
        }
    }
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int r = rb + 16 * tt + ii;
        const typename Mfma<T>::v4 dre = acc[tt].re(), dim = acc[tt].im();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = cs + Mfma<T>::row(lane, v);
            if (r < n && c < n && r >= c) A[r + c * ldi] = c_sub(x[tt][v], cpx<T>{dre[v], dim[v]});
        }
    }
}

// The same update with 32 x 64 tiles (32 rows, 64 columns) and 16 KiB of LDS:
// only the rows' V, W strips are staged; each wavefront loads the V, W
// entries of its own 16 columns (the A operand) from L2 into registers.  Its
// workgroups fit beside a chase workgroup on one CU, which the 64 x 64 tiles
// (64 KiB) do not.  Lower tiles (bi, bj) have bj <= bi / 2; with a = bi / 2
// rows 2a and 2a + 1 hold a + 1 tiles each, so tile t lies in rows 2a or
// 2a + 1 for a (a + 1) <= t < (a + 1) (a + 2).
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void band_update32_kernel(
    cpx<T> *__restrict__ Hall, int64_t ld, const int64_t *__restrict__ offs, const int32_t *__restrict__ n_in,
    cpx<T> *__restrict__ wall, int64_t stride, int p, int64_t batch, int64_t tiles, int min_m) {
    constexpr int R = kUpdBlk / 2;  // rows per tile
    __shared__ cpx<T> sVr[kB][R], sWr[kB][R];
    int64_t u, tile;
    xcd_tile(blockIdx.x, tiles, u, tile);
    if (u >= batch) return;
    const int n = n_in[u];
    const int s = p + kB;
    if (n < 0 || n > ld || n - s < min_m) return;
    int a = (int)((sqrt(4.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((int64_t)a * (a + 1) > tile) --a;
    while ((int64_t)(a + 1) * (a + 2) <= tile) ++a;
    const int64_t t0 = tile - (int64_t)a * (a + 1);
    const int bi = t0 < a + 1 ? 2 * a : 2 * a + 1;
    const int bj = (int)(t0 < a + 1 ? t0 : t0 - (a + 1));
    const int rb = s + bi * R, cb = s + bj * kUpdBlk;
    if (rb >= n || cb > rb + R - 1) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int ii = lane & 15, kk = lane >> 4;
    const TwoView<T> w(wall, stride, ld, u);
    const int ldi = (int)ld;
    // Row strips (16 x 32 of V and of W: two entries per thread).
    cpx<T> fv[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int idx = t + 256 * q, k = idx / R, l = idx % R, r = rb + l;
        fv[q][0] = w.V[r < n ? k * ldi + r : 0];
        fv[q][1] = w.W[r < n ? k * ldi + r : 0];
    }
    // This wavefront's columns cs + ii: the A operand of step k0 is
    // conj(Q[c, k0 + kk]) with Q = [W V] (k < 2 kB); and its part of the tile,
    // rows rb + 16 tt + ii, columns cs + row(lane, v).
    const int cs = cb + wid * 16, c = cs + ii;
    cpx<T> af[2 * kB / 4];
#pragma unroll
    for (int q = 0; q < 2 * kB / 4; ++q) {
        const int k = 4 * q + kk;
        af[q] = (k < kB ? w.W : w.V)[c < n ? (k & (kB - 1)) * ldi + c : 0];
    }
    cpx<T> *A = Hall + mat_offset(offs, u, ld);
    cpx<T> x[2][4];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const int r = rb + 16 * tt + ii;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int cc = cs + Mfma<T>::row(lane, v);
            x[tt][v] = A[(r < n && cc < n && r >= cc) ? r + cc * ldi : 0];
        }
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int idx = t + 256 * q, k = idx / R, l = idx % R;
        const bool ok = rb + l < n;
        sVr[k][l] = {ok ? fv[q][0].re : T(0), ok ? fv[q][0].im : T(0)};
        sWr[k][l] = {ok ? fv[q][1].re : T(0), ok ? fv[q][1].im : T(0)};
    }
    __syncthreads();
    if (cs >= n || cs > rb + R - 1) return;
    CAcc3<T> acc[2];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) acc[tt].zero();
    // Row tiles wholly above this wavefront's columns lie in the upper
    // triangle (never stored) and are skipped.
    const int tt0 = __builtin_amdgcn_readfirstlane(rb + 15 < cs ? 1 : 0);
#pragma unroll
    for (int q = 0; q < 2 * kB / 4; ++q) {
        const int k = 4 * q + kk;
        const bool ok = c < n;
        const cpx<T> ac = {ok ? af[q].re : T(0), ok ? -af[q].im : T(0)};
        const T as = ac.re + ac.im;
#pragma unroll
        for (int tt = 0; tt < 2; ++tt) {
            if (tt < tt0) continue;
            const cpx<T> b = (k < kB) ? sVr[k][16 * tt + ii] : sWr[k - kB][16 * tt + ii];
            acc[tt].mma(ac, as, b, b.re + b.im);
        }
    }
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
        const int r = rb + 16 * tt + ii;
        const typename Mfma<T>::v4 dre = acc[tt].re(), dim = acc[tt].im();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int cc = cs + Mfma<T>::row(lane, v);
            if (r < n && cc < n && r >= cc) A[r + cc * ldi] = c_sub(x[tt][v], cpx<T>{dre[v], dim[v]});
        }
    }
}

// Panel p's V [16][ld] and T [16][16] of every matrix into its reflector
// store (slot p / 16); matrices whose panel has no reflectors (fewer than two
// rows below the band) are skipped, as the panel kernels skip them.
template <typename T>
__global__ __launch_bounds__(256) void keep_panel_kernel(const int32_t *__restrict__ n_in, int64_t ld,
                                                         const cpx<T> *__restrict__ wall, int64_t stride, int p,
                                                         cpx<T> *__restrict__ keep, int64_t keep_stride) {
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 0 || n > ld || m < 2) return;
    const TwoView<T> w(const_cast<cpx<T> *>(wall), stride, ld, u);
    cpx<T> *kp = keep + u * keep_stride + (int64_t)(p / kB) * (kB * ld + kB * kB);
    for (int64_t idx = threadIdx.x; idx < (int64_t)kB * m; idx += 256) {
        const int c = (int)(idx / m), r = s + (int)(idx % m);
        kp[(int64_t)c * ld + r] = w.V[(int64_t)c * ld + r];
    }
    for (int idx = threadIdx.x; idx < kB * kB; idx += 256) kp[(int64_t)kB * ld + idx] = w.Tm[idx];
}

template <typename T>
hipError_t band_reduce_impl(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work, hipStream_t s,
                            int64_t stride, const int64_t *offs, int upd_rows, cpx<T> *keep, int64_t keep_stride);

template <typename T>
hipError_t launch_band_reduce(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                              hipStream_t s, int64_t stride, const int64_t *offs, int upd_rows) {
    return band_reduce_impl<T>(H, ld, n_in, batch, work, s, stride, offs, upd_rows, nullptr, 0);
}

template <typename T>
hipError_t launch_band_reduce_keep(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                   hipStream_t s, int64_t stride, const int64_t *offs, cpx<T> *keep,
                                   int64_t keep_stride) {
    if (!keep || keep_stride < eigh_keep_elems(ld)) return hipErrorInvalidValue;
    return band_reduce_impl<T>(H, ld, n_in, batch, work, s, stride, offs, 32, keep, keep_stride);
}

template <typename T>
hipError_t band_reduce_impl(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work, hipStream_t s,
                            int64_t stride, const int64_t *offs, int upd_rows, cpx<T> *keep, int64_t keep_stride) {
    if (upd_rows != 32 && upd_rows != 64) return hipErrorInvalidValue;
    if (batch == 0) return hipSuccess;
    if (stride == 0) stride = (int64_t)tridiag_twostage_work_elems<T>(ld);
    if (stride < (int64_t)tridiag_twostage_work_elems<T>(ld)) return hipErrorInvalidValue;
    const unsigned B = (unsigned)batch;
    for (int p = 0; p + kB + 1 < ld; p += kB) {
        const int64_t mmax = ld - p - kB;
        hipError_t err = timed_call("s1_panel", s, [&]() {
            if (mmax <= 64)
                hipLaunchKernelGGL((qr_panel_reg_kernel<T, 64>), dim3(B), dim3(64), 0, s, H, ld, offs, n_in, work,
                                   stride, p);
            else if (mmax <= 128)
                hipLaunchKernelGGL((qr_panel_reg_kernel<T, 128>), dim3(B), dim3(128), 0, s, H, ld, offs, n_in, work,
                                   stride, p);
            else if (mmax <= 256)
                hipLaunchKernelGGL((qr_panel_reg_kernel<T, 256>), dim3(B), dim3(256), 0, s, H, ld, offs, n_in, work,
                                   stride, p);
            else if (mmax <= 512)
                hipLaunchKernelGGL((qr_panel_reg_kernel<T, 512>), dim3(B), dim3(512), 0, s, H, ld, offs, n_in, work,
                                   stride, p);
            else if (mmax <= 1024)
                hipLaunchKernelGGL((qr_panel_blk_kernel<T, 512, 2, kBlkW<T>(2)>), dim3(B), dim3(512), 0, s, H, ld,
                                   offs, n_in, work, stride, p);
            else if (mmax <= 2048)
                hipLaunchKernelGGL((qr_panel_blk_kernel<T, 512, 4, kBlkW<T>(4)>), dim3(B), dim3(512), 0, s, H, ld,
                                   offs, n_in, work, stride, p);
            else if (mmax <= 4096)
                hipLaunchKernelGGL((qr_panel_blk_kernel<T, 512, 8, kBlkW<T>(8)>), dim3(B), dim3(512), 0, s, H, ld,
                                   offs, n_in, work, stride, p);
            else if (mmax <= 8192)
                hipLaunchKernelGGL((qr_panel_blk_kernel<T, 512, 16, kBlkW<T>(16)>), dim3(B), dim3(512), 0, s, H, ld,
                                   offs, n_in, work, stride, p);
            else if (sizeof(T) == 4 && mmax <= 16384)  // (32 complex128 rows per thread would not fit)
                hipLaunchKernelGGL((qr_panel_blk_kernel<T, 512, kBlkR32<T>, kBlkW<T>(kBlkR32<T>)>), dim3(B),
                                   dim3(512), 0, s, H, ld, offs, n_in, work, stride, p);
            else
                hipLaunchKernelGGL(qr_panel_kernel<T>, dim3(B), dim3(kQrThreads), 0, s, H, ld, offs, n_in, work,
                                   stride, p);
            return hipGetLastError();
        });
        if (err != hipSuccess) return err;
        if (keep) {
            hipLaunchKernelGGL(keep_panel_kernel<T>, dim3(B), dim3(256), 0, s, n_in, ld, work, stride, p, keep,
                               keep_stride);
            err = hipGetLastError();
            if (err != hipSuccess) return err;
        }
        // Row tiles per wavefront: four, unless the batch gives fewer than
        // four wavefronts per SIMD that way (a small batch of large matrices).
        const int64_t waves4 = (int64_t)kXcds * ((batch + kXcds - 1) / kXcds) * ((mmax + 63) / 64);
        const int ntl = waves4 >= 4096 ? 4 : (2 * waves4 >= 4096 ? 2 : 1);
        const int hemm_rows = 16 * ntl;
        const int64_t hrows = (mmax + hemm_rows - 1) / hemm_rows;
        err = timed_call("s1_hemm", s, [&]() {
            const cpx<T> *vt = work + 2 * (int64_t)kB * ld;
            cpx<T> *xo = work + (int64_t)kB * ld, *zo = work + hemm_partials_offset(ld);
            if (ntl == 4)
                hipLaunchKernelGGL((hemm_kernel<T, 4>), dim3(xcd_grid(batch, hrows)), dim3(64), 0, s, H, ld, offs,
                                   n_in, vt, work, xo, zo, stride, p, batch, hrows);
            else if (ntl == 2)
                hipLaunchKernelGGL((hemm_kernel<T, 2>), dim3(xcd_grid(batch, hrows)), dim3(64), 0, s, H, ld, offs,
                                   n_in, vt, work, xo, zo, stride, p, batch, hrows);
            else
                hipLaunchKernelGGL((hemm_kernel<T, 1>), dim3(xcd_grid(batch, hrows)), dim3(64), 0, s, H, ld, offs,
                                   n_in, vt, work, xo, zo, stride, p, batch, hrows);
            return hipGetLastError();
        });
        if (err != hipSuccess) return err;
        err = timed_call("s1_wfactor", s, [&]() {
            const int64_t rmax = (mmax + kWThreads - 1) / kWThreads;
            const int rblocks = (int)std::max<int64_t>(1, std::min<int64_t>(rmax, (512 + batch - 1) / batch));
            hipLaunchKernelGGL(wfactor_kernel<T>, dim3(B * rblocks), dim3(kWThreads), 0, s, n_in, ld, work, stride,
                               p, rblocks);
            return hipGetLastError();
        });
        if (err != hipSuccess) return err;
        err = timed_call("s1_update", s, [&]() {
            if (upd_rows == 32) {
                const int64_t nb32 = (mmax + kUpdBlk / 2 - 1) / (kUpdBlk / 2), ha = (nb32 - 1) / 2;
                const int64_t ntile = (nb32 % 2 == 0) ? (ha + 1) * (ha + 2) : (ha + 1) * (ha + 1);
                hipLaunchKernelGGL(band_update32_kernel<T>, dim3(xcd_grid(batch, ntile)), dim3(256), 0, s, H, ld,
                                   offs, n_in, work, stride, p, batch, ntile, 2);
            } else {
                const int64_t nblk = (mmax + kUpdBlk - 1) / kUpdBlk, ntile = nblk * (nblk + 1) / 2;
                hipLaunchKernelGGL(band_update_kernel<T>, dim3(xcd_grid(batch, ntile)), dim3(256), 0, s, H, ld,
                                   offs, n_in, work, stride, p, batch, ntile, 2);
            }
            return hipGetLastError();
        });
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// A22 <- A22 - V W^H - W V^H on the lower triangle of the trailing matrix
// below panel p (rows and columns p + 16 .. n - 1), V and W from the
// per-matrix workspace (stride elements apart); skipped when fewer than
// min_m trailing rows remain.
template <typename T>
hipError_t launch_rank2k_update(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, cpx<T> *work,
                                int64_t stride, int p, int min_m, hipStream_t s) {
    if (batch == 0 || p + kB >= ld) return hipSuccess;
    const int64_t mmax = ld - p - kB;
    const int64_t nblk = (mmax + kUpdBlk - 1) / kUpdBlk, ntile = nblk * (nblk + 1) / 2;
    hipLaunchKernelGGL(band_update_kernel<T>, dim3(xcd_grid(batch, ntile)), dim3(256), 0, s, H, ld,
                       (const int64_t *)nullptr, n_in, work, stride,
                       p, batch, ntile, min_m);
    return hipGetLastError();
}

template hipError_t launch_rank2k_update<double>(cpx<double> *, int64_t, const int32_t *, int64_t, cpx<double> *,
                                                 int64_t, int, int, hipStream_t);
template hipError_t launch_rank2k_update<float>(cpx<float> *, int64_t, const int32_t *, int64_t, cpx<float> *,
                                                int64_t, int, int, hipStream_t);
template size_t tridiag_twostage_work_elems<double>(int64_t);
template size_t tridiag_twostage_work_elems<float>(int64_t);
template hipError_t launch_band_reduce_keep<double>(cpx<double> *, int64_t, const int32_t *, int64_t,
                                                    cpx<double> *, hipStream_t, int64_t, const int64_t *,
                                                    cpx<double> *, int64_t);
template hipError_t launch_band_reduce_keep<float>(cpx<float> *, int64_t, const int32_t *, int64_t, cpx<float> *,
                                                   hipStream_t, int64_t, const int64_t *, cpx<float> *, int64_t);
template hipError_t launch_band_reduce<double>(cpx<double> *, int64_t, const int32_t *, int64_t, cpx<double> *,
                                               hipStream_t, int64_t, const int64_t *, int);
template hipError_t launch_band_reduce<float>(cpx<float> *, int64_t, const int32_t *, int64_t, cpx<float> *,
                                              hipStream_t, int64_t, const int64_t *, int);

}  // namespace mlmc
