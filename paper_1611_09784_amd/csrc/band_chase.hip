// Stage 2 of the two-stage Householder tridiagonalisation: band of
// half-width kB -> tridiagonal (d, e), by bulge chasing, one wavefront per
// matrix.  The band is copied to a compact column-major band array with room
// for the bulge (2*kB sub-diagonals).  Sweep j annihilates column j below the
// sub-diagonal with a reflector on rows j+1..j+kB, applied two-sidedly to the
// kB x kB diagonal block and from the right to the block below, which fills
// it; the fill's first column is then annihilated by the next reflector, and
// so on down the band.  Each 16 x 16 block lives in registers (16 row lanes x
// 4 column lanes, 4 columns per lane); each step's blocks are loaded one step
// ahead, and two sweeps are in flight at a time.
#include "twostage_common.hpp"

namespace mlmc {

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

// Block loads are split into a raw load (every lane loads from a valid
// address, masked lanes from element 0) and a fix-up (mask, conjugation)
// applied where the block is first used, so that a prefetch stays in flight
// across the current step's arithmetic instead of being waited for at once.
// Raw load of A[r0 + r, c0 + c] (r < nrow, c < ncol); every such element lies
// on or below the diagonal and within the stored band.
template <typename T>
__device__ __forceinline__ void load_blk_raw(const cpx<T> *band, int r0, int c0, int nrow, int ncol, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        const bool ok = r < nrow && c < ncol;
        const int64_t idx = ok ? (int64_t)(c0 + c) * kBandLd + (r0 + r - c0 - c) : 0;
        b.e[tt] = band[idx];
    }
}
template <typename T>
__device__ __forceinline__ void fix_blk(int nrow, int ncol, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const bool ok = r < nrow && g + 4 * tt < ncol;
        if (!ok) b.e[tt] = {T(0), T(0)};
    }
}
// Raw load of the Hermitian diagonal block A[r0.., r0..] of size L: every
// lane loads the stored (lower) element of its mirrored position.
template <typename T>
__device__ __forceinline__ void load_diag_raw(const cpx<T> *band, int r0, int L, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        const bool ok = r < L && c < L;
        const int hi = r > c ? r : c, lo = r > c ? c : r;
        const int64_t idx = ok ? (int64_t)(r0 + lo) * kBandLd + (hi - lo) : 0;
        b.e[tt] = band[idx];
    }
}
template <typename T>
__device__ __forceinline__ void fix_diag(int L, Blk<T> &b) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        const cpx<T> x = b.e[tt];
        const T im = (r == c) ? T(0) : ((r < c) ? -x.im : x.im);
        b.e[tt] = (r < L && c < L) ? cpx<T>{x.re, im} : cpx<T>{T(0), T(0)};
    }
}

template <typename T>
__device__ __forceinline__ cpx<T> sum16(cpx<T> x) {  // over the 16 row lanes of a column group
    return {row_sum(x.re), row_sum(x.im)};
}
template <typename T>
__device__ __forceinline__ cpx<T> sum4g(cpx<T> x) {  // over the 4 column groups of a row
    return {col_sum(x.re), col_sum(x.im)};
}

// State of one sweep of the chase: B (the block below the previous
// diagonal block, in registers) and the raw loads of the current step's
// diagonal block D and block below E; rows lo..hi carry the current
// reflector, lo1..hi1 the block below, col0 is the first column of B.
template <typename T>
struct Sweep {
    Blk<T> B, D, E;
    int lo, hi, L, lo1, hi1, L1, col0, Lprev, steps;
    bool on;
};

template <typename T>
__device__ __forceinline__ void sweep_start(const cpx<T> *band, int n, int j, Sweep<T> &S) {
    S.lo = j + 1;
    S.hi = min(j + kB, n - 1);
    S.L = S.hi - S.lo + 1;
    S.lo1 = S.hi + 1;
    S.hi1 = min(S.hi + kB, n - 1);
    S.L1 = S.hi1 - S.lo1 + 1;
    S.col0 = j;  // step 0: the "previous block" is column j itself
    S.Lprev = 1;
    S.steps = 0;
    S.on = true;
    load_blk_raw(band, S.lo, j, S.L, 1, S.B);
    load_diag_raw(band, S.lo, S.L, S.D);
    load_blk_raw(band, S.lo1, S.lo, S.L1, S.L, S.E);
}

// One step of a sweep: reflector from the first column of B on rows lo..hi,
// applied as B <- H B, D <- H D H, E <- E H; B and D are final and stored;
// E becomes the next B.  The next step's D and E are loaded first (they are
// disjoint from this step's stores).
template <typename T>
__device__ __forceinline__ void sweep_step(cpx<T> *band, int n, int64_t discard, Sweep<T> &S) {
    const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
    const cpx<T> zero = {T(0), T(0)};
    if (S.steps == 0) fix_blk(S.L, 1, S.B);
    Blk<T> B = S.B, D = S.D, E = S.E;
    fix_diag(S.L, D);
    fix_blk(S.L1, S.L, E);
    const int lo2 = S.hi1 + 1, hi2 = min(S.hi1 + kB, n - 1), L2 = hi2 - lo2 + 1;
    load_diag_raw(band, S.lo1, S.L1, S.D);
    load_blk_raw(band, lo2, S.lo1, L2, S.L1, S.E);
    const int L = S.L;
    // reflector from the first column of B (held by column group 0, tt = 0)
    const cpx<T> xr = csel(r < L, B.e[0], zero);
    const double nrm2 = (double)lane0(row_sum(c_abs2(xr)));
    const cpx<T> x0 = {lane0(B.e[0].re), lane0(B.e[0].im)};
    T tau;
    cpx<T> v0, alpha;
    make_reflector<T>(nrm2, x0, tau, v0, alpha);
    // every lane takes row r of B's first column (held by row group 0)
    const cpx<T> xsrc = {from_row0(B.e[0].re), from_row0(B.e[0].im)};
    const cpx<T> vr = csel(r == 0, v0, csel(r < L, xsrc, zero));
    cpx<T> vcol[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) vcol[tt] = shfl_c(vr, g + 4 * tt);  // v at this lane's columns
    // B <- H B
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const cpx<T> sc = sum16(c_cmul(vr, B.e[tt]));
        B.e[tt] = c_sub(B.e[tt], c_scale(tau, c_mul(vr, sc)));
    }
    // the annihilated column is exactly (alpha, 0, ..., 0)
    B.e[0] = csel(g == 0 && r < L, csel(r == 0, alpha, zero), B.e[0]);
    // D <- H D H
    cpx<T> pr = zero;
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
    // E <- E H (E is zero when there is no block below)
    {
        cpx<T> q = zero;
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
        const bool okb = r < L && c < S.Lprev, okd = r < L && c < L && r >= c;
        band[okb ? (int64_t)(S.col0 + c) * kBandLd + (S.lo + r - S.col0 - c) : discard] = B.e[tt];
        band[okd ? (int64_t)(S.lo + c) * kBandLd + (r - c) : discard] = D.e[tt];
    }
    if (S.L1 < 2) {  // nothing left to chase (a 1-row block needs no annihilation)
        if (S.L1 == 1) {
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                const int c = g + 4 * tt;
                if (r < 1 && c < L) band[(int64_t)(S.lo + c) * kBandLd + (S.lo1 + r - S.lo - c)] = E.e[tt];
            }
        }
        S.on = false;
        return;
    }
    // advance: the filled block below becomes the next B
    S.B = E;
    S.col0 = S.lo;
    S.Lprev = L;
    S.lo = S.lo1;
    S.hi = S.hi1;
    S.L = S.L1;
    S.lo1 = lo2;
    S.hi1 = hi2;
    S.L1 = L2;
    S.steps += 1;
}

// Two sweeps are in flight in one wavefront, the younger kChaseLag steps
// behind the older: step k of sweep j + 1 reads what steps <= k + 2 of sweep j
// wrote, and its blocks are loaded one step ahead, so a lag of 4 keeps every
// load after the stores it depends on in program order (the wavefront's
// memory operations reach the cache in order).  The two sweeps touch nearby
// columns, so the younger one mostly re-reads what the older one just wrote.
constexpr int kChaseLag = 4;

template <typename T>
__global__ __launch_bounds__(64) void chase_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                   const int32_t *__restrict__ n_in, double *__restrict__ dall,
                                                   double *__restrict__ eall, int64_t lde, cpx<T> *__restrict__ wall,
                                                   int64_t stride) {
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    double *d = dall + u * lde;
    double *e = eall + u * lde;
    const int lane = threadIdx.x;
    if (n < 0 || n > ld) {
        for (int64_t i = lane; i < lde; i += 64) d[i] = NAN;
        return;
    }
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *band = w.band;
    const cpx<T> *A = Hall + u * ld * ld;
    const int64_t discard = ld * kBandLd;
    for (int64_t q = lane; q < (int64_t)n * kBandLd; q += 64) {
        const int c = (int)(q / kBandLd), o = (int)(q % kBandLd);
        band[q] = (o <= kB && c + o < n) ? A[(c + o) + (int64_t)c * ld] : cpx<T>{T(0), T(0)};
    }
    __syncthreads();
    Sweep<T> S0, S1;
    S0.on = false;
    S1.on = false;
    S0.steps = S1.steps = 0;
    int next = 0;     // next sweep to start (sweeps j = 0 .. n - 3)
    int young = -1;   // slot of the most recently started sweep
    while (true) {
        // a sweep may start once the previous one is kChaseLag steps ahead or done
        if (!S0.on && next + 2 < n) {
            const bool ok = young < 0 || (young == 1 ? (!S1.on || S1.steps >= kChaseLag) : true);
            if (ok) {
                sweep_start(band, n, next++, S0);
                young = 0;
            }
        }
        if (!S1.on && next + 2 < n) {
            const bool ok = young < 0 || (young == 0 ? (!S0.on || S0.steps >= kChaseLag) : true);
            if (ok) {
                sweep_start(band, n, next++, S1);
                young = 1;
            }
        }
        if (!S0.on && !S1.on) break;
        if (S0.on) sweep_step(band, n, discard, S0);
        if (S1.on) sweep_step(band, n, discard, S1);
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
        d[i] = (double)band[(int64_t)i * kBandLd].re;
        if (i + 1 < n) e[i] = sqrt((double)c_abs2(band[(int64_t)i * kBandLd + 1]));
    }
}

template <typename T>
hipError_t launch_band_chase(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                             int64_t lde, cpx<T> *work, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int64_t stride = (int64_t)tridiag_twostage_work_elems<T>(ld);
    hipLaunchKernelGGL(chase_kernel<T>, dim3((unsigned)batch), dim3(64), 0, s, H, ld, n_in, d, e, lde, work, stride);
    return hipGetLastError();
}

template hipError_t launch_band_chase<double>(const cpx<double> *, int64_t, const int32_t *, int64_t, double *,
                                              double *, int64_t, cpx<double> *, hipStream_t);
template hipError_t launch_band_chase<float>(const cpx<float> *, int64_t, const int32_t *, int64_t, double *,
                                             double *, int64_t, cpx<float> *, hipStream_t);

}  // namespace mlmc
