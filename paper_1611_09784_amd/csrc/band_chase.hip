// Stage 2 of the two-stage Householder tridiagonalisation: band of
// half-width kB -> tridiagonal (d, e), by bulge chasing.  Sweep j annihilates
// column j below the sub-diagonal with a reflector on rows j+1..j+kB, applied
// two-sidedly to the kB x kB diagonal block and from the right to the block
// below, which fills it; the fill's first column is then annihilated by the
// next reflector, and so on down the band.  The fill left behind reaches
// 2kB - 1 sub-diagonals, so a column of the band holds 2kB entries.
//
// One workgroup of S wavefronts per matrix, one sweep per wavefront at a time.
// Each 16 x 16 block of a step lives in registers, 4 elements per lane: the
// diagonal block D and the block below it E with the row on the lane's low 4
// bits (products with v sum over a lane's own columns and the 4 lane groups),
// the block B that carries the column to annihilate transposed (so that v^H B
// also sums over a lane's own elements and the 4 lane groups, never across
// the 16 lanes of a group).  The band is staged through a ring of WC columns
// in LDS: S consecutive sweeps run down the matrix together, sweep j + 1 three
// steps behind sweep j (step k of sweep j + 1 needs steps <= k + 2 of sweep j,
// and the two footprints are then disjoint), one step per wavefront per phase
// with a workgroup barrier between phases.  Columns enter the ring from global
// memory two phases before the oldest sweep reaches them and leave it once
// the youngest sweep has finished them, so the band crosses HBM once per S
// sweeps instead of once per sweep.  When the rest of the band fits in the
// ring it stays there, and sweeps start as soon as their predecessor is far
// enough ahead and a wavefront is free.
#include "twostage_common.hpp"

namespace mlmc {

template <typename T>
struct Blk {  // 16 x 16 block: lane (r = lane & 15, g = lane >> 4) holds columns g + 4t
    cpx<T> e[4];
};

// ---------------------------------------------------------------------------
// The LDS ring: column c of the band sits in slot c % WC, sub-diagonal
// o = row - c at offset o (o < kWinDiag).  Extra regions: one element that
// is always zero (masked loads read it), one sink element per lane (masked
// stores write it), so that every access of a block is a single
// unconditional instruction, and 32 elements per wavefront through which a
// vector is re-laid out across lanes.
// ---------------------------------------------------------------------------
constexpr int kWinDiag = 2 * kB;

template <int WC>
struct Ring {
    static_assert((WC & (WC - 1)) == 0 && WC >= 16 * kB, "ring of a power-of-two number of columns");
    static constexpr int kZero = WC * kWinDiag;
    static constexpr int kSink = kZero + 1;
    static constexpr int kVec = kSink + 64;  // per wavefront: v (16 elements) and w (16)
    static constexpr int elems(int S) { return kVec + 32 * S; }
    static __device__ __forceinline__ int at(int row, int col) { return ((col & (WC - 1)) * kWinDiag) + (row - col); }
};

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// An index chosen by a select, hidden from the optimiser: a load from a
// selected address would otherwise become two loads and a branch.
__device__ __forceinline__ int opaque(int i) {
    asm volatile("" : "+v"(i));
    return i;
}
// A loaded value that is used only under a condition: keeps the load
// unconditional instead of sinking it into a branch that then waits for it.
template <typename T>
__device__ __forceinline__ T keep(T x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Barrier between phases: orders this workgroup's LDS traffic only, so that
// global loads and stores stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A[r0 + r, c0 + c] for r < nrow, c < ncol, zero elsewhere (FULL: the block
// is known to be whole, nrow = ncol = kB).
template <typename T, int WC, bool FULL>
__device__ __forceinline__ void ring_blk(const cpx<T> *win, int r0, int c0, int nrow, int ncol, Blk<T> &b) {
    const int lane = lane_id(), r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        const bool ok = FULL || (r < nrow && c < ncol);
        b.e[tt] = win[opaque(ok ? Ring<WC>::at(r0 + r, c0 + c) : Ring<WC>::kZero)];
    }
}

// Transposed: lane (c = lane & 15, g = lane >> 4) holds A[r0 + g + 4t, c0 + c].
template <typename T, int WC, bool FULL>
__device__ __forceinline__ void ring_blk_t(const cpx<T> *win, int r0, int c0, int nrow, int ncol, Blk<T> &b) {
    const int lane = lane_id(), c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int r = g + 4 * tt;
        const bool ok = FULL || (r < nrow && c < ncol);
        b.e[tt] = win[opaque(ok ? Ring<WC>::at(r0 + r, c0 + c) : Ring<WC>::kZero)];
    }
}

// The Hermitian diagonal block A[r0.., r0..] of size L from its stored lower
// triangle: lanes above the diagonal take the conjugate of their mirror.
template <typename T, int WC, bool FULL>
__device__ __forceinline__ void ring_diag(const cpx<T> *win, int r0, int L, Blk<T> &b) {
    const int lane = lane_id(), r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int c = g + 4 * tt;
        const int hi = r > c ? r : c, lo = r > c ? c : r;
        const bool ok = FULL || (r < L && c < L);
        const cpx<T> x = win[opaque(ok ? Ring<WC>::at(r0 + hi, r0 + lo) : Ring<WC>::kZero)];
        const T f = (r == c) ? T(0) : ((r < c) ? T(-1) : T(1));  // lane constant: conjugate above, real diagonal
        b.e[tt] = {x.re, f * x.im};
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

// Complex multiply-adds as two fused multiply-adds per real component.
template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmat<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
template <typename T>  // acc + a b
__device__ __forceinline__ cpx<T> cfma(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fmat(a.re, b.re, fmat(-a.im, b.im, acc.re)), fmat(a.re, b.im, fmat(a.im, b.re, acc.im))};
}
template <typename T>  // acc + conj(a) b
__device__ __forceinline__ cpx<T> cfma_ca(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fmat(a.re, b.re, fmat(a.im, b.im, acc.re)), fmat(a.re, b.im, fmat(-a.im, b.re, acc.im))};
}
template <typename T>  // acc - a b
__device__ __forceinline__ cpx<T> cfms(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fmat(-a.re, b.re, fmat(a.im, b.im, acc.re)), fmat(-a.re, b.im, fmat(-a.im, b.re, acc.im))};
}
template <typename T>  // acc - a conj(b)
__device__ __forceinline__ cpx<T> cfms_cb(cpx<T> acc, cpx<T> a, cpx<T> b) {
    return {fmat(-a.re, b.re, fmat(-a.im, b.im, acc.re)), fmat(-a.im, b.re, fmat(a.re, b.im, acc.im))};
}

// One reflection: the reflector H = I - tau v v^H taking the first column of
// B (rows 0..L-1) to (alpha, 0, ..., 0) is applied as B <- H B (B transposed
// across lanes), D <- H D H and E <- E H.  vb indexes this wavefront's 32
// scratch elements in the ring array, sink its lane's sink element.  Every
// update is written as fused multiply-adds (two per real component of a
// complex multiply-add).
template <typename T>
__device__ __forceinline__ void chase_reflect(cpx<T> *win, int vb, int sink, int L, Blk<T> &B, Blk<T> &D,
                                              Blk<T> &E) {
    const int lane = lane_id(), r = lane & 15, g = lane >> 4;
    const cpx<T> zero = {T(0), T(0)};
    // B's first column: lanes r == 0 (column 0), rows g + 4t; rows >= L of
    // B were loaded as zero and stay zero
    T s = T(0);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) s = fmat(B.e[tt].re, B.e[tt].re, fmat(B.e[tt].im, B.e[tt].im, s));
    const double nrm2 = (double)lane0(col_sum(s));
    const cpx<T> x0 = {lane0(B.e[0].re), lane0(B.e[0].im)};
    T tau;
    cpx<T> v0, alpha;
    make_reflector<T>(nrm2, x0, tau, v0, alpha);
    // v (v0, then the first column below it) through LDS, whose operations a
    // wavefront completes in order: by row (vr: row r) and by column
    // (vcol[t]: column g + 4t)
#pragma unroll
    for (int tt = 0; tt < 4; ++tt)
        win[opaque(r == 0 ? vb + g + 4 * tt : sink)] = (tt == 0) ? csel(g == 0, v0, B.e[0]) : B.e[tt];
    const cpx<T> vr = win[vb + r];
    cpx<T> vcol[4];
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) vcol[tt] = win[vb + g + 4 * tt];
    // B <- H B: sc[c] = sum_i conj(v_i) B[i][c]; lane (c = r, g) holds rows g + 4t
    cpx<T> sc = zero;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) sc = cfma_ca(sc, vcol[tt], B.e[tt]);
    sc = c_scale(tau, sum4g(sc));
    // The annihilated column (lanes r == 0) becomes exactly (alpha, 0, ..., 0):
    // its lanes keep m = 0 of the old value and add alpha where it belongs.
    const T m = r == 0 ? T(0) : T(1);
    const T ma = (r == 0 && g == 0) ? T(1) : T(0);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const cpx<T> x = cfms(B.e[tt], vcol[tt], sc);
        if (tt == 0)
            B.e[0] = {fmat(m, x.re, ma * alpha.re), fmat(m, x.im, ma * alpha.im)};
        else
            B.e[tt] = {m * x.re, m * x.im};
    }
    // D <- H D H
    cpx<T> pr = zero;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) pr = cfma(pr, D.e[tt], vcol[tt]);
    pr = c_scale(tau, sum4g(pr));
    const cpx<T> vhp = sum16(cfma_ca(zero, vr, pr));
    const T K = (T)0.5 * tau * vhp.re;
    const cpx<T> wr = {fmat(-K, vr.re, pr.re), fmat(-K, vr.im, pr.im)};
    win[opaque(g == 0 ? vb + 16 + r : sink)] = wr;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const cpx<T> wc = win[vb + 16 + g + 4 * tt];
        D.e[tt] = cfms_cb(cfms_cb(D.e[tt], vr, wc), wr, vcol[tt]);
    }
    // E <- E H (E is zero when there is no block below): E - (tau q) v^H
    cpx<T> q = zero;
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) q = cfma(q, E.e[tt], vcol[tt]);
    q = c_scale(tau, sum4g(q));
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) E.e[tt] = cfms_cb(E.e[tt], q, vcol[tt]);
}

// Number of steps of sweep j: step k works on rows j + 1 + kB k ..; the sweep
// ends at the first step whose block below has fewer than two rows.
__device__ __forceinline__ int sweep_steps(int n, int j) {
    const int x = n - j - kB - 3;
    return x < 0 ? 1 : x / kB + 2;
}

// State of one sweep between steps: rows lo..hi carry the next reflector,
// lo1..hi1 the block below; the block B to reflect (rows lo..hi, columns
// col0..col0+Lprev-1) is in the ring: column j itself at the first step, the
// block written back as E by the previous step after that.
struct Sweep {
    int lo, hi, L, lo1, hi1, L1, col0, Lprev;
};

__device__ __forceinline__ void sweep_begin(int n, int j, Sweep &S) {
    S.lo = j + 1;
    S.hi = min(j + kB, n - 1);
    S.L = S.hi - S.lo + 1;
    S.lo1 = S.hi + 1;
    S.hi1 = min(S.hi + kB, n - 1);
    S.L1 = S.hi1 - S.lo1 + 1;
    S.col0 = j;
    S.Lprev = 1;
}

// One step: load B (transposed), the diagonal block D and the block below E,
// reflect, store B (final for this sweep), the lower triangle of D and E
// (the next step's B).  Returns true when the sweep has ended.  FULL: an
// interior step, all three blocks whole (L = L1 = Lprev = kB), no masks.
template <typename T, int WC, bool FULL>
__device__ __forceinline__ bool sweep_step(cpx<T> *win, int vb, int n, Sweep &S) {
    const int lane = lane_id(), r = lane & 15, g = lane >> 4;
    const int sink = Ring<WC>::kSink + lane;
    const int L = FULL ? kB : S.L, L1 = FULL ? kB : S.L1, Lprev = FULL ? kB : S.Lprev;
    Blk<T> B, D, E;
    ring_blk_t<T, WC, FULL>(win, S.lo, S.col0, L, Lprev, B);
    ring_diag<T, WC, FULL>(win, S.lo, L, D);
    ring_blk<T, WC, FULL>(win, S.lo1, S.lo, L1, L, E);
    chase_reflect<T>(win, vb, sink, L, B, D, E);
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        const int i = g + 4 * tt;  // row of B held at tt; column of D and E held at tt
        const bool okb = FULL || (i < L && r < Lprev), okd = (FULL || (r < L && i < L)) && r >= i,
                   oke = FULL || (r < L1 && i < L);
        win[opaque(okb ? Ring<WC>::at(S.lo + i, S.col0 + r) : sink)] = B.e[tt];
        win[opaque(okd ? Ring<WC>::at(S.lo + r, S.lo + i) : sink)] = D.e[tt];
        win[opaque(oke ? Ring<WC>::at(S.lo1 + r, S.lo + i) : sink)] = E.e[tt];
    }
    if (!FULL && S.L1 < 2) return true;  // nothing left to chase (a 1-row block needs no annihilation)
    S.col0 = S.lo;
    S.Lprev = L;
    S.lo = S.lo1;
    S.hi = S.hi1;
    S.L = S.L1;
    S.lo1 = S.hi1 + 1;
    S.hi1 = min(S.hi1 + kB, n - 1);
    S.L1 = S.hi1 - S.lo1 + 1;
    return false;
}

template <typename T, int WC>
__device__ __forceinline__ bool sweep_advance(cpx<T> *win, int vb, int n, Sweep &S) {
    if (S.L == kB && S.L1 == kB && S.Lprev == kB) return sweep_step<T, WC, true>(win, vb, n, S);
    return sweep_step<T, WC, false>(win, vb, n, S);
}

// ---------------------------------------------------------------------------
// Column traffic between the ring and global memory, 16 columns (2kB
// sub-diagonals each) at a time over the NT threads of the workgroup:
// element q of a chunk is column cb + q / 2kB, sub-diagonal q % 2kB.  The
// source is either the matrix itself (column stride ld + 1 from the diagonal,
// kB sub-diagonals valid) or the band array (column stride kBandLd).
// ---------------------------------------------------------------------------
template <int NT>
struct Chunk {
    static constexpr int kPer = 16 * kWinDiag / NT;
    static_assert(kPer * NT == 16 * kWinDiag, "chunk spread evenly over the workgroup");
};

template <typename T>
struct ColSource {
    const cpx<T> *base;
    int64_t cstride;
    int omax;
};

template <typename T, int NT>
__device__ __forceinline__ void chunk_fetch(const ColSource<T> &src, int n, int cb, int ce,
                                            cpx<T> (&x)[Chunk<NT>::kPer]) {
#pragma unroll
    for (int q = 0; q < Chunk<NT>::kPer; ++q) {
        const int idx = (int)threadIdx.x + NT * q, c = cb + idx / kWinDiag, o = idx % kWinDiag;
        const bool ok = c < ce && o <= src.omax && c + o < n;
        x[q] = src.base[opaque(ok ? (int)((int64_t)c * src.cstride + o) : 0)];
    }
}

template <typename T, int NT, int WC>
__device__ __forceinline__ void chunk_put(cpx<T> *win, const ColSource<T> &src, int n, int cb, int ce,
                                          const cpx<T> (&x)[Chunk<NT>::kPer]) {
    const cpx<T> zero = {T(0), T(0)};
#pragma unroll
    for (int q = 0; q < Chunk<NT>::kPer; ++q) {
        const int idx = (int)threadIdx.x + NT * q, c = cb + idx / kWinDiag, o = idx % kWinDiag;
        const bool in = c < ce, ok = in && o <= src.omax && c + o < n;
        win[in ? Ring<WC>::at(c + o, c) : Ring<WC>::kSink + lane_id()] = csel(ok, x[q], zero);
    }
}

// Columns cb..ce-1 (at most 16) from the ring to the band array; lanes past
// ce store to the band array's discard column.
template <typename T, int NT, int WC>
__device__ __forceinline__ void chunk_writeback(const cpx<T> *win, cpx<T> *band, int64_t sink, int cb, int ce) {
#pragma unroll
    for (int q = 0; q < Chunk<NT>::kPer; ++q) {
        const int idx = (int)threadIdx.x + NT * q, c = cb + idx / kWinDiag, o = idx % kWinDiag;
        const bool in = c < ce;
        const cpx<T> x = win[opaque(in ? Ring<WC>::at(c + o, c) : Ring<WC>::kZero)];
        band[in ? (int64_t)c * kBandLd + o : sink] = x;
    }
}

template <typename T, int NT, int WC>
__device__ __forceinline__ void ring_to_global(cpx<T> *win, const ColSource<T> &src, int n, int cb, int ce) {
    for (; cb < ce; cb += 16) {
        cpx<T> x[Chunk<NT>::kPer];
        chunk_fetch<T, NT>(src, n, cb, min(cb + 16, ce), x);
        chunk_put<T, NT, WC>(win, src, n, cb, min(cb + 16, ce), x);
    }
}

// Tridiagonal entries of columns c0..c1-1: d = A[c, c], e = |A[c + 1, c]|.
template <typename T, int NT, int WC>
__device__ __forceinline__ void extract_de(const cpx<T> *win, int n, int c0, int c1, double *d, double *e) {
    for (int c = c0 + (int)threadIdx.x; c < c1; c += NT) {
        d[c] = (double)win[Ring<WC>::at(c, c)].re;
        if (c + 1 < n) e[c] = sqrt((double)c_abs2(win[Ring<WC>::at(c + 1, c)]));
    }
}

// Columns the oldest sweep of a batch (j0) touches up to and including
// phase t: < need(t).
__device__ __forceinline__ int batch_need(int n, int j0, int t) { return min(n, j0 + kB + 1 + kB * t); }

// Phase t of a batch of S sweeps j0..j0+S-1 (wavefront w runs sweep j0 + w,
// step t - 3w):
//   1. columns that the youngest sweep finished by phase t - 1 go back to the
//      band array (at most 16 per phase, which keeps up with the sweep);
//   2. after every sweep of the batch has made its first step, the batch's
//      own columns are final: their tridiagonal entries are written out;
//   3. the columns first needed in phase t + 2 are fetched into registers;
//   4. this wavefront's step;
//   5. the columns fetched in phase t - 1 go into the ring.
template <typename T, int S, int WC>
__device__ __forceinline__ void batch_phase(cpx<T> *win, cpx<T> *band, int64_t gsink, const ColSource<T> &src, int n,
                                            int j0, int t, int wid, int Kw, int Ky, int &wb_lo, Sweep &sw,
                                            double *d, double *e, cpx<T> (&fetch)[Chunk<64 * S>::kPer],
                                            const cpx<T> (&put)[Chunk<64 * S>::kPer]) {
    constexpr int NT = 64 * S;
    const int ky = t - 1 - 3 * (S - 1);
    const int fin = ky < 0 ? wb_lo : (ky >= Ky - 1 ? n : j0 + S + kB * ky);
    const int wb_hi = max(wb_lo, min(wb_lo + 16, fin));
    chunk_writeback<T, NT, WC>(win, band, gsink, wb_lo, wb_hi);
    wb_lo = wb_hi;
    if (t == 3 * (S - 1) + 1) extract_de<T, NT, WC>(win, n, j0, j0 + S, d, e);
    chunk_fetch<T, NT>(src, n, batch_need(n, j0, t + 1), batch_need(n, j0, t + 2), fetch);
    const int k = t - 3 * wid;
    if (k >= 0 && k < Kw) {
        if (k == 0) sweep_begin(n, j0 + wid, sw);
        sweep_advance<T, WC>(win, Ring<WC>::kVec + 32 * wid, n, sw);
    }
    const int pb = batch_need(n, j0, t);
    chunk_put<T, NT, WC>(win, src, n, pb, t >= 1 ? batch_need(n, j0, t + 1) : pb, put);
    lds_barrier();
}

// The whole chase of matrix u by one workgroup (ring and schedule in LDS).
template <typename T, int S, int WC>
__device__ __forceinline__ void chase_matrix(int64_t u, cpx<T> *win, int *sched, const cpx<T> *__restrict__ Hall,
                                             int64_t ld, const int64_t *__restrict__ offs,
                                             const int32_t *__restrict__ n_in, double *__restrict__ dall,
                                             double *__restrict__ eall, int64_t lde, cpx<T> *__restrict__ wall,
                                             int64_t stride) {
    constexpr int NT = 64 * S;
    constexpr int kPer = Chunk<NT>::kPer;
    const int n = n_in[u];
    double *d = dall + u * lde;
    double *e = eall + u * lde;
    if (n < 0 || n > ld) {
        for (int64_t i = threadIdx.x; i < lde; i += NT) d[i] = NAN;
        return;
    }
    const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const TwoView<T> w(wall, stride, ld, u);
    cpx<T> *band = w.band;
    const int64_t gsink = ld * kBandLd;
    const ColSource<T> from_h = {Hall + mat_offset(offs, u, ld), ld + 1, kB};
    const ColSource<T> from_band = {band, kBandLd, kWinDiag - 1};
    if (threadIdx.x == 0) win[Ring<WC>::kZero] = {T(0), T(0)};
    const int nsw = max(n - 2, 0);  // sweeps j = 0 .. n - 3
    Sweep sw;
    int j0 = 0;
    for (; j0 < nsw && n - j0 > WC; j0 += S) {
        const ColSource<T> src = j0 == 0 ? from_h : from_band;
        ring_to_global<T, NT, WC>(win, src, n, j0, batch_need(n, j0, 1));
        lds_barrier();
        // Phases of the batch, rounded up to even (the loop runs phases in
        // pairs, swapping the two fetch buffers; a last idle phase is harmless).
        int T_b = 0;
#pragma unroll
        for (int i = 0; i < S; ++i) T_b = max(T_b, 3 * i + sweep_steps(n, j0 + i));
        T_b += T_b & 1;
        const int Kw = sweep_steps(n, j0 + wid), Ky = sweep_steps(n, j0 + S - 1);
        int wb_lo = j0 + S;
        cpx<T> ra[kPer], rb[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) ra[q] = rb[q] = {T(0), T(0)};
        for (int t = 0; t < T_b; t += 2) {
            batch_phase<T, S, WC>(win, band, gsink, src, n, j0, t, wid, Kw, Ky, wb_lo, sw, d, e, ra, rb);
            batch_phase<T, S, WC>(win, band, gsink, src, n, j0, t + 1, wid, Kw, Ky, wb_lo, sw, d, e, rb, ra);
        }
        for (int cb = wb_lo; cb < n; cb += 16) chunk_writeback<T, NT, WC>(win, band, gsink, cb, min(cb + 16, n));
        if (T_b <= 3 * (S - 1) + 1) extract_de<T, NT, WC>(win, n, j0, j0 + S, d, e);
        // The band array is complete (and no stale copy of it is cached)
        // before the next batch reads it.
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // The rest of the band fits in the ring: load it once and run the
    // remaining sweeps without global traffic.  Sweep j starts once sweep
    // j - 1 has made min(3, its step count) steps and its wavefront
    // ((j - j0) % S) has finished sweep j - S.
    ring_to_global<T, NT, WC>(win, j0 == 0 ? from_h : from_band, n, j0, n);
    if (threadIdx.x == 0) {
        int last = 0, Klast = 0, Tr = 0;
        for (int i = 0; i < S; ++i) sched[WC + i] = 0;
        for (int j = j0; j < nsw; ++j) {
            const int ws = (j - j0) % S, K = sweep_steps(n, j);
            const int P = (j == j0) ? 0 : max(last + min(3, Klast), sched[WC + ws]);
            sched[j - j0] = P;
            sched[WC + ws] = P + K;
            Tr = max(Tr, P + K);
            last = P;
            Klast = K;
        }
        sched[WC + S] = Tr;
    }
    lds_barrier();
    const int Tr = __builtin_amdgcn_readfirstlane(sched[WC + S]);
    int jw = j0 + wid;
    for (int t = 0; t < Tr; ++t) {
        if (jw < nsw) {
            const int P = __builtin_amdgcn_readfirstlane(sched[jw - j0]);
            if (t >= P) {
                if (t == P) sweep_begin(n, jw, sw);
                if (sweep_advance<T, WC>(win, Ring<WC>::kVec + 32 * wid, n, sw)) jw += S;
            }
        }
        lds_barrier();
    }
    extract_de<T, NT, WC>(win, n, j0, n, d, e);
}

// One workgroup per CU at most (the ring fills most of its LDS); workgroup b
// chases matrices b, b + gridDim.x, ... so that a grid smaller than the batch
// leaves the other CUs to other work.
template <typename T, int S, int WC>
__global__ __launch_bounds__(64 * S) void chase_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                       const int64_t *__restrict__ offs,
                                                       const int32_t *__restrict__ n_in, int64_t batch,
                                                       double *__restrict__ dall, double *__restrict__ eall,
                                                       int64_t lde, cpx<T> *__restrict__ wall, int64_t stride) {
    __shared__ cpx<T> win[Ring<WC>::elems(S)];
    __shared__ int sched[WC + S + 1];  // resident phase: start phase per sweep, end phase per wavefront, length
    for (int64_t u = blockIdx.x; u < batch; u += gridDim.x) {
        chase_matrix<T, S, WC>(u, win, sched, Hall, ld, offs, n_in, dall, eall, lde, wall, stride);
        __syncthreads();  // every wavefront is done with the ring before the next matrix refills it
    }
}

// FP64: 4 sweeps in a ring of 256 columns (128 KiB of LDS, one workgroup per
// CU); FP32: 8 sweeps in 512 columns (128 KiB), so that bands of up to 512
// columns never leave the ring.
template <typename T>
struct ChaseShape;
template <>
struct ChaseShape<double> {
    static constexpr int S = 4, WC = 256;
};
template <>
struct ChaseShape<float> {
    static constexpr int S = 8, WC = 512;
};

template <typename T>
hipError_t launch_band_chase(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                             int64_t lde, cpx<T> *work, hipStream_t s, int64_t max_blocks, int64_t stride,
                             const int64_t *offs) {
    if (batch == 0) return hipSuccess;
    if (ld > 46340) return hipErrorInvalidValue;  // element offsets into H are 32-bit
    constexpr int S = ChaseShape<T>::S, WC = ChaseShape<T>::WC;
    if (stride == 0) stride = (int64_t)tridiag_twostage_work_elems<T>(ld);
    if (stride < (int64_t)tridiag_twostage_work_elems<T>(ld)) return hipErrorInvalidValue;
    const int64_t grid = (max_blocks > 0 && max_blocks < batch) ? max_blocks : batch;
    hipLaunchKernelGGL((chase_kernel<T, S, WC>), dim3((unsigned)grid), dim3(64 * S), 0, s, H, ld, offs, n_in, batch, d,
                       e, lde, work, stride);
    return hipGetLastError();
}

template hipError_t launch_band_chase<double>(const cpx<double> *, int64_t, const int32_t *, int64_t, double *,
                                              double *, int64_t, cpx<double> *, hipStream_t, int64_t, int64_t,
                                              const int64_t *);
template hipError_t launch_band_chase<float>(const cpx<float> *, int64_t, const int32_t *, int64_t, double *,
                                             double *, int64_t, cpx<float> *, hipStream_t, int64_t, int64_t,
                                             const int64_t *);

}  // namespace mlmc
