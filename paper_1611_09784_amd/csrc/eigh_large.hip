// Eigenvectors of matrices above the LDS-resident size (complex128 or
// complex64 storage, computed in double).  After stage 1 (dense -> band of
// half-width kB, each panel's block reflector kept) and the eigenvalues
// (chase + bisection), the eigenvectors are
//   band_ii_kernel   inverse iteration on the band matrix B, one wavefront
//                    per eigenvalue: pivoted band LU of B - lam I, two
//                    solves from a hashed start vector
//   cluster_orth_kernel  the vectors of each cluster of close eigenvalues
//                    orthonormalised, their Rayleigh quotients, sorted
//   group_t_kernel, group_bt_kernel  X <- (I - V T V^H) X for groups of four
//                    panels from last to first, which takes B's eigenvectors
//                    to H's
// The chase's rotations are not needed: B's own eigenvectors are computed.
#include <cfloat>

#include "eigh_large.hpp"

namespace mlmc {

namespace {

constexpr int kWR = kB + 1;          // rows of the elimination window
constexpr int kWC = 2 * kB + 1;      // its columns (U has 2 kB superdiagonals after pivoting)
constexpr int kSt = kIIStep;         // steps per staged block
constexpr int kRowPer = (kSt * kWC + 63) / 64;
constexpr int kLPer = (kSt * kB + 63) / 64;
// Solves per eigenvalue: the shift is within the bisection's 1e-12 of the
// eigenvalue, so each solve shrinks the other eigenvectors' share by their
// distance over 1e-12 (the members of a cluster mix, and are orthogonalised).
constexpr int kIISolves = 2;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Whole-entry loads and stores of a complex value (one 16-byte access, no
// struct copy through the stack).
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cpx<double> ld2(const cpx<double> *p) {
    const d2v v = *reinterpret_cast<const d2v *>(p);
    return {v.x, v.y};
}
__device__ __forceinline__ void st2(cpx<double> *p, cpx<double> x) { *reinterpret_cast<d2v *>(p) = d2v{x.re, x.im}; }
// An entry of the matrices or of the reflector store, complex128 or complex64,
// widened to complex128 (the banded path computes in double either way).
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cpx<double> ldc(const cpx<double> *p) { return ld2(p); }
__device__ __forceinline__ cpx<double> ldc(const cpx<float> *p) {
    const f2v v = *reinterpret_cast<const f2v *>(p);
    return {(double)v.x, (double)v.y};
}

// Orders this wavefront's LDS traffic (the workgroup is one wavefront; its
// LDS operations complete in order, so only the compiler is held back).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// Makes this wavefront's global stores visible to its later global loads.
__device__ __forceinline__ void wave_global_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// Deterministic start vector entry in (-1, 1) for (eigenvalue k, row r, part).
__device__ __forceinline__ double start_value(int k, int r, int part) {
    uint32_t h = (uint32_t)k * 0x9E3779B1u ^ ((uint32_t)(2 * r + part) + 0x7F4A7C15u) * 0x85EBCA6Bu;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return ((double)h + 0.5) * (2.0 / 4294967296.0) - 1.0;
}

// LU factors of B - lam I in a wavefront's scratch slice, row by row in the
// order the elimination produces them (blocks of kSt steps, so the slice has
// room for ld + kSt steps):
//   U[k kWC + j] = U(k, k + j) for 1 <= j <= 2 kB, U[k kWC] = 1 / U(k, k)
//   L[k kB + i]  = multiplier of row k + 1 + i at elimination step k
//   piv[k]       = the row swapped with row k at step k
//   y[r]         = the iterated vector
struct IIFactors {
    cpx<double> *U, *L, *y;
    int *piv;
    __device__ IIFactors(char *base, int64_t ld) {
        U = reinterpret_cast<cpx<double> *>(base);
        L = U + (ld + kSt) * kWC;
        y = L + (ld + kSt) * kB;
        piv = reinterpret_cast<int *>(y + ld);
    }
};

// LDS of a wavefront: the elimination window, kSt steps of incoming band rows
// (or of U's columns in the backward solve), of outgoing U rows and
// multipliers (or of the forward solve's multipliers), the pivots, and a ring
// of kIIYRing entries of the iterated vector around the solves' current row.
constexpr int kYR = kIIYRing;
struct IILds {
    cpx<double> *win, *rows, *outU, *outL, *yr;
    int *outP;
    __device__ IILds(unsigned char *base) {
        win = reinterpret_cast<cpx<double> *>(base);
        rows = win + kWR * kWC;
        outU = rows + kSt * kWC;
        outL = outU + kSt * kWC;
        yr = outL + kSt * kB;
        outP = reinterpret_cast<int *>(yr + kYR);
    }
};

// Offset of row slot r in the window (a 24-bit multiply: slots are small).
__device__ __forceinline__ int wrow(int r) { return (int)__umul24((unsigned)r, (unsigned)kWC); }

// The elimination window is a ring: at step k it holds row positions
// k .. k + kB (position r in slot r mod (kB + 1), holding what an explicit
// row interchange would have put there) and columns k .. k + 2 kB (column c
// in slot c mod (2 kB + 1)).

// B[r][c] - lam delta_rc of the band matrix of half-width kB whose lower
// triangle stage 1 left in H (column-major, ld); zero outside the band and
// outside the n x n matrix (n >= 1); the diagonal is taken real.  The load is
// unconditional (from H[0] for an entry outside), so that a block of such
// loads stays in flight together.
template <typename T>
__device__ __forceinline__ cpx<double> band_ld(const cpx<T> *H, int64_t ld, int n, int r, int c, double lam) {
    const int d = r - c;
    const bool in = r >= 0 && c >= 0 && r < n && c < n && d <= kB && d >= -kB;
    const bool up = d < 0;
    const int64_t at = in ? (up ? (int64_t)c + (int64_t)r * ld : (int64_t)r + (int64_t)c * ld) : 0;
    const cpx<double> x = ldc(H + at);
    // factors instead of selects, so that both halves are always used
    const double keep = in ? 1.0 : 0.0, sgn = d == 0 ? 0.0 : (up ? -keep : keep);
    return {(x.re - (d == 0 ? lam : 0.0)) * keep, x.im * sgn};
}

// Band rows k0 + kWR + i, columns k0 + i + 1 .. k0 + i + 2 kB + 1 (i < kSt):
// what the steps k0 .. k0 + kSt - 1 slide into the window.
template <typename T>
__device__ __forceinline__ void fetch_rows(const cpx<T> *H, int64_t ld, int n, double lam, int k0,
                                           cpx<double> (&pre)[kRowPer]) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kRowPer; ++q) {
        const int idx = min(lane + 64 * q, kSt * kWC - 1), i = idx / kWC, j = idx % kWC;
        pre[q] = band_ld(H, ld, n, k0 + kWR + i, k0 + i + 1 + j, lam);
    }
}

// The largest key over lanes 0..31 (DPP within the two 16-lane rows).
__device__ __forceinline__ int max_key32(int key) {
    key = max(key, dpp_word<kDppXor1>(key));
    key = max(key, dpp_word<kDppXor2>(key));
    key = max(key, dpp_word<kDppHalfMirror>(key));
    key = max(key, dpp_word<kDppMirror>(key));
    return max(__builtin_amdgcn_readlane(key, 0), __builtin_amdgcn_readlane(key, 16));
}

// Block kb's factors (staged in LDS) to the scratch slice.
__device__ __forceinline__ void flush_factors(const IILds &sm, const IIFactors &f, int kb) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kRowPer; ++q) {
        const int idx = lane + 64 * q;
        if (idx < kSt * kWC) st2(f.U + (int64_t)kb * kWC + idx, ld2(sm.outU + idx));
    }
#pragma unroll
    for (int q = 0; q < kLPer; ++q) st2(f.L + (int64_t)kb * kB + lane + 64 * q, ld2(sm.outL + lane + 64 * q));
    if (lane < kSt) f.piv[kb + lane] = sm.outP[lane];
}

// Pivoted LU of B - lam I (kB sub- and superdiagonals) by one wavefront.
// Step k takes the largest entry of column k in rows k .. k + kB as the pivot
// (its magnitude compared in single precision; equals go to the upper row),
// records U's row k and the multipliers, eliminates, and slides the window
// down and right by one.  The swap of rows k and p is implicit: row k's slot
// leaves the window, and p's slot takes row k's eliminated entries.  A step
// reads everything that does not depend on the pivot at once, then the pivot
// row, and touches LDS only: the band rows it slides in are fetched a block
// ahead, and its factors go out a block behind.
template <typename T>
__device__ __forceinline__ void band_lu(const cpx<T> *H, int64_t ld, int n, double lam, double tiny, const IILds &sm,
                                        const IIFactors &f) {
    static_assert(kSt * kB == 64 * kLPer, "whole multiplier blocks");
    const int lane = lane_id();
    const int cc = 1 + (lane & 31), rh = lane >> 5;  // this lane: column k + cc, rows k + 1 + rh + 2q
    for (int idx = lane; idx < kWR * kWC; idx += 64) {
        const int r = idx / kWC, c = idx % kWC;
        st2(sm.win + r * kWC + c, band_ld(H, ld, n, r, c, lam));
    }
    cpx<double> pre[kRowPer];
    fetch_rows(H, ld, n, lam, 0, pre);
    int ks = 0, kc = 0;  // window slots of row k and column k
    for (int k0 = 0; k0 < n; k0 += kSt) {
        wave_lds_sync();
        if (k0 > 0) flush_factors(sm, f, k0 - kSt);
#pragma unroll
        for (int q = 0; q < kRowPer; ++q)
            if (lane + 64 * q < kSt * kWC) st2(sm.rows + lane + 64 * q, pre[q]);
        fetch_rows(H, ld, n, lam, k0 + kSt, pre);  // in flight during this block
        wave_lds_sync();
        const int k1 = min(k0 + kSt, n);
        for (int k = k0; k < k1; ++k) {
            const int i = k - k0;
            // the pivot search's candidates are read first, so that it waits for them only
            const int ksl = ks + lane >= kWR ? ks + lane - kWR : ks + lane;
            const cpx<double> cand = ld2(sm.win + wrow(lane < kWR ? ksl : ks) + kc);
            const int csl = kc + cc >= kWC ? kc + cc - kWC : kc + cc;
            cpx<double> colk[kB / 2], xr[kB / 2];
            int rsl[kB / 2];
#pragma unroll
            for (int q = 0; q < kB / 2; ++q) {
                const int rr = 1 + rh + 2 * q;
                rsl[q] = wrow(ks + rr >= kWR ? ks + rr - kWR : ks + rr);
                colk[q] = ld2(sm.win + rsl[q] + kc);
                xr[q] = ld2(sm.win + rsl[q] + csl);
            }
            const cpx<double> rowk = ld2(sm.win + wrow(ks) + csl), dkk = ld2(sm.win + wrow(ks) + kc);
            const cpx<double> inrow = ld2(sm.rows + i * kWC + (lane < kWC ? lane : 0));
            const int ml = lane & (kB - 1);  // lane < kB: the multiplier of row k + 1 + ml
            const int mls = ks + 1 + ml >= kWR ? ks + 1 + ml - kWR : ks + 1 + ml;
            const cpx<double> colm = ld2(sm.win + wrow(mls) + kc);
            const int key = lane < kWR && k + lane < n
                                ? (int)((__float_as_uint((float)c_abs2(cand)) & ~31u) | (uint32_t)(31 - lane))
                                : 0;
            const int pr = 31 - (max_key32(key) & 31);  // the pivot row is k + pr
            const int psl = wrow(ks + pr >= kWR ? ks + pr - kWR : ks + pr);
            cpx<double> piv = ld2(sm.win + psl + kc);
            const cpx<double> rowp = ld2(sm.win + psl + csl);
            double a2 = c_abs2(piv);
            if (!(a2 >= tiny * tiny)) {  // singular to working precision: lam is an eigenvalue
                piv = {tiny, 0.0};
                a2 = tiny * tiny;
            }
            const double ia2 = 1.0 / a2;
            const cpx<double> rp = {piv.re * ia2, -piv.im * ia2};
            // rows k + 1 .. k + kB -= l * (pivot row) over columns k + 1 .. k + 2 kB; the
            // row in p's slot stands for row k from here on, so its entries are
            // rewritten from row k's after the loop (the loop leaves zeros there)
#pragma unroll
            for (int q = 0; q < kB / 2; ++q) {
                const cpx<double> l = c_mul(colk[q], rp);
                st2(sm.win + rsl[q] + csl, c_sub(xr[q], c_mul(l, rowp)));
            }
            const cpx<double> lk = c_mul(dkk, rp);
            if (pr > 0 && rh == ((pr - 1) & 1)) st2(sm.win + psl + csl, c_sub(rowk, c_mul(lk, rowp)));
            if (lane < kB) st2(sm.outL + i * kB + ml, c_mul(csel(ml + 1 == pr, dkk, colm), rp));
            if (lane < 2 * kB) st2(sm.outU + i * kWC + 1 + lane, rowp);
            if (lane == 0) {
                st2(sm.outU + i * kWC, rp);
                sm.outP[i] = k + pr;
            }
            // row k's slot takes row k + kB + 1 (columns k + 1 .. k + 2 kB + 1); column
            // k's slot becomes column k + 2 kB + 1, zero in rows k + 1 .. k + kB
            if (lane < kWC) {
                const int c = kc + 1 + lane;
                st2(sm.win + wrow(ks) + (c >= kWC ? c - kWC : c), inrow);
            }
            if (lane < kB) {
                const int sl = ks + 1 + lane;
                st2(sm.win + wrow(sl >= kWR ? sl - kWR : sl) + kc, cpx<double>{0.0, 0.0});
            }
            ks = ks + 1 == kWR ? 0 : ks + 1;
            kc = kc + 1 == kWC ? 0 : kc + 1;
            __builtin_amdgcn_wave_barrier();  // the wavefront's LDS operations complete in order
        }
    }
    wave_lds_sync();
    flush_factors(sm, f, (n - 1) / kSt * kSt);
    wave_lds_sync();
    wave_global_sync();
}

// Multipliers and pivots of steps k0 .. k0 + kSt - 1.
__device__ __forceinline__ void fetch_l(const IIFactors &f, int k0, cpx<double> (&pl)[kLPer], int &pp) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kLPer; ++q) pl[q] = ld2(f.L + (int64_t)k0 * kB + lane + 64 * q);
    pp = f.piv[k0 + (lane & (kSt - 1))];
}
// U's columns lo .. lo + kSt - 1 as entries (c, j) = U(c - j, c), j = 0 .. 2 kB
// (entries outside the matrix read U's first entry and are never used).
__device__ __forceinline__ void fetch_u(const IIFactors &f, int n, int lo, cpx<double> (&pu)[kRowPer]) {
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kRowPer; ++q) {
        const int idx = min(lane + 64 * q, kSt * kWC - 1), c = lo + idx / kWC, j = idx % kWC;
        const int r = c - j;
        pu[q] = ld2(f.U + (r >= 0 && c < n ? (int64_t)r * kWC + j : 0));
    }
}

// Entry j of the vector entering a forward solve, times `scale` (zero at and
// beyond n; the load is unconditional, from entry 0 there).
__device__ __forceinline__ cpx<double> y_in(const cpx<double> *yb, int n, int j, double scale) {
    const cpx<double> v = ld2(yb + (j < n ? j : 0));
    const double g = j < n ? scale : 0.0;
    return {v.re * g, v.im * g};
}

// y <- L^{-1} P (scale y), in place in the scratch vector.  Step k swaps y[k]
// with y[piv[k]] and updates rows k + 1 .. k + kB, in an LDS ring that holds
// y[k0 .. k0 + kSt + kB - 1] at the start of block k0: each block's entering
// entries are fetched a block ahead, its finished entries written a block
// behind, and its multipliers and pivots fetched a block ahead.
__device__ __forceinline__ void solve_forward(int n, const IILds &sm, const IIFactors &f, double scale) {
    const int lane = lane_id(), l8 = lane & (kSt - 1);
    cpx<double> *yr = sm.yr;
    if (lane < kSt + kB) st2(yr + lane, y_in(f.y, n, lane, scale));
    cpx<double> pre = y_in(f.y, n, kSt + kB + l8, scale);
    cpx<double> pl[kLPer];
    int pp;
    fetch_l(f, 0, pl, pp);
    int k0 = 0;
    for (; k0 < n - 1; k0 += kSt) {
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < kLPer; ++q) st2(sm.outL + lane + 64 * q, pl[q]);
        const int pblk = pp;  // lane i: the pivot of step k0 + i
        if (k0 + kSt < n - 1) fetch_l(f, k0 + kSt, pl, pp);
        if (k0 > 0 && lane < kSt) {
            st2(f.y + k0 - kSt + lane, ld2(yr + ((k0 - kSt + lane) & (kYR - 1))));
            st2(yr + ((k0 + kB + lane) & (kYR - 1)), pre);
            pre = y_in(f.y, n, k0 + kSt + kB + lane, scale);
        }
        wave_lds_sync();
        const int k1 = min(k0 + kSt, n - 1);
        for (int k = k0; k < k1; ++k) {
            const int p = __builtin_amdgcn_readlane(pblk, k - k0);
            const cpx<double> yk = ld2(yr + (k & (kYR - 1))), yp = ld2(yr + (p & (kYR - 1)));
            if (lane < kB && k + 1 + lane < n) {
                const int r = (k + 1 + lane) & (kYR - 1);
                const cpx<double> x = csel(k + 1 + lane == p, yk, ld2(yr + r));
                st2(yr + r, c_sub(x, c_mul(ld2(sm.outL + (k - k0) * kB + lane), yp)));
            }
            if (lane == 0) st2(yr + (k & (kYR - 1)), yp);
            __builtin_amdgcn_wave_barrier();
        }
    }
    wave_lds_sync();
    for (int j = max(k0 - kSt, 0) + lane; j < n; j += 64) st2(f.y + j, ld2(yr + (j & (kYR - 1))));
}

// y <- U^{-1} y, in place in the scratch vector, by columns: y[c] <- y[c] /
// U(c, c), then rows c - 2 kB .. c - 1 -= U(., c) y[c].  A block holds
// columns lo .. lo + kSt - 1 (entry (c, j) = U(c - j, c) staged in LDS); the
// ring holds y[lo - 2 kB .. lo + kSt - 1] at its start.  Returns the sum and
// the largest of |y_r|^2 over the result.
__device__ __forceinline__ void solve_backward(int n, const IILds &sm, const IIFactors &f, double &nrm2,
                                               double &mx2) {
    const int lane = lane_id();
    cpx<double> *yr = sm.yr;
    const int lo0 = (n - 1) / kSt * kSt;
    if (lane < 2 * kB + kSt) {
        const int j = lo0 - 2 * kB + lane;
        const cpx<double> v = ld2(f.y + (j >= 0 && j < n ? j : 0));
        if (j >= 0 && j < n) st2(yr + (j & (kYR - 1)), v);
    }
    cpx<double> pre = ld2(f.y + max(lo0 - kSt - 2 * kB + (lane & (kSt - 1)), 0));
    cpx<double> pu[kRowPer];
    fetch_u(f, n, lo0, pu);
    double s2 = 0.0, m2 = 0.0;
    for (int lo = lo0; lo >= 0; lo -= kSt) {
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < kRowPer; ++q)
            if (lane + 64 * q < kSt * kWC) st2(sm.rows + lane + 64 * q, pu[q]);
        if (lo > 0) fetch_u(f, n, lo - kSt, pu);
        if (lo != lo0 && lane < kSt) {
            const int j = lo + kSt + lane;  // the previous block's results out
            if (j < n) {
                const cpx<double> x = ld2(yr + (j & (kYR - 1)));
                st2(f.y + j, x);
                s2 += c_abs2(x);
                m2 = fmax(m2, c_abs2(x));
            }
            const int ji = lo - 2 * kB + lane;  // this block's lowest rows in
            if (ji >= 0) st2(yr + (ji & (kYR - 1)), pre);
            pre = ld2(f.y + max(ji - kSt, 0));
        }
        wave_lds_sync();
        for (int c = min(lo + kSt, n) - 1; c >= lo; --c) {
            const cpx<double> *uc = sm.rows + (c - lo) * kWC;
            const cpx<double> yc = c_mul(ld2(yr + (c & (kYR - 1))), ld2(uc));
            if (lane < 2 * kB && c - 1 - lane >= 0) {
                const int r = (c - 1 - lane) & (kYR - 1);
                st2(yr + r, c_sub(ld2(yr + r), c_mul(ld2(uc + 1 + lane), yc)));
            }
            if (lane == 0) st2(yr + (c & (kYR - 1)), yc);
            __builtin_amdgcn_wave_barrier();
        }
    }
    wave_lds_sync();
    if (lane < kSt && lane < n) {  // the last block (columns 0 .. kSt - 1)
        const cpx<double> x = ld2(yr + lane);
        st2(f.y + lane, x);
        s2 += c_abs2(x);
        m2 = fmax(m2, c_abs2(x));
    }
    nrm2 = wave_sum(s2);
    mx2 = wave_max(m2);
    wave_global_sync();
}

// Rayleigh quotient y^H B y of a unit vector y from B's lower
// triangle: sum_r B_rr |y_r|^2 + 2 Re sum_{r > c} conj(y_r) B_rc y_c.
template <typename T>
__device__ __forceinline__ double band_rayleigh(const cpx<T> *H, int64_t ld, int n, const cpx<double> *y) {
    const int lane = lane_id();
    double acc = 0.0;
    for (int r = lane; r < n; r += 64) {
        const cpx<double> yr = ld2(y + r);
        cpx<double> off = {0.0, 0.0};
        for (int c = max(r - kB, 0); c < r; ++c) off = c_add(off, c_mul(ldc(H + (int64_t)r + (int64_t)c * ld), ld2(y + c)));
        acc += ldc(H + (int64_t)r + (int64_t)r * ld).re * c_abs2(yr) + 2.0 * c_cmul(yr, off).re;
    }
    return wave_sum(acc);
}

// Eigenvalues closer than 1e-3 of the spectral radius (or 4e-12) form a
// cluster; its vectors are orthogonalised against each other.
__device__ __forceinline__ double cluster_tol(const double *w, int n) {
    return fmax(1e-3 * fmax(fabs(w[0]), fabs(w[n - 1])), 4e-12);
}

// One wavefront per eigenvalue: inverse iteration (LU of B - lam I,
// kIISolves solves from a hashed start vector, each rescaled) with lam = w_in[k],
// kept at least a few ulps above the shift of the previous member of its
// cluster (the shifts of a cluster are w_i0, then max(w_j, previous + 10 eps
// max(|w_j|, ||B||))).  Writes column k of V and its Rayleigh quotient.  The
// members of a cluster run in parallel; cluster_orth_kernel orthogonalises
// them afterwards.  Jobs (matrix, eigenvalue) are taken in a fixed stride
// over the grid.
// (Three wavefronts per SIMD: a few registers go to scratch, and the ten
// wavefronts per CU that the LDS then allows hide more of each step's latency
// than the eight that fit without spilling.)
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void band_ii_kernel(const cpx<T> *__restrict__ Hall, int64_t ld,
                                                     const int32_t *__restrict__ n_in, int64_t batch,
                                                     const double *__restrict__ w_in, double *__restrict__ w_out,
                                                     int64_t ldw, cpx<double> *__restrict__ Vall, int64_t ldv,
                                                     char *scratch, int64_t wave_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    const IILds sm(smem);
    const IIFactors f(scratch + (int64_t)blockIdx.x * wave_bytes, ld);
    const int lane = lane_id();
    for (int64_t job = blockIdx.x; job < batch * ld; job += gridDim.x) {
        const int64_t u = job / ld;
        const int k = (int)(job % ld);
        const int n = n_in[u];
        if (n < 0 || n > ld) {  // a side outside [0, ld]: NaN eigenvalues
            if (lane == 0) w_out[u * ldw + k] = NAN;
            continue;
        }
        if (k >= n) continue;
        const double *w = w_in + u * ld;
        const double tn = fmax(fabs(w[0]), fabs(w[n - 1]));
        const double ortol = cluster_tol(w, n);
        int i0 = k;
        while (i0 > 0 && w[i0] - w[i0 - 1] <= ortol) --i0;
        double lam = w[i0];
        for (int j = i0 + 1; j <= k; ++j) lam = fmax(w[j], lam + 10.0 * DBL_EPSILON * fmax(fabs(w[j]), tn));
        const cpx<T> *H = Hall + u * ld * ld;
        band_lu(H, ld, n, lam, fmax(DBL_EPSILON * tn, 1e-280), sm, f);
        for (int r = lane; r < n; r += 64) st2(f.y + r, cpx<double>{start_value(k, r, 0), start_value(k, r, 1)});
        wave_global_sync();
        double scale = 1.0, inv = 0.0;
        for (int it = 0; it < kIISolves; ++it) {
            solve_forward(n, sm, f, scale);
            wave_global_sync();
            double nrm2, mx2;
            solve_backward(n, sm, f, nrm2, mx2);
            scale = mx2 > 0.0 ? 1.0 / sqrt(mx2) : 1.0;  // the next solve starts from entries of at most 1
            inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
        }
        cpx<double> *vk = Vall + u * ldv * ldv + (int64_t)k * ldv;
        for (int r = lane; r < n; r += 64) st2(vk + r, c_scale(inv, ld2(f.y + r)));
        wave_global_sync();
        const double rq = band_rayleigh(H, ld, n, vk);
        if (lane == 0) w_out[u * ldw + k] = rq;
        wave_lds_sync();
    }
}

// One workgroup per cluster of two or more eigenvalues: the members' vectors
// orthonormalised in order by classical Gram-Schmidt applied twice (the dots
// with the earlier members by the sixteen wavefronts in turn, then one
// update), their Rayleigh quotients recomputed, and the members sorted by
// them with their columns.
constexpr int kOrthThreads = 1024;
template <typename T>
__global__ __launch_bounds__(kOrthThreads) void cluster_orth_kernel(const cpx<T> *__restrict__ Hall,
                                                                    int64_t ld, const int32_t *__restrict__ n_in,
                                                                    int64_t batch, const double *__restrict__ w_in,
                                                                    double *__restrict__ w_out, int64_t ldw,
                                                                    cpx<double> *__restrict__ Vall, int64_t ldv) {
    constexpr int NW = kOrthThreads / 64;
    __shared__ cpx<double> dots[kOrthThreads];
    __shared__ double red[NW];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    // jobs (eigenvalue index, matrix) with the matrix fastest: the matrices of a
    // batch often have their large clusters at the same indices, which would
    // otherwise all fall to one workgroup
    for (int64_t job = blockIdx.x; job < batch * ld; job += gridDim.x) {
        const int64_t u = job % batch;
        const int i0 = (int)(job / batch);
        const int n = n_in[u];
        if (n < 1 || n > ld || i0 >= n) continue;
        const double *w = w_in + u * ld;
        const double ortol = cluster_tol(w, n);
        if (i0 > 0 && w[i0] - w[i0 - 1] <= ortol) continue;  // not the first of its cluster
        int i1 = i0 + 1;
        while (i1 < n && w[i1] - w[i1 - 1] <= ortol) ++i1;
        if (i1 - i0 < 2) continue;
        cpx<double> *V = Vall + u * ldv * ldv;
        double *wo = w_out + u * ldw;
        for (int j = i0 + 1; j < i1; ++j) {
            cpx<double> *vj = V + (int64_t)j * ldv;
            for (int pass = 0; pass < 2; ++pass) {
                for (int c0 = i0; c0 < j; c0 += kOrthThreads) {
                    const int c1 = min(c0 + kOrthThreads, j);
                    for (int i = c0 + wid; i < c1; i += NW) {
                        const cpx<double> *vi = V + (int64_t)i * ldv;
                        double re = 0.0, im = 0.0;
                        for (int r = lane; r < n; r += 64) {
                            const cpx<double> d = c_cmul(ld2(vi + r), ld2(vj + r));
                            re += d.re;
                            im += d.im;
                        }
                        re = wave_sum(re);
                        im = wave_sum(im);
                        if (lane == 0) dots[i - c0] = {re, im};
                    }
                    __syncthreads();
                    for (int r = t; r < n; r += kOrthThreads) {
                        cpx<double> x = ld2(vj + r);
                        for (int i = c0; i < c1; ++i) x = c_sub(x, c_mul(ld2(V + (int64_t)i * ldv + r), dots[i - c0]));
                        st2(vj + r, x);
                    }
                    __syncthreads();
                }
            }
            double nrm = 0.0;
            for (int r = t; r < n; r += kOrthThreads) nrm += c_abs2(ld2(vj + r));
            nrm = wave_sum(nrm);
            if (lane == 0) red[wid] = nrm;
            __syncthreads();
            nrm = 0.0;
            for (int q = 0; q < NW; ++q) nrm += red[q];
            const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
            for (int r = t; r < n; r += kOrthThreads) st2(vj + r, c_scale(inv, ld2(vj + r)));
            __syncthreads();
        }
        const cpx<T> *H = Hall + u * ld * ld;
        for (int i = i0 + wid; i < i1; i += NW) {
            const double rq = band_rayleigh(H, ld, n, V + (int64_t)i * ldv);
            if (lane == 0) wo[i] = rq;
        }
        __syncthreads();
        for (int k = i0 + 1; k < i1; ++k) {  // insertion sort, columns along
            for (int j = k; j > i0; --j) {
                const double a = wo[j - 1], b = wo[j];
                __syncthreads();  // every thread has read the pair before it changes
                if (!(b < a)) break;
                cpx<double> *va = V + (int64_t)(j - 1) * ldv, *vb = V + (int64_t)j * ldv;
                for (int r = t; r < n; r += kOrthThreads) {
                    const cpx<double> x = ld2(va + r);
                    st2(va + r, ld2(vb + r));
                    st2(vb + r, x);
                }
                if (t == 0) {
                    wo[j - 1] = b;
                    wo[j] = a;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// The back-transformation takes the panels four at a time: with V = [V_a]
// (the four panels' reflectors side by side, zero above each panel's rows)
// Q_a Q_a+1 Q_a+2 Q_a+3 = I - V T V^H, T upper triangular 64 x 64 with the
// panels' T_a on its diagonal and, column block by column block,
// T[0:b, b] = -T[0:b, 0:b] (V[0:b]^H V_b) T_b.  A panel that ran no
// reflectors (fewer than two rows below its band, or past the last panel)
// counts as zero.  X is then read twice and written once per four panels.
constexpr int kGP = 4;         // panels per group
constexpr int kGR = kGP * kB;  // reflectors per group

__device__ __forceinline__ bool panel_ran(int pi, int npan, int n) { return pi < npan && n - (pi + 1) * kB >= 2; }

// Thread (rr, j): sum over rows r = s + rr + 16 q < n of conj(A[r][i]) B[r][j]
// for i < 16 (A, B column-major with leading dimensions lda, ldb), summed
// over the 16 consecutive lanes rr, into dst[i * kB] (LDS, a complex128
// array) from lane rr = 0; eight i at a time, to bound the registers in flight.
template <typename TA, typename TB>
__device__ __forceinline__ void gram16(const cpx<TA> *A, int64_t lda, const cpx<TB> *B, int64_t ldb, int s, int n,
                                       int rr, int j, cpx<double> *dst) {
#pragma unroll
    for (int h = 0; h < kB; h += kB / 2) {
        cpx<double> part[kB / 2];
#pragma unroll
        for (int i = 0; i < kB / 2; ++i) part[i] = {0.0, 0.0};
        for (int r = s + rr; r < n; r += kB) {
            const cpx<double> x = ldc(B + (int64_t)j * ldb + r);
#pragma unroll
            for (int i = 0; i < kB / 2; ++i) part[i] = c_add(part[i], c_cmul(ldc(A + (int64_t)(h + i) * lda + r), x));
        }
#pragma unroll
        for (int i = 0; i < kB / 2; ++i) {
#pragma unroll
            for (int o = 1; o < kB; o <<= 1) {
                part[i].re += __shfl_xor(part[i].re, o, 64);
                part[i].im += __shfl_xor(part[i].im, o, 64);
            }
            if (rr == 0) dst[(h + i) * kB] = part[i];
        }
    }
}

// One workgroup per (matrix, group of four panels): the group's T into
// tg + (u G + g) kGR^2, row-major, complex128.
template <typename T>
__global__ __launch_bounds__(256) void group_t_kernel(const cpx<T> *__restrict__ keep, int64_t keep_stride,
                                                      int64_t ld, const int32_t *__restrict__ n_in, int64_t batch,
                                                      int npan, int groups, cpx<double> *__restrict__ tg) {
    __shared__ cpx<double> Tp[kGP * (kGP + 1) / 2][kB][kB];  // block (a, b), a <= b, packed by rows
    __shared__ cpx<double> M[kGP - 1][kB][kB];                // G[c][b] T_b of the current column block b
    auto Tb = [&](int a, int b) -> cpx<double>(&)[kB][kB] { return Tp[a * kGP - a * (a - 1) / 2 + (b - a)]; };
    const int64_t u = blockIdx.x / groups;
    const int g = (int)(blockIdx.x % groups);
    if (u >= batch) return;
    const int n = n_in[u];
    if (n < 1 || n > ld) return;
    const int t = threadIdx.x, rr = t & (kB - 1), j = t >> 4;
    const cpx<T> *kp = keep + u * keep_stride;
    auto vpan = [&](int pi) { return kp + (int64_t)pi * (kB * ld + kB * kB); };
    for (int a = 0; a < kGP; ++a)
        for (int b = a; b < kGP; ++b) Tb(a, b)[j][rr] = {0.0, 0.0};
    __syncthreads();
    for (int b = 0; b < kGP; ++b) {
        const int pb = kGP * g + b;
        if (!panel_ran(pb, npan, n)) continue;  // T_b and its column block stay zero
        Tb(b, b)[j][rr] = ldc(vpan(pb) + kB * ld + j * kB + rr);
        __syncthreads();
        if (b == 0) continue;
        for (int c = 0; c < b; ++c) {  // M[c] = G[c][b] first, entry (i, j); then G[c][b] T_b
            const int pc = kGP * g + c;
            if (panel_ran(pc, npan, n)) gram16(vpan(pc), ld, vpan(pb), ld, (pb + 1) * kB, n, rr, j, &M[c][0][j]);
            else if (rr == 0)
                for (int i = 0; i < kB; ++i) M[c][i][j] = {0.0, 0.0};
            __syncthreads();
            cpx<double> m = {0.0, 0.0};  // entry (j, rr) of G T_b
            for (int l = 0; l <= rr; ++l) m = c_add(m, c_mul(M[c][j][l], Tb(b, b)[l][rr]));
            __syncthreads();
            M[c][j][rr] = m;
            __syncthreads();
        }
        for (int a = 0; a < b; ++a) {  // T[a][b] = -sum_{c = a}^{b - 1} T[a][c] M[c]
            cpx<double> x = {0.0, 0.0};
            for (int c = a; c < b; ++c)
                for (int l = 0; l < kB; ++l) x = c_add(x, c_mul(Tb(a, c)[j][l], M[c][l][rr]));
            Tb(a, b)[j][rr] = {-x.re, -x.im};
        }
        __syncthreads();
    }
    cpx<double> *out = tg + ((int64_t)u * groups + g) * kGR * kGR;
    for (int idx = t; idx < kGR * kGR; idx += 256) {
        const int r = idx / kGR, c = idx % kGR, a = r / kB, b = c / kB;
        st2(out + idx, a <= b ? Tb(a, b)[r % kB][c % kB] : cpx<double>{0.0, 0.0});
    }
}

// Group g of four panels applied to 16 columns of X: X <- X - V (T (V^H X))
// over the rows below the group's first panel.  V^H X: thread (b, j, rr) of
// 1024 takes panel b, column j and rows p_b + kB + rr + 16 q; T (V^H X): one
// entry per thread; the update: wavefront w takes the 16-row blocks w, w + 16,
// ..., lane (row l, column group cg) the row's four columns 4 cg .. 4 cg + 3,
// so that every reflector row is read once per workgroup.
template <typename T>
__global__ __launch_bounds__(1024) void group_bt_kernel(const cpx<T> *__restrict__ keep, int64_t keep_stride,
                                                        int64_t ld, const int32_t *__restrict__ n_in, int64_t batch,
                                                        int npan, int groups, const cpx<double> *__restrict__ tg,
                                                        int g, cpx<double> *__restrict__ Vall, int64_t ldv,
                                                        int64_t tiles) {
    __shared__ cpx<double> Ws[kGR][kB], Ys[kGR][kB];
    const int64_t u = blockIdx.x / tiles;
    const int tile = (int)(blockIdx.x % tiles);
    if (u >= batch) return;
    const int n = n_in[u];
    if (n < 1 || n > ld || !panel_ran(kGP * g, npan, n)) return;  // no reflectors in the group
    const int col0 = tile * kB;
    if (col0 >= n) return;
    const int t = threadIdx.x, s0 = (kGP * g + 1) * kB;
    const cpx<T> *kp = keep + u * keep_stride;
    cpx<double> *X = Vall + u * ldv * ldv;
    {
        const int rr = t & (kB - 1), j = (t >> 4) & (kB - 1), b = t >> 8, pb = kGP * g + b;
        const int col = min(col0 + j, n - 1);
        if (panel_ran(pb, npan, n))
            gram16(kp + (int64_t)pb * (kB * ld + kB * kB), ld, X + (int64_t)col * ldv, ldv, (pb + 1) * kB,
                   col0 + j < n ? n : 0, rr, 0, &Ws[b * kB][j]);
        else if (rr == 0)
            for (int i = 0; i < kB; ++i) Ws[b * kB + i][j] = {0.0, 0.0};
    }
    __syncthreads();
    {
        const int i = t >> 4, j = t & (kB - 1);
        const cpx<double> *trow = tg + ((int64_t)u * groups + g) * kGR * kGR + (int64_t)i * kGR;
        cpx<double> y = {0.0, 0.0};
        for (int l = i; l < kGR; ++l) y = c_add(y, c_mul(ld2(trow + l), Ws[l][j]));
        Ys[i][j] = y;
    }
    __syncthreads();
    const int wv = t >> 6, l = t & (kB - 1), cg = (t >> 4) & 3;
    for (int r0 = s0 + kB * wv; r0 < n; r0 += kB * (1024 / 64)) {
        const int r = r0 + l;
        cpx<double> acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
        if (r < n) {
#pragma unroll 1
            for (int b = 0; b < kGP; ++b) {
                const int pb = kGP * g + b;
                if (!panel_ran(pb, npan, n) || r < (pb + 1) * kB) continue;
                const cpx<T> *vb = kp + (int64_t)pb * (kB * ld + kB * kB) + r;
#pragma unroll
                for (int h = 0; h < kB; h += kB / 2) {
                    cpx<double> v8[kB / 2];  // eight of the row's reflector entries in flight together
#pragma unroll
                    for (int i = 0; i < kB / 2; ++i) v8[i] = ldc(vb + (int64_t)(h + i) * ld);
#pragma unroll
                    for (int i = 0; i < kB / 2; ++i) {
                        const cpx<double> *yrow = &Ys[b * kB + h + i][4 * cg];
#pragma unroll
                        for (int c = 0; c < 4; ++c) acc[c] = c_add(acc[c], c_mul(v8[i], yrow[c]));
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int col = col0 + 4 * cg + c;
                if (col < n) {
                    cpx<double> *x = X + (int64_t)col * ldv + r;
                    st2(x, c_sub(ld2(x), acc[c]));
                }
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const cpx<T> *__restrict__ H, int64_t ld,
                                                     const int64_t *__restrict__ offs, const int32_t *__restrict__ n_in,
                                                     cpx<T> *__restrict__ dst) {
    const int64_t u = blockIdx.y;
    const int n = n_in[u];
    if (n < 1 || n > ld) return;
    const cpx<T> *src = H + (offs ? offs[u] : u * ld * ld);
    cpx<T> *out = dst + u * ld * ld;
    const int64_t total = ld * (int64_t)n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) out[i] = src[i];
}

// The leading n_u x n_u block of each complex128 matrix (ld apart) rounded
// to complex64 into dst (ldv apart).
__global__ __launch_bounds__(256) void narrow_kernel(const cpx<double> *__restrict__ src, int64_t ld,
                                                     const int32_t *__restrict__ n_in, cpx<float> *__restrict__ dst,
                                                     int64_t ldv) {
    const int64_t u = blockIdx.y;
    const int n = n_in[u];
    if (n < 1 || n > ld) return;
    const int64_t total = (int64_t)n * n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t c = i / n, r = i % n;
        const cpx<double> x = ld2(src + u * ld * ld + c * ld + r);
        dst[u * ldv * ldv + c * ldv + r] = {(float)x.re, (float)x.im};
    }
}

}  // namespace

template <typename T>
hipError_t launch_gather_matrices(const cpx<T> *H, int64_t ld, const int64_t *offs, const int32_t *n_in,
                                  int64_t batch, cpx<T> *dst, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_kernel<T>, dim3(64, (unsigned)batch), dim3(256), 0, s, H, ld, offs, n_in, dst);
    return hipGetLastError();
}

hipError_t launch_narrow_vectors(const cpx<double> *src, int64_t ld, const int32_t *n_in, int64_t batch,
                                 cpx<float> *dst, int64_t ldv, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(narrow_kernel, dim3(64, (unsigned)batch), dim3(256), 0, s, src, ld, n_in, dst, ldv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_band_inverse_iteration(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch,
                                         const double *w_in, double *w_out, int64_t ldw, cpx<double> *V, int64_t ldv,
                                         void *scratch, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (ld > kEighLargeMax) return hipErrorInvalidValue;
    const int64_t lds = band_ii_lds_bytes(ld);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(band_ii_kernel<T>),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    // as many wavefronts as the CUs hold at once (registers and LDS), within the
    // workspace's slices
    int per_cu = 0, dev = 0, cus = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(band_ii_kernel<T>), 64,
                                                       (size_t)lds);
    if (err != hipSuccess) return err;
    err = hipGetDevice(&dev);
    if (err != hipSuccess) return err;
    err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (err != hipSuccess) return err;
    const int64_t waves = std::max<int64_t>(1, std::min<int64_t>(band_ii_waves(ld, batch), (int64_t)per_cu * cus));
    hipLaunchKernelGGL(band_ii_kernel<T>, dim3((unsigned)waves), dim3(64), (size_t)lds, s, H, ld, n_in, batch, w_in,
                       w_out, ldw, V, ldv, static_cast<char *>(scratch), band_ii_wave_bytes(ld));
    err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t groups = std::min<int64_t>(batch * ld, 2048);
    hipLaunchKernelGGL(cluster_orth_kernel<T>, dim3((unsigned)groups), dim3(kOrthThreads), 0, s, H, ld, n_in, batch,
                       w_in, w_out, ldw, V, ldv);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_panel_backtransform(const cpx<T> *keep, int64_t keep_stride, int64_t ld, const int32_t *n_in,
                                      int64_t batch, cpx<double> *V, int64_t ldv, cpx<double> *tg, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int npan = eigh_panels(ld), groups = eigh_panel_groups(ld);
    if (groups == 0) return hipSuccess;
    hipLaunchKernelGGL(group_t_kernel<T>, dim3((unsigned)(batch * groups)), dim3(256), 0, s, keep, keep_stride, ld,
                       n_in, batch, npan, groups, tg);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int64_t tiles = (ld + kB - 1) / kB;
    for (int g = groups - 1; g >= 0; --g) {
        hipLaunchKernelGGL(group_bt_kernel<T>, dim3((unsigned)(batch * tiles)), dim3(1024), 0, s, keep, keep_stride,
                           ld, n_in, batch, npan, groups, tg, g, V, ldv, tiles);
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

#define MLMC_EIGH_LARGE(T)                                                                                           \
    template hipError_t launch_gather_matrices<T>(const cpx<T> *, int64_t, const int64_t *, const int32_t *, int64_t, \
                                                  cpx<T> *, hipStream_t);                                           \
    template hipError_t launch_band_inverse_iteration<T>(const cpx<T> *, int64_t, const int32_t *, int64_t,          \
                                                         const double *, double *, int64_t, cpx<double> *, int64_t,  \
                                                         void *, hipStream_t);                                       \
    template hipError_t launch_panel_backtransform<T>(const cpx<T> *, int64_t, int64_t, const int32_t *, int64_t,     \
                                                      cpx<double> *, int64_t, cpx<double> *, hipStream_t);
MLMC_EIGH_LARGE(double)
MLMC_EIGH_LARGE(float)
#undef MLMC_EIGH_LARGE

}  // namespace mlmc
