// Eigenvectors of matrices above the LDS-resident size (complex128).  After
// stage 1 (dense -> band of half-width kB, each panel's block reflector kept)
// and the eigenvalues (chase + bisection), the eigenvectors are
//   band_ii_kernel   inverse iteration on the band matrix B, one wavefront
//                    per cluster of close eigenvalues: pivoted band LU of
//                    B - lam I, three solves from a hashed start vector,
//                    each followed by orthogonalisation against the
//                    cluster's earlier vectors
//   panel_bt_kernel  X <- (I - V_p T_p V_p^H) X for the panels from last to
//                    first, which takes B's eigenvectors to H's
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

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

// Whole-entry loads and stores of a complex value (one 16-byte access, no
// struct copy through the stack).
typedef double d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cpx<double> ld2(const cpx<double> *p) {
    const d2v v = *reinterpret_cast<const d2v *>(p);
    return {v.x, v.y};
}
__device__ __forceinline__ void st2(cpx<double> *p, cpx<double> x) { *reinterpret_cast<d2v *>(p) = d2v{x.re, x.im}; }

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
struct IIFactors {
    cpx<double> *U, *L;
    int *piv;
    __device__ IIFactors(char *base, int64_t ld) {
        U = reinterpret_cast<cpx<double> *>(base);
        L = U + (ld + kSt) * kWC;
        piv = reinterpret_cast<int *>(L + (ld + kSt) * kB);
    }
};

struct IILds {
    cpx<double> *win, *lbuf, *rows, *outU, *outL, *y;
    int *outP;
    __device__ IILds(unsigned char *base, int64_t ld) {
        win = reinterpret_cast<cpx<double> *>(base);
        lbuf = win + kWR * kWC;
        rows = lbuf + kB;
        outU = rows + kSt * kWC;
        outL = outU + kSt * kWC;
        y = outL + kSt * kB;
        outP = reinterpret_cast<int *>(y + ld);
    }
};

// Window slot of (row r, column c): the window holds rows k .. k + kB and
// columns k .. k + 2 kB at elimination step k.
__device__ __forceinline__ int wat(int r, int c) { return (r % kWR) * kWC + (c % kWC); }

// B[r][c] - lam delta_rc of the band matrix of half-width kB whose lower
// triangle stage 1 left in H (column-major, ld); zero outside the band and
// outside the n x n matrix (n >= 1); the diagonal is taken real.  The load is
// unconditional (from H[0] for an entry outside), so that a block of such
// loads stays in flight together.
__device__ __forceinline__ cpx<double> band_ld(const cpx<double> *H, int64_t ld, int n, int r, int c, double lam) {
    const int d = r - c;
    const bool in = r >= 0 && c >= 0 && r < n && c < n && d <= kB && d >= -kB;
    const bool up = d < 0;
    const int64_t at = in ? (up ? (int64_t)c + (int64_t)r * ld : (int64_t)r + (int64_t)c * ld) : 0;
    const cpx<double> x = ld2(H + at);
    // factors instead of selects, so that both halves are always used
    const double keep = in ? 1.0 : 0.0, sgn = d == 0 ? 0.0 : (up ? -keep : keep);
    return {(x.re - (d == 0 ? lam : 0.0)) * keep, x.im * sgn};
}

// Band rows k0 + kWR + i, columns k0 + i + 1 .. k0 + i + 2 kB + 1 (i < kSt):
// what the steps k0 .. k0 + kSt - 1 slide into the window.
__device__ __forceinline__ void fetch_rows(const cpx<double> *H, int64_t ld, int n, double lam, int k0,
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
// down and right by one.  The steps touch LDS only: the band rows they slide
// in are fetched a block ahead, and their factors go out a block behind.
__device__ __forceinline__ void band_lu(const cpx<double> *H, int64_t ld, int n, double lam, double tiny, const IILds &sm,
                        const IIFactors &f) {
    static_assert(kSt * kB == 64 * kLPer, "whole multiplier blocks");
    const int lane = lane_id();
    for (int idx = lane; idx < kWR * kWC; idx += 64) {
        const int r = idx / kWC, c = idx % kWC;
        sm.win[wat(r, c)] = band_ld(H, ld, n, r, c, lam);
    }
    cpx<double> pre[kRowPer];
    fetch_rows(H, ld, n, lam, 0, pre);
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
            int key = 0;
            if (lane < kWR && k + lane < n)
                key = (int)((__float_as_uint((float)c_abs2(sm.win[wat(k + lane, k)])) & ~31u) | (uint32_t)(31 - lane));
            const int p = k + 31 - (max_key32(key) & 31);
            if (p != k && lane < kWC) {
                const int c = k + lane;
                const cpx<double> a = ld2(sm.win + wat(k, c)), b = ld2(sm.win + wat(p, c));
                st2(sm.win + wat(k, c), b);
                st2(sm.win + wat(p, c), a);
            }
            wave_lds_sync();
            cpx<double> piv = sm.win[wat(k, k)];
            double a2 = c_abs2(piv);
            if (!(a2 >= tiny * tiny)) {  // singular to working precision: lam is an eigenvalue
                piv = {tiny, 0.0};
                a2 = tiny * tiny;
            }
            const cpx<double> rp = {piv.re / a2, -piv.im / a2};
            if (lane < kB) {
                const int r = k + 1 + lane;
                const cpx<double> l = csel(r < n, c_mul(sm.win[wat(r, k)], rp), cpx<double>{0.0, 0.0});
                sm.lbuf[lane] = l;
                sm.outL[i * kB + lane] = l;
            }
            if (lane == 0) sm.outP[i] = p;
            if (lane < kWC) sm.outU[i * kWC + lane] = csel(lane == 0, rp, sm.win[wat(k, k + lane)]);
            wave_lds_sync();
            {  // rows k + 1 .. k + kB -= l * row k over columns k + 1 .. k + 2 kB
                const int cc = 1 + (lane & 31);
                const cpx<double> urow = sm.win[wat(k, k + cc)];
#pragma unroll
                for (int q = 0; q < kB / 2; ++q) {
                    const int rr = 1 + (lane >> 5) + 2 * q;
                    const cpx<double> l = sm.lbuf[rr - 1];
                    const int at = wat(k + rr, k + cc);
                    sm.win[at] = c_sub(sm.win[at], c_mul(l, urow));
                }
            }
            wave_lds_sync();
            // row k's slot takes row k + kB + 1 (columns k + 1 .. k + 2 kB + 1); column
            // k's slot becomes column k + 2 kB + 1, zero in rows k + 1 .. k + kB
            if (lane < kWC) sm.win[wat(k + kWR, k + 1 + lane)] = sm.rows[i * kWC + lane];
            if (lane < kB) sm.win[wat(k + 1 + lane, k + kWC)] = {0.0, 0.0};
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

// y <- (B - lam I)^{-1} y from the factors (y in LDS); the factors of a block
// of kSt steps are fetched while the previous block is applied.
__device__ __forceinline__ void band_solve(int n, const IILds &sm, const IIFactors &f) {
    const int lane = lane_id();
    // forward: y <- L^{-1} P y; step k swaps y[k] with y[piv[k]] and updates rows k + 1 .. k + kB
    cpx<double> pl[kLPer];
    int pp;
    fetch_l(f, 0, pl, pp);
    for (int k0 = 0; k0 < n - 1; k0 += kSt) {
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < kLPer; ++q) st2(sm.outL + lane + 64 * q, pl[q]);
        if (lane < kSt) sm.outP[lane] = pp;
        if (k0 + kSt < n - 1) fetch_l(f, k0 + kSt, pl, pp);
        wave_lds_sync();
        const int k1 = min(k0 + kSt, n - 1);
        for (int k = k0; k < k1; ++k) {
            const int p = sm.outP[k - k0];
            const cpx<double> yk = sm.y[k], yp = sm.y[p];
            if (lane < kB && k + 1 + lane < n) {
                const int r = k + 1 + lane;
                const cpx<double> x = csel(r == p, yk, sm.y[r]);
                sm.y[r] = c_sub(x, c_mul(sm.outL[(k - k0) * kB + lane], yp));
            }
            if (lane == 0) sm.y[k] = yp;
            wave_lds_sync();
        }
    }
    // backward, by columns: y[c] <- y[c] / U(c, c), then rows c - 2 kB .. c - 1 -= U(., c) y[c];
    // a block holds columns lo .. lo + kSt - 1, entry (c, j) = U(c - j, c)
    cpx<double> pu[kRowPer];
    int lo = (n - 1) / kSt * kSt;
    fetch_u(f, n, lo, pu);
    for (; lo >= 0; lo -= kSt) {
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < kRowPer; ++q)
            if (lane + 64 * q < kSt * kWC) st2(sm.rows + lane + 64 * q, pu[q]);
        if (lo > 0) fetch_u(f, n, lo - kSt, pu);
        wave_lds_sync();
        for (int c = min(lo + kSt, n) - 1; c >= lo; --c) {
            const cpx<double> *uc = sm.rows + (c - lo) * kWC;
            const cpx<double> yc = c_mul(sm.y[c], uc[0]);
            if (lane < 2 * kB && c - 1 - lane >= 0) {
                const int r = c - 1 - lane;
                sm.y[r] = c_sub(sm.y[r], c_mul(uc[1 + lane], yc));
            }
            if (lane == 0) sm.y[c] = yc;
            wave_lds_sync();
        }
    }
}

// Rayleigh quotient y^H B y of a unit vector y (in LDS) from B's lower
// triangle: sum_r B_rr |y_r|^2 + 2 Re sum_{r > c} conj(y_r) B_rc y_c.
__device__ __forceinline__ double band_rayleigh(const cpx<double> *H, int64_t ld, int n, const cpx<double> *y) {
    const int lane = lane_id();
    double acc = 0.0;
    for (int r = lane; r < n; r += 64) {
        const cpx<double> yr = y[r];
        cpx<double> off = {0.0, 0.0};
        for (int c = max(r - kB, 0); c < r; ++c) off = c_add(off, c_mul(H[(int64_t)r + (int64_t)c * ld], y[c]));
        acc += H[(int64_t)r + (int64_t)r * ld].re * c_abs2(yr) + 2.0 * c_cmul(yr, off).re;
    }
    return wave_sum(acc);
}

// One wavefront per cluster of eigenvalues (neighbours closer than 1e-3 of
// the spectral radius): each member's shift is kept at least a few ulps above
// the previous member's, and its vector is orthogonalised against the
// cluster's earlier vectors after every solve.  The eigenvalues go out as the
// vectors' Rayleigh quotients, the cluster's members sorted ascending with
// their columns.  Jobs (matrix, first eigenvalue of a cluster) are taken in a
// fixed stride over the grid; w_in (from the bisection) is only read, so
// every wavefront finds the same clusters.
__global__ __launch_bounds__(64) void band_ii_kernel(const cpx<double> *__restrict__ Hall, int64_t ld,
                                                     const int32_t *__restrict__ n_in, int64_t batch,
                                                     const double *__restrict__ w_in, double *__restrict__ w_out,
                                                     int64_t ldw, cpx<double> *__restrict__ Vall, int64_t ldv,
                                                     char *scratch, int64_t wave_bytes) {
    extern __shared__ __align__(16) unsigned char smem[];
    const IILds sm(smem, ld);
    const IIFactors f(scratch + (int64_t)blockIdx.x * wave_bytes, ld);
    const int lane = lane_id();
    for (int64_t job = blockIdx.x; job < batch * ld; job += gridDim.x) {
        const int64_t u = job / ld;
        const int i0 = (int)(job % ld);
        const int n = n_in[u];
        if (n < 0 || n > ld) {  // a side outside [0, ld]: NaN eigenvalues
            if (lane == 0) w_out[u * ldw + i0] = NAN;
            continue;
        }
        if (i0 >= n) continue;
        const double *w = w_in + u * ld;
        double *wo = w_out + u * ldw;
        const double tn = fmax(fabs(w[0]), fabs(w[n - 1]));
        const double ortol = fmax(1e-3 * tn, 4e-12);
        if (i0 > 0 && w[i0] - w[i0 - 1] <= ortol) continue;  // not the first of its cluster
        int i1 = i0 + 1;
        while (i1 < n && w[i1] - w[i1 - 1] <= ortol) ++i1;
        const cpx<double> *H = Hall + u * ld * ld;
        cpx<double> *V = Vall + u * ldv * ldv;
        const double tiny = fmax(DBL_EPSILON * tn, 1e-280);
        double shift_prev = 0.0;
        for (int k = i0; k < i1; ++k) {
            double lam = w[k];
            if (k > i0) lam = fmax(lam, shift_prev + 10.0 * DBL_EPSILON * fmax(fabs(lam), tn));
            shift_prev = lam;
            band_lu(H, ld, n, lam, tiny, sm, f);
            for (int r = lane; r < n; r += 64) sm.y[r] = {start_value(k, r, 0), start_value(k, r, 1)};
            for (int it = 0; it < 3; ++it) {
                wave_lds_sync();
                band_solve(n, sm, f);
                double mx = 0.0;
                for (int r = lane; r < n; r += 64) mx = fmax(mx, c_abs2(sm.y[r]));
                mx = wave_max(mx);
                const double sc = mx > 0.0 ? 1.0 / sqrt(mx) : 1.0;
                for (int r = lane; r < n; r += 64) sm.y[r] = c_scale(sc, sm.y[r]);
                for (int q = i0; q < k; ++q) {  // against the cluster's earlier vectors
                    const cpx<double> *vq = V + (int64_t)q * ldv;
                    double dre = 0.0, dim = 0.0;
                    for (int r = lane; r < n; r += 64) {
                        const cpx<double> d = c_cmul(vq[r], sm.y[r]);
                        dre += d.re;
                        dim += d.im;
                    }
                    const cpx<double> dot = {wave_sum(dre), wave_sum(dim)};
                    for (int r = lane; r < n; r += 64) sm.y[r] = c_sub(sm.y[r], c_mul(vq[r], dot));
                }
                double nrm = 0.0;
                for (int r = lane; r < n; r += 64) nrm += c_abs2(sm.y[r]);
                nrm = wave_sum(nrm);
                const double inv = nrm > 0.0 ? 1.0 / sqrt(nrm) : 0.0;
                for (int r = lane; r < n; r += 64) sm.y[r] = c_scale(inv, sm.y[r]);
            }
            wave_lds_sync();
            const double rq = band_rayleigh(H, ld, n, sm.y);
            cpx<double> *vk = V + (int64_t)k * ldv;
            for (int r = lane; r < n; r += 64) vk[r] = sm.y[r];
            if (lane == 0) wo[k] = rq;
            wave_lds_sync();
            wave_global_sync();  // the cluster's next member reads this column
        }
        // insertion sort of the cluster's Rayleigh quotients, columns along
        for (int k = i0 + 1; k < i1; ++k) {
            for (int j = k; j > i0; --j) {
                const double a = wo[j - 1], b = wo[j];
                if (!(b < a)) break;
                cpx<double> *va = V + (int64_t)(j - 1) * ldv, *vb = V + (int64_t)j * ldv;
                for (int r = lane; r < n; r += 64) {
                    const cpx<double> t = ld2(va + r);
                    st2(va + r, ld2(vb + r));
                    st2(vb + r, t);
                }
                if (lane == 0) {
                    wo[j - 1] = b;
                    wo[j] = a;
                }
                wave_global_sync();
            }
        }
    }
}

// Panel p's block reflector applied to 16 columns of X: X <- X - V_p (T_p (V_p^H X))
// over the rows s = p + kB .. n - 1.  Thread (rr, j) takes column j of the
// tile and rows s + rr + 16 q.
__global__ __launch_bounds__(256) void panel_bt_kernel(const cpx<double> *__restrict__ keep, int64_t keep_stride,
                                                       int64_t ld, const int32_t *__restrict__ n_in, int64_t batch,
                                                       cpx<double> *__restrict__ Vall, int64_t ldv, int p,
                                                       int64_t tiles) {
    __shared__ cpx<double> Ws[kB][kB], Ys[kB][kB];
    const int64_t u = blockIdx.x / tiles;
    const int tile = (int)(blockIdx.x % tiles);
    if (u >= batch) return;
    const int n = n_in[u];
    const int s = p + kB, m = n - s;
    if (n < 1 || n > ld || m < 2) return;  // the panel had no reflectors
    const int col0 = tile * kB;
    if (col0 >= n) return;
    const cpx<double> *Vp = keep + u * keep_stride + (int64_t)(p / kB) * (kB * ld + kB * kB);
    const cpx<double> *Tp = Vp + kB * ld;
    cpx<double> *X = Vall + u * ldv * ldv;
    const int t = threadIdx.x, rr = t & 15, j = t >> 4, col = col0 + j;
    const bool live = col < n;
    cpx<double> acc[kB];
#pragma unroll
    for (int i = 0; i < kB; ++i) acc[i] = {0.0, 0.0};
    if (live) {
        for (int r = s + rr; r < n; r += kB) {
            const cpx<double> x = X[(int64_t)col * ldv + r];
#pragma unroll
            for (int i = 0; i < kB; ++i) acc[i] = c_add(acc[i], c_cmul(Vp[(int64_t)i * ld + r], x));
        }
    }
#pragma unroll
    for (int i = 0; i < kB; ++i) {  // over the 16 consecutive lanes of a column
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            acc[i].re += __shfl_xor(acc[i].re, o, 64);
            acc[i].im += __shfl_xor(acc[i].im, o, 64);
        }
    }
    if (rr == 0) {
#pragma unroll
        for (int i = 0; i < kB; ++i) Ws[i][j] = acc[i];
    }
    __syncthreads();
    {  // Y = T W, T upper triangular: entry (rr, j)
        cpx<double> yv = {0.0, 0.0};
        for (int l = rr; l < kB; ++l) yv = c_add(yv, c_mul(Tp[rr * kB + l], Ws[l][j]));
        Ys[rr][j] = yv;
    }
    __syncthreads();
    if (live) {
        for (int r = s + rr; r < n; r += kB) {
            cpx<double> sum = {0.0, 0.0};
#pragma unroll
            for (int i = 0; i < kB; ++i) sum = c_add(sum, c_mul(Vp[(int64_t)i * ld + r], Ys[i][j]));
            cpx<double> &x = X[(int64_t)col * ldv + r];
            x = c_sub(x, sum);
        }
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const cpx<double> *__restrict__ H, int64_t ld,
                                                     const int64_t *__restrict__ offs, const int32_t *__restrict__ n_in,
                                                     cpx<double> *__restrict__ dst) {
    const int64_t u = blockIdx.y;
    const int n = n_in[u];
    if (n < 1 || n > ld) return;
    const cpx<double> *src = H + (offs ? offs[u] : u * ld * ld);
    cpx<double> *out = dst + u * ld * ld;
    const int64_t total = ld * (int64_t)n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) out[i] = src[i];
}

}  // namespace

hipError_t launch_gather_matrices(const cpx<double> *H, int64_t ld, const int64_t *offs, const int32_t *n_in,
                                  int64_t batch, cpx<double> *dst, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gather_kernel, dim3(64, (unsigned)batch), dim3(256), 0, s, H, ld, offs, n_in, dst);
    return hipGetLastError();
}

hipError_t launch_band_inverse_iteration(const cpx<double> *H, int64_t ld, const int32_t *n_in, int64_t batch,
                                         const double *w_in, double *w_out, int64_t ldw, cpx<double> *V, int64_t ldv,
                                         void *scratch, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (ld > kEighLargeMax) return hipErrorInvalidValue;
    const int64_t lds = band_ii_lds_bytes(ld);
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(band_ii_kernel),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(band_ii_kernel, dim3((unsigned)band_ii_waves(ld, batch)), dim3(64), (size_t)lds, s, H, ld,
                       n_in, batch, w_in, w_out, ldw, V, ldv, static_cast<char *>(scratch), band_ii_wave_bytes(ld));
    return hipGetLastError();
}

hipError_t launch_panel_backtransform(const cpx<double> *keep, int64_t keep_stride, int64_t ld, const int32_t *n_in,
                                      int64_t batch, cpx<double> *V, int64_t ldv, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int64_t tiles = (ld + kB - 1) / kB;
    int last = -1;
    for (int p = 0; p + kB + 1 < ld; p += kB) last = p;  // the panels stage 1 ran
    for (int p = last; p >= 0; p -= kB) {
        hipLaunchKernelGGL(panel_bt_kernel, dim3((unsigned)(batch * tiles)), dim3(256), 0, s, keep, keep_stride, ld,
                           n_in, batch, V, ldv, p, tiles);
        const hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

}  // namespace mlmc
