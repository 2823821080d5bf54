// Device building blocks shared by the kernels of this library.
#pragma once

#include <cfloat>

#include "internal.hpp"

namespace mlmc {

__device__ __forceinline__ int wrap_index(int a, int N) {
    int r = a % N;
    return r < 0 ? r + N : r;
}

// Present-orbital map of one outcome (Sections 3.1-3.2): idx[(i*N + j)*n_orb + m]
// is the row of orbital m of cell (i, j) in H, or -1 when its group is vacant.
// Present orbitals keep their order.  Returns n to every thread.
// `scan` holds >= 17 ints of LDS.  blockDim.x must be a multiple of 64.
__device__ inline int build_present_index(const uint8_t *__restrict__ mask, const int32_t *__restrict__ orb_group,
                                          int n_orb, int G, int total, int *idx, int *scan) {
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6, nw = blockDim.x >> 6;
    int carry = 0;
    for (int base = 0; base < total; base += blockDim.x) {
        const int o = base + t;
        int present = 0;
        if (o < total) present = mask[(o / n_orb) * G + orb_group[o % n_orb]] ? 0 : 1;
        int incl = present;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if (lane >= off) incl += y;
        }
        if (lane == 63) scan[wid] = incl;
        __syncthreads();
        int before = 0, chunk = 0;
        for (int i = 0; i < nw; ++i) {
            if (i < wid) before += scan[i];
            chunk += scan[i];
        }
        if (o < total) idx[o] = present ? carry + before + incl - 1 : -1;
        carry += chunk;
        __syncthreads();
    }
    return carry;
}

// Walk the hopping table of eq. (tightbinding) for one outcome at reduced
// wave vector (k1, k2) of the N x N supercell.  For every row and every cell
// whose source and target orbitals are present, `sink(pass, a, b, z, amp,
// onsite)` is called with a = row of (cell, from), b = row of (cell + R, to),
// amp = h and z = h exp(2 pi i (k1 d1 + k2 d2) / N).  Each row is visited in
// two passes separated by barriers; within one pass distinct cells never
// address the same element, so the sink may update without atomics.
template <typename Sink>
__device__ inline void walk_hops(const DevLattice &lat, int N, double k1, double k2, const int *idx, Sink &&sink) {
    const int cells = N * N;
    for (int h = 0; h < lat.n_hops; ++h) {
        const int4 hi = lat.hop_i[h];
        const double4 hf = lat.hop_f[h];
        const bool onsite = hi.x == 0 && hi.y == 0 && hi.z == hi.w;
        double x = (k1 * hf.z + k2 * hf.w) / N;
        x -= floor(x);
        double sn, cs;
        sincospi(2.0 * x, &sn, &cs);
        const cpx<double> amp = {hf.x, hf.y};
        const cpx<double> z = {hf.x * cs - hf.y * sn, hf.x * sn + hf.y * cs};
        for (int pass = 0; pass < 2; ++pass) {
            for (int c = threadIdx.x; c < cells; c += blockDim.x) {
                const int i = c / N, j = c - (c / N) * N;
                const int c2 = wrap_index(i + hi.x, N) * N + wrap_index(j + hi.y, N);
                const int a = idx[c * lat.n_orb + hi.z];
                const int b = idx[c2 * lat.n_orb + hi.w];
                if (a < 0 || b < 0) continue;
                sink(pass, a, b, z, amp, onsite);
            }
            __syncthreads();
        }
    }
}

// Column start of the packed lower triangle (column-major) of an n x n matrix.
__device__ __forceinline__ int packed_col(int c, int n) { return c * n - (c * (c - 1)) / 2; }

// Householder reduction of a Hermitian matrix held as a packed lower triangle
// in LDS to real tridiagonal form: d[n] diagonal, e[n-1] non-negative
// sub-diagonal (moduli of the reduced sub-diagonal).  Reflector j is
// I - tau v v^H with v = x - alpha e_1, alpha = -e^{i arg x_0} |x|, x the
// column below the diagonal; the trailing block is updated as
// A <- A - v w^H - w v^H, w = p - (tau/2)(v^H p) v, p = tau A v.
// O(n^2) work per column runs in T; scalar reductions run in double.
// Requires blockDim.x even; v, pw hold >= n entries, part >= 2*cap.
// With refl != NULL the reflectors are kept for a back-transformation:
// refl[j] = (v_j[0], tau_j) as cpx with tau in .re of refl[cap + j] (v_j below
// its first entry stays in L's column j, which the reduction does not touch
// after step j), and alpha[j] = the reduced complex sub-diagonal entry
// (alpha[n - 2] the last one, left unreflected).
template <typename T>
__device__ void tridiag_packed(cpx<T> *L, int n, int cap, cpx<T> *v, cpx<T> *pw, cpx<T> *part, double *d, double *e,
                               double *red, cpx<T> *refl = nullptr, cpx<T> *alpha_out = nullptr) {
    const int t = threadIdx.x, nt = blockDim.x, half = nt >> 1;
    const bool row_half = t < half;
    const int hl = row_half ? t : t - half;
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        const cpx<T> *x = L + packed_col(j, n) + 1;
        double np = 0.0;
        for (int i = t; i < m; i += nt) np += (double)c_abs2(x[i]);
        const double nrm2 = block_sum(np, red);
        const double xnorm = sqrt(nrm2);
        const cpx<T> x0 = x[0];
        T tau = T(0);
        cpx<T> alpha = {T(0), T(0)}, v0 = {T(0), T(0)};
        if (xnorm > 0.0) {
            const double ax0 = sqrt((double)c_abs2(x0));
            const double pr = ax0 > 0.0 ? (double)x0.re / ax0 : 1.0;
            const double pi = ax0 > 0.0 ? (double)x0.im / ax0 : 0.0;
            const double are = -pr * xnorm, aim = -pi * xnorm;
            const double v0r = (double)x0.re - are, v0i = (double)x0.im - aim;
            const double vn2 = nrm2 - ax0 * ax0 + v0r * v0r + v0i * v0i;
            tau = (T)(2.0 / vn2);
            alpha = {(T)are, (T)aim};
            v0 = {(T)v0r, (T)v0i};
        }
        if (t == 0) {
            d[j] = (double)L[packed_col(j, n)].re;
            e[j] = xnorm;
            if (refl) {
                refl[j] = v0;
                refl[cap + j] = {tau, T(0)};
                alpha_out[j] = alpha;
            }
        }
        for (int i = t; i < m; i += nt) v[i] = (i == 0) ? v0 : x[i];
        __syncthreads();
        // p = tau A22 v: the row half sums the stored lower part of each row,
        // the column half the conjugated part above the diagonal.
        const int base = j + 1;
        for (int rr = hl; rr < m; rr += half) {
            cpx<T> acc = {T(0), T(0)};
            if (row_half) {
                for (int cc = 0; cc <= rr; ++cc) {
                    const cpx<T> a = L[packed_col(base + cc, n) + rr - cc];
                    acc = c_add(acc, c_mul(a, v[cc]));
                }
            } else {
                const cpx<T> *col = L + packed_col(base + rr, n);
                for (int cc = rr + 1; cc < m; ++cc) acc = c_add(acc, c_cmul(col[cc - rr], v[cc]));
            }
            part[(row_half ? 0 : cap) + rr] = acc;
        }
        __syncthreads();
        double kp = 0.0;
        for (int i = t; i < m; i += nt) {
            const cpx<T> p = c_scale(tau, c_add(part[i], part[cap + i]));
            pw[i] = p;
            kp += (double)v[i].re * (double)p.re + (double)v[i].im * (double)p.im;
        }
        const double vhp = block_sum(kp, red);
        const T K = (T)(0.5 * (double)tau * vhp);
        for (int i = t; i < m; i += nt) pw[i] = c_sub(pw[i], c_scale(K, v[i]));
        __syncthreads();
        for (int rr = hl; rr < m; rr += half) {
            const cpx<T> vr = v[rr], wr = pw[rr];
            for (int cc = row_half ? 0 : 1; cc <= rr; cc += 2) {
                const int k = packed_col(base + cc, n) + rr - cc;
                const cpx<T> upd = c_add(c_mulc(vr, pw[cc]), c_mulc(wr, v[cc]));
                L[k] = c_sub(L[k], upd);
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            d[n - 2] = (double)L[packed_col(n - 2, n)].re;
            const cpx<T> s = L[packed_col(n - 2, n) + 1];
            e[n - 2] = sqrt((double)s.re * (double)s.re + (double)s.im * (double)s.im);
            d[n - 1] = (double)L[packed_col(n - 1, n)].re;
            if (alpha_out) alpha_out[n - 2] = s;
        } else if (n == 1) {
            d[0] = (double)L[0].re;
        }
    }
    __syncthreads();
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x: the
// count of negative pivots of T - x I (Sturm sequence), with tiny pivots
// replaced by -pivmin.  e2 holds the squared sub-diagonal.
// 1/q for |q| >= pivmin (a normal number) and |q| finite: the hardware
// reciprocal estimate refined by two Newton steps (within about an ulp).
__device__ __forceinline__ double sturm_recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    double h = fma(-q, r, 1.0);
    r = fma(r, h, r);
    h = fma(-q, r, 1.0);
    return fma(r, h, r);
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x, from
// the signs of the pivots of T - x I = L D L^T (e2 = e^2).  Pivots are kept
// at least pivmin in magnitude, so every pivot and quotient stays finite.
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x, double pivmin) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
#pragma unroll 4
    for (int i = 1; i < n; ++i) {
        q = fma(-e2[i - 1], sturm_recip(q), d[i] - x);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
    }
    return c;
}

// The count of sturm_count and, in dx, the Newton correction -f/f' at x for
// f(x) = det(T - x I) = prod q_i: f'/f = sum q_i'/q_i with q_i' = -1 +
// e2_{i-1} q_{i-1}' / q_{i-1}^2, carried along the same pivots.
__device__ __forceinline__ int sturm_count_newton(const double *d, const double *e2, int n, double x, double pivmin,
                                                  double *dx) {
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int c = q < 0.0 ? 1 : 0;
    double r = sturm_recip(q), dq = -1.0, s = -r;
#pragma unroll 4
    for (int i = 1; i < n; ++i) {
        const double t = e2[i - 1] * r;
        dq = fma(t * r, dq, -1.0);
        q = fma(-e2[i - 1], r, d[i] - x);
        if (fabs(q) < pivmin) q = -pivmin;
        c += q < 0.0 ? 1 : 0;
        r = sturm_recip(q);
        s = fma(dq, r, s);
    }
    *dx = -1.0 / s;
    return c;
}

// Absolute width at which an eigenvalue's bracket is final (eV): far below
// what the smoothed IDoS resolves (a shift dE of one eigenvalue moves I by at
// most dE g'_max / (delta N^2 |F|)).
constexpr double kBisectAbsTol = 1e-12;
// Counts per eigenvalue that may take Newton or closing points; later counts
// bisect.  On the honeycomb tridiagonals an eigenvalue takes about 10 to 25.
constexpr int kNewtonCounts = 48;

// All eigenvalues of (d, e) by bisection on Sturm counts, in double
// precision.  The Gershgorin interval is first cut at blockDim.x points
// (one count per thread).  Thread t then takes eigenvalues t, t + blockDim.x,
// ... in turn, narrowing a bracket [lo, hi] with count(lo) <= i < count(hi)
// until its width reaches kBisectAbsTol (or a few ulps of the spectral
// radius, if that is larger).  Each count also gives the Newton correction
// of det(T - x I), scaled by the number m of eigenvalues in the bracket (the
// step to an m-fold root, also right for a tight cluster).  The next point
// is the Newton iterate while it lies inside the bracket and each correction
// at least halves the previous one, the midpoint otherwise; a correction
// below 0.45 of the final width is followed by counts at the iterate -/+
// that much, which close the bracket around it.  Every point only moves a
// side of a bracket that the counts certify, so the result has the bound of
// plain bisection; on the honeycomb tridiagonals the slowest thread makes
// about a third of the counts.  After kNewtonCounts counts on one
// eigenvalue every further point is the midpoint, so every further count
// halves the bracket: from the first cut (1/256 of the Gershgorin interval)
// to the final width takes at most log2(1 / (256 eps)) < 45 halvings, and the
// loop never stops before the bracket is final.  One count per loop turn, at whatever point
// each thread chose, keeps the threads of a wavefront in step; a thread
// moves on to its next eigenvalue as soon as one is done.
// e is squared in place.  w[i] = i-th smallest eigenvalue.
// cnt holds blockDim.x + 1 ints of LDS.  With parts > 1 the workgroup takes
// only the eigenvalues i = part nt + t + q parts nt of the matrix (the other
// parts go to other workgroups, each with its own copy of d and e).
__device__ inline void bisect_block(const double *d, double *e, int n, double *w, double *red, int *cnt,
                                    int part = 0, int parts = 1) {
    const int t = threadIdx.x, nt = blockDim.x, stride = parts * nt;
    if (n <= 0) return;
    double lo_p = INFINITY, hi_p = -INFINITY, e2max = 0.0;
    for (int i = t; i < n; i += nt) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        lo_p = fmin(lo_p, d[i] - r);
        hi_p = fmax(hi_p, d[i] + r);
        if (i + 1 < n) e2max = fmax(e2max, e[i] * e[i]);
    }
    double gl = block_min(lo_p, red);
    double gu = block_max(hi_p, red);
    const double emax2 = block_max(e2max, red);
    for (int i = t; i + 1 < n; i += nt) e[i] = e[i] * e[i];
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double bnorm = fmax(fabs(gl), fabs(gu));
    const double margin = 2.0 * DBL_EPSILON * bnorm * (double)n + 2.0 * pivmin;
    gl -= margin;
    gu += margin;
    const double atol = fmax(kBisectAbsTol, 2.0 * DBL_EPSILON * bnorm);
    __syncthreads();
    const double step = (gu - gl) / nt;
    cnt[t + 1] = (t + 1 == nt) ? n : sturm_count(d, e, n, gl + step * (t + 1), pivmin);
    if (t == 0) cnt[0] = 0;
    __syncthreads();
    int i = part * nt + t;
    double lo = 0.0, hi = 0.0, xn = NAN, dxprev = INFINITY, xc = 0.0, h = 0.0;
    int clo = 0, chi = 0, mode = 0, its = 0;  // mode 1 / 2: count at xc - h / xc + h next
    auto start = [&]() {
        int a = 0, b = nt;  // find g with cnt[g] <= i < cnt[g + 1]
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (cnt[mid] <= i) a = mid; else b = mid;
        }
        lo = gl + step * a;
        hi = (a + 1 == nt) ? gu : gl + step * (a + 1);
        clo = cnt[a];
        chi = cnt[a + 1];
        xn = NAN;
        dxprev = INFINITY;
        mode = 0;
        its = 0;
    };
    if (i < n) start();
    while (i < n) {
        const double width = hi - lo;
        const double tolw = fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
        const double mid = lo + 0.5 * width;
        bool done = width <= tolw;
        double x = mid;
        int kind = 0;  // 0 midpoint, 1 Newton iterate, 2 / 3 closing counts
        if (!done && its >= kNewtonCounts) {  // past the Newton budget: bisect
            if (mid <= lo || mid >= hi) done = true;
        } else if (!done) {
            if (mode == 1) {
                if (xc - h > lo && xc - h < hi) { x = xc - h; kind = 2; } else mode = 2;
            }
            if (mode == 2 && kind == 0) {
                if (xc + h > lo && xc + h < hi) { x = xc + h; kind = 3; } else mode = 0;
            }
            if (mode == 0 && kind == 0) {
                if (xn > lo && xn < hi) { x = xn; kind = 1; }
                else if (mid <= lo || mid >= hi) done = true;
            }
        }
        if (done) {
            w[i] = lo + 0.5 * (hi - lo);
            i += stride;
            if (i < n) start();
            continue;
        }
        double dx;
        const int c = sturm_count_newton(d, e, n, x, pivmin, &dx);
        ++its;
        if (c > i) { hi = x; chi = c; } else { lo = x; clo = c; }
        const double st = (double)(chi - clo) * dx;
        if (kind == 2) {
            mode = 2;
        } else if (kind == 3) {
            mode = 0;
            xn = NAN;
        } else if (kind == 1) {
            xn = (fabs(st) <= 0.5 * dxprev) ? x + st : NAN;
            dxprev = fabs(st);
            const double h0 = 0.45 * tolw;
            if (fabs(st) <= h0) {
                xc = x + st;
                h = h0;
                mode = 1;
                xn = NAN;
            }
        } else {
            xn = x + st;
            dxprev = INFINITY;
        }
    }
}

}  // namespace mlmc
