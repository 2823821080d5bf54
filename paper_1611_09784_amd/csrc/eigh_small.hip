// Eigenstates (eigenvalues and eigenvectors) of small Hermitian matrices,
// one workgroup per matrix: the eigenstates of H(k) that a conductivity
// estimate needs besides the energies (the paper names the Kubo-Greenwood
// conductivity as the next quantity of interest).
//
// 1. The lower triangle is loaded into a packed triangle in LDS and reduced
//    to real tridiagonal form as on the eigenvalue path, keeping the
//    reflectors: H = Q T_c Q^H, T_c with complex sub-diagonal alpha_j, made
//    real by D = diag(delta) (delta_0 = 1, delta_{j+1} = delta_j alpha_j /
//    |alpha_j|): T_c = D T D^H.
// 2. Eigenvalues of T by the Sturm bisection of the eigenvalue path (refined
//    to working accuracy by the Rayleigh quotients of step 3's vectors).
// 3. Eigenvectors z_i of T by inverse iteration with partial pivoting, one
//    thread per cluster of eigenvalues closer than 1e-3 ||T|| (each member
//    from its own start vector, shifts kept apart by a few ulps, and
//    orthogonalised against the cluster's earlier members in every
//    iteration; Golub & Van Loan Section 8.2.2, Wilkinson's cluster
//    treatment), the vectors in a device workspace.
// 4. Back-transformation V = Q D Z with each eigenvector held in the
//    registers of four lanes, the reflectors read from LDS.
#include "device_common.hpp"

namespace mlmc {

struct EighLayout {
    size_t L, v, pw, part, d, e, e1, red, cnt, refl, alpha, delta, bytes;
};

template <typename T>
__host__ __device__ inline EighLayout eigh_layout(int cap, int threads) {
    EighLayout o{};
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p += (bytes + 15) & ~size_t(15);
        return at;
    };
    o.L = take(sizeof(cpx<T>) * (size_t)packed_size(cap));
    o.v = take(sizeof(cpx<T>) * (size_t)cap);
    o.pw = take(sizeof(cpx<T>) * (size_t)cap);
    o.part = take(sizeof(cpx<T>) * 2 * (size_t)cap);
    o.d = take(sizeof(double) * (size_t)cap);
    o.e = take(sizeof(double) * (size_t)cap);
    o.e1 = take(sizeof(double) * (size_t)cap);
    o.red = take(sizeof(double) * 32);
    o.cnt = take(sizeof(int) * (size_t)(threads + 1));
    o.refl = take(sizeof(cpx<T>) * 2 * (size_t)cap);
    o.alpha = take(sizeof(cpx<T>) * (size_t)cap);
    o.delta = take(sizeof(cpx<double>) * (size_t)cap);
    o.bytes = p;
    return o;
}

// Doubles of device workspace per matrix of side bound cap: Z [cap][cap] and
// the inverse iteration's scratch, 6 cap per eigenvalue (later the complex
// working copy of V); both parts start at even offsets (16-byte aligned).
__host__ __device__ inline int64_t eigh_zsize(int64_t cap) { return (cap * cap + 1) & ~int64_t(1); }
__host__ __device__ inline int64_t eigh_work_doubles(int64_t cap) { return eigh_zsize(cap) + 6 * cap * cap; }

// Deterministic start vector entry in (-1, 1) for (eigenvalue k, row r).
__device__ __forceinline__ double start_entry(int k, int r) {
    uint32_t h = (uint32_t)k * 0x9E3779B1u ^ ((uint32_t)r + 0x7F4A7C15u) * 0x85EBCA6Bu;
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return ((double)h + 0.5) * (2.0 / 4294967296.0) - 1.0;
}

// Eigenvectors of the symmetric tridiagonal (d, e) for the eigenvalues
// w[i0..i1) (one cluster), into Z columns i0..i1-1 (Z row-major: entry
// (r, k) at r ldz + k, so that threads taking consecutive vectors touch
// consecutive addresses later on).
// scr: 6 n doubles (the pivoted LU of T - lambda I: diagonal, two upper
// diagonals, multipliers, interchange flags; and the iterate).  rq[i0..i1):
// the refined eigenvalues.
__device__ void cluster_vectors(const double *d, const double *e, int n, const double *w, int i0, int i1,
                                double tnorm, double *scr, double *Z, int64_t ldz, double *rq) {
    double *dg = scr, *u1 = scr + n, *u2 = scr + 2 * n, *lm = scr + 3 * n, *pv = scr + 4 * n, *y = scr + 5 * n;
    const double eps = DBL_EPSILON;
    // pivots smaller than eps ||T|| are raised to it (keeping their sign), so
    // that a solve grows the iterate by at most about 1 / (eps ||T||)
    const double tiny = fmax(eps * tnorm, 1e-280);
    auto raise = [&](double x) { return fabs(x) >= tiny ? x : (x < 0.0 ? -tiny : tiny); };
    double shift_prev = 0.0;
    for (int k = i0; k < i1; ++k) {
        double lam = w[k];
        if (k > i0) {  // keep the shifts of a cluster's members apart
            const double pertol = 10.0 * eps * fmax(fabs(lam), tnorm);
            if (lam < shift_prev + pertol) lam = shift_prev + pertol;
        }
        shift_prev = lam;
        // pivoted LU of T - lam I; the running pivot row stays in registers
        // and the factors are only stored (dg as reciprocals of the pivots),
        // so that no step waits on memory
        double dcur = d[0] - lam, ucur = n > 1 ? e[0] : 0.0;
        for (int r = 0; r + 1 < n; ++r) {
            const double c = e[r], dnext = d[r + 1] - lam, er1 = (r + 2 < n) ? e[r + 1] : 0.0;
            double l, dn, un;
            if (fabs(dcur) >= fabs(c)) {
                dcur = raise(dcur);
                l = c / dcur;
                dg[r] = 1.0 / dcur;
                u1[r] = ucur;
                u2[r] = 0.0;
                pv[r] = 0.0;
                dn = dnext - l * ucur;
                un = er1;
            } else {
                l = dcur / c;
                dg[r] = 1.0 / c;
                u1[r] = dnext;
                u2[r] = er1;
                pv[r] = 1.0;
                dn = ucur - l * dnext;
                un = -l * er1;
            }
            lm[r] = l;
            dcur = dn;
            ucur = un;
        }
        dg[n - 1] = 1.0 / raise(dcur);
        u1[n - 1] = 0.0;
        u2[n - 1] = 0.0;
        for (int r = 0; r < n; ++r) y[r] = start_entry(k, r);
        for (int it = 0; it < 3; ++it) {
            // solve L U x = y in place, the recurrences' operands in registers
            double ycur = y[0];
            for (int r = 0; r + 1 < n; ++r) {
                double ynext = y[r + 1];
                if (pv[r] != 0.0) {
                    const double tmp = ycur;
                    ycur = ynext;
                    ynext = tmp;
                }
                ynext -= lm[r] * ycur;
                y[r] = ycur;
                ycur = ynext;
            }
            y[n - 1] = ycur;
            double y1 = 0.0, y2 = 0.0, mx = 0.0;
            for (int r = n - 1; r >= 0; --r) {
                const double v = (y[r] - u1[r] * y1 - u2[r] * y2) * dg[r];
                y[r] = v;
                y2 = y1;
                y1 = v;
                mx = fmax(mx, fabs(v));
            }
            // scale, orthogonalise against the cluster's earlier members, normalise
            const double sc = mx > 0.0 ? 1.0 / mx : 1.0;
            for (int r = 0; r < n; ++r) y[r] *= sc;
            for (int q = i0; q < k; ++q) {
                double dot = 0.0;
                for (int r = 0; r < n; ++r) dot += Z[(int64_t)r * ldz + q] * y[r];
                for (int r = 0; r < n; ++r) y[r] -= dot * Z[(int64_t)r * ldz + q];
            }
            double nrm = 0.0;
            for (int r = 0; r < n; ++r) nrm += y[r] * y[r];
            nrm = sqrt(nrm);
            const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
            for (int r = 0; r < n; ++r) y[r] *= inv;
        }
        for (int r = 0; r < n; ++r) Z[(int64_t)r * ldz + k] = y[r];
    }
    // Rayleigh quotients z^T T z: the eigenvalues to working accuracy (the
    // bisection stops at its absolute bound); the cluster's members sorted by
    // them (clusters are further apart than either bound, so the whole
    // spectrum stays ascending)
    for (int k = i0; k < i1; ++k) {
        double q = 0.0;
        for (int r = 0; r < n; ++r) {
            const double zr = Z[(int64_t)r * ldz + k];
            q += zr * (d[r] * zr + (r + 1 < n ? 2.0 * e[r] * Z[(int64_t)(r + 1) * ldz + k] : 0.0));
        }
        rq[k] = q;
    }
    for (int k = i0 + 1; k < i1; ++k) {
        for (int q = k; q > i0 && rq[q] < rq[q - 1]; --q) {
            const double tq = rq[q];
            rq[q] = rq[q - 1];
            rq[q - 1] = tq;
            for (int r = 0; r < n; ++r) {
                double *a = Z + (int64_t)r * ldz + q;
                const double tr = a[0];
                a[0] = a[-1];
                a[-1] = tr;
            }
        }
    }
}

template <typename T, int RPT>
__global__ __launch_bounds__(256) void eigh_small_kernel(const cpx<T> *__restrict__ Hin, int64_t ld,
                                                         const int64_t *__restrict__ offs,
                                                         const int32_t *__restrict__ n_in, double *__restrict__ w,
                                                         int64_t ldw, cpx<T> *__restrict__ Vall, int64_t ldv,
                                                         double *__restrict__ work, int cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    const EighLayout lay = eigh_layout<T>(cap, blockDim.x);
    cpx<T> *L = reinterpret_cast<cpx<T> *>(smem + lay.L);
    cpx<T> *v = reinterpret_cast<cpx<T> *>(smem + lay.v);
    cpx<T> *pw = reinterpret_cast<cpx<T> *>(smem + lay.pw);
    cpx<T> *part = reinterpret_cast<cpx<T> *>(smem + lay.part);
    double *d = reinterpret_cast<double *>(smem + lay.d);
    double *e = reinterpret_cast<double *>(smem + lay.e);
    double *e1 = reinterpret_cast<double *>(smem + lay.e1);
    double *red = reinterpret_cast<double *>(smem + lay.red);
    int *cnt = reinterpret_cast<int *>(smem + lay.cnt);
    cpx<T> *refl = reinterpret_cast<cpx<T> *>(smem + lay.refl);
    cpx<T> *alpha = reinterpret_cast<cpx<T> *>(smem + lay.alpha);
    cpx<double> *delta = reinterpret_cast<cpx<double> *>(smem + lay.delta);
    const int64_t u = blockIdx.x;
    const int t = threadIdx.x, nt = blockDim.x;
    double *wu = w + u * ldw;
    cpx<T> *V = Vall + u * ldv * ldv;
    const int n = n_in[u];
    if (n < 0 || n > cap) {
        for (int64_t i = t; i < ldw && i < ld; i += nt) wu[i] = NAN;
        return;
    }
    if (n == 0) return;
    const cpx<T> *H = Hin + (offs ? offs[u] : u * ld * ld);
    for (int c = 0; c < n; ++c) {
        const int base = packed_col(c, n) - c;
        for (int r = c + t; r < n; r += nt) L[base + r] = H[r + (int64_t)c * ld];
    }
    for (int j = t; j < n; j += nt) {
        refl[j] = {T(0), T(0)};
        refl[cap + j] = {T(0), T(0)};
        alpha[j] = {T(0), T(0)};
    }
    __syncthreads();
    tridiag_packed<T>(L, n, cap, v, pw, part, d, e, red, refl, alpha);
    // the unsquared sub-diagonal for the eigenvectors (the bisection squares e)
    for (int i = t; i < n; i += nt) e1[i] = (i + 1 < n) ? e[i] : 0.0;
    if (t == 0) {
        delta[0] = {1.0, 0.0};
        for (int j = 0; j + 1 < n; ++j) {
            const double ar = (double)alpha[j].re, ai = (double)alpha[j].im, m = sqrt(ar * ar + ai * ai);
            const cpx<double> ph = m > 0.0 ? cpx<double>{ar / m, ai / m} : cpx<double>{1.0, 0.0};
            delta[j + 1] = c_mul(delta[j], ph);
        }
    }
    __syncthreads();
    bisect_block(d, e, n, wu, red, cnt);
    __syncthreads();
    // tridiagonal eigenvectors, a cluster per thread
    double tn = 0.0;
    for (int i = 0; i < n; ++i) tn = fmax(tn, fabs(d[i]) + (i > 0 ? e1[i - 1] : 0.0) + e1[i]);
    // eigenvalues closer than this form a cluster (never closer than the
    // bisection's absolute bound, so equal eigenvalues always do)
    const double ortol = fmax(1e-3 * tn, 4.0 * kBisectAbsTol);
    double *Zu = work + u * eigh_work_doubles(cap);
    for (int i = t; i < n; i += nt) {
        if (i > 0 && wu[i] - wu[i - 1] <= ortol) continue;  // not the first of its cluster
        int j = i + 1;
        while (j < n && wu[j] - wu[j - 1] <= ortol) ++j;
        // e (squared by the bisection) is free now: it takes the refined eigenvalues
        cluster_vectors(d, e1, n, wu, i, j, tn, Zu + eigh_zsize(cap) + (int64_t)6 * cap * i, Zu, cap, e);
    }
    __syncthreads();
    for (int i = t; i < n; i += nt) wu[i] = e[i];
    // V = Q D Z with each eigenvector in registers: four lanes per vector,
    // lane `sub` holding rows sub, sub + 4, ...; nt / 4 vectors at a time.
    // Every reflector is read from LDS (lanes of one quarter share the
    // address) and its product with the vector summed over the four lanes.
    constexpr int kRpt = RPT;  // rows per lane: 4 kRpt >= cap
    const int sub = t & 3, vpp = nt >> 2;
    for (int i0 = 0; i0 < n; i0 += vpp) {
        const int i = i0 + (t >> 2);
        const bool live = i < n;
        cpx<T> y[kRpt];
#pragma unroll
        for (int q = 0; q < kRpt; ++q) {
            const int r = sub + 4 * q;
            const double z = (live && r < n) ? Zu[(int64_t)r * cap + i] : 0.0;
            const cpx<double> dl = r < n ? delta[r] : cpx<double>{0.0, 0.0};
            y[q] = {(T)(dl.re * z), (T)(dl.im * z)};
        }
        for (int jj = n - 3; jj >= 0; --jj) {
            const T tau = refl[cap + jj].re;
            if (tau == T(0)) continue;  // uniform: the reflector is the identity
            const int base = packed_col(jj, n) - jj;  // L[base + r] = v_j[r] for rows r > jj + 1
            cpx<T> v[kRpt];
            cpx<T> sp = {T(0), T(0)};
#pragma unroll
            for (int q = 0; q < kRpt; ++q) {
                const int r = sub + 4 * q;
                const bool in = r > jj && r < n;
                const cpx<T> lv = L[in ? (r == jj + 1 ? 0 : base + r) : 0];
                v[q] = in ? (r == jj + 1 ? refl[jj] : lv) : cpx<T>{T(0), T(0)};
                sp = c_add(sp, c_cmul(v[q], y[q]));
            }
            sp.re += __shfl_xor(sp.re, 1, 64);
            sp.im += __shfl_xor(sp.im, 1, 64);
            sp.re += __shfl_xor(sp.re, 2, 64);
            sp.im += __shfl_xor(sp.im, 2, 64);
            const cpx<T> sc = c_scale(tau, sp);
#pragma unroll
            for (int q = 0; q < kRpt; ++q) y[q] = c_sub(y[q], c_mul(v[q], sc));
        }
        if (live) {
#pragma unroll
            for (int q = 0; q < kRpt; ++q) {
                const int r = sub + 4 * q;
                if (r < n) V[(int64_t)i * ldv + r] = y[q];
            }
        }
    }
}

template <typename T>
size_t eigh_small_lds_bytes(int cap) {
    const int threads = cap <= 32 ? 64 : (cap <= 64 ? 128 : 256);
    return eigh_layout<T>(cap, threads).bytes;
}

template <typename T>
hipError_t launch_eigh_small(const cpx<T> *H, int64_t ld, const int64_t *offs, const int32_t *n_in, int64_t batch,
                             double *w, int64_t ldw, cpx<T> *V, int64_t ldv, double *work, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const int cap = (int)ld;
    const int threads = cap <= 32 ? 64 : (cap <= 64 ? 128 : 256);
    const EighLayout lay = eigh_layout<T>(cap, threads);
    // rows per lane of the back-transformation: 32 (sides up to 128) or 45 (up to 180)
    const void *fn = cap <= 128 ? reinterpret_cast<const void *>(eigh_small_kernel<T, 32>)
                                : reinterpret_cast<const void *>(eigh_small_kernel<T, 45>);
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.bytes);
    if (err != hipSuccess) return err;
    if (cap <= 128)
        hipLaunchKernelGGL((eigh_small_kernel<T, 32>), dim3((unsigned)batch), dim3(threads), lay.bytes, s, H, ld, offs,
                           n_in, w, ldw, V, ldv, work, cap);
    else
        hipLaunchKernelGGL((eigh_small_kernel<T, 45>), dim3((unsigned)batch), dim3(threads), lay.bytes, s, H, ld, offs,
                           n_in, w, ldw, V, ldv, work, cap);
    return hipGetLastError();
}

template size_t eigh_small_lds_bytes<double>(int);
template size_t eigh_small_lds_bytes<float>(int);
template hipError_t launch_eigh_small<double>(const cpx<double> *, int64_t, const int64_t *, const int32_t *, int64_t,
                                              double *, int64_t, cpx<double> *, int64_t, double *, hipStream_t);
template hipError_t launch_eigh_small<float>(const cpx<float> *, int64_t, const int64_t *, const int32_t *, int64_t,
                                             double *, int64_t, cpx<float> *, int64_t, double *, hipStream_t);

}  // namespace mlmc
