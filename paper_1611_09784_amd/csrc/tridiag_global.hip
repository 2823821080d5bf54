// One-stage Householder tridiagonalisation of Hermitian matrices held in
// device memory (full storage, column-major), one workgroup per matrix.
//
// Step j applies the pending reflector j-1 lazily: column j is brought up to
// date first, reflector j is formed from it, and a single pass over the
// trailing block both applies reflector j-1 (A <- A - v w^H - w v^H) and
// accumulates p = A v_j.  Each trailing element is therefore read and written
// once per step.  Threads own rows (coalesced along columns); four column
// groups produce partial products that are summed in a fixed order.
#include "device_common.hpp"

namespace mlmc {

constexpr int kRowLanes = 128;
constexpr int kColGroups = 4;
constexpr int kGlobalThreads = kRowLanes * kColGroups;

template <typename T>
size_t tridiag_global_partial_elems(int64_t ld) {
    return (size_t)kColGroups * (size_t)ld;
}

template <typename T>
__global__ __launch_bounds__(kGlobalThreads) void tridiag_global_kernel(cpx<T> *__restrict__ Hall, int64_t ld,
                                                                        const int32_t *__restrict__ n_in,
                                                                        double *__restrict__ dall,
                                                                        double *__restrict__ eall, int64_t lde,
                                                                        cpx<T> *__restrict__ partial_all) {
    extern __shared__ __align__(16) unsigned char smem[];
    cpx<T> *slot0 = reinterpret_cast<cpx<T> *>(smem);
    cpx<T> *slot1 = slot0 + ld;
    cpx<T> *slot2 = slot1 + ld;
    double *red = reinterpret_cast<double *>(slot2 + ld);
    const int64_t u = blockIdx.x;
    const int n = n_in[u];
    double *d = dall + u * lde;
    double *e = eall + u * lde;
    const int t = threadIdx.x, nt = blockDim.x;
    if (n < 0 || n > ld) {
        for (int64_t i = t; i < lde; i += nt) d[i] = NAN;
        return;
    }
    cpx<T> *H = Hall + u * ld * ld;
    cpx<T> *part = partial_all + u * (int64_t)kColGroups * ld;
    cpx<T> *vp = slot0, *wp = slot1, *vc = slot2;  // pending (v, w) and current v
    bool pending = false;
    const int lane_r = t % kRowLanes, cg = t / kRowLanes;
    for (int j = 0; j + 2 < n; ++j) {
        const int m = n - j - 1;
        // Column j (rows j..n-1) up to date; x = rows j+1.. goes to vc.
        double np = 0.0;
        for (int r = j + t; r < n; r += nt) {
            cpx<T> a = H[r + (int64_t)j * ld];
            if (pending) a = c_sub(a, c_add(c_mulc(vp[r], wp[j]), c_mulc(wp[r], vp[j])));
            if (r == j) {
                d[j] = (double)a.re;
            } else {
                vc[r] = a;
                np += (double)c_abs2(a);
            }
        }
        const double nrm2 = block_sum(np, red);
        const double xnorm = sqrt(nrm2);
        const cpx<T> x0 = vc[j + 1];
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
        if (t == 0) e[j] = xnorm;
        __syncthreads();
        if (t == 0) vc[j + 1] = v0;
        __syncthreads();
        // Fused pass over the trailing block: apply reflector j-1, accumulate A v_j.
        const int chunk = (m + kColGroups - 1) / kColGroups;
        const int c_begin = j + 1 + cg * chunk;
        const int c_end = min(n, c_begin + chunk);
        for (int r = j + 1 + lane_r; r < n; r += kRowLanes) {
            cpx<T> vpr = {T(0), T(0)}, wpr = {T(0), T(0)};
            if (pending) {
                vpr = vp[r];
                wpr = wp[r];
            }
            cpx<T> acc = {T(0), T(0)};
            cpx<T> *col = H + r;
            if (pending) {
#pragma unroll 4
                for (int c = c_begin; c < c_end; ++c) {
                    cpx<T> a = col[(int64_t)c * ld];
                    a = c_sub(a, c_add(c_mulc(vpr, wp[c]), c_mulc(wpr, vp[c])));
                    col[(int64_t)c * ld] = a;
                    acc = c_add(acc, c_mul(a, vc[c]));
                }
            } else {
#pragma unroll 4
                for (int c = c_begin; c < c_end; ++c) acc = c_add(acc, c_mul(col[(int64_t)c * ld], vc[c]));
            }
            part[(int64_t)cg * ld + r] = acc;
        }
        __syncthreads();
        // p = tau * sum of partials; w = p - (tau/2)(v^H p) v  (written over vp).
        double kp = 0.0;
        for (int r = j + 1 + t; r < n; r += nt) {
            cpx<T> s = part[r];
#pragma unroll
            for (int g = 1; g < kColGroups; ++g) s = c_add(s, part[(int64_t)g * ld + r]);
            const cpx<T> p = c_scale(tau, s);
            vp[r] = p;
            kp += (double)vc[r].re * (double)p.re + (double)vc[r].im * (double)p.im;
        }
        const double vhp = block_sum(kp, red);
        const T K = (T)(0.5 * (double)tau * vhp);
        for (int r = j + 1 + t; r < n; r += nt) vp[r] = c_sub(vp[r], c_scale(K, vc[r]));
        __syncthreads();
        cpx<T> *w_new = vp, *free_slot = wp;
        vp = vc;
        wp = w_new;
        vc = free_slot;
        pending = true;
    }
    if (t == 0) {
        if (n >= 2) {
            const int j = n - 2;
            cpx<T> a00 = H[j + (int64_t)j * ld], a10 = H[j + 1 + (int64_t)j * ld], a11 = H[j + 1 + (int64_t)(j + 1) * ld];
            if (pending) {
                a00 = c_sub(a00, c_add(c_mulc(vp[j], wp[j]), c_mulc(wp[j], vp[j])));
                a10 = c_sub(a10, c_add(c_mulc(vp[j + 1], wp[j]), c_mulc(wp[j + 1], vp[j])));
                a11 = c_sub(a11, c_add(c_mulc(vp[j + 1], wp[j + 1]), c_mulc(wp[j + 1], vp[j + 1])));
            }
            d[j] = (double)a00.re;
            e[j] = sqrt((double)c_abs2(a10));
            d[j + 1] = (double)a11.re;
        } else if (n == 1) {
            d[0] = (double)H[0].re;
        }
    }
}

template <typename T>
hipError_t launch_tridiag_global(cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *d, double *e,
                                 int64_t lde, cpx<T> *partial, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    const size_t lds = 3 * sizeof(cpx<T>) * (size_t)ld + 32 * sizeof(double);
    auto kern = tridiag_global_kernel<T>;
    hipError_t err =
        hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)batch), dim3(kGlobalThreads), lds, s, H, ld, n_in, d, e, lde, partial);
    return hipGetLastError();
}

template size_t tridiag_global_partial_elems<double>(int64_t);
template size_t tridiag_global_partial_elems<float>(int64_t);
template hipError_t launch_tridiag_global<double>(cpx<double> *, int64_t, const int32_t *, int64_t, double *, double *,
                                                  int64_t, cpx<double> *, hipStream_t);
template hipError_t launch_tridiag_global<float>(cpx<float> *, int64_t, const int32_t *, int64_t, double *, double *,
                                                 int64_t, cpx<float> *, hipStream_t);

}  // namespace mlmc
