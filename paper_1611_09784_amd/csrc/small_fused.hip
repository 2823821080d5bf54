// Fused LDS-resident path for small supercells: one workgroup per H(k).
// The matrix is assembled (or loaded) straight into a packed lower triangle
// in LDS, reduced to tridiagonal form there, and its eigenvalues found by
// Sturm bisection in the same workgroup; H never touches device memory.
#include "device_common.hpp"

namespace mlmc {

struct SmallLayout {
    size_t L, v, pw, part, d, e, red, cnt, idx, scan, bytes;
};

template <typename T>
__host__ __device__ inline SmallLayout small_layout(int cap, int threads) {
    SmallLayout o{};
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
    o.red = take(sizeof(double) * 32);
    o.cnt = take(sizeof(int) * (size_t)(threads + 1));
    o.idx = take(sizeof(int) * (size_t)cap);
    o.scan = take(sizeof(int) * 32);
    o.bytes = p;
    return o;
}

template <typename T, bool FROM_LATTICE>
__global__ __launch_bounds__(256) void small_eig_kernel(DevLattice lat, int N, const uint8_t *__restrict__ masks,
                                                        const double *__restrict__ kred, int n_k,
                                                        const cpx<T> *__restrict__ Hin, int64_t ld,
                                                        const int64_t *__restrict__ offs,
                                                        const int32_t *__restrict__ n_in, double *__restrict__ w,
                                                        int64_t ldw, int32_t *__restrict__ n_out, int cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    const SmallLayout lay = small_layout<T>(cap, blockDim.x);
    cpx<T> *L = reinterpret_cast<cpx<T> *>(smem + lay.L);
    cpx<T> *v = reinterpret_cast<cpx<T> *>(smem + lay.v);
    cpx<T> *pw = reinterpret_cast<cpx<T> *>(smem + lay.pw);
    cpx<T> *part = reinterpret_cast<cpx<T> *>(smem + lay.part);
    double *d = reinterpret_cast<double *>(smem + lay.d);
    double *e = reinterpret_cast<double *>(smem + lay.e);
    double *red = reinterpret_cast<double *>(smem + lay.red);
    int *cnt = reinterpret_cast<int *>(smem + lay.cnt);
    const int64_t u = blockIdx.x;
    double *wu = w + u * ldw;
    int n;
    if constexpr (FROM_LATTICE) {
        int *idx = reinterpret_cast<int *>(smem + lay.idx);
        int *scan = reinterpret_cast<int *>(smem + lay.scan);
        const int64_t s = u / n_k;
        const int k = (int)(u % n_k);
        const int G = lat.n_groups;
        n = build_present_index(masks + s * (int64_t)N * N * G, lat.orb_group, lat.n_orb, G, N * N * lat.n_orb, idx,
                                scan);
        for (int q = threadIdx.x; q < packed_size(n); q += blockDim.x) L[q] = {T(0), T(0)};
        __syncthreads();
        // Lower-triangle accumulation: a hop term lands on (max(a,b), min(a,b));
        // pass 0 takes a >= b, pass 1 takes a < b, so two cells that reach the
        // same element (possible when 2R = 0 mod N) are in different passes.
        walk_hops(lat, N, kred[2 * k], kred[2 * k + 1], idx,
                  [&](int pass, int a, int b, cpx<double> z, cpx<double> amp, bool onsite) {
                      if (pass == 0 && a >= b) {
                          cpx<T> &h = L[packed_col(b, n) + a - b];
                          if (onsite) {
                              h.re += (T)amp.re;
                          } else if (a == b) {
                              h.re += (T)(2.0 * z.re);
                          } else {
                              h.re += (T)z.re;
                              h.im += (T)z.im;
                          }
                      } else if (pass == 1 && a < b) {
                          cpx<T> &h = L[packed_col(a, n) + b - a];
                          h.re += (T)z.re;
                          h.im -= (T)z.im;
                      }
                  });
        if (threadIdx.x == 0) n_out[u] = n;
    } else {
        n = n_in[u];
        if (n < 0 || n > cap) {
            for (int64_t i = threadIdx.x; i < ldw && i < ld; i += blockDim.x) wu[i] = NAN;
            return;
        }
        const cpx<T> *H = Hin + (offs ? offs[u] : u * ld * ld);
        for (int c = 0; c < n; ++c) {
            const int base = packed_col(c, n) - c;
            for (int r = c + threadIdx.x; r < n; r += blockDim.x) L[base + r] = H[r + (int64_t)c * ld];
        }
        __syncthreads();
    }
    tridiag_packed<T>(L, n, cap, v, pw, part, d, e, red);
    bisect_block(d, e, n, wu, red, cnt);
}

template <typename T>
static int small_threads(int cap) {
    return cap <= 32 ? 64 : (cap <= 64 ? 128 : 256);
}

template <typename T, bool FROM_LATTICE>
static hipError_t launch_small(int64_t units, int cap, hipStream_t s, DevLattice lat, int N, const uint8_t *masks,
                               const double *kred, int n_k, const cpx<T> *Hin, int64_t ld, const int32_t *n_in,
                               double *w, int64_t ldw, int32_t *n_out, const int64_t *offs = nullptr) {
    if (units == 0) return hipSuccess;
    const int threads = small_threads<T>(cap);
    const SmallLayout lay = small_layout<T>(cap, threads);
    auto kern = small_eig_kernel<T, FROM_LATTICE>;
    hipError_t err = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lay.bytes);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(kern, dim3((unsigned)units), dim3(threads), lay.bytes, s, lat, N, masks, kred, n_k, Hin, ld,
                       offs, n_in, w, ldw, n_out, cap);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_small_from_lattice(const DevLattice &lat, int N, const uint8_t *masks, int64_t n_samples,
                                     const double *kred, int n_k, double *w, int64_t ldw, int32_t *n_out,
                                     hipStream_t s) {
    const int cap = N * N * lat.n_orb;
    return launch_small<T, true>(n_samples * n_k, cap, s, lat, N, masks, kred, n_k, nullptr, 0, nullptr, w, ldw,
                                 n_out);
}

template <typename T>
hipError_t launch_small_from_matrix(const cpx<T> *H, int64_t ld, const int32_t *n_in, int64_t batch, double *w,
                                    int64_t ldw, hipStream_t s, const int64_t *offs) {
    DevLattice none{};
    return launch_small<T, false>(batch, (int)ld, s, none, 0, nullptr, nullptr, 1, H, ld, n_in, w, ldw, nullptr, offs);
}

template hipError_t launch_small_from_lattice<double>(const DevLattice &, int, const uint8_t *, int64_t,
                                                      const double *, int, double *, int64_t, int32_t *,
                                                      hipStream_t);
template hipError_t launch_small_from_lattice<float>(const DevLattice &, int, const uint8_t *, int64_t,
                                                     const double *, int, double *, int64_t, int32_t *, hipStream_t);
template hipError_t launch_small_from_matrix<double>(const cpx<double> *, int64_t, const int32_t *, int64_t, double *,
                                                     int64_t, hipStream_t, const int64_t *);
template hipError_t launch_small_from_matrix<float>(const cpx<float> *, int64_t, const int32_t *, int64_t, double *,
                                                    int64_t, hipStream_t, const int64_t *);

}  // namespace mlmc
