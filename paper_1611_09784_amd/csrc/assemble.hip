// H(k) assembly into device memory (column-major; full Hermitian storage, or
// the lower triangle only for the eigensolvers, which read nothing else).
#include "device_common.hpp"

namespace mlmc {

// One workgroup per (outcome s, k-point k) unit u = s*n_k + k.
// With unit_diag the matrix starts from the identity (the overlap S(k) of a
// non-orthogonal basis, whose table the caller passes in place of the hops).
// With lower only entries (r, c), r >= c, are written.
template <typename T>
__global__ __launch_bounds__(256) void assemble_kernel(DevLattice lat, int N, const uint8_t *__restrict__ masks,
                                                       const double *__restrict__ kred, int n_k, cpx<T> *__restrict__ Hall,
                                                       int64_t ld, int32_t *__restrict__ n_out, int unit_diag,
                                                       int lower) {
    extern __shared__ __align__(16) unsigned char smem[];
    int *scan = reinterpret_cast<int *>(smem);
    int *idx = scan + 32;
    const int64_t u = blockIdx.x;
    const int64_t s = u / n_k;
    const int k = (int)(u % n_k);
    const int G = lat.n_groups;
    const int total = N * N * lat.n_orb;
    const int n = build_present_index(masks + s * (int64_t)N * N * G, lat.orb_group, lat.n_orb, G, total, idx, scan);
    cpx<T> *H = Hall + u * ld * ld;
    const int64_t nn = (int64_t)n * n;
    for (int64_t q = threadIdx.x; q < nn; q += blockDim.x) {
        const int64_t c = q / n, r = q - c * n;
        if (!lower || r >= c) H[r + c * ld] = {(unit_diag && r == c) ? T(1) : T(0), T(0)};
    }
    __syncthreads();
    walk_hops(lat, N, kred[2 * k], kred[2 * k + 1], idx,
              [&](int pass, int a, int b, cpx<double> z, cpx<double> amp, bool onsite) {
                  if (pass == 0) {
                      if (lower && a < b) return;
                      cpx<T> &h = H[a + (int64_t)b * ld];
                      if (onsite) {
                          h.re += (T)amp.re;
                      } else {
                          h.re += (T)z.re;
                          h.im += (T)z.im;
                      }
                  } else if (!onsite) {
                      if (lower && b < a) return;
                      cpx<T> &h = H[b + (int64_t)a * ld];
                      h.re += (T)z.re;
                      h.im -= (T)z.im;
                  }
              });
    if (threadIdx.x == 0) n_out[u] = n;
}

template <typename T>
hipError_t launch_assemble(const DevLattice &lat, int N, const uint8_t *masks, int64_t n_samples, const double *kred,
                           int n_k, cpx<T> *H, int64_t ld, int32_t *n_out, hipStream_t s, bool overlap, bool lower) {
    const int64_t units = n_samples * n_k;
    if (units == 0) return hipSuccess;
    DevLattice tab = lat;
    if (overlap) {  // S(k): identity plus the Bloch sum of the overlap table
        tab.hop_i = lat.ovl_i;
        tab.hop_f = lat.ovl_f;
        tab.n_hops = lat.n_ovl;
    }
    const size_t lds = sizeof(int) * (32 + (size_t)N * N * lat.n_orb);
    hipLaunchKernelGGL(assemble_kernel<T>, dim3((unsigned)units), dim3(256), lds, s, tab, N, masks, kred, n_k, H, ld,
                       n_out, overlap ? 1 : 0, lower ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_assemble<double>(const DevLattice &, int, const uint8_t *, int64_t, const double *, int,
                                            cpx<double> *, int64_t, int32_t *, hipStream_t, bool, bool);
template hipError_t launch_assemble<float>(const DevLattice &, int, const uint8_t *, int64_t, const double *, int,
                                           cpx<float> *, int64_t, int32_t *, hipStream_t, bool, bool);

}  // namespace mlmc
