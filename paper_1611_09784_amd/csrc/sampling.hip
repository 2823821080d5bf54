// Vacancy outcomes (Philox4x64-10), control-variate partition and k-grids.
#include "internal.hpp"

namespace mlmc {

// Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw, SC'11): ten
// rounds of two 64x64->128 multiplies with a Weyl-sequence key schedule.
__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ULL, kMul1 = 0xCA5A826395121157ULL;
    constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ULL, kWeyl1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += kWeyl0;
            k1 += kWeyl1;
        }
        const uint64_t hi0 = __umul64hi(kMul0, x[0]), lo0 = kMul0 * x[0];
        const uint64_t hi1 = __umul64hi(kMul1, x[2]), lo1 = kMul1 * x[2];
        const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
    }
}

// One thread per (sample, block of four groups).  The first sample index is
// `first`, plus *first_dev when that is given (a device-resident counter).
__global__ void sample_vacancies_kernel(const uint8_t *__restrict__ removable, int G, int64_t groups,
                                        int64_t blocks_per_sample, uint64_t threshold, uint64_t seed, uint64_t tag,
                                        int64_t first, const int64_t *__restrict__ first_dev, int64_t n_samples,
                                        uint8_t *__restrict__ mask) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_samples * blocks_per_sample) return;
    if (first_dev) first += *first_dev;
    const int64_t s = t / blocks_per_sample, blk = t % blocks_per_sample;
    uint64_t x[4] = {(uint64_t)(first + s), (uint64_t)blk, 0, 0};
    philox4x64_10(x, seed, tag);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int64_t g = blk * 4 + w;
        if (g < groups) {
            const int local = (int)(g % G);
            mask[s * groups + g] = (uint8_t)(removable[local] && (x[w] >> 11) < threshold);
        }
    }
}

hipError_t launch_sample_vacancies(const DevLattice &lat, int N, uint64_t threshold, uint64_t seed, uint64_t tag,
                                   int64_t first, int64_t n_samples, uint8_t *mask, hipStream_t s,
                                   const int64_t *first_dev) {
    const int64_t groups = (int64_t)N * N * lat.n_groups;
    const int64_t bps = (groups + 3) / 4;
    const int64_t total = n_samples * bps;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (total + threads - 1) / threads;
    hipLaunchKernelGGL(sample_vacancies_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, lat.removable,
                       lat.n_groups, groups, bps, threshold, seed, tag, first, first_dev, n_samples, mask);
    return hipGetLastError();
}

// *counter += delta (one thread).
__global__ void advance_counter_kernel(int64_t *counter, int64_t delta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter += delta;
}

hipError_t launch_advance_counter(int64_t *counter, int64_t delta, hipStream_t s) {
    hipLaunchKernelGGL(advance_counter_kernel, dim3(1), dim3(64), 0, s, counter, delta);
    return hipGetLastError();
}

// Quarter q = 2*qi + qj of each N x N outcome, as an N/2 supercell.
__global__ void partition_kernel(int N, int G, const uint8_t *__restrict__ mask, int64_t n_samples,
                                 uint8_t *__restrict__ quarters) {
    const int h = N / 2;
    const int64_t per_sample = (int64_t)4 * h * h * G;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_samples * per_sample) return;
    const int64_t s = t / per_sample;
    int64_t r = t % per_sample;
    const int g = (int)(r % G);
    r /= G;
    const int jj = (int)(r % h);
    r /= h;
    const int ii = (int)(r % h);
    const int q = (int)(r / h);
    const int qi = q >> 1, qj = q & 1;
    const int64_t src = ((int64_t)(qi * h + ii) * N + (qj * h + jj)) * G + g;
    quarters[t] = mask[s * (int64_t)N * N * G + src];
}

hipError_t launch_partition(int N, int G, const uint8_t *mask, int64_t n_samples, uint8_t *quarters, hipStream_t s) {
    const int64_t total = n_samples * (int64_t)N * N * G;
    if (total == 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(partition_kernel, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, N, G,
                       mask, n_samples, quarters);
    return hipGetLastError();
}

__global__ void kgrid_kernel(int kind, int K, double *__restrict__ kred, double *__restrict__ kweight) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (kind == MLMC_KGRID_RHOMBI) {
        // point t = a*K + j: a in [0, 3K), b = (-a mod 3) + 3j, kappa = (a, b) / (3K)
        const int M3 = 3 * K;
        if (t >= M3 * K) return;
        const int a = t / K, j = t % K;
        const int b = (3 - a % 3) % 3 + 3 * j;
        kred[2 * t] = (double)a / (double)M3;
        kred[2 * t + 1] = (double)b / (double)M3;
        kweight[t] = 1.0 / ((double)M3 * (double)K);
        return;
    }
    if (t >= K * K) return;
    const int r1 = t / K, r2 = t % K;
    if (kind == MLMC_KGRID_MP) {
        kred[2 * t] = (2.0 * r1 - K + 1.0) / (2.0 * K);
        kred[2 * t + 1] = (2.0 * r2 - K + 1.0) / (2.0 * K);
    } else {
        kred[2 * t] = (double)r1 / K;
        kred[2 * t + 1] = (double)r2 / K;
    }
    kweight[t] = 1.0 / ((double)K * (double)K);
}

int kgrid_count(int kind, int K) { return kind == MLMC_KGRID_RHOMBI ? 3 * K * K : K * K; }

hipError_t launch_kgrid(int kind, int K, double *kred, double *kweight, hipStream_t s) {
    const int threads = 256;
    const int blocks = (kgrid_count(kind, K) + threads - 1) / threads;
    hipLaunchKernelGGL(kgrid_kernel, dim3(blocks), dim3(threads), 0, s, kind, K, kred, kweight);
    return hipGetLastError();
}

}  // namespace mlmc
