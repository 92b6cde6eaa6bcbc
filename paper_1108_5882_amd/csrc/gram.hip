// MC integral matrix of the expanded likelihood (Berger, Section 2, Eq. 3):
//   M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb
// While only the production amplitudes V vary, M is fixed; each evaluation
// then needs S = V^H M V and M V (O(k^2)) instead of a pass over the MC rows.
//
// Built once per MC sample: every block stages a tile of rows in LDS as FP64,
// each thread owns a few (a, b) entries and accumulates in FP64 (products of
// FP32 amplitudes are exact in FP64).  A second kernel adds the block partials
// in block order and divides by N_gen.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kGramThreads = 256;
constexpr int kGramRows = 32;
constexpr int kGramMaxPer = (PWA_MAX_K * PWA_MAX_K + kGramThreads - 1) / kGramThreads;

template <typename T>
__global__ __launch_bounds__(kGramThreads) void gram_partial_kernel(const T *__restrict__ A,
                                                                    const T *__restrict__ w,
                                                                    int64_t n, int64_t ld, int k,
                                                                    double *__restrict__ partials) {
    __shared__ double tile[kGramRows][2 * PWA_MAX_K];
    __shared__ double tw[kGramRows];
    const int tid = threadIdx.x;
    const int kk = k * k;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;

    double accr[kGramMaxPer], acci[kGramMaxPer];
#pragma unroll
    for (int m = 0; m < kGramMaxPer; ++m) accr[m] = acci[m] = 0.0;

    for (int64_t base = r0; base < r1; base += kGramRows) {
        const int rows = (int)(r1 - base < kGramRows ? r1 - base : kGramRows);
        __syncthreads();
        for (int idx = tid; idx < kGramRows * 2 * k; idx += kGramThreads) {
            const int r = idx / (2 * k), q = idx % (2 * k);
            tile[r][q] = r < rows ? (double)A[2 * (base + r) * ld + q] : 0.0;
        }
        for (int r = tid; r < kGramRows; r += kGramThreads)
            tw[r] = r < rows ? (w ? (double)w[base + r] : 1.0) : 0.0;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kGramMaxPer; ++m) {
            const int e = tid + m * kGramThreads;
            if (e >= kk) break;
            const int a = e / k, b = e % k;
            double sr = accr[m], si = acci[m];
            for (int r = 0; r < rows; ++r) {
                const double ar = tile[r][2 * a], ai = tile[r][2 * a + 1];
                const double br = tile[r][2 * b], bi = tile[r][2 * b + 1];
                // conj(A_a) A_b = (ar br + ai bi) + i (ar bi - ai br)
                const double pr = fma(ar, br, ai * bi);
                const double pi = fma(ar, bi, -(ai * br));
                sr = fma(tw[r], pr, sr);
                si = fma(tw[r], pi, si);
            }
            accr[m] = sr;
            acci[m] = si;
        }
    }
    double *out = partials + (int64_t)blockIdx.x * 2 * kk;
#pragma unroll
    for (int m = 0; m < kGramMaxPer; ++m) {
        const int e = tid + m * kGramThreads;
        if (e >= kk) break;
        out[2 * e] = accr[m];
        out[2 * e + 1] = acci[m];
    }
}

__global__ void gram_finish_kernel(const double *__restrict__ partials, int nblocks, int k,
                                   double inv_ngen, double *__restrict__ M) {
    const int kk2 = 2 * k * k;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kk2; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * kk2 + e];
        M[e] = s * inv_ngen;
    }
}

}  // namespace

size_t gram_partial_doubles(int k, int blocks) { return (size_t)blocks * 2 * k * k; }

hipError_t launch_gram(pwa_prec prec, const void *A, const void *w, int64_t n, int64_t ld, int k,
                       double n_gen, double *partials, int blocks, double *M, hipStream_t stream) {
    if (k < 1 || k > PWA_MAX_K || blocks < 1) return hipErrorInvalidValue;
    if (prec == PWA_F32)
        hipLaunchKernelGGL(gram_partial_kernel<float>, dim3(blocks), dim3(kGramThreads), 0, stream,
                           static_cast<const float *>(A), static_cast<const float *>(w), n, ld, k,
                           partials);
    else
        hipLaunchKernelGGL(gram_partial_kernel<double>, dim3(blocks), dim3(kGramThreads), 0, stream,
                           static_cast<const double *>(A), static_cast<const double *>(w), n, ld, k,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int kk2 = 2 * k * k;
    hipLaunchKernelGGL(gram_finish_kernel, dim3((kk2 + 255) / 256), dim3(256), 0, stream, partials,
                       blocks, k, 1.0 / n_gen, M);
    return hipGetLastError();
}

}  // namespace pwa
