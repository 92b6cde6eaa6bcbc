// Checks of caller-owned samples that the library uses in place (borrowed
// device arrays): the padding columns of every row must be zero, because the
// kernels read whole rows of the device layout and weight the padding by the
// zero entries of V (a non-finite padding value would still reach the sums).
#include "internal.hpp"

namespace pwa {
namespace {

// Counts rows whose columns [k, ld) hold a nonzero value (real or imaginary
// part); one thread per (row, padding column) pair, grid-stride.
template <typename T>
__global__ __launch_bounds__(256) void pad_check_kernel(const T *A, int64_t n, int64_t ld, int k,
                                                        unsigned *bad) {
    const int64_t pad = ld - k;
    const int64_t total = n * pad;
    unsigned found = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / pad, col = k + i % pad;
        const T *e = A + 2 * (row * ld + col);
        found |= (e[0] != T(0) || e[1] != T(0)) ? 1u : 0u;
    }
    if (found) atomicOr(bad, 1u);
}

}  // namespace

hipError_t launch_pad_check(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, unsigned *bad,
                            hipStream_t stream) {
    if (n == 0 || ld == k) return hipSuccess;
    const int64_t total = n * (ld - k);
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
    if (prec == PWA_F32)
        hipLaunchKernelGGL(pad_check_kernel<float>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<const float *>(A), n, ld, k, bad);
    else
        hipLaunchKernelGGL(pad_check_kernel<double>, dim3(blocks), dim3(256), 0, stream,
                           static_cast<const double *>(A), n, ld, k, bad);
    return hipGetLastError();
}

}  // namespace pwa
