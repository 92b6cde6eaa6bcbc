// Second derivatives of the NLL in the real parameters x (x_{2a} = Re V_a,
// x_{2a+1} = Im V_a): the error matrix of a fit is the inverse of this matrix
// (Berger, Section 4 on the cost of error calculations).
//
// Data term.  ln I_i = 2 Re ln z_i and ln z_i is holomorphic in V, with
// d2 ln z_i / dV_a dV_c = -A_ia A_ic / z_i^2.  With the complex symmetric
//   T_ac = sum_i A_ia A_ic / z_i^2
// the Hessian of sum_i ln I_i has, per wave pair (a, c), the 2 x 2 block
//   [[-2 Re T_ac, 2 Im T_ac], [2 Im T_ac, 2 Re T_ac]]   (rows x_a, y_a; columns x_c, y_c).
// Normalisation term.  S = V^H M V with the MC matrix M of Eq. 3 (1/N_gen
// folded in, see gram.hip): dS = (2 Re (MV)_a, 2 Im (MV)_a) and d2S has the
// blocks [[2 Re M_ac, -2 Im M_ac], [2 Im M_ac, 2 Re M_ac]].
//   Eq. 2 form:  H = -d2(sum ln I) + N_D (d2S / S - dS dS^T / S^2)
//   Eq. 3 form:  H = -d2(sum ln I) + d2S
//
// One pass over the data rows: each block stages a tile of rows in LDS as
// FP64, forms z and 1/z^2 per row in FP64 and accumulates its share of T;
// the block partials are added in block order, then one block assembles H.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kHThreads = 256;
constexpr int kHRows = 32;
constexpr int kHMaxPer = (PWA_MAX_K * PWA_MAX_K + kHThreads - 1) / kHThreads;

__global__ void hess_clear_kernel(unsigned *flag) { *flag = 0u; }

template <typename T>
__global__ __launch_bounds__(kHThreads) void hess_partial_kernel(const T *__restrict__ A, int64_t n, int64_t ld,
                                                                 int k, const double *__restrict__ V,
                                                                 double *__restrict__ partials,
                                                                 unsigned *__restrict__ flag) {
    __shared__ double tile[kHRows][2 * PWA_MAX_K];
    __shared__ double cw[kHRows][2];          // 1 / z^2 per row (0 for absent rows)
    const int tid = threadIdx.x;
    const int kk = k * k;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;

    double accr[kHMaxPer], acci[kHMaxPer];
#pragma unroll
    for (int m = 0; m < kHMaxPer; ++m) accr[m] = acci[m] = 0.0;
    bool bad = false;

    for (int64_t base = r0; base < r1; base += kHRows) {
        const int rows = (int)(r1 - base < kHRows ? r1 - base : kHRows);
        __syncthreads();
        for (int idx = tid; idx < kHRows * 2 * k; idx += kHThreads) {
            const int r = idx / (2 * k), q = idx % (2 * k);
            tile[r][q] = r < rows ? (double)A[2 * (base + r) * ld + q] : 0.0;
        }
        __syncthreads();
        if (tid < kHRows) {
            double wr = 0.0, wi = 0.0;
            if (tid < rows) {
                double zr = 0.0, zi = 0.0;
                for (int a = 0; a < k; ++a) {
                    const double ar = tile[tid][2 * a], ai = tile[tid][2 * a + 1];
                    zr = fma(V[2 * a], ar, fma(-V[2 * a + 1], ai, zr));
                    zi = fma(V[2 * a], ai, fma(V[2 * a + 1], ar, zi));
                }
                const double I = zr * zr + zi * zi;
                if (I > 0.0 && isfinite(I)) {
                    // 1 / z^2 = conj(z)^2 / I^2
                    const double i2 = 1.0 / (I * I);
                    wr = (zr * zr - zi * zi) * i2;
                    wi = -2.0 * zr * zi * i2;
                } else {
                    bad = true;
                }
            }
            cw[tid][0] = wr;
            cw[tid][1] = wi;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kHMaxPer; ++m) {
            const int e = tid + m * kHThreads;
            if (e >= kk) break;
            const int a = e / k, c = e % k;
            double sr = accr[m], si = acci[m];
            for (int r = 0; r < rows; ++r) {
                const double ar = tile[r][2 * a], ai = tile[r][2 * a + 1];
                const double br = tile[r][2 * c], bi = tile[r][2 * c + 1];
                // A_a A_c, then times 1 / z^2
                const double pr = fma(ar, br, -(ai * bi));
                const double pi = fma(ar, bi, ai * br);
                sr = fma(pr, cw[r][0], fma(-pi, cw[r][1], sr));
                si = fma(pr, cw[r][1], fma(pi, cw[r][0], si));
            }
            accr[m] = sr;
            acci[m] = si;
        }
    }
    if (bad) atomicOr(flag, 1u);
    double *out = partials + (int64_t)blockIdx.x * 2 * kk;
#pragma unroll
    for (int m = 0; m < kHMaxPer; ++m) {
        const int e = tid + m * kHThreads;
        if (e >= kk) break;
        out[2 * e] = accr[m];
        out[2 * e + 1] = acci[m];
    }
}

// T = sum of the block partials in block order.
__global__ void hess_finish_kernel(const double *__restrict__ partials, int nblocks, int k,
                                   double *__restrict__ Tm) {
    const int kk2 = 2 * k * k;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kk2; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * kk2 + e];
        Tm[e] = s;
    }
}

// One block: H (2k x 2k, row-major) from T, M and V; H[2k * 2k] = status flags.
__global__ void hess_assemble_kernel(const double *__restrict__ Tm, const double *__restrict__ M,
                                     const double *__restrict__ V, int k, double nd, int extended,
                                     const unsigned *__restrict__ flag, double *__restrict__ H) {
    __shared__ double mv[2 * PWA_MAX_K];      // M V
    __shared__ double s_S;
    const int tid = threadIdx.x, n2 = 2 * k;
    for (int a = tid; a < k; a += blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < k; ++c) {
            const double mr = M[2 * (a * k + c)], mi = M[2 * (a * k + c) + 1];
            re = fma(mr, V[2 * c], fma(-mi, V[2 * c + 1], re));
            im = fma(mr, V[2 * c + 1], fma(mi, V[2 * c], im));
        }
        mv[2 * a] = re;
        mv[2 * a + 1] = im;
    }
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;                        // S = Re sum_a conj(V_a) (M V)_a
        for (int a = 0; a < k; ++a) s = fma(V[2 * a], mv[2 * a], fma(V[2 * a + 1], mv[2 * a + 1], s));
        s_S = s;
    }
    __syncthreads();
    const double S = s_S;
    for (int idx = tid; idx < n2 * n2; idx += blockDim.x) {
        const int m = idx / n2, n = idx % n2;
        const int a = m >> 1, c = n >> 1, pa = m & 1, pc = n & 1;
        const double tr = Tm[2 * (a * k + c)], ti = Tm[2 * (a * k + c) + 1];
        const double mr = M[2 * (a * k + c)], mi = M[2 * (a * k + c) + 1];
        // block entries of d2(sum ln I) and d2S for (x or y of a, x or y of c)
        double hl, d2s;
        if (!pa && !pc) { hl = -2.0 * tr; d2s = 2.0 * mr; }
        else if (!pa && pc) { hl = 2.0 * ti; d2s = -2.0 * mi; }
        else if (pa && !pc) { hl = 2.0 * ti; d2s = 2.0 * mi; }
        else { hl = 2.0 * tr; d2s = 2.0 * mr; }
        double h;
        if (extended) {
            h = -hl + d2s;
        } else if (nd == 0.0) {
            h = 0.0;
        } else {
            const double dsm = 2.0 * mv[m], dsn = 2.0 * mv[n];     // dS: (2 Re MV, 2 Im MV) interleaved
            h = -hl + nd * (d2s / S - dsm * dsn / (S * S));
        }
        H[idx] = h;
    }
    if (tid == 0) {
        const bool dom = (*flag != 0u) || (!extended && nd > 0.0 && !(S > 0.0));
        H[n2 * n2] = dom ? 1.0 : 0.0;
    }
}

}  // namespace

size_t hessian_partial_doubles(int k, int blocks) { return (size_t)blocks * 2 * k * k; }

hipError_t launch_hessian(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, const double *V_dev,
                          const double *M, double nd, int extended, double *partials, int blocks, double *Tm,
                          unsigned *flag, double *H, hipStream_t stream) {
    if (k < 1 || k > PWA_MAX_K || blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hess_clear_kernel, dim3(1), dim3(1), 0, stream, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > 0) {
        if (prec == PWA_F32)
            hipLaunchKernelGGL(hess_partial_kernel<float>, dim3(blocks), dim3(kHThreads), 0, stream,
                               static_cast<const float *>(A), n, ld, k, V_dev, partials, flag);
        else
            hipLaunchKernelGGL(hess_partial_kernel<double>, dim3(blocks), dim3(kHThreads), 0, stream,
                               static_cast<const double *>(A), n, ld, k, V_dev, partials, flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        blocks = 0;
    }
    const int kk2 = 2 * k * k;
    hipLaunchKernelGGL(hess_finish_kernel, dim3((kk2 + 255) / 256), dim3(256), 0, stream, partials, blocks, k, Tm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(hess_assemble_kernel, dim3(1), dim3(256), 0, stream, Tm, M, V_dev, k, nd, extended, flag, H);
    return hipGetLastError();
}

}  // namespace pwa
