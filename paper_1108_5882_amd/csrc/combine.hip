// Final combination of the likelihood kernel's block partials (Berger,
// Section 2, Eq. 2 and 3; the double-precision final sum of the paper's
// precision remark).
//
// One block adds the FP64 partials of the data blocks and of the MC blocks in
// a fixed order (a group of threads per column, each striding the blocks,
// then the group's sums in thread order), so the result is bitwise
// reproducible, and then forms
//   Eq. 2 form:  NLL = -sum ln I + N_D ln S,        c = N_D / (N_gen S)
//   Eq. 3 form:  NLL = -sum ln I + S,                c = 1 / N_gen
//   gradient     = 2 (-G + c H)   (real parts, imaginary parts interleaved)
// with G = sum conj(A) z / I over data rows and H = sum w conj(A) z over MC
// rows, or, with the precomputed MC matrix M (1/N_gen folded in),
// S = V^H M V and H replaced by M V with N_gen = 1.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kCombineThreads = 1024;
constexpr int kMaxCols = 2 * (1 + 2 * PWA_MAX_K);
constexpr int kUnroll = 8;

__global__ __launch_bounds__(kCombineThreads) void nll_combine_kernel(StreamArgs p,
                                                                      double log_scale) {
    __shared__ double tot[kMaxCols];
    __shared__ double mv[2 * PWA_MAX_K];
    __shared__ double s_c;
    __shared__ double part[kCombineThreads];
    const int tid = threadIdx.x;
    const int ps = p.pstride;
    const int ncol = 2 * ps;                        // data columns, then MC columns
    const int nbt = p.nb[0] + p.nb[1];
    // tpc threads per column; thread t' of a column adds blocks t', t' + tpc, ...
    // with kUnroll independent accumulators (loads clamped into the column and
    // masked, so all of them are in flight at once), then the tpc sums of a
    // column are added in thread order: a fixed order throughout.
    const int tpc = kCombineThreads / ncol;         // >= 3 since ncol <= 258
    if (tid < tpc * ncol) {
        const int col = tid / tpc, tp = tid % tpc;
        const int sg = col < ps ? 0 : 1;
        const int cc = col - sg * ps;
        const int nb = p.nb[sg];
        const double *src = p.partials + (int64_t)cc * nbt + (sg ? p.nb[0] : 0);
        double acc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc[u] = 0.0;
        for (int b0 = tp; b0 < nb; b0 += kUnroll * tpc) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int b = b0 + u * tpc;
                const double v = src[b < nb ? b : nb - 1];
                acc[u] += b < nb ? v : 0.0;
            }
        }
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) s += acc[u];
        part[tid] = s;
    }
    __syncthreads();
    for (int col = tid; col < ncol; col += kCombineThreads) {
        double s = 0.0;
        for (int tp = 0; tp < tpc; ++tp) s += part[col * tpc + tp];
        tot[col] = s;
    }
    __syncthreads();

    const int k = p.k;
    const double *V = p.v_dev ? p.v_dev : p.v_arg;
    if (p.gram) {
        for (int a = tid; a < k; a += kCombineThreads) {
            double r = 0.0, i = 0.0;
            for (int b = 0; b < k; ++b) {
                const double mr = p.gram[2 * (a * k + b)], mi = p.gram[2 * (a * k + b) + 1];
                r += mr * V[2 * b] - mi * V[2 * b + 1];
                i += mr * V[2 * b + 1] + mi * V[2 * b];
            }
            mv[2 * a] = r;
            mv[2 * a + 1] = i;
        }
        __syncthreads();
    }
    const double *td = tot;          // data: [0] sum log, [1 + i] G
    const double *tm = tot + ps;     // MC:   [0] sum w I, [1 + i] H
    if (tid == 0) {
        const double nd = p.nd_total;
        const double sum_log = td[0] * log_scale;
        double S, c;
        if (p.gram) {
            double s = 0.0;
            for (int a = 0; a < k; ++a) s += V[2 * a] * mv[2 * a] + V[2 * a + 1] * mv[2 * a + 1];
            S = s;                                  // Re V^H (M V)
            c = p.extended ? 1.0 : nd / S;
        } else {
            S = tm[0] / p.n_gen;
            c = p.extended ? 1.0 / p.n_gen : nd / tm[0];
        }
        double nll;
        unsigned flags = 0;
        if (!p.extended && nd == 0.0) {
            nll = 0.0;                              // empty product: ln L = 0
            c = 0.0;
        } else {
            nll = p.extended ? -sum_log + S : -sum_log + nd * log(S);
            if (!isfinite(nll) || (!p.extended && !(S > 0.0))) {
                nll = INFINITY;
                flags = 1;
            }
        }
        p.out[0] = nll;
        p.out[1 + 2 * k] = (double)flags;
        s_c = c;
    }
    __syncthreads();
    const double c = s_c;
    const bool zero = !p.extended && p.nd_total == 0.0;
    for (int i = tid; i < 2 * k; i += kCombineThreads) {
        const double h = p.gram ? mv[i] : tm[1 + i];
        p.out[1 + i] = zero ? 0.0 : 2.0 * (-td[1 + i] + c * h);
    }
}

}  // namespace

hipError_t launch_combine(const StreamArgs &args, double log_scale, hipStream_t stream) {
    hipLaunchKernelGGL(nll_combine_kernel, dim3(1), dim3(kCombineThreads), 0, stream, args,
                       log_scale);
    return hipGetLastError();
}

}  // namespace pwa
