// Many independent fits in one persistent launch (Berger, Section 2: fits are
// repeated from many starting points and models, each needing the likelihood
// of Eq. 2 and its gradient at every iteration).
//
// Every fit f has its own samples (N_D, N_MC, K_f) and its own trial vector.
// The rows of all fits are cut into work items (one sample of one fit, a
// range of tiles); blocks take items from an atomic counter, stream the rows
// of the item with the fused single-V arithmetic (FP32 storage, FP64 z, I,
// z/I and sums) and write one FP64 partial per item.  Because each item has
// its own slot, results do not depend on which block took which item.  A
// combine kernel adds each fit's item partials in item order and forms NLL
// and gradient; a minimiser kernel then advances each fit's L-BFGS state.
// The three kernels are captured once in a HIP graph and replayed per step.
//
// Row widths differ between fits (K from 4 to 48): each item carries its
// width and the block dispatches to the compiled tile shape for it.
#include "nll_stream_impl.hpp"

namespace pwa {
namespace {

using stream_detail::EventMath;
using stream_detail::Stage;

constexpr int kMT = kStreamThreads;     // threads per block
constexpr int kMW = kMT / 64;

// Streams tiles [t0, t1) of one sample with shape (L, C, U); waves take tiles
// t0 + wave, t0 + wave + kMW, ...; returns the block's partial in red.
constexpr int kRedSlot = 2 * 6 + 1;      // largest 2C + 1 of the shapes below

// Wave index of lane j's local complex c.  Contiguous (CH = false): lane j
// holds waves [jC, jC + C).  Chunked (CH = true, C even): lane j holds the
// 2-wave chunks j, j + L, j + 2L, ..., so each 16-byte load instruction of a
// lane group covers one contiguous span of the row (used for rows of 24 and
// 48 waves, which three contiguous waves per lane would read in 8-byte pieces).
template <int L, int C, bool CH>
__device__ __forceinline__ int wave_of(int j, int c) {
    if constexpr (CH) return 2 * (j + L * (c >> 1)) + (c & 1);
    else return j * C + c;
}

// Row loads of the chunked layout (same registers as Stage::load fills), row
// stride L * C complex.  FULL: every row of the tile exists (wave-uniform tile
// base, constant offsets, no clamping; SEG 1 then needs W); otherwise rows
// are clamped into [0, n).
template <int L, int C, int U, int SEG, bool FULL>
__device__ __forceinline__ void load_chunked(Stage<float, L, C, U, SEG> &st, const float *__restrict__ A,
                                             const float *__restrict__ W, int64_t n, int64_t tile,
                                             int g, int j) {
    typedef float f4c __attribute__((ext_vector_type(4)));
    typedef const f4c __attribute__((address_space(1))) *gp4;
    typedef const float __attribute__((address_space(1))) *gpf;
    constexpr int G = 64 / L;
    constexpr int64_t LD = L * C;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int64_t row = tile * (G * U) + (int64_t)u * G + g;
        if constexpr (!FULL) row = row < n ? row : n - 1;
        if constexpr (SEG == 1) st.w[u] = FULL || W ? __builtin_nontemporal_load((gpf)(W + row)) : 1.f;
#pragma unroll
        for (int i = 0; i < C / 2; ++i) {
            const f4c v = __builtin_nontemporal_load((gp4)(A + 2 * (row * LD + 2 * (j + L * i))));
            st.a[u][4 * i + 0] = v.x;
            st.a[u][4 * i + 1] = v.y;
            st.a[u][4 * i + 2] = v.z;
            st.a[u][4 * i + 3] = v.w;
        }
    }
}

template <int L, int C, int U, int SEG, bool CH = false>
__device__ __forceinline__ void multi_item(const MultiItem &it, const MultiFit &fit, double *slot, double *red) {
    constexpr int SLOT = 2 * C + 1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int g = lane / L, j = lane % L;
    const float *A = SEG ? fit.A_mc : fit.A_data;
    const float *W = SEG ? fit.w_mc : nullptr;
    const int64_t n = SEG ? fit.n_mc : fit.n_data;
    const double *V = fit.V;
    double vr[C], vi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = wave_of<L, C, CH>(j, c);
        vr[c] = a < fit.k ? V[2 * a] : 0.0;
        vi[c] = a < fit.k ? V[2 * a + 1] : 0.0;
    }
    // row stride L * C (the item's width selected this shape)
    auto ld_stage = [&](Stage<float, L, C, U, SEG> &st, int64_t tt) {
        if constexpr (CH) load_chunked<L, C, U, SEG, false>(st, A, W, n, tt, g, j);
        else st.load(A, W, n, (int64_t)(L * C), tt, g, j);
    };
    auto ld_full = [&](Stage<float, L, C, U, SEG> &st, int64_t tt) {
        if constexpr (CH) load_chunked<L, C, U, SEG, true>(st, A, W, n, tt, g, j);
        else st.load_full(A, W, tt, g, j);
    };
    double acc_t = 0.0, acc_r[C], acc_i[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc_r[c] = acc_i[c] = 0.0;
    constexpr int ROWS = (64 / L) * U;
    const int64_t nfull = n / ROWS;   // tiles whose rows all exist
    int64_t t = it.t0 + wid;
    if (t < it.t1) {
        Stage<float, L, C, U, SEG> s0, s1;
        // the same two-stage schedule as the single-fit pass: whole tiles
        // without clamping or masks while they last, then the clamped loads
        if (t + kMW < it.t1 && t + 2 * kMW < nfull) {
            ld_full(s0, t);
            stream_detail::fence_sched();
            do {
                ld_full(s1, t + kMW);
                stream_detail::fence_sched();
                s0.template compute<false>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
                t += kMW;
                ld_full(s0, t + kMW);
                stream_detail::fence_sched();
                s1.template compute<false>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
                t += kMW;
            } while (t + kMW < it.t1 && t + 2 * kMW < nfull);
        } else {
            ld_stage(s0, t);
            stream_detail::fence_sched();
        }
        // s0 holds tile t
        while (t < it.t1) {
            ld_stage(s1, t + kMW);
            stream_detail::fence_sched();
            s0.template compute<true>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
            t += kMW;
            if (t >= it.t1) break;
            ld_stage(s0, t + kMW);
            stream_detail::fence_sched();
            s1.template compute<true>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
            t += kMW;
        }
    }
#pragma unroll
    for (int off = L; off < 64; off <<= 1) {
        acc_t += __shfl_xor(acc_t, off);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc_r[c] += __shfl_xor(acc_r[c], off);
            acc_i[c] += __shfl_xor(acc_i[c], off);
        }
    }
    auto R = [&](int w, int jj, int s_) -> double & { return red[(w * 64 + jj) * SLOT + s_]; };
    if (lane < L) {
        R(wid, j, 0) = acc_t;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            R(wid, j, 1 + 2 * c) = acc_r[c];
            R(wid, j, 2 + 2 * c) = acc_i[c];
        }
    }
    __syncthreads();
    const int ps = 1 + 2 * L * C;
    for (int idx = threadIdx.x; idx < ps; idx += kMT) {
        double s = 0.0;
        if (idx == 0) {
            for (int w = 0; w < kMW; ++w) s += R(w, 0, 0);
        } else {
            const int a = (idx - 1) >> 1, q = (idx - 1) & 1;
            // lane and local complex of wave a (inverse of wave_of)
            int jj, cc;
            if constexpr (CH) {
                jj = (a >> 1) % L;
                cc = 2 * ((a >> 1) / L) + (a & 1);
            } else {
                jj = a / C;
                cc = a % C;
            }
            for (int w = 0; w < kMW; ++w) s += R(w, jj, 1 + 2 * cc + q);
        }
        slot[idx] = s;
    }
    __syncthreads();
}

template <int SEG>
__device__ __forceinline__ void dispatch_item(const MultiItem &it, const MultiFit &fit, double *slot, double *red) {
    switch (fit.ld) {
        case 4: multi_item<2, 2, 4, SEG>(it, fit, slot, red); break;
        case 6: multi_item<2, 3, 2, SEG>(it, fit, slot, red); break;
        case 8: multi_item<4, 2, 4, SEG>(it, fit, slot, red); break;
        case 12: multi_item<4, 3, 2, SEG>(it, fit, slot, red); break;
        case 16: multi_item<8, 2, 4, SEG>(it, fit, slot, red); break;
        case 24: multi_item<4, 6, 2, SEG, true>(it, fit, slot, red); break;
        case 32: multi_item<16, 2, 4, SEG>(it, fit, slot, red); break;
        case 48: multi_item<8, 6, 2, SEG, true>(it, fit, slot, red); break;
        default: break;
    }
}

__global__ __launch_bounds__(kMT) void multi_stream_kernel(MultiArgs p) {
    __shared__ int s_item;
    __shared__ double red[kMW * 64 * kRedSlot];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(p.item_counter, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= p.n_items) break;
        const MultiItem it = p.items[item];
        const MultiFit fit = p.fits[it.fit];
        double *slot = p.partials + (int64_t)item * kMultiSlot;
        // MC rows with weights (segment kind 1) or unit weights (2): a
        // compile-time choice, so the row loop holds no branch on it
        if (it.seg == 0)
            dispatch_item<0>(it, fit, slot, red);
        else if (fit.w_mc)
            dispatch_item<1>(it, fit, slot, red);
        else
            dispatch_item<2>(it, fit, slot, red);
    }
}

// One block per fit: adds the fit's item partials and forms NLL and gradient
// (Eq. 2 form), written to out[fit][2k + 2].  Slice s of a column adds items
// i0 + s, i0 + s + kSlices, ... (independent loads, several in flight); the
// slices are then added in slice order, so the result does not depend on
// which block evaluated which item.
constexpr int kCombineThreads = 1024;
constexpr int kSlices = 16;

__global__ __launch_bounds__(kCombineThreads) void multi_combine_kernel(MultiArgs p) {
    __shared__ double part[kSlices][2][1 + 2 * kMultiMaxLd];
    __shared__ double tot[2][1 + 2 * kMultiMaxLd];
    __shared__ double s_c;
    const int f = blockIdx.x, tid = threadIdx.x;
    const MultiFit fit = p.fits[f];
    const int k = fit.k, ps = 1 + 2 * (int)fit.ld;
    for (int idx = tid; idx < kSlices * 2 * ps; idx += kCombineThreads) {
        const int sl = idx / (2 * ps), rem = idx % (2 * ps);
        const int sg = rem / ps, cc = rem % ps;
        const int i0 = sg ? fit.item_mc0 : fit.item_data0;
        const int i1 = sg ? fit.item_mc1 : fit.item_data1;
        double s = 0.0;
#pragma unroll 4
        for (int i = i0 + sl; i < i1; i += kSlices) s += p.partials[(int64_t)i * kMultiSlot + cc];
        part[sl][sg][cc] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < 2 * ps; idx += kCombineThreads) {
        const int sg = idx / ps, cc = idx % ps;
        double s = 0.0;
        for (int sl = 0; sl < kSlices; ++sl) s += part[sl][sg][cc];
        tot[sg][cc] = s;
    }
    __syncthreads();
    double *out = p.out + (int64_t)f * kMultiOut;
    if (tid == 0) {
        const double nd = (double)fit.n_data;
        const double sum_log = tot[0][0] * EventMath<float>::kLogScale;
        const double s_raw = tot[1][0];
        double nll, c;
        unsigned flags = 0;
        if (nd == 0.0) {
            nll = 0.0;
            c = 0.0;
        } else {
            const double S = s_raw / fit.n_gen;
            nll = -sum_log + nd * log(S);
            c = nd / s_raw;
            if (!isfinite(nll) || !(S > 0.0)) {
                nll = INFINITY;
                flags = 1;
            }
        }
        out[0] = nll;
        out[1 + 2 * k] = (double)flags;
        s_c = c;
    }
    __syncthreads();
    for (int i = tid; i < 2 * k; i += kCombineThreads) out[1 + i] = 2.0 * (-tot[0][1 + i] + s_c * tot[1][1 + i]);
    if (f == 0 && tid == 0) *p.item_counter = 0u;      // ready for the next launch
}

}  // namespace

hipError_t launch_multi_eval(const MultiArgs &args, int blocks, hipStream_t stream) {
    hipLaunchKernelGGL(multi_stream_kernel, dim3(blocks), dim3(kMT), 0, stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(multi_combine_kernel, dim3(args.n_fits), dim3(kCombineThreads), 0, stream, args);
    return hipGetLastError();
}

bool multi_ld_supported(int64_t ld) {
    return ld == 4 || ld == 6 || ld == 8 || ld == 12 || ld == 16 || ld == 24 || ld == 32 || ld == 48;
}

int64_t multi_layout_ld(int k) {
    static const int widths[] = {4, 6, 8, 12, 16, 24, 32, 48};
    for (int w : widths)
        if (w >= k) return w;
    return -1;
}

int multi_rows_per_tile(int64_t ld) {
    switch (ld) {
        case 4: return 32 * 4;
        case 6: return 32 * 2;
        case 8: return 16 * 4;
        case 12: return 16 * 2;
        case 16: return 8 * 4;
        case 24: return 16 * 2;
        case 32: return 4 * 4;
        case 48: return 8 * 2;
        default: return 0;
    }
}

}  // namespace pwa
