// Fused single-V negative log-likelihood and gradient (Berger, Section 2, Eq. 1-3).
//
// One launch streams the data rows and the MC rows once each:
//   data row i:  z_i = sum_a V_a A_ia;  I_i = |z_i|^2;  accumulate ln I_i and
//                conj(A_ia) z_i / I_i                  (Eq. 2 data term and its derivative)
//   MC row j:    accumulate w_j I_j and w_j conj(A_ja) z_j   (MC estimate of the
//                normalisation integral and its derivative)
// Each block writes one FP64 partial.  The same launch then combines them:
// the last block to finish in each group of kFinishGroup consecutive blocks
// (found with an arrival counter) adds its group's partials in block order,
// and the last group to finish adds the group sums in group order and forms
// NLL and the real gradient.  Every addition has a fixed place in that order,
// so results are bitwise reproducible for a launch configuration.
//
// Layout and mapping (gfx950, 64-lane waves): an event row is ld = L*C complex
// values; L consecutive lanes share a row and lane j holds complexes
// [jC, jC+C), so one wave instruction reads 64/L whole rows contiguously.
// Each lane group takes U rows per stage; the loop keeps two stages in
// registers so the next stage's loads are in flight while the current one is
// computed.  While every row of the tiles in flight exists, a stage's loads
// are a wave-uniform tile address plus per-lane and per-row constant offsets
// with no masks; the last tiles of each wave load with the row index clamped
// into the sample (always a valid address, so the loads stay unconditional
// and the compiler can count them) and mask rows past the end in the
// arithmetic.  The partial coherent sums are combined across
// the L lanes with DPP row operations.
//
// Precision (the paper's remark in Section 2): FP32 contexts store and stream
// the amplitudes in single precision; z, I and z/I are formed in FP64 from the
// exactly upcast values and log2 I is taken in FP32.  Every per-lane
// accumulator is FP64, so no sum over events runs in single precision.  FP64
// contexts are double throughout.  Block partials are reduced in a fixed
// order: results are bitwise reproducible for a given launch configuration.
#pragma once

#include <cmath>
#include <type_traits>

#include "block_reduce.hpp"
#include "internal.hpp"

namespace pwa {
namespace stream_detail {

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

constexpr double kLn2 = 0.69314718055994530942;

// ------------------------------------------------------------ row loads
// Streamed rows are read once per evaluation: non-temporal loads through the
// global address space.
template <typename V>
__device__ __forceinline__ V load_nt(const V *p) {
    typedef const V __attribute__((address_space(1))) *gptr;
    return __builtin_nontemporal_load((gptr)p);
}

template <typename T, int C>
struct RowLoad;

template <int C>
struct RowLoad<float, C> {
    static __device__ __forceinline__ void load(const float *p, float (&a)[2 * C]) {
        if constexpr (C % 2 == 0) {
#pragma unroll
            for (int q = 0; q < C / 2; ++q) {
                f4v v = load_nt(reinterpret_cast<const f4v *>(p) + q);
                a[4 * q + 0] = v.x;
                a[4 * q + 1] = v.y;
                a[4 * q + 2] = v.z;
                a[4 * q + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < C; ++q) {
                f2v v = load_nt(reinterpret_cast<const f2v *>(p) + q);
                a[2 * q + 0] = v.x;
                a[2 * q + 1] = v.y;
            }
        }
    }
};

template <int C>
struct RowLoad<double, C> {
    static __device__ __forceinline__ void load(const double *p, double (&a)[2 * C]) {
#pragma unroll
        for (int q = 0; q < C; ++q) {
            d2v v = load_nt(reinterpret_cast<const d2v *>(p) + q);
            a[2 * q + 0] = v.x;
            a[2 * q + 1] = v.y;
        }
    }
};

// ------------------------------------------------ sums over L lanes (DPP)
// Each step adds a value from a partner lane in the other half of the current
// group; fp addition is commutative, so every lane ends with the same bits.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    v.x = dpp_i<CTRL>(v.x);
    v.y = dpp_i<CTRL>(v.y);
    return *reinterpret_cast<double *>(&v);
}

template <int L>
__device__ __forceinline__ double group_sum(double x) {
    if constexpr (L >= 2) x += dpp_d<0xB1>(x);    // quad_perm [1,0,3,2]
    if constexpr (L >= 4) x += dpp_d<0x4E>(x);    // quad_perm [2,3,0,1]
    if constexpr (L >= 8) x += dpp_d<0x141>(x);   // row_half_mirror
    if constexpr (L >= 16) x += dpp_d<0x140>(x);  // row_mirror
    if constexpr (L >= 32) x += __shfl_xor(x, 16);
    if constexpr (L >= 64) x += __shfl_xor(x, 32);
    return x;
}

// ------------------------------------------------- per-event arithmetic
// z and I are formed in FP64 from the stored values (exact upcast of FP32
// amplitudes); FP64 FMA runs at the FP32 rate here and the loop is bound by
// HBM, so this removes the cancellation error of an FP32 coherent sum near
// interference minima at no throughput cost.
template <typename T>
struct EventMath;

template <>
struct EventMath<float> {
    // FP32 log2 of the rounded intensity (the combine multiplies the FP64 sum by ln 2)
    static __device__ __forceinline__ double logsum_term(double I) {
        return (double)__log2f((float)I);
    }
    // hardware reciprocal refined by one Newton step
    static __device__ __forceinline__ double recip(double I) {
        double r = __builtin_amdgcn_rcp(I);
        const double e = fma(-I, r, 1.0);
        return fma(r, e, r);
    }
    static constexpr double kLogScale = kLn2;
};

template <>
struct EventMath<double> {
    static __device__ __forceinline__ double logsum_term(double I) { return log(I); }
    static __device__ __forceinline__ double recip(double I) { return 1.0 / I; }
    static constexpr double kLogScale = 1.0;
};

// ------------------------------------------- combine of the block partials
// Called by every block after it stored its partial with st_dev (PS doubles:
// the summed log term or w I, then the complex adjoint sums).  The last block
// of the launch forms NLL and gradient from the totals.
template <int PS, int NT>
__device__ __forceinline__ void finish(const StreamArgs &p, double log_scale) {
    __shared__ double tot[2 * PS];
    __shared__ double mv[PS];
    __shared__ double s_c;
    const int tid = threadIdx.x;
    if (!reduce_blocks<PS, NT>(ReduceBufs{p.partials, p.gsums, p.counters, p.nb[0], p.nb[0] + p.nb[1]}, tot))
        return;

    // Eq. 2 form:  NLL = -sum ln I + N_D ln S,   c = N_D / (N_gen S)
    // Eq. 3 form:  NLL = -sum ln I + S,          c = 1 / N_gen
    // gradient     = 2 (-G + c H), H = sum w conj(A) z over MC rows, or with the
    // MC matrix M (1/N_gen folded in): S = V^H M V and H replaced by M V, N_gen = 1
    const int k = p.k;
    const double *V = p.v_dev ? p.v_dev : p.v_arg;
    if (p.gram) {
        for (int a = tid; a < k; a += NT) {
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
    const double *tm = tot + PS;     // MC:   [0] sum w I, [1 + i] H
    const bool empty = !p.extended && p.nd_total == 0.0;
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
        if (empty) {
            nll = 0.0;                              // empty product: ln L = 0
            c = 0.0;
        } else {
            nll = p.extended ? -sum_log + S : -sum_log + nd * log(S);
            if (!isfinite(nll) || (!p.extended && !(S > 0.0))) {
                nll = INFINITY;
                flags = 1;
            }
        }
        st_sys(p.out, nll);
        st_sys(p.out + 1 + 2 * k, (double)flags);
        s_c = c;
    }
    __syncthreads();
    const double c = s_c;
    for (int i = tid; i < 2 * k; i += NT) {
        const double h = p.gram ? mv[i] : tm[1 + i];
        st_sys(p.out + 1 + i, empty ? 0.0 : 2.0 * (-td[1 + i] + c * h));
    }
    if (p.done) {
        // the result reaches host memory before the sequence number that announces it
        wait_stores();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(p.done, p.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Keeps the compiler's scheduler from moving instructions across this point:
// a stage's loads are issued before the previous stage is computed, so two
// stages are in flight while it runs (left to itself, the scheduler sinks the
// loads below the arithmetic and waits for every load at the top of the loop).
__device__ __forceinline__ void fence_sched() { __builtin_amdgcn_sched_barrier(0); }

// One stage: U rows per lane group.
template <typename T, int L, int C, int U, int SEG>
struct Stage {
    T a[U][2 * C];
    T w[U];

    static constexpr int G = 64 / L;
    static constexpr int LD = L * C;   // row stride in complex values: the layout width

    // rows t*ROWS + u*G + g, clamped into [0, n): always a valid address
    // (ld: row stride in complex values)
    __device__ __forceinline__ void load(const T *__restrict__ A, const T *__restrict__ W,
                                         int64_t n, int64_t ld, int64_t tile, int g, int j) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int64_t row = tile * (G * U) + (int64_t)u * G + g;
            row = row < n ? row : n - 1;
            RowLoad<T, C>::load(A + 2 * (row * ld + (int64_t)j * C), a[u]);
            if constexpr (SEG == 1) w[u] = W ? load_nt(W + row) : T(1);
        }
    }

    // A tile whose rows all exist, row stride LD: the tile's base address is
    // the same in every lane (tile is wave-uniform), each lane adds a fixed
    // offset, and the rows u*G apart are constant offsets from it, so no
    // per-row address arithmetic or clamping is needed.  SEG 1 here needs W.
    __device__ __forceinline__ void load_full(const T *__restrict__ A, const T *__restrict__ W,
                                              int64_t tile, int g, int j) {
        if constexpr (SEG == 1) {
            const T *Wl = W + tile * (int64_t)(G * U) + g;
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = load_nt(Wl + u * G);
        }
        const T *At = A + tile * (int64_t)(G * U * LD * 2);
        const T *Al = At + (g * LD + j * C) * 2;
#pragma unroll
        for (int u = 0; u < U; ++u) RowLoad<T, C>::load(Al + u * G * LD * 2, a[u]);
    }

    // MASK: rows past n exist in the tile (clamped loads) and add nothing.
    template <bool MASK>
    __device__ __forceinline__ void compute(int64_t n, int64_t tile, int g, const double (&vr)[C],
                                            const double (&vi)[C], double &acc_t,
                                            double (&acc_r)[C], double (&acc_i)[C]) const {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool valid = !MASK || tile * (G * U) + (int64_t)u * G + g < n;
            double da[2 * C];
#pragma unroll
            for (int q = 0; q < 2 * C; ++q) da[q] = (double)a[u][q];
            double zr = 0.0, zi = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double ar = da[2 * c], ai = da[2 * c + 1];
                zr = fma(vr[c], ar, fma(-vi[c], ai, zr));
                zi = fma(vr[c], ai, fma(vi[c], ar, zi));
            }
            zr = group_sum<L>(zr);
            zi = group_sum<L>(zi);
            const double I = fma(zr, zr, zi * zi);
            double ur, ui;
            if constexpr (SEG == 0) {
                if (!valid) continue;
                acc_t += EventMath<T>::logsum_term(I);
                const double rI = EventMath<T>::recip(I);
                ur = zr * rI;
                ui = zi * rI;
            } else {
                const double wd = valid ? (SEG == 2 ? 1.0 : (double)w[u]) : 0.0;
                acc_t = fma(wd, I, acc_t);
                ur = wd * zr;
                ui = wd * zi;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double ar = da[2 * c], ai = da[2 * c + 1];
                // conj(A) u = (ar ur + ai ui) + i (ar ui - ai ur)
                acc_r[c] = fma(ar, ur, fma(ai, ui, acc_r[c]));
                acc_i[c] = fma(ar, ui, fma(-ai, ur, acc_i[c]));
            }
        }
    }
};

// Streams one segment.  SEG 0: data (ln I, conj(A) z / I); SEG 1: MC with
// weights w (w I, w conj(A) z); SEG 2: MC with unit weights (I, conj(A) z).
// Whether the MC rows carry weights is a compile-time choice: a run-time test
// around the weight load would put a branch in the loop, at whose join the
// compiler waits for every load in flight, the next stage's prefetch included.
template <typename T, int L, int C, int U, int SEG>
__device__ __forceinline__ void stream_segment(const T *__restrict__ A, const T *__restrict__ W,
                                               int64_t n, int64_t wave0,
                                               int64_t nwaves, const double (&vr)[C],
                                               const double (&vi)[C], double &acc_t,
                                               double (&acc_r)[C], double (&acc_i)[C]) {
    constexpr int ROWS = (64 / L) * U;
    constexpr int64_t LD = L * C;
    const int lane = threadIdx.x & 63;
    const int g = lane / L;
    const int j = lane % L;
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    const int64_t nfull = n / ROWS;   // tiles whose rows all exist
    int64_t t = wave0;
    if (t >= ntiles) return;
    Stage<T, L, C, U, SEG> s0, s1;
    if (t + 2 * nwaves < nfull) {
        // every tile loaded here is whole: no clamping, no row masks
        s0.load_full(A, W, t, g, j);
        fence_sched();
        do {
            s1.load_full(A, W, t + nwaves, g, j);
            fence_sched();
            s0.template compute<false>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
            t += nwaves;
            s0.load_full(A, W, t + nwaves, g, j);
            fence_sched();
            s1.template compute<false>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
            t += nwaves;
        } while (t + 2 * nwaves < nfull);
    } else {
        s0.load(A, W, n, LD, t, g, j);
        fence_sched();
    }
    // the last tiles of this wave (s0 holds tile t): clamped loads, masked rows
    for (;;) {
        s1.load(A, W, n, LD, t + nwaves, g, j);
        fence_sched();
        s0.template compute<true>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
        t += nwaves;
        if (t >= ntiles) break;
        s0.load(A, W, n, LD, t + nwaves, g, j);
        fence_sched();
        s1.template compute<true>(n, t, g, vr, vi, acc_t, acc_r, acc_i);
        t += nwaves;
        if (t >= ntiles) break;
    }
}

template <typename T, int L, int C, int U, int NT>
__global__ __launch_bounds__(NT) void nll_stream_kernel(StreamArgs p) {
    constexpr int NW = NT / 64;
    constexpr int SLOT = 2 * C + 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int j = lane % L;

    // V slice of this lane (FP64)
    double vr[C], vi[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int a = j * C + c;
        double r = 0.0, i = 0.0;
        if (a < p.k) {
            r = p.v_dev ? p.v_dev[2 * a] : p.v_arg[2 * a];
            i = p.v_dev ? p.v_dev[2 * a + 1] : p.v_arg[2 * a + 1];
        }
        vr[c] = r;
        vi[c] = i;
    }

    const int seg = (int)blockIdx.x < p.nb[0] ? 0 : 1;
    const int bseg = seg ? (int)blockIdx.x - p.nb[0] : (int)blockIdx.x;
    const int64_t wave0 = (int64_t)bseg * NW + wid;
    const int64_t nwaves = (int64_t)p.nb[seg] * NW;

    double acc_t = 0.0;
    double acc_r[C], acc_i[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc_r[c] = acc_i[c] = 0.0;

    if (seg == 0)
        stream_segment<T, L, C, U, 0>(static_cast<const T *>(p.A[0]), nullptr, p.n[0], wave0,
                                      nwaves, vr, vi, acc_t, acc_r, acc_i);
    else if (p.w)
        stream_segment<T, L, C, U, 1>(static_cast<const T *>(p.A[1]), static_cast<const T *>(p.w),
                                      p.n[1], wave0, nwaves, vr, vi, acc_t, acc_r, acc_i);
    else
        stream_segment<T, L, C, U, 2>(static_cast<const T *>(p.A[1]), nullptr, p.n[1], wave0,
                                      nwaves, vr, vi, acc_t, acc_r, acc_i);

    // lanes with the same j across the wave's row groups
#pragma unroll
    for (int off = L; off < 64; off <<= 1) {
        acc_t += __shfl_xor(acc_t, off);
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc_r[c] += __shfl_xor(acc_r[c], off);
            acc_i[c] += __shfl_xor(acc_i[c], off);
        }
    }

    __shared__ double red[NW][L][SLOT];
    if (lane < L) {
        red[wid][j][0] = acc_t;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            red[wid][j][1 + 2 * c] = acc_r[c];
            red[wid][j][2 + 2 * c] = acc_i[c];
        }
    }
    __syncthreads();

    // block partial [block][PS]: column 0 the scalar sum, 1 + 2a + {0,1} the
    // complex sums, a < ld
    constexpr int PS = 1 + 2 * L * C;
    for (int idx = tid; idx < PS; idx += NT) {
        double s = 0.0;
        if (idx == 0) {
            for (int w = 0; w < NW; ++w) s += red[w][0][0];
        } else {
            const int a = (idx - 1) >> 1, q = (idx - 1) & 1;
            const int jj = a / C, c = a % C;
            for (int w = 0; w < NW; ++w) s += red[w][jj][1 + 2 * c + q];
        }
        st_dev(p.partials + (int64_t)blockIdx.x * PS + idx, s);
    }
    finish<PS, NT>(p, EventMath<T>::kLogScale);
}

template <typename T, int L, int C, int U>
hipError_t launch_cfg(int blocks, const StreamArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL((nll_stream_kernel<T, L, C, U, kStreamThreads>), dim3(blocks),
                       dim3(kStreamThreads), 0, stream, args);
    return hipGetLastError();
}

// Instantiates every (L, U) of one complex-per-lane C; L * C <= 64.
template <typename T, int C, int U>
hipError_t dispatch_l(int L, int blocks, const StreamArgs &args, hipStream_t stream) {
    switch (L) {
        case 1: return launch_cfg<T, 1, C, U>(blocks, args, stream);
        case 2: return launch_cfg<T, 2, C, U>(blocks, args, stream);
        case 4: return launch_cfg<T, 4, C, U>(blocks, args, stream);
        case 8:
            if constexpr (8 * C <= 64) return launch_cfg<T, 8, C, U>(blocks, args, stream);
            break;
        case 16:
            if constexpr (16 * C <= 64) return launch_cfg<T, 16, C, U>(blocks, args, stream);
            break;
        case 32:
            if constexpr (32 * C <= 64) return launch_cfg<T, 32, C, U>(blocks, args, stream);
            break;
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace stream_detail
}  // namespace pwa
