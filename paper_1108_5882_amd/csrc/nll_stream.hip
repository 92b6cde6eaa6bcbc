// Fused single-V negative log-likelihood and gradient (Berger, Section 2, Eq. 1-3).
//
// One launch streams the data rows and the MC rows once each:
//   data row i:  z_i = sum_a V_a A_ia;  I_i = |z_i|^2;  accumulate ln I_i and
//                conj(A_ia) z_i / I_i                  (Eq. 2 data term and its derivative)
//   MC row j:    accumulate w_j I_j and w_j conj(A_ja) z_j   (MC estimate of the
//                normalisation integral and its derivative)
// and the last block to finish combines the FP64 block partials in a fixed
// order into NLL and the real gradient.
//
// Layout and mapping (gfx950, 64-lane waves): an event row is ld = L*C complex
// values; L consecutive lanes share a row and lane j holds complexes
// [jC, jC+C), so one wave instruction reads 64/L whole rows contiguously.
// The partial coherent sums are combined across the L lanes with DPP row
// operations (no LDS), after which every lane of the group holds the same z.
//
// Precision (the paper's remark in Section 2): FP32 contexts store and stream
// the amplitudes in single precision; z, I and z/I are formed in FP64 from the
// exactly upcast values and log2 I is taken in FP32.  Every per-lane
// accumulator is FP64, so no sum over events runs in single precision.  FP64
// contexts are double throughout.  Block partials are reduced in a fixed order: results are
// bitwise reproducible for a given launch shape.
#include "internal.hpp"

#include <cmath>
#include <type_traits>

namespace pwa {
namespace {

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
__device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    v.x = dpp_i<CTRL>(v.x);
    v.y = dpp_i<CTRL>(v.y);
    return *reinterpret_cast<double *>(&v);
}

template <int L, typename T>
__device__ __forceinline__ T group_sum(T x) {
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (L >= 2) x += dpp_f<0xB1>(x);    // quad_perm [1,0,3,2]
        if constexpr (L >= 4) x += dpp_f<0x4E>(x);    // quad_perm [2,3,0,1]
        if constexpr (L >= 8) x += dpp_f<0x141>(x);   // row_half_mirror
        if constexpr (L >= 16) x += dpp_f<0x140>(x);  // row_mirror
    } else {
        if constexpr (L >= 2) x += dpp_d<0xB1>(x);
        if constexpr (L >= 4) x += dpp_d<0x4E>(x);
        if constexpr (L >= 8) x += dpp_d<0x141>(x);
        if constexpr (L >= 16) x += dpp_d<0x140>(x);
    }
    if constexpr (L >= 32) x += __shfl_xor(x, 16);
    if constexpr (L >= 64) x += __shfl_xor(x, 32);
    return x;
}

// ------------------------------------------------- per-event arithmetic
// z and I are formed in FP64 from the stored values (exact upcast of FP32
// amplitudes); FP64 FMA runs at the FP32 rate here and the loop is bound by
// HBM, so this costs no throughput and removes the cancellation error of an
// FP32 coherent sum near interference minima.
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

template <typename T, int C>
constexpr int unroll_rows() {
    return stream_unroll(2 * (int)sizeof(T) * C);
}

// Streams one segment.  SEG 0: data (ln I, conj(A) z / I); SEG 1: MC (w I, w conj(A) z).
template <typename T, int L, int C, int SEG>
__device__ __forceinline__ void stream_segment(const T *__restrict__ A, const T *__restrict__ w,
                                               int64_t n, int64_t ld, int64_t wave0,
                                               int64_t nwaves, const double (&vr)[C],
                                               const double (&vi)[C],
                                               double &acc_t, double (&acc_r)[C],
                                               double (&acc_i)[C]) {
    constexpr int U = unroll_rows<T, C>();
    constexpr int G = 64 / L;
    constexpr int ROWS = G * U;
    const int lane = threadIdx.x & 63;
    const int g = lane / L;
    const int j = lane % L;
    const int64_t ntiles = (n + ROWS - 1) / ROWS;
    for (int64_t tile = wave0; tile < ntiles; tile += nwaves) {
        T a[U][2 * C];
        T wv[U];
        bool valid[U];
        const int64_t row0 = tile * ROWS + g;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row = row0 + (int64_t)u * G;
            valid[u] = row < n;
            if (valid[u]) {
                RowLoad<T, C>::load(A + 2 * (row * ld + (int64_t)j * C), a[u]);
            } else {
#pragma unroll
                for (int q = 0; q < 2 * C; ++q) a[u][q] = T(0);
            }
            if constexpr (SEG == 1) wv[u] = (w && valid[u]) ? load_nt(w + row) : T(valid[u] ? 1 : 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
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
                if (!valid[u]) continue;
                acc_t += EventMath<T>::logsum_term(I);
                const double rI = EventMath<T>::recip(I);
                ur = zr * rI;
                ui = zi * rI;
            } else {
                const double wd = (double)wv[u];
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
}

template <typename T, int L, int C, int NT>
__global__ __launch_bounds__(NT) void nll_stream_kernel(StreamArgs p) {
    constexpr int NW = NT / 64;
    constexpr int SLOT = 2 * C + 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
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
        stream_segment<T, L, C, 0>(static_cast<const T *>(p.A[0]), nullptr, p.n[0], p.ld, wave0,
                                   nwaves, vr, vi, acc_t, acc_r, acc_i);
    else
        stream_segment<T, L, C, 1>(static_cast<const T *>(p.A[1]), static_cast<const T *>(p.w),
                                   p.n[1], p.ld, wave0, nwaves, vr, vi, acc_t, acc_r, acc_i);

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
    __shared__ bool s_last;
    if (lane < L) {
        red[wid][j][0] = acc_t;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            red[wid][j][1 + 2 * c] = acc_r[c];
            red[wid][j][2 + 2 * c] = acc_i[c];
        }
    }
    __syncthreads();

    // block partial: [0] scalar sum, [1 + 2a + {0,1}] complex sums, a < ld
    double *part = p.partials + (int64_t)blockIdx.x * p.pstride;
    for (int idx = tid; idx < p.pstride; idx += NT) {
        double s = 0.0;
        if (idx == 0) {
            for (int w = 0; w < NW; ++w) s += red[w][0][0];
        } else {
            const int a = (idx - 1) >> 1, q = (idx - 1) & 1;
            const int jj = a / C, c = a % C;
            for (int w = 0; w < NW; ++w) s += red[w][jj][1 + 2 * c + q];
        }
        __hip_atomic_store(part + idx, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned total = (unsigned)(p.nb[0] + p.nb[1]);
        const unsigned prev = __hip_atomic_fetch_add(p.counter, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == total - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();

    // ---------------- last block: fixed-order FP64 combine of all partials
    constexpr int NPARTS = NT > 2 * (1 + 2 * PWA_MAX_K) ? NT : 2 * (1 + 2 * PWA_MAX_K);
    __shared__ double parts[NPARTS];
    __shared__ double tot[2][1 + 2 * PWA_MAX_K];
    __shared__ double mv[2 * PWA_MAX_K];
    __shared__ double s_c;
    const int ncol = 2 * p.pstride;
    const int P = NPARTS / ncol > 0 ? NPARTS / ncol : 1;
    for (int idx = tid; idx < P * ncol; idx += NT) {
        const int col = idx / P, pp = idx % P;
        const int sg = col / p.pstride, cc = col % p.pstride;
        const int base = sg ? p.nb[0] : 0;
        double s = 0.0;
        for (int b = pp; b < p.nb[sg]; b += P)
            s += __hip_atomic_load(p.partials + (int64_t)(base + b) * p.pstride + cc,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        parts[idx] = s;
    }
    __syncthreads();
    for (int col = tid; col < ncol; col += NT) {
        double s = 0.0;
        for (int pp = 0; pp < P; ++pp) s += parts[col * P + pp];
        const int sg = col / p.pstride, cc = col % p.pstride;
        if (cc < 1 + 2 * PWA_MAX_K) tot[sg][cc] = s;
    }
    __syncthreads();

    const int k = p.k;
    // MC quantities: streamed (S_raw, H) or from the precomputed matrix (V^H M V, M V)
    if (p.gram) {
        for (int a = tid; a < k; a += NT) {
            double r = 0.0, i = 0.0;
            for (int b = 0; b < k; ++b) {
                const double mr = p.gram[2 * (a * k + b)], mi = p.gram[2 * (a * k + b) + 1];
                const double vr_ = p.v_dev ? p.v_dev[2 * b] : p.v_arg[2 * b];
                const double vi_ = p.v_dev ? p.v_dev[2 * b + 1] : p.v_arg[2 * b + 1];
                r += mr * vr_ - mi * vi_;
                i += mr * vi_ + mi * vr_;
            }
            mv[2 * a] = r;
            mv[2 * a + 1] = i;
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double nd = p.nd_total;
        const double sum_log = tot[0][0] * EventMath<T>::kLogScale;
        double S, c;
        if (p.gram) {
            double s = 0.0;
            for (int a = 0; a < k; ++a) {
                const double vr_ = p.v_dev ? p.v_dev[2 * a] : p.v_arg[2 * a];
                const double vi_ = p.v_dev ? p.v_dev[2 * a + 1] : p.v_arg[2 * a + 1];
                s += vr_ * mv[2 * a] + vi_ * mv[2 * a + 1];   // Re conj(V_a) (M V)_a
            }
            S = s;
            c = p.extended ? 1.0 : nd / S;
        } else {
            S = tot[1][0] / p.n_gen;
            c = p.extended ? 1.0 / p.n_gen : nd / tot[1][0];
        }
        double nll;
        unsigned flags = 0;
        if (!p.extended && nd == 0.0) {
            nll = 0.0;
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
    for (int idx = tid; idx < 2 * k; idx += NT) {
        const double h = p.gram ? mv[idx] : tot[1][1 + idx];
        p.out[1 + idx] = zero ? 0.0 : 2.0 * (-tot[0][1 + idx] + c * h);
    }
    if (tid == 0) __hip_atomic_store(p.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------- dispatch
constexpr int kThreads = kStreamThreads;

template <typename T, int L, int C>
hipError_t launch_one(int blocks, const StreamArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL((nll_stream_kernel<T, L, C, kThreads>), dim3(blocks), dim3(kThreads), 0,
                       stream, args);
    return hipGetLastError();
}

template <typename T, int C>
hipError_t launch_c(int L, int blocks, const StreamArgs &args, hipStream_t stream) {
    switch (L) {
        case 1: return launch_one<T, 1, C>(blocks, args, stream);
        case 2: return launch_one<T, 2, C>(blocks, args, stream);
        case 4: return launch_one<T, 4, C>(blocks, args, stream);
        case 8: return launch_one<T, 8, C>(blocks, args, stream);
        case 16: return launch_one<T, 16, C>(blocks, args, stream);
        case 32:
            if constexpr (C <= 2) return launch_one<T, 32, C>(blocks, args, stream);
            break;
        default: break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

StreamShape choose_shape(pwa_prec prec, int k) {
    // candidates in order of preference for equal padded width
    static const int pref32[] = {2, 4, 1, 3};
    static const int pref64[] = {1, 2, 3};
    const int *pref = prec == PWA_F32 ? pref32 : pref64;
    const int npref = prec == PWA_F32 ? 4 : 3;
    StreamShape best{0, 0};
    int best_ld = 1 << 30;
    for (int i = 0; i < npref; ++i) {
        const int C = pref[i];
        for (int L = 1; L <= 32; L <<= 1) {
            if (L == 32 && C > 2) continue;
            const int ld = L * C;
            if (ld < k) continue;
            if (ld < best_ld) {
                best_ld = ld;
                best = StreamShape{L, C};
            }
            break;   // larger L only pads more
        }
    }
    return best;
}

hipError_t launch_stream(pwa_prec prec, StreamShape s, int threads, int blocks,
                         const StreamArgs &args, hipStream_t stream) {
    if (threads != kThreads) return hipErrorInvalidValue;
    if (prec == PWA_F32) {
        switch (s.C) {
            case 1: return launch_c<float, 1>(s.L, blocks, args, stream);
            case 2: return launch_c<float, 2>(s.L, blocks, args, stream);
            case 3: return launch_c<float, 3>(s.L, blocks, args, stream);
            case 4: return launch_c<float, 4>(s.L, blocks, args, stream);
            default: break;
        }
    } else {
        switch (s.C) {
            case 1: return launch_c<double, 1>(s.L, blocks, args, stream);
            case 2: return launch_c<double, 2>(s.L, blocks, args, stream);
            case 3: return launch_c<double, 3>(s.L, blocks, args, stream);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
