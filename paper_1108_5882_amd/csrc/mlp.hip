// Surrogate of the NLL over production vectors for multi-start screening.
//
// Fits are repeated from many starting points to find the global minimum
// (Berger, Section 2 and Section 4, "Fits with large numbers of parameters").
// A small network f(V^) ~ ln(1 + NLL(V) - NLL_min) over the canonical vector
// V^ = V e^{-i arg V_0} / |V| ranks candidate starts; the exact likelihood
// judges and refines the best of them.
//
// Network: 2k -> H -> H -> 1, exact-erf GELU, weights held in FP32 (master)
// and used in FP16 by the matrix cores; every GEMM rounds both operands to
// FP16 when they are staged and accumulates in FP32 (v_mfma_f32_16x16x32_f16).
// Loss: mean squared error.  Optimiser: Adam (0.9, 0.999, 1e-8) on the FP32
// master weights.  The kernels of a training step are captured in HIP graphs
// (one step, and groups of 16 steps) and replayed.
#include "internal.hpp"

#include <cmath>

namespace pwa {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 256;          // GEMM block: 4 waves, 64 x 64 output tile
constexpr int kGK = 32;           // k step (one MFMA)
constexpr int kGKS = 256;         // k range staged in LDS at once
constexpr int kGS = kGKS + 8;     // LDS row stride in halfs (16-byte aligned rows)

template <typename T>
__device__ __forceinline__ float ld_f(const T *p, int64_t i) { return (float)p[i]; }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// GEMM epilogues: plain store; Z = C + b (per column) stored with H = GELU(Z);
// C * GELU'(Z) (the backward through the activation).
enum GemmEpi { kEpiNone, kEpiBiasGelu, kEpiGeluBack };
struct EpiArgs {
    const float *b;
    float *H;
    const float *Z;
};

// dst[r][c] = fp16(src(r0 + r, s0 + c)) for the 64 rows of a tile and the
// staged columns c < kw (zero outside the matrix or at k >= s1), where
// src(r, k) = src[r ld + k] (TR false) or src[k ld + r] (TR true).  Four
// consecutive elements per thread and load (16 bytes where the layout allows);
// all loads of the stage are issued before the first LDS store.
template <bool TR, typename T>
__device__ __forceinline__ void gemm_stage(_Float16 *dst, const T *src, int ld, int r0, int R, int s0, int s1,
                                           int kw, int tid) {
    constexpr int NIT = 64 * kGKS / 4 / kGT;     // items of four elements per thread at the full stage width
    const bool vec = sizeof(T) == 4 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0;
    const int per_row = kw / 4;                  // !TR: items per row; TR: 16 items per column
    const int items = TR ? 16 * kw : 64 * per_row;
    float4 v[NIT];
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int it = tid + i * kGT;
        const int r = TR ? 4 * (it % 16) : it / per_row, c = TR ? it / 16 : 4 * (it % per_row);
        const int rr = r0 + r, k = s0 + c;
        v[i] = float4{0.f, 0.f, 0.f, 0.f};
        if (it >= items) continue;
        if (!TR) {
            if (vec && rr < R && k + 3 < s1) {
                v[i] = *reinterpret_cast<const float4 *>(src + (int64_t)rr * ld + k);
            } else if (rr < R) {
                v[i].x = k < s1 ? ld_f(src, (int64_t)rr * ld + k) : 0.f;
                v[i].y = k + 1 < s1 ? ld_f(src, (int64_t)rr * ld + k + 1) : 0.f;
                v[i].z = k + 2 < s1 ? ld_f(src, (int64_t)rr * ld + k + 2) : 0.f;
                v[i].w = k + 3 < s1 ? ld_f(src, (int64_t)rr * ld + k + 3) : 0.f;
            }
        } else {
            if (vec && rr + 3 < R && k < s1) {
                v[i] = *reinterpret_cast<const float4 *>(src + (int64_t)k * ld + rr);
            } else if (k < s1) {
                v[i].x = rr < R ? ld_f(src, (int64_t)k * ld + rr) : 0.f;
                v[i].y = rr + 1 < R ? ld_f(src, (int64_t)k * ld + rr + 1) : 0.f;
                v[i].z = rr + 2 < R ? ld_f(src, (int64_t)k * ld + rr + 2) : 0.f;
                v[i].w = rr + 3 < R ? ld_f(src, (int64_t)k * ld + rr + 3) : 0.f;
            }
        }
    }
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int it = tid + i * kGT;
        if (it >= items) continue;
        const int r = TR ? 4 * (it % 16) : it / per_row, c = TR ? it / 16 : 4 * (it % per_row);
        if (!TR) {
            *reinterpret_cast<h4 *>(dst + r * kGS + c) =
                h4{(_Float16)v[i].x, (_Float16)v[i].y, (_Float16)v[i].z, (_Float16)v[i].w};
        } else {
            dst[r * kGS + c] = (_Float16)v[i].x;
            dst[(r + 1) * kGS + c] = (_Float16)v[i].y;
            dst[(r + 2) * kGS + c] = (_Float16)v[i].z;
            dst[(r + 3) * kGS + c] = (_Float16)v[i].w;
        }
    }
}

// C[M x N] = sum_k fp16(A(m, k)) fp16(B(n, k)), FP32 accumulation.
// A(m, k) = A[m lda + k] (TA false) or A[k lda + m] (TA true); same for B.
// Split K: block z covers k in [z kc, (z + 1) kc) and writes its slice of the
// sum to C + z M N (a workspace the split reduction then adds in z order).
// The block stages up to 256 of its k in LDS at once, then runs the MFMAs of
// those k-steps in order.
template <typename TAe, typename TBe, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kGT) void gemm_kernel(int M, int N, int K, const TAe *A, int lda,
                                                   const TBe *B, int ldb, float *C, int ldc, int kc, EpiArgs ep) {
    __shared__ __attribute__((aligned(16))) _Float16 as[64 * kGS];
    __shared__ __attribute__((aligned(16))) _Float16 bs[64 * kGS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int kb = blockIdx.z * kc, ke = kb + kc < K ? kb + kc : K;
    C += (int64_t)blockIdx.z * M * N;
    for (int s0 = kb; s0 < ke; s0 += kGKS) {
        const int s1 = s0 + kGKS < ke ? s0 + kGKS : ke;
        const int kw = (s1 - s0 + kGK - 1) / kGK * kGK;
        __syncthreads();
        gemm_stage<TA>(as, A, lda, m0, M, s0, s1, kw, tid);
        gemm_stage<TB>(bs, B, ldb, n0, N, s0, s1, kw, tid);
        __syncthreads();
        for (int kk = 0; kk < kw; kk += kGK) {
            h8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const h8 *>(&as[(wm + 16 * i + r16) * kGS + kk + 8 * q]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const h8 *>(&bs[(wn + 16 * j + r16) * kGS + kk + 8 * q]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * i + 4 * q + e, n = n0 + wn + 16 * j + r16;
                if (m < M && n < N) {
                    const int64_t o = (int64_t)m * ldc + n;
                    float v = acc[i][j][e];
                    if constexpr (EPI == kEpiBiasGelu) {
                        v += ep.b[n];
                        ep.H[o] = gelu(v);
                    } else if constexpr (EPI == kEpiGeluBack) {
                        v *= gelu_d(ep.Z[o]);
                    }
                    C[o] = v;
                }
            }
}

// out[i] = sum_z part[z n + i], z = 0 .. S-1 in order.
__global__ void reduce_slices_kernel(const float *part, int S, int64_t n, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < S; ++z) s += part[(int64_t)z * n + i];
        out[i] = s;
    }
}

// Plain launch (S = 1), or split K over S slices through the workspace ws
// (S M N floats) and an ordered reduction; C must then be dense (ldc = N).
// An epilogue other than kEpiNone needs S = 1 and dense outputs (ldc = N).
template <typename TAe, typename TBe, bool TA, bool TB, int EPI = kEpiNone>
hipError_t gemm(int M, int N, int K, const TAe *A, int lda, const TBe *B, int ldb, float *C, int ldc,
                hipStream_t s, int S = 1, float *ws = nullptr, EpiArgs ep = EpiArgs{nullptr, nullptr, nullptr}) {
    const int kc = S > 1 ? ((K + S - 1) / S + kGK - 1) / kGK * kGK : K;
    const int z = S > 1 ? (K + kc - 1) / kc : 1;
    if (EPI != kEpiNone && (z > 1 || ldc != N)) return hipErrorInvalidValue;
    const dim3 grid((N + 63) / 64, (M + 63) / 64, z);
    hipLaunchKernelGGL((gemm_kernel<TAe, TBe, TA, TB, EPI>), grid, dim3(kGT), 0, s, M, N, K, A, lda, B, ldb,
                       z > 1 ? ws : C, z > 1 ? N : ldc, kc, ep);
    if (z == 1) return hipGetLastError();
    const int64_t n = (int64_t)M * N;
    hipLaunchKernelGGL(reduce_slices_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       s, ws, z, n, C);
    return hipGetLastError();
}

// Head and loss: y_b = sum_j fp16(H_bj) fp16(w_j) + c.  Training: dy_b = 2 (y_b - t_b)
// (gradient of the sum of squares: the 1/B of the mean is applied to the
// finished gradient, which keeps the FP16 operands of the weight-gradient
// products out of the subnormal range) and dZ_bj = dy_b fp16(w_j) GELU'(Z_bj).
// One block per row.
__global__ __launch_bounds__(256) void head_kernel(const float *H, const float *Z, const float *w3, const float *b3,
                                                   const float *t, float *y, float *dy, float *dZ, float *loss_rows,
                                                   int Hn, int train) {
    const int b = blockIdx.x, tid = threadIdx.x;
    __shared__ float red[256];
    float s = 0.f;
    for (int j = tid; j < Hn; j += 256) s += (float)(_Float16)H[(int64_t)b * Hn + j] * (float)(_Float16)w3[j];
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    const float yb = red[0] + b3[0];
    if (tid == 0) y[b] = yb;
    if (!train) return;
    const float d = 2.f * (yb - t[b]);
    if (tid == 0) {
        dy[b] = d;
        loss_rows[b] = (yb - t[b]) * (yb - t[b]);
    }
    for (int j = tid; j < Hn; j += 256)
        dZ[(int64_t)b * Hn + j] = d * (float)(_Float16)w3[j] * gelu_d(Z[(int64_t)b * Hn + j]);
}

// Column sums with optional row weights: part[z][n] = sum over the rows of
// slice z of w_m f(X[m][n]), f = identity or FP16 rounding.  Block (x, z)
// covers 64 columns and the rows [z rc, (z + 1) rc); within a block each of
// kCsRows row groups sums its rows in order and the groups are added in
// order, and the slices are added in order by reduce_slices_kernel, so the
// result does not depend on scheduling.
constexpr int kCsRows = 16;

template <bool ROUND>
__global__ __launch_bounds__(64 * kCsRows) void colsum_kernel(const float *X, const float *w, int M, int N, int rc,
                                                              float *part) {
    __shared__ float acc[kCsRows][64];
    const int c = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int m0 = blockIdx.y * rc, m1 = m0 + rc < M ? m0 + rc : M;
    float s = 0.f;
    if (n < N)
        for (int m = m0 + rg; m < m1; m += kCsRows) {
            const float x = X[(int64_t)m * N + n];
            const float v = ROUND ? (float)(_Float16)x : x;
            s += w ? w[m] * v : v;
        }
    acc[rg][c] = s;
    __syncthreads();
    if (rg == 0 && n < N) {
        float t = 0.f;
        for (int g = 0; g < kCsRows; ++g) t += acc[g][c];
        part[(int64_t)blockIdx.y * N + n] = t;
    }
}

// db3 = sum_b dy_b and the mean of the per-row losses (also hist[*batch] when
// hist is set): one block, strided per-thread sums, then a fixed-order tree.
__global__ __launch_bounds__(1024) void head_sums_kernel(const float *dy, const float *lrow, int M, float *db3,
                                                         float *loss, float *hist, const int *batch) {
    __shared__ float a[1024], b[1024];
    const int t = threadIdx.x;
    float s = 0.f, l = 0.f;
    for (int m = t; m < M; m += 1024) {
        s += dy[m];
        l += lrow[m];
    }
    a[t] = s;
    b[t] = l;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (t < off) {
            a[t] += a[t + off];
            b[t] += b[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        *db3 = a[0];
        *loss = b[0] / (float)M;
        if (hist) hist[*batch] = b[0] / (float)M;
    }
}

// out = x * scale.
__global__ void scale_kernel(const float *x, int64_t n, float scale, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[i] * scale;
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

// Adam on all parameters (one flat FP32 array), step count in *step.
__global__ void adam_kernel(float *p, const float *g, float gscale, float *m, float *v, int64_t n, const int *step,
                            float lr, float b1, float b2, float eps) {
    const int t = *step + 1;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i] * gscale;
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void step_inc_kernel(int *step, int *batch) {
    *step += 1;
    *batch += 1;
}

// Mini-batch gather: rows perm[*batch * B + r] of the feature and target
// arrays.  An index outside [0, n) reads row 0 and sets *bad.
__global__ void gather_kernel(const float *X, const float *t, const int *perm, const int *batch, int B, int in,
                              int64_t n, float *Xb, float *tb, int *bad) {
    const int64_t total = (int64_t)B * in;
    const int64_t base = (int64_t)*batch * B;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / in), c = (int)(i % in);
        int64_t src = perm[base + r];
        if (src < 0 || src >= n) {
            *bad = 1;
            src = 0;
        }
        Xb[i] = X[src * in + c];
        if (c == 0) tb[r] = t[src];
    }
}

// Features: V^ = V e^{-i arg V_0} / |V|, interleaved (re, im), FP32.
__global__ void features_kernel(const double *V, int64_t n, int k, float *X) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const double *v = V + r * 2 * k;
        double nrm = 0.0;
        for (int a = 0; a < 2 * k; ++a) nrm += v[a] * v[a];
        nrm = sqrt(nrm);
        const double m0 = hypot(v[0], v[1]);
        const double cr = m0 > 0.0 ? v[0] / m0 : 1.0, ci = m0 > 0.0 ? -v[1] / m0 : 0.0;   // e^{-i arg V_0}
        const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
        X[r * 2 * k] = (float)(m0 * inv);                  // V_0 e^{-i arg V_0} = |V_0|: real
        X[r * 2 * k + 1] = 0.f;
        for (int a = 1; a < k; ++a) {
            const double re = v[2 * a], im = v[2 * a + 1];
            X[r * 2 * k + 2 * a] = (float)((re * cr - im * ci) * inv);
            X[r * 2 * k + 2 * a + 1] = (float)((re * ci + im * cr) * inv);
        }
    }
}

// Targets: t = ln(1 + NLL - min NLL) over finite values; a non-finite NLL gets
// the largest finite target + 1 (all zero when no value is finite).
__global__ void targets_kernel(const double *nll, int64_t n, float *t) {
    __shared__ double smin[256], smax[256];
    const int tid = threadIdx.x;
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = tid; i < n; i += 256)
        if (isfinite(nll[i])) {
            mn = fmin(mn, nll[i]);
            mx = fmax(mx, nll[i]);
        }
    smin[tid] = mn;
    smax[tid] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            smin[tid] = fmin(smin[tid], smin[tid + off]);
            smax[tid] = fmax(smax[tid], smax[tid + off]);
        }
        __syncthreads();
    }
    const double lo = smin[0], cap = log1p(smax[0] - smin[0]) + 1.0;
    const bool any = isfinite(lo);
    for (int64_t i = tid; i < n; i += 256)
        t[i] = !any ? 0.f : isfinite(nll[i]) ? (float)log1p(nll[i] - lo) : (float)cap;
}

// Top-k smallest (ties by index, NaN as +inf): each block sorts a chunk of
// kChunk (key, index) pairs in LDS (bitonic) and keeps its k best; rounds
// repeat on the survivors until one chunk is left.
constexpr int kChunk = 4096;

__device__ __forceinline__ bool less_kv(float ka, int ia, float kb, int ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__global__ __launch_bounds__(1024) void topk_chunk_kernel(const float *keys, const int *ids, int n, int k,
                                                          float *ok, int *oi) {
    __shared__ float key[kChunk];
    __shared__ int idx[kChunk];
    const int base = blockIdx.x * kChunk;
    for (int i = threadIdx.x; i < kChunk; i += blockDim.x) {
        const int g = base + i;
        const float v = g < n ? keys[g] : INFINITY;
        key[i] = isnan(v) ? INFINITY : v;
        idx[i] = g < n ? (ids ? ids[g] : g) : 0x7fffffff;
    }
    __syncthreads();
    for (int size = 2; size <= kChunk; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < kChunk; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const bool sw = up ? less_kv(key[j], idx[j], key[i], idx[i])
                                       : less_kv(key[i], idx[i], key[j], idx[j]);
                    if (sw) {
                        const float tk = key[i];
                        key[i] = key[j];
                        key[j] = tk;
                        const int ti = idx[i];
                        idx[i] = idx[j];
                        idx[j] = ti;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        ok[blockIdx.x * k + i] = key[i];
        oi[blockIdx.x * k + i] = idx[i];
    }
}

}  // namespace

// ------------------------------------------------------------------ host side
namespace {

// out[n] = sum_m w_m f(X[m][n]) through slices in the workspace ws (>= 16 N floats).
template <bool ROUND>
hipError_t colsum(const float *X, const float *w, int M, int N, float *out, float *ws, hipStream_t s) {
    const int S = std::max(1, std::min(16, (M + 63) / 64));
    const int rc = (M + S - 1) / S;
    hipLaunchKernelGGL((colsum_kernel<ROUND>), dim3((N + 63) / 64, S), dim3(64 * kCsRows), 0, s, X, w, M, N, rc, ws);
    hipLaunchKernelGGL(reduce_slices_kernel, dim3((N + 255) / 256), dim3(256), 0, s, ws, S, (int64_t)N, out);
    return hipGetLastError();
}

// Slices for a split-K weight-gradient product over K = B rows.
int ksplit(int K) { return std::max(1, std::min(16, K / 64)); }

}  // namespace

int64_t mlp_param_count(int in, int hidden) {
    return (int64_t)hidden * in + hidden + (int64_t)hidden * hidden + hidden + hidden + 1;
}

hipError_t mlp_features(const double *V, int64_t n, int k, float *X, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(features_kernel, dim3(blocks), dim3(256), 0, s, V, n, k, X);
    return hipGetLastError();
}

hipError_t mlp_targets(const double *nll, int64_t n, float *t, hipStream_t s) {
    hipLaunchKernelGGL(targets_kernel, dim3(1), dim3(256), 0, s, nll, n, t);
    return hipGetLastError();
}

// Forward pass over B rows of Xb into y; with train, the loss (and
// hist[*batch] if hist is set) and the gradient of the summed squared error
// into m.G.
hipError_t mlp_pass(const MlpBuffers &m, int B, const float *Xb, const float *tb, float *y, bool train, float *hist,
                    hipStream_t s) {
    const int in = m.in, H = m.hidden;
    const float *W1 = m.P, *b1 = W1 + (int64_t)H * in, *W2 = b1 + H, *b2 = W2 + (int64_t)H * H, *w3 = b2 + H,
                *b3 = w3 + H;
    float *gW1 = m.G, *gb1 = gW1 + (int64_t)H * in, *gW2 = gb1 + H, *gb2 = gW2 + (int64_t)H * H, *gw3 = gb2 + H,
          *gb3 = gw3 + H;
    hipError_t e;
    // Z = X W^T + b and H = GELU(Z), per layer (bias and activation in the GEMM epilogue)
    if ((e = gemm<float, float, false, false, kEpiBiasGelu>(B, H, in, Xb, in, W1, in, m.Z1, H, s, 1, nullptr,
                                                            EpiArgs{b1, m.H1, nullptr})) != hipSuccess)
        return e;
    if ((e = gemm<float, float, false, false, kEpiBiasGelu>(B, H, H, m.H1, H, W2, H, m.Z2, H, s, 1, nullptr,
                                                            EpiArgs{b2, m.H2, nullptr})) != hipSuccess)
        return e;
    hipLaunchKernelGGL(head_kernel, dim3(B), dim3(256), 0, s, m.H2, m.Z2, w3, b3, tb, y, m.dy, m.dZ2, m.lrow, H,
                       train ? 1 : 0);
    if (!train) return hipGetLastError();
    // dw3_j = sum_b dy_b fp16(H2_bj); db3 = sum_b dy_b and the mean loss
    if ((e = colsum<true>(m.H2, m.dy, B, H, gw3, m.ws, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(head_sums_kernel, dim3(1), dim3(1024), 0, s, m.dy, m.lrow, B, gb3, m.loss, hist, m.batch);
    // layer 2: dW2 = dZ2^T H1, db2 = column sums of dZ2, dZ1 = (dZ2 W2) GELU'(Z1)
    if ((e = gemm<float, float, true, true>(H, H, B, m.dZ2, H, m.H1, H, gW2, H, s, ksplit(B), m.ws)) != hipSuccess)
        return e;
    if ((e = colsum<false>(m.dZ2, nullptr, B, H, gb2, m.ws, s)) != hipSuccess) return e;
    if ((e = gemm<float, float, false, true, kEpiGeluBack>(B, H, H, m.dZ2, H, W2, H, m.dZ1, H, s, 1, nullptr,
                                                           EpiArgs{nullptr, nullptr, m.Z1})) != hipSuccess)
        return e;
    // layer 1: dW1 = dZ1^T X, db1 = column sums of dZ1
    if ((e = gemm<float, float, true, true>(H, in, B, m.dZ1, H, Xb, in, gW1, in, s, ksplit(B), m.ws)) != hipSuccess)
        return e;
    if ((e = colsum<false>(m.dZ1, nullptr, B, H, gb1, m.ws, s)) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t mlp_scale(const float *x, int64_t n, float scale, float *out, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(scale_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s, x, n, scale, out);
    return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers &m, float gscale, float lr, hipStream_t s) {
    const int blocks = (int)std::min<int64_t>((m.nparams + 255) / 256, 4096);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, s, m.P, m.G, gscale, m.M1, m.M2, m.nparams, m.step,
                       lr, 0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t mlp_gather(const MlpBuffers &m, const float *X, const float *t, int64_t n, const int *perm, int B,
                      hipStream_t s) {
    const int blocks = (int)std::min<int64_t>(((int64_t)B * m.in + 255) / 256, 4096);
    hipLaunchKernelGGL(gather_kernel, dim3(blocks), dim3(256), 0, s, X, t, perm, m.batch, B, m.in, n, m.Xb, m.tb,
                       m.bad);
    return hipGetLastError();
}

hipError_t mlp_step_inc(const MlpBuffers &m, hipStream_t s) {
    hipLaunchKernelGGL(step_inc_kernel, dim3(1), dim3(1), 0, s, m.step, m.batch);
    return hipGetLastError();
}

hipError_t mlp_set_int(int *p, int v, hipStream_t s) {
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

int topk_chunk() { return kChunk; }

size_t topk_scratch(int64_t n, int k) {
    const int64_t chunks = (n + kChunk - 1) / kChunk;
    return (size_t)std::max<int64_t>(chunks, 1) * k;
}

// Indices of the k smallest of n keys into out (k <= kChunk / 2); sk, si:
// two ping-pong scratch areas of topk_scratch(n, k) pairs each.
hipError_t mlp_topk(const float *keys, int64_t n, int k, float *sk[2], int *si[2], int *out, hipStream_t s) {
    if (k < 1 || k > kChunk / 2 || n < k) return hipErrorInvalidValue;
    const float *kin = keys;
    const int *iin = nullptr;
    int64_t m = n;
    int buf = 0;
    for (;;) {
        const int64_t chunks = (m + kChunk - 1) / kChunk;
        hipLaunchKernelGGL(topk_chunk_kernel, dim3((unsigned)chunks), dim3(1024), 0, s, kin, iin, (int)m, k, sk[buf],
                           si[buf]);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        kin = sk[buf];
        iin = si[buf];
        m = chunks * k;
        buf ^= 1;
        if (chunks == 1) break;
    }
    return hipMemcpyAsync(out, iin, sizeof(int) * k, hipMemcpyDeviceToDevice, s);
}

}  // namespace pwa
