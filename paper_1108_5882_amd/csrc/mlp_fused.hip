// Fused training pass of the surrogate network at hidden width 256: one
// launch computes, per slice of 16 mini-batch rows, the forward pass, the
// loss and every parameter gradient of the slice; a second launch adds the
// slices in order and applies Adam (or returns the summed gradient).  The
// arithmetic is that of the layer-by-layer kernels in mlp.hip: every matrix
// product rounds both operands to FP16 and accumulates in FP32
// (v_mfma_f32_16x16x32_f16), biases and activations are FP32, the head and
// the weight-3 gradient use the FP16-rounded activations.  Only the order in
// which the rows of a mini-batch are added differs (slices of 16 rows, added
// in slice order).
#include "internal.hpp"

namespace pwa {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));   // a register array of these stays in registers

constexpr int kFR = 16;                 // rows per slice (one workgroup)
constexpr int kFK = 32;                 // k of the row-sum MFMAs (rows kFR .. kFK - 1 are zero)
constexpr int kFH = 256;                // hidden width of the fused path
constexpr int kFT = 256;                // threads per workgroup
constexpr int kSH = kFH + 8;            // row stride (halfs) of [32][256] planes
constexpr int kST = kFK + 8;            // row stride (halfs) of transposed [256][32] planes

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

struct FusedArgs {
    const float *P;                     // parameters W1 [H][in], b1, W2 [H][H], b2, w3, b3
    const float *X, *t;                 // features [n][in] and targets [n]
    const int *perm;                    // null: rows 0 .. B-1 of X; else rows perm[*batch B + r]
    const int *batch;                   // mini-batch index (with perm)
    const int *step;                    // Adam steps taken
    int *tnext;                         // the step the following Adam update makes (*step + 1)
    int64_t n;
    int B, in;
    int64_t nparams;
    float *part;                        // [slice][nparams] gradient sums of the slice's rows
    float *lossp;                       // [slice] sum of the squared errors
    const _Float16 *w1h;                // fp16(W1) [256][INP] (zero past in)
    const _Float16 *w2h;                // fp16(W2) [256][256]
    const _Float16 *w2th;               // fp16(W2) transposed [256][256]
    int *bad;
};

// C[16 x 64] += A[16 x K] B[64 x K]^T, A and B FP16 in LDS with k contiguous
// (row strides sa, sb); wave w owns column tile w; item e of acc is row 4 q + e,
// column 16 w + r16 of the chunk.
__device__ __forceinline__ void chunk_mfma(const _Float16 *A, int sa, const _Float16 *B, int sb, int K, f4 &acc,
                                           int wave, int q, int r16) {
    for (int kk = 0; kk < K; kk += 32) {
        const h8 a = *reinterpret_cast<const h8 *>(A + r16 * sa + kk + 8 * q);
        const h8 b = *reinterpret_cast<const h8 *>(B + (16 * wave + r16) * sb + kk + 8 * q);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
    }
}

// A chunk of 64 rows of an FP16 matrix with row length W (halfs) moves from
// global memory through registers (issued early) into LDS rows of stride sd.
template <int W>
struct Chunk {
    static constexpr int N = 64 * W / 8 / kFT;          // 16-byte pieces per thread
    u4 v[N];
    __device__ __forceinline__ void load(const _Float16 *src, int r0, int tid) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int it = tid + i * kFT, r = it / (W / 8), c = 8 * (it % (W / 8));
            v[i] = *reinterpret_cast<const u4 *>(src + (int64_t)(r0 + r) * W + c);
        }
    }
    __device__ __forceinline__ void store(_Float16 *dst, int sd, int tid) const {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int it = tid + i * kFT, r = it / (W / 8), c = 8 * (it % (W / 8));
            *reinterpret_cast<u4 *>(dst + r * sd + c) = v[i];
        }
    }
};

template <int INP>
struct FusedSmem {
    static constexpr int SX = INP + 8;
    _Float16 xr[kFR * SX];              // X, rows
    _Float16 xt[INP * kST];             // X, transposed
    _Float16 h1r[kFR * kSH];            // fp16(H1), rows
    _Float16 h1t[kFH * kST];            // fp16(H1), transposed
    _Float16 d2r[kFR * kSH];            // fp16(dZ2), rows
    _Float16 d2t[kFH * kST];            // fp16(dZ2), transposed
    _Float16 hx[kFH * kST];             // fp16(H2) rows (first kFR * kSH), later fp16(dZ1) transposed
    _Float16 w[64 * (kFH + 8 > INP + 8 ? kFH + 8 : INP + 8)];   // one staged 64-row weight chunk
    float z1[kFR * kFH];                // Z1, later dZ1 (FP32)
    float z2[kFR * kFH];                // Z2 (FP32)
    float tgt[kFR], dy[kFR], lrow[kFR];
    int src[kFR];
};

// One workgroup per slice of 16 rows.
template <int INP>
__global__ __launch_bounds__(kFT) void mlp_fused_kernel(FusedArgs a) {
    static_assert(kFR * kSH <= kFH * kST, "H2 rows must fit in the dZ1 plane");
    __shared__ __attribute__((aligned(16))) FusedSmem<INP> sm;
    constexpr int SX = FusedSmem<INP>::SX;
    constexpr int SW = kFH + 8;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r16 = lane & 15;
    const int slice = blockIdx.x, in = a.in;
    const float *W1 = a.P, *b1 = W1 + (int64_t)kFH * in, *W2 = b1 + kFH, *b2 = W2 + (int64_t)kFH * kFH,
                *w3 = b2 + kFH, *b3 = w3 + kFH;
    float *G = a.part + (int64_t)slice * a.nparams;
    float *gW1 = G, *gb1 = gW1 + (int64_t)kFH * in, *gW2 = gb1 + kFH, *gb2 = gW2 + (int64_t)kFH * kFH,
          *gw3 = gb2 + kFH, *gb3 = gw3 + kFH;
    float *Z1 = sm.z1, *Z2 = sm.z2;
    const int rows = a.B - slice * kFR < kFR ? a.B - slice * kFR : kFR;

    if (slice == 0 && tid == 0) *a.tnext = *a.step + 1;   // for the Adam update of this pass
    // rows of the slice (a bad permutation entry reads row 0 and raises the flag)
    if (tid < kFR) {
        int64_t s = -1;
        if (tid < rows) {
            const int64_t gr = (int64_t)slice * kFR + tid;
            s = a.perm ? (int64_t)a.perm[(int64_t)(*a.batch) * a.B + gr] : gr;
            if (s < 0 || s >= a.n) {
                atomicOr(a.bad, 1);
                s = 0;
            }
        }
        sm.src[tid] = (int)s;
        sm.tgt[tid] = s >= 0 ? a.t[s] : 0.f;
    }
    // rows kFR .. kFK - 1 of the transposed planes are zero (k padding of the row sums)
    {
        const u4 z = u4{0u, 0u, 0u, 0u};
        for (int i = tid; i < kFH; i += kFT) {
            *reinterpret_cast<u4 *>(sm.h1t + i * kST + kFR) = z;
            *reinterpret_cast<u4 *>(sm.h1t + i * kST + kFR + 8) = z;
            *reinterpret_cast<u4 *>(sm.d2t + i * kST + kFR) = z;
            *reinterpret_cast<u4 *>(sm.d2t + i * kST + kFR + 8) = z;
        }
        for (int i = tid; i < INP; i += kFT) {
            *reinterpret_cast<u4 *>(sm.xt + i * kST + kFR) = z;
            *reinterpret_cast<u4 *>(sm.xt + i * kST + kFR + 8) = z;
        }
    }
    __syncthreads();
    // X rows and their transpose (zero past the slice's rows and past in)
    for (int it = tid; it < kFR * INP; it += kFT) {
        const int r = it / INP, c = it % INP;
        const int s = sm.src[r];
        const _Float16 v = (_Float16)((s >= 0 && c < in) ? a.X[(int64_t)s * in + c] : 0.f);
        sm.xr[r * SX + c] = v;
        sm.xt[c * kST + r] = v;
    }

    // layer 1: Z1 = X W1^T + b1, H1 = GELU(Z1), 64 features per chunk (the next
    // chunk's weights in flight while the current one is multiplied)
    {
        Chunk<INP> ck;
        ck.load(a.w1h, 0, tid);
        for (int f0 = 0; f0 < kFH; f0 += 64) {
            __syncthreads();
            ck.store(sm.w, SX, tid);
            __syncthreads();
            if (f0 + 64 < kFH) ck.load(a.w1h, f0 + 64, tid);
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            chunk_mfma(sm.xr, SX, sm.w, SX, INP, acc, wave, q, r16);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * q + e, f = f0 + 16 * wave + r16;
                    const float z = acc[e] + b1[f];
                    const _Float16 h = (_Float16)gelu(z);
                    Z1[r * kFH + f] = z;
                    sm.h1r[r * kSH + f] = h;
                    sm.h1t[f * kST + r] = h;
                }
        }
    }
    // layer 2: Z2 = H1 W2^T + b2, fp16(H2) rows into hx
    _Float16 *h2r = sm.hx;
    {
        Chunk<kFH> ck;
        ck.load(a.w2h, 0, tid);
        for (int f0 = 0; f0 < kFH; f0 += 64) {
            __syncthreads();
            ck.store(sm.w, SW, tid);
            __syncthreads();
            if (f0 + 64 < kFH) ck.load(a.w2h, f0 + 64, tid);
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            chunk_mfma(sm.h1r, kSH, sm.w, SW, kFH, acc, wave, q, r16);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * q + e, f = f0 + 16 * wave + r16;
                    const float z = acc[e] + b2[f];
                    Z2[r * kFH + f] = z;
                    h2r[r * kSH + f] = (_Float16)gelu(z);
                }
        }
    }
    __syncthreads();
    // head: y = fp16(H2) . fp16(w3) + b3 (16 lanes per row, lane-order sums), dy, loss
    {
        const int r = tid >> 4, l16 = tid & 15;
        float s = 0.f;
        for (int j = l16; j < kFH; j += 16) s += (float)h2r[r * kSH + j] * (float)(_Float16)w3[j];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        if (l16 == 0) {
            const float yb = s + b3[0];
            const bool ok = r < rows;
            sm.dy[r] = ok ? 2.f * (yb - sm.tgt[r]) : 0.f;
            sm.lrow[r] = ok ? (yb - sm.tgt[r]) * (yb - sm.tgt[r]) : 0.f;
        }
    }
    __syncthreads();
    // dZ2 = dy fp16(w3) GELU'(Z2) (rows and transpose); per feature j: db2, dw3; db3 and the loss
    {
        const int j = tid;
        const float wj = (float)(_Float16)w3[j];
        float sb = 0.f, sw = 0.f;
        for (int r0 = 0; r0 < kFR; r0 += 8) {
            float z2[8];                                // eight rows of the column's Z2
#pragma unroll
            for (int u = 0; u < 8; ++u) z2[u] = Z2[(r0 + u) * kFH + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = r0 + u;
                const float d = sm.dy[r] * wj * gelu_d(z2[u]);
                const _Float16 dh = (_Float16)d;
                sm.d2r[r * kSH + j] = dh;
                sm.d2t[j * kST + r] = dh;
                sb += d;
                sw += sm.dy[r] * (float)h2r[r * kSH + j];
            }
        }
        gb2[j] = sb;
        gw3[j] = sw;
        if (j == 0) {
            float sd = 0.f, sl = 0.f;
            for (int r = 0; r < kFR; ++r) {
                sd += sm.dy[r];
                sl += sm.lrow[r];
            }
            gb3[0] = sd;
            a.lossp[slice] = sl;
        }
    }
    __syncthreads();
    // dW2[i][j] = sum_r fp16(dZ2[r][i]) fp16(H1[r][j]): 256 tiles of 16 x 16, one MFMA each
    for (int tl = wave; tl < (kFH / 16) * (kFH / 16); tl += 4) {
        const int ti = tl / (kFH / 16), tj = tl % (kFH / 16);
        const h8 av = *reinterpret_cast<const h8 *>(sm.d2t + (16 * ti + r16) * kST + 8 * q);
        const h8 bv = *reinterpret_cast<const h8 *>(sm.h1t + (16 * tj + r16) * kST + 8 * q);
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) gW2[(int64_t)(16 * ti + 4 * q + e) * kFH + 16 * tj + r16] = d[e];
    }
    // dH1 = dZ2 W2 (rows of the transposed W2, 64 input features per chunk), dZ1 = dH1 GELU'(Z1)
    _Float16 *d1t = sm.hx;                              // H2 rows are no longer read
    for (int i = tid; i < kFH; i += kFT) {              // its k padding (H2 rows lay there)
        *reinterpret_cast<u4 *>(d1t + i * kST + kFR) = u4{0u, 0u, 0u, 0u};
        *reinterpret_cast<u4 *>(d1t + i * kST + kFR + 8) = u4{0u, 0u, 0u, 0u};
    }
    {
        Chunk<kFH> ck;
        ck.load(a.w2th, 0, tid);
        for (int c0 = 0; c0 < kFH; c0 += 64) {
            __syncthreads();
            ck.store(sm.w, SW, tid);
            __syncthreads();
            if (c0 + 64 < kFH) ck.load(a.w2th, c0 + 64, tid);
            f4 acc = f4{0.f, 0.f, 0.f, 0.f};
            chunk_mfma(sm.d2r, kSH, sm.w, SW, kFH, acc, wave, q, r16);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = 4 * q + e, i = c0 + 16 * wave + r16;
                    const float d = acc[e] * gelu_d(Z1[r * kFH + i]);
                    Z1[r * kFH + i] = d;                // dZ1 in place of Z1 (the same thread read it)
                    d1t[i * kST + r] = (_Float16)d;
                }
        }
    }
    __syncthreads();
    // db1[i] = sum_r dZ1[r][i]
    {
        const int i = tid;
        float s = 0.f;
        for (int r0 = 0; r0 < kFR; r0 += 8) {
            float d1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d1[u] = Z1[(r0 + u) * kFH + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += d1[u];
        }
        gb1[i] = s;
    }
    // dW1[i][c] = sum_r fp16(dZ1[r][i]) fp16(X[r][c])
    for (int tl = wave; tl < (kFH / 16) * (INP / 16); tl += 4) {
        const int ti = tl / (INP / 16), tc = tl % (INP / 16);
        const h8 av = *reinterpret_cast<const h8 *>(d1t + (16 * ti + r16) * kST + 8 * q);
        const h8 bv = *reinterpret_cast<const h8 *>(sm.xt + (16 * tc + r16) * kST + 8 * q);
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        const int c = 16 * tc + r16;
        if (c < in) {
#pragma unroll
            for (int e = 0; e < 4; ++e) gW1[(int64_t)(16 * ti + 4 * q + e) * in + c] = d[e];
        }
    }
}

// fp16 copies of W1 (rows padded to inp with zeros) and W2 (and its transpose).
__global__ void mlp_fused_weights_kernel(const float *P, int in, int inp, _Float16 *w1h, _Float16 *w2h,
                                         _Float16 *w2th) {
    const float *W1 = P, *W2 = P + (int64_t)kFH * in + kFH;
    const int n1 = kFH * inp, n2 = kFH * kFH;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1 + n2; i += gridDim.x * blockDim.x) {
        if (i < n1) {
            const int f = i / inp, c = i % inp;
            w1h[i] = (_Float16)(c < in ? W1[f * in + c] : 0.f);
        } else {
            const int j = i - n1, o = j / kFH, c = j % kFH;
            const _Float16 h = (_Float16)W2[j];
            w2h[j] = h;
            w2th[c * kFH + o] = h;
        }
    }
}

// Slice sums in slice order: G = sum_s part[s] (loss: sum_s lossp[s] / B, also
// hist[*batch]).  With Adam the sum times gscale updates P, M1, M2 at step
// *tnext (written by the slice pass) and the fp16 weight copies; workgroup 0
// then advances *step and *batch (no other workgroup reads them).
__global__ __launch_bounds__(256) void mlp_fused_reduce_kernel(const float *part, const float *lossp, int S,
                                                               int64_t np, int B, int in, int inp, float *G,
                                                               float *loss, float *hist, int adam, float *P,
                                                               float *M1, float *M2, float gscale, float lr,
                                                               _Float16 *w1h, _Float16 *w2h, _Float16 *w2th,
                                                               const int *tnext, int *step, int *batch) {
    const int t = adam ? *tnext : 0;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = adam ? 1.f - powf(b1, (float)t) : 1.f, c2 = adam ? 1.f - powf(b2, (float)t) : 1.f;
    const int64_t o2 = (int64_t)kFH * in + kFH, e2 = o2 + (int64_t)kFH * kFH;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        float g = 0.f;
        for (int s0 = 0; s0 < S; s0 += 32) {           // 32 slice loads in flight, added in slice order
            float v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) v[u] = s0 + u < S ? part[(int64_t)(s0 + u) * np + i] : 0.f;
#pragma unroll
            for (int u = 0; u < 32; ++u) g += v[u];
        }
        if (!adam) {
            G[i] = g;
        } else {
            const float gi = g * gscale;
            const float mi = b1 * M1[i] + (1.f - b1) * gi;
            const float vi = b2 * M2[i] + (1.f - b2) * gi * gi;
            M1[i] = mi;
            M2[i] = vi;
            const float p = P[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
            P[i] = p;
            if (i < (int64_t)kFH * in) {
                w1h[(i / in) * inp + i % in] = (_Float16)p;
            } else if (i >= o2 && i < e2) {
                const int64_t j = i - o2;
                w2h[j] = (_Float16)p;
                w2th[(j % kFH) * kFH + j / kFH] = (_Float16)p;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float l = 0.f;
        for (int s = 0; s < S; ++s) l += lossp[s];
        *loss = l / (float)B;
        if (hist) hist[*batch] = l / (float)B;
        if (adam) {
            *step = t;
            *batch += 1;
        }
    }
}

template <int INP>
hipError_t launch_fused(const FusedArgs &a, int S, hipStream_t s) {
    hipLaunchKernelGGL(mlp_fused_kernel<INP>, dim3(S), dim3(kFT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool mlp_fused_ok(const MlpBuffers &m) { return m.hidden == kFH && m.in >= 1 && m.in <= 128 && m.fpart; }

int mlp_fused_slices(int B) { return (B + kFR - 1) / kFR; }

size_t mlp_fused_wh_halfs() { return (size_t)kFH * 128 + 2 * (size_t)kFH * kFH; }

hipError_t mlp_fused_weights(const MlpBuffers &m, hipStream_t s) {
    if (!mlp_fused_ok(m)) return hipErrorInvalidValue;
    const int inp = (m.in + 31) / 32 * 32;
    hipLaunchKernelGGL(mlp_fused_weights_kernel, dim3(256), dim3(256), 0, s, m.P, m.in, inp, m.fwh,
                       m.fwh + (size_t)kFH * 128, m.fwh + (size_t)kFH * 128 + (size_t)kFH * kFH);
    return hipGetLastError();
}

hipError_t mlp_fused_pass(const MlpBuffers &m, int B, const float *X, const float *t, const int *perm, int64_t n,
                          bool adam, float gscale, float lr, float *hist, hipStream_t s) {
    if (!mlp_fused_ok(m) || B < 1 || B > m.max_batch) return hipErrorInvalidValue;
    const int S = mlp_fused_slices(B);
    const int inp = (m.in + 31) / 32 * 32;
    _Float16 *w1h = m.fwh, *w2h = w1h + (size_t)kFH * 128, *w2th = w2h + (size_t)kFH * kFH;
    FusedArgs a{m.P, X, t, perm, m.batch, m.step, m.ftnext, n, B, m.in, m.nparams, m.fpart, m.floss, w1h, w2h, w2th,
                m.bad};
    hipError_t e;
    e = inp == 32 ? launch_fused<32>(a, S, s)
        : inp == 64 ? launch_fused<64>(a, S, s)
        : inp == 96 ? launch_fused<96>(a, S, s)
                    : launch_fused<128>(a, S, s);
    if (e != hipSuccess) return e;
    const int blocks = (int)std::min<int64_t>((m.nparams + 255) / 256, 1024);
    hipLaunchKernelGGL(mlp_fused_reduce_kernel, dim3(blocks), dim3(256), 0, s, m.fpart, m.floss, S, m.nparams, B, m.in,
                       inp, m.G, m.loss, hist, adam ? 1 : 0, m.P, m.M1, m.M2, gscale, lr, w1h, w2h, w2th, m.ftnext,
                       m.step, m.batch);
    return hipGetLastError();
}

}  // namespace pwa
