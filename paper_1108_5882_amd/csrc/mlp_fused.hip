// Fused training pass of the surrogate network at hidden width 256, in two
// launches.  The row pass takes one workgroup per slice of 16 mini-batch rows:
// forward pass, loss, dZ2 and dZ1 of the slice, written to HBM as FP16 planes
// whose rows are features (X, H1, dZ2 and dZ1 transposed, mini-batch rows
// contiguous), and the slice's sums for the bias and head gradients.  The
// weight pass takes one workgroup per 16 x 16 tile of W2 or W1: dW = dZ^T H
// over every row of the mini-batch on the matrix cores (wave w takes the 32-row
// chunks w, w + 4, ..., the four waves' sums are added in wave order), then
// Adam on the tile (or the summed gradient); thirteen more workgroups add the
// slices' sums of the bias and head gradients and of the loss in a fixed order.
// The arithmetic is that of the layer-by-layer kernels in mlp.hip: every
// matrix product rounds both operands to FP16 and accumulates in FP32
// (v_mfma_f32_16x16x32_f16), biases and activations are FP32, the head and the
// weight-3 gradient use the FP16-rounded activations.  Only the order in which
// the rows of a mini-batch are added differs.
#include "internal.hpp"

namespace pwa {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));   // a register array of these stays in registers

constexpr int kFR = 16;                 // rows per slice (one workgroup of the row pass)
constexpr int kFH = 256;                // hidden width of the fused path
constexpr int kFT = 256;                // threads per workgroup
constexpr int kSH = kFH + 8;            // row stride (halfs) of [16][256] planes in LDS
constexpr int kFV = 3 * kFH + 8;        // floats per slice of vector sums: db1, db2, dw3, db3, loss

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
    _Float16 *act;                      // planes H1^T, dZ2^T, dZ1^T [256][bp] and X^T [INP][bp]
    int64_t bp;                         // their row stride: B rounded up to 32
    float *vsum;                        // [slice][kFV] vector sums of the slice's rows
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
struct RowSmem {
    static constexpr int SX = INP + 8;
    _Float16 xr[kFR * SX];              // X, rows
    _Float16 h1r[kFR * kSH];            // fp16(H1), rows
    _Float16 h2r[kFR * kSH];            // fp16(H2), rows
    _Float16 d2r[kFR * kSH];            // fp16(dZ2), rows
    _Float16 w[64 * (kFH + 8 > INP + 8 ? kFH + 8 : INP + 8)];   // one staged 64-row weight chunk
    float z1[kFR * kFH];                // Z1, later dZ1 (FP32)
    float z2[kFR * kFH];                // Z2 (FP32)
    float tgt[kFR], dy[kFR], lrow[kFR];
    int src[kFR];
};

// Row pass: one workgroup per slice of 16 rows.
template <int INP>
__global__ __launch_bounds__(kFT) void mlp_rows_kernel(FusedArgs a) {
    __shared__ __attribute__((aligned(16))) RowSmem<INP> sm;
    constexpr int SX = RowSmem<INP>::SX;
    constexpr int SW = kFH + 8;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r16 = lane & 15;
    const int slice = blockIdx.x, in = a.in;
    const float *W1 = a.P, *b1 = W1 + (int64_t)kFH * in, *b2 = b1 + kFH + (int64_t)kFH * kFH, *w3 = b2 + kFH,
                *b3 = w3 + kFH;
    const int64_t bp = a.bp, rb = (int64_t)slice * kFR;  // first plane column of the slice
    _Float16 *H1T = a.act, *D2T = H1T + kFH * bp, *D1T = D2T + kFH * bp, *XT = D1T + kFH * bp;
    float *V = a.vsum + (int64_t)slice * kFV;
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
    __syncthreads();
    // X rows (zero past the slice's rows and past in)
    for (int it = tid; it < kFR * INP; it += kFT) {
        const int r = it / INP, c = it % INP;
        const int s = sm.src[r];
        sm.xr[r * SX + c] = (_Float16)((s >= 0 && c < in) ? a.X[(int64_t)s * in + c] : 0.f);
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
            const int f = f0 + 16 * wave + r16;
            h4 hv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * q + e;
                const float z = acc[e] + b1[f];
                const _Float16 h = (_Float16)gelu(z);
                Z1[r * kFH + f] = z;
                sm.h1r[r * kSH + f] = h;
                hv[e] = h;
            }
            *reinterpret_cast<h4 *>(H1T + f * bp + rb + 4 * q) = hv;
        }
    }
    // layer 2: Z2 = H1 W2^T + b2, fp16(H2) rows
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
                sm.h2r[r * kSH + f] = (_Float16)gelu(z);
            }
        }
    }
    __syncthreads();
    // X transposed (the slice's 16 rows of feature c)
    if (tid < INP) {
        h8 lo, hi;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            lo[r] = sm.xr[r * SX + tid];
            hi[r] = sm.xr[(r + 8) * SX + tid];
        }
        *reinterpret_cast<h8 *>(XT + tid * bp + rb) = lo;
        *reinterpret_cast<h8 *>(XT + tid * bp + rb + 8) = hi;
    }
    // head: y = fp16(H2) . fp16(w3) + b3 (16 lanes per row, lane-order sums), dy, loss
    {
        const int r = tid >> 4, l16 = tid & 15;
        float s = 0.f;
        for (int j = l16; j < kFH; j += 16) s += (float)sm.h2r[r * kSH + j] * (float)(_Float16)w3[j];
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
    // dZ2 = dy fp16(w3) GELU'(Z2) (rows into LDS, the feature's 16 rows into
    // dZ2^T); per feature j the slice's db2 and dw3; db3 and the loss
    {
        const int j = tid;
        const float wj = (float)(_Float16)w3[j];
        float sb = 0.f, sw = 0.f;
        h8 dv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float z2[8];                                // eight rows of the column's Z2
#pragma unroll
            for (int u = 0; u < 8; ++u) z2[u] = Z2[(8 * h + u) * kFH + j];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int r = 8 * h + u;
                const float d = sm.dy[r] * wj * gelu_d(z2[u]);
                const _Float16 dh = (_Float16)d;
                sm.d2r[r * kSH + j] = dh;
                dv[h][u] = dh;
                sb += d;
                sw += sm.dy[r] * (float)sm.h2r[r * kSH + j];
            }
        }
        *reinterpret_cast<h8 *>(D2T + j * bp + rb) = dv[0];
        *reinterpret_cast<h8 *>(D2T + j * bp + rb + 8) = dv[1];
        V[kFH + j] = sb;
        V[2 * kFH + j] = sw;
        if (j == 0) {
            float sd = 0.f, sl = 0.f;
            for (int r = 0; r < kFR; ++r) {
                sd += sm.dy[r];
                sl += sm.lrow[r];
            }
            V[3 * kFH] = sd;
            V[3 * kFH + 1] = sl;
        }
    }
    // dH1 = dZ2 W2 (rows of the transposed W2, 64 input features per chunk),
    // dZ1 = dH1 GELU'(Z1) (in place of Z1, and the feature's rows into dZ1^T)
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
            const int i = c0 + 16 * wave + r16;
            h4 dv;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * q + e;
                const float d = acc[e] * gelu_d(Z1[r * kFH + i]);
                Z1[r * kFH + i] = d;                    // the same thread read it
                dv[e] = (_Float16)d;
            }
            *reinterpret_cast<h4 *>(D1T + i * bp + rb + 4 * q) = dv;
        }
    }
    __syncthreads();
    // db1[i] = sum_r dZ1[r][i]
    {
        const int i = tid;
        float s = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float d1[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d1[u] = Z1[(8 * h + u) * kFH + i];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += d1[u];
        }
        V[i] = s;
    }
}

struct UpdateArgs {
    const _Float16 *act;                // the row pass's planes
    int64_t bp;                         // their row stride
    int S;                              // slices (plane columns 16 S .. bp - 1 were not written)
    const float *vsum;                  // [slice][kFV]
    int in, B, adam;
    float gscale, lr;
    float *P, *M1, *M2, *G, *loss, *hist;
    _Float16 *w1h, *w2h, *w2th;
    const int *tnext;
    int *step, *batch;
};

// Adam on parameter i with gradient sum g (the update of mlp.hip's Adam
// kernel), from the parameter and moments read beforehand; or g into G.
// Returns the new parameter.
struct AdamIn {
    float p, m1, m2;
};
__device__ __forceinline__ AdamIn adam_load(const UpdateArgs &a, int64_t i) {
    return a.adam ? AdamIn{a.P[i], a.M1[i], a.M2[i]} : AdamIn{0.f, 0.f, 0.f};
}
__device__ __forceinline__ float apply(const UpdateArgs &a, int64_t i, const AdamIn &o, float g, float c1, float c2) {
    if (!a.adam) {
        a.G[i] = g;
        return 0.f;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g * a.gscale;
    const float mi = b1 * o.m1 + (1.f - b1) * gi;
    const float vi = b2 * o.m2 + (1.f - b2) * gi * gi;
    a.M1[i] = mi;
    a.M2[i] = vi;
    const float p = o.p - a.lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    a.P[i] = p;
    return p;
}

constexpr int kVecBlocks = 3 * (kFH / 64) + 1;   // workgroups of the vector sums

// Weight pass: workgroups 0 .. 255 the tiles of W2, then the tiles of W1
// (16 x INP/16), then the vector sums: 64 entries of b1, b2 or w3 per
// workgroup, and one for b3 and the loss.  A tile's Adam state is read before
// its products.  With Adam the tile workgroups refresh the fp16 weight copies;
// the loss workgroup writes the loss (hist[*batch] too) and advances *step and
// *batch (no other workgroup reads them).
template <int INP>
__global__ __launch_bounds__(kFT) void mlp_update_kernel(UpdateArgs a) {
    constexpr int N2 = (kFH / 16) * (kFH / 16), N1 = (kFH / 16) * (INP / 16);
    __shared__ float red[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, q = lane >> 4, r16 = lane & 15;
    const int t = a.adam ? *a.tnext : 0;
    const float c1 = a.adam ? 1.f - powf(0.9f, (float)t) : 1.f, c2 = a.adam ? 1.f - powf(0.999f, (float)t) : 1.f;
    const int in = a.in;
    const int64_t o2 = (int64_t)kFH * in + kFH, e2 = o2 + (int64_t)kFH * kFH;
    const int bt = blockIdx.x;
    if (bt < N2 + N1) {
        const int64_t bp = a.bp, rows = (int64_t)kFR * a.S;
        const _Float16 *H1T = a.act, *D2T = H1T + kFH * bp, *D1T = D2T + kFH * bp, *XT = D1T + kFH * bp;
        const bool w2 = bt < N2;
        const int ti = w2 ? bt / (kFH / 16) : (bt - N2) / (INP / 16);
        const int tj = w2 ? bt % (kFH / 16) : (bt - N2) % (INP / 16);
        // this thread's parameter: row tid / 16, column tid % 16 of the tile
        const int row = 16 * ti + (tid >> 4), col = 16 * tj + (tid & 15);
        const bool mine = w2 || col < in;
        const int64_t ip = w2 ? o2 + (int64_t)row * kFH + col : (int64_t)row * in + col;
        const AdamIn st = mine ? adam_load(a, ip) : AdamIn{0.f, 0.f, 0.f};
        const _Float16 *pa = (w2 ? D2T : D1T) + (16 * ti + r16) * bp + 8 * q;
        const _Float16 *pb = (w2 ? H1T : XT) + (16 * tj + r16) * bp + 8 * q;
        // D[i][j] = sum_r A[i][r] B[j][r] over the wave's chunks in order (rows
        // 16 S .. bp - 1 count as zero); four chunks' loads in flight
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
        for (int64_t k0 = 32 * wave; k0 < rows; k0 += 512) {
            h8 av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t kk = k0 + 128 * u;
                const bool ok = kk + 8 * q < rows;
                av[u] = ok ? *reinterpret_cast<const h8 *>(pa + kk) : h8{};
                bv[u] = ok ? *reinterpret_cast<const h8 *>(pb + kk) : h8{};
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[u], bv[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) red[wave][(4 * q + e) * 16 + r16] = acc[e];
        __syncthreads();
        const float g = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
        if (!mine) return;
        const float p = apply(a, ip, st, g, c1, c2);
        if (a.adam) {
            if (w2) {
                a.w2h[row * kFH + col] = (_Float16)p;
                a.w2th[col * kFH + row] = (_Float16)p;
            } else {
                a.w1h[row * INP + col] = (_Float16)p;
            }
        }
        return;
    }
    // vector sums: entry c (64 per workgroup) of vector v (db1, db2, dw3; v = 3:
    // db3 and the loss); wave w adds slices w, w + 4, ... in order (sixteen
    // loads in flight), the waves' sums are added in wave order
    const int vb = bt - N2 - N1, v = vb / (kFH / 64), c = 64 * (vb % (kFH / 64)) + lane;
    const bool live = v < 3 || c < 2;
    const int64_t off = (int64_t)v * kFH + (live ? c : 0);
    const int64_t ip = v == 0 ? (int64_t)kFH * in + c : v == 1 ? e2 + c : v == 2 ? e2 + kFH + c : e2 + 2 * kFH;
    const bool param = live && !(v == 3 && c == 1);
    const AdamIn st = param && wave == 0 ? adam_load(a, ip) : AdamIn{0.f, 0.f, 0.f};
    float sum = 0.f;
    for (int s0 = wave; s0 < a.S; s0 += 64) {
        float x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int sl = s0 + 4 * u;
            x[u] = a.vsum[(int64_t)(sl < a.S ? sl : a.S - 1) * kFV + off];
            if (sl >= a.S) x[u] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) sum += x[u];
    }
    red[wave][lane] = sum;
    __syncthreads();
    if (wave != 0 || !live) return;
    const float g = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    if (param) {
        apply(a, ip, st, g, c1, c2);
        return;
    }
    *a.loss = g / (float)a.B;                           // v = 3, c = 1: the loss
    if (a.hist) a.hist[*a.batch] = g / (float)a.B;
    if (a.adam) {
        *a.step = t;
        *a.batch += 1;
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

template <int INP>
hipError_t launch_fused(const FusedArgs &a, const UpdateArgs &u, int S, hipStream_t s) {
    hipLaunchKernelGGL(mlp_rows_kernel<INP>, dim3(S), dim3(kFT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int blocks = (kFH / 16) * (kFH / 16) + (kFH / 16) * (INP / 16) + kVecBlocks;
    hipLaunchKernelGGL(mlp_update_kernel<INP>, dim3(blocks), dim3(kFT), 0, s, u);
    return hipGetLastError();
}

int64_t plane_stride(int B) { return ((int64_t)B + 31) / 32 * 32; }

}  // namespace

bool mlp_fused_ok(const MlpBuffers &m) { return m.hidden == kFH && m.in >= 1 && m.in <= 128 && m.fact; }

int mlp_fused_slices(int B) { return (B + kFR - 1) / kFR; }

size_t mlp_fused_wh_halfs() { return (size_t)kFH * 128 + 2 * (size_t)kFH * kFH; }

size_t mlp_fused_act_halfs(int max_batch) { return (size_t)(3 * kFH + 128) * (size_t)plane_stride(max_batch); }

size_t mlp_fused_vec_floats(int max_batch) { return (size_t)mlp_fused_slices(max_batch) * kFV; }

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
    const int64_t bp = plane_stride(B);
    _Float16 *w1h = m.fwh, *w2h = w1h + (size_t)kFH * 128, *w2th = w2h + (size_t)kFH * kFH;
    const FusedArgs a{m.P, X, t, perm, m.batch, m.step, m.ftnext, n, B, m.in, m.fact, bp, m.fvec, w1h, w2h, w2th,
                      m.bad};
    const UpdateArgs u{m.fact, bp,   S,      m.fvec, m.in, B,       adam ? 1 : 0, gscale,  lr,     m.P,
                       m.M1,   m.M2, m.G,    m.loss, hist, w1h,     w2h,          w2th,    m.ftnext, m.step,
                       m.batch};
    return inp == 32   ? launch_fused<32>(a, u, S, s)
           : inp == 64 ? launch_fused<64>(a, u, S, s)
           : inp == 96 ? launch_fused<96>(a, u, S, s)
                       : launch_fused<128>(a, u, S, s);
}

}  // namespace pwa
