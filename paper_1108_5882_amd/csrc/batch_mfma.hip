// Many production vectors at once on the matrix cores (Berger, Section 2:
// repeated fits from many starting points; Eq. 1-3 for each vector).
//
// For nv vectors the per-event coherent sums of all vectors form a dense
// contraction: with A_r the N x 2K real view of the amplitude rows
// (re, im interleaved) and W the 2K x 2nv real matrix whose columns for V_b
// are (Re V_b, -Im V_b) and (Im V_b, Re V_b) interleaved per wave,
//     Z = A_r W            (Re z_ib, Im z_ib in columns 2b, 2b + 1).
// The adjoint sums are a second contraction over events,
//     P = U^T A_r,  U_ib = z_ib / I_ib (data) or w_i z_ib (MC),
//     Re G_ba = P[ur_b, 2a] + P[ui_b, 2a+1],  Im G_ba = P[ui_b, 2a] - P[ur_b, 2a+1].
// Both run on v_mfma_f32_16x16x32_* in one kernel per event tile; U never
// leaves registers: the forward's output layout is the adjoint's A operand
// once the adjoint's event order is permuted the same way in both operands.
//
// Operand planes: the split amplitudes do not depend on V, so they are formed
// once per sample (batch_planes_kernel) in the order and layout the tile's LDS
// buffers take them, 32-event tiles one after another; per tile a block
// copies them to LDS with 16-byte loads and stores and no conversion.
//
// Arithmetic (split): the forward uses two-term FP16 splits (hi + lo) of the
// amplitudes, scaled by a power of two per wave, and of W, scaled by a power
// of two per column: products hi*hi + hi*lo + lo*hi, 22-bit operands.  The
// adjoint uses two-term BF16 splits of U and of the amplitudes (BF16 keeps
// FP32's range, so the unbounded z/I needs no scale): 3 products.  MFMA
// accumulation is FP32 within a block; each block covers at most
// kTilesPerBlock tiles of one sample (spread evenly over whole rounds of
// compute units) and writes FP64 partials per vector,
// which a second kernel adds in block order (FP64) before forming NLL and
// gradient per vector.
#include "internal.hpp"

#include <algorithm>
#include <cmath>

// v_writelane_b32 (the LLVM intrinsic): writes a wave-uniform value into one lane
// of a register, leaving the other lanes as they are
__device__ unsigned writelane_u32(unsigned v, int lane, unsigned old) __asm("llvm.amdgcn.writelane.i32");

namespace pwa {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int kTile = 32;          // events per tile (two 16-row MFMA tiles)
constexpr int kWaves = 8;          // waves per block
constexpr int kThreads = 64 * kWaves;

__device__ __forceinline__ int dpp_xor1(int x) {
    return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
}
__device__ __forceinline__ float xor1_f(float x) { return __int_as_float(dpp_xor1(__float_as_int(x))); }

// Block b covers tiles [b tpb, (b + 1) tpb) of one segment (SEG: 0 data,
// 1 MC) for the vectors of blockIdx.y; each wave takes VPW = 8 CT vectors
// (2 CT real columns in CT column tiles: re and im of 16 vectors per tile
// pair).  Lanes of vectors past nv compute on zero weights and are never
// written out; only the last, partial tile of the data segment masks events
// (an absent data row would give z = 0 and a non-finite z / I, while an absent
// MC row has weight 0).
template <int KS, int CT>
struct BatchSmem {
    static constexpr int K2 = 32 * KS;          // padded real width
    // row stride (halfs) of the row-major FP16 planes: 16 halfs of padding (measured:
    // fewer LDS bank conflicts than 8 or 24, none is worse by 3.5x)
    static constexpr int RS16 = K2 + 16;
    static constexpr int RST = kTile + 8;       // row stride (bf16) of the transposed planes (16-byte rows)
    _Float16 ah[kTile * RS16];
    _Float16 al[kTile * RS16];
    __bf16 bh[K2 * RST];
    __bf16 bl[K2 * RST];
    float wts[kTile];
};

// Two LDS buffers (one barrier per tile: the next tile is staged into the
// other buffer after the current one is computed) when they fit in 64 KB.
template <int KS, int CT>
constexpr int batch_buffers() { return 2 * sizeof(BatchSmem<KS, CT>) <= 64 * 1024 ? 2 : 1; }

// REF (data segment only): events whose coherent sum is small against the
// bound |z| <= |V| |A_i| (|Z'|^2 < c^2 t_v^2 |V|^2 |A_i|^2, c^2 = p.cthr2) are
// left out of the sums and marked in p.flags, one 64-bit lane mask per
// (vector group, tile, group g, rt, e), in that order of significance, so the
// words of one vector group over consecutive tiles are contiguous;
// batch_refine_kernel adds them exactly.
template <int KS, int CT, int SEG, bool REF>
__device__ __forceinline__ void batch_block(const BatchArgs &p, BatchSmem<KS, CT> *bufs, int bseg) {
    constexpr int NB = batch_buffers<KS, CT>();
    constexpr int kVPerWave = 8 * CT;
    constexpr int K2 = BatchSmem<KS, CT>::K2;
    constexpr int RS16 = BatchSmem<KS, CT>::RS16;
    constexpr int RST = BatchSmem<KS, CT>::RST;
    constexpr int kChunks = 16 * K2;            // 16-byte chunks of a tile's four planes
    constexpr int kPer = (kChunks + kThreads - 1) / kThreads;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int64_t n = p.n[SEG];
    const float *A = p.A[SEG];
    const float *w = SEG ? p.w : nullptr;
    const int64_t tile0 = (int64_t)bseg * p.tpb;
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t tile1 = tile0 + p.tpb < ntiles ? tile0 + p.tpb : ntiles;
    const int vg = (int)blockIdx.y * kWaves + wave;          // this wave's vector group
    const int v0 = vg * kVPerWave;
    const bool active = v0 < p.nv;                           // wave-uniform
    constexpr bool kRef = REF && SEG == 0;
    // flag thresholds of this lane's vectors: c^2 t_v^2 |V|^2 (-1 for vectors past nv),
    // and 1 / t_v^2 (a power of two): the log is taken of the unscaled I = I' / t_v^2,
    // whose magnitude keeps the FP32 log and the FP32 tile sums accurate
    float thr[CT / 2], inv_t2[CT / 2];
#pragma unroll
    for (int g = 0; g < CT / 2; ++g) {
        thr[g] = -1.f;
        inv_t2[g] = 1.f;
        const int v = v0 + 16 * g + r16;
        if (SEG == 0 && v < p.nv) inv_t2[g] = (float)(1.0 / (p.vscale[v] * p.vscale[v]));
        if (kRef && v < p.nv) {
            const double *Vv = p.V + (int64_t)v * p.vstride;
            double n2 = 0.0;
            for (int a = 0; a < 2 * p.k; ++a) n2 += Vv[a] * Vv[a];
            thr[g] = (float)((double)p.cthr2 * p.vscale[v] * p.vscale[v] * n2);
        }
    }

    // forward weights of this wave's vectors, fragment order [hi/lo][ct][ks][lane]
    h8 wh[CT][KS], wl[CT][KS];
    {
        const h8 *src = reinterpret_cast<const h8 *>(p.wfrag) + (int64_t)vg * 2 * CT * KS * 64;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                wh[ct][ks] = src[((0 * CT + ct) * KS + ks) * 64 + lane];
                wl[ct][ks] = src[((1 * CT + ct) * KS + ks) * 64 + lane];
            }
    }

    // adjoint accumulators D[ct][rtile]: lane holds rows 4q+e (columns of U) x col r16 (real)
    f4 D[CT][2 * KS];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int rt = 0; rt < 2 * KS; ++rt) D[ct][rt] = f4{0.f, 0.f, 0.f, 0.f};
    double tsum[CT / 2];            // per lane: sum over its events for vectors 16g + r16
#pragma unroll
    for (int g = 0; g < CT / 2; ++g) tsum[g] = 0.0;

    const int nreal = 2 * p.k;                      // real columns present in a row
    // The next tile's operand planes are loaded into registers while the current
    // tile is computed; each thread holds kPer 16-byte chunks and one MC weight.
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    const u4 *planes = static_cast<const u4 *>(p.planes[SEG]);
    u4 xr[kPer];
    float wr = 0.f;
    auto load_tile = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int c = tid + i * kThreads;
            if (c < kChunks) {
                typedef const u4 __attribute__((address_space(1))) *gptr;
                xr[i] = __builtin_nontemporal_load((gptr)(planes + t * kChunks + c));
            }
        }
        if ((SEG || kRef) && tid < kTile) {
            const int64_t row = t * kTile + tid;
            wr = row < n ? (SEG ? (w ? w[row] : 1.f) : p.rnorm[row]) : 0.f;
        }
    };

    // epilogue of one tile: per (event, vector) I, log2 I (data) or w I (MC),
    // and U = z / I (data) or w z (MC), split into BF16 hi/lo in the adjoint's
    // operand order (slot 4 rt + e holds event 16 rt + 4 q + e)
    // (column group g: column tiles 2g and 2g + 1, vectors 16 g + r16)
    auto epilogue = [&](const float (&wv)[8], const f4 (&Z)[2][CT], b8 (&uh)[CT], b8 (&ul)[CT], int nvalid,
                        int64_t t, const int g) {
        {
            float ts = 0.f;
            // the flag masks of (g, slot): with one k-step (KS = 1) lane `slot` gathers
            // them for one store per group; with more, registers are short (the
            // gather costs spills) and every lane stores each (wave-uniform) mask to
            // its word, one store instruction with no branch around it (a store by
            // lane 0 alone put an exec-mask branch per slot into the epilogue, whose
            // blocks the scheduler cannot interleave matrix products across)
            unsigned fw_lo = 0u, fw_hi = 0u;
#pragma unroll
            for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int slot = 4 * rt + e;
                    const float zr = Z[rt][2 * g][e], zi = Z[rt][2 * g + 1][e];
                    const float I = fmaf(zr, zr, zi * zi);
                    float ur, ui;
                    if (SEG == 0) {
                        const bool absent = nvalid < kTile && 16 * rt + 4 * q + e >= nvalid;
                        const bool flag = kRef && !absent && I < thr[g] * wv[slot];
                        if (kRef) {
                            const unsigned long long mask = __ballot(flag);
                            if constexpr (KS == 1) {
                                fw_lo = writelane_u32((unsigned)mask, slot, fw_lo);
                                fw_hi = writelane_u32((unsigned)(mask >> 32), slot, fw_hi);
                            } else {
                                p.flags[((int64_t)vg * ntiles + t) * (8 * (CT / 2)) + 8 * g + slot] = mask;
                            }
                        }
                        if (absent || flag) {
                            ur = ui = 0.f;
                        } else {
                            ts += __log2f(I * inv_t2[g]);
                            const float rI = __builtin_amdgcn_rcpf(I);
                            ur = zr * rI;
                            ui = zi * rI;
                        }
                    } else {
                        ts = fmaf(wv[slot], I, ts);
                        ur = wv[slot] * zr;
                        ui = wv[slot] * zi;
                    }
                    const __bf16 hr = (__bf16)ur, hi_ = (__bf16)ui;
                    uh[2 * g][slot] = hr;
                    uh[2 * g + 1][slot] = hi_;
                    ul[2 * g][slot] = (__bf16)(ur - (float)hr);
                    ul[2 * g + 1][slot] = (__bf16)(ui - (float)hi_);
                }
            tsum[g] += (double)ts;
            if (kRef && KS == 1 && lane < 8)
                p.flags[((int64_t)vg * ntiles + t) * (8 * (CT / 2)) + 8 * g + lane] =
                    ((unsigned long long)fw_hi << 32) | fw_lo;
        }
    };

    // stage a tile from the registers into buffer b: plane 0 / 1 are the FP16 hi /
    // lo row-major planes (K2 halfs per event), plane 2 / 3 the BF16 hi / lo
    // transposed planes (32 events per real column, in the adjoint's operand
    // order); each 16-byte chunk goes to its place in the padded LDS rows
    auto stage = [&](BatchSmem<KS, CT> &b) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int c = tid + i * kThreads;
            if (c < kChunks) {
                const int plane = c / (4 * K2), u = 8 * (c % (4 * K2));
                u4 *dst;
                if (plane < 2) {
                    const int e = u / K2, r = u % K2;
                    dst = reinterpret_cast<u4 *>((plane == 0 ? b.ah : b.al) + e * RS16 + r);
                } else {
                    const int rr = u / kTile, pos = u % kTile;
                    dst = reinterpret_cast<u4 *>((plane == 2 ? b.bh : b.bl) + rr * RST + pos);
                }
                *dst = xr[i];
            }
        }
        if ((SEG || kRef) && tid < kTile) b.wts[tid] = wr;
    };

    // forward, epilogue and adjoint of the tile in buffer sm
    // forward products of column group g only (used when the groups are interleaved)
    auto forward_g = [&](const BatchSmem<KS, CT> &sm, f4 (&Z)[2][CT], const int g) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                const int off = (16 * rt + r16) * RS16 + 32 * ks + 8 * q;
                const h8 a_h = *reinterpret_cast<const h8 *>(&sm.ah[off]);
                const h8 a_l = *reinterpret_cast<const h8 *>(&sm.al[off]);
#pragma unroll
                for (int ct = 2 * g; ct < 2 * g + 2; ++ct) {
                    Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, wh[ct][ks], Z[rt][ct], 0, 0, 0);
                    Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, wl[ct][ks], Z[rt][ct], 0, 0, 0);
                    Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, wh[ct][ks], Z[rt][ct], 0, 0, 0);
                }
            }
    };
    // adjoint D[ct][rt] += U^T (16 columns x 32 events) . A (32 events x 16 reals) for the
    // column tiles [c0, c1)
    auto adjoint = [&](const BatchSmem<KS, CT> &sm, const b8 (&uh)[CT], const b8 (&ul)[CT], const int c0,
                       const int c1) {
#pragma unroll
        for (int rt = 0; rt < 2 * KS; ++rt) {
            const int rr = 16 * rt + r16;
            const b8 b_h = *reinterpret_cast<const b8 *>(&sm.bh[rr * RST + 8 * q]);
            const b8 b_l = *reinterpret_cast<const b8 *>(&sm.bl[rr * RST + 8 * q]);
#pragma unroll
            for (int ct = c0; ct < c1; ++ct) {
                D[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uh[ct], b_h, D[ct][rt], 0, 0, 0);
                D[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(uh[ct], b_l, D[ct][rt], 0, 0, 0);
                D[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ul[ct], b_h, D[ct][rt], 0, 0, 0);
            }
        }
    };

    // one tile; nvalid < kTile only for the data segment's last tile
    auto tile_body = [&](const BatchSmem<KS, CT> &sm, int64_t t, const int nvalid) __attribute__((always_inline)) {
        f4 Z[2][CT];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) Z[rt][ct] = f4{0.f, 0.f, 0.f, 0.f};
        b8 uh[CT], ul[CT];
        float wv[8];                // MC weights, or the rows' |A|^2 when flagging
        auto load_wv = [&]() __attribute__((always_inline)) {
            if (SEG || kRef) {
                const f4 w0 = *reinterpret_cast<const f4 *>(&sm.wts[4 * q]);
                const f4 w1 = *reinterpret_cast<const f4 *>(&sm.wts[16 + 4 * q]);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    wv[e] = w0[e];
                    wv[4 + e] = w1[e];
                }
            }
        };

        if constexpr (KS == 1 || CT < 4) {
            // forward of all column tiles (one A fragment load each), epilogue, adjoint
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int rt = 0; rt < 2; ++rt) {
                    const int off = (16 * rt + r16) * RS16 + 32 * ks + 8 * q;
                    const h8 a_h = *reinterpret_cast<const h8 *>(&sm.ah[off]);
                    const h8 a_l = *reinterpret_cast<const h8 *>(&sm.al[off]);
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) {
                        Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, wh[ct][ks], Z[rt][ct], 0, 0, 0);
                        Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, wl[ct][ks], Z[rt][ct], 0, 0, 0);
                        Z[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, wh[ct][ks], Z[rt][ct], 0, 0, 0);
                    }
                }
            load_wv();
            if (nvalid < kTile) {
#pragma unroll
                for (int g = 0; g < CT / 2; ++g) epilogue(wv, Z, uh, ul, nvalid, t, g);
            } else {
#pragma unroll
                for (int g = 0; g < CT / 2; ++g) epilogue(wv, Z, uh, ul, kTile, t, g);
            }
            adjoint(sm, uh, ul, 0, CT);
        } else {
            // two column groups with two or more k-steps: the matrix products of one
            // group are interleaved with the vector epilogue of the other (F0 | F1 with
            // E0 | A0 with E1 | A1), one product per three vector instructions; the two
            // waves sharing a SIMD otherwise run the same phase of a tile
            constexpr int kM = 12 * KS;                 // products per group and direction
            forward_g(sm, Z, 0);
            forward_g(sm, Z, 1);
            load_wv();
            epilogue(wv, Z, uh, ul, nvalid, t, 0);
            adjoint(sm, uh, ul, 0, 2);
            epilogue(wv, Z, uh, ul, nvalid, t, 1);
            adjoint(sm, uh, ul, 2, 4);
#pragma unroll
            for (int i = 0; i < kM; ++i) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
            for (int i = 0; i < 2 * kM; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
            }
#pragma unroll
            for (int i = 0; i < kM; ++i) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
    };
    auto compute = [&](const BatchSmem<KS, CT> &sm, int64_t t) {
        const int64_t left = n - t * kTile;
        tile_body(sm, t, (SEG == 0 && left < kTile) ? (int)left : kTile);
    };

    if (tile0 < tile1) load_tile(tile0);
    if (NB == 2) {
        // stage the first tile, then per tile: compute it, stage the next one
        // into the other buffer, load the one after into registers, one barrier
        if (tile0 < tile1) {
            stage(bufs[0]);
            if (tile0 + 1 < tile1) load_tile(tile0 + 1);
        }
        __syncthreads();
        for (int64_t t = tile0; t < tile1; ++t) {
            const int cur = (int)((t - tile0) & 1);
            if (active) compute(bufs[cur], t);
            if (t + 1 < tile1) {
                stage(bufs[cur ^ 1]);
                if (t + 2 < tile1) load_tile(t + 2);
            }
            __syncthreads();
        }
    } else {
        for (int64_t t = tile0; t < tile1; ++t) {
            __syncthreads();
            stage(bufs[0]);
            __syncthreads();
            if (t + 1 < tile1) load_tile(t + 1);
            if (active) compute(bufs[0], t);
        }
    }
    if (!active) return;

    // ---- per-vector scalar sums: lanes r16, r16 + 16, r16 + 32, r16 + 48 share a vector
#pragma unroll
    for (int g = 0; g < CT / 2; ++g) {
        tsum[g] += __shfl_xor(tsum[g], 16);
        tsum[g] += __shfl_xor(tsum[g], 32);
    }
    // partial layout [v][block][1 + 2 ld]: [0] scalar, [1 + 2a + c] complex sums
    const int pst = p.pstride;
    const int nblk = p.nb[0] + p.nb[1];
    if (q == 0) {
#pragma unroll
        for (int g = 0; g < CT / 2; ++g) {
            const int v = v0 + 16 * g + r16;
            if (v < p.nv) p.partials[((int64_t)v * nblk + blockIdx.x) * pst] = tsum[g];
        }
    }
    // gradient sums: lane pairs (2a, 2a+1) in r16 hold the re and im real rows of wave a
#pragma unroll
    for (int g = 0; g < CT / 2; ++g)
#pragma unroll
        for (int rt = 0; rt < 2 * KS; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float pr = D[2 * g][rt][e];       // P[ur_v, real r]
                const float pi = D[2 * g + 1][rt][e];   // P[ui_v, real r]
                const float pr_o = xor1_f(pr), pi_o = xor1_f(pi);   // the odd real row
                const int v = v0 + 16 * g + 4 * q + e;
                const int rr = 16 * rt + r16;
                if ((r16 & 1) == 0 && v < p.nv && rr < nreal) {
                    const int a = rr >> 1;
                    double *dst = p.partials + ((int64_t)v * nblk + blockIdx.x) * pst + 1 + 2 * a;
                    dst[0] = (double)pr + (double)pi_o;      // Re G = P[ur, 2a] + P[ui, 2a+1]
                    dst[1] = (double)pi - (double)pr_o;      // Im G = P[ui, 2a] - P[ur, 2a+1]
                }
            }
}

template <int KS, int CT, bool REF>
__global__ __launch_bounds__(kThreads) void nll_batch_kernel(BatchArgs p) {
    __shared__ __attribute__((aligned(16))) BatchSmem<KS, CT> bufs[batch_buffers<KS, CT>()];
    if ((int)blockIdx.x < p.nb[0])
        batch_block<KS, CT, 0, REF>(p, bufs, (int)blockIdx.x);
    else
        batch_block<KS, CT, 1, REF>(p, bufs, (int)blockIdx.x - p.nb[0]);
}

// Exact terms of the flagged data events: block (b, y) and its wave w take the
// flag words of data block b's tiles for vector group 8 y + w, in tile, word and
// bit order, and add each flagged event's terms, in the units of the block
// partials (log2 I, conj(A) z / (I t_v)), to the partial of its
// vector and block: every partial is updated by one wave, in a fixed order.
// z is formed in FP64 from the FP32 amplitudes (one wave per event, lanes over
// waves a), like the single-V path.
template <int CT>
__global__ __launch_bounds__(kThreads) void batch_refine_kernel(BatchArgs p) {
    constexpr int kVPerWave = 8 * CT;
    constexpr int kWords = 8 * (CT / 2);
    constexpr int kLoads = 4;                       // flag words in flight per lane
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int vg = (int)blockIdx.y * kWaves + wave;
    const int v0 = vg * kVPerWave;
    if (v0 >= p.nv) return;
    const int64_t n = p.n[0];
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t tile0 = (int64_t)blockIdx.x * p.tpb;
    const int64_t tile1 = tile0 + p.tpb < ntiles ? tile0 + p.tpb : ntiles;
    const int nblk = p.nb[0] + p.nb[1];
    const int k = p.k;
    // this wave's words for tiles [tile0, tile1) are contiguous: the lanes read
    // 64 of them per load and the wave visits only the nonzero ones, in order
    const int64_t nwords = (tile1 - tile0) * kWords;
    const unsigned long long *fw = p.flags + ((int64_t)vg * ntiles + tile0) * kWords;
    for (int64_t base = 0; base < nwords; base += 64 * kLoads) {
        unsigned long long mw[kLoads];
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            const int64_t i = base + 64 * j + lane;
            mw[j] = i < nwords ? fw[i] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < kLoads; ++j) {
            unsigned long long nz = __ballot(mw[j] != 0ull);
            while (nz) {
                const int src = __builtin_ctzll(nz);
                nz &= nz - 1;
                unsigned long long m = __shfl(mw[j], src);
                const int64_t i = base + 64 * j + src;
                const int64_t t = tile0 + i / kWords;
                const int wi = (int)(i % kWords);
                const int g = wi / 8, rt = (wi % 8) / 4, e = wi % 4;
                while (m) {
                    const int l = __builtin_ctzll(m);
                    m &= m - 1;
                    const int ev = 16 * rt + 4 * (l >> 4) + e;
                    const int v = v0 + 16 * g + (l & 15);
                    const int64_t row = t * kTile + ev;
                    const double *V = p.V + (int64_t)v * p.vstride;
                    double ar = 0.0, ai = 0.0, zr = 0.0, zi = 0.0;
                    if (lane < k) {
                        ar = (double)p.A[0][2 * (row * p.ld + lane)];
                        ai = (double)p.A[0][2 * (row * p.ld + lane) + 1];
                        zr = V[2 * lane] * ar - V[2 * lane + 1] * ai;
                        zi = V[2 * lane] * ai + V[2 * lane + 1] * ar;
                    }
#pragma unroll
                    for (int off = 1; off < 64; off <<= 1) {
                        zr += __shfl_xor(zr, off);
                        zi += __shfl_xor(zi, off);
                    }
                    const double I = zr * zr + zi * zi;
                    const double tv = p.vscale[v];
                    double *dst = p.partials + ((int64_t)v * nblk + blockIdx.x) * p.pstride;
                    if (lane == 0) dst[0] += log2(I);
                    if (lane < k) {
                        const double ur = zr / (I * tv), ui = zi / (I * tv);
                        dst[1 + 2 * lane] += ar * ur + ai * ui;        // Re conj(A_a) u
                        dst[2 + 2 * lane] += ar * ui - ai * ur;        // Im conj(A_a) u
                    }
                }
            }
        }
    }
}

// Operand planes of one sample, tile after tile (4 planes x 32 x K2 values of 2
// bytes per tile): FP16 hi / lo of the amplitudes scaled by the power of two
// of their wave (event-major rows), then BF16 hi / lo of the unscaled
// amplitudes transposed (real-column-major, event e at position
// 8 ((e mod 16) / 4) + (e mod 4) + 4 (e / 16)).  Rows past n and columns past
// 2k hold zeros.  One thread per (event, pair of real columns).
__global__ void batch_planes_kernel(const float *A, int64_t n, int64_t ld, int nreal, int K2, int64_t ntiles,
                                    const float *ascale, unsigned short *out) {
    const int64_t total = ntiles * kTile * (K2 / 2);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t eg = idx / (K2 / 2);
        const int r = 2 * (int)(idx % (K2 / 2));
        const int64_t t = eg / kTile;
        const int e = (int)(eg % kTile);
        float x0 = 0.f, x1 = 0.f;
        if (eg < n && r < nreal) {
            x0 = A[2 * eg * ld + r];
            x1 = A[2 * eg * ld + r + 1];
        }
        unsigned short *base = out + t * (128 * (int64_t)K2);
        const float y0 = x0 * ascale[r], y1 = x1 * ascale[r + 1];
        const _Float16 h0 = (_Float16)y0, h1 = (_Float16)y1;
        const _Float16 l0 = (_Float16)(y0 - (float)h0), l1 = (_Float16)(y1 - (float)h1);
        const int pe = 8 * ((e & 15) >> 2) + (e & 3) + 4 * (e >> 4);
        const __bf16 g0 = (__bf16)x0, g1 = (__bf16)x1;
        const __bf16 m0 = (__bf16)(x0 - (float)g0), m1 = (__bf16)(x1 - (float)g1);
        _Float16 *ah = reinterpret_cast<_Float16 *>(base);
        _Float16 *al = ah + kTile * K2;
        __bf16 *bh = reinterpret_cast<__bf16 *>(base + 2 * kTile * K2);
        __bf16 *bl = bh + kTile * K2;
        ah[e * K2 + r] = h0;
        ah[e * K2 + r + 1] = h1;
        al[e * K2 + r] = l0;
        al[e * K2 + r + 1] = l1;
        bh[r * kTile + pe] = g0;
        bh[(r + 1) * kTile + pe] = g1;
        bl[r * kTile + pe] = m0;
        bl[(r + 1) * kTile + pe] = m1;
    }
}

// |A_i|^2 of each row (FP64 sums of the FP32 values, stored as FP32): 8 lanes per
// row, each reading 16-byte chunks (two complex values), summed over the 8 lanes.
// Only the first k complex values count (a borrowed sample's padding is not read
// as data).  Rows are 16-byte aligned (ld even).
__global__ void rownorm_kernel(const float *A, int64_t n, int64_t ld, int k, float *out) {
    typedef float f4r __attribute__((ext_vector_type(4)));
    const int sub = threadIdx.x & 7;
    const int nch = (k + 1) / 2;
    const int64_t groups = (int64_t)gridDim.x * blockDim.x / 8;
    // the 8 lanes of a row share r, so they leave the loop together
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 8; r < n; r += groups) {
        const f4r *x = reinterpret_cast<const f4r *>(A + 2 * r * ld);
        double s = 0.0;
        for (int c = sub; c < nch; c += 8) {
            const f4r v = x[c];
            s += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
            if (2 * c + 1 < k) s += (double)v.z * (double)v.z + (double)v.w * (double)v.w;
        }
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (sub == 0) out[r] = (float)s;
    }
}

// The FP16 hi + lo pair the forward weights carry for a weight x (scaled by
// t / s); the combine evaluates the same expression to know the weights the
// matrix cores used.
struct WeightSplit {
    _Float16 hi, lo;
};
__device__ __forceinline__ WeightSplit split_weight(double x) {
    const _Float16 hi = (_Float16)(float)x;
    return WeightSplit{hi, (_Float16)(float)(x - (double)(float)hi)};
}

// Per vector v (one block each): add the block partials of each segment in
// block order, undo the per-vector scale t_v of the forward weights, and form
// NLL and gradient (Eq. 2 or Eq. 3 form; streamed MC or the MC matrix).
//
// The matrix cores summed with the weights V~ the FP16 hi + lo pairs hold,
// not V; the difference dV = V - V~ (about 2^-22 |V|) is the same for every
// event, so it does not average out over the sums.  Its first-order effect is
// added here from the adjoint sums the pass produced:
//   sum_i ln I_i(V) = sum_i ln I_i(V~) + 2 Re sum_a dV_a conj(G_a),
//   sum_j w_j I_j(V) = sum_j w_j I_j(V~) + 2 Re sum_a dV_a conj(H_a),
// with G_a = sum_i conj(A_ia) z_i / I_i and H_a = sum_j w_j conj(A_ja) z_j
// (the second-order terms are about 2^-44 of the sums).
// The block partials of a segment are summed by G = kCombineThreads / pstride
// thread groups (group g takes blocks g, g + G, ...; threads of a group take
// the pstride values of a block, so each block's partial row is read
// contiguously; eight loads in flight per thread), then the G group sums are
// added in group order: the order is fixed.  One block per vector reads a few
// MB of partials, so the block is large to keep many loads in flight.
constexpr int kCombineThreads = 1024;

__global__ __launch_bounds__(kCombineThreads) void nll_batch_combine_kernel(BatchArgs p) {
    __shared__ double tot[2][1 + 2 * PWA_MAX_K];
    __shared__ double grp[kCombineThreads];
    __shared__ double mv[2 * PWA_MAX_K];
    __shared__ double dv[2 * PWA_MAX_K];
    __shared__ double s_c;
    const int v = blockIdx.x, tid = threadIdx.x;
    const int pst = p.pstride;
    const int nblk = p.nb[0] + p.nb[1];
    const int k = p.k;
    const double *base = p.partials + (int64_t)v * nblk * pst;
    const int G = kCombineThreads / pst, g = tid / pst, cc = tid % pst;
    for (int sg = 0; sg < 2; ++sg) {
        const int b0 = sg ? p.nb[0] : 0, b1 = sg ? nblk : p.nb[0];
        if (g < G) {
            double s = 0.0;
#pragma unroll 8
            for (int b = b0 + g; b < b1; b += G) s += base[(int64_t)b * pst + cc];
            grp[tid] = s;
        }
        __syncthreads();
        if (tid < pst) {
            double s = 0.0;
            for (int h = 0; h < G; ++h) s += grp[h * pst + tid];
            tot[sg][tid] = s;
        }
        __syncthreads();
    }
    const double tv = p.vscale[v];
    const double *V = p.V + (int64_t)v * p.vstride;
    for (int i = tid; i < 2 * k; i += kCombineThreads) {
        const double sr = (double)p.ascale[i];
        const WeightSplit ws = split_weight(V[i] * tv / sr);
        dv[i] = V[i] - ((double)ws.hi + (double)ws.lo) * sr / tv;
    }
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
    }
    __syncthreads();
    double *out = p.out + (int64_t)v * p.ostride;
    if (tid == 0) {
        const double nd = p.nd_total;
        // Z' = t_v z: the data sums hold log2 I (unscaled) and conj(A) u / t_v; sum w I = sum w I' / t_v^2
        // first-order terms of the weight rounding (data: G = t_v x data sums;
        // MC: H = MC sums / t_v); the data's log sum is of the unscaled I
        double dlog = 0.0, ds = 0.0;
        for (int i = 0; i < 2 * k; ++i) {
            dlog += dv[i] * tot[0][1 + i] * tv;
            ds += dv[i] * tot[1][1 + i] / tv;
        }
        const double sum_log = tot[0][0] * 0.69314718055994530942 + 2.0 * dlog;
        double S, c;
        if (p.gram) {
            double s = 0.0;
            for (int a = 0; a < k; ++a) s += V[2 * a] * mv[2 * a] + V[2 * a + 1] * mv[2 * a + 1];
            S = s;
            c = p.extended ? 1.0 : nd / S;
        } else {
            const double s_raw = tot[1][0] / (tv * tv) + 2.0 * ds;
            S = s_raw / p.n_gen;
            c = p.extended ? 1.0 / p.n_gen : nd / s_raw;
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
        out[0] = nll;
        out[1 + 2 * k] = (double)flags;
        s_c = c;
    }
    __syncthreads();
    const double c = s_c;
    const bool zero = !p.extended && p.nd_total == 0.0;
    // data sums carry u = t_v Z'/I' (x t_v); MC sums carry w Z' = t_v w z (/ t_v)
    for (int i = tid; i < 2 * k; i += kCombineThreads) {
        const double g = tot[0][1 + i] * tv;
        const double h = p.gram ? mv[i] : tot[1][1 + i] / tv;
        out[1 + i] = zero ? 0.0 : 2.0 * (-g + c * h);
    }
}

// Largest |re| or |im| of each wave over a sample's rows (FP32), as float bits
// in an atomicMax (non-negative floats order like their bit patterns).
__global__ void amax_kernel(const float *A, int64_t n, int64_t ld, int k, unsigned *out) {
    __shared__ unsigned sm[PWA_MAX_K];
    for (int a = threadIdx.x; a < k; a += blockDim.x) sm[a] = 0u;
    __syncthreads();
    const int64_t total = n * (int64_t)k;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / k;
        const int a = (int)(i % k);
        const float *x = A + 2 * (row * ld + a);
        const float m = fmaxf(fabsf(x[0]), fabsf(x[1]));
        atomicMax(&sm[a], __float_as_uint(m));
    }
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += blockDim.x) atomicMax(&out[a], sm[a]);
}

// Per vector: power of two t_v with max_a |V_a| / s_a * t_v in [2^13, 2^14).
__global__ void batch_vscale_kernel(BatchArgs p) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= p.nv) return;
    const double *V = p.V + (int64_t)v * p.vstride;
    double m = 0.0;
    for (int a = 0; a < p.k; ++a)
        m = fmax(m, fmax(fabs(V[2 * a]), fabs(V[2 * a + 1])) / (double)p.ascale[2 * a]);
    double t = 1.0;
    if (m > 0.0) {
        int e;
        frexp(m, &e);                 // m in [2^(e-1), 2^e)
        t = ldexp(1.0, 14 - e);
    }
    const_cast<double *>(p.vscale)[v] = t;
}

// Forward weights W' = W t_v / s_r split into FP16 hi + lo, in the B-operand
// fragment order [group][hi/lo][ct][ks][lane][8] the batched kernel loads.
template <int KS, int CT>
__global__ void batch_wfrag_kernel(BatchArgs p, int ngroups_pad) {
    const int64_t total = (int64_t)ngroups_pad * CT * KS * 64 * 8;
    _Float16 *wf = reinterpret_cast<_Float16 *>(const_cast<void *>(p.wfrag));
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int e = idx % 8;
        const int lane = (idx / 8) % 64;
        const int kk = (idx / (8 * 64)) % KS;
        const int ct = (idx / (8 * 64 * KS)) % CT;
        const int grp = (int)(idx / (8 * 64 * KS * CT));
        const int r = 32 * kk + 8 * (lane >> 4) + e;
        const int v = grp * 8 * CT + 16 * (ct >> 1) + (lane & 15);
        double x = 0.0;
        if (v < p.nv && r < 2 * p.k) {
            const double *V = p.V + (int64_t)v * p.vstride;
            const int a = r >> 1;
            const double vr = V[2 * a], vi = V[2 * a + 1];
            const double wv = (ct & 1) == 0 ? ((r & 1) == 0 ? vr : -vi) : ((r & 1) == 0 ? vi : vr);
            x = wv * p.vscale[v] / (double)p.ascale[r];
        }
        const WeightSplit ws = split_weight(x);
        const _Float16 hi = ws.hi, lo = ws.lo;
        const size_t base = ((((size_t)grp * 2 + 0) * CT + ct) * KS + kk) * 64 + lane;
        const size_t basel = ((((size_t)grp * 2 + 1) * CT + ct) * KS + kk) * 64 + lane;
        wf[base * 8 + e] = hi;
        wf[basel * 8 + e] = lo;
    }
}

}  // namespace

hipError_t launch_batch_weights(const BatchArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL(batch_vscale_kernel, dim3((args.nv + 255) / 256), dim3(256), 0, stream, args);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int gpad = (batch_vector_groups(args.nv, args.k) + kWaves - 1) / kWaves * kWaves;
    const int64_t total = (int64_t)gpad * batch_ct(args.k) * batch_ks(args.k) * 64 * 8;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    switch (batch_ks(args.k)) {
        case 1: hipLaunchKernelGGL((batch_wfrag_kernel<1, 4>), dim3(blocks), dim3(256), 0, stream, args, gpad); break;
        case 2: hipLaunchKernelGGL((batch_wfrag_kernel<2, 4>), dim3(blocks), dim3(256), 0, stream, args, gpad); break;
        case 3: hipLaunchKernelGGL((batch_wfrag_kernel<3, 2>), dim3(blocks), dim3(256), 0, stream, args, gpad); break;
        case 4: hipLaunchKernelGGL((batch_wfrag_kernel<4, 2>), dim3(blocks), dim3(256), 0, stream, args, gpad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

size_t batch_partial_doubles(int64_t n0, int64_t n1, int tpb, int nv, int k) {
    const int64_t nb = batch_blocks(n0, tpb) + batch_blocks(n1, tpb);
    return (size_t)nb * (size_t)nv * (size_t)(1 + 2 * k);
}

int batch_tiles_per_block(int64_t n0, int64_t n1, int cu) {
    const int64_t tiles = (n0 + kTile - 1) / kTile + (n1 + kTile - 1) / kTile;
    if (tiles == 0 || cu < 1) return kTilesPerBlock;
    const int64_t rounds = (tiles + (int64_t)cu * kTilesPerBlock - 1) / ((int64_t)cu * kTilesPerBlock);
    const int64_t tpb = (tiles + rounds * cu - 1) / (rounds * cu);
    return (int)(tpb < 1 ? 1 : tpb);
}

int64_t batch_blocks(int64_t n, int tpb) {
    const int64_t tiles = (n + kTile - 1) / kTile;
    return (tiles + tpb - 1) / tpb;
}

int batch_ks(int k) { return (2 * k + 31) / 32; }

int batch_ct(int k) { return batch_ks(k) <= 2 ? 4 : 2; }

int batch_vectors_per_wave(int k) { return 8 * batch_ct(k); }

int batch_vector_groups(int nv, int k) {
    const int vpw = batch_vectors_per_wave(k);
    return (nv + vpw - 1) / vpw;
}

hipError_t launch_amax(const float *A, int64_t n, int64_t ld, int k, unsigned *out,
                       hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int64_t blocks64 = (n * k + 255) / 256;
    const int blocks = (int)(blocks64 < 4096 ? blocks64 : 4096);
    hipLaunchKernelGGL(amax_kernel, dim3(blocks), dim3(256), 0, stream, A, n, ld, k, out);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs &args, bool refine, hipStream_t stream) {
    const int nblk = args.nb[0] + args.nb[1];
    if (nblk > 0) {
        const int gy = (batch_vector_groups(args.nv, args.k) + kWaves - 1) / kWaves;
        const dim3 grid(nblk, gy);
#define PWA_BATCH_LAUNCH(KS_, CT_)                                                                   \
    do {                                                                                             \
        if (refine)                                                                                  \
            hipLaunchKernelGGL((nll_batch_kernel<KS_, CT_, true>), grid, dim3(kThreads), 0, stream, args);  \
        else                                                                                         \
            hipLaunchKernelGGL((nll_batch_kernel<KS_, CT_, false>), grid, dim3(kThreads), 0, stream, args); \
    } while (0)
        switch (batch_ks(args.k)) {
            case 1: PWA_BATCH_LAUNCH(1, 4); break;
            case 2: PWA_BATCH_LAUNCH(2, 4); break;
            case 3: PWA_BATCH_LAUNCH(3, 2); break;
            case 4: PWA_BATCH_LAUNCH(4, 2); break;
            default: return hipErrorInvalidValue;
        }
#undef PWA_BATCH_LAUNCH
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_batch_refine(const BatchArgs &args, hipStream_t stream) {
    if (args.nb[0] == 0) return hipSuccess;
    const int gy = (batch_vector_groups(args.nv, args.k) + kWaves - 1) / kWaves;
    const dim3 grid(args.nb[0], gy);
    if (batch_ct(args.k) == 4)
        hipLaunchKernelGGL((batch_refine_kernel<4>), grid, dim3(kThreads), 0, stream, args);
    else
        hipLaunchKernelGGL((batch_refine_kernel<2>), grid, dim3(kThreads), 0, stream, args);
    return hipGetLastError();
}

size_t batch_flag_words(int64_t n0, int nv, int k) {
    const int64_t tiles = (n0 + kTile - 1) / kTile;
    const int gpad = (batch_vector_groups(nv, k) + kWaves - 1) / kWaves * kWaves;
    return (size_t)tiles * gpad * 8 * (batch_ct(k) / 2);
}

size_t batch_plane_bytes(int64_t n, int k) {
    const int64_t ntiles = (n + kTile - 1) / kTile;
    return (size_t)ntiles * 256 * (size_t)(32 * batch_ks(k));
}

hipError_t launch_batch_planes(const float *A, int64_t n, int64_t ld, int k, const float *ascale, void *out,
                               hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int K2 = 32 * batch_ks(k);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t total = ntiles * kTile * (K2 / 2);
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(batch_planes_kernel, dim3(blocks), dim3(256), 0, stream, A, n, ld, 2 * k, K2, ntiles, ascale,
                       static_cast<unsigned short *>(out));
    return hipGetLastError();
}

hipError_t launch_rownorm(const float *A, int64_t n, int64_t ld, int k, float *out, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>((8 * n + 255) / 256, 16384);
    hipLaunchKernelGGL(rownorm_kernel, dim3(blocks), dim3(256), 0, stream, A, n, ld, k, out);
    return hipGetLastError();
}

hipError_t launch_batch_combine(const BatchArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL(nll_batch_combine_kernel, dim3(args.nv), dim3(kCombineThreads), 0, stream, args);
    return hipGetLastError();
}

}  // namespace pwa
