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
// One pass over the data rows on the FP64 matrix cores (hess_mfma_kernel);
// the block partials are added in block order, then one block assembles H.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kHThreads = 256;
__global__ void hess_clear_kernel(unsigned *flag) { *flag = 0u; }

// Matrix-core pass.  With u_i = 1 / z_i and B_i = A_i u_i (complex, K values),
// T = sum_i B_i B_i^T (no conjugate).  In real terms, with the row
// X_i = (Re B_i padded to KP, Im B_i padded to KP) of 2 KP reals,
//     G = sum_i X_i X_i^T = [[Grr, Gri], [Gri^T, Gii]],
//     Re T = Grr - Gii,   Im T = Gri + Gri^T,
// so the pass is a symmetric rank-N update of a 2KP x 2KP FP64 matrix, run as
// v_mfma_f64_16x16x4f64 on 16 x 16 tiles of its upper triangle.  Per step a
// block forms X for 64 events in LDS (4 threads per event: z from a quarter
// of the waves each and a DPP sum, then u and B); the waves then multiply:
// with few tiles each wave takes every tile for 16 of the 64 events, with
// many each wave takes every fourth tile for all 64.  The waves' sums are
// added in wave order and the block writes its full G (lower tiles mirrored).
template <typename T, int KP>
__global__ __launch_bounds__(kHThreads) void hess_mfma_kernel(const T *__restrict__ A, int64_t n, int64_t ld, int k,
                                                              const double *__restrict__ V,
                                                              double *__restrict__ partials,
                                                              unsigned *__restrict__ flag) {
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int NC = 2 * KP;                  // columns of X
    constexpr int NT = NC / 16;                 // tile rows
    constexpr int NTU = NT * (NT + 1) / 2;      // upper-triangle tiles
    constexpr bool SPLIT_EVENTS = NTU <= 10;
    constexpr int MAXT = SPLIT_EVENTS ? NTU : (NTU + 3) / 4;
    constexpr int EV = 64;                      // events per step
    constexpr int XS = NC + 2;                  // LDS row stride (doubles)
    constexpr int WPT = KP / 4;                 // waves per thread when forming z and B
    __shared__ __attribute__((aligned(16))) double X[EV][XS];
    __shared__ double Gs[SPLIT_EVENTS ? NC : 1][SPLIT_EVENTS ? NC + 1 : 1];   // the waves' sums (split events)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;

    // this wave's tiles (p <= q) in upper-triangle order
    int tp[MAXT], tq[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
        const int t = SPLIT_EVENTS ? i : wave + 4 * i;
        tp[i] = tq[i] = -1;
        if (t < NTU) {
            int a = 0, row = NT, r = t;
            while (r >= row) {
                r -= row;
                ++a;
                --row;
            }
            tp[i] = a;
            tq[i] = a + r;
        }
    }
    d4 acc[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};

    // this thread's V slice
    const int el = tid >> 2, sub = tid & 3;
    double vr[WPT], vi[WPT];
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
        const int a = sub * WPT + w;
        vr[w] = a < k ? V[2 * a] : 0.0;
        vi[w] = a < k ? V[2 * a + 1] : 0.0;
    }
    bool bad = false;
    for (int64_t base = r0; base < r1; base += EV) {
        const int64_t e = base + el;
        const bool valid = e < r1;
        double ar[WPT], ai[WPT];
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int w = 0; w < WPT; ++w) {
            const int a = sub * WPT + w;
            ar[w] = (valid && a < k) ? (double)A[2 * (e * ld + a)] : 0.0;
            ai[w] = (valid && a < k) ? (double)A[2 * (e * ld + a) + 1] : 0.0;
            zr = fma(vr[w], ar[w], fma(-vi[w], ai[w], zr));
            zi = fma(vr[w], ai[w], fma(vi[w], ar[w], zi));
        }
        zr += __shfl_xor(zr, 1);
        zi += __shfl_xor(zi, 1);
        zr += __shfl_xor(zr, 2);
        zi += __shfl_xor(zi, 2);
        const double I = zr * zr + zi * zi;
        double ur = 0.0, ui = 0.0;
        if (valid) {
            if (I > 0.0 && isfinite(I)) {
                ur = zr / I;                         // 1 / z = conj(z) / I
                ui = -zi / I;
            } else {
                bad = true;
            }
        }
        __syncthreads();                             // the previous step's X is consumed
#pragma unroll
        for (int w = 0; w < WPT; ++w) {
            const int a = sub * WPT + w;
            X[el][a] = fma(ar[w], ur, -ai[w] * ui);          // Re (A u)
            X[el][KP + a] = fma(ar[w], ui, ai[w] * ur);      // Im (A u)
        }
        __syncthreads();
        // rows of the k-step: 4 events, lane l takes event l / 16 and column l % 16
        const int er = lane >> 4, ec = lane & 15;
        if (SPLIT_EVENTS) {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const double *row = X[16 * wave + 4 * ks + er];
#pragma unroll
                for (int i = 0; i < MAXT; ++i)
                    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * tp[i] + ec], row[16 * tq[i] + ec], acc[i],
                                                                  0, 0, 0);
            }
        } else {
#pragma unroll 4
            for (int ks = 0; ks < EV / 4; ++ks) {
                const double *row = X[4 * ks + er];
#pragma unroll
                for (int i = 0; i < MAXT; ++i)
                    if (tp[i] >= 0)
                        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * tp[i] + ec], row[16 * tq[i] + ec],
                                                                      acc[i], 0, 0, 0);
            }
        }
    }
    if (bad) atomicOr(flag, 1u);
    // FP64 MFMA result layout: item j of lane l is row l / 16 + 4 j, column l % 16 of a tile
    const int rb = lane >> 4, cb = lane & 15;
    double *out = partials + (int64_t)blockIdx.x * NC * NC;
    if (SPLIT_EVENTS) {
        // every wave holds every tile for its quarter of the events: their sums in wave order
        for (int idx = tid; idx < NC * NC; idx += kHThreads) Gs[idx / NC][idx % NC] = 0.0;
        for (int w = 0; w < 4; ++w) {
            __syncthreads();
            if (wave == w) {
#pragma unroll
                for (int i = 0; i < MAXT; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) Gs[16 * tp[i] + rb + 4 * j][16 * tq[i] + cb] += acc[i][j];
            }
        }
        __syncthreads();
        // block partial: the full G (lower tiles as the transposes of the upper ones)
        for (int idx = tid; idx < NC * NC; idx += kHThreads) {
            const int r = idx / NC, c = idx % NC;
            out[idx] = (r >> 4) <= (c >> 4) ? Gs[r][c] : Gs[c][r];
        }
    } else {
        // each tile belongs to one wave: written with its transpose
#pragma unroll
        for (int i = 0; i < MAXT; ++i) {
            if (tp[i] < 0) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 16 * tp[i] + rb + 4 * j, c = 16 * tq[i] + cb;
                out[(int64_t)r * NC + c] = acc[i][j];
                if (tp[i] != tq[i]) out[(int64_t)c * NC + r] = acc[i][j];
            }
        }
    }
}

// G = sum of the block partials: one block per entry, fixed-order tree.
constexpr int kFinThreads = 64;
__global__ __launch_bounds__(kFinThreads) void hess_finish_kernel(const double *__restrict__ partials, int nblocks,
                                                                  int entries, double *__restrict__ Tm) {
    const int e = blockIdx.x;
    double s = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblocks; b += kFinThreads) s += partials[(int64_t)b * entries + e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) Tm[e] = s;
}

// One block: H (2k x 2k, row-major) from G (2 kp x 2 kp, see hess_mfma_kernel),
// M and V; H[2k * 2k] = status flags.
__global__ void hess_assemble_kernel(const double *__restrict__ Gm, int kp, const double *__restrict__ M,
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
        // Re T = Grr - Gii, Im T = Gri + Gri^T
        const int nc = 2 * kp;
        const double tr = Gm[a * nc + c] - Gm[(kp + a) * nc + kp + c];
        const double ti = Gm[a * nc + kp + c] + Gm[(kp + a) * nc + c];
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

int hessian_kp(int k) { return 8 * ((k + 7) / 8); }
size_t hessian_g_doubles(int k) { return (size_t)(2 * hessian_kp(k)) * (size_t)(2 * hessian_kp(k)); }
size_t hessian_partial_doubles(int k, int blocks) { return (size_t)blocks * hessian_g_doubles(k); }

template <typename T>
hipError_t launch_hess_mfma(const T *A, int64_t n, int64_t ld, int k, const double *V, double *partials,
                            unsigned *flag, int blocks, hipStream_t s) {
    switch (hessian_kp(k)) {
#define PWA_HESS_CASE(KP_)                                                                                   \
    case KP_:                                                                                                \
        hipLaunchKernelGGL((hess_mfma_kernel<T, KP_>), dim3(blocks), dim3(kHThreads), 0, s, A, n, ld, k, V, \
                           partials, flag);                                                                  \
        break;
        PWA_HESS_CASE(8) PWA_HESS_CASE(16) PWA_HESS_CASE(24) PWA_HESS_CASE(32)
        PWA_HESS_CASE(40) PWA_HESS_CASE(48) PWA_HESS_CASE(56) PWA_HESS_CASE(64)
#undef PWA_HESS_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_hessian(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, const double *V_dev,
                          const double *M, double nd, int extended, double *partials, int blocks, double *Gm,
                          unsigned *flag, double *H, hipStream_t stream) {
    if (k < 1 || k > PWA_MAX_K || blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hess_clear_kernel, dim3(1), dim3(1), 0, stream, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > 0) {
        e = prec == PWA_F32
                ? launch_hess_mfma(static_cast<const float *>(A), n, ld, k, V_dev, partials, flag, blocks, stream)
                : launch_hess_mfma(static_cast<const double *>(A), n, ld, k, V_dev, partials, flag, blocks, stream);
        if (e != hipSuccess) return e;
    } else {
        blocks = 0;
    }
    const int entries = (int)hessian_g_doubles(k);
    hipLaunchKernelGGL(hess_finish_kernel, dim3(entries), dim3(kFinThreads), 0, stream, partials, blocks, entries, Gm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(hess_assemble_kernel, dim3(1), dim3(256), 0, stream, Gm, hessian_kp(k), M, V_dev, k, nd,
                       extended, flag, H);
    return hipGetLastError();
}

}  // namespace pwa
