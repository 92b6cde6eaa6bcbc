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
// Launches: the data pass on the FP64 matrix cores (hess_mfma_kernel, one
// launch per group of at most 21 output tiles), the fixed-order sum of its
// block partials (hess_sum_kernel) and the assembly of H.
#include <atomic>
#include <utility>

#include "internal.hpp"

namespace pwa {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kHThreads = 256;
constexpr int kHWaves = kHThreads / 64;
constexpr int kHRows = 16;        // events per wave per step (four k-steps of the 16x16x4 MFMA)
constexpr int kHMaxTiles = 21;    // accumulator tiles per wave in one launch

// Output tiles: the upper triangle of the NT x NT grid of 16 x 16 tiles of G,
// numbered row by row.
constexpr int tile_p(int t, int nt) {
    int p = 0;
    while (t >= nt - p) {
        t -= nt - p;
        ++p;
    }
    return p;
}
constexpr int tile_q(int t, int nt) {
    int p = 0;
    while (t >= nt - p) {
        t -= nt - p;
        ++p;
    }
    return p + t;
}
constexpr int tile_count(int nt) { return nt * (nt + 1) / 2; }
constexpr int tile_groups(int nt) { return (tile_count(nt) + kHMaxTiles - 1) / kHMaxTiles; }
// Wave slab layout: logical column c of event row r sits at r * XS + sh(r) + c
// with sh(r) = 8 ((r >> 1) & 1) + 4 ((r >> 2) & 1) and XS = 16 mod 32
// doubles.  The row writes (lanes: 8 rows x 4 consecutive columns per
// half-wave) and the MFMA operand reads (lanes: 2 rows x 16 consecutive
// columns per half-wave) then touch distinct banks, and both take one base
// address per lane plus immediate offsets.
constexpr int slab_stride(int nc) {
    int x = nc + 12;
    while (x % 32 != 16) ++x;
    return x;
}
__device__ __forceinline__ int slab_shift(int r) { return 8 * ((r >> 1) & 1) + 4 * ((r >> 2) & 1); }

// Lane exchange inside groups of four lanes (DPP quad permutation): 0xB1
// swaps neighbours (lane ^ 1), 0x4E swaps pairs (lane ^ 2).
template <int CTRL>
__device__ __forceinline__ double quad_swap(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// V by value in the kernel arguments (no upload before the launches).
struct HessV {
    double v[2 * PWA_MAX_K];
};

template <typename T> struct Pair;
template <> struct Pair<float> { typedef float v __attribute__((ext_vector_type(2))); };
template <> struct Pair<double> { typedef double v __attribute__((ext_vector_type(2))); };

// acc[I] += X^T X on tile T0 + I for the four events of one k-step; colv[c]
// holds column block c of this lane's event row.
template <int NT, int T0, int... I>
__device__ __forceinline__ void mfma_tiles(d4 *acc, const double *colv, std::integer_sequence<int, I...>) {
    ((acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(colv[std::integral_constant<int, tile_p(T0 + I, NT)>::value],
                                                    colv[std::integral_constant<int, tile_q(T0 + I, NT)>::value],
                                                    acc[I], 0, 0, 0)),
     ...);
}

// Data pass on the FP64 matrix cores.  With u_i = 1 / z_i and B_i = A_i u_i
// (complex, K values), T = sum_i B_i B_i^T (no conjugate).  In real terms,
// with the row X_i = (Re B_i padded to KP, Im B_i padded to KP) of NC = 2 KP
// reals,
//     G = sum_i X_i X_i^T = [[Grr, Gri], [Gri^T, Gii]],
//     Re T = Grr - Gii,   Im T = Gri + Gri^T,
// a symmetric rank-N update of an NC x NC FP64 matrix, run as
// v_mfma_f64_16x16x4f64 on the 16 x 16 tiles T0 .. T0 + NTL - 1 of its upper
// triangle.  Every wave works alone on 16 events per step: four lanes per
// event form z (each a quarter of the waves, then two lane swaps), u and the
// row X in the wave's own LDS slab, then the wave multiplies its slab into
// all of its tiles while the next step's amplitude rows are in flight (no
// block barrier inside the loop).  At the end the four waves' tiles are added
// in wave order and the block writes them to its partial (tile-major, NTU
// tiles of 256 doubles).  Per event the pass computes 4 K (K + 1) flops of the
// symmetric contraction plus about 14 K for z, u and B.
template <typename T, int KP, int T0, int NTL>
__global__ __launch_bounds__(kHThreads) void hess_mfma_kernel(const T *__restrict__ A, int64_t n, int64_t ld, int k,
                                                              const HessV V, int ntu,
                                                              double *__restrict__ partials,
                                                              unsigned *__restrict__ flag) {
    constexpr int NC = 2 * KP;
    constexpr int NT = NC / 16;
    constexpr int XS = slab_stride(NC);
    constexpr int WPT = KP / 4;                         // waves per lane when forming z and B
    constexpr int STEP = kHWaves * kHRows;              // events per block step
    constexpr bool V_LDS = WPT > 4;                     // V from LDS (fewer live registers) at large K
    constexpr int SLAB = kHRows * XS;                   // doubles of one wave's slab
    static_assert(NTL * 256 <= kHWaves * SLAB, "the tile sums must fit in the slabs");
    typedef typename Pair<T>::v TP;
    __shared__ __attribute__((aligned(16))) double lds[kHWaves * SLAB];
    __shared__ __attribute__((aligned(16))) double vs[V_LDS ? 2 * KP : 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double *X = lds + wave * SLAB;                      // this wave's slab
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
    // forming: event row of the slab and the waves a = 4 w + sub
    const int row = lane >> 2, sub = lane & 3;
    const int wofs = row * XS + slab_shift(row) + sub;
    // multiplying: lane (er, ec) feeds event row 4 ks + er, column ec of a tile;
    // slab_shift(4 ks + er) = 8 (er >> 1) + 4 (ks & 1)
    const int er = lane >> 4, ec = lane & 15;
    const int mofs = er * XS + 8 * (er >> 1) + ec;

    double vr[V_LDS ? 1 : WPT], vi[V_LDS ? 1 : WPT];
    if constexpr (V_LDS) {
        for (int i = tid; i < 2 * KP; i += kHThreads) vs[i] = i < 2 * k ? V.v[i] : 0.0;
        __syncthreads();
    } else {
#pragma unroll
        for (int w = 0; w < WPT; ++w) {
            const int a = 4 * w + sub;
            vr[w] = a < k ? V.v[2 * a] : 0.0;
            vi[w] = a < k ? V.v[2 * a + 1] : 0.0;
        }
    }
    d4 acc[NTL];
#pragma unroll
    for (int i = 0; i < NTL; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};

    // amplitudes of event e (row index clamped into the sample).  With rows of
    // at least KP elements every load stays inside its row and takes the row as
    // it is: a row outside the block's range gets u = 0 when it is formed (the
    // block whose row it is forms and checks it), and the columns past k meet
    // V = 0 in z and reach only entries of G past k, which are not read.  With
    // narrower rows the element index is clamped and the values past k or
    // outside the range are zeroed.  Either way the loads need no branch.
    const bool wide = ld >= KP;
    auto fetch = [&](TP (&dst)[WPT], int64_t e) {
        const bool ok_e = e < r1;
        const T *rp = A + 2 * ((e < n ? e : n - 1) * ld);
        if (wide) {
            const TP *q = reinterpret_cast<const TP *>(rp) + sub;
#pragma unroll
            for (int w = 0; w < WPT; ++w) dst[w] = q[4 * w];
        } else {
#pragma unroll
            for (int w = 0; w < WPT; ++w) {
                const int a = 4 * w + sub;
                const TP v = reinterpret_cast<const TP *>(rp)[a < k ? a : k - 1];
                dst[w] = (ok_e && a < k) ? v : TP{};
            }
        }
    };
    bool bad = false;
    // Forming the slab rows of one step: (0) z partial sums, (1) z over the
    // four lanes and u, (2, 3) the two halves of the row writes.
    double zr, zi, ur, ui;
    auto form = [&](int part, const TP (&src)[WPT], double *Xs, bool valid) {
        if (part == 0) {
            zr = 0.0;
            zi = 0.0;
#pragma unroll
            for (int w = 0; w < WPT; ++w) {
                const double ar = (double)src[w].x, ai = (double)src[w].y;
                double wr, wi;
                if constexpr (V_LDS) {
                    const int a = 4 * w + sub;
                    wr = vs[2 * a];
                    wi = vs[2 * a + 1];
                } else {
                    wr = vr[w];
                    wi = vi[w];
                }
                zr = fma(wr, ar, fma(-wi, ai, zr));
                zi = fma(wr, ai, fma(wi, ar, zi));
            }
        } else if (part == 1) {
            zr += quad_swap<0xB1>(zr);
            zi += quad_swap<0xB1>(zi);
            zr += quad_swap<0x4E>(zr);
            zi += quad_swap<0x4E>(zi);
            const double I = zr * zr + zi * zi;
            ur = 0.0;
            ui = 0.0;
            if (valid) {
                if (I > 0.0 && isfinite(I)) {
                    // 1 / z = conj(z) / I; 1 / I from the hardware reciprocal and
                    // two Newton steps (a few ulp at most)
                    double rI = __builtin_amdgcn_rcp(I);
                    rI = fma(rI, fma(-I, rI, 1.0), rI);
                    rI = fma(rI, fma(-I, rI, 1.0), rI);
                    ur = zr * rI;
                    ui = -zi * rI;
                } else {
                    bad = true;
                }
            }
        } else {
            double *xw = Xs + wofs;
            constexpr int H = (WPT + 1) / 2;
#pragma unroll
            for (int w = part == 2 ? 0 : H; w < (part == 2 ? H : WPT); ++w) {
                TP s = src[w];
                // at large K the amplitudes are converted again here rather than
                // kept in FP64 from the z sums (twice the registers over the
                // forming phase); the empty statement hides that the value is the same
                if constexpr (V_LDS) __asm__ volatile("" : "+v"(s));
                const double ar = (double)s.x, ai = (double)s.y;
                xw[4 * w] = fma(ar, ur, -ai * ui);              // Re (A u), column 4 w + sub
                xw[KP + 4 * w] = fma(ar, ui, ai * ur);          // Im (A u)
            }
        }
    };
    auto slab_fence = [] {
        // LDS operations of one wave complete in order; the fences keep the compiler
        // from moving slab reads and writes across this point
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // one step: form the step's rows from buf, refill buf with the next step's
    // rows (in flight during the MFMAs), then the step's MFMAs
    auto step = [&](TP (&buf)[WPT], int64_t b) {
        const bool valid = b + row < r1;
        form(0, buf, X, valid);
        form(1, buf, X, valid);
        slab_fence();                                   // the previous step's reads come first
        form(2, buf, X, valid);
        form(3, buf, X, valid);
        fetch(buf, b + STEP + row);
        __builtin_amdgcn_sched_barrier(0);              // the loads stay ahead of the MFMAs
        slab_fence();
        const double *xm = X + mofs;
        if constexpr (NT <= 2) {
            // few column blocks: every k-step's operands are read before the first MFMA
            double colv[kHRows / 4][NT];
#pragma unroll
            for (int ks = 0; ks < kHRows / 4; ++ks)
#pragma unroll
                for (int c = 0; c < NT; ++c) colv[ks][c] = xm[4 * ks * XS + 4 * (ks & 1) + 16 * c];
            __builtin_amdgcn_sched_barrier(0);          // the reads stay ahead of the MFMAs
#pragma unroll
            for (int ks = 0; ks < kHRows / 4; ++ks)
                mfma_tiles<NT, T0>(acc, colv[ks], std::make_integer_sequence<int, NTL>{});
        } else {
#pragma unroll
            for (int ks = 0; ks < kHRows / 4; ++ks) {
                double colv[NT];
#pragma unroll
                for (int c = 0; c < NT; ++c) colv[c] = xm[4 * ks * XS + 4 * (ks & 1) + 16 * c];
                mfma_tiles<NT, T0>(acc, colv, std::make_integer_sequence<int, NTL>{});
            }
        }
    };
    // one register buffer of rows, refilled once the step has read it (at large
    // K, with the amplitudes converted twice, 21 tiles fit two waves per SIMD)
    int64_t base = r0 + kHRows * wave;
    TP buf[WPT];
    fetch(buf, base + row);
    for (; base < r1; base += STEP) step(buf, base);
    if (bad) atomicOr(flag, 1u);
    // tile sums in wave order; item j of lane l is row l / 16 + 4 j, column l % 16
    double *Gs = lds;
#pragma unroll
    for (int w = 0; w < kHWaves; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < NTL; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    double &g = Gs[i * 256 + (er + 4 * j) * 16 + ec];
                    g = w == 0 ? acc[i][j] : g + acc[i][j];
                }
        }
    }
    __syncthreads();
    double *out = partials + (int64_t)blockIdx.x * ntu * 256 + T0 * 256;
    for (int idx = tid; idx < NTL * 256; idx += kHThreads) out[idx] = Gs[idx];
}

// Sum of the block partials into G in one fixed order: a block of 256 threads
// takes 16 entries; thread r of an entry (r = 0 .. 15) adds the partials of
// blocks r, r + 16, ... in block order (32 loads in flight), then the 16 sums
// of the entry are added in r order.
constexpr int kHSumSlices = 16;
__global__ __launch_bounds__(256) void hess_sum_kernel(const double *__restrict__ partials, int nblocks, int entries,
                                                       double *__restrict__ Gm) {
    __shared__ double part[kHSumSlices][16];
    const int tid = threadIdx.x, el = tid & 15, r = tid >> 4;
    const int e = blockIdx.x * 16 + el;
    double s = 0.0;
    if (e < entries) {
        for (int b0 = r; b0 < nblocks; b0 += 32 * kHSumSlices) {
            double v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                const int b = b0 + u * kHSumSlices;
                v[u] = b < nblocks ? partials[(int64_t)b * entries + e] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 32; ++u) s += v[u];
        }
    }
    part[r][el] = s;
    __syncthreads();
    if (r == 0 && e < entries) {
        double t = 0.0;
        for (int q = 0; q < kHSumSlices; ++q) t += part[q][el];
        Gm[e] = t;
    }
}

// G[r][c] from the tile-major upper triangle (NT column blocks).
__device__ __forceinline__ double g_at(const double *Gm, int nt, int r, int c) {
    if ((r >> 4) > (c >> 4)) {
        const int t = r;
        r = c;
        c = t;
    }
    const int p = r >> 4, q = c >> 4;
    const int tile = p * nt - p * (p - 1) / 2 + (q - p);
    return Gm[tile * 256 + (r & 15) * 16 + (c & 15)];
}

// H (2k x 2k, row-major) from G, M and V; H[2k * 2k] = status flags.  Every
// block forms M V (four threads per wave index, lane-order sums) and S; block
// 0 reads the status word of the data pass and clears it for the next call.
__global__ __launch_bounds__(256) void hess_assemble_kernel(const double *__restrict__ Gm, int kp,
                                                            const double *__restrict__ M,
                                                            const HessV V, int k, double nd,
                                                            int extended, unsigned *__restrict__ flag,
                                                            double *__restrict__ H) {
    __shared__ double mv[2 * PWA_MAX_K];
    __shared__ double s_S;
    const int tid = threadIdx.x, n2 = 2 * k;
    {
        const int a = tid >> 2, q = tid & 3;
        double re = 0.0, im = 0.0;
        if (M && a < k)
            for (int c = q; c < k; c += 4) {
                const double mr = M[2 * (a * k + c)], mi = M[2 * (a * k + c) + 1];
                re = fma(mr, V.v[2 * c], fma(-mi, V.v[2 * c + 1], re));
                im = fma(mr, V.v[2 * c + 1], fma(mi, V.v[2 * c], im));
            }
        re += quad_swap<0xB1>(re);
        im += quad_swap<0xB1>(im);
        re += quad_swap<0x4E>(re);
        im += quad_swap<0x4E>(im);
        if (q == 0 && a < k) {
            mv[2 * a] = re;
            mv[2 * a + 1] = im;
        }
    }
    __syncthreads();
    if (tid < 64) {                                     // S = Re sum_a conj(V_a) (M V)_a
        double sv = tid < k ? fma(V.v[2 * tid], mv[2 * tid], V.v[2 * tid + 1] * mv[2 * tid + 1]) : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) sv += __shfl_xor(sv, off);
        if (tid == 0) s_S = sv;
    }
    __syncthreads();
    const double S = s_S;
    const int nt = kp / 8;
    const int idx = blockIdx.x * 256 + tid;
    if (idx < n2 * n2) {
        const int m = idx / n2, nn = idx % n2;
        const int a = m >> 1, c = nn >> 1, pa = m & 1, pc = nn & 1;
        // Re T = Grr - Gii, Im T = Gri + Gri^T
        const double tr = g_at(Gm, nt, a, c) - g_at(Gm, nt, kp + a, kp + c);
        const double ti = g_at(Gm, nt, a, kp + c) + g_at(Gm, nt, kp + a, c);
        const double mr = M ? M[2 * (a * k + c)] : 0.0, mi = M ? M[2 * (a * k + c) + 1] : 0.0;
        // block entries of d2(sum ln I) and d2S for (x or y of a, x or y of c)
        double hl, d2s;
        if (!pa && !pc) {
            hl = -2.0 * tr;
            d2s = 2.0 * mr;
        } else if (!pa && pc) {
            hl = 2.0 * ti;
            d2s = -2.0 * mi;
        } else if (pa && !pc) {
            hl = 2.0 * ti;
            d2s = 2.0 * mi;
        } else {
            hl = 2.0 * tr;
            d2s = 2.0 * mr;
        }
        double h;
        if (extended) {
            h = -hl + d2s;
        } else if (nd == 0.0) {
            h = 0.0;
        } else {
            const double dsm = 2.0 * mv[m], dsn = 2.0 * mv[nn];     // dS: (2 Re MV, 2 Im MV) interleaved
            h = -hl + nd * (d2s / S - dsm * dsn / (S * S));
        }
        H[idx] = h;
    }
    if (blockIdx.x == 0 && tid == 0) {
        const bool dom = (*flag != 0u) || (!extended && nd > 0.0 && !(S > 0.0));
        H[n2 * n2] = dom ? 1.0 : 0.0;
        *flag = 0u;
    }
}

template <typename T, int KP, int G>
hipError_t launch_group(const T *A, int64_t n, int64_t ld, int k, const HessV &V, double *partials,
                        unsigned *flag, int blocks, hipStream_t s) {
    constexpr int NT = KP / 8, NTU = tile_count(NT), NG = tile_groups(NT), NTLM = (NTU + NG - 1) / NG;
    constexpr int T0 = G * NTLM, NTL = NTU - T0 < NTLM ? NTU - T0 : NTLM;
    hipLaunchKernelGGL((hess_mfma_kernel<T, KP, T0, NTL>), dim3(blocks), dim3(kHThreads), 0, s, A, n, ld, k, V, NTU,
                       partials, flag);
    return hipGetLastError();
}

template <typename T, int KP, int... G>
hipError_t launch_groups(const T *A, int64_t n, int64_t ld, int k, const HessV &V, double *partials,
                         unsigned *flag, int blocks, hipStream_t s, std::integer_sequence<int, G...>) {
    hipError_t e = hipSuccess;
    ((e = e == hipSuccess ? launch_group<T, KP, G>(A, n, ld, k, V, partials, flag, blocks, s) : e), ...);
    return e;
}

template <typename T, int KP>
hipError_t launch_pass(const T *A, int64_t n, int64_t ld, int k, const HessV &V, double *partials, unsigned *flag,
                       int blocks, hipStream_t s) {
    return launch_groups<T, KP>(A, n, ld, k, V, partials, flag, blocks, s,
                                std::make_integer_sequence<int, tile_groups(KP / 8)>{});
}

// Resident blocks per CU of the first tile group's kernel.
template <typename T, int KP>
int pass_occupancy() {
    constexpr int NT = KP / 8, NTU = tile_count(NT), NG = tile_groups(NT), NTLM = (NTU + NG - 1) / NG;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, hess_mfma_kernel<T, KP, 0, NTLM>, kHThreads, 0) !=
        hipSuccess)
        nb = 1;
    return nb > 0 ? nb : 1;
}

template <typename T>
int occupancy(int kp) {
    switch (kp) {
        case 8: return pass_occupancy<T, 8>();
        case 16: return pass_occupancy<T, 16>();
        case 24: return pass_occupancy<T, 24>();
        case 32: return pass_occupancy<T, 32>();
        case 40: return pass_occupancy<T, 40>();
        case 48: return pass_occupancy<T, 48>();
        case 56: return pass_occupancy<T, 56>();
        default: return pass_occupancy<T, 64>();
    }
}

template <typename T>
hipError_t launch_data_pass(const T *A, int64_t n, int64_t ld, int k, const HessV &V, double *partials,
                            unsigned *flag, int blocks, hipStream_t s) {
    switch (8 * ((k + 7) / 8)) {
        case 8: return launch_pass<T, 8>(A, n, ld, k, V, partials, flag, blocks, s);
        case 16: return launch_pass<T, 16>(A, n, ld, k, V, partials, flag, blocks, s);
        case 24: return launch_pass<T, 24>(A, n, ld, k, V, partials, flag, blocks, s);
        case 32: return launch_pass<T, 32>(A, n, ld, k, V, partials, flag, blocks, s);
        case 40: return launch_pass<T, 40>(A, n, ld, k, V, partials, flag, blocks, s);
        case 48: return launch_pass<T, 48>(A, n, ld, k, V, partials, flag, blocks, s);
        case 56: return launch_pass<T, 56>(A, n, ld, k, V, partials, flag, blocks, s);
        case 64: return launch_pass<T, 64>(A, n, ld, k, V, partials, flag, blocks, s);
        default: return hipErrorInvalidValue;
    }
}

int hess_kp(int k) { return 8 * ((k + 7) / 8); }
size_t hess_entries(int k) { return (size_t)tile_count(hess_kp(k) / 8) * 256; }

}  // namespace

int hessian_blocks(pwa_prec prec, int k, int cu_count, int64_t n) {
    if (k < 1 || k > PWA_MAX_K) return 1;
    const int kp = hess_kp(k);
    static std::atomic<int> cache[2][PWA_MAX_K / 8 + 1];   // resident blocks per CU, 0 = not asked yet
    std::atomic<int> &slot = cache[prec == PWA_F32 ? 0 : 1][kp / 8];
    int occ = slot.load(std::memory_order_relaxed);
    if (occ == 0) {
        occ = prec == PWA_F32 ? occupancy<float>(kp) : occupancy<double>(kp);
        slot.store(occ, std::memory_order_relaxed);
    }
    const int64_t want = (int64_t)cu_count * occ, need = (n + kHWaves * kHRows - 1) / (kHWaves * kHRows);
    return (int)std::max<int64_t>(1, std::min(want, need));
}

size_t hessian_work_doubles(int k, int blocks) {
    const size_t entries = hess_entries(k);
    return (size_t)blocks * entries + entries;          // block partials, then G
}

hipError_t launch_hessian(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, const double *V,
                          const double *M, double nd, int extended, double *work, int blocks, bool clear,
                          unsigned *flag, double *H, hipStream_t stream) {
    if (k < 1 || k > PWA_MAX_K || blocks < 1) return hipErrorInvalidValue;
    HessV hv{};
    for (int i = 0; i < 2 * k; ++i) hv.v[i] = V[i];
    const int entries = (int)hess_entries(k);
    double *partials = work;
    double *Gm = partials + (size_t)blocks * entries;
    hipError_t e;
    if (clear) {            // the status word rests at zero between calls
        if ((e = hipMemsetAsync(flag, 0, sizeof(unsigned), stream)) != hipSuccess) return e;
    }
    if (n > 0) {
        e = prec == PWA_F32
                ? launch_data_pass(static_cast<const float *>(A), n, ld, k, hv, partials, flag, blocks, stream)
                : launch_data_pass(static_cast<const double *>(A), n, ld, k, hv, partials, flag, blocks, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(hess_sum_kernel, dim3(entries / 16), dim3(256), 0, stream, partials, n > 0 ? blocks : 0,
                       entries, Gm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(hess_assemble_kernel, dim3((4 * k * k + 255) / 256), dim3(256), 0, stream, Gm, hess_kp(k), M,
                       hv, k, nd, extended, flag, H);
    return hipGetLastError();
}

}  // namespace pwa
