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
// One pass over the data rows: each block stages a tile of rows in LDS as
// FP64, forms z and 1/z^2 per row in FP64 and accumulates its share of T;
// the block partials are added in block order, then one block assembles H.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kHThreads = 256;
constexpr int kHRows = 32;
constexpr int kHMaxTiles = 3;     // 2 x 2 entry tiles per thread (k = 64: 528 tiles over 256 threads)

__global__ void hess_clear_kernel(unsigned *flag) { *flag = 0u; }

// Upper-triangle 2 x 2 tile t -> (ta, tc), ta <= tc, of nt tile rows (row-major order).
__device__ __forceinline__ void tile_index(int t, int nt, int &ta, int &tc) {
    int a = 0, row = nt;
    while (t >= row) {
        t -= row;
        ++a;
        --row;
    }
    ta = a;
    tc = a + t;
}

// T is complex symmetric: each thread accumulates 2 x 2 tiles (ta, tc) of the
// upper triangle (rows 2 ta, 2 ta + 1, columns 2 tc, 2 tc + 1).  With fewer
// tiles than threads the block forms RG = 256 / ntile row groups that take every
// RG-th row of the LDS tile; the groups' sums are added in group order at the
// end.  z comes from 8 lanes per row.
template <typename T>
__global__ __launch_bounds__(kHThreads) void hess_partial_kernel(const T *__restrict__ A, int64_t n, int64_t ld,
                                                                 int k, const double *__restrict__ V,
                                                                 double *__restrict__ partials,
                                                                 unsigned *__restrict__ flag) {
    __shared__ __attribute__((aligned(16))) double tile[kHRows][2 * PWA_MAX_K + 4];
    __shared__ __attribute__((aligned(16))) double cw[kHRows][2];   // 1 / z^2 per row (0 for absent rows)
    __shared__ double red[kHThreads][8];              // row-group sums (one tile per slot then)
    const int tid = threadIdx.x;
    const int nt = (k + 1) / 2;                       // tile rows
    const int ntile = nt * (nt + 1) / 2;
    const int S = ntile < kHThreads ? ntile : kHThreads;   // tile slots per row group
    const int RG = kHThreads / S;                     // row groups (threads past RG S idle)
    const int rg = tid / S, slot = tid % S;
    const int kk = k * k;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * chunk;
    const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;

    int tA[kHMaxTiles], tC[kHMaxTiles];
#pragma unroll
    for (int m = 0; m < kHMaxTiles; ++m) {
        const int t = slot + m * S;
        tA[m] = tC[m] = -1;
        if (rg < RG && t < ntile) tile_index(t, nt, tA[m], tC[m]);
    }
    double acc[kHMaxTiles][8];                         // (re, im) of entries 00, 01, 10, 11
#pragma unroll
    for (int m = 0; m < kHMaxTiles; ++m)
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[m][q] = 0.0;
    bool bad = false;

    // the next tile's values are loaded into registers while the current one is used
    constexpr int kPre = kHRows * 2 * PWA_MAX_K / kHThreads;
    T pre[kPre];
    const int width = 4 * nt;                          // staged columns (zero beyond 2k)
    auto fetch = [&](int64_t b) {
        const int rws = (int)(r1 - b < kHRows ? r1 - b : kHRows);
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
            const int idx = tid + i * kHThreads;
            const int r = idx / width, q = idx % width;
            pre[i] = (idx < kHRows * width && r < rws && q < 2 * k) ? A[2 * (b + r) * ld + q] : T(0);
        }
    };
    if (r0 < r1) fetch(r0);
    for (int64_t base = r0; base < r1; base += kHRows) {
        const int rows = (int)(r1 - base < kHRows ? r1 - base : kHRows);
        __syncthreads();
        // rows as FP64, zero beyond k (an odd k's last tile reads one zero column)
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
            const int idx = tid + i * kHThreads;
            if (idx < kHRows * width) tile[idx / width][idx % width] = (double)pre[i];
        }
        __syncthreads();
        if (base + kHRows < r1) fetch(base + kHRows);
        {
            // z of row tid / 8 from 8 lanes (waves sub, sub + 8, ...), summed over the lanes
            const int row = tid >> 3, sub = tid & 7;
            double zr = 0.0, zi = 0.0;
            if (row < rows)
                for (int a = sub; a < k; a += 8) {
                    const double ar = tile[row][2 * a], ai = tile[row][2 * a + 1];
                    zr = fma(V[2 * a], ar, fma(-V[2 * a + 1], ai, zr));
                    zi = fma(V[2 * a], ai, fma(V[2 * a + 1], ar, zi));
                }
#pragma unroll
            for (int off = 1; off < 8; off <<= 1) {
                zr += __shfl_xor(zr, off);
                zi += __shfl_xor(zi, off);
            }
            if (sub == 0) {
                double wr = 0.0, wi = 0.0;
                if (row < rows) {
                    const double I = zr * zr + zi * zi;
                    if (I > 0.0 && isfinite(I)) {
                        // 1 / z^2 = conj(z)^2 / I^2
                        const double i2 = 1.0 / (I * I);
                        wr = (zr * zr - zi * zi) * i2;
                        wi = -2.0 * zr * zi * i2;
                    } else {
                        bad = true;
                    }
                }
                cw[row][0] = wr;
                cw[row][1] = wi;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < kHMaxTiles; ++m) {
            if (tA[m] < 0) continue;
            const int a0 = 2 * tA[m], c0 = 2 * tC[m];
            double s[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) s[q] = acc[m][q];
            for (int r = rg; r < rows; r += RG) {
                const double wr = cw[r][0], wi = cw[r][1];
                const double x0r = tile[r][2 * a0], x0i = tile[r][2 * a0 + 1];
                const double x1r = tile[r][2 * a0 + 2], x1i = tile[r][2 * a0 + 3];
                const double y0r = tile[r][2 * c0], y0i = tile[r][2 * c0 + 1];
                const double y1r = tile[r][2 * c0 + 2], y1i = tile[r][2 * c0 + 3];
                // (w x) then times y, for the four entries
                const double u0r = fma(wr, x0r, -(wi * x0i)), u0i = fma(wr, x0i, wi * x0r);
                const double u1r = fma(wr, x1r, -(wi * x1i)), u1i = fma(wr, x1i, wi * x1r);
                s[0] = fma(u0r, y0r, fma(-u0i, y0i, s[0]));
                s[1] = fma(u0r, y0i, fma(u0i, y0r, s[1]));
                s[2] = fma(u0r, y1r, fma(-u0i, y1i, s[2]));
                s[3] = fma(u0r, y1i, fma(u0i, y1r, s[3]));
                s[4] = fma(u1r, y0r, fma(-u1i, y0i, s[4]));
                s[5] = fma(u1r, y0i, fma(u1i, y0r, s[5]));
                s[6] = fma(u1r, y1r, fma(-u1i, y1i, s[6]));
                s[7] = fma(u1r, y1i, fma(u1i, y1r, s[7]));
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[m][q] = s[q];
        }
    }
    if (bad) atomicOr(flag, 1u);
    // add the row groups in group order; with RG > 1 there are fewer tiles than
    // slots, so each slot holds only its first tile
    __syncthreads();
    if (RG > 1) {
#pragma unroll
        for (int q = 0; q < 8; ++q) red[tid][q] = acc[0][q];
        __syncthreads();
        if (rg == 0) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                double v = red[slot][q];
                for (int g = 1; g < RG; ++g) v += red[g * S + slot][q];
                acc[0][q] = v;
            }
        }
    }
    if (rg != 0) return;
    double *out = partials + (int64_t)blockIdx.x * 2 * kk;
#pragma unroll
    for (int m = 0; m < kHMaxTiles; ++m) {
        if (tA[m] < 0) continue;
#pragma unroll
        for (int ea = 0; ea < 2; ++ea)
#pragma unroll
            for (int ec = 0; ec < 2; ++ec) {
                const int a = 2 * tA[m] + ea, c = 2 * tC[m] + ec;
                if (a >= k || c >= k) continue;
                const double vr = acc[m][4 * ea + 2 * ec], vi = acc[m][4 * ea + 2 * ec + 1];
                out[2 * (a * k + c)] = vr;
                out[2 * (a * k + c) + 1] = vi;
                out[2 * (c * k + a)] = vr;          // T is symmetric
                out[2 * (c * k + a) + 1] = vi;
            }
    }
}

// T = sum of the block partials: one block per entry, fixed-order tree.
constexpr int kFinThreads = 64;
__global__ __launch_bounds__(kFinThreads) void hess_finish_kernel(const double *__restrict__ partials, int nblocks,
                                                                  int k, double *__restrict__ Tm) {
    const int kk2 = 2 * k * k;
    const int e = blockIdx.x;
    double s = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x; b < nblocks; b += kFinThreads) s += partials[(int64_t)b * kk2 + e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    if (threadIdx.x == 0) Tm[e] = s;
}

// One block: H (2k x 2k, row-major) from T, M and V; H[2k * 2k] = status flags.
__global__ void hess_assemble_kernel(const double *__restrict__ Tm, const double *__restrict__ M,
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
        const double tr = Tm[2 * (a * k + c)], ti = Tm[2 * (a * k + c) + 1];
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

size_t hessian_partial_doubles(int k, int blocks) { return (size_t)blocks * 2 * k * k; }

hipError_t launch_hessian(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, const double *V_dev,
                          const double *M, double nd, int extended, double *partials, int blocks, double *Tm,
                          unsigned *flag, double *H, hipStream_t stream) {
    if (k < 1 || k > PWA_MAX_K || blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hess_clear_kernel, dim3(1), dim3(1), 0, stream, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > 0) {
        if (prec == PWA_F32)
            hipLaunchKernelGGL(hess_partial_kernel<float>, dim3(blocks), dim3(kHThreads), 0, stream,
                               static_cast<const float *>(A), n, ld, k, V_dev, partials, flag);
        else
            hipLaunchKernelGGL(hess_partial_kernel<double>, dim3(blocks), dim3(kHThreads), 0, stream,
                               static_cast<const double *>(A), n, ld, k, V_dev, partials, flag);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        blocks = 0;
    }
    const int kk2 = 2 * k * k;
    hipLaunchKernelGGL(hess_finish_kernel, dim3(kk2), dim3(kFinThreads), 0, stream, partials, blocks, k, Tm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(hess_assemble_kernel, dim3(1), dim3(256), 0, stream, Tm, M, V_dev, k, nd, extended, flag, H);
    return hipGetLastError();
}

}  // namespace pwa
