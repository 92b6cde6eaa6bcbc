// Internal declarations of the gfx950 partial-wave likelihood library.
// Not part of the C ABI (include/pwa.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "pwa.h"

namespace pwa {

// Arguments of the fused single-V likelihood kernel.  Segment 0 is the data
// sample, segment 1 the MC sample; blocks [0, nb[0]) take segment 0.
struct StreamArgs {
    const void *A[2];          // device rows, ld complex each, zero padded past k
    const void *w;             // MC weights (context precision) or nullptr
    int64_t n[2];              // rows per segment
    int64_t ld;                // complex per row of the device layout
    int32_t nb[2];             // blocks per segment
    int32_t k;                 // waves
    int32_t pstride;           // doubles per block partial (1 + 2 ld)
    const double *v_dev;       // V on the device (2k doubles) or nullptr
    double *partials;          // [nb[0] + nb[1]][pstride]
    unsigned int *counter;     // finished-block counter, zero between launches
    double *out;               // [nll, grad[2k], flags]
    const double *gram;        // MC matrix (k x k complex FP64, 1/N_gen folded) or nullptr
    double n_gen;              // N_gen of the MC estimate (stream mode)
    double nd_total;           // N_D as a double
    int32_t extended;          // 0: Eq. 2 form, 1: Eq. 3 form
    int32_t pad_;
    double v_arg[2 * PWA_MAX_K];   // V by value when v_dev is null
};

// Tile shape of the streaming kernel: L lanes cooperate on one event row,
// each lane holding C consecutive complex amplitudes (ld = L * C).
struct StreamShape {
    int L;
    int C;
};

// Rows each lane group loads per loop iteration (enough independent loads in
// flight per lane); host and device share it to size the grid.
__host__ __device__ constexpr int stream_unroll(int bytes_per_lane_row) {
    return bytes_per_lane_row >= 32 ? 2 : (bytes_per_lane_row >= 16 ? 4 : 8);
}

// Rows one wave covers per loop iteration.
inline int stream_rows_per_wave(pwa_prec prec, StreamShape s) {
    const int bytes = (prec == PWA_F32 ? 8 : 16) * s.C;
    return (64 / s.L) * stream_unroll(bytes);
}

constexpr int kStreamThreads = 256;

// Chooses the shape for k waves in the given precision (smallest padded row,
// then the preferred per-lane load width).
StreamShape choose_shape(pwa_prec prec, int k);

// Launches the fused kernel with the given shape; returns hipSuccess or the launch error.
hipError_t launch_stream(pwa_prec prec, StreamShape s, int threads, int blocks,
                         const StreamArgs &args, hipStream_t stream);

// Gram matrix of the MC rows (Eq. 3 bracket), FP64 result on the device.
//   partials: device scratch of at least gram_partial_doubles(k, blocks) doubles.
hipError_t launch_gram(pwa_prec prec, const void *A, const void *w, int64_t n, int64_t ld, int k,
                       double n_gen, double *partials, int blocks, double *M, hipStream_t stream);
size_t gram_partial_doubles(int k, int blocks);

}  // namespace pwa
