// Fixed-order reduction of per-block FP64 partials inside the launch that
// produced them (no second kernel): blocks are grouped by kFinishGroup; the
// last block to arrive in each group (arrival counter) adds the group's
// partials in block order, and the last group to arrive adds the group sums
// in group order.  Every addition has a fixed place in that order, so results
// are bitwise reproducible for a launch configuration.  Both levels are
// compensated (Neumaier) sums, each folding its running error term into its
// result.
#pragma once

#include "internal.hpp"

namespace pwa {

// ------------------------------------------- combine of the block partials
// Partials and group sums cross blocks, and so the XCDs' separate L2 caches.
// They are stored and loaded as device-scope atomics (written through to, and
// read from, the device's coherence point), and each block waits for its own
// stores to complete before the arrival count that announces them.  A
// device-scope fence would order plain stores too, but on gfx950 it writes
// back and invalidates the whole L2 of the block's XCD, which costs far more
// than the pass over the rows when every block pays it.
__device__ __forceinline__ void st_dev(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the result may go to host memory: written through at system scope
__device__ __forceinline__ void st_sys(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// s + x with the rounding error of the addition added to c (Neumaier's form of
// Kahan summation: the error of the larger operand's sum is exact either way)
__device__ __forceinline__ void comp_add(double &s, double &c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// every memory operation this wave issued has completed
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0); }

// Where the block partials of one launch go: nb0 data blocks, then the MC
// blocks up to nbt, PS doubles each; group sums; arrival counters.
struct ReduceBufs {
    double *partials;
    double *gsums;
    unsigned *counters;
    int nb0, nbt;
};

// Called by every block after it stored its partial with st_dev.  The last
// block of each group adds the group's partials; the last group adds the
// group sums.  Returns true in that one block only (the same value in all its
// threads), with tot[0 .. PS) the data totals and tot[PS .. 2 PS) the MC totals.
template <int PS, int NT>
__device__ __forceinline__ bool reduce_blocks(const ReduceBufs &p, double *tot) {
    __shared__ unsigned s_last;
    const int tid = threadIdx.x;
    const int nbt = p.nbt;
    const int grp = (int)blockIdx.x / kFinishGroup;
    const int g0 = grp * kFinishGroup;
    const int gn = min(kFinishGroup, nbt - g0);
    const int ngroups = (nbt + kFinishGroup - 1) / kFinishGroup;

    wait_stores();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&p.counters[1 + grp], 1u) == (unsigned)(gn - 1);
    __syncthreads();
    if (!s_last) return false;

    // group sums: data columns then MC columns, blocks in order (all loads of a
    // column in flight at once; blocks outside the group or the segment add 0)
    for (int col = tid; col < 2 * PS; col += NT) {
        const int sg = col >= PS ? 1 : 0;
        const int c = col - sg * PS;
        double v[kFinishGroup];
#pragma unroll
        for (int i = 0; i < kFinishGroup; ++i)
            v[i] = ld_dev(p.partials + (int64_t)(g0 + (i < gn ? i : gn - 1)) * PS + c);
        double s = 0.0, e = 0.0;
#pragma unroll
        for (int i = 0; i < kFinishGroup; ++i) {
            const bool take = i < gn && ((g0 + i >= p.nb0) == (sg == 1));
            comp_add(s, e, take ? v[i] : 0.0);
        }
        st_dev(p.gsums + (int64_t)grp * 2 * PS + col, s + e);
    }
    if (tid == 0) __hip_atomic_store(&p.counters[1 + grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    wait_stores();
    __syncthreads();
    if (tid == 0) s_last = atomicAdd(&p.counters[0], 1u) == (unsigned)(ngroups - 1);
    __syncthreads();
    if (!s_last) return false;

    // totals over the groups: TPC threads per column, thread r adding groups
    // r, r + TPC, ... in order (16 loads in flight), then the TPC sums of a
    // column in thread order
    constexpr int NCOL = 2 * PS;
    constexpr int TPC = NT / NCOL > 0 ? NT / NCOL : 1;
    __shared__ double part[NCOL * TPC], part_e[NCOL * TPC];
    for (int slot = tid; slot < NCOL * TPC; slot += NT) {
        const int col = slot / TPC, r = slot % TPC;
        double s = 0.0, e = 0.0;
        for (int gb = r; gb < ngroups; gb += 16 * TPC) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int gi = gb + u * TPC;
                v[u] = ld_dev(p.gsums + (int64_t)(gi < ngroups ? gi : ngroups - 1) * NCOL + col);
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) comp_add(s, e, gb + u * TPC < ngroups ? v[u] : 0.0);
        }
        part[slot] = s;
        part_e[slot] = e;
    }
    if (tid == 0) __hip_atomic_store(&p.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    for (int col = tid; col < NCOL; col += NT) {
        double s = 0.0, e = 0.0;
        for (int r = 0; r < TPC; ++r) {
            comp_add(s, e, part[col * TPC + r]);
            e += part_e[col * TPC + r];
        }
        tot[col] = s + e;
    }
    __syncthreads();
    return true;
}

}  // namespace pwa
