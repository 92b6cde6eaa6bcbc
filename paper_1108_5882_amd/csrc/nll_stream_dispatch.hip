// Variant table, layout width and launch dispatch of the fused likelihood kernel.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "internal.hpp"

namespace pwa {

hipError_t stream_dispatch_f32_c1(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f32_c2(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f32_c3(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f32_c4(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f32_c8(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f64_c1(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f64_c2(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f64_c3(int, int, int, const StreamArgs &, hipStream_t);
hipError_t stream_dispatch_f64_c4(int, int, int, const StreamArgs &, hipStream_t);

namespace {

// (C, U) pairs compiled per precision; L runs over powers of two with L * C <= 64.
struct CU {
    int C, U;
};
const CU kF32[] = {{1, 4}, {1, 8}, {2, 2}, {2, 4}, {3, 1}, {3, 2}, {4, 1}, {4, 2}, {8, 1}};
const CU kF64[] = {{1, 2}, {1, 4}, {2, 1}, {2, 2}, {3, 1}, {4, 1}};

struct Table {
    StreamCfg v[128];
    int n = 0;
    Table(const CU *cu, int ncu) {
        for (int i = 0; i < ncu; ++i)
            for (int L = 1; L <= 32; L <<= 1)
                if (L * cu[i].C <= 64) v[n++] = StreamCfg{L, cu[i].C, cu[i].U, 0};
    }
};

const Table &table(pwa_prec prec) {
    static const Table f32(kF32, sizeof kF32 / sizeof kF32[0]);
    static const Table f64(kF64, sizeof kF64 / sizeof kF64[0]);
    return prec == PWA_F32 ? f32 : f64;
}

}  // namespace

const StreamCfg *stream_variants(pwa_prec prec, int *count) {
    const Table &t = table(prec);
    *count = t.n;
    return t.v;
}

bool stream_cfg_available(pwa_prec prec, const StreamCfg &c) {
    const Table &t = table(prec);
    for (int i = 0; i < t.n; ++i)
        if (t.v[i].L == c.L && t.v[i].C == c.C && t.v[i].U == c.U) return true;
    return false;
}

int stream_layout_ld(pwa_prec prec, int k) {
    const Table &t = table(prec);
    int best = 1 << 30;
    for (int i = 0; i < t.n; ++i) {
        const int ld = t.v[i].L * t.v[i].C;
        if (ld >= k && ld < best) best = ld;
    }
    return best;
}

StreamCfg stream_default_cfg(pwa_prec prec, int ld) {
    // Preference: about 32 B per lane per row (fewer lanes per row means less
    // redundant per-event work), 64 B per lane per stage, 4 blocks per CU.
    const Table &t = table(prec);
    const int eb = prec == PWA_F32 ? 8 : 16;
    StreamCfg best{0, 0, 0, 4};
    int best_score = 1 << 30;
    for (int i = 0; i < t.n; ++i) {
        const StreamCfg &c = t.v[i];
        if (c.L * c.C != ld) continue;
        const int row_bytes = c.C * eb, stage_bytes = row_bytes * c.U;
        const int score = std::abs(row_bytes - 32) * 4 + std::abs(stage_bytes - 64);
        if (score < best_score) {
            best_score = score;
            best = StreamCfg{c.L, c.C, c.U, 4};
        }
    }
    return best;
}

void stream_grid(const StreamCfg &cfg, int64_t budget, int64_t n0, int64_t n1, int32_t nb[2]) {
    const int64_t rows_per_block = (int64_t)stream_rows_per_wave(cfg) * (kStreamThreads / 64);
    const int64_t need[2] = {(n0 + rows_per_block - 1) / rows_per_block, (n1 + rows_per_block - 1) / rows_per_block};
    if (need[0] + need[1] <= budget) {
        nb[0] = (int32_t)need[0];
        nb[1] = (int32_t)need[1];
        return;
    }
    const double frac = (double)n0 / (double)(n0 + n1);
    int64_t b0 = (int64_t)std::llround(frac * (double)budget);
    if (n0 > 0) b0 = std::max<int64_t>(b0, 1);
    if (n1 > 0) b0 = std::min<int64_t>(b0, budget - 1);
    b0 = std::min(b0, need[0]);
    const int64_t b1 = std::min(budget - b0, need[1]);
    nb[0] = (int32_t)b0;
    nb[1] = (int32_t)b1;
}

hipError_t launch_stream(pwa_prec prec, const StreamCfg &c, int blocks, const StreamArgs &args,
                         hipStream_t stream) {
    // the kernel takes the row stride from its (L, C): the layout width
    if (!stream_cfg_available(prec, c) || blocks < 1 || args.ld != (int64_t)c.L * c.C) return hipErrorInvalidValue;
    if (prec == PWA_F32) {
        switch (c.C) {
            case 1: return stream_dispatch_f32_c1(c.L, c.U, blocks, args, stream);
            case 2: return stream_dispatch_f32_c2(c.L, c.U, blocks, args, stream);
            case 3: return stream_dispatch_f32_c3(c.L, c.U, blocks, args, stream);
            case 4: return stream_dispatch_f32_c4(c.L, c.U, blocks, args, stream);
            case 8: return stream_dispatch_f32_c8(c.L, c.U, blocks, args, stream);
            default: break;
        }
    } else {
        switch (c.C) {
            case 1: return stream_dispatch_f64_c1(c.L, c.U, blocks, args, stream);
            case 2: return stream_dispatch_f64_c2(c.L, c.U, blocks, args, stream);
            case 3: return stream_dispatch_f64_c3(c.L, c.U, blocks, args, stream);
            case 4: return stream_dispatch_f64_c4(c.L, c.U, blocks, args, stream);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace pwa
