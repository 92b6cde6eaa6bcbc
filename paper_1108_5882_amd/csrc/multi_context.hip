// C ABI of the multi-fit minimiser: staging of every fit's samples, the work
// item list of the persistent evaluation kernel, the L-BFGS state, and the
// HIP graph that holds one minimiser iteration (evaluate all fits, combine,
// advance all fits).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace pwa;

struct pwa_multi {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cu_count = 0;
    int nfits = 0;
    std::vector<MultiFit> fits;            // host copy (device pointers inside)
    std::vector<void *> rows;              // device allocations to free
    MultiFit *d_fits = nullptr;
    MultiItem *d_items = nullptr;
    int n_items = 0;
    unsigned *d_counter = nullptr;
    double *d_partials = nullptr;
    double *d_out = nullptr;
    LbfgsState *d_states = nullptr;
    int64_t item_bytes = 256 * 1024;       // target bytes of rows per work item
    int blocks_per_cu = 2;
    int m = 8;
    double c1 = 1e-4, ftol = 1e-12;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_merr;

pwa_status mfail(pwa_multi *m, pwa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (m ? m->err : g_merr) = buf;
    return st;
}

#define M_HIP(m, call, what)                                                                       \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return mfail(m, e_ == hipErrorOutOfMemory ? PWA_E_NOMEM : PWA_E_HIP, "%s: %s", what,   \
                         hipGetErrorString(e_));                                                   \
    } while (0)

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void drop_graph(pwa_multi *m) {
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->exec = nullptr;
    m->graph = nullptr;
}

// Cuts every fit's samples into work items of about item_bytes of rows.
pwa_status build_items(pwa_multi *m) {
    const int waves = kStreamThreads / 64;
    std::vector<MultiItem> items;
    for (int f = 0; f < m->nfits; ++f) {
        MultiFit &ft = m->fits[f];
        const int rpt = multi_rows_per_tile(ft.ld);
        const int64_t tile_bytes = (int64_t)rpt * 8 * ft.ld;
        int64_t tpi = std::max<int64_t>(waves, m->item_bytes / tile_bytes);
        tpi = (tpi + waves - 1) / waves * waves;
        for (int seg = 0; seg < 2; ++seg) {
            const int64_t n = seg ? ft.n_mc : ft.n_data;
            const int64_t tiles = (n + rpt - 1) / rpt;
            const int first = (int)items.size();
            for (int64_t t = 0; t < tiles; t += tpi) items.push_back(MultiItem{f, seg, t, std::min(t + tpi, tiles)});
            (seg ? ft.item_mc0 : ft.item_data0) = first;
            (seg ? ft.item_mc1 : ft.item_data1) = (int)items.size();
        }
    }
    if (m->d_items) (void)hipFree(m->d_items);
    if (m->d_partials) (void)hipFree(m->d_partials);
    m->d_items = nullptr;
    m->d_partials = nullptr;
    m->n_items = (int)items.size();
    const size_t ni = std::max<size_t>(1, items.size());
    M_HIP(m, hipMalloc(&m->d_items, sizeof(MultiItem) * ni), "hipMalloc(items)");
    M_HIP(m, hipMalloc(&m->d_partials, sizeof(double) * kMultiSlot * ni), "hipMalloc(partials)");
    if (!items.empty())
        M_HIP(m, hipMemcpy(m->d_items, items.data(), sizeof(MultiItem) * items.size(), hipMemcpyHostToDevice),
              "hipMemcpy(items)");
    M_HIP(m, hipMemcpy(m->d_fits, m->fits.data(), sizeof(MultiFit) * m->nfits, hipMemcpyHostToDevice),
          "hipMemcpy(fits)");
    drop_graph(m);
    return PWA_OK;
}

MultiArgs args_of(const pwa_multi *m) {
    MultiArgs a;
    a.fits = m->d_fits;
    a.items = m->d_items;
    a.n_fits = m->nfits;
    a.n_items = m->n_items;
    a.item_counter = m->d_counter;
    a.partials = m->d_partials;
    a.out = m->d_out;
    return a;
}

int grid_of(const pwa_multi *m) {
    return std::max(1, std::min(m->n_items, m->cu_count * m->blocks_per_cu));
}

pwa_status ensure_graph(pwa_multi *m) {
    if (m->exec) return PWA_OK;
    M_HIP(m, hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    hipError_t e = launch_multi_eval(args_of(m), grid_of(m), m->stream);
    if (e == hipSuccess)
        e = launch_lbfgs(m->d_fits, 0, m->d_out, kMultiOut, m->d_states, m->nfits, m->m, m->c1, m->ftol, m->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(m->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return mfail(m, PWA_E_HIP, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    m->graph = g;
    M_HIP(m, hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return PWA_OK;
}

// Writes every fit's start vector into its L-BFGS state (phase 0).
pwa_status reset_states(pwa_multi *m, const double *V0) {
    std::vector<LbfgsState> st(m->nfits);
    size_t off = 0;
    for (int f = 0; f < m->nfits; ++f) {
        LbfgsState &s = st[f];
        std::memset(&s, 0, sizeof s);
        const int n = 2 * m->fits[f].k;
        for (int i = 0; i < n; ++i) s.xt[i] = V0[off + i];
        off += n;
    }
    M_HIP(m, hipMemcpy(m->d_states, st.data(), sizeof(LbfgsState) * m->nfits, hipMemcpyHostToDevice),
          "hipMemcpy(states)");
    return PWA_OK;
}

}  // namespace

extern "C" {

pwa_status pwa_multi_create(pwa_multi **out, int device, int32_t nfits, const pwa_fit_desc *fits,
                            void *stream) {
    if (!out || nfits < 1 || !fits) return mfail(nullptr, PWA_E_INVAL, "bad arguments");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return mfail(nullptr, PWA_E_INVAL, "device %d not available", device);
    for (int f = 0; f < nfits; ++f) {
        const pwa_fit_desc &d = fits[f];
        if (d.k < 1 || d.k > kMultiMaxLd) return mfail(nullptr, PWA_E_UNSUPPORTED, "fit %d: k must be 1..%d", f, kMultiMaxLd);
        if (d.ld < d.k || d.n_data < 0 || d.n_mc < 0 || !d.V0) return mfail(nullptr, PWA_E_INVAL, "fit %d: bad sizes", f);
        if ((d.n_data > 0 && !d.A_data) || (d.n_mc > 0 && !d.A_mc)) return mfail(nullptr, PWA_E_INVAL, "fit %d: null rows", f);
        if (d.n_data > 0 && d.n_mc == 0) return mfail(nullptr, PWA_E_INVAL, "fit %d: no MC rows", f);
        for (int i = 0; i < 2 * d.k; ++i)
            if (!std::isfinite(d.V0[i])) return mfail(nullptr, PWA_E_INVAL, "fit %d: V0 not finite", f);
    }
    DevGuard dg(device);
    pwa_multi *m = new (std::nothrow) pwa_multi();
    if (!m) return mfail(nullptr, PWA_E_NOMEM, "out of host memory");
    m->device = device;
    m->nfits = nfits;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete m;
        return mfail(nullptr, PWA_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
    }
    m->cu_count = prop.multiProcessorCount;
    if (stream) {
        m->stream = static_cast<hipStream_t>(stream);
    } else if ((e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking)) != hipSuccess) {
        delete m;
        return mfail(nullptr, PWA_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
    } else {
        m->own_stream = true;
    }
    pwa_status st = PWA_OK;
    auto bail = [&](pwa_status s_) {
        g_merr = m->err;
        pwa_multi_destroy(m);
        return s_;
    };
    m->fits.resize(nfits);
    std::vector<double> V0;
    for (int f = 0; f < nfits; ++f) {
        const pwa_fit_desc &d = fits[f];
        MultiFit &ft = m->fits[f];
        std::memset(&ft, 0, sizeof ft);
        ft.k = d.k;
        ft.ld = multi_layout_ld(d.k);
        ft.n_data = d.n_data;
        ft.n_mc = d.n_mc;
        ft.n_gen = d.n_gen > 0 ? d.n_gen : (d.n_mc > 0 ? (double)d.n_mc : 1.0);
        const size_t row = 8 * (size_t)ft.ld;
        for (int seg = 0; seg < 2; ++seg) {
            const int64_t n = seg ? d.n_mc : d.n_data;
            if (n == 0) continue;
            void *buf = nullptr;
            if ((e = hipMalloc(&buf, row * n)) != hipSuccess) {
                mfail(m, PWA_E_NOMEM, "hipMalloc(rows): %s", hipGetErrorString(e));
                return bail(PWA_E_NOMEM);
            }
            m->rows.push_back(buf);
            const void *src = seg ? (const void *)d.A_mc : (const void *)d.A_data;
            if ((e = stage_rows(buf, row, src, 8 * (size_t)d.ld, 8 * (size_t)d.k, n, hipMemcpyHostToDevice,
                                m->stream)) != hipSuccess) {
                mfail(m, PWA_E_HIP, "staging rows: %s", hipGetErrorString(e));
                return bail(PWA_E_HIP);
            }
            (seg ? ft.A_mc : ft.A_data) = static_cast<const float *>(buf);
        }
        if (d.w_mc && d.n_mc > 0) {
            void *buf = nullptr;
            if ((e = hipMalloc(&buf, sizeof(float) * d.n_mc)) != hipSuccess ||
                (e = hipMemcpy(buf, d.w_mc, sizeof(float) * d.n_mc, hipMemcpyHostToDevice)) != hipSuccess) {
                if (buf) m->rows.push_back(buf);
                mfail(m, PWA_E_HIP, "staging weights: %s", hipGetErrorString(e));
                return bail(PWA_E_HIP);
            }
            m->rows.push_back(buf);
            ft.w_mc = static_cast<const float *>(buf);
        }
        V0.insert(V0.end(), d.V0, d.V0 + 2 * d.k);
    }
    if ((e = hipMalloc(&m->d_fits, sizeof(MultiFit) * nfits)) != hipSuccess ||
        (e = hipMalloc(&m->d_counter, sizeof(unsigned))) != hipSuccess ||
        (e = hipMemset(m->d_counter, 0, sizeof(unsigned))) != hipSuccess ||
        (e = hipMalloc(&m->d_out, sizeof(double) * kMultiOut * nfits)) != hipSuccess ||
        (e = hipMalloc(&m->d_states, sizeof(LbfgsState) * nfits)) != hipSuccess) {
        mfail(m, PWA_E_NOMEM, "hipMalloc: %s", hipGetErrorString(e));
        return bail(PWA_E_NOMEM);
    }
    for (int f = 0; f < nfits; ++f) m->fits[f].V = m->d_states[f].xt;   // evaluation reads the trial point
    if ((st = build_items(m)) != PWA_OK) return bail(st);
    if ((st = reset_states(m, V0.data())) != PWA_OK) return bail(st);
    *out = m;
    return PWA_OK;
}

pwa_status pwa_multi_destroy(pwa_multi *m) {
    if (!m) return PWA_OK;
    DevGuard dg(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    drop_graph(m);
    for (void *b : m->rows) (void)hipFree(b);
    for (void *b : {(void *)m->d_fits, (void *)m->d_items, (void *)m->d_counter, (void *)m->d_partials,
                    (void *)m->d_out, (void *)m->d_states})
        if (b) (void)hipFree(b);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return PWA_OK;
}

pwa_status pwa_multi_reset(pwa_multi *m, const double *V0) {
    if (!m || !V0) return mfail(m, PWA_E_INVAL, "null argument");
    DevGuard dg(m->device);
    M_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return reset_states(m, V0);
}

pwa_status pwa_multi_eval(pwa_multi *m, const double *V, double *nll, double *grad) {
    if (!m || !V || !nll) return mfail(m, PWA_E_INVAL, "null argument");
    DevGuard dg(m->device);
    M_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    size_t off = 0;
    for (int f = 0; f < m->nfits; ++f) {
        const int n = 2 * m->fits[f].k;
        M_HIP(m, hipMemcpyAsync(m->d_states[f].xt, V + off, sizeof(double) * n, hipMemcpyHostToDevice, m->stream),
              "hipMemcpyAsync(V)");
        off += n;
    }
    hipError_t e = launch_multi_eval(args_of(m), grid_of(m), m->stream);
    if (e != hipSuccess) return mfail(m, PWA_E_HIP, "multi-fit launch: %s", hipGetErrorString(e));
    std::vector<double> out((size_t)kMultiOut * m->nfits);
    M_HIP(m, hipMemcpyAsync(out.data(), m->d_out, sizeof(double) * out.size(), hipMemcpyDeviceToHost, m->stream),
          "hipMemcpyAsync(out)");
    M_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    off = 0;
    bool domain = false;
    for (int f = 0; f < m->nfits; ++f) {
        const int k = m->fits[f].k;
        const double *o = out.data() + (size_t)f * kMultiOut;
        nll[f] = o[0];
        domain |= o[1 + 2 * k] != 0.0;
        if (grad) std::copy(o + 1, o + 1 + 2 * k, grad + off);
        off += 2 * k;
    }
    return domain ? mfail(m, PWA_E_DOMAIN, "non-positive intensity or normalisation") : PWA_OK;
}

pwa_status pwa_multi_step(pwa_multi *m, int32_t steps, double *avg_ms) {
    if (!m || steps < 0) return mfail(m, PWA_E_INVAL, "bad arguments");
    DevGuard dg(m->device);
    pwa_status st = ensure_graph(m);
    if (st != PWA_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (avg_ms) {
        M_HIP(m, hipEventCreate(&e0), "hipEventCreate");
        M_HIP(m, hipEventCreate(&e1), "hipEventCreate");
        M_HIP(m, hipEventRecord(e0, m->stream), "hipEventRecord");
    }
    for (int s = 0; s < steps; ++s) M_HIP(m, hipGraphLaunch(m->exec, m->stream), "hipGraphLaunch");
    if (avg_ms) {
        M_HIP(m, hipEventRecord(e1, m->stream), "hipEventRecord");
        M_HIP(m, hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0.f;
        M_HIP(m, hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        *avg_ms = steps ? ms / steps : 0.0;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    M_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_multi_get(pwa_multi *m, double *V, double *nll, int32_t *status, int32_t *iters) {
    if (!m) return mfail(nullptr, PWA_E_INVAL, "null argument");
    DevGuard dg(m->device);
    M_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    std::vector<LbfgsState> st(m->nfits);
    M_HIP(m, hipMemcpy(st.data(), m->d_states, sizeof(LbfgsState) * m->nfits, hipMemcpyDeviceToHost),
          "hipMemcpy(states)");
    size_t off = 0;
    for (int f = 0; f < m->nfits; ++f) {
        const int n = 2 * m->fits[f].k;
        // before the first evaluation the accepted point is the start point
        const bool started = st[f].phase != 0;
        if (V) for (int i = 0; i < n; ++i) V[off + i] = started ? st[f].x[i] : st[f].xt[i];
        if (nll) nll[f] = started ? st[f].f : NAN;
        if (status) status[f] = st[f].status;
        if (iters) iters[f] = st[f].iter;
        off += n;
    }
    return PWA_OK;
}

pwa_status pwa_multi_autotune(pwa_multi *m, int32_t reps, int64_t *item_bytes, int32_t *blocks_per_cu,
                              double *best_ms) {
    if (!m) return mfail(nullptr, PWA_E_INVAL, "null argument");
    if (reps < 1) reps = 1;
    DevGuard dg(m->device);
    static const int64_t kBytes[] = {64 << 10, 128 << 10, 256 << 10, 512 << 10, 1 << 20, 2 << 20, 4 << 20};
    static const int kBpc[] = {1, 2, 3, 4, 6, 8, 12, 16};
    hipEvent_t e0, e1;
    M_HIP(m, hipEventCreate(&e0), "hipEventCreate");
    M_HIP(m, hipEventCreate(&e1), "hipEventCreate");
    int64_t best_b = m->item_bytes;
    int best_c = m->blocks_per_cu;
    double best_t = 1e30;
    pwa_status st = PWA_OK;
    for (int64_t b : kBytes) {
        m->item_bytes = b;
        if ((st = build_items(m)) != PWA_OK) break;
        for (int c : kBpc) {
            m->blocks_per_cu = c;
            hipError_t e = launch_multi_eval(args_of(m), grid_of(m), m->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, m->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_multi_eval(args_of(m), grid_of(m), m->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, m->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = mfail(m, PWA_E_HIP, "autotune: %s", hipGetErrorString(e));
                break;
            }
            if (ms / reps < best_t) {
                best_t = ms / reps;
                best_b = b;
                best_c = c;
            }
        }
        if (st != PWA_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    m->item_bytes = best_b;
    m->blocks_per_cu = best_c;
    pwa_status st2 = build_items(m);
    if (st != PWA_OK) return st;
    if (st2 != PWA_OK) return st2;
    if (item_bytes) *item_bytes = best_b;
    if (blocks_per_cu) *blocks_per_cu = best_c;
    if (best_ms) *best_ms = best_t;
    return PWA_OK;
}

const char *pwa_multi_last_error(const pwa_multi *m) { return m ? m->err.c_str() : g_merr.c_str(); }

}  // extern "C"
