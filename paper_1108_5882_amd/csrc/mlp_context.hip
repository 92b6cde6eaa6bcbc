// C ABI of the NLL surrogate network: device buffers, parameter I/O, the
// training steps captured in HIP graphs (one step, and groups of 16), chunked inference and top-k
// selection.  Every entry point orders its work on the object's stream and
// waits for it before returning.
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

struct pwa_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    MlpBuffers m{};
    std::vector<void *> allocs;
    float *tk_key[2] = {nullptr, nullptr};
    int *tk_idx[2] = {nullptr, nullptr};
    size_t tk_cap = 0;
    hipGraph_t graph = nullptr, graph_n = nullptr;      // one training step; kGroupSteps steps
    hipGraphExec_t exec = nullptr, exec_n = nullptr;
    struct Key {
        const float *X, *t;
        int64_t n;
        const int *perm;
        int B;
        float lr;
        float *hist;
        bool operator==(const Key &o) const {
            return X == o.X && t == o.t && n == o.n && perm == o.perm && B == o.B && lr == o.lr && hist == o.hist;
        }
    } key{};
    std::string err;
};

namespace {

thread_local std::string g_lerr;

pwa_status lfail(pwa_mlp *m, pwa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (m ? m->err : g_lerr) = buf;
    return st;
}

#define L_HIP(m, call, what)                                                                              \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return lfail(m, e_ == hipErrorOutOfMemory ? PWA_E_NOMEM : PWA_E_HIP, "%s: %s", what,         \
                         hipGetErrorString(e_));                                                          \
    } while (0)

struct Guard {
    int prev = -1;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Guard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <typename T>
pwa_status alloc(pwa_mlp *m, T **p, size_t count) {
    void *q = nullptr;
    L_HIP(m, hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1)), "hipMalloc");
    m->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return PWA_OK;
}

void drop_graph(pwa_mlp *m) {
    for (hipGraphExec_t *x : {&m->exec, &m->exec_n}) {
        if (*x) (void)hipGraphExecDestroy(*x);
        *x = nullptr;
    }
    for (hipGraph_t *g : {&m->graph, &m->graph_n}) {
        if (*g) (void)hipGraphDestroy(*g);
        *g = nullptr;
    }
}

// Training steps replayed as one graph (the launch gap between graphs is paid
// once per group).
constexpr int kGroupSteps = 16;

// count training steps captured into *g and instantiated into *x.
hipError_t capture_steps(pwa_mlp *m, const float *X, const float *t, int64_t n, const int32_t *perm, int batch,
                         float lr, float *loss_hist, int count, hipGraph_t *g, hipGraphExec_t *x) {
    const MlpBuffers &b = m->m;
    hipError_t e = hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t ec = hipSuccess;
    for (int i = 0; i < count && ec == hipSuccess; ++i) {
        if (mlp_fused_ok(b)) {   // two launches: row pass, then weight gradients with Adam
            ec = mlp_fused_pass(b, batch, X, t, perm, n, true, 1.0f / (float)batch, lr, loss_hist, m->stream);
        } else {
            ec = mlp_gather(b, X, t, n, perm, batch, m->stream);
            if (ec == hipSuccess) ec = mlp_pass(b, batch, b.Xb, b.tb, b.y, true, loss_hist, m->stream);
            if (ec == hipSuccess) ec = mlp_adam(b, 1.0f / (float)batch, lr, m->stream);
            if (ec == hipSuccess) ec = mlp_step_inc(b, m->stream);
        }
    }
    e = hipStreamEndCapture(m->stream, g);
    if (ec != hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(x, *g, nullptr, nullptr, 0);
    return e;
}

}  // namespace

extern "C" {

int64_t pwa_mlp_param_count(int32_t in, int32_t hidden) {
    if (in < 1 || hidden < 1) return -1;
    return mlp_param_count(in, hidden);
}

pwa_status pwa_mlp_create(pwa_mlp **out, int device, int32_t in, int32_t hidden, int32_t max_batch,
                          void *stream) {
    if (!out) return lfail(nullptr, PWA_E_INVAL, "null output pointer");
    if (in < 1 || in > 2 * PWA_MAX_K || hidden < 1 || hidden > 4096 || max_batch < 1 || max_batch > 65536)
        return lfail(nullptr, PWA_E_INVAL, "bad network shape (in 1..%d, hidden 1..4096, max_batch 1..65536)",
                     2 * PWA_MAX_K);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return lfail(nullptr, PWA_E_INVAL, "device %d not available", device);
    Guard g(device);
    pwa_mlp *m = new (std::nothrow) pwa_mlp();
    if (!m) return lfail(nullptr, PWA_E_NOMEM, "out of host memory");
    m->device = device;
    if (stream) {
        m->stream = static_cast<hipStream_t>(stream);
    } else if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) {
        delete m;
        return lfail(nullptr, PWA_E_HIP, "hipStreamCreate failed");
    } else {
        m->own_stream = true;
    }
    MlpBuffers &b = m->m;
    b.in = in;
    b.hidden = hidden;
    b.max_batch = max_batch;
    b.nparams = mlp_param_count(in, hidden);
    const size_t act = (size_t)max_batch * hidden;
    int *ints = nullptr;
    pwa_status st;
    if ((st = alloc(m, &b.P, b.nparams)) || (st = alloc(m, &b.G, b.nparams)) || (st = alloc(m, &b.M1, b.nparams)) ||
        (st = alloc(m, &b.M2, b.nparams)) || (st = alloc(m, &b.Z1, act)) || (st = alloc(m, &b.H1, act)) ||
        (st = alloc(m, &b.Z2, act)) || (st = alloc(m, &b.H2, act)) || (st = alloc(m, &b.dZ1, act)) ||
        (st = alloc(m, &b.dZ2, act)) || (st = alloc(m, &b.y, max_batch)) || (st = alloc(m, &b.dy, max_batch)) ||
        (st = alloc(m, &b.lrow, max_batch)) || (st = alloc(m, &b.loss, 1)) ||
        (st = alloc(m, &b.Xb, (size_t)max_batch * in)) || (st = alloc(m, &b.tb, max_batch)) ||
        (st = alloc(m, &b.ws, (size_t)mlp_workspace_floats(in, hidden))) ||
        (st = alloc(m, &ints, 4))) {
        g_lerr = m->err;
        pwa_mlp_destroy(m);
        return st;
    }
    b.step = ints;
    b.batch = ints + 1;
    b.bad = ints + 2;
    b.ftnext = ints + 3;
    if (hidden == 256 && in <= 128) {   // buffers of the fused training pass
        if ((st = alloc(m, &b.fact, mlp_fused_act_halfs(max_batch))) ||
            (st = alloc(m, &b.fvec, mlp_fused_vec_floats(max_batch))) ||
            (st = alloc(m, &b.fwh, mlp_fused_wh_halfs()))) {
            g_lerr = m->err;
            pwa_mlp_destroy(m);
            return st;
        }
    }
    hipError_t e = hipMemsetAsync(b.P, 0, sizeof(float) * b.nparams, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.M1, 0, sizeof(float) * b.nparams, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.M2, 0, sizeof(float) * b.nparams, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(ints, 0, sizeof(int) * 4, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        g_lerr = std::string("initialisation: ") + hipGetErrorString(e);
        pwa_mlp_destroy(m);
        return PWA_E_HIP;
    }
    *out = m;
    return PWA_OK;
}

pwa_status pwa_mlp_destroy(pwa_mlp *m) {
    if (!m) return PWA_OK;
    Guard g(m->device);
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    drop_graph(m);
    for (void *p : m->allocs) (void)hipFree(p);
    for (int i = 0; i < 2; ++i) {
        if (m->tk_key[i]) (void)hipFree(m->tk_key[i]);
        if (m->tk_idx[i]) (void)hipFree(m->tk_idx[i]);
    }
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    delete m;
    return PWA_OK;
}

pwa_status pwa_mlp_set_params(pwa_mlp *m, const float *P, pwa_where where) {
    if (!m || !P) return lfail(m, PWA_E_INVAL, "null argument");
    Guard g(m->device);
    const MlpBuffers &b = m->m;
    L_HIP(m, hipMemcpyAsync(b.P, P, sizeof(float) * b.nparams,
                            where == PWA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, m->stream),
          "hipMemcpyAsync(params)");
    L_HIP(m, hipMemsetAsync(b.M1, 0, sizeof(float) * b.nparams, m->stream), "hipMemsetAsync");
    L_HIP(m, hipMemsetAsync(b.M2, 0, sizeof(float) * b.nparams, m->stream), "hipMemsetAsync");
    L_HIP(m, hipMemsetAsync(b.step, 0, sizeof(int), m->stream), "hipMemsetAsync");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_mlp_get_params(pwa_mlp *m, float *P, pwa_where where) {
    if (!m || !P) return lfail(m, PWA_E_INVAL, "null argument");
    Guard g(m->device);
    L_HIP(m, hipMemcpyAsync(P, m->m.P, sizeof(float) * m->m.nparams,
                            where == PWA_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, m->stream),
          "hipMemcpyAsync(params)");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_mlp_features(pwa_mlp *m, const double *V, int64_t n, int32_t k, float *X) {
    if (!m || (n > 0 && (!V || !X)) || n < 0) return lfail(m, PWA_E_INVAL, "bad arguments");
    if (2 * k != m->m.in) return lfail(m, PWA_E_INVAL, "2k = %d does not match the input width %d", 2 * k, m->m.in);
    Guard g(m->device);
    L_HIP(m, mlp_features(V, n, k, X, m->stream), "features launch");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_mlp_targets(pwa_mlp *m, const double *nll, int64_t n, float *t) {
    if (!m || n < 1 || !nll || !t) return lfail(m, PWA_E_INVAL, "bad arguments");
    Guard g(m->device);
    L_HIP(m, mlp_targets(nll, n, t, m->stream), "targets launch");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_mlp_predict(pwa_mlp *m, const float *X, int64_t n, float *y) {
    if (!m || n < 0 || (n > 0 && (!X || !y))) return lfail(m, PWA_E_INVAL, "bad arguments");
    Guard g(m->device);
    const MlpBuffers &b = m->m;
    for (int64_t off = 0; off < n; off += b.max_batch) {
        const int B = (int)std::min<int64_t>(b.max_batch, n - off);
        L_HIP(m, mlp_pass(b, B, X + off * b.in, nullptr, y + off, false, nullptr, m->stream), "forward launch");
    }
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

pwa_status pwa_mlp_loss_grad(pwa_mlp *m, const float *X, const float *t, int32_t B, float *loss, float *G) {
    if (!m || !X || !t || !G) return lfail(m, PWA_E_INVAL, "null argument");
    if (B < 1 || B > m->m.max_batch) return lfail(m, PWA_E_INVAL, "batch %d outside 1..%d", B, m->m.max_batch);
    Guard g(m->device);
    const MlpBuffers &b = m->m;
    if (mlp_fused_ok(b)) {
        L_HIP(m, mlp_set_int(b.bad, 0, m->stream), "reset launch");
        L_HIP(m, mlp_fused_weights(b, m->stream), "weights launch");
        L_HIP(m, mlp_fused_pass(b, B, X, t, nullptr, B, false, 1.0f, 0.0f, nullptr, m->stream),
              "fused training pass launch");
    } else {
        L_HIP(m, mlp_pass(b, B, X, t, b.y, true, nullptr, m->stream), "training pass launch");
    }
    L_HIP(m, mlp_scale(b.G, b.nparams, 1.0f / (float)B, G, m->stream), "scale launch");
    float l = 0.f;
    L_HIP(m, hipMemcpyAsync(&l, b.loss, sizeof(float), hipMemcpyDeviceToHost, m->stream), "hipMemcpyAsync(loss)");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    if (loss) *loss = l;
    return PWA_OK;
}

pwa_status pwa_mlp_train(pwa_mlp *m, const float *X, const float *t, int64_t n, const int32_t *perm, int32_t batch,
                         int32_t nsteps, float lr, float *loss_hist, double *avg_ms) {
    if (!m || !X || !t || !perm || n < 1) return lfail(m, PWA_E_INVAL, "bad arguments");
    if (batch < 1 || batch > m->m.max_batch) return lfail(m, PWA_E_INVAL, "batch %d outside 1..%d", batch, m->m.max_batch);
    if (nsteps < 0 || !(lr > 0.f) || !std::isfinite(lr)) return lfail(m, PWA_E_INVAL, "bad step count or rate");
    if (nsteps == 0) return PWA_OK;
    Guard g(m->device);
    const MlpBuffers &b = m->m;
    const pwa_mlp::Key key{X, t, n, perm, batch, lr, loss_hist};
    if (!m->exec || !(m->key == key)) {
        drop_graph(m);
        hipError_t e = capture_steps(m, X, t, n, perm, batch, lr, loss_hist, 1, &m->graph, &m->exec);
        if (e == hipSuccess)
            e = capture_steps(m, X, t, n, perm, batch, lr, loss_hist, kGroupSteps, &m->graph_n, &m->exec_n);
        if (e != hipSuccess) {
            drop_graph(m);
            return lfail(m, PWA_E_HIP, "training graph: %s", hipGetErrorString(e));
        }
        m->key = key;
    }
    L_HIP(m, mlp_set_int(b.batch, 0, m->stream), "reset launch");
    L_HIP(m, mlp_set_int(b.bad, 0, m->stream), "reset launch");
    if (mlp_fused_ok(b)) L_HIP(m, mlp_fused_weights(b, m->stream), "weights launch");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (avg_ms) {
        L_HIP(m, hipEventCreate(&e0), "hipEventCreate");
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return lfail(m, PWA_E_HIP, "hipEventCreate failed");
        }
    }
    hipError_t e = avg_ms ? hipEventRecord(e0, m->stream) : hipSuccess;
    int32_t s = 0;
    for (; s + kGroupSteps <= nsteps && e == hipSuccess; s += kGroupSteps) e = hipGraphLaunch(m->exec_n, m->stream);
    for (; s < nsteps && e == hipSuccess; ++s) e = hipGraphLaunch(m->exec, m->stream);
    if (e == hipSuccess && avg_ms) e = hipEventRecord(e1, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e == hipSuccess && avg_ms) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, e0, e1);
        *avg_ms = ms / nsteps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return lfail(m, PWA_E_HIP, "training: %s", hipGetErrorString(e));
    int bad = 0;
    L_HIP(m, hipMemcpy(&bad, b.bad, sizeof(int), hipMemcpyDeviceToHost), "hipMemcpy(flag)");
    if (bad) return lfail(m, PWA_E_INVAL, "a permutation entry is outside [0, n): row 0 was used in its place");
    return PWA_OK;
}

pwa_status pwa_mlp_select(pwa_mlp *m, const float *keys, int64_t n, int32_t k, int32_t *idx) {
    if (!m || !keys || !idx) return lfail(m, PWA_E_INVAL, "null argument");
    if (k < 1 || k > topk_chunk() / 2 || n < k || n > INT32_MAX)
        return lfail(m, PWA_E_INVAL, "need 1 <= k <= %d and k <= n < 2^31", topk_chunk() / 2);
    Guard g(m->device);
    const size_t need = topk_scratch(n, k);
    if (need > m->tk_cap) {
        for (int i = 0; i < 2; ++i) {
            if (m->tk_key[i]) (void)hipFree(m->tk_key[i]);
            if (m->tk_idx[i]) (void)hipFree(m->tk_idx[i]);
            m->tk_key[i] = nullptr;
            m->tk_idx[i] = nullptr;
        }
        m->tk_cap = 0;
        for (int i = 0; i < 2; ++i) {
            L_HIP(m, hipMalloc(&m->tk_key[i], sizeof(float) * need), "hipMalloc(top-k)");
            L_HIP(m, hipMalloc(&m->tk_idx[i], sizeof(int) * need), "hipMalloc(top-k)");
        }
        m->tk_cap = need;
    }
    L_HIP(m, mlp_topk(keys, n, k, m->tk_key, m->tk_idx, idx, m->stream), "top-k launch");
    L_HIP(m, hipStreamSynchronize(m->stream), "hipStreamSynchronize");
    return PWA_OK;
}

const char *pwa_mlp_last_error(const pwa_mlp *m) { return m ? m->err.c_str() : g_lerr.c_str(); }

}  // extern "C"
