// Context-free NLL and gradient that allocates nothing: the streaming kernel of
// pwa_nll_grad_async over caller-owned device samples, with its block
// partials, group sums and arrival counters in a static device array of the
// library instead of a context's workspace.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"

using namespace pwa;

namespace {

// Scratch: arrival counters first, then block partials and group sums (FP64).
constexpr size_t kScratchBytes = PWA_NOALLOC_SCRATCH_BYTES;
constexpr size_t kCounterWords = 256;                          // 1 + groups, at most 255 groups
constexpr size_t kCounterBytes = kCounterWords * sizeof(unsigned);
constexpr size_t kScratchDoubles = (kScratchBytes - kCounterBytes) / sizeof(double);

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DeviceScratch {
    void *ptr = nullptr;     // device address of this device's copy of `scratch`
    int cu_count = 0;
};
DeviceScratch g_dev[kMaxDevices];
std::mutex g_mu;
// Errors are reported through pwa_last_error(NULL).
pwa_status fail(pwa_status st, const char *msg) {
    set_global_error(msg);
    return st;
}

pwa_status fail_hip(hipError_t e, const char *what) {
    set_global_error((std::string(what) + ": " + hipGetErrorString(e)).c_str());
    return PWA_E_HIP;
}

// Per-device set-up on the first call on a device (that device current): the
// address of the device's copy of the scratch array, and its compute units.
pwa_status device_scratch(int dev, DeviceScratch *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    DeviceScratch &d = g_dev[dev];
    if (!d.ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        int cu = 0;
        e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute");
        d.cu_count = cu;
        d.ptr = p;
    }
    *out = d;
    return PWA_OK;
}

bool aligned16(const void *p) { return reinterpret_cast<uintptr_t>(p) % 16 == 0; }

}  // namespace

extern "C" {

pwa_status pwa_nll_grad_noalloc(pwa_prec prec, const void *A_data, int64_t n_data, const void *A_mc,
                                int64_t n_mc, const void *w_mc, double n_gen, int32_t k, int64_t ld,
                                int extended, const double *V_dev, double *out_dev, void *stream) {
    if (prec != PWA_F32 && prec != PWA_F64) return fail(PWA_E_INVAL, "bad precision");
    if (k < 1) return fail(PWA_E_INVAL, "k must be >= 1");
    if (k > PWA_MAX_K) return fail(PWA_E_UNSUPPORTED, "k exceeds PWA_MAX_K");
    if (ld != stream_layout_ld(prec, k)) return fail(PWA_E_INVAL, "ld must be the device layout width pwa_layout_ld(k)");
    if (n_data < 0 || n_mc < 0) return fail(PWA_E_INVAL, "negative sample size");
    if (extended != 0 && extended != 1) return fail(PWA_E_INVAL, "extended must be 0 or 1");
    if (!V_dev || !out_dev) return fail(PWA_E_INVAL, "null V_dev or out_dev");
    if ((n_data > 0 && (!A_data || !aligned16(A_data))) || (n_mc > 0 && (!A_mc || !aligned16(A_mc))))
        return fail(PWA_E_INVAL, "A_data and A_mc must be 16-byte aligned device arrays");
    if (w_mc && reinterpret_cast<uintptr_t>(w_mc) % (prec == PWA_F32 ? 4 : 8) != 0)
        return fail(PWA_E_INVAL, "w_mc must be aligned to its element size");
    const bool need_mc = extended || n_data > 0;
    if (n_data > 0 && n_mc == 0) return fail(PWA_E_INVAL, "MC sample is empty: no normalisation");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(PWA_E_UNSUPPORTED, "device ordinal too large");
    DeviceScratch ds;
    pwa_status st = device_scratch(dev, &ds);
    if (st != PWA_OK) return st;

    StreamCfg cfg;
    const int64_t nm_used = need_mc ? n_mc : 0;
    if (!stream_tuned_cfg(dev, prec, ld, n_data, nm_used, &cfg)) cfg = stream_default_cfg(prec, (int)ld);
    const int ps = (int)(1 + 2 * ld);
    // blocks the scratch holds: partials and group sums of every block, one
    // counter per group
    int64_t cap = (int64_t)ds.cu_count * cfg.blocks_per_cu;
    while (cap > 1 && (stream_scratch_doubles((int)cap, ps) > kScratchDoubles ||
                       stream_counter_words((int)cap) > kCounterWords))
        --cap;

    StreamArgs a;
    std::memset(&a, 0, sizeof a);
    a.A[0] = A_data;
    a.A[1] = A_mc;
    a.w = w_mc;
    a.n[0] = n_data;
    a.n[1] = nm_used;
    a.ld = ld;
    a.k = k;
    a.pstride = ps;
    a.v_dev = V_dev;
    a.counters = static_cast<unsigned *>(ds.ptr);
    a.partials = reinterpret_cast<double *>(static_cast<unsigned char *>(ds.ptr) + kCounterBytes);
    a.n_gen = n_gen > 0 ? n_gen : (n_mc > 0 ? (double)n_mc : 1.0);
    a.nd_total = (double)n_data;
    a.extended = extended;
    a.out = out_dev;
    stream_grid(cfg, cap, a.n[0], a.n[1], a.nb);
    int blocks = a.nb[0] + a.nb[1];
    if (blocks == 0) {
        a.nb[0] = 1;     // one block still writes the (trivial) result
        blocks = 1;
    }
    a.gsums = a.partials + (size_t)blocks * ps;
    e = launch_stream(prec, cfg, blocks, a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e, "likelihood kernel launch");
    return PWA_OK;
}

}  // extern "C"
