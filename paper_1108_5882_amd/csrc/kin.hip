// NLL and gradients with the decay amplitudes formed on the device from each
// event's kinematics, so that resonance masses and widths can be fit
// parameters (Berger, Section 2: amplitudes can be precomputed only while the
// masses and widths of the resonances are kept constant).
//
// Per event the kernel reads 8 bytes, (m, cos theta) in FP32, and forms for
// every wave a
//     A_a = BW_a(m) Y_{J_a}^0(x),  BW_a = 1 / (m_a^2 - m^2 - i m_a Gamma_a),
//     Y_J^0 = sqrt((2J + 1) / (4 pi)) P_J(x),
// then z = sum_a V_a A_a and I = |z|^2 (Eq. 1) and, for data (c = 1/I) or MC
// (c = w) events, the sums of ln I or w I, of c conj(A_a) z (the V gradient)
// and of c dI/dt for t = m_a, Gamma_a, with
//     dI/dt = 2 Re(conj(z) V_a Y_a dBW_a/dt),
//     dBW_a/dm_a = -(2 m_a - i Gamma_a) BW_a^2,   dBW_a/dGamma_a = i m_a BW_a^2.
// The reads are tiny and the work is tens of FP64 operations per (event,
// wave): the kernel is bound by vector arithmetic, not by HBM.  All of it is
// FP64 (on gfx950 a non-packed FP32 operation issues at the FP64 rate, so
// single precision would not be faster here, only less exact).
//
// Mapping: L lanes share an event, lane j holding waves [4j, 4j + 4); the
// partial coherent sums meet through DPP row operations, as in the streaming
// kernel.  Each block ends with its FP64 partial, and the launch combines the
// partials in a fixed order (block_reduce.hpp) and forms
//     NLL    = -sum ln I + N_D ln S   (Eq. 2)   or   -sum ln I + S   (Eq. 3)
//     dNLL/dV   = 2 (-G + c H)          (Re, Im interleaved)
//     dNLL/dt   = -R_data + c R_MC      (d/dm_a, d/dGamma_a interleaved)
// with c = N_D / (N_gen S) or 1 / N_gen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>

#include "block_reduce.hpp"
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kKinThreads = 256;
constexpr int kKinW = 4;            // waves per lane
constexpr int kKinMaxSpin = 4;
constexpr int kKinBlocksPerCu = 4;

struct KinArgs {
    const float2 *mx[2];            // (m, cos theta) per event: data, MC
    const float *w;                 // MC weights or nullptr
    int64_t n[2];
    int32_t nb[2];
    int32_t k;
    int32_t extended;
    double n_gen;
    double nd_total;
    const double *v_dev;            // V (2k) on the device, or nullptr: v_arg
    const double *res_dev;          // (m_a, Gamma_a) on the device, or nullptr: res_arg
    double *partials;
    double *gsums;
    unsigned *counters;
    double *out;                    // [nll, dV[2k], dres[2k], flags]
    unsigned long long *done;       // or nullptr (host-mapped sequence word)
    unsigned long long seq;
    int32_t spin[PWA_MAX_K];
    double v_arg[2 * PWA_MAX_K];
    double res_arg[2 * PWA_MAX_K];
};

template <int CTRL>
__device__ __forceinline__ int kdpp_i(int x) {
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double kdpp_d(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    v.x = kdpp_i<CTRL>(v.x);
    v.y = kdpp_i<CTRL>(v.y);
    return *reinterpret_cast<double *>(&v);
}

// sum over the L lanes of an event (every lane ends with the same bits)
template <int L>
__device__ __forceinline__ double lane_group_sum(double x) {
    if constexpr (L >= 2) x += kdpp_d<0xB1>(x);    // quad_perm [1,0,3,2]
    if constexpr (L >= 4) x += kdpp_d<0x4E>(x);    // quad_perm [2,3,0,1]
    if constexpr (L >= 8) x += kdpp_d<0x141>(x);   // row_half_mirror
    if constexpr (L >= 16) x += kdpp_d<0x140>(x);  // row_mirror
    return x;
}

// 1 / d for d > 0: hardware estimate refined by one Newton step
__device__ __forceinline__ double recip(double d) {
    const double r = __builtin_amdgcn_rcp(d);
    return fma(r, fma(-d, r, 1.0), r);
}

template <int L>
__global__ __launch_bounds__(kKinThreads) void kin_kernel(KinArgs p) {
    constexpr int NW = kKinThreads / 64;
    constexpr int G = 64 / L;               // events per wave per step
    constexpr int WAVES = L * kKinW;        // padded waves
    constexpr int PS = 1 + 4 * WAVES;       // [log or w I sum][dV 2 per wave][dres 2 per wave]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int j = lane % L, g = lane / L;

    // per-lane wave constants (padded waves: V = 0 and a harmless lineshape):
    // V, m_a^2, m_a Gamma_a and its square, and Y_J^0 as a polynomial in
    // x = cos theta, yc[q][i] the coefficient of x^i (the normalisation folded
    // in), so that every wave evaluates it with the same four FMAs whatever its
    // spin (a per-wave choice among the Legendre polynomials would branch on
    // the lane's spin)
    double vr[kKinW], vi[kKinW], ma[kKinW], ga[kKinW], ma2[kKinW], mg[kKinW], mg2[kKinW];
    double yc[kKinW][5];
#pragma unroll
    for (int q = 0; q < kKinW; ++q) {
        const int a = j * kKinW + q;
        const bool live = a < p.k;
        const double *V = p.v_dev ? p.v_dev : p.v_arg;
        const double *R = p.res_dev ? p.res_dev : p.res_arg;
        vr[q] = live ? V[2 * a] : 0.0;
        vi[q] = live ? V[2 * a + 1] : 0.0;
        ma[q] = live ? R[2 * a] : 1.0;
        ga[q] = live ? R[2 * a + 1] : 1.0;
        ma2[q] = ma[q] * ma[q];
        mg[q] = ma[q] * ga[q];
        mg2[q] = mg[q] * mg[q];
        const int J = live ? p.spin[a] : 0;
        const double yn = live ? sqrt((2.0 * J + 1.0) * 0.079577471545947667884) : 0.0;   // 1 / (4 pi)
        // P_0 = 1, P_1 = x, P_2 = (3x^2 - 1)/2, P_3 = (5x^3 - 3x)/2, P_4 = (35x^4 - 30x^2 + 3)/8
        yc[q][0] = yn * (J == 0 ? 1.0 : J == 2 ? -0.5 : J == 4 ? 0.375 : 0.0);
        yc[q][1] = yn * (J == 1 ? 1.0 : J == 3 ? -1.5 : 0.0);
        yc[q][2] = yn * (J == 2 ? 1.5 : J == 4 ? -3.75 : 0.0);
        yc[q][3] = yn * (J == 3 ? 2.5 : 0.0);
        yc[q][4] = yn * (J == 4 ? 4.375 : 0.0);
    }

    const int seg = (int)blockIdx.x < p.nb[0] ? 0 : 1;
    const int bseg = seg ? (int)blockIdx.x - p.nb[0] : (int)blockIdx.x;
    const int64_t n = p.n[seg];
    const float2 *mx = p.mx[seg];
    const float *W = seg ? p.w : nullptr;
    const int64_t ntiles = (n + G - 1) / G;
    const int64_t stride = (int64_t)p.nb[seg] * NW;

    // data: sum ln I as sum ln(product of frexp mantissas) + ln 2 * sum of exponents
    // (one logarithm per 32 events instead of one per event); MC: sum w I
    double acc_t = 0.0, pm = 1.0;
    int pe = 0, cnt = 0;
    // gvr, gvi: per wave the sums of g = conj(A_a) u (u = c z); gm, gg: the sums
    // of BW_a conj(g).  The mass and width terms need e = (V_a BW_a) conj(g):
    // V_a and the constant factors of dI/dm_a and dI/dGamma_a are applied to
    // the sums once after the loop
    double gvr[kKinW], gvi[kKinW], gm[kKinW], gg[kKinW];
#pragma unroll
    for (int q = 0; q < kKinW; ++q) gvr[q] = gvi[q] = gm[q] = gg[q] = 0.0;

    // each step's (m, cos theta) and weight are loaded one step ahead (row
    // index clamped into the sample: always a valid address); the weight load
    // reads the events themselves when there are no weights, so the loop holds
    // no branch on it
    const bool has_w = seg && W;
    const float *Wl = has_w ? W : reinterpret_cast<const float *>(mx);
    int64_t t = (int64_t)bseg * NW + wid;
    float2 kin_n = {0.f, 0.f};
    float w_n = 1.f;
    if (t < ntiles) {
        const int64_t e0 = min(t * G + g, n - 1);
        kin_n = mx[e0];
        w_n = Wl[e0];
    }
    // Tiles below n / G hold no event past the sample: their steps need no
    // per-event check, and only the last, partial tile (one wave's step at
    // most) takes it.
    const int64_t nfull = n / G;
    auto event_step = [&](auto check) {
        const bool valid = !decltype(check)::value || t * G + g < n;
        const float2 kin = kin_n;
        const float wf = has_w ? w_n : 1.0f;
        {
            const int64_t en = min((t + stride) * G + g, n - 1);
            kin_n = mx[en];
            w_n = Wl[en];
        }
        const double x = kin.y;
        // m^2 of an FP32 mass is exact in FP64 (24-bit mantissa squared)
        const double m2 = (double)kin.x * (double)kin.x;
        double bre[kKinW], bim[kKinW], ar[kKinW], ai[kKinW];
        double zr = 0.0, zi = 0.0;
#pragma unroll
        for (int q = 0; q < kKinW; ++q) {
            // BW = 1 / (dre - i mg) = (dre + i mg) / (dre^2 + mg^2), dre = m_a^2 - m^2
            const double dre = ma2[q] - m2;
            const double r = recip(fma(dre, dre, mg2[q]));
            bre[q] = dre * r;
            bim[q] = mg[q] * r;
            const double y = fma(fma(fma(fma(yc[q][4], x, yc[q][3]), x, yc[q][2]), x, yc[q][1]), x, yc[q][0]);
            // A_a = BW_a Y_a, then its share of z = sum_a V_a A_a
            ar[q] = bre[q] * y;
            ai[q] = bim[q] * y;
            zr = fma(vr[q], ar[q], zr);
            zr = fma(-vi[q], ai[q], zr);
            zi = fma(vr[q], ai[q], zi);
            zi = fma(vi[q], ar[q], zi);
        }
        zr = lane_group_sum<L>(zr);
        zi = lane_group_sum<L>(zi);
        const double I = fma(zr, zr, zi * zi);
        double ce;
        if (seg == 0) {
            int ex = 0;
            pm *= valid ? frexp(I, &ex) : 1.0;
            pe += ex;
            if (++cnt == 32) {      // the same count in every lane: no divergence
                acc_t += log(pm);
                pm = 1.0;
                cnt = 0;
            }
            ce = valid ? recip(I) : 0.0;
        } else {
            ce = valid ? (double)wf : 0.0;
            acc_t = fma(ce, I, acc_t);
        }
        const double ur = ce * zr, ui = ce * zi;
#pragma unroll
        for (int q = 0; q < kKinW; ++q) {
            // g = conj(A_a) u  (the V-gradient term)
            const double gr_ = fma(ar[q], ur, ai[q] * ui);
            const double gi_ = fma(ar[q], ui, -ai[q] * ur);
            gvr[q] += gr_;
            gvi[q] += gi_;
            // BW_a conj(g) = conj(u) Y_a BW_a^2; times V_a after the loop it is e
            gm[q] = fma(bre[q], gr_, gm[q]);
            gm[q] = fma(bim[q], gi_, gm[q]);
            gg[q] = fma(bim[q], gr_, gg[q]);
            gg[q] = fma(-bre[q], gi_, gg[q]);
        }
    };
    for (; t < nfull; t += stride) event_step(std::false_type{});
    for (; t < ntiles; t += stride) event_step(std::true_type{});
    if (seg == 0) acc_t += log(pm) + (double)pe * 0.69314718055994530942;

    // lanes with the same j across the wave's event groups
#pragma unroll
    for (int off = L; off < 64; off <<= 1) {
        acc_t += __shfl_xor(acc_t, off);
#pragma unroll
        for (int q = 0; q < kKinW; ++q) {
            gvr[q] += __shfl_xor(gvr[q], off);
            gvi[q] += __shfl_xor(gvi[q], off);
            gm[q] += __shfl_xor(gm[q], off);
            gg[q] += __shfl_xor(gg[q], off);
        }
    }
    // e = V_a (sum of BW_a conj(g)); then
    // 2 Re(e (-(2 m_a - i Gamma_a))) = -4 m_a Re e - 2 Gamma_a Im e;  2 Re(e (i m_a)) = -2 m_a Im e
#pragma unroll
    for (int q = 0; q < kKinW; ++q) {
        const double sr = fma(vr[q], gm[q], -vi[q] * gg[q]);
        const double si = fma(vr[q], gg[q], vi[q] * gm[q]);
        gm[q] = fma(-4.0 * ma[q], sr, -2.0 * ga[q] * si);
        gg[q] = -2.0 * ma[q] * si;
    }
    __shared__ double red[NW][L][1 + 4 * kKinW];
    if (lane < L) {
        red[wid][j][0] = acc_t;
#pragma unroll
        for (int q = 0; q < kKinW; ++q) {
            red[wid][j][1 + 4 * q] = gvr[q];
            red[wid][j][2 + 4 * q] = gvi[q];
            red[wid][j][3 + 4 * q] = gm[q];
            red[wid][j][4 + 4 * q] = gg[q];
        }
    }
    __syncthreads();
    // block partial: [0] the sum, [1 + 2a + r] dV of wave a, [1 + 2 WAVES + 2a + r] dres
    for (int idx = tid; idx < PS; idx += kKinThreads) {
        int jj = 0, slot = 0;
        if (idx > 0) {
            const int c = idx - 1;
            const bool res_part = c >= 2 * WAVES;
            const int a = (res_part ? c - 2 * WAVES : c) >> 1, r = c & 1;
            jj = a / kKinW;
            slot = 1 + 4 * (a % kKinW) + (res_part ? 2 : 0) + r;
        }
        double s = 0.0;
        for (int ww = 0; ww < NW; ++ww) s += red[ww][jj][slot];
        st_dev(p.partials + (int64_t)blockIdx.x * PS + idx, s);
    }

    __shared__ double tot[2 * PS];
    __shared__ double s_c;
    if (!reduce_blocks<PS, kKinThreads>(ReduceBufs{p.partials, p.gsums, p.counters, p.nb[0], p.nb[0] + p.nb[1]},
                                        tot))
        return;
    const int k = p.k;
    const double *td = tot;          // data: [0] sum ln I, [1 + i] G, [1 + 2 WAVES + i] R_data
    const double *tm = tot + PS;     // MC:   [0] sum w I, [1 + i] H, [1 + 2 WAVES + i] R_MC
    const bool empty = !p.extended && p.nd_total == 0.0;
    if (tid == 0) {
        const double nd = p.nd_total;
        const double S = tm[0] / p.n_gen;
        double c = p.extended ? 1.0 / p.n_gen : nd / tm[0];
        double nll;
        unsigned flags = 0;
        if (empty) {
            nll = 0.0;
            c = 0.0;
        } else {
            nll = p.extended ? -td[0] + S : -td[0] + nd * log(S);
            if (!isfinite(nll) || (!p.extended && !(S > 0.0))) {
                nll = INFINITY;
                flags = 1;
            }
        }
        st_sys(p.out, nll);
        st_sys(p.out + 1 + 4 * k, (double)flags);
        s_c = c;
    }
    __syncthreads();
    const double c = s_c;
    for (int i = tid; i < 2 * k; i += kKinThreads) {
        st_sys(p.out + 1 + i, empty ? 0.0 : 2.0 * (-td[1 + i] + c * tm[1 + i]));
        st_sys(p.out + 1 + 2 * k + i, empty ? 0.0 : -td[1 + 2 * WAVES + i] + c * tm[1 + 2 * WAVES + i]);
    }
    if (p.done) {
        wait_stores();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(p.done, p.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// lanes per event for k waves (4 waves per lane)
int kin_lanes(int k) {
    int L = 1;
    while (L * kKinW < k) L <<= 1;
    return L;
}

int kin_pstride(int k) { return 1 + 4 * kin_lanes(k) * kKinW; }

hipError_t launch_kin(const KinArgs &a, int blocks, hipStream_t s) {
    switch (kin_lanes(a.k)) {
        case 1: hipLaunchKernelGGL(kin_kernel<1>, dim3(blocks), dim3(kKinThreads), 0, s, a); break;
        case 2: hipLaunchKernelGGL(kin_kernel<2>, dim3(blocks), dim3(kKinThreads), 0, s, a); break;
        case 4: hipLaunchKernelGGL(kin_kernel<4>, dim3(blocks), dim3(kKinThreads), 0, s, a); break;
        case 8: hipLaunchKernelGGL(kin_kernel<8>, dim3(blocks), dim3(kKinThreads), 0, s, a); break;
        case 16: hipLaunchKernelGGL(kin_kernel<16>, dim3(blocks), dim3(kKinThreads), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace pwa

using namespace pwa;

struct pwa_kin {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cu_count = 0;
    int32_t k = 0;
    int32_t spin[PWA_MAX_K] = {};
    int extended = 0;
    struct Events {
        float2 *mx = nullptr;
        float *w = nullptr;
        bool owned = true;
        int64_t n = 0;
        double n_gen = 0.0;
        bool set = false;
    } ev[2];
    int max_blocks = 0;
    double *partials = nullptr;
    double *gsums = nullptr;
    unsigned *counters = nullptr;
    double *out_host = nullptr, *out_host_dev = nullptr;
    unsigned long long *done_host = nullptr, *done_dev = nullptr;
    unsigned long long seq = 0;
    std::string err;
};

namespace {

thread_local std::string g_kin_err;

pwa_status kfail(pwa_kin *kc, pwa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (kc ? kc->err : g_kin_err) = buf;
    return st;
}

pwa_status kfail_hip(pwa_kin *kc, hipError_t e, const char *what) {
    return kfail(kc, e == hipErrorOutOfMemory ? PWA_E_NOMEM : PWA_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

struct KinDeviceGuard {
    int prev = -1;
    explicit KinDeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~KinDeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void free_events(pwa_kin::Events &e) {
    if (e.owned && e.mx) (void)hipFree(e.mx);
    if (e.owned && e.w) (void)hipFree(e.w);
    e = pwa_kin::Events{};
}

bool is_device_ptr(const void *p, int device) {
    hipPointerAttribute_t at;
    std::memset(&at, 0, sizeof at);
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.isManaged || (at.type == hipMemoryTypeDevice && at.device == device);
}

// Arguments of one evaluation; *blocks = 0 when nothing needs a launch.
pwa_status kin_prepare(pwa_kin *kc, KinArgs &a, int *blocks) {
    if (!kc->ev[0].set) return kfail(kc, PWA_E_STATE, "data events not set");
    const int64_t nd = kc->ev[0].n;
    const bool need_mc = kc->extended || nd > 0;
    if (need_mc && !kc->ev[1].set) return kfail(kc, PWA_E_STATE, "MC events not set");
    if (need_mc && kc->ev[1].n == 0 && nd > 0) return kfail(kc, PWA_E_STATE, "MC sample is empty: no normalisation");
    std::memset(&a, 0, sizeof a);
    a.mx[0] = kc->ev[0].mx;
    a.mx[1] = kc->ev[1].mx;
    a.w = kc->ev[1].w;
    a.n[0] = nd;
    a.n[1] = need_mc ? kc->ev[1].n : 0;
    a.k = kc->k;
    a.extended = kc->extended;
    a.n_gen = kc->ev[1].n_gen > 0 ? kc->ev[1].n_gen : 1.0;
    a.nd_total = (double)nd;
    a.partials = kc->partials;
    a.gsums = kc->gsums;
    a.counters = kc->counters;
    std::memcpy(a.spin, kc->spin, sizeof a.spin);
    // blocks in proportion to events (the per-event work is the same in both samples)
    const int L = kin_lanes(kc->k);
    const int64_t per_block = (int64_t)(64 / L) * (kKinThreads / 64);
    const int64_t need0 = (a.n[0] + per_block - 1) / per_block, need1 = (a.n[1] + per_block - 1) / per_block;
    const int64_t budget = kc->max_blocks;
    if (need0 + need1 <= budget) {
        a.nb[0] = (int32_t)need0;
        a.nb[1] = (int32_t)need1;
    } else {
        int64_t b0 = (int64_t)std::llround((double)a.n[0] / (double)(a.n[0] + a.n[1]) * (double)budget);
        if (a.n[0] > 0) b0 = std::max<int64_t>(b0, 1);
        if (a.n[1] > 0) b0 = std::min<int64_t>(b0, budget - 1);
        b0 = std::min(b0, need0);
        a.nb[0] = (int32_t)b0;
        a.nb[1] = (int32_t)std::min(budget - b0, need1);
    }
    *blocks = a.nb[0] + a.nb[1];
    if (*blocks == 0) {
        a.nb[0] = 1;   // one block still writes the (trivial) result
        *blocks = 1;
    }
    return PWA_OK;
}

}  // namespace

extern "C" {

pwa_status pwa_kin_create(pwa_kin **out, int device, int32_t k, const int32_t *spin, void *stream) {
    if (!out) return kfail(nullptr, PWA_E_INVAL, "null output pointer");
    if (k < 1 || !spin) return kfail(nullptr, PWA_E_INVAL, "k must be >= 1 and spins given");
    if (k > PWA_MAX_K) return kfail(nullptr, PWA_E_UNSUPPORTED, "k = %d exceeds %d", k, PWA_MAX_K);
    for (int a = 0; a < k; ++a)
        if (spin[a] < 0 || spin[a] > kKinMaxSpin)
            return kfail(nullptr, PWA_E_UNSUPPORTED, "spin %d of wave %d: 0..%d supported", spin[a], a, kKinMaxSpin);
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return kfail(nullptr, PWA_E_INVAL, "device %d not available", device);
    KinDeviceGuard dg(device);
    pwa_kin *kc = new (std::nothrow) pwa_kin();
    if (!kc) return kfail(nullptr, PWA_E_NOMEM, "out of host memory");
    kc->device = device;
    kc->k = k;
    std::memcpy(kc->spin, spin, sizeof(int32_t) * k);
    hipError_t e = hipDeviceGetAttribute(&kc->cu_count, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess && !stream) {
        e = hipStreamCreateWithFlags(&kc->stream, hipStreamNonBlocking);
        kc->own_stream = e == hipSuccess;
    } else if (stream) {
        kc->stream = static_cast<hipStream_t>(stream);
    }
    kc->max_blocks = kc->cu_count * kKinBlocksPerCu;
    const int ps = kin_pstride(k);
    const size_t cw = stream_counter_words(kc->max_blocks);
    const size_t out_doubles = 4 * (size_t)k + 2;
    if (e == hipSuccess) e = hipMalloc(&kc->partials, sizeof(double) * stream_scratch_doubles(kc->max_blocks, ps));
    if (e == hipSuccess) e = hipMalloc(&kc->counters, sizeof(unsigned) * cw);
    if (e == hipSuccess) e = hipMemsetAsync(kc->counters, 0, sizeof(unsigned) * cw, kc->stream);
    if (e == hipSuccess)
        e = hipHostMalloc(&kc->out_host, sizeof(double) * (out_doubles + 1), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&kc->out_host_dev, kc->out_host, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(kc->stream);
    if (e != hipSuccess) {
        pwa_status st = kfail_hip(nullptr, e, "kinematic context allocation");
        pwa_kin_destroy(kc);
        return st;
    }
    kc->gsums = kc->partials + (size_t)kc->max_blocks * ps;
    kc->done_host = reinterpret_cast<unsigned long long *>(kc->out_host + out_doubles);
    kc->done_dev = reinterpret_cast<unsigned long long *>(kc->out_host_dev + out_doubles);
    *kc->done_host = 0;
    *out = kc;
    return PWA_OK;
}

pwa_status pwa_kin_destroy(pwa_kin *kc) {
    if (!kc) return PWA_OK;
    KinDeviceGuard dg(kc->device);
    if (kc->stream) (void)hipStreamSynchronize(kc->stream);
    for (auto &e : kc->ev) free_events(e);
    if (kc->partials) (void)hipFree(kc->partials);
    if (kc->counters) (void)hipFree(kc->counters);
    if (kc->out_host) (void)hipHostFree(kc->out_host);
    if (kc->own_stream && kc->stream) (void)hipStreamDestroy(kc->stream);
    delete kc;
    return PWA_OK;
}

pwa_status pwa_kin_set_events(pwa_kin *kc, pwa_set which, const float *mx, int64_t n, pwa_where where,
                              const float *w, double n_gen) {
    if (!kc) return kfail(nullptr, PWA_E_INVAL, "null context");
    if (which != PWA_DATA && which != PWA_MC) return kfail(kc, PWA_E_INVAL, "bad sample id");
    if (where != PWA_HOST && where != PWA_DEVICE && where != PWA_BORROW)
        return kfail(kc, PWA_E_INVAL, "bad memory space");
    if (n < 0 || (n > 0 && !mx)) return kfail(kc, PWA_E_INVAL, "bad events");
    if (which == PWA_DATA && w) return kfail(kc, PWA_E_INVAL, "weights apply to the MC sample only");
    KinDeviceGuard dg(kc->device);
    if (where != PWA_HOST && n > 0) {
        if (!is_device_ptr(mx, kc->device) || (w && !is_device_ptr(w, kc->device)))
            return kfail(kc, PWA_E_INVAL, "events are not device memory of the context's device");
        if (reinterpret_cast<uintptr_t>(mx) % 8 != 0 || reinterpret_cast<uintptr_t>(w) % 4 != 0)
            return kfail(kc, PWA_E_INVAL, "misaligned events or weights");
    }
    pwa_kin::Events &ev = kc->ev[which];
    free_events(ev);
    if (where == PWA_BORROW) {
        ev.mx = n > 0 ? reinterpret_cast<float2 *>(const_cast<float *>(mx)) : nullptr;
        ev.w = n > 0 ? const_cast<float *>(w) : nullptr;
        ev.owned = false;
    } else if (n > 0) {
        const hipMemcpyKind kind = where == PWA_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
        hipError_t e = hipMalloc(&ev.mx, sizeof(float2) * (size_t)n);
        if (e == hipSuccess) e = hipMemcpyAsync(ev.mx, mx, sizeof(float2) * (size_t)n, kind, kc->stream);
        if (e == hipSuccess && w) e = hipMalloc(&ev.w, sizeof(float) * (size_t)n);
        if (e == hipSuccess && w) e = hipMemcpyAsync(ev.w, w, sizeof(float) * (size_t)n, kind, kc->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(kc->stream);
        if (e != hipSuccess) {
            free_events(ev);
            return kfail_hip(kc, e, "staging events");
        }
    }
    ev.n = n;
    ev.n_gen = which == PWA_MC ? (n_gen > 0 ? n_gen : (double)n) : 0.0;
    ev.set = true;
    return PWA_OK;
}

pwa_status pwa_kin_set_mode(pwa_kin *kc, int extended) {
    if (!kc) return kfail(nullptr, PWA_E_INVAL, "null context");
    if (extended != 0 && extended != 1) return kfail(kc, PWA_E_INVAL, "extended must be 0 or 1");
    kc->extended = extended;
    return PWA_OK;
}

pwa_status pwa_kin_nll_grad(pwa_kin *kc, const double *V, const double *res, double *nll, double *grad_v,
                            double *grad_res) {
    if (!kc) return kfail(nullptr, PWA_E_INVAL, "null context");
    if (!V || !res || !nll) return kfail(kc, PWA_E_INVAL, "null V, res or nll");
    const int k = kc->k;
    for (int i = 0; i < 2 * k; ++i) {
        if (!std::isfinite(V[i])) return kfail(kc, PWA_E_INVAL, "V[%d] is not finite", i);
        if (!std::isfinite(res[i]) || !(res[i] > 0.0))
            return kfail(kc, PWA_E_INVAL, "masses and widths must be finite and positive (res[%d])", i);
    }
    KinDeviceGuard dg(kc->device);
    KinArgs a;
    int blocks = 0;
    pwa_status st = kin_prepare(kc, a, &blocks);
    if (st != PWA_OK) return st;
    std::memcpy(a.v_arg, V, sizeof(double) * 2 * k);
    std::memcpy(a.res_arg, res, sizeof(double) * 2 * k);
    a.out = kc->out_host_dev;
    a.done = kc->done_dev;
    a.seq = ++kc->seq;
    hipError_t e = launch_kin(a, blocks, kc->stream);
    if (e != hipSuccess) return kfail_hip(kc, e, "kinematic kernel launch");
    // the kernel writes the result to mapped host memory, then the sequence number
    const volatile unsigned long long *done = kc->done_host;
    for (unsigned spin = 1; *done != a.seq; ++spin) {
        if ((spin & 4095u) == 0) {
            const hipError_t q = hipStreamQuery(kc->stream);
            if (q == hipSuccess) {
                if (*done == a.seq) break;
                return kfail(kc, PWA_E_HIP, "kinematic kernel finished without writing its result");
            }
            if (q != hipErrorNotReady) return kfail_hip(kc, q, "kinematic kernel");
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    const double *r = kc->out_host;
    *nll = r[0];
    if (grad_v) std::memcpy(grad_v, r + 1, sizeof(double) * 2 * k);
    if (grad_res) std::memcpy(grad_res, r + 1 + 2 * k, sizeof(double) * 2 * k);
    if (r[1 + 4 * k] != 0.0) return kfail(kc, PWA_E_DOMAIN, "non-positive intensity or normalisation");
    return PWA_OK;
}

pwa_status pwa_kin_nll_grad_async(pwa_kin *kc, const double *V_dev, const double *res_dev, double *out_dev) {
    if (!kc) return kfail(nullptr, PWA_E_INVAL, "null context");
    if (!V_dev || !res_dev || !out_dev) return kfail(kc, PWA_E_INVAL, "null device pointer");
    KinDeviceGuard dg(kc->device);
    if (!is_device_ptr(V_dev, kc->device) || !is_device_ptr(res_dev, kc->device) ||
        !is_device_ptr(out_dev, kc->device))
        return kfail(kc, PWA_E_INVAL, "V_dev, res_dev and out_dev must be device memory of the context's device");
    KinArgs a;
    int blocks = 0;
    pwa_status st = kin_prepare(kc, a, &blocks);
    if (st != PWA_OK) return st;
    a.v_dev = V_dev;
    a.res_dev = res_dev;
    a.out = out_dev;
    hipError_t e = launch_kin(a, blocks, kc->stream);
    if (e != hipSuccess) return kfail_hip(kc, e, "kinematic kernel launch");
    return PWA_OK;
}

const char *pwa_kin_last_error(const pwa_kin *kc) { return kc ? kc->err.c_str() : g_kin_err.c_str(); }

}  // extern "C"
