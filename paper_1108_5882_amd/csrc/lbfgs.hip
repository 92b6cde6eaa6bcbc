// Device L-BFGS for many independent fits (one block per fit), advanced once
// per evaluation so that the whole iteration (evaluate every fit's trial
// point, then update every fit) can be captured in a HIP graph.
//
// Each fit minimises its NLL over the real vector x = (Re V_0, Im V_0, ...)
// (minimisers work on real parameters, Berger Section 4).  State machine per
// fit, entered after its trial point xt was evaluated (f_t, g_t):
//   phase 0 (start):  accept xt, choose a direction.
//   phase 1 (search): Armijo test f_t <= f + c1 alpha g.d.  Accepted: the pair
//     s = xt - x, y = g_t - g enters the history if s.y > 0, the point moves
//     and a new direction is chosen.  Rejected: alpha halves and the trial
//     point moves back along the same direction.
//   direction: d = -H g by the two-loop recursion over the last m pairs with
//     H0 = (s.y / y.y) of the newest pair (Nocedal & Wright, Alg. 7.4); if it
//     is not a descent direction the history is dropped and d = -g.  The first
//     trial step of a fresh history moves x by 1% of |x| (alpha = 0.01 |x| / |d|).
//   stop: status 1 when an accepted step changes f by at most ftol (1 + |f|),
//     status 2 when the step underflows.
// Dot products are summed by one thread in index order: deterministic.
#include "internal.hpp"

namespace pwa {
namespace {

constexpr int kLT = 128;

__device__ double block_dot(const double *a, const double *b, int n, double *scratch) {
    const int tid = threadIdx.x;
    if (tid < n) scratch[tid] = a[tid] * b[tid];
    __syncthreads();
    __shared__ double s_res;
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += scratch[i];
        s_res = s;
    }
    __syncthreads();
    const double r = s_res;
    __syncthreads();
    return r;
}

__device__ double block_maxabs(const double *a, int n, double *scratch) {
    const int tid = threadIdx.x;
    if (tid < n) scratch[tid] = fabs(a[tid]);
    __syncthreads();
    __shared__ double s_res;
    if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s = fmax(s, scratch[i]);
        s_res = s;
    }
    __syncthreads();
    const double r = s_res;
    __syncthreads();
    return r;
}

// d = -H g by the two-loop recursion; returns g.d.  Resets to steepest descent
// when the result is not a descent direction.
__device__ double new_direction(LbfgsState *st, int n, int m, double *q, double *scratch) {
    __shared__ double alpha_i[kLbfgsMaxHist];
    const int tid = threadIdx.x;
    if (tid < n) q[tid] = st->g[tid];
    __syncthreads();
    const int cnt = st->count;
    for (int t = 0; t < cnt; ++t) {                       // newest to oldest
        const int i = (st->head - 1 - t + m) % m;
        const double a = st->rho[i] * block_dot(st->S[i], q, n, scratch);
        if (tid == 0) alpha_i[i] = a;
        if (tid < n) q[tid] -= a * st->Y[i][tid];
        __syncthreads();
    }
    if (cnt > 0) {
        const int i = (st->head - 1 + m) % m;
        const double gamma = block_dot(st->S[i], st->Y[i], n, scratch) /
                             block_dot(st->Y[i], st->Y[i], n, scratch);
        if (tid < n) q[tid] *= gamma;
        __syncthreads();
    }
    for (int t = cnt - 1; t >= 0; --t) {                  // oldest to newest
        const int i = (st->head - 1 - t + m) % m;
        const double b = st->rho[i] * block_dot(st->Y[i], q, n, scratch);
        if (tid < n) q[tid] += st->S[i][tid] * (alpha_i[i] - b);
        __syncthreads();
    }
    if (tid < n) st->d[tid] = -q[tid];
    __syncthreads();
    double gtd = block_dot(st->g, st->d, n, scratch);
    if (!(gtd < 0.0)) {
        if (tid == 0) st->count = 0;
        if (tid < n) st->d[tid] = -st->g[tid];
        __syncthreads();
        gtd = block_dot(st->g, st->d, n, scratch);
    }
    return gtd;
}

__global__ __launch_bounds__(kLT) void lbfgs_kernel(const MultiFit *fits, int k_all,
                                                    const double *out, int64_t ostride,
                                                    LbfgsState *states, int m, double c1,
                                                    double ftol) {
    __shared__ double scratch[kLT];
    __shared__ double q[kLT];
    __shared__ int s_accept;
    const int f = blockIdx.x, tid = threadIdx.x;
    LbfgsState *st = states + f;
    const int n = 2 * (fits ? fits[f].k : k_all);
    if (st->status != 0) return;
    const double *o = out + (int64_t)f * ostride;
    const double ft = o[0];
    const double *gt = o + 1;

    bool new_dir = false;
    if (st->phase == 0) {
        if (tid < n) {
            st->x[tid] = st->xt[tid];
            st->g[tid] = gt[tid];
        }
        if (tid == 0) st->f = ft;
        __syncthreads();
        new_dir = true;
    } else {
        if (tid == 0) s_accept = isfinite(ft) && ft <= st->f + c1 * st->alpha * st->gtd;
        __syncthreads();
        if (s_accept) {
            // history pair s = xt - x, y = g_t - g (written into the slot at head)
            const int h = st->head;
            if (tid < n) {
                st->S[h][tid] = st->xt[tid] - st->x[tid];
                st->Y[h][tid] = gt[tid] - st->g[tid];
            }
            __syncthreads();
            const double sy = block_dot(st->S[h], st->Y[h], n, scratch);
            const double fold = st->f;
            if (tid < n) {
                st->x[tid] = st->xt[tid];
                st->g[tid] = gt[tid];
            }
            if (tid == 0) {
                if (sy > 0.0) {
                    st->rho[h] = 1.0 / sy;
                    st->head = (h + 1) % m;
                    st->count = st->count < m ? st->count + 1 : m;
                }
                st->f = ft;
                st->iter += 1;
                if (fabs(fold - ft) <= ftol * (1.0 + fabs(ft))) st->status = 1;
            }
            __syncthreads();
            if (st->status != 0) {
                if (tid < n) st->xt[tid] = st->x[tid];
                return;
            }
            new_dir = true;
        } else {
            if (tid == 0) st->alpha *= 0.5;
            __syncthreads();
            const double dmax = block_maxabs(st->d, n, scratch);
            const double xmax = block_maxabs(st->x, n, scratch);
            if (st->alpha * dmax <= 1e-15 * (1.0 + xmax)) {
                if (tid == 0) st->status = 2;
                if (tid < n) st->xt[tid] = st->x[tid];
                return;
            }
            if (tid < n) st->xt[tid] = st->x[tid] + st->alpha * st->d[tid];
            if (tid == 0) st->nbacktrack += 1;
            return;
        }
    }
    if (new_dir) {
        const double gtd = new_direction(st, n, m, q, scratch);
        const bool fresh = st->count == 0;      // empty history, or reset to steepest descent
        double alpha = 1.0;
        if (fresh) {
            const double xn = sqrt(block_dot(st->x, st->x, n, scratch));
            const double dn = sqrt(block_dot(st->d, st->d, n, scratch));
            alpha = dn > 0.0 ? 0.01 * (xn > 0.0 ? xn : 1.0) / dn : 0.0;
        }
        if (tid == 0) {
            st->gtd = gtd;
            st->alpha = alpha;
            st->phase = 1;
        }
        __syncthreads();
        if (tid < n) st->xt[tid] = st->x[tid] + alpha * st->d[tid];
    }
}

}  // namespace

hipError_t launch_lbfgs(const MultiFit *fits, int k_all, const double *out, int64_t ostride,
                        LbfgsState *states, int nfits, int m, double c1, double ftol,
                        hipStream_t stream) {
    hipLaunchKernelGGL(lbfgs_kernel, dim3(nfits), dim3(kLT), 0, stream, fits, k_all, out, ostride,
                       states, m, c1, ftol);
    return hipGetLastError();
}

}  // namespace pwa
