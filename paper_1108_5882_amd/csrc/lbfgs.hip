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
//
// Polar mode (the other representation Section 4 discusses): parameters
// (|V_a|, arg V_a) per wave.  The gradient in them follows from the one in
// (Re V_a, Im V_a) by the chain rule, d/d|V| = cos(phi) d/dRe + sin(phi) d/dIm,
// d/dphi = |V| (-sin(phi) d/dRe + cos(phi) d/dIm).  arg V_0 is held at 0 (the
// likelihood does not change under a global phase, so fixing it removes a flat
// direction).  The lower bound |V_a| >= rmin is kept by projecting every trial
// point onto it, dropping direction components that push a magnitude at the
// bound further down, and testing the Armijo condition along the projected
// step, f_t <= f + c1 g.(x_t - x).  Phases are periodic: after each accepted
// step they are wrapped into [-pi, pi] (the history keeps the step taken).
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

// Polar mode: st->gtd = g.(xt - x), the slope along the projected step the
// Armijo test uses.
__device__ void step_slope(LbfgsState *st, int n, double *scratch, double *tmp) {
    const int tid = threadIdx.x;
    if (tid < n) tmp[tid] = st->xt[tid] - st->x[tid];
    __syncthreads();
    const double v = block_dot(st->g, tmp, n, scratch);
    if (tid == 0) st->gtd = v;
    __syncthreads();
}

// Polar mode: trial point projected onto |V_a| >= rmin (arg V_0 stays 0), and
// the V it stands for written to vt.
__device__ void polar_trial(LbfgsState *st, int n, double rmin) {
    const int tid = threadIdx.x;
    __syncthreads();
    if (tid < n && (tid & 1) == 0) {
        const double r = fmax(st->xt[tid], rmin);
        const double ph = tid == 0 ? 0.0 : st->xt[tid + 1];
        st->xt[tid] = r;
        if (tid == 0) st->xt[1] = 0.0;
        st->vt[tid] = r * cos(ph);
        st->vt[tid + 1] = r * sin(ph);
    }
    __syncthreads();
}

__global__ __launch_bounds__(kLT) void lbfgs_kernel(const MultiFit *fits, int k_all,
                                                    const double *out, int64_t ostride,
                                                    LbfgsState *states, int m, double c1,
                                                    double ftol, int polar, double rmin) {
    __shared__ double scratch[kLT];
    __shared__ double q[kLT];
    __shared__ double gp[kLT];
    __shared__ int s_accept;
    const int f = blockIdx.x, tid = threadIdx.x;
    LbfgsState *st = states + f;
    const int n = 2 * (fits ? fits[f].k : k_all);
    if (st->status != 0) return;
    const double *o = out + (int64_t)f * ostride;
    const double ft = o[0];
    const double *gt = o + 1;
    if (polar) {
        // gradient in (|V_a|, arg V_a) at the trial point (arg V_0 held fixed)
        if (tid < n && (tid & 1) == 0) {
            const double r = st->xt[tid], ph = st->xt[tid + 1];
            const double c = cos(ph), sn = sin(ph);
            gp[tid] = c * gt[tid] + sn * gt[tid + 1];
            gp[tid + 1] = tid == 0 ? 0.0 : r * (-sn * gt[tid] + c * gt[tid + 1]);
        }
        __syncthreads();
        gt = gp;
    }

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
        if (tid == 0) s_accept = isfinite(ft) && ft <= st->f + c1 * (polar ? st->gtd : st->alpha * st->gtd);
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
            if (polar && tid < n && (tid & 1) == 1) {
                // periodic phases back into [-pi, pi]
                const double w = remainder(st->x[tid], 6.283185307179586476925286766559);
                st->x[tid] = w;
                st->xt[tid] = w;
            }
            __syncthreads();
            if (st->status != 0) {
                if (tid < n) st->xt[tid] = st->x[tid];
                if (polar) polar_trial(st, n, rmin);
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
                if (polar) polar_trial(st, n, rmin);
                return;
            }
            if (tid < n) st->xt[tid] = st->x[tid] + st->alpha * st->d[tid];
            if (tid == 0) st->nbacktrack += 1;
            if (polar) {
                polar_trial(st, n, rmin);
                step_slope(st, n, scratch, q);
            }
            return;
        }
    }
    if (new_dir) {
        double gtd = new_direction(st, n, m, q, scratch);
        if (polar) {
            // no component that pushes a magnitude at its bound further down
            if (tid < n && (tid & 1) == 0 && st->x[tid] <= rmin && st->d[tid] < 0.0) st->d[tid] = 0.0;
            __syncthreads();
            gtd = block_dot(st->g, st->d, n, scratch);
            if (!(gtd < 0.0)) {
                if (tid == 0) st->count = 0;
                if (tid < n) st->d[tid] = (tid & 1) == 0 && st->x[tid] <= rmin && st->g[tid] > 0.0 ? 0.0 : -st->g[tid];
                __syncthreads();
                gtd = block_dot(st->g, st->d, n, scratch);
                if (!(gtd < 0.0)) {          // stationary on the bound
                    if (tid == 0) st->status = 1;
                    if (tid < n) st->xt[tid] = st->x[tid];
                    polar_trial(st, n, rmin);
                    return;
                }
            }
        }
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
        if (polar) {
            polar_trial(st, n, rmin);
            step_slope(st, n, scratch, q);
        }
    }
}

}  // namespace

hipError_t launch_lbfgs(const MultiFit *fits, int k_all, const double *out, int64_t ostride,
                        LbfgsState *states, int nfits, int m, double c1, double ftol,
                        hipStream_t stream, int polar, double rmin) {
    hipLaunchKernelGGL(lbfgs_kernel, dim3(nfits), dim3(kLT), 0, stream, fits, k_all, out, ostride,
                       states, m, c1, ftol, polar, rmin);
    return hipGetLastError();
}

}  // namespace pwa
