/*
 * pwa.h -- C ABI of the MI355X (gfx950) partial-wave-analysis likelihood library.
 *
 * The library evaluates the unbinned negative log-likelihood of a partial
 * wave analysis and its gradient with respect to the complex production
 * amplitudes V, over precomputed complex decay amplitudes A (Berger, "Partial
 * Wave Analysis using Graphics Cards", Section 2):
 *
 *   Eq. 1   I(Omega) = | sum_a V_a A_a(Omega) |^2
 *   Eq. 2   -ln L = -sum_{i in data} ln I_i + N_D ln S,
 *           S = (1/N_gen) sum_{j in accepted MC} w_j I_j
 *           (MC normalisation integral; weights per the footnote on
 *           non-uniform MC; N_gen counts generated events, acceptance is
 *           expressed by supplying only accepted MC rows)
 *   Eq. 3   extended form: -ln L = -sum ln I_i + S
 *           and its bracket M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb, which
 *           can be precomputed while only V varies, giving S = V^H M V.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Complex arrays are interleaved (re, im) in the context's precision.  A
 * sample of n events with k waves is row-major: event i, wave a at complex
 * index i*ld + a (ld >= k).
 *
 * V is always FP64 on the host for the synchronous calls: 2k doubles
 * (Re V_0, Im V_0, Re V_1, ...).  The gradient has the same layout and holds
 * dNLL/dRe V_a and dNLL/dIm V_a (minimisers see real parameters only, Section
 * 4, "Fits with complex parameters").  Equivalently grad = 2 (Re g, Im g) with
 * g the Wirtinger derivative dNLL/d conj(V).
 *
 * Precision: PWA_F32 stores and streams the amplitudes in single precision;
 * each event's z, I and z/I are formed in double precision from the exact
 * single-precision values and ln I is taken in single precision; every sum
 * over events is in double precision (the paper's remark on precision in
 * Section 2).  PWA_F64 is double precision throughout.
 *
 * Errors: every call returns a pwa_status.  On an error nothing is written to
 * the caller's outputs, except PWA_E_DOMAIN, which writes NLL = +inf (and an
 * unspecified gradient) so a minimiser can reject the step.  Calls never
 * abort, print or throw; pwa_last_error() describes the last failure.
 *
 * Concurrency: a context is not thread-safe.  All its device work is ordered
 * on its stream.  The synchronous calls wait on that stream; the _async calls
 * neither wait nor allocate, so they can be captured into a HIP graph.
 */
#ifndef PWA_H
#define PWA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwa_ctx pwa_ctx;

typedef enum {
    PWA_OK = 0,
    PWA_E_INVAL = 1,        /* bad argument (null pointer, size, k mismatch, ...) */
    PWA_E_NOMEM = 2,        /* device or pinned host allocation failed */
    PWA_E_HIP = 3,          /* a HIP runtime call or kernel launch failed */
    PWA_E_DOMAIN = 4,       /* some data I <= 0, S <= 0 or a non-finite value: NLL = +inf */
    PWA_E_STATE = 5,        /* call needs samples that have not been set */
    PWA_E_UNSUPPORTED = 6   /* valid request this build does not implement (e.g. k > 64) */
} pwa_status;

typedef enum { PWA_F32 = 0, PWA_F64 = 1 } pwa_prec;
typedef enum { PWA_DATA = 0, PWA_MC = 1 } pwa_set;
typedef enum { PWA_MC_STREAM = 0, PWA_MC_GRAM = 1 } pwa_mc_mode;
/* Where an array lives: host memory, device memory (copied), or device
 * memory the library uses in place without a copy (pwa_set_amplitudes). */
typedef enum { PWA_HOST = 0, PWA_DEVICE = 1, PWA_BORROW = 2 } pwa_where;

/* Largest number of waves a context accepts. */
#define PWA_MAX_K 64

/* Create a context on HIP device `device` with amplitude precision `prec`.
 * `stream` is a hipStream_t to order all work on, or NULL for a stream the
 * context creates and owns.  A borrowed stream must outlive the context.
 * *out receives the context.  Errors: PWA_E_INVAL (null out, bad prec or
 * device), PWA_E_HIP, PWA_E_NOMEM. */
pwa_status pwa_create(pwa_ctx **out, int device, pwa_prec prec, void *stream);

/* Free every device and host resource of the context.  NULL is accepted. */
pwa_status pwa_destroy(pwa_ctx *ctx);

/* Store one sample (data or MC; Eq. 2's two sums).
 *   A      n x k complex in the context's precision, row stride ld complex,
 *          on the host or the device as `where` says.
 *          PWA_HOST, PWA_DEVICE: the library copies A into its own padded
 *          device layout; the caller may free A when the call returns.
 *          PWA_BORROW: A (and w) are device memory of the context's device
 *          that the library reads in place with no copy and no allocation of
 *          sample memory.  A must already have the device layout: ld equal to
 *          pwa_layout_ld() for k, a 16-byte aligned base, and zeros in columns
 *          k..ld-1 of every row (checked with one pass over those columns).
 *          The arrays must stay valid and unchanged until the sample is
 *          replaced or the context destroyed; the library never frees them.
 *          PWA_DEVICE and PWA_BORROW pointers that are not device memory of
 *          the context's device are rejected with PWA_E_INVAL.
 *   n      number of events (0 allowed)
 *   k      number of waves, 1..PWA_MAX_K; data and MC must agree
 *   w      MC only: n per-event weights in the context's precision, in the
 *          same memory space as A, or NULL for unit weights (footnote on
 *          weighted MC).  Must be NULL for the data sample.
 *   n_gen  MC only: number of generated events N_gen of Eq. 3's 1/N_gen;
 *          <= 0 means n.  Ignored for data.
 * Replacing a sample whose k differs from the other sample's drops the other
 * sample.  Errors: PWA_E_INVAL, PWA_E_NOMEM, PWA_E_HIP, PWA_E_UNSUPPORTED. */
pwa_status pwa_set_amplitudes(pwa_ctx *ctx, pwa_set which, const void *A, int64_t n,
                              int32_t k, int64_t ld, pwa_where where, const void *w,
                              double n_gen);

/* Select how the normalisation is evaluated and which likelihood form is used.
 *   mode      PWA_MC_STREAM: stream the MC rows on every evaluation.
 *             PWA_MC_GRAM: precompute M (Eq. 3 bracket, FP64, k x k) once from
 *             the MC rows; each evaluation then streams only the data rows
 *             and uses S = V^H M V.
 *   extended  0: Eq. 2 form (N_D ln S), 1: Eq. 3 form (+S).
 * Errors: PWA_E_INVAL. */
pwa_status pwa_set_mc_mode(pwa_ctx *ctx, pwa_mc_mode mode, int extended);

/* NLL at V (host, 2k doubles) into *nll.  Waits for the result.
 * Errors: PWA_E_INVAL, PWA_E_STATE (a sample missing; N_D = 0 needs no MC
 * and gives NLL = 0 in the Eq. 2 form), PWA_E_DOMAIN, PWA_E_HIP. */
pwa_status pwa_nll(pwa_ctx *ctx, const double *V, double *nll);

/* NLL and gradient (host, 2k doubles) at V.  One launch: a fused pass over
 * the rows that ends with the fixed-order combine of its block partials and
 * writes the result to mapped host memory, which the call polls.
 * Errors as pwa_nll. */
pwa_status pwa_nll_grad(pwa_ctx *ctx, const double *V, double *nll, double *grad);

/* Device-side variant of pwa_nll_grad for graph capture and device minimisers.
 *   V_dev    device pointer, 2k doubles, read when the kernel runs
 *   out_dev  device pointer, 2k + 2 doubles, written when the kernel runs:
 *            [0] NLL (+inf on a domain failure), [1 .. 2k] gradient,
 *            [2k + 1] status flags (0 = ok, nonzero = PWA_E_DOMAIN)
 * Enqueues on the context's stream and returns; no wait, no allocation.
 * Errors (detected on the host only): PWA_E_INVAL (also for pointers that are
 * not device memory of the context's device), PWA_E_STATE, PWA_E_HIP. */
pwa_status pwa_nll_grad_async(pwa_ctx *ctx, const double *V_dev, double *out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the NLL and
 * gradient of pwa_nll_grad_async over caller-owned device samples, with no
 * context, no allocation and no wait.  The kernel's workspace (block
 * partials, group sums, arrival counters) is a static device array of
 * PWA_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; it bounds the launch's grid, not the sample sizes.
 * The work goes to the current device.  Calls on one GPU share that array:
 * calls that may overlap on one GPU (different streams, or threads) race and
 * must be serialised by the caller; calls ordered on one stream are safe.
 *   prec        amplitude precision of the samples
 *   A_data      n_data rows, A_mc n_mc rows: device arrays in the library's
 *               layout (row stride ld = pwa_layout_ld() for k, 16-byte aligned
 *               base, zeros in columns k..ld-1; the zeros are not checked)
 *   w_mc        device MC weights (precision of A) or NULL; n_gen <= 0: n_mc
 *   extended    0: Eq. 2 form, 1: Eq. 3 form (the MC rows are streamed)
 *   V_dev       device, 2k doubles; out_dev device, 2k + 2 doubles written as
 *               by pwa_nll_grad_async; stream: hipStream_t or NULL
 * The launch configuration is the one pwa_autotune chose for these sizes in
 * this process, else the default.  Errors (host-side checks only, reported by
 * pwa_last_error(NULL)): PWA_E_INVAL, PWA_E_UNSUPPORTED (k > PWA_MAX_K),
 * PWA_E_HIP. */
#define PWA_NOALLOC_SCRATCH_BYTES (2u << 20)
pwa_status pwa_nll_grad_noalloc(pwa_prec prec, const void *A_data, int64_t n_data, const void *A_mc,
                                int64_t n_mc, const void *w_mc, double n_gen, int32_t k, int64_t ld,
                                int extended, const double *V_dev, double *out_dev, void *stream);

/* NLL (and optionally gradients) for nv production vectors in one pass over
 * the events (many fits / many starting points, Section 2 on repeated fits).
 *   V      host, nv x 2k doubles (row b is V_b as above)
 *   nll    host, nv doubles
 *   grad   host, nv x 2k doubles, or NULL for NLL only
 *   split  arithmetic of the dense contraction:
 *            0  one streaming pass per vector (the single-V kernel; any precision)
 *            2  matrix cores, one pass over the rows for all vectors: the
 *               coherent sums z = A W use two-term FP16 splits (hi + lo) of
 *               the amplitudes (power-of-two scale per wave) and of V (power-
 *               of-two scale per vector); the adjoint sums conj(A) u use
 *               two-term BF16 splits of u and of the amplitudes; FP32
 *               accumulation within a block of at most 4096 events, FP64 across
 *               blocks; the first-order effect of rounding V to the split
 *               weights is added from the adjoint sums.  A data event whose
 *               coherent sum is small against |V| |A_i| gets a large relative
 *               error in z / I; the gradient error is stated, not bounded.
 *            3  as 2, but data events with |z| < c |V| |A_i| are left out
 *               of the matrix-core sums, flagged, and their terms recomputed
 *               exactly in FP64 by a second kernel (c^2 = min(1/64, sqrt(k)/N_D):
 *               the gradient scale grows with N_D, one event's error does
 *               not): NLL and gradient of every vector within 1e-6.
 *            Splits 2 and 3 need an FP32 context.
 * V may hold any number of vectors; the FP64 results land in host memory.
 * Errors as pwa_nll (PWA_E_DOMAIN if some vector's NLL is +inf; every output
 * is written); PWA_E_UNSUPPORTED for another split, or split 2 or 3 in an FP64
 * context. */
pwa_status pwa_nll_batch(pwa_ctx *ctx, int32_t nv, const double *V, double *nll,
                         double *grad, int32_t split);

/* Device-side variant of pwa_nll_batch for graph capture and device
 * minimisers (the same arithmetic, launch configuration and results).
 *   V_dev    device pointer, nv x 2k doubles, read when the kernels run
 *   out_dev  device pointer, nv x (2k + 2) doubles, written when the kernels
 *            run: per vector [0] NLL (+inf on a domain failure), [1 .. 2k]
 *            gradient, [2k + 1] status flags (0 = ok, nonzero = domain failure)
 *   split    0, 2 or 3 as in pwa_nll_batch (0: nv single-V launches)
 * Enqueues on the context's stream and returns: no wait, no allocation, no
 * host copy.  Splits 2 and 3 use workspace and lazily built inputs (operand
 * scales, the Gram matrix in PWA_MC_GRAM mode, row norms for split 3) that a
 * synchronous pwa_nll_batch call with at least nv vectors and the same split
 * on the current samples creates; without them the call returns PWA_E_STATE
 * and enqueues nothing.  V_dev and out_dev must not overlap.
 * Errors (detected on the host only): PWA_E_INVAL (also for pointers that are
 * not device memory of the context's device), PWA_E_STATE,
 * PWA_E_UNSUPPORTED, PWA_E_HIP. */
pwa_status pwa_nll_batch_async(pwa_ctx *ctx, int32_t nv, const double *V_dev, double *out_dev,
                               int32_t split);

/* Hessian of the NLL in the real parameters at V: the matrix whose inverse is
 * the fit's error matrix (Section 4 on the cost of error calculations).
 *   V   host, 2k doubles (Re V_a, Im V_a interleaved, as for the gradient)
 *   H   host, 2k x 2k doubles, row-major: H[m * 2k + n] = d2 NLL / dx_m dx_n
 *       with x_{2a} = Re V_a, x_{2a+1} = Im V_a; symmetric.
 * Eq. 2 or Eq. 3 form as set by pwa_set_mc_mode.  One pass over the data rows
 * (per event the second derivative of 2 Re ln z_i: the complex symmetric
 * sum_i A_ia A_ic / z_i^2, FP64 from the stored amplitudes) plus the MC matrix
 * of Eq. 3 (built once per MC sample, as in PWA_MC_GRAM mode) for the
 * normalisation term.  Synchronous; allocates workspace on first use.
 * Errors: PWA_E_INVAL, PWA_E_STATE (a sample missing), PWA_E_DOMAIN (a data
 * event with z = 0, or S <= 0; H then holds non-finite values), PWA_E_HIP. */
pwa_status pwa_hessian(pwa_ctx *ctx, const double *V, double *H);

/* Parameters the batched minimiser works in (Section 4, "Fits with complex
 * parameters": minimisers see real numbers, and both representations of a
 * complex parameter have their issues).
 *   PWA_PARAM_CARTESIAN  (Re V_a, Im V_a) per wave, unbounded.
 *   PWA_PARAM_POLAR      (|V_a|, arg V_a) per wave with the lower bound
 *                        |V_a| >= rmin kept by projected steps, periodic phases
 *                        wrapped into [-pi, pi] after each accepted step, and
 *                        arg V_0 held at 0 (the likelihood does not depend on
 *                        the global phase). */
typedef enum { PWA_PARAM_CARTESIAN = 0, PWA_PARAM_POLAR = 1 } pwa_param;

/* Minimise the NLL from nv starting vectors at once on the context's samples
 * (multi-start, Section 2): every iteration evaluates all trial vectors with
 * the matrix-core pass of pwa_nll_batch with split 3 (small coherent sums
 * recomputed exactly: NLL and gradient within 1e-6 of the oracle's) and
 * advances one device L-BFGS state per vector (two-loop recursion, history 8,
 * Armijo backtracking) in the parameters `param` selects (rmin: the polar
 * magnitude bound, >= 0; ignored for PWA_PARAM_CARTESIAN); the iteration is
 * captured in a HIP graph and replayed `iters` times.  Outputs (host, any may
 * be NULL): V nv x 2k accepted points as (Re V_a, Im V_a) (in polar form with
 * V_0 real and non-negative), nll[nv] their NLL, status[nv] (0 running,
 * 1 converged, 2 step underflow), avg_ms time per iteration.  FP32 contexts,
 * k <= 48.  Errors as pwa_nll_batch, PWA_E_INVAL for a bad param or rmin. */
pwa_status pwa_batch_fit(pwa_ctx *ctx, int32_t nv, const double *V0, int32_t iters, pwa_param param,
                         double rmin, double *V, double *nll, int32_t *status, double *avg_ms);

/* Status flags of the last synchronous evaluation (0 = none). */
pwa_status pwa_last_flags(pwa_ctx *ctx, uint32_t *flags);

/* Message for the last failing call on this context (or on a NULL context). */
const char *pwa_last_error(const pwa_ctx *ctx);

/* Row stride (complex elements) of the library's device layout for k waves. */
pwa_status pwa_layout_ld(pwa_ctx *ctx, int32_t k, int64_t *ld);

/* Launch configuration of the single-V streaming kernel (a tile shape and grid
 * size; none of it changes results beyond summation order).
 *   lanes_per_row     L: lanes that share one event row (power of two)
 *   complex_per_lane  C: consecutive complex amplitudes per lane; L * C must
 *                     equal the layout width pwa_layout_ld() gives for k
 *   rows_per_stage    U: rows each lane group loads per pipeline stage
 *   blocks_per_cu     grid blocks per compute unit, 1..16 (fewer when the
 *                     rows need fewer) */
typedef struct {
    int32_t lanes_per_row;
    int32_t complex_per_lane;
    int32_t rows_per_stage;
    int32_t blocks_per_cu;
} pwa_stream_cfg;

/* Current configuration (after set_amplitudes fixed k). Errors: PWA_E_INVAL, PWA_E_STATE. */
pwa_status pwa_get_stream_cfg(pwa_ctx *ctx, pwa_stream_cfg *cfg);

/* Use `cfg` for later evaluations.  PWA_E_UNSUPPORTED if this (L, C, U) is
 * not compiled or does not match the layout width; PWA_E_INVAL for a bad
 * blocks_per_cu. */
pwa_status pwa_set_stream_cfg(pwa_ctx *ctx, const pwa_stream_cfg *cfg);

/* Autotuner: times every compiled configuration of the current layout width
 * (and blocks_per_cu in {2, 3, 4, 6, 8, 12, 16}) on the samples currently set,
 * `reps` evaluations each (the pass over the rows and the combine of its
 * block partials) after one warm-up, keeps the fastest (of those within 1% of
 * it, the one with the fewest blocks per CU, then rows per stage, then lanes
 * per row, so that tuning the same shapes again settles on one configuration)
 * in the context and
 * in a per-process cache keyed by (device, precision, width, sample sizes),
 * which later contexts of the same shape start from.  Writes the chosen
 * configuration and its average kernel time (ms) if the pointers are non-NULL.
 * Needs both samples set.  Errors: PWA_E_STATE, PWA_E_HIP. */
pwa_status pwa_autotune(pwa_ctx *ctx, int32_t reps, pwa_stream_cfg *best, double *best_ms);

/* Kernel timing: average duration in ms of the streaming kernel (the pass over
 * the rows and the combine of its block partials, one launch) over the
 * single-V evaluations since the last query, measured with HIP events on the
 * context's stream while timing is enabled with pwa_set_timing(ctx, 1).
 * Timing records an event pair per call (events are reused). */
pwa_status pwa_set_timing(pwa_ctx *ctx, int enable);
pwa_status pwa_kernel_time(pwa_ctx *ctx, double *avg_ms, int64_t *count);

/* Same for the matrix-core pass of pwa_nll_batch (split 2), without its
 * per-vector combine kernel. */
pwa_status pwa_batch_kernel_time(pwa_ctx *ctx, double *avg_ms, int64_t *count);

/* Same for pwa_hessian: events recorded on the context's stream before its
 * first kernel and after its last (the data pass, the partial sums and the
 * assembly of H), without the H readback.  A synchronous call starts on an
 * idle stream, so the interval includes the wait for the first launch. */
pwa_status pwa_hessian_kernel_time(pwa_ctx *ctx, double *avg_ms, int64_t *count);

/* ------------------------------------------------------------------------
 * Amplitudes formed on the device from each event's kinematics, so that the
 * masses and widths of the resonances can be fit parameters (Section 2: the
 * amplitudes can be precomputed only while masses and widths are constant).
 * Each event is (m, cos theta) in FP32 (8 bytes) and wave a has a spin J_a
 * (0..4); per evaluation, with resonance parameters (m_a, Gamma_a),
 *     A_a = BW_a(m) Y_{J_a}^0(cos theta),
 *     BW_a(m) = 1 / (m_a^2 - m^2 - i m_a Gamma_a)   (fixed-width Breit-Wigner),
 *     Y_J^0(x) = sqrt((2 J + 1) / (4 pi)) P_J(x)   (Legendre polynomial P_J),
 * and the NLL of Eq. 2 (or Eq. 3) over these amplitudes, its gradient in V
 * (as pwa_nll_grad) and its gradient in (m_a, Gamma_a):
 *     dNLL/dt = -sum_data (1/I) dI/dt + c sum_MC w dI/dt,
 *     dI/dt = 2 Re(conj(z) V_a Y_a dBW_a/dt),
 *     dBW_a/dm_a = -(2 m_a - i Gamma_a) BW_a^2,  dBW_a/dGamma_a = i m_a BW_a^2,
 * c = N_D / (N_gen S) (Eq. 2) or 1 / N_gen (Eq. 3).  Everything after the
 * FP32 kinematics is FP64; the MC rows are streamed on every evaluation (the
 * MC bracket changes with the masses and widths).
 * ------------------------------------------------------------------------ */
typedef struct pwa_kin pwa_kin;

/* Create a kinematic context for k waves (1..PWA_MAX_K) with spins spin[k]
 * (each 0..4; PWA_E_UNSUPPORTED otherwise) on `device`; stream as in
 * pwa_create.  Errors: PWA_E_INVAL, PWA_E_UNSUPPORTED, PWA_E_NOMEM, PWA_E_HIP. */
pwa_status pwa_kin_create(pwa_kin **out, int device, int32_t k, const int32_t *spin, void *stream);
pwa_status pwa_kin_destroy(pwa_kin *kc);

/* Store the events of one sample: mx = n pairs (m, cos theta) of FP32, w (MC
 * only) n FP32 weights or NULL, n_gen as in pwa_set_amplitudes.  `where` as in
 * pwa_set_amplitudes (PWA_BORROW: device arrays used in place, 8-byte aligned
 * events, valid until replaced or destroyed).  Errors: PWA_E_INVAL,
 * PWA_E_NOMEM, PWA_E_HIP. */
pwa_status pwa_kin_set_events(pwa_kin *kc, pwa_set which, const float *mx, int64_t n, pwa_where where,
                              const float *w, double n_gen);

/* 0: Eq. 2 form, 1: Eq. 3 form. */
pwa_status pwa_kin_set_mode(pwa_kin *kc, int extended);

/* NLL at V (host, 2k doubles) and res (host, 2k doubles: m_a, Gamma_a
 * interleaved, finite and positive); grad_v (2k, as pwa_nll_grad) and
 * grad_res (2k: dNLL/dm_a, dNLL/dGamma_a interleaved) may be NULL.  One
 * launch; waits for the result.  Errors: PWA_E_INVAL, PWA_E_STATE,
 * PWA_E_DOMAIN (NLL = +inf), PWA_E_HIP. */
pwa_status pwa_kin_nll_grad(pwa_kin *kc, const double *V, const double *res, double *nll, double *grad_v,
                            double *grad_res);

/* Device-side variant: V_dev and res_dev (2k doubles each) read when the
 * kernel runs, out_dev (4k + 2 doubles) written as [NLL, grad_v[2k],
 * grad_res[2k], flags] (flags nonzero: domain failure, NLL = +inf).  No wait,
 * no allocation.  res_dev must hold positive values (not checked).
 * Errors (host-side only): PWA_E_INVAL, PWA_E_STATE, PWA_E_HIP. */
pwa_status pwa_kin_nll_grad_async(pwa_kin *kc, const double *V_dev, const double *res_dev, double *out_dev);

/* Message for the last failing call on this context (or on a NULL context). */
const char *pwa_kin_last_error(const pwa_kin *kc);

/* ------------------------------------------------------------------------
 * Many independent fits (Section 2: fits are repeated from many starting
 * points and with many models).  Every fit has its own samples and its own
 * production vector; one minimiser iteration of all fits is one persistent
 * evaluation launch over the rows of every fit (uneven sizes balanced by a
 * work-item queue), a per-fit combine, and one L-BFGS update per fit on the
 * device, captured in a HIP graph and replayed per step.  FP32 amplitudes, the
 * Eq. 2 form, streamed MC.
 * ------------------------------------------------------------------------ */
typedef struct pwa_multi pwa_multi;

/* One fit: host arrays, FP32 interleaved complex rows of stride ld (>= k). */
typedef struct {
    const float *A_data;
    int64_t n_data;
    const float *A_mc;
    int64_t n_mc;          /* > 0 when n_data > 0 */
    const float *w_mc;     /* MC weights or NULL */
    double n_gen;          /* <= 0: n_mc */
    int32_t k;             /* 1..48 */
    int64_t ld;
    const double *V0;      /* 2k start vector */
} pwa_fit_desc;

/* Copy every fit's samples to the device and set each minimiser at its V0.
 * `stream`: hipStream_t or NULL (owned).  Errors: PWA_E_INVAL, PWA_E_NOMEM,
 * PWA_E_HIP, PWA_E_UNSUPPORTED (k > 48). */
pwa_status pwa_multi_create(pwa_multi **out, int device, int32_t nfits, const pwa_fit_desc *fits,
                            void *stream);
pwa_status pwa_multi_destroy(pwa_multi *m);

/* Evaluate every fit at V (host; the fits' 2k vectors concatenated) in one
 * persistent launch: nll[nfits], grad (concatenated, may be NULL).  Overwrites
 * the minimisers' trial points; call pwa_multi_reset before stepping again.
 * PWA_E_DOMAIN if some fit's NLL is +inf (all outputs written). */
pwa_status pwa_multi_eval(pwa_multi *m, const double *V, double *nll, double *grad);

/* Restart every minimiser at V0 (concatenated). */
pwa_status pwa_multi_reset(pwa_multi *m, const double *V0);

/* Replay `steps` minimiser iterations (the captured graph).  Each replay
 * evaluates every fit's trial point and advances its L-BFGS state (Armijo
 * backtracking; history 8).  avg_ms (optional): HIP-event time per replay. */
pwa_status pwa_multi_step(pwa_multi *m, int32_t steps, double *avg_ms);

/* Current accepted points (concatenated), NLL values, status (0 running,
 * 1 converged, 2 step underflow) and accepted iterations per fit; any pointer
 * may be NULL. */
pwa_status pwa_multi_get(pwa_multi *m, double *V, double *nll, int32_t *status, int32_t *iters);

/* Autotuner of the persistent launch: times the evaluation of all fits for
 * work items of 64 KB .. 4 MB of rows and 1 .. 16 blocks per compute unit,
 * `reps` launches each, keeps the fastest (and rebuilds the graph). */
pwa_status pwa_multi_autotune(pwa_multi *m, int32_t reps, int64_t *item_bytes, int32_t *blocks_per_cu,
                              double *best_ms);

const char *pwa_multi_last_error(const pwa_multi *m);

/* ------------------------------------------------------------------------
 * Surrogate of the NLL for screening starting points.  Fits are repeated
 * from many starting points to find the global minimum (Section 2), and fits
 * with many parameters are expensive (Section 4); a small network trained on
 * exact (V, NLL) pairs ranks candidate starts cheaply, and only the best are
 * refined with the exact likelihood (pwa_batch_fit).
 *
 * Network: in -> hidden -> hidden -> 1 with exact-erf GELU after both hidden
 * layers, y = w3 . GELU(W2 GELU(W1 x + b1) + b2) + b3.  Parameters: one FP32
 * array [W1 (hidden x in, row-major) | b1 | W2 (hidden x hidden) | b2 | w3 | b3]
 * (FP32 master copy); matrix products round both operands to FP16 and
 * accumulate in FP32 on the matrix cores; the head rounds its activations and
 * weights to FP16 too.  Loss: mean squared error.  Optimiser: Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Inputs:  features  V^ = V e^{-i arg V_0} / |V| as (Re, Im) pairs (the Eq. 2
 *          NLL depends on V only through these);  targets t = ln(1 + NLL -
 *          min NLL).
 *
 * All array arguments are device pointers (FP32 unless stated) on the
 * object's device; every call orders its work on the object's stream and
 * waits for it before returning.  Errors: PWA_E_INVAL for bad sizes or null
 * pointers, PWA_E_NOMEM, PWA_E_HIP.
 * ------------------------------------------------------------------------ */
typedef struct pwa_mlp pwa_mlp;

/* Number of FP32 parameters of an in -> hidden -> hidden -> 1 network (-1 if a size is < 1). */
int64_t pwa_mlp_param_count(int32_t in, int32_t hidden);

/* Create a network on `device` (parameters zero; set them with
 * pwa_mlp_set_params).  in 1..128, hidden 1..4096; max_batch 1..65536 rows
 * bounds the training batch and the rows one inference pass holds.
 * `stream`: hipStream_t or NULL (owned). */
pwa_status pwa_mlp_create(pwa_mlp **out, int device, int32_t in, int32_t hidden, int32_t max_batch,
                          void *stream);
pwa_status pwa_mlp_destroy(pwa_mlp *m);

/* Copy all parameters in (host or device memory per `where`); resets the
 * Adam moments and step count. */
pwa_status pwa_mlp_set_params(pwa_mlp *m, const float *P, pwa_where where);
pwa_status pwa_mlp_get_params(pwa_mlp *m, float *P, pwa_where where);

/* X [n][2k] = canonical features of V [n][2k] (FP64, interleaved complex);
 * 2k must equal the input width.  A zero vector gives zero features. */
pwa_status pwa_mlp_features(pwa_mlp *m, const double *V, int64_t n, int32_t k, float *X);

/* t[n] = ln(1 + NLL - min NLL) from nll[n] (FP64); non-finite NLL values get
 * the largest finite target + 1. */
pwa_status pwa_mlp_targets(pwa_mlp *m, const double *nll, int64_t n, float *t);

/* y[n] = network output for the rows of X [n][in]. */
pwa_status pwa_mlp_predict(pwa_mlp *m, const float *X, int64_t n, float *y);

/* One forward and backward pass over B <= max_batch rows without an update:
 * *loss (host) = mean squared error, G = its gradient (layout of the
 * parameters). */
pwa_status pwa_mlp_loss_grad(pwa_mlp *m, const float *X, const float *t, int32_t B, float *loss, float *G);

/* nsteps Adam steps with learning rate lr; step s uses the rows
 * perm[s * batch .. s * batch + batch - 1] of X [n][in] and t[n] (perm: int32
 * device array of nsteps * batch entries in [0, n); the random order is the
 * caller's).  One step (gather, forward, backward, Adam) and a group of 16
 * steps are captured in HIP graphs and replayed (whole groups first).  loss_hist (device, nsteps floats, or NULL) receives
 * each step's batch loss; avg_ms (host, optional) the time per step.
 * PWA_E_INVAL after the run if some perm entry was out of range (row 0 was
 * used in its place). */
pwa_status pwa_mlp_train(pwa_mlp *m, const float *X, const float *t, int64_t n, const int32_t *perm,
                         int32_t batch, int32_t nsteps, float lr, float *loss_hist, double *avg_ms);

/* idx[k] = indices of the k smallest of keys[n], ascending (ties by index,
 * NaN counts as +inf); 1 <= k <= 2048, k <= n < 2^31. */
pwa_status pwa_mlp_select(pwa_mlp *m, const float *keys, int64_t n, int32_t k, int32_t *idx);

const char *pwa_mlp_last_error(const pwa_mlp *m);

#ifdef __cplusplus
}
#endif

#endif /* PWA_H */
