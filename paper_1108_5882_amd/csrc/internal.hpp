// Internal declarations of the gfx950 partial-wave likelihood library.
// Not part of the C ABI (include/pwa.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
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
    double *partials;          // [nb[0] + nb[1]][pstride] block partials
    double *gsums;             // [groups][2 pstride] sums of groups of kFinishGroup blocks
    unsigned *counters;        // [1 + groups] arrival counts: zero before a launch and after it
    double *out;               // [nll, grad[2k], flags]
    unsigned long long *done;  // or nullptr: receives seq once out is written (host-mapped memory)
    unsigned long long seq;
    const double *gram;        // MC matrix (k x k complex FP64, 1/N_gen folded) or nullptr
    double n_gen;              // N_gen of the MC estimate (stream mode)
    double nd_total;           // N_D as a double
    int32_t extended;          // 0: Eq. 2 form, 1: Eq. 3 form
    int32_t pad_;
    double v_arg[2 * PWA_MAX_K];   // V by value when v_dev is null
};

// Launch configuration of the streaming kernel: L lanes cooperate on one
// event row, each lane holding C consecutive complex amplitudes (the device
// layout's row width is ld = L * C); each lane group takes U rows per pipeline
// stage; the grid has blocks_per_cu blocks per compute unit (fewer if the
// rows need fewer).
struct StreamCfg {
    int L;
    int C;
    int U;
    int blocks_per_cu;
};

constexpr int kStreamThreads = 256;
constexpr int kMaxBlocksPerCu = 16;

// Rows one wave covers per pipeline stage.
inline int stream_rows_per_wave(const StreamCfg &c) { return (64 / c.L) * c.U; }

// Every (L, C, U) compiled for the precision (blocks_per_cu left 0).
const StreamCfg *stream_variants(pwa_prec prec, int *count);

// Row width of the device layout for k waves: the smallest L * C >= k.
int stream_layout_ld(pwa_prec prec, int k);

// Default configuration for a layout width (used until a tuned one is set).
StreamCfg stream_default_cfg(pwa_prec prec, int ld);

// True if (L, C, U) is compiled for the precision.
bool stream_cfg_available(pwa_prec prec, const StreamCfg &c);

// Grid of one evaluation over n0 data and n1 MC rows: blocks per segment, at
// most what the rows need and at most `budget` in all, split in proportion to
// the rows.
void stream_grid(const StreamCfg &cfg, int64_t budget, int64_t n0, int64_t n1, int32_t nb[2]);

// Message pwa_last_error(NULL) returns on this thread.
void set_global_error(const char *msg);

// Configuration pwa_autotune chose for these sample sizes in this process, if any.
bool stream_tuned_cfg(int device, pwa_prec prec, int64_t ld, int64_t nd, int64_t nm, StreamCfg *cfg);

// The streaming kernel ends with the combine of its block partials: the last
// block of each group of kFinishGroup consecutive blocks adds the group's
// partials in block order, and the last group to finish adds the group sums
// in group order and writes [nll, grad[2k], flags] to args.out (a fixed order
// throughout, so results are bitwise reproducible for a launch configuration).
constexpr int kFinishGroup = 16;
inline int stream_groups(int blocks) { return (blocks + kFinishGroup - 1) / kFinishGroup; }
// Doubles of block partials and group sums a launch of `blocks` blocks needs.
inline size_t stream_scratch_doubles(int blocks, int pstride) {
    return (size_t)blocks * pstride + (size_t)stream_groups(blocks) * 2 * pstride;
}
// Counters a launch of `blocks` blocks needs (zero before the first launch).
inline size_t stream_counter_words(int blocks) { return 1 + (size_t)stream_groups(blocks); }

// Launches the streaming kernel (the pass over the rows and the combine of its
// block partials); returns hipSuccess or the launch error.
hipError_t launch_stream(pwa_prec prec, const StreamCfg &cfg, int blocks, const StreamArgs &args,
                         hipStream_t stream);

// Arguments of the batched (many-V) kernels.
struct BatchArgs {
    const float *A[2];         // FP32 device rows (data, MC), ld complex each
    const float *w;            // MC weights or nullptr
    int64_t n[2];
    int64_t ld;
    int32_t k;
    int32_t nv;                // number of production vectors
    int32_t nb[2];             // blocks per segment (tpb tiles each)
    int32_t tpb;               // tiles (32 rows) per block
    int32_t pstride;           // doubles per (vector, block) partial: 1 + 2k
    int32_t extended;
    const void *planes[2];     // split operand planes per segment (batch_plane_bytes each)
    const void *wfrag;         // FP16 forward weights in MFMA fragment order
    const float *ascale;       // power-of-two scale per real column (32 * ks entries)
    const double *vscale;      // power-of-two scale of each vector's weights
    const double *V;           // production vectors (FP64), vector v at V + v * vstride
    int64_t vstride;           // doubles between vectors (>= 2k)
    int64_t ostride;           // doubles between vectors' results in out (>= 2k + 2)
    const double *gram;        // MC matrix or nullptr
    double n_gen;
    double nd_total;
    double *partials;          // [nv][blocks][pstride]
    double *out;               // [nv][ostride]: nll, grad[2k], flags
    // exact refinement of small coherent sums (data segment; pwa_nll_batch split 3)
    const float *rnorm;        // |A_i|^2 per data row
    unsigned long long *flags; // batch_flag_words() lane masks
    float cthr2;               // c^2 of the flag test |z| < c |V| |A_i|
    int32_t ngroups_pad;       // vector groups rounded up to whole blocks
};

constexpr int kTilesPerBlock = 128;  // most tiles a block of the batched pass takes
constexpr int kBatchWaves = 8;       // waves (vector groups) per block of the batched kernel

// Tiles per block for samples of n0 and n1 rows on cu compute units: the
// fewest rounds of cu blocks with at most kTilesPerBlock tiles each, the
// tiles spread evenly over them.
int batch_tiles_per_block(int64_t n0, int64_t n1, int cu);
int64_t batch_blocks(int64_t n, int tpb);
int batch_ks(int k);
int batch_ct(int k);                 // column tiles per wave (4 for k <= 32, else 2)
int batch_vectors_per_wave(int k);   // 8 * batch_ct(k)
int batch_vector_groups(int nv, int k);
size_t batch_partial_doubles(int64_t n0, int64_t n1, int tpb, int nv, int k);
hipError_t launch_amax(const float *A, int64_t n, int64_t ld, int k, unsigned *out,
                       hipStream_t stream);
// The matrix-core pass (block partials per vector), then the per-vector combine.
// With refine, data events with small coherent sums are flagged instead of
// summed, and launch_batch_refine adds them exactly (before the combine).
hipError_t launch_batch(const BatchArgs &args, bool refine, hipStream_t stream);
hipError_t launch_batch_refine(const BatchArgs &args, hipStream_t stream);
size_t batch_flag_words(int64_t n0, int nv, int k);
hipError_t launch_rownorm(const float *A, int64_t n, int64_t ld, int k, float *out, hipStream_t stream);
// The batched pass's operand planes of one sample (FP16 hi / lo scaled by ascale,
// BF16 hi / lo transposed; 32-event tiles) and their size in bytes.
size_t batch_plane_bytes(int64_t n, int k);
hipError_t launch_batch_planes(const float *A, int64_t n, int64_t ld, int k, const float *ascale, void *out,
                               hipStream_t stream);
constexpr float kRefineC2 = 1.0f / 64.0f;     // largest c^2 (c = 1/8); batch_setup lowers it as sqrt(k) / N_D
hipError_t launch_batch_combine(const BatchArgs &args, hipStream_t stream);
// Device-side forward weights from args.V: the per-vector scales, then the
// FP16 fragments (args.wfrag, sized for the padded vector groups).
hipError_t launch_batch_weights(const BatchArgs &args, hipStream_t stream);

// ---------------------------------------------------------------- multi-fit
constexpr int kMultiMaxLd = 48;                   // widest row of the multi-fit kernel
constexpr int kMultiSlot = 1 + 2 * kMultiMaxLd;   // doubles per item partial
constexpr int kMultiOut = 2 * kMultiMaxLd + 2;    // doubles per fit result
constexpr int kLbfgsMaxHist = 16;
constexpr int kLbfgsMaxN = 2 * kMultiMaxLd;

struct MultiFit {
    const float *A_data;       // device rows, ld complex each, zero padded
    const float *A_mc;
    const float *w_mc;         // MC weights or nullptr
    int64_t n_data, n_mc;
    int64_t ld;                // row width: one of multi_layout_ld's widths
    int32_t k;
    int32_t item_data0, item_data1, item_mc0, item_mc1;   // item ranges of the two samples
    int32_t pad_;
    double n_gen;
    const double *V;           // trial vector (2k doubles) the evaluation reads
};

struct MultiItem {
    int32_t fit;
    int32_t seg;               // 0 data, 1 MC
    int64_t t0, t1;            // tile range within the sample
};

struct MultiArgs {
    const MultiFit *fits;
    const MultiItem *items;
    int32_t n_fits, n_items;
    unsigned *item_counter;    // zero before a launch; the combine resets it
    double *partials;          // [items][kMultiSlot]
    double *out;               // [fits][kMultiOut]: nll, grad[2k], flags
};

// L-BFGS state of one fit (device memory).
// Parameters x are (Re V_a, Im V_a) per wave, or in polar mode (|V_a|, arg V_a)
// with arg V_0 held at 0; vt is the trial point as V (Re, Im) in polar mode.
struct LbfgsState {
    double x[kLbfgsMaxN], g[kLbfgsMaxN], xt[kLbfgsMaxN], d[kLbfgsMaxN], vt[kLbfgsMaxN];
    double S[kLbfgsMaxHist][kLbfgsMaxN], Y[kLbfgsMaxHist][kLbfgsMaxN], rho[kLbfgsMaxHist];
    double f, alpha, gtd;
    int32_t head, count, phase, iter, status, nbacktrack;
};

int64_t multi_layout_ld(int k);              // -1 if k is too large
bool multi_ld_supported(int64_t ld);
int multi_rows_per_tile(int64_t ld);         // rows one wave covers per tile
hipError_t launch_multi_eval(const MultiArgs &args, int blocks, hipStream_t stream);
// One L-BFGS update per fit: fit f has 2 * k_f parameters (k_f = fits[f].k, or
// k_all when fits is null) and its result [nll, grad] at out + f * ostride.
// polar: parameters (|V_a|, arg V_a) with |V_a| >= rmin (projected steps),
// arg V_0 fixed at 0 and phases wrapped into [-pi, pi] after each accepted
// step; the evaluation reads vt.  Otherwise (Re V_a, Im V_a) and the
// evaluation reads xt.
hipError_t launch_lbfgs(const MultiFit *fits, int k_all, const double *out, int64_t ostride,
                        LbfgsState *states, int nfits, int m, double c1, double ftol,
                        hipStream_t stream, int polar = 0, double rmin = 0.0);

// Copies n rows of `width` bytes from src (rows src_pitch apart; host or
// device memory per kind) to dst (rows dst_pitch apart, the bytes past width
// zeroed).  Contiguous copies go in one transfer; host rows that need
// re-striding are packed on the host in chunks first (a pitched copy from
// pageable host memory moves row by row).  Returns when the rows are on the
// device.
hipError_t stage_rows(void *dst, size_t dst_pitch, const void *src, size_t src_pitch, size_t width, size_t n,
                      hipMemcpyKind kind, hipStream_t stream);

// Sets *bad (device word, zeroed by the caller) to 1 if a row of the sample
// (n rows of ld complex in the precision) holds a nonzero value in columns
// [k, ld).  Nothing is launched when ld == k.
hipError_t launch_pad_check(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, unsigned *bad,
                            hipStream_t stream);

// Gram matrix of the MC rows (Eq. 3 bracket), FP64 result on the device.
//   partials: device scratch of at least gram_partial_doubles(k, blocks) doubles.
hipError_t launch_gram(pwa_prec prec, const void *A, const void *w, int64_t n, int64_t ld, int k,
                       double n_gen, double *partials, int blocks, double *M, hipStream_t stream);
size_t gram_partial_doubles(int k, int blocks);

// Hessian of the NLL in the real parameters (hessian.hip): one pass over the n
// data rows (A, row stride ld complex) at V (2k doubles, host; passed to the
// kernels by value) with the
// MC matrix M (k x k complex, FP64, 1/N_gen folded in; null when the
// likelihood has no normalisation term), nd data events and the likelihood
// form; writes H (2k x 2k row-major, then one status double: 0 ok, 1 domain
// failure) to H, device memory or mapped host memory.  blocks:
// hessian_blocks(prec, k, cu_count, n); work: hessian_work_doubles(k, blocks)
// doubles; flag: one unsigned.  The status word is left at zero by every call
// that completes; clear = true zeroes it first (a new buffer, or after a call
// that did not complete).
hipError_t launch_hessian(pwa_prec prec, const void *A, int64_t n, int64_t ld, int k, const double *V,
                          const double *M, double nd, int extended, double *work, int blocks, bool clear,
                          unsigned *flag, double *H, hipStream_t stream);
int hessian_blocks(pwa_prec prec, int k, int cu_count, int64_t n);
size_t hessian_work_doubles(int k, int blocks);

// ---------------------------------------------------------------- surrogate MLP
// Device buffers of the in -> hidden -> hidden -> 1 network (FP32 master
// parameters P in the layout [W1 hidden x in][b1][W2 hidden x hidden][b2][w3][b3]).
struct MlpBuffers {
    int in, hidden, max_batch;
    int64_t nparams;
    float *P, *G, *M1, *M2;           // parameters, gradient, Adam moments
    float *Z1, *H1, *Z2, *H2;         // pre-activations and activations [max_batch][hidden]
    float *dZ1, *dZ2;                 // their gradients
    float *y, *dy, *lrow, *loss;      // outputs, output gradient, per-row loss, mean loss
    float *Xb, *tb;                   // gathered mini-batch features and targets
    float *ws;                        // reduction workspace, mlp_workspace_floats(in, hidden) floats
    int *step, *batch, *bad;          // Adam step count, mini-batch index, bad-index flag (device)
    // fused path (hidden width 256): the row pass's FP16 planes (H1, dZ2, dZ1, X
    // transposed) and per-slice vector sums
    _Float16 *fact = nullptr;
    float *fvec = nullptr;
    _Float16 *fwh = nullptr;          // fp16 W1 [256][128], W2 [256][256], W2^T [256][256]
    int *ftnext = nullptr;            // Adam step of the pending update (device)
};

int64_t mlp_param_count(int in, int hidden);
inline int64_t mlp_workspace_floats(int in, int hidden) {
    return 16 * (int64_t)hidden * (hidden > in ? hidden : in);
}
// Canonical features of n vectors (FP64, 2k doubles each) into X [n][2k] FP32.
hipError_t mlp_features(const double *V, int64_t n, int k, float *X, hipStream_t s);
// Targets ln(1 + NLL - min NLL) (one block).
hipError_t mlp_targets(const double *nll, int64_t n, float *t, hipStream_t s);
// Forward pass over B rows of Xb into y; with train, the loss (hist[*m.batch]
// too when hist is set) and the gradient of the summed squared error into m.G.
hipError_t mlp_pass(const MlpBuffers &m, int B, const float *Xb, const float *tb, float *y, bool train, float *hist,
                    hipStream_t s);
hipError_t mlp_scale(const float *x, int64_t n, float scale, float *out, hipStream_t s);
// Fused training pass (mlp_fused.hip), hidden width 256 and in <= 128 only: per
// slice of 16 rows (X rows perm[*m.batch B + r] when perm is set, else rows
// 0 .. B-1) the forward pass, loss and activation gradients, then the weight
// gradients over the whole mini-batch into m.G and m.loss (hist[*m.batch] too
// when set); with adam, Adam on m.P with m.G * gscale at step *m.step + 1
// instead of writing m.G, and *m.step, *m.batch advanced.
bool mlp_fused_ok(const MlpBuffers &m);
int mlp_fused_slices(int B);
size_t mlp_fused_wh_halfs();
size_t mlp_fused_act_halfs(int max_batch);
size_t mlp_fused_vec_floats(int max_batch);
// fp16 copies of the current weights for the fused pass (after any change of m.P
// other than the fused pass's own Adam steps)
hipError_t mlp_fused_weights(const MlpBuffers &m, hipStream_t s);
hipError_t mlp_fused_pass(const MlpBuffers &m, int B, const float *X, const float *t, const int *perm, int64_t n,
                          bool adam, float gscale, float lr, float *hist, hipStream_t s);
// Adam on m.P with gradient m.G * gscale; step count at m.step (not advanced here).
hipError_t mlp_adam(const MlpBuffers &m, float gscale, float lr, hipStream_t s);
// Rows perm[*m.batch * B + r] of X [n][in] and t into m.Xb, m.tb (*m.bad set
// for an index outside [0, n)).
hipError_t mlp_gather(const MlpBuffers &m, const float *X, const float *t, int64_t n, const int *perm, int B,
                      hipStream_t s);
hipError_t mlp_step_inc(const MlpBuffers &m, hipStream_t s);
hipError_t mlp_set_int(int *p, int v, hipStream_t s);
// Indices of the k smallest keys (ties by index; NaN counts as +inf), ascending.
int topk_chunk();
size_t topk_scratch(int64_t n, int k);
hipError_t mlp_topk(const float *keys, int64_t n, int k, float *sk[2], int *si[2], int *out, hipStream_t s);

}  // namespace pwa
