/*
 * FP64 reference (oracle) for the unbinned partial-wave likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header or constant with it.
 *
 * What it computes (Berger, "Partial Wave Analysis using Graphics Cards",
 * Section 2):
 *   Eq. 1   I(Omega) = | sum_a V_a A_a(Omega) |^2
 *   Eq. 2   L ~ prod_i I(Omega_i) / integral(eps I), the integral estimated by
 *           the MC sum S = (1/N_gen) sum_{accepted j} w_j I(Omega_j)
 *           (footnote on weighted MC; accepted-events remark), so
 *           NLL = -sum_i ln I_i + N_D ln S                (Eq. 2 form)
 *   Eq. 3   the expanded form with a linear normalisation term:
 *           NLL_ext = -sum_i ln I_i + S                     (Eq. 3 form)
 *   The bracket of Eq. 3 (the MC integral matrix) can be precomputed when
 *   only V varies:  M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb,  S = V^H M V.
 *
 * Gradient convention (minimisers see only real parameters, Section 4, "Fits
 * with complex parameters"): grad[2a] = dNLL/dRe V_a, grad[2a+1] = dNLL/dIm V_a.
 * With the Wirtinger derivative g_a = dNLL/d conj(V_a) this is (2 Re g_a, 2 Im g_a).
 *   g_a = - sum_i conj(A_ia) z_i / I_i + c * sum_j w_j conj(A_ja) z_j
 *   with c = N_D / (N_gen S) (Eq. 2 form) or c = 1 / N_gen (Eq. 3 form).
 *
 * Arithmetic: plain double loops; every sum over events is a Neumaier
 * (compensated) sum in event order (the paper stresses that the final sum is
 * in double precision and that the summation algorithm matters).  The
 * chunked form (orc_nll_grad_chunked) cuts the events into fixed chunks,
 * sums each chunk in event order and adds the chunk sums in chunk order, so
 * its result does not depend on how many threads run the chunks.
 *
 * Layout: complex arrays are interleaved (re, im) doubles; an event row holds
 * k complex values starting at row * ld complex (ld >= k).
 *
 * Return value of every function: 0 on success, -1 on invalid arguments.
 * NLL is +inf when some data intensity is not positive, or (Eq. 2 form) S is
 * not positive.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
static int omp_default_threads(void) { return omp_get_max_threads(); }
#else
static int omp_default_threads(void) { return 1; }
#endif

typedef struct { double s, c; } nsum;   /* Neumaier accumulator */

static void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* z = sum_a V_a A_a for one event row (Eq. 1 inner sum). */
static void coherent_sum(const double *row, const double *V, int32_t k, double *zr, double *zi) {
    double r = 0.0, i = 0.0;
    for (int32_t a = 0; a < k; ++a) {
        double ar = row[2 * a], ai = row[2 * a + 1];
        double vr = V[2 * a], vi = V[2 * a + 1];
        r += vr * ar - vi * ai;
        i += vr * ai + vi * ar;
    }
    *zr = r;
    *zi = i;
}

/* Eq. 1 for every row: I[i] = |sum_a V_a A_ia|^2. */
int orc_intensity(int64_t n, int32_t k, const double *A, int64_t ld, const double *V, double *I) {
    if (n < 0 || k < 1 || ld < k || (n > 0 && (!A || !I)) || !V) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double zr, zi;
        coherent_sum(A + 2 * ld * i, V, k, &zr, &zi);
        I[i] = zr * zr + zi * zi;
    }
    return 0;
}

/* Raw sums over a sample.
 *   data (weights NULL, log_term = 1): T = sum ln I_i,      G_a = sum conj(A_ia) z_i / I_i
 *   MC   (log_term = 0):               T = sum w_j I_j,     G_a = sum w_j conj(A_ja) z_j
 * G is interleaved complex [k].  Returns 1 if a data intensity is <= 0 or not finite. */
static int raw_sums(int64_t n, int32_t k, const double *A, int64_t ld, const double *w,
                    const double *V, int log_term, double *T, double *G) {
    nsum t = {0.0, 0.0};
    nsum *g = (nsum *)calloc((size_t)(2 * k), sizeof(nsum));
    int bad = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double *row = A + 2 * ld * i;
        double zr, zi;
        coherent_sum(row, V, k, &zr, &zi);
        double I = zr * zr + zi * zi;
        double ur, ui;          /* per-event factor multiplying conj(A) */
        if (log_term) {
            if (!(I > 0.0) || !isfinite(I)) bad = 1;
            nadd(&t, log(I));
            ur = zr / I;
            ui = zi / I;
        } else {
            double wj = w ? w[i] : 1.0;
            nadd(&t, wj * I);
            ur = wj * zr;
            ui = wj * zi;
        }
        for (int32_t a = 0; a < k; ++a) {
            double ar = row[2 * a], ai = row[2 * a + 1];
            /* conj(A) * u = (ar - i ai)(ur + i ui) */
            nadd(&g[2 * a], ar * ur + ai * ui);
            nadd(&g[2 * a + 1], ar * ui - ai * ur);
        }
    }
    *T = nval(&t);
    for (int32_t a = 0; a < 2 * k; ++a) G[a] = nval(&g[a]);
    free(g);
    return bad;
}

/* Final combination of the raw sums into NLL and the real gradient.
 *   sum_log = sum_i ln I_i, GD = sum_i conj(A_i) z_i/I_i,
 *   s_raw = sum_j w_j I_j,  HM = sum_j w_j conj(A_j) z_j.
 * The Gram form passes n_gen = 1, s_raw = V^H M V and HM = M V. */
static void combine(int64_t nd, double n_gen, int32_t k, int extended,
                    double sum_log, const double *GD, double s_raw, const double *HM,
                    int bad, double *nll, double *grad) {
    double S = s_raw / n_gen;
    double c;
    if (nd == 0 && !extended) {
        *nll = 0.0;
        if (grad) for (int32_t a = 0; a < 2 * k; ++a) grad[a] = 0.0;
        return;
    }
    if (extended) {
        *nll = -sum_log + S;
        c = 1.0 / n_gen;
    } else {
        *nll = -sum_log + (double)nd * log(S);
        c = (double)nd / s_raw;
    }
    if (bad || (!extended && !(S > 0.0)) || !isfinite(*nll)) *nll = INFINITY;
    if (grad)
        for (int32_t a = 0; a < 2 * k; ++a) grad[a] = 2.0 * (-GD[a] + c * HM[a]);
}

/* NLL and gradient by streaming both samples.
 * parts (optional, 2 + 4k doubles): sum_log, s_raw, GD[2k], HM[2k]. */
int orc_nll_grad(int64_t nd, const double *Ad, int64_t ldd,
                 int64_t nm, const double *Am, int64_t ldm, const double *w, double n_gen,
                 int32_t k, const double *V, int extended,
                 double *nll, double *grad, double *parts) {
    if (k < 1 || nd < 0 || nm < 0 || ldd < k || ldm < k || !V || !nll) return -1;
    if ((nd > 0 && !Ad) || (nm > 0 && !Am)) return -1;
    if (nd > 0 && nm == 0) return -1;
    if (n_gen <= 0.0) n_gen = nm > 0 ? (double)nm : 1.0;
    double *GD = (double *)calloc((size_t)(4 * k), sizeof(double));
    double *HM = GD + 2 * k;
    double sum_log = 0.0, s_raw = 0.0;
    int bad = raw_sums(nd, k, Ad, ldd, NULL, V, 1, &sum_log, GD);
    raw_sums(nm, k, Am, ldm, w, V, 0, &s_raw, HM);
    combine(nd, n_gen, k, extended, sum_log, GD, s_raw, HM, bad, nll, grad);
    if (parts) {
        parts[0] = sum_log;
        parts[1] = s_raw;
        for (int32_t a = 0; a < 2 * k; ++a) { parts[2 + a] = GD[a]; parts[2 + 2 * k + a] = HM[a]; }
    }
    free(GD);
    return 0;
}

/* MC integral matrix of the Eq. 3 bracket: M_ab = (1/N_gen) sum_j w_j conj(A_ja) A_jb.
 * M is k x k interleaved complex, row a, column b. */
int orc_gram(int64_t nm, const double *Am, int64_t ldm, const double *w, double n_gen,
             int32_t k, double *M) {
    if (k < 1 || nm < 0 || ldm < k || (nm > 0 && !Am) || !M) return -1;
    if (n_gen <= 0.0) n_gen = nm > 0 ? (double)nm : 1.0;
    nsum *acc = (nsum *)calloc((size_t)(2 * k * k), sizeof(nsum));
    for (int64_t j = 0; j < nm; ++j) {
        const double *row = Am + 2 * ldm * j;
        double wj = w ? w[j] : 1.0;
        for (int32_t a = 0; a < k; ++a)
            for (int32_t b = 0; b < k; ++b) {
                double ar = row[2 * a], ai = row[2 * a + 1];
                double br = row[2 * b], bi = row[2 * b + 1];
                /* conj(A_a) A_b = (ar - i ai)(br + i bi) */
                nadd(&acc[2 * (a * k + b)], wj * (ar * br + ai * bi));
                nadd(&acc[2 * (a * k + b) + 1], wj * (ar * bi - ai * br));
            }
    }
    for (int32_t e = 0; e < 2 * k * k; ++e) M[e] = (nm > 0) ? nval(&acc[e]) / n_gen : 0.0;
    free(acc);
    return 0;
}

/* NLL and gradient with the precomputed MC matrix M: S = V^H M V, MC term of g = c N_gen (M V). */
int orc_nll_grad_gram(int64_t nd, const double *Ad, int64_t ldd, int32_t k, const double *M,
                      const double *V, int extended, double *nll, double *grad) {
    if (k < 1 || nd < 0 || ldd < k || (nd > 0 && !Ad) || !M || !V || !nll) return -1;
    double *GD = (double *)calloc((size_t)(4 * k), sizeof(double));
    double *MV = GD + 2 * k;
    double sum_log = 0.0;
    int bad = raw_sums(nd, k, Ad, ldd, NULL, V, 1, &sum_log, GD);
    double Sr = 0.0, Si = 0.0;
    for (int32_t a = 0; a < k; ++a) {
        double r = 0.0, i = 0.0;
        for (int32_t b = 0; b < k; ++b) {
            double mr = M[2 * (a * k + b)], mi = M[2 * (a * k + b) + 1];
            double vr = V[2 * b], vi = V[2 * b + 1];
            r += mr * vr - mi * vi;
            i += mr * vi + mi * vr;
        }
        MV[2 * a] = r;
        MV[2 * a + 1] = i;
        /* conj(V_a) (M V)_a */
        Sr += V[2 * a] * r + V[2 * a + 1] * i;
        Si += V[2 * a] * i - V[2 * a + 1] * r;
    }
    (void)Si;   /* zero up to rounding: M is Hermitian */
    /* With N_gen = 1 the raw MC quantities are S and M V themselves. */
    combine(nd, 1.0, k, extended, sum_log, GD, Sr, MV, bad, nll, grad);
    free(GD);
    return 0;
}

/* Rows per chunk of the chunked form. */
#define ORC_CHUNK 65536

/* Raw sums of one sample in chunks: chunk c holds rows [c ORC_CHUNK,
 * (c + 1) ORC_CHUNK); each chunk's sums are raw_sums in row order, and the
 * chunk sums are added in chunk order with Neumaier sums.  The chunks run on
 * up to nthreads OpenMP threads; the order of every addition is fixed by the
 * chunk layout alone.  Returns 1 if some data intensity is bad (as raw_sums). */
static int raw_sums_chunked(int64_t n, int32_t k, const double *A, int64_t ld, const double *w,
                            const double *V, int log_term, int nthreads, double *T, double *G) {
    const int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *ct = (double *)calloc((size_t)(nch > 0 ? nch : 1), sizeof(double));
    double *cg = (double *)calloc((size_t)(nch > 0 ? nch : 1) * (size_t)(2 * k), sizeof(double));
    int *cb = (int *)calloc((size_t)(nch > 0 ? nch : 1), sizeof(int));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t c = 0; c < nch; ++c) {
        const int64_t r0 = c * ORC_CHUNK;
        const int64_t m = n - r0 < ORC_CHUNK ? n - r0 : ORC_CHUNK;
        cb[c] = raw_sums(m, k, A + 2 * ld * r0, ld, w ? w + r0 : NULL, V, log_term, &ct[c], &cg[c * 2 * k]);
    }
    nsum t = {0.0, 0.0};
    nsum *g = (nsum *)calloc((size_t)(2 * k), sizeof(nsum));
    int bad = 0;
    for (int64_t c = 0; c < nch; ++c) {
        nadd(&t, ct[c]);
        for (int32_t a = 0; a < 2 * k; ++a) nadd(&g[a], cg[c * 2 * k + a]);
        bad |= cb[c];
    }
    *T = nval(&t);
    for (int32_t a = 0; a < 2 * k; ++a) G[a] = nval(&g[a]);
    free(g);
    free(cb);
    free(cg);
    free(ct);
    return bad;
}

/* orc_nll_grad on up to nthreads threads (<= 0: the OpenMP default) with the
 * chunked sums above.  Same arguments and outputs as orc_nll_grad. */
int orc_nll_grad_chunked(int64_t nd, const double *Ad, int64_t ldd,
                         int64_t nm, const double *Am, int64_t ldm, const double *w, double n_gen,
                         int32_t k, const double *V, int extended, int nthreads,
                         double *nll, double *grad, double *parts) {
    if (k < 1 || nd < 0 || nm < 0 || ldd < k || ldm < k || !V || !nll) return -1;
    if ((nd > 0 && !Ad) || (nm > 0 && !Am)) return -1;
    if (nd > 0 && nm == 0) return -1;
    if (n_gen <= 0.0) n_gen = nm > 0 ? (double)nm : 1.0;
    if (nthreads <= 0) nthreads = omp_default_threads();
    double *GD = (double *)calloc((size_t)(4 * k), sizeof(double));
    double *HM = GD + 2 * k;
    double sum_log = 0.0, s_raw = 0.0;
    int bad = raw_sums_chunked(nd, k, Ad, ldd, NULL, V, 1, nthreads, &sum_log, GD);
    raw_sums_chunked(nm, k, Am, ldm, w, V, 0, nthreads, &s_raw, HM);
    combine(nd, n_gen, k, extended, sum_log, GD, s_raw, HM, bad, nll, grad);
    if (parts) {
        parts[0] = sum_log;
        parts[1] = s_raw;
        for (int32_t a = 0; a < 2 * k; ++a) { parts[2 + a] = GD[a]; parts[2 + 2 * k + a] = HM[a]; }
    }
    free(GD);
    return 0;
}
