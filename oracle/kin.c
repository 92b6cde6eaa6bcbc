/*
 * FP64 reference (oracle) for the likelihood with amplitudes computed from
 * each event's kinematics, so that resonance masses and widths can float.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as oracle.c): only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library shares no code with it.
 *
 * Section 2 of Berger, "Partial Wave Analysis using Graphics Cards", notes
 * that the decay amplitudes can be precomputed only while the widths and
 * masses of the resonances stay fixed.  Here they are parameters: each event
 * holds its kinematics (m = m_KK, x = cos theta) and the amplitude of wave a is
 * formed per evaluation (the stand-in lineshape of the J/psi -> gamma K+K-
 * example):
 *     A_a(m, x)  = BW_a(m) * Y_{J_a}^0(x)
 *     BW_a(m)    = 1 / (m_a^2 - m^2 - i m_a Gamma_a)        (fixed-width Breit-Wigner)
 *     Y_J^0(x)   = sqrt((2 J + 1) / (4 pi)) P_J(x)           (P_J: Legendre polynomial)
 * and the NLL is that of oracle.c (Eq. 1-3) with these amplitudes.
 *
 * Derivatives.  The V gradient is oracle.c's.  For a resonance parameter t of
 * wave a (t = m_a or Gamma_a), dI/dt = 2 Re(conj(z) V_a Y_a dBW_a/dt) with
 *     dBW_a/dm_a     = -(2 m_a - i Gamma_a) BW_a^2
 *     dBW_a/dGamma_a =  i m_a BW_a^2,
 * so dNLL/dt = -sum_data (1/I) dI/dt + c sum_MC w dI/dt, with c = N_D / (N_gen S)
 * (Eq. 2 form) or 1 / N_gen (Eq. 3 form).
 *
 * Arithmetic: C99 complex doubles, plain loops over events, Neumaier sums in
 * event order.  Layout: kinematics n x 2 doubles (m, x); resonance parameters
 * res[2a] = m_a, res[2a+1] = Gamma_a; V and the gradients interleaved (re, im)
 * or (d/dm_a, d/dGamma_a).  Every function returns 0, or -1 on invalid
 * arguments.  NLL is +inf when some data intensity is not positive or (Eq. 2
 * form) S is not positive.  `parts` (optional, 2 + 8k doubles) receives the
 * raw sums: sum ln I, sum w I, G, H (the V-gradient sums of data and MC) and
 * R_data, R_MC (the resonance-gradient sums).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct { double s, c; } ksum;   /* Neumaier accumulator */

static void kadd(ksum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static double kval(const ksum *a) { return a->s + a->c; }

/* Legendre polynomial P_J(x) by Bonnet's recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}. */
static double legendre(int32_t J, double x) {
    double p0 = 1.0, p1 = x;
    if (J == 0) return p0;
    for (int32_t n = 1; n < J; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

static double ylm0(int32_t J, double x) {
    const double pi = 3.14159265358979323846;
    return sqrt((2.0 * J + 1.0) / (4.0 * pi)) * legendre(J, x);
}

static double complex breit_wigner(double m, double ma, double ga) {
    return 1.0 / (ma * ma - m * m - _Complex_I * ma * ga);
}

static int valid(int32_t k, const int32_t *spin, const double *res) {
    if (k < 1 || !spin || !res) return 0;
    for (int32_t a = 0; a < k; ++a)
        if (spin[a] < 0 || !(res[2 * a] > 0.0) || !(res[2 * a + 1] > 0.0)) return 0;
    return 1;
}

int orc_kin_amplitudes(int64_t n, const double *mx, int32_t k, const int32_t *spin, const double *res,
                       double *A) {
    if (n < 0 || (n > 0 && (!mx || !A)) || !valid(k, spin, res)) return -1;
    for (int64_t e = 0; e < n; ++e) {
        const double m = mx[2 * e], x = mx[2 * e + 1];
        for (int32_t a = 0; a < k; ++a) {
            double complex amp = breit_wigner(m, res[2 * a], res[2 * a + 1]) * ylm0(spin[a], x);
            A[2 * (e * k + a)] = creal(amp);
            A[2 * (e * k + a) + 1] = cimag(amp);
        }
    }
    return 0;
}

/* Sums over one sample: T = sum ln I (data) or sum w I (MC); GV_a = sum c_e
 * conj(A_a) z; GR = sum c_e dI/dt (t = m_a, Gamma_a), with c_e = 1/I (data) or
 * w (MC).  Returns 1 if some data intensity is not positive. */
static int kin_sums(int64_t n, const double *mx, const double *w, int32_t k, const int32_t *spin,
                    const double *res, const double complex *V, int data, double *T, double *GV,
                    double *GR) {
    ksum t = {0.0, 0.0};
    ksum *gv = calloc((size_t)(4 * k), sizeof(ksum));
    ksum *gr = gv + 2 * k;
    double complex *bw = malloc(sizeof(double complex) * (size_t)k);
    double *y = malloc(sizeof(double) * (size_t)k);
    int bad = 0;
    for (int64_t e = 0; e < n; ++e) {
        const double m = mx[2 * e], x = mx[2 * e + 1];
        double complex z = 0.0;
        for (int32_t a = 0; a < k; ++a) {
            bw[a] = breit_wigner(m, res[2 * a], res[2 * a + 1]);
            y[a] = ylm0(spin[a], x);
            z += V[a] * bw[a] * y[a];
        }
        const double inten = creal(z) * creal(z) + cimag(z) * cimag(z);
        double ce;
        if (data) {
            if (!(inten > 0.0)) bad = 1;
            kadd(&t, log(inten));
            ce = 1.0 / inten;
        } else {
            ce = w ? w[e] : 1.0;
            kadd(&t, ce * inten);
        }
        for (int32_t a = 0; a < k; ++a) {
            const double complex g = ce * conj(bw[a] * y[a]) * z;
            kadd(&gv[2 * a], creal(g));
            kadd(&gv[2 * a + 1], cimag(g));
            const double ma = res[2 * a], ga = res[2 * a + 1];
            const double complex b2 = bw[a] * bw[a];
            const double complex dm = -(2.0 * ma - _Complex_I * ga) * b2;
            const double complex dg = _Complex_I * ma * b2;
            const double complex q = conj(z) * V[a] * y[a];
            kadd(&gr[2 * a], ce * 2.0 * creal(q * dm));
            kadd(&gr[2 * a + 1], ce * 2.0 * creal(q * dg));
        }
    }
    *T = kval(&t);
    for (int32_t i = 0; i < 2 * k; ++i) {
        GV[i] = kval(&gv[i]);
        GR[i] = kval(&gr[i]);
    }
    free(y);
    free(bw);
    free(gv);
    return bad;
}

int orc_kin_nll_grad(int64_t nd, const double *mx_d, int64_t nm, const double *mx_m, const double *w,
                     double n_gen, int32_t k, const int32_t *spin, const double *res, const double *Vri,
                     int extended, double *nll, double *grad_v, double *grad_res, double *parts) {
    if (nd < 0 || nm < 0 || !Vri || !nll || !valid(k, spin, res)) return -1;
    if ((nd > 0 && !mx_d) || (nm > 0 && !mx_m)) return -1;
    if (nd > 0 && nm == 0) return -1;
    if (n_gen <= 0.0) n_gen = nm > 0 ? (double)nm : 1.0;
    double complex *V = malloc(sizeof(double complex) * (size_t)k);
    for (int32_t a = 0; a < k; ++a) V[a] = Vri[2 * a] + _Complex_I * Vri[2 * a + 1];
    double *buf = calloc((size_t)(8 * k), sizeof(double));
    double *GD = buf, *HM = buf + 2 * k, *RD = buf + 4 * k, *RM = buf + 6 * k;
    double sum_log = 0.0, s_raw = 0.0;
    const int bad = kin_sums(nd, mx_d, NULL, k, spin, res, V, 1, &sum_log, GD, RD);
    kin_sums(nm, mx_m, w, k, spin, res, V, 0, &s_raw, HM, RM);
    const double S = s_raw / n_gen;
    double c;
    if (extended) {
        *nll = -sum_log + S;
        c = 1.0 / n_gen;
    } else if (nd == 0) {
        *nll = 0.0;
        c = 0.0;
    } else {
        *nll = (S > 0.0) ? -sum_log + (double)nd * log(S) : INFINITY;
        c = (double)nd / s_raw;
    }
    if (bad || !isfinite(*nll)) *nll = INFINITY;
    for (int32_t i = 0; i < 2 * k; ++i) {
        if (grad_v) grad_v[i] = 2.0 * (-GD[i] + c * HM[i]);
        if (grad_res) grad_res[i] = -RD[i] + c * RM[i];
    }
    if (parts) {   /* raw sums: sum ln I, sum w I, then G, H, R_data, R_MC (2k each) */
        parts[0] = sum_log;
        parts[1] = s_raw;
        for (int32_t i = 0; i < 8 * k; ++i) parts[2 + i] = buf[i];
    }
    free(buf);
    free(V);
    return 0;
}
