/*
 * FP64 CPU oracle for the spectrum-reweighting likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so the HIP path can be checked against a plain,
 * slow, obviously correct implementation written straight from the paper
 * (arXiv:2607.00488).  It shares no source, header, table or constant with
 * the HIP path.
 *
 * Every step follows the paper's definition directly, in double precision,
 * with no blocking, fusion or algebraic regrouping:
 *
 *   couplings          Sec. II.A (tree-level chiral couplings)
 *   NSI shift          Sec. II.B, Eqs. (g_tilde), (xs_nsi)
 *   weak dsigma/dT     Sec. II.A, Eq. (sm_cross_section)
 *   magnetic moment    Sec. II.C, Eqs. (xs_mm), (xs_total)
 *   recoil spectrum    Sec. III.A, Eq. (fT), flavour sum as in Eq. (rate_sm)
 *   weights            Sec. III.A, Eqs. (fT_norm), (reweight_factor)
 *   fold               Sec. III.B, Eqs. (Rij), (fNp_reweight); Sec. III.C,
 *                      Eq. (mu_total)
 *   likelihood         Sec. III.C, Eq. (logL)
 *
 * Readings taken where the paper is silent (each is listed with its reason
 * in the design notes of the repository):
 *   - physical constants m_e, G_F, sin^2(theta_W) (tree level), alpha_em;
 *   - the kinematic limit T <= T_max(E) = 2E^2/(m_e+2E) (two-body
 *     kinematics; not written in the paper), ties included;
 *   - nu_mu / nu_tau share of 1-P_ee split by tau_frac (default 1/2);
 *   - the representative recoil energy of bin l is its centre;
 *   - w_l := 1 where the SM spectrum is zero;
 *   - unnormalised weights: rate_k carries the integrated cross section, so
 *     the 1/sum_l f_T prefactor of Eq. (fNp_reweight) cancels and
 *     mu_j = f_bkg b_j + sum_l m_l R_lj w_l with m_l = N_sig * fhat_SM(l)
 *     (the joint response of Eq. (Rij) written as the conditional response
 *     times the normalised SM reference) unless the caller gives m;
 *   - the magnetic moment enters as m2 = (mu_nu / 1e-11 mu_B)^2.
 *
 * Parameter vector: theta = [eps_eL, eps_eR, eps_tauL, eps_tauR, m2, f_8B,
 * f_bkg]; eps_mumu = 0.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NTH 7
#define OR_MAXSRC 32

typedef struct {
    int kind, n, group;
    double *E, *w, *pee;
} or_src;

typedef struct {
    double me, gf, sw2, alpha, tau_frac;
    int n_src;
    or_src src[OR_MAXSRC];
    int n_t;
    double t_lo, t_hi;
    int n_reco;
    float *R;        /* [n_t][n_reco] as given */
    double *m;       /* caller-given row factors, or NULL */
    double n_sig;
    double *n, *b;   /* [n_reco] */
    double pull_mean[OR_NTH], pull_sigma[OR_NTH];
} or_ctx;

or_ctx *or_create(void)
{
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    if (!c) return NULL;
    c->me = 0.51099895;          /* MeV */
    c->gf = 1.1663788e-11;       /* MeV^-2 */
    c->sw2 = 0.23122;            /* tree-level weak mixing */
    c->alpha = 1.0 / 137.035999084;
    c->tau_frac = 0.5;
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    for (int k = 0; k < c->n_src; ++k) {
        free(c->src[k].E); free(c->src[k].w); free(c->src[k].pee);
    }
    free(c->R); free(c->m); free(c->n); free(c->b);
    free(c);
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_physics(or_ctx *c, double me, double gf, double sw2, double alpha,
                    double tau_frac)
{
    c->me = me; c->gf = gf; c->sw2 = sw2; c->alpha = alpha;
    c->tau_frac = tau_frac;
}

static double *dup_d(const double *p, int n)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (q) memcpy(q, p, sizeof(double) * (size_t)n);
    return q;
}

int or_add_source(or_ctx *c, int kind, int n, const double *E, const double *w,
                  const double *pee, int group)
{
    if (c->n_src >= OR_MAXSRC || n <= 0) return -1;
    or_src *s = &c->src[c->n_src++];
    s->kind = kind; s->n = n; s->group = group;
    s->E = dup_d(E, n); s->w = dup_d(w, n); s->pee = dup_d(pee, n);
    return 0;
}

int or_set_grid(or_ctx *c, int n_t, double t_lo, double t_hi)
{
    if (n_t <= 0 || !(t_hi > t_lo)) return -1;
    c->n_t = n_t; c->t_lo = t_lo; c->t_hi = t_hi;
    return 0;
}

int or_set_response(or_ctx *c, const float *R, int n_t, int n_reco,
                    const double *m, double n_sig)
{
    if (n_t != c->n_t || n_reco <= 0) return -1;
    free(c->R); free(c->m);
    size_t sz = (size_t)n_t * (size_t)n_reco;
    c->R = (float *)malloc(sizeof(float) * sz);
    if (!c->R) return -4;
    memcpy(c->R, R, sizeof(float) * sz);
    c->m = m ? dup_d(m, n_t) : NULL;
    c->n_sig = n_sig;
    c->n_reco = n_reco;
    return 0;
}

int or_set_data(or_ctx *c, const double *n, const double *b, int n_reco,
                const double *pull_mean, const double *pull_sigma)
{
    if (n_reco != c->n_reco) return -1;
    free(c->n); free(c->b);
    c->n = dup_d(n, n_reco);
    c->b = dup_d(b, n_reco);
    for (int i = 0; i < OR_NTH; ++i) {
        c->pull_mean[i] = pull_mean ? pull_mean[i] : 0.0;
        c->pull_sigma[i] = pull_sigma ? pull_sigma[i] : 0.0;
    }
    return 0;
}

/* Recoil-bin centre: the representative energy of bin l. */
static double t_centre(const or_ctx *c, int l)
{
    return c->t_lo + (l + 0.5) * (c->t_hi - c->t_lo) / c->n_t;
}

/* Chiral couplings of flavour a (0 = e, 1 = mu, 2 = tau) after the NSI
 * shift of Eq. (g_tilde); eps_mumu = 0. */
static void couplings(const or_ctx *c, int a, const double *th, double *gl,
                      double *gr)
{
    double gL = (a == 0 ? 0.5 : -0.5) + c->sw2;
    double gR = c->sw2;
    if (a == 0) { gL += th[0]; gR += th[1]; }
    if (a == 2) { gL += th[2]; gR += th[3]; }
    *gl = gL; *gr = gR;
}

/* Eq. (sm_cross_section) with the couplings of Eq. (xs_nsi), plus the
 * magnetic-moment term of Eq. (xs_mm) summed incoherently as in
 * Eq. (xs_total).  Natural units, MeV^-3.  No kinematic cut here. */
double or_dsigma(const or_ctx *c, int a, double E, double T, const double *th)
{
    const double pi = 3.14159265358979323846;
    double gl, gr;
    couplings(c, a, th, &gl, &gr);
    double pref = 2.0 * c->gf * c->gf * c->me / pi;
    double weak = pref * (gl * gl + gr * gr * (1.0 - T / E) * (1.0 - T / E)
                          - gl * gr * c->me * T / (E * E));
    double mu2 = th[4] * 1e-22;                  /* (mu_nu/mu_B)^2 */
    double mm = pi * c->alpha * c->alpha / (c->me * c->me) * mu2
                * (1.0 / T - 1.0 / E);
    return weak + mm;
}

/* Two-body kinematics: a recoil T is reachable from E iff T <= T_max(E). */
static int reachable(const or_ctx *c, double E, double T)
{
    return T <= 2.0 * E * E / (c->me + 2.0 * E);
}

/* Eq. (fT) for one recoil bin: sum over sources k and nodes j of
 * f_k * weight_kj * sum_a P_a(E_j) dsigma_a/dT(E_j, T_l).  Optionally also
 * the six derivatives d/d(eps_eL, eps_eR, eps_tauL, eps_tauR, m2, f_8B). */
static double spectrum_bin(const or_ctx *c, const double *th, int l, double *d)
{
    const double pi = 3.14159265358979323846;
    double T = t_centre(c, l);
    double S = 0.0;
    double pref = 2.0 * c->gf * c->gf * c->me / pi;
    double kmm = pi * c->alpha * c->alpha / (c->me * c->me) * 1e-22;
    if (d) for (int i = 0; i < 6; ++i) d[i] = 0.0;
    for (int k = 0; k < c->n_src; ++k) {
        const or_src *s = &c->src[k];
        double f = s->group == 1 ? th[5] : 1.0;
        for (int j = 0; j < s->n; ++j) {
            double E = s->E[j];
            if (!reachable(c, E, T)) continue;
            double P[3];
            P[0] = s->pee[j];
            P[1] = (1.0 - s->pee[j]) * (1.0 - c->tau_frac);
            P[2] = (1.0 - s->pee[j]) * c->tau_frac;
            double val = 0.0;
            for (int a = 0; a < 3; ++a) val += P[a] * or_dsigma(c, a, E, T, th);
            S += f * s->w[j] * val;
            if (d) {
                double y = 1.0 - T / E, x = c->me * T / (E * E);
                double gl, gr;
                couplings(c, 0, th, &gl, &gr);
                d[0] += f * s->w[j] * P[0] * pref * (2.0 * gl - gr * x);
                d[1] += f * s->w[j] * P[0] * pref * (2.0 * gr * y * y - gl * x);
                couplings(c, 2, th, &gl, &gr);
                d[2] += f * s->w[j] * P[2] * pref * (2.0 * gl - gr * x);
                d[3] += f * s->w[j] * P[2] * pref * (2.0 * gr * y * y - gl * x);
                d[4] += f * s->w[j] * (P[0] + P[1] + P[2]) * kmm
                        * (1.0 / T - 1.0 / E);
                if (s->group == 1) d[5] += s->w[j] * val;
            }
        }
    }
    return S;
}

int or_spectrum(const or_ctx *c, const double *th, double *S)
{
    if (c->n_t <= 0 || c->n_src <= 0) return -2;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int l = 0; l < c->n_t; ++l) S[l] = spectrum_bin(c, th, l, NULL);
    return 0;
}

static const double TH_SM[OR_NTH] = {0, 0, 0, 0, 0, 1, 1};

/* Eqs. (fT_norm), (reweight_factor): w_l = S_theta(T_l) / S_SM(T_l). */
int or_weights(const or_ctx *c, const double *th, double *w)
{
    if (c->n_t <= 0 || c->n_src <= 0) return -2;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int l = 0; l < c->n_t; ++l) {
        double ssm = spectrum_bin(c, TH_SM, l, NULL);
        w[l] = ssm > 0.0 ? spectrum_bin(c, th, l, NULL) / ssm : 1.0;
    }
    return 0;
}

/* The row factors m_l of the fold: the caller's, or N_sig * fhat_SM(l). */
int or_row_factors(const or_ctx *c, double *m)
{
    if (c->n_t <= 0 || !c->R) return -2;
    if (c->m) { memcpy(m, c->m, sizeof(double) * (size_t)c->n_t); return 0; }
    double tot = 0.0;
    or_spectrum(c, TH_SM, m);
    for (int l = 0; l < c->n_t; ++l) tot += m[l];
    for (int l = 0; l < c->n_t; ++l) m[l] = c->n_sig * m[l] / tot;
    return 0;
}

/* Fold of a per-bin vector v through the response:
 * out_j = sum_l m_l R_lj v_l  (Eqs. (fNp_reweight), (mu_total)). */
static void fold(const or_ctx *c, const double *m, const double *v, double *out)
{
    int nr = c->n_reco;
    #pragma omp parallel for schedule(static)
    for (int j = 0; j < nr; ++j) {
        double acc = 0.0;
        for (int l = 0; l < c->n_t; ++l)
            acc += m[l] * (double)c->R[(size_t)l * nr + j] * v[l];
        out[j] = acc;
    }
}

int or_mu(const or_ctx *c, const double *th, double *mu)
{
    if (c->n_t <= 0 || c->n_src <= 0 || !c->R) return -2;
    double *w = (double *)malloc(sizeof(double) * (size_t)c->n_t);
    double *m = (double *)malloc(sizeof(double) * (size_t)c->n_t);
    or_weights(c, th, w);
    or_row_factors(c, m);
    fold(c, m, w, mu);
    for (int j = 0; j < c->n_reco; ++j) mu[j] += th[6] * (c->b ? c->b[j] : 0.0);
    free(w); free(m);
    return 0;
}

/* Eq. (logL) for an expected spectrum mu. */
static double nll_of(const or_ctx *c, const double *th, const double *mu)
{
    double s = 0.0;
    for (int j = 0; j < c->n_reco; ++j) {
        double n = c->n[j];
        if (n > 0.0 && !(mu[j] > 0.0)) return INFINITY;
        double t = mu[j] + lgamma(n + 1.0);
        if (n > 0.0) t -= n * log(mu[j]);
        s += t;
    }
    s *= 2.0;
    for (int i = 0; i < OR_NTH; ++i)
        if (c->pull_sigma[i] > 0.0) {
            double z = (th[i] - c->pull_mean[i]) / c->pull_sigma[i];
            s += z * z;
        }
    return s;
}

double or_nll(const or_ctx *c, const double *th)
{
    if (!c->n || !c->R || c->n_src <= 0) return NAN;
    double *mu = (double *)malloc(sizeof(double) * (size_t)c->n_reco);
    or_mu(c, th, mu);
    double r = nll_of(c, th, mu);
    free(mu);
    return r;
}

/* d(-2lnL)/d mu_j from Eq. (logL): the bin term is 2 (mu_j - n_j ln mu_j), so
 * the derivative is 2 (1 - n_j / mu_j); an empty bin (n_j = 0) contributes
 * 2 mu_j, whose derivative is 2 whatever mu_j is (also at mu_j = 0). */
static double dnll_dmu(double n, double mu)
{
    return n > 0.0 ? 2.0 * (1.0 - n / mu) : 2.0;
}

/* Analytic gradient of Eq. (logL): chain rule through mu_j (Eq. mu_total),
 * the fold, the weights and the spectrum derivatives. */
double or_nll_grad(const or_ctx *c, const double *th, double *grad)
{
    if (!c->n || !c->R || c->n_src <= 0) return NAN;
    int nt = c->n_t, nr = c->n_reco;
    double *dw = (double *)calloc((size_t)6 * nt, sizeof(double));
    double *w = (double *)malloc(sizeof(double) * (size_t)nt);
    double *m = (double *)malloc(sizeof(double) * (size_t)nt);
    double *mu = (double *)malloc(sizeof(double) * (size_t)nr);
    double *dmu = (double *)malloc(sizeof(double) * (size_t)nr);
    double *col = (double *)malloc(sizeof(double) * (size_t)nt);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int l = 0; l < nt; ++l) {
        double d[6];
        double ssm = spectrum_bin(c, TH_SM, l, NULL);
        double s = spectrum_bin(c, th, l, d);
        if (ssm > 0.0) {
            w[l] = s / ssm;
            for (int i = 0; i < 6; ++i) dw[(size_t)i * nt + l] = d[i] / ssm;
        } else {
            w[l] = 1.0;
        }
    }
    or_row_factors(c, m);
    fold(c, m, w, mu);
    for (int j = 0; j < nr; ++j) mu[j] += th[6] * c->b[j];
    double val = nll_of(c, th, mu);
    for (int i = 0; i < OR_NTH; ++i) grad[i] = 0.0;
    for (int i = 0; i < 6; ++i) {
        for (int l = 0; l < nt; ++l) col[l] = dw[(size_t)i * nt + l];
        fold(c, m, col, dmu);
        double g = 0.0;
        for (int j = 0; j < nr; ++j) g += dnll_dmu(c->n[j], mu[j]) * dmu[j];
        grad[i] = g;
    }
    {
        double g = 0.0;
        for (int j = 0; j < nr; ++j) g += dnll_dmu(c->n[j], mu[j]) * c->b[j];
        grad[6] = g;
    }
    for (int i = 0; i < OR_NTH; ++i)
        if (c->pull_sigma[i] > 0.0)
            grad[i] += 2.0 * (th[i] - c->pull_mean[i])
                       / (c->pull_sigma[i] * c->pull_sigma[i]);
    free(dw); free(w); free(m); free(mu); free(dmu); free(col);
    return val;
}
