/* Drives every entry of the FP64 oracle on a small problem, for a build
 * with the address and undefined-behaviour sanitizers: any out-of-bounds
 * access, use after free, leak or undefined operation ends the run with a
 * sanitizer report and a non-zero status.  Inputs are made here (two
 * continua and a line, a pseudo-random response); the checks are that
 * every result is finite and the gradient matches central differences. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct or_ctx or_ctx;
or_ctx* or_create(void);
void or_destroy(or_ctx* c);
void or_set_physics(or_ctx* c, double me, double gf, double sw2, double alpha, double tau_frac);
int or_add_source(or_ctx* c, int kind, int n, const double* E, const double* w,
                  const double* pee, int group);
int or_set_grid(or_ctx* c, int n_t, double t_lo, double t_hi);
int or_set_response(or_ctx* c, const float* R, int n_t, int n_reco, const double* m,
                    double n_sig);
int or_set_data(or_ctx* c, const double* n, const double* b, int n_reco,
                const double* pull_mean, const double* pull_sigma);
double or_dsigma(const or_ctx* c, int a, double E, double T, const double* th);
int or_spectrum(const or_ctx* c, const double* th, double* S);
int or_weights(const or_ctx* c, const double* th, double* w);
int or_row_factors(const or_ctx* c, double* m);
int or_mu(const or_ctx* c, const double* th, double* mu);
double or_nll(const or_ctx* c, const double* th);
double or_nll_grad(const or_ctx* c, const double* th, double* grad);

static unsigned long long lcg = 12345;
static double urand(void) {
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

int main(void) {
    enum { NT = 48, NR = 20, NE = 16 };
    or_ctx* c = or_create();
    or_set_physics(c, 0.51099895, 1.1663788e-11, 0.23122, 1.0 / 137.035999084, 0.5);
    double E[NE], w[NE], p[NE];
    for (int s = 0; s < 2; ++s) {
        const double e0 = s ? 16.0 : 1.73;
        for (int j = 0; j < NE; ++j) {
            E[j] = (j + 0.5) * e0 / NE;
            w[j] = 1.0 + j;
            p[j] = 0.32 + 0.23 / (1.0 + (E[j] / 2.0) * (E[j] / 2.0));
        }
        if (or_add_source(c, 1, NE, E, w, p, s)) return 1;
    }
    const double El = 0.862, wl = 5.0, pl = 0.55;
    if (or_add_source(c, 0, 1, &El, &wl, &pl, 0)) return 1;
    if (or_set_grid(c, NT, 0.0, 16.0)) return 1;
    float* R = (float*)malloc(sizeof(float) * NT * NR);
    for (int i = 0; i < NT * NR; ++i) R[i] = (float)(urand() / NR);
    if (or_set_response(c, R, NT, NR, NULL, 1.0e4)) return 1;
    free(R);
    double n[NR], b[NR], pm[7] = {0, 0, 0, 0, 0, 1, 1}, ps[7] = {0, 0, 0, 0, 0, 0.1, 0.1};
    for (int j = 0; j < NR; ++j) {
        b[j] = 10.0;
        n[j] = (j % 5 == 0) ? 0.0 : floor(200.0 * urand());
    }
    if (or_set_data(c, n, b, NR, pm, ps)) return 1;
    const double th[7] = {0.1, -0.2, 0.3, 0.05, 3.0, 1.1, 0.9};
    double S[NT], wt[NT], m[NT], mu[NR], g[7];
    if (or_spectrum(c, th, S) || or_weights(c, th, wt) || or_row_factors(c, m) ||
        or_mu(c, th, mu))
        return 1;
    for (int l = 0; l < NT; ++l)
        if (!isfinite(S[l]) || !isfinite(wt[l]) || !isfinite(m[l])) return 3;
    for (int j = 0; j < NR; ++j)
        if (!isfinite(mu[j])) return 3;
    const double v = or_nll_grad(c, th, g);
    if (!isfinite(v) || fabs(v - or_nll(c, th)) > 1e-9 * fabs(v)) return 4;
    for (int i = 0; i < 7; ++i) {
        double tp[7], tm[7];
        for (int k = 0; k < 7; ++k) tp[k] = tm[k] = th[k];
        tp[i] += 1e-5;
        tm[i] -= 1e-5;
        const double fd = (or_nll(c, tp) - or_nll(c, tm)) / 2e-5;
        if (fabs(fd - g[i]) > 1e-4 * fabs(g[i]) + 1e-4) {
            fprintf(stderr, "grad %d: %g vs %g\n", i, g[i], fd);
            return 5;
        }
    }
    if (!isfinite(or_dsigma(c, 0, 1.0, 0.5, th))) return 3;
    or_destroy(c);
    printf("oracle checked run: nll %.6f\n", v);
    return 0;
}
