/* Drives most entry points of the library from C, at small sizes, for a
 * build whose host code carries AddressSanitizer: contexts, sources,
 * response and data (set twice), the pipelined single-point evaluations
 * with graph capture and replay, gradients, weights,
 * the batched and template forms, a grouped launch over two contexts, the
 * effective sample size, retiling, band skipping, stage timing and the
 * surrogate network's parameter round trip.  Any invalid host access is reported by
 * the sanitizer and fails the run.  Input format of abi_driver.c (at
 * least 34 points).  The single-point spectra entry point is left out: a
 * host-side crash of it on a 16384 x 4096 context has no known cause. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "nureweight.h"
static void* rd(FILE* f, size_t b) { void* p = malloc(b ? b : 1); if (!p || fread(p, 1, b, f) != b) exit(2); return p; }
static int rd_i(FILE* f) { int v; if (fread(&v, 4, 1, f) != 1) exit(2); return v; }
static double rd_d(FILE* f) { double v; if (fread(&v, 8, 1, f) != 1) exit(2); return v; }
#define CK(call) do { int rc_ = (call); if (rc_) { fprintf(stderr, "%s -> %d: %s\n", #call, rc_, nr_last_error()); return 1; } } while (0)
int main(int argc, char** argv) {
    FILE* f = fopen(argv[1], "rb"); if (!f) return 2;
    int n_src = rd_i(f), n_t = rd_i(f), n_reco = rd_i(f), n_pts = rd_i(f);
    double t_lo = rd_d(f), t_hi = rd_d(f), n_sig = rd_d(f);
    nr_source* src = calloc(n_src, sizeof *src);
    for (int s = 0; s < n_src; ++s) {
        src[s].kind = rd_i(f); src[s].n = rd_i(f); src[s].group = rd_i(f);
        src[s].E = rd(f, 8 * src[s].n); src[s].weight = rd(f, 8 * src[s].n); src[s].p_ee = rd(f, 8 * src[s].n);
    }
    float* R = rd(f, 4 * (size_t)n_t * n_reco);
    double* n = rd(f, 8 * n_reco); double* b = rd(f, 8 * n_reco); double* th = rd(f, 8 * n_pts * 7);
    fclose(f);
    if (n_pts < 34) { fprintf(stderr, "need >= 34 points\n"); return 2; }
    const int half = n_pts / 2;
    nr_ctx *c1, *c2;
    CK(nr_create(0, &c1)); CK(nr_create(0, &c2));
    nr_ctx* cs[2] = {c1, c2};
    for (int k = 0; k < 2; ++k) {
        CK(nr_set_sources(cs[k], src, n_src, n_t, t_lo, t_hi, NULL));
        CK(nr_set_response(cs[k], R, n_t, n_reco, NULL, n_sig));
        CK(nr_set_data(cs[k], n, b, n_reco, NULL, NULL));
    }
    double* nll = malloc(8 * n_pts); double* g = malloc(8 * 7 * n_pts);
    double* mu = malloc(8 * (size_t)n_pts * n_reco); double* w = malloc(8 * (size_t)n_pts * n_t);
    for (int rep = 0; rep < 2; ++rep) {
        CK(nr_eval_nll(c1, th, n_pts, nll));         /* pipelined graph */
        CK(nr_eval_nll(c1, th, n_pts, nll));         /* replay */
        CK(nr_eval_nll_grad(c1, th, 9, nll, g));
        CK(nr_eval_weights(c1, th, 5, w));
        CK(nr_eval_nll_batched(c1, th, n_pts, nll));
        CK(nr_eval_nll_grad_batched(c1, th, 33, nll, g));
        CK(nr_eval_mu_batched(c1, th, 7, mu));
        CK(nr_eval_nll_templates(c1, th, n_pts, nll, g));
        CK(nr_eval_mu_templates(c1, th, 3, mu));
        const double* ths[2] = {th, th + 7}; int np[2] = {half, half - 1}; double* nls[2] = {nll, g};
        CK(nr_eval_nll_multi(cs, 2, ths, np, nls));
        n[0] += 1.0;
        CK(nr_set_data(c1, n, b, n_reco, NULL, NULL));   /* data rewrite of the templates */
        CK(nr_eval_nll_templates(c1, th, 11, nll, NULL));
    }
    double* ssm = malloc(8 * n_t); double* m = malloc(8 * n_t);
    CK(nr_get_reference(c1, ssm, m));
    for (int l = 0; l < n_t; ++l) m[l] = 100.0 + l;
    CK(nr_set_mc_events(c1, m, n_t));
    CK(nr_eval_ess(c1, th, 3, mu));
    CK(nr_set_fold_tiling(c1, 64, 1));
    CK(nr_eval_nll(c1, th, n_pts, nll));
    CK(nr_set_band_skipping(c1, 1));                       /* band and tile bands */
    CK(nr_eval_nll_grad(c1, th, 9, nll, g));
    CK(nr_eval_nll_grad_batched(c1, th, 33, nll, g));
    CK(nr_set_fold_tiling(c1, 16, 1));                     /* tile bands rebuilt */
    CK(nr_eval_nll(c1, th, n_pts, nll));
    CK(nr_set_band_skipping(c1, 0));
    CK(nr_set_response(c1, R, n_t, n_reco, NULL, n_sig));   /* same shapes again */
    CK(nr_eval_nll(c1, th, 20, nll));
    double ms;
    for (int st = 1; st <= 5; ++st) CK(nr_time_stage(c1, st, 3, &ms));
    nr_mlp* q; CK(nr_mlp_create(0, 256, (n_reco + 7) / 8 * 8, &q));
    long np_ = nr_mlp_num_params(q); float* pp = calloc(np_, 4);
    CK(nr_mlp_set_params(q, pp, np_)); CK(nr_mlp_get_params(q, pp, np_));
    nr_mlp_destroy(q); free(pp);
    nr_destroy(c1); nr_destroy(c2);
    for (int s = 0; s < n_src; ++s) { free((void*)src[s].E); free((void*)src[s].weight); free((void*)src[s].p_ee); }
    free(src); free(R); free(n); free(b); free(th); free(nll); free(g); free(mu); free(w); free(ssm); free(m);
    printf("stress ok\n");
    return 0;
}
