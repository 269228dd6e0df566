/* A C caller of the library's boundary: reads a problem from a binary file,
 * runs it through the C ABI only (sources, response, data, plain and
 * template evaluations with gradients) and writes the results and the
 * status codes of a few invalid calls for the Python side to check.
 * Host arrays are freed right after each set_* call: the library keeps its
 * own copies.
 *
 * Input (little-endian): int32 n_src, n_t, n_reco, n_pts; double t_lo, t_hi,
 * n_sig; per source int32 kind, n, group and double E[n], weight[n],
 * p_ee[n]; float R[n_t][n_reco]; double n[n_reco], b[n_reco],
 * theta[n_pts][7].
 * Output: double nll[n_pts], grad[n_pts][7], nll_t[n_pts],
 * grad_t[n_pts][7]; int32 codes[7]: five status codes of invalid calls,
 * then 1 if the evaluations with band skipping equal the ones without bit
 * for bit, then the status of band skipping asked for on a fresh context. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nureweight.h"

static void* rd(FILE* f, size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static int rd_i(FILE* f) {
    int v;
    if (fread(&v, sizeof v, 1, f) != 1) exit(2);
    return v;
}

static double rd_d(FILE* f) {
    double v;
    if (fread(&v, sizeof v, 1, f) != 1) exit(2);
    return v;
}

#define CHECK(call)                                                        \
    do {                                                                   \
        int rc_ = (call);                                                  \
        if (rc_ != NR_OK) {                                                \
            fprintf(stderr, "%s -> %d: %s\n", #call, rc_, nr_last_error()); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: abi_driver in.bin out.bin\n");
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    const int n_src = rd_i(f), n_t = rd_i(f), n_reco = rd_i(f), n_pts = rd_i(f);
    const double t_lo = rd_d(f), t_hi = rd_d(f), n_sig = rd_d(f);
    nr_source* src = (nr_source*)calloc((size_t)n_src, sizeof(nr_source));
    for (int s = 0; s < n_src; ++s) {
        src[s].kind = rd_i(f);
        src[s].n = rd_i(f);
        src[s].group = rd_i(f);
        src[s].E = (const double*)rd(f, sizeof(double) * src[s].n);
        src[s].weight = (const double*)rd(f, sizeof(double) * src[s].n);
        src[s].p_ee = (const double*)rd(f, sizeof(double) * src[s].n);
    }
    float* R = (float*)rd(f, sizeof(float) * (size_t)n_t * n_reco);
    double* n = (double*)rd(f, sizeof(double) * n_reco);
    double* b = (double*)rd(f, sizeof(double) * n_reco);
    double* th = (double*)rd(f, sizeof(double) * n_pts * NR_NTHETA);
    fclose(f);

    int codes[7];
    nr_ctx* ctx = NULL;
    CHECK(nr_create(0, &ctx));
    codes[0] = nr_eval_nll(ctx, th, 1, n);                /* before set_*: ESTATE */
    codes[1] = nr_set_sources(ctx, NULL, n_src, n_t, t_lo, t_hi, NULL);  /* EINVAL */
    codes[2] = nr_last_error()[0] != '\0';                /* a message is set */
    CHECK(nr_set_sources(ctx, src, n_src, n_t, t_lo, t_hi, NULL));
    for (int s = 0; s < n_src; ++s) {
        free((void*)src[s].E);
        free((void*)src[s].weight);
        free((void*)src[s].p_ee);
    }
    free(src);
    CHECK(nr_set_response(ctx, R, n_t, n_reco, NULL, n_sig));
    free(R);
    CHECK(nr_set_data(ctx, n, b, n_reco, NULL, NULL));
    free(n);
    free(b);

    double* nll = (double*)malloc(sizeof(double) * n_pts);
    double* grad = (double*)malloc(sizeof(double) * n_pts * NR_NTHETA);
    double* nll_t = (double*)malloc(sizeof(double) * n_pts);
    double* grad_t = (double*)malloc(sizeof(double) * n_pts * NR_NTHETA);
    CHECK(nr_eval_nll_grad(ctx, th, n_pts, nll, grad));
    CHECK(nr_eval_nll_templates(ctx, th, n_pts, nll_t, grad_t));
    {
        /* the same evaluations reading only R's non-zero column bands */
        double* nll_b = (double*)malloc(sizeof(double) * n_pts);
        double* grad_b = (double*)malloc(sizeof(double) * n_pts * NR_NTHETA);
        CHECK(nr_set_band_skipping(ctx, 1));
        CHECK(nr_eval_nll_grad(ctx, th, n_pts, nll_b, grad_b));
        CHECK(nr_set_band_skipping(ctx, 0));
        codes[5] = memcmp(nll_b, nll, sizeof(double) * n_pts) == 0 &&
                   memcmp(grad_b, grad, sizeof(double) * n_pts * NR_NTHETA) == 0;
        free(nll_b);
        free(grad_b);
        nr_ctx* fresh = NULL;
        CHECK(nr_create(0, &fresh));
        codes[6] = nr_set_band_skipping(fresh, 1);  /* no response yet: ESTATE */
        nr_destroy(fresh);
    }
    double bad[NR_NTHETA], tmp = 0.0;
    memcpy(bad, th, sizeof bad);
    bad[2] = NAN;
    codes[3] = nr_eval_nll(ctx, bad, 1, &tmp);            /* non-finite theta: EINVAL */
    codes[4] = nr_eval_nll(NULL, th, 1, &tmp);            /* null context: EINVAL */
    nr_destroy(ctx);

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(nll, sizeof(double), n_pts, o);
    fwrite(grad, sizeof(double), (size_t)n_pts * NR_NTHETA, o);
    fwrite(nll_t, sizeof(double), n_pts, o);
    fwrite(grad_t, sizeof(double), (size_t)n_pts * NR_NTHETA, o);
    fwrite(codes, sizeof(int), 7, o);
    fclose(o);
    free(th);
    free(nll);
    free(grad);
    free(nll_t);
    free(grad_t);
    printf("abi_driver: %d points through the C ABI\n", n_pts);
    return 0;
}
