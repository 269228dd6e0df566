/*
 * nureweight -- spectrum-reweighting likelihood for solar neutrino-electron
 * scattering on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Plain pointers and sizes only.  One context = one analysis (a set
 * of solar sources on a recoil grid, one detector response, one binned data
 * set) bound to one device and one HIP stream.
 *
 * The method (arXiv:2607.00488):
 *   - NSI-shifted chiral couplings, Sec. II.B, Eq. (g_tilde);
 *   - weak dsigma/dT, Sec. II.A, Eq. (sm_cross_section), with Eq. (xs_nsi);
 *   - magnetic-moment term summed incoherently, Sec. II.C, Eqs. (xs_mm),
 *     (xs_total);
 *   - recoil spectrum S_theta(T_l), Sec. III.A, Eq. (fT), flavour sum as in
 *     Eq. (rate_sm); the kinematic limit T <= 2E^2/(m_e+2E);
 *   - weights w_l = S_theta(T_l) / S_SM(T_l), Eqs. (fT_norm),
 *     (reweight_factor), with w_l := 1 where S_SM(T_l) = 0;
 *   - fold mu_j = f_bkg b_j + sum_l m_l R_lj w_l, Eqs. (Rij),
 *     (fNp_reweight), (mu_total) (matrix form Eq. (matrix_reweight));
 *   - -2lnL = 2 sum_j [mu_j - n_j ln mu_j + lnGamma(n_j+1)]
 *             + sum_m (theta_m - mean_m)^2 / sigma_m^2,  Eq. (logL).
 *
 * Parameter point: 7 doubles,
 *   theta = [eps_eL, eps_eR, eps_tauL, eps_tauR, m2, f_8B, f_bkg],
 * eps_ee^{L,R} and eps_tautau^{L,R} of Eq. (g_tilde) (eps_mumu = 0),
 * m2 = (mu_nu / 1e-11 mu_B)^2 (the square of the moment of Eq. (xs_mm)),
 * f_8B scales every source with group = 1, f_bkg scales the background b.
 * A context in the multi-component form (nr_set_components) takes
 * nr_num_theta(ctx) doubles per point instead; every theta array below has
 * rows of that length.
 *
 * Status codes: 0 ok; NR_EINVAL (-1) bad argument (null pointer, size <= 0,
 * non-finite value, negative counts, size mismatch between the set_* calls);
 * NR_ESTATE (-2) an eval before set_sources, set_response and set_data;
 * NR_EHIP (-3) a HIP runtime error; NR_ENOMEM (-4) allocation failure.
 * On a non-zero return nr_last_error() gives a message (thread-local).
 * A point whose expectation mu_j <= 0 in a bin with n_j > 0 returns
 * -2lnL = +inf with status 0.
 *
 * Ownership: every set_* call copies what it is given before returning; the
 * caller keeps its arrays.  Outputs are caller-allocated.  The _dev entry
 * points borrow device pointers, enqueue on the given stream and do not
 * synchronise; a NULL stream means the HIP default stream (the work is
 * ordered after what is already on it, and later work on it waits for the
 * results).  A context is not thread-safe, and the evaluations of one
 * context share its device work buffers: work enqueued on different streams
 * must not overlap in time (the synchronous entry points use the context
 * stream and wait for it).  Distinct contexts may be used from different
 * threads: every entry point holds one process-wide lock while it does its
 * host-side work (for a synchronous entry point, until its results are
 * back), so calls from different threads run one at a time on the host
 * while their device work may overlap.  The lock exists because a call may
 * capture a HIP graph on its stream, and the HIP runtime fails an open
 * capture when another thread issues a default-stream operation; the
 * caller's own default-stream work in other threads can do the same.
 */
#ifndef NUREWEIGHT_H
#define NUREWEIGHT_H

#ifdef __cplusplus
extern "C" {
#endif

#define NR_OK 0
#define NR_EINVAL (-1)
#define NR_ESTATE (-2)
#define NR_EHIP (-3)
#define NR_ENOMEM (-4)

#define NR_NTHETA 7

typedef struct nr_ctx nr_ctx;

/* One solar source (Sec. III.A).  kind 1: tabulated continuum whose node
 * weights are phi(E_j) * dE (Eq. (fT)); kind 0: a line, whose single node
 * carries the line flux.  p_ee: nu_e survival probability at each node
 * (the nu_mu and nu_tau shares of 1 - p_ee are set by tau_frac).  group 1:
 * scaled by f_8B.  Node order is free. */
typedef struct {
    int kind;
    int n;
    const double *E;       /* [n] MeV, > 0 */
    const double *weight;  /* [n] >= 0; only ratios between nodes matter */
    const double *p_ee;    /* [n] in [0, 1] */
    int group;             /* 0 fixed, 1 scaled by f_8B */
} nr_source;

/* Physical constants; NULL in nr_set_sources selects the defaults
 * m_e = 0.51099895 MeV, G_F = 1.1663788e-11 MeV^-2, sin^2 theta_W = 0.23122
 * (tree level, Sec. II.A), alpha_em = 1/137.035999084, tau_frac = 0.5. */
typedef struct {
    double me, gf, sw2, alpha_em, tau_frac;
} nr_physics;

/* Create a context on HIP device `device`.  *out receives the handle. */
int nr_create(int device, nr_ctx **out);
void nr_destroy(nr_ctx *ctx);

/* Sources and the recoil grid: n_t bins on [t_lo, t_hi], bin l represented
 * by its centre (Sec. VI.A, the single representative energy per bin).
 * Computes the SM reference S_SM(T_l) on the device (Eq. (fT) at theta_SM,
 * Sec. III.A last paragraph) and every theta-independent table. */
int nr_set_sources(nr_ctx *ctx, const nr_source *src, int n_src, int n_t,
                   double t_lo, double t_hi, const nr_physics *phys);

/* Detector response R[l][j] (row-major, l = true recoil bin, j = observed
 * bin; float32, n_t * n_reco values) and the row factors m_l of the fold
 * (Eq. (Rij) with the joint response written as m_l R_lj).  m == NULL
 * selects m_l = n_sig * S_SM(T_l) / sum_l' S_SM(T_l') -- R is then the
 * conditional response P(E_vis,j | T_l) of Eq. (visible_spectrum) and the
 * SM prediction holds n_sig * efficiency signal counts; this needs
 * nr_set_sources first.  Copies R to device memory. */
int nr_set_response(nr_ctx *ctx, const float *R, int n_t, int n_reco,
                    const double *m, double n_sig);

/* Binned data n_j >= 0 (real values allowed: Asimov data), background
 * template b_j >= 0 (scaled by f_bkg; ignored, and may be NULL, in the
 * multi-component form), and optional Gaussian pulls on the nr_num_theta
 * parameters (pull_sigma[i] <= 0: no pull on i; both NULL: none). */
int nr_set_data(nr_ctx *ctx, const double *n, const double *b, int n_reco,
                const double *pull_mean, const double *pull_sigma);

/* -2lnL for n_pts points (theta: [n_pts][7], host), one plain single-point
 * evaluation per point: device E-integral (Eq. (fT) summed per source over
 * the reachable nodes, as suffix sums of the per-node Laurent coefficients
 * in T), weights, HBM-streaming fold and likelihood reduction.  Successive
 * points overlap: one launch folds point p while it forms the weights of
 * p + 1, the node table of p + 2, reduces the fold of p - 1 and completes
 * the likelihood of p - 2.  nll: [n_pts] host.  Synchronous. */
int nr_eval_nll(nr_ctx *ctx, const double *theta, int n_pts, double *nll);

/* -2lnL and its gradient d(-2lnL)/d theta ([n_pts][7]) per point, through
 * the adjoint of the fold (a second pass over R).  Synchronous. */
int nr_eval_nll_grad(nr_ctx *ctx, const double *theta, int n_pts,
                     double *nll, double *grad);

/* Expected spectrum mu ([n_pts][n_reco], host) per point.  Synchronous. */
int nr_eval_mu(nr_ctx *ctx, const double *theta, int n_pts, double *mu);

/* Device-pointer variant of nr_eval_nll / nr_eval_nll_grad: d_theta
 * [n_pts][7] double, d_nll [n_pts] double, d_grad [n_pts][7] double or
 * NULL.  Enqueued on `stream` (hipStream_t, NULL = the default stream);
 * returns without waiting.  Replays a cached HIP graph for repeated
 * (pointer, n_pts) combinations. */
int nr_eval_nll_dev(nr_ctx *ctx, const double *d_theta, int n_pts,
                    double *d_nll, double *d_grad, void *stream);

/* Band skipping in the single-point path.  The conditional response
 * R_ij = P(E_vis,j | T_i) of Sec. II.D (Eq. (visible_spectrum)) is non-zero
 * only within a few resolution widths of the light an electron of recoil
 * T_i makes, so every row of R, and every 128-row fold tile, has a column
 * band outside which all entries are exact zeros (nr_set_response and
 * nr_set_components record the bands).  With `on` non-zero the fold of
 * Eq. (matrix_reweight) and the adjoint pass of the gradient read only the
 * 16-byte column groups inside those bands and write zero partial sums for
 * the rest; in the batched forms every tile of the forward and adjoint
 * matrix products reduces only over the K-steps of 16 whose response
 * entries for it are not all zero.  The skipped terms are exact zeros and
 * no sum changes order, so every result is bitwise the one of the full
 * read (for the batched forms at the same tile shape; the tuner, which
 * times the banded and the dense products separately, may pick another).
 * Off by default: the full dense read of R, as the method is written.
 * Applies to nr_eval_nll, nr_eval_nll_grad, nr_eval_mu, nr_eval_nll_dev,
 * nr_eval_nll_dev_noalloc and the batched and grouped entry points;
 * NR_EINVAL for a null context, NR_ESTATE before a response is set. */
int nr_set_band_skipping(nr_ctx *ctx, int on);

/* Size in bytes of the static workspace of nr_eval_nll_dev_noalloc, one per
 * device. */
#define NR_NOALLOC_WORKSPACE_BYTES 16777216

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation, arguments and results of nr_eval_nll_dev, through the same
 * kernels, with nothing allocated.  The pipeline's node tables, fold vectors,
 * partial sums and adjoint buffers live in a static workspace of the library
 * (NR_NOALLOC_WORKSPACE_BYTES per device, held from the first nr_create on
 * that device until the process ends) instead of the context's buffers, and
 * the launches go directly onto `stream` with no graph of the library's own,
 * so that the caller may capture them in a graph of its own.  Every call on
 * one device shares that workspace: calls that overlap on one device, from
 * any context or thread, race, and the caller must order them (one stream,
 * or events).  No part of the workspace needs to start at zero: each call
 * writes every value it reads.  Returns NR_EINVAL when the context's shapes
 * need more workspace than that (about 2 KiB per reco bin at the default
 * tiling, plus 64 bytes per energy node and 16 per recoil row: a
 * 16384 x 4096 response takes 9.3 MB), besides the status codes of
 * nr_eval_nll_dev. */
int nr_eval_nll_dev_noalloc(nr_ctx *ctx, const double *d_theta, int n_pts,
                            double *d_nll, double *d_grad, void *stream);

/* Batched form: n_pts points of one analysis at once.  The weights of all
 * points (from the theta-independent recoil basis, exact for Eq. (fT)) form
 * a matrix W[p][l] = m_l w_l(theta_p), and the fold of Eq. (mu_total)
 * becomes the dense product W R on the FP64 matrix cores (R widened from
 * FP32 as it is staged) with the Poisson reduction of Eq. (logL) fused into
 * its epilogue.  Synchronous; theta and nll are host arrays as in
 * nr_eval_nll. */
int nr_eval_nll_batched(nr_ctx *ctx, const double *theta, int n_pts,
                        double *nll);

/* Batched likelihood and gradient: the adjoint a = d(-2lnL)/d mu is
 * propagated back through R as a second matrix product (U = A R^T) and
 * contracted with the weight derivatives.  grad: [n_pts][7] host. */
int nr_eval_nll_grad_batched(nr_ctx *ctx, const double *theta, int n_pts,
                             double *nll, double *grad);

/* Expected spectra of the batched form ([n_pts][n_reco], host). */
int nr_eval_mu_batched(nr_ctx *ctx, const double *theta, int n_pts,
                       double *mu);

/* Several analyses (datasets with their own binning and response, all on
 * one device) in one grouped persistent launch: theta[d] ([n_pts[d]][7],
 * host), nll[d] ([n_pts[d]], host).  The stream of ctx[0] is used. */
int nr_eval_nll_multi(nr_ctx *const *ctx, int n_ctx,
                      const double *const *theta, const int *n_pts,
                      double *const *nll);

/* Device-pointer variant of nr_eval_nll_multi (and of the batched gradient
 * when d_grad is not NULL: d_grad[d] is [n_pts[d]][7]).  Enqueued on
 * `stream` (NULL = the default stream); a cached HIP graph of the whole
 * grouped evaluation is replayed for repeated pointer sets. */
int nr_eval_nll_multi_dev(nr_ctx *const *ctx, int n_ctx,
                          const double *const *d_theta, const int *n_pts,
                          double *const *d_nll, double *const *d_grad,
                          void *stream);

/* Weights w_l = S_theta(T_l) / S_SM(T_l) ([n_pts][n_t], host) as the
 * single-point path forms them before the fold.  Synchronous. */
int nr_eval_weights(nr_ctx *ctx, const double *theta, int n_pts, double *w);

/* ---- Multi-component form (Sec. III.B-C, the paper's production
 * likelihood).  Signal component k (a set of sources) has its own SM Monte
 * Carlo histogram N^(k)_ij over (true recoil bin i, observed bin j), live-time
 * mask M^(k)_j and scale s^(k); its response is Eq. (Rij),
 *   R^(k)_ij = (N^(k)_ij / M^(k)_j) / sum_{i'j'} (N^(k)_i'j' / M^(k)_j') s^(k),
 * and with the component's recoil spectrum f^(k)_T (Eq. (fT) over its
 * sources) the prediction of Eqs. (fNp_reweight), (mu_total) is
 *   mu_j = MT M_j [ sum_k r_k Rate_k sum_i R^(k)_ij w^(k)_i
 *                   + sum_b r_b Rate_b pdf_b(j) ],
 * w^(k)_i = f^(k)_T(T_i; theta) / f^(k)_T(T_i; SM) (1 where the SM spectrum
 * is zero): the rate of a signal component carries its integrated cross
 * section, so the normalisation of Eq. (fNp_reweight) cancels.  The
 * parameter vector becomes
 *   theta = [eps_eL, eps_eR, eps_tauL, eps_tauR, m2, r_1..r_K, r_b1..r_bB]
 * (nr_num_theta entries; no f_8B / f_bkg: every component has its own rate
 * r and source groups are ignored).  The fold streams the K responses
 * stacked row-wise (K N_T rows), so an evaluation reads K times the bytes of
 * the single-component form. */
typedef struct {
    int n_comp;                  /* K >= 1 signal components */
    const int *comp_of_source;   /* [n_src] component of every source */
    const float *hist;           /* [K][n_t][n_reco] SM MC histograms, >= 0 */
    const double *comp_mask;     /* [K][n_reco] M^(k)_j > 0, or NULL (1) */
    const double *scale;         /* [K] s^(k) > 0 */
    const double *rate_sm;       /* [K] SM rates Rate_k >= 0 */
    int n_bkg;                   /* B >= 0 background components */
    const double *bkg_pdf;       /* [B][n_reco] 1D PDFs pdf_b(j) >= 0 */
    const double *bkg_rate;      /* [B] rates Rate_b >= 0 */
    const double *mask;          /* [n_reco] common mask M_j >= 0, or NULL */
    double exposure;             /* MT > 0 */
} nr_components;

/* Switch the context to the multi-component form (needs nr_set_sources;
 * 5 + K + B <= 32).  Replaces any response; the data must be set again
 * (nr_set_data with b = NULL allowed and pulls of nr_num_theta entries).
 * Available afterwards: nr_eval_nll, nr_eval_mu, nr_eval_nll_dev without a
 * gradient, nr_time_stage; the gradient, batched, weights, ESS, reference
 * and surrogate entry points return NR_ESTATE.  nr_set_response returns to
 * the single-component form; nr_set_sources drops the components. */
int nr_set_components(nr_ctx *ctx, const nr_components *cmp, int n_reco);

/* Parameters per point of the context's current form (7 for the
 * single-component form, 5 + K + B for the multi-component one): the row
 * length of every theta array and of the pull arrays. */
int nr_num_theta(nr_ctx *ctx);

/* Monte-Carlo events generated in each true recoil bin (n_events [n_t],
 * finite, >= 0): the counts N_lj = R_lj n_events[l] behind the response,
 * for the effective-sample-size diagnostic.  Needs nr_set_response. */
int nr_set_mc_events(nr_ctx *ctx, const double *n_events, int n_t);

/* Effective sample size of the reweighted Monte Carlo in every observed
 * bin, ESS_j = (sum_l N_lj w_l)^2 / sum_l N_lj w_l^2 (0 where no weighted
 * event lands), with the weights w_l of the single-point path: how many
 * unweighted events the reweighted prediction of bin j is worth (the
 * reweighting's statistical support, Sec. VI.A).  ESS_j = sum_l N_lj at
 * theta_SM.  ess: [n_pts][n_reco] host.  NR_ESTATE before
 * nr_set_mc_events.  Synchronous. */
int nr_eval_ess(nr_ctx *ctx, const double *theta, int n_pts, double *ess);

/* Copies the recoil spectra the context holds: S_SM [n_t] (device FP64
 * E-integral at theta_SM) and the row factors m [n_t] in use. */
int nr_get_reference(nr_ctx *ctx, double *s_sm, double *m);

/* The context's HIP stream (hipStream_t), for callers that order their own
 * work against it. */
void *nr_stream(nr_ctx *ctx);

/* Average device time in milliseconds of one stage of the single-point
 * path, launched `iters` times back to back on the context stream between
 * HIP events (stage 1: E-integral node table + weights, 2: fold +
 * likelihood, 3: adjoint, 4: the R-streaming fold alone, 5: the
 * steady-state launch of the point pipeline, all four roles at once).  The
 * launches run on the context's own inputs at the SM point (no stage's work
 * depends on theta) and write only library-internal buffers.  For roofline
 * measurements.  NR_ESTATE before set_sources, set_response and set_data
 * (stage 3: also for a multi-component context). */
int nr_time_stage(nr_ctx *ctx, int stage, int iters, double *avg_ms);

/* Tuning knobs for sweeps.  rows_per_wg > 0: recoil rows per fold tile (a
 * multiple of 8, at most 2048; 0 keeps the current value; NR_ESTATE before
 * nr_set_response).  use_graph: 1 replays cached HIP graphs of repeated
 * (pointer, n_pts) calls, 0 launches every kernel directly, -1 keeps the
 * current setting.  Drops every cached graph. */
int nr_set_fold_tiling(nr_ctx *ctx, int rows_per_wg, int use_graph);

/* ---- Learned surrogate (not in the paper): an MLP theta -> log mu_j,
 * 7 -> hidden -> hidden -> hidden -> n_out with SiLU activations, BF16
 * weights and activations on the matrix cores, FP32 accumulation, FP32
 * master weights and Adam moments.  The parameters are one flat FP32 vector:
 * for each layer l, W_l^T as [n_out_l][k_l] rows with the bias in column
 * n_in_l (the layer input carries a constant one there); k_0 = 32 (7 inputs,
 * bias at 7), k_l = hidden + 8 (bias at hidden) for l > 0.  Inputs are
 * mapped from the box [lo, hi] to [-1, 1]; outputs are standardised log mu
 * (log mu_j = mean_j + std_j * y_j). */
typedef struct nr_mlp nr_mlp;

int nr_mlp_create(int device, int hidden, int n_out, nr_mlp **out);
void nr_mlp_destroy(nr_mlp *mlp);
long nr_mlp_num_params(nr_mlp *mlp);
int nr_mlp_set_params(nr_mlp *mlp, const float *params, long n);
int nr_mlp_get_params(nr_mlp *mlp, float *params, long n);
/* Gradient of the last training step (same layout as the parameters). */
int nr_mlp_get_grads(nr_mlp *mlp, float *grads, long n);
int nr_mlp_set_box(nr_mlp *mlp, const double *lo, const double *hi);
int nr_mlp_set_output_norm(nr_mlp *mlp, const float *mean, const float *std);

/* Standardised log mu targets from expected spectra d_mu [P][n_out]
 * (device, FP64) into d_t [P][n_out] (device, FP32). */
int nr_mlp_targets_dev(nr_mlp *mlp, const double *d_mu, int P, float *d_t,
                       void *stream);

/* One Adam step on the mean squared error of the standardised log mu for a
 * batch (B a multiple of 8): d_theta [B][7] FP64, d_t [B][n_out] FP32.
 * *loss (host, may be NULL) receives the batch loss (synchronises). */
int nr_mlp_train_step_dev(nr_mlp *mlp, const double *d_theta, const float *d_t,
                          int B, float lr, double *loss, void *stream);

/* Predicted log mu [B][n_out] (device FP32). */
int nr_mlp_logmu_dev(nr_mlp *mlp, const double *d_theta, int B,
                     float *d_logmu, void *stream);

/* Surrogate -2lnL against ctx's data (Eq. (logL) with mu = exp of the
 * prediction; the output layer, exp and the Poisson deviance are fused):
 * d_nll [B] device FP64; d_outside [B] (device int, may be NULL) flags
 * points outside the training box. */
int nr_mlp_nll_dev(nr_mlp *mlp, nr_ctx *ctx, const double *d_theta, int B,
                   double *d_nll, int *d_outside, void *stream);

/* Expected spectra of the batched form on device pointers: d_theta
 * [n_pts][7], d_mu [n_pts][n_reco] FP64 (training data for the surrogate). */
int nr_eval_mu_batched_dev(nr_ctx *ctx, const double *d_theta, int n_pts,
                           double *d_mu, void *stream);

/* Template form.  The cross section of
 * Eqs. (xs_nsi) and (xs_mm) is linear in the coupling products, m2 and
 * f_8B, so S_theta of Eq. (fT) is sum_b c_b(theta) I_b over 20
 * theta-independent basis spectra, and the fold of Eq. (matrix_reweight)
 * separates exactly:
 *   mu_j = f_bkg b_j + G0_j + sum_b c_b(theta) G_bj,
 *   G_bj = sum_l R_lj m_l I_b(T_l) / S_SM(T_l) over rows with S_SM > 0,
 *   G0_j = sum_l R_lj m_l over rows with S_SM = 0 (weight 1).
 * The templates G are folded once (one FP64 pass over R); a point then
 * costs 21 products and one logarithm per reco bin.  Same results as the
 * plain and batched forms up to rounding order.
 *
 * On a multi-component context (nr_set_components) each component's
 * sources give 10 basis spectra and its row block is folded with its own
 * SM spectrum, so per bin
 *   mu_j = M_j [sum_k r_k (G0^(k)_j + sum_b c_b G^(k)_bj) + sum_q r_q B_qj]
 * (Eqs. (Rij), (fNp_reweight), (mu_total)), and the gradient covers every
 * parameter of that layout, which the streaming path does not provide.
 * Up to 8 components and 8 background templates (NR_EINVAL beyond).
 *
 * nr_build_templates folds them now (synchronous; allocates).
 * nr_set_sources, nr_set_response and nr_set_components invalidate them,
 * and the first evaluation after such a call folds them again
 * (synchronising and allocating); nr_set_data only has the data slots
 * beside them rewritten (one small kernel, synchronising).  Partial-sum
 * buffers grow (allocating) with the point count and the gradient flag.
 * Before capturing an evaluation in a graph, run it once eagerly with at
 * least as many points (and the same gradient flag), so that nothing is
 * folded or allocated inside the capture. */
int nr_build_templates(nr_ctx *ctx);

/* -2lnL ([n_pts], host) and, when grad is not NULL, its gradient
 * ([n_pts][n_theta], host; n_theta = nr_num_theta) by the template form;
 * theta is [n_pts][n_theta].  Synchronous. */
int nr_eval_nll_templates(nr_ctx *ctx, const double *theta, int n_pts,
                          double *nll, double *grad);

/* Expected spectra ([n_pts][n_reco], host) by the template form. */
int nr_eval_mu_templates(nr_ctx *ctx, const double *theta, int n_pts,
                         double *mu);

/* Device-pointer variant: d_theta [n_pts][n_theta], d_nll [n_pts], d_grad
 * [n_pts][n_theta] or NULL, all FP64 on the context's device; enqueued on
 * `stream` (NULL = the default stream), returns without waiting.  Calls
 * that overlap on one context share its partial-sum buffers and race. */
int nr_eval_nll_templates_dev(nr_ctx *ctx, const double *d_theta, int n_pts,
                              double *d_nll, double *d_grad, void *stream);

/* Diagnostic: the FP64 matrix-core rate the device sustains, from a stream
 * of independent v_mfma_f64_16x16x4_f64 on register operands (8 chains per
 * wave, `blocks` work-groups of 4 waves, `iters` trips of 16 rounds over
 * the chains; no memory traffic while timed).  *tflops receives the rate; the batched GEMM (Sec. III.B's
 * fold as a matrix product) is compared with it.  Returns NR_EINVAL for
 * bad arguments (blocks in 1..65536), NR_EHIP / NR_ENOMEM on device
 * errors; it does not set the nr_last_error message. */
int nr_probe_mfma_f64(int device, int blocks, int iters, double *tflops);

/* Diagnostic: the HBM read rate the device sustains, from `reps` streaming
 * sums (16-byte non-temporal loads) over a zero-filled buffer of `bytes`
 * (1 MiB .. 64 GiB, a multiple of 16; allocated and freed here).  *gbs
 * receives GB/s (1e9 B/s); the single-point fold is compared with it.
 * Status codes as nr_probe_mfma_f64. */
int nr_probe_hbm_read(int device, long long bytes, int reps, double *gbs);

/* Flags of nr_probe_read. */
#define NR_PROBE_CACHED 1    /* ordinary loads, which allocate in L2 and the
                                Infinity Cache, instead of non-temporal ones */
#define NR_PROBE_ALTERNATE 2 /* odd passes walk the buffer last to first */

/* Diagnostic: the read rate of the same streaming sum with a choice of load
 * kind and pass order (`flags`, a combination of the NR_PROBE_ bits above;
 * 0 is nr_probe_hbm_read).  With both flags over a buffer of the response's
 * size it reads memory the way consecutive points of the single-point fold
 * do (a forward pass, then a backward one, each starting on what the last
 * left in the caches), the rate the fold's bytes per second are compared
 * with besides the HBM rate.  Arguments, units and status codes as
 * nr_probe_hbm_read; NR_EINVAL for unknown flag bits. */
int nr_probe_read(int device, long long bytes, int reps, int flags, double *gbs);

/* Message for the last non-zero status on this thread. */
const char *nr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
