/*
 * ara.h -- C ABI of libara, an MI355X (gfx950) engine for aggregate risk
 * analysis with primary and secondary uncertainty (Varghese & Rau-Chaplin,
 * WHPCF'13).
 *
 * The calls follow the paper's problem statement: the inputs are the Year
 * Event Table (YET), the extended event loss tables (XELTs) with their
 * financial terms I, and layers of a portfolio with occurrence/aggregate terms
 * T (section 2.1); the output is the Year Loss Table (YLT, Algorithm 1,
 * section 2.2) and the risk measures PML and TVaR derived from it (section 2.4).
 *
 * Conventions for every call:
 *   - No C++ exception crosses this ABI.  Every call returns an ara_status;
 *     ara_last_error() gives a human-readable detail of the last failure.
 *   - Inputs are owned by the caller and copied on load; they may be freed as
 *     soon as the call returns.  Handles belong to the context until freed or
 *     until ara_destroy().
 *   - Outputs are caller-allocated.  A device pointer (for example a torch
 *     tensor's data_ptr()) makes the call asynchronous on the given stream; a
 *     host pointer makes it synchronous.
 *   - Every call is ordered on the device behind the context's previous call,
 *     whatever streams they use.  Loads of XELTs and preparations of layers
 *     return once their inputs are copied to the context's pinned staging,
 *     without waiting for the device work they start.
 *   - hip_stream is a hipStream_t; NULL is the HIP null (default) stream,
 *     which is also torch's default stream.
 *   - One context per host thread; calls on one context must not overlap.
 *   - All validation happens at load time, so kernels never see bad data.
 */
#ifndef ARA_H
#define ARA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ara_ctx ara_ctx;     /* opaque; owns all device memory it allocates */
typedef int32_t ara_status;

#define ARA_OK        0
#define ARA_E_INVAL  (-1)   /* bad argument, non-finite value, mean <= 0, max <= mean,
                               share outside [0,1], duplicate event in an ELT          */
#define ARA_E_RANGE  (-2)   /* event id outside [0, catalog), or floor(N/RP) < 1      */
#define ARA_E_NOMEM  (-3)   /* host allocation failed                                 */
#define ARA_E_BUDGET (-4)   /* the context's HBM budget would be exceeded             */
#define ARA_E_DEVICE (-5)   /* HIP runtime error; the context is unusable afterwards  */
#define ARA_E_STATE  (-6)   /* unknown or freed handle, poisoned context              */

typedef enum {
    ARA_MODE_MEAN = 0,       /* primary uncertainty only: each loss is the XELT mean   */
    ARA_MODE_PLAIN = 1,      /* secondary uncertainty, exact inverse Beta (section 3)  */
    ARA_MODE_SURROGATE = 2,  /* secondary uncertainty, MLP sampler with exact fallback */
    ARA_MODE_TABLE = 3       /* secondary uncertainty, per-entry tabulated inverse     */
} ara_mode;

/* Context on HIP device `device`.  hbm_budget_bytes caps the device memory the
 * context may hold (0 = no cap); a load or run that would exceed it fails with
 * ARA_E_BUDGET and changes nothing. */
ara_status  ara_create(int device, uint64_t hbm_budget_bytes, ara_ctx **out);
void        ara_destroy(ara_ctx *ctx);
/* Detail of the last failure on ctx; owned by ctx, valid until the next call. */
const char *ara_last_error(const ara_ctx *ctx);
/* Device bytes currently held by ctx (tables, YETs, workspaces). */
uint64_t    ara_bytes_in_use(const ara_ctx *ctx);

/*
 * Load a YET (section 2.1: trials of event occurrences in time order; the
 * time stamps are implied by position).  event_ids: int32, host or device.
 * trial_offsets == NULL: fixed length, trial i is event_ids[i*K .. i*K+K).
 * Otherwise trial i is event_ids[trial_offsets[i] .. trial_offsets[i+1])
 * (int64 [n_trials+1], host memory, non-decreasing, starting at 0) and
 * events_per_trial is ignored.  Every id must lie in [0, catalog_size)
 * (ARA_E_RANGE otherwise).  n_trials must be below 2^32 and no trial may
 * hold 2^24 or more events (ARA_E_INVAL otherwise).
 */
ara_status ara_load_yet(ara_ctx *ctx, const int32_t *event_ids, const int64_t *trial_offsets,
                        int64_t n_trials, int32_t events_per_trial, int32_t catalog_size,
                        int32_t *yet_handle);
ara_status ara_free_yet(ara_ctx *ctx, int32_t yet_handle);

/*
 * One XELT (section 2.1): per entry the event id, mean loss mu_l, independent
 * and correlated standard deviations sigma_I, sigma_C (sigma_c == NULL means
 * all zero) and maximum loss max_l; plus the XELT's financial terms I, read as
 * (deductible, limit, share) and applied as share*min(max(l - ded, 0), limit).
 * All arrays are host memory.  Requirements (ARA_E_INVAL otherwise): distinct
 * event ids in [0, catalog_size), 0 < mean < max_loss, sigmas >= 0 and finite,
 * deductible >= 0, limit > 0 (+inf allowed), share in [0, 1].
 */
typedef struct {
    int32_t n_entries;
    const int32_t *event_id;
    const double *mean;
    const double *sigma_i;
    const double *sigma_c;      /* NULL => 0 */
    const double *max_loss;
    double deductible;
    double limit;               /* +inf allowed */
    double share;
} ara_elt_desc;

/* Load n_elts XELTs; the per-entry Beta parameters (section 3.3) are derived on
 * the device at load time.  elt_handles: out[n_elts].  The raw entries of all
 * n_elts XELTs pass through one pinned host block of the context (grown to the
 * largest call so far, kept until ara_destroy). */
ara_status ara_load_elts(ara_ctx *ctx, int32_t catalog_size, const ara_elt_desc *elts,
                         int32_t n_elts, int32_t *elt_handles);
ara_status ara_free_elts(ara_ctx *ctx, const int32_t *elt_handles, int32_t n);

/*
 * A layer (section 2.1): a set of 1..64 loaded XELTs, in the order their
 * losses are summed, and the layer terms T = (OccR, OccL, AggR, AggL) of
 * section 2.3, applied as min(max(l - R, 0), L) per occurrence and to the
 * trial's cumulative occurrence loss.  program_id keys the program-specific
 * random numbers z_(Prog,E) of section 3.1.
 */
typedef struct {
    int32_t n_elts;
    const int32_t *elt_handles;
    double occ_retention;
    double occ_limit;           /* +inf allowed */
    double agg_retention;
    double agg_limit;           /* +inf allowed */
    uint32_t program_id;
} ara_layer_desc;

/*
 * Algorithm 1 for one layer over the whole YET: ylt_out[i] = year loss of
 * trial i (float, n_trials entries).  The random numbers of section 3.1 are
 * u_I = U(Philox4x32-10(key (seed, program_id), counter (trial, slot, j, 0)))
 * with j the XELT's position in the layer, and, for sigma_C > 0,
 * u_C = U(Philox4x32-10(key (seed, 0xFFFFFFFF), counter (trial, slot,
 * 0xFFFFFFFF, 1))), first output word, U(w) = (2*(w>>9)+1)*2^-24.
 * The result is a deterministic function of the inputs and seed: it does not
 * depend on the stream, launch shape or what else runs on the device.  In the
 * sampling modes a draw whose loss would lie within its XELT's retention or
 * beyond retention + limit takes its term (0 or the limit) from the entry's
 * term thresholds, without the inverse: the year losses are those of
 * inverting every draw, up to the inverse's own rounding.
 * max_occ_out (optional, NULL to skip) receives the largest occurrence loss
 * net of occurrence terms per trial (the occurrence exceedance basis).
 */
ara_status ara_run_layer(ara_ctx *ctx, int32_t yet_handle, const ara_layer_desc *layer,
                         ara_mode mode, uint32_t seed, float *ylt_out, void *hip_stream);
ara_status ara_run_layer_ex(ara_ctx *ctx, int32_t yet_handle, const ara_layer_desc *layer,
                            ara_mode mode, uint32_t seed, int64_t trial_begin, int64_t trial_end,
                            float *ylt_out, float *max_occ_out, void *hip_stream);

/*
 * Year event loss table: the per-occurrence view behind the year losses
 * (section 2.4; the occurrence exceedance basis).  As ara_run_layer_ex, and
 * yelt_out receives, for every event occurrence k of every trial i in
 * [trial_begin, trial_end), its loss net of XELT and occurrence terms --
 * the values whose sum the aggregate terms turn into the year loss -- at
 * yelt_out[row(i) + k - row(trial_begin)], where row(i) = i * K for a
 * fixed-length YET and trial_offsets[i] otherwise.  yelt_out: float, device
 * (asynchronous) or host (synchronous), row(trial_end) - row(trial_begin)
 * entries; must not be NULL.  ylt_out and max_occ_out are exactly what
 * ara_run_layer_ex writes for the same arguments.
 */
ara_status ara_run_layer_yelt(ara_ctx *ctx, int32_t yet_handle, const ara_layer_desc *layer,
                              ara_mode mode, uint32_t seed, int64_t trial_begin, int64_t trial_end,
                              float *ylt_out, float *max_occ_out, float *yelt_out, void *hip_stream);

/*
 * Per-occurrence aggregate increments (section 2.3 applies the aggregate terms
 * to the cumulative sum of a trial's occurrence losses, so each occurrence's
 * share of the year loss depends on the events before it; section 2.4 lists
 * per-occurrence reports among the outputs).  yelt holds, in the layout
 * ara_run_layer_yelt writes for trials [trial_begin, trial_end), each
 * occurrence's loss o_k net of XELT and occurrence terms.  With S_k the sum of
 * the trial's o_0..o_k (FP64) and A_k = min(max(S_k - agg_retention, 0),
 * agg_limit), inc_out[same index] = A_k - A_{k-1} (A_{-1} = 0), rounded to
 * FP32: the increments of a trial add up to its year loss, and unlike the
 * year loss they depend on the order of its events.  yelt and inc_out: float,
 * both device (asynchronous on hip_stream) or both host (synchronous).
 * agg_retention >= 0 and finite, agg_limit >= 0 (+inf allowed); ARA_E_INVAL
 * otherwise.
 */
ara_status ara_yelt_increments(ara_ctx *ctx, int32_t yet_handle, int64_t trial_begin, int64_t trial_end,
                               double agg_retention, double agg_limit, const float *yelt, float *inc_out,
                               void *hip_stream);

/*
 * The Beta parameters a loaded XELT's entries were given on the device at load
 * time (section 3.3: mu_beta = mean/max_l, sigma_beta = min(sigma/max_l,
 * 0.999 sigma_beta_max), nu = (sigma_beta_max/sigma_beta)^2 - 1,
 * alpha = mu_beta nu, beta = (1 - mu_beta) nu, all in FP64).  alpha_out,
 * beta_out: host, n_entries doubles each, in the XELT's entry order; both are
 * 0 for an entry with sigma_I + sigma_C = 0 (its loss is the mean).
 * Synchronous.
 */
ara_status ara_elt_params(ara_ctx *ctx, int32_t elt_handle, double *alpha_out, double *beta_out);

/*
 * A batch of layers over one YET: in the plain and table modes the layers go
 * to the GPU in groups whose tables together stay within 24 MB (consecutive
 * in the given order, one launch per group, so a group's solve records stay
 * in the caches; the mean and surrogate modes take the batch in one launch); one
 * wavefront takes its trial through every layer of its group, re-reading the
 * trial's event ids per layer.  ylt_outs[l] receives layer l's YLT (device
 * pointers only).
 */
ara_status ara_run_layers(ara_ctx *ctx, int32_t yet_handle, const ara_layer_desc *layers,
                          int32_t n_layers, ara_mode mode, uint32_t seed,
                          float *const *ylt_outs, void *hip_stream);

/*
 * Prepared layers: the layer tables of `layer` for `mode` are built once and
 * kept (they no longer refer to the XELTs, which may be freed).
 * ara_run_prepared evaluates n prepared layers (all of one mode) over trials
 * [trial_begin, trial_end), grouped into launches as ara_run_layers groups
 * them, each with its own seed, writing
 * ylt_outs[l][i - trial_begin] (device pointers) and, where max_occ_outs is not
 * NULL and its entry not NULL, the largest occurrence loss per trial.
 * Results are those of ara_run_layer_ex for each layer alone.
 */
ara_status ara_prepare_layer(ara_ctx *ctx, const ara_layer_desc *layer, ara_mode mode, int32_t *layer_handle);
ara_status ara_free_layer(ara_ctx *ctx, int32_t layer_handle);
ara_status ara_run_prepared(ara_ctx *ctx, int32_t yet_handle, const int32_t *layer_handles, int32_t n_layers,
                            const uint32_t *seeds, int64_t trial_begin, int64_t trial_end,
                            float *const *ylt_outs, float *const *max_occ_outs, void *hip_stream);

/*
 * Trial tile: the layer kernels evaluate one trial per 64-lane wavefront and
 * group `wpb` wavefronts (1, 2, 4 or 8; 8 not in surrogate mode) per
 * workgroup (defaults: 1 for the plain mode, 4 for the surrogate mode).
 * ara_set_trial_tile fixes it for a mode; ara_autotune times each
 * choice on the first n_trials trials for the given prepared layers (all of
 * one mode), keeps the fastest for that mode (the current tile unless another
 * is more than 3% faster) and returns it (ms_out,
 * optional: the time of each candidate 1, 2, 4, 8, float [4]).  Results do not
 * depend on the choice.  The mean mode has a fixed launch shape (catalog
 * slices of the per-event table in LDS, 16 wavefronts per workgroup) and
 * ignores the tile.
 */
ara_status ara_set_trial_tile(ara_ctx *ctx, ara_mode mode, int32_t wpb);

/*
 * Layout of the per-layer event table the kernels look events up in
 * (section 4.1 weighs direct-access tables against compact ones for the
 * lookup step of Algorithm 1).  ARA_TABLE_DIRECT (the default): one 16-byte
 * row per catalog event, read with one access.  ARA_TABLE_HASHED: rows only for
 * the events some XELT of the layer holds, in a table of 2^b slots (b the
 * smallest with 2^b >= 2 x min(catalog, entries); 32 bytes a slot, the event
 * id beside its row), found by a multiplicative hash and linear probing; it is smaller than the direct table
 * when the layer's XELTs cover a small share of a large catalog.  Applies to
 * the tables of runs and of layers prepared after the call (plain, table and
 * surrogate modes; the mean mode keeps its per-event table).  Results do not
 * depend on the layout.  ARA_E_INVAL for another value.
 */
#define ARA_TABLE_DIRECT 0
#define ARA_TABLE_HASHED 1
ara_status ara_set_table_kind(ara_ctx *ctx, int32_t kind);
ara_status ara_autotune(ara_ctx *ctx, int32_t yet_handle, const int32_t *layer_handles, int32_t n_layers,
                        int64_t n_trials, int32_t *best_wpb_out, float *ms_out);

/*
 * Portfolio and program totals (section 2.1: a portfolio is a set of
 * programs, a program a set of layers): out[i] = the sum over l of
 * ylts[l][i] for i < n_trials, accumulated in FP64 in the order given and
 * rounded to FP32.  ylts: host array of n device pointers (n <= 32768), out:
 * device; asynchronous on hip_stream.  PML/TVaR of a total (ara_risk_measures)
 * are the program- or portfolio-level measures; a total without one program
 * gives that program's marginal contribution.
 */
ara_status ara_sum_ylts(ara_ctx *ctx, const float *const *ylts, int32_t n, int64_t n_trials, float *out,
                        void *hip_stream);

/*
 * PML and TVaR (section 2.4) of a YLT of n_trials floats (device or host):
 * for each return period RP, k = floor(n_trials / RP) (ARA_E_RANGE if k < 1);
 * PML = the k-th largest year loss; TVaR = the mean of the k largest, summed in
 * FP64.  pml_out/tvar_out: host, n_rp doubles each; the call returns when they
 * are written.  n_rp <= 16.
 */
ara_status ara_risk_measures(ara_ctx *ctx, const float *ylt, int64_t n_trials,
                             const double *return_periods, int32_t n_rp,
                             double *pml_out, double *tvar_out, void *hip_stream);

/*
 * The same PML and TVaR, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): this
 * call allocates nothing and does not synchronise.  ylt: device, n_trials
 * floats (n_trials < 2^32); return_periods: host, n_rp doubles, read before
 * the call returns; out: device, 2*n_rp doubles written asynchronously on
 * hip_stream (NULL = the null stream) as out[2r] = PML, out[2r+1] = TVaR of
 * return period r.  The kernels are those of ara_risk_measures, so the
 * results are identical.  Their scratch (64 KiB: histograms, select state,
 * per-block sums) is a static device array, one per GPU, held until the
 * process ends and addressed from ara_create.  Limits: n_rp <= 16
 * (ARA_E_INVAL beyond that, the scratch's size); host ylt or out is
 * ARA_E_INVAL.  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (several streams or contexts at once) race and must be
 * ordered by the caller.
 */
ara_status ara_risk_measures_noalloc(ara_ctx *ctx, const float *ylt, int64_t n_trials,
                                     const double *return_periods, int32_t n_rp,
                                     double *out, void *hip_stream);

/*
 * Auxiliary device calls (the building blocks of ara_run_layer, exposed for
 * per-draw checks and for labelling training data of the sampling surrogate).
 *
 * ara_philox_uniforms: out[i] = U(Philox4x32-10(counter ctr[4i..4i+3],
 * key (key0, key1)) word 0), U(w) = (2*(w>>9)+1)*2^-24 (section 3.1's random
 * numbers as this library generates them).  ctr: uint32 [4n]; out: float [n];
 * host or device pointers (host => synchronous).
 *
 * ara_beta_quantile: x[i] = InvCDF_beta(u[i]; a[i], b[i]) (section 3.3), the
 * plain inverse of the regularised incomplete beta that ara_run_layer uses,
 * computed on the device.  a, b > 0 and 0 < u < 1 (ARA_E_INVAL otherwise when
 * the arrays are host memory; device arrays are not inspected).  All four
 * arrays are double [n], host or device (host => synchronous).
 */
/*
 * Kernel timing: when enabled, ara_run_layer* record HIP events on their stream
 * immediately around the launch of the layer kernel (table building and
 * output copies excluded); ara_last_kernel_ms waits for the last such launch
 * and returns its duration in milliseconds.
 */
ara_status ara_set_profiling(ara_ctx *ctx, int32_t enabled);
ara_status ara_last_kernel_ms(ara_ctx *ctx, double *ms_out);

/*
 * Sampling surrogate for the inverse-Beta step of section 3.3 (a fast method
 * for the step the paper's timings show dominating; mode ARA_MODE_SURROGATE).
 *
 * Model: x = sigmoid(m + s v + NN(ln a / 2, ln b / 2, v / 3)) with v = Phi^-1(u),
 * m = psi(a) - psi(b), s = sqrt(psi'(a) + psi'(b)) (the logit-normal
 * approximation of the Beta quantile) and NN a 3 -> 64 -> 64 -> 1 perceptron
 * with the GELU-like activation g(z) = z S(z), S(z) = w^2 (3 - 2w),
 * w = clamp(z/5 + 1/2, 0, 1) (a cubic gate in place of the Gaussian CDF),
 * weights rounded to BF16 and evaluated as FP16, FP16 activations and FP32
 * accumulation on the matrix cores (v_mfma_f32_16x16x32_f16).  Domain: a, b in [0.2, 50].  A table over
 * 16 x 16 x 16 cells of (ln a, ln b, v) holds the largest absolute error in x
 * seen on held-out points; draws outside the domain or in a cell whose bound
 * exceeds the tolerance use the plain inverse.
 *
 * ara_surrogate_train: draws n_tuples training tuples on the device ((a, b)
 * log-uniform on the domain; u on the 2^-24 grid, half uniform, half
 * logit-uniform), labels them with the plain inverse, and runs `epochs` epochs
 * of Adam (batch a multiple of 64, <= 65536; peak learning rate lr; warm-up
 * then cosine decay) with the library's MFMA forward/backward kernels.
 * Training continues from the current weights (fresh weights on the first
 * call).  epoch_loss_out (optional, host, epochs doubles): mean squared error
 * in x per epoch.
 * Training clears the region table (bias and fallback marks).
 * ara_surrogate_calibrate: fills the region table from n_val fresh held-out
 * tuples: each cell's mean signed error becomes its bias, which inference
 * subtracts from x, and cells whose largest error after that correction,
 * times a margin of 1.5, exceeds tol, or that saw fewer than 64 points, are
 * marked for fallback to the exact inverse.  The table is a deterministic
 * function of the weights, n_val and seed.  Outputs (optional, host): per-cell largest |error| after the
 * correction and the bias (float [4096] each), number of marked cells.
 * ara_surrogate_grad: loss and gradient (float [4481], host) of the mean
 * squared error over n host tuples (f0, f1, f2, base, x; n a multiple of 64,
 * <= 65536) at the current weights, without an update (gradient checks).
 * ara_surrogate_tuples: n training tuples for seed (host float [n][5]).
 * ara_surrogate_export / _import: FP32 weights (float [4481]), Adam moments
 * (float [4481] each), step count, fallback mask (uint8 [4096]) and region
 * bias (float [4096], |bias| <= 1); any pointer but the weights' may be NULL
 * (a NULL mask or bias imports as all zero).  Import makes the surrogate ready.
 * ara_surrogate_eval: x[i] for host (a, b, u) arrays, through the same
 * surrogate-or-exact decision as the layer kernel; used_out[i] = 1 where the
 * surrogate answered.
 */
ara_status ara_surrogate_train(ara_ctx *ctx, int64_t n_tuples, int32_t epochs, int32_t batch, double lr,
                               uint32_t seed, double *epoch_loss_out);
ara_status ara_surrogate_calibrate(ara_ctx *ctx, int64_t n_val, uint32_t seed, double tol,
                                   float *cell_max_out, float *cell_bias_out, int32_t *n_marked_out);
ara_status ara_surrogate_grad(ara_ctx *ctx, const float *tuples, int32_t n, float *grad_out, double *loss_out);
ara_status ara_surrogate_tuples(ara_ctx *ctx, int64_t n, uint32_t seed, float *out);
ara_status ara_surrogate_export(ara_ctx *ctx, float *params, float *adam_m, float *adam_v, int64_t *step,
                                uint8_t *mask, float *cell_bias);
ara_status ara_surrogate_import(ara_ctx *ctx, const float *params, const float *adam_m, const float *adam_v,
                                int64_t step, const uint8_t *mask, const float *cell_bias);
ara_status ara_surrogate_eval(ara_ctx *ctx, const double *a, const double *b, const double *u, int64_t n,
                              double *x_out, int32_t *used_out);

ara_status ara_philox_uniforms(ara_ctx *ctx, const uint32_t *ctr, int64_t n, uint32_t key0, uint32_t key1,
                               float *out, void *hip_stream);
/* ara_normal_quantile: Phi^-1(p[i]) for host arrays of n doubles in (0, 1)
 * (ARA_E_INVAL otherwise), as the correlated draws of section 3.2 compute it
 * (FP64; synchronous). */
ara_status ara_normal_quantile(ara_ctx *ctx, const double *p, int64_t n, double *x_out);
ara_status ara_beta_quantile(ara_ctx *ctx, const double *a, const double *b, const double *u, int64_t n,
                             double *x_out, void *hip_stream);
/* ara_beta_quantile_layer: the per-draw inverse exactly as the plain layer
 * kernel applies it -- the continued-fraction FP32 solve where min(a, b) >=
 * 0.2; below that the FP32 series form of the incomplete beta on the side of
 * the small shape, with ln p, c0 and the residual's sum in FP64.  Same
 * arguments as ara_beta_quantile. */
ara_status ara_beta_quantile_layer(ara_ctx *ctx, const double *a, const double *b, const double *u, int64_t n,
                                   double *x_out, void *hip_stream);
/* ara_beta_quantile_table: the per-draw inverse of the table mode (section 3.3's
 * inverse Beta read from a per-entry table, the paper's call for fast methods):
 * seventeen FP32 Hermite knots per side of t_s around the leading-term
 * asymptote, built in FP64, no iteration; relative error below 1e-4 and
 * absolute error in x below 1e-5 on the paper's shapes.  u is taken in FP32
 * (the draws are on the 2^-24 grid).  Same arguments as ara_beta_quantile. */
ara_status ara_beta_quantile_table(ara_ctx *ctx, const double *a, const double *b, const double *u, int64_t n,
                                   double *x_out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ARA_H */
