/*
 * hmle.h -- C ABI of the MI355X H-MLE library.
 *
 * The library evaluates the Gaussian log-likelihood of Section 1, eq. (1),
 *
 *     L(theta) = -n/2 log(2 pi) - 1/2 log|C(theta)| - 1/2 Z^T C(theta)^{-1} Z,
 *
 * for the Matern covariance of eq. (2) with theta = (sigma^2, ell, nu, tau^2),
 * replacing C by its H-matrix approximation (Section 2: recursive block
 * partition, low-rank far-field blocks built without dense sub-matrices,
 * dense near-field blocks), factorising it by an H-Cholesky C ~ L L^T
 * (Section 2, "Storage and complexity"), and taking log|C| = 2 sum log L_ii
 * and Z^T C^{-1} Z = ||L^{-1} Z||^2. hmle_fit maximises L over theta
 * (Section 2, "Maximization of the log-likelihood"; coordinates and start of
 * Section 5.1).
 *
 * Conventions for every call:
 *   - Every call returns hmle_status; nothing throws or aborts across the ABI.
 *     On an error the outputs are left untouched and hmle_last_error() holds a
 *     message.
 *   - Pointers documented "device" are HIP device pointers to contiguous
 *     float64 data owned by the caller; the library never frees them and reads
 *     them on the problem's stream. Pointers documented "host" are ordinary
 *     host memory.
 *   - Z and sampled fields are always in the caller's point order; the
 *     internal permutation never leaks.
 *   - One problem is used by one host thread at a time. Distinct problems may
 *     run concurrently on distinct streams.
 *   - State machine: build_tree -> assemble -> factor -> loglik / sample /
 *     predict / predict_var. A call out of order returns HMLE_E_STATE. A new
 *     assemble invalidates the factor.
 */
#ifndef HMLE_H
#define HMLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmle_problem_s* hmle_problem;

/* Matern parameters: variance sigma^2, range ell, smoothness nu, nugget tau^2
 * (eq. (2); the paper's theta = (sigma, ell, nu, tau) holds standard
 * deviations, this struct their squares). */
typedef struct {
  double sigma2;
  double range;
  double nu;
  double tau2;
} hmle_theta;

typedef enum {
  HMLE_OK = 0,
  HMLE_E_INVALID = 1,   /* bad argument; nothing changed                        */
  HMLE_E_NOMEM = 2,     /* device allocation failed                             */
  HMLE_E_NOT_SPD = 3,   /* a Cholesky pivot was <= 0 (message: leaf, pivot)      */
  HMLE_E_STATE = 4,     /* call out of order                                    */
  HMLE_E_HIP = 5,       /* HIP runtime error                                    */
  HMLE_E_NOCONV = 6     /* hmle_fit hit max_iter (theta_hat still written)      */
} hmle_status;

typedef enum { HMLE_FP64 = 0, HMLE_MIXED = 1 } hmle_precision;

/* H-matrix options.
 *   leaf_size  clusters with at most this many points are leaves (1..128)
 *   eta        admissibility: min(diam t, diam s) <= eta * dist(t, s) (> 0)
 *   aca_tol    relative Frobenius accuracy per low-rank block, used by the
 *              adaptive cross approximation, the recompression and the
 *              truncation of updated blocks (0 < aca_tol < 1)
 *   max_rank   width of the low-rank storage per block (rank cap), 4..64
 *   precision  HMLE_FP64, or HMLE_MIXED (float32 assembly, cross
 *              approximation and low-rank/near-field updates; float64
 *              diagonal leaves, log-determinant and quadratic form)
 *   pair_chunk    schedule: external pair products of a dense target block per
 *                 workgroup (0 = default 1; 1..16)
 *   sketch_group  schedule: work budget of a low-rank sketch chunk, counted in
 *                 low-rank x low-rank pairs, a pair with a dense block taking
 *                 the whole budget (0 = default 8; 1..16)
 *   spd_margin    definiteness floor of the accuracy (<= 1; negative, the
 *                 default, means automatic: 0.5 in FP64, 0 in the mixed mode,
 *                 whose float32 storage alone perturbs C by about 6e-8 ||C||_2,
 *                 beyond any floor once that exceeds the nugget): with a
 *                 nugget tau^2 > 0 and N low-rank blocks, every cross
 *                 approximation and every truncation of an updated block also
 *                 stops no later than at the absolute Frobenius error
 *                 delta = spd_margin * tau^2 / sqrt(2 N). The errors of the
 *                 assembly and of the factorisation (each a symmetric matrix of
 *                 N mirrored blocks) then stay below spd_margin * tau^2 in
 *                 spectral norm each, and C = M + tau^2 I keeps C~ and the
 *                 factor's matrix positive definite for spd_margin <= 1/2
 *                 (Section 2 remarks that rounding can make small diagonal
 *                 entries negative). 0: the relative accuracy aca_tol alone.
 *   seg_entries   schedule: chunk outputs per workgroup of a low-rank target's
 *                 128-row sketch-sum tile (0 = default 8; 1..32)
 *   gseg_rows     schedule: rows per workgroup of an input-side product U^T X
 *                 of a sketch pass (0 = default 512; 64..4096)
 *   sum_kc        tile shape: inner-dimension columns staged at a time by the
 *                 sketch-sum tiles (0 = default 16; 16 or 32)
 * The schedule options and the tile shape change which workgroup computes
 * which products and so the order of some sums, never the H-matrix or its
 * accuracy; hmle_autotune picks them by measurement. */
typedef struct {
  int32_t leaf_size;
  double eta;
  double aca_tol;
  int32_t max_rank;
  hmle_precision precision;
  int32_t pair_chunk;
  int32_t sketch_group;
  double spd_margin;
  int32_t seg_entries;
  int32_t gseg_rows;
  int32_t sum_kc;
} hmle_opts;

/* Optimiser options (hmle_fit).
 *   max_iter    iteration limit (the paper uses 400)
 *   tol         simplex size tolerance (the paper's threshold 1e-4)
 *   step        initial simplex step per transformed coordinate
 *   use_backoff if the start point is not positive definite, decrease the
 *               nugget exponent tau0 by 1 until it is (at most 30 times)
 *   report_every if > 0, one line on stderr every report_every evaluations
 *               (evaluation count, best log-likelihood so far and its theta);
 *               0 (the default) prints nothing
 *   profile_variance  if nonzero, the variance is profiled out: with the nugget
 *               written tau^2 = r sigma^2, eq. (1) is maximised over sigma^2 in
 *               closed form (sigma^2 = Z^T (R + r I)^{-1} Z / n, R the
 *               unit-variance Matern correlation) and the search runs over
 *               (ell0, nu0, tau0) only, tau0 now coding sqrt(r); each vertex is
 *               one factorisation of R + r I. The estimate maximises eq. (1);
 *               report->logL is its log-likelihood. 0 (the default): the
 *               four-parameter search. */
typedef struct {
  int32_t max_iter;
  double tol;
  double step;
  int32_t use_backoff;
  int32_t report_every;
  int32_t profile_variance;
} hmle_fit_opts;

typedef struct {
  int32_t evals;
  int32_t iters;
  int32_t failed_evals;
  int32_t converged;
  double logL;
  double wall_s;
} hmle_fit_report;

/* Fill *o with the defaults: leaf 64, eta 2, aca_tol 1e-6, max_rank 32, FP64,
 * pair_chunk 1, sketch_group 8, spd_margin -1 (automatic), seg_entries 8,
 * gseg_rows 512, sum_kc 16. */
void hmle_default_opts(hmle_opts* o);
/* Fill *o with the defaults: 400 iterations, tol 1e-4, step 1, backoff on, no
 * progress lines, the four-parameter search. */
void hmle_default_fit_opts(hmle_fit_opts* o);

/* Build the cluster tree and the block tree (Section 2, recursive partition)
 * for n points of dimension dim (2 or 3) and plan the factorisation.
 *   pts        device, n*dim float64, row-major (point i at pts[i*dim ..])
 *   opts       NULL -> defaults
 *   hip_stream hipStream_t the problem's work is queued on (NULL: default)
 *   out        receives the new problem; NULL on error
 * Errors: HMLE_E_INVALID (n < 1, dim not 2/3, non-finite coordinates, bad
 * options), HMLE_E_NOMEM, HMLE_E_HIP. */
hmle_status hmle_build_tree(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts,
                            void* hip_stream, hmle_problem* out);

/* Caller-supplied device memory. alloc returns a device pointer to at least
 * `bytes` bytes usable on `stream` (the problem's hip_stream), or NULL on
 * failure; free releases a pointer alloc returned, with the same stream and
 * user. Used for all device storage of a problem (trees, plan, H-matrix,
 * factor, workspaces), allocated during the build and lazily by the calls
 * that need extra workspace (prediction, the H-matrix-vector product,
 * assembly reuse, candidate fits); everything is freed in hmle_destroy after
 * the problem's streams are drained. The Python binding binds PyTorch's
 * caching allocator here. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} hmle_allocator;

/* hmle_build_tree / hmle_build_batch with the caller's allocator (alloc NULL:
 * hipMalloc / hipFree, as the calls without it). A NULL from alloc gives
 * HMLE_E_NOMEM and frees what was obtained so far; HMLE_E_INVALID for an
 * allocator whose alloc or free is NULL. */
hmle_status hmle_build_tree_alloc(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts,
                                  const hmle_allocator* alloc, void* hip_stream, hmle_problem* out);
hmle_status hmle_build_batch_alloc(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                                   const hmle_opts* opts, const hmle_allocator* alloc, void* hip_stream,
                                   hmle_problem* out);

/* Assemble the H-matrix approximation of C(theta) (eq. (2) plus tau^2 on the
 * diagonal): dense near-field blocks and low-rank far-field blocks computed
 * by adaptive cross approximation without forming them, then recompressed.
 * Reuse (single problems; the conclusion's remedy of updating the matrix by
 * scaling and a new diagonal instead of recomputing it): when theta differs
 * from the last full assembly only in sigma2 and tau2, the saved near field is
 * scaled by sigma2 / sigma2_0 with the nugget replaced on the diagonal, and
 * the cross-approximation factors are scaled in place, without evaluating
 * the Matern function; with the definiteness floor on (spd_margin > 0) only
 * if tau2 / sigma2 did not decrease (the saved ranks then meet the new
 * floor). hmle_assembly_info reports whether the last call reused.
 * Errors: HMLE_E_INVALID (sigma2 <= 0, range <= 0, nu outside [0.05, 8],
 * tau2 < 0, non-finite), HMLE_E_STATE. */
hmle_status hmle_assemble(hmle_problem p, const hmle_theta* theta);

/* H-Cholesky factorisation of the assembled matrix, in place, in the same
 * block structure. Errors: HMLE_E_NOT_SPD (pivot <= 0; message names the
 * leaf), HMLE_E_STATE. */
hmle_status hmle_factor(hmle_problem p);

/* Log-likelihood of data z (device, n float64, caller's order) under the
 * factorised matrix. out (host, 3 doubles) receives logL, log|C~|, and
 * Z^T C~^{-1} Z. Synchronises the problem's stream. */
hmle_status hmle_loglik(hmle_problem p, const double* z, double out[3]);

/* Maximum-likelihood fit: Nelder-Mead on -L in the coordinates of Section
 * 5.1 (sigma = 2/1.1^s0, ell = 1/1.5^l0, nu = 1/1.2^n0, tau = 1/2^t0), each
 * vertex one assemble+factor+loglik; a vertex that is not positive definite
 * or leaves the parameter box (sigma2 in [1e-6, 1e6], range in [1e-4, 10], nu
 * in [0.05, 8], tau2 in [0, 1e3]; with profile_variance the box applies to
 * the point evaluated, sigma2 = 1 and tau2 = r) gets -L = +inf without being
 * evaluated.
 *   z          device, n float64
 *   start      NULL -> the paper's start (2, 2, 1, 15) in transformed coordinates
 *   opts       NULL -> defaults
 *   theta_hat  receives the estimate (also on HMLE_E_NOCONV)
 *   report     may be NULL */
hmle_status hmle_fit(hmle_problem p, const double* z, const hmle_theta* start,
                     const hmle_fit_opts* opts, hmle_theta* theta_hat, hmle_fit_report* report);

/* Size in bytes of a fit checkpoint (hmle_fit_resumable). */
#define HMLE_FIT_STATE_BYTES 320

/* The fit of hmle_fit with a checkpoint (for long fits that may be stopped and
 * continued). state: host buffer of exactly HMLE_FIT_STATE_BYTES bytes owned
 * by the caller. If it does not hold a checkpoint (e.g. all zero), the fit
 * starts from `start` as hmle_fit does; if it holds one written by an earlier
 * call on a problem of the same size with the same profile_variance, the same
 * data z and the same leaf size, eta, aca_tol, max_rank, precision and
 * definiteness floor (a 32-bit fingerprint of these is stored in the
 * checkpoint), the fit continues from the iteration where that call stopped
 * and `start` is ignored. On HMLE_OK and HMLE_E_NOCONV the buffer receives the
 * checkpoint at exit (the sorted simplex, its values and the counters). A fit
 * stopped by max_iter = k and continued with a larger max_iter evaluates
 * exactly the points of the uninterrupted fit and returns its estimate; report
 * counts are cumulative, report->wall_s covers this call only. Errors:
 * HMLE_E_INVALID (NULL arguments, wrong state_len, a checkpoint of another
 * problem size, search kind, data or accuracy options), else as hmle_fit. */
hmle_status hmle_fit_resumable(hmle_problem p, const double* z, const hmle_theta* start,
                               const hmle_fit_opts* opts, void* state, int64_t state_len,
                               hmle_theta* theta_hat, hmle_fit_report* report);

/* The same fit with theta candidates evaluated together. batch: a batch
 * (hmle_build_batch) of count >= 1 identical copies of one point set;
 * HMLE_E_INVALID (message via hmle_last_error) if its problems differ in size,
 * ordering or coordinates. z: device, n1 float64 for one copy (the library
 * replicates it in a device buffer of count * n1 values that the batch keeps
 * until hmle_destroy, allocated by its first fit). Before
 * each iteration the points the iteration may need are announced
 * (reflection, inside and outside contraction, expansion; the shrunken
 * vertices; the initial simplex); a value not yet known is computed with up
 * to count - 1 other announced points in one batched evaluation
 * (hmle_eval_batch). Batched values equal single evaluations bit for bit, so
 * theta_hat, report->evals/iters/failed_evals/logL are exactly those of
 * hmle_fit on one copy with the same options; *rounds (may be NULL) receives
 * the number of batched evaluations. */
hmle_status hmle_fit_batch(hmle_problem batch, const double* z, const hmle_theta* start,
                           const hmle_fit_opts* opts, hmle_theta* theta_hat, hmle_fit_report* report,
                           int32_t* rounds);

/* Kriging prediction (Section 2, eq. (4)): after hmle_factor at theta (for
 * instance the fit's estimate), the conditional mean at m new points
 *   z2 = C21 C~^{-1} z1,
 * C~ the H-matrix of the training points (with nugget) and C21 the Matern
 * cross-covariance of the new points to the training points (no nugget).
 * C~^{-1} z1 takes a forward and a backward substitution with the H-factor;
 * C21 is applied exactly, entry by entry over all n training points
 * (m * n Matern evaluations). Single problems only (HMLE_E_INVALID for a batch).
 *   z1    device, n float64 (the training data, caller order)
 *   pts2  device, m x dim float64 row-major (the new points)
 *   z2    device, m float64 (output) */
hmle_status hmle_predict(hmle_problem p, const double* z1, const double* pts2, int64_t m, double* z2);

/* Kriging variance (Section 3, the mean squared prediction error of eq. (4)
 * under the assumed parameters): after hmle_factor at theta,
 *   var_k = sigma^2 - c_k^T C~^{-1} c_k,   c_k = C12[:, k],
 * the variance of the field (without nugget) at new point k given the
 * training data, by forward substitution of the columns P c_k with the
 * H-factor, 32 points at a time. Single problems only.
 *   pts2  device, m x dim float64 row-major;  var  device, m float64 (output) */
hmle_status hmle_predict_var(hmle_problem p, const double* pts2, int64_t m, double* var);

/* Prediction-error measures of Section 3, eqs. (5) and (6), at m new
 * points: pa factorised at the estimated parameters theta_a, pt at the true
 * ones theta_t, both built on the same points with the same leaf size (same
 * internal order) and on one stream; single problems. For new point s with
 * kriging weights w_a = C~_a^{-1} c_a (eq. (4) with theta_a) the expected
 * squared errors under the true model, for a zero-mean Gaussian model, are
 *   e_ta = w_a^T C~_t w_a - 2 w_a^T c_t + Var_t(Z)       (estimated predictor),
 *   e_tt = Var_t(Z) - c_t^T C~_t^{-1} c_t               (true predictor),
 *   e_aa = Var_a(Z) - c_a^T C~_a^{-1} c_a               (estimated predictor, its own model),
 * with Var(Z) = sigma^2 + tau^2 for a noisy target (noisy != 0: a held-out
 * observation) else sigma^2; w_a^T C~_t w_a = |L~_t^T w_a|^2 by the true
 * factor. out (host): MLOE = mean(e_ta / e_tt - 1), MMOM = mean(e_aa / e_ta - 1).
 * e_ta, e_tt, e_aa: device, m float64 each, or NULL (library workspace).
 * Per point one backward substitution with L~_a and one product with
 * L~_t^T; the forward substitutions run 32 points at a time. */
hmle_status hmle_mloe_mmom(hmle_problem pa, hmle_problem pt, const double* pts2, int64_t m, int32_t noisy,
                           double* e_ta, double* e_tt, double* e_aa, double out[2]);

/* H-matrix-vector product y = C~ x with the assembled H-matrix (Section 2:
 * dense near-field blocks and low-rank far-field blocks U V^T, the upper
 * triangle by symmetry), e.g. to measure the approximation error
 * ||C~ x - C x|| / ||C x|| against an exact product. Only between
 * hmle_assemble and hmle_factor (the factorisation overwrites the assembled
 * near field in place): HMLE_E_STATE otherwise. x, y: device, n float64 each,
 * the caller's point order (for a batch: concatenated, the product of the
 * block-diagonal batch matrix). Sums in a fixed order; synchronises the
 * problem's stream. */
hmle_status hmle_matvec(hmle_problem p, const double* x, double* y);

/* Field sampler: after hmle_factor, z = P^T L~ w (device n float64 each), a
 * draw from N(0, C~) in the caller's order given standard normals w (given in
 * the internal order, i.e. any order: w is white noise). */
hmle_status hmle_sample(hmle_problem p, const double* w, double* z);

/* ---- Batches of independent problems ------------------------------------
 * A batch holds `count` problems, each its own point set (the H-matrix of a
 * batch is block diagonal; no block couples two problems). Each problem's
 * log-likelihood is eq. (1) for its own theta, computed with exactly the
 * arithmetic of the same problem built alone (same trees, blocks, test
 * matrices and summation order), so its results equal the single-problem
 * results. The factorisation steps run over the s-th leaf column of every
 * problem at once: the batch takes as many steps as its largest problem has
 * leaves, not their sum.
 *
 * hmle_build_batch: pts (device, row-major float64) holds the problems' points
 *   one problem after another; offsets (host, count+1 int64) with offsets[0]=0
 *   and offsets[q+1] > offsets[q] delimit problem q; the total must not exceed
 *   2^30. Other arguments and errors as hmle_build_tree. The handle works with
 *   every call taking an hmle_problem except hmle_loglik, hmle_fit,
 *   hmle_predict and hmle_predict_var, which return HMLE_E_INVALID for
 *   count > 1 (hmle_fit_batch takes a batch of copies of one point set). hmle_assemble gives every problem the
 *   same theta; hmle_sample takes and returns concatenated w and z.
 * hmle_assemble_batch: thetas (host, count) one per problem; E_INVALID names
 *   the first invalid one and changes nothing.
 * hmle_factor on a batch of count > 1 returns HMLE_OK when every kernel ran;
 *   problems whose matrix is not positive definite are reported per problem by
 *   hmle_factor_status (host, count statuses: HMLE_OK or HMLE_E_NOT_SPD).
 * hmle_loglik_batch: z (device, total float64, concatenated in the caller's
 *   order of each problem); out (host, count*3): logL, log|C~|, quad per
 *   problem, NaN for a problem that is not positive definite; per_problem
 *   (host, count) its status.
 * hmle_eval_batch: assemble_batch + factor + loglik_batch in one call. The
 *   whole evaluation (assembly, factorisation, solve and reductions of all
 *   problems) is captured once into a HIP graph on a stream the handle owns,
 *   and every later call replays it: per call, one parameter upload, one copy
 *   of z, one graph launch and one read-back. Synchronises the caller's stream
 *   first (z must be ready) and the handle's stream before returning. */
hmle_status hmle_build_batch(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                             const hmle_opts* opts, void* hip_stream, hmle_problem* out);
hmle_status hmle_assemble_batch(hmle_problem p, const hmle_theta* thetas);
hmle_status hmle_factor_status(hmle_problem p, hmle_status* per_problem);
hmle_status hmle_loglik_batch(hmle_problem p, const double* z, double* out, hmle_status* per_problem);
hmle_status hmle_eval_batch(hmle_problem p, const hmle_theta* thetas, const double* z, double* out,
                            hmle_status* per_problem);

/* ---- Learned starting point ---------------------------------------------
 * The optimiser's iteration count depends on its start (Section 5.1 and the
 * conclusion, which proposes precomputing the initial guess). A small fully
 * connected network (Section 4's architecture family; tanh activations and
 * Adam as in Section 6) maps variogram features of the data to a start.
 *
 * hmle_variogram: features of `count` fields. pts (device, row-major float64,
 *   dim 2 or 3) and z (device float64) hold the fields one after another at
 *   the host offsets offsets[0..count] (offsets[0] = 0). sel (device int32,
 *   may be NULL = every point) lists, per field q, the local indices of the
 *   points used at sel[sel_offsets[q] .. sel_offsets[q+1]) (host offsets);
 *   at most 65536 points per field. out (device, count*33 float32): for the
 *   pairs i < j of the points used with distance h < 1/2, bin floor(64 h),
 *   feature b = log(max(gamma_b, 1e-30)) with gamma_b = sum of (z_i-z_j)^2 /
 *   (2 count_b), 0 for an empty bin; feature 32 = log(points used). The bin is
 *   the largest k with k^2 <= 4096 h^2 (h^2 without fused multiply-adds).
 *   Sums in float64 in a fixed order (deterministic). Synchronises stream.
 *   Its device workspace is kept per GPU between calls and grown when a call
 *   needs more; calls on one GPU are serialised inside the library.
 *   E_INVALID for an index outside its field.
 * The network: 33 -> 128 -> 128 -> 128 -> 4, tanh hidden layers, linear
 *   output, y = x W^T + b per layer, float32; hmle_mlp_param_count() = 37892
 *   parameters, flat: W1 (128x33 row-major), b1, W2 (128x128), b2, W3, b3,
 *   W4 (4x128), b4. Inputs enter standardised (x - mu_x)/sd_x; the outputs
 *   are standardised log(sigma2, range, nu, tau2): t = (log theta - mu_y)/sd_y.
 *   norm (74 floats): mu_x[33], sd_x[33], mu_y[4], sd_y[4].
 * hmle_mlp_create: params (host) copied; Adam moments zero; norm = (0, 1).
 * hmle_mlp_set_params / get_params: host copies; set_params resets Adam.
 * hmle_mlp_set_norm / get_norm: host; hmle_mlp_fit_norm: column means and
 *   standard deviations of x (device rows*33) and of the log targets lt
 *   (device rows*4); a feature whose deviation is below 1e-6 (constant over
 *   the data, so it cannot inform the prediction) gets the scale 1e30, which
 *   switches it off; a target's deviation is floored at 1e-6.
 * hmle_mlp_forward: x (device rows*33 raw features) -> y (device rows*4,
 *   predicted log theta).
 * hmle_mlp_grad: loss = mean over rows and outputs of (y - t)^2 for rows
 *   x[idx[r]], lt[idx[r]] (idx device, may be NULL = rows 0..rows-1; indices
 *   checked against total) and its gradient (device, 37892 floats); loss
 *   (host) may be NULL.
 * hmle_mlp_train_step: the same gradient, then one Adam update (beta1 0.9,
 *   beta2 0.999, eps 1e-8, bias-corrected) with learning rate lr.
 * hmle_propose: feat (device, 33 raw features) -> start (host): exp of the
 *   predicted log parameters, clipped into the optimiser's parameter box.
 * Errors: hmle_last_error(NULL). */
typedef struct hmle_mlp_s* hmle_mlp;
int64_t hmle_mlp_param_count(void);
hmle_status hmle_variogram(const double* pts, const double* z, const int64_t* offsets, int32_t count, int32_t dim,
                           const int32_t* sel, const int64_t* sel_offsets, void* hip_stream, float* out);
/* hmle_variogram_noalloc: for callers that cannot allocate device memory
 *   (code under HIP graph capture, tight serving loops, harnesses that forbid
 *   hipMalloc). Same arguments, checks and output as hmle_variogram, bit for
 *   bit; it calls no allocating routine: its workspace (the two offset arrays
 *   and count * max_tiles * 64 partial sums, max_tiles = t(t+1)/2 with t =
 *   ceil(points used / 128) of the largest field) is a fixed 16 MiB device
 *   array per GPU, held until the process ends. HMLE_E_INVALID (nothing
 *   launched) when a call needs more than 16 MiB, e.g. more than 62 fields of
 *   4096 points. Every call on one GPU shares that GPU's array: calls that
 *   overlap on one GPU (other host threads, other streams) race and must be
 *   serialised by the caller; a call synchronises its stream before returning,
 *   so consecutive calls do not. Errors as hmle_variogram. */
hmle_status hmle_variogram_noalloc(const double* pts, const double* z, const int64_t* offsets, int32_t count,
                                   int32_t dim, const int32_t* sel, const int64_t* sel_offsets, void* hip_stream,
                                   float* out);
hmle_status hmle_mlp_create(const float* params, void* hip_stream, hmle_mlp* out);
hmle_status hmle_mlp_set_params(hmle_mlp net, const float* params);
hmle_status hmle_mlp_get_params(hmle_mlp net, float* params);
hmle_status hmle_mlp_set_norm(hmle_mlp net, const float* norm);
hmle_status hmle_mlp_get_norm(hmle_mlp net, float* norm);
hmle_status hmle_mlp_fit_norm(hmle_mlp net, const float* x, const float* lt, int64_t rows);
hmle_status hmle_mlp_forward(hmle_mlp net, const float* x, int32_t rows, float* y);
hmle_status hmle_mlp_grad(hmle_mlp net, const float* x, const float* lt, const int32_t* idx, int32_t rows,
                          int64_t total, float* grad, float* loss);
hmle_status hmle_mlp_train_step(hmle_mlp net, const float* x, const float* lt, const int32_t* idx, int32_t rows,
                                int64_t total, float lr, float* loss);
hmle_status hmle_propose(hmle_mlp net, const float* feat, hmle_theta* start);
void hmle_mlp_destroy(hmle_mlp net);

/* Matern function of eq. (2) (no nugget) evaluated on the device at
 * distances h (device, count float64) into out (device, count float64), in
 * float64 (precision HMLE_FP64) or float32 arithmetic (HMLE_MIXED). */
hmle_status hmle_matern(const double* h, int64_t count, const hmle_theta* theta,
                        hmle_precision precision, void* hip_stream, double* out);

/* Introspection (host outputs; sizes from hmle_sizes):
 *   sizes[0..5] = n, dim, n_nodes, n_dense, n_lowrank, n_leaves
 *   perm (n int64): perm[k] = caller index of the k-th internal point
 *   nodes (n_nodes*4 int64): lo, hi, child0, child1 per node (level order)
 *   dense/lowrank ((n_dense|n_lowrank)*2 int64): (row node, col node),
 *   sorted by (col lo, row lo). */
hmle_status hmle_sizes(hmle_problem p, int64_t sizes[6]);
hmle_status hmle_export_tree(hmle_problem p, int64_t* perm, int64_t* nodes, double* bmin, double* bmax);
hmle_status hmle_export_blocks(hmle_problem p, int64_t* dense, int64_t* lowrank);

/* Export block `which` of the current matrix (assembled C~ after
 * hmle_assemble, the factor L~ after hmle_factor) to host memory, in the
 * internal order. For a dense block of m rows and k columns: data holds the
 * m*k entries column-major and *rank = -1. For a low-rank block: data holds
 * U (m*rank, column-major) followed by V (k*rank, column-major), block =
 * U V^T, and *rank its rank. cap_doubles bounds the copy.
 * kind: 0 = dense list index, 1 = low-rank list index. */
hmle_status hmle_export_block(hmle_problem p, int32_t kind, int64_t which, double* data,
                              int64_t cap_doubles, int32_t* rank);

/* Structure only, from HOST points (pts: n*dim float64, row-major): the
 * cluster tree, block tree and factorisation plan, without touching the GPU.
 * Only hmle_sizes, hmle_export_tree, hmle_export_blocks, hmle_plan_stats and
 * hmle_destroy accept such a problem; the numerical calls return
 * HMLE_E_STATE. Meant for inspecting the partition of a point set. */
hmle_status hmle_structure_host(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts,
                                hmle_problem* out);
/* The same for a batch (host pts and offsets as in hmle_build_batch). */
hmle_status hmle_structure_batch_host(const double* pts, const int64_t* offsets, int32_t count, int32_t dim,
                                      const hmle_opts* opts, hmle_problem* out);

/* Plan statistics: s[0] external-update pairs, s[1] inner updates,
 * s[2] dense entries (diagonal leaves as full squares), s[3] sum of (m + k)
 * over low-rank blocks, s[4] leaves, s[5] low-rank storage width, s[6] column
 * solves (sum over leaves of blocks in that column), s[7] pairs into low-rank
 * targets, s[8] distinct low-rank x low-rank pairs (cached Gram matrices),
 * s[9] pairs that use a cached Gram matrix, s[10] factorisation steps (the
 * largest leaf count of the batch's problems), s[11] problems, s[12..15]
 * pairs into low-rank targets whose (x, y) are dense-dense, dense-low-rank,
 * low-rank-dense, low-rank-low-rank. */
hmle_status hmle_plan_stats(hmle_problem p, int64_t s[16]);

/* Assembly reuse: info[0] = 1 if the last hmle_assemble scaled the saved
 * assembly instead of recomputing it, else 0; info[1] = such reuses so far. */
hmle_status hmle_assembly_info(hmle_problem p, int64_t info[2]);

/* Per-stage timings of the last calls (milliseconds, HIP events):
 * t[0] assemble, t[1] factor, t[2] loglik; counters: c[0] sum of low-rank
 * ranks after the last factor, c[1] max rank, c[2] rank-cap hits. */
hmle_status hmle_stats(hmle_problem p, double t[3], int64_t c[3]);

/* Live timing of the three largest factorisation kernels: the external
 * pair products of dense target blocks (k_dpairs, main stream), the sketch
 * passes of low-rank target blocks (k_rpass, second stream) and the
 * diagonal-leaf Cholesky with the inverse of its factor (k_potrf, main
 * stream). enable = 1 records HIP events around their launches, on the
 * stream each runs on, in every following hmle_factor (and clears the
 * counters), 0 stops, -1 leaves the setting. out (host, may be NULL)
 * receives, summed over the factorisations since enabling: [0] dense-pair GPU
 * time in ms, [1] its launches, [2] its algorithmic flops (products of the
 * stored factors, with the ranks of each factorisation); [3..5] the same for
 * the sketch passes; [6..8] for the diagonal leaves (m^3 / 3 flops per leaf
 * of m points: the Cholesky; the factor's inverse formed beside it is not
 * counted). */
hmle_status hmle_profile(hmle_problem p, int32_t enable, double out[9]);

/* One candidate of the autotuner: the options and the time in ms of a warm
 * factorisation with them. */
typedef struct {
  hmle_opts opts;
  double ms;
} hmle_tune_entry;

/* Autotuner of the schedule options and the tile shape by coordinate search:
 * starting from opts (zeros: the defaults), it varies one option at a time
 * over its candidates -- pair_chunk {1, 2, 4}, sketch_group {2, 4, 8, 16},
 * seg_entries {2, 4, 8, 16}, gseg_rows {128, 256, 512, 1024}, sum_kc {16, 32} -- and
 * keeps the fastest, in two sweeps over the five options. Each candidate
 * builds the problem (pts, n, dim, hip_stream as in hmle_build_tree, the other
 * options from opts), assembles at theta and factorises twice; the second
 * factorisation (the replayed one, as in repeated evaluations) is timed with
 * HIP events. best receives the options of the fastest candidate. tried
 * (host, may be NULL) receives up to max_tried candidates in the order they
 * were measured and *n_tried (may be NULL) their number (each distinct
 * candidate is measured once; at most 1 + 2 * (2 + 3 + 3 + 3 + 1) = 25). A
 * candidate whose matrix is not positive definite is still timed. Errors as
 * hmle_build_tree / hmle_assemble; HMLE_E_INVALID for max_tried < 0. */
hmle_status hmle_autotune(const double* pts, int64_t n, int32_t dim, const hmle_opts* opts, const hmle_theta* theta,
                          void* hip_stream, hmle_opts* best, hmle_tune_entry* tried, int32_t max_tried,
                          int32_t* n_tried);

/* Message for the last error on this problem (NULL: thread-local last error
 * of calls without a problem). Valid until the next call on that problem. */
const char* hmle_last_error(hmle_problem p);

/* Free everything the problem owns (waits for its stream). NULL is a no-op. */
void hmle_destroy(hmle_problem p);

#ifdef __cplusplus
}
#endif

#endif /* HMLE_H */
