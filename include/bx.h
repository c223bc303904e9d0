/*
 * bx.h -- C ABI of the MI355X spectral-fit likelihood library (libbx.so).
 *
 * The library evaluates, on one gfx950 GPU, the model that every step of a
 * binned spectral fit repeats (Ding et al., arXiv:1805.11125):
 *
 *   - the deposited spectrum of every species folded with an analytic detector
 *     response on the true x reco energy grid (Sec. 3, Eq. 1);
 *   - the pile-up convolution with a random-trigger spectrum (Sec. 3, Eq. 2);
 *   - the binned Poisson negative log-likelihood over the TFC-vetoed and
 *     TFC-tagged energy histograms (Sec. 3, Eq. 3), plus the radial and
 *     pulse-shape terms of the multivariate likelihood (Sec. 3, Eq. 4);
 *   - its analytic gradient, and a quasi-Newton minimiser that varies the
 *     parameters until the likelihood is optimal (Sec. 4, workflow steps 5-7).
 *
 * Conventions used by every call
 *   - NLL = sum over all terms and bins of (mu - n ln mu).  The data-only
 *     constant sum ln Gamma(n+1) is left out (see bx_model_lnfact).  A bin with
 *     n = 0 contributes mu.  mu < 0, or mu = 0 with n > 0, is a domain error.
 *   - Parameters theta = [r_0 .. r_{S-1} | response parameters]; r_s is the
 *     expected number of events of species s over its whole deposited spectrum
 *     (times the exposure).  Gaussian response: (a, b) with
 *     sigma(E)^2 = a E + b E^2, mean E.  Generalized-gamma response with fixed
 *     exponent p: (L, v0, v1, v2) with mean m = L Q(E) E and variance
 *     s^2 = v0 + v1 m + v2 m^2, shape and scale moment-matched.
 *   - The cell R[j][i] is the probability that an event deposited in true bin i
 *     (at its centre) is reconstructed in reco bin [x_j, x_j+1).  Counts falling
 *     outside [x_0, x_N) are lost.  A zero-width Gaussian puts all of its mass
 *     in the reco bin holding its mean.
 *   - Arrays are row-major and host memory unless a name says "dev".
 *   - No C++ exception crosses this interface.  Every call returns a bx_status;
 *     bx_last_error() gives a message for the calling thread.
 *   - A bx_model is not thread-safe; a bx_server is (submit and poll).
 */
#ifndef BX_H
#define BX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BX_OK = 0,
  BX_PENDING = 1,        /* bx_fit_poll: the fit is still queued or running */
  BX_E_INVAL = -1,       /* invalid argument (sizes, ordering, null pointers) */
  BX_E_NOMEM = -2,       /* device memory could not be allocated */
  BX_E_DEVICE = -3,      /* HIP runtime error or no usable GPU */
  BX_E_DOMAIN = -4,      /* parameters outside the model's domain */
  BX_E_BUSY = -5,        /* object in use, or request larger than the budget */
  BX_E_NOTFOUND = -6     /* unknown ticket */
} bx_status;

/* Detector response of Eq. 1: Gaussian in the energy (a, b); generalized
 * gamma in photoelectrons (L, v0, v1, v2); a tabulated (Monte Carlo) response;
 * or the count estimator: reco bin j is the single count n_j = reco_edges[j]
 * (integer edges of unit width, e.g. the number of fired PMTs), negative
 * binomial with mean m = L Q E and variance v0 + v1 m + v2 m^2 > m (the same
 * four parameters as the generalized gamma; mean <= 0 or variance <= mean is
 * a domain error).  The count estimator is evaluated in FP64. */
typedef enum { BX_RESP_GAUSS = 0, BX_RESP_GG = 1, BX_RESP_TABLE = 2, BX_RESP_COUNT = 3 } bx_response;
typedef enum { BX_PREC_F32 = 0, BX_PREC_F64 = 1 } bx_precision;

/* Model description (Sec. 4, workflow step 2: spectra, response, dataset and
 * likelihood terms).  All arrays are copied by bx_model_build. */
typedef struct {
  int32_t T;                  /* true-energy bins (>= 1) */
  int32_t N;                  /* reco bins (>= 1) */
  int32_t S;                  /* species (1..16) */
  const double* true_edges;   /* [T+1] strictly increasing */
  const double* reco_edges;   /* [N+1] strictly increasing */
  const double* spectra;      /* [S][T] deposited spectra, >= 0, each row > 0
                                 (normalised to unit sum in FP64 at build) */
  int32_t response;           /* bx_response */
  double gg_p;                /* GG exponent p > 0 (GG only) */
  const double* quench;       /* [T] quenching factor at bin centres (GG and count) */
  double exposure;            /* > 0 */
  int32_t pu_K;               /* random-trigger spectrum length, 0 = no pile-up */
  const double* pu_g;         /* [pu_K] >= 0 with positive sum (normalised at build) */
  double pu_frac;             /* pile-up fraction p in [0, 1]; needs uniform reco bins */
  int32_t win_lo, win_hi;     /* fit window [win_lo, win_hi) over reco bins */
  int32_t precision;          /* bx_precision of the response cells; sums are FP64
                                 (a tabulated response is evaluated in FP64) */
  /* multivariate terms (Eqs. 3-4); multivariate = 0 ignores the rest */
  int32_t multivariate;
  const double* tag_frac;     /* [S] TFC tag fraction of each species, in [0, 1] */
  int32_t n_rad;              /* radial bins (0..128; 0 = no radial term) */
  const double* rad_tmpl;     /* [S][n_rad] radial template per species */
  int32_t rad_lo, rad_hi;     /* reco window whose vetoed counts feed the radial term */
  int32_t n_ps;               /* pulse-shape bins (0..64; 0 = no PS term) */
  const double* ps_tmpl;      /* [S][n_ps] pulse-shape template per species */
  /* 1: the pile-up fraction is a fit parameter, the last entry of theta
   * (needs pu_K > 0; pu_frac is then unused); an evaluation with it outside
   * [0, 1] is a domain error.  0: pu_frac is fixed. */
  int32_t pu_float;
  /* Tabulated response (response = BX_RESP_TABLE): the Monte Carlo
   * alternative to the analytic response of Eq. 1 (Sec. 3 names both).
   * n_grid matrices R_g [N][T] (rtab, row-major, g slowest; R_g[j][i] is the
   * probability that an event deposited in true bin i is reconstructed in
   * reco bin j, >= 0, columns may lose mass) given at the strictly increasing
   * values grid[g] of one response coordinate lam.  theta = rates, lam (when
   * n_grid >= 2), then the pile-up fraction when it floats; R(lam) is the
   * linear interpolation between the two grid points around lam (the cell
   * above at an interior grid point, for the gradient), and lam outside
   * [grid[0], grid[n_grid - 1]] is a domain error.  n_grid = 1: a fixed
   * matrix, no response parameter.  1 <= n_grid <= 64.  Ignored for the
   * analytic responses. */
  int32_t n_grid;
  const double* grid;         /* [n_grid] */
  const double* rtab;         /* [n_grid][N][T] */
  /* 1: a joint energy x radius x pulse-shape term replaces the vetoed
   * energy, radial and pulse-shape terms (the alternative the paper names to
   * its additive terms, Sec. 3): the vetoed events of the fit window in one
   * histogram bx_data.joint [N][n_rad][n_ps] with expected counts
   * lambda_jkl = sum_s M'_js (1 - t_s) r_s rad_tmpl[s][k] ps_tmpl[s][l]; the
   * tagged term stays.  Needs multivariate = 1, n_rad >= 1, n_ps >= 1 and
   * N * n_rad * n_ps < 2^31; rad_lo, rad_hi and bx_data.energy, radial, ps
   * are then unused.  The device holds the histogram as the list of its
   * non-zero bins per row, with room for every bin (12 bytes per bin), so
   * bx_model_set_data accepts any new histogram of the same shape. */
  int32_t joint;
} bx_model_desc;

/* Observed histograms (FP64 counts; integers or Asimov values >= 0). */
typedef struct {
  const double* energy;       /* [N] energy histogram (TFC-vetoed if multivariate) */
  const double* tagged;       /* [N] TFC-tagged histogram (multivariate) */
  const double* radial;       /* [n_rad] */
  const double* ps;           /* [N][n_ps] energy x pulse-shape histogram */
  const double* joint;        /* [N][n_rad][n_ps] vetoed events (joint term only) */
} bx_data;

typedef struct bx_model bx_model;
typedef struct bx_server bx_server;

/* Sec. 4, workflow steps 1-2: load the configuration, histograms and
 * exposure, and construct the spectra, the response, the dataset and the
 * likelihood terms.  Build a model: validate, copy every array to device
 * memory, allocate the evaluation workspace.  hip_stream: a hipStream_t the model uses for all of
 * its work (borrowed), or NULL for a stream the model owns.
 * Errors: BX_E_INVAL for bad sizes, non-increasing edges, negative spectra or
 * all-zero rows, non-uniform reco bins with pile-up on, a window out of range;
 * BX_E_NOMEM; BX_E_DEVICE.  On error *out is NULL. */
bx_status bx_model_build(const bx_model_desc* desc, const bx_data* data, void* hip_stream,
                         bx_model** out);

/* Sec. 4, workflow step 1 (a new histogram for the same configuration):
 * replace the observed histograms (same shapes).  Stream-ordered copy. */
bx_status bx_model_set_data(bx_model* m, const bx_data* data);

/* Sec. 4, workflow step 7 (the fit is over): release the model and its
 * device memory.  BX_E_BUSY while a server fit uses it. */
bx_status bx_model_free(bx_model* m);

/* The parameters the minimiser varies (Sec. 4, step 5): the species rates
 * and the response parameters p_0, p_1, ... of Eq. 1.  Number of parameters
 * P = S + (2 Gaussian | 4 GG or count | 1 table with n_grid >= 2
 * | 0 one-matrix table) + (1 when the pile-up fraction floats). */
int32_t bx_model_nparams(const bx_model* m);

/* The data-only part of the Poisson likelihood terms of Eqs. 3-4: sum of
 * ln Gamma(n+1) over every bin in the NLL (FP64, computed at build and on
 * bx_model_set_data).  NLL + lnfact is the full negative log-likelihood. */
bx_status bx_model_lnfact(const bx_model* m, double* out);

/* Sec. 4, step 6: one evaluation of the likelihood the minimiser requests --
 * the expected counts of every bin (Eqs. 1-2 folded with the rates) and the
 * terms of Eqs. 3-4.  NLL at theta[P] (host).  Synchronous.  Domain errors
 * return BX_E_DOMAIN and
 * *nll = +INFINITY (non-finite theta, sigma^2 < 0, GG mean or variance <= 0,
 * mu < 0 or mu = 0 < n). */
bx_status bx_nll_eval(bx_model* m, const double* theta, double* nll);

/* Eqs. 1-4 and Sec. 4, steps 5-6: the evaluation of bx_nll_eval and the
 * analytic gradient the minimiser steps along.  NLL and its gradient grad[P]
 * (host).  Synchronous.  Domain errors as for
 * bx_nll_eval; the gradient is undefined (BX_E_DOMAIN) when some Gaussian
 * width is exactly zero.  On BX_E_DOMAIN grad is left untouched. */
bx_status bx_nll_grad(bx_model* m, const double* theta, double* nll, double* grad);

/* Eqs. 1-4 and Sec. 4, steps 5-6, for a minimiser that keeps its state on
 * the device: device-pointer variant for stream-ordered use (autograd): reads
 * d_theta[P], writes d_out[0] = NLL (+INFINITY on a domain error) and
 * d_out[1..P] = gradient.  stream: hipStream_t to run on (NULL = the model's).
 * Asynchronous; the status describes the enqueue only. */
bx_status bx_nll_grad_dev(bx_model* m, const double* d_theta, double* d_out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as bx_nll_grad_dev, with the same results bit for bit, whose
 * per-evaluation workspace (about 2 MB for a 3000 x 900 single-histogram
 * model, 3.5 MB multivariate) comes from one 16 MiB array in device memory
 * that the library holds on each GPU it runs on until the process ends,
 * instead of the model's own workspace.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine); the caller passes the
 * inputs and outputs.  Must run on the model's device (BX_E_INVAL otherwise);
 * a model whose workspace exceeds the array is rejected with BX_E_INVAL.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (on different streams, or from different threads) race and must be
 * serialised by the caller.  Asynchronous on `stream` (NULL = the model's);
 * the status describes the enqueue only. */
bx_status bx_nll_grad_dev_noalloc(bx_model* m, const double* d_theta, double* d_out, void* stream);

/* Eqs. 1-4: expected counts of every likelihood term at theta (what Sec. 4,
 * step 6 evaluates per bin), for the full reco range:
 * out = [mu_energy[N] | mu_tagged[N] | nu_radial[n_rad] | lambda_ps[N][n_ps]]
 * (single histogram: mu[N] only).  bx_model_expected_size gives the length. */
int64_t bx_model_expected_size(const bx_model* m);
bx_status bx_model_expected(bx_model* m, const double* theta, double* out);

/* Diagnostics of the evaluation of Sec. 4, step 6 (Eqs. 1-4): average
 * duration (milliseconds) of each stage of one NLL + gradient evaluation at
 * theta.  After one evaluation at theta, each stage's kernels are launched
 * `reps` times back to back on the model's stream between two HIP events
 * (each launch recomputes that stage's output from the previous stages'
 * results); ms[8] times `reps` whole evaluations launched kernel by kernel
 * (no graph) the same way.  ms[11] = {column parameters, forward cell sweep +
 * species contraction (with its fix-up sweep), partial-sum reduction, pile-up
 * + likelihood terms, radial term, pile-up adjoint, backward cell sweep (with
 * its fix-up sweep), final sums, whole evaluation, forward main sweep alone,
 * backward main sweep alone}; a stage the model does not have reads ~0.  A
 * tabulated response reports its interpolation as the first stage; the
 * joint term's kernel is timed with the radial stage. */
bx_status bx_model_stage_times(bx_model* m, const double* theta, int32_t reps, double* ms);

/* Diagnostics (Sec. 4, step 6, for many fits at once): the same per-stage
 * timing for a batch.  `copies` independent fits of this model (its data,
 * theta) are placed in device memory as the fit server places them and
 * evaluated together, one launch per stage with blockIdx.y selecting the fit;
 * ms[11] as above, per batched launch.  Device
 * memory for the batch is allocated and freed inside the call (BX_E_NOMEM if
 * it does not fit).  Synchronous on the model's stream. */
bx_status bx_model_batch_times(bx_model* m, const double* theta, int32_t copies, int32_t reps, double* ms);

/* Diagnostics of the cells of Eq. 1 (the response integrated over one reco
 * bin): the rate (cells per second) that the cell arithmetic of this model's
 * response reaches on its own (the one-interval quadrature of the cell and its
 * two column-parameter derivatives, as the backward sweep forms them; the
 * per-cell pmf for the count estimator), measured with the column constants
 * and supports at theta: 256 x 8 workgroups of 4 waves, each wave one (true
 * tile, reco tile) pair of the workload in the sweeps' lane layout (4 cells
 * per lane), evaluated `reps` times from registers (no tile lists,
 * contraction or memory traffic).  It is the measured ceiling of the cell
 * sweeps.  BX_E_INVAL for a tabulated response (no cell function).
 * Synchronous on the model's stream. */
bx_status bx_model_cell_ceiling(bx_model* m, const double* theta, int32_t reps, double* cells_per_s);

/* ---- fitting (Sec. 4, steps 5-7) ---- */
typedef enum { BX_FIT = 0, BX_EVAL_GRAD = 1 } bx_request_kind;
typedef enum { BX_CONVERGED = 0, BX_MAXITER = 1, BX_FAILED = 2 } bx_fit_status;

typedef struct {
  int32_t kind;            /* bx_request_kind */
  const double* x0;        /* [P] start (FIT) or evaluation point (EVAL_GRAD) */
  const uint8_t* float_mask; /* [P] 1 = varied, 0 = fixed; NULL = all varied */
  const double* lo;        /* [P] lower bounds or NULL (rates and a floated pile-up
                              fraction default to 0) */
  const double* hi;        /* [P] upper bounds or NULL (a floated pile-up fraction
                              defaults to 1, the rest to none) */
  double edm_tol;          /* stop when EDM = g^T H^-1 g / 2 < edm_tol (<= 0: 1e-9) */
  int32_t max_iter;        /* quasi-Newton iterations (<= 0: 500) */
  int32_t max_eval;        /* NLL + gradient evaluations (<= 0: 200 + 100 n + 5 n^2,
                              n = varied parameters); reaching it ends the fit with
                              BX_MAXITER at the best point accepted so far */
  /* Mixed-precision fit: an FP64 model of the same fit (same description but
   * for the precision, same data; NULL = none).  The fit runs on the model it
   * was submitted with until EDM < polish_edm (or until its line search can
   * make no more progress), then evaluates again at that point with `polish`
   * and goes on from there, with the same Hessian approximation, until
   * EDM < edm_tol: FP32 cells for the bulk of the iterations, the minimum
   * and its EDM those of the FP64 model.  BX_E_INVAL if the shapes differ or
   * polish is not FP64; the server keeps `polish` busy like the model. */
  bx_model* polish;
  double polish_edm;       /* <= 0: 1e-8 */
} bx_fit_opts;

typedef struct {
  int32_t status;          /* bx_fit_status */
  double nll;
  double x[32];            /* parameters at the end (first P used) */
  double grad[32];         /* gradient at x */
  double edm;
  int32_t n_iter, n_eval;
  int64_t t_submit_ns, t_admit_ns, t_done_ns;   /* steady-clock timestamps */
} bx_fit_result;

/* Sec. 4, steps 5-7: vary the parameters until the likelihood is optimal
 * and hand the result back.  Plain path: fit one model on the calling thread
 * (host BFGS, one device evaluation per step). */
bx_status bx_fit(bx_model* m, const bx_fit_opts* o, bx_fit_result* r);

/* Sec. 4, steps 5-7 for a batch of fits at once (a toy study): fit model
 * models[i] from opts[i] (as for bx_fit, a polishing model included) for
 * i < n, with the fits' minimisers on the device.  Each fit is placed once
 * (inputs shared with its model, its own workspace); one iteration of all of
 * them -- the evaluation launches of every launch group, then a kernel that
 * runs each fit's minimiser step (one wave per fit) -- is captured as a HIP
 * graph and replayed until no fit is running, the host reading the count of
 * running fits every check_every replays (<= 0: 4).  results[i] equal
 * bx_fit's bit for bit (the minimiser is the same code, compiled for the
 * device with the same arithmetic).  The models must be on one device;
 * their pending work is waited for first.  Synchronous; the batch's device
 * memory is allocated and freed inside the call (BX_E_NOMEM if it does not
 * fit). */
bx_status bx_fit_batch(bx_model* const* models, const bx_fit_opts* opts, int32_t n, bx_fit_result* results,
                       int32_t check_every);

/* Sec. 4, steps 5-7 for many fits at once (toy studies, served requests).
 * Fit server: admits requests while their device memory fits hbm_budget_bytes
 * (0 = the device's free memory) and max_slots (<= 0: 4096), keeps each admitted
 * fit's parameters, optimiser state and histograms resident, and advances
 * every active fit by one quasi-Newton step per batched evaluation
 * (continuous batching: fits join and leave at step boundaries).  The server
 * owns a worker thread and its own stream (hip_stream NULL) or borrows one. */
bx_status bx_server_create(size_t hbm_budget_bytes, int32_t max_slots, void* hip_stream,
                           bx_server** out);
/* Sec. 4, step 7 for the server: finish the queued fits, then release the
 * worker, stream and device memory. */
bx_status bx_server_destroy(bx_server* s);

/* Sec. 4, step 5 (start a minimisation) or step 6 (one evaluation): queue
 * a request on model m (borrowed until the ticket reaches a terminal
 * state; the model's current data are copied at submission).  o is copied.
 * BX_E_BUSY if the request can never fit the budget. */
bx_status bx_fit_submit(bx_server* s, bx_model* m, const bx_fit_opts* o, uint64_t* ticket);

/* Sec. 4, step 7 (the minimum found, the result handed back): result of a
 * ticket: BX_PENDING while running; BX_OK with *r filled once
 * terminal (the ticket is then retired); BX_E_NOTFOUND otherwise. */
bx_status bx_fit_poll(bx_server* s, uint64_t ticket, bx_fit_result* r);

/* Sec. 4, step 7 for every queued fit: block until every submitted ticket
 * is terminal. */
bx_status bx_server_drain(bx_server* s);

/* The reason a call above failed (a domain error of Eqs. 1-4, a bad size,
 * a device error): message of the last error on the calling thread (static
 * storage). */
const char* bx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BX_H */
