/*
 * oci.h -- C ABI of the MI355X one-cell-inversion (OCI) transport library.
 *
 * The library solves transient, mono-energetic, isotropically scattering
 * slab-geometry S_N transport (Sec. "Derivation of MB-SCB", the S_N equation
 * with its initial and boundary conditions), discretised with simple corner
 * balance in space and multiple balance in time (eq:scb-mb-a .. eq:scb-mb-d,
 * with the cell-midpoint average closure and the upstream cell-edge closure).
 * Each time step is iterated to tolerance either by one-cell inversion
 * (Sec. "One-Cell Inversion (OCI)": every cell solves its dense 4N x 4N
 * all-angle system (A - S) Psi = c with the incident fluxes of its neighbours
 * from the previous iterate -- parallel block Jacobi) or by source iteration
 * (Sec. "Source Iteration (SI)": 4x4 solves per cell and angle in transport
 * sweeps with a lagged scalar flux).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Angles: N even, Gauss-Legendre (Sec. "ONE-CELL INVERSION": Gauss-Legendre
 *   in all explorations), ascending mu, so angles 0 .. N/2-1 have mu < 0 and
 *   angle N-1-m mirrors angle m; weights sum to 2.
 * Cells: J = sum of the region cell counts, numbered left to right; region r
 *   has uniform width dx_r = width_r / cells_r and data Sigma_r, Sigma_s,r, Q_r.
 * Scalar flux phi: [J][4] per cell, components
 *   phi_{k,L}, phi_{k,R}, phi_{k+1/2,L}, phi_{k+1/2,R}
 *   (time-average and time-edge values on the left and right half cells),
 *   phi = sum_n w_n psi_n (SI subsection).
 * Time-edge state psi_edge: [J][N][2] = psi_{m,k+1/2} on the L and R half
 *   cells of every cell and angle; it is the psi_{k-1/2} of the next step.
 * Stopping rule (the paper iterates "until the flux stops changing" without
 *   naming a norm; reading taken here): iterate l is accepted when
 *   e_l = max|phi^(l) - phi^(l-1)| / max|phi^(l)| <= tol over all cells and
 *   components; with OCI_FLAG_STRICT also e_l*rho/(1-rho) <= tol with
 *   rho = e_l/e_{l-1} clamped to [0, 0.9999].  OCI's first iterate of a step
 *   has no predecessor and is never accepted.
 * Warm start: the first step starts OCI from zero incident fluxes and SI from
 *   zero scalar flux; later steps start from the previous step's last iterate.
 * Reflecting edges: the incoming flux of angle m equals the outgoing flux of
 *   angle N-1-m at the same edge and time level; OCI takes it from the
 *   previous iterate (like every incident flux), SI sweeps the reflected
 *   direction second and takes it from the same iteration (when both edges
 *   reflect, the right edge is lagged by one iteration).
 * Streams: a context is bound to the HIP stream given to oci_setup; all GPU
 *   work is enqueued on it.  Calls on one context are not thread-safe;
 *   separate contexts are independent.
 * Memory: the library owns every device allocation it makes (in oci_setup,
 *   released by oci_destroy).  Caller buffers are only read or written during
 *   the call that receives them.  A pointer argument documented as "host or
 *   device" is a device pointer when the matching on_device flag is nonzero.
 * Errors: every int-returning call returns an OCI_* code; no C++ exception
 *   crosses this boundary.  oci_last_error() gives a message for the last
 *   failure on a context.  OCI_NOT_CONVERGED is positive: the step finished
 *   with its last iterate and the state advanced.
 */
#ifndef OCI_H
#define OCI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OCI_OK = 0,
  OCI_NOT_CONVERGED = 1, /* max_iters reached; state advanced with the last iterate */
  OCI_EINVAL = -1,       /* invalid argument; nothing was changed */
  OCI_ENOMEM = -2,       /* device allocation failed */
  OCI_EDEVICE = -3,      /* a HIP call failed */
  OCI_ENONFINITE = -4,   /* the scalar flux became NaN or Inf; the step is abandoned */
  OCI_ESTATE = -5        /* call not valid in the context's current state */
};

enum { OCI_BC_VACUUM = 0, OCI_BC_REFLECT = 1, OCI_BC_INCIDENT = 2 };

/* OCI_PREC_FP64: every iterate in FP64.  OCI_PREC_FP32: mixed precision,
 * FP64 defect correction with FP32 inner iterations (see oci_setup); the
 * accepted iterate of every step is still an FP64 application of the
 * operator, judged by the same stopping rule. */
enum { OCI_PREC_FP64 = 0, OCI_PREC_FP32 = 1 };

/* flags */
#define OCI_FLAG_STRICT 1u /* add the a-posteriori error bound to the stopping rule */
#define OCI_FLAG_COMPACT 2u /* iterate rings of at most 64 MiB (at least 7 slots per step
                               parity instead of 9): for many contexts side by side */

#define OCI_MAX_ANGLES 256

typedef struct oci_ctx oci_ctx;

/* Problem description, read only during oci_setup (which copies it). */
typedef struct {
  int32_t n_angles;          /* N: even, 2 .. OCI_MAX_ANGLES */
  const double *mu, *w;      /* [N] quadrature override (ascending, mirror-symmetric,
                                nonzero mu), or both NULL for Gauss-Legendre */
  int32_t n_regions;         /* R >= 1 */
  const int32_t *cells;      /* [R] cells per region, each >= 1 */
  const double *width;       /* [R] region widths, > 0 */
  const double *sigma_t;     /* [R] total cross sections, > 0 */
  const double *sigma_s;     /* [R] scattering cross sections, >= 0 */
  const double *source;      /* [R] isotropic sources Q, >= 0, time-constant */
  double dt;                 /* time step, > 0 */
  double speed;              /* particle speed v, > 0; +inf gives the steady equations */
  int32_t bc_left, bc_right; /* OCI_BC_* */
  const double *inc_left;    /* [N/2] incident psi at x = 0 for the mu > 0 angles
                                (ascending), time-constant; required iff bc_left is
                                OCI_BC_INCIDENT */
  const double *inc_right;   /* [N/2] incident psi at x = X for the mu < 0 angles */
  const double *psi0;        /* [J][N][2] initial psi on the L and R half cells, or NULL = 0 */
  double tol;                /* stopping tolerance, >= 0 */
  int32_t max_iters;         /* >= 1 iterations per step */
  int32_t precision;         /* OCI_PREC_FP64 or OCI_PREC_FP32 (not with OCI_FLAG_STRICT) */
  uint32_t flags;            /* OCI_FLAG_* */
} oci_problem;

typedef struct {
  int32_t iterations;  /* iterations done in the step (OCI_PREC_FP32: FP64 iterates) */
  int32_t status;      /* OCI_OK, OCI_NOT_CONVERGED or OCI_ENONFINITE */
  double residual;     /* e of the accepted (or last) iterate; -1 if undefined */
  double ms;           /* stream time of the step, milliseconds; steps queued
                          together share their window's time evenly */
  double iter_ms;      /* source iteration: stream time of the iteration
                          launches alone; OCI: for a step resumed after its
                          queued launches left it undecided, the time of the
                          resumed part, otherwise equal to ms */
  int32_t launches;    /* iterates computed for the step (>= iterations:
                          a queued step computes a planned count and its end
                          picks the accepted one; OCI_PREC_FP32: FP64 and FP32
                          iterates), in kernels of up to
                          oci_iterates_per_launch() iterates each */
  int32_t corrections;  /* learned corrections kept in the step (oci_set_corrector) */
  double err_bound;    /* a-posteriori error bound of the accepted iterate:
                          e_l rho / (1 - rho) with rho = e_l / e_{l-1} clamped to
                          [0, 0.9999] (the bound OCI_FLAG_STRICT tests against
                          tol); -1 when e_{l-1} is undefined (l = 1 of OCI) and
                          always with OCI_PREC_FP32, whose consecutive FP64
                          iterates do not give OCI's contraction rate */
} oci_step_info;

/* Build a context: validates *p, computes the quadrature, uploads the region
 * table, solves every region's cell system (A - S) Y = [B | T | q] on the
 * GPU (one solve per region because all cells of a region share A - S;
 * Sec. "PERFORMANCE ANALYSIS" does it by dense LU, here it goes through the
 * rank-4 scattering coupling: the same solution up to rounding), and forms
 * the operators applied each iteration.  hip_stream is a hipStream_t
 * (NULL = the null stream).  On success *out owns all device memory.
 * With precision OCI_PREC_FP32 a step is solved by defect correction: each
 * FP64 iterate x' = T(y) (one OCI iteration of the current point y) gives the
 * defect d = x' - y; the correction c = G c + d (the same block-Jacobi
 * iteration without its constant part, Sec. "One-Cell Inversion (OCI)") is
 * iterated in FP32 and y + c is the next point.  The first FP64 iterate
 * starts from the previous step's accepted one; a step's FP64 iterates are
 * judged by the OCI stopping rule (Sec. "One-Cell Inversion (OCI)": relative
 * change of the scalar flux), so the result is an FP64 iterate.  max_iters then bounds
 * the FP64 iterates.
 * Launch shape: a queued FP64 step runs its iterates in launches of up to
 * four (each launch recomputes the halo cells it needs on the tile's edges);
 * the environment variable OCI_ITERATES_PER_LAUNCH = 1, 2, 3 or 4, read here,
 * caps that number (results agree to rounding order either way).
 * Errors: OCI_EINVAL (bad problem, out == NULL), OCI_ENOMEM, OCI_EDEVICE. */
int oci_setup(const oci_problem *p, void *hip_stream, oci_ctx **out);

/* Rebuild every region's operator for new region data (widths, cross
 * sections, sources, dt, speed, tolerance) without reallocating: p must have
 * the same n_angles, n_regions, cells, boundary-condition kinds and quadrature
 * as the problem the context was built with (else OCI_EINVAL, context
 * unchanged).  The time-edge state and the warm-start iterate are kept; psi0
 * and the incident fluxes of p are ignored. */
int oci_refactor(oci_ctx *c, const oci_problem *p);

/* Advance one MB time step with OCI iterations to the stopping rule
 * (Sec. "One-Cell Inversion (OCI)").  info may be NULL.
 * Returns OCI_OK, OCI_NOT_CONVERGED, OCI_ENONFINITE or a negative error. */
int oci_step(oci_ctx *c, oci_step_info *info);

/* Advance one MB time step with source iteration (Sec. "Source Iteration
 * (SI)"): the same step, the same stopping rule, on the same state, so OCI
 * and SI steps may be mixed on one context.  max_iters = 1 gives one sweep. */
int si_step(oci_ctx *c, oci_step_info *info);

/* n_steps >= 0 calls of oci_step.  phi_out (host or device, per
 * phi_out_on_device) receives [n_steps][J][4] scalar fluxes, or is NULL;
 * infos receives [n_steps] records, or is NULL.  Stops early at the first
 * negative code and returns it; otherwise returns OCI_NOT_CONVERGED if any
 * step did not converge, else OCI_OK. */
int oci_solve(oci_ctx *c, int32_t n_steps, double *phi_out, int32_t phi_out_on_device,
              oci_step_info *infos);

/* A batch of independent problems: oci_solve(ctx[i], n_steps, phi_out[i],
 * phi_out_on_device, infos[i]) for i < n_ctx, with the contexts driven
 * concurrently by up to n_threads host threads (0: min(n_ctx, 16)), each
 * taking the next unsolved context, so that the problems' launches overlap on
 * the GPU.  The contexts must be distinct, and to overlap they must be bound
 * to distinct streams.  phi_out and infos may be NULL, or hold NULL entries.
 * Returns the first negative code in context order (that context's
 * oci_last_error has the message; the other contexts still ran), else
 * OCI_NOT_CONVERGED if any step of any context did not converge, else
 * OCI_OK.  OCI_EINVAL: n_ctx < 1, a NULL or repeated context, n_steps < 0. */
int oci_solve_batch(oci_ctx **ctx, int32_t n_ctx, int32_t n_steps, double **phi_out,
                    int32_t phi_out_on_device, oci_step_info **infos, int32_t n_threads);

/* An ensemble of independent problems advanced together: n_steps OCI steps of
 * every context.  Each step makes one launch per iteration, or per three or
 * four iterations for N = 8 .. 64 (up to the context's iterates-per-launch
 * cap), for each angle count and launch shape present.  Each launch runs over
 * a device work queue of (problem, tile) entries covering the tiles of every
 * such problem; kernels are built for N = 8 .. 128 where the count is one of
 * those, else for any N.  A problem keeps its own operators, iterate rings,
 * residual records and control block, so its iterates, stopping decisions
 * and results are those of its own steps (to rounding).  Then one
 * end-of-step launch runs over all tiles; problems
 * still undecided continue in further launches over their own tiles only
 * (per-problem flags), while the decided ones wait for the next step.  All
 * work goes to the first context's stream (the other contexts' streams are
 * waited for first).  Contexts: distinct, OCI_PREC_FP64, no corrector, N a
 * multiple of 8, all at the same step parity (e.g. all fresh).  phi_out: NULL
 * or [n_ctx] device pointers (NULL entries allowed) receiving [n_steps][J][4];
 * infos: NULL or [n_ctx] arrays of n_steps records (NULL entries allowed;
 * ms is the whole ensemble's step time).  The call allocates its own work
 * tables (device memory and a pinned host staging buffer, a few tens of bytes
 * per tile and an argument block per problem) and frees them before it
 * returns.  Returns OCI_OK, OCI_NOT_CONVERGED
 * (some step of some context) or the first error (OCI_ENONFINITE abandons that
 * context's step as oci_step does and stops the ensemble). */
int oci_solve_ensemble(oci_ctx **ctx, int32_t n_ctx, int32_t n_steps, double **phi_out,
                       oci_step_info **infos);

/* Scalar flux of the last completed step, [J][4] (host or device).
 * OCI_ESTATE before the first step. */
int oci_get_flux(oci_ctx *c, double *phi, int32_t on_device);

/* Copy out the time-edge state [J][N][2] (host) and the number of completed
 * steps.  Together with the warm-start iterate kept inside the context this
 * is everything a later step reads; set_state restarts from psi_edge with a
 * cold iterate (zero incident fluxes, zero scalar flux), exactly like the
 * first step.  Either pointer may be NULL. */
int oci_get_state(oci_ctx *c, double *psi_edge, int64_t *step);
int oci_set_state(oci_ctx *c, const double *psi_edge, int64_t step);

/* Quadrature and problem sizes of a context (host outputs; any may be NULL). */
int oci_get_quadrature(const oci_ctx *c, double *mu, double *w);
int oci_get_sizes(const oci_ctx *c, int32_t *n_angles, int32_t *n_cells, int32_t *n_regions);

/* Launch shape of a queued FP64 step: the most iterates one iteration kernel
 * computes (a launch of k > 1 iterates stages its tile with k-1 halo cells on
 * each side and recomputes them level by level, Sec. "One-Cell Inversion
 * (OCI)": each cell's iterate needs only its neighbours' previous iterate).
 * 1 with OCI_PREC_FP32.  Returns the count (>= 1), or OCI_EINVAL for NULL. */
int oci_iterates_per_launch(const oci_ctx *c);

/* Set the launch shape: at most k (>= 1) iterates per iteration kernel,
 * clamped to what the problem allows (up to 4 for N = 8, 16, 32, 64, fewer
 * where a region is narrower than three cells, else 2; a fresh context starts
 * at that limit,
 * except from N = 128 on, where it starts at 1: the two-iterate kernel is
 * slower per iterate there).  Results do not depend on it
 * (the iterates are the same; only their grouping into launches changes);
 * it is a tuning knob (see the autotuner in the Python package).  Waits for
 * the context's stream when the shape changes (cached step graphs are
 * rebuilt); not to be called while another thread drives the context.
 * Returns the shape now in effect (1 with OCI_PREC_FP32, where it has no
 * effect), or OCI_EINVAL for NULL or k < 1. */
int oci_set_iterates_per_launch(oci_ctx *c, int32_t k);

/* Whether the end of a queued step also computes the next step's first
 * iterate (1, the default) or leaves it to the next step's iteration launches
 * (0).  Iterate 1 of step k+1 reads only the cell's new step constant and its
 * neighbours' accepted outgoing fluxes (Sec. "One-Cell Inversion (OCI)"), so
 * the end of step k can form it; whether that pays depends on the problem
 * (one launch fewer per step against a longer end-of-step kernel and one
 * iterate fewer per iteration launch).  Results do not depend on it (same
 * iterates, grouped differently); it is a tuning knob like the iterates per
 * launch, with the same waiting and threading rules.  oci_set_end_fusion
 * returns the setting now in effect (0 or 1), or OCI_EINVAL for NULL. */
int oci_end_fusion(const oci_ctx *c);
int oci_set_end_fusion(oci_ctx *c, int32_t on);

/* Mixed precision (OCI_PREC_FP32): FP32 inner iterations per correction.
 * By default the count is searched while a solve runs (doubled when a window
 * of queued steps needs four or more FP64 iterates per step, else lowered by
 * one until that costs an FP64 iterate).  oci_set_inner_iterations with m in
 * [1, 64] fixes it (a tuning knob: the accepted iterates are still FP64
 * iterates judged by the stopping rule; only their number and the work between
 * them change), m = 0 returns to the search from the current count.  Waits
 * for the context's stream when the count changes (cached step graphs are
 * rebuilt).  Both return the count in effect, 0 for an FP64 context, or
 * OCI_EINVAL (NULL, m outside [0, 64]). */
int oci_inner_iterations(const oci_ctx *c);
int oci_set_inner_iterations(oci_ctx *c, int32_t m);

/* Per-region operator, for inspection and tests: [2N+4+2N][4N+1] row-major,
 * rows = (outgoing flux 2N, phi 4, psi_edge 2N), columns = (incident flux 2N,
 * psi_{k-1/2} 2N, source 1), i.e. the needed rows of (A - S)^{-1} applied to
 * the columns through which the cell's right-hand side c enters.
 * Outgoing / incident order: index 2m+t, t = 0 level k, 1 level k+1/2; the
 * first N entries are the mu < 0 angles (left-half flux leaving / right
 * neighbour's left-half flux entering), the last N the mu > 0 angles. */
int oci_get_operator(oci_ctx *c, int32_t region, double *op);

/* Release everything the context owns (waits for its stream).  NULL is a no-op. */
void oci_destroy(oci_ctx *c);

const char *oci_strerror(int code);
const char *oci_last_error(const oci_ctx *c);

/* Host-only helper: the N-point Gauss-Legendre rule, ascending (no GPU use).
 * Returns OCI_EINVAL for n < 1 or n > 4096 or NULL outputs. */
int oci_gauss_legendre(int32_t n, double *mu, double *w);

/* ---- Learned iterate corrector ----
 * A small network that learns, from OCI iterate histories the solver
 * generates, the remaining error of an iterate from its latest differences,
 * to damp OCI's slow convergence in optically thin cells (the weakness the
 * paper states in its introduction and conclusions; the paper itself has no
 * corrector).  Network: four 1-D convolutions over cells, kernel width 5
 * with two cells of zero padding at each mesh end, 32 channels between
 * layers, no biases, ReLU after the first three (positively homogeneous:
 * f(a x) = a f(x), a > 0).  Loss: mean squared error over all outputs.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8).  FP64.
 * Layout: inputs x [batch][c_in][cells], outputs [batch][c_out][cells],
 * cells contiguous; weights of layer l [c_o][c_i][5], the four layers
 * concatenated (oci_corrector_num_weights() doubles).
 * Device pointers (x, y, target) must hold the sizes stated and stay valid
 * until the call returns; every call runs on the stream given at creation
 * and returns after it completes, except oci_corrector_forward, which only
 * enqueues.  A corrector keeps its activations between the forward and
 * backward passes: calls on one corrector must not overlap (one host thread,
 * one stream).  Errors: OCI_EINVAL (NULL pointer, batch or cells outside
 * [1, the maximum given at creation], channels not multiples of 4),
 * OCI_ENOMEM, OCI_EDEVICE; oci_corrector_last_error() gives the message. */
typedef struct oci_corrector oci_corrector;

/* c_in, c_out: multiples of 4 in [4, 1024]; max_batch * max_cells sizes the
 * activation buffers.  Weights and Adam moments start at zero. */
int oci_corrector_create(int32_t c_in, int32_t c_out, int32_t max_batch, int32_t max_cells,
                         void *hip_stream, oci_corrector **out);
/* Number of weights (>= 0), or OCI_EINVAL for NULL. */
int64_t oci_corrector_num_weights(const oci_corrector *k);
/* Copy all weights from / to host memory; setting them also clears Adam's
 * moments and step count. */
int oci_corrector_set_weights(oci_corrector *k, const double *w);
int oci_corrector_get_weights(oci_corrector *k, double *w);
/* y = f(x) (device pointers; enqueued on the stream, not waited for). */
int oci_corrector_forward(oci_corrector *k, const double *x, int32_t batch, int32_t cells,
                          double *y);
/* Mean squared error of f(x) against target (device pointers) and its
 * gradient wrt every weight: *loss and grad[num_weights] are host memory,
 * either may be NULL. */
int oci_corrector_grad(oci_corrector *k, const double *x, const double *target, int32_t batch,
                       int32_t cells, double *loss, double *grad);
/* The gradient, then one Adam step of learning rate lr > 0; *loss (host, may
 * be NULL) is the loss before the step. */
int oci_corrector_train_step(oci_corrector *k, const double *x, const double *target,
                             int32_t batch, int32_t cells, double lr, double *loss);
/* FP32 inference on the matrix cores (v_mfma_f32_16x16x4f32): y = f(x) with the
 * weights rounded to FP32, x [batch][c_in][cells] and y [batch][c_out][cells]
 * FP32 device pointers; enqueued on the corrector's stream, not waited for.
 * c_in and c_out at most 32, else OCI_EINVAL. */
int oci_corrector_forward32(oci_corrector *k, const float *x, int32_t batch, int32_t cells,
                            float *y);
const char *oci_corrector_last_error(const oci_corrector *k);

/* Learned corrections inside the OCI iteration of a context (OCI_PREC_FP64).
 * With a corrector attached (8 or 12 input channels, 4 outputs, taking at
 * least J cells), every OCI step is driven from the host in batches of
 * single-iterate launches, and iterate l = first, first + period, ... of a
 * step (when not accepted) is corrected: the corrector predicts a scalar-flux
 * correction dphi from [phi^(l) - phi^(l-1), phi^(l-1) - phi^(l-2)] (and with
 * 12 channels also rho/(1-rho) (phi^(l) - phi^(l-1)), rho = e_l / e_{l-1}
 * clamped to [0, 0.9999]) in FP32 on the matrix cores; the iterate's scalar
 * flux becomes phi^(l) + dphi and each outgoing
 * flux moves by the isotropic angular flux of that change on its half cell
 * and time level, dphi / sum(w) (the slow error of OCI in thin, scattering
 * cells, Sec. "ONE-CELL INVERSION", is the nearly isotropic scattering mode;
 * it lives in the incident fluxes the next iterate reads, Sec. "One-Cell
 * Inversion (OCI)").  Iterate l+1 is the plain
 * OCI iterate of that point; it is kept when its change e_{l+1} is below
 * rho e_l (rho = e_l / e_{l-1}: the correction lowered the residual below what
 * a plain iterate reaches), otherwise iterate l is restored bit for bit,
 * iterate l+1 recomputed from it and the period to the next correction
 * doubled (up to 1024; back to `period` after a kept correction).  Every accepted iterate is therefore a plain OCI iterate of its
 * predecessor judged by the stopping rule, and with a corrector whose every
 * correction is rejected the steps equal plain host-driven steps bit for bit.
 * The corrector must outlive its attachment and not be used by another
 * stream meanwhile.  k = NULL detaches.  oci_step_info.corrections counts the
 * kept corrections.  OCI_EINVAL: NULL context, mixed precision, first < 3,
 * period < 1, wrong channel counts or too few cells; OCI_ENOMEM. */
int oci_set_corrector(oci_ctx *c, oci_corrector *k, int32_t first, int32_t period);

/* One plain OCI step (as oci_step, driven from the host in batches of
 * single-iterate launches) that also copies the scalar flux of its iterates
 * first .. first + n_hist - 1, as they are formed, into phi_hist
 * [n_hist][J][4] (host or device per on_device; entries past the accepted
 * iterate are left as they were).  Training data for the corrector, from one
 * solve, O(n_hist) copies.  OCI_EINVAL: first < 1, n_hist < 0, phi_hist NULL
 * with n_hist > 0, mixed precision. */
int oci_step_history(oci_ctx *c, int32_t first, int32_t n_hist, double *phi_hist,
                     int32_t on_device, oci_step_info *info);
/* Release the corrector (waits for its stream).  NULL is a no-op. */
void oci_corrector_destroy(oci_corrector *k);

/* Allocation-free forward pass, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): y = f(x) for the network with c_in inputs and c_out
 * outputs (multiples of 4 in [4, 1024]) whose weights w sit in device memory
 * in the layout of oci_corrector_num_weights() / _get_weights().  x
 * [batch][c_in][cells] and y [batch][c_out][cells] are device pointers
 * (caller-owned).  The hidden activations live in a fixed device array of
 * the library (32 MiB per GPU, held until the process ends), which limits
 * batch * cells to 65,536; nothing in it needs to start at zero.  Enqueued on
 * hip_stream (a hipStream_t, NULL = the null stream), not waited for; calls
 * that overlap on one GPU (other streams, other threads) share that array and
 * race.  No allocation, no synchronisation.  Returns OCI_OK, OCI_EINVAL (NULL
 * pointer, channels or sizes out of range; nothing enqueued) or OCI_EDEVICE. */
int oci_corrector_forward_noalloc(const double *w, int32_t c_in, int32_t c_out, const double *x,
                                  int32_t batch, int32_t cells, double *y, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* OCI_H */
