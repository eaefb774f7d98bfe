/*
 * ncs.h -- C ABI of the near-circulant splitting (NCS) solver for gfx950.
 *
 * Method (Ryu, Ko, Won, "Splitting with Near-Circulant Linear Systems:
 * Applications to Total Variation CT and PET"): minimize g(Ax - b) (eq. RCP)
 * with the iteration of eq. (NCS)
 *
 *     x+ = x - M^+ A^T u
 *     u+ = prox_{alpha g*}(u + alpha (A(2x+ - x) - b)),
 *
 * where M = gamma I + alpha C is circulant and applied through the FFT
 * (Section 1.2).  The library implements the CT and PET instances of
 * Section 4: A stacks a parallel-beam projector E with the scaled finite
 * differences (beta/alpha) D; the data term is 1/2 |y|^2 (CT, Section 4.1) or
 * the Poisson negative log-likelihood (PET, Section 4.2); the TV term is
 * anisotropic |Dx|_1 (the paper) or isotropic sum_p |(Dx)_p|_2.
 *
 * Conventions shared by every call:
 *
 *  - Geometry: an N x N image of unit pixels stored row-major (index
 *    r*N + c, row r along y), N_theta angles theta_a = pi a / N_theta and N_s
 *    unit detector bins centred on the image centre; sinograms are stored
 *    angle-major (index a*N_s + d).  The projector is the Joseph ray-driven
 *    discretisation of the Radon transform of eq. (radon-def) (Section 2);
 *    rays step through rows when 4a <= N_theta or 4a >= 3 N_theta, else
 *    through columns.  N must be a power of two in [16, 1024]; N_theta >= 1;
 *    N_s >= 2.
 *  - Precision: a handle is created for NCS_F32 or NCS_F64.  Every device
 *    buffer passed to it holds float (NCS_F32) or double (NCS_F64); all
 *    scalars returned to the host are double.  Reductions (objective,
 *    residuals) are accumulated in double in both modes.
 *  - Memory: pointers named *_dev are device pointers on the device that was
 *    current when the handle was created; the caller owns them and keeps
 *    them alive while the handle uses them (b and bg for the handle's life).
 *    The library owns its workspace (iterates, spectra, tables, partial sums)
 *    from ncs_setup to ncs_destroy.  Host pointers are read or written
 *    before the call returns.
 *  - Streams: work is queued on the hipStream_t given to ncs_setup (NULL is
 *    the default stream).  Calls that return host values synchronise that
 *    stream; the others return once the work is queued.
 *  - Errors: no C++ exception crosses this interface.  Arguments are checked
 *    before anything is queued; a failing call returns a negative status and
 *    leaves a message for ncs_last_error().  Iterations that produce a NaN
 *    objective stop on the device and report NCS_ERR_NONFINITE.
 *  - Threads: a handle is used by one host thread at a time.
 */
#ifndef NCS_H
#define NCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NCS_OK = 0,
    NCS_NOT_CONVERGED = 1,     /* ncs_solve: iteration budget used before the target */
    NCS_ERR_INVALID_ARG = -1,  /* bad size, pointer, parameter or state */
    NCS_ERR_HIP = -2,          /* a HIP runtime call failed */
    NCS_ERR_OOM = -3,          /* device allocation failed */
    NCS_ERR_NONFINITE = -4,    /* the objective became NaN */
    NCS_ERR_DIVERGED = -5      /* the objective grew for the configured number of checks */
} ncs_status;

typedef enum { NCS_F32 = 0, NCS_F64 = 1 } ncs_dtype;

/* Data term g_data: 1/2|y|^2 (Section 4.1) or sum l(y_i + r_i; b_i) (Section 4.2). */
typedef enum { NCS_DATA_QUADRATIC = 0, NCS_DATA_POISSON = 1 } ncs_data_term;

/* TV term: anisotropic |Dx|_1 (Section 4.1, box projection Pi_[-s,s]) or
 * isotropic sum_p |(Dx)_p|_2 (per-pixel l2-ball projection). */
typedef enum { NCS_TV_ANISO = 0, NCS_TV_ISO = 1 } ncs_tv_term;

/* Beam geometry.  Parallel: N_theta angles over [0, pi), unit bins (Section
 * 4.1).  Fan (Section 4.1.1, divergent beam): N_theta source positions
 * S_a = R_s (cos beta_a, sin beta_a), beta_a = 2 pi a / N_theta, over a full
 * turn; N_s bins on an equi-angular detector whose fan just covers the circle
 * of radius N / sqrt(2) around the image (ray d leaves S_a at angle
 * beta_a + pi + (d - (N_s-1)/2) dgamma, dgamma = 2 asin(N / (sqrt(2) R_s)) /
 * (N_s - 1)); Joseph interpolation along each ray's own stepping axis. */
typedef enum { NCS_BEAM_PARALLEL = 0, NCS_BEAM_FAN = 1 } ncs_beam;

typedef struct {
    int32_t n_side;    /* N: image is N x N */
    int32_t n_angles;  /* N_theta: parallel angles, or fan source positions */
    int32_t n_bins;    /* N_s */
    int32_t beam;      /* ncs_beam */
    double source_radius; /* fan: R_s in pixels, > 1.01 N / sqrt(2); ignored for parallel */
} ncs_geometry;

/* The splitting: NCS with the circulant M of Section 4.1.1; PDHG (eq. PDHG,
 * Section 1), the same iteration with M = gamma I; or ADMM (eq. DRS/ADMM),
 * M = alpha A^T A, with each linear system solved by cg_iters conjugate-
 * gradient steps from zero (Section 5's comparison method), optionally
 * preconditioned by alpha M^+ with the NCS circulant M (single slices only). */
typedef enum { NCS_METHOD_NCS = 0, NCS_METHOD_PDHG = 1, NCS_METHOD_ADMM_CG = 2 } ncs_method;

typedef struct {
    double alpha;      /* > 0: dual step alpha of eq. (NCS) */
    double beta;       /* > 0: TV block scaling, A = [E; (beta/alpha) D] (Section 4.1) */
    double gamma;      /* >= 0: M = gamma I + alpha C (Section 1.2) */
    double lambda;     /* >= 0: TV weight */
    double c_r;        /* C_R of eq. (circ_R); <= 0 selects N_theta N / pi */
    double mu_dc;      /* DC eigenvalue of M (Section 4.1.1, Remark on the DC
                          component); <= 0 selects gamma + alpha |E 1|^2 / n */
    int32_t data_term; /* ncs_data_term */
    int32_t tv_term;   /* ncs_tv_term */
    int32_t check_every;    /* ncs_solve: iterations between host checks; <= 0 selects 50 */
    int32_t diverge_checks; /* ncs_solve: stop with NCS_ERR_DIVERGED after this many
                               consecutive checks with a growing objective; <= 0 disables */
    int32_t projector; /* forward-projector kernel: 0 = time all at setup and keep the
                          fastest, 1 = each step's 96-element row window copied through LDS
                          (two steps' windows per 16-byte load), 2 = direct loads, one
                          8-byte gather per ray and step, 3 = two adjacent rays per lane,
                          one 16-byte load per step */
    int32_t graph_chunk; /* largest number of iterations per replayed HIP graph; 0 selects 32,
                            < 0 disables graphs (every kernel launched directly).  One graph
                            per power of two up to it is captured at the first iteration
                            request, so every count k is replayed (largest chunk repeated,
                            then the binary digits of the remainder). */
    double dual_ramp;    /* ncs_set_init with dual_from_x0: width tau of the ramp of the TV
                            dual, v = s clamp(D x0 / tau, -1, 1) (anisotropic) or
                            s (D x0)_p / max(|(D x0)_p|, tau) (isotropic); <= 0 gives the
                            sign, v = s sign(D x0) */
    int32_t backprojector; /* backprojector kernel: 0 = time all at setup and keep the fastest,
                              1 = LDS-staged detector windows (16 x 16 pixel tiles,
                                  2 x 2 pixels per lane),
                              2 = direct global loads (8 x 8 pixel tiles),
                              3 = 2 x 2 pixels per lane, one 16-byte load per angle */
    int32_t method;        /* ncs_method: NCS (M circulant), PDHG (M = gamma I; needs
                              gamma > alpha lambda_max(A^T A) to converge) or ADMM-CG */
    int32_t cg_iters;      /* ADMM-CG: CG steps per linear solve; 0 selects 10 */
    int32_t cg_precondition; /* ADMM-CG: 1 = precondition CG with alpha M^+, 0 = plain CG
                                (double precision only: NCS_F32 gives NCS_ERR_INVALID_ARG,
                                since plain CG amplifies single-precision rounding by about
                                the condition number of A^T A) */
    int32_t positivity;    /* 1: constrain x >= 0 (remark in Section 4.2): A gains the rows I with
                              the indicator of the nonnegative orthant in g, a dual t (N*N,
                              zero at ncs_set_init) updated as t = min(t + alpha xbar, 0), the
                              backprojection gains alpha t and, for NCS, every eigenvalue of M
                              is raised by alpha (for PDHG, gamma must cover the extra rows).
                              The reported objective leaves out the indicator.  Not with
                              ADMM-CG. */
    int32_t probes;        /* > 0: E^T E's multiplier estimated by eq. H-fan from this many
                              probes (Rademacher images from SplitMix64 seeded by the probe
                              index; least-squares average of (F E^T E v)_i / (F v)_i) instead
                              of alpha C_R / |omega|; 0: the analytic multiplier for parallel
                              beams and 16 probes for fan beams.  The products E^T E v run
                              through the library's double-precision kernels for handles of
                              either precision (a single-precision handle builds a temporary
                              double-precision twin at setup), so both run the same M. */
} ncs_params;

typedef struct ncs_handle ncs_handle;

/* Create a solver.  b_dev (N_theta*N_s values: CT sinogram or PET counts) may
 * be NULL for a handle used only for the operators below; bg_dev is the PET
 * background r (N_theta*N_s values, NULL = zero) and is ignored for CT.
 * Precomputes, in double precision on the host, the per-angle table, the
 * Fourier multiplier h = 1/mu of Section 4.1.1 (eq. circ_R + eq. circ_D,
 * DC entry mu_dc) and the FFT twiddles, and sets the state to x = u = v = 0.
 * stream is a hipStream_t (NULL = default stream). */
ncs_status ncs_setup(const ncs_geometry* geom, const ncs_params* params, int32_t dtype,
                     const void* b_dev, const void* bg_dev, void* stream,
                     ncs_handle** out);

/* Reset the iterate: x = x0 (NULL = zeros), iteration counter 0.  With
 * dual_from_x0 = 0 the duals are u = 0, v = 0.  With dual_from_x0 = 1 they
 * are taken from the fixed-point relations of the optimality conditions
 * (Section 3.2, Fact on fixed points): u = grad g_data(E x0) and
 * v = s sign(D x0) (anisotropic) or s (D x0)/|(D x0)_p| (isotropic) where the
 * difference is nonzero, 0 elsewhere, with s = lambda alpha / beta.  With
 * params.dual_ramp = tau > 0 the sign is replaced by the ramp
 * clamp(D x0 / tau, -1, 1), so that near-flat regions of x0 (where the
 * optimal v is strictly inside [-s, s]) start near v = 0. */
ncs_status ncs_set_init(ncs_handle* h, const void* x0_dev, int32_t dual_from_x0);

/* Replace the iterate x by x_dev (N*N values) and recompute E x; the duals
 * u, v and the iteration count are kept.  This is the restart point of the
 * learned warm start (ncs_cnn.h): a few plain iterations, a corrected x,
 * then NCS continues with its own duals. */
ncs_status ncs_set_x(ncs_handle* h, const void* x_dev);

/* Run exactly k >= 0 iterations (each: one x-update, one (u, v)-update, one
 * objective f(x^{k+1}) in double).  obj_host (length k, may be NULL) receives
 * the objective after each iteration; when it is non-NULL the call
 * synchronises.  Returns NCS_ERR_NONFINITE if an objective was NaN; the
 * iterations queued after it do nothing, and the state holds the values of
 * the iteration that produced the NaN. */
ncs_status ncs_iterate(ncs_handle* h, int32_t k, double* obj_host);

/* Iterate until f(x^k) <= f_target (NaN: no target), at most max_iters
 * iterations.  The objective is tested on the device after every iteration;
 * the host checks every params.check_every iterations.  fp_residual_tol > 0
 * adds a second stop, tested at those checks only: the fixed-point residual
 * of the primal iterate |x^k - x^{k-1}|_2 <= fp_residual_tol |x^k|_2 (the
 * iterates converge to a fixed point of the NCS map, Theorem 1, so the step
 * vanishes; it is formed in double from x^k and xbar = 2 x^k - x^{k-1}, so
 * with NCS_F32 its floor is about 1e-7).  fp_residual_tol <= 0 disables it;
 * NaN is NCS_ERR_INVALID_ARG.  iters_done and f_final (either may be NULL)
 * receive the iterations run in this call and the last objective.  Returns
 * NCS_OK when the target or the residual tolerance was reached,
 * NCS_NOT_CONVERGED when the budget ran out, or an error. */
ncs_status ncs_solve(ncs_handle* h, int32_t max_iters, double f_target, double fp_residual_tol,
                     int32_t* iters_done, double* f_final);

/* Objective history: obj_host[i] = f after iteration first + i (iterations
 * counted from the last ncs_set_init), for the most recent 65536 iterations. */
ncs_status ncs_get_objectives(ncs_handle* h, int32_t first, int32_t count, double* obj_host);

/* Number of iterations since the last ncs_set_init (host value). */
ncs_status ncs_get_iteration(ncs_handle* h, int32_t* iters);

/* Copy the current image x (N*N values, row-major) to x_out_dev. */
ncs_status ncs_get_x(ncs_handle* h, void* x_out_dev);

/* Copy the current data dual u (N_theta*N_s values) to u_out_dev. */
ncs_status ncs_get_u(ncs_handle* h, void* u_out_dev);

/* Copy the current TV dual v (2*N*N values: the horizontal-difference plane,
 * then the vertical one, each row-major) to v_out_dev. */
ncs_status ncs_get_v(ncs_handle* h, void* v_out_dev);

/* Copy the positivity dual t (N*N values, row-major; params.positivity = 1
 * only, NCS_ERR_INVALID_ARG otherwise) to t_out_dev. */
ncs_status ncs_get_t(ncs_handle* h, void* t_out_dev);

/* Checkpoint: the full state (x, u, v, E x, t, iteration count) as an opaque
 * host blob.  With host_buf NULL, *bytes receives the size needed.  Resuming
 * from a saved state reproduces the uninterrupted run bit for bit. */
ncs_status ncs_get_state(ncs_handle* h, void* host_buf, size_t* bytes);
ncs_status ncs_set_state(ncs_handle* h, const void* host_buf, size_t bytes);

/* Operators of the handle's geometry, usable without data:
 *   ncs_forward:   y = E x      (x: N*N, y: N_theta*N_s)
 *   ncs_adjoint:   x = E^T y
 *   ncs_apply_minv: out = M^+ w = F^-1 diag(h) F w (N*N real, Section 4.1)
 *   ncs_objective: f(x) for the handle's data term, TV term and lambda. */
ncs_status ncs_forward(ncs_handle* h, const void* x_dev, void* y_dev);
ncs_status ncs_adjoint(ncs_handle* h, const void* y_dev, void* x_dev);
ncs_status ncs_apply_minv(ncs_handle* h, const void* w_dev, void* out_dev);
ncs_status ncs_objective(ncs_handle* h, const void* x_dev, double* f);

/* y = E x like ncs_forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no handle, no allocation of any kind.  Parallel beam
 * (geom->beam = 0), single precision; x_dev: N*N floats, row-major; y_dev:
 * N_theta*N_s floats (a*N_s + d); both caller-owned device memory.  The
 * projector is the direct kernel (projector 2).  Its workspace (descriptor,
 * angle tables, the padded image and its transpose) lives in one fixed
 * 6 MiB device array per GPU, held until the process ends; geometries whose
 * workspace exceeds it (about 2 N (N + 192) * 4 bytes plus 100 bytes per
 * angle) return NCS_ERR_INVALID_ARG.  Asynchronous on `stream`.  Calls that
 * overlap on one GPU share that array and race: serialise them (one stream,
 * or an event between them). */
ncs_status ncs_forward_noalloc(const ncs_geometry* geom, const float* x_dev, float* y_dev, void* stream);

/* Filtered backprojection with the method's own circulant inverse:
 * x = alpha M^+ E^T y (N*N values from N_theta*N_s).  Since E^T E is close to
 * the circulant of eq. (circ_R), this approximates the least-squares image
 * (E^T E)^-1 E^T y with the regularisation that M adds; it is also (1 + alpha)
 * times the second CT iterate of NCS started from zero.  It is the input of
 * the learned warm start (ncs_cnn.h). */
ncs_status ncs_prefilter(ncs_handle* h, const void* y_dev, void* x_dev);

/* Filtered backprojection x = (pi / N_theta) E^T (h * y): each projection is
 * convolved over the detector with the Shepp-Logan filter for unit bin
 * spacing, h(n) = -2 / (pi^2 (4 n^2 - 1)) (zero outside the detector), then
 * backprojected.  It approximates the image whose line integrals are y, and
 * is the input of the learned warm start (ncs_cnn.h).  At most 4096 bins. */
ncs_status ncs_fbp(ncs_handle* h, const void* y_dev, void* x_dev);

/* Facts about a handle, computed in double on the host at setup. */
typedef struct {
    int64_t nnz;       /* nonzero entries of E (Joseph taps with weight != 0 inside the image) */
    double c_r;        /* C_R in use */
    double mu_dc;      /* DC eigenvalue of M in use */
    double norm_e1_sq; /* |E 1|^2 */
    int32_t projector;     /* forward-projector kernel in use (1, 2 or 3) */
    int32_t backprojector; /* backprojector kernel in use (1, 2 or 3) */
    double projector_ms[3];     /* setup timing of the three variants (0 when not timed) */
    double backprojector_ms[3]; /* setup timing of the three variants (0 when not timed) */
} ncs_info;

ncs_status ncs_get_info(ncs_handle* h, ncs_info* info);

/* Per-kernel timing: one iteration, then each phase launched `iters` >= 1
 * times back to back between two HIP events on the handle's stream; returns in
 * ms_host[0..NCS_N_PHASES-1] the mean duration of one launch of each phase, in
 * the order backprojection (with D^T v), row DFT, column DFT + multiplier,
 * inverse row DFT + x-update, projection + data prox + TV update, objective
 * reduction.  The launches change the state (x, duals, iteration count): time
 * on a handle whose iterate is not needed afterwards, or call ncs_set_init.
 * Synchronises. */
#define NCS_N_PHASES 6
ncs_status ncs_time_phases(ncs_handle* h, int32_t iters, double* ms_host);

/* The eigenvalues mu of M actually used (N*N doubles, numpy FFT order,
 * host memory), after the C_R and mu_dc defaults are resolved. */
ncs_status ncs_get_eigenvalues(ncs_handle* h, double* mu_host);

void ncs_destroy(ncs_handle* h);

/* ---- Batches: many independent slices of uneven size in shared launches ----
 *
 * Every phase of an iteration is one launch over the workgroups of all active
 * slices (a workgroup -> slice map; slices are pinned to XCDs so that a
 * slice's workgroups share one L2).  Each slice keeps its own geometry,
 * parameters, data, state, objective history and device stop flag (the
 * workgroups of a stopped slice exit at once).  The iterations between two
 * host checks (params[0].check_every) are one replayed HIP graph, captured on
 * a private stream at first use; params[0].graph_chunk < 0 gives direct
 * launches instead.  At a check the maps are rebuilt without the stopped
 * slices (and the graph re-captured) once a quarter of the projection
 * workgroups in them belong to stopped slices. */
typedef struct ncs_batch ncs_batch;

/* geoms, params, b_dev: arrays of n_slices (b_dev entries non-NULL); bg_dev:
 * NULL or an array of n_slices (entries may be NULL).  The slices are all
 * parallel-beam or all fan-beam (each fan slice estimates its own multiplier
 * from probes); methods NCS or PDHG.  For parallel beams the projector is
 * params[0].projector, or (0) the faster variant on the largest slice; fan
 * beams have one projector pair. */
ncs_status ncs_batch_setup(int32_t n_slices, const ncs_geometry* geoms, const ncs_params* params,
                           int32_t dtype, const void* const* b_dev, const void* const* bg_dev,
                           void* stream, ncs_batch** out);

/* ncs_set_init for every slice (x0_dev NULL or an array of n_slices
 * pointers, entries may be NULL). */
ncs_status ncs_batch_set_init(ncs_batch* b, const void* const* x0_dev, int32_t dual_from_x0);

/* Iterate every slice until its objective reaches f_target[i] (NULL or NaN:
 * none), at most max_iters iterations.  f_target[i] = -infinity makes slice i
 * sit out this call (no iterations, its state untouched), so a long solve can
 * be split into calls that leave finished slices alone.  iters_done and
 * f_final (NULL or arrays of n_slices) receive per-slice results.  Returns
 * NCS_OK when every slice taking part reached its target, NCS_NOT_CONVERGED
 * otherwise, NCS_ERR_NONFINITE if a slice produced a NaN objective. */
ncs_status ncs_batch_solve(ncs_batch* b, int32_t max_iters, const double* f_target,
                           int32_t* iters_done, double* f_final);

/* Borrow the handle of slice i (owned by the batch; valid until
 * ncs_batch_destroy) for ncs_get_x, ncs_get_objectives, ncs_forward, ... */
ncs_status ncs_batch_slice(ncs_batch* b, int32_t i, ncs_handle** slice);

void ncs_batch_destroy(ncs_batch* b);

/* Message of the last failure on the calling thread ("" if none). */
const char* ncs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NCS_H */
