/*
 * ncs_cone.h -- C ABI of the NCS solver for cone-beam CT on volumes (gfx950).
 *
 * Section 4.1.1 (fan beam and cone beam geometry): the CT problem of
 * Section 4.1, minimize 1/2 |E x - b|^2 + lambda |D x|_1, on a volume, with E a
 * discretisation of the cone-beam transform, D the forward differences of
 * Section 2 along x, y and z, and the circulant M = F^-1 diag(mu) F (F the 3D
 * DFT) with E^T E's multiplier estimated from probes as in eq. (H-fan):
 *
 *     mu = gamma + alpha h_E + (beta^2/alpha) 4 (sin^2(pi j/N) + sin^2(pi k/N)
 *          + sin^2(pi l/N_z)),     h_E = Re sum_v conj(F v) F(E^T E v) / sum_v |F v|^2,
 *
 * the DC entry gamma + alpha |E 1|^2 / n (or params.mu_dc), and the iteration
 * of eq. (NCS) in the CT form of Section 4.1:
 *
 *     x+ = x - (1/alpha) F^-1 diag(1/mu) F (alpha E^T u + beta D^T v)
 *     u+ = (u + alpha (E(2x+ - x) - b)) / (1 + alpha)
 *     v+ = clamp(v + beta D(2x+ - x), -s, s),   s = lambda alpha / beta.
 *
 * METHOD_PDHG replaces M by gamma I (eq. PDHG).
 *
 * Geometry (the paper fixes none; the reading shared with the test oracle):
 *
 *  - Volume: N x N x N_z unit voxels, centres (c - (N-1)/2, r - (N-1)/2,
 *    z - (N_z-1)/2), stored (z N + r) N + c.  N a power of two in [16, 512],
 *    N_z a power of two in [4, 256].
 *  - Orbit: the source circles in the plane z = 0 at radius R_s; view a of N_v
 *    sits at R_s (cos b_a, sin b_a, 0), b_a = 2 pi a / N_v.
 *  - Detector: cylindrical, centred on the source.  Columns d of N_s are the
 *    equi-angular fan bins of ncs.h's fan beam (fan step
 *    2 asin(N / (sqrt 2 R_s)) / (N_s - 1), central ray towards the axis);
 *    rows rho of N_r have slopes z_rho = (rho - (N_r-1)/2) dz,
 *    dz = 2 z_max / (N_r - 1), z_max = (N_z/2) / (R_s - N/sqrt 2).  Ray
 *    (a, rho, d) is the half line S_a + s (cos th, sin th, z_rho), s >= 0;
 *    sinograms are stored (a N_r + rho) N_s + d.
 *  - Joseph's method: the ray steps through the rows (|u_y| >= |u_x| - 1e-12)
 *    or columns of every slice; at each plane it takes the bilinear weights
 *    of the four voxels around its (column or row, slice) coordinates, times
 *    sqrt(1 + z_rho^2) / |u_y| (or / |u_x|).  E^T is the adjoint of that
 *    matrix, evaluated voxel by voxel: the same taps and weights, up to the
 *    rounding of each tap's slice coordinate.
 *  - 1 <= N_v <= 65535, N_s >= 2, 2 <= N_r <= 65535, N_r N_s <= 2^24,
 *    R_s >= N/sqrt 2 + 4.
 *
 * Conventions (as in ncs.h): a handle is NCS_F32 or NCS_F64 and every device
 * buffer holds that type; *_dev pointers are device pointers owned by the
 * caller (b_dev must stay alive for the handle's life); the library owns its
 * workspace from ncs_cone_setup to ncs_cone_destroy; work is queued on the
 * stream given to ncs_cone_setup; calls returning host values synchronise it;
 * a failing call returns a negative ncs_status and leaves a message for
 * ncs_last_error(); no C++ exception crosses the interface; one host thread
 * at a time per handle.
 */
#ifndef NCS_CONE_H
#define NCS_CONE_H

#include <stddef.h>
#include <stdint.h>

#include "ncs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t n_side;        /* N */
    int32_t n_slices;      /* N_z */
    int32_t n_views;       /* N_v source positions over a full turn */
    int32_t n_bins;        /* N_s detector columns */
    int32_t n_rows;        /* N_r detector rows */
    int32_t reserved;      /* must be 0 */
    double source_radius;  /* R_s, in voxels */
} ncs_cone_geometry;

typedef struct {
    double alpha, beta, gamma, lambda;
    double mu_dc;          /* <= 0: gamma + alpha |E 1|^2 / n */
    int32_t method;        /* NCS_METHOD_NCS or NCS_METHOD_PDHG */
    int32_t probes;        /* probes of eq. (H-fan), 0: 16; Rademacher images from SplitMix64
                              seeded by the probe index, bit j of output k giving voxel 64 k + j */
    int32_t positivity;    /* 1: constrain x >= 0 (the remark in Section 4.2): A gains the rows I
                              with the indicator of x >= 0, a dual t with t+ = min(t + alpha xbar, 0),
                              alpha t in the backprojection and every eigenvalue of M raised by alpha
                              (NCS; PDHG keeps M = gamma I) */
    int32_t reserved;      /* must be 0 */
} ncs_cone_params;

typedef struct ncs_cone ncs_cone;

/* Create a solver.  b_dev (N_v N_r N_s values) may be NULL for a handle used
 * only for the operators.  Builds the ray tables in double precision on the
 * host, estimates h_E on the device (params.probes products E^T E v and their
 * 3D DFTs, accumulated in double, always with the double-precision kernels: a
 * single-precision handle builds a temporary double-precision twin for it, so
 * both precisions run the same M), and sets x = u = v = 0. */
ncs_status ncs_cone_setup(const ncs_cone_geometry* geom, const ncs_cone_params* params, int32_t dtype,
                          const void* b_dev, void* stream, ncs_cone** out);

/* x = x0_dev (NULL: zeros), u = v = 0 (and t = 0), iteration counter 0. */
ncs_status ncs_cone_set_init(ncs_cone* h, const void* x0_dev);

/* Run k >= 0 iterations; obj_host (length k, may be NULL) receives f(x^{k+1})
 * after each one (double accumulation); non-NULL synchronises.  Needs b. */
ncs_status ncs_cone_iterate(ncs_cone* h, int32_t k, double* obj_host);

/* Copies of the state: x (N_z N^2), u (N_v N_r N_s), v (3 N_z N^2: the x-,
 * y- and z-difference volumes, each (z N + r) N + c), t (N_z N^2, the
 * positivity dual; NCS_ERR_INVALID_ARG without params.positivity). */
ncs_status ncs_cone_get_x(ncs_cone* h, void* x_out_dev);
ncs_status ncs_cone_get_u(ncs_cone* h, void* u_out_dev);
ncs_status ncs_cone_get_v(ncs_cone* h, void* v_out_dev);
ncs_status ncs_cone_get_t(ncs_cone* h, void* t_out_dev);

/* Checkpoint: the full state (x, u, v, E x, t, iteration count) as an opaque
 * host blob; with host_buf NULL, *bytes receives the size needed.  A handle
 * with the same geometry, parameters and precision resumes from it bit for
 * bit. */
ncs_status ncs_cone_get_state(ncs_cone* h, void* host_buf, size_t* bytes);
ncs_status ncs_cone_set_state(ncs_cone* h, const void* host_buf, size_t bytes);

/* Operators: y = E x, x = E^T y, out = F^-1 diag(1/mu) F w (real volume). */
ncs_status ncs_cone_forward(ncs_cone* h, const void* x_dev, void* y_dev);
ncs_status ncs_cone_adjoint(ncs_cone* h, const void* y_dev, void* x_dev);
ncs_status ncs_cone_apply_minv(ncs_cone* h, const void* w_dev, void* out_dev);

/* The eigenvalues mu of M (N_z N^2 doubles, numpy fftn order [l, j, k]). */
ncs_status ncs_cone_get_eigenvalues(ncs_cone* h, double* mu_host);

typedef struct {
    int64_t nnz;           /* nonzeros of E (taps of nonzero weight inside the volume) */
    double norm_e1_sq;     /* |E 1|^2 */
    double mu_dc;          /* the DC eigenvalue used */
    int32_t bin_window;    /* W: fan bins tested per voxel and view on each side */
} ncs_cone_info;

/* Sizes and setup values of the handle.  nnz is counted on the host in double
 * precision the first time it is asked for (a pass over every ray and step). */
ncs_status ncs_cone_get_info(ncs_cone* h, ncs_cone_info* info);

/* Milliseconds per launch of each phase of the iteration, from HIP events
 * around iters back-to-back launches of that phase on the handle's stream:
 * ms_host[0] backprojection (w), [1] the five DFT passes with the update,
 * [2] projection with the data dual, [3] TV dual, [4] objective.  The state
 * is left changed: call ncs_cone_set_init before iterating again.  Needs b. */
ncs_status ncs_cone_time_phases(ncs_cone* h, int32_t iters, double* ms_host);

void ncs_cone_destroy(ncs_cone* h);

#ifdef __cplusplus
}
#endif

#endif /* NCS_CONE_H */
