// Internal declarations shared by the host API (ncs_api.cpp) and the kernels
// (ncs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

// Pointers inside descriptors that kernels read from device memory are marked
// global in the device pass of the kernel source, so that loads through them
// are global (uniform ones scalar) rather than flat; everywhere else they are
// plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__) && defined(NCS_KERNEL_SOURCE)
#define NCS_G __attribute__((address_space(1)))
#else
#define NCS_G
#endif

namespace ncs {

// Zero columns on each side of a row of the padded image copies (x bar, its
// transpose and the scratch pair).  A 64-ray projector block spans at most
// 63 sqrt(2) < 90 columns, and every step of its range has some ray within
// [-2, N + 1] (two steps of margin included), so each tap of every ray of the
// block lies in [-96, N + 95]: the direct projector reads them without a clamp.
constexpr int kPadL = 96;

// Per-angle geometry, precomputed in double on the host and stored in T.
//   forward (ray-driven):  sampled coordinate of ray d at step s
//                          xi(d, s) = fma(s, k2, fma(d, k1, k0))
//                          (s = row r and xi = column when axis == 0,
//                           s = column c and xi = row when axis == 1)
//   backward (pixel-driven): detector coordinate of pixel (r, c)
//                          t(r, c) = fma(c, q1, fma(r, q2, q0))
//   weight of ray d on pixel (r, c): kappa * max(0, 1 - kappa |d - t(r, c)|),
//   kappa = 1/|cos theta| (axis 0) or 1/|sin theta| (axis 1).
template <class T>
struct AngleT {
    T k1, k2, k0;
    T q1, q2, q0;
    T kappa, kappa2, kd;   // kd = kappa - kappa2
    T omk;                 // 1 - kappa
};

// Fan beam: one ray of the equi-angular fan.  Along its stepping axis
// (axis 0: image rows, axis 1: columns) the ray crosses step s at the
// coordinate k0 + k2 s of the other axis; kappa is its length per step.
template <class T>
struct RayT {
    T k0, k2, kappa;
    int32_t axis;
};

// Fan beam: one source position (its coordinates and the direction of its
// central ray), used by the backprojector to find the rays near a pixel.
template <class T>
struct ViewT {
    T sx, sy, theta_c, pad;
};

// Device control block of one slice.
struct Control {
    int32_t stop;        // 1: iteration kernels of this slice return immediately
    int32_t status;      // 0 running, 1 target reached, -4 NaN objective
    int32_t iter;        // iterations completed since the last init
    int32_t pad0;
    double f_target;     // NaN: none
    double f_last;       // objective after the last iteration
    double data_const;   // constant added to the data term (PET: sum log Gamma(b+1))
    double eval_out;     // result slot of a one-off objective evaluation
    double step_sq;      // |x^k - x^{k-1}|^2 at the last residual evaluation
    double x_sq;         // |x^k|^2 at the same evaluation
};

constexpr int kHistCap = 65536;   // objective history ring (doubles)

enum { DATA_QUAD = 0, DATA_POISSON = 1 };
enum { TV_ANISO = 0, TV_ISO = 1 };

// Device pointers and scalars of one slice.  Kernels read it from a device
// array indexed by slice, so one launch can serve many slices.
template <class T>
struct DevCtx {
    int N, log2N, NA, NS, PU;        // PU: padded sinogram pitch = NS + 3 (entry d at a*PU + 1 + d)
    int P;                           // padded image pitch = N + 2 kPadL (pixel c of a row at offset c + kPadL)
    int nb_proj, nb_tv;              // (angle, 64-ray block) pairs and TV tiles of this slice
    int nwg_proj;                    // projection workgroups of a launch (>= nb_proj with aorder)
    // single parallel-beam slices: the angles ordered by stepping axis (row-
    // stepping ones first, nar of them); a projection launch then sends
    // row-stepping blocks to XCDs 0-3 and column-stepping ones to XCDs 4-7
    // (workgroup b runs on XCD b mod 8), so each XCD's L2 holds one image copy.
    // Null: workgroup b takes block b (batches, fan beams).
    const NCS_G int32_t* aorder;
    int nar;
    const NCS_G AngleT<T>* ang;
    const NCS_G double* ang64;       // per angle k1, k2, k0, q1, q2, q0 in double (both precisions)
    const NCS_G int32_t* axis;
    NCS_G T* x;        // N*N current image
    NCS_G T* xbar;     // N*P padded extrapolated image 2x+ - x (kPadL zero columns each side)
    NCS_G T* xbarT;    // N*P padded transpose of xbar (row c holds column c)
    NCS_G T* xsc;      // N*P padded scratch image (plain projections)
    NCS_G T* xscT;     // N*P padded scratch transpose
    NCS_G T* u;        // NA*PU padded data dual
    NCS_G T* p;        // NA*PU padded projection E x (kept by recurrence)
    NCS_G T* v;        // 2*N*N TV dual (horizontal plane, vertical plane)
    NCS_G T* w;        // N*N backprojection + divergence
    NCS_G T* spec;     // (N/2+1)*N complex, transposed half spectrum: spec[2*(k*N + j) + {0,1}]
    const NCS_G T* hh; // (N/2+1)*N real multiplier h/(alpha N^2), transposed like spec
    const NCS_G T* tw; // N/2 complex twiddles exp(-2 pi i k / N)
    const NCS_G T* b;  // NA*NS data (caller-owned)
    const NCS_G T* bg; // NA*NS PET background or nullptr
    NCS_G T* ysc;      // NA*PU padded scratch sinogram
    NCS_G double* part_data;   // nb_proj partial data terms (also reused by evaluations)
    NCS_G double* part_tv;     // nb_tv partial TV terms
    NCS_G Control* ctl;
    NCS_G double* hist;
    // ADMM with CG inner solves only (null otherwise): CG vectors (N*N), an
    // unpadded sinogram scratch, per-block dot-product partials and the CG
    // scalars [r.z, p.q, a, b]
    NCS_G T* cg_d;
    NCS_G T* cg_r;
    NCS_G T* cg_z;
    NCS_G T* cg_p;
    NCS_G T* cg_q;
    NCS_G T* cg_y;
    NCS_G double* cg_part;
    NCS_G double* cg_s;
    NCS_G T* tpos;     // N*N positivity dual t (nullptr without the constraint x >= 0)
    // fan beam only (beam == 1): ray and view tables, the first ray's fan angle,
    // the fan step, and the half-width in bins of the rays that can touch a pixel
    const NCS_G RayT<T>* rays;
    const NCS_G ViewT<T>* views;
    T gamma0, dgamma;
    int beam, fan_w;
    T alpha, beta, s_tv, inv1pa;
    T dual_ramp;                     // TV-dual ramp width of the warm start (<= 0: sign)
    double lambda;
    int data_term, tv_term;
};

// Workgroup -> (slice, workgroup within the slice) for batched launches; a
// null map means one slice and local workgroup = blockIdx.x.
struct Slot {
    int32_t slice, local;
};

// One phase of a batched iteration launch.
struct PhaseGrid {
    const Slot* map;   // device array or nullptr (single slice)
    int blocks;        // total workgroups
};

// Everything one (batched) NCS iteration needs.
template <class T>
struct IterLaunch {
    const DevCtx<T>* ctxs;   // device array of slice descriptors
    PhaseGrid bp, rows, cols, proj, fin;   // rows is shared by the forward and inverse row DFTs
    int max_N;               // largest image side (dynamic LDS of the DFT kernels)
    int projector;           // 1: LDS-staged row windows, 2: direct coalesced loads, 3: ray pairs
    int backprojector;       // 1: LDS-staged detector windows, 2 x 2 pixels per lane (16 x 16 tiles),
                             // 2: direct (8 x 8 tiles), 3: 2 x 2 pixels per lane with 16-byte loads
                             // (16 x 16 tiles)
};

constexpr int kNumBackprojectors = 3;
constexpr int kFanProbes = 16;   // default probes of eq. H-fan for fan beams

constexpr int kNumPhases = 6;   // backprojection, row DFT, column DFT, inverse row DFT + x-update,
                                // projection + data prox + TV update, objective

// The backprojection launch of an iteration (fin_prev: reduce the previous
// iteration's objective first).
template <class T> hipError_t launch_bp_iter(const IterLaunch<T>& L, int fin_prev, hipStream_t st);

// k iterations of ADMM with cg_iters conjugate-gradient steps per linear
// solve (precond: circulant alpha M^+ preconditioner); hc is the host copy
// of the single slice's descriptor.
template <class T> hipError_t launch_admm_iterations(const IterLaunch<T>& L, const DevCtx<T>& hc, int k, int cg_iters,
                                                     int precond, hipStream_t st);
int cg_blocks(int N);

// k iterations (five launches each plus one finalize at the end).
template <class T> hipError_t launch_iterations(const IterLaunch<T>& L, int k, hipStream_t st);
// One phase of an iteration, unfused (phase 0 does not reduce the previous
// objective; phase 5 is the finalize launch): used for per-kernel timing.
template <class T> hipError_t launch_iteration_phase(const IterLaunch<T>& L, int phase, hipStream_t st);

// Single-slice operators.  `hc` is the host copy of the descriptor (launch
// sizes), `dc` its device copy.
template <class T> hipError_t launch_backproject_plain(const DevCtx<T>& hc, const DevCtx<T>* dc, int variant, const T* y_padded, T* out, hipStream_t st);
// Filtered backprojection: Shepp-Logan filter per projection (into the padded
// scratch sinogram), then the backprojection; out = N*N image.
template <class T> hipError_t launch_fbp(const DevCtx<T>& hc, const DevCtx<T>* dc, int backprojector, const T* y, T* out, hipStream_t st);
template <class T> hipError_t launch_apply_minv(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* w, T* out, T scale, hipStream_t st);
template <class T> hipError_t launch_pad_image(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* img, hipStream_t st);
// a parallel beam's descriptor (by value) and tables written on the device
hipError_t launch_parallel_tables(const DevCtx<float>& hc, DevCtx<float>* dst, AngleT<float>* ang, double* ang64,
                                  int32_t* axis, hipStream_t st);
// the padded scratch pair including its zero margins
template <class T> hipError_t launch_pad_image_full(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* img, hipStream_t st);
// Plain projections read the padded scratch pair (xsc, xscT): pad first.
template <class T> hipError_t launch_project_plain(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, T* out, hipStream_t st);
template <class T> hipError_t launch_project_setp(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, hipStream_t st);
template <class T> hipError_t launch_eval_objective(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, const T* img, hipStream_t st);
template <class T> hipError_t launch_pad_sinogram(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* y, T* y_padded, hipStream_t st);
template <class T> hipError_t launch_unpad_sinogram(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* y_padded, T* y, hipStream_t st);
template <class T> hipError_t launch_data_const(const DevCtx<T>& hc, const DevCtx<T>* dc, hipStream_t st);
template <class T> hipError_t launch_dual_init(const DevCtx<T>& hc, const DevCtx<T>* dc, hipStream_t st);
// |E 1|^2 into ctl->eval_out (projection of the ones image, double sum)
template <class T> hipError_t launch_e1_norm(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, hipStream_t st);
// |x^k - x^{k-1}|^2 and |x^k|^2 of one slice into its control block
template <class T> hipError_t launch_step_residual(const DevCtx<T>* dc, hipStream_t st);

// Control block updates queued on the stream (no memset nodes, capturable):
//   op 0: reset  (iter = 0, stop = 0, status = 0, f_target)
//   op 1: arm    (stop = 0, status = 0, f_target), iteration count kept
//   op 2: set    (iter = iter_value, stop = 0, status = 0, f_target)
hipError_t launch_control(Control* ctl, int op, int iter_value, double f_target, hipStream_t st);

// Sets the message returned by ncs_last_error() on this thread.
void set_error_message(const char* msg);

int project_blocks(int NA, int NS);
// projection workgroups when the blocks are split by stepping axis over the XCDs
int project_wgs_split(int NA, int NS, int nar);
int tv_blocks(int N);
int bp_blocks(int N, int variant);

}  // namespace ncs
