// Internal declarations shared by the host API (ncs_api.cpp) and the kernels
// (ncs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ncs {

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
    T pad;
};

// Device control block of one solver.
struct Control {
    int32_t stop;        // 1: iteration kernels return immediately
    int32_t status;      // 0 running, 1 target reached, -4 NaN objective
    int32_t iter;        // iterations completed since the last init
    int32_t pad0;
    double f_target;     // NaN: none
    double f_last;       // objective after the last iteration
    double data_const;   // constant added to the data term (PET: sum log Gamma(b+1))
    double eval_out;     // result slot of a one-off objective evaluation
};

constexpr int kHistCap = 65536;   // objective history ring (doubles)

enum { DATA_QUAD = 0, DATA_POISSON = 1 };
enum { TV_ANISO = 0, TV_ISO = 1 };

// Raw device pointers and scalars handed to every kernel by value.
template <class T>
struct DevCtx {
    int N, log2N, NA, NS, PU;        // PU: padded sinogram pitch = NS + 3 (entry d at a*PU + 1 + d)
    int P;                           // padded image pitch = N + 4 (pixel c of a row at offset c + 2)
    int projector;                   // 1: LDS-staged tiles, 2: direct coalesced loads
    const AngleT<T>* ang;
    const int32_t* axis;
    T* x;        // N*N current image
    T* xbar;     // N*P padded extrapolated image 2x+ - x (two zero columns each side)
    T* xbarT;    // N*P padded transpose of xbar (row c holds column c)
    T* xsc;      // N*P padded scratch image (plain projections)
    T* xscT;     // N*P padded scratch transpose
    T* u;        // NA*PU padded data dual
    T* p;        // NA*PU padded projection E x (kept by recurrence)
    T* v;        // 2*N*N TV dual (horizontal plane, vertical plane)
    T* w;        // N*N backprojection + divergence
    T* spec;     // (N/2+1)*N complex, transposed half spectrum: spec[2*(k*N + j) + {0,1}]
    const T* hh; // (N/2+1)*N real multiplier h/(alpha N^2), transposed like spec
    const T* tw; // N/2 complex twiddles exp(-2 pi i k / N)
    const T* b;  // NA*NS data (caller-owned)
    const T* bg; // NA*NS PET background or nullptr
    T* ysc;      // NA*PU padded scratch sinogram
    double* part_data;
    double* part_tv;
    Control* ctl;
    double* hist;
    T alpha, beta, s_tv, inv1pa;
    double lambda;
    int data_term, tv_term;
};

// Launch helpers (ncs_kernels.hip).  All enqueue on `st` and return the
// launch status.
template <class T> hipError_t launch_backproject_iter(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_backproject_plain(const DevCtx<T>& c, const T* y_padded, T* out, hipStream_t st);
template <class T> hipError_t launch_fft_rows_fwd(const DevCtx<T>& c, const T* src, bool iter, hipStream_t st);
template <class T> hipError_t launch_fft_cols(const DevCtx<T>& c, T scale, bool iter, hipStream_t st);
template <class T> hipError_t launch_fft_rows_inv_update(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_fft_rows_inv_plain(const DevCtx<T>& c, T* out, hipStream_t st);
template <class T> hipError_t launch_tv_update(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_project_iter(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_pad_image(const DevCtx<T>& c, const T* img, hipStream_t st);
// Plain projections read the padded scratch pair (xsc, xscT): call
// launch_pad_image first.
template <class T> hipError_t launch_project_plain(const DevCtx<T>& c, T* out, hipStream_t st);
template <class T> hipError_t launch_project_setp(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_finalize_iter(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_eval_objective(const DevCtx<T>& c, const T* img, hipStream_t st);   // pads img itself
template <class T> hipError_t launch_pad_sinogram(const DevCtx<T>& c, const T* y, T* y_padded, hipStream_t st);
template <class T> hipError_t launch_unpad_sinogram(const DevCtx<T>& c, const T* y_padded, T* y, hipStream_t st);
template <class T> hipError_t launch_data_const(const DevCtx<T>& c, hipStream_t st);
template <class T> hipError_t launch_dual_init(const DevCtx<T>& c, hipStream_t st);

// Control block updates queued on the stream (no memset nodes, capturable):
//   op 0: reset  (iter = 0, stop = 0, status = 0, f_target)
//   op 1: arm    (stop = 0, status = 0, f_target), iteration count kept
//   op 2: set    (iter = iter_value, stop = 0, status = 0, f_target)
hipError_t launch_control(Control* ctl, int op, int iter_value, double f_target, hipStream_t st);

int project_blocks(int NA, int NS);
int tv_blocks(int N);

}  // namespace ncs
