// Cone-beam NCS on volumes for gfx950 (Section 4.1.1, eq. H-fan, eq. NCS in
// the CT form of Section 4.1): kernels and the host side of the C ABI in
// ncs_cone.h.
//
// One iteration is eight launches on the handle's stream:
//   1. k_cone_backproject<ITER>: w = alpha E^T u + beta D^T v, voxel-driven
//      (each run of voxels along z gathers the rays whose Joseph taps
//      include them);
//   2-6. the 3D DFT of w as five line passes over an interleaved complex
//      volume (x forward from the real w, y forward, z forward x (1/mu) z
//      inverse, y inverse, x inverse with the update x+ = x - Re(.)/(n alpha),
//      xbar = 2 x+ - x written into zero-padded copies for the projector);
//      PDHG replaces them by one elementwise update (M = gamma I);
//   7. k_cone_project<ITER>: E xbar ray by ray (one lane per ray), the data
//      dual u+, E x+ = (E xbar + E x)/2 and the data term of f(x+);
//   8. k_cone_tv: the TV dual v+ and the TV term of f(x+); then one
//      workgroup adds the partial sums in a fixed order (k_cone_objective).
// Reductions are in double; every sum has a fixed order, so runs repeat bit
// for bit.
#include "ncs_cone.h"
#include "ncs_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

namespace {

constexpr int kWaves = 4;          // projector: waves per workgroup (split the steps)
constexpr int kBpWaves = 8;        // backprojector: waves per 8 x 8 voxel tile (split the views)
constexpr int kHits = 2;           // backprojector: rays collected per lane before their rows are summed
constexpr int kBpRunMax = 16;      // backprojector: longest run of voxels along z per lane
constexpr int kFftLds = 32768;     // bytes of LDS per DFT workgroup
constexpr int kHist = 65536;       // objective ring (doubles)
constexpr double kPi = 3.14159265358979323846;

template <class T>
struct ConeRay {   // in-plane part of the rays (a, ., d): coordinates as linear functions of the step
    T k0, k2;      // interpolated in-plane coordinate xi = k0 + step k2
    T s0, s2;      // in-plane distance from the source s = s0 + step s2
    T kxy;         // in-plane length per plane, 1/|u_y| or 1/|u_x|
    int axis;      // 0: steps through rows, 1: through columns
};

// What the adjoint needs of a ray to find the voxels it reaches: the
// in-plane coordinate k0 + step k2, the length per plane kxy and the axis.
// At a voxel's plane the in-plane distance from the source is the offset
// from the source along the stepping axis times kxy.
template <class T>
struct alignas(4 * sizeof(T)) ConeRayHead {
    T k0, k2, kxy;
    int axis;
};

template <class T>
struct ConeView {
    T sx, sy, thc, pad;
};

template <class T>
struct ConeCtx {
    int N, NZ, NV, NS, NR, P;   // P = N + 4: padded row
    int W;                      // half-window of fan bins in the gather
    int n_part_data, n_part_tv;
    T half, half_z, gamma0, inv_dgamma, inv_dzeta, cr;
    T alpha, beta, s_tv, inv_na;   // inv_na = 1 / (n alpha)
    double lambda;
    const ConeRay<T>* rays;
    const ConeRayHead<T>* heads;
    const ConeView<T>* views;
    const T* zeta;   // row slopes
    const T* kz;     // sqrt(1 + zeta^2)
    const T* b;
    const T* h;      // 1 / mu
    const T* hh;     // 1 / mu on the half spectrum (k <= N/2 along x)
    const T* tw_n;   // cos, -sin of 2 pi k / N
    const T* tw_z;   // cos, -sin of 2 pi k / N_z
    T *x, *xbar, *xbarT, *u, *p, *v, *w, *spec;
    T* tpos;         // positivity dual t (NULL without the constraint)
    double *part_data, *part_tv, *obj;
};

template <class T>
__device__ inline T clampT(T v, T lo, T hi) { return fmin(fmax(v, lo), hi); }
template <>
__device__ inline float clampT<float>(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Two consecutive elements read with one load (element alignment only).
template <class T>
struct alignas(sizeof(T)) Pair2 {
    T a, b;
};

// Padded layout of the projector's input: (N_z + 4) slices of N rows of P
// elements; voxel (z, r, c) at ((z + 2) N + r) P + c + 2; the pads stay zero.
__device__ inline size_t pad_index(int z, int r, int c, int N, int P) {
    return ((size_t)(z + 2) * N + r) * P + (c + 2);
}

// ---------------------------------------------------------------------------
// Projector: lane = detector column d of one (view a, row rho); the 4 waves of
// a workgroup split the N steps.  Two zero columns and two zero slices on
// every side absorb taps off the volume, so no step needs a bounds test.
// ---------------------------------------------------------------------------
template <class T, bool ITER>
__global__ __launch_bounds__(256) void k_cone_project(ConeCtx<T> c, const T* __restrict__ img,
                                                      const T* __restrict__ imgT, T* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int d = blockIdx.x * 64 + lane;
    const int rho = blockIdx.y, a = blockIdx.z;
    const bool valid = d < c.NS;
    const ConeRay<T> R = c.rays[(size_t)a * c.NS + (valid ? d : c.NS - 1)];
    const T zr = c.zeta[rho];
    const T* src = R.axis == 0 ? img : imgT;
    const int N = c.N, P = c.P;
    const size_t slice = (size_t)N * P;
    const int SW = N / kWaves;
    int s_begin = wave * SW, s_end = s_begin + SW;
    // steps whose in-plane coordinate lies in [-2, N+1]; the others read pads only
    const T lo_x = T(-2), hi_x = T(N + 1);
    if (!valid) {
        s_end = s_begin;
    } else if (R.k2 > T(0)) {
        s_begin = max(s_begin, (int)fmax(floor((lo_x - R.k0) / R.k2), T(-1e9)) - 1);
        s_end = min(s_end, (int)fmin(ceil((hi_x - R.k0) / R.k2), T(1e9)) + 2);
    } else if (R.k2 < T(0)) {
        s_begin = max(s_begin, (int)fmax(floor((hi_x - R.k0) / R.k2), T(-1e9)) - 1);
        s_end = min(s_end, (int)fmin(ceil((lo_x - R.k0) / R.k2), T(1e9)) + 2);
    } else if (R.k0 < lo_x || R.k0 > hi_x) {
        s_end = s_begin;
    }
    const T cmax = (T)N, zmax = (T)c.NZ;
    T acc = T(0);
#pragma unroll 4
    for (int s = s_begin; s < s_end; ++s) {
        const T xi = fma((T)s, R.k2, R.k0);
        const T fl = clampT(floor(xi), T(-2), cmax);
        const T f = xi - fl;
        const T sd = fma((T)s, R.s2, R.s0);
        const T ze = fma(sd, zr, c.half_z);
        const T zl = clampT(floor(ze), T(-2), zmax);
        const T g = ze - zl;
        // a 32-bit byte offset from the volume's base (the padded volume is far below 4 GiB)
        const unsigned e0 = ((unsigned)((int)zl + 2) * (unsigned)N + (unsigned)s) * (unsigned)P + (unsigned)((int)fl + 2);
        const char* p0 = reinterpret_cast<const char*>(src) + e0 * (unsigned)sizeof(T);
        const Pair2<T> v0 = *reinterpret_cast<const Pair2<T>*>(p0);
        const Pair2<T> v1 = *reinterpret_cast<const Pair2<T>*>(p0 + slice * sizeof(T));
        const T lo = fma(f, v0.b - v0.a, v0.a);
        const T hi = fma(f, v1.b - v1.a, v1.a);
        acc += fma(g, hi - lo, lo);
    }
    __shared__ T red[kWaves * 64];
    red[threadIdx.x] = acc;
    __syncthreads();
    if (wave != 0) return;
    const T q = ((red[lane] + red[64 + lane]) + (red[128 + lane] + red[192 + lane])) * (R.kxy * c.kz[rho]);
    const size_t i = ((size_t)a * c.NR + rho) * c.NS + d;
    if (!ITER) {
        if (valid) out[i] = q;
        return;
    }
    double dterm = 0.0;
    if (valid) {
        const T bb = c.b[i];
        const T un = (c.u[i] + c.alpha * (q - bb)) / (T(1) + c.alpha);
        const T pn = T(0.5) * (q + c.p[i]);   // E x+ = (E xbar + E x) / 2
        c.u[i] = un;
        c.p[i] = pn;
        const double r = (double)pn - (double)bb;
        dterm = 0.5 * r * r;
    }
    dterm = wave_sum_d(dterm);
    if (lane == 0) c.part_data[((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = dterm;
}

// ---------------------------------------------------------------------------
// Backprojector: an 8 x 8 voxel tile per workgroup, each lane a run of ZR
// voxels along z of one (row, column) (ZR = min(N_z, 16), halved while the
// workgroup's LDS would exceed the device's limit); the 8 waves split the
// views.  For each view the lane finds the fan bins within W of its own fan
// angle and recomputes each ray's in-plane coordinate at its plane from the
// projector's k0 and k2 (once for the run); for a ray that reaches it, the
// detector rows whose slice coordinate falls within one slice of the run
// are summed into the run.  Joseph's weights are the tents max(0, 1 -
// |coordinate - voxel index|) in each interpolated axis, so E^T is the
// adjoint of the projector's matrix term by term, up to the rounding of the
// slice coordinate (the projector forms the in-plane distance from its step,
// the adjoint from the voxels' offset to the source).  Along z a row's slice
// coordinate ze lies between voxels floor(ze) and floor(ze) + 1 of the run,
// the only two with nonzero tents, (1 - f) and f for f = ze - floor(ze): the
// row adds those two terms to the lane's accumulators in LDS (slots padded by
// two voxels on each side, which take the terms of voxels outside the run).
// Each lane owns its slots, so a plain read-modify-write suffices (LDS float
// atomics measured several times slower) and every sum keeps the row order.
// ---------------------------------------------------------------------------
template <class T>
struct alignas(2 * sizeof(T)) ZetaKz {   // a detector row's slope and sqrt(1 + slope^2)
    T z, k;
};

// Rows up to this count keep their (slope, sqrt(1 + slope^2)) pairs in LDS.
constexpr int kBpTableRows = 2048;
constexpr int kRowBatch = 4;   // detector rows whose loads the adjoint issues together

// Reciprocal and reciprocal square root where only a conservative bound is
// needed (row ranges carry a guard row, bin windows 0.01 bin, far above the
// hardware approximations' error of about 1e-7 relative): the approximations
// in FP32, exact operations in FP64.
template <class T>
__device__ inline T rcp_bound(T v) { return T(1) / v; }
template <>
__device__ inline float rcp_bound<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <class T>
__device__ inline T rsqrt_bound(T v) { return T(1) / sqrt(v); }
template <>
__device__ inline float rsqrt_bound<float>(float v) { return __builtin_amdgcn_rsqf(v); }

template <class T, bool ITER, int ZR, bool TAB>
__global__ __launch_bounds__(kBpWaves * 64) void k_cone_backproject(ConeCtx<T> c, const T* __restrict__ ysrc,
                                                                     T* __restrict__ out) {
    // LDS: per wave and lane up to kHits rays that reach the lane's voxels
    // (bin, weight, in-plane distance) and the run's accumulators (slot j:
    // voxel j - 2); with TAB, the rows' (slope, sqrt(1 + slope^2)) after them.
    constexpr int kSlots = ZR + 4;
    constexpr int kHitBytes = kBpWaves * kHits * 64 * (4 + 2 * (int)sizeof(T));
    constexpr int kAccBytes = kBpWaves * kSlots * 64 * (int)sizeof(T);
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    T* hit_c = reinterpret_cast<T*>(smem) + (size_t)wave * kHits * 64;
    T* hit_s = reinterpret_cast<T*>(smem) + (size_t)(kBpWaves + wave) * kHits * 64;
    int* hit_d = reinterpret_cast<int*>(reinterpret_cast<T*>(smem) + (size_t)2 * kBpWaves * kHits * 64) +
                 wave * kHits * 64;
    T* const accs = reinterpret_cast<T*>(smem + kHitBytes);
    T* const acc_l = accs + (size_t)wave * kSlots * 64 + lane;   // slot j at acc_l[j * 64]
    ZetaKz<T>* const zk = reinterpret_cast<ZetaKz<T>*>(smem + kHitBytes + kAccBytes);
    const int N = c.N, NS = c.NS, NR = c.NR;
    const int tiles_x = N / 8;
    const int z0 = blockIdx.y * ZR;
    const int tx = (blockIdx.x % tiles_x) * 8, ty = (blockIdx.x / tiles_x) * 8;
    const int col = tx + (lane & 7), row = ty + (lane >> 3);
    const T px = (T)col - c.half, py = (T)row - c.half;
    const T fc = (T)col, fr = (T)row;
    const T zlo = T(z0 - 1) - c.half_z, zhi = T(z0 + ZR) - c.half_z;
    const T two_pi = T(6.283185307179586476925286766559);
#pragma unroll
    for (int j = 0; j < kSlots; ++j) acc_l[j * 64] = T(0);
    if (TAB) {
        for (int r = threadIdx.x; r < NR; r += kBpWaves * 64) zk[r] = ZetaKz<T>{c.zeta[r], c.kz[r]};
        __syncthreads();
    }
    for (int a = wave; a < c.NV; a += kBpWaves) {
        const ConeView<T> V = c.views[a];
        const T dx = px - V.sx, dy = py - V.sy;
        T gang = atan2(dy, dx) - V.thc;
        gang -= two_pi * rint(gang / two_pi);
        const int dc = (int)floor((gang - c.gamma0) * c.inv_dgamma + T(0.5));
        // A ray that reaches the voxels passes within one voxel of their centre
        // line, so its fan angle is within asin(1/dist) of theirs, dist >= 4:
        // asin(x) <= 1.02 x for x <= 1/4.  dc is the nearest bin to their fan
        // angle (half a bin), and 0.01 bin covers the rounding of both (about
        // 1e-4 bin in FP32).
        const int wv = min((int)ceil(T(1.02) * c.inv_dgamma * rsqrt_bound(fma(dx, dx, dy * dy)) + T(0.51)), c.W);
        int d = max(dc - wv, 0);
        const int d_hi = min(dc + wv, NS - 1);
        const ConeRayHead<T>* rr = c.heads + (size_t)a * NS;
        const T* ya = ysrc + (size_t)a * NR * NS;
        // Lanes reach different candidate bins, so each first collects the rays
        // that reach it (up to kHits at a time) and then all lanes sum their
        // j-th ray together: the row loop runs once per hit, not per candidate.
        while (__any(d <= d_hi)) {
            int nh = 0;
            for (; d <= d_hi && nh < kHits; ++d) {
                const ConeRayHead<T> R = rr[d];
                const T st = R.axis == 0 ? fr : fc;   // the ray's step at this column of voxels
                const T tp = R.axis == 0 ? fc : fr;   // the voxels' place along the interpolated axis
                const T xi = fma(st, R.k2, R.k0);
                const T wxy = fmax(T(0), T(1) - fabs(xi - tp));
                if (wxy > T(0)) {
                    hit_d[nh * 64 + lane] = d;
                    hit_c[nh * 64 + lane] = wxy * R.kxy;
                    hit_s[nh * 64 + lane] = fabs(R.axis == 0 ? dy : dx) * R.kxy;   // in-plane distance
                    ++nh;
                }
            }
            for (int j = 0; __any(j < nh); ++j) {
                if (j >= nh) continue;
                const int dj = hit_d[j * 64 + lane];
                const T coef = hit_c[j * 64 + lane];
                const T sd = hit_s[j * 64 + lane];
                // rows with slice coordinate hz + sd (rho - cr) dz in (z0 - 1, z0 + ZR): those
                // strictly between the two roots, and one row beyond each for rounding
                const T inv = c.inv_dzeta * rcp_bound(sd);
                const int r_lo = max((int)floor(fma(zlo, inv, c.cr)), 0);
                const int r_hi = min((int)ceil(fma(zhi, inv, c.cr)), NR - 1);
                const T* yr = ya + dj + (size_t)r_lo * NS;   // row rho of bin dj
                // rows in groups of kRowBatch: their loads are issued before
                // the group's LDS updates, so they are in flight together
                for (int rho = r_lo; rho <= r_hi; rho += kRowBatch, yr += (size_t)kRowBatch * NS) {
                    T yk[kRowBatch];
                    ZetaKz<T> tk[kRowBatch];
                    const unsigned left = (unsigned)(r_hi - rho);   // rows past rho still in range
#pragma unroll
                    for (int k = 0; k < kRowBatch; ++k) {
                        const unsigned dk = min((unsigned)k, left);  // the last row stands in for rows past r_hi
                        yk[k] = yr[__umul24(dk, (unsigned)NS)];     // N_s < 2^24
                        tk[k] = TAB ? zk[rho + dk] : ZetaKz<T>{c.zeta[rho + dk], c.kz[rho + dk]};
                    }
                    // an empty statement that takes each value keeps the compiler
                    // from moving the loads into the guarded steps below
#pragma unroll
                    for (int k = 0; k < kRowBatch; ++k) asm volatile("" : "+v"(yk[k]));
#pragma unroll
                    for (int k = 0; k < kRowBatch; ++k) {
                        if (rho + k > r_hi) break;
                        // the ray's slice coordinate at the voxels' plane, less z0
                        const T ze = fma(sd, tk[k].z, c.half_z) - T(z0);
                        const T yv = yk[k] * (coef * tk[k].k);
                        const T fl = clampT(floor(ze), T(-2), T(ZR));
                        const T f = ze - fl;
                        T* const ap = acc_l + ((int)fl + 2) * 64;
                        const T a0 = ap[0], a1 = ap[64];
                        ap[0] = a0 + yv * (T(1) - f);
                        ap[64] = a1 + yv * f;
                    }
                }
            }
        }
    }
    __syncthreads();   // every wave's accumulators are complete
    const size_t n2 = (size_t)N * N;
    const size_t n = n2 * c.NZ;
    for (int o = threadIdx.x; o < 64 * ZR; o += kBpWaves * 64) {
        const int l = o & 63, k = o >> 6;
        T bp = accs[(k + 2) * 64 + l];
#pragma unroll
        for (int w = 1; w < kBpWaves; ++w) bp += accs[(w * kSlots + k + 2) * 64 + l];
        const int cc = tx + (l & 7), rw = ty + (l >> 3), z = z0 + k;
        const size_t i = (size_t)z * n2 + (size_t)rw * N + cc;
        if (!ITER) {
            out[i] = bp;
            continue;
        }
        // D^T v with the differences of Section 2 (rows [1, -1], last row zero) on each axis
        const T* vx = c.v;
        const T* vy = c.v + n;
        const T* vz = c.v + 2 * n;
        T dtv = T(0);
        if (cc < N - 1) dtv += vx[i];
        if (cc > 0) dtv -= vx[i - 1];
        if (rw < N - 1) dtv += vy[i];
        if (rw > 0) dtv -= vy[i - N];
        if (z < c.NZ - 1) dtv += vz[i];
        if (z > 0) dtv -= vz[i - n2];
        T wv = fma(c.alpha, bp, c.beta * dtv);
        if (c.tpos) wv = fma(c.alpha, c.tpos[i], wv);   // the rows I of x >= 0 (remark in Section 4.2)
        c.w[i] = wv;
    }
}

// ---------------------------------------------------------------------------
// 3D DFT: line passes over an interleaved complex volume.  Line (A, B) of a
// pass has its L elements at (A L + l) B + b; a workgroup holds TB lines in
// LDS (element-major, l TB + j): adjacent b for strided passes (coalesced
// loads across lines), adjacent rows for the x pass (B = 1, contiguous).
// Radix-2: decimation in time from bit-reversed order for forward
// transforms, decimation in frequency to bit-reversed order for inverse ones,
// two stages per LDS round trip.  The circulant solve works on the half
// spectrum of its real volume (k = 0..N/2 along x, B = N/2 + 1 for the y
// lines); the setup's transforms of the probes use the full layout.
// ---------------------------------------------------------------------------
enum { FFT_FWD = 0, FFT_INV = 1, FFT_FWD_MUL_INV = 2 };
enum { OUT_REAL = 1, OUT_UPDATE = 2 };   // the solve's result: M+ w, or the NCS update

__device__ inline int bitrev_n(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

template <class T>
__device__ inline void bfly_dit(T& ar, T& ai, T& br, T& bi, T wr, T wi) {
    const T tr = br * wr - bi * wi, ti = br * wi + bi * wr;
    br = ar - tr;
    bi = ai - ti;
    ar = ar + tr;
    ai = ai + ti;
}

template <class T>
__device__ inline void bfly_dif(T& ar, T& ai, T& br, T& bi, T wr, T wi) {
    const T dr = ar - br, di = ai - bi;
    ar = ar + br;
    ai = ai + bi;
    br = dr * wr - di * wi;
    bi = dr * wi + di * wr;
}

// Stages ls and ls + 1 close over the quads (i0, i0 + h, i0 + 2h, i0 + 3h),
// h = 2^ls: each thread takes a quad of one line through both stages in
// registers (one LDS round trip and barrier per two stages); an odd last
// stage runs alone.
template <class T>
__device__ void lds_dit(T* re, T* im, const T* __restrict__ tw, int L, int logL, int TB, int logTB, T sign) {
    int ls = 0;
    for (; ls + 1 < logL; ls += 2) {
        const int h = 1 << ls;
        __syncthreads();
        for (int t = threadIdx.x; t < (TB * L) >> 2; t += blockDim.x) {
            const int j = t & (TB - 1), q = t >> logTB;
            const int pos = q & (h - 1);
            const int i0 = ((q >> ls) << (ls + 2)) + pos;
            const int t1 = pos * (L >> (ls + 1)), t2 = pos * (L >> (ls + 2)), t3 = (pos + h) * (L >> (ls + 2));
            const int p0 = i0 * TB + j, p1 = (i0 + h) * TB + j, p2 = (i0 + 2 * h) * TB + j, p3 = (i0 + 3 * h) * TB + j;
            T r0 = re[p0], m0 = im[p0], r1 = re[p1], m1 = im[p1], r2 = re[p2], m2 = im[p2], r3 = re[p3], m3 = im[p3];
            const T w1r = tw[2 * t1], w1i = sign * tw[2 * t1 + 1];
            bfly_dit(r0, m0, r1, m1, w1r, w1i);
            bfly_dit(r2, m2, r3, m3, w1r, w1i);
            bfly_dit(r0, m0, r2, m2, tw[2 * t2], sign * tw[2 * t2 + 1]);
            bfly_dit(r1, m1, r3, m3, tw[2 * t3], sign * tw[2 * t3 + 1]);
            re[p0] = r0; im[p0] = m0; re[p1] = r1; im[p1] = m1;
            re[p2] = r2; im[p2] = m2; re[p3] = r3; im[p3] = m3;
        }
    }
    if (ls < logL) {
        const int h = 1 << ls;
        __syncthreads();
        for (int t = threadIdx.x; t < (TB * L) >> 1; t += blockDim.x) {
            const int j = t & (TB - 1), bf = t >> logTB;
            const int k = bf & (h - 1);
            const int i0 = ((bf >> ls) << (ls + 1)) + k;
            const int ti = k * (L >> (ls + 1));
            const int p0 = i0 * TB + j, p1 = (i0 + h) * TB + j;
            T r0 = re[p0], m0 = im[p0], r1 = re[p1], m1 = im[p1];
            bfly_dit(r0, m0, r1, m1, tw[2 * ti], sign * tw[2 * ti + 1]);
            re[p0] = r0; im[p0] = m0; re[p1] = r1; im[p1] = m1;
        }
    }
    __syncthreads();
}

template <class T>
__device__ void lds_dif(T* re, T* im, const T* __restrict__ tw, int L, int logL, int TB, int logTB, T sign) {
    int ls = logL - 1;
    for (; ls >= 1; ls -= 2) {   // stages ls and ls - 1 on quads (i0, i0 + h, i0 + H, i0 + H + h)
        const int H = 1 << ls, h = H >> 1;
        __syncthreads();
        for (int t = threadIdx.x; t < (TB * L) >> 2; t += blockDim.x) {
            const int j = t & (TB - 1), q = t >> logTB;
            const int pos = q & (h - 1);
            const int i0 = ((q >> (ls - 1)) << (ls + 1)) + pos;
            const int t1 = pos * (L >> (ls + 1)), t2 = (pos + h) * (L >> (ls + 1)), t3 = pos * (L >> ls);
            const int p0 = i0 * TB + j, p1 = (i0 + h) * TB + j, p2 = (i0 + H) * TB + j, p3 = (i0 + H + h) * TB + j;
            T r0 = re[p0], m0 = im[p0], r1 = re[p1], m1 = im[p1], r2 = re[p2], m2 = im[p2], r3 = re[p3], m3 = im[p3];
            bfly_dif(r0, m0, r2, m2, tw[2 * t1], sign * tw[2 * t1 + 1]);
            bfly_dif(r1, m1, r3, m3, tw[2 * t2], sign * tw[2 * t2 + 1]);
            const T w3r = tw[2 * t3], w3i = sign * tw[2 * t3 + 1];
            bfly_dif(r0, m0, r1, m1, w3r, w3i);
            bfly_dif(r2, m2, r3, m3, w3r, w3i);
            re[p0] = r0; im[p0] = m0; re[p1] = r1; im[p1] = m1;
            re[p2] = r2; im[p2] = m2; re[p3] = r3; im[p3] = m3;
        }
    }
    if (ls == 0) {
        __syncthreads();
        for (int t = threadIdx.x; t < (TB * L) >> 1; t += blockDim.x) {
            const int j = t & (TB - 1), bf = t >> logTB;
            const int p0 = (2 * bf) * TB + j, p1 = (2 * bf + 1) * TB + j;
            T r0 = re[p0], m0 = im[p0], r1 = re[p1], m1 = im[p1];
            bfly_dif(r0, m0, r1, m1, tw[0], sign * tw[1]);
            re[p0] = r0; im[p0] = m0; re[p1] = r1; im[p1] = m1;
        }
    }
    __syncthreads();
}

template <class T>
__global__ __launch_bounds__(256) void k_cone_fft(ConeCtx<T> c, int mode, int L, int logL, int B, int TB, int logTB,
                                                  const T* __restrict__ tw, const T* __restrict__ real_in,
                                                  T* __restrict__ zc) {
    extern __shared__ unsigned char smem_raw[];
    T* re = reinterpret_cast<T*>(smem_raw);
    T* im = re + TB * L;
    const int tot = TB * L;
    const bool bitrev_in = mode != FFT_INV;
    // Element l of line j: contiguous lines (B = 1) at line L + l; in strided
    // passes a thread keeps one j (TB divides the block size), so the line's
    // base (line / B) L B + line % B is computed once.
    const unsigned jt = threadIdx.x & (TB - 1);
    size_t sbase = 0;
    if (B > 1) {
        const size_t line = (size_t)blockIdx.x * TB + jt;
        sbase = (line / (size_t)B) * (size_t)L * B + line % (size_t)B;
    }
    auto elem = [&](int t, int& j, int& l) -> size_t {
        if (B == 1) {
            l = t & (L - 1);
            j = t >> logL;
            return ((size_t)blockIdx.x * TB + j) * (size_t)L + l;
        }
        j = (int)jt;
        l = t >> logTB;
        return sbase + (size_t)l * B;
    };
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        int j, l;
        const size_t e = elem(t, j, l);
        const int pos = (bitrev_in ? bitrev_n(l, logL) : l) * TB + j;
        if (real_in) {
            re[pos] = real_in[e];
            im[pos] = T(0);
        } else {
            re[pos] = zc[2 * e];
            im[pos] = zc[2 * e + 1];
        }
    }
    if (mode == FFT_FWD || mode == FFT_FWD_MUL_INV) lds_dit(re, im, tw, L, logL, TB, logTB, T(1));
    if (mode == FFT_FWD_MUL_INV) {   // a strided pass (the z lines)
        for (int t = threadIdx.x; t < tot; t += blockDim.x) {
            int j, l;
            const size_t e = elem(t, j, l);
            const T hv = c.hh[e];   // the multiplied pass runs on the half spectrum
            re[l * TB + j] *= hv;
            im[l * TB + j] *= hv;
        }
    }
    if (mode == FFT_INV || mode == FFT_FWD_MUL_INV) lds_dif(re, im, tw, L, logL, TB, logTB, T(-1));
    const bool bitrev_out = mode != FFT_FWD;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
        int j, l;
        const size_t e = elem(t, j, l);
        const int pos = (bitrev_out ? bitrev_n(l, logL) : l) * TB + j;
        zc[2 * e] = re[pos];
        zc[2 * e + 1] = im[pos];
    }
}

// Result of the circulant solve for voxel (row, col), row = z N + r:
// OUT_REAL writes v / n (inv_na holds 1/n then); OUT_UPDATE does
// x+ = x - v / (n alpha), xbar = 2 x+ - x into both padded copies, and the
// positivity dual.
template <class T>
__device__ inline void x_result(const ConeCtx<T>& c, int out_mode, T* __restrict__ real_out, int row, int col, T v) {
    const int N = c.N, P = c.P;
    const size_t e = (size_t)row * N + col;
    if (out_mode == OUT_REAL) {
        real_out[e] = v * c.inv_na;
        return;
    }
    const int r = row & (N - 1), z = row >> (31 - __builtin_clz((unsigned)N));   // N a power of two
    const T xo = c.x[e];
    const T xn = xo - v * c.inv_na;
    const T xb = T(2) * xn - xo;
    c.x[e] = xn;
    if (c.tpos) c.tpos[e] = fmin(fma(c.alpha, xb, c.tpos[e]), T(0));   // t+ = min(t + alpha xbar, 0)
    c.xbar[pad_index(z, r, col, N, P)] = xb;
    c.xbarT[pad_index(z, col, r, N, P)] = xb;
}

// x passes on the half spectrum: the rows of the volume are real, so two rows
// a, b share one complex transform of a + i b.  Forward: the transform Z of
// the pair gives A[k] = (Z[k] + conj Z[N-k]) / 2 and B[k] = (Z[k] -
// conj Z[N-k]) / 2i, stored for k = 0..N/2 at (row) (N/2 + 1) + k.  Inverse:
// Z[k] = A[k] + i B[k] with A, B extended by conjugate symmetry; the inverse
// transform's real and imaginary parts are rows a and b.  TP pairs of rows
// per workgroup, element l of pair j at LDS l TP + j.
template <class T>
__global__ __launch_bounds__(256) void k_cone_fft_xpair(ConeCtx<T> c, int inverse, int out_mode, int TP, int logTP,
                                                        const T* __restrict__ tw, const T* __restrict__ real_in,
                                                        T* __restrict__ zh, T* __restrict__ real_out) {
    extern __shared__ unsigned char smem_raw[];
    const int N = c.N, logN = 31 - __builtin_clz((unsigned)c.N), H = N / 2 + 1;
    T* re = reinterpret_cast<T*>(smem_raw);
    T* im = re + TP * N;
    const int row0 = blockIdx.x * TP * 2;   // first row of the workgroup's pairs
    if (!inverse) {
        for (int t = threadIdx.x; t < TP * N; t += blockDim.x) {
            const int l = t & (N - 1), j = t >> logN;
            const size_t ea = (size_t)(row0 + 2 * j) * N + l;
            const int pos = bitrev_n(l, logN) * TP + j;
            re[pos] = real_in[ea];
            im[pos] = real_in[ea + N];
        }
        lds_dit(re, im, tw, N, logN, TP, logTP, T(1));
        for (int t = threadIdx.x; t < TP * H; t += blockDim.x) {
            const int j = t / H, k = t - j * H;
            const int m = (N - k) & (N - 1);
            const T zr = re[k * TP + j], zi = im[k * TP + j], mr = re[m * TP + j], mi = im[m * TP + j];
            T* oa = zh + 2 * ((size_t)(row0 + 2 * j) * H + k);
            T* ob = oa + 2 * H;
            oa[0] = (zr + mr) * T(0.5);
            oa[1] = (zi - mi) * T(0.5);
            ob[0] = (zi + mi) * T(0.5);
            ob[1] = (mr - zr) * T(0.5);
        }
        return;
    }
    for (int t = threadIdx.x; t < TP * H; t += blockDim.x) {
        const int j = t / H, k = t - j * H;
        const T* ia = zh + 2 * ((size_t)(row0 + 2 * j) * H + k);
        const T* ib = ia + 2 * H;
        const T ar = ia[0], ai = ia[1], br = ib[0], bi = ib[1];
        re[k * TP + j] = ar - bi;   // Z[k] = A[k] + i B[k]
        im[k * TP + j] = ai + br;
        if (k > 0 && k < N / 2) {   // Z[N-k] = conj A[k] + i conj B[k]
            re[(N - k) * TP + j] = ar + bi;
            im[(N - k) * TP + j] = br - ai;
        }
    }
    lds_dif(re, im, tw, N, logN, TP, logTP, T(-1));
    for (int t = threadIdx.x; t < TP * N; t += blockDim.x) {
        const int l = t & (N - 1), j = t >> logN;
        const int pos = bitrev_n(l, logN) * TP + j;
        x_result(c, out_mode, real_out, row0 + 2 * j, l, re[pos]);
        x_result(c, out_mode, real_out, row0 + 2 * j + 1, l, im[pos]);
    }
}

// x+ = x - w / (alpha gamma) (PDHG: M = gamma I), xbar into the padded copies
template <class T>
__global__ __launch_bounds__(256) void k_cone_update_direct(ConeCtx<T> c, T scale) {
    const size_t n = (size_t)c.N * c.N * c.NZ;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N = c.N, col = (int)(i % N), r = (int)((i / N) % N), z = (int)(i / ((size_t)N * N));
    const T xo = c.x[i];
    const T xn = xo - c.w[i] * scale;
    const T xb = T(2) * xn - xo;
    c.x[i] = xn;
    if (c.tpos) c.tpos[i] = fmin(fma(c.alpha, xb, c.tpos[i]), T(0));   // t+ = min(t + alpha xbar, 0)
    c.xbar[pad_index(z, r, col, N, c.P)] = xb;
    c.xbarT[pad_index(z, col, r, N, c.P)] = xb;
}

// a plain volume into padded copies (projector input)
template <class T>
__global__ __launch_bounds__(256) void k_cone_pad(ConeCtx<T> c, const T* __restrict__ img, T* __restrict__ pad,
                                                  T* __restrict__ padT) {
    const size_t n = (size_t)c.N * c.N * c.NZ;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int N = c.N, col = (int)(i % N), r = (int)((i / N) % N), z = (int)(i / ((size_t)N * N));
    const T v = img[i];
    pad[pad_index(z, r, col, N, c.P)] = v;
    padT[pad_index(z, col, r, N, c.P)] = v;
}

// TV dual v+ = clamp(v + beta D xbar, -s, s) and the TV term |D x+|_1
template <class T>
__global__ __launch_bounds__(256) void k_cone_tv(ConeCtx<T> c) {
    const int N = c.N, NZ = c.NZ, P = c.P;
    const size_t n2 = (size_t)N * N, n = n2 * NZ;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double tv = 0.0;
    if (i < n) {
        const int col = (int)(i % N), r = (int)((i / N) % N), z = (int)(i / n2);
        const size_t pi = pad_index(z, r, col, N, P);
        const T xb = c.xbar[pi];
        const T gx = col < N - 1 ? xb - c.xbar[pi + 1] : T(0);
        const T gy = r < N - 1 ? xb - c.xbar[pi + P] : T(0);
        const T gz = z < NZ - 1 ? xb - c.xbar[pi + (size_t)N * P] : T(0);
        T* vx = c.v;
        T* vy = c.v + n;
        T* vz = c.v + 2 * n;
        vx[i] = clampT(fma(c.beta, gx, vx[i]), -c.s_tv, c.s_tv);
        vy[i] = clampT(fma(c.beta, gy, vy[i]), -c.s_tv, c.s_tv);
        vz[i] = clampT(fma(c.beta, gz, vz[i]), -c.s_tv, c.s_tv);
        const T xv = c.x[i];
        if (col < N - 1) tv += fabs((double)xv - (double)c.x[i + 1]);
        if (r < N - 1) tv += fabs((double)xv - (double)c.x[i + N]);
        if (z < NZ - 1) tv += fabs((double)xv - (double)c.x[i + n2]);
    }
    __shared__ double sh[4];
    tv = wave_sum_d(tv);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = tv;
    __syncthreads();
    if (threadIdx.x == 0) c.part_tv[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// f(x+) from the partial sums, in a fixed order
template <class T>
__global__ __launch_bounds__(256) void k_cone_objective(ConeCtx<T> c, int slot) {
    double d = 0.0, t = 0.0;
    for (int k = threadIdx.x; k < c.n_part_data; k += 256) d += c.part_data[k];
    for (int k = threadIdx.x; k < c.n_part_tv; k += 256) t += c.part_tv[k];
    __shared__ double sd[4], st[4];
    d = wave_sum_d(d);
    t = wave_sum_d(t);
    if ((threadIdx.x & 63) == 0) {
        sd[threadIdx.x >> 6] = d;
        st[threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        c.obj[slot] = ((sd[0] + sd[1]) + (sd[2] + sd[3])) + c.lambda * ((st[0] + st[1]) + (st[2] + st[3]));
}

// num += Re(conj(F v) F z), den += |F v|^2 (the probe average of eq. H-fan)
template <class T>
__global__ __launch_bounds__(256) void k_cone_probe_acc(const T* __restrict__ fv, const T* __restrict__ fz,
                                                        double* __restrict__ num, double* __restrict__ den, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double vr = fv[2 * i], vi = fv[2 * i + 1], zr = fz[2 * i], zi = fz[2 * i + 1];
    num[i] += vr * zr + vi * zi;
    den[i] += vr * vr + vi * vi;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void set_err(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ncs::set_error_message(buf);
}

#define CONE_HIP(expr)                                                                              \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            set_err("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);     \
            return NCS_ERR_HIP;                                                                     \
        }                                                                                           \
    } while (0)

#define CONE_TRY(expr)                   \
    do {                                 \
        ncs_status s_ = (expr);          \
        if (s_ != NCS_OK) return s_;     \
    } while (0)

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

}  // namespace

struct ncs_cone {
    ncs_cone_geometry g{};
    ncs_cone_params p{};
    int dtype = NCS_F32;
    size_t tsize = 4;
    hipStream_t stream = nullptr;
    size_t n = 0, m = 0, npad = 0;
    int W = 0;
    double dgamma = 0, gamma0 = 0, dzeta = 0, norm_e1_sq = 0, mu_dc = 0;
    std::vector<double> mu;
    const void* b = nullptr;
    int iter = 0;
    int nbx = 0;   // projector workgroups along the detector columns
    int bp_run = 4;   // adjoint: voxels per lane along z (chosen at setup)
    bool operators_only = false;   // tables and workspace only (no multiplier)
    long long nnz = -1;   // counted on first request
    // device memory
    std::vector<void*> allocs;
    void *rays = nullptr, *heads = nullptr, *views = nullptr, *zeta = nullptr, *kz = nullptr, *h = nullptr;
    void* hh = nullptr;   // 1 / mu on the half spectrum
    void *tw_n = nullptr, *tw_z = nullptr;
    void *x = nullptr, *xbar = nullptr, *xbarT = nullptr, *xsc = nullptr, *xscT = nullptr;
    void *u = nullptr, *pp = nullptr, *v = nullptr, *w = nullptr, *spec = nullptr, *ysc = nullptr;
    void* tpos = nullptr;   // positivity dual (params.positivity only)
    double *part_data = nullptr, *part_tv = nullptr, *obj = nullptr;
};

namespace {

ncs_status dalloc(ncs_cone* H, void** ptr, size_t bytes) {
    *ptr = nullptr;
    hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 256));
    if (e != hipSuccess) {
        set_err("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return NCS_ERR_OOM;
    }
    H->allocs.push_back(*ptr);
    e = hipMemsetAsync(*ptr, 0, std::max<size_t>(bytes, 256), H->stream);
    if (e != hipSuccess) {
        set_err("hipMemsetAsync failed: %s", hipGetErrorString(e));
        return NCS_ERR_HIP;
    }
    return NCS_OK;
}

template <class T>
ConeCtx<T> make_ctx(const ncs_cone* H) {
    ConeCtx<T> c{};
    const ncs_cone_geometry& g = H->g;
    c.N = g.n_side;
    c.NZ = g.n_slices;
    c.NV = g.n_views;
    c.NS = g.n_bins;
    c.NR = g.n_rows;
    c.P = g.n_side + 4;
    c.W = H->W;
    c.n_part_data = g.n_views * g.n_rows * H->nbx;
    c.n_part_tv = (int)((H->n + 255) / 256);
    c.half = (T)(0.5 * (g.n_side - 1));
    c.half_z = (T)(0.5 * (g.n_slices - 1));
    c.gamma0 = (T)H->gamma0;
    c.inv_dgamma = (T)(1.0 / H->dgamma);
    c.inv_dzeta = (T)(1.0 / H->dzeta);
    c.cr = (T)(0.5 * (g.n_rows - 1));
    c.alpha = (T)H->p.alpha;
    c.beta = (T)H->p.beta;
    c.s_tv = (T)(H->p.lambda * H->p.alpha / H->p.beta);
    c.inv_na = (T)(1.0 / ((double)H->n * H->p.alpha));
    c.lambda = H->p.lambda;
    c.rays = static_cast<const ConeRay<T>*>(H->rays);
    c.heads = static_cast<const ConeRayHead<T>*>(H->heads);
    c.views = static_cast<const ConeView<T>*>(H->views);
    c.zeta = static_cast<const T*>(H->zeta);
    c.kz = static_cast<const T*>(H->kz);
    c.b = static_cast<const T*>(H->b);
    c.h = static_cast<const T*>(H->h);
    c.hh = static_cast<const T*>(H->hh);
    c.tw_n = static_cast<const T*>(H->tw_n);
    c.tw_z = static_cast<const T*>(H->tw_z);
    c.x = static_cast<T*>(H->x);
    c.xbar = static_cast<T*>(H->xbar);
    c.xbarT = static_cast<T*>(H->xbarT);
    c.u = static_cast<T*>(H->u);
    c.p = static_cast<T*>(H->pp);
    c.v = static_cast<T*>(H->v);
    c.w = static_cast<T*>(H->w);
    c.spec = static_cast<T*>(H->spec);
    c.tpos = static_cast<T*>(H->tpos);
    c.part_data = H->part_data;
    c.part_tv = H->part_tv;
    c.obj = H->obj;
    return c;
}

template <class T>
hipError_t launch_pad(const ncs_cone* H, const ConeCtx<T>& c, const void* img, void* pad, void* padT) {
    const unsigned blocks = (unsigned)((H->n + 255) / 256);
    hipLaunchKernelGGL((k_cone_pad<T>), dim3(blocks), dim3(256), 0, H->stream, c, static_cast<const T*>(img),
                       static_cast<T*>(pad), static_cast<T*>(padT));
    return hipGetLastError();
}

template <class T, bool ITER>
hipError_t launch_project(const ncs_cone* H, const ConeCtx<T>& c, const void* img, const void* imgT, void* out) {
    hipLaunchKernelGGL((k_cone_project<T, ITER>), dim3(H->nbx, H->g.n_rows, H->g.n_views), dim3(256), 0, H->stream,
                       c, static_cast<const T*>(img), static_cast<const T*>(imgT), static_cast<T*>(out));
    return hipGetLastError();
}

// Bytes of LDS per adjoint workgroup: hit lists, accumulators and, with the
// row table, N_r (slope, sqrt(1 + slope^2)) pairs.
template <class T>
size_t bp_lds_bytes(int zr, bool tab, int n_rows) {
    return (size_t)kBpWaves * kHits * 64 * (4 + 2 * sizeof(T)) + (size_t)kBpWaves * (zr + 4) * 64 * sizeof(T) +
           (tab ? (size_t)n_rows * sizeof(ZetaKz<T>) : 0);
}

template <class T, bool ITER, int ZR, bool TAB>
void launch_backproject_zr(const ncs_cone* H, const ConeCtx<T>& c, const void* y, void* out) {
    const int N = H->g.n_side, NZ = H->g.n_slices;
    hipLaunchKernelGGL((k_cone_backproject<T, ITER, ZR, TAB>), dim3((N / 8) * (N / 8), NZ / ZR),
                       dim3(kBpWaves * 64), bp_lds_bytes<T>(ZR, TAB, H->g.n_rows), H->stream, c,
                       static_cast<const T*>(y), static_cast<T*>(out));
}

template <class T, int ZR, bool TAB>
hipError_t allow_bp_lds(size_t bytes) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cone_backproject<T, false, ZR, TAB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cone_backproject<T, true, ZR, TAB>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <class T, bool ITER>
hipError_t launch_backproject(const ncs_cone* H, const ConeCtx<T>& c, const void* y, void* out) {
    // runs of H->bp_run voxels, a power of two in [4, N_z]
    const bool tab = H->g.n_rows <= kBpTableRows;
    const int zr = H->bp_run;
    if (zr == 16) {
        if (tab) launch_backproject_zr<T, ITER, 16, true>(H, c, y, out);
        else launch_backproject_zr<T, ITER, 16, false>(H, c, y, out);
    } else if (zr == 8) {
        if (tab) launch_backproject_zr<T, ITER, 8, true>(H, c, y, out);
        else launch_backproject_zr<T, ITER, 8, false>(H, c, y, out);
    } else {
        if (tab) launch_backproject_zr<T, ITER, 4, true>(H, c, y, out);
        else launch_backproject_zr<T, ITER, 4, false>(H, c, y, out);
    }
    return hipGetLastError();
}

// One line pass of the 3D DFT along the axis with L elements at stride B.
template <class T>
hipError_t launch_fft(const ncs_cone* H, const ConeCtx<T>& c, int mode, int L, int B, size_t total, const void* tw,
                      const void* real_in, void* zc) {
    // lines per workgroup: enough workgroups to fill the chip (about 2048),
    // at least 8 adjacent lines in strided passes (64-byte segments; 16 lines
    // measured 3-8% slower); a power of two that divides both the block size
    // and the line count (the half spectrum's y lines number N_z (N/2 + 1))
    const size_t lines = total / L;
    const int cap = (int)(kFftLds / (2 * sizeof(T)) / L);
    int TB = 1;
    while ((size_t)TB * 2 <= lines / 2048 && TB * 2 <= cap) TB *= 2;
    if (B > 1) TB = std::min(std::max(TB, std::min(8, cap)), B);
    TB = (int)std::min<size_t>(TB, lines);
    TB = std::min(TB, 256);
    while (lines % TB != 0) TB >>= 1;
    const unsigned blocks = (unsigned)(lines / TB);
    const size_t lds = 2 * sizeof(T) * (size_t)TB * L;
    hipLaunchKernelGGL((k_cone_fft<T>), dim3(blocks), dim3(256), lds, H->stream, c, mode, L, log2i(L), B, TB,
                       log2i(TB), static_cast<const T*>(tw), static_cast<const T*>(real_in), static_cast<T*>(zc));
    return hipGetLastError();
}

// x passes of the half spectrum: pairs of real rows (forward from real_in
// into zh) or pairs of half-spectrum rows (inverse into out_mode's result).
template <class T>
hipError_t launch_xpair(const ncs_cone* H, const ConeCtx<T>& c, bool inverse, int out_mode, const void* real_in,
                        void* zh, void* real_out) {
    const int N = H->g.n_side;
    const size_t pairs = (size_t)H->g.n_slices * N / 2;
    const int cap = (int)(kFftLds / (2 * sizeof(T)) / N);
    int TP = 1;
    while ((size_t)TP * 2 <= pairs / 2048 && TP * 2 <= cap && TP * 2 <= 256) TP *= 2;
    const unsigned blocks = (unsigned)(pairs / TP);   // pairs and TP are powers of two
    const size_t lds = 2 * sizeof(T) * (size_t)TP * N;
    hipLaunchKernelGGL((k_cone_fft_xpair<T>), dim3(blocks), dim3(256), lds, H->stream, c, inverse ? 1 : 0, out_mode,
                       TP, log2i(TP), static_cast<const T*>(H->tw_n), static_cast<const T*>(real_in),
                       static_cast<T*>(zh), static_cast<T*>(real_out));
    return hipGetLastError();
}

// The forward 3D DFT of a real volume into zc (full complex layout).
template <class T>
hipError_t launch_fft3_forward(const ncs_cone* H, const ConeCtx<T>& c, const void* real_in, void* zc) {
    const int N = H->g.n_side, NZ = H->g.n_slices;
    hipError_t e;
    if ((e = launch_fft<T>(H, c, FFT_FWD, N, 1, H->n, H->tw_n, real_in, zc)) != hipSuccess) return e;
    if ((e = launch_fft<T>(H, c, FFT_FWD, N, N, H->n, H->tw_n, nullptr, zc)) != hipSuccess) return e;
    return launch_fft<T>(H, c, FFT_FWD, NZ, N * N, H->n, H->tw_z, nullptr, zc);
}

// w (real) -> F^-1 diag(h) F w on the half spectrum (N_z N (N/2 + 1) complex
// values, ((z N + r) (N/2 + 1) + k)): x forward by pairs of rows, y forward,
// z forward x h inverse, y inverse, x inverse by pairs into real_out (scaled
// by 1/n) or into the NCS update.
template <class T>
hipError_t launch_minv(const ncs_cone* H, const ConeCtx<T>& c, const void* w, int out_mode, void* real_out) {
    const int N = H->g.n_side, NZ = H->g.n_slices, Hh = N / 2 + 1;
    const size_t half = (size_t)NZ * N * Hh;
    hipError_t e;
    if ((e = launch_xpair<T>(H, c, false, out_mode, w, H->spec, nullptr)) != hipSuccess) return e;
    if ((e = launch_fft<T>(H, c, FFT_FWD, N, Hh, half, H->tw_n, nullptr, H->spec)) != hipSuccess) return e;
    if ((e = launch_fft<T>(H, c, FFT_FWD_MUL_INV, NZ, N * Hh, half, H->tw_z, nullptr, H->spec)) != hipSuccess) return e;
    if ((e = launch_fft<T>(H, c, FFT_INV, N, Hh, half, H->tw_n, nullptr, H->spec)) != hipSuccess) return e;
    return launch_xpair<T>(H, c, true, out_mode, nullptr, H->spec, real_out);
}

template <class T>
hipError_t launch_update(const ncs_cone* H, const ConeCtx<T>& c) {
    if (H->p.method == NCS_METHOD_PDHG) {
        const unsigned blocks = (unsigned)((H->n + 255) / 256);
        hipLaunchKernelGGL((k_cone_update_direct<T>), dim3(blocks), dim3(256), 0, H->stream, c,
                           (T)(1.0 / (H->p.alpha * H->p.gamma)));
        return hipGetLastError();
    }
    return launch_minv<T>(H, c, H->w, OUT_UPDATE, nullptr);
}

template <class T>
hipError_t launch_tv(const ncs_cone* H, const ConeCtx<T>& c) {
    hipLaunchKernelGGL((k_cone_tv<T>), dim3((unsigned)((H->n + 255) / 256)), dim3(256), 0, H->stream, c);
    return hipGetLastError();
}

template <class T>
hipError_t launch_objective(const ncs_cone* H, const ConeCtx<T>& c, int slot) {
    hipLaunchKernelGGL((k_cone_objective<T>), dim3(1), dim3(256), 0, H->stream, c, slot);
    return hipGetLastError();
}

template <class T>
ncs_status run_iterations(ncs_cone* H, int k) {
    const ConeCtx<T> c = make_ctx<T>(H);
    for (int it = 0; it < k; ++it) {
        CONE_HIP((launch_backproject<T, true>(H, c, H->u, nullptr)));
        CONE_HIP(launch_update<T>(H, c));
        CONE_HIP((launch_project<T, true>(H, c, H->xbar, H->xbarT, nullptr)));
        CONE_HIP(launch_tv<T>(H, c));
        CONE_HIP(launch_objective<T>(H, c, (H->iter + it) & (kHist - 1)));
    }
    return NCS_OK;
}

// y = E x for a plain volume x (device), through the scratch padded copies
template <class T>
ncs_status forward_plain(ncs_cone* H, const void* x, void* y) {
    const ConeCtx<T> c = make_ctx<T>(H);
    CONE_HIP(launch_pad<T>(H, c, x, H->xsc, H->xscT));
    CONE_HIP((launch_project<T, false>(H, c, H->xsc, H->xscT, y)));
    return NCS_OK;
}

void build_tables(ncs_cone* H, std::vector<double>& rays, std::vector<double>& views, std::vector<double>& zeta) {
    const ncs_cone_geometry& g = H->g;
    const int N = g.n_side, NV = g.n_views, NS = g.n_bins, NR = g.n_rows;
    const double half = 0.5 * (N - 1), rs = g.source_radius, r_fov = N / std::sqrt(2.0);
    H->dgamma = 2.0 * std::asin(r_fov / rs) / (NS - 1);
    H->gamma0 = -0.5 * (NS - 1) * H->dgamma;
    H->W = (int)std::ceil(std::asin(1.0 / (rs - r_fov)) / H->dgamma + 0.5) + 1;
    const double z_max = 0.5 * g.n_slices / (rs - r_fov);
    H->dzeta = 2.0 * z_max / (NR - 1);
    rays.assign(6 * (size_t)NV * NS, 0.0);
    views.assign(4 * (size_t)NV, 0.0);
    zeta.assign(NR, 0.0);
    for (int r = 0; r < NR; ++r) zeta[r] = (r - 0.5 * (NR - 1)) * H->dzeta;
    for (int a = 0; a < NV; ++a) {
        const double beta = 2.0 * kPi * a / NV;
        const double sx = rs * std::cos(beta), sy = rs * std::sin(beta), thc = beta + kPi;
        views[4 * (size_t)a] = sx;
        views[4 * (size_t)a + 1] = sy;
        views[4 * (size_t)a + 2] = thc;
        for (int d = 0; d < NS; ++d) {
            const double th = thc + (d - 0.5 * (NS - 1)) * H->dgamma;
            const double ux = std::cos(th), uy = std::sin(th);
            double* t = &rays[6 * ((size_t)a * NS + d)];
            if (std::fabs(uy) >= std::fabs(ux) - 1e-12) {   // rows: column coordinate and distance at row r
                const double k2 = ux / uy;
                t[0] = sx - (half + sy) * k2 + half;
                t[1] = k2;
                t[2] = (-half - sy) / uy;
                t[3] = 1.0 / uy;
                t[4] = 1.0 / std::fabs(uy);
                t[5] = 0.0;
            } else {                                         // columns: row coordinate and distance at column c
                const double k2 = uy / ux;
                t[0] = sy - (half + sx) * k2 + half;
                t[1] = k2;
                t[2] = (-half - sx) / ux;
                t[3] = 1.0 / ux;
                t[4] = 1.0 / std::fabs(ux);
                t[5] = 1.0;
            }
        }
    }
}

// Probe k: n values +-1, entry 64 j + b = bit b of the j-th output of
// SplitMix64 (Steele, Lea and Flood) started from state k.
void probe_values(uint64_t index, size_t n, std::vector<double>& v) {
    v.assign(n, 0.0);
    uint64_t x = index;
    for (size_t j = 0; 64 * j < n; ++j) {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        for (int b = 0; b < 64 && 64 * j + b < n; ++b) v[64 * j + b] = ((z >> b) & 1u) ? 1.0 : -1.0;
    }
}

template <class T>
ncs_status upload(ncs_cone* H, void* dst, const std::vector<double>& src) {
    std::vector<T> tmp(src.begin(), src.end());
    CONE_HIP(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, H->stream));
    CONE_HIP(hipStreamSynchronize(H->stream));
    return NCS_OK;
}

// The adjoint's LDS depends on N_r: check it against the device's limit per
// workgroup and allow it for the two instantiations this geometry launches.
template <class T>
ncs_status prepare_backproject(ncs_cone* H) {
    const bool tab = H->g.n_rows <= kBpTableRows;
    int dev = 0, limit = 0;
    CONE_HIP(hipGetDevice(&dev));
    CONE_HIP(hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    // the longest run (up to N_z and kBpRunMax) whose accumulators fit
    int zr = std::min(H->g.n_slices, kBpRunMax);
    while (zr > 4 && bp_lds_bytes<T>(zr, tab, H->g.n_rows) > (size_t)limit) zr /= 2;
    H->bp_run = zr;
    const size_t bytes = bp_lds_bytes<T>(zr, tab, H->g.n_rows);
    if (bytes > (size_t)limit) {
        set_err("the adjoint needs %zu bytes of LDS per workgroup; the device allows %d", bytes, limit);
        return NCS_ERR_INVALID_ARG;
    }
    // the attribute belongs to the kernel, shared by every handle in the
    // process: allow the device's whole limit, so that a later handle with a
    // smaller table does not lower it under an earlier one's launches
    const size_t lim = (size_t)limit;
    const hipError_t e = zr == 16 ? (tab ? allow_bp_lds<T, 16, true>(lim) : allow_bp_lds<T, 16, false>(lim))
                         : zr == 8 ? (tab ? allow_bp_lds<T, 8, true>(lim) : allow_bp_lds<T, 8, false>(lim))
                                   : (tab ? allow_bp_lds<T, 4, true>(lim) : allow_bp_lds<T, 4, false>(lim));
    CONE_HIP(e);
    return NCS_OK;
}

template <class T>
ncs_status setup_typed(ncs_cone* H);

// num = sum_k Re(conj(F v_k) F(E^T E v_k)), den = sum_k |F v_k|^2 over the
// probes v_k (eq. H-fan), accumulated in double on the device with this
// handle's projector pair and 3D DFT.
template <class T>
ncs_status probe_estimate(ncs_cone* H, int probes, std::vector<double>& hn, std::vector<double>& hd) {
    const ConeCtx<T> c = make_ctx<T>(H);
    double *num = nullptr, *den = nullptr;
    void* spec2 = nullptr;
    CONE_TRY(dalloc(H, reinterpret_cast<void**>(&num), H->n * sizeof(double)));
    CONE_TRY(dalloc(H, reinterpret_cast<void**>(&den), H->n * sizeof(double)));
    CONE_TRY(dalloc(H, &spec2, 2 * H->n * H->tsize));
    std::vector<double> pv;
    for (int k = 0; k < probes; ++k) {
        probe_values((uint64_t)k, H->n, pv);
        CONE_TRY(upload<T>(H, H->w, pv));
        CONE_TRY(forward_plain<T>(H, H->w, H->ysc));
        CONE_HIP((launch_backproject<T, false>(H, c, H->ysc, H->x)));
        CONE_HIP(launch_fft3_forward<T>(H, c, H->w, H->spec));
        CONE_HIP(launch_fft3_forward<T>(H, c, H->x, spec2));
        hipLaunchKernelGGL((k_cone_probe_acc<T>), dim3((unsigned)((H->n + 255) / 256)), dim3(256), 0, H->stream,
                           static_cast<const T*>(H->spec), static_cast<const T*>(spec2), num, den, H->n);
        CONE_HIP(hipGetLastError());
    }
    hn.resize(H->n);
    hd.resize(H->n);
    CONE_HIP(hipMemcpyAsync(hn.data(), num, H->n * sizeof(double), hipMemcpyDeviceToHost, H->stream));
    CONE_HIP(hipMemcpyAsync(hd.data(), den, H->n * sizeof(double), hipMemcpyDeviceToHost, H->stream));
    CONE_HIP(hipStreamSynchronize(H->stream));
    // the temporaries are the last three allocations
    for (int r = 0; r < 3; ++r) {
        CONE_HIP(hipFree(H->allocs.back()));
        H->allocs.pop_back();
    }
    CONE_HIP(hipMemsetAsync(H->x, 0, H->n * H->tsize, H->stream));
    return NCS_OK;
}

// The probe estimate for a handle of either precision: a single-precision
// handle borrows a double-precision twin (same geometry, tables and
// workspace only), so that both precisions run the same M.
ncs_status probe_estimate_fp64(ncs_cone* H, int probes, std::vector<double>& hn, std::vector<double>& hd) {
    if (H->dtype == NCS_F64) return probe_estimate<double>(H, probes, hn, hd);
    ncs_cone* twin = new (std::nothrow) ncs_cone();
    if (!twin) {
        set_err("out of host memory");
        return NCS_ERR_OOM;
    }
    twin->g = H->g;
    twin->p = H->p;
    twin->dtype = NCS_F64;
    twin->tsize = 8;
    twin->stream = H->stream;
    twin->operators_only = true;
    ncs_status s = setup_typed<double>(twin);
    if (s == NCS_OK) s = probe_estimate<double>(twin, probes, hn, hd);
    ncs_cone_destroy(twin);
    return s;
}

template <class T>
ncs_status setup_typed(ncs_cone* H) {
    const ncs_cone_geometry& g = H->g;
    CONE_TRY(prepare_backproject<T>(H));
    const int N = g.n_side, NZ = g.n_slices;
    H->n = (size_t)N * N * NZ;
    H->m = (size_t)g.n_views * g.n_rows * g.n_bins;
    H->npad = (size_t)(NZ + 4) * N * (N + 4);
    H->nbx = (g.n_bins + 63) / 64;
    std::vector<double> rays, views, zeta;
    build_tables(H, rays, views, zeta);
    // device tables
    std::vector<ConeRay<T>> rt((size_t)g.n_views * g.n_bins);
    for (size_t i = 0; i < rt.size(); ++i) {
        const double* t = &rays[6 * i];
        rt[i] = ConeRay<T>{(T)t[0], (T)t[1], (T)t[2], (T)t[3], (T)t[4], (int)t[5]};
    }
    std::vector<ConeRayHead<T>> ht(rt.size());
    for (size_t i = 0; i < rt.size(); ++i) ht[i] = ConeRayHead<T>{rt[i].k0, rt[i].k2, rt[i].kxy, rt[i].axis};
    std::vector<ConeView<T>> vt(g.n_views);
    for (int a = 0; a < g.n_views; ++a)
        vt[a] = ConeView<T>{(T)views[4 * a], (T)views[4 * a + 1], (T)views[4 * a + 2], T(0)};
    std::vector<double> kz(zeta.size());
    for (size_t r = 0; r < zeta.size(); ++r) kz[r] = std::sqrt(1.0 + zeta[r] * zeta[r]);
    auto twiddles = [](int L) {
        std::vector<double> t(L, 0.0);
        for (int k = 0; k < L / 2; ++k) {
            t[2 * k] = std::cos(2.0 * kPi * k / L);
            t[2 * k + 1] = -std::sin(2.0 * kPi * k / L);
        }
        return t;
    };
    const size_t ts = sizeof(T);
    CONE_TRY(dalloc(H, &H->rays, rt.size() * sizeof(ConeRay<T>)));
    CONE_TRY(dalloc(H, &H->heads, ht.size() * sizeof(ConeRayHead<T>)));
    CONE_TRY(dalloc(H, &H->views, vt.size() * sizeof(ConeView<T>)));
    CONE_TRY(dalloc(H, &H->zeta, zeta.size() * ts));
    CONE_TRY(dalloc(H, &H->kz, kz.size() * ts));
    CONE_TRY(dalloc(H, &H->tw_n, (size_t)N * ts));
    CONE_TRY(dalloc(H, &H->tw_z, (size_t)NZ * ts));
    CONE_TRY(dalloc(H, &H->h, H->n * ts));
    CONE_TRY(dalloc(H, &H->hh, (size_t)NZ * N * (N / 2 + 1) * ts));
    CONE_TRY(dalloc(H, &H->x, H->n * ts));
    CONE_TRY(dalloc(H, &H->xbar, H->npad * ts));
    CONE_TRY(dalloc(H, &H->xbarT, H->npad * ts));
    CONE_TRY(dalloc(H, &H->xsc, H->npad * ts));
    CONE_TRY(dalloc(H, &H->xscT, H->npad * ts));
    CONE_TRY(dalloc(H, &H->u, H->m * ts));
    CONE_TRY(dalloc(H, &H->pp, H->m * ts));
    CONE_TRY(dalloc(H, &H->ysc, H->m * ts));
    CONE_TRY(dalloc(H, &H->v, 3 * H->n * ts));
    CONE_TRY(dalloc(H, &H->w, H->n * ts));
    CONE_TRY(dalloc(H, &H->spec, 2 * H->n * ts));
    if (H->p.positivity) CONE_TRY(dalloc(H, &H->tpos, H->n * ts));
    CONE_TRY(dalloc(H, reinterpret_cast<void**>(&H->part_data), (size_t)g.n_views * g.n_rows * H->nbx * sizeof(double)));
    CONE_TRY(dalloc(H, reinterpret_cast<void**>(&H->part_tv), ((H->n + 255) / 256) * sizeof(double)));
    CONE_TRY(dalloc(H, reinterpret_cast<void**>(&H->obj), kHist * sizeof(double)));
    CONE_HIP(hipMemcpyAsync(H->rays, rt.data(), rt.size() * sizeof(ConeRay<T>), hipMemcpyHostToDevice, H->stream));
    CONE_HIP(hipMemcpyAsync(H->heads, ht.data(), ht.size() * sizeof(ConeRayHead<T>), hipMemcpyHostToDevice,
                            H->stream));
    CONE_HIP(hipMemcpyAsync(H->views, vt.data(), vt.size() * sizeof(ConeView<T>), hipMemcpyHostToDevice, H->stream));
    CONE_TRY(upload<T>(H, H->zeta, zeta));
    CONE_TRY(upload<T>(H, H->kz, kz));
    CONE_TRY(upload<T>(H, H->tw_n, twiddles(N)));
    CONE_TRY(upload<T>(H, H->tw_z, twiddles(NZ)));
    if (H->operators_only) {   // a twin for probe_estimate_fp64
        CONE_HIP(hipStreamSynchronize(H->stream));
        return NCS_OK;
    }
    // |E 1|^2 (the DC eigenvalue)
    {
        std::vector<double> ones(H->n, 1.0);
        CONE_TRY(upload<T>(H, H->w, ones));
        CONE_TRY(forward_plain<T>(H, H->w, H->ysc));
        std::vector<T> y(H->m);
        CONE_HIP(hipMemcpyAsync(y.data(), H->ysc, H->m * ts, hipMemcpyDeviceToHost, H->stream));
        CONE_HIP(hipStreamSynchronize(H->stream));
        double s = 0.0;
        for (size_t i = 0; i < H->m; ++i) s += (double)y[i] * (double)y[i];
        H->norm_e1_sq = s;
    }
    const ncs_cone_params& p = H->p;
    H->mu_dc = p.mu_dc > 0.0 ? p.mu_dc : p.gamma + p.alpha * H->norm_e1_sq / (double)H->n;
    H->mu.assign(H->n, p.gamma);
    if (p.method == NCS_METHOD_NCS) {
        // eq. H-fan with the 3D DFT, always through double-precision kernels
        std::vector<double> hn, hd;
        CONE_TRY(probe_estimate_fp64(H, p.probes > 0 ? p.probes : 16, hn, hd));
        std::vector<double> s2(N), s2z(NZ);
        for (int k = 0; k < N; ++k) s2[k] = std::pow(std::sin(k * kPi / N), 2);
        for (int l = 0; l < NZ; ++l) s2z[l] = std::pow(std::sin(l * kPi / NZ), 2);
        const double ratio = p.beta * p.beta / p.alpha;
        for (int l = 0; l < NZ; ++l)
            for (int j = 0; j < N; ++j)
                for (int k = 0; k < N; ++k) {
                    const size_t i = ((size_t)l * N + j) * N + k;
                    const double he = hd[i] > 0.0 ? hn[i] / hd[i] : 0.0;
                    H->mu[i] = p.gamma + p.alpha * he + ratio * 4.0 * (s2z[l] + s2[j] + s2[k]);
                }
        H->mu[0] = H->mu_dc;
        // x >= 0 (remark in Section 4.2): A gains the rows I, so alpha A^T A and M gain alpha I
        if (p.positivity)
            for (double& m : H->mu) m += p.alpha;
    }
    std::vector<double> hv(H->n);
    for (size_t i = 0; i < H->n; ++i) hv[i] = H->mu[i] != 0.0 ? 1.0 / H->mu[i] : 0.0;
    CONE_TRY(upload<T>(H, H->h, hv));
    {   // the half spectrum's copy: k = 0..N/2 of every (z, r) line
        const int Hh = N / 2 + 1;
        std::vector<double> hhv((size_t)NZ * N * Hh);
        for (size_t row = 0; row < (size_t)NZ * N; ++row)
            for (int k = 0; k < Hh; ++k) hhv[row * Hh + k] = hv[row * N + k];
        CONE_TRY(upload<T>(H, H->hh, hhv));
    }
    CONE_HIP(hipMemsetAsync(H->w, 0, H->n * ts, H->stream));
    CONE_HIP(hipStreamSynchronize(H->stream));
    return NCS_OK;
}

// Nonzeros of E: per ray and step, the in-plane taps inside the image with
// nonzero weight times the slice taps inside the volume with nonzero weight.
long long count_nnz(const ncs_cone* H) {
    std::vector<double> rays, views, zeta;
    ncs_cone tmp;   // the tables need the geometry only
    tmp.g = H->g;
    build_tables(&tmp, rays, views, zeta);
    const ncs_cone_geometry& g = H->g;
    const int N = g.n_side, NZ = g.n_slices;
    const double hz = 0.5 * (NZ - 1);
    long long total = 0;
    for (size_t r = 0; r < rays.size() / 6; ++r) {
        const double* t = &rays[6 * r];
        for (int s = 0; s < N; ++s) {
            const double xi = s * t[1] + t[0];
            const double fl = std::floor(xi), f = xi - fl;
            const int c0 = (int)fl;
            const int cxy = (c0 >= 0 && c0 < N && f != 1.0) + (c0 + 1 >= 0 && c0 + 1 < N && f != 0.0);
            if (cxy == 0) continue;
            const double sd = s * t[3] + t[2];
            for (int rho = 0; rho < g.n_rows; ++rho) {
                const double ze = sd * zeta[rho] + hz;
                const double zl = std::floor(ze), gz = ze - zl;
                const int z0 = (int)zl;
                total += cxy * ((z0 >= 0 && z0 < NZ && gz != 1.0) + (z0 + 1 >= 0 && z0 + 1 < NZ && gz != 0.0));
            }
        }
    }
    return total;
}

constexpr uint64_t kConeStateMagic = 0x454e4f4353434e31ull;   // blob tag

struct ConeStateHeader {
    uint64_t magic;
    int32_t dtype, n_side, n_slices, n_views, n_bins, n_rows, iter, positivity, pad;
};

ncs_status check_handle(const ncs_cone* H) {
    if (!H) {
        set_err("null handle");
        return NCS_ERR_INVALID_ARG;
    }
    return NCS_OK;
}

}  // namespace

extern "C" {

ncs_status ncs_cone_setup(const ncs_cone_geometry* geom, const ncs_cone_params* params, int32_t dtype,
                          const void* b_dev, void* stream, ncs_cone** out) {
    if (!geom || !params || !out) {
        set_err("null argument");
        return NCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    const ncs_cone_geometry& g = *geom;
    const ncs_cone_params& p = *params;
    if (!is_pow2(g.n_side) || g.n_side < 16 || g.n_side > 512) {
        set_err("n_side must be a power of two in [16, 512] (got %d)", g.n_side);
        return NCS_ERR_INVALID_ARG;
    }
    if (!is_pow2(g.n_slices) || g.n_slices < 4 || g.n_slices > 256) {
        set_err("n_slices must be a power of two in [4, 256] (got %d)", g.n_slices);
        return NCS_ERR_INVALID_ARG;
    }
    if (g.n_views < 1 || g.n_bins < 2 || g.n_rows < 2 || g.reserved != 0) {
        set_err("need n_views >= 1, n_bins >= 2, n_rows >= 2 and reserved = 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (g.n_views > 65535 || g.n_rows > 65535 || (int64_t)g.n_rows * g.n_bins > (int64_t)1 << 24) {
        set_err("need n_views <= 65535, n_rows <= 65535 and n_rows * n_bins <= 2^24");
        return NCS_ERR_INVALID_ARG;
    }
    if (!(std::isfinite(g.source_radius) && g.source_radius >= g.n_side / std::sqrt(2.0) + 4.0)) {
        set_err("source_radius must be finite and >= n_side / sqrt(2) + 4");
        return NCS_ERR_INVALID_ARG;
    }
    if (dtype != NCS_F32 && dtype != NCS_F64) {
        set_err("dtype must be NCS_F32 or NCS_F64");
        return NCS_ERR_INVALID_ARG;
    }
    if (!(p.alpha > 0.0 && p.beta > 0.0 && p.gamma >= 0.0 && p.lambda >= 0.0) || !std::isfinite(p.alpha) ||
        !std::isfinite(p.beta) || !std::isfinite(p.gamma) || !std::isfinite(p.lambda)) {
        set_err("need alpha > 0, beta > 0, gamma >= 0, lambda >= 0 (finite)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method != NCS_METHOD_NCS && p.method != NCS_METHOD_PDHG) {
        set_err("cone beams run NCS_METHOD_NCS or NCS_METHOD_PDHG");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method == NCS_METHOD_PDHG && !(p.gamma > 0.0)) {
        set_err("PDHG needs gamma > 0");
        return NCS_ERR_INVALID_ARG;
    }
    if ((p.positivity != 0 && p.positivity != 1) || p.reserved != 0) {
        set_err("positivity must be 0 or 1 and reserved 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.probes < 0 || p.probes > 4096) {
        set_err("probes must be in [0, 4096]");
        return NCS_ERR_INVALID_ARG;
    }
    const double n = (double)g.n_side * g.n_side * g.n_slices;
    const double m = (double)g.n_views * g.n_rows * g.n_bins;
    if (m > 2.0e9 || n > 2.0e9) {
        set_err("volume or sinogram too large");
        return NCS_ERR_INVALID_ARG;
    }
    ncs_cone* H = new (std::nothrow) ncs_cone();
    if (!H) {
        set_err("out of host memory");
        return NCS_ERR_OOM;
    }
    H->g = g;
    H->p = p;
    H->dtype = dtype;
    H->tsize = dtype == NCS_F64 ? 8 : 4;
    H->stream = static_cast<hipStream_t>(stream);
    H->b = b_dev;
    const ncs_status s = dtype == NCS_F64 ? setup_typed<double>(H) : setup_typed<float>(H);
    if (s != NCS_OK) {
        ncs_cone_destroy(H);
        return s;
    }
    *out = H;
    return NCS_OK;
}

void ncs_cone_destroy(ncs_cone* h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void* p : h->allocs) (void)hipFree(p);
    delete h;
}

ncs_status ncs_cone_set_init(ncs_cone* h, const void* x0_dev) {
    CONE_TRY(check_handle(h));
    const size_t ts = h->tsize;
    if (x0_dev) CONE_HIP(hipMemcpyAsync(h->x, x0_dev, h->n * ts, hipMemcpyDeviceToDevice, h->stream));
    else CONE_HIP(hipMemsetAsync(h->x, 0, h->n * ts, h->stream));
    CONE_HIP(hipMemsetAsync(h->u, 0, h->m * ts, h->stream));
    CONE_HIP(hipMemsetAsync(h->v, 0, 3 * h->n * ts, h->stream));
    if (h->tpos) CONE_HIP(hipMemsetAsync(h->tpos, 0, h->n * ts, h->stream));
    // p = E x0
    if (x0_dev) {
        CONE_TRY(h->dtype == NCS_F64 ? forward_plain<double>(h, h->x, h->pp) : forward_plain<float>(h, h->x, h->pp));
    } else {
        CONE_HIP(hipMemsetAsync(h->pp, 0, h->m * ts, h->stream));
    }
    h->iter = 0;
    return NCS_OK;
}

ncs_status ncs_cone_iterate(ncs_cone* h, int32_t k, double* obj_host) {
    CONE_TRY(check_handle(h));
    if (k < 0 || (obj_host && k > kHist)) {
        set_err("k must be in [0, %d] when objectives are returned", kHist);
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("this handle has no data b");
        return NCS_ERR_INVALID_ARG;
    }
    const int first = h->iter;
    CONE_TRY(h->dtype == NCS_F64 ? run_iterations<double>(h, k) : run_iterations<float>(h, k));
    h->iter += k;
    if (!obj_host || k == 0) return NCS_OK;
    CONE_HIP(hipStreamSynchronize(h->stream));
    int done = 0;
    while (done < k) {
        const int slot = (first + done) & (kHist - 1);
        const int cnt = std::min(k - done, kHist - slot);
        CONE_HIP(hipMemcpy(obj_host + done, h->obj + slot, cnt * sizeof(double), hipMemcpyDeviceToHost));
        done += cnt;
    }
    for (int i = 0; i < k; ++i)
        if (std::isnan(obj_host[i])) {
            set_err("the objective became NaN at iteration %d", first + i + 1);
            return NCS_ERR_NONFINITE;
        }
    return NCS_OK;
}

ncs_status ncs_cone_get_x(ncs_cone* h, void* x_out_dev) {
    CONE_TRY(check_handle(h));
    if (!x_out_dev) { set_err("null output"); return NCS_ERR_INVALID_ARG; }
    CONE_HIP(hipMemcpyAsync(x_out_dev, h->x, h->n * h->tsize, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_cone_get_u(ncs_cone* h, void* u_out_dev) {
    CONE_TRY(check_handle(h));
    if (!u_out_dev) { set_err("null output"); return NCS_ERR_INVALID_ARG; }
    CONE_HIP(hipMemcpyAsync(u_out_dev, h->u, h->m * h->tsize, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_cone_get_v(ncs_cone* h, void* v_out_dev) {
    CONE_TRY(check_handle(h));
    if (!v_out_dev) { set_err("null output"); return NCS_ERR_INVALID_ARG; }
    CONE_HIP(hipMemcpyAsync(v_out_dev, h->v, 3 * h->n * h->tsize, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_cone_get_t(ncs_cone* h, void* t_out_dev) {
    CONE_TRY(check_handle(h));
    if (!t_out_dev || !h->tpos) {
        set_err(!t_out_dev ? "null output" : "ncs_cone_get_t: the handle has no positivity constraint");
        return NCS_ERR_INVALID_ARG;
    }
    CONE_HIP(hipMemcpyAsync(t_out_dev, h->tpos, h->n * h->tsize, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_cone_get_state(ncs_cone* h, void* host_buf, size_t* bytes) {
    CONE_TRY(check_handle(h));
    if (!bytes) { set_err("null size"); return NCS_ERR_INVALID_ARG; }
    const size_t ts = h->tsize, n = h->n, m = h->m;
    const size_t need = sizeof(ConeStateHeader) + ts * (n + 2 * m + 3 * n + (h->tpos ? n : 0));
    if (!host_buf) { *bytes = need; return NCS_OK; }
    if (*bytes < need) { set_err("buffer of %zu bytes, need %zu", *bytes, need); return NCS_ERR_INVALID_ARG; }
    ConeStateHeader hd{kConeStateMagic, h->dtype, h->g.n_side, h->g.n_slices, h->g.n_views, h->g.n_bins,
                       h->g.n_rows, h->iter, h->tpos ? 1 : 0, 0};
    unsigned char* o = static_cast<unsigned char*>(host_buf);
    std::memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    const std::pair<const void*, size_t> parts[] = {{h->x, n}, {h->u, m}, {h->pp, m}, {h->v, 3 * n}, {h->tpos, n}};
    for (const auto& pt : parts) {
        if (!pt.first) continue;
        CONE_HIP(hipMemcpyAsync(o, pt.first, pt.second * ts, hipMemcpyDeviceToHost, h->stream));
        o += pt.second * ts;
    }
    CONE_HIP(hipStreamSynchronize(h->stream));
    *bytes = need;
    return NCS_OK;
}

ncs_status ncs_cone_set_state(ncs_cone* h, const void* host_buf, size_t bytes) {
    CONE_TRY(check_handle(h));
    ConeStateHeader hd{};
    if (!host_buf || bytes < sizeof(hd)) { set_err("no state blob"); return NCS_ERR_INVALID_ARG; }
    std::memcpy(&hd, host_buf, sizeof(hd));
    const size_t ts = h->tsize, n = h->n, m = h->m;
    const size_t need = sizeof(hd) + ts * (n + 2 * m + 3 * n + (h->tpos ? n : 0));
    if (hd.magic != kConeStateMagic || hd.dtype != h->dtype || hd.n_side != h->g.n_side ||
        hd.n_slices != h->g.n_slices || hd.n_views != h->g.n_views || hd.n_bins != h->g.n_bins ||
        hd.n_rows != h->g.n_rows || hd.positivity != (h->tpos ? 1 : 0) || bytes != need) {
        set_err("the state blob does not match this handle");
        return NCS_ERR_INVALID_ARG;
    }
    const unsigned char* in = static_cast<const unsigned char*>(host_buf) + sizeof(hd);
    void* parts_dst[] = {h->x, h->u, h->pp, h->v, h->tpos};
    const size_t parts_n[] = {n, m, m, 3 * n, n};
    for (int i = 0; i < 5; ++i) {
        if (!parts_dst[i]) continue;
        CONE_HIP(hipMemcpyAsync(parts_dst[i], in, parts_n[i] * ts, hipMemcpyHostToDevice, h->stream));
        in += parts_n[i] * ts;
    }
    // x-bar = x is not needed: every iteration writes x-bar before reading it
    CONE_HIP(hipStreamSynchronize(h->stream));
    h->iter = hd.iter;
    return NCS_OK;
}

ncs_status ncs_cone_forward(ncs_cone* h, const void* x_dev, void* y_dev) {
    CONE_TRY(check_handle(h));
    if (!x_dev || !y_dev) { set_err("null argument"); return NCS_ERR_INVALID_ARG; }
    return h->dtype == NCS_F64 ? forward_plain<double>(h, x_dev, y_dev) : forward_plain<float>(h, x_dev, y_dev);
}

ncs_status ncs_cone_adjoint(ncs_cone* h, const void* y_dev, void* x_dev) {
    CONE_TRY(check_handle(h));
    if (!x_dev || !y_dev) { set_err("null argument"); return NCS_ERR_INVALID_ARG; }
    if (h->dtype == NCS_F64) CONE_HIP((launch_backproject<double, false>(h, make_ctx<double>(h), y_dev, x_dev)));
    else CONE_HIP((launch_backproject<float, false>(h, make_ctx<float>(h), y_dev, x_dev)));
    return NCS_OK;
}

ncs_status ncs_cone_apply_minv(ncs_cone* h, const void* w_dev, void* out_dev) {
    CONE_TRY(check_handle(h));
    if (!w_dev || !out_dev) { set_err("null argument"); return NCS_ERR_INVALID_ARG; }
    if (h->dtype == NCS_F64) {
        ConeCtx<double> c = make_ctx<double>(h);
        c.inv_na = 1.0 / (double)h->n;
        CONE_HIP(launch_minv<double>(h, c, w_dev, OUT_REAL, out_dev));
    } else {
        ConeCtx<float> c = make_ctx<float>(h);
        c.inv_na = (float)(1.0 / (double)h->n);
        CONE_HIP(launch_minv<float>(h, c, w_dev, OUT_REAL, out_dev));
    }
    return NCS_OK;
}

ncs_status ncs_cone_get_info(ncs_cone* h, ncs_cone_info* info) {
    CONE_TRY(check_handle(h));
    if (!info) { set_err("null output"); return NCS_ERR_INVALID_ARG; }
    if (h->nnz < 0) h->nnz = count_nnz(h);
    info->nnz = h->nnz;
    info->norm_e1_sq = h->norm_e1_sq;
    info->mu_dc = h->mu_dc;
    info->bin_window = h->W;
    return NCS_OK;
}

ncs_status ncs_cone_get_eigenvalues(ncs_cone* h, double* mu_host) {
    CONE_TRY(check_handle(h));
    if (!mu_host) { set_err("null output"); return NCS_ERR_INVALID_ARG; }
    std::memcpy(mu_host, h->mu.data(), h->n * sizeof(double));
    return NCS_OK;
}

}  // extern "C"

namespace {

template <class T>
ncs_status time_phases_typed(ncs_cone* H, int iters, double* ms) {
    const ConeCtx<T> c = make_ctx<T>(H);
    hipEvent_t e0, e1;
    CONE_HIP(hipEventCreate(&e0));
    CONE_HIP(hipEventCreate(&e1));
    for (int ph = 0; ph < 5; ++ph) {
        auto launch = [&]() -> hipError_t {
            switch (ph) {
                case 0: return launch_backproject<T, true>(H, c, H->u, nullptr);
                case 1: return launch_update<T>(H, c);
                case 2: return launch_project<T, true>(H, c, H->xbar, H->xbarT, nullptr);
                case 3: return launch_tv<T>(H, c);
                default: return launch_objective<T>(H, c, 0);
            }
        };
        CONE_HIP(launch());   // warm
        CONE_HIP(hipEventRecord(e0, H->stream));
        for (int i = 0; i < iters; ++i) CONE_HIP(launch());
        CONE_HIP(hipEventRecord(e1, H->stream));
        CONE_HIP(hipEventSynchronize(e1));
        float t = 0.0f;
        CONE_HIP(hipEventElapsedTime(&t, e0, e1));
        ms[ph] = (double)t / iters;
    }
    CONE_HIP(hipEventDestroy(e0));
    CONE_HIP(hipEventDestroy(e1));
    return NCS_OK;
}

}  // namespace

extern "C" ncs_status ncs_cone_time_phases(ncs_cone* h, int32_t iters, double* ms_host) {
    CONE_TRY(check_handle(h));
    if (iters < 1 || !ms_host) {
        set_err("need iters >= 1 and an output array of 5 doubles");
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("this handle has no data b");
        return NCS_ERR_INVALID_ARG;
    }
    return h->dtype == NCS_F64 ? time_phases_typed<double>(h, iters, ms_host) : time_phases_typed<float>(h, iters, ms_host);
}
