// HIP kernels of the NCS iteration for gfx950 (CDNA4), templated on the
// iterate precision T (float or double).  One NCS iteration (Section 4.1 /
// Section 4.2 of the paper) is the six phases below; in a sequence of
// iterations the objective of iteration i is reduced by the first workgroup of
// iteration i + 1's backprojection, so only the last iteration launches
// k_finalize_iter and an iteration is five launches.
//
//   k_backproject     w = alpha E^T u + beta D^T v          (pixel-driven gather;
//                     LDS-staged detector windows, direct loads or 16-byte
//                     windows per 2 x 2 pixel block)
//   k_fft_rows_fwd    row DFTs of w, two real rows per complex transform
//   k_fft_cols        column DFT, multiply by h/(alpha N^2), inverse column DFT
//   k_fft_rows_inv    inverse row DFTs; x+ = x - Delta, xbar = 2x+ - x (padded
//                     row-major copy and padded transposed copy)
//   k_project         q = E xbar (ray-driven; direct coalesced loads,
//                     LDS-staged row windows or ray pairs); u+ = prox(u + ...), p+ = (q + p)/2 =
//                     E x+, data term of x+.  Extra workgroups of the same
//                     launch do v+ = Pi(v + beta D xbar) and the TV term of
//                     x+ (double partial sums)
//   k_finalize_iter   f(x+) = partial sums added in a fixed order, history,
//                     the slice's stop flag
//
// Every kernel reads its slice's descriptor from a device array, through a
// workgroup -> (slice, local workgroup) map when several slices share one
// launch.  Iteration kernels of a slice whose stop flag is set return at
// once, so queued or replayed iterations end cleanly after the stopping test.
#define NCS_KERNEL_SOURCE 1
#include "ncs_internal.h"

#include <cmath>

namespace ncs {

namespace {

// Unroll factors of the tap loops (loads in flight per wave).
#ifndef NCS_UNROLL_BP
#define NCS_UNROLL_BP 4
#endif
#ifndef NCS_UNROLL_PAIR
#define NCS_UNROLL_PAIR 4
#endif
#ifndef NCS_UNROLL_BPQ
#define NCS_UNROLL_BPQ 2
#endif

constexpr int kRays = 64;      // rays per projector workgroup (one per lane)
constexpr int kWaves = 4;      // waves per projector / TV workgroup
constexpr int kRowWin = 96;    // LDS-window projector: padded-row elements staged per step (16-byte multiple)
#ifndef NCS_STAGE_ROWS
#define NCS_STAGE_ROWS 8
#endif
constexpr int kStageRows = NCS_STAGE_ROWS;   // LDS-window projector: steps (windows) in flight per wave
constexpr int kBpWaves = 8;    // direct backprojector: waves per 8 x 8 pixel tile
constexpr int kFftThreads = 256;
constexpr int kFinGroup = 8;  // objective partials loaded per thread before they are added

template <class T>
__device__ inline const DevCtx<T>& slot_ctx(const DevCtx<T>* __restrict__ ctxs, const Slot* __restrict__ map,
                                            int& local) {
    if (map) {
        const Slot s = map[blockIdx.x];
        local = s.local;
        return ctxs[s.slice];
    }
    local = blockIdx.x;
    return ctxs[0];
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum of a double over 256 threads; result in thread 0.
__device__ inline double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return r;
}

__device__ inline int bitrev(int i, int logn) {
    return (int)(__brev((unsigned)i) >> (32 - logn));
}

// Two consecutive elements read with one load (element alignment only).
template <class T>
struct alignas(sizeof(T)) Pair {
    T a, b;
};

template <class T>
__device__ inline Pair<T> load_pair(const T* p) {
    return *reinterpret_cast<const Pair<T>*>(p);
}

// float -> int with saturation (finite bounds for the loop-range arithmetic)
template <class T>
__device__ inline int sat_int(T v) {
    return (int)fmin(fmax(v, T(-1.0e9)), T(1.0e9));
}

template <class T>
__device__ inline T med3(T v, T lo, T hi);
template <>
__device__ inline float med3<float>(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }
template <>
__device__ inline double med3<double>(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

// floor(v) as an integer and v - floor(v), one instruction each in single
// precision (v_cvt_flr_i32_f32, v_fract_f32).
template <class T>
__device__ inline int floor_int(T v) {
    return (int)floor(v);
}
template <>
__device__ inline int floor_int<float>(float v) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}
template <class T>
__device__ inline T frac_part(T v) {
    return v - floor(v);
}
template <>
__device__ inline float frac_part<float>(float v) {
    return __builtin_amdgcn_fractf(v);
}

// Coordinates are formed as an integer from a double-precision anchor plus a
// small offset in T: the coordinate at step s + j is i + t with
// (i, t0) = (floor, fraction) of fma(s, k2, base) in double and
// t = fma(j, k2, t0) in T.  In single precision a coordinate near 300 held
// whole would carry about 1.5e-5 of rounding, and a trajectory of some
// thousand iterations amplifies those tap-weight errors by about 50 in the
// image; the split form keeps each coordinate within about 1e-6.
struct Anchor {
    int i;
    double t;
};
__device__ inline Anchor make_anchor(double x) {
    const double fl = floor(x);
    return Anchor{(int)fl, x - fl};
}

// One radix-2 butterfly of each kind on values in registers: decimation in
// time (x0, x1) <- (x0 + w x1, x0 - w x1); in frequency (x0, x1) <- (x0 + x1,
// (x0 - x1) w).
template <class T>
__device__ inline void bfly_dit(T& ar, T& ai, T& br, T& bi, T wr, T wi) {
    const T tr = wr * br - wi * bi;
    const T tim = wr * bi + wi * br;
    br = ar - tr;
    bi = ai - tim;
    ar = ar + tr;
    ai = ai + tim;
}

template <class T>
__device__ inline void bfly_dif(T& ar, T& ai, T& br, T& bi, T wr, T wi) {
    const T dr = ar - br, di = ai - bi;
    ar = ar + br;
    ai = ai + bi;
    br = wr * dr - wi * di;
    bi = wr * di + wi * dr;
}

// Radix-2 decimation-in-time transform in LDS: input in bit-reversed order,
// output in natural order.  tw[2k], tw[2k+1] = cos, -sin of 2 pi k / N.
// Stages ls and ls + 1 close over the quads (i0, i0 + h, i0 + 2h, i0 + 3h),
// h = 2^ls, so each thread takes a quad through both stages in registers:
// one LDS round trip and one barrier per two stages, the same arithmetic.
template <class T>
__device__ void fft_dit(T* re, T* im, const T* __restrict__ tw, int N, int logN, bool inverse,
                        int tid, int nthr) {
    const T sg = inverse ? T(-1) : T(1);
    int ls = 0;
    for (; ls + 1 < logN; ls += 2) {
        const int h = 1 << ls;
        __syncthreads();
        for (int q = tid; q < (N >> 2); q += nthr) {
            const int pos = q & (h - 1);
            const int i0 = ((q >> ls) << (ls + 2)) + pos;
            const int t1 = pos << (logN - ls - 1);
            const int t2 = pos << (logN - ls - 2), t3 = (pos + h) << (logN - ls - 2);
            T r0 = re[i0], m0 = im[i0], r1 = re[i0 + h], m1 = im[i0 + h];
            T r2 = re[i0 + 2 * h], m2 = im[i0 + 2 * h], r3 = re[i0 + 3 * h], m3 = im[i0 + 3 * h];
            const T w1r = tw[2 * t1], w1i = sg * tw[2 * t1 + 1];
            bfly_dit(r0, m0, r1, m1, w1r, w1i);
            bfly_dit(r2, m2, r3, m3, w1r, w1i);
            bfly_dit(r0, m0, r2, m2, tw[2 * t2], sg * tw[2 * t2 + 1]);
            bfly_dit(r1, m1, r3, m3, tw[2 * t3], sg * tw[2 * t3 + 1]);
            re[i0] = r0;
            im[i0] = m0;
            re[i0 + h] = r1;
            im[i0 + h] = m1;
            re[i0 + 2 * h] = r2;
            im[i0 + 2 * h] = m2;
            re[i0 + 3 * h] = r3;
            im[i0 + 3 * h] = m3;
        }
    }
    if (ls < logN) {   // odd stage count: the last stage alone
        const int h = 1 << ls;
        __syncthreads();
        for (int bi = tid; bi < (N >> 1); bi += nthr) {
            const int pos = bi & (h - 1);
            const int i0 = ((bi >> ls) << (ls + 1)) + pos;
            const int ti = pos << (logN - ls - 1);
            T r0 = re[i0], m0 = im[i0], r1 = re[i0 + h], m1 = im[i0 + h];
            bfly_dit(r0, m0, r1, m1, tw[2 * ti], sg * tw[2 * ti + 1]);
            re[i0] = r0;
            im[i0] = m0;
            re[i0 + h] = r1;
            im[i0 + h] = m1;
        }
    }
    __syncthreads();
}

// Radix-2 decimation-in-frequency transform in LDS: input natural, output in
// bit-reversed order; stages ls and ls - 1 are taken together on quads.
template <class T>
__device__ void fft_dif(T* re, T* im, const T* __restrict__ tw, int N, int logN, bool inverse,
                        int tid, int nthr) {
    const T sg = inverse ? T(-1) : T(1);
    int ls = logN - 1;
    for (; ls >= 1; ls -= 2) {
        const int H = 1 << ls, h = H >> 1;
        __syncthreads();
        for (int q = tid; q < (N >> 2); q += nthr) {
            const int pos = q & (h - 1);
            const int i0 = ((q >> (ls - 1)) << (ls + 1)) + pos;
            const int t1 = pos << (logN - ls - 1), t2 = (pos + h) << (logN - ls - 1);
            const int t3 = pos << (logN - ls);
            T r0 = re[i0], m0 = im[i0], r1 = re[i0 + h], m1 = im[i0 + h];
            T r2 = re[i0 + H], m2 = im[i0 + H], r3 = re[i0 + H + h], m3 = im[i0 + H + h];
            bfly_dif(r0, m0, r2, m2, tw[2 * t1], sg * tw[2 * t1 + 1]);
            bfly_dif(r1, m1, r3, m3, tw[2 * t2], sg * tw[2 * t2 + 1]);
            const T w3r = tw[2 * t3], w3i = sg * tw[2 * t3 + 1];
            bfly_dif(r0, m0, r1, m1, w3r, w3i);
            bfly_dif(r2, m2, r3, m3, w3r, w3i);
            re[i0] = r0;
            im[i0] = m0;
            re[i0 + h] = r1;
            im[i0 + h] = m1;
            re[i0 + H] = r2;
            im[i0 + H] = m2;
            re[i0 + H + h] = r3;
            im[i0 + H + h] = m3;
        }
    }
    if (ls == 0) {   // odd stage count: the last stage alone
        __syncthreads();
        for (int bi = tid; bi < (N >> 1); bi += nthr) {
            const int i0 = bi << 1;
            T r0 = re[i0], m0 = im[i0], r1 = re[i0 + 1], m1 = im[i0 + 1];
            bfly_dif(r0, m0, r1, m1, tw[0], sg * tw[1]);
            re[i0] = r0;
            im[i0] = m0;
            re[i0 + 1] = r1;
            im[i0 + 1] = m1;
        }
    }
    __syncthreads();
}

// The N/2 complex twiddles are copied to LDS (after the data area) in the
// same loop that loads a pass's data, so that the two loads are in flight
// together and no butterfly stage waits on a global load.

// The slice's stop flag through the vector-memory path (a relaxed atomic
// load): the wait for it is the wait for the data loads issued after it, so
// the two latencies overlap instead of adding up.
template <class T>
__device__ inline int stop_flag(const DevCtx<T>& c) {
    return __hip_atomic_load(&c.ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Objective of a slice after an iteration: the partial sums of the projection
// launch added in a fixed order (double) by the first 256 threads of the
// calling workgroup, the history entry and the stop test.  Every thread of
// the workgroup calls it (it synchronises).  It runs either as its own
// kernel after the last iteration of a launch sequence or at the start of
// the next iteration's backprojection; the kernel boundary orders it after
// every workgroup of the projection launch either way.
template <class T>
__device__ inline void finalize_slice(const DevCtx<T>& c, double* sh) {
    double sd = 0.0, st = 0.0;
    if (threadIdx.x < 256) {
        // each thread adds its partials in increasing index order; the loads of
        // a group of kFinGroup are issued before the first add so that the
        // group costs one memory round trip
        for (int i0 = threadIdx.x; i0 < c.nb_proj; i0 += 256 * kFinGroup) {
            double v[kFinGroup];
#pragma unroll
            for (int u = 0; u < kFinGroup; ++u) v[u] = i0 + 256 * u < c.nb_proj ? c.part_data[i0 + 256 * u] : 0.0;
#pragma unroll
            for (int u = 0; u < kFinGroup; ++u) sd += v[u];
        }
        for (int i0 = threadIdx.x; i0 < c.nb_tv; i0 += 256 * kFinGroup) {
            double v[kFinGroup];
#pragma unroll
            for (int u = 0; u < kFinGroup; ++u) v[u] = i0 + 256 * u < c.nb_tv ? c.part_tv[i0 + 256 * u] : 0.0;
#pragma unroll
            for (int u = 0; u < kFinGroup; ++u) st += v[u];
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    sd = wave_sum(sd);
    st = wave_sum(st);
    if (lane == 0 && wave < 4) {
        sh[wave] = sd;
        sh[4 + wave] = st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sd = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        st = (sh[4] + sh[5]) + (sh[6] + sh[7]);
        NCS_G Control* k = c.ctl;
        const double f = (sd + k->data_const) + c.lambda * st;
        const int it = k->iter;
        c.hist[it & (kHistCap - 1)] = f;
        k->iter = it + 1;
        k->f_last = f;
        if (f != f) {
            k->status = -4;
            k->stop = 1;
        } else if (f <= k->f_target) {
            k->status = 1;
            k->stop = 1;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Backprojection (pixel-driven gather, matched to the ray-driven projector).
// Three kernels compute the same taps: the direct one reads every tap pair
// from the sinogram in global memory, the quad one reads one 16-byte window
// per 2 x 2 pixel block, and the LDS one stages detector windows.  The
// setup timing keeps the fastest for a geometry (and, for a batch, for the
// whole batch).
//
// Direct: an 8 x 8 pixel tile per workgroup; each of the 8 waves takes every
// 8th angle; the partial sums are added in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kBpTileD = 8;   // direct kernel's tile side
constexpr int kBpTile = 16;   // LDS and quad kernels' tile side

template <class T, bool ITER>
__global__ __launch_bounds__(kBpWaves * 64) void k_backproject_direct(const DevCtx<T>* __restrict__ ctxs,
                                                                      const Slot* __restrict__ map,
                                                                      const T* __restrict__ ysrc_plain,
                                                                      T* __restrict__ out, int fin_prev) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    __shared__ T red[kBpWaves * 64];
    if (ITER) {
        __shared__ int stop_sh;
        __shared__ double fin_sh[8];
        if (threadIdx.x == 0) stop_sh = c.ctl->stop;   // one read per workgroup: the flag may change below
        __syncthreads();
        if (stop_sh) return;
        if (fin_prev && local == 0) finalize_slice(c, fin_sh);   // objective of the previous iteration
    }
    const T* ysrc = ITER ? c.u : ysrc_plain;
    const int N = c.N;
    const int tiles_x = N / kBpTileD;
    const int tx = local % tiles_x, ty = local / tiles_x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = tx * kBpTileD + (lane & 7);
    const int row = ty * kBpTileD + (lane >> 3);
    const double oc = (double)(tx * kBpTileD), orow = (double)(ty * kBpTileD);
    const T lcf = (T)(lane & 7), lrf = (T)(lane >> 3);
    const int PU = c.PU;
    const int NA = c.NA, NS = c.NS;
    const AngleT<T>* ang = c.ang;
    T acc = T(0);
#pragma unroll NCS_UNROLL_BP
    for (int a = wave; a < NA; a += kBpWaves) {
        const AngleT<T> A = ang[a];
        // the pixel's detector coordinate as the tile origin's (an integer and a
        // fraction, from double precision) plus a small offset in T; outside
        // the detector both taps land on the zero pads at d = -1, N_s, N_s + 1
        const NCS_G double* g = c.ang64 + 6 * a;
        const Anchor an = make_anchor(fma(oc, g[3], fma(orow, g[4], g[5])));
        const T tr = fma(lcf, A.q1, fma(lrf, A.q2, (T)an.t));
        const int lraw = an.i + floor_int(tr);
        const T f = lraw < -1 ? T(0) : frac_part(tr);
        const int fl = min(max(lraw, -1), NS);
        const unsigned off = (unsigned)(fl + 1);
        const Pair<T> y = load_pair(ysrc + (size_t)a * PU + off);
        const T w0 = fmax(T(0), fma(-A.kappa2, f, A.kappa));
        const T w1 = fmax(T(0), fma(A.kappa2, f, A.kd));
        acc = fma(w0, y.a, acc);
        acc = fma(w1, y.b, acc);
    }
    red[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    T bp = red[lane];
#pragma unroll
    for (int w = 1; w < kBpWaves; ++w) bp += red[w * 64 + lane];
    const size_t pix = (size_t)row * N + col;
    if (!ITER) {
        out[pix] = bp;
        return;
    }
    // D^T v with D of Section 2 (rows [1, -1]) on each axis, padded planes.
    const T* vh = c.v;
    const T* vv = c.v + (size_t)N * N;
    T dtv = T(0);
    if (col < N - 1) dtv += vh[pix];
    if (col > 0) dtv -= vh[pix - 1];
    if (row < N - 1) dtv += vv[pix];
    if (row > 0) dtv -= vv[pix - N];
    T wv = fma(c.alpha, bp, c.beta * dtv);
    if (c.tpos) wv = fma(c.alpha, c.tpos[pix], wv);   // the rows I of x >= 0 (remark in Section 4.2)
    c.w[pix] = wv;
}

// Fan beam: the direct kernel's layout (8 x 8 pixel tile, 8 waves over the
// source positions).  A ray touches a pixel only if it passes within one pixel
// of the pixel's centre, i.e. within asin(1 / |S - p|) of the centre's fan
// angle; fan_w bins on either side of the centre's bin cover that for every
// pixel of the image.  Each candidate ray's taps at this pixel are recomputed
// exactly as the projector computes them (its coordinate at the pixel's step
// along the ray's own axis), so this is the transpose of the fan projector.
template <class T, bool ITER>
__global__ __launch_bounds__(kBpWaves * 64) void k_backproject_fan(const DevCtx<T>* __restrict__ ctxs,
                                                                   const Slot* __restrict__ map,
                                                                   const T* __restrict__ ysrc_plain,
                                                                   T* __restrict__ out, int fin_prev) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    __shared__ T red[kBpWaves * 64];
    if (ITER) {
        __shared__ int stop_sh;
        __shared__ double fin_sh[8];
        if (threadIdx.x == 0) stop_sh = c.ctl->stop;   // one read per workgroup: the flag may change below
        __syncthreads();
        if (stop_sh) return;
        if (fin_prev && local == 0) finalize_slice(c, fin_sh);   // objective of the previous iteration
    }
    const T* ysrc = ITER ? c.u : ysrc_plain;
    const int N = c.N;
    const int tiles_x = N / kBpTileD;
    const int tx = local % tiles_x, ty = local / tiles_x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = tx * kBpTileD + (lane & 7);
    const int row = ty * kBpTileD + (lane >> 3);
    const T half = T(0.5) * (T)(N - 1);
    const T px = (T)col - half, py = (T)row - half;
    const T fc = (T)col, fr = (T)row, cmax = (T)N;
    const int NS = c.NS, PU = c.PU, NA = c.NA, W = c.fan_w;
    const T inv_dg = T(1) / c.dgamma;
    const T two_pi = T(6.283185307179586476925286766559);
    T acc = T(0);
    for (int a = wave; a < NA; a += kBpWaves) {
        const ViewT<T> V = c.views[a];
        // fan angle of the pixel centre from the source, relative to the central ray
        T g = atan2(py - V.sy, px - V.sx) - V.theta_c;
        g -= two_pi * rint(g / two_pi);
        const int dc = (int)floor((g - c.gamma0) * inv_dg + T(0.5));
        const int d_lo = max(dc - W, 0), d_hi = min(dc + W, NS - 1);
        const RayT<T>* rr = c.rays + (size_t)a * NS;
        const T* yrow = ysrc + (size_t)a * PU + 1;
        for (int d = d_lo; d <= d_hi; ++d) {
            const RayT<T> R = rr[d];
            const T st = R.axis == 0 ? fr : fc;   // the ray's step at this pixel
            const T tp = R.axis == 0 ? fc : fr;   // the pixel's place along the interpolated axis
            const T xi = fma(st, R.k2, R.k0);
            const T fl = med3(floor(xi), T(-2), cmax);
            const T f = xi - fl;
            const T w = tp == fl ? T(1) - f : (tp == fl + T(1) ? f : T(0));
            acc = fma(R.kappa * w, yrow[d], acc);
        }
    }
    red[wave * 64 + lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    T bp = red[lane];
#pragma unroll
    for (int w = 1; w < kBpWaves; ++w) bp += red[w * 64 + lane];
    const size_t pix = (size_t)row * N + col;
    if (!ITER) {
        out[pix] = bp;
        return;
    }
    // D^T v with D of Section 2 (rows [1, -1]) on each axis, padded planes.
    const T* vh = c.v;
    const T* vv = c.v + (size_t)N * N;
    T dtv = T(0);
    if (col < N - 1) dtv += vh[pix];
    if (col > 0) dtv -= vh[pix - 1];
    if (row < N - 1) dtv += vv[pix];
    if (row > 0) dtv -= vv[pix - N];
    T wv = fma(c.alpha, bp, c.beta * dtv);
    if (c.tpos) wv = fma(c.alpha, c.tpos[pix], wv);   // the rows I of x >= 0 (remark in Section 4.2)
    c.w[pix] = wv;
}

// Quad: a 16 x 16 pixel tile per workgroup of 16 waves; each lane takes a
// 2 x 2 pixel block and each wave every 16th angle.  The detector coordinates
// of a 2 x 2 block span |q1| + |q2| <= sqrt(2) < 2 bins, so the eight taps of
// an angle lie in 4 consecutive bins, read with one 16-byte load.  Each
// pixel's coordinate and taps are computed exactly as in the direct kernel;
// the per-pixel sums over the 16 angle groups are added in a fixed order.
constexpr int kBpQuadWaves = 16;

template <class T>
struct alignas(sizeof(T)) Four {
    T a, b, c, d;
};

template <class T>
__device__ inline T pick(int j, T v0, T v1, T v2) {
    return j == 0 ? v0 : (j == 1 ? v1 : v2);
}

template <class T, bool ITER>
__global__ __launch_bounds__(kBpQuadWaves * 64) void k_backproject_quad(const DevCtx<T>* __restrict__ ctxs,
                                                                        const Slot* __restrict__ map,
                                                                        const T* __restrict__ ysrc_plain,
                                                                        T* __restrict__ out, int fin_prev) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    if (ITER) {
        __shared__ int stop_sh;
        __shared__ double fin_sh[8];
        if (threadIdx.x == 0) stop_sh = c.ctl->stop;   // one read per workgroup: the flag may change below
        __syncthreads();
        if (stop_sh) return;
        if (fin_prev && local == 0) finalize_slice(c, fin_sh);   // objective of the previous iteration
    }
    __shared__ T red[kBpQuadWaves * kBpTile * kBpTile];
    const T* ysrc = ITER ? c.u : ysrc_plain;
    const int N = c.N;
    const int tiles_x = N / kBpTile;
    const int tx = local % tiles_x, ty = local / tiles_x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lc = 2 * (lane & 7), lr = 2 * (lane >> 3);          // block corner within the tile
    const double oc = (double)(tx * kBpTile), orow = (double)(ty * kBpTile);
    const T lc0 = (T)lc, lc1 = lc0 + T(1), lr0 = (T)lr, lr1 = lr0 + T(1);
    const int PU = c.PU, NA = c.NA, NS = c.NS;
    const AngleT<T>* ang = c.ang;
    T a00 = T(0), a01 = T(0), a10 = T(0), a11 = T(0);
#pragma unroll NCS_UNROLL_BPQ
    for (int a = wave; a < NA; a += kBpQuadWaves) {
        const AngleT<T> A = ang[a];
        // the direct kernel's coordinate of each pixel: the tile origin's (an
        // integer and a fraction, from double precision) plus a small offset in
        // T; outside the detector the taps land on the zero pads at
        // d = -1, N_s, N_s + 1 (a coordinate below -1 counts as -1)
        const NCS_G double* g = c.ang64 + 6 * a;
        const Anchor an = make_anchor(fma(oc, g[3], fma(orow, g[4], g[5])));
        const T t0 = (T)an.t;
        const T t00 = fma(lc0, A.q1, fma(lr0, A.q2, t0)), t01 = fma(lc1, A.q1, fma(lr0, A.q2, t0));
        const T t10 = fma(lc0, A.q1, fma(lr1, A.q2, t0)), t11 = fma(lc1, A.q1, fma(lr1, A.q2, t0));
        const int r00 = an.i + floor_int(t00), r01 = an.i + floor_int(t01);
        const int r10 = an.i + floor_int(t10), r11 = an.i + floor_int(t11);
        const int l00 = min(max(r00, -1), NS), l01 = min(max(r01, -1), NS);
        const int l10 = min(max(r10, -1), NS), l11 = min(max(r11, -1), NS);
        // window start: the smallest bin, kept <= N_s - 2 so that the 4 bins stay
        // inside the padded row (bins -1 .. N_s + 1)
        const int base = min(min(min(l00, l01), min(l10, l11)), NS - 2);
        const Four<T> y = *reinterpret_cast<const Four<T>*>(ysrc + (size_t)a * PU + 1 + base);
#define NCS_BP_TAP(acc, t, l, r)                                                           \
        {                                                                                  \
            const T f = r < -1 ? T(0) : frac_part(t);                                      \
            const int j = min(max(l - base, 0), 2);                                        \
            const T y0 = pick(j, y.a, y.b, y.c), y1 = pick(j, y.b, y.c, y.d);              \
            const T w0 = fmax(T(0), fma(-A.kappa2, f, A.kappa));                           \
            const T w1 = fmax(T(0), fma(A.kappa2, f, A.kd));                               \
            acc = fma(w0, y0, acc);                                                        \
            acc = fma(w1, y1, acc);                                                        \
        }
        NCS_BP_TAP(a00, t00, l00, r00)
        NCS_BP_TAP(a01, t01, l01, r01)
        NCS_BP_TAP(a10, t10, l10, r10)
        NCS_BP_TAP(a11, t11, l11, r11)
#undef NCS_BP_TAP
    }
    T* rw = red + wave * (kBpTile * kBpTile);
    rw[lr * kBpTile + lc] = a00;
    rw[lr * kBpTile + lc + 1] = a01;
    rw[(lr + 1) * kBpTile + lc] = a10;
    rw[(lr + 1) * kBpTile + lc + 1] = a11;
    __syncthreads();
    if (threadIdx.x >= kBpTile * kBpTile) return;
    const int p = threadIdx.x;
    T bp = red[p];
#pragma unroll
    for (int w = 1; w < kBpQuadWaves; ++w) bp += red[w * (kBpTile * kBpTile) + p];
    const int col = tx * kBpTile + (p & (kBpTile - 1)), row = ty * kBpTile + p / kBpTile;
    const size_t pix = (size_t)row * N + col;
    if (!ITER) {
        out[pix] = bp;
        return;
    }
    // D^T v with D of Section 2 (rows [1, -1]) on each axis, padded planes.
    const T* vh = c.v;
    const T* vv = c.v + (size_t)N * N;
    T dtv = T(0);
    if (col < N - 1) dtv += vh[pix];
    if (col > 0) dtv -= vh[pix - 1];
    if (row < N - 1) dtv += vv[pix];
    if (row > 0) dtv -= vv[pix - N];
    T wv = fma(c.alpha, bp, c.beta * dtv);
    if (c.tpos) wv = fma(c.alpha, c.tpos[pix], wv);   // the rows I of x >= 0 (remark in Section 4.2)
    c.w[pix] = wv;
}

// Hat weights clamped to [0, 1] (the clamp folds into the multiply-add).
template <class T>
__device__ inline T clamp01(T v);
template <>
__device__ inline float clamp01<float>(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
template <>
__device__ inline double clamp01<double>(double v) { return fmin(fmax(v, 0.0), 1.0); }

// LDS: a 16 x 16 pixel tile per workgroup of 16 waves, a 2 x 2 pixel block
// per lane and every 16th angle per wave (the quad kernel's layout), with the
// taps read from LDS.  For each angle the tile's detector coordinates span
// 15 (|q1| + |q2|) <= 21.3 bins, so both taps of every pixel lie in the
// kBpWin bins starting one below the floor of the tile's smallest coordinate
// (a bin of rounding margin on each side).  Those windows are staged for a
// chunk of angles with zeros for bins outside the detector, which gives the
// direct kernel's result for pixels whose coordinate is clamped there, so the
// compute loop needs no clamp.  Per pixel and angle it is the coordinate, the
// floor, the fraction, one LDS address, one two-element LDS read and the hat
// weights kappa clamp01(1 - kappa f) and kappa clamp01(1 - kappa + kappa f):
// the direct kernel's max(0, kappa - kappa^2 f) and
// max(0, kappa - kappa^2 + kappa^2 f) up to rounding, with kappa applied once
// per pixel and angle (about 12 vector instructions against the quad
// kernel's 21).
// ---------------------------------------------------------------------------
constexpr int kBpWin = 26;
template <class T>
constexpr int bp_chunk() { return sizeof(T) == 4 ? 384 : 192; }

// woffb: LDS byte offset, relative to win, of detector bin 0 in this angle's
// window; the window holds kappa u (the angle's weight scale folded in at
// staging), so each tap is the floor as an integer, the fraction, the two
// clamped weights and two multiply-adds.
template <class T>
__device__ inline void bp_window_tap(T& acc, T tc, const T* __restrict__ win, int woffb, const AngleT<T>& A) {
    const int fl = floor_int(tc);
    const T f = frac_part(tc);
    const T* wp = reinterpret_cast<const T*>(reinterpret_cast<const char*>(win) + fl * (int)sizeof(T) + woffb);
    const T y0 = wp[0], y1 = wp[1];
    const T w0 = clamp01(fma(-A.kappa, f, T(1)));
    const T w1 = clamp01(fma(A.kappa, f, A.omk));
    acc = fma(w1, y1, fma(w0, y0, acc));
}

template <class T, bool ITER>
__global__ __launch_bounds__(kBpQuadWaves * 64) void k_backproject_lds(const DevCtx<T>* __restrict__ ctxs,
                                                                       const Slot* __restrict__ map,
                                                                       const T* __restrict__ ysrc_plain,
                                                                       T* __restrict__ out, int fin_prev) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    if (ITER) {
        __shared__ int stop_sh;
        __shared__ double fin_sh[8];
        if (threadIdx.x == 0) stop_sh = c.ctl->stop;   // one read per workgroup: the flag may change below
        __syncthreads();
        if (stop_sh) return;
        if (fin_prev && local == 0) finalize_slice(c, fin_sh);   // objective of the previous iteration
    }
    constexpr int CH = bp_chunk<T>();
    constexpr int NT = kBpQuadWaves * 64;
    __shared__ T win[CH * kBpWin];
    __shared__ int wbase[CH];
    __shared__ T tref[CH];
    __shared__ T kap[CH];
    __shared__ T red[kBpQuadWaves * kBpTile * kBpTile];
    const T* ysrc = ITER ? c.u : ysrc_plain;
    const int N = c.N;
    const int tiles_x = N / kBpTile;
    const int tx = local % tiles_x, ty = local / tiles_x;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lc = 2 * (lane & 7), lr = 2 * (lane >> 3);          // block corner within the tile
    const T lc0 = (T)lc, lc1 = lc0 + T(1), lr0 = (T)lr, lr1 = lr0 + T(1);
    const int PU = c.PU, NA = c.NA, NS = c.NS;
    const double c0 = (double)(tx * kBpTile), r0 = (double)(ty * kBpTile), span = (double)(kBpTile - 1);
    const AngleT<T>* ang = c.ang;
    // the epilogue's reads (D^T v and the positivity dual of one pixel per
    // thread of the first 256) are issued now, so the staging hides them
    const int pcol = tx * kBpTile + (threadIdx.x & (kBpTile - 1)), prow = ty * kBpTile + (threadIdx.x & 255) / kBpTile;
    const size_t ppix = (size_t)prow * N + pcol;
    T dtv = T(0), tp = T(0);
    if (ITER && threadIdx.x < kBpTile * kBpTile) {
        const T* vh = c.v;
        const T* vv = c.v + (size_t)N * N;
        if (pcol < N - 1) dtv += vh[ppix];
        if (pcol > 0) dtv -= vh[ppix - 1];
        if (prow < N - 1) dtv += vv[ppix];
        if (prow > 0) dtv -= vv[ppix - N];
        if (c.tpos) tp = c.tpos[ppix];
    }
    T a00 = T(0), a01 = T(0), a10 = T(0), a11 = T(0);
    for (int a0 = 0; a0 < NA; a0 += CH) {
        const int nch = min(CH, NA - a0);
        __syncthreads();   // the previous chunk has been consumed
        // window of angle a: bins wbase .. wbase + kBpWin - 1 from one below the
        // floor of the smallest (unclamped) coordinate of the tile
        // (and the tile origin's coordinate relative to the window, in double
        // then T: a small number, so each pixel's coordinate stays within ~1e-6)
        for (int k = threadIdx.x; k < nch; k += NT) {
            const NCS_G double* g = c.ang64 + 6 * (a0 + k);
            const double q1 = g[3], q2 = g[4];
            const double torg = fma(c0, q1, fma(r0, q2, g[5]));
            const int wb = (int)floor(torg + span * (fmin(q1, 0.0) + fmin(q2, 0.0))) - 1;
            wbase[k] = wb;
            tref[k] = (T)(torg - (double)wb);
            kap[k] = ang[a0 + k].kappa;
        }
        __syncthreads();
        {
            // every load of this thread is issued before any is stored, so the
            // staging costs one memory latency; bins off the detector are zero
            constexpr int R = (CH * kBpWin + NT - 1) / NT;
            T vals[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = threadIdx.x + r * NT;
                const int k = e / kBpWin, j = e - k * kBpWin;
                const int d = e < nch * kBpWin ? wbase[k] + j : -1;
                vals[r] = (d >= 0 && d < NS) ? ysrc[(size_t)(a0 + k) * PU + 1 + d] : T(0);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = threadIdx.x + r * NT;
                if (e < nch * kBpWin) win[e] = kap[e / kBpWin] * vals[r];
            }
        }
        __syncthreads();
        for (int k = wave; k < nch; k += kBpQuadWaves) {
            const AngleT<T> A = ang[a0 + k];
            // coordinates relative to angle k's window (a wave-uniform offset, so
            // that each pixel's address is one shift-and-add)
            const int woffb = __builtin_amdgcn_readfirstlane(k * kBpWin * (int)sizeof(T));
            const T tr = tref[k];
            const T q0r0 = fma(lr0, A.q2, tr), q0r1 = fma(lr1, A.q2, tr);
            bp_window_tap(a00, fma(lc0, A.q1, q0r0), win, woffb, A);
            bp_window_tap(a01, fma(lc1, A.q1, q0r0), win, woffb, A);
            bp_window_tap(a10, fma(lc0, A.q1, q0r1), win, woffb, A);
            bp_window_tap(a11, fma(lc1, A.q1, q0r1), win, woffb, A);
        }
    }
    T* rw = red + wave * (kBpTile * kBpTile);
    rw[lr * kBpTile + lc] = a00;
    rw[lr * kBpTile + lc + 1] = a01;
    rw[(lr + 1) * kBpTile + lc] = a10;
    rw[(lr + 1) * kBpTile + lc + 1] = a11;
    __syncthreads();
    if (threadIdx.x >= kBpTile * kBpTile) return;
    const int p = threadIdx.x;
    T bp = red[p];
#pragma unroll
    for (int w = 1; w < kBpQuadWaves; ++w) bp += red[w * (kBpTile * kBpTile) + p];
    if (!ITER) {
        out[ppix] = bp;
        return;
    }
    // D^T v with D of Section 2 (rows [1, -1]) on each axis (read above)
    T wv = fma(c.alpha, bp, c.beta * dtv);
    if (c.tpos) wv = fma(c.alpha, tp, wv);   // the rows I of x >= 0 (remark in Section 4.2)
    c.w[ppix] = wv;
}

// ---------------------------------------------------------------------------
// Forward projection (Joseph, ray-driven) with the data prox, fused with the
// TV update and the objective reduction in iteration mode.
// ---------------------------------------------------------------------------
enum { PMODE_PLAIN = 0, PMODE_SETP = 1, PMODE_ITER = 2 };

// Ray sum -> output / state update.  Returns this lane's data term (ITER).
template <class T, int MODE>
__device__ inline double project_epilogue(const DevCtx<T>& c, int a, int d, T q, T* __restrict__ out) {
    const int NS = c.NS;
    const bool valid = d < NS;
    if (MODE == PMODE_PLAIN) {
        if (valid) out[(size_t)a * NS + d] = q;
        return 0.0;
    }
    if (MODE == PMODE_SETP) {
        if (valid) c.p[(size_t)a * c.PU + 1 + d] = q;
        return 0.0;
    }
    double dterm = 0.0;
    if (valid) {
        const size_t i = (size_t)a * NS + d;
        const size_t ip = (size_t)a * c.PU + 1 + d;
        const T bb = c.b[i];
        const T uu = c.u[ip];
        const T pp = c.p[ip];
        const T pn = (q + pp) * T(0.5);   // E x+ = (E xbar + E x)/2
        T un;
        if (c.data_term == DATA_QUAD) {
            un = (uu + c.alpha * (q - bb)) * c.inv1pa;
            const double e = (double)pn - (double)bb;
            dterm = 0.5 * e * e;
        } else {
            const T r = c.bg ? c.bg[i] : T(0);
            const T wv = uu + c.alpha * (q + r);
            const T cc = c.alpha * bb;
            const T t = wv - T(1);
            const T sq = sqrt(fma(t, t, T(4) * cc));
            // S(w; c) = 1 + (t - sqrt(t^2 + 4c))/2, rationalised when t > 0
            un = t > T(0) ? T(1) - T(2) * cc / (t + sq) : T(1) + (t - sq) * T(0.5);
            const double y = (double)pn + (double)r;
            const double bd = (double)bb;
            if (bd > 0.0) dterm = y > 0.0 ? y - bd * log(y) : INFINITY;
            else dterm = y;   // zero counts: l = y (indicator not reported)
        }
        c.u[ip] = un;
        c.p[ip] = pn;
    }
    return dterm;
}

// Steps [s_begin, s_end) of part `part` of `nparts` of the steps where some ray
// of the 64-ray block starting at d0 has its coordinate in [-2, N + 1]: that
// range, split evenly, so the waves of a workgroup (one per SIMD) get equal
// shares whatever the angle and block.  All rays of an angle share the slope
// k2 in s, so the block's coordinates at step s span [blo, bhi] + s k2; one
// step of margin on each side keeps the range conservative under rounding.
template <class T>
__device__ inline void block_step_range(const AngleT<T>& A, int N, int d0, int part, int nparts, int& s_begin,
                                        int& s_end) {
    const T bA = fma((T)d0, A.k1, A.k0), bB = fma((T)(d0 + kRays - 1), A.k1, A.k0);
    const T blo = fmin(bA, bB), bhi = fmax(bA, bB);
    const T lo_x = T(-2), hi_x = T(N + 1);
    int sb = 0, se = N;
    if (A.k2 > T(0)) {
        sb = max(sb, sat_int(floor((lo_x - bhi) / A.k2)) - 1);
        se = min(se, sat_int(ceil((hi_x - blo) / A.k2)) + 2);
    } else if (A.k2 < T(0)) {
        sb = max(sb, sat_int(floor((hi_x - blo) / A.k2)) - 1);
        se = min(se, sat_int(ceil((lo_x - bhi) / A.k2)) + 2);
    } else if (bhi < lo_x || blo > hi_x) {
        se = sb;
    }
    const int len = max(se - sb, 0);
    s_begin = sb + (part * len) / nparts;
    s_end = sb + ((part + 1) * len) / nparts;
}

// Ray sum of the lane's ray by the direct method: one lane per ray, the waves
// of the workgroup split the steps.  Column-stepping angles read the
// transposed copy so that every angle walks along contiguous rows.  The
// kPadL zero columns on each side of a row hold every tap of the block's rays
// at the steps of its range, so a tap is read without a clamp: per step the
// coordinate's offset from an anchor taken every 8 steps (one multiply-add),
// its floor as an integer and its fraction, one byte offset from the
// wave-uniform row address, one 8-byte load and the linear interpolation.
template <class T>
__device__ inline T ray_sum_direct(const DevCtx<T>& c, const T* __restrict__ img, const T* __restrict__ imgT,
                                   const AngleT<T>& A, int a, int axis, int d0, int d, int part, int nparts) {
    const int P = c.P;
    const T* src = axis == 0 ? img : imgT;
    const NCS_G double* g = c.ang64 + 6 * a;
    const double k2d = g[1], based = fma((double)d, g[0], g[2]);
    int s_begin, s_end;
    block_step_range(A, c.N, d0, part, nparts, s_begin, s_end);
    const T k2 = A.k2;
    T acc = T(0);
    // the row address is the same for the whole wave (scalar registers); each
    // lane adds a 32-bit byte offset (the zero margin keeps it nonnegative)
    const char* row = reinterpret_cast<const char*>(src + (size_t)max(s_begin, 0) * P);
    const size_t pitch = (size_t)P * sizeof(T);
    constexpr unsigned pad_bytes = kPadL * sizeof(T);
    constexpr int B = 8;   // steps per anchor and unrolled group (loads in flight per lane)
    int s = s_begin;
    for (; s + B <= s_end; s += B) {
        const Anchor an = make_anchor(fma((double)s, k2d, based));
        const T t0 = (T)an.t;
        Pair<T> v[B];
        T f[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const T t = j == 0 ? t0 : fma((T)j, k2, t0);
            f[j] = frac_part(t);
            const unsigned boff = (unsigned)(an.i + floor_int(t)) * (unsigned)sizeof(T) + pad_bytes;
            v[j] = *reinterpret_cast<const Pair<T>*>(row + (size_t)j * pitch + boff);
        }
#pragma unroll
        for (int j = 0; j < B; ++j) acc += fma(f[j], v[j].b - v[j].a, v[j].a);
        row += B * pitch;
    }
    for (; s < s_end; ++s) {
        const Anchor an = make_anchor(fma((double)s, k2d, based));
        const T t = (T)an.t;
        const unsigned boff = (unsigned)an.i * (unsigned)sizeof(T) + pad_bytes;
        const Pair<T> v = *reinterpret_cast<const Pair<T>*>(row + boff);
        acc += fma(t, v.b - v.a, v.a);
        row += pitch;
    }
    return acc;
}

// Ray sums of two adjacent rays per lane: lane (h, p) of a wave takes rays
// d0 + 2p and d0 + 2p + 1 over step range 2 wave + h of 8.  The two rays'
// coordinates at a step differ by |k1| <= sqrt(2) < 2 columns, so their four
// taps lie in 4 consecutive padded-row elements, read with one 16-byte load;
// each tap's arithmetic is that of the direct method.  Partial sums of the 8
// step ranges go to red[range * 64 + ray].
template <class T>
__device__ inline void ray_sum_pair(const DevCtx<T>& c, const T* __restrict__ img, const T* __restrict__ imgT,
                                    const AngleT<T>& A, int a, int axis, int d0, int lane, int wave, T* red) {
    const int N = c.N, P = c.P;
    const T* src = axis == 0 ? img : imgT;
    const int h = lane >> 5, pr = lane & 31;
    const int da = d0 + 2 * pr;
    const NCS_G double* g = c.ang64 + 6 * a;
    const double k2d = g[1], b0d = fma((double)da, g[0], g[2]), b1d = fma((double)(da + 1), g[0], g[2]);
    const T bA = fma((T)d0, A.k1, A.k0), bB = fma((T)(d0 + kRays - 1), A.k1, A.k0);
    const T blo = fmin(bA, bB), bhi = fmax(bA, bB);
    const T lo_x = T(-2), hi_x = T(N + 1);
    const int range = 2 * wave + h;
    const int SW = N / (2 * kWaves);
    int s_begin = range * SW, s_end = s_begin + SW;
    if (A.k2 > T(0)) {
        s_begin = max(s_begin, sat_int(floor((lo_x - bhi) / A.k2)) - 1);
        s_end = min(s_end, sat_int(ceil((hi_x - blo) / A.k2)) + 2);
    } else if (A.k2 < T(0)) {
        s_begin = max(s_begin, sat_int(floor((hi_x - blo) / A.k2)) - 1);
        s_end = min(s_end, sat_int(ceil((lo_x - bhi) / A.k2)) + 2);
    } else if (bhi < lo_x || blo > hi_x) {
        s_end = s_begin;
    }
    const T k2 = A.k2;
    T acc0 = T(0), acc1 = T(0);
    for (int s0 = s_begin; s0 < s_end; s0 += NCS_UNROLL_PAIR) {
        // anchors of both rays every NCS_UNROLL_PAIR steps (coordinates as integer + offset)
        const Anchor a0 = make_anchor(fma((double)s0, k2d, b0d)), a1 = make_anchor(fma((double)s0, k2d, b1d));
        const T t00 = (T)a0.t, t10 = (T)a1.t;
#pragma unroll
        for (int j = 0; j < NCS_UNROLL_PAIR; ++j) {
            if (s0 + j >= s_end) break;
            const T t0 = j == 0 ? t00 : fma((T)j, k2, t00), t1 = j == 0 ? t10 : fma((T)j, k2, t10);
            // taps off the image read the zero columns
            const int l0 = min(max(a0.i + floor_int(t0), -2), N), l1 = min(max(a1.i + floor_int(t1), -2), N);
            // the 4 elements from the smaller tap, kept inside the padded row
            const int base = min(min(l0, l1), N - 2);
            const Four<T> v = *reinterpret_cast<const Four<T>*>(src + (size_t)(s0 + j) * P + base + kPadL);
            const int j0 = min(max(l0 - base, 0), 2), j1 = min(max(l1 - base, 0), 2);
            const T f0 = frac_part(t0), f1 = frac_part(t1);
            const T u0 = pick(j0, v.a, v.b, v.c), w0 = pick(j0, v.b, v.c, v.d);
            const T u1 = pick(j1, v.a, v.b, v.c), w1 = pick(j1, v.b, v.c, v.d);
            acc0 += fma(f0, w0 - u0, u0);
            acc1 += fma(f1, w1 - u1, u1);
        }
    }
    red[range * kRays + 2 * pr] = acc0;
    red[range * kRays + 2 * pr + 1] = acc1;
}

// Ray sum through LDS row windows.  At step s the 64 rays of a block read
// padded-row elements within 93 of the block's smallest tap (the block spans
// 63 |k1| <= 89.1 columns, plus the second tap), so the wave copies the
// kRowWin-element window that starts at the smallest tap, rounded down to 16
// bytes, into LDS with coalesced 16-byte loads, and each lane reads its two
// taps there.  The texture-address unit spends about 16 cycles on any vector
// load instruction, whatever its lanes and width, so what counts is loads per
// step: in FP32 a window is 24 lanes' worth, and one instruction loads two
// steps' windows (lanes 0-23 and 32-55), half a load per step against one
// gather per step in the direct method.  The smallest tap is the first
// lane's for k1 > 0 and the last lane's otherwise (the coordinate is monotone
// in the ray index).  Steps, anchors and the arithmetic of every tap are those
// of the direct method; each wave holds kStageRows windows (its steps in
// flight).
typedef unsigned int Bytes16 __attribute__((ext_vector_type(4)));

__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ inline T ray_sum_lds(const DevCtx<T>& c, const T* __restrict__ img, const T* __restrict__ imgT,
                                const AngleT<T>& A, int a, int axis, int d0, int d, int lane, int part, int nparts,
                                T* slots) {
    const int P = c.P;
    const T* src = axis == 0 ? img : imgT;
    const NCS_G double* g = c.ang64 + 6 * a;
    const double k2d = g[1], based = fma((double)d, g[0], g[2]);
    int s_begin, s_end;
    block_step_range(A, c.N, d0, part, nparts, s_begin, s_end);
    const T k2 = A.k2;
    const int lmin = __builtin_amdgcn_readfirstlane(A.k1 > T(0) ? 0 : kRays - 1);
    constexpr int EQ = 16 / (int)sizeof(T);   // elements per 16-byte load
    constexpr int NQ = kRowWin / EQ;          // lanes per window (24 in FP32, 48 in FP64)
    constexpr int WPI = NQ <= 32 ? 2 : 1;     // windows per load instruction
    constexpr int B = kStageRows;
    static_assert(B % WPI == 0, "steps per group must be a multiple of the windows per load");
    const int half = WPI == 2 ? lane >> 5 : 0;
    const int hmask = -half;                  // all ones in the upper half of the wave
    const int ql = WPI == 2 ? lane & 31 : lane;
    const bool loader = ql < NQ;
    const int wmaxb = (P - kRowWin) * (int)sizeof(T);   // last window start inside the row (bytes)
    const int pitch32 = P * (int)sizeof(T);
    const unsigned lane_off = (unsigned)(half * pitch32 + ql * 16);
    T* const st = slots + half * kRowWin + ql * EQ;
    const char* row = reinterpret_cast<const char*>(src + (size_t)max(s_begin, 0) * P);
    T acc = T(0);
    int s = s_begin;
    // coordinates of the B steps from sg: fractions, tap element indices, window
    // starts (in bytes, so that neither the loads nor the LDS reads rescale them)
    auto coords = [&](int sg, T(&f)[B], int(&e)[B], int(&w)[B]) {
        const Anchor an = make_anchor(fma((double)sg, k2d, based));
        const T t0 = (T)an.t;
        const int ei = an.i + kPadL;
        const int eimin = __builtin_amdgcn_readlane(ei, lmin);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const T t = j == 0 ? t0 : fma((T)j, k2, t0);
            const int fl = floor_int(t);
            f[j] = frac_part(t);
            e[j] = ei + fl;
            w[j] = min(((eimin + __builtin_amdgcn_readlane(fl, lmin)) * (int)sizeof(T)) & ~15, wmaxb);
        }
    };
    // the group's window loads, all in flight together (scalar base, 32-bit lane offset)
    auto issue = [&](const char* rg, const int(&w)[B], Bytes16(&v)[B / WPI]) {
        if (loader) {
#pragma unroll
            for (int p = 0; p < B / WPI; ++p) {
                // the lane's window start, w[2p] or w[2p + 1] (bytes), without an indexed access
                const int wb0 = w[WPI * p];
                const int dwb = WPI == 2 ? w[2 * p + 1] - w[2 * p] : 0;
                const unsigned off = lane_off + (unsigned)wb0 + (unsigned)(dwb & hmask);
                v[p] = *reinterpret_cast<const Bytes16*>(rg + (unsigned)(WPI * p * pitch32) + off);
            }
        }
    };
    // windows into LDS, then each lane's two taps per step
    auto consume = [&](const T(&f)[B], const int(&e)[B], const int(&w)[B], const Bytes16(&v)[B / WPI]) {
        wave_lds_sync();   // the previous group's taps have been read
        if (loader) {
#pragma unroll
            for (int p = 0; p < B / WPI; ++p) *reinterpret_cast<Bytes16*>(st + WPI * p * kRowWin) = v[p];
        }
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < B; ++j) {
            const T* tp = reinterpret_cast<const T*>(reinterpret_cast<const char*>(slots + j * kRowWin) - w[j]) + e[j];
            acc += fma(f[j], tp[1] - tp[0], tp[0]);
        }
    };
    const size_t gstep = (size_t)B * pitch32;
    const int ng = (s_end - s) / B;   // whole groups (s_end >= s)
    for (int gi = 0; gi < ng; ++gi) {
        T f[B];
        int e[B], w[B];
        Bytes16 v[B / WPI];
        coords(s, f, e, w);
        issue(row, w, v);
        consume(f, e, w, v);
        s += B;
        row += gstep;
    }
    for (; s < s_end; ++s) {   // remaining steps one at a time (window slot 0, loaded by the lower half)
        const Anchor an = make_anchor(fma((double)s, k2d, based));
        const T t = (T)an.t;
        const int e = an.i + kPadL;
        const int w = min((__builtin_amdgcn_readlane(e, lmin) * (int)sizeof(T)) & ~15, wmaxb);
        Bytes16 v;
        const bool ld = loader && half == 0;
        if (ld) v = *reinterpret_cast<const Bytes16*>(row + ((unsigned)w + lane_off));
        wave_lds_sync();
        if (ld) *reinterpret_cast<Bytes16*>(st) = v;
        wave_lds_sync();
        const T* tp = reinterpret_cast<const T*>(reinterpret_cast<const char*>(slots) - w) + e;
        acc += fma(t, tp[1] - tp[0], tp[0]);
        row += pitch32;
    }
    return acc;
}

// Fan beam: the lane's ray summed over this wave's quarter of the steps.  Each
// ray steps along its own axis (from the table), so lanes of one wave may read
// the row-major or the transposed copy; each lane keeps to the steps where its
// coordinate lies in [-2, N+1] (the zero columns each side absorb the taps of
// the steps next to those).  The arithmetic of a tap is the direct method's.
template <class T>
__device__ inline T ray_sum_fan(const DevCtx<T>& c, const T* __restrict__ img, const T* __restrict__ imgT,
                                const RayT<T>& R, bool valid, int wave) {
    const int N = c.N, P = c.P;
    const T* src = R.axis == 0 ? img : imgT;
    const int SW = N / kWaves;
    int s_begin = wave * SW, s_end = s_begin + SW;
    const T lo_x = T(-2), hi_x = T(N + 1);
    if (!valid) {
        s_end = s_begin;
    } else if (R.k2 > T(0)) {
        s_begin = max(s_begin, sat_int(floor((lo_x - R.k0) / R.k2)) - 1);
        s_end = min(s_end, sat_int(ceil((hi_x - R.k0) / R.k2)) + 2);
    } else if (R.k2 < T(0)) {
        s_begin = max(s_begin, sat_int(floor((hi_x - R.k0) / R.k2)) - 1);
        s_end = min(s_end, sat_int(ceil((lo_x - R.k0) / R.k2)) + 2);
    } else if (R.k0 < lo_x || R.k0 > hi_x) {
        s_end = s_begin;
    }
    const T cmax = (T)N;
    T acc = T(0);
    for (int s = s_begin; s < s_end; ++s) {
        const T xi = fma((T)s, R.k2, R.k0);
        const T fl = med3(floor(xi), T(-2), cmax);   // taps off the image read the zero columns
        const T f = xi - fl;
        const char* row = reinterpret_cast<const char*>(src + (size_t)s * P);   // the same for the wave
        const Pair<T> v = *reinterpret_cast<const Pair<T>*>(row + (unsigned)((int)fl + kPadL) * (unsigned)sizeof(T));
        acc += fma(f, v.b - v.a, v.a);
    }
    return acc;
}

// TV dual update of one 256-pixel tile and the TV term of x+ (ITER only).
template <class T>
__device__ inline double tv_pixel(const DevCtx<T>& c, size_t pix) {
    const int N = c.N;
    const size_t NN = (size_t)N * N;
    if (pix >= NN) return 0.0;
    const int r = (int)(pix >> c.log2N);
    const int col = (int)(pix & (size_t)(N - 1));
    const bool hx = col < N - 1, hy = r < N - 1;
    const T* xbp = c.xbar + (size_t)r * c.P + col + kPadL;
    const T xb = xbp[0];
    const T dh = hx ? xb - xbp[1] : T(0);
    const T dv = hy ? xb - xbp[c.P] : T(0);
    T* vh = c.v;
    T* vv = c.v + NN;
    const T gh = fma(c.beta, dh, vh[pix]);
    const T gv = fma(c.beta, dv, vv[pix]);
    const T s = c.s_tv;
    if (c.tv_term == TV_ANISO) {
        vh[pix] = fmin(fmax(gh, -s), s);
        vv[pix] = fmin(fmax(gv, -s), s);
    } else {
        const T nrm = sqrt(fma(gh, gh, gv * gv));
        const T sc = nrm > s ? s / nrm : T(1);
        vh[pix] = gh * sc;
        vv[pix] = gv * sc;
    }
    const double xx = (double)c.x[pix];
    const double th = hx ? xx - (double)c.x[pix + 1] : 0.0;
    const double tw = hy ? xx - (double)c.x[pix + N] : 0.0;
    return c.tv_term == TV_ANISO ? fabs(th) + fabs(tw) : sqrt(th * th + tw * tw);
}

template <class T>
__device__ inline double tv_tile(const DevCtx<T>& c, int tile) {
    return tv_pixel(c, (size_t)tile * 256 + threadIdx.x);
}

template <class T>
__global__ __launch_bounds__(256) void k_finalize_iter(const DevCtx<T>* __restrict__ ctxs,
                                                       const Slot* __restrict__ map) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    if (c.ctl->stop) return;
    __shared__ double sh[8];
    finalize_slice(c, sh);
}

template <class T, int MODE, int VARIANT>
__global__ __launch_bounds__(256) void k_project(const DevCtx<T>* __restrict__ ctxs, const Slot* __restrict__ map,
                                                 T* __restrict__ out) {
    int local;
    const DevCtx<T>& c = slot_ctx(ctxs, map, local);
    // the stop flag is read at the start, with the angle's coefficients, and
    // tested before the first global write (a stopped slice computes the ray
    // sums and discards them)
    const int stop = MODE == PMODE_ITER ? c.ctl->stop : 0;
    __shared__ T red[2 * kWaves * kRays];
    __shared__ double shd[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T* img = MODE == PMODE_ITER ? c.xbar : c.xsc;
    const T* imgT = MODE == PMODE_ITER ? c.xbarT : c.xscT;
    if (MODE == PMODE_ITER && local >= c.nwg_proj) {
        if (c.ctl->stop) return;   // its own read: the TV workgroups write v at once
        const double tv = block_sum256(tv_tile(c, local - c.nwg_proj), shd);
        if (threadIdx.x == 0) c.part_tv[local - c.nwg_proj] = tv;
        return;
    }
    const int nb = (c.NS + kRays - 1) / kRays;
    int a, rb;
    if (c.aorder) {   // XCDs 0-3: row-stepping blocks, XCDs 4-7: column-stepping blocks
        const int xcd = local & 7, k = (local >> 3) * 4 + (xcd & 3);
        const bool colsax = xcd >= 4;
        const int nang = colsax ? c.NA - c.nar : c.nar;
        if (k >= nang * nb) return;   // an idle slot of the split grid
        // longest first: the central ray blocks of every angle are dispatched
        // before the outer ones, whose rays cross less of the image (many
        // none), so the workgroups left after the first resident round are
        // the short ones.  Order of rb: c0, c0 + 1, c0 - 1, c0 + 2, ...
        const int rbi = k / nang, j = k - rbi * nang;
        rb = (nb - 1) / 2 + ((rbi & 1) ? (rbi + 1) >> 1 : -(rbi >> 1));
        a = c.aorder[(colsax ? c.nar : 0) + j];
    } else {
        a = local / nb;
        rb = local - a * nb;
    }
    const int blk = a * nb + rb;   // this block's data partial
    const int d0 = rb * kRays;
    const int d = d0 + lane;
    const AngleT<T> A = c.ang[a];
    const int axis = c.axis[a];
    if (VARIANT == 4) {   // fan beam: per-ray coefficients and axis
        const bool valid = d < c.NS;
        const RayT<T> R = c.rays[(size_t)a * c.NS + (valid ? d : c.NS - 1)];
        red[wave * kRays + lane] = ray_sum_fan(c, img, imgT, R, valid, wave);
        __syncthreads();
        if (wave != 0 || stop) return;   // a stopped slice writes nothing
        const T q = ((red[lane] + red[kRays + lane]) + (red[2 * kRays + lane] + red[3 * kRays + lane])) * R.kappa;
        const double dterm = wave_sum(project_epilogue<T, MODE>(c, a, d, q, out));
        if (MODE == PMODE_ITER && lane == 0) c.part_data[blk] = dterm;
        return;
    }
    if (VARIANT == 3) {
        ray_sum_pair(c, img, imgT, A, a, axis, d0, lane, wave, red);
        __syncthreads();
        if (wave != 0 || stop) return;   // a stopped slice writes nothing
        T sum = red[lane];
#pragma unroll
        for (int r = 1; r < 2 * kWaves; ++r) sum += red[r * kRays + lane];
        const T q = sum * A.kappa;
        const double dterm = wave_sum(project_epilogue<T, MODE>(c, a, d, q, out));
        if (MODE == PMODE_ITER && lane == 0) c.part_data[blk] = dterm;
        return;
    }
    T acc;
    if (VARIANT == 1) {
        __shared__ __attribute__((aligned(16))) T stage[kWaves * kStageRows * kRowWin];
        acc = ray_sum_lds(c, img, imgT, A, a, axis, d0, d, lane, wave, kWaves, stage + wave * kStageRows * kRowWin);
    } else {
        acc = ray_sum_direct(c, img, imgT, A, a, axis, d0, d, wave, kWaves);
    }
    red[wave * kRays + lane] = acc;
    __syncthreads();
    if (wave != 0 || stop) return;   // a stopped slice writes nothing
    const T q = ((red[lane] + red[kRays + lane]) + (red[2 * kRays + lane] + red[3 * kRays + lane])) * A.kappa;
    const double dterm = wave_sum(project_epilogue<T, MODE>(c, a, d, q, out));
    if (MODE == PMODE_ITER && lane == 0) c.part_data[blk] = dterm;
}

// ---------------------------------------------------------------------------
// Circulant solve: 2D DFT as row transforms (two real rows packed in one
// complex transform), column transforms with the multiplier, inverse rows.
// ---------------------------------------------------------------------------
template <class T, bool ITER>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_fwd(const DevCtx<T>* __restrict__ ctxs,
                                                              const Slot* __restrict__ map,
                                                              const T* __restrict__ src_plain) {
    int pr;
    const DevCtx<T>& c = slot_ctx(ctxs, map, pr);
    // the stop flag is read while the rows load (its latency overlaps theirs);
    // nothing global is written before it is tested
    const int stop = ITER ? stop_flag(c) : 0;
    extern __shared__ unsigned char smem_raw[];
    T* re = reinterpret_cast<T*>(smem_raw);
    T* im = re + c.N;
    T* twl = im + c.N;
    const T* tw = twl;
    const int N = c.N, logN = c.log2N;
    const T* src = ITER ? c.w : src_plain;
    const T* ra = src + (size_t)(2 * pr) * N;
    const T* rb = ra + N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const T t = c.tw[n], va = ra[n], vb = rb[n];
        const int i = bitrev(n, logN);
        twl[n] = t;
        re[i] = va;
        im[i] = vb;
    }
    if (stop) return;   // uniform: the whole workgroup returns before its first barrier
    fft_dit(re, im, tw, N, logN, false, threadIdx.x, blockDim.x);
    for (int k = threadIdx.x; k <= (N >> 1); k += blockDim.x) {
        const int m = (N - k) & (N - 1);
        const T zr = re[k], zi = im[k], mr = re[m], mi = im[m];
        T* o = c.spec + 2 * ((size_t)k * N + 2 * pr);
        o[0] = (zr + mr) * T(0.5);   // row 2pr:   (Z[k] + conj Z[N-k]) / 2
        o[1] = (zi - mi) * T(0.5);
        o[2] = (zi + mi) * T(0.5);   // row 2pr+1: (Z[k] - conj Z[N-k]) / 2i
        o[3] = (mr - zr) * T(0.5);
    }
}

template <class T, bool ITER>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(const DevCtx<T>* __restrict__ ctxs,
                                                          const Slot* __restrict__ map, T scale) {
    int k;
    const DevCtx<T>& c = slot_ctx(ctxs, map, k);
    const int stop = ITER ? stop_flag(c) : 0;   // read with the column; tested before any global write
    extern __shared__ unsigned char smem_raw[];
    T* re = reinterpret_cast<T*>(smem_raw);
    T* im = re + c.N;
    T* twl = im + c.N;
    const T* tw = twl;
    const int N = c.N, logN = c.log2N;
    T* colp = c.spec + 2 * (size_t)k * N;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const T t = c.tw[n], vr = colp[2 * n], vi = colp[2 * n + 1];
        const int i = bitrev(n, logN);
        twl[n] = t;
        re[i] = vr;
        im[i] = vi;
    }
    // the multiplier of this thread's first entry is read now, so that the
    // forward transform hides its latency
    const T* hk = c.hh + (size_t)k * N;
    const T h0 = (int)threadIdx.x < N ? hk[threadIdx.x] : T(0);
    if (stop) return;   // uniform: the whole workgroup returns before its first barrier
    fft_dit(re, im, tw, N, logN, false, threadIdx.x, blockDim.x);
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const T hv = (j == (int)threadIdx.x ? h0 : hk[j]) * scale;
        re[j] *= hv;
        im[j] *= hv;
    }
    fft_dif(re, im, tw, N, logN, true, threadIdx.x, blockDim.x);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int i = bitrev(n, logN);
        colp[2 * n] = re[i];
        colp[2 * n + 1] = im[i];
    }
}

template <class T, bool ITER>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_inv(const DevCtx<T>* __restrict__ ctxs,
                                                              const Slot* __restrict__ map, T* __restrict__ out) {
    int pr;
    const DevCtx<T>& c = slot_ctx(ctxs, map, pr);
    const int stop = ITER ? stop_flag(c) : 0;   // read with the spectrum; tested before any global write
    extern __shared__ unsigned char smem_raw[];
    T* re = reinterpret_cast<T*>(smem_raw);
    T* im = re + c.N;
    T* twl = im + c.N;
    const T* tw = twl;
    const int N = c.N, logN = c.log2N;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        const int kk = k <= (N >> 1) ? k : N - k;
        const T* s = c.spec + 2 * ((size_t)kk * N + 2 * pr);
        const T t = c.tw[k];
        const T ar = s[0], br = s[2];
        T ai = s[1], bi = s[3];
        twl[k] = t;
        if (k > (N >> 1)) {   // Hermitian extension of both real-row spectra
            ai = -ai;
            bi = -bi;
        }
        re[k] = ar - bi;      // Z = Ya + i Yb
        im[k] = ai + br;
    }
    const size_t ra = (size_t)(2 * pr) * N, rb = ra + N;
    // the iterate's values of this thread's first column are read before the
    // transform, so that their latency overlaps it
    T xa0 = T(0), xb0 = T(0);
    if (ITER && (int)threadIdx.x < N) {
        xa0 = c.x[ra + threadIdx.x];
        xb0 = c.x[rb + threadIdx.x];
    }
    if (stop) return;   // uniform: the whole workgroup returns before its first barrier
    fft_dif(re, im, tw, N, logN, true, threadIdx.x, blockDim.x);
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        const int i = bitrev(n, logN);
        const T da = re[i], db = im[i];
        if (!ITER) {
            out[ra + n] = da;
            out[rb + n] = db;
            continue;
        }
        const bool first = n == (int)threadIdx.x;
        const T xa = first ? xa0 : c.x[ra + n], xb = first ? xb0 : c.x[rb + n];
        const T na = xa - da, nb = xb - db;
        c.x[ra + n] = na;
        c.x[rb + n] = nb;
        const T ba = fma(T(2), na, -xa), bb = fma(T(2), nb, -xb);
        if (c.tpos) {   // t+ = min(t + alpha xbar, 0): the conjugate prox of the indicator of x >= 0
            c.tpos[ra + n] = fmin(fma(c.alpha, ba, c.tpos[ra + n]), T(0));
            c.tpos[rb + n] = fmin(fma(c.alpha, bb, c.tpos[rb + n]), T(0));
        }
        c.xbar[(size_t)(2 * pr) * c.P + n + kPadL] = ba;
        c.xbar[(size_t)(2 * pr + 1) * c.P + n + kPadL] = bb;
        *reinterpret_cast<Pair<T>*>(c.xbarT + (size_t)n * c.P + 2 * pr + kPadL) = Pair<T>{ba, bb};
    }
}

// ---------------------------------------------------------------------------
// Single-slice helpers: objective evaluation, padding, duals, data constant.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_tv_eval(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ img) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const int N = c.N;
    const size_t NN = (size_t)N * N;
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    double tvv = 0.0;
    if (pix < NN) {
        const int r = (int)(pix >> c.log2N);
        const int col = (int)(pix & (size_t)(N - 1));
        const double xx = (double)img[pix];
        const double th = col < N - 1 ? xx - (double)img[pix + 1] : 0.0;
        const double tw = r < N - 1 ? xx - (double)img[pix + N] : 0.0;
        tvv = c.tv_term == TV_ANISO ? fabs(th) + fabs(tw) : sqrt(th * th + tw * tw);
    }
    const double tot = block_sum256(tvv, sh);
    if (threadIdx.x == 0) c.part_tv[blockIdx.x] = tot;
}

// Data term of a projected image q (unpadded, NA*NS) (objective evaluation).
template <class T>
__global__ __launch_bounds__(256) void k_data_eval(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ q) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const size_t m = (size_t)c.NA * c.NS;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    double dterm = 0.0;
    if (i < m) {
        const double y0 = (double)q[i];
        const double bd = (double)c.b[i];
        if (c.data_term == DATA_QUAD) {
            const double e = y0 - bd;
            dterm = 0.5 * e * e;
        } else {
            const double y = y0 + (c.bg ? (double)c.bg[i] : 0.0);
            if (bd > 0.0) dterm = y > 0.0 ? y - bd * log(y) : INFINITY;
            else dterm = y;
        }
    }
    const double tot = block_sum256(dterm, sh);
    if (threadIdx.x == 0) c.part_data[blockIdx.x] = tot;
}

// PET constant sum_i log Gamma(b_i + 1).
template <class T>
__global__ __launch_bounds__(256) void k_lgamma_part(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const size_t m = (size_t)c.NA * c.NS;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (i < m) v = lgamma((double)c.b[i] + 1.0);
    const double tot = block_sum256(v, sh);
    if (threadIdx.x == 0) c.part_data[blockIdx.x] = tot;
}

// Sum of squares of a sinogram (|E 1|^2 at setup).
template <class T>
__global__ __launch_bounds__(256) void k_sumsq(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ q) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const size_t m = (size_t)c.NA * c.NS;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (i < m) {
        const double y = (double)q[i];
        v = y * y;
    }
    const double tot = block_sum256(v, sh);
    if (threadIdx.x == 0) c.part_data[blockIdx.x] = tot;
}

// Fill the interior of the padded scratch pair with ones.
template <class T>
__global__ __launch_bounds__(256) void k_ones_image(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (size_t)c.N * c.N) return;
    const int r = (int)(pix >> c.log2N);
    const int col = (int)(pix & (size_t)(c.N - 1));
    c.xsc[(size_t)r * c.P + col + kPadL] = T(1);
    c.xscT[(size_t)col * c.P + r + kPadL] = T(1);
}

// Fixed-point residual of the primal iterate: |x^k - x^{k-1}|^2, formed as
// |xbar - x^k|^2 since xbar = 2 x^k - x^{k-1}, and |x^k|^2, both in double,
// into the control block.  One workgroup strides over the image (evaluated at
// host checks only).
template <class T>
__global__ __launch_bounds__(256) void k_step_residual(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh_d[kWaves], sh_x[kWaves];
    const size_t nn = (size_t)c.N * c.N;
    double ds = 0.0, xs = 0.0;
    for (size_t pix = threadIdx.x; pix < nn; pix += 256) {
        const int r = (int)(pix >> c.log2N);
        const int col = (int)(pix & (size_t)(c.N - 1));
        const double xp = (double)c.x[pix];
        const double d = (double)c.xbar[(size_t)r * c.P + col + kPadL] - xp;
        ds = fma(d, d, ds);
        xs = fma(xp, xp, xs);
    }
    const double td = block_sum256(ds, sh_d);
    const double tx = block_sum256(xs, sh_x);
    if (threadIdx.x == 0) {
        c.ctl->step_sq = td;
        c.ctl->x_sq = tx;
    }
}

// which: 1 = evaluation (eval_out = data + constant + lambda TV),
//        2 = data constant (data_const = sum of data partials),
//        3 = plain sum (eval_out = sum of data partials).
template <class T>
__global__ __launch_bounds__(256) void k_finalize(const DevCtx<T>* __restrict__ ctxs, int nd, int nt, int which) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    double sd = 0.0, st = 0.0;
    for (int i = threadIdx.x; i < nd; i += 256) sd += c.part_data[i];
    for (int i = threadIdx.x; i < nt; i += 256) st += c.part_tv[i];
    sd = block_sum256(sd, sh);
    __syncthreads();
    st = block_sum256(st, sh);
    if (threadIdx.x != 0) return;
    Control* k = c.ctl;
    if (which == 2) {
        k->data_const = sd;
        return;
    }
    if (which == 3) {
        k->eval_out = sd;
        return;
    }
    k->eval_out = (sd + k->data_const) + c.lambda * st;
}

template <class T>
__global__ __launch_bounds__(256) void k_pad(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ y,
                                             T* __restrict__ yp) {
    const DevCtx<T>& c = ctxs[0];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t tot = (size_t)c.NA * c.PU;
    if (i >= tot) return;
    const int a = (int)(i / c.PU);
    const int j = (int)(i - (size_t)a * c.PU) - 1;
    yp[i] = (j >= 0 && j < c.NS) ? y[(size_t)a * c.NS + j] : T(0);
}

template <class T>
__global__ __launch_bounds__(256) void k_unpad(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ yp,
                                               T* __restrict__ y) {
    const DevCtx<T>& c = ctxs[0];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t tot = (size_t)c.NA * c.NS;
    if (i >= tot) return;
    const int a = (int)(i / c.NS);
    const int d = (int)(i - (size_t)a * c.NS);
    y[i] = yp[(size_t)a * c.PU + 1 + d];
}

// Write an image into the padded scratch pair (row-major and transposed).
template <class T>
__global__ __launch_bounds__(256) void k_pad_image(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ img) {
    const DevCtx<T>& c = ctxs[0];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t NN = (size_t)c.N * c.N;
    if (pix >= NN) return;
    const int r = (int)(pix >> c.log2N);
    const int col = (int)(pix & (size_t)(c.N - 1));
    const T v = img[pix];
    c.xsc[(size_t)r * c.P + col + kPadL] = v;
    c.xscT[(size_t)col * c.P + r + kPadL] = v;
}

// Descriptor and per-angle tables of a parallel beam written on the device
// (the descriptor arrives by value as a kernel argument): angle a's AngleT
// fields and its double-precision coefficients, as the host computes them for
// a handle (Joseph reading of Section 4.1.1; integer 45-degree test).
__global__ __launch_bounds__(256) void k_parallel_tables(DevCtx<float> c, DevCtx<float>* __restrict__ dst,
                                                         AngleT<float>* __restrict__ ang, double* __restrict__ ang64,
                                                         int32_t* __restrict__ axis) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    if (a == 0) *dst = c;
    if (a >= c.NA) return;
    const int N = c.N, NA = c.NA, NS = c.NS;
    const double hn = 0.5 * (N - 1), hs = 0.5 * (NS - 1);
    const double th = 3.14159265358979323846 * a / NA;
    const double ct = cos(th), st = sin(th);
    const bool rows = (4 * (long long)a <= NA) || (4 * (long long)a >= 3 * (long long)NA);
    double t[10];
    if (rows) {
        t[0] = 1.0 / ct;
        t[1] = -st / ct;
        t[2] = -hs / ct + hn * st / ct + hn;
        t[6] = 1.0 / fabs(ct);
    } else {
        t[0] = 1.0 / st;
        t[1] = -ct / st;
        t[2] = -hs / st + hn * ct / st + hn;
        t[6] = 1.0 / fabs(st);
    }
    t[3] = ct;
    t[4] = st;
    t[5] = hs - hn * (ct + st);
    t[7] = t[6] * t[6];
    t[8] = t[6] - t[7];
    t[9] = 1.0 - t[6];
    AngleT<float> A;
    A.k1 = (float)t[0];
    A.k2 = (float)t[1];
    A.k0 = (float)t[2];
    A.q1 = (float)t[3];
    A.q2 = (float)t[4];
    A.q0 = (float)t[5];
    A.kappa = (float)t[6];
    A.kappa2 = (float)t[7];
    A.kd = (float)t[8];
    A.omk = (float)t[9];
    ang[a] = A;
    for (int k = 0; k < 6; ++k) ang64[6 * a + k] = t[k];
    axis[a] = rows ? 0 : 1;
}

// The whole padded scratch pair, margins included: row-major and transposed
// copies of img with kPadL zero columns on each side (for scratch memory whose
// margins hold another call's values).
template <class T>
__global__ __launch_bounds__(256) void k_pad_image_full(const DevCtx<T>* __restrict__ ctxs,
                                                        const T* __restrict__ img) {
    const DevCtx<T>& c = ctxs[0];
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t tot = (size_t)c.N * c.P;
    if (e >= tot) return;
    const int r = (int)(e / (size_t)c.P);
    const int col = (int)(e - (size_t)r * c.P) - kPadL;
    const bool in = col >= 0 && col < c.N;
    c.xsc[e] = in ? img[(size_t)r * c.N + col] : T(0);
    c.xscT[e] = in ? img[(size_t)col * c.N + r] : T(0);
}

// Dual initialisation from x0 (fixed-point relations of the optimality
// conditions): u = grad g_data(E x0) from p = E x0; v from D x0.
template <class T>
__global__ __launch_bounds__(256) void k_dual_init_u(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t m = (size_t)c.NA * c.NS;
    if (i >= m) return;
    const int a = (int)(i / c.NS);
    const int d = (int)(i - (size_t)a * c.NS);
    const size_t ip = (size_t)a * c.PU + 1 + d;
    const T pp = c.p[ip];
    const T bb = c.b[i];
    T un;
    if (c.data_term == DATA_QUAD) {
        un = pp - bb;
    } else {
        const T y = pp + (c.bg ? c.bg[i] : T(0));
        // grad of l(y; b) = 1 - b/y on the domain; the dual of a ray outside
        // the domain is left at 0
        un = y > T(0) ? T(1) - bb / y : T(0);
    }
    c.u[ip] = un;
}

template <class T>
__global__ __launch_bounds__(256) void k_dual_init_v(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    const int N = c.N;
    const size_t NN = (size_t)N * N;
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= NN) return;
    const int r = (int)(pix >> c.log2N);
    const int col = (int)(pix & (size_t)(N - 1));
    const T xx = c.x[pix];
    const T dh = col < N - 1 ? xx - c.x[pix + 1] : T(0);
    const T dv = r < N - 1 ? xx - c.x[pix + N] : T(0);
    const T s = c.s_tv;
    const T tau = c.dual_ramp;
    T vh, vv;
    if (c.tv_term == TV_ANISO) {
        if (tau > T(0)) {
            vh = s * fmin(fmax(dh / tau, T(-1)), T(1));
            vv = s * fmin(fmax(dv / tau, T(-1)), T(1));
        } else {
            vh = dh > T(0) ? s : (dh < T(0) ? -s : T(0));
            vv = dv > T(0) ? s : (dv < T(0) ? -s : T(0));
        }
    } else {
        const T nrm = sqrt(fma(dh, dh, dv * dv));
        const T den = fmax(nrm, tau);
        vh = den > T(0) ? s * dh / den : T(0);
        vv = den > T(0) ? s * dv / den : T(0);
    }
    c.v[pix] = vh;
    c.v[pix + NN] = vv;
}

// Shepp-Logan filtering of each projection (filtered backprojection): with
// unit bin spacing the filter is h(n) = -2 / (pi^2 (4 n^2 - 1)), applied as a
// linear convolution over the detector (zero outside it).  The output goes to
// the padded sinogram, scaled by pi / N_theta so that one backprojection gives
// the FBP image.  One workgroup per angle; the projection and the filter taps
// are staged in LDS.
constexpr int kFbpMaxBins = 4096;

template <class T>
__global__ __launch_bounds__(256) void k_fbp_filter(const DevCtx<T>* __restrict__ ctxs, const T* __restrict__ y,
                                                    T* __restrict__ ypad) {
    const DevCtx<T>& c = ctxs[0];
    extern __shared__ unsigned char fbp_smem[];
    T* yl = reinterpret_cast<T*>(fbp_smem);
    T* hl = yl + c.NS;
    const int a = blockIdx.x, NS = c.NS;
    const double pi = 3.14159265358979323846;
    for (int k = threadIdx.x; k < NS; k += 256) {
        yl[k] = y[(size_t)a * NS + k];
        const double nn = (double)k;
        hl[k] = (T)(-2.0 / (pi * pi * (4.0 * nn * nn - 1.0)));
    }
    __syncthreads();
    const T scale = (T)(pi / (double)c.NA);
    T* out = ypad + (size_t)a * c.PU;
    for (int d = threadIdx.x; d < NS; d += 256) {
        T acc = T(0);
        for (int k = 0; k < NS; ++k) acc = fma(hl[d > k ? d - k : k - d], yl[k], acc);
        out[1 + d] = acc * scale;
    }
    if (threadIdx.x == 0) {
        out[0] = T(0);
        out[NS + 1] = T(0);
        out[NS + 2] = T(0);
    }
}

// ---------------------------------------------------------------------------
// ADMM with conjugate-gradient inner solves (the comparison method of
// Section 5): x+ = x - d / alpha with d ~ (A^T A)^-1 g, g = E^T u + (beta/alpha)
// D^T v = w / alpha, by a fixed number of (preconditioned) CG steps from
// d = 0.  Dot products use per-block partial sums added in a fixed order;
// the CG scalars stay in device memory (cg_s: r.z, p.q, a, b).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_cg_start(const DevCtx<T>* __restrict__ ctxs, int precond) {
    const DevCtx<T>& c = ctxs[0];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (size_t)c.N * c.N) return;
    const T r = c.w[pix] / c.alpha;
    c.cg_d[pix] = T(0);
    c.cg_r[pix] = r;
    if (!precond) c.cg_z[pix] = r;
}

// part[block] = sum over the block's pixels of a * b
template <class T>
__global__ __launch_bounds__(256) void k_cg_dot(const DevCtx<T>* __restrict__ ctxs, int which) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (pix < (size_t)c.N * c.N) v = which == 0 ? (double)c.cg_r[pix] * (double)c.cg_z[pix] : 0.0;
    v = block_sum256(v, sh);
    if (threadIdx.x == 0) c.cg_part[blockIdx.x] = v;
}

// q += (beta/alpha)^2 D^T D p (q holds E^T E p), and part[block] = p . q
template <class T>
__global__ __launch_bounds__(256) void k_cg_normal(const DevCtx<T>* __restrict__ ctxs, T ratio2) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    const int N = c.N;
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (pix < (size_t)N * N) {
        const int r = (int)(pix >> c.log2N), col = (int)(pix & (size_t)(N - 1));
        const T* p = c.cg_p;
        // D of Section 2 on each axis: (D p)_h = p(r, c) - p(r, c + 1), zero in the last column
        auto dh = [&](size_t i, int cc) { return cc < N - 1 ? p[i] - p[i + 1] : T(0); };
        auto dv = [&](size_t i, int rr) { return rr < N - 1 ? p[i] - p[i + N] : T(0); };
        T dtd = dh(pix, col) + dv(pix, r);
        if (col > 0) dtd -= dh(pix - 1, col - 1);
        if (r > 0) dtd -= dv(pix - N, r - 1);
        const T q = fma(ratio2, dtd, c.cg_q[pix]);
        c.cg_q[pix] = q;
        v = (double)p[pix] * (double)q;
    }
    v = block_sum256(v, sh);
    if (threadIdx.x == 0) c.cg_part[blockIdx.x] = v;
}

// One workgroup: the sum of the partials and the scalar update.
//   op 0: r.z;  op 1: p.q and a = r.z / p.q;  op 2: b = r.z' / r.z and r.z = r.z'
// A zero denominator gives a zero step (the oracle's convention).
template <class T>
__global__ __launch_bounds__(256) void k_cg_scalar(const DevCtx<T>* __restrict__ ctxs, int nb, int op) {
    const DevCtx<T>& c = ctxs[0];
    __shared__ double sh[kWaves];
    double v = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) v += c.cg_part[i];
    v = block_sum256(v, sh);
    if (threadIdx.x != 0) return;
    NCS_G double* s = c.cg_s;
    if (op == 0) {
        s[0] = v;
    } else if (op == 1) {
        s[1] = v;
        s[2] = v != 0.0 ? s[0] / v : 0.0;
    } else {
        s[3] = s[0] != 0.0 ? v / s[0] : 0.0;
        s[0] = v;
    }
}

// d += a p, r -= a q (and z = r without a preconditioner)
template <class T>
__global__ __launch_bounds__(256) void k_cg_step(const DevCtx<T>* __restrict__ ctxs, int precond) {
    const DevCtx<T>& c = ctxs[0];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (size_t)c.N * c.N) return;
    const T a = (T)c.cg_s[2];
    c.cg_d[pix] = fma(a, c.cg_p[pix], c.cg_d[pix]);
    const T r = fma(-a, c.cg_q[pix], c.cg_r[pix]);
    c.cg_r[pix] = r;
    if (!precond) c.cg_z[pix] = r;
}

// p = z (first direction) or p = z + b p
template <class T>
__global__ __launch_bounds__(256) void k_cg_dir(const DevCtx<T>* __restrict__ ctxs, int first) {
    const DevCtx<T>& c = ctxs[0];
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (size_t)c.N * c.N) return;
    c.cg_p[pix] = first ? c.cg_z[pix] : fma((T)c.cg_s[3], c.cg_p[pix], c.cg_z[pix]);
}

// x+ = x - d / alpha, xbar = 2 x+ - x (padded row-major and padded transpose);
// an iteration after the stopping one leaves the state alone
template <class T>
__global__ __launch_bounds__(256) void k_admm_update(const DevCtx<T>* __restrict__ ctxs) {
    const DevCtx<T>& c = ctxs[0];
    if (c.ctl->stop) return;
    const int N = c.N;
    const size_t pix = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (pix >= (size_t)N * N) return;
    const int r = (int)(pix >> c.log2N), col = (int)(pix & (size_t)(N - 1));
    const T x = c.x[pix];
    const T xn = x - c.cg_d[pix] / c.alpha;
    c.x[pix] = xn;
    const T xb = fma(T(2), xn, -x);
    c.xbar[(size_t)r * c.P + col + kPadL] = xb;
    c.xbarT[(size_t)col * c.P + r + kPadL] = xb;
}

__global__ void k_control(Control* ctl, int op, int iter_value, double f_target) {
    if (threadIdx.x != 0) return;
    if (op == 3 || op == 4) {   // raise / clear the stop flag alone (dry replays of captured graphs)
        ctl->stop = op == 3 ? 1 : 0;
        return;
    }
    if (op == 0) ctl->iter = 0;
    if (op == 2) ctl->iter = iter_value;
    ctl->stop = 0;
    ctl->status = 0;
    ctl->f_target = f_target;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

template <class T>
inline size_t fft_lds(int N) { return 3 * (size_t)N * sizeof(T); }   // re, im, twiddles

template <class T, int MODE>
hipError_t launch_project(const DevCtx<T>* ctxs, const Slot* map, int blocks, int projector, T* out,
                          hipStream_t st) {
    if (projector == 4)
        hipLaunchKernelGGL((k_project<T, MODE, 4>), dim3(blocks), dim3(256), 0, st, ctxs, map, out);
    else if (projector == 1)
        hipLaunchKernelGGL((k_project<T, MODE, 1>), dim3(blocks), dim3(256), 0, st, ctxs, map, out);
    else if (projector == 3)
        hipLaunchKernelGGL((k_project<T, MODE, 3>), dim3(blocks), dim3(256), 0, st, ctxs, map, out);
    else
        hipLaunchKernelGGL((k_project<T, MODE, 2>), dim3(blocks), dim3(256), 0, st, ctxs, map, out);
    return hipGetLastError();
}

}  // namespace

int project_blocks(int NA, int NS) { return NA * ((NS + kRays - 1) / kRays); }

int project_wgs_split(int NA, int NS, int nar) {
    const int nb = (NS + kRays - 1) / kRays;
    const int items = std::max(nar, NA - nar) * nb;
    return 8 * ((items + 3) / 4);
}

int tv_blocks(int N) { return (int)blocks_for((size_t)N * N); }
int cg_blocks(int N) { return (int)blocks_for((size_t)N * N); }

int bp_blocks(int N, int variant) {
    const int t = (variant == 2 || variant == 4) ? kBpTileD : kBpTile;
    return (N / t) * (N / t);
}

hipError_t launch_control(Control* ctl, int op, int iter_value, double f_target, hipStream_t st) {
    hipLaunchKernelGGL(k_control, dim3(1), dim3(64), 0, st, ctl, op, iter_value, f_target);
    return hipGetLastError();
}

template <class T>
hipError_t launch_bp_iter(const IterLaunch<T>& L, int fin_prev, hipStream_t st) {
    if (L.backprojector == 4)
        hipLaunchKernelGGL((k_backproject_fan<T, true>), dim3(L.bp.blocks), dim3(kBpWaves * 64), 0, st, L.ctxs,
                           L.bp.map, (const T*)nullptr, (T*)nullptr, fin_prev);
    else if (L.backprojector == 3)
        hipLaunchKernelGGL((k_backproject_quad<T, true>), dim3(L.bp.blocks), dim3(kBpQuadWaves * 64), 0, st, L.ctxs,
                           L.bp.map, (const T*)nullptr, (T*)nullptr, fin_prev);
    else if (L.backprojector == 1)
        hipLaunchKernelGGL((k_backproject_lds<T, true>), dim3(L.bp.blocks), dim3(kBpQuadWaves * 64), 0, st, L.ctxs,
                           L.bp.map, (const T*)nullptr, (T*)nullptr, fin_prev);
    else
        hipLaunchKernelGGL((k_backproject_direct<T, true>), dim3(L.bp.blocks), dim3(kBpWaves * 64), 0, st, L.ctxs,
                           L.bp.map, (const T*)nullptr, (T*)nullptr, fin_prev);
    return hipGetLastError();
}

template <class T>
hipError_t launch_iteration_phase(const IterLaunch<T>& L, int phase, hipStream_t st) {
    const size_t sm = fft_lds<T>(L.max_N);
    switch (phase) {
        case 0:
            return launch_bp_iter<T>(L, 0, st);
        case 1:
            hipLaunchKernelGGL((k_fft_rows_fwd<T, true>), dim3(L.rows.blocks), dim3(kFftThreads), sm, st, L.ctxs,
                               L.rows.map, (const T*)nullptr);
            break;
        case 2:
            hipLaunchKernelGGL((k_fft_cols<T, true>), dim3(L.cols.blocks), dim3(kFftThreads), sm, st, L.ctxs,
                               L.cols.map, T(1));
            break;
        case 3:
            hipLaunchKernelGGL((k_fft_rows_inv<T, true>), dim3(L.rows.blocks), dim3(kFftThreads), sm, st, L.ctxs,
                               L.rows.map, (T*)nullptr);
            break;
        case 4:
            return launch_project<T, PMODE_ITER>(L.ctxs, L.proj.map, L.proj.blocks, L.projector, (T*)nullptr, st);
        default:
            hipLaunchKernelGGL((k_finalize_iter<T>), dim3(L.fin.blocks), dim3(256), 0, st, L.ctxs, L.fin.map);
            break;
    }
    return hipGetLastError();
}

// k iterations: the objective of iteration i is reduced at the start of
// iteration i + 1's backprojection, and that of the last by one finalize
// launch, so each iteration is five launches.
template <class T>
hipError_t launch_iterations(const IterLaunch<T>& L, int k, hipStream_t st) {
    for (int i = 0; i < k; ++i) {
        hipError_t e = launch_bp_iter<T>(L, i > 0 ? 1 : 0, st);
        for (int ph = 1; ph < kNumPhases - 1 && e == hipSuccess; ++ph) e = launch_iteration_phase<T>(L, ph, st);
        if (e != hipSuccess) return e;
    }
    return k > 0 ? launch_iteration_phase<T>(L, kNumPhases - 1, st) : hipSuccess;
}

template <class T>
hipError_t launch_admm_iterations(const IterLaunch<T>& L, const DevCtx<T>& hc, int k, int cg_iters, int precond,
                                  hipStream_t st) {
    const DevCtx<T>* dc = L.ctxs;
    const int nb = cg_blocks(hc.N);
    const T ratio2 = (hc.beta / hc.alpha) * (hc.beta / hc.alpha);
    const T a2 = hc.alpha * hc.alpha;   // the column pass scales h/(alpha N^2): alpha^2 gives alpha M^+
    const size_t sm = fft_lds<T>(hc.N);
    auto precondition = [&]() {
        hipLaunchKernelGGL((k_fft_rows_fwd<T, false>), dim3(hc.N / 2), dim3(kFftThreads), sm, st, dc,
                           (const Slot*)nullptr, (const T*)hc.cg_r);
        hipLaunchKernelGGL((k_fft_cols<T, false>), dim3(hc.N / 2 + 1), dim3(kFftThreads), sm, st, dc,
                           (const Slot*)nullptr, a2);
        hipLaunchKernelGGL((k_fft_rows_inv<T, false>), dim3(hc.N / 2), dim3(kFftThreads), sm, st, dc,
                           (const Slot*)nullptr, (T*)hc.cg_z);
    };
    for (int i = 0; i < k; ++i) {
        hipError_t e = launch_bp_iter<T>(L, i > 0 ? 1 : 0, st);   // w = alpha E^T u + beta D^T v
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_cg_start<T>), dim3(nb), dim3(256), 0, st, dc, precond);
        if (precond) precondition();
        hipLaunchKernelGGL((k_cg_dot<T>), dim3(nb), dim3(256), 0, st, dc, 0);
        hipLaunchKernelGGL((k_cg_scalar<T>), dim3(1), dim3(256), 0, st, dc, nb, 0);
        hipLaunchKernelGGL((k_cg_dir<T>), dim3(nb), dim3(256), 0, st, dc, 1);
        for (int j = 0; j < cg_iters; ++j) {
            // q = A^T A p = E^T E p + (beta/alpha)^2 D^T D p
            hipLaunchKernelGGL((k_pad_image<T>), dim3(tv_blocks(hc.N)), dim3(256), 0, st, dc, (const T*)hc.cg_p);
            if ((e = launch_project_plain<T>(hc, dc, L.projector, (T*)hc.cg_y, st)) != hipSuccess) return e;
            if ((e = launch_pad_sinogram<T>(hc, dc, (const T*)hc.cg_y, hc.ysc, st)) != hipSuccess) return e;
            if ((e = launch_backproject_plain<T>(hc, dc, L.backprojector, hc.ysc, hc.cg_q, st)) != hipSuccess)
                return e;
            hipLaunchKernelGGL((k_cg_normal<T>), dim3(nb), dim3(256), 0, st, dc, ratio2);
            hipLaunchKernelGGL((k_cg_scalar<T>), dim3(1), dim3(256), 0, st, dc, nb, 1);
            hipLaunchKernelGGL((k_cg_step<T>), dim3(nb), dim3(256), 0, st, dc, precond);
            if (precond) precondition();
            hipLaunchKernelGGL((k_cg_dot<T>), dim3(nb), dim3(256), 0, st, dc, 0);
            hipLaunchKernelGGL((k_cg_scalar<T>), dim3(1), dim3(256), 0, st, dc, nb, 2);
            hipLaunchKernelGGL((k_cg_dir<T>), dim3(nb), dim3(256), 0, st, dc, 0);
        }
        hipLaunchKernelGGL((k_admm_update<T>), dim3(nb), dim3(256), 0, st, dc);
        if ((e = launch_iteration_phase<T>(L, 4, st)) != hipSuccess) return e;   // projection, duals, TV, partials
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return k > 0 ? launch_iteration_phase<T>(L, kNumPhases - 1, st) : hipSuccess;
}

template <class T>
hipError_t launch_backproject_plain(const DevCtx<T>& hc, const DevCtx<T>* dc, int variant, const T* y_padded,
                                    T* out, hipStream_t st) {
    if (variant == 4)
        hipLaunchKernelGGL((k_backproject_fan<T, false>), dim3(bp_blocks(hc.N, 4)), dim3(kBpWaves * 64), 0, st, dc,
                           (const Slot*)nullptr, y_padded, out, 0);
    else if (variant == 3)
        hipLaunchKernelGGL((k_backproject_quad<T, false>), dim3(bp_blocks(hc.N, 3)), dim3(kBpQuadWaves * 64), 0, st,
                           dc, (const Slot*)nullptr, y_padded, out, 0);
    else if (variant == 1)
        hipLaunchKernelGGL((k_backproject_lds<T, false>), dim3(bp_blocks(hc.N, 1)), dim3(kBpQuadWaves * 64), 0, st, dc,
                           (const Slot*)nullptr, y_padded, out, 0);
    else
        hipLaunchKernelGGL((k_backproject_direct<T, false>), dim3(bp_blocks(hc.N, 2)), dim3(kBpWaves * 64), 0, st,
                           dc, (const Slot*)nullptr, y_padded, out, 0);
    return hipGetLastError();
}

template <class T>
hipError_t launch_fbp(const DevCtx<T>& hc, const DevCtx<T>* dc, int backprojector, const T* y, T* out,
                      hipStream_t st) {
    if (hc.NS > kFbpMaxBins) return hipErrorInvalidValue;
    const size_t sm = 2 * (size_t)hc.NS * sizeof(T);
    hipLaunchKernelGGL((k_fbp_filter<T>), dim3(hc.NA), dim3(256), sm, st, dc, y, hc.ysc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_backproject_plain<T>(hc, dc, backprojector, hc.ysc, out, st);
}

template <class T>
hipError_t launch_apply_minv(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* w, T* out, T scale,
                             hipStream_t st) {
    const size_t sm = fft_lds<T>(hc.N);
    hipLaunchKernelGGL((k_fft_rows_fwd<T, false>), dim3(hc.N / 2), dim3(kFftThreads), sm, st, dc, (const Slot*)nullptr,
                       w);
    hipLaunchKernelGGL((k_fft_cols<T, false>), dim3(hc.N / 2 + 1), dim3(kFftThreads), sm, st, dc,
                       (const Slot*)nullptr, scale);
    hipLaunchKernelGGL((k_fft_rows_inv<T, false>), dim3(hc.N / 2), dim3(kFftThreads), sm, st, dc, (const Slot*)nullptr, out);
    return hipGetLastError();
}

hipError_t launch_parallel_tables(const DevCtx<float>& hc, DevCtx<float>* dst, AngleT<float>* ang, double* ang64,
                                  int32_t* axis, hipStream_t st) {
    hipLaunchKernelGGL(k_parallel_tables, dim3(blocks_for((size_t)hc.NA)), dim3(256), 0, st, hc, dst, ang, ang64, axis);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pad_image_full(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* img, hipStream_t st) {
    hipLaunchKernelGGL((k_pad_image_full<T>), dim3(blocks_for((size_t)hc.N * hc.P)), dim3(256), 0, st, dc, img);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pad_image(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* img, hipStream_t st) {
    hipLaunchKernelGGL((k_pad_image<T>), dim3(tv_blocks(hc.N)), dim3(256), 0, st, dc, img);
    return hipGetLastError();
}

template <class T>
hipError_t launch_project_plain(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, T* out, hipStream_t st) {
    return launch_project<T, PMODE_PLAIN>(dc, nullptr, hc.nwg_proj, projector, out, st);
}

template <class T>
hipError_t launch_project_setp(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, hipStream_t st) {
    return launch_project<T, PMODE_SETP>(dc, nullptr, hc.nwg_proj, projector, (T*)nullptr, st);
}

// f(img): project into the scratch sinogram (unpadded view), data and TV
// partials, then reduce into ctl->eval_out.
template <class T>
hipError_t launch_eval_objective(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, const T* img,
                                 hipStream_t st) {
    const size_t m = (size_t)hc.NA * hc.NS;
    hipError_t e;
    if ((e = launch_pad_image<T>(hc, dc, img, st)) != hipSuccess) return e;
    if ((e = launch_project_plain<T>(hc, dc, projector, hc.ysc, st)) != hipSuccess) return e;
    const unsigned nd = blocks_for(m);
    hipLaunchKernelGGL((k_data_eval<T>), dim3(nd), dim3(256), 0, st, dc, (const T*)hc.ysc);
    hipLaunchKernelGGL((k_tv_eval<T>), dim3(tv_blocks(hc.N)), dim3(256), 0, st, dc, img);
    hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(256), 0, st, dc, (int)nd, tv_blocks(hc.N), 1);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pad_sinogram(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* y, T* y_padded, hipStream_t st) {
    hipLaunchKernelGGL((k_pad<T>), dim3(blocks_for((size_t)hc.NA * hc.PU)), dim3(256), 0, st, dc, y, y_padded);
    return hipGetLastError();
}

template <class T>
hipError_t launch_unpad_sinogram(const DevCtx<T>& hc, const DevCtx<T>* dc, const T* y_padded, T* y,
                                 hipStream_t st) {
    hipLaunchKernelGGL((k_unpad<T>), dim3(blocks_for((size_t)hc.NA * hc.NS)), dim3(256), 0, st, dc, y_padded, y);
    return hipGetLastError();
}

template <class T>
hipError_t launch_data_const(const DevCtx<T>& hc, const DevCtx<T>* dc, hipStream_t st) {
    const unsigned nd = blocks_for((size_t)hc.NA * hc.NS);
    hipLaunchKernelGGL((k_lgamma_part<T>), dim3(nd), dim3(256), 0, st, dc);
    hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(256), 0, st, dc, (int)nd, 0, 2);
    return hipGetLastError();
}

template <class T>
hipError_t launch_dual_init(const DevCtx<T>& hc, const DevCtx<T>* dc, hipStream_t st) {
    hipLaunchKernelGGL((k_dual_init_u<T>), dim3(blocks_for((size_t)hc.NA * hc.NS)), dim3(256), 0, st, dc);
    hipLaunchKernelGGL((k_dual_init_v<T>), dim3(tv_blocks(hc.N)), dim3(256), 0, st, dc);
    return hipGetLastError();
}

template <class T>
hipError_t launch_e1_norm(const DevCtx<T>& hc, const DevCtx<T>* dc, int projector, hipStream_t st) {
    const unsigned nd = blocks_for((size_t)hc.NA * hc.NS);
    hipLaunchKernelGGL((k_ones_image<T>), dim3(tv_blocks(hc.N)), dim3(256), 0, st, dc);
    hipError_t e;
    if ((e = launch_project_plain<T>(hc, dc, projector, hc.ysc, st)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_sumsq<T>), dim3(nd), dim3(256), 0, st, dc, (const T*)hc.ysc);
    hipLaunchKernelGGL((k_finalize<T>), dim3(1), dim3(256), 0, st, dc, (int)nd, 0, 3);
    return hipGetLastError();
}

template <class T>
hipError_t launch_step_residual(const DevCtx<T>* dc, hipStream_t st) {
    hipLaunchKernelGGL((k_step_residual<T>), dim3(1), dim3(256), 0, st, dc);
    return hipGetLastError();
}

#define NCS_INSTANTIATE(T)                                                                                        \
    template hipError_t launch_iterations<T>(const IterLaunch<T>&, int, hipStream_t);                            \
    template hipError_t launch_bp_iter<T>(const IterLaunch<T>&, int, hipStream_t);                                \
    template hipError_t launch_admm_iterations<T>(const IterLaunch<T>&, const DevCtx<T>&, int, int, int, hipStream_t); \
    template hipError_t launch_iteration_phase<T>(const IterLaunch<T>&, int, hipStream_t);                       \
    template hipError_t launch_backproject_plain<T>(const DevCtx<T>&, const DevCtx<T>*, int, const T*, T*, hipStream_t); \
    template hipError_t launch_apply_minv<T>(const DevCtx<T>&, const DevCtx<T>*, const T*, T*, T, hipStream_t);  \
    template hipError_t launch_fbp<T>(const DevCtx<T>&, const DevCtx<T>*, int, const T*, T*, hipStream_t);       \
    template hipError_t launch_pad_image<T>(const DevCtx<T>&, const DevCtx<T>*, const T*, hipStream_t);          \
    template hipError_t launch_pad_image_full<T>(const DevCtx<T>&, const DevCtx<T>*, const T*, hipStream_t);     \
    template hipError_t launch_project_plain<T>(const DevCtx<T>&, const DevCtx<T>*, int, T*, hipStream_t);       \
    template hipError_t launch_project_setp<T>(const DevCtx<T>&, const DevCtx<T>*, int, hipStream_t);            \
    template hipError_t launch_eval_objective<T>(const DevCtx<T>&, const DevCtx<T>*, int, const T*, hipStream_t); \
    template hipError_t launch_pad_sinogram<T>(const DevCtx<T>&, const DevCtx<T>*, const T*, T*, hipStream_t);   \
    template hipError_t launch_unpad_sinogram<T>(const DevCtx<T>&, const DevCtx<T>*, const T*, T*, hipStream_t); \
    template hipError_t launch_data_const<T>(const DevCtx<T>&, const DevCtx<T>*, hipStream_t);                   \
    template hipError_t launch_dual_init<T>(const DevCtx<T>&, const DevCtx<T>*, hipStream_t);                   \
    template hipError_t launch_e1_norm<T>(const DevCtx<T>&, const DevCtx<T>*, int, hipStream_t);                 \
    template hipError_t launch_step_residual<T>(const DevCtx<T>*, hipStream_t);

NCS_INSTANTIATE(float)
NCS_INSTANTIATE(double)

}  // namespace ncs
