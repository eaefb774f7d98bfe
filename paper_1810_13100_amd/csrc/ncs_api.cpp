// Host side of the NCS C ABI: argument checking, double-precision setup of the
// per-angle table, the Fourier multiplier and the twiddles, workspace
// ownership, and the iteration driver (direct launches or a replayed HIP
// graph of a chunk of iterations, with the stopping test on the device), for
// one slice or for a batch of uneven slices sharing every launch.
#include "ncs.h"
#include "ncs_internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <limits>
#include <vector>

using namespace ncs;

namespace {

thread_local std::string g_err;

void set_err(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}

}  // namespace

// Error message for ncs_last_error(), shared with the network's host code.
void ncs::set_error_message(const char* msg) { g_err = msg; }

namespace {

#define NCS_HIP(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            set_err("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);     \
            return NCS_ERR_HIP;                                                                     \
        }                                                                                           \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr uint64_t kStateMagic = 0x3130303331303831ull;  // blob tag
constexpr int kXcds = 8;                                 // XCDs of an MI355X (round-robin dispatch)
constexpr int kGraphLevels = 8;                          // replayed chunks of 1, 2, 4, ..., 128 iterations

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

}  // namespace

struct ncs_handle {
    ncs_geometry g{};
    ncs_params p{};
    int dtype = NCS_F32;
    size_t esz = 4;
    hipStream_t stream = nullptr;
    int device = 0;
    int log2N = 0, PU = 0;
    size_t n = 0, m = 0, mp = 0;

    // device workspace (library-owned)
    void* x = nullptr;
    void* xbar = nullptr;
    void* xbarT = nullptr;
    void* xsc = nullptr;
    void* xscT = nullptr;
    void* u = nullptr;
    void* pj = nullptr;
    void* v = nullptr;
    void* w = nullptr;
    void* spec = nullptr;
    void* hh = nullptr;
    void* tw = nullptr;
    void* ang = nullptr;
    double* ang64 = nullptr;   // k1, k2, k0, q1, q2, q0 per angle in double
    int32_t* axis = nullptr;
    void* ysc = nullptr;
    double* part_data = nullptr;
    double* part_tv = nullptr;
    Control* ctl = nullptr;     // owned, or an element of a batch's control array
    double* hist = nullptr;
    void* dctx = nullptr;       // device copy of this slice's DevCtx<T>
    // ADMM with CG inner solves (method NCS_METHOD_ADMM_CG) only
    void* cg_vec = nullptr;     // d, r, z, p, q: 5 N*N vectors
    void* cg_y = nullptr;       // unpadded sinogram scratch
    double* cg_part = nullptr;  // dot-product partials
    double* cg_s = nullptr;     // CG scalars
    void* tpos = nullptr;       // positivity dual t (params.positivity only)
    // fan beam: per-ray and per-view tables (typed), the fan angles and the
    // half-width in bins of the rays that can touch a pixel
    void* rays = nullptr;
    void* views = nullptr;
    double gamma0 = 0.0, dgamma = 0.0;
    int fan_w = 0;
    std::vector<double> fan_tab;   // per ray: k0, k2, kappa, axis (double)

    const void* b = nullptr;    // caller-owned
    const void* bg = nullptr;   // caller-owned

    std::vector<double> tab;    // per-angle table (double)
    std::vector<double> mu;     // eigenvalues of M, N x N, numpy FFT order
    double c_r = 0.0, mu_dc = 0.0, norm_e1_sq = 0.0;
    int64_t nnz = -1;           // counted on request
    int projector = 2;
    double projector_ms[3] = {0.0, 0.0, 0.0};
    int backprojector = 2;
    double backprojector_ms[3] = {0.0, 0.0, 0.0};
    int32_t* aorder = nullptr;            // angles by stepping axis (single parallel-beam slices)
    int nar = 0;                          // row-stepping angles
    int graph_chunk = 32;                 // largest replayed chunk; <= 0: no graphs
    hipStream_t cap_stream = nullptr;     // private stream used only for graph capture
    int graph_levels = 0;                 // graphs[l] holds 2^l iterations, l < graph_levels
    hipGraphExec_t graphs[kGraphLevels] = {};
    int iter_host = 0;                    // iteration count as last seen by the host
    std::vector<void*> allocs;
};

struct ncs_batch {
    int n = 0;
    int dtype = NCS_F32;
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<ncs_handle*> slices;
    Control* ctls = nullptr;      // device array, one per slice
    void* dctxs = nullptr;        // device array of DevCtx<T>
    Slot* maps[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // bp, rows, cols, proj, fin
    size_t map_cap[5] = {0, 0, 0, 0, 0};
    int blocks[5] = {0, 0, 0, 0, 0};
    std::vector<int> xcd_of;      // slice -> XCD it is pinned to
    std::vector<char> active;
    std::vector<char> mapped;     // the active flags the maps were built from
    int max_N = 0;
    int projector = 2;
    int backprojector = 2;
    int check_every = 50;
    // the iterations between two host checks replayed as one captured graph,
    // one per chunk length (two kept); dropped whenever the maps are rebuilt
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    int graph_k[2] = {0, 0};
    hipGraphExec_t graph[2] = {nullptr, nullptr};
};

namespace {

template <class T>
DevCtx<T> make_ctx(const ncs_handle* h) {
    DevCtx<T> c{};
    c.N = h->g.n_side;
    c.log2N = h->log2N;
    c.NA = h->g.n_angles;
    c.NS = h->g.n_bins;
    c.PU = h->PU;
    c.P = h->g.n_side + 2 * kPadL;
    c.nb_proj = project_blocks(c.NA, c.NS);
    c.aorder = h->aorder;
    c.nar = h->nar;
    c.nwg_proj = h->aorder ? project_wgs_split(c.NA, c.NS, h->nar) : c.nb_proj;
    c.nb_tv = tv_blocks(c.N);
    c.ang = static_cast<const AngleT<T>*>(h->ang);
    c.ang64 = h->ang64;
    c.axis = h->axis;
    c.x = static_cast<T*>(h->x);
    c.xbar = static_cast<T*>(h->xbar);
    c.xbarT = static_cast<T*>(h->xbarT);
    c.xsc = static_cast<T*>(h->xsc);
    c.xscT = static_cast<T*>(h->xscT);
    c.u = static_cast<T*>(h->u);
    c.p = static_cast<T*>(h->pj);
    c.v = static_cast<T*>(h->v);
    c.w = static_cast<T*>(h->w);
    c.spec = static_cast<T*>(h->spec);
    c.hh = static_cast<const T*>(h->hh);
    c.tw = static_cast<const T*>(h->tw);
    c.b = static_cast<const T*>(h->b);
    c.bg = static_cast<const T*>(h->bg);
    c.ysc = static_cast<T*>(h->ysc);
    c.part_data = h->part_data;
    c.part_tv = h->part_tv;
    c.ctl = h->ctl;
    c.hist = h->hist;
    if (h->cg_vec) {
        T* v = static_cast<T*>(h->cg_vec);
        c.cg_d = v;
        c.cg_r = v + h->n;
        c.cg_z = v + 2 * h->n;
        c.cg_p = v + 3 * h->n;
        c.cg_q = v + 4 * h->n;
        c.cg_y = static_cast<T*>(h->cg_y);
        c.cg_part = h->cg_part;
        c.cg_s = h->cg_s;
    }
    c.tpos = static_cast<T*>(h->tpos);
    c.rays = static_cast<const RayT<T>*>(h->rays);
    c.views = static_cast<const ViewT<T>*>(h->views);
    c.gamma0 = (T)h->gamma0;
    c.dgamma = (T)h->dgamma;
    c.beam = h->g.beam;
    c.fan_w = h->fan_w;
    c.alpha = (T)h->p.alpha;
    c.beta = (T)h->p.beta;
    c.s_tv = (T)(h->p.lambda * h->p.alpha / h->p.beta);
    c.dual_ramp = (T)(h->p.dual_ramp > 0.0 ? h->p.dual_ramp : 0.0);
    c.inv1pa = (T)(1.0 / (1.0 + h->p.alpha));
    c.lambda = h->p.lambda;
    c.data_term = h->p.data_term;
    c.tv_term = h->p.tv_term;
    return c;
}

template <class T>
const DevCtx<T>* dctx(const ncs_handle* h) {
    return static_cast<const DevCtx<T>*>(h->dctx);
}

template <class T>
IterLaunch<T> single_launch(const ncs_handle* h) {
    IterLaunch<T> L{};
    const int N = h->g.n_side;
    L.ctxs = dctx<T>(h);
    L.bp = {nullptr, bp_blocks(N, h->backprojector)};
    L.rows = {nullptr, N / 2};
    L.cols = {nullptr, N / 2 + 1};
    L.proj = {nullptr, (h->aorder ? project_wgs_split(h->g.n_angles, h->g.n_bins, h->nar)
                                  : project_blocks(h->g.n_angles, h->g.n_bins)) + tv_blocks(N)};
    L.fin = {nullptr, 1};
    L.max_N = N;
    L.projector = h->projector;
    L.backprojector = h->backprojector;
    return L;
}

ncs_status dev_alloc(ncs_handle* h, void** ptr, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        set_err("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? NCS_ERR_OOM : NCS_ERR_HIP;
    }
    h->allocs.push_back(*ptr);
    return NCS_OK;
}

// nnz(E) in double on the host from the same geometry as the kernels: for
// each ray and step, the taps floor(xi) and floor(xi) + 1 with weights 1 - f
// and f, kept when inside [0, N-1] and nonzero.
int64_t count_nnz(const ncs_geometry& g, const std::vector<double>& tab) {
    const int N = g.n_side;
    int64_t taps = 0;
    for (int a = 0; a < g.n_angles; ++a) {
        const double* t = &tab[10 * (size_t)a];
        const double k1 = t[0], k2 = t[1], k0 = t[2];
        for (int d = 0; d < g.n_bins; ++d) {
            const double base = d * k1 + k0;
            for (int st = 0; st < N; ++st) {
                const double xi = st * k2 + base;
                if (xi <= -1.0 || xi >= (double)N) continue;
                const double fl = std::floor(xi);
                const double f = xi - fl;
                const int c0 = (int)fl;
                if (c0 >= 0) ++taps;
                if (c0 + 1 <= N - 1 && f != 0.0) ++taps;
            }
        }
    }
    return taps;
}

// ---- fan beam ----------------------------------------------------------------
// Per ray (a*N_s + d) the stepping axis and the affine coordinate of the
// other axis along it (Joseph), from the source position and direction in
// double: rows are stepped when |u_y| >= |u_x| - 1e-12.  Per view the source
// and the direction of the central ray.  w bins on either side of a pixel's
// bin hold every ray that passes within one pixel of its centre.
void build_fan_tables(ncs_handle* h, std::vector<double>& views) {
    const ncs_geometry& g = h->g;
    const int N = g.n_side, NA = g.n_angles, NS = g.n_bins;
    const double half = 0.5 * (N - 1), rs = g.source_radius, r_fov = N / std::sqrt(2.0);
    h->dgamma = 2.0 * std::asin(r_fov / rs) / (NS - 1);
    h->gamma0 = -0.5 * (NS - 1) * h->dgamma;
    h->fan_w = (int)std::ceil(std::asin(1.0 / (rs - r_fov)) / h->dgamma + 0.5) + 1;
    h->fan_tab.assign(4 * (size_t)NA * NS, 0.0);
    views.assign(4 * (size_t)NA, 0.0);
    for (int a = 0; a < NA; ++a) {
        const double beta = 2.0 * kPi * a / NA;
        const double sx = rs * std::cos(beta), sy = rs * std::sin(beta), thc = beta + kPi;
        views[4 * (size_t)a] = sx;
        views[4 * (size_t)a + 1] = sy;
        views[4 * (size_t)a + 2] = thc;
        for (int d = 0; d < NS; ++d) {
            const double th = thc + (d - 0.5 * (NS - 1)) * h->dgamma;
            const double ux = std::cos(th), uy = std::sin(th);
            double* t = &h->fan_tab[4 * ((size_t)a * NS + d)];
            if (std::fabs(uy) >= std::fabs(ux) - 1e-12) {   // rows: column coordinate at row r
                const double k2 = ux / uy;
                t[0] = sx - (half + sy) * k2 + half;
                t[1] = k2;
                t[2] = 1.0 / std::fabs(uy);
                t[3] = 0.0;
            } else {                                         // columns: row coordinate at column c
                const double k2 = uy / ux;
                t[0] = sy - (half + sx) * k2 + half;
                t[1] = k2;
                t[2] = 1.0 / std::fabs(ux);
                t[3] = 1.0;
            }
        }
    }
}

template <class T>
ncs_status upload_fan(ncs_handle* h, const std::vector<double>& views) {
    const size_t m = h->fan_tab.size() / 4, na = views.size() / 4;
    std::vector<RayT<T>> r(m);
    for (size_t i = 0; i < m; ++i)
        r[i] = RayT<T>{(T)h->fan_tab[4 * i], (T)h->fan_tab[4 * i + 1], (T)h->fan_tab[4 * i + 2],
                       (int32_t)h->fan_tab[4 * i + 3]};
    std::vector<ViewT<T>> v(na);
    for (size_t i = 0; i < na; ++i) v[i] = ViewT<T>{(T)views[4 * i], (T)views[4 * i + 1], (T)views[4 * i + 2], T(0)};
    NCS_HIP(hipMemcpy(h->rays, r.data(), m * sizeof(RayT<T>), hipMemcpyHostToDevice));
    NCS_HIP(hipMemcpy(h->views, v.data(), na * sizeof(ViewT<T>), hipMemcpyHostToDevice));
    return NCS_OK;
}

int64_t count_nnz_fan(const ncs_handle* h) {
    const int N = h->g.n_side;
    int64_t taps = 0;
    for (size_t i = 0; i < h->fan_tab.size() / 4; ++i) {
        const double k0 = h->fan_tab[4 * i], k2 = h->fan_tab[4 * i + 1];
        for (int st = 0; st < N; ++st) {
            const double xi = st * k2 + k0;
            if (xi <= -1.0 || xi >= (double)N) continue;
            const double fl = std::floor(xi);
            const double f = xi - fl;
            const int c0 = (int)fl;
            if (c0 >= 0) ++taps;
            if (c0 + 1 <= N - 1 && f != 0.0) ++taps;
        }
    }
    return taps;
}

// ---- eq. H-fan: the multiplier of E^T E estimated from probes --------------
// Probe k: n values +-1, entry 64 j + b = bit b of the j-th output of
// SplitMix64 (Steele, Lea and Flood) started from state k.
void rademacher_probe(uint64_t index, size_t n, std::vector<double>& v) {
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

// In-place radix-2 DFT with the forward sign, sum_t a_t exp(-2 pi i f t / n).
void dft_pow2(std::complex<double>* a, int n) {
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * kPi / len;
        for (int i = 0; i < n; i += len)
            for (int k = 0; k < len / 2; ++k) {
                const std::complex<double> w(std::cos(ang * k), std::sin(ang * k));
                const std::complex<double> u = a[i + k], t = w * a[i + k + len / 2];
                a[i + k] = u + t;
                a[i + k + len / 2] = u - t;
            }
    }
}

// 2D DFT of an N x N real image (row-major), the numpy fft2 convention.
void dft2_real(const std::vector<double>& img, int N, std::vector<std::complex<double>>& out) {
    out.assign((size_t)N * N, 0.0);
    for (size_t i = 0; i < out.size(); ++i) out[i] = img[i];
    for (int r = 0; r < N; ++r) dft_pow2(&out[(size_t)r * N], N);
    std::vector<std::complex<double>> col(N);
    for (int c = 0; c < N; ++c) {
        for (int r = 0; r < N; ++r) col[r] = out[(size_t)r * N + c];
        dft_pow2(col.data(), N);
        for (int r = 0; r < N; ++r) out[(size_t)r * N + c] = col[r];
    }
}

// he = Re( sum_v conj(F v) F(E^T E v) / sum_v |F v|^2 ) over the probes, with
// E^T E v from the handle's own projector and backprojector.
template <class T>
ncs_status estimate_normal_multiplier(ncs_handle* h, int probes, std::vector<double>& he) {
    const int N = h->g.n_side;
    const size_t n = h->n, m = h->m;
    T *v = nullptr, *y = nullptr, *z = nullptr;
    ncs_status s;
    if ((s = dev_alloc(h, reinterpret_cast<void**>(&v), n * sizeof(T))) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&y), m * sizeof(T))) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&z), n * sizeof(T))))
        return s;
    const DevCtx<T> c = make_ctx<T>(h);
    std::vector<double> vd, zd(n);
    std::vector<T> vt(n), zt(n);
    std::vector<std::complex<double>> fv, fz, num(n, 0.0);
    std::vector<double> den(n, 0.0);
    for (int k = 0; k < probes; ++k) {
        rademacher_probe((uint64_t)k, n, vd);
        for (size_t i = 0; i < n; ++i) vt[i] = (T)vd[i];
        NCS_HIP(hipMemcpyAsync(v, vt.data(), n * sizeof(T), hipMemcpyHostToDevice, h->stream));
        NCS_HIP(launch_pad_image<T>(c, dctx<T>(h), v, h->stream));
        NCS_HIP(launch_project_plain<T>(c, dctx<T>(h), h->projector, y, h->stream));
        NCS_HIP(launch_pad_sinogram<T>(c, dctx<T>(h), y, c.ysc, h->stream));
        NCS_HIP(launch_backproject_plain<T>(c, dctx<T>(h), h->backprojector, c.ysc, z, h->stream));
        NCS_HIP(hipMemcpyAsync(zt.data(), z, n * sizeof(T), hipMemcpyDeviceToHost, h->stream));
        NCS_HIP(hipStreamSynchronize(h->stream));
        for (size_t i = 0; i < n; ++i) zd[i] = (double)zt[i];
        dft2_real(vd, N, fv);
        dft2_real(zd, N, fz);
        for (size_t i = 0; i < n; ++i) {
            num[i] += std::conj(fv[i]) * fz[i];
            den[i] += std::norm(fv[i]);
        }
    }
    he.assign(n, 0.0);
    for (size_t i = 0; i < n; ++i) he[i] = den[i] > 0.0 ? std::real(num[i] / den[i]) : 0.0;
    return NCS_OK;
}

template <class T>
ncs_status upload(void* dst, const std::vector<double>& src) {
    std::vector<T> tmp(src.size());
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
    NCS_HIP(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
    return NCS_OK;
}

ncs_status upload_typed(const ncs_handle* h, void* dst, const std::vector<double>& src) {
    return h->dtype == NCS_F64 ? upload<double>(dst, src) : upload<float>(dst, src);
}

template <class T>
ncs_status upload_ctx(ncs_handle* h) {
    const DevCtx<T> c = make_ctx<T>(h);
    NCS_HIP(hipMemcpy(h->dctx, &c, sizeof(c), hipMemcpyHostToDevice));
    return NCS_OK;
}

ncs_status upload_ctx_typed(ncs_handle* h) {
    return h->dtype == NCS_F64 ? upload_ctx<double>(h) : upload_ctx<float>(h);
}

// ---- iteration launch -----------------------------------------------------
hipError_t launch_eager(ncs_handle* h, int k, hipStream_t st) {
    if (h->p.method == NCS_METHOD_ADMM_CG) {
        const int cg = h->p.cg_iters > 0 ? h->p.cg_iters : 10;
        return h->dtype == NCS_F64
                   ? launch_admm_iterations<double>(single_launch<double>(h), make_ctx<double>(h), k, cg,
                                                    h->p.cg_precondition, st)
                   : launch_admm_iterations<float>(single_launch<float>(h), make_ctx<float>(h), k, cg,
                                                   h->p.cg_precondition, st);
    }
    return h->dtype == NCS_F64 ? launch_iterations<double>(single_launch<double>(h), k, st)
                               : launch_iterations<float>(single_launch<float>(h), k, st);
}

hipError_t launch_phase(ncs_handle* h, int ph) {
    return h->dtype == NCS_F64 ? launch_iteration_phase<double>(single_launch<double>(h), ph, h->stream)
                               : launch_iteration_phase<float>(single_launch<float>(h), ph, h->stream);
}

// Capture one graph per power of two up to graph_chunk iterations (on a
// private stream), all at the first iteration request, and keep the
// executable graphs: any k is then replayed as the largest chunk repeated plus
// the binary digits of the remainder, at most log2(graph_chunk) + k/graph_chunk
// launches.  Any capture failure switches the handle to direct launches.
void drop_graphs(ncs_handle* h) {
    for (int l = 0; l < h->graph_levels; ++l)
        if (h->graphs[l]) (void)hipGraphExecDestroy(h->graphs[l]);
    for (auto& g : h->graphs) g = nullptr;
    h->graph_levels = 0;
}

void ensure_graphs(ncs_handle* h) {
    if (h->graph_levels > 0 || h->graph_chunk <= 0) return;
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        h->graph_chunk = 0;
        return;
    }
    int levels = 0;
    while (levels < kGraphLevels && (1 << levels) <= h->graph_chunk) ++levels;
    for (int l = 0; l < levels; ++l) {
        bool ok = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const hipError_t le = launch_eager(h, 1 << l, h->cap_stream);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(h->cap_stream, &graph);
            ok = le == hipSuccess && ee == hipSuccess && graph &&
                 hipGraphInstantiate(&h->graphs[l], graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            // move the executable graph to the device now rather than at its first launch
            if (ok) ok = hipGraphUpload(h->graphs[l], h->stream) == hipSuccess;
        }
        if (!ok) {
            (void)hipGetLastError();
            h->graphs[l] = nullptr;
            h->graph_levels = l;
            drop_graphs(h);
            h->graph_chunk = 0;
            return;
        }
        h->graph_levels = l + 1;
    }
    // One dry replay of every graph with the stop flag raised (each kernel
    // returns before touching the state): a graph's first launch costs
    // extra, and it should not fall inside a caller's timed or latency-bound
    // call.  Called from launch_iters right after the control block was reset
    // for the request, so clearing the flag restores it.
    bool primed = launch_control(h->ctl, 3, 0, 0.0, h->stream) == hipSuccess;
    for (int l = 0; primed && l < h->graph_levels; ++l) primed = hipGraphLaunch(h->graphs[l], h->stream) == hipSuccess;
    if (launch_control(h->ctl, 4, 0, 0.0, h->stream) != hipSuccess || !primed) {
        (void)hipGetLastError();
        drop_graphs(h);
        h->graph_chunk = 0;
    }
}

hipError_t launch_iters(ncs_handle* h, int k) {
    if (h->graph_chunk > 0 && k > 0) {
        ensure_graphs(h);
        if (h->graph_levels > 0) {
            const int top = h->graph_levels - 1;
            for (; k >= (1 << top); k -= 1 << top) {
                const hipError_t e = hipGraphLaunch(h->graphs[top], h->stream);
                if (e != hipSuccess) return e;
            }
            for (int l = top - 1; l >= 0; --l) {
                if (!(k & (1 << l))) continue;
                const hipError_t e = hipGraphLaunch(h->graphs[l], h->stream);
                if (e != hipSuccess) return e;
                k -= 1 << l;
            }
        }
    }
    return k > 0 ? launch_eager(h, k, h->stream) : hipSuccess;
}

// Forward-projector selection: time both variants on this geometry (plain
// projections of the scratch image) and keep the faster.
template <class T>
ncs_status autotune_projector(ncs_handle* h) {
    hipEvent_t e0, e1;
    NCS_HIP(hipEventCreate(&e0));
    NCS_HIP(hipEventCreate(&e1));
    const DevCtx<T> c = make_ctx<T>(h);
    T* out = static_cast<T*>(h->ysc);
    const int reps = 5;
    for (int variant = 1; variant <= 3; ++variant) {
        NCS_HIP(launch_project_plain<T>(c, dctx<T>(h), variant, out, h->stream));   // warm-up
        NCS_HIP(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) NCS_HIP(launch_project_plain<T>(c, dctx<T>(h), variant, out, h->stream));
        NCS_HIP(hipEventRecord(e1, h->stream));
        NCS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        NCS_HIP(hipEventElapsedTime(&ms, e0, e1));
        h->projector_ms[variant - 1] = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int best = 1;
    for (int v = 2; v <= 3; ++v)
        if (h->projector_ms[v - 1] < h->projector_ms[best - 1]) best = v;
    h->projector = best;
    return NCS_OK;
}

// Backprojector selection: time every variant on this geometry (plain
// backprojections of the scratch sinogram) and keep the fastest.
template <class T>
ncs_status autotune_backprojector(ncs_handle* h) {
    hipEvent_t e0, e1;
    NCS_HIP(hipEventCreate(&e0));
    NCS_HIP(hipEventCreate(&e1));
    const DevCtx<T> c = make_ctx<T>(h);
    const T* src = static_cast<const T*>(h->ysc);
    T* out = static_cast<T*>(h->w);
    const int reps = 5;
    for (int variant = 1; variant <= kNumBackprojectors; ++variant) {
        NCS_HIP(launch_backproject_plain<T>(c, dctx<T>(h), variant, src, out, h->stream));   // warm-up
        NCS_HIP(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) NCS_HIP(launch_backproject_plain<T>(c, dctx<T>(h), variant, src, out, h->stream));
        NCS_HIP(hipEventRecord(e1, h->stream));
        NCS_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        NCS_HIP(hipEventElapsedTime(&ms, e0, e1));
        h->backprojector_ms[variant - 1] = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int best = 1;
    for (int v = 2; v <= kNumBackprojectors; ++v)
        if (h->backprojector_ms[v - 1] < h->backprojector_ms[best - 1]) best = v;
    h->backprojector = best;
    return NCS_OK;
}

ncs_status read_control(ncs_handle* h, Control* out) {
    NCS_HIP(hipMemcpyAsync(out, h->ctl, sizeof(Control), hipMemcpyDeviceToHost, h->stream));
    NCS_HIP(hipStreamSynchronize(h->stream));
    h->iter_host = out->iter;
    return NCS_OK;
}

ncs_status check_handle(ncs_handle* h) {
    if (!h) {
        set_err("null handle");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(hipSetDevice(h->device));
    return NCS_OK;
}

ncs_status validate(const ncs_geometry& g, const ncs_params& p, int32_t dtype) {
    if (!is_pow2(g.n_side) || g.n_side < 16 || g.n_side > 1024) {
        set_err("n_side must be a power of two in [16, 1024] (got %d)", g.n_side);
        return NCS_ERR_INVALID_ARG;
    }
    if (g.n_angles < 1 || g.n_angles > (1 << 20) || g.n_bins < 2 || g.n_bins > (1 << 20)) {
        set_err("need 1 <= n_angles and 2 <= n_bins (got %d, %d)", g.n_angles, g.n_bins);
        return NCS_ERR_INVALID_ARG;
    }
    if (dtype != NCS_F32 && dtype != NCS_F64) {
        set_err("dtype must be NCS_F32 or NCS_F64");
        return NCS_ERR_INVALID_ARG;
    }
    if (g.beam != NCS_BEAM_PARALLEL && g.beam != NCS_BEAM_FAN) {
        set_err("beam must be NCS_BEAM_PARALLEL (0) or NCS_BEAM_FAN (1)");
        return NCS_ERR_INVALID_ARG;
    }
    if (g.beam == NCS_BEAM_FAN && !(std::isfinite(g.source_radius) && g.source_radius > 1.01 * g.n_side / std::sqrt(2.0))) {
        set_err("a fan beam needs a finite source_radius > 1.01 n_side / sqrt(2)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.probes < 0 || p.probes > 4096) {
        set_err("probes must be in [0, 4096]");
        return NCS_ERR_INVALID_ARG;
    }
    if (!(p.alpha > 0.0) || !(p.beta > 0.0) || !(p.gamma >= 0.0) || !(p.lambda >= 0.0) ||
        !std::isfinite(p.alpha) || !std::isfinite(p.beta) || !std::isfinite(p.gamma) ||
        !std::isfinite(p.lambda) || !std::isfinite(p.c_r) || !std::isfinite(p.mu_dc) || !std::isfinite(p.dual_ramp)) {
        set_err("need finite alpha > 0, beta > 0, gamma >= 0, lambda >= 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.data_term != NCS_DATA_QUADRATIC && p.data_term != NCS_DATA_POISSON) {
        set_err("unknown data_term %d", p.data_term);
        return NCS_ERR_INVALID_ARG;
    }
    if (p.tv_term != NCS_TV_ANISO && p.tv_term != NCS_TV_ISO) {
        set_err("unknown tv_term %d", p.tv_term);
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method != NCS_METHOD_NCS && p.method != NCS_METHOD_PDHG && p.method != NCS_METHOD_ADMM_CG) {
        set_err("method must be NCS_METHOD_NCS (0), NCS_METHOD_PDHG (1) or NCS_METHOD_ADMM_CG (2)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method == NCS_METHOD_ADMM_CG && (p.cg_iters < 0 || p.cg_iters > 1000 || p.cg_precondition < 0 ||
                                           p.cg_precondition > 1)) {
        set_err("ADMM-CG needs 0 <= cg_iters <= 1000 (0 selects 10) and cg_precondition 0 or 1");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method == NCS_METHOD_ADMM_CG && p.cg_precondition == 0 && dtype == NCS_F32) {
        // unpreconditioned CG amplifies FP32 rounding by about the condition
        // number of A^T A; its single-precision trajectories leave the FP64
        // method by more than 1e-4, so only double precision runs it
        set_err("ADMM-CG without the preconditioner runs in double precision only (NCS_F64)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.positivity != 0 && p.positivity != 1) {
        set_err("positivity must be 0 or 1");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.positivity && p.method == NCS_METHOD_ADMM_CG) {
        set_err("the positivity constraint runs with NCS or PDHG, not ADMM-CG");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.method == NCS_METHOD_PDHG && !(p.gamma > 0.0)) {
        set_err("PDHG needs gamma > 0 (the step is 1/gamma)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.backprojector < 0 || p.backprojector > kNumBackprojectors) {
        set_err("backprojector must be 0 (auto), 1 (LDS), 2 (direct) or 3 (quad)");
        return NCS_ERR_INVALID_ARG;
    }
    if (p.projector < 0 || p.projector > 3) {
        set_err("projector must be 0 (auto), 1 (LDS), 2 (direct) or 3 (ray pairs)");
        return NCS_ERR_INVALID_ARG;
    }
    if (g.beam == NCS_BEAM_FAN && (p.projector != 0 || p.backprojector != 0)) {
        set_err("a fan beam has one projector pair; leave projector and backprojector at 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (g.beam == NCS_BEAM_FAN && p.method == NCS_METHOD_ADMM_CG) {
        set_err("fan beams run NCS or PDHG, not ADMM-CG");
        return NCS_ERR_INVALID_ARG;
    }
    return NCS_OK;
}

// One slice: tables, workspace, multiplier.  ext_ctl (nullable) is a control
// block owned by a batch; autotune = time the projector variants.
// Per-angle geometry of a parallel beam in double (the AngleT fields in
// order: k1, k2, k0, q1, q2, q0, kappa, kappa^2, kappa - kappa^2, 1 - kappa)
// and each angle's stepping axis (0: rows).  Section 4.1.1 leaves the
// discretisation open; this is the Joseph reading with the integer 45-degree
// test.
void angle_table(const ncs_geometry& g, std::vector<double>& tab, std::vector<int>& axis) {
    const int N = g.n_side, NA = g.n_angles, NS = g.n_bins;
    tab.assign(10 * (size_t)NA, 0.0);
    axis.assign(NA, 0);
    const double hn = 0.5 * (N - 1), hs = 0.5 * (NS - 1);
    for (int a = 0; a < NA; ++a) {
        const double th = kPi * a / NA;
        const double ct = std::cos(th), st = std::sin(th);
        const bool rows = (4 * (long long)a <= NA) || (4 * (long long)a >= 3 * (long long)NA);
        axis[a] = rows ? 0 : 1;
        double* t = &tab[10 * (size_t)a];
        if (rows) {   // xi = column of ray d on row r
            t[0] = 1.0 / ct;
            t[1] = -st / ct;
            t[2] = -hs / ct + hn * st / ct + hn;
            t[6] = 1.0 / std::fabs(ct);
        } else {      // eta = row of ray d on column c
            t[0] = 1.0 / st;
            t[1] = -ct / st;
            t[2] = -hs / st + hn * ct / st + hn;
            t[6] = 1.0 / std::fabs(st);
        }
        t[3] = ct;
        t[4] = st;
        t[5] = hs - hn * (ct + st);
        t[7] = t[6] * t[6];
        t[8] = t[6] - t[7];
        t[9] = 1.0 - t[6];
    }
}

ncs_status setup_slice(const ncs_geometry& g, const ncs_params& p, int32_t dtype, const void* b_dev,
                       const void* bg_dev, hipStream_t stream, Control* ext_ctl, bool autotune,
                       ncs_handle** out, bool operators_only = false);

// eq. H-fan for a handle of either precision: the probes always go through
// double-precision kernels, so that a single-precision handle runs the same M
// as a double-precision one.  A single-precision handle borrows a
// double-precision twin (same geometry, no data, no multiplier) for this.
ncs_status estimate_multiplier_fp64(ncs_handle* h, int probes, std::vector<double>& he) {
    if (h->dtype == NCS_F64) return estimate_normal_multiplier<double>(h, probes, he);
    ncs_params q = h->p;
    q.mu_dc = 1.0;   // the twin evaluates no |E 1|^2
    ncs_handle* twin = nullptr;
    ncs_status s = setup_slice(h->g, q, NCS_F64, nullptr, nullptr, h->stream, nullptr, false, &twin, true);
    if (s) return s;
    s = estimate_normal_multiplier<double>(twin, probes, he);
    ncs_destroy(twin);
    return s;
}

ncs_status setup_slice(const ncs_geometry& g, const ncs_params& p, int32_t dtype, const void* b_dev,
                       const void* bg_dev, hipStream_t stream, Control* ext_ctl, bool autotune,
                       ncs_handle** out, bool operators_only) {
    ncs_handle* h = new ncs_handle();
    h->g = g;
    h->p = p;
    if (h->p.check_every <= 0) h->p.check_every = 50;
    h->graph_chunk = p.graph_chunk == 0 ? 32 : (p.graph_chunk < 0 ? 0 : p.graph_chunk);
    if (p.method == NCS_METHOD_ADMM_CG && h->graph_chunk > 2) h->graph_chunk = 2;   // ~15 launches per CG step
    h->projector = p.projector == 0 ? 2 : p.projector;
    h->backprojector = p.backprojector == 0 ? 2 : p.backprojector;
    if (g.beam == NCS_BEAM_FAN) h->projector = h->backprojector = 4;   // the fan pair
    h->dtype = dtype;
    h->esz = dtype == NCS_F64 ? 8 : 4;
    h->stream = stream;
    h->b = b_dev;
    h->bg = bg_dev;
    const int N = g.n_side;
    while ((1 << h->log2N) < N) ++h->log2N;
    h->PU = g.n_bins + 3;
    h->n = (size_t)N * N;
    h->m = (size_t)g.n_angles * g.n_bins;
    h->mp = (size_t)g.n_angles * h->PU;
    auto fail = [&](ncs_status s) {
        ncs_destroy(h);
        return s;
    };
    if (hipGetDevice(&h->device) != hipSuccess) {
        set_err("ncs_setup: hipGetDevice failed");
        delete h;
        return NCS_ERR_HIP;
    }

    // ---- per-angle table (double) --------------------------------------
    const int NA = g.n_angles, NS = g.n_bins;
    std::vector<int> axis;
    angle_table(g, h->tab, axis);
    // ---- workspace ---------------------------------------------------------
    const size_t e = h->esz;
    const int NH = N / 2 + 1;
    const size_t padded = (size_t)N * (N + 2 * kPadL) * e;
    const size_t nparts = std::max<size_t>({(size_t)project_blocks(NA, NS), (h->m + 255) / 256, (size_t)1});
    const size_t ctx_bytes = dtype == NCS_F64 ? sizeof(DevCtx<double>) : sizeof(DevCtx<float>);
    ncs_status s;
    if ((s = dev_alloc(h, &h->x, h->n * e)) || (s = dev_alloc(h, &h->xbar, padded)) ||
        (s = dev_alloc(h, &h->xbarT, padded)) || (s = dev_alloc(h, &h->xsc, padded)) ||
        (s = dev_alloc(h, &h->xscT, padded)) || (s = dev_alloc(h, &h->u, h->mp * e)) ||
        (s = dev_alloc(h, &h->pj, h->mp * e)) || (s = dev_alloc(h, &h->v, 2 * h->n * e)) ||
        (s = dev_alloc(h, &h->w, h->n * e)) || (s = dev_alloc(h, &h->spec, 2 * (size_t)NH * N * e)) ||
        (s = dev_alloc(h, &h->hh, (size_t)NH * N * e)) || (s = dev_alloc(h, &h->tw, (size_t)N * e)) ||
        (s = dev_alloc(h, &h->ang, 10 * (size_t)NA * e)) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&h->ang64), 6 * (size_t)NA * sizeof(double))) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&h->axis), (size_t)NA * sizeof(int32_t))) ||
        (s = dev_alloc(h, &h->ysc, h->mp * e)) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&h->part_data), nparts * sizeof(double))) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&h->part_tv), (size_t)tv_blocks(N) * sizeof(double))) ||
        (s = dev_alloc(h, reinterpret_cast<void**>(&h->hist), (size_t)kHistCap * sizeof(double))) ||
        (s = dev_alloc(h, &h->dctx, ctx_bytes)))
        return fail(s);
    if (p.method == NCS_METHOD_ADMM_CG &&
        ((s = dev_alloc(h, &h->cg_vec, 5 * h->n * e)) || (s = dev_alloc(h, &h->cg_y, h->m * e)) ||
         (s = dev_alloc(h, reinterpret_cast<void**>(&h->cg_part), (size_t)cg_blocks(N) * sizeof(double))) ||
         (s = dev_alloc(h, reinterpret_cast<void**>(&h->cg_s), 4 * sizeof(double)))))
        return fail(s);
    if (p.positivity && (s = dev_alloc(h, &h->tpos, h->n * e))) return fail(s);
    if (g.beam == NCS_BEAM_FAN) {
        std::vector<double> views;
        build_fan_tables(h, views);
        const size_t ray_bytes = dtype == NCS_F64 ? sizeof(RayT<double>) : sizeof(RayT<float>);
        const size_t view_bytes = dtype == NCS_F64 ? sizeof(ViewT<double>) : sizeof(ViewT<float>);
        if ((s = dev_alloc(h, &h->rays, (size_t)NA * NS * ray_bytes)) ||
            (s = dev_alloc(h, &h->views, (size_t)NA * view_bytes)) ||
            (s = dtype == NCS_F64 ? upload_fan<double>(h, views) : upload_fan<float>(h, views)))
            return fail(s);
    }
    // a single parallel-beam slice splits its projection blocks over the XCDs
    // by stepping axis (batches map their workgroups themselves)
    if (!ext_ctl && g.beam == NCS_BEAM_PARALLEL) {
        std::vector<int32_t> order;
        order.reserve(NA);
        for (int a = 0; a < NA; ++a)
            if (axis[a] == 0) order.push_back(a);
        h->nar = (int)order.size();
        for (int a = 0; a < NA; ++a)
            if (axis[a] != 0) order.push_back(a);
        if ((s = dev_alloc(h, reinterpret_cast<void**>(&h->aorder), (size_t)NA * sizeof(int32_t)))) return fail(s);
        if (hipMemcpy(h->aorder, order.data(), (size_t)NA * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
            set_err("ncs_setup: angle order upload failed");
            return fail(NCS_ERR_HIP);
        }
    }
    if (ext_ctl) {
        h->ctl = ext_ctl;
    } else if ((s = dev_alloc(h, reinterpret_cast<void**>(&h->ctl), sizeof(Control)))) {
        return fail(s);
    }
    if ((s = upload_typed(h, h->ang, h->tab))) return fail(s);
    {
        std::vector<double> t64(6 * (size_t)NA);
        for (int a = 0; a < NA; ++a)
            for (int k = 0; k < 6; ++k) t64[6 * (size_t)a + k] = h->tab[10 * (size_t)a + k];
        if ((s = upload<double>(h->ang64, t64))) return fail(s);
    }
    Control c0{};
    c0.f_target = std::nan("");
    if (hipMemcpy(h->axis, axis.data(), NA * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->ctl, &c0, sizeof(Control), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->x, 0, h->n * e) != hipSuccess || hipMemset(h->xbar, 0, padded) != hipSuccess ||
        hipMemset(h->xbarT, 0, padded) != hipSuccess || hipMemset(h->xsc, 0, padded) != hipSuccess ||
        hipMemset(h->xscT, 0, padded) != hipSuccess || hipMemset(h->u, 0, h->mp * e) != hipSuccess ||
        hipMemset(h->pj, 0, h->mp * e) != hipSuccess || hipMemset(h->v, 0, 2 * h->n * e) != hipSuccess ||
        hipMemset(h->ysc, 0, h->mp * e) != hipSuccess ||
        hipMemset(h->hist, 0, (size_t)kHistCap * sizeof(double)) != hipSuccess) {
        set_err("ncs_setup: workspace initialisation failed");
        return fail(NCS_ERR_HIP);
    }
    if ((s = upload_ctx_typed(h))) return fail(s);

    // ---- |E 1|^2 on the device (this handle's own projector and precision) --
    h->c_r = p.c_r > 0.0 ? p.c_r : (double)NA * N / kPi;
    if (p.mu_dc > 0.0) {
        h->mu_dc = p.mu_dc;
    } else {
        const hipError_t le =
            dtype == NCS_F64 ? launch_e1_norm<double>(make_ctx<double>(h), dctx<double>(h), h->projector, stream)
                             : launch_e1_norm<float>(make_ctx<float>(h), dctx<float>(h), h->projector, stream);
        Control cc;
        if (le != hipSuccess ||
            hipMemcpyAsync(&cc, h->ctl, sizeof(Control), hipMemcpyDeviceToHost, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess) {
            set_err("ncs_setup: |E 1|^2 evaluation failed");
            return fail(NCS_ERR_HIP);
        }
        h->norm_e1_sq = cc.eval_out;
        h->mu_dc = p.gamma + p.alpha * h->norm_e1_sq / (double)h->n;
    }

    // ---- multiplier (Section 4.1.1: eq. circ_R or eq. H-fan, eq. circ_D, DC entry)
    h->mu.assign(h->n, 0.0);
    const double bta = p.beta * p.beta / p.alpha;
    const int probes = p.probes > 0 ? p.probes : (g.beam == NCS_BEAM_FAN ? kFanProbes : 0);
    std::vector<double> he;   // eq. H-fan estimate of E^T E's multiplier (when probes > 0)
    if (operators_only) {   // a twin for estimate_multiplier_fp64: tables and workspace only
        *out = h;
        return hipStreamSynchronize(stream) == hipSuccess ? NCS_OK : fail(NCS_ERR_HIP);
    }
    if (probes > 0 && (s = estimate_multiplier_fp64(h, probes, he))) return fail(s);
    for (int j = 0; j < N; ++j) {
        const double jj = std::min(j, N - j);
        const double sj = std::sin(kPi * j / N);
        for (int k = 0; k < N; ++k) {
            const double kk = std::min(k, N - k);
            const double sk = std::sin(kPi * k / N);
            const double rad2 = jj * jj + kk * kk;
            double mu = p.gamma + bta * 4.0 * (sj * sj + sk * sk);
            if (probes > 0)
                mu += p.alpha * he[(size_t)j * N + k];
            else if (rad2 > 0.0)
                mu += p.alpha * h->c_r / std::sqrt(rad2);
            h->mu[(size_t)j * N + k] = mu;
        }
    }
    h->mu[0] = h->mu_dc;
    // x >= 0 (remark in Section 4.2): A gains the rows I, so alpha A^T A and M gain alpha I
    if (p.positivity)
        for (double& m : h->mu) m += p.alpha;
    if (p.method == NCS_METHOD_PDHG) std::fill(h->mu.begin(), h->mu.end(), p.gamma);   // M = gamma I (eq. PDHG)
    std::vector<double> hh((size_t)NH * N);
    const double scale = 1.0 / (p.alpha * (double)N * (double)N);
    for (int k = 0; k < NH; ++k)
        for (int j = 0; j < N; ++j) {
            const double mu = h->mu[(size_t)j * N + k];
            hh[(size_t)k * N + j] = mu != 0.0 ? scale / mu : 0.0;   // diag(mu)^+ (Section 2)
        }
    std::vector<double> tw(N);
    for (int k = 0; k < N / 2; ++k) {
        tw[2 * k] = std::cos(2.0 * kPi * k / N);
        tw[2 * k + 1] = -std::sin(2.0 * kPi * k / N);
    }
    if ((s = upload_typed(h, h->hh, hh)) || (s = upload_typed(h, h->tw, tw))) return fail(s);

    if (b_dev && p.data_term == NCS_DATA_POISSON) {
        const hipError_t le = dtype == NCS_F64 ? launch_data_const<double>(make_ctx<double>(h), dctx<double>(h), stream)
                                               : launch_data_const<float>(make_ctx<float>(h), dctx<float>(h), stream);
        if (le != hipSuccess) {
            set_err("ncs_setup: data constant launch failed: %s", hipGetErrorString(le));
            return fail(NCS_ERR_HIP);
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        set_err("ncs_setup: stream synchronisation failed");
        return fail(NCS_ERR_HIP);
    }
    if (autotune && p.projector == 0 && g.beam == NCS_BEAM_PARALLEL) {
        s = dtype == NCS_F64 ? autotune_projector<double>(h) : autotune_projector<float>(h);
        if (s) return fail(s);
    }
    if (autotune && p.backprojector == 0 && g.beam == NCS_BEAM_PARALLEL) {
        s = dtype == NCS_F64 ? autotune_backprojector<double>(h) : autotune_backprojector<float>(h);
        if (s) return fail(s);
    }
    *out = h;
    return NCS_OK;
}

template <class T>
ncs_status init_state(ncs_handle* h, const void* x0_dev, int32_t dual_from_x0) {
    const size_t e = h->esz;
    const DevCtx<T> c = make_ctx<T>(h);
    NCS_HIP(hipMemsetAsync(h->u, 0, h->mp * e, h->stream));
    NCS_HIP(hipMemsetAsync(h->pj, 0, h->mp * e, h->stream));
    NCS_HIP(hipMemsetAsync(h->v, 0, 2 * h->n * e, h->stream));
    if (h->tpos) NCS_HIP(hipMemsetAsync(h->tpos, 0, h->n * e, h->stream));
    if (x0_dev) {
        NCS_HIP(hipMemcpyAsync(h->x, x0_dev, h->n * e, hipMemcpyDeviceToDevice, h->stream));
        NCS_HIP(launch_pad_image<T>(c, dctx<T>(h), c.x, h->stream));
        NCS_HIP(launch_project_setp<T>(c, dctx<T>(h), h->projector, h->stream));
        if (dual_from_x0) NCS_HIP(launch_dual_init<T>(c, dctx<T>(h), h->stream));
    } else {
        NCS_HIP(hipMemsetAsync(h->x, 0, h->n * e, h->stream));
    }
    NCS_HIP(launch_control(h->ctl, 0, 0, std::nan(""), h->stream));
    h->iter_host = 0;
    return NCS_OK;
}

}  // namespace

extern "C" {

const char* ncs_last_error(void) { return g_err.c_str(); }

ncs_status ncs_setup(const ncs_geometry* geom, const ncs_params* params, int32_t dtype,
                     const void* b_dev, const void* bg_dev, void* stream, ncs_handle** out) {
    g_err.clear();
    if (!geom || !params || !out) {
        set_err("ncs_setup: null geometry, params or out pointer");
        return NCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    ncs_status s = validate(*geom, *params, dtype);
    if (s) return s;
    return setup_slice(*geom, *params, dtype, b_dev, bg_dev, static_cast<hipStream_t>(stream), nullptr, true, out);
}

void ncs_destroy(ncs_handle* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (void* ptr : h->allocs) (void)hipFree(ptr);
    delete h;
}

ncs_status ncs_set_init(ncs_handle* h, const void* x0_dev, int32_t dual_from_x0) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (dual_from_x0 && (!x0_dev || !h->b)) {
        set_err("ncs_set_init: dual_from_x0 needs x0 and data b");
        return NCS_ERR_INVALID_ARG;
    }
    return h->dtype == NCS_F64 ? init_state<double>(h, x0_dev, dual_from_x0)
                               : init_state<float>(h, x0_dev, dual_from_x0);
}

ncs_status ncs_set_x(ncs_handle* h, const void* x_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev) {
        set_err("ncs_set_x: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    // x = x_dev and p = E x; the duals and the iteration count are kept
    NCS_HIP(hipMemcpyAsync(h->x, x_dev, h->n * h->esz, hipMemcpyDeviceToDevice, h->stream));
    if (h->dtype == NCS_F64) {
        const DevCtx<double> c = make_ctx<double>(h);
        NCS_HIP(launch_pad_image<double>(c, dctx<double>(h), c.x, h->stream));
        NCS_HIP(launch_project_setp<double>(c, dctx<double>(h), h->projector, h->stream));
    } else {
        const DevCtx<float> c = make_ctx<float>(h);
        NCS_HIP(launch_pad_image<float>(c, dctx<float>(h), c.x, h->stream));
        NCS_HIP(launch_project_setp<float>(c, dctx<float>(h), h->projector, h->stream));
    }
    NCS_HIP(launch_control(h->ctl, 1, 0, std::nan(""), h->stream));
    return NCS_OK;
}

ncs_status ncs_iterate(ncs_handle* h, int32_t k, double* obj_host) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (k < 0) {
        set_err("ncs_iterate: k must be >= 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("ncs_iterate: handle has no data (b_dev was NULL)");
        return NCS_ERR_INVALID_ARG;
    }
    if (obj_host && k > kHistCap) {
        set_err("ncs_iterate: at most %d objectives can be returned per call", kHistCap);
        return NCS_ERR_INVALID_ARG;
    }
    if (k == 0) return NCS_OK;
    NCS_HIP(launch_control(h->ctl, 1, 0, std::nan(""), h->stream));
    const int start = h->iter_host;
    NCS_HIP(launch_iters(h, k));
    if (!obj_host) {
        h->iter_host += k;
        return NCS_OK;
    }
    Control c;
    if ((s = read_control(h, &c))) return s;
    const int done = c.iter - start;
    std::vector<double> hist(kHistCap);
    NCS_HIP(hipMemcpy(hist.data(), h->hist, kHistCap * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < k; ++i) obj_host[i] = i < done ? hist[(start + i) & (kHistCap - 1)] : std::nan("");
    if (c.status == -4) {
        set_err("ncs_iterate: objective became NaN at iteration %d", c.iter);
        return NCS_ERR_NONFINITE;
    }
    return NCS_OK;
}

ncs_status ncs_solve(ncs_handle* h, int32_t max_iters, double f_target, double fp_residual_tol, int32_t* iters_done,
                     double* f_final) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (max_iters < 0) {
        set_err("ncs_solve: max_iters must be >= 0");
        return NCS_ERR_INVALID_ARG;
    }
    if (fp_residual_tol != fp_residual_tol) {
        set_err("ncs_solve: fp_residual_tol is NaN");
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("ncs_solve: handle has no data (b_dev was NULL)");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(launch_control(h->ctl, 1, 0, f_target, h->stream));
    Control c;
    if ((s = read_control(h, &c))) return s;
    const int start = c.iter;
    int remaining = max_iters;
    int grow = 0;
    double f_prev = std::nan("");
    ncs_status result = NCS_NOT_CONVERGED;
    while (remaining > 0) {
        const int chunk = std::min(remaining, (int)h->p.check_every);
        NCS_HIP(launch_iters(h, chunk));
        remaining -= chunk;
        if (fp_residual_tol > 0.0) {
            if (h->dtype == NCS_F64) {
                NCS_HIP(launch_step_residual<double>(dctx<double>(h), h->stream));
            } else {
                NCS_HIP(launch_step_residual<float>(dctx<float>(h), h->stream));
            }
        }
        if ((s = read_control(h, &c))) return s;
        if (c.status == -4) {
            set_err("ncs_solve: objective became NaN at iteration %d", c.iter);
            result = NCS_ERR_NONFINITE;
            break;
        }
        if (c.status == 1) {
            result = NCS_OK;
            break;
        }
        if (fp_residual_tol > 0.0 && c.iter > 0 && std::sqrt(c.step_sq) <= fp_residual_tol * std::sqrt(c.x_sq)) {
            result = NCS_OK;
            break;
        }
        if (h->p.diverge_checks > 0) {
            grow = (f_prev == f_prev && c.f_last > f_prev) ? grow + 1 : 0;
            f_prev = c.f_last;
            if (grow >= h->p.diverge_checks) {
                set_err("ncs_solve: objective grew over %d consecutive checks (f = %g)", grow, c.f_last);
                result = NCS_ERR_DIVERGED;
                break;
            }
        }
    }
    if (iters_done) *iters_done = c.iter - start;
    if (f_final) *f_final = c.f_last;
    return result;
}

ncs_status ncs_get_objectives(ncs_handle* h, int32_t first, int32_t count, double* obj_host) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (count < 0 || first < 0 || (count > 0 && !obj_host) || count > kHistCap) {
        set_err("ncs_get_objectives: bad range");
        return NCS_ERR_INVALID_ARG;
    }
    Control c;
    if ((s = read_control(h, &c))) return s;
    if (first + count > c.iter || first < c.iter - kHistCap) {
        set_err("ncs_get_objectives: range [%d, %d) outside the stored history (iteration %d)", first,
                first + count, c.iter);
        return NCS_ERR_INVALID_ARG;
    }
    std::vector<double> hist(kHistCap);
    NCS_HIP(hipMemcpy(hist.data(), h->hist, kHistCap * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < count; ++i) obj_host[i] = hist[(first + i) & (kHistCap - 1)];
    return NCS_OK;
}

ncs_status ncs_get_iteration(ncs_handle* h, int32_t* iters) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!iters) {
        set_err("ncs_get_iteration: null output");
        return NCS_ERR_INVALID_ARG;
    }
    Control c;
    if ((s = read_control(h, &c))) return s;
    *iters = c.iter;
    return NCS_OK;
}

ncs_status ncs_get_x(ncs_handle* h, void* x_out_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_out_dev) {
        set_err("ncs_get_x: null output");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(hipMemcpyAsync(x_out_dev, h->x, h->n * h->esz, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_get_u(ncs_handle* h, void* u_out_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!u_out_dev) {
        set_err("ncs_get_u: null output");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(h->dtype == NCS_F64 ? launch_unpad_sinogram<double>(make_ctx<double>(h), dctx<double>(h),
                                                                (const double*)h->u, (double*)u_out_dev, h->stream)
                                : launch_unpad_sinogram<float>(make_ctx<float>(h), dctx<float>(h),
                                                               (const float*)h->u, (float*)u_out_dev, h->stream));
    return NCS_OK;
}

ncs_status ncs_get_v(ncs_handle* h, void* v_out_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!v_out_dev) {
        set_err("ncs_get_v: null output");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(hipMemcpyAsync(v_out_dev, h->v, 2 * h->n * h->esz, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

ncs_status ncs_get_t(ncs_handle* h, void* t_out_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!t_out_dev || !h->tpos) {
        set_err(!t_out_dev ? "ncs_get_t: null output" : "ncs_get_t: the handle has no positivity constraint");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(hipMemcpyAsync(t_out_dev, h->tpos, h->n * h->esz, hipMemcpyDeviceToDevice, h->stream));
    return NCS_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t dtype, n_side, n_angles, n_bins, iter, pad;
};
}  // namespace

ncs_status ncs_get_state(ncs_handle* h, void* host_buf, size_t* bytes) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!bytes) {
        set_err("ncs_get_state: null size pointer");
        return NCS_ERR_INVALID_ARG;
    }
    const size_t e = h->esz;
    const size_t need = sizeof(StateHeader) + (h->n + 2 * h->n + 2 * h->mp + (h->tpos ? h->n : 0)) * e;
    if (!host_buf) {
        *bytes = need;
        return NCS_OK;
    }
    if (*bytes < need) {
        set_err("ncs_get_state: buffer of %zu bytes, need %zu", *bytes, need);
        return NCS_ERR_INVALID_ARG;
    }
    Control c;
    if ((s = read_control(h, &c))) return s;
    StateHeader hd{kStateMagic, h->dtype, h->g.n_side, h->g.n_angles, h->g.n_bins, c.iter, 0};
    unsigned char* o = static_cast<unsigned char*>(host_buf);
    std::memcpy(o, &hd, sizeof(hd));
    o += sizeof(hd);
    NCS_HIP(hipMemcpy(o, h->x, h->n * e, hipMemcpyDeviceToHost));
    o += h->n * e;
    NCS_HIP(hipMemcpy(o, h->v, 2 * h->n * e, hipMemcpyDeviceToHost));
    o += 2 * h->n * e;
    NCS_HIP(hipMemcpy(o, h->u, h->mp * e, hipMemcpyDeviceToHost));
    o += h->mp * e;
    NCS_HIP(hipMemcpy(o, h->pj, h->mp * e, hipMemcpyDeviceToHost));
    if (h->tpos) {
        o += h->mp * e;
        NCS_HIP(hipMemcpy(o, h->tpos, h->n * e, hipMemcpyDeviceToHost));
    }
    *bytes = need;
    return NCS_OK;
}

ncs_status ncs_set_state(ncs_handle* h, const void* host_buf, size_t bytes) {
    ncs_status s = check_handle(h);
    if (s) return s;
    const size_t e = h->esz;
    const size_t need = sizeof(StateHeader) + (h->n + 2 * h->n + 2 * h->mp + (h->tpos ? h->n : 0)) * e;
    if (!host_buf || bytes != need) {
        set_err("ncs_set_state: blob of %zu bytes, expected %zu", bytes, need);
        return NCS_ERR_INVALID_ARG;
    }
    StateHeader hd;
    std::memcpy(&hd, host_buf, sizeof(hd));
    if (hd.magic != kStateMagic || hd.dtype != h->dtype || hd.n_side != h->g.n_side ||
        hd.n_angles != h->g.n_angles || hd.n_bins != h->g.n_bins || hd.iter < 0) {
        set_err("ncs_set_state: blob does not match this handle");
        return NCS_ERR_INVALID_ARG;
    }
    const unsigned char* i = static_cast<const unsigned char*>(host_buf) + sizeof(hd);
    NCS_HIP(hipStreamSynchronize(h->stream));
    NCS_HIP(hipMemcpy(h->x, i, h->n * e, hipMemcpyHostToDevice));
    i += h->n * e;
    NCS_HIP(hipMemcpy(h->v, i, 2 * h->n * e, hipMemcpyHostToDevice));
    i += 2 * h->n * e;
    NCS_HIP(hipMemcpy(h->u, i, h->mp * e, hipMemcpyHostToDevice));
    i += h->mp * e;
    NCS_HIP(hipMemcpy(h->pj, i, h->mp * e, hipMemcpyHostToDevice));
    if (h->tpos) {
        i += h->mp * e;
        NCS_HIP(hipMemcpy(h->tpos, i, h->n * e, hipMemcpyHostToDevice));
    }
    NCS_HIP(launch_control(h->ctl, 2, hd.iter, std::nan(""), h->stream));
    NCS_HIP(hipStreamSynchronize(h->stream));
    h->iter_host = hd.iter;
    return NCS_OK;
}

ncs_status ncs_forward(ncs_handle* h, const void* x_dev, void* y_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev || !y_dev) {
        set_err("ncs_forward: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (h->dtype == NCS_F64) {
        const DevCtx<double> c = make_ctx<double>(h);
        NCS_HIP(launch_pad_image<double>(c, dctx<double>(h), (const double*)x_dev, h->stream));
        NCS_HIP(launch_project_plain<double>(c, dctx<double>(h), h->projector, (double*)y_dev, h->stream));
    } else {
        const DevCtx<float> c = make_ctx<float>(h);
        NCS_HIP(launch_pad_image<float>(c, dctx<float>(h), (const float*)x_dev, h->stream));
        NCS_HIP(launch_project_plain<float>(c, dctx<float>(h), h->projector, (float*)y_dev, h->stream));
    }
    return NCS_OK;
}

}  // extern "C"

// ---- E x without allocating: workspace in a fixed device array -----------
namespace {

// Descriptor, angle tables and the padded image pair of ncs_forward_noalloc.
// Every call on a device uses that device's copy, which keeps the last call's
// contents (each call rewrites all it reads before reading it).
constexpr size_t kNoAllocScratch = (size_t)6 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The device address of this device's scratch array (the host-side symbol is
// only a stand-in): looked up once per device, with that device current.
ncs_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_err("ncs_forward_noalloc: device %d outside [0, %d)", dev, kMaxDevices);
        return NCS_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_err("ncs_forward_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return NCS_ERR_HIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return NCS_OK;
}

}  // namespace

extern "C" {

ncs_status ncs_forward_noalloc(const ncs_geometry* geom, const float* x_dev, float* y_dev, void* stream) {
    if (!geom || !x_dev || !y_dev) {
        set_err("ncs_forward_noalloc: null geometry, input or output pointer");
        return NCS_ERR_INVALID_ARG;
    }
    const ncs_geometry& g = *geom;
    if (g.beam != NCS_BEAM_PARALLEL) {
        set_err("ncs_forward_noalloc: parallel beams only (beam 0)");
        return NCS_ERR_INVALID_ARG;
    }
    if (!is_pow2(g.n_side) || g.n_side < 16 || g.n_side > 1024 || g.n_angles < 1 || g.n_angles > (1 << 20) ||
        g.n_bins < 2 || g.n_bins > (1 << 20)) {
        set_err("ncs_forward_noalloc: need n_side a power of two in [16, 1024], n_angles >= 1, n_bins >= 2");
        return NCS_ERR_INVALID_ARG;
    }
    const int N = g.n_side, NA = g.n_angles, NS = g.n_bins;
    const size_t P = (size_t)N + 2 * kPadL;
    // layout: descriptor | AngleT table | double coefficients | axes | padded image | padded transpose
    const size_t o_ang = align256(sizeof(DevCtx<float>));
    const size_t o_ang64 = o_ang + align256((size_t)NA * sizeof(AngleT<float>));
    const size_t o_axis = o_ang64 + align256((size_t)NA * 6 * sizeof(double));
    const size_t o_img = o_axis + align256((size_t)NA * sizeof(int32_t));
    const size_t o_imgT = o_img + align256((size_t)N * P * sizeof(float));
    const size_t need = o_imgT + (size_t)N * P * sizeof(float);
    if (need > kNoAllocScratch) {
        set_err("ncs_forward_noalloc: geometry %d^2, %d x %d needs %zu bytes of workspace, more than the %zu "
                "the fixed array holds", N, NA, NS, need, kNoAllocScratch);
        return NCS_ERR_INVALID_ARG;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_err("ncs_forward_noalloc: hipGetDevice failed");
        return NCS_ERR_HIP;
    }
    unsigned char* base = nullptr;
    ncs_status s = scratch_address(dev, &base);
    if (s) return s;
    DevCtx<float> c{};
    c.N = N;
    while ((1 << c.log2N) < N) ++c.log2N;
    c.NA = NA;
    c.NS = NS;
    c.PU = NS + 3;
    c.P = (int)P;
    c.nb_proj = project_blocks(NA, NS);
    c.nwg_proj = c.nb_proj;
    c.nb_tv = tv_blocks(N);
    c.ang = reinterpret_cast<const AngleT<float>*>(base + o_ang);
    c.ang64 = reinterpret_cast<const double*>(base + o_ang64);
    c.axis = reinterpret_cast<const int32_t*>(base + o_axis);
    c.xsc = reinterpret_cast<float*>(base + o_img);
    c.xscT = reinterpret_cast<float*>(base + o_imgT);
    DevCtx<float>* dc = reinterpret_cast<DevCtx<float>*>(base);
    hipStream_t st = static_cast<hipStream_t>(stream);
    NCS_HIP(launch_parallel_tables(c, dc, reinterpret_cast<AngleT<float>*>(base + o_ang),
                                   reinterpret_cast<double*>(base + o_ang64), reinterpret_cast<int32_t*>(base + o_axis),
                                   st));
    NCS_HIP(launch_pad_image_full<float>(c, dc, x_dev, st));
    NCS_HIP(launch_project_plain<float>(c, dc, 2, y_dev, st));
    return NCS_OK;
}

ncs_status ncs_adjoint(ncs_handle* h, const void* y_dev, void* x_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev || !y_dev) {
        set_err("ncs_adjoint: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (h->dtype == NCS_F64) {
        const DevCtx<double> c = make_ctx<double>(h);
        NCS_HIP(launch_pad_sinogram<double>(c, dctx<double>(h), (const double*)y_dev, c.ysc, h->stream));
        NCS_HIP(launch_backproject_plain<double>(c, dctx<double>(h), h->backprojector, c.ysc, (double*)x_dev, h->stream));
    } else {
        const DevCtx<float> c = make_ctx<float>(h);
        NCS_HIP(launch_pad_sinogram<float>(c, dctx<float>(h), (const float*)y_dev, c.ysc, h->stream));
        NCS_HIP(launch_backproject_plain<float>(c, dctx<float>(h), h->backprojector, c.ysc, (float*)x_dev, h->stream));
    }
    return NCS_OK;
}

ncs_status ncs_apply_minv(ncs_handle* h, const void* w_dev, void* out_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!w_dev || !out_dev) {
        set_err("ncs_apply_minv: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(h->dtype == NCS_F64
                ? launch_apply_minv<double>(make_ctx<double>(h), dctx<double>(h), (const double*)w_dev,
                                            (double*)out_dev, (double)h->p.alpha, h->stream)
                : launch_apply_minv<float>(make_ctx<float>(h), dctx<float>(h), (const float*)w_dev,
                                           (float*)out_dev, (float)h->p.alpha, h->stream));
    return NCS_OK;
}

ncs_status ncs_prefilter(ncs_handle* h, const void* y_dev, void* x_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev || !y_dev) {
        set_err("ncs_prefilter: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    // E^T y into the handle's backprojection buffer (not live between
    // iterations), then alpha M^+: the column pass scales h/(alpha N^2) by alpha^2
    if (h->dtype == NCS_F64) {
        const DevCtx<double> c = make_ctx<double>(h);
        const double a = h->p.alpha;
        NCS_HIP(launch_pad_sinogram<double>(c, dctx<double>(h), (const double*)y_dev, c.ysc, h->stream));
        NCS_HIP(launch_backproject_plain<double>(c, dctx<double>(h), h->backprojector, c.ysc, c.w, h->stream));
        NCS_HIP(launch_apply_minv<double>(c, dctx<double>(h), c.w, (double*)x_dev, a * a, h->stream));
    } else {
        const DevCtx<float> c = make_ctx<float>(h);
        const float a2 = (float)(h->p.alpha * h->p.alpha);
        NCS_HIP(launch_pad_sinogram<float>(c, dctx<float>(h), (const float*)y_dev, c.ysc, h->stream));
        NCS_HIP(launch_backproject_plain<float>(c, dctx<float>(h), h->backprojector, c.ysc, c.w, h->stream));
        NCS_HIP(launch_apply_minv<float>(c, dctx<float>(h), c.w, (float*)x_dev, a2, h->stream));
    }
    return NCS_OK;
}

ncs_status ncs_fbp(ncs_handle* h, const void* y_dev, void* x_dev) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev || !y_dev) {
        set_err("ncs_fbp: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (h->g.n_bins > 4096) {
        set_err("ncs_fbp: at most 4096 detector bins (got %d)", h->g.n_bins);
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(h->dtype == NCS_F64
                ? launch_fbp<double>(make_ctx<double>(h), dctx<double>(h), h->backprojector, (const double*)y_dev, (double*)x_dev, h->stream)
                : launch_fbp<float>(make_ctx<float>(h), dctx<float>(h), h->backprojector, (const float*)y_dev, (float*)x_dev, h->stream));
    return NCS_OK;
}

ncs_status ncs_objective(ncs_handle* h, const void* x_dev, double* f) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (!x_dev || !f) {
        set_err("ncs_objective: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("ncs_objective: handle has no data (b_dev was NULL)");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(h->dtype == NCS_F64 ? launch_eval_objective<double>(make_ctx<double>(h), dctx<double>(h), h->projector,
                                                                (const double*)x_dev, h->stream)
                                : launch_eval_objective<float>(make_ctx<float>(h), dctx<float>(h), h->projector,
                                                               (const float*)x_dev, h->stream));
    Control c;
    if ((s = read_control(h, &c))) return s;
    *f = c.eval_out;
    return NCS_OK;
}

ncs_status ncs_time_phases(ncs_handle* h, int32_t iters, double* ms_host) {
    ncs_status s = check_handle(h);
    if (s) return s;
    if (iters < 1 || !ms_host) {
        set_err("ncs_time_phases: need iters >= 1 and an output array");
        return NCS_ERR_INVALID_ARG;
    }
    if (!h->b) {
        set_err("ncs_time_phases: handle has no data (b_dev was NULL)");
        return NCS_ERR_INVALID_ARG;
    }
    if (h->p.method == NCS_METHOD_ADMM_CG) {
        set_err("ncs_time_phases: the phases are those of NCS and PDHG, not of ADMM-CG");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(launch_control(h->ctl, 1, 0, std::nan(""), h->stream));
    // one full iteration first, so that every phase starts from warm state
    hipError_t le = hipSuccess;
    for (int ph = 0; ph < NCS_N_PHASES && le == hipSuccess; ++ph) le = launch_phase(h, ph);
    // each phase: iters back-to-back launches between two events, so that the
    // event overhead is spread over them (the launches of an iteration run
    // back to back in the replayed graphs too)
    std::vector<hipEvent_t> ev(2 * NCS_N_PHASES);
    for (auto& e : ev) NCS_HIP(hipEventCreate(&e));
    for (int ph = 0; ph < NCS_N_PHASES && le == hipSuccess; ++ph) {
        (void)hipEventRecord(ev[2 * ph], h->stream);
        for (int i = 0; i < iters && le == hipSuccess; ++i) le = launch_phase(h, ph);
        (void)hipEventRecord(ev[2 * ph + 1], h->stream);
    }
    hipError_t se = hipStreamSynchronize(h->stream);
    for (int ph = 0; ph < NCS_N_PHASES; ++ph) ms_host[ph] = 0.0;
    if (le == hipSuccess && se == hipSuccess) {
        for (int ph = 0; ph < NCS_N_PHASES; ++ph) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[2 * ph], ev[2 * ph + 1]);
            ms_host[ph] = ms / iters;
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    NCS_HIP(le);
    NCS_HIP(se);
    Control c;
    return read_control(h, &c);
}

ncs_status ncs_get_info(ncs_handle* h, ncs_info* info) {
    if (!h || !info) {
        set_err("ncs_get_info: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (h->nnz < 0) h->nnz = h->g.beam == NCS_BEAM_FAN ? count_nnz_fan(h) : count_nnz(h->g, h->tab);
    info->nnz = h->nnz;
    info->c_r = h->c_r;
    info->mu_dc = h->mu_dc;
    info->norm_e1_sq = h->norm_e1_sq;
    info->projector = h->projector;
    info->backprojector = h->backprojector;
    info->projector_ms[0] = h->projector_ms[0];
    info->projector_ms[1] = h->projector_ms[1];
    info->projector_ms[2] = h->projector_ms[2];
    info->backprojector_ms[0] = h->backprojector_ms[0];
    info->backprojector_ms[1] = h->backprojector_ms[1];
    info->backprojector_ms[2] = h->backprojector_ms[2];
    return NCS_OK;
}

ncs_status ncs_get_eigenvalues(ncs_handle* h, double* mu_host) {
    if (!h || !mu_host) {
        set_err("ncs_get_eigenvalues: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    std::memcpy(mu_host, h->mu.data(), h->mu.size() * sizeof(double));
    return NCS_OK;
}

}  // extern "C"

// ===========================================================================
// Batches of slices
// ===========================================================================
namespace {

// Rebuild the workgroup maps of the active slices.  Slices are pinned to XCDs
// (longest-processing-time assignment by projector workgroups); workgroup b
// of a launch is dispatched to XCD b mod 8, so the map interleaves the eight
// per-XCD lists and each slice's workgroups share one XCD's L2.
void drop_batch_graphs(ncs_batch* B) {
    for (int j = 0; j < 2; ++j) {
        if (B->graph[j]) (void)hipGraphExecDestroy(B->graph[j]);
        B->graph[j] = nullptr;
        B->graph_k[j] = 0;
    }
}

// Projector workgroups of slice i (with its TV tiles): the unit of the map's
// size and of the work that stopped slices leave idle in it.
int proj_work(const ncs_batch* B, int i) {
    const ncs_handle* h = B->slices[i];
    return project_blocks(h->g.n_angles, h->g.n_bins) + tv_blocks(h->g.n_side);
}

ncs_status build_maps(ncs_batch* B) {
    drop_batch_graphs(B);
    const int nphase = 5;
    std::vector<std::vector<Slot>> lists[5];
    for (int ph = 0; ph < nphase; ++ph) lists[ph].assign(kXcds, {});
    for (int i = 0; i < B->n; ++i) {
        if (!B->active[i]) continue;
        const ncs_handle* h = B->slices[i];
        const int N = h->g.n_side;
        const int cnt[5] = {bp_blocks(N, B->backprojector), N / 2, N / 2 + 1, proj_work(B, i), 1};
        const int x = B->xcd_of[i];
        for (int ph = 0; ph < nphase; ++ph)
            for (int l = 0; l < cnt[ph]; ++l) lists[ph][x].push_back(Slot{i, l});
    }
    for (int ph = 0; ph < nphase; ++ph) {
        std::vector<Slot> flat;
        size_t longest = 0;
        for (auto& l : lists[ph]) longest = std::max(longest, l.size());
        for (size_t r = 0; r < longest; ++r)
            for (int x = 0; x < kXcds; ++x)
                if (r < lists[ph][x].size()) flat.push_back(lists[ph][x][r]);
        B->blocks[ph] = (int)flat.size();
        if (flat.empty()) continue;
        if (flat.size() > B->map_cap[ph]) {
            if (B->maps[ph]) (void)hipFree(B->maps[ph]);
            B->maps[ph] = nullptr;
            B->map_cap[ph] = 0;
            NCS_HIP(hipMalloc(reinterpret_cast<void**>(&B->maps[ph]), flat.size() * sizeof(Slot)));
            B->map_cap[ph] = flat.size();
        }
        NCS_HIP(hipMemcpy(B->maps[ph], flat.data(), flat.size() * sizeof(Slot), hipMemcpyHostToDevice));
    }
    B->mapped = B->active;
    return NCS_OK;
}

template <class T>
hipError_t batch_iterate(ncs_batch* B, int k) {
    if (B->blocks[3] == 0) return hipSuccess;
    IterLaunch<T> L{};
    L.ctxs = static_cast<const DevCtx<T>*>(B->dctxs);
    L.bp = {B->maps[0], B->blocks[0]};
    L.rows = {B->maps[1], B->blocks[1]};
    L.cols = {B->maps[2], B->blocks[2]};
    L.proj = {B->maps[3], B->blocks[3]};
    L.fin = {B->maps[4], B->blocks[4]};
    L.max_N = B->max_N;
    L.projector = B->projector;
    L.backprojector = B->backprojector;
    return launch_iterations<T>(L, k, B->stream);
}

hipError_t batch_iterate_any(ncs_batch* B, int k, hipStream_t st) {
    hipStream_t keep = B->stream;
    B->stream = st;
    const hipError_t e = B->dtype == NCS_F64 ? batch_iterate<double>(B, k) : batch_iterate<float>(B, k);
    B->stream = keep;
    return e;
}

// k batch iterations as a replayed graph: captured on a private stream at the
// first request for this k after the maps were (re)built.  A capture failure
// switches the batch to direct launches.
hipError_t batch_launch(ncs_batch* B, int k) {
    if (k <= 0 || B->blocks[3] == 0) return hipSuccess;
    if (B->use_graphs) {
        int j = B->graph_k[0] == k ? 0 : B->graph_k[1] == k ? 1 : -1;
        if (j < 0) {
            j = B->graph[0] ? 1 : 0;
            if (B->graph[j]) (void)hipGraphExecDestroy(B->graph[j]);
            B->graph[j] = nullptr;
            B->graph_k[j] = 0;
            bool ok = B->cap_stream || hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking) == hipSuccess;
            if (ok) ok = hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                const hipError_t le = batch_iterate_any(B, k, B->cap_stream);
                hipGraph_t graph = nullptr;
                const hipError_t ee = hipStreamEndCapture(B->cap_stream, &graph);
                ok = le == hipSuccess && ee == hipSuccess && graph &&
                     hipGraphInstantiate(&B->graph[j], graph, nullptr, nullptr, 0) == hipSuccess;
                if (graph) (void)hipGraphDestroy(graph);
                if (ok) ok = hipGraphUpload(B->graph[j], B->stream) == hipSuccess;
            }
            if (!ok) {
                (void)hipGetLastError();
                B->graph[j] = nullptr;
                drop_batch_graphs(B);
                B->use_graphs = false;
                return batch_iterate_any(B, k, B->stream);
            }
            B->graph_k[j] = k;
        }
        return hipGraphLaunch(B->graph[j], B->stream);
    }
    return batch_iterate_any(B, k, B->stream);
}


// Kernel selection for a batch: time a few batched iterations of every
// candidate (projector, backprojector) pair on the zeroed state of all
// slices and keep the fastest (the whole batch loads the GPU differently from
// the single-slice timing done at slice setup).
template <class T>
ncs_status autotune_batch(ncs_batch* B, bool tune_p, bool tune_b) {
    for (ncs_handle* h : B->slices) {
        ncs_status s = init_state<T>(h, nullptr, 0);
        if (s) return s;
    }
    const int p0 = B->projector, b0 = B->backprojector;
    hipEvent_t e0, e1;
    NCS_HIP(hipEventCreate(&e0));
    NCS_HIP(hipEventCreate(&e1));
    float best = -1.f;
    int bp = p0, bb = b0;
    for (int pv = 1; pv <= 3; ++pv) {
        if (!tune_p && pv != p0) continue;
        for (int bv = 1; bv <= kNumBackprojectors; ++bv) {
            if (!tune_b && bv != b0) continue;
            B->projector = pv;
            B->backprojector = bv;
            ncs_status s = build_maps(B);
            if (s) return s;
            NCS_HIP(batch_iterate<T>(B, 1));
            NCS_HIP(hipEventRecord(e0, B->stream));
            NCS_HIP(batch_iterate<T>(B, 3));
            NCS_HIP(hipEventRecord(e1, B->stream));
            NCS_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            NCS_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (best < 0.f || ms < best) {
                best = ms;
                bp = pv;
                bb = bv;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->projector = bp;
    B->backprojector = bb;
    for (ncs_handle* h : B->slices) {
        h->projector = bp;
        h->backprojector = bb;
    }
    return build_maps(B);
}

template <class T>
ncs_status batch_upload_ctxs(ncs_batch* B) {
    std::vector<DevCtx<T>> all(B->n);
    for (int i = 0; i < B->n; ++i) all[i] = make_ctx<T>(B->slices[i]);
    NCS_HIP(hipMemcpy(B->dctxs, all.data(), all.size() * sizeof(DevCtx<T>), hipMemcpyHostToDevice));
    return NCS_OK;
}

ncs_status check_batch(ncs_batch* B) {
    if (!B) {
        set_err("null batch");
        return NCS_ERR_INVALID_ARG;
    }
    NCS_HIP(hipSetDevice(B->device));
    return NCS_OK;
}

}  // namespace

extern "C" {

ncs_status ncs_batch_setup(int32_t n_slices, const ncs_geometry* geoms, const ncs_params* params, int32_t dtype,
                           const void* const* b_dev, const void* const* bg_dev, void* stream, ncs_batch** out) {
    g_err.clear();
    if (!out || !geoms || !params || !b_dev || n_slices < 1) {
        set_err("ncs_batch_setup: need n_slices >= 1 and non-null geometry, params, data and out");
        return NCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    for (int i = 0; i < n_slices; ++i) {
        ncs_status s = validate(geoms[i], params[i], dtype);
        if (s) {
            const std::string msg = g_err;
            set_err("ncs_batch_setup: slice %d: %s", i, msg.c_str());
            return s;
        }
        if (!b_dev[i]) {
            set_err("ncs_batch_setup: slice %d has no data", i);
            return NCS_ERR_INVALID_ARG;
        }
        if (params[i].method == NCS_METHOD_ADMM_CG) {
            set_err("ncs_batch_setup: slice %d: batches run NCS or PDHG, not ADMM-CG", i);
            return NCS_ERR_INVALID_ARG;
        }
        if (geoms[i].beam != geoms[0].beam) {
            set_err("ncs_batch_setup: slice %d: the slices of a batch are all parallel-beam or all fan-beam", i);
            return NCS_ERR_INVALID_ARG;
        }
    }
    const bool fan = geoms[0].beam == NCS_BEAM_FAN;   // fan slices have one projector pair
    ncs_batch* B = new ncs_batch();
    B->n = n_slices;
    B->dtype = dtype;
    B->stream = static_cast<hipStream_t>(stream);
    B->check_every = params[0].check_every > 0 ? params[0].check_every : 50;
    B->use_graphs = params[0].graph_chunk >= 0;
    auto fail = [&](ncs_status s) {
        ncs_batch_destroy(B);
        return s;
    };
    if (hipGetDevice(&B->device) != hipSuccess) {
        set_err("ncs_batch_setup: hipGetDevice failed");
        delete B;
        return NCS_ERR_HIP;
    }
    if (hipMalloc(reinterpret_cast<void**>(&B->ctls), (size_t)n_slices * sizeof(Control)) != hipSuccess) {
        set_err("ncs_batch_setup: control array allocation failed");
        B->ctls = nullptr;
        return fail(NCS_ERR_OOM);
    }
    const size_t ctx_bytes = dtype == NCS_F64 ? sizeof(DevCtx<double>) : sizeof(DevCtx<float>);
    if (hipMalloc(&B->dctxs, (size_t)n_slices * ctx_bytes) != hipSuccess) {
        set_err("ncs_batch_setup: descriptor array allocation failed");
        B->dctxs = nullptr;
        return fail(NCS_ERR_OOM);
    }
    // projector choice: params[0].projector, or (0) timed on the largest slice
    int largest = 0;
    for (int i = 1; i < n_slices; ++i)
        if ((long long)geoms[i].n_side * geoms[i].n_angles > (long long)geoms[largest].n_side * geoms[largest].n_angles)
            largest = i;
    B->slices.assign(n_slices, nullptr);
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < n_slices; ++i) {
            if ((pass == 0) != (i == largest)) continue;
            ncs_params p = params[i];
            p.graph_chunk = -1;
            if (pass == 1 && !fan) {
                p.projector = B->projector;
                p.backprojector = B->backprojector;
            }
            ncs_status s = setup_slice(geoms[i], p, dtype, b_dev[i], bg_dev ? bg_dev[i] : nullptr, B->stream,
                                       B->ctls + i, pass == 0, &B->slices[i]);
            if (s) {
                const std::string msg = g_err;
                set_err("ncs_batch_setup: slice %d: %s", i, msg.c_str());
                return fail(s);
            }
            if (pass == 0) {
                B->projector = B->slices[i]->projector;
                B->backprojector = B->slices[i]->backprojector;
            }
            B->max_N = std::max(B->max_N, geoms[i].n_side);
        }
    }
    // LPT assignment of slices to XCDs by projector workgroups x image side
    std::vector<int> order(n_slices);
    std::iota(order.begin(), order.end(), 0);
    auto cost = [&](int i) {
        const ncs_handle* h = B->slices[i];
        return (double)project_blocks(h->g.n_angles, h->g.n_bins) * h->g.n_side;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    std::vector<double> load(kXcds, 0.0);
    B->xcd_of.assign(n_slices, 0);
    for (int i : order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        B->xcd_of[i] = x;
        load[x] += cost(i);
    }
    B->active.assign(n_slices, 1);
    ncs_status s = dtype == NCS_F64 ? batch_upload_ctxs<double>(B) : batch_upload_ctxs<float>(B);
    if (s) return fail(s);
    if ((s = build_maps(B))) return fail(s);
    const bool tune_p = !fan && params[0].projector == 0, tune_b = !fan && params[0].backprojector == 0;
    if (tune_p || tune_b) {
        s = dtype == NCS_F64 ? autotune_batch<double>(B, tune_p, tune_b) : autotune_batch<float>(B, tune_p, tune_b);
        if (s) return fail(s);
    }
    *out = B;
    return NCS_OK;
}

void ncs_batch_destroy(ncs_batch* B) {
    if (!B) return;
    (void)hipSetDevice(B->device);
    (void)hipStreamSynchronize(B->stream);
    for (ncs_handle* h : B->slices) ncs_destroy(h);
    drop_batch_graphs(B);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    for (Slot* m : B->maps)
        if (m) (void)hipFree(m);
    if (B->dctxs) (void)hipFree(B->dctxs);
    if (B->ctls) (void)hipFree(B->ctls);
    delete B;
}

ncs_status ncs_batch_set_init(ncs_batch* B, const void* const* x0_dev, int32_t dual_from_x0) {
    ncs_status s = check_batch(B);
    if (s) return s;
    for (int i = 0; i < B->n; ++i) {
        if ((s = ncs_set_init(B->slices[i], x0_dev ? x0_dev[i] : nullptr, dual_from_x0))) return s;
        B->active[i] = 1;
    }
    return B->mapped != B->active ? build_maps(B) : NCS_OK;
}

ncs_status ncs_batch_solve(ncs_batch* B, int32_t max_iters, const double* f_target, int32_t* iters_done,
                           double* f_final) {
    ncs_status s = check_batch(B);
    if (s) return s;
    if (max_iters < 0) {
        set_err("ncs_batch_solve: max_iters must be >= 0");
        return NCS_ERR_INVALID_ARG;
    }
    std::vector<int> start(B->n);
    std::vector<char> skip(B->n, 0);
    for (int i = 0; i < B->n; ++i) {
        const double t = f_target ? f_target[i] : std::nan("");
        skip[i] = t == -std::numeric_limits<double>::infinity();
        if (!skip[i]) NCS_HIP(launch_control(B->ctls + i, 1, 0, t, B->stream));
        B->active[i] = !skip[i];
    }
    std::vector<Control> c(B->n);
    NCS_HIP(hipMemcpyAsync(c.data(), B->ctls, B->n * sizeof(Control), hipMemcpyDeviceToHost, B->stream));
    NCS_HIP(hipStreamSynchronize(B->stream));
    for (int i = 0; i < B->n; ++i) start[i] = c[i].iter;
    if (B->mapped != B->active && (s = build_maps(B))) return s;
    int remaining = max_iters;
    bool any_nan = false;
    while (remaining > 0) {
        const int chunk = std::min(remaining, B->check_every);
        NCS_HIP(batch_launch(B, chunk));
        remaining -= chunk;
        NCS_HIP(hipMemcpyAsync(c.data(), B->ctls, B->n * sizeof(Control), hipMemcpyDeviceToHost, B->stream));
        NCS_HIP(hipStreamSynchronize(B->stream));
        int left = 0, work = 0;
        for (int i = 0; i < B->n; ++i) {
            if (B->active[i] && c[i].stop) {
                B->active[i] = 0;
                any_nan |= c[i].status == -4;
            }
            left += B->active[i];
            if (B->active[i]) work += proj_work(B, i);
        }
        if (left == 0) break;
        // stopped slices' workgroups exit at once; the maps (and the graphs
        // replaying them) are rebuilt only when a quarter of the projection
        // workgroups in them belong to stopped slices
        if (4 * (B->blocks[3] - work) >= B->blocks[3] && (s = build_maps(B))) return s;
    }
    bool all_reached = true;
    for (int i = 0; i < B->n; ++i) {
        if (iters_done) iters_done[i] = c[i].iter - start[i];
        if (f_final) f_final[i] = c[i].f_last;
        all_reached &= skip[i] || c[i].status == 1;
        B->slices[i]->iter_host = c[i].iter;
    }
    if (any_nan) {
        set_err("ncs_batch_solve: a slice's objective became NaN");
        return NCS_ERR_NONFINITE;
    }
    return all_reached ? NCS_OK : NCS_NOT_CONVERGED;
}

ncs_status ncs_batch_slice(ncs_batch* B, int32_t i, ncs_handle** slice) {
    ncs_status s = check_batch(B);
    if (s) return s;
    if (i < 0 || i >= B->n || !slice) {
        set_err("ncs_batch_slice: index %d outside [0, %d)", i, B->n);
        return NCS_ERR_INVALID_ARG;
    }
    *slice = B->slices[i];
    return NCS_OK;
}

}  // extern "C"
