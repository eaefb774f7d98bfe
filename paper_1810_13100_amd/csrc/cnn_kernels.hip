// HIP kernels of the warm-start network for gfx950 (CDNA4): 3x3 "same"
// convolutions on NHWC bfloat16 activations with FP32 accumulation on the
// matrix cores (v_mfma_f32_16x16x32_bf16), the weight gradients, the loss and
// Adam on FP32 master weights.
//
// Convolution as an implicit GEMM per 16 x 16 output tile: the output
// channels are the M side of the matrix instruction, the 16 pixels of one
// tile row the N side, and the 32 input channels of one tap the K side, so
// one tap of one tile row is one instruction per 16 output channels.  The
// tile and its one-pixel halo are staged in LDS with 80-byte pixel pitch
// (32 channels + 8 pad), which makes the 16-byte operand reads of 16
// consecutive pixels conflict-free.
//
// Weight gradient (32 -> 32): the pixels are the K side.  The output gradient
// and three column-shifted copies of the input halo are staged channel-major,
// so that 8 consecutive pixels of one channel are one aligned 16-byte read for
// every tap.  Each wave owns one (16 output, 16 input) channel block for all
// nine taps; the bias gradient is one more instruction against a ones matrix.
// Per-workgroup partial sums are added afterwards in a fixed order.
//
// Register layout of v_mfma_f32_16x16x32_bf16 (64 lanes, l = lane):
//   A (16 x 32): lane l holds row l % 16, k = 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16): lane l holds column l % 16, the same k range
//   D (16 x 16): lane l holds column l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3
// (any k order shared by A and B gives the same product).
#include "cnn_internal.h"

namespace ncs {
namespace cnn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kHalo = kTile + 2;     // staged tile side with the halo
constexpr int kPixPitch = 40;        // LDS elements per staged pixel (32 channels + 8)
constexpr int kDzPitch = 264;        // LDS elements per channel of a staged output gradient (256 + 8)
constexpr int kXPitch = 296;         // LDS elements per channel of a shifted input copy (18 x 16 + 8)

__device__ inline float bf2f(uint32_t h) { return __uint_as_float((h & 0xFFFFu) << 16); }
__device__ inline uint32_t f2bf(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, static_cast<__bf16>(f)); }
__device__ inline bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct TileXY {
    int b, y0, x0;
};

__device__ inline int tiles_of(int B, int H, int W) {
    return B * ((H + kTile - 1) / kTile) * ((W + kTile - 1) / kTile);
}

__device__ inline TileXY tile_of(int idx, int H, int W) {
    const int tx_n = (W + kTile - 1) / kTile, ty_n = (H + kTile - 1) / kTile;
    TileXY t;
    const int tx = idx % tx_n;
    idx /= tx_n;
    const int ty = idx % ty_n;
    t.b = idx / ty_n;
    t.y0 = ty * kTile;
    t.x0 = tx * kTile;
    return t;
}

// Output of a convolution tile.  Lane (li, lg) of wave `wave` holds, for row i
// of the wave's four tile rows, pixel column li and output channels
// ct * 16 + 4 lg + e.
template <int COUT, int EPI, int NCT>
__device__ inline void conv_epilogue(const ConvArgs& a, const TileXY& T, size_t img, int wave, int li, int lg,
                                     const f32x4 (&acc)[4][NCT]) {
    const int x = T.x0 + li;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int y = T.y0 + wave * 4 + i;
        if (y >= a.H || x >= a.W) continue;
        const size_t pix = img + (size_t)y * a.W + x;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int co0 = ct * 16 + lg * 4;
            if (co0 >= COUT) continue;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = acc[i][ct][e] + ((a.bias && co0 + e < COUT) ? a.bias[co0 + e] : 0.f);
            if constexpr (EPI == EPI_RELU_BF16 || EPI == EPI_MASK_BF16) {
                uint16_t* o = static_cast<uint16_t*>(a.out) + pix * COUT + co0;
                if constexpr (EPI == EPI_RELU_BF16) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = fmaxf(v[e], 0.f);
                } else {
                    const u32x2 m = *reinterpret_cast<const u32x2*>(a.mask + pix * COUT + co0);
                    v[0] = bf2f(m.x) > 0.f ? v[0] : 0.f;
                    v[1] = bf2f(m.x >> 16) > 0.f ? v[1] : 0.f;
                    v[2] = bf2f(m.y) > 0.f ? v[2] : 0.f;
                    v[3] = bf2f(m.y >> 16) > 0.f ? v[3] : 0.f;
                }
                u32x2 r;
                r.x = f2bf(v[0]) | (f2bf(v[1]) << 16);
                r.y = f2bf(v[2]) | (f2bf(v[3]) << 16);
                *reinterpret_cast<u32x2*>(o) = r;
            } else if constexpr (EPI == EPI_F32) {
                float* o = static_cast<float*>(a.out) + pix * COUT + co0;
                if constexpr (COUT == 1) {
                    o[0] = v[0];
                } else {
                    f32x4 r = {v[0], v[1], v[2], v[3]};
                    *reinterpret_cast<f32x4*>(o) = r;
                }
            } else {
                static_cast<float*>(a.out)[pix] = a.resid[pix] + v[0];
            }
        }
    }
}

// 32 input channels -> COUT (32 or 1) output channels.
template <int COUT, int EPI>
__global__ __launch_bounds__(256) void k_conv32(ConvArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t tile[kHalo * kHalo * kPixPitch];
    const TileXY T = tile_of(blockIdx.x, a.H, a.W);
    const size_t img = (size_t)T.b * a.H * a.W;
    for (int c = threadIdx.x; c < kHalo * kHalo * 4; c += 256) {
        const int pix = c >> 2, part = c & 3;
        const int ry = pix / kHalo, rx = pix - ry * kHalo;
        const int y = T.y0 - 1 + ry, x = T.x0 - 1 + rx;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (y >= 0 && y < a.H && x >= 0 && x < a.W)
            v = *reinterpret_cast<const u32x4*>(a.in + (img + (size_t)y * a.W + x) * kChannels + part * 8);
        *reinterpret_cast<u32x4*>(tile + pix * kPixPitch + part * 8) = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    constexpr int NCT = COUT == 1 ? 1 : 2;
    bf16x8 wa[9][NCT];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const int co = ct * 16 + li;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (co < COUT) v = *reinterpret_cast<const u32x4*>(a.w + ((size_t)t * COUT + co) * kChannels + lg * 8);
            wa[t][ct] = as_bf16x8(v);
        }
    __syncthreads();
    f32x4 acc[4][NCT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) acc[i][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = wave * 4 + i;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;    // tap offset + 1
            const bf16x8 bv = as_bf16x8(
                *reinterpret_cast<const u32x4*>(tile + ((r + dy) * kHalo + li + dx) * kPixPitch + lg * 8));
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) acc[i][ct] = mfma(wa[t][ct], bv, acc[i][ct]);
        }
    }
    conv_epilogue<COUT, EPI, NCT>(a, T, img, wave, li, lg, acc);
}

// 1 input channel -> 32 output channels: the nine taps are the K side.
template <int EPI>
__global__ __launch_bounds__(256) void k_conv1(ConvArgs a) {
    __shared__ uint16_t tile[kHalo * kHalo];
    const TileXY T = tile_of(blockIdx.x, a.H, a.W);
    const size_t img = (size_t)T.b * a.H * a.W;
    for (int p = threadIdx.x; p < kHalo * kHalo; p += 256) {
        const int ry = p / kHalo, rx = p - ry * kHalo;
        const int y = T.y0 - 1 + ry, x = T.x0 - 1 + rx;
        tile[p] = (y >= 0 && y < a.H && x >= 0 && x < a.W) ? a.in[img + (size_t)y * a.W + x] : (uint16_t)0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    bf16x8 wa[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int t = lg * 8 + e;
            h[e] = t < 9 ? (uint32_t)a.w[t * kChannels + ct * 16 + li] : 0u;
        }
        const u32x4 v = {h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
        wa[ct] = as_bf16x8(v);
    }
    __syncthreads();
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = wave * 4 + i;
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int t = lg * 8 + e;
            h[e] = t < 9 ? (uint32_t)tile[(r + t / 3) * kHalo + li + t % 3] : 0u;
        }
        const u32x4 v = {h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
        const bf16x8 bv = as_bf16x8(v);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[i][ct] = mfma(wa[ct], bv, f32x4{0.f, 0.f, 0.f, 0.f});
    }
    conv_epilogue<kChannels, EPI, 2>(a, T, img, wave, li, lg, acc);
}

// Weight and bias gradient of a 32 -> 32 convolution (matrix cores).
__global__ __launch_bounds__(256) void k_wgrad32(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz,
                                                 int B, int H, int W, float* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) uint16_t dzs[kChannels * kDzPitch];
    __shared__ __attribute__((aligned(16))) uint16_t xs[3 * kChannels * kXPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int cot = wave >> 1, cit = wave & 1;   // this wave's output / input channel block
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 accb = {0.f, 0.f, 0.f, 0.f};
    const bf16x8 ones = as_bf16x8(u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u});
    const int ntiles = tiles_of(B, H, W);
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const TileXY T = tile_of(tl, H, W);
        const size_t img = (size_t)T.b * H * W;
        __syncthreads();
        {
            // output gradient of the tile, channel-major; zero outside the image
            const int p = threadIdx.x;
            const int y = T.y0 + (p >> 4), xx = T.x0 + (p & 15);
            const bool in = y < H && xx < W;
            const uint16_t* src = dz + (img + (size_t)(in ? y : 0) * W + (in ? xx : 0)) * kChannels;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                u32x4 v = {0u, 0u, 0u, 0u};
                if (in) v = *reinterpret_cast<const u32x4*>(src + q * 8);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    dzs[(q * 8 + 2 * j) * kDzPitch + p] = (uint16_t)(v[j] & 0xFFFFu);
                    dzs[(q * 8 + 2 * j + 1) * kDzPitch + p] = (uint16_t)(v[j] >> 16);
                }
            }
        }
        // input halo, channel-major, in three copies shifted by dx = -1, 0, 1:
        // copy d at (row ry, column cx) holds pixel (y0 - 1 + ry, x0 + cx + d - 1)
        for (int hpix = threadIdx.x; hpix < kHalo * kHalo; hpix += 256) {
            const int ry = hpix / kHalo, hx = hpix - ry * kHalo;
            const int y = T.y0 - 1 + ry, xx = T.x0 - 1 + hx;
            const bool in = y >= 0 && y < H && xx >= 0 && xx < W;
            const uint16_t* src = x + (img + (size_t)(in ? y : 0) * W + (in ? xx : 0)) * kChannels;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                u32x4 v = {0u, 0u, 0u, 0u};
                if (in) v = *reinterpret_cast<const u32x4*>(src + q * 8);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int cx = hx - d;
                    if (cx < 0 || cx >= kTile) continue;
                    uint16_t* dst = xs + (size_t)d * kChannels * kXPitch + ry * kTile + cx;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        dst[(q * 8 + 2 * j) * kXPitch] = (uint16_t)(v[j] & 0xFFFFu);
                        dst[(q * 8 + 2 * j + 1) * kXPitch] = (uint16_t)(v[j] >> 16);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int s = 0; s < kTile / 2; ++s) {
            // K side: 32 pixels, rows 2s and 2s + 1; lane group lg holds 8 of them
            const int prow = 2 * s + (lg >> 1), pcol = (lg & 1) * 8;
            const bf16x8 av = as_bf16x8(
                *reinterpret_cast<const u32x4*>(dzs + (cot * 16 + li) * kDzPitch + prow * kTile + pcol));
            if (cit == 0) accb = mfma(av, ones, accb);
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3, d = t % 3;
                const bf16x8 bv = as_bf16x8(*reinterpret_cast<const u32x4*>(
                    xs + (d * kChannels + cit * 16 + li) * kXPitch + (prow + dy) * kTile + pcol));
                acc[t] = mfma(av, bv, acc[t]);
            }
        }
    }
    // D rows are output channels cot*16 + 4 lg + e, columns input channels cit*16 + li
    float* out = part + (size_t)blockIdx.x * (9 * kChannels * kChannels + kChannels);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            out[(t * kChannels + cot * 16 + 4 * lg + e) * kChannels + cit * 16 + li] = acc[t][e];
    if (cit == 0 && li == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[9 * kChannels * kChannels + cot * 16 + 4 * lg + e] = accb[e];
    }
}

// Weight and bias gradient of a layer with one input or one output channel
// (288 weights): one thread per weight, sums over the staged tile.
// Stages a side x side block of pixels (one pixel of halo when HALO) of a
// channels-last bfloat16 tensor into LDS as floats, zero outside the image.
// With a multiple of 8 channels each thread reads whole 16-byte groups of 8
// channels; every load of a thread is issued before its values are stored.
template <int CH, int SIDE, int HALO>
__device__ inline void stage_small(const uint16_t* __restrict__ src, size_t img, const TileXY& T, int H, int W,
                                   float* __restrict__ dst) {
    if constexpr (CH % 8 == 0) {
        constexpr int G = CH / 8, NG = SIDE * SIDE * G, R = (NG + 255) / 256;
        uint4 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = threadIdx.x + r * 256;
            const int px = e / G, g = e - px * G;
            const int y = T.y0 - HALO + px / SIDE, xx = T.x0 - HALO + px % SIDE;
            v[r] = make_uint4(0u, 0u, 0u, 0u);
            if (e < NG && y >= 0 && y < H && xx >= 0 && xx < W)
                v[r] = *reinterpret_cast<const uint4*>(src + (img + (size_t)y * W + xx) * CH + 8 * g);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = threadIdx.x + r * 256;
            if (e >= NG) continue;
            float* d = dst + 8 * e;   // pixel px, channels 8 g .. 8 g + 7
            const uint32_t w[4] = {v[r].x, v[r].y, v[r].z, v[r].w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                d[2 * k] = bf2f(w[k]);
                d[2 * k + 1] = bf2f(w[k] >> 16);
            }
        }
    } else {
        constexpr int NE = SIDE * SIDE * CH, R = (NE + 255) / 256;
        float v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = threadIdx.x + r * 256;
            const int px = e / CH, ch = e - px * CH;
            const int y = T.y0 - HALO + px / SIDE, xx = T.x0 - HALO + px % SIDE;
            v[r] = (e < NE && y >= 0 && y < H && xx >= 0 && xx < W) ? bf2f(src[(img + (size_t)y * W + xx) * CH + ch])
                                                                      : 0.f;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = threadIdx.x + r * 256;
            if (e < NE) dst[e] = v[r];
        }
    }
}

template <int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad_small(const uint16_t* __restrict__ x, const uint16_t* __restrict__ dz,
                                                     int B, int H, int W, float* __restrict__ part) {
    constexpr int NW = 9 * CIN * COUT, NP = NW + COUT;
    static_assert(NP <= 512, "two entries per thread");
    __shared__ float xs[kHalo * kHalo * CIN];
    __shared__ float dzs[kTile * kTile * COUT];
    float acc[2] = {0.f, 0.f};
    const int ntiles = tiles_of(B, H, W);
    for (int tl = blockIdx.x; tl < ntiles; tl += gridDim.x) {
        const TileXY T = tile_of(tl, H, W);
        const size_t img = (size_t)T.b * H * W;
        __syncthreads();
        stage_small<CIN, kHalo, 1>(x, img, T, H, W, xs);
        stage_small<COUT, kTile, 0>(dz, img, T, H, W, dzs);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int q = threadIdx.x + k * 256;
            if (q >= NP) continue;
            float s = 0.f;
            if (q < NW) {
                const int t = q / (CIN * COUT), r = q - t * (CIN * COUT);
                const int o = r / CIN, i = r - o * CIN;
                const int dy = t / 3, dx = t % 3;
                for (int p = 0; p < kTile * kTile; ++p) {
                    const int py = p / kTile, px = p % kTile;
                    s = fmaf(dzs[p * COUT + o], xs[((py + dy) * kHalo + px + dx) * CIN + i], s);
                }
            } else {
                const int o = q - NW;
                for (int p = 0; p < kTile * kTile; ++p) s += dzs[p * COUT + o];
            }
            acc[k] += s;
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int q = threadIdx.x + k * 256;
        if (q < NP) part[(size_t)blockIdx.x * NP + q] = acc[k];
    }
}

// out[j] = sum over g of part[g][j], in double.  A workgroup takes 64
// parameters; its 16 waves take the partials g = w, w + 16, ... (each wave
// reads 64 consecutive parameters of a partial row), and the 16 wave sums are
// added in wave order, so the result is the same on every run.
constexpr int kReduceWaves = 16;

__global__ __launch_bounds__(kReduceWaves * 64) void k_reduce_parts(const float* __restrict__ part, int blocks,
                                                                   int n, float* __restrict__ out) {
    __shared__ double sh[kReduceWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (j < n) {
#pragma unroll 8
        for (int g = wave; g < blocks; g += kReduceWaves) s += (double)part[(size_t)g * n + j];
    }
    sh[wave][lane] = s;
    __syncthreads();
    if (wave != 0 || j >= n) return;
    double t = sh[0][lane];
#pragma unroll
    for (int w = 1; w < kReduceWaves; ++w) t += sh[w][lane];
    out[j] = (float)t;
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (uint16_t)f2bf(in[i]);
}

constexpr int kLossPerThread = 8;

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ x0, const float* __restrict__ tgt, int64_t n,
                                              uint16_t* __restrict__ dz, double* __restrict__ part) {
    __shared__ double sh[4];
    const float g = 2.f / (float)n;
    double s = 0.0;
    const int64_t base = (int64_t)blockIdx.x * 256 * kLossPerThread + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kLossPerThread; ++k) {
        const int64_t i = base + (int64_t)k * 256;
        if (i < n) {
            const float r = x0[i] - tgt[i];
            s += (double)r * (double)r;
            dz[i] = (uint16_t)f2bf(g * r);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int blocks, int64_t n,
                                                    double* __restrict__ loss) {
    __shared__ double sh[4];
    double s = 0.0;
    for (int g = threadIdx.x; g < blocks; g += 256) s += part[g];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = ((sh[0] + sh[1]) + (sh[2] + sh[3])) / (double)n;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, const float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                              float beta1, float beta2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = fmaf(beta1, m[i], (1.f - beta1) * g);
    const float vi = fmaf(beta2, v[i], (1.f - beta2) * g * g);
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ __launch_bounds__(256) void k_repack(const float* __restrict__ tw, int cin, int cout,
                                                uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int n = 9 * cin * cout;
    if (e >= n) return;
    const int t = e / (cin * cout), r = e - t * (cin * cout);
    const int o = r / cin, i = r - o * cin;
    const uint16_t v = (uint16_t)f2bf(tw[e]);
    wf[e] = v;
    if (wb) wb[((8 - t) * cin + i) * cout + o] = v;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs& a, hipStream_t st) {
    const int tiles = a.B * ((a.H + kTile - 1) / kTile) * ((a.W + kTile - 1) / kTile);
    const dim3 g(tiles), b(256);
    if (cin == 32 && cout == 32) {
        if (epi == EPI_RELU_BF16) hipLaunchKernelGGL((k_conv32<32, EPI_RELU_BF16>), g, b, 0, st, a);
        else if (epi == EPI_MASK_BF16) hipLaunchKernelGGL((k_conv32<32, EPI_MASK_BF16>), g, b, 0, st, a);
        else if (epi == EPI_F32) hipLaunchKernelGGL((k_conv32<32, EPI_F32>), g, b, 0, st, a);
        else return hipErrorInvalidValue;
    } else if (cin == 32 && cout == 1) {
        if (epi == EPI_RESID_F32) hipLaunchKernelGGL((k_conv32<1, EPI_RESID_F32>), g, b, 0, st, a);
        else if (epi == EPI_F32) hipLaunchKernelGGL((k_conv32<1, EPI_F32>), g, b, 0, st, a);
        else return hipErrorInvalidValue;
    } else if (cin == 1 && cout == 32) {
        if (epi == EPI_RELU_BF16) hipLaunchKernelGGL((k_conv1<EPI_RELU_BF16>), g, b, 0, st, a);
        else if (epi == EPI_MASK_BF16) hipLaunchKernelGGL((k_conv1<EPI_MASK_BF16>), g, b, 0, st, a);
        else if (epi == EPI_F32) hipLaunchKernelGGL((k_conv1<EPI_F32>), g, b, 0, st, a);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int wgrad_blocks(int B, int H, int W) {
    const int tiles = B * ((H + kTile - 1) / kTile) * ((W + kTile - 1) / kTile);
    return tiles < 512 ? tiles : 512;
}

hipError_t launch_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dz, int B, int H, int W, float* part,
                        int blocks, hipStream_t st) {
    if (blocks < 1 || blocks > kMaxWgradBlocks) return hipErrorInvalidValue;
    if (cin == 32 && cout == 32)
        hipLaunchKernelGGL(k_wgrad32, dim3(blocks), dim3(256), 0, st, x, dz, B, H, W, part);
    else if (cin == 1 && cout == 32)
        hipLaunchKernelGGL((k_wgrad_small<1, 32>), dim3(blocks), dim3(256), 0, st, x, dz, B, H, W, part);
    else if (cin == 32 && cout == 1)
        hipLaunchKernelGGL((k_wgrad_small<32, 1>), dim3(blocks), dim3(256), 0, st, x, dz, B, H, W, part);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce_parts(const float* part, int blocks, int n, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_parts, dim3((n + 63) / 64), dim3(kReduceWaves * 64), 0, st, part, blocks, n, out);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

int loss_blocks(int64_t n) { return (int)((n + 256 * kLossPerThread - 1) / (256 * kLossPerThread)); }

hipError_t launch_loss(const float* x0, const float* target, int64_t n, uint16_t* dz, double* part, hipStream_t st) {
    hipLaunchKernelGGL(k_loss, dim3(loss_blocks(n)), dim3(256), 0, st, x0, target, n, dz, part);
    return hipGetLastError();
}

hipError_t launch_loss_final(const double* part, int blocks, int64_t n, double* loss_out, hipStream_t st) {
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, blocks, n, loss_out);
    return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, theta, grad, m, v, n, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_repack(const float* theta_w, int cin, int cout, uint16_t* wf, uint16_t* wb, hipStream_t st) {
    hipLaunchKernelGGL(k_repack, dim3(blocks_for(9 * cin * cout)), dim3(256), 0, st, theta_w, cin, cout, wf, wb);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace ncs
