// Internal declarations of the warm-start network kernels (cnn_kernels.hip),
// used by the host side (cnn_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace ncs {
namespace cnn {

constexpr int kChannels = 32;       // hidden channels
constexpr int kTile = 16;           // output tile side of the convolution kernels
constexpr int kNumLayers = 6;       // 1 -> 32, 4 x (32 -> 32), 32 -> 1

// Epilogues of a convolution launch.
enum Epilogue {
    EPI_RELU_BF16 = 0,    // out = bf16(max(acc + bias, 0))
    EPI_RESID_F32 = 1,    // out = resid + acc + bias (one output channel)
    EPI_MASK_BF16 = 2,    // out = bf16(mask > 0 ? acc : 0)        (input gradient through a ReLU)
    EPI_F32 = 3,          // out = acc + bias, float
};

// One 3x3 "same" convolution over a batch of B images of H x W pixels.
// Activations are NHWC bfloat16 (stored as uint16_t), weights bfloat16
// [9][cout][cin] with tap t = 3 (dy + 1) + (dx + 1), bias float [cout].
struct ConvArgs {
    const uint16_t* in;
    const uint16_t* w;
    const float* bias;      // may be null (no bias)
    const uint16_t* mask;   // EPI_MASK_BF16: NHWC [.., cout]
    const float* resid;     // EPI_RESID_F32: [B][H][W]
    void* out;
    int B, H, W;
};

// (cin, cout) in {(1, 32), (32, 32), (32, 1)}.
hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs& a, hipStream_t st);

// Weight and bias gradient of one convolution: for every tap t,
// dw[t][o][i] = sum_p dz[p][o] x[p + o_t][i] and dbias[o] = sum_p dz[p][o],
// written as per-workgroup partial sums part[g][9 cout cin + cout]; `blocks`
// is the number of workgroups (<= max_wgrad_blocks()).
hipError_t launch_wgrad(int cin, int cout, const uint16_t* x, const uint16_t* dz, int B, int H, int W,
                        float* part, int blocks, hipStream_t st);
int wgrad_blocks(int B, int H, int W);
constexpr int kMaxWgradBlocks = 1024;

// out[j] = sum over g < blocks of part[g * n + j] (fixed order, double).
hipError_t launch_reduce_parts(const float* part, int blocks, int n, float* out, hipStream_t st);

// float -> bfloat16 (round to nearest even).
hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t st);

// Mean squared error: per-block partial sums of (x0 - t)^2 in double and the
// output gradient dz = bf16(2 (x0 - t) / n).
int loss_blocks(int64_t n);
hipError_t launch_loss(const float* x0, const float* target, int64_t n, uint16_t* dz, double* part,
                       hipStream_t st);
// loss_out[0] = (sum of the partials in a fixed order) / n
hipError_t launch_loss_final(const double* part, int blocks, int64_t n, double* loss_out, hipStream_t st);

// Adam on FP32 master parameters; c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
hipError_t launch_adam(float* theta, const float* grad, float* m, float* v, int n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st);

// bfloat16 copies of one layer's weights from the master vector: forward
// layout wf[t][o][i] and, when wb is non-null, the input-gradient layout
// wb[8 - t][i][o] (the transposed, tap-reversed kernel).
hipError_t launch_repack(const float* theta_w, int cin, int cout, uint16_t* wf, uint16_t* wb, hipStream_t st);

}  // namespace cnn
}  // namespace ncs
