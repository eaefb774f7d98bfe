// Host side of the warm-start network ABI (include/ncs_cnn.h): workspace,
// the layer sequence of the forward and backward passes, Adam and the
// bfloat16 weight copies.
#include "ncs_cnn.h"
#include "cnn_internal.h"
#include "ncs_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

using namespace ncs::cnn;

namespace {

void set_err(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ncs::set_error_message(buf);
}

#define CNN_HIP(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            set_err("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);     \
            return NCS_ERR_HIP;                                                                     \
        }                                                                                           \
    } while (0)

constexpr int kCin[kNumLayers] = {1, 32, 32, 32, 32, 32};
constexpr int kCout[kNumLayers] = {32, 32, 32, 32, 32, 1};

int param_offset(int l) {   // first weight of layer l in the flat vector
    int o = 0;
    for (int k = 0; k < l; ++k) o += 9 * kCin[k] * kCout[k] + kCout[k];
    return o;
}

int weight_offset(int l) {  // first weight of layer l in the bfloat16 copies
    int o = 0;
    for (int k = 0; k < l; ++k) o += 9 * kCin[k] * kCout[k];
    return o;
}

}  // namespace

struct ncs_cnn {
    int max_batch = 0, max_h = 0, max_w = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    float* theta = nullptr;    // master parameters
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    float* grad = nullptr;
    uint16_t* wf = nullptr;    // bfloat16 weights, forward layout
    uint16_t* wb = nullptr;    // bfloat16 weights, input-gradient layout (layers 1..5)
    uint16_t* act[kNumLayers] = {};   // act[0]: input image; act[l]: ReLU output of layer l - 1
    uint16_t* dz32[2] = {};    // output gradients of the 32-channel layers (ping-pong)
    uint16_t* dz1 = nullptr;   // gradient of the network output
    float* part = nullptr;     // weight-gradient partial sums
    double* loss_part = nullptr;
    double* loss = nullptr;
    int step = 0;
    std::vector<void*> allocs;
};

namespace {

ncs_status dev_alloc(ncs_cnn* n, size_t bytes, void** p) {
    *p = nullptr;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_err("ncs_cnn: out of device memory (%zu bytes)", bytes);
        return NCS_ERR_OOM;
    }
    n->allocs.push_back(*p);
    return NCS_OK;
}

ncs_status check_net(ncs_cnn* n) {
    if (!n) {
        set_err("null network handle");
        return NCS_ERR_INVALID_ARG;
    }
    CNN_HIP(hipSetDevice(n->device));
    return NCS_OK;
}

ncs_status check_shape(const ncs_cnn* n, int32_t batch, int32_t h, int32_t w, const char* who) {
    if (batch < 1 || h < 1 || w < 1 || batch > n->max_batch || h > n->max_h || w > n->max_w) {
        set_err("%s: batch %d of %d x %d outside the workspace (max %d of %d x %d)", who, batch, h, w,
                n->max_batch, n->max_h, n->max_w);
        return NCS_ERR_INVALID_ARG;
    }
    return NCS_OK;
}

ncs_status repack_all(ncs_cnn* n) {
    for (int l = 0; l < kNumLayers; ++l) {
        CNN_HIP(launch_repack(n->theta + param_offset(l), kCin[l], kCout[l], n->wf + weight_offset(l),
                              l > 0 ? n->wb + weight_offset(l) : nullptr, n->stream));
    }
    return NCS_OK;
}

ConvArgs conv_args(const uint16_t* in, const uint16_t* w, const float* bias, const uint16_t* mask,
                   const float* resid, void* out, int B, int H, int W) {
    ConvArgs a;
    a.in = in;
    a.w = w;
    a.bias = bias;
    a.mask = mask;
    a.resid = resid;
    a.out = out;
    a.B = B;
    a.H = H;
    a.W = W;
    return a;
}

// Forward pass; keeps every stored activation for the backward pass.
ncs_status forward(ncs_cnn* n, const float* z, float* x0, int B, int H, int W) {
    const int64_t npix = (int64_t)B * H * W;
    CNN_HIP(launch_to_bf16(z, n->act[0], npix, n->stream));
    for (int l = 0; l < kNumLayers; ++l) {
        const float* bias = n->theta + param_offset(l) + 9 * kCin[l] * kCout[l];
        const uint16_t* w = n->wf + weight_offset(l);
        if (l < kNumLayers - 1) {
            CNN_HIP(launch_conv(kCin[l], kCout[l], EPI_RELU_BF16,
                                conv_args(n->act[l], w, bias, nullptr, nullptr, n->act[l + 1], B, H, W), n->stream));
        } else {
            CNN_HIP(launch_conv(kCin[l], kCout[l], EPI_RESID_F32,
                                conv_args(n->act[l], w, bias, nullptr, z, x0, B, H, W), n->stream));
        }
    }
    return NCS_OK;
}

ncs_status gradient(ncs_cnn* n, const float* z, const float* target, int B, int H, int W, float* x0_scratch) {
    ncs_status s = forward(n, z, x0_scratch, B, H, W);
    if (s) return s;
    const int64_t npix = (int64_t)B * H * W;
    const int lb = loss_blocks(npix);
    CNN_HIP(launch_loss(x0_scratch, target, npix, n->dz1, n->loss_part, n->stream));
    CNN_HIP(launch_loss_final(n->loss_part, lb, npix, n->loss, n->stream));
    const int wb = wgrad_blocks(B, H, W);
    // layer l maps act[l] to act[l + 1] (or to the output); dz is the gradient
    // at its output, already multiplied by the ReLU mask
    const uint16_t* dz = n->dz1;
    int ping = 0;
    for (int l = kNumLayers - 1; l >= 0; --l) {
        const int np = 9 * kCin[l] * kCout[l] + kCout[l];
        CNN_HIP(launch_wgrad(kCin[l], kCout[l], n->act[l], dz, B, H, W, n->part, wb, n->stream));
        CNN_HIP(launch_reduce_parts(n->part, wb, np, n->grad + param_offset(l), n->stream));
        if (l == 0) break;
        // input gradient: transposed, tap-reversed kernel (c_out -> c_in), masked by act[l] > 0
        uint16_t* dzn = n->dz32[ping];
        CNN_HIP(launch_conv(kCout[l], kCin[l], EPI_MASK_BF16,
                            conv_args(dz, n->wb + weight_offset(l), nullptr, n->act[l], nullptr, dzn, B, H, W),
                            n->stream));
        dz = dzn;
        ping ^= 1;
    }
    return NCS_OK;
}

ncs_status adam(ncs_cnn* n, float lr, float beta1, float beta2, float eps) {
    n->step += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, n->step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, n->step)));
    CNN_HIP(launch_adam(n->theta, n->grad, n->m, n->v, NCS_CNN_N_PARAMS, lr, beta1, beta2, eps, c1, c2, n->stream));
    return repack_all(n);
}

}  // namespace

extern "C" {

ncs_status ncs_cnn_create(int32_t max_batch, int32_t max_height, int32_t max_width, void* stream, ncs_cnn** out) {
    if (!out) {
        set_err("ncs_cnn_create: null output pointer");
        return NCS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (max_batch < 1 || max_height < 1 || max_width < 1 || (int64_t)max_batch * max_height * max_width > (1ll << 28)) {
        set_err("ncs_cnn_create: need positive sizes with batch x height x width <= 2^28");
        return NCS_ERR_INVALID_ARG;
    }
    static_assert(NCS_CNN_CHANNELS == kChannels && NCS_CNN_LAYERS == kNumLayers, "layer table");
    if (param_offset(kNumLayers) != NCS_CNN_N_PARAMS) {
        set_err("ncs_cnn_create: inconsistent parameter count");
        return NCS_ERR_INVALID_ARG;
    }
    ncs_cnn* n = new ncs_cnn();
    n->max_batch = max_batch;
    n->max_h = max_height;
    n->max_w = max_width;
    n->stream = (hipStream_t)stream;
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        set_err("ncs_cnn_create: no HIP device");
        return NCS_ERR_HIP;
    }
    const size_t npix = (size_t)max_batch * max_height * max_width;
    const size_t nw = (size_t)weight_offset(kNumLayers);
    void* p;
    ncs_status s = NCS_OK;
    auto A = [&](size_t bytes) -> void* {
        if (s) return nullptr;
        s = dev_alloc(n, bytes, &p);
        return p;
    };
    n->theta = (float*)A(NCS_CNN_N_PARAMS * sizeof(float));
    n->m = (float*)A(NCS_CNN_N_PARAMS * sizeof(float));
    n->v = (float*)A(NCS_CNN_N_PARAMS * sizeof(float));
    n->grad = (float*)A(NCS_CNN_N_PARAMS * sizeof(float));
    n->wf = (uint16_t*)A(nw * 2);
    n->wb = (uint16_t*)A(nw * 2);
    n->act[0] = (uint16_t*)A(npix * 2);
    for (int l = 1; l < kNumLayers; ++l) n->act[l] = (uint16_t*)A(npix * kChannels * 2);
    n->dz32[0] = (uint16_t*)A(npix * kChannels * 2);
    n->dz32[1] = (uint16_t*)A(npix * kChannels * 2);
    n->dz1 = (uint16_t*)A(npix * 2);
    n->part = (float*)A((size_t)kMaxWgradBlocks * (9 * kChannels * kChannels + kChannels) * sizeof(float));
    n->loss_part = (double*)A((size_t)loss_blocks((int64_t)npix) * sizeof(double));
    n->loss = (double*)A(sizeof(double));
    if (s) {
        ncs_cnn_destroy(n);
        return s;
    }
    // zero parameters and moments (kernels, so that nothing is a memset node)
    std::vector<float> zero(NCS_CNN_N_PARAMS, 0.f);
    ncs_status r = ncs_cnn_set_params(n, zero.data());
    if (r) {
        ncs_cnn_destroy(n);
        return r;
    }
    *out = n;
    return NCS_OK;
}

ncs_status ncs_cnn_set_params(ncs_cnn* n, const float* params_host) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!params_host) {
        set_err("ncs_cnn_set_params: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    const size_t bytes = NCS_CNN_N_PARAMS * sizeof(float);
    std::vector<float> zero(NCS_CNN_N_PARAMS, 0.f);
    CNN_HIP(hipMemcpyAsync(n->theta, params_host, bytes, hipMemcpyHostToDevice, n->stream));
    CNN_HIP(hipMemcpyAsync(n->m, zero.data(), bytes, hipMemcpyHostToDevice, n->stream));
    CNN_HIP(hipMemcpyAsync(n->v, zero.data(), bytes, hipMemcpyHostToDevice, n->stream));
    CNN_HIP(hipMemcpyAsync(n->grad, zero.data(), bytes, hipMemcpyHostToDevice, n->stream));
    n->step = 0;
    if ((s = repack_all(n))) return s;
    CNN_HIP(hipStreamSynchronize(n->stream));   // the host buffers may be released on return
    return NCS_OK;
}

ncs_status ncs_cnn_get_params(ncs_cnn* n, float* params_host) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!params_host) {
        set_err("ncs_cnn_get_params: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    CNN_HIP(hipMemcpyAsync(params_host, n->theta, NCS_CNN_N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    CNN_HIP(hipStreamSynchronize(n->stream));
    return NCS_OK;
}

ncs_status ncs_cnn_forward(ncs_cnn* n, const float* z_dev, float* x0_dev, int32_t batch, int32_t height,
                           int32_t width) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!z_dev || !x0_dev || z_dev == x0_dev) {
        set_err("ncs_cnn_forward: null or aliased pointers");
        return NCS_ERR_INVALID_ARG;
    }
    if ((s = check_shape(n, batch, height, width, "ncs_cnn_forward"))) return s;
    return forward(n, z_dev, x0_dev, batch, height, width);
}

ncs_status ncs_cnn_gradient(ncs_cnn* n, const float* z_dev, const float* target_dev, int32_t batch, int32_t height,
                            int32_t width, double* loss_host, float* grad_host) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!z_dev || !target_dev) {
        set_err("ncs_cnn_gradient: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if ((s = check_shape(n, batch, height, width, "ncs_cnn_gradient"))) return s;
    // the network output is written into the second gradient buffer (unused until
    // the backward pass of layer 4 has read it)
    float* x0 = reinterpret_cast<float*>(n->dz32[1]);
    if ((s = gradient(n, z_dev, target_dev, batch, height, width, x0))) return s;
    if (grad_host)
        CNN_HIP(hipMemcpyAsync(grad_host, n->grad, NCS_CNN_N_PARAMS * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    if (loss_host) CNN_HIP(hipMemcpyAsync(loss_host, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    if (grad_host || loss_host) CNN_HIP(hipStreamSynchronize(n->stream));
    return NCS_OK;
}

ncs_status ncs_cnn_adam_step(ncs_cnn* n, float lr, float beta1, float beta2, float eps) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f)) {
        set_err("ncs_cnn_adam_step: need lr >= 0, 0 <= beta < 1, eps > 0");
        return NCS_ERR_INVALID_ARG;
    }
    return adam(n, lr, beta1, beta2, eps);
}

ncs_status ncs_cnn_train_step(ncs_cnn* n, const float* z_dev, const float* target_dev, int32_t batch,
                              int32_t height, int32_t width, float lr, double* loss_host) {
    ncs_status s = ncs_cnn_gradient(n, z_dev, target_dev, batch, height, width, nullptr, nullptr);
    if (s) return s;
    if ((s = ncs_cnn_adam_step(n, lr, 0.9f, 0.999f, 1e-8f))) return s;
    if (loss_host) return ncs_cnn_last_loss(n, loss_host);
    return NCS_OK;
}

ncs_status ncs_cnn_last_loss(ncs_cnn* n, double* loss_host) {
    ncs_status s = check_net(n);
    if (s) return s;
    if (!loss_host) {
        set_err("ncs_cnn_last_loss: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    CNN_HIP(hipMemcpyAsync(loss_host, n->loss, sizeof(double), hipMemcpyDeviceToHost, n->stream));
    CNN_HIP(hipStreamSynchronize(n->stream));
    return NCS_OK;
}

void ncs_cnn_destroy(ncs_cnn* n) {
    if (!n) return;
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    for (void* p : n->allocs) (void)hipFree(p);
    delete n;
}

ncs_status ncs_conv3x3_bf16(const void* in_dev, const void* w_dev, const float* bias_dev, const void* mask_dev,
                            const float* resid_dev, void* out_dev, int32_t batch, int32_t height, int32_t width,
                            int32_t c_in, int32_t c_out, int32_t epilogue, void* stream) {
    if (!in_dev || !w_dev || !out_dev) {
        set_err("ncs_conv3x3_bf16: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (((uintptr_t)in_dev | (uintptr_t)w_dev | (uintptr_t)out_dev | (uintptr_t)mask_dev) % 16 != 0) {
        set_err("ncs_conv3x3_bf16: tensors must be 16-byte aligned (read in groups of 8 channels)");
        return NCS_ERR_INVALID_ARG;
    }
    if (batch < 1 || height < 1 || width < 1 || (int64_t)batch * height * width > (1ll << 28)) {
        set_err("ncs_conv3x3_bf16: bad shape %d x %d x %d", batch, height, width);
        return NCS_ERR_INVALID_ARG;
    }
    const bool shape_ok = (c_in == 1 && c_out == 32) || (c_in == 32 && c_out == 32) || (c_in == 32 && c_out == 1);
    bool epi_ok = false;
    switch (epilogue) {
        case NCS_CONV_RELU_BF16: epi_ok = c_out == 32 && bias_dev; break;
        case NCS_CONV_RESID_F32: epi_ok = c_out == 1 && bias_dev && resid_dev; break;
        case NCS_CONV_MASK_BF16: epi_ok = c_out == 32 && mask_dev; break;
        case NCS_CONV_F32: epi_ok = true; break;
        default: break;
    }
    if (!shape_ok || !epi_ok) {
        set_err("ncs_conv3x3_bf16: unsupported (c_in %d, c_out %d, epilogue %d) or missing operand", c_in, c_out,
                epilogue);
        return NCS_ERR_INVALID_ARG;
    }
    CNN_HIP(launch_conv(c_in, c_out, epilogue,
                        conv_args((const uint16_t*)in_dev, (const uint16_t*)w_dev, bias_dev, (const uint16_t*)mask_dev,
                                  resid_dev, out_dev, batch, height, width),
                        (hipStream_t)stream));
    return NCS_OK;
}

ncs_status ncs_conv3x3_wgrad_bf16(const void* x_dev, const void* dz_dev, int32_t batch, int32_t height,
                                  int32_t width, int32_t c_in, int32_t c_out, float* grad_dev, void* stream) {
    if (!x_dev || !dz_dev || !grad_dev) {
        set_err("ncs_conv3x3_wgrad_bf16: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (((uintptr_t)x_dev | (uintptr_t)dz_dev) % 16 != 0) {
        set_err("ncs_conv3x3_wgrad_bf16: x and dz must be 16-byte aligned (read in groups of 8 channels)");
        return NCS_ERR_INVALID_ARG;
    }
    if (batch < 1 || height < 1 || width < 1 || (int64_t)batch * height * width > (1ll << 28)) {
        set_err("ncs_conv3x3_wgrad_bf16: bad shape %d x %d x %d", batch, height, width);
        return NCS_ERR_INVALID_ARG;
    }
    if (!((c_in == 1 && c_out == 32) || (c_in == 32 && c_out == 32) || (c_in == 32 && c_out == 1))) {
        set_err("ncs_conv3x3_wgrad_bf16: unsupported (c_in %d, c_out %d)", c_in, c_out);
        return NCS_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const int blocks = wgrad_blocks(batch, height, width);
    const int np = 9 * c_in * c_out + c_out;
    float* part = nullptr;
    CNN_HIP(hipMalloc((void**)&part, (size_t)blocks * np * sizeof(float)));
    hipError_t e = launch_wgrad(c_in, c_out, (const uint16_t*)x_dev, (const uint16_t*)dz_dev, batch, height, width,
                                part, blocks, st);
    if (e == hipSuccess) e = launch_reduce_parts(part, blocks, np, grad_dev, st);
    const hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(part);
    CNN_HIP(e);
    CNN_HIP(se);
    return NCS_OK;
}

ncs_status ncs_to_bf16(const float* in_dev, void* out_dev, int64_t n, void* stream) {
    if ((!in_dev || !out_dev) && n > 0) {
        set_err("ncs_to_bf16: null pointer");
        return NCS_ERR_INVALID_ARG;
    }
    if (n < 0) {
        set_err("ncs_to_bf16: negative length");
        return NCS_ERR_INVALID_ARG;
    }
    CNN_HIP(launch_to_bf16(in_dev, (uint16_t*)out_dev, n, (hipStream_t)stream));
    return NCS_OK;
}

}  // extern "C"
