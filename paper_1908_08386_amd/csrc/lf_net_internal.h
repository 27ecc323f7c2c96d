// Internal interface between the network runtime (lbmfvm_net.cpp) and the
// network kernels (k_net.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

// Geometry of one 3x3 convolution (zero padding 1).  H, W: spatial size of
// the convolution's input (after any upsampling); Ho = H / stride.  Channel
// counts are multiples of 8.  Tensors are NHWC.
struct ConvGeom {
  int n, H, W, Ho, Wo, Cin, Cout, stride;
};

// z = conv(x, w) + bias; if z32 != null it receives z; if a16 != null it
// receives act(z) (+ skip), rounded to bfloat16.  act: 1 SiLU, 0 identity.
// x: bf16 [n][H][W][Cin]; w: bf16 [Cout][9][Cin].
hipError_t launch_conv_fwd(const ConvGeom& g, const uint16_t* x, const uint16_t* w,
                           const float* bias, const uint16_t* skip, float* z32,
                           uint16_t* a16, int act, hipStream_t s);
// dx[n][H][W][Cin] (FP32) = input gradient for dz (bf16 [n][Ho][Wo][Cout])
// with the transposed weights wt: bf16 [9][Cin][Cout].
hipError_t launch_conv_bwd_data(const ConvGeom& g, const uint16_t* dz, const uint16_t* wt,
                                float* dx, hipStream_t s);
// Weight and bias gradients: grad_w [Cout][9][Cin] and grad_b [Cout] (FP32,
// contiguous: bias right after the weights).  part: split-K partials,
// part_floats long; conv_bwd_weight_part_floats(g) is enough for every batch
// size of g's layer (hipErrorInvalidValue, and nothing launched, if short).
size_t conv_bwd_weight_part_floats(const ConvGeom& g);
hipError_t launch_conv_bwd_weight(const ConvGeom& g, const uint16_t* x, const uint16_t* dz,
                                  float* part, size_t part_floats, float* grad_wb,
                                  hipStream_t s);

// Network inputs from per-sample features (log10 Ra, Pr, A): bf16
// [n][R][R][8]; idx (or null for 0..n-1) selects rows of feat.
hipError_t launch_net_inputs(const float* feat, const int* idx, int n, int R, uint16_t* x,
                             hipStream_t s);
// out[n][2h][2w][C] = nearest x2 upsampling of in[n][h][w][C] (bf16).
hipError_t launch_upsample2(const uint16_t* in, int n, int h, int w, int C, uint16_t* out,
                            hipStream_t s);
// da = (pool ? 2x2 sum of dx : dx) + add (add may be null); dz = da * act'(z)
// as bf16; da_out (may be null) receives da.  Sizes are those of z: n*h*w*C.
hipError_t launch_act_grad(const float* dx, int pool, const float* add, const float* z, int n,
                           int h, int w, int C, uint16_t* dz, float* da_out, hipStream_t s);
// Loss over the first 3 channels of y [n][R][R][C] against target planes
// [N][3][R][R] (rows selected by idx or 0..n-1): dz = dL/dy as bf16 (zero on
// channels >= 3); loss_out (device float, may be null) = mean squared error.
// part: at least net_mse_part_doubles(n, R) doubles.
size_t net_mse_part_doubles(int n, int R);
hipError_t launch_mse(const float* y, int C, const float* target, const int* idx, int n, int R,
                      uint16_t* dz, double* part, float* loss_out, hipStream_t s);
// y [n][R][R][C] (channels 0..2) -> planes [n][3][R][R].
hipError_t launch_unpack_pred(const float* y, int C, int n, int R, float* planes, hipStream_t s);
// Adam update of w, m, v from g (count elements); c1 = 1 / (1 - beta1^t),
// c2 = 1 / (1 - beta2^t).
hipError_t launch_adam(float* w, float* m, float* v, const float* g, long long count, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t s);
// Per layer: bf16 copies wb [Cout][9][Cin] and wt [9][Cin][Cout] of the FP32
// weights w [Cout][9][Cin].
hipError_t launch_weights_bf16(const float* w, int Cout, int Cin, uint16_t* wb, uint16_t* wt,
                               hipStream_t s);
// Bilinear resampling of a cell-centred field (see lf_resample).
hipError_t launch_resample(const void* src, int src_f64, int snx, int sny, long long sstride,
                           void* dst, int dst_f64, int dnx, int dny, double scale,
                           double offset, int antisym, hipStream_t s);

}  // namespace lf
