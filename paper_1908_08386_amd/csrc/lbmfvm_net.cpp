// Host runtime of the learned initial guess: layer geometry, workspace
// layout, and the launch sequences of the forward pass, the backward pass
// and Adam.  All arithmetic runs in the kernels of k_net.hip.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "lf_host.h"
#include "lf_net_internal.h"

namespace {

struct Layer {
  lf::ConvGeom g1;   // geometry for batch 1 (n is set per call)
  int up;            // input is the x2 upsampling of the previous activation
  int skip;          // index of the encoder activation added after SiLU, or -1
  long long w_off;   // offset of the weights in the flat parameters (floats)
  size_t off_wb, off_wt, off_z, off_a, off_u;  // workspace offsets (bytes)
};

constexpr int kLayers = 10;

}  // namespace

struct lf_net {
  lf_ctx* ctx;
  lf_net_desc d;
  Layer L[kLayers];
  long long nparam;
  size_t off_w, off_m, off_v, off_g, off_x0, off_dx, off_dz[2], off_sg[4], off_part, off_mse,
      off_loss, total;
  size_t part_floats;  // capacity of the weight-gradient split partials
  uint8_t* ws;
  size_t ws_bytes;
  int t;           // Adam steps taken
  int last_batch;  // batch of the last forward pass
};

namespace {

lf::ConvGeom at_batch(const Layer& l, int n) {
  lf::ConvGeom g = l.g1;
  g.n = n;
  return g;
}

template <typename T>
T* P(lf_net* net, size_t off) {
  return (T*)(net->ws + off);
}

lf_status layout(lf_net* net) {
  const lf_net_desc& d = net->d;
  const int R = d.res, B = d.max_batch;
  const int* w = d.widths;
  // (Cout, Cin, stride, up, input size)
  const int co[kLayers] = {w[0], w[1], w[2], w[3], w[4], w[3], w[2], w[1], w[0], d.cout};
  const int ci[kLayers] = {d.cin, w[0], w[1], w[2], w[3], w[4], w[3], w[2], w[1], w[0]};
  const int st[kLayers] = {1, 2, 2, 2, 2, 1, 1, 1, 1, 1};
  const int up[kLayers] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 0};
  const int in[kLayers] = {R, R, R / 2, R / 4, R / 8, R / 8, R / 4, R / 2, R, R};
  const int sk[kLayers] = {-1, -1, -1, -1, -1, 3, 2, 1, 0, -1};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += lf_align_up(bytes, 256);
    return r;
  };
  long long np = 0;
  for (int l = 0; l < kLayers; ++l) {
    Layer& Ly = net->L[l];
    Ly.g1.n = 1;
    Ly.g1.H = Ly.g1.W = in[l];
    Ly.g1.Ho = Ly.g1.Wo = in[l] / st[l];
    Ly.g1.Cin = ci[l];
    Ly.g1.Cout = co[l];
    Ly.g1.stride = st[l];
    Ly.up = up[l];
    Ly.skip = sk[l];
    Ly.w_off = np;
    np += (long long)co[l] * 9 * ci[l] + co[l];
  }
  net->nparam = np;
  net->off_w = take(np * 4);
  net->off_m = take(np * 4);
  net->off_v = take(np * 4);
  net->off_g = take(np * 4);
  net->off_x0 = take((size_t)B * R * R * d.cin * 2);
  size_t dx_max = 0, dz_max = 0, part_max = 0;
  for (int l = 0; l < kLayers; ++l) {
    Layer& Ly = net->L[l];
    const lf::ConvGeom g = at_batch(Ly, B);
    const size_t out_px = (size_t)B * g.Ho * g.Wo;
    Ly.off_wb = take((size_t)g.Cout * 9 * g.Cin * 2);
    Ly.off_wt = take((size_t)g.Cout * 9 * g.Cin * 2);
    Ly.off_z = take(out_px * g.Cout * 4);
    Ly.off_a = l < kLayers - 1 ? take(out_px * g.Cout * 2) : 0;
    Ly.off_u = Ly.up ? take((size_t)B * g.H * g.W * g.Cin * 2) : 0;
    if (l > 0) dx_max = dx_max > (size_t)B * g.H * g.W * g.Cin ? dx_max : (size_t)B * g.H * g.W * g.Cin;
    dz_max = dz_max > out_px * g.Cout ? dz_max : out_px * g.Cout;
    const size_t pf = lf::conv_bwd_weight_part_floats(g);
    part_max = part_max > pf ? part_max : pf;
  }
  net->off_dx = take(dx_max * 4);
  net->off_dz[0] = take(dz_max * 2);
  net->off_dz[1] = take(dz_max * 2);
  for (int k = 0; k < 4; ++k) {
    const lf::ConvGeom g = at_batch(net->L[k], B);  // e_k has the shape of layer k's output
    net->off_sg[k] = take((size_t)B * g.Ho * g.Wo * g.Cout * 4);
  }
  net->off_part = take(part_max * 4);
  net->part_floats = part_max;
  net->off_mse = take(lf::net_mse_part_doubles(B, R) * 8);
  net->off_loss = take(256);
  net->total = o;
  return LF_OK;
}

lf_status check_ready(const lf_net* net) {
  if (!net) return lf_fail(LF_EINVAL, "NULL net");
  if (!net->ws) return lf_fail(LF_EWORKSPACE, "no workspace bound");
  return LF_OK;
}

lf_status convert_weights(lf_net* net) {
  hipStream_t s = net->ctx->stream;
  for (int l = 0; l < kLayers; ++l) {
    const Layer& Ly = net->L[l];
    LF_HIP_TRY(lf::launch_weights_bf16(P<float>(net, net->off_w) + Ly.w_off, Ly.g1.Cout,
                                       Ly.g1.Cin, P<uint16_t>(net, Ly.off_wb),
                                       P<uint16_t>(net, Ly.off_wt), s));
  }
  return LF_OK;
}

lf_status forward_impl(lf_net* net, const float* feat, const int* idx, int B) {
  hipStream_t s = net->ctx->stream;
  const int R = net->d.res;
  LF_HIP_TRY(lf::launch_net_inputs(feat, idx, B, R, P<uint16_t>(net, net->off_x0), s));
  for (int l = 0; l < kLayers; ++l) {
    const Layer& Ly = net->L[l];
    const lf::ConvGeom g = at_batch(Ly, B);
    const uint16_t* x;
    if (l == 0) {
      x = P<uint16_t>(net, net->off_x0);
    } else if (Ly.up) {
      const Layer& prev = net->L[l - 1];
      LF_HIP_TRY(lf::launch_upsample2(P<uint16_t>(net, prev.off_a), B, prev.g1.Ho, prev.g1.Wo,
                                      prev.g1.Cout, P<uint16_t>(net, Ly.off_u), s));
      x = P<uint16_t>(net, Ly.off_u);
    } else {
      x = P<uint16_t>(net, net->L[l - 1].off_a);
    }
    const float* bias = P<float>(net, net->off_w) + Ly.w_off + (long long)g.Cout * 9 * g.Cin;
    const uint16_t* skip = Ly.skip >= 0 ? P<uint16_t>(net, net->L[Ly.skip].off_a) : nullptr;
    const bool last = l == kLayers - 1;
    LF_HIP_TRY(lf::launch_conv_fwd(g, x, P<uint16_t>(net, Ly.off_wb), bias, skip,
                                   P<float>(net, Ly.off_z),
                                   last ? nullptr : P<uint16_t>(net, Ly.off_a), last ? 0 : 1, s));
  }
  net->last_batch = B;
  return LF_OK;
}

lf_status backward_impl(lf_net* net, const float* target, const int* idx, int B, float* loss) {
  hipStream_t s = net->ctx->stream;
  const int R = net->d.res;
  int cur = 0;
  const Layer& head = net->L[kLayers - 1];
  LF_HIP_TRY(lf::launch_mse(P<float>(net, head.off_z), head.g1.Cout, target, idx, B, R,
                            P<uint16_t>(net, net->off_dz[cur]), P<double>(net, net->off_mse),
                            loss, s));
  for (int l = kLayers - 1; l >= 0; --l) {
    const Layer& Ly = net->L[l];
    const lf::ConvGeom g = at_batch(Ly, B);
    const uint16_t* x = l == 0 ? P<uint16_t>(net, net->off_x0)
                        : Ly.up ? P<uint16_t>(net, Ly.off_u)
                                : P<uint16_t>(net, net->L[l - 1].off_a);
    const uint16_t* dz = P<uint16_t>(net, net->off_dz[cur]);
    LF_HIP_TRY(lf::launch_conv_bwd_weight(g, x, dz, P<float>(net, net->off_part),
                                          net->part_floats, P<float>(net, net->off_g) + Ly.w_off,
                                          s));
    if (l == 0) break;
    LF_HIP_TRY(lf::launch_conv_bwd_data(g, dz, P<uint16_t>(net, Ly.off_wt),
                                        P<float>(net, net->off_dx), s));
    // gradient of the previous layer's output, then of its pre-activation
    const Layer& prev = net->L[l - 1];
    const float* add = (l >= 1 && l <= 4) ? P<float>(net, net->off_sg[l - 1]) : nullptr;
    float* keep = (l >= 6) ? P<float>(net, net->off_sg[kLayers - 1 - l]) : nullptr;
    LF_HIP_TRY(lf::launch_act_grad(P<float>(net, net->off_dx), Ly.up, add,
                                   P<float>(net, prev.off_z), B, prev.g1.Ho, prev.g1.Wo,
                                   prev.g1.Cout, P<uint16_t>(net, net->off_dz[cur ^ 1]), keep,
                                   s));
    cur ^= 1;
  }
  return LF_OK;
}

lf_status check_batch(const lf_net* net, int batch) {
  if (batch < 1 || batch > net->d.max_batch)
    return lf_fail(LF_EINVAL, "batch %d outside 1..%d", batch, net->d.max_batch);
  return LF_OK;
}

}  // namespace

extern "C" {

lf_status lf_net_create(lf_ctx* ctx, const lf_net_desc* d, lf_net** out) {
  if (!ctx || !d || !out) return lf_fail(LF_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->res < 16 || d->res % 16) return lf_fail(LF_EINVAL, "res must be a multiple of 16");
  if (d->cin != 8 || d->cout < 8 || d->cout % 8)
    return lf_fail(LF_EINVAL, "cin must be 8 and cout a multiple of 8");
  for (int k = 0; k < 5; ++k)
    if (d->widths[k] < 8 || d->widths[k] % 8) return lf_fail(LF_EINVAL, "widths: multiples of 8");
  if (d->max_batch < 1) return lf_fail(LF_EINVAL, "max_batch < 1");
  if ((long long)d->max_batch * d->res * d->res * 128 > (1LL << 31))
    return lf_fail(LF_EINVAL, "max_batch * res^2 too large");
  lf_net* net = new (std::nothrow) lf_net();
  if (!net) return lf_fail(LF_ENOMEM, "host allocation");
  net->ctx = ctx;
  net->d = *d;
  net->ws = nullptr;
  net->ws_bytes = 0;
  net->t = 0;
  net->last_batch = 0;
  layout(net);
  *out = net;
  return LF_OK;
}

lf_status lf_net_destroy(lf_net* net) {
  delete net;
  return LF_OK;
}

lf_status lf_net_param_count(const lf_net* net, int64_t* n) {
  if (!net || !n) return lf_fail(LF_EINVAL, "NULL argument");
  *n = net->nparam;
  return LF_OK;
}

lf_status lf_net_workspace_bytes(const lf_net* net, size_t* bytes) {
  if (!net || !bytes) return lf_fail(LF_EINVAL, "NULL argument");
  *bytes = net->total;
  return LF_OK;
}

lf_status lf_net_bind_workspace(lf_net* net, void* p, size_t bytes) {
  if (!net || !p) return lf_fail(LF_EINVAL, "NULL argument");
  if (bytes < net->total) return lf_fail(LF_EWORKSPACE, "workspace %zu < %zu", bytes, net->total);
  if ((uintptr_t)p % 256) return lf_fail(LF_EWORKSPACE, "workspace not 256-byte aligned");
  net->ws = (uint8_t*)p;
  net->ws_bytes = bytes;
  return LF_OK;
}

lf_status lf_net_set_weights(lf_net* net, const float* host, int64_t n) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (!host || n != net->nparam) return lf_fail(LF_EINVAL, "need %lld weights", net->nparam);
  hipStream_t s = net->ctx->stream;
  LF_HIP_TRY(hipMemcpyAsync(net->ws + net->off_w, host, n * 4, hipMemcpyHostToDevice, s));
  LF_HIP_TRY(hipMemsetAsync(net->ws + net->off_m, 0, n * 4, s));
  LF_HIP_TRY(hipMemsetAsync(net->ws + net->off_v, 0, n * 4, s));
  LF_HIP_TRY(hipMemsetAsync(net->ws + net->off_g, 0, n * 4, s));
  net->t = 0;
  st = convert_weights(net);
  if (st != LF_OK) return st;
  LF_HIP_TRY(hipStreamSynchronize(s));
  return LF_OK;
}

static lf_status get_flat(lf_net* net, size_t off, float* host, int64_t n) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (!host || n != net->nparam) return lf_fail(LF_EINVAL, "need %lld values", net->nparam);
  hipStream_t s = net->ctx->stream;
  LF_HIP_TRY(hipMemcpyAsync(host, net->ws + off, n * 4, hipMemcpyDeviceToHost, s));
  LF_HIP_TRY(hipStreamSynchronize(s));
  return LF_OK;
}

lf_status lf_net_get_weights(lf_net* net, float* host, int64_t n) {
  return get_flat(net, net ? net->off_w : 0, host, n);
}

lf_status lf_net_get_grads(lf_net* net, float* host, int64_t n) {
  return get_flat(net, net ? net->off_g : 0, host, n);
}

lf_status lf_net_forward(lf_net* net, const float* feat, const int* idx, int batch, float* pred) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (!feat) return lf_fail(LF_EINVAL, "NULL feat");
  if ((st = check_batch(net, batch)) != LF_OK) return st;
  if ((st = forward_impl(net, feat, idx, batch)) != LF_OK) return st;
  if (pred) {
    const Layer& head = net->L[kLayers - 1];
    LF_HIP_TRY(lf::launch_unpack_pred(P<float>(net, head.off_z), head.g1.Cout, batch,
                                      net->d.res, pred, net->ctx->stream));
  }
  return LF_OK;
}

lf_status lf_net_get_output(lf_net* net, float* host, size_t n) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  const Layer& head = net->L[kLayers - 1];
  const size_t need = (size_t)net->last_batch * net->d.res * net->d.res * head.g1.Cout;
  if (!host || n != need) return lf_fail(LF_EINVAL, "need %zu values", need);
  hipStream_t s = net->ctx->stream;
  LF_HIP_TRY(hipMemcpyAsync(host, net->ws + head.off_z, need * 4, hipMemcpyDeviceToHost, s));
  LF_HIP_TRY(hipStreamSynchronize(s));
  return LF_OK;
}

lf_status lf_net_backward(lf_net* net, const float* feat, const float* target, const int* idx,
                          int batch, float* loss) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (!feat || !target) return lf_fail(LF_EINVAL, "NULL feat or target");
  if ((st = check_batch(net, batch)) != LF_OK) return st;
  if ((st = forward_impl(net, feat, idx, batch)) != LF_OK) return st;
  return backward_impl(net, target, idx, batch, loss);
}

lf_status lf_net_adam(lf_net* net, float lr) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (!(lr >= 0.f)) return lf_fail(LF_EINVAL, "lr < 0");
  const double b1 = 0.9, b2 = 0.999;
  net->t += 1;
  const float c1 = (float)(1.0 / (1.0 - pow(b1, net->t)));
  const float c2 = (float)(1.0 / (1.0 - pow(b2, net->t)));
  LF_HIP_TRY(lf::launch_adam(P<float>(net, net->off_w), P<float>(net, net->off_m),
                             P<float>(net, net->off_v), P<float>(net, net->off_g), net->nparam,
                             lr, (float)b1, (float)b2, 1e-8f, c1, c2, net->ctx->stream));
  return convert_weights(net);
}

lf_status lf_net_train_step(lf_net* net, const float* feat, const float* target, const int* idx,
                            int batch, float lr, float* loss) {
  lf_status st = lf_net_backward(net, feat, target, idx, batch, loss);
  return st != LF_OK ? st : lf_net_adam(net, lr);
}

lf_status lf_net_flops(const lf_net* net, double* fwd, double* train) {
  if (!net || !fwd || !train) return lf_fail(LF_EINVAL, "NULL argument");
  double f = 0.0, t = 0.0;
  for (int l = 0; l < kLayers; ++l) {
    const lf::ConvGeom& g = net->L[l].g1;
    const double mac = (double)g.Ho * g.Wo * g.Cout * 9.0 * g.Cin;
    f += 2.0 * mac;
    t += 2.0 * mac * (l == 0 ? 2.0 : 3.0);  // no input gradient for the first layer
  }
  *fwd = f;
  *train = t;
  return LF_OK;
}

lf_status lf_net_profile_train(lf_net* net, const float* feat, const float* target,
                               const int* idx, int batch, float lr, int nsteps, double* avg_ms) {
  lf_status st = check_ready(net);
  if (st != LF_OK) return st;
  if (nsteps < 1 || !avg_ms) return lf_fail(LF_EINVAL, "nsteps < 1 or NULL avg_ms");
  hipStream_t s = net->ctx->stream;
  hipEvent_t e0, e1;
  LF_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return lf_fail(LF_EDEVICE, "hipEventCreate");
  }
  float ms = 0.f;
  hipError_t e = hipEventRecord(e0, s);
  for (int k = 0; k < nsteps && e == hipSuccess && st == LF_OK; ++k)
    st = lf_net_train_step(net, feat, target, idx, batch, lr, nullptr);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LF_OK) return st;
  if (e != hipSuccess) return lf_fail(LF_EDEVICE, "%s", hipGetErrorString(e));
  *avg_ms = ms / nsteps;
  return LF_OK;
}

lf_status lf_resample(lf_ctx* ctx, const void* src, int src_is_f64, int snx, int sny,
                      int64_t src_row_stride, void* dst, int dst_is_f64, int dnx, int dny,
                      double scale, double offset, int flags) {
  if (!ctx || !src || !dst) return lf_fail(LF_EINVAL, "NULL argument");
  if (snx < 1 || sny < 1 || dnx < 1 || dny < 1 || src_row_stride < snx)
    return lf_fail(LF_EINVAL, "bad sizes");
  if (flags & ~LF_RESAMPLE_ANTISYM) return lf_fail(LF_EINVAL, "unknown flags %d", flags);
  LF_HIP_TRY(lf::launch_resample(src, src_is_f64, snx, sny, src_row_stride, dst, dst_is_f64, dnx,
                                 dny, scale, offset, flags & LF_RESAMPLE_ANTISYM, ctx->stream));
  return LF_OK;
}

}  // extern "C"
