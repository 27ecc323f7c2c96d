// Kernels of the learned initial guess: 3x3 convolutions as implicit GEMMs
// on the bf16 matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the forward pass and both backward passes, plus the
// element-wise pieces (inputs, upsampling, activation gradient, MSE, Adam,
// weight conversion) and the bilinear resampling between the network's
// canvas and a cavity grid.
//
// GEMM views (K is walked in chunks of 32 = four groups of 8 channels, so
// every lane loads 16 contiguous bytes of an NHWC tensor):
//   forward      M = output pixels, N = Cout, K = 9 taps x Cin
//   input grad   M = input pixels,  N = Cin,  K = 9 taps x Cout
//   weight grad  M = Cout, N = 9 taps x Cin (+ one group whose first column
//                is the constant 1, giving the bias gradient), K = output
//                pixels, split over blocks and summed in a fixed order.
#include "lf_net_internal.h"

namespace lf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  // round to nearest, ties to even (inputs here are finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

enum { FWD = 0, BWD_DATA = 1, BWD_WEIGHT = 2 };
constexpr int BK = 32;        // K per matrix-core step
constexpr int LDK = BK + 8;   // LDS row stride in elements (80 bytes)

struct ConvArgs {
  ConvGeom g;
  const uint16_t* x;     // convolution input (forward, weight grad)
  const uint16_t* w;     // forward: [Cout][9][Cin]; input grad: [9][Cin][Cout]
  const uint16_t* dz;    // output gradient (input grad, weight grad)
  const float* bias;
  const uint16_t* skip;
  float* z32;
  uint16_t* a16;
  float* out;            // input grad: dx; weight grad: split partials
  int act;
  int M, N, nchunks, cps;  // cps: K chunks per split
};

template <int MODE, int BM, int BN>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2 * BM * LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2 * BN * LDK];
  const ConvGeom& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
  const int wm0 = (wave >> 1) * WM, wn0 = (wave & 1) * WN;
  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int kc0 = blockIdx.z * a.cps;
  const int kc1 = min(a.nchunks, kc0 + a.cps);
  const int CK = MODE == FWD ? g.Cin : g.Cout;  // channels along K (FWD, BWD_DATA)
  const int cg = CK >> 3, G = 9 * cg;
  const int P = g.n * g.Ho * g.Wo;              // output pixels (BWD_WEIGHT)

  // Everything a thread's loads depend on apart from the K chunk is worked
  // out once: its tile rows' pixel coordinates and, along K, the tap and
  // channel group it is at (advanced by four groups per chunk).
  constexpr int AV = BM * 4 / 256;  // A vectors per thread (FWD / BWD_DATA; BWD_WEIGHT too)
  static_assert(BM % 64 == 0 && BK == 32, "loader lanes assume 64-row A tiles, 32-wide K");
  static_assert(MODE != BWD_WEIGHT || BN <= 64, "one B vector per thread");
  const int q = tid & 3, rq = tid >> 2;   // FWD / BWD_DATA: K quarter and first A row
  const int pl = tid % BK, grp = tid / BK;  // BWD_WEIGHT: pixel in the chunk, 8-row group
  int pb[AV], p1[AV], p2[AV];
  bool pok[AV];
  if (MODE != BWD_WEIGHT) {
#pragma unroll
    for (int k = 0; k < AV; ++k) {
      const int m = m0 + rq + 64 * k;
      pok[k] = m < a.M;
      const int W = MODE == FWD ? g.Wo : g.W, hw = (MODE == FWD ? g.Ho : g.H) * W;
      const int mm = pok[k] ? m : 0;
      pb[k] = mm / hw;
      const int rm = mm - pb[k] * hw;
      p1[k] = rm / W;            // FWD: oy; BWD_DATA: y
      p2[k] = rm - p1[k] * W;    // FWD: ox; BWD_DATA: x
    }
  } else {
    // pixel kc0 * BK + pl, advanced by BK per chunk
    const int p = kc0 * BK + pl, hw = g.Ho * g.Wo;
    pb[0] = p / hw;
    const int rm = p - pb[0] * hw;
    p1[0] = rm / g.Wo;
    p2[0] = rm - p1[0] * g.Wo;
    pok[0] = true;
  }
  int gi = kc0 * 4 + q;          // K group of this thread's quarter
  int tap = gi / cg, cgp = gi - tap * cg;
  // BWD_WEIGHT: the B rows' tap and channel group are fixed
  const int bn8 = n0 + grp * 8;
  const int wtap = bn8 / g.Cin, wci0 = bn8 - wtap * g.Cin;
  const int wky = wtap / 3, wkx = wtap - wky * 3;

  // A chunk is staged in registers (ra, rb) from global memory, then stored
  // to one of two LDS buffers: the loads of chunk k + 1 are in flight while
  // the matrix cores work on chunk k, and one barrier per chunk suffices
  // (the buffer a store overwrites was last read before the previous
  // barrier).
  constexpr int BV = MODE == BWD_WEIGHT ? 1 : (BN * 4 + 255) / 256;  // B vectors per thread
  uint4 ra[AV], rb[BV];
  auto load_chunk = [&](int kc) {
    if (MODE != BWD_WEIGHT) {
      const bool gok = gi < G;
      const int ky = tap >= 6 ? 2 : (tap >= 3 ? 1 : 0), kx = tap - 3 * ky, c0 = cgp << 3;
#pragma unroll
      for (int k = 0; k < AV; ++k) {
        uint4 val = {0u, 0u, 0u, 0u};
        if (gok && pok[k]) {
          if (MODE == FWD) {
            const int iy = p1[k] * g.stride + ky - 1, ix = p2[k] * g.stride + kx - 1;
            if (iy >= 0 && iy < g.H && ix >= 0 && ix < g.W)
              val = *(const uint4*)(a.x + ((size_t)(pb[k] * g.H + iy) * g.W + ix) * g.Cin + c0);
          } else {
            const int ty = p1[k] + 1 - ky, tx = p2[k] + 1 - kx;  // = stride * output index
            const bool even = g.stride == 1 || (((ty | tx) & 1) == 0);
            if (ty >= 0 && tx >= 0 && even) {
              const int oy = g.stride == 1 ? ty : ty >> 1, ox = g.stride == 1 ? tx : tx >> 1;
              if (oy < g.Ho && ox < g.Wo)
                val = *(const uint4*)(a.dz + ((size_t)(pb[k] * g.Ho + oy) * g.Wo + ox) * g.Cout + c0);
            }
          }
        }
        ra[k] = val;
      }
#pragma unroll
      for (int k = 0; k < BV; ++k) {
        const int v = tid + 256 * k, r = v >> 2, nn = n0 + r;  // v & 3 == q
        uint4 val = {0u, 0u, 0u, 0u};
        if (v < BN * 4 && gok && nn < a.N) {
          if (MODE == FWD)
            val = *(const uint4*)(a.w + ((size_t)nn * 9 + tap) * g.Cin + c0);
          else
            val = *(const uint4*)(a.w + ((size_t)tap * g.Cin + nn) * g.Cout + c0);
        }
        rb[k] = val;
      }
      gi += 4;
      cgp += 4;
      while (cgp >= cg) {
        cgp -= cg;
        ++tap;
      }
    } else {
      // K = output pixels: 16-byte loads along channels
      const bool pin = kc * BK + pl < P;
#pragma unroll
      for (int k = 0; k < AV; ++k) {
        const int gk = grp + (256 / BK) * k, co0 = m0 + gk * 8;
        uint4 val = {0u, 0u, 0u, 0u};
        if (pin && co0 < g.Cout)
          val = *(const uint4*)(a.dz + (size_t)(kc * BK + pl) * g.Cout + co0);
        ra[k] = val;
      }
      uint4 val = {0u, 0u, 0u, 0u};
      if (tid < (BN / 8) * BK && pin) {
        if (bn8 < 9 * g.Cin) {
          const int iy = p1[0] * g.stride + wky - 1, ix = p2[0] * g.stride + wkx - 1;
          if (iy >= 0 && iy < g.H && ix >= 0 && ix < g.W)
            val = *(const uint4*)(a.x + ((size_t)(pb[0] * g.H + iy) * g.W + ix) * g.Cin + wci0);
        } else if (bn8 == 9 * g.Cin) {
          val.x = 0x3F80u;  // bf16 1.0 in the first column: the bias gradient
        }
      }
      rb[0] = val;
      // next chunk's pixel
      p2[0] += BK;
      while (p2[0] >= g.Wo) {
        p2[0] -= g.Wo;
        if (++p1[0] == g.Ho) {
          p1[0] = 0;
          ++pb[0];
        }
      }
    }
  };
  auto store_chunk = [&](int buf) {
    uint16_t* A = As + buf * BM * LDK;
    uint16_t* B = Bs + buf * BN * LDK;
    if (MODE != BWD_WEIGHT) {
#pragma unroll
      for (int k = 0; k < AV; ++k) *(uint4*)&A[(rq + 64 * k) * LDK + q * 8] = ra[k];
#pragma unroll
      for (int k = 0; k < BV; ++k) {
        const int v = tid + 256 * k;
        if (v < BN * 4) *(uint4*)&B[(v >> 2) * LDK + q * 8] = rb[k];
      }
    } else {
      // transposed into LDS (K = pixels along the rows' inner dimension)
#pragma unroll
      for (int k = 0; k < AV; ++k) {
        const int gk = grp + (256 / BK) * k;
        const uint16_t* e = (const uint16_t*)&ra[k];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) A[(gk * 8 + jj) * LDK + pl] = e[jj];
      }
      if (tid < (BN / 8) * BK) {
        const uint16_t* e = (const uint16_t*)&rb[0];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) B[(grp * 8 + jj) * LDK + pl] = e[jj];
      }
    }
  };
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  auto compute = [&](int buf) {
    const uint16_t* A = As + buf * BM * LDK;
    const uint16_t* B = Bs + buf * BN * LDK;
    bf16x8 av[FM], bv[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) av[i] = *(const bf16x8*)&A[(wm0 + i * 16 + lr) * LDK + lk];
#pragma unroll
    for (int j = 0; j < FN; ++j) bv[j] = *(const bf16x8*)&B[(wn0 + j * 16 + lr) * LDK + lk];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
  };
  if (kc0 < kc1) {
    load_chunk(kc0);
    store_chunk(0);
  }
  __syncthreads();
  int buf = 0;
  for (int kc = kc0; kc < kc1; ++kc) {
    const bool more = kc + 1 < kc1;
    if (more) load_chunk(kc + 1);
    compute(buf);
    if (more) store_chunk(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // accumulator element r of block (i, j): row 4 * (lane / 16) + r, column lane % 16
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        const int nn = n0 + wn0 + j * 16 + (lane & 15);
        if (m >= a.M || nn >= a.N) continue;
        const float c = acc[i][j][r];
        if (MODE == FWD) {
          const float zv = c + a.bias[nn];
          const size_t o = (size_t)m * g.Cout + nn;
          if (a.z32) a.z32[o] = zv;
          if (a.a16) {
            float v = a.act ? silu(zv) : zv;
            if (a.skip) v += from_bf16(a.skip[o]);
            a.a16[o] = to_bf16(v);
          }
        } else if (MODE == BWD_DATA) {
          a.out[(size_t)m * g.Cin + nn] = c;
        } else {
          a.out[((size_t)blockIdx.z * g.Cout + m) * a.N + nn] = c;
        }
      }
}

// Sum of the split partials in split order; weights then bias.  The loads
// of 16 splits are issued before their additions (which stay in split
// order), so a thread waits for one round trip per 16 partials.
__global__ __launch_bounds__(64) void k_wgrad_reduce(const float* __restrict__ part, int splits,
                                                     int Cout, int K9, int N,
                                                     float* __restrict__ grad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Cout * (K9 + 1)) return;
  const int co = i / (K9 + 1), col = i - co * (K9 + 1);
  const size_t zs = (size_t)Cout * N;
  const float* p = part + (size_t)co * N + col;
  float s = 0.f;
  int z = 0;
  for (; z + 16 <= splits; z += 16) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = p[(size_t)(z + k) * zs];
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
  }
  for (; z < splits; ++z) s += p[(size_t)z * zs];
  if (col < K9) grad[(size_t)co * K9 + col] = s;
  else grad[(size_t)Cout * K9 + co] = s;
}

__global__ void k_net_inputs(const float* __restrict__ feat, const int* __restrict__ idx, int n,
                             int R, uint16_t* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * R * R) return;
  const int px = (int)(i % R), py = (int)((i / R) % R), b = (int)(i / ((long long)R * R));
  const int s = idx ? idx[b] : b;
  const float* f = feat + 3 * (size_t)s;
  float v[8];
  v[0] = ((float)px + 0.5f) / (float)R;
  v[1] = ((float)py + 0.5f) / (float)R;
  v[2] = (f[0] - 4.5f) / 1.5f;
  v[3] = (f[1] - 3.855f) / 3.145f;
  v[4] = f[2] / 4.0f;
  v[5] = v[6] = v[7] = 0.f;
  uint16_t h[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) h[c] = to_bf16(v[c]);
  *(uint4*)(x + 8 * i) = *(const uint4*)h;
}

__global__ void k_upsample2(const uint16_t* __restrict__ in, int n, int h, int w, int C,
                            uint16_t* __restrict__ out) {
  // one thread per output pixel and group of 8 channels
  const int cg = C >> 3;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * 4 * h * w * cg) return;
  const int q = (int)(i % cg);
  long long p = i / cg;
  const int X = (int)(p % (2 * w));
  p /= 2 * w;
  const int Y = (int)(p % (2 * h));
  const long long b = p / (2 * h);
  *(uint4*)(out + i * 8) = *(const uint4*)(in + (((b * h + (Y >> 1)) * w + (X >> 1)) * C + q * 8));
}

__global__ void k_act_grad(const float* __restrict__ dx, int pool, const float* __restrict__ add,
                           const float* __restrict__ z, int n, int h, int w, int C,
                           uint16_t* __restrict__ dz, float* __restrict__ da_out) {
  const long long total = (long long)n * h * w * C;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float d;
  if (pool) {
    const int c = (int)(i % C);
    long long p = i / C;
    const int xx = (int)(p % w);
    p /= w;
    const int y = (int)(p % h);
    const long long b = p / h;
    const size_t row = (size_t)2 * w * C;
    const float* q = dx + ((size_t)(b * 2 * h + 2 * y) * 2 * w + 2 * xx) * C + c;
    d = (q[0] + q[C]) + (q[row] + q[row + C]);
  } else {
    d = dx[i];
  }
  if (add) d += add[i];
  if (da_out) da_out[i] = d;
  const float zz = z[i];
  const float sg = 1.0f / (1.0f + __expf(-zz));
  dz[i] = to_bf16(d * (sg * (1.0f + zz * (1.0f - sg))));
}

// One thread per pixel; block sums of squared errors in FP64, reduced in a
// fixed order by k_mse_fold.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, int C,
                                             const float* __restrict__ target,
                                             const int* __restrict__ idx, int n, int R,
                                             float inv_count, uint16_t* __restrict__ dz,
                                             double* __restrict__ part) {
  __shared__ double sh[256];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < (long long)n * R * R) {
    const long long RR = (long long)R * R;
    const int b = (int)(i / RR);
    const long long pix = i - (long long)b * RR;
    const int smp = idx ? idx[b] : b;
    const float* t = target + (size_t)smp * 3 * RR + pix;
    for (int c = 0; c < C; ++c) {
      float g = 0.f;
      if (c < 3) {
        const float d = y[i * C + c] - t[c * RR];
        s += (double)d * d;
        g = 2.0f * d * inv_count;
      }
      dz[i * C + c] = to_bf16(g);
    }
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_mse_fold(const double* __restrict__ part, int nb,
                                                  double inv_count, float* __restrict__ loss) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) s += part[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] * inv_count);
}

__global__ void k_unpack_pred(const float* __restrict__ y, int C, int n, int R,
                              float* __restrict__ planes) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long RR = (long long)R * R;
  if (i >= (long long)n * 3 * RR) return;
  const long long pix = i % RR;
  const int c = (int)((i / RR) % 3);
  const long long b = i / (3 * RR);
  planes[i] = y[(b * RR + pix) * C + c];
}

__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long long count, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_weights_bf16(const float* __restrict__ w, int Cout, int Cin,
                               uint16_t* __restrict__ wb, uint16_t* __restrict__ wt) {
  const int K9 = 9 * Cin;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Cout * K9) return;
  const int co = i / K9, r = i - co * K9, tap = r / Cin, ci = r - tap * Cin;
  const uint16_t h = to_bf16(w[i]);
  wb[i] = h;
  wt[((size_t)tap * Cin + ci) * Cout + co] = h;
}

template <typename Tin>
__device__ __forceinline__ double bilinear_at(const Tin* __restrict__ src, int snx, int sny,
                                              long long sstride, int x, int y, int dnx,
                                              int dny) {
  double qx = ((double)x + 0.5) * snx / dnx - 0.5;
  double qy = ((double)y + 0.5) * sny / dny - 0.5;
  qx = fmin(fmax(qx, 0.0), (double)(snx - 1));
  qy = fmin(fmax(qy, 0.0), (double)(sny - 1));
  const int x0 = min((int)floor(qx), snx - 1), x1 = min(x0 + 1, snx - 1);
  const int y0 = min((int)floor(qy), sny - 1), y1 = min(y0 + 1, sny - 1);
  const double fx = qx - x0, fy = qy - y0;
  const double s00 = (double)src[y0 * sstride + x0], s01 = (double)src[y0 * sstride + x1];
  const double s10 = (double)src[y1 * sstride + x0], s11 = (double)src[y1 * sstride + x1];
  const double top = s00 * (1.0 - fx) + s01 * fx;
  const double bot = s10 * (1.0 - fx) + s11 * fx;
  return top * (1.0 - fy) + bot * fy;
}

// antisym: the result is made odd under the 180-degree rotation of the
// rectangle, r(p) = (v(p) - v(rot p)) / 2 with v = value * scale + offset.
template <typename Tin, typename Tout>
__global__ void k_resample(const Tin* __restrict__ src, int snx, int sny, long long sstride,
                           Tout* __restrict__ dst, int dnx, int dny, double scale,
                           double offset, int antisym) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)dnx * dny) return;
  const int x = (int)(i % dnx), y = (int)(i / dnx);
  const double v = bilinear_at(src, snx, sny, sstride, x, y, dnx, dny) * scale + offset;
  if (!antisym) {
    dst[i] = (Tout)v;
    return;
  }
  const double w =
      bilinear_at(src, snx, sny, sstride, dnx - 1 - x, dny - 1 - y, dnx, dny) * scale + offset;
  dst[i] = (Tout)(0.5 * (v - w));
}

inline unsigned nblocks(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct SplitPlan {
  int gx, gy, splits, cps, nchunks, N, max_splits;
};
// max_splits depends on the layer's channel counts only, not on the batch:
// splits = ceil(nchunks / ceil(nchunks / w)) <= w for w = min(max_splits,
// nchunks), so max_splits * Cout * N floats hold the partials of any batch.
inline SplitPlan wgrad_plan(const ConvGeom& g) {
  SplitPlan p;
  p.N = 9 * g.Cin + 8;
  p.gx = (g.Cout + 63) / 64;
  p.gy = (p.N + 63) / 64;
  const long long P = (long long)g.n * g.Ho * g.Wo;
  p.nchunks = (int)((P + BK - 1) / BK);
  int want = 1024 / (p.gx * p.gy);
  if (want < 1) want = 1;
  if (want > 256) want = 256;
  p.max_splits = want;
  if (want > p.nchunks) want = p.nchunks;
  p.cps = (p.nchunks + want - 1) / want;
  p.splits = (p.nchunks + p.cps - 1) / p.cps;
  return p;
}

}  // namespace

hipError_t launch_conv_fwd(const ConvGeom& g, const uint16_t* x, const uint16_t* w,
                           const float* bias, const uint16_t* skip, float* z32, uint16_t* a16,
                           int act, hipStream_t s) {
  ConvArgs a{};
  a.g = g;
  a.x = x;
  a.w = w;
  a.bias = bias;
  a.skip = skip;
  a.z32 = z32;
  a.a16 = a16;
  a.act = act;
  a.M = g.n * g.Ho * g.Wo;
  a.N = g.Cout;
  a.nchunks = (9 * g.Cin + BK - 1) / BK;
  a.cps = a.nchunks;
  if (g.Cout <= 32) {
    hipLaunchKernelGGL((k_conv<FWD, 128, 32>), dim3((a.M + 127) / 128, (a.N + 31) / 32, 1),
                       dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_conv<FWD, 64, 64>), dim3((a.M + 63) / 64, (a.N + 63) / 64, 1),
                       dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_conv_bwd_data(const ConvGeom& g, const uint16_t* dz, const uint16_t* wt,
                                float* dx, hipStream_t s) {
  ConvArgs a{};
  a.g = g;
  a.w = wt;
  a.dz = dz;
  a.out = dx;
  a.M = g.n * g.H * g.W;
  a.N = g.Cin;
  a.nchunks = (9 * g.Cout + BK - 1) / BK;
  a.cps = a.nchunks;
  if (g.Cin <= 32) {
    hipLaunchKernelGGL((k_conv<BWD_DATA, 128, 32>), dim3((a.M + 127) / 128, (a.N + 31) / 32, 1),
                       dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_conv<BWD_DATA, 64, 64>), dim3((a.M + 63) / 64, (a.N + 63) / 64, 1),
                       dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

size_t conv_bwd_weight_part_floats(const ConvGeom& g) {
  const SplitPlan p = wgrad_plan(g);
  return (size_t)p.max_splits * g.Cout * p.N;
}

hipError_t launch_conv_bwd_weight(const ConvGeom& g, const uint16_t* x, const uint16_t* dz,
                                  float* part, size_t part_floats, float* grad_wb,
                                  hipStream_t s) {
  const SplitPlan p = wgrad_plan(g);
  if ((size_t)p.splits * g.Cout * p.N > part_floats) return hipErrorInvalidValue;
  ConvArgs a{};
  a.g = g;
  a.x = x;
  a.dz = dz;
  a.out = part;
  a.M = g.Cout;
  a.N = p.N;
  a.nchunks = p.nchunks;
  a.cps = p.cps;
  hipLaunchKernelGGL((k_conv<BWD_WEIGHT, 64, 64>), dim3(p.gx, p.gy, p.splits), dim3(256), 0, s,
                     a);
  const int K9 = 9 * g.Cin;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)(((long long)g.Cout * (K9 + 1) + 63) / 64)),
                     dim3(64), 0, s, part, p.splits, g.Cout, K9, p.N, grad_wb);
  return hipGetLastError();
}

hipError_t launch_net_inputs(const float* feat, const int* idx, int n, int R, uint16_t* x,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_net_inputs, dim3(nblocks((long long)n * R * R)), dim3(256), 0, s, feat,
                     idx, n, R, x);
  return hipGetLastError();
}

hipError_t launch_upsample2(const uint16_t* in, int n, int h, int w, int C, uint16_t* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_upsample2, dim3(nblocks((long long)n * 4 * h * w * (C / 8))), dim3(256),
                     0, s, in, n, h, w, C, out);
  return hipGetLastError();
}

hipError_t launch_act_grad(const float* dx, int pool, const float* add, const float* z, int n,
                           int h, int w, int C, uint16_t* dz, float* da_out, hipStream_t s) {
  hipLaunchKernelGGL(k_act_grad, dim3(nblocks((long long)n * h * w * C)), dim3(256), 0, s, dx,
                     pool, add, z, n, h, w, C, dz, da_out);
  return hipGetLastError();
}

size_t net_mse_part_doubles(int n, int R) { return nblocks((long long)n * R * R); }

hipError_t launch_mse(const float* y, int C, const float* target, const int* idx, int n, int R,
                      uint16_t* dz, double* part, float* loss_out, hipStream_t s) {
  const unsigned nb = nblocks((long long)n * R * R);
  const double count = 3.0 * n * R * R;
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, y, C, target, idx, n, R,
                     (float)(1.0 / count), dz, part);
  if (loss_out)
    hipLaunchKernelGGL(k_mse_fold, dim3(1), dim3(256), 0, s, part, (int)nb, 1.0 / count,
                       loss_out);
  return hipGetLastError();
}

hipError_t launch_unpack_pred(const float* y, int C, int n, int R, float* planes,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_pred, dim3(nblocks((long long)n * 3 * R * R)), dim3(256), 0, s, y,
                     C, n, R, planes);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, long long count, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nblocks(count)), dim3(256), 0, s, w, m, v, g, count, lr,
                     beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_weights_bf16(const float* w, int Cout, int Cin, uint16_t* wb, uint16_t* wt,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_weights_bf16, dim3(nblocks((long long)Cout * 9 * Cin)), dim3(256), 0, s,
                     w, Cout, Cin, wb, wt);
  return hipGetLastError();
}

hipError_t launch_resample(const void* src, int src_f64, int snx, int sny, long long sstride,
                           void* dst, int dst_f64, int dnx, int dny, double scale, double offset,
                           int antisym, hipStream_t s) {
  const dim3 grid(nblocks((long long)dnx * dny)), blk(256);
  if (src_f64 && dst_f64)
    hipLaunchKernelGGL((k_resample<double, double>), grid, blk, 0, s, (const double*)src, snx,
                       sny, sstride, (double*)dst, dnx, dny, scale, offset, antisym);
  else if (src_f64)
    hipLaunchKernelGGL((k_resample<double, float>), grid, blk, 0, s, (const double*)src, snx,
                       sny, sstride, (float*)dst, dnx, dny, scale, offset, antisym);
  else if (dst_f64)
    hipLaunchKernelGGL((k_resample<float, double>), grid, blk, 0, s, (const float*)src, snx,
                       sny, sstride, (double*)dst, dnx, dny, scale, offset, antisym);
  else
    hipLaunchKernelGGL((k_resample<float, float>), grid, blk, 0, s, (const float*)src, snx,
                       sny, sstride, (float*)dst, dnx, dny, scale, offset, antisym);
  return hipGetLastError();
}

}  // namespace lf
