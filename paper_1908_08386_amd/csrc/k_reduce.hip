// k_reduce.hip -- deterministic reductions: residual, Nusselt numbers, mass.
//
// All sums accumulate in FP64.  Each reduction is two-pass: a fixed grid of
// blocks writes per-block partials (wave64 shuffle reduction, then a small
// LDS tree across the block's waves), and one block folds the partials in a
// fixed order.  Results are therefore bitwise reproducible run to run and
// independent of the step kernel's tiling.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum K values per thread across the block; thread 0 receives the totals.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*sh)[K]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[wid][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) s += sh[w][k];
      v[k] = s;
    }
  }
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

// residual partials: rows are distributed over blocks round-robin
template <typename real>
__global__ __launch_bounds__(kThreads) void k_resid_partial(
    int nx, int ny, int pitch, int plane, const real* __restrict__ mom,
    const real* __restrict__ T, real* __restrict__ snap, double* __restrict__ part) {
  __shared__ double sh[kThreads / 64][7];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int j = blockIdx.x; j < ny; j += gridDim.x) {
    for (int i = threadIdx.x; i < nx; i += kThreads) {
      const int o = j * pitch + i;
      const double u = (double)mom[plane + o], v = (double)mom[2 * plane + o];
      const double t = (double)T[o];
      const double su = (double)snap[o], sv = (double)snap[plane + o];
      const double st = (double)snap[2 * plane + o];
      acc[0] += (u - su) * (u - su);
      acc[1] += u * u;
      acc[2] += (v - sv) * (v - sv);
      acc[3] += v * v;
      acc[4] += (t - st) * (t - st);
      acc[5] += t * t;
      if (!(finite_d(u) && finite_d(v) && finite_d(t))) acc[6] += 1.0;
      snap[o] = mom[plane + o];
      snap[plane + o] = mom[2 * plane + o];
      snap[2 * plane + o] = T[o];
    }
  }
  block_sum<7>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) part[blockIdx.x * 8 + k] = acc[k];
}

template <int K>
__global__ __launch_bounds__(kThreads) void k_fold(const double* __restrict__ part,
                                                   int nblocks, double* __restrict__ out) {
  __shared__ double sh[kThreads / 64][K];
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += part[b * 8 + k];
  block_sum<K>(acc, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[k] = acc[k];
}

// Nusselt numbers of the west and east walls, one block.
template <typename real>
__global__ __launch_bounds__(kThreads) void k_nusselt(int nx, int ny, int pitch,
                                                      const real* __restrict__ T, double Th,
                                                      double Tc, double* __restrict__ out) {
  __shared__ double sh[kThreads / 64][4];
  __shared__ double mx[kThreads][2];
  __shared__ int at[kThreads][2];
  double dT = Th - Tc;
  if (dT == 0.0) dT = 1.0;
  const double H = (double)ny;
  double acc[4] = {0, 0, 0, 0};
  double mh = -INFINITY, mc = -INFINITY;
  int jh = 0x7fffffff, jc = 0x7fffffff;
  for (int j = threadIdx.x; j < ny; j += kThreads) {
    const double t0 = (double)T[j * pitch], t1 = (double)T[j * pitch + 1];
    const double tn = (double)T[j * pitch + nx - 1], tm = (double)T[j * pitch + nx - 2];
    const double nh = 2.0 * H * (Th - t0) / dT;
    const double nc = 2.0 * H * (tn - Tc) / dT;
    acc[0] += nh;
    acc[1] += nc;
    acc[2] += H * (8.0 * Th - 9.0 * t0 + t1) / (3.0 * dT);
    acc[3] += H * (9.0 * tn - 8.0 * Tc - tm) / (3.0 * dT);
    if (nh > mh) { mh = nh; jh = j; }  // j increases: keeps the lowest j on ties
    if (nc > mc) { mc = nc; jc = j; }
  }
  mx[threadIdx.x][0] = mh;
  mx[threadIdx.x][1] = mc;
  at[threadIdx.x][0] = jh;
  at[threadIdx.x][1] = jc;
  block_sum<4>(acc, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    double bh = -INFINITY, bc = -INFINITY;
    int bjh = 0x7fffffff, bjc = 0x7fffffff;
    for (int t = 0; t < kThreads; ++t) {
      if (mx[t][0] > bh || (mx[t][0] == bh && at[t][0] < bjh)) { bh = mx[t][0]; bjh = at[t][0]; }
      if (mx[t][1] > bc || (mx[t][1] == bc && at[t][1] < bjc)) { bc = mx[t][1]; bjc = at[t][1]; }
    }
    out[0] = acc[0] / ny;
    out[1] = acc[1] / ny;
    out[2] = bh;
    out[3] = (bjh + 0.5) / ny;
    out[4] = bc;
    out[5] = (bjc + 0.5) / ny;
    out[6] = acc[2] / ny;
    out[7] = acc[3] / ny;
  }
}

template <typename real>
__global__ __launch_bounds__(kThreads) void k_mass_partial(int nx, int ny, int pitch, int plane,
                                                           const real* __restrict__ f,
                                                           const real* __restrict__ T,
                                                           double* __restrict__ part) {
  __shared__ double sh[kThreads / 64][2];
  double acc[2] = {0, 0};
  for (int j = blockIdx.x; j < ny; j += gridDim.x)
    for (int i = threadIdx.x; i < nx; i += kThreads) {
      const int o = j * pitch + i;
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) s += (double)f[q * plane + o];
      acc[0] += s;
      acc[1] += (double)T[o];
    }
  block_sum<2>(acc, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 8] = acc[0];
    part[blockIdx.x * 8 + 1] = acc[1];
  }
}

template <typename real>
__global__ __launch_bounds__(kThreads) void k_unpack(int nx, int ny, int pitch,
                                                     const real* __restrict__ src, void* dst,
                                                     int as_f64, int pressure) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx) return;
  const real v = src[j * pitch + i];
  // pressure: kinematic p = c_s^2 (rho - 1) from the density plane
  const double d = pressure ? ((double)v - 1.0) / 3.0 : (double)v;
  if (as_f64) static_cast<double*>(dst)[j * nx + i] = d;
  else static_cast<real*>(dst)[j * nx + i] = pressure ? (real)d : v;
}

}  // namespace

template <typename real>
hipError_t launch_residual(const Grid& g, const real* mom, const real* T, real* snap,
                           double* partials, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_partial<real>, dim3(nblocks), dim3(kThreads), 0, s, g.nx, g.ny,
                     g.pitch, (int)g.plane, mom, T, snap, partials);
  hipLaunchKernelGGL(k_fold<7>, dim3(1), dim3(kThreads), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_nusselt(const Grid& g, const WallSet& w, const real* T, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_nusselt<real>, dim3(1), dim3(kThreads), 0, s, g.nx, g.ny, g.pitch, T,
                     w.Tw[0], w.Tw[1], out);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_mass(const Grid& g, const real* f, const real* T, double* partials,
                       int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mass_partial<real>, dim3(nblocks), dim3(kThreads), 0, s, g.nx, g.ny,
                     g.pitch, (int)g.plane, f, T, partials);
  hipLaunchKernelGGL(k_fold<2>, dim3(1), dim3(kThreads), 0, s, partials, nblocks, out);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_unpack(const Grid& g, const real* plane, void* dst, int as_f64,
                         hipStream_t s, int pressure) {
  dim3 grid((g.nx + kThreads - 1) / kThreads, g.ny);
  hipLaunchKernelGGL(k_unpack<real>, grid, dim3(kThreads), 0, s, g.nx, g.ny, g.pitch, plane,
                     dst, as_f64, pressure);
  return hipGetLastError();
}

#define LF_INST(real)                                                                      \
  template hipError_t launch_residual<real>(const Grid&, const real*, const real*, real*,  \
                                            double*, int, double*, hipStream_t);           \
  template hipError_t launch_nusselt<real>(const Grid&, const WallSet&, const real*,       \
                                           double*, hipStream_t);                          \
  template hipError_t launch_mass<real>(const Grid&, const real*, const real*, double*,    \
                                        int, double*, hipStream_t);                        \
  template hipError_t launch_unpack<real>(const Grid&, const real*, void*, int, hipStream_t, int);
LF_INST(float)
LF_INST(double)
#undef LF_INST

}  // namespace lf
