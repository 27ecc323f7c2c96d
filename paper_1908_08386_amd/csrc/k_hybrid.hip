// k_hybrid.hip -- fused Mode H time step for gfx950 (CDNA4).
//
// One time step of the variable-split hybrid (Sec. 5.1 of Li, Yang & Zhang,
// arXiv:1908.08386; coupling order of Sec. 6.2):
//   pull streaming with half-way bounce-back  -> moments rho, V (Eq 16-17)
//   explicit FV energy balance on the fresh V (Eq 24 / Eq 76, QUICK)
//   BGK collision + buoyancy force from the fresh T (Eq 5, 8, 18, 81)
// fused into a single pass over HBM: each node's 9 populations and its
// temperature are read once and written once (80 B per node in FP32).
//
// Work decomposition.  A 64-lane wavefront owns a strip of 64 consecutive
// columns; lanes 1..62 produce output, lanes 0 and 63 are halo columns whose
// moments and temperatures feed the x-faces of the strip edges.  The wave
// marches up a band of rows.  x-neighbour values (u at i+-1, T at i+-1,
// i+-2) come from neighbouring lanes through cross-lane permutes; y-neighbour
// values (v at j+-1, T at j-2..j+2) live in a rolling register window.
// There is no LDS and no barrier: waves are independent, so a launch of
// ceil(nx/62) * ceil(ny/band) waves keeps every CU busy with no tail
// synchronisation.  The halo costs 2/64 of the lanes plus two pulled rows
// per band, which are re-reads of lines other waves fetch (cache hits).
//
// Populations are stored shifted, f~ = f - w_q: the FP32 round-off of a
// stored value is then relative to the (small) deviation from rest instead of
// to w_q, which keeps FP32 results within 1e-4 of FP64 over long runs.
#include "lf_internal.h"

namespace lf {
namespace {

constexpr int kOut = 62;  // output columns per wave (lanes 1..62)

// D2Q9 (Eq 4, Eq 9): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
__host__ __device__ constexpr int ex(int q) {
  return (q == 1 || q == 5 || q == 8) ? 1 : (q == 3 || q == 6 || q == 7) ? -1 : 0;
}
__host__ __device__ constexpr int ey(int q) {
  return (q == 2 || q == 5 || q == 6) ? 1 : (q == 4 || q == 7 || q == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int q) {
  return q == 0 ? 0 : q < 5 ? ((q + 1) % 4) + 1 : ((q - 3) % 4) + 5;
}
template <typename real>
__host__ __device__ constexpr real wq(int q) {
  return q == 0 ? real(4) / real(9) : q < 5 ? real(1) / real(9) : real(1) / real(36);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

template <typename real>
struct StepArgs {
  const real* __restrict__ fin;
  real* __restrict__ fout;
  const real* __restrict__ Tin;
  real* __restrict__ Tout;
  real* __restrict__ mom;
  int plane;  // elements per plane
  int nx, ny, pitch, band, nstrips, nwaves;
  int xper, yper, conv;
  int tfix[4];
  real omega, alpha, gbeta, Tref, gx, gy;
  real uw[4];
  real Tw[4];
};

__device__ __forceinline__ int wrap_any(int c, int n) {
  int m = c % n;
  return m < 0 ? m + n : m;
}
__device__ __forceinline__ int wrap_one(int c, int n) {
  return c < 0 ? c + n : (c >= n ? c - n : c);
}
__device__ __forceinline__ int clampi(int c, int lo, int hi) {
  return c < lo ? lo : (c > hi ? hi : c);
}

// Temperature of cell (c, r) of the previous step, extended one cell past
// every non-periodic side by the wall's ghost value: 2 T_w - T_edge for a
// fixed-temperature wall, T_edge for an adiabatic one.  Values further out
// are clamped and never used.
template <typename real>
__device__ __forceinline__ real T_at(const StepArgs<real>& a, int c, int r) {
  const int cc = a.xper ? wrap_any(c, a.nx) : clampi(c, 0, a.nx - 1);
  const int rr = a.yper ? wrap_any(r, a.ny) : clampi(r, 0, a.ny - 1);
  real t = a.Tin[rr * a.pitch + cc];
  if (!a.xper) {
    if (c < 0 && a.tfix[0]) t = real(2) * a.Tw[0] - t;
    else if (c >= a.nx && a.tfix[1]) t = real(2) * a.Tw[1] - t;
  }
  if (!a.yper) {
    if (r < 0 && a.tfix[2]) t = real(2) * a.Tw[2] - t;
    else if (r >= a.ny && a.tfix[3]) t = real(2) * a.Tw[3] - t;
  }
  return t;
}

// Pull the 9 streamed populations of node (ic, r) (r is wrapped or clamped
// into the grid) and form its moments.  A link whose upstream node lies
// beyond a wall returns the node's own reversed population plus the moving
// wall term 6 w_q (e_q . u_w); at a corner the south/north wall is taken.
template <typename real>
__device__ __forceinline__ void pull_row(const StepArgs<real>& a, int ic, int r,
                                         real f[9], real& drho, real& ux,
                                         real& uy) {
  const int rr = a.yper ? wrap_any(r, a.ny) : clampi(r, 0, a.ny - 1);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int sx = ic - ex(q), sy = rr - ey(q);
    int side = -1;
    if (a.xper) sx = wrap_one(sx, a.nx);
    else if (sx < 0) side = 0;
    else if (sx >= a.nx) side = 1;
    if (a.yper) sy = wrap_one(sy, a.ny);
    else if (sy < 0) side = 2;
    else if (sy >= a.ny) side = 3;
    real v;
    if (side < 0) {
      v = a.fin[q * a.plane + sy * a.pitch + sx];
    } else {
      const real uwall = a.uw[side];
      const real eu = side >= 2 ? real(ex(q)) * uwall : real(ey(q)) * uwall;
      v = a.fin[opp(q) * a.plane + rr * a.pitch + ic] + real(6) * wq<real>(q) * eu;
    }
    f[q] = v;
  }
  real s = real(0), jx = real(0), jy = real(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    s += f[q];
    if (ex(q) > 0) jx += f[q];
    if (ex(q) < 0) jx -= f[q];
    if (ey(q) > 0) jy += f[q];
    if (ey(q) < 0) jy -= f[q];
  }
  drho = s;
  const real inv = real(1) / (real(1) + s);
  ux = jx * inv;
  uy = jy * inv;
}

// Face value of the convected temperature between cells L and R; tll is
// upstream of L, trr downstream of R.  QUICK: quadratic through the two
// neighbours and the next upstream cell.
template <typename real>
__device__ __forceinline__ real face_value(int conv, real uf, real tll, real tl,
                                           real tr, real trr) {
  if (conv == 1) return real(0.5) * (tl + tr);
  if (conv == 2) return uf >= real(0) ? tl : tr;
  return uf >= real(0) ? (real(6) * tl + real(3) * tr - tll) * real(0.125)
                       : (real(6) * tr + real(3) * tl - trr) * real(0.125);
}

// BGK collision with the buoyancy force, on shifted populations.
//   f_eq = rho w (1 + P),  P = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u       (Eq 8)
//   F    = 3 w (G.(e - u)) (1 + P)  = G.(e - u) f_eq / (rho c_s^2) (Eq 18)
//   f*   = f + (f_eq - f) / tau + F                           (Eq 5 / 19)
// with G = (gx, g beta (T - T_ref) + gy) (Eq 81).  In shifted form
// f~_eq = w (drho + rho P).
template <typename real>
__device__ __forceinline__ void collide(const StepArgs<real>& a, const real f[9],
                                        real drho, real ux, real uy, real T,
                                        real out[9]) {
  const real rho = real(1) + drho;
  const real Gx = a.gx;
  const real Gy = a.gbeta * (T - a.Tref) + a.gy;
  const real usq = real(1.5) * (ux * ux + uy * uy);
  const real Gu = Gx * ux + Gy * uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const real eu = real(ex(q)) * ux + real(ey(q)) * uy;
    const real P = real(3) * eu + real(4.5) * eu * eu - usq;
    const real feq = wq<real>(q) * (drho + rho * P);
    const real Ge = real(ex(q)) * Gx + real(ey(q)) * Gy;
    const real F = real(3) * wq<real>(q) * (Ge - Gu) * (real(1) + P);
    out[q] = f[q] + a.omega * (feq - f[q]) + F;
  }
}

template <typename real>
__global__ __launch_bounds__(256) void k_hybrid_step(StepArgs<real> a) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (wave >= a.nwaves) return;  // uniform per wave
  const int strip = wave % a.nstrips;
  const int bnd = wave / a.nstrips;
  const int i = strip * kOut + lane - 1;  // this lane's column
  const int ic = a.xper ? wrap_any(i, a.nx) : clampi(i, 0, a.nx - 1);
  const bool act = lane >= 1 && lane <= kOut && i < a.nx;
  const int j0 = bnd * a.band;
  const int j1 = min(j0 + a.band, a.ny);
  const int ix2 = lane < 32 ? i - 2 : i + 2;  // second T column (lanes 1, 62)
  const real al = a.alpha;

  real fc[9], fn[9];
  real dr_c, ux_c, uy_c, dr_n, ux_n, uy_n, uy_p;
  {
    real ft[9], d, u;
    pull_row(a, ic, j0 - 1, ft, d, u, uy_p);
  }
  pull_row(a, ic, j0, fc, dr_c, ux_c, uy_c);
  real t0 = T_at(a, i, j0 - 2), t1 = T_at(a, i, j0 - 1), t2 = T_at(a, i, j0);
  real t3 = T_at(a, i, j0 + 1), t4 = T_at(a, i, j0 + 2);

  for (int j = j0; j < j1; ++j) {
    pull_row(a, ic, j + 1, fn, dr_n, ux_n, uy_n);
    const real tx2 = T_at(a, ix2, j);
    // x-neighbours from the adjacent lanes (all lanes take part)
    const real tW1 = __shfl_up(t2, 1, 64);
    const real tE1 = __shfl_down(t2, 1, 64);
    real tW2 = __shfl_up(t2, 2, 64);
    real tE2 = __shfl_down(t2, 2, 64);
    const real uW = __shfl_up(ux_c, 1, 64);
    const real uE = __shfl_down(ux_c, 1, 64);
    if (lane == 1) tW2 = tx2;
    if (lane == kOut) tE2 = tx2;

    // fluxes through the four faces, positive towards +x / +y
    real Fw, Fe, Fs, Fn;
    if (!a.xper && i == 0) {
      Fw = a.tfix[0] ? real(-2) * al * (t2 - a.Tw[0]) : real(0);
    } else {
      const real uf = real(0.5) * (uW + ux_c);
      Fw = uf * face_value(a.conv, uf, tW2, tW1, t2, tE1) - al * (t2 - tW1);
    }
    if (!a.xper && i == a.nx - 1) {
      Fe = a.tfix[1] ? real(-2) * al * (a.Tw[1] - t2) : real(0);
    } else {
      const real uf = real(0.5) * (ux_c + uE);
      Fe = uf * face_value(a.conv, uf, tW1, t2, tE1, tE2) - al * (tE1 - t2);
    }
    if (!a.yper && j == 0) {
      Fs = a.tfix[2] ? real(-2) * al * (t2 - a.Tw[2]) : real(0);
    } else {
      const real vf = real(0.5) * (uy_p + uy_c);
      Fs = vf * face_value(a.conv, vf, t0, t1, t2, t3) - al * (t2 - t1);
    }
    if (!a.yper && j == a.ny - 1) {
      Fn = a.tfix[3] ? real(-2) * al * (a.Tw[3] - t2) : real(0);
    } else {
      const real vf = real(0.5) * (uy_c + uy_n);
      Fn = vf * face_value(a.conv, vf, t1, t2, t3, t4) - al * (t3 - t2);
    }
    const real Tnew = t2 - (Fe - Fw) - (Fn - Fs);

    if (act) {
      real fo[9];
      collide(a, fc, dr_c, ux_c, uy_c, Tnew, fo);
      const int o = j * a.pitch + i;
#pragma unroll
      for (int q = 0; q < 9; ++q) a.fout[q * a.plane + o] = fo[q];
      a.Tout[o] = Tnew;
      if (a.mom) {
        a.mom[o] = real(1) + dr_c;
        a.mom[a.plane + o] = ux_c;
        a.mom[2 * a.plane + o] = uy_c;
      }
    }

    uy_p = uy_c;
#pragma unroll
    for (int q = 0; q < 9; ++q) fc[q] = fn[q];
    dr_c = dr_n;
    ux_c = ux_n;
    uy_c = uy_n;
    t0 = t1;
    t1 = t2;
    t2 = t3;
    t3 = t4;
    t4 = T_at(a, i, j + 3);
  }
}

// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_init(int nx, int ny, int pitch, int plane,
                                              const double* __restrict__ T0,
                                              const double* __restrict__ u0,
                                              const double* __restrict__ v0,
                                              real* __restrict__ f, real* __restrict__ T,
                                              real* __restrict__ mom,
                                              real* __restrict__ snap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx) return;
  const int d = j * nx + i, o = j * pitch + i;
  const double u = u0 ? u0[d] : 0.0, v = v0 ? v0[d] : 0.0, t = T0 ? T0[d] : 0.0;
  const double usq = 1.5 * (u * u + v * v);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double eu = ex(q) * u + ey(q) * v;
    // f_eq(1, u) - w = w (3 e.u + 9/2 (e.u)^2 - 3/2 u.u)
    f[q * plane + o] = real(wq<double>(q) * (3.0 * eu + 4.5 * eu * eu - usq));
  }
  T[o] = real(t);
  mom[o] = real(1);
  mom[plane + o] = real(u);
  mom[2 * plane + o] = real(v);
  snap[o] = real(u);
  snap[plane + o] = real(v);
  snap[2 * plane + o] = real(t);
}

}  // namespace

template <typename real>
hipError_t launch_hybrid_step(const Grid& g, const WallSet& w, const HybridParams& p,
                              const real* fin, real* fout, const real* Tin, real* Tout,
                              real* mom, int band, hipStream_t s) {
  StepArgs<real> a;
  a.fin = fin;
  a.fout = fout;
  a.Tin = Tin;
  a.Tout = Tout;
  a.mom = mom;
  a.plane = (int)g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.pitch = g.pitch;
  a.band = band < 1 ? 1 : band;
  a.nstrips = (g.nx + kOut - 1) / kOut;
  const int nbands = (g.ny + a.band - 1) / a.band;
  a.nwaves = a.nstrips * nbands;
  a.xper = w.xper;
  a.yper = w.yper;
  a.conv = p.conv;
  for (int k = 0; k < 4; ++k) {
    a.tfix[k] = w.tfix[k];
    a.uw[k] = real(w.uw[k]);
    a.Tw[k] = real(w.Tw[k]);
  }
  a.omega = real(p.omega);
  a.alpha = real(p.alpha);
  a.gbeta = real(p.gbeta);
  a.Tref = real(p.T_ref);
  a.gx = real(p.gx);
  a.gy = real(p.gy);
  const int blocks = (a.nwaves + 3) / 4;
  hipLaunchKernelGGL(k_hybrid_step<real>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_init(const Grid& g, const double* T0, const double* u0, const double* v0,
                       real* f, real* T, real* mom, real* snap, hipStream_t s) {
  dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL(k_init<real>, grid, dim3(256), 0, s, g.nx, g.ny, g.pitch,
                     (int)g.plane, T0, u0, v0, f, T, mom, snap);
  return hipGetLastError();
}

template hipError_t launch_hybrid_step<float>(const Grid&, const WallSet&, const HybridParams&,
                                              const float*, float*, const float*, float*,
                                              float*, int, hipStream_t);
template hipError_t launch_hybrid_step<double>(const Grid&, const WallSet&, const HybridParams&,
                                               const double*, double*, const double*, double*,
                                               double*, int, hipStream_t);
template hipError_t launch_init<float>(const Grid&, const double*, const double*, const double*,
                                       float*, float*, float*, float*, hipStream_t);
template hipError_t launch_init<double>(const Grid&, const double*, const double*, const double*,
                                        double*, double*, double*, double*, hipStream_t);

}  // namespace lf
