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

// Floating-point contraction is off in this file and every fused
// multiply-add is written out (fma_): the interior and the general march
// then execute the same operations in the same order for a node, so results
// do not depend on how the grid is cut into strips and bands.
#pragma clang fp contract(off)

namespace lf {
namespace {

template <typename real>
__device__ __forceinline__ real fma_(real a, real b, real c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fma_<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

constexpr int kOut = 62;  // output columns per wave (lanes 1..62)

// Minimum waves per SIMD the step kernel is compiled for (register budget):
// for FP32 4 when waves march bands of several rows (up to 128 VGPRs: two
// rows in flight), 5 when every wave forms a single row (up to 96 VGPRs,
// nothing to hold ahead; small grids, where all waves are resident at once
// and the step is the issue time of the slowest); FP64 is left its full
// register file.
#define LF_STEP_WAVES(real, ROW1) (sizeof(real) == 4 ? ((ROW1) ? 5 : 4) : 2)

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
  // low-word codes of a compensated (hi + lo) temperature, or null
  const tlo_t* __restrict__ Tlo_in;
  tlo_t* __restrict__ Tlo_out;
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

template <typename real>
__device__ __forceinline__ real recip(real x) {
  return real(1) / x;
}
template <>
__device__ __forceinline__ float recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);  // v_rcp_f32, 1 ulp
}

// Temperature update on a compensated pair: T = hi + lo advances by delta;
// the rounding error of hi + delta (TwoSum, exact without contraction) is
// carried in lo, so per-step increments far below ulp(T) still accumulate.
template <typename real>
__device__ __forceinline__ void t_update(real hi, real lo, real delta, real& nhi, real& nlo) {
  const real s = hi + delta;
  const real bp = s - hi;
  const real err = (hi - (s - bp)) + (delta - bp);
  const real l2 = lo + err;
  nhi = s + l2;
  nlo = l2 - (nhi - s);
}

// The low word is stored as a signed byte k with lo = k 2^-8 ulp(hi), where
// ulp(hi) = 2^(e - 24) for hi = m 2^e, 1/2 <= |m| < 1: the pair resolves T to
// 2^-32 of its binade at 5 bytes per node instead of 8.  The renormalised
// pair has |lo| <= ulp(hi) / 2, so |k| <= 128 (clamped to 127).  Only FP32
// runs carry a low word; the FP64 forms exist for the templates.
__device__ __forceinline__ int lo_encode(float hi, float lo) {
  const int e = __builtin_amdgcn_frexp_expf(hi);
  const float k = __builtin_rintf(__builtin_ldexpf(lo, 32 - e));
  return (int)__builtin_fminf(__builtin_fmaxf(k, -127.0f), 127.0f);
}
__device__ __forceinline__ float lo_decode(float hi, int k) {
  return __builtin_ldexpf((float)k, __builtin_amdgcn_frexp_expf(hi) - 32);
}
__device__ __forceinline__ int lo_encode(double, double) { return 0; }
__device__ __forceinline__ double lo_decode(double, int) { return 0.0; }

// Moments of 9 streamed (shifted) populations.
template <typename real>
__device__ __forceinline__ void moments(const real f[9], real& drho, real& ux, real& uy) {
  const real s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
  drho = s;
  const real inv = recip<real>(real(1) + s);
  ux = jx * inv;
  uy = jy * inv;
}

// Temperature of cell (c, r) of the previous step, extended one cell past
// every non-periodic side by the wall's ghost value: 2 T_w - T_edge for a
// fixed-temperature wall, T_edge for an adiabatic one.  Values further out
// are clamped and never used.
// Face value of the convected temperature between cells L and R; tll is
// upstream of L, trr downstream of R.  QUICK: quadratic through the two
// neighbours and the next upstream cell.
template <typename real>
__device__ __forceinline__ real face_value(const int conv, real uf, real tll, real tl,
                                           real tr, real trr) {
  if (conv == 1) return real(0.5) * (tl + tr);
  if (conv == 2) return uf >= real(0) ? tl : tr;
  // (6 t_near + 3 t_far - t_up) / 8
  return uf >= real(0) ? fma_(real(0.75), tl, fma_(real(0.375), tr, real(-0.125) * tll))
                       : fma_(real(0.75), tr, fma_(real(0.375), tl, real(-0.125) * trr));
}

// x / 3 from an unevaluated pair hi + lo = 1/3 (hi the nearest value):
// within an ulp of the exact quotient and without the common relative error
// a rounded constant 1/3 would give every node.
template <typename real>
__device__ __forceinline__ real third(real x);
template <>
__device__ __forceinline__ float third<float>(float x) {
  return __builtin_fmaf(x, 0x1.555556p-2f, x * -0x1.555556p-27f);
}
template <>
__device__ __forceinline__ double third<double>(double x) {
  return __builtin_fma(x, 0x1.5555555555555p-2, x * 0x1.5555555555555p-56);
}

// BGK collision with the buoyancy force, on shifted populations.
//   f_eq = rho w (1 + P),  P = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u       (Eq 8)
//   F    = 3 w (G.(e - u)) (1 + P)  = G.(e - u) f_eq / (rho c_s^2) (Eq 18)
//   f*   = f + (f_eq - f) / tau + F                           (Eq 5 / 19)
// with G = (gx, g beta (T - T_ref) + gy) (Eq 81).  In shifted form
//   f~_eq = w (drho + rho A) + 3 w e.j,  A = 9/2 (e.u)^2 - 3/2 u.u,
// with j = sum e f~ the streamed momentum (3 w = 1/3 on the axes, 1/12 on
// the diagonals).  The linear term is built from j itself, not as rho * u:
// rho = 1 + drho and the weights rounded to FP32 carry relative errors of up
// to 6e-8 that are the same over regions of nodes, and through the
// relaxation such an error acts as a body force proportional to the local
// momentum, which the slowly decaying large-scale modes of a steady cavity
// amplify by ~ L^2 / nu.  Opposite directions share e.u and e.j up to sign,
// so they are evaluated in pairs.
// Each post-collision population goes to put(q, value) as soon as it is
// formed, so that the nine need not be held together.
template <typename real, typename Put>
__device__ __forceinline__ void collide(const StepArgs<real>& a, const real f[9],
                                        real drho, real ux, real uy, real T, Put&& put) {
  const real rho = real(1) + drho;
  const real Gx = a.gx;
  const real Gy = fma_(a.gbeta, T - a.Tref, a.gy);
  const real usq = real(1.5) * fma_(ux, ux, uy * uy);
  const real Gu = fma_(Gx, ux, Gy * uy);
  const real om = a.omega;
  // streamed momentum, summed as in moments()
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
  {
    const real w = wq<real>(0);
    const real P = -usq;
    const real feq = w * fma_(rho, P, drho);
    const real F = (real(3) * w) * (-Gu) * (real(1) + P);
    put(0, fma_(om, feq - f[0], f[0]) + F);
  }
  auto pair = [&](int q, int qb, real eu, real ej, real Ge, real w, bool diag) {
    const real A = fma_(real(4.5) * eu, eu, -usq);
    const real B = real(3) * eu;
    const real Pq = A + B, Pb = A - B;
    const real base = w * fma_(rho, A, drho);
    const real lin = diag ? real(0.25) * third(ej) : third(ej);
    const real fq = base + lin, fb = base - lin;
    const real cq = (real(3) * w) * (Ge - Gu), cb = (real(3) * w) * (-Ge - Gu);
    put(q, fma_(om, fq - f[q], f[q]) + fma_(cq, Pq, cq));
    put(qb, fma_(om, fb - f[qb], f[qb]) + fma_(cb, Pb, cb));
  };
  pair(1, 3, ux, jx, Gx, wq<real>(1), false);
  pair(2, 4, uy, jy, Gy, wq<real>(2), false);
  pair(5, 7, ux + uy, jx + jy, Gx + Gy, wq<real>(5), true);
  pair(6, 8, uy - ux, jy - jx, Gy - Gx, wq<real>(6), true);
}

// Flux through the face between cells L and R (positive from L to R):
// u_f T_f - alpha (T_R - T_L) with u_f the mean of the two cell velocities.
// tll is upstream of L, trr downstream of R.
template <typename real, int CONV>
__device__ __forceinline__ real face_flux(real al, real uL, real uR, real tll, real tl, real tr,
                                          real trr) {
  const real uf = real(0.5) * (uL + uR);
  return fma_(uf, face_value<real>(CONV, uf, tll, tl, tr, trr), -al * (tr - tl));
}

template <typename real>
__device__ __forceinline__ void store_node(const StepArgs<real>& a, int o, real Tnew, real drho,
                                           real ux, real uy) {
  a.Tout[o] = Tnew;
  if (a.mom) {
    a.mom[o] = real(1) + drho;
    a.mom[a.plane + o] = ux;
    a.mom[2 * a.plane + o] = uy;
  }
}

// General march: any wave, including those touching walls or periodic seams.
// Each cell evaluates its four face fluxes (wall faces by the wall rule).
// Periodicity is a compile-time property of the instance, and every wall
// rule is a select on per-lane flags computed once, so the wave's loads are
// not split by branches: everything the first row needs is requested before
// any arithmetic (one memory round trip for a short band) and later rows'
// inputs one row ahead.
//   Pull: a link whose upstream node lies beyond a wall takes the node's own
//   reversed population plus the moving-wall term 6 w_q (e_q . u_w); at a
//   corner the south/north wall is taken.  T beyond a wall is the ghost
//   2 T_w - T_edge (fixed T) or T_edge (adiabatic).
// Helpers of the general march.  They take scalars, not a struct: a select
// between fields of a local struct would be turned into a load through a
// selected address, which keeps the struct in scratch memory.
template <bool YP>
__device__ __forceinline__ int gen_row(int r, int ny) {
  return YP ? wrap_one(r, ny) : clampi(r, 0, ny - 1);
}

// T of column c (wrapped or clamped) at row r, with the ghost rules: x-ghosts
// by the lane's flags gW / gE, y-ghosts by the row
template <typename real, bool YP>
__device__ __forceinline__ real gen_T(const real* __restrict__ Tin, int P, int ny, int c, int r,
                                      bool gW, bool gE, real TwW, real TwE, bool fixS,
                                      bool fixN, real TwS, real TwN) {
  real t = Tin[gen_row<YP>(r, ny) * P + c];
  t = gW ? real(2) * TwW - t : t;
  t = gE ? real(2) * TwE - t : t;
  if (!YP) {
    t = (r < 0 && fixS) ? real(2) * TwS - t : t;
    t = (r >= ny && fixN) ? real(2) * TwN - t : t;
  }
  return t;
}

// the 9 streamed populations of node (ic, r) and its moments
template <typename real, bool XP, bool YP>
__device__ __forceinline__ void gen_pull(const real* __restrict__ fin, int nx, int ny, int P,
                                         int plane, int ic, int r, real uwW, real uwE,
                                         real uwS, real uwN, real f[9], real& drho, real& ux,
                                         real& uy) {
  const int rr = gen_row<YP>(r, ny);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    int sx = ic - ex(q), sy = rr - ey(q);
    bool ox = false, oy = false;
    if (XP) sx = wrap_one(sx, nx);
    else ox = sx < 0 || sx >= nx;
    if (YP) sy = wrap_one(sy, ny);
    else oy = sy < 0 || sy >= ny;
    const bool out = ox || oy;
    const real raw = fin[out ? opp(q) * plane + rr * P + ic : q * plane + sy * P + sx];
    const real uwall = oy ? (sy < 0 ? uwS : uwN) : (sx < 0 ? uwW : uwE);
    const real eu = oy ? real(ex(q)) * uwall : real(ey(q)) * uwall;
    f[q] = out ? raw + real(6) * wq<real>(q) * eu : raw;
  }
  moments(f, drho, ux, uy);
}

template <typename real, int CONV, bool XP, bool YP>
__device__ void march_general(const StepArgs<real>& a, int lane, int i, int j0, int j1) {
  const int nx = a.nx, ny = a.ny, P = a.pitch;
  const bool act = lane >= 1 && lane <= kOut && i < nx;
  const int ix2 = lane < 32 ? i - 2 : i + 2;  // second T column (lanes 1, 62)
  const real al = a.alpha;
  const real TwW = a.Tw[0], TwE = a.Tw[1], TwS = a.Tw[2], TwN = a.Tw[3];
  const bool fixW = a.tfix[0], fixE = a.tfix[1], fixS = a.tfix[2], fixN = a.tfix[3];
  const int plane = a.plane;
  const int ic = XP ? wrap_any(i, nx) : clampi(i, 0, nx - 1);
  const int ic2 = XP ? wrap_any(ix2, nx) : clampi(ix2, 0, nx - 1);
  // x-ghost rules of the two T columns this lane reads
  const bool g1W = !XP && i < 0 && fixW, g1E = !XP && i >= nx && fixE;
  const bool g2W = !XP && ix2 < 0 && fixW, g2E = !XP && ix2 >= nx && fixE;
  const real uwW = a.uw[0], uwE = a.uw[1], uwS = a.uw[2], uwN = a.uw[3];
  const real* __restrict__ fin = a.fin;
  const real* __restrict__ Tin = a.Tin;
  // the low-word codes of a compensated T are read from T itself (and
  // ignored) when absent, which keeps the loads unconditional
  const tlo_t* tlo = a.Tlo_in ? a.Tlo_in : (const tlo_t*)a.Tin;
#define LF_PULL(r, f, d, u, v) \
  gen_pull<real, XP, YP>(fin, nx, ny, P, plane, ic, (r), uwW, uwE, uwS, uwN, f, d, u, v)
#define LF_T1(r) gen_T<real, YP>(Tin, P, ny, ic, (r), g1W, g1E, TwW, TwE, fixS, fixN, TwS, TwN)
#define LF_T2(r) gen_T<real, YP>(Tin, P, ny, ic2, (r), g2W, g2E, TwW, TwE, fixS, fixN, TwS, TwN)

  real fc[9], fn[9];
  real dr_c, ux_c, uy_c, dr_n, ux_n, uy_n, uy_p;
  {
    real ft[9], d, u;
    LF_PULL(j0 - 1, ft, d, u, uy_p);
  }
  LF_PULL(j0, fc, dr_c, ux_c, uy_c);
  LF_PULL(j0 + 1, fn, dr_n, ux_n, uy_n);
  real t0 = LF_T1(j0 - 2), t1 = LF_T1(j0 - 1);
  real t2 = LF_T1(j0), t3 = LF_T1(j0 + 1);
  real t4 = LF_T1(j0 + 2);
  real tx2 = LF_T2(j0);
  int lo = tlo[j0 * P + ic];

  for (int j = j0; j < j1; ++j) {
    const real tW1 = __shfl_up(t2, 1, 64);
    const real tE1 = __shfl_down(t2, 1, 64);
    real tW2 = __shfl_up(t2, 2, 64);
    real tE2 = __shfl_down(t2, 2, 64);
    const real uW = __shfl_up(ux_c, 1, 64);
    const real uE = __shfl_down(ux_c, 1, 64);
    if (lane == 1) tW2 = tx2;
    if (lane == kOut) tE2 = tx2;
    const real fw = face_flux<real, CONV>(al, uW, ux_c, tW2, tW1, t2, tE1);
    const real fe = face_flux<real, CONV>(al, ux_c, uE, tW1, t2, tE1, tE2);
    const real fs = face_flux<real, CONV>(al, uy_p, uy_c, t0, t1, t2, t3);
    const real fnn = face_flux<real, CONV>(al, uy_c, uy_n, t1, t2, t3, t4);
    const real wW = fixW ? real(-2) * al * (t2 - TwW) : real(0);
    const real wE = fixE ? real(-2) * al * (TwE - t2) : real(0);
    const real wS = fixS ? real(-2) * al * (t2 - TwS) : real(0);
    const real wN = fixN ? real(-2) * al * (TwN - t2) : real(0);
    const real Fw = (!XP && i == 0) ? wW : fw;
    const real Fe = (!XP && i == nx - 1) ? wE : fe;
    const real Fs = (!YP && j == 0) ? wS : fs;
    const real Fn = (!YP && j == ny - 1) ? wN : fnn;
    real Tnew, Tlo = real(0);
    if (a.Tlo_in) {
      t_update(t2, lo_decode(t2, lo), -(Fe - Fw) - (Fn - Fs), Tnew, Tlo);
    } else {
      Tnew = t2 - (Fe - Fw) - (Fn - Fs);
    }
    if (act) {
      const int o = j * P + i;
      collide(a, fc, dr_c, ux_c, uy_c, Tnew, [&](int q, real v) { a.fout[q * plane + o] = v; });
      store_node(a, o, Tnew, dr_c, ux_c, uy_c);
      if (a.Tlo_out) a.Tlo_out[j * P + i] = (tlo_t)lo_encode(Tnew, Tlo);
    }
    if (j + 1 == j1) break;
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
    // inputs of row j + 1
    LF_PULL(j + 2, fn, dr_n, ux_n, uy_n);
    t4 = LF_T1(j + 3);
    tx2 = LF_T2(j + 1);
    lo = tlo[(j + 1) * P + ic];
  }
#undef LF_PULL
#undef LF_T1
#undef LF_T2
}

template <typename real, int CONV>
__device__ __forceinline__ void march_general_any(const StepArgs<real>& a, int lane, int i,
                                                  int j0, int j1) {
  if (!a.xper && !a.yper) march_general<real, CONV, false, false>(a, lane, i, j0, j1);
  else if (a.xper && !a.yper) march_general<real, CONV, true, false>(a, lane, i, j0, j1);
  else if (!a.xper) march_general<real, CONV, false, true>(a, lane, i, j0, j1);
  else march_general<real, CONV, true, true>(a, lane, i, j0, j1);
}

// Buffer-resource access: one descriptor per array, a per-lane byte offset
// (row * pitch + column) and a wave-uniform byte offset in an SGPR (the
// direction's plane and upstream shift), so an access costs no VALU work.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename real>
__device__ __forceinline__ real bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return __builtin_bit_cast(double, v);
}
template <typename real>
__device__ __forceinline__ void bstore(real v, __amdgpu_buffer_rsrc_t r, int voff, int soff);
// cache policy of the step's output stores (2 = non-temporal)
#ifndef LF_STORE_AUX
#define LF_STORE_AUX 0
#endif
template <>
__device__ __forceinline__ void bstore<float>(float v, __amdgpu_buffer_rsrc_t r, int voff,
                                              int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, LF_STORE_AUX);
}
template <>
__device__ __forceinline__ void bstore<double>(double v, __amdgpu_buffer_rsrc_t r, int voff,
                                               int soff) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, LF_STORE_AUX);
}

// Interior march: every pulled node, its upstream nodes and the T stencil
// lie inside the grid and no face is a wall.  Each lane evaluates only the
// east face of its cell (the west face is the east face of the lane to the
// left) and the north face (the south face is the previous row's north
// face), and the next row's populations are requested one row ahead.
//
// DIR is the march direction: +1 up from j0, -1 down from j1 - 1.  Bands
// alternate, so the two waves on either side of a band boundary pull its
// shared rows at the same time (both at their start or both at their end)
// and the second pull hits in L2.  A node's arithmetic does not depend on
// the direction: the face between rows r and r + 1 is always evaluated
// from (v_r, v_r+1, T_r-1 .. T_r+2) in that order.
//
// SIDE 1 / 2: the strip holds the west / east wall (rows still clear of the
// south and north walls), with the wall-adjacent column an output lane and
// the column beyond it a lane of the wave.  The march is the interior one
// plus the general march's wall rules, with the same arithmetic: the three
// links of the wall lane that cross the wall take the node's own reversed
// population plus 6 w_q (e_q . u_w) (these three loads carry their whole
// shift in the per-lane offset: the link's upstream shift, or on the wall
// lane its own reversed plane; both are non-negative, as the buffer's range
// check needs),
// the lane beyond the wall carries the ghost T (2 T_w - T_edge fixed,
// T_edge adiabatic) for its neighbours' stencils, and the wall face takes
// the wall rule.  Lanes beyond the wall compute values nobody keeps.
template <typename real, int CONV, int DIR, int SIDE = 0>
__device__ void march_interior(const StepArgs<real>& a, int lane, int i, int j0, int j1) {
  static_assert(DIR == 1 || DIR == -1, "march direction");
  static_assert(SIDE >= 0 && SIDE <= 2, "side wall");
  constexpr int es = sizeof(real);
  const int P = a.pitch;
  const bool act = lane >= 1 && lane <= kOut && (SIDE != 2 || i < a.nx);
  // the wall-adjacent lane and the lane beyond the wall
  const bool wlane = SIDE == 1 ? i == 0 : SIDE == 2 ? i == a.nx - 1 : false;
  const bool glane = SIDE == 1 ? i == -1 : SIDE == 2 ? i == a.nx : false;
  // links crossing the wall (pulled from beyond it) and their reverses
  constexpr int xq0 = SIDE == 2 ? 3 : 1, xq1 = SIDE == 2 ? 6 : 5, xq2 = SIDE == 2 ? 7 : 8;
  const real uwall = SIDE == 2 ? a.uw[1] : a.uw[0];
  const bool wfix = SIDE == 2 ? a.tfix[1] : a.tfix[0];
  const real wallT = SIDE == 2 ? a.Tw[1] : a.Tw[0];
  const unsigned fbytes = 9u * (unsigned)a.plane * es, pbytes = (unsigned)a.plane * es;
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(a.fin, fbytes);
  const __amdgpu_buffer_rsrc_t rT = make_rsrc(a.Tin, pbytes);
  const __amdgpu_buffer_rsrc_t wf = make_rsrc(a.fout, fbytes);
  const __amdgpu_buffer_rsrc_t wT = make_rsrc(a.Tout, pbytes);
  // low-word codes of a compensated T, one byte per node (read from T
  // itself, and ignored, when absent)
  const __amdgpu_buffer_rsrc_t rL =
      make_rsrc(a.Tlo_in ? (const void*)a.Tlo_in : (const void*)a.Tin, (unsigned)a.plane);
  const __amdgpu_buffer_rsrc_t wL =
      make_rsrc(a.Tlo_out ? (const void*)a.Tlo_out : (const void*)a.Tout, (unsigned)a.plane);
  int sq[9];  // uniform byte offset of direction q's upstream node
#pragma unroll
  for (int q = 0; q < 9; ++q) sq[q] = (q * a.plane - ey(q) * P - ex(q)) * es;
  // lane 0 needs T one column further west, lane 62 one further east
  const int xoff = (lane < 32 ? -1 : 2) * es;
  const real al = a.alpha;

  // byte shifts of the crossing links: the upstream shift sq[q], or on the
  // wall lane the node's own reversed population (plane opp(q))
  int xs[3] = {0, 0, 0};
  if constexpr (SIDE != 0) {
    xs[0] = wlane ? opp(xq0) * a.plane * es : sq[xq0];
    xs[1] = wlane ? opp(xq1) * a.plane * es : sq[xq1];
    xs[2] = wlane ? opp(xq2) * a.plane * es : sq[xq2];
  }
  auto load_row = [&](int r, real f[9]) {
    const int vo = (r * P + i) * es;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      if (SIDE != 0 && (q == xq0 || q == xq1 || q == xq2))
        f[q] = bload<real>(rf, vo + (q == xq0 ? xs[0] : q == xq1 ? xs[1] : xs[2]), 0);
      else
        f[q] = bload<real>(rf, vo, sq[q]);
    }
  };
  // the wall lane's crossing links: reversed population + moving-wall term
  auto wall_fix = [&](real f[9]) {
    if constexpr (SIDE != 0) {
      const real e0 = real(ey(xq0)) * uwall, e1 = real(ey(xq1)) * uwall,
                 e2 = real(ey(xq2)) * uwall;
      f[xq0] = wlane ? f[xq0] + real(6) * wq<real>(xq0) * e0 : f[xq0];
      f[xq1] = wlane ? f[xq1] + real(6) * wq<real>(xq1) * e1 : f[xq1];
      f[xq2] = wlane ? f[xq2] + real(6) * wq<real>(xq2) * e2 : f[xq2];
    }
  };
  auto T_row = [&](int r) { return bload<real>(rT, (r * P + i) * es, 0); };
  // first output row; rows "behind" it are r - DIR, rows "ahead" r + DIR
  const int js = DIR > 0 ? j0 : j1 - 1;
  auto inside = [&](int r) { return DIR > 0 ? r < j1 : r >= j0; };
  // rows whose populations are pulled: the band and one row beyond each end
  auto pulled = [&](int r) { return DIR > 0 ? r <= j1 : r >= j0 - 1; };

  // rows js-D .. js+2D requested up front; row j+3D is requested while row j
  // is computed (two rows ahead).  Four arrays rotate by unrolling.
  real A[9], B[9], C[9], D[9];
  real dr_c, ux_c, uy_c, uy_p, d_unused, u_unused;
  load_row(js - DIR, D);
  load_row(js, A);
  load_row(js + DIR, B);
  if (pulled(js + 2 * DIR)) load_row(js + 2 * DIR, C);
  const real tm2 = T_row(js - 2 * DIR);
  real t1 = T_row(js - DIR), t2 = T_row(js), t3 = T_row(js + DIR), t4 = T_row(js + 2 * DIR);
  const int r5 = js + 3 * DIR;
  real t5 = T_row((DIR > 0 ? r5 < a.ny : r5 >= 0) ? r5 : js + 2 * DIR);
  // the column beyond the halo lanes and the low words, one row ahead
  auto tx_row = [&](int r) { return bload<real>(rT, (r * P + i) * es + xoff, 0); };
  // (the column is the per-lane offset, the row a wave-uniform one)
  auto lo_row = [&](int r) {
    return (int)(signed char)__builtin_amdgcn_raw_buffer_load_b8(rL, i, r * P, 0);
  };
  real txa = tx_row(js);
  int loa = lo_row(js);
  wall_fix(D);
  wall_fix(A);
  moments(D, d_unused, u_unused, uy_p);
  moments(A, dr_c, ux_c, uy_c);
  // the face behind the first row
  real Fb = DIR > 0 ? face_flux<real, CONV>(al, uy_p, uy_c, tm2, t1, t2, t3)
                    : face_flux<real, CONV>(al, uy_c, uy_p, t3, t2, t1, tm2);

  auto row = [&](int j, const real (&fc)[9], real (&fn)[9], real (&fl)[9]) {
    if (pulled(j + 3 * DIR)) load_row(j + 3 * DIR, fl);  // two rows ahead
    real dr_n, ux_n, uy_n;
    wall_fix(fn);
    moments(fn, dr_n, ux_n, uy_n);
    const real tx = txa;
    const int lo = loa;
    if (inside(j + DIR)) {
      txa = tx_row(j + DIR);
      loa = lo_row(j + DIR);
    }
    if constexpr (SIDE != 0) {  // the ghost T beyond the wall
      const real te = SIDE == 1 ? __shfl_down(t2, 1, 64) : __shfl_up(t2, 1, 64);
      t2 = glane ? (wfix ? real(2) * wallT - te : te) : t2;
    }
    real tW1 = __shfl_up(t2, 1, 64);
    const real tE1 = __shfl_down(t2, 1, 64);
    real tE2 = __shfl_down(t2, 2, 64);
    const real uE = __shfl_down(ux_c, 1, 64);
    if (lane == 0) tW1 = tx;
    if (lane == kOut) tE2 = tx;
    real Fe = face_flux<real, CONV>(al, ux_c, uE, tW1, t2, tE1, tE2);
    real Fw = __shfl_up(Fe, 1, 64);
    if constexpr (SIDE == 1) {
      const real wW = wfix ? real(-2) * al * (t2 - wallT) : real(0);
      Fw = wlane ? wW : Fw;
    } else if constexpr (SIDE == 2) {
      const real wE = wfix ? real(-2) * al * (wallT - t2) : real(0);
      Fe = wlane ? wE : Fe;
    }
    // the face ahead; north minus south either way
    const real Fa = DIR > 0 ? face_flux<real, CONV>(al, uy_c, uy_n, t1, t2, t3, t4)
                            : face_flux<real, CONV>(al, uy_n, uy_c, t4, t3, t2, t1);
    const real dFy = DIR > 0 ? Fa - Fb : Fb - Fa;
    real Tnew, Tlo = real(0);
    if (a.Tlo_in) {
      t_update(t2, lo_decode(t2, lo), -(Fe - Fw) - dFy, Tnew, Tlo);
    } else {
      Tnew = t2 - (Fe - Fw) - dFy;
    }
    if (act) {
      const int vo = (j * P + i) * es;
      collide(a, fc, dr_c, ux_c, uy_c, Tnew,
              [&](int q, real v) { bstore<real>(v, wf, vo, q * a.plane * es); });
      if (a.Tlo_out)
        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)lo_encode(Tnew, Tlo), wL, i, j * P,
                                             LF_STORE_AUX);
      bstore<real>(Tnew, wT, vo, 0);
      if (a.mom) {
        const int o = j * P + i;
        a.mom[o] = real(1) + dr_c;
        a.mom[a.plane + o] = ux_c;
        a.mom[2 * a.plane + o] = uy_c;
      }
    }
    Fb = Fa;
    uy_p = uy_c;
    dr_c = dr_n;
    ux_c = ux_n;
    uy_c = uy_n;
    t1 = t2;
    t2 = t3;
    t3 = t4;
    t4 = t5;
    const int r4 = j + 4 * DIR;
    if (DIR > 0 ? r4 < a.ny : r4 >= 0) t5 = T_row(r4);
  };
  for (int j = js; inside(j); j += 4 * DIR) {
    row(j, A, B, D);
    if (!inside(j + DIR)) break;
    row(j + DIR, B, C, A);
    if (!inside(j + 2 * DIR)) break;
    row(j + 2 * DIR, C, D, B);
    if (!inside(j + 3 * DIR)) break;
    row(j + 3 * DIR, D, A, C);
  }
}

// Order of the step kernels' blocks over the 8 XCDs (blocks are dealt to
// them round-robin: block b runs on XCD b mod 8).  Renumbered so that each
// XCD works on neighbouring strips and bands, whose shared halo lines then
// stay in one L2: below kXcdChunkFrom blocks each XCD takes one contiguous
// eighth of the grid, from it on the XCDs take turns in chunks of
// kXcdChunk blocks.  Measured (contiguous eighths / chunks of 64 / the plain
// order): the 256-cavity sweep (53 k blocks) 0.957 / 0.935 / 1.016 ms,
// 4096^2 (17 k) 321 / 313 / 336 us, 3072^2 (9.6 k) 185.7 / 182.3 us, 2560^2
// (6.7 k) 131.3 / 132.9 us, 2048^2 (4.4 k) 85.6 / 90.7 / 94.6 us, 512^2
// (1.2 k) 6.7 / 7.4 / 9.7 us.
constexpr int kXcdChunk = 64;
constexpr int kXcdChunkFrom = 8192;
__device__ __forceinline__ int xcd_order(int b, int nb) {
  if (nb >= kXcdChunkFrom) {
    const int full = nb / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (b >= full) return b;  // the last partial round keeps the plain order
    const int x = b % 8, k = b / 8;
    return ((k / kXcdChunk) * 8 + x) * kXcdChunk + k % kXcdChunk;
  }
  const int per = nb / 8, rem = nb % 8, x = b % 8;
  return x * per + (x < rem ? x : rem) + b / 8;
}

// ROW1: every wave forms one row (a.band == 1).
template <typename real, int CONV, bool ROW1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LF_STEP_WAVES(real, ROW1))))
void k_hybrid_step(StepArgs<real> a) {
  // XCD-aware block order (xcd_order)
  const int lb = xcd_order((int)blockIdx.x, (int)gridDim.x);
  // uniform per wave: held in an SGPR, so are the strip, band and row bounds
  const int wave = __builtin_amdgcn_readfirstlane(lb * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wave >= a.nwaves) return;
  const int strip = wave % a.nstrips;
  const int bnd = wave / a.nstrips;
  const int lane = threadIdx.x & 63;
  const int c0 = strip * kOut;   // first output column
  const int i = c0 + lane - 1;   // this lane's column
  const int band = ROW1 ? 1 : a.band;
  const int j0 = bnd * band;
  const int j1 = ROW1 ? j0 + 1 : min(j0 + band, a.ny);
  const bool rows_in = j0 - 1 >= 2 && j1 <= a.ny - 2;
  // strips holding the west / east wall: the wall column an output lane with
  // room for the column beyond it, and no periodic seam
  const bool west = !a.xper && c0 == 0 && kOut <= a.nx - 2;
  const bool east = !a.xper && c0 - 1 >= 1 && a.nx - c0 <= kOut - 2;
  if (rows_in && c0 - 1 >= 1 && c0 + kOut <= a.nx - 2) {
    if (bnd & 1) march_interior<real, CONV, -1>(a, lane, i, j0, j1);
    else march_interior<real, CONV, 1>(a, lane, i, j0, j1);
  } else if (rows_in && west) {  // upward only: a downward instance spills registers
    march_interior<real, CONV, 1, 1>(a, lane, i, j0, j1);
  } else if (rows_in && east) {
    march_interior<real, CONV, 1, 2>(a, lane, i, j0, j1);
  } else {
    // The general march does about 2.6x the interior work per row and its
    // waves (the rows along the south and north walls) end last; all waves
    // are resident from the start on small grids, so they set the step time.
    // Raising their issue priority lets them finish alongside the rest
    // (512^2: 8.5 -> 7.6 us; skipping them outright would give 7.2 us).
    __builtin_amdgcn_s_setprio(3);
    march_general_any<real, CONV>(a, lane, i, j0, j1);
  }
}

// ---------------------------------------------------------------------------
// Batched step: many cavities, one launch.  The work list is a table of
// tiles (cavity, strip, first row, end row); each wave takes one tile and
// runs exactly the march of the single-cavity kernel on it, with the
// cavity's geometry, parameters and buffers read from a descriptor table in
// device memory (wave-uniform, so they land in scalar registers).  Buffer
// [cur ^ parity] is read and [cur ^ parity ^ 1] written, so a sequence of
// launches with alternating parity can be captured in a graph once and
// replayed; the number of live tiles is read from device memory, so the
// same graph serves a shrinking set of unconverged cavities.
// The batched kernel is compiled for 4 waves per SIMD (up to 128 VGPRs): with
// the side-wall marches it needs 120 and would spill at 5.  Measured on the
// 256-cavity sweep, 1.076 ms per step at 4 waves with the side-wall marches
// against 1.131 ms at 5 waves with the general march on those strips.  When
// every live tile is a single row (ROW1: a small live set), nothing is held
// ahead and the kernel fits 5 waves.
#define LF_BATCH_WAVES(real, ROW1) (sizeof(real) == 4 ? ((ROW1) ? 5 : 4) : 2)

template <typename real, int CONV, bool ROW1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LF_BATCH_WAVES(real, ROW1))))
void k_batch_step(const TileDesc* __restrict__ tiles, const int* __restrict__ ntiles,
                  const CavDesc<real>* __restrict__ cavs, int parity, int write_mom) {
  // The grid covers the live tile table (between one and two times its
  // size, so a graph captured for it serves a shrinking set); only the
  // first ceil(live / waves-per-block) blocks have work.
  // Those are spread round-robin over the 8 XCDs, so the XCD-aware order
  // (xcd_order) is taken over them alone: taken over the whole grid it
  // would hand every live tile to the first XCDs.
  const int wpb = blockDim.x >> 6;
  const int live = *ntiles;
  const int nb = (live + wpb - 1) / wpb, b = blockIdx.x;
  if (b >= nb) return;
  const int lb = xcd_order(b, nb);
  // the wave index is uniform; telling the compiler so makes the tile and
  // cavity descriptors scalar loads held in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(lb * wpb + (threadIdx.x >> 6));
  if (wave >= live) return;  // uniform per wave
  const TileDesc t = tiles[wave];
  const CavDesc<real>& cd = cavs[t.cav];
  StepArgs<real> a;
  const int in = cd.cur ^ parity;
  a.fin = cd.f[in];
  a.fout = cd.f[in ^ 1];
  a.Tin = cd.T[in];
  a.Tout = cd.T[in ^ 1];
  a.Tlo_in = cd.Tlo[in];
  a.Tlo_out = cd.Tlo[in ^ 1];
  a.mom = write_mom ? cd.mom : nullptr;
  a.plane = cd.plane;
  a.nx = cd.nx;
  a.ny = cd.ny;
  a.pitch = cd.pitch;
  a.band = t.j1 - t.j0;
  a.nstrips = 0;
  a.nwaves = 0;
  a.xper = 0;
  a.yper = 0;
  a.conv = CONV;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a.tfix[k] = cd.tfix[k];
    a.uw[k] = real(cd.uw[k]);
    a.Tw[k] = real(cd.Tw[k]);
  }
  a.omega = real(cd.omega);
  a.alpha = real(cd.alpha);
  a.gbeta = real(cd.gbeta);
  a.Tref = real(cd.Tref);
  a.gx = real(0);
  a.gy = real(0);
  const int lane = threadIdx.x & 63;
  const int c0 = t.strip * kOut;
  const int i = c0 + lane - 1;
  const int j0 = t.j0, j1 = ROW1 ? t.j0 + 1 : t.j1;
  const bool rows_in = j0 - 1 >= 2 && j1 <= a.ny - 2;
  const bool interior = c0 - 1 >= 1 && c0 + kOut <= a.nx - 2 && rows_in;
  // strips holding the west / east wall, as in the single-cavity kernel
  const bool west = c0 == 0 && kOut <= a.nx - 2;
  const bool east = c0 - 1 >= 1 && a.nx - c0 <= kOut - 2;
  // march direction alternates with the band index (a cavity's last, shorter
  // band may share its neighbour's direction; only cache reuse depends on it)
  if (interior) {
    if ((j0 / (j1 - j0)) & 1) march_interior<real, CONV, -1>(a, lane, i, j0, j1);
    else march_interior<real, CONV, 1>(a, lane, i, j0, j1);
  } else if (rows_in && west) {
    march_interior<real, CONV, 1, 1>(a, lane, i, j0, j1);
  } else if (rows_in && east) {
    march_interior<real, CONV, 1, 2>(a, lane, i, j0, j1);
  } else {
    march_general<real, CONV, false, false>(a, lane, i, j0, j1);  // batches: no periodic sides
  }
}

// Batched residual, pass 1: one block per (cavity, row range); six FP64
// sums and a non-finite count per block, snapshot updated.
template <typename real>
__global__ __launch_bounds__(256) void k_batch_resid(const ResidTile* __restrict__ rt,
                                                     const int* __restrict__ nrt,
                                                     const CavDesc<real>* __restrict__ cavs,
                                                     double* __restrict__ part) {
  if ((int)blockIdx.x >= *nrt) return;
  __shared__ double sh[4][7];
  const ResidTile t = rt[blockIdx.x];
  const CavDesc<real>& cd = cavs[t.cav];
  const real* mom = cd.mom;
  const real* T = cd.T[cd.cur];
  real* snap = cd.snap;
  const int P = cd.plane;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int j = t.j0; j < t.j1; ++j)
    for (int i = threadIdx.x; i < cd.nx; i += 256) {
      const int o = j * cd.pitch + i;
      const double u = (double)mom[P + o], v = (double)mom[2 * P + o], tt = (double)T[o];
      const double su = (double)snap[o], sv = (double)snap[P + o], st = (double)snap[2 * P + o];
      acc[0] += (u - su) * (u - su);
      acc[1] += u * u;
      acc[2] += (v - sv) * (v - sv);
      acc[3] += v * v;
      acc[4] += (tt - st) * (tt - st);
      acc[5] += tt * tt;
      if (!(isfinite(u) && isfinite(v) && isfinite(tt))) acc[6] += 1.0;
      snap[o] = mom[P + o];
      snap[P + o] = mom[2 * P + o];
      snap[2 * P + o] = T[o];
    }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) sh[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k)
      part[blockIdx.x * 8 + k] = ((sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]));
}

// Batched residual, pass 2: per live cavity, its blocks' partials in order.
__global__ __launch_bounds__(256) void k_batch_fold(const FoldDesc* __restrict__ fd,
                                                    const int* __restrict__ nfold,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= *nfold) return;
  const FoldDesc d = fd[k];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = 0; b < d.count; ++b)
    for (int q = 0; q < 7; ++q) acc[q] += part[(d.start + b) * 8 + q];
  for (int q = 0; q < 7; ++q) out[d.cav * 8 + q] = acc[q];
}

// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_init(int nx, int ny, int pitch, int plane,
                                              const double* __restrict__ T0,
                                              const double* __restrict__ u0,
                                              const double* __restrict__ v0,
                                              real* __restrict__ f, real* __restrict__ T,
                                              real* __restrict__ mom,
                                              real* __restrict__ snap,
                                              tlo_t* __restrict__ Tlo) {
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
  if (Tlo) Tlo[o] = (tlo_t)lo_encode(real(t), real(t - (double)real(t)));
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
                              const tlo_t* Tlo_in, tlo_t* Tlo_out, real* mom, int band,
                              hipStream_t s) {
  StepArgs<real> a;
  a.Tlo_in = Tlo_in;
  a.Tlo_out = Tlo_out;
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
  if (a.band == 1) {
    if (p.conv == 1)
      hipLaunchKernelGGL((k_hybrid_step<real, 1, true>), dim3(blocks), dim3(256), 0, s, a);
    else if (p.conv == 2)
      hipLaunchKernelGGL((k_hybrid_step<real, 2, true>), dim3(blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_hybrid_step<real, 0, true>), dim3(blocks), dim3(256), 0, s, a);
  } else {
    if (p.conv == 1)
      hipLaunchKernelGGL((k_hybrid_step<real, 1, false>), dim3(blocks), dim3(256), 0, s, a);
    else if (p.conv == 2)
      hipLaunchKernelGGL((k_hybrid_step<real, 2, false>), dim3(blocks), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_hybrid_step<real, 0, false>), dim3(blocks), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <typename real>
hipError_t launch_init(const Grid& g, const double* T0, const double* u0, const double* v0,
                       real* f, real* T, real* mom, real* snap, tlo_t* Tlo, hipStream_t s) {
  dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL(k_init<real>, grid, dim3(256), 0, s, g.nx, g.ny, g.pitch,
                     (int)g.plane, T0, u0, v0, f, T, mom, snap, Tlo);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_batch_step(const TileDesc* tiles, const int* ntiles, int max_tiles,
                             const CavDesc<real>* cavs, int parity, int write_mom, int conv,
                             int row1, hipStream_t s) {
  const int blocks = (max_tiles + 3) / 4;
  if (blocks < 1) return hipSuccess;
#define LF_BATCH_LAUNCH(C, R1)                                                                \
  hipLaunchKernelGGL((k_batch_step<real, C, R1>), dim3(blocks), dim3(256), 0, s, tiles, ntiles, \
                     cavs, parity, write_mom)
  if (row1) {
    if (conv == 1) LF_BATCH_LAUNCH(1, true);
    else if (conv == 2) LF_BATCH_LAUNCH(2, true);
    else LF_BATCH_LAUNCH(0, true);
  } else {
    if (conv == 1) LF_BATCH_LAUNCH(1, false);
    else if (conv == 2) LF_BATCH_LAUNCH(2, false);
    else LF_BATCH_LAUNCH(0, false);
  }
#undef LF_BATCH_LAUNCH
  return hipGetLastError();
}

template <typename real>
hipError_t launch_batch_residual(const ResidTile* rt, const int* nrt, int max_rt,
                                 const FoldDesc* fd, const int* nfold, int max_fold,
                                 const CavDesc<real>* cavs, double* part, double* out,
                                 hipStream_t s) {
  if (max_rt < 1 || max_fold < 1) return hipSuccess;
  hipLaunchKernelGGL(k_batch_resid<real>, dim3(max_rt), dim3(256), 0, s, rt, nrt, cavs, part);
  hipLaunchKernelGGL(k_batch_fold, dim3((max_fold + 255) / 256), dim3(256), 0, s, fd, nfold,
                     part, out);
  return hipGetLastError();
}

template hipError_t launch_batch_step<float>(const TileDesc*, const int*, int,
                                             const CavDesc<float>*, int, int, int, int,
                                             hipStream_t);
template hipError_t launch_batch_step<double>(const TileDesc*, const int*, int,
                                              const CavDesc<double>*, int, int, int, int,
                                              hipStream_t);
template hipError_t launch_batch_residual<float>(const ResidTile*, const int*, int, const FoldDesc*,
                                                 const int*, int, const CavDesc<float>*, double*,
                                                 double*, hipStream_t);
template hipError_t launch_batch_residual<double>(const ResidTile*, const int*, int,
                                                  const FoldDesc*, const int*, int,
                                                  const CavDesc<double>*, double*, double*,
                                                  hipStream_t);
template hipError_t launch_hybrid_step<float>(const Grid&, const WallSet&, const HybridParams&,
                                              const float*, float*, const float*, float*,
                                              const tlo_t*, tlo_t*, float*, int, hipStream_t);
template hipError_t launch_hybrid_step<double>(const Grid&, const WallSet&, const HybridParams&,
                                               const double*, double*, const double*, double*,
                                               const tlo_t*, tlo_t*, double*, int, hipStream_t);
template hipError_t launch_init<float>(const Grid&, const double*, const double*, const double*,
                                       float*, float*, float*, float*, tlo_t*, hipStream_t);
template hipError_t launch_init<double>(const Grid&, const double*, const double*, const double*,
                                        double*, double*, double*, double*, tlo_t*, hipStream_t);

}  // namespace lf
