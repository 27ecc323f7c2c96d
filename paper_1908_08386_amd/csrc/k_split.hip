// k_split.hip -- domain-decomposed LBM|FVM step (Sec. 4 of Li, Yang & Zhang,
// arXiv:1908.08386) for gfx950.
//
// Layout (one cavity, nx even, s = nx / 2):
//   LBM zone   nodes  0 .. ib (ib = s + 1, the artificial boundary x_b),
//              D2Q9 populations f (stored shifted, f - w_q) and D2Q5 g,
//              [q][ny][pitch_L] planes, ping-pong buffers;
//   FV zone    cells  c0 .. nx-1 (c0 = s - 1) on a staggered grid, stored
//              for columns c0-2 .. nx (two ghost columns in the LBM zone
//              and the east wall face): u on x-faces [ny][pitch_F], v on
//              y-faces [ny+1][pitch_F], p and T at centres [ny][pitch_F];
//   shared columns c0, c0+1, c0+2 = ib.
// One step is three launches on one stream:
//   k_dd_fv       the interior of the FV zone in one pass: u*, v* (QUICK
//                 convection, central diffusion, pressure gradient,
//                 buoyancy; Eq 74-75 explicit), then p <- p - c_s^2 div u*
//                 and the conservative QUICK energy balance on u* (Eq 76);
//                 the frame of faces and cells the walls' mirror and ghost
//                 rules or the inflow face reach is formed by other blocks of
//                 the same launch;
//   k_dd_lbm      pull-stream + bounce-back / anti-bounce-back walls,
//                 moments, BGK collision with buoyancy from T = sum g
//                 (Eq 5, 18, 19-23) for nodes 0 .. ib-1; the streamed state
//                 of x_f = ib-1 is kept for the boundary node; one more
//                 column of blocks sums, per 256 rows, the new FV pressure
//                 over the shared columns (p_bar) and the mass the LBM zone
//                 gains through the links to x_b in this step (its running
//                 total is the zone's mass change since init: the walls
//                 conserve mass);
//   k_dd_xb       x_b from the FV zone: rho_b by Eq 93 with its level
//                 shifted to hold the LBM zone's mass, u_b, v_b, T_b by
//                 face averages, populations by non-equilibrium
//                 extrapolation (Eq 60 / Eq 94-95) or by the
//                 finite-difference velocity-gradient closure (Eq 70-72);
//                 then its collision; then the ghost columns of the next
//                 step's FV zone from the LBM moments (two-point averages;
//                 the mean of the inflow face is removed: global continuity
//                 of the FV zone) and the sums for the next rho0 = mean LBM
//                 density over the shared columns (Eq 91-93).
// The north wall may slide along +x (the lid-driven cavity of Sec. 3.3):
// moving-wall bounce-back in the LBM zone, ghost u = 2 u_lid - u_edge in the
// FV zone.
// The LBM zone is 112 B per node (FP32), the FV zone 32 B per cell (u, v, p,
// T read and written once); the interface work is O(ny).  The interface's
// sums over all rows are per-block sums that each consumer adds in block
// order itself, so no launch is spent on folding them.
// The single-method cavities of the Sec. 4.2 comparison run the same zone
// kernels on the whole box: FV only (momentum + pressure/energy, with the
// west wall's mirror and ghost rules) or LBM only (k_dd_lbm with an east
// wall), without the interface launches.
#include "lf_internal.h"

#pragma clang fp contract(off)

namespace lf {
namespace {

__host__ __device__ constexpr int ex9(int q) {
  return (q == 1 || q == 5 || q == 8) ? 1 : (q == 3 || q == 6 || q == 7) ? -1 : 0;
}
__host__ __device__ constexpr int ey9(int q) {
  return (q == 2 || q == 5 || q == 6) ? 1 : (q == 4 || q == 7 || q == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp9(int q) {
  return q == 0 ? 0 : q < 5 ? ((q + 1) % 4) + 1 : ((q - 3) % 4) + 5;
}
template <typename real>
__host__ __device__ constexpr real w9(int q) {
  return q == 0 ? real(4) / real(9) : q < 5 ? real(1) / real(9) : real(1) / real(36);
}
// D2Q5 (Eq 22): 0 rest, 1 E, 2 N, 3 W, 4 S
__host__ __device__ constexpr int ex5(int q) { return q == 1 ? 1 : q == 3 ? -1 : 0; }
__host__ __device__ constexpr int ey5(int q) { return q == 2 ? 1 : q == 4 ? -1 : 0; }
__host__ __device__ constexpr int opp5(int q) { return q == 0 ? 0 : ((q + 1) % 4) + 1; }
template <typename real>
__host__ __device__ constexpr real w5(int q) {
  return q == 0 ? real(1) / real(3) : real(1) / real(6);
}

template <typename real>
__device__ __forceinline__ real fmad(real a, real b, real c) {
  return __builtin_fma(a, b, c);
}
template <>
__device__ __forceinline__ float fmad<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}

// shifted f_eq: f_eq - w = w (drho + rho P), P = 3 e.u + 9/2 (e.u)^2 - 3/2 u.u
template <typename real>
__device__ __forceinline__ real feq_s(int q, real drho, real ux, real uy) {
  const real rho = real(1) + drho;
  const real eu = real(ex9(q)) * ux + real(ey9(q)) * uy;
  const real P = fmad(real(4.5) * eu, eu, real(3) * eu) - real(1.5) * fmad(ux, ux, uy * uy);
  return w9<real>(q) * fmad(rho, P, drho);
}

// gains of the level of Eq 93 on the LBM zone's mass deficit and on its
// running sum over the steps
constexpr double kLevelP = 0.25, kLevelI = 1.0 / 64.0;

template <typename real>
struct SplitArgs {
  // LBM zone
  const real* __restrict__ fin;
  real* __restrict__ fout;
  const real* __restrict__ gin;
  real* __restrict__ gout;
  real* __restrict__ mom;  // rho, u, v, T planes of the LBM zone
  real* __restrict__ xf;   // streamed state of column ib-1: 9 f + 5 g + rho u v T per row
  int pL, planeL, nl;      // pitch, plane size, LBM columns (ib + 1)
  // FV zone (stored columns c0-2 .. nx)
  const real* __restrict__ u;
  const real* __restrict__ v;
  const real* __restrict__ T;
  real* __restrict__ us;  // u*
  real* __restrict__ vs;  // v*
  real* __restrict__ Tn;
  const real* __restrict__ pin;  // pressure of the last step
  real* __restrict__ p;          // pressure of this step
  int pF;
  // interface scalars and per-block sums (layout at kIfacePart)
  double* __restrict__ iface;
  int nx, ny, s, c0, ib;
  // grid setting 2: coarse planes (see SplitPtrs::gc), sizes and pitch
  real* __restrict__ gc[10];
  int NXc, NYc, pC;
  int* __restrict__ mcm_count;
  unsigned long long* __restrict__ mcm_stats;
  int gdir;        // gravity along -y (0) or along -x (1, the transposed horizontal division)
  int transposed;  // fields are handed in and out transposed (user x = stored y)
  int west_wall;  // FV zone closed by a wall at x = 0 (FV-only cavity)
  int east_wall;  // LBM zone closed by a wall at x = nx (LBM-only cavity)
  int kind, mom_all;
  int par;       // parity of the step (the buffer set read), selects the interface's slots
  int iface_on;  // the divided cavity (interface launches and sums)
  // mean velocity of the inflow face over its rows, removed from the stored
  // inflow face (column c0 of u) wherever the FV step reads it (global
  // continuity of the FV zone); formed at the start of the FV launch
  real umean;
  real omega, omegaT, tau, nu, alpha, gbeta, Tref;
  real ulid;  // north wall velocity along +x
  int tfix[4];
  real Tw[4];
};

// ---- FV-zone accessors (real column x, ghost rules of the walls) -------
template <typename real>
__device__ __forceinline__ int fidx(const SplitArgs<real>& a, int x) {
  return x - (a.c0 - 2);
}
// corr: subtracted from the stored inflow face (column c0), see umean
template <typename real>
__device__ __forceinline__ real U_at(const SplitArgs<real>& a, const real* u, int x, int j,
                                     real corr = real(0)) {
  real sg = real(1), lid = real(0);
  if (j < 0) { j = -1 - j; sg = -sg; }
  else if (j >= a.ny) { j = 2 * a.ny - 1 - j; sg = -sg; lid = real(2) * a.ulid; }
  if (x > a.nx) { x = 2 * a.nx - x; sg = -sg; }
  else if (x < 0 && a.west_wall) { x = -x; sg = -sg; }
  return lid + sg * (u[j * a.pF + fidx(a, x)] - (x == a.c0 ? corr : real(0)));
}
template <typename real>
__device__ __forceinline__ real V_at(const SplitArgs<real>& a, const real* v, int x, int jf) {
  real sg = real(1);
  if (jf < 0) { jf = -jf; sg = -sg; }
  else if (jf > a.ny) { jf = 2 * a.ny - jf; sg = -sg; }
  if (x >= a.nx) { x = 2 * a.nx - 1 - x; sg = -sg; }
  else if (x < 0 && a.west_wall) { x = -1 - x; sg = -sg; }
  return sg * v[jf * a.pF + fidx(a, x)];
}
template <typename real>
__device__ __forceinline__ real T_at(const SplitArgs<real>& a, const real* T, int x, int j) {
  const int jj = j < 0 ? 0 : (j >= a.ny ? a.ny - 1 : j);
  real t;
  if (x >= a.nx) {
    t = T[jj * a.pF + fidx(a, a.nx - 1)];
    if (a.tfix[1]) t = real(2) * a.Tw[1] - t;
  } else if (x < 0 && a.west_wall) {
    t = T[jj * a.pF + fidx(a, 0)];
    if (a.tfix[0]) t = real(2) * a.Tw[0] - t;
  } else {
    t = T[jj * a.pF + fidx(a, x)];
  }
  if (j < 0 && a.tfix[2]) t = real(2) * a.Tw[2] - t;
  if (j >= a.ny && a.tfix[3]) t = real(2) * a.Tw[3] - t;
  return t;
}
template <typename real>
__device__ __forceinline__ real P_at(const SplitArgs<real>& a, int x, int j) {
  return a.pin[j * a.pF + fidx(a, x)];
}

// Interface scalars and sums (FP64, one array):
//   [2 + 2 p], [3 + 2 p]  the LBM zone's mass change since init and its
//                         running sum, read by the step of parity p (the
//                         step writes them for the next one into the other
//                         pair, so no block reads what another one writes);
//   from kIfacePart       per unit of kIfBlock rows: the ghost sums of the
//                         steps of parity 0 and of parity 1 (inflow face,
//                         density over the shared columns), then the p_bar
//                         sums (pressure over the shared columns, mass flux).
// Every consumer folds the per-unit sums itself, in one fixed order (fold_units),
// so all of them hold the same bits and no launch is spent on folding.  A
// unit is one wave, a thread per row: every access of the interface's
// kernels is row-strided (a cache line per value), so small units spread
// those lines over many CUs.
constexpr int kIfacePart = 8;
constexpr int kIfBlock = 64;  // rows per interface unit (one wave, one thread per row)

__host__ __device__ __forceinline__ int iface_blocks(int ny) {
  return (ny + 1 + kIfBlock - 1) / kIfBlock;  // rows and y-faces 0 .. ny
}
__device__ __forceinline__ double* ghost_sums(double* iface, int ny, int parity) {
  return iface + kIfacePart + 2 * iface_blocks(ny) * (parity & 1);
}
__device__ __forceinline__ double* pbar_sums(double* iface, int ny) {
  return iface + kIfacePart + 4 * iface_blocks(ny);
}

// Sums of two per-row terms over a unit's rows (one wave) in a fixed order:
// a butterfly, after which every lane holds the same bits (IEEE addition
// commutes).
static_assert(kIfBlock == 64, "an interface unit is one wave");
__device__ __forceinline__ void wave_sum2(double& t0, double& t1) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    t0 += __shfl_xor(t0, off, 64);
    t1 += __shfl_xor(t1, off, 64);
  }
}

// Sum of the first (k = 0) or second (k = 1) of n per-unit pairs, in one
// fixed order: lane l adds pairs l, l + 64, ... in turn, then the lanes'
// partials are added by a butterfly.  Called by all 64 lanes of a wave; every
// lane of every caller gets the same bits.
__device__ __forceinline__ double fold_units(const double* __restrict__ sums, int n, int k) {
  const int lane = (int)(threadIdx.x & 63);
  double t = 0.0;
  for (int b = lane; b < n; b += 64) t += sums[2 * b + k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
  return t;
}

// ---- field access relative to a thread's face / cell (x, j) ------------
// GenAcc applies the wall mirror and ghost rules of U_at, V_at and T_at.
template <typename real>
struct GenAcc {
  const SplitArgs<real>& a;
  int x, j;
  __device__ real u(int dx, int dy) const { return U_at(a, a.u, x + dx, j + dy, a.umean); }
  __device__ real v(int dx, int dy) const { return V_at(a, a.v, x + dx, j + dy); }
  __device__ real us(int dx, int dy) const { return U_at(a, a.us, x + dx, j + dy); }
  __device__ real vs(int dx, int dy) const { return V_at(a, a.vs, x + dx, j + dy); }
  __device__ real T(int dx, int dy) const { return T_at(a, a.T, x + dx, j + dy); }
  __device__ real p(int dx, int dy) const { return P_at(a, x + dx, j + dy); }
};

// face value of the convection scheme (Eq 76's QUICK, or central / upwind),
// both upwind candidates evaluated and one selected
template <typename real, int CONV>
__device__ __forceinline__ real face_value(real uf, real ll, real l, real r, real rr) {
  if constexpr (CONV == 1) {
    return real(0.5) * (l + r);
  } else if constexpr (CONV == 2) {
    return uf >= real(0) ? l : r;
  } else {
    const real up = fmad(real(0.75), l, fmad(real(0.375), r, real(-0.125) * ll));
    const real dn = fmad(real(0.75), r, fmad(real(0.375), l, real(-0.125) * rr));
    return uf >= real(0) ? up : dn;
  }
}

// 2. momentum: u* on x-faces c0+1 .. nx-1, v* on y-faces 1 .. ny-1 of the
//    FV cells; wall and prescribed faces copied (face c0: the inflow face
//    of the split cavity, or the west wall).
// u* at a regular x-face (x, j) from an accessor centred there (Eq 74-75,
// explicit): convection of u by QUICK (or central / upwind), central
// diffusion, the pressure gradient, and buoyancy on x-faces when gravity
// points along -x.  Every path that forms a face (the per-face kernels and
// the fused march) goes through these functions, so a face gets the same
// bits whichever path forms it.
template <typename real, int CONV, typename Acc>
__device__ __forceinline__ real ustar_val(const SplitArgs<real>& a, const Acc& F) {
  const real nu = a.nu;
  real Fc[2], Gc[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int dm = k - 1;  // cell m = x - 1 + k
    const real ub = real(0.5) * (F.u(dm, 0) + F.u(dm + 1, 0));
    const real uh = face_value<real, CONV>(ub, F.u(dm - 1, 0), F.u(dm, 0), F.u(dm + 1, 0),
                                           F.u(dm + 2, 0));
    Fc[k] = ub * uh;
    const real vb = real(0.5) * (F.v(-1, k) + F.v(0, k));  // y-face j + k
    const real uh2 = face_value<real, CONV>(vb, F.u(0, k - 2), F.u(0, k - 1), F.u(0, k),
                                            F.u(0, k + 1));
    Gc[k] = vb * uh2;
  }
  const real uc = F.u(0, 0);
  const real lap = F.u(1, 0) + F.u(-1, 0) + F.u(0, 1) + F.u(0, -1) - real(4) * uc;
  const real dp = F.p(0, 0) - F.p(-1, 0);
  real out = uc - (Fc[1] - Fc[0]) - (Gc[1] - Gc[0]) + nu * lap - dp;
  if (a.gdir) {  // buoyancy on the x-face from the two adjacent cells
    const real Tfx = real(0.5) * (F.T(-1, 0) + F.T(0, 0));
    out = out + a.gbeta * (Tfx - a.Tref);
  }
  return out;
}

// v* at a regular y-face (x, jf) from an accessor centred there
template <typename real, int CONV, typename Acc>
__device__ __forceinline__ real vstar_val(const SplitArgs<real>& a, const Acc& F) {
  const real nu = a.nu;
  real Fc[2], Gc[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int dm = k - 1;  // cell row m = jf - 1 + k
    const real vb = real(0.5) * (F.v(0, dm) + F.v(0, dm + 1));
    const real vh = face_value<real, CONV>(vb, F.v(0, dm - 1), F.v(0, dm), F.v(0, dm + 1),
                                           F.v(0, dm + 2));
    Fc[k] = vb * vh;
    const real ub = real(0.5) * (F.u(k, -1) + F.u(k, 0));  // x-face x + k
    const real vh2 = face_value<real, CONV>(ub, F.v(k - 2, 0), F.v(k - 1, 0), F.v(k, 0),
                                            F.v(k + 1, 0));
    Gc[k] = ub * vh2;
  }
  const real vc = F.v(0, 0);
  const real lap = F.v(1, 0) + F.v(-1, 0) + F.v(0, 1) + F.v(0, -1) - real(4) * vc;
  const real dp = F.p(0, 0) - F.p(0, -1);
  const real Tf = real(0.5) * (F.T(0, -1) + F.T(0, 0));
  real out = vc - (Gc[1] - Gc[0]) - (Fc[1] - Fc[0]) + nu * lap - dp;
  if (!a.gdir) out = out + a.gbeta * (Tf - a.Tref);
  return out;
}

// 3. pressure (artificial compressibility, beta = c_s^2) and energy on u*:
// new p and T of cell (x, j) from an accessor of u*, v* and T centred there
template <typename real, int CONV, bool INNER, typename Acc>
__device__ __forceinline__ void press_energy_val(const SplitArgs<real>& a, const Acc& F, int x,
                                                 int j, real pin, real Tc, real& pnew,
                                                 real& Tnew) {
  const real al = a.alpha;
  const real ue = (!INNER && x == a.nx - 1) ? real(0) : F.us(1, 0);
  const real uw = F.us(0, 0);
  const real vn = F.vs(0, 1), vsd = F.vs(0, 0);
  pnew = pin - real(1) / real(3) * ((ue - uw) + (vn - vsd));
  real Fx[2], Gy[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!INNER && x + k == a.nx) {
      Fx[k] = a.tfix[1] ? real(-2) * al * (a.Tw[1] - Tc) : real(0);
    } else if (!INNER && a.west_wall && x + k == 0) {
      Fx[k] = a.tfix[0] ? real(-2) * al * (Tc - a.Tw[0]) : real(0);
    } else {
      const real uf = F.us(k, 0);  // x-face x + k
      const real th = face_value<real, CONV>(uf, F.T(k - 2, 0), F.T(k - 1, 0), F.T(k, 0),
                                             F.T(k + 1, 0));
      Fx[k] = fmad(uf, th, -al * (F.T(k, 0) - F.T(k - 1, 0)));
    }
    const int jf = j + k;
    if (!INNER && jf == 0) {
      Gy[k] = a.tfix[2] ? real(-2) * al * (Tc - a.Tw[2]) : real(0);
    } else if (!INNER && jf == a.ny) {
      Gy[k] = a.tfix[3] ? real(-2) * al * (a.Tw[3] - Tc) : real(0);
    } else {
      const real vf = F.vs(0, k);  // y-face j + k
      const real th = face_value<real, CONV>(vf, F.T(0, k - 2), F.T(0, k - 1), F.T(0, k),
                                             F.T(0, k + 1));
      Gy[k] = fmad(vf, th, -al * (F.T(0, k) - F.T(0, k - 1)));
    }
  }
  Tnew = Tc - (Fx[1] - Fx[0]) - (Gy[1] - Gy[0]);
}

// ---- FV step in one launch ----------------------------------------------
// The interior: a 64-lane wave owns the columns x0 .. x0 + 63 of a strip
// and marches a band of rows upward; lanes 2 .. 60 are its cells, the others
// halos (QUICK reaches two cells, and u* at a cell's east face is formed by
// the lane to its right).  Each lane keeps a rolling window of its own
// column (u on rows j-2 .. j+2, v on faces j-1 .. j+3, p on rows j, j+1, T
// on rows j-2 .. j+2); values of neighbouring columns come by cross-lane
// permutes.  Per row a lane forms u* on its cell's west face and v* on its
// north face, then the cell's new p and T, while the loads of the row two
// ahead are in flight: the FV zone's 32 bytes per cell, read and written
// once.  Strips start at xa + 59 s; when they do not reach column nx - 4 a
// last strip at nx - 64 forms the cells east of X1 only.
// The frame (cells and faces the walls' mirror and ghost rules or the inflow
// face reach) is formed in the same launch by other blocks, one thread per
// face / cell position, each forming the faces its cell needs itself: the
// march and the frame share no memory within the launch, and a face both
// form is formed by the same arithmetic from the same values.
constexpr int kFvOut = 59;

// The fused region and the frame (set on the host, fv_region): nst strips of
// kFvOut cells whose lane 0 sits at column xa + kFvOut s, plus npart = 1 last
// strip at nx - 64 writing cells x > xcut only; bands of `band` rows from
// row 2; fused cells X0 .. X1 on rows 2 .. ny - 3 (X0 > X1: none).  The
// frame's positions: nbt bottom / top rows over the nfc face columns, then
// the middle rows over wl columns west of X0 and wr east of X1; its nfrb
// blocks come first in the grid.
struct FvRegion {
  int nst, npart, xcut, band, nbands, nwaves;
  int xa, X0, X1;
  int nfc, nbt, wl, wr, nframe, nfrb;
};

template <typename real>
__device__ __forceinline__ real lane_get(real v, int d) {
  return d > 0 ? __shfl_down(v, d, 64) : d < 0 ? __shfl_up(v, -d, 64) : v;
}

// raw buffer access: a per-lane byte offset (the column) and a wave-uniform
// one (the row); the record size bounds every access
__device__ __forceinline__ __amdgpu_buffer_rsrc_t fv_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
template <typename real>
__device__ __forceinline__ real fv_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(real) == 4) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}
template <typename real>
__device__ __forceinline__ void fv_store(real v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(real) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
  } else {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  }
}

// window accessors: u* at (x, j) and v* at (x, j + 1) from the window of
// row j (wu: rows j-2 .. j+2, wv: faces j-1 .. j+3, wp: rows j, j+1, wT:
// rows j-2 .. j+2), and the cell (x, j) from its faces' u*, v*
template <typename real>
struct WinU {
  const real (&wu)[5], (&wv)[5], (&wp)[2], (&wT)[5];
  __device__ real u(int dx, int dy) const { return dy == 0 ? lane_get(wu[2], dx) : wu[2 + dy]; }
  __device__ real v(int dx, int dy) const { return lane_get(wv[1 + dy], dx); }
  __device__ real p(int dx, int) const { return lane_get(wp[0], dx); }
  __device__ real T(int dx, int) const { return lane_get(wT[2], dx); }
};
template <typename real>
struct WinV {
  const real (&wu)[5], (&wv)[5], (&wp)[2], (&wT)[5];
  __device__ real v(int dx, int dy) const { return dy == 0 ? lane_get(wv[2], dx) : wv[2 + dy]; }
  __device__ real u(int dx, int dy) const { return lane_get(wu[3 + dy], dx); }
  __device__ real p(int, int dy) const { return wp[1 + dy]; }
  __device__ real T(int, int dy) const { return wT[3 + dy]; }
};
template <typename real>
struct WinE {
  real usw, use, vss, vsn;
  const real (&wT)[5];
  __device__ real us(int dx, int) const { return dx == 0 ? usw : use; }
  __device__ real vs(int, int dy) const { return dy == 0 ? vss : vsn; }
  __device__ real T(int dx, int dy) const { return dy == 0 ? lane_get(wT[2], dx) : wT[2 + dy]; }
};
// a frame cell: the faces' u*, v* it formed, T through the ghost rules
template <typename real>
struct FrameE {
  real usw, use, vss, vsn;
  GenAcc<real> g;
  __device__ real us(int dx, int) const { return dx == 0 ? usw : use; }
  __device__ real vs(int, int dy) const { return dy == 0 ? vss : vsn; }
  __device__ real T(int dx, int dy) const { return g.T(dx, dy); }
};

// u* on x-face (x, j < ny) and v* on y-face (x < nx, jf) with the rules of
// the prescribed inflow face, the walls and their mirror and ghost rules
template <typename real, int CONV>
__device__ __forceinline__ real face_u(const SplitArgs<real>& a, int x, int j) {
  if (x == a.c0) return a.u[j * a.pF + fidx(a, x)] - a.umean;
  if (x == a.nx) return real(0);
  return ustar_val<real, CONV>(a, GenAcc<real>{a, x, j});
}
template <typename real, int CONV>
__device__ __forceinline__ real face_v(const SplitArgs<real>& a, int x, int jf) {
  if (jf == 0 || jf == a.ny) return real(0);
  return vstar_val<real, CONV>(a, GenAcc<real>{a, x, jf});
}

// frame position idx: rows 0 .. 2 and ny - 2 .. ny over every face column
// c0 .. nx (all rows when ny < 5), then rows 3 .. ny - 3 over the columns
// outside [X0, X1]
template <typename real>
__device__ __forceinline__ void frame_xy(const SplitArgs<real>& a, const FvRegion& R, int idx,
                                         int& x, int& j) {
  const int nA = R.nbt * R.nfc;
  if (idx < nA) {
    const int r = idx / R.nfc;
    x = a.c0 + idx % R.nfc;
    j = (R.nbt < 6 || r < 3) ? r : a.ny - 5 + r;
    return;
  }
  idx -= nA;
  const int w = R.wl + R.wr;
  const int k = idx % w;
  x = k < R.wl ? a.c0 + k : R.X1 + 1 + (k - R.wl);
  j = 3 + idx / w;
}

template <typename real, int CONV>
__device__ __forceinline__ void fv_frame(const SplitArgs<real>& a, const FvRegion& R, int idx) {
  if (idx >= R.nframe) return;
  int x, j;
  frame_xy(a, R, idx, x, j);
  const bool incols = x >= R.X0 && x <= R.X1;
  const bool cell = x < a.nx && j < a.ny && !(incols && j >= 2 && j <= a.ny - 3);
  const bool do_u = j < a.ny && !(incols && j >= 2 && j <= a.ny - 3);
  const bool do_v = x < a.nx && !(incols && j >= 3 && j <= a.ny - 2);
  const int o = j * a.pF + fidx(a, x);
  real uw = real(0), vsd = real(0);
  if (do_u) {
    uw = face_u<real, CONV>(a, x, j);
    a.us[o] = uw;
  }
  if (x < a.nx) {
    vsd = face_v<real, CONV>(a, x, j);
    if (do_v) a.vs[o] = vsd;
  }
  if (!cell) return;
  const real ue = face_u<real, CONV>(a, x + 1, j);
  const real vn = face_v<real, CONV>(a, x, j + 1);
  real pn, Tn;
  press_energy_val<real, CONV, false>(a, FrameE<real>{uw, ue, vsd, vn, GenAcc<real>{a, x, j}}, x,
                                      j, a.pin[o], a.T[o], pn, Tn);
  a.p[o] = pn;
  a.Tn[o] = Tn;
}

// IFACE: the divided cavity, whose inflow face carries its mean; the FV-only
// cavity has none (a separate instance, without the corrections' registers)
template <typename real, int CONV, bool IFACE>
__global__ __launch_bounds__(256) void k_dd_fv(SplitArgs<real> a0, FvRegion R) {
  // the mean of the inflow face the boundary-node launch stored, from its
  // per-block sums in block order (the same bits in every wave)
  SplitArgs<real> a = a0;
  a.umean = IFACE ? (real)(fold_units(ghost_sums(a.iface, a.ny, a.par), iface_blocks(a.ny), 0) /
                           a.ny)
                  : real(0);
  // blocks renumbered so that each XCD works on a contiguous range
  const int nb = gridDim.x, b = blockIdx.x;
  const int per = nb / 8, rem = nb % 8, xcd = b % 8;
  const int lb = xcd * per + (xcd < rem ? xcd : rem) + b / 8;
  if (lb < R.nfrb) {
    fv_frame<real, CONV>(a, R, lb * 256 + (int)threadIdx.x);
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane((lb - R.nfrb) * 4 + (int)(threadIdx.x >> 6));
  if (wave >= R.nwaves) return;
  const int lane = threadIdx.x & 63;
  const int ns = R.nst + R.npart;
  const int strip = wave % ns, bnd = wave / ns;
  const bool part = strip == R.nst;
  const int x = (part ? a.nx - 64 : R.xa + kFvOut * strip) + lane;
  const int j0 = 2 + bnd * R.band;
  const int j1 = min(j0 + R.band, a.ny - 2);
  const bool out = lane >= 2 && lane <= 60 && (!part || x > R.xcut);
  const unsigned bytes = (unsigned)((size_t)(a.ny + 1) * a.pF * sizeof(real));
  const __amdgpu_buffer_rsrc_t rU = fv_rsrc(a.u, bytes), rV = fv_rsrc(a.v, bytes),
                               rP = fv_rsrc(a.pin, bytes), rT = fv_rsrc(a.T, bytes);
  const int vo = fidx(a, x) * (int)sizeof(real), rowb = a.pF * (int)sizeof(real);
  real u[5], v[5], p[2], T[5];
  // the lane on the inflow face reads it less its mean
  const real ucorr = x == a.c0 ? a.umean : real(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    u[k] = fv_load<real>(rU, vo, (j0 - 2 + k) * rowb) - ucorr;
    v[k] = fv_load<real>(rV, vo, (j0 - 1 + k) * rowb);
    T[k] = fv_load<real>(rT, vo, (j0 - 2 + k) * rowb);
  }
  p[0] = fv_load<real>(rP, vo, j0 * rowb);
  p[1] = fv_load<real>(rP, vo, (j0 + 1) * rowb);
  // v* on the band's south face j0: the window of row j0 - 1
  real vsouth;
  {
    real u1[5], v1[5], p1[2], T1[5];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u1[k + 1] = u[k];
      v1[k + 1] = v[k];
      T1[k + 1] = T[k];
    }
    u1[0] = u[0];  // row j0 - 3: not used by v* on face j0
    T1[0] = T[0];  // row j0 - 3: not used
    v1[0] = fv_load<real>(rV, vo, (j0 - 2) * rowb);
    p1[0] = fv_load<real>(rP, vo, (j0 - 1) * rowb);
    p1[1] = p[0];
    vsouth = vstar_val<real, CONV>(a, WinV<real>{u1, v1, p1, T1});
  }
  // every window load has landed (vmcnt 0): the march's loop then starts
  // with no load of its own in flight
  __builtin_amdgcn_s_waitcnt(0x0F70);
  const __amdgpu_buffer_rsrc_t rUs = fv_rsrc(a.us, bytes), rVs = fv_rsrc(a.vs, bytes),
                               rPn = fv_rsrc(a.p, bytes), rTn = fv_rsrc(a.Tn, bytes);
  // the values the window takes on when it moves up to row r: u row r+2,
  // v face r+3, p row r+1, T row r+2.  Loads and stores are issued
  // unconditionally (rows past the band clamped to stored ones, lanes that
  // own no cell storing to an offset past the buffer's record size, which
  // the hardware drops), so every trip issues the same memory operations
  // and the waits for a row's loads count exactly the operations after them.
  const int rmax = a.ny - 3;
  auto issue = [&](real (&q)[4], int r) {
    r = min(r, rmax);
    q[0] = fv_load<real>(rU, vo, (r + 2) * rowb) - ucorr;
    q[1] = fv_load<real>(rV, vo, (r + 3) * rowb);
    q[2] = fv_load<real>(rP, vo, (r + 1) * rowb);
    q[3] = fv_load<real>(rT, vo, (r + 2) * rowb);
  };
  const int vst = out ? vo : (int)0x80000000;
  auto advance = [&](const real (&q)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u[k] = u[k + 1];
      v[k] = v[k + 1];
      T[k] = T[k + 1];
    }
    u[4] = q[0];
    v[4] = q[1];
    p[0] = p[1];
    p[1] = q[2];
    T[4] = q[3];
  };
  auto row = [&](int j) {
    const real us = ustar_val<real, CONV>(a, WinU<real>{u, v, p, T});
    const real vnorth = vstar_val<real, CONV>(a, WinV<real>{u, v, p, T});
    const real ue = __shfl_down(us, 1, 64);
    real pnew, Tnew;
    press_energy_val<real, CONV, true>(a, WinE<real>{us, ue, vsouth, vnorth, T}, x, j, p[0],
                                       T[2], pnew, Tnew);
    fv_store(us, rUs, vst, j * rowb);
    fv_store(vnorth, rVs, vst, (j + 1) * rowb);
    fv_store(pnew, rPn, vst, j * rowb);
    fv_store(Tnew, rTn, vst, j * rowb);
    vsouth = vnorth;
  };
  // two rows per trip: the loads of both are issued at the top of the trip,
  // so that each set is in flight over one or two rows of arithmetic and no
  // load is still in flight across the loop's back edge
  real qa[4] = {real(0), real(0), real(0), real(0)};
  real qb[4] = {real(0), real(0), real(0), real(0)};
  for (int j = j0;; j += 2) {
    issue(qa, j + 1);
    issue(qb, j + 2);
    row(j);
    if (j + 1 >= j1) break;
    advance(qa);
    row(j + 1);
    if (j + 2 >= j1) break;
    advance(qb);
  }
}

// 4. p_bar sums of unit b of the interface's rows (b < iface_blocks; one
//    wave): the
//    new FV pressure over the shared columns, and the net mass this step's
//    stream moves into the LBM zone through the links to x_b: the
//    post-collision populations x_b sent west (W, NW, SW) less those x_f
//    sent east (E, NE, SE), each only where its target row exists (a
//    diagonal leaving through a wall returns to its own node).  Both sets
//    carry the same weights, so the shifted values give the same sum.  Run
//    by extra blocks of the LBM launch (they read only what that launch
//    does not write).
template <typename real>
__device__ void pbar_block(const SplitArgs<real>& a, int b) {
  const int ny = a.ny, ib = a.ib;
  if (b >= iface_blocks(ny)) return;  // uniform per wave
  const int j = b * kIfBlock + (int)(threadIdx.x & 63);
  double ps = 0.0, fl = 0.0;
  if (j < ny) {
    for (int x = a.c0; x <= ib; ++x) ps += (double)a.p[j * a.pF + fidx(a, x)];
    const int PL = a.planeL, ob = j * a.pL + ib, of = ob - 1;
    double in = (double)a.fin[3 * PL + ob], out = (double)a.fin[1 * PL + of];
    if (j + 1 < ny) {
      in += (double)a.fin[6 * PL + ob];
      out += (double)a.fin[5 * PL + of];
    }
    if (j > 0) {
      in += (double)a.fin[7 * PL + ob];
      out += (double)a.fin[8 * PL + of];
    }
    fl = in - out;
  }
  wave_sum2(ps, fl);
  if ((threadIdx.x & 63) == 0) {
    double* out = pbar_sums(a.iface, ny);
    out[2 * b] = ps;
    out[2 * b + 1] = fl;
  }
}

// 5. LBM zone, nodes 0 .. ib-1: stream, moments, collide
// x / 3 from an unevaluated pair hi + lo = 1/3: within an ulp of the exact
// quotient, with no relative error common to all nodes.
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

// BGK collision with buoyancy on shifted populations (Eq 5, 8, 18):
//   f~_eq = w (drho + rho A) + 3 w e.j,  A = 9/2 (e.u)^2 - 3/2 u.u,
// with j = sum e f~ the streamed momentum (3 w = 1/3 on the axes, 1/12 on the
// diagonals).  Building the linear term from j itself, not as rho * u with
// rho = 1 + drho and FP32-rounded weights, keeps the equilibrium's momentum
// free of relative errors shared by whole regions of nodes, which would act
// as a body force proportional to the momentum.
template <typename real>
__device__ __forceinline__ void collide_f(const SplitArgs<real>& a, real f[9], real drho, real ux,
                                          real uy, real T) {
  const real rho = real(1) + drho;
  // buoyancy G along +y, or along +x when gravity points along -x
  const real G = a.gbeta * (T - a.Tref);
  const real Gu = G * (a.gdir ? ux : uy);
  const real usq = real(1.5) * fmad(ux, ux, uy * uy);
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const real eu = real(ex9(q)) * ux + real(ey9(q)) * uy;
    const real A = fmad(real(4.5) * eu, eu, -usq);
    const real P = A + real(3) * eu;
    const real ej = ex9(q) == 0 ? real(ey9(q)) * jy
                    : ey9(q) == 0 ? real(ex9(q)) * jx
                                  : real(ex9(q)) * jx + real(ey9(q)) * jy;
    const real lin = q == 0 ? real(0) : q < 5 ? third(ej) : real(0.25) * third(ej);
    const real fe = w9<real>(q) * fmad(rho, A, drho) + lin;
    const real eG = real(a.gdir ? ex9(q) : ey9(q)) * G;
    const real c = (real(3) * w9<real>(q)) * (eG - Gu);
    f[q] = fmad(a.omega, fe - f[q], f[q]) + fmad(c, P, c);
  }
}

// D2Q5 heat collision (Eq 19-22): g_eq = T w (1 + 3 e.u); the rest
// population takes T minus the four moving ones, so that sum g_eq = T holds
// without the common relative error of FP32-rounded weights (T / 6 is formed
// from the unbiased T / 3).
template <typename real>
__device__ __forceinline__ void collide_fg(const SplitArgs<real>& a, real f[9], real g[5],
                                           real drho, real ux, real uy, real T) {
  collide_f(a, f, drho, ux, uy, T);
  const real t6 = real(0.5) * third(T);
  const real gE = t6 * (real(1) + real(3) * ux), gW = t6 * (real(1) - real(3) * ux);
  const real gN = t6 * (real(1) + real(3) * uy), gS = t6 * (real(1) - real(3) * uy);
  const real ge[5] = {T - ((gE + gW) + (gN + gS)), gE, gN, gW, gS};
#pragma unroll
  for (int q = 0; q < 5; ++q) g[q] = fmad(a.omegaT, ge[q] - g[q], g[q]);
}

template <typename real>
__device__ __forceinline__ void moments9(const real f[9], real& drho, real& ux, real& uy) {
  const real s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const real jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  const real jy = (f[2] - f[4]) + ((f[5] - f[7]) + (f[6] - f[8]));
  drho = s;
  const real inv = real(1) / (real(1) + s);
  ux = jx * inv;
  uy = jy * inv;
}

template <typename real>
__global__ __launch_bounds__(256) void k_dd_lbm(SplitArgs<real> a, int pbar_rows) {
  // the first pbar_rows rows of blocks (dispatched first) form the p_bar
  // sums, one unit per wave
  if ((int)blockIdx.y < pbar_rows) {
    pbar_block(a, (int)(blockIdx.y * gridDim.x + blockIdx.x) * 4 + (int)(threadIdx.x >> 6));
    return;
  }
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = (blockIdx.y - pbar_rows) * 4 + (threadIdx.x >> 6);
  if (i >= a.ib || j >= a.ny) return;
  const int pL = a.pL, PL = a.planeL;
  real f[9], g[5];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int sx = i - ex9(q), sy = j - ey9(q);
    if (sx >= 0 && !(a.east_wall && sx >= a.nx) && sy >= 0 && sy < a.ny)
      f[q] = a.fin[q * PL + sy * pL + sx];
    else if (sy >= a.ny)  // the north wall, sliding at ulid: + 6 w_q (e_q . u_w)
      f[q] = a.fin[opp9(q) * PL + j * pL + i] + real(6) * w9<real>(q) * real(ex9(q)) * a.ulid;
    else f[q] = a.fin[opp9(q) * PL + j * pL + i];  // walls at rest: bounce-back
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const int sx = i - ex5(q), sy = j - ey5(q);
    const int side = sy < 0 ? 2 : sy >= a.ny ? 3 : sx < 0 ? 0 : (a.east_wall && sx >= a.nx) ? 1 : -1;
    if (side < 0) g[q] = a.gin[q * PL + sy * pL + sx];
    else if (a.tfix[side])  // anti-bounce-back: fixed temperature
      g[q] = -a.gin[opp5(q) * PL + j * pL + i] + real(2) * w5<real>(q) * a.Tw[side];
    else  // bounce-back: adiabatic
      g[q] = a.gin[opp5(q) * PL + j * pL + i];
  }
  real drho, ux, uy;
  moments9(f, drho, ux, uy);
  const real T = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
  const int o = j * pL + i;
  if (!a.east_wall && i == a.ib - 1) {  // keep x_f's streamed state for the boundary node
    real* xf = a.xf + j * 18;
#pragma unroll
    for (int q = 0; q < 9; ++q) xf[q] = f[q];
#pragma unroll
    for (int q = 0; q < 5; ++q) xf[9 + q] = g[q];
    xf[14] = drho;
    xf[15] = ux;
    xf[16] = uy;
    xf[17] = T;
  }
  if (a.mom_all || i >= a.c0 - 2) {
    a.mom[o] = real(1) + drho;
    a.mom[PL + o] = ux;
    a.mom[2 * PL + o] = uy;
    a.mom[3 * PL + o] = T;
  }
  collide_fg(a, f, g, drho, ux, uy, T);
#pragma unroll
  for (int q = 0; q < 9; ++q) a.fout[q * PL + o] = f[q];
#pragma unroll
  for (int q = 0; q < 5; ++q) a.gout[q * PL + o] = g[q];
}

// 6. the artificial boundary node x_b = ib of row j: rho_b by Eq 93 with
//    its level, u_b, v_b, T_b by face averages of the new FV state,
//    populations by non-equilibrium extrapolation or the finite-difference
//    closure, then its collision.  mchange: the LBM zone's mass change since
//    init after this step's stream; msum: the running sum of its deficit.
template <typename real>
__device__ __forceinline__ void xb_row(const SplitArgs<real>& a, int j, double rho0, double pbar,
                                       double mchange, double msum) {
  const int ib = a.ib, ny = a.ny;
  // FV state at the new time level (u*, v*, p, T_new)
  const real ub = real(0.5) * (a.us[j * a.pF + fidx(a, ib)] + a.us[j * a.pF + fidx(a, ib + 1)]);
  const real vb = real(0.5) * (a.vs[j * a.pF + fidx(a, ib)] + a.vs[(j + 1) * a.pF + fidx(a, ib)]);
  const real Tb = a.Tn[j * a.pF + fidx(a, ib)];
  // Eq 93: rho_b = rho0 ((p_S - p_bar) / (rho0 c_s^2) + 1), its level shifted
  // uniformly over the rows by kLevelP times the amount that, carried by the
  // rest weights of the populations x_b sends into the zone (W, NW, SW; one
  // diagonal fewer on the wall rows), would return the zone to its mass at
  // init, plus kLevelI times the running sum of that deficit over the steps.
  // The sum holds the zone's mass at its value at init in any steady state,
  // whatever the two gains; the partial correction keeps the
  // finite-difference closure stable (its populations answer the FV
  // pressure one step later, and a whole correction per step overshoots).
  const double wsum = a.ny * ((1.0 / 9.0 + 1.0 / 36.0) + 1.0 / 36.0) - 1.0 / 36.0 - 1.0 / 36.0;
  const double e = -mchange;
  const double delta = (kLevelP * e + kLevelI * msum) / wsum;
  const double rb =
      rho0 * (((double)a.p[j * a.pF + fidx(a, ib)] - pbar) / (rho0 / 3.0) + 1.0) + delta;
  const real drb = (real)(rb - 1.0);
  const real* xf = a.xf + j * 18;
  real f[9], g[5];
  if (a.kind == 0) {
    // non-equilibrium extrapolation: f_b = f_eq(b) + f_f - f_eq(f)
#pragma unroll
    for (int q = 0; q < 9; ++q)
      f[q] = feq_s<real>(q, drb, ub, vb) + (xf[q] - feq_s<real>(q, xf[14], xf[15], xf[16]));
  } else {
    // f_b = f_eq(b) - (tau w rho_b / c_s^2) Q : S, S from the FV velocities
    const real dudx = a.us[j * a.pF + fidx(a, ib + 1)] - a.us[j * a.pF + fidx(a, ib)];
    auto ucell = [&](int jj) {
      return real(0.5) * (a.us[jj * a.pF + fidx(a, ib)] + a.us[jj * a.pF + fidx(a, ib + 1)]);
    };
    const real um = j > 0 ? ucell(j - 1) : -ub;
    const real up = j < ny - 1 ? ucell(j + 1) : real(2) * a.ulid - ub;
    const real vw = real(0.5) * (a.vs[j * a.pF + fidx(a, ib - 1)] + a.vs[(j + 1) * a.pF + fidx(a, ib - 1)]);
    const real ve = real(0.5) * (a.vs[j * a.pF + fidx(a, ib + 1)] + a.vs[(j + 1) * a.pF + fidx(a, ib + 1)]);
    const real Sxx = dudx, Syy = -dudx;
    const real Sxy = real(0.5) * (real(0.5) * (up - um) + real(0.5) * (ve - vw));
    const real rbr = (real)rb;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const real cx = real(ex9(q)), cy = real(ey9(q));
      const real QS = (cx * cx - real(1) / real(3)) * Sxx + real(2) * cx * cy * Sxy +
                      (cy * cy - real(1) / real(3)) * Syy;
      f[q] = feq_s<real>(q, drb, ub, vb) - a.tau * w9<real>(q) * rbr * real(3) * QS;
    }
  }
  // g by non-equilibrium extrapolation (Eq 95)
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const real gb = Tb * w5<real>(q) * (real(1) + real(3) * (real(ex5(q)) * ub + real(ey5(q)) * vb));
    const real gf = xf[17] * w5<real>(q) *
                    (real(1) + real(3) * (real(ex5(q)) * xf[15] + real(ey5(q)) * xf[16]));
    g[q] = gb + (xf[9 + q] - gf);
  }
  real drho, ux, uy;
  moments9(f, drho, ux, uy);
  const real T = ((g[0] + g[1]) + (g[2] + g[3])) + g[4];
  const int o = j * a.pL + ib;
  a.mom[o] = real(1) + drho;
  a.mom[a.planeL + o] = ux;
  a.mom[2 * a.planeL + o] = uy;
  a.mom[3 * a.planeL + o] = T;
  collide_fg(a, f, g, drho, ux, uy, T);
#pragma unroll
  for (int q = 0; q < 9; ++q) a.fout[q * a.planeL + o] = f[q];
#pragma unroll
  for (int q = 0; q < 5; ++q) a.gout[q * a.planeL + o] = g[q];
}

// 7. ghost columns of the next step's FV zone (its input buffers: this
//    step's output set us, vs, Tn) from the LBM moments of this step, for
//    row j (j < ny) and y-face j (j <= ny): two-point averages of the LBM
//    velocities on the faces c0 - 1 and c0 (the inflow face, whose mean over
//    the rows the FV step removes where it reads it: global continuity of
//    the FV zone), the
//    LBM temperatures on the ghost cells.  Returns the row's inflow velocity
//    and density over the shared columns c0 .. ib (for rho0, Eq 91-93).
template <typename real>
__device__ __forceinline__ void ghost_row(const SplitArgs<real>& a, int j, double& su,
                                          double& sr) {
  const int c0 = a.c0, ny = a.ny;
  const real* rho = a.mom;
  const real* ux = a.mom + a.planeL;
  const real* uy = a.mom + 2 * a.planeL;
  const real* TL = a.mom + 3 * a.planeL;
  su = 0.0;
  sr = 0.0;
  if (j < ny) {
    const int o = j * a.pL;
    const real uf1 = real(0.5) * (ux[o + c0 - 1] + ux[o + c0]);
    a.us[j * a.pF + fidx(a, c0 - 1)] = real(0.5) * (ux[o + c0 - 2] + ux[o + c0 - 1]);
    a.us[j * a.pF + fidx(a, c0)] = uf1;
    a.Tn[j * a.pF + fidx(a, c0 - 2)] = TL[o + c0 - 2];
    a.Tn[j * a.pF + fidx(a, c0 - 1)] = TL[o + c0 - 1];
    su = (double)uf1;
    sr = (double)rho[o + c0] + (double)rho[o + c0 + 1] + (double)rho[o + c0 + 2];
  }
  if (j <= ny) {
    for (int x = c0 - 2; x <= c0 - 1; ++x) {
      real vv = real(0);
      if (j > 0 && j < ny) vv = real(0.5) * (uy[(j - 1) * a.pL + x] + uy[j * a.pL + x]);
      a.vs[j * a.pF + fidx(a, x)] = vv;
    }
  }
}

// The interface's end of a step (one thread per row and y-face):
//  (a) unless ghost_only: every unit folds the per-unit sums (fold_units) --
//      p_bar, the mean new FV pressure over the shared columns (written by
//      the LBM launch), the net mass this step's stream moved into the LBM
//      zone through the links to x_b (same launch), and rho0, the mean LBM
//      density over the shared columns at the start of the step (the ghost
//      sums of this step's parity); unit 0 stores the zone's new mass
//      change and running sum for the next step; then x_b of its row;
//  (b) the ghost values of the next step (ghost_row) and the unit's sums
//      of them (the ghost sums of the next parity); the next FV launch folds
//      the inflow sums and removes their mean where it reads the inflow face
//      (umean).
// ghost_only (at init, with the arguments of parity 1, so that the values
// land in the buffers and sums step 0 reads) runs (b) alone.
template <typename real>
__global__ __launch_bounds__(kIfBlock) void k_dd_xb(SplitArgs<real> a, int ghost_only) {
  const int ny = a.ny, nb = (int)gridDim.x;
  const int j = blockIdx.x * kIfBlock + threadIdx.x;
  if (!ghost_only) {
    const double* ps = pbar_sums(a.iface, ny);
    const double fold[3] = {fold_units(ps, nb, 0), fold_units(ps, nb, 1),
                            fold_units(ghost_sums(a.iface, ny, a.par), nb, 1)};
    const double pbar = fold[0] / (3.0 * ny), rho0 = fold[2] / (3.0 * ny);
    const int sl = 2 + 2 * (a.par & 1), sn = 2 + 2 * ((a.par & 1) ^ 1);
    const double mchange = a.iface[sl] + fold[1];  // the zone's mass change since init
    const double msum = a.iface[sl + 1] - mchange;  // running sum of its deficit
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.iface[sn] = mchange;
      a.iface[sn + 1] = msum;
    }
    if (j < ny) xb_row(a, j, rho0, pbar, mchange, msum);
  }
  double su, sr;
  ghost_row(a, j, su, sr);
  wave_sum2(su, sr);
  if (threadIdx.x == 0) {
    double* gn = ghost_sums(a.iface, ny, a.par ^ 1);
    gn[2 * blockIdx.x] = su;
    gn[2 * blockIdx.x + 1] = sr;
  }
}

// dense output: LBM values for columns < s, FV (face-averaged) for >= s
template <typename real>
__global__ __launch_bounds__(256) void k_dd_output(SplitArgs<real> a, real* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (x >= a.nx) return;
  const int n = a.nx * a.ny;
  // transposed: the caller's (x, y) is the stored (j, x), its u the stored v
  const int d = a.transposed ? x * a.ny + j : j * a.nx + x;
  real r, u, v, t;
  if (x < a.s) {
    const int o = j * a.pL + x;
    r = a.mom[o];
    u = a.mom[a.planeL + o];
    v = a.mom[2 * a.planeL + o];
    t = a.mom[3 * a.planeL + o];
  } else {
    const int o = j * a.pF + fidx(a, x);
    const real ue = x == a.nx - 1 ? real(0) : a.u[j * a.pF + fidx(a, x + 1)];
    u = real(0.5) * (a.u[o] + ue);
    v = real(0.5) * (a.v[o] + a.v[(j + 1) * a.pF + fidx(a, x)]);
    t = a.T[o];
    r = real(1) + real(3) * a.pin[o];
  }
  out[d] = r;
  out[n + d] = a.transposed ? v : u;
  out[2 * n + d] = a.transposed ? u : v;
  out[3 * n + d] = t;
}

template <typename real>
__global__ __launch_bounds__(256) void k_dd_init(SplitArgs<real> a, const double* __restrict__ T0) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (j >= a.ny) return;
  const auto t0_at = [&](int xx) { return a.transposed ? T0[xx * a.ny + j] : T0[j * a.nx + xx]; };
  const double t0 = (x < a.nx && T0) ? t0_at(x) : 0.0;
  if (x == 0 && j == 0) {
    // the LBM zone's mass change and its running sum, both parities
    for (int k = 2; k < 6; ++k) a.iface[k] = 0.0;
  }
  if (x < a.nl) {
    const int o = j * a.pL + x;
    real* f = const_cast<real*>(a.fin);
    real* g = const_cast<real*>(a.gin);
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q * a.planeL + o] = real(0);  // f = w at rest
#pragma unroll
    for (int q = 0; q < 5; ++q) g[q * a.planeL + o] = real(w5<double>(q) * t0);
    a.mom[o] = real(1);
    a.mom[a.planeL + o] = real(0);
    a.mom[2 * a.planeL + o] = real(0);
    a.mom[3 * a.planeL + o] = real(t0);
  }
  const int xf = x + a.c0 - 2;  // stored FV column
  if (a.pF > 0 && xf <= a.nx) {
    const int o = j * a.pF + (xf - (a.c0 - 2));
    real* u = const_cast<real*>(a.u);
    real* v = const_cast<real*>(a.v);
    real* T = const_cast<real*>(a.T);
    u[o] = real(0);
    a.us[o] = real(0);
    a.p[o] = real(0);
    T[o] = real((xf < a.nx && xf >= 0 && T0) ? t0_at(xf) : 0.0);
    a.Tn[o] = T[o];
    v[o] = real(0);
    a.vs[o] = real(0);
    if (j == a.ny - 1) {
      v[(j + 1) * a.pF + (xf - (a.c0 - 2))] = real(0);
      a.vs[(j + 1) * a.pF + (xf - (a.c0 - 2))] = real(0);
    }
  }
}

// ---- grid setting 2 (Sec. 5.1, Fig. 30) -------------------------------
// The lattice covers all nx x ny nodes; the temperature lives on NXc x NYc
// control volumes of 2 x 2 nodes (h = 2).  Every lattice step takes its
// buoyancy from the node temperatures (mom plane 3), which are the coarse
// field interpolated bilinearly and are refreshed after each energy step.
// One energy step of length dt lattice steps is backward Euler: upwind
// convection and central diffusion in the matrix, QUICK minus upwind from
// the old field as a deferred correction, face velocities the mean of the
// four node velocities straddling each coarse face; its system is relaxed
// by K sweeps of x-lines then y-lines, each line solved by the Thomas
// algorithm with the other direction's neighbours from the previous iterate.
enum { G2_TA = 0, G2_TB, G2_AP, G2_AW, G2_AE, G2_AS, G2_AN, G2_B, G2_CP, G2_RP };

template <typename real>
__global__ __launch_bounds__(256) void k_gs2_lbm(SplitArgs<real> a) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= a.nx || j >= a.ny) return;
  const int pL = a.pL, PL = a.planeL;
  real f[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int sx = i - ex9(q), sy = j - ey9(q);
    if (sx >= 0 && sx < a.nx && sy >= 0 && sy < a.ny) f[q] = a.fin[q * PL + sy * pL + sx];
    else f[q] = a.fin[opp9(q) * PL + j * pL + i];  // walls at rest: bounce-back
  }
  real drho, ux, uy;
  moments9(f, drho, ux, uy);
  const int o = j * pL + i;
  if (a.mom_all) {
    a.mom[o] = real(1) + drho;
    a.mom[PL + o] = ux;
    a.mom[2 * PL + o] = uy;
  }
  collide_f(a, f, drho, ux, uy, a.mom[3 * PL + o]);
#pragma unroll
  for (int q = 0; q < 9; ++q) a.fout[q * PL + o] = f[q];
}

// coarse temperature with one ghost layer: the x rule on the (clamped) row,
// then the y rule (2 T_w - T for a fixed wall, T for an adiabatic one)
template <typename real>
__device__ __forceinline__ real tc_at(const SplitArgs<real>& a, const real* T, int I, int J) {
  const int Jc = J < 0 ? 0 : (J >= a.NYc ? a.NYc - 1 : J);
  real t;
  if (I < 0) {
    t = T[Jc * a.pC];
    if (a.tfix[0]) t = real(2) * a.Tw[0] - t;
  } else if (I >= a.NXc) {
    t = T[Jc * a.pC + a.NXc - 1];
    if (a.tfix[1]) t = real(2) * a.Tw[1] - t;
  } else {
    t = T[Jc * a.pC + I];
  }
  if (J < 0 && a.tfix[2]) t = real(2) * a.Tw[2] - t;
  if (J >= a.NYc && a.tfix[3]) t = real(2) * a.Tw[3] - t;
  return t;
}

// node temperatures: node i sits at coarse coordinate (2i - 1) / 4, between
// coarse cells (i - 1) >> 1 and the next with weight 3/4 (i even) or 1/4
template <typename real>
__global__ __launch_bounds__(256) void k_gs2_interp(SplitArgs<real> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= a.nx) return;
  const real* T = a.gc[G2_TA];
  const int I0 = (i - 1) >> 1, J0 = (j - 1) >> 1;
  const real wx = (i & 1) ? real(0.25) : real(0.75), wy = (j & 1) ? real(0.25) : real(0.75);
  const real t00 = tc_at(a, T, I0, J0), t10 = tc_at(a, T, I0 + 1, J0);
  const real t01 = tc_at(a, T, I0, J0 + 1), t11 = tc_at(a, T, I0 + 1, J0 + 1);
  a.mom[3 * a.planeL + j * a.pL + i] =
      (real(1) - wy) * ((real(1) - wx) * t00 + wx * t10) + wy * ((real(1) - wx) * t01 + wx * t11);
}

template <typename real>
__device__ __forceinline__ real quick8(real w, real ll, real l, real r, real rr) {
  return w >= real(0) ? (real(6) * l + real(3) * r - ll) / real(8)
                      : (real(6) * r + real(3) * l - rr) / real(8);
}

// x-face I (between coarse cells I-1 and I) of coarse row J: face velocity
// from the lattice and the deferred-correction flux h w (T_QUICK - T_up)
template <typename real>
__device__ __forceinline__ void xface(const SplitArgs<real>& a, int I, int J, real& w, real& dc) {
  const real* ux = a.mom + a.planeL;
  const int r0 = 2 * J * a.pL, r1 = r0 + a.pL, c = 2 * I;
  w = real(0.25) * ((ux[r0 + c - 1] + ux[r0 + c]) + (ux[r1 + c - 1] + ux[r1 + c]));
  const real* T = a.gc[G2_TA];
  const real tl = T[J * a.pC + I - 1], tr = T[J * a.pC + I];
  const real q = quick8(w, tc_at(a, T, I - 2, J), tl, tr, tc_at(a, T, I + 1, J));
  dc = real(2) * w * (q - (w >= real(0) ? tl : tr));
}
template <typename real>
__device__ __forceinline__ void yface(const SplitArgs<real>& a, int I, int J, real& w, real& dc) {
  const real* uy = a.mom + 2 * a.planeL;
  const int r0 = (2 * J - 1) * a.pL, r1 = r0 + a.pL, c = 2 * I;
  w = real(0.25) * ((uy[r0 + c] + uy[r1 + c]) + (uy[r0 + c + 1] + uy[r1 + c + 1]));
  const real* T = a.gc[G2_TA];
  const real tl = T[(J - 1) * a.pC + I], tr = T[J * a.pC + I];
  const real q = quick8(w, tc_at(a, T, I, J - 2), tl, tr, tc_at(a, T, I, J + 1));
  dc = real(2) * w * (q - (w >= real(0) ? tl : tr));
}

// coefficients of a_P T_P - a_W T_W - a_E T_E - a_S T_S - a_N T_N = b
template <typename real>
__global__ __launch_bounds__(256) void k_gs2_assemble(SplitArgs<real> a, int dt) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
  if (I >= a.NXc) return;
  const real al = a.alpha, h = real(2), zero = real(0);
  const int o = J * a.pC + I;
  real aW = zero, aE = zero, aS = zero, aN = zero;
  real cW = zero, cE = zero, cS = zero, cN = zero;
  real sW = zero, sE = zero, sS = zero, sN = zero;
  real w, dc;
  if (I >= 1) {
    xface(a, I, J, w, dc);
    aW = al + h * fmax(w, zero);
    cW = al + h * fmax(-w, zero);
    sW = dc;
  } else if (a.tfix[0]) {
    cW = real(2) * al;
    sW = real(2) * al * a.Tw[0];
  }
  if (I <= a.NXc - 2) {
    xface(a, I + 1, J, w, dc);
    aE = al + h * fmax(-w, zero);
    cE = al + h * fmax(w, zero);
    sE = -dc;
  } else if (a.tfix[1]) {
    cE = real(2) * al;
    sE = real(2) * al * a.Tw[1];
  }
  if (J >= 1) {
    yface(a, I, J, w, dc);
    aS = al + h * fmax(w, zero);
    cS = al + h * fmax(-w, zero);
    sS = dc;
  } else if (a.tfix[2]) {
    cS = real(2) * al;
    sS = real(2) * al * a.Tw[2];
  }
  if (J <= a.NYc - 2) {
    yface(a, I, J + 1, w, dc);
    aN = al + h * fmax(-w, zero);
    cN = al + h * fmax(w, zero);
    sN = -dc;
  } else if (a.tfix[3]) {
    cN = real(2) * al;
    sN = real(2) * al * a.Tw[3];
  }
  const real ct = h * h / real(dt);
  a.gc[G2_AP][o] = (((ct + cW) + cE) + cS) + cN;
  a.gc[G2_AW][o] = aW;
  a.gc[G2_AE][o] = aE;
  a.gc[G2_AS][o] = aS;
  a.gc[G2_AN][o] = aN;
  a.gc[G2_B][o] = ((((ct * a.gc[G2_TA][o]) + sW) + sE) + sS) + sN;
}

// One line of a sweep by the Thomas algorithm: n unknowns at X + k * step,
// lower -lo, diagonal aP, upper -up; the right-hand side b + c1 * Y1 + c2 * Y2
// with the other direction's neighbours Y1, Y2 (zero-weighted at walls) read
// from the previous iterate X0.
template <typename real>
__device__ __forceinline__ void thomas_line(const SplitArgs<real>& a, int base, int step, int n,
                                            int lo_k, int up_k, int c1_k, int c2_k, int d1, int d2,
                                            const real* __restrict__ X0, real* __restrict__ X) {
  // distinct planes: restrict lets the unrolled loop issue later unknowns'
  // loads before earlier unknowns' stores
  const real* __restrict__ aP = a.gc[G2_AP];
  const real* __restrict__ L = a.gc[lo_k];
  const real* __restrict__ U = a.gc[up_k];
  const real* __restrict__ C1 = a.gc[c1_k];
  const real* __restrict__ C2 = a.gc[c2_k];
  const real* __restrict__ b = a.gc[G2_B];
  real* __restrict__ cp = a.gc[G2_CP];
  real* __restrict__ rp = a.gc[G2_RP];
  real cprev = real(0), rprev = real(0);
  // unrolled so that the loads of several unknowns are in flight at once:
  // only c' and r' carry from one unknown to the next
#pragma unroll 8
  for (int k = 0; k < n; ++k) {
    const int o = base + k * step;
    const real c1 = C1[o], c2 = C2[o];
    const real y1 = c1 != real(0) ? X0[o + d1] : real(0);
    const real y2 = c2 != real(0) ? X0[o + d2] : real(0);
    const real rhs = (b[o] + c1 * y1) + c2 * y2;
    const real lo = -L[o], up = -U[o];
    real cpk, rpk;
    if (k == 0) {
      cpk = up / aP[o];
      rpk = rhs / aP[o];
    } else {
      const real m = aP[o] - lo * cprev;
      cpk = up / m;
      rpk = (rhs - lo * rprev) / m;
    }
    cp[o] = cpk;
    rp[o] = rpk;
    cprev = cpk;
    rprev = rpk;
  }
  real x = rprev;
  X[base + (n - 1) * step] = x;
#pragma unroll 8
  for (int k = n - 2; k >= 0; --k) {
    const int o = base + k * step;
    x = rp[o] - cp[o] * x;
    X[o] = x;
  }
}

// x-lines: one thread per coarse row, iterate A -> B
template <typename real>
__global__ __launch_bounds__(64) void k_gs2_xlines(SplitArgs<real> a) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= a.NYc) return;
  thomas_line(a, J * a.pC, 1, a.NXc, G2_AW, G2_AE, G2_AS, G2_AN, -a.pC, a.pC, a.gc[G2_TA],
              a.gc[G2_TB]);
}
// y-lines: one thread per coarse column, iterate B -> A
template <typename real>
__global__ __launch_bounds__(64) void k_gs2_ylines(SplitArgs<real> a) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= a.NXc) return;
  thomas_line(a, I, a.pC, a.NYc, G2_AS, G2_AN, G2_AW, G2_AE, -1, 1, a.gc[G2_TB], a.gc[G2_TA]);
}

// coarse temperature from a dense T0 (mean of each 2 x 2 block), or 0
template <typename real>
__global__ __launch_bounds__(256) void k_gs2_init(SplitArgs<real> a, const double* __restrict__ T0) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y;
  if (I >= a.NXc) return;
  double t = 0.0;
  if (T0) {
    const int r0 = 2 * J * a.nx, r1 = r0 + a.nx, c = 2 * I;
    t = 0.25 * ((T0[r0 + c] + T0[r0 + c + 1]) + (T0[r1 + c] + T0[r1 + c + 1]));
  }
  a.gc[G2_TA][J * a.pC + I] = real(t);
}

// ---- LBM-MCM (Sec. 6, Eq 97-102) ------------------------------------------
// A walker at node (i, j) steps to x+, y+, x- or y- with Eq 99's
// probabilities from the node velocity (link weights alpha - u, alpha - v,
// alpha, alpha over their sum, Eq 100); the link through a fixed-temperature
// wall (half a spacing away) has its weight doubled and absorbs the walker;
// a step into an adiabatic wall is refused.  Eq 101 picks the direction by
// the cumulative thresholds in FP64 from one uniform draw per step.  Draws:
// splitmix64 (Steele, Lea and Flood; Vigna's constants), draw k of walker w
// at node p is mix(s0 + (k + 1) gamma) with s0 = mix(seed + (1 + p N + w)
// gamma), RN = (draw >> 11) 2^-53.  Each node counts its walkers per
// absorbing wall (integer atomics, so the estimate of Eq 102 does not depend
// on the order in which walks finish).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr unsigned long long kGamma = 0x9E3779B97F4A7C15ull;

template <typename real>
__global__ __launch_bounds__(256) void k_mcm_clear(SplitArgs<real> a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 5 * a.nx * a.ny) a.mcm_count[k] = 0;
  if (k == 0) a.mcm_stats[0] = 0ull;
}

// Eq 101's cumulative thresholds of every node, once per solve (they depend
// only on the node's velocity and walls): 4 doubles per node (the fourth is
// padding), so a step reads one 32-byte record; c3 = -1 marks a node where
// Eq 99 loses positivity (|u| or |v| >= alpha)
template <typename real>
__global__ __launch_bounds__(256) void k_mcm_prep(SplitArgs<real> a, double* __restrict__ cth) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= a.nx) return;
  const double al = (double)a.alpha;
  const double u = (double)a.mom[a.planeL + j * a.pL + i];
  const double v = (double)a.mom[2 * a.planeL + j * a.pL + i];
  const double fe = (a.tfix[1] && i == a.nx - 1) ? 2.0 : 1.0;
  const double fn = (a.tfix[3] && j == a.ny - 1) ? 2.0 : 1.0;
  const double fw = (a.tfix[0] && i == 0) ? 2.0 : 1.0;
  const double fs = (a.tfix[2] && j == 0) ? 2.0 : 1.0;
  const double we = fe * (al - u), wn = fn * (al - v), ww = fw * al, ws = fs * al;
  const double D = ((we + wn) + ww) + ws;
  double4* rec = (double4*)cth + (j * a.nx + i);
  if (!(we >= 0.0 && wn >= 0.0 && D > 0.0)) {
    *rec = double4{-1.0, -1.0, -1.0, 0.0};
    return;
  }
  const double c1 = we / D;
  const double c2 = c1 + wn / D;
  *rec = double4{c1, c2, c2 + ww / D, 0.0};
}

template <typename real>
__global__ __launch_bounds__(256) void k_mcm_walk(SplitArgs<real> a, const double* __restrict__ cth,
                                                  int walkers, unsigned long long seed,
                                                  long long max_steps) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nodes = (long long)a.nx * a.ny;
  if (t >= nodes * walkers) return;
  const int node = (int)(t / walkers), w = (int)(t - (long long)node * walkers);
  int i = node % a.nx, j = node / a.nx;
  const unsigned long long s0 =
      mix64(seed + (1ull + (unsigned long long)node * (unsigned long long)walkers +
                    (unsigned long long)w) * kGamma);
  int side = -1;
  for (long long k = 0; k < max_steps; ++k) {
    const double rn = (double)(mix64(s0 + (unsigned long long)(k + 1) * kGamma) >> 11) *
                      (1.0 / 9007199254740992.0);
    const double4 rec = ((const double4*)cth)[j * a.nx + i];
    const double c1 = rec.x, c2 = rec.y, c3 = rec.z;
    // a node past Eq 99's positivity stops the walker (counted as capped)
    if (c3 < 0.0) break;
    int ti = i, tj = j, s;
    if (rn < c1) { ti = i + 1; s = 1; }
    else if (rn < c2) { tj = j + 1; s = 3; }
    else if (rn < c3) { ti = i - 1; s = 0; }
    else { tj = j - 1; s = 2; }
    if (ti >= 0 && ti < a.nx && tj >= 0 && tj < a.ny) {
      i = ti;
      j = tj;
    } else if (a.tfix[s]) {
      side = s;
      break;
    }
  }
  atomicAdd(&a.mcm_count[5 * node + (side < 0 ? 4 : side)], 1);
}

// node temperatures: the mean wall temperature recorded by the absorbed
// walkers (sides summed in a fixed order); the cap count is totalled
template <typename real>
__global__ __launch_bounds__(256) void k_mcm_finish(SplitArgs<real> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= a.nx) return;
  const int* c = a.mcm_count + 5 * (j * a.nx + i);
  const int absorbed = ((c[0] + c[1]) + c[2]) + c[3];
  double t = 0.0;
  for (int s = 0; s < 4; ++s) t += (double)c[s] * (double)a.Tw[s];
  a.mom[3 * a.planeL + j * a.pL + i] = absorbed > 0 ? real(t / absorbed) : real(0);
  if (c[4]) atomicAdd(a.mcm_stats, (unsigned long long)c[4]);
}

}  // namespace

// doubles of the interface record for ny rows: the scalars, then per unit
// the ghost sums of both parities and the p_bar sums
int split_iface_doubles(int ny) { return kIfacePart + 6 * iface_blocks(ny); }

template <typename real>
static SplitArgs<real> make_args(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                                 int cur, int mom_all) {
  SplitArgs<real> a;
  const int nxt = cur ^ 1;
  a.fin = P.f[cur];
  a.fout = P.f[nxt];
  a.gin = P.g[cur];
  a.gout = P.g[nxt];
  a.mom = P.mom;
  a.xf = P.xf;
  a.pL = G.pL;
  a.planeL = G.planeL;
  a.nl = G.fv_only ? 0 : (G.lbm_only || G.gs2 || G.mcm) ? G.nx : G.ib + 1;
  a.u = P.u[cur];
  a.v = P.v[cur];
  a.T = P.T[cur];
  a.us = P.u[nxt];
  a.vs = P.v[nxt];
  a.Tn = P.T[nxt];
  a.pin = P.p[cur];
  a.p = P.p[nxt];
  a.pF = G.pF;
  a.iface = P.iface;
  a.nx = G.nx;
  a.ny = G.ny;
  a.s = G.s;
  a.c0 = G.c0;
  a.ib = G.ib;
  for (int k = 0; k < 10; ++k) a.gc[k] = P.gc[k];
  a.mcm_count = P.mcm_count;
  a.mcm_stats = P.mcm_stats;
  a.NXc = G.NXc;
  a.NYc = G.NYc;
  a.pC = G.pC;
  a.gdir = G.gdir;
  a.transposed = G.transposed;
  a.west_wall = G.fv_only;
  a.east_wall = G.lbm_only;
  a.kind = S.kind;
  a.mom_all = mom_all;
  a.par = cur;
  a.iface_on = !G.fv_only && !G.lbm_only && !G.gs2 && !G.mcm;
  a.umean = real(0);
  a.omega = real(1.0 / S.tau);
  a.omegaT = real(1.0 / S.tauT);
  a.tau = real(S.tau);
  a.nu = real(S.nu);
  a.alpha = real(S.alpha);
  a.gbeta = real(S.gbeta);
  a.Tref = real(S.T_ref);
  a.ulid = real(S.ulid);
  for (int k = 0; k < 4; ++k) {
    a.tfix[k] = S.tfix[k];
    a.Tw[k] = real(S.Tw[k]);
  }
  return a;
}

// Fused region for a band height: strips need the whole 64-lane window
// inside the stored columns (x0 + 63 <= nx - 1) and at least one row clear
// of the walls' ghost rules (ny >= 5).
static FvRegion fv_region(const SplitGeom& G, int band) {
  FvRegion r{};
  r.xa = G.c0 - 1 + (G.fv_only ? 1 : 0);
  const int span = G.nx - 64 - r.xa;
  r.nst = (span < 0 || G.ny < 5) ? 0 : span / kFvOut + 1;
  r.band = band;
  if (r.nst) {
    r.xcut = r.xa + kFvOut * r.nst + 1;  // east end of the whole strips
    r.npart = r.xcut < G.nx - 4 ? 1 : 0;
    r.nbands = (G.ny - 4 + band - 1) / band;
    r.X0 = r.xa + 2;
    r.X1 = G.nx - 4;
  } else {
    r.X0 = G.nx + 1;
    r.X1 = G.nx;
  }
  r.nwaves = (r.nst + r.npart) * r.nbands;
  r.nfc = G.nx - G.c0 + 1;
  r.nbt = G.ny + 1 < 6 ? G.ny + 1 : 6;
  const int nmid = G.ny - 5 > 0 ? G.ny - 5 : 0;
  r.wl = r.X0 - G.c0;
  r.wr = G.nx - r.X1;
  r.nframe = r.nbt * r.nfc + nmid * (r.wl + r.wr);
  r.nfrb = (r.nframe + 255) / 256;
  return r;
}

// rows per wave of the march: the longest of 32, 24, 16, 12, 8, 4 that still
// gives the chip 2048 waves (a band's halo costs 4.5 row loads; measured on
// MI355X, us per step at 32 / 24 / 16 / 12 rows: FV-only 4096^2 148 / 153 /
// 158 / -, 2048^2 37.3 / 33.2 / 38.4 / 40.7, 1024^2 24.0 / 19.3 / 14.3 /
// 12.8; the 4096^2 divided cavity 319 / 327 / 328 / -)
static FvRegion fv_region_auto(const SplitGeom& G) {
  const int bands[6] = {32, 24, 16, 12, 8, 4};
  FvRegion r{};
  for (int k = 0; k < 6; ++k) {
    r = fv_region(G, bands[k]);
    if (r.nwaves >= 2048) break;
  }
  return r;
}

template <typename real, int CONV>
static void launch_fv(const SplitArgs<real>& a, const FvRegion& R, hipStream_t s) {
  const int nb = R.nfrb + (R.nwaves + 3) / 4;
  if (a.iface_on)
    hipLaunchKernelGGL((k_dd_fv<real, CONV, true>), dim3(nb), dim3(256), 0, s, a, R);
  else
    hipLaunchKernelGGL((k_dd_fv<real, CONV, false>), dim3(nb), dim3(256), 0, s, a, R);
}

template <typename real>
hipError_t launch_split_step(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int cur, int mom_all, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, cur, mom_all);
  // the march addresses the FV arrays with 32-bit byte offsets
  if ((size_t)(G.ny + 1) * G.pF * sizeof(real) >= ((size_t)1 << 31)) return hipErrorInvalidValue;
  const dim3 gl((a.nl + 63) / 64, (G.ny + 3) / 4);
  if (G.lbm_only) {  // one zone kernel per step
    hipLaunchKernelGGL(k_dd_lbm<real>, gl, dim3(256), 0, s, a, 0);
    return hipGetLastError();
  }
  const bool split = !G.fv_only;
  const FvRegion R = fv_region_auto(G);
  if (S.conv == 1) launch_fv<real, 1>(a, R, s);
  else if (S.conv == 2) launch_fv<real, 2>(a, R, s);
  else launch_fv<real, 0>(a, R, s);
  if (split) {
    // the LBM zone, after rows of blocks for the p_bar sums
    const int nbx = (G.ib + 63) / 64, pr = (iface_blocks(G.ny) + 4 * nbx - 1) / (4 * nbx);
    hipLaunchKernelGGL(k_dd_lbm<real>, dim3(nbx, (G.ny + 3) / 4 + pr), dim3(256), 0, s, a, pr);
    hipLaunchKernelGGL(k_dd_xb<real>, dim3(iface_blocks(G.ny)), dim3(kIfBlock), 0, s, a, 0);
  }
  return hipGetLastError();
}

template <typename real>
hipError_t launch_split_init(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             const double* T0, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, 0, 1);
  // LBM nodes 0 .. nl-1 and stored FV columns c0-2 .. nx
  const int wf = G.pF > 0 ? G.nx - G.c0 + 3 : 0;
  const int w = wf > a.nl ? wf : a.nl;
  hipLaunchKernelGGL(k_dd_init<real>, dim3((w + 255) / 256, G.ny), dim3(256), 0, s, a, T0);
  // the second FV buffers start equal to the first (prescribed/wall faces)
  const SplitArgs<real> b = make_args<real>(G, P, S, 1, 1);
  hipLaunchKernelGGL(k_dd_init<real>, dim3((w + 255) / 256, G.ny), dim3(256), 0, s, b, T0);
  // the ghost values and sums step 0 reads (written as by a step of parity 1)
  if (b.iface_on)
    hipLaunchKernelGGL(k_dd_xb<real>, dim3(iface_blocks(G.ny)), dim3(kIfBlock), 0, s, b, 1);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_split_output(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                               int cur, real* out, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, cur, 1);
  hipLaunchKernelGGL(k_dd_output<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a, out);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_gs2_lbm(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                          int cur, int mom_all, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, cur, mom_all);
  hipLaunchKernelGGL(k_gs2_lbm<real>, dim3((G.nx + 63) / 64, (G.ny + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_gs2_energy(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int dt, int K, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, 0, 0);
  hipLaunchKernelGGL(k_gs2_assemble<real>, dim3((G.NXc + 255) / 256, G.NYc), dim3(256), 0, s, a,
                     dt);
  for (int k = 0; k < K; ++k) {
    hipLaunchKernelGGL(k_gs2_xlines<real>, dim3((G.NYc + 63) / 64), dim3(64), 0, s, a);
    hipLaunchKernelGGL(k_gs2_ylines<real>, dim3((G.NXc + 63) / 64), dim3(64), 0, s, a);
  }
  hipLaunchKernelGGL(k_gs2_interp<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_gs2_init(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                           const double* T0, hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, 0, 1);
  hipLaunchKernelGGL(k_dd_init<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a, T0);
  const SplitArgs<real> b = make_args<real>(G, P, S, 1, 1);
  hipLaunchKernelGGL(k_dd_init<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, b, T0);
  hipLaunchKernelGGL(k_gs2_init<real>, dim3((G.NXc + 255) / 256, G.NYc), dim3(256), 0, s, a, T0);
  hipLaunchKernelGGL(k_gs2_interp<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename real>
hipError_t launch_mcm_energy(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int walkers, unsigned long long seed, long long max_steps,
                             hipStream_t s) {
  const SplitArgs<real> a = make_args<real>(G, P, S, 0, 0);
  const long long nodes = (long long)G.nx * G.ny, threads = nodes * walkers;
  double* cth = P.mcm_cth;
  hipLaunchKernelGGL(k_mcm_clear<real>, dim3((unsigned)((5 * nodes + 255) / 256)), dim3(256), 0, s,
                     a);
  hipLaunchKernelGGL(k_mcm_prep<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a, cth);
  hipLaunchKernelGGL(k_mcm_walk<real>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, a,
                     (const double*)cth, walkers, seed, max_steps);
  hipLaunchKernelGGL(k_mcm_finish<real>, dim3((G.nx + 255) / 256, G.ny), dim3(256), 0, s, a);
  return hipGetLastError();
}

#define LF_SPLIT_INST(real)                                                                   \
  template hipError_t launch_split_step<real>(const SplitGeom&, const SplitPtrs<real>&,        \
                                              const SplitParams&, int, int, hipStream_t);      \
  template hipError_t launch_split_init<real>(const SplitGeom&, const SplitPtrs<real>&,        \
                                              const SplitParams&, const double*, hipStream_t); \
  template hipError_t launch_split_output<real>(const SplitGeom&, const SplitPtrs<real>&,      \
                                                const SplitParams&, int, real*, hipStream_t);  \
  template hipError_t launch_gs2_lbm<real>(const SplitGeom&, const SplitPtrs<real>&,           \
                                           const SplitParams&, int, int, hipStream_t);         \
  template hipError_t launch_gs2_energy<real>(const SplitGeom&, const SplitPtrs<real>&,        \
                                              const SplitParams&, int, int, hipStream_t);      \
  template hipError_t launch_gs2_init<real>(const SplitGeom&, const SplitPtrs<real>&,          \
                                            const SplitParams&, const double*, hipStream_t);   \
  template hipError_t launch_mcm_energy<real>(const SplitGeom&, const SplitPtrs<real>&,        \
                                              const SplitParams&, int, unsigned long long,     \
                                              long long, hipStream_t);
LF_SPLIT_INST(float)
LF_SPLIT_INST(double)
#undef LF_SPLIT_INST

}  // namespace lf
