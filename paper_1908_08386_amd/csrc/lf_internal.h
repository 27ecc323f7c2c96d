// Internal interface between the host runtime (lbmfvm_api.cpp) and the HIP
// kernels (*.hip).  Not installed; the public ABI is include/lbmfvm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

// Low word of a compensated FP32 temperature T = hi + lo, stored as a signed
// byte: lo in units of 2^-8 ulp(hi), one byte per node and plane.
typedef signed char tlo_t;

// Wall description as the kernels see it (sides W, E, S, N).
struct WallSet {
  int xper, yper;     // periodic along x / y
  double uw[4];       // tangential wall speed per side
  int tfix[4];        // 1: fixed-temperature wall, 0: adiabatic
  double Tw[4];       // wall temperature of fixed-temperature walls
};

// Scalar parameters of the Mode H step.
struct HybridParams {
  double omega;       // 1 / tau
  double alpha;       // thermal diffusivity (lattice units)
  double gbeta;       // g * beta
  double T_ref;       // reference temperature of the buoyancy term
  double gx, gy;      // extra body acceleration
  int conv;           // 0 QUICK, 1 central, 2 upwind
};

// Geometry of one cavity's planes inside the workspace.
struct Grid {
  int nx, ny, pitch;  // pitch: row stride in elements (multiple of 64)
  long long plane;    // elements between successive planes: ny * pitch plus a pad
};

// ---- batched Mode H -------------------------------------------------------
// One wave-sized tile of one cavity: 62 output columns from strip * 62,
// rows j0 .. j1 - 1.
struct TileDesc {
  int cav, strip, j0, j1;
};
// One cavity of a batch: buffers, geometry, parameters, walls (no periodic
// sides).  cur: buffer holding the state at the start of a launch sequence.
template <typename real>
struct CavDesc {
  real* f[2];
  real* T[2];
  tlo_t* Tlo[2];  // compensated temperature low words (codes), or null
  real* mom;   // rho, u, v planes
  real* snap;  // residual snapshot u, v, T planes
  int nx, ny, pitch, plane;
  int cur, pad0;
  int tfix[4];
  double Tw[4];
  double uw[4];
  double omega, alpha, gbeta, Tref;
};
// Residual work unit (rows j0 .. j1 - 1 of one cavity) and per-cavity fold
// of consecutive partials.
struct ResidTile {
  int cav, j0, j1, pad;
};
struct FoldDesc {
  int cav, start, count, pad;
};

template <typename real>
// row1: every live tile is a single row (j1 = j0 + 1)
hipError_t launch_batch_step(const TileDesc* tiles, const int* ntiles, int max_tiles,
                             const CavDesc<real>* cavs, int parity, int write_mom, int conv,
                             int row1, hipStream_t s);
// residual sums per live cavity into out[cav * 8 + 0 .. 6]
template <typename real>
hipError_t launch_batch_residual(const ResidTile* rt, const int* nrt, int max_rt,
                                 const FoldDesc* fd, const int* nfold, int max_fold,
                                 const CavDesc<real>* cavs, double* part, double* out,
                                 hipStream_t s);

// One fused Mode H step: pull-stream + bounce-back + moments + explicit FV
// energy update + BGK collision with buoyancy.  f planes are stored shifted
// (f - w_q).  mom (rho, u, v planes) is written only when non-null.
// Tlo_in / Tlo_out: low-word codes of a compensated temperature (or null;
// FP32 only).
template <typename real>
hipError_t launch_hybrid_step(const Grid& g, const WallSet& w,
                              const HybridParams& p, const real* fin,
                              real* fout, const real* Tin, real* Tout,
                              const tlo_t* Tlo_in, tlo_t* Tlo_out,
                              real* mom, int band, hipStream_t s);

// f = f_eq(1, u0) - w, T = T0, mom = (1, u0, v0), snapshots = (u0, v0, T0)
// from dense double staging arrays (u0 / v0 may be null for zero).
// Tlo (or null) receives the code of T0 - T (FP32 only).
template <typename real>
hipError_t launch_init(const Grid& g, const double* T0, const double* u0,
                       const double* v0, real* f, real* T, real* mom,
                       real* snap, tlo_t* Tlo, hipStream_t s);

// Residual partial sums: per block six FP64 sums
// {sum (u-us)^2, sum u^2, sum (v-vs)^2, sum v^2, sum (T-Ts)^2, sum T^2}
// plus a non-finite flag; then a single-block pass in fixed order writes
// out[0..5] and out[6] = count of non-finite values.  Snapshot updated.
template <typename real>
hipError_t launch_residual(const Grid& g, const real* mom, const real* T,
                           real* snap, double* partials, int nblocks,
                           double* out, hipStream_t s);

// Nusselt numbers of the west and east walls into out[0..7] (lf_nusselt
// order).
template <typename real>
hipError_t launch_nusselt(const Grid& g, const WallSet& w, const real* T,
                          double* out, hipStream_t s);

// out[0] = sum of the post-collision populations (unshifted), out[1] = sum T
template <typename real>
hipError_t launch_mass(const Grid& g, const real* f, const real* T,
                       double* partials, int nblocks, double* out,
                       hipStream_t s);

// Dense copy of one plane into dst ([ny][nx]) as double or as real.
template <typename real>
hipError_t launch_unpack(const Grid& g, const real* plane, void* dst,
                         int as_f64, hipStream_t s, int pressure = 0);

}  // namespace lf

namespace lf {

// ---- domain-decomposed mode ---------------------------------------------
// Geometry: nx even, s = nx / 2, FV cells from c0 = s - 1, LBM nodes up to
// ib = s + 1; pL / pF are the row pitches of the LBM and FV arrays.
// Single-method cavities use the same zone kernels: fv_only (s = c0 = 0, a
// wall on the FV zone's west side, no LBM zone) or lbm_only (s = ib = nx, a
// wall on the LBM zone's east side, no FV zone).
// gs2: grid setting 2 of the coupled method (lattice on all nx x ny nodes,
// temperature on the NXc x NYc coarse control volumes of 2 x 2 nodes, row
// pitch pC), with s = ib = nx like lbm_only.
struct SplitGeom {
  int nx, ny, s, c0, ib, pL, pF;
  int planeL;  // elements between successive LBM-zone planes (ny * pL plus a pad)
  int fv_only, lbm_only;
  int gs2, NXc, NYc, pC;
  // horizontally divided cavity: stored transposed (the caller's x is the
  // stored y) with gravity along the stored -x
  int gdir, transposed;
  // LBM-MCM (Sec. 6): lattice on all nodes like gs2, node temperatures from
  // Monte Carlo walkers (mom plane 3)
  int mcm;
};

template <typename real>
struct SplitPtrs {
  real* f[2];   // 9 planes, planeL apart (shifted populations)
  real* g[2];   // 5 planes
  real* mom;    // rho, u, v, T planes of the LBM zone
  real* xf;     // 18 values per row: streamed state of column ib - 1
  real* u[2];   // x-faces, ny rows * pF
  real* v[2];   // y-faces, (ny + 1) rows * pF
  real* T[2];   // centres
  real* p[2];   // centres (ping-pong: each FV step reads one and writes the other)
  double* iface;  // interface scalars (the LBM zone's mass change since init
                  // and its running sum), from [8] per 64 rows the ghost sums
                  // of both step parities and the p_bar sums
                  // (split_iface_doubles(ny) doubles in all)
  // grid setting 2, NYc rows * pC each: T (iterate A), T (iterate B),
  // a_P, a_W, a_E, a_S, a_N, b, and the Thomas sweep's c', r'
  real* gc[10];
  // LBM-MCM: per node the walkers absorbed by each wall (W, E, S, N) and
  // those still walking at the step cap; [0] of stats: the cap count total
  int* mcm_count;
  unsigned long long* mcm_stats;
  double* mcm_cth;  // Eq 101's thresholds per node, 4 doubles (one padding)
};

struct SplitParams {
  double tau, tauT, nu, alpha, gbeta, T_ref;
  int conv;   // 0 QUICK, 1 central, 2 upwind
  int kind;   // 0 non-equilibrium extrapolation, 1 finite-difference gradient
  int tfix[4];
  double Tw[4];
  double ulid;  // tangential velocity of the north wall (split, FV-only, LBM-only)
};

// doubles of the split mode's interface record (SplitPtrs::iface) for ny rows
int split_iface_doubles(int ny);

// One step; the state is read from buffers [cur] and written to [cur ^ 1].
// mom_all: write the moments of every LBM node (else only the shared and
// ghost columns the next step needs).
template <typename real>
hipError_t launch_split_step(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int cur, int mom_all, hipStream_t s);
// Rest state, T = T0 (dense [ny][nx] doubles in device memory, or null).
template <typename real>
hipError_t launch_split_init(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             const double* T0, hipStream_t s);
// Grid setting 2: one lattice step (mom_all: write rho, u, v of every node,
// which the energy step and the output read); one energy step of length dt
// lattice steps with K line sweeps, then the node temperatures; the coarse
// temperature from T0 (dense [ny][nx] doubles in device memory, or null)
// as the mean of each 2 x 2 block, then the node temperatures.
template <typename real>
hipError_t launch_gs2_lbm(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                          int cur, int mom_all, hipStream_t s);
template <typename real>
hipError_t launch_gs2_energy(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int dt, int K, hipStream_t s);
template <typename real>
hipError_t launch_gs2_init(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                           const double* T0, hipStream_t s);
// LBM-MCM: one Monte Carlo solve of the node temperatures with the velocity
// of the last lattice step: `walkers` walks per node, stream seed `seed`, at
// most `max_steps` steps each.
template <typename real>
hipError_t launch_mcm_energy(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                             int walkers, unsigned long long seed, long long max_steps,
                             hipStream_t s);
// Dense rho, u, v, T planes ([4][ny][nx]) of the current state.
template <typename real>
hipError_t launch_split_output(const SplitGeom& G, const SplitPtrs<real>& P, const SplitParams& S,
                               int cur, real* out, hipStream_t s);

}  // namespace lf
