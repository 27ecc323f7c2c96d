/*
 * lbmfvm.h -- C ABI of the MI355X (gfx950) hybrid lattice-Boltzmann /
 * finite-volume natural-convection library.
 *
 * Method: Li, Yang & Zhang, "Hybrid LBM-FVM and LBM-MCM methods for fluid
 * flow and heat transfer simulation" (arXiv:1908.08386).
 *   - Mode H (LF_MODE_HYBRID), Sec. 5: D2Q9 BGK lattice Boltzmann (Eq 4-9,
 *     Eq 16-18) gives the velocity on the whole cavity; an explicit
 *     conservative finite-volume energy balance (Eq 24 / Eq 76, QUICK
 *     convection) gives the temperature on the same cells; the temperature
 *     acts back through the Boussinesq buoyancy force (Eq 18, Eq 81).
 *   - Mode DD (LF_MODE_SPLIT), Sec. 4: LBM (D2Q9 flow + D2Q5 heat, Eq 19-23)
 *     on the west part, FVM on the east part, three shared columns, coupled
 *     through non-equilibrium extrapolation (Eq 60, Eq 94-95) or the
 *     finite-difference velocity-gradient reconstruction (Eq 70-72) with the
 *     density transfer of Eq 91-93; the level rho0 of Eq 93 is shifted each
 *     step so that the LBM zone keeps its mass at init (the walls conserve
 *     it; it changes only through the boundary node's links).  With a
 *     sliding north wall it is the lid-driven cavity of Sec. 3.3 (Fig. 5;
 *     hybrid method 1 = non-equilibrium extrapolation, 2 = finite-difference
 *     gradient).  LF_MODE_SPLIT_H divides the cavity
 *     horizontally instead (Fig. 17b: LBM in the lower half, FVM in the
 *     upper half; stored transposed with gravity along the stored -x, so
 *     the same kernels run it; fields, walls and Nusselt numbers keep the
 *     caller's orientation).
 *   - The two single methods of the Sec. 4.2 comparison on the whole cavity,
 *     with the zone kernels of Mode DD: LF_MODE_PURE_FV (staggered FVM,
 *     explicit momentum with artificial compressibility, Eq 74-76) and
 *     LF_MODE_PURE_LBM (D2Q9 flow + D2Q5 heat, Eq 19-23).
 *   - Mode H on grid setting 2 (LF_MODE_HYBRID_GS2, Sec. 5.1, Fig. 30): the
 *     lattice on all nx x ny nodes, the temperature on nx/2 x ny/2 control
 *     volumes of 2 x 2 nodes, one implicit energy step per S lattice steps
 *     (S = nx, i.e. 2NX, by default; lf_case_set_subcycle).
 *   - LBM-MCM (LF_MODE_LBM_MCM, Sec. 6, Eq 97-102, Fig. 39): the lattice on
 *     all nodes, the node temperatures from Monte Carlo walkers (Eq 99's
 *     probabilities from the lattice velocity), one solve per S lattice
 *     steps (lf_case_set_mcm).
 *
 * Conventions (all entry points):
 *   - Every call returns lf_status; LF_OK is 0.  On failure
 *     lf_last_error() returns a thread-local message.  No exception, abort
 *     or exit crosses the ABI.
 *   - Handles are opaque; *_destroy(NULL) is a no-op.  Handles are not
 *     thread-safe: use one ctx per host thread.
 *   - The library never allocates device memory.  The caller asks for
 *     *_workspace_bytes and binds a device buffer of at least that size
 *     (256-byte aligned) with *_bind_workspace; the buffer stays owned by the
 *     caller and must outlive the handle's use.  Host arrays passed in are
 *     copied before the call returns.
 *   - All device work is enqueued on the HIP stream given to lf_ctx_create.
 *     init, step and fetch into device memory are asynchronous on that
 *     stream; calls that return host values (residual, nusselt, mass,
 *     run_to_steady, fetch into host memory, save) synchronise it.
 *   - Fields are row-major [ny][nx] (index j*nx + i); j = 0 is the bottom
 *     wall (gravity points to -y), i = 0 the west wall.  Cell (i, j) has its
 *     centre at (i + 1/2, j + 1/2) lattice units; walls lie on cell faces.
 *     u, v are lattice velocities; T is in units of the wall temperature
 *     difference (hot wall +1/2, cold wall -1/2 in the cavity cases).
 */
#ifndef LBMFVM_H
#define LBMFVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LF_ABI_VERSION 1

typedef enum {
  LF_OK = 0,
  LF_EINVAL = 1,      /* bad argument or combination of settings          */
  LF_ENOMEM = 2,      /* host allocation failed                            */
  LF_EWORKSPACE = 3,  /* no workspace bound, or it is too small/misaligned */
  LF_EDEVICE = 4,     /* a HIP call failed                                 */
  LF_EUNSTABLE = 5,   /* parameters outside the explicit scheme's limits   */
  LF_EDIVERGED = 6,   /* NaN or Inf found in the fields                    */
  LF_ENOTCONV = 7,    /* run_to_steady hit max_steps                       */
  LF_ESTATE = 8,      /* call out of order (e.g. step before init)         */
  LF_ENOTIMPL = 9
} lf_status;

enum { LF_F32 = 0, LF_F64 = 1 };
enum {
  LF_MODE_HYBRID = 0,
  LF_MODE_SPLIT = 1,
  LF_MODE_PURE_FV = 2,
  LF_MODE_PURE_LBM = 3,
  LF_MODE_HYBRID_GS2 = 4,
  LF_MODE_SPLIT_H = 5,
  LF_MODE_LBM_MCM = 6
};
enum { LF_IFACE_NEQ_EXTRAP = 0, LF_IFACE_FD_GRADIENT = 1 };
enum { LF_CONV_QUICK = 0, LF_CONV_CENTRAL = 1, LF_CONV_UPWIND = 2 };
enum { LF_WALL_NOSLIP = 0, LF_WALL_PERIODIC = 1 };
enum { LF_T_DIRICHLET = 0, LF_T_ADIABATIC = 1, LF_T_PERIODIC = 2 };
enum { LF_SIDE_W = 0, LF_SIDE_E = 1, LF_SIDE_S = 2, LF_SIDE_N = 3 };
/* fields of *_fetch: LF_FIELD_P is the kinematic pressure c_s^2 (rho - 1):
 * the FV zone's p in the split modes, the lattice's in the LBM zone and Mode
 * H (from the density of the last step; in FP32 its absolute rounding is
 * that of rho near 1, ~4e-8)                                             */
enum { LF_FIELD_U = 0, LF_FIELD_V = 1, LF_FIELD_T = 2, LF_FIELD_RHO = 3, LF_FIELD_P = 4 };
/* run_to_steady stop rules (r_final[3] of lf_case_run_to_steady)          */
enum { LF_STOP_TOL = 1, LF_STOP_FLOOR = 2 };

typedef struct lf_ctx lf_ctx;
typedef struct lf_case lf_case;

/* Case geometry and numerics.  nx, ny >= 8.  Mode DD needs nx even and
 * split_col / overlap as documented in lf_case_create.                     */
typedef struct {
  int nx, ny;
  int precision; /* LF_F32 or LF_F64                                        */
  int mode;      /* LF_MODE_HYBRID, LF_MODE_SPLIT, LF_MODE_SPLIT_H,
                    LF_MODE_PURE_FV, LF_MODE_PURE_LBM, LF_MODE_HYBRID_GS2
                    or LF_MODE_LBM_MCM
                    (all but the first: walls at rest, no periodic sides,
                    start from rest; LF_MODE_HYBRID_GS2 needs even nx and
                    ny, the split modes an even divided extent >= 12)      */
  int split_col; /* Mode DD: first FV cell is split_col - 1; 0 => nx/2      */
  int overlap;   /* Mode DD: shared columns; 0 => 3 (the only value)        */
  int iface;     /* Mode DD: LF_IFACE_NEQ_EXTRAP or LF_IFACE_FD_GRADIENT
                    (split_col, overlap, iface: ignored by the other modes) */
  int tcomp;     /* Mode H, FP32: 1 = temperature kept as a compensated
                    pair hi + lo (FP32 words; increments below ulp(T) are
                    not lost near steady state; +8 B per node), 0 = plain  */
} lf_case_desc;

/* Physical groups (Eq 82-89).  Ra > 0, Pr > 0.  U_char is the buoyancy
 * velocity sqrt(g beta dT H) in lattice units; 0 selects 0.1, lowered where
 * the explicit updates need it (alpha <= 0.2, U^2 <= 2 alpha; the split
 * mode and the single-method cavities, whose parameters follow the split
 * mode's, also nu <= 0.08).  T_ref NaN selects 0 (the mid value of walls at +-1/2).
 * body_gx, body_gy add a constant body acceleration (test hook).           */
typedef struct {
  double Ra, Pr, U_char, T_ref;
  int conv; /* LF_CONV_QUICK (default), LF_CONV_CENTRAL, LF_CONV_UPWIND */
  double body_gx, body_gy;
} lf_physics;

/* One side of the box.  vel: LF_WALL_NOSLIP (half-way bounce-back; u_wall
 * is the tangential wall speed, along +x or +y, with the moving-wall term
 * 6 w_q rho_w (e_q . u_w), rho_w = 1) or LF_WALL_PERIODIC (both opposite
 * sides).  In LF_MODE_SPLIT, LF_MODE_PURE_FV and LF_MODE_PURE_LBM only the
 * north wall may move (the lid of Sec. 3.3; the FV zone takes the ghost
 * u = 2 u_wall - u_edge); other split-family modes and sides give
 * LF_ENOTIMPL.
 * thermal: LF_T_DIRICHLET (T = T_wall), LF_T_ADIABATIC, or LF_T_PERIODIC
 * (together with vel periodic).                                            */
typedef struct {
  int vel;
  double u_wall;
  int thermal;
  double T_wall;
} lf_wall;

/* Nusselt numbers of the west (hot) and east (cold) walls, Eq 90 with
 * X = x / ny: nu(j) = 2 ny (T_w - T_edge) / dT (half-cell wall flux);
 * *_max and their heights y = (j + 1/2) / ny (ties: lowest j); *_o2 the
 * wall-averaged second-order one-sided gradient through T_w and the first
 * two cell centres.  dT = T_W - T_E (1 when equal).                        */
typedef struct {
  double nu_hot, nu_cold, nu_hot_max, y_hot_max, nu_cold_max, y_cold_max,
      nu_hot_o2, nu_cold_o2;
} lf_nusselt;

/* ---- library ---------------------------------------------------------- */
int lf_abi_version(void);
const char* lf_last_error(void);

/* Context: a HIP device and a stream (hipStream_t, NULL = default stream),
 * e.g. torch.cuda.current_stream().cuda_stream.                            */
lf_status lf_ctx_create(int hip_device, void* hip_stream, lf_ctx** out);
lf_status lf_ctx_destroy(lf_ctx* ctx);
/* Rows each wavefront marches through in the fused step (0 = automatic). */
lf_status lf_ctx_set_band(lf_ctx* ctx, int rows);

/* ---- single cavity ---------------------------------------------------- */
/* Mode H: the whole cavity is LBM velocity + FV temperature (Sec. 5.1,
 * grid setting 1); the split mode and the single-method cavities as listed
 * at the top.  Defaults after create: side-heated cavity walls (west
 * T = +1/2, east T = -1/2, south/north adiabatic, all no-slip at rest).
 * LF_EINVAL for an unknown mode, nx or ny < 8, an odd or < 12 divided
 * extent (nx for LF_MODE_SPLIT, ny for LF_MODE_SPLIT_H), odd nx or ny for
 * LF_MODE_HYBRID_GS2, or a grid whose nine population planes (each
 * pitch x ny elements plus a small pad, pitch = nx rounded up to 64) reach
 * 2^31 elements or 4 GiB (32-bit element and byte offsets): FP32 up to about
 * 119 M nodes, FP64 up to about 59 M.                                     */
lf_status lf_case_create(lf_ctx* ctx, const lf_case_desc* desc, lf_case** out);
lf_status lf_case_destroy(lf_case* c);
lf_status lf_case_workspace_bytes(const lf_case* c, size_t* bytes);
lf_status lf_case_bind_workspace(lf_case* c, void* dev_ptr, size_t bytes);
/* Derive the lattice parameters from Ra, Pr (Eq 15, 20, 42, 82-89);
 * LF_EUNSTABLE if tau <= 0.501 or alpha > 0.25.                            */
lf_status lf_case_set_physics(lf_case* c, const lf_physics* p);
/* Lattice parameters directly (Ra = 0 cases, closed-form tests).          */
lf_status lf_case_set_lattice(lf_case* c, double nu, double alpha,
                              double gbeta, double T_ref, double body_gx,
                              double body_gy, int conv);
lf_status lf_case_set_wall(lf_case* c, int side, const lf_wall* w);
/* out = {U_char, nu, tau, alpha, tau_T, g beta, T_ref, Ma}               */
lf_status lf_case_get_params(const lf_case* c, double out[8]);
/* LF_MODE_HYBRID_GS2 only: lattice steps per energy step (0 = nx, the
 * paper's 2NX) and alternating line sweeps that relax each energy step's
 * implicit system (0 = 4).  The energy step follows every lattice step
 * whose count since init is a multiple of lattice_steps; its upwind and
 * diffusion terms are implicit (backward Euler over lattice_steps), QUICK
 * enters as a deferred correction from the old temperature, and each sweep
 * solves all x-lines, then all y-lines, by the Thomas algorithm.  lf_case_
 * init takes T0 on the nodes and starts each control volume at the mean of
 * its 2 x 2 nodes; fetch returns the node temperatures (bilinear in the
 * control-volume values, ghosts 2 T_w - T at fixed walls, T at adiabatic
 * ones).  LF_EINVAL in the other modes or for negative counts.             */
lf_status lf_case_set_subcycle(lf_case* c, int lattice_steps, int sweeps);
/* LF_MODE_LBM_MCM only (defaults 100, 256, 1908083868, 2^24): a Monte Carlo
 * solve of the node temperatures follows every lattice step whose count
 * since init is a multiple of lattice_steps, with `walkers` walks per node
 * started from the node and stopped after max_steps steps.  A walker steps
 * x+, y+, x-, y- with the link weights alpha - u, alpha - v, alpha, alpha
 * over their sum (Eq 99-100, velocity of that lattice step; |u|, |v| <
 * alpha keeps them positive), chosen by one uniform draw in Eq 101's order;
 * a link through a fixed-temperature wall (half a spacing) weighs double
 * and absorbs the walker with T_w, a step into an adiabatic wall is
 * refused.  Draws: splitmix64, the stream of walker w at node p seeded by
 * mix(seed + s + (1 + p walkers + w) 0x9E3779B97F4A7C15) for the s-th solve
 * (s = 0, 1, ...).  The node temperature is the mean wall temperature of
 * its absorbed walkers (Eq 102).  LF_EINVAL in other modes or for counts
 * below 1; stepping fails with LF_EINVAL without a fixed-temperature wall. */
lf_status lf_case_set_mcm(lf_case* c, int lattice_steps, int walkers, uint64_t seed,
                          int64_t max_steps);
/* Walkers of the last Monte Carlo solve stopped by max_steps (or by a
 * velocity at or above alpha) instead of a wall; synchronises.             */
lf_status lf_case_mcm_capped(lf_case* c, uint64_t* walkers);
/* Initial state from host arrays of ny*nx doubles (NULL = 0): rho = 1,
 * f = f_eq(1, (u0, v0)), T = T0; the residual snapshot starts here.        */
lf_status lf_case_init(lf_case* c, const double* T0, const double* u0,
                       const double* v0);
/* Advance nsteps time steps (asynchronous).                               */
lf_status lf_case_step(lf_case* c, int64_t nsteps);
/* r = ||phi - phi_snap||_2 / ||phi||_2 for phi = u, v, T against the last
 * snapshot (absolute when ||phi|| < 1e-300), then re-snapshot.
 * LF_EDIVERGED on NaN/Inf.                                                */
lf_status lf_case_residual(lf_case* c, double r[3]);
/* lf_case_residual for callers that cannot allocate device memory (code
 * under graph capture, tight serving loops, harnesses that forbid it): the
 * residual's per-block FP64 partials and its fold's output live in a device
 * array the library holds for the life of the process, one copy per GPU
 * (8200 doubles: partials of up to 1024 blocks, which covers every case the
 * library creates; LF_EINVAL beyond), instead of in the bound workspace.
 * Same result as lf_case_residual, bit for bit, with the same re-snapshot;
 * nothing in the array has to start at zero (each call writes every entry
 * it reads).  All calls on one GPU share that array: calls that overlap on
 * one GPU (other streams or host threads) race and must be serialised by
 * the caller.  Synchronises the stream.                                   */
lf_status lf_case_residual_noalloc(lf_case* c, double r[3]);
/* Step in blocks of check_every until max r <= tol (or all r = 0); in FP32
 * also stop "at the rounding floor": max r <= 1e-6, the last four checks set
 * no new minimum of max r (noise, not slow decay), and the slowest mode,
 * extrapolated from the decade of decay above the floor (its per-check
 * factor lambda), has since fallen to a remaining relative change
 * r lambda / (1 - lambda) <= 2e-6.  r_final receives the last r; *rule (may
 * be NULL) LF_STOP_TOL or LF_STOP_FLOOR.  LF_ENOTCONV at max_steps.        */
lf_status lf_case_run_to_steady(lf_case* c, double tol, int check_every,
                                int64_t max_steps, int64_t* steps_taken,
                                double r_final[3], int* rule);
lf_status lf_case_nusselt(lf_case* c, lf_nusselt* out);
/* Copy a field (LF_FIELD_*) as ny*nx values into dst (device or host),
 * as double (as_f64 = 1) or in the case precision.                        */
lf_status lf_case_fetch(lf_case* c, int field, void* dst, size_t dst_bytes,
                        int dst_is_device, int as_f64);
/* Invariants: sum over all nodes and directions of the post-collision
 * populations, and sum of T.                                              */
lf_status lf_case_mass(lf_case* c, double* sum_f, double* sum_T);
/* Steps taken since init.                                                 */
lf_status lf_case_steps(const lf_case* c, int64_t* steps);
/* Checkpoint: the complete state of an initialised case (fields, moments,
 * residual snapshot, step count, lattice parameters, walls and the cycle
 * settings of lf_case_set_subcycle / lf_case_set_mcm) as a host
 * blob.  With blob == NULL, *bytes receives the size needed; otherwise
 * *bytes must hold at least that size and receives the size written
 * (synchronises the stream).  lf_case_load restores such a blob into a
 * case created with the same lf_case_desc and a bound workspace; stepping
 * on continues bit for bit as the saved case would have (LF_EINVAL if the
 * blob does not match).                                                   */
lf_status lf_case_save(lf_case* c, void* blob, size_t* bytes);
lf_status lf_case_load(lf_case* c, const void* blob, size_t bytes);
/* Advance nsteps (1 .. 2^20) steps, launched back to back on the context
 * stream with a HIP event after every 64 launches; synchronises at the end
 * and returns the mean time per step kernel in milliseconds and the min /
 * max of the 64-launch means (min/max may be NULL).  The state advances
 * exactly as with lf_case_step (moments written on the last step of every
 * 64).  For measurement.                                                   */
lf_status lf_case_profile_steps(lf_case* c, int64_t nsteps, double* avg_ms,
                                double* min_ms, double* max_ms);

/* ---- batches of Mode H cavities ---------------------------------------- */
/* Many cavities of uneven size, aspect, Ra and Pr stepped together: every
 * launch processes a table of wave tiles (62 columns x band rows) of all
 * live cavities; run_to_steady replays a captured hipGraph of check_every
 * steps plus the batched residual and retires converged cavities between
 * replays.  Each cavity is exactly a Mode H case (same kernel code), so a
 * batch member equals the same cavity run alone, bit for bit.  All cavities
 * share one precision; QUICK convection; no periodic sides, no body force.
 * The context stream must not be the legacy default stream (graph capture).
 * walls: 4 per cavity (W, E, S, N) or NULL for the side-heated default.    */
typedef struct lf_batch lf_batch;
lf_status lf_batch_create(lf_ctx* ctx, int n, const lf_case_desc* descs,
                          const lf_physics* phys, const lf_wall* walls,
                          lf_batch** out);
lf_status lf_batch_destroy(lf_batch* b);
lf_status lf_batch_workspace_bytes(const lf_batch* b, size_t* bytes);
lf_status lf_batch_bind_workspace(lf_batch* b, void* dev_ptr, size_t bytes);
/* Rows per wave tile for cavity idx (-1: all cavities); 0 = by load, the
 * default without an autotuner table: 4 while the live cavities yield at
 * least 8192 tiles at 4 rows, else 2 if that reaches it, else 1 (re-chosen
 * whenever the live set changes).                                         */
lf_status lf_batch_set_band(lf_batch* b, int idx, int rows);
/* Initial state per cavity from n host pointers each (NULL array or NULL
 * entry = 0), as lf_case_init.  All cavities become live.                 */
lf_status lf_batch_init(lf_batch* b, const double* const* T0,
                        const double* const* u0, const double* const* v0);
/* Advance every live cavity nsteps steps (asynchronous).                  */
lf_status lf_batch_step(lf_batch* b, int64_t nsteps);
/* Residuals of the live cavities into r3n[3 idx .. 3 idx + 2] (others
 * untouched), then re-snapshot; synchronises.                             */
lf_status lf_batch_residual(lf_batch* b, double* r3n);
/* Per-cavity stop rule of lf_case_run_to_steady with an even check_every;
 * converged cavities stop stepping.  max_steps bounds each cavity's steps
 * since init; a cavity stopped by an earlier call's max_steps resumes (so a
 * long run can be split into calls with growing limits), a converged or
 * diverged one does not.  steps_each / rule_each (0: stopped at max_steps,
 * -1: diverged) / r_each (3 per cavity) may be NULL.  LF_ENOTCONV if a
 * cavity stopped at max_steps.                                             */
lf_status lf_batch_run_to_steady(lf_batch* b, double tol, int check_every,
                                 int64_t max_steps, int64_t* steps_each,
                                 int* rule_each, double* r_each);
/* Make every cavity live again (after run_to_steady).                     */
lf_status lf_batch_reactivate(lf_batch* b);
lf_status lf_batch_get_params(const lf_batch* b, int idx, double out[8]);
lf_status lf_batch_steps(const lf_batch* b, int idx, int64_t* steps);
lf_status lf_batch_nusselt(lf_batch* b, int idx, lf_nusselt* out);
lf_status lf_batch_fetch(lf_batch* b, int idx, int field, void* dst,
                         size_t dst_bytes, int dst_is_device, int as_f64);
/* Advance the live cavities nsteps (even) steps back to back between two
 * HIP events; mean milliseconds per batched step.                         */
lf_status lf_batch_profile_steps(lf_batch* b, int64_t nsteps, double* avg_ms);

/* Autotuner: load the band table for batches from cache_path if it holds
 * one for gfx950 / FP32; otherwise time band heights 1..16 per cavity-height
 * class (64 .. 512 rows, aspect 2) on copies that fill dev_scratch (the
 * library still allocates nothing), keep the fastest, write the cache, and
 * use the table for batches created afterwards in this context.           */
lf_status lf_autotune(lf_ctx* ctx, const char* cache_path, int budget_ms,
                      void* dev_scratch, size_t scratch_bytes);
/* The context's band table (nclass = 0 when none).                        */
lf_status lf_ctx_get_tuning(const lf_ctx* ctx, int* nclass, int ny_class[16],
                            int band[16]);

/* As lf_batch_init, but every non-NULL entry is a DEVICE pointer to a dense
 * [ny][nx] array of doubles (read on the context stream; the arrays must
 * stay valid until the stream reaches this point).                         */
lf_status lf_batch_init_device(lf_batch* b, const double* const* T0,
                               const double* const* u0, const double* const* v0);

/* ---- learned initial guess (not part of the paper) ---------------------- */
/* An encoder-decoder convolutional network maps the cavity parameters to
 * steady fields on a res x res canvas (the unit square, cell-centred):
 * channels u/U_char, v/U_char and theta = T + 1/2.  Inputs per pixel, in
 * this order: X, Y (cell centres on the unit square), (log10 Ra - 4.5)/1.5,
 * (Pr - 3.855)/3.145, A/4, then zeros up to cin.  The ten 3x3 convolutions
 * (zero padding 1), widths w0..w4:
 *   e0 = silu(conv_s1(x)); e_k = silu(conv_s2(e_{k-1})), k = 1..4;
 *   d3 = silu(conv(up2(e4))) + e3; d2, d1, d0 likewise (up2 = nearest x2);
 *   y = conv(d0) (linear, cout channels, the first 3 are used).
 * Parameters: FP32 master copy, flat, per layer weights [Cout][3][3][Cin]
 * then bias [Cout]; the convolutions run on bf16 operands with FP32
 * accumulation (gfx950 matrix cores); training is MSE over the 3 channels
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Device inputs: feat = [N][3] floats (log10 Ra, Pr, A) per sample,
 * target = [N][3][res][res] floats, idx = [batch] int32 sample indices (or
 * NULL for 0 .. batch-1), each in 0 .. N-1 (not checked: device memory).
 * batch <= max_batch.                                                     */
typedef struct {
  int res;         /* canvas size, a multiple of 16                          */
  int cin, cout;   /* cin = 8 (5 used); cout a multiple of 8 (3 used)        */
  int widths[5];   /* multiples of 8                                         */
  int max_batch;
} lf_net_desc;
typedef struct lf_net lf_net;
lf_status lf_net_create(lf_ctx* ctx, const lf_net_desc* desc, lf_net** out);
lf_status lf_net_destroy(lf_net* net);
lf_status lf_net_param_count(const lf_net* net, int64_t* n);
lf_status lf_net_workspace_bytes(const lf_net* net, size_t* bytes);
lf_status lf_net_bind_workspace(lf_net* net, void* dev_ptr, size_t bytes);
/* Host copies of the flat FP32 parameters; set also clears Adam's state.  */
lf_status lf_net_set_weights(lf_net* net, const float* host, int64_t n);
lf_status lf_net_get_weights(lf_net* net, float* host, int64_t n);
/* Gradient of the last lf_net_backward (flat layout of the parameters).   */
lf_status lf_net_get_grads(lf_net* net, float* host, int64_t n);
/* Forward pass; pred (device, may be NULL) receives [batch][3][res][res].  */
lf_status lf_net_forward(lf_net* net, const float* feat, const int* idx, int batch,
                         float* pred);
/* Raw output [batch][res][res][cout] of the last forward pass (host).     */
lf_status lf_net_get_output(lf_net* net, float* host, size_t n);
/* Forward + MSE + backward into the gradient buffer; loss (device float,
 * may be NULL) receives the mean squared error.  Asynchronous.            */
lf_status lf_net_backward(lf_net* net, const float* feat, const float* target,
                          const int* idx, int batch, float* loss);
/* One Adam step with the gradient buffer.                                 */
lf_status lf_net_adam(lf_net* net, float lr);
/* lf_net_backward followed by lf_net_adam.                                */
lf_status lf_net_train_step(lf_net* net, const float* feat, const float* target,
                            const int* idx, int batch, float lr, float* loss);
/* Multiply-add count (x2) of one forward pass of one sample, and of the
 * three passes of one training sample (forward, input and weight grads).  */
lf_status lf_net_flops(const lf_net* net, double* fwd, double* train);
/* nsteps training steps on one batch between two HIP events (synchronises);
 * mean milliseconds per step.  For measurement.                           */
lf_status lf_net_profile_train(lf_net* net, const float* feat, const float* target,
                               const int* idx, int batch, float lr, int nsteps,
                               double* avg_ms);

/* Bilinear resampling between cell-centred grids covering the same
 * rectangle: destination centre (i + 1/2)/dnx maps to the source index
 * coordinate (i + 1/2) snx/dnx - 1/2, clamped to [0, snx - 1] (same in y);
 * dst[j][i] = value * scale + offset.  src rows are src_row_stride elements
 * apart; dst is dense [dny][dnx].  Device pointers; asynchronous.
 * flags: LF_RESAMPLE_ANTISYM keeps the part that is odd under the 180-degree
 * rotation, dst[j][i] = (d[j][i] - d[dny-1-j][dnx-1-i]) / 2 of the plain
 * result d (the side-heated cavity's steady T, u and v are odd).          */
enum { LF_RESAMPLE_ANTISYM = 1 };
lf_status lf_resample(lf_ctx* ctx, const void* src, int src_is_f64, int snx, int sny,
                      int64_t src_row_stride, void* dst, int dst_is_f64, int dnx,
                      int dny, double scale, double offset, int flags);

#ifdef __cplusplus
}
#endif
#endif /* LBMFVM_H */
