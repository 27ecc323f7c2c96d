// lbmfvm_api.cpp -- host runtime behind the C ABI of include/lbmfvm.h.
//
// Owns no device memory: every case lays its state out inside the workspace
// the caller binds.  All device work goes to the context's stream.
#include <math.h>
#include <stdio.h>
#include <stdarg.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbmfvm.h"
#include "lf_host.h"
#include "lf_internal.h"

namespace {
thread_local char g_err[512] = "";
}  // namespace

lf_status lf_fail(lf_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

#define fail lf_fail
#define HIP_TRY LF_HIP_TRY
#define align_up lf_align_up

struct lf_case {
  lf_ctx* ctx;
  lf_case_desc desc;
  size_t es;  // bytes per element
  lf::Grid g;
  lf::WallSet w;
  lf::HybridParams p;
  double params[8];
  bool have_params;
  char* ws;
  size_t ws_bytes;
  size_t off_f[2], off_T[2], off_mom, off_snap, off_part, off_out, off_stage, need;
  size_t off_Tlo[2];  // compensated-temperature low words (0 if unused)
  bool tcomp;
  int nblk;  // blocks of the reduction passes
  int cur;   // buffer holding the current state
  int64_t steps;
  bool inited;
  // domain-decomposed mode
  bool split;
  lf::SplitGeom sg;
  lf::SplitParams sp;
  size_t off_sf[2], off_sg[2], off_smom, off_sxf, off_su[2], off_sv[2], off_sT[2], off_sp[2],
      off_siface, off_dense, off_dsnap;
  // grid setting 2: the coarse planes, lattice steps per energy step and
  // line sweeps per energy step
  size_t off_gs2[10];
  int gs2_S, gs2_K;
  // LBM-MCM: walker counts per node and wall, the cap total; lattice steps
  // per Monte Carlo solve, walkers per node, stream seed, step cap
  size_t off_mcm_count, off_mcm_stats, off_mcm_cth;
  int mcm_S, mcm_N;
  unsigned long long mcm_seed;
  long long mcm_max;
  // captured runs of kGraphSteps steps starting from buffer set 0 / 1, and
  // the signature of the settings they were captured with
  hipGraphExec_t gexec[2];
  uint64_t gsig[2];
};

static void drop_graphs(lf_case* c);

template <typename real>
static real* fptr(lf_case* c, size_t off) { return (real*)(c->ws + off); }

// Domain-decomposed layout: LBM zone (f, g ping-pong, moments, x_f rows),
// FV zone (u, v, T ping-pong, p), interface scalars, dense output and
// snapshot planes for residual / Nusselt / fetch.
static void layout_split(lf_case* c) {
  const lf::SplitGeom& G = c->sg;
  const size_t pbL = align_up((size_t)G.planeL * c->es, 256);
  const size_t pbF = align_up((size_t)G.pF * (G.ny + 1) * c->es, 256);
  const size_t n = (size_t)G.nx * G.ny;
  const size_t pbD = align_up(n * c->es, 256);
  size_t o = 0;
  for (int k = 0; k < 2; ++k) { c->off_sf[k] = o; o += 9 * pbL; }
  for (int k = 0; k < 2; ++k) { c->off_sg[k] = o; o += 5 * pbL; }
  c->off_smom = o; o += 4 * pbL;
  c->off_sxf = o; o += align_up((size_t)18 * G.ny * c->es, 256);
  for (int k = 0; k < 2; ++k) { c->off_su[k] = o; o += pbF; }
  for (int k = 0; k < 2; ++k) { c->off_sv[k] = o; o += pbF; }
  for (int k = 0; k < 2; ++k) { c->off_sT[k] = o; o += pbF; }
  c->off_sp[0] = o; o += pbF;
  c->off_sp[1] = o; o += pbF;
  // interface scalars, then per unit of rows two ghost sums of each parity
  // and two p_bar sums
  c->off_siface = o;
  o += align_up((size_t)lf::split_iface_doubles(G.ny) * sizeof(double), 256);
  for (int k = 0; k < 10; ++k) {
    c->off_gs2[k] = o;
    if (G.gs2) o += align_up((size_t)G.pC * G.NYc * c->es, 256);
  }
  c->off_mcm_count = o;
  if (G.mcm) o += align_up((size_t)5 * G.nx * G.ny * sizeof(int), 256);
  c->off_mcm_stats = o;
  if (G.mcm) o += 256;
  c->off_mcm_cth = o;
  if (G.mcm) o += align_up((size_t)4 * G.nx * G.ny * sizeof(double), 256);
  c->off_dense = o; o += 4 * pbD;
  c->off_dsnap = o; o += 3 * pbD;
  c->off_part = o; o += align_up((size_t)c->nblk * 8 * sizeof(double), 256);
  c->off_out = o; o += 256 * sizeof(double);
  c->off_stage = o; o += align_up((size_t)3 * n * sizeof(double), 256);
  c->need = o;
}

template <typename real>
static lf::SplitPtrs<real> split_ptrs(lf_case* c) {
  lf::SplitPtrs<real> P;
  const lf::SplitGeom& G = c->sg;
  const size_t pbL = align_up((size_t)G.planeL * c->es, 256);
  for (int k = 0; k < 2; ++k) {
    P.f[k] = (real*)(c->ws + c->off_sf[k]);
    P.g[k] = (real*)(c->ws + c->off_sg[k]);
    P.u[k] = (real*)(c->ws + c->off_su[k]);
    P.v[k] = (real*)(c->ws + c->off_sv[k]);
    P.T[k] = (real*)(c->ws + c->off_sT[k]);
  }
  (void)pbL;
  P.mom = (real*)(c->ws + c->off_smom);
  P.xf = (real*)(c->ws + c->off_sxf);
  P.p[0] = (real*)(c->ws + c->off_sp[0]);
  P.p[1] = (real*)(c->ws + c->off_sp[1]);
  P.iface = (double*)(c->ws + c->off_siface);
  for (int k = 0; k < 10; ++k) P.gc[k] = (real*)(c->ws + c->off_gs2[k]);
  P.mcm_count = (int*)(c->ws + c->off_mcm_count);
  P.mcm_stats = (unsigned long long*)(c->ws + c->off_mcm_stats);
  P.mcm_cth = (double*)(c->ws + c->off_mcm_cth);
  return P;
}

// dense [ny][nx] planes used by the reductions in the split mode
static lf::Grid dense_grid(const lf_case* c) {
  lf::Grid g;  // the caller's orientation
  g.nx = c->g.nx;
  g.ny = c->g.ny;
  g.pitch = c->g.nx;
  g.plane = (long long)c->g.nx * c->g.ny;
  return g;
}

template <typename real>
static lf_status split_init(lf_case* c, const double* dT) {
  hipStream_t s = c->ctx->stream;
  const lf::SplitPtrs<real> P = split_ptrs<real>(c);
  if (c->sg.gs2)
    HIP_TRY(lf::launch_gs2_init<real>(c->sg, P, c->sp, dT, s));
  else
    HIP_TRY(lf::launch_split_init<real>(c->sg, P, c->sp, dT, s));
  if (c->sg.mcm) HIP_TRY(hipMemsetAsync(c->ws + c->off_mcm_stats, 0, 8, s));
  real* dense = (real*)(c->ws + c->off_dense);
  HIP_TRY(lf::launch_split_output<real>(c->sg, P, c->sp, 0, dense, s));
  const size_t n = (size_t)c->sg.nx * c->sg.ny;
  // residual snapshot: the u, v, T planes (contiguous after rho)
  HIP_TRY(hipMemcpyAsync(c->ws + c->off_dsnap, dense + n, 3 * n * sizeof(real),
                         hipMemcpyDeviceToDevice, s));
  return LF_OK;
}

// n steps; the last writes every node's moments when mom_last is set
template <typename real>
static lf_status split_steps(lf_case* c, int64_t n, bool mom_last = true) {
  hipStream_t s = c->ctx->stream;
  const lf::SplitPtrs<real> P = split_ptrs<real>(c);
  if (c->sg.gs2 || c->sg.mcm) {
    // lattice steps; after every S-th (counted since init) one energy step
    // (implicit FV on the coarse grid, or a Monte Carlo solve whose stream
    // seed advances with the solve's index), which reads the moments of
    // that lattice step
    const int S = c->sg.gs2 ? c->gs2_S : c->mcm_S;
    if (c->sg.mcm && !(c->sp.tfix[0] || c->sp.tfix[1] || c->sp.tfix[2] || c->sp.tfix[3]))
      return fail(LF_EINVAL, "the Monte Carlo solve needs a wall with a fixed temperature");
    for (int64_t k = 0; k < n; ++k) {
      const int64_t done = c->steps + k + 1;
      const bool energy = done % S == 0;
      HIP_TRY(lf::launch_gs2_lbm<real>(c->sg, P, c->sp, c->cur, (energy || k == n - 1) ? 1 : 0, s));
      c->cur ^= 1;
      if (!energy) continue;
      if (c->sg.gs2)
        HIP_TRY(lf::launch_gs2_energy<real>(c->sg, P, c->sp, c->gs2_S, c->gs2_K, s));
      else
        HIP_TRY(lf::launch_mcm_energy<real>(c->sg, P, c->sp, c->mcm_N,
                                            c->mcm_seed + (unsigned long long)(done / S - 1),
                                            c->mcm_max, s));
    }
    c->steps += n;
    return LF_OK;
  }
  for (int64_t k = 0; k < n; ++k) {
    HIP_TRY(lf::launch_split_step<real>(c->sg, P, c->sp, c->cur,
                                        (mom_last && k == n - 1) ? 1 : 0, s));
    c->cur ^= 1;
  }
  c->steps += n;
  return LF_OK;
}

// dense rho, u, v, T planes of the current split-mode state
template <typename real>
static lf_status split_dense(lf_case* c) {
  const lf::SplitPtrs<real> P = split_ptrs<real>(c);
  HIP_TRY(lf::launch_split_output<real>(c->sg, P, c->sp, c->cur, (real*)(c->ws + c->off_dense),
                                        c->ctx->stream));
  return LF_OK;
}

extern "C" {

int lf_abi_version(void) { return LF_ABI_VERSION; }
const char* lf_last_error(void) { return g_err; }

}  // extern "C"

// Scratch of lf_case_residual_noalloc: the residual's per-block FP64
// partials (8 doubles per block, at most kNoallocBlocks blocks) followed by
// the fold's 8 outputs, in a device array the process holds instead of the
// case workspace's partials area.  Each GPU has its own copy at its own
// address, looked up once per device when a context is created on it; host
// code uses only that address (the array's name is a host-side stand-in).
namespace {
constexpr int kNoallocBlocks = 1024;
constexpr int kNoallocDoubles = kNoallocBlocks * 8 + 8;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];
}  // namespace
static __device__ __align__(256) double scratch[kNoallocDoubles];

// with `dev` current
static lf_status scratch_lookup(int dev) {
  if (dev >= kMaxDevices) return fail(LF_EINVAL, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return LF_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(LF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                hipGetErrorString(e));
  g_scratch_ptr[dev] = (double*)p;
  return LF_OK;
}

extern "C" {

lf_status lf_ctx_create(int hip_device, void* hip_stream, lf_ctx** out) {
  if (!out) return fail(LF_EINVAL, "out is NULL");
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n)
    return fail(LF_EINVAL, "device %d out of range (%d devices)", hip_device, n);
  HIP_TRY(hipSetDevice(hip_device));
  const lf_status ss = scratch_lookup(hip_device);
  if (ss != LF_OK) return ss;
  lf_ctx* c = new (std::nothrow) lf_ctx;
  if (!c) return fail(LF_ENOMEM, "ctx allocation");
  memset(c, 0, sizeof(*c));
  c->device = hip_device;
  c->stream = (hipStream_t)hip_stream;
  c->band = 0;
  *out = c;
  return LF_OK;
}

lf_status lf_ctx_destroy(lf_ctx* ctx) {
  delete ctx;
  return LF_OK;
}

lf_status lf_ctx_set_band(lf_ctx* ctx, int rows) {
  if (!ctx || rows < 0 || rows > 4096) return fail(LF_EINVAL, "band must be in [0, 4096]");
  ctx->band = rows;
  return LF_OK;
}

static void layout(lf_case* c) {
  const lf::Grid& g = c->g;
  const size_t pb = align_up((size_t)g.plane * c->es, 256);
  size_t o = 0;
  c->off_f[0] = o; o += 9 * pb;
  c->off_f[1] = o; o += 9 * pb;
  c->off_T[0] = o; o += pb;
  c->off_T[1] = o; o += pb;
  c->off_mom = o; o += 3 * pb;
  c->off_snap = o; o += 3 * pb;
  c->off_Tlo[0] = c->off_Tlo[1] = 0;
  if (c->tcomp) {  // one byte per node and plane
    const size_t pl = align_up((size_t)g.plane, 256);
    c->off_Tlo[0] = o; o += pl;
    c->off_Tlo[1] = o; o += pl;
  }
  c->off_part = o; o += align_up((size_t)c->nblk * 8 * sizeof(double), 256);
  c->off_out = o; o += 256 * sizeof(double);
  c->off_stage = o; o += align_up((size_t)3 * g.nx * g.ny * sizeof(double), 256);
  c->need = o;
}

lf_status lf_case_create(lf_ctx* ctx, const lf_case_desc* d, lf_case** out) {
  if (!ctx || !d || !out) return fail(LF_EINVAL, "NULL argument");
  if (d->nx < 8 || d->ny < 8) return fail(LF_EINVAL, "nx, ny must be >= 8 (got %d, %d)", d->nx, d->ny);
  if (d->precision != LF_F32 && d->precision != LF_F64)
    return fail(LF_EINVAL, "precision must be LF_F32 or LF_F64");
  if (d->mode != LF_MODE_HYBRID && d->mode != LF_MODE_SPLIT && d->mode != LF_MODE_PURE_FV &&
      d->mode != LF_MODE_PURE_LBM && d->mode != LF_MODE_HYBRID_GS2 && d->mode != LF_MODE_SPLIT_H &&
      d->mode != LF_MODE_LBM_MCM)
    return fail(LF_EINVAL, "mode %d unknown", d->mode);
  if (d->mode == LF_MODE_HYBRID_GS2 && (d->nx % 2 || d->ny % 2))
    return fail(LF_EINVAL, "grid setting 2 needs even nx, ny (got %d, %d)", d->nx, d->ny);
  if (d->mode == LF_MODE_SPLIT || d->mode == LF_MODE_SPLIT_H) {
    // the divided extent: nx (vertical division) or ny (horizontal)
    const int ext = d->mode == LF_MODE_SPLIT ? d->nx : d->ny;
    if (ext % 2 || ext < 12)
      return fail(LF_EINVAL, "the divided extent must be even and >= 12 (got %d)", ext);
    if (d->split_col != 0 && d->split_col != ext / 2)
      return fail(LF_ENOTIMPL, "split_col must be half the divided extent (0 selects it)");
    if (d->overlap != 0 && d->overlap != 3) return fail(LF_ENOTIMPL, "overlap must be 3");
    if (d->iface != LF_IFACE_NEQ_EXTRAP && d->iface != LF_IFACE_FD_GRADIENT)
      return fail(LF_EINVAL, "bad iface %d", d->iface);
  }
  const long long pitch = (d->nx + 63) / 64 * 64;
  const long long plane = lf_plane_elems(pitch, d->ny);
  if (!lf_planes_fit(plane, d->precision == LF_F64 ? 8 : 4))
    return fail(LF_EINVAL, "grid too large: nine planes must stay under 4 GiB and 2^31 elements");
  lf_case* c = new (std::nothrow) lf_case;
  if (!c) return fail(LF_ENOMEM, "case allocation");
  memset(c, 0, sizeof(*c));
  c->ctx = ctx;
  c->desc = *d;
  c->es = d->precision == LF_F64 ? 8 : 4;
  c->g.nx = d->nx;
  c->g.ny = d->ny;
  c->g.pitch = (int)pitch;
  c->g.plane = plane;
  c->nblk = d->ny < 1024 ? d->ny : 1024;
  // default: side-heated cavity
  c->w.xper = c->w.yper = 0;
  c->w.tfix[LF_SIDE_W] = 1; c->w.Tw[LF_SIDE_W] = 0.5;
  c->w.tfix[LF_SIDE_E] = 1; c->w.Tw[LF_SIDE_E] = -0.5;
  c->p.omega = 1.0;
  if (d->mode != LF_MODE_HYBRID) {
    c->split = true;
    lf::SplitGeom& G = c->sg;
    // the horizontally divided cavity is stored transposed, gravity along -x
    G.transposed = G.gdir = d->mode == LF_MODE_SPLIT_H;
    G.nx = G.transposed ? d->ny : d->nx;
    G.ny = G.transposed ? d->nx : d->ny;
    G.fv_only = d->mode == LF_MODE_PURE_FV;
    G.lbm_only = d->mode == LF_MODE_PURE_LBM;
    G.gs2 = d->mode == LF_MODE_HYBRID_GS2;
    G.mcm = d->mode == LF_MODE_LBM_MCM;
    if (G.mcm) {  // lattice and Monte Carlo temperatures on all nodes
      G.s = G.ib = G.nx;
      G.c0 = G.nx + 2;
      G.pL = (G.nx + 63) / 64 * 64;
      G.pF = 0;
      c->mcm_S = 100;
      c->mcm_N = 256;
      c->mcm_seed = 1908083868ull;
      c->mcm_max = 1ll << 24;
    } else if (G.gs2) {  // lattice on all nodes, temperature on 2 x 2 blocks
      G.s = G.ib = G.nx;
      G.c0 = G.nx + 2;
      G.pL = (G.nx + 63) / 64 * 64;
      G.pF = 0;
      G.NXc = G.nx / 2;
      G.NYc = G.ny / 2;
      G.pC = (G.NXc + 63) / 64 * 64;
      c->gs2_S = G.nx;  // 2NX lattice steps per energy step
      c->gs2_K = 4;
    } else if (G.fv_only) {  // FV cells 0 .. nx-1, wall faces 0 and nx
      G.s = G.c0 = G.ib = 0;
      G.pL = 0;
      G.pF = (G.nx + 3 + 63) / 64 * 64;
    } else if (G.lbm_only) {  // LBM nodes 0 .. nx-1
      G.s = G.ib = G.nx;
      G.c0 = G.nx + 2;  // no FV cell
      G.pL = (G.nx + 63) / 64 * 64;
      G.pF = 0;
    } else {
      G.s = G.nx / 2;
      G.c0 = G.s - 1;
      G.ib = G.s + 1;
      G.pL = (G.ib + 1 + 63) / 64 * 64;
      G.pF = (G.nx - G.c0 + 3 + 63) / 64 * 64;
    }
    // the LBM zone's planes are spaced like Mode H's (lf_plane_elems): pure
    // LBM at 4096^2 0.366 -> 0.356 ms per step, grid setting 2 0.252 -> 0.233
    G.planeL = (int)lf_plane_elems(G.pL, G.ny);
    c->sp.kind = d->iface;
    c->sp.tau = c->sp.tauT = 1.0;
    // stored sides of the caller's hot west and cold east walls
    const int sw = G.transposed ? LF_SIDE_S : LF_SIDE_W, se = G.transposed ? LF_SIDE_N : LF_SIDE_E;
    c->sp.tfix[sw] = 1; c->sp.Tw[sw] = 0.5;
    c->sp.tfix[se] = 1; c->sp.Tw[se] = -0.5;
    layout_split(c);
  } else {
    c->tcomp = d->precision == LF_F32 && d->tcomp;
    layout(c);
  }
  *out = c;
  return LF_OK;
}

lf_status lf_case_destroy(lf_case* c) {
  if (c) drop_graphs(c);
  delete c;
  return LF_OK;
}

lf_status lf_case_workspace_bytes(const lf_case* c, size_t* bytes) {
  if (!c || !bytes) return fail(LF_EINVAL, "NULL argument");
  *bytes = c->need;
  return LF_OK;
}

lf_status lf_case_bind_workspace(lf_case* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return fail(LF_EINVAL, "NULL argument");
  if (bytes < c->need) return fail(LF_EWORKSPACE, "workspace %zu bytes < %zu needed", bytes, c->need);
  if ((uintptr_t)dev_ptr % 256) return fail(LF_EWORKSPACE, "workspace must be 256-byte aligned");
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  c->inited = false;
  return LF_OK;
}

static lf_status check_stable(double tau, double alpha) {
  if (!(tau > 0.501)) return fail(LF_EUNSTABLE, "tau = %.6g must exceed 0.501", tau);
  if (!(alpha >= 0.0 && alpha <= 0.25))
    return fail(LF_EUNSTABLE, "alpha = %.6g outside [0, 0.25] (explicit 2-D diffusion limit)", alpha);
  return LF_OK;
}

static lf_status apply_lattice(lf_case* c, double nu, double alpha, double gbeta, double T_ref,
                               double gx, double gy, int conv) {
  if (conv < LF_CONV_QUICK || conv > LF_CONV_UPWIND) return fail(LF_EINVAL, "bad conv %d", conv);
  if (!(nu > 0.0)) return fail(LF_EINVAL, "nu must be > 0");
  const double tau = 3.0 * nu + 0.5;  // Eq 15 with c_s^2 = 1/3, Eq 42
  lf_status st = check_stable(tau, alpha);
  if (st != LF_OK) return st;
  if (c->split && !c->sg.lbm_only && !c->sg.gs2 && !c->sg.mcm && nu > 1.0 / 12.0)
    return fail(LF_EUNSTABLE, "nu = %.6g: the explicit artificial-compressibility FV zone is "
                "linearly stable only for nu <= 1/12", nu);
  if (c->split && (gx != 0.0 || gy != 0.0))
    return fail(LF_ENOTIMPL, "body forces are not available in the split mode");
  c->sp.tau = tau;
  c->sp.tauT = 3.0 * alpha + 0.5;
  c->sp.nu = nu;
  c->sp.alpha = alpha;
  c->sp.gbeta = gbeta;
  c->sp.T_ref = T_ref;
  c->sp.conv = conv;
  if (c->split && !(c->sp.tauT > 0.501))
    return fail(LF_EUNSTABLE, "tau_T = %.6g must exceed 0.501", c->sp.tauT);
  c->p.omega = 1.0 / tau;
  c->p.alpha = alpha;
  c->p.gbeta = gbeta;
  c->p.T_ref = T_ref;
  c->p.gx = gx;
  c->p.gy = gy;
  c->p.conv = conv;
  return LF_OK;
}

lf_status lf_case_set_lattice(lf_case* c, double nu, double alpha, double gbeta, double T_ref,
                              double gx, double gy, int conv) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  lf_status st = apply_lattice(c, nu, alpha, gbeta, T_ref, gx, gy, conv);
  if (st != LF_OK) return st;
  c->params[0] = 0.0;
  c->params[1] = nu;
  c->params[2] = 3.0 * nu + 0.5;
  c->params[3] = alpha;
  c->params[4] = 3.0 * alpha + 0.5;
  c->params[5] = gbeta;
  c->params[6] = T_ref;
  c->params[7] = 0.0;
  c->have_params = true;
  return LF_OK;
}

}  // extern "C"

// Lattice parameters from the physical groups (Eq 15, 20, 42, 82-89), shared
// by single cavities and batches.  out = {U_char, nu, tau, alpha, tau_T,
// g beta, T_ref, Ma}.
lf_status lf_derive_params(const lf_physics* ph, int ny, int split, double out[8]) {
  if (!(ph->Ra > 0.0) || !(ph->Pr > 0.0)) return fail(LF_EINVAL, "Ra and Pr must be > 0");
  const double H = (double)ny;
  double U = ph->U_char;
  if (!(U > 0.0)) {
    // buoyancy velocity sqrt(g beta dT H) in lattice units: 0.1 unless the
    // explicit updates need less (alpha <= 0.2, U^2 <= 2 alpha; split mode
    // also nu <= 0.08)
    U = 0.1;
    const double ua = 0.2 * sqrt(ph->Ra * ph->Pr) / H;
    if (ua < U) U = ua;
    if (split) {
      // the artificial-compressibility FV zone needs nu <= 1/12
      const double un = 0.08 * sqrt(ph->Ra / ph->Pr) / H;
      if (un < U) U = un;
    }
    const double ud = 2.0 * H / sqrt(ph->Ra * ph->Pr);
    if (ud < U) U = ud;
  }
  // Eq 87-89 in lattice units: nu = U H sqrt(Pr/Ra), alpha = nu / Pr,
  // g beta dT = U^2 / H with dT = 1
  const double nu = U * H * sqrt(ph->Pr / ph->Ra);
  const double alpha = nu / ph->Pr;
  out[0] = U;
  out[1] = nu;
  out[2] = 3.0 * nu + 0.5;
  out[3] = alpha;
  out[4] = 3.0 * alpha + 0.5;
  out[5] = U * U / H;
  out[6] = isnan(ph->T_ref) ? 0.0 : ph->T_ref;
  out[7] = U * sqrt(3.0);  // Ma = U / c_s (Eq 84)
  return LF_OK;
}

extern "C" {

lf_status lf_case_set_physics(lf_case* c, const lf_physics* ph) {
  if (!c || !ph) return fail(LF_EINVAL, "NULL argument");
  double prm[8];
  lf_status st = lf_derive_params(ph, c->g.ny, c->split && !c->sg.gs2 && !c->sg.mcm, prm);
  if (st != LF_OK) return st;
  st = apply_lattice(c, prm[1], prm[3], prm[5], prm[6], ph->body_gx, ph->body_gy, ph->conv);
  if (st != LF_OK) return st;
  memcpy(c->params, prm, sizeof(prm));
  c->have_params = true;
  return LF_OK;
}

lf_status lf_case_set_wall(lf_case* c, int side, const lf_wall* w) {
  if (!c || !w) return fail(LF_EINVAL, "NULL argument");
  if (side < LF_SIDE_W || side > LF_SIDE_N) return fail(LF_EINVAL, "bad side %d", side);
  const bool per = w->vel == LF_WALL_PERIODIC;
  if (w->vel != LF_WALL_NOSLIP && !per) return fail(LF_EINVAL, "bad vel %d", w->vel);
  if (per != (w->thermal == LF_T_PERIODIC))
    return fail(LF_EINVAL, "periodic velocity and periodic temperature go together");
  if (!per && w->thermal != LF_T_DIRICHLET && w->thermal != LF_T_ADIABATIC)
    return fail(LF_EINVAL, "bad thermal %d", w->thermal);
  if (c->split) {
    if (per) return fail(LF_ENOTIMPL, "periodic sides are not available in the split mode");
    // a sliding lid (Sec. 3.3): the north wall of the split, FV-only and
    // LBM-only cavities as stored untransposed
    if (w->u_wall != 0.0 &&
        (side != LF_SIDE_N || c->sg.transposed || c->sg.gs2 || c->sg.mcm))
      return fail(LF_ENOTIMPL,
                  "in the split-family modes only the north wall of LF_MODE_SPLIT, "
                  "LF_MODE_PURE_FV and LF_MODE_PURE_LBM may move");
    if (side == LF_SIDE_N && !c->sg.transposed) c->sp.ulid = w->u_wall;
    // stored side (transposed storage: W, E, S, N -> S, N, W, E)
    static const int tmap[4] = {LF_SIDE_S, LF_SIDE_N, LF_SIDE_W, LF_SIDE_E};
    const int ss = c->sg.transposed ? tmap[side] : side;
    c->sp.tfix[ss] = w->thermal == LF_T_DIRICHLET;
    c->sp.Tw[ss] = w->T_wall;
  }
  const int other = side ^ 1;  // W<->E, S<->N
  const bool axis_per = side < 2 ? c->w.xper : c->w.yper;
  // periodicity is a property of the axis: it is switched on/off for both sides
  if (per) {
    if (side < 2) c->w.xper = 1; else c->w.yper = 1;
    c->w.uw[side] = c->w.uw[other] = 0.0;
    c->w.tfix[side] = c->w.tfix[other] = 0;
  } else {
    if (axis_per) {
      if (side < 2) c->w.xper = 0; else c->w.yper = 0;
    }
    c->w.uw[side] = w->u_wall;
    c->w.tfix[side] = w->thermal == LF_T_DIRICHLET;
    c->w.Tw[side] = w->T_wall;
  }
  return LF_OK;
}

lf_status lf_case_set_subcycle(lf_case* c, int lattice_steps, int sweeps) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  if (!c->split || !c->sg.gs2) return fail(LF_EINVAL, "set_subcycle applies to LF_MODE_HYBRID_GS2");
  if (lattice_steps < 0 || sweeps < 0 || sweeps > 4096)
    return fail(LF_EINVAL, "lattice_steps >= 0 and 0 <= sweeps <= 4096 (0: default)");
  c->gs2_S = lattice_steps > 0 ? lattice_steps : c->sg.nx;
  c->gs2_K = sweeps > 0 ? sweeps : 4;
  return LF_OK;
}

lf_status lf_case_set_mcm(lf_case* c, int lattice_steps, int walkers, uint64_t seed,
                          int64_t max_steps) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  if (!c->split || !c->sg.mcm) return fail(LF_EINVAL, "set_mcm applies to LF_MODE_LBM_MCM");
  if (lattice_steps < 1 || walkers < 1 || max_steps < 1)
    return fail(LF_EINVAL, "lattice_steps, walkers and max_steps must be >= 1");
  if ((long long)walkers * c->sg.nx * c->sg.ny > (1ll << 40))
    return fail(LF_EINVAL, "walkers x nodes above 2^40");
  c->mcm_S = lattice_steps;
  c->mcm_N = walkers;
  c->mcm_seed = (unsigned long long)seed;
  c->mcm_max = (long long)max_steps;
  return LF_OK;
}

lf_status lf_case_mcm_capped(lf_case* c, uint64_t* walkers) {
  if (!c || !walkers) return fail(LF_EINVAL, "NULL argument");
  if (!c->split || !c->sg.mcm) return fail(LF_EINVAL, "mcm_capped applies to LF_MODE_LBM_MCM");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, c->ws + c->off_mcm_stats, sizeof(h), hipMemcpyDeviceToHost,
                         c->ctx->stream));
  HIP_TRY(hipStreamSynchronize(c->ctx->stream));
  *walkers = (uint64_t)h;
  return LF_OK;
}

lf_status lf_case_get_params(const lf_case* c, double out[8]) {
  if (!c || !out) return fail(LF_EINVAL, "NULL argument");
  if (!c->have_params) return fail(LF_ESTATE, "no parameters set");
  memcpy(out, c->params, sizeof(c->params));
  return LF_OK;
}

lf_status lf_case_init(lf_case* c, const double* T0, const double* u0, const double* v0) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  if (!c->ws) return fail(LF_EWORKSPACE, "no workspace bound");
  hipStream_t s = c->ctx->stream;
  const size_t n = (size_t)c->g.nx * c->g.ny;
  double* st = (double*)(c->ws + c->off_stage);
  const double* dT = nullptr; const double* du = nullptr; const double* dv = nullptr;
  if (T0) { HIP_TRY(hipMemcpyAsync(st, T0, n * 8, hipMemcpyHostToDevice, s)); dT = st; }
  if (u0) { HIP_TRY(hipMemcpyAsync(st + n, u0, n * 8, hipMemcpyHostToDevice, s)); du = st + n; }
  if (v0) { HIP_TRY(hipMemcpyAsync(st + 2 * n, v0, n * 8, hipMemcpyHostToDevice, s)); dv = st + 2 * n; }
  c->cur = 0;
  if (c->split) {
    if (u0 || v0) return fail(LF_ENOTIMPL, "the split mode starts from rest (u0 = v0 = NULL)");
    lf_status st = c->desc.precision == LF_F32 ? split_init<float>(c, dT) : split_init<double>(c, dT);
    if (st != LF_OK) return st;
  } else if (c->desc.precision == LF_F32) {
    HIP_TRY(lf::launch_init<float>(c->g, dT, du, dv, fptr<float>(c, c->off_f[0]),
                                   fptr<float>(c, c->off_T[0]), fptr<float>(c, c->off_mom),
                                   fptr<float>(c, c->off_snap),
                                   c->tcomp ? (lf::tlo_t*)(c->ws + c->off_Tlo[0]) : nullptr, s));
  } else {
    HIP_TRY(lf::launch_init<double>(c->g, dT, du, dv, fptr<double>(c, c->off_f[0]),
                                    fptr<double>(c, c->off_T[0]), fptr<double>(c, c->off_mom),
                                    fptr<double>(c, c->off_snap), nullptr, s));
  }
  // the host arrays may be freed on return: wait for the uploads
  HIP_TRY(hipStreamSynchronize(s));
  c->steps = 0;
  c->inited = true;
  return LF_OK;
}

static int auto_band(const lf_case* c) {
  if (c->ctx->band > 0) return c->ctx->band;
  // Rows per wave: single rows run the step kernel's 5-wave form (nothing
  // held ahead) and keep the most waves in flight; bands of 4 rows re-pull
  // fewer halo rows.  Measured on MI355X (us per step, band 1 / 2 / 4):
  // 768^2 11.4 / 13.0 / -, 1024^2 17.0 / 19.5 / -, 1536^2 38.8 / 38.2 / 37.3,
  // 2048^2 100.3 / 88.7 / 86.7, 4096^2 - / 359 / 327 (8 rows: 334).
  return lf_rows_per_wave((long long)((c->g.nx + 61) / 62) * c->g.ny);
}

}  // extern "C"

// n steps; the last writes the moment planes when mom_last is set
template <typename real>
static lf_status step_impl(lf_case* c, int64_t n, bool mom_last = true) {
  hipStream_t s = c->ctx->stream;
  const int band = auto_band(c);
  for (int64_t k = 0; k < n; ++k) {
    const int a = c->cur, b = a ^ 1;
    real* mom = (mom_last && k == n - 1) ? fptr<real>(c, c->off_mom) : nullptr;
    HIP_TRY(lf::launch_hybrid_step<real>(
        c->g, c->w, c->p, fptr<real>(c, c->off_f[a]), fptr<real>(c, c->off_f[b]),
        fptr<real>(c, c->off_T[a]), fptr<real>(c, c->off_T[b]),
        c->tcomp ? (lf::tlo_t*)(c->ws + c->off_Tlo[a]) : nullptr,
        c->tcomp ? (lf::tlo_t*)(c->ws + c->off_Tlo[b]) : nullptr, mom, band, s));
    c->cur = b;
  }
  c->steps += n;
  return LF_OK;
}

// Steps launched one call at a time (the last writing the moments when
// mom_last is set).
static lf_status eager_steps(lf_case* c, int64_t n, bool mom_last) {
  if (c->split)
    return c->desc.precision == LF_F32 ? split_steps<float>(c, n, mom_last)
                                       : split_steps<double>(c, n, mom_last);
  return c->desc.precision == LF_F32 ? step_impl<float>(c, n, mom_last)
                                     : step_impl<double>(c, n, mom_last);
}

// Long step calls replay a captured hipGraph of kGraphSteps steps (an even
// count, so a run starts and ends on the same buffer set) and launch the
// remaining 1 .. kGraphSteps steps one by one, the last writing the
// moments.  A run's kernel arguments hold the case's buffers and settings,
// so it is captured again when the signature of those changes.  Grid
// setting 2 and LBM-MCM launch an energy step every S lattice steps counted
// since init (and MCM a new stream seed each time): launched one by one.
constexpr int64_t kGraphSteps = 64;

static uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
  return h;
}

static uint64_t graph_signature(const lf_case* c) {
  uint64_t h = 14695981039346656037ull;
  h = fnv1a(h, &c->ws, sizeof(c->ws));
  h = fnv1a(h, &c->ctx->band, sizeof(c->ctx->band));
  h = fnv1a(h, &c->g, sizeof(c->g));
  h = fnv1a(h, &c->w, sizeof(c->w));
  h = fnv1a(h, &c->p, sizeof(c->p));
  h = fnv1a(h, &c->sg, sizeof(c->sg));
  h = fnv1a(h, &c->sp, sizeof(c->sp));
  return h;
}

static void drop_graphs(lf_case* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
    c->gexec[k] = nullptr;
    c->gsig[k] = 0;
  }
}

// the run of kGraphSteps steps from the current buffer set, captured if need be
static lf_status ensure_run(lf_case* c, uint64_t sig) {
  const int slot = c->cur;
  if (c->gexec[slot] && c->gsig[slot] == sig) return LF_OK;
  if (c->gexec[slot]) (void)hipGraphExecDestroy(c->gexec[slot]);
  c->gexec[slot] = nullptr;
  hipStream_t s = c->ctx->stream;
  const int cur0 = c->cur;
  const int64_t steps0 = c->steps;
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  lf_status st = eager_steps(c, kGraphSteps, false);  // recorded, not run
  c->cur = cur0;
  c->steps = steps0;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != LF_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != LF_OK ? st : fail(LF_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  const hipError_t ei = hipGraphInstantiate(&c->gexec[slot], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->gexec[slot] = nullptr;
    return fail(LF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  c->gsig[slot] = sig;
  return LF_OK;
}

static lf_status run_steps(lf_case* c, int64_t n) {
  const bool cyclic = c->split && (c->sg.gs2 || c->sg.mcm);
  if (cyclic || n <= kGraphSteps) return eager_steps(c, n, true);
  const uint64_t sig = graph_signature(c);
  for (int64_t reps = (n - 1) / kGraphSteps; reps > 0; --reps) {
    lf_status st = ensure_run(c, sig);
    if (st != LF_OK) return st;
    HIP_TRY(hipGraphLaunch(c->gexec[c->cur], c->ctx->stream));
    c->steps += kGraphSteps;
    n -= kGraphSteps;
  }
  return eager_steps(c, n, true);
}

extern "C" {

lf_status lf_case_step(lf_case* c, int64_t nsteps) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  if (nsteps < 0) return fail(LF_EINVAL, "nsteps < 0");
  if (!c->inited) return fail(LF_ESTATE, "init before step");
  if (!c->have_params) return fail(LF_ESTATE, "set_physics or set_lattice before step");
  if (nsteps == 0) return LF_OK;
  return run_steps(c, nsteps);
}

lf_status lf_case_profile_steps(lf_case* c, int64_t nsteps, double* avg_ms, double* min_ms,
                                double* max_ms) {
  if (!c || !avg_ms) return fail(LF_EINVAL, "NULL argument");
  if (nsteps < 1 || nsteps > (1 << 20)) return fail(LF_EINVAL, "nsteps must be in [1, 2^20]");
  if (!c->inited) return fail(LF_ESTATE, "init before step");
  if (!c->have_params) return fail(LF_ESTATE, "set_physics or set_lattice before step");
  // launches run back to back; an event is recorded every `chunk` launches
  // and read after the last one, so the timing adds no synchronisation
  const int64_t chunk = nsteps < 64 ? nsteps : 64;
  const int64_t nchunks = (nsteps + chunk - 1) / chunk;
  std::vector<hipEvent_t> ev((size_t)nchunks + 1, nullptr);
  lf_status st = LF_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) { st = fail(LF_EDEVICE, "hipEventCreate"); break; }
  hipStream_t s = c->ctx->stream;
  std::vector<double> per;
  if (st == LF_OK && hipEventRecord(ev[0], s) != hipSuccess) st = fail(LF_EDEVICE, "hipEventRecord");
  int64_t done = 0;
  for (int64_t k = 0; st == LF_OK && k < nchunks; ++k) {
    const int64_t m = (nsteps - done) < chunk ? (nsteps - done) : chunk;
    if (c->split)
      st = c->desc.precision == LF_F32 ? split_steps<float>(c, m) : split_steps<double>(c, m);
    else
      st = c->desc.precision == LF_F32 ? step_impl<float>(c, m) : step_impl<double>(c, m);
    if (st == LF_OK && hipEventRecord(ev[(size_t)k + 1], s) != hipSuccess)
      st = fail(LF_EDEVICE, "hipEventRecord");
    done += m;
    per.push_back((double)m);
  }
  double total = 0.0, lo = 1e300, hi = 0.0;
  if (st == LF_OK && hipEventSynchronize(ev[(size_t)nchunks]) != hipSuccess)
    st = fail(LF_EDEVICE, "hipEventSynchronize");
  for (int64_t k = 0; st == LF_OK && k < nchunks; ++k) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev[(size_t)k], ev[(size_t)k + 1]) != hipSuccess) {
      st = fail(LF_EDEVICE, "hipEventElapsedTime");
      break;
    }
    total += ms;
    const double a = ms / per[(size_t)k];
    lo = a < lo ? a : lo;
    hi = a > hi ? a : hi;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (st != LF_OK) return st;
  *avg_ms = total / (double)nsteps;
  if (min_ms) *min_ms = lo;
  if (max_ms) *max_ms = hi;
  return LF_OK;
}

lf_status lf_case_steps(const lf_case* c, int64_t* steps) {
  if (!c || !steps) return fail(LF_EINVAL, "NULL argument");
  *steps = c->steps;
  return LF_OK;
}

}  // extern "C"

// the residual with its partials in `part` (c->nblk blocks x 8 doubles) and
// the fold's output in `out` (7 doubles)
static lf_status case_residual(lf_case* c, double* part, double* out, double r[3]) {
  hipStream_t s = c->ctx->stream;
  if (c->split) {
    const lf::Grid dg = dense_grid(c);
    const size_t n = (size_t)dg.plane;
    if (c->desc.precision == LF_F32) {
      lf_status st = split_dense<float>(c);
      if (st != LF_OK) return st;
      float* d = fptr<float>(c, c->off_dense);
      HIP_TRY(lf::launch_residual<float>(dg, d, d + 3 * n, fptr<float>(c, c->off_dsnap), part,
                                         c->nblk, out, s));
    } else {
      lf_status st = split_dense<double>(c);
      if (st != LF_OK) return st;
      double* d = fptr<double>(c, c->off_dense);
      HIP_TRY(lf::launch_residual<double>(dg, d, d + 3 * n, fptr<double>(c, c->off_dsnap), part,
                                          c->nblk, out, s));
    }
  } else if (c->desc.precision == LF_F32) {
    HIP_TRY(lf::launch_residual<float>(c->g, fptr<float>(c, c->off_mom),
                                       fptr<float>(c, c->off_T[c->cur]),
                                       fptr<float>(c, c->off_snap), part, c->nblk, out, s));
  } else {
    HIP_TRY(lf::launch_residual<double>(c->g, fptr<double>(c, c->off_mom),
                                        fptr<double>(c, c->off_T[c->cur]),
                                        fptr<double>(c, c->off_snap), part, c->nblk, out, s));
  }
  double h[7];
  HIP_TRY(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < 3; ++k) {
    const double num = sqrt(h[2 * k]), den = sqrt(h[2 * k + 1]);
    r[k] = den < 1e-300 ? num : num / den;
  }
  if (h[6] != 0.0) return fail(LF_EDIVERGED, "%.0f non-finite values after %lld steps", h[6],
                               (long long)c->steps);
  return LF_OK;
}

extern "C" {

lf_status lf_case_residual(lf_case* c, double r[3]) {
  if (!c || !r) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  return case_residual(c, (double*)(c->ws + c->off_part), (double*)(c->ws + c->off_out), r);
}

lf_status lf_case_residual_noalloc(lf_case* c, double r[3]) {
  if (!c || !r) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  if (c->nblk > kNoallocBlocks)
    return fail(LF_EINVAL, "residual needs %d partial blocks, the static scratch holds %d",
                c->nblk, kNoallocBlocks);
  double* part = g_scratch_ptr[c->ctx->device];
  if (!part) return fail(LF_ESTATE, "no scratch address for device %d", c->ctx->device);
  return case_residual(c, part, part + (size_t)kNoallocBlocks * 8, r);
}

lf_status lf_case_run_to_steady(lf_case* c, double tol, int check_every, int64_t max_steps,
                                int64_t* steps_taken, double r_final[3], int* rule) {
  if (!c) return fail(LF_EINVAL, "NULL case");
  if (!(tol > 0.0) || check_every < 1 || max_steps < 0) return fail(LF_EINVAL, "bad stop settings");
  double r[3] = {0, 0, 0};
  lf_status st = lf_case_residual(c, r);  // snapshot the current state
  if (st != LF_OK) return st;
  std::vector<double> hist;
  // the slowest diffusive mode the FP32 floor rule waits for
  const double lam_min = lf_slow_mode(c->params[3], c->params[1], c->desc.nx, c->desc.ny,
                                      c->w.tfix, c->w.xper, c->w.yper, check_every);
  int64_t done = 0;
  int fired = 0;
  while (done < max_steps) {
    const int64_t k = (max_steps - done) < check_every ? (max_steps - done) : check_every;
    st = lf_case_step(c, k);
    if (st != LF_OK) return st;
    done += k;
    st = lf_case_residual(c, r);
    if (st != LF_OK) break;
    const double m = fmax(r[0], fmax(r[1], r[2]));
    hist.push_back(m);
    if (m <= tol || (r[0] == 0.0 && r[1] == 0.0 && r[2] == 0.0)) { fired = LF_STOP_TOL; break; }
    if (c->desc.precision == LF_F32 && lf_at_floor(hist, lam_min)) {
      fired = LF_STOP_FLOOR;
      break;
    }
  }
  if (steps_taken) *steps_taken = done;
  if (r_final) memcpy(r_final, r, sizeof(r));
  if (rule) *rule = fired;
  if (st != LF_OK) return st;
  if (!fired) return fail(LF_ENOTCONV, "max residual %.3g after %lld steps", fmax(r[0], fmax(r[1], r[2])),
                          (long long)done);
  return LF_OK;
}

lf_status lf_case_nusselt(lf_case* c, lf_nusselt* out) {
  if (!c || !out) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  hipStream_t s = c->ctx->stream;
  double* dout = (double*)(c->ws + c->off_out) + 16;
  if (c->split) {
    const lf::Grid dg = dense_grid(c);
    const size_t n = (size_t)dg.plane;
    lf_status st = c->desc.precision == LF_F32 ? split_dense<float>(c) : split_dense<double>(c);
    if (st != LF_OK) return st;
    if (c->desc.precision == LF_F32)
      HIP_TRY(lf::launch_nusselt<float>(dg, c->w, fptr<float>(c, c->off_dense) + 3 * n, dout, s));
    else
      HIP_TRY(lf::launch_nusselt<double>(dg, c->w, fptr<double>(c, c->off_dense) + 3 * n, dout, s));
  } else if (c->desc.precision == LF_F32)
    HIP_TRY(lf::launch_nusselt<float>(c->g, c->w, fptr<float>(c, c->off_T[c->cur]), dout, s));
  else
    HIP_TRY(lf::launch_nusselt<double>(c->g, c->w, fptr<double>(c, c->off_T[c->cur]), dout, s));
  double h[8];
  HIP_TRY(hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  out->nu_hot = h[0]; out->nu_cold = h[1]; out->nu_hot_max = h[2]; out->y_hot_max = h[3];
  out->nu_cold_max = h[4]; out->y_cold_max = h[5]; out->nu_hot_o2 = h[6]; out->nu_cold_o2 = h[7];
  return LF_OK;
}

lf_status lf_case_fetch(lf_case* c, int field, void* dst, size_t dst_bytes, int dst_is_device,
                        int as_f64) {
  if (!c || !dst) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  const size_t n = (size_t)c->g.nx * c->g.ny;
  const size_t need = n * (as_f64 ? 8 : c->es);
  if (dst_bytes < need) return fail(LF_EINVAL, "dst holds %zu bytes, %zu needed", dst_bytes, need);
  const size_t pb = align_up((size_t)c->g.plane * c->es, 256);
  size_t off;
  switch (field) {
    case LF_FIELD_RHO: case LF_FIELD_P: off = c->off_mom; break;
    case LF_FIELD_U: off = c->off_mom + pb; break;
    case LF_FIELD_V: off = c->off_mom + 2 * pb; break;
    case LF_FIELD_T: off = c->off_T[c->cur]; break;
    default: return fail(LF_EINVAL, "bad field %d", field);
  }
  const int pressure = field == LF_FIELD_P ? 1 : 0;
  hipStream_t s = c->ctx->stream;
  void* target = dst_is_device ? dst : (void*)(c->ws + c->off_stage);
  lf::Grid g = c->g;
  if (c->split) {
    g = dense_grid(c);
    lf_status st = c->desc.precision == LF_F32 ? split_dense<float>(c) : split_dense<double>(c);
    if (st != LF_OK) return st;
    // U, V, T, RHO, P -> dense planes rho, u, v, T (P from rho)
    const int plane_of[5] = {1, 2, 3, 0, 0};
    off = c->off_dense + (size_t)plane_of[field] * (size_t)g.plane * c->es;
  }
  if (c->desc.precision == LF_F32)
    HIP_TRY(lf::launch_unpack<float>(g, fptr<float>(c, off), target, as_f64, s, pressure));
  else
    HIP_TRY(lf::launch_unpack<double>(g, fptr<double>(c, off), target, as_f64, s, pressure));
  if (!dst_is_device) {
    HIP_TRY(hipMemcpyAsync(dst, target, need, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return LF_OK;
}

// checkpoint blob: header, then the bound workspace's first `need` bytes
namespace {
struct CaseBlobHeader {
  char magic[8];  // "LFCASE2"
  int abi;
  lf_case_desc desc;
  size_t es, need;
  int cur, have_params;
  int64_t steps;
  double params[8];
  lf::WallSet w;
  lf::HybridParams p;
  lf::SplitParams sp;
  // cycle settings of grid setting 2 and of LBM-MCM
  int gs2_S, gs2_K, mcm_S, mcm_N;
  unsigned long long mcm_seed;
  long long mcm_max;
};
}  // namespace

lf_status lf_case_save(lf_case* c, void* blob, size_t* bytes) {
  if (!c || !bytes) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  const size_t total = sizeof(CaseBlobHeader) + c->need;
  if (!blob) {
    *bytes = total;
    return LF_OK;
  }
  if (*bytes < total) return fail(LF_EINVAL, "blob holds %zu bytes, %zu needed", *bytes, total);
  CaseBlobHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "LFCASE2", 8);
  h.abi = LF_ABI_VERSION;
  h.desc = c->desc;
  h.es = c->es;
  h.need = c->need;
  h.cur = c->cur;
  h.have_params = c->have_params ? 1 : 0;
  h.steps = c->steps;
  memcpy(h.params, c->params, sizeof(h.params));
  h.w = c->w;
  h.p = c->p;
  h.sp = c->sp;
  h.gs2_S = c->gs2_S;
  h.gs2_K = c->gs2_K;
  h.mcm_S = c->mcm_S;
  h.mcm_N = c->mcm_N;
  h.mcm_seed = c->mcm_seed;
  h.mcm_max = c->mcm_max;
  memcpy(blob, &h, sizeof(h));
  hipStream_t s = c->ctx->stream;
  HIP_TRY(hipMemcpyAsync((char*)blob + sizeof(h), c->ws, c->need, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *bytes = total;
  return LF_OK;
}

lf_status lf_case_load(lf_case* c, const void* blob, size_t bytes) {
  if (!c || !blob) return fail(LF_EINVAL, "NULL argument");
  if (!c->ws) return fail(LF_EWORKSPACE, "no workspace bound");
  CaseBlobHeader h;
  if (bytes < sizeof(h)) return fail(LF_EINVAL, "blob too short");
  memcpy(&h, blob, sizeof(h));
  if (memcmp(h.magic, "LFCASE2", 8) != 0 || h.abi != LF_ABI_VERSION)
    return fail(LF_EINVAL, "not a checkpoint of this library");
  if (memcmp(&h.desc, &c->desc, sizeof(lf_case_desc)) != 0 || h.es != c->es || h.need != c->need)
    return fail(LF_EINVAL, "checkpoint of a different case geometry or precision");
  if (bytes < sizeof(h) + h.need) return fail(LF_EINVAL, "blob truncated");
  hipStream_t s = c->ctx->stream;
  HIP_TRY(hipMemcpyAsync(c->ws, (const char*)blob + sizeof(h), h.need, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  c->cur = h.cur;
  c->have_params = h.have_params != 0;
  c->steps = h.steps;
  memcpy(c->params, h.params, sizeof(h.params));
  c->w = h.w;
  c->p = h.p;
  c->sp = h.sp;
  c->gs2_S = h.gs2_S;
  c->gs2_K = h.gs2_K;
  c->mcm_S = h.mcm_S;
  c->mcm_N = h.mcm_N;
  c->mcm_seed = h.mcm_seed;
  c->mcm_max = h.mcm_max;
  c->inited = true;
  return LF_OK;
}

lf_status lf_case_mass(lf_case* c, double* sum_f, double* sum_T) {
  if (!c || !sum_f || !sum_T) return fail(LF_EINVAL, "NULL argument");
  if (!c->inited) return fail(LF_ESTATE, "init first");
  hipStream_t s = c->ctx->stream;
  double* out = (double*)(c->ws + c->off_out) + 32;
  double* part = (double*)(c->ws + c->off_part);
  if (c->split && c->sg.fv_only) {
    // no populations: the FV density 1 + 3 p and T summed over the cells
    const size_t n = (size_t)c->sg.nx * c->sg.ny;
    std::vector<double> r(n), T(n);
    lf_status st = lf_case_fetch(c, LF_FIELD_RHO, r.data(), n * sizeof(double), 0, 1);
    if (st == LF_OK) st = lf_case_fetch(c, LF_FIELD_T, T.data(), n * sizeof(double), 0, 1);
    if (st != LF_OK) return st;
    double sr = 0.0, sT = 0.0;
    for (size_t k = 0; k < n; ++k) {
      sr += r[k];
      sT += T[k];
    }
    *sum_f = sr;
    *sum_T = sT;
    return LF_OK;
  }
  if (c->split) {
    // populations of the LBM zone (nodes 0 .. ib, all nx nodes without an FV
    // zone); T summed over the whole cavity from the output field
    lf::Grid gl;
    gl.nx = (c->sg.lbm_only || c->sg.gs2 || c->sg.mcm) ? c->sg.nx : c->sg.ib + 1;
    gl.ny = c->sg.ny;
    gl.pitch = c->sg.pL;
    gl.plane = c->sg.planeL;
    const size_t n = (size_t)c->sg.nx * c->sg.ny;
    std::vector<double> T(n);
    lf_status st = lf_case_fetch(c, LF_FIELD_T, T.data(), n * sizeof(double), 0, 1);
    if (st != LF_OK) return st;
    if (c->desc.precision == LF_F32)
      HIP_TRY(lf::launch_mass<float>(gl, fptr<float>(c, c->off_sf[c->cur]),
                                     fptr<float>(c, c->off_smom), part, c->nblk, out, s));
    else
      HIP_TRY(lf::launch_mass<double>(gl, fptr<double>(c, c->off_sf[c->cur]),
                                      fptr<double>(c, c->off_smom), part, c->nblk, out, s));
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sT = 0.0;
    for (double t : T) sT += t;
    *sum_f = h[0] + (double)gl.nx * gl.ny;
    *sum_T = sT;
    return LF_OK;
  }
  if (c->desc.precision == LF_F32)
    HIP_TRY(lf::launch_mass<float>(c->g, fptr<float>(c, c->off_f[c->cur]),
                                   fptr<float>(c, c->off_T[c->cur]), part, c->nblk, out, s));
  else
    HIP_TRY(lf::launch_mass<double>(c->g, fptr<double>(c, c->off_f[c->cur]),
                                    fptr<double>(c, c->off_T[c->cur]), part, c->nblk, out, s));
  double h[2];
  HIP_TRY(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // populations are stored as f - w_q; the weights of a node sum to one
  *sum_f = h[0] + (double)c->g.nx * c->g.ny;
  *sum_T = h[1];
  return LF_OK;
}

}  // extern "C"
