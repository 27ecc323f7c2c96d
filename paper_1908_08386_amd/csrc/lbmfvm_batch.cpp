// lbmfvm_batch.cpp -- batched Mode H cavities behind the C ABI.
//
// A batch lays out every cavity's planes (populations ping-pong, T
// ping-pong, rho/u/v, residual snapshot) in one caller-bound workspace, plus
// device tables: cavity descriptors, the tile list of the live cavities, the
// residual work list and per-cavity folds.  run_to_steady captures "K steps
// + batched residual" once as a hipGraph and replays it; between replays the
// host reads the per-cavity residuals, retires converged cavities and
// uploads the shrunk tables (the graph reads the live counts from device
// memory, so it never has to be re-captured).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "lf_host.h"
#include "lf_internal.h"

namespace {

struct Cav {
  int nx, ny, pitch;
  long long plane;
  size_t off_f[2], off_T[2], off_mom, off_snap, off_Tlo[2];
  int band;
  double prm[8];
  int tfix[4];
  double Tw[4], uw[4];
  int cur;
  bool active;
  int64_t steps;
  std::vector<double> hist;
  int rule;
  double r[3];
};

constexpr int kOut = 62;  // output columns per wave tile

// The band a cavity starts with: the autotuner's table entry for its height
// class if the context holds one, else 0 ("by load", see load_band).
int default_band(const lf_ctx* ctx, int ny) {
  if (ctx->tune.valid) {
    int best = -1;
    for (int k = 0; k < ctx->tune.nclass; ++k)
      if (ctx->tune.ny_class[k] <= ny &&
          (best < 0 || ctx->tune.ny_class[k] > ctx->tune.ny_class[best]))
        best = k;
    if (best < 0 && ctx->tune.nclass > 0) best = 0;
    if (best >= 0) return ctx->tune.band[best];
  }
  return 0;
}

}  // namespace

struct lf_batch {
  lf_ctx* ctx;
  int n;
  int precision;
  bool tcomp;
  size_t es;
  std::vector<Cav> cav;
  char* ws;
  size_t need;
  size_t off_cavdesc, off_tiles, off_ntiles, off_rt, off_nrt, off_fold, off_nfold, off_part,
      off_out, off_stage;
  int max_tiles, max_rt, max_fold;
  size_t stage_elems;
  // host copies of the live tables (kept alive across async uploads)
  std::vector<lf::TileDesc> tiles;
  std::vector<lf::ResidTile> rts;
  std::vector<lf::FoldDesc> folds;
  int counts[3];
  std::vector<unsigned char> cavdesc;
  int row1;  // every live tile is a single row (the step kernel's 5-wave form)
  // tiles the step launches are sized for: at least the live table, and
  // re-sized when the table outgrows it or falls below half of it, so a
  // shrinking live set is recaptured O(log) times while blocks with no tile
  // stay under half of the grid
  int grid_tiles;
  hipGraphExec_t gexec;
  int graph_K, graph_row1, graph_tiles;
  bool inited;
};

static int tiles_of(const Cav& c, int band) {
  return ((c.nx + kOut - 1) / kOut) * ((c.ny + band - 1) / band);
}
static int rtiles_of(const Cav& c) { return c.ny < 16 ? c.ny : 16; }

static void batch_layout(lf_batch* b) {
  size_t o = 0;
  for (auto& c : b->cav) {
    const size_t pb = lf_align_up((size_t)c.plane * b->es, 256);
    c.off_f[0] = o; o += 9 * pb;
    c.off_f[1] = o; o += 9 * pb;
    c.off_T[0] = o; o += pb;
    c.off_T[1] = o; o += pb;
    c.off_mom = o; o += 3 * pb;
    c.off_snap = o; o += 3 * pb;
    c.off_Tlo[0] = c.off_Tlo[1] = 0;
    if (b->tcomp) {  // one byte per node and plane
      const size_t pl = lf_align_up((size_t)c.plane, 256);
      c.off_Tlo[0] = o; o += pl;
      c.off_Tlo[1] = o; o += pl;
    }
  }
  b->max_tiles = 0;
  b->max_rt = 0;
  size_t stage = 0;
  for (const auto& c : b->cav) {
    // any band >= 1 fits in the table sized for band 1
    b->max_tiles += tiles_of(c, 1);
    b->max_rt += rtiles_of(c);
    stage = stage > (size_t)c.nx * c.ny ? stage : (size_t)c.nx * c.ny;
  }
  b->max_fold = b->n;
  b->stage_elems = 3 * stage;
  const size_t descsz = b->precision == LF_F32 ? sizeof(lf::CavDesc<float>) : sizeof(lf::CavDesc<double>);
  b->off_cavdesc = o; o += lf_align_up(descsz * b->n, 256);
  b->off_tiles = o; o += lf_align_up(sizeof(lf::TileDesc) * b->max_tiles, 256);
  b->off_ntiles = o; o += 256;
  b->off_rt = o; o += lf_align_up(sizeof(lf::ResidTile) * b->max_rt, 256);
  b->off_nrt = o; o += 256;
  b->off_fold = o; o += lf_align_up(sizeof(lf::FoldDesc) * b->max_fold, 256);
  b->off_nfold = o; o += 256;
  b->off_part = o; o += lf_align_up(8 * sizeof(double) * b->max_rt, 256);
  b->off_out = o; o += lf_align_up(8 * sizeof(double) * b->n, 256);
  b->off_stage = o; o += lf_align_up(sizeof(double) * b->stage_elems, 256);
  b->need = o;
}

template <typename real>
static void fill_desc(lf_batch* b) {
  b->cavdesc.assign(sizeof(lf::CavDesc<real>) * b->n, 0);
  lf::CavDesc<real>* d = (lf::CavDesc<real>*)b->cavdesc.data();
  for (int k = 0; k < b->n; ++k) {
    const Cav& c = b->cav[k];
    d[k].f[0] = (real*)(b->ws + c.off_f[0]);
    d[k].f[1] = (real*)(b->ws + c.off_f[1]);
    d[k].T[0] = (real*)(b->ws + c.off_T[0]);
    d[k].T[1] = (real*)(b->ws + c.off_T[1]);
    d[k].Tlo[0] = b->tcomp ? (lf::tlo_t*)(b->ws + c.off_Tlo[0]) : nullptr;
    d[k].Tlo[1] = b->tcomp ? (lf::tlo_t*)(b->ws + c.off_Tlo[1]) : nullptr;
    d[k].mom = (real*)(b->ws + c.off_mom);
    d[k].snap = (real*)(b->ws + c.off_snap);
    d[k].nx = c.nx;
    d[k].ny = c.ny;
    d[k].pitch = c.pitch;
    d[k].plane = (int)c.plane;
    d[k].cur = c.cur;
    for (int s = 0; s < 4; ++s) {
      d[k].tfix[s] = c.tfix[s];
      d[k].Tw[s] = c.Tw[s];
      d[k].uw[s] = c.uw[s];
    }
    d[k].omega = 1.0 / c.prm[2];
    d[k].alpha = c.prm[3];
    d[k].gbeta = c.prm[5];
    d[k].Tref = c.prm[6];
  }
}

// rebuild and upload the live tables and the descriptors
// Rows per wave tile for the cavities whose band is chosen by load: the
// single-cavity rule (lf_rows_per_wave) applied to the live set's rows, so
// that a small live set (a single 512^2 cavity, or the last unconverged
// cavities of a sweep) runs single rows spread over the whole chip and the
// full sweep bands of 4.
static int load_band(const lf_batch* b) {
  long long w1 = 0;
  for (const auto& c : b->cav)
    if (c.active && c.band == 0) w1 += tiles_of(c, 1);
  return lf_rows_per_wave(w1);
}

static lf_status upload_tables(lf_batch* b) {
  b->tiles.clear();
  b->rts.clear();
  b->folds.clear();
  const int lband = load_band(b);
  for (int k = 0; k < b->n; ++k) {
    const Cav& c = b->cav[k];
    if (!c.active) continue;
    const int strips = (c.nx + kOut - 1) / kOut;
    const int band = c.band > 0 ? c.band : lband;
    for (int j0 = 0; j0 < c.ny; j0 += band)
      for (int s = 0; s < strips; ++s) {
        lf::TileDesc t;
        t.cav = k;
        t.strip = s;
        t.j0 = j0;
        t.j1 = j0 + band < c.ny ? j0 + band : c.ny;
        b->tiles.push_back(t);
      }
    const int nr = rtiles_of(c);
    lf::FoldDesc f;
    f.cav = k;
    f.start = (int)b->rts.size();
    f.count = nr;
    f.pad = 0;
    for (int r = 0; r < nr; ++r) {
      lf::ResidTile t;
      t.cav = k;
      t.j0 = (int)((long long)c.ny * r / nr);
      t.j1 = (int)((long long)c.ny * (r + 1) / nr);
      t.pad = 0;
      b->rts.push_back(t);
    }
    b->folds.push_back(f);
  }
  if ((int)b->tiles.size() > b->max_tiles) return lf_fail(LF_EINVAL, "tile table overflow");
  b->row1 = 1;
  for (const auto& t : b->tiles)
    if (t.j1 - t.j0 != 1) b->row1 = 0;
  b->counts[0] = (int)b->tiles.size();
  if (b->counts[0] > b->grid_tiles || 2 * b->counts[0] < b->grid_tiles)
    b->grid_tiles = b->counts[0] > 0 ? b->counts[0] : 1;
  b->counts[1] = (int)b->rts.size();
  b->counts[2] = (int)b->folds.size();
  if (b->precision == LF_F32) fill_desc<float>(b);
  else fill_desc<double>(b);
  hipStream_t s = b->ctx->stream;
  LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_cavdesc, b->cavdesc.data(), b->cavdesc.size(),
                            hipMemcpyHostToDevice, s));
  if (!b->tiles.empty())
    LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_tiles, b->tiles.data(),
                              b->tiles.size() * sizeof(lf::TileDesc), hipMemcpyHostToDevice, s));
  if (!b->rts.empty())
    LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_rt, b->rts.data(),
                              b->rts.size() * sizeof(lf::ResidTile), hipMemcpyHostToDevice, s));
  if (!b->folds.empty())
    LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_fold, b->folds.data(),
                              b->folds.size() * sizeof(lf::FoldDesc), hipMemcpyHostToDevice, s));
  LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_ntiles, &b->counts[0], sizeof(int),
                            hipMemcpyHostToDevice, s));
  LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_nrt, &b->counts[1], sizeof(int),
                            hipMemcpyHostToDevice, s));
  LF_HIP_TRY(hipMemcpyAsync(b->ws + b->off_nfold, &b->counts[2], sizeof(int),
                            hipMemcpyHostToDevice, s));
  // the host vectors are rewritten only after this point has been reached
  LF_HIP_TRY(hipStreamSynchronize(s));
  return LF_OK;
}

template <typename real>
static hipError_t enqueue_steps(lf_batch* b, int64_t k0, int64_t n, bool write_mom_last) {
  const lf::CavDesc<real>* d = (const lf::CavDesc<real>*)(b->ws + b->off_cavdesc);
  for (int64_t k = 0; k < n; ++k) {
    hipError_t e = lf::launch_batch_step<real>(
        (const lf::TileDesc*)(b->ws + b->off_tiles), (const int*)(b->ws + b->off_ntiles),
        b->grid_tiles, d, (int)((k0 + k) & 1), (write_mom_last && k == n - 1) ? 1 : 0, 0,
        b->row1, b->ctx->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename real>
static hipError_t enqueue_residual(lf_batch* b) {
  return lf::launch_batch_residual<real>(
      (const lf::ResidTile*)(b->ws + b->off_rt), (const int*)(b->ws + b->off_nrt), b->max_rt,
      (const lf::FoldDesc*)(b->ws + b->off_fold), (const int*)(b->ws + b->off_nfold),
      b->max_fold, (const lf::CavDesc<real>*)(b->ws + b->off_cavdesc),
      (double*)(b->ws + b->off_part), (double*)(b->ws + b->off_out), b->ctx->stream);
}

static hipError_t enqueue_steps_any(lf_batch* b, int64_t k0, int64_t n, bool mom) {
  return b->precision == LF_F32 ? enqueue_steps<float>(b, k0, n, mom)
                                : enqueue_steps<double>(b, k0, n, mom);
}
static hipError_t enqueue_residual_any(lf_batch* b) {
  return b->precision == LF_F32 ? enqueue_residual<float>(b) : enqueue_residual<double>(b);
}

static void drop_graph(lf_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->graph_K = 0;
}

// K steps (K even) followed by the batched residual, captured once per K,
// per form of the step kernel and per grid size
static lf_status ensure_graph(lf_batch* b, int K) {
  if (b->gexec && b->graph_K == K && b->graph_row1 == b->row1 && b->graph_tiles == b->grid_tiles)
    return LF_OK;
  drop_graph(b);
  hipStream_t s = b->ctx->stream;
  LF_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_steps_any(b, 0, K, true);
  if (e == hipSuccess) e = enqueue_residual_any(b);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return lf_fail(LF_EDEVICE, "graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->gexec = nullptr;
    return lf_fail(LF_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  b->graph_K = K;
  b->graph_row1 = b->row1;
  b->graph_tiles = b->grid_tiles;
  return LF_OK;
}

static void residual_of(const double* h, double r[3]) {
  for (int q = 0; q < 3; ++q) {
    const double num = sqrt(h[2 * q]), den = sqrt(h[2 * q + 1]);
    r[q] = den < 1e-300 ? num : num / den;
  }
}

extern "C" {

lf_status lf_batch_create(lf_ctx* ctx, int n, const lf_case_desc* descs, const lf_physics* phys,
                          const lf_wall* walls, lf_batch** out) {
  if (!ctx || !descs || !phys || !out || n < 1) return lf_fail(LF_EINVAL, "bad arguments");
  const int prec = descs[0].precision;
  if (prec != LF_F32 && prec != LF_F64) return lf_fail(LF_EINVAL, "bad precision");
  lf_batch* b = new (std::nothrow) lf_batch();
  if (!b) return lf_fail(LF_ENOMEM, "batch allocation");
  b->ctx = ctx;
  b->n = n;
  b->precision = prec;
  b->es = prec == LF_F64 ? 8 : 4;
  b->tcomp = prec == LF_F32 && descs[0].tcomp;
  b->cav.resize(n);
  for (int k = 0; k < n; ++k) {
    const lf_case_desc& d = descs[k];
    Cav& c = b->cav[k];
    if (d.precision != prec || d.mode != LF_MODE_HYBRID || d.nx < 8 || d.ny < 8) {
      delete b;
      return lf_fail(LF_EINVAL, "cavity %d: batches hold Mode H cavities of one precision, "
                     "nx, ny >= 8", k);
    }
    c.nx = d.nx;
    c.ny = d.ny;
    c.pitch = (d.nx + 63) / 64 * 64;
    c.plane = lf_plane_elems(c.pitch, d.ny);
    if (!lf_planes_fit(c.plane, b->es)) {
      delete b;
      return lf_fail(LF_EINVAL, "cavity %d too large: nine planes must stay under 4 GiB", k);
    }
    lf_status st = lf_derive_params(&phys[k], d.ny, 0, c.prm);
    if (st != LF_OK) {
      delete b;
      return st;
    }
    if (!(c.prm[2] > 0.501) || c.prm[3] > 0.25) {
      delete b;
      return lf_fail(LF_EUNSTABLE, "cavity %d: tau %.4g, alpha %.4g outside the explicit limits",
                     k, c.prm[2], c.prm[3]);
    }
    if (phys[k].conv != LF_CONV_QUICK || phys[k].body_gx != 0.0 || phys[k].body_gy != 0.0) {
      delete b;
      return lf_fail(LF_ENOTIMPL, "cavity %d: batches use QUICK and no body force", k);
    }
    // default: side-heated cavity
    c.tfix[0] = 1; c.Tw[0] = 0.5;
    c.tfix[1] = 1; c.Tw[1] = -0.5;
    c.tfix[2] = 0; c.Tw[2] = 0.0;
    c.tfix[3] = 0; c.Tw[3] = 0.0;
    for (int s = 0; s < 4; ++s) c.uw[s] = 0.0;
    if (walls) {
      for (int s = 0; s < 4; ++s) {
        const lf_wall& w = walls[4 * k + s];
        if (w.vel != LF_WALL_NOSLIP || w.thermal == LF_T_PERIODIC) {
          delete b;
          return lf_fail(LF_ENOTIMPL, "cavity %d: batches have no periodic sides", k);
        }
        c.tfix[s] = w.thermal == LF_T_DIRICHLET;
        c.Tw[s] = w.T_wall;
        c.uw[s] = w.u_wall;
      }
    }
    c.band = default_band(ctx, d.ny);
    c.cur = 0;
    c.active = false;
    c.steps = 0;
    c.rule = 0;
    c.r[0] = c.r[1] = c.r[2] = 0.0;
  }
  batch_layout(b);
  *out = b;
  return LF_OK;
}

lf_status lf_batch_destroy(lf_batch* b) {
  if (!b) return LF_OK;
  drop_graph(b);
  delete b;
  return LF_OK;
}

lf_status lf_batch_workspace_bytes(const lf_batch* b, size_t* bytes) {
  if (!b || !bytes) return lf_fail(LF_EINVAL, "NULL argument");
  *bytes = b->need;
  return LF_OK;
}

lf_status lf_batch_bind_workspace(lf_batch* b, void* dev, size_t bytes) {
  if (!b || !dev) return lf_fail(LF_EINVAL, "NULL argument");
  if (bytes < b->need) return lf_fail(LF_EWORKSPACE, "workspace %zu < %zu bytes", bytes, b->need);
  if ((uintptr_t)dev % 256) return lf_fail(LF_EWORKSPACE, "workspace must be 256-byte aligned");
  drop_graph(b);
  b->ws = (char*)dev;
  b->inited = false;
  return LF_OK;
}

lf_status lf_batch_set_band(lf_batch* b, int idx, int rows) {
  if (!b || rows < 0 || rows > 4096 || idx < -1 || idx >= b->n)
    return lf_fail(LF_EINVAL, "bad band setting");
  for (int k = 0; k < b->n; ++k)
    if (idx < 0 || idx == k) b->cav[k].band = rows;
  return b->inited ? upload_tables(b) : LF_OK;
}

static lf_status init_impl(lf_batch* b, const double* const* T0, const double* const* u0,
                           const double* const* v0, bool on_device) {
  if (!b) return lf_fail(LF_EINVAL, "NULL batch");
  if (!b->ws) return lf_fail(LF_EWORKSPACE, "no workspace bound");
  hipStream_t s = b->ctx->stream;
  double* st = (double*)(b->ws + b->off_stage);
  for (int k = 0; k < b->n; ++k) {
    Cav& c = b->cav[k];
    const size_t n = (size_t)c.nx * c.ny;
    const double* dT = nullptr; const double* du = nullptr; const double* dv = nullptr;
    if (on_device) {
      dT = T0 ? T0[k] : nullptr;
      du = u0 ? u0[k] : nullptr;
      dv = v0 ? v0[k] : nullptr;
    } else {
      if (T0 && T0[k]) { LF_HIP_TRY(hipMemcpyAsync(st, T0[k], n * 8, hipMemcpyHostToDevice, s)); dT = st; }
      if (u0 && u0[k]) { LF_HIP_TRY(hipMemcpyAsync(st + n, u0[k], n * 8, hipMemcpyHostToDevice, s)); du = st + n; }
      if (v0 && v0[k]) { LF_HIP_TRY(hipMemcpyAsync(st + 2 * n, v0[k], n * 8, hipMemcpyHostToDevice, s)); dv = st + 2 * n; }
    }
    lf::Grid g;
    g.nx = c.nx;
    g.ny = c.ny;
    g.pitch = c.pitch;
    g.plane = c.plane;
    if (b->precision == LF_F32)
      LF_HIP_TRY(lf::launch_init<float>(g, dT, du, dv, (float*)(b->ws + c.off_f[0]),
                                        (float*)(b->ws + c.off_T[0]), (float*)(b->ws + c.off_mom),
                                        (float*)(b->ws + c.off_snap),
                                        b->tcomp ? (lf::tlo_t*)(b->ws + c.off_Tlo[0]) : nullptr, s));
    else
      LF_HIP_TRY(lf::launch_init<double>(g, dT, du, dv, (double*)(b->ws + c.off_f[0]),
                                         (double*)(b->ws + c.off_T[0]),
                                         (double*)(b->ws + c.off_mom),
                                         (double*)(b->ws + c.off_snap), nullptr, s));
    // staging is reused for the next cavity: wait for this one
    if (!on_device) LF_HIP_TRY(hipStreamSynchronize(s));
    c.cur = 0;
    c.active = true;
    c.steps = 0;
    c.rule = 0;
    c.hist.clear();
  }
  b->inited = true;
  return upload_tables(b);
}

lf_status lf_batch_init(lf_batch* b, const double* const* T0, const double* const* u0,
                        const double* const* v0) {
  return init_impl(b, T0, u0, v0, false);
}

lf_status lf_batch_init_device(lf_batch* b, const double* const* T0, const double* const* u0,
                               const double* const* v0) {
  return init_impl(b, T0, u0, v0, true);
}

lf_status lf_batch_step(lf_batch* b, int64_t nsteps) {
  if (!b) return lf_fail(LF_EINVAL, "NULL batch");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  if (nsteps <= 0) return nsteps == 0 ? LF_OK : lf_fail(LF_EINVAL, "nsteps < 0");
  LF_HIP_TRY(enqueue_steps_any(b, 0, nsteps, true));
  for (auto& c : b->cav)
    if (c.active) {
      c.steps += nsteps;
      c.cur ^= (int)(nsteps & 1);
    }
  return (nsteps & 1) ? upload_tables(b) : LF_OK;
}

lf_status lf_batch_residual(lf_batch* b, double* r3n) {
  if (!b || !r3n) return lf_fail(LF_EINVAL, "NULL argument");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  LF_HIP_TRY(enqueue_residual_any(b));
  std::vector<double> h((size_t)8 * b->n);
  hipStream_t s = b->ctx->stream;
  LF_HIP_TRY(hipMemcpyAsync(h.data(), b->ws + b->off_out, h.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
  LF_HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < b->n; ++k) {
    if (!b->cav[k].active) continue;
    residual_of(&h[8 * k], &r3n[3 * k]);
    if (h[8 * k + 6] != 0.0) return lf_fail(LF_EDIVERGED, "cavity %d has non-finite values", k);
  }
  return LF_OK;
}

lf_status lf_batch_run_to_steady(lf_batch* b, double tol, int check_every, int64_t max_steps,
                                 int64_t* steps_each, int* rule_each, double* r_each) {
  if (!b) return lf_fail(LF_EINVAL, "NULL batch");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  if (!(tol > 0.0) || check_every < 2 || (check_every & 1) || max_steps < 0)
    return lf_fail(LF_EINVAL, "tol > 0 and an even check_every >= 2 are required");
  hipStream_t s = b->ctx->stream;
  // cavities stopped by an earlier call's step limit (rule 0) resume while
  // under this call's limit; converged or diverged ones stay stopped
  bool resumed = false;
  for (auto& c : b->cav)
    if (!c.active && c.rule == 0 && c.steps < max_steps) {
      c.active = true;
      resumed = true;
    }
  if (resumed) {
    lf_status su = upload_tables(b);
    if (su != LF_OK) return su;
  }
  // snapshot the live cavities, then replay "K steps + residual"
  LF_HIP_TRY(enqueue_residual_any(b));
  lf_status st = ensure_graph(b, check_every);
  if (st != LF_OK) return st;
  std::vector<double> h((size_t)8 * b->n);
  lf_status result = LF_OK;
  for (;;) {
    bool any = false;
    for (const auto& c : b->cav) any = any || c.active;
    if (!any) break;
    LF_HIP_TRY(hipGraphLaunch(b->gexec, s));
    LF_HIP_TRY(hipMemcpyAsync(h.data(), b->ws + b->off_out, h.size() * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    LF_HIP_TRY(hipStreamSynchronize(s));
    bool changed = false;
    for (int k = 0; k < b->n; ++k) {
      Cav& c = b->cav[k];
      if (!c.active) continue;
      c.steps += check_every;
      residual_of(&h[8 * k], c.r);
      const double m = fmax(c.r[0], fmax(c.r[1], c.r[2]));
      c.hist.push_back(m);
      if (h[8 * k + 6] != 0.0) {
        c.active = false;
        c.rule = -1;
        changed = true;
        result = lf_fail(LF_EDIVERGED, "cavity %d diverged after %lld steps", k,
                         (long long)c.steps);
        continue;
      }
      int fired = 0;
      if (m <= tol || (c.r[0] == 0.0 && c.r[1] == 0.0 && c.r[2] == 0.0)) fired = LF_STOP_TOL;
      else if (b->precision == LF_F32 &&
               lf_at_floor(c.hist, lf_slow_mode(c.prm[3], c.prm[1], c.nx, c.ny, c.tfix, 0, 0,
                                                check_every)))
        fired = LF_STOP_FLOOR;
      if (fired || c.steps >= max_steps) {
        c.active = false;
        c.rule = fired;
        changed = true;
        if (!fired && result == LF_OK)
          result = lf_fail(LF_ENOTCONV, "cavity %d: max residual %.3g after %lld steps", k, m,
                           (long long)c.steps);
      }
    }
    if (changed) {
      st = upload_tables(b);
      if (st != LF_OK) return st;
      // the live set's rows per tile may have changed the step kernel's form
      st = ensure_graph(b, check_every);
      if (st != LF_OK) return st;
    }
  }
  for (int k = 0; k < b->n; ++k) {
    if (steps_each) steps_each[k] = b->cav[k].steps;
    if (rule_each) rule_each[k] = b->cav[k].rule;
    if (r_each) memcpy(&r_each[3 * k], b->cav[k].r, 3 * sizeof(double));
  }
  return result;
}

lf_status lf_batch_reactivate(lf_batch* b) {
  if (!b || !b->inited) return lf_fail(LF_ESTATE, "init first");
  for (auto& c : b->cav) {
    c.active = true;
    c.rule = 0;
    c.hist.clear();
  }
  return upload_tables(b);
}

lf_status lf_batch_get_params(const lf_batch* b, int idx, double out[8]) {
  if (!b || !out || idx < 0 || idx >= b->n) return lf_fail(LF_EINVAL, "bad arguments");
  memcpy(out, b->cav[idx].prm, sizeof(b->cav[idx].prm));
  return LF_OK;
}

lf_status lf_batch_steps(const lf_batch* b, int idx, int64_t* steps) {
  if (!b || !steps || idx < 0 || idx >= b->n) return lf_fail(LF_EINVAL, "bad arguments");
  *steps = b->cav[idx].steps;
  return LF_OK;
}

lf_status lf_batch_nusselt(lf_batch* b, int idx, lf_nusselt* out) {
  if (!b || !out || idx < 0 || idx >= b->n) return lf_fail(LF_EINVAL, "bad arguments");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  const Cav& c = b->cav[idx];
  lf::Grid g;
  g.nx = c.nx;
  g.ny = c.ny;
  g.pitch = c.pitch;
  g.plane = c.plane;
  lf::WallSet w;
  memset(&w, 0, sizeof(w));
  for (int s = 0; s < 4; ++s) {
    w.tfix[s] = c.tfix[s];
    w.Tw[s] = c.Tw[s];
  }
  hipStream_t s = b->ctx->stream;
  double* dout = (double*)(b->ws + b->off_stage);
  if (b->precision == LF_F32)
    LF_HIP_TRY(lf::launch_nusselt<float>(g, w, (float*)(b->ws + c.off_T[c.cur]), dout, s));
  else
    LF_HIP_TRY(lf::launch_nusselt<double>(g, w, (double*)(b->ws + c.off_T[c.cur]), dout, s));
  double h[8];
  LF_HIP_TRY(hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, s));
  LF_HIP_TRY(hipStreamSynchronize(s));
  out->nu_hot = h[0]; out->nu_cold = h[1]; out->nu_hot_max = h[2]; out->y_hot_max = h[3];
  out->nu_cold_max = h[4]; out->y_cold_max = h[5]; out->nu_hot_o2 = h[6]; out->nu_cold_o2 = h[7];
  return LF_OK;
}

lf_status lf_batch_fetch(lf_batch* b, int idx, int field, void* dst, size_t dst_bytes,
                         int dst_is_device, int as_f64) {
  if (!b || !dst || idx < 0 || idx >= b->n) return lf_fail(LF_EINVAL, "bad arguments");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  const Cav& c = b->cav[idx];
  const size_t n = (size_t)c.nx * c.ny;
  const size_t need = n * (as_f64 ? 8 : b->es);
  if (dst_bytes < need) return lf_fail(LF_EINVAL, "dst holds %zu bytes, %zu needed", dst_bytes, need);
  const size_t pb = lf_align_up((size_t)c.plane * b->es, 256);
  size_t off;
  switch (field) {
    case LF_FIELD_RHO: case LF_FIELD_P: off = c.off_mom; break;
    case LF_FIELD_U: off = c.off_mom + pb; break;
    case LF_FIELD_V: off = c.off_mom + 2 * pb; break;
    case LF_FIELD_T: off = c.off_T[c.cur]; break;
    default: return lf_fail(LF_EINVAL, "bad field %d", field);
  }
  lf::Grid g;
  g.nx = c.nx;
  g.ny = c.ny;
  g.pitch = c.pitch;
  g.plane = c.plane;
  hipStream_t s = b->ctx->stream;
  void* target = dst_is_device ? dst : (void*)(b->ws + b->off_stage);
  const int pressure = field == LF_FIELD_P ? 1 : 0;
  if (b->precision == LF_F32)
    LF_HIP_TRY(lf::launch_unpack<float>(g, (float*)(b->ws + off), target, as_f64, s, pressure));
  else
    LF_HIP_TRY(lf::launch_unpack<double>(g, (double*)(b->ws + off), target, as_f64, s, pressure));
  if (!dst_is_device) {
    LF_HIP_TRY(hipMemcpyAsync(dst, target, need, hipMemcpyDeviceToHost, s));
    LF_HIP_TRY(hipStreamSynchronize(s));
  }
  return LF_OK;
}

lf_status lf_batch_profile_steps(lf_batch* b, int64_t nsteps, double* avg_ms) {
  if (!b || !avg_ms || nsteps < 2 || (nsteps & 1)) return lf_fail(LF_EINVAL, "even nsteps >= 2");
  if (!b->inited) return lf_fail(LF_ESTATE, "init first");
  hipStream_t s = b->ctx->stream;
  hipEvent_t e0, e1;
  LF_HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return lf_fail(LF_EDEVICE, "hipEventCreate");
  }
  hipError_t e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = enqueue_steps_any(b, 0, nsteps, true);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return lf_fail(LF_EDEVICE, "profile: %s", hipGetErrorString(e));
  for (auto& c : b->cav)
    if (c.active) c.steps += nsteps;
  *avg_ms = ms / (double)nsteps;
  return LF_OK;
}

// ---- autotuner -------------------------------------------------------------
// For each cavity-height class (aspect 2), time the batched step with band
// heights 1, 2, 4, 8, 16 on a batch of copies filling about 8 M nodes of the
// caller's scratch buffer, keep the fastest, and cache the table as JSON
// keyed by architecture and precision.  An existing cache is loaded instead.
static bool load_tuning(lf_ctx* ctx, const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char buf[4096];
  size_t n = fread(buf, 1, sizeof(buf) - 1, f);
  fclose(f);
  buf[n] = 0;
  if (!strstr(buf, "\"arch\": \"gfx950\"") || !strstr(buf, "\"precision\": \"f32\"")) return false;
  const char* p = strstr(buf, "\"bands\"");
  if (!p) return false;
  lf_tuning t;
  memset(&t, 0, sizeof(t));
  p = strchr(p, '{');
  while (p && t.nclass < 16) {
    const char* q = strchr(p, '"');
    if (!q) break;
    int ny = 0, band = 0;
    if (sscanf(q, "\"%d\": %d", &ny, &band) != 2) break;
    t.ny_class[t.nclass] = ny;
    t.band[t.nclass] = band;
    t.nclass++;
    p = strchr(q + 1, ',');
  }
  if (t.nclass == 0) return false;
  t.valid = 1;
  ctx->tune = t;
  return true;
}

lf_status lf_autotune(lf_ctx* ctx, const char* cache_path, int budget_ms, void* dev_scratch,
                      size_t scratch_bytes) {
  if (!ctx) return lf_fail(LF_EINVAL, "NULL ctx");
  if (cache_path && load_tuning(ctx, cache_path)) return LF_OK;
  if (!dev_scratch) return lf_fail(LF_EWORKSPACE, "no cache at %s and no scratch buffer",
                                   cache_path ? cache_path : "(null)");
  const int classes[7] = {64, 96, 128, 192, 256, 384, 512};
  const int bands[5] = {1, 2, 4, 8, 16};
  lf_tuning t;
  memset(&t, 0, sizeof(t));
  const int per_class_ms = budget_ms > 0 ? budget_ms / 7 : 200;
  for (int ci = 0; ci < 7; ++ci) {
    const int ny = classes[ci], nx = 2 * ny;
    int m = (int)(8000000LL / ((long long)nx * ny));
    if (m < 1) m = 1;
    std::vector<lf_case_desc> d(m);
    std::vector<lf_physics> ph(m);
    for (int k = 0; k < m; ++k) {
      d[k].nx = nx; d[k].ny = ny; d[k].precision = LF_F32; d[k].mode = LF_MODE_HYBRID;
      d[k].split_col = 0; d[k].overlap = 0; d[k].iface = 0; d[k].tcomp = 1;
      ph[k].Ra = 1e5; ph[k].Pr = 0.71; ph[k].U_char = 0.0; ph[k].T_ref = NAN;
      ph[k].conv = LF_CONV_QUICK; ph[k].body_gx = 0.0; ph[k].body_gy = 0.0;
    }
    lf_batch* b = nullptr;
    lf_status st = lf_batch_create(ctx, m, d.data(), ph.data(), nullptr, &b);
    if (st != LF_OK) return st;
    while (m > 1 && b->need > scratch_bytes) {  // shrink to the scratch
      lf_batch_destroy(b);
      m /= 2;
      st = lf_batch_create(ctx, m, d.data(), ph.data(), nullptr, &b);
      if (st != LF_OK) return st;
    }
    if (b->need > scratch_bytes) {
      lf_batch_destroy(b);
      return lf_fail(LF_EWORKSPACE, "scratch too small for a %dx%d cavity", nx, ny);
    }
    st = lf_batch_bind_workspace(b, dev_scratch, scratch_bytes);
    if (st == LF_OK) st = lf_batch_init(b, nullptr, nullptr, nullptr);
    double best = 1e300;
    int best_band = 4;
    for (int bi = 0; bi < 5 && st == LF_OK; ++bi) {
      st = lf_batch_set_band(b, -1, bands[bi]);
      double ms = 0.0;
      if (st == LF_OK) st = lf_batch_profile_steps(b, 4, &ms);  // warm-up
      if (st == LF_OK) {
        int reps = (int)(per_class_ms / 5 / (ms > 1e-3 ? ms : 1e-3));
        reps = reps < 10 ? 10 : (reps > 400 ? 400 : reps);
        reps += reps & 1;
        st = lf_batch_profile_steps(b, reps, &ms);
      }
      if (st == LF_OK && ms < best) {
        best = ms;
        best_band = bands[bi];
      }
    }
    lf_batch_destroy(b);
    if (st != LF_OK) return st;
    t.ny_class[ci] = ny;
    t.band[ci] = best_band;
  }
  t.nclass = 7;
  t.valid = 1;
  ctx->tune = t;
  if (cache_path) {
    FILE* f = fopen(cache_path, "w");
    if (!f) return lf_fail(LF_EINVAL, "cannot write %s", cache_path);
    fprintf(f, "{\"arch\": \"gfx950\", \"precision\": \"f32\", \"mode\": \"hybrid\", \"bands\": {");
    for (int k = 0; k < t.nclass; ++k)
      fprintf(f, "%s\"%d\": %d", k ? ", " : "", t.ny_class[k], t.band[k]);
    fprintf(f, "}}\n");
    fclose(f);
  }
  return LF_OK;
}

lf_status lf_ctx_get_tuning(const lf_ctx* ctx, int* nclass, int ny_class[16], int band[16]) {
  if (!ctx || !nclass) return lf_fail(LF_EINVAL, "NULL argument");
  *nclass = ctx->tune.valid ? ctx->tune.nclass : 0;
  for (int k = 0; k < *nclass; ++k) {
    if (ny_class) ny_class[k] = ctx->tune.ny_class[k];
    if (band) band[k] = ctx->tune.band[k];
  }
  return LF_OK;
}

}  // extern "C"
