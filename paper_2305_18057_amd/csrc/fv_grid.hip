// Grid API of the C ABI: one instance in a caller-supplied workspace.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "fv_grid_impl.h"

using namespace fvrt;

namespace fvgrid {

int upload_tiles(fv_grid* g) {
  build_tiles(g->hg, g->shape, 0, 0, g->htiles);
  const int nt = (int)g->htiles.size();
  if (nt > g->L.max_tiles) return set_error(FV_E_INVAL, "tile list exceeds its capacity");
  FV_HIP(hipMemcpyAsync(g->d_tiles, g->htiles.data(), sizeof(fvk::DevTile) * nt,
                        hipMemcpyHostToDevice, g->stream));
  FV_HIP(hipMemcpyAsync(g->d_ntiles, &nt, sizeof(int), hipMemcpyHostToDevice, g->stream));
  // the instance's tile count sizes its partials (value-major) and their
  // reductions: it follows the tile list at once, on the host and the device
  g->hinst.ntiles = nt;
  FV_HIP(hipMemcpyAsync((char*)g->d_inst + offsetof(fvk::DevInstance, ntiles), &g->hinst.ntiles,
                        sizeof(int), hipMemcpyHostToDevice, g->stream));
  g->plan = fvexec::StepPlan();
  g->plan.blocks = g->d_blocks;
  g->plan.insts = g->d_inst;
  g->plan.active = nullptr;
  g->plan.ninst = 1;
  fvexec::LaunchSet ls;
  ls.tiles = g->d_tiles;
  ls.ntiles_dev = g->d_ntiles;
  ls.ntiles = nt;
  // graphs are captured again after every change of the tile list (below)
  ls.count_fixed = true;
  ls.kind = fvexec::set_kind(g->hg.ndim, g->hg.gen3, g->shape.ny);
  g->plan.sets.push_back(ls);
  g->graphs.clear();
  // the tile list and the instance's tile count must be on the device before
  // the next launch; the caller's stream orders that
  FV_HIP(hipStreamSynchronize(g->stream));
  return FV_OK;
}

int put_inst(fv_grid* g, bool whole) {
  const size_t n = whole ? sizeof(fvk::DevInstance) : offsetof(fvk::DevInstance, t);
  FV_HIP(hipMemcpyAsync(g->d_inst, &g->hinst, n, hipMemcpyHostToDevice, g->stream));
  return FV_OK;
}

int get_inst(fv_grid* g) {
  FV_HIP(hipMemcpyAsync(&g->hinst, g->d_inst, sizeof(fvk::DevInstance), hipMemcpyDeviceToHost,
                        g->stream));
  FV_HIP(hipStreamSynchronize(g->stream));
  return FV_OK;
}

void fill_info(const fv_grid* g, fv_step_info* info) {
  if (!info) return;
  const fvk::DevInstance& I = g->hinst;
  info->steps = I.steps;
  info->t = I.t;
  info->dt_last = I.dt_last;
  for (int v = 0; v < 5; ++v) info->norms[v] = I.norms[v];
  info->norm = I.norm;
  info->drop = I.drop;
  info->flags = I.flags;
}

int cfl_pass(fv_grid* g) {
  const int err = fvexec::enqueue_cfl(g->plan, g->stream);
  if (err) return err;
  FV_HIP(fvk::launch_cfl_init(g->stream, g->d_inst, nullptr, 1));
  g->cfl_mu = g->hinst.mu;
  g->cfl_pr = g->hinst.prandtl;
  return get_inst(g);
}

// 2D grids run the Navier-Stokes stage kernel for a viscosity, a no-slip
// face or a source term
bool ns_kernel(const HostGrid& hg, const fv_params* p) {
  return hg.ndim == 2 && (p->mu > 0.0 || hg.has_noslip || hg.with_source);
}

// The stage kernels these parameters take: a viscosity or a no-slip face
// needs the Navier-Stokes kernel (2D grids).  Called after the parameters
// are on the device; when the viscosity differs from the one the current
// time-step bound was formed with, the bound is formed again.
int use_params(fv_grid* g, const fv_params* p) {
  if (p->mu > 0.0 && g->hg.ndim != 2)
    return set_error(FV_E_UNSUPPORTED, "the viscous flux is provided for 2D grids only");
  g->plan.ns = ns_kernel(g->hg, p);
  if (g->have_state && (g->hinst.mu != g->cfl_mu || g->hinst.prandtl != g->cfl_pr)) {
    const int st = cfl_pass(g);
    if (st) return st;
  }
  return FV_OK;
}

}  // namespace fvgrid

using namespace fvgrid;

extern "C" size_t fv_grid_workspace_bytes(const fv_grid_desc* desc, int precision) {
  (void)precision;
  HostGrid hg;
  if (validate_and_copy(desc, hg) != FV_OK) return 0;
  return layout_of(hg).total;
}

extern "C" int fv_create_grid(const fv_grid_desc* desc, void* d_workspace, size_t bytes,
                              void* hip_stream, fv_grid** out) {
  if (!out) return set_error(FV_E_INVAL, "null output handle");
  *out = nullptr;
  HostGrid hg;
  const int st = validate_and_copy(desc, hg);
  if (st) return st;
  return fvgrid::create(std::move(hg), d_workspace, bytes, hip_stream, out);
}

int fvgrid::create(HostGrid&& hg, void* d_workspace, size_t bytes, void* hip_stream, fv_grid** out) {
  *out = nullptr;
  fv_grid* g = new (std::nothrow) fv_grid();
  if (!g) return set_error(FV_E_NOMEM, "host allocation failed");
  g->hg = std::move(hg);
  int st = FV_OK;
  g->L = layout_of(g->hg);
  if (!d_workspace || bytes < g->L.total) {
    const size_t need = g->L.total;
    delete g;
    return set_error(FV_E_NOMEM, "workspace of %zu bytes, need %zu", bytes, need);
  }
  if (((uintptr_t)d_workspace) % kAlign) {
    delete g;
    return set_error(FV_E_INVAL, "workspace must be %zu-byte aligned", kAlign);
  }
  g->stream = (hipStream_t)hip_stream;
  g->ws = (char*)d_workspace;
  g->ws_bytes = bytes;
  g->d_blocks = (fvk::DevBlock*)(g->ws + g->L.blocks);
  g->d_inst = (fvk::DevInstance*)(g->ws + g->L.inst);
  g->d_ntiles = (int*)(g->ws + g->L.ntiles);
  g->d_tiles = (fvk::DevTile*)(g->ws + g->L.tiles);
  g->d_part = (double*)(g->ws + g->L.part);
  g->d_segs = (fvk::GhostSeg*)(g->ws + g->L.segs);
  for (int s = 0; s < 3; ++s) g->d_u[s] = (double*)(g->ws + g->L.u[s]);

  build_blocks(g->hg, g->ws, g->L, 0, g->hblocks, 0);
  std::vector<fvk::GhostSeg> segs;
  build_segs(g->hg, segs);
  auto fail = [&](int e) {
    delete g;
    return e;
  };
  hipError_t he = hipMemcpyAsync(g->d_blocks, g->hblocks.data(),
                                 sizeof(fvk::DevBlock) * g->hblocks.size(), hipMemcpyHostToDevice,
                                 g->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(g->d_segs, segs.data(), sizeof(fvk::GhostSeg) * segs.size(),
                        hipMemcpyHostToDevice, g->stream);
  if (he != hipSuccess)
    return fail(set_error(FV_E_DEVICE, "upload of block descriptors failed: %s", hipGetErrorString(he)));
  // node coordinates; the source starts at zero
  he = upload_nodes(g->hg, g->ws + g->L.nodes, g->stream);
  if (he != hipSuccess)
    return fail(set_error(FV_E_DEVICE, "upload of node coordinates failed: %s", hipGetErrorString(he)));
  if (g->hg.with_source) {
    he = hipMemsetAsync(g->ws + g->L.src, 0, sizeof(double) * (size_t)g->hg.state_size, g->stream);
    if (he != hipSuccess)
      return fail(set_error(FV_E_DEVICE, "clearing the source failed: %s", hipGetErrorString(he)));
  }
  std::memset(&g->hinst, 0, sizeof(g->hinst));
  fv_params p;
  fv_default_params(&p);
  params_to_inst(&p, g->hg.gamma, g->hinst);
  g->hinst.ndim = g->hg.ndim;
  g->hinst.nv = g->hg.nv;
  g->hinst.ncells = g->hg.compute_cells();
  g->hinst.part = g->d_part;
  g->hinst.step_limit = 0;
  g->hinst.stopped = 1;
  g->hinst.flags = fvk::FLAG_NONPHYS;  // no state yet
  // tile shape: autotune table for this size class, else the default
  TileShape sh = default_shape(g->hg);
  const char* tp = tune_path(nullptr);
  TileShape tsh;
  if (tune_lookup(tp, tune_key(g->hg, FV_FP64), tsh)) sh = tsh;
  g->shape = sh;
  st = fvgrid::upload_tiles(g);
  if (st) return fail(st);
  st = fvgrid::put_inst(g, true);
  if (st) return fail(st);
  he = hipStreamSynchronize(g->stream);
  if (he != hipSuccess)
    return fail(set_error(FV_E_DEVICE, "stream synchronisation failed: %s", hipGetErrorString(he)));
  *out = g;
  return FV_OK;
}

extern "C" int fv_destroy_grid(fv_grid* g) {
  if (!g) return FV_E_INVAL;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  g->graphs.clear();
  delete g;
  return FV_OK;
}

extern "C" int fv_set_state(fv_grid* g, const double* U, int on_device) {
  if (!g || !U) return set_error(FV_E_INVAL, "null argument");
  FV_HIP(hipMemcpyAsync(g->d_u[0], U, sizeof(double) * g->hg.state_size,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, g->stream));
  fvk::DevInstance& I = g->hinst;
  I.t = I.dt = I.dt_last = I.raw_min = I.norm_first = I.norm = I.drop = 0.0;
  for (int v = 0; v < 5; ++v) I.norms[v] = I.rnorms[v] = 0.0;
  I.steps = 0;
  I.flags = 0;
  I.stopped = 0;
  I.have_first = 0;
  I.last_step = 0;
  int st = put_inst(g, true);
  if (st) return st;
  st = cfl_pass(g);
  if (st) return st;
  g->have_state = 1;
  if (g->hinst.flags & fvk::FLAG_NONPHYS)
    return set_error(FV_E_NONPHYSICAL, "initial state has a cell with rho <= 0, p <= 0 or a non-finite value");
  return FV_OK;
}

extern "C" int fv_set_source(fv_grid* g, const double* S, int on_device) {
  if (!g) return set_error(FV_E_INVAL, "null grid");
  if (!g->hg.with_source)
    return set_error(FV_E_INVAL, "the grid was created without a source buffer (with_source = 0)");
  const size_t bytes = sizeof(double) * (size_t)g->hg.state_size;
  if (S)
    FV_HIP(hipMemcpyAsync(g->ws + g->L.src, S, bytes,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, g->stream));
  else
    FV_HIP(hipMemsetAsync(g->ws + g->L.src, 0, bytes, g->stream));
  FV_HIP(hipStreamSynchronize(g->stream));
  return FV_OK;
}

extern "C" int fv_get_state(const fv_grid* gc, double* U, int on_device) {
  fv_grid* g = const_cast<fv_grid*>(gc);
  if (!g || !U) return set_error(FV_E_INVAL, "null argument");
  FV_HIP(hipMemcpyAsync(U, g->d_u[0], sizeof(double) * g->hg.state_size,
                        on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream));
  FV_HIP(hipStreamSynchronize(g->stream));
  return FV_OK;
}

extern "C" int fv_residual(fv_grid* g, const fv_params* p, double* R, int on_device,
                           double norms[5]) {
  if (!g) return set_error(FV_E_INVAL, "null grid");
  int st = check_params(p);
  if (st) return st;
  if (!g->have_state) return set_error(FV_E_INVAL, "no state set");
  params_to_inst(p, g->hg.gamma, g->hinst);
  st = put_inst(g, false);
  if (st) return st;
  if ((st = use_params(g, p))) return st;
  double* dst = (R && on_device) ? R : g->d_u[1];
  g->plan.lim = p->limiter;
  st = fvexec::enqueue_stage(g->plan, 0, p->precision == FV_FP32_FLUX, dst, g->stream);
  if (st) return st;
  FV_HIP(fvk::launch_rnorms(g->stream, g->d_inst, nullptr, 1));
  if (R && !on_device)
    FV_HIP(hipMemcpyAsync(R, g->d_u[1], sizeof(double) * g->hg.state_size, hipMemcpyDeviceToHost,
                          g->stream));
  st = get_inst(g);
  if (st) return st;
  if (norms)
    for (int v = 0; v < 5; ++v) norms[v] = g->hinst.rnorms[v];
  return FV_OK;
}

extern "C" size_t fv_ghost_count(const fv_grid* g) { return g ? (size_t)g->L.ghost_doubles : 0; }

extern "C" int fv_ghosts(fv_grid* g, double* G, int on_device) {
  if (!g || !G) return set_error(FV_E_INVAL, "null argument");
  if (!g->have_state) return set_error(FV_E_INVAL, "no state set");
  double* dst = G;
  if (!on_device) {
    if (g->L.ghost_doubles > g->hg.state_size)
      return set_error(FV_E_NOMEM, "ghost dump larger than a state buffer: pass a device buffer");
    dst = g->d_u[2];
  }
  FV_HIP(fvk::launch_ghosts(g->stream, g->d_blocks, g->d_segs, g->L.nseg, g->L.ghost_cells,
                            g->hg.nv, dst));
  if (!on_device)
    FV_HIP(hipMemcpyAsync(G, dst, sizeof(double) * g->L.ghost_doubles, hipMemcpyDeviceToHost,
                          g->stream));
  FV_HIP(hipStreamSynchronize(g->stream));
  return FV_OK;
}

static int run_steps(fv_grid* g, const fv_params* p, long long nsteps, double drop_tol,
                     fv_step_info* info) {
  if (!g) return set_error(FV_E_INVAL, "null grid");
  int st = check_params(p);
  if (st) return st;
  if (!g->have_state) return set_error(FV_E_INVAL, "no state set");
  if (nsteps < 0) return set_error(FV_E_INVAL, "negative step count");
  params_to_inst(p, g->hg.gamma, g->hinst);
  g->hinst.drop_tol = drop_tol;
  g->hinst.step_limit = g->hinst.steps + nsteps;
  st = put_inst(g, false);
  if (st) return st;
  if ((st = use_params(g, p))) return st;
  FV_HIP(fvk::launch_prepare(g->stream, g->d_inst, nullptr, 1));
  const int fp32 = p->precision == FV_FP32_FLUX;
  g->plan.rk = fvrt::rk_of(p);
  g->plan.lim = p->limiter;
  const int chunk = fvexec::graph_chunk();
  long long left = nsteps;
  long long since_check = 0;
  const bool check = drop_tol > 0.0;
  while (left > 0) {
    const int c = (int)std::min<long long>(left, chunk);
    st = fvexec::enqueue_steps(g->plan, fp32, c, g->stream, &g->graphs);
    if (st) return st;
    left -= c;
    since_check += c;
    if (check && since_check >= 4LL * chunk && left > 0) {
      since_check = 0;
      st = get_inst(g);
      if (st) return st;
      if (g->hinst.stopped) break;
    }
  }
  st = get_inst(g);
  if (st) return st;
  fill_info(g, info);
  if (g->hinst.flags & fvk::FLAG_NONPHYS)
    return set_error(FV_E_NONPHYSICAL, "state turned non-physical after %lld steps", g->hinst.steps);
  return FV_OK;
}

extern "C" int fv_step(fv_grid* g, const fv_params* p, int nsteps, fv_step_info* info) {
  return run_steps(g, p, nsteps, 0.0, info);
}

extern "C" int fv_step_timed(fv_grid* g, const fv_params* p, int nsteps, fv_step_info* info,
                             double stage_ms[4]) {
  if (!g || !stage_ms) return set_error(FV_E_INVAL, "null argument");
  int st = check_params(p);
  if (st) return st;
  if (fvrt::rk_of(p) != 3) return set_error(FV_E_UNSUPPORTED, "per-stage timing is for SSP-RK3 (rk = 3)");
  g->plan.rk = 3;
  g->plan.lim = p->limiter;
  if (!g->have_state) return set_error(FV_E_INVAL, "no state set");
  if (nsteps < 0) return set_error(FV_E_INVAL, "negative step count");
  params_to_inst(p, g->hg.gamma, g->hinst);
  g->hinst.drop_tol = 0.0;
  g->hinst.step_limit = g->hinst.steps + nsteps;
  st = put_inst(g, false);
  if (st) return st;
  if ((st = use_params(g, p))) return st;
  FV_HIP(fvk::launch_prepare(g->stream, g->d_inst, nullptr, 1));
  const int fp32 = p->precision == FV_FP32_FLUX;
  // the events are released on every return path
  struct Events {
    std::vector<hipEvent_t> v;
    ~Events() {
      for (auto& e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } evs;
  evs.v.assign(5 * (size_t)std::max(nsteps, 1), nullptr);
  std::vector<hipEvent_t>& ev = evs.v;
  for (auto& e : ev) FV_HIP(hipEventCreate(&e));
  for (int k = 0; k < nsteps; ++k) {
    hipEvent_t* E = &ev[5 * (size_t)k];
    FV_HIP(hipEventRecord(E[0], g->stream));
    for (int m = 1; m <= 3; ++m) {
      st = fvexec::enqueue_stage(g->plan, m, fp32, nullptr, g->stream);
      if (st) break;
      FV_HIP(hipEventRecord(E[m], g->stream));
    }
    if (st) break;
    FV_HIP(fvk::launch_finalize(g->stream, g->d_inst, nullptr, 1));
    FV_HIP(hipEventRecord(E[4], g->stream));
  }
  if (!st) {
    FV_HIP(hipStreamSynchronize(g->stream));
    for (int s = 0; s < 4; ++s) stage_ms[s] = 0.0;
    for (int k = 0; k < nsteps; ++k)
      for (int s = 0; s < 4; ++s) {
        float ms = 0.f;
        FV_HIP(hipEventElapsedTime(&ms, ev[5 * (size_t)k + s], ev[5 * (size_t)k + s + 1]));
        stage_ms[s] += ms;
      }
    for (int s = 0; s < 4; ++s) g->last_ms[s] = stage_ms[s];
  }
  if (st) return st;
  st = get_inst(g);
  if (st) return st;
  fill_info(g, info);
  if (g->hinst.flags & fvk::FLAG_NONPHYS)
    return set_error(FV_E_NONPHYSICAL, "state turned non-physical after %lld steps", g->hinst.steps);
  return FV_OK;
}

extern "C" int fv_solve(fv_grid* g, const fv_params* p, double drop_tol, long long max_steps,
                        fv_step_info* info) {
  if (!(drop_tol >= 0.0)) return set_error(FV_E_INVAL, "drop_tol must be >= 0");
  return run_steps(g, p, max_steps, drop_tol, info);
}

extern "C" int fv_grid_get_stats(const fv_grid* g, fv_grid_stats* out) {
  if (!g || !out) return set_error(FV_E_INVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->cells = g->hg.ncells;
  out->tiles = (long long)g->htiles.size();
  out->tile_rows = g->shape.rows;
  out->tile_cols = 64;
  out->tile_ny = g->hg.ndim == 3 ? g->shape.ny : 1;
  out->launch_blocks = g->plan.sets.empty() ? 0 : fvexec::launch_grid(g->plan.sets[0], 0);
  out->workspace_bytes = g->L.total;
  for (int s = 0; s < 4; ++s) out->last_stage_ms[s] = g->last_ms[s];
  return FV_OK;
}

// Candidate tile shapes of the grid's size class are timed on the device with
// the grid's own state (saved on the host and restored afterwards).
extern "C" int fv_tune(fv_grid* g, const fv_params* p, const char* cache_path) {
  if (!g) return set_error(FV_E_INVAL, "null grid");
  int st = check_params(p);
  if (st) return st;
  if (!g->have_state) return set_error(FV_E_INVAL, "no state set");
  // Navier-Stokes grids time (and record) the shapes of their own kernel
  if (p->mu > 0.0 && g->hg.ndim != 2)
    return set_error(FV_E_UNSUPPORTED, "the viscous flux is provided for 2D grids only");
  const bool tns = ns_kernel(g->hg, p);
  g->plan.ns = tns;
  {
    // a shape already recorded for this size class and precision is applied
    // as is; the state is untouched, only the per-tile minima are redone
    TileShape rec;
    if (tune_lookup(tune_path(cache_path), tune_key(g->hg, p->precision, tns), rec)) {
      if (rec.rows != g->shape.rows || rec.ny != g->shape.ny) {
        g->shape = rec;
        if ((st = upload_tiles(g))) return st;
        if ((st = cfl_pass(g))) return st;
      }
      return FV_OK;
    }
  }
  std::vector<double> saved((size_t)g->hg.state_size);
  st = fv_get_state(g, saved.data(), 0);
  if (st) return st;
  const fvk::DevInstance keep = g->hinst;
  std::vector<TileShape> cands;
  if (g->hg.ndim == 2) {
    for (int r : {2, 3, 4, 5, 6, 8, 12, 16, 32, 64}) {
      TileShape s;
      s.rows = r;
      s.ny = 1;
      cands.push_back(s);
    }
  } else if (g->hg.gen3) {
    for (int r : {4, 8, 12, 16, 24, 32, 48, 64}) {
      TileShape s;
      s.rows = r;
      s.ny = 4;
      cands.push_back(s);
    }
  } else {
    for (int y : {3, 7})
      for (int r : {8, 12, 16, 20, 24, 28, 32, 40, 48, 52, 56, 64}) {
        TileShape s;
        s.rows = r;
        s.ny = y;
        cands.push_back(s);
      }
  }
  const int fp32 = p->precision == FV_FP32_FLUX;
  const int rk = fvrt::rk_of(p);
  // the two timing events are released on every return path
  struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  FV_HIP(hipEventCreate(&ev.a));
  FV_HIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  // per-step time of one candidate: steps run as they do in fv_step (graphs
  // of the step sequence), from the saved state; a warm-up, then the best of
  // three batches (a single short batch is too noisy to separate shapes a few
  // per cent apart; the first batch also pays for capturing its graph).
  // Small grids take longer batches, whose per-step time matches long runs;
  // large grids take batches of at least about 8 ms.
  const int reps = g->hg.ncells < (1LL << 21) ? 64 : 8;
  auto time_shape = [&](const TileShape& c, double& per) -> int {
    g->shape = c;
    int e = upload_tiles(g);
    if (e) return e;
    // same starting state for every candidate (with this candidate's tiles)
    g->hinst = keep;
    g->hinst.ntiles = (int)g->htiles.size();
    params_to_inst(p, g->hg.gamma, g->hinst);
    g->hinst.step_limit = keep.steps + 1000000;
    g->hinst.drop_tol = 0.0;
    g->hinst.stopped = 0;
    g->hinst.flags = 0;
    g->plan.rk = rk;
    g->plan.lim = p->limiter;
    if ((e = put_inst(g, true))) return e;
    if ((e = fvexec::enqueue_steps(g->plan, fp32, reps, g->stream, &g->graphs))) return e;
    per = 1e30;
    for (int b = 0; b < 3 && !e; ++b) {
      FV_HIP(hipEventRecord(e0, g->stream));
      e = fvexec::enqueue_steps(g->plan, fp32, reps, g->stream, &g->graphs);
      FV_HIP(hipEventRecord(e1, g->stream));
      FV_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      FV_HIP(hipEventElapsedTime(&ms, e0, e1));
      per = std::min(per, (double)ms / reps);
    }
    FV_HIP(hipMemcpyAsync(g->d_u[0], saved.data(), sizeof(double) * saved.size(),
                          hipMemcpyHostToDevice, g->stream));
    return e;
  };
  // The GPU's clocks rise over tens of milliseconds of load: the first
  // candidate runs untimed for about 60 ms of steps before anything counts
  // (timed from idle, the first candidates would be measured on the ramp).
  for (int w = 0, done = 0; w < 32 && done < 60 && !st; ++w) {
    double per = 0.0;
    st = time_shape(cands[0], per);
    done += (int)(per * 4 * reps);
  }
  // pass 1 over every candidate; pass 2 times the three fastest again in the
  // reverse order (so that a drift of the clocks during tuning cancels) and
  // each keeps its better time
  std::vector<double> ms(cands.size(), 1e30);
  for (size_t c = 0; c < cands.size() && !st; ++c) st = time_shape(cands[c], ms[c]);
  std::vector<size_t> order(cands.size());
  for (size_t c = 0; c < order.size(); ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return ms[x] < ms[y]; });
  const size_t top = std::min<size_t>(3, order.size());
  for (size_t r = top; r-- > 0 && !st;) {
    double again = 1e30;
    st = time_shape(cands[order[r]], again);
    ms[order[r]] = std::min(ms[order[r]], again);
  }
  TileShape best = g->shape;
  double best_ms = 1e30;
  for (size_t c = 0; c < cands.size(); ++c)
    if (ms[c] < best_ms) {
      best_ms = ms[c];
      best = cands[c];
    }
  if (st) return st;
  g->shape = best;
  st = upload_tiles(g);
  if (st) return st;
  FV_HIP(hipMemcpyAsync(g->d_u[0], saved.data(), sizeof(double) * saved.size(),
                        hipMemcpyHostToDevice, g->stream));
  g->hinst = keep;
  g->hinst.ntiles = (int)g->htiles.size();
  st = put_inst(g, true);
  if (st) return st;
  // the per-tile spectral minima of the restored state
  st = cfl_pass(g);
  if (st) return st;
  g->hinst.steps = keep.steps;
  g->hinst.t = keep.t;
  tune_store(tune_path(cache_path), tune_key(g->hg, p->precision, tns), best, best_ms);
  return FV_OK;
}
