// Launch sequencing and hipGraph capture of RK steps.
#include "fv_exec.h"

#include <algorithm>
#include <cstdlib>

#include "fv_launch.h"
#include "fv_runtime.h"

namespace fvexec {

void GraphCache::clear() {
  for (auto& kv : m_)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  m_.clear();
}

int graph_chunk() {
  static int c = 0;
  if (c == 0) {
    const char* e = getenv("FV_GRAPH_STEPS");
    c = e ? std::max(1, atoi(e)) : 10;
  }
  return c;
}

static bool graphs_enabled() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("FV_NO_GRAPH");
    on = (e && e[0] == '1') ? 0 : 1;
  }
  return on == 1;
}

int launch_grid(const LaunchSet& s, int fp32, bool ns) {
  if (s.ntiles <= 0) return 0;
  int cap;
  if ((s.kind == kSet2D && ns) || s.kind == kSet2DNS) {
    // one 256-thread workgroup per tile
    cap = fvrt::occupancy_blocks(fvk::stage2d_ns_kernel_ptr(fp32), 256);
    cap = std::min(cap, s.ntiles);
  } else if (s.kind == kSet2D) {
    cap = fvrt::occupancy_blocks(fvk::stage2d_kernel_ptr(1, fp32), 256);
    const int need = (s.ntiles + 3) / 4;
    cap = std::min(cap, need);
  } else if (s.kind == kSet3DG) {
    cap = fvrt::occupancy_blocks(fvk::stage3d_gen_kernel_ptr(fp32), 256);
    cap = std::min(cap, s.ntiles);
  } else {
    const int ny = s.kind == kSet3D7 ? 7 : 3;
    cap = fvrt::occupancy_blocks(fvk::stage3d_kernel_ptr(1, fp32, ny), 64 * (ny + 1));
    cap = std::min(cap, s.ntiles);
  }
  if (s.max_grid > 0) cap = std::min(cap, s.max_grid);
  // a multiple of the XCD count, so that every XCD walks its own part of the
  // tile list (see xcd_walk)
  if (cap >= fvk::kXcds) cap -= cap % fvk::kXcds;
  return std::max(cap, 1);
}

int enqueue_stage(const StepPlan& P, int mode, int fp32, double* rout, hipStream_t st) {
  for (const LaunchSet& s : P.sets) {
    if (s.ntiles <= 0) continue;
    const int grid = launch_grid(s, fp32, P.ns);
    const int nfix = s.count_fixed ? s.ntiles : -1;
    hipError_t e;
    if ((s.kind == kSet2D && P.ns) || s.kind == kSet2DNS)
      e = fvk::launch_stage2d_ns(mode, fp32, grid, st, s.tiles, s.ntiles_dev, nfix, P.blocks, P.insts,
                                 rout);
    else if (s.kind == kSet2D)
      e = fvk::launch_stage2d(mode, fp32, grid, 256, st, s.tiles, s.ntiles_dev, nfix, P.lim, P.blocks,
                              P.insts, rout);
    else if (s.kind == kSet3DG)
      e = fvk::launch_stage3d_gen(mode, fp32, grid, st, s.tiles, s.ntiles_dev, nfix, P.lim, P.blocks,
                                  P.insts, rout);
    else
      e = fvk::launch_stage3d(mode, fp32, s.kind == kSet3D7 ? 7 : 3, grid, st, s.tiles, s.ntiles_dev,
                              nfix, P.lim, P.blocks, P.insts, rout);
    if (e != hipSuccess)
      return fvrt::set_error(FV_E_DEVICE, "stage launch failed: %s", hipGetErrorString(e));
  }
  return FV_OK;
}

int enqueue_cfl(const StepPlan& P, hipStream_t st) {
  for (const LaunchSet& s : P.sets) {
    if (s.ntiles <= 0) continue;
    hipError_t e;
    if (s.kind == kSet2D || s.kind == kSet2DNS)
      e = fvk::launch_cfl2d(std::max(1, std::min((s.ntiles + 3) / 4, 4096)), 256, st, s.tiles,
                            s.ntiles_dev, P.blocks, P.insts);
    else
      e = fvk::launch_cfl3d(std::max(1, std::min(s.ntiles, 8192)), 256, st, s.tiles, s.ntiles_dev,
                            P.blocks, P.insts);
    if (e != hipSuccess)
      return fvrt::set_error(FV_E_DEVICE, "time-step pass launch failed: %s", hipGetErrorString(e));
  }
  return FV_OK;
}

// stage kinds of one step of each scheme (StageKind in fv_device.h)
static const int kStages3[] = {1, 2, 3};
static const int kStages2[] = {1, 6};
static const int kStages4[] = {1, 4, 5, 6};

static int enqueue_one_step(const StepPlan& P, int fp32, hipStream_t st) {
  const int* modes = P.rk == 2 ? kStages2 : (P.rk == 4 ? kStages4 : kStages3);
  const int ns = P.rk == 2 ? 2 : (P.rk == 4 ? 4 : 3);
  for (int m = 0; m < ns; ++m) {
    const int e = enqueue_stage(P, modes[m], fp32, nullptr, st);
    if (e) return e;
  }
  const hipError_t e = fvk::launch_finalize(st, P.insts, P.active, P.ninst, P.ninst_dev);
  if (e != hipSuccess)
    return fvrt::set_error(FV_E_DEVICE, "finalize launch failed: %s", hipGetErrorString(e));
  return FV_OK;
}

int enqueue_steps(const StepPlan& P, int fp32, int nsteps, hipStream_t st, GraphCache* cache,
                  int variant) {
  if (nsteps <= 0) return FV_OK;
  if (!cache || !graphs_enabled()) {
    for (int k = 0; k < nsteps; ++k) {
      const int e = enqueue_one_step(P, fp32, st);
      if (e) return e;
    }
    return FV_OK;
  }
  // a captured graph depends on the step count, the precision, the scheme,
  // the limiter given at launch and the caller's variant
  const long long key = ((long long)(unsigned)variant << 40) | ((long long)(P.ns ? 1 : 0) << 39) |
                        ((long long)(P.lim + 1) << 36) | ((long long)P.rk << 32) |
                        ((long long)nsteps << 1) | (fp32 ? 1 : 0);
  hipGraphExec_t ex = cache->get(key);
  if (!ex) {
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
      return fvrt::set_error(FV_E_DEVICE, "capture stream creation failed");
    hipGraph_t gr = nullptr;
    int err = FV_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      return fvrt::set_error(FV_E_DEVICE, "graph capture could not start");
    }
    for (int k = 0; k < nsteps && !err; ++k) err = enqueue_one_step(P, fp32, cs);
    const hipError_t ec = hipStreamEndCapture(cs, &gr);
    (void)hipStreamDestroy(cs);
    if (err) {
      if (gr) (void)hipGraphDestroy(gr);
      return err;
    }
    if (ec != hipSuccess || !gr)
      return fvrt::set_error(FV_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess)
      return fvrt::set_error(FV_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    cache->put(key, ex);
  }
  const hipError_t e = hipGraphLaunch(ex, st);
  if (e != hipSuccess) return fvrt::set_error(FV_E_DEVICE, "graph launch failed: %s", hipGetErrorString(e));
  return FV_OK;
}

}  // namespace fvexec
