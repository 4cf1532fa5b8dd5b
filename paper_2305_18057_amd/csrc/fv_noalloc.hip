// Allocation-free variant of the step entry point: fv_step_noalloc advances a
// caller's device state in place with the same kernels as fv_step, with every
// buffer beyond that state (block table, instance record, tile list, tile
// partials, node coordinates and the two RK stage buffers) placed in one
// file-scope device array of fixed size.  No hipMalloc, hipFree or other
// device allocation happens on this path.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "fv_exec.h"
#include "fv_launch.h"
#include "fv_runtime.h"

using namespace fvrt;

namespace {

constexpr size_t kScratchBytes = (size_t)FV_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per device the library runs on, held until the process ends.  In
// host code this name only stands in for the symbol: its device address comes
// from hipGetSymbolAddress, per device, below.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;  // one call at a time in the process: the array is shared
char* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of the array (device current)
int scratch_of_device(char** out) {
  int dev = -1;
  FV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(FV_E_UNSUPPORTED, "device index %d beyond the %d devices this path tracks", dev,
                     kMaxDevices);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(FV_E_DEVICE, "hipGetSymbolAddress of the static scratch array failed: %s",
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return FV_OK;
}

// Scratch layout: the grid layout of an instance without its U^n buffer (the
// caller's state takes that role), i.e. descriptors, tiles, partials, ghost
// segments, nodes, then the two stage buffers.
InstLayout noalloc_layout(const HostGrid& hg) {
  InstLayout L = layout_of(hg);
  const size_t sbytes = align_up(sizeof(double) * (size_t)hg.state_size);
  L.u[1] = L.u[0];
  L.u[2] = L.u[0] + sbytes;
  L.total = L.u[0] + 2 * sbytes;
  return L;
}

}  // namespace

extern "C" size_t fv_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int fv_step_noalloc(const fv_grid_desc* desc, double* d_U, const fv_params* p, int nsteps,
                               void* hip_stream, fv_step_info* info) {
  if (!d_U) return set_error(FV_E_INVAL, "null state");
  int st = check_params(p);
  if (st) return st;
  if (nsteps < 0) return set_error(FV_E_INVAL, "negative step count");
  HostGrid hg;
  st = validate_and_copy(desc, hg);
  if (st) return st;
  if (hg.with_source)
    return set_error(FV_E_UNSUPPORTED, "a source term needs a grid handle (fv_create_grid, "
                                       "fv_set_source): the allocation-free path takes none");
  if (p->mu > 0.0 && hg.ndim != 2)
    return set_error(FV_E_UNSUPPORTED, "the viscous flux is provided for 2D grids only");
  const bool ns = p->mu > 0.0 || hg.has_noslip;
  const InstLayout L = noalloc_layout(hg);
  if (L.total > kScratchBytes)
    return set_error(FV_E_NOMEM,
                     "grid needs %zu bytes of static scratch (descriptors, tiles, partials, nodes, "
                     "two stage buffers); the allocation-free path holds at most %zu",
                     L.total, kScratchBytes);
  if (((uintptr_t)d_U) % sizeof(double))
    return set_error(FV_E_INVAL, "state pointer must be 8-byte aligned");

  std::lock_guard<std::mutex> lock(g_mu);
  char* base = nullptr;
  st = scratch_of_device(&base);
  if (st) return st;
  hipStream_t s = (hipStream_t)hip_stream;

  // descriptors: the stage buffers in scratch, U^n the caller's array
  std::vector<fvk::DevBlock> hblocks;
  build_blocks(hg, base, L, 0, hblocks, 0);
  {
    long long soff = 0;
    for (auto& B : hblocks) {
      B.u[0] = d_U + soff;
      soff += B.ncell * hg.nv;
    }
  }
  TileShape sh = default_shape(hg);
  {
    TileShape tsh;
    if (tune_lookup(tune_path(nullptr), tune_key(hg, p->precision, ns), tsh)) sh = tsh;
  }
  std::vector<fvk::DevTile> htiles;
  build_tiles(hg, sh, 0, 0, htiles);
  const int nt = (int)htiles.size();
  if (nt > L.max_tiles) return set_error(FV_E_INVAL, "tile list exceeds its capacity");

  fvk::DevBlock* d_blocks = (fvk::DevBlock*)(base + L.blocks);
  fvk::DevInstance* d_inst = (fvk::DevInstance*)(base + L.inst);
  int* d_ntiles = (int*)(base + L.ntiles);
  fvk::DevTile* d_tiles = (fvk::DevTile*)(base + L.tiles);

  // instance record: written whole, so nothing of an earlier call survives
  fvk::DevInstance I;
  std::memset(&I, 0, sizeof(I));
  params_to_inst(p, hg.gamma, I);
  I.ndim = hg.ndim;
  I.nv = hg.nv;
  I.ncells = hg.ncells;
  I.ntiles = nt;
  I.part = (double*)(base + L.part);
  I.drop_tol = 0.0;
  I.step_limit = nsteps;

  // every return below first waits for the copies of the host records above
  struct SyncOnExit {
    hipStream_t s;
    ~SyncOnExit() { (void)hipStreamSynchronize(s); }
  } sync_on_exit{s};
  FV_HIP(hipMemcpyAsync(d_blocks, hblocks.data(), sizeof(fvk::DevBlock) * hblocks.size(),
                        hipMemcpyHostToDevice, s));
  FV_HIP(hipMemcpyAsync(d_tiles, htiles.data(), sizeof(fvk::DevTile) * nt, hipMemcpyHostToDevice, s));
  FV_HIP(hipMemcpyAsync(d_ntiles, &nt, sizeof(int), hipMemcpyHostToDevice, s));
  FV_HIP(upload_nodes(hg, base + L.nodes, s));
  FV_HIP(hipMemcpyAsync(d_inst, &I, sizeof(I), hipMemcpyHostToDevice, s));

  fvexec::StepPlan plan;
  plan.blocks = d_blocks;
  plan.insts = d_inst;
  plan.active = nullptr;
  plan.ninst = 1;
  plan.rk = rk_of(p);
  plan.lim = p->limiter;
  plan.ns = ns;
  fvexec::LaunchSet ls;
  ls.tiles = d_tiles;
  ls.ntiles_dev = d_ntiles;
  ls.ntiles = nt;
  ls.count_fixed = true;
  ls.kind = fvexec::set_kind(hg.ndim, hg.gen3, sh.ny);
  plan.sets.push_back(ls);

  // time-step bound and physical check of the initial state, as a new state
  // gets in fv_set_state
  st = fvexec::enqueue_cfl(plan, s);
  if (st) return st;
  FV_HIP(fvk::launch_cfl_init(s, d_inst, nullptr, 1));
  // read back into its own record: the upload of I above is not overwritten
  fvk::DevInstance R;
  FV_HIP(hipMemcpyAsync(&R, d_inst, sizeof(R), hipMemcpyDeviceToHost, s));
  FV_HIP(hipStreamSynchronize(s));
  auto fill = [&](const fvk::DevInstance& J) {
    if (!info) return;
    info->steps = J.steps;
    info->t = J.t;
    info->dt_last = J.dt_last;
    for (int v = 0; v < 5; ++v) info->norms[v] = J.norms[v];
    info->norm = J.norm;
    info->drop = J.drop;
    info->flags = J.flags;
  };
  if (R.flags & fvk::FLAG_NONPHYS) {
    fill(R);
    return set_error(FV_E_NONPHYSICAL, "initial state has a cell with rho <= 0, p <= 0 or a non-finite value");
  }
  if (nsteps > 0) {
    FV_HIP(fvk::launch_prepare(s, d_inst, nullptr, 1));
    // kernels launched one by one: no graph is instantiated on this path
    st = fvexec::enqueue_steps(plan, p->precision == FV_FP32_FLUX, nsteps, s, nullptr);
    if (st) return st;
    FV_HIP(hipMemcpyAsync(&R, d_inst, sizeof(R), hipMemcpyDeviceToHost, s));
  }
  FV_HIP(hipStreamSynchronize(s));
  fill(R);
  if (R.flags & fvk::FLAG_NONPHYS)
    return set_error(FV_E_NONPHYSICAL, "state turned non-physical after %lld steps", R.steps);
  return FV_OK;
}
