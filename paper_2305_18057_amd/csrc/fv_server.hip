// Continuous-batching solve server over one caller-supplied device arena.
//
// Requests (grid, initial state, parameters, stop rule) queue on the host.  A
// worker thread admits them, in arrival order with backfill, while an
// instance slot is free and the arena has room for the request's footprint
// (its state buffers, node coordinates and reduction partials), uploads them,
// and appends their tiles to the device-resident work-lists.  Every resident
// instance is then advanced together: each batched launch replays a captured
// graph of `steps_per_launch` SSP-RK3 steps whose persistent stage kernels
// walk the union work-list (the list length is read on the device, so the
// graph stays valid as instances come and go).  An instance stops on the
// device at exactly its own stop step (drop <= tol, max steps, t_end or a
// non-physical state); the worker then copies its state out, frees its slot
// and arena range, and the next requests are admitted.  An instance's results
// depend only on its own tiles, so they are the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "fv_exec.h"
#include "fv_runtime.h"

using namespace fvrt;

namespace {

constexpr int kMaxBlocksPerInst = 64;
constexpr int kKinds = fvexec::kSetKinds;

enum ReqState { RQ_QUEUED = 0, RQ_RESIDENT = 1, RQ_DONE = 2 };

struct Request {
  unsigned long long ticket = 0;
  HostGrid hg;
  std::vector<double> U0;
  std::vector<double> src;  // S_h in the state layout (grids with a source)
  fv_params params{};
  double drop_tol = 0.0;
  long long max_steps = 0;
  TileShape shape;
  int kind = fvexec::kSet2D;
  std::vector<fvk::DevTile> tiles;  // local indices; slot and block offset filled at admission
  std::vector<fvk::DevBlock> blocks;  // device descriptors (kept until the copy has run)
  size_t footprint = 0;
  size_t off_part = 0, off_nodes = 0, off_src = 0, off_u[3] = {0, 0, 0};
  // life cycle
  int state = RQ_QUEUED;
  int status = FV_OK;
  bool cancel = false;
  int slot = -1;
  size_t arena_off = 0;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  std::vector<double> result;
  fv_step_info info{};
  long long dry_steps = 0;
};

// first-fit allocator over [0, cap) with 256-byte granularity
class Arena {
 public:
  void reset(size_t cap) {
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t n, size_t& off) {
    n = align_up(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = align_up(n);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

}  // namespace

struct fv_server {
  fv_server_desc d{};
  bool dry = false;
  int device = 0;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  int max_inst = 0;
  int spl = 10;
  int fp32 = 0;
  std::string tune_path;
  // header of the arena
  size_t tile_cap = 0, heap_off = 0, heap_cap = 0;
  fvk::DevInstance* d_inst = nullptr;
  fvk::DevBlock* d_blocks = nullptr;
  int* d_active = nullptr;
  int* d_newlist = nullptr;
  int* d_counts = nullptr;  // ntiles per kind, then the live instance count
  fvk::DevTile* d_tiles[kKinds] = {};
  Arena heap;
  std::vector<fvk::DevInstance> h_inst;
  std::vector<Request*> slot_req;
  long long tiles_in_use[kKinds] = {};
  // requests
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<unsigned long long, Request*> reqs;
  unsigned long long next_ticket = 1;
  bool stop = false;
  std::thread worker;
  fvexec::GraphCache graphs;
  std::chrono::steady_clock::time_point t0;
  // statistics
  fv_server_stats st{};

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

// the tile list (and stage kernel) of an instance: 2D Euler or Navier-Stokes,
// general 3D (curvilinear blocks or oriented links), or uniform 3D by tile rows
int kind_of(const HostGrid& g, const TileShape& sh, bool ns) {
  if (g.ndim == 2) return ns ? fvexec::kSet2DNS : fvexec::kSet2D;
  if (g.gen3) return fvexec::kSet3DG;
  return sh.ny >= 7 ? fvexec::kSet3D7 : fvexec::kSet3D3;
}

// arena footprint of one instance: reduction partials, node coordinates and
// the three state buffers
void region_layout(Request* r) {
  size_t off = 0;
  r->off_part = off;
  off += align_up(sizeof(double) * fvk::kPartStride * std::max<size_t>(1, r->tiles.size()));
  r->off_nodes = off;
  off += align_up(sizeof(double) * (size_t)r->hg.node_doubles);
  r->off_src = off;
  off += r->hg.with_source ? align_up(sizeof(double) * (size_t)r->hg.state_size) : 0;
  for (int s = 0; s < 3; ++s) {
    r->off_u[s] = off;
    off += align_up(sizeof(double) * (size_t)r->hg.state_size);
  }
  r->footprint = off;
}

void finish(fv_server* S, Request* r, int status) {
  r->state = RQ_DONE;
  r->status = status;
  r->t_done = S->now();
  if (status == FV_OK || status == FV_E_NONPHYSICAL) S->st.completed++;
  else if (status == FV_E_CANCELLED) S->st.cancelled++;
  else S->st.failed++;
}

int upload(fv_server* S, Request* r) {
  char* base = S->arena + S->heap_off + r->arena_off;
  const int slot = r->slot;
  const int boff = slot * kMaxBlocksPerInst;
  InstLayout L{};
  L.nodes = r->off_nodes;
  L.src = r->off_src;
  for (int s = 0; s < 3; ++s) L.u[s] = r->off_u[s];
  build_blocks(r->hg, base, L, slot, r->blocks, boff);
  FV_HIP(hipMemcpyAsync(S->d_blocks + boff, r->blocks.data(), sizeof(fvk::DevBlock) * r->blocks.size(),
                        hipMemcpyHostToDevice, S->stream));
  FV_HIP(upload_nodes(r->hg, base + r->off_nodes, S->stream));
  if (r->hg.with_source)
    FV_HIP(hipMemcpyAsync(base + r->off_src, r->src.data(), sizeof(double) * r->src.size(),
                          hipMemcpyHostToDevice, S->stream));
  FV_HIP(hipMemcpyAsync(base + r->off_u[0], r->U0.data(), sizeof(double) * r->U0.size(),
                        hipMemcpyHostToDevice, S->stream));
  fvk::DevInstance I;
  std::memset(&I, 0, sizeof(I));
  params_to_inst(&r->params, r->hg.gamma, I);
  I.ndim = r->hg.ndim;
  I.nv = r->hg.nv;
  I.ncells = r->hg.ncells;
  I.ntiles = (int)r->tiles.size();
  I.part = (double*)(base + r->off_part);
  I.step_limit = r->max_steps;
  I.drop_tol = r->drop_tol;
  S->h_inst[slot] = I;
  FV_HIP(hipMemcpyAsync(S->d_inst + slot, &S->h_inst[slot], sizeof(I), hipMemcpyHostToDevice,
                        S->stream));
  return FV_OK;
}

// device work-lists = concatenation of the resident instances' tiles
int rebuild_lists(fv_server* S, const std::vector<Request*>& resident) {
  std::vector<fvk::DevTile> lists[kKinds];
  std::vector<int> active;
  for (Request* r : resident) {
    active.push_back(r->slot);
    const int boff = r->slot * kMaxBlocksPerInst;
    for (fvk::DevTile t : r->tiles) {
      t.blk += boff;
      t.inst = r->slot;
      lists[r->kind].push_back(t);
    }
  }
  int counts[kKinds + 1] = {};
  counts[kKinds] = (int)active.size();
  for (int k = 0; k < kKinds; ++k) {
    counts[k] = (int)lists[k].size();
    if (counts[k])
      FV_HIP(hipMemcpyAsync(S->d_tiles[k], lists[k].data(), sizeof(fvk::DevTile) * counts[k],
                            hipMemcpyHostToDevice, S->stream));
  }
  if (!active.empty())
    FV_HIP(hipMemcpyAsync(S->d_active, active.data(), sizeof(int) * active.size(),
                          hipMemcpyHostToDevice, S->stream));
  FV_HIP(hipMemcpyAsync(S->d_counts, counts, sizeof(counts), hipMemcpyHostToDevice, S->stream));
  // the host arrays above go out of scope: wait for the copies
  FV_HIP(hipStreamSynchronize(S->stream));
  return FV_OK;
}

fvexec::StepPlan plan_of(fv_server* S, unsigned mask) {
  fvexec::StepPlan P;
  P.blocks = S->d_blocks;
  P.insts = S->d_inst;
  P.active = S->d_active;
  P.ninst = S->max_inst;
  P.ninst_dev = S->d_counts + kKinds;
  for (int k = 0; k < kKinds; ++k) {
    if (!(mask & (1u << k))) continue;
    fvexec::LaunchSet ls;
    ls.tiles = S->d_tiles[k];
    ls.ntiles_dev = S->d_counts + k;
    ls.ntiles = 1 << 28;  // size the persistent grid for a full device
    ls.kind = k;
    P.sets.push_back(ls);
  }
  return P;
}

// time-step bound and stop flags of newly admitted instances
int start_instances(fv_server* S, const std::vector<Request*>& fresh, unsigned mask) {
  std::vector<int> slots;
  for (Request* r : fresh) slots.push_back(r->slot);
  FV_HIP(hipMemcpyAsync(S->d_newlist, slots.data(), sizeof(int) * slots.size(), hipMemcpyHostToDevice,
                        S->stream));
  fvexec::StepPlan P = plan_of(S, mask);
  for (auto& ls : P.sets) ls.ntiles = (int)S->tiles_in_use[ls.kind];
  int e = fvexec::enqueue_cfl(P, S->stream);
  if (e) return e;
  FV_HIP(fvk::launch_cfl_init(S->stream, S->d_inst, S->d_newlist, (int)slots.size()));
  FV_HIP(fvk::launch_prepare(S->stream, S->d_inst, S->d_newlist, (int)slots.size()));
  FV_HIP(hipStreamSynchronize(S->stream));
  return FV_OK;
}

int retire(fv_server* S, Request* r, const fvk::DevInstance& I) {
  r->result.resize(r->U0.size());
  if (!S->dry) {
    char* base = S->arena + S->heap_off + r->arena_off;
    FV_HIP(hipMemcpyAsync(r->result.data(), base + r->off_u[0], sizeof(double) * r->result.size(),
                          hipMemcpyDeviceToHost, S->stream));
    FV_HIP(hipStreamSynchronize(S->stream));
  } else {
    r->result = r->U0;
  }
  r->info.steps = I.steps;
  r->info.t = I.t;
  r->info.dt_last = I.dt_last;
  for (int v = 0; v < 5; ++v) r->info.norms[v] = I.norms[v];
  r->info.norm = I.norm;
  r->info.drop = I.drop;
  r->info.flags = I.flags;
  return FV_OK;
}

void worker_main(fv_server* S) {
  if (!S->dry) (void)hipSetDevice(S->device);
  std::vector<Request*> resident;
  std::vector<Request*> free_list;
  auto fail_all = [&](int status) {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Request* r : resident) finish(S, r, status);
    for (Request* r : S->queue) finish(S, r, status);
    S->queue.clear();
    resident.clear();
    S->cv.notify_all();
  };
  while (true) {
    std::vector<Request*> fresh, gone;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (resident.empty())
        S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->stop) break;
      for (Request* r : resident)
        if (r->cancel) gone.push_back(r);
      // admission: arrival order, later requests may fill in when the head
      // of the queue does not fit yet
      for (auto it = S->queue.begin(); it != S->queue.end();) {
        Request* r = *it;
        int slot = -1;
        for (int s = 0; s < S->max_inst; ++s)
          if (!S->slot_req[s]) {
            slot = s;
            break;
          }
        if (slot < 0) break;
        size_t off = 0;
        if (S->tiles_in_use[r->kind] + (long long)r->tiles.size() > (long long)S->tile_cap ||
            !S->heap.alloc(r->footprint, off)) {
          ++it;
          continue;
        }
        S->tiles_in_use[r->kind] += (long long)r->tiles.size();
        r->slot = slot;
        r->arena_off = off;
        r->state = RQ_RESIDENT;
        r->t_admit = S->now();
        S->slot_req[slot] = r;
        S->st.admitted++;
        fresh.push_back(r);
        it = S->queue.erase(it);
      }
      S->st.arena_used = S->heap.used();
      S->st.arena_peak = S->heap.peak();
    }
    // cancelled resident requests leave before the next launch
    for (Request* r : gone) {
      resident.erase(std::find(resident.begin(), resident.end(), r));
      std::lock_guard<std::mutex> lk(S->mu);
      S->heap.release(r->arena_off, r->footprint);
      S->tiles_in_use[r->kind] -= (long long)r->tiles.size();
      S->slot_req[r->slot] = nullptr;
      finish(S, r, FV_E_CANCELLED);
      S->cv.notify_all();
    }
    int err = FV_OK;
    if (!S->dry) {
      for (Request* r : fresh)
        if ((err = upload(S, r))) break;
    } else {
      for (Request* r : fresh) {
        fvk::DevInstance I;
        std::memset(&I, 0, sizeof(I));
        I.step_limit = r->max_steps;
        S->h_inst[r->slot] = I;
      }
    }
    for (Request* r : fresh) resident.push_back(r);
    unsigned mask = 0;
    for (Request* r : resident) mask |= 1u << r->kind;
    if (!err && !S->dry && (!fresh.empty() || !gone.empty())) err = rebuild_lists(S, resident);
    if (!err && !S->dry && !fresh.empty()) err = start_instances(S, fresh, mask);
    if (err) {
      fail_all(FV_E_DEVICE);
      continue;
    }
    if (resident.empty()) continue;
    // ---- one batched launch of spl steps over every resident instance
    long long before = 0;
    for (Request* r : resident) before += S->h_inst[r->slot].steps * r->hg.ncells;
    if (!S->dry) {
      fvexec::StepPlan P = plan_of(S, mask);
      err = fvexec::enqueue_steps(P, S->fp32, S->spl, S->stream, &S->graphs, (int)mask);
      if (!err && hipMemcpyAsync(S->h_inst.data(), S->d_inst, sizeof(fvk::DevInstance) * S->max_inst,
                                 hipMemcpyDeviceToHost, S->stream) != hipSuccess)
        err = FV_E_DEVICE;
      if (!err && hipStreamSynchronize(S->stream) != hipSuccess) err = FV_E_DEVICE;
      if (err) {
        fail_all(FV_E_DEVICE);
        continue;
      }
    } else {
      // a dry-run launch stands for some device time, so residency overlaps
      std::this_thread::sleep_for(std::chrono::microseconds(200));
      for (Request* r : resident) {
        fvk::DevInstance& I = S->h_inst[r->slot];
        const long long take = std::min<long long>(S->spl, I.step_limit - I.steps);
        I.steps += std::max(0LL, take);
        if (I.steps >= I.step_limit) {
          I.stopped = 1;
          I.flags |= fvk::FLAG_STEPLIMIT;
        }
      }
    }
    long long after = 0;
    for (Request* r : resident) after += S->h_inst[r->slot].steps * r->hg.ncells;
    // ---- retire the instances that stopped
    std::vector<Request*> keep;
    bool changed = false;
    for (Request* r : resident) {
      const fvk::DevInstance I = S->h_inst[r->slot];
      if (!I.stopped) {
        keep.push_back(r);
        continue;
      }
      changed = true;
      const int e = retire(S, r, I);
      std::lock_guard<std::mutex> lk(S->mu);
      S->heap.release(r->arena_off, r->footprint);
      S->tiles_in_use[r->kind] -= (long long)r->tiles.size();
      S->slot_req[r->slot] = nullptr;
      finish(S, r, e ? e : ((I.flags & fvk::FLAG_NONPHYS) ? FV_E_NONPHYSICAL : FV_OK));
    }
    resident.swap(keep);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->st.launches++;
      S->st.cell_steps += after - before;
      S->st.arena_used = S->heap.used();
      S->cv.notify_all();
    }
    if (changed && !S->dry && rebuild_lists(S, resident)) fail_all(FV_E_DEVICE);
  }
}

}  // namespace

extern "C" int fv_server_create(const fv_server_desc* d, fv_server** out) {
  if (!d || !out) return set_error(FV_E_INVAL, "null argument");
  *out = nullptr;
  if (d->max_instances < 1 || d->max_instances > 1024)
    return set_error(FV_E_INVAL, "max_instances must be in 1..1024");
  if (d->precision != FV_FP64 && d->precision != FV_FP32_FLUX)
    return set_error(FV_E_INVAL, "unknown precision %d", d->precision);
  const bool dry = (d->flags & FV_SERVER_DRYRUN) != 0;
  if (!dry && (!d->d_arena || ((uintptr_t)d->d_arena) % kAlign))
    return set_error(FV_E_INVAL, "arena must be a %zu-byte aligned device pointer", kAlign);
  fv_server* S = new (std::nothrow) fv_server();
  if (!S) return set_error(FV_E_NOMEM, "host allocation failed");
  S->d = *d;
  S->dry = dry;
  S->stream = (hipStream_t)d->hip_stream;
  S->arena = (char*)d->d_arena;
  S->max_inst = d->max_instances;
  S->spl = d->steps_per_launch > 0 ? d->steps_per_launch : 10;
  S->fp32 = d->precision == FV_FP32_FLUX;
  if (d->autotune_cache) S->tune_path = d->autotune_cache;
  S->t0 = std::chrono::steady_clock::now();
  // header: instances, blocks, active list, new list, counts, tile lists
  S->tile_cap = d->arena_bytes / 16384 + 4096;
  size_t off = 0;
  const size_t o_inst = off;
  off += align_up(sizeof(fvk::DevInstance) * S->max_inst);
  const size_t o_blk = off;
  off += align_up(sizeof(fvk::DevBlock) * (size_t)S->max_inst * kMaxBlocksPerInst);
  const size_t o_act = off;
  off += align_up(sizeof(int) * S->max_inst);
  const size_t o_new = off;
  off += align_up(sizeof(int) * S->max_inst);
  const size_t o_cnt = off;
  off += align_up(sizeof(int) * (kKinds + 1));
  size_t o_t[kKinds];
  for (int k = 0; k < kKinds; ++k) {
    o_t[k] = off;
    off += align_up(sizeof(fvk::DevTile) * S->tile_cap);
  }
  if (off >= d->arena_bytes) {
    delete S;
    return set_error(FV_E_NOMEM, "arena of %zu bytes cannot hold the %zu-byte header", d->arena_bytes, off);
  }
  S->heap_off = off;
  S->heap_cap = d->arena_bytes - off;
  S->heap.reset(S->heap_cap);
  if (!dry) {
    if (hipGetDevice(&S->device) != hipSuccess) {
      delete S;
      return set_error(FV_E_DEVICE, "hipGetDevice failed");
    }
    S->d_inst = (fvk::DevInstance*)(S->arena + o_inst);
    S->d_blocks = (fvk::DevBlock*)(S->arena + o_blk);
    S->d_active = (int*)(S->arena + o_act);
    S->d_newlist = (int*)(S->arena + o_new);
    S->d_counts = (int*)(S->arena + o_cnt);
    for (int k = 0; k < kKinds; ++k) S->d_tiles[k] = (fvk::DevTile*)(S->arena + o_t[k]);
    int zero[kKinds + 1] = {};
    std::vector<fvk::DevInstance> blank(S->max_inst);
    std::memset(blank.data(), 0, sizeof(fvk::DevInstance) * blank.size());
    for (auto& I : blank) I.stopped = 1;
    if (hipMemcpyAsync(S->d_counts, zero, sizeof(zero), hipMemcpyHostToDevice, S->stream) != hipSuccess ||
        hipMemcpyAsync(S->d_inst, blank.data(), sizeof(fvk::DevInstance) * blank.size(),
                       hipMemcpyHostToDevice, S->stream) != hipSuccess ||
        hipStreamSynchronize(S->stream) != hipSuccess) {
      delete S;
      return set_error(FV_E_DEVICE, "arena header initialisation failed");
    }
  }
  try {
    S->h_inst.assign(S->max_inst, fvk::DevInstance{});
    S->slot_req.assign(S->max_inst, nullptr);
    S->worker = std::thread(worker_main, S);
  } catch (const std::exception&) {
    delete S;
    return set_error(FV_E_NOMEM, "the serving thread could not be started");
  }
  *out = S;
  return FV_OK;
}

namespace {

int submit(fv_server* S, const fv_grid_desc* desc, const double* U0, const double* src,
           const fv_params* p, double drop_tol, long long max_steps, unsigned long long* ticket) {
  if (!S || !U0 || !ticket) return set_error(FV_E_INVAL, "null argument");
  int st = check_params(p);
  if (st) return st;
  // resident instances share graph replays of one stage sequence
  if (rk_of(p) != 3) return set_error(FV_E_UNSUPPORTED, "the server runs SSP-RK3 (rk = 3) only");
  if (max_steps < 1) return set_error(FV_E_INVAL, "max_steps must be >= 1");
  if (!(drop_tol >= 0.0)) return set_error(FV_E_INVAL, "drop_tol must be >= 0");
  Request* r = new (std::nothrow) Request();
  if (!r) return set_error(FV_E_NOMEM, "host allocation failed");
  st = validate_and_copy(desc, r->hg);
  if (st) {
    delete r;
    return st;
  }
  if (r->hg.nblocks > kMaxBlocksPerInst) {
    delete r;
    return set_error(FV_E_UNSUPPORTED, "at most %d blocks per served grid", kMaxBlocksPerInst);
  }
  if (p->mu > 0.0 && r->hg.ndim != 2) {
    delete r;
    return set_error(FV_E_UNSUPPORTED, "the viscous flux is provided for 2D grids only");
  }
  if (r->hg.with_source != (src != nullptr)) {
    const bool reserved = r->hg.with_source;
    delete r;
    return set_error(FV_E_INVAL, reserved
                                     ? "a grid with with_source = 1 is submitted with its source "
                                       "(fv_submit_with_source)"
                                     : "fv_submit_with_source needs a descriptor with with_source = 1");
  }
  // 2D instances with a viscosity, a no-slip face or a source take the
  // Navier-Stokes kernel (the choice of the grid API)
  const bool ns = r->hg.ndim == 2 && (p->mu > 0.0 || r->hg.has_noslip || r->hg.with_source);
  r->params = *p;
  r->params.precision = S->d.precision;
  r->drop_tol = drop_tol;
  r->max_steps = max_steps;
  TileShape sh = default_shape(r->hg);
  TileShape tsh;
  if (tune_lookup(tune_path(S->tune_path.empty() ? nullptr : S->tune_path.c_str()),
                  tune_key(r->hg, S->d.precision, ns), tsh))
    sh = tsh;
  r->shape = sh;
  r->kind = kind_of(r->hg, sh, ns);
  try {
    r->U0.assign(U0, U0 + r->hg.state_size);
    if (src) r->src.assign(src, src + r->hg.state_size);
    build_tiles(r->hg, sh, 0, 0, r->tiles);
  } catch (const std::bad_alloc&) {
    delete r;
    return set_error(FV_E_NOMEM, "host allocation failed");
  }
  region_layout(r);
  if (r->footprint > S->heap_cap) {
    const size_t need = r->footprint;
    delete r;
    return set_error(FV_E_NOMEM, "request needs %zu arena bytes, the arena holds %zu", need, S->heap_cap);
  }
  if ((long long)r->tiles.size() > (long long)S->tile_cap) {
    const size_t need = r->tiles.size();
    delete r;
    return set_error(FV_E_NOMEM, "request needs %zu tiles, the server's tile list holds %zu", need,
                     S->tile_cap);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) {
    delete r;
    return set_error(FV_E_INVAL, "server is shutting down");
  }
  r->ticket = S->next_ticket++;
  r->t_submit = S->now();
  S->reqs[r->ticket] = r;
  S->queue.push_back(r);
  S->st.submitted++;
  *ticket = r->ticket;
  S->cv.notify_all();
  return FV_OK;
}

}  // namespace

extern "C" int fv_submit(fv_server* S, const fv_grid_desc* desc, const double* U0, const fv_params* p,
                         double drop_tol, long long max_steps, unsigned long long* ticket) {
  return submit(S, desc, U0, nullptr, p, drop_tol, max_steps, ticket);
}

extern "C" int fv_submit_with_source(fv_server* S, const fv_grid_desc* desc, const double* U0,
                                     const double* S_h, const fv_params* p, double drop_tol,
                                     long long max_steps, unsigned long long* ticket) {
  if (!S_h) return set_error(FV_E_INVAL, "null source");
  return submit(S, desc, U0, S_h, p, drop_tol, max_steps, ticket);
}

extern "C" int fv_poll(fv_server* S, unsigned long long ticket, double* U_out, size_t cap,
                       fv_step_info* info) {
  if (!S) return set_error(FV_E_INVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(FV_E_NOTFOUND, "unknown ticket %llu", ticket);
  Request* r = it->second;
  if (r->state != RQ_DONE) return FV_PENDING;
  if (U_out && !r->result.empty()) {
    if (cap < r->result.size())
      return set_error(FV_E_INVAL, "output buffer of %zu doubles, need %zu", cap, r->result.size());
    std::memcpy(U_out, r->result.data(), sizeof(double) * r->result.size());
  }
  if (info) *info = r->info;
  const int status = r->status;
  S->reqs.erase(it);
  delete r;
  return status;
}

extern "C" int fv_cancel(fv_server* S, unsigned long long ticket) {
  if (!S) return set_error(FV_E_INVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(FV_E_NOTFOUND, "unknown ticket %llu", ticket);
  Request* r = it->second;
  if (r->state == RQ_QUEUED) {
    S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
    finish(S, r, FV_E_CANCELLED);
    S->cv.notify_all();
  } else if (r->state == RQ_RESIDENT) {
    r->cancel = true;
  }
  return FV_OK;
}

extern "C" int fv_request_times(fv_server* S, unsigned long long ticket, double times[3]) {
  if (!S || !times) return set_error(FV_E_INVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(FV_E_NOTFOUND, "unknown ticket %llu", ticket);
  times[0] = it->second->t_submit;
  times[1] = it->second->t_admit;
  times[2] = it->second->t_done;
  return FV_OK;
}

extern "C" double fv_server_clock(fv_server* S) { return S ? S->now() : 0.0; }

extern "C" int fv_server_get_stats(fv_server* S, fv_server_stats* out) {
  if (!S || !out) return set_error(FV_E_INVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->st;
  int resident = 0;
  for (Request* r : S->slot_req) resident += r != nullptr;
  out->resident = resident;
  out->queued = (int)S->queue.size();
  out->arena_used = S->heap.used();
  out->arena_peak = S->heap.peak();
  return FV_OK;
}

extern "C" int fv_server_destroy(fv_server* S) {
  if (!S) return set_error(FV_E_INVAL, "null server");
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  if (!S->dry && S->stream) (void)hipStreamSynchronize(S->stream);
  S->graphs.clear();
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return FV_OK;
}
