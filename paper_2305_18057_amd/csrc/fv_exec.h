// Launch sequencing shared by the grid API and the server: a step plan is a
// set of tile lists (2D, 3D with 4 or 8 rows per tile) over one block table
// and one instance table.  One step = stage 1, 2, 3 over every list, then the
// per-instance finalize.  Steps are replayed from captured hipGraphs.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <vector>

#include "fv_device.h"

namespace fvexec {

// tile sets: 2D, 3D with 3 j-rows per tile (4-wave workgroups), 3D with 7
// (8 waves), general 3D (curvilinear blocks or a source; 4 j-rows, 4 waves)
// kSet2DNS: 2D tiles that always take the Navier-Stokes stage kernel (the
// server's viscous instances; a grid's own plan chooses by StepPlan::ns)
enum { kSet2D = 0, kSet3D3 = 1, kSet3D7 = 2, kSet3DG = 3, kSet2DNS = 4 };
constexpr int kSetKinds = 5;
// the set kind of a grid: 2D, general 3D, or uniform 3D by its tile rows
inline int set_kind(int ndim, bool general3d, int ny) {
  if (ndim == 2) return kSet2D;
  if (general3d) return kSet3DG;
  return ny >= 7 ? kSet3D7 : kSet3D3;
}

struct LaunchSet {
  fvk::DevTile* tiles = nullptr;
  int* ntiles_dev = nullptr;  // device-resident count (graphs read it at run time)
  int ntiles = 0;             // host view, sizes the persistent grid
  bool count_fixed = false;   // ntiles is the exact count for as long as the plan is used
  int kind = kSet2D;
  int max_grid = 0;           // 0: as many workgroups as co-reside on the device
};

struct StepPlan {
  fvk::DevBlock* blocks = nullptr;
  fvk::DevInstance* insts = nullptr;
  const int* active = nullptr;  // device list of instance indices (nullptr: 0..ninst-1)
  int ninst = 0;                // finalize grid (the capacity when ninst_dev is set)
  const int* ninst_dev = nullptr;  // device-resident live instance count
  int rk = 3;                   // 3: SSP-RK3; 2, 4: the 2- and 4-stage second-order schemes
  int lim = -1;                 // >= 0: the limiter of every instance; -1: each instance's own
  bool ns = false;              // 2D sets run the Navier-Stokes stage kernel (viscous flux,
                                // no-slip walls, source term)
  std::vector<LaunchSet> sets;
};

class GraphCache {
 public:
  ~GraphCache() { clear(); }
  void clear();
  hipGraphExec_t get(long long key) const {
    auto it = m_.find(key);
    return it == m_.end() ? nullptr : it->second;
  }
  void put(long long key, hipGraphExec_t e) { m_[key] = e; }

 private:
  std::map<long long, hipGraphExec_t> m_;
};

int graph_chunk();                       // steps per captured graph
int launch_grid(const LaunchSet& s, int fp32, bool ns = false);
int enqueue_stage(const StepPlan& P, int mode, int fp32, double* rout, hipStream_t s);
int enqueue_cfl(const StepPlan& P, hipStream_t s);
// nsteps full steps; with a cache, replays (and captures on first use) a graph
// (variant tells apart plans with different launch sets in one cache)
int enqueue_steps(const StepPlan& P, int fp32, int nsteps, hipStream_t s, GraphCache* cache,
                  int variant = 0);

}  // namespace fvexec
