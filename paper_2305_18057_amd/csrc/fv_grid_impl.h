// Grid handle internals, shared by the grid API and the CPU-GPU split
// (private to the library).
#pragma once
#include "fv_exec.h"
#include "fv_runtime.h"

struct fv_grid {
  fvrt::HostGrid hg;
  fvrt::InstLayout L;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  fvk::DevBlock* d_blocks = nullptr;
  fvk::DevInstance* d_inst = nullptr;
  int* d_ntiles = nullptr;
  fvk::DevTile* d_tiles = nullptr;
  double* d_part = nullptr;
  fvk::GhostSeg* d_segs = nullptr;
  double* d_u[3] = {nullptr, nullptr, nullptr};
  std::vector<fvk::DevBlock> hblocks;
  std::vector<fvk::DevTile> htiles;
  fvk::DevInstance hinst;
  fvrt::TileShape shape;
  fvexec::StepPlan plan;
  fvexec::GraphCache graphs;
  int have_state = 0;
  double last_ms[4] = {0, 0, 0, 0};
  // viscosity with which the device's time-step bound of the current state
  // was formed (the viscous term enters it)
  double cfl_mu = 0.0, cfl_pr = 0.0;
};

namespace fvgrid {

// a grid over a validated host grid (the descriptor path and the CPU-GPU
// split's GPU part, whose halo block is read but never computed)
int create(fvrt::HostGrid&& hg, void* d_workspace, size_t bytes, void* hip_stream, fv_grid** out);
int upload_tiles(fv_grid* g);
int put_inst(fv_grid* g, bool whole);
int get_inst(fv_grid* g);
int cfl_pass(fv_grid* g);
int use_params(fv_grid* g, const fv_params* p);

}  // namespace fvgrid
