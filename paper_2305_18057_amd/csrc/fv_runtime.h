// Host-side runtime shared by the grid API and the server (private).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <map>
#include <string>
#include <vector>

#include "fv.h"
#include "fv_device.h"
#include "fv_launch.h"

namespace fvrt {

int set_error(int status, const char* fmt, ...);

#define FV_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::fvrt::set_error(FV_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// tile shape of an instance: 2D rows per tile; 3D ny rows and planes per tile
struct TileShape {
  int rows = 8;   // 2D: rows per tile; 3D: planes per tile
  int ny = 7;     // 3D only: j-rows per tile (3 or 7)
  bool operator<(const TileShape& o) const { return rows < o.rows || (rows == o.rows && ny < o.ny); }
};

// validated, host-side copy of a grid description
struct HostGrid {
  int ndim = 2, nv = 4, nblocks = 0;
  double gamma = 1.4;
  std::vector<fv_block_desc> blocks;           // pointers below are owned copies
  std::vector<std::vector<double>> xs, ys, zs; // node coordinates (curvilinear blocks)
  long long ncells = 0, state_size = 0;
  long long node_doubles = 0;
  bool has_noslip = false;   // a no-slip face: the Navier-Stokes stage kernel runs it
  bool with_source = false;  // a source buffer S_h (2D: the Navier-Stokes kernel runs it)
  bool gen3 = false;         // 3D with curvilinear blocks, a source or an oriented block
                             // link: the general 3D kernel
  // trailing blocks that are read only, as the neighbours of block links,
  // and never computed (the halo block of the CPU-GPU split's GPU part)
  int nphantom = 0;
  long long phantom_cells = 0;
  long long compute_cells() const { return ncells - phantom_cells; }
};

int validate_and_copy(const fv_grid_desc* d, HostGrid& out);

// size of the per-instance device region and its layout
struct InstLayout {
  size_t blocks, inst, ntiles, tiles, part, segs, nodes, src, u[3], total;
  long long max_tiles;
  int nseg;
  long long ghost_cells, ghost_doubles;
};
long long max_tiles_of(const HostGrid& g);
InstLayout layout_of(const HostGrid& g);

// fill host mirrors (blocks, ghost segments) for an instance placed at `base`
void build_blocks(const HostGrid& g, char* base, const InstLayout& L, int inst_index,
                  std::vector<fvk::DevBlock>& out, int block_index_offset);
void build_segs(const HostGrid& g, std::vector<fvk::GhostSeg>& segs);
// node coordinates of every curvilinear block to dst (the layout's node
// region): per block x, y (and z in 3D), in block order
hipError_t upload_nodes(const HostGrid& g, char* dst, hipStream_t s);
void build_tiles(const HostGrid& g, const TileShape& sh, int inst_index, int block_index_offset,
                 std::vector<fvk::DevTile>& out);
TileShape default_shape(const HostGrid& g);
int size_class(const HostGrid& g);

// autotune table (JSON file of "key": {"rows": r, "ny": y})
std::string tune_key(const HostGrid& g, int precision, bool ns = false);
bool tune_lookup(const char* path, const std::string& key, TileShape& sh);
void tune_store(const char* path, const std::string& key, const TileShape& sh, double ms);
const char* tune_path(const char* given);

void params_to_inst(const fv_params* p, double gamma, fvk::DevInstance& I);
int check_params(const fv_params* p);
int rk_of(const fv_params* p);  // the scheme: 2, 3 or 4 (rk = 0 means 3)
int device_cu_count();
int occupancy_blocks(const void* kernel, int block_threads);

}  // namespace fvrt
