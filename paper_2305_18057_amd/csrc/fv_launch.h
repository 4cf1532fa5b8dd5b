// Launch wrappers of the device kernels (private to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "fv_device.h"

namespace fvk {

// 2D: mode 0 = residual only (writes rout), 1..6 = RK stage kinds (StageKind
// in fv_device.h: 1..3 SSP-RK3; 1, 4, 5, 6 the 2- and 4-stage schemes)
// ntiles_fixed >= 0: the tile count, known when the launch is recorded (the
// kernels then skip the read of *ntiles); -1: the count is read at run time.
// lim_fixed >= 0: the limiter of every instance in the launch; -1: each
// instance's own
hipError_t launch_stage2d(int mode, int fp32, int grid, int block, hipStream_t s,
                          const DevTile* tiles, const int* ntiles, int ntiles_fixed, int lim_fixed,
                          const DevBlock* blocks, DevInstance* insts, double* rout);
hipError_t launch_cfl2d(int grid, int block, hipStream_t s, const DevTile* tiles,
                        const int* ntiles, const DevBlock* blocks, DevInstance* insts);
const void* stage2d_kernel_ptr(int mode, int fp32);

// 2D Navier-Stokes stage (viscous flux added; one 256-thread workgroup per
// tile); the same stage kinds as launch_stage2d
hipError_t launch_stage2d_ns(int mode, int fp32, int grid, hipStream_t s, const DevTile* tiles,
                             const int* ntiles, int ntiles_fixed, const DevBlock* blocks,
                             DevInstance* insts, double* rout);
const void* stage2d_ns_kernel_ptr(int fp32);

// 3D: one workgroup per tile of ny j-rows (ny + 1 waves)
hipError_t launch_stage3d(int mode, int fp32, int ny, int grid, hipStream_t s,
                          const DevTile* tiles, const int* ntiles, int ntiles_fixed, int lim_fixed,
                          const DevBlock* blocks, DevInstance* insts, double* rout);
hipError_t launch_cfl3d(int grid, int block, hipStream_t s, const DevTile* tiles,
                        const int* ntiles, const DevBlock* blocks, DevInstance* insts);
const void* stage3d_kernel_ptr(int mode, int fp32, int ny);

// general 3D stage (curvilinear blocks, source term; one 256-thread
// workgroup per tile of 4 j-rows); the same stage kinds and arguments
hipError_t launch_stage3d_gen(int mode, int fp32, int grid, hipStream_t s, const DevTile* tiles,
                              const int* ntiles, int ntiles_fixed, int lim_fixed,
                              const DevBlock* blocks, DevInstance* insts, double* rout);
const void* stage3d_gen_kernel_ptr(int fp32);

// per-instance bookkeeping (one wavefront per instance)
//   prepare:  stop flags and time step of the coming steps from the parameters
//   finalize: step end: norms, first norm, drop, t, steps, spectral minimum,
//             flags, stop rule, next time step
//   cfl_init: spectral minimum and physical check after a new state
//   rnorms:   norms of a residual-only evaluation
hipError_t launch_prepare(hipStream_t s, DevInstance* insts, const int* active, int n);
hipError_t launch_finalize(hipStream_t s, DevInstance* insts, const int* active, int n,
                           const int* n_dev = nullptr);
hipError_t launch_cfl_init(hipStream_t s, DevInstance* insts, const int* active, int n);
hipError_t launch_rnorms(hipStream_t s, DevInstance* insts, const int* active, int n);

// ghost values of the current state in the documented dump layout
struct GhostSeg {
  int blk, face, n1, n2;
  long long cell_off;  // first ghost cell of this segment (both layers)
  long long out_off;   // first output double of this segment
};
hipError_t launch_ghosts(hipStream_t s, const DevBlock* blocks, const GhostSeg* segs, int nseg,
                         long long ncells, int nv, double* out);

}  // namespace fvk
