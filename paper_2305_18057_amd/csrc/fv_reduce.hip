// Per-instance bookkeeping kernels: parameters -> time step and stop flags,
// step-end reductions of the per-tile partials (fixed order: lane l sums
// tiles l, l+64, ... then a fixed butterfly), and the ghost dump.
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

// time step of the coming step: dt_fixed, or CFL times the spectral minimum
// of U^n; a positive t_end clamps the step so that t lands on t_end and stops
// the instance once t has reached it
__device__ __forceinline__ void next_dt(DevInstance& I) {
  double dt = I.dt_fixed > 0.0 ? I.dt_fixed : I.cfl * I.raw_min;
  int last = 0;
  if (I.t_end > 0.0) {
    if (I.t >= I.t_end) {
      I.stopped = 1;
      I.flags |= FLAG_TEND;
    } else if (dt >= I.t_end - I.t) {
      dt = I.t_end - I.t;
      last = 1;
    }
  }
  I.dt = dt;
  I.last_step = last;
}

__global__ void k_prepare(DevInstance* insts, const int* active, int n) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  DevInstance& I = insts[active ? active[x] : x];
  I.flags &= FLAG_NONPHYS;
  I.stopped = (I.flags & FLAG_NONPHYS) ? 1 : 0;
  if (I.steps >= I.step_limit) {
    I.stopped = 1;
    I.flags |= FLAG_STEPLIMIT;
  }
  if (!I.stopped) next_dt(I);
}

// Sums of the per-tile partials of one instance by a workgroup of kRedThreads
// threads.  Thread x takes the tiles x, x + kRedThreads, ... in that order
// (the loads of two tiles are in flight together), each wavefront combines
// its lanes by a fixed butterfly, and wavefront 0 combines the wavefront
// results by the same butterfly: the result depends only on the tile count,
// never on timing.  Result valid in wavefront 0.
constexpr int kRedThreads = 1024;
constexpr int kRedWaves = kRedThreads / 64;

struct RedOut {
  double s[5];
  double mn;
  int bad;
};

__device__ __forceinline__ void reduce_parts(int nt, const double* __restrict__ part, bool sums,
                                             bool mins, RedOut& out) {
  __shared__ double sh[kRedWaves][6];
  __shared__ int shb[kRedWaves];
  const int x = threadIdx.x;
  const int lane = x & 63, w = x >> 6;
  double a[5] = {0, 0, 0, 0, 0};
  double m = INFINITY;
  int b = 0;
  for (int t0 = x; t0 < nt; t0 += 2 * kRedThreads) {
    double p[2][7];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = t0 + u * kRedThreads;
      const double* q = part + min(t, nt - 1);
#pragma unroll
      for (int v = 0; v < 7; ++v) p[u][v] = ldg(q + (long long)v * nt);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (t0 + u * kRedThreads < nt) {
        if (sums) {
#pragma unroll
          for (int v = 0; v < 5; ++v) a[v] += p[u][v];
        }
        if (mins) {
          m = fmin(m, p[u][5]);
          b |= p[u][6] != 0.0;
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) a[v] = wave_sum(a[v]);
  m = wave_min(m);
  b = wave_or(b);
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sh[w][v] = a[v];
    sh[w][5] = m;
    shb[w] = b;
  }
  __syncthreads();
  if (w == 0) {
    // wavefront 0 combines the wavefront results by the same butterfly
    const bool has = lane < kRedWaves;
    const int y = has ? lane : 0;
#pragma unroll
    for (int v = 0; v < 5; ++v) out.s[v] = wave_sum(has ? sh[y][v] : 0.0);
    out.mn = wave_min(has ? sh[y][5] : INFINITY);
    out.bad = wave_or(has ? shb[y] : 0);
  }
}

__device__ __forceinline__ void norms_from_sums(int nv, long long ncells, const double* qref,
                                                const double* s, double* norms, double& comb) {
  double cs = 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    norms[v] = v < nv ? sqrt(s[v] / (double)ncells) : 0.0;
    if (v < nv) {
      const double q = qref[v] != 0.0 ? qref[v] : 1.0;
      const double r = norms[v] / q;
      cs += r * r;
    }
  }
  comb = sqrt(cs);
}

__global__ __launch_bounds__(kRedThreads) void k_finalize(DevInstance* insts, const int* active,
                                                         int n, const int* n_dev) {
  // with a device-resident count the grid is sized for the capacity and the
  // workgroups beyond the live count leave at once (graphs stay valid)
  if (n_dev && (int)blockIdx.x >= *n_dev) return;
  DevInstance& I = insts[active ? active[blockIdx.x] : blockIdx.x];
  // every field the step end reads is fetched here, in one batch with the
  // partials' addresses; the bookkeeping then runs in registers and writes
  // the marching state back once
  const int stopped0 = I.stopped, nt = I.ntiles, nv = I.nv;
  const double* part = I.part;
  const long long ncells = I.ncells, step_limit = I.step_limit;
  double qref[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qref[v] = I.qref[v];
  const double cfl = I.cfl, dt_fixed = I.dt_fixed, t_end = I.t_end, drop_tol = I.drop_tol;
  double t = I.t, dt = I.dt, norm_first = I.norm_first;
  long long steps = I.steps;
  int flags = I.flags, have_first = I.have_first, last_step = I.last_step;
  if (stopped0) return;
  RedOut R;
  reduce_parts(nt, part, true, true, R);
  if (threadIdx.x != 0) return;
  double comb, nrm[5];
  norms_from_sums(nv, ncells, qref, R.s, nrm, comb);
  if (!have_first) {
    norm_first = comb;
    have_first = 1;
  }
  const double drop = norm_first > 0.0 ? comb / norm_first : 0.0;
  t = last_step ? t_end : t + dt;
  const double dt_last = dt;
  steps += 1;
  int stopped = 0;
  if (R.bad) {
    flags |= FLAG_NONPHYS;
    stopped = 1;
  }
  if (drop_tol > 0.0 && drop <= drop_tol) {
    flags |= FLAG_CONVERGED;
    stopped = 1;
  }
  if (steps >= step_limit) {
    flags |= FLAG_STEPLIMIT;
    stopped = 1;
  }
  // next time step (the rule of next_dt)
  if (!stopped) {
    dt = dt_fixed > 0.0 ? dt_fixed : cfl * R.mn;
    last_step = 0;
    if (t_end > 0.0) {
      if (t >= t_end) {
        stopped = 1;
        flags |= FLAG_TEND;
      } else if (dt >= t_end - t) {
        dt = t_end - t;
        last_step = 1;
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) I.norms[v] = nrm[v];
  I.norm = comb;
  I.norm_first = norm_first;
  I.have_first = have_first;
  I.drop = drop;
  I.t = t;
  I.dt_last = dt_last;
  I.steps = steps;
  I.raw_min = R.mn;
  I.flags = flags;
  I.stopped = stopped;
  I.dt = dt;
  I.last_step = last_step;
}

__global__ __launch_bounds__(kRedThreads) void k_cfl_init(DevInstance* insts, const int* active,
                                                         int n) {
  DevInstance& I = insts[active ? active[blockIdx.x] : blockIdx.x];
  RedOut R;
  reduce_parts(I.ntiles, I.part, false, true, R);
  if (threadIdx.x != 0) return;
  I.raw_min = R.mn;
  I.flags = R.bad ? FLAG_NONPHYS : 0;
  I.stopped = R.bad ? 1 : 0;
}

__global__ __launch_bounds__(kRedThreads) void k_rnorms(DevInstance* insts, const int* active,
                                                       int n) {
  DevInstance& I = insts[active ? active[blockIdx.x] : blockIdx.x];
  const int nv = I.nv;
  const long long ncells = I.ncells;
  double qref[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) qref[v] = I.qref[v];
  RedOut R;
  reduce_parts(I.ntiles, I.part, true, false, R);
  if (threadIdx.x != 0) return;
  double comb, rn[5];
  norms_from_sums(nv, ncells, qref, R.s, rn, comb);
#pragma unroll
  for (int v = 0; v < 5; ++v) I.rnorms[v] = rn[v];
}

// One thread per ghost cell.  Segment = (block, face): both layers.
__global__ void k_ghosts(const DevBlock* __restrict__ blocks, const GhostSeg* __restrict__ segs,
                         int nseg, long long ncells, int nv, double* __restrict__ out) {
  const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ncells) return;
  int s = 0;
  while (s + 1 < nseg && segs[s + 1].cell_off <= x) ++s;
  const GhostSeg& G = segs[s];
  const long long loc = x - G.cell_off;
  const long long per = (long long)G.n1 * G.n2;
  const int g = 1 + (int)(loc / per);
  const long long rem = loc % per;
  const int t2 = (int)(rem / G.n1), t1 = (int)(rem % G.n1);
  const DevBlock& B = blocks[G.blk];
  const int d = G.face >> 1, side = G.face & 1;
  const int n = d == 0 ? B.ni : (d == 1 ? B.nj : B.nk);
  const int along = side == 0 ? -g : n - 1 + g;
  int i, j, k;
  if (d == 0) { i = along; j = t1; k = t2; }
  else if (d == 1) { i = t1; j = along; k = t2; }
  else { i = t1; j = t2; k = along; }
  double q[5];
  if (nv == 4) resolve_cell<4>(blocks, B, 0, i, j, k, q);
  else resolve_cell<5>(blocks, B, 0, i, j, k, q);
  double* o = out + G.out_off + (long long)(g - 1) * nv * per + rem;
  for (int v = 0; v < nv; ++v) o[(long long)v * per] = q[v];
}

}  // namespace

hipError_t launch_prepare(hipStream_t s, DevInstance* insts, const int* active, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prepare, dim3((n + 63) / 64), dim3(64), 0, s, insts, active, n);
  return hipGetLastError();
}
hipError_t launch_finalize(hipStream_t s, DevInstance* insts, const int* active, int n,
                           const int* n_dev) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(n), dim3(kRedThreads), 0, s, insts, active, n, n_dev);
  return hipGetLastError();
}
hipError_t launch_cfl_init(hipStream_t s, DevInstance* insts, const int* active, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cfl_init, dim3(n), dim3(kRedThreads), 0, s, insts, active, n);
  return hipGetLastError();
}
hipError_t launch_rnorms(hipStream_t s, DevInstance* insts, const int* active, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rnorms, dim3(n), dim3(kRedThreads), 0, s, insts, active, n);
  return hipGetLastError();
}
hipError_t launch_ghosts(hipStream_t s, const DevBlock* blocks, const GhostSeg* segs, int nseg,
                         long long ncells, int nv, double* out) {
  if (ncells <= 0) return hipSuccess;
  const long long nb = (ncells + 255) / 256;
  hipLaunchKernelGGL(k_ghosts, dim3((unsigned)nb), dim3(256), 0, s, blocks, segs, nseg, ncells, nv,
                     out);
  return hipGetLastError();
}

}  // namespace fvk
