// 3D stage kernels (uniform grids): MUSCL + Roe residual, SSP-RK3 stage
// update and fused reductions.  One workgroup per tile.
//
// A tile is 64 columns i (lane) by ny rows j (one wavefront per row) and
// marches over n planes k.  The workgroup has NY + 1 waves: waves 0..NY-1 own
// the rows; wave NY owns no cells: it fetches the four j-halo rows of each
// plane (one plane ahead) and forms the j-face flux at the tile's top edge.
// Per plane k:
//   - each row wave forms the k-face flux at k-1/2 (planes k-1, k, k+1 of its
//     column in registers, k+2 in flight), completes the residual of plane
//     k-1, applies the stage update and stores it;
//   - the plane k is staged in LDS (rows j0-2 .. j0+ny+1); every row wave forms
//     its j-face flux at j-1/2 from LDS and its i-face flux at i-1/2 (DPP lane
//     shifts, halo lanes, right-edge pre-pass in LDS as in 2D); the j-face
//     fluxes are exchanged through LDS and each row keeps the in-plane part
//     of its residual for the next plane.
// Every face flux of the tile is formed once (tile edges aside).
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

template <typename T>
struct Ctx3D {
  const DevBlock* blocks;
  const DevBlock* B;
  int buf;
  Recon<T> rc;
  FluxK<T> K;
  T ax, ay, az;
};

// i-face at column ie of row j, plane kr, from the four cells ie-2 .. ie+1
template <typename T>
__device__ void edge_face3(const Ctx3D<T>& C, int ie, int j, int kr, T (&G)[5]) {
  const DevBlock& B = *C.B;
  double a[5], b[5], c[5], d[5];
  load_cell<5>(C.blocks, B, C.buf, ie - 2, j, kr, a);
  load_cell<5>(C.blocks, B, C.buf, ie - 1, j, kr, b);
  load_cell<5>(C.blocks, B, C.buf, ie, j, kr, c);
  load_cell<5>(C.blocks, B, C.buf, ie + 1, j, kr, d);
  T qL[5], qR[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T ta = T(a[v]), tb = T(b[v]), tc = T(c[v]), td = T(d[v]);
    T ep, em, ep2, em2;
    extrap(C.rc, tb - ta, tc - tb, ep, em);
    extrap(C.rc, tc - tb, td - tc, ep2, em2);
    qL[v] = tb + ep;
    qR[v] = tc - em2;
  }
  roe_flux<T, 3, 0>(qL, qR, nullptr, C.ax, C.K, G);
}

template <typename T, int NY>
struct Smem3 {
  T q[(NY + 4) * 5 * kWave];    // plane k, rows j0-2 .. j0+NY+1
  T f[(NY + 1) * 5 * kWave];    // j-face fluxes at j-1/2, rows j0 .. j0+NY
  T edge[NY][kWave * 5];        // right-edge i-face fluxes, per row wave
  T halo[NY][3][5];             // i-halo cells of plane k: i0-1, i0-2, i0+ncol
  double red[(NY + 1) * 8];
};

template <typename T>
__device__ __forceinline__ void setup3(Ctx3D<T>& C, const DevBlock* blocks, const DevBlock& B, int buf,
                                       const DevInstance& I) {
  C.blocks = blocks;
  C.B = &B;
  C.buf = buf;
  C.rc.lim = I.limiter;
  C.rc.heps = T(0.5 * I.eps);
  C.rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  C.rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  C.K.gm1 = T(I.gamma - 1.0);
  C.K.efix = T(I.efix);
  C.K.iefix = T(I.efix > 0.0 ? 1.0 / I.efix : 0.0);
  C.ax = T(B.area[0]);
  C.ay = T(B.area[1]);
  C.az = T(B.area[2]);
}

// j-face flux at j-1/2 from the LDS rows j-2 .. j+1 (slots s .. s+3), to SF(s)
template <typename T, int NY>
__device__ __forceinline__ void jface3(const Ctx3D<T>& C, Smem3<T, NY>& sm, int s, int lane) {
  T qL[5], qR[5], Gj[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T a = sm.q[(s * 5 + v) * kWave + lane], b = sm.q[((s + 1) * 5 + v) * kWave + lane];
    const T c = sm.q[((s + 2) * 5 + v) * kWave + lane], d = sm.q[((s + 3) * 5 + v) * kWave + lane];
    T ep, em, ep2, em2;
    extrap(C.rc, b - a, c - b, ep, em);
    extrap(C.rc, c - b, d - c, ep2, em2);
    qL[v] = b + ep;
    qR[v] = c - em2;
  }
  roe_flux<T, 3, 1>(qL, qR, nullptr, C.ay, C.K, Gj);
#pragma unroll
  for (int v = 0; v < 5; ++v) sm.f[(s * 5 + v) * kWave + lane] = Gj[v];
}

// The helper wave: per plane, stage the j-halo rows and the i-halo cells in
// LDS (fetched one plane ahead) and form the tile's top-edge j-face flux.
template <int MODE, typename T, int NY>
__device__ void helper3d(const DevTile& tl, const DevBlock* __restrict__ blocks, const DevInstance& I,
                         int lane, Smem3<T, NY>& sm) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, n = tl.n, nc = tl.ncol, ny = tl.ny;
  const int bin = MODE == 0 ? 0 : MODE - 1;
  const int ic = lane < nc ? i0 + lane : ni - 1;
  Ctx3D<T> C;
  setup3(C, blocks, B, bin, I);
  const int hrows[4] = {j0 - 2, j0 - 1, j0 + ny, j0 + ny + 1};
  const int hslot[4] = {0, 1, ny + 2, ny + 3};
  // i-halo lane assignment: lane = 3 * row + which, which 0: i0-1, 1: i0-2, 2: i0+ncol
  const int hr = lane / 3, hw = lane - 3 * (lane / 3);
  const bool hlane = hr < ny;
  const int hcol = hw == 0 ? i0 - 1 : (hw == 1 ? i0 - 2 : i0 + nc);
  double hrow[4][5], hcell[5] = {0, 0, 0, 0, 0};
  if (n > 0) {
#pragma unroll
    for (int h = 0; h < 4; ++h) load_cell<5>(blocks, B, bin, ic, hrows[h], k0, hrow[h]);
    if (hlane) load_cell<5>(blocks, B, bin, hcol, j0 + hr, k0, hcell);
  }
  for (int r = 0; r < n; ++r) {
    const int k = k0 + r;
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.q[(hslot[h] * 5 + v) * kWave + lane] = T(hrow[h][v]);
    if (hlane) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.halo[hr][hw][v] = T(hcell[v]);
    }
    if (r + 1 < n) {
#pragma unroll
      for (int h = 0; h < 4; ++h) load_cell<5>(blocks, B, bin, ic, hrows[h], k + 1, hrow[h]);
      if (hlane) load_cell<5>(blocks, B, bin, hcol, j0 + hr, k + 1, hcell);
    }
    __syncthreads();
    jface3<T, NY>(C, sm, ny, lane);
    __syncthreads();
  }
}

template <int MODE, typename T, int NY>
__device__ void tile3d(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                       double* __restrict__ rout, int lane, int w, Smem3<T, NY>& sm) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni, nj = B.nj;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, n = tl.n, nc = tl.ncol, ny = tl.ny;
  const bool rowact = w < ny;
  const int j = j0 + w;
  const int i = i0 + lane;
  const bool act = lane < nc;
  const int ic = act ? i : ni - 1;
  const int jc = rowact ? j : j0;
  const int last = nc - 1;
  const int bin = MODE == 0 ? 0 : MODE - 1;
  const int bout = MODE == 1 ? 1 : (MODE == 2 ? 2 : 0);

  Ctx3D<T> C;
  setup3(C, blocks, B, bin, I);
  const double gamma = I.gamma;
  const double dt = I.dt;
  const double vol = B.vol;
  const double ivol = 1.0 / vol;
  const long long ncell = B.ncell;
  double* __restrict__ Uout = B.u[bout];
  const double* __restrict__ Un = B.u[0];

  // ---- prologue
  double qm1[5] = {0, 0, 0, 0, 0}, q0[5] = {0, 0, 0, 0, 0}, qn[5] = {0, 0, 0, 0, 0};
  T epm1[5] = {T(0), T(0), T(0), T(0), T(0)};
  if (rowact) {
    double qa[5];
    load_cell<5>(blocks, B, bin, ic, jc, k0 - 2, qa);
    load_cell<5>(blocks, B, bin, ic, jc, k0 - 1, qm1);
    load_cell<5>(blocks, B, bin, ic, jc, k0, q0);
    load_cell<5>(blocks, B, bin, ic, jc, k0 + 1, qn);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      T em;
      extrap(C.rc, T(qm1[v]) - T(qa[v]), T(q0[v]) - T(qm1[v]), epm1[v], em);
    }
  }

  double rg[5] = {0, 0, 0, 0, 0};
  double nacc[5] = {0, 0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  for (int r = 0; r <= n; ++r) {
    const int k = k0 + r;
    const bool more = r < n;
    T Gk[5], ep0[5];
    double qnn[5] = {0, 0, 0, 0, 0};
    if (rowact) {
      // ---- (1) the next plane of the own column
      if (more) load_cell<5>(blocks, B, bin, ic, jc, k + 2, qnn);
      // ---- (2) right-edge i-face fluxes of the next 64 planes
      if (more && (r & 63) == 0) {
        const int rr = min(lane, n - r - 1);
        T ge[5];
        edge_face3(C, i0 + nc, jc, k + rr, ge);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.edge[w][lane * 5 + v] = ge[v];
        __builtin_amdgcn_wave_barrier();
      }
      // ---- (3) k-face at k-1/2
      T qL[5], qR[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T a = T(qm1[v]), b = T(q0[v]), c = T(qn[v]);
        T em;
        extrap(C.rc, b - a, c - b, ep0[v], em);
        qL[v] = a + epm1[v];
        qR[v] = b - em;
      }
      roe_flux<T, 3, 2>(qL, qR, nullptr, C.az, C.K, Gk);
      // ---- (4) complete plane k-1
      if (r >= 1 && act) {
        const long long idx = ((long long)(k - 1) * nj + j) * ni + i;
        double R[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = rg[v] + (double)Gk[v];
        if (MODE == 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            stg(rout + B.out_off + v * ncell + idx, R[v]);
            const double rv = R[v] * ivol;
            nacc[v] += rv * rv;
          }
        } else {
          const double f = dt * ivol;
          double out[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double us = qm1[v] - f * R[v];
            if (MODE == 1) out[v] = us;
            else if (MODE == 2) out[v] = 0.75 * ldg(Un + v * ncell + idx) + 0.25 * us;
            else out[v] = (1.0 / 3.0) * ldg(Un + v * ncell + idx) + (2.0 / 3.0) * us;
            stg(Uout + v * ncell + idx, out[v]);
          }
          if (MODE == 1) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              const double rv = R[v] * ivol;
              nacc[v] += rv * rv;
            }
          }
          if (MODE == 3) {
            const double Sb[3][3] = {{B.area[0], 0.0, 0.0}, {0.0, B.area[1], 0.0},
                                     {0.0, 0.0, B.area[2]}};
            dmin = fmin(dmin, cell_dt_limit<3>(out, Sb, vol, gamma, bad));
          }
        }
      }
    }
    // ---- (5) in-plane faces of plane k
    if (more) {
      if (rowact) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.q[((w + 2) * 5 + v) * kWave + lane] = T(q0[v]);
      }
      __syncthreads();
      T Gi[5], Gr[5];
      if (rowact) {
        jface3<T, NY>(C, sm, w, lane);
        T qL[5], qR[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T c = T(q0[v]);
          const T h0 = sm.halo[w][0][v];  // Q(i0-1)
          const T h1 = sm.halo[w][1][v];  // Q(i0-2)
          const T h2 = sm.halo[w][2][v];  // Q(i0+ncol)
          const T left = shr1(c);
          const T right = shl1(c);
          const T qim1 = lane == 0 ? h0 : left;
          const T qip1 = lane == last ? h2 : right;
          T epc, emc;
          extrap(C.rc, c - qim1, qip1 - c, epc, emc);
          T ep0l, em0l;
          extrap(C.rc, h0 - h1, c - h0, ep0l, em0l);
          const T epl = shr1(epc);
          qL[v] = qim1 + (lane == 0 ? ep0l : epl);
          qR[v] = c - emc;
        }
        roe_flux<T, 3, 0>(qL, qR, nullptr, C.ax, C.K, Gi);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T ge = sm.edge[w][(r & 63) * 5 + v];
          const T gs = shl1(Gi[v]);
          Gr[v] = lane == last ? ge : gs;
        }
      }
      __syncthreads();
      if (rowact) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
          rg[v] = (((double)Gr[v] - (double)Gi[v]) +
                   ((double)sm.f[((w + 1) * 5 + v) * kWave + lane] -
                    (double)sm.f[(w * 5 + v) * kWave + lane])) -
                  (double)Gk[v];
      }
    }
    if (rowact) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        qm1[v] = q0[v];
        q0[v] = qn[v];
        qn[v] = qnn[v];
        epm1[v] = ep0[v];
      }
    }
  }

  // ---- per-tile partials of this row wave
  if (MODE == 0 || MODE == 1 || MODE == 3) {
    double s[5] = {0, 0, 0, 0, 0};
    double m = 0.0;
    int b = 0;
    if (MODE == 3) {
      m = wave_min(dmin);
      b = wave_or(bad);
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) s[v] = wave_sum(nacc[v]);
    }
    if (lane == 0) {
      if (MODE == 3) {
        sm.red[w * 8 + 5] = m;
        sm.red[w * 8 + 6] = (double)b;
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.red[w * 8 + v] = s[v];
      }
    }
  }
}

// tile partials: the row waves' sums in row order (fixed order)
template <int MODE, int NY>
__device__ void tile_partials3d(const DevTile& tl, DevInstance& I, const double* red) {
  double* part = I.part + (long long)tl.local * kPartStride;
  if (MODE == 3) {
    double mm = INFINITY;
    double bb = 0.0;
    for (int x = 0; x < tl.ny; ++x) {
      mm = fmin(mm, red[x * 8 + 5]);
      bb = fmax(bb, red[x * 8 + 6]);
    }
    part[5] = mm;
    part[6] = bb;
  } else if (MODE == 0 || MODE == 1) {
    for (int v = 0; v < 5; ++v) {
      double a = 0.0;
      for (int x = 0; x < tl.ny; ++x) a += red[x * 8 + v];
      part[v] = a;
    }
  }
}

template <int MODE, typename T, int NY>
__global__ __launch_bounds__(64 * (NY + 1)) void k_stage3d(const DevTile* __restrict__ tiles,
                                                           const int* __restrict__ ntiles_p,
                                                           const DevBlock* __restrict__ blocks,
                                                           DevInstance* __restrict__ insts,
                                                           double* __restrict__ rout) {
  __shared__ Smem3<T, NY> sm;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;
    // the row waves and the helper wave take the same barriers
    if (w < NY) tile3d<MODE, T, NY>(tl, blocks, I, rout, lane, w, sm);
    else helper3d<MODE, T, NY>(tl, blocks, I, lane, sm);
    __syncthreads();
    if (threadIdx.x == 0) tile_partials3d<MODE, NY>(tl, I, sm.red);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_cfl3d(const DevTile* __restrict__ tiles,
                                               const int* __restrict__ ntiles_p,
                                               const DevBlock* __restrict__ blocks,
                                               DevInstance* __restrict__ insts) {
  __shared__ double s_m[4];
  __shared__ int s_b[4];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    const DevBlock& B = blocks[tl.blk];
    const double Sb[3][3] = {{B.area[0], 0, 0}, {0, B.area[1], 0}, {0, 0, B.area[2]}};
    double dmin = INFINITY;
    int bad = 0;
    const int i = tl.i0 + lane;
    if (lane < tl.ncol) {
      for (int y = w; y < tl.ny; y += 4)
        for (int r = 0; r < tl.n; ++r) {
          const long long idx = ((long long)(tl.k0 + r) * B.nj + (tl.j0 + y)) * B.ni + i;
          double q[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) q[v] = ldg(B.u[0] + v * B.ncell + idx);
          dmin = fmin(dmin, cell_dt_limit<3>(q, Sb, B.vol, I.gamma, bad));
        }
    }
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      s_m[w] = m;
      s_b[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double* part = I.part + (long long)tl.local * kPartStride;
      part[5] = fmin(fmin(s_m[0], s_m[1]), fmin(s_m[2], s_m[3]));
      part[6] = (double)(s_b[0] | s_b[1] | s_b[2] | s_b[3]);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_stage3d(int mode, int fp32, int ny, int grid, hipStream_t s, const DevTile* tiles,
                          const int* ntiles, const DevBlock* blocks, DevInstance* insts,
                          double* rout) {
#define FV_L3(M, T, N)                                                                          \
  hipLaunchKernelGGL((k_stage3d<M, T, N>), dim3(grid), dim3(64 * (N + 1)), 0, s, tiles, ntiles, \
                     blocks, insts, rout)
#define FV_L3N(M, T) \
  if (ny == 8) FV_L3(M, T, 8); else FV_L3(M, T, 4)
  if (fp32) {
    switch (mode) {
      case 0: FV_L3N(0, float); break;
      case 1: FV_L3N(1, float); break;
      case 2: FV_L3N(2, float); break;
      default: FV_L3N(3, float); break;
    }
  } else {
    switch (mode) {
      case 0: FV_L3N(0, double); break;
      case 1: FV_L3N(1, double); break;
      case 2: FV_L3N(2, double); break;
      default: FV_L3N(3, double); break;
    }
  }
#undef FV_L3N
#undef FV_L3
  return hipGetLastError();
}

hipError_t launch_cfl3d(int grid, int block, hipStream_t s, const DevTile* tiles, const int* ntiles,
                        const DevBlock* blocks, DevInstance* insts) {
  (void)block;
  hipLaunchKernelGGL(k_cfl3d, dim3(grid), dim3(256), 0, s, tiles, ntiles, blocks, insts);
  return hipGetLastError();
}

const void* stage3d_kernel_ptr(int mode, int fp32, int ny) {
#define FV_P3(M, T) (ny == 8 ? (const void*)&k_stage3d<M, T, 8> : (const void*)&k_stage3d<M, T, 4>)
  if (fp32) {
    switch (mode) {
      case 0: return FV_P3(0, float);
      case 1: return FV_P3(1, float);
      case 2: return FV_P3(2, float);
      default: return FV_P3(3, float);
    }
  }
  switch (mode) {
    case 0: return FV_P3(0, double);
    case 1: return FV_P3(1, double);
    case 2: return FV_P3(2, double);
    default: return FV_P3(3, double);
  }
#undef FV_P3
}

}  // namespace fvk
