// 2D stage kernels: MUSCL + Roe residual, SSP-RK3 stage update and the
// fused reductions, one wavefront per tile.
//
// A tile is 64 consecutive columns i (lane = column) by n rows.  The wave
// marches up the rows.  At row j it
//   - loads Q(j+1) of its column (the j-stencil needs rows j-2 .. j+1 and
//     rows j-1, j are carried in registers),
//   - forms the j-face flux at j-1/2 from the carried extrapolation of cell
//     j-1 and the one of cell j, and with it completes the residual of row
//     j-1, which it then updates and stores (coalesced along i),
//   - forms the i-face flux at i-1/2 of row j: the neighbour values come
//     from lane shuffles, the three halo cells (i0-2, i0-1, i0+ncol) from
//     lanes 0..2, and the flux leaving through i+1/2 is the next lane's
//     i-1/2 flux.  The tile's right-edge fluxes are formed 64 rows at a time
//     by a batched pre-pass (lane r: row r), so every face flux of the tile
//     is formed exactly once, except the shared edges between tiles.
// Ghost cells are never stored; reads outside the block go through the
// boundary rule (resolve_cell).
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

template <typename T>
struct Ctx2D {
  const DevBlock* blocks;
  const DevBlock* B;
  int buf;  // stage input buffer
  Recon<T> rc;
  T gm1, efix;
};

// load one cell (interior fast path, boundary rule otherwise)
__device__ __forceinline__ void load2d(const DevBlock* blocks, const DevBlock& B, int buf, int i,
                                       int j, double (&q)[4]) {
  if (i >= 0 && i < B.ni && j >= 0 && j < B.nj) {
    const double* s = B.u[buf] + (long long)j * B.ni + i;
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = s[v * B.ncell];
  } else {
    resolve_cell<4>(blocks, B, buf, i, j, 0, q);
  }
}

// area vector of i-face (i, j) and j-face (i, j), from nodes or uniform
__device__ __forceinline__ void ivec(const DevBlock& B, double xa, double ya, double xb,
                                     double yb, double (&S)[2]) {
  // nodes a = (i, j), b = (i, j+1)
  if (B.xn) {
    S[0] = yb - ya;
    S[1] = -(xb - xa);
  } else {
    S[0] = B.area[0];
    S[1] = 0.0;
  }
}
__device__ __forceinline__ void jvec(const DevBlock& B, double xa, double ya, double xb,
                                     double yb, double (&S)[2]) {
  // nodes a = (i, j), b = (i+1, j)
  if (B.xn) {
    S[0] = -(yb - ya);
    S[1] = xb - xa;
  } else {
    S[0] = 0.0;
    S[1] = B.area[1];
  }
}

template <typename T>
__device__ __forceinline__ void face_flux2d(const Ctx2D<T>& C, const T (&qL)[4], const T (&qR)[4],
                                            const double (&S)[2], T (&G)[4]) {
  T n[2], area;
  if (C.B->xn) {
    const double A = sqrt(S[0] * S[0] + S[1] * S[1]);
    const double iA = 1.0 / A;
    n[0] = T(S[0] * iA);
    n[1] = T(S[1] * iA);
    area = T(A);
  } else {
    area = T(S[0] + S[1]);  // one component is zero
    n[0] = T(S[0] != 0.0 ? 1.0 : 0.0);
    n[1] = T(S[1] != 0.0 ? 1.0 : 0.0);
  }
  roe_flux<T, 2>(qL, qR, n, area, C.gm1, C.efix, G);
}

// i-face flux at the right edge of the tile for row jr (column ie = i0+ncol)
template <typename T>
__device__ void edge_face(const Ctx2D<T>& C, int ie, int jr, T (&G)[4]) {
  const DevBlock& B = *C.B;
  double a[4], b[4], c[4], d[4];
  load2d(C.blocks, B, C.buf, ie - 2, jr, a);
  load2d(C.blocks, B, C.buf, ie - 1, jr, b);
  load2d(C.blocks, B, C.buf, ie, jr, c);
  load2d(C.blocks, B, C.buf, ie + 1, jr, d);
  T qL[4], qR[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T ta = T(a[v]), tb = T(b[v]), tc = T(c[v]), td = T(d[v]);
    T ep, em, ep2, em2;
    extrap(C.rc, tb - ta, tc - tb, ep, em);    // cell ie-1
    extrap(C.rc, tc - tb, td - tc, ep2, em2);  // cell ie
    qL[v] = tb + ep;
    qR[v] = tc - em2;
  }
  double S[2];
  if (B.xn)
    ivec(B, nodex(B, ie, jr), nodey(B, ie, jr), nodex(B, ie, jr + 1), nodey(B, ie, jr + 1), S);
  else
    ivec(B, 0, 0, 0, 0, S);
  face_flux2d(C, qL, qR, S, G);
}

template <int MODE, typename T>
__device__ void tile2d(const DevTile& tl, const DevBlock* __restrict__ blocks,
                       DevInstance& I, double* __restrict__ rout, int lane) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni;
  const int i0 = tl.i0, j0 = tl.j0, n = tl.n, nc = tl.ncol;
  const int i = i0 + lane;
  const bool act = lane < nc;
  const int ic = act ? i : ni - 1;  // safe column for inactive lanes
  const int bin = MODE == 0 ? 0 : MODE - 1;
  const int bout = MODE == 1 ? 1 : (MODE == 2 ? 2 : 0);
  const bool curv = B.xn != nullptr;

  Ctx2D<T> C;
  C.blocks = blocks;
  C.B = &B;
  C.buf = bin;
  C.rc.lim = I.limiter;
  C.rc.heps = T(0.5 * I.eps);
  C.rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  C.rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  C.gm1 = T(I.gamma - 1.0);
  C.efix = T(I.efix);
  const double gamma = I.gamma;
  const double dt = I.dt;

  const double* __restrict__ Uin = B.u[bin];
  double* __restrict__ Uout = B.u[bout];
  const double* __restrict__ Un = B.u[0];
  const long long ncell = B.ncell;

  // ---- prologue: rows j0-2, j0-1, j0 of the own column
  double qa_d[4], qb_d[4], q0_d[4];
  load2d(blocks, B, bin, ic, j0 - 2, qa_d);
  load2d(blocks, B, bin, ic, j0 - 1, qb_d);
  load2d(blocks, B, bin, ic, j0, q0_d);
  T qm1[4], q0[4], epm1[4];
  double qm1_d[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T ta = T(qa_d[v]), tb = T(qb_d[v]), tc = T(q0_d[v]);
    T em;
    extrap(C.rc, tb - ta, tc - tb, epm1[v], em);
    qm1[v] = tb;
    q0[v] = tc;
    qm1_d[v] = qb_d[v];
  }
  // node rows j-1 (m), j (0), j+1 (1): own column and the next one
  double xm = 0, ym = 0, xmr = 0, ymr = 0, x0 = 0, y0 = 0, x0r = 0, y0r = 0;
  if (curv) {
    x0 = nodex(B, ic, j0);
    y0 = nodey(B, ic, j0);
    x0r = nodex(B, ic + 1, j0);
    y0r = nodey(B, ic + 1, j0);
  }

  double ri[4] = {0, 0, 0, 0};  // i-direction part of the residual of the carried row
  T gbot[4] = {T(0), T(0), T(0), T(0)};
  T edge[4] = {T(0), T(0), T(0), T(0)};
  double nacc[4] = {0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  for (int r = 0; r <= n; ++r) {
    const int j = j0 + r;
    if (r < n && (r & 63) == 0) {
      // right-edge i-faces of rows j .. j+63 of this tile, one per lane
      const int rr = min(lane, n - r - 1);
      edge_face(C, i0 + nc, j + rr, edge);
    }
    // ---- Q(j+1) of the own column
    double qn_d[4];
    load2d(blocks, B, bin, ic, j + 1, qn_d);
    T qn[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) qn[v] = T(qn_d[v]);
    double x1 = 0, y1 = 0, x1r = 0, y1r = 0;
    if (curv && r < n) {
      x1 = nodex(B, ic, j + 1);
      y1 = nodey(B, ic, j + 1);
      x1r = nodex(B, ic + 1, j + 1);
      y1r = nodey(B, ic + 1, j + 1);
    }
    // ---- j-face at j-1/2
    T ep0[4], em0[4], qL[4], qR[4], Gj[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      extrap(C.rc, q0[v] - qm1[v], qn[v] - q0[v], ep0[v], em0[v]);
      qL[v] = qm1[v] + epm1[v];
      qR[v] = q0[v] - em0[v];
    }
    {
      double S[2];
      jvec(B, x0, y0, x0r, y0r, S);
      face_flux2d(C, qL, qR, S, Gj);
    }
    // ---- complete, update and store row j-1
    if (r >= 1 && act) {
      const long long idx = (long long)(j - 1) * ni + i;
      double R[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) R[v] = ri[v] + ((double)Gj[v] - (double)gbot[v]);
      double vol;
      if (curv) {
        vol = 0.5 * ((x0r - xm) * (y0 - ymr) - (x0 - xmr) * (y0r - ym));
      } else {
        vol = B.vol;
      }
      if (MODE == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          rout[B.out_off + v * ncell + idx] = R[v];
          const double rv = R[v] / vol;
          nacc[v] += rv * rv;
        }
      } else {
        const double f = dt / vol;
        double out[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double us = qm1_d[v] - f * R[v];
          if (MODE == 1) {
            out[v] = us;
          } else if (MODE == 2) {
            out[v] = 0.75 * Un[v * ncell + idx] + 0.25 * us;
          } else {
            out[v] = (1.0 / 3.0) * Un[v * ncell + idx] + (2.0 / 3.0) * us;
          }
          Uout[v * ncell + idx] = out[v];
        }
        if (MODE == 1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double rv = R[v] / vol;
            nacc[v] += rv * rv;
          }
        }
        if (MODE == 3) {
          double Sb[2][3];
          if (curv) {
            Sb[0][0] = 0.5 * ((y0 - ym) + (y0r - ymr));
            Sb[0][1] = -0.5 * ((x0 - xm) + (x0r - xmr));
            Sb[1][0] = -0.5 * ((ymr - ym) + (y0r - y0));
            Sb[1][1] = 0.5 * ((xmr - xm) + (x0r - x0));
          } else {
            Sb[0][0] = B.area[0];
            Sb[0][1] = 0.0;
            Sb[1][0] = 0.0;
            Sb[1][1] = B.area[1];
          }
          Sb[0][2] = Sb[1][2] = 0.0;
          dmin = fmin(dmin, cell_dt_limit<2>(out, Sb, vol, gamma, bad));
        }
      }
    }
    // ---- i-faces of row j
    if (r < n) {
      double hv_d[4] = {0, 0, 0, 0};
      if (lane < 3) {
        const int hi = lane == 0 ? i0 - 1 : (lane == 1 ? i0 - 2 : i0 + nc);
        load2d(blocks, B, bin, hi, j, hv_d);
      }
      T Gi[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T hv = T(hv_d[v]);
        const T left = __shfl(q0[v], lane - 1 < 0 ? 0 : lane - 1, kWave);
        const T right = __shfl(q0[v], lane + 1 > 63 ? 63 : lane + 1, kWave);
        const T h1 = __shfl(hv, 1, kWave);  // Q(i0-2)
        const T h2 = __shfl(hv, 2, kWave);  // Q(i0+ncol)
        const T qim1 = lane == 0 ? hv : left;
        const T qip1 = lane == nc - 1 ? h2 : right;
        T epc, emc;
        extrap(C.rc, q0[v] - qim1, qip1 - q0[v], epc, emc);
        // extrapolation of cell i-1 towards i-1/2
        const T epl = __shfl(epc, lane - 1 < 0 ? 0 : lane - 1, kWave);
        T ep0l, em0l;
        extrap(C.rc, hv - h1, q0[v] - hv, ep0l, em0l);  // cell i0-1 (lane 0)
        const T epi = lane == 0 ? ep0l : epl;
        qL[v] = qim1 + epi;
        qR[v] = q0[v] - emc;
      }
      double S[2];
      ivec(B, x0, y0, x1, y1, S);
      face_flux2d(C, qL, qR, S, Gi);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T gr = __shfl(Gi[v], lane + 1 > 63 ? 63 : lane + 1, kWave);
        const T ge = __shfl(edge[v], r & 63, kWave);
        const T grr = lane == nc - 1 ? ge : gr;
        ri[v] = (double)grr - (double)Gi[v];
        gbot[v] = Gj[v];
      }
    }
    // ---- shift the carried rows
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      qm1[v] = q0[v];
      q0[v] = qn[v];
      epm1[v] = ep0[v];
      qm1_d[v] = q0_d[v];
      q0_d[v] = qn_d[v];
    }
    xm = x0; ym = y0; xmr = x0r; ymr = y0r;
    x0 = x1; y0 = y1; x0r = x1r; y0r = y1r;
  }

  // ---- per-tile partials (fixed-order wave reductions)
  double* part = I.part + (long long)tl.local * kPartStride;
  if (MODE == 0 || MODE == 1) {
    double s[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = wave_sum(nacc[v]);
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) part[v] = s[v];
      part[4] = 0.0;
    }
  }
  if (MODE == 3) {
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      part[5] = m;
      part[6] = (double)b;
    }
  }
}

template <int MODE, typename T>
__global__ __launch_bounds__(256) void k_stage2d(const DevTile* __restrict__ tiles,
                                                 const int* __restrict__ ntiles_p,
                                                 const DevBlock* __restrict__ blocks,
                                                 DevInstance* __restrict__ insts,
                                                 double* __restrict__ rout) {
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwv = blockDim.x >> 6;
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x * nwv + wid; t < ntiles; t += gridDim.x * nwv) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;
    tile2d<MODE, T>(tl, blocks, I, rout, lane);
  }
}

// Spectral minimum and physical check of U^n (buffer 0), per tile.
__global__ __launch_bounds__(256) void k_cfl2d(const DevTile* __restrict__ tiles,
                                               const int* __restrict__ ntiles_p,
                                               const DevBlock* __restrict__ blocks,
                                               DevInstance* __restrict__ insts) {
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwv = blockDim.x >> 6;
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x * nwv + wid; t < ntiles; t += gridDim.x * nwv) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    const DevBlock& B = blocks[tl.blk];
    const bool act = lane < tl.ncol;
    const int i = tl.i0 + lane;
    double dmin = INFINITY;
    int bad = 0;
    if (act) {
      for (int r = 0; r < tl.n; ++r) {
        const int j = tl.j0 + r;
        const long long idx = (long long)j * B.ni + i;
        double q[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = B.u[0][v * B.ncell + idx];
        double Sb[2][3], vol;
        if (B.xn) {
          const double xa = nodex(B, i, j), ya = nodey(B, i, j);
          const double xb = nodex(B, i + 1, j), yb = nodey(B, i + 1, j);
          const double xc = nodex(B, i, j + 1), yc = nodey(B, i, j + 1);
          const double xd = nodex(B, i + 1, j + 1), yd = nodey(B, i + 1, j + 1);
          vol = 0.5 * ((xd - xa) * (yc - yb) - (xc - xb) * (yd - ya));
          Sb[0][0] = 0.5 * ((yc - ya) + (yd - yb));
          Sb[0][1] = -0.5 * ((xc - xa) + (xd - xb));
          Sb[1][0] = -0.5 * ((yb - ya) + (yd - yc));
          Sb[1][1] = 0.5 * ((xb - xa) + (xd - xc));
        } else {
          vol = B.vol;
          Sb[0][0] = B.area[0];
          Sb[0][1] = 0.0;
          Sb[1][0] = 0.0;
          Sb[1][1] = B.area[1];
        }
        Sb[0][2] = Sb[1][2] = 0.0;
        dmin = fmin(dmin, cell_dt_limit<2>(q, Sb, vol, I.gamma, bad));
      }
    }
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      double* part = I.part + (long long)tl.local * kPartStride;
      part[5] = m;
      part[6] = (double)b;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_stage2d(int mode, int fp32, int grid, int block, hipStream_t s, const DevTile* tiles,
                          const int* ntiles, const DevBlock* blocks, DevInstance* insts,
                          double* rout) {
#define FV_L2(M, T) hipLaunchKernelGGL((k_stage2d<M, T>), dim3(grid), dim3(block), 0, s, tiles, ntiles, blocks, insts, rout)
  if (fp32) {
    switch (mode) {
      case 0: FV_L2(0, float); break;
      case 1: FV_L2(1, float); break;
      case 2: FV_L2(2, float); break;
      default: FV_L2(3, float); break;
    }
  } else {
    switch (mode) {
      case 0: FV_L2(0, double); break;
      case 1: FV_L2(1, double); break;
      case 2: FV_L2(2, double); break;
      default: FV_L2(3, double); break;
    }
  }
#undef FV_L2
  return hipGetLastError();
}

hipError_t launch_cfl2d(int grid, int block, hipStream_t s, const DevTile* tiles, const int* ntiles,
                        const DevBlock* blocks, DevInstance* insts) {
  hipLaunchKernelGGL(k_cfl2d, dim3(grid), dim3(block), 0, s, tiles, ntiles, blocks, insts);
  return hipGetLastError();
}

const void* stage2d_kernel_ptr(int mode, int fp32) {
  if (fp32) {
    switch (mode) {
      case 0: return (const void*)&k_stage2d<0, float>;
      case 1: return (const void*)&k_stage2d<1, float>;
      case 2: return (const void*)&k_stage2d<2, float>;
      default: return (const void*)&k_stage2d<3, float>;
    }
  }
  switch (mode) {
    case 0: return (const void*)&k_stage2d<0, double>;
    case 1: return (const void*)&k_stage2d<1, double>;
    case 2: return (const void*)&k_stage2d<2, double>;
    default: return (const void*)&k_stage2d<3, double>;
  }
}

}  // namespace fvk
