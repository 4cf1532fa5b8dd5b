// 2D stage kernels: MUSCL + Roe residual, SSP-RK3 stage update and the
// fused reductions, one wavefront per tile.
//
// A tile is 64 consecutive columns i (lane = column; ncol of them active) by
// n rows.  The wave marches up the rows; at row j it
//   - forms the j-face flux at j-1/2 from the extrapolation of cell j-1
//     (carried) and of cell j (rows j-1, j, j+1 of the own column are in
//     registers; row j+2 is already being fetched for the next step),
//   - completes the residual of row j-1 with it, applies the RK stage update
//     and stores the row (coalesced along i), adding the fused reductions,
//   - forms the i-face flux at i-1/2 of row j.  Neighbour values come from
//     the lanes next door (DPP wave shifts), the three halo cells i0-2,
//     i0-1, i0+ncol from lanes 0..2, and the flux through i+1/2 is the next
//     lane's i-1/2 flux.  The right-edge fluxes of the tile are formed 64 rows
//     at a time by a pre-pass (lane r: row r) and kept in LDS.
// Every face flux of the tile is formed once (tile edges aside).  Ghost cells
// are never stored: reads outside the block follow the boundary rule.
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

constexpr int kWavesPerWG = 4;

template <typename T>
struct Ctx2D {
  const DevBlock* blocks;
  const DevBlock* B;
  int buf;
  Recon<T> rc;
  FluxK<T> K;
};

template <typename T>
__device__ __forceinline__ void setup(Ctx2D<T>& C, const DevBlock* blocks, const DevBlock& B,
                                      int buf, const DevInstance& I) {
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
}

// flux across a face of area vector S (curvilinear) or along axis AX (uniform)
template <typename T, int AX>
__device__ __forceinline__ void face_flux(const Ctx2D<T>& C, const T (&qL)[4], const T (&qR)[4],
                                          double Sx, double Sy, T (&G)[4]) {
  if (C.B->xn) {
    double A, h;
    M<double>::sqrt2(Sx * Sx + Sy * Sy, A, h);
    const double iA = 2.0 * h;
    const T n[2] = {T(Sx * iA), T(Sy * iA)};
    roe_flux<T, 2, -1>(qL, qR, n, T(A), C.K, G);
  } else {
    roe_flux<T, 2, AX>(qL, qR, nullptr, T(C.B->area[AX]), C.K, G);
  }
}

// i-face flux at column ie, row jr from the four cells ie-2 .. ie+1
template <typename T>
__device__ void edge_face(const Ctx2D<T>& C, int ie, int jr, T (&G)[4]) {
  const DevBlock& B = *C.B;
  double a[4], b[4], c[4], d[4];
  load_cell<4>(C.blocks, B, C.buf, ie - 2, jr, 0, a);
  load_cell<4>(C.blocks, B, C.buf, ie - 1, jr, 0, b);
  load_cell<4>(C.blocks, B, C.buf, ie, jr, 0, c);
  load_cell<4>(C.blocks, B, C.buf, ie + 1, jr, 0, d);
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
  double Sx = 0.0, Sy = 0.0;
  if (B.xn) {
    Sx = nodey(B, ie, jr + 1) - nodey(B, ie, jr);
    Sy = -(nodex(B, ie, jr + 1) - nodex(B, ie, jr));
  }
  face_flux<T, 0>(C, qL, qR, Sx, Sy, G);
}

template <int MODE, typename T>
__device__ void tile2d(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                       double* __restrict__ rout, int lane, T* __restrict__ s_edge) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni;
  const int i0 = tl.i0, j0 = tl.j0, n = tl.n, nc = tl.ncol;
  const int i = i0 + lane;
  const bool act = lane < nc;
  const int ic = act ? i : ni - 1;  // safe column for idle lanes
  const int last = nc - 1;          // lane owning the tile's right edge
  const int bin = MODE == 0 ? 0 : MODE - 1;
  const int bout = MODE == 1 ? 1 : (MODE == 2 ? 2 : 0);
  const bool curv = B.xn != nullptr;
  // halo lanes: 0 -> column i0-1, 1 -> i0-2, 2 -> i0+ncol
  const int hcol = lane == 0 ? i0 - 1 : (lane == 1 ? i0 - 2 : i0 + nc);
  const bool hlane = lane < 3;

  Ctx2D<T> C;
  setup(C, blocks, B, bin, I);
  const double gamma = I.gamma;
  const double dt = I.dt;
  double* __restrict__ Uout = B.u[bout];
  const double* __restrict__ Un = B.u[0];
  const long long ncell = B.ncell;

  // ---- prologue: rows j0-2 .. j0+1 of the own column, nodes of row j0
  double qa[4], qm1[4], q0[4], qn[4];
  load_cell<4>(blocks, B, bin, ic, j0 - 2, 0, qa);
  load_cell<4>(blocks, B, bin, ic, j0 - 1, 0, qm1);
  load_cell<4>(blocks, B, bin, ic, j0, 0, q0);
  load_cell<4>(blocks, B, bin, ic, j0 + 1, 0, qn);
  double xm = 0, ym = 0, x0 = 0, y0 = 0, xhm = 0, yhm = 0, xh0 = 0, yh0 = 0;
  if (curv) {
    x0 = nodex(B, ic, j0);
    y0 = nodey(B, ic, j0);
    double hx = 0, hy = 0;
    if (lane == 2) {
      hx = nodex(B, i0 + nc, j0);
      hy = nodey(B, i0 + nc, j0);
    }
    xh0 = lane_value(hx, 2);
    yh0 = lane_value(hy, 2);
  }
  T epm1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T em;
    extrap(C.rc, T(qm1[v]) - T(qa[v]), T(q0[v]) - T(qm1[v]), epm1[v], em);
  }

  double rg[4] = {0, 0, 0, 0};  // (G_i+1/2 - G_i-1/2) - G_j-1/2 of the carried row
#ifdef FV_EDGE_REGS
  T edge_r[4] = {T(0), T(0), T(0), T(0)};
#endif
  double nacc[4] = {0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  for (int r = 0; r <= n; ++r) {
    const int j = j0 + r;
    const bool more = r < n;
    // ---- (1) loads for later in this step and for the next step
    double qnn[4] = {0, 0, 0, 0}, hv[4] = {0, 0, 0, 0}, un[4] = {0, 0, 0, 0};
    double x1 = 0, y1 = 0, hx1 = 0, hy1 = 0;
    if (more) {
      load_cell<4>(blocks, B, bin, ic, j + 2, 0, qnn);
      if (hlane) load_cell<4>(blocks, B, bin, hcol, j, 0, hv);
      if (curv) {
        x1 = nodex(B, ic, j + 1);
        y1 = nodey(B, ic, j + 1);
        if (lane == 2) {
          hx1 = nodex(B, i0 + nc, j + 1);
          hy1 = nodey(B, i0 + nc, j + 1);
        }
      }
    }
    if (MODE >= 2 && r >= 1 && act) {
      const long long idx = (long long)(j - 1) * ni + i;
#pragma unroll
      for (int v = 0; v < 4; ++v) un[v] = ldg(Un + v * ncell + idx);
    }
    // ---- (2) right-edge i-face fluxes of the next 64 rows (LDS)
    if (more && (r & 63) == 0) {
      const int rr = min(lane, n - r - 1);
#ifdef FV_EDGE_REGS
      edge_face(C, i0 + nc, j + rr, edge_r);
#else
      T ge[4];
      edge_face(C, i0 + nc, j + rr, ge);
#pragma unroll
      for (int v = 0; v < 4; ++v) s_edge[lane * 4 + v] = ge[v];
      __builtin_amdgcn_wave_barrier();
#endif
    }
    // ---- (3) j-face at j-1/2
    T qLj[4], qRj[4], ep0[4], Gj[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T a = T(qm1[v]), b = T(q0[v]), c = T(qn[v]);
      T em;
      extrap(C.rc, b - a, c - b, ep0[v], em);
      qLj[v] = a + epm1[v];
      qRj[v] = b - em;
    }
    // lane shifts are taken by every lane, then selected (a conditional
    // expression would run them under a partial EXEC mask)
    const double x0s = shl1(x0), y0s = shl1(y0);
    const double x0r = lane == last ? xh0 : x0s;
    const double y0r = lane == last ? yh0 : y0s;
    face_flux<T, 1>(C, qLj, qRj, -(y0r - y0), x0r - x0, Gj);
    // ---- (4) complete, update and store row j-1
    const double xms = shl1(xm), yms = shl1(ym);
    const double xmr = lane == last ? xhm : xms;
    const double ymr = lane == last ? yhm : yms;
    if (r >= 1 && act) {
      const long long idx = (long long)(j - 1) * ni + i;
      double R[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) R[v] = rg[v] + (double)Gj[v];
      const double vol = curv ? 0.5 * ((x0r - xm) * (y0 - ymr) - (x0 - xmr) * (y0r - ym)) : B.vol;
      if (MODE == 0) {
        const double iv = 1.0 / vol;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          stg(rout + B.out_off + v * ncell + idx, R[v]);
          const double rv = R[v] * iv;
          nacc[v] += rv * rv;
        }
      } else {
        const double f = dt / vol;
        double out[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double us = qm1[v] - f * R[v];
          if (MODE == 1) out[v] = us;
          else if (MODE == 2) out[v] = 0.75 * un[v] + 0.25 * us;
          else out[v] = (1.0 / 3.0) * un[v] + (2.0 / 3.0) * us;
          stg(Uout + v * ncell + idx, out[v]);
        }
        if (MODE == 1) {
          const double iv = 1.0 / vol;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double rv = R[v] * iv;
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
    // ---- (5) i-face at i-1/2 of row j
    if (more) {
      const double xh1 = lane_value(hx1, 2), yh1 = lane_value(hy1, 2);
      T qLi[4], qRi[4], Gi[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T c = T(q0[v]);
        const T h = T(hv[v]);
        const T left = shr1(c);
        const T right = shl1(c);
        const T hright = lane_value(h, 2);  // Q(i0+ncol)
        const T hfar = shl1(h);             // lane 0: Q(i0-2) from lane 1
        const T qim1 = lane == 0 ? h : left;
        const T qip1 = lane == last ? hright : right;
        T epc, emc;
        extrap(C.rc, c - qim1, qip1 - c, epc, emc);
        T ep0l, em0l;
        extrap(C.rc, h - hfar, c - h, ep0l, em0l);  // cell i0-1 (used by lane 0)
        const T epl = shr1(epc);
        qLi[v] = qim1 + (lane == 0 ? ep0l : epl);
        qRi[v] = c - emc;
      }
      face_flux<T, 0>(C, qLi, qRi, y1 - y0, -(x1 - x0), Gi);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#ifdef FV_EDGE_REGS
        const T ge = lane_value(edge_r[v], r & 63);
#else
        const T ge = s_edge[(r & 63) * 4 + v];
#endif
        const T gs = shl1(Gi[v]);
        const T gr = lane == last ? ge : gs;
        rg[v] = ((double)gr - (double)Gi[v]) - (double)Gj[v];
      }
      xhm = xh0; yhm = yh0;
      xh0 = xh1; yh0 = yh1;
    }
    // ---- (6) rotate the carried rows
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      qm1[v] = q0[v];
      q0[v] = qn[v];
      qn[v] = qnn[v];
      epm1[v] = ep0[v];
    }
    xm = x0; ym = y0;
    x0 = x1; y0 = y1;
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
  __shared__ T s_edge[kWavesPerWG][64 * 4];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x * kWavesPerWG + wid; t < ntiles; t += gridDim.x * kWavesPerWG) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;
    tile2d<MODE, T>(tl, blocks, I, rout, lane, s_edge[wid]);
  }
}

// Spectral minimum and physical check of U^n (buffer 0), per tile.
__global__ __launch_bounds__(256) void k_cfl2d(const DevTile* __restrict__ tiles,
                                               const int* __restrict__ ntiles_p,
                                               const DevBlock* __restrict__ blocks,
                                               DevInstance* __restrict__ insts) {
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x * kWavesPerWG + wid; t < ntiles; t += gridDim.x * kWavesPerWG) {
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
        for (int v = 0; v < 4; ++v) q[v] = ldg(B.u[0] + v * B.ncell + idx);
        double Sb[2][3], vol;
        if (B.xn) {
          // nodes a = (i, j), b = (i+1, j), c = (i, j+1), d = (i+1, j+1)
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
