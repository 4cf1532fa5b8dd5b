// 3D stage kernels (uniform grids): MUSCL + Roe residual, SSP-RK3 stage
// update and fused reductions.  One workgroup per tile.
//
// A tile is 64 columns i (lane) by ny rows j (one wavefront per row) and
// marches over n planes k.  The workgroup has ny + 1 waves: waves 0..ny-1
// own the rows; wave ny owns no cells, it loads the four j-halo rows of each
// plane and forms the j-face flux at the tile's top edge.  Per plane k:
//   - each row wave loads Q(k+1) of its column (k-stencil rows k-1, k carried
//     in registers), forms the k-face flux at k-1/2, completes the residual of
//     plane k-1 and updates/stores it;
//   - the plane k is staged in LDS (rows j0-2 .. j0+ny+1), then every row wave
//     forms its i-face flux (lane shuffles, halo lanes, batched right-edge
//     pre-pass as in 2D) and its j-face flux at j-1/2 (LDS rows), the j-face
//     fluxes are exchanged through LDS, and each row keeps the in-plane part
//     of its residual for the next iteration.
// Every face flux of the tile is formed once (tile edges aside).
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

__device__ __forceinline__ void load3d(const DevBlock* blocks, const DevBlock& B, int buf, int i,
                                       int j, int k, double (&q)[5]) {
  if (i >= 0 && i < B.ni && j >= 0 && j < B.nj && k >= 0 && k < B.nk) {
    const double* s = B.u[buf] + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = s[v * B.ncell];
  } else {
    resolve_cell<5>(blocks, B, buf, i, j, k, q);
  }
}

// Roe flux across a face whose unit normal is the coordinate axis AX
template <typename T, int AX>
__device__ __forceinline__ void axis_flux(const T (&qL)[5], const T (&qR)[5], T area, T gm1, T efix,
                                          T (&F)[5]) {
  const T n[3] = {T(AX == 0 ? 1 : 0), T(AX == 1 ? 1 : 0), T(AX == 2 ? 1 : 0)};
  roe_flux<T, 3>(qL, qR, n, area, gm1, efix, F);
}

template <typename T>
struct Ctx3D {
  const DevBlock* blocks;
  const DevBlock* B;
  int buf;
  Recon<T> rc;
  T gm1, efix;
  T ax, ay, az;  // face areas
};

// i-face at the right edge of the tile for row j, plane kr (column ie)
template <typename T>
__device__ void edge_face3(const Ctx3D<T>& C, int ie, int j, int kr, T (&G)[5]) {
  const DevBlock& B = *C.B;
  double a[5], b[5], c[5], d[5];
  load3d(C.blocks, B, C.buf, ie - 2, j, kr, a);
  load3d(C.blocks, B, C.buf, ie - 1, j, kr, b);
  load3d(C.blocks, B, C.buf, ie, j, kr, c);
  load3d(C.blocks, B, C.buf, ie + 1, j, kr, d);
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
  axis_flux<T, 0>(qL, qR, C.ax, C.gm1, C.efix, G);
}

template <int MODE, typename T, int NY>
__device__ void tile3d(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                       double* __restrict__ rout, int lane, int w, T* s_q, T* s_f,
                       double* s_red) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni, nj = B.nj;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, n = tl.n, nc = tl.ncol, ny = tl.ny;
  const bool rowwave = w < NY;
  const bool rowact = w < ny;           // this wave owns a row of cells
  const int j = j0 + (rowwave ? w : ny);  // ghost wave: the row above the tile
  const int i = i0 + lane;
  const bool act = lane < nc;
  const int ic = act ? i : ni - 1;
  const int jc = rowact ? j : j0;       // safe row for idle waves
  const int bin = MODE == 0 ? 0 : MODE - 1;
  const int bout = MODE == 1 ? 1 : (MODE == 2 ? 2 : 0);

  Ctx3D<T> C;
  C.blocks = blocks;
  C.B = &B;
  C.buf = bin;
  C.rc.lim = I.limiter;
  C.rc.heps = T(0.5 * I.eps);
  C.rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  C.rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  C.gm1 = T(I.gamma - 1.0);
  C.efix = T(I.efix);
  C.ax = T(B.area[0]);
  C.ay = T(B.area[1]);
  C.az = T(B.area[2]);
  const double gamma = I.gamma;
  const double dt = I.dt;
  const double vol = B.vol;
  const long long ncell = B.ncell;
  double* __restrict__ Uout = B.u[bout];
  const double* __restrict__ Un = B.u[0];

  // LDS slots: s_q[(row slot)][v][lane], row slot = j - j0 + 2
  auto SQ = [&](int slot, int v) -> T& { return s_q[(slot * 5 + v) * kWave + lane]; };
  auto SF = [&](int slot, int v) -> T& { return s_f[(slot * 5 + v) * kWave + lane]; };

  // ---- prologue (row waves): planes k0-2, k0-1, k0 of the own column
  T qkm1[5], qk[5], epm1[5];
  double qkm1_d[5], qk_d[5];
  if (rowact) {
    double a[5], b[5], c[5];
    load3d(blocks, B, bin, ic, jc, k0 - 2, a);
    load3d(blocks, B, bin, ic, jc, k0 - 1, b);
    load3d(blocks, B, bin, ic, jc, k0, c);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T ta = T(a[v]), tb = T(b[v]), tc = T(c[v]);
      T em;
      extrap(C.rc, tb - ta, tc - tb, epm1[v], em);
      qkm1[v] = tb;
      qk[v] = tc;
      qkm1_d[v] = b[v];
      qk_d[v] = c[v];
    }
  }
  double rij[5] = {0, 0, 0, 0, 0};
  T gkb[5] = {T(0), T(0), T(0), T(0), T(0)};
  T edge[5] = {T(0), T(0), T(0), T(0), T(0)};
  double nacc[5] = {0, 0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  for (int r = 0; r <= n; ++r) {
    const int k = k0 + r;
    T qn[5], ep0[5];
    double qn_d[5];
    if (rowact) {
      if (r < n && (r & 63) == 0) {
        const int rr = min(lane, n - r - 1);
        edge_face3(C, i0 + nc, jc, k + rr, edge);
      }
      load3d(blocks, B, bin, ic, jc, k + 1, qn_d);
      // ---- k-face at k-1/2
      T em0[5], qL[5], qR[5], Gk[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        qn[v] = T(qn_d[v]);
        extrap(C.rc, qk[v] - qkm1[v], qn[v] - qk[v], ep0[v], em0[v]);
        qL[v] = qkm1[v] + epm1[v];
        qR[v] = qk[v] - em0[v];
      }
      axis_flux<T, 2>(qL, qR, C.az, C.gm1, C.efix, Gk);
      // ---- complete plane k-1
      if (r >= 1 && act) {
        const long long idx = ((long long)(k - 1) * nj + j) * ni + i;
        double R[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = rij[v] + ((double)Gk[v] - (double)gkb[v]);
        if (MODE == 0) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            rout[B.out_off + v * ncell + idx] = R[v];
            const double rv = R[v] / vol;
            nacc[v] += rv * rv;
          }
        } else {
          const double f = dt / vol;
          double out[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double us = qkm1_d[v] - f * R[v];
            if (MODE == 1) out[v] = us;
            else if (MODE == 2) out[v] = 0.75 * Un[v * ncell + idx] + 0.25 * us;
            else out[v] = (1.0 / 3.0) * Un[v * ncell + idx] + (2.0 / 3.0) * us;
            Uout[v * ncell + idx] = out[v];
          }
          if (MODE == 1) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              const double rv = R[v] / vol;
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
#pragma unroll
      for (int v = 0; v < 5; ++v) gkb[v] = Gk[v];
    }
    // ---- in-plane faces of plane k
    if (r < n) {
      if (rowact) {
#pragma unroll
        for (int v = 0; v < 5; ++v) SQ(w + 2, v) = qk[v];
      }
      if (!rowwave) {
        // j-halo rows of plane k: j0-2, j0-1, j0+ny, j0+ny+1
        const int rows[4] = {j0 - 2, j0 - 1, j0 + ny, j0 + ny + 1};
        const int slots[4] = {0, 1, ny + 2, ny + 3};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          double q[5];
          load3d(blocks, B, bin, ic, rows[h], k, q);
#pragma unroll
          for (int v = 0; v < 5; ++v) SQ(slots[h], v) = T(q[v]);
        }
      }
      __syncthreads();
      if (rowact || !rowwave) {
        // j-face at j-1/2: rows j-2 .. j+1 = slots s .. s+3 with s = j - j0
        const int s = j - j0;
        T qL[5], qR[5], Gj[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T a = SQ(s, v), b = SQ(s + 1, v), c = SQ(s + 2, v), d = SQ(s + 3, v);
          T ep, em, ep2, em2;
          extrap(C.rc, b - a, c - b, ep, em);
          extrap(C.rc, c - b, d - c, ep2, em2);
          qL[v] = b + ep;
          qR[v] = c - em2;
        }
        axis_flux<T, 1>(qL, qR, C.ay, C.gm1, C.efix, Gj);
#pragma unroll
        for (int v = 0; v < 5; ++v) SF(s, v) = Gj[v];
      }
      T Gi[5], Gr[5];
      if (rowact) {
        // i-face at i-1/2 of row j, plane k
        double hv_d[5] = {0, 0, 0, 0, 0};
        if (lane < 3) {
          const int hi = lane == 0 ? i0 - 1 : (lane == 1 ? i0 - 2 : i0 + nc);
          load3d(blocks, B, bin, hi, jc, k, hv_d);
        }
        T qL[5], qR[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T hv = T(hv_d[v]);
          const T left = __shfl(qk[v], lane - 1 < 0 ? 0 : lane - 1, kWave);
          const T right = __shfl(qk[v], lane + 1 > 63 ? 63 : lane + 1, kWave);
          const T h1 = __shfl(hv, 1, kWave);
          const T h2 = __shfl(hv, 2, kWave);
          const T qim1 = lane == 0 ? hv : left;
          const T qip1 = lane == nc - 1 ? h2 : right;
          T epc, emc;
          extrap(C.rc, qk[v] - qim1, qip1 - qk[v], epc, emc);
          const T epl = __shfl(epc, lane - 1 < 0 ? 0 : lane - 1, kWave);
          T ep0l, em0l;
          extrap(C.rc, hv - h1, qk[v] - hv, ep0l, em0l);
          qL[v] = qim1 + (lane == 0 ? ep0l : epl);
          qR[v] = qk[v] - emc;
        }
        axis_flux<T, 0>(qL, qR, C.ax, C.gm1, C.efix, Gi);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T gr = __shfl(Gi[v], lane + 1 > 63 ? 63 : lane + 1, kWave);
          const T ge = __shfl(edge[v], r & 63, kWave);
          Gr[v] = lane == nc - 1 ? ge : gr;
        }
      }
      __syncthreads();
      if (rowact) {
        const int s = j - j0;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          rij[v] = ((double)Gr[v] - (double)Gi[v]) + ((double)SF(s + 1, v) - (double)SF(s, v));
      }
    }
    if (rowact) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        qkm1[v] = qk[v];
        qk[v] = qn[v];
        epm1[v] = ep0[v];
        qkm1_d[v] = qk_d[v];
        qk_d[v] = qn_d[v];
      }
    }
  }

  // ---- per-tile partials: wave reductions, then the row waves in order
  if (MODE == 0 || MODE == 1 || MODE == 3) {
    double s[5];
    double m = 0.0;
    int b = 0;
    if (MODE == 3) {
      m = wave_min(dmin);
      b = wave_or(bad);
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) s[v] = wave_sum(nacc[v]);
    }
    if (lane == 0 && rowwave) {
      if (MODE == 3) {
        s_red[w * 8 + 5] = m;
        s_red[w * 8 + 6] = (double)b;
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) s_red[w * 8 + v] = s[v];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double* part = I.part + (long long)tl.local * kPartStride;
      if (MODE == 3) {
        double mm = INFINITY;
        double bb = 0.0;
        for (int x = 0; x < ny; ++x) {
          mm = fmin(mm, s_red[x * 8 + 5]);
          bb = fmax(bb, s_red[x * 8 + 6]);
        }
        part[5] = mm;
        part[6] = bb;
      } else {
        for (int v = 0; v < 5; ++v) {
          double a = 0.0;
          for (int x = 0; x < ny; ++x) a += s_red[x * 8 + v];
          part[v] = a;
        }
      }
    }
    __syncthreads();
  }
}

template <int MODE, typename T, int NY>
__global__ __launch_bounds__(64 * (NY + 1)) void k_stage3d(const DevTile* __restrict__ tiles,
                                                           const int* __restrict__ ntiles_p,
                                                           const DevBlock* __restrict__ blocks,
                                                           DevInstance* __restrict__ insts,
                                                           double* __restrict__ rout) {
  __shared__ T s_q[(NY + 4) * 5 * kWave];
  __shared__ T s_f[(NY + 1) * 5 * kWave];
  __shared__ double s_red[(NY + 1) * 8];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = *ntiles_p;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DevTile tl = tiles[t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;
    tile3d<MODE, T, NY>(tl, blocks, I, rout, lane, w, s_q, s_f, s_red);
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
          for (int v = 0; v < 5; ++v) q[v] = B.u[0][v * B.ncell + idx];
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
