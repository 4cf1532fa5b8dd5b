// 2D Navier-Stokes stage kernel: the residual of Sec. 3.1, Eq. (residual)
// with both parts of the face flux, F_{i,n} - F_{nu,n} (Sec. 2), and the
// source term - |Omega| S_h, fused with the RK stage update and the step-end
// partials, like the Euler stage kernel.  It runs every 2D grid whose
// parameters carry a viscosity, whose faces include a no-slip wall or that
// has a source.
//
// One workgroup of 256 threads takes a tile (64 columns by n rows) in slabs
// of 4 rows, one cell per thread:
//   1. the slab's state with a two-cell halo on every side (corner ghosts
//      included) is resolved into LDS, then u, v, p/rho and the cell
//      centres of the slab and its first halo ring, and the node
//      coordinates of the slab;
//   2. every face of the slab gets its flux once: Roe's flux of the MUSCL
//      face states (times |S|) minus the viscous flux F_nu . S, whose face
//      gradients come from Green-Gauss over the face's diamond (the two
//      cell centres and the two face nodes, node values the mean of the four
//      cells around the node);
//   3. each cell sums its four faces, updates its state (the stage kinds of
//      the Euler kernel) and adds to the tile's partials.
// Readings of the viscous flux: Stokes's hypothesis with constant mu;
// Theta = tau u + (mu/Pr) gamma/(gamma-1) grad(p/rho); ghost-cell centres
// across block links are the neighbour's, across periodic faces the image
// moved by the offset between the faces, and elsewhere the interior
// centre reflected through the face midpoint; a corner ghost follows the
// i-face rule and then the j-face rule of the block that rule lands in.
// In FP32-flux mode the flux arithmetic (reconstruction, Roe, the gradient,
// stresses and F.S) runs in FP32 on differences formed in FP64; sums,
// update and reductions stay in FP64.
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

constexpr int kNsThreads = 256;
constexpr int kNsRows = 4;          // rows per slab (4 x 64 cells, one per thread)
constexpr int kQW = 64 + 4;         // state columns i0-2 .. i0+65
constexpr int kQH = kNsRows + 4;    // state rows j0-2 .. j0+5
constexpr int kWW = 64 + 2;         // primitive / centre columns i0-1 .. i0+64
constexpr int kWH = kNsRows + 2;    // rows j0-1 .. j0+4

// The face fluxes of a slab are formed in registers and then written over the
// state and primitive arrays, which no thread reads any more by then (the
// right and top edges have slots of their own): 51 KB per workgroup, three
// workgroups per CU (their VGPR budget is the limit as well).
struct NsLds {
  union {
    struct {
      double q[4][kQH][kQW];        // conserved state of the slab and its halo
      double w[3][kWH][kWW];        // u, v, p/rho
    } s;
    struct {
      double fi[4][kNsRows][65];    // i-face fluxes (flux times area, minus viscous)
      double fj[4][kNsRows + 1][64];  // j-face fluxes
    } f;
  } u;
  double cx[kWH][kWW], cy[kWH][kWW];  // cell centres
  double nx[kNsRows + 3][67], ny[kNsRows + 3][67];  // nodes of the slab and one ring
                                                    // (rows j0-1.., columns i0-1..)
  double un[4][kNsRows][64];        // U^n of the slab (stage kinds that read it)
  double er[4][kNsRows];            // fluxes of the slab's right edge
  double et[4][64];                 // fluxes of the slab's top edge
  double red[4][8];                 // per-wave partials
};

// node (i, j) of block B: stored coordinates, or the uniform lattice
__device__ __forceinline__ void node_of(const DevBlock& B, int i, int j, double& x, double& y) {
  if (B.xn) {
    x = nodex(B, i, j);
    y = nodey(B, i, j);
  } else {
    x = B.org[0] + i * B.area[1];
    y = B.org[1] + j * B.area[0];
  }
}

__device__ __forceinline__ void centre_of(const DevBlock& B, int i, int j, double& cx, double& cy) {
  double x0, y0, x1, y1, x2, y2, x3, y3;
  node_of(B, i, j, x0, y0);
  node_of(B, i + 1, j, x1, y1);
  node_of(B, i, j + 1, x2, y2);
  node_of(B, i + 1, j + 1, x3, y3);
  cx = 0.25 * (((x0 + x1) + x2) + x3);
  cy = 0.25 * (((y0 + y1) + y2) + y3);
}

// area vector of the wall face of side f (0..3) of B at transverse index t
__device__ __forceinline__ void wall_vec(const DevBlock& B, int f, int t, double& sx, double& sy) {
  const int d = f >> 1, side = f & 1;
  if (B.xn == nullptr) {
    sx = d == 0 ? 1.0 : 0.0;
    sy = d == 0 ? 0.0 : 1.0;
    return;
  }
  double x0, y0, x1, y1;
  if (d == 0) {
    const int w = side == 0 ? 0 : B.ni;
    node_of(B, w, t, x0, y0);
    node_of(B, w, t + 1, x1, y1);
    sx = y1 - y0;
    sy = -(x1 - x0);
  } else {
    const int w = side == 0 ? 0 : B.nj;
    node_of(B, t, w, x0, y0);
    node_of(B, t + 1, w, x1, y1);
    sx = -(y1 - y0);
    sy = x1 - x0;
  }
}

// momentum mirrored about the unit normal of the area vector (sx, sy)
__device__ __forceinline__ void slip_mirror(double* q, double sx, double sy) {
  const double ms = fmad(q[1], sx, q[2] * sy), ss = fmad(sx, sx, sy * sy);
  const double fct = 2.0 * ms / ss;
  q[1] -= fct * sx;
  q[2] -= fct * sy;
}

// Conserved state of cell (i, j) of block Bp in buffer buf; i and j may each
// lie up to two cells outside.  The i-face rule first (source block and
// column, and the i-wall transform), then the j-face rule of the source
// block, then the transforms in reverse order.
__device__ void ns_cell(const DevBlock* __restrict__ blocks, const DevBlock* Bp, int buf, int i,
                        int j, double* q) {
  const DevBlock* S = Bp;
  int si = i, sj = j;
  int ikind = -1, iface = 0;
  if (i < 0 || i >= Bp->ni) {
    const int side = i < 0 ? 0 : 1;
    const int g = side == 0 ? -i : i - Bp->ni + 1;
    iface = side;
    ikind = Bp->bc_kind[iface];
    if (ikind == BC_INFLOW) {
#pragma unroll
      for (int v = 0; v < 4; ++v) q[v] = Bp->bc_q[iface][v];
      return;
    }
    if (ikind == BC_BLOCK) S = &blocks[Bp->bc_nbr[iface]];
    const int n = S->ni;
    if (ikind == BC_PERIODIC || ikind == BC_BLOCK) si = side == 0 ? n - g : g - 1;
    else if (ikind == BC_EXTRAP) si = side == 0 ? 0 : n - 1;
    else si = side == 0 ? g - 1 : n - g;
  }
  int jkind = -1, jface = 2;
  const DevBlock* S2 = S;
  if (j < 0 || j >= S->nj) {
    const int side = j < 0 ? 0 : 1;
    const int g = side == 0 ? -j : j - S->nj + 1;
    jface = 2 + side;
    jkind = S->bc_kind[jface];
    if (jkind == BC_INFLOW) {
#pragma unroll
      for (int v = 0; v < 4; ++v) q[v] = S->bc_q[jface][v];
      jkind = -2;  // the state is set; only the i-transform follows
    } else {
      if (jkind == BC_BLOCK) S2 = &blocks[S->bc_nbr[jface]];
      const int n = S2->nj;
      if (jkind == BC_PERIODIC || jkind == BC_BLOCK) sj = side == 0 ? n - g : g - 1;
      else if (jkind == BC_EXTRAP) sj = side == 0 ? 0 : n - 1;
      else sj = side == 0 ? g - 1 : n - g;
    }
  }
  if (jkind != -2) {
    const double* p = S2->u[buf] + (long long)sj * S2->ni + si;
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = ldg(p + v * S2->ncell);
    if (jkind == BC_SLIPWALL) {
      double sx, sy;
      wall_vec(*S, jface, si, sx, sy);
      slip_mirror(q, sx, sy);
    } else if (jkind == BC_NOSLIP) {
      noslip_mirror<2>(q, S->bc_q[jface]);
    }
  }
  if (ikind == BC_SLIPWALL) {
    double sx, sy;
    wall_vec(*Bp, iface, min(max(j, 0), Bp->nj - 1), sx, sy);
    slip_mirror(q, sx, sy);
  } else if (ikind == BC_NOSLIP) {
    noslip_mirror<2>(q, Bp->bc_q[iface]);
  }
}

// Centre of cell (i, j) of B, inside or one ghost layer outside one face
__device__ void ns_centre(const DevBlock* __restrict__ blocks, const DevBlock& B, int i, int j,
                          double& cx, double& cy) {
  const bool iin = i >= 0 && i < B.ni, jin = j >= 0 && j < B.nj;
  if (iin && jin) {
    centre_of(B, i, j, cx, cy);
    return;
  }
  if (!iin && !jin) {  // corner: never a face's neighbour
    cx = cy = 0.0;
    return;
  }
  const int d = iin ? 1 : 0;
  const int side = (d == 0 ? i : j) < 0 ? 0 : 1;
  const int f = 2 * d + side;
  const int n = d == 0 ? B.ni : B.nj;
  // midpoint of the boundary face
  double x0, y0, x1, y1;
  const int w = side == 0 ? 0 : n;
  if (d == 0) {
    node_of(B, w, j, x0, y0);
    node_of(B, w, j + 1, x1, y1);
  } else {
    node_of(B, i, w, x0, y0);
    node_of(B, i + 1, w, x1, y1);
  }
  const double mx = 0.5 * (x0 + x1), my = 0.5 * (y0 + y1);
  const int kind = B.bc_kind[f];
  if (kind == BC_BLOCK) {
    const DevBlock& N = blocks[B.bc_nbr[f]];
    const int along = side == 0 ? (d == 0 ? N.ni : N.nj) - 1 : 0;
    centre_of(N, d == 0 ? along : i, d == 0 ? j : along, cx, cy);
  } else if (kind == BC_PERIODIC) {
    const int along = side == 0 ? n - 1 : 0;
    const int wo = side == 0 ? n : 0;
    if (d == 0) {
      node_of(B, wo, j, x0, y0);
      node_of(B, wo, j + 1, x1, y1);
    } else {
      node_of(B, i, wo, x0, y0);
      node_of(B, i + 1, wo, x1, y1);
    }
    const double ox = 0.5 * (x0 + x1), oy = 0.5 * (y0 + y1);
    centre_of(B, d == 0 ? along : i, d == 0 ? j : along, cx, cy);
    cx += mx - ox;
    cy += my - oy;
  } else {
    const int along = side == 0 ? 0 : n - 1;
    centre_of(B, d == 0 ? along : i, d == 0 ? j : along, cx, cy);
    cx = 2.0 * mx - cx;
    cy = 2.0 * my - cy;
  }
}

template <int LIM, typename T>
__device__ __forceinline__ void inv_flux(const Recon<T>& rc, const FluxK<T>& K, const double* c0,
                                         const double* c1, const double* c2, const double* c3,
                                         double Sx, double Sy, T* G) {
  T qL[4], qR[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T ep, em, ep2, em2;
    extrap<LIM, T>(rc, T(c1[v] - c0[v]), T(c2[v] - c1[v]), ep, em);
    extrap<LIM, T>(rc, T(c2[v] - c1[v]), T(c3[v] - c2[v]), ep2, em2);
    qL[v] = T(c1[v]) + ep;
    qR[v] = T(c2[v]) - em2;
  }
  double A, h;
  M<double>::sqrt2(fmad(Sx, Sx, Sy * Sy), A, h);
  const double iA = 2.0 * h;
  const T n[2] = {T(Sx * iA), T(Sy * iA)};
  roe_flux<T, 2, -1>(qL, qR, n, T(A), K, G);
}

template <int MODE, typename T, int LIM>
__device__ void tile_ns(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                        double* __restrict__ rout, NsLds& L) {
  using SK = StageKind<MODE>;
  constexpr int bin = SK::bin;
  constexpr int bout = SK::bout;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const DevBlock& B = blocks[tl.blk];
  if (MODE != 0 && I.stopped) return;
  const int ni = B.ni;
  const long long ncell = B.ncell;
  const int i0 = tl.i0, nc = tl.ncol;
  Recon<T> rc;
  rc.lim = I.limiter;
  rc.heps = T(0.5 * I.eps);
  rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  FluxK<T> K;
  K.gm1 = T(I.gamma - 1.0);
  K.efix = T(I.efix);
  K.iefix = T(I.efix > 0.0 ? 1.0 / I.efix : 0.0);
  const double gamma = I.gamma, mu = I.mu;
  const T tmu = T(mu);
  const T kq = T(mu > 0.0 ? mu / I.prandtl * gamma / (gamma - 1.0) : 0.0);
  const double dt = stage_dt<MODE>(I);
  double nacc[4] = {0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  for (int js = tl.j0; js < tl.j0 + tl.n; js += kNsRows) {
    const int nr = min(kNsRows, tl.j0 + tl.n - js);
    // ---- 1. state of the slab and its halo, then u, v, p/rho, centres, nodes
    for (int x = tid; x < (nr + 4) * (nc + 4); x += kNsThreads) {
      const int r = x / (nc + 4), c = x - r * (nc + 4);
      double q[4];
      ns_cell(blocks, &B, bin, i0 - 2 + c, js - 2 + r, q);
#pragma unroll
      for (int v = 0; v < 4; ++v) L.u.s.q[v][r][c] = q[v];
    }
    // nodes of the slab and one ring around it (clamped into the block: the
    // ring nodes outside it are never used); face vectors and volumes
    for (int x = tid; x < (nr + 3) * (nc + 3); x += kNsThreads) {
      const int r = x / (nc + 3), c = x - r * (nc + 3);
      double xx, yy;
      node_of(B, min(max(i0 - 1 + c, 0), ni), min(max(js - 1 + r, 0), B.nj), xx, yy);
      L.nx[r][c] = xx;
      L.ny[r][c] = yy;
    }
    if constexpr (SK::reads_un) {
      for (int x = tid; x < nr * nc; x += kNsThreads) {
        const int r = x / nc, c = x - r * nc;
        const double* p = B.u[0] + (long long)(js + r) * ni + i0 + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) L.un[v][r][c] = ldg(p + v * ncell);
      }
    }
    __syncthreads();
    // u, v, p/rho and the centres of the slab's cells and their ring: a
    // centre inside the block from the staged nodes (the four around it, in
    // the order of centre_of), a ghost centre by its rule
    for (int x = tid; x < (nr + 2) * (nc + 2); x += kNsThreads) {
      const int r = x / (nc + 2), c = x - r * (nc + 2);
      const int ci = i0 - 1 + c, cj = js - 1 + r;
      double cx, cy;
      if (ci >= 0 && ci < ni && cj >= 0 && cj < B.nj) {
        cx = 0.25 * (((L.nx[r][c] + L.nx[r][c + 1]) + L.nx[r + 1][c]) + L.nx[r + 1][c + 1]);
        cy = 0.25 * (((L.ny[r][c] + L.ny[r][c + 1]) + L.ny[r + 1][c]) + L.ny[r + 1][c + 1]);
      } else {
        ns_centre(blocks, B, ci, cj, cx, cy);
      }
      L.cx[r][c] = cx;
      L.cy[r][c] = cy;
      const double rho = L.u.s.q[0][r + 1][c + 1];
      const double ir = M<double>::rcp(rho);
      const double u = L.u.s.q[1][r + 1][c + 1] * ir, v = L.u.s.q[2][r + 1][c + 1] * ir;
      const double p = (gamma - 1.0) * (L.u.s.q[3][r + 1][c + 1] - 0.5 * rho * (u * u + v * v));
      L.u.s.w[0][r][c] = u;
      L.u.s.w[1][r][c] = v;
      L.u.s.w[2][r][c] = p * ir;
    }
    __syncthreads();

    // ---- 2. face fluxes, one thread per cell (its left and bottom faces;
    //         the right column and top row also take the far faces)
    const int li = lane, lj = wv;
    const bool act = li < nc && lj < nr;
    // node value (u, v, p/rho) of node (c, r) in w coordinates: mean of the
    // cells (c-1, r-1), (c, r-1), (c-1, r), (c, r)
    auto node_w = [&](int c, int r, double* o) {
#pragma unroll
      for (int k = 0; k < 3; ++k)
        o[k] = 0.25 * (((L.u.s.w[k][r - 1][c - 1] + L.u.s.w[k][r - 1][c]) + L.u.s.w[k][r][c - 1]) + L.u.s.w[k][r][c]);
    };
    // i-face at node column fc (0..nc) of slab row `row`
    auto iface = [&](int fc, int row, double (&F)[4]) {
      const int qr = row + 2, wr = row + 1;
      double c0[4], c1[4], c2[4], c3[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        c0[v] = L.u.s.q[v][qr][fc];
        c1[v] = L.u.s.q[v][qr][fc + 1];
        c2[v] = L.u.s.q[v][qr][fc + 2];
        c3[v] = L.u.s.q[v][qr][fc + 3];
      }
      // area vector: from the nodes, or exactly h_y e_x on a uniform block
      const double Sx = B.xn ? L.ny[row + 2][fc + 1] - L.ny[row + 1][fc + 1] : B.area[0];
      const double Sy = B.xn ? -(L.nx[row + 2][fc + 1] - L.nx[row + 1][fc + 1]) : 0.0;
      T G[4];
      inv_flux<LIM, T>(rc, K, c0, c1, c2, c3, Sx, Sy, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) F[v] = (double)G[v];
      if (mu > 0.0) {
        double wL[3], wR[3], wA[3], wB[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          wL[k] = L.u.s.w[k][wr][fc];
          wR[k] = L.u.s.w[k][wr][fc + 1];
        }
        node_w(fc + 1, wr, wA);      // node (i, j)
        node_w(fc + 1, wr + 1, wB);  // node (i, j+1)
        const double dx = L.cx[wr][fc + 1] - L.cx[wr][fc], dy = L.cy[wr][fc + 1] - L.cy[wr][fc];
        T Fv[4];
        visc_flux<T>(wL, wR, wA, wB, dx, dy, Sx, Sy, tmu, kq, Fv);
#pragma unroll
        for (int v = 0; v < 4; ++v) F[v] -= (double)Fv[v];
      }
    };
    // j-face at node row fr (0..nr) of slab column li
    auto jface = [&](int fr, double (&F)[4]) {
      const int qc = li + 2, wc = li + 1;
      double c0[4], c1[4], c2[4], c3[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        c0[v] = L.u.s.q[v][fr][qc];
        c1[v] = L.u.s.q[v][fr + 1][qc];
        c2[v] = L.u.s.q[v][fr + 2][qc];
        c3[v] = L.u.s.q[v][fr + 3][qc];
      }
      const double Sx = B.xn ? -(L.ny[fr + 1][li + 2] - L.ny[fr + 1][li + 1]) : 0.0;
      const double Sy = B.xn ? L.nx[fr + 1][li + 2] - L.nx[fr + 1][li + 1] : B.area[1];
      T G[4];
      inv_flux<LIM, T>(rc, K, c0, c1, c2, c3, Sx, Sy, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) F[v] = (double)G[v];
      if (mu > 0.0) {
        double wL[3], wR[3], wA[3], wB[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          wL[k] = L.u.s.w[k][fr][wc];
          wR[k] = L.u.s.w[k][fr + 1][wc];
        }
        node_w(wc + 1, fr + 1, wA);  // node (i+1, j)
        node_w(wc, fr + 1, wB);      // node (i, j)
        const double dx = L.cx[fr + 1][wc] - L.cx[fr][wc], dy = L.cy[fr + 1][wc] - L.cy[fr][wc];
        T Fv[4];
        visc_flux<T>(wL, wR, wA, wB, dx, dy, Sx, Sy, tmu, kq, Fv);
#pragma unroll
        for (int v = 0; v < 4; ++v) F[v] -= (double)Fv[v];
      }
    };
    double Fl[4], Fb[4], qin[4];
    // the slab's right-edge i-faces, one row per lane, in wave 0, and its
    // top-edge j-faces in the top row's wave: each edge costs one wave-wide
    // flux, where a right-edge face in every wave's last lane cost four
    if (wv == 0 && lane < nr) {
      double Fr[4];
      iface(nc, lane, Fr);
#pragma unroll
      for (int v = 0; v < 4; ++v) L.er[v][lane] = Fr[v];
    }
    if (act) {
      if (lj == nr - 1) {
        double Ft[4];
        jface(nr, Ft);
#pragma unroll
        for (int v = 0; v < 4; ++v) L.et[v][li] = Ft[v];
      }
      iface(li, lj, Fl);
      jface(lj, Fb);
#pragma unroll
      for (int v = 0; v < 4; ++v) qin[v] = L.u.s.q[v][lj + 2][li + 2];
    }
    __syncthreads();  // state and primitives are read no more: the fluxes take their place
    if (act) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        L.u.f.fi[v][lj][li] = Fl[v];
        L.u.f.fj[v][lj][li] = Fb[v];
      }
    }
    __syncthreads();

    // ---- 3. residual, update, partials
    if (act) {
      const int i = i0 + li, j = js + lj;
      double R[4];
#pragma unroll
      for (int v = 0; v < 4; ++v)
      {
        const double fr = li == nc - 1 ? L.er[v][lj] : L.u.f.fi[v][lj][li + 1];
        const double ft = lj == nr - 1 ? L.et[v][li] : L.u.f.fj[v][lj + 1][li];
        R[v] = (0.0 + (fr - Fl[v])) + (ft - Fb[v]);
      }
      const double xa = L.nx[lj + 1][li + 1], ya = L.ny[lj + 1][li + 1];
      const double xb = L.nx[lj + 1][li + 2], yb = L.ny[lj + 1][li + 2];
      const double xc = L.nx[lj + 2][li + 1], yc = L.ny[lj + 2][li + 1];
      const double xd = L.nx[lj + 2][li + 2], yd = L.ny[lj + 2][li + 2];
      const double vol = B.xn ? 0.5 * fmad(xd - xa, yc - yb, -((xc - xb) * (yd - ya))) : B.vol;
      const double iv = M<double>::rcp(vol);
      const long long ro = (long long)j * ni + i;
      if (B.src != nullptr) {  // the source part of Eq. (residual): - |Omega| S_h
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] -= vol * ldg(B.src + v * ncell + ro);
      }
      if (MODE == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          stg(rout + B.out_off + v * ncell + ro, R[v]);
          const double rv = R[v] * iv;
          nacc[v] = fmad(rv, rv, nacc[v]);
        }
      } else {
        const double f = dt * iv;
        double out[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double un = 0.0;
          if constexpr (SK::reads_un) un = L.un[v][lj][li];
          if constexpr (SK::low) {
            out[v] = fmad(-f, R[v], un);
          } else {
            const double us = fmad(-f, R[v], qin[v]);
            if (MODE == 1) out[v] = us;
            else if (MODE == 2) out[v] = fmad(0.75, un, 0.25 * us);
            else out[v] = fmad(1.0 / 3.0, un, (2.0 / 3.0) * us);
          }
          stg(B.u[bout] + v * ncell + ro, out[v]);
        }
        if (MODE == 1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double rv = R[v] * iv;
            nacc[v] = fmad(rv, rv, nacc[v]);
          }
        }
        if constexpr (SK::cfl) {
          double Sb[2][3];
          if (B.xn) {
            Sb[0][0] = 0.5 * ((yc - ya) + (yd - yb));
            Sb[0][1] = -0.5 * ((xc - xa) + (xd - xb));
            Sb[1][0] = -0.5 * ((yb - ya) + (yd - yc));
            Sb[1][1] = 0.5 * ((xb - xa) + (xd - xc));
          } else {
            Sb[0][0] = B.area[0];
            Sb[0][1] = 0.0;
            Sb[1][0] = 0.0;
            Sb[1][1] = B.area[1];
          }
          Sb[0][2] = Sb[1][2] = 0.0;
          dmin = fmin(dmin, mu > 0.0 ? cell_dt_limit_visc(out, Sb, vol, gamma, mu, I.prandtl, bad)
                                     : cell_dt_limit<2>(out, Sb, vol, gamma, bad));
        }
      }
    }
    __syncthreads();  // the LDS slab is reused by the next slab
  }

  // ---- per-tile partials: fixed-order wave reductions, then the four waves
  double* part = I.part + tl.local;
  const long long ps = I.ntiles;
  if (MODE == 0 || MODE == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double s = wave_sum(nacc[v]);
      if (lane == 0) L.red[wv][v] = s;
    }
  }
  if (SK::cfl) {
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      L.red[wv][4] = m;
      L.red[wv][5] = (double)b;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (MODE == 0 || MODE == 1) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        part[v * ps] = ((L.red[0][v] + L.red[1][v]) + L.red[2][v]) + L.red[3][v];
      part[4 * ps] = 0.0;
    }
    if (SK::cfl) {
      part[5 * ps] = fmin(fmin(L.red[0][4], L.red[1][4]), fmin(L.red[2][4], L.red[3][4]));
      part[6 * ps] = (L.red[0][5] + L.red[1][5] + L.red[2][5] + L.red[3][5]) != 0.0 ? 1.0 : 0.0;
    }
  }
  __syncthreads();  // L.red is reused by the next tile
}

template <int MODE, typename T>
__global__ __launch_bounds__(kNsThreads, 3) void k_stage2d_ns(const DevTile* __restrict__ tiles,
                                                         const int* __restrict__ ntiles_p, int nfix,
                                                         const DevBlock* __restrict__ blocks,
                                                         DevInstance* __restrict__ insts,
                                                         double* __restrict__ rout) {
  __shared__ NsLds s_lds;
  const int ntiles = nfix >= 0 ? nfix : *ntiles_p;
  for (TileWalk tw = xcd_walk(ntiles, 1, 0); tw.t < tw.end; tw.t += tw.stride) {
    const DevTile tl = tiles[tw.t];
    DevInstance& I = insts[tl.inst];
    // minmod, the common limiter, is compiled with the limiter fixed
    if (I.limiter == LIM_MINMOD) tile_ns<MODE, T, LIM_MINMOD>(tl, blocks, I, rout, s_lds);
    else tile_ns<MODE, T, -1>(tl, blocks, I, rout, s_lds);
  }
}

}  // namespace

hipError_t launch_stage2d_ns(int mode, int fp32, int grid, hipStream_t s, const DevTile* tiles,
                             const int* ntiles, int ntiles_fixed, const DevBlock* blocks,
                             DevInstance* insts, double* rout) {
  if (mode < 0 || mode > 6) return hipErrorInvalidValue;
#define FV_LN(M, T) hipLaunchKernelGGL((k_stage2d_ns<M, T>), dim3(grid), dim3(kNsThreads), 0, s, tiles, ntiles, ntiles_fixed, blocks, insts, rout)
#define FV_LN_ALL(T)              \
  switch (mode) {                 \
    case 0: FV_LN(0, T); break;   \
    case 1: FV_LN(1, T); break;   \
    case 2: FV_LN(2, T); break;   \
    case 3: FV_LN(3, T); break;   \
    case 4: FV_LN(4, T); break;   \
    case 5: FV_LN(5, T); break;   \
    default: FV_LN(6, T); break;  \
  }
  if (fp32) {
    FV_LN_ALL(float)
  } else {
    FV_LN_ALL(double)
  }
#undef FV_LN_ALL
#undef FV_LN
  return hipGetLastError();
}

const void* stage2d_ns_kernel_ptr(int fp32) {
  return fp32 ? (const void*)&k_stage2d_ns<1, float> : (const void*)&k_stage2d_ns<1, double>;
}

}  // namespace fvk
