// General 3D stage kernel: the residual of Sec. 3.1, Eq. (residual) on 3D
// grids with curvilinear blocks (face area vectors and volumes from the node
// coordinates) or a cell-averaged source S_h, fused with the RK stage update
// and the step-end partials like the uniform 3D kernel.  Uniform blocks of
// such a grid run here too, with their exact axis-aligned metrics.
//
// One workgroup of 256 threads (4 waves) takes a tile of 64 columns i (lane)
// by 4 rows j (wave) and marches over its n planes k, one cell per thread:
//   - each thread keeps the states of its column at k-1 .. k+2 in registers
//     and forms the k-face flux at k+1/2; the flux at k-1/2 is the one it
//     formed for the plane before;
//   - plane k is staged in LDS with its in-plane halo (two cells beyond the
//     tile in i and in j), and each thread forms the i-face flux at i-1/2
//     and the j-face flux at j-1/2 of its cell from LDS (the right column and
//     the top row also form the tile's edge faces);
//   - node planes k and k+1 of the tile sit in LDS (curvilinear blocks):
//     each thread forms the six area vectors of its cell from them, and its
//     volume as 1/3 of the sum of (outward area vector . face centre).
// Every face flux of a tile is formed once (tile edges aside); a face shared
// by two tiles is formed by both from the same operands, so bitwise alike.
// In FP32-flux mode the reconstruction and Roe's flux run in FP32 on
// differences formed in FP64; geometry, sums, update and reductions stay in
// FP64.
#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

constexpr int kGT = 256;
constexpr int kGR = 4;           // j-rows per tile, one wave each
constexpr int kGQW = 64 + 4;     // state columns i0-2 .. i0+65
constexpr int kGQH = kGR + 4;    // state rows j0-2 .. j0+5
constexpr int kGHalo = 4 * (64 + kGR);  // halo cells of a tile plane (at most)

// 78 KB: two workgroups (eight waves) per CU, as the registers allow
struct GenLds {
  double q[5][kGQH][kGQW];       // plane k with its in-plane halo (a cross:
                                 // the corner slots are never read)
  double fi[5][kGR][65];         // i-face fluxes (times area), faces i0 .. i0+nc
  double fj[5][kGR + 1][64];     // j-face fluxes, faces j0 .. j0+nr
  double ci[kGR][65];            // S . centre of those faces (curvilinear volumes)
  double cj[kGR + 1][64];
  double nd[3][3][kGR + 1][65];  // node planes k0 + r in slot r % 3: x, y, z
  double red[4][8];              // per-wave partials
  // source of each halo cell, resolved once per tile (the same for every
  // plane): the cell in plane 0 of its block's input buffer, that block's
  // variable and plane strides, and kind | face << 4 | transverse index << 8
  // (kind 0: copy, 1: inflow state of the face, 2: copy mirrored about the
  // slip-wall face)
  const double* hp[kGHalo];
  long long hvs[kGHalo];
  int hps[kGHalo];
  int hkf[kGHalo];
};

// halo cell x of a tile plane: its row and column in the LDS plane
__device__ __forceinline__ void halo_slot(int x, int nc, int nr, int& qr, int& qc) {
  if (x < 4 * nc) {  // rows j0-2, j0-1, j0+nr, j0+nr+1
    const int a = x / nc;
    qc = x - a * nc + 2;
    qr = a < 2 ? a : nr + a;
  } else {           // columns i0-2, i0-1, i0+nc, i0+nc+1
    const int y = x - 4 * nc, a = y >> 2, b = y & 3;
    qr = a + 2;
    qc = b < 2 ? b : nc + b;
  }
}

// Source of the in-plane cell (ii, jj) of block B (at most one of the two
// outside, by at most 2): the rules of load_cell, without the plane.  The
// cell of plane k is at p + k * ps: through an oriented block link the
// planes of B may run along any axis of the neighbour, either way.
__device__ void halo_source(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf, int ii,
                            int jj, const double*& p, long long& vs, int& ps, int& kf) {
  const DevBlock* S = &B;
  int si = ii, sj = jj, kind = 0, f = 0, t = 0;
  long long c0 = -1, plane = (long long)B.ni * B.nj;  // c0 >= 0: start set by a block link
  if (ii < 0 || ii >= B.ni || jj < 0 || jj >= B.nj) {
    const int d = (ii < 0 || ii >= B.ni) ? 0 : 1;
    const int x = d == 0 ? ii : jj, n0 = d == 0 ? B.ni : B.nj;
    const int side = x < 0 ? 0 : 1, g = side == 0 ? -x : x - n0 + 1;
    f = 2 * d + side;
    t = d == 0 ? jj : ii;
    const int bk = B.bc_kind[f];
    if (bk == BC_INFLOW) {
      kind = 1;
    } else if (bk == BC_BLOCK) {
      // the cells of planes 0 and 1 give the neighbour's start and stride
      S = &blocks[B.bc_nbr[f]];
      int sk, ai, aj, ak;
      link_cell(*S, B.bc_link[f], g, t, 0, si, sj, sk);
      link_cell(*S, B.bc_link[f], g, t, 1, ai, aj, ak);
      c0 = ((long long)sk * S->nj + sj) * S->ni + si;
      plane = ((long long)ak * S->nj + aj) * S->ni + ai - c0;
    } else {
      const int n = d == 0 ? B.ni : B.nj;
      int along;
      if (bk == BC_PERIODIC) along = side == 0 ? n - g : g - 1;
      else if (bk == BC_EXTRAP) along = side == 0 ? 0 : n - 1;
      else along = side == 0 ? g - 1 : n - g;  // slip wall
      if (d == 0) si = along;
      else sj = along;
      kind = bk == BC_SLIPWALL ? 2 : 0;
    }
  }
  if (c0 < 0) c0 = (long long)sj * S->ni + si;
  p = kind == 1 ? nullptr : S->u[buf] + c0;
  vs = S->ncell;
  ps = (int)plane;
  kf = kind | (f << 4) | (t << 8);
}

// momentum of q mirrored about the slip-wall face f (an i- or j-face) of B
// at transverse index t in plane k: m - 2 (m.S)/(S.S) S, as load_cell
__device__ void slip_mirror3(const DevBlock& B, int f, int t, int k, double* q) {
  const int d = f >> 1, side = f & 1;
  double Sv[3] = {0.0, 0.0, 0.0};
  if (B.zn != nullptr) {
    const int w = side == 0 ? 0 : (d == 0 ? B.ni : B.nj);
    double cs;
    face3(B, d, d == 0 ? w : t, d == 0 ? t : w, k, Sv, cs);
  } else {
    Sv[d] = 1.0;
  }
  double ms = 0.0, ss = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ms += q[1 + a] * Sv[a];
    ss += Sv[a] * Sv[a];
  }
  const double fct = 2.0 * ms / ss;
#pragma unroll
  for (int a = 0; a < 3; ++a) q[1 + a] -= fct * Sv[a];
}

template <int LIM, typename T>
__device__ __forceinline__ void inv_flux3(const Recon<T>& rc, const FluxK<T>& K, const double* c0,
                                          const double* c1, const double* c2, const double* c3,
                                          const double* S, T* G) {
  T qL[5], qR[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    T ep, em, ep2, em2;
    extrap<LIM, T>(rc, T(c1[v] - c0[v]), T(c2[v] - c1[v]), ep, em);
    extrap<LIM, T>(rc, T(c2[v] - c1[v]), T(c3[v] - c2[v]), ep2, em2);
    qL[v] = T(c1[v]) + ep;
    qR[v] = T(c2[v]) - em2;
  }
  double A, h;
  M<double>::sqrt2(fmad(S[0], S[0], fmad(S[1], S[1], S[2] * S[2])), A, h);
  const double iA = 2.0 * h;
  const T n[3] = {T(S[0] * iA), T(S[1] * iA), T(S[2] * iA)};
  roe_flux<T, 3, -1>(qL, qR, n, T(A), K, G);
}

template <int MODE, typename T, int LIM>
__device__ void tile_gen(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                         double* __restrict__ rout, GenLds& L) {
  using SK = StageKind<MODE>;
  constexpr int bin = SK::bin;
  constexpr int bout = SK::bout;
  const int tid = threadIdx.x, li = tid & 63, lj = tid >> 6;
  const DevBlock& B = blocks[tl.blk];
  const long long ncell = B.ncell;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, nc = tl.ncol, nr = tl.ny, nz = tl.n;
  const bool curv = B.zn != nullptr;
  const bool act = li < nc && lj < nr;
  const int i = i0 + li, j = j0 + lj;
  Recon<T> rc;
  rc.lim = I.limiter;
  rc.heps = T(0.5 * I.eps);
  rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  FluxK<T> K;
  K.gm1 = T(I.gamma - 1.0);
  K.efix = T(I.efix);
  K.iefix = T(I.efix > 0.0 ? 1.0 / I.efix : 0.0);
  const double gamma = I.gamma;
  const double dt = stage_dt<MODE>(I);
  double nacc[5] = {0, 0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;

  // node plane k of the tile, (nr + 1) x (nc + 1) nodes, into slot par
  auto stage_nodes = [&](int k, int par) {
    for (int x = tid; x < (nr + 1) * (nc + 1); x += kGT) {
      const int r = x / (nc + 1), c = x - r * (nc + 1);
      double p[3];
      node3(B, i0 + c, j0 + r, k, p);
      L.nd[par][0][r][c] = p[0];
      L.nd[par][1][r][c] = p[1];
      L.nd[par][2][r][c] = p[2];
    }
  };
  auto ndp = [&](int par, int r, int c, double* o) {
    o[0] = L.nd[par][0][r][c];
    o[1] = L.nd[par][1][r][c];
    o[2] = L.nd[par][2][r][c];
  };
  // Area vector S (and S . centre) of the face of direction d on side
  // `side` (0: at i-1/2, j-1/2 or k-1/2; 1: the far face) of the cell at row
  // fr, column fc of the tile in plane k, whose bottom and top node planes
  // are in slots p0, p1.  Uniform blocks: the axis times the face area.
  auto face_at = [&](int d, int side, int p0, int p1, int fr, int fc, double* S, double& cs) {
    if (!curv) {
      S[0] = d == 0 ? B.area[0] : 0.0;
      S[1] = d == 1 ? B.area[1] : 0.0;
      S[2] = d == 2 ? B.area[2] : 0.0;
      cs = 0.0;
      return;
    }
    double a[3], b[3], c[3], e[3];
    if (d == 0) {
      const int cc = fc + side;
      ndp(p0, fr, cc, a);
      ndp(p0, fr + 1, cc, b);
      ndp(p1, fr + 1, cc, c);
      ndp(p1, fr, cc, e);
    } else if (d == 1) {
      const int rr = fr + side;
      ndp(p0, rr, fc, a);
      ndp(p0, rr, fc + 1, b);
      ndp(p1, rr, fc + 1, c);
      ndp(p1, rr, fc, e);
    } else {
      const int pp = side ? p1 : p0;
      ndp(pp, fr, fc, a);
      ndp(pp, fr, fc + 1, b);
      ndp(pp, fr + 1, fc + 1, c);
      ndp(pp, fr + 1, fc, e);
    }
    quad_face(a, b, c, e, d == 1, S, cs);
  };

  // column states at k-1, k, k+1, k+2 (at the loop head) and the k-face
  // flux at k-1/2
  double ca[5], cb[5], cc[5], cd[5], fk[5], csk = 0.0;
  for (int x = tid; x < 4 * (nc + nr); x += kGT) {
    int qr, qc;
    halo_slot(x, nc, nr, qr, qc);
    halo_source(blocks, B, bin, i0 - 2 + qc, j0 - 2 + qr, L.hp[x], L.hvs[x], L.hps[x], L.hkf[x]);
  }
  if (curv) stage_nodes(k0, 0);
  __syncthreads();
  if (act) {
    load_cell<5>(blocks, B, bin, i, j, k0 - 2, ca);
    load_cell<5>(blocks, B, bin, i, j, k0 - 1, cb);
    load_cell<5>(blocks, B, bin, i, j, k0, cc);
    load_cell<5>(blocks, B, bin, i, j, k0 + 1, cd);
    double S[3];
    face_at(2, 0, 0, 0, lj, li, S, csk);  // node plane k0 (slot 0)
    T G[5];
    inv_flux3<LIM, T>(rc, K, ca, cb, cc, cd, S, G);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      fk[v] = (double)G[v];
      ca[v] = cb[v];
      cb[v] = cc[v];
      cc[v] = cd[v];
    }
    load_cell<5>(blocks, B, bin, i, j, k0 + 2, cd);
  }

  for (int r = 0; r < nz; ++r) {
    const int k = k0 + r;
    // node slots of planes k (bottom) and k+1 (top); the third slot still
    // holds plane k-1, which a wave behind may read until the next barrier
    const int p0 = r % 3, p1 = (r + 1) % 3;
    // ---- 1. plane k into LDS: the tile's cells from registers, the halo
    //         cross (rows j0-2, j0-1, j0+nr, j0+nr+1 and columns i0-2, i0-1,
    //         i0+nc, i0+nc+1) from memory; node plane k+1
    if (act) {
#pragma unroll
      for (int v = 0; v < 5; ++v) L.q[v][lj + 2][li + 2] = cb[v];
    }
    {
      // every load of the plane's halo first (one per halo cell: its source
      // is known), then the LDS writes
      const int nh = 4 * (nc + nr);
      double hq[2][5];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = tid + h * kGT;
        if (x < nh) {
          const int kf = L.hkf[x];
          if ((kf & 15) == 1) {
#pragma unroll
            for (int v = 0; v < 5; ++v) hq[h][v] = B.bc_q[(kf >> 4) & 15][v];
          } else {
            const double* q = L.hp[x] + (long long)k * L.hps[x];
            const long long vs = L.hvs[x];
#pragma unroll
            for (int v = 0; v < 5; ++v) hq[h][v] = ldg(q + v * vs);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int x = tid + h * kGT;
        if (x < nh) {
          const int kf = L.hkf[x];
          if ((kf & 15) == 2) slip_mirror3(B, (kf >> 4) & 15, kf >> 8, k, hq[h]);
          int qr, qc;
          halo_slot(x, nc, nr, qr, qc);
#pragma unroll
          for (int v = 0; v < 5; ++v) L.q[v][qr][qc] = hq[h][v];
        }
      }
    }
    if (curv) stage_nodes(k + 1, p1);
    __syncthreads();

    // ---- 2. in-plane face fluxes to LDS, one face per thread and pass:
    //         the i-face at i-1/2 and the j-face at j-1/2 of the thread's
    //         cell, then the tile's nr right-edge and nc top-edge faces as
    //         one list of tasks, dealt to the waves in an order that turns
    //         with the plane (so that no SIMD always gets the extra pass)
    auto in_plane = [&](int d, int fr, int fc) {
      // face of direction d at row fr, column fc of the tile (i-face: at
      // i0+fc-1/2 of row j0+fr; j-face: at j0+fr-1/2 of column i0+fc)
      double S[3], cs, c0[5], c1[5], c2[5], c3[5];
      if (d == 0) {
        face_at(0, 0, p0, p1, fr, fc, S, cs);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          c0[v] = L.q[v][fr + 2][fc];
          c1[v] = L.q[v][fr + 2][fc + 1];
          c2[v] = L.q[v][fr + 2][fc + 2];
          c3[v] = L.q[v][fr + 2][fc + 3];
        }
      } else {
        face_at(1, 0, p0, p1, fr, fc, S, cs);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          c0[v] = L.q[v][fr][fc + 2];
          c1[v] = L.q[v][fr + 1][fc + 2];
          c2[v] = L.q[v][fr + 2][fc + 2];
          c3[v] = L.q[v][fr + 3][fc + 2];
        }
      }
      T G[5];
      inv_flux3<LIM, T>(rc, K, c0, c1, c2, c3, S, G);
      if (d == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) L.fi[v][fr][fc] = (double)G[v];
        L.ci[fr][fc] = cs;
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) L.fj[v][fr][fc] = (double)G[v];
        L.cj[fr][fc] = cs;
      }
    };
    // U^n and the source of the cell, loaded before the fluxes are formed
    // so that their latency hides behind them
    const long long idx = ((long long)k * B.nj + j) * B.ni + i;
    double unp[5] = {0, 0, 0, 0, 0}, srp[5] = {0, 0, 0, 0, 0};
    if (act) {
      if constexpr (SK::reads_un) {
#pragma unroll
        for (int v = 0; v < 5; ++v) unp[v] = ldg(B.u[0] + v * ncell + idx);
      }
      if (B.src != nullptr) {
#pragma unroll
        for (int v = 0; v < 5; ++v) srp[v] = ldg(B.src + v * ncell + idx);
      }
      in_plane(0, lj, li);
      in_plane(1, lj, li);
    }
    {
      const int e = (tid + 64 * (r & 3)) & (kGT - 1);
      if (e < nr) in_plane(0, e, nc);
      else if (e < nr + nc) in_plane(1, nr, e - nr);
    }
    // k-face at k+1/2 from the column's k-1 .. k+2 (registers)
    double Fh[5], cskt = 0.0;
    if (act) {
      double S[3];
      face_at(2, 1, p0, p1, lj, li, S, cskt);
      T G[5];
      inv_flux3<LIM, T>(rc, K, ca, cb, cc, cd, S, G);
#pragma unroll
      for (int v = 0; v < 5; ++v) Fh[v] = (double)G[v];
    }
    __syncthreads();

    // ---- 3. residual, source, update, partials; the column moves up
    if (act) {
      double R[5];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        R[v] = ((0.0 + (L.fi[v][lj][li + 1] - L.fi[v][lj][li])) +
                (L.fj[v][lj + 1][li] - L.fj[v][lj][li])) + (Fh[v] - fk[v]);
      // volume: 1/3 of the sum over the faces of the outward S . centre
      const double vol = curv ? (((0.0 + (L.ci[lj][li + 1] - L.ci[lj][li])) +
                                  (L.cj[lj + 1][li] - L.cj[lj][li])) + (cskt - csk)) / 3.0
                              : B.vol;
      if (B.src != nullptr) {  // the source part of Eq. (residual): - |Omega| S_h
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] -= vol * srp[v];
      }
      const double iv = M<double>::rcp(vol);
      if (MODE == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          stg(rout + B.out_off + v * ncell + idx, R[v]);
          const double rv = R[v] * iv;
          nacc[v] = fmad(rv, rv, nacc[v]);
        }
      } else {
        const double f = dt * iv;
        double out[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          double un = 0.0;
          if constexpr (SK::reads_un) un = unp[v];
          if constexpr (SK::low) {
            out[v] = fmad(-f, R[v], un);
          } else {
            const double us = fmad(-f, R[v], cb[v]);
            if (MODE == 1) out[v] = us;
            else if (MODE == 2) out[v] = fmad(0.75, un, 0.25 * us);
            else out[v] = fmad(1.0 / 3.0, un, (2.0 / 3.0) * us);
          }
          stg(B.u[bout] + v * ncell + idx, out[v]);
        }
        if (MODE == 1) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double rv = R[v] * iv;
            nacc[v] = fmad(rv, rv, nacc[v]);
          }
        }
        if constexpr (SK::cfl) {
          // mean area vectors per direction (formed again here: one stage in three)
          double Sb[3][3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            double Sm[3], Sp[3], cm, cp;
            face_at(d, 0, p0, p1, lj, li, Sm, cm);
            face_at(d, 1, p0, p1, lj, li, Sp, cp);
#pragma unroll
            for (int x = 0; x < 3; ++x) Sb[d][x] = 0.5 * (Sm[x] + Sp[x]);
          }
          dmin = fmin(dmin, cell_dt_limit<3>(out, Sb, vol, gamma, bad));
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        fk[v] = Fh[v];
        ca[v] = cb[v];
        cb[v] = cc[v];
        cc[v] = cd[v];
      }
      csk = cskt;
      if (r + 1 < nz) load_cell<5>(blocks, B, bin, i, j, k + 3, cd);
    }
    // no barrier here: the next plane's staging writes q (read before the
    // last barrier) and the node slot of plane k+2 (neither k nor k+1), and
    // its flux writes follow the next barrier, which every wave reaches only
    // after this update
  }
  __syncthreads();

  // ---- per-tile partials: fixed-order wave reductions, then the four waves
  double* part = I.part + tl.local;
  const long long ps = I.ntiles;
  if (MODE == 0 || MODE == 1) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double s = wave_sum(nacc[v]);
      if (li == 0) L.red[lj][v] = s;
    }
  }
  if (SK::cfl) {
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (li == 0) {
      L.red[lj][5] = m;
      L.red[lj][6] = (double)b;
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (MODE == 0 || MODE == 1) {
#pragma unroll
      for (int v = 0; v < 5; ++v)
        part[v * ps] = ((L.red[0][v] + L.red[1][v]) + L.red[2][v]) + L.red[3][v];
    }
    if (SK::cfl) {
      part[5 * ps] = fmin(fmin(L.red[0][5], L.red[1][5]), fmin(L.red[2][5], L.red[3][5]));
      part[6 * ps] = (L.red[0][6] + L.red[1][6] + L.red[2][6] + L.red[3][6]) != 0.0 ? 1.0 : 0.0;
    }
  }
  __syncthreads();  // L.red is reused by the next tile
}

template <int MODE, typename T>
__global__ __launch_bounds__(kGT, 2) void k_stage3d_gen(const DevTile* __restrict__ tiles,
                                                       const int* __restrict__ ntiles_p, int nfix,
                                                       int lim_fixed,
                                                       const DevBlock* __restrict__ blocks,
                                                       DevInstance* __restrict__ insts,
                                                       double* __restrict__ rout) {
  __shared__ GenLds s_lds;
  const int ntiles = nfix >= 0 ? nfix : *ntiles_p;
  for (TileWalk tw = xcd_walk(ntiles, 1, 0); tw.t < tw.end; tw.t += tw.stride) {
    const DevTile tl = tiles[tw.t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;  // the same value for the whole workgroup
    const int lim = lim_fixed >= 0 ? lim_fixed : I.limiter;
    if (lim == LIM_MINMOD) tile_gen<MODE, T, LIM_MINMOD>(tl, blocks, I, rout, s_lds);
    else tile_gen<MODE, T, -1>(tl, blocks, I, rout, s_lds);
  }
}

}  // namespace

hipError_t launch_stage3d_gen(int mode, int fp32, int grid, hipStream_t s, const DevTile* tiles,
                              const int* ntiles, int ntiles_fixed, int lim_fixed,
                              const DevBlock* blocks, DevInstance* insts, double* rout) {
  if (mode < 0 || mode > 6) return hipErrorInvalidValue;
#define FV_LG(M, T)                                                                          \
  hipLaunchKernelGGL((k_stage3d_gen<M, T>), dim3(grid), dim3(kGT), 0, s, tiles, ntiles,      \
                     ntiles_fixed, lim_fixed, blocks, insts, rout)
#define FV_LG_ALL(T)              \
  switch (mode) {                 \
    case 0: FV_LG(0, T); break;   \
    case 1: FV_LG(1, T); break;   \
    case 2: FV_LG(2, T); break;   \
    case 3: FV_LG(3, T); break;   \
    case 4: FV_LG(4, T); break;   \
    case 5: FV_LG(5, T); break;   \
    default: FV_LG(6, T); break;  \
  }
  if (fp32) {
    FV_LG_ALL(float)
  } else {
    FV_LG_ALL(double)
  }
#undef FV_LG_ALL
#undef FV_LG
  return hipGetLastError();
}

const void* stage3d_gen_kernel_ptr(int fp32) {
  return fp32 ? (const void*)&k_stage3d_gen<1, float> : (const void*)&k_stage3d_gen<1, double>;
}

}  // namespace fvk
