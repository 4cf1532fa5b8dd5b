// 2D stage kernels: MUSCL + Roe residual, SSP-RK3 stage update and the
// fused reductions, one wavefront per tile.
//
// A tile is 64 consecutive columns i (lane = column; ncol of them active) by
// n rows.  The wave marches up the rows; at row j it
//   - forms the j-face flux at j-1/2 from the extrapolations of cells j-1
//     (carried) and j (rows j-1, j, j+1 of the own column are in registers),
//   - completes the residual of row j-1 with it, applies the RK stage update
//     and stores the row (coalesced along i), adding the fused reductions,
//   - forms the i-face flux at i-1/2 of row j.  The row, with its three halo
//     cells i0-2, i0-1 and i0+ncol, goes through a per-wave LDS row buffer,
//     from which every lane reads its neighbours; the flux through i+1/2 is
//     the next lane's i-1/2 flux (the tile's right-edge fluxes come from a
//     pre-pass over the tile's rows, one row per lane).
// Everything a row needs from memory (the row two ahead, the halo cells, the
// node row two ahead, U^n) is requested one row ahead, with addresses that are
// always inside the arrays, so loads overlap a whole row of arithmetic.  Ghost
// cells are never stored: a cell outside the block is resolved to its source
// (a cell of this or a neighbour block, the inflow state, or a mirrored cell)
// before the load and corrected after it.
#include <type_traits>

#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

constexpr int kWavesPerWG = 4;
constexpr int kSlots = 72;  // LDS row slots: column i0 + c at slot c + 2; slot 71 is scratch

template <typename T>
struct Lds2D {
  T q[4][kSlots];     // stencil row of the i-faces
  T g[4][kSlots];     // i-face fluxes of the row
  T edge[4][kSlots];  // right-edge fluxes of the tile, row r at [v][r]
};

// order LDS accesses of the wave (the wave executes them in program order;
// this keeps the compiler from moving them across each other)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// wave-uniform read-only value (scalar load)
typedef __attribute__((address_space(4))) const double k_cdouble;
__device__ __forceinline__ double ldk(const double* p) { return *(const k_cdouble*)p; }

// global loads / stores at a wave-uniform base plus a per-lane byte offset
__device__ __forceinline__ double ldo(const double* base, unsigned off) {
  return *(g_cdouble*)((const char*)base + off);
}
__device__ __forceinline__ void sto(double* base, unsigned off, double v) {
  *(g_double*)((char*)base + off) = v;
}

// Where the value of cell (i, j) of block B comes from, without touching
// memory: a cell of B or of a neighbour block (kind 0), the inflow state of
// face f (kind 1; p is then some valid cell of B) or a cell mirrored about
// the wall face f (kind 2).  rs is the row stride of the source block.
struct Src2 {
  const double* p;
  long long vs;
  int rs, kind, f, t;  // t: index along the wall of the mirrored cell
};

// The ghost layer g (1 or 2) beyond face f of block B is a copy of one line
// of cells of a source block (a column for i-faces, a row for j-faces), or the
// inflow state.  With f and g the same for the whole wavefront, this is
// scalar work (no per-lane memory reads).
struct GLine {
  const double* u;  // source state buffer
  long long vs;     // its variable stride
  int rs;           // its row stride
  int along;        // source column (i-faces) or row (j-faces)
  int kind;         // 0 copy, 1 inflow state, 2 mirrored copy
};

__device__ __forceinline__ GLine ghost_line(const DevBlock* __restrict__ blocks, const DevBlock& B,
                                            int buf, int f, int g) {
  const int d = f >> 1, side = f & 1;
  const int kind = B.bc_kind[f];
  const DevBlock* S = kind == BC_BLOCK ? &blocks[B.bc_nbr[f]] : &B;
  const int n = d == 0 ? S->ni : S->nj;
  int along;
  if (kind == BC_PERIODIC || kind == BC_BLOCK) along = side == 0 ? n - g : g - 1;
  else if (kind == BC_SLIPWALL) along = side == 0 ? g - 1 : n - g;
  else along = side == 0 ? 0 : n - 1;  // EXTRAP, or INFLOW (any valid line)
  GLine L;
  L.u = S->u[buf];
  L.vs = S->ncell;
  L.rs = S->ni;
  L.along = along;
  L.kind = kind == BC_INFLOW ? 1 : (kind == BC_SLIPWALL ? 2 : 0);
  return L;
}

// cell (col, jr) of the own column with jr wave-uniform (inside the block, or
// up to two rows beyond a j-face)
__device__ __forceinline__ Src2 col_src(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf,
                                        int col, int jr) {
  Src2 s;
  s.f = 0;
  s.t = col;
  if (jr >= 0 && jr < B.nj) {
    s.p = B.u[buf] + (long long)jr * B.ni + col;
    s.vs = B.ncell;
    s.rs = B.ni;
    s.kind = 0;
    return s;
  }
  const int f = jr < 0 ? 2 : 3;
  const GLine L = ghost_line(blocks, B, buf, f, jr < 0 ? -jr : jr - B.nj + 1);
  s.p = L.u + (long long)L.along * L.rs + col;
  s.vs = L.vs;
  s.rs = L.rs;
  s.kind = L.kind;
  s.f = f;
  return s;
}

// cell (ic_, row) with the column ic_ wave-uniform (inside the block, or up to
// two columns beyond an i-face) and the row inside the block
__device__ __forceinline__ Src2 row_src(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf,
                                        int icol, int row) {
  Src2 s;
  s.f = 0;
  s.t = row;
  if (icol >= 0 && icol < B.ni) {
    s.p = B.u[buf] + (long long)row * B.ni + icol;
    s.vs = B.ncell;
    s.rs = B.ni;
    s.kind = 0;
    return s;
  }
  const int f = icol < 0 ? 0 : 1;
  const GLine L = ghost_line(blocks, B, buf, f, icol < 0 ? -icol : icol - B.ni + 1);
  s.p = L.u + (long long)row * L.rs + L.along;
  s.vs = L.vs;
  s.rs = L.rs;
  s.kind = L.kind;
  s.f = f;
  return s;
}

// inflow state, or the mirror m - 2 (m.S)/(S.S) S about a wall face of area
// vector (sx, sy) given by the caller
__device__ __forceinline__ void fix_with(const Src2& s, const DevBlock& B, double sx, double sy,
                                         double (&q)[4]) {
  if (s.kind == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = B.bc_q[s.f][v];
  } else if (s.kind == 2) {
    const double ms = q[1] * sx + q[2] * sy;
    const double ss = sx * sx + sy * sy;
    const double fct = 2.0 * ms / ss;
    q[1] -= fct * sx;
    q[2] -= fct * sy;
  }
}

__device__ __forceinline__ void load2(const Src2& s, double (&q)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) q[v] = ldg(s.p + v * s.vs);
}

// inflow state or slip-wall mirror: m - 2 (m.S)/(S.S) S with S the area
// vector of the wall face next to the ghost cell
template <bool CURV>
__device__ __forceinline__ void fix2(const Src2& s, const DevBlock& B, double (&q)[4]) {
  if (s.kind == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = B.bc_q[s.f][v];
  } else if (s.kind == 2) {
    double Sx, Sy;
    if (CURV) {
      const long long w1 = B.ni + 1;
      if (s.f < 2) {
        const int w = s.f == 0 ? 0 : B.ni;
        Sx = ldg(B.yn + (long long)(s.t + 1) * w1 + w) - ldg(B.yn + (long long)s.t * w1 + w);
        Sy = -(ldg(B.xn + (long long)(s.t + 1) * w1 + w) - ldg(B.xn + (long long)s.t * w1 + w));
      } else {
        const long long w = s.f == 2 ? 0 : B.nj;
        Sx = -(ldg(B.yn + w * w1 + s.t + 1) - ldg(B.yn + w * w1 + s.t));
        Sy = ldg(B.xn + w * w1 + s.t + 1) - ldg(B.xn + w * w1 + s.t);
      }
    } else {
      Sx = s.f < 2 ? 1.0 : 0.0;
      Sy = s.f < 2 ? 0.0 : 1.0;
    }
    const double ms = q[1] * Sx + q[2] * Sy;
    const double ss = Sx * Sx + Sy * Sy;
    const double fct = 2.0 * ms / ss;
    q[1] -= fct * Sx;
    q[2] -= fct * Sy;
  }
}

// flux across a face of area vector (Sx, Sy) (curvilinear) or of the
// uniform area `area` along axis AX
template <typename T, int AX, bool CURV>
__device__ __forceinline__ void face_flux(const FluxK<T>& K, const T (&qL)[4], const T (&qR)[4],
                                          double Sx, double Sy, double area, T (&G)[4]) {
  if constexpr (CURV) {
    double A, h;
    M<double>::sqrt2(fmad(Sx, Sx, Sy * Sy), A, h);
    const double iA = 2.0 * h;
    const T n[2] = {T(Sx * iA), T(Sy * iA)};
    roe_flux<T, 2, -1>(qL, qR, n, T(A), K, G);
  } else {
    roe_flux<T, 2, AX>(qL, qR, nullptr, T(area), K, G);
  }
}

template <int MODE, typename T, bool CURV, int LIM>
__device__ __forceinline__ void tile2d(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                       double* __restrict__ rout, int lane, Lds2D<T>& L) {
  prio_by_progress(0);
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni, nj = B.nj;
  const int i0 = tl.i0, j0 = tl.j0, n = tl.n, nc = tl.ncol;
  const bool act = lane < nc;
  const int ic = act ? i0 + lane : ni - 1;  // safe column for idle lanes
  const int last = nc - 1;                  // lane owning the tile's right edge
  using SK = StageKind<MODE>;
  constexpr int bin = SK::bin;
  constexpr int bout = SK::bout;
  const long long ncell = B.ncell;
  const double* __restrict__ Q = B.u[bin];
  const double* __restrict__ Un = B.u[0];
  double* __restrict__ Uout = B.u[bout];
  const double* __restrict__ X = B.xn;
  const double* __restrict__ Y = B.yn;
  const long long nrow = ni + 1;           // node row length
  const unsigned cb = (unsigned)ic * 8u;   // own column, bytes
  const int ir = i0 + nc;                  // node column right of the tile

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
  const double areaI = B.area[0], areaJ = B.area[1], uvol = B.vol;

  // ---- halo lanes: 0 -> column i0-1, 1 -> i0-2, 2 -> i0+ncol (others: own column)
  const Src2 h0 = row_src(blocks, B, bin, i0 - 1, 0);
  const Src2 h1 = row_src(blocks, B, bin, i0 - 2, 0);
  const Src2 h2 = row_src(blocks, B, bin, ir, 0);
  const Src2 hown = row_src(blocks, B, bin, ic, 0);
  const Src2 hs = lane == 0 ? h0 : (lane == 1 ? h1 : (lane == 2 ? h2 : hown));  // row j: hs.p + j * hs.rs
  const bool hfix = __builtin_amdgcn_ballot_w64(hs.kind != 0) != 0;
  const int hslot = lane == 0 ? 1 : (lane == 1 ? 0 : (lane == 2 ? nc + 2 : kSlots - 1));
  auto halo_load = [&](int j, double (&h)[4]) {
    const int jc = min(j, nj - 1);
    const double* p = hs.p + (long long)jc * hs.rs;
#pragma unroll
    for (int v = 0; v < 4; ++v) h[v] = ldg(p + v * hs.vs);
  };
  auto halo_fix = [&](int j, double (&h)[4]) {
    if (hfix) {
      Src2 s = hs;
      s.t = j;
      fix2<CURV>(s, B, h);
    }
  };
  // own column, row j (inside the block)
  auto row_load = [&](const double* base, int j, double (&q)[4]) {
    const double* p = base + (long long)j * ni;
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = ldo(p + v * ncell, cb);
  };

  // ---- prologue: rows j0-2 .. j0+1, halo of row j0, node rows j0, j0+1,
  //      and everything the right-edge pre-pass reads (issued together)
  double qa[4], qm1[4], q0[4], qn[4], hv[4], un[4] = {0, 0, 0, 0};
  const Src2 sa = col_src(blocks, B, bin, ic, j0 - 2);
  const Src2 sb = col_src(blocks, B, bin, ic, j0 - 1);
  const Src2 sd = col_src(blocks, B, bin, ic, j0 + 1);
  // area vectors of the bottom / top wall faces of the own column, for the
  // slip-wall ghosts of this tile (read with the prologue)
  double bwx = 0, bwy = 1, twx = 0, twy = 1;
  const bool bwall = j0 < 2 && B.bc_kind[2] == BC_SLIPWALL;
  const bool twall = j0 + n + 2 > nj && B.bc_kind[3] == BC_SLIPWALL;
  if constexpr (CURV) {
    if (bwall) {
      bwx = -(ldo(Y + 1, cb) - ldo(Y, cb));
      bwy = ldo(X + 1, cb) - ldo(X, cb);
    }
    if (twall) {
      const double* xw = X + (long long)nj * nrow;
      const double* yw = Y + (long long)nj * nrow;
      twx = -(ldo(yw + 1, cb) - ldo(yw, cb));
      twy = ldo(xw + 1, cb) - ldo(xw, cb);
    }
  }
  load2(sa, qa);
  load2(sb, qm1);
  row_load(Q, j0, q0);
  load2(sd, qn);
  halo_load(j0, hv);
  double x0 = 0, y0 = 0, x1 = 0, y1 = 0, xR0 = 0, yR0 = 0, xR1 = 0, yR1 = 0;
  if constexpr (CURV) {
    const double* xr = X + j0 * nrow;
    const double* yr = Y + j0 * nrow;
    x0 = ldo(xr, cb);
    y0 = ldo(yr, cb);
    x1 = ldo(xr + nrow, cb);
    y1 = ldo(yr + nrow, cb);
    xR0 = ldk(xr + ir);
    yR0 = ldk(yr + ir);
    xR1 = ldk(xr + nrow + ir);
    yR1 = ldk(yr + nrow + ir);
  }
  // pre-pass: i-face flux through the tile's right edge for row j0 + lane
  const int er = j0 + min(lane, n - 1);
  Src2 se[4];
  double ce[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    se[c] = row_src(blocks, B, bin, ir - 2 + c, er);
    load2(se[c], ce[c]);
  }
  double ex0 = 0, ey0 = 0, ex1 = 0, ey1 = 0;
  if constexpr (CURV) {
    ex0 = ldg(X + er * nrow + ir);
    ey0 = ldg(Y + er * nrow + ir);
    ex1 = ldg(X + (er + 1) * nrow + ir);
    ey1 = ldg(Y + (er + 1) * nrow + ir);
  }
  // the first row step's next row (j0 + 2), issued last in the prologue batch
  // so that it has arrived by the end of that step
  double q2p[4];
  Src2 s2p;
  s2p.kind = 0;
  s2p.f = 0;
  if (j0 + 2 < nj) {
    row_load(Q, j0 + 2, q2p);
  } else {
    s2p = col_src(blocks, B, bin, ic, j0 + 2);
    load2(s2p, q2p);
  }
  double x2p = 0, y2p = 0, xR2p = 0, yR2p = 0;
  if constexpr (CURV) {
    const long long jr = min(j0 + 2, nj);
    x2p = ldo(X + jr * nrow, cb);
    y2p = ldo(Y + jr * nrow, cb);
    xR2p = ldk(X + jr * nrow + ir);
    yR2p = ldk(Y + jr * nrow + ir);
  }
  // a stopped instance's tiles leave here, before any store: the check waits
  // on a load issued together with the descriptors, not ahead of them
  if (MODE != 0 && I.stopped) return;
  // ghost corrections of the prologue cells
  fix_with(sa, B, bwx, bwy, qa);
  fix_with(sb, B, bwx, bwy, qm1);
  fix_with(sd, B, twx, twy, qn);
#pragma unroll
  for (int c = 0; c < 4; ++c) fix2<CURV>(se[c], B, ce[c]);
  T epm1[4];  // + side extrapolation of cell j-1
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T em;
    extrap<LIM>(rc, T(qm1[v]) - T(qa[v]), T(q0[v]) - T(qm1[v]), epm1[v], em);
  }
  // right neighbour's node of row j0 (the last lane takes the node right of the tile)
  double x0r = 0, y0r = 0;
  if constexpr (CURV) {
    const double xs = shl1(x0), ys = shl1(y0);
    x0r = lane == last ? xR0 : xs;
    y0r = lane == last ? yR0 : ys;
  }
  double xm = 0, ym = 0, xmr = 0, ymr = 0;  // node row j-1 (own, right neighbour)
  double rg[4] = {0, 0, 0, 0};  // (G_i+1/2 - G_i-1/2) - G_j-1/2 of the pending row j-1
  double nacc[4] = {0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;
  // LDS addresses of this lane
  T* const qs_own = &L.q[0][lane + 2];
  T* const qs_halo = &L.q[0][hslot];
  T* const gs_own = &L.g[0][lane];

  // one row of the march; FIRST: no pending row below, LASTR: the row above the tile
  auto step = [&](auto first_t, auto last_t, int r) {
    constexpr bool FIRST = decltype(first_t)::value;
    constexpr bool LASTR = decltype(last_t)::value;
    const int j = j0 + r;
    // ---- (1) requests for the next row
    double q2[4];
    double x2 = 0, y2 = 0, xR2 = 0, yR2 = 0;
    Src2 s2;
    s2.kind = 0;
    s2.f = 0;
    if constexpr (FIRST) {
#pragma unroll
      for (int v = 0; v < 4; ++v) q2[v] = q2p[v];
      s2 = s2p;
      x2 = x2p;
      y2 = y2p;
      xR2 = xR2p;
      yR2 = yR2p;
    } else if constexpr (!LASTR) {
      if (j + 2 < nj) {
        row_load(Q, j + 2, q2);
      } else {  // a ghost row beyond the top face
        s2 = col_src(blocks, B, bin, ic, j + 2);
        load2(s2, q2);
      }
      if constexpr (CURV) {
        const long long jr = min(j + 2, nj);
        x2 = ldo(X + jr * nrow, cb);
        y2 = ldo(Y + jr * nrow, cb);
        xR2 = ldk(X + jr * nrow + ir);
        yR2 = ldk(Y + jr * nrow + ir);
      }
    }
    // ---- (2) row j through the LDS row buffer: i-neighbours and halo cells
    T qim2[4], qim1[4], qip1[4];
    if constexpr (!LASTR) {
      halo_fix(j, hv);
#pragma unroll
      for (int v = 0; v < 4; ++v) qs_own[v * kSlots] = T(q0[v]);
#pragma unroll
      for (int v = 0; v < 4; ++v) qs_halo[v * kSlots] = T(hv[v]);
      wave_lds_sync();
      halo_load(j + 1, hv);  // halo of the next row
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qim2[v] = qs_own[v * kSlots - 2];
        qim1[v] = qs_own[v * kSlots - 1];
        qip1[v] = qs_own[v * kSlots + 1];
      }
    }
    // ---- (3) j-face at j-1/2 and i-face at i-1/2 (independent: their
    //      arithmetic interleaves in one scheduling region)
    T ep0[4], Gj[4], Gi[4];
    {
      T qL[4], qR[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T a = T(qm1[v]), b = T(q0[v]), c = T(qn[v]);
        T em;
        extrap<LIM>(rc, b - a, c - b, ep0[v], em);
        qL[v] = a + epm1[v];
        qR[v] = b - em;
      }
      face_flux<T, 1, CURV>(K, qL, qR, -(y0r - y0), x0r - x0, areaJ, Gj);
    }
    if constexpr (!LASTR) {
      T qL[4], qR[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T c = T(q0[v]);
        T epl, eml, epc, emc;
        extrap<LIM>(rc, qim1[v] - qim2[v], c - qim1[v], epl, eml);  // cell i-1
        extrap<LIM>(rc, c - qim1[v], qip1[v] - c, epc, emc);        // cell i
        qL[v] = qim1[v] + epl;
        qR[v] = c - emc;
      }
      face_flux<T, 0, CURV>(K, qL, qR, y1 - y0, -(x1 - x0), areaI, Gi);
    }
    if constexpr (FIRST) {
      // the pre-pass: i-face flux through the tile's right edge for row j0 + lane
      // (independent of the row's two fluxes; formed alongside them)
      T qL[4], qR[4], G[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T a = T(ce[0][v]), b = T(ce[1][v]), c = T(ce[2][v]), d = T(ce[3][v]);
        T ep, em, ep2, em2;
        extrap<LIM>(rc, b - a, c - b, ep, em);    // cell ir-1
        extrap<LIM>(rc, c - b, d - c, ep2, em2);  // cell ir
        qL[v] = b + ep;
        qR[v] = c - em2;
      }
      face_flux<T, 0, CURV>(K, qL, qR, ey1 - ey0, -(ex1 - ex0), areaI, G);
#pragma unroll
      for (int v = 0; v < 4; ++v) L.edge[v][lane] = G[v];
    }
    // ---- (4) complete, update and store row j-1
    if constexpr (!FIRST) {
      if (act) {
        const long long ro = (long long)(j - 1) * ni;
        double R[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) R[v] = rg[v] + (double)Gj[v];
        double vol = uvol;
        if constexpr (CURV) vol = 0.5 * fmad(x0r - xm, y0 - ymr, -((x0 - xmr) * (y0r - ym)));
        const double iv = M<double>::rcp(vol);
        if (MODE == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            sto(rout + B.out_off + v * ncell + ro, cb, R[v]);
            const double rv = R[v] * iv;
            nacc[v] = fmad(rv, rv, nacc[v]);
          }
        } else {
          const double f = dt * iv;
          double out[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if constexpr (SK::low) {
              out[v] = fmad(-f, R[v], un[v]);
            } else {
              const double us = fmad(-f, R[v], qm1[v]);
              if (MODE == 1) out[v] = us;
              else if (MODE == 2) out[v] = fmad(0.75, un[v], 0.25 * us);
              else out[v] = fmad(1.0 / 3.0, un[v], (2.0 / 3.0) * us);
            }
            sto(Uout + v * ncell + ro, cb, out[v]);
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
            if constexpr (CURV) {
              Sb[0][0] = 0.5 * ((y0 - ym) + (y0r - ymr));
              Sb[0][1] = -0.5 * ((x0 - xm) + (x0r - xmr));
              Sb[1][0] = -0.5 * ((ymr - ym) + (y0r - y0));
              Sb[1][1] = 0.5 * ((xmr - xm) + (x0r - x0));
            } else {
              Sb[0][0] = areaI;
              Sb[0][1] = 0.0;
              Sb[1][0] = 0.0;
              Sb[1][1] = areaJ;
            }
            Sb[0][2] = Sb[1][2] = 0.0;
            dmin = fmin(dmin, cell_dt_limit<2>(out, Sb, vol, gamma, bad));
          }
        }
      }
    }
    // U^n of row j, for the update at the next row
    if constexpr (!LASTR) {
      if constexpr (SK::reads_un) row_load(Un, j, un);
    }
    // ---- (5) the right neighbours' i-face fluxes: pending part of row j
    if constexpr (!LASTR) {
#pragma unroll
      for (int v = 0; v < 4; ++v) gs_own[v * kSlots] = Gi[v];
      wave_lds_sync();
      const T* gsrc = lane == last ? &L.edge[0][r] : &L.g[0][lane + 1];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T gr = gsrc[v * kSlots];
        rg[v] = ((double)gr - (double)Gi[v]) - (double)Gj[v];
      }
      wave_lds_sync();
    }
    // ---- (6) rotate the carried rows
    if constexpr (!LASTR) {
      if (j + 2 >= nj) fix_with(s2, B, twx, twy, q2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        qm1[v] = q0[v];
        q0[v] = qn[v];
        qn[v] = q2[v];
        epm1[v] = ep0[v];
      }
      if constexpr (CURV) {
        xm = x0;
        ym = y0;
        xmr = x0r;
        ymr = y0r;
        const double xs = shl1(x1), ys = shl1(y1);
        x0r = lane == last ? xR1 : xs;
        y0r = lane == last ? yR1 : ys;
        x0 = x1;
        y0 = y1;
        x1 = x2;
        y1 = y2;
        xR1 = xR2;
        yR1 = yR2;
      }
    }
  };

  using F = std::integral_constant<bool, false>;
  using Tr = std::integral_constant<bool, true>;
  step(Tr(), F(), 0);
  prio_by_progress(1);
  for (int r = 1; r < n; ++r) {
    step(F(), F(), r);
    prio_by_progress(r + 1);
  }
  step(F(), Tr(), n);

  // ---- per-tile partials (fixed-order wave reductions)
  double* part = I.part + tl.local;
  const long long ps = I.ntiles;
  if (MODE == 0 || MODE == 1) {
    double s[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = wave_sum(nacc[v]);
    if (lane == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) part[v * ps] = s[v];
      part[4 * ps] = 0.0;
    }
  }
  if (SK::cfl) {
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      part[5 * ps] = m;
      part[6 * ps] = (double)b;
    }
  }
}

// at most 256 VGPRs: two waves per SIMD
template <int MODE, typename T>
__global__ __launch_bounds__(256, 2) void k_stage2d(const DevTile* __restrict__ tiles,
                                                 const int* __restrict__ ntiles_p, int nfix, int lim_fixed,
                                                 const DevBlock* __restrict__ blocks,
                                                 DevInstance* __restrict__ insts,
                                                 double* __restrict__ rout) {
  __shared__ Lds2D<T> s_lds[kWavesPerWG];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // a count fixed at launch saves one dependent load before the first tile
  const int ntiles = nfix >= 0 ? nfix : *ntiles_p;
  for (TileWalk tw = xcd_walk(ntiles, kWavesPerWG, wid); tw.t < tw.end; tw.t += tw.stride) {
    const DevTile tl = tiles[tw.t];
    DevInstance& I = insts[tl.inst];
    // the common configuration (minmod) is compiled with the limiter fixed.
    // With the limiter given at launch and the block kind in the tile, the
    // choice needs no descriptor read: the tile routine reads the instance
    // and block descriptors in one batch (and checks for a stopped instance
    // there).
    const int lim = lim_fixed >= 0 ? lim_fixed : I.limiter;
    if (lim == LIM_MINMOD) {
      if (tl.curv) tile2d<MODE, T, true, LIM_MINMOD>(tl, blocks, I, rout, lane, s_lds[wid]);
      else tile2d<MODE, T, false, LIM_MINMOD>(tl, blocks, I, rout, lane, s_lds[wid]);
    } else {
      if (tl.curv) tile2d<MODE, T, true, -1>(tl, blocks, I, rout, lane, s_lds[wid]);
      else tile2d<MODE, T, false, -1>(tl, blocks, I, rout, lane, s_lds[wid]);
    }
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
          vol = 0.5 * fmad(xd - xa, yc - yb, -((xc - xb) * (yd - ya)));
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
        dmin = fmin(dmin, I.mu > 0.0
                              ? cell_dt_limit_visc(q, Sb, vol, I.gamma, I.mu, I.prandtl, bad)
                              : cell_dt_limit<2>(q, Sb, vol, I.gamma, bad));
      }
    }
    const double m = wave_min(dmin);
    const int b = wave_or(bad);
    if (lane == 0) {
      double* part = I.part + tl.local;
      const long long ps = I.ntiles;
      part[5 * ps] = m;
      part[6 * ps] = (double)b;
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_stage2d(int mode, int fp32, int grid, int block, hipStream_t s, const DevTile* tiles,
                          const int* ntiles, int ntiles_fixed, int lim_fixed, const DevBlock* blocks,
                          DevInstance* insts, double* rout) {
  if (mode < 0 || mode > 6) return hipErrorInvalidValue;
#define FV_L2(M, T) hipLaunchKernelGGL((k_stage2d<M, T>), dim3(grid), dim3(block), 0, s, tiles, ntiles, ntiles_fixed, lim_fixed, blocks, insts, rout)
#define FV_L2_ALL(T)              \
  switch (mode) {                 \
    case 0: FV_L2(0, T); break;   \
    case 1: FV_L2(1, T); break;   \
    case 2: FV_L2(2, T); break;   \
    case 3: FV_L2(3, T); break;   \
    case 4: FV_L2(4, T); break;   \
    case 5: FV_L2(5, T); break;   \
    default: FV_L2(6, T); break;  \
  }
  if (fp32) {
    FV_L2_ALL(float)
  } else {
    FV_L2_ALL(double)
  }
#undef FV_L2_ALL
#undef FV_L2
  return hipGetLastError();
}
hipError_t launch_cfl2d(int grid, int block, hipStream_t s, const DevTile* tiles, const int* ntiles,
                        const DevBlock* blocks, DevInstance* insts) {
  hipLaunchKernelGGL(k_cfl2d, dim3(grid), dim3(block), 0, s, tiles, ntiles, blocks, insts);
  return hipGetLastError();
}
const void* stage2d_kernel_ptr(int mode, int fp32) {
  static const void* const kf[7] = {(const void*)&k_stage2d<0, float>, (const void*)&k_stage2d<1, float>,
                                    (const void*)&k_stage2d<2, float>, (const void*)&k_stage2d<3, float>,
                                    (const void*)&k_stage2d<4, float>, (const void*)&k_stage2d<5, float>,
                                    (const void*)&k_stage2d<6, float>};
  static const void* const kd[7] = {(const void*)&k_stage2d<0, double>, (const void*)&k_stage2d<1, double>,
                                    (const void*)&k_stage2d<2, double>, (const void*)&k_stage2d<3, double>,
                                    (const void*)&k_stage2d<4, double>, (const void*)&k_stage2d<5, double>,
                                    (const void*)&k_stage2d<6, double>};
  const int m = mode < 0 ? 0 : (mode > 6 ? 6 : mode);
  return fp32 ? kf[m] : kd[m];
}

}  // namespace fvk
