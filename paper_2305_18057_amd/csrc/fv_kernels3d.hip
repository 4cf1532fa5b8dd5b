// 3D stage kernels (uniform grids): MUSCL + Roe residual, SSP-RK3 stage
// update and fused reductions.  One workgroup per tile.
//
// A tile is 64 columns i (lane) by ny <= NY rows j (one wavefront per row)
// and marches over n <= 64 planes k.  The workgroup has NY + 1 waves: waves
// 0..NY-1 own the rows; wave NY (the helper) owns no cells: one plane ahead it
// fetches the four j-halo rows and the i-halo cells of the tile, stages them
// in LDS, and forms the j-face flux through the tile's top edge and the i-face
// fluxes through its right edge (one row per lane).  Per plane k:
//   - each row wave forms the k-face flux at k-1/2 (planes k-1, k, k+1 of its
//     column in registers, k+2 in flight), completes the residual of plane
//     k-1, applies the stage update and stores it;
//   - the plane is staged in LDS (rows j0-2 .. j0+ny+1, each row with the
//     i-halo slots i0-2, i0-1, i0+ncol, i0+ncol+1); every row wave forms its
//     j-face flux at j-1/2 and its i-face flux at i-1/2 from LDS; the fluxes
//     are exchanged through LDS and each row keeps the in-plane part of its
//     residual for the next plane.
// Two workgroup barriers per plane; every face flux of the tile is formed
// once (tile edges aside).  Loads for the next plane are issued one plane
// ahead at addresses inside the arrays; ghost cells are resolved to their
// source before the load and corrected after it.
#include <type_traits>

#include "fv_device.h"
#include "fv_launch.h"

namespace fvk {

namespace {

constexpr int kS3 = 72;  // LDS row slots: column i0 + c at slot c + 2; slot 71 is scratch

// q and f are double-buffered by plane parity: plane r of a tile is staged
// in q[r & 1] and its j-face fluxes go to f[r & 1], so the waves of a
// workgroup meet once per plane (they write plane r + 1 while others may
// still read plane r).  g is read and written by its own row wave only.
template <typename T, int NY>
struct Smem3 {
  T q[2][NY + 4][5][kS3];  // plane k: rows j0-2 .. j0+NY+1
  T f[2][NY + 1][5][64];   // j-face fluxes at j-1/2, rows j0 .. j0+NY
  T g[NY][5][kS3];         // i-face fluxes of each row
  T edge[NY][5][64];       // right-edge i-face fluxes, per row, plane r at [r]
  double red[(NY + 1) * 8];
};

// Where a cell of block B comes from, without touching memory (as in 2D):
// kind 0 a cell of B or a neighbour block, 1 the inflow state of face f, 2 the
// cell mirrored about the wall face f.  p points at the cell (or, for the
// column forms below, at its plane 0); vs, ps, rs: variable, plane and row
// strides of the source block.
struct Src3 {
  const double* p;
  long long vs, ps;
  int rs, kind, f;
};

// The ghost layer g (1 or 2) beyond face f of block B copies the plane of
// index `along` (along the face normal) of a source block, or takes the inflow
// state.  f and g are the same for the whole wavefront: scalar work.
struct GPlane3 {
  const double* u;
  long long vs;
  int ni, nj, along, kind;
};

__device__ __forceinline__ GPlane3 ghost_plane3(const DevBlock* __restrict__ blocks,
                                                const DevBlock& B, int buf, int f, int g) {
  const int d = f >> 1, side = f & 1;
  const int kind = B.bc_kind[f];
  const DevBlock* S = kind == BC_BLOCK ? &blocks[B.bc_nbr[f]] : &B;
  const int n = d == 0 ? S->ni : (d == 1 ? S->nj : S->nk);
  int along;
  if (kind == BC_PERIODIC || kind == BC_BLOCK) along = side == 0 ? n - g : g - 1;
  else if (kind == BC_SLIPWALL) along = side == 0 ? g - 1 : n - g;
  else along = side == 0 ? 0 : n - 1;  // EXTRAP, or INFLOW (any valid plane)
  GPlane3 G;
  G.u = S->u[buf];
  G.vs = S->ncell;
  G.ni = S->ni;
  G.nj = S->nj;
  G.along = along;
  G.kind = kind == BC_INFLOW ? 1 : (kind == BC_SLIPWALL ? 2 : 0);
  return G;
}

__device__ __forceinline__ Src3 own3(const DevBlock& B, int buf, long long off) {
  Src3 s;
  s.p = B.u[buf] + off;
  s.vs = B.ncell;
  s.ps = (long long)B.ni * B.nj;
  s.rs = B.ni;
  s.kind = 0;
  s.f = 0;
  return s;
}

__device__ __forceinline__ Src3 from_ghost3(const GPlane3& G, int f, long long off) {
  Src3 s;
  s.p = G.u + off;
  s.vs = G.vs;
  s.ps = (long long)G.ni * G.nj;
  s.rs = G.ni;
  s.kind = G.kind;
  s.f = f;
  return s;
}

// per-field select (a select of whole structs can end up in scratch memory)
__device__ __forceinline__ Src3 sel3(bool c, const Src3& a, const Src3& b) {
  Src3 s;
  s.p = c ? a.p : b.p;
  s.vs = c ? a.vs : b.vs;
  s.ps = c ? a.ps : b.ps;
  s.rs = c ? a.rs : b.rs;
  s.kind = c ? a.kind : b.kind;
  s.f = c ? a.f : b.f;
  return s;
}

// cell (i, j, k) with k wave-uniform, i and j inside the block
__device__ __forceinline__ Src3 src3_k(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf,
                                       int i, int j, int k) {
  if (k >= 0 && k < B.nk) return own3(B, buf, ((long long)k * B.nj + j) * B.ni + i);
  const int f = k < 0 ? 4 : 5;
  const GPlane3 G = ghost_plane3(blocks, B, buf, f, k < 0 ? -k : k - B.nk + 1);
  return from_ghost3(G, f, ((long long)G.along * G.nj + j) * G.ni + i);
}

// column (i, j) with i wave-uniform (inside the block or up to two cells past
// an i-face) and j inside the block; p is its plane 0 (add k * ps)
__device__ __forceinline__ Src3 src3_i(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf,
                                       int i, int j) {
  if (i >= 0 && i < B.ni) return own3(B, buf, (long long)j * B.ni + i);
  const int f = i < 0 ? 0 : 1;
  const GPlane3 G = ghost_plane3(blocks, B, buf, f, i < 0 ? -i : i - B.ni + 1);
  return from_ghost3(G, f, (long long)j * G.ni + G.along);
}

// column (i, j) with j wave-uniform (inside the block or up to two cells past
// a j-face) and i inside the block; p is its plane 0
__device__ __forceinline__ Src3 src3_j(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf,
                                       int i, int j) {
  if (j >= 0 && j < B.nj) return own3(B, buf, (long long)j * B.ni + i);
  const int f = j < 0 ? 2 : 3;
  const GPlane3 G = ghost_plane3(blocks, B, buf, f, j < 0 ? -j : j - B.nj + 1);
  return from_ghost3(G, f, (long long)G.along * G.ni + i);
}

__device__ __forceinline__ void load3(const double* p, long long vs, double (&q)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = ldg(p + v * vs);
}

// inflow state, or the uniform-grid slip-wall mirror (normal momentum negated)
__device__ __forceinline__ void fix3(int kind, int f, const DevBlock& B, double (&q)[5]) {
  if (kind == 1) {
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = B.bc_q[f][v];
  } else if (kind == 2) {
    // m - 2 (m.S)/(S.S) S with S along axis f/2: the normal component flips
    // (selected per component: a run-time index would put q in scratch memory)
    const int d = f >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) q[1 + a] -= a == d ? 2.0 * q[1 + a] : 0.0;
  }
}

__device__ __forceinline__ double ldo3(const double* base, unsigned off) {
  return *(g_cdouble*)((const char*)base + off);
}
__device__ __forceinline__ void sto3(double* base, unsigned off, double v) {
  *(g_double*)((char*)base + off) = v;
}

template <int LIM, typename T>
__device__ __forceinline__ void face_states(const Recon<T>& rc, T a, T b, T c, T d, T& qL, T& qR) {
  T ep, em, ep2, em2;
  extrap<LIM>(rc, b - a, c - b, ep, em);    // cell of b
  extrap<LIM>(rc, c - b, d - c, ep2, em2);  // cell of c
  qL = b + ep;
  qR = c - em2;
}

template <typename T>
__device__ __forceinline__ void setup_consts(const DevInstance& I, Recon<T>& rc, FluxK<T>& K) {
  rc.lim = I.limiter;
  rc.heps = T(0.5 * I.eps);
  rc.c1 = T(0.25 * I.eps * (1.0 - I.kappa));
  rc.c2 = T(0.25 * I.eps * (1.0 + I.kappa));
  K.gm1 = T(I.gamma - 1.0);
  K.efix = T(I.efix);
  K.iefix = T(I.efix > 0.0 ? 1.0 / I.efix : 0.0);
}

// The helper wave: per plane, stage the j-halo rows and the i-halo cells in
// LDS (fetched one plane ahead) and form the tile's top-edge j-face flux and
// right-edge i-face fluxes.
template <int MODE, typename T, int NY, int LIM>
__device__ void helper3d(const DevTile& tl, const DevBlock* __restrict__ blocks, const DevInstance& I,
                         int lane, Smem3<T, NY>& sm) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, n = tl.n, nc = tl.ncol, ny = tl.ny;
  constexpr int bin = StageKind<MODE>::bin;
  const int ic = lane < nc ? i0 + lane : ni - 1;
  Recon<T> rc;
  FluxK<T> K;
  setup_consts(I, rc, K);
  const T ax = T(B.area[0]), ay = T(B.area[1]);
  // j-halo rows of the own column: j0-2, j0-1, j0+ny, j0+ny+1
  const int hrow[4] = {j0 - 2, j0 - 1, j0 + ny, j0 + ny + 1};
  Src3 hs[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) hs[h] = src3_j(blocks, B, bin, ic, hrow[h]);
  // i-halo cells: lane = 4 * row + which; which 0: i0-1, 1: i0-2, 2: i0+ncol,
  // 3: i0+ncol+1 (four wave-uniform columns, the row per lane)
  const int hr = lane >> 2, hw = lane & 3;
  const bool hlane = hr < ny;
  const Src3 c0 = src3_i(blocks, B, bin, i0 - 1, 0);
  const Src3 c1 = src3_i(blocks, B, bin, i0 - 2, 0);
  const Src3 c2 = src3_i(blocks, B, bin, i0 + nc, 0);
  const Src3 c3 = src3_i(blocks, B, bin, i0 + nc + 1, 0);
  const Src3 cown = own3(B, bin, (long long)j0 * ni + ic);
  Src3 cs = sel3(!hlane, cown, sel3(hw == 0, c0, sel3(hw == 1, c1, sel3(hw == 2, c2, c3))));
  if (hlane) cs.p += (long long)(j0 + hr) * cs.rs;
  const int cslot = hw == 0 ? 1 : (hw == 1 ? 0 : (hw == 2 ? nc + 2 : nc + 3));
  const int crow = hlane ? hr + 2 : 0;
  const bool fixrows = __builtin_amdgcn_ballot_w64(hs[0].kind != 0 || hs[1].kind != 0 ||
                                                    hs[2].kind != 0 || hs[3].kind != 0) != 0;
  const bool fixcells = __builtin_amdgcn_ballot_w64(hlane && cs.kind != 0) != 0;
  double hv[4][5], cv[5];
#pragma unroll
  for (int h = 0; h < 4; ++h) load3(hs[h].p + (long long)k0 * hs[h].ps, hs[h].vs, hv[h]);
  load3(cs.p + (long long)k0 * cs.ps, cs.vs, cv);
  // the halo of plane r into buffer b, then the loads of plane r + 1
  // (clamped inside the tile; the last one is not used)
  auto stage = [&](int r, int b) {
    if (fixrows) {
#pragma unroll
      for (int h = 0; h < 4; ++h) fix3(hs[h].kind, hs[h].f, B, hv[h]);
    }
    if (fixcells && hlane) fix3(cs.kind, cs.f, B, cv);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      sm.q[b][0][v][lane + 2] = T(hv[0][v]);
      sm.q[b][1][v][lane + 2] = T(hv[1][v]);
      sm.q[b][ny + 2][v][lane + 2] = T(hv[2][v]);
      sm.q[b][ny + 3][v][lane + 2] = T(hv[3][v]);
    }
    if (hlane) {
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.q[b][crow][v][cslot] = T(cv[v]);
    }
    const long long kn = k0 + min(r + 1, n - 1);
#pragma unroll
    for (int h = 0; h < 4; ++h) load3(hs[h].p + kn * hs[h].ps, hs[h].vs, hv[h]);
    load3(cs.p + kn * cs.ps, cs.vs, cv);
  };
  stage(0, 0);
  __syncthreads();
  for (int r = 0; r < n; ++r) {
    const int b = r & 1;
    // top-edge j-face at j0+ny-1/2 from rows ny .. ny+3 (slots)
    {
      T qL[5], qR[5], G[5];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        face_states<LIM>(rc, sm.q[b][ny][v][lane + 2], sm.q[b][ny + 1][v][lane + 2],
                         sm.q[b][ny + 2][v][lane + 2], sm.q[b][ny + 3][v][lane + 2], qL[v], qR[v]);
      roe_flux<T, 3, 1>(qL, qR, nullptr, ay, K, G);
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.f[b][ny][v][lane] = G[v];
    }
    // right-edge i-face at i0+ncol-1/2 of every row (lane = row) from slots
    // ncol .. ncol+3
    {
      const int er = lane < ny ? lane : 0;
      T qL[5], qR[5], G[5];
#pragma unroll
      for (int v = 0; v < 5; ++v)
        face_states<LIM>(rc, sm.q[b][er + 2][v][nc], sm.q[b][er + 2][v][nc + 1], sm.q[b][er + 2][v][nc + 2],
                         sm.q[b][er + 2][v][nc + 3], qL[v], qR[v]);
      roe_flux<T, 3, 0>(qL, qR, nullptr, ax, K, G);
      if (lane < ny) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.edge[lane][v][r] = G[v];
      }
    }
    // as the row waves: lower priority once the plane's fluxes are formed
    __builtin_amdgcn_s_setprio(0);
    if (r + 1 < n) stage(r + 1, b ^ 1);
    __syncthreads();
    __builtin_amdgcn_s_setprio(2);
  }
}

template <int MODE, typename T, int NY, int LIM>
__device__ void tile3d(const DevTile& tl, const DevBlock* __restrict__ blocks, DevInstance& I,
                       double* __restrict__ rout, int lane, int w, Smem3<T, NY>& sm) {
  const DevBlock& B = blocks[tl.blk];
  const int ni = B.ni, nj = B.nj, nk = B.nk;
  const int i0 = tl.i0, j0 = tl.j0, k0 = tl.k0, n = tl.n, nc = tl.ncol, ny = tl.ny;
  const bool rowact = w < ny;
  const int jc = rowact ? j0 + w : j0;
  const bool act = lane < nc;
  const int ic = act ? i0 + lane : ni - 1;
  const int last = nc - 1;
  using SK = StageKind<MODE>;
  constexpr int bin = SK::bin;
  constexpr int bout = SK::bout;
  Recon<T> rc;
  FluxK<T> K;
  setup_consts(I, rc, K);
  const T ax = T(B.area[0]), ay = T(B.area[1]), az = T(B.area[2]);
  const double gamma = I.gamma;
  const double dt = stage_dt<MODE>(I);
  const double vol = B.vol;
  const double ivol = 1.0 / vol;
  const long long ncell = B.ncell;
  const long long pstr = (long long)ni * nj;
  const double* __restrict__ Q = B.u[bin];
  const double* __restrict__ Un = B.u[0];
  double* __restrict__ Uout = B.u[bout];
  // own column at row jc: element (k) at Q + k * pstr + jc * ni + ic
  const unsigned cb = (unsigned)(jc * ni + ic) * 8u;

  auto col_load = [&](const double* base, int k, double (&q)[5]) {
    const double* p = base + (long long)k * pstr;
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = ldo3(p + v * ncell, cb);
  };

  // ---- prologue: planes k0-2 .. k0+1 of the own column (the right-edge
  //      i-face of each plane comes from the helper wave)
  // the k-window: planes k-1, k, k+1 and the incoming k+2 live in the four
  // buffers qb0..qb3, the + side extrapolations of planes k-1 and k in eb0,
  // eb1; the buffers' roles rotate (below), the values stay in place
  double qa[5], qb0[5], qb1[5], qb2[5], qb3[5], un[5] = {0, 0, 0, 0, 0};
  const Src3 sa = src3_k(blocks, B, bin, ic, jc, k0 - 2);
  const Src3 sb = src3_k(blocks, B, bin, ic, jc, k0 - 1);
  const Src3 sd = src3_k(blocks, B, bin, ic, jc, k0 + 1);
  load3(sa.p, sa.vs, qa);
  load3(sb.p, sb.vs, qb0);
  col_load(Q, k0, qb1);
  load3(sd.p, sd.vs, qb2);
  fix3(sa.kind, sa.f, B, qa);
  fix3(sb.kind, sb.f, B, qb0);
  fix3(sd.kind, sd.f, B, qb2);
  T eb0[5], eb1[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    T em;
    extrap<LIM>(rc, T(qb0[v]) - T(qa[v]), T(qb1[v]) - T(qb0[v]), eb0[v], em);
    eb1[v] = T(0);
  }
  double rg[5] = {0, 0, 0, 0, 0};
  double nacc[5] = {0, 0, 0, 0, 0};
  double dmin = INFINITY;
  int bad = 0;
  const int qr = rowact ? w + 2 : 0;  // own row in the LDS planes
  // plane k0 into buffer 0 (the helper stages its halo alongside)
  if (rowact && act) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sm.q[0][qr][v][lane + 2] = T(qb1[v]);
  }
  __syncthreads();

  // one plane; qm1, q0, qn: planes k-1, k, k+1, q2 receives plane k+2;
  // epm1 / ep0: + side extrapolations of planes k-1 / k (ep0 is written).
  // ROT: end by moving the window down one buffer (qm1 <- q0 <- qn <- q2,
  // epm1 <- ep0); without it the caller passes the next plane's roles.
  auto step = [&](auto first_t, auto last_t, auto rot_t, int r, double (&qm1)[5], double (&q0)[5],
                  double (&qn)[5], double (&q2)[5], T (&epm1)[5], T (&ep0)[5]) {
    constexpr bool FIRST = decltype(first_t)::value;
    constexpr bool LASTP = decltype(last_t)::value;
    constexpr bool ROT = decltype(rot_t)::value;
    const int k = k0 + r;
    const int b = r & 1;
    T* const qrow = &sm.q[b][qr][0][0];
    // ---- (1) the plane k+2 of the own column
    Src3 s2;
    if constexpr (!LASTP) {
      if (k + 2 < nk) {
        col_load(Q, k + 2, q2);
        s2.kind = 0;
        s2.f = 0;
      } else {
        s2 = src3_k(blocks, B, bin, ic, jc, k + 2);
        load3(s2.p, s2.vs, q2);
      }
    }
    // ---- (2) plane k is in LDS buffer b (staged one plane ahead)
    T Gk[5] = {T(0), T(0), T(0), T(0), T(0)};
    T Gi[5];
    // ---- (3) k-face at k-1/2, and (in-plane) j-face at j-1/2 and i-face at
    //      i-1/2 from LDS: independent, their arithmetic interleaves
    if (rowact) {
      {
        T qL[5], qR[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T a = T(qm1[v]), b = T(q0[v]), c = T(qn[v]);
          T em;
          extrap<LIM>(rc, b - a, c - b, ep0[v], em);
          qL[v] = a + epm1[v];
          qR[v] = b - em;
        }
        roe_flux<T, 3, 2>(qL, qR, nullptr, az, K, Gk);
      }
      if constexpr (!LASTP) {
        T qL[5], qR[5], Gj[5];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          face_states<LIM>(rc, sm.q[b][w][v][lane + 2], sm.q[b][w + 1][v][lane + 2],
                           sm.q[b][w + 2][v][lane + 2], sm.q[b][w + 3][v][lane + 2], qL[v], qR[v]);
        roe_flux<T, 3, 1>(qL, qR, nullptr, ay, K, Gj);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.f[b][w][v][lane] = Gj[v];
#pragma unroll
        for (int v = 0; v < 5; ++v)
          face_states<LIM>(rc, qrow[v * kS3 + lane], qrow[v * kS3 + lane + 1], T(q0[v]),
                           qrow[v * kS3 + lane + 3], qL[v], qR[v]);
        roe_flux<T, 3, 0>(qL, qR, nullptr, ax, K, Gi);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.g[w][v][lane] = Gi[v];
      }
    }
    // ---- (3b) stage plane k + 1 (the next step's) in the other buffer
    if constexpr (!LASTP) {
      if (r + 1 < n && rowact && act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.q[b ^ 1][qr][v][lane + 2] = T(qn[v]);
      }
    }
    // this plane's fluxes are formed: the other wave of the SIMD goes first
    // until the barrier (both must reach it; the older one would run ahead)
    __builtin_amdgcn_s_setprio(0);
    // ---- (4) complete plane k-1
    if constexpr (!FIRST) {
      if (rowact && act) {
        double* const orow = Uout + (long long)(k - 1) * pstr;
        double R[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] = rg[v] + (double)Gk[v];
        if (MODE == 0) {
          double* const rrow = rout + B.out_off + (long long)(k - 1) * pstr;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            sto3(rrow + v * ncell, cb, R[v]);
            const double rv = R[v] * ivol;
            nacc[v] = fmad(rv, rv, nacc[v]);
          }
        } else {
          const double fct = dt * ivol;
          double out[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if constexpr (SK::low) {
              out[v] = fmad(-fct, R[v], un[v]);
            } else {
              const double us = fmad(-fct, R[v], qm1[v]);
              if (MODE == 1) out[v] = us;
              else if (MODE == 2) out[v] = fmad(0.75, un[v], 0.25 * us);
              else out[v] = fmad(1.0 / 3.0, un[v], (2.0 / 3.0) * us);
            }
            sto3(orow + v * ncell, cb, out[v]);
          }
          if (MODE == 1) {
#pragma unroll
            for (int v = 0; v < 5; ++v) {
              const double rv = R[v] * ivol;
              nacc[v] = fmad(rv, rv, nacc[v]);
            }
          }
          if constexpr (SK::cfl) {
            const double Sb[3][3] = {{B.area[0], 0.0, 0.0}, {0.0, B.area[1], 0.0},
                                     {0.0, 0.0, B.area[2]}};
            dmin = fmin(dmin, cell_dt_limit<3>(out, Sb, vol, gamma, bad));
          }
        }
      }
    }
    if constexpr (!LASTP) {
      // U^n of plane k for the next update
      if constexpr (SK::reads_un) col_load(Un, k, un);
      __syncthreads();
      __builtin_amdgcn_s_setprio(2);
      // ---- (5) the pending in-plane part of plane k
      if (rowact) {
        const T* gsrc = lane == last ? &sm.edge[w][0][r] : &sm.g[w][0][lane + 1];
        const int gstr = lane == last ? 64 : kS3;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          rg[v] = (((double)gsrc[v * gstr] - (double)Gi[v]) +
                   ((double)sm.f[b][w + 1][v][lane] - (double)sm.f[b][w][v][lane])) -
                  (double)Gk[v];
      }
      // the next step rewrites this wave's g row: its lanes' reads above
      // come first
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // ---- (6) ghost correction of the incoming plane; rotate
      if (k + 2 >= nk) fix3(s2.kind, s2.f, B, q2);
      if constexpr (ROT) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          qm1[v] = q0[v];
          q0[v] = qn[v];
          qn[v] = q2[v];
          epm1[v] = ep0[v];
        }
      }
    }
  };

  using F = std::integral_constant<bool, false>;
  using Tr = std::integral_constant<bool, true>;
  step(Tr(), F(), Tr(), 0, qb0, qb1, qb2, qb3, eb0, eb1);
  // four planes per pass with the roles renamed, so that the window needs no
  // register moves; after four planes the roles are back where they started.
  // The stage kinds with the time-step limit keep the moves: with the limit's
  // registers the renamed pass would spill.
  int r = 1;
  for (; !SK::cfl && r + 4 <= n; r += 4) {
    step(F(), F(), F(), r, qb0, qb1, qb2, qb3, eb0, eb1);
    step(F(), F(), F(), r + 1, qb1, qb2, qb3, qb0, eb1, eb0);
    step(F(), F(), F(), r + 2, qb2, qb3, qb0, qb1, eb0, eb1);
    step(F(), F(), F(), r + 3, qb3, qb0, qb1, qb2, eb1, eb0);
  }
  for (; r < n; ++r) step(F(), F(), Tr(), r, qb0, qb1, qb2, qb3, eb0, eb1);
  step(F(), Tr(), F(), n, qb0, qb1, qb2, qb3, eb0, eb1);

  // ---- per-tile partials of this row wave
  if (SK::norms || SK::cfl) {
    double s[5] = {0, 0, 0, 0, 0};
    double m = 0.0;
    int b = 0;
    if (SK::cfl) {
      m = wave_min(dmin);
      b = wave_or(bad);
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) s[v] = wave_sum(nacc[v]);
    }
    if (lane == 0) {
      if (SK::cfl) {
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
template <int MODE>
__device__ void tile_partials3d(const DevTile& tl, DevInstance& I, const double* red) {
  double* part = I.part + tl.local;
  const long long ps = I.ntiles;
  if (StageKind<MODE>::cfl) {
    double mm = INFINITY;
    double bb = 0.0;
    for (int x = 0; x < tl.ny; ++x) {
      mm = fmin(mm, red[x * 8 + 5]);
      bb = fmax(bb, red[x * 8 + 6]);
    }
    part[5 * ps] = mm;
    part[6 * ps] = bb;
  } else if (MODE == 0 || MODE == 1) {
    for (int v = 0; v < 5; ++v) {
      double a = 0.0;
      for (int x = 0; x < tl.ny; ++x) a += red[x * 8 + v];
      part[v * ps] = a;
    }
  }
}

template <int MODE, typename T, int NY, int LIM>
__device__ __forceinline__ void run_tile3d(const DevTile& tl, const DevBlock* __restrict__ blocks,
                                           DevInstance& I, double* __restrict__ rout, int lane, int w,
                                           Smem3<T, NY>& sm) {
  // the row waves and the helper wave take the same barriers
  if (w < NY) tile3d<MODE, T, NY, LIM>(tl, blocks, I, rout, lane, w, sm);
  else helper3d<MODE, T, NY, LIM>(tl, blocks, I, lane, sm);
}

// at most 256 VGPRs: two waves per SIMD
template <int MODE, typename T, int NY>
__global__ __launch_bounds__(64 * (NY + 1), 2) void k_stage3d(const DevTile* __restrict__ tiles,
                                                              const int* __restrict__ ntiles_p, int nfix,
                                                              int lim_fixed,
                                                              const DevBlock* __restrict__ blocks,
                                                              DevInstance* __restrict__ insts,
                                                              double* __restrict__ rout) {
  __shared__ Smem3<T, NY> sm;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // a count fixed at launch saves one dependent load before the first tile
  const int ntiles = nfix >= 0 ? nfix : *ntiles_p;
  // one tile per workgroup at a time, the XCD's workgroups on consecutive
  // tiles: the tiles that run together are j-neighbours of one k-slab, so
  // their halo rows are read once into the XCD's L2 and shared
  for (TileWalk tw = xcd_walk(ntiles, 1, 0); tw.t < tw.end; tw.t += tw.stride) {
    const DevTile tl = tiles[tw.t];
    DevInstance& I = insts[tl.inst];
    if (MODE != 0 && I.stopped) continue;
    // the limiter given at launch (grid path) needs no descriptor read
    const int lim = lim_fixed >= 0 ? lim_fixed : I.limiter;
    if (lim == LIM_MINMOD) run_tile3d<MODE, T, NY, LIM_MINMOD>(tl, blocks, I, rout, lane, w, sm);
    else run_tile3d<MODE, T, NY, -1>(tl, blocks, I, rout, lane, w, sm);
    __syncthreads();
    if (threadIdx.x == 0) tile_partials3d<MODE>(tl, I, sm.red);
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
          if (B.zn != nullptr) {  // curvilinear: the cell's own metrics
            double Sc[3][3], vol;
            cell_geom3(B, i, tl.j0 + y, tl.k0 + r, Sc, vol);
            dmin = fmin(dmin, cell_dt_limit<3>(q, Sc, vol, I.gamma, bad));
          } else {
            dmin = fmin(dmin, cell_dt_limit<3>(q, Sb, B.vol, I.gamma, bad));
          }
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
      double* part = I.part + tl.local;
      const long long ps = I.ntiles;
      part[5 * ps] = fmin(fmin(s_m[0], s_m[1]), fmin(s_m[2], s_m[3]));
      part[6 * ps] = (double)(s_b[0] | s_b[1] | s_b[2] | s_b[3]);
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_stage3d(int mode, int fp32, int ny, int grid, hipStream_t s, const DevTile* tiles,
                          const int* ntiles, int ntiles_fixed, int lim_fixed, const DevBlock* blocks,
                          DevInstance* insts, double* rout) {
  if (mode < 0 || mode > 6) return hipErrorInvalidValue;
#define FV_L3(M, T, N)                                                                          \
  hipLaunchKernelGGL((k_stage3d<M, T, N>), dim3(grid), dim3(64 * (N + 1)), 0, s, tiles, ntiles, \
                     ntiles_fixed, lim_fixed, blocks, insts, rout)
#define FV_L3N(M, T) \
  if (ny >= 7) FV_L3(M, T, 7); else FV_L3(M, T, 3)
#define FV_L3_ALL(T)               \
  switch (mode) {                  \
    case 0: FV_L3N(0, T); break;   \
    case 1: FV_L3N(1, T); break;   \
    case 2: FV_L3N(2, T); break;   \
    case 3: FV_L3N(3, T); break;   \
    case 4: FV_L3N(4, T); break;   \
    case 5: FV_L3N(5, T); break;   \
    default: FV_L3N(6, T); break;  \
  }
  if (fp32) {
    FV_L3_ALL(float)
  } else {
    FV_L3_ALL(double)
  }
#undef FV_L3_ALL
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
#define FV_P3(M, T) (ny >= 7 ? (const void*)&k_stage3d<M, T, 7> : (const void*)&k_stage3d<M, T, 3>)
  const int m = mode < 0 ? 0 : (mode > 6 ? 6 : mode);
  if (fp32) {
    switch (m) {
      case 0: return FV_P3(0, float);
      case 1: return FV_P3(1, float);
      case 2: return FV_P3(2, float);
      case 3: return FV_P3(3, float);
      case 4: return FV_P3(4, float);
      case 5: return FV_P3(5, float);
      default: return FV_P3(6, float);
    }
  }
  switch (m) {
    case 0: return FV_P3(0, double);
    case 1: return FV_P3(1, double);
    case 2: return FV_P3(2, double);
    case 3: return FV_P3(3, double);
    case 4: return FV_P3(4, double);
    case 5: return FV_P3(5, double);
    default: return FV_P3(6, double);
  }
#undef FV_P3
}

}  // namespace fvk
