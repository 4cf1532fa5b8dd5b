// Device-side data structures and per-face arithmetic of the finite-volume
// Euler hot path (gfx950).  Shared by the 2D and 3D stage kernels.
//
// Layout in HBM (one instance = one grid):
//   state buffers u[0] = U^n, u[1], u[2]: per block [var][k][j][i], i fastest,
//   interior cells only (ghost cells are never stored: every stencil read
//   outside a block is resolved on the fly from the boundary rule).
//   node coordinates of curvilinear blocks: x, y of (nj+1)(ni+1) nodes (2D);
//   x, y, z of (nk+1)(nj+1)(ni+1) nodes (3D), i fastest.
//   source S_h (grids created with one): per block [var][k][j][i].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvk {

constexpr int kWave = 64;
// per-tile partials: 5 norm sums, spectral minimum, flag (and a spare slot),
// stored value-major: value v of tile t at part[v * ntiles + t]
constexpr int kPartStride = 8;

enum { BC_PERIODIC = 0, BC_BLOCK = 1, BC_INFLOW = 2, BC_EXTRAP = 3, BC_SLIPWALL = 4, BC_NOSLIP = 5 };
enum { LIM_MINMOD = 0, LIM_NONE = 1, LIM_FIRST = 2 };
enum { FLAG_NONPHYS = 1, FLAG_CONVERGED = 2, FLAG_TEND = 4, FLAG_STEPLIMIT = 8 };

struct DevBlock {
  int ni, nj, nk, inst;
  long long ncell;          // ni*nj*nk: stride between variables
  double* u[3];             // U^n, stage buffer a, stage buffer b
  const double* xn;         // node coordinates or nullptr (uniform)
  const double* yn;
  const double* zn;         // 3D curvilinear blocks: z of the nodes (nullptr otherwise)
  const double* src;        // cell-averaged source S_h, [var][k][j][i], or nullptr
  double area[3];           // uniform: face area per direction
  double vol;               // uniform: cell volume
  double org[3];            // uniform: position of node (0, 0, 0)
  long long out_off;        // offset of this block in a residual output array
  int bc_kind[6];
  int bc_nbr[6];
  int bc_link[6];           // BLOCK: neighbour face | orientation << 3 (see link_cell)
  double bc_q[6][5];        // INFLOW: conserved ghost state; NOSLIP: wall velocity in [1..3]
};

struct DevInstance {
  // parameters (written by the host before a call)
  double cfl, dt_fixed, t_end, eps, kappa, efix, gamma;
  double qref[5];
  double drop_tol;
  long long step_limit;
  long long ncells;
  int limiter, ndim, nv, ntiles;
  int rk, rk_pad;
  double rk_c[4];           // stage coefficients (see StageKind)
  double mu, prandtl;       // viscosity (0: Euler) and Prandtl number
  double* part;             // [kPartStride][ntiles], value-major
  // marching state (device)
  double t, dt, dt_last, raw_min, norm_first, norm, drop;
  double norms[5];
  double rnorms[5];         // norms of the last residual-only evaluation
  long long steps;
  int flags, stopped, have_first, last_step;
};

// A tile: 64 consecutive cells along i (ncol of them active), in rows
// [j0, j0 + ny) (3D) and marching over n rows (2D: along j) or n planes
// (3D: along k).  `local` is the tile's index within its instance.
struct DevTile {
  int blk, inst, local, ncol;
  int i0, j0, k0, n;
  int ny;
  int curv;  // 2D: the block has node coordinates (curvilinear)
  int pad1, pad2;
};

// --------------------------------------------------------------------------
// Stage kinds of the stage kernels (template MODE):
//   0  residual only
//   SSP-RK3 in Shu-Osher form (Sec. 3.2; a reading):
//   1  U^n -> a:  a = U^n + c0 dt L(U^n)        (c0 = 1)
//   2  a -> b:    b = 3/4 U^n + 1/4 (a + dt L(a))
//   3  b -> U^n:  U^{n+1} = 1/3 U^n + 2/3 (b + dt L(b))
//   The 2- and 4-stage second-order schemes (Sec. 3.2, Eq. runge_kutta with
//   one nonzero a per row and b = e_s), stage k writing U^n + c_k dt L(input):
//   1  U^n -> a   (c0: 1/2 or 1/4)
//   4  a -> b     (c1 = 1/3)
//   5  b -> a     (c2 = 1/2)
//   6  a -> U^n   (c3 = 1, last)
// with L(U) = -R(U)/|Omega|.  Stage 1 also sums the residual norms of U^n;
// the last stage (3 or 6) forms the per-cell CFL limits of U^{n+1}.
// --------------------------------------------------------------------------
template <int MODE>
struct StageKind {
  static constexpr int bin = MODE <= 1 ? 0 : (MODE == 2 || MODE == 4 || MODE == 6 ? 1 : 2);
  static constexpr int bout = MODE == 1 || MODE == 5 ? 1 : (MODE == 2 || MODE == 4 ? 2 : 0);
  static constexpr bool reads_un = MODE >= 2;        // U^n read pointwise
  static constexpr bool norms = MODE <= 1;           // residual norms of U^n
  static constexpr bool cfl = MODE == 3 || MODE == 6;
  static constexpr bool low = MODE >= 4;             // U^n + c dt L(input)
  static constexpr int coef = MODE == 1 ? 0 : (MODE == 4 ? 1 : (MODE == 5 ? 2 : (MODE == 6 ? 3 : -1)));
};

// dt times the stage coefficient (exactly dt where the coefficient is 1)
template <int MODE>
__device__ __forceinline__ double stage_dt(const DevInstance& I) {
  constexpr int c = StageKind<MODE>::coef;
  if constexpr (c < 0) return I.dt;
  else return I.dt * I.rk_c[c];
}

// --------------------------------------------------------------------------
// memory access: the state and node arrays are global memory; their pointers
// come from descriptors, so the address space is stated explicitly to get
// global (not flat) loads and stores
// --------------------------------------------------------------------------
typedef __attribute__((address_space(1))) const double g_cdouble;
typedef __attribute__((address_space(1))) double g_double;
__device__ __forceinline__ double ldg(const double* p) { return *(g_cdouble*)p; }
__device__ __forceinline__ void stg(double* p, double v) { *(g_double*)p = v; }

// --------------------------------------------------------------------------
// arithmetic helpers
// --------------------------------------------------------------------------
// Reciprocal and square root from the hardware estimates (v_rcp, v_rsq)
// refined by Newton-Raphson (reciprocal) and Goldschmidt (square root and its
// reciprocal together) iterations.  In FP64 the result is within a few ulp of
// the correctly rounded value for the normal-range arguments met here; in FP32
// the hardware estimates are used directly.  The flux arithmetic below also
// runs on the host (the host-core worker of the CPU-GPU split): there these
// are the correctly rounded IEEE operations.
template <typename T>
struct M;
template <>
struct M<double> {
#if !defined(__HIP_DEVICE_COMPILE__)
  static __host__ inline double rcp(double x) { return 1.0 / x; }
  static __host__ inline void sqrt2(double x, double& s, double& h) {
    s = __builtin_sqrt(x);
    h = 0.5 / s;
  }
#else
  static __device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
  }
  // s = sqrt(x), h = 1 / (2 sqrt(x))
  static __device__ __forceinline__ void sqrt2(double x, double& s, double& h) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    s = __builtin_fma(d, h, g);
  }
#endif
};
template <>
struct M<float> {
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ void sqrt2(float x, float& s, float& h) {
    const float y = __builtin_amdgcn_rsqf(x);
    s = x * y;
    h = 0.5f * y;
  }
};

// wave-wide neighbour shifts (DPP): shr1 gives lane l the value of lane l-1,
// shl1 the value of lane l+1; the lane without a source keeps its own value
__device__ __forceinline__ int dpp_shr1(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shl1(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ double shr1(double x) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = dpp_shr1(v.x);
  v.y = dpp_shr1(v.y);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ double shl1(double x) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = dpp_shl1(v.x);
  v.y = dpp_shl1(v.y);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ float shr1(float x) {
  return __builtin_bit_cast(float, dpp_shr1(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float shl1(float x) {
  return __builtin_bit_cast(float, dpp_shl1(__builtin_bit_cast(int, x)));
}
// value of a given lane, as a wave-uniform value
__device__ __forceinline__ double lane_value(double x, int l) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_readlane(v.x, l);
  v.y = __builtin_amdgcn_readlane(v.y, l);
  return __builtin_bit_cast(double, v);
}
__device__ __forceinline__ float lane_value(float x, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
}

// a * b + c rounded once.  The library is compiled without automatic
// contraction, so every inlined copy of a formula rounds the same way (a face
// flux formed by two different tiles is bitwise the same); the fused forms
// are written out where they belong.
__host__ __device__ __forceinline__ double fmad(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__host__ __device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__host__ __device__ __forceinline__ T minmod(T a, T b) {
  const bool same = (a > T(0) && b > T(0)) || (a < T(0) && b < T(0));
  const T m = fabs(a) < fabs(b) ? a : b;
  return same ? m : T(0);
}

// MUSCL extrapolations of one cell from its two one-sided differences
// dm = Q_m - Q_{m-1}, dp = Q_{m+1} - Q_m (Sec. 5, Eq. (flux)):
//   ep: Q^L at the face m+1/2 is Q_m + ep
//   em: Q^R at the face m-1/2 is Q_m - em
// minmod: ep = em = eps/2 minmod(dm, dp) (the kappa terms coincide for a
// symmetric limiter); no limiter: ep = c1 dm + c2 dp, em = c2 dm + c1 dp
// with c1 = eps(1-kappa)/4, c2 = eps(1+kappa)/4; first order: 0.
template <typename T>
struct Recon {
  int lim;
  T heps, c1, c2;
};

// LIM >= 0 fixes the limiter at compile time; LIM < 0 reads it from R.lim
// eps/2 minmod(a, b) by sign injection: (copysign(eps/4, a) + copysign(eps/4, b))
// is eps/2, -eps/2 or 0 exactly, times min(|a|, |b|): the same value as the
// select form (bitwise, up to the sign of a zero result), with no compares
template <typename T>
__host__ __device__ __forceinline__ T half_eps_minmod(T qeps, T a, T b) {
  return (copysign(qeps, a) + copysign(qeps, b)) * fmin(fabs(a), fabs(b));
}
// In FP32 the hardware median of three does it in one instruction: the
// median of a, b and 0 is min(a, b) when both are positive, max(a, b) when
// both are negative and 0 otherwise, i.e. minmod(a, b); times eps/2 (2 qeps,
// exact) it rounds once, as the form above
template <>
__host__ __device__ __forceinline__ float half_eps_minmod(float qeps, float a, float b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (2.0f * qeps) * __builtin_amdgcn_fmed3f(a, b, 0.0f);
#else
  return (copysignf(qeps, a) + copysignf(qeps, b)) * fminf(fabsf(a), fabsf(b));
#endif
}

template <int LIM = -1, typename T>
__host__ __device__ __forceinline__ void extrap(const Recon<T>& R, T dm, T dp, T& ep, T& em) {
  if constexpr (LIM == LIM_MINMOD) {
    const T s = half_eps_minmod(T(0.5) * R.heps, dm, dp);
    ep = s;
    em = s;
    return;
  }
  if (R.lim == LIM_MINMOD) {
    const T s = R.heps * minmod(dm, dp);
    ep = s;
    em = s;
  } else if (R.lim == LIM_NONE) {
    ep = fmad(R.c1, dm, R.c2 * dp);
    em = fmad(R.c2, dm, R.c1 * dp);
  } else {
    ep = T(0);
    em = T(0);
  }
}

// constants of the flux
template <typename T>
struct FluxK {
  T gm1;    // gamma - 1
  T efix;   // Harten delta / c
  T iefix;  // 1 / efix (0 when the fix is off)
};

// Roe's numerical flux of the inviscid normal flux (Sec. 2 flux definition),
// arranged as
//   F = 1/2 [F(Q_L).n + F(Q_R).n] - 1/2 [ |V_n| dQ + d1 (1, u, H) + d2 (0, n, V_n) ]
// with Roe averages (u, H, c, rho~), lbar = (|V_n+c| + |V_n-c|)/2 - |V_n|,
// ld = (|V_n+c| - |V_n-c|)/2,
//   d1 = lbar dp / c^2 + ld rho~ dV_n / c,   d2 = lbar rho~ dV_n + ld dp / c,
// and Harten's fix on the two acoustic eigenvalues (delta = efix * c).
// Returns the flux times the face area.  ND = 2 or 3; AX >= 0: the unit
// normal is the coordinate axis AX (n unused), AX < 0: general unit normal n.
template <typename T, int ND, int AX>
__host__ __device__ __forceinline__ void roe_flux(const T* __restrict__ qL, const T* __restrict__ qR,
                                         const T* __restrict__ n, T area, const FluxK<T>& K,
                                         T* __restrict__ F) {
  constexpr int E = ND + 1;
  const T half = T(0.5);
  T sL, hL, sR, hR;
  M<T>::sqrt2(qL[0], sL, hL);
  M<T>::sqrt2(qR[0], sR, hR);
  const T irL = T(4) * hL * hL;  // 1 / rho
  const T irR = T(4) * hR * hR;
  T uL[ND], uR[ND];
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    uL[a] = qL[1 + a] * irL;
    uR[a] = qR[1 + a] * irR;
  }
  T keL = uL[0] * qL[1], keR = uR[0] * qR[1];
#pragma unroll
  for (int a = 1; a < ND; ++a) {
    keL = fmad(uL[a], qL[1 + a], keL);
    keR = fmad(uR[a], qR[1 + a], keR);
  }
  T VnL, VnR;
  if constexpr (AX >= 0) {
    VnL = uL[AX];
    VnR = uR[AX];
  } else {
    VnL = uL[0] * n[0];
    VnR = uR[0] * n[0];
#pragma unroll
    for (int a = 1; a < ND; ++a) {
      VnL = fmad(uL[a], n[a], VnL);
      VnR = fmad(uR[a], n[a], VnR);
    }
  }
  const T pL = K.gm1 * fmad(-half, keL, qL[E]);
  const T pR = K.gm1 * fmad(-half, keR, qR[E]);
  const T HL = (qL[E] + pL) * irL;
  const T HR = (qR[E] + pR) * irR;
  const T is = M<T>::rcp(sL + sR);
  const T wL = sL * is, wR = sR * is;
  T ut[ND];
#pragma unroll
  for (int a = 0; a < ND; ++a) ut[a] = fmad(wL, uL[a], wR * uR[a]);
  T q2 = ut[0] * ut[0];
#pragma unroll
  for (int a = 1; a < ND; ++a) q2 = fmad(ut[a], ut[a], q2);
  T Vn;
  if constexpr (AX >= 0) {
    Vn = ut[AX];
  } else {
    Vn = ut[0] * n[0];
#pragma unroll
    for (int a = 1; a < ND; ++a) Vn = fmad(ut[a], n[a], Vn);
  }
  const T Ht = fmad(wL, HL, wR * HR);
  const T rt = sL * sR;
  const T c2 = K.gm1 * fmad(-half, q2, Ht);
  T c, hc;
  M<T>::sqrt2(c2, c, hc);
  const T ic = T(2) * hc;
  const T dp = pR - pL;
  const T dVn = VnR - VnL;
  const T lc = fabs(Vn);
  T lm = fabs(Vn - c);
  T lp = fabs(Vn + c);
  const T del = K.efix * c;
  const T idel = K.iefix * ic;
  lm = lm < del ? half * fmad(lm * lm, idel, del) : lm;
  lp = lp < del ? half * fmad(lp * lp, idel, del) : lp;
  const T lbar = fmad(half, lp + lm, -lc);
  const T ld = half * (lp - lm);
  const T rdv = rt * dVn;
  const T dpc = dp * ic;
  const T d1 = fmad(lbar, dpc, ld * rdv) * ic;
  const T d2 = fmad(lbar, rdv, ld * dpc);
  const T ha = half * area;
  const T pLR = pL + pR;
  F[0] = ha * (fmad(qL[0], VnL, qR[0] * VnR) - fmad(lc, qR[0] - qL[0], d1));
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    T m = fmad(qL[1 + a], VnL, qR[1 + a] * VnR);
    T dd = fmad(lc, qR[1 + a] - qL[1 + a], d1 * ut[a]);
    if constexpr (AX >= 0) {
      if (a == AX) {
        m += pLR;
        dd += d2;
      }
    } else {
      m = fmad(pLR, n[a], m);
      dd = fmad(d2, n[a], dd);
    }
    F[1 + a] = ha * (m - dd);
  }
  F[E] = ha * (fmad(qL[E] + pL, VnL, (qR[E] + pR) * VnR) -
               fmad(lc, qR[E] - qL[E], fmad(d1, Ht, d2 * Vn)));
}

// --------------------------------------------------------------------------
// node coordinates (2D curvilinear)
// --------------------------------------------------------------------------
__device__ __forceinline__ double nodex(const DevBlock& B, int i, int j) {
  return ldg(B.xn + (long long)j * (B.ni + 1) + i);
}
__device__ __forceinline__ double nodey(const DevBlock& B, int i, int j) {
  return ldg(B.yn + (long long)j * (B.ni + 1) + i);
}

// --------------------------------------------------------------------------
// 3D curvilinear geometry.  The face (d, i, j, k) of a cell has the corners
// p0 = node (i, j, k), p1 = p0 + e_t1, p2 = p0 + e_t1 + e_t2, p3 = p0 + e_t2
// with (t1, t2) = (j, k), (i, k), (i, j) for d = 0, 1, 2.  Its area vector,
// oriented towards increasing index d, is half the cross product of the
// diagonals p2 - p0 and p3 - p1 (the opposite sign for d = 1, where that
// order winds the other way); its centre is the mean of the corners.
// The volume of a cell is 1/3 of the sum over its faces of the outward area
// vector dotted with the face centre (the divergence theorem for x).
// --------------------------------------------------------------------------
__device__ __forceinline__ void node3(const DevBlock& B, int i, int j, int k, double* p) {
  const long long n = ((long long)k * (B.nj + 1) + j) * (B.ni + 1) + i;
  p[0] = ldg(B.xn + n);
  p[1] = ldg(B.yn + n);
  p[2] = ldg(B.zn + n);
}

// area vector S and S . centre of a face from its corners p0..p3 (above)
__device__ __forceinline__ void quad_face(const double* p0, const double* p1, const double* p2,
                                          const double* p3, bool flip, double* S, double& cs) {
  double a[3], b[3], c[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    a[x] = p2[x] - p0[x];
    b[x] = flip ? p1[x] - p3[x] : p3[x] - p1[x];
    c[x] = 0.25 * (((p0[x] + p1[x]) + p2[x]) + p3[x]);
  }
  S[0] = 0.5 * (a[1] * b[2] - a[2] * b[1]);
  S[1] = 0.5 * (a[2] * b[0] - a[0] * b[2]);
  S[2] = 0.5 * (a[0] * b[1] - a[1] * b[0]);
  cs = (c[0] * S[0] + c[1] * S[1]) + c[2] * S[2];
}

// face (d, i, j, k) of a 3D curvilinear block, corners read from memory
__device__ __forceinline__ void face3(const DevBlock& B, int d, int i, int j, int k, double* S,
                                      double& cs) {
  double p[4][3];
  const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;  // transverse axes
  int o[4][3] = {{i, j, k}, {i, j, k}, {i, j, k}, {i, j, k}};
  o[1][a1] += 1;
  o[2][a1] += 1;
  o[2][a2] += 1;
  o[3][a2] += 1;
#pragma unroll
  for (int m = 0; m < 4; ++m) node3(B, o[m][0], o[m][1], o[m][2], p[m]);
  quad_face(p[0], p[1], p[2], p[3], d == 1, S, cs);
}

// mean area vectors Sb[d] = (S_d- + S_d+)/2 and the volume of cell (i, j, k)
__device__ inline void cell_geom3(const DevBlock& B, int i, int j, int k, double (*Sb)[3],
                                  double& vol) {
  double v = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double Sm[3], Sp[3], cm, cp;
    face3(B, d, i, j, k, Sm, cm);
    face3(B, d, i + (d == 0), j + (d == 1), k + (d == 2), Sp, cp);
#pragma unroll
    for (int x = 0; x < 3; ++x) Sb[d][x] = 0.5 * (Sm[x] + Sp[x]);
    v += cp - cm;
  }
  vol = v / 3.0;
}

// --------------------------------------------------------------------------
// ghost resolution: value of cell (i, j, k) of block B in state buffer buf,
// where at most one index lies outside the block, by at most 2 cells.  The
// boundary rule gives a source cell (same block, a neighbour block, or the
// inflow state) and, for slip walls, the wall face's area vector about whose
// normal the momentum is mirrored: m - 2 (m.S)/(S.S) S.
// --------------------------------------------------------------------------
// no-slip wall ghost of a copied interior state: velocity 2 w - u with rho
// and p kept, in conserved form m' = 2 rho w - m, rho e_t' = rho e_t +
// (|m'|^2 - |m|^2) / (2 rho) (a wall at rest: m' = -m, rho e_t unchanged)
template <int ND>
__host__ __device__ __forceinline__ void noslip_mirror(double* q, const double* w) {
  double m2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    const double m = q[1 + a];
    const double mp = 2.0 * q[0] * w[1 + a] - m;
    m2 = fmad(m, m, m2);
    n2 = fmad(mp, mp, n2);
    q[1 + a] = mp;
  }
  q[ND + 1] += 0.5 * (n2 - m2) / q[0];
}

// Cell (si, sj, sk) of block S that ghost layer g (1 or 2) copies through a
// block link (the multi-block grids of Sec. 2) whose far side is face nf = link & 7
// of S with orientation o = link >> 3.  (t1, t2) are the ghost's transverse
// indices on its own face, in the order (j, k), (i, k), (i, j) for faces
// normal to i, j, k.  Bit 0 of o swaps them; bits 1 and 2 then reverse the
// first and the second along S's face.  The copied cell lies g - 1 cells
// inside face nf.
__device__ __forceinline__ void link_cell(const DevBlock& S, int link, int g, int t1, int t2,
                                          int& si, int& sj, int& sk) {
  const int nf = link & 7, o = link >> 3, sd = nf >> 1;
  const int m1 = sd == 0 ? S.nj : S.ni;
  const int m2 = sd == 2 ? S.nj : S.nk;
  int s1 = (o & 1) ? t2 : t1;
  int s2 = (o & 1) ? t1 : t2;
  if (o & 2) s1 = m1 - 1 - s1;
  if (o & 4) s2 = m2 - 1 - s2;
  const int n = sd == 0 ? S.ni : (sd == 1 ? S.nj : S.nk);
  const int along = (nf & 1) == 0 ? g - 1 : n - g;
  si = sd == 0 ? along : s1;
  sj = sd == 1 ? along : (sd == 0 ? s1 : s2);
  sk = sd == 2 ? along : s2;
}

template <int NV>
__device__ __forceinline__ void load_cell(const DevBlock* __restrict__ blocks, const DevBlock& B,
                                          int buf, int i, int j, int k, double* q) {
  constexpr int ND = NV - 2;
  if (i >= 0 && i < B.ni && j >= 0 && j < B.nj && k >= 0 && k < B.nk) {
    const double* s = B.u[buf] + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = ldg(s + v * B.ncell);
    return;
  }
  int f, g;
  if (i < 0) { f = 0; g = -i; }
  else if (i >= B.ni) { f = 1; g = i - B.ni + 1; }
  else if (j < 0) { f = 2; g = -j; }
  else if (j >= B.nj) { f = 3; g = j - B.nj + 1; }
  else if (k < 0) { f = 4; g = -k; }
  else { f = 5; g = k - B.nk + 1; }
  const int d = f >> 1, side = f & 1;
  const int kind = B.bc_kind[f];
  if (kind == BC_INFLOW) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = B.bc_q[f][v];
    return;
  }
  const DevBlock* S = &B;
  const int n = d == 0 ? B.ni : (d == 1 ? B.nj : B.nk);
  int si = i, sj = j, sk = k;
  if (kind == BC_BLOCK) {
    S = &blocks[B.bc_nbr[f]];
    link_cell(*S, B.bc_link[f], g, d == 0 ? j : i, d == 2 ? j : k, si, sj, sk);
  } else {
    int along;
    if (kind == BC_PERIODIC) along = side == 0 ? n - g : g - 1;
    else if (kind == BC_EXTRAP) along = side == 0 ? 0 : n - 1;
    else along = side == 0 ? g - 1 : n - g;  // SLIPWALL, NOSLIP
    if (d == 0) si = along;
    else if (d == 1) sj = along;
    else sk = along;
  }
  const double* s = S->u[buf] + ((long long)sk * S->nj + sj) * S->ni + si;
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = ldg(s + v * S->ncell);
  if (kind == BC_SLIPWALL) {
    double Sv[3] = {0.0, 0.0, 0.0};
    if (B.zn != nullptr) {
      // the wall face at the ghost's transverse position
      const int w = side == 0 ? 0 : n;
      double cs;
      face3(B, d, d == 0 ? w : i, d == 1 ? w : j, d == 2 ? w : k, Sv, cs);
    } else if (B.xn != nullptr) {
      const double* X = B.xn;
      const double* Y = B.yn;
      const long long w1 = B.ni + 1;
      if (d == 0) {
        const int w = side == 0 ? 0 : B.ni;
        Sv[0] = ldg(Y + (long long)(j + 1) * w1 + w) - ldg(Y + (long long)j * w1 + w);
        Sv[1] = -(ldg(X + (long long)(j + 1) * w1 + w) - ldg(X + (long long)j * w1 + w));
      } else {
        const int w = side == 0 ? 0 : B.nj;
        Sv[0] = -(ldg(Y + (long long)w * w1 + i + 1) - ldg(Y + (long long)w * w1 + i));
        Sv[1] = ldg(X + (long long)w * w1 + i + 1) - ldg(X + (long long)w * w1 + i);
      }
    } else {
      Sv[d] = 1.0;
    }
    double ms = 0.0, ss = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      ms += q[1 + a] * Sv[a];
      ss += Sv[a] * Sv[a];
    }
    const double fct = 2.0 * ms / ss;
#pragma unroll
    for (int a = 0; a < ND; ++a) q[1 + a] -= fct * Sv[a];
  } else if (kind == BC_NOSLIP) {
    noslip_mirror<ND>(q, B.bc_q[f]);
  }
}

// kept for the ghost dump (out of the hot path)
template <int NV>
__device__ void resolve_cell(const DevBlock* __restrict__ blocks, const DevBlock& B, int buf, int i,
                             int j, int k, double* q) {
  load_cell<NV>(blocks, B, buf, i, j, k, q);
}

// --------------------------------------------------------------------------
// XCD-aware assignment of tiles to persistent workgroups.  Workgroups are
// dealt to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8).  Each
// XCD walks one contiguous eighth of the tile list, so tiles that are
// neighbours in the grid (and read each other's halo rows) are processed by
// one XCD at about the same time, through its L2.  Every tile is taken by
// exactly one (workgroup, slot); the order does not change any result.
// --------------------------------------------------------------------------
constexpr int kXcds = 8;

struct TileWalk {
  int t, end, stride;
};

__device__ __forceinline__ TileWalk xcd_walk(int ntiles, int slots_per_wg, int slot) {
  const int G = gridDim.x;
  TileWalk w;
  if (G % kXcds != 0) {  // plain grid-stride order
    w.t = blockIdx.x * slots_per_wg + slot;
    w.end = ntiles;
    w.stride = G * slots_per_wg;
    return w;
  }
  const int x = blockIdx.x % kXcds, k = blockIdx.x / kXcds;
  const int chunk = (ntiles + kXcds - 1) / kXcds;
  const int beg = x * chunk;
  w.t = beg + k * slots_per_wg + slot;
  w.end = min(ntiles, beg + chunk);
  w.stride = (G / kXcds) * slots_per_wg;
  return w;
}

// Issue priority of a wavefront from its progress through a 2D tile.  Two
// tiles share each SIMD; with equal priorities the older wavefront is issued
// first, runs ahead, and the younger one ends its tile alone with nothing to
// hide its latencies.  A wavefront that has finished more rows steps down, so
// the one behind is preferred and the two end their tiles together.  Only
// the order of issue changes, never a result.
__device__ __forceinline__ void prio_by_progress(int rows_done) {
  if (rows_done <= 0) __builtin_amdgcn_s_setprio(3);
  else if (rows_done == 1) __builtin_amdgcn_s_setprio(2);
  else if (rows_done == 2) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// --------------------------------------------------------------------------
// wave-wide deterministic reductions (fixed butterfly order)
// --------------------------------------------------------------------------
// DPP lane permutations of a double (both halves moved alike): quad_perm,
// row_half_mirror and row_mirror keep every lane's source inside its row
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int2 v = __builtin_bit_cast(int2, x);
  v.x = __builtin_amdgcn_update_dpp(v.x, v.x, CTRL, 0xf, 0xf, false);
  v.y = __builtin_amdgcn_update_dpp(v.y, v.y, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, v);
}
// sum over the wave in a fixed order: within each row of 16 lanes by four
// DPP exchange steps (every lane of a row ends with the row sum, combined in
// the same pattern on every lane), then the four row sums in row order
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  const double r0 = lane_value(v, 0), r1 = lane_value(v, 16);
  const double r2 = lane_value(v, 32), r3 = lane_value(v, 48);
  return ((r0 + r1) + r2) + r3;
}
__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, dpp_d<0xB1>(v));
  v = fmin(v, dpp_d<0x4E>(v));
  v = fmin(v, dpp_d<0x141>(v));
  v = fmin(v, dpp_d<0x140>(v));
  return fmin(fmin(lane_value(v, 0), lane_value(v, 16)), fmin(lane_value(v, 32), lane_value(v, 48)));
}
__device__ __forceinline__ int wave_or(int v) {
  v |= __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false);
  v |= __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false);
  v |= __builtin_amdgcn_update_dpp(v, v, 0x141, 0xf, 0xf, false);
  v |= __builtin_amdgcn_update_dpp(v, v, 0x140, 0xf, 0xf, false);
  return __builtin_amdgcn_readlane(v, 0) | __builtin_amdgcn_readlane(v, 16) |
         __builtin_amdgcn_readlane(v, 32) | __builtin_amdgcn_readlane(v, 48);
}

// local time-step limit |Omega| / sum_d(|u.Sbar_d| + c|Sbar_d|) of a cell and
// the physical check (rho > 0, p > 0, finite)
template <int ND>
__host__ __device__ __forceinline__ double cell_dt_limit(const double* q, const double (*Sb)[3], double vol,
                                                double gamma, int& bad) {
  constexpr int E = ND + 1;
  bool ok = true;
#pragma unroll
  for (int v = 0; v < ND + 2; ++v) ok = ok && __builtin_isfinite(q[v]);
  const double rho = q[0];
  const double ir = 1.0 / rho;
  double u[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < ND; ++a) u[a] = q[1 + a] * ir;
  double ke = u[0] * q[1];
#pragma unroll
  for (int a = 1; a < ND; ++a) ke = fmad(u[a], q[1 + a], ke);
  const double p = (gamma - 1.0) * fmad(-0.5, ke, q[E]);
  ok = ok && rho > 0.0 && p > 0.0;
  if (!ok) {
    bad = 1;
    return INFINITY;
  }
  const double c = sqrt(gamma * p * ir);
  double lam = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double us = u[0] * Sb[d][0], ss = Sb[d][0] * Sb[d][0];
#pragma unroll
    for (int a = 1; a < ND; ++a) {
      us = fmad(u[a], Sb[d][a], us);
      ss = fmad(Sb[d][a], Sb[d][a], ss);
    }
    lam += fmad(c, sqrt(ss), fabs(us));
  }
  return vol / lam;
}

// Viscous flux F_nu . S (Sec. 2) of a face from u, v, p/rho at its cells L,
// R (centres dx, dy apart) and its nodes A, B (B - A turned by -90 degrees
// is S): Green-Gauss gradients over the face's diamond, Stokes stresses
// with constant mu, heat flux kq grad(p/rho).  Differences in FP64, the
// rest in T.
template <typename T>
__host__ __device__ __forceinline__ void visc_flux(const double* wL, const double* wR,
                                                   const double* wA, const double* wB, double dx,
                                                   double dy, double Sx, double Sy, T mu, T kq,
                                                   T* F) {
  const T tSx = T(Sx), tSy = T(Sy), tdx = T(dx), tdy = T(dy);
  const T iD = M<T>::rcp(fmad(tdx, tSx, tdy * tSy));
  T gx[3], gy[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T a = T(wR[k] - wL[k]), t = T(wB[k] - wA[k]);
    gx[k] = fmad(a, tSx, -(t * tdy)) * iD;
    gy[k] = fmad(a, tSy, t * tdx) * iD;
  }
  const T dv = gx[0] + gy[1];
  const T c23 = T(2.0 / 3.0);
  const T txx = mu * fmad(T(2), gx[0], -(c23 * dv));
  const T tyy = mu * fmad(T(2), gy[1], -(c23 * dv));
  const T txy = mu * (gy[0] + gx[1]);
  const T uf = T(0.5 * (wL[0] + wR[0])), vf = T(0.5 * (wL[1] + wR[1]));
  const T thx = fmad(uf, txx, fmad(vf, txy, kq * gx[2]));
  const T thy = fmad(uf, txy, fmad(vf, tyy, kq * gy[2]));
  F[0] = T(0);
  F[1] = fmad(txx, tSx, txy * tSy);
  F[2] = fmad(txy, tSx, tyy * tSy);
  F[3] = fmad(thx, tSx, thy * tSy);
}

// the same limit with the viscous term of a Navier-Stokes step:
// |Omega| / (sum_d(|u.Sbar_d| + c|Sbar_d|) + 2 max(4/3, gamma/Pr) (mu/rho)
// sum_d |Sbar_d|^2 / |Omega|)
__host__ __device__ __forceinline__ double cell_dt_limit_visc(const double* q, const double (*Sb)[3],
                                                              double vol, double gamma, double mu,
                                                              double prandtl, int& bad) {
  const double rho = q[0];
  double ir = 1.0 / rho, u = q[1] * ir, v = q[2] * ir;
  const double p = (gamma - 1.0) * fmad(-0.5, fmad(u, q[1], v * q[2]), q[3]);
  const bool ok = __builtin_isfinite(q[0]) && __builtin_isfinite(q[1]) &&
                  __builtin_isfinite(q[2]) && __builtin_isfinite(q[3]) && rho > 0.0 && p > 0.0;
  if (!ok) {
    bad = 1;
    return INFINITY;
  }
  const double c = sqrt(gamma * p * ir);
  double lam = 0.0, ss = 0.0;
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const double us = fmad(u, Sb[d][0], v * Sb[d][1]);
    const double s2 = fmad(Sb[d][0], Sb[d][0], Sb[d][1] * Sb[d][1]);
    lam += fmad(c, sqrt(s2), fabs(us));
    ss += s2;
  }
  const double f = fmax(4.0 / 3.0, gamma / prandtl);
  lam += 2.0 * f * (mu * ir) * ss / vol;
  return vol / lam;
}

}  // namespace fvk
