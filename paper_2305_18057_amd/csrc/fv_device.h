// Device-side data structures and per-face arithmetic of the finite-volume
// Euler hot path (gfx950).  Shared by the 2D and 3D stage kernels.
//
// Layout in HBM (one instance = one grid):
//   state buffers u[0] = U^n, u[1], u[2]: per block [var][k][j][i], i fastest,
//   interior cells only (ghost cells are never stored: every stencil read
//   outside a block is resolved on the fly from the boundary rule).
//   2D curvilinear node coordinates x, y: (nj+1)(ni+1) per block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvk {

constexpr int kWave = 64;
constexpr int kPartStride = 8;  // per-tile partials: 5 norm sums, spectral min, flag, spare

enum { BC_PERIODIC = 0, BC_BLOCK = 1, BC_INFLOW = 2, BC_EXTRAP = 3, BC_SLIPWALL = 4 };
enum { LIM_MINMOD = 0, LIM_NONE = 1, LIM_FIRST = 2 };
enum { FLAG_NONPHYS = 1, FLAG_CONVERGED = 2, FLAG_TEND = 4, FLAG_STEPLIMIT = 8 };

struct DevBlock {
  int ni, nj, nk, inst;
  long long ncell;          // ni*nj*nk: stride between variables
  double* u[3];             // U^n, stage buffer a, stage buffer b
  const double* xn;         // 2D node coordinates or nullptr (uniform)
  const double* yn;
  double area[3];           // uniform: face area per direction
  double vol;               // uniform: cell volume
  long long out_off;        // offset of this block in a residual output array
  int bc_kind[6];
  int bc_nbr[6];
  double bc_q[6][5];        // INFLOW: conserved ghost state
};

struct DevInstance {
  // parameters (written by the host before a call)
  double cfl, dt_fixed, t_end, eps, kappa, efix, gamma;
  double qref[5];
  double drop_tol;
  long long step_limit;
  long long ncells;
  int limiter, ndim, nv, ntiles;
  double* part;             // [ntiles][kPartStride]
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
  int ny, pad0, pad1, pad2;
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
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

template <typename T>
__device__ __forceinline__ void extrap(const Recon<T>& R, T dm, T dp, T& ep, T& em) {
  if (R.lim == LIM_MINMOD) {
    const T s = R.heps * minmod(dm, dp);
    ep = s;
    em = s;
  } else if (R.lim == LIM_NONE) {
    ep = R.c1 * dm + R.c2 * dp;
    em = R.c2 * dm + R.c1 * dp;
  } else {
    ep = T(0);
    em = T(0);
  }
}

// Roe's numerical flux of the inviscid normal flux (Sec. 2 flux definition),
// arranged as
//   F = 1/2 [F(Q_L).n + F(Q_R).n] - 1/2 [ |V_n| dQ + d1 (1, u, H) + d2 (0, n, V_n) ]
// with Roe averages (u, H, c, rho~), lbar = (|V_n+c| + |V_n-c|)/2 - |V_n|,
// ld = (|V_n+c| - |V_n-c|)/2,
//   d1 = lbar dp / c^2 + ld rho~ dV_n / c,   d2 = lbar rho~ dV_n + ld dp / c,
// and Harten's fix on the two acoustic eigenvalues (delta = efix * c).
// Returns the flux times the face area.  ND = 2 or 3, NV = ND + 2.
template <typename T, int ND>
__device__ __forceinline__ void roe_flux(const T* __restrict__ qL, const T* __restrict__ qR,
                                         const T* __restrict__ n, T area, T gm1, T efix,
                                         T* __restrict__ F) {
  constexpr int E = ND + 1;
  const T half = T(0.5);
  const T irL = T(1) / qL[0];
  const T irR = T(1) / qR[0];
  T uL[ND], uR[ND];
  T keL = T(0), keR = T(0), VnL = T(0), VnR = T(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    uL[a] = qL[1 + a] * irL;
    uR[a] = qR[1 + a] * irR;
    keL += uL[a] * qL[1 + a];
    keR += uR[a] * qR[1 + a];
    VnL += uL[a] * n[a];
    VnR += uR[a] * n[a];
  }
  const T pL = gm1 * (qL[E] - half * keL);
  const T pR = gm1 * (qR[E] - half * keR);
  const T HL = (qL[E] + pL) * irL;
  const T HR = (qR[E] + pR) * irR;
  const T sL = sqrt(qL[0]);
  const T sR = sqrt(qR[0]);
  const T is = T(1) / (sL + sR);
  const T wL = sL * is, wR = sR * is;
  T ut[ND];
  T q2 = T(0), Vn = T(0);
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    ut[a] = wL * uL[a] + wR * uR[a];
    q2 += ut[a] * ut[a];
    Vn += ut[a] * n[a];
  }
  const T Ht = wL * HL + wR * HR;
  const T rt = sL * sR;
  const T c2 = gm1 * (Ht - half * q2);
  const T c = sqrt(c2);
  const T ic = T(1) / c;
  const T dp = pR - pL;
  const T dVn = VnR - VnL;
  const T lc = fabs(Vn);
  T lm = fabs(Vn - c);
  T lp = fabs(Vn + c);
  const T del = efix * c;
  if (del > T(0)) {
    const T idel = T(1) / del;
    lm = lm < del ? half * (lm * lm * idel + del) : lm;
    lp = lp < del ? half * (lp * lp * idel + del) : lp;
  }
  const T lbar = half * (lp + lm) - lc;
  const T ld = half * (lp - lm);
  const T rdv = rt * dVn;
  const T d1 = (lbar * dp * ic + ld * rdv) * ic;
  const T d2 = lbar * rdv + ld * dp * ic;
  const T ha = half * area;
  F[0] = ha * ((qL[0] * VnL + qR[0] * VnR) - (lc * (qR[0] - qL[0]) + d1));
#pragma unroll
  for (int a = 0; a < ND; ++a)
    F[1 + a] = ha * ((qL[1 + a] * VnL + qR[1 + a] * VnR + (pL + pR) * n[a]) -
                     (lc * (qR[1 + a] - qL[1 + a]) + d1 * ut[a] + d2 * n[a]));
  F[E] = ha * (((qL[E] + pL) * VnL + (qR[E] + pR) * VnR) -
               (lc * (qR[E] - qL[E]) + d1 * Ht + d2 * Vn));
}

// --------------------------------------------------------------------------
// node coordinates (2D curvilinear)
// --------------------------------------------------------------------------
__device__ __forceinline__ double nodex(const DevBlock& B, int i, int j) {
  return B.xn[(long long)j * (B.ni + 1) + i];
}
__device__ __forceinline__ double nodey(const DevBlock& B, int i, int j) {
  return B.yn[(long long)j * (B.ni + 1) + i];
}

// --------------------------------------------------------------------------
// ghost resolution: value of cell (i, j, k) of block B in state buffer buf,
// where at most one index lies outside the block, by at most 2 cells.
// --------------------------------------------------------------------------
template <int NV>
__device__ __noinline__ void resolve_cell(const DevBlock* __restrict__ blocks, const DevBlock& B,
                                          int buf, int i, int j, int k, double* q) {
  constexpr int ND = NV - 2;
  int f, g;
  if (i < 0) { f = 0; g = -i; }
  else if (i >= B.ni) { f = 1; g = i - B.ni + 1; }
  else if (j < 0) { f = 2; g = -j; }
  else if (j >= B.nj) { f = 3; g = j - B.nj + 1; }
  else if (k < 0) { f = 4; g = -k; }
  else if (k >= B.nk) { f = 5; g = k - B.nk + 1; }
  else {
    const double* s = B.u[buf] + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = s[v * B.ncell];
    return;
  }
  const int d = f >> 1, side = f & 1;
  const int kind = B.bc_kind[f];
  if (kind == BC_INFLOW) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = B.bc_q[f][v];
    return;
  }
  const DevBlock* S = &B;
  if (kind == BC_BLOCK) S = &blocks[B.bc_nbr[f]];
  const int n = d == 0 ? S->ni : (d == 1 ? S->nj : S->nk);
  int along;
  if (kind == BC_PERIODIC || kind == BC_BLOCK) along = side == 0 ? n - g : g - 1;
  else if (kind == BC_EXTRAP) along = side == 0 ? 0 : n - 1;
  else along = side == 0 ? g - 1 : n - g;  // SLIPWALL
  int si = i, sj = j, sk = k;
  if (d == 0) si = along;
  else if (d == 1) sj = along;
  else sk = along;
  const double* s = S->u[buf] + ((long long)sk * S->nj + sj) * S->ni + si;
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = s[v * S->ncell];
  if (kind == BC_SLIPWALL) {
    // mirror the momentum about the wall face's normal: m - 2 (m.S)/(S.S) S
    double Sv[3] = {0.0, 0.0, 0.0};
    if (B.xn != nullptr) {
      if (d == 0) {
        const int w = side == 0 ? 0 : B.ni;
        Sv[0] = nodey(B, w, j + 1) - nodey(B, w, j);
        Sv[1] = -(nodex(B, w, j + 1) - nodex(B, w, j));
      } else {
        const int w = side == 0 ? 0 : B.nj;
        Sv[0] = -(nodey(B, i + 1, w) - nodey(B, i, w));
        Sv[1] = nodex(B, i + 1, w) - nodex(B, i, w);
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
  }
}

// --------------------------------------------------------------------------
// wave-wide deterministic reductions (fixed butterfly order)
// --------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

// local time-step limit |Omega| / sum_d(|u.Sbar_d| + c|Sbar_d|) of a cell and
// the physical check (rho > 0, p > 0, finite)
template <int ND>
__device__ __forceinline__ double cell_dt_limit(const double* q, const double (*Sb)[3], double vol,
                                                double gamma, int& bad) {
  constexpr int E = ND + 1;
  bool ok = true;
#pragma unroll
  for (int v = 0; v < ND + 2; ++v) ok = ok && isfinite(q[v]);
  const double rho = q[0];
  const double ir = 1.0 / rho;
  double u[3] = {0.0, 0.0, 0.0};
  double ke = 0.0;
#pragma unroll
  for (int a = 0; a < ND; ++a) {
    u[a] = q[1 + a] * ir;
    ke += u[a] * q[1 + a];
  }
  const double p = (gamma - 1.0) * (q[E] - 0.5 * ke);
  ok = ok && rho > 0.0 && p > 0.0;
  if (!ok) {
    bad = 1;
    return INFINITY;
  }
  const double c = sqrt(gamma * p * ir);
  double lam = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double us = 0.0, ss = 0.0;
#pragma unroll
    for (int a = 0; a < ND; ++a) {
      us += u[a] * Sb[d][a];
      ss += Sb[d][a] * Sb[d][a];
    }
    lam += fabs(us) + c * sqrt(ss);
  }
  return vol / lam;
}

}  // namespace fvk
