/*
 * Plain FP64 CPU reference of the explicit finite-volume Euler residual and
 * the explicit RK time update (SSP-RK3, and the paper's 2- and 4-stage
 * second-order schemes) on structured multi-block grids.
 *
 * TEST INFRASTRUCTURE ONLY.  The test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does.  It
 * shares no code with the HIP library.  It is written to be read against the
 * paper, not to be fast: every face flux is formed once from ghost-padded
 * arrays, every cell residual is summed from stored face fluxes, and the
 * stages run one after another over whole arrays.  OpenMP splits the loops
 * over independent faces or cells only; every sum over cells runs serially in
 * natural order (block, k, j, i).
 *
 * Where it follows the paper:
 *   Q and the inviscid normal flux F_{i,n} ........ Sec. 2 (conserved vector, flux definitions)
 *   semi-discrete form |Omega| dU/dt + R = 0 ....... Sec. 3.1, Eq. (spatial_residual)
 *   R = sum over the f faces of (F_{i,n} - F_{nu,n}) ds - |Omega| S_h   Sec. 3.1, Eq. (residual);
 *   F_{nu,n} with Stokes stresses tau and Theta ... Sec. 2 (viscous flux; 2D)
 *   explicit RK in Butcher form ..................... Sec. 3.2, Eq. (runge_kutta)
 *   MUSCL face states with limiter values Psi ...... Sec. 5, Eq. (flux)
 *   ghost cells refreshed before every RK substep .. Sec. 4 (workflow) and Sec. 5 (ghost extrapolation)
 *   cell-update counting (ssspnt) ................... Sec. 7, Eq. (ssspnt)
 * Readings where the paper is silent (named at each function): Roe's flux with
 * Harten's entropy fix, minmod limiter, SSP-RK3 in Shu-Osher form and the
 * coefficients of the 2- and 4-stage second-order schemes, a global
 * CFL time step from U^n, the ghost rules per boundary kind, an RMS residual
 * norm; for the viscous flux: constant viscosity and Prandtl number, face
 * gradients by Green-Gauss over the diamond of the face (the two cell
 * centres and the two face nodes, node values the mean of the four cells
 * around the node), corner ghosts, ghost-cell centres, a no-slip wall rule and
 * a viscous term in the time-step limit; for 3D curvilinear cells: face area
 * vectors from the cross product of the face diagonals and volumes from the
 * divergence theorem over the six faces.
 */
#include "fv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long long i64;

typedef struct {
  int ni, nj, nk;      /* interior cells */
  int pi, pj, pk;      /* padded extents (2 ghost layers per side) */
  int gk;              /* ghost offset along k: 2 in 3D, 0 in 2D */
  i64 npad;            /* padded cells per variable */
  i64 ncell;           /* interior cells */
  double* xn;          /* node coordinates (owned copies) or NULL when uniform:  */
  double* yn;          /* 2D (nj+1)(ni+1); 3D (nk+1)(nj+1)(ni+1), i fastest  */
  double* zn;          /* 3D curvilinear only                                   */
  double* src;         /* nv * ncell: cell-averaged source S_h, or NULL         */
  double h[3];
  double origin[3];    /* uniform blocks: position of node (0, 0) */
  orc_bc bc[6];
  double* q;           /* nv * npad: state of the current stage, with ghosts */
  double* qn;          /* nv * npad: U^n */
  double* res;         /* nv * ncell: residual */
  double* flux;        /* nv * (faces of one direction): area-weighted face fluxes */
  i64 nflux;           /* capacity of flux per variable */
} blk_t;

struct orc_grid {
  int ndim, nv, nblocks;
  double gamma;
  blk_t* b;
  i64 ncells;
  /* time-marching record */
  double t, dt_last, raw_min;
  i64 steps;
  double norms[5], norm, norm_first, drop;
  int have_first, physical;
  /* viscosity of the time-step limit (that of the last run) */
  double mu, prandtl;
};

/* ------------------------------------------------------------------------ */
/* indexing                                                                  */
/* ------------------------------------------------------------------------ */
static inline i64 pidx(const blk_t* b, int i, int j, int k) {
  return ((i64)(k + b->gk) * b->pj + (j + 2)) * b->pi + (i + 2);
}
static inline i64 cidx(const blk_t* b, int i, int j, int k) {
  return ((i64)k * b->nj + j) * b->ni + i;
}
static inline int ext(const blk_t* b, int d) { return d == 0 ? b->ni : (d == 1 ? b->nj : b->nk); }

/* ------------------------------------------------------------------------ */
/* geometry (Sec. 3.1: face area ds, outward unit normal, volume |Omega|)   */
/* ------------------------------------------------------------------------ */
static inline double X(const blk_t* b, int i, int j) { return b->xn[(i64)j * (b->ni + 1) + i]; }
static inline double Y(const blk_t* b, int i, int j) { return b->yn[(i64)j * (b->ni + 1) + i]; }
/* node (i, j, k) of a 3D curvilinear block */
static inline void P3(const blk_t* b, int i, int j, int k, double p[3]) {
  const i64 n = ((i64)k * (b->nj + 1) + j) * (b->ni + 1) + i;
  p[0] = b->xn[n];
  p[1] = b->yn[n];
  p[2] = b->zn[n];
}

/* 3D curvilinear face (d, i, j, k): the quadrilateral of nodes
 *   d = 0: (i,j,k) (i,j+1,k) (i,j+1,k+1) (i,j,k+1)
 *   d = 1: (i,j,k) (i+1,j,k) (i+1,j,k+1) (i,j,k+1)
 *   d = 2: (i,j,k) (i+1,j,k) (i+1,j+1,k) (i,j+1,k)
 * with a, b, c, e its corners in this order.  Area vector (a reading: the
 * vector area of the bilinear face, which the paper's face area ds and
 * normal n come from): S = (c - a) x (e - b) / 2 oriented towards +index,
 * i.e. half the cross product of the diagonals.  Face centre: the mean of
 * the four corners. */
static void face3(const blk_t* b, int d, int i, int j, int k, double S[3], double C[3]) {
  int q[4][3];
  for (int m = 0; m < 4; ++m) {
    q[m][0] = i;
    q[m][1] = j;
    q[m][2] = k;
  }
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;  /* the two transverse axes */
  q[1][t1] += 1;
  q[2][t1] += 1;
  q[2][t2] += 1;
  q[3][t2] += 1;
  double p[4][3];
  for (int m = 0; m < 4; ++m) P3(b, q[m][0], q[m][1], q[m][2], p[m]);
  double d1[3], d2[3];
  for (int a = 0; a < 3; ++a) {
    d1[a] = p[2][a] - p[0][a];
    d2[a] = p[3][a] - p[1][a];
  }
  S[0] = 0.5 * (d1[1] * d2[2] - d1[2] * d2[1]);
  S[1] = 0.5 * (d1[2] * d2[0] - d1[0] * d2[2]);
  S[2] = 0.5 * (d1[0] * d2[1] - d1[1] * d2[0]);
  if (d == 1) {
    /* (i,j,k) (i+1,j,k) (i+1,j,k+1) (i,j,k+1) winds about -y: flip */
    S[0] = -S[0];
    S[1] = -S[1];
    S[2] = -S[2];
  }
  for (int a = 0; a < 3; ++a) C[a] = 0.25 * (((p[0][a] + p[1][a]) + p[2][a]) + p[3][a]);
}

/* Area vector of face (i,j,k) along direction d, pointing towards +index.
 * Face (i,j,k) of direction 0 separates cells (i-1,j,k) and (i,j,k).
 * 2D: the face is the segment between two nodes; its area vector is that
 * segment turned by -90 degrees (length = face length, per unit depth). */
static void face_vec(const blk_t* b, int nd, int d, int i, int j, int k, double S[3]) {
  S[0] = S[1] = S[2] = 0.0;
  if (b->zn) {
    double C[3];
    face3(b, d, i, j, k, S, C);
    return;
  }
  if (b->xn) {
    if (d == 0) {
      S[0] = Y(b, i, j + 1) - Y(b, i, j);
      S[1] = -(X(b, i, j + 1) - X(b, i, j));
    } else {
      S[0] = -(Y(b, i + 1, j) - Y(b, i, j));
      S[1] = X(b, i + 1, j) - X(b, i, j);
    }
    return;
  }
  if (nd == 2) {
    S[d] = (d == 0) ? b->h[1] : b->h[0];
  } else {
    S[d] = (d == 0) ? b->h[1] * b->h[2] : (d == 1 ? b->h[0] * b->h[2] : b->h[0] * b->h[1]);
  }
}

/* Cell volume: half the cross product of the two diagonals (2D), or hx*hy[*hz]. */
static double cell_vol(const blk_t* b, int nd, int i, int j, int k) {
  if (b->zn) {
    /* 3D curvilinear (a reading): the divergence theorem with x . n taken at
     * the face centres, |Omega| = (1/3) sum over the six faces of C_f . S_f
     * with outward area vectors; exact for parallelepipeds, and the sum
     * over a mesh telescopes to its boundary */
    double v = 0.0;
    for (int d = 0; d < 3; ++d) {
      int e[3] = {0, 0, 0};
      e[d] = 1;
      double Sm[3], Cm[3], Sp[3], Cp[3];
      face3(b, d, i, j, k, Sm, Cm);
      face3(b, d, i + e[0], j + e[1], k + e[2], Sp, Cp);
      v += (Cp[0] * Sp[0] + Cp[1] * Sp[1] + Cp[2] * Sp[2]) - (Cm[0] * Sm[0] + Cm[1] * Sm[1] + Cm[2] * Sm[2]);
    }
    return v / 3.0;
  }
  (void)k;
  if (b->xn) {
    double a = (X(b, i + 1, j + 1) - X(b, i, j)) * (Y(b, i, j + 1) - Y(b, i + 1, j));
    double c = (X(b, i, j + 1) - X(b, i + 1, j)) * (Y(b, i + 1, j + 1) - Y(b, i, j));
    return 0.5 * (a - c);
  }
  return nd == 2 ? b->h[0] * b->h[1] : b->h[0] * b->h[1] * b->h[2];
}

/* ------------------------------------------------------------------------ */
/* gas relations and the inviscid normal flux (Sec. 2)                      */
/* ------------------------------------------------------------------------ */
static void primitives(const double* q, int nd, double g, double* rho, double v[3], double* p,
                       double* H) {
  double ke = 0.0;
  *rho = q[0];
  v[0] = v[1] = v[2] = 0.0;
  for (int a = 0; a < nd; ++a) {
    v[a] = q[1 + a] / q[0];
    ke += v[a] * v[a];
  }
  *p = (g - 1.0) * (q[nd + 1] - 0.5 * q[0] * ke);
  *H = (q[nd + 1] + *p) / q[0];
}

/* F_{i,n} = (rho V_n, rho u V_n + n_x p, ..., rho h_t V_n) with V_n = n . u */
static void normal_flux(const double* q, const double* n, int nd, double g, double* F) {
  double rho, v[3], p, H;
  primitives(q, nd, g, &rho, v, &p, &H);
  double Vn = 0.0;
  for (int a = 0; a < nd; ++a) Vn += v[a] * n[a];
  F[0] = rho * Vn;
  for (int a = 0; a < nd; ++a) F[1 + a] = rho * v[a] * Vn + n[a] * p;
  F[nd + 1] = rho * H * Vn;
}

static void cons_from_prim(const double prim[5], int nd, double g, double* q) {
  double ke = 0.0;
  q[0] = prim[0];
  for (int a = 0; a < nd; ++a) {
    q[1 + a] = prim[0] * prim[1 + a];
    ke += prim[1 + a] * prim[1 + a];
  }
  q[nd + 1] = prim[4] / (g - 1.0) + 0.5 * prim[0] * ke;
}

/* ------------------------------------------------------------------------ */
/* Roe's approximate Riemann solver (the paper names no flux function; Roe  */
/* is the reading taken), written as the explicit sum over waves            */
/*     D = sum_k |lambda_k| alpha_k r_k                                     */
/* with Roe-averaged eigenvalues lambda, wave strengths alpha and right     */
/* eigenvectors r of the normal-flux Jacobian.  mode 0: |lambda| with       */
/* Harten's fix on the two acoustic waves (delta = entropy_fix * c);        */
/* mode 1: signed lambda (then D = F(Q_R).n - F(Q_L).n, Roe's property);    */
/* mode 2: lambda = 1 (then D = Q_R - Q_L, the wave decomposition).          */
/* ------------------------------------------------------------------------ */
static double harten(double l, double delta) {
  l = fabs(l);
  if (delta > 0.0 && l < delta) l = (l * l + delta * delta) / (2.0 * delta);
  return l;
}

static void roe_waves(const double* qL, const double* qR, const double* n, int nd, double g,
                      double efix, int mode, double* D) {
  double rL, vL[3], pL, HL, rR, vR[3], pR, HR;
  primitives(qL, nd, g, &rL, vL, &pL, &HL);
  primitives(qR, nd, g, &rR, vR, &pR, &HR);

  /* Roe averages */
  double Rt = sqrt(rR / rL);
  double rho_t = Rt * rL;
  double ut[3] = {0.0, 0.0, 0.0};
  double q2 = 0.0, Vn = 0.0;
  for (int a = 0; a < nd; ++a) {
    ut[a] = (vL[a] + Rt * vR[a]) / (1.0 + Rt);
    q2 += ut[a] * ut[a];
    Vn += ut[a] * n[a];
  }
  double Ht = (HL + Rt * HR) / (1.0 + Rt);
  double c2 = (g - 1.0) * (Ht - 0.5 * q2);
  double c = sqrt(c2);

  /* jumps of the primitive variables */
  double drho = rR - rL, dp = pR - pL, du[3] = {0.0, 0.0, 0.0}, dVn = 0.0, udu = 0.0;
  for (int a = 0; a < nd; ++a) {
    du[a] = vR[a] - vL[a];
    dVn += du[a] * n[a];
    udu += ut[a] * du[a];
  }

  /* eigenvalues: V_n - c, V_n (entropy and shear waves), V_n + c */
  double l1 = Vn - c, l2 = Vn, l5 = Vn + c;
  if (mode == 0) {
    l1 = harten(l1, efix * c);
    l2 = fabs(l2);
    l5 = harten(l5, efix * c);
  } else if (mode == 2) {
    l1 = l2 = l5 = 1.0;
  }

  /* wave strengths */
  double a1 = (dp - rho_t * c * dVn) / (2.0 * c2);
  double a5 = (dp + rho_t * c * dVn) / (2.0 * c2);
  double a2 = drho - dp / c2;

  /* acoustic wave  (1, u - c n, H - c V_n)
   * entropy wave   (1, u, |u|^2/2)
   * shear waves    rho (0, du - dV_n n, u.du - V_n dV_n)
   * acoustic wave  (1, u + c n, H + c V_n) */
  D[0] = l1 * a1 + l2 * a2 + l5 * a5;
  for (int a = 0; a < nd; ++a)
    D[1 + a] = l1 * a1 * (ut[a] - c * n[a]) + l2 * (a2 * ut[a] + rho_t * (du[a] - dVn * n[a])) +
               l5 * a5 * (ut[a] + c * n[a]);
  D[nd + 1] = l1 * a1 * (Ht - c * Vn) + l2 * (a2 * 0.5 * q2 + rho_t * (udu - Vn * dVn)) +
              l5 * a5 * (Ht + c * Vn);
}

/* Numerical flux per unit area: F = (F(Q_L).n + F(Q_R).n)/2 - D/2. */
static void roe_flux(const double* qL, const double* qR, const double* n, int nd, double g,
                     double efix, double* F) {
  double FL[5], FR[5], D[5];
  normal_flux(qL, n, nd, g, FL);
  normal_flux(qR, n, nd, g, FR);
  roe_waves(qL, qR, n, nd, g, efix, 0, D);
  for (int v = 0; v < nd + 2; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * D[v];
}

void orc_roe(const double* qL, const double* qR, const double* n, int nd, double gamma,
             double entropy_fix, int mode, double* out) {
  if (mode < 0) {
    roe_flux(qL, qR, n, nd, gamma, entropy_fix, out);
  } else if (mode == 3) {
    normal_flux(qL, n, nd, gamma, out);
  } else {
    roe_waves(qL, qR, n, nd, gamma, entropy_fix, mode, out);
  }
}

/* ------------------------------------------------------------------------ */
/* MUSCL extrapolation, Sec. 5, Eq. (flux).  For the face between cells m   */
/* and m+1, with Q = (Q_{m-1}, Q_m, Q_{m+1}, Q_{m+2}):                       */
/*   Q^L = Q_m     + eps/4 [(1-k) Psi+_{m-1/2} (Q_m - Q_{m-1})              */
/*                        + (1+k) Psi-_{m+1/2} (Q_{m+1} - Q_m)]             */
/*   Q^R = Q_{m+1} - eps/4 [(1+k) Psi+_{m+1/2} (Q_{m+1} - Q_m)              */
/*                        + (1-k) Psi-_{m+3/2} (Q_{m+2} - Q_{m+1})]         */
/* Reading of the limiter values (the paper only calls them limiter         */
/* function values): Psi+_{m-1/2} = Psi(r) with r = (Q_{m+1}-Q_m)/(Q_m -    */
/* Q_{m-1}), Psi-_{m+1/2} = Psi(r) with r = (Q_m - Q_{m-1})/(Q_{m+1}-Q_m),  */
/* and likewise one cell on for Q^R.  Psi is minmod, Psi(r) = max(0,        */
/* min(1, r)); the unlimited scheme takes Psi = 1 and the first-order       */
/* scheme eps = 0.  The product Psi(num/den) * den is what enters; for a    */
/* zero den it is taken as its limit 0 (minmod is bounded by 1).            */
/* ------------------------------------------------------------------------ */
static double psi_times(int limiter, double num, double den) {
  if (limiter == ORC_UNLIMITED) return den;
  if (den == 0.0) return 0.0;
  double r = num / den;
  double psi = r < 1.0 ? r : 1.0;
  if (psi < 0.0) psi = 0.0;
  return psi * den;
}

static void muscl(const double q[4], int limiter, double eps, double kappa, double* qL,
                  double* qR) {
  if (limiter == ORC_FIRST_ORDER) eps = 0.0;
  double dm = q[1] - q[0]; /* Q_m     - Q_{m-1} */
  double d0 = q[2] - q[1]; /* Q_{m+1} - Q_m     */
  double dp = q[3] - q[2]; /* Q_{m+2} - Q_{m+1} */
  *qL = q[1] + 0.25 * eps *
                   ((1.0 - kappa) * psi_times(limiter, d0, dm) +
                    (1.0 + kappa) * psi_times(limiter, dm, d0));
  *qR = q[2] - 0.25 * eps *
                   ((1.0 + kappa) * psi_times(limiter, dp, d0) +
                    (1.0 - kappa) * psi_times(limiter, d0, dp));
}

void orc_reconstruct(const double* q4, int limiter, double eps, double kappa, double* qL,
                     double* qR) {
  muscl(q4, limiter, eps, kappa, qL, qR);
}

/* ------------------------------------------------------------------------ */
/* ghost cells (2 layers), refreshed before every residual evaluation.      */
/* Readings of the boundary rules (the paper names only ghost extrapolation */
/* and inter-block exchange):                                                */
/*   PERIODIC  ghost = interior cell the same distance in from the opposite  */
/*             face of the same block                                        */
/*   BLOCK     ghost = neighbour block's interior cell the same distance in  */
/*             from its matching face (1:1 points, same orientation)         */
/*   INFLOW    ghost = Q of the prescribed primitive state                   */
/*   EXTRAP    ghost = nearest interior cell (zeroth-order extrapolation)    */
/*   SLIPWALL  ghost g = interior cell g-1 from the wall with its momentum   */
/*             mirrored about the unit normal of that wall face; rho and     */
/*             rho*e_t copied                                                */
/*   NOSLIP    ghost g = interior cell g-1 from the wall with the velocity   */
/*             2 w - u (w the wall velocity), density and pressure kept: the */
/*             face average of the velocity is w and the wall is adiabatic   */
/* The inviscid stencil reads one direction at a time; the viscous flux     */
/* (2D) also reads the first corner ghost of each block corner (below).     */
/* ------------------------------------------------------------------------ */
/* no-slip ghost of a copied interior state q: in conserved variables the
 * momentum becomes m' = 2 rho w - m and the total energy gains the change of
 * kinetic energy, (|m'|^2 - |m|^2) / (2 rho), so that rho and p are kept.
 * A wall at rest gives m' = -m and rho e_t unchanged, exactly. */
static void noslip_ghost(double* q, const double* wall, int nd) {
  double m2 = 0.0, n2 = 0.0;
  for (int a = 0; a < nd; ++a) {
    const double m = q[1 + a];
    const double mp = 2.0 * q[0] * wall[1 + a] - m;
    m2 += m * m;
    n2 += mp * mp;
    q[1 + a] = mp;
  }
  q[nd + 1] += 0.5 * (n2 - m2) / q[0];
}

static void set3(int d, int along, int t1, int t2, int* i, int* j, int* k) {
  if (d == 0) { *i = along; *j = t1; *k = t2; }
  else if (d == 1) { *i = t1; *j = along; *k = t2; }
  else { *i = t1; *j = t2; *k = along; }
}
static void trans_ext(const blk_t* b, int d, int* n1, int* n2) {
  if (d == 0) { *n1 = b->nj; *n2 = b->nk; }
  else if (d == 1) { *n1 = b->ni; *n2 = b->nk; }
  else { *n1 = b->ni; *n2 = b->nj; }
}

/* ghost value of block b, face f, layer g (1 or 2), transverse (t1, t2) */
static void ghost_value(const orc_grid* G, int bi, int f, int g, int t1, int t2, double* out) {
  const blk_t* b = &G->b[bi];
  const int nd = G->ndim, nv = G->nv;
  const int d = f / 2, side = f % 2, n = ext(b, d);
  const orc_bc* bc = &b->bc[f];
  const blk_t* src = b;
  int along;
  int sd = d, s1 = t1, s2 = t2; /* source direction and transverse indices */
  int i, j, k;
  switch (bc->kind) {
    case ORC_PERIODIC:
      along = side == 0 ? n - g : g - 1;
      break;
    case ORC_BLOCK: {
      /* the neighbour's cell g-1 in from its face nbr_face, at the transverse
       * position the orientation gives (t1, t2): swapped (bit 0), then each
       * reversed (bits 1, 2) in the neighbour's own index range */
      src = &G->b[bc->nbr_block];
      sd = bc->nbr_face / 2;
      const int nside = bc->nbr_face % 2;
      int m1, m2;
      trans_ext(src, sd, &m1, &m2);
      s1 = (bc->orient & 1) ? t2 : t1;
      s2 = (bc->orient & 1) ? t1 : t2;
      if (bc->orient & 2) s1 = m1 - 1 - s1;
      if (bc->orient & 4) s2 = m2 - 1 - s2;
      along = nside == 0 ? g - 1 : ext(src, sd) - g;
      break;
    }
    case ORC_INFLOW:
      cons_from_prim(bc->prim, nd, G->gamma, out);
      return;
    case ORC_EXTRAP:
      along = side == 0 ? 0 : n - 1;
      break;
    case ORC_SLIPWALL:
    case ORC_NOSLIP:
      along = side == 0 ? g - 1 : n - g;
      break;
    default:
      for (int v = 0; v < nv; ++v) out[v] = NAN;
      return;
  }
  set3(sd, along, s1, s2, &i, &j, &k);
  i64 p = pidx(src, i, j, k);
  for (int v = 0; v < nv; ++v) out[v] = src->q[v * src->npad + p];
  if (bc->kind == ORC_SLIPWALL) {
    double S[3];
    int wi, wj, wk;
    set3(d, side == 0 ? 0 : n, t1, t2, &wi, &wj, &wk);
    face_vec(b, nd, d, wi, wj, wk, S);
    double A = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
    double nh[3] = {S[0] / A, S[1] / A, S[2] / A};
    double mn = 0.0;
    for (int a = 0; a < nd; ++a) mn += out[1 + a] * nh[a];
    for (int a = 0; a < nd; ++a) out[1 + a] -= 2.0 * mn * nh[a];
  }
  if (bc->kind == ORC_NOSLIP) noslip_ghost(out, bc->prim, nd);
}

/* Value of cell (i, j) of 2D block bi, where i and j may each lie up to two
 * cells outside the block.  A cell outside in i follows the i-face rule
 * first; the cell that rule names (in this block or, through a block link,
 * in the neighbour) is then resolved in its own block, by that block's
 * j-face rule when j lies outside too, and the i-rule's wall mirror is
 * applied last.  A cell outside in j only follows the j-face rule, which is
 * the edge ghost above.  The corner ghosts this defines are read only by
 * the viscous node values; across a block link they are the neighbour's own
 * ghosts, so a node on the link has one value for both blocks. */
static void cell_value_2d(const orc_grid* G, int bi, int i, int j, double* out) {
  const blk_t* b = &G->b[bi];
  const int nv = G->nv;
  if (i >= 0 && i < b->ni && j >= 0 && j < b->nj) {
    const i64 p = pidx(b, i, j, 0);
    for (int v = 0; v < nv; ++v) out[v] = b->q[v * b->npad + p];
    return;
  }
  const int d = (i < 0 || i >= b->ni) ? 0 : 1;
  const int n = ext(b, d), x = d == 0 ? i : j;
  const int side = x < 0 ? 0 : 1, g = side == 0 ? -x : x - n + 1;
  const orc_bc* bc = &b->bc[2 * d + side];
  int src = bi, along;
  switch (bc->kind) {
    case ORC_INFLOW:
      cons_from_prim(bc->prim, 2, G->gamma, out);
      return;
    case ORC_PERIODIC:
      along = side == 0 ? n - g : g - 1;
      break;
    case ORC_BLOCK:
      src = bc->nbr_block;
      along = side == 0 ? ext(&G->b[src], d) - g : g - 1;
      break;
    case ORC_EXTRAP:
      along = side == 0 ? 0 : n - 1;
      break;
    default: /* SLIPWALL, NOSLIP */
      along = side == 0 ? g - 1 : n - g;
      break;
  }
  cell_value_2d(G, src, d == 0 ? along : i, d == 0 ? j : along, out);
  if (bc->kind == ORC_SLIPWALL) {
    /* wall face of the nearest row (column) inside the block */
    const int t = d == 0 ? j : i, tn = d == 0 ? b->nj : b->ni;
    const int tc = t < 0 ? 0 : (t >= tn ? tn - 1 : t);
    double S[3];
    face_vec(b, 2, d, d == 0 ? (side == 0 ? 0 : n) : tc, d == 0 ? tc : (side == 0 ? 0 : n), 0, S);
    const double A = sqrt(S[0] * S[0] + S[1] * S[1]);
    const double nh[2] = {S[0] / A, S[1] / A};
    const double mn = out[1] * nh[0] + out[2] * nh[1];
    for (int a = 0; a < 2; ++a) out[1 + a] -= 2.0 * mn * nh[a];
  } else if (bc->kind == ORC_NOSLIP) {
    noslip_ghost(out, bc->prim, 2);
  }
}

static void fill_ghosts(orc_grid* G) {
  const int nd = G->ndim, nv = G->nv;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    for (int f = 0; f < 2 * nd; ++f) {
      const int d = f / 2, side = f % 2, n = ext(b, d);
      int n1, n2;
      trans_ext(b, d, &n1, &n2);
      for (int t2 = 0; t2 < n2; ++t2)
        for (int t1 = 0; t1 < n1; ++t1)
          for (int g = 1; g <= 2; ++g) {
            double val[5];
            ghost_value(G, bi, f, g, t1, t2, val);
            int i, j, k;
            set3(d, side == 0 ? -g : n - 1 + g, t1, t2, &i, &j, &k);
            i64 p = pidx(b, i, j, k);
            for (int v = 0; v < nv; ++v) b->q[v * b->npad + p] = val[v];
          }
    }
  }
  /* 2D: the corner ghosts (both layers), after every edge ghost is known */
  if (nd != 2) return;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    const int ci[4] = {-2, -1, b->ni, b->ni + 1}, cj[4] = {-2, -1, b->nj, b->nj + 1};
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 4; ++c) {
        double val[5];
        cell_value_2d(G, bi, ci[a], cj[c], val);
        const i64 p = pidx(b, ci[a], cj[c], 0);
        for (int v = 0; v < nv; ++v) b->q[v * b->npad + p] = val[v];
      }
  }
}

/* ------------------------------------------------------------------------ */
/* residual, Sec. 3.1, Eq. (residual):                                      */
/*   R_cell = sum over its f faces of (F_{i,n} - F_{nu,n}) ds (outward      */
/*   normals; the viscous part when mu > 0, 2D) - |Omega| S_h, the source   */
/*   term when one is set.                                                  */
/* Each face flux is formed once, stored times its area, then each cell     */
/* sums, direction by direction (i, j, k), the flux leaving through its     */
/* +face minus the flux entering through its -face.                          */
/* ------------------------------------------------------------------------ */
static void face_flux_at(const orc_grid* G, const blk_t* b, const orc_params* P, int d, int i,
                         int j, int k, double* F) {
  const int nd = G->ndim, nv = G->nv;
  int e[3] = {0, 0, 0};
  e[d] = 1;
  double qL[5], qR[5];
  for (int v = 0; v < nv; ++v) {
    const double* q = b->q + (i64)v * b->npad;
    double s[4];
    for (int m = 0; m < 4; ++m) {
      int o = m - 2; /* cells f-2, f-1, f, f+1 along d */
      s[m] = q[pidx(b, i + o * e[0], j + o * e[1], k + o * e[2])];
    }
    muscl(s, P->limiter, P->eps, P->kappa, &qL[v], &qR[v]);
  }
  double S[3];
  face_vec(b, nd, d, i, j, k, S);
  double A = sqrt(S[0] * S[0] + S[1] * S[1] + S[2] * S[2]);
  double n[3] = {S[0] / A, S[1] / A, S[2] / A};
  double Fu[5];
  roe_flux(qL, qR, n, nd, G->gamma, P->entropy_fix, Fu);
  for (int v = 0; v < nv; ++v) F[v] = Fu[v] * A;
}


/* ------------------------------------------------------------------------ */
/* viscous normal flux of Sec. 2 (2D): F_{nu,n} ds = (0, tau_x . S,         */
/* tau_y . S, Theta . S) with S the face's area vector.  Readings (the     */
/* paper names Stokes's hypothesis and "heat conduction and work of the     */
/* viscous stresses" only):                                                 */
/*   tau = mu (grad u + grad u^T) - (2/3) mu (div u) I, mu constant;        */
/*   Theta = tau u + k grad T, Fourier's law with a constant Prandtl number:*/
/*   k grad T = (mu / Pr) gamma/(gamma-1) grad(p/rho) for an ideal gas.     */
/* Face gradients by Green-Gauss over the diamond of the face, whose        */
/* corners are the centres L, R of its two cells and its end nodes A, B     */
/* (ordered so that B - A turned by -90 degrees is S):                      */
/*   grad phi = [(phi_R - phi_L) S - (phi_B - phi_A) d_perp] / (d . S),     */
/*   d = x_R - x_L, d_perp = (d_y, -d_x),                                   */
/* which gives d . grad phi = phi_R - phi_L and (B - A) . grad phi =        */
/* phi_B - phi_A, i.e. the exact gradient of a linear field.  Node values   */
/* are the mean of the four cells around the node (ghosts and corner ghosts */
/* included), cell centres the mean of their four nodes, and u at the face  */
/* the mean of L and R.  The differentiated variables are u, v and p/rho.  */
/* ------------------------------------------------------------------------ */
static void node_xy(const blk_t* b, int i, int j, double* x, double* y) {
  if (b->xn) {
    *x = X(b, i, j);
    *y = Y(b, i, j);
  } else {
    *x = b->origin[0] + i * b->h[0];
    *y = b->origin[1] + j * b->h[1];
  }
}

static void centre_xy(const blk_t* b, int i, int j, double c[2]) {
  double x0, y0, x1, y1, x2, y2, x3, y3;
  node_xy(b, i, j, &x0, &y0);
  node_xy(b, i + 1, j, &x1, &y1);
  node_xy(b, i, j + 1, &x2, &y2);
  node_xy(b, i + 1, j + 1, &x3, &y3);
  c[0] = 0.25 * (((x0 + x1) + x2) + x3);
  c[1] = 0.25 * (((y0 + y1) + y2) + y3);
}

/* midpoint of face (d, i, j): nodes (i, j) and (i, j+1) for d = 0, (i, j)
 * and (i+1, j) for d = 1 */
static void face_mid(const blk_t* b, int d, int i, int j, double m[2]) {
  double x0, y0, x1, y1;
  node_xy(b, i, j, &x0, &y0);
  node_xy(b, d == 0 ? i : i + 1, d == 0 ? j + 1 : j, &x1, &y1);
  m[0] = 0.5 * (x0 + x1);
  m[1] = 0.5 * (y0 + y1);
}

/* Centre of cell (i, j) of block bi, or of a first-layer ghost outside one
 * face (a reading for ghost cells): across a block link the neighbour's
 * cell; across a periodic face the image cell moved by the offset between
 * the two periodic faces; otherwise the interior neighbour's centre
 * reflected through the boundary face's midpoint. */
static void cell_centre_2d(const orc_grid* G, int bi, int i, int j, double c[2]) {
  const blk_t* b = &G->b[bi];
  if (i >= 0 && i < b->ni && j >= 0 && j < b->nj) {
    centre_xy(b, i, j, c);
    return;
  }
  const int d = (i < 0 || i >= b->ni) ? 0 : 1;
  const int n = ext(b, d), side = (d == 0 ? i : j) < 0 ? 0 : 1;
  const orc_bc* bc = &b->bc[2 * d + side];
  double m[2];
  face_mid(b, d, d == 0 ? (side ? n : 0) : i, d == 0 ? j : (side ? n : 0), m);
  if (bc->kind == ORC_BLOCK) {
    const blk_t* nb = &G->b[bc->nbr_block];
    const int along = side == 0 ? ext(nb, d) - 1 : 0;
    centre_xy(nb, d == 0 ? along : i, d == 0 ? j : along, c);
  } else if (bc->kind == ORC_PERIODIC) {
    const int along = side == 0 ? n - 1 : 0;
    double mo[2];
    face_mid(b, d, d == 0 ? (side ? 0 : n) : i, d == 0 ? j : (side ? 0 : n), mo);
    centre_xy(b, d == 0 ? along : i, d == 0 ? j : along, c);
    c[0] += m[0] - mo[0];
    c[1] += m[1] - mo[1];
  } else {
    const int along = side == 0 ? 0 : n - 1;
    centre_xy(b, d == 0 ? along : i, d == 0 ? j : along, c);
    c[0] = 2.0 * m[0] - c[0];
    c[1] = 2.0 * m[1] - c[1];
  }
}

/* u, v and p/rho of the padded cell (i, j) */
static void cell_uvt(const blk_t* b, int i, int j, double g, double o[3]) {
  const i64 p = pidx(b, i, j, 0);
  const double r = b->q[p], mx = b->q[b->npad + p], my = b->q[2 * b->npad + p];
  const double E = b->q[3 * b->npad + p];
  o[0] = mx / r;
  o[1] = my / r;
  const double pr = (g - 1.0) * (E - 0.5 * r * (o[0] * o[0] + o[1] * o[1]));
  o[2] = pr / r;
}

/* node (i, j): mean of cells (i-1, j-1), (i, j-1), (i-1, j), (i, j) */
static void node_uvt(const blk_t* b, int i, int j, double g, double o[3]) {
  double a[3], s[3] = {0.0, 0.0, 0.0};
  const int ci[4] = {i - 1, i, i - 1, i}, cj[4] = {j - 1, j - 1, j, j};
  for (int c = 0; c < 4; ++c) {
    cell_uvt(b, ci[c], cj[c], g, a);
    for (int k = 0; k < 3; ++k) s[k] += a[k];
  }
  for (int k = 0; k < 3; ++k) o[k] = 0.25 * s[k];
}

/* F_{nu,n} ds of face (d, i, j) of block bi (ghosts filled) */
static void viscous_flux_2d(const orc_grid* G, int bi, const orc_params* P, int d, int i, int j,
                            double* F) {
  const blk_t* b = &G->b[bi];
  const double g = G->gamma, mu = P->mu;
  const int iL = d == 0 ? i - 1 : i, jL = d == 0 ? j : j - 1;
  const int ia = d == 0 ? i : i + 1, ja = j, ib = i, jb = d == 0 ? j + 1 : j;
  double wL[3], wR[3], wA[3], wB[3], xL[2], xR[2], S[3];
  cell_uvt(b, iL, jL, g, wL);
  cell_uvt(b, i, j, g, wR);
  node_uvt(b, ia, ja, g, wA);
  node_uvt(b, ib, jb, g, wB);
  cell_centre_2d(G, bi, iL, jL, xL);
  cell_centre_2d(G, bi, i, j, xR);
  face_vec(b, 2, d, i, j, 0, S);
  const double dx = xR[0] - xL[0], dy = xR[1] - xL[1];
  const double D = dx * S[0] + dy * S[1];
  double gx[3], gy[3];
  for (int k = 0; k < 3; ++k) {
    const double a = wR[k] - wL[k], t = wB[k] - wA[k];
    gx[k] = (a * S[0] - t * dy) / D;
    gy[k] = (a * S[1] + t * dx) / D;
  }
  const double dv = gx[0] + gy[1];
  const double txx = mu * (2.0 * gx[0] - (2.0 / 3.0) * dv);
  const double tyy = mu * (2.0 * gy[1] - (2.0 / 3.0) * dv);
  const double txy = mu * (gy[0] + gx[1]);
  const double uf = 0.5 * (wL[0] + wR[0]), vf = 0.5 * (wL[1] + wR[1]);
  const double kq = mu / P->prandtl * g / (g - 1.0);
  const double thx = uf * txx + vf * txy + kq * gx[2];
  const double thy = uf * txy + vf * tyy + kq * gy[2];
  F[0] = 0.0;
  F[1] = txx * S[0] + txy * S[1];
  F[2] = txy * S[0] + tyy * S[1];
  F[3] = thx * S[0] + thy * S[1];
}

static void residual_block(const orc_grid* G, int bi, const orc_params* P, double* scale) {
  blk_t* b = &G->b[bi];
  const int nd = G->ndim, nv = G->nv;
  memset(b->res, 0, sizeof(double) * (size_t)nv * (size_t)b->ncell);
  if (scale) memset(scale, 0, sizeof(double) * (size_t)nv * (size_t)b->ncell);
  for (int d = 0; d < nd; ++d) {
    const int fi = b->ni + (d == 0), fj = b->nj + (d == 1), fk = b->nk + (d == 2);
    const i64 nf = (i64)fi * fj * fk;
    double* fl = b->flux;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < fk; ++k)
      for (int j = 0; j < fj; ++j)
        for (int i = 0; i < fi; ++i) {
          double F[5];
          face_flux_at(G, b, P, d, i, j, k, F);
          if (P->mu > 0.0) {
            double Fv[4];
            viscous_flux_2d(G, bi, P, d, i, j, Fv);
            for (int v = 0; v < nv; ++v) F[v] -= Fv[v];
          }
          i64 f = ((i64)k * fj + j) * fi + i;
          for (int v = 0; v < nv; ++v) fl[v * nf + f] = F[v];
        }
    int e[3] = {0, 0, 0};
    e[d] = 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < b->nk; ++k)
      for (int j = 0; j < b->nj; ++j)
        for (int i = 0; i < b->ni; ++i) {
          i64 c = cidx(b, i, j, k);
          i64 fm = ((i64)k * fj + j) * fi + i;
          i64 fp = ((i64)(k + e[2]) * fj + (j + e[1])) * fi + (i + e[0]);
          for (int v = 0; v < nv; ++v) {
            b->res[v * b->ncell + c] += fl[v * nf + fp] - fl[v * nf + fm];
            if (scale) scale[v * b->ncell + c] += fabs(fl[v * nf + fp]) + fabs(fl[v * nf + fm]);
          }
        }
  }
  /* the source part of Eq. (residual): - |Omega| S_h, after every face */
  if (!b->src) return;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < b->nk; ++k)
    for (int j = 0; j < b->nj; ++j)
      for (int i = 0; i < b->ni; ++i) {
        const i64 c = cidx(b, i, j, k);
        const double vol = cell_vol(b, nd, i, j, k);
        for (int v = 0; v < nv; ++v) {
          const double s = vol * b->src[v * b->ncell + c];
          b->res[v * b->ncell + c] -= s;
          if (scale) scale[v * b->ncell + c] += fabs(s);
        }
      }
}

static void residual_all(orc_grid* G, const orc_params* P, double** scales) {
  fill_ghosts(G);
  for (int bi = 0; bi < G->nblocks; ++bi)
    residual_block(G, bi, P, scales ? scales[bi] : NULL);
}

/* RMS of R/|Omega| per variable over every interior cell of every block,
 * in natural order; combined norm sqrt(sum_v (r_v / qref_v)^2).           */
static void norms_of_residual(orc_grid* G, const orc_params* P, double* norms, double* comb) {
  const int nd = G->ndim, nv = G->nv;
  double s[5] = {0, 0, 0, 0, 0};
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    for (int k = 0; k < b->nk; ++k)
      for (int j = 0; j < b->nj; ++j)
        for (int i = 0; i < b->ni; ++i) {
          double vol = cell_vol(b, nd, i, j, k);
          i64 c = cidx(b, i, j, k);
          for (int v = 0; v < nv; ++v) {
            double r = b->res[v * b->ncell + c] / vol;
            s[v] += r * r;
          }
        }
  }
  double cs = 0.0;
  for (int v = 0; v < 5; ++v) norms[v] = 0.0;
  for (int v = 0; v < nv; ++v) {
    norms[v] = sqrt(s[v] / (double)G->ncells);
    double qv = P->qref[v] != 0.0 ? P->qref[v] : 1.0;
    cs += (norms[v] / qv) * (norms[v] / qv);
  }
  *comb = sqrt(cs);
}

/* ------------------------------------------------------------------------ */
/* time step (reading: global CFL step from U^n).  For each cell the local  */
/* limit is |Omega| / sum_d (|u . Sbar_d| + c |Sbar_d|), Sbar_d the mean of */
/* the cell's two face vectors of direction d; dt = CFL * min over every    */
/* cell of every block.  With viscosity (a reading) the sum gains the       */
/* diffusive term 2 max(4/3, gamma/Pr) (mu/rho) sum_d |Sbar_d|^2 / |Omega|. */
/* The state is also checked: rho > 0, p > 0, finite.                       */
/* ------------------------------------------------------------------------ */
int orc_spectral_min(orc_grid* G, double* raw_min) {
  const int nd = G->ndim, nv = G->nv;
  double mn = INFINITY;
  int ok = 1;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    for (int k = 0; k < b->nk; ++k)
      for (int j = 0; j < b->nj; ++j)
        for (int i = 0; i < b->ni; ++i) {
          double q[5], rho, v[3], p, H;
          i64 pp = pidx(b, i, j, k);
          for (int a = 0; a < nv; ++a) {
            q[a] = b->q[a * b->npad + pp];
            if (!isfinite(q[a])) ok = 0;
          }
          primitives(q, nd, G->gamma, &rho, v, &p, &H);
          if (!(rho > 0.0) || !(p > 0.0)) {
            ok = 0;
            continue;
          }
          double c = sqrt(G->gamma * p / rho);
          double lam = 0.0, ss = 0.0;
          for (int d = 0; d < nd; ++d) {
            double Sm[3], Sp[3];
            int e[3] = {0, 0, 0};
            e[d] = 1;
            face_vec(b, nd, d, i, j, k, Sm);
            face_vec(b, nd, d, i + e[0], j + e[1], k + e[2], Sp);
            double Sb[3] = {0.5 * (Sm[0] + Sp[0]), 0.5 * (Sm[1] + Sp[1]), 0.5 * (Sm[2] + Sp[2])};
            double us = v[0] * Sb[0] + v[1] * Sb[1] + v[2] * Sb[2];
            lam += fabs(us) + c * sqrt(Sb[0] * Sb[0] + Sb[1] * Sb[1] + Sb[2] * Sb[2]);
            ss += Sb[0] * Sb[0] + Sb[1] * Sb[1] + Sb[2] * Sb[2];
          }
          const double vol = cell_vol(b, nd, i, j, k);
          if (G->mu > 0.0) {
            const double f = fmax(4.0 / 3.0, G->gamma / G->prandtl);
            lam += 2.0 * f * (G->mu / rho) * ss / vol;
          }
          double loc = vol / lam;
          if (loc < mn) mn = loc;
        }
  }
  *raw_min = mn;
  G->raw_min = mn;
  G->physical = ok;
  return ok ? ORC_OK : ORC_E_NONPHYSICAL;
}

/* ------------------------------------------------------------------------ */
/* SSP-RK3 (Shu-Osher form), the explicit RK of Sec. 3.2, Eq. (runge_kutta) */
/* with c = (0, 1, 1/2), a21 = 1, a31 = a32 = 1/4, b = (1/6, 1/6, 2/3) and  */
/* the step scaled by 1/|Omega| as Eq. (spatial_residual) requires:         */
/*   U1 = U^n + dt L(U^n)                                                   */
/*   U2 = 3/4 U^n + 1/4 (U1 + dt L(U1))                                     */
/*   U^{n+1} = 1/3 U^n + 2/3 (U2 + dt L(U2)),   L(U) = -R(U)/|Omega|.       */
/* Ghosts are refreshed before every L.  Norms come from R(U^n).            */
/* ------------------------------------------------------------------------ */
static const double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

static void rk3_step(orc_grid* G, const orc_params* P, double dt) {
  const int nd = G->ndim, nv = G->nv;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    memcpy(b->qn, b->q, sizeof(double) * (size_t)nv * (size_t)b->npad);
  }
  for (int s = 0; s < 3; ++s) {
    residual_all(G, P, NULL);
    if (s == 0) norms_of_residual(G, P, G->norms, &G->norm);
    for (int bi = 0; bi < G->nblocks; ++bi) {
      blk_t* b = &G->b[bi];
#pragma omp parallel for collapse(2) schedule(static)
      for (int k = 0; k < b->nk; ++k)
        for (int j = 0; j < b->nj; ++j)
          for (int i = 0; i < b->ni; ++i) {
            double vol = cell_vol(b, nd, i, j, k);
            i64 c = cidx(b, i, j, k), p = pidx(b, i, j, k);
            for (int v = 0; v < nv; ++v) {
              double un = b->qn[v * b->npad + p];
              double us = b->q[v * b->npad + p];
              double r = b->res[v * b->ncell + c];
              b->q[v * b->npad + p] = RK_A[s] * un + RK_B[s] * (us - dt / vol * r);
            }
          }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Explicit RK in the Butcher form of Sec. 3.2, Eq. (runge_kutta), with R  */
/* per unit volume (Eq. spatial_residual):                                  */
/*   U^i     = U^n - dt sum_{j<i} a_ij R(U^j)/|Omega|,   i = 1..s          */
/*   U^{n+1} = U^n - dt sum_i   b_i  R(U^i)/|Omega|.                        */
/* The paper uses second-order 2-stage and 4-stage schemes and leaves the   */
/* coefficients to a reference.  Taken here (a reading):                    */
/*   2 stages: a21 = 1/2,                     b = (0, 1)                    */
/*   4 stages: a21 = 1/4, a32 = 1/3, a43 = 1/2, b = (0, 0, 0, 1)            */
/* Every stage residual R(U^i) is kept, as the form is written; ghosts are  */
/* refreshed before each residual.  Norms come from R(U^1) = R(U^n).        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int s;
  double a[4][4];
  double b[4];
} tableau_t;

static int tableau_of(int rk, tableau_t* T) {
  memset(T, 0, sizeof(*T));
  if (rk == 2) {
    T->s = 2;
    T->a[1][0] = 0.5;
    T->b[1] = 1.0;
    return 1;
  }
  if (rk == 4) {
    T->s = 4;
    T->a[1][0] = 0.25;
    T->a[2][1] = 1.0 / 3.0;
    T->a[3][2] = 0.5;
    T->b[3] = 1.0;
    return 1;
  }
  if (rk == 103) {
    /* SSP-RK3 written in this form (a check of the form against the
     * Shu-Osher arrangement above; selected by tests only) */
    T->s = 3;
    T->a[1][0] = 1.0;
    T->a[2][0] = 0.25;
    T->a[2][1] = 0.25;
    T->b[0] = 1.0 / 6.0;
    T->b[1] = 1.0 / 6.0;
    T->b[2] = 2.0 / 3.0;
    return 1;
  }
  return 0;
}

static int butcher_step(orc_grid* G, const orc_params* P, double dt, const tableau_t* T) {
  const int nd = G->ndim, nv = G->nv, s = T->s;
  double** rs = (double**)calloc((size_t)G->nblocks * (size_t)s, sizeof(double*));
  if (!rs) return ORC_E_NOMEM;
  int st = ORC_OK;
  for (int bi = 0; bi < G->nblocks && st == ORC_OK; ++bi) {
    blk_t* b = &G->b[bi];
    memcpy(b->qn, b->q, sizeof(double) * (size_t)nv * (size_t)b->npad);
    for (int i = 0; i < s; ++i) {
      rs[bi * s + i] = (double*)malloc(sizeof(double) * (size_t)nv * (size_t)b->ncell);
      if (!rs[bi * s + i]) st = ORC_E_NOMEM;
    }
  }
  for (int i = 0; i < s && st == ORC_OK; ++i) {
    /* stage state U^i (U^1 = U^n, already in q) */
    if (i > 0) {
      for (int bi = 0; bi < G->nblocks; ++bi) {
        blk_t* b = &G->b[bi];
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < b->nk; ++k)
          for (int j = 0; j < b->nj; ++j)
            for (int ii = 0; ii < b->ni; ++ii) {
              double vol = cell_vol(b, nd, ii, j, k);
              i64 c = cidx(b, ii, j, k), p = pidx(b, ii, j, k);
              for (int v = 0; v < nv; ++v) {
                double acc = 0.0;
                for (int jj = 0; jj < i; ++jj) acc += T->a[i][jj] * rs[bi * s + jj][v * b->ncell + c];
                b->q[v * b->npad + p] = b->qn[v * b->npad + p] - dt * acc / vol;
              }
            }
      }
    }
    residual_all(G, P, NULL);
    if (i == 0) norms_of_residual(G, P, G->norms, &G->norm);
    for (int bi = 0; bi < G->nblocks; ++bi) {
      blk_t* b = &G->b[bi];
      memcpy(rs[bi * s + i], b->res, sizeof(double) * (size_t)nv * (size_t)b->ncell);
    }
  }
  if (st == ORC_OK) {
    for (int bi = 0; bi < G->nblocks; ++bi) {
      blk_t* b = &G->b[bi];
#pragma omp parallel for collapse(2) schedule(static)
      for (int k = 0; k < b->nk; ++k)
        for (int j = 0; j < b->nj; ++j)
          for (int ii = 0; ii < b->ni; ++ii) {
            double vol = cell_vol(b, nd, ii, j, k);
            i64 c = cidx(b, ii, j, k), p = pidx(b, ii, j, k);
            for (int v = 0; v < nv; ++v) {
              double acc = 0.0;
              for (int jj = 0; jj < s; ++jj) acc += T->b[jj] * rs[bi * s + jj][v * b->ncell + c];
              b->q[v * b->npad + p] = b->qn[v * b->npad + p] - dt * acc / vol;
            }
          }
    }
  }
  for (int i = 0; i < G->nblocks * s; ++i) free(rs[i]);
  free(rs);
  return st;
}

/* ------------------------------------------------------------------------ */
/* public entry points                                                      */
/* ------------------------------------------------------------------------ */
orc_grid* orc_create(int ndim, int nblocks, const orc_block_desc* desc, double gamma) {
  if ((ndim != 2 && ndim != 3) || nblocks <= 0 || !desc) return NULL;
  orc_grid* G = (orc_grid*)calloc(1, sizeof(orc_grid));
  if (!G) return NULL;
  G->ndim = ndim;
  G->nv = ndim + 2;
  G->nblocks = nblocks;
  G->gamma = gamma;
  G->b = (blk_t*)calloc((size_t)nblocks, sizeof(blk_t));
  if (!G->b) { free(G); return NULL; }
  for (int bi = 0; bi < nblocks; ++bi) {
    const orc_block_desc* d = &desc[bi];
    blk_t* b = &G->b[bi];
    b->ni = d->ni;
    b->nj = d->nj;
    b->nk = ndim == 3 ? d->nk : 1;
    if (b->ni <= 0 || b->nj <= 0 || b->nk <= 0) { orc_destroy(G); return NULL; }
    b->pi = b->ni + 4;
    b->pj = b->nj + 4;
    b->pk = ndim == 3 ? b->nk + 4 : 1;
    b->gk = ndim == 3 ? 2 : 0;
    b->npad = (i64)b->pi * b->pj * b->pk;
    b->ncell = (i64)b->ni * b->nj * b->nk;
    for (int a = 0; a < 3; ++a) {
      b->h[a] = d->h[a];
      b->origin[a] = d->origin[a];
    }
    memcpy(b->bc, d->bc, sizeof(b->bc));
    if (ndim == 3 && (d->x || d->y || d->z) && !(d->x && d->y && d->z)) {
      orc_destroy(G);
      return NULL;
    }
    if (d->x && d->y && (ndim == 2 || d->z)) {
      size_t nn = (size_t)(b->ni + 1) * (size_t)(b->nj + 1) * (size_t)(ndim == 3 ? b->nk + 1 : 1);
      b->xn = (double*)malloc(nn * sizeof(double));
      b->yn = (double*)malloc(nn * sizeof(double));
      if (!b->xn || !b->yn) { orc_destroy(G); return NULL; }
      memcpy(b->xn, d->x, nn * sizeof(double));
      memcpy(b->yn, d->y, nn * sizeof(double));
      if (ndim == 3) {
        b->zn = (double*)malloc(nn * sizeof(double));
        if (!b->zn) { orc_destroy(G); return NULL; }
        memcpy(b->zn, d->z, nn * sizeof(double));
      }
    }
    i64 nfmax = 0;
    for (int dd = 0; dd < ndim; ++dd) {
      i64 nf = (i64)(b->ni + (dd == 0)) * (b->nj + (dd == 1)) * (b->nk + (dd == 2));
      if (nf > nfmax) nfmax = nf;
    }
    b->nflux = nfmax;
    b->q = (double*)calloc((size_t)G->nv * (size_t)b->npad, sizeof(double));
    b->qn = (double*)calloc((size_t)G->nv * (size_t)b->npad, sizeof(double));
    b->res = (double*)calloc((size_t)G->nv * (size_t)b->ncell, sizeof(double));
    b->flux = (double*)calloc((size_t)G->nv * (size_t)nfmax, sizeof(double));
    if (!b->q || !b->qn || !b->res || !b->flux) { orc_destroy(G); return NULL; }
    G->ncells += b->ncell;
  }
  /* block links: in 2D opposite faces, same orientation; in 3D any face
   * pair whose transverse extents agree under the orientation */
  for (int bi = 0; bi < nblocks; ++bi)
    for (int f = 0; f < 2 * ndim; ++f) {
      const orc_bc* bc = &G->b[bi].bc[f];
      if (bc->kind < ORC_PERIODIC || bc->kind > ORC_NOSLIP) { orc_destroy(G); return NULL; }
      if (bc->kind != ORC_BLOCK) continue;
      int nb = bc->nbr_block;
      if (nb < 0 || nb >= nblocks || bc->nbr_face < 0 || bc->nbr_face >= 2 * ndim ||
          bc->orient < 0 || bc->orient > 7 ||
          (ndim == 2 && (bc->nbr_face != (f ^ 1) || bc->orient != 0))) {
        orc_destroy(G);
        return NULL;
      }
      int n1, n2, m1, m2;
      trans_ext(&G->b[bi], f / 2, &n1, &n2);
      trans_ext(&G->b[nb], bc->nbr_face / 2, &m1, &m2);
      if ((bc->orient & 1) ? (n1 != m2 || n2 != m1) : (n1 != m1 || n2 != m2)) {
        orc_destroy(G);
        return NULL;
      }
    }
  return G;
}

void orc_destroy(orc_grid* G) {
  if (!G) return;
  if (G->b) {
    for (int bi = 0; bi < G->nblocks; ++bi) {
      blk_t* b = &G->b[bi];
      free(b->xn); free(b->yn); free(b->zn); free(b->src);
      free(b->q); free(b->qn); free(b->res); free(b->flux);
    }
    free(G->b);
  }
  free(G);
}

int orc_set_state(orc_grid* G, const double* U) {
  const int nv = G->nv;
  i64 o = 0;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    for (int v = 0; v < nv; ++v)
      for (int k = 0; k < b->nk; ++k)
        for (int j = 0; j < b->nj; ++j)
          for (int i = 0; i < b->ni; ++i) b->q[v * b->npad + pidx(b, i, j, k)] = U[o++];
  }
  G->t = 0.0;
  G->steps = 0;
  G->dt_last = 0.0;
  G->have_first = 0;
  G->norm = G->norm_first = G->drop = 0.0;
  for (int v = 0; v < 5; ++v) G->norms[v] = 0.0;
  double mn;
  return orc_spectral_min(G, &mn);
}

void orc_get_state(const orc_grid* G, double* U) {
  const int nv = G->nv;
  i64 o = 0;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    const blk_t* b = &G->b[bi];
    for (int v = 0; v < nv; ++v)
      for (int k = 0; k < b->nk; ++k)
        for (int j = 0; j < b->nj; ++j)
          for (int i = 0; i < b->ni; ++i) U[o++] = b->q[v * b->npad + pidx(b, i, j, k)];
  }
}

/* viscosity parameters: mu >= 0; mu > 0 needs a 2D grid and Pr > 0.  The
 * time-step limit follows the viscosity of the latest call. */
static int use_viscosity(orc_grid* G, const orc_params* P) {
  if (!(P->mu >= 0.0) || !isfinite(P->mu)) return ORC_E_INVAL;
  if (P->mu > 0.0 && (G->ndim != 2 || !(P->prandtl > 0.0))) return ORC_E_INVAL;
  if (P->mu != G->mu || (P->mu > 0.0 && P->prandtl != G->prandtl)) {
    G->mu = P->mu;
    G->prandtl = P->prandtl;
    double mn;
    (void)orc_spectral_min(G, &mn);
  }
  return ORC_OK;
}

int orc_residual(orc_grid* G, const orc_params* P, double* R, double* norms, double* scale) {
  const int nv = G->nv;
  if (use_viscosity(G, P) != ORC_OK) return ORC_E_INVAL;
  double** scales = NULL;
  if (scale) {
    scales = (double**)malloc(sizeof(double*) * (size_t)G->nblocks);
    i64 o = 0;
    for (int bi = 0; bi < G->nblocks; ++bi) {
      scales[bi] = scale + o;
      o += (i64)nv * G->b[bi].ncell;
    }
  }
  residual_all(G, P, scales);
  free(scales);
  if (R) {
    i64 o = 0;
    for (int bi = 0; bi < G->nblocks; ++bi) {
      blk_t* b = &G->b[bi];
      memcpy(R + o, b->res, sizeof(double) * (size_t)nv * (size_t)b->ncell);
      o += (i64)nv * b->ncell;
    }
  }
  if (norms) {
    double comb;
    norms_of_residual(G, P, norms, &comb);
  }
  return ORC_OK;
}

void orc_get_info(const orc_grid* G, orc_info* info) {
  info->steps = G->steps;
  info->t = G->t;
  info->dt_last = G->dt_last;
  for (int v = 0; v < 5; ++v) info->norms[v] = G->norms[v];
  info->norm = G->norm;
  info->norm_first = G->norm_first;
  info->drop = G->drop;
  info->status = G->physical ? ORC_OK : ORC_E_NONPHYSICAL;
}

/* Advance up to nsteps steps.  dt = dt_fixed if positive, else CFL times the
 * spectral minimum of U^n; a positive t_end clamps the last step so that t
 * lands on t_end and no step starts at or after it.  After each step the new
 * state is checked (rho > 0, p > 0, finite) and its spectral minimum kept for
 * the next dt.  With drop_tol > 0 the run also ends after the first step whose
 * residual norm (from R(U^n)) is at most drop_tol times the first step's. */
int orc_run(orc_grid* G, const orc_params* P, long long nsteps, double drop_tol, orc_info* info,
            double* dt_hist) {
  if (P->rk != 0 && P->rk != 2 && P->rk != 3 && P->rk != 4 && P->rk != 103) return ORC_E_INVAL;
  if (use_viscosity(G, P) != ORC_OK) return ORC_E_INVAL;
  int status = G->physical ? ORC_OK : ORC_E_NONPHYSICAL;
  for (long long s = 0; s < nsteps && status == ORC_OK; ++s) {
    double dt = P->dt_fixed > 0.0 ? P->dt_fixed : P->cfl * G->raw_min;
    int last = 0;
    if (P->t_end > 0.0) {
      if (G->t >= P->t_end) break;
      if (dt >= P->t_end - G->t) {
        dt = P->t_end - G->t;
        last = 1;
      }
    }
    if (P->rk == 2 || P->rk == 4 || P->rk == 103) {
      tableau_t T;
      tableau_of(P->rk, &T);
      const int e = butcher_step(G, P, dt, &T);
      if (e != ORC_OK) {
        status = e;
        break;
      }
    } else {
      rk3_step(G, P, dt);
    }
    G->t = last ? P->t_end : G->t + dt;
    G->dt_last = dt;
    if (dt_hist) dt_hist[s] = dt;
    if (!G->have_first) {
      G->norm_first = G->norm;
      G->have_first = 1;
    }
    G->drop = G->norm_first > 0.0 ? G->norm / G->norm_first : 0.0;
    G->steps++;
    double mn;
    status = orc_spectral_min(G, &mn);
    if (drop_tol > 0.0 && G->drop <= drop_tol) break;
  }
  if (info) {
    orc_get_info(G, info);
    info->status = status;
  }
  return status;
}

/* Ghost values of the current state, laid out [block][face][layer g=1,2]
 * [var][t2][t1] with (t1, t2) = (j, k) on i-faces, (i, k) on j-faces and
 * (i, j) on k-faces. */
int orc_ghosts(orc_grid* G, double* out) {
  const int nd = G->ndim, nv = G->nv;
  i64 o = 0;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    for (int f = 0; f < 2 * nd; ++f) {
      int n1, n2;
      trans_ext(b, f / 2, &n1, &n2);
      for (int g = 1; g <= 2; ++g)
        for (int v = 0; v < nv; ++v)
          for (int t2 = 0; t2 < n2; ++t2)
            for (int t1 = 0; t1 < n1; ++t1) {
              double val[5];
              ghost_value(G, bi, f, g, t1, t2, val);
              out[o++] = val[v];
            }
    }
  }
  return ORC_OK;
}

int orc_face_flux(orc_grid* G, const orc_params* P, int block, int dir, int i, int j, int k,
                  double* F) {
  if (block < 0 || block >= G->nblocks || dir < 0 || dir >= G->ndim) return ORC_E_INVAL;
  fill_ghosts(G);
  face_flux_at(G, &G->b[block], P, dir, i, j, k, F);
  return ORC_OK;
}

int orc_viscous_flux(orc_grid* G, const orc_params* P, int block, int dir, int i, int j,
                     double* F) {
  if (block < 0 || block >= G->nblocks || dir < 0 || dir > 1 || G->ndim != 2) return ORC_E_INVAL;
  if (use_viscosity(G, P) != ORC_OK) return ORC_E_INVAL;
  fill_ghosts(G);
  viscous_flux_2d(G, block, P, dir, i, j, F);
  return ORC_OK;
}

void orc_metrics_2d(const orc_grid* G, int block, double* Sxi, double* Seta, double* vol) {
  const blk_t* b = &G->b[block];
  double S[3];
  for (int j = 0; j < b->nj; ++j)
    for (int i = 0; i <= b->ni; ++i) {
      face_vec(b, 2, 0, i, j, 0, S);
      Sxi[2 * ((i64)j * (b->ni + 1) + i)] = S[0];
      Sxi[2 * ((i64)j * (b->ni + 1) + i) + 1] = S[1];
    }
  for (int j = 0; j <= b->nj; ++j)
    for (int i = 0; i < b->ni; ++i) {
      face_vec(b, 2, 1, i, j, 0, S);
      Seta[2 * ((i64)j * b->ni + i)] = S[0];
      Seta[2 * ((i64)j * b->ni + i) + 1] = S[1];
    }
  for (int j = 0; j < b->nj; ++j)
    for (int i = 0; i < b->ni; ++i) vol[(i64)j * b->ni + i] = cell_vol(b, 2, i, j, 0);
}

void orc_metrics_3d(const orc_grid* G, int block, double* S, double* vol) {
  /* S: [dir][k][j][i][3] over each direction's (ni+e0)(nj+e1)(nk+e2) faces */
  const blk_t* b = &G->b[block];
  i64 o = 0;
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < b->nk + (d == 2); ++k)
      for (int j = 0; j < b->nj + (d == 1); ++j)
        for (int i = 0; i < b->ni + (d == 0); ++i) {
          face_vec(b, 3, d, i, j, k, S + 3 * o);
          ++o;
        }
  for (int k = 0; k < b->nk; ++k)
    for (int j = 0; j < b->nj; ++j)
      for (int i = 0; i < b->ni; ++i) vol[((i64)k * b->nj + j) * b->ni + i] = cell_vol(b, 3, i, j, k);
}

int orc_set_source(orc_grid* G, const double* S) {
  const int nv = G->nv;
  i64 o = 0;
  for (int bi = 0; bi < G->nblocks; ++bi) {
    blk_t* b = &G->b[bi];
    const size_t n = (size_t)nv * (size_t)b->ncell;
    if (!S) {
      free(b->src);
      b->src = NULL;
      continue;
    }
    if (!b->src) b->src = (double*)malloc(n * sizeof(double));
    if (!b->src) return ORC_E_INVAL;
    memcpy(b->src, S + o, n * sizeof(double));
    o += (i64)n;
  }
  return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the following runs (timing only: results do not depend on it) */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
