/*
 * Reference (oracle) interface of the plain FP64 CPU implementation of the
 * explicit finite-volume Euler residual and SSP-RK3 time update.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, by the package smoke
 * check and by the benchmark's CPU-baseline leg; never by the product path.
 * It shares no code, header, table or helper with the HIP library.
 */
#ifndef FV_ORACLE_H
#define FV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_BLOCK = 1, ORC_INFLOW = 2, ORC_EXTRAP = 3, ORC_SLIPWALL = 4,
       ORC_NOSLIP = 5 };
enum { ORC_MINMOD = 0, ORC_UNLIMITED = 1, ORC_FIRST_ORDER = 2 };
enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOMEM = -2, ORC_E_NONPHYSICAL = -4 };

typedef struct {
  int kind;        /* ORC_PERIODIC .. ORC_NOSLIP */
  int nbr_block;   /* ORC_BLOCK: neighbour block */
  int nbr_face;    /* ORC_BLOCK: neighbour face (2D: the opposite face; 3D: any face) */
  int orient;      /* ORC_BLOCK, 3D: how this face's transverse indices (t1, t2)
                      map onto the neighbour face's (t1', t2'): bit 0 swaps them,
                      bits 1 and 2 reverse t1' and t2'.  0 with the opposite
                      face is the plain 1:1 link. */
  double prim[5];  /* ORC_INFLOW: rho, u, v, w, p; ORC_NOSLIP: wall velocity in prim[1..3] */
} orc_bc;

typedef struct {
  int ni, nj, nk;        /* interior cells (nk = 1 in 2D) */
  const double *x, *y;   /* node coordinates, i fastest: 2D (nj+1)*(ni+1); 3D with z,
                            (nk+1)*(nj+1)*(ni+1); NULL: uniform */
  const double* z;       /* 3D node coordinates (curvilinear 3D blocks) */
  double origin[3], h[3];
  orc_bc bc[6];          /* imin, imax, jmin, jmax, kmin, kmax */
} orc_block_desc;

typedef struct {
  double cfl, dt_fixed, t_end;
  int limiter;
  double eps, kappa, entropy_fix;
  double qref[5];
  int rk;                /* 3 (or 0): SSP-RK3; 2, 4: the 2- and 4-stage second-order
                            schemes of Sec. 3.2 in Butcher form; 103: SSP-RK3 in
                            Butcher form (tests) */
  double mu;             /* dynamic viscosity (0: Euler); 2D only */
  double prandtl;        /* Prandtl number of the heat flux (mu > 0) */
} orc_params;

typedef struct {
  long long steps;
  double t, dt_last;
  double norms[5], norm, norm_first, drop;
  int status;
} orc_info;

typedef struct orc_grid orc_grid;

orc_grid* orc_create(int ndim, int nblocks, const orc_block_desc* blocks, double gamma);
void orc_destroy(orc_grid* g);
int orc_set_state(orc_grid* g, const double* U);      /* interior, [block][var][k][j][i] */
void orc_get_state(const orc_grid* g, double* U);
int orc_residual(orc_grid* g, const orc_params* p, double* R, double* norms, double* scale);
int orc_run(orc_grid* g, const orc_params* p, long long nsteps, double drop_tol,
            orc_info* info, double* dt_hist);
void orc_get_info(const orc_grid* g, orc_info* info);
int orc_ghosts(orc_grid* g, double* G);
int orc_spectral_min(orc_grid* g, double* raw_min);
int orc_face_flux(orc_grid* g, const orc_params* p, int block, int dir, int i, int j, int k,
                  double* F);
int orc_viscous_flux(orc_grid* g, const orc_params* p, int block, int dir, int i, int j,
                     double* F);
void orc_metrics_2d(const orc_grid* g, int block, double* Sxi, double* Seta, double* vol);
void orc_roe(const double* qL, const double* qR, const double* n, int nd, double gamma,
             double entropy_fix, int mode, double* out);
void orc_reconstruct(const double* q4, int limiter, double eps, double kappa,
                     double* qL, double* qR);
int orc_num_threads(void);
/* cell-averaged source S_h of Eq. (residual), [block][var][k][j][i] (NULL
 * removes it); the residual becomes sum_faces F ds - |Omega| S_h */
int orc_set_source(orc_grid* g, const double* S);
void orc_metrics_3d(const orc_grid* g, int block, double* S, double* vol);

#ifdef __cplusplus
}
#endif
#endif
