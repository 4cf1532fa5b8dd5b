/*
 * fv.h - C ABI of the MI355X (gfx950) explicit finite-volume Euler library.
 *
 * The library evaluates, on one GPU, the hot path of a cell-centred
 * finite-volume solver for the compressible Euler equations on structured
 * multi-block grids:
 *   - ghost-cell / boundary fill before every RK substep and block-to-block
 *     halo exchange (Sec. 4 workflow; Sec. 5 "ghost cell extrapolation on
 *     the GPU"; exchange between workers becomes on-device reads),
 *   - MUSCL extrapolation of the face states with limiter values
 *     (Sec. 5, Eq. (flux)),
 *   - an upwind numerical normal flux of the inviscid flux F_{i,n}
 *     (Sec. 2, flux definitions; Roe's solver is the reading taken),
 *   - the residual R = sum over the cell's faces of (F_{i,n} - F_{nu,n}) ds
 *     - |Omega| S_h (Sec. 3.1, Eq. (residual); the viscous part F_{nu,n} of
 *     Sec. 2 on 2D grids with mu > 0, the cell-averaged source S_h on grids
 *     created with a source buffer),
 *   - the explicit Runge-Kutta update |Omega| dU/dt + R = 0
 *     (Sec. 3.1, Eq. (spatial_residual); Sec. 3.2, Eq. (runge_kutta),
 *     taken as the three-stage strong-stability-preserving scheme),
 *   - the residual norm ("residual print", Sec. 4) and the CFL time step.
 *
 * Conventions
 *   - Status codes: 0 success, > 0 informational, < 0 error.  No C++
 *     exception crosses this interface.  fv_last_error() returns a detail
 *     string for the calling thread's last failing call.
 *   - The library never allocates device memory.  Device workspace and arena
 *     are supplied by the caller (e.g. PyTorch tensors) and must outlive the
 *     handle that uses them; the allocation-free path (fv_step_noalloc) uses
 *     a fixed static device array instead.  Every host array passed in is copied before the
 *     call returns; the caller keeps ownership.
 *   - Grids: structured blocks, uniform (spacing h) or curvilinear (node
 *     coordinates) in 2D and 3D; face area vectors and cell volumes of
 *     curvilinear cells come from the nodes (see fv_block_desc).
 *   - State layout (host or device): [block][var][k][j][i], i fastest,
 *     interior cells only, IEEE binary64.  2D: var = rho, rho*u, rho*v,
 *     rho*e_t (4 vars); 3D: rho, rho*u, rho*v, rho*w, rho*e_t (5 vars).
 *   - Units are the caller's, consistent with gamma.
 *   - A grid handle is single-threaded and works on the HIP stream given at
 *     creation.  fv_step / fv_solve / fv_residual block until their results
 *     are on the host.
 */
#ifndef FV_H
#define FV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  FV_OK = 0,
  FV_PENDING = 1,          /* fv_poll: request not finished yet */
  FV_E_INVAL = -1,         /* bad argument or descriptor */
  FV_E_NOMEM = -2,         /* workspace, arena or tile list too small, or a host
                              allocation (descriptor copy, serving thread) failed */
  FV_E_DEVICE = -3,        /* a HIP call failed */
  FV_E_NONPHYSICAL = -4,   /* rho <= 0, p <= 0 or a non-finite state value */
  FV_E_UNSUPPORTED = -5,   /* valid request this build does not provide */
  FV_E_BUSY = -6,          /* server queue full */
  FV_E_NOTFOUND = -7,      /* unknown ticket */
  FV_E_CANCELLED = -8      /* request cancelled before it finished */
};

/* boundary kinds.  Ghost rules (two ghost layers per face):
 *   PERIODIC  ghost = interior cell the same distance in from the opposite
 *             face of the same block
 *   BLOCK     ghost = interior cell of block nbr_block, the same distance in
 *             from its face nbr_face (1:1 points).  2D: nbr_face is the
 *             opposite face of the same direction, same orientation.  3D:
 *             any face, with the transverse indices mapped by orient (see
 *             fv_bc); the transverse extents must agree under that map
 *   INFLOW    ghost = conserved state of prim_in = (rho, u, v, w, p)
 *   EXTRAP    ghost = nearest interior cell (zeroth-order extrapolation)
 *   SLIPWALL  ghost layer g = interior cell g-1 from the wall with its
 *             momentum mirrored about the unit normal of that wall face;
 *             rho and rho*e_t copied
 *   NOSLIP    (2D) ghost layer g = interior cell g-1 from the wall with
 *             rho and p kept and the velocity 2 w - u, w = prim_in[1..3]
 *             the wall velocity (an adiabatic wall; a reading: the paper
 *             names no wall rule).  Grids with no-slip faces take the
 *             Navier-Stokes stage kernel.
 * PERIODIC, BLOCK, SLIPWALL and NOSLIP read two distinct cells across the
 * face, so the source block needs at least 2 cells along that direction
 * (FV_E_INVAL otherwise).  In 2D a corner ghost (outside both an i- and a
 * j-face; read only by the viscous flux) follows the i-face rule, then the
 * j-face rule of the block that rule lands in. */
enum { FV_BC_PERIODIC = 0, FV_BC_BLOCK = 1, FV_BC_INFLOW = 2, FV_BC_EXTRAP = 3, FV_BC_SLIPWALL = 4,
       FV_BC_NOSLIP = 5 };
enum { FV_IMIN = 0, FV_IMAX = 1, FV_JMIN = 2, FV_JMAX = 3, FV_KMIN = 4, FV_KMAX = 5 };

/* arithmetic of reconstruction + flux: FP64 throughout, or FP32 from the
 * face states through F.ds with the state, the residual sum, the RK update,
 * the norms and the time step kept in FP64 */
enum { FV_FP64 = 0, FV_FP32_FLUX = 1 };

/* MUSCL variants (Sec. 5, Eq. (flux)): minmod limiter values, no limiter
 * (Psi = 1), or first order (eps = 0) */
enum { FV_LIM_MINMOD = 0, FV_LIM_NONE = 1, FV_FIRST_ORDER = 2 };

/* fv_step_info.flags */
enum {
  FV_FLAG_NONPHYSICAL = 1,  /* the state after the last step is not physical */
  FV_FLAG_CONVERGED = 2,    /* residual drop reached drop_tol (fv_solve) */
  FV_FLAG_T_END = 4,        /* t reached t_end */
  FV_FLAG_STEP_LIMIT = 8    /* the step budget of the call was used up */
};

typedef struct fv_bc {
  int kind;          /* FV_BC_* */
  int nbr_block;     /* FV_BC_BLOCK: neighbour block index */
  int nbr_face;      /* FV_BC_BLOCK: neighbour face (FV_IMIN..FV_KMAX).  2D: the
                        opposite face (f ^ 1).  3D: any face (the multi-block
                        structured grids of Sec. 2: blocks meet face to face,
                        each in its own index frame) */
  int orient;        /* FV_BC_BLOCK, 3D: how the transverse indices (t1, t2) of
                        this face map onto (s1, s2) of the neighbour's face.
                        Transverse indices of a face normal to i, j, k are
                        (j, k), (i, k), (i, j).  Bit 0: s1 = t2, s2 = t1 (else
                        s1 = t1, s2 = t2); bit 1: then s1 -> m1 - 1 - s1; bit 2:
                        then s2 -> m2 - 1 - s2, (m1, m2) the neighbour face's
                        transverse sizes.  Ghost layer g (1, 2) copies the
                        neighbour's cell at depth g - 1 inside its face.  Must
                        be 0 in 2D.  A 3D grid with a link that is not
                        opposite-face and unoriented is stepped by the general
                        3D kernel. */
  double prim_in[5]; /* FV_BC_INFLOW: rho, u, v, w, p; FV_BC_NOSLIP: wall u, v, w
                        in prim_in[1..3] */
} fv_bc;

typedef struct fv_block_desc {
  int ni, nj, nk;          /* interior cells; nk = 1 in 2D */
  const double *x, *y, *z; /* node coordinates, i fastest, or all NULL (uniform
                              spacing h):
                              2D: x, y of (nj+1)*(ni+1) nodes, z NULL;
                              3D: x, y, z of (nk+1)*(nj+1)*(ni+1) nodes.
                              3D curvilinear cells (a reading of the paper's
                              face area ds, normal n and volume |Omega| for
                              hexahedra with bilinear faces): the area vector
                              of a face is half the cross product of its two
                              diagonals, oriented towards increasing index;
                              the volume is one third of the sum over the six
                              faces of (outward area vector . face centre), the
                              centre the mean of the face's four nodes.  Both
                              are exact for the trilinear cell.  Slip walls
                              mirror about the wall face's own normal. */
  double origin[3], h[3];  /* uniform spacing per direction */
  fv_bc face[6];           /* imin, imax, jmin, jmax, kmin, kmax */
} fv_block_desc;

typedef struct fv_grid_desc {
  int ndim;                     /* 2 or 3 */
  int nblocks;
  const fv_block_desc* blocks;
  double gamma;                 /* ratio of specific heats */
  int with_source;              /* 1: reserve a cell-averaged source S_h (Sec. 2,
                                   the source term; Sec. 3.1, Eq. (residual)),
                                   zero until fv_set_source; 0: none.  The
                                   server takes it with fv_submit_with_source;
                                   fv_step_noalloc refuses it
                                   (FV_E_UNSUPPORTED). */
} fv_grid_desc;

typedef struct fv_params {
  double cfl;          /* CFL number of the global time step */
  double dt_fixed;     /* > 0: use this time step instead of the CFL step */
  double t_end;        /* > 0: clamp the last step so that t lands on t_end */
  int precision;       /* FV_FP64 or FV_FP32_FLUX */
  int limiter;         /* FV_LIM_MINMOD, FV_LIM_NONE, FV_FIRST_ORDER */
  double eps, kappa;   /* MUSCL parameters of Eq. (flux) */
  double entropy_fix;  /* Harten's delta / c on the acoustic waves (0: off) */
  int rk;              /* explicit RK of Sec. 3.2, Eq. (runge_kutta):
                          3 (or 0): SSP-RK3 in Shu-Osher form;
                          2: the 2-stage second-order scheme, a21 = 1/2, b = (0, 1);
                          4: the 4-stage second-order scheme, a21 = 1/4, a32 = 1/3,
                             a43 = 1/2, b = (0, 0, 0, 1)
                          (the coefficients are a reading: the paper cites them).
                          Other values: FV_E_UNSUPPORTED.  The server and
                          fv_step_timed take 3 only. */
  double qref[5];      /* reference magnitudes of the combined residual norm
                          (0 entries count as 1) */
  double mu;           /* dynamic viscosity: > 0 adds the viscous normal flux
                          F_{nu,n} of Sec. 2 to Eq. (residual) (2D grids only;
                          FV_E_UNSUPPORTED in 3D).  Stokes's
                          hypothesis with constant mu; heat flux by Fourier's law
                          with k = mu c_p / prandtl, i.e. k grad T =
                          (mu/prandtl) gamma/(gamma-1) grad(p/rho); face gradients
                          by Green-Gauss over the face's diamond (two cell
                          centres, two face nodes).  The time-step limit gains
                          2 max(4/3, gamma/prandtl) (mu/rho) sum_d |S_d|^2/|Omega|. */
  double prandtl;      /* Prandtl number (> 0 when mu > 0) */
} fv_params;

typedef struct fv_step_info {
  long long steps;     /* steps taken since the last fv_set_state */
  double t;            /* simulated time */
  double dt_last;      /* time step of the last step */
  double norms[5];     /* RMS over cells of R_v/|Omega| at the last step's U^n */
  double norm;         /* sqrt(sum_v (norms_v / qref_v)^2) */
  double drop;         /* norm / norm of the first step after fv_set_state */
  int flags;           /* FV_FLAG_* */
} fv_step_info;

typedef struct fv_grid fv_grid;

/* Human-readable text of a status code (static storage). */
const char* fv_strerror(int status);
/* Detail of the calling thread's last failing call ("" if none). */
const char* fv_last_error(void);
/* Defaults: cfl 0.5, FP64, minmod, eps 1, kappa -1, entropy_fix 0.1, rk 3,
 * mu 0 (Euler), prandtl 0.72. */
void fv_default_params(fv_params* p);

/* Device bytes a grid needs (state buffers, node coordinates, descriptors,
 * tile list and reduction partials).  Returns 0 for an invalid descriptor. */
size_t fv_grid_workspace_bytes(const fv_grid_desc* desc, int precision);

/* Build a grid in the caller's device workspace (d_workspace, >= the bytes
 * above, 256-byte aligned) on the HIP stream hip_stream (NULL: the null
 * stream).  Validates the descriptor (FV_E_INVAL), copies node coordinates
 * and boundary data to the device, and lays out the tile work-list with the
 * tile shape the autotune table (or the default) gives for this grid. */
int fv_create_grid(const fv_grid_desc* desc, void* d_workspace, size_t bytes, void* hip_stream,
                   fv_grid** out);
int fv_destroy_grid(fv_grid* g);

/* Copy a conserved state in (U: host or device pointer per on_device), reset
 * t, the step count and the first-step norm, and compute the time-step
 * bound.  Returns FV_E_NONPHYSICAL (state kept) if a cell is not physical. */
int fv_set_state(fv_grid* g, const double* U, int on_device);
int fv_get_state(const fv_grid* g, double* U, int on_device);

/* Cell-averaged source S_h of Eq. (residual) (Sec. 3.1): body forces,
 * chemistry or a manufactured solution's forcing, in the state layout (host
 * or device per on_device); the residual of every later call is
 * R = sum_faces (F_{i,n} - F_{nu,n}) ds - |Omega| S_h.  S = NULL sets it to
 * zero.  FV_E_INVAL unless the grid was created with with_source = 1.  The
 * time-step bound does not depend on it. */
int fv_set_source(fv_grid* g, const double* S, int on_device);

/* Residual R(U) of the current state (Sec. 3.1, Eq. (residual), with the
 * source when the grid has one) after the ghost fill, in the state layout;
 * norms (may be NULL) receives the RMS of R_v/|Omega| per variable.  The
 * state is not changed. */
int fv_residual(fv_grid* g, const fv_params* p, double* R, int on_device, double norms[5]);

/* Ghost values the boundary rules give for the current state, laid out
 * [block][face][layer g = 1, 2][var][t2][t1], (t1, t2) = (j, k) on i-faces,
 * (i, k) on j-faces, (i, j) on k-faces, faces of a 2D grid: imin..jmax. */
size_t fv_ghost_count(const fv_grid* g);
int fv_ghosts(fv_grid* g, double* G, int on_device);

/* Advance nsteps steps of the scheme p->rk (SSP-RK3 by default; fewer if
 * t_end is reached or the state turns non-physical: then FV_E_NONPHYSICAL
 * and info->steps counts the completed steps).  The time step is dt_fixed, or cfl times the minimum
 * over cells of |Omega| / sum_d(|u . S_d| + c |S_d|) at U^n. */
int fv_step(fv_grid* g, const fv_params* p, int nsteps, fv_step_info* info);

/* Step until the residual drop (norm / first-step norm) is <= drop_tol, or
 * max_steps steps in this call, or t_end.  Chunked internally; the stop is
 * taken on the device at exactly the step where it holds. */
int fv_solve(fv_grid* g, const fv_params* p, double drop_tol, long long max_steps,
             fv_step_info* info);

/* Measurement variant of fv_step (SSP-RK3 only): the same kernels launched
 * one by one (no graph) with HIP events around each launch on the grid's
 * stream.  stage_ms[0..2] receives the summed device time of the three RK
 * stage kernels and stage_ms[3] that of the step-end reductions, over the
 * call. */
int fv_step_timed(fv_grid* g, const fv_params* p, int nsteps, fv_step_info* info,
                  double stage_ms[4]);

/* Time the candidate tile shapes of this grid's size class on the device,
 * keep the fastest for this grid and record it in the autotune table
 * (cache_path: JSON file, NULL: environment FV_AUTOTUNE_CACHE or none).
 * The state is saved and restored.  When the table already holds a shape for
 * this size class and precision, that shape is applied without timing. */
int fv_tune(fv_grid* g, const fv_params* p, const char* cache_path);

typedef struct fv_grid_stats {
  long long cells;        /* interior cells */
  long long tiles;        /* work-list entries */
  int tile_rows;          /* 2D: rows per tile; 3D: planes per tile */
  int tile_cols;          /* cells per tile row (i) */
  int tile_ny;            /* 3D: j-rows per tile (1 in 2D) */
  int launch_blocks;      /* persistent workgroups per stage launch */
  size_t workspace_bytes;
  double last_stage_ms[4];/* last timed launch of stage 1, 2, 3, finalize */
} fv_grid_stats;
int fv_grid_get_stats(const fv_grid* g, fv_grid_stats* out);

/* ---------------------------------------------------------------------- */
/* CPU-GPU heterogeneous stepping (Sec. 4 workflow, Sec. 6 model).         */
/* ---------------------------------------------------------------------- */
/* The residual and RK update of one 2D block shared by the GPU and host-core
 * workers, the paper's synchronous heterogeneous mode with a 1D domain
 * decomposition along i (Sec. 6): the GPU takes columns [0, split), the
 * host takes [split, ni), itself split by rows over cpu_workers threads.
 * Every RK substep: the two columns on each side of the cut are exchanged
 * (device-to-host and host-to-device copies on the handle's stream), both
 * workers then compute the substep at once, and all of them synchronize.
 * The step end combines the norms (RMS over every cell) and the time-step
 * bound (minimum over every cell) of both parts; the host then sets the
 * common time step.  Results are those of fv_step on the whole block (the
 * same formulas; the host's divisions and roots are the correctly rounded
 * IEEE ones).
 * The Euler and the Navier-Stokes solver (Sec. 8 runs both in this mode): a
 * viscosity (p->mu > 0) or a no-slip face runs the Navier-Stokes stage kernel
 * on the GPU part, and the host part forms the same viscous flux (diamond
 * gradients with the kernel's corner-ghost and ghost-centre rules).
 * Grids: 2D, one block, no source, i-faces neither periodic nor linked
 * (FV_E_UNSUPPORTED otherwise);
 * 2 <= split <= ni - 2 (FV_E_INVAL).  The workspace is device memory the
 * caller owns (>= fv_hetero_workspace_bytes); the host worker's arrays and
 * pinned exchange buffers are allocated by the handle and freed by
 * fv_hetero_destroy. */
typedef struct fv_hetero fv_hetero;
size_t fv_hetero_workspace_bytes(const fv_grid_desc* desc, int split);
int fv_hetero_create(const fv_grid_desc* desc, int split, int cpu_workers, void* d_workspace,
                     size_t bytes, void* hip_stream, fv_hetero** out);
/* whole-block state in the usual layout, host memory */
int fv_hetero_set_state(fv_hetero* h, const double* U);
int fv_hetero_get_state(fv_hetero* h, double* U);
/* nsteps steps of p->rk (2, 3 or 4; p->precision applies to the GPU part,
 * the host computes in FP64); times_ms (may be NULL) receives the summed
 * wall time of the GPU stage kernels [0] (events), of the host substeps [1],
 * of the exchanges with their synchronizations [2], and the whole call [3]. */
int fv_hetero_step(fv_hetero* h, const fv_params* p, int nsteps, fv_step_info* info,
                   double times_ms[4]);
int fv_hetero_destroy(fv_hetero* h);

/* ---------------------------------------------------------------------- */
/* Allocation-free stepping.                                                */
/* ---------------------------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fv_step_noalloc is fv_step without a grid handle or workspace.  d_U is the
 * caller's device state ([block][var][k][j][i], interior cells, FP64, 8-byte
 * aligned), advanced in place by nsteps steps of the scheme p->rk from t = 0,
 * with the same kernels, tile shapes and results as fv_create_grid +
 * fv_set_state + fv_step.  Every other buffer (block table, instance record,
 * tile list, reduction partials, node coordinates, the two RK stage buffers)
 * lives in one static device array of FV_NOALLOC_SCRATCH_BYTES per device,
 * held until the process ends; a grid that needs more is rejected with
 * FV_E_NOMEM before any device work (the 4 x 512 x 256 inlet grid needs about
 * 42 MB).  The call calls no hipMalloc/hipFree, launches the kernels one by
 * one (no graph) on hip_stream and returns when info is on the host.  All
 * calls of the process on one device share the array: they are serialized by
 * a lock and each waits for its own work, so they never overlap; work of
 * another call on the same device that reaches the array by other means
 * would race with it.  The info's t, steps and drop count from this call. */
#define FV_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t fv_noalloc_scratch_bytes(void);
int fv_step_noalloc(const fv_grid_desc* desc, double* d_U, const fv_params* p, int nsteps,
                    void* hip_stream, fv_step_info* info);

/* ---------------------------------------------------------------------- */
/* Batched execution and serving (continuous batching over one arena).     */
/* ---------------------------------------------------------------------- */
enum { FV_SERVER_DRYRUN = 1 };  /* fv_server_desc.flags: no device work at all;
                                   every resident instance "takes" one step per
                                   step slot and returns its initial state
                                   (tests the scheduling logic on any host) */

typedef struct fv_server_desc {
  void* d_arena;           /* caller's device memory for resident instances */
  size_t arena_bytes;
  void* hip_stream;        /* stream the server launches on */
  int max_instances;       /* resident slots (1..1024) */
  const char* autotune_cache; /* JSON autotune table or NULL */
  int precision;           /* FV_FP64 or FV_FP32_FLUX for every instance */
  int steps_per_launch;    /* RK steps per batched graph launch (0: 10) */
  int flags;               /* FV_SERVER_* */
} fv_server_desc;

typedef struct fv_server fv_server;

int fv_server_create(const fv_server_desc* desc, fv_server** out);
/* Queue a solve (thread-safe): grid, initial state (host), parameters,
 * stop rule (drop <= drop_tol or max_steps steps).  The descriptor and U0
 * are copied.  Any grid of the grid API: 2D Euler and Navier-Stokes (a
 * viscosity or a no-slip face), uniform and general 3D (curvilinear blocks,
 * oriented links); each kind of grid has its own tile list and stage kernel
 * in the batched launches.  A descriptor with with_source = 1 goes through
 * fv_submit_with_source (FV_E_INVAL here).  FV_E_NOMEM if the request can
 * never fit the arena or the server's tile list, or if its host copy
 * fails; FV_E_UNSUPPORTED for rk other than 3 (resident
 * instances share one stage sequence) or a viscosity on a 3D grid. */
int fv_submit(fv_server* s, const fv_grid_desc* desc, const double* U0, const fv_params* p,
              double drop_tol, long long max_steps, unsigned long long* ticket);
/* fv_submit for a grid with a cell-averaged source S_h of Eq. (residual)
 * (Sec. 3.1; the residual gains - |Omega| S_h): desc->with_source must be 1
 * (FV_E_INVAL otherwise); S_h is host memory in the state layout, copied
 * with U0 and held in the instance's arena region. */
int fv_submit_with_source(fv_server* s, const fv_grid_desc* desc, const double* U0,
                          const double* S_h, const fv_params* p, double drop_tol,
                          long long max_steps, unsigned long long* ticket);
/* FV_PENDING until done; then the final state (host, cap_doubles >= state
 * size) and its info, and the request's own status.  Thread-safe. */
int fv_poll(fv_server* s, unsigned long long ticket, double* U_out, size_t cap_doubles,
            fv_step_info* info);
int fv_cancel(fv_server* s, unsigned long long ticket);
/* Timestamps (seconds on the server's steady clock) of a request that
 * fv_poll has not yet collected: submission, admission (resident), and
 * completion (negative while not reached).  FV_E_NOTFOUND otherwise. */
int fv_request_times(fv_server* s, unsigned long long ticket, double times[3]);
/* Seconds on the server's steady clock (the clock of fv_request_times). */
double fv_server_clock(fv_server* s);
typedef struct fv_server_stats {
  long long submitted, admitted, completed, cancelled, failed;
  long long launches, cell_steps;
  int resident, queued;
  size_t arena_used, arena_peak;
} fv_server_stats;
int fv_server_get_stats(fv_server* s, fv_server_stats* out);
int fv_server_destroy(fv_server* s);

#ifdef __cplusplus
}
#endif
#endif /* FV_H */
