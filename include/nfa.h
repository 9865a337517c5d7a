/*
 * libnfa -- pressure projection of a cartesian-grid / VOF ship-wave solver
 * on one AMD Instinct MI355X (gfx950).
 *
 * Implements the projection of Dommermuth et al., "The numerical simulation
 * of ship waves using cartesian-grid and volume-of-fluid methods": the
 * second-order variable-coefficient Poisson equation of the Formulation
 * section (eq. pois; stage form eqs. poisson1 / poisson2) on a stretched
 * cartesian grid (Gridding section), with two-fluid coefficients from the
 * volume fraction (eq. density, Density Smoothing section), an immersed
 * body entered by fractional face areas with small cells merged (Enforcement
 * of Body Boundary Conditions, eqs. integral1-integral2), solved by
 * preconditioned conjugate gradients (Introduction).
 *
 * The library solves the positive semidefinite form  A' p = b'  where
 *   (A p)_c = sum_f T_f (p_c - p_nb(f)),   T_f = (open area_f * beta_f) / h_f,
 *   beta_f  = 2 / (rho_L + rho_R) inside, 1/rho_c on a boundary face,
 *   A' = P^T A P  (P copies a merge group's root value to its slaves),
 * i.e. minus the cell integral of div((1/rho) grad p), and
 *   b = -((D F~) + B) / dt,  F~_f = open area_f * u~_f,  B_c = v_body . S_c
 * (eq. integral2 with the no-flux hull condition, eq. bc2).
 *
 * Conventions
 *  - Arrays are contiguous, x fastest:  cells (nz,ny,nx); nodes
 *    (nz+1,ny+1,nx+1); x-faces (nz,ny,nx+1); y-faces (nz,ny+1,nx);
 *    z-faces (nz+1,ny,nx).  Pointers marked DEVICE are device memory of the
 *    current HIP device; HOST pointers are ordinary host memory.
 *  - Ownership: the caller owns every buffer it passes and keeps it alive
 *    until the call returns (or, for asynchronous calls, until the stream
 *    has passed it).  The operator's and the network's device memory is a
 *    caller-owned workspace (nfa_poisson_workspace_bytes,
 *    nfa_unet_workspace_bytes; the network's parameter state in caller arrays
 *    through nfa_unet_bind).  Grids and multigrid handles allocate their own
 *    when they are created or a body is set.  Nothing allocates device memory
 *    on the assemble / apply / rhs / solve path.
 *  - Streams: `nfa_stream` is a hipStream_t (NULL = default stream); work is
 *    ordered on it.  Calls marked ASYNC return before the device finishes.
 *  - Errors: a negative status means nothing was launched (argument errors)
 *    or a HIP call failed; nfa_last_error() gives a thread-local message.
 *    NFA_NOT_CONVERGED (> 0) is a warning: outputs are filled.
 *  - Handles are not thread-safe; use one per thread.
 */
#ifndef NFA_H
#define NFA_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int nfa_status;
#define NFA_OK 0
#define NFA_NOT_CONVERGED 1
#define NFA_ERR_INVALID (-1)
#define NFA_ERR_NOMEM (-2)
#define NFA_ERR_HIP (-3)
#define NFA_ERR_BREAKDOWN (-4)
#define NFA_ERR_NUMERIC (-5)

typedef struct nfa_grid_s* nfa_grid;
typedef struct nfa_poisson_s* nfa_poisson;
typedef void* nfa_stream; /* hipStream_t */

/* boundary flags, order -x,+x,-y,+y,-z,+z */
#define NFA_BC_NEUMANN 0   /* no flux (free slip wall, exit with zero data) */
#define NFA_BC_DIRICHLET 1 /* p = 0 on the boundary face (half-cell distance) */

/* element types */
#define NFA_F64 0
#define NFA_F32 1
#define NFA_BF16 2

/* Thread-local message of the last failing call (empty if none). */
const char* nfa_last_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int nfa_version(void);

/* nfa_stream_copy -- dst = src over `bytes` bytes with a plain streaming
 * kernel (16-byte non-temporal loads and stores, four in flight per lane).
 * Not a step of the method: the attainable HBM bandwidth that the rates of
 * the sweeps are set against.
 *   dst, src : DEVICE, 16-byte aligned, not overlapping; owned by the caller.
 *   bytes    : a multiple of 16 (0: nothing to do).
 * NFA_ERR_INVALID for a misaligned pointer or size, or a null pointer with
 * bytes > 0.  ASYNC on s. */
nfa_status nfa_stream_copy(void* dst, const void* src, size_t bytes, nfa_stream s);

/* nfa_stream_fill -- every 32-bit word of dst set to `value` over `bytes`
 * bytes with a plain streaming kernel (16-byte stores, four per lane).  Not a
 * step of the method: the attainable HBM write bandwidth, against which the
 * write-dominated network layers are set.
 *   dst   : DEVICE, 16-byte aligned; owned by the caller.
 *   bytes : a multiple of 16 (0: nothing to do).
 * NFA_ERR_INVALID for a misaligned pointer or size, or a null pointer with
 * bytes > 0.  ASYNC on s. */
nfa_status nfa_stream_fill(void* dst, unsigned value, size_t bytes, nfa_stream s);

/* ------------------------------------------------------------------ grid
 * nfa_grid_create -- stretched cartesian grid (Gridding section).
 *   nx, ny, nz : cells per axis, each >= 1.
 *   xf, yf, zf : HOST, nx+1 / ny+1 / nz+1 strictly increasing face
 *                coordinates (copied).
 *   bc         : HOST, 6 flags NFA_BC_* (copied).
 *   out        : receives the handle.
 * Computes the 1-D metrics (widths, centre distances) and sets "no body"
 * (every face open).  Allocates device memory.  Errors: NFA_ERR_INVALID on
 * non-increasing coordinates, bad sizes or flags; NFA_ERR_HIP.
 */
nfa_status nfa_grid_create(int nx, int ny, int nz, const double* xf, const double* yf,
                           const double* zf, const int* bc, nfa_grid* out);

/* nfa_grid_set_body -- immersed body from its signed distance (Enforcement
 * of Body Boundary Conditions section: psi > 0 in the fluid; fractional
 * areas; cells with cut volume below `theta` merged with the neighbour along
 * the steepest gradient of psi).
 *   psi_nodes : DEVICE double, node array; NULL removes the body.
 *   theta     : merge threshold in [0,1) (0.25 in the paper).
 *   samples   : S >= 1 sub-samples per face edge / cell edge (8).
 * Face fractions = share of S*S midpoint samples of the bilinear
 * interpolant that are > 0; cell fractions likewise with S^3 trilinear
 * samples.  Cells with fraction 0 or without an open coupling become
 * inactive (no unknown).  Synchronous (merge groups are resolved on the
 * host).  A new body leaves every operator of the grid stale: until it is
 * assembled again, nfa_poisson_apply, _solve, _residual, _project,
 * nfa_poisson_velocity, the learned and multigrid preconditioners return
 * NFA_ERR_INVALID.  Errors: NFA_ERR_INVALID, NFA_ERR_HIP.
 */
/* nfa_stretch_axis -- face coordinates of one stretched axis (Gridding
 * section, eq. grid): the n + 1 nodes x_0 = a < ... < x_n = b that solve
 * (w x_xi)_xi = 0 in its conservative discrete form
 *   w(m_{i+1/2}) (x_{i+1} - x_i) = w(m_{i-1/2}) (x_i - x_{i-1}),
 * m the midpoints, by Picard iteration from uniform nodes (weights frozen at
 * the current midpoints, the tridiagonal system solved exactly) until no
 * node moves by more than tol (b - a).  The weight is levels[0] before the
 * first transition zone, the section's cosine transition
 *   w = (w0 - w1)/2 (1 + cos(pi (x - x0)/(x1 - x0))) + w1
 * from levels[k] to levels[k+1] across zone k = [zones[2k], zones[2k+1]],
 * and levels[k+1] after it; a large weight clusters nodes (the spacing is
 * inversely proportional to w).
 *   levels : HOST, nzones + 1 finite weights > 0.
 *   zones  : HOST, 2 nzones coordinates, increasing, not overlapping.
 *   nodes  : HOST out, n + 1 doubles (pass them to nfa_grid_create).
 *   iterations : HOST out, sweeps taken.
 * Runs on the host (no device work).  Returns NFA_OK, NFA_NOT_CONVERGED
 * after max_iter sweeps (nodes filled with the last iterate), or
 * NFA_ERR_INVALID. */
nfa_status nfa_stretch_axis(double a, double b, int n, int nzones, const double* levels,
                            const double* zones, double tol, int max_iter, double* nodes,
                            int* iterations);

/* nfa_panels_psi -- signed distance psi of a triangulated body at the grid
 * nodes (Enforcement of Body Boundary Conditions section): the least
 * distance to the panels (closest point inside a panel, on an edge or at a
 * vertex), negative inside the body and positive outside, inside told by
 * Gauss's theorem on the solid angle the panels subtend (4 pi inside, 0
 * outside a closed surface; a node outside the panels' bounding box is
 * outside).  FP64.
 *   panels : DEVICE double, m panels of 9 values: vertices a, b, c as
 *            (x, y, z); a closed surface, consistently oriented.
 *   psi    : DEVICE double, node array [nz+1][ny+1][nx+1] (output; feed it
 *            to nfa_grid_set_body).
 * Allocates and frees its work memory (the Morton-sorted panels, 72 bytes a
 * panel, and their bounding boxes); synchronous.  Errors: NFA_ERR_INVALID
 * (NULL, m < 1 or m > 2^30), NFA_ERR_HIP. */
nfa_status nfa_panels_psi(nfa_grid g, const double* panels, long long m, double* psi, nfa_stream s);

/* nfa_panels_psi_noalloc -- nfa_panels_psi for callers that cannot allocate
 * device memory (serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same result, bit for bit, with the work memory in a
 * static device array of 4.6 MiB that each GPU the library runs on holds
 * until the process ends.  Calls no hipMalloc or hipFree.
 *   m : 1 <= m <= 65536 panels; more returns NFA_ERR_INVALID before any
 *       device work.  Other arguments as nfa_panels_psi.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  Synchronous (the panels are sorted on the host
 * as in nfa_panels_psi).  Errors: NFA_ERR_INVALID, NFA_ERR_HIP. */
nfa_status nfa_panels_psi_noalloc(nfa_grid g, const double* panels, long long m, double* psi, nfa_stream s);

nfa_status nfa_grid_set_body(nfa_grid g, const double* psi_nodes, double theta, int samples,
                             nfa_stream s);

typedef struct {
  int nx, ny, nz;
  long long cells, active, reduced; /* reduced = number of unknowns */
  int groups, slaves;               /* merge groups and merged (slave) cells */
  int all_neumann;                  /* 1: singular system, zero-mean gauge */
} nfa_grid_info;
nfa_status nfa_grid_get_info(nfa_grid g, nfa_grid_info* info);

/* what to export from a grid (DEVICE destination, natural layout) */
#define NFA_EXPORT_FRAC_X 1  /* double, x-faces */
#define NFA_EXPORT_FRAC_Y 2  /* double, y-faces */
#define NFA_EXPORT_FRAC_Z 3  /* double, z-faces */
#define NFA_EXPORT_VFRAC 4   /* double, cells */
#define NFA_EXPORT_OPEN_X 5  /* double, x-faces: open area */
#define NFA_EXPORT_OPEN_Y 6
#define NFA_EXPORT_OPEN_Z 7
#define NFA_EXPORT_ACTIVE 8  /* uint8, cells */
#define NFA_EXPORT_ROOT 9    /* int32, cells: merge root, -1 inactive */
#define NFA_EXPORT_REDUCED 10 /* uint8, cells: 1 where an unknown lives */
nfa_status nfa_grid_export(nfa_grid g, int what, void* dst, nfa_stream s); /* ASYNC */
void nfa_grid_destroy(nfa_grid g);

/* --------------------------------------------------------------- poisson */
typedef struct {
  double rho_liquid; /* rho of water (phi = 1), e.g. 1000 */
  double rho_gas;    /* rho of air (phi = 0), e.g. 1.2 */
  int smooth;        /* 1: (1/4,1/2,1/4) smoothing along x, y, z */
  int phi_dtype;     /* NFA_F64 or NFA_F32 */
} nfa_assemble_params;

/* nfa_poisson_workspace_bytes -- bytes of device workspace an operator on
 * grid g needs: its coefficients in FP64 and FP32 (3 face arrays and the
 * Jacobi inverse diagonal), the density, the work vectors of the FP64 and
 * FP32 solvers, reduction partials and the residual history (about 150 bytes
 * per cell: eleven FP64 and nine FP32 cell arrays and the face arrays).  0 for
 * a NULL grid. */
size_t nfa_poisson_workspace_bytes(nfa_grid g);

/* nfa_poisson_create -- operator + solver state on grid g (the grid must
 * outlive it; set the body first).
 *   workspace : DEVICE, 256-byte aligned, ws_bytes >= nfa_poisson_workspace_bytes(g),
 *               owned by the caller (a torch tensor, say) and kept alive and
 *               untouched while the operator exists; every device buffer of the
 *               operator and its solvers is a slice of it, so assemble, apply,
 *               rhs, project and solve never allocate device memory.  NULL:
 *               the library allocates the same buffers itself, here.
 * The handle itself, two pinned host scalars and two HIP events are the
 * library's.  Errors: NFA_ERR_NOMEM (workspace shorter than needed; nothing is
 * created), NFA_ERR_INVALID (misaligned workspace, grid too wide), NFA_ERR_HIP. */
nfa_status nfa_poisson_create(nfa_grid g, void* workspace, size_t ws_bytes, nfa_poisson* out);

/* nfa_poisson_assemble -- coefficients for one projection (eq. density,
 * Density Smoothing, eq. integral2): rho = rho_g + (rho_l - rho_g)
 * clip(phi,0,1), optional smoothing, T_f on every face in FP64 and FP32, the
 * Jacobi inverse diagonal of the merged operator.
 *   phi : DEVICE, cells, dtype p->phi_dtype.   ASYNC. */
nfa_status nfa_poisson_assemble(nfa_poisson op, const void* phi, const nfa_assemble_params* p,
                                nfa_stream s);

/* nfa_poisson_apply -- y = A' x = P^T A P x (eqs. pois / integral2, merged).
 *   x, y : DEVICE, cells, dtype NFA_F64 (FP64 coefficients) or NFA_F32 (FP32
 *          coefficients).  x is read only (slave entries are ignored: P takes
 *          each group's root value); y has 0 on slaves and inactive cells.
 *   x and y must not overlap.  ASYNC. */
nfa_status nfa_poisson_apply(nfa_poisson op, const void* x, void* y, int dtype, nfa_stream s);

/* nfa_poisson_rhs -- b' = P^T b, b = -((D F~) + B)/dt (eq. integral2 with
 * u~ = u^k + dt R of eq. poisson1, and the body flux of eq. bc2), zero mean
 * over the unknowns when every boundary is Neumann.
 *   u, v, w  : DEVICE double on x-, y-, z-faces (provisional velocity).
 *   dt       : time step > 0.
 *   body_vel : HOST, 3 doubles, body velocity in the body-fixed frame.
 *   b        : DEVICE double, cells (output).   ASYNC. */
nfa_status nfa_poisson_rhs(nfa_poisson op, const double* u, const double* v, const double* w,
                           double dt, const double* body_vel, double* b, nfa_stream s);

/* nfa_poisson_project -- face fluxes after projection (eq. runge1 in flux
 * form): F_f = open area_f u~_f - dt T_f (p_+ - p_-), p = 0 beyond a
 * Dirichlet face.  p: DEVICE double cells (slaves take their root's value).
 * fu, fv, fw: DEVICE double face arrays (outputs).  ASYNC. */
nfa_status nfa_poisson_project(nfa_poisson op, const double* u, const double* v, const double* w,
                               const double* p, double dt, double* fu, double* fv, double* fw,
                               nfa_stream s);

/* nfa_poisson_divergence -- P^T (D F + B): discrete conservation per merged
 * cell (eq. diverge plus the body flux).  div: DEVICE double cells.  ASYNC. */
nfa_status nfa_poisson_divergence(nfa_poisson op, const double* fu, const double* fv,
                                  const double* fw, const double* body_vel, double* div,
                                  nfa_stream s);

/* preconditioners and precisions */
#define NFA_PC_JACOBI 1
#define NFA_PC_UNET 2
#define NFA_PC_TEST_SABOTAGE 3 /* test hook: preconditioner replaced by a fixed
                                  unrelated field, to exercise the fallback */
#define NFA_PC_JACOBI_FCG 4    /* flexible CG driver with the Jacobi preconditioner
                                  (reference run of the flexible path) */
#define NFA_PC_MG 5            /* aggregation multigrid V-cycle (opts->mg) */
#define NFA_PREC_F64 0   /* FP64 Jacobi-PCG */
#define NFA_PREC_MIXED 1 /* FP32 CG recurrence, FP64 solution and residual
                            replacement (the FP64 residual decides) */

typedef struct {
  double tol;            /* FP64 true relative residual ||b'-A'x||/||b'|| */
  int max_iters;         /* total (inner) iterations */
  int precond;           /* NFA_PC_* */
  int precision;         /* NFA_PREC_* */
  double replace_drop;   /* mixed: FP64 residual replacement each time the FP32
                            recursive residual has dropped by this factor (0.1);
                            CG goes on with the same direction and its own beta,
                            so the iteration count stays near FP64's */
  int fcg_m;             /* flexible CG truncation; 1 (FCG(1)) is supported */
  double fallback_ratio; /* switch to Jacobi-PCG when the mean reduction per
                            iteration over a window exceeds this (0.99) */
  int fallback_window;   /* window length in iterations (10) */
  int warm_start;        /* 1: x holds the initial guess */
  int check_every;       /* iterations between host polls of ||r|| (at most 2
                            with NFA_PC_MG) */
  void* unet;            /* nfa_unet handle when precond == NFA_PC_UNET */
  double* history;       /* optional HOST buffer of ||r_k||/||b'|| (inner) */
  int history_cap;
  void* mg;              /* nfa_mg handle when precond == NFA_PC_MG */
} nfa_solve_opts;

typedef struct {
  int iterations;     /* CG iterations */
  int outer;          /* FP64 true-residual evaluations (residual replacements) */
  int fallback;       /* 1: switched to Jacobi-PCG */
  int history_len;    /* entries written to opts->history */
  double relres;      /* final FP64 true relative residual */
  double ms;          /* wall time of the solve on the stream */
} nfa_solve_info;

/* Fills opts with defaults: tol 1e-8, Jacobi, FP64, replace_drop 0.1,
 * fallback 0.99 over 10 iterations, check_every 16. */
void nfa_solve_opts_default(nfa_solve_opts* opts);

/* ------------------------------------------------------------------------
 * Aggregation multigrid preconditioner (the paper names PCG and no
 * preconditioner; Jacobi is the default, this the stronger option).
 * Levels: 0 = A' over the reduced unknowns; l+1 = the Galerkin product
 * P^T A_l P with P the piecewise-constant prolongation from blocks of
 * 2 x 2 x 2 cells (an unknown of level 0 belongs to the block of its cell;
 * level 1 is assembled from the faces, merge groups included, and drops
 * couplings to blocks more than one apart while keeping their diagonal
 * terms); at least one coarsening; the coarsest level (at most 600 cells)
 * solved with a dense inverse (empty rows identity; c v v^T added when
 * every boundary is Neumann).  V-cycle in FP32: damped Jacobi (0.9), one
 * sweep before and one after the coarse correction -- symmetric.  Levels
 * >= 1 are held in FP32 as (D^-1, +x, +y, +z couplings) per cell plus a
 * side list of the rows that merges couple beyond the 7 points; the levels
 * from the first with at most the "tail" cell count (nfa_mg_set_tail) down
 * to the coarsest run in a single workgroup.
 * ------------------------------------------------------------------------ */
typedef struct nfa_mg_s* nfa_mg;
/* nfa_mg_create -- allocates the hierarchy of op's grid (op must outlive it):
 * per coarse cell 27 FP64 stencil entries, a float4 and two FP32 vectors
 * (about 2.5 GB per 10^7 cells of level 1), side lists sized for the grid's
 * current merge set (at most 12 rows per merged cell, a bound its rows never
 * exceed), and the merged rows' correction-term lists of the grid's current
 * body (16 bytes a term, a few per merged cell; the roots they need are
 * gathered on the device).  Set the body first; a handle serves that body
 * only.  Errors: NFA_ERR_INVALID (a single-cell grid), NFA_ERR_HIP. */
nfa_status nfa_mg_create(nfa_poisson op, nfa_mg* out);
void nfa_mg_destroy(nfa_mg mg);
/* nfa_mg_setup -- builds every level from op's current FP64 coefficients
 * (call after each nfa_poisson_assemble; nfa_poisson_solve with NFA_PC_MG
 * calls it when the operator has changed).  Synchronous (the side lists
 * are scanned and the coarsest inverse formed on the host).  Allocates no
 * device memory.  Errors: NFA_ERR_INVALID (not assembled, or the grid's body
 * set after the handle was created), NFA_ERR_NUMERIC (coarsest matrix not
 * positive definite), NFA_ERR_HIP. */
nfa_status nfa_mg_setup(nfa_mg mg, nfa_stream s);
/* nfa_mg_set_tail -- the single-workgroup part of the cycle starts at the
 * first level with at most max_cells cells whose two vectors and float4
 * cycle storage (with those of every coarser level) fit in 64 KiB of LDS;
 * 0: only the coarsest level;
 * < 0: the default, 1024.  Changes no result beyond FP32 rounding order. */
nfa_status nfa_mg_set_tail(nfa_mg mg, int max_cells);
/* nfa_mg_apply -- z = V(r), one V-cycle; r, z: DEVICE float cells (r zero
 * off the reduced unknowns; z's slaves take their root's value).  ASYNC. */
nfa_status nfa_mg_apply(nfa_mg mg, const float* r, float* z, nfa_stream s);
/* nfa_mg_info -- number of levels and, if dims is not NULL, (nz, ny, nx) of
 * each level (HOST, 3 * levels ints, at most 48). */
nfa_status nfa_mg_info(nfa_mg mg, int* levels, int* dims);
/* nfa_mg_set_params -- omega: damping of the Jacobi sweeps (0 < omega < 1,
 * default 0.9); alpha: scale of every coarse-grid correction, z += alpha P z_c
 * (0 < alpha < 2, default 1; any such alpha keeps the cycle symmetric
 * positive definite).  Errors: NFA_ERR_INVALID. */
nfa_status nfa_mg_set_params(nfa_mg mg, double omega, double alpha);
/* nfa_mg_set_coef -- the precision in which the cycle's level-0 sweeps read
 * the face coefficients and D^-1: NFA_F32 (the operator's FP32 copies) or
 * NFA_BF16 (those rounded to BF16, nearest even; made at set-up, half the
 * bytes; the first call asking for them allocates their 8 bytes per cell).
 * The operator of the CG itself is unaffected.  Takes effect at the next
 * set-up.  Errors: NFA_ERR_INVALID, NFA_ERR_HIP. */
nfa_status nfa_mg_set_coef(nfa_mg mg, int dtype);
/* nfa_mg_side_rows -- rows of level >= 1 (below the coarsest) held in the
 * side list by the last set-up (couplings beyond the 7 points). */
nfa_status nfa_mg_side_rows(nfa_mg mg, int level, int* rows);
/* nfa_mg_export -- level >= 1's FP64 stencil, 27 x n doubles (entry
 * o = (dz+1) 9 + (dy+1) 3 + (dx+1) of cell c at [o n + c]) into DEVICE dst.
 * ASYNC. */
nfa_status nfa_mg_export(nfa_mg mg, int level, double* dst, nfa_stream s);

/* nfa_poisson_solve -- x = A'^-1 b' by preconditioned CG (Introduction:
 * "preconditioned conjugate-gradient"; Jacobi by default).
 *   b : DEVICE double cells (as produced by nfa_poisson_rhs).
 *   x : DEVICE double cells: initial guess if warm_start, else overwritten;
 *       on return the solution with slaves = root value, inactive = 0 and,
 *       if every boundary is Neumann, zero mean over the unknowns.
 * The recursive residual is polled every check_every iterations; on
 * convergence the true FP64 residual decides (restart if above tol).
 * Synchronous.  Returns NFA_OK, NFA_NOT_CONVERGED (info filled), or an
 * error (NFA_ERR_NUMERIC on NaN/Inf). */
nfa_status nfa_poisson_solve(nfa_poisson op, const double* b, double* x, const nfa_solve_opts* opts,
                             nfa_stream s, nfa_solve_info* info);

/* Timing of the operator sweeps inside solves.  nfa_poisson_profile(op, 1)
 * brackets the first 4096 timed launches of each later solve (sweep A of
 * every iteration; with NFA_PC_MG also the fused level-0 down and up sweeps
 * of each V-cycle; with NFA_PC_UNET each network application) with HIP events on the solve's stream (creating the
 * events here, not in the solve) and resets the counters;
 * nfa_poisson_profile(op, 0) stops.  Only launches of iterations that ran
 * are counted. */
#define NFA_PROF_MG_DOWN 2
#define NFA_PROF_MG_UP 3
#define NFA_PROF_F32_FLEX 4 /* sweep A of the flexible (FCG) FP32 iteration */
#define NFA_PROF_UNET 5     /* one application of the learned preconditioner */
#define NFA_PROF_F64_X2 6   /* FP64 Jacobi-PCG sweep A applying two owed x steps */
#define NFA_PROF_F32_X2 7   /* FP32 Jacobi-PCG sweep A applying two owed x steps */
typedef struct {
  long long launches; /* stencil launches timed */
  double ms;          /* their summed duration */
  long long cells;    /* cells swept per launch */
} nfa_kernel_stats;
nfa_status nfa_poisson_profile(nfa_poisson op, int enable);
/* dtype NFA_F64 or NFA_F32: the Jacobi-PCG sweep A of that precision that
 * leaves x alone (every other iteration); NFA_PROF_F64_X2 / NFA_PROF_F32_X2:
 * the one in between, which applies the two owed x steps (Jacobi-PCG defers
 * the x update over two iterations); NFA_PROF_F32_FLEX: the flexible FP32
 * sweep A (x updated every iteration); NFA_PROF_MG_DOWN /
 * NFA_PROF_MG_UP: the V-cycle's fused level-0 sweeps (FP32); NFA_PROF_UNET:
 * whole applications of the learned preconditioner.  Synchronous. */
nfa_status nfa_poisson_profile_read(nfa_poisson op, int dtype, nfa_kernel_stats* out);

/* nfa_poisson_residual -- r = b' - A'x in FP64 (the true residual that
 * decides convergence); x is read as P x (slaves take their root's value).
 *   b, x, r : DEVICE double cells; r may not alias x.
 *   rr      : HOST out, ||r||^2 over the unknowns (NULL: not computed).
 * Synchronous when rr is given, else ASYNC. */
nfa_status nfa_poisson_residual(nfa_poisson op, const double* b, const double* x, double* r, double* rr,
                                nfa_stream s);

/* what to export from an operator (DEVICE destination, natural layout) */
#define NFA_EXPORT_RHO 20    /* double cells */
#define NFA_EXPORT_TX 21     /* double x-faces */
#define NFA_EXPORT_TY 22     /* double y-faces */
#define NFA_EXPORT_TZ 23     /* double z-faces */
#define NFA_EXPORT_DINV 24   /* double cells */
#define NFA_EXPORT_TX32 25   /* float x-faces */
#define NFA_EXPORT_TY32 26   /* float y-faces */
#define NFA_EXPORT_TZ32 27   /* float z-faces */
#define NFA_EXPORT_DINV32 28 /* float cells */
nfa_status nfa_poisson_export(nfa_poisson op, int what, void* dst, nfa_stream s); /* ASYNC */
void nfa_poisson_destroy(nfa_poisson op);

/* ------------------------------------------------------------------------
 * The Runge-Kutta projection cycle around the solve (Numerical Time
 * Integration, eqs. poisson1, runge1, poisson2, runge2).  Velocities live on
 * faces: x-faces [nz][ny][nx+1], y-faces [nz][ny+1][nx], z-faces
 * [nz+1][ny][nx], DEVICE doubles.
 * ------------------------------------------------------------------------ */

/* nfa_poisson_velocity -- velocity form of eqs. runge1 / runge2 on every face:
 *   u = scale * (u~ - dt * (g * (p+ - p-))),   g = beta_f / h_f,
 * beta_f = 2/(rho_L + rho_R) inside and 1/rho_c with the half width on a
 * Dirichlet boundary face (p = 0 beyond it), with rho of the last assembly;
 * g = 0 on Neumann boundary faces and on closed faces (zero open area), which
 * keep scale * u~.
 *   ut_x, ut_y, ut_z : DEVICE provisional velocity (may alias the outputs).
 *   p                : DEVICE double cells; read as P p (slaves take their
 *                      root's value).
 *   dt > 0; scale finite (1 for stage 1, 1/2 for stage 2).
 *   u_x, u_y, u_z    : DEVICE outputs.   ASYNC.
 * Errors: NFA_ERR_INVALID (NULL, not assembled, dt <= 0). */
nfa_status nfa_poisson_velocity(nfa_poisson op, const double* ut_x, const double* ut_y,
                                const double* ut_z, const double* p, double dt, double scale,
                                double* u_x, double* u_y, double* u_z, nfa_stream s);

/* nfa_poisson_rhs_cells -- nfa_poisson_rhs with a body velocity that varies
 * from cell to cell (the integral of v* . n over the body surface in eq.
 * integral2, for rotating or deforming bodies): B_c = v_c . S_c.
 *   vbx, vby, vbz : DEVICE double cells, body velocity per cell (read only on
 *                   cells the body cuts).  Other arguments as nfa_poisson_rhs.
 * ASYNC. */
nfa_status nfa_poisson_rhs_cells(nfa_poisson op, const double* u, const double* v,
                                 const double* w, double dt, const double* vbx, const double* vby,
                                 const double* vbz, double* b, nfa_stream s);

/* nfa_exit_velocity -- the exit condition of the Radiation Conditions section
 * (eqs. orlanski, exit): on the outflow plane (the +x boundary x-faces),
 *   ut_x = u_e - ((uc dt) / dx) (u_e - u_i)
 * with u_e, u_i the x-velocities of uk_x on the exit face and one cell inward
 * and dx the width of the last cell: the upwind step of du/dt + uc du/dx = 0.
 * The result is the exit face's provisional velocity; its flux enters the
 * right-hand side through nfa_poisson_rhs like any face flux, the face being a
 * Neumann face of the pressure.  Only the exit plane of ut_x is written.
 *   uk_x, ut_x : DEVICE double x-faces [nz][ny][nx+1] (may alias).
 *   0 <= uc dt <= dx (Courant number at most 1), dt > 0, nx >= 2.   ASYNC. */
nfa_status nfa_exit_velocity(nfa_grid g, const double* uk_x, double uc, double dt, double* ut_x,
                             nfa_stream s);

/* nfa_faces_combine -- out = (a + b) + s * c on n DEVICE doubles, or a + s * c
 * when b is NULL: the provisional fields u~1 = u^k + dt R and
 * u~2 = (u* + u^k) + dt R.  out may alias a or b.  ASYNC. */
nfa_status nfa_faces_combine(long long n, const double* a, const double* b, double s,
                             const double* c, double* out, nfa_stream st);

typedef struct {
  double dt;                 /* time step > 0 */
  double body_vel[3];        /* body velocity (body-fixed frame): stage 1 uses v,
                                stage 2 the flux of 2v (u~2 sums two fields) */
  nfa_assemble_params rho;   /* densities, smoothing, dtype of phi_k and phi_star */
} nfa_rk2_params;

/* nfa_rk2_cycle -- one cycle: assemble with phi_k; u~1 = u^k + dt R; solve
 * for P*; u* = u~1 - dt beta grad P*; assemble with phi_star (the advected
 * volume fraction, an input); u~2 = (u* + u^k) + dt R; solve for P;
 * u^{k+1} = (u~2 - dt beta grad P) / 2.
 *   phi_k, phi_star : DEVICE cells of rho->phi_dtype.
 *   uk, R           : three DEVICE face arrays each (x, y, z faces).
 *   ut              : three DEVICE face arrays of workspace (caller-owned).
 *   ustar, unext    : three DEVICE face arrays each, outputs u* and u^{k+1}.
 *   pstar, p        : DEVICE double cells, outputs P* and P (also the warm
 *                     starts when opts->warm_start).
 *   opts            : solve options of both stages.
 *   info            : HOST, two entries (stage 1, stage 2).
 * Leaves the operator assembled with phi_star.  Synchronous.  Returns the
 * worse of the two solves' statuses (NFA_NOT_CONVERGED is a warning) or the
 * first error. */
nfa_status nfa_rk2_cycle(nfa_poisson op, const void* phi_k, const void* phi_star,
                         const nfa_rk2_params* prm, const double* const* uk, const double* const* R,
                         double* const* ut, double* const* ustar, double* pstar, double* p,
                         double* const* unext, const nfa_solve_opts* opts, nfa_stream s,
                         nfa_solve_info* info);

/* ------------------------------------------------------------------------
 * Split VOF advection of the water fraction (Interface reconstruction and
 * advection section: eq. vof advanced by three one-directional sweeps, the
 * flux correction that restores eq. diverge cell by cell, piecewise-planar
 * interfaces).  Fractions are DEVICE double cells; u, v, w are DEVICE double
 * face velocities relative to the body on x-, y- and z-faces.  The fluxes
 * are F = A u with A the grid's open face areas (zero on faces of inactive
 * cells).  Inactive cells keep their fraction.
 * ------------------------------------------------------------------------ */

/* nfa_vof_create -- work memory of the advection on grid g (which must
 * outlive it; its body is read at every call, so it may be set or changed
 * later): a plane table (32 bytes per cell), two cell lists (4 bytes per cell
 * each) and one fraction buffer (8 bytes per cell).  Errors: NFA_ERR_HIP. */
typedef struct nfa_vof_s* nfa_vof;
nfa_status nfa_vof_create(nfa_grid g, nfa_vof* out);
void nfa_vof_destroy(nfa_vof v);

/* nfa_vof_sweep -- one sweep along dir (0 x, 1 y, 2 z):
 *   phi_out = phi - (F_d[uhat+] - F_d[uhat-]) / V + dilation,
 * uhat = dx_d F~ / V with the z-faces of each cell corrected by its share of
 * the cell's flux imbalance E (in proportion to the two z areas) so that
 * its six fluxes balance.  F_d moves across a face the water in the slab of
 * thickness |uhat| dt of the upwind cell next to it (below that cell's
 * interface plane, or times its fraction when it has none; a face on the
 * domain boundary draws from the cell inside).  The dilation is
 * dt phi (uhat+ - uhat-) / dx_d with the input phi (implicit = 0) or
 * phi_out (1 - dt (uhat+ - uhat-) / dx_d) = the rest (implicit = 1).
 * Interface planes: in each cell with 1e-12 < phi < 1 - 1e-12 and a non-zero
 * normal; normal -grad phi by weighted (1/4, 1/2, 1/4) central differences
 * over the 3x3x3 neighbourhood (the edge cell repeats beyond the domain, a
 * neighbour inside the body takes the cell's own fraction), constant by 64
 * bisection steps on the cube's volume function.
 *   dt > 0; the slab is capped at the full cell (|uhat| dt <= dx_d is the
 *   caller's Courant condition).  phi_out must not overlap phi.  Calls on
 *   one handle are ordered by their streams; calls that may overlap need
 *   handles of their own.   ASYNC.
 * Errors: NFA_ERR_INVALID (NULL, dt, dir, overlap). */
nfa_status nfa_vof_sweep(nfa_vof vof, const double* phi, const double* u, const double* v,
                         const double* w, double dt, int dir, int implicit, double* phi_out,
                         nfa_stream s);

/* nfa_vof_advect -- one time step: sweeps x, y, z on even `step`, z, y, x on
 * odd ones (the order alternates from step to step), the first two explicit
 * and the last implicit.  The face velocities are those of the step (u^k in
 * stage 1, (u* + u^k)/2 in stage 2 of the Runge-Kutta cycle).
 *   phi     : DEVICE double cells, input (not written).
 *   phi_out : DEVICE double cells, output; must not overlap phi.   ASYNC. */
nfa_status nfa_vof_advect(nfa_vof vof, const double* phi, const double* u, const double* v,
                          const double* w, double dt, int step, double* phi_out, nfa_stream s);

#ifdef __cplusplus
}
#endif
#endif /* NFA_H */
