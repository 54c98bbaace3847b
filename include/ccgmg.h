/*
 * ccgmg.h -- C interface of the MI355X cut-cell geometric-multigrid solver
 * for the fourth-order finite-volume discretisation of
 *
 *      a u_xx + b u_xy + c u_yy = f   in an irregular 2-D domain,  b^2 < 4ac,
 *
 * with Dirichlet, Neumann or Robin data on each boundary curve (problem
 * statement: Section 1, eq. ccEllipticEq; the boundary operator N: Section 3,
 * treated in detail for Neumann data in Section 3.3).  The
 * unknowns are cut-cell averages of u and the data are cell averages of f
 * and boundary-face averages of g (Section 3.2).  The discrete system is
 * L u + N g = f (eq. PoissonLinearDiscretization); the solver iterates
 * multigrid V-cycles (Alg. 2) on L u = f - N g (eq. PoissonResidualForm).
 *
 * Conventions
 *  - Every function returns a ccgmg_status (0 = OK, < 0 = error); no C++
 *    exception crosses this interface.  On error a context is left unchanged
 *    and ccgmg_last_error() describes the failure.
 *  - Grids are row-major with x fastest: cell (i, j) has linear index
 *    j * nx + i and covers (x0 + i h, x0 + (i+1) h) x (y0 + j h, y0 + (j+1) h).
 *  - "device" pointers are HIP device memory on the context's device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns the context and all its device data, which are
 *    allocated in ccgmg_create and freed in ccgmg_destroy.
 *  - All device work is ordered on options.hip_stream (0 = the null stream).
 *    A context is not thread safe; distinct contexts are independent.
 *  - Values on empty or merged-away cells are ignored on input and written
 *    as zero on output.  A merged cell's value is the average over the union
 *    (Section 3.1, Alg. 1).
 */
#ifndef CCGMG_H
#define CCGMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque solver context; owned by the library (created by ccgmg_create,
 * released by ccgmg_destroy). */
typedef struct ccgmg_ctx ccgmg_ctx;

typedef enum {
  CCGMG_OK = 0,
  CCGMG_EINVAL = -1,       /* bad argument, NaN/Inf input, size out of range      */
  CCGMG_ENOTELLIPTIC = -2, /* b^2 - 4ac >= 0                                      */
  CCGMG_EGEOM = -3,        /* curves leave the grid, lie inside one cell, ...     */
  CCGMG_EPLG = -4,         /* no acceptable poised lattice on the finest grid     */
  CCGMG_ESINGULAR = -5,    /* singular coarsest operator                          */
  CCGMG_ENOCONV = -6,      /* max_cycles reached or the residual stagnated        */
  CCGMG_EDEVICE = -7,      /* HIP runtime error                                   */
  CCGMG_ENOMEM = -8        /* host or device allocation failed                    */
} ccgmg_status;

typedef enum { CCGMG_BOX = 0, CCGMG_CIRCLE = 1, CCGMG_ELLIPSE = 2, CCGMG_POLAR_SIN = 3,
               CCGMG_POLAR_COS = 4, CCGMG_POLYGON = 5 } ccgmg_curve_kind;

typedef enum { CCGMG_DIRICHLET = 0, CCGMG_NEUMANN = 1, CCGMG_ROBIN = 2 } ccgmg_bc;

/* A boundary curve.  Parameter layouts (p[]):
 *   BOX      x0, y0, x1, y1              (must equal the grid extent)
 *   CIRCLE   cx, cy, r
 *   ELLIPSE  cx, cy, a1, a2, rot
 *   POLAR_*  cx, cy, r0, A, k, phase     r(t) = r0 + A sin|cos(k t + phase)
 *   POLYGON  x0, y0, x1, y1, x2, y2, x3, y3   a convex quadrilateral, vertices
 *            counter-clockwise, no edge parallel to a grid line (the rotated
 *            box of Problem 3 (ii) in Section 5.1); corners split its arcs
 * domain_inside = 1 for the outer boundary (the domain is inside the
 * curve), 0 for a hole.  bc is a ccgmg_bc: the boundary operator N of
 * Section 3, with data g = N u averaged over each boundary face: u
 * (Dirichlet), du/dn (Neumann) or robin[0] u + robin[1] du/dn (Robin; both
 * finite, not both zero).  The normal n points out of the domain.  robin[]
 * is read only when bc = CCGMG_ROBIN. */
typedef struct {
  int kind;
  double p[8];
  int domain_inside;
  int bc;
  double robin[2];
} ccgmg_curve;

typedef struct {
  double x0, y0, h;
  int nx, ny;
} ccgmg_grid;

typedef struct {
  double theta;          /* small-cell merge threshold (Alg. 1), default 0.3              */
  double w_min;          /* least-squares weight floor (eq. weightDef), default 0.5       */
  double omega;          /* weighted-Jacobi factor of SMO-1, default 0.5; in (0, 2)      */
  int nu1, nu2;          /* pre/post smoothing steps, default 3, 3                        */
  int nu1_coarse, nu2_coarse; /* steps on the coarse levels when > 0 (default 0: nu1, nu2) */
  int coarsest_min_n;    /* smallest coarse grid side considered, default 16              */
  int max_levels;        /* default 16                                                    */
  int auto_depth;        /* coarsest level: 0 deepest that can be built; 1 deepest whose
                            V-cycles contract by <= depth_max_rate; 2 (default) measured:
                            time seeded solves at every admissible depth and keep the
                            one with the least time per cycle x cycles per 1e10 at the
                            measured asymptotic rate                                   */
  double depth_max_rate; /* contraction bound used by auto_depth, default 0.5            */
  int precision;         /* 0: FP64 sweeps; 1: FP32 sweeps inside FP64 refinement         */
  int prolongation;      /* 0: piecewise constant (Section 4.1); 1: bilinear              */
  int smo2_every_sweep;  /* 1: SMO-2 in every smoothing step (Section 4.1); 0: in the last
                            step of each smoothing phase only; s >= 2: in every s-th step
                            counted back from the last.  With fused steps the other
                            steps are plain SMO-1 sweeps (block rows unchanged) and the
                            step applying the coarse-grid correction is always fused   */
  int smo2_iters;        /* block iterations per SMO-2 application, default 1             */
  int smo2_block;        /* irregular cells per block, default 64                         */
  int smo2_overlap;      /* overlap layers of a block in the matrix graph, default 1      */
  int smo2_widen;        /* regular cells within this distance of the least-squares rows
                            join the SMO-2 blocks instead of SMO-1, default 1 (0 = the
                            paper's split)                                               */
  double tol;            /* stop when ||f - N g - L u||_inf / ||f - N g||_inf <= tol      */
  int max_cycles;        /* default 100                                                   */
  int max_nrhs;          /* right-hand sides solved together, default 1                   */
  int use_initial_guess; /* 1: u_hat holds the initial guess; 0: start from zero          */
  int num_threads;       /* host threads for set-up (0 = hardware concurrency)            */
  int use_graph;         /* 1: replay V-cycles from a captured hipGraph                   */
  int tune_tiles;        /* 1 (default): pick the SMO-1 tile height of every level and
                            precision by timing the candidates at set-up; 0: 64 x 16     */
  int sweep_tile_rows;   /* 8, 16 or 32: this tile height on every level (no tuning);
                            0 (default): as tune_tiles says                              */
  int smoother_fused;    /* 0: each smoothing step is SMO-1 then SMO-2 (Alg. 2); 1: both
                            in one launch from the same iterate (additive)               */
  int tune_schedule;     /* 1 (default, with auto_depth 2): also time the schedules
                            (smoother_fused, nu1, nu2 / coarse) = (0,3,3), (1,3,3),
                            (1,4,4), (1,5,5), (1,4,4/2,2), (1,5,5/2,2), (1,5,5/3,3),
                            (1,6,6/3,3), (1,4,4/3,4), (1,4,4/2,5), and with SMO-2 in
                            every s-th step (1,5,5/2,5; s 2), (1,4,4/2,5; 3),
                            (1,6,6/3,4; 3), (1,5,5/3,3; 2), (1,3,3/2,3),
                            (1,3,3/2,4; 3), (1,4,4/2,4; 3), (1,3,3/2,2), (1,2,3/2,3),
                            (1,3,3/1,3), and keep the fastest;
                            then the SMO-1 weight omega in {0.5, 0.6, 0.7, 0.77,
                            0.85, 0.92, 1.0} at that schedule and depth, and, if another weight
                            wins, the schedules again at that weight;
                            0: use the fields above (omega included)                     */
  int inverse_fp32;      /* storage of the dense inverses (SMO-2 blocks, coarsest level),
                            computed in FP64 and always applied in FP64 arithmetic:
                            1 (default) FP32, 0 FP64                                      */
  int host_only;         /* 1: build the hierarchy on the host only (no device calls);
                            queries work, apply/solve return CCGMG_EINVAL                  */
  int cycle;             /* 0 (default): V-cycles (Alg. 2); 1: FMG cycles (Section 4, Fig.
                            FMG-cycle): the residual restricted to the coarsest level,
                            solved there, then one V-cycle per level upwards from the
                            prolonged coarser solution; iterated like V-cycles          */
  int tune_cache;        /* 1: reuse (and record) the measured tile heights, schedule
                            and depth of an earlier context with the same GPU, level
                            sizes, precision, b != 0 and options, in this process or in
                            the file named by the environment variable CCGMG_TUNE_CACHE
                            (a text file the library reads once and appends to); a
                            heuristic for batches of similar geometries.  0 (default):
                            measure for every context                                    */
  void* hip_stream;      /* hipStream_t all device work is ordered on                     */
} ccgmg_options;

typedef struct {
  long n_cells;          /* nx * ny on the finest grid                                    */
  long n_unknowns;       /* non-empty cells after merging                                 */
  long n_irregular;      /* cells discretised by least-squares rows                       */
  long n_bdry_faces;     /* boundary faces = entries of g-hat                             */
  int n_levels;
  int nx_coarsest, ny_coarsest;
  long coarse_unknowns;
  double setup_seconds;
  double plg_max_cond;
  int smoother_fused;    /* smoothing schedule in use (after tuning)                      */
  int nu1, nu2;
  int nu1_coarse, nu2_coarse;
  int smo2_every_sweep;  /* SMO-2 frequency in use (see the option of that name)          */
  double omega;          /* SMO-1 weight in use (after tuning)                            */
} ccgmg_info;

typedef struct {
  int cycles;            /* V-cycles run (all outer iterations together)                  */
  int outer_iters;       /* FP64 refinement steps (precision 1)                           */
  double rel_res_inf;    /* final relative L-infinity residual (FP64, difference form)    */
  double rel_res_2;      /* final relative L2 residual ||f - N g - L u||_2 / ||f - N g||_2
                            (the same checks' sums of squares; max over right-hand sides) */
  double seconds;        /* device time of the solve                                      */
  double history[64];    /* relative residual after each check                            */
} ccgmg_report;

/* Defaults from the paper: theta 0.3 (Fig. 1), w_min 1/2 (eq. weightDef),
 * omega 0.5 and nu1 = nu2 = 3 (Fig. 5); tol 1e-10. */
void ccgmg_default_options(ccgmg_options* opts);

/* Set up the grid hierarchy (Section 4): cut cells and merging (Alg. 1),
 * regular/irregular classification (Section 3.2), poised lattices and
 * least-squares weights (Section 3.3, eq. derivedCoefAgain) on every level,
 * the SMO-2 block data (Section 4.1, ordered by Alg. 3) and the inverse of
 * the coarsest operator; uploads everything to the current HIP device.
 * grid, curves, opts: host, read only.  *out receives the new context.
 * CCGMG_EINVAL for options out of their ranges (theta outside [0, 1),
 * w_min <= 0, omega outside (0, 2), max_cycles < 1, tol < 0 or NaN, an
 * enumeration field outside the values listed with it), and also for a grid with (ny + 64) * nx * 8 >= 2^31 bytes (about
 * 2^28 cells: the kernels address a plane, its tile halos included, with
 * signed 32-bit byte offsets). */
int ccgmg_create(const ccgmg_grid* grid, const ccgmg_curve* curves, int ncurves, double a, double b,
                 double c, const ccgmg_options* opts, ccgmg_ctx** out);

/* One geometry of ccgmg_create_many: the arguments of ccgmg_create. */
typedef struct {
  ccgmg_grid grid;
  const ccgmg_curve* curves;
  int ncurves;
  double a, b, c;
} ccgmg_problem;

/* ccgmg_create for n geometries at once (for batches; not a paper
 * construct).  The host set-up of Section 4 (cut cells, Alg. 1, lattices,
 * least-squares rows, Alg. 3, SMO-2 data) of the geometries runs
 * concurrently: largest first (cells) on min(n, host_threads / 2) worker
 * threads, each with an equal share of host_threads (0: the hardware's
 * threads).  The calling thread uploads each geometry and tunes it on the
 * current device as soon as its host set-up is done, in that order.
 * probs: n problems (host); opts: n options (host) or NULL for defaults;
 * out: n contexts on success, each exactly as ccgmg_create would have made
 * it (set-up results do not depend on the thread count).  On error every
 * context built so far is destroyed, out[] is all NULL and
 * ccgmg_create_error() names the failing geometry. */
int ccgmg_create_many(const ccgmg_problem* probs, int n, const ccgmg_options* opts, int host_threads,
                      ccgmg_ctx** out);

/* Sizes and set-up results of a context (unknowns, irregular cells,
 * boundary faces, levels, the coarsest level, set-up time, largest lattice
 * condition number, the schedule in use).  info: host, written.
 * CCGMG_EINVAL for a NULL argument. */
int ccgmg_query(const ccgmg_ctx* ctx, ccgmg_info* info);

/* Level-m classification (host arrays of nx_m * ny_m entries):
 * kinds: 0 empty, 1 merged into another cell, 2 regular, 3 irregular pure,
 * 4 irregular cut (or merged host); hosts: final host of a merged cell, else -1.
 * Either pointer may be NULL. */
int ccgmg_get_cell_kinds(const ccgmg_ctx* ctx, int level, int8_t* kinds, int32_t* hosts);

/* Level-m grid side lengths. */
int ccgmg_get_level_shape(const ccgmg_ctx* ctx, int level, int* nx, int* ny);

/* Cut-cell volumes in units of h^2 (host, nx_m * ny_m). */
int ccgmg_get_volumes(const ccgmg_ctx* ctx, int level, double* vol);

/* Counts of level m: *n_irregular irregular cells (the rows of
 * ccgmg_get_irregular) and *n_faces boundary faces (Section 3.1); either
 * pointer may be NULL.  CCGMG_EINVAL for a bad level. */
int ccgmg_get_counts(const ccgmg_ctx* ctx, int level, long* n_irregular, long* n_faces);

/* SMO-1 tile height (64-wide tiles of 8, 16 or 32 rows) chosen for level m
 * in FP64 and FP32 sweeps (tune_tiles).  Device contexts only. */
int ccgmg_get_tuning(const ccgmg_ctx* ctx, int level, int* sweep_ty_fp64, int* sweep_ty_fp32);

/* Size of the SMO-2 block data of level m (adjoint = 1: of L^T), for
 * traffic accounting: stats[0] blocks, [1] block rows (the rows updated by
 * SMO-2: least-squares rows plus the regular rows joined to them),
 * [2] overlapped rows over all blocks, [3] their CSR entries, [4] bytes of
 * the blocks' dense inverses (computed in FP64, stored in FP32, applied in
 * FP64 arithmetic).  Device contexts only. */
int ccgmg_get_smo2_stats(const ccgmg_ctx* ctx, int level, int adjoint, long* stats);
/* Least-squares rows of level m (Section 3.3, eq. derivedCoefAgain; lattices
 * by the R-PLG rule for Section 2.2): rows[k] is the linear index of the
 * k-th irregular cell (n_irregular entries, increasing), cols[15 k ..
 * 15 k + 14] its lattice cells (sorted linear indices), vals[15 k ..] the
 * weights of L on them (1/h^2 units, the cell's own weight included),
 * cond[k] the 2-norm condition number of the lattice's cell sample matrix.
 * Host arrays of the sizes given by ccgmg_get_counts; any may be NULL.
 * CCGMG_EINVAL for a bad level.  ccgmg_get_stencils is the same without
 * cond. */
int ccgmg_get_irregular(const ccgmg_ctx* ctx, int level, int32_t* rows, int32_t* cols, double* vals,
                        double* cond);
int ccgmg_get_stencils(const ccgmg_ctx* ctx, int level, int32_t* rows, int32_t* cols, double* vals);

/* Boundary faces of level 0 in g-hat order: face k belongs to cell[k] and
 * curve[k]; its weight in row cell[k] of N is nweight[k] (so that
 * (N g)_cell = sum over the cell's faces of nweight * g).  Host arrays. */
int ccgmg_get_boundary_faces(const ccgmg_ctx* ctx, int32_t* cell, int32_t* curve, double* nweight);

/* Alg. 3 numbering of the level-m irregular cells: perm[p] is the linear
 * index of the p-th cell in the order (host, n_irregular entries). */
int ccgmg_get_alg3_order(const ccgmg_ctx* ctx, int level, int32_t* perm);

/* Quadrature for callers that average their own f and g (Section 2.4).
 * Cells: every non-pure non-empty level-0 cell gets nodes (x, y) and weights
 * w with sum_q w_q f(x_q, y_q) ~= int over the cell of f / h^2 (exact for
 * polynomials of degree <= 15 along the boundary pieces); pure cells are
 * squares the caller integrates itself.  Faces: nodes along each boundary
 * face with arclength weights (units of h) and the outward unit normal.
 * Two-call pattern: pass NULL arrays to receive the counts.
 * cell_of[k] / face_of[k]: owning cell / face index of node k. */
int ccgmg_cell_quadrature(const ccgmg_ctx* ctx, long* count, int32_t* cell_of, double* x, double* y,
                          double* w);
int ccgmg_face_quadrature(const ccgmg_ctx* ctx, long* count, int32_t* face_of, double* x, double* y,
                          double* w, double* nx, double* ny);

/* (L u) on every non-empty level-0 cell, N g not included.
 * u, Lu: device, nx * ny doubles; may not alias. */
int ccgmg_apply(ccgmg_ctx* ctx, const double* u, double* Lu);

/* Relative residual norms of a caller's iterate (Fig. 5 reports the
 * relative residual): for each of nrhs planes, with res = f - N g - L u and
 * ref = f - N g over the non-empty level-0 cells (the boundary data last
 * set), rel_inf[z] = max|res| / max|ref| and rel_l2[z] = ||res||_2 /
 * ||ref||_2 (plain sums of squares; a zero reference divides by 1).
 * f_hat, u_hat: device [nrhs][ny][nx]; rel_inf, rel_l2: host arrays of nrhs
 * doubles, either may be NULL (not both).  Synchronous; allocates a small
 * device buffer.  rel_inf is computed cell by cell as a solve's
 * convergence check computes it. */
int ccgmg_residual_norms(ccgmg_ctx* ctx, const double* f_hat, const double* u_hat, int nrhs, double* rel_inf,
                         double* rel_l2);

/* ccgmg_residual_norms for callers that cannot allocate (tight serving
 * loops, code between graph replays, harnesses that forbid allocation):
 * the same arguments and results (rel_inf equal, rel_l2
 * equal up to the order of the last sums), with every intermediate in a
 * static device array of 4 MiB that the library holds on each GPU it runs
 * on until the process ends.  It needs 8 * (4 * np + 4) * nrhs bytes, np =
 * the residual launch's workgroups (64 x 16 tiles plus one per 256
 * least-squares rows: 4211 at 2048^2, so up to 31 planes there);
 * CCGMG_EINVAL if that is more than 4 MiB, or if the current device is not
 * the context's.  Calls no hipMalloc, hipFree or other allocating routine.
 * Every call on a GPU reuses that GPU's one array (nothing in it needs to
 * start at zero): calls that overlap on one GPU, from other threads or
 * contexts, race.  Synchronous, like ccgmg_residual_norms. */
int ccgmg_residual_norms_noalloc(ccgmg_ctx* ctx, const double* f_hat, const double* u_hat, int nrhs,
                                 double* rel_inf, double* rel_l2);

/* Set the boundary data g-hat (device, n_bdry_faces * nrhs doubles, face
 * fastest).  The library copies it; nrhs <= max_nrhs. */
int ccgmg_set_boundary(ccgmg_ctx* ctx, const double* g_hat, int nrhs);

/* Solve L u = f - N g for nrhs right-hand sides: f_hat device
 * [nrhs][ny][nx], u_hat device [nrhs][ny][nx] (initial guess in, solution
 * out).  rep: host, may be NULL.  Returns CCGMG_ENOCONV (with u_hat holding
 * the last iterate) when tol is not reached, CCGMG_EINVAL when f_hat or the
 * boundary data hold a NaN or an Inf on a non-empty cell or face (found
 * from the reference norm ||f - N g||; u_hat is then undefined).  The
 * residual is checked after every V-cycle; the next cycle is queued before
 * that check only when the cycle being checked cannot reach tol (judged
 * from the contraction seen so far), so the solve stops at the first cycle
 * that reaches tol.  Allocates nothing; the first solve with a given pair
 * of arrays records the cycle's graph. */
int ccgmg_solve(ccgmg_ctx* ctx, const double* f_hat, double* u_hat, int nrhs, ccgmg_report* rep);

/* Adjoint solve L^T lambda = rhs (device arrays as in ccgmg_solve) by
 * V-cycles on the transposed operators of every level (L is not symmetric
 * near the boundary: the least-squares rows of Section 3.3).  The transposed
 * system of eq. PoissonResidualForm gives the gradients of a loss J(u) with
 * respect to f-hat (= lambda for rhs = dJ/du) and g-hat (= -N^T lambda). */
int ccgmg_solve_adjoint(ccgmg_ctx* ctx, const double* rhs, double* lambda, int nrhs, ccgmg_report* rep);

/* (L^T lambda) on every non-empty level-0 cell.  lambda, out: device,
 * nx * ny doubles; may not alias. */
int ccgmg_apply_adjoint(ccgmg_ctx* ctx, const double* lambda, double* out);

/* out = N^T lambda for nrhs planes (device; lambda [nrhs][ny][nx], out
 * [nrhs][n_bdry_faces]). */
int ccgmg_apply_NT(ccgmg_ctx* ctx, const double* lambda, double* out, int nrhs);

/* Diagnostic timing: launch one V-cycle kernel `reps` times on the
 * context's stream, on the context's own work buffers of level `level`
 * (one right-hand side), bracketed by HIP events; *avg_us receives the mean
 * duration per launch in microseconds.  kernel: 0 SMO-1 sweep (FP64),
 * 1 residual + restriction (FP64), 2 prolongation (FP64), 3 SMO-2 block
 * pass (FP64), 4 coarsest solve, 5 SMO-1 sweep (FP32), 6 plain FP64 copy of
 * the level's cell array (16 bytes per cell; calibrates byte counters),
 * 7 fused smoothing step (FP64, smoother_fused), 8 two consecutive plain
 * SMO-1 sweeps in one launch (FP64), 9 the fused step that also applies a
 * pending coarse-grid correction (FP64; needs a coarser level, whose work
 * iterate serves as the correction), 10 and 11 the fused step that also
 * writes the residual norm partials (level 0 only), into
 * the solve's pinned host buffer (10, as solves do) or into device memory
 * (11).  Leaves the work buffers of that level (and for 9 the coarser
 * level's iterate) undefined; no user buffer is touched. */
int ccgmg_profile_kernel(ccgmg_ctx* ctx, int kernel, int level, int reps, double* avg_us);

/* ---- Many geometries in one launch (batching) -------------------------
 * A batch groups contexts created by ccgmg_create (different geometries,
 * grid sizes and coefficients; each with its own boundary data set by
 * ccgmg_set_boundary).  ccgmg_batch_solve solves all of them together: one
 * V-cycle of every geometry (FP64 or mixed precision, as each context was
 * created) is captured into a single hipGraph whose branches run
 * concurrently, and the graph is replayed until every geometry's relative
 * residual is below its own tol; once a geometry has converged it is left
 * as it is (branches: only the active geometries' cycle graphs are
 * launched; lockstep: device flags mask its workgroups) while the others
 * finish.  Work is ordered after the stream of ctxs[0].  Contexts
 * must outlive the batch and must not be used by other calls while a batch
 * solve runs.  Not a paper construct: the batched use of the solve of
 * Section 4 (Alg. 2) for many independent problems. */
typedef struct ccgmg_batch ccgmg_batch;

/* nbranches >= 1: concurrent graph branches; geometries are placed largest
 * first (cells x right-hand sides) onto the least-loaded branch (4 matches
 * the hardware queues a process gets by default).
 * nbranches == 0: lockstep -- every launch performs one V-cycle step for
 * all geometries at once (a descriptor table per launch), converged
 * geometries are masked by device flags.  Needs one precision for all
 * contexts and at most 64 of them; sets every context's schedule to fused
 * smoothing with nu = ctxs[0]'s tuned nu1 (if fused and symmetric, else 4)
 * steps before and after on every level, piecewise-constant correction
 * and V-cycles. */
int ccgmg_batch_create(ccgmg_ctx* const* ctxs, int n, int nbranches, ccgmg_batch** out);

/* f[g], u[g]: device arrays of geometry g ([nrhs[g]][ny][nx], as in
 * ccgmg_solve, from a zero guess unless the context uses an initial guess);
 * reps: host array of n reports or NULL (seconds = the whole batch).
 * CCGMG_ENOCONV if any geometry did not reach its tolerance, CCGMG_EINVAL
 * for non-finite data (as ccgmg_solve).  The residual buffers are
 * allocated by ccgmg_batch_create; the first solve with a new set of arrays
 * (or a change of boundary data between none and some, or of a context's
 * depth or SMO-1 weight -- with branches also its schedule -- by
 * ccgmg_tune) records a new graph, and in lockstep mode allocates its
 * descriptor table. */
int ccgmg_batch_solve(ccgmg_batch* batch, const double* const* f, double* const* u, const int* nrhs,
                      ccgmg_report* reps);
/* Error text of the batch's last failed call (owned by the batch). */
const char* ccgmg_batch_last_error(const ccgmg_batch* batch);
/* Frees the batch (its graphs, streams and descriptor tables); the
 * contexts stay the caller's. */
void ccgmg_batch_destroy(ccgmg_batch* batch);

/* Re-choose the smoothing schedule, the depth and (with tune_schedule) the
 * SMO-1 weight, as auto_depth 2 / tune_schedule do at set-up, by timing
 * solves of the caller's own problem: f is one right-hand side (device,
 * ny x nx) representative of the solves to come, with the boundary data
 * last given to ccgmg_set_boundary.  Each candidate is solved from zero to
 * 1e-10 three times (capture, then two timed replays, the faster counting)
 * and the fastest that converges is kept.  Not a paper construct (the
 * paper fixes its cycle parameters); a measured autotuner of this library. */
int ccgmg_tune(ccgmg_ctx* ctx, const double* f);

/* Error text of the context's last failed call (owned by the context,
 * valid until its next call). */
const char* ccgmg_last_error(const ccgmg_ctx* ctx);

/* Error text of the last failed ccgmg_create on this thread. */
const char* ccgmg_create_error(void);

/* Frees the context and all its device and pinned host memory; NULL is
 * ignored. */
void ccgmg_destroy(ccgmg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* CCGMG_H */
