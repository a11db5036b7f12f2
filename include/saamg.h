/*
 * saamg.h - C interface of the MI355X (gfx950) SA-AMG preconditioned CG Poisson solver.
 *
 * The library solves the finite-difference Poisson problem  -Laplace(phi) = rho  on a
 * beam-pipe domain embedded in a regular lattice, with phi = 0 on the wall
 * (Adelmann, Arbenz, Ineichen, "A fast parallel Poisson solver on irregular domains
 * applied to beam dynamics simulations"):
 *
 *   - Section 2: 7-point star (eq. 7pt-star); at the curved wall an outside neighbour is
 *     replaced by constant (eq. const_extrapol), linear (eq. lin_extrapol) or quadratic
 *     (eqs. quad_extrapol, quad_extrapol1) extrapolation; the system is scaled to unit
 *     diagonal by D^-1/2 A D^-1/2.
 *   - Section 3.1: conjugate gradients, also for the mildly nonsymmetric quadratic rule.
 *   - Section 3.2 / Table 1: smoothed-aggregation AMG V-cycle (Algorithm 1) as the
 *     preconditioner; 3^3 cube aggregates, damped-Jacobi prolongator smoothing,
 *     R = P^T, Chebyshev pre- and post-smoothing, direct solve on the coarsest level
 *     (at most 1000 unknowns).
 *   - Section 5 (solver comparison): stop when ||r||_2 <= tol ||b||_2.
 *
 * All solve-time work runs in HIP kernels on the GPU.  Every entry point returns a
 * status code (saamg_status); no C++ exception crosses this interface.  The message
 * of the last failure on the calling thread is available from saamg_last_error().
 *
 * Layout conventions
 *   A "box vector" is an array of nx*ny*nz values, x fastest, then y, then z
 *   (C order (nz, ny, nx)).  Entries at nodes that are not unknowns are ignored on
 *   input and written as 0 on output.
 *   Device pointers must point to memory of the device that was current when
 *   saamg_setup ran; streams are hipStream_t values passed as void* (NULL = the
 *   default stream of that device).
 */
#ifndef SAAMG_H
#define SAAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAAMG_OK = 0,
    SAAMG_INVALID_ARG = 1,   /* bad size, pointer, domain or option */
    SAAMG_NOMEM = 2,         /* a device or host allocation failed */
    SAAMG_HIP_ERROR = 3,     /* a HIP runtime call failed */
    SAAMG_NOT_CONVERGED = 4, /* max_iter reached; x holds the last iterate */
    SAAMG_BREAKDOWN = 5,     /* p.Ap <= 0 or r.z <= 0; x holds the last iterate */
    SAAMG_NONFINITE = 6      /* NaN or Inf met in the iteration; x holds the last iterate */
} saamg_status;

/* Wall rule at the curved boundary (Section 2). */
enum { SAAMG_VARIANT_CONST = 0, SAAMG_VARIANT_LIN = 1, SAAMG_VARIANT_QUAD = 2 };
/* Precision policy: all fp64, or fp32 hierarchy / V-cycle with fp64 outer CG,
 * dot products, true residual and coarse direct solve. */
enum { SAAMG_FP64 = 0, SAAMG_MIXED = 1 };
/* Coarsest-level solver (Section 3.2): dense direct solve, or Gauss-Seidel sweeps. */
enum { SAAMG_COARSE_DIRECT = 0, SAAMG_COARSE_GS = 1 };
/* Analytic pipe shapes for saamg_domain_from_shape. */
enum { SAAMG_SHAPE_CYLINDER = 0, SAAMG_SHAPE_ELLIPSE = 1, SAAMG_SHAPE_BOXBORE = 2 };

/*
 * Discrete domain (Section 2, lattice Omega_h and Figure "boundary").
 *   mask       host, nx*ny*nz bytes, nonzero = the node is an unknown.  No unknown may
 *              lie on a face of the box.
 *   wall_*     host, n_wall entries: for an unknown node (box-linear index wall_node)
 *              whose neighbour in direction wall_dir (0..5 = -x,+x,-y,+y,-z,+z) is not
 *              an unknown, the wall sits at fraction wall_s in (0, 1] of the spacing.
 *              An outside neighbour without an entry means s = 1 (the neighbour is on
 *              the wall).  Entries may come in any order; duplicates are an error.
 *   robin_d    0: every outside neighbour is a Dirichlet wall (phi = 0).  > 0: open ends
 *              (eq. poisson, Robin condition dphi/dn + phi/d = 0 on Gamma_2, discretised
 *              by eq. inlet) with d = robin_d: the box planes z = 0 and z = nz-1 are ghost
 *              planes, and every unknown on planes 1 and nz-2 takes its outside z-neighbour
 *              from eq. inlet (its inner z-neighbour must be an unknown).  Those rows and
 *              their right-hand side are divided by 2, which leaves the solution unchanged
 *              and keeps the constant and linear rules symmetric.
 * The library copies what it needs; the caller keeps ownership.
 */
typedef struct {
    int32_t nx, ny, nz;
    double hx, hy, hz;
    const uint8_t* mask;
    int64_t n_wall;
    const int64_t* wall_node;
    const uint8_t* wall_dir;
    const double* wall_s;
    double robin_d;
} saamg_domain;

/* Preconditioner and solver options; saamg_default_options fills the defaults. */
typedef struct {
    int32_t precision;     /* SAAMG_FP64 or SAAMG_MIXED                        default FP64 */
    int32_t max_levels;    /* hierarchy depth limit                            default 10   */
    int32_t max_coarse;    /* stop coarsening at <= this many unknowns (Table 1) default 1000 */
    int32_t cheb_degree;   /* Chebyshev polynomial degree, 1..8                default 2    */
    double cheb_ratio;     /* smoothing interval [lambda_hi/ratio, lambda_hi]  default 10   */
    double cheb_boost;     /* lambda_hi = boost * spectral estimate            default 1.1  */
    int32_t eig_iters;     /* Lanczos steps per level (spectral estimate)      default 15   */
    double omega_scale;    /* prolongator damping omega = scale / lambda_est   default 4/3  */
    int32_t coarse_solver; /* SAAMG_COARSE_DIRECT: dense fp64 inverse of the coarsest operator;
                              SAAMG_COARSE_GS: coarse_sweeps Gauss-Seidel sweeps from 0, in fp64,
                              unknowns visited by colour (parities of the logical coordinates;
                              multilevel hierarchies; the level's box with its ghost layer must
                              hold at most 8192 nodes)                         default DIRECT */
    int32_t coarse_sweeps; /* Gauss-Seidel sweeps (Section 3.2 uses 3)         default 3    */
    /* Level-0 launch shape of the solve-time kernels (results agree up to the order of
       the dot products' partial sums): planes per block along z (0 = automatic; else a
       power of two 2..32, capped at 14 for fp32 and 30 for fp64 on 16-byte lanes) and
       64-node segments per block along x (0 = automatic; else 1, 2 or 4, at most the
       segments of a line; one-node lanes only).                         default 0, 0 */
    int32_t l0_planes;
    int32_t l0_tile_x;
    /* Device memory.  Every buffer of the hierarchy, of the solve states created on it
       and of the library's temporaries comes from alloc(alloc_ctx, bytes, stream), which
       returns memory of the current device aligned to 256 bytes (NULL: failure, reported
       as SAAMG_NOMEM; a misaligned block is freed again and reported as
       SAAMG_INVALID_ARG) that
       may be used in stream order on `stream` (a hipStream_t; NULL = the default stream),
       and goes back through free(alloc_ctx, ptr, stream) once no queued work uses it.
       Both NULL: the library's own pool (per device; new memory from hipMalloc, freed
       blocks kept and reused once the work queued before their release has completed,
       at most 16 GiB cached).  The library zero-fills new buffers on the stream itself
       (stream-ordered, no host synchronisation).  Both callbacks may be called from any
       thread that calls into the library with this hierarchy. */
    void* (*alloc)(void* alloc_ctx, size_t bytes, void* stream);
    void (*free)(void* alloc_ctx, void* ptr, void* stream);
    void* alloc_ctx;
    /* Lanes of the level-0 V-cycle and CG kernels: 1 = one node per lane (a wavefront
       marches one 64-node segment of a line); 2 = 16 bytes per lane (4 consecutive fp32
       or 2 fp64 nodes, a wavefront marching 256 or 128 nodes of a line: a quarter or half
       of the vector memory instructions per node; needs nx a multiple of 4); 0 =
       automatic (2 where nx is a multiple of 4 and above 128, else 1).    default 0 */
    int32_t l0_wide;
    /* CG directions kept on 16-byte-lane hierarchies before x takes them (x is updated
       from all of them in one pass when they are all in use and before x is read):
       0 = automatic (32, fewer where 32 directions of the box would exceed 8 GiB, at least
       2); else 2..32.  The iterates do not depend on it.                  default 0 */
    int32_t cg_ring;
} saamg_options;

/* Outcome of one solve. rel_res_* are ||r||/||b|| of the scaled system. */
typedef struct {
    int32_t iterations;        /* products with A inside the CG loop */
    int32_t status;            /* saamg_status */
    int32_t replacements;      /* true-residual replacements */
    double rel_res_true;       /* from b - A x recomputed in fp64 at exit */
    double rel_res_recursive;  /* from the recursively updated residual */
    double t_solve_ms;         /* host wall time of the solve call */
} saamg_result;

/* Shape of a built hierarchy (for reporting and tests). */
#define SAAMG_MAX_LEVELS 16
typedef struct {
    int32_t n_levels;
    int32_t variant;
    int32_t precision;
    int32_t dims[SAAMG_MAX_LEVELS][3];    /* logical box of each level (level 0 = lattice) */
    int64_t n_unknowns[SAAMG_MAX_LEVELS];
    double lambda_est[SAAMG_MAX_LEVELS];  /* Lanczos estimate of lambda_max(D^-1 (A+A^T)/2) */
    double omega[SAAMG_MAX_LEVELS];
    int64_t n_irregular;                  /* level-0 rows with a non-constant stencil */
    int64_t device_bytes;                 /* device memory held by the hierarchy */
    double t_setup_ms;
    double t_refresh_ms;                  /* last saamg_refresh (host wall time), 0 if none */
    int32_t l0_planes;                    /* level-0 launch shape in use: planes per block, */
    int32_t l0_tile_x;                    /* 64-node segments per block along x            */
    int64_t table_rows[SAAMG_MAX_LEVELS]; /* stored coefficient rows of A_l (level 0: of   */
                                          /* its irregular rows, lines repeating the line  */
                                          /* below sharing rows)                           */
    int64_t table_rows_t[SAAMG_MAX_LEVELS]; /* and of A_l^T (nonsymmetric levels)           */
    /* host wall time of the setup's phases: domain checks (host), level-0 operator (masks,
       table, scaling), spectral estimates, Galerkin products and their compression, the
       coarsest-level solver, fp32 copies */
    double t_setup_phase_ms[6];
    int32_t l0_wide;                      /* 1: level-0 kernels on 16-byte lanes          */
    int32_t l0_wide_planes[2];            /* their planes per block: fp32, fp64 lanes     */
} saamg_info;

typedef struct saamg_hierarchy saamg_hierarchy;
typedef struct saamg_state saamg_state;

/* Thread-local message of the last failing call ("" if none). */
const char* saamg_last_error(void);

void saamg_default_options(saamg_options* opt);

/*
 * Build the discrete domain of an analytic pipe on a lattice spanning its bounding box
 * (Section 4, irregular domains: grid / wall intersections from the implicit surface).
 *   kind          SAAMG_SHAPE_*; a, b: half-extents of the box along x and y (radius,
 *                 semi-axes, or cavity half-width); length: extent along z; bore_r and
 *                 cavity_half_len: BOXBORE only (ignored otherwise).
 *   nx, ny, nz    lattice nodes per axis, end points included.
 *   open_ends     0: the end planes are Dirichlet walls and the box is the lattice.
 *                 1: the end planes hold unknowns (set robin_d = length/2 in the domain)
 *                 and the box has nz + 2 planes, the lattice's plane k at box plane k + 1.
 *   mask_out      host, nx*ny*(box planes) bytes, written.
 *   wall_cap      capacity of the three wall_* output arrays (host); may be 0 to query.
 *   n_wall_out    number of entries with s < 1.  If it exceeds a nonzero wall_cap the
 *                 first wall_cap entries are written and SAAMG_INVALID_ARG is returned.
 *   h_out         (nullable) host, 4 doubles: the spacings hx = 2a/(nx-1), hy = 2b/(ny-1),
 *                 hz = length/(nz-1) and the Robin parameter d of the domain (length/2
 *                 with open ends, else 0), i.e. the saamg_domain fields hx, hy, hz, robin_d.
 * Node coordinates are a*(2i-(n-1))/(n-1) per axis; unknowns lie strictly inside (a node
 * inside only within a relative 1e-12 of the wall counts as on the wall).  The entries
 * are written in node order; the work is split over up to 16 host threads.  Host-only and
 * reentrant.
 */
int saamg_domain_from_shape(int kind, double a, double b, double length, double bore_r,
                            double cavity_half_len, int nx, int ny, int nz, int open_ends,
                            uint8_t* mask_out, int64_t wall_cap, int64_t* wall_node,
                            uint8_t* wall_dir, double* wall_s, int64_t* n_wall_out,
                            double* h_out);

/*
 * Build the scaled operator and the SA-AMG hierarchy on the current device.
 *   Section 2: the 7-point operator with the wall rule of `variant` (SAAMG_VARIANT_*:
 *   eq. const_extrapol, eq. lin_extrapol, eqs. quad_extrapol / quad_extrapol1) and its
 *   scaling to unit diagonal; Section 3.2 and Table 1: 3^3 cube aggregates, one
 *   damped-Jacobi step on the tentative prolongator, Galerkin coarse operators
 *   A_{l+1} = P^T A_l P, a Chebyshev smoother per level, coarsening until at most
 *   max_coarse unknowns, and a direct (or Gauss-Seidel) solver on the coarsest level.
 *   A level whose aggregates would not reduce the number of unknowns ends the
 *   coarsening and becomes the coarsest level.
 *   dom       host domain (copied; the caller keeps ownership).
 *   opt       may be NULL (defaults).  Its allocator, if any, serves every later call on
 *             the hierarchy and on the states created on it.
 *   stream    work is queued on it (hipStream_t, NULL = default stream); the call
 *             returns after the hierarchy is complete.
 *   *out      owns all device memory of the hierarchy until saamg_destroy.
 * Errors: SAAMG_INVALID_ARG for a bad domain or option (nothing allocated),
 * SAAMG_NOMEM, SAAMG_HIP_ERROR.  Setups, solves and steps of other hierarchies may run
 * at the same time on other threads and streams of the device.
 */
int saamg_setup(const saamg_domain* dom, int variant, const saamg_options* opt, void* stream,
                saamg_hierarchy** out);

/*
 * Solve A x = b with preconditioned CG (Section 3.1, also for the nonsymmetric quadratic
 * rule), one V-cycle of Algorithm 1 per step as the preconditioner (Section 3.2), on the
 * scaled system of Section 2; stop when ||r||_2 <= tol ||b||_2 of the scaled system
 * (Section 5), confirmed by a true residual b - A x recomputed in fp64.  A previous
 * solution as x0 is the warm start of Section 4.
 *   d_b    device, box vector of rho (unscaled right-hand side), fp64.
 *   d_x0   device box vector of the initial guess (unscaled), fp64, or NULL for 0.
 *   d_x    device box vector, fp64, receives the solution (may alias d_x0).
 *   tol    relative residual of the scaled system (> 0); max_iter >= 0.
 *   stream work is queued on it; the call returns after completion.
 * res (nullable) receives the outcome.  The work vectors are allocated on the first
 * solve of H (with H's allocator) and kept with H.  Errors: SAAMG_INVALID_ARG (NULL or
 * bad argument), SAAMG_NOMEM, SAAMG_HIP_ERROR; SAAMG_NOT_CONVERGED, SAAMG_BREAKDOWN
 * and SAAMG_NONFINITE still write the last iterate to d_x.
 */
int saamg_solve(saamg_hierarchy* H, const double* d_b, const double* d_x0, double* d_x,
                double tol, int max_iter, void* stream, saamg_result* res);

/*
 * saamg_solve for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same solve and the
 * same results (on 16-byte-lane hierarchies x takes the CG directions from a ring of 2
 * instead of up to 16, the same updates in the same order), with every work vector (PCG vectors,
 * the V-cycle's vectors on all levels, block partials, scalars) carved out of a static
 * 64 MiB device array inside the library instead of allocated.  No hipMalloc, hipFree,
 * pinned host allocation, event creation or allocator callback happens in the call; the
 * work vectors are zero-filled by a kernel on `stream` first.  Arguments, results and
 * errors as for saamg_solve, plus SAAMG_INVALID_ARG (nothing queued) when the hierarchy
 * needs more than 64 MiB of work space (about a million box nodes in mixed precision;
 * saamg_solve has no such limit).  All calls on one device share that device's array:
 * calls that overlap on one device (other threads or streams) race and must be
 * serialised by the caller.  Each device keeps its array until the process ends.
 */
int saamg_solve_noalloc(saamg_hierarchy* H, const double* d_b, const double* d_x0, double* d_x,
                        double tol, int max_iter, void* stream, saamg_result* res);

/*
 * Numeric-only re-setup reusing the aggregation hierarchy (Section 5.2, reuse of the
 * aggregation hierarchy; Table 6 times it): keeps H's aggregates (the tentative
 * prolongators), storage and buffers, and recomputes every number from dom: level-0
 * stencil weights and scaling, spectral estimates, smoothed prolongators, Galerkin
 * operators, Chebyshev coefficients and the coarsest-level solver.  The result equals a
 * fresh saamg_setup of dom with H's variant and options.  Typical use: a bunch that
 * elongates, so that the spacings change while the lattice does not.
 *   dom     host domain as for saamg_setup; it must have H's box, the same unknowns and
 *           near-wall rows (nodes with a cut wall, plus the end planes with open ends)
 *           and the same end condition kind; spacings, wall fractions and robin_d may
 *           differ.
 *   stream  work is queued on it; the call returns when H is complete.
 * Errors: SAAMG_INVALID_ARG when dom fails those checks or a solve state created on H
 * still exists (H unchanged).  A failure after the checks (HIP error) leaves H unusable:
 * destroy it.
 */
int saamg_refresh(saamg_hierarchy* H, const saamg_domain* dom, void* stream);

/*
 * Reuse of the preconditioner (Section 5.2, reusing the preconditioner): later solves on H
 * iterate with the system operator of dom (its level-0 stencil weights, wall rows and
 * scaling D^-1/2), while the preconditioner -- every level's operator, smoother,
 * transfer operators and the coarsest-level solver -- stays the one H was built (or last
 * refreshed) for.  The paper keeps the first time step's preconditioner through a
 * simulation and recomputes it only once the iteration count exceeds a threshold; the
 * caller decides that and calls saamg_refresh(H, dom), which rebuilds the preconditioner
 * for dom and ends the reuse.  saamg_operator_apply and saamg_scaling report the
 * operator in use; saamg_level_apply and saamg_level_coefficients the preconditioner's
 * levels.
 *   dom     host domain with H's box, unknowns and near-wall rows and the same end
 *           condition kind (as for saamg_refresh); copied.
 *   stream  work is queued on it; the call returns when the operator is complete.
 * Errors: SAAMG_INVALID_ARG when dom fails those checks or a solve state created on H
 * still exists (H unchanged); SAAMG_NOMEM, SAAMG_HIP_ERROR.
 */
int saamg_set_operator(saamg_hierarchy* H, const saamg_domain* dom, void* stream);

/* Free the hierarchy (NULL is accepted). */
int saamg_destroy(saamg_hierarchy* H);

int saamg_hierarchy_info(const saamg_hierarchy* H, saamg_info* info);

/*
 * Device bytes a hierarchy and one solve state would take for a box of the given size
 * (upper bounds from the box, used for admission control).
 */
int saamg_footprint_bytes(int nx, int ny, int nz, int variant, int precision,
                          int64_t* hier_bytes, int64_t* state_bytes);

/* ---- incremental solves (continuous batching) --------------------------------------
 * A state owns the CG vectors of one solve.  saamg_batch_step advances every state that
 * is not finished by exactly one PCG step (or finishes it); states may belong to
 * different hierarchies.  Each state's work is queued on its own stream, so steps of
 * different states overlap on the device.  A state's iterates are identical to those of
 * saamg_solve on the same inputs.
 */
int saamg_state_create(saamg_hierarchy* H, const double* d_b, const double* d_x0, double tol,
                       int max_iter, void* stream, saamg_state** out);
/* n states; *n_done_out (nullable) receives how many are finished after the step. */
int saamg_batch_step(saamg_state* const* states, int n, int* n_done_out);
/*
 * The same step machine without waiting: every unfinished state whose step has completed
 * on the device is taken through its host-side test (and finished, or given its next
 * step), and every unfinished state with no step queued gets one.  Returns at once, so a
 * caller that polls it lets each state advance at its own pace: a small solve is never
 * held back by a large one in the same batch.  The host-side test can still wait briefly
 * where it recomputes a true residual (at convergence).  *n_done_out: finished states;
 * *n_stepped_out: states that completed a step in this call (both nullable).
 */
int saamg_batch_advance(saamg_state* const* states, int n, int* n_done_out, int* n_stepped_out);
/* done = 1 when the state has finished (any status); res as for saamg_solve. */
int saamg_state_query(const saamg_state* S, int* done, saamg_result* res);
/* Write the (unscaled) current iterate to the device box vector d_x on the state's
 * stream; returns after the write is complete.  Earlier writes of d_x on other streams
 * must be complete before the call. */
int saamg_state_finish(saamg_state* S, double* d_x);
int saamg_state_destroy(saamg_state* S);

/* ---- component entry points (parity tests and diagnostics) ------------------------
 * Host-pointer, fp64, logical-box-layout access to single steps of the method.  Level
 * l vectors are (mz, my, mx) arrays of the level's logical box (info.dims[l]).  The
 * precision argument selects the fp64 data or, for a MIXED hierarchy, its fp32 copy.
 */
enum {
    SAAMG_OP_APPLY = 0,     /* out = A_l in                                  */
    SAAMG_OP_APPLY_T = 1,   /* out = A_l^T in                                */
    SAAMG_OP_PRESMOOTH = 2, /* out = Chebyshev smoother from 0 with rhs in   */
    SAAMG_OP_RESTRICT = 3,  /* out (level l+1) = P_l^T in (level l)          */
    SAAMG_OP_PROLONG = 4    /* out (level l) = P_l in (level l+1)            */
};
int saamg_level_apply(saamg_hierarchy* H, int level, int op, int precision, const double* h_in,
                      double* h_out);
/* Coefficients A_l(I, I+o) as [27][mz][my][mx] fp64 (o = (dx,dy,dz), index
 * (dx+1) + 3(dy+1) + 9(dz+1)); for level 0 the scaled operator. */
int saamg_level_coefficients(saamg_hierarchy* H, int level, double* h_out);
/* One V-cycle z = M^-1 r on device box vectors of the scaled level-0 system (fp64). */
int saamg_precond_apply(saamg_hierarchy* H, const double* d_r, double* d_z, void* stream);
/* Scaled operator y = D^-1/2 A D^-1/2 x on device box vectors (fp64, 16-byte aligned,
   else SAAMG_INVALID_ARG). */
int saamg_operator_apply(saamg_hierarchy* H, const double* d_x, double* d_y, void* stream);
/* D^-1/2 as a device box vector (0 at non-unknowns), fp64. */
int saamg_scaling(saamg_hierarchy* H, double* d_sigma, void* stream);

/* The explicit inverse of the coarsest operator held by the direct coarse level solver
 * (Section 3.2, coarse level solver: the coarsest system is solved exactly).  *n_out
 * receives its order n.  h_rows (nullable, host, n int64): the logical box index
 * x + mx (y + my z) on the coarsest level of each row (and column), ascending.  h_inv
 * (nullable, host, n * n fp64): the inverse, row-major.  Synchronous.  Errors:
 * SAAMG_INVALID_ARG when H uses Gauss-Seidel sweeps as its coarse solver (no inverse). */
int saamg_coarse_inverse(saamg_hierarchy* H, int32_t* n_out, int64_t* h_rows, double* h_inv);

/* ---- particle coupling (Section 1 and Section 4: charge to the grid, field back) -------
 * A grid is the box of a discrete domain (nx, ny, nz), the box plane of the lattice's
 * plane 0 (1 with open ends, else 0), the coordinates of lattice node (0, 0, 0), the
 * spacings, and robin_d (> 0: open ends, as in saamg_domain).  The lattice has nx, ny and
 * nz - 2*z_offset nodes; its cells are [i, i+1) x [j, j+1) x [k, k+1).
 */
typedef struct {
    int32_t nx, ny, nz;
    int32_t z_offset;
    double origin[3];
    double h[3];
    double robin_d;
} saamg_grid;

typedef struct saamg_pic saamg_pic;

/*
 * Context for up to max_particles particles on grid g (copied).  mask: host, nx*ny*nz
 * bytes, nonzero = unknown (the domain's mask), or NULL for "every node".  Allocates the
 * sort buffers on the current device once.
 */
int saamg_pic_create(const saamg_grid* g, const uint8_t* mask, int64_t max_particles,
                     saamg_pic** out);
/*
 * Cloud-in-cell deposition: d_pos is device (n, 3) fp64 positions (x, y, z interleaved),
 * each particle carries charge q; d_rho (device, box vector, fp64) receives the density
 * nodal charge / (hx hy hz) at every box node (0 where no particle contributes).
 * Particles outside every lattice cell are dropped.  Deterministic: each node sums its
 * adjacent cells' particles in a fixed order (cells by index, particles by cell after a
 * stable sort), so repeated calls give bitwise equal results.  Queued on stream.
 */
int saamg_pic_deposit(saamg_pic* P, const double* d_pos, int64_t n, double q, double* d_rho,
                      void* stream);
/*
 * Field gather: d_E (device, (n, 3) fp64) receives E = -grad(phi) at the particles, the
 * trilinear interpolation of central differences of phi (device box vector, e.g. a
 * solution of saamg_solve) at the eight corners of each particle's cell.  phi counts as 0
 * off the domain and beyond the box; beyond an open end it is eq. inlet's
 * u(x'') - (2 h_z / d) u(x).  Particles outside every cell get E = 0.  Queued on stream.
 */
int saamg_pic_gather(saamg_pic* P, const double* d_phi, const double* d_pos, int64_t n,
                     double* d_E, void* stream);
int saamg_pic_destroy(saamg_pic* P);

/* ---- kernel timing (diagnostics) ----------------------------------------------------
 * When enabled for a kernel class, every call that launches kernels of that class binds
 * a pair of HIP events to its first and last kernel dispatch on its own stream (no marker
 * is inserted between kernels); saamg_timer_read synchronises on them and returns the
 * summed start-to-end time, the launch count and the algorithmic bytes moved (each
 * array the kernel must read or write counted once over the unknowns it covers).
 * Classes: 0 level-0 Chebyshev steps, 1 level-0 residual, 2 restriction to level 1,
 * 3 prolongation from level 1, 4 CG direction update + product with A, 5 CG r update,
 * 6 all coarse-level kernels, 7 reduction finalisation, 8 x update from the ring of fp32
 * CG directions (mixed precision on 16-byte lanes; the other forms update x in class 4).
 * At most 65536 launches are kept between resets; later ones are not timed.
 */
int saamg_timer_enable(int kind, int enable);
int saamg_timer_read(int kind, double* total_ms, int64_t* launches, int64_t* alg_bytes);
int saamg_timer_reset(void);

#ifdef __cplusplus
}
#endif
#endif /* SAAMG_H */
