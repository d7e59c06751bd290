/*
 * lsp.h -- C ABI of the MI355X (gfx950) solver for the discretised
 * Lippmann-Schwinger equation with the sparsifying preconditioner
 * (L. Ying, "Sparsifying Preconditioner for the Lippmann-Schwinger
 * Equation", 2014).
 *
 * Problem (Section 1, eq:ls; Section 2.1, eq:lsd / eq:lso): on the uniform
 * grid of the unit square / cube with n points per axis, h = 1/n, grid
 * points x_i = (i + 1/2) h, find the scattered field u with
 *
 *     (I + K w^2 m) u = g,   K(i, j) = k_{i-j},   g = K(-w^2 m u_I),
 *
 * where k_t = h^d G(h t) (t != 0) samples the free-space Green's function
 * G of -(Laplacian + w^2) and k_0 is the integral of G over the disk/ball
 * of one cell's area/volume.  The solver is GMRES right-preconditioned by
 * P = M^{-1} Q (eq:PC): Q = [A; B] holds the 3^d-point stencils that make
 * Q K numerically local (eq:Fmin, eq:Emin, eq:Cmin and their 3D sets),
 * M = [A + C w^2 m; B] (eq:ABop) is factored by nested dissection and the
 * multifrontal method (Section 2.2, Section 3.2).
 *
 * Conventions for every entry point:
 *  - Grid vectors have N = n^d entries, linear index l = i1 + n i2 + n^2 i3
 *    (i1 fastest).  A block of nrhs vectors is contiguous, [nrhs][N].
 *  - Complex values are interleaved (re, im) pairs: complex128 = two
 *    doubles, complex64 = two floats.  The medium m is real double.
 *  - Pointers named *_dev are device (HBM) pointers of the GPU current
 *    when the problem was set up; *_host are host pointers.  The caller
 *    owns every buffer it passes; the library never frees them.
 *  - Device work is ordered on the HIP stream given to lsp_setup.  Calls
 *    that return host data synchronise that stream; the rest only enqueue.
 *  - No C++ exception crosses this boundary: every function returns an
 *    lsp_status, and lsp_last_error() gives a message for the calling
 *    thread's last failure.
 *  - A problem is used by one host thread at a time.  Distinct problems on
 *    distinct streams may run concurrently.
 */
#ifndef LSP_H
#define LSP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSP_OK = 0,
  LSP_ERR_ARG = 1,       /* invalid argument: d not in {2,3}, n < 4, w <= 0,
                            null pointer, workspace too small, nrhs too large */
  LSP_ERR_OOM = 2,       /* a host allocation failed */
  LSP_ERR_HIP = 3,       /* a HIP runtime call failed */
  LSP_ERR_STATE = 4,     /* call out of order (e.g. solve before factor) */
  LSP_ERR_SINGULAR = 5,  /* a zero or tiny pivot in a frontal factorisation */
  LSP_ERR_NOCONV = 6     /* GMRES hit max_iters; u holds the last iterate */
} lsp_status;

typedef enum {
  LSP_FP64 = 0,   /* every step in complex128 */
  LSP_MIXED = 1   /* preconditioner (Q apply, fronts, triangular solves) and the
                     operator inside the Arnoldi step in complex64; Arnoldi
                     orthogonalisation, true residual, iterate update in
                     complex128 */
} lsp_precision;

typedef enum {
  LSP_RHS_INCIDENT = 0,  /* rhs holds u_I; the library forms g = K(-w^2 m u_I) */
  LSP_RHS_G = 1,         /* rhs holds g itself */
  LSP_RHS_SOURCE = 2     /* rhs holds a source density f on the grid; the
                            library forms g = K f (the right-hand side G * f
                            of Section 5's eq:lslap; a discrete delta source
                            at grid point j is f = e_j / h^d) */
} lsp_rhs_kind;

typedef enum {
  LSP_HELMHOLTZ = 0,  /* eq:lsd: (I + K w^2 m) u = g, G the Helmholtz
                         Green's function of Section 1, w > 0 */
  LSP_LAPLACE = 1     /* Section 5 (eq:lap, eq:lslap), 3D only: (I + K V) u =
                         K f with G(x) = 1/(4 pi |x|), the limit w -> 0 of
                         the 3D Helmholtz G; lsp_setup takes w = 0 and the
                         potential V in place of the medium m */
} lsp_equation;

typedef struct {
  double tol;        /* relative residual ||g - A u|| / ||g|| to reach (1e-8) */
  int restart;       /* GMRES restart length (30), 1..31 */
  int max_iters;     /* total Arnoldi steps allowed per right-hand side (1000) */
  int precision;     /* lsp_precision (LSP_FP64) */
  int buffer_b;      /* b of Section 3.1: boundary far sets exclude offsets
                        within b of the boundary plane (2); 1 <= b < n/2 */
  int leaf;          /* nested-dissection leaf side in grid points (0 = auto) */
  int panel;         /* frontal LU panel width: 0 = auto (32) or 32 */
  int dense_sweeps;  /* 1 (default): on the tree levels with at most 16
                        fronts, at least two panels and fronts of at most
                        1024 rows, lsp_factor also forms each front's
                        forward and backward sweep operators (2 m p entries
                        per front) and the sweeps apply them as dense
                        products; in plans for blocks of right-hand sides
                        (max_nrhs >= 4) the levels of more than 16 fronts
                        of at most 64 pivots and 256 rows are swept by
                        panel chains on the matrix cores (one wave per
                        front and group of 16 right-hand sides); 2: those
                        small-front levels whatever max_nrhs; 0: every
                        level uses the panel chain (or the blocked
                        sweeps) */
  int blocked_sweeps; /* 1 (default): on the levels (not swept with dense
                        operators) whose fronts have more than 1024 rows,
                        or with at most 32 fronts of more than two panels,
                        the sweeps run blocked: a panel chain per 256-row
                        super-block of the pivots and wide matrix-vector
                        products for the rest of the front; 2: every
                        level that is neither swept densely nor by the
                        small-front kernels; 0: the panel chain of one
                        workgroup per front */
  int self_term;     /* k_0, the kernel table's self term (Section 2.1 uses a
                        local quadrature correction it does not print):
                        0 (default): the integral of G over the disk (2D) /
                        ball (3D) of one cell's area / volume; 1: the
                        integral of G over the grid cell itself (square /
                        cube of side h), by Gauss-Legendre quadrature of
                        its closed-form radial integral; 2: the one-point
                        correction of the trapezoid rule (fourth order)
                        fitted so that the corrected rule integrates G
                        times a unit Gaussian of width max(0.05, 3h)
                        exactly (lsp_self_term) */
  int equation;      /* lsp_equation (LSP_HELMHOLTZ); LSP_LAPLACE needs d = 3 */
  const char* tile_cache; /* NULL (default), or a text file of tuned
                        trailing-update tile tables, one line per
                        (n, d, precision): lsp_plan_create takes the tiles
                        from the line of its (n, d, precision) when the file
                        has one with the plan's level count (a missing file
                        or malformed line is ignored); the string is read
                        during lsp_plan_create only */
} lsp_options;

typedef struct {
  int iters;            /* total Arnoldi steps for this right-hand side */
  int converged;        /* 1 if the true relative residual met tol */
  double relres_true;   /* ||g - A u|| / ||g||, recomputed in complex128 */
  double relres_est;    /* GMRES estimate at the last step */
  double t_setup;       /* milliseconds of the problem's lsp_setup work on the
                           device (HIP events on its stream, kernel table to
                           matrix M), the same for every right-hand side */
  double t_factor;      /* milliseconds of its last lsp_factor on the stream
                           (the factorisation and the pivot report; the
                           operator formation on the side stream overlaps
                           it and is not included) */
  double t_solve;       /* milliseconds of this lsp_solve on the stream, from
                           its first launch to its last report */
} lsp_rhs_info;

typedef struct {
  int n, d, N, L;             /* grid size, N = n^d, FFT length L = 2n */
  int nfronts, nlevels;       /* nested-dissection tree nodes and levels */
  int max_front, max_pivots;  /* largest front order and fully-summed block */
  double factor_entries;      /* stored L and U entries over all fronts */
  double front_entries;       /* sum of squared front orders (storage) */
  double factor_flops;        /* real flops of the numeric factorisation */
  double sweep_entries;       /* factor entries one forward (or backward) sweep
                                 reads: panels below / right of each diagonal
                                 block plus the inverted diagonal blocks */
  double update_flops;        /* real flops of the trailing-update products
                                 F22 -= L21 U12 (the MFMA part of the factor) */
  double panel_blocks;        /* diagonal-block factorisations per lsp_factor:
                                 the sum over fronts of ceil(p / panel) */
  double fused_blocks;        /* of those, the ones not factored by a
                                 diagonal-block launch of their own: inside
                                 the previous panel's update launch
                                 (lookahead), by the panel-strip launches
                                 of the upper levels (complex64), or, on the
                                 two-panel levels, the second panel's block
                                 by the cross-update launch; depends on the
                                 tile table and the plan's precision */
  double fused_update_flops;  /* of update_flops, the part in update
                                 launches that also factor a block */
  double dense_entries;       /* entries of the formed dense sweep operators
                                 one forward (or backward) sweep reads (sum
                                 of m p over the dense levels' fronts; those
                                 levels' panels are not in sweep_entries) */
  int dense_levels;           /* tree levels swept with dense operators */
  int blocked_levels;         /* tree levels swept blocked (blocked_sweeps) */
  double blocked_entries;     /* entries of the formed 256 x 256 super-block
                                 operators one forward (or backward) sweep
                                 reads on the blocked levels (their panels
                                 outside the super-blocks' diagonal blocks
                                 are in sweep_entries) */
  double chain_entries;       /* of sweep_entries, the part on the levels swept
                                 by panel chains (neither dense nor blocked) */
  double blocked_panel_entries; /* factor entries one sweep's matrix-vector
                                 products read on the blocked levels (each
                                 super-block's columns below it, or its rows
                                 right of it, outside its diagonal block) */
  double trsm_flops;          /* real flops of the panel products U12 =
                                 L11^{-1} P F12, L21 = F21 U11^{-1} run as
                                 launches of their own (the rest run inside
                                 the panel-strip launches) */
  double assemble_entries;    /* front entries the assembly writes plus the
                                 children's update-matrix entries it reads */
  int mchain_levels;          /* small-front levels swept by panel chains
                                 on the matrix cores (dense_sweeps) */
  double mchain_entries;      /* factor entries one sweep of them reads
                                 (inverse diagonal blocks and the panels'
                                 entries below or right of them) */
  double pair_update_flops;   /* of update_flops, the two-panel products
                                 over [k0 + kb, m)^2 (kb the two panels'
                                 columns) on the levels of large fronts */
  double cross_update_flops;  /* of update_flops, the first panel's update
                                 of the second panel's column and row
                                 strips on those levels */
  double mchain_pivots;       /* of the matrix-core levels' fronts: the sum of
                                 p (rows gathered from / scattered to the
                                 grid), */
  double mchain_rows;         /* the sum of p + q (front vector rows), and */
  double mchain_child_rows;   /* the sum of their children's q (update rows
                                 the forward sweep adds in) */
  int domain_points;          /* grid points of the domain: N, or |Omega| of a
                                 general-domain plan */
  int boundary_points;        /* general domains: points of Omega with a
                                 neighbour outside Omega (or the grid) */
  int sketch_cols;            /* general domains: columns r of the sketch */
} lsp_plan_stats;

typedef struct lsp_plan lsp_plan;        /* opaque; host-side, plus one device copy of
                                           its constant arrays per device used */
typedef struct lsp_problem lsp_problem;  /* opaque, owns no device memory */

/* Defaults: tol 1e-8, restart 30, max_iters 1000, FP64, b = 2, auto leaf and
 * panel.  Returns LSP_ERR_ARG on a null pointer. */
lsp_status lsp_options_default(lsp_options* opts);

/* Host-side symbolic analysis (Section 2.2: nested dissection of the 3^d
 * stencil graph): recursive 1-wide separator planes, elimination tree,
 * front index lists and extend-add maps.  Integer work only; no device
 * memory is touched here.  max_nrhs bounds the right-hand sides of one solve.
 * The plan is immutable once created and may be shared by problems (also
 * from several threads).  The first lsp_setup on a device uploads the plan's
 * constant arrays (front descriptors, index lists, extend-add maps, class
 * geometry, FFT twiddles) to that device once; the plan owns that memory and
 * lsp_plan_destroy frees it, so destroy a plan only after its problems. */
lsp_status lsp_plan_create(int n, int d, int max_nrhs, const lsp_options* opts,
                           lsp_plan** plan);
void lsp_plan_destroy(lsp_plan* plan);
lsp_status lsp_plan_stats_get(const lsp_plan* plan, lsp_plan_stats* stats);

/* General domains (Section 4: the support Omega of m is not a rectangle).
 * mask: host array of n^d bytes, nonzero at the grid points of Omega (the
 * unknowns of the problem; m must vanish outside Omega), read during this
 * call only.  sketch_cols: columns r of the Gaussian sketch R (0 = 2 * 3^d,
 * a constant multiple of the stencil size as the section asks).  Points of
 * Omega whose whole 3^d block lies in Omega take the rectangle's interior
 * rows (Section 3.1); the others ("boundary points") take their own row
 * B(i, mu(i)), mu(i) = the 3^d block intersected with Omega, from the
 * sketch (lsp_setup_general).  The dissection is that of the n^d grid;
 * points outside Omega stay in it as identity rows of M and Q, decoupled
 * from Omega.  Helmholtz only (LSP_ERR_ARG for Laplace options, an empty
 * mask, a null mask, r outside [1, 4096]). */
lsp_status lsp_plan_create_general(int n, int d, int max_nrhs, const lsp_options* opts,
                                   const unsigned char* mask, int sketch_cols,
                                   lsp_plan** plan);

/* Trailing-update tile shape (32, 64 or 128: square MFMA tile of the
 * F22 -= L21 U12 products) per elimination-tree level, leaves first.  The
 * plan starts with a size heuristic; an autotuner may replace it.  Setting
 * tiles changes only the speed of later lsp_factor calls of problems built
 * on this plan, never their results' meaning (the products are the same,
 * rounding order aside).  get: copies min(cap, nlevels) entries and returns
 * LSP_OK.  set: n must equal nlevels and every entry be 32, 64 or 128,
 * else LSP_ERR_ARG.  Not thread-safe against a concurrent lsp_factor. */
lsp_status lsp_plan_get_tiles(const lsp_plan* plan, int* tiles, int cap);
lsp_status lsp_plan_set_tiles(lsp_plan* plan, const int* tiles, int n);
/* Writes the plan's tile table to the cache file `path` (the format
 * lsp_options.tile_cache reads: "n d precision nlevels t_0 ... t_{L-1}"),
 * replacing the line of the same (n, d, precision) and keeping the others;
 * the file is rewritten through a temporary and renamed.  LSP_ERR_ARG on a
 * null argument or when the file cannot be written. */
lsp_status lsp_plan_save_tiles(const lsp_plan* plan, const char* path);

/* Device bytes the caller must provide: *problem_bytes for lsp_setup (kernel
 * table, spectrum, stencils, matrix M, frontal factors),
 * *solve_bytes for lsp_solve with nrhs right-hand sides (Krylov basis,
 * FFT work arrays, solve buffers).  precision selects the factor type. */
lsp_status lsp_plan_bytes(const lsp_plan* plan, int precision, int nrhs,
                          size_t* problem_bytes, size_t* solve_bytes);

/* Set-up steps before the factorisation, all on the GPU:
 *   kernel table k_t (Section 2.1) with k_0 the cell integral of G,
 *   spectrum of its (2n)^d circulant embedding,
 *   the 3^d stencil null vectors alpha_c (eq:Fmin, eq:Emin, eq:Cmin) and
 *   C_c = alpha_c K(mu_c, mu_c) (Section 2.2),
 *   the stencil matrix M (eq:ABop) in N x 3^d form.
 * m_dev: [N] real double medium m (Helmholtz) or potential V (Laplace:
 * omega must be 0, V takes the place of w^2 m everywhere, and k_0 is the
 * w -> 0 limit of the Helmholtz self term: rho^2 / 2 for the ball, the
 * cube's potential at its centre for the cell), read during this call only.
 * ws_dev / ws_bytes: device workspace of at least problem_bytes; it must
 * outlive the problem.  stream: a hipStream_t (NULL = default stream).
 * precision comes from the plan's options.  Errors: LSP_ERR_ARG (w <= 0 or
 * not finite for Helmholtz, w != 0 for Laplace, null pointers, small
 * workspace), LSP_ERR_OOM (the plan's
 * first upload to this device), LSP_ERR_HIP.  Only enqueues device work. */
lsp_status lsp_setup(const lsp_plan* plan, double omega, const double* m_dev,
                     void* ws_dev, size_t ws_bytes, void* stream,
                     lsp_problem** problem);
/* lsp_setup for a plan of lsp_plan_create_general (Section 4).  R_dev: the
 * sketch, [r][N] real double on the device (row c = column c of the
 * section's N x r Gaussian matrix R; entries outside Omega are not used),
 * read during this call only.  Besides lsp_setup's steps it forms
 * T = (K w^2 m) R over Omega's columns (r K products on the GPU) and, per
 * boundary point i, alpha = the conjugate of the least left singular vector
 * of T(mu(i), :) (unit norm, centre entry real positive), which becomes
 * row i of Q and of M.  On such a problem every operator application
 * (lsp_apply_op, lsp_apply_K, lsp_solve) returns its output restricted to
 * Omega (zero outside), the iterates live on Omega, and an LSP_RHS_G
 * right-hand side must vanish outside Omega.  Errors as lsp_setup; also
 * LSP_ERR_ARG when the plan and the call do not match. */
lsp_status lsp_setup_general(const lsp_plan* plan, double omega, const double* m_dev,
                             const double* R_dev, void* ws_dev, size_t ws_bytes,
                             void* stream, lsp_problem** problem);
/* A general-domain problem's boundary rows (synchronises the stream):
 * points [nbnd] (int, linear grid indices, increasing), alpha [nbnd][27]
 * complex128 (slot q = sum_a (s_a+1) 3^a, zero for slots outside Omega),
 * sigma [nbnd][27] (singular values of T(mu(i), :), descending, zero-
 * padded); nbnd = lsp_plan_stats.boundary_points; host pointers, any may
 * be NULL.  LSP_ERR_ARG on a rectangle problem. */
lsp_status lsp_get_boundary_stencils(lsp_problem* problem, int* points_host, double* alpha_host,
                                     double* sigma_host);
void lsp_problem_destroy(lsp_problem* problem);

/* Numeric multifrontal LU of M (Section 2.2, nested dissection and the
 * multifrontal method), level by level from the leaves, with partial
 * pivoting inside each front's fully-summed block.  On the dense sweep
 * levels (lsp_options.dense_sweeps) it then forms each front's forward and
 * backward sweep operators from the factor, on a side stream the library
 * keeps per device (default priority; each level's formation waits for that
 * level's factorisation through an event); the next sweeps on the problem's
 * stream, the next lsp_factor and lsp_problem_destroy wait for it.  Waits
 * for the stream to report the pivot-health figure (reduced on the device
 * into pinned host memory, which the calling thread polls), not for the
 * formation.  Errors: LSP_ERR_SINGULAR (in
 * some 32-wide panel the smallest pivot modulus |re| + |im| is at most 64
 * eps times the largest, or is NaN; eps of the factor precision),
 * LSP_ERR_HIP. */
lsp_status lsp_factor(lsp_problem* problem);

/* Restarted right-preconditioned GMRES (Section 3.3), one independent
 * Krylov process per right-hand side run in lockstep, each identical to
 * its solo run.  rhs_dev: [nrhs][N] complex128 (u_I or g per rhs_kind);
 * u_dev: [nrhs][N] complex128 output; ws_dev: >= solve_bytes for nrhs;
 * info_host: [nrhs] (may be NULL).  Synchronises the stream: the stopping
 * decisions are taken on the device, which reports the number of right-hand
 * sides still iterating into pinned host memory (allocated per problem on
 * the first solve, and again when nrhs grows); the calling thread polls it
 * after each Arnoldi step and cycle (a busy wait, no device-to-host copy).
 * Errors: LSP_ERR_STATE (not factored), LSP_ERR_ARG, LSP_ERR_NOCONV,
 * LSP_ERR_HIP (also when the stream ends without the report). */
lsp_status lsp_solve(lsp_problem* problem, int nrhs, int rhs_kind,
                     const void* rhs_dev, void* u_dev, void* ws_dev,
                     size_t ws_bytes, lsp_rhs_info* info_host);

/* ---- single steps of the path (each enqueued on the problem's stream) ---- */

/* y = x + K (w^2 m .* x)   (eq:lso), by zero-padded FFT convolution.
 * precision LSP_FP64: x, y complex128; LSP_MIXED: the convolution runs in
 * complex64 (x, y still complex128).  ws_dev as for lsp_solve(nrhs). */
lsp_status lsp_apply_op(lsp_problem* problem, int nrhs, int precision,
                        const void* x_dev, void* y_dev, void* ws_dev, size_t ws_bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operator y = x + K (w^2 m .* x) of lsp_apply_op, with the FFT work array
 * in a static per-device scratch array of 32 MiB instead of a caller
 * workspace.  Calls no allocator.  Requires nrhs (2n)^d elements of 16 bytes
 * (LSP_FP64) or 8 bytes (LSP_MIXED) to fit in 32 MiB, else LSP_ERR_ARG with
 * the sizes in the message (e.g. 2D n = 256: up to 8 right-hand sides in
 * FP64).  Every call on a device shares that device's scratch and its
 * contents persist between calls (nothing in it needs clearing: each call
 * writes every element it reads before reading it); calls that overlap on
 * one device, on different streams, race.  x_dev, y_dev: [nrhs][N]
 * complex128.  Results equal lsp_apply_op's bit for bit. */
lsp_status lsp_apply_op_noalloc(lsp_problem* problem, int nrhs, int precision,
                                const void* x_dev, void* y_dev);

/* y = K x  (the plain convolution; g = K(-w^2 m u_I) uses it). */
lsp_status lsp_apply_K(lsp_problem* problem, int nrhs, int precision,
                       const void* x_dev, void* y_dev, void* ws_dev, size_t ws_bytes);

/* y = Q x with Q = [A; B] (eq:PC); complex128 in and out. */
lsp_status lsp_apply_Q(lsp_problem* problem, int nrhs, const void* x_dev, void* y_dev);

/* x = M^{-1} z with the multifrontal factors, complex128 in and out (the
 * factors' precision is the problem's).  ws_dev as for lsp_solve(nrhs). */
lsp_status lsp_solve_M(lsp_problem* problem, int nrhs, const void* z_dev, void* x_dev,
                       void* ws_dev, size_t ws_bytes);

/* x = M^{-1} Q v  (the preconditioner of eq:PC). */
lsp_status lsp_apply_precond(lsp_problem* problem, int nrhs, const void* v_dev, void* x_dev,
                             void* ws_dev, size_t ws_bytes);

/* Copies out (synchronising the stream):
 *   kernel table: (n+1)^d complex128 on the device, index t1 + (n+1) t2 (+ ...);
 *   stencils: alpha [3^d][3^d] complex128 (padded slot q = sum_a (s_a+1) 3^a,
 *             zero outside the class), sigma [3^d][3^d] double (singular
 *             values of each class, descending, zero-padded), C like alpha;
 *             host pointers, any may be NULL;
 *   matrix: M as [N][3^d] complex128 on the device (slot as above, zero
 *             where the neighbour is outside the grid). */
lsp_status lsp_get_kernel_table(lsp_problem* problem, void* k_dev);
lsp_status lsp_get_stencils(lsp_problem* problem, double* alpha_host, double* sigma_host,
                            double* C_host);
lsp_status lsp_get_matrix(lsp_problem* problem, void* mval_dev);

/* The scattered field away from the grid (Section 1: once u is known on
 * Omega, u(x) = - int G(x - y) w^2 m(y) (u(y) + u_I(y)) dy everywhere, which
 * meets the radiation condition), by the grid quadrature of Section 2.1:
 *   lsp_exterior_field: u(x_p) = - sum_j h^d G(x_p - x_j) w^2 m_j
 *       (u_j + u_I,j) at points_dev [npts][d] (the cell-centred grid
 *       x_j = (j + 1/2) h; a point equal to a grid point takes k_0 there,
 *       so at the grid points it returns the solution itself);
 *   lsp_far_field: the far-field pattern A(xhat_p) = - c_d sum_j h^d
 *       e^{-i w xhat_p . x_j} w^2 m_j (u_j + u_I,j) for unit directions
 *       dirs_dev [ndirs][d], with u(x) = A(xhat) e^{i w |x|} |x|^{-(d-1)/2}
 *       + O(|x|^{-(d+1)/2}), c_2 = e^{i pi/4} / sqrt(8 pi w), c_3 = 1/(4 pi).
 * u_dev, uI_dev: [nrhs][N] complex128 (the solution of lsp_solve and the
 * incident field); out_dev: [nrhs][npts] complex128; all device pointers.
 * ws_dev: device workspace of lsp_field_bytes(plan, npts) bytes.  Helmholtz
 * problems only; a general-domain problem's u vanishes outside Omega and is
 * used as is.  Only enqueues device work.  Errors: LSP_ERR_ARG (null
 * pointers, counts < 1, Laplace problems, small workspace), LSP_ERR_HIP. */
lsp_status lsp_field_bytes(const lsp_plan* plan, int npts, size_t* bytes);

/* The kernel table's self term k_0 (Section 2.1) for grid step h,
 * frequency omega (0: the 3D Laplace kernel) and mode (lsp_options.
 * self_term): mode 2 is k_0 = int G g dx - sum_{t != 0} h^d G(h t) g(h t)
 * for g(x) = exp(-|x|^2 / (2 sigma^2)), sigma = max(0.05, 3h) (the integral
 * in closed form, the lattice sum over 0 < |t| h <= 12 sigma; cached per
 * (h, omega, d) since it takes up to a second at large n).  Host-only
 * computation; k0[0], k0[1] receive the real and imaginary parts.  Errors:
 * LSP_ERR_ARG. */
lsp_status lsp_self_term(double h, double omega, int d, int mode, double* k0);
lsp_status lsp_exterior_field(lsp_problem* problem, int nrhs, const void* u_dev, const void* uI_dev,
                              int npts, const double* points_dev, void* out_dev, void* ws_dev,
                              size_t ws_bytes);
lsp_status lsp_far_field(lsp_problem* problem, int nrhs, const void* u_dev, const void* uI_dev,
                         int ndirs, const double* dirs_dev, void* out_dev, void* ws_dev,
                         size_t ws_bytes);

/* ---- kernel timing (profiling aid) ----
 * When enabled, every kernel launch of the library is bracketed by two HIP
 * events recorded on the stream the kernel runs on.  lsp_timing_count()
 * waits for the recorded events and returns the number of distinct kernels
 * seen (-1 on a HIP error); lsp_timing_get(i, ...) reports kernel i's name
 * (with a [c128]/[c64] tag for templated kernels), the summed event-to-event
 * milliseconds and the launch count.  Process-wide, thread-safe; adds a few
 * microseconds per launch while enabled. */
lsp_status lsp_timing_enable(int enable);
lsp_status lsp_timing_reset(void);
int lsp_timing_count(void);
lsp_status lsp_timing_get(int i, char* name, size_t len, double* total_ms, long long* launches);

const char* lsp_status_string(lsp_status s);
/* Copies the calling thread's last error message (NUL-terminated). */
void lsp_last_error(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* LSP_H */
