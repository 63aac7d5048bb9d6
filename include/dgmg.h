/*
 * dgmg.h - C ABI of the MI355X (gfx950) p-multigrid Poisson solver for nodal
 * discontinuous Galerkin discretisations on Cartesian grids.
 *
 * Method: Stiller, "Robust multigrid for high-order discontinuous Galerkin
 * methods: a fast Poisson solver suitable for high-aspect ratio Cartesian
 * grids" (arXiv:1603.02524).  The library solves A u = g, the unified IP/LDG
 * nodal DG system of eq. (discrete problem), with the inexact
 * multigrid-preconditioned conjugate gradient method (Alg. 2), a polynomial
 * multigrid V-cycle (Alg. 1) and overlapping additive Schwarz smoothers with
 * element-centred (EA) or face-centred (FA) subdomains solved by fast
 * diagonalisation (Sec. 3.1).  3D and non-periodic (homogeneous Dirichlet)
 * grids extend the paper's 2D periodic setting.
 *
 * Conventions for every entry point below
 * ---------------------------------------
 * Vector layout: element-major GLL order.  For level l with order P_l and
 *   N_P = P_l + 1 nodes per direction, entry
 *     e * N_P^D + (k * N_P + j) * N_P + i,   e = m1 + N1 * (m2 + N2 * m3)
 *   holds the coefficient u_{ijk} of element (m1, m2, m3) (all 0-based,
 *   direction 1 fastest; in 2D k and m3 are absent).
 * Memory: every vector argument is a caller-owned DEVICE pointer (e.g. the
 *   data pointer of a torch tensor on the GPU) unless stated otherwise; the
 *   library never frees caller memory.  The handle owns its host tables; all
 *   device scratch and tables live in one workspace the caller allocates and
 *   binds (dgmg_workspace_bytes / dgmg_bind_workspace).
 * Streams: work is enqueued asynchronously on the handle's stream (a
 *   hipStream_t passed as void*; NULL = default stream) unless stated
 *   otherwise.  A handle must not be used from two host threads at once.
 * dtype: DGMG_F64 (double) or DGMG_F32 (float) selects the element type of
 *   the vector arguments of level operations; tables exist in both precisions.
 * Continuous counterpart (opts.disc = DGMG_DISC_SE; Sec. 4.3 compares it with
 *   the DG method): C0 spectral elements of order P on the same grid, system
 *   matrix by direct stiffness summation of the GLL element Laplacians, the
 *   same V-cycle and MGCG, and the element-centred weighted additive smoother
 *   (DGMG_SMOOTHER_EA only) on continuous subdomains: element m's nodes plus
 *   N_O node layers of each neighbour beyond the shared boundary node, N_O =
 *   (the DG overlap value) - 1, so that the subdomain covers the same region
 *   and excludes the same node layer as the DG one (the DG subdomain counts
 *   the neighbour node coinciding with the element's own as a layer); overlap
 *   width eta_{N_O+1} + 1; weights of eq. (weight function:ec).  Vectors of
 *   such a handle are LATTICE vectors: per direction the node positions
 *   g = m P + i (neighbouring elements share g = m P); a Dirichlet direction
 *   stores g = 1 .. N P - 1 at index g - 1 (nl = N P - 1 entries), a periodic
 *   one g mod N P (nl = N P); entry s1 + nl1 (s2 + nl2 s3).  3D needs P <= 16;
 *   flux, beta and mu_star are ignored; batches take DG grids only.
 * Errors: 0 on success; > 0 non-fatal status (DGMG_NOT_CONVERGED,
 *   DGMG_FELLBACK); < 0 error
 *   (DGMG_EINVAL bad argument, DGMG_EHIP runtime failure, DGMG_ENOMEM
 *   workspace missing or too small, DGMG_EUNSUPPORTED configuration not
 *   built, DGMG_ENONFINITE NaN/Inf met).  dgmg_last_error() returns the
 *   message of the most recent failure on that handle.  No exception or
 *   signal crosses the ABI.
 */
#ifndef DGMG_H
#define DGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGMG_OK 0
#define DGMG_NOT_CONVERGED 1
#define DGMG_FELLBACK 2 /* learned weights rejected by the probe; fixed weights kept */
#define DGMG_EINVAL (-1)
#define DGMG_EHIP (-2)
#define DGMG_ENOMEM (-3)
#define DGMG_EUNSUPPORTED (-4)
#define DGMG_ENONFINITE (-5)

#define DGMG_F64 0
#define DGMG_F32 1

#define DGMG_FLUX_IP 0  /* interior penalty fluxes (Sec. 2.3) */
#define DGMG_FLUX_LDG 1 /* local DG fluxes with parameter beta (Sec. 2.3) */

#define DGMG_SMOOTHER_EA 0 /* element-centred weighted additive Schwarz */
#define DGMG_SMOOTHER_FA 1 /* face-centred weighted additive Schwarz */
#define DGMG_SMOOTHER_EM 2 /* element-centred multiplicative Schwarz */
#define DGMG_SMOOTHER_FM 3 /* face-centred multiplicative Schwarz */

/* Subdomain order of the multiplicative smoothers (Sec. 3.1): */
#define DGMG_ORDER_LEX 0    /* one after another, lexicographic (direction 1 fastest) */
#define DGMG_ORDER_COLOUR 1 /* colour classes of subdomains that share no node and no
                               matrix entry, each class solved at once */

#define DGMG_OVERLAP_LEVEL (-1)       /* N_O = 1 + round(P_l / 8) on each level */
#define DGMG_OVERLAP_LEVEL_FLOOR (-2) /* N_O = 1 + floor(P_l / 8) as printed */
/* N_O >= 0: the same overlap on every level (0 = the paper's "0" variants) */

#define DGMG_WEIGHT_QUINTIC 0
#define DGMG_WEIGHT_CUBIC 1
#define DGMG_WEIGHT_ARITH 2 /* arithmetic averaging (phi~ = 0) */
#define DGMG_WEIGHT_NONE 3  /* conventional additive Schwarz (phi = 1) */

#define DGMG_VCYCLE_CLASSICAL 0 /* (N_S1, N_S2) on every level */
#define DGMG_VCYCLE_VARIABLE 1  /* counts doubled on each coarser level */

#define DGMG_DISC_DG 0 /* nodal DG (eq. (discrete problem)) */
#define DGMG_DISC_SE 1 /* the continuous spectral-element counterpart (Sec. 4.3), see below */

#define DGMG_PREC_FP64 0  /* everything in double precision */
#define DGMG_PREC_MIXED 1 /* V-cycle in float (coarse solve in double) inside FP64 PCG */

typedef struct dgmg_handle dgmg_handle;
typedef struct dgmg_batch dgmg_batch;

/* Cartesian grid (Sec. 2.2).  dx[d] points to n_elem[d] HOST doubles > 0. */
typedef struct {
  int dim;              /* 2 or 3 */
  int n_elem[3];        /* elements per direction (>= 1; >= 3 if periodic) */
  const double* dx[3];  /* element sizes Delta x_d^m per direction */
  int periodic[3];      /* 0: homogeneous Dirichlet, 1: periodic */
} dgmg_grid;

typedef struct {
  int P;             /* top-level order, 1 <= P <= 32: compiled kernels for P_l in 1,2,3,4,6,8,12,16,32,
                        run-time kernels (same results, slower) for the other orders; 3D takes
                        P <= 17 or P = 32 (the run-time patch tiles must fit the LDS) */
  int flux;          /* DGMG_FLUX_IP or DGMG_FLUX_LDG */
  double beta[3];    /* LDG parameter per direction (Sec. 2.3); ignored for IP */
  double mu_star;    /* penalty factor mu_star > 0 of mu = mu_0 (1 + mu_star) */
  int smoother;      /* DGMG_SMOOTHER_* */
  int overlap;       /* DGMG_OVERLAP_LEVEL, DGMG_OVERLAP_LEVEL_FLOOR or N_O >= 0 */
  int weighting;     /* DGMG_WEIGHT_* */
  int vcycle;        /* DGMG_VCYCLE_* */
  int ns_pre;        /* pre-smoothing steps N_S1 (>= 0) */
  int ns_post;       /* post-smoothing steps N_S2 (>= 0) */
  int precision;     /* DGMG_PREC_* */
  int max_iter;      /* i_max of Alg. 2 */
  int order;         /* DGMG_ORDER_* (multiplicative smoothers; ignored otherwise) */
  int disc;          /* DGMG_DISC_* (default DGMG_DISC_DG) */
} dgmg_opts;

/* Statistics of one dgmg_solve call (host struct, filled on return). */
typedef struct {
  int iterations;          /* PCG iterations performed */
  int converged;           /* 1 if ||r|| and ||g - A x|| are <= tol ||r_0|| */
  double r0;               /* ||g - A x_0||_2 */
  double r_final;          /* ||r|| of the recursively updated residual at exit */
  double rho;              /* (r_final / r0)^(1/iterations), eq. (rho) */
  double history[256];     /* ||r_i||, i = 0..min(iterations, 255) */
  double r_true;           /* ||g - A x||_2 at the last exit check (0 if none ran) */
  int replacements;        /* exit checks that failed: r replaced by g - A x */
} dgmg_stats;

/* Fill *o with the defaults: IP, beta = 0, mu_star = 1, FA, level overlap,
 * quintic weights, classical V(1,1), FP64, max_iter = 100.  P is set to 4. */
int dgmg_opts_default(dgmg_opts* o);

/* Host-side setup (Sec. 2.4, Sec. 3.1, Sec. 3.2): builds the level series
 * P_L = P, P_{l-1} = floor(P_l / 2), ..., 1; per level the 1D DG operators of
 * eq. (L:generic) with their face penalties; per subdomain and direction the
 * generalised eigenpairs of (L_{s,d}, M_{s,d}) and the 1D weights; the
 * embedded interpolation; and the global 1D eigenpairs used for the exact
 * coarse solve.  All in double precision on the host.  No device memory is
 * touched.  On success *out owns a new handle (free with dgmg_destroy).
 * Errors: DGMG_EINVAL for dim not in {2,3}, P out of range, n_elem < 1,
 * dx <= 0 or not finite, mu_star <= 0, |beta| > 1, periodic with n_elem < 3,
 * bad enum values, more than 2^31 - 1 unknowns on the top level;
 * DGMG_EUNSUPPORTED for (P, N_O) pairs without kernels. */
int dgmg_setup(const dgmg_grid* g, const dgmg_opts* o, dgmg_handle** out);

/* Bytes of device workspace the handle needs (tables, level vectors, patch
 * buffers, PCG vectors, reduction scratch).  *bytes is a host size_t. */
int dgmg_workspace_bytes(const dgmg_handle* h, size_t* bytes);

/* Bind caller-allocated device memory of at least dgmg_workspace_bytes bytes
 * (256-byte aligned) and upload the tables on `stream` (synchronised before
 * return).  The memory must stay valid until dgmg_destroy or the next bind. */
int dgmg_bind_workspace(dgmg_handle* h, void* dev, size_t bytes, void* stream);

/* Change the stream later work is enqueued on. */
int dgmg_set_stream(dgmg_handle* h, void* stream);

/* Number of levels L + 1 and, per level l (0 = coarsest), its order P_l,
 * overlap N_O,l and number of unknowns (host outputs; NULL allowed). */
int dgmg_num_levels(const dgmg_handle* h);
int dgmg_level_info(const dgmg_handle* h, int level, int* P, int* n_o, int64_t* n_dof);

/* Host copy of the 1D node coordinates of level `level` in direction d
 * (n_elem[d] * (P_l + 1) doubles, element by element; element map of
 * Sec. 2.2 with the grid starting at 0).  Continuous handles: the nl stored
 * lattice nodes of the direction. */
int dgmg_node_coords(const dgmg_handle* h, int level, int d, double* x_host);

/* y = A_l x (eq. (discrete problem); sum factorised).  x, y: device vectors
 * of level l, distinct. */
int dgmg_apply(dgmg_handle* h, int level, const void* x, void* y, int dtype);

/* r = f - A_l x (residual form of Sec. 3.1).  r must not alias x. */
int dgmg_residual(dgmg_handle* h, int level, const void* f, const void* x, void* r, int dtype);

/* nsteps Schwarz iterations on level l >= 1 (Smoother of Alg. 1): EA = one
 * additive sweep over all element-centred subdomains per step; FA = one sweep
 * per orientation d = 1..D in sequence, the residual recomputed before each
 * (eq. (correction:global), eq. (weight function:ec), eq. (weight
 * function:fc)).  EM / FM (multiplicative, Sec. 3.1): the subdomains of a
 * partition one after another (DGMG_ORDER_LEX) or colour class by colour
 * class (DGMG_ORDER_COLOUR), each on the residual left by the previous ones,
 * u += R_s^T A_ss^{-1} R_s (f - A u) unweighted; FM sweeps the orientations
 * d = 1..D; every second step of one call runs backwards (reversed subdomain
 * and orientation order), so an even nsteps is symmetric.  Colour classes:
 * per direction the subdomain indices modulo k (k = 2 along the face-centred
 * normal and without overlap, 3 with overlap), on a periodic direction whose
 * count is not a multiple of k the last (count mod k) indices one by one;
 * classes in lexicographic order of their per-direction colours (direction 1
 * fastest).  u is updated in place; f unchanged. */
int dgmg_smooth(dgmg_handle* h, int level, void* u, const void* f, int nsteps, int dtype);

/* One additive Schwarz sweep over one partition of level l >= 1 (Sec. 3.1):
 * u += sum_s R_s^T (w_s (.) A_ss^{-1} R_s (f - A_l u)).  normal = -1: the
 * element-centred partition; normal = d: the face-centred partition with
 * faces normal to direction d.  Either kind may be used whatever the
 * handle's additive smoother (DGMG_EUNSUPPORTED if no patch kernel exists
 * for the tile).  A multiplicative handle (EM, FM) runs one forward
 * multiplicative sweep instead, over its own kind of partition only
 * (DGMG_EINVAL otherwise).  Uses the level's internal residual scratch. */
int dgmg_sweep(dgmg_handle* h, int level, void* u, const void* f, int normal, int dtype);

/* f_{l-1} = I_l^T r_l: restriction by the transpose of the embedded
 * interpolation (Sec. 3.2).  level >= 1. */
int dgmg_restrict(dgmg_handle* h, int level, const void* r_fine, void* f_coarse, int dtype);

/* u_l += I_l u_{l-1}: prolongation by embedded interpolation.  level >= 1. */
int dgmg_prolong(dgmg_handle* h, int level, const void* u_coarse, void* u_fine, int dtype);

/* u_0 = A_0^+ f_0 on the coarsest level (P = 1), line of Alg. 1: computed
 * exactly by global fast diagonalisation of the Kronecker-sum operator, in
 * double precision (float vectors are converted).  For periodic grids f_0 is
 * made orthogonal to the constants and the mean-free solution is returned. */
int dgmg_coarse_solve(dgmg_handle* h, const void* f0, void* u0, int dtype);

/* z = MultigridCycle(0, r) (Alg. 1) on the top level.  In mixed precision the
 * V-cycle runs in float; r and z are then float vectors (dtype DGMG_F32). */
int dgmg_vcycle(dgmg_handle* h, const void* r, void* z, int dtype);

/* Solve A x = rhs by MGCG (Alg. 2, with beta = z^T (r - r_old) / delta) until
 * ||r||_2 <= tol ||rhs - A x_0||_2 or max_iter iterations.  The exit test on
 * the recursively updated residual r is confirmed by the true residual
 * rhs - A x (FP64): only when that also meets the bound does the solve stop;
 * otherwise r is replaced by the true residual and the iteration continues.
 * rhs, x: FP64
 * device vectors of the top level; x holds the initial guess on entry and the
 * iterate on exit.  Synchronises the stream once per iteration (exit test).
 * st (host, may be NULL) receives iteration count and residual history.
 * On a grid periodic in every direction A is singular (constants span its
 * null space) and rhs must sum to zero, |sum rhs| <= 1e-10 sum |rhs|; the
 * returned x is then determined up to a constant.
 * Returns DGMG_OK, DGMG_NOT_CONVERGED or an error (DGMG_EINVAL for a fully
 * periodic rhs that does not sum to zero, DGMG_ENONFINITE when a residual norm
 * is NaN/Inf). */
int dgmg_solve(dgmg_handle* h, const double* rhs, double* x, double tol, dgmg_stats* st);

/* g = M f: the GLL load vector of Sec. 2.4 from nodal values f (FP64 device
 * vectors of the top level; continuous handles: the assembled lumped mass). */
int dgmg_mass(dgmg_handle* h, const double* f_nodal, double* g);

/* Per-kernel timing with HIP events on the handle's stream.  enable = k >= 1
 * starts recording the top-level Schwarz patch-solve launches, every k-th one
 * (1: every launch; a stride keeps the event overhead out of most launches,
 * and a stride prime to the number of sweep normals samples them all), and
 * clears the totals; 0 stops.  dgmg_kernel_time reads, after synchronisation,
 * the summed milliseconds, launch count and algorithmic flops and bytes of the
 * recorded launches (host outputs; NULL allowed). */
int dgmg_kernel_timing(dgmg_handle* h, int enable);
int dgmg_kernel_time(dgmg_handle* h, double* total_ms, int64_t* launches, double* flops,
                     double* bytes);

/* Replay the two per-iteration phases of dgmg_solve (operator + update; V-cycle +
 * direction update) from hipGraphs captured on first use (enable != 0), or
 * launch them eagerly (0, the default).  Graphs are recaptured when x, the
 * stream or a tuning choice changes. */
int dgmg_use_graphs(dgmg_handle* h, int enable);

/* Autotuner: time the patch-solve block shapes (1, 2, 4 or 8 wavefronts per
 * patch) of every smoothing sweep on the bound workspace and keep the fastest
 * (synchronises; results are bitwise independent of the choice).
 * dgmg_tune_get/set read or impose the choice for (level >= 1, kind), kind
 * 0..2 = face-centred sweep normal to direction kind, 3 = element-centred;
 * waves 0 = built-in default.  ms: mean time of one launch when timed. */
int dgmg_autotune(dgmg_handle* h);
int dgmg_tune_get(const dgmg_handle* h, int level, int kind, int* waves, double* ms);
int dgmg_tune_set(dgmg_handle* h, int level, int kind, int waves);

/* Release host tables and HIP objects of the handle (not the workspace). */
void dgmg_destroy(dgmg_handle* h);

/* Message of the last failure on h (or of the last failed dgmg_setup when h
 * is NULL).  The string is owned by the library. */
const char* dgmg_last_error(const dgmg_handle* h);

/* ---------------------------------------------------------------- batches
 * Many independent grids (own sizes, orders, options) solved together:
 * MGCG runs in lock step with one host synchronisation per iteration for all
 * grids; converged grids are masked by a device flag that every kernel
 * checks.  When all grids share the multigrid precision, the smoothing counts
 * and the V-cycle kind, use additive smoothers and have no 3D P = 32 level,
 * each phase of an iteration is a work-list plan: every step of every grid's
 * phase is keyed by its position (the top-level apply; in the V-cycle the
 * depth below the top level, smoothing step, sweep, sub-step), and the steps
 * at one position that use the same kernel instance (order, tile, mode) run as
 * ONE launch over all those grids' elements or patches, with per-grid
 * argument descriptors in the workspace; vector updates, fills and coarse
 * solves stay per grid.  When a grid's top level has at least 2^20 unknowns
 * (its levels that large keep their own launches), the per-grid steps of one
 * position run round robin on three side streams the batch creates at bind
 * (default priority; forked from and joined back into the batch stream by
 * events) and overlap that position's shared launches; results do not depend
 * on it.  Otherwise each grid's chain is issued on its own.
 * Either way a phase is issued eagerly (the default; the per-grid
 * operations of converged grids are then left out) or captured once as a
 * hipGraph and replayed.  Vectors of all grids are
 * concatenated (FP64, element-major per grid) at the offsets reported by
 * dgmg_batch_offsets.  Extension beyond the paper (many-grid throughput). */

/* Set up `count` grids (host work only); grids[i], opts[i] as for dgmg_setup. */
int dgmg_batch_setup(int count, const dgmg_grid* grids, const dgmg_opts* opts, dgmg_batch** out);
int dgmg_batch_workspace_bytes(const dgmg_batch* b, size_t* bytes);
/* The execution plan (host outputs, NULL allowed): planned = 1 when the phases
 * run as work-list plans; kernels = batched launches per MGCG iteration (both
 * phases), grid_ops = per-grid operations per iteration. */
int dgmg_batch_plan_info(const dgmg_batch* b, int* planned, int* kernels, int* grid_ops);
/* Bind one caller-allocated device workspace (256-byte aligned) for all grids;
 * a planned batch also creates its three side streams and their events here
 * (released by dgmg_batch_destroy).  DGMG_EHIP if they cannot be created. */
int dgmg_batch_bind_workspace(dgmg_batch* b, void* dev, size_t bytes, void* stream);
/* Host array of count + 1 offsets of each grid's unknowns in the concatenation. */
int dgmg_batch_offsets(const dgmg_batch* b, int64_t* offsets);
/* Borrow the handle of grid i (level operations on one grid; do not destroy,
 * do not call dgmg_solve on it). */
int dgmg_batch_handle(dgmg_batch* b, int i, dgmg_handle** h);
/* Autotune every grid's sweeps (shapes with identical tiles and patch counts
 * are timed once). */
int dgmg_batch_autotune(dgmg_batch* b);
/* Graph replay of each phase on, or eager launches (the default: an eager
 * phase leaves out the per-grid operations of converged grids). */
int dgmg_batch_use_graphs(dgmg_batch* b, int enable);
/* Solve all grids to ||r_i|| <= tol ||r_i,0|| (each grid's own max_iter);
 * st: host array of count dgmg_stats (may be NULL).  DGMG_NOT_CONVERGED if
 * any grid stopped unconverged; DGMG_EINVAL if a fully periodic grid's part of
 * rhs does not sum to zero (as for dgmg_solve). */
int dgmg_batch_solve(dgmg_batch* b, const double* rhs, double* x, double tol, dgmg_stats* st);
const char* dgmg_batch_last_error(const dgmg_batch* b);
void dgmg_batch_destroy(dgmg_batch* b);

/* ---------------------------------------------------------- learned weights
 * Extension beyond the paper.  The face-centred smoother (FA) may replace the
 * fixed normal weights of its patches (eq. (weight function:fc) of Sec. 3.1,
 * read as w_F = 1/2 [1 + phi(1 - |xi_F|)]) by weights with a transition width
 * theta_f and a damping factor omega_f per face f:
 *   w_f = omega_f wt_f / (sum of wt_f' over the patches of the same
 *         orientation that cover the node),  wt_f = 1/2 [1 + phi((1 - |xi_F|) / theta_f)].
 * The normalisation keeps a partition of unity for omega = 1 whatever the
 * widths; theta = omega = 1 gives the fixed weights.  Lateral (element-centred)
 * weights are unchanged.
 *
 * Faces are enumerated level by level (l = 1 .. L, the smoothing levels),
 * then by normal direction d = 0 .. D-1, then face f = 0 .. nf_d - 1
 * (nf_d = N_d periodic, N_d + 1 Dirichlet; face f lies between elements f-1
 * and f).  A small MLP maps per-face features to (theta, omega):
 *   x (DGMG_MLP_IN) -> tanh(W1 x + b1) -> tanh(W2 h1 + b2) (DGMG_MLP_HIDDEN each)
 *   -> y = W3 h2 + b3 (DGMG_MLP_OUT),
 *   theta = THETA_MIN + (THETA_MAX - THETA_MIN) sigmoid(y0),
 *   omega = OMEGA_MIN + (OMEGA_MAX - OMEGA_MIN) sigmoid(y1).
 * Parameter vector (FP32, DGMG_MLP_PARAMS values): W1 (HIDDEN x IN, row-major),
 * b1, W2 (HIDDEN x HIDDEN), b2, W3 (OUT x HIDDEN), b3.  Features per face:
 *   P_l / 32, log2(dx_left / h_lat) / 5, log2(dx_right / h_lat) / 5,
 *   1 on a Dirichlet boundary face else 0, D - 2, N_O,l / (P_l + 1),
 * with dx_left / dx_right the normal sizes of the adjoining elements (the
 * existing one at a boundary face) and h_lat the geometric mean of all element
 * sizes of the other directions. */
#define DGMG_MLP_IN 6
#define DGMG_MLP_HIDDEN 64
#define DGMG_MLP_OUT 2
#define DGMG_MLP_PARAMS 4738
#define DGMG_THETA_MIN 0.25
#define DGMG_THETA_MAX 2.0
#define DGMG_OMEGA_MIN 0.5
#define DGMG_OMEGA_MAX 1.5

/* Number of faces of all smoothing levels (the length of the per-face arrays
 * below), or DGMG_EINVAL.  Host only; needs no workspace. */
int dgmg_face_count(const dgmg_handle* h);
/* Features of every face, host float array [count][DGMG_MLP_IN]. */
int dgmg_face_features(const dgmg_handle* h, float* X);
/* Impose (theta, omega) per face (host arrays of dgmg_face_count doubles,
 * finite and > 0), or restore the fixed weights with theta = omega = NULL.
 * FA smoother only (else DGMG_EUNSUPPORTED); needs a bound workspace;
 * synchronises the stream.  Captured graphs stay valid (tables are
 * overwritten in place). */
int dgmg_set_face_params(dgmg_handle* h, const double* theta, const double* omega);
/* Current (theta, omega) per face into host arrays; returns 1 when learned
 * parameters are in use, 0 for the fixed weights (all ones reported). */
int dgmg_get_face_params(const dgmg_handle* h, double* theta, double* omega);

/* MLP kernels (FP32, on `stream`; all arrays device, row-major, caller-owned).
 * forward: X [B][IN] -> Y [B][OUT]; work [B][2 HIDDEN] receives h1, h2.
 * backward: gradient of L = (1/B) sum_b sum_o (Y_bo - T_bo)^2 with respect to
 *   the parameters into grad [PARAMS] (overwritten), from the X, Y, work of the
 *   matching forward call; scratch holds B (2 HIDDEN + OUT) floats.  Sums over
 *   the batch run in sample order (reproducible).
 * adam: one Adam step (Kingma and Ba) on n parameters at step t >= 1:
 *   m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * dgmg_mlp_param_count returns DGMG_MLP_PARAMS. */
int dgmg_mlp_param_count(void);
int dgmg_mlp_forward(const float* params, const float* X, int B, float* Y, float* work, void* stream);
int dgmg_mlp_backward(const float* params, const float* X, const float* T, int B, const float* Y,
                      const float* work, float* grad, float* scratch, void* stream);
int dgmg_mlp_adam(float* params, const float* grad, float* m, float* v, int n, int t, float lr, float b1,
                  float b2, float eps, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * forward pass as dgmg_mlp_forward, without the work argument.  The hidden
 * activations go to a static device array of the library holding
 * DGMG_MLP_NOALLOC_MAX_ROWS rows (4 MiB, one copy per GPU, kept until the
 * process ends); its device address is looked up on the first call on each
 * device, with that device current.  The call allocates nothing.  B above
 * DGMG_MLP_NOALLOC_MAX_ROWS is rejected with DGMG_EINVAL (message in
 * dgmg_last_error(NULL)); B = 0 does nothing.  stream must belong to the
 * current device.  All calls on one GPU share the array (nothing in it needs
 * to start at zero: every call writes the rows it reads), so calls that
 * overlap on one GPU, on different streams or host threads, race. */
#define DGMG_MLP_NOALLOC_MAX_ROWS 8192
int dgmg_mlp_forward_noalloc(const float* params, const float* X, int B, float* Y, void* stream);

/* Device work bytes needed by dgmg_apply_mlp on this handle. */
int dgmg_mlp_work_bytes(const dgmg_handle* h, size_t* bytes);
/* Learned weights with fallback: evaluate the MLP (device params) on the
 * handle's face features, then probe both weight sets with probe_iters MGCG
 * iterations from x = 0 on a fixed pseudo-random right-hand side (the same for
 * both).  Keeps the learned weights when their residual reduction
 * ||r_k|| / ||r_0|| is no worse than that of the fixed weights (DGMG_OK), else
 * restores the fixed weights and returns DGMG_FELLBACK (also when the MLP
 * output is not finite or the probe breaks down).  work: device buffer of
 * dgmg_mlp_work_bytes bytes, 256-byte aligned.  ratios (host, may be NULL)
 * receives {learned, fixed} reductions.  Single (non-batch) handles; FA only;
 * synchronises. */
int dgmg_apply_mlp(dgmg_handle* h, const float* params, void* work, size_t bytes, int probe_iters,
                   double* ratios);

#ifdef __cplusplus
}
#endif
#endif /* DGMG_H */
