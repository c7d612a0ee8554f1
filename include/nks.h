/*
 * libnks -- C ABI of the MI355X (gfx950) Newton-Krylov-Schwarz hot path for
 * fully implicit compressible gas flow with the Peng-Robinson equation of
 * state (arXiv 2007.13966: Li, Yang, Yang, "multilevel restricted Schwarz
 * preconditioners").
 *
 * Conventions shared by every entry point
 *  - Cells of a reservoir are numbered lexicographically, x fastest:
 *    cell (x,y,z) -> x + nx*(y + ny*z); z grows downward (depth).
 *  - A grid may hold several independent reservoirs ("blocks") concatenated
 *    in one cell range; reservoir b owns cells [off[b], off[b+1]).  Newton,
 *    GMRES and the line search run independently per reservoir.
 *  - Unless stated otherwise a "double*" argument is a DEVICE pointer of
 *    length ncells owned by the caller; the library never frees it.
 *  - Work is enqueued on the grid's stream (hipStream_t passed as void*).
 *    Entry points returning statistics synchronise that stream.
 *  - Every call returns 0 (NKS_OK) or a negative NKS_E* code;
 *    nks_last_error() gives a thread-local message.  No C++ exception
 *    crosses the ABI.  Handles are not thread safe.
 *  - Units are SI: Pa, m, m^2 (permeability), kg/s (well rates, +injection),
 *    s, K, kg/mol, J/(mol K), Pa s.
 */
#ifndef NKS_H
#define NKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NKS_OK 0
#define NKS_EINVAL (-1)          /* bad argument or descriptor */
#define NKS_EHIP (-2)            /* HIP runtime error */
#define NKS_EZEROPIVOT (-3)      /* zero pivot in a subdomain ILU(0) factorization */
#define NKS_ENONPHYSICAL (-4)    /* p <= 0, Z <= B or a non-finite value */
#define NKS_ENOTCONVERGED (-5)   /* iteration limit or line-search failure; stats filled */
#define NKS_ENOMEM (-6)          /* allocation failed */

typedef struct nks_grid nks_grid;
typedef struct nks_matrix nks_matrix;
typedef struct nks_ras nks_ras;

/* Device allocator callback pair (e.g. a framework's caching allocator).
 * alloc returns a device pointer of at least `bytes` bytes or NULL. */
typedef void *(*nks_alloc_fn)(size_t bytes, void *ctx);
typedef void (*nks_free_fn)(void *ptr, void *ctx);

/* Fluid constants of Section 2: critical temperature Tc and pressure pc,
 * acentric factor omega (m(omega) of the first fit for omega <= 0.491, the
 * second above), temperature T, molar mass W, gas constant R, viscosity mu.
 * Tb > 0 (0 < Tb < Tc): normal boiling point; omega is then computed from it
 * by the correlation of Section 2 (omega = (-ln(pc / 1 atm) - f0(Tbr)) /
 * f1(Tbr), Tbr = Tb/Tc) and the omega given is ignored.  Tb = 0: omega used. */
typedef struct {
    double Tc, pc, omega, T, W, R, mu;
    double Tb;
} nks_fluid;

/* Boundary condition types of a reservoir's outer faces (Section 2: p = p^D
 * on the Dirichlet part of the boundary, v.n = q^N on the Neumann part). */
#define NKS_BC_CLOSED 0      /* no flow */
#define NKS_BC_DIRICHLET 1   /* value: p^D in Pa (> 0), the state at the face centre */
#define NKS_BC_NEUMANN 2     /* value: q^N = v.n in m/s, n the outward normal (inflow < 0) */

/* One reservoir: nx*ny*nz cells of size dx*dy*dz (2D: nz = 1, dz is the
 * thickness).  kx, ky, kz, phi: DEVICE arrays of nx*ny*nz values (diagonal
 * permeability tensor, porosity); read during nks_setup_grid only.
 * Wells: HOST arrays of nwells reservoir-local cell indices and mass rates.
 * bc_type, bc_value: HOST arrays of 6 entries for the outer faces in the
 * order -x, +x, -y, +y, -z, +z (the -z face is the top: depth grows with z),
 * each NKS_BC_* with its value; NULL for both: every face closed.  A
 * Dirichlet face flows through the one-sided transmissibility 2 K A / Delta
 * of its cells; a Neumann face adds the scaled mass flux m q^N A of each of
 * its cells, the density taken from the cell.  Read during nks_setup_grid
 * only; a bad type or a non-positive p^D is NKS_EINVAL. */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    const double *kx, *ky, *kz, *phi;
    int nwells;
    const int *well_cell;
    const double *well_rate;
    const int *bc_type;
    const double *bc_value;
} nks_reservoir_desc;

typedef struct {
    int nres;                        /* number of reservoirs, >= 1 */
    const nks_reservoir_desc *res;   /* HOST array of nres descriptors */
    nks_fluid fluid;
    int gravity;                     /* 0: g = 0 */
    double g;                        /* gravitational acceleration */
    void *stream;                    /* hipStream_t; NULL = default stream */
    nks_alloc_fn alloc;              /* NULL: hipMalloc / hipFree */
    nks_free_fn free;
    void *alloc_ctx;
    int accum;                       /* NKS_ACCUM_CONSERVATIVE (0) or NKS_ACCUM_CHAIN_RULE */
} nks_grid_desc;

/* Accumulation forms of the residual.  Conservative: (V phi/dt) times
 * m(p) - m(p^n) (BDF1) or (3 m(p) - 4 m(p^n) + m(p^{n-1}))/2 (BDF2), m = p/Z;
 * it conserves mass step by step and its linearisation at p is the paper's
 * coefficient.  Chain rule: the BDF1 and BDF2 equations of Section 2 as
 * printed, (V phi/dt) m'(p) times p - p^n or (3p - 4p^n + p^{n-1})/2, with
 * m'(p) = (p/Z)(1/p - Z'/Z) at the new level; its Jacobian adds m''(p) times
 * that difference.  The discrete adjoint (nks_adjoint) is defined for the
 * conservative form only. */
#define NKS_ACCUM_CONSERVATIVE 0
#define NKS_ACCUM_CHAIN_RULE 1

/* Builds the face transmissibilities T = A_f / (d/(2K_i) + d/(2K_j))
 * (two-point flux of the cell-centred scheme, Section 2 Remark 1), pore
 * volumes and the well source term Q R T / W.  Copies what it needs. */
int nks_setup_grid(const nks_grid_desc *desc, nks_grid **out);
/* Handles may be destroyed in any order: a grid's memory is released once its
 * own handle and every matrix and preconditioner made on it are destroyed
 * (they hold a reference to it), and a matrix's once its handle and every
 * preconditioner set up on it are; until then those stay usable. */
int nks_destroy_grid(nks_grid *g);
/* ncells: total cells; nres: reservoirs; offsets: HOST array of nres+1
 * (may be NULL). */
int nks_grid_info(const nks_grid *g, int *ncells, int *nres, int *offsets);

/* Hydrostatic initial state: p = p_top in the top layer and, down every
 * column, p_{k+1} - p_k = (rho_k + rho_{k+1})/2 g dz.  p: device, out. */
int nks_hydrostatic_init(nks_grid *g, double p_top, double *p);

/* Residual of the pressure form of the governing equation (Section 2)
 * integrated over each cell, in conservative form:
 *   F_i = (V phi_i / dt) Acc_i + sum_j T_ij lambda_up dPhi_ij - Q_i R T / W
 * with m = p/Z (Z the largest real root of the PR cubic), lambda = m/mu from the
 * upwind cell of dPhi_ij = (p_i - p_j) - (rho_i + rho_j)/2 g (h_i - h_j),
 * Acc = m - m^n (bdf_order 1, the BDF1 scheme of Section 2) or
 * (3m - 4m^n + m^{n-1})/2 (bdf_order 2, the BDF2 scheme of Section 2).
 * p, p_n, p_nm1 (ignored for order 1), F: device arrays.  Asynchronous. */
int nks_residual(nks_grid *g, const double *p, const double *p_n, const double *p_nm1,
                 double dt, int bdf_order, double *F);

/* Allocation-free form of nks_residual, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and the same F, bit for bit; its
 * intermediates (the BDF history term and the PR properties m, dm/dp of each
 * cell, the per-reservoir non-physical flags) live in one fixed device array
 * of the library instead of the grid's buffers.  That array holds
 * NKS_NOALLOC_MAX_CELLS cells (60 MiB plus 16 KiB), is kept on every GPU the
 * library runs on until the process ends, and is shared by all calls on that
 * GPU, which keep the last call's contents: calls that overlap on one GPU
 * (other streams or threads) race.  Larger grids (or more than 4096
 * reservoirs): NKS_EINVAL.  Calls no device or pinned-host allocation.
 * Asynchronous on the grid's stream. */
#define NKS_NOALLOC_MAX_CELLS 2621440
int nks_residual_noalloc(nks_grid *g, const double *p, const double *p_n, const double *p_nm1,
                         double dt, int bdf_order, double *F);

/* Sparse Jacobian dF/dp of nks_residual (Section 3, the Jacobian entries), stored
 * as a structured stencil (5 points in 2D, 7 in 3D), FP64.  Writes F too
 * when F != NULL.  J must come from nks_matrix_create on the same grid. */
int nks_matrix_create(nks_grid *g, nks_matrix **out);
int nks_destroy_matrix(nks_matrix *J);
int nks_jacobian(nks_grid *g, const double *p, const double *p_n, const double *p_nm1,
                 double dt, int bdf_order, nks_matrix *J, double *F);
/* nnz of the CSR form; export to HOST arrays (rowptr ncells+1, col/val nnz),
 * columns sorted, structural zeros at closed faces dropped.  Synchronises. */
int nks_matrix_nnz(const nks_matrix *J, int *nnz);
int nks_matrix_export_csr(const nks_matrix *J, int *rowptr, int *col, double *val);
/* y = J x and y = J^T x (device).  Asynchronous. */
int nks_matrix_apply(nks_matrix *J, const double *x, double *y);
int nks_jacobian_transpose_apply(nks_matrix *J, const double *x, double *y);
/* out = (dF/d theta)^T lam with theta_c = ln of a multiplier on all K
 * components of cell c (device arrays).  Asynchronous. */
int nks_residual_dlogk_transpose_apply(nks_grid *g, const double *p, const double *lam,
                                       double *out);

/* Multilevel restricted additive Schwarz preconditioner (Section 3).
 * Subdomains: px*py*pz boxes per reservoir, box q of P along n cells gets
 * floor(n/P) + (q < n mod P) cells, extended by `overlap` and clipped at the
 * domain boundary; the same box grid on every level.  Subdomain solve:
 * ILU(0) of R_i^delta A R_i^delta^T in local lexicographic order.
 * Levels: ratio r per direction (nz = 1 stays 1), the first- (1),
 * second- (2) or third-order (3) interpolation of Section 3.2, restriction
 * P^T, Galerkin coarse operators P^T A P; coarsest level solved by GMRES
 * with the one-level preconditioner to coarse_rtol (Remark 2). */
#define NKS_LEFT_RAS 0           /* Section 3.1 left-RAS (default) */
#define NKS_AS 1                 /* Section 3.1 classical AS */
#define NKS_RIGHT_RAS 2          /* Section 3.1 right-RAS */
#define NKS_VCYCLE 0             /* Section 3.2 V-cycle, mu/nu smoothing steps */
#define NKS_LEFT_KASKADE 1       /* Section 3.2 left Kaskade */
#define NKS_RIGHT_KASKADE 2      /* Section 3.2 right Kaskade */
#define NKS_ADDITIVE 3           /* Section 3.2 additive two-level */
#define NKS_COARSE_ONLY 4        /* Section 3.2 coarse-only */
#define NKS_FP64 0               /* factors and subdomain sweeps in FP64 */
#define NKS_FP32 1               /* FP32 factors, FP32 sweeps */
#define NKS_BF16 2               /* BF16 off-diagonal factors, FP32 1/diag and sweeps */

typedef struct {
    int px, py, pz;
    int levels;                  /* >= 1, at most 6 */
    int overlap[8];              /* per level, index 0 = finest */
    int variant;                 /* NKS_LEFT_RAS | NKS_AS | NKS_RIGHT_RAS */
    int interp_order;            /* 1, 2 (default), 3 */
    int cycle;                   /* NKS_VCYCLE ... */
    int mu, nu;                  /* smoothing steps of the V-cycle family */
    double coarse_rtol;          /* 0.2 in the paper */
    int coarse_maxit;
    int coarse_restart;
    int precision;               /* NKS_FP64 | NKS_FP32 | NKS_BF16 */
    int tx, ty, tz;              /* > 0: box edge in cells on the finest level, so each
                                    reservoir gets ceil(n/t) boxes in that direction */
    int fill;                    /* subdomain ILU level of fill k, 0..4 (0: ILU(0)): ILU on
                                    the level-k pattern of the stencil on an unbounded grid,
                                    restricted to the box (an entry's level is the least number
                                    of interior vertices on a path to it through smaller
                                    cells); k > 0 runs the hyperplane kernels.  With boxes at
                                    most k + 1 cells wide (2D) this is the exact LU of the box */
    int ratio;                   /* coarse-to-fine mesh ratio per direction, 2..16 (0: 2;
                                    Section 4.2 compares 2, 4, 8 and 16): coarse cell J covers
                                    fine cells rJ .. min(rJ + r, n) - 1 and sits at their
                                    centroid; orders 2 and 3 interpolate in the coordinate
                                    linear between consecutive centroids */
    int coarse_op;               /* NKS_COARSE_GALERKIN (0): P^T A P on every coarse level;
                                    NKS_COARSE_REDISCRETIZED: the Jacobian of the upscaled
                                    coarse problem (cells of r^d fine cells, each permeability
                                    component their mean, pore volume their sum, the fine
                                    stencil) at the coarsened state (the mean of the children)
                                    of the last nks_jacobian; every size above one must be a
                                    multiple of r on every coarse level; not for the transpose */
    int coarse_kernel;           /* how the coarsest level's GMRES runs (the same iteration
                                    either way): NKS_COARSE_AUTO (0) the persistent form where
                                    the level allows it and each reservoir's factors on it take
                                    at most 256 KiB (one CU streams them every sweep), else
                                    chunks; NKS_COARSE_CHUNKED one
                                    launch per kernel step, replayed in captured chunks of
                                    iterations with a host test of convergence after each;
                                    NKS_COARSE_PERSISTENT one launch for the whole solve, a
                                    workgroup per reservoir iterating until its own test
                                    stops it (no host round trip), which needs a 2D coarsest
                                    level swept by rows, the left-RAS variant and at most
                                    4096 cells per reservoir on that level (NKS_EINVAL
                                    otherwise) */
} nks_ras_desc;

#define NKS_COARSE_GALERKIN 0
#define NKS_COARSE_REDISCRETIZED 1
#define NKS_COARSE_AUTO 0
#define NKS_COARSE_CHUNKED 1
#define NKS_COARSE_PERSISTENT 2

/* Creates (*inout == NULL) or refactors in place (*inout from an earlier
 * call on a matrix of the same grid and an identical descriptor).  Keeps a
 * reference to J (the finest level's operator), which therefore lives until
 * the preconditioner is destroyed or set up on another matrix; J's values are
 * read at every apply.  Asynchronous.  A zero
 * pivot is reported by the next synchronising call as NKS_EZEROPIVOT.  The 3D
 * sweeps of boxes split into slabs wait on their neighbouring slab with a
 * spin limit; a wait that reaches it marks the level, and the next call that
 * checks the factors (nks_gmres_solve, nks_newton_step, nks_adjoint) fails
 * with NKS_EHIP instead of returning a correction built on stale values. */
int nks_ras_setup(nks_matrix *J, const nks_ras_desc *d, nks_ras **inout);
int nks_destroy_ras(nks_ras *M);
/* z = M^{-1} r on the finest level (device).  With levels > 1 it runs the
 * coarse GMRES: asynchronous in the persistent form, synchronising in the
 * chunked one (coarse_kernel). */
int nks_ras_apply(nks_ras *M, const double *r, double *z);
/* One-level Schwarz apply on `level` (0 = finest) with vectors of that
 * level's size (device).  Asynchronous. */
int nks_ras_apply_level(nks_ras *M, int level, const double *r, double *z);
/* x = the coarsest level's GMRES solve of A_c x = b (Remark 2: x0 = 0, the
 * one-level preconditioner, stopped at coarse_rtol ||b|| or coarse_maxit
 * iterations) with vectors of that level's size (device); levels > 1.
 * Asynchronous in the persistent form. */
int nks_ras_coarse_solve(nks_ras *M, const double *b, double *x);
/* Per reservoir, the iterations and the last residual estimate of the
 * latest coarse solve (host arrays of one entry per reservoir; either may be
 * NULL).  Synchronises the grid's stream. */
int nks_ras_coarse_stats(nks_ras *M, int *its, double *res);
/* z = M^{-T} r (device): the preconditioner with the same boxes and levels
 * built on J^T, left- and right-RAS exchanged (AS stays AS).  ILU(0) of A^T
 * on a symmetric pattern is the transpose of ILU(0) of A, and the Galerkin
 * product commutes with transposition, so for one level this is exactly the
 * transpose; with levels it is the transposed composition (the mu and nu
 * smoothing counts trade places, left and right Kaskade exchange) up to the
 * inexact coarse solve.  Built and factored on first use after each nks_ras_setup.
 * Synchronous on the grid's stream when it refactors. */
int nks_ras_apply_transpose(nks_ras *M, const double *r, double *z);
/* info[0..7] = n, stencil points, subdomains, nx, ny, nz (first reservoir),
 * number of levels, nnz of the level operator. Synchronises. */
int nks_ras_level_info(nks_ras *M, int level, int *info);
/* Kernel form of the level's last one-level sweep, for reports: *form =
 * one of NKS_SWEEP_* (NKS_SWEEP_NONE before the level's first sweep), and
 * the workgroups it launched.  The form follows from the boxes' shapes, the
 * precision and the device's occupancy: hyperplane kernel; 2D row sweep of
 * one box per workgroup with four or one wavefronts; packed 2D row sweep
 * (several small boxes in one wavefront); 3D row sweep. */
enum { NKS_SWEEP_NONE = 0, NKS_SWEEP_HYPERPLANE = 1, NKS_SWEEP_ROWS4 = 2, NKS_SWEEP_ROWS1 = 3,
       NKS_SWEEP_PACKED = 4, NKS_SWEEP_ROWS3D = 5 };
int nks_ras_level_sweep(nks_ras *M, int level, int *form, int *workgroups);
/* Level operator (Galerkin product on coarse levels) as CSR in HOST arrays. */
int nks_ras_level_export(nks_ras *M, int level, int *rowptr, int *col, double *val);
/* Restriction P^T (fine level -> level+1) and prolongation-add
 * (level+1 -> fine: z += P e) on device vectors.  Asynchronous. */
int nks_ras_restrict(nks_ras *M, int level, const double *r_fine, double *r_coarse);
int nks_ras_prolong_add(nks_ras *M, int level, const double *e_coarse, double *z_fine);

/* Right-preconditioned GMRES(restart) / FGMRES(restart) (Section 3,
 * the Jacobian system; Remark 2): x holds the initial guess (zero it for x0 = 0);
 * stops per reservoir when ||b - J x|| <= max(rtol ||b||, atol).
 * Orthogonalisation: classical Gram-Schmidt with one reorthogonalisation,
 * FP64.  transpose != 0 solves J^T x = b, preconditioned by
 * nks_ras_apply_transpose when M is given. */
typedef struct {
    int restart;
    double rtol, atol;
    int maxit;
    int flexible;
    int transpose;
} nks_gmres_desc;

typedef struct {
    int iterations;              /* max over reservoirs */
    int total_iterations;        /* sum over reservoirs */
    double residual;             /* max over reservoirs of the final residual norm (the
                                    GMRES estimate |g_{k+1}| when every reservoir converged
                                    inside a cycle; the recomputed ||b - J x|| otherwise) */
    int converged;               /* reservoirs that met the tolerance */
    int *its;                    /* optional HOST array [nres]: iterations */
    double *res;                 /* optional HOST array [nres]: final ||r|| */
} nks_gmres_stats;

int nks_gmres_solve(nks_matrix *J, nks_ras *M, const double *b, double *x,
                    const nks_gmres_desc *d, nks_gmres_stats *st);

/* One implicit time step (Section 3): X^{k+1} = X^k + lambda s with
 * J s = -F solved by Schwarz-preconditioned (F)GMRES to
 * max{eta_r ||F||, eta_a}, lambda from a cubic backtracking line search with
 * ||F(X + lambda s)|| <= (1 - alpha lambda)||F(X)||, until
 * ||F|| <= max{eps_r ||F(X^0)||, eps_a} or ||lambda s|| <= stol ||X|| in every
 * reservoir (the step test is that of the PETSc solver used in Section 4), or,
 * with floor_test, when ||F|| is at the binary64 rounding floor of its own
 * evaluation, u || |J| |X| || (the componentwise bound of the stencil product
 * that makes up the flux terms; needed where eps_r ||F(X^0)|| is below what
 * binary64 can resolve).  The
 * step test is also taken on the full step before the line search: a full step
 * that small is taken as it is (lambda = 1, no decrease test, since at the
 * FP64 rounding floor ||F|| cannot decrease) and the reservoir stops.  Each
 * reservoir stops on its own; the call returns when all have.
 * p: device in (initial guess, usually p_n) / out. */
typedef struct {
    double eps_r, eps_a;
    double eta_r, eta_a;
    int restart, maxit;
    int flexible;                /* -1: FGMRES iff levels > 1 or precision != FP64 */
    double alpha;
    int max_newton, max_backtracks;
    double stol;                 /* also stop after a full step with ||s|| <= stol ||X^k||
                                    or when ||lambda s|| <= stol ||X^{k+1}|| (0: off) */
    int floor_test;              /* nonzero: also stop when ||F(X)|| <= u || |J(X)| |X| ||,
                                    u = 2^-53, the rounding floor of evaluating F */
    int lag;                     /* >= 0: subdomain ILU factorisations at Newton iterations
                                    0, lag, 2 lag, ... of the step (0 or 1: every one).  In
                                    between, the factors of the last one are reused while
                                    the operators stay current: the Jacobian on the finest
                                    level and its Galerkin products below */
} nks_newton_desc;

typedef struct {
    int newton_its;              /* max over reservoirs */
    int linear_its;              /* sum over Newton iterations of the max over reservoirs */
    int status;                  /* 0 ok, 1 Newton limit, 2 line search failed, 3 non-physical */
    double fnorm0, fnorm;        /* max over reservoirs */
    double fnorms[64];           /* max over reservoirs after each iteration */
    int lits[64];
    double lambdas[64];          /* min over active reservoirs */
    double t_residual, t_jacobian, t_setup, t_gmres, t_linesearch;  /* seconds */
    int *stop_reason;            /* optional HOST array [nres] (caller-owned, NULL: not wanted):
                                    why each reservoir stopped, NKS_STOP_* */
    double *rel_res;             /* optional HOST array [nres]: final ||F|| / ||F(X^0)|| */
    int host_waits;              /* times the host waited on the device during the step */
    int graph_chunk;             /* FGMRES iterations per captured graph in the step (0: none;
                                    captured when the preconditioner runs without host
                                    round trips: one level, or the persistent coarse solve) */
} nks_newton_stats;

#define NKS_STOP_NONE 0          /* still iterating when the call returned (limit or failure) */
#define NKS_STOP_TOL 1           /* ||F|| <= max{eps_r ||F(X^0)||, eps_a} */
#define NKS_STOP_FLOOR 2         /* ||F|| at the rounding floor u || |J| |X| || (floor_test) */
#define NKS_STOP_STEP 3          /* the relative step test (stol) */

int nks_newton_step(nks_grid *g, double *p, const double *p_n, const double *p_nm1,
                    double dt, int bdf_order, const nks_newton_desc *nd,
                    const nks_ras_desc *rd, nks_newton_stats *st);

/* J^T as a matrix on the same grid and stencil: JT[q][i] = J[opp(q)][i + off_q].
 * Both created by nks_matrix_create on one grid; asynchronous on its stream. */
int nks_matrix_transpose(nks_matrix *J, nks_matrix *JT);

/* Discrete adjoint of nsteps implicit steps for an objective G(p^1..p^n)
 * whose gradient in each state is given.  With the Lagrangian
 * G + sum_n lambda_n^T F^n(p^n, p^{n-1}, p^{n-2}; ln K), the multipliers
 * solve, from the last step back,
 *   J_n^T lambda_n = -dG/dp^n - (dF^{n+1}/dp^n)^T lambda_{n+1} - (dF^{n+2}/dp^n)^T lambda_{n+2}
 * (the couplings are diagonal: the accumulation's dependence on the earlier
 * states, Section 2's BDF1/BDF2), and
 *   dG/dln K = sum_n (dF^n/dln K)^T lambda_n,
 * with ln K of a cell scaling all three components together.  Each J_n^T
 * system is solved by (F)GMRES (gd: restart, rtol, atol, maxit, flexible;
 * transpose ignored) preconditioned with the transpose of the Schwarz
 * preconditioner rd describes (see nks_ras_apply_transpose), x0 = 0.
 *   p_hist   HOST array of nsteps+1 device pointers: p^0 (initial state,
 *            independent of K) and the converged p^1..p^nsteps
 *   orders   HOST array of nsteps ints: BDF order of step n at [n-1]
 *            (1, or 2 from the second step on)
 *   dGdp     HOST array of nsteps+1 device pointers, NULL for a zero
 *            gradient; entry 0 is ignored
 *   grad     device [N], overwritten with dG/dln K
 *   lam_out  optional HOST array of nsteps+1 device pointers receiving
 *            lambda_n (NULL array or entries: not wanted)
 * NKS_ENOTCONVERGED when a linear solve misses its tolerance (grad is still
 * written). */
typedef struct {
    int linear_its[64];          /* iterations of the J_n^T solve, step n at [n-1] */
    int total_linear_its;
    int status;                  /* 0 ok, 1 a solve did not converge */
    double t_total;              /* seconds */
} nks_adjoint_stats;

int nks_adjoint(nks_grid *g, int nsteps, const double *const *p_hist, const int *orders, double dt,
                const double *const *dGdp, const nks_ras_desc *rd, const nks_gmres_desc *gd,
                double *grad, double *const *lam_out, nks_adjoint_stats *st);

/* Autotuner of the subdomain tile edge, overlap and coarse-to-fine
 * ratio for the batch form.  At the state (p, p_n, p_nm1, dt, order) it
 * forms the first Newton system J s = -F, and for every (tile, overlap,
 * ratio) triple builds the preconditioner base describes with tx = ty (= tz
 * in 3D) = tile, the overlap on every level = overlap and ratio = ratio (ratios NULL or
 * nratios 0: base's ratio only), then times, averaged over `repeats` runs
 * after one untimed run: the factorisation (setup) and one (F)GMRES solve to
 * gd's tolerance (solve).  best receives the descriptor with the smallest
 * setup + solve time.  table (optional HOST array of ntiles * noverlaps *
 * nratios, tile-major then overlap) receives every candidate's times;
 * candidates that cannot be set up (e.g. a box larger than LDS allows) have
 * ok = 0.  Synchronous. */
typedef struct {
    int tile, overlap;
    int ok;
    int iterations;              /* of the timed solve, max over reservoirs */
    double setup_ms, solve_ms;
    int ratio;
} nks_autotune_entry;

int nks_ras_autotune(nks_grid *g, const double *p, const double *p_n, const double *p_nm1, double dt,
                     int bdf_order, const nks_ras_desc *base, const int *tiles, int ntiles,
                     const int *overlaps, int noverlaps, const int *ratios, int nratios,
                     const nks_gmres_desc *gd, int repeats, nks_ras_desc *best, nks_autotune_entry *table);

/* Kernel timing with HIP events on the launching stream.  Single-kernel
 * records carry the events on the dispatch itself (the kernel's own
 * execution time): "ras_apply_l<level>" (one-level Schwarz sweeps),
 * "ilu_factor_l<level>", "rap_l<level>", "spmv_l<0|1>" (7-or-fewer-point /
 * wider stencils).  Span records bracket several kernels: "gmres_arnoldi"
 * (the Arnoldi step after the preconditioner), "residual_jacobian".  Launches inside captured graphs are not recorded.
 * enable != 0 clears the records and starts recording, 0 stops; enable = 2
 * also runs the iterations otherwise replayed from captured graphs (the
 * chunked coarse GMRES, the captured FGMRES iterations) as plain launches,
 * so every launch is recorded.  query
 * synchronises and returns the number of launches and their summed duration
 * (ms); unknown names give 0.  durations writes the first min(cap, count)
 * per-launch durations (ms, launch order) to host array ms and the record
 * count to *count, so a caller can separate dispatches that found every
 * reservoir masked out (speculative Krylov iterations past convergence). */
int nks_profile_enable(int enable);
/* Restrict recording to the named records (comma-separated, e.g.
 * "ras_apply_l0,ras_apply_l1"); NULL or "" records every name.  Launches
 * outside the set take no events and no host bookkeeping. */
int nks_profile_filter(const char *names);
int nks_profile_query(const char *name, int *count, double *total_ms);
int nks_profile_durations(const char *name, double *ms, int cap, int *count);
/* For the one-level Schwarz sweep records ("ras_apply_l<level>"): cells[0] =
 * extended cells and cells[1] = owned cells of the subdomains the recorded
 * launches swept, summed over those launches (subdomains of reservoirs masked
 * out are not counted), so the bytes a launch moves follow from the per-cell
 * factor and vector bytes.  Synchronises the device; 0 for unknown names. */
int nks_profile_units(const char *name, double *cells);

/* Thread-local message of the last failing call (empty when none). */
const char *nks_last_error(void);
/* Library version string. */
const char *nks_version(void);

#ifdef __cplusplus
}
#endif
#endif
