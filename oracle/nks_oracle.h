/*
 * Plain FP64 CPU oracle for the Newton-Krylov-Schwarz hot path of
 * "Multilevel restricted Schwarz preconditioners for fully implicit
 * subsurface flow with the Peng-Robinson equation of state" (arXiv 2007.13966).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this code; it exists so the tests can check the GPU path against an
 * obviously correct, slow implementation written straight from the paper.
 *
 * Every array is lexicographic with x fastest: cell (x,y,z) has index
 * x + nx*(y + ny*z).  Units are SI.
 */
#ifndef NKS_ORACLE_H
#define NKS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_problem orc_problem;
typedef struct orc_mg orc_mg;

typedef struct {
    int px, py, pz;         /* subdomain boxes per direction, same on every level */
    int levels;             /* L >= 1 */
    int overlap[8];         /* overlap per level, index 0 = finest */
    int variant;            /* 0 left-RAS, 1 classical AS, 2 right-RAS */
    int subsolve;           /* 0 ILU(0), 1 exact dense LU */
    int interp_order;       /* 1 nearest, 2 bilinear, 3 bicubic */
    int cycle;              /* 0 V-cycle, 1 left-Kaskade, 2 right-Kaskade, 3 additive, 4 coarse-only */
    int mu, nu;             /* pre/post smoothing counts (V-cycle family) */
    double coarse_rtol;     /* coarsest GMRES relative tolerance */
    int coarse_maxit;
    int coarse_restart;
    int tx, ty, tz;         /* > 0: box edge in cells on the finest level (boxes = ceil(n/t)) */
    int fill;               /* subdomain ILU level of fill k (0: ILU(0)): ILU on the level-k pattern */
    int ratio;              /* coarse-to-fine mesh ratio per direction (0: 2) */
    int coarse_op;          /* ORC_COARSE_GALERKIN or ORC_COARSE_REDISCRETISED */
} orc_mg_desc;

#define ORC_COARSE_GALERKIN 0        /* P^T A P */
#define ORC_COARSE_REDISCRETISED 1   /* Jacobian of the upscaled coarse problem */

typedef struct {
    double eps_r, eps_a;    /* Newton stopping */
    double eta_r, eta_a;    /* linear stopping (max of the two) */
    int restart, maxit;
    int flexible;           /* FGMRES when nonzero */
    double alpha;           /* line-search sufficient decrease */
    int max_newton, max_backtracks;
    double stol;            /* stop when ||lambda s|| <= stol ||X^{k+1}|| (0: off) */
    int floor_test;         /* nonzero: also stop when ||F|| <= u || |J| |X| || */
    int lag;                /* ILU factorisations at iterations 0, lag, 2 lag, ... (0 or 1:
                               every one); in between the subdomain factors are kept while
                               the operators (J and its Galerkin products) are current */
} orc_newton_desc;

typedef struct {
    int newton_its;
    int linear_its;         /* total over the Newton iterations */
    int status;             /* 0 ok, 1 Newton not converged, 2 line search failed, 3 non-physical */
    double fnorm0, fnorm;   /* ||F|| at the first and final iterate */
    double fnorms[64];      /* ||F|| after each Newton iteration (first 64) */
    int lits[64];           /* GMRES iterations per Newton iteration */
    double lambdas[64];     /* accepted step lengths */
} orc_newton_stats;

/* ---- problem ---- */
orc_problem *orc_problem_new(int nx, int ny, int nz, double dx, double dy, double dz,
                             const double *kx, const double *ky, const double *kz,
                             const double *phi, int nw, const int *wcell, const double *wrate,
                             double Tc, double pc, double omega, double T, double W,
                             double R, double mu, int gravity, double g);
void orc_problem_free(orc_problem *pr);
/* boundary condition types of the outer faces -x,+x,-y,+y,-z,+z */
#define ORC_BC_CLOSED 0      /* no flow (the default) */
#define ORC_BC_DIRICHLET 1   /* value: p^D in Pa */
#define ORC_BC_NEUMANN 2     /* value: q^N = v.n in m/s, n the outward normal */
int orc_problem_set_bc(orc_problem *pr, int face, int type, double value);
/* accumulation forms */
#define ORC_ACCUM_CONSERVATIVE 0   /* phi V (m(p^{l+1}) - m(p^l))/dt and its BDF2 analogue */
#define ORC_ACCUM_CHAIN_RULE 1     /* phi V m'(p^{l+1}) (p^{l+1} - p^l)/dt, as Section 2 prints it */
int orc_problem_set_accum(orc_problem *pr, int form);

/* PR-EOS */
void orc_pr_params(double Tc, double pc, double omega, double T, double R,
                   double *a, double *b, double *m);
void orc_acentric_terms(double Tr, double *f0, double *f1);
double orc_acentric(double pc, double Tc, double Tb);
int orc_pr_z(double a, double b, double T, double R, double p, double *Z, double *dZdp);
int orc_pr_z2(double a, double b, double T, double R, double p, double *Z, double *dZ, double *d2Z,
              double *d2m);
void orc_pr_eval(const orc_problem *pr, int n, const double *p, double *Z, double *dZ,
                 double *msc, double *dmsc);

/* Discretization */
void orc_transmissibility(const orc_problem *pr, double *tx, double *ty, double *tz);
void orc_residual(const orc_problem *pr, const double *p, const double *pn, const double *pnm1,
                  double dt, int order, double *F);
int orc_jacobian(const orc_problem *pr, const double *p, const double *pn, const double *pnm1,
                 double dt, int order, int *rp, int *ci, double *v);
void orc_hydrostatic(const orc_problem *pr, double p_top, double *p);
void orc_residual_dlogk_t(const orc_problem *pr, const double *p, const double *lam, double *out);

/* Multilevel Schwarz preconditioner built from a fine CSR matrix on the problem grid */
orc_mg *orc_mg_new(int nx, int ny, int nz, int n, const int *rp, const int *ci,
                   const double *v, const orc_mg_desc *d);
/* with rediscretised coarse levels: the problem and the state they are evaluated from */
orc_mg *orc_mg_new_problem(const orc_problem *pr, const double *p, double dt, int order, const int *rp,
                           const int *ci, const double *v, const orc_mg_desc *d);
orc_problem *orc_problem_coarsen(const orc_problem *pr, int ratio);
void orc_mg_free(orc_mg *mg);
void orc_mg_apply(orc_mg *mg, const double *r, double *z);
void orc_mg_apply_transpose(orc_mg *mg, const double *r, double *z);
void orc_mg_apply_onelevel(orc_mg *mg, int level, const double *r, double *z);
int orc_mg_level_info(const orc_mg *mg, int level, int *info /* n,nnz,nx,ny,nz,nsub,nc,pnnz */);
void orc_mg_level_matrix(const orc_mg *mg, int level, int *rp, int *ci, double *v);
void orc_mg_level_prolong(const orc_mg *mg, int level, int *rp, int *ci, double *v);
int orc_mg_sub_info(const orc_mg *mg, int level, int s, int *info /* next,nnz,lo3,hi3,elo3,ehi3 */);
void orc_mg_sub_factors(const orc_mg *mg, int level, int s, int *cells, int *owned,
                        int *rp, int *ci, double *v);

/* Sparse utilities */
void orc_csr_matvec(int n, const int *rp, const int *ci, const double *v, const double *x, double *y);
void orc_interp_1d(int nf, int order, int *rp, int *ci, double *w);  /* rows nf, cols ceil(nf/2), <=4 per row */
void orc_interp_1d_r(int nf, int order, int ratio, int *rp, int *ci, double *w);  /* cols ceil(nf/ratio) */
void orc_ilu0(int n, const int *rp, const int *ci, double *v);        /* in place, sorted columns */
void orc_ilu0_solve(int n, const int *rp, const int *ci, const double *v, const double *r, double *z);

/* Krylov: right-preconditioned GMRES(m) / FGMRES(m) with MGS.  M may be NULL. */
int orc_gmres(int n, const int *rp, const int *ci, const double *v, orc_mg *M, int transpose,
              const double *b, double *x, int restart, double rtol, double atol, int maxit,
              int flexible, double *res_out, int *its_out);

/* One implicit time step: p in = initial guess (previous step), out = new level */
int orc_newton_step(const orc_problem *pr, const orc_mg_desc *md, const orc_newton_desc *nd,
                    double *p, const double *pn, const double *pnm1, double dt, int order,
                    orc_newton_stats *st);

#ifdef __cplusplus
}
#endif
#endif
