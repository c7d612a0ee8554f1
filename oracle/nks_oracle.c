/*
 * Plain FP64 CPU oracle (test infrastructure only; see nks_oracle.h).
 *
 * Written from the paper's text in the order it presents the method:
 *   Section 2: Peng-Robinson density (rho = cW, c = p/(ZRT), the Z cubic,
 *              the criticality relations for a(T) and b, m(w)), the pressure
 *              form of the governing equation and its dZ/dp, cell-centred
 *              finite differences (Remark 1), the BDF1 and BDF2 schemes.
 *   Section 3: inexact Newton with cubic line search (the Newton update and
 *              the sufficient-decrease test), right-preconditioned GMRES on
 *              the Jacobian system, the linear and nonlinear stopping tests,
 *              restriction matrices R_i^delta / R_i^0, classical AS, left-RAS,
 *              right-RAS (Section 3.1), the multigrid V-cycle (Algorithm 1 and
 *              the two-level preconditioner built from it), the Kaskade,
 *              additive and coarse-only compositions, the iterative coarse
 *              solve with FGMRES outside (Remark 2) and the first-, second-
 *              and third-order interpolation operators (Section 3.2).
 *   Section 4: stopping values and GMRES restart 30.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes): the largest real cubic root; conservative accumulation
 * phi V (m^{n+1} - m^n)/dt whose linearisation is the paper's coefficient;
 * harmonic face transmissibility; phase-potential upwinding of p/(mu Z) with
 * ties to the row cell; arithmetic-mean face density; depth h increasing with
 * the z index; linear stop with max{eta_r ||F||, eta_a}; restriction = P^T;
 * Galerkin coarse operators P^T A P; the same subdomain box grid on every
 * level; clamped interpolation at the domain boundary; a Dirichlet face's
 * state at the face centre, half a cell away; a Neumann face's density from
 * the cell.
 *
 * No blocking, fusion or reordering beyond what the definitions state.
 */
#include "nks_oracle.h"

#include <limits.h>
#include <stdio.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXLEV 8

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s ? s : 1);
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------------ */
/* Problem                                                             */
/* ------------------------------------------------------------------ */
struct orc_problem {
    int nx, ny, nz, N;
    double dx, dy, dz;
    double *kx, *ky, *kz, *phi;
    int nw;
    int *wcell;
    double *wrate;
    double Tc, pc, omega, T, W, R, mu, g;
    double a, b, mpr;   /* PR a(T), b and m(omega) */
    int bct[6];         /* boundary faces -x,+x,-y,+y,-z,+z: ORC_BC_* (zero: closed) */
    double bcv[6];      /* p^D (Pa) or q^N (m/s, outward normal) */
    int accum;          /* ORC_ACCUM_CONSERVATIVE or ORC_ACCUM_CHAIN_RULE */
};

orc_problem *orc_problem_new(int nx, int ny, int nz, double dx, double dy, double dz,
                             const double *kx, const double *ky, const double *kz,
                             const double *phi, int nw, const int *wcell, const double *wrate,
                             double Tc, double pc, double omega, double T, double W,
                             double R, double mu, int gravity, double g) {
    orc_problem *pr = (orc_problem *)xcalloc(1, sizeof(orc_problem));
    int N = nx * ny * nz;
    pr->nx = nx; pr->ny = ny; pr->nz = nz; pr->N = N;
    pr->dx = dx; pr->dy = dy; pr->dz = dz;
    pr->kx = (double *)xcalloc(N, sizeof(double));
    pr->ky = (double *)xcalloc(N, sizeof(double));
    pr->kz = (double *)xcalloc(N, sizeof(double));
    pr->phi = (double *)xcalloc(N, sizeof(double));
    memcpy(pr->kx, kx, N * sizeof(double));
    memcpy(pr->ky, ky, N * sizeof(double));
    memcpy(pr->kz, kz, N * sizeof(double));
    memcpy(pr->phi, phi, N * sizeof(double));
    pr->nw = nw;
    pr->wcell = (int *)xcalloc(nw, sizeof(int));
    pr->wrate = (double *)xcalloc(nw, sizeof(double));
    if (nw) {
        memcpy(pr->wcell, wcell, nw * sizeof(int));
        memcpy(pr->wrate, wrate, nw * sizeof(double));
    }
    pr->Tc = Tc; pr->pc = pc; pr->omega = omega; pr->T = T; pr->W = W; pr->R = R;
    pr->mu = mu;
    pr->g = gravity ? g : 0.0;
    orc_pr_params(Tc, pc, omega, T, R, &pr->a, &pr->b, &pr->mpr);
    return pr;
}

/* Boundary condition of one outer face (Section 2: p = p^D on the Dirichlet
 * part, v.n = q^N on the Neumann part, n the outward normal).  Returns 0, or
 * -1 for a bad face index or type. */
int orc_problem_set_bc(orc_problem *pr, int face, int type, double value) {
    if (face < 0 || face > 5 || type < ORC_BC_CLOSED || type > ORC_BC_NEUMANN) return -1;
    if (type == ORC_BC_DIRICHLET && !(value > 0.0)) return -1;
    pr->bct[face] = type;
    pr->bcv[face] = type == ORC_BC_CLOSED ? 0.0 : value;
    return 0;
}

/* Accumulation form: ORC_ACCUM_CONSERVATIVE (the reading this oracle takes by
 * default) or ORC_ACCUM_CHAIN_RULE (the BDF1 and BDF2 equations of Section 2
 * as printed: the coefficient of dp/dt at the new level times the difference
 * quotient of p).  Returns 0, or -1 for an unknown form. */
int orc_problem_set_accum(orc_problem *pr, int form) {
    if (form != ORC_ACCUM_CONSERVATIVE && form != ORC_ACCUM_CHAIN_RULE) return -1;
    pr->accum = form;
    return 0;
}

void orc_problem_free(orc_problem *pr) {
    if (!pr) return;
    free(pr->kx); free(pr->ky); free(pr->kz); free(pr->phi);
    free(pr->wcell); free(pr->wrate);
    free(pr);
}

/* ------------------------------------------------------------------ */
/* Peng-Robinson equation of state (Section 2)                         */
/* ------------------------------------------------------------------ */

/* the criticality relations for a(T) and b (Section 2) with m(w) from its first branch (0 <= w <= 0.491) or the
 * second branch (0.491 <= w <= 2.0). */
void orc_pr_params(double Tc, double pc, double omega, double T, double R,
                   double *a, double *b, double *m) {
    double w = omega, mm;
    if (w <= 0.491)
        mm = 0.37464 + 1.54226 * w - 0.26992 * w * w;
    else
        mm = 0.3796 + 1.485 * w - 0.1644 * w * w + 0.01667 * w * w * w;
    double Tr = T / Tc;
    double s = 1.0 + mm * (1.0 - sqrt(Tr));
    *a = 0.45724 * R * R * Tc * Tc / pc * s * s;
    *b = 0.0778 * R * Tc / pc;
    *m = mm;
}

/* Acentric factor from the normal boiling point (Section 2): the reduced
 * vapour-pressure correlation ln(p_r) = f0(T_r) + w f1(T_r) with the two
 * polynomials in (1 - T_r) printed there, solved for w at T_r = T_b/T_c where
 * p = 1 atm. */
void orc_acentric_terms(double Tr, double *f0, double *f1) {
    double t = 1.0 - Tr;
    *f0 = (-5.97616 * t + 1.29874 * pow(t, 1.5) - 0.60394 * pow(t, 2.5) - 1.06841 * pow(t, 5.0)) / Tr;
    *f1 = (-5.03365 * t + 1.11505 * pow(t, 1.5) - 5.41217 * pow(t, 2.5) - 7.46628 * pow(t, 5.0)) / Tr;
}

double orc_acentric(double pc, double Tc, double Tb) {
    double f0, f1;
    orc_acentric_terms(Tb / Tc, &f0, &f1);
    return (-log(pc / 101325.0) - f0) / f1;
}

/* Largest real root of the PR cubic (Section 2),
 *   Z^3 - (1-B) Z^2 + (A - 3B^2 - 2B) Z - (AB - B^2 - B^3) = 0,
 * by Cardano's formula (one real root) or the trigonometric form (three real
 * roots), then dZ/dp from the closed form printed after the pressure form of the governing equation (Section 2).
 * Returns 0 on success, 1 if the root is non-physical (Z <= B or p <= 0). */
int orc_pr_z(double a, double b, double T, double R, double p, double *Z, double *dZdp) {
    double RT = R * T;
    double A = a * p / (RT * RT);
    double B = b * p / RT;
    /* monic cubic Z^3 + c2 Z^2 + c1 Z + c0 */
    double c2 = -(1.0 - B);
    double c1 = A - 3.0 * B * B - 2.0 * B;
    double c0 = -(A * B - B * B - B * B * B);
    /* depressed cubic t^3 + P t + Q with Z = t - c2/3 */
    double P = c1 - c2 * c2 / 3.0;
    double Q = 2.0 * c2 * c2 * c2 / 27.0 - c2 * c1 / 3.0 + c0;
    double D = 0.25 * Q * Q + P * P * P / 27.0;
    double z;
    if (D > 0.0) {
        double sq = sqrt(D);
        z = cbrt(-0.5 * Q + sq) + cbrt(-0.5 * Q - sq) - c2 / 3.0;
    } else {
        double r = sqrt(-P / 3.0);
        double arg = (r > 0.0) ? (-0.5 * Q) / (r * r * r) : 0.0;
        if (arg > 1.0) arg = 1.0;
        if (arg < -1.0) arg = -1.0;
        double th = acos(arg);
        z = 2.0 * r * cos(th / 3.0) - c2 / 3.0;   /* k = 0 branch: the largest */
    }
    /* two Newton steps on the cubic remove the rounding the closed form loses
     * near a double root (the same root is kept: it is simple and the
     * closed form is already within a few ulps of it) */
    for (int it = 0; it < 2; ++it) {
        double f = ((z + c2) * z + c1) * z + c0;
        double df = (3.0 * z + 2.0 * c2) * z + c1;
        if (df != 0.0) z -= f / df;
    }
    /* dZ/dp by the closed form of Section 2 */
    double C = 3.0 * z * z - 2.0 * (1.0 - B) * z + (A - 2.0 * B - 3.0 * B * B);
    double dz = -b / (RT * C) * z * z
                - (a / (RT * RT * C) - (2.0 * b + 6.0 * B * b) / (RT * C)) * z
                + (2.0 * a * b * p / (RT * RT * RT * C) - (2.0 * B * b + 3.0 * B * B * b) / (RT * C));
    *Z = z;
    *dZdp = dz;
    return (p <= 0.0 || z <= B || !isfinite(z)) ? 1 : 0;
}

/* scaled density m = p/Z (rho = m W/(R T)) and dm/dp = (p/Z)(1/p - Z'/Z),
 * the coefficient of dp/dt in the pressure form of the governing equation (Section 2) divided by phi */
static int pr_m(const orc_problem *pr, double p, double *m, double *dm) {
    double Z, dZ;
    int bad = orc_pr_z(pr->a, pr->b, pr->T, pr->R, p, &Z, &dZ);
    *m = p / Z;
    *dm = 1.0 / Z - p * dZ / (Z * Z);
    return bad;
}

/* Second pressure derivatives of Z and of m = p/Z, by differentiating the
 * cubic G(Z, p) = Z^3 + c2 Z^2 + c1 Z + c0 = 0 of Section 2 twice along its
 * root (A = alpha p, B = beta p):
 *   Z'  = -G_p / G_Z,
 *   Z'' = -(G_pp + 2 G_Zp Z' + G_ZZ Z'^2) / G_Z,
 *   m'' = -(2 Z' + p Z'') / Z^2 + 2 p Z'^2 / Z^3.
 * Needed by the Jacobian of the chain-rule accumulation, whose coefficient is
 * m' itself. */
int orc_pr_z2(double a, double b, double T, double R, double p, double *Z, double *dZ, double *d2Z,
              double *d2m) {
    double RT = R * T;
    double al = a / (RT * RT), be = b / RT;
    double z, dz;
    int bad = orc_pr_z(a, b, T, R, p, &z, &dz);
    double B = be * p;
    double c2 = -(1.0 - B);
    double c1p = al - 6.0 * be * be * p - 2.0 * be, c1pp = -6.0 * be * be;
    double c0p = -(2.0 * al * be * p - 2.0 * be * be * p - 3.0 * be * be * be * p * p);
    double c0pp = -(2.0 * al * be - 2.0 * be * be - 6.0 * be * be * be * p);
    double c1 = al * p - 3.0 * B * B - 2.0 * B;
    double GZ = 3.0 * z * z + 2.0 * c2 * z + c1;
    double GZZ = 6.0 * z + 2.0 * c2;
    double Gp = be * z * z + c1p * z + c0p;
    double GZp = 2.0 * be * z + c1p;
    double Gpp = c1pp * z + c0pp;
    double z1 = -Gp / GZ;
    double z2 = -(Gpp + 2.0 * GZp * z1 + GZZ * z1 * z1) / GZ;
    if (Z) *Z = z;
    if (dZ) *dZ = z1;
    if (d2Z) *d2Z = z2;
    if (d2m) *d2m = -(2.0 * z1 + p * z2) / (z * z) + 2.0 * p * z1 * z1 / (z * z * z);
    (void)dz;
    return bad;
}

void orc_pr_eval(const orc_problem *pr, int n, const double *p, double *Z, double *dZ,
                 double *msc, double *dmsc) {
    for (int i = 0; i < n; ++i) {
        double z, d;
        orc_pr_z(pr->a, pr->b, pr->T, pr->R, p[i], &z, &d);
        if (Z) Z[i] = z;
        if (dZ) dZ[i] = d;
        if (msc) msc[i] = p[i] / z;
        if (dmsc) dmsc[i] = 1.0 / z - p[i] * d / (z * z);
    }
}

/* ------------------------------------------------------------------ */
/* Cell-centred finite differences (Section 2, Remark 1)               */
/* ------------------------------------------------------------------ */

/* Two-point face transmissibility T = A_f / (d/(2 K_i) + d/(2 K_j)) with the
 * K component normal to the face (harmonic mean).  tx[i] is the face between
 * cell i and its +x neighbour (0 on the last column); likewise ty, tz. */
void orc_transmissibility(const orc_problem *pr, double *tx, double *ty, double *tz) {
    int nx = pr->nx, ny = pr->ny, nz = pr->nz;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int i = x + nx * (y + ny * z);
                tx[i] = ty[i] = tz[i] = 0.0;
                if (x + 1 < nx) {
                    int j = i + 1;
                    tx[i] = pr->dy * pr->dz /
                            (pr->dx / (2.0 * pr->kx[i]) + pr->dx / (2.0 * pr->kx[j]));
                }
                if (y + 1 < ny) {
                    int j = i + nx;
                    ty[i] = pr->dx * pr->dz /
                            (pr->dy / (2.0 * pr->ky[i]) + pr->dy / (2.0 * pr->ky[j]));
                }
                if (z + 1 < nz) {
                    int j = i + nx * ny;
                    tz[i] = pr->dx * pr->dy /
                            (pr->dz / (2.0 * pr->kz[i]) + pr->dz / (2.0 * pr->kz[j]));
                }
            }
}

/* depth of the cell centre; the z index increases downward */
static double depth_of(const orc_problem *pr, int i) {
    int z = i / (pr->nx * pr->ny);
    return (z + 0.5) * pr->dz;
}

/* Neighbour list of cell i in the order -z, -y, -x, +x, +y, +z, with the
 * transmissibility of the shared face.  Returns the count. */
static int neighbours(const orc_problem *pr, const double *tx, const double *ty,
                      const double *tz, int i, int *nb, double *tf) {
    int nx = pr->nx, ny = pr->ny, nz = pr->nz, nxy = nx * ny;
    int x = i % nx, y = (i / nx) % ny, z = i / nxy, c = 0;
    if (z > 0) { nb[c] = i - nxy; tf[c++] = tz[i - nxy]; }
    if (y > 0) { nb[c] = i - nx; tf[c++] = ty[i - nx]; }
    if (x > 0) { nb[c] = i - 1; tf[c++] = tx[i - 1]; }
    if (x + 1 < nx) { nb[c] = i + 1; tf[c++] = tx[i]; }
    if (y + 1 < ny) { nb[c] = i + nx; tf[c++] = ty[i]; }
    if (z + 1 < nz) { nb[c] = i + nxy; tf[c++] = tz[i]; }
    return c;
}

/* Outer faces of cell i that carry a boundary condition.  A Dirichlet face
 * holds the state p^D at the face centre, half a cell from the cell centre:
 * transmissibility 2 K A / Delta (the one-sided form of the harmonic face
 * rule), potential difference (p_i - p^D) - rho_avg g (h_i - h_face) with
 * rho_avg the mean of the cell's and the face state's densities, mobility
 * from the upwind side.  A Neumann face carries the prescribed outward
 * Darcy velocity q^N: scaled mass flux m_i q^N A, the density taken from the
 * cell.  Adds the outward flux to *F, its derivative in p_i to *dF and, if
 * dlk is given, its derivative in ln K_i (a Dirichlet face's T is linear in
 * K_i, a Neumann face's flux does not depend on K). */
static void boundary_faces(const orc_problem *pr, int i, double pi, double *F, double *dF, double *dlk) {
    int nx = pr->nx, ny = pr->ny, nxy = nx * ny;
    int x = i % nx, y = (i / nx) % ny, z = i / nxy;
    double c_rho = pr->W / (pr->R * pr->T);
    double mi, dmi;
    pr_m(pr, pi, &mi, &dmi);
    for (int f = 0; f < 6; ++f) {
        if (pr->bct[f] == ORC_BC_CLOSED) continue;
        int on = f == 0 ? x == 0 : f == 1 ? x == nx - 1 : f == 2 ? y == 0 : f == 3 ? y == ny - 1
                 : f == 4 ? z == 0 : z == pr->nz - 1;
        if (!on) continue;
        double area, delta, k, dh = 0.0;
        if (f < 2) { area = pr->dy * pr->dz; delta = pr->dx; k = pr->kx[i]; }
        else if (f < 4) { area = pr->dx * pr->dz; delta = pr->dy; k = pr->ky[i]; }
        else {
            area = pr->dx * pr->dy; delta = pr->dz; k = pr->kz[i];
            dh = f == 4 ? 0.5 * pr->dz : -0.5 * pr->dz;   /* h_i - h_face, depth grows with z */
        }
        if (pr->bct[f] == ORC_BC_NEUMANN) {
            *F += mi * pr->bcv[f] * area;
            *dF += dmi * pr->bcv[f] * area;
            continue;
        }
        double pd = pr->bcv[f], md, dmd;
        pr_m(pr, pd, &md, &dmd);
        double T = 2.0 * k * area / delta;
        double rho_avg = 0.5 * (mi + md) * c_rho;
        double dphi = (pi - pd) - rho_avg * pr->g * dh;
        int up_i = dphi >= 0.0;
        double lam = (up_i ? mi : md) / pr->mu;
        double dlam = up_i ? dmi / pr->mu : 0.0;
        *F += T * lam * dphi;
        *dF += T * (dlam * dphi + lam * (1.0 - 0.5 * dmi * c_rho * pr->g * dh));
        if (dlk) *dlk += T * lam * dphi;
    }
}

/* Accumulation term of BDF1 (the BDF1 scheme of Section 2) or BDF2
 * (the BDF2 scheme of Section 2) in conservative form: returns the bracket
 * multiplying phi V / dt and its derivative with respect to p^{l+1}. */
static void accumulation(const orc_problem *pr, int order, double p, double pn, double pnm1,
                         double *acc, double *dacc) {
    double m, dm, mn, dmn, mnm1, dmnm1;
    pr_m(pr, p, &m, &dm);
    if (pr->accum == ORC_ACCUM_CHAIN_RULE) {
        /* the printed form: [phi p/Z (1/p - Z'/Z)]^{l+1} times the BDF
         * difference of p, so the bracket is m'(p^{l+1}) D_t p */
        double d2m;
        orc_pr_z2(pr->a, pr->b, pr->T, pr->R, p, NULL, NULL, NULL, &d2m);
        double dtp = order == 2 ? (3.0 * p - 4.0 * pn + pnm1) / 2.0 : p - pn;
        *acc = dm * dtp;
        *dacc = d2m * dtp + (order == 2 ? 1.5 : 1.0) * dm;
        return;
    }
    pr_m(pr, pn, &mn, &dmn);
    if (order == 2) {
        pr_m(pr, pnm1, &mnm1, &dmnm1);
        *acc = (3.0 * m - 4.0 * mn + mnm1) / 2.0;
        *dacc = 1.5 * dm;
    } else {
        *acc = m - mn;
        *dacc = dm;
    }
}

/* F_i = (V phi / dt) Acc_i + sum_j T_ij lambda_up dPhi_ij - Q_i R T / W,
 * the cell integral of the pressure form of the governing equation (Section 2); dPhi_ij = (p_i - p_j) - rho_avg g (h_i - h_j),
 * lambda = p/(mu Z) taken from the upwind cell of dPhi. */
void orc_residual(const orc_problem *pr, const double *p, const double *pn, const double *pnm1,
                  double dt, int order, double *F) {
    int N = pr->N;
    double *tx = (double *)xcalloc(N, sizeof(double));
    double *ty = (double *)xcalloc(N, sizeof(double));
    double *tz = (double *)xcalloc(N, sizeof(double));
    orc_transmissibility(pr, tx, ty, tz);
    double V = pr->dx * pr->dy * pr->dz;
    double c_rho = pr->W / (pr->R * pr->T);
    for (int i = 0; i < N; ++i) {
        double acc, dacc;
        accumulation(pr, order, p[i], pn[i], order == 2 ? pnm1[i] : 0.0, &acc, &dacc);
        double Fi = V * pr->phi[i] / dt * acc;
        double mi, dmi;
        pr_m(pr, p[i], &mi, &dmi);
        int nb[6];
        double tf[6];
        int cnt = neighbours(pr, tx, ty, tz, i, nb, tf);
        for (int q = 0; q < cnt; ++q) {
            int j = nb[q];
            double mj, dmj;
            pr_m(pr, p[j], &mj, &dmj);
            double rho_avg = 0.5 * (mi + mj) * c_rho;
            double dphi = (p[i] - p[j]) - rho_avg * pr->g * (depth_of(pr, i) - depth_of(pr, j));
            double lam = (dphi >= 0.0 ? mi : mj) / pr->mu;
            Fi += tf[q] * lam * dphi;
        }
        double dFb = 0.0;
        boundary_faces(pr, i, p[i], &Fi, &dFb, NULL);
        F[i] = Fi;
    }
    for (int w = 0; w < pr->nw; ++w)
        F[pr->wcell[w]] -= pr->wrate[w] * pr->R * pr->T / pr->W;
    free(tx); free(ty); free(tz);
}

/* Analytic Jacobian of orc_residual as CSR with sorted columns (the upwind
 * branch chosen in the residual is differentiated).  Returns nnz. */
int orc_jacobian(const orc_problem *pr, const double *p, const double *pn, const double *pnm1,
                 double dt, int order, int *rp, int *ci, double *v) {
    int N = pr->N;
    double *tx = (double *)xcalloc(N, sizeof(double));
    double *ty = (double *)xcalloc(N, sizeof(double));
    double *tz = (double *)xcalloc(N, sizeof(double));
    orc_transmissibility(pr, tx, ty, tz);
    double V = pr->dx * pr->dy * pr->dz;
    double c_rho = pr->W / (pr->R * pr->T);
    int nnz = 0;
    rp[0] = 0;
    for (int i = 0; i < N; ++i) {
        double acc, dacc;
        accumulation(pr, order, p[i], pn[i], order == 2 ? pnm1[i] : 0.0, &acc, &dacc);
        double diag = V * pr->phi[i] / dt * dacc;
        double mi, dmi;
        pr_m(pr, p[i], &mi, &dmi);
        int nb[6];
        double tf[6], off[6];
        int cnt = neighbours(pr, tx, ty, tz, i, nb, tf);
        for (int q = 0; q < cnt; ++q) {
            int j = nb[q];
            double mj, dmj;
            pr_m(pr, p[j], &mj, &dmj);
            double dh = depth_of(pr, i) - depth_of(pr, j);
            double rho_avg = 0.5 * (mi + mj) * c_rho;
            double dphi = (p[i] - p[j]) - rho_avg * pr->g * dh;
            int up_i = dphi >= 0.0;
            double lam = (up_i ? mi : mj) / pr->mu;
            double dlam_i = up_i ? dmi / pr->mu : 0.0;
            double dlam_j = up_i ? 0.0 : dmj / pr->mu;
            double ddphi_i = 1.0 - 0.5 * dmi * c_rho * pr->g * dh;
            double ddphi_j = -1.0 - 0.5 * dmj * c_rho * pr->g * dh;
            diag += tf[q] * (dlam_i * dphi + lam * ddphi_i);
            off[q] = tf[q] * (dlam_j * dphi + lam * ddphi_j);
        }
        double Fb = 0.0;
        boundary_faces(pr, i, p[i], &Fb, &diag, NULL);
        /* neighbours come in increasing column order: -z,-y,-x, then diag, +x,+y,+z */
        int q = 0;
        for (; q < cnt && nb[q] < i; ++q) { ci[nnz] = nb[q]; v[nnz++] = off[q]; }
        ci[nnz] = i; v[nnz++] = diag;
        for (; q < cnt; ++q) { ci[nnz] = nb[q]; v[nnz++] = off[q]; }
        rp[i + 1] = nnz;
    }
    free(tx); free(ty); free(tz);
    return nnz;
}

/* Hydrostatic initial state: p = p_top in the top layer and, down each
 * column, p_{k+1} - p_k = rho_avg g dz (so the gravity-corrected potential
 * difference of every vertical face is zero), solved by scalar Newton. */
void orc_hydrostatic(const orc_problem *pr, double p_top, double *p) {
    int nx = pr->nx, ny = pr->ny, nz = pr->nz, nxy = nx * ny;
    double c_rho = pr->W / (pr->R * pr->T);
    for (int c = 0; c < nxy; ++c) {
        p[c] = p_top;
        for (int k = 0; k + 1 < nz; ++k) {
            double pk = p[c + k * nxy], mk, dmk;
            pr_m(pr, pk, &mk, &dmk);
            double q = pk;
            for (int it = 0; it < 50; ++it) {
                double mq, dmq;
                pr_m(pr, q, &mq, &dmq);
                double f = q - pk - 0.5 * (mk + mq) * c_rho * pr->g * pr->dz;
                double df = 1.0 - 0.5 * dmq * c_rho * pr->g * pr->dz;
                double dq = -f / df;
                q += dq;
                if (fabs(dq) <= 1e-15 * fabs(q)) break;
            }
            p[c + (k + 1) * nxy] = q;
        }
    }
}

/* (dF/d theta)^T lam with theta_c = ln of a multiplier on all K components of
 * cell c.  Only the face transmissibilities depend on K:
 * dT_ij/d theta_i = T_ij K_j / (K_i + K_j) (same direction component), and a
 * Dirichlet boundary face's one-sided T, linear in K_i. */
void orc_residual_dlogk_t(const orc_problem *pr, const double *p, const double *lam, double *out) {
    int N = pr->N, nx = pr->nx, ny = pr->ny, nz = pr->nz, nxy = nx * ny;
    double *tx = (double *)xcalloc(N, sizeof(double));
    double *ty = (double *)xcalloc(N, sizeof(double));
    double *tz = (double *)xcalloc(N, sizeof(double));
    orc_transmissibility(pr, tx, ty, tz);
    double c_rho = pr->W / (pr->R * pr->T);
    for (int i = 0; i < N; ++i) {
        double Fb = 0.0, dFb = 0.0, dlk = 0.0;
        boundary_faces(pr, i, p[i], &Fb, &dFb, &dlk);
        out[i] = lam[i] * dlk;
    }
    for (int i = 0; i < N; ++i) {
        int x = i % nx, y = (i / nx) % ny, z = i / nxy;
        for (int d = 0; d < 3; ++d) {
            int j;
            double T, ki, kj;
            if (d == 0) { if (x + 1 >= nx) continue; j = i + 1; T = tx[i]; ki = pr->kx[i]; kj = pr->kx[j]; }
            else if (d == 1) { if (y + 1 >= ny) continue; j = i + nx; T = ty[i]; ki = pr->ky[i]; kj = pr->ky[j]; }
            else { if (z + 1 >= nz) continue; j = i + nxy; T = tz[i]; ki = pr->kz[i]; kj = pr->kz[j]; }
            double mi, dmi, mj, dmj;
            pr_m(pr, p[i], &mi, &dmi);
            pr_m(pr, p[j], &mj, &dmj);
            double rho_avg = 0.5 * (mi + mj) * c_rho;
            double dphi = (p[i] - p[j]) - rho_avg * pr->g * (depth_of(pr, i) - depth_of(pr, j));
            double lamup = (dphi >= 0.0 ? mi : mj) / pr->mu;
            double fl = lamup * dphi;          /* flux / T, enters F_i with +, F_j with - */
            double w = (lam[i] - lam[j]) * fl;
            out[i] += w * T * kj / (ki + kj);
            out[j] += w * T * ki / (ki + kj);
        }
    }
    free(tx); free(ty); free(tz);
}

/* ------------------------------------------------------------------ */
/* Sparse helpers                                                      */
/* ------------------------------------------------------------------ */
void orc_csr_matvec(int n, const int *rp, const int *ci, const double *v, const double *x, double *y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

static void csr_matvec_t(int n, int m, const int *rp, const int *ci, const double *v,
                         const double *x, double *y) {
    for (int j = 0; j < m; ++j) y[j] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) y[ci[k]] += v[k] * x[i];
}

typedef struct {
    int n, m;
    int *rp, *ci;
    double *v;
} csr;

static void csr_free(csr *a) { free(a->rp); free(a->ci); free(a->v); memset(a, 0, sizeof(*a)); }

static csr csr_transpose(const csr *a) {
    csr t;
    t.n = a->m; t.m = a->n;
    t.rp = (int *)xcalloc(t.n + 1, sizeof(int));
    int nnz = a->rp[a->n];
    t.ci = (int *)xcalloc(nnz, sizeof(int));
    t.v = (double *)xcalloc(nnz, sizeof(double));
    for (int k = 0; k < nnz; ++k) t.rp[a->ci[k] + 1]++;
    for (int j = 0; j < t.n; ++j) t.rp[j + 1] += t.rp[j];
    int *pos = (int *)xcalloc(t.n, sizeof(int));
    for (int j = 0; j < t.n; ++j) pos[j] = t.rp[j];
    for (int i = 0; i < a->n; ++i)
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int q = pos[a->ci[k]]++;
            t.ci[q] = i;
            t.v[q] = a->v[k];
        }
    free(pos);
    return t;
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* C = A B (Gustavson, dense accumulator), columns sorted, structural zeros kept */
static csr csr_matmul(const csr *a, const csr *b) {
    csr c;
    c.n = a->n; c.m = b->m;
    c.rp = (int *)xcalloc(c.n + 1, sizeof(int));
    int *mark = (int *)xcalloc(c.m, sizeof(int));
    double *acc = (double *)xcalloc(c.m, sizeof(double));
    int *cols = (int *)xcalloc(c.m, sizeof(int));
    for (int j = 0; j < c.m; ++j) mark[j] = -1;
    int cap = 16 * (a->n + 1), nnz = 0;
    c.ci = (int *)xcalloc(cap, sizeof(int));
    c.v = (double *)xcalloc(cap, sizeof(double));
    for (int i = 0; i < a->n; ++i) {
        int nc = 0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            int r = a->ci[k];
            double av = a->v[k];
            for (int q = b->rp[r]; q < b->rp[r + 1]; ++q) {
                int j = b->ci[q];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[nc++] = j; }
                acc[j] += av * b->v[q];
            }
        }
        qsort(cols, nc, sizeof(int), cmp_int);
        if (nnz + nc > cap) {
            while (nnz + nc > cap) cap *= 2;
            c.ci = (int *)realloc(c.ci, cap * sizeof(int));
            c.v = (double *)realloc(c.v, cap * sizeof(double));
            if (!c.ci || !c.v) abort();
        }
        for (int q = 0; q < nc; ++q) { c.ci[nnz] = cols[q]; c.v[nnz++] = acc[cols[q]]; }
        c.rp[i + 1] = nnz;
    }
    free(mark); free(acc); free(cols);
    return c;
}

/* ------------------------------------------------------------------ */
/* Interpolation operators (Section 3.2, first/second/third order) */
/* ------------------------------------------------------------------ */

/* Cubic convolution weight W(s) of the third-order interpolation of Section 3.2 (values at integer s by continuity). */
static double keys_w(double s) {
    s = fabs(s);
    if (s < 1.0) return 1.5 * s * s * s - 2.5 * s * s + 1.0;
    if (s < 2.0) return -0.5 * s * s * s + 2.5 * s * s - 4.0 * s + 2.0;
    return 0.0;
}

/* One-dimensional factor of the interpolation from nc = ceil(nf/r) coarse
 * cells to nf fine cells, coarse-to-fine ratio r (Section 3.2 with its mesh
 * ratios; cell-centred nesting).  Fine centre x_i = i + 1/2 (fine cell units);
 * coarse cell J covers fine cells rJ .. min(rJ + r, nf) - 1 and sits at their
 * centroid c_J (the last one is short when r does not divide nf).
 *
 * Orders 2 and 3 interpolate in the coarse index coordinate s(x): piecewise
 * linear through the points (c_J, J), continued beyond both ends with slope
 * 1/r (virtual centroids one coarse spacing outside).  Order 2 is the linear
 * interpolant between the two centroids around x (the hat function in s);
 * order 3 weights coarse cells J0-1 .. J0+2 (J0 = floor(s)) by the cubic
 * convolution kernel W(s - J).  On uniform spacing s = (x - c_0)/r and these
 * are the printed weights; at a short last cell they use its actual centroid.
 * Order 1: the parent cell.  Coarse indices beyond the domain are clamped to
 * the edge cell and their weights merged, so every row sums to 1.
 * Row i holds at most 4 entries (sorted columns); rp has nf+1 entries. */
void orc_interp_1d_r(int nf, int order, int ratio, int *rp, int *ci, double *w) {
    int r = ratio;
    int nc = (nf + r - 1) / r;
    int nnz = 0;
    rp[0] = 0;
    for (int i = 0; i < nf; ++i) {
        double x = i + 0.5;
        int cj[4];
        double cw[4];
        int cnt = 0;
        if (nf == 1) {
            cj[0] = 0; cw[0] = 1.0; cnt = 1;
        } else if (order == 1) {
            /* the parent cell (the first-order interpolation of Section 3.2) */
            cj[0] = i / r; cw[0] = 1.0; cnt = 1;
        } else {
            /* index coordinate of x */
            double first = 0.5 * (double)(r < nf ? r : nf);
            int lo_last = r * (nc - 1);
            double last = 0.5 * (double)(lo_last + nf);
            double sx;
            if (x <= first) sx = (x - first) / r;
            else if (x >= last) sx = (nc - 1) + (x - last) / r;
            else {
                /* c_J = rJ + r/2 for every full cell, and x < last <= c_{nc-2} + r */
                int J = (int)floor((x - first) / r);
                if (J > nc - 2) J = nc - 2;
                double cJ = r * J + 0.5 * r;
                double cJ1 = (J + 1 == nc - 1) ? last : cJ + r;
                sx = J + (x - cJ) / (cJ1 - cJ);
            }
            int J0 = (int)floor(sx);
            double t = sx - J0;
            if (order == 2) {
                /* the second-order interpolation of Section 3.2 along one direction */
                cj[0] = J0; cw[0] = 1.0 - t;
                cj[1] = J0 + 1; cw[1] = t;
                cnt = 2;
            } else {
                /* the third-order interpolation of Section 3.2 along one direction */
                for (int l = -1; l <= 2; ++l) {
                    cj[cnt] = J0 + l; cw[cnt] = keys_w(sx - (J0 + l)); cnt++;
                }
            }
        }
        /* clamp out-of-range coarse indices and merge equal columns */
        int oj[4];
        double ow[4];
        int oc = 0;
        for (int q = 0; q < cnt; ++q) {
            int J = cj[q];
            if (J < 0) J = 0;
            if (J > nc - 1) J = nc - 1;
            int f = -1;
            for (int rr = 0; rr < oc; ++rr) if (oj[rr] == J) f = rr;
            if (f < 0) { oj[oc] = J; ow[oc] = cw[q]; oc++; }
            else ow[f] += cw[q];
        }
        /* sort by column, drop exact zeros */
        for (int a = 0; a < oc; ++a)
            for (int b = a + 1; b < oc; ++b)
                if (oj[b] < oj[a]) { int tt = oj[a]; oj[a] = oj[b]; oj[b] = tt; double u = ow[a]; ow[a] = ow[b]; ow[b] = u; }
        for (int q = 0; q < oc; ++q) {
            if (ow[q] == 0.0) continue;
            ci[nnz] = oj[q]; w[nnz++] = ow[q];
        }
        rp[i + 1] = nnz;
    }
}

/* ratio 2 */
void orc_interp_1d(int nf, int order, int *rp, int *ci, double *w) {
    orc_interp_1d_r(nf, order, 2, rp, ci, w);
}

/* Tensor product of the 1D factors: P (nf x nc) on the cell-centred grid */
static csr interp_matrix(int nx, int ny, int nz, int order, int ratio, int *cnx, int *cny, int *cnz) {
    int ncx = nx > 1 ? (nx + ratio - 1) / ratio : 1;
    int ncy = ny > 1 ? (ny + ratio - 1) / ratio : 1;
    int ncz = nz > 1 ? (nz + ratio - 1) / ratio : 1;
    *cnx = ncx; *cny = ncy; *cnz = ncz;
    int *rx = (int *)xcalloc(nx + 1, sizeof(int)), *cx = (int *)xcalloc(4 * nx, sizeof(int));
    int *ry = (int *)xcalloc(ny + 1, sizeof(int)), *cy = (int *)xcalloc(4 * ny, sizeof(int));
    int *rz = (int *)xcalloc(nz + 1, sizeof(int)), *cz = (int *)xcalloc(4 * nz, sizeof(int));
    double *wx = (double *)xcalloc(4 * nx, sizeof(double));
    double *wy = (double *)xcalloc(4 * ny, sizeof(double));
    double *wz = (double *)xcalloc(4 * nz, sizeof(double));
    orc_interp_1d_r(nx, order, ratio, rx, cx, wx);
    orc_interp_1d_r(ny, order, ratio, ry, cy, wy);
    orc_interp_1d_r(nz, order, ratio, rz, cz, wz);
    csr P;
    P.n = nx * ny * nz;
    P.m = ncx * ncy * ncz;
    P.rp = (int *)xcalloc(P.n + 1, sizeof(int));
    P.ci = (int *)xcalloc((size_t)P.n * 64, sizeof(int));
    P.v = (double *)xcalloc((size_t)P.n * 64, sizeof(double));
    int nnz = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int i = x + nx * (y + ny * z);
                /* columns come out sorted: z outer, then y, then x */
                for (int a = rz[z]; a < rz[z + 1]; ++a)
                    for (int b = ry[y]; b < ry[y + 1]; ++b)
                        for (int c = rx[x]; c < rx[x + 1]; ++c) {
                            P.ci[nnz] = cx[c] + ncx * (cy[b] + ncy * cz[a]);
                            P.v[nnz++] = wx[c] * wy[b] * wz[a];
                        }
                P.rp[i + 1] = nnz;
            }
    free(rx); free(cx); free(ry); free(cy); free(rz); free(cz);
    free(wx); free(wy); free(wz);
    return P;
}

/* ------------------------------------------------------------------ */
/* Subdomain solvers                                                   */
/* ------------------------------------------------------------------ */

/* ILU(0) in IKJ form on a CSR matrix with sorted columns (in place):
 * for each row i and each k < i in its pattern (ascending), a_ik /= a_kk and
 * a_ij -= a_ik a_kj for every j > k present in both rows.  Afterwards the
 * strict lower part holds L (unit diagonal implied) and the rest holds U. */
void orc_ilu0(int n, const int *rp, const int *ci, double *v) {
    int *pos = (int *)xcalloc(n, sizeof(int));
    int *dg = (int *)xcalloc(n, sizeof(int));
    for (int j = 0; j < n; ++j) pos[j] = -1;
    for (int i = 0; i < n; ++i) {
        dg[i] = -1;
        for (int k = rp[i]; k < rp[i + 1]; ++k) if (ci[k] == i) dg[i] = k;
    }
    for (int i = 0; i < n; ++i) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = k;
        for (int k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) {
            int r = ci[k];
            v[k] /= v[dg[r]];
            for (int q = dg[r] + 1; q < rp[r + 1]; ++q) {
                int j = ci[q];
                if (pos[j] >= 0) v[pos[j]] -= v[k] * v[q];
            }
        }
        for (int k = rp[i]; k < rp[i + 1]; ++k) pos[ci[k]] = -1;
    }
    free(pos); free(dg);
}

/* Level-of-fill pattern of ILU(k) (Section 3.1's subdomain solver with k
 * levels of fill): an original entry has level 0; eliminating row k < i from
 * row i gives entry (i, j), j > k, the level lev(i,k) + lev(k,j) + 1, kept
 * (as the minimum over k) when it is at most k_fill.  Rows are processed in
 * order and the lower entries of a row in increasing column order, so every
 * level used is final.  a is replaced by the expanded matrix: its own values,
 * zero at the fill positions, columns sorted.  ILU(0) on that pattern is
 * ILU(k). */
static void iluk_pattern(csr *a, int kfill) {
    const int n = a->n;
    int *lev = (int *)xcalloc(n, sizeof(int));
    double *val = (double *)xcalloc(n, sizeof(double));
    int *touched = (int *)xcalloc(n, sizeof(int));
    for (int j = 0; j < n; ++j) lev[j] = INT_MAX;
    int cap = a->rp[n] * 2 + 16, nnz = 0;
    int *rp = (int *)xcalloc(n + 1, sizeof(int));
    int *ci = (int *)xcalloc(cap, sizeof(int));
    int *lv = (int *)xcalloc(cap, sizeof(int));
    double *v = (double *)xcalloc(cap, sizeof(double));
    for (int i = 0; i < n; ++i) {
        int nt = 0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; ++k) {
            lev[a->ci[k]] = 0;
            val[a->ci[k]] = a->v[k];
            touched[nt++] = a->ci[k];
        }
        for (int k = 0; k < i; ++k) {
            if (lev[k] > kfill) continue;
            for (int q = rp[k]; q < rp[k + 1]; ++q) {
                const int j = ci[q];
                if (j <= k) continue;
                const int l = lev[k] + lv[q] + 1;
                if (l <= kfill && l < lev[j]) {
                    if (lev[j] == INT_MAX) touched[nt++] = j;
                    lev[j] = l;
                }
            }
        }
        /* row i in increasing column order */
        for (int j = 0; j < n; ++j) {
            if (lev[j] > kfill) continue;
            if (nnz == cap) {
                cap *= 2;
                ci = (int *)realloc(ci, (size_t)cap * sizeof(int));
                lv = (int *)realloc(lv, (size_t)cap * sizeof(int));
                v = (double *)realloc(v, (size_t)cap * sizeof(double));
                if (!ci || !lv || !v) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
            }
            ci[nnz] = j;
            lv[nnz] = lev[j];
            v[nnz++] = val[j];
        }
        rp[i + 1] = nnz;
        for (int t = 0; t < nt; ++t) {
            lev[touched[t]] = INT_MAX;
            val[touched[t]] = 0.0;
        }
    }
    free(a->rp); free(a->ci); free(a->v);
    a->rp = rp;
    a->ci = ci;
    a->v = v;
    free(lv); free(lev); free(val); free(touched);
}

/* Solve (L U) z = r with the factors of orc_ilu0 */
void orc_ilu0_solve(int n, const int *rp, const int *ci, const double *v, const double *r, double *z) {
    for (int i = 0; i < n; ++i) {
        double s = r[i];
        for (int k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) s -= v[k] * z[ci[k]];
        z[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i], d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            if (ci[k] > i) s -= v[k] * z[ci[k]];
            else if (ci[k] == i) d = v[k];
        }
        z[i] = s / d;
    }
}

/* transpose solve: (L U)^T z = r, i.e. U^T w = r then L^T z = w */
static void ilu0_solve_t(int n, const int *rp, const int *ci, const double *v, const double *r, double *z) {
    double *w = (double *)xcalloc(n, sizeof(double));
    memcpy(w, r, n * sizeof(double));
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) if (ci[k] == i) d = v[k];
        w[i] /= d;
        for (int k = rp[i]; k < rp[i + 1]; ++k) if (ci[k] > i) w[ci[k]] -= v[k] * w[i];
    }
    for (int i = n - 1; i >= 0; --i)
        for (int k = rp[i]; k < rp[i + 1] && ci[k] < i; ++k) w[ci[k]] -= v[k] * w[i];
    memcpy(z, w, n * sizeof(double));
    free(w);
}

/* dense LU with partial pivoting (exact subdomain solve) */
static void dense_lu(int n, double *a, int *piv) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i) if (fabs(a[i * n + k]) > fabs(a[p * n + k])) p = i;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = a[k * n + j]; a[k * n + j] = a[p * n + j]; a[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            a[i * n + k] /= a[k * n + k];
            for (int j = k + 1; j < n; ++j) a[i * n + j] -= a[i * n + k] * a[k * n + j];
        }
    }
}

static void dense_lu_solve(int n, const double *a, const int *piv, const double *r, double *z, int trans) {
    double *y = (double *)xcalloc(n, sizeof(double));
    memcpy(y, r, n * sizeof(double));
    if (!trans) {
        for (int k = 0; k < n; ++k) { double t = y[k]; y[k] = y[piv[k]]; y[piv[k]] = t; }
        for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) y[i] -= a[i * n + j] * y[j];
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i + 1; j < n; ++j) y[i] -= a[i * n + j] * y[j];
            y[i] /= a[i * n + i];
        }
    } else {
        /* A = P^T L U  ->  A^T = U^T L^T P */
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < i; ++j) y[i] -= a[j * n + i] * y[j];
            y[i] /= a[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) for (int j = i + 1; j < n; ++j) y[i] -= a[j * n + i] * y[j];
        for (int k = n - 1; k >= 0; --k) { double t = y[k]; y[k] = y[piv[k]]; y[piv[k]] = t; }
    }
    memcpy(z, y, n * sizeof(double));
    free(y);
}

/* ------------------------------------------------------------------ */
/* One-level Schwarz (Section 3.1)                                     */
/* ------------------------------------------------------------------ */
typedef struct {
    int next;            /* |Omega_i^delta| */
    int *cells;          /* global index of each local cell, local lexicographic order */
    int *owned;          /* 1 if the cell is in Omega_i */
    int lo[3], hi[3], elo[3], ehi[3];
    csr a;               /* principal submatrix R^delta A R^delta^T, then its ILU(0) */
    double *lu;          /* dense LU (exact solve) */
    int *piv;
} subdomain;

typedef struct {
    int nx, ny, nz, n;
    csr A;
    int nsub;
    subdomain *sub;
    csr P;               /* interpolation from the next coarser level to this one */
    int has_p;
} level;

struct orc_mg {
    orc_mg_desc d;
    int L;
    level lev[MAXLEV];   /* lev[0] is the finest, lev[L-1] the coarsest */
    double *work[MAXLEV][4];
    /* rediscretised coarse operators: the upscaled problem of each coarse
     * level (cprob[0] unused: the fine problem is the caller's) */
    orc_problem *cprob[MAXLEV];
    double odt;
    int oorder;
};

/* Lagged refactorisation: the current Jacobian's values (same pattern) on the
 * finest level and fresh Galerkin products P^T A P below it; the subdomain
 * ILU factors of the last build are kept. */
static void rediscretise(orc_mg *mg, const orc_problem *pr, const double *p);

static void mg_refresh_operators(orc_mg *mg, const double *v, const orc_problem *pr, const double *p) {
    level *f = &mg->lev[0];
    memcpy(f->A.v, v, (size_t)f->A.rp[f->A.n] * sizeof(double));
    if (mg->d.coarse_op == ORC_COARSE_REDISCRETISED) {
        if (mg->L > 1) rediscretise(mg, pr, p);
        return;
    }
    for (int l = 0; l + 1 < mg->L; ++l) {
        level *fl = &mg->lev[l], *cl = &mg->lev[l + 1];
        csr AP = csr_matmul(&fl->A, &fl->P);
        csr Pt = csr_transpose(&fl->P);
        csr_free(&cl->A);
        cl->A = csr_matmul(&Pt, &AP);
        csr_free(&AP); csr_free(&Pt);
    }
}

/* box q of P boxes along n cells: floor(n/P) cells plus one for the first n mod P */
static void box_range(int n, int P, int q, int *lo, int *hi) {
    int base = n / P, rem = n % P;
    *lo = q * base + (q < rem ? q : rem);
    *hi = *lo + base + (q < rem ? 1 : 0);
}

static void build_subdomains(level *lv, const int *Pbox, int delta) {
    int P[3] = {Pbox[0], Pbox[1], Pbox[2]};
    int n[3] = {lv->nx, lv->ny, lv->nz};
    for (int k = 0; k < 3; ++k) if (P[k] > n[k]) P[k] = n[k];
    lv->nsub = P[0] * P[1] * P[2];
    lv->sub = (subdomain *)xcalloc(lv->nsub, sizeof(subdomain));
    int *loc = (int *)xcalloc(lv->n, sizeof(int));
    for (int sz = 0; sz < P[2]; ++sz)
        for (int sy = 0; sy < P[1]; ++sy)
            for (int sx = 0; sx < P[0]; ++sx) {
                subdomain *s = &lv->sub[sx + P[0] * (sy + P[1] * sz)];
                int q[3] = {sx, sy, sz};
                for (int k = 0; k < 3; ++k) {
                    box_range(n[k], P[k], q[k], &s->lo[k], &s->hi[k]);
                    s->elo[k] = s->lo[k] - delta < 0 ? 0 : s->lo[k] - delta;
                    s->ehi[k] = s->hi[k] + delta > n[k] ? n[k] : s->hi[k] + delta;
                }
                int ex = s->ehi[0] - s->elo[0], ey = s->ehi[1] - s->elo[1], ez = s->ehi[2] - s->elo[2];
                s->next = ex * ey * ez;
                s->cells = (int *)xcalloc(s->next, sizeof(int));
                s->owned = (int *)xcalloc(s->next, sizeof(int));
                int c = 0;
                for (int z = s->elo[2]; z < s->ehi[2]; ++z)
                    for (int y = s->elo[1]; y < s->ehi[1]; ++y)
                        for (int x = s->elo[0]; x < s->ehi[0]; ++x) {
                            s->cells[c] = x + n[0] * (y + n[1] * z);
                            s->owned[c] = x >= s->lo[0] && x < s->hi[0] && y >= s->lo[1] &&
                                          y < s->hi[1] && z >= s->lo[2] && z < s->hi[2];
                            c++;
                        }
            }
    free(loc);
}

/* A_i = R_i^delta A (R_i^delta)^T: rows and columns of the extended cells */
static void factor_subdomains(level *lv, const orc_mg_desc *d) {
    int *map = (int *)xcalloc(lv->n, sizeof(int));
    for (int i = 0; i < lv->n; ++i) map[i] = -1;
    for (int si = 0; si < lv->nsub; ++si) {
        subdomain *s = &lv->sub[si];
        for (int c = 0; c < s->next; ++c) map[s->cells[c]] = c;
        csr_free(&s->a);
        s->a.n = s->a.m = s->next;
        s->a.rp = (int *)xcalloc(s->next + 1, sizeof(int));
        int cap = 0;
        for (int c = 0; c < s->next; ++c) {
            int g = s->cells[c];
            cap += lv->A.rp[g + 1] - lv->A.rp[g];
        }
        s->a.ci = (int *)xcalloc(cap, sizeof(int));
        s->a.v = (double *)xcalloc(cap, sizeof(double));
        int nnz = 0;
        for (int c = 0; c < s->next; ++c) {
            int g = s->cells[c];
            for (int k = lv->A.rp[g]; k < lv->A.rp[g + 1]; ++k) {
                int lc = map[lv->A.ci[k]];
                if (lc < 0) continue;
                s->a.ci[nnz] = lc;
                s->a.v[nnz++] = lv->A.v[k];
            }
            s->a.rp[c + 1] = nnz;
        }
        /* local numbering is lexicographic, and so is the global one, so the
         * columns of each row stay sorted */
        if (d->subsolve == 1) {
            free(s->lu); free(s->piv);
            s->lu = (double *)xcalloc((size_t)s->next * s->next, sizeof(double));
            s->piv = (int *)xcalloc(s->next, sizeof(int));
            for (int r = 0; r < s->next; ++r)
                for (int k = s->a.rp[r]; k < s->a.rp[r + 1]; ++k)
                    s->lu[(size_t)r * s->next + s->a.ci[k]] = s->a.v[k];
            dense_lu(s->next, s->lu, s->piv);
        } else {
            if (d->fill > 0) iluk_pattern(&s->a, d->fill);
            orc_ilu0(s->next, s->a.rp, s->a.ci, s->a.v);
        }
        for (int c = 0; c < s->next; ++c) map[s->cells[c]] = -1;
    }
    free(map);
}

static void sub_solve(const subdomain *s, int subsolve, const double *r, double *z, int trans) {
    if (subsolve == 1) dense_lu_solve(s->next, s->lu, s->piv, r, z, trans);
    else if (!trans) orc_ilu0_solve(s->next, s->a.rp, s->a.ci, s->a.v, r, z);
    else ilu0_solve_t(s->next, s->a.rp, s->a.ci, s->a.v, r, z);
}

/* z = M^{-1} r for the one-level preconditioner of the left-RAS operator of Section 3.1 (left-RAS:
 * sum_i R_i^0^T A_i^{-1} R_i^delta), the classical AS operator of Section 3.1 (AS) or the right-RAS operator of Section 3.1
 * (right-RAS: sum_i R_i^delta^T A_i^{-1} R_i^0).  trans applies M^{-T}. */
static void onelevel_apply(const level *lv, const orc_mg_desc *d, const double *r, double *z, int trans) {
    int var = d->variant;
    if (trans) { if (var == 0) var = 2; else if (var == 2) var = 0; }
    for (int i = 0; i < lv->n; ++i) z[i] = 0.0;
    int maxn = 0;
    for (int si = 0; si < lv->nsub; ++si) if (lv->sub[si].next > maxn) maxn = lv->sub[si].next;
    double *rl = (double *)xcalloc(maxn, sizeof(double));
    double *zl = (double *)xcalloc(maxn, sizeof(double));
    for (int si = 0; si < lv->nsub; ++si) {
        const subdomain *s = &lv->sub[si];
        for (int c = 0; c < s->next; ++c)
            rl[c] = (var == 2 && !s->owned[c]) ? 0.0 : r[s->cells[c]];
        sub_solve(s, d->subsolve, rl, zl, trans);
        for (int c = 0; c < s->next; ++c)
            if (var != 0 || s->owned[c]) z[s->cells[c]] += zl[c];
    }
    free(rl); free(zl);
}

/* ------------------------------------------------------------------ */
/* GMRES / FGMRES (Section 3, the Jacobian system; Remark 2)                  */
/* ------------------------------------------------------------------ */
typedef void (*op_fn)(void *ctx, const double *x, double *y);

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Right-preconditioned GMRES(m) with modified Gram-Schmidt and Givens
 * rotations; x holds the initial guess on entry.  Stops when the residual
 * norm is <= max(rtol ||b||, atol).  flexible keeps Z_j = M^{-1} v_j (FGMRES). */
static int gmres_core(int n, op_fn A, void *actx, op_fn M, void *mctx, const double *b, double *x,
                      int m, double rtol, double atol, int maxit, int flexible,
                      double *res_out, int *its_out) {
    double *V = (double *)xcalloc((size_t)(m + 1) * n, sizeof(double));
    double *Zs = flexible ? (double *)xcalloc((size_t)m * n, sizeof(double)) : NULL;
    double *H = (double *)xcalloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)xcalloc(m, sizeof(double)), *sn = (double *)xcalloc(m, sizeof(double));
    double *g = (double *)xcalloc(m + 1, sizeof(double)), *y = (double *)xcalloc(m, sizeof(double));
    double *w = (double *)xcalloc(n, sizeof(double)), *t = (double *)xcalloc(n, sizeof(double));
    double bnorm = sqrt(dot(n, b, b));
    double tol = rtol * bnorm > atol ? rtol * bnorm : atol;
    int its = 0, conv = 0;
    double res = 0.0;
    while (1) {
        A(actx, x, w);
        for (int i = 0; i < n; ++i) V[i] = b[i] - w[i];
        double beta = sqrt(dot(n, V, V));
        res = beta;
        if (beta <= tol) { conv = 1; break; }
        if (its >= maxit) break;
        for (int i = 0; i < n; ++i) V[i] /= beta;
        for (int k = 0; k <= m; ++k) g[k] = 0.0;
        g[0] = beta;
        int j = 0;
        for (; j < m && its < maxit; ++j) {
            double *vj = V + (size_t)j * n;
            double *zj = flexible ? Zs + (size_t)j * n : t;
            if (M) M(mctx, vj, zj); else memcpy(zj, vj, n * sizeof(double));
            A(actx, zj, w);
            for (int k = 0; k <= j; ++k) {
                double h = dot(n, w, V + (size_t)k * n);
                H[k * m + j] = h;
                for (int i = 0; i < n; ++i) w[i] -= h * V[(size_t)k * n + i];
            }
            double hn = sqrt(dot(n, w, w));
            H[(j + 1) * m + j] = hn;
            if (hn > 0.0) for (int i = 0; i < n; ++i) V[(size_t)(j + 1) * n + i] = w[i] / hn;
            for (int k = 0; k < j; ++k) {
                double a = H[k * m + j], bb = H[(k + 1) * m + j];
                H[k * m + j] = cs[k] * a + sn[k] * bb;
                H[(k + 1) * m + j] = -sn[k] * a + cs[k] * bb;
            }
            double a = H[j * m + j], bb = H[(j + 1) * m + j];
            double den = sqrt(a * a + bb * bb);
            cs[j] = den > 0.0 ? a / den : 1.0;
            sn[j] = den > 0.0 ? bb / den : 0.0;
            H[j * m + j] = den;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            its++;
            res = fabs(g[j + 1]);
            if (res <= tol || hn == 0.0) { j++; conv = 1; break; }
        }
        /* back substitution and update */
        for (int k = j - 1; k >= 0; --k) {
            double s = g[k];
            for (int q = k + 1; q < j; ++q) s -= H[k * m + q] * y[q];
            y[k] = s / H[k * m + k];
        }
        if (flexible) {
            for (int k = 0; k < j; ++k)
                for (int i = 0; i < n; ++i) x[i] += y[k] * Zs[(size_t)k * n + i];
        } else {
            for (int i = 0; i < n; ++i) w[i] = 0.0;
            for (int k = 0; k < j; ++k)
                for (int i = 0; i < n; ++i) w[i] += y[k] * V[(size_t)k * n + i];
            if (M) M(mctx, w, t); else memcpy(t, w, n * sizeof(double));
            for (int i = 0; i < n; ++i) x[i] += t[i];
        }
        if (conv) {
            A(actx, x, w);
            for (int i = 0; i < n; ++i) w[i] = b[i] - w[i];
            res = sqrt(dot(n, w, w));
            break;
        }
        if (its >= maxit) {
            A(actx, x, w);
            for (int i = 0; i < n; ++i) w[i] = b[i] - w[i];
            res = sqrt(dot(n, w, w));
            break;
        }
    }
    if (res_out) *res_out = res;
    if (its_out) *its_out = its;
    free(V); free(Zs); free(H); free(cs); free(sn); free(g); free(y); free(w); free(t);
    return conv ? 0 : 1;
}

typedef struct { const csr *a; int trans; } csr_op;

static void csr_op_apply(void *ctx, const double *x, double *y) {
    csr_op *o = (csr_op *)ctx;
    if (o->trans) csr_matvec_t(o->a->n, o->a->m, o->a->rp, o->a->ci, o->a->v, x, y);
    else orc_csr_matvec(o->a->n, o->a->rp, o->a->ci, o->a->v, x, y);
}

/* ------------------------------------------------------------------ */
/* Multilevel Schwarz (Section 3.2, Algorithm 1)                       */
/* ------------------------------------------------------------------ */
typedef struct { orc_mg *mg; int lev; int trans; } onelev_ctx;

static void onelev_op(void *ctx, const double *r, double *z) {
    onelev_ctx *c = (onelev_ctx *)ctx;
    onelevel_apply(&c->mg->lev[c->lev], &c->mg->d, r, z, c->trans);
}

/* coarsest correction: A_{h_0} X = b by one-level Schwarz preconditioned
 * GMRES from X = 0 to the coarse relative tolerance (Remark 2) */
static void coarse_solve(orc_mg *mg, const double *b, double *x, int trans) {
    int c = mg->L - 1;
    level *lv = &mg->lev[c];
    for (int i = 0; i < lv->n; ++i) x[i] = 0.0;
    csr_op aop = {&lv->A, trans};
    onelev_ctx mc = {mg, c, trans};
    gmres_core(lv->n, csr_op_apply, &aop, onelev_op, &mc, b, x, mg->d.coarse_restart,
               mg->d.coarse_rtol, 0.0, mg->d.coarse_maxit, 0, NULL, NULL);
}

/* r = b - A x, or b - A^T x when trans */
static void residual_update(const level *lv, const double *b, const double *x, double *r, int trans) {
    if (trans) csr_matvec_t(lv->n, lv->n, lv->A.rp, lv->A.ci, lv->A.v, x, r);
    else orc_csr_matvec(lv->n, lv->A.rp, lv->A.ci, lv->A.v, x, r);
    for (int i = 0; i < lv->n; ++i) r[i] = b[i] - r[i];
}

/* X = MG(b, level, 0) of Algorithm 1 with the composition chosen by the
 * cycle type; lev indexes from the finest (0) down to the coarsest (L-1).
 * trans applies the transpose of that linear map (exact when the coarse
 * solve is): every factor of the composition is transposed and their order
 * reversed, so A, the smoother and the coarse solve become their transposes,
 * P and P^T keep their places, and the mu pre- and nu post-smoothing steps
 * trade places (left and right Kaskade exchange). */
static void mg_cycle(orc_mg *mg, int li, const double *b, double *x, int trans) {
    level *lv = &mg->lev[li];
    int n = lv->n;
    if (li == mg->L - 1) { coarse_solve(mg, b, x, trans); return; }
    level *cl = &mg->lev[li + 1];
    double *r = mg->work[li][0], *t = mg->work[li][1];
    double *bc = mg->work[li + 1][2], *xc = mg->work[li + 1][3];
    int cyc = mg->d.cycle;
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    if (cyc == 3 || cyc == 4) {
        /* additive two-level form: I P M0 P^T b + M b;  coarse-only form: I P M0 P^T b */
        csr_matvec_t(n, cl->n, lv->P.rp, lv->P.ci, lv->P.v, b, bc);
        mg_cycle(mg, li + 1, bc, xc, trans);
        orc_csr_matvec(n, lv->P.rp, lv->P.ci, lv->P.v, xc, x);
        if (cyc == 3) {
            onelevel_apply(lv, &mg->d, b, t, trans);
            for (int i = 0; i < n; ++i) x[i] += t[i];
        }
        return;
    }
    int mu = mg->d.mu, nu = mg->d.nu;
    if (cyc == 1) { mu = 0; nu = 1; }        /* left Kaskade */
    else if (cyc == 2) { mu = 1; nu = 0; }   /* right Kaskade */
    if (trans) { int tmp = mu; mu = nu; nu = tmp; }
    /* presmoothing: Schwarz-preconditioned Richardson, mu sweeps */
    for (int s = 0; s < mu; ++s) {
        residual_update(lv, b, x, r, trans);
        onelevel_apply(lv, &mg->d, r, t, trans);
        for (int i = 0; i < n; ++i) x[i] += t[i];
    }
    /* residual restriction with P^T, recursive correction, interpolation */
    residual_update(lv, b, x, r, trans);
    csr_matvec_t(n, cl->n, lv->P.rp, lv->P.ci, lv->P.v, r, bc);
    mg_cycle(mg, li + 1, bc, xc, trans);
    orc_csr_matvec(n, lv->P.rp, lv->P.ci, lv->P.v, xc, t);
    for (int i = 0; i < n; ++i) x[i] += t[i];
    /* postsmoothing, nu sweeps */
    for (int s = 0; s < nu; ++s) {
        residual_update(lv, b, x, r, trans);
        onelevel_apply(lv, &mg->d, r, t, trans);
        for (int i = 0; i < n; ++i) x[i] += t[i];
    }
}

/* Rediscretised coarse problem (the alternative to the Galerkin product for
 * the coarse matrices of Section 3.2): cells of r x r (x r) fine cells, each
 * permeability component the arithmetic mean of the children's, porosity the
 * mean (so the pore volume is the children's sum), r times the cell size,
 * the same fluid, gravity, outer-face conditions and wells (moved to the
 * coarse cell holding them).  Every size above one must be a multiple of r;
 * returns NULL otherwise. */
orc_problem *orc_problem_coarsen(const orc_problem *pr, int r) {
    int n[3] = {pr->nx, pr->ny, pr->nz}, nc[3], rr[3];
    for (int k = 0; k < 3; ++k) {
        rr[k] = n[k] > 1 ? r : 1;
        if (n[k] % rr[k]) return NULL;
        nc[k] = n[k] / rr[k];
    }
    int Nc = nc[0] * nc[1] * nc[2];
    double *kx = (double *)xcalloc(Nc, sizeof(double)), *ky = (double *)xcalloc(Nc, sizeof(double));
    double *kz = (double *)xcalloc(Nc, sizeof(double)), *ph = (double *)xcalloc(Nc, sizeof(double));
    double inv = 1.0 / (rr[0] * rr[1] * rr[2]);
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                int i = x + n[0] * (y + n[1] * z);
                int I = x / rr[0] + nc[0] * (y / rr[1] + nc[1] * (z / rr[2]));
                kx[I] += inv * pr->kx[i];
                ky[I] += inv * pr->ky[i];
                kz[I] += inv * pr->kz[i];
                ph[I] += inv * pr->phi[i];
            }
    int *wc = (int *)xcalloc(pr->nw, sizeof(int));
    for (int w = 0; w < pr->nw; ++w) {
        int i = pr->wcell[w];
        int x = i % n[0], y = (i / n[0]) % n[1], z = i / (n[0] * n[1]);
        wc[w] = x / rr[0] + nc[0] * (y / rr[1] + nc[1] * (z / rr[2]));
    }
    orc_problem *c = orc_problem_new(nc[0], nc[1], nc[2], pr->dx * rr[0], pr->dy * rr[1], pr->dz * rr[2],
                                     kx, ky, kz, ph, pr->nw, wc, pr->wrate, pr->Tc, pr->pc, pr->omega, pr->T,
                                     pr->W, pr->R, pr->mu, pr->g != 0.0, pr->g);
    for (int f = 0; f < 6; ++f) c->bct[f] = pr->bct[f], c->bcv[f] = pr->bcv[f];
    c->accum = pr->accum;
    /* the fine problem's constants as they are (omega may have come from T_b) */
    c->a = pr->a; c->b = pr->b; c->mpr = pr->mpr;
    free(kx); free(ky); free(kz); free(ph); free(wc);
    return c;
}

/* the coarse state: each coarse cell takes the mean of its children */
static void coarsen_state(const orc_problem *f, const orc_problem *c, const double *pf, double *pc) {
    int rx = f->nx / c->nx, ry = f->ny / c->ny, rz = f->nz / c->nz;
    for (int I = 0; I < c->N; ++I) pc[I] = 0.0;
    double inv = 1.0 / (rx * ry * rz);
    for (int z = 0; z < f->nz; ++z)
        for (int y = 0; y < f->ny; ++y)
            for (int x = 0; x < f->nx; ++x)
                pc[x / rx + c->nx * (y / ry + c->ny * (z / rz))] += inv * pf[x + f->nx * (y + f->ny * z)];
}

/* coarse matrices of the rediscretised hierarchy: the Jacobian of each
 * coarse problem at the coarsened state, with no BDF difference (the
 * accumulation enters through its coefficient alone) */
static void rediscretise(orc_mg *mg, const orc_problem *pr, const double *p) {
    const orc_problem *fp = pr;
    double *ps = (double *)xcalloc(pr->N, sizeof(double));
    memcpy(ps, p, pr->N * sizeof(double));
    for (int l = 1; l < mg->L; ++l) {
        const orc_problem *cp = mg->cprob[l];
        double *pc = (double *)xcalloc(cp->N, sizeof(double));
        coarsen_state(fp, cp, ps, pc);
        level *cl = &mg->lev[l];
        csr_free(&cl->A);
        cl->A.n = cl->A.m = cp->N;
        cl->A.rp = (int *)xcalloc(cp->N + 1, sizeof(int));
        cl->A.ci = (int *)xcalloc((size_t)7 * cp->N, sizeof(int));
        cl->A.v = (double *)xcalloc((size_t)7 * cp->N, sizeof(double));
        orc_jacobian(cp, pc, pc, pc, mg->odt, mg->oorder, cl->A.rp, cl->A.ci, cl->A.v);
        free(ps);
        ps = pc;
        fp = cp;
    }
    free(ps);
}

/* The level hierarchy: the fine matrix, interpolation to each coarser level,
 * coarse matrices (Galerkin P^T A P, or the rediscretised problems' Jacobians
 * at the coarsened state when pr and p are given), then every level's
 * subdomains and their factors.  NULL when rediscretisation is asked for
 * without a problem or on sizes the ratio does not divide. */
static orc_mg *mg_build(int nx, int ny, int nz, int n, const int *rp, const int *ci, const double *v,
                        const orc_mg_desc *d, const orc_problem *pr, const double *p, double dt, int order) {
    orc_mg *mg = (orc_mg *)xcalloc(1, sizeof(orc_mg));
    mg->d = *d;
    mg->L = d->levels < 1 ? 1 : (d->levels > MAXLEV ? MAXLEV : d->levels);
    int ratio = d->ratio > 0 ? d->ratio : 2;
    int redisc = d->coarse_op == ORC_COARSE_REDISCRETISED && mg->L > 1;
    level *f = &mg->lev[0];
    f->nx = nx; f->ny = ny; f->nz = nz; f->n = n;
    f->A.n = f->A.m = n;
    int nnz = rp[n];
    f->A.rp = (int *)xcalloc(n + 1, sizeof(int));
    f->A.ci = (int *)xcalloc(nnz, sizeof(int));
    f->A.v = (double *)xcalloc(nnz, sizeof(double));
    memcpy(f->A.rp, rp, (n + 1) * sizeof(int));
    memcpy(f->A.ci, ci, nnz * sizeof(int));
    memcpy(f->A.v, v, nnz * sizeof(double));
    for (int l = 0; l + 1 < mg->L; ++l) {
        level *fl = &mg->lev[l], *cl = &mg->lev[l + 1];
        fl->P = interp_matrix(fl->nx, fl->ny, fl->nz, d->interp_order, ratio, &cl->nx, &cl->ny, &cl->nz);
        fl->has_p = 1;
        cl->n = cl->nx * cl->ny * cl->nz;
        if (redisc) {
            const orc_problem *fine = l == 0 ? pr : mg->cprob[l];
            mg->cprob[l + 1] = fine ? orc_problem_coarsen(fine, ratio) : NULL;
            if (!mg->cprob[l + 1]) { orc_mg_free(mg); return NULL; }
            continue;
        }
        /* Galerkin coarse operator A_c = P^T A P */
        csr AP = csr_matmul(&fl->A, &fl->P);
        csr Pt = csr_transpose(&fl->P);
        cl->A = csr_matmul(&Pt, &AP);
        csr_free(&AP); csr_free(&Pt);
    }
    if (redisc) {
        mg->odt = dt;
        mg->oorder = order;
        rediscretise(mg, pr, p);
    }
    /* the same box grid on every level: box counts from the finest level */
    int Pbox[3] = {d->px, d->py, d->pz};
    int t[3] = {d->tx, d->ty, d->tz}, nf[3] = {nx, ny, nz};
    for (int k = 0; k < 3; ++k)
        if (t[k] > 0) Pbox[k] = (nf[k] + t[k] - 1) / t[k];
    for (int l = 0; l < mg->L; ++l) {
        level *lv = &mg->lev[l];
        int delta = d->overlap[l < 8 ? l : 7];
        build_subdomains(lv, Pbox, delta);
        factor_subdomains(lv, d);
        for (int k = 0; k < 4; ++k) mg->work[l][k] = (double *)xcalloc(lv->n, sizeof(double));
    }
    return mg;
}

orc_mg *orc_mg_new(int nx, int ny, int nz, int n, const int *rp, const int *ci,
                   const double *v, const orc_mg_desc *d) {
    return mg_build(nx, ny, nz, n, rp, ci, v, d, NULL, NULL, 0.0, 1);
}

/* As orc_mg_new on the problem's grid, with the problem and the state p (and
 * dt, BDF order) that rediscretised coarse levels are evaluated from. */
orc_mg *orc_mg_new_problem(const orc_problem *pr, const double *p, double dt, int order, const int *rp,
                           const int *ci, const double *v, const orc_mg_desc *d) {
    return mg_build(pr->nx, pr->ny, pr->nz, pr->N, rp, ci, v, d, pr, p, dt, order);
}

void orc_mg_free(orc_mg *mg) {
    if (!mg) return;
    for (int l = 0; l < MAXLEV; ++l) orc_problem_free(mg->cprob[l]);
    for (int l = 0; l < mg->L; ++l) {
        level *lv = &mg->lev[l];
        csr_free(&lv->A);
        if (lv->has_p) csr_free(&lv->P);
        for (int s = 0; s < lv->nsub; ++s) {
            free(lv->sub[s].cells); free(lv->sub[s].owned);
            csr_free(&lv->sub[s].a);
            free(lv->sub[s].lu); free(lv->sub[s].piv);
        }
        free(lv->sub);
        for (int k = 0; k < 4; ++k) free(mg->work[l][k]);
    }
    free(mg);
}

void orc_mg_apply(orc_mg *mg, const double *r, double *z) {
    if (mg->L == 1) onelevel_apply(&mg->lev[0], &mg->d, r, z, 0);
    else mg_cycle(mg, 0, r, z, 0);
}

/* M^{-T} (used by the adjoint).  One level:
 * (sum R0^T A_i^{-1} Rd)^T = sum Rd^T A_i^{-T} R0, the right-RAS structure
 * on the transposed factors.  Several levels: the transposed composition of
 * mg_cycle, whose coarsest solve is GMRES on A_0^T with the transposed
 * one-level preconditioner (the exact transpose when that solve converges). */
void orc_mg_apply_transpose(orc_mg *mg, const double *r, double *z) {
    if (mg->L == 1) onelevel_apply(&mg->lev[0], &mg->d, r, z, 1);
    else mg_cycle(mg, 0, r, z, 1);
}

void orc_mg_apply_onelevel(orc_mg *mg, int lev, const double *r, double *z) {
    onelevel_apply(&mg->lev[lev], &mg->d, r, z, 0);
}

int orc_mg_level_info(const orc_mg *mg, int l, int *info) {
    if (l < 0 || l >= mg->L) return -1;
    const level *lv = &mg->lev[l];
    info[0] = lv->n; info[1] = lv->A.rp[lv->n];
    info[2] = lv->nx; info[3] = lv->ny; info[4] = lv->nz;
    info[5] = lv->nsub;
    info[6] = lv->has_p ? lv->P.m : 0;
    info[7] = lv->has_p ? lv->P.rp[lv->P.n] : 0;
    return mg->L;
}

void orc_mg_level_matrix(const orc_mg *mg, int l, int *rp, int *ci, double *v) {
    const level *lv = &mg->lev[l];
    memcpy(rp, lv->A.rp, (lv->n + 1) * sizeof(int));
    memcpy(ci, lv->A.ci, lv->A.rp[lv->n] * sizeof(int));
    memcpy(v, lv->A.v, lv->A.rp[lv->n] * sizeof(double));
}

void orc_mg_level_prolong(const orc_mg *mg, int l, int *rp, int *ci, double *v) {
    const level *lv = &mg->lev[l];
    memcpy(rp, lv->P.rp, (lv->P.n + 1) * sizeof(int));
    memcpy(ci, lv->P.ci, lv->P.rp[lv->P.n] * sizeof(int));
    memcpy(v, lv->P.v, lv->P.rp[lv->P.n] * sizeof(double));
}

int orc_mg_sub_info(const orc_mg *mg, int l, int s, int *info) {
    const subdomain *sd = &mg->lev[l].sub[s];
    info[0] = sd->next;
    info[1] = sd->a.rp ? sd->a.rp[sd->next] : 0;
    for (int k = 0; k < 3; ++k) {
        info[2 + k] = sd->lo[k]; info[5 + k] = sd->hi[k];
        info[8 + k] = sd->elo[k]; info[11 + k] = sd->ehi[k];
    }
    return mg->lev[l].nsub;
}

void orc_mg_sub_factors(const orc_mg *mg, int l, int s, int *cells, int *owned,
                        int *rp, int *ci, double *v) {
    const subdomain *sd = &mg->lev[l].sub[s];
    memcpy(cells, sd->cells, sd->next * sizeof(int));
    memcpy(owned, sd->owned, sd->next * sizeof(int));
    memcpy(rp, sd->a.rp, (sd->next + 1) * sizeof(int));
    memcpy(ci, sd->a.ci, sd->a.rp[sd->next] * sizeof(int));
    memcpy(v, sd->a.v, sd->a.rp[sd->next] * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* Krylov entry point                                                  */
/* ------------------------------------------------------------------ */
typedef struct { orc_mg *mg; int trans; } mg_ctx;

static void mg_op(void *ctx, const double *r, double *z) {
    mg_ctx *c = (mg_ctx *)ctx;
    if (c->trans) orc_mg_apply_transpose(c->mg, r, z);
    else orc_mg_apply(c->mg, r, z);
}

int orc_gmres(int n, const int *rp, const int *ci, const double *v, orc_mg *M, int transpose,
              const double *b, double *x, int restart, double rtol, double atol, int maxit,
              int flexible, double *res_out, int *its_out) {
    csr a;
    a.n = a.m = n;
    a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    csr_op aop = {&a, transpose};
    mg_ctx mc = {M, transpose};
    return gmres_core(n, csr_op_apply, &aop, M ? mg_op : NULL, &mc, b, x, restart, rtol, atol,
                      maxit, flexible, res_out, its_out);
}

/* ------------------------------------------------------------------ */
/* Inexact Newton with cubic backtracking (Section 3)                  */
/* ------------------------------------------------------------------ */
static double norm2(int n, const double *a) { return sqrt(dot(n, a, a)); }

static int nonphysical(const orc_problem *pr, const double *p) {
    for (int i = 0; i < pr->N; ++i) {
        double Z, dZ;
        if (!isfinite(p[i]) || orc_pr_z(pr->a, pr->b, pr->T, pr->R, p[i], &Z, &dZ)) return 1;
    }
    return 0;
}

/* X^{k+1} = X^k + lambda^k s^k with J_k s^k = -F(X^k) solved by Schwarz
 * preconditioned (F)GMRES to max{eta_r ||F||, eta_a}; lambda^k by a cubic
 * backtracking line search (Dennis-Schnabel) until
 * ||F(X^k + lambda s)|| <= (1 - alpha lambda) ||F(X^k)||; stop when
 * ||F(X^{k+1})|| <= max{eps_r ||F(X^0)||, eps_a}, or when the step is below
 * stol relative to the iterate (the relative step test of the PETSc solver
 * used in Section 4; without it FP64 rounding of the residual can put
 * eps_r ||F(X^0)|| below the attainable floor).  The step test is taken on the
 * full Newton step before the line search too: a full step that small is taken
 * as it is (lambda = 1, no decrease test, since at the rounding floor ||F||
 * cannot decrease) and Newton stops.
 *
 * Rounding floor (floor_test): the flux part of F is a stencil product in X
 * for frozen mobilities, so evaluating F in binary64 carries an error of
 * order u |J| |X| per cell (the componentwise bound of a matrix-vector
 * product; u = 2^-53).  When ||F(X^k)|| <= u || |J(X^k)| |X^k| || the iterate
 * solves F = 0 as well as F can be evaluated, and Newton stops there. */
int orc_newton_step(const orc_problem *pr, const orc_mg_desc *md, const orc_newton_desc *nd,
                    double *p, const double *pn, const double *pnm1, double dt, int order,
                    orc_newton_stats *st) {
    int N = pr->N;
    memset(st, 0, sizeof(*st));
    double *F = (double *)xcalloc(N, sizeof(double));
    double *Ft = (double *)xcalloc(N, sizeof(double));
    double *s = (double *)xcalloc(N, sizeof(double));
    double *b = (double *)xcalloc(N, sizeof(double));
    double *Js = (double *)xcalloc(N, sizeof(double));
    double *pt = (double *)xcalloc(N, sizeof(double));
    int *rp = (int *)xcalloc(N + 1, sizeof(int));
    int *ci = (int *)xcalloc((size_t)7 * N, sizeof(int));
    double *v = (double *)xcalloc((size_t)7 * N, sizeof(double));
    orc_residual(pr, p, pn, pnm1, dt, order, F);
    double f0 = norm2(N, F), fn = f0;
    st->fnorm0 = f0;
    double stop = nd->eps_r * f0 > nd->eps_a ? nd->eps_r * f0 : nd->eps_a;
    int status = 1;
    if (f0 <= stop) status = 0;
    orc_mg *M = NULL;
    for (int k = 0; k < nd->max_newton && status != 0; ++k) {
        orc_jacobian(pr, p, pn, pnm1, dt, order, rp, ci, v);
        if (nd->floor_test) {
            double fl = 0.0;
            for (int i = 0; i < N; ++i) {
                double a = 0.0;
                for (int q = rp[i]; q < rp[i + 1]; ++q) a += fabs(v[q]) * fabs(p[ci[q]]);
                fl += a * a;
            }
            if (fn <= ldexp(sqrt(fl), -53)) { status = 0; break; }
        }
        if (!M || nd->lag <= 1 || k % nd->lag == 0) {
            orc_mg_free(M);
            M = orc_mg_new_problem(pr, p, dt, order, rp, ci, v, md);
            if (!M) { status = 4; break; }
        } else {
            mg_refresh_operators(M, v, pr, p);
        }
        for (int i = 0; i < N; ++i) { b[i] = -F[i]; s[i] = 0.0; }
        double lres;
        int lits;
        double ltol_r = nd->eta_r, ltol_a = nd->eta_a;
        orc_gmres(N, rp, ci, v, M, 0, b, s, nd->restart, ltol_r, ltol_a, nd->maxit,
                  nd->flexible, &lres, &lits);
        st->linear_its += lits;
        if (k < 64) st->lits[k] = lits;
        const int small = nd->stol > 0.0 && norm2(N, s) <= nd->stol * norm2(N, p);
        /* line search on ||F||, merit f = ||F||^2 / 2 with slope F^T J s */
        orc_csr_matvec(N, rp, ci, v, s, Js);
        double fx = 0.5 * fn * fn, slope = dot(N, F, Js);
        double lam = 1.0, lam_prev = 0.0, f_prev = 0.0, ft_norm = 0.0;
        int ok = 0;
        for (int bt = 0; bt <= nd->max_backtracks; ++bt) {
            for (int i = 0; i < N; ++i) pt[i] = p[i] + lam * s[i];
            if (nonphysical(pr, pt)) {
                ft_norm = INFINITY;
            } else {
                orc_residual(pr, pt, pn, pnm1, dt, order, Ft);
                ft_norm = norm2(N, Ft);
            }
            if ((small && isfinite(ft_norm)) || ft_norm <= (1.0 - nd->alpha * lam) * fn) { ok = 1; break; }
            if (bt == nd->max_backtracks) break;
            double ft = 0.5 * ft_norm * ft_norm, lt;
            if (!isfinite(ft) || slope >= 0.0) {
                lt = 0.5 * lam;
            } else if (bt == 0) {
                lt = -slope / (2.0 * (ft - fx - slope));
            } else {
                double t1 = ft - fx - lam * slope, t2 = f_prev - fx - lam_prev * slope;
                double a = (t1 / (lam * lam) - t2 / (lam_prev * lam_prev)) / (lam - lam_prev);
                double bb = (-lam_prev * t1 / (lam * lam) + lam * t2 / (lam_prev * lam_prev)) / (lam - lam_prev);
                if (a == 0.0) lt = -slope / (2.0 * bb);
                else {
                    double disc = bb * bb - 3.0 * a * slope;
                    lt = disc >= 0.0 ? (-bb + sqrt(disc)) / (3.0 * a) : 0.5 * lam;
                }
            }
            if (!(lt <= 0.5 * lam)) lt = 0.5 * lam;
            if (!(lt >= 0.1 * lam)) lt = 0.1 * lam;
            lam_prev = lam; f_prev = ft;
            lam = lt;
        }
        if (!ok) { status = 2; break; }
        memcpy(p, pt, N * sizeof(double));
        memcpy(F, Ft, N * sizeof(double));
        fn = ft_norm;
        st->newton_its = k + 1;
        if (k < 64) { st->fnorms[k] = fn; st->lambdas[k] = lam; }
        if (fn <= stop || (small && lam == 1.0)) status = 0;
        /* relative step test of the PETSc nonlinear solver the paper ran on */
        if (nd->stol > 0.0 && lam * norm2(N, s) <= nd->stol * norm2(N, p)) status = 0;
    }
    st->fnorm = fn;
    st->status = status;
    orc_mg_free(M);
    free(F); free(Ft); free(s); free(b); free(Js); free(pt); free(rp); free(ci); free(v);
    return status;
}
