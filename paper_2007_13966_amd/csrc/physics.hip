// Peng-Robinson density, cell-centred residual and analytic Jacobian
// (Section 2: the PR density, Z cubic and criticality relations, the pressure
// form of the governing equation, the BDF1/BDF2 schemes; Remark 1 for the
// two-point flux).
//
// Every kernel is one thread per cell over the concatenated cells of all
// reservoirs; a cell finds its reservoir by binary search over the block
// offsets.  All arithmetic is FP64.
#include "nks_internal.h"

namespace nks {

// ---------------------------------------------------------------- PR cubic
// Largest real root of Z^3 + c2 Z^2 + c1 Z + c0 with
//   c2 = -(1-B), c1 = A - 3B^2 - 2B, c0 = -(AB - B^2 - B^3),
// A = a p/(RT)^2, B = b p/(RT).  Depressed cubic t^3 + P t + Q (Z = t - c2/3):
// one real root (discriminant > 0) by Cardano, otherwise the largest of the
// three trigonometric roots; two Newton steps on the cubic then remove the
// rounding of the closed form near a double root.  dZ/dp follows from
// implicit differentiation of the cubic (the closed form of Section 2).
struct PRState {
    double Z, dZ;
    bool bad;
};

__device__ __forceinline__ PRState pr_solve(double a, double b, double RT, double p) {
    const double A = a * p / (RT * RT);
    const double B = b * p / RT;
    const double c2 = B - 1.0;
    const double c1 = A - B * (3.0 * B + 2.0);
    const double c0 = B * (B + B * B - A);
    const double third = 1.0 / 3.0;
    const double sh = c2 * third;
    const double P = c1 - c2 * sh;
    const double Q = sh * (2.0 * sh * sh - c1) + c0;
    const double disc = 0.25 * Q * Q + P * P * P * (1.0 / 27.0);
    double z;
    if (disc > 0.0) {
        const double sq = sqrt(disc);
        z = cbrt(-0.5 * Q + sq) + cbrt(-0.5 * Q - sq) - sh;
    } else {
        const double r = sqrt(-P * third);
        double c = (r > 0.0) ? (-0.5 * Q) / (r * r * r) : 0.0;
        c = fmin(1.0, fmax(-1.0, c));
        z = 2.0 * r * cos(acos(c) * third) - sh;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double f = ((z + c2) * z + c1) * z + c0;
        const double df = (3.0 * z + 2.0 * c2) * z + c1;
        if (df != 0.0) z -= f / df;
    }
    // implicit derivative: dZ/dp = -(df/dp)/(df/dZ)
    const double dA = a / (RT * RT), dB = b / RT;
    const double dfdZ = (3.0 * z + 2.0 * c2) * z + c1;
    const double dfdp = dB * z * z + (dA - 6.0 * B * dB - 2.0 * dB) * z -
                        (dA * B + A * dB - 2.0 * B * dB - 3.0 * B * B * dB);
    PRState s;
    s.Z = z;
    s.dZ = -dfdp / dfdZ;
    s.bad = !(p > 0.0) || !(z > B) || !isfinite(z);
    return s;
}

// m = p/Z (density times RT/W) and dm/dp = 1/Z - p Z'/Z^2
__device__ __forceinline__ void scaled_density(double a, double b, double RT, double p,
                                               double &m, double &dm, bool &bad) {
    PRState s = pr_solve(a, b, RT, p);
    m = p / s.Z;
    dm = 1.0 / s.Z - p * s.dZ / (s.Z * s.Z);
    bad = s.bad;
}

struct CellPos {
    int b, x, y, z, nx, ny, nz;
};

__device__ __forceinline__ CellPos cell_pos_in(const Blk *blk, int b, int i) {
    CellPos c;
    c.b = b;
    const Blk k = blk[c.b];
    const int l = i - k.off;
    c.nx = k.nx; c.ny = k.ny; c.nz = k.nz;
    c.x = l % k.nx;
    c.y = (l / k.nx) % k.ny;
    c.z = l / (k.nx * k.ny);
    return c;
}

__device__ __forceinline__ CellPos cell_pos(const Blk *blk, int B, int i) {
    return cell_pos_in(blk, find_blk(blk, B, i), i);
}

// ---------------------------------------------------------------- setup kernels
__global__ void k_transmissibility(const Blk *blk, int B, int N, const double *geo,
                                   const double *kx, const double *ky, const double *kz,
                                   double *tx, double *ty, double *tz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const CellPos c = cell_pos(blk, B, i);
    const double dx = geo[3 * c.b], dy = geo[3 * c.b + 1], dz = geo[3 * c.b + 2];
    double t = 0.0;
    if (c.x + 1 < c.nx) t = dy * dz / (dx / (2.0 * kx[i]) + dx / (2.0 * kx[i + 1]));
    tx[i] = t;
    t = 0.0;
    if (c.y + 1 < c.ny) t = dx * dz / (dy / (2.0 * ky[i]) + dy / (2.0 * ky[i + c.nx]));
    ty[i] = t;
    t = 0.0;
    if (c.z + 1 < c.nz) t = dx * dy / (dz / (2.0 * kz[i]) + dz / (2.0 * kz[i + c.nx * c.ny]));
    tz[i] = t;
}

__global__ void k_pore_volume(const Blk *blk, int B, int N, const double *geo, const double *phi,
                              double *pv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int b = find_blk(blk, B, i);
    pv[i] = geo[3 * b] * geo[3 * b + 1] * geo[3 * b + 2] * phi[i];
}

// d2m/dp2 for m = p/Z, from the second derivative of the cubic along its
// root: with f(Z, p) = Z^3 + c2 Z^2 + c1 Z + c0 (A = a p/(RT)^2, B = b p/RT),
// Z' = -f_p/f_Z and Z'' = -(f_pp + 2 f_Zp Z' + f_ZZ Z'^2)/f_Z, then
// m'' = 2 p Z'^2/Z^3 - (2 Z' + p Z'')/Z^2.  Only the chain-rule
// accumulation's Jacobian needs it (its coefficient is m' itself).
__device__ __forceinline__ double density_curvature(double a, double b, double RT, double p) {
    const PRState s = pr_solve(a, b, RT, p);
    const double z = s.Z, z1 = s.dZ;
    const double al = a / (RT * RT), be = b / RT;
    const double B = be * p;
    const double fZ = (3.0 * z + 2.0 * (B - 1.0)) * z + (al * p - B * (3.0 * B + 2.0));
    const double fZZ = 6.0 * z + 2.0 * (B - 1.0);
    const double c1p = al - 2.0 * be - 6.0 * be * B;
    const double fZp = 2.0 * be * z + c1p;
    const double fpp = -6.0 * be * be * z - 2.0 * be * (al - be - 3.0 * be * B);
    const double z2 = -(fpp + 2.0 * fZp * z1 + fZZ * z1 * z1) / fZ;
    return 2.0 * p * z1 * z1 / (z * z * z) - (2.0 * z1 + p * z2) / (z * z);
}

// ---------------------------------------------------------------- PR per cell
// m, dm at p (and d2m when asked); flags[b] |= 1 on a non-physical state.
__global__ void k_props(const Blk *blk, int B, int N, double a, double b, double RT,
                        const double *p, double *m, double *dm, double *d2m, int *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double mi, dmi;
    bool bad;
    scaled_density(a, b, RT, p[i], mi, dmi, bad);
    m[i] = mi;
    dm[i] = dmi;
    if (d2m) d2m[i] = density_curvature(a, b, RT, p[i]);
    if (bad && flags) atomicOr(&flags[find_blk(blk, B, i)], 1);
}

// history part of the accumulation.  Conservative form: order 1: -m(p_n);
// order 2: (-4 m(p_n) + m(p_nm1))/2.  Chain-rule form (the printed BDF
// equations): the same combinations of p instead of m.
__global__ void k_history(int N, double a, double b, double RT, const double *pn,
                          const double *pnm1, int order, int chain, double *hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (chain) {
        hist[i] = order == 2 ? 0.5 * (pnm1[i] - 4.0 * pn[i]) : -pn[i];
        return;
    }
    double mn, d;
    bool bad;
    scaled_density(a, b, RT, pn[i], mn, d, bad);
    if (order == 2) {
        double mnm1;
        scaled_density(a, b, RT, pnm1[i], mnm1, d, bad);
        hist[i] = 0.5 * (mnm1 - 4.0 * mn);
    } else {
        hist[i] = -mn;
    }
}

// ---------------------------------------------------------------- residual + Jacobian
struct FluxArgs {
    const Blk *blk;
    const Chunk *tiles;                    // k_flux: a workgroup per tile (a run of cells of one block)
    int B, N, dim;
    const double *geo, *tx, *ty, *tz, *pv, *src;
    const double *p, *m, *dm, *hist;
    const double *d2m;                     // chain-rule accumulation: m'' per cell, else unused
    int chain;                             // 1: accumulation m'(p) D_t p (the printed BDF form)
    double cacc, inv_dt, inv_mu, crho_g;   // crho_g = g W/(RT)
    double *F;
    double *J;                             // K*N stencil coefficients or nullptr
    // outer-face boundary conditions: 6 per block (-x,+x,-y,+y,-z,+z), or nullptr
    const int *bct;
    const double *bcv;
    const double *kx, *ky, *kz;
    double a, b, RT;                       // PR constants for the Dirichlet face states
};

// Outer faces of cell i with a boundary condition.  Dirichlet: the face
// state p^D sits half a cell from the centre, one-sided transmissibility
// 2 K A / Delta, face density the mean of the cell's and the face state's,
// mobility from the upwind side; Neumann: scaled mass flux m_i q^N A through
// the face (q^N along the outward normal).  Adds the outward flux to Fi, its
// p_i derivative to diag and, for dF/dlnK, the part linear in K_i to dlk.
// Inlined: a call would take the argument block by reference, which puts a
// copy of it in every lane's private memory.
__device__ __forceinline__ void boundary_faces(const FluxArgs &A, const CellPos &c, int i, double pi, double mi,
                                            double dmi, double &Fi, double &diag, double &dlk) {
    const double dx = A.geo[3 * c.b], dy = A.geo[3 * c.b + 1], dz = A.geo[3 * c.b + 2];
    const bool at[6] = {c.x == 0, c.x + 1 == c.nx, c.y == 0, c.y + 1 == c.ny, c.z == 0, c.z + 1 == c.nz};
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int t = A.bct[6 * c.b + f];
        if (t == 0 || !at[f]) continue;
        const int ax = f >> 1;
        const double area = ax == 0 ? dy * dz : (ax == 1 ? dx * dz : dx * dy);
        const double v = A.bcv[6 * c.b + f];
        if (t == 2) {
            Fi += mi * v * area;
            diag += dmi * v * area;
            continue;
        }
        const double len = ax == 0 ? dx : (ax == 1 ? dy : dz);
        const double K = ax == 0 ? A.kx[i] : (ax == 1 ? A.ky[i] : A.kz[i]);
        const double T = 2.0 * K * area / len;
        const double dh = f == 4 ? 0.5 * dz : (f == 5 ? -0.5 * dz : 0.0);   // h_i - h_face
        double md, dmd;
        bool bad;
        scaled_density(A.a, A.b, A.RT, v, md, dmd, bad);
        const double dphi = (pi - v) - 0.5 * (mi + md) * A.crho_g * dh;
        const bool up = dphi >= 0.0;
        const double lam = (up ? mi : md) * A.inv_mu;
        Fi += T * lam * dphi;
        diag += T * ((up ? dmi * A.inv_mu : 0.0) * dphi + lam * (1.0 - 0.5 * dmi * A.crho_g * dh));
        dlk += T * lam * dphi;
    }
}

__device__ __forceinline__ bool on_boundary(const CellPos &c) {
    return c.x == 0 || c.x + 1 == c.nx || c.y == 0 || c.y + 1 == c.ny || c.z == 0 || c.z + 1 == c.nz;
}

// One face of cell i: neighbour j, transmissibility T, depth difference
// h_i - h_j.  Accumulates the flux into Fi and, for the Jacobian, the
// diagonal and the off-diagonal coefficient.
__device__ __forceinline__ void face(const FluxArgs &A, double pi, double mi, double dmi, int j,
                                     double T, double dh, double &Fi, double &diag, double &off) {
    const double pj = A.p[j], mj = A.m[j];
    const double dphi = (pi - pj) - 0.5 * (mi + mj) * A.crho_g * dh;
    const bool up = dphi >= 0.0;
    const double lam = (up ? mi : mj) * A.inv_mu;
    Fi += T * lam * dphi;
    if (A.J) {
        const double dmj = A.dm[j];
        const double dli = up ? dmi * A.inv_mu : 0.0;
        const double dlj = up ? 0.0 : dmj * A.inv_mu;
        diag += T * (dli * dphi + lam * (1.0 - 0.5 * dmi * A.crho_g * dh));
        off = T * (dlj * dphi + lam * (-1.0 - 0.5 * dmj * A.crho_g * dh));
    }
}

__global__ void k_flux(FluxArgs A) {
    const Chunk ch = A.tiles[blockIdx.x];
    const int i = ch.start + (int)threadIdx.x;
    if (i >= ch.end) return;
    const CellPos c = cell_pos_in(A.blk, ch.blk, i);
    const int sx = 1, sy = c.nx, sz = c.nx * c.ny;
    const double dz = A.geo[3 * c.b + 2];
    const double pi = A.p[i], mi = A.m[i], dmi = A.dm[i];
    double Fi, diag;
    if (A.chain) {
        // [phi m'(p)]^{l+1} times the BDF difference of p; its p derivative
        // adds m''(p) times that difference
        const double dtp = A.cacc * pi + A.hist[i];
        Fi = A.pv[i] * A.inv_dt * dmi * dtp;
        diag = A.J ? A.pv[i] * A.inv_dt * (A.d2m[i] * dtp + A.cacc * dmi) : 0.0;
    } else {
        Fi = A.pv[i] * A.inv_dt * (A.cacc * mi + A.hist[i]);
        diag = A.pv[i] * A.inv_dt * A.cacc * dmi;
    }
    double o[6] = {0, 0, 0, 0, 0, 0};
    // neighbour order -z, -y, -x, +x, +y, +z (increasing cell index)
    if (A.dim == 3 && c.z > 0) face(A, pi, mi, dmi, i - sz, A.tz[i - sz], dz, Fi, diag, o[0]);
    if (c.y > 0) face(A, pi, mi, dmi, i - sy, A.ty[i - sy], 0.0, Fi, diag, o[1]);
    if (c.x > 0) face(A, pi, mi, dmi, i - sx, A.tx[i - sx], 0.0, Fi, diag, o[2]);
    if (c.x + 1 < c.nx) face(A, pi, mi, dmi, i + sx, A.tx[i], 0.0, Fi, diag, o[3]);
    if (c.y + 1 < c.ny) face(A, pi, mi, dmi, i + sy, A.ty[i], 0.0, Fi, diag, o[4]);
    if (A.dim == 3 && c.z + 1 < c.nz) face(A, pi, mi, dmi, i + sz, A.tz[i], -dz, Fi, diag, o[5]);
    if (A.bct && on_boundary(c)) {
        double dlk = 0.0;
        boundary_faces(A, c, i, pi, mi, dmi, Fi, diag, dlk);
    }
    if (A.F) A.F[i] = Fi - A.src[i];
    if (A.J) {
        const int N = A.N;
        if (A.dim == 3) {
            A.J[0 * N + i] = o[0];
            A.J[1 * N + i] = o[1];
            A.J[2 * N + i] = o[2];
            A.J[3 * N + i] = diag;
            A.J[4 * N + i] = o[3];
            A.J[5 * N + i] = o[4];
            A.J[6 * N + i] = o[5];
        } else {
            A.J[0 * N + i] = o[1];
            A.J[1 * N + i] = o[2];
            A.J[2 * N + i] = diag;
            A.J[3 * N + i] = o[3];
            A.J[4 * N + i] = o[4];
        }
    }
}

// ---------------------------------------------------------------- hydrostatic init
// one thread per (reservoir, column); scalar Newton down the column
__global__ void k_hydrostatic(const Blk *blk, int B, int ncol_total, const int *colstart,
                              const double *geo, double a, double b, double RT, double crho_g,
                              double p_top, double *p) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncol_total) return;
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (colstart[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const Blk k = blk[lo];
    const int col = t - colstart[lo];
    const int nxy = k.nx * k.ny;
    const double dz = geo[3 * lo + 2];
    double pk = p_top;
    p[k.off + col] = pk;
    for (int z = 1; z < k.nz; ++z) {
        double mk, dmk;
        bool bad;
        scaled_density(a, b, RT, pk, mk, dmk, bad);
        double q = pk;
        for (int it = 0; it < 50; ++it) {
            double mq, dmq;
            scaled_density(a, b, RT, q, mq, dmq, bad);
            const double f = q - pk - 0.5 * (mk + mq) * crho_g * dz;
            const double df = 1.0 - 0.5 * dmq * crho_g * dz;
            const double step = f / df;
            q -= step;
            if (fabs(step) <= 1e-15 * fabs(q)) break;
        }
        pk = q;
        p[k.off + col + z * nxy] = pk;
    }
}

// ---------------------------------------------------------------- dF/dlnK transpose
// out_c = sum over faces (c,n): (lam_c - lam_n) * lambda_up dPhi_cn * T K_n/(K_c + K_n),
// K the component normal to the face (dT/dln K_c = T K_n/(K_c + K_n)); ln K_c
// scales all three components of cell c together; a Dirichlet boundary face of
// c adds lam_c times its flux (its one-sided T is linear in K_c).
// accumulate: out += instead of =.
__global__ void k_dlogk_t(FluxArgs A, const double *kx, const double *ky, const double *kz,
                          const double *lam, double *out, int accumulate) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.N) return;
    const CellPos c = cell_pos(A.blk, A.B, i);
    const int sy = c.nx, sz = c.nx * c.ny;
    const double dz = A.geo[3 * c.b + 2];
    const double pi = A.p[i], mi = A.m[i], li = lam[i];
    double acc = 0.0;
    auto term = [&](int j, double T, double dh, double ki, double kj) {
        const double pj = A.p[j], mj = A.m[j];
        const double dphi = (pi - pj) - 0.5 * (mi + mj) * A.crho_g * dh;
        const double lm = (dphi >= 0.0 ? mi : mj) * A.inv_mu;
        acc += (li - lam[j]) * lm * dphi * T * kj / (ki + kj);
    };
    if (A.dim == 3 && c.z > 0) term(i - sz, A.tz[i - sz], dz, kz[i], kz[i - sz]);
    if (c.y > 0) term(i - sy, A.ty[i - sy], 0.0, ky[i], ky[i - sy]);
    if (c.x > 0) term(i - 1, A.tx[i - 1], 0.0, kx[i], kx[i - 1]);
    if (c.x + 1 < c.nx) term(i + 1, A.tx[i], 0.0, kx[i], kx[i + 1]);
    if (c.y + 1 < c.ny) term(i + sy, A.ty[i], 0.0, ky[i], ky[i + sy]);
    if (A.dim == 3 && c.z + 1 < c.nz) term(i + sz, A.tz[i], -dz, kz[i], kz[i + sz]);
    if (A.bct && on_boundary(c)) {
        // a Dirichlet face's transmissibility is linear in K_i
        double Fb = 0.0, db = 0.0, dlk = 0.0;
        boundary_faces(A, c, i, pi, mi, A.dm[i], Fb, db, dlk);
        acc += li * dlk;
    }
    out[i] = accumulate ? out[i] + acc : acc;
}

// ---------------------------------------------------------------- adjoint right-hand side
// Step n of the discrete adjoint: out = -dG/dp^n - (V phi/dt) m'(p^n) (c1 lam1 + c2 lam2),
// where c1 (c2) is the coefficient of m(p^n) in the accumulation of step n+1
// (n+2): -1 or -2 (BDF1 or BDF2) and 1/2 (BDF2); absent terms have null vectors.
__global__ void k_adj_rhs(int N, double a, double b, double RT, const double *pn, const double *pv,
                          double inv_dt, double c1, const double *l1, double c2, const double *l2,
                          const double *dg, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double m, dm;
    bool bad;
    scaled_density(a, b, RT, pn[i], m, dm, bad);
    double c = 0.0;
    if (l1) c += c1 * l1[i];
    if (l2) c += c2 * l2[i];
    out[i] = -(dg ? dg[i] : 0.0) - pv[i] * inv_dt * dm * c;
}

// ---------------------------------------------------------------- host side
static inline int nblk(int n, int t) { return (n + t - 1) / t; }

void grid_setup_kernels(Grid &g, const double *kx, const double *ky, const double *kz,
                        const double *phi) {
    const int N = g.sp.N, B = g.sp.B;
    k_transmissibility<<<nblk(N, 256), 256, 0, g.s>>>(g.sp.blk.p, B, N, g.geo.p, kx, ky, kz,
                                                      g.tx.p, g.ty.p, g.tz.p);
    KCHECK();
    k_pore_volume<<<nblk(N, 256), 256, 0, g.s>>>(g.sp.blk.p, B, N, g.geo.p, phi, g.pv.p);
    KCHECK();
}

static FluxArgs flux_args(Grid &g, const double *p, double dt, int order, double *F, double *J) {
    FluxArgs A;
    A.blk = g.sp.blk.p;
    A.tiles = g.sp.tile.p;
    A.B = g.sp.B;
    A.N = g.sp.N;
    A.dim = g.dim;
    A.geo = g.geo.p;
    A.tx = g.tx.p; A.ty = g.ty.p; A.tz = g.tz.p;
    A.pv = g.pv.p;
    A.src = g.src.p;
    A.p = p;
    A.m = g.m.p;
    A.dm = g.dm.p;
    A.hist = g.hist.p;
    A.d2m = g.d2m.p;
    A.chain = g.accum == NKS_ACCUM_CHAIN_RULE ? 1 : 0;
    A.cacc = order == 2 ? 1.5 : 1.0;
    A.inv_dt = 1.0 / dt;
    A.inv_mu = 1.0 / g.mu;
    A.crho_g = g.g * g.W / g.RT;
    A.F = F;
    A.J = J;
    A.bct = g.bct.p;
    A.bcv = g.bcv.p;
    A.kx = g.kx.p; A.ky = g.ky.p; A.kz = g.kz.p;
    A.a = g.a; A.b = g.b; A.RT = g.RT;
    return A;
}

void launch_history(Grid &g, const double *pn, const double *pnm1, int order) {
    const int N = g.sp.N;
    k_history<<<nblk(N, 256), 256, 0, g.s>>>(N, g.a, g.b, g.RT, pn, order == 2 ? pnm1 : pn,
                                             order, g.accum == NKS_ACCUM_CHAIN_RULE ? 1 : 0, g.hist.p);
    KCHECK();
}

void launch_props(Grid &g, const double *p) {
    const int N = g.sp.N;
    k_props<<<nblk(N, 256), 256, 0, g.s>>>(g.sp.blk.p, g.sp.B, N, g.a, g.b, g.RT, p, g.m.p,
                                           g.dm.p, g.accum == NKS_ACCUM_CHAIN_RULE ? g.d2m.p : nullptr,
                                           g.flags.p);
    KCHECK();
}

// F (and J) at p, with the history term already in g.hist and props at p in g.m/g.dm
void launch_flux(Grid &g, const double *p, double dt, int order, double *F, double *J) {
    FluxArgs A = flux_args(g, p, dt, order, F, J);
    k_flux<<<(int)g.sp.htile.size(), TILE, 0, g.s>>>(A);
    KCHECK();
}

// The residual with caller-provided intermediates: the history term into
// hist, the PR properties at p into m / dm and the non-physical flags into
// flags (B ints), then F from those (the grid's own buffers are not touched).
void launch_residual_into(Grid &g, const double *p, const double *pn, const double *pnm1, double dt,
                          int order, double *F, double *hist, double *m, double *dm, int *flags) {
    const int N = g.sp.N;
    k_history<<<nblk(N, 256), 256, 0, g.s>>>(N, g.a, g.b, g.RT, pn, order == 2 ? pnm1 : pn, order,
                                             g.accum == NKS_ACCUM_CHAIN_RULE ? 1 : 0, hist);
    KCHECK();
    k_props<<<nblk(N, 256), 256, 0, g.s>>>(g.sp.blk.p, g.sp.B, N, g.a, g.b, g.RT, p, m, dm, nullptr, flags);
    KCHECK();
    FluxArgs A = flux_args(g, p, dt, order, F, nullptr);
    A.m = m;
    A.dm = dm;
    A.hist = hist;
    k_flux<<<(int)g.sp.htile.size(), TILE, 0, g.s>>>(A);
    KCHECK();
}

// ---------------------------------------------------------------- rediscretised coarse grids
// coarse cell I of a block whose fine sizes are r times its own (1 where a
// size is 1): permeabilities averaged over the children, pore volumes summed
__global__ void k_upscale(const Blk *fblk, const Blk *cblk, int B, int Nc, const double *kx, const double *ky,
                          const double *kz, const double *pv, double *ckx, double *cky, double *ckz, double *cpv) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= Nc) return;
    const int b = find_blk(cblk, B, I);
    const Blk cb = cblk[b], fb = fblk[b];
    const int l = I - cb.off;
    const int X = l % cb.nx, Y = (l / cb.nx) % cb.ny, Z = l / (cb.nx * cb.ny);
    const int rx = fb.nx / cb.nx, ry = fb.ny / cb.ny, rz = fb.nz / cb.nz;
    double sx = 0.0, sy = 0.0, sz = 0.0, sv = 0.0;
    for (int z = Z * rz; z < (Z + 1) * rz; ++z)
        for (int y = Y * ry; y < (Y + 1) * ry; ++y)
            for (int x = X * rx; x < (X + 1) * rx; ++x) {
                const int i = fb.off + x + fb.nx * (y + fb.ny * z);
                sx += kx[i];
                sy += ky[i];
                sz += kz[i];
                sv += pv[i];
            }
    const double inv = 1.0 / (rx * ry * rz);
    ckx[I] = sx * inv;
    cky[I] = sy * inv;
    ckz[I] = sz * inv;
    cpv[I] = sv;
}

__global__ void k_coarsen_mean(const Blk *fblk, const Blk *cblk, int B, int Nc, const double *pf, double *pc) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= Nc) return;
    const int b = find_blk(cblk, B, I);
    const Blk cb = cblk[b], fb = fblk[b];
    const int l = I - cb.off;
    const int X = l % cb.nx, Y = (l / cb.nx) % cb.ny, Z = l / (cb.nx * cb.ny);
    const int rx = fb.nx / cb.nx, ry = fb.ny / cb.ny, rz = fb.nz / cb.nz;
    double s = 0.0;
    for (int z = Z * rz; z < (Z + 1) * rz; ++z)
        for (int y = Y * ry; y < (Y + 1) * ry; ++y)
            for (int x = X * rx; x < (X + 1) * rx; ++x) s += pf[fb.off + x + fb.nx * (y + fb.ny * z)];
    pc[I] = s / (rx * ry * rz);
}

void coarsen_grid(const Grid &f, int ratio, Grid &c) {
    std::vector<Blk> cb;
    std::vector<double> geo(3 * (size_t)f.sp.B);
    std::vector<double> fgeo(3 * (size_t)f.sp.B);
    HIPC(hipMemcpyAsync(fgeo.data(), f.geo.p, fgeo.size() * 8, hipMemcpyDeviceToHost, f.s));
    HIPC(hipStreamSynchronize(f.s));
    for (int b = 0; b < f.sp.B; ++b) {
        const Blk &k = f.sp.hblk[b];
        const int n[3] = {k.nx, k.ny, k.nz};
        int m[3];
        for (int a = 0; a < 3; ++a) {
            const int r = n[a] > 1 ? ratio : 1;
            if (n[a] % r) fail(NKS_EINVAL, "rediscretised coarse level: reservoir %d size %d is not a multiple of %d",
                               b, n[a], r);
            m[a] = n[a] / r;
            geo[3 * b + a] = fgeo[3 * b + a] * r;
        }
        cb.push_back({m[0], m[1], m[2], 0});
    }
    c.al = f.al;
    c.s = f.s;
    c.dim = f.dim;
    c.sp.build(&c.al, cb, c.s);
    const int N = c.sp.N;
    c.geo.upload(&c.al, geo, c.s);
    c.kx.alloc(&c.al, N); c.ky.alloc(&c.al, N); c.kz.alloc(&c.al, N);
    c.pv.alloc(&c.al, N);
    c.tx.alloc(&c.al, N); c.ty.alloc(&c.al, N); c.tz.alloc(&c.al, N);
    k_upscale<<<nblk(N, 256), 256, 0, c.s>>>(f.sp.blk.p, c.sp.blk.p, c.sp.B, N, f.kx.p, f.ky.p, f.kz.p, f.pv.p,
                                             c.kx.p, c.ky.p, c.kz.p, c.pv.p);
    KCHECK();
    k_transmissibility<<<nblk(N, 256), 256, 0, c.s>>>(c.sp.blk.p, c.sp.B, N, c.geo.p, c.kx.p, c.ky.p, c.kz.p,
                                                      c.tx.p, c.ty.p, c.tz.p);
    KCHECK();
    c.src.alloc(&c.al, N);
    HIPC(hipMemsetAsync(c.src.p, 0, sizeof(double) * N, c.s));
    if (f.bct.p) {
        std::vector<int> bct(f.bct.n);
        std::vector<double> bcv(f.bcv.n);
        HIPC(hipMemcpyAsync(bct.data(), f.bct.p, bct.size() * 4, hipMemcpyDeviceToHost, f.s));
        HIPC(hipMemcpyAsync(bcv.data(), f.bcv.p, bcv.size() * 8, hipMemcpyDeviceToHost, f.s));
        HIPC(hipStreamSynchronize(f.s));
        c.bct.upload(&c.al, bct, c.s);
        c.bcv.upload(&c.al, bcv, c.s);
    }
    c.a = f.a; c.b = f.b; c.RT = f.RT; c.W = f.W; c.mu = f.mu; c.g = f.g;
    c.accum = NKS_ACCUM_CONSERVATIVE;
    c.m.alloc(&c.al, N);
    c.dm.alloc(&c.al, N);
    c.hist.alloc(&c.al, N);
    c.tmp.alloc(&c.al, N);
    c.flags.alloc(&c.al, c.sp.B);
    HIPC(hipMemsetAsync(c.flags.p, 0, sizeof(int) * c.sp.B, c.s));
}

void launch_coarsen_mean(const Grid &f, const Grid &c, const double *pf, double *pc) {
    const int N = c.sp.N;
    k_coarsen_mean<<<nblk(N, 256), 256, 0, c.s>>>(f.sp.blk.p, c.sp.blk.p, c.sp.B, N, pf, pc);
    KCHECK();
}

void remember_state(Matrix &J, const double *p, double dt, int order) {
    Grid &g = *J.g;
    J.state.alloc(&g.al, g.sp.N);
    HIPC(hipMemcpyAsync(J.state.p, p, sizeof(double) * g.sp.N, hipMemcpyDeviceToDevice, g.s));
    J.dt = dt;
    J.order = order;
    J.has_state = true;
}

void launch_hydrostatic(Grid &g, double p_top, double *p) {
    std::vector<int> cs(g.sp.B);
    int tot = 0;
    for (int b = 0; b < g.sp.B; ++b) {
        cs[b] = tot;
        tot += g.sp.hblk[b].nx * g.sp.hblk[b].ny;
    }
    DBuf<int> d;
    d.upload(&g.al, cs, g.s);
    k_hydrostatic<<<nblk(tot, 128), 128, 0, g.s>>>(g.sp.blk.p, g.sp.B, tot, d.p, g.geo.p, g.a,
                                                   g.b, g.RT, g.g * g.W / g.RT, p_top, p);
    KCHECK();
    HIPC(hipStreamSynchronize(g.s));
}

void launch_dlogk_t(Grid &g, const double *p, const double *lam, double *out, bool accumulate) {
    launch_props(g, p);
    FluxArgs A = flux_args(g, p, 1.0, 1, nullptr, nullptr);
    k_dlogk_t<<<nblk(A.N, 256), 256, 0, g.s>>>(A, g.kx.p, g.ky.p, g.kz.p, lam, out, accumulate ? 1 : 0);
    KCHECK();
}

void launch_adj_rhs(Grid &g, const double *pn, double dt, double c1, const double *l1, double c2,
                    const double *l2, const double *dg, double *out) {
    const int N = g.sp.N;
    k_adj_rhs<<<nblk(N, 256), 256, 0, g.s>>>(N, g.a, g.b, g.RT, pn, g.pv.p, 1.0 / dt, c1, l1, c2, l2, dg, out);
    KCHECK();
}

}  // namespace nks
