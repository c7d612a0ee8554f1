"""Workload records: grid, rock, fluid, wells, time stepping and solver settings.

Units are SI throughout.  Permeabilities are stored in m^2 (1 mD =
9.869233e-16 m^2), rates in kg/s (positive = injection), times in seconds.

The five workloads:
  case_2d_32          2D 32x32, homogeneous 100 mD, one-level left-RAS 4x4 subdomains, overlap 1
  case_2d_512         2D 512x512 log-normal (sigma 1, corr. length 8), five-spot, two-level V-cycle
  case_3d_128         3D 128x128x64 layered log-normal (sigma 1.5), gravity, three-level, mixed precision
  case_batch64        64 independent 2D reservoirs, sides 64..256, FP32 preconditioner
  case_3d_96_adjoint  3D 96x96x48 channelised (1000 mD channels in 10 mD), gravity, adjoint gradient
"""
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

from .fields import lognormal_perm, layered_perm, channel_perm, hzone_mask

MD = 9.869233e-16     # m^2 per millidarcy
DAY = 86400.0         # s
ATM = 101325.0        # Pa


@dataclass
class Fluid:
    """Single-component gas: critical point, acentric factor, temperature,
    molar mass, gas constant and constant viscosity (Pa s)."""
    Tc: float = 190.6
    pc: float = 4.599e6
    omega: float = 0.011
    T: float = 350.0
    W: float = 0.016
    R: float = 8.3147295
    mu: float = 11.067e-3 * 1e-3   # 11.067e-3 cP
    Tb: Optional[float] = None     # normal boiling point (K): omega is computed from it


@dataclass
class Problem:
    """One reservoir on an nx*ny*nz cell-centred grid, x fastest in every array."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    kx: np.ndarray          # (N,) m^2
    ky: np.ndarray
    kz: np.ndarray
    phi: np.ndarray         # (N,)
    well_cells: np.ndarray  # (nw,) int32 linear cell index
    well_rates: np.ndarray  # (nw,) float64 kg/s
    fluid: Fluid = field(default_factory=Fluid)
    gravity: bool = False
    g: float = 9.80665
    p_init: float = 20e6    # uniform, or top-layer pressure when gravity is on
    # outer faces -x, +x, -y, +y, -z, +z: 0 closed, 1 Dirichlet (value p^D, Pa),
    # 2 Neumann (value q^N = v.n, m/s, n the outward normal: inflow < 0)
    bc_type: Tuple[int, ...] = (0, 0, 0, 0, 0, 0)
    bc_value: Tuple[float, ...] = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    # accumulation form: "conservative" (phi V (m(p) - m(p^n))/dt) or "chain_rule"
    # (phi V m'(p) (p - p^n)/dt, the BDF equations as printed); every
    # reservoir of one GPU grid shares the first reservoir's form
    accum: str = "conservative"

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    @property
    def dims(self):
        return 3 if self.nz > 1 else 2


@dataclass
class SolverSettings:
    """Newton / (F)GMRES / multilevel Schwarz settings.  Defaults are the
    stopping values of the paper's experiments (Section 4.2)."""
    px: int = 4
    py: int = 4
    pz: int = 1
    overlap: Tuple[int, ...] = (1,)      # finest level first
    tile: Tuple[int, int, int] = (0, 0, 0)   # > 0: box edge in cells (boxes per reservoir = ceil(n/t))
    levels: int = 1
    interp_order: int = 2                # 1 nearest, 2 bilinear, 3 bicubic
    cycle: str = "vcycle"                # vcycle | left_kaskade | right_kaskade | additive | coarse_only
    variant: str = "left_ras"            # left_ras | as | right_ras
    subsolve: str = "ilu0"               # ilu0 | lu (oracle only)
    fill: int = 0                        # subdomain ILU level of fill k: ILU(k) (0: ILU(0))
    ratio: int = 2                       # coarse-to-fine mesh ratio per direction between levels
    coarse_op: str = "galerkin"          # galerkin (P^T A P) | rediscretised (upscaled coarse problem)
    coarse_kernel: str = "auto"          # coarsest GMRES: auto | chunked (captured launches) | persistent
    mu: int = 1
    nu: int = 1
    coarse_rtol: float = 0.2
    coarse_maxit: int = 200
    coarse_restart: int = 30
    restart: int = 30
    eta_r: float = 1e-5
    eta_a: float = 1e-8
    maxit: int = 10000
    eps_r: float = 1e-6
    eps_a: float = 1e-10
    alpha: float = 1e-4
    max_newton: int = 50
    max_backtracks: int = 20
    stol: float = 0.0                    # relative Newton step test (PETSc's; 0 = off)
    floor_test: bool = True              # stop at the FP64 rounding floor u || |J| |X| ||
    lag: int = 1                         # refactor the preconditioner every lag Newton iterations
    precision: str = "fp64"              # fp64 | fp32 | bf16
    flexible: Optional[bool] = None      # None: FGMRES iff levels > 1 or precision != fp64


@dataclass
class Case:
    name: str
    problems: List[Problem]
    dt: float
    nsteps: int
    solver: SolverSettings
    description: str = ""


def _wells(cells, rates):
    return np.asarray(cells, dtype=np.int32), np.asarray(rates, dtype=np.float64)


def _lin(nx, ny, x, y, z=0):
    return x + nx * (y + ny * z)


def small_case(nx=8, ny=8, nz=1, seed=0, sigma=1.0, corr=3.0, gravity=False,
               rate=1e-3, px=2, py=2, pz=1, overlap=(1,), levels=1, dt=DAY,
               nsteps=2, kv_ratio=1.0, p_init=20e6, kmean_md=100.0, bc=(), **solver_kw):
    """Small seeded problem for tests: log-normal K around kmean_md, porosity in
    [0.1, 0.3], injector at the first cell and producer at the last (rate 0: no
    wells).  bc: (face, type, value) triples for the outer faces."""
    shape = (nz, ny, nx)
    kh = lognormal_perm(shape, kmean_md * MD, sigma, corr, seed).ravel()
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    phi = rng.uniform(0.1, 0.3, size=nx * ny * nz)
    N = nx * ny * nz
    wc, wr = _wells([0, N - 1], [rate, -rate]) if rate else _wells([], [])
    bt, bv = [0] * 6, [0.0] * 6
    for f, t, v in bc:
        bt[f], bv[f] = t, v
    prob = Problem(nx, ny, nz, 10.0, 10.0, 10.0, kh.copy(), kh.copy(), kv_ratio * kh,
                   phi, wc, wr, gravity=gravity, p_init=p_init, bc_type=tuple(bt), bc_value=tuple(bv))
    s = SolverSettings(px=px, py=py, pz=pz, overlap=tuple(overlap), levels=levels, **solver_kw)
    return Case("small", [prob], dt, nsteps, s)


def case_2d_flood(nx=64, ny=64, px=4, py=4, seed=4):
    """Pressure-driven flood between two Dirichlet faces, the boundary regime
    of the paper's first 2D test: gas at 1 atm and 298 K, p^D = 10 atm on the
    -y face and 1 atm on the +y face, the x faces closed, no wells, no
    gravity; log-normal K (100 mD, sigma 1); steps of 0.06 day.  The first
    steps are strongly nonlinear (a tenfold pressure rise sweeps the domain)."""
    case = small_case(nx=nx, ny=ny, nz=1, seed=seed, rate=0.0, px=px, py=py, overlap=(1,),
                      dt=0.06 * DAY, nsteps=4, p_init=ATM,
                      bc=((2, 1, 10 * ATM), (3, 1, ATM)))
    prob = case.problems[0]
    # the paper's methane constants (Section 4), omega from the boiling point
    prob.fluid = replace(prob.fluid, T=298.0, Tc=190.58, pc=4.604e6, Tb=111.67)
    return replace(case, name=f"2d_{nx}x{ny}_flood_dirichlet", description=case_2d_flood.__doc__)


def case_2d_flood_512():
    """The Dirichlet flood at 512x512 with the 512x512 workload's solver: 16x16
    subdomains, overlap 2 on both levels of a two-level V-cycle, FGMRES(30),
    FP64; 10 steps of 0.06 day."""
    case = case_2d_flood(512, 512, 16, 16)
    case = with_solver(case, levels=2, overlap=(2, 2))
    return replace(case, nsteps=10, description=case_2d_flood_512.__doc__)


# permeabilities of the H-zone stand-ins: a jump of two orders of magnitude
HZONE_IN_MD = 500.0
HZONE_OUT_MD = 5.0


def case_2d_hzone(n=512, anisotropic=False, px=16, py=16, nsteps=100):
    """Stand-in for the paper's first 2D test (its H-zone field is shown only as
    a figure): the (0, 100 m)^2 square on n x n cells, an H-shaped zone of
    500 mD in a 5 mD background (isotropic), or with k_yy = k_xx/10 inside the
    zone (anisotropic: the two domains differ in isotropy); gas at 1 atm and
    298 K with the paper's methane constants; p^D = 10 atm on the -y face and
    1 atm on the +y face, x faces closed, no wells, no gravity; phi 0.2;
    steps of 0.1 day (100 steps to 10 days); two-level V-cycle, 16x16
    subdomains, overlap 2 on both levels, FP64."""
    mask = hzone_mask(n, n).ravel()
    kx = np.where(mask, HZONE_IN_MD, HZONE_OUT_MD) * MD
    ky = kx * np.where(mask, 0.1, 1.0) if anisotropic else kx.copy()
    h = 100.0 / n
    prob = Problem(n, n, 1, h, h, h, kx, ky, kx.copy(), np.full(n * n, 0.2), *_wells([], []),
                   p_init=ATM, bc_type=(0, 0, 1, 1, 0, 0), bc_value=(0.0, 0.0, 10 * ATM, ATM, 0.0, 0.0))
    prob.fluid = replace(prob.fluid, T=298.0, Tc=190.58, pc=4.604e6, Tb=111.67)
    s = SolverSettings(px=px, py=py, pz=1, overlap=(2, 2), levels=2)
    kind = "aniso" if anisotropic else "iso"
    return Case(f"2d_{n}x{n}_hzone_{kind}", [prob], 0.1 * DAY, nsteps, s, case_2d_hzone.__doc__)


def case_3d_layered_flood(n=128, px=8, py=8, pz=8, nsteps=5):
    """Stand-in for the paper's 3D layered test: the (0, 100 m)^3 cube on n^3
    cells whose layers with z in [25, 75] m carry the H-zone field of the 2D
    stand-in (isotropic, 500 mD in 5 mD) and the others the 5 mD background;
    gas at 1 atm and 298 K (paper's methane constants), gravity on with the
    hydrostatic state from 1 atm at the top; p^D = 10 atm on the +y face (the
    behind face) and 1 atm on the -y face (the front), the other faces
    closed, no wells; phi 0.2; steps of 0.1 day; three-level V-cycle with
    first-order interpolation, 8x8x8 subdomains, overlap 1, FP64."""
    mask2 = hzone_mask(n, n)
    zc = (np.arange(n) + 0.5) / n
    layer = (zc >= 0.25) & (zc <= 0.75)
    k = np.where(layer[:, None, None] & mask2[None, :, :], HZONE_IN_MD, HZONE_OUT_MD).ravel() * MD
    h = 100.0 / n
    prob = Problem(n, n, n, h, h, h, k, k.copy(), k.copy(), np.full(n ** 3, 0.2), *_wells([], []),
                   gravity=True, p_init=ATM, bc_type=(0, 0, 1, 1, 0, 0),
                   bc_value=(0.0, 0.0, ATM, 10 * ATM, 0.0, 0.0))
    prob.fluid = replace(prob.fluid, T=298.0, Tc=190.58, pc=4.604e6, Tb=111.67)
    s = SolverSettings(px=px, py=py, pz=pz, overlap=(1, 1, 1), levels=3, interp_order=1)
    return Case(f"3d_{n}x{n}x{n}_layered_flood", [prob], 0.1 * DAY, nsteps, s, case_3d_layered_flood.__doc__)


def case_2d_32():
    """2D 32x32, homogeneous 100 mD, phi 0.2, p0 20 MPa, injector (0,0) and
    producer (31,31) at 1e-3 kg/s, no gravity, 2 steps of 1 day (BDF1 then BDF2),
    one-level left-RAS with 4x4 subdomains, overlap 1, ILU(0), FP64."""
    nx = ny = 32
    N = nx * ny
    k = np.full(N, 100.0 * MD)
    wc, wr = _wells([_lin(nx, ny, 0, 0), _lin(nx, ny, 31, 31)], [1e-3, -1e-3])
    prob = Problem(nx, ny, 1, 10.0, 10.0, 10.0, k.copy(), k.copy(), k.copy(),
                   np.full(N, 0.2), wc, wr)
    s = SolverSettings(px=4, py=4, pz=1, overlap=(1,), levels=1)
    return Case("2d_32x32_onelevel", [prob], DAY, 2, s, case_2d_32.__doc__)


def case_2d_512(n=512):
    """2D 512x512, ln K = ln(100 mD) + 1.0 G (corr. length 8 cells, seed 2),
    porosity U[0.1, 0.3] (seed 12), five-spot: centre injector +4e-3 kg/s and
    four corner producers -1e-3 kg/s, 10 steps of 5 days, two-level V-cycle,
    16x16 subdomains, overlap 2 on both levels, FGMRES(30), FP64."""
    nx = ny = n
    N = nx * ny
    k = lognormal_perm((ny, nx), 100.0 * MD, 1.0, 8.0, 2).ravel()
    phi = np.random.Generator(np.random.PCG64(12)).uniform(0.1, 0.3, size=N)
    c = n // 2
    wc, wr = _wells([_lin(nx, ny, c, c), _lin(nx, ny, 0, 0), _lin(nx, ny, n - 1, 0),
                     _lin(nx, ny, 0, n - 1), _lin(nx, ny, n - 1, n - 1)],
                    [4e-3, -1e-3, -1e-3, -1e-3, -1e-3])
    prob = Problem(nx, ny, 1, 10.0, 10.0, 10.0, k.copy(), k.copy(), k.copy(), phi, wc, wr)
    # overlap 2 on both levels: 7% faster per step than a coarse overlap of 1
    s = SolverSettings(px=16, py=16, pz=1, overlap=(2, 2), levels=2)
    return Case(f"2d_{n}x{n}_twolevel_fp64", [prob], 5 * DAY, 10, s, case_2d_512.__doc__)


def _column_wells(nx, ny, nz, inj_xy, prod_xy, rate):
    cells, rates = [], []
    for z in range(nz):
        cells.append(_lin(nx, ny, inj_xy[0], inj_xy[1], z))
        rates.append(rate / nz)
    for z in range(nz):
        cells.append(_lin(nx, ny, prod_xy[0], prod_xy[1], z))
        rates.append(-rate / nz)
    return _wells(cells, rates)


def case_3d_128(nx=128, ny=128, nz=64, precision="fp32"):
    """3D 128x128x64, per-layer mean K log-uniform in [10, 1000] mD, sigma 1.5,
    corr. length 8 (seed 3), kv = 0.1 kh, phi 0.2, gravity with hydrostatic
    initial state (20 MPa top layer), injector column (0,0,:) and producer
    column (127,127,:) at 1e-3 kg/s split over layers, 5 steps of 5 days,
    three-level V-cycle, 8x8x4 subdomains on every level, overlap 1,
    first-order interpolation, FP32 or BF16 ILU factors with FP64 FGMRES(30)
    and residual."""
    kh = layered_perm(nx, ny, nz, 10.0, 1000.0, 1.5, 8.0, 3).ravel() * MD
    N = nx * ny * nz
    wc, wr = _column_wells(nx, ny, nz, (0, 0), (nx - 1, ny - 1), 1e-3)
    prob = Problem(nx, ny, nz, 10.0, 10.0, 10.0, kh.copy(), kh.copy(), 0.1 * kh,
                   np.full(N, 0.2), wc, wr, gravity=True)
    # first-order interpolation: in 3D the Galerkin products of the
    # second-order one grow to ~63-125-point stencils, 3.4x slower per step
    s = SolverSettings(px=8, py=8, pz=4, overlap=(1, 1, 1), levels=3, precision=precision,
                       interp_order=1)
    return Case(f"3d_{nx}x{ny}x{nz}_threelevel_{precision}", [prob], 5 * DAY, 5, s,
                case_3d_128.__doc__)


def case_batch64(nres=64, nmin=64, nmax=256, tile=32, overlap=2, ratio=4, coarse_kernel="chunked"):
    """64 independent 2D reservoirs, side n_b uniform in {64..256}, sigma_b
    uniform in [0.5, 2], corr. length 8, mean 100 mD, phi 0.2, one injector and
    one producer (+-1e-3 kg/s) at seeded cells at least n_b/4 apart
    (seeds 400..463), 3 steps of 5 days, two-level V-cycle, FP32 preconditioner
    with FP64 outer solve.  Subdomain tile side, overlap and coarse-to-fine
    ratio are tunable (one overlap on both levels); the defaults are among the
    autotuner's choice on MI355X (tile 32, overlap 2, ratio 4).  The coarse
    GMRES runs in captured chunks of launches; its persistent form, at its own
    best settings (ratio 8, overlap 1), runs about 9% slower here with a third
    of the host waits."""
    rng = np.random.Generator(np.random.PCG64(4000))
    probs = []
    for b in range(nres):
        n = int(rng.integers(nmin, nmax + 1))
        sig = float(rng.uniform(0.5, 2.0))
        k = lognormal_perm((n, n), 100.0 * MD, sig, 8.0, 400 + b).ravel()
        wr_rng = np.random.Generator(np.random.PCG64(400 + b + 10000))
        while True:
            a = wr_rng.integers(0, n, size=2)
            c = wr_rng.integers(0, n, size=2)
            if np.hypot(*(a - c)) >= n / 4:
                break
        wc, wr = _wells([_lin(n, n, a[0], a[1]), _lin(n, n, c[0], c[1])], [1e-3, -1e-3])
        probs.append(Problem(n, n, 1, 10.0, 10.0, 10.0, k.copy(), k.copy(), k.copy(),
                             np.full(n * n, 0.2), wc, wr))
    s = SolverSettings(px=1, py=1, pz=1, tile=(tile, tile, 0), overlap=(overlap, overlap), levels=2,
                       precision="fp32", ratio=ratio, coarse_kernel=coarse_kernel)
    return Case(f"batch{nres}_2d_fp32prec", probs, 5 * DAY, 3, s, case_batch64.__doc__)


def case_3d_96_adjoint(nx=96, ny=96, nz=48):
    """3D 96x96x48 channelised: 10 mD background with 8 sinusoidal 1000 mD
    channels (seed 5), kv/kh 0.1, phi 0.2, gravity, column wells as in the 128x128x64 case,
    3 steps of 5 days, two-level FP64, first-order interpolation.  Objective: producer-column mean
    pressure at the final step; gradient with respect to ln K per cell."""
    kh = channel_perm(nx, ny, nz, 10.0, 1000.0, 8, 5).ravel() * MD
    N = nx * ny * nz
    wc, wr = _column_wells(nx, ny, nz, (0, 0), (nx - 1, ny - 1), 1e-3)
    prob = Problem(nx, ny, nz, 10.0, 10.0, 10.0, kh.copy(), kh.copy(), 0.1 * kh,
                   np.full(N, 0.2), wc, wr, gravity=True)
    s = SolverSettings(px=6, py=6, pz=3, overlap=(1, 1), levels=2, interp_order=1)
    return Case(f"3d_{nx}x{ny}x{nz}_adjoint", [prob], 5 * DAY, 3, s, case_3d_96_adjoint.__doc__)


def with_solver(case, **kw):
    return replace(case, solver=replace(case.solver, **kw))
