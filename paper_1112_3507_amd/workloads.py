"""Seeded synthetic inputs for the pressure solve (host, FP64, NumPy).

This module only draws coefficient fields and right-hand sides; it contains none of the solver's
arithmetic, so both the GPU path and the CPU oracle are fed from here.

The fields stand in for the paper's workloads, which are not available: the stratified,
convectively unstable polytropic layer of Section 5 ("Physical Setting": ideal gas with
gamma = 5/3, polytropic index alpha = 1/(gamma - 1) = 1.5, linear temperature gradient), on the
equidistant box with horizontally periodic and vertically closed boundaries, and the Mach-number
ladder of the Gresho-vortex test (Ma = 0.1, 0.01, 0.001). Normalisation: T = 1 + 9 z (10x
contrast), rho = T^1.5, c2 = T (all constants 1), and dt from an advective CFL of 1 with
|u| = Ma * c_ref, c_ref = 1: dt = h / Ma, so dt^2 c^2 / h^2 = Ma^-2 at the cool end.

Layout: arrays shaped (nz, ny, nx), C order, x fastest. Axis order of n/h/bc is (x, y, z).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PERIODIC = 0
NEUMANN = 1


@dataclass
class Problem:
    name: str
    n: tuple          # (nx, ny, nz)
    h: tuple          # (hx, hy, hz)
    bc: tuple         # (bcx, bcy, bcz)
    rho: np.ndarray   # (nz, ny, nx) float64; with two densities: rho^n (the mass term's)
    c2: np.ndarray    # (nz, ny, nx) float64
    dt: float
    rho_face: np.ndarray | None = None  # rho^{n+1} (the face coefficients'); None: same as rho
    f: np.ndarray | None = None         # a given right-hand side (before boundary data)
    neumann: dict | None = None         # {(axis, side): prescribed outward normal flux per face}

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def ncells(self):
        return self.n[0] * self.n[1] * self.n[2]


def z_centres(nz: int, hz: float) -> np.ndarray:
    return (np.arange(nz) + 0.5) * hz


def exp_atmosphere_2d(nx: int = 64, nz: int = 64, courant2: float = 100.0) -> Problem:
    """2D nx x 1 x nz on the unit box: rho = exp(-z / 0.5), c2 = 1, dt^2 c^2 / h^2 = courant2."""
    h = 1.0 / nz
    z = z_centres(nz, h)
    rho = np.broadcast_to(np.exp(-z / 0.5)[:, None, None], (nz, 1, nx)).copy()
    c2 = np.ones((nz, 1, nx))
    dt = float(np.sqrt(courant2)) * h
    return Problem("exp2d_%dx%d" % (nx, nz), (nx, 1, nz), (h, h, h), (PERIODIC, PERIODIC, NEUMANN),
                   rho, c2, dt)


def polytrope(n, mach: float, seed: int = 0, noise: float = 0.01, contrast: float = 10.0,
              index: float = 1.5, h: float | None = None, mu=None) -> Problem:
    """Stratified polytropic box, periodic in x and y, Neumann in z.

    T = 1 + (contrast - 1) z, rho = T^index * mu * (1 + noise U), c2 = (T / mu) * (1 + noise U'),
    U, U' independent uniform(-1, 1) per cell from NumPy PCG64 seeded with `seed`
    (rho first, then c2). h defaults to 1 / nz on every axis; dt = h / mach.
    `mu` (optional) is a function of z giving the mean molecular weight profile.
    """
    nx, ny, nz = (int(v) for v in n)
    if h is None:
        h = 1.0 / nz
    z = z_centres(nz, h)
    T = 1.0 + (contrast - 1.0) * z
    muz = np.ones(nz) if mu is None else np.asarray(mu(z), dtype=np.float64)
    rho_z = T ** index * muz
    c2_z = T / muz
    rho = np.broadcast_to(rho_z[:, None, None], (nz, ny, nx)).copy()
    c2 = np.broadcast_to(c2_z[:, None, None], (nz, ny, nx)).copy()
    if noise:
        rng = np.random.default_rng(seed)
        rho *= 1.0 + noise * rng.uniform(-1.0, 1.0, size=rho.shape)
        c2 *= 1.0 + noise * rng.uniform(-1.0, 1.0, size=c2.shape)
    dt = h / mach
    tag = "polytrope_%dx%dx%d_Ma%g%s" % (nx, ny, nz, mach, "" if noise else "_smooth")
    return Problem(tag, (nx, ny, nz), (h, h, h), (PERIODIC, PERIODIC, NEUMANN), rho, c2, dt)


def rhs_white(n, seed: int) -> np.ndarray:
    """N(0, 1) per cell (NumPy PCG64, `seed`), minus its mean."""
    nx, ny, nz = (int(v) for v in n)
    b = np.random.default_rng(seed).standard_normal((nz, ny, nx))
    return b - b.mean()


def rhs_smooth(n, seed: int, modes: int = 16, kmax: int = 4) -> np.ndarray:
    """Smooth field: sum of `modes` terms a cos(2 pi (kx x + ky y) + phi) cos(pi kz z), minus mean.

    a ~ N(0, 1), kx, ky in {-kmax..kmax}, kz in {0..kmax}, phi ~ U(0, 2 pi) (PCG64, `seed`);
    coordinates are cell centres of the unit box.
    """
    nx, ny, nz = (int(v) for v in n)
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    b = np.zeros((nz, ny, nx))
    for _ in range(modes):
        a = rng.standard_normal()
        kx, ky = rng.integers(-kmax, kmax + 1, size=2)
        kz = rng.integers(0, kmax + 1)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        hor = np.cos(2 * np.pi * (kx * x[None, :] + ky * y[:, None]) + phi)
        b += a * np.cos(np.pi * kz * z)[:, None, None] * hor[None, :, :]
    return b - b.mean()


def rhs_modes_2d(nx: int, nz: int, seed: int, modes: int = 8) -> np.ndarray:
    """Sum of `modes` terms a_j sin(2 pi kx_j x) cos(pi kz_j z) on cell centres of the unit box.

    a_j ~ N(0, 1), kx_j uniform in {1..8}, kz_j uniform in {0..8} (NumPy PCG64, `seed`).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(modes)
    kx = rng.integers(1, 9, size=modes)
    kz = rng.integers(0, 9, size=modes)
    x = (np.arange(nx) + 0.5) / nx
    z = (np.arange(nz) + 0.5) / nz
    b = np.zeros((nz, 1, nx))
    for j in range(modes):
        b[:, 0, :] += a[j] * np.cos(np.pi * kz[j] * z)[:, None] * np.sin(2 * np.pi * kx[j] * x)[None, :]
    return b


def config0() -> Problem:
    """2D 64 x 64, periodic x / Neumann z, rho = exp(-z/0.5), c2 = 1, dt^2 c^2 / h^2 = 100."""
    return exp_atmosphere_2d(64, 64, 100.0)


def config1(mach: float = 0.01, n: int = 256, seed: int = 0, noise: float = 0.01) -> Problem:
    """256^3 polytrope, coefficient seed 0, Ma = 0.01 (dt = 100 h)."""
    return polytrope((n, n, n), mach, seed=seed, noise=noise)


def semiconvection_mu(z):
    """Mean-molecular-weight step mu(z) = 1 + 0.1 tanh((z - 0.5) / 0.02)."""
    return 1.0 + 0.1 * np.tanh((np.asarray(z) - 0.5) / 0.02)


def with_density_change(p: Problem, seed: int, change: float = 0.01) -> Problem:
    """Two densities on the grid of `p`: rho^n = p.rho and rho^{n+1} = rho^n (1 + change U),
    U uniform(-1, 1) per cell (PCG64, `seed`), standing in for the density after one explicit
    step (eqs. cpoiss and kappapoiss take rho^n in the mass term and rho^{n+1} in kappa)."""
    rng = np.random.default_rng(seed)
    rf = p.rho * (1.0 + change * rng.uniform(-1.0, 1.0, size=p.rho.shape))
    return Problem(p.name + "_two_density", p.n, p.h, p.bc, p.rho, p.c2, p.dt, rho_face=rf)


STABILITY_CASES = ("unperturbed", "f", "kappa", "c")


def stability_problem(nx: int, case: str, seed: int = 0, ny: int | None = None,
                      amplitude: float = 1e-2) -> Problem:
    """The stability problem of Section 2 (Table perturbtest): -Laplace(phi) + phi = 0 on the
    unit square, Neumann in x with outward normal derivatives -e^0 at x = 0 and e^1 at x = 1,
    periodic in y; exact solution phi = e^x. As the dt^2-scaled operator: dt = 1, rho^n = 1,
    c2 = 1 (m = c~ = 1), rho^{n+1} = 1 (kappa = 1), f = 0, on nx x ny x 1 cells of size 1/nx.
    The boundary data are the prescribed outward normal fluxes kappa dphi/dn of the unperturbed
    problem (kappa = 1), which a perturbation of kappa leaves unchanged.

    case: "unperturbed"; "f", "kappa" or "c" add random perturbations of amplitude `amplitude`
    (uniform(-1, 1) per cell, PCG64 `seed`) to f, to kappa (rho^{n+1} = 1 / (1 + a U)) or to
    c~ (c2 = 1 / (1 + a U), so m = 1 + a U)."""
    if case not in STABILITY_CASES:
        raise ValueError("unknown case %r" % case)
    ny = nx if ny is None else ny
    h = 1.0 / nx
    shape = (1, ny, nx)
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)
    rho = np.ones(shape)
    rf = np.ones(shape)
    c2 = np.ones(shape)
    f = np.zeros(shape)
    if case == "kappa":
        rf = 1.0 / (1.0 + amplitude * u)
    elif case == "c":
        c2 = 1.0 / (1.0 + amplitude * u)
    elif case == "f":
        f = amplitude * u
    neu = {(0, 0): np.full((1, ny), -np.exp(0.0)), (0, 1): np.full((1, ny), np.exp(1.0))}
    return Problem("stability_%d_%s" % (nx, case), (nx, ny, 1), (h, h, h), (NEUMANN, PERIODIC, NEUMANN),
                   rho, c2, 1.0, rho_face=rf, f=f, neumann=neu)


@dataclass
class HydroState:
    """The fields either side of one pressure solve (arrays (nz, ny, nx); momenta (3, nz, ny, nx)
    with x, y, z components)."""
    p: Problem                  # grid, boundaries, dt; p.rho = rho^n, p.c2 = c2^n, p.rho_face = rho^{n+1}
    p_n: np.ndarray             # pressure P^n
    mom_n: np.ndarray           # (rho u)^n
    mom_star: np.ndarray        # (rho u)* after the explicit step
    e_star: np.ndarray          # total energy e* after the explicit step
    visc: np.ndarray            # viscous / heat-conduction group of eq. fpoiss at time n
    temp_n: np.ndarray          # temperature T^n (two-component term of eq. fpoiss2)
    conc_n: np.ndarray          # helium mass fraction c^n
    rkc_n: np.ndarray           # rho^n kappa_c
    r_gas: float = 1.0


def hydro_state(n, mach: float, seed: int = 0) -> HydroState:
    """A seeded stand-in for the state of the stratified box at one time step: the polytrope of
    `polytrope` (rho^n, c2^n; P^n = rho T = T^2.5 with T = 1 + 9z before noise), rho^{n+1} with a
    1% change, a smooth random velocity of magnitude ~Ma (sum of low Fourier modes) vanishing at
    the closed z ends, (rho u)^n = rho^n u, (rho u)* = (rho u)^n plus 1% of noise, e* = P / (gamma - 1)
    + rho |u|^2 / 2 (gamma = 5/3), a viscous group of size ~Ma^2, and for the two-component term
    T = 1 + 9z, a helium mass fraction step c = 0.25 + 0.05 tanh((z - 0.5) / 0.02) and
    rho kappa_c = 1e-3 rho. All draws PCG64 from `seed`."""
    nx, ny, nz = (int(v) for v in n)
    base = polytrope(n, mach, seed=seed)
    rng = np.random.default_rng(seed + 7919)
    rho_n = base.rho
    rho_np1 = rho_n * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=rho_n.shape))
    h = base.h[2]
    x = (np.arange(nx) + 0.5) * base.h[0]
    y = (np.arange(ny) + 0.5) * base.h[1]
    z = z_centres(nz, h)
    T = 1.0 + 9.0 * z
    p_n = np.broadcast_to((T ** 2.5)[:, None, None], rho_n.shape).copy()
    p_n *= 1.0 + 1e-4 * rng.uniform(-1.0, 1.0, size=p_n.shape)
    Lx, Ly = nx * base.h[0], ny * base.h[1]
    u = np.zeros((3,) + rho_n.shape)
    for _ in range(6):
        kx, ky = rng.integers(-3, 4, size=2)
        kz = rng.integers(1, 4)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
        amp = rng.standard_normal(3) * mach
        hx = np.cos(2 * np.pi * (kx * x[None, :] / Lx + ky * y[:, None] / Ly) + ph[0])[None]
        u[0] += amp[0] * hx * np.cos(np.pi * kz * z + ph[1])[:, None, None]
        u[1] += amp[1] * hx * np.cos(np.pi * kz * z + ph[2])[:, None, None]
        u[2] += amp[2] * hx * np.sin(np.pi * kz * z)[:, None, None]
    mom_n = rho_n[None] * u
    mom_star = mom_n * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=mom_n.shape))
    e_star = p_n / (5.0 / 3.0 - 1.0) + 0.5 * rho_np1 * np.sum(u * u, axis=0)
    visc = mach ** 2 * rng.standard_normal(rho_n.shape)
    temp = np.broadcast_to(T[:, None, None], rho_n.shape).copy()
    conc = np.broadcast_to((0.25 + 0.05 * np.tanh((z - 0.5) / 0.02))[:, None, None], rho_n.shape).copy()
    p = Problem(base.name + "_hydro", base.n, base.h, base.bc, rho_n, base.c2, base.dt, rho_face=rho_np1)
    return HydroState(p, p_n, mom_n, mom_star, e_star, visc, temp, conc, 1e-3 * rho_n)


def gresho(n: int, mach: float, gamma: float = 5.0 / 3.0):
    """The Gresho vortex of Section 5 on the unit square, n x n x 1 cells, periodic in x and y
    (the z axis has one cell). rho = 1; with r the distance from (0.5, 0.5) and theta its angle,
    u_phi = 5r (r <= 0.2), 2 - 5r (0.2 <= r <= 0.4), 0 beyond; P = P0 + 12.5 r^2,
    P0 + 12.5 r^2 + 4 (1 - 5r - ln 0.2 + ln r), P0 - 2 + 4 ln 2 in the same ranges,
    P0 = rho / (gamma Ma^2). The velocity is the rotation u = u_phi (-sin theta, cos theta), whose
    centrifugal force this pressure balances (the paper's text prints the x component without its
    minus sign). Returns (Problem, rho, momentum (3, 1, n, n), total energy e, P)."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")          # (ny, nx)
    dx, dy = X - 0.5, Y - 0.5
    r = np.sqrt(dx * dx + dy * dy)
    th = np.arctan2(dy, dx)
    uphi = np.where(r <= 0.2, 5.0 * r, np.where(r <= 0.4, 2.0 - 5.0 * r, 0.0))
    p0 = 1.0 / (gamma * mach * mach)
    rs = np.maximum(r, 1e-300)
    P = np.where(r <= 0.2, p0 + 12.5 * r * r,
                 np.where(r <= 0.4, p0 + 12.5 * r * r + 4.0 * (1.0 - 5.0 * r - np.log(0.2) + np.log(rs)),
                          p0 - 2.0 + 4.0 * np.log(2.0)))
    rho = np.ones((1, n, n))
    mom = np.zeros((3, 1, n, n))
    mom[0, 0] = -np.sin(th) * uphi
    mom[1, 0] = np.cos(th) * uphi
    P = P.reshape(1, n, n)
    e = P / (gamma - 1.0) + 0.5 * np.sum(mom * mom, axis=0) / rho
    prob = Problem("gresho_%d_Ma%g" % (n, mach), (n, n, 1), (h, h, h), (PERIODIC, PERIODIC, NEUMANN),
                   rho, np.full(rho.shape, gamma * p0), 1.0)
    return prob, rho, mom, e, P
