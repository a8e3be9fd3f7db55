"""Pins of the oracle's steps either side of the pressure solve (CPU only).

The interface interpolation of eq. pbnd, the gradient of eq. nablaP, the interface velocity of
eq. step1, the right-hand side of eqs. fpoiss / fpoiss2 and the updates of steps (vii)-(ix) are
checked against what they must satisfy: closed forms (constant density gives the arithmetic
mean; linear pressure has an exact gradient), the defining property of eq. pbnd (the specific
acceleration is continuous through the interface), its tie to the face-velocity update of
step (viii), conservation (momentum in a periodic box; no flux through closed walls), a uniform
state as a fixed point of rhs -> solve -> update, and, the strongest, that after a whole step
the new interface velocities satisfy the discrete pressure equation, which links these NumPy
formulas to the independently assembled operator of the C oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import hydro
from paper_1112_3507_amd import workloads as wl

P, N = 0, 1


def _rand(shape, seed, lo=0.5, hi=3.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def test_interface_pressure_constant_density_is_the_mean():
    shape = (4, 5, 6)
    Pr = np.random.default_rng(1).standard_normal(shape)
    rho = np.full(shape, 2.5)
    for d in range(3):
        f = hydro.interface_pressure(Pr, rho, d, (P, P, P))
        assert np.allclose(f, 0.5 * (Pr + np.roll(Pr, -1, axis=2 - d)), rtol=1e-15, atol=1e-15)


def test_interface_pressure_makes_specific_acceleration_continuous():
    """(P_f - P_i) / rho_i = (P_{i+1} - P_f) / rho_{i+1} = (P_{i+1} - P_i) / (rho_i + rho_{i+1})."""
    shape = (3, 4, 7)
    rng = np.random.default_rng(2)
    Pr = rng.standard_normal(shape)
    rho = _rand(shape, 3)
    f = hydro.interface_pressure(Pr, rho, 0, (P, P, N))
    Pp, rp = np.roll(Pr, -1, axis=2), np.roll(rho, -1, axis=2)
    a1 = (f - Pr) / rho
    a2 = (Pp - f) / rp
    a3 = (Pp - Pr) / (rho + rp)
    assert np.allclose(a1, a2, rtol=1e-12, atol=1e-14) and np.allclose(a1, a3, rtol=1e-12, atol=1e-14)


def test_cell_acceleration_is_mean_of_step_viii_interface_accelerations():
    """(grad P)_i / rho_i = (a_{i+1/2} + a_{i-1/2}) / 2 with a_f = 2 (P_b - P_a) / ((rho_a + rho_b) h)
    the acceleration of the face-velocity update (step (viii)), on a periodic axis."""
    n, h = (9, 4, 3), (0.3, 0.5, 0.25)
    shape = (3, 4, 9)
    Pr = np.random.default_rng(4).standard_normal(shape)
    rho = _rand(shape, 5)
    g = hydro.grad_p(Pr, rho, n, h, (P, P, P))
    Pp, rp = np.roll(Pr, -1, axis=2), np.roll(rho, -1, axis=2)
    a_hi = 2.0 * (Pp - Pr) / ((rho + rp) * h[0])
    a_lo = np.roll(a_hi, 1, axis=2)
    assert np.allclose(g[0] / rho, 0.5 * (a_hi + a_lo), rtol=1e-12, atol=1e-13)


def test_gradient_of_linear_pressure_is_exact_and_walls_are_one_sided():
    n, h = (5, 6, 8), (0.2, 0.25, 0.125)
    shape = (8, 6, 5)
    k = np.arange(8)[:, None, None] * np.ones(shape)
    Pr = 3.0 + 0.7 * (k + 0.5) * h[2]
    rho = np.full(shape, 1.7)
    g = hydro.grad_p(Pr, rho, n, h, (P, P, N))
    assert np.allclose(g[2][1:-1], 0.7, rtol=1e-13) and np.allclose(g[0], 0) and np.allclose(g[1], 0)
    # at a closed end the wall value is the cell's own: a one-sided half difference
    assert np.allclose(g[2][0], 0.35, rtol=1e-13) and np.allclose(g[2][-1], 0.35, rtol=1e-13)


def test_gradient_converges_at_second_order():
    errs = []
    for nx in (32, 64, 128):
        h = 1.0 / nx
        x = (np.arange(nx) + 0.5) * h
        Pr = np.broadcast_to(np.sin(2 * np.pi * x)[None, None, :], (1, 1, nx)).copy()
        rho = np.broadcast_to((1.5 + np.cos(2 * np.pi * x))[None, None, :], (1, 1, nx)).copy()
        g = hydro.grad_p(Pr, rho, (nx, 1, 1), (h, h, h), (P, P, P))
        errs.append(np.max(np.abs(g[0] - 2 * np.pi * np.cos(2 * np.pi * x))))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_interface_velocity_is_the_centre_of_mass_velocity():
    """Eq. step1: the interface velocity is the combined momentum of the two cells over their
    combined mass. Hand-computed cases: (rho, u) = (1, 1) next to (3, 0) gives 1/4 (not the
    plain mean 1/2); (2, -1) next to (2, 3) gives 1; equal velocities give that velocity for any
    densities."""
    rho = np.array([1.0, 3.0, 2.0, 2.0, 0.7, 5.0]).reshape(1, 1, 6)
    u = np.array([1.0, 0.0, -1.0, 3.0, 0.4, 0.4]).reshape(1, 1, 6)
    f = hydro.interface_velocity(rho * u, rho, 0, (P, P, P))
    assert f[0, 0, 0] == 0.25 and f[0, 0, 2] == 1.0
    assert np.isclose(f[0, 0, 4], 0.4, rtol=1e-15)


def test_interface_velocity_and_closed_walls():
    """Eq. step1 with equal densities is the mean velocity; no flow through closed walls: the
    interface velocity vanishes at a closed high end and a closed low end counts as zero, so the
    divergence summed over a closed box is zero (discrete Gauss theorem)."""
    n, h = (6, 4, 5), (0.2, 0.3, 0.25)
    shape = (5, 4, 6)
    rng = np.random.default_rng(6)
    mom = rng.standard_normal((3,) + shape)
    rho = np.full(shape, 2.0)
    u = hydro.interface_velocity(mom[0], rho, 0, (P, P, N))
    assert np.allclose(u, 0.25 * (mom[0] + np.roll(mom[0], -1, axis=2)), rtol=1e-15)
    rho = _rand(shape, 7)
    bc = (N, N, N)
    uf = np.stack([hydro.interface_velocity(mom[d], rho, d, bc) for d in range(3)])
    assert np.all(uf[0][:, :, -1] == 0) and np.all(uf[1][:, -1, :] == 0) and np.all(uf[2][-1] == 0)
    div = hydro.div_interfaces(uf, n, h, bc)
    assert abs(np.sum(div)) <= 1e-13 * np.sum(np.abs(div))


def test_two_component_diffusion_term():
    """div(rho kappa_c grad c): zero for constant c; conserved (sums to zero) in a closed box;
    for linear c with constant rho kappa_c zero inside, +-flux/h in the boundary cells."""
    n, h = (4, 3, 10), (0.25, 0.3, 0.1)
    shape = (10, 3, 4)
    rk = _rand(shape, 8)
    bc = (P, P, N)
    assert np.allclose(hydro.div_kappa_grad(np.full(shape, 0.3), rk, n, h, bc), 0.0)
    c = np.random.default_rng(9).standard_normal(shape)
    d = hydro.div_kappa_grad(c, rk, n, h, bc)
    assert abs(d.sum()) <= 1e-12 * np.abs(d).sum()
    k = np.arange(10)[:, None, None] * np.ones(shape)
    cl = 0.2 * k * h[2]
    d = hydro.div_kappa_grad(cl, np.full(shape, 2.0), n, h, bc)
    assert np.allclose(d[1:-1], 0.0, atol=1e-13)
    assert np.allclose(d[0], 2.0 * 0.2 / h[2]) and np.allclose(d[-1], -2.0 * 0.2 / h[2])


def test_rhs_at_rest_is_mass_term_times_pressure():
    s = wl.hydro_state((8, 4, 6), 0.01, seed=1)
    p = s.p
    z = np.zeros_like(s.mom_n)
    b = hydro.pressure_rhs(p.n, p.h, p.bc, p.dt, p.rho, p.c2, s.p_n, z, p.rho_face, z)
    assert np.allclose(b, s.p_n / (p.rho * p.c2), rtol=1e-15)


def test_uniform_state_is_a_fixed_point_of_a_whole_step():
    """Constant density and pressure, uniform velocity, periodic box: the rhs is m P, the solve
    returns P (A const = m const), the momentum and energy are unchanged and the interface
    velocities are the uniform velocity."""
    n, h, bc = (6, 4, 8), (0.2, 0.25, 0.125), (P, P, P)
    shape = (8, 4, 6)
    rho = np.full(shape, 1.3)
    c2 = np.full(shape, 2.0)
    Pr = np.full(shape, 4.0)
    u = np.array([0.1, -0.05, 0.02])
    mom = rho[None] * u[:, None, None, None] * np.ones((3,) + shape)
    e = np.full(shape, 7.0)
    dt = 0.4
    b = hydro.pressure_rhs(n, h, bc, dt, rho, c2, Pr, mom, rho, mom)
    assert np.allclose(b, Pr / (rho * c2), rtol=1e-14)
    x, st = oracle.reference_solve(n, h, bc, rho, c2, dt, b)
    assert np.allclose(x, Pr, rtol=1e-11)
    mom1, uf, e1 = hydro.pressure_update(n, h, bc, dt, x, rho, mom, e)
    assert np.allclose(mom1, mom, rtol=1e-10, atol=1e-12)
    assert np.allclose(e1, e, rtol=1e-10)
    for d in range(3):
        assert np.allclose(uf[d], u[d], rtol=1e-10, atol=1e-12)


def test_momentum_is_conserved_in_a_periodic_box():
    n, h, bc = (8, 6, 4), (0.125, 0.2, 0.25), (P, P, P)
    shape = (4, 6, 8)
    rng = np.random.default_rng(10)
    Pr = rng.standard_normal(shape)
    rho = _rand(shape, 11)
    mom = rng.standard_normal((3,) + shape)
    mom1, _, _ = hydro.pressure_update(n, h, bc, 0.3, Pr, rho, mom, np.zeros(shape))
    for d in range(3):
        assert abs(mom1[d].sum() - mom[d].sum()) <= 1e-12 * np.abs(mom[d]).sum()


@pytest.mark.parametrize("two_component", [False, True])
def test_whole_step_satisfies_the_discrete_pressure_equation(two_component):
    """rhs (eq. fpoiss / fpoiss2) -> the two-density solve (C oracle, CSR assembled from its own
    face loop) -> update (step (viii)): the new interface velocities satisfy
        m (P - P^n + dt u^n . grad P^n) + dt div u^{n+1} + S = 0
    to the solve's accuracy (S the source terms of the rhs): the discrete pressure-evolution
    equation the scheme is built on. A mismatch between the rhs's div u*, the operator's faces and
    the face update of step (viii) fails this."""
    s = wl.hydro_state((12, 8, 10), 0.01, seed=2)
    p = s.p
    kw = dict(visc=s.visc)
    if two_component:
        kw.update(temp_n=s.temp_n, conc_n=s.conc_n, rkc_n=s.rkc_n, r_gas=s.r_gas)
    b = hydro.pressure_rhs(p.n, p.h, p.bc, p.dt, p.rho, p.c2, s.p_n, s.mom_n, p.rho_face, s.mom_star, **kw)
    x, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b, rho_face=p.rho_face)
    mom1, uf, e1 = hydro.pressure_update(p.n, p.h, p.bc, p.dt, x, p.rho_face, s.mom_star, s.e_star)
    m = 1.0 / (p.rho * p.c2)
    adv = np.sum(s.mom_n / p.rho[None] * hydro.grad_p(s.p_n, p.rho, p.n, p.h, p.bc), axis=0)
    src = (2.0 * p.dt / 3.0) * (m / p.rho) * s.visc
    if two_component:
        src = src + (3.0 * p.dt / 4.0) * m * s.r_gas * s.temp_n * hydro.div_kappa_grad(
            s.conc_n, s.rkc_n, p.n, p.h, p.bc)
    res = m * (x - s.p_n + p.dt * adv) + p.dt * hydro.div_interfaces(uf, p.n, p.h, p.bc) + src
    # algebraically res = A x - b: it equals minus the oracle's own residual of the solve (whatever
    # accuracy the solve reached), up to the rounding of terms of size |m x| and |dt div u|
    r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, x, b, rho_face=p.rho_face).reshape(x.shape)
    scale = np.linalg.norm(m * x) + np.linalg.norm(p.dt * hydro.div_interfaces(uf, p.n, p.h, p.bc))
    assert np.linalg.norm(res + r) <= 1e-13 * scale
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(b)
    # and the same without the solve is far from zero (the equation is not trivially met)
    res0 = m * (0.0 - s.p_n + p.dt * adv) + p.dt * hydro.div_interfaces(
        np.stack([hydro.interface_velocity(s.mom_star[d], p.rho_face, d, p.bc) for d in range(3)]),
        p.n, p.h, p.bc) + src
    assert np.linalg.norm(res0) > 0.1 * np.linalg.norm(b)
