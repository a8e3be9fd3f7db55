"""Pins of the oracle's paper-faithful operator variants (CPU only).

* Two densities (Section 2, eqs. cpoiss and kappapoiss): the mass term takes rho^n, the face
  coefficient rho^{n+1}. Pinned by the face-velocity update of step (viii) of the algorithm
  (with rho^{n+1}) and the mass term of eq. cpoiss (with rho^n), by the separable FFT +
  tridiagonal reduction with two different density profiles, and by invariances.
* Inhomogeneous Neumann data (the stability problem of Section 2): a discrete field of constant
  flux through variable coefficients is reproduced exactly; the stability problem converges at
  second order to e^x; its perturbation rows (Table perturbtest) fall in a band around the
  paper's printed errors (its discretisation is FEM, so only magnitudes are comparable).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import mg, separable
from paper_1112_3507_amd import workloads as wl

P, N = 0, 1


def _two_densities(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 3.0, shape), rng.uniform(0.5, 3.0, shape), rng.uniform(0.5, 3.0, shape)


def test_equal_densities_give_the_one_density_operator():
    n, bc, h = (6, 4, 5), (P, P, N), (0.25, 0.5, 0.2)
    shape = (5, 4, 6)
    rho, _, c2 = _two_densities(shape, 1)
    a = oracle.assemble(n, h, bc, rho, c2, 0.7)
    b = oracle.assemble(n, h, bc, rho, c2, 0.7, rho_face=rho.copy())
    assert np.array_equal(a.rowptr, b.rowptr) and np.array_equal(a.colind, b.colind)
    assert np.array_equal(a.val, b.val)


def test_two_density_operator_is_mass_plus_divergence_of_step_viii_face_velocity():
    """A p = p / (rho^n c2) + dt div_h(u) with u the face velocity of step (viii) for u* = 0,
    u_{i+1/2} = -dt (p_{i+1} - p_i) / h * 2 / (rho^{n+1}_{i+1} + rho^{n+1}_i): rho^n only in the
    mass term (eq. cpoiss), rho^{n+1} only in the faces (eq. kappapoiss)."""
    n, bc, h = (6, 4, 5), (P, N, N), (0.25, 0.5, 0.2)
    shape = (5, 4, 6)
    rho_n, rho_np1, c2 = _two_densities(shape, 2)
    dt = 0.7
    p = np.random.default_rng(3).standard_normal(shape)
    div = np.zeros(shape)
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        pp = np.roll(p, -1, axis=ax)
        rr = np.roll(rho_np1, -1, axis=ax)
        u_plus = -dt * (pp - p) / h[d] * 2.0 / (rr + rho_np1)
        if bc[d] == N:
            idx = [slice(None)] * 3
            idx[ax] = -1
            u_plus[tuple(idx)] = 0.0
        div += (u_plus - np.roll(u_plus, 1, axis=ax)) / h[d]
    expected = p / (rho_n * c2) + dt * div
    got = oracle.assemble(n, h, bc, rho_n, c2, dt, rho_face=rho_np1).matvec(p).reshape(shape)
    assert np.allclose(got, expected, rtol=1e-12, atol=1e-12 * np.abs(expected).max())
    r = oracle.residual(n, h, bc, rho_n, c2, dt, p, np.zeros(shape), rho_face=rho_np1).reshape(shape)
    assert np.allclose(-r, expected, rtol=1e-12, atol=1e-12 * np.abs(expected).max())


def test_two_density_separable_reduction():
    """z-only rho^n and rho^{n+1} that differ (a 3% density change over the step): PCG on the
    assembled operator against FFT in x, y plus a tridiagonal solve per mode in z."""
    n = (32, 16, 24)
    p = wl.polytrope(n, 0.001, noise=0.0)
    rz = p.rho[:, 0, 0]
    rfz = rz * (1.0 + 0.03 * np.sin(7.0 * np.arange(n[2])))
    rf = np.broadcast_to(rfz[:, None, None], p.shape).copy()
    b = wl.rhs_white(n, 22)
    xs = separable.solve_stratified(p.n, p.h, p.bc, rz, p.c2[:, 0, 0], p.dt, b, rho_face_z=rfz)
    x, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b, rho_face=rf)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
    # the one-density solution is a different one (the faces matter)
    x1 = separable.solve_stratified(p.n, p.h, p.bc, rz, p.c2[:, 0, 0], p.dt, b)
    assert np.linalg.norm(x1 - xs) > 1e-3 * np.linalg.norm(xs)


def test_two_density_invariances():
    """rho^n -> s rho^n with c2 -> c2 / s keeps m; rho^{n+1} -> s rho^{n+1} with dt -> dt sqrt(s)
    keeps every face weight: both leave the operator unchanged (to rounding)."""
    n, bc, h = (4, 6, 5), (P, P, N), (0.3, 0.2, 0.25)
    shape = (5, 6, 4)
    rho_n, rho_np1, c2 = _two_densities(shape, 4)
    dt = 0.9
    a = oracle.assemble(n, h, bc, rho_n, c2, dt, rho_face=rho_np1).to_dense()
    b = oracle.assemble(n, h, bc, 3.0 * rho_n, c2 / 3.0, dt, rho_face=rho_np1).to_dense()
    c = oracle.assemble(n, h, bc, rho_n, c2, dt * np.sqrt(2.5), rho_face=2.5 * rho_np1).to_dense()
    scale = np.abs(a).max()
    assert np.allclose(a, b, rtol=0, atol=1e-14 * scale)
    assert np.allclose(a, c, rtol=0, atol=1e-14 * scale)


def test_two_density_hierarchy_uses_face_density_and_mass():
    n = (16, 8, 12)
    shape = (12, 8, 16)
    rho_n, rho_np1, c2 = _two_densities(shape, 5)
    lv = mg.build_hierarchy(n, (1 / 16, 1 / 8, 1 / 12), (P, P, N), rho_n, c2, 0.05, coarsest_max=64,
                            rho_face=rho_np1)
    assert np.array_equal(lv[0].rho, rho_np1)
    assert np.array_equal(lv[0].m, 1.0 / (rho_n * c2))
    A = oracle.assemble(n, lv[0].h, (P, P, N), rho_n, c2, 0.05, rho_face=rho_np1)
    x = np.random.default_rng(6).standard_normal(shape)
    assert np.allclose(mg.apply(lv[0], x).reshape(-1), A.matvec(x), rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ Neumann data

@pytest.mark.parametrize("axis", [0, 2])
def test_constant_flux_field_is_reproduced_exactly(axis):
    """A discrete field whose flux kappa_f (phi_b - phi_a) / h is the same constant F through
    every face along `axis` (phi_{i+1} = phi_i + F h (rho_i + rho_{i+1}) / 2 with rho = rho^{n+1},
    varying) is the exact solution when the rhs is m phi plus the boundary fluxes -F (low end,
    outward normal -e_axis) and +F (high end): the interior fluxes cancel, and the boundary
    terms supply exactly the flux the operator omits. A sign, scale or spacing mistake in the
    boundary term fails this."""
    n = (12, 4, 10)
    bc = [P, P, P]
    bc[axis] = N
    bc = tuple(bc)
    h = (0.1, 0.25, 0.125)
    shape = (n[2], n[1], n[0])
    rng = np.random.default_rng(7)
    rho_face_1d = rng.uniform(0.5, 2.5, n[axis])
    F = 0.37
    phi_1d = np.empty(n[axis])
    phi_1d[0] = 1.3
    for i in range(n[axis] - 1):
        phi_1d[i + 1] = phi_1d[i] + F * h[axis] * (rho_face_1d[i] + rho_face_1d[i + 1]) / 2.0
    ax = 2 - axis  # array axis of the grid axis
    bshape = [1, 1, 1]
    bshape[ax] = n[axis]
    phi = np.broadcast_to(phi_1d.reshape(bshape), shape).copy()
    rho_np1 = np.broadcast_to(rho_face_1d.reshape(bshape), shape).copy()
    rho_n = rng.uniform(0.5, 2.0, shape)
    c2 = rng.uniform(0.5, 2.0, shape)
    dt = 0.8
    plane = tuple(v for k, v in enumerate(shape) if k != ax)
    b = phi / (rho_n * c2)
    b = oracle.neumann_rhs(n, h, bc, dt, axis, 0, np.full(plane, -F), b)
    b = oracle.neumann_rhs(n, h, bc, dt, axis, 1, np.full(plane, F), b)
    x, st = oracle.reference_solve(n, h, bc, rho_n, c2, dt, b, rho_face=rho_np1)
    assert np.max(np.abs(x - phi)) <= 1e-11 * np.max(np.abs(phi))


def test_neumann_data_rejected_on_a_periodic_axis():
    with pytest.raises(ValueError):
        oracle.neumann_rhs((4, 4, 4), (1, 1, 1), (P, P, N), 1.0, 0, 0, np.zeros((4, 4)))


def _stability_errors(nx, case, seed=0):
    p = wl.stability_problem(nx, case, seed)
    b = p.f.copy()
    for (axis, side), q in p.neumann.items():
        b = oracle.neumann_rhs(p.n, p.h, p.bc, p.dt, axis, side, q, b)
    x, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b, rho_face=p.rho_face)
    assert st["converged"] or st["stagnated"]
    xc = (np.arange(nx) + 0.5) / nx
    e = np.abs(x - np.exp(xc)[None, None, :])
    return np.array([e.mean(), np.sqrt((e ** 2).mean()), e.max()])


def test_stability_problem_through_neumann_data_second_order():
    e = [_stability_errors(nx, "unperturbed") for nx in (25, 50, 100)]
    for k in range(3):
        assert 3.6 < e[0][k] / e[1][k] < 4.4
        assert 3.6 < e[1][k] / e[2][k] < 4.4


def _golden_e2():
    path = os.path.join(os.path.dirname(__file__), "golden", "e2_perturbtest.txt")
    rows = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, l1, l2, linf = line.split()
        rows[name] = np.array([float(l1), float(l2), float(linf)])
    return rows


def test_stability_table_rows_in_band_of_the_paper():
    """The paper's stability problem at 100 x 100 with the perturbation rows of Table perturbtest
    (random perturbations of amplitude 1e-2 in f, kappa or c~). The random fields are not the
    paper's and the discretisation differs (FV here, FEM there), so the L1, L2 and Linf errors
    against e^x (mean over four perturbation seeds) are held to a band of [1/5, 5] times the
    paper's single-core values; and, as the paper observes, perturbing kappa or c~ raises the
    error several times over the unperturbed one."""
    gold = _golden_e2()
    got = {}
    for case, row in (("unperturbed", "unperturbed_1core"), ("f", "f_perturbed_1core"),
                      ("kappa", "kappa_perturbed_1core"), ("c", "c_perturbed_1core")):
        seeds = [0] if case == "unperturbed" else [0, 1, 2, 3]
        got[case] = np.mean([_stability_errors(100, case, s) for s in seeds], axis=0)
        ratio = got[case] / gold[row]
        assert np.all(ratio > 0.2) and np.all(ratio < 5.0), (case, got[case], gold[row])
    for case in ("kappa", "c"):
        assert np.all(got[case] > 3.0 * got["unperturbed"]), case
