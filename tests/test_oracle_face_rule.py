"""Pins of the oracle's second face rule (CPU only).

Section 2 gives kappa = 1/rho per cell (eq. kappapoiss) and leaves its value on a face to the
discretisation. Face rule 0 (the default) takes kappa_f = 2 / (rho_a + rho_b), the factor of the
face-velocity update of step (viii); face rule 1 takes the mean of the two cells' kappa,
(1/rho_a + 1/rho_b) / 2. The pins: constant density makes the rules coincide bit for bit; on two
cells the operator is written out by hand, and the difference of the rules is the closed form
(rho_a - rho_b)^2 / (2 rho_a rho_b (rho_a + rho_b)); the operator stays symmetric with A 1 = m
and A - diag(m) positive semidefinite; the matrix-free residual, the multigrid module's apply on
every level and the CSR assembly (three separately written paths) agree.
"""
import numpy as np
import pytest

import oracle
from oracle import mg

P, N = 0, 1


def _fields(shape, seed, lo=0.4, hi=3.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, shape), rng.uniform(0.5, 2.0, shape)


def test_constant_density_rules_coincide_bitwise():
    n, bc, h = (6, 4, 5), (P, N, N), (0.25, 0.5, 0.2)
    shape = (5, 4, 6)
    _, c2 = _fields(shape, 1)
    rho = np.full(shape, 1.7)
    a = oracle.assemble(n, h, bc, rho, c2, 0.3, face_rule=0)
    b = oracle.assemble(n, h, bc, rho, c2, 0.3, face_rule=1)
    assert np.array_equal(a.colind, b.colind) and np.array_equal(a.val, b.val)


def test_two_cells_by_hand_and_difference_of_the_rules():
    """Two cells along x with closed walls: A = [[ma + w, -w], [-w, mb + w]], w = dt^2 kappa_f / h^2."""
    ra, rb, ca, cb, dt, hx = 0.8, 2.9, 1.3, 0.6, 0.45, 0.3
    n, h, bc = (2, 1, 1), (hx, 1.0, 1.0), (N, N, N)
    rho = np.array([ra, rb]).reshape(1, 1, 2)
    c2 = np.array([ca, cb]).reshape(1, 1, 2)
    ma, mb = 1.0 / (ra * ca), 1.0 / (rb * cb)
    s = dt * dt / (hx * hx)
    for rule, kappa in ((0, 2.0 / (ra + rb)), (1, 0.5 * (1.0 / ra + 1.0 / rb))):
        A = oracle.assemble(n, h, bc, rho, c2, dt, face_rule=rule).to_dense()
        w = s * kappa
        assert np.allclose(A, [[ma + w, -w], [-w, mb + w]], rtol=1e-15, atol=0)
    A0 = oracle.assemble(n, h, bc, rho, c2, dt, face_rule=0).to_dense()
    A1 = oracle.assemble(n, h, bc, rho, c2, dt, face_rule=1).to_dense()
    gap = s * (ra - rb) ** 2 / (2.0 * ra * rb * (ra + rb))
    assert np.isclose(A0[0, 1] - A1[0, 1], gap, rtol=1e-13) and gap > 0


@pytest.mark.parametrize("bc", [(P, P, P), (N, N, N), (P, N, P)])
def test_rule_one_operator_is_symmetric_with_mass_row_sums(bc):
    n, h = (6, 4, 4), (0.2, 0.25, 0.3)
    shape = (4, 4, 6)
    rho, c2 = _fields(shape, 2)
    A = oracle.assemble(n, h, bc, rho, c2, 0.6, face_rule=1).to_dense()
    m = (1.0 / (rho * c2)).reshape(-1)
    assert np.array_equal(A, A.T)
    assert np.allclose(A @ np.ones(A.shape[0]), m, rtol=1e-13, atol=0)
    ev = np.linalg.eigvalsh(A - np.diag(m))
    assert ev.min() >= -1e-12 * ev.max()
    # rule 1 is never below rule 0 on a face (the arithmetic mean of 1/rho bounds the harmonic
    # one), so A1 - A0 is itself a positive semidefinite sum of face terms
    A0 = oracle.assemble(n, h, bc, rho, c2, 0.6, face_rule=0).to_dense()
    assert np.linalg.eigvalsh(A - A0).min() >= -1e-12


def test_rule_one_paths_agree_matrix_free_csr_and_multigrid_levels():
    n, h, bc = (16, 8, 12), (1 / 16, 1 / 8, 1 / 12), (P, P, N)
    shape = (12, 8, 16)
    rho, c2 = _fields(shape, 3)
    rf, _ = _fields(shape, 4)
    dt = 0.05
    rng = np.random.default_rng(5)
    x = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    A = oracle.assemble(n, h, bc, rho, c2, dt, rho_face=rf, face_rule=1)
    r_mf = oracle.residual(n, h, bc, rho, c2, dt, x, b, rho_face=rf, face_rule=1)
    r_csr = b.reshape(-1) - A.matvec(x.reshape(-1))
    scale = np.abs(b).max() + np.abs(A.matvec(x.reshape(-1))).max()
    assert np.max(np.abs(r_mf - r_csr)) <= 1e-14 * scale
    levels = mg.build_hierarchy(n, h, bc, rho, c2, dt, coarsest_max=64, rho_face=rf, face_rule=1)
    assert len(levels) >= 3
    for L in levels:
        # the level's operator is the oracle's assembly on that grid with the level's (child-
        # mean) face density and mass term (c2 chosen so that 1 / (rho c2) = m)
        xl = rng.standard_normal(L.shape)
        Al = oracle.assemble(L.n, L.h, L.bc, L.rho, 1.0 / (L.rho * L.m), L.dt, face_rule=1)
        y = Al.matvec(xl.reshape(-1))
        assert np.allclose(mg.apply(L, xl).reshape(-1), y, rtol=1e-13, atol=1e-13 * np.abs(y).max())


def test_rule_one_solve_converges_and_differs_from_rule_zero_as_the_faces_do():
    """The rules give different pressures when the density jumps (R2: with a few per cent face
    jumps the difference is far above the 1e-9 parity bar), and identical ones for constant rho."""
    n, h, bc = (12, 12, 8), (1 / 12, 1 / 12, 1 / 8), (P, P, N)
    shape = (8, 12, 12)
    rho, c2 = _fields(shape, 6)
    b = np.random.default_rng(7).standard_normal(shape)
    dt = 0.02
    x0, s0 = oracle.reference_solve(n, h, bc, rho, c2, dt, b, face_rule=0)
    x1, s1 = oracle.reference_solve(n, h, bc, rho, c2, dt, b, face_rule=1)
    assert s0["converged"] and s1["converged"] or (s0["stagnated"] and s1["stagnated"])
    r1 = oracle.residual(n, h, bc, rho, c2, dt, x1, b, face_rule=1)
    assert np.linalg.norm(r1) <= 1e-12 * np.linalg.norm(b)
    assert np.linalg.norm(x1 - x0) > 1e-6 * np.linalg.norm(x0)
    with pytest.raises(ValueError):
        oracle.assemble(n, h, bc, rho, c2, dt, face_rule=2)
