"""Pins of the oracle's multigrid building blocks (CPU only).

The blocks are checked against closed forms (transfers reproduce constants and linear functions),
defining properties (a Gauss-Seidel half sweep zeroes the residual on its colour; the V-cycle is
a symmetric positive definite operator), the independent C assembly (level operators), and the
PCG oracle (sweeps converge to its solution; the V-cycle preconditions it).
"""
import numpy as np
import pytest

import oracle
from oracle import mg
from paper_1112_3507_amd import workloads as wl


def _levels(n=(16, 8, 12), mach=0.01, seed=3, coarsest_max=64):
    p = wl.polytrope(n, mach, seed=seed)
    return p, mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=coarsest_max)


def test_hierarchy_shapes_and_rules():
    p = wl.polytrope((24, 8, 20), 0.01, seed=1, noise=0.0)
    lv = mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=16)
    dims = [L.n for L in lv]
    # x periodic 24 -> 12 -> 6 (6/2 = 3 odd periodic: stop); y periodic 8 -> 4 -> 2 (stop);
    # z Neumann 20 -> 10 -> 5 (odd: stop)
    assert dims == [(24, 8, 20), (12, 4, 10), (6, 2, 5)]
    assert lv[1].coarsened == (True, True, True)
    assert lv[1].h == (2 * p.h[0], 2 * p.h[1], 2 * p.h[2])


def test_level_operator_matches_c_assembly():
    p, lv = _levels()
    rng = np.random.default_rng(0)
    for L in lv:
        x = rng.standard_normal(L.shape)
        c2 = 1.0 / (L.rho * L.m)
        A = oracle.assemble(L.n, L.h, L.bc, L.rho, c2, L.dt)
        y1 = A.matvec(x).reshape(L.shape)
        y2 = mg.apply(L, x)
        assert np.linalg.norm(y1 - y2) <= 1e-13 * np.linalg.norm(y1)


def test_half_sweep_zeroes_residual_on_its_colour():
    p, lv = _levels()
    L = lv[0]
    rng = np.random.default_rng(1)
    r = rng.standard_normal(L.shape)
    z = rng.standard_normal(L.shape)
    col = mg.colour(L)
    for c in (0, 1):
        z2 = mg.half_sweep(L, r, z, c)
        res = r - mg.apply(L, z2)
        scale = np.max(mg.diagonal(L) * np.abs(z2)) + np.max(np.abs(r))   # size of the terms
        assert np.max(np.abs(res[col == c])) <= 1e-14 * scale
        assert np.array_equal(z2[col != c], z[col != c])


def test_symmetric_sweeps_converge_to_solution():
    p = wl.polytrope((8, 4, 6), 2.0, seed=4)
    L = mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=10_000)[0]
    b = wl.rhs_white(p.n, 5)
    x_ref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    z = np.zeros(L.shape)
    for _ in range(3000):
        z = mg.half_sweep(L, b, z, 0)
        z = mg.half_sweep(L, b, z, 1)
    assert np.linalg.norm(z - x_ref) <= 1e-8 * np.linalg.norm(x_ref)


def _linear(L, coef):
    nz, ny, nx = L.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (coef[0] * (i + 0.5) * L.h[0] + coef[1] * (j + 0.5) * L.h[1]
            + coef[2] * (k + 0.5) * L.h[2] + coef[3])


def test_transfers_closed_forms():
    p, lv = _levels((16, 8, 12))
    Lf, Lc = lv[0], lv[1]
    # constants are reproduced by P and R everywhere
    assert np.allclose(mg.prolong(Lf, Lc, np.ones(Lc.shape)), 1.0, rtol=0, atol=1e-15)
    assert np.allclose(mg.restrict(Lf, Lc, np.ones(Lf.shape)), 1.0, rtol=0, atol=1e-15)
    # linear functions are reproduced exactly away from the boundaries (cell centres)
    coef = (0.7, -1.3, 2.1, 0.4)
    uc = _linear(Lc, coef)
    uf = mg.prolong(Lf, Lc, uc)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.allclose(uf[inner], _linear(Lf, coef)[inner], rtol=0, atol=1e-13)
    rf = mg.restrict(Lf, Lc, _linear(Lf, coef))
    assert np.allclose(rf[inner], uc[inner], rtol=0, atol=1e-13)
    # Neumann ends: the mirror makes the boundary fine cell copy its parent
    e = np.random.default_rng(2).standard_normal(Lc.shape)
    pf = mg.prolong(Lf, Lc, e)
    assert np.allclose(pf[0, 2, 2], 0.75 * 0.75 * e[0, 1, 1] + 0.75 * 0.25 * e[0, 1, 0]
                       + 0.25 * 0.75 * e[0, 0, 1] + 0.25 * 0.25 * e[0, 0, 0])
    # adjointness R = P^T / 8
    rng = np.random.default_rng(3)
    u = rng.standard_normal(Lf.shape)
    v = rng.standard_normal(Lc.shape)
    lhs = np.sum(mg.restrict(Lf, Lc, u) * v)
    rhs = np.sum(u * mg.prolong(Lf, Lc, v)) / 8.0
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(u)) * np.max(np.abs(v))


def test_vcycle_symmetric_positive_and_contracting():
    p, lv = _levels((16, 8, 12), mach=0.001)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(lv[0].shape)
    y = rng.standard_normal(lv[0].shape)
    Mx, My = mg.vcycle(lv, x), mg.vcycle(lv, y)
    assert abs(np.sum(Mx * y) - np.sum(x * My)) <= 1e-12 * np.linalg.norm(Mx) * np.linalg.norm(y)
    assert np.sum(Mx * x) > 0
    # as a stationary iteration the V-cycle contracts the error strongly
    b = wl.rhs_white(p.n, 6)
    x_ref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    xk = np.zeros(lv[0].shape)
    errs = []
    for _ in range(4):
        xk = xk + mg.vcycle(lv, b - mg.apply(lv[0], xk))
        errs.append(np.linalg.norm(xk - x_ref))
    assert errs[-1] / errs[-2] < 0.5


def test_vcycle_preconditioned_cg_reaches_oracle():
    p, lv = _levels((16, 8, 12), mach=0.001, seed=7)
    b = wl.rhs_white(p.n, 8)
    x_ref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    L = lv[0]
    x = np.zeros(L.shape)
    r = b.copy()
    z = mg.vcycle(lv, r)
    pp = z.copy()
    rz = np.sum(r * z)
    its = 0
    while np.linalg.norm(r) > 1e-10 * np.linalg.norm(b):
        q = mg.apply(L, pp)
        a = rz / np.sum(pp * q)
        x += a * pp
        r -= a * q
        z = mg.vcycle(lv, r)
        rz, rz_old = np.sum(r * z), rz
        pp = z + (rz / rz_old) * pp
        its += 1
        assert its < 40
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("flags", [(True, True, True), (True, False, True), (False, True, False)])
def test_child_mean_of_an_affine_field_is_its_centroid_value(flags):
    """The coarse coefficients are 8-child (or 4-, 2-child) means: for the affine field
    a(i, j, k) = i + 10 j + 100 k (exact in FP64) the mean over the children of coarse cell
    (I, J, K) is the field at the children's centroid, e.g. 2I + 1/2 in x on a coarsened axis and
    I itself on one that is not coarsened."""
    nz, ny, nx = 6, 4, 8
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = i + 10.0 * j + 100.0 * k
    got = mg.child_mean(a, flags)
    fx, fy, fz = (2 if flags[0] else 1), (2 if flags[1] else 1), (2 if flags[2] else 1)
    assert got.shape == (nz // fz, ny // fy, nx // fx)
    K, J, I = np.meshgrid(np.arange(nz // fz), np.arange(ny // fy), np.arange(nx // fx), indexing="ij")
    cx = fx * I + (0.5 if flags[0] else 0.0)
    cy = fy * J + (0.5 if flags[1] else 0.0)
    cz = fz * K + (0.5 if flags[2] else 0.0)
    assert np.array_equal(got, cx + 10.0 * cy + 100.0 * cz)
    # a positive field keeps its total (mean preserving) and stays within the children's range
    b = np.random.default_rng(4).uniform(0.5, 2.0, (nz, ny, nx))
    cb = mg.child_mean(b, flags)
    assert abs(cb.sum() * fx * fy * fz - b.sum()) <= 1e-12 * b.sum()
    assert cb.min() >= b.min() and cb.max() <= b.max()
