"""GPU parity of the second face rule (HP_OPT_FACE_RULE = 1: kappa_f = (1/rho_a + 1/rho_b)/2)
against the oracle's implementation of the same rule, element by element.

The inputs are polytropes with 30% coefficient noise, so that neighbouring densities differ by
up to a factor of ~2 and the two rules give operators (and pressures) that differ far beyond the
parity bars; each test also checks that it can tell the rules apart. Tolerances as in the
parity tests of the default rule: building blocks 1e-13 (apply) / 1e-12 (half sweeps) in FP64
and 2e-5 in FP32, the V-cycle 1e-9 (1e-4 FP32), full solves 1e-9 relative L2 at a true relative
residual of 1e-10.
"""
import functools

import numpy as np
import pytest

import oracle
from oracle import mg
from paper_1112_3507_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP GPU")]

import paper_1112_3507_amd as hp  # noqa: E402

DEV = "cuda:0"
RAGGED = (80, 24, 40)
DEEP = (256, 32, 32)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@functools.lru_cache(maxsize=None)
def problem(n, mach=0.001):
    return wl.polytrope(n, mach, seed=3, noise=0.3)


def make(p, rule, mode=None, layout=None):
    s = hp.setup(p.n, p.h, p.bc, dev(p.rho), dev(p.c2), p.dt, mode)
    s.set_option(hp.OPT_FACE_RULE, rule)
    if layout is not None:
        s.set_option(hp.OPT_LAYOUT, layout)
    return s


def test_face_rule_option_values():
    p = problem(RAGGED)
    with hp.setup(p.n, p.h, p.bc, dev(p.rho), dev(p.c2), p.dt) as s:
        assert s.get_option(hp.OPT_FACE_RULE) == 0
        for bad in (2, -1, 0.5):
            with pytest.raises(hp.HPError) as ei:
                s.set_option(hp.OPT_FACE_RULE, bad)
            assert ei.value.code == hp.EINVAL
        s.set_option(hp.OPT_FACE_RULE, 1)
        assert s.get_option(hp.OPT_FACE_RULE) == 1


@pytest.mark.parametrize("grid", [RAGGED, DEEP])
@pytest.mark.parametrize("layout", [1, 0])
@pytest.mark.parametrize("f32", [False, True])
def test_rule_one_building_blocks(f32, layout, grid):
    """Apply on every level, the R, B, B, R half sweeps, the coarsest solve and the V-cycle."""
    p = problem(grid)
    lv = mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=512, face_rule=1)
    lv0 = mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=512, face_rule=0)
    rng = np.random.default_rng(7)
    dt = torch.float32 if f32 else torch.float64
    rnd = (lambda a: a.astype(np.float32).astype(np.float64)) if f32 else (lambda a: a)
    with make(p, 1, layout=layout) as s:
        assert s.num_levels() == len(lv)
        for l, L in enumerate(lv):
            x = rnd(rng.standard_normal(L.shape))
            y = torch.empty(L.shape, dtype=dt, device=DEV)
            s.apply(l, dev(x, dt), y, f32=f32)
            ref = mg.apply(L, x)
            assert relerr(host(y), ref) <= (2e-5 if f32 else 1e-13), (l, f32)
            assert relerr(mg.apply(lv0[l], x), ref) > 1e-3   # the rules differ here
        for l, L in enumerate(lv[:-1]):
            r = rnd(rng.standard_normal(L.shape))
            z0 = rnd(rng.standard_normal(L.shape))
            zt, rt, ref = dev(z0, dt), dev(r, dt), z0
            for c in (0, 1, 1, 0):
                s.smooth(l, rt, zt, c, f32=f32)
                ref = mg.half_sweep(L, r, ref, c)
                assert relerr(host(zt), ref) <= (2e-5 if f32 else 1e-12), (l, c)
        Lc = lv[-1]
        b = rnd(rng.standard_normal(Lc.shape))
        xc = torch.empty(Lc.shape, dtype=dt, device=DEV)
        s.coarse_solve(dev(b, dt), xc, f32=f32)
        assert relerr(host(xc), mg.coarse_solve(Lc, b)) <= (1e-6 if f32 else 1e-10)
        r = rnd(rng.standard_normal(lv[0].shape))
        z = torch.empty(lv[0].shape, dtype=dt, device=DEV)
        s.precond(dev(r, dt), z, f32=f32)
        assert relerr(host(z), mg.vcycle(lv, r)) <= (1e-4 if f32 else 1e-9)


@functools.lru_cache(maxsize=None)
def reference(rule):
    p = problem(RAGGED)
    b = wl.rhs_white(p.n, 11)
    x, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b, face_rule=rule)
    assert st["converged"] or st["stagnated"]
    return b, x


@pytest.mark.parametrize("mode", [hp.MODE_FP64_MGPCG, hp.MODE_MIXED_IR, hp.MODE_JACOBI_PCG])
def test_rule_one_solves_match_oracle(mode):
    p = problem(RAGGED)
    b, xref = reference(1)
    _, xref0 = reference(0)
    assert relerr(xref0, xref) > 1e-4      # the rules give different pressures
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p, 1, mode=mode) as s:
        st = s.solve(dev(b), x, tol=1e-10)
    xg = host(x)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, xg, b, face_rule=1)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    # Jacobi-PCG leaves its residual in low modes: its error bound is kappa * tol
    assert relerr(xg, xref) <= (1e-8 if mode == hp.MODE_JACOBI_PCG else 1e-9), mode


def test_switching_the_rule_back_reproduces_a_fresh_handle():
    """Setting rule 1 and then rule 0 recomputes the rule-dependent setup: the solve is bit for
    bit that of a handle that never left rule 0 (the solver is deterministic)."""
    p = problem(RAGGED)
    b, _ = reference(0)
    xa = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    xb = torch.zeros_like(xa)
    with make(p, 0) as s:
        s.solve(dev(b), xa, tol=1e-10)
    with make(p, 1) as s:
        x1 = torch.zeros_like(xa)
        s.solve(dev(b), x1, tol=1e-10)
        s.set_option(hp.OPT_FACE_RULE, 0)
        s.solve(dev(b), xb, tol=1e-10)
    assert torch.equal(xa, xb)
    assert relerr(host(x1), host(xa)) > 1e-4
