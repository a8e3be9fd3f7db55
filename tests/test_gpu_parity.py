"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle, element by element.

Sizes span several workgroup tiles with ragged tails (80 x 24 x 40: x tiles of 64 with a tail of
16, odd coarse sizes) and finish in seconds on the oracle; the full-size cases (256^3, the
benchmark's launch configuration) are checked against the separable FFT + tridiagonal reduction
(noise off) and by the oracle's matrix-free residual certificate (noise on).

Tolerances: building blocks in FP64 are compared to 1e-12 relative (only the summation order
of at most 64 products differs, each rounding contributes ~1e-16, amplified by the cancellation
between the m and w terms of at most |terms| / |result|); the V-cycle to 1e-9 (its coarsest solve
goes through an explicit inverse of an operator with condition number ~1e5); full solves to the
bar of 1e-9 relative L2 at true residual 1e-10. FP32 blocks are compared with 2e-5 (a few FP32
ulps through the same cancellations).
"""
import functools

import numpy as np
import pytest

import oracle
from oracle import mg, separable
from paper_1112_3507_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP GPU")]

import paper_1112_3507_amd as hp  # noqa: E402

DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a).ravel() - np.asarray(b).ravel())
                 / max(np.linalg.norm(np.asarray(b).ravel()), 1e-300))


def make(p, mode=None, layout=None):
    s = hp.setup(p.n, p.h, p.bc, dev(p.rho), dev(p.c2), p.dt, mode)
    if layout is not None:
        s.set_option(hp.OPT_LAYOUT, layout)
        assert s.get_option(hp.OPT_LAYOUT) == layout
    return s


# finest-level storage: red-black split (the default where the grid allows it) and natural
LAYOUTS = [1, 0]


@functools.lru_cache(maxsize=None)
def problem(n, mach, seed=1, noise=0.01):
    return wl.polytrope(n, mach, seed=seed, noise=noise)


@functools.lru_cache(maxsize=None)
def reference(n, mach, seed, rhs_seed):
    p = problem(n, mach, seed)
    b = wl.rhs_white(p.n, rhs_seed)
    x, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    assert st["converged"] or st["stagnated"]
    return b, x


RAGGED = (80, 24, 40)
# 256 x 32 x 32: the split layout reaches levels 1 (128 x 16 x 16) and 2 (64 x 8 x 8) as well
DEEP = (256, 32, 32)
GRIDS = [RAGGED, DEEP]


# ------------------------------------------------------------------ building blocks (FP64/FP32)

def _hier(p):
    return mg.build_hierarchy(p.n, p.h, p.bc, p.rho, p.c2, p.dt, coarsest_max=512)


def test_hierarchy_matches_oracle_levels():
    p = problem(RAGGED, 0.001)
    lv = _hier(p)
    with make(p) as s:
        assert s.num_levels() == len(lv)
        for l, L in enumerate(lv):
            n, h = s.level_info(l)
            assert n == L.n
            assert np.allclose(h, L.h, rtol=0, atol=0)


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("f32", [False, True])
def test_apply_parity_every_level(f32, layout, grid):
    p = problem(grid, 0.001)
    lv = _hier(p)
    rng = np.random.default_rng(0)
    dt = torch.float32 if f32 else torch.float64
    with make(p, layout=layout) as s:
        for l, L in enumerate(lv):
            x = rng.standard_normal(L.shape)
            y = torch.empty(L.shape, dtype=dt, device=DEV)
            s.apply(l, dev(x, dt), y, f32=f32)
            ref = mg.apply(L, x if not f32 else x.astype(np.float32).astype(np.float64))
            assert relerr(host(y), ref) <= (2e-5 if f32 else 1e-13), (l, f32)


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("f32", [False, True])
def test_smoother_half_sweeps_parity(f32, layout, grid):
    p = problem(grid, 0.001)
    lv = _hier(p)
    rng = np.random.default_rng(1)
    dt = torch.float32 if f32 else torch.float64
    with make(p, layout=layout) as s:
        for l, L in enumerate(lv[:-1]):
            r = rng.standard_normal(L.shape)
            z0 = rng.standard_normal(L.shape)
            if f32:
                r = r.astype(np.float32).astype(np.float64)
                z0 = z0.astype(np.float32).astype(np.float64)
            zt = dev(z0, dt)
            rt = dev(r, dt)
            ref = z0
            for c in (0, 1, 1, 0):
                s.smooth(l, rt, zt, c, f32=f32)
                ref = mg.half_sweep(L, r, ref, c)
                assert relerr(host(zt), ref) <= (2e-5 if f32 else 1e-12), (l, c)


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("f32", [False, True])
def test_restrict_and_prolong_parity(f32, layout, grid):
    p = problem(grid, 0.001)
    lv = _hier(p)
    rng = np.random.default_rng(2)
    dt = torch.float32 if f32 else torch.float64
    with make(p, layout=layout) as s:
        for l in range(len(lv) - 1):
            Lf, Lc = lv[l], lv[l + 1]
            r = rng.standard_normal(Lf.shape)
            z = rng.standard_normal(Lf.shape) * 1e-3
            if f32:
                r = r.astype(np.float32).astype(np.float64)
                z = z.astype(np.float32).astype(np.float64)
            rc = torch.empty(Lc.shape, dtype=dt, device=DEV)
            s.restrict_residual(l, dev(r, dt), dev(z, dt), rc, f32=f32)
            ref = mg.restrict(Lf, Lc, r - mg.apply(Lf, z))
            assert relerr(host(rc), ref) <= (2e-4 if f32 else 1e-12), l
            ec = rng.standard_normal(Lc.shape)
            zf = rng.standard_normal(Lf.shape)
            if f32:
                ec = ec.astype(np.float32).astype(np.float64)
                zf = zf.astype(np.float32).astype(np.float64)
            zt = dev(zf, dt)
            s.prolong_add(l, dev(ec, dt), zt, f32=f32)
            assert relerr(host(zt), zf + mg.prolong(Lf, Lc, ec)) <= (1e-6 if f32 else 1e-15), l


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("f32", [False, True])
def test_coarse_solve_and_vcycle_parity(f32, layout, grid):
    p = problem(grid, 0.001)
    lv = _hier(p)
    rng = np.random.default_rng(3)
    dt = torch.float32 if f32 else torch.float64
    with make(p, layout=layout) as s:
        Lc = lv[-1]
        b = rng.standard_normal(Lc.shape)
        if f32:
            b = b.astype(np.float32).astype(np.float64)
        x = torch.empty(Lc.shape, dtype=dt, device=DEV)
        s.coarse_solve(dev(b, dt), x, f32=f32)
        assert relerr(host(x), mg.coarse_solve(Lc, b)) <= (1e-6 if f32 else 1e-10)
        r = rng.standard_normal(lv[0].shape)
        if f32:
            r = r.astype(np.float32).astype(np.float64)
        z = torch.empty(lv[0].shape, dtype=dt, device=DEV)
        s.precond(dev(r, dt), z, f32=f32)
        assert relerr(host(z), mg.vcycle(lv, r)) <= (1e-4 if f32 else 1e-9)


# coarsest levels of 8 cells (less than one 32-wide elimination block), 240 (a ragged last
# block) and 3332 (14 x 14 x 17: odd sizes stop the coarsening above the usual 512; 104 full
# blocks and a ragged one)
@pytest.mark.parametrize("grid,nc", [((2, 2, 2), 8), ((10, 6, 4), 240), ((28, 28, 17), 3332)])
def test_coarse_solve_parity_across_coarsest_sizes(grid, nc):
    p = problem(grid, 0.01)
    Lc = _hier(p)[-1]
    assert int(np.prod(Lc.shape)) == nc
    rng = np.random.default_rng(5)
    with make(p) as s:
        assert s.get_option(hp.OPT_COARSEST_MAX) == 512
        b = rng.standard_normal(Lc.shape)
        x = torch.empty(Lc.shape, dtype=torch.float64, device=DEV)
        s.coarse_solve(dev(b), x)
        assert relerr(host(x), mg.coarse_solve(Lc, b)) <= 1e-10


# ------------------------------------------------------------------ full solves

@pytest.mark.parametrize("mach,rhs_seed", [(0.001, 2), (0.01, 3)])
def test_fp64_mgpcg_matches_oracle(mach, rhs_seed):
    p = problem(RAGGED, mach)
    b, xref = reference(RAGGED, mach, 1, rhs_seed)
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p) as s:
        st = s.solve(dev(b), x, tol=1e-10)
    xg = host(x)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert relerr(xg, xref) <= 1e-9
    assert np.max(np.abs(xg - xref)) <= 1e-8 * np.max(np.abs(xref))
    # the oracle's own residual of the GPU result
    r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, xg, b)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_mixed_ir_matches_oracle():
    p = problem(RAGGED, 0.001)
    b, xref = reference(RAGGED, 0.001, 1, 2)
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p, hp.MODE_MIXED_IR) as s:
        st = s.solve(dev(b), x, tol=1e-10)
    assert st["converged"] and st["rel_residual"] <= 1e-10 and st["outer_iterations"] >= 1
    assert relerr(host(x), xref) <= 1e-9


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("mode", ["fp64", "mixed"])
def test_layouts_give_the_same_solve(mode, grid):
    """Natural and red-black split storage (the finest level; on the deeper grid level 1 too):
    both solves meet the bar against the oracle, and agree with each other to solver accuracy."""
    p = problem(grid, 0.001)
    b, xref = reference(grid, 0.001, 1, 2)
    m = hp.MODE_MIXED_IR if mode == "mixed" else hp.MODE_FP64_MGPCG
    xs = {}
    for layout in LAYOUTS:
        with make(p, m, layout=layout) as s:
            x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
            st = s.solve(dev(b), x, tol=1e-10)
            assert st["converged"] and st["rel_residual"] <= 1e-10, (layout, st)
            xs[layout] = host(x)
            assert relerr(xs[layout], xref) <= 1e-9, layout
    assert relerr(xs[1], xs[0]) <= 1e-9


def test_layout_option():
    """The split layout is the default where the grid allows it and refused where it does not."""
    with make(problem(RAGGED, 0.001)) as s:
        assert s.get_option(hp.OPT_LAYOUT) == 1
    small = problem((32, 8, 8), 0.001)
    with make(small) as s:
        assert s.get_option(hp.OPT_LAYOUT) == 0
        with pytest.raises(hp.HPError):
            s.set_option(hp.OPT_LAYOUT, 1)


def test_jacobi_pcg_config0():
    p = wl.config0()
    b = wl.rhs_modes_2d(64, 64, seed=0)
    xref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    xs = separable.solve_stratified(p.n, p.h, p.bc, p.rho[:, 0, 0], p.c2[:, 0, 0], p.dt, b)
    for mode in (hp.MODE_JACOBI_PCG, hp.MODE_FP64_MGPCG, hp.MODE_MIXED_IR):
        x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        with make(p, mode) as s:
            st = s.solve(dev(b), x, tol=1e-10)
        assert st["converged"] and st["rel_residual"] <= 1e-10
        # Jacobi-PCG leaves its residual in low modes: its error bound is kappa * tol
        assert relerr(host(x), xref) <= (1e-8 if mode == hp.MODE_JACOBI_PCG else 1e-9), mode
        assert relerr(xref, xs) <= 1e-11


@pytest.mark.parametrize("n,bc", [((2, 1, 6), (0, 0, 1)), ((4, 4, 4), (0, 0, 1)),
                                  ((16, 16, 16), (1, 1, 1)), ((8, 8, 8), (0, 0, 0)),
                                  ((12, 8, 15), (1, 0, 1)), ((64, 1, 64), (0, 0, 1)),
                                  ((1, 1, 40), (0, 0, 1)), ((36, 20, 7), (0, 0, 1))])
def test_solve_edge_shapes(n, bc):
    p = wl.polytrope(n, 0.01, seed=4)
    p.bc = bc
    b = wl.rhs_white(n, 5)
    xref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    for mode in (hp.MODE_FP64_MGPCG, hp.MODE_MIXED_IR):
        x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        with make(p, mode) as s:
            st = s.solve(dev(b), x, tol=1e-10)
        assert st["converged"], (n, bc, mode, st)
        assert relerr(host(x), xref) <= 1e-9, (n, bc, mode)


def test_warm_start_zero_rhs_and_errors():
    p = problem(RAGGED, 0.001)
    b, xref = reference(RAGGED, 0.001, 1, 2)
    with make(p) as s:
        # rhs = 0 gives p = 0 and no iterations
        x = torch.ones(p.shape, dtype=torch.float64, device=DEV)
        st = s.solve(torch.zeros_like(x), x, tol=1e-10)
        assert st["iterations"] == 0 and float(x.abs().max()) == 0.0
        # the converged solution as a warm start needs no iterations
        x = dev(xref)
        st = s.solve(dev(b), x, tol=1e-10)
        assert st["iterations"] == 0 and st["converged"]
        # iteration cap: HP_ENOCONV with the last iterate and stats filled
        s.set_option(hp.OPT_MAX_ITER, 1)
        x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        st = s.solve(dev(b), x, tol=1e-10, check=False)
        assert st["rc"] == hp.ENOCONV and st["iterations"] == 1 and st["rel_residual"] < 1.0
        s.set_option(hp.OPT_MAX_ITER, 1000)
        # non-finite right-hand side
        bn = dev(b)
        bn[3, 2, 1] = float("nan")
        with pytest.raises(hp.HPError) as e:
            s.solve(bn, x, tol=1e-10)
        assert e.value.code == hp.ENAN
        with pytest.raises(hp.HPError):
            s.set_option(hp.OPT_MODE, 7)
    rho = p.rho.copy()
    rho[5, 5, 5] = -1.0
    with pytest.raises(hp.HPError) as e:
        hp.setup(p.n, p.h, p.bc, dev(rho), dev(p.c2), p.dt)
    assert e.value.code == hp.EDOMAIN


def test_update_coefficients_matches_fresh_setup():
    p1 = problem(RAGGED, 0.001, seed=1)
    p2 = problem(RAGGED, 0.01, seed=2)
    b, xref = reference(RAGGED, 0.01, 2, 7)
    x = torch.zeros(p1.shape, dtype=torch.float64, device=DEV)
    with make(p1) as s:
        s.update_coefficients(dev(p2.rho), dev(p2.c2), p2.dt)
        st = s.solve(dev(b), x, tol=1e-10)
    assert st["converged"] and relerr(host(x), xref) <= 1e-9


# On 256 x 32 x 32 the split layout reaches levels 0, 1 and 2: an update rewrites arrays whose
# buffers the previous layout change rotated, writes the FP32 copies and Jacobi diagonals of those
# levels in split order directly and relays the rest; the solves must equal those of a fresh
# handle on the same coefficients bit for bit (same kernels, same order), in FP64 and mixed
# precision.
@pytest.mark.parametrize("mode", [hp.MODE_FP64_MGPCG, hp.MODE_MIXED_IR])
def test_update_on_split_levels_equals_fresh_setup(mode):
    p1 = problem(DEEP, 0.001, seed=1)
    p2 = problem(DEEP, 0.01, seed=2)
    b = dev(wl.rhs_white(p2.n, 7))
    out = []
    with make(p1, mode) as s:
        assert s.get_option(hp.OPT_LAYOUT) == 1
        s.update_coefficients(dev(p2.rho), dev(p2.c2), p2.dt)
        x = torch.zeros(p2.shape, dtype=torch.float64, device=DEV)
        st1 = s.solve(b, x, tol=1e-10)
        out.append(host(x))
        # and once more, from the state the first update left
        s.update_coefficients(dev(p2.rho), dev(p2.c2), p2.dt)
        x = torch.zeros(p2.shape, dtype=torch.float64, device=DEV)
        s.solve(b, x, tol=1e-10)
        out.append(host(x))
    with make(p2, mode) as s:
        x = torch.zeros(p2.shape, dtype=torch.float64, device=DEV)
        st2 = s.solve(b, x, tol=1e-10)
        out.append(host(x))
    assert st1["converged"] and st2["converged"] and st1["iterations"] == st2["iterations"]
    assert np.array_equal(out[0], out[2]) and np.array_equal(out[1], out[2])


@pytest.mark.parametrize("max_iter", [1, 2, 3])
def test_capped_solves_from_zero_return_their_iterate(max_iter):
    """A solve from a zero guess stopped after 1-3 iterations (HP_ENOCONV) returns its last
    iterate: the first update writes x = alpha p into an iterate never written before (the zero
    guess is only checked), on every path (the final update alone, or the look-ahead direction
    update), and the reported residual is the oracle's residual of what comes back."""
    p = problem(DEEP, 0.001)
    b = wl.rhs_white(p.n, 12)
    with make(p) as s:
        s.set_option(hp.OPT_MAX_ITER, max_iter)
        x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        st = s.solve(dev(b), x, tol=1e-10, check=False)
    assert st["rc"] == hp.ENOCONV and st["iterations"] == max_iter
    xg = host(x)
    assert np.all(np.isfinite(xg)) and np.linalg.norm(xg) > 0.0
    r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, xg, b)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    assert abs(rel - st["rel_residual"]) <= 1e-8 * rel
    assert rel < 1.0


def test_kernel_timing_counts_the_finest_launches():
    """HP_OPT_KERNEL_TIMING: on a split finest level every operator apply of a new direction and
    both post-smoothing half sweeps of every V-cycle are timed (events attached to the
    dispatches), the timing changes nothing in the result, and with natural storage nothing is
    timed."""
    p = problem(DEEP, 0.001)
    b = dev(wl.rhs_white(p.n, 9))
    with make(p) as s:
        x0 = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        st0 = s.solve(b, x0, tol=1e-10)
        assert st0["timed_sweeps"] == 0 and st0["timed_applies"] == 0
        s.set_option(hp.OPT_KERNEL_TIMING, 1)
        x1 = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        st1 = s.solve(b, x1, tol=1e-10)
        assert np.array_equal(host(x0), host(x1))
        its = st1["iterations"]
        assert st1["timed_sweeps"] % 2 == 0 and its <= st1["timed_sweeps"] // 2 <= its + 1
        assert its - 1 <= st1["timed_applies"] <= its
        assert 0.0 < st1["sweep_ms"] < st1["time_ms"] and 0.0 < st1["apply_ms"] < st1["time_ms"]
        s.set_option(hp.OPT_LAYOUT, 0)
        x2 = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        st2 = s.solve(b, x2, tol=1e-10)
        assert st2["converged"] and st2["timed_sweeps"] == 0 and st2["timed_applies"] == 0


def test_solve_is_deterministic():
    p = problem(RAGGED, 0.001)
    b, _ = reference(RAGGED, 0.001, 1, 2)
    outs = []
    with make(p) as s:
        for _ in range(2):
            x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
            s.solve(dev(b), x, tol=1e-10)
            outs.append(host(x))
    assert np.array_equal(outs[0], outs[1])


# ------------------------------------------------------------------ full size (256^3)

@pytest.mark.parametrize("mach", [0.01, 0.001])
def test_full_size_separable_pin(mach):
    n = (256, 256, 256)
    p = wl.polytrope(n, mach, noise=0.0)
    b = wl.rhs_white(n, 100)
    xs = separable.solve_stratified(p.n, p.h, p.bc, p.rho[:, 0, 0], p.c2[:, 0, 0], p.dt, b)
    for mode in (hp.MODE_FP64_MGPCG, hp.MODE_MIXED_IR):
        x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
        with make(p, mode) as s:
            st = s.solve(dev(b), x, tol=1e-10)
        assert st["converged"] and st["rel_residual"] <= 1e-10
        err = relerr(host(x), xs)
        print("256^3 separable Ma=%g mode=%d iterations=%d err=%.2e" % (mach, mode,
              st["iterations"], err), flush=True)
        assert err <= 1e-9


@pytest.mark.parametrize("mach", [0.01, 0.001])
def test_full_size_noisy_matches_oracle(mach):
    """The benchmarked configuration itself: the noisy 256^3 polytrope (coefficient seed 0) at
    Ma = 0.01 and 0.001 with a benchmark right-hand side (seed 105), solved by FP64 MG-PCG, the
    mixed-precision form, the learned warm start followed by FP64 MG-PCG and learned FCG (the
    shipped checkpoint), each compared element by element with the oracle's reference solution
    (Jacobi-PCG to a true relative residual of 1e-13): relative L2 error <= 1e-9 and max-abs
    error <= 1e-8 of max |x|, plus the oracle's own residual of each GPU result."""
    import os
    n = (256, 256, 256)
    p = wl.config1(mach=mach)
    b = wl.rhs_white(n, 105)
    xref, st_ref = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    assert st_ref["converged"] or st_ref["stagnated"]
    bt = dev(b)
    rho, c2 = dev(p.rho), dev(p.c2)
    forms = [("fp64", hp.MODE_FP64_MGPCG, False), ("mixed", hp.MODE_MIXED_IR, False)]
    wpath = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         "paper_1112_3507_amd", "weights", "unet128.npz")
    net = None
    if os.path.exists(wpath):
        from paper_1112_3507_amd import train as tr
        theta, scale = tr.load(wpath)
        net = hp.Net(n)
        net.set_params(torch.from_numpy(theta).to(DEV))
        net.set_output_scale(scale)
        forms += [("warm_start", hp.MODE_FP64_MGPCG, True), ("learned_fcg", hp.MODE_LEARNED, False)]
    xnorm = np.linalg.norm(xref)
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        if net is not None:
            s.attach_net(net)
        for name, mode, warm in forms:
            s.set_option(hp.OPT_MODE, mode)
            x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
            if warm:
                s.warm_start(bt, x)
            st = s.solve(bt, x, tol=1e-10)
            assert st["converged"] and st["rel_residual"] <= 1e-10, (name, st)
            xg = host(x)
            err = np.linalg.norm(xg - xref) / xnorm
            emax = np.max(np.abs(xg - xref)) / np.max(np.abs(xref))
            r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, xg, b)
            rres = np.linalg.norm(r) / np.linalg.norm(b)
            print("256^3 noisy Ma=%g %-11s iterations=%d err_vs_oracle=%.2e max_abs_rel=%.2e "
                  "oracle_residual=%.2e" % (mach, name, st["iterations"], err, emax, rres), flush=True)
            assert err <= 1e-9, (name, err)
            assert emax <= 1e-8, (name, emax)
            assert rres <= 1.01e-10, (name, rres)
        if net is not None:
            s.attach_net(None)
    if net is not None:
        net.close()


# ------------------------------------------------------------------ the largest configurations

def test_512_mixed_separable_pin():
    """512³, Ma = 0.001, mixed precision, noise off: against the FFT + tridiagonal reduction."""
    n = (512, 512, 512)
    p = wl.polytrope(n, 0.001, noise=0.0)
    b = wl.rhs_white(n, 100)
    xs = separable.solve_stratified(p.n, p.h, p.bc, p.rho[:, 0, 0], p.c2[:, 0, 0], p.dt, b)
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p, hp.MODE_MIXED_IR) as s:
        st = s.solve(dev(b), x, tol=1e-10)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    err = relerr(host(x), xs)
    print("512^3 separable mixed iterations=%d outer=%d err=%.2e" % (st["iterations"],
          st["outer_iterations"], err), flush=True)
    assert err <= 1e-9


def test_512_mixed_noisy_residual_certificate():
    n = (512, 512, 512)
    p = wl.polytrope(n, 0.001, seed=0)
    b = wl.rhs_white(n, 101)
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p, hp.MODE_MIXED_IR) as s:
        st = s.solve(dev(b), x, tol=1e-10)
    assert st["converged"]
    r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, host(x), b)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_semiconvection_1024x1024x512_sequence():
    """The two-component box: 1024 x 1024 x 512 on [0,2]² x [0,1] (h = 1/512), rho and c² from T
    and the mean-molecular-weight step, Ma = 0.001, mixed precision. A second coefficient set
    (the step moved up by one cell, new noise) goes through hp_update_coefficients without
    reallocation and is solved from the previous pressure. Each solve is certified by the
    oracle's matrix-free residual ("residual-certified, oracle-unpinned" at this size)."""
    n = (1024, 1024, 512)
    p = wl.polytrope(n, 0.001, seed=7, mu=wl.semiconvection_mu)
    b = wl.rhs_white(n, 7)
    bt = dev(b)
    x = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    with make(p, hp.MODE_MIXED_IR) as s:
        assert s.get_option(hp.OPT_LAYOUT) == 1
        st = s.solve(bt, x, tol=1e-10)
        assert st["converged"]
        r = oracle.residual(p.n, p.h, p.bc, p.rho, p.c2, p.dt, host(x), b)
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
        its0 = st["iterations"]
        del p
        q = wl.polytrope(n, 0.001, seed=8, mu=lambda z: wl.semiconvection_mu(np.asarray(z) - 1.0 / 512))
        s.update_coefficients(dev(q.rho), dev(q.c2), q.dt)
        st = s.solve(bt, x, tol=1e-10)
        assert st["converged"]
        r = oracle.residual(q.n, q.h, q.bc, q.rho, q.c2, q.dt, host(x), b)
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
        print("1024x1024x512 mixed: %d inner iterations from zero, %d from the previous pressure"
              % (its0, st["iterations"]), flush=True)


# ------------------------------------------------------------------ reductions

@pytest.mark.parametrize("n", [0, 1, 255, 1_000_003])
def test_dot_within_the_summation_bound(n):
    """hp_dot against the exactly rounded sum of the products (math.fsum): the difference stays
    within n u sum |x_i y_i| (u = 2^-53), the bound of any summation order; the result is the
    same on a second call (fixed reduction order)."""
    import math
    rng = np.random.default_rng(n + 5)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-4, 4, n))
    y = rng.standard_normal(n)
    ref = math.fsum((x * y).tolist())
    bound = n * 2.0 ** -53 * float(np.sum(np.abs(x * y)))
    # a handle of 2^20 cells: its partial-sum capacity covers vectors up to its own size
    p = problem((256, 64, 64), 0.001)
    with make(p) as s:
        xt = dev(x) if n else torch.zeros(0, dtype=torch.float64, device=DEV)
        yt = dev(y) if n else torch.zeros(0, dtype=torch.float64, device=DEV)
        got = s.dot(xt, yt)
        again = s.dot(xt, yt)
    assert got == again
    assert abs(got - ref) <= bound, (got, ref, bound)


@pytest.mark.parametrize("n", [(1 << 21) - 5, 1 << 21])
def test_dot_with_more_partials_than_one_pass_of_the_second_stage(n):
    """Vectors of 2^21 entries give 2048 first-stage partials, more than the second stage loads in
    its first pass (four per thread of one workgroup): the strided remainder is summed too, within
    the summation bound of math.fsum, and reproducibly."""
    import math
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) * np.exp(rng.uniform(-4, 4, n))
    y = rng.standard_normal(n)
    ref = math.fsum((x * y).tolist())
    bound = n * 2.0 ** -53 * float(np.sum(np.abs(x * y)))
    p = problem((128, 128, 128), 0.001)
    with make(p) as s:
        xt, yt = dev(x), dev(y)
        got = s.dot(xt, yt)
        assert got == s.dot(xt, yt)
    assert abs(got - ref) <= bound, (got, ref, bound)
    # a partial sum of only the first half of the products is far outside that bound
    assert abs(math.fsum((x[: n // 2] * y[: n // 2]).tolist()) - ref) > 100 * bound


def test_dot_exact_cancellation():
    """x = (h, h), y = (h, -h): the exact dot product is 0; the GPU result stays within the
    summation bound of it."""
    p = problem(RAGGED, 0.001)
    h = np.random.default_rng(9).standard_normal(1000)
    x = np.concatenate([h, h])
    y = np.concatenate([h, -h])
    with make(p) as s:
        got = s.dot(dev(x), dev(y))
    assert abs(got) <= 2000 * 2.0 ** -53 * float(np.sum(np.abs(x * y)))


@pytest.mark.parametrize("n", [0, 1, 7, 2048, (1 << 20) + 3])
def test_stream_copy(n):
    """hp_stream_copy (the benchmark's bandwidth reference) copies every entry, odd tails too, and
    refuses overlapping or misaligned buffers."""
    src = torch.rand(max(n, 1), dtype=torch.float64, device=DEV)[:n]
    dst = torch.full((max(n, 1),), -1.0, dtype=torch.float64, device=DEV)[:n]
    hp.stream_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    if n >= 8:
        with pytest.raises(hp.HPError):
            hp.stream_copy(src[: n - 2], src[2:])
        buf = torch.zeros(n + 1, dtype=torch.float64, device=DEV)
        with pytest.raises(hp.HPError):
            hp.stream_copy(src[: n - 1], buf[1:n])
