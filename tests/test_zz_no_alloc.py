"""GPU check of the entry point that allocates nothing (hp_dot_noalloc) against hp_dot.

Both run the same two reduction kernels with the same grid, so the results agree bitwise; the
no-allocation form keeps its partial sums in the library's static device array, which the second
call (a smaller length) reuses after the first one left it full.
"""
import math

import numpy as np
import pytest

from paper_1112_3507_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP GPU")]

import paper_1112_3507_amd as hp  # noqa: E402

DEV = "cuda:0"


def _vec(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) * np.exp(rng.uniform(-3, 3, n))


def test_dot_noalloc_matches_hp_dot_on_two_calls():
    p = wl.polytrope((256, 64, 64), 0.001, seed=3)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    stream = torch.cuda.Stream()
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        for n, seed in ((1_000_003, 1), (77_777, 2), (0, 3)):
            x = _vec(n, seed)
            y = _vec(n, seed + 100)
            xt = torch.from_numpy(x).to(DEV)
            yt = torch.from_numpy(y).to(DEV)
            ref = s.dot(xt, yt)
            out = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                hp.dot_noalloc(xt, yt, out, stream)
            stream.synchronize()
            got = float(out.cpu()[0])
            assert got == ref, (n, got, ref)
            assert abs(got - math.fsum((x * y).tolist())) <= n * 2.0 ** -53 * float(np.sum(np.abs(x * y)))


def test_dot_noalloc_rejects_bad_arguments():
    out = torch.zeros(1, dtype=torch.float64, device=DEV)
    x = torch.zeros(4, dtype=torch.float64, device=DEV)
    lib = hp.load_library()
    import ctypes
    assert lib.hp_dot_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), -1,
                              ctypes.c_void_p(out.data_ptr()), None) == hp.EINVAL
    assert lib.hp_dot_noalloc(None, None, 4, ctypes.c_void_p(out.data_ptr()), None) == hp.EINVAL
    assert lib.hp_dot_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 4,
                              None, None) == hp.EINVAL
    assert b"null" in lib.hp_noalloc_last_error()
