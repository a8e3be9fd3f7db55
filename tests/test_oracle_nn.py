"""Pins of the FP64 network reference (CPU only): convolution against SciPy's correlation,
backward passes against central finite differences, transfer adjoints, the first Adam step in
closed form, and bfloat16 rounding against PyTorch's conversion."""
import numpy as np
import pytest
from scipy import signal

from oracle import nn


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7, 3))
    W = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    out = nn.conv3(x, W, b)
    # pad: periodic in y and x, zeros in z
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="wrap")
    xp = np.pad(xp, ((1, 1), (0, 0), (0, 0), (0, 0)), mode="constant")
    for o in range(2):
        ref = np.full(x.shape[:3], b[o])
        for c in range(3):
            ref += signal.correlate(xp[..., c], W[o, :, c].reshape(3, 3, 3), mode="valid")
        assert np.allclose(out[..., o], ref, rtol=1e-12, atol=1e-12)


def _fd_check(f, x, g_analytic, rng, n_dirs=4, eps=1e-6, tol=1e-6):
    for _ in range(n_dirs):
        u = rng.standard_normal(x.shape)
        fd = (f(x + eps * u) - f(x - eps * u)) / (2 * eps)
        an = float(np.sum(g_analytic * u))
        assert abs(fd - an) <= tol * max(1.0, abs(an)), (fd, an)


def test_conv3_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 4, 6, 3))
    W = rng.standard_normal((5, 27, 3))
    b = rng.standard_normal(5)
    g = rng.standard_normal((4, 4, 6, 5))
    gx, gW, gb = nn.conv3_backward(x, W, g)
    _fd_check(lambda xx: float(np.sum(g * nn.conv3(xx, W, b))), x, gx, rng)
    _fd_check(lambda ww: float(np.sum(g * nn.conv3(x, ww, b))), W, gW, rng)
    _fd_check(lambda bb: float(np.sum(g * nn.conv3(x, W, bb))), b, gb, rng)


def test_pool_up_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(nn.pool2(x) * y), np.sum(x * nn.pool2_backward(y)))
    assert np.isclose(np.sum(nn.up2(y) * x), np.sum(y * nn.up2_backward(x)))
    assert np.allclose(nn.pool2(nn.up2(y)), y)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(3)
    theta = nn.init_params(7) + 0.01 * rng.standard_normal(nn.num_params())
    inp = rng.standard_normal((8, 8, 8, 4))
    target = rng.standard_normal((8, 8, 8))
    loss, grad = nn.loss_and_grad(theta, inp, target)
    assert grad.shape == (nn.num_params(),)
    # one random direction per parameter block; steps small enough that no ReLU changes side
    offs = np.cumsum([0] + [27 * a * b + b for a, b in nn.CONVS] + [17])
    for lo, hi in zip(offs[:-1], offs[1:]):
        u = np.zeros_like(theta)
        u[lo:hi] = rng.standard_normal(hi - lo)
        eps = 1e-7
        lp = nn.loss_and_grad(theta + eps * u, inp, target)[0]
        lm = nn.loss_and_grad(theta - eps * u, inp, target)[0]
        fd = (lp - lm) / (2 * eps)
        an = float(grad @ u)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (lo, fd, an)


def test_param_count_and_layout():
    assert nn.num_params() == sum(27 * a * b + b for a, b in nn.CONVS) + 17
    theta = np.arange(nn.num_params(), dtype=np.float64)
    assert np.array_equal(nn.pack(*nn.unpack(theta)), theta)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    th = rng.standard_normal(10)
    g = rng.standard_normal(10)
    t1, m, v = nn.adam_step(th, g, np.zeros(10), np.zeros(10), 1, lr=1e-2)
    # bias-corrected first moments equal g and g^2 after one step
    assert np.allclose(t1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    a = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nn.bf16_round(a), ref)


def test_features_hand_built_2x2x2():
    """Input channels of the network (b / s, log rho, log c2, p_prev / s, s = RMS(b)) on a
    hand-built 2x2x2 input whose values are exact: b = +-2 gives s = 2, rho = e^k, c2 = e^-k,
    p_prev = 2k."""
    k = np.arange(8, dtype=np.float64).reshape(2, 2, 2)
    b = np.where(k % 2 == 0, 2.0, -2.0)
    rho = np.exp(k)
    c2 = np.exp(-k)
    inp, s = nn.features(b, rho, c2, 2.0 * k)
    assert s == 2.0 and inp.shape == (2, 2, 2, 4)
    assert np.array_equal(inp[..., 0], np.where(k % 2 == 0, 1.0, -1.0))
    assert np.allclose(inp[..., 1], k, rtol=0, atol=1e-15)
    assert np.allclose(inp[..., 2], -k, rtol=0, atol=1e-15)
    assert np.array_equal(inp[..., 3], k)


def test_features_scale_invariance_and_mass_term():
    """Scaling b and p_prev together leaves every channel unchanged and scales s; log c2 equals
    -log(rho m) with the mass term m = 1 / (rho c2) the solver holds; b = 0 gives s = 1."""
    rng = np.random.default_rng(7)
    shape = (3, 4, 5)
    b = rng.standard_normal(shape)
    rho = rng.uniform(0.5, 30.0, shape)
    c2 = rng.uniform(1.0, 10.0, shape)
    pp = rng.standard_normal(shape)
    inp, s = nn.features(b, rho, c2, pp)
    assert np.isclose(s, np.sqrt(np.mean(b * b)), rtol=1e-15)
    inp2, s2 = nn.features(8.0 * b, rho, c2, 8.0 * pp)
    assert s2 == 8.0 * s and np.array_equal(inp2, inp)
    m = 1.0 / (rho * c2)
    assert np.allclose(inp[..., 2], -np.log(rho * m), rtol=0, atol=1e-14)
    z, s0 = nn.features(np.zeros(shape), rho, c2, np.zeros(shape))
    assert s0 == 1.0 and not np.any(z[..., 0]) and not np.any(z[..., 3])
