"""GPU checks of the learned warm start / preconditioner against the FP64 network oracle.

Forward and gradient parity use inputs and weights rounded to bfloat16 and the oracle's
bfloat16-emulating mode (it rounds activations, pooled tensors and masked gradients at the same
points as the GPU pipeline), so what remains is FP32 (MFMA) versus FP64 accumulation order plus
the rare bfloat16 rounding flips it causes: ~1e-3 relative on outputs, a few 1e-3 on gradients.
"""
import functools
import math
import os
import time

import numpy as np
import pytest

import oracle
from oracle import nn
from paper_1112_3507_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a HIP GPU")]

import paper_1112_3507_amd as hp  # noqa: E402

DEV = "cuda:0"
SHAPE = (8, 8, 16)     # (nz, ny, nx)
N3 = (16, 8, 8)        # (nx, ny, nz)


def _inputs(seed):
    rng = np.random.default_rng(seed)
    theta = (nn.init_params(seed) + 0.02 * rng.standard_normal(nn.num_params())).astype(np.float32)
    inp = nn.bf16_round(rng.standard_normal(SHAPE + (4,)))
    target = rng.standard_normal(SHAPE).astype(np.float32)
    return theta, inp, target


def _dev_inp(inp):
    x8 = np.zeros(SHAPE + (8,), dtype=np.float32)
    x8[..., :4] = inp
    return torch.from_numpy(x8).to(DEV).to(torch.bfloat16).contiguous()


def test_param_count_matches_oracle():
    assert hp.num_params() == nn.num_params()


def test_forward_parity_bf16():
    theta, inp, _ = _inputs(0)
    net = hp.Net(N3, training=False)
    net.set_params(torch.from_numpy(theta).to(DEV))
    y = torch.empty(SHAPE, dtype=torch.float32, device=DEV)
    net.forward_raw(_dev_inp(inp), y)
    torch.cuda.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    yr = nn.forward(theta.astype(np.float64), inp, bf16=True)
    err = np.linalg.norm(yg - yr) / np.linalg.norm(yr)
    assert err <= 5e-3, err
    assert np.max(np.abs(yg - yr)) <= 2e-2 * np.max(np.abs(yr))
    net.close()


def test_gradient_parity_bf16_and_adam():
    theta, inp, target = _inputs(1)
    net = hp.Net(N3, training=True)
    net.set_params(torch.from_numpy(theta).to(DEV))
    loss = net.loss_grad_raw(_dev_inp(inp), torch.from_numpy(target).to(DEV))
    g = net.get_grad().cpu().numpy().astype(np.float64)
    loss_r, g_r = nn.loss_and_grad(theta.astype(np.float64), inp, target.astype(np.float64), bf16=True)
    assert abs(loss - loss_r) <= 2e-3 * loss_r
    offs = np.cumsum([0] + [27 * a * b + b for a, b in nn.CONVS] + [17])
    for lo, hi in zip(offs[:-1], offs[1:]):
        a, b = g[lo:hi], g_r[lo:hi]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
        assert rel <= 3e-2 and cos >= 0.999, (lo, rel, cos)
    # one Adam step from zero moments with the GPU gradient
    lr = 1e-3
    net.adam(lr)
    th1 = net.get_params().cpu().numpy().astype(np.float64)
    ref, _, _ = nn.adam_step(theta.astype(np.float64), g.astype(np.float32).astype(np.float64),
                             np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert np.allclose(th1, ref, rtol=1e-5, atol=2e-8)
    net.close()


@functools.lru_cache(maxsize=None)
def _training_set(n=32, count=6):
    """FP64 MG-PCG solutions of random polytropes (index in [1, 2], contrast in [3, 30])."""
    rng = np.random.default_rng(50)
    samples = []
    for q in range(count):
        idx = rng.uniform(1.0, 2.0)
        con = rng.uniform(3.0, 30.0)
        p = wl.polytrope((n, n, n), 0.001, seed=60 + q, contrast=con, index=idx)
        b = wl.rhs_white(p.n, 70 + q)
        rho = torch.from_numpy(p.rho).to(DEV)
        c2 = torch.from_numpy(p.c2).to(DEV)
        bt = torch.from_numpy(b).to(DEV)
        x = torch.zeros_like(bt)
        with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
            st = s.solve(bt, x, tol=1e-10)
        assert st["converged"]
        samples.append((bt, rho, c2, x))
    return samples


def test_training_reduces_loss():
    torch.manual_seed(0)
    samples = _training_set()
    net = hp.Net((32, 32, 32), training=True)
    theta = nn.init_params(3).astype(np.float32)
    net.set_params(torch.from_numpy(theta).to(DEV))
    ratio = np.mean([float(x.norm() / b.norm()) for b, _, _, x in samples])
    net.set_output_scale(ratio)
    losses = []
    for step in range(90):
        b, rho, c2, x = samples[step % len(samples)]
        losses.append(net.train_step(b, rho, c2, None, x, 3e-3))
    first = np.mean(losses[:6])
    last = np.mean(losses[-6:])
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
    net.close()


def test_anorm_training_reduces_loss():
    """Training on the relative A-norm error through the solver handle lowers it."""
    n = (32, 32, 32)
    p = wl.polytrope(n, 0.001, seed=81)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    net = hp.Net(n, training=True)
    net.set_params(torch.from_numpy(nn.init_params(4).astype(np.float32)).to(DEV))
    losses = []
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        data = []
        for q in range(4):
            bt = torch.from_numpy(wl.rhs_white(n, 90 + q)).to(DEV)
            x = torch.zeros_like(bt)
            s.solve(bt, x, tol=1e-10)
            data.append((bt, x))
        for step in range(80):
            bt, x = data[step % 4]
            net.set_output_scale(float(x.norm() / bt.norm()))
            losses.append(s.train_step_anorm(net, bt, x, 2e-3))
    assert np.isfinite(losses[-1]) and np.mean(losses[-4:]) < 0.5 * np.mean(losses[:4]), losses[::10]
    net.close()


@pytest.mark.parametrize("layout", [1, 0])
def test_learned_fcg_matches_oracle(layout):
    n = (80, 24, 40)
    p = wl.polytrope(n, 0.001, seed=1)
    b = wl.rhs_white(n, 2)
    xref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    bt = torch.from_numpy(b).to(DEV)
    net = hp.Net(n, training=False)
    net.set_params(torch.from_numpy(nn.init_params(5).astype(np.float32)).to(DEV))
    net.set_output_scale(float(np.linalg.norm(xref) / np.linalg.norm(b)))
    x = torch.zeros_like(bt)
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt, hp.MODE_LEARNED) as s:
        s.set_option(hp.OPT_LAYOUT, layout)
        s.attach_net(net)
        st = s.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    assert st["converged"] and st["rel_residual"] <= 1e-10
    err = np.linalg.norm(x.cpu().numpy() - xref) / np.linalg.norm(xref)
    assert err <= 1e-9, err
    # the network's own warm start is an initial guess only: the solve still meets the bar
    x0 = torch.empty_like(bt)
    net.forward(bt, rho, c2, None, x0)
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        st = s.solve(bt, x0, tol=1e-10)
    assert st["converged"]
    assert np.linalg.norm(x0.cpu().numpy() - xref) / np.linalg.norm(xref) <= 1e-9
    net.close()


def test_network_paths_agree_across_layouts():
    """Warm start and A-norm training step give the same values with the natural and the split
    storage of the finest level (the network itself always sees natural order)."""
    n = (64, 16, 16)
    p = wl.polytrope(n, 0.001, seed=7)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    bt = torch.from_numpy(wl.rhs_white(n, 8)).to(DEV)
    theta = torch.from_numpy(nn.init_params(6).astype(np.float32)).to(DEV)
    out = {}
    for layout in (1, 0):
        net = hp.Net(n, training=True)
        net.set_params(theta)
        net.set_output_scale(1e-3)
        with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
            s.set_option(hp.OPT_LAYOUT, layout)
            x = torch.zeros_like(bt)
            assert s.solve(bt, x, tol=1e-10)["converged"]
            s.attach_net(net)
            x0 = torch.empty_like(bt)
            s.warm_start(bt, x0)
            loss = s.train_step_anorm(net, bt, x, 1e-3)
            s.attach_net(None)
        out[layout] = (x0.cpu().numpy(), loss, net.get_params().cpu().numpy())
        net.close()
    a, b = out[1], out[0]
    assert np.linalg.norm(a[0] - b[0]) <= 1e-12 * np.linalg.norm(b[0])
    assert abs(a[1] - b[1]) <= 1e-9 * abs(b[1])
    assert np.allclose(a[2], b[2], rtol=1e-5, atol=1e-9)


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1112_3507_amd", "weights", "unet128.npz")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained checkpoint")
def test_trained_network_gain():
    """What training gains, against plain MG-PCG (the method without the network): A-norm error of
    the warm start x0 = g net(b), MG-PCG iterations and time after that warm start, and learned-FCG
    iterations and time, for the trained checkpoint and the untrained (initial) network, on a
    held-out 128^3 polytrope at Ma = 0.001 with a white and a smooth right-hand side.

    A start with A-norm error e saves about ln(e) / ln(q) iterations of a CG whose error contracts
    by q per iteration (q from the plain solve: tol^(1/iterations)); the trained network's
    e ~ 0.65-0.7 is worth ~0.2 of an iteration of this V-cycle, so the warm-started solve must take
    the plain count to within one iteration. The times (each solve's own HIP-event time, the
    forward timed around its call) are printed next to the plain solve's."""
    from paper_1112_3507_amd import train as tr
    n = (128, 128, 128)
    tol = 1e-10
    p = wl.polytrope(n, 0.001, seed=424242, contrast=12.0, index=1.4)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    theta_t, scale = tr.load(WEIGHTS)
    nets = {"trained": hp.Net(n), "untrained": hp.Net(n)}
    nets["trained"].set_params(torch.from_numpy(theta_t).to(DEV))
    nets["untrained"].set_params(torch.from_numpy(tr.he_uniform(0)).to(DEV))
    for v in nets.values():
        v.set_output_scale(scale)
    report = {}
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        for kind, b in (("white", wl.rhs_white(n, 9001)), ("smooth", wl.rhs_smooth(n, 9002))):
            bt = torch.from_numpy(b).to(DEV)
            s.set_option(hp.OPT_MODE, hp.MODE_FP64_MGPCG)
            xr = torch.zeros_like(bt)
            s.solve(bt, xr, tol=1e-12)
            ax = torch.empty_like(bt)
            s.apply(0, xr, ax)
            xnorm = float(torch.dot(xr.flatten(), ax.flatten())) ** 0.5
            x = torch.zeros_like(bt)
            s.solve(bt, x, tol=tol)                   # warm-up of the timed path
            x.zero_()
            st0 = s.solve(bt, x, tol=tol)
            its0, t0 = st0["iterations"], st0["time_ms"]
            for name, net in nets.items():
                s.attach_net(net)
                x0 = torch.empty_like(bt)
                s.warm_start(bt, x0)                  # warm-up
                torch.cuda.synchronize()
                w0 = time.perf_counter()
                s.warm_start(bt, x0)
                torch.cuda.synchronize()
                t_fwd = (time.perf_counter() - w0) * 1e3
                e = x0 - xr
                s.apply(0, e, ax)
                err = float(torch.dot(e.flatten(), ax.flatten())) ** 0.5 / xnorm
                s.set_option(hp.OPT_MODE, hp.MODE_FP64_MGPCG)
                st_ws = s.solve(bt, x0, tol=tol)
                s.set_option(hp.OPT_MODE, hp.MODE_LEARNED)
                x = torch.zeros_like(bt)
                st = s.solve(bt, x, tol=tol)
                assert st_ws["converged"] and st["converged"]
                report[(kind, name)] = dict(err=err, its_ws=st_ws["iterations"], t_ws=t_fwd + st_ws["time_ms"],
                                            t_fwd=t_fwd, its_fcg=st["iterations"], t_fcg=st["time_ms"],
                                            fb=st["fallback"], its0=its0, t0=t0)
            s.attach_net(None)
    for (kind, name), r in sorted(report.items()):
        q = tol ** (1.0 / r["its0"])
        r["pred"] = math.log(r["err"]) / math.log(q)
        print("gain %s %-9s A-err %.3f (predicted saving %.2f its) | plain MG-PCG %d its %.2f ms | "
              "warm start + MG-PCG %d its (%+d) %.2f ms (x%.2f; forward %.2f ms) | learned FCG %d its (%+d) "
              "%.2f ms (x%.2f), fallback %d"
              % (kind, name, r["err"], r["pred"], r["its0"], r["t0"], r["its_ws"], r["its_ws"] - r["its0"],
                 r["t_ws"], r["t_ws"] / r["t0"], r["t_fwd"], r["its_fcg"], r["its_fcg"] - r["its0"], r["t_fcg"],
                 r["t_fcg"] / r["t0"], r["fb"]), flush=True)
    for kind in ("white", "smooth"):
        tr_, un = report[(kind, "trained")], report[(kind, "untrained")]
        assert tr_["err"] < un["err"] and tr_["err"] < 0.9
        # iteration deltas against plain MG-PCG: the warm start is worth less than one iteration
        # here, so the warm-started count stays within one of the plain count
        assert tr_["pred"] < 1.0 and abs(tr_["its_ws"] - tr_["its0"]) <= 1
        # the learned FCG converges without the fallback, within a few iterations of plain
        assert tr_["fb"] == 0 and tr_["its_fcg"] <= tr_["its0"] + 5
        # the warm-started solve pays the forward on top of about the plain solve's time
        assert tr_["t_ws"] > tr_["t_fwd"]


@pytest.mark.parametrize("with_prev", [False, True])
def test_physical_units_path_matches_oracle(with_prev):
    """hp_nn_forward and hp_warm_start in physical units against the oracle: the features
    (b/s, log rho, log c2, p_prev/s with s = RMS(b)), the bfloat16 network, the output scaling
    s * out_scale, and for the warm start the A-norm-optimal step g = <b, y> / <y, A y> with A the
    oracle's operator. 256-wide rows (the split finest level with two-wave row tiles)."""
    n = (256, 16, 16)
    p = wl.polytrope(n, 0.001, seed=31)
    rng = np.random.default_rng(32)
    b = wl.rhs_white(n, 33) * 7.5
    pp = rng.standard_normal(p.shape) * 3.0 if with_prev else np.zeros(p.shape)
    theta = (nn.init_params(9) + 0.02 * rng.standard_normal(nn.num_params())).astype(np.float32)
    out_scale = 2.5e-4
    inp, s = nn.features(b, p.rho, p.c2, pp)
    x_ref = s * out_scale * nn.forward(theta.astype(np.float64), inp, bf16=True)
    A = oracle.assemble(p.n, p.h, p.bc, p.rho, p.c2, p.dt)
    ax = A.matvec(x_ref).reshape(p.shape)
    g_ref = float(np.sum(b * x_ref) / np.sum(x_ref * ax))
    assert g_ref > 0.0

    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    bt = torch.from_numpy(b).to(DEV)
    ppt = torch.from_numpy(pp).to(DEV) if with_prev else None
    net = hp.Net(n)
    net.set_params(torch.from_numpy(theta).to(DEV))
    net.set_output_scale(out_scale)
    x = torch.empty_like(bt)
    net.forward(bt, rho, c2, ppt, x)
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as sv:
        assert sv.get_option(hp.OPT_LAYOUT) == 1
        sv.attach_net(net)
        xw = torch.empty_like(bt)
        sv.warm_start(bt, xw, p_prev=ppt)
        sv.attach_net(None)
    torch.cuda.synchronize()
    xg, xwg = x.cpu().numpy(), xw.cpu().numpy()
    err = np.linalg.norm(xg - x_ref) / np.linalg.norm(x_ref)
    # Both sides round the features, ten convolution outputs and two pooled tensors to bfloat16
    # (8-bit significand: one unit in the last place is 2^-8 = 3.9e-3 relative); FP32 (MFMA)
    # against FP64 accumulation flips a few of those roundings by one unit, which moves the
    # output by a few 1e-3 relative. The bar is four units in the last place.
    tol = 4 * 2.0 ** -8
    print("physical units (p_prev=%s): forward rel err %.2e (bar %.2e), g_ref %.4e"
          % (with_prev, err, tol, g_ref), flush=True)
    assert err <= tol, err
    # the bar separates the right features and scaling from plausible mistakes: the oracle with
    # log rho and log c2 swapped, with p_prev not divided by s, or with the output not scaled by
    # s is at least four bars away
    wrong = [inp[..., [0, 2, 1, 3]], ]
    if with_prev:
        wrong.append(np.concatenate([inp[..., :3], pp[..., None]], axis=-1))
    for wi in wrong:
        xw_ref = s * out_scale * nn.forward(theta.astype(np.float64), wi, bf16=True)
        assert np.linalg.norm(xg - xw_ref) / np.linalg.norm(x_ref) > 4 * tol
    assert abs(s - 1.0) > 0.5 and np.linalg.norm(xg - x_ref / s) / np.linalg.norm(x_ref) > 4 * tol
    werr = np.linalg.norm(xwg - g_ref * x_ref) / np.linalg.norm(g_ref * x_ref)
    assert werr <= 2 * tol, werr
    # g is the A-norm-optimal step <b, y> / <y, A y>: the GPU's agrees with the oracle's to the
    # network's own deviation, and differs by orders of magnitude from <b, y> / <y, y>
    g_gpu = float(np.sum(xwg * xg) / np.sum(xg * xg))
    assert abs(g_gpu - g_ref) <= 2 * tol * g_ref, (g_gpu, g_ref)
    g_wrong = float(np.sum(b * x_ref) / np.sum(x_ref * x_ref))
    assert abs(g_wrong - g_ref) > 10.0 * g_ref
    net.close()


def test_train_then_attach_then_learned_solve():
    """The A-norm training step may come before hp_attach_net: the learned stage's work vectors
    are then allocated by the training step, and a learned (FCG) solve on the split finest level
    afterwards meets the bar against the oracle."""
    n = (64, 16, 16)
    p = wl.polytrope(n, 0.001, seed=41)
    b = wl.rhs_white(n, 42)
    xref, _ = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    rho = torch.from_numpy(p.rho).to(DEV)
    c2 = torch.from_numpy(p.c2).to(DEV)
    bt = torch.from_numpy(b).to(DEV)
    net = hp.Net(n, training=True)
    net.set_params(torch.from_numpy(nn.init_params(10).astype(np.float32)).to(DEV))
    net.set_output_scale(float(np.linalg.norm(xref) / np.linalg.norm(b)))
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        assert s.get_option(hp.OPT_LAYOUT) == 1
        xt = torch.from_numpy(xref).to(DEV)
        loss = s.train_step_anorm(net, bt, xt, 1e-4)
        assert np.isfinite(loss)
        s.attach_net(net)
        s.set_option(hp.OPT_MODE, hp.MODE_LEARNED)
        x = torch.zeros_like(bt)
        st = s.solve(bt, x, tol=1e-10)
    torch.cuda.synchronize()
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert np.linalg.norm(x.cpu().numpy() - xref) / np.linalg.norm(xref) <= 1e-9
    net.close()


def test_checkpoint_save_load_roundtrip(tmp_path):
    """hp_nn_save / hp_nn_load: the file holds the documented layout (read back here with numpy),
    a load on a network of another grid restores the parameters and output scale exactly (the
    forwards of saver and loader agree bit for bit), and a wrong magic, a wrong count or a
    truncated file give HP_EIO and leave the network as it was."""
    theta, inp, _ = _inputs(11)
    a = hp.Net(N3, training=False)
    a.set_params(torch.from_numpy(theta).to(DEV))
    a.set_output_scale(2.5e-4)
    path = str(tmp_path / "net.ckpt")
    a.save(path)
    raw = open(path, "rb").read()
    assert raw[:8] == b"HPNET01\x00"
    count = int(np.frombuffer(raw[8:16], dtype="<i8")[0])
    scale = float(np.frombuffer(raw[16:24], dtype="<f8")[0])
    params = np.frombuffer(raw[24:], dtype="<f4")
    assert count == nn.num_params() == params.size and scale == 2.5e-4
    assert np.array_equal(params, theta)

    b = hp.Net((32, 32, 32), training=False)
    b.load(path)
    assert np.array_equal(b.get_params().cpu().numpy(), theta)
    c = hp.Net(N3, training=False)
    c.load(path)
    ya = torch.empty(SHAPE, dtype=torch.float32, device=DEV)
    yc = torch.empty_like(ya)
    a.forward_raw(_dev_inp(inp), ya)
    c.forward_raw(_dev_inp(inp), yc)
    torch.cuda.synchronize()
    assert torch.equal(ya, yc)

    before = b.get_params().cpu().numpy().copy()
    bad = {"magic": b"HPNET02\x00" + raw[8:],
           "count": raw[:8] + np.array([count - 1], dtype="<i8").tobytes() + raw[16:],
           "truncated": raw[:-4]}
    for name, blob in bad.items():
        q = tmp_path / ("bad_" + name)
        q.write_bytes(blob)
        with pytest.raises(hp.HPError) as ei:
            b.load(str(q))
        assert ei.value.code == hp.EIO, name
    with pytest.raises(hp.HPError) as ei:
        b.load(str(tmp_path / "missing"))
    assert ei.value.code == hp.EIO
    assert np.array_equal(b.get_params().cpu().numpy(), before)
    for n_ in (a, b, c):
        n_.close()


def test_network_grid_limits():
    """hp_nn_create rejects grids the convolutions cannot index (2^31 cells or more) and sizes
    that are not multiples of 4, before allocating anything."""
    for n in ((2048, 1024, 1024), (12, 8, 6), (0, 8, 8)):
        with pytest.raises(hp.HPError) as ei:
            hp.Net(n)
        assert ei.value.code == hp.EINVAL, n
