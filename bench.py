#!/usr/bin/env python3
"""Throughput of the implicit pressure solve on one MI355X.

Workload (the benchmark line's `value`): the 256^3 stratified polytropic box (T = 1 + 9z,
rho = T^1.5, c2 = T, +-1% multiplicative noise from seed 0, periodic x/y, Neumann z), Ma = 0.01
(dt = 100 h), white-noise zero-mean right-hand sides with seeds 100, 101, ..., solved from a
zero initial guess to true relative residual 1e-10 with FP64 multigrid-preconditioned CG.
One step = one solve of a fresh right-hand side; inputs are resident in HBM before timing.

Also reported on the same line: the Ma = 0.001 box with FP64 MG-PCG, the mixed-precision form
and the learned forms (speedup at the same accuracy; every timed mixed-precision solve is
compared with the FP64 solve of the same right-hand side), the roofline of the dominant kernel
(measured with HIP events on the solver's stream) beside the whole solve's fraction, and the CPU
oracle leg: the oracle timed on the host cores on a bounded sample, and its reference solution of
the first timed right-hand side at both Mach numbers, against which every form's error is stated
(computed after all timing).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pressure solves/s at 256³ to 1e-10 residual; FP64 MGPCG vs mixed/learned"
HBM_PEAK_GBS = 8000.0
TOL = 1e-10

# Algorithmic (compulsory) FP64 bytes per fine cell for one launch of each level-0 kernel:
# every array the kernel must touch is counted once.
ALG_BYTES = {
    # q = A p with <p, q>: read p, rho, m; write q
    "apply": 32.0,
    # one red-black half sweep: read rho (all cells), r, m and the other colour's z (half the
    # cells each), write this colour's z (half); the split layout of the finest level lets the
    # kernel touch only these
    "rbgs_half_sweep": 24.0,
}

# Algorithmic FP64 bytes per finest-level cell and MG-PCG iteration (every pass of the
# iteration with the arrays it must touch once): apply 32, r -= alpha q with ||r||^2 folded into
# the next zero-guess pre-smoothing 48 (read r, q, dinv, rho; write r', z), red residual 16,
# red-only restriction 5, red-only prolongation 9, black sweep 24, red sweep 24 (the two sweeps
# each reduce their own half of <r, z>), x += alpha p with p = z + beta p 40; plus the coarser
# levels (1/7 of the V-cycle's finest-level 110 bytes: 16).
ITER_BYTES_PER_CELL = 32 + 48 + 16 + 5 + 9 + 24 + 24 + 40 + 16


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_rhs(n, seeds, dev):
    import torch
    from paper_1112_3507_amd import workloads as wl
    return [torch.from_numpy(wl.rhs_white(n, s)).to(dev) for s in seeds]


def run_solves(solver, rhs, x, warmup, steps, keep=None):
    """Warm up, then time `steps` solves (each from a zero initial guess). With `keep` (a list
    of zeroed solution buffers, one per timed solve, resident before timing) every timed solve
    writes its own buffer, so the solutions can be compared afterwards; else all use x (zeroed
    inside the timed loop). Returns (seconds, stats list)."""
    import torch
    for k in range(warmup):
        x.zero_()
        solver.solve(rhs[k % len(rhs)], x, tol=TOL)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(steps):
        if keep is None:
            x.zero_()
            stats.append(solver.solve(rhs[warmup + k], x, tol=TOL))
        else:
            stats.append(solver.solve(rhs[warmup + k], keep[k], tol=TOL))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, stats


def rel_diff(a, b):
    """||a - b|| / ||b|| of two device vectors (FP64, on the GPU)."""
    return float((a - b).norm() / b.norm())


def kernel_time_ms(fn, reps=50):
    """Average duration of one launch of fn() on the current stream, timed with HIP events."""
    import torch
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline(solver, rhs, x, n_cells, dev, warmup):
    """Roofline of the dominant finest-level kernel, measured live: the solver's own HIP-event
    timing (on its stream; the events are attached to the dispatches themselves) of every CG
    operator apply and every post-smoothing half sweep on the finest level inside FP64 solves of
    the benchmark's right-hand sides; the library's streaming copy of 1 GiB (beyond the 256 MB
    last-level cache) as the measured streaming reference."""
    import torch
    import paper_1112_3507_amd as hp
    solver.set_option(hp.OPT_KERNEL_TIMING, 1)
    acc = {"rbgs_half_sweep": [0.0, 0], "apply": [0.0, 0]}
    for k in range(len(rhs) - warmup):
        x.zero_()
        st = solver.solve(rhs[warmup + k], x, tol=TOL)
        acc["rbgs_half_sweep"][0] += st["sweep_ms"] * st["timed_sweeps"]
        acc["rbgs_half_sweep"][1] += st["timed_sweeps"]
        acc["apply"][0] += st["apply_ms"] * st["timed_applies"]
        acc["apply"][1] += st["timed_applies"]
    solver.set_option(hp.OPT_KERNEL_TIMING, 0)
    times = {k: v[0] / max(v[1], 1) for k, v in acc.items()}
    src = torch.rand(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    # the library's streaming copy (16-byte non-temporal loads and stores), 1 GiB each way
    copy_ms = kernel_time_ms(lambda: hp.stream_copy(src, dst), reps=20)
    assert torch.equal(src, dst)
    del src, dst
    # the dominant kernel takes the largest share of the solve: the half sweep (two launches per
    # CG iteration, the kernel with the largest total time in the rocprofv3 summary) ahead of the
    # apply (one launch)
    dom = max(acc, key=lambda k: acc[k][0])
    gbs = ALG_BYTES[dom] * n_cells / (times[dom] * 1e-3) / 1e9
    kern = {k: {"ms": round(v, 5), "launches_timed": acc[k][1], "alg_bytes_per_cell": ALG_BYTES[k],
                "achieved_GBs": round(ALG_BYTES[k] * n_cells / (v * 1e-3) / 1e9, 1) if v > 0 else None}
            for k, v in times.items()}
    copy_gbs = 2.0 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    return {"kernel": dom, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(dom, n_cells),
            "per_launch_ms": round(times[dom], 5), "kernels": kern,
            "copy_reference": {"bytes": 2 * (1 << 30), "ms": round(copy_ms, 5), "GBs": round(copy_gbs, 1),
                               "frac_of_copy": round(gbs / copy_gbs, 4)}}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_256cube.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1112_3507_amd", "csrc", "hp_kernels.hip")


def measured_traffic(kernel, n_cells):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a plain copy of known size), or
    None when there is none for this size or the kernel source changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_FILE):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(TRAFFIC_FILE).read(), re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if d.get("n_cells") != n_cells or d.get("kernels_source_sha256") != sha:
        return None
    return d.get("per_launch_bytes", {}).get(kernel)


def learned_leg(p3, rho3, c23, rhs, x, W, K, dev, base, sols):
    """The trained network at 256^3, Ma = 0.001: (a) warm start x0 = g net(b) followed by FP64
    MG-PCG, timed including the network; (b) flexible CG with the network + V-cycle
    preconditioner. Both stop on the same FP64 true residual 1e-10. The solution of the first
    timed solve of each form goes into sols (for its error against the oracle)."""
    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import train as tr
    path = os.path.join(ROOT, "paper_1112_3507_amd", "weights", "unet128.npz")
    if not os.path.exists(path):
        return None
    theta, scale = tr.load(path)
    net = hp.Net(p3.n)
    net.set_params(torch.from_numpy(theta).to(dev))
    net.set_output_scale(scale)
    out = {}
    s = hp.setup(p3.n, p3.h, p3.bc, rho3, c23, p3.dt, hp.MODE_FP64_MGPCG)
    s.attach_net(net)
    first = torch.zeros_like(x)
    for name in ("warm_start", "fcg"):
        log("bench: Ma=0.001 learned %s" % name)
        if name == "fcg":
            s.set_option(hp.OPT_MODE, hp.MODE_LEARNED)
        stats = []
        first.zero_()
        for k in range(W + K):
            if k == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            xk = first if k == W else x
            if name == "warm_start":
                s.warm_start(rhs[k], xk)
            elif k != W:
                x.zero_()
            st = s.solve(rhs[k], xk, tol=TOL)
            if k >= W:
                stats.append(st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        sols["learned_" + name] = first.clone()
        v = K / secs
        out[name] = {"value": round(v, 3), "unit": "solves/s", "ms_per_step": round(1e3 * secs / K, 4),
                     "iterations_mean": sum(q["iterations"] for q in stats) / K,
                     "fallbacks": sum(q["fallback"] for q in stats),
                     "max_rel_residual": max(q["rel_residual"] for q in stats),
                     "all_converged": all(q["converged"] for q in stats),
                     "speedup_vs_fp64_mgpcg": round(v / base, 3)}
    out.update(previous_pressure_leg(s, rhs, x, W, K, base))
    s.close()
    net.close()
    out["training"] = training_leg(dev)
    return out


def previous_pressure_leg(s, rhs, x, W, K, base):
    """With a previous pressure, the network's fourth input (the case a time step gives): p_prev
    is the FP64 solution for the rhs plus 10% white noise (the perturbation the training samples
    use), computed outside the timed region. Plain FP64 MG-PCG started from p_prev against the
    warm start x0 = g net(b, p_prev) followed by FP64 MG-PCG; both to the same true residual."""
    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import workloads as wl
    s.set_option(hp.OPT_MODE, hp.MODE_FP64_MGPCG)
    log("bench: Ma=0.001 previous-pressure inputs")
    prevs = []
    for k in range(W + K):
        noise = torch.from_numpy(wl.rhs_white(tuple(s.n), 5000 + k)).to(x.device)
        bp = rhs[k] + 0.1 * (rhs[k].norm() / noise.norm()) * noise
        pk = torch.zeros_like(x)
        s.solve(bp, pk, tol=TOL)
        prevs.append(pk)
    out = {}
    for name in ("prev_plain", "prev_warm_start"):
        log("bench: Ma=0.001 %s" % name)
        stats = []
        for k in range(W + K):
            if k == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if name == "prev_plain":
                x.copy_(prevs[k])
            else:
                s.warm_start(rhs[k], x, p_prev=prevs[k])
            st = s.solve(rhs[k], x, tol=TOL)
            if k >= W:
                stats.append(st)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        v = K / secs
        out[name] = {"value": round(v, 3), "unit": "solves/s", "ms_per_step": round(1e3 * secs / K, 4),
                     "iterations_mean": sum(q["iterations"] for q in stats) / K,
                     "max_rel_residual": max(q["rel_residual"] for q in stats),
                     "all_converged": all(q["converged"] for q in stats),
                     "speedup_vs_fp64_mgpcg": round(v / base, 3)}
    out["prev_warm_start"]["speedup_vs_prev_plain"] = round(out["prev_warm_start"]["value"] /
                                                            out["prev_plain"]["value"], 3)
    del prevs
    return out


def training_leg(dev, steps=10):
    """One step of the A-norm training (network forward, loss through the solver's operator,
    backward, Adam) on a 128^3 polytrope sample, as the training driver runs it."""
    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import train as tr
    from paper_1112_3507_amd import workloads as wl
    p = wl.polytrope((128, 128, 128), 0.001, seed=12345, contrast=12.0, index=1.4)
    rho, c2 = torch.from_numpy(p.rho).to(dev), torch.from_numpy(p.c2).to(dev)
    b = torch.from_numpy(wl.rhs_white(p.n, 12346)).to(dev)
    x = torch.zeros_like(b)
    net = hp.Net(p.n, training=True)
    net.set_params(torch.from_numpy(tr.he_uniform(0)).to(dev))
    with hp.setup(p.n, p.h, p.bc, rho, c2, p.dt) as s:
        s.solve(b, x, tol=TOL)
        net.set_output_scale(float(x.norm() / b.norm()))
        for _ in range(2):
            s.train_step_anorm(net, b, x, 1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.train_step_anorm(net, b, x, 1e-4)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
    net.close()
    return {"grid": [128, 128, 128], "ms_per_step": round(ms, 3), "steps_timed": steps}


def semiconvection_leg(dev, steps=20, seed=7, n=(1024, 1024, 512)):
    """The two-component sequence: the 1024 x 1024 x 512 box [0,2]^2 x [0,1] (h = 1/512), T = 1 + 9z,
    the mean-molecular-weight step mu(z), rho = T^1.5 mu (1 +- 1%), c2 = (T / mu)(1 +- 1%) (seed 7),
    Ma = 0.001, and `steps` consecutive solves whose coefficients are carried one step further
    each time by a seeded divergence-free horizontal velocity (|u|max = Ma, one cell per step,
    semi-Lagrangian bilinear interpolation, periodic in x and y). Solve n: rhs m_n p_{n-1} - dt D_n
    (D a seeded zero-mean field carried along; p is the pressure perturbation about the hydrostatic
    background, p_0 = 0), from p_{n-1}; the coefficient update (hp_update_coefficients) and the
    solve are timed per step, for the mixed-precision form and for FP64 MG-PCG (iteration cap 300).
    Input generation (the advection) is plain torch arithmetic outside the timing."""
    import numpy as np
    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import workloads as wl
    nx, ny, nz = n
    log("bench: semiconvection inputs %s" % (n,))
    p = wl.polytrope(n, 0.001, seed=seed, mu=wl.semiconvection_mu)
    h, dt = p.h[0], p.dt
    rho0 = torch.from_numpy(p.rho).to(dev)
    c20 = torch.from_numpy(p.c2).to(dev)
    del p
    z = (torch.arange(nz, device=dev, dtype=torch.float64) + 0.5) * h
    rng = np.random.default_rng(seed + 1)
    D0 = torch.from_numpy(rng.standard_normal((nz, ny, nx))).to(dev)
    D0 -= D0.mean()
    # streamfunction psi = g(z) sum_q a_q cos(2 pi (kx x + ky y) / 2 + phi_q): u = (d psi/dy, -d psi/dx, 0)
    x = (torch.arange(nx, device=dev, dtype=torch.float64) + 0.5) * h
    y = (torch.arange(ny, device=dev, dtype=torch.float64) + 0.5) * h
    ux = torch.zeros((ny, nx), device=dev, dtype=torch.float64)
    uy = torch.zeros_like(ux)
    for _ in range(6):
        kx, ky = rng.integers(-2, 3, size=2)
        if kx == 0 and ky == 0:
            kx = 1
        a, ph = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
        arg = 2 * np.pi * (kx * x[None, :] + ky * y[:, None]) / 2.0 + ph
        ux += -a * np.pi * ky * torch.sin(arg)
        uy += a * np.pi * kx * torch.sin(arg)
    gz = 1.0 + 0.5 * torch.cos(np.pi * z)
    scale = 0.001 / float(torch.sqrt(ux * ux + uy * uy).max() * gz.max())
    # departure points in cell units, their cells and bilinear weights (the velocity is steady)
    sx = (ux[None] * gz[:, None, None] * (scale * dt / h))
    sy = (uy[None] * gz[:, None, None] * (scale * dt / h))
    del ux, uy
    ii = torch.arange(nx, device=dev, dtype=torch.float64).view(1, 1, nx)
    jj = torch.arange(ny, device=dev, dtype=torch.float64).view(1, ny, 1)
    xd, yd = ii - sx, jj - sy
    del sx, sy
    fx, fy = torch.floor(xd), torch.floor(yd)
    wx, wy = xd - fx, yd - fy
    del xd, yd
    i0 = torch.remainder(fx.long(), nx)
    j0 = torch.remainder(fy.long(), ny)
    del fx, fy
    kk = (torch.arange(nz, device=dev, dtype=torch.int64) * (nx * ny)).view(nz, 1, 1)
    r0 = kk + j0 * nx
    r1 = kk + torch.remainder(j0 + 1, ny) * nx
    c1 = torch.remainder(i0 + 1, nx)
    taps = (r0 + i0, r0 + c1, r1 + i0, r1 + c1)
    del r0, r1, c1, j0, i0, kk

    def advect(f):
        v = f.view(-1)
        a = torch.take(v, taps[0]) * (1 - wx) + torch.take(v, taps[1]) * wx
        b = torch.take(v, taps[2]) * (1 - wx) + torch.take(v, taps[3]) * wx
        return a * (1 - wy) + b * wy

    out = {}
    for name, mode in (("mixed_ir", hp.MODE_MIXED_IR), ("fp64_mgpcg", hp.MODE_FP64_MGPCG)):
        log("bench: semiconvection %s, %d steps" % (name, steps))
        rho, c2, D = rho0.clone(), c20.clone(), D0.clone()
        x = torch.zeros_like(rho0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = hp.setup(n, (h, h, h), (hp.PERIODIC, hp.PERIODIC, hp.NEUMANN), rho, c2, dt, mode)
        s.set_option(hp.OPT_MAX_ITER, 300)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0)
        upd, sol, its, res, conv = [], [], [], [], []
        for step in range(steps):
            rho, c2, D = advect(rho), advect(c2), advect(D)
            b = x / (rho * c2) - dt * D
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.update_coefficients(rho, c2, dt)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = s.solve(b, x, tol=TOL, check=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            upd.append(1e3 * (t1 - t0))
            sol.append(1e3 * (t2 - t1))
            its.append(st["iterations"])
            res.append(st["rel_residual"])
            conv.append(bool(st["converged"]))
            log("bench: semiconvection %s step %d: update %.1f ms, solve %.1f ms, %d iterations, "
                "residual %.2e" % (name, step, upd[-1], sol[-1], its[-1], res[-1]))
            del b
        s.close()
        per = [a + b for a, b in zip(upd, sol)]
        out[name] = {"solves_per_s_incl_update": round(1e3 * steps / sum(per), 3),
                     "update_ms_median": round(sorted(upd)[steps // 2], 3),
                     "solve_ms_median": round(sorted(sol)[steps // 2], 3),
                     "setup_ms": round(setup_ms, 1), "iterations": its,
                     "max_rel_residual": max(res), "all_converged": all(conv)}
        del rho, c2, D, x
    out["grid"] = list(n)
    out["steps"] = steps
    out["speedup_mixed_vs_fp64"] = round(out["mixed_ir"]["solves_per_s_incl_update"]
                                         / out["fp64_mgpcg"]["solves_per_s_incl_update"], 3)
    return out


def gresho_leg(dev, n=256, steps=100):
    """The Gresho-vortex Mach ladder of Section 5 with the semi-implicit GPU stepper (TVD-RK2,
    the whole fractional step in each stage, hp_advect + hp_pressure_rhs + two-density solve +
    hp_pressure_update + EOS): kinetic energy after `steps` steps relative to the start, time per
    step and solve iterations, for (a) one common time step (the sound-speed step of Ma = 0.1:
    acoustic Courant numbers 0.5, 4.5, 45), (b) each Mach number's own sound-speed step (Courant
    number 0.5, the paper's setting), (c) Ma = 0.001 at four times its sound-speed step."""
    import numpy as np
    import torch
    from paper_1112_3507_amd import workloads as wl
    from paper_1112_3507_amd.stepper import SemiImplicitStepper
    gamma = 5.0 / 3.0

    def sound_dt(mach, cfl=0.5):
        prob, rho, mom, e, P = wl.gresho(n, mach)
        c = np.sqrt(gamma * P / rho).max()
        umax = np.sqrt(np.sum(mom * mom, axis=0)).max() / rho.min()
        return cfl * prob.h[0] / (umax + c)

    def run(mach, dt):
        prob, rho, mom, e, _ = wl.gresho(n, mach)
        ke0 = 0.5 * float(np.sum(np.sum(mom * mom, axis=0) / rho))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        st = SemiImplicitStepper(prob.n, prob.h, prob.bc, dt, gamma, t(rho), t(mom), t(e))
        st.step()                      # warm-up step (not timed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps - 1):
            st.step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / (steps - 1)
        ke = 0.5 * float(torch.sum(torch.sum(st.mom * st.mom, dim=0) / st.rho))
        its = [q["iterations"] for q in st.stats]
        ok = all(q["converged"] for q in st.stats)
        st.close()
        return {"dt": dt, "ke_ratio": ke / ke0, "ms_per_step": round(ms, 3),
                "iterations_mean": round(sum(its) / len(its), 2), "all_converged": ok}

    out = {"grid": [n, n], "steps": steps}
    dtc = sound_dt(0.1)
    for mach in (0.1, 0.01, 0.001):
        log("bench: gresho Ma=%g" % mach)
        out["common_dt_Ma%g" % mach] = run(mach, dtc)
        out["sound_dt_Ma%g" % mach] = run(mach, sound_dt(mach))
    out["sound_dt_x4_Ma0.001"] = run(0.001, 4 * sound_dt(0.001))
    ks = [out["common_dt_Ma%g" % m]["ke_ratio"] for m in (0.1, 0.01, 0.001)]
    out["common_dt_ke_ratio_spread"] = max(ks) - min(ks)
    return out


def host_cpu():
    """CPU model name and the number of host threads the process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(p, b, n, mach, budget_s=15.0):
    """The FP64 oracle (CSR Jacobi-PCG) on the host cores, on a bounded sample of iterations.

    The sample is scaled to solves/s by the iteration count of the oracle's full solve of the
    same input, recorded by oracle/full_size_iterations.py.
    """
    import oracle
    path = os.path.join(ROOT, "oracle", "full_size_iterations.json")
    rows = json.load(open(path)) if os.path.exists(path) else []
    full = [r["iterations"] for r in rows if r["n"] == n and r["mach"] == mach]
    if not full:
        return None
    full_iterations = full[0]
    A = oracle.assemble(p.n, p.h, p.bc, p.rho, p.c2, p.dt)
    oracle.pcg_fixed(A, b, 2)
    t0 = time.perf_counter()
    oracle.pcg_fixed(A, b, 5)
    per_it = (time.perf_counter() - t0) / 5
    k = max(5, min(400, int(budget_s / max(per_it, 1e-6))))
    t0 = time.perf_counter()
    oracle.pcg_fixed(A, b, k)
    per_it = (time.perf_counter() - t0) / k
    model, nproc = host_cpu()
    return {"value": 1.0 / (per_it * full_iterations), "unit": "solves/s",
            "cores": oracle.max_threads(), "kind": "oracle",
            "cpu_model": model, "nproc": nproc,
            "sample": "%d Jacobi-PCG iterations of the CPU oracle on the same 256^3 input "
                      "(%.3f s/iteration), scaled by the %d iterations its full solve to 1e-10 "
                      "takes" % (k, per_it, full_iterations)}


def oracle_errors(p, b, sols):
    """Part of the CPU-oracle leg: the oracle's reference solution (Jacobi-PCG to a true
    relative residual of 1e-13) of one timed right-hand side, and each GPU form's relative L2
    and max-abs error against it. sols maps a form's name to its solution of b (device)."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    xref, st = oracle.reference_solve(p.n, p.h, p.bc, p.rho, p.c2, p.dt, b)
    out = {"reference": {"iterations": st["iterations"], "rel_residual": st["rel_residual"],
                         "seconds": round(time.perf_counter() - t0, 1)}}
    xn = float(np.linalg.norm(xref))
    xm = float(np.max(np.abs(xref)))
    for name, xg in sols.items():
        d = xg.detach().cpu().numpy().reshape(xref.shape) - xref
        out[name] = {"rel_l2": float(np.linalg.norm(d)) / xn, "max_abs_rel": float(np.max(np.abs(d))) / xm}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-variants", action="store_true", help="skip the Ma=0.001 forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-semiconvection", action="store_true",
                    help="skip the 1024x1024x512 two-component sequence")
    ap.add_argument("--no-gresho", action="store_true", help="skip the Gresho-vortex Mach ladder")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1112_3507_amd as hp
    from paper_1112_3507_amd import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = (args.n, args.n, args.n)
    K, W = args.steps, args.warmup
    seeds = list(range(100, 100 + W + K))

    log("bench: generating %s inputs" % (n,))
    p = wl.config1(mach=0.01, n=args.n)
    rhs = make_rhs(n, seeds, dev)
    x = torch.zeros(p.shape, dtype=torch.float64, device=dev)
    rho, c2 = torch.from_numpy(p.rho).to(dev), torch.from_numpy(p.c2).to(dev)

    log("bench: FP64 MG-PCG, Ma=0.01, %d warmup + %d timed solves" % (W, K))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver = hp.setup(p.n, p.h, p.bc, rho, c2, p.dt, hp.MODE_FP64_MGPCG)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    keep = [torch.zeros_like(x) for _ in range(K)]
    secs, stats = run_solves(solver, rhs, x, W, K, keep)
    sols01 = {"fp64_mgpcg": keep[0].clone()}
    del keep
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.update_coefficients(rho, c2, p.dt)
    torch.cuda.synchronize()
    update_ms = 1e3 * (time.perf_counter() - t0)
    value = K / secs
    its = [s["iterations"] for s in stats]
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(1e3 * secs / K, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "polytrope %dx%dx%d Ma=0.01 FP64 MG-PCG, tol 1e-10 true relative "
                               "residual, rho/c2 noise seed 0, rhs seeds %d-%d"
                               % (args.n, args.n, args.n, seeds[W], seeds[-1]),
                   "grid": list(n), "mach": 0.01, "tol": TOL, "mode": "fp64_mgpcg"},
        "iterations_mean": sum(its) / len(its),
        "solve_ms_median": round(sorted(s["time_ms"] for s in stats)[len(stats) // 2], 4),
        "solve_ms_min": round(min(s["time_ms"] for s in stats), 4),
        "setup_ms": round(setup_ms, 2), "update_coefficients_ms": round(update_ms, 2),
        "max_rel_residual": max(s["rel_residual"] for s in stats),
        "all_converged": all(s["converged"] for s in stats),
    }
    log("bench: %.2f solves/s, %.1f iterations/solve" % (value, result["iterations_mean"]))

    per_iter_bytes = ITER_BYTES_PER_CELL * p.ncells
    eff = per_iter_bytes * result["iterations_mean"] / (secs / K) / 1e9
    result["mgpcg_effective"] = {
        "bytes_per_cell_iteration": ITER_BYTES_PER_CELL, "GBs": round(eff, 1),
        "frac_of_peak": round(eff / HBM_PEAK_GBS, 4),
        "note": "whole-solve algorithmic bytes (model) / wall time per solve"}
    if not args.no_roofline:
        result["roofline"] = roofline(solver, rhs, x, p.ncells, dev, W)
        # the kernel figure is cache-assisted (it reads what the previous pass left in the
        # 256 MB memory-side cache); the whole solve's fraction is stated beside it
        result["roofline"]["whole_solve_frac"] = result["mgpcg_effective"]["frac_of_peak"]
        result["roofline"]["cache_assisted"] = result["roofline"]["copy_reference"]["frac_of_copy"] > 1.0
        log("bench: roofline %s" % json.dumps(result["roofline"]))
    solver.close()

    sols001 = {}
    if not args.no_variants:
        p3 = wl.config1(mach=0.001, n=args.n)
        rho3, c23 = torch.from_numpy(p3.rho).to(dev), torch.from_numpy(p3.c2).to(dev)
        var = {}
        base = None
        kept = {}
        for name, mode in (("fp64_mgpcg", hp.MODE_FP64_MGPCG), ("mixed_ir", hp.MODE_MIXED_IR)):
            log("bench: Ma=0.001 %s" % name)
            s3 = hp.setup(p3.n, p3.h, p3.bc, rho3, c23, p3.dt, mode)
            keep = [torch.zeros_like(x) for _ in range(K)]
            secs3, st3 = run_solves(s3, rhs, x, W, K, keep)
            s3.close()
            kept[name] = keep
            sols001[name] = keep[0]
            v = K / secs3
            var[name] = {"value": round(v, 3), "unit": "solves/s",
                         "ms_per_step": round(1e3 * secs3 / K, 4),
                         "iterations_mean": sum(s["iterations"] for s in st3) / K,
                         "outer_mean": sum(s["outer_iterations"] for s in st3) / K,
                         "max_rel_residual": max(s["rel_residual"] for s in st3),
                         "all_converged": all(s["converged"] for s in st3)}
            if base is None:
                base = v
            var[name]["speedup_vs_fp64_mgpcg"] = round(v / base, 3)
        # every timed mixed-precision solve against the FP64 solve of the same right-hand side
        diffs = [rel_diff(a, b) for a, b in zip(kept["mixed_ir"], kept["fp64_mgpcg"])]
        var["mixed_ir"]["rel_l2_vs_fp64_per_solve"] = [float("%.3e" % d) for d in diffs]
        var["mixed_ir"]["max_rel_l2_vs_fp64"] = max(diffs)
        sols001 = {k: v.clone() for k, v in sols001.items()}
        del kept, keep
        result["ma0.001"] = var
        lv = learned_leg(p3, rho3, c23, rhs, x, W, K, dev, base, sols001)
        if lv is not None:
            var["learned_warm_start"] = lv["warm_start"]
            var["learned_fcg"] = lv["fcg"]
            var["from_previous_pressure"] = {"plain": lv["prev_plain"],
                                             "learned_warm_start": lv["prev_warm_start"]}
            result["learned_training"] = lv["training"]
        del rho3, c23

    if not args.no_gresho:
        result["gresho_ladder"] = gresho_leg(dev)

    if not args.no_semiconvection:
        result["semiconvection_1024x1024x512"] = semiconvection_leg(dev)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        from paper_1112_3507_amd import workloads as wl2
        b0 = wl2.rhs_white(n, seeds[W])
        result["cpu_baseline"] = cpu_baseline(p, b0, args.n, 0.01)
        # the oracle's reference solutions of the first timed right-hand side: error of every
        # form against the FP64 oracle (computed after all timing)
        log("bench: oracle reference, Ma=0.01")
        errs = {"rhs_seed": seeds[W], "ma0.01": oracle_errors(p, b0, sols01)}
        if sols001:
            log("bench: oracle reference, Ma=0.001")
            errs["ma0.001"] = oracle_errors(wl.config1(mach=0.001, n=args.n), b0, sols001)
        result["err_vs_oracle"] = errs
        result["err_vs_oracle_max"] = max(v["rel_l2"] for m in ("ma0.01", "ma0.001") if m in errs
                                          for k, v in errs[m].items() if k != "reference")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
