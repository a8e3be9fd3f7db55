"""A whole semi-implicit time step of the fractional-step scheme (FP64, NumPy): the explicit
advective part, the pressure solve and the updates, for inviscid single-component flow.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2 ("The Algorithm", steps (i)-(x)) written out for the inviscid equations of the paper's
Gresho-vortex test (Section 5): conserved variables rho, rho u (stacked (3, nz, ny, nx)) and the
total energy e; ideal gas P = (gamma - 1)(e - rho |u|^2 / 2), c_s^2 = gamma P / rho.

  (i)   interface velocities u_{i+1/2} from eq. step1;
  (ii)  the modified advective flux of every conserved q is q_face * u_{i+1/2}, with q_face
        reconstructed componentwise on the upwind side of the interface (the eigenvalues of the
        advective Jacobian all equal u, so the characteristic projection is the identity):
        second-order ENO, q_i + D/2 from the left cell with D the smaller in magnitude of
        q_i - q_{i-1} and q_{i+1} - q_i (ties take the second), mirrored for the right cell;
  (iii) rho^{n+1}, (rho u)*, e* = q^n - dt * div(flux);
  (iv)-(ix) the rhs, solve and updates of ``oracle.hydro`` with the two-density operator
        (rho^n and c_s^2 at time n in the mass term, rho^{n+1} in the faces);
  (x)   P^{n+1} from the equation of state.

Time integration: the second-order TVD Runge-Kutta scheme with the whole fractional step in
each stage (the variant the paper uses): U1 = L(U^n), U^{n+1} = (U^n + L(U1)) / 2.

Readings: at a closed boundary the interface velocity is zero and the reconstruction mirrors the
edge cell (zero gradient); periodic axes wrap; axes of one cell carry no flux. The paper uses
fifth-order WENO for step (ii); second-order ENO is the minimal member of the same family.
"""
from __future__ import annotations

import numpy as np

from . import hydro, reference_solve

PERIODIC = 0
NEUMANN = 1
_AX = {0: 2, 1: 1, 2: 0}


def _shift(a, d, s, bc):
    """a at the neighbour s cells away along axis d (s = +-1, +-2); periodic wrap, or the edge
    cell repeated beyond a closed boundary (mirror of a zero-gradient field)."""
    ax = _AX[d]
    if bc[d] == PERIODIC:
        return np.roll(a, -s, axis=ax)
    n = a.shape[ax]
    idx = np.clip(np.arange(n) + s, 0, n - 1)
    return np.take(a, idx, axis=ax)


def _eno_slope(dm, dp):
    """The smaller in magnitude of two one-sided differences (second-order ENO)."""
    return np.where(np.abs(dm) < np.abs(dp), dm, dp)


def eno2_face(q, uf, d, bc):
    """q at the high interface of every cell along axis d, reconstructed on the upwind side of the
    interface velocity uf (uf >= 0: the cell itself, else its high neighbour)."""
    qm, qp, qpp = _shift(q, d, -1, bc), _shift(q, d, 1, bc), _shift(q, d, 2, bc)
    left = q + 0.5 * _eno_slope(q - qm, qp - q)
    right = qp - 0.5 * _eno_slope(qp - q, qpp - qp)
    return np.where(uf >= 0.0, left, right)


def advect(n, h, bc, dt, rho, mom, e):
    """Steps (i)-(iii): returns rho^{n+1}, (rho u)*, e*."""
    qs = [rho, mom[0], mom[1], mom[2], e]
    out = [q.copy() for q in qs]
    for d in range(3):
        if n[d] == 1:
            continue
        uf = hydro.interface_velocity(mom[d], rho, d, bc)
        for q, o in zip(qs, out):
            flux = uf * eno2_face(q, uf, d, bc)
            lo = np.roll(flux, 1, axis=_AX[d])
            if bc[d] == NEUMANN:
                idx = [slice(None)] * 3
                idx[_AX[d]] = 0
                lo[tuple(idx)] = 0.0
            o -= dt * (flux - lo) / h[d]
    return out[0], np.stack(out[1:4]), out[4]


def eos(rho, mom, e, gamma):
    """Ideal gas: P = (gamma - 1)(e - |rho u|^2 / (2 rho)) and c_s^2 = gamma P / rho."""
    p = (gamma - 1.0) * (e - 0.5 * np.sum(mom * mom, axis=0) / rho)
    return p, gamma * p / rho


def fractional_step(n, h, bc, dt, gamma, rho, mom, e, tol=1e-13):
    """L(U): one whole fractional step (i)-(x) from (rho, rho u, e); returns the new state and the
    solve's statistics."""
    p, c2 = eos(rho, mom, e, gamma)
    rho1, mom_s, e_s = advect(n, h, bc, dt, rho, mom, e)
    b = hydro.pressure_rhs(n, h, bc, dt, rho, c2, p, mom, rho1, mom_s)
    x, st = reference_solve(n, h, bc, rho, c2, dt, b, rho_face=rho1)
    mom1, _, e1 = hydro.pressure_update(n, h, bc, dt, x.reshape(rho.shape), rho1, mom_s, e_s)
    return rho1, mom1, e1, st


def rk2_step(n, h, bc, dt, gamma, rho, mom, e):
    """One time step of the TVD Runge-Kutta scheme of second order with the whole fractional step
    in each stage."""
    r1, m1, e1, _ = fractional_step(n, h, bc, dt, gamma, rho, mom, e)
    r2, m2, e2, _ = fractional_step(n, h, bc, dt, gamma, r1, m1, e1)
    return 0.5 * (rho + r2), 0.5 * (mom + m2), 0.5 * (e + e2)


def kinetic_energy(rho, mom):
    return float(0.5 * np.sum(np.sum(mom * mom, axis=0) / rho))
