"""The steps of the fractional-step algorithm either side of the pressure solve (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 2, "The Algorithm", written out step by step on the cell-centred grid of the solve
(arrays shaped (nz, ny, nx), axis order of n / h / bc is (x, y, z); 0 = periodic, 1 = closed
(Neumann) boundary). Momentum arrays are stacked (3, nz, ny, nx): x, y and z components.

Before the solve (steps (iv)-(v)):
  * the pressure at a cell interface (eq. pbnd): P_{i+1/2} = (P_{i+1} rho_i + P_i rho_{i+1}) /
    (rho_i + rho_{i+1});
  * the cell gradient (eq. nablaP): (grad P)_i = (P_{i+1/2} - P_{i-1/2}) / h;
  * the interface velocity (eq. step1, applied to u* = (rho u)* / rho^{n+1} as step (iv) says):
    u_{i+1/2} = ((rho u)_i + (rho u)_{i+1}) / (rho_i + rho_{i+1}), and its divergence by the
    same central difference;
  * the right-hand side f of eq. fpoiss (one component) or eq. fpoiss2 (two components), here
    multiplied by dt^2 like the operator (b = dt^2 f):
        b = m (P^n - dt u^n . grad P^n) - dt div u* - (2 dt / 3) (m / rho^n) G
            - (3 dt / 4) m R_gas T^n div(rho^n kappa_c grad c^n),
    m = 1 / (rho^n c2^n), u^n = (rho u)^n / rho^n, G = u.div(tau) - div(u.tau) + div(K grad T)
    (the viscous and heat-conduction group of the explicit part, given per cell).

After the solve (steps (vii)-(ix)), with the predicted pressure P (the solution):
  * momentum (eq. momupdate): (rho u)^{n+1} = (rho u)* - dt grad P, grad P by eqs. pbnd and
    nablaP with rho^{n+1};
  * interface velocity (step (viii)): u^{n+1}_{i+1/2} = u*_{i+1/2}
        - dt (P_{i+1} - P_i) / h * 2 / (rho^{n+1}_{i+1} + rho^{n+1}_i);
  * energy (eq. enupdate, step (ix)): e^{n+1} = e* - dt (P div u^{n+1} + u^{n+1} . grad P), the
    divergence from the new interface velocities, u^{n+1} = (rho u)^{n+1} / rho^{n+1} at the cell.

Readings where the paper is silent (the same on the GPU): at a closed boundary the interface
velocity is zero (no flow through the wall) and the interface pressure is the adjacent cell's
(zero normal gradient, eq. vonNeumannBC); periodic axes wrap; an axis of one cell contributes no
gradient or divergence. The interface value of rho^n kappa_c in div(rho kappa_c grad c) is the
arithmetic mean of the two cells, with zero flux through closed boundaries. The returned
interface velocities are those on the high side of each cell along each axis (zero at a closed
high end).
"""
from __future__ import annotations

import numpy as np

PERIODIC = 0
NEUMANN = 1

# array axis of grid axis d (arrays are (nz, ny, nx))
_AX = {0: 2, 1: 1, 2: 0}


def _plus(a, d):
    """a at the neighbour on the high side along grid axis d (wrapped)."""
    return np.roll(a, -1, axis=_AX[d])


def _high_end_mask(shape, d):
    """True on the cells whose high side along grid axis d is the boundary."""
    m = np.zeros(shape, dtype=bool)
    idx = [slice(None)] * 3
    idx[_AX[d]] = -1
    m[tuple(idx)] = True
    return m


def _low_end_mask(shape, d):
    m = np.zeros(shape, dtype=bool)
    idx = [slice(None)] * 3
    idx[_AX[d]] = 0
    m[tuple(idx)] = True
    return m


def interface_pressure(P, rho, d, bc):
    """P at the high interface of every cell along axis d (eq. pbnd); at a closed high end the
    cell's own value (zero normal gradient)."""
    Pp, rp = _plus(P, d), _plus(rho, d)
    face = (Pp * rho + P * rp) / (rho + rp)
    if bc[d] == NEUMANN:
        face = np.where(_high_end_mask(P.shape, d), P, face)
    return face


def _low_interface(face_high, own, d, bc):
    """The interface on the low side of each cell: its low neighbour's high interface; at a
    closed low end `own` (the boundary value)."""
    low = np.roll(face_high, 1, axis=_AX[d])
    if bc[d] == NEUMANN:
        low = np.where(_low_end_mask(face_high.shape, d), own, low)
    return low


def grad_p(P, rho, n, h, bc):
    """Cell gradient of P (eqs. pbnd and nablaP), stacked (3, nz, ny, nx)."""
    g = np.zeros((3,) + P.shape)
    for d in range(3):
        if n[d] == 1:
            continue
        hi = interface_pressure(P, rho, d, bc)
        lo = _low_interface(hi, P, d, bc)
        g[d] = (hi - lo) / h[d]
    return g


def interface_velocity(mom_d, rho, d, bc):
    """Velocity at the high interface along axis d from the momentum component d (eq. step1);
    zero at a closed high end."""
    u = (mom_d + _plus(mom_d, d)) / (rho + _plus(rho, d))
    if bc[d] == NEUMANN:
        u = np.where(_high_end_mask(mom_d.shape, d), 0.0, u)
    return u


def div_interfaces(uf, n, h, bc):
    """Central-difference divergence of high-interface velocities uf (3, nz, ny, nx); the low
    interface of a cell at a closed low end carries zero velocity."""
    out = np.zeros(uf.shape[1:])
    for d in range(3):
        if n[d] == 1:
            continue
        lo = _low_interface(uf[d], np.zeros_like(uf[d]), d, bc)
        out += (uf[d] - lo) / h[d]
    return out


def div_kappa_grad(c, rk, n, h, bc):
    """div(rk grad c) by fluxes through interfaces: rk at an interface is the mean of the two
    cells, the flux (rk)_f (c_{i+1} - c_i) / h, zero through closed boundaries."""
    out = np.zeros(c.shape)
    for d in range(3):
        if n[d] == 1:
            continue
        flux = 0.5 * (rk + _plus(rk, d)) * (_plus(c, d) - c) / h[d]
        if bc[d] == NEUMANN:
            flux = np.where(_high_end_mask(c.shape, d), 0.0, flux)
        lo = _low_interface(flux, np.zeros_like(flux), d, bc)
        out += (flux - lo) / h[d]
    return out


def pressure_rhs(n, h, bc, dt, rho_n, c2_n, p_n, mom_n, rho_np1, mom_star, visc=None,
                 temp_n=None, conc_n=None, rkc_n=None, r_gas=1.0):
    """b = dt^2 f with f of eq. fpoiss (or eq. fpoiss2 when temp_n, conc_n and rkc_n are given);
    steps (iv) and (v)."""
    m = 1.0 / (rho_n * c2_n)
    u_n = mom_n / rho_n[None]
    gp = grad_p(p_n, rho_n, n, h, bc)
    adv = np.sum(u_n * gp, axis=0)
    uf_star = np.stack([interface_velocity(mom_star[d], rho_np1, d, bc) for d in range(3)])
    b = m * (p_n - dt * adv) - dt * div_interfaces(uf_star, n, h, bc)
    if visc is not None:
        b = b - (2.0 * dt / 3.0) * (m / rho_n) * visc
    if temp_n is not None:
        b = b - (3.0 * dt / 4.0) * m * r_gas * temp_n * div_kappa_grad(conc_n, rkc_n, n, h, bc)
    return b


def pressure_update(n, h, bc, dt, p, rho_np1, mom_star, e_star):
    """Steps (vii)-(ix): returns (rho u)^{n+1} (3, ...), the high-interface velocities
    u^{n+1} (3, ...) and e^{n+1}."""
    gp = grad_p(p, rho_np1, n, h, bc)
    mom = mom_star - dt * gp
    uf = np.zeros_like(mom_star)
    for d in range(3):
        if n[d] == 1:
            continue
        us = interface_velocity(mom_star[d], rho_np1, d, bc)
        du = dt * (_plus(p, d) - p) / h[d] * 2.0 / (_plus(rho_np1, d) + rho_np1)
        if bc[d] == NEUMANN:
            du = np.where(_high_end_mask(p.shape, d), 0.0, du)
        uf[d] = us - du
    u_cell = mom / rho_np1[None]
    e = e_star - dt * (p * div_interfaces(uf, n, h, bc) + np.sum(u_cell * gp, axis=0))
    return mom, uf, e
