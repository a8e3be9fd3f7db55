"""Separable solve of the pressure system when rho and c2 depend on z only.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

This is a textbook reduction of the same discrete operator, used to pin the PCG oracle and as an
exact full-size reference. When rho and c2 are functions of the vertical index k alone and the
horizontal axes are periodic (or have a single cell), every horizontal face inside plane k has
kappa = 2 / (rho_k + rho_k) = 1 / rho_k, so the horizontal part of A is diagonalised by the
discrete Fourier transform: the periodic second difference has eigenvalues
mu = 4 sin^2(pi q / n), q = 0 .. n-1 (this counts both wrap faces when n = 2). What remains per
horizontal mode is a symmetric tridiagonal system in z:

    [m_k + (dt^2 / rho_k)(mu_x / hx^2 + mu_y / hy^2)] q_k
        + (dt^2 / hz^2) [ w_{k+1/2} (q_k - q_{k+1}) + w_{k-1/2} (q_k - q_{k-1}) ] = bhat_k,

w_{k+1/2} = 2 / (rho_k + rho_{k+1}); on a Neumann z axis the end faces are absent, on a periodic
z axis this is not supported here. The system is diagonally dominant, so Thomas elimination
without pivoting is stable. All arithmetic is FP64.
"""
from __future__ import annotations

import numpy as np


def horizontal_symbol(n: int) -> np.ndarray:
    """Eigenvalues of the periodic second-difference matrix of size n (0 for n = 1)."""
    q = np.arange(n)
    if n == 1:
        return np.zeros(1)
    return 4.0 * np.sin(np.pi * q / n) ** 2


def _thomas_batched(lower, diag, upper, rhs):
    """Solve tridiagonal systems along axis 0; lower[k] couples k to k-1, upper[k] to k+1.

    diag has shape (nz, M), rhs (nz, M) complex; lower/upper shape (nz,) (shared by all modes).
    """
    nz = diag.shape[0]
    cp = np.empty_like(diag)
    dp = np.empty_like(rhs)
    cp[0] = upper[0] / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, nz):
        den = diag[k] - lower[k] * cp[k - 1]
        cp[k] = upper[k] / den
        dp[k] = (rhs[k] - lower[k] * dp[k - 1]) / den
    x = np.empty_like(rhs)
    x[nz - 1] = dp[nz - 1]
    for k in range(nz - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def solve_stratified(n, h, bc, rho_z, c2_z, dt, b, rho_face_z=None) -> np.ndarray:
    """Solve A x = b for rho, c2 given per z-plane (length nz arrays); b shaped (nz, ny, nx).

    bc must be periodic (or n = 1) on x and y and Neumann on z. With two densities
    (eqs. cpoiss and kappapoiss) rho_z is rho^n (mass term m_k = 1 / (rho^n_k c2_k)) and
    rho_face_z is rho^{n+1} (horizontal kappa 1 / rho^{n+1}_k, vertical faces
    2 / (rho^{n+1}_k + rho^{n+1}_{k+1})); rho_face_z = None means rho^{n+1} = rho^n.
    """
    nx, ny, nz = (int(v) for v in n)
    hx, hy, hz = (float(v) for v in h)
    if not ((bc[0] == 0 or nx == 1) and (bc[1] == 0 or ny == 1)):
        raise ValueError("horizontal axes must be periodic")
    if bc[2] != 1:
        raise ValueError("z axis must be Neumann")
    rho_z = np.asarray(rho_z, dtype=np.float64).reshape(nz)
    c2_z = np.asarray(c2_z, dtype=np.float64).reshape(nz)
    rf = rho_z if rho_face_z is None else np.asarray(rho_face_z, dtype=np.float64).reshape(nz)
    b = np.asarray(b, dtype=np.float64).reshape(nz, ny, nx)
    dt2 = float(dt) ** 2
    m = 1.0 / (rho_z * c2_z)
    # vertical face weights, w[k] between k and k+1
    wv = dt2 * (2.0 / (rf[:-1] + rf[1:])) / (hz * hz)
    lower = np.zeros(nz)
    upper = np.zeros(nz)
    lower[1:] = -wv
    upper[:-1] = -wv
    vsum = np.zeros(nz)
    vsum[:-1] += wv
    vsum[1:] += wv
    mux = horizontal_symbol(nx)[: nx // 2 + 1]          # rfft along x keeps q = 0 .. nx/2
    muy = horizontal_symbol(ny)
    hsym = (muy[:, None] / (hy * hy) + mux[None, :] / (hx * hx)).reshape(-1)  # (ny*(nx//2+1))
    diag = (m + vsum)[:, None] + (dt2 / rf)[:, None] * hsym[None, :]
    bh = np.fft.rfft2(b, axes=(1, 2)).reshape(nz, -1)
    xh = _thomas_batched(lower, diag, upper, bh)
    x = np.fft.irfft2(xh.reshape(nz, ny, nx // 2 + 1), s=(ny, nx), axes=(1, 2))
    return x


def eigenpair(n, h, bc, rho0, c20, dt, q):
    """Closed-form eigenpair of A for constant rho0, c20.

    q = (qx, qy, qz) mode numbers. Periodic axis: phi = cos(2 pi q i / n) with
    mu = 4 sin^2(pi q / n). Neumann axis: phi = cos(pi q (i+1/2)/n) with mu = 4 sin^2(pi q/(2n)).
    Returns (lambda, phi shaped (nz, ny, nx)).
    """
    dt2 = float(dt) ** 2
    lam = 1.0 / (rho0 * c20)
    vecs = []
    for d in range(3):
        nd = int(n[d])
        i = np.arange(nd) + 0.5
        if nd == 1:
            mu = 0.0
            v = np.ones(1)
        elif bc[d] == 0:
            mu = 4.0 * np.sin(np.pi * q[d] / nd) ** 2
            v = np.cos(2.0 * np.pi * q[d] * (i - 0.5) / nd)
        else:
            mu = 4.0 * np.sin(np.pi * q[d] / (2.0 * nd)) ** 2
            v = np.cos(np.pi * q[d] * i / nd)
        lam += dt2 / rho0 * mu / (float(h[d]) ** 2)
        vecs.append(v)
    phi = vecs[2][:, None, None] * vecs[1][None, :, None] * vecs[0][None, None, :]
    return lam, phi
