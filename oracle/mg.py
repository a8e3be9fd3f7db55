"""Plain definitions of the geometric-multigrid building blocks (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper solves the generalized Poisson equation with preconditioned CG (Section 2) and names
multigrid as the scalable alternative (Section 6, scaling discussion); it gives no multigrid
details, so this module fixes them. None of these choices changes the converged solution, only
how fast PCG gets there; the GPU V-cycle is checked against these definitions element by element.

Hierarchy. Level 0 is the fine grid. An axis is coarsened (n -> n/2, h -> 2h) when n is even and
n/2 >= 2, and, on a periodic axis, n/2 is even (red-black colouring needs even periodic sizes).
Coarsening stops when the level has at most `coarsest_max` cells or no axis can be coarsened.
Coarse coefficients are the means of the children: rho_c = mean(rho), m_c = mean(m); the coarse
operator is the same face rule rediscretised on the coarse grid (w = dt^2 * 2/(rho_a+rho_b)/h^2).

Transfers, per coarsened axis (tensor products over axes):
  P (coarse -> fine, trilinear at cell centres): fine i has parent I = i // 2 and the second
    nearest coarse cell I - 1 (i even) or I + 1 (i odd); weights 3/4 and 1/4. Off the end of a
    Neumann axis the second cell is the parent itself (mirror), on a periodic axis it wraps.
  R (fine -> coarse) = P^T / 2 per coarsened axis, i.e. (1, 3, 3, 1) / 8 in the interior.

Smoother: red-black Gauss-Seidel, red = (i + j + k) even with level-local indices. A half sweep
of colour c sets, for every cell a of colour c,
    z_a <- (r_a + sum_f w_f z_b) / (m_a + sum_f w_f),
using the current values of the other colour (cells of one colour do not couple).

V-cycle (z = M r): on the coarsest level z = A_c^-1 r (dense solve). Otherwise z = 0, nu_pre
times (red, black), then r_c = R (r - A z), z += P V(r_c), then nu_post times (black, red).
This ordering makes M symmetric; it is positive definite because the coarse operators are SPD.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Level:
    n: tuple            # (nx, ny, nz)
    h: tuple            # (hx, hy, hz)
    bc: tuple
    rho: np.ndarray     # (nz, ny, nx)
    m: np.ndarray       # (nz, ny, nx)
    dt: float
    coarsened: tuple = (False, False, False)   # relative to the previous (finer) level
    extra: dict = field(default_factory=dict)
    face_rule: int = 0  # 0: kappa_f = 2 / (rho_a + rho_b); 1: kappa_f = (1/rho_a + 1/rho_b) / 2

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])


def can_coarsen(n: int, bc: int) -> bool:
    if n % 2 or n // 2 < 2:
        return False
    if bc == 0 and (n // 2) % 2:
        return False
    return True


def build_hierarchy(n, h, bc, rho, c2, dt, coarsest_max: int = 512, rho_face=None, face_rule=0):
    """Levels from the fine coefficients. Level.rho is the density of the face coefficients and
    Level.m the mass term; with two densities (eqs. cpoiss and kappapoiss) rho is rho^n
    (m = 1 / (rho^n c2)) and rho_face is rho^{n+1} (None: the same as rho). Every level takes
    the face rule `face_rule` (see Level)."""
    if face_rule not in (0, 1):
        raise ValueError("face_rule must be 0 or 1")
    rho = np.asarray(rho, dtype=np.float64).reshape(n[2], n[1], n[0])
    c2 = np.asarray(c2, dtype=np.float64).reshape(n[2], n[1], n[0])
    rf = rho if rho_face is None else np.asarray(rho_face, dtype=np.float64).reshape(n[2], n[1], n[0])
    levels = [Level(tuple(n), tuple(float(v) for v in h), tuple(bc), rf, 1.0 / (rho * c2),
                    float(dt), face_rule=int(face_rule))]
    while True:
        L = levels[-1]
        ncell = L.n[0] * L.n[1] * L.n[2]
        flags = tuple(can_coarsen(L.n[d], L.bc[d]) for d in range(3))
        if ncell <= coarsest_max or not any(flags):
            break
        nn = tuple(L.n[d] // 2 if flags[d] else L.n[d] for d in range(3))
        hh = tuple(L.h[d] * 2 if flags[d] else L.h[d] for d in range(3))
        levels.append(Level(nn, hh, L.bc, child_mean(L.rho, flags), child_mean(L.m, flags),
                            L.dt, flags, face_rule=L.face_rule))
    return levels


def child_mean(a: np.ndarray, flags) -> np.ndarray:
    """Mean over the children of each coarse cell (2 per coarsened axis)."""
    nz, ny, nx = a.shape
    fz, fy, fx = (2 if flags[2] else 1), (2 if flags[1] else 1), (2 if flags[0] else 1)
    v = a.reshape(nz // fz, fz, ny // fy, fy, nx // fx, fx)
    return v.mean(axis=(1, 3, 5))


def _neighbors(L: Level):
    """Yield (axis, weight array, neighbour index gather) for every face direction of every cell.

    Each yielded item is (mask, nb_flat, w) over all cells: mask False where there is no face.
    """
    nz, ny, nx = L.shape
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    rho = L.rho
    out = []
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        nd = L.n[d]
        if nd == 1:
            continue
        for s in (-1, 1):
            nb = np.roll(idx, -s, axis=ax)           # nb[..i..] = idx[..i+s..] (wrapped)
            mask = np.ones_like(idx, dtype=bool)
            if L.bc[d] == 1:
                pos = np.arange(nd)
                valid = (pos + s >= 0) & (pos + s < nd)
                shape = [1, 1, 1]
                shape[ax] = nd
                mask = np.broadcast_to(valid.reshape(shape), idx.shape)
            rho_b = rho.reshape(-1)[nb]
            kappa = 0.5 * (1.0 / rho + 1.0 / rho_b) if L.face_rule == 1 else 2.0 / (rho + rho_b)
            w = L.dt ** 2 * kappa / (L.h[d] ** 2)
            out.append((mask, nb, np.where(mask, w, 0.0)))
    return out


def apply(L: Level, x: np.ndarray) -> np.ndarray:
    """y = A x in flux form: m_a x_a + sum_f w_f (x_a - x_b)."""
    x = np.asarray(x, dtype=np.float64).reshape(L.shape)
    y = L.m * x
    xf = x.reshape(-1)
    for mask, nb, w in _neighbors(L):
        y = y + w * (x - xf[nb])
    return y


def diagonal(L: Level) -> np.ndarray:
    d = L.m.copy()
    for mask, nb, w in _neighbors(L):
        d = d + w
    return d


def colour(L: Level) -> np.ndarray:
    nz, ny, nx = L.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j + k) % 2


def half_sweep(L: Level, r: np.ndarray, z: np.ndarray, c: int) -> np.ndarray:
    """One red-black Gauss-Seidel half sweep of colour c (returns the new z)."""
    r = np.asarray(r, dtype=np.float64).reshape(L.shape)
    z = np.asarray(z, dtype=np.float64).reshape(L.shape).copy()
    zf = z.reshape(-1).copy()
    num = r.copy()
    den = L.m.copy()
    for mask, nb, w in _neighbors(L):
        num = num + w * zf[nb]
        den = den + w
    upd = colour(L) == c
    z[upd] = (num / den)[upd]
    return z


def _axis_P(nf: int, bc: int) -> np.ndarray:
    """1D prolongation matrix (nf x nf/2) for one coarsened axis."""
    nc = nf // 2
    P = np.zeros((nf, nc))
    for i in range(nf):
        parent = i // 2
        other = parent - 1 if i % 2 == 0 else parent + 1
        if other < 0 or other >= nc:
            other = parent if bc == 1 else other % nc
        P[i, parent] += 0.75
        P[i, other] += 0.25
    return P


def prolong(Lf: Level, Lc: Level, ec: np.ndarray) -> np.ndarray:
    """Trilinear prolongation of a coarse vector to the fine grid of Lf."""
    e = np.asarray(ec, dtype=np.float64).reshape(Lc.shape)
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        if Lc.coarsened[d]:
            P = _axis_P(Lf.n[d], Lf.bc[d])
            e = np.moveaxis(np.tensordot(P, np.moveaxis(e, ax, 0), axes=(1, 0)), 0, ax)
    return e


def restrict(Lf: Level, Lc: Level, rf: np.ndarray) -> np.ndarray:
    """R = P^T / 2 per coarsened axis."""
    r = np.asarray(rf, dtype=np.float64).reshape(Lf.shape)
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        if Lc.coarsened[d]:
            R = _axis_P(Lf.n[d], Lf.bc[d]).T / 2.0
            r = np.moveaxis(np.tensordot(R, np.moveaxis(r, ax, 0), axes=(1, 0)), 0, ax)
    return r


def dense_operator(L: Level) -> np.ndarray:
    N = L.n[0] * L.n[1] * L.n[2]
    A = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        A[:, c] = apply(L, e).reshape(-1)
    return A


def coarse_solve(L: Level, r: np.ndarray) -> np.ndarray:
    if "A" not in L.extra:
        L.extra["A"] = dense_operator(L)
    return np.linalg.solve(L.extra["A"], np.asarray(r, dtype=np.float64).reshape(-1)).reshape(L.shape)


def vcycle(levels, r: np.ndarray, nu_pre: int = 1, nu_post: int = 1, l: int = 0) -> np.ndarray:
    L = levels[l]
    r = np.asarray(r, dtype=np.float64).reshape(L.shape)
    if l == len(levels) - 1:
        return coarse_solve(L, r)
    z = np.zeros(L.shape)
    for _ in range(nu_pre):
        z = half_sweep(L, r, z, 0)
        z = half_sweep(L, r, z, 1)
    rc = restrict(L, levels[l + 1], r - apply(L, z))
    z = z + prolong(L, levels[l + 1], vcycle(levels, rc, nu_pre, nu_post, l + 1))
    for _ in range(nu_post):
        z = half_sweep(L, r, z, 1)
        z = half_sweep(L, r, z, 0)
    return z
