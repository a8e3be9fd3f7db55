"""FP64 CPU oracle for the generalized Poisson (Helmholtz) pressure solve.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the benchmark's
CPU-baseline leg, never by the GPU library or its Python binding.

The operator (paper, Section 2, eqs. Poiss, cpoiss, kappapoiss, vonNeumannBC; face factor from
step (viii) of the fractional-step algorithm), multiplied by dt^2:

    (A p)_a = m_a p_a + sum_{faces f at a} w_f (p_a - p_b),
    m_a = 1 / (rho_a c2_a),   w_f = dt^2 * (2 / (rho_a + rho_b)) / h_d^2.

With two densities (eqs. cpoiss and kappapoiss: rho^n in the mass term, rho^{n+1} in kappa) the
functions take ``rho`` as rho^n and ``rho_face`` as rho^{n+1}: m_a = 1 / (rho^n_a c2_a) and
w_f = dt^2 (2 / (rho^{n+1}_a + rho^{n+1}_b)) / h_d^2. ``rho_face=None`` means rho^{n+1} = rho^n.

``face_rule=1`` replaces the face factor 2 / (rho_a + rho_b) by the mean of kappa = 1/rho of the
two cells, (1/rho_a + 1/rho_b) / 2 (the other reading of eq. kappapoiss); the default 0 is the
factor of the face-velocity update.

Arrays are cell-centred, shaped (nz, ny, nx) in C order (x fastest). ``bc`` holds one entry per
axis (x, y, z): 0 = periodic, 1 = homogeneous Neumann.

Modules:
  * this file   -- ctypes front end of ``hp_oracle.c``: CSR assembly, Jacobi-PCG (the paper's
                   preconditioned conjugate gradient, Section 2), matrix-free residual.
  * separable   -- FFT + tridiagonal (Thomas) solve for coefficients that depend on z only.
  * mg          -- plain definitions of the multigrid building blocks (red-black Gauss-Seidel,
                   restriction, trilinear prolongation, coarse operators, V-cycle).
  * nn          -- FP64 3D convolution network reference (forward and backward).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hp_oracle.c")
_LIB = os.path.join(_HERE, "libhporacle.so")
_lock = threading.Lock()
_lib = None

PERIODIC = 0
NEUMANN = 1


def build(force: bool = False) -> str:
    """Compile hp_oracle.c with gcc (plain C, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("h", ctypes.c_double * 3), ("bc", ctypes.c_int * 3)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("converged", ctypes.c_int), ("stagnated", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("n_coef", ctypes.c_int)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.POINTER
            d_p = P(ctypes.c_double)
            i64_p = P(ctypes.c_int64)
            lib.or_ncells.restype = ctypes.c_int64
            lib.or_ncells.argtypes = [P(_Grid)]
            lib.or_assemble3.restype = ctypes.c_int64
            lib.or_assemble3.argtypes = [P(_Grid), d_p, d_p, d_p, ctypes.c_double, ctypes.c_int,
                                         i64_p, i64_p, d_p]
            lib.or_spmv.restype = None
            lib.or_spmv.argtypes = [ctypes.c_int64, i64_p, i64_p, d_p, d_p, d_p]
            lib.or_dot.restype = ctypes.c_double
            lib.or_dot.argtypes = [ctypes.c_int64, d_p, d_p]
            lib.or_residual_mf3.restype = None
            lib.or_residual_mf3.argtypes = [P(_Grid), d_p, d_p, d_p, ctypes.c_double, ctypes.c_int,
                                            d_p, d_p, d_p]
            lib.or_neumann_rhs.restype = None
            lib.or_neumann_rhs.argtypes = [P(_Grid), ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                           d_p, d_p]
            lib.or_pcg.restype = ctypes.c_int
            lib.or_pcg.argtypes = [ctypes.c_int64, i64_p, i64_p, d_p, d_p, d_p, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, d_p, d_p, ctypes.c_int,
                                   P(_Stats)]
            lib.or_pcg_fixed.restype = ctypes.c_double
            lib.or_pcg_fixed.argtypes = [ctypes.c_int64, i64_p, i64_p, d_p, d_p, d_p,
                                         ctypes.c_int]
            lib.or_max_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _grid(n, h, bc) -> _Grid:
    g = _Grid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.h[d] = float(h[d])
        g.bc[d] = int(bc[d])
    return g


def _f64(a, N=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)
    if N is not None and a.size != N:
        raise ValueError("array has %d entries, grid has %d cells" % (a.size, N))
    return a


def max_threads() -> int:
    return int(_load().or_max_threads())


class CSR:
    """Assembled operator: rowptr/colind/val (int64, int64, float64)."""

    def __init__(self, rowptr, colind, val):
        self.rowptr, self.colind, self.val = rowptr, colind, val
        self.n = rowptr.size - 1

    def matvec(self, x: np.ndarray) -> np.ndarray:
        x = _f64(x, self.n)
        y = np.empty_like(x)
        _load().or_spmv(self.n, _iptr(self.rowptr), _iptr(self.colind), _dptr(self.val),
                        _dptr(x), _dptr(y))
        return y

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _rule(face_rule) -> int:
    if face_rule not in (0, 1):
        raise ValueError("face_rule must be 0 or 1")
    return int(face_rule)


def assemble(n, h, bc, rho, c2, dt, rho_face=None, face_rule=0) -> CSR:
    """Assemble A (see module docstring) by looping over faces; duplicate faces are summed."""
    lib = _load()
    g = _grid(n, h, bc)
    N = int(lib.or_ncells(ctypes.byref(g)))
    rho = _f64(rho, N)
    c2 = _f64(c2, N)
    rf = rho if rho_face is None else _f64(rho_face, N)
    rowptr = np.zeros(N + 1, dtype=np.int64)
    colind = np.zeros(7 * N, dtype=np.int64)
    val = np.zeros(7 * N, dtype=np.float64)
    nnz = lib.or_assemble3(ctypes.byref(g), _dptr(rho), _dptr(rf), _dptr(c2), float(dt),
                           _rule(face_rule), _iptr(rowptr), _iptr(colind), _dptr(val))
    return CSR(rowptr, colind[:nnz].copy(), val[:nnz].copy())


def residual(n, h, bc, rho, c2, dt, x, b, rho_face=None, face_rule=0) -> np.ndarray:
    """Matrix-free r = b - A x (same face definition, no CSR; any size that fits in memory)."""
    lib = _load()
    g = _grid(n, h, bc)
    N = int(lib.or_ncells(ctypes.byref(g)))
    rho, c2, x, b = _f64(rho, N), _f64(c2, N), _f64(x, N), _f64(b, N)
    rf = rho if rho_face is None else _f64(rho_face, N)
    r = np.empty(N, dtype=np.float64)
    lib.or_residual_mf3(ctypes.byref(g), _dptr(rho), _dptr(rf), _dptr(c2), float(dt),
                        _rule(face_rule), _dptr(x), _dptr(b), _dptr(r))
    return r


def neumann_rhs(n, h, bc, dt, axis: int, side: int, q, b=None) -> np.ndarray:
    """Right-hand side term of inhomogeneous Neumann data: for every cell next to boundary `side`
    (0 low, 1 high) of the Neumann axis `axis` (0 x, 1 y, 2 z), b += dt^2 q / h_axis with q the
    prescribed outward normal flux kappa dphi/dn through that boundary face. q is shaped like the
    boundary plane of the (nz, ny, nx) array with that axis removed. Returns b (a new zero array
    if b is None), shaped (nz, ny, nx)."""
    lib = _load()
    if bc[axis] != NEUMANN:
        raise ValueError("Neumann data needs a Neumann axis")
    gr = _grid(n, h, bc)
    N = int(lib.or_ncells(ctypes.byref(gr)))
    out = np.zeros(N) if b is None else _f64(b, N).copy()
    qv = _f64(q)
    others = [d for d in range(3) if d != axis]
    if qv.size != n[others[0]] * n[others[1]]:
        raise ValueError("boundary data has %d entries, the boundary has %d faces"
                         % (qv.size, n[others[0]] * n[others[1]]))
    lib.or_neumann_rhs(ctypes.byref(gr), float(dt), int(axis), int(side), _dptr(qv), _dptr(out))
    return out.reshape(n[2], n[1], n[0])


def dot(x, y) -> float:
    x = _f64(x)
    y = _f64(y, x.size)
    return float(_load().or_dot(x.size, _dptr(x), _dptr(y)))


def pcg(A: CSR, b, x0=None, tol=1e-10, maxiter=1_000_000, stag_window=0, coef_cap=0):
    """Jacobi-PCG on an assembled operator. Returns (x, stats dict)."""
    lib = _load()
    b = _f64(b, A.n)
    x = np.zeros(A.n) if x0 is None else _f64(x0, A.n).copy()
    st = _Stats()
    al = np.zeros(max(coef_cap, 1))
    be = np.zeros(max(coef_cap, 1))
    status = lib.or_pcg(A.n, _iptr(A.rowptr), _iptr(A.colind), _dptr(A.val), _dptr(b), _dptr(x),
                        float(tol), int(maxiter), int(stag_window),
                        _dptr(al) if coef_cap else None, _dptr(be) if coef_cap else None,
                        int(coef_cap), ctypes.byref(st))
    stats = dict(status=int(status), iterations=st.iterations, restarts=st.restarts,
                 converged=bool(st.converged), stagnated=bool(st.stagnated),
                 rel_residual=st.rel_residual)
    if coef_cap:
        stats["alpha"] = al[: st.n_coef].copy()
        stats["beta"] = be[: st.n_coef].copy()
    return x, stats


def pcg_fixed(A: CSR, b, iters: int) -> float:
    """Exactly `iters` Jacobi-PCG iterations from zero (timing unit); returns the relative residual."""
    b = _f64(b, A.n)
    x = np.zeros(A.n)
    return float(_load().or_pcg_fixed(A.n, _iptr(A.rowptr), _iptr(A.colind), _dptr(A.val),
                                      _dptr(b), _dptr(x), int(iters)))


def solve(n, h, bc, rho, c2, dt, b, x0=None, tol=1e-10, maxiter=1_000_000, stag_window=0,
          coef_cap=0, rho_face=None, face_rule=0):
    """Assemble and solve A x = b with Jacobi-PCG. Returns (x shaped like b, stats)."""
    shape = np.shape(b)
    A = assemble(n, h, bc, rho, c2, dt, rho_face, face_rule)
    x, st = pcg(A, b, x0, tol, maxiter, stag_window, coef_cap)
    return x.reshape(shape), st


def reference_solve(n, h, bc, rho, c2, dt, b, maxiter=1_000_000, rho_face=None, face_rule=0):
    """Reference solution for parity: tol 1e-13 or stagnation of the true residual."""
    return solve(n, h, bc, rho, c2, dt, b, tol=1e-13, maxiter=maxiter, stag_window=50,
                 rho_face=rho_face, face_rule=face_rule)


def lanczos_extremes(alpha: np.ndarray, beta: np.ndarray):
    """Extreme Ritz values of D^-1 A from the CG coefficients (Lanczos tridiagonal)."""
    k = len(alpha)
    if k == 0:
        return float("nan"), float("nan")
    d = np.empty(k)
    e = np.empty(max(k - 1, 0))
    for j in range(k):
        d[j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j < k - 1:
            e[j] = np.sqrt(beta[j]) / alpha[j]
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])
