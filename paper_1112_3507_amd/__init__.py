"""MI355X (gfx950) implicit pressure solve for the semi-implicit low-Mach scheme.

Thin ctypes binding over ``libhp.so`` (declared in ``include/hp.h``): it only checks and
marshals arguments (torch device tensors -> device pointers, the current torch stream -> the
handle's HIP stream); every step of the solve runs in the library's HIP kernels. There is no
CPU fallback: if the library is not built, loading fails with an error.

Arrays are cell-centred, shaped (nz, ny, nx) (or flat), x fastest, on the current HIP device.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhp.so")

PERIODIC, NEUMANN = 0, 1
MODE_JACOBI_PCG, MODE_FP64_MGPCG, MODE_MIXED_IR, MODE_LEARNED = 0, 1, 2, 3
OPT_MODE, OPT_MAX_ITER, OPT_NU_PRE, OPT_NU_POST = 1, 2, 3, 4
OPT_INNER_TOL, OPT_MAX_OUTER, OPT_COARSEST_MAX = 5, 6, 7
OPT_LAYOUT = 8  # finest-level storage inside the handle: 1 red-black split, 0 natural
OPT_KERNEL_TIMING = 9  # 1: time finest-level sweeps and applies inside FP64 solves
OPT_FACE_RULE = 10  # face value of kappa: 0 = 2/(rho_a + rho_b) (default), 1 = (1/rho_a + 1/rho_b)/2

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, ENAN, ENOCONV, EBREAKDOWN, EIO = 0, -1, -2, -3, -4, -5, -6, -7, -8
_CODE_NAMES = {EINVAL: "HP_EINVAL", EDOMAIN: "HP_EDOMAIN", ENOMEM: "HP_ENOMEM", EHIP: "HP_EHIP",
               ENAN: "HP_ENAN", ENOCONV: "HP_ENOCONV", EBREAKDOWN: "HP_EBREAKDOWN", EIO: "HP_EIO"}

# every symbol include/hp.h declares
EXPORTS = [
    "hp_setup", "hp_solve", "hp_free", "hp_set_stream", "hp_set_option", "hp_get_option",
    "hp_update_coefficients", "hp_get_stats", "hp_last_error", "hp_num_levels", "hp_level_info",
    "hp_apply", "hp_apply_f32", "hp_smooth", "hp_smooth_f32", "hp_restrict_residual",
    "hp_restrict_residual_f32", "hp_prolong_add", "hp_prolong_add_f32", "hp_coarse_solve",
    "hp_coarse_solve_f32", "hp_precond", "hp_precond_f32", "hp_residual", "hp_dot",
    "hp_nn_num_params", "hp_nn_create", "hp_nn_free", "hp_nn_set_stream", "hp_nn_last_error",
    "hp_nn_set_params", "hp_nn_get_params", "hp_nn_get_grad", "hp_nn_set_output_scale",
    "hp_nn_save", "hp_nn_load",
    "hp_nn_forward", "hp_nn_train_step", "hp_nn_forward_raw", "hp_nn_loss_grad_raw", "hp_nn_adam",
    "hp_attach_net", "hp_warm_start", "hp_nn_train_step_anorm",
    "hp_dot_noalloc", "hp_noalloc_last_error",
    "hp_setup_two_density", "hp_update_coefficients_two_density", "hp_neumann_rhs",
    "hp_pressure_rhs", "hp_pressure_update", "hp_stream_copy", "hp_advect", "hp_eos_ideal",
    "hp_axpby",
]


class HPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_CODE_NAMES.get(code, "HP_?"), code, msg))
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double)]


class BC(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int), ("y", ctypes.c_int), ("z", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("converged", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("levels", ctypes.c_int), ("status", ctypes.c_int), ("fallback", ctypes.c_int),
                ("timed_sweeps", ctypes.c_int), ("sweep_ms", ctypes.c_double),
                ("timed_applies", ctypes.c_int), ("apply_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RhsFields(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("rho_n", "c2_n", "p_n", "mom_n", "rho_np1", "mom_star",
                                                "visc", "temp_n", "conc_n", "rkc_n")] + [("r_gas", ctypes.c_double)]


class UpdateFields(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("p", "rho_np1", "mom_star", "e_star", "mom_out", "uface_out",
                                                "e_out")]


_lock = threading.Lock()
_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhp.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError("libhp.so is not built (%s); run `python -m "
                                  "paper_1112_3507_amd.build`" % path)
            lib = ctypes.CDLL(path)
            vp, dp, fp, ip = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int
            H = ctypes.c_void_p
            sig = {
                "hp_setup": (ip, [ctypes.POINTER(Grid), dp, dp, ctypes.c_double,
                                  ctypes.POINTER(BC), ctypes.POINTER(ctypes.c_void_p)]),
                "hp_solve": (ip, [H, dp, dp, ctypes.c_double]),
                "hp_free": (None, [H]),
                "hp_set_stream": (ip, [H, vp]),
                "hp_set_option": (ip, [H, ip, ctypes.c_double]),
                "hp_get_option": (ip, [H, ip, ctypes.POINTER(ctypes.c_double)]),
                "hp_update_coefficients": (ip, [H, dp, dp, ctypes.c_double]),
                "hp_get_stats": (ip, [H, ctypes.POINTER(Stats)]),
                "hp_last_error": (ctypes.c_char_p, []),
                "hp_num_levels": (ip, [H]),
                "hp_level_info": (ip, [H, ip, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double)]),
                "hp_apply": (ip, [H, ip, dp, dp]),
                "hp_apply_f32": (ip, [H, ip, fp, fp]),
                "hp_smooth": (ip, [H, ip, dp, dp, ip]),
                "hp_smooth_f32": (ip, [H, ip, fp, fp, ip]),
                "hp_restrict_residual": (ip, [H, ip, dp, dp, dp]),
                "hp_restrict_residual_f32": (ip, [H, ip, fp, fp, fp]),
                "hp_prolong_add": (ip, [H, ip, dp, dp]),
                "hp_prolong_add_f32": (ip, [H, ip, fp, fp]),
                "hp_coarse_solve": (ip, [H, dp, dp]),
                "hp_coarse_solve_f32": (ip, [H, fp, fp]),
                "hp_precond": (ip, [H, dp, dp]),
                "hp_precond_f32": (ip, [H, fp, fp]),
                "hp_residual": (ip, [H, dp, dp, dp, ctypes.POINTER(ctypes.c_double)]),
                "hp_dot": (ip, [H, dp, dp, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double)]),
                "hp_nn_num_params": (ctypes.c_longlong, []),
                "hp_nn_create": (ip, [ip, ip, ip, ip, ctypes.POINTER(ctypes.c_void_p)]),
                "hp_nn_free": (None, [vp]),
                "hp_nn_set_stream": (ip, [vp, vp]),
                "hp_nn_last_error": (ctypes.c_char_p, []),
                "hp_nn_set_params": (ip, [vp, vp]),
                "hp_nn_get_params": (ip, [vp, vp]),
                "hp_nn_get_grad": (ip, [vp, vp]),
                "hp_nn_set_output_scale": (ip, [vp, ctypes.c_double]),
                "hp_nn_save": (ip, [vp, ctypes.c_char_p]),
                "hp_nn_load": (ip, [vp, ctypes.c_char_p]),
                "hp_nn_forward": (ip, [vp, dp, dp, dp, dp, dp]),
                "hp_nn_train_step": (ip, [vp, dp, dp, dp, dp, dp, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_double)]),
                "hp_nn_forward_raw": (ip, [vp, vp, vp]),
                "hp_nn_loss_grad_raw": (ip, [vp, vp, vp, ctypes.POINTER(ctypes.c_double)]),
                "hp_nn_adam": (ip, [vp, ctypes.c_float]),
                "hp_attach_net": (ip, [H, vp]),
                "hp_warm_start": (ip, [H, dp, dp, dp]),
                "hp_nn_train_step_anorm": (ip, [H, vp, dp, dp, dp, ctypes.c_float,
                                                ctypes.POINTER(ctypes.c_double)]),
                "hp_dot_noalloc": (ip, [dp, dp, ctypes.c_longlong, dp, vp]),
                "hp_noalloc_last_error": (ctypes.c_char_p, []),
                "hp_setup_two_density": (ip, [ctypes.POINTER(Grid), dp, dp, dp, ctypes.c_double,
                                              ctypes.POINTER(BC), ctypes.POINTER(ctypes.c_void_p)]),
                "hp_update_coefficients_two_density": (ip, [H, dp, dp, dp, ctypes.c_double]),
                "hp_neumann_rhs": (ip, [H, ip, ip, dp, dp]),
                "hp_pressure_rhs": (ip, [H, ctypes.POINTER(RhsFields), dp]),
                "hp_pressure_update": (ip, [H, ctypes.POINTER(UpdateFields)]),
                "hp_stream_copy": (ip, [dp, dp, ctypes.c_longlong, vp]),
                "hp_advect": (ip, [H, dp, dp, dp, dp, dp, dp]),
                "hp_eos_ideal": (ip, [H, dp, dp, dp, ctypes.c_double, dp, dp]),
                "hp_axpby": (ip, [H, ctypes.c_double, dp, ctypes.c_double, dp, ctypes.c_longlong]),
            }
            for name, (res, args) in sig.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def _check(rc: int):
    if rc != OK:
        msg = load_library().hp_last_error()
        raise HPError(rc, msg.decode() if msg else "")


def _check_nn(rc: int):
    if rc != OK:
        msg = load_library().hp_nn_last_error()
        raise HPError(rc, msg.decode() if msg else "")


def _torch():
    import torch
    return torch


def _ptr(t, dtype_name: str, numel: int, device_index: int):
    torch = _torch()
    dt = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda" or t.device.index != device_index:
        raise ValueError("tensor must live on cuda:%d" % device_index)
    if t.dtype != dt:
        raise TypeError("expected dtype %s, got %s" % (dt, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if t.numel() != numel:
        raise ValueError("tensor has %d entries, expected %d" % (t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Handle around hp_setup / hp_solve / hp_free (one grid, one coefficient set at a time)."""

    def __init__(self, n, h, bc, rho, c2, dt: float, mode: int | None = None, rho_face=None):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self.n = tuple(int(v) for v in n)
        self.bc = tuple(int(v) for v in bc)
        self.ncells = self.n[0] * self.n[1] * self.n[2]
        self.device = torch.cuda.current_device()
        g = Grid(self.n[0], self.n[1], self.n[2], float(h[0]), float(h[1]), float(h[2]))
        b = BC(int(bc[0]), int(bc[1]), int(bc[2]))
        handle = ctypes.c_void_p()
        rp = _ptr(rho, "f64", self.ncells, self.device)
        cp = _ptr(c2, "f64", self.ncells, self.device)
        torch.cuda.current_stream().synchronize()
        if rho_face is None:
            _check(lib.hp_setup(ctypes.byref(g), rp, cp, float(dt), ctypes.byref(b),
                                ctypes.byref(handle)))
        else:
            fp_ = _ptr(rho_face, "f64", self.ncells, self.device)
            _check(lib.hp_setup_two_density(ctypes.byref(g), rp, fp_, cp, float(dt), ctypes.byref(b),
                                            ctypes.byref(handle)))
        self._h = handle
        self.set_stream(torch.cuda.current_stream())
        if mode is not None:
            self.set_option(OPT_MODE, mode)

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None):
            self._lib.hp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- configuration --
    def set_stream(self, stream):
        _check(self._lib.hp_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def set_option(self, key: int, value: float):
        _check(self._lib.hp_set_option(self._h, int(key), float(value)))

    def get_option(self, key: int) -> float:
        v = ctypes.c_double()
        _check(self._lib.hp_get_option(self._h, int(key), ctypes.byref(v)))
        return v.value

    def update_coefficients(self, rho, c2, dt: float, rho_face=None):
        rp = _ptr(rho, "f64", self.ncells, self.device)
        cp = _ptr(c2, "f64", self.ncells, self.device)
        if rho_face is None:
            _check(self._lib.hp_update_coefficients(self._h, rp, cp, float(dt)))
        else:
            _check(self._lib.hp_update_coefficients_two_density(
                self._h, rp, _ptr(rho_face, "f64", self.ncells, self.device), cp, float(dt)))

    def neumann_rhs(self, axis: int, side: int, q, rhs):
        """hp_neumann_rhs: rhs += dt^2 q / h on the cells next to that boundary (q: prescribed
        outward normal flux per boundary face)."""
        others = [d for d in range(3) if d != axis]
        nf = self.n[others[0]] * self.n[others[1]]
        _check(self._lib.hp_neumann_rhs(self._h, int(axis), int(side), _ptr(q, "f64", nf, self.device),
                                        _ptr(rhs, "f64", self.ncells, self.device)))

    # -- the steps either side of the solve --
    def pressure_rhs(self, rho_n, c2_n, p_n, mom_n, rho_np1, mom_star, rhs, visc=None, temp_n=None,
                     conc_n=None, rkc_n=None, r_gas=1.0):
        """hp_pressure_rhs: rhs = dt^2 f of the pressure equation from the fields of time n and
        the explicit step (momenta are (3, nz, ny, nx) tensors)."""
        c, d = self.ncells, self.device
        opt = lambda t: _ptr(t, "f64", c, d) if t is not None else None
        f = RhsFields(_ptr(rho_n, "f64", c, d), _ptr(c2_n, "f64", c, d), _ptr(p_n, "f64", c, d),
                      _ptr(mom_n, "f64", 3 * c, d), _ptr(rho_np1, "f64", c, d),
                      _ptr(mom_star, "f64", 3 * c, d), opt(visc), opt(temp_n), opt(conc_n), opt(rkc_n),
                      float(r_gas))
        _check(self._lib.hp_pressure_rhs(self._h, ctypes.byref(f), _ptr(rhs, "f64", c, d)))

    def pressure_update(self, p, rho_np1, mom_star, e_star, mom_out, uface_out, e_out):
        """hp_pressure_update: momentum, interface velocities and energy after the solve."""
        c, d = self.ncells, self.device
        f = UpdateFields(_ptr(p, "f64", c, d), _ptr(rho_np1, "f64", c, d), _ptr(mom_star, "f64", 3 * c, d),
                         _ptr(e_star, "f64", c, d), _ptr(mom_out, "f64", 3 * c, d),
                         _ptr(uface_out, "f64", 3 * c, d), _ptr(e_out, "f64", c, d))
        _check(self._lib.hp_pressure_update(self._h, ctypes.byref(f)))

    def advect(self, rho, mom, e, rho_out, mom_out, e_out):
        """hp_advect: rho^{n+1}, (rho u)*, e* of the explicit inviscid step (handle's dt)."""
        c, d = self.ncells, self.device
        _check(self._lib.hp_advect(self._h, _ptr(rho, "f64", c, d), _ptr(mom, "f64", 3 * c, d),
                                   _ptr(e, "f64", c, d), _ptr(rho_out, "f64", c, d),
                                   _ptr(mom_out, "f64", 3 * c, d), _ptr(e_out, "f64", c, d)))

    def eos_ideal(self, rho, mom, e, gamma, p, c2=None):
        """hp_eos_ideal: pressure (and squared sound speed) of an ideal gas."""
        c, d = self.ncells, self.device
        _check(self._lib.hp_eos_ideal(self._h, _ptr(rho, "f64", c, d), _ptr(mom, "f64", 3 * c, d),
                                      _ptr(e, "f64", c, d), float(gamma), _ptr(p, "f64", c, d),
                                      _ptr(c2, "f64", c, d) if c2 is not None else None))

    def axpby(self, a, x, b, y):
        """hp_axpby: y = a x + b y on the handle's stream."""
        n, d = x.numel(), self.device
        _check(self._lib.hp_axpby(self._h, float(a), _ptr(x, "f64", n, d), float(b), _ptr(y, "f64", n, d), n))

    # -- the solve --
    def solve(self, rhs, p, tol: float = 1e-10, check: bool = True) -> dict:
        rc = self._lib.hp_solve(self._h, _ptr(rhs, "f64", self.ncells, self.device),
                                _ptr(p, "f64", self.ncells, self.device), float(tol))
        st = self.stats()
        if check:
            _check(rc)
        st["rc"] = rc
        return st

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.hp_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    # -- building blocks --
    def num_levels(self) -> int:
        return int(self._lib.hp_num_levels(self._h))

    def level_info(self, level: int):
        n = (ctypes.c_int * 3)()
        hs = (ctypes.c_double * 3)()
        _check(self._lib.hp_level_info(self._h, int(level), n, hs))
        return tuple(n), tuple(hs)

    def level_cells(self, level: int) -> int:
        n, _ = self.level_info(level)
        return n[0] * n[1] * n[2]

    def _vec(self, t, level, f32=False):
        return _ptr(t, "f32" if f32 else "f64", self.level_cells(level), self.device)

    def apply(self, level, x, y, f32=False):
        fn = self._lib.hp_apply_f32 if f32 else self._lib.hp_apply
        _check(fn(self._h, level, self._vec(x, level, f32), self._vec(y, level, f32)))

    def smooth(self, level, r, z, colour, f32=False):
        fn = self._lib.hp_smooth_f32 if f32 else self._lib.hp_smooth
        _check(fn(self._h, level, self._vec(r, level, f32), self._vec(z, level, f32), int(colour)))

    def restrict_residual(self, level, r, z, rc, f32=False):
        fn = self._lib.hp_restrict_residual_f32 if f32 else self._lib.hp_restrict_residual
        _check(fn(self._h, level, self._vec(r, level, f32), self._vec(z, level, f32),
                  self._vec(rc, level + 1, f32)))

    def prolong_add(self, level, ec, z, f32=False):
        fn = self._lib.hp_prolong_add_f32 if f32 else self._lib.hp_prolong_add
        _check(fn(self._h, level, self._vec(ec, level + 1, f32), self._vec(z, level, f32)))

    def coarse_solve(self, b, x, f32=False):
        last = self.num_levels() - 1
        fn = self._lib.hp_coarse_solve_f32 if f32 else self._lib.hp_coarse_solve
        _check(fn(self._h, self._vec(b, last, f32), self._vec(x, last, f32)))

    def precond(self, r, z, f32=False):
        fn = self._lib.hp_precond_f32 if f32 else self._lib.hp_precond
        _check(fn(self._h, self._vec(r, 0, f32), self._vec(z, 0, f32)))

    def residual(self, rhs, p, r) -> float:
        rel = ctypes.c_double()
        _check(self._lib.hp_residual(self._h, self._vec(rhs, 0), self._vec(p, 0), self._vec(r, 0),
                                     ctypes.byref(rel)))
        return rel.value

    def dot(self, x, y) -> float:
        out = ctypes.c_double()
        n = x.numel()
        _check(self._lib.hp_dot(self._h, _ptr(x, "f64", n, self.device),
                                _ptr(y, "f64", n, self.device), n, ctypes.byref(out)))
        return out.value

    def attach_net(self, net):
        self._net = net
        _check(self._lib.hp_attach_net(self._h, net._h if net is not None else None))

    def train_step_anorm(self, net, rhs, x, lr, p_prev=None) -> float:
        loss = ctypes.c_double()
        _check(self._lib.hp_nn_train_step_anorm(
            self._h, net._h, self._vec(rhs, 0), self._vec(p_prev, 0) if p_prev is not None else None,
            self._vec(x, 0), float(lr), ctypes.byref(loss)))
        return loss.value

    def warm_start(self, rhs, x, p_prev=None):
        _check(self._lib.hp_warm_start(self._h, self._vec(rhs, 0),
                                       self._vec(p_prev, 0) if p_prev is not None else None,
                                       self._vec(x, 0)))


def dot_noalloc(x, y, result, stream=None):
    """hp_dot_noalloc: result[0] = <x, y> (device FP64 tensors; result has one entry), enqueued on
    `stream` (default: torch's current stream) without allocating or synchronising."""
    torch = _torch()
    lib = load_library()
    d = torch.cuda.current_device()
    n = x.numel()
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.hp_dot_noalloc(_ptr(x, "f64", n, d) if n else None, _ptr(y, "f64", n, d) if n else None,
                            n, _ptr(result, "f64", 1, d), ctypes.c_void_p(st.cuda_stream))
    if rc != OK:
        msg = lib.hp_noalloc_last_error()
        raise HPError(rc, msg.decode() if msg else "")


def stream_copy(src, dst, stream=None):
    """hp_stream_copy: dst = src (device FP64 tensors of equal size) on `stream` (default: torch's
    current stream)."""
    torch = _torch()
    d = torch.cuda.current_device()
    n = src.numel()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load_library().hp_stream_copy(_ptr(src, "f64", n, d), _ptr(dst, "f64", n, d), n,
                                         ctypes.c_void_p(st.cuda_stream)))


def num_params() -> int:
    return int(load_library().hp_nn_num_params())


class Net:
    """Handle around the learned warm start / preconditioner network (hp_nn_*)."""

    def __init__(self, n, training: bool = False):
        torch = _torch()
        lib = load_library()
        self._lib = lib
        self.n = tuple(int(v) for v in n)
        self.ncells = self.n[0] * self.n[1] * self.n[2]
        self.device = torch.cuda.current_device()
        self.nparam = num_params()
        h = ctypes.c_void_p()
        _check_nn(lib.hp_nn_create(self.n[0], self.n[1], self.n[2], 1 if training else 0,
                                   ctypes.byref(h)))
        self._h = h
        _check_nn(lib.hp_nn_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hp_nn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _p(self, t, kind, numel):
        torch = _torch()
        want = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[kind]
        if t.dtype != want or t.device.type != "cuda" or not t.is_contiguous() or t.numel() != numel:
            raise ValueError("expected a contiguous %s cuda tensor of %d entries" % (want, numel))
        return ctypes.c_void_p(t.data_ptr())

    def set_params(self, theta):
        _check_nn(self._lib.hp_nn_set_params(self._h, self._p(theta, "f32", self.nparam)))

    def get_params(self):
        torch = _torch()
        out = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check_nn(self._lib.hp_nn_get_params(self._h, self._p(out, "f32", self.nparam)))
        return out

    def get_grad(self):
        torch = _torch()
        out = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check_nn(self._lib.hp_nn_get_grad(self._h, self._p(out, "f32", self.nparam)))
        return out

    def set_output_scale(self, s: float):
        _check_nn(self._lib.hp_nn_set_output_scale(self._h, float(s)))

    def save(self, path: str):
        """Write the parameters and the output scale to a checkpoint file (hp_nn_save)."""
        _check_nn(self._lib.hp_nn_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Replace the parameters and the output scale from a checkpoint file (hp_nn_load)."""
        _check_nn(self._lib.hp_nn_load(self._h, os.fsencode(path)))

    def forward(self, b, rho, c2, p_prev, x):
        n = self.ncells
        _check_nn(self._lib.hp_nn_forward(self._h, self._p(b, "f64", n), self._p(rho, "f64", n),
                                          self._p(c2, "f64", n),
                                          self._p(p_prev, "f64", n) if p_prev is not None else None,
                                          self._p(x, "f64", n)))

    def train_step(self, b, rho, c2, p_prev, x_target, lr: float) -> float:
        n = self.ncells
        loss = ctypes.c_double()
        _check_nn(self._lib.hp_nn_train_step(
            self._h, self._p(b, "f64", n), self._p(rho, "f64", n), self._p(c2, "f64", n),
            self._p(p_prev, "f64", n) if p_prev is not None else None, self._p(x_target, "f64", n),
            float(lr), ctypes.byref(loss)))
        return loss.value

    def forward_raw(self, inp_bf16, y):
        _check_nn(self._lib.hp_nn_forward_raw(self._h, self._p(inp_bf16, "bf16", self.ncells * 8),
                                              self._p(y, "f32", self.ncells)))

    def loss_grad_raw(self, inp_bf16, target) -> float:
        loss = ctypes.c_double()
        _check_nn(self._lib.hp_nn_loss_grad_raw(self._h, self._p(inp_bf16, "bf16", self.ncells * 8),
                                                self._p(target, "f32", self.ncells),
                                                ctypes.byref(loss)))
        return loss.value

    def adam(self, lr: float):
        _check_nn(self._lib.hp_nn_adam(self._h, float(lr)))


def setup(n, h, bc, rho, c2, dt, mode=None, rho_face=None) -> Solver:
    """Python spelling of hp_setup (hp_setup_two_density when rho_face, the density of the face
    coefficients at time level n+1, is given; rho is then the density of the mass term)."""
    return Solver(n, h, bc, rho, c2, dt, mode, rho_face)
