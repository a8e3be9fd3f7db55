"""Semi-implicit time steps of the fractional-step scheme on the GPU (inviscid, one component).

Section 2, "The Algorithm", steps (i)-(x), as a sequence of library calls on device tensors (this
module only orders them and holds the buffers; every arithmetic step runs in the HIP kernels of
libhp.so):

    stage L(U):  hp_eos_ideal       P^n, c_s^2 from (rho, rho u, e)                 (step (x) of the
                                                                                      previous stage)
                 hp_advect          rho^{n+1}, (rho u)*, e*                          (steps (i)-(iii))
                 hp_pressure_rhs    b = dt^2 f of eq. fpoiss                          (steps (iv)-(v))
                 hp_update_coefficients_two_density(rho^n, rho^{n+1}, c_s^2, dt)
                 hp_solve           predicted pressure, from P^n                     (step (vi))
                 hp_pressure_update (rho u)^{n+1}, interface velocities, e^{n+1}     (steps (vii)-(ix))
    time step:   U1 = L(U^n); U2 = L(U1); U^{n+1} = (U^n + U2) / 2 (hp_axpby): the second-order
                 TVD Runge-Kutta scheme with the whole fractional step in every stage, the variant
                 the paper uses.

The paper's explicit part uses fifth-order WENO; hp_advect uses second-order ENO of the same
family. Used for the Gresho-vortex Mach ladder of Section 5.
"""
from __future__ import annotations

import paper_1112_3507_amd as hp


class SemiImplicitStepper:
    """State (rho, rho u, e) on the device and one solver handle on its grid."""

    def __init__(self, n, h, bc, dt, gamma, rho, mom, e, tol=1e-10, mode=None):
        import torch
        self.n, self.h, self.bc = tuple(n), tuple(h), tuple(bc)
        self.dt, self.gamma, self.tol = float(dt), float(gamma), float(tol)
        dev = rho.device
        shape = rho.shape
        f = lambda: torch.empty(shape, dtype=torch.float64, device=dev)
        m = lambda: torch.empty((3,) + tuple(shape), dtype=torch.float64, device=dev)
        self.rho, self.mom, self.e = rho.clone(), mom.clone(), e.clone()     # U^n
        self.u1 = (f(), m(), f())
        self.u2 = (f(), m(), f())
        self.p, self.c2, self.b, self.x = f(), f(), f(), f()
        self.mom_s, self.e_s, self.uf = m(), f(), m()
        # the handle's coefficients are replaced before every solve; it starts from rho for both
        self.solver = hp.setup(self.n, self.h, self.bc, self.rho, self.rho, self.dt,
                               hp.MODE_FP64_MGPCG if mode is None else mode)
        self.stats = []

    def close(self):
        self.solver.close()

    def pressure(self, out=None):
        """P of the current state (step (x))."""
        import torch
        p = out if out is not None else torch.empty_like(self.rho)
        self.solver.eos_ideal(self.rho, self.mom, self.e, self.gamma, p)
        return p

    def stage(self, rho, mom, e, out):
        """One whole fractional step L from (rho, mom, e) into out = (rho', mom', e')."""
        s = self.solver
        rho1, mom1, e1 = out
        s.eos_ideal(rho, mom, e, self.gamma, self.p, self.c2)
        s.advect(rho, mom, e, rho1, self.mom_s, self.e_s)
        s.pressure_rhs(rho, self.c2, self.p, mom, rho1, self.mom_s, self.b)
        s.update_coefficients(rho, self.c2, self.dt, rho_face=rho1)
        hp.stream_copy(self.p, self.x)           # the solve starts from P^n
        st = s.solve(self.b, self.x, tol=self.tol)
        s.pressure_update(self.x, rho1, self.mom_s, self.e_s, mom1, self.uf, e1)
        self.stats.append(st)
        return st

    def step(self):
        """One time step (two stages and the average)."""
        self.stage(self.rho, self.mom, self.e, self.u1)
        self.stage(*self.u1, self.u2)
        s = self.solver
        for cur, new in zip((self.rho, self.mom, self.e), self.u2):
            s.axpby(0.5, new, 0.5, cur)
