"""Host-side time loop around the C ABI.

Sec. 3.2: the first step's outer tolerance is 1e-4, later steps use
min(1e-4, dt * eps_s) with eps_s the previous step's rate of change; Sec. 4.1:
a steady run stops when the spatially averaged rate of change falls below a
tolerance. The first step of a run without a known u^{n-1} uses BDF1.
"""
from __future__ import annotations

import torch

from . import binding as B


def outer_tolerance(dt: float, eps_prev: float | None, first: bool, cap: float = 1e-4) -> float:
    return cap if first or eps_prev is None else min(cap, dt * eps_prev)


class Solver:
    """Stencils, operators and fields of one point cloud, resident on one GPU."""

    def __init__(self, ctx: B.Context, cloud, poly_degree: int, q: int = 0, phs_power: int = 3,
                 precision: int = B.RBFFD_FP64, device: str = "cuda"):
        self.ctx = ctx
        self.dcloud = B.DeviceCloud.from_numpy(cloud, device) if not isinstance(cloud, B.DeviceCloud) else cloud
        self.k = poly_degree
        self.phs = phs_power
        self.precision = precision
        self.nbr, self.w, _ = B.rbffd_build_stencils(ctx, self.dcloud, poly_degree, q, phs_power)
        self.q = self.nbr.shape[1]
        self.ops = B.rbffd_assemble(ctx, self.dcloud, self.nbr, self.w, poly_degree, self.q, phs_power, precision)

    @property
    def n(self) -> int:
        return self.dcloud.n

    @property
    def dim(self) -> int:
        return self.dcloud.dim

    def cylinder_forces(self, u: torch.Tensor, p: torch.Tensor, centre, diameter: float, mu: float,
                        nsurf: int = 360, rho: float | None = None, u_ref: float | None = None,
                        return_traction: bool = False):
        """Force (and with rho, u_ref the drag and lift coefficients) on a
        circular cylinder of this 2D cloud; see B.rbffd_cylinder_forces."""
        return B.rbffd_cylinder_forces(self.ctx, self.dcloud, self.ops, u.contiguous(), p.contiguous(), centre, diameter,
                                       mu, nsurf, rho, u_ref, return_traction)

    def dt_from_courant(self, u0: torch.Tensor, co: float, rho: float, mu: float, iters: int = 200) -> float:
        lam = B.rbffd_convdiff_lambda(self.ctx, self.ops, u0.contiguous(), rho, mu, iters)
        return 2.0 * co / lam

    def step(self, u, u_prev, p, u_bc, rho, mu, dt, alpha=B.BDF2, **kw):
        return B.simple_step(self.ctx, self.ops, u, u_prev, p, u_bc, rho, mu, dt, alpha,
                             precision=kw.pop("precision", self.precision), **kw)

    def run_steady(self, u, p, u_bc, rho, mu, dt, steady_tol=1e-8, max_steps=100000, krylov_factor=1e-2,
                   krylov_floor=1e-13, max_outer=50, max_krylov=5000, callback=None, p_bc=None):
        """March from (u, p) with constant Dirichlet data until the steady error
        max_c mean|u^{n+1} - u^n| / dt <= steady_tol; u, p are updated in place."""
        u_prev = u.clone()
        eps = None
        hist = []
        for step in range(max_steps):
            tol_o = outer_tolerance(dt, eps, first=(step == 0))
            tol_k = max(krylov_floor, krylov_factor * tol_o)
            st = self.step(u, u_prev, p, u_bc, rho, mu, dt, B.BDF1 if step == 0 else B.BDF2,
                           tol_outer=tol_o, tol_krylov=tol_k, max_outer=max_outer, max_krylov=max_krylov,
                           p_bc=p_bc)
            eps = st["eps_steady"]
            hist.append(st)
            if callback:
                callback(step, st)
            if eps <= steady_tol:
                break
        return hist

    def run_transient(self, u, u_prev, p, bc_fn, rho, mu, dt, nsteps, t0=0.0, first_bdf1=False, tol_outer=1e-8,
                      tol_krylov=1e-10, max_outer=50, max_krylov=5000, callback=None, pbc_fn=None):
        """nsteps steps from t0 with Dirichlet data bc_fn(t) -> device [dim, n] and,
        on prescribed-pressure points, pbc_fn(t) -> device [n]."""
        hist = []
        for step in range(nsteps):
            t_next = t0 + (step + 1) * dt
            alpha = B.BDF1 if (step == 0 and first_bdf1) else B.BDF2
            st = self.step(u, u_prev, p, bc_fn(t_next), rho, mu, dt, alpha, tol_outer=tol_outer,
                           tol_krylov=tol_krylov, max_outer=max_outer, max_krylov=max_krylov,
                           p_bc=None if pbc_fn is None else pbc_fn(t_next))
            hist.append(st)
            if callback:
                callback(step, st)
        return hist
