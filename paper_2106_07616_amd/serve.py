"""Serving flow requests on one GPU with continuous admission.

A request is a short flow solve on its own point cloud: its stencils and
operators (Sec. 2), then `steps` BDF time steps of the semi-implicit outer
iteration (Sec. 3, the step list of Sec. 3.2: the first step BDF1, the outer
tolerance min(1e-4, dt eps_s) after a first 1e-4, momentum and
pressure-correction Krylov solves to `tol_krylov`), from the exact flow at
t = 0 with the exact Dirichlet data of every step.

The server runs `slots` worker threads. Each holds its own library context and
its own HIP stream at the default priority, so the kernels of requests in
different slots run concurrently on the device: one request's operator build
overlaps another's Krylov iterations instead of pausing them. A queued request
is admitted when a slot is free and its device-memory estimate fits in what is
left of the HBM budget; its memory returns to the budget when it finishes. Every
kernel of the library is deterministic and a request's work touches only its
own buffers, so a request's result does not depend on what runs beside it.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .driver import Solver, outer_tolerance


@dataclass
class FlowRequest:
    """One flow solve: `cloud` is a workloads.Cloud whose meta names its
    closed-form flow (used for the initial state and the Dirichlet data)."""
    cloud: object
    poly_degree: int
    steps: int = 3
    courant: float = 5.0
    rho: float = 1.0
    tol_krylov: float = 1e-6
    max_outer: int = 5
    max_krylov: int = 20000
    flow_fields: object = None   # callable (cloud, t) -> (vel [dim, n], p [n])
    tag: object = None
    precision: int = B.RBFFD_FP64             # Krylov sweeps of the steps
    preconditioner: int = B.RBFFD_PREC_JACOBI  # of the pressure-correction solves


@dataclass
class FlowResult:
    tag: object
    u: np.ndarray
    p: np.ndarray
    stats: list
    dt: float
    t_queue: float = 0.0       # arrival -> admitted
    t_build: float = 0.0       # stencils + operators
    t_steps: float = 0.0       # the time steps
    latency: float = 0.0       # arrival -> result
    slot: int = -1
    bytes_reserved: int = 0
    extra: dict = field(default_factory=dict)


def estimate_bytes(dim: int, n: int, q: int) -> int:
    """Device bytes of one request: coordinates, normals and kinds; clouds and
    weights (4q + 8Rq); the sparse operators (4q + 2q column indices, 8Rq
    values, 8q pressure-correction and 8q momentum values); Krylov vectors
    (7 per right-hand side, up to d right-hand sides); the step's fields
    (8(4d + 4)) and the caller's fields and Dirichlet data (8 (4d + 2))."""
    R = dim + 1
    per = (16 * dim + 1) + (4 * q + 8 * R * q) + (6 * q + 8 * R * q + 16 * q + 16) + 56 * dim + 8 * (4 * dim + 4) \
        + 8 * (4 * dim + 2)
    return int(n * per)


def run_request(ctx: B.Context, req: FlowRequest) -> FlowResult:
    """The request's whole solve on the calling thread's current stream."""
    c = req.cloud
    ff = req.flow_fields
    dev = "cuda"
    t0 = time.perf_counter()
    sv = Solver(ctx, c, req.poly_degree, precision=req.precision)
    vel0, p0 = ff(c, 0.0)
    u = torch.tensor(vel0, device=dev)
    nu = float(c.meta.get("nu", 1.0 / c.meta.get("Re", 40.0)))
    dt = sv.dt_from_courant(u, req.courant, req.rho, nu * req.rho)
    velm, _ = ff(c, -dt)
    up = torch.tensor(velm, device=dev)
    p = torch.tensor(p0, device=dev)
    torch.cuda.current_stream().synchronize()
    t1 = time.perf_counter()
    stats = []
    eps = None
    for i in range(req.steps):
        ub, pb = ff(c, (i + 1) * dt)
        tol_o = outer_tolerance(dt, eps, first=(i == 0))
        st = sv.step(u, up, p, torch.tensor(ub, device=dev), req.rho, nu * req.rho, dt,
                     B.BDF1 if i == 0 else B.BDF2, tol_outer=tol_o, tol_krylov=req.tol_krylov,
                     max_outer=req.max_outer, max_krylov=req.max_krylov, p_bc=torch.tensor(pb, device=dev),
                     preconditioner=req.preconditioner)
        eps = st["eps_steady"]
        stats.append(st)
    res = FlowResult(req.tag, u.cpu().numpy(), p.cpu().numpy(), stats, dt)
    t2 = time.perf_counter()
    res.t_build, res.t_steps = t1 - t0, t2 - t1
    sv.ops.free()
    return res


class FlowServer:
    """Continuous admission of flow requests into `slots` concurrent workers
    under an HBM budget (bytes; 0 = no limit)."""

    def __init__(self, slots: int = 4, hbm_budget: int = 0, device: int = 0):
        B.lib()
        self.device = device
        self.budget = int(hbm_budget)
        self.reserved = 0
        self.peak_reserved = 0
        self.peak_active = 0
        self.active = 0
        self._cv = threading.Condition()
        self._queue: list = []          # (request, future, arrival time)
        self._stop = False
        self._threads = [threading.Thread(target=self._work, args=(i,), daemon=True) for i in range(slots)]
        for t in self._threads:
            t.start()

    def submit(self, req: FlowRequest, arrival: float | None = None) -> Future:
        """Queue a request; the future yields a FlowResult. `arrival` (a
        time.perf_counter() value) defaults to now."""
        fut: Future = Future()
        if req.flow_fields is None:
            import workloads as W
            req.flow_fields = W.flow_fields
        with self._cv:
            if self._stop:
                raise RuntimeError("server closed")
            self._queue.append((req, fut, time.perf_counter() if arrival is None else arrival))
            self._cv.notify_all()
        return fut

    def _bytes_of(self, req: FlowRequest) -> int:
        q, _, _ = B.rbffd_stencil_sizes(req.cloud.dim, req.poly_degree)
        return estimate_bytes(req.cloud.dim, req.cloud.n, q)

    def _take(self):
        """The first queued request that fits the budget (FIFO among those that
        fit; one that can never fit fails at once)."""
        with self._cv:
            while True:
                if self._stop and not self._queue:
                    return None
                for i, (req, fut, arr) in enumerate(self._queue):
                    need = self._bytes_of(req)
                    if self.budget and need > self.budget:
                        self._queue.pop(i)
                        fut.set_exception(B.RbffdError(B.RBFFD_E_OOM, f"request needs {need} bytes, budget "
                                                                      f"{self.budget}"))
                        break
                    if not self.budget or self.reserved + need <= self.budget:
                        self._queue.pop(i)
                        self.reserved += need
                        self.peak_reserved = max(self.peak_reserved, self.reserved)
                        self.active += 1
                        self.peak_active = max(self.peak_active, self.active)
                        return req, fut, arr, need
                else:
                    self._cv.wait()

    def _release(self, need):
        with self._cv:
            self.reserved -= need
            self.active -= 1
            self._cv.notify_all()

    def _work(self, slot: int):
        torch.cuda.set_device(self.device)
        ctx = B.Context(self.device)
        stream = torch.cuda.Stream()
        try:
            with torch.cuda.stream(stream):
                while True:
                    item = self._take()
                    if item is None:
                        return
                    req, fut, arrival, need = item
                    t_adm = time.perf_counter()
                    try:
                        res = run_request(ctx, req)
                        stream.synchronize()
                        res.t_queue = t_adm - arrival
                        res.latency = time.perf_counter() - arrival
                        res.slot = slot
                        res.bytes_reserved = need
                        fut.set_result(res)
                    except BaseException as e:   # handed to the caller through the future
                        fut.set_exception(e)
                    finally:
                        self._release(need)
        finally:
            ctx.close()

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def serve_stream(requests, arrivals, slots=4, hbm_budget=0):
    """Serve `requests` arriving at the given offsets (seconds from now) and
    return their results in submission order, with latencies from arrival."""
    results = [None] * len(requests)
    with FlowServer(slots, hbm_budget) as sv:
        t0 = time.perf_counter()
        futs = []
        for req, a in zip(requests, arrivals):
            now = time.perf_counter() - t0
            if now < a:
                time.sleep(a - now)
            futs.append(sv.submit(req, arrival=t0 + a))
        for i, f in enumerate(futs):
            results[i] = f.result()
        peak = sv.peak_active
    return results, peak


__all__ = ["FlowRequest", "FlowResult", "FlowServer", "estimate_bytes", "run_request", "serve_stream"]

