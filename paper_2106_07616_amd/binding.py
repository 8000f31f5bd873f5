"""ctypes binding of librbffd.so (the gfx950 HIP library declared in include/rbffd.h).

Argument marshalling only: every computation runs in the library's kernels.
Device arrays are torch tensors on a ROCm device; work is enqueued on torch's
current stream. There is no CPU fallback: importing this module on a machine
without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbffd.so")

RBFFD_OK, RBFFD_E_ARG, RBFFD_E_OOM, RBFFD_E_SINGULAR = 0, -1, -2, -3
RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN, RBFFD_E_DEVICE = -4, -5, -6
RBFFD_FP64, RBFFD_FP32_IR, RBFFD_FP32_MATRIX = 0, 1, 2
RBFFD_PREC_JACOBI, RBFFD_PREC_BLOCK64 = 0, 1
RBFFD_NOALLOC_MAX_N = 1179648   # rows the allocation-free solve's scratch array holds
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_OOM", -3: "E_SINGULAR", -4: "E_NOCONV",
                -5: "E_BREAKDOWN", -6: "E_DEVICE"}

EXPORTED = ["rbffd_last_error", "rbffd_ctx_create", "rbffd_ctx_destroy", "rbffd_ctx_bytes_in_use",
            "rbffd_ctx_set_graphs", "rbffd_ctx_set_solver_choice", "rbffd_autotune_krylov",
            "rbffd_stencil_sizes", "rbffd_build_stencils", "rbffd_build_stencils_batched", "rbffd_assemble",
            "rbffd_ops_free",
            "rbffd_ops_info", "rbffd_ops_export_csr", "rbffd_ops_export_block_inverse", "rbffd_apply", "rbffd_interpolate", "rbffd_cylinder_forces", "poisson_solve",
            "poisson_solve_noalloc", "poisson_solve_batched", "rbffd_krylov_kernel_times",
            "rbffd_server_create", "rbffd_server_destroy", "rbffd_server_submit", "rbffd_server_run",
            "rbffd_server_poll", "simple_step", "simple_step_batched", "rbffd_convdiff_lambda"]


class RbffdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class CloudT(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64), ("xyz", C.c_void_p), ("kind", C.c_void_p),
                ("normal", C.c_void_p), ("pin", C.c_int64), ("period", C.c_double * 3)]


class StencilOptsT(C.Structure):
    _fields_ = [("phs_power", C.c_int), ("poly_degree", C.c_int), ("q", C.c_int)]


class KrylovOptsT(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int), ("preconditioner", C.c_int)]


class KrylovStatsT(C.Structure):
    _fields_ = [("iters", C.c_int), ("status", C.c_int), ("refinements", C.c_int), ("fp64_fallback", C.c_int),
                ("relres", C.c_double)]


class StepOptsT(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double), ("alpha", C.c_double * 3),
                ("tol_outer", C.c_double), ("tol_krylov", C.c_double), ("max_outer", C.c_int),
                ("max_krylov", C.c_int), ("precision", C.c_int), ("preconditioner", C.c_int),
                ("force", C.c_double * 3)]


class StepStatsT(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("krylov_mom", C.c_int), ("krylov_p", C.c_int),
                ("krylov_b", C.c_int), ("status", C.c_int), ("delta", C.c_double),
                ("eps_steady", C.c_double), ("div_l1", C.c_double), ("final_relres_p", C.c_double),
                ("krylov_relres_max", C.c_double)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"the HIP library {path} is not built; run __graft_entry__.build()")
    L = C.CDLL(path)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    L.rbffd_last_error.restype = C.c_char_p
    L.rbffd_ctx_create.argtypes = [C.POINTER(P), I, C.c_size_t]
    L.rbffd_ctx_destroy.argtypes = [P]
    L.rbffd_ctx_bytes_in_use.argtypes = [P]
    L.rbffd_ctx_set_graphs.argtypes = [P, I]
    L.rbffd_ctx_set_solver_choice.argtypes = [P, I64, I, I]
    L.rbffd_autotune_krylov.argtypes = [P, P, I, C.POINTER(I), C.POINTER(D), P]
    L.rbffd_ctx_bytes_in_use.restype = C.c_size_t
    L.rbffd_stencil_sizes.argtypes = [I, C.POINTER(StencilOptsT), C.POINTER(I), C.POINTER(I), C.POINTER(I)]
    L.rbffd_build_stencils.argtypes = [P, C.POINTER(CloudT), C.POINTER(StencilOptsT), P, P, C.POINTER(I64), P]
    L.rbffd_build_stencils_batched.argtypes = [P, I, C.POINTER(CloudT), C.POINTER(StencilOptsT), C.POINTER(P),
                                               C.POINTER(P), C.POINTER(I64), P]
    L.rbffd_assemble.argtypes = [P, C.POINTER(CloudT), C.POINTER(StencilOptsT), P, P, I, C.POINTER(P), P]
    L.rbffd_ops_free.argtypes = [P]
    L.rbffd_ops_info.argtypes = [P, C.POINTER(I64), C.POINTER(I), C.POINTER(I), C.POINTER(I64)]
    L.rbffd_ops_export_csr.argtypes = [P, P, P, P]
    L.rbffd_ops_export_block_inverse.argtypes = [P, P, P]
    L.rbffd_apply.argtypes = [P, P, I, P, P, P]
    L.rbffd_interpolate.argtypes = [P, C.POINTER(CloudT), C.POINTER(StencilOptsT), I64, P, I, P, P, P, P,
                                    C.POINTER(I64), P]
    L.rbffd_cylinder_forces.argtypes = [P, C.POINTER(CloudT), P, P, P, C.POINTER(D), D, D, I, D, D, C.POINTER(D),
                                        C.POINTER(D), P, C.POINTER(I64), P]
    L.poisson_solve.argtypes = [P, P, P, P, C.POINTER(KrylovOptsT), C.POINTER(KrylovStatsT), P]
    L.rbffd_krylov_kernel_times.argtypes = [P, P, P, P, I, C.POINTER(D), P]
    L.poisson_solve_noalloc.argtypes = [P, P, P, C.POINTER(KrylovOptsT), C.POINTER(KrylovStatsT), P]
    L.poisson_solve_batched.argtypes = [P, I, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(KrylovOptsT),
                                        C.POINTER(KrylovStatsT), P]
    L.rbffd_server_create.argtypes = [P, C.POINTER(P)]
    L.rbffd_server_destroy.argtypes = [P]
    L.rbffd_server_submit.argtypes = [P, P, P, P, C.POINTER(KrylovOptsT), C.POINTER(I64)]
    L.rbffd_server_run.argtypes = [P, I, C.POINTER(I), P]
    L.rbffd_server_poll.argtypes = [P, I, C.POINTER(I64), C.POINTER(KrylovStatsT), C.POINTER(I)]
    L.simple_step.argtypes = [P, P, P, P, P, P, P, C.POINTER(StepOptsT), C.POINTER(StepStatsT), P]
    L.simple_step_batched.argtypes = [P, I, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                      C.POINTER(P), C.POINTER(StepOptsT), C.POINTER(StepStatsT), P]
    L.rbffd_convdiff_lambda.argtypes = [P, P, P, D, D, I, C.POINTER(D), P]
    return L


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(code: int, allow=()):
    if code != RBFFD_OK and code not in allow:
        raise RbffdError(code, lib().rbffd_last_error().decode())
    return code


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor | None, numel: int, what: str):
    """Pointer to a contiguous FP64 device tensor of exactly `numel` entries:
    the library takes raw pointers and trusts their extents."""
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise ValueError(f"{what}: float64 tensor expected, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{what}: {numel} entries expected, got {t.numel()}")
    return _ptr(t)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """rbffd_ctx: a device, an HBM budget (bytes, 0 = none), and workspace."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.device = device
        h = C.c_void_p()
        _check(lib().rbffd_ctx_create(C.byref(h), device, hbm_budget_bytes))
        self.handle = h

    def bytes_in_use(self) -> int:
        return lib().rbffd_ctx_bytes_in_use(self.handle)

    def set_solver_choice(self, n: int, q: int, choice: int):
        """FP64 Jacobi BiCGSTAB path for systems of (n, q): 0 multi-kernel,
        256 / 512 / 1024 one workgroup of that many threads, -1 the default."""
        _check(lib().rbffd_ctx_set_solver_choice(self.handle, int(n), int(q), int(choice)))

    def set_graphs(self, enable: bool):
        """Replay BiCGSTAB iteration chunks as HIP graphs or launch them kernel
        by kernel (the default); the results are bitwise the same."""
        _check(lib().rbffd_ctx_set_graphs(self.handle, int(bool(enable))))

    def close(self):
        if self.handle:
            lib().rbffd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class DeviceCloud:
    dim: int
    n: int
    xyz: torch.Tensor      # [n, dim] float64
    kind: torch.Tensor     # [n] uint8
    normal: torch.Tensor   # [n, dim] float64
    pin: int
    period: tuple = (0.0, 0.0, 0.0)   # > 0: periodic along that axis

    @staticmethod
    def from_numpy(cloud, device="cuda"):
        return DeviceCloud(cloud.dim, cloud.n,
                           torch.as_tensor(cloud.xyz, dtype=torch.float64, device=device).contiguous(),
                           torch.as_tensor(cloud.kind, dtype=torch.uint8, device=device).contiguous(),
                           torch.as_tensor(cloud.normal, dtype=torch.float64, device=device).contiguous(),
                           int(cloud.pin), tuple(float(v) for v in getattr(cloud, "period", (0.0, 0.0, 0.0))))

    def struct(self) -> CloudT:
        return CloudT(self.dim, self.n, _ptr(self.xyz), _ptr(self.kind), _ptr(self.normal), self.pin,
                      (C.c_double * 3)(*self.period))


def rbffd_stencil_sizes(dim: int, poly_degree: int, q: int = 0, phs_power: int = 3):
    o = StencilOptsT(phs_power, poly_degree, q)
    qq, mm, rr = C.c_int(), C.c_int(), C.c_int()
    _check(lib().rbffd_stencil_sizes(dim, C.byref(o), C.byref(qq), C.byref(mm), C.byref(rr)))
    return qq.value, mm.value, rr.value


def rbffd_build_stencils(ctx: Context, cloud: DeviceCloud, poly_degree: int, q: int = 0, phs_power: int = 3,
                         allow_singular: bool = False):
    """Clouds nbr[n, q] (int32) and weights w[R, n, q] (float64) on the device."""
    q, m, R = rbffd_stencil_sizes(cloud.dim, poly_degree, q, phs_power)
    dev = cloud.xyz.device
    nbr = torch.empty((cloud.n, q), dtype=torch.int32, device=dev)
    w = torch.empty((R, cloud.n, q), dtype=torch.float64, device=dev)
    o = StencilOptsT(phs_power, poly_degree, q)
    cs = cloud.struct()
    bad = C.c_int64(-1)
    st = lib().rbffd_build_stencils(ctx.handle, C.byref(cs), C.byref(o), _ptr(nbr), _ptr(w), C.byref(bad), _stream())
    _check(st, allow=(RBFFD_E_SINGULAR,) if allow_singular else ())
    return nbr, w, bad.value


def rbffd_build_stencils_batched(ctx: Context, clouds: list, poly_degrees: list, qs: list | None = None,
                                 phs_powers: list | None = None, allow_singular: bool = False):
    """Clouds and weights of many clouds (one weight launch per dimension):
    returns (nbr list, w list, bad-point list)."""
    count = len(clouds)
    qs = qs or [0] * count
    phs_powers = phs_powers or [3] * count
    cl = (CloudT * count)(*[c.struct() for c in clouds])
    op = (StencilOptsT * count)(*[StencilOptsT(ph, k, q) for ph, k, q in zip(phs_powers, poly_degrees, qs)])
    nbrs, ws = [], []
    for c, k, q, ph in zip(clouds, poly_degrees, qs, phs_powers):
        qq, _, R = rbffd_stencil_sizes(c.dim, k, q, ph)
        nbrs.append(torch.empty((c.n, qq), dtype=torch.int32, device=c.xyz.device))
        ws.append(torch.empty((R, c.n, qq), dtype=torch.float64, device=c.xyz.device))
    pn = (C.c_void_p * count)(*[_ptr(t) for t in nbrs])
    pw = (C.c_void_p * count)(*[_ptr(t) for t in ws])
    bad = (C.c_int64 * count)()
    st = lib().rbffd_build_stencils_batched(ctx.handle, count, cl, op, pn, pw, bad, _stream())
    _check(st, allow=(RBFFD_E_SINGULAR,) if allow_singular else ())
    return nbrs, ws, list(bad)


def rbffd_interpolate(ctx: Context, cloud: DeviceCloud, poly_degree: int, qxyz: torch.Tensor,
                      fields: torch.Tensor | None = None, q: int = 0, phs_power: int = 3,
                      return_stencils: bool = False):
    """Interpolated fields out[nfield, nq] at the query points qxyz[nq, dim]
    from fields[nfield, n] on the cloud; with return_stencils, also the
    clouds nbr[nq, q] and weights w[nq, q]."""
    q, m, R = rbffd_stencil_sizes(cloud.dim, poly_degree, q, phs_power)
    dev = cloud.xyz.device
    if qxyz.dim() != 2 or qxyz.shape[1] != cloud.dim:
        raise ValueError(f"qxyz must be [nq, {cloud.dim}]")
    nq = qxyz.shape[0]
    nf = 0
    if fields is not None:
        if fields.dim() == 1:
            fields = fields.reshape(1, -1)
        nf = fields.shape[0]
        _f64(fields, nf * cloud.n, "fields")
    out = torch.empty((nf, nq), dtype=torch.float64, device=dev) if nf else None
    nbr = torch.empty((nq, q), dtype=torch.int32, device=dev) if return_stencils else None
    w = torch.empty((nq, q), dtype=torch.float64, device=dev) if return_stencils else None
    o = StencilOptsT(phs_power, poly_degree, q)
    cs = cloud.struct()
    bad = C.c_int64(-1)
    _check(lib().rbffd_interpolate(ctx.handle, C.byref(cs), C.byref(o), nq, _f64(qxyz, nq * cloud.dim, "qxyz"), nf,
                                   _ptr(fields) if nf else None, _ptr(out), _ptr(nbr), _ptr(w), C.byref(bad),
                                   _stream()))
    if return_stencils:
        return out, nbr, w
    return out


def rbffd_cylinder_forces(ctx: Context, cloud: DeviceCloud, ops: "Operators", u: torch.Tensor, p: torch.Tensor,
                          centre, diameter: float, mu: float, nsurf: int = 360, rho: float | None = None,
                          u_ref: float | None = None, return_traction: bool = False):
    """Force per unit length (F_x, F_y) on a circular cylinder of a 2D flow
    from its surface stresses; with rho and u_ref also (C_D, C_L); with
    return_traction also the traction [2, nsurf] at the surface points.
    u: [2, n] velocity, p: [n] pressure on the cloud."""
    n = cloud.n
    f = (C.c_double * 2)()
    cf = (C.c_double * 2)() if (rho is not None and u_ref is not None) else None
    tr = torch.empty((2, nsurf), dtype=torch.float64, device=cloud.xyz.device) if return_traction else None
    cen = (C.c_double * 2)(float(centre[0]), float(centre[1]))
    cs = cloud.struct()
    bad = C.c_int64(-1)
    _check(lib().rbffd_cylinder_forces(ctx.handle, C.byref(cs), ops.handle, _f64(u, 2 * n, "u"), _f64(p, n, "p"), cen,
                                       float(diameter), float(mu), int(nsurf), float(rho or 0.0), float(u_ref or 0.0),
                                       f, cf, _ptr(tr), C.byref(bad), _stream()))
    out = [[f[0], f[1]]]
    if cf is not None:
        out.append([cf[0], cf[1]])
    if return_traction:
        out.append(tr)
    return out[0] if len(out) == 1 else tuple(out)


class Operators:
    """rbffd_ops handle (library-owned device operators)."""

    def __init__(self, handle, ctx: Context, cloud: DeviceCloud, poly_degree: int, q: int, precision: int):
        self.handle = handle
        self.ctx = ctx
        self.cloud = cloud
        self.k = poly_degree
        self.q = q
        self.precision = precision
        n, qq, dim, nb = C.c_int64(), C.c_int(), C.c_int(), C.c_int64()
        _check(lib().rbffd_ops_info(handle, C.byref(n), C.byref(qq), C.byref(dim), C.byref(nb)))
        self.n, self.dim, self.n_boundary = n.value, dim.value, nb.value

    def export_csr(self):
        col = torch.empty((self.n, self.q), dtype=torch.int32, device=self.cloud.xyz.device)
        val = torch.empty((self.dim + 2, self.n, self.q), dtype=torch.float64, device=self.cloud.xyz.device)
        _check(lib().rbffd_ops_export_csr(self.handle, _ptr(col), _ptr(val), _stream()))
        return col, val

    def export_block_inverse(self):
        """[ceil(n/64), 64 (column), 64 (row)] inverses of the diagonal blocks
        (the solver's FP16 values times their per-block scale, in FP32)."""
        nb = (self.n + 63) // 64
        out = torch.empty((nb, 64, 64), dtype=torch.float32, device=self.cloud.xyz.device)
        _check(lib().rbffd_ops_export_block_inverse(self.handle, _ptr(out), _stream()))
        return out

    def apply(self, which: int, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        _check(lib().rbffd_apply(self.ctx.handle, self.handle, which, _f64(x, self.n, "x"), _ptr(y), _stream()))
        return y

    def free(self):
        if self.handle:
            lib().rbffd_ops_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rbffd_assemble(ctx: Context, cloud: DeviceCloud, nbr: torch.Tensor, w: torch.Tensor, poly_degree: int,
                   q: int = 0, phs_power: int = 3, precision: int = RBFFD_FP64) -> Operators:
    q, m, R = rbffd_stencil_sizes(cloud.dim, poly_degree, q, phs_power)
    o = StencilOptsT(phs_power, poly_degree, q)
    cs = cloud.struct()
    h = C.c_void_p()
    _check(lib().rbffd_assemble(ctx.handle, C.byref(cs), C.byref(o), _ptr(nbr), _ptr(w), precision, C.byref(h),
                                _stream()))
    return Operators(h, ctx, cloud, poly_degree, q, precision)


def poisson_solve(ctx: Context, ops: Operators, rhs: torch.Tensor, x: torch.Tensor, tol: float = 1e-10,
                  max_iter: int = 5000, precision: int = RBFFD_FP64, allow_noconv: bool = False,
                  preconditioner: int = RBFFD_PREC_JACOBI):
    o = KrylovOptsT(tol, max_iter, precision, preconditioner)
    s = KrylovStatsT()
    st = lib().poisson_solve(ctx.handle, ops.handle, _f64(rhs, ops.n, "rhs"), _f64(x, ops.n, "x"), C.byref(o),
                             C.byref(s), _stream())
    _check(st, allow=(RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN) if allow_noconv else ())
    return dict(iters=s.iters, status=s.status, refinements=s.refinements, fp64_fallback=s.fp64_fallback,
                relres=s.relres)


def rbffd_krylov_kernel_times(ctx: Context, ops: Operators, rhs: torch.Tensor, x: torch.Tensor, reps: int = 100):
    """Mean kernel durations (us) of one FP64 Jacobi BiCGSTAB iteration on the
    pressure-correction matrix: dict kv, ks, kt, kx, iteration."""
    us = (C.c_double * 5)()
    _check(lib().rbffd_krylov_kernel_times(ctx.handle, ops.handle, _f64(rhs, ops.n, "rhs"), _f64(x, ops.n, "x"),
                                           reps, us, _stream()))
    return dict(zip(("kv", "ks", "kt", "kx", "iteration"), list(us)))


def rbffd_autotune_krylov(ctx: Context, ops: Operators, iterations: int = 40):
    """Time the solver paths on the operators' pressure-correction system and
    record the fastest for its size: returns (choice, {choice: us/iteration})."""
    ch = C.c_int(-1)
    us = (C.c_double * 4)()
    _check(lib().rbffd_autotune_krylov(ctx.handle, ops.handle, iterations, C.byref(ch), us, _stream()))
    return ch.value, {c: v for c, v in zip((0, 256, 512, 1024), list(us)) if v >= 0}


def poisson_solve_noalloc(ops: Operators, rhs: torch.Tensor, x: torch.Tensor, tol: float = 1e-10,
                          max_iter: int = 5000, allow_noconv: bool = False):
    """poisson_solve (FP64, Jacobi) with its workspace in the library's fixed
    device scratch array: allocates nothing."""
    o = KrylovOptsT(tol, max_iter, RBFFD_FP64, RBFFD_PREC_JACOBI)
    s = KrylovStatsT()
    st = lib().poisson_solve_noalloc(ops.handle, _f64(rhs, ops.n, "rhs"), _f64(x, ops.n, "x"), C.byref(o),
                                     C.byref(s), _stream())
    _check(st, allow=(RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN) if allow_noconv else ())
    return dict(iters=s.iters, status=s.status, relres=s.relres)


def poisson_solve_batched(ctx: Context, ops: list, rhs: list, x: list, tol: float = 1e-10, max_iter: int = 5000,
                          allow_noconv: bool = False, preconditioner: int = RBFFD_PREC_JACOBI,
                          precision: int = RBFFD_FP64):
    """Pressure-correction solves of several independent systems in one batch
    (FP64, or FP32 matrix values with FP64 vectors and residuals); x[j] is
    updated in place. Returns one stats dict per system."""
    m = len(ops)
    if not (m == len(rhs) == len(x)) or m == 0:
        raise ValueError("ops, rhs and x must be non-empty lists of the same length")
    arr = C.c_void_p * m
    o = KrylovOptsT(tol, max_iter, precision, preconditioner)
    stats = (KrylovStatsT * m)()
    rp = [_f64(t, op.n, f"rhs[{j}]") for j, (t, op) in enumerate(zip(rhs, ops))]
    xp = [_f64(t, op.n, f"x[{j}]") for j, (t, op) in enumerate(zip(x, ops))]
    st = lib().poisson_solve_batched(ctx.handle, m, arr(*[op.handle for op in ops]), arr(*rp), arr(*xp),
                                     C.byref(o), stats, _stream())
    _check(st, allow=(RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN) if allow_noconv else ())
    return [dict(iters=s_.iters, status=s_.status, relres=s_.relres) for s_ in stats]


class Server:
    """Continuous batching of FP64 pressure-correction solves (rbffd_server_*)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().rbffd_server_create(ctx.handle, C.byref(h)))
        self.handle = h
        self._keep = {}   # ticket -> tensors that must outlive the solve

    def submit(self, ops: Operators, rhs: torch.Tensor, x: torch.Tensor, tol: float = 1e-6,
               max_iter: int = 20000, preconditioner: int = RBFFD_PREC_JACOBI, precision: int = RBFFD_FP64) -> int:
        t = C.c_int64()
        o = KrylovOptsT(tol, max_iter, precision, preconditioner)
        _check(lib().rbffd_server_submit(self.handle, ops.handle, _f64(rhs, ops.n, "rhs"), _f64(x, ops.n, "x"),
                                         C.byref(o), C.byref(t)))
        self._keep[t.value] = (ops, rhs, x)
        return t.value

    def run(self, iterations: int = 32) -> int:
        a = C.c_int()
        _check(lib().rbffd_server_run(self.handle, iterations, C.byref(a), _stream()))
        return a.value

    def poll(self, max_items: int = 1024):
        tickets = (C.c_int64 * max_items)()
        stats = (KrylovStatsT * max_items)()
        cnt = C.c_int()
        _check(lib().rbffd_server_poll(self.handle, max_items, tickets, stats, C.byref(cnt)))
        out = []
        for i in range(cnt.value):
            self._keep.pop(tickets[i], None)
            out.append((tickets[i], dict(iters=stats[i].iters, status=stats[i].status, relres=stats[i].relres)))
        return out

    def close(self):
        if self.handle:
            lib().rbffd_server_destroy(self.handle)
            self.handle = None


BDF2 = (1.5, -2.0, 0.5)
BDF1 = (1.0, -1.0, 0.0)


def simple_step(ctx: Context, ops: Operators, u: torch.Tensor, u_prev: torch.Tensor, p: torch.Tensor,
                u_bc: torch.Tensor, rho: float, mu: float, dt: float, alpha=BDF2, tol_outer: float = 1e-6,
                tol_krylov: float = 1e-10, max_outer: int = 50, max_krylov: int = 5000,
                precision: int = RBFFD_FP64, p_bc: torch.Tensor | None = None,
                preconditioner: int = RBFFD_PREC_JACOBI, force=(0.0, 0.0, 0.0)):
    """One time step in place on u [dim, n], u_prev [dim, n], p [n]; returns stats.
    p_bc [n]: pressure at t^{n+1} on prescribed-pressure points. A limit reached
    (E_NOCONV) or a Krylov breakdown (E_BREAKDOWN) is reported in the stats,
    not raised."""
    o = StepOptsT(rho, mu, dt, (C.c_double * 3)(*alpha), tol_outer, tol_krylov, max_outer, max_krylov, precision,
                  preconditioner, (C.c_double * 3)(*(tuple(force) + (0.0,) * (3 - len(force)))))
    s = StepStatsT()
    dn = ops.dim * ops.n
    st = lib().simple_step(ctx.handle, ops.handle, _f64(u, dn, "u"), _f64(u_prev, dn, "u_prev"), _f64(p, ops.n, "p"),
                           _f64(u_bc, dn, "u_bc"), _f64(p_bc, ops.n, "p_bc"), C.byref(o), C.byref(s), _stream())
    _check(st, allow=(RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN))
    return dict(outer_iters=s.outer_iters, krylov_mom=s.krylov_mom, krylov_p=s.krylov_p, krylov_b=s.krylov_b,
                status=s.status, delta=s.delta, eps_steady=s.eps_steady, div_l1=s.div_l1,
                final_relres_p=s.final_relres_p, krylov_relres_max=s.krylov_relres_max)


def _stats_dict(s):
    return dict(outer_iters=s.outer_iters, krylov_mom=s.krylov_mom, krylov_p=s.krylov_p, krylov_b=s.krylov_b,
                status=s.status, delta=s.delta, eps_steady=s.eps_steady, div_l1=s.div_l1,
                final_relres_p=s.final_relres_p, krylov_relres_max=s.krylov_relres_max)


def simple_step_batched(ctx: Context, ops: list, u: list, u_prev: list, p: list, u_bc: list, rho: float, mu: float,
                        dts: list, alpha=BDF2, tol_outer=1e-6, tol_krylov: float = 1e-10, max_outer: int = 50,
                        max_krylov: int = 5000, p_bc: list | None = None, preconditioner: int = RBFFD_PREC_JACOBI):
    """One time step of many clouds at once, in place on each cloud's u, u_prev,
    p (FP64); dts[j] is cloud j's time step, tol_outer a value for all or one
    per cloud. Returns the list of per-cloud stats; limits reached and
    breakdowns are reported there, not raised."""
    cnt = len(ops)
    tols = list(tol_outer) if isinstance(tol_outer, (list, tuple)) else [tol_outer] * cnt
    if not (len(u) == len(u_prev) == len(p) == len(u_bc) == len(dts) == cnt):
        raise ValueError("one entry per cloud in every list")
    p_bc = p_bc or [None] * cnt
    PA = C.c_void_p * cnt
    hs = (C.c_void_p * cnt)(*[o.handle.value if hasattr(o.handle, "value") else o.handle for o in ops])
    uu = PA(*[_f64(a, o.dim * o.n, "u") for a, o in zip(u, ops)])
    up = PA(*[_f64(a, o.dim * o.n, "u_prev") for a, o in zip(u_prev, ops)])
    pp = PA(*[_f64(a, o.n, "p") for a, o in zip(p, ops)])
    ub = PA(*[_f64(a, o.dim * o.n, "u_bc") for a, o in zip(u_bc, ops)])
    pb = PA(*[_f64(a, o.n, "p_bc") for a, o in zip(p_bc, ops)])
    opts = (StepOptsT * cnt)(*[StepOptsT(rho, mu, dt, (C.c_double * 3)(*alpha), to, tol_krylov, max_outer,
                                         max_krylov, RBFFD_FP64, preconditioner, (C.c_double * 3)(0.0, 0.0, 0.0))
                               for dt, to in zip(dts, tols)])
    stats = (StepStatsT * cnt)()
    st = lib().simple_step_batched(ctx.handle, cnt, hs, uu, up, pp, ub, pb, opts, stats, _stream())
    _check(st, allow=(RBFFD_E_NOCONV, RBFFD_E_BREAKDOWN))
    return [_stats_dict(s) for s in stats]


def rbffd_convdiff_lambda(ctx: Context, ops: Operators, u0: torch.Tensor, rho: float, mu: float,
                          iters: int = 200) -> float:
    lam = C.c_double()
    _check(lib().rbffd_convdiff_lambda(ctx.handle, ops.handle, _ptr(u0), rho, mu, iters, C.byref(lam), _stream()))
    return lam.value
