"""FP64 CPU oracle for the semi-implicit PHS-RBF method (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import this package. It shares no code with the HIP library: the C source
``rbffd_oracle.c`` is compiled here with gcc (``-O2 -ffp-contract=off``), and this
module only marshals numpy arrays into it and drives the time loop.

Function-to-paper map (Shahane & Vanka, arXiv 2106.07616):
  knn                -> Sec. 2 ("cloud of neighbouring points"), Sec. 3.1 (one-sided
                        clouds at boundaries)
  weights            -> Sec. 2, Eqs. RBF_interp, RBF_constraint, RBF_interp_mat_vec,
                        RBF_interp_L ... RBF_interp_mat_vec_L_solve (centre row of B1)
  interp_weights     -> Eq. RBF_interp evaluated away from the nodes
  cylinder_forces    -> Sec. 4, Eqs. cylinder forces, cylinder stress and cylinder
                        lift drag (surface stresses, Simpson's rule, C_D and C_L)
  csr                -> Sec. 2 closing remark: B1 precomputed and stored
  poisson_values     -> Eq. pressure poisson with the Sec. 3.1 boundary conditions
  bicgstab           -> Sec. 3 "preconditioned BiCGSTAB" (right Jacobi)
  simple_step        -> Sec. 3 Eqs. u:tilde ... p:correction, Eq. normal momentum,
                        and the eight-step summary of Sec. 3.2
  convdiff_lambda    -> Sec. 3.2: Courant number from the convection-diffusion
                        operator's extreme eigenvalue
  run_steady / run_transient -> Sec. 3.2 tolerance rule and Sec. 4.1 steady error
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbffd_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_lib = None

ORC_OK, ORC_E_ARG, ORC_E_OOM, ORC_E_SINGULAR, ORC_E_NOCONV = 0, -1, -2, -3, -4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            P = C.c_void_p
            i64 = C.c_int64
            L.orc_num_monomials.argtypes = [C.c_int, C.c_int]
            L.orc_monomial_exponents.argtypes = [C.c_int, C.c_int, P]
            L.orc_knn.argtypes = [C.c_int, i64, P, C.c_int, i64, P, P]
            L.orc_saddle_system.argtypes = [C.c_int, i64, P, C.c_int, P, C.c_int, C.c_int, i64, P, P, P]
            L.orc_weights.argtypes = [C.c_int, i64, P, C.c_int, P, C.c_int, C.c_int, i64, P, P, P]
            L.orc_interp_weights.argtypes = [C.c_int, P, C.c_int, P, P, C.c_int, C.c_int, P]
            L.orc_csr.argtypes = [i64, C.c_int, P, C.c_int, P, P, P]
            L.orc_spmv.argtypes = [i64, C.c_int, P, P, P, P]
            L.orc_spmv.restype = None
            L.orc_poisson_values.argtypes = [C.c_int, i64, C.c_int, P, P, i64, P, P, P, P]
            L.orc_bicgstab.argtypes = [i64, C.c_int, P, P, P, P, C.c_double, C.c_int, P, P]
            L.orc_simple_step.argtypes = [P, P, P, P, P, P, P]
            L.orc_convdiff_lambda.argtypes = [C.c_int, i64, C.c_int, P, P, P, P, C.c_double, C.c_double, C.c_int]
            L.orc_convdiff_lambda.restype = C.c_double
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_monomials(dim: int, k: int) -> int:
    return lib().orc_num_monomials(dim, k)


def monomial_exponents(dim: int, k: int) -> np.ndarray:
    m = num_monomials(dim, k)
    ex = np.zeros((m, 3), np.int32)
    lib().orc_monomial_exponents(dim, k, _p(ex))
    return ex


def default_q(dim: int, k: int) -> int:
    """Cloud size when none is given: twice the monomial count."""
    return 2 * num_monomials(dim, k)


def knn(xyz: np.ndarray, q: int, queries=None) -> np.ndarray:
    xyz = _c(xyz, np.float64)
    n, dim = xyz.shape
    qi = None if queries is None else _c(queries, np.int64)
    nq = n if qi is None else len(qi)
    nbr = np.zeros((nq, q), np.int32)
    st = lib().orc_knn(dim, n, _p(xyz), q, nq, _p(qi), _p(nbr))
    if st != ORC_OK:
        raise ValueError(f"orc_knn failed ({st}): duplicate points or q > n")
    return nbr


def saddle_system(xyz, nbr, k, i, phs=3):
    xyz = _c(xyz, np.float64)
    nbr = _c(nbr, np.int32)
    n, dim = xyz.shape
    q = nbr.shape[1]
    m = num_monomials(dim, k)
    ns = q + m
    A = np.zeros((ns, ns))
    B = np.zeros((ns, dim + 1))
    s = np.zeros(1)
    st = lib().orc_saddle_system(dim, n, _p(xyz), q, _p(nbr), k, phs, i, _p(A), _p(B), _p(s))
    if st != ORC_OK:
        raise ValueError("orc_saddle_system failed")
    return A, B, float(s[0])


def weights(xyz, nbr, k, phs=3, queries=None, allow_singular=False):
    """Returns w[R, nq, q]; nbr holds the clouds of all points (n, q)."""
    xyz = _c(xyz, np.float64)
    nbr = _c(nbr, np.int32)
    n, dim = xyz.shape
    q = nbr.shape[1]
    qi = None if queries is None else _c(queries, np.int64)
    nq = n if qi is None else len(qi)
    w = np.zeros((dim + 1, nq, q))
    bad = np.zeros(1, np.int64)
    st = lib().orc_weights(dim, n, _p(xyz), q, _p(nbr), k, phs, nq, _p(qi), _p(w), _p(bad))
    if st == ORC_E_SINGULAR and not allow_singular:
        raise np.linalg.LinAlgError(f"singular stencil at point {int(bad[0])}")
    if st not in (ORC_OK, ORC_E_SINGULAR):
        raise ValueError(f"orc_weights failed ({st})")
    return w


def knn_points(xyz, q, points):
    """Brute-force q nearest cloud points of arbitrary points (Sec. 2 clouds):
    order (squared distance, index), squared distance formed as
    ((dx*dx + dy*dy) + dz*dz) with dx = x_j - x* in FP64 without fused
    multiply-adds (numpy never fuses)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64).reshape(-1, xyz.shape[1])
    out = np.zeros((len(pts), q), np.int32)
    idx = np.arange(len(xyz))
    for t, x in enumerate(pts):
        d = xyz - x
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
        if xyz.shape[1] == 3:
            d2 = d2 + d[:, 2] * d[:, 2]
        out[t] = np.lexsort((idx, d2))[:q]
    return out


def wrap_points(xyz, points, period):
    """Query points moved into the cloud's periodic box: along a periodic axis
    of period L, a coordinate outside [lo, lo + L) (lo the cloud's smallest) is
    replaced by lo + r, r = fmod(x - lo, L) taken into [0, L); coordinates
    inside are kept as they are."""
    xyz = np.asarray(xyz, dtype=np.float64)
    pts = np.array(points, dtype=np.float64).reshape(-1, xyz.shape[1])
    for d in range(xyz.shape[1]):
        L = period[d]
        if not L > 0:
            continue
        lo = float(xyz[:, d].min())
        for t in range(len(pts)):
            x = float(pts[t, d])
            if x < lo or x >= lo + L:
                r = math.fmod(x - lo, L)
                if r < 0:
                    r += L
                pts[t, d] = lo + r
    return pts


def interpolate(xyz, k, points, fields, q=None, phs=3, period=None):
    """Evaluate the local PHS + polynomial interpolant of each point's q-point
    cloud (Sec. 2, Eq. RBF_interp) at arbitrary points: returns
    (values[nfield, np], nbr[np, q], w[np, q]). With a period (Sec. 3.1
    periodic boundaries) the points are wrapped into the periodic box
    (wrap_points), each takes its cloud among all images of the cloud's
    points (periodic_images), the weights use the images' coordinates, and
    the cloud is written with the indices of the points the images stand for."""
    xyz = np.asarray(xyz, dtype=np.float64)
    dim = xyz.shape[1]
    q = default_q(dim, k) if q is None else q
    periodic = period is not None and any(p > 0 for p in period[:dim])
    if periodic:
        pts = wrap_points(xyz, points, period)
        src, owner = periodic_images(xyz, period)
    else:
        pts = np.asarray(points, dtype=np.float64).reshape(-1, dim)
        src, owner = xyz, np.arange(len(xyz))
    nbr = knn_points(src, q, pts)
    w = np.zeros((len(pts), q))
    for t in range(len(pts)):
        w[t] = interp_weights(src, nbr[t], pts[t], k, phs)
    nbr = owner[nbr].astype(np.int32)
    if periodic and any(len(set(r)) != q for r in nbr):
        raise ValueError("a cloud holds two images of one point: period too small for q")
    f = np.asarray(fields, dtype=np.float64).reshape(-1, len(xyz))
    vals = np.array([[w[t] @ fi[nbr[t]] for t in range(len(pts))] for fi in f])
    return vals, nbr, w


def interp_weights(xyz, cloud_idx, xstar, k, phs=3):
    xyz = _c(xyz, np.float64)
    cl = _c(cloud_idx, np.int32)
    xs = _c(xstar, np.float64)
    dim = xyz.shape[1]
    w = np.zeros(len(cl))
    st = lib().orc_interp_weights(dim, _p(xyz), len(cl), _p(cl), _p(xs), k, phs, _p(w))
    if st != ORC_OK:
        raise np.linalg.LinAlgError("singular interpolation system")
    return w


def csr(nbr, w):
    """(col[n, q] sorted per row, val[R, n, q]) from clouds and weights."""
    nbr = _c(nbr, np.int32)
    w = _c(w, np.float64)
    n, q = nbr.shape
    R = w.shape[0]
    col = np.zeros((n, q), np.int32)
    val = np.zeros((R, n, q))
    lib().orc_csr(n, q, _p(nbr), R, _p(w), _p(col), _p(val))
    return col, val


def spmv(col, val, x):
    col = _c(col, np.int32)
    val = _c(val, np.float64)
    x = _c(x, np.float64)
    n, q = col.shape
    y = np.zeros(n)
    lib().orc_spmv(n, q, _p(col), _p(val), _p(x), _p(y))
    return y


def apply_ops(col, val, x):
    """Apply every operator row set in val[R] to x: returns [R, n]."""
    return np.stack([spmv(col, val[r], x) for r in range(val.shape[0])])


def poisson_values(cloud, col, val, rows=None):
    """Pressure-correction matrix: Laplacian rows inside, N . grad rows on
    velocity-Dirichlet boundary points, identity at the pinned point and at
    prescribed-pressure points. With rows (the global indices of the given
    rows), cloud.kind and cloud.normal hold just those rows and cloud.pin
    stays a global index."""
    col = _c(col, np.int32)
    val = _c(val, np.float64)
    n, q = col.shape
    kind = _c(cloud.kind, np.uint8)
    nrm = _c(cloud.normal, np.float64)
    ri = None if rows is None else _c(rows, np.int64)
    pv = np.zeros((n, q))
    lib().orc_poisson_values(cloud.dim, n, q, _p(kind), _p(nrm), int(cloud.pin), _p(col), _p(val), _p(ri), _p(pv))
    return pv


def bicgstab(col, val, b, x0=None, tol=1e-10, maxit=5000):
    col = _c(col, np.int32)
    val = _c(val, np.float64)
    b = _c(b, np.float64)
    n, q = col.shape
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    its = np.zeros(1, np.int32)
    rr = np.zeros(1)
    st = lib().orc_bicgstab(n, q, _p(col), _p(val), _p(b), _p(x), tol, maxit, _p(its), _p(rr))
    return x, int(its[0]), float(rr[0]), st


@dataclass
class Operators:
    """Oracle operators of one cloud."""
    cloud: object
    k: int
    q: int
    phs: int
    nbr: np.ndarray       # (n, q) clouds in distance order
    w: np.ndarray         # (R, n, q) weights in cloud order
    col: np.ndarray       # (n, q) sorted CSR columns
    val: np.ndarray       # (R, n, q) CSR values: d/dx, d/dy, (d/dz), Laplacian
    pval: np.ndarray      # (n, q) pressure-correction matrix


def periodic_images(xyz, period):
    """The points followed by all their images x_j + m L e (m in {-1, 0, 1}
    along each periodic axis, not all 0), image coordinates formed as x + L or
    x - L; returns (coordinates, index of the point each row is an image of)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    n, dim = xyz.shape
    rows, owner = [xyz], [np.arange(n)]
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                m = (a, b, c)
                if m == (0, 0, 0) or any(m[d] != 0 and (d >= dim or not period[d] > 0) for d in range(3)):
                    continue
                y = xyz.copy()
                for d in range(dim):
                    if m[d] > 0:
                        y[:, d] = xyz[:, d] + period[d]
                    elif m[d] < 0:
                        y[:, d] = xyz[:, d] - period[d]
                rows.append(y)
                owner.append(np.arange(n))
    return np.concatenate(rows), np.concatenate(owner)


def build_operators(cloud, k, q=None, phs=3) -> Operators:
    """Clouds, weights and operators (Sec. 2). A periodic cloud (Sec. 3.1)
    takes its clouds among all images of its points, by brute force; the
    weights use the images' coordinates and the clouds are then written with
    the indices of the points the images stand for."""
    q = default_q(cloud.dim, k) if q is None else q
    period = tuple(getattr(cloud, "period", (0.0, 0.0, 0.0)))
    if any(p > 0 for p in period[:cloud.dim]):
        n = cloud.n
        imgs, owner = periodic_images(cloud.xyz, period)
        nb_img = knn_points(imgs, q, cloud.xyz)
        full = np.zeros((len(imgs), q), np.int32)
        full[:n] = nb_img
        w = weights(imgs, full, k, phs, queries=np.arange(n))
        nbr = owner[nb_img].astype(np.int32)
        if any(len(set(r)) != q for r in nbr):
            raise ValueError("a cloud holds two images of one point: period too small for q")
    else:
        nbr = knn(cloud.xyz, q)
        w = weights(cloud.xyz, nbr, k, phs)
    col, val = csr(nbr, w)
    pv = poisson_values(cloud, col, val)
    return Operators(cloud, k, q, phs, nbr, w, col, val, pv)


class _StepCfg(C.Structure):
    _fields_ = [("dim", C.c_int), ("q", C.c_int), ("n", C.c_int64),
                ("kind", C.c_void_p), ("normal", C.c_void_p), ("pin", C.c_int64),
                ("col", C.c_void_p), ("val", C.c_void_p), ("pval", C.c_void_p),
                ("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("alpha", C.c_double * 3),
                ("tol_outer", C.c_double), ("tol_krylov", C.c_double),
                ("max_outer", C.c_int), ("max_krylov", C.c_int), ("force", C.c_double * 3)]


class _StepStats(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("krylov_mom", C.c_int), ("krylov_p", C.c_int),
                ("krylov_b", C.c_int), ("status", C.c_int), ("delta", C.c_double),
                ("eps_steady", C.c_double), ("div_l1", C.c_double), ("final_relres_p", C.c_double),
                ("krylov_relres_max", C.c_double)]


BDF2 = (1.5, -2.0, 0.5)
BDF1 = (1.0, -1.0, 0.0)


def simple_step(ops: Operators, u, u_prev, p, u_bc, rho, mu, dt, alpha=BDF2,
                tol_outer=1e-6, tol_krylov=1e-10, max_outer=50, max_krylov=5000, p_bc=None, force=(0.0, 0.0, 0.0)):
    """One time step; returns (u_new, u_n, p_new, stats dict). Inputs are not modified.
    p_bc: pressure at t^{n+1} on prescribed-pressure (kind 2) and outlet points.
    force: constant body force per unit volume (a mean pressure gradient)."""
    cl = ops.cloud
    n, dim = cl.n, cl.dim
    u = np.array(u, dtype=np.float64, copy=True).reshape(dim, n)
    up = np.array(u_prev, dtype=np.float64, copy=True).reshape(dim, n)
    p = np.array(p, dtype=np.float64, copy=True).reshape(n)
    ubc = _c(u_bc, np.float64).reshape(dim, n)
    kind = _c(cl.kind, np.uint8)
    nrm = _c(cl.normal, np.float64)
    col = _c(ops.col, np.int32)
    val = _c(ops.val, np.float64)
    pv = _c(ops.pval, np.float64)
    cfg = _StepCfg(dim, ops.q, n, _p(kind).value, _p(nrm).value, int(cl.pin), _p(col).value,
                   _p(val).value, _p(pv).value, rho, mu, dt, (C.c_double * 3)(*alpha),
                   tol_outer, tol_krylov, max_outer, max_krylov,
                   (C.c_double * 3)(*(tuple(force) + (0.0,) * (3 - len(force)))))
    st = _StepStats()
    pbc = None if p_bc is None else _c(p_bc, np.float64).reshape(n)
    if pbc is None and ((cl.kind == 2) | (cl.kind == 3)).any():
        raise ValueError("p_bc is required on clouds with prescribed-pressure points")
    lib().orc_simple_step(C.byref(cfg), _p(u), _p(up), _p(p), _p(ubc), _p(pbc), C.byref(st))
    stats = dict(outer_iters=st.outer_iters, krylov_mom=st.krylov_mom, krylov_p=st.krylov_p,
                 krylov_b=st.krylov_b, status=st.status, delta=st.delta, eps_steady=st.eps_steady,
                 div_l1=st.div_l1, final_relres_p=st.final_relres_p, krylov_relres_max=st.krylov_relres_max)
    return u, up, p, stats


def convdiff_lambda(ops: Operators, u0, rho, mu, iters=200) -> float:
    cl = ops.cloud
    kind = _c(cl.kind, np.uint8)
    col = _c(ops.col, np.int32)
    val = _c(ops.val, np.float64)
    u0 = _c(u0, np.float64).reshape(cl.dim, cl.n)
    return lib().orc_convdiff_lambda(cl.dim, cl.n, ops.q, _p(kind), _p(col), _p(val), _p(u0), rho, mu, iters)


def dt_from_courant(ops: Operators, u0, co, rho, mu, iters=200) -> float:
    """Courant number Co = |lambda|max dt / 2."""
    return 2.0 * co / convdiff_lambda(ops, u0, rho, mu, iters)


def outer_tolerance(dt, eps_prev, first=False, cap=1e-4):
    """Sec. 3.2: 1e-4 at first, then min(1e-4, dt * eps_s)."""
    return cap if first or eps_prev is None else min(cap, dt * eps_prev)


def run_steady(ops: Operators, u0, p0, u_bc, rho, mu, dt, steady_tol=1e-8, max_steps=100000,
               krylov_factor=1e-2, krylov_floor=1e-13, max_outer=50, max_krylov=5000, callback=None,
               p_bc=None):
    """March in time until the steady error max_c mean|u^{n+1}-u^n|/dt <= steady_tol.
    The first step is BDF1, later steps BDF2; the outer tolerance follows Sec. 3.2
    and the Krylov tolerance is max(floor, factor * outer tolerance)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    up = u.copy()
    p = np.array(p0, dtype=np.float64, copy=True)
    eps = None
    hist = []
    for step in range(max_steps):
        tol_o = outer_tolerance(dt, eps, first=(step == 0))
        tol_k = max(krylov_floor, krylov_factor * tol_o)
        u, up, p, st = simple_step(ops, u, up, p, u_bc, rho, mu, dt,
                                   alpha=BDF1 if step == 0 else BDF2,
                                   tol_outer=tol_o, tol_krylov=tol_k, max_outer=max_outer,
                                   max_krylov=max_krylov, p_bc=p_bc)
        eps = st["eps_steady"]
        hist.append(st)
        if callback:
            callback(step, u, p, st)
        if eps <= steady_tol:
            break
    return u, p, hist


def run_transient(ops: Operators, u0, p0, bc_fn, rho, mu, dt, nsteps, tol_outer=1e-8,
                  tol_krylov=1e-10, max_outer=50, max_krylov=5000, u_prev0=None, t0=0.0, pbc_fn=None):
    """nsteps time steps from t0 with Dirichlet data bc_fn(t) -> [dim, n] (and
    pbc_fn(t) -> [n] on prescribed-pressure points); the first step is BDF1
    unless u_prev0 (velocity at t0 - dt) is given."""
    u = np.array(u0, dtype=np.float64, copy=True)
    up = u.copy() if u_prev0 is None else np.array(u_prev0, dtype=np.float64, copy=True)
    p = np.array(p0, dtype=np.float64, copy=True)
    hist = []
    for step in range(nsteps):
        t_next = t0 + (step + 1) * dt
        first = (step == 0 and u_prev0 is None)
        u, up, p, st = simple_step(ops, u, up, p, bc_fn(t_next), rho, mu, dt,
                                   alpha=BDF1 if first else BDF2, tol_outer=tol_outer,
                                   tol_krylov=tol_krylov, max_outer=max_outer, max_krylov=max_krylov,
                                   p_bc=None if pbc_fn is None else pbc_fn(t_next))
        hist.append(st)
    return u, p, hist


def cylinder_forces(ops: Operators, u, p, centre, diameter, mu, nsurf=360, rho=None, u_ref=None):
    """Force per unit length on a circular cylinder in a 2D flow (Sec. 4, Eqs.
    cylinder forces and cylinder stress), in the order the paper takes it:

    1. strain rates at the nodes from the cloud's d/dx and d/dy operators;
    2. pressure and strain rates interpolated (Eq. RBF_interp off the nodes,
       with the operators' k, q and PHS power; on a periodic cloud as
       interpolate does there) to nsurf uniform points
       x_j = centre + (D/2)(cos t_j, sin t_j), t_j = 2 pi j / nsurf;
    3. sigma = -p I + mu (grad u + grad u^T) there, and the traction
       sigma . (cos t, sin t), the normal pointing from the cylinder into the
       fluid;
    4. F = (D/2) * integral over t in [0, 2 pi] of the traction, by the
       composite Simpson rule over the nsurf panels of the closed curve
       (nsurf even).

    With rho and u_ref, also C_D, C_L = F / (rho u_ref^2 D / 2) (Eq. cylinder
    lift drag). Returns (F[2], traction[2, nsurf]) or (F, traction, C[2])."""
    cloud = ops.cloud
    if cloud.dim != 2:
        raise ValueError("cylinder forces are defined for 2D clouds")
    if nsurf < 4 or nsurf % 2:
        raise ValueError("nsurf must be even and at least 4")
    n = cloud.n
    u = np.asarray(u, dtype=np.float64).reshape(2, n)
    p = np.asarray(p, dtype=np.float64).reshape(n)
    grads = [spmv(ops.col, ops.val[d], u[comp]) for comp in range(2) for d in range(2)]   # ux, uy, vx, vy
    r = 0.5 * diameter
    cs = [math.cos(2.0 * math.pi * j / nsurf) for j in range(nsurf)]
    sn = [math.sin(2.0 * math.pi * j / nsurf) for j in range(nsurf)]
    pts = np.array([[centre[0] + r * cs[j], centre[1] + r * sn[j]] for j in range(nsurf)])
    vals, _, _ = interpolate(cloud.xyz, ops.k, pts, np.stack([p] + grads), q=ops.q, phs=ops.phs,
                             period=getattr(cloud, "period", None))
    trac = np.zeros((2, nsurf))
    for j in range(nsurf):
        pj, ux, uy, vx, vy = vals[:, j]
        sxx = -pj + 2.0 * mu * ux
        syy = -pj + 2.0 * mu * vy
        sxy = mu * (uy + vx)
        trac[0, j] = sxx * cs[j] + sxy * sn[j]
        trac[1, j] = sxy * cs[j] + syy * sn[j]
    # the closed curve's end point repeats its start: even points weigh 2h/3,
    # odd points 4h/3
    h = 2.0 * math.pi / nsurf
    force = np.zeros(2)
    for d in range(2):
        acc = 0.0
        for j in range(nsurf):
            acc += (4.0 if j % 2 else 2.0) * trac[d, j]
        force[d] = r * (h / 3.0) * acc
    if rho is None or u_ref is None:
        return force, trac
    return force, trac, force / (0.5 * rho * u_ref * u_ref * diameter)
