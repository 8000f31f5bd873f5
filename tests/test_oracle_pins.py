"""Pins of the FP64 oracle to what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: values printed
in the paper, closed forms, exact polynomial reproduction, library routines on
the same inputs, brute force, invariances and convergence orders.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl
from scipy.spatial.distance import cdist

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- closed forms

def test_closed_forms_satisfy_navier_stokes():
    """Kovasznay, Taylor-Green and Ethier-Steinman flows are divergence free and
    solve the incompressible Navier-Stokes equations exactly (rho = 1)."""
    import sympy as s
    x, y, z, t = s.symbols("x y z t", real=True)
    Re = s.Integer(40)
    nu = 1 / Re
    lam = Re / 2 - s.sqrt(Re ** 2 / 4 + 4 * s.pi ** 2)
    u = 1 - s.exp(lam * x) * s.cos(2 * s.pi * y)
    v = lam / (2 * s.pi) * s.exp(lam * x) * s.sin(2 * s.pi * y)
    p = s.Rational(1, 2) * (1 - s.exp(2 * lam * x))
    _check_ns2(s, x, y, t, u, v, p, nu)
    nu = s.Rational(1, 100)
    F = s.exp(-2 * nu * t)
    u = s.cos(x) * s.sin(y) * F
    v = -s.sin(x) * s.cos(y) * F
    p = -s.Rational(1, 4) * (s.cos(2 * x) + s.cos(2 * y)) * F ** 2
    _check_ns2(s, x, y, t, u, v, p, nu)
    a, d = s.pi / 4, s.pi / 2
    G = s.exp(-nu * d ** 2 * t)
    U = [-a * (s.exp(a * x) * s.sin(a * y + d * z) + s.exp(a * z) * s.cos(a * x + d * y)) * G,
         -a * (s.exp(a * y) * s.sin(a * z + d * x) + s.exp(a * x) * s.cos(a * y + d * z)) * G,
         -a * (s.exp(a * z) * s.sin(a * x + d * y) + s.exp(a * y) * s.cos(a * z + d * x)) * G]
    P = -a ** 2 / 2 * (s.exp(2 * a * x) + s.exp(2 * a * y) + s.exp(2 * a * z)
                       + 2 * s.sin(a * x + d * y) * s.cos(a * z + d * x) * s.exp(a * (y + z))
                       + 2 * s.sin(a * y + d * z) * s.cos(a * x + d * y) * s.exp(a * (z + x))
                       + 2 * s.sin(a * z + d * x) * s.cos(a * y + d * z) * s.exp(a * (x + y))) * G ** 2
    X = [x, y, z]
    div = sum(s.diff(U[i], X[i]) for i in range(3))
    pts = [(0.1, 0.3, 0.7, 0.2), (0.9, 0.4, 0.15, 1.3)]
    for pt in pts:
        sub = dict(zip((x, y, z, t), pt))
        assert abs(float(div.subs(sub))) < 1e-12
        for i in range(3):
            res = (s.diff(U[i], t) + sum(U[j] * s.diff(U[i], X[j]) for j in range(3))
                   + s.diff(P, X[i]) - nu * sum(s.diff(U[i], X[j], 2) for j in range(3)))
            assert abs(float(res.subs(sub))) < 1e-10
    # the numpy versions used as inputs agree with the symbolic ones
    xs, ys, zs, ts = 0.3, 0.55, 0.8, 0.4
    un, vn, wn, pn = W.beltrami(xs, ys, zs, ts)
    sub = {x: xs, y: ys, z: zs, t: ts}
    assert abs(un - float(U[0].subs(sub))) < 1e-13 and abs(pn - float(P.subs(sub))) < 1e-13


def test_couette_closed_form():
    """Cylindrical Couette flow (Sec. 4.1, Eq. couette v_theta): the numpy
    velocity and pressure solve the steady Navier-Stokes equations for any
    viscosity, the inner wall turns at omega r1 and the outer wall is at rest."""
    import sympy as s
    x, y, t = s.symbols("x y t", real=True)
    r1, r2, om = s.Rational(1, 2), s.Integer(1), s.Integer(2)
    r = s.sqrt(x * x + y * y)
    vt = r1 * om * r1 * r2 / (r2 ** 2 - r1 ** 2) * (r2 / r - r / r2)    # the paper's form
    u, v = -vt * y / r, vt * x / r
    a = om * r1 ** 2 * r2 ** 2 / (r2 ** 2 - r1 ** 2)
    b = -om * r1 ** 2 / (r2 ** 2 - r1 ** 2)
    p = -a ** 2 / (2 * r ** 2) + 2 * a * b * s.log(r) + b ** 2 * r ** 2 / 2
    for nu in (s.Rational(1, 100), s.Integer(1)):
        _check_ns2(s, x, y, t, u, v, p, nu, pts=[(0.6, 0.2, 0.0), (-0.3, -0.7, 0.0), (0.1, 0.95, 0.0)])
    xs = np.array([0.5, 0.0, -0.6, 0.3]); ys = np.array([0.0, -1.0, 0.45, 0.6])
    un, vn, pn = W.couette(xs, ys)
    for i in range(4):
        sub = {x: xs[i], y: ys[i]}
        assert abs(un[i] - float(u.subs(sub))) < 1e-13 and abs(vn[i] - float(v.subs(sub))) < 1e-13
    # pressure up to its level: differences between points agree
    dp = float((p.subs({x: xs[2], y: ys[2]}) - p.subs({x: xs[3], y: ys[3]})))
    assert abs((pn[2] - pn[3]) - dp) < 1e-13
    # walls: |v| = omega r1 on r = r1, 0 on r = r2
    assert abs(np.hypot(un[0], vn[0]) - 1.0) < 1e-14 and abs(np.hypot(un[1], vn[1])) < 1e-14
    # plane Poiseuille flow (the outlet workload)
    U, mu = s.Integer(1), s.Rational(1, 100)
    _check_ns2(s, x, y, t, 4 * U * y * (1 - y), s.Integer(0) * x, -8 * mu * U * x, mu,
               pts=[(0.3, 0.2, 0.0), (2.5, 0.7, 0.0)])
    up, vp, pp = W.poiseuille(np.array([0.3]), np.array([0.2]), 1.0, 0.01)
    assert abs(up[0] - 4 * 0.2 * 0.8) < 1e-15 and vp[0] == 0.0 and abs(pp[0] + 8 * 0.01 * 0.3) < 1e-15


def _check_ns2(s, x, y, t, u, v, p, nu, pts=((0.2, 0.3, 0.1), (-0.4, 1.2, 0.7), (1.1, -0.3, 2.0))):
    div = s.diff(u, x) + s.diff(v, y)
    ru = s.diff(u, t) + u * s.diff(u, x) + v * s.diff(u, y) + s.diff(p, x) - nu * (s.diff(u, x, 2) + s.diff(u, y, 2))
    rv = s.diff(v, t) + u * s.diff(v, x) + v * s.diff(v, y) + s.diff(p, y) - nu * (s.diff(v, x, 2) + s.diff(v, y, 2))
    for pt in pts:
        sub = {x: pt[0], y: pt[1], t: pt[2]}
        for e in (div, ru, rv):
            assert abs(float(e.subs(sub))) < 1e-10


# ---------------------------------------------------------------- monomials

def test_monomial_order_matches_paper(orc):
    ref = np.loadtxt(os.path.join(GOLDEN, "monomials_2d_k2.txt"), dtype=int)
    ex = orc.monomial_exponents(2, 2)
    assert ex.shape == (6, 3)
    np.testing.assert_array_equal(ex[:, :2], ref)
    for dim in (2, 3):
        for k in range(0, 7):
            m = orc.num_monomials(dim, k)
            from math import comb
            assert m == comb(k + dim, dim)
            ex = orc.monomial_exponents(dim, k)
            tot = ex.sum(axis=1)
            assert (np.diff(tot) >= 0).all()            # graded
            assert len({tuple(r) for r in ex}) == m     # distinct
            assert tot.max() == k


# ---------------------------------------------------------------- kNN

def _brute_knn(xyz, q, idx):
    d = xyz - xyz[idx]
    if xyz.shape[1] == 2:
        d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    else:
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    return np.lexsort((np.arange(len(xyz)), d2))[:q]


@pytest.mark.parametrize("gen,q", [(lambda: W.kovasznay_square(nx=20), 20),
                                   (lambda: W.beltrami_cube(n=6), 40),
                                   (lambda: W.holed_square(900, seed=1003), 12)])
def test_knn_matches_brute_force(orc, gen, q):
    c = gen()
    nbr = orc.knn(c.xyz, q)
    assert nbr.shape == (c.n, q)
    assert (nbr[:, 0] == np.arange(c.n)).all()
    for i in range(0, c.n, max(1, c.n // 97)):
        np.testing.assert_array_equal(nbr[i], _brute_knn(c.xyz, q, i))


def test_knn_ties_broken_by_index(orc):
    # an exact lattice: many equal distances; order must follow the index
    g = np.arange(7, dtype=np.float64)
    X, Y = np.meshgrid(g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel()], 1)
    nbr = orc.knn(xyz, 9)
    i = 3 * 7 + 3
    assert list(nbr[i]) == [24, 17, 23, 25, 31, 16, 18, 30, 32]


# ---------------------------------------------------------------- weights

@pytest.mark.parametrize("dim,k,gen", [(2, 2, lambda: W.kovasznay_square(nx=12)),
                                       (2, 3, lambda: W.kovasznay_square(nx=12)),
                                       (2, 5, lambda: W.kovasznay_square(nx=14)),
                                       (3, 2, lambda: W.beltrami_cube(n=5)),
                                       (3, 3, lambda: W.beltrami_cube(n=6))])
def test_weights_reproduce_polynomials(orc, dim, k, gen):
    """The moment constraints (Eq. RBF_constraint) force exact differentiation of
    every monomial of degree <= k, at interior and one-sided boundary clouds."""
    c = gen()
    q = orc.default_q(dim, k)
    nbr = orc.knn(c.xyz, q)
    w = orc.weights(c.xyz, nbr, k)
    x = c.xyz
    h = c.h
    for ex in orc.monomial_exponents(dim, k):
        f = np.prod([x[:, e] ** ex[e] for e in range(dim)], axis=0)
        vals = f[nbr]                                    # (n, q)
        got = np.einsum("rnq,nq->rn", w, vals)
        ref = []
        for e in range(dim):
            if ex[e] == 0:
                ref.append(np.zeros(c.n))
            else:
                ee = ex.copy(); ee[e] -= 1
                ref.append(ex[e] * np.prod([x[:, j] ** ee[j] for j in range(dim)], axis=0))
        lap = np.zeros(c.n)
        for e in range(dim):
            if ex[e] >= 2:
                ee = ex.copy(); ee[e] -= 2
                lap += ex[e] * (ex[e] - 1) * np.prod([x[:, j] ** ee[j] for j in range(dim)], axis=0)
        ref.append(lap)
        ref = np.stack(ref)
        scale = np.abs(w).sum(axis=2) * (np.abs(vals).max(axis=1) + 1.0)
        assert (np.abs(got - ref) <= 1e-10 * scale + 1e-12).all(), (ex, np.abs(got - ref).max())
    del h


def test_saddle_system_blocks_and_library_solve(orc):
    """A = [Phi P; P^T 0] with Phi = r^3 of the scaled cloud (Eqs. RBF_interp_mat_vec,
    RBF_interp_phi, RBF_interp_poly); the oracle's LU solution matches LAPACK's."""
    c = W.kovasznay_square(nx=10)
    k, q = 3, 20
    nbr = orc.knn(c.xyz, q)
    w = orc.weights(c.xyz, nbr, k)
    for i in (0, 5, c.pin, c.n - 1):
        A, B, s = orc.saddle_system(c.xyz, nbr, k, i)
        xi = (c.xyz[nbr[i]] - c.xyz[i]) / s
        np.testing.assert_allclose(A[:q, :q], cdist(xi, xi) ** 3, rtol=1e-13, atol=1e-15)
        ex = orc.monomial_exponents(2, k)
        Pm = np.stack([xi[:, 0] ** a * xi[:, 1] ** b for a, b, _ in ex], 1)
        np.testing.assert_allclose(A[:q, q:], Pm, rtol=1e-13, atol=1e-15)
        np.testing.assert_array_equal(A[q:, :q], A[:q, q:].T)
        assert (A[q:, q:] == 0).all()
        assert np.isclose(s, np.linalg.norm(c.xyz[nbr[i, -1]] - c.xyz[i]))
        X = np.linalg.solve(A, B)
        sc = np.array([s, s, s * s])
        ref = (X[:q] / sc).T
        np.testing.assert_allclose(w[:, i, :], ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


def test_weights_translation_and_scale_covariance(orc):
    c = W.kovasznay_square(nx=10)
    k, q = 3, 20
    nbr = orc.knn(c.xyz, q)
    w = orc.weights(c.xyz, nbr, k)
    w_t = orc.weights(c.xyz + np.array([3.25, -1.5]), nbr, k)
    np.testing.assert_allclose(w_t, w, rtol=1e-9, atol=1e-9 * np.abs(w).max())
    sig = 0.37
    w_s = orc.weights(c.xyz * sig, nbr, k)
    np.testing.assert_allclose(w_s[:2] * sig, w[:2], rtol=1e-9, atol=1e-9 * np.abs(w[:2]).max())
    np.testing.assert_allclose(w_s[2] * sig * sig, w[2], rtol=1e-9, atol=1e-9 * np.abs(w[2]).max())


def _fit_slope(hs, errs):
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


@pytest.mark.parametrize("k", [2, 3, 4])
def test_derivative_errors_fall_at_expected_order(orc, k):
    """Expected orders k (gradient) and k-1 (Laplacian) of the PHS-RBF operators
    (Sec. 4.1, orders k+1 / k / k-1 for interpolation / gradient / Laplacian);
    band of +-0.7 on interior points of jittered lattices."""
    f = lambda x, y: np.exp(x) * np.sin(np.pi * y)
    fx = lambda x, y: np.exp(x) * np.sin(np.pi * y)
    lap = lambda x, y: (1 - np.pi ** 2) * np.exp(x) * np.sin(np.pi * y)
    hs, ex, el = [], [], []
    for nx in (16, 24, 36, 54):
        c = W.scattered_square(nx, seed=11, lo=0.0, hi=1.0)
        ops = orc.build_operators(c, k)
        x, y = c.xyz[:, 0], c.xyz[:, 1]
        d = orc.apply_ops(ops.col, ops.val, f(x, y))
        m = c.kind == 0
        hs.append(1.0 / nx)
        ex.append(np.abs(d[0] - fx(x, y))[m].mean())
        el.append(np.abs(d[2] - lap(x, y))[m].mean())
    sx, sl = _fit_slope(hs, ex), _fit_slope(hs, el)
    assert k - 0.7 <= sx, (sx, ex)
    assert k - 1 - 0.7 <= sl, (sl, el)


@pytest.mark.parametrize("k", [3, 4])
def test_couette_operators_converge_on_the_annulus(orc, k):
    """On the three annulus clouds of the Couette study (about 2080, 4033 and
    8078 points, Sec. 4.1) the operators applied to the exact Couette fields
    converge at the expected orders on interior points, curved walls and
    one-sided near-wall clouds included: the gradient of the pressure at order
    k, the Laplacian of the velocity (exactly zero for this flow) and the steady
    momentum residual (u.grad)u + grad p - nu Lap u at order k - 1 (band -0.7)."""
    hs, eg, el, er = [], [], [], []
    for npts in sorted(W.COUETTE_RADII):
        c = W.couette_annulus(W.COUETTE_RADII[npts])
        ops = orc.build_operators(c, k)
        vel, p = W.flow_fields(c)
        m = c.kind == 0
        x, y = c.xyz[:, 0], c.xyz[:, 1]
        rr = np.hypot(x, y)
        a = 2.0 * 0.25 / 0.75
        b = -2.0 * 0.25 / 0.75
        dpdr = (a / rr + b * rr) ** 2 / rr           # dp/dr = v_theta^2 / r
        du = [orc.apply_ops(ops.col, ops.val, vel[e]) for e in range(2)]
        dp = orc.apply_ops(ops.col, ops.val, p)
        eg.append(np.abs(dp[0] - dpdr * x / rr)[m].mean() + np.abs(dp[1] - dpdr * y / rr)[m].mean())
        el.append(np.abs(du[0][2])[m].mean() + np.abs(du[1][2])[m].mean())
        res = [vel[0] * du[e][0] + vel[1] * du[e][1] + dp[e] - c.meta["nu"] * du[e][2] for e in range(2)]
        er.append(sum(np.abs(r_)[m].mean() for r_ in res))
        hs.append(c.h)
    sg, sl, sr = _fit_slope(hs, eg), _fit_slope(hs, el), _fit_slope(hs, er)
    assert sg >= k - 0.7, (sg, eg)
    assert sl >= k - 1 - 0.7, (sl, el)
    assert sr >= k - 1 - 0.7, (sr, er)
    assert er[-1] < er[0] / 2


def test_interpolation_error_falls_at_order_k_plus_1(orc):
    f = lambda x, y: np.cos(2 * x) * np.exp(y)
    k = 3
    rng = np.random.default_rng(5)
    hs, errs = [], []
    for nx in (12, 18, 27, 40):
        c = W.scattered_square(nx, seed=3, lo=0.0, hi=1.0)
        q = orc.default_q(2, k)
        xs = rng.uniform(0.3, 0.7, size=(25, 2))
        e = []
        for p in xs:
            d2 = ((c.xyz - p) ** 2).sum(1)
            cl = np.lexsort((np.arange(c.n), d2))[:q]
            w = orc.interp_weights(c.xyz, cl, p, k)
            e.append(abs(w @ f(c.xyz[cl, 0], c.xyz[cl, 1]) - f(*p)))
        hs.append(1.0 / nx)
        errs.append(np.mean(e))
    assert _fit_slope(hs, errs) >= k + 1 - 0.7


def test_singular_stencil_is_reported(orc):
    # five collinear points cannot carry the y monomials: the system is singular
    xyz = np.stack([np.arange(8.0), np.zeros(8)], 1)
    nbr = orc.knn(xyz, 6)
    with pytest.raises(np.linalg.LinAlgError):
        orc.weights(xyz, nbr, 1)


# ---------------------------------------------------------------- CSR

def test_csr_is_a_permutation_matching_scipy(orc):
    c = W.kovasznay_square(nx=15)
    k, q = 3, 20
    nbr = orc.knn(c.xyz, q)
    w = orc.weights(c.xyz, nbr, k)
    col, val = orc.csr(nbr, w)
    assert (np.diff(col, axis=1) > 0).all()
    for r in range(3):
        A = sp.csr_matrix((w[r].ravel().copy(), nbr.ravel().copy(), np.arange(0, c.n * q + 1, q)),
                          shape=(c.n, c.n))
        A.sort_indices()
        np.testing.assert_array_equal(A.indices.reshape(c.n, q), col)
        np.testing.assert_array_equal(A.data.reshape(c.n, q), val[r])   # bit-exact


def test_poisson_matrix_rows(orc):
    c = W.kovasznay_square(nx=12)
    ops = orc.build_operators(c, 3)
    inter = (c.kind == 0) & (np.arange(c.n) != c.pin)
    np.testing.assert_array_equal(ops.pval[inter], ops.val[2][inter])
    b = c.kind != 0
    ref = c.normal[b, 0:1] * ops.val[0][b] + c.normal[b, 1:2] * ops.val[1][b]
    np.testing.assert_allclose(ops.pval[b], ref, rtol=1e-15, atol=1e-15)
    np.testing.assert_array_equal(ops.pval[c.pin], (ops.col[c.pin] == c.pin).astype(float))
    # homogeneous Neumann rows annihilate constants and the pin row fixes the level
    ones = orc.spmv(ops.col, ops.pval, np.ones(c.n))
    assert np.abs(ones[b]).max() < 1e-9 * np.abs(ops.pval[b]).max()


# ---------------------------------------------------------------- Krylov

def test_bicgstab_matches_direct_solve(orc):
    c = W.kovasznay_square(nx=16)
    ops = orc.build_operators(c, 3)
    n, q = ops.col.shape
    A = sp.csr_matrix((ops.pval.ravel(), ops.col.ravel(), np.arange(0, n * q + 1, q)), shape=(n, n))
    b = np.random.default_rng(1).standard_normal(n)
    x, its, rr, st = orc.bicgstab(ops.col, ops.pval, b, tol=1e-12)
    assert st == 0 and rr <= 1e-11     # true residual after the restart rule (<= 10 tol)
    xd = spl.spsolve(A.tocsc(), b)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)   # true vs recursive residual drift
    assert np.abs(x - xd).max() <= 1e-7 * np.abs(xd).max()
    # zero right-hand side gives the zero solution
    x0, its0, _, st0 = orc.bicgstab(ops.col, ops.pval, np.zeros(n), x0=np.ones(n))
    assert st0 == 0 and its0 == 0 and not x0.any()


def test_momentum_like_solve(orc):
    c = W.kovasznay_square(nx=16)
    ops = orc.build_operators(c, 3)
    n, q = ops.col.shape
    mval = 20.0 * (ops.col == np.arange(n)[:, None]) - 0.025 * ops.val[2]
    A = sp.csr_matrix((mval.ravel(), ops.col.ravel(), np.arange(0, n * q + 1, q)), shape=(n, n))
    b = np.random.default_rng(2).standard_normal(n)
    x, its, rr, st = orc.bicgstab(ops.col, mval, b, tol=1e-13)
    assert st == 0
    np.testing.assert_allclose(x, spl.spsolve(A.tocsc(), b), rtol=1e-10, atol=1e-11)


# ---------------------------------------------------------------- time step

def _one_step_change(orc, nx, dt=0.005):
    c = W.kovasznay_square(nx=nx)
    ops = orc.build_operators(c, 3)
    vel, p = W.flow_fields(c)
    u, up, pn, st = orc.simple_step(ops, vel, vel, p, vel, 1.0, 1.0 / 40, dt, alpha=orc.BDF2,
                                    tol_outer=0.0, tol_krylov=1e-12, max_outer=1)
    pe = p - p.mean()
    return (np.abs(u - vel).mean(), np.abs((pn - pn.mean()) - pe)[c.kind != 0].mean(), st)


def test_exact_steady_flow_is_near_a_fixed_point(orc):
    """Started from the exact Kovasznay solution, one outer iteration (momentum,
    pressure correction, boundary pressure from the normal momentum equation,
    corrections) moves the fields only by the discretization error, which
    shrinks with h. A sign error in any term of Eqs. u:tilde ... p:correction or
    in the normal momentum equation makes the change O(1)."""
    du1, dp1, st1 = _one_step_change(orc, 20)
    du2, dp2, st2 = _one_step_change(orc, 40)
    # a sign error in the advection or pressure-gradient term alone moves u by
    # ~dt |u.grad u| ~ 5e-2 here
    assert du1 < 2e-3 and du2 < 1e-3 and du2 < du1, (du1, du2)
    assert st1["status"] in (0, -4) and np.isfinite(dp1) and np.isfinite(dp2)


def test_courant_time_step_scaling(orc):
    """|lambda|max of the convection-diffusion operator grows like 1/h^2 when
    diffusion dominates: halving h cuts dt by between 2x and 4x (Sec. 4.1 notes
    about 3.5x for its explicit scheme)."""
    dts = []
    for nx in (16, 32):
        c = W.kovasznay_square(nx=nx)
        ops = orc.build_operators(c, 3)
        vel, _ = W.flow_fields(c)
        dts.append(orc.dt_from_courant(ops, vel, 1.0, 1.0, 1.0 / 40))
    assert 2.0 <= dts[0] / dts[1] <= 4.5, dts


def test_bdf_coefficients_fixture(orc):
    a = np.loadtxt(os.path.join(GOLDEN, "bdf2.txt"))
    assert tuple(a) == orc.BDF2
    # BDF2 differentiates quadratics in t exactly at t^{n+1}
    for f, df in ((lambda t: 3 * t * t - t + 2, lambda t: 6 * t - 1),):
        dt, t1 = 0.1, 1.0
        approx = (a[0] * f(t1) + a[1] * f(t1 - dt) + a[2] * f(t1 - 2 * dt)) / dt
        assert abs(approx - df(t1)) < 1e-12


@pytest.mark.parametrize("dim,boundary_kind,k", [(2, W.DIRICHLET, 2), (2, W.DIRICHLET, 3),
                                                 (2, W.PRESCRIBED_PRESSURE, 3), (3, W.DIRICHLET, 2),
                                                 (3, W.PRESCRIBED_PRESSURE, 2)])
@pytest.mark.parametrize("which", ["stagnation", "uniform"])
@pytest.mark.parametrize("bdf", ["BDF1", "BDF2"])
def test_polynomial_flows_are_reproduced(orc, dim, boundary_kind, k, which, bdf):
    """Exact Navier-Stokes solutions with quadratic-in-space, linear-in-time
    fields are fixed points of the discrete step: the operators reproduce
    polynomials up to degree k >= 2 (Eq. RBF_constraint) and BDF1/BDF2 are exact
    for linear-in-time fields (Eqs. u:n+1, v:n+1). One time step from the exact
    state must land on the exact state at t^{n+1}: interior momentum (mass,
    advection, viscous and pressure terms, Eqs. u:tilde, v:tilde), the Poisson
    right-hand side (Eq. pressure poisson), the boundary pressure from the normal
    momentum equation (Sec. 3.1) or a prescribed pressure, and the corrections
    (Eqs. u:correction ... p:correction). A wrong sign or coefficient in any of
    them, or a misplaced BDF coefficient, moves the result by O(dt)."""
    c = (W.kovasznay_square(nx=12, boundary_kind=boundary_kind) if dim == 2
         else W.scattered_cube(7, seed=3, boundary_kind=boundary_kind))
    ops = orc.build_operators(c, k)
    rho, mu, dt, t = 1.3, 0.05, 0.05, 0.3
    un, pn = W.polynomial_flow(c.xyz, t, which, rho)
    um, _ = W.polynomial_flow(c.xyz, t - dt, which, rho)
    ue, pe = W.polynomial_flow(c.xyz, t + dt, which, rho)
    pbc = pe if boundary_kind == W.PRESCRIBED_PRESSURE else None
    u, u_n, p, st = orc.simple_step(ops, un, um, pn, ue, rho, mu, dt, alpha=getattr(orc, bdf),
                                    tol_outer=1e-12, tol_krylov=1e-13, max_outer=4, max_krylov=20000, p_bc=pbc)
    assert st["status"] == 0, st
    np.testing.assert_array_equal(u_n, un)
    assert np.abs(u - ue).max() <= 1e-10 * max(1.0, np.abs(ue).max())
    assert np.abs(p - pe).max() <= 1e-9 * max(1.0, np.abs(pe).max())


@pytest.mark.parametrize("mu,scale", [(1.0 / 40, 1.0), (1.0, 0.0)])
def test_courant_lambda_matches_dense_eigenvalues(orc, mu, scale):
    """The convection-diffusion eigenvalue used for the Courant number (Sec. 3.2)
    from power iteration matches the largest eigenvalue modulus of the dense
    interior operator -rho u0.grad + mu Lap computed by LAPACK, and never exceeds
    its 2-norm (the bound of any power-iteration estimate)."""
    c = W.kovasznay_square(nx=12)
    ops = orc.build_operators(c, 3)
    vel, _ = W.flow_fields(c)
    u0 = vel * scale
    lam = orc.convdiff_lambda(ops, u0, 1.0, mu, 200)
    n = c.n
    A = np.zeros((n, n))
    for i in np.nonzero(c.kind == W.INTERIOR)[0]:
        for a in range(ops.q):
            A[i, ops.col[i, a]] += (-(u0[0, i] * ops.val[0, i, a] + u0[1, i] * ops.val[1, i, a])
                                    + mu * ops.val[2, i, a])
    lam_ref = np.abs(np.linalg.eigvals(A)).max()
    assert abs(lam - lam_ref) <= 1e-3 * lam_ref, (lam, lam_ref)
    assert lam <= np.linalg.norm(A, 2) * (1 + 1e-12)


def test_knn_points_matches_cloud_knn_and_kdtree(orc):
    """Off-node neighbour search: at the cloud's own points it equals the C
    search; at arbitrary points its distances equal a k-d tree's."""
    from scipy.spatial import cKDTree
    c = W.kovasznay_square(nx=14)
    q = 20
    np.testing.assert_array_equal(orc.knn_points(c.xyz, q, c.xyz[:50]), orc.knn(c.xyz, q)[:50])
    pts = np.random.default_rng(8).uniform(-0.4, 1.4, size=(40, 2))
    nb = orc.knn_points(c.xyz, q, pts)
    d_tree, _ = cKDTree(c.xyz).query(pts, q)
    d_ours = np.sqrt(((c.xyz[nb] - pts[:, None, :]) ** 2).sum(-1))
    np.testing.assert_allclose(d_ours, d_tree, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("dim,k", [(2, 3), (2, 6), (3, 2), (3, 4)])
def test_interpolation_reproduces_polynomials_off_node(orc, dim, k):
    """The interpolant of a degree-k polynomial is the polynomial itself at any
    point (the appended monomials, Eq. RBF_constraint); at a node it returns
    the nodal value of any field."""
    c = W.kovasznay_square(nx=16) if dim == 2 else W.scattered_cube(9, seed=5)
    rng = np.random.default_rng(9)
    lo, hi = c.xyz.min(0), c.xyz.max(0)
    pts = lo + (hi - lo) * rng.uniform(0.1, 0.9, size=(12, dim))
    import itertools
    ex = [e for e in itertools.product(range(k + 1), repeat=dim) if sum(e) <= k]
    coef = rng.standard_normal(len(ex))
    def poly(x):
        return sum(cf * np.prod(x ** np.array(e), axis=1) for cf, e in zip(coef, ex))
    vals, _, _ = orc.interpolate(c.xyz, k, pts, poly(c.xyz))
    np.testing.assert_allclose(vals[0], poly(pts), rtol=1e-9, atol=1e-9 * np.abs(poly(pts)).max())
    f = np.sin(3 * c.xyz[:, 0]) + c.xyz[:, 1] ** 2
    v_node, _, _ = orc.interpolate(c.xyz, k, c.xyz[7:9], f)
    np.testing.assert_allclose(v_node[0], f[7:9], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_poiseuille_outlet_is_a_fixed_point(orc, k):
    """Plane Poiseuille flow is quadratic, so PHS operators with degree >= 2
    polynomials reproduce it exactly: started from it, one BDF2 step with an
    outlet (zero normal velocity gradient, prescribed pressure; Sec. 3.1)
    returns it to solver accuracy. The step must not read u_bc on outlet points
    nor p_bc elsewhere: both are set to garbage there."""
    c = W.poiseuille_channel()
    ops = orc.build_operators(c, k)
    vel, p = W.flow_fields(c)
    out = c.kind == W.OUTLET
    ubc = np.where(out[None, :], 123.0, vel)
    pbc = np.where(out, p, -77.0)
    u1, _, p1, st = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2, p_bc=pbc,
                                    tol_outer=1e-13, tol_krylov=1e-14, max_outer=3, max_krylov=20000)
    assert np.abs(u1 - vel).max() <= 1e-10, np.abs(u1 - vel).max()
    assert np.abs(p1 - p).max() <= 1e-10 * np.abs(p).max(), np.abs(p1 - p).max()
    # a wrong outlet row shows: a uniform shift of the outlet pressure moves the flow
    _, _, p2, _ = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2,
                                  p_bc=pbc + 0.01 * out, tol_outer=1e-13, tol_krylov=1e-14, max_outer=3,
                                  max_krylov=20000)
    assert np.abs(p2 - p).max() > 1e-3


@pytest.mark.parametrize("k", [2, 3])
def test_symmetry_plane_keeps_the_stagnation_flow(orc, k):
    """The stagnation flow u = (x, -y), p = -|u|^2/2 has the symmetry line
    y = 0 (v = 0, du/dy = 0; Sec. 3.1 symmetry conditions). Quadratic, so with
    degree >= 2 one BDF2 step returns it to solver accuracy; u_bc on the
    symmetry points is garbage and must not be read."""
    c = W.symmetric_square()
    ops = orc.build_operators(c, k)
    vel, p = W.flow_fields(c)
    sym = c.kind == W.SYMMETRY
    ubc = np.where(sym[None, :], 55.0, vel)
    u1, _, p1, st = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2,
                                    tol_outer=1e-13, tol_krylov=1e-14, max_outer=3, max_krylov=20000)
    assert np.abs(u1 - vel).max() <= 1e-10, np.abs(u1 - vel).max()
    assert np.abs(p1 - p).max() <= 1e-9, np.abs(p1 - p).max()
    # the symmetry rows matter: imposing u_bc there instead would move the flow
    assert np.abs(ubc - vel).max() > 1.0


def test_symmetry_strip_keeps_kovasznay_flow(orc):
    """Kovasznay flow between its symmetry lines y = 0 and y = 0.5: started
    from the exact state, one outer iteration moves the velocity only by the
    discretization error, which shrinks with h."""
    changes = []
    for nx, ny in ((20, 5), (40, 10)):
        c = W.kovasznay_strip(nx=nx, ny=ny)
        ops = orc.build_operators(c, 3)
        vel, p = W.flow_fields(c)
        u1, _, _, st = orc.simple_step(ops, vel, vel, p, vel, 1.0, 1.0 / 40, 0.01, alpha=orc.BDF2,
                                       tol_outer=0.0, tol_krylov=1e-12, max_outer=1, max_krylov=20000)
        changes.append(np.abs(u1 - vel).mean())
    assert changes[1] < changes[0] / 2 and changes[1] < 2e-3, changes


def test_periodic_clouds_wrap_the_seam(orc):
    """A periodic cloud (Sec. 3.1) takes its neighbours across the seam: its
    neighbour distances equal scipy's periodic k-d tree's, and derivative
    errors near the seam match those inside, falling at orders k (gradient)
    and k - 1 (Laplacian), band -0.7."""
    from scipy.spatial import cKDTree
    c = W.taylor_green_periodic(nx=24)
    ops = orc.build_operators(c, 4)
    L = 2 * np.pi
    dt_tree, _ = cKDTree(c.xyz, boxsize=L).query(c.xyz, ops.q)
    imgs, owner = orc.periodic_images(c.xyz, c.period)
    nb_img = orc.knn_points(imgs, ops.q, c.xyz)
    d_ours = np.sqrt(((imgs[nb_img] - c.xyz[:, None, :]) ** 2).sum(-1))
    np.testing.assert_allclose(d_ours, dt_tree, rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(owner[nb_img], ops.nbr)
    k = 4
    hs, eg, el, ratio = [], [], [], []
    for nx in (24, 36, 54):
        c = W.taylor_green_periodic(nx=nx)
        ops = orc.build_operators(c, k)
        x, y = c.xyz[:, 0], c.xyz[:, 1]
        f = np.sin(x) * np.cos(2 * y)
        d = orc.apply_ops(ops.col, ops.val, f)
        ex = np.abs(d[0] - np.cos(x) * np.cos(2 * y))
        near = (x < 3 * c.h) | (x > L - 3 * c.h) | (y < 3 * c.h) | (y > L - 3 * c.h)
        hs.append(c.h)
        eg.append(ex.mean())
        el.append(np.abs(d[2] + 5 * f).mean())
        ratio.append(ex[near].max() / ex[~near].max())
    assert _fit_slope(hs, eg) >= k - 0.7 and _fit_slope(hs, el) >= k - 1 - 0.7
    assert max(ratio) < 2.0, ratio


@pytest.mark.parametrize("k", [2, 3])
def test_forced_periodic_channel_is_a_fixed_point(orc, k):
    """A channel periodic in x, driven by the body force 8 nu U e_x (the mean
    pressure gradient of a periodic channel, Sec. 4, Eq. bellow dp_dx), holds
    Poiseuille flow at constant pressure exactly (quadratic fields, k >= 2).
    Without the force the flow decays: the term is used."""
    c = W.periodic_channel()
    ops = orc.build_operators(c, k)
    vel, p = W.flow_fields(c)
    kw = dict(tol_outer=1e-13, tol_krylov=1e-14, max_outer=3, max_krylov=20000)
    u1, _, p1, st = orc.simple_step(ops, vel, vel, p, vel, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2,
                                    force=c.meta["force"], **kw)
    assert np.abs(u1 - vel).max() <= 1e-10, np.abs(u1 - vel).max()
    assert np.abs(p1 - p).max() <= 1e-10, np.abs(p1 - p).max()
    u0, _, _, _ = orc.simple_step(ops, vel, vel, p, vel, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2, **kw)
    assert np.abs(u0 - vel).max() > 1e-4


# ---- drag and lift on a cylinder (Sec. 4, Eqs. cylinder forces, cylinder stress) ----
_CUBIC = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]


def _poly(coef, ex, X, Y, dx=0, dy=0):
    """sum_c coef_c d^dx/dX d^dy/dY (X^i Y^j), differentiated term by term."""
    t = 0.0
    for cf, (i, j) in zip(coef, ex):
        if i < dx or j < dy:
            continue
        f = (math.factorial(i) // math.factorial(i - dx)) * (math.factorial(j) // math.factorial(j - dy))
        t = t + cf * f * X ** (i - dx) * Y ** (j - dy)
    return t


def _cubic_case(seed=5, n=3000):
    c = W.holed_square(n, seed=seed, n_holes=1)
    cx, cy, r = c.meta["holes"][0]
    rng = np.random.default_rng(3)
    a, b, g = rng.standard_normal(10), rng.standard_normal(10), rng.standard_normal(6)
    X, Y = c.xyz[:, 0] - 0.5, c.xyz[:, 1] - 0.5
    u = np.stack([_poly(a, _CUBIC, X, Y), _poly(b, _CUBIC, X, Y)])
    p = _poly(g, _CUBIC[:6], X, Y)
    return c, (cx, cy, r), (a, b, g), u, p


def _exact_traction(coefs, centre, r, mu, th):
    a, b, g = coefs
    X, Y = centre[0] - 0.5 + r * np.cos(th), centre[1] - 0.5 + r * np.sin(th)
    P = _poly(g, _CUBIC[:6], X, Y)
    ux, uy = _poly(a, _CUBIC, X, Y, 1, 0), _poly(a, _CUBIC, X, Y, 0, 1)
    vx, vy = _poly(b, _CUBIC, X, Y, 1, 0), _poly(b, _CUBIC, X, Y, 0, 1)
    sxx, syy, sxy = -P + 2 * mu * ux, -P + 2 * mu * vy, mu * (uy + vx)
    return np.stack([sxx * np.cos(th) + sxy * np.sin(th), sxy * np.cos(th) + syy * np.sin(th)])


@pytest.mark.parametrize("k", [3, 4])
def test_cylinder_force_divergence_theorem(orc, k):
    """Cubic velocity, quadratic pressure: the derivative operators and the
    interpolation reproduce them exactly (k >= 3), Simpson's rule integrates
    the resulting trigonometric polynomial exactly, and by the divergence
    theorem the force is pi R^2 (div sigma)(centre), div sigma being linear.
    A pure pressure p = -G x gives (G pi R^2, 0). C_D, C_L scale F by
    rho U^2 D / 2."""
    c, (cx, cy, r), (a, b, g), u, p = _cubic_case()
    ops = orc.build_operators(c, k)
    mu = 0.7
    F, trac, coef = orc.cylinder_forces(ops, u, p, (cx, cy), 2 * r, mu, 360, rho=1.3, u_ref=0.9)
    X0, Y0 = cx - 0.5, cy - 0.5
    div = np.array([
        -_poly(g, _CUBIC[:6], X0, Y0, 1, 0) + 2 * mu * _poly(a, _CUBIC, X0, Y0, 2, 0)
        + mu * (_poly(a, _CUBIC, X0, Y0, 0, 2) + _poly(b, _CUBIC, X0, Y0, 1, 1)),
        -_poly(g, _CUBIC[:6], X0, Y0, 0, 1) + 2 * mu * _poly(b, _CUBIC, X0, Y0, 0, 2)
        + mu * (_poly(a, _CUBIC, X0, Y0, 1, 1) + _poly(b, _CUBIC, X0, Y0, 2, 0))])
    np.testing.assert_allclose(F, math.pi * r * r * div, rtol=0, atol=1e-11)
    np.testing.assert_allclose(coef, F / (0.5 * 1.3 * 0.9 ** 2 * 2 * r), rtol=1e-15)
    th = 2 * np.pi * np.arange(360) / 360
    np.testing.assert_allclose(trac, _exact_traction((a, b, g), (cx, cy), r, mu, th), rtol=0, atol=1e-10)
    G = 1.7
    Fp, _ = orc.cylinder_forces(ops, np.zeros_like(u), -G * c.xyz[:, 0], (cx, cy), 2 * r, mu, 360)
    np.testing.assert_allclose(Fp, [G * math.pi * r * r, 0.0], rtol=0, atol=1e-12)


def test_cylinder_force_simpson_rule(orc):
    """The quadrature is the composite Simpson rule of the closed curve, not
    the trapezoidal rule: with 6 panels its value is Richardson's
    (4 T_6 - T_3) / 3 of the trapezoidal sums of the exact traction, which the
    degree-3 content of the integrand sets apart from the exact integral."""
    c, (cx, cy, r), coefs, u, p = _cubic_case()
    ops = orc.build_operators(c, 3)
    mu = 0.7

    def trap(N):
        th = 2 * np.pi * np.arange(N) / N
        return r * (2 * np.pi / N) * _exact_traction(coefs, (cx, cy), r, mu, th).sum(axis=1)

    F6, _ = orc.cylinder_forces(ops, u, p, (cx, cy), 2 * r, mu, 6)
    np.testing.assert_allclose(F6, (4 * trap(6) - trap(3)) / 3, rtol=0, atol=1e-12)
    assert np.abs(F6 - trap(360)).max() > 1e-3
    with pytest.raises(ValueError):
        orc.cylinder_forces(ops, u, p, (cx, cy), 2 * r, mu, 7)


def test_cylinder_force_kovasznay_converges(orc):
    """Kovasznay flow past a hole: the force approaches the exact surface
    integral (exact fields, central-difference strain rates, 4096-point
    trapezoidal rule) at the order of the operators."""
    Re = 40.0
    mu = 1.0 / Re

    def fields(x, y):
        return W.kovasznay(x, y, Re)

    def exact(cx, cy, r, N=4096, e=1e-6):
        th = 2 * np.pi * np.arange(N) / N
        X, Y = cx + r * np.cos(th), cy + r * np.sin(th)
        _, _, P = fields(X, Y)
        d = [(np.array(fields(X + e, Y)[i]) - fields(X - e, Y)[i]) / (2 * e) for i in (0, 1)]
        dy = [(np.array(fields(X, Y + e)[i]) - fields(X, Y - e)[i]) / (2 * e) for i in (0, 1)]
        sxx, syy, sxy = -P + 2 * mu * d[0], -P + 2 * mu * dy[1], mu * (dy[0] + d[1])
        return r * (2 * np.pi / N) * np.array([(sxx * np.cos(th) + sxy * np.sin(th)).sum(),
                                               (sxy * np.cos(th) + syy * np.sin(th)).sum()])
    errs = {}
    for nt in (3000, 12000):
        c = W.holed_square(nt, seed=5, n_holes=1)
        cx, cy, r = c.meta["holes"][0]
        Fe = exact(cx, cy, r)
        u, v, p = fields(c.xyz[:, 0], c.xyz[:, 1])
        for k in (3, 4):
            F, _ = orc.cylinder_forces(orc.build_operators(c, k), np.stack([u, v]), p, (cx, cy), 2 * r, mu)
            errs[nt, k] = np.abs(F - Fe).max() / np.abs(Fe).max()
    assert errs[3000, 3] < 3e-4 and errs[3000, 4] < 3e-6, errs
    assert errs[12000, 3] < errs[3000, 3] / 4, errs


# ---- interpolation on periodic clouds (Sec. 2 off the nodes, Sec. 3.1 periodic) ----
def _periodic_queries(c, rng, m=120):
    L = c.period[0]
    h = c.h
    near = rng.uniform(0, L, size=(m, 2))
    near[: m // 2, 0] = rng.choice([-1, 1], m // 2) * rng.uniform(0, h, m // 2) % L   # within h of the x seam
    near[m // 2:, 1] = rng.choice([-1, 1], m - m // 2) * rng.uniform(0, h, m - m // 2) % L
    inner = rng.uniform(0.3 * L, 0.7 * L, size=(m, 2))
    return near, inner


def test_periodic_interpolation_clouds_and_exactness(orc):
    """The clouds of query points near the seams are the q nearest by
    minimum-image distance (scipy's periodic k-d tree, independent code);
    constants are reproduced at any point, and a query on a node returns the
    nodal value."""
    from scipy.spatial import cKDTree
    c = W.taylor_green_periodic(nx=24)
    L = c.period[0]
    k = 3
    rng = np.random.default_rng(2)
    near, _ = _periodic_queries(c, rng)
    ones = np.ones(c.n)
    f = np.sin(c.xyz[:, 0]) * np.cos(c.xyz[:, 1])
    vals, nbr, w = orc.interpolate(c.xyz, k, near, [ones, f], period=c.period)
    q = nbr.shape[1]
    d_tree, _ = cKDTree(c.xyz, boxsize=L).query(near, q)
    dd = np.abs(c.xyz[nbr] - near[:, None, :])
    dd = np.minimum(dd, L - dd)
    d_ours = np.sort(np.sqrt((dd ** 2).sum(-1)), axis=1)
    np.testing.assert_allclose(d_ours, d_tree, rtol=0, atol=1e-12)
    np.testing.assert_allclose(vals[0], 1.0, rtol=0, atol=1e-12)
    nodes = c.xyz[rng.choice(c.n, 20, replace=False)]
    vn, _, _ = orc.interpolate(c.xyz, k, nodes, [f], period=c.period)
    fn = np.sin(nodes[:, 0]) * np.cos(nodes[:, 1])
    np.testing.assert_allclose(vn[0], fn, rtol=0, atol=1e-12)


def test_periodic_interpolation_seams_and_shifts(orc):
    """A smooth periodic field is interpolated as accurately next to the seams
    as inside (error ratio < 3), and queries moved by a period (outside the
    box) give the same values."""
    c = W.taylor_green_periodic(nx=32)
    L = c.period[0]
    k = 4
    rng = np.random.default_rng(4)
    near, inner = _periodic_queries(c, rng)
    f = np.sin(c.xyz[:, 0]) * np.cos(2 * c.xyz[:, 1])
    ex = lambda P: np.sin(P[:, 0]) * np.cos(2 * P[:, 1])     # noqa: E731
    vn, _, _ = orc.interpolate(c.xyz, k, near, [f], period=c.period)
    vi, _, _ = orc.interpolate(c.xyz, k, inner, [f], period=c.period)
    en, ei = np.abs(vn[0] - ex(near)).max(), np.abs(vi[0] - ex(inner)).max()
    assert en < 3 * ei and en < 1e-4, (en, ei)
    shifted = near + np.array([L, -L]) * rng.choice([0, 1], size=(len(near), 2))
    vs, _, _ = orc.interpolate(c.xyz, k, shifted, [f], period=c.period)
    np.testing.assert_allclose(vs[0], vn[0], rtol=0, atol=1e-12)


def test_cylinder_force_periodic_cell(orc):
    """One cell of a periodic cylinder array: near the cylinder no cloud
    reaches a seam, so cubic velocity and quadratic pressure are still
    reproduced there and the force is the divergence-theorem value
    pi R^2 (div sigma)(centre)."""
    c = W.periodic_cylinder_cell()
    cx, cy, r = c.meta["holes"][0]
    rng = np.random.default_rng(3)
    a, b, g = rng.standard_normal(10), rng.standard_normal(10), rng.standard_normal(6)
    X, Y = c.xyz[:, 0] - 0.5, c.xyz[:, 1] - 0.5
    u = np.stack([_poly(a, _CUBIC, X, Y), _poly(b, _CUBIC, X, Y)])
    p = _poly(g, _CUBIC[:6], X, Y)
    mu = 0.7
    F, _ = orc.cylinder_forces(orc.build_operators(c, 3), u, p, (cx, cy), 2 * r, mu, 360)
    X0, Y0 = cx - 0.5, cy - 0.5
    div = np.array([
        -_poly(g, _CUBIC[:6], X0, Y0, 1, 0) + 2 * mu * _poly(a, _CUBIC, X0, Y0, 2, 0)
        + mu * (_poly(a, _CUBIC, X0, Y0, 0, 2) + _poly(b, _CUBIC, X0, Y0, 1, 1)),
        -_poly(g, _CUBIC[:6], X0, Y0, 0, 1) + 2 * mu * _poly(b, _CUBIC, X0, Y0, 0, 2)
        + mu * (_poly(a, _CUBIC, X0, Y0, 1, 1) + _poly(b, _CUBIC, X0, Y0, 2, 0))])
    np.testing.assert_allclose(F, math.pi * r * r * div, rtol=0, atol=1e-11)


@pytest.mark.parametrize("k", [2, 3])
def test_inclined_symmetry_plane_keeps_the_stagnation_flow(orc, k):
    """The stagnation-flow square turned by 0.5 rad: its symmetry line is off
    the axes, so both velocity components are nonzero there and the two
    conditions (u . n = 0, no normal derivative of the tangential velocity)
    couple them. One BDF2 step from the exact (quadratic) flow returns it to
    solver accuracy; u_bc on the symmetry points is garbage and unread."""
    c = W.rotated(W.symmetric_square(), 0.5)
    ops = orc.build_operators(c, k)
    vel, p = W.flow_fields(c)
    sym = c.kind == W.SYMMETRY
    assert (np.abs(vel[:, sym]) > 1e-3).all()
    ubc = np.where(sym[None, :], 55.0, vel)
    u1, _, p1, st = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2,
                                    tol_outer=1e-13, tol_krylov=1e-14, max_outer=3, max_krylov=20000)
    assert np.abs(u1 - vel).max() <= 1e-10, np.abs(u1 - vel).max()
    assert np.abs(p1 - p).max() <= 1e-9, np.abs(p1 - p).max()


def test_inclined_symmetry_strip_keeps_kovasznay_flow(orc):
    """Kovasznay flow between its symmetry lines, the strip turned by 0.3 rad:
    from the exact state one outer iteration moves the velocity only by the
    discretization error, which shrinks with h (as on the unturned strip)."""
    changes = []
    for nx, ny in ((20, 5), (40, 10)):
        c = W.rotated(W.kovasznay_strip(nx=nx, ny=ny), 0.3)
        ops = orc.build_operators(c, 3)
        vel, p = W.flow_fields(c)
        u1, _, _, st = orc.simple_step(ops, vel, vel, p, vel, 1.0, 1.0 / 40, 0.01, alpha=orc.BDF2,
                                       tol_outer=0.0, tol_krylov=1e-12, max_outer=1, max_krylov=20000)
        changes.append(np.abs(u1 - vel).mean())
    assert changes[1] < changes[0] / 2 and changes[1] < 2e-3, changes


@pytest.mark.parametrize("angle", [0.0, 0.4])
def test_symmetry_plane_3d_keeps_the_stagnation_flow(orc, angle):
    """The 3D stagnation flow u = (x, y, -2z) with its symmetry plane z = 0,
    also with the cube turned by 0.4 rad about (1, 1, 0): the plane's normal
    then has three nonzero components, one normal and two tangential
    conditions couple all three velocity components. One BDF2 step from the
    exact (quadratic) flow returns it to solver accuracy."""
    c = W.symmetric_cube()
    if angle:
        c = W.rotated(c, angle, axis=(1.0, 1.0, 0.0))
    ops = orc.build_operators(c, 2)
    vel, p = W.flow_fields(c)
    sym = c.kind == W.SYMMETRY
    ubc = np.where(sym[None, :], 55.0, vel)
    u1, _, p1, st = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], 0.05, alpha=orc.BDF2, p_bc=p,
                                    tol_outer=1e-13, tol_krylov=1e-14, max_outer=3, max_krylov=20000)
    assert st["status"] == 0
    assert np.abs(u1 - vel).max() <= 1e-10, np.abs(u1 - vel).max()
    assert np.abs(p1 - p).max() <= 1e-9, np.abs(p1 - p).max()
