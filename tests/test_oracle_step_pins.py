"""Pins of the oracle's time step that the step's own output cannot supply:
hand values of its reductions, the discrete continuity of the new velocity,
the temporal order of BDF2, the Beltrami near fixed point, and the linear
analysis of the outer iteration (CPU only).

Each pin is chosen so that a plausible slip fails it:
  - Delta and eps_s (Sec. 3.2 step 7; Sec. 4.1 steady error) on a flow whose
    per-step change is known by hand: a missing 1/n, a max for a sum (or the
    reverse), or a mean over the wrong points moves them by factors;
  - the continuity error (Eq. continuity:n+1) reported by the step must be
    the interior mean of |D . u| of the new velocity;
  - BDF2 (Eqs. u:n+1, v:n+1) must be second order in dt: a BDF1 step or a
    misplaced coefficient drops the ratio of errors at dt and dt/2 from 4 to 2
    or less;
  - one outer iteration from the exact Ethier-Steinman flow must land within
    a discretization error of the exact flow at t + dt, shrinking with h;
  - the outer iteration's linearisation (assembled densely below from the
    oracle's own operators) must reproduce one oracle outer iteration, and its
    spectral radius tells whether the iteration contracts.
"""
import numpy as np
import pytest

import workloads as W


# ------------------------------------------------------------- reductions

@pytest.mark.parametrize("dim,kind", [(2, W.DIRICHLET), (2, W.PRESCRIBED_PRESSURE), (3, W.PRESCRIBED_PRESSURE)])
@pytest.mark.parametrize("bdf", ["BDF1", "BDF2"])
def test_step_reductions_hand_values(orc, dim, kind, bdf):
    """The uniform flow u(t) = a0 + a1 t (driven by p = -rho a1 . x) is
    reproduced exactly in one outer iteration (degree >= 2). Over that
    iteration the interior points move by a1 dt and the velocity-prescribed
    boundary points, which start at their t^{n+1} values, do not move:
      Delta = sum_c |a1_c| dt * n_interior / n,
    while over the step every point moves by a1 dt:
      eps_s = max_c |a1_c|.
    A second outer iteration changes nothing (Delta = 0), and the constant
    field has no discrete divergence."""
    c = (W.kovasznay_square(nx=12, boundary_kind=kind) if dim == 2
         else W.scattered_cube(7, seed=3, boundary_kind=kind))
    ops = orc.build_operators(c, 2)
    rho, mu, dt, t = 1.0, 0.05, 0.04, 0.3
    un, pn = W.polynomial_flow(c.xyz, t, "uniform", rho)
    um, _ = W.polynomial_flow(c.xyz, t - dt, "uniform", rho)
    ue, pe = W.polynomial_flow(c.xyz, t + dt, "uniform", rho)
    a1 = np.array([0.5, 0.3, -0.4])[:dim]       # the generator's du/dt
    np.testing.assert_allclose(ue[:, 0] - un[:, 0], a1 * dt, rtol=1e-14)
    pbc = pe if kind == W.PRESCRIBED_PRESSURE else None
    n_int = int((c.kind == W.INTERIOR).sum())
    kw = dict(tol_outer=0.0, tol_krylov=1e-13, max_krylov=20000, p_bc=pbc)
    u1, _, _, st1 = orc.simple_step(ops, un, um, pn, ue, rho, mu, dt, alpha=getattr(orc, bdf), max_outer=1, **kw)
    u2, _, _, st2 = orc.simple_step(ops, un, um, pn, ue, rho, mu, dt, alpha=getattr(orc, bdf), max_outer=2, **kw)
    assert np.abs(u1 - ue).max() <= 1e-10
    delta_hand = np.abs(a1).sum() * dt * n_int / c.n
    assert st1["delta"] == pytest.approx(delta_hand, rel=1e-9)
    assert st1["eps_steady"] == pytest.approx(np.abs(a1).max(), rel=1e-9)
    assert st2["eps_steady"] == pytest.approx(np.abs(a1).max(), rel=1e-9)
    assert st2["delta"] <= 1e-10 * delta_hand
    assert st1["div_l1"] <= 1e-11


# ------------------------------------------------------ discrete continuity

def test_continuity_error_of_the_step(orc):
    """The step's div_l1 is the mean |Dx u + Dy v| over interior points of the
    new velocity (Eq. continuity:n+1), recomputed here from the operators, on
    the Taylor-Green disk (prescribed-pressure boundary) at Courant number 10
    and at half its dt. It stays far below the velocity's derivative scale
    (|u| ~ 1 per unit length) but well above the exact field's own discrete
    divergence: the outer iteration stops short of the fixed point where the
    pressure correction would remove it, so the error shrinks with dt rather
    than with h (the same cloud at half the dt, 20 outer iterations each)."""
    c = W.taylor_green_disk(r=0.08)
    ops = orc.build_operators(c, 4)
    vel, p = W.flow_fields(c, 0.0)
    inner = c.kind == W.INTERIOR
    dt10 = orc.dt_from_courant(ops, vel, 10.0, 1.0, c.meta["nu"])
    d_exact = orc.spmv(ops.col, ops.val[0], vel[0]) + orc.spmv(ops.col, ops.val[1], vel[1])
    out = []
    for dt in (dt10, dt10 / 2):
        ubc, pbc = W.flow_fields(c, dt)
        u, _, _, st = orc.simple_step(ops, vel, vel, p, ubc, 1.0, c.meta["nu"], dt, alpha=orc.BDF1, tol_outer=0.0,
                                      tol_krylov=1e-12, max_outer=20, max_krylov=20000, p_bc=pbc)
        div = orc.spmv(ops.col, ops.val[0], u[0]) + orc.spmv(ops.col, ops.val[1], u[1])
        d_mean = float(np.abs(div[inner]).mean())
        assert st["div_l1"] == pytest.approx(d_mean, rel=1e-9)
        assert d_mean < 1e-2
        out.append(d_mean)
    print(f"[continuity] dt {dt10:.3f}: {out[0]:.3e}, dt/2: {out[1]:.3e}; exact field "
          f"{np.abs(d_exact[inner]).mean():.3e}")
    assert out[1] < out[0]
    assert out[1] > 10 * float(np.abs(d_exact[inner]).mean())


# ------------------------------------------------------------- BDF2 order

def test_bdf2_is_second_order_in_time(orc):
    """Periodic Taylor-Green vortex (no boundary, nu = 0.1) on one fixed
    cloud to T = 0.5: the difference from a run at dt = T/64 falls 4x when dt
    halves (Eqs. u:n+1, v:n+1 with a BDF1 first step), and the kinetic energy
    decays as exp(-4 nu t), the closed form's rate."""
    nu, T, k = 0.1, 0.5, 4
    c = W.taylor_green_periodic(nx=24, nu=nu)
    ops = orc.build_operators(c, k)
    x, y = c.xyz[:, 0], c.xyz[:, 1]
    u0, v0, p0 = W.taylor_green(x, y, 0.0, nu=nu)
    vel = np.stack([u0, v0])

    def run(m):
        u, _, _ = orc.run_transient(ops, vel, p0, lambda t: vel, 1.0, nu, T / m, m, tol_outer=0.0,
                                    tol_krylov=1e-12, max_outer=40, max_krylov=20000)
        return u

    ref = run(32)
    e = [float(np.abs(run(m) - ref).max()) for m in (4, 8)]
    ratio = e[0] / e[1]
    print(f"[bdf2] errors {e}, ratio {ratio:.2f}")
    assert 3.5 <= ratio <= 4.7
    ke = lambda u: float((u * u).sum())
    decay = ke(ref) / ke(vel)
    assert decay == pytest.approx(np.exp(-4 * nu * T), rel=5e-3)


# ---------------------------------------------------------- Beltrami (3D)

def test_beltrami_flow_is_a_near_fixed_point(orc):
    """One outer iteration (BDF2, dt = 0.01) from the exact Ethier-Steinman
    flow at t = 0.1 lands within a discretization error of the exact flow at
    t + dt on the interior points, falling with h at order >= 2."""
    errs = []
    for n in (6, 10):
        c = W.beltrami_cube(n=n)
        ops = orc.build_operators(c, 3)
        x, y, z = c.xyz.T

        def flow(t):
            u, v, w, p = W.beltrami(x, y, z, t)
            return np.stack([u, v, w]), p

        t0, dt = 0.1, 0.01
        un, pn = flow(t0)
        um, _ = flow(t0 - dt)
        ue, pe = flow(t0 + dt)
        u, _, _, st = orc.simple_step(ops, un, um, pn, ue, 1.0, 0.01, dt, alpha=orc.BDF2, tol_outer=0.0,
                                      tol_krylov=1e-12, max_outer=1, max_krylov=20000, p_bc=pe)
        inner = c.kind == W.INTERIOR
        errs.append((1.0 / n, float(np.abs(u - ue)[:, inner].mean())))
        # a sign slip in advection moves u by ~dt |u.grad u| ~ 1e-2
        assert errs[-1][1] < 1e-4
    (h1, e1), (h2, e2) = errs
    order = np.log(e1 / e2) / np.log(h1 / h2)
    print(f"[beltrami] one-iteration errors {errs}, order {order:.2f}")
    assert order >= 2.0


# ------------------------------------- linear analysis of the outer iteration

def _dense(col, val):
    n, q = col.shape
    A = np.zeros((n, n))
    np.add.at(A, (np.repeat(np.arange(n), q), col.ravel()), val.ravel())
    return A


def _stokes_outer_jacobian(c, ops, rho, mu, dt, a1):
    """d p^{r+1} / d p^r of one outer iteration for Stokes flow (zero base
    velocity and zero data, so the map is linear): momentum (Eq. u:tilde without
    advection) with identity rows on velocity-prescribed points, pressure
    correction (Eq. pressure poisson), interior p += p', boundary pressure from
    the normal momentum block (Eq. normal momentum with the other pressures
    held), assembled densely from the oracle's operators."""
    n, d = c.n, c.dim
    D = [_dense(ops.col, ops.val[e]) for e in range(d)]
    L = _dense(ops.col, ops.val[d])
    P = _dense(ops.col, ops.pval)
    inner = c.kind == W.INTERIOR
    A = rho * a1 / dt * np.eye(n) - mu * L
    A[~inner] = 0.0
    bi = np.where(~inner)[0]
    A[bi, bi] = 1.0
    Ainv = np.linalg.inv(A)
    Ut = []
    for e in range(d):
        G = D[e].copy()
        G[~inner] = 0.0
        Ut.append(-Ainv @ G)
    F = rho * a1 / dt * sum(D[e] @ Ut[e] for e in range(d))
    F[~inner] = 0.0
    if c.pin >= 0:
        F[c.pin] = 0.0
    J = np.eye(n) + np.linalg.solve(P, F)
    J[~inner] = 0.0
    nb = (c.kind == W.DIRICHLET) | (c.kind == W.SYMMETRY)
    if nb.any():
        b = np.where(nb)[0]
        RB = np.zeros((len(b), n))
        for e in range(d):
            comp = -rho * a1 / dt * Ut[e] + mu * (L @ Ut[e])
            RB += c.normal[b, e][:, None] * comp[b]
        Pother = P[b].copy()
        Pother[:, b] = 0.0
        J[b] = np.linalg.solve(P[np.ix_(b, b)], RB - Pother @ J)
    return J


@pytest.mark.parametrize("kind", [W.DIRICHLET, W.PRESCRIBED_PRESSURE])
def test_outer_iteration_linearisation(orc, kind):
    """On a 741-point Couette annulus (k = 3, dt = 0.05) the dense Jacobian of
    the Stokes outer iteration reproduces one oracle outer iteration from a
    random pressure. Its spectral radius is the iteration's contraction
    factor: with velocity walls and homogeneous Neumann p' (the paper's
    closure) it exceeds 8, the dominant mode living on the wall pressures;
    with prescribed-pressure walls it is near 1. This is why the steady
    Couette and Kovasznay marches of Sec. 4 do not converge under these
    readings."""
    c = W.couette_annulus(0.05, boundary_kind=kind)
    ops = orc.build_operators(c, 3)
    rho, mu, dt = 1.0, 0.01, 0.05
    J = _stokes_outer_jacobian(c, ops, rho, mu, dt, 1.5)
    p0 = np.random.default_rng(5).standard_normal(c.n)
    z = np.zeros((2, c.n))
    _, _, p1, st = orc.simple_step(ops, z, z, p0, z, rho, mu, dt, alpha=orc.BDF2, tol_outer=0.0, tol_krylov=1e-11,
                                   max_outer=1, max_krylov=50000, p_bc=np.zeros(c.n) if kind != W.DIRICHLET else None)
    jp = J @ p0
    err = np.abs(p1 - jp).max() / np.abs(jp).max()
    ev = np.linalg.eigvals(J)
    rad = float(np.abs(ev).max())
    print(f"[outer] kind {kind}: n={c.n}, one iteration vs Jacobian {err:.1e}, spectral radius {rad:.3f}")
    assert err <= 1e-7
    if kind == W.DIRICHLET:
        assert rad > 8.0
        v = np.abs(np.linalg.eig(J)[1][:, np.argmax(np.abs(ev))])
        assert c.kind[np.argmax(v)] == W.DIRICHLET
    else:
        assert 0.9 < rad < 1.1


def _outer_jacobian_variant(c, ops, rho, mu, dt, a1, base, pop):
    """Pressure-to-pressure Jacobian of one outer iteration, linearised about a
    frozen advecting velocity `base`, under two alternative readings studied
    for velocity walls:
      - the p' operator is either the PHS Laplacian (`pop` = "lap", Eq.
        pressure poisson discretised directly) or the discrete divergence of
        the interior-corrected gradient (`pop` = "divgrad": imposing the
        discrete continuity equation on the corrected velocity, as the
        equation is derived in Sec. 3);
      - the wall pressure comes from the normal momentum block (Eq. normal
        momentum) with its right-hand side taken from time level n, so that
        within the step it follows the interior pressure only.
    Homogeneous Neumann p' rows at the walls and the pin row as in the
    oracle."""
    n, d = c.n, c.dim
    D = [_dense(ops.col, ops.val[e]) for e in range(d)]
    L = _dense(ops.col, ops.val[d])
    inner = c.kind == W.INTERIOR
    b = np.where(~inner)[0]
    A = rho * a1 / dt * np.eye(n) - mu * L + rho * sum(base[f][:, None] * D[f] for f in range(d))
    A[~inner] = 0.0
    A[b, b] = 1.0
    Ainv = np.linalg.inv(A)
    Gi = []
    for e in range(d):
        G = D[e].copy()
        G[~inner] = 0.0
        Gi.append(G)
    F = rho * a1 / dt * sum(D[e] @ (-Ainv @ Gi[e]) for e in range(d))
    F[~inner] = 0.0
    P = L.copy() if pop == "lap" else sum(D[e] @ Gi[e] for e in range(d))
    Nd = sum(c.normal[:, e][:, None] * D[e] for e in range(d))
    P[b] = Nd[b]
    P[c.pin] = 0.0
    P[c.pin, c.pin] = 1.0
    F[c.pin] = 0.0
    J = np.eye(n) + np.linalg.solve(P, F)
    Po = Nd[b].copy()
    Po[:, b] = 0.0
    J[b] = np.linalg.solve(Nd[np.ix_(b, b)], -Po @ J)
    return J


def test_outer_iteration_alternative_readings(orc):
    """The alternative readings for velocity walls, on the same 741-point
    annulus (k = 3) with the advection of the exact Couette flow: with the
    PHS Laplacian as the p' operator the iteration diverges at every Courant
    number; with the divergence of the interior-corrected gradient and a
    time-level-n wall pressure it contracts at Co 1 but not at Co 8 (the
    paper's setting), where its largest eigenvalue besides the pressure
    level's exceeds 1. None of the readings therefore gives the paper's
    converged Co 8-12 Couette march."""
    c = W.couette_annulus(0.05)
    ops = orc.build_operators(c, 3)
    vel, _ = W.flow_fields(c)
    nu = c.meta["nu"]
    lam = orc.convdiff_lambda(ops, vel, 1.0, nu)
    rad = {}
    for co in (1.0, 8.0):
        for pop in ("lap", "divgrad"):
            J = _outer_jacobian_variant(c, ops, 1.0, nu, 2 * co / lam, 1.5, vel, pop)
            ev = np.linalg.eigvals(J)
            ev = ev[np.abs(ev - 1.0) > 1e-7]   # the pressure level: p' leaves it unchanged
            rad[(co, pop)] = float(np.abs(ev).max())
    print("[outer] spectral radii", {k: round(v, 3) for k, v in rad.items()})
    assert rad[(1.0, "lap")] > 1.5 and rad[(8.0, "lap")] > 1.5
    assert rad[(1.0, "divgrad")] < 0.9
    assert rad[(8.0, "divgrad")] > 1.02
