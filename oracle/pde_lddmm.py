"""Plain FP64 NumPy oracle of PDE-constrained LDDMM with velocity fields over time
(the comparison method of Section 2.3 of the paper: stationary and non-stationary
parameterisations, Gauss-Newton-Krylov on the reduced space).

TEST INFRASTRUCTURE ONLY (like the rest of this package): never part of the
product path.  Every step follows Section 2.3, written with whole-array NumPy and
the primitives of ``lddmm_oracle`` (L, K, central differences, periodic trilinear
interpolation, inner products).

Readings (the paper states the continuous equations only; each is also recorded
in the design notes):

M1  Time grid t_n = n dt, n = 0..nt, dt = 1/nt.  Non-stationary: one velocity
    field per time point, v_0..v_nt; the time integral of the regulariser is the
    trapezoid rule, int <L v_t, v_t> dt ~ sum_n w_n dt <L v_n, v_n>, w_0 = w_nt = 1/2,
    else 1.  Stationary: v_t = v for all t, regulariser <L v, v>.
M2  Energy exactly as printed (eq. LS-LDDMM, no 1/2 on either term); hence the
    L2 gradient per time point is 2 L v_t + lambda(t) grad m(t) (the printed
    "L v_t + lambda grad m" of eq. FirstOrder3 drops the 2 of the printed energy),
    with lambda(1) = -(2/sigma^2)(m(1) - I_1) as printed.
M3  State equation (eq. FirstOrder1) by semi-Lagrangian transport of the image
    itself: m_{n+1}(x) = m_n(X_n(x)), X_n = x - dt/2 (v_{n+1}(x) + v_n(x - dt v_{n+1}(x)))
    (Heun backtrace, as for the displacement of the main method).
M4  Adjoint equation (eq. FirstOrder2), -d_t lambda - div(lambda v) = 0, i.e.
    d_t lambda + v . grad lambda = -lambda div v, backward from t = 1 along the
    forward characteristics: lambda_n(x) = lambda_{n+1}(Y_n(x)) exp(dt/2 (div v_n(x) +
    div v_{n+1}(Y_n(x)))), Y_n = x + dt/2 (v_n(x) + v_{n+1}(x + dt v_n(x))) (Heun trace
    forward; trapezoid for the divergence factor; div by central differences).
M5  Incremental state (eq. SecondOrder1) by the same SL step with a trapezoidal
    source: dm_{n+1}(x) = dm_n(X_n) + dt/2 (s_n(X_n) + s_{n+1}(x)), s_n = -grad m_n . dv_n.
M6  Gauss-Newton (end of Section 2.3: drop the terms with lambda): incremental
    adjoint d_t dlambda + div(dlambda v) = 0 by M4 from dlambda_nt = -(2/sigma^2) dm_nt,
    and (H dv)_n = 2 L dv_n + dlambda_n grad m_n.  Stationary: the time integral of
    the pointwise terms, H dv = 2 L dv + sum_n w_n dt dlambda_n grad m_n.
M7  Optimise-then-discretise: the gradient and Hessian are the discretised
    continuous expressions, exact only up to discretisation error (pinned by
    convergence, not by identities).
M8  Solver (Section 2.3: Newton-Krylov on the reduced system with preconditioner
    K): Gauss-Newton, PCG in the L2 product over space and time (the M1 weights)
    with preconditioner K per time point, forcing eta = min(0.5, sqrt(||g||/||g_0||)),
    Armijo backtracking v <- v + tau p (the sign reading A1 of the main method).
"""

from __future__ import annotations

import math

import numpy as np

from . import lddmm_oracle as O


def weights(p, stationary):
    """Quadrature weights w_n dt of the time integral (M1); stationary: one field, weight 1."""
    if stationary:
        return np.array([1.0])
    w = np.full(p.nt + 1, p.dt)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def velocities(v, p, stationary):
    """The velocity at every time point: v_0..v_nt (M1)."""
    return [v] * (p.nt + 1) if stationary else [v[n] for n in range(p.nt + 1)]


def inner_t(a, b, p, stationary):
    """L2 product over space and time: sum_n w_n dt <a_n, b_n> (M1)."""
    w = weights(p, stationary)
    if stationary:
        return O.inner(a, b, p)
    return float(sum(w[n] * O.inner(a[n], b[n], p) for n in range(p.nt + 1)))


def div(v, p):
    """Central-difference divergence of a vector field."""
    return sum(O.ddx(v[d], d, p) for d in range(3))


def backtrace(v_old, v_new, p, x):
    """Foot at t_n of the characteristic through x at t_{n+1} (M3)."""
    return x - 0.5 * p.dt * (v_new + O.interp(v_old, x - p.dt * v_new, p))


def forward_trace(v_old, v_new, p, x):
    """Point at t_{n+1} of the characteristic through x at t_n (M4)."""
    return x + 0.5 * p.dt * (v_old + O.interp(v_new, x + p.dt * v_old, p))


def state(vs, I0, p):
    """m_0 = I_0, m_{n+1} = m_n o X_n (eq. FirstOrder1 by M3); returns [m_0 .. m_nt]."""
    x = O.grid_coords(p)
    m = [np.asarray(I0, dtype=np.float64)]
    for n in range(p.nt):
        m.append(O.interp(m[n], backtrace(vs[n], vs[n + 1], p, x), p))
    return m


def displacement(vs, p):
    """Inverse-map displacement of the PDE-LDDMM flow: u_0 = 0,
    u_{n+1}(x) = u_n(X_n(x)) + (X_n(x) - x) with the Heun foot X_n of M3, so that
    the deformed template is I_0 o (id + u_1); det(I + D u_1) gives the Jacobian
    extrema the paper reports for every method (Table 1)."""
    x = O.grid_coords(p)
    u = np.zeros((3,) + tuple(p.n))
    for n in range(p.nt):
        X = backtrace(vs[n], vs[n + 1], p, x)
        u = O.interp(u, X, p) + (X - x)
    return u


def adjoint(vs, lam1, p):
    """lambda_nt = lam1, backward by M4 (eq. FirstOrder2); returns [lambda_0 .. lambda_nt]."""
    x = O.grid_coords(p)
    lam = [None] * (p.nt + 1)
    lam[p.nt] = np.asarray(lam1, dtype=np.float64)
    for n in reversed(range(p.nt)):
        Y = forward_trace(vs[n], vs[n + 1], p, x)
        growth = 0.5 * p.dt * (div(vs[n], p) + O.interp(div(vs[n + 1], p), Y, p))
        lam[n] = O.interp(lam[n + 1], Y, p) * np.exp(growth)
    return lam


def energy(v, I0, I1, p, stationary, m=None):
    """E(v) = int <L v_t, v_t> dt + sigma^-2 ||m(1) - I_1||^2 (eq. LS-LDDMM, M1)."""
    vs = velocities(v, p, stationary)
    if m is None:
        m = state(vs, I0, p)
    w = weights(p, stationary)
    if stationary:
        ereg = O.inner(O.apply_L(v, p), v, p)
    else:
        ereg = float(sum(w[n] * O.inner(O.apply_L(vs[n], p), vs[n], p) for n in range(p.nt + 1)))
    r = m[-1] - I1
    return ereg + O.inner(r, r, p) / p.sigma2


class Linearization:
    """State, adjoint and energy at one v."""

    def __init__(self, v, I0, I1, p, stationary):
        self.v = np.array(v, dtype=np.float64)
        self.stationary = stationary
        self.vs = velocities(self.v, p, stationary)
        self.m = state(self.vs, I0, p)
        self.grad_m = [O.grad(mn, p) for mn in self.m]
        self.E = energy(self.v, I0, I1, p, stationary, self.m)
        self.residual = self.m[-1] - I1


def gradient(v, I0, I1, p, stationary, lin=None):
    """L2 gradient (eq. FirstOrder3 with M2): g_n = 2 L v_n + lambda_n grad m_n, or its
    time integral for the stationary velocity.  Returns (g, lin)."""
    if lin is None:
        lin = Linearization(v, I0, I1, p, stationary)
    lam = adjoint(lin.vs, -(2.0 / p.sigma2) * lin.residual, p)
    terms = [lam[n][None] * lin.grad_m[n] for n in range(p.nt + 1)]
    if stationary:
        w = weights(p, False)
        return 2.0 * O.apply_L(lin.v, p) + sum(w[n] * terms[n] for n in range(p.nt + 1)), lin
    return np.stack([2.0 * O.apply_L(lin.vs[n], p) + terms[n] for n in range(p.nt + 1)]), lin


def incremental_state(dvs, lin, p):
    """dm_0 = 0; dm_{n+1} = dm_n o X_n + dt/2 (s_n o X_n + s_{n+1}), s_n = -grad m_n . dv_n
    (eq. SecondOrder1 by M5); returns dm_nt."""
    x = O.grid_coords(p)
    dm = np.zeros(p.n)
    s = -np.sum(lin.grad_m[0] * dvs[0], axis=0)
    for n in range(p.nt):
        X = backtrace(lin.vs[n], lin.vs[n + 1], p, x)
        s_next = -np.sum(lin.grad_m[n + 1] * dvs[n + 1], axis=0)
        dm = O.interp(dm, X, p) + 0.5 * p.dt * (O.interp(s, X, p) + s_next)
        s = s_next
    return dm


def hessvec(dv, lin, p):
    """Gauss-Newton Hessian in L2 (eqs. SecondOrder1-3 with the lambda terms dropped, M6)."""
    dvs = velocities(np.asarray(dv, dtype=np.float64), p, lin.stationary)
    dm1 = incremental_state(dvs, lin, p)
    dlam = adjoint(lin.vs, -(2.0 / p.sigma2) * dm1, p)
    terms = [dlam[n][None] * lin.grad_m[n] for n in range(p.nt + 1)]
    if lin.stationary:
        w = weights(p, False)
        return 2.0 * O.apply_L(dv, p) + sum(w[n] * terms[n] for n in range(p.nt + 1))
    return np.stack([2.0 * O.apply_L(dvs[n], p) + terms[n] for n in range(p.nt + 1)])


def precondition(r, p, stationary):
    """K per time point (the preconditioner of Section 2.3)."""
    return O.apply_K(r, p) if stationary else np.stack([O.apply_K(r[n], p) for n in range(p.nt + 1)])


def pcg(hess, g, p, stationary, eta, maxit):
    """PCG in the space-time L2 product for H x = -g with preconditioner K; stops at
    ||r|| <= eta ||g|| or on non-positive curvature.  Returns (x, iterations)."""
    ip = lambda a, b: inner_t(a, b, p, stationary)
    x = np.zeros_like(g)
    r = -np.asarray(g, dtype=np.float64)
    z = precondition(r, p, stationary)
    d = z.copy()
    rz = ip(r, z)
    tol = eta * math.sqrt(ip(g, g))
    it = 0
    for it in range(1, maxit + 1):
        q = hess(d)
        dq = ip(d, q)
        if dq <= 0.0:
            it -= 1
            break
        a = rz / dq
        x = x + a * d
        r = r - a * q
        if math.sqrt(ip(r, r)) <= tol:
            break
        z = precondition(r, p, stationary)
        rz_new = ip(r, z)
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, it


def gn_solve(I0, I1, p, stationary, gn_iters=10, cg_iters=20, c1=1e-4, max_halvings=10, gtol=1e-3, v0=None):
    """Gauss-Newton-Krylov for PDE-LDDMM (Section 2.3, M8).  Returns (v, log, lin) with
    log entries (E, g_norm, cg_iters, eta, tau) per outer iteration."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    shape = (3,) + tuple(p.n) if stationary else (p.nt + 1, 3) + tuple(p.n)
    v = np.zeros(shape) if v0 is None else np.array(v0, dtype=np.float64)
    log = []
    g0 = None
    for _ in range(gn_iters):
        g, lin = gradient(v, I0, I1, p, stationary)
        gn = math.sqrt(inner_t(g, g, p, stationary))
        if g0 is None:
            g0 = gn
        if g0 == 0.0 or gn / g0 <= gtol:
            break
        eta = min(0.5, math.sqrt(gn / g0))
        step, its = pcg(lambda d: hessvec(d, lin, p), g, p, stationary, eta, cg_iters)
        gp = inner_t(g, step, p, stationary)
        tau, accepted = 1.0, False
        for _ in range(max_halvings + 1):
            if energy(v + tau * step, I0, I1, p, stationary) <= lin.E + c1 * tau * gp:
                accepted = True
                break
            tau *= 0.5
        log.append(dict(E=lin.E, g_norm=gn, cg_iters=its, eta=eta, tau=tau if accepted else 0.0))
        if not accepted:
            break
        v = v + tau * step
    return v, log, Linearization(v, I0, I1, p, stationary)
