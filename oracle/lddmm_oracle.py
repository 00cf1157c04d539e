"""Plain FP64 NumPy oracle of the PDE-EPDiff LDDMM hot path.

TEST INFRASTRUCTURE ONLY (see the package docstring): never part of the product
path.  It is written for readability, not speed: every operator is a whole-array
NumPy expression following the paper's equations in the paper's order.

Paper: M. Hernandez, "PDE-constrained LDDMM via geodesic shooting and inexact
Gauss-Newton-Krylov optimization using the incremental adjoint Jacobi equations"
(arXiv 1807.04638).  References below name its sections and equations.

The paper states the continuous equations only.  The discrete readings used here
(each one also recorded in the design notes) are:

R1  Domain [0, 2*pi)^3, periodic; h_d = 2*pi / N_d; <a, b> = h0 h1 h2 sum a.b.
R2  L = (Id - alpha*Laplacian)^s applied spectrally with integer wavenumbers:
    L^(k) = (1 + alpha |k|^2)^s, K^ = 1 / L^ (Section 2.1, metric operator).
R3  Second-order periodic central differences delta_d.
R4  ad_v w = (Dv) w - (Dw) v, the sign for which the printed ad* of the EPDiff
    equation (Section 2.2) is its L2 adjoint.
R5  ad*_v mu in conservative form: (Dv)^T mu + sum_d delta_d(mu v_d); equal to the
    printed (Dv)^T mu + D(mu) v + mu div v by the product rule, and the exact
    discrete transpose of ad_v.
R6  Heun (RK2) in time on the momentum mu = L v with dt = 1/nt; the predictors
    (mu*_n, v*_n) are stored.
R7  State equation (Section 2.3, transport of the image) by semi-Lagrangian
    transport of the inverse-map displacement u along Heun-backtraced
    characteristics and one trilinear composition J_1 = I_0 o (id + u_1).
R8  Incremental state in Jacobi form: delta m_1 = -grad(J_1) . X_1 with
    dX/dt = delta v + ad_v X, X_0 = 0.
A1  The update is v0 <- v0 + tau p with H p = -g (the printed "minus epsilon"
    step with H delta v = -grad E would ascend); tau by Armijo backtracking.
A2  Incremental initial condition delta v(0) = the PCG direction (the printed
    delta v(0) = 0 would make the linear system trivially zero).
A3  Gauss-Newton drops every term containing the first-order adjoint fields and
    lambda(1) grad(delta m(1)); the incremental adjoint sweep is then the adjoint
    Jacobi sweep with a new final condition, and H = 2 I + (2/sigma^2) F* F.
A17 "GN, L2" (Section 3, last remark; Table 1): gradient L g_V and Hessian
    L H_V in the L2 product, solved by PCG with preconditioner K; every norm of
    that solve (CG stop, forcing term, outer stop) is the L2 norm.
A18 Gradient descent in V (Section 2.2): v0 <- v0 - tau g_V, tau by Armijo
    backtracking from tau0 = 1/2, the exact minimiser along -g of the
    regularisation term (its V-Hessian is 2 I).
A19 Full Newton (Section 3 before the Gauss-Newton drops): the incremental adjoint
    sweep is the exact linearisation of the discrete adjoint sweep with respect to
    the trajectory (tangent stage variations), plus lambda_1 grad(delta m_1) in its
    final condition, delta m_1 in Jacobi form (R8).  CG meeting non-positive
    curvature on its first direction returns -g (steepest descent).
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

_WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------------------
# Parameters and grid (R1)
# ---------------------------------------------------------------------------


@dataclass
class Params:
    """Grid and model constants: n = (N0, N1, N2), alpha and s of L, nt time steps, sigma^2."""

    n: tuple
    alpha: float
    s: int
    nt: int
    sigma2: float = 1.0

    @property
    def h(self):
        return tuple(2.0 * math.pi / N for N in self.n)

    @property
    def dt(self):
        return 1.0 / self.nt

    @property
    def cell(self):
        h = self.h
        return h[0] * h[1] * h[2]


def inner(a, b, p):
    """L2 inner product <a, b> = h0 h1 h2 sum_i sum_c a_c[i] b_c[i] (R1)."""
    return p.cell * float(np.sum(np.asarray(a, dtype=np.float64) * np.asarray(b, dtype=np.float64)))


def inner_V(a, b, p):
    """V inner product <a, b>_V = <L a, b> (Section 2.1, metric of V)."""
    return inner(apply_L(a, p), b, p)


def grid_coords(p):
    """Physical coordinates x_i = i * h_d as a (3, N0, N1, N2) array."""
    h = p.h
    ax = [np.arange(N, dtype=np.float64) * h[d] for d, N in enumerate(p.n)]
    X = np.meshgrid(*ax, indexing="ij")
    return np.stack(X)


# ---------------------------------------------------------------------------
# O1: the metric operator L and its inverse K (Section 2.1; R2)
# ---------------------------------------------------------------------------


def symbol_L(p):
    """Fourier symbol (1 + alpha |k|^2)^s on the real-FFT half spectrum, integer k."""
    n = p.n
    k0 = sfft.fftfreq(n[0], 1.0 / n[0])
    k1 = sfft.fftfreq(n[1], 1.0 / n[1])
    k2 = sfft.rfftfreq(n[2], 1.0 / n[2])
    kk = k0[:, None, None] ** 2 + k1[None, :, None] ** 2 + k2[None, None, :] ** 2
    return (1.0 + p.alpha * kk) ** p.s


def _spectral(f, p, mult):
    f = np.asarray(f, dtype=np.float64)
    F = sfft.rfftn(f, axes=(-3, -2, -1), workers=_WORKERS)
    return sfft.irfftn(F * mult, s=p.n, axes=(-3, -2, -1), workers=_WORKERS)


def apply_L(f, p):
    """L f for a scalar (N0,N1,N2) or vector (3,N0,N1,N2) field."""
    return _spectral(f, p, symbol_L(p))


def apply_K(f, p):
    """K f = L^{-1} f."""
    return _spectral(f, p, 1.0 / symbol_L(p))


# ---------------------------------------------------------------------------
# O2: derivatives, ad and ad* (Section 2.2, EPDiff equation; R3-R5)
# ---------------------------------------------------------------------------


def ddx(f, d, p):
    """Periodic central difference along axis d: (f[i+e_d] - f[i-e_d]) / (2 h_d)."""
    ax = f.ndim - 3 + d
    return (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2.0 * p.h[d])


def grad(f, p):
    """Central-difference gradient of a scalar field, shape (3, N0, N1, N2)."""
    return np.stack([ddx(f, d, p) for d in range(3)])


def ad(v, w, p):
    """ad_v w = (Dv) w - (Dw) v, with (Dv)_{cd} = delta_d v_c (R4)."""
    out = np.zeros_like(w, dtype=np.float64)
    for c in range(3):
        for d in range(3):
            out[c] += ddx(v[c], d, p) * w[d] - ddx(w[c], d, p) * v[d]
    return out


def ad_star(v, mu, p):
    """ad*_v mu = (Dv)^T mu + sum_d delta_d(mu v_d) (conservative form, R5)."""
    out = np.zeros_like(mu, dtype=np.float64)
    for c in range(3):
        for d in range(3):
            out[c] += ddx(v[d], c, p) * mu[d] + ddx(mu[c] * v[d], d, p)
    return out


def ad_dagger(v, w, p):
    """ad^dagger_v w = K ad*_v L w, the V-adjoint of ad_v (Section 2.2)."""
    return apply_K(ad_star(v, apply_L(w, p), p), p)


# ---------------------------------------------------------------------------
# Trilinear periodic interpolation (R7)
# ---------------------------------------------------------------------------


def interp(f, y, p):
    """Evaluate f at physical points y (3, ...) by periodic trilinear interpolation.

    q = y / h, j = floor(q), t = q - j, neighbour indices taken modulo N.
    ``f`` is scalar (N0,N1,N2) or has leading component axes.
    """
    n, h = p.n, p.h
    j, t = [], []
    for d in range(3):
        q = y[d] / h[d]
        jd = np.floor(q)
        t.append(q - jd)
        j.append(jd.astype(np.int64))
    lead = f.shape[:-3]
    out = np.zeros(lead + y.shape[1:], dtype=np.float64)
    for c0 in (0, 1):
        w0 = t[0] if c0 else 1.0 - t[0]
        i0 = (j[0] + c0) % n[0]
        for c1 in (0, 1):
            w1 = t[1] if c1 else 1.0 - t[1]
            i1 = (j[1] + c1) % n[1]
            for c2 in (0, 1):
                w2 = t[2] if c2 else 1.0 - t[2]
                i2 = (j[2] + c2) % n[2]
                out += (w0 * w1 * w2) * f[..., i0, i1, i2]
    return out


def sl_step(u, v_old, v_new, p, x=None):
    """One semi-Lagrangian step of the inverse-map displacement (Section 2.3, state equation; R7).

    Foot point by Heun backtracing with grid-time velocities:
      X = x - dt/2 (v_new(x) + v_old(x - dt v_new(x))),  u_new(x) = u(X) + (X - x).
    """
    if x is None:
        x = grid_coords(p)
    dt = p.dt
    pred = x - dt * v_new
    X = x - 0.5 * dt * (v_new + interp(v_old, pred, p))
    return interp(u, X, p) + (X - x)


# ---------------------------------------------------------------------------
# O3/O4: forward shooting (Section 3 constraints: EPDiff + state equation)
# ---------------------------------------------------------------------------


@dataclass
class Trajectory:
    """Stored geodesic: (mu_n, v_n) for n = 0..nt and Heun predictors (mu*_n, v*_n), n < nt."""

    mu: list
    v: list
    mu_star: list
    v_star: list
    u: np.ndarray = None
    J1: np.ndarray = None
    drift: list = field(default_factory=list)


def shoot(v0, p, I0=None):
    """EPDiff geodesic shooting in momentum form with Heun steps (R6).

    mu_0 = L v0, v_0 = v0;  mu*_n = mu_n - dt ad*_{v_n} mu_n, v*_n = K mu*_n;
    mu_{n+1} = 1/2 mu_n + 1/2 (mu*_n - dt ad*_{v*_n} mu*_n), v_{n+1} = K mu_{n+1}.
    If I0 is given, the displacement u is transported alongside and J_1 = I0 o (id + u_nt).
    """
    dt = p.dt
    v = np.array(v0, dtype=np.float64)
    mu = apply_L(v, p)
    tr = Trajectory([mu], [v], [], [])
    e0 = inner(mu, v, p)
    tr.drift.append(0.0)
    x = grid_coords(p) if I0 is not None else None
    u = np.zeros_like(v) if I0 is not None else None
    for _ in range(p.nt):
        ms = mu - dt * ad_star(v, mu, p)
        vs = apply_K(ms, p)
        mu_new = 0.5 * mu + 0.5 * (ms - dt * ad_star(vs, ms, p))
        v_new = apply_K(mu_new, p)
        if I0 is not None:
            u = sl_step(u, v, v_new, p, x)
        tr.mu_star.append(ms)
        tr.v_star.append(vs)
        tr.mu.append(mu_new)
        tr.v.append(v_new)
        mu, v = mu_new, v_new
        tr.drift.append(inner(mu, v, p) / e0 - 1.0 if e0 != 0.0 else 0.0)
    if I0 is not None:
        tr.u = u
        tr.J1 = interp(np.asarray(I0, dtype=np.float64), x + u, p)
    return tr


def sl_transport(vs, p):
    """Run only the semi-Lagrangian part (R7) over a prescribed velocity list v_0..v_nt."""
    x = grid_coords(p)
    u = np.zeros_like(vs[0], dtype=np.float64)
    for n in range(p.nt):
        u = sl_step(u, vs[n], vs[n + 1], p, x)
    return u


def compose(I0, u, p):
    """J = I0 o (id + u) by periodic trilinear interpolation."""
    return interp(np.asarray(I0, dtype=np.float64), grid_coords(p) + u, p)


# ---------------------------------------------------------------------------
# O5: energy and final conditions (Section 3 energy; Section 2.3 lambda(1))
# ---------------------------------------------------------------------------


def energy_terms(v0, J1, I1, p, mu0=None):
    """E = <L v0, v0> + sigma^-2 ||J_1 - I_1||^2, returned as (E, E_reg, E_data)."""
    if mu0 is None:
        mu0 = apply_L(v0, p)
    r = J1 - I1
    e_reg = inner(mu0, v0, p)
    e_data = inner(r, r, p) / p.sigma2
    return e_reg + e_data, e_reg, e_data


def energy(v0, I0, I1, p):
    tr = shoot(v0, p, I0)
    return energy_terms(v0, tr.J1, I1, p, tr.mu[0])[0]


# ---------------------------------------------------------------------------
# O6: backward (adjoint) Jacobi sweep (Section 2.2 reduced adjoint Jacobi field
# equations, in momentum form U^ = L U; reused by Section 3 for both sweeps)
# ---------------------------------------------------------------------------


def _adjoint_rhs(U, w, v, mu, p):
    """(ad*_v U^,  K(U^ + ad*_w mu) - ad_v w): the transpose of the tangent operator."""
    return ad_star(v, U, p), apply_K(U + ad_star(w, mu, p), p) - ad(v, w, p)


def backward_sweep(U_T, tr, p):
    """Integrate the adjoint Jacobi system from t = 1 (U^ = U_T, w = 0) back to t = 0.

    Each step is the transpose of the forward Heun step: the stage at the stored
    predictor (v*_n, mu*_n) is applied first, then the stage at (v_n, mu_n).
    Returns (U^_0, w_0).
    """
    dt = p.dt
    U = np.array(U_T, dtype=np.float64)
    w = np.zeros_like(U)
    for n in reversed(range(p.nt)):
        fU, fw = _adjoint_rhs(U, w, tr.v_star[n], tr.mu_star[n], p)
        Us, ws = U + dt * fU, w + dt * fw
        gU, gw = _adjoint_rhs(Us, ws, tr.v[n], tr.mu[n], p)
        U = 0.5 * U + 0.5 * (Us + dt * gU)
        w = 0.5 * w + 0.5 * (ws + dt * gw)
    return U, w


@dataclass
class Linearization:
    """Everything the gradient and the Hessian-vector product need at one v0."""

    v0: np.ndarray
    tr: Trajectory
    G: np.ndarray  # central-difference gradient of J_1
    E: float
    E_reg: float
    E_data: float
    residual: np.ndarray  # J_1 - I_1


def linearize(v0, I0, I1, p):
    """Shoot with trajectory store, then r = J_1 - I_1, E and G = grad_h J_1."""
    tr = shoot(v0, p, I0)
    E, er, ed = energy_terms(np.asarray(v0, dtype=np.float64), tr.J1, I1, p, tr.mu[0])
    return Linearization(np.array(v0, dtype=np.float64), tr, grad(tr.J1, p), E, er, ed, tr.J1 - I1)


def gradient(v0, I0, I1, p, lin=None):
    """V-gradient g = 2 v0 + w_0 with the final condition U^(1) = lambda_1 grad J_1,
    lambda_1 = -(2/sigma^2)(J_1 - I_1) (Section 3 gradient at t = 1; Section 2.3 lambda(1)).
    Returns (g, lin)."""
    if lin is None:
        lin = linearize(v0, I0, I1, p)
    lam = -(2.0 / p.sigma2) * lin.residual
    _, w0 = backward_sweep(lam[None] * lin.G, lin.tr, p)
    return 2.0 * lin.v0 + w0, lin


# ---------------------------------------------------------------------------
# O8/O9: tangent sweep and the Gauss-Newton Hessian-vector product (Section 3)
# ---------------------------------------------------------------------------


def _tangent_rhs(X, dmu, v, mu, p):
    """(K dmu + ad_v X,  -ad*_{K dmu} mu - ad*_v dmu): Jacobi field + incremental EPDiff."""
    dv = apply_K(dmu, p)
    return dv + ad(v, X, p), -ad_star(dv, mu, p) - ad_star(v, dmu, p)


def tangent(dv, tr, p, keep_history=False):
    """Forward tangent sweep from X_0 = 0, delta mu_0 = L dv along the stored geodesic.

    Same Heun stages as the shooting: (v_n, mu_n) then (v*_n, mu*_n).  Returns
    (X_nt, delta mu_nt) and, if requested, the list of delta mu_n for n = 0..nt.
    """
    dt = p.dt
    dmu = apply_L(np.asarray(dv, dtype=np.float64), p)
    X = np.zeros_like(dmu)
    hist = [dmu]
    for n in range(p.nt):
        aX, am = _tangent_rhs(X, dmu, tr.v[n], tr.mu[n], p)
        Xs, ms = X + dt * aX, dmu + dt * am
        bX, bm = _tangent_rhs(Xs, ms, tr.v_star[n], tr.mu_star[n], p)
        X = 0.5 * X + 0.5 * (Xs + dt * bX)
        dmu = 0.5 * dmu + 0.5 * (ms + dt * bm)
        if keep_history:
            hist.append(dmu)
    return (X, dmu, hist) if keep_history else (X, dmu)


def incremental_image(dv, lin, p):
    """delta m_1 = -grad J_1 . X_nt (R8)."""
    X, _ = tangent(dv, lin.tr, p)
    return -np.sum(lin.G * X, axis=0)


def hessvec(dv, lin, p):
    """Gauss-Newton Hessian-vector product in V: 2 dv + w_0 with
    U^(1) = delta lambda(1) grad J_1 = -(2/sigma^2) delta m_1 grad J_1 (A3)."""
    dm1 = incremental_image(dv, lin, p)
    U_T = (-(2.0 / p.sigma2) * dm1)[None] * lin.G
    _, w0 = backward_sweep(U_T, lin.tr, p)
    return 2.0 * np.asarray(dv, dtype=np.float64) + w0


# ---------------------------------------------------------------------------
# Full Newton Hessian-vector product (Section 3: the incremental adjoint Jacobi
# system with every term kept; A19)
# ---------------------------------------------------------------------------


def tangent_stages(dv, tr, p):
    """Tangent sweep that also returns, for each step n, the variation of the two
    trajectory points the Heun step visits: (delta mu_n, delta mu*_n).  Returns
    (X_nt, [(delta mu_n, delta mu*_n) for n < nt])."""
    dt = p.dt
    dmu = apply_L(np.asarray(dv, dtype=np.float64), p)
    X = np.zeros_like(dmu)
    stages = []
    for n in range(p.nt):
        aX, am = _tangent_rhs(X, dmu, tr.v[n], tr.mu[n], p)
        Xs, ms = X + dt * aX, dmu + dt * am
        stages.append((dmu, ms))
        bX, bm = _tangent_rhs(Xs, ms, tr.v_star[n], tr.mu_star[n], p)
        X = 0.5 * X + 0.5 * (Xs + dt * bX)
        dmu = 0.5 * dmu + 0.5 * (ms + dt * bm)
    return X, stages


def _adjoint_rhs_variation(U, w, dv, dmu, mu, p):
    """Change of the adjoint right-hand side when the trajectory point moves by
    (dv, dmu) = (K dmu, dmu) with the adjoint state (U^, w) held:
    (ad*_{dv} U^,  K(ad*_w dmu) - ad_{dv} w) - the ad^dagger_{dv} U, ad^dagger_w dv
    and -ad_{dv} w terms of the incremental adjoint Jacobi system (Section 3)."""
    return ad_star(dv, U, p), apply_K(ad_star(w, dmu, p), p) - ad(dv, w, p)


def newton_sweep(U_T, dU_T, stages, tr, p):
    """Linearisation of backward_sweep(U_T, trajectory) when the trajectory varies by
    `stages` (from tangent_stages) and the final condition by dU_T.  Carries the
    first-order adjoint (U^, w) and its variation (dU^, dw) through the same
    transposed Heun steps.  Returns dw_0."""
    dt = p.dt
    U = np.array(U_T, dtype=np.float64)
    w = np.zeros_like(U)
    dU = np.array(dU_T, dtype=np.float64)
    dw = np.zeros_like(dU)
    for n in reversed(range(p.nt)):
        dmu_n, dmus_n = stages[n]
        # stage at the predictor point (v*_n, mu*_n)
        fU, fw = _adjoint_rhs(U, w, tr.v_star[n], tr.mu_star[n], p)
        lU, lw = _adjoint_rhs(dU, dw, tr.v_star[n], tr.mu_star[n], p)
        eU, ew = _adjoint_rhs_variation(U, w, apply_K(dmus_n, p), dmus_n, tr.mu_star[n], p)
        Us, ws = U + dt * fU, w + dt * fw
        dUs, dws = dU + dt * (lU + eU), dw + dt * (lw + ew)
        # stage at (v_n, mu_n)
        gU, gw = _adjoint_rhs(Us, ws, tr.v[n], tr.mu[n], p)
        kU, kw = _adjoint_rhs(dUs, dws, tr.v[n], tr.mu[n], p)
        e2U, e2w = _adjoint_rhs_variation(Us, ws, apply_K(dmu_n, p), dmu_n, tr.mu[n], p)
        U, w = 0.5 * U + 0.5 * (Us + dt * gU), 0.5 * w + 0.5 * (ws + dt * gw)
        dU = 0.5 * dU + 0.5 * (dUs + dt * (kU + e2U))
        dw = 0.5 * dw + 0.5 * (dws + dt * (kw + e2w))
    return dw


def hessvec_newton(dv, lin, p):
    """Newton Hessian-vector product in V (Section 3 with nothing dropped, A19):
    2 dv + dw_0, where the final condition keeps lambda_1 grad(delta m_1),
    dU^(1) = -(2/sigma^2) delta m_1 grad J_1 + lambda_1 grad_h(delta m_1), and the
    sweep keeps the terms of the first-order adjoint (U^, w) of the gradient."""
    X, stages = tangent_stages(dv, lin.tr, p)
    dm1 = -np.sum(lin.G * X, axis=0)
    lam = -(2.0 / p.sigma2) * lin.residual
    U_T = lam[None] * lin.G
    dU_T = (-(2.0 / p.sigma2) * dm1)[None] * lin.G + lam[None] * grad(dm1, p)
    return 2.0 * np.asarray(dv, dtype=np.float64) + newton_sweep(U_T, dU_T, stages, lin.tr, p)


def vjp_J1(gbar, lin, p):
    """Plain-array gradient of l(J_1) w.r.t. v0 given gbar = dl/dJ_1 (entrywise):
    L w_0 with U^(1) = -gbar grad J_1 (the h^3 factors of the pairing cancel)."""
    U_T = -np.asarray(gbar, dtype=np.float64)[None] * lin.G
    _, w0 = backward_sweep(U_T, lin.tr, p)
    return apply_L(w0, p)


# ---------------------------------------------------------------------------
# O10/O11: CG in V and the inexact Gauss-Newton loop (Section 2.3 reduced KKT
# system with preconditioner K; Section 3 update and "CG on V")
# ---------------------------------------------------------------------------


def cg_v(hess, g, p, eta, maxit):
    """Solve H x = -g by CG in the V inner product, stop at ||r||_V <= eta ||g||_V.

    CG in V is PCG in L2 with preconditioner K.  On non-positive curvature it stops
    with the current iterate, or with the steepest-descent direction -g if that
    happens on the first direction (A19).  Returns (x, iterations).
    """
    x = np.zeros_like(g)
    r = -np.asarray(g, dtype=np.float64)
    d = r.copy()
    rr = inner_V(r, r, p)
    tol = eta * math.sqrt(inner_V(g, g, p))
    it = 0
    for it in range(1, maxit + 1):
        Hd = hess(d)
        dHd = inner_V(d, Hd, p)
        if dHd <= 0.0:  # negative curvature (Newton Hessian far from a minimum)
            if it == 1:
                x = d.copy()  # steepest descent -g
            it -= 1
            break
        a = rr / dHd
        x = x + a * d
        r = r - a * Hd
        rr_new = inner_V(r, r, p)
        if math.sqrt(rr_new) <= tol:
            break
        d = r + (rr_new / rr) * d
        rr = rr_new
    return x, it


def pcg_l2(hess, g, p, eta, maxit, precond):
    """Preconditioned CG in the L2 product for H x = -g (H symmetric in L2) with
    preconditioner `precond`; stops at ||r||_L2 <= eta ||g||_L2 or on
    non-positive curvature.  Returns (x, iterations)."""
    g = np.asarray(g, dtype=np.float64)
    x = np.zeros_like(g)
    r = -g
    z = precond(r)
    d = z.copy()
    rz = inner(r, z, p)
    tol = eta * math.sqrt(inner(g, g, p))
    it = 0
    for it in range(1, maxit + 1):
        q = hess(d)
        dq = inner(d, q, p)
        if dq <= 0.0:
            it -= 1
            break
        a = rz / dq
        x = x + a * d
        r = r - a * q
        if math.sqrt(inner(r, r, p)) <= tol:
            break
        z = precond(r)
        rz_new = inner(r, z, p)
        d = z + (rz_new / rz) * d
        rz = rz_new
    return x, it


def gradient_l2(v0, I0, I1, p):
    """L2-gradient of E (A17): L g_V, so that dE[d] = <g_L2, d>."""
    g, lin = gradient(v0, I0, I1, p)
    return apply_L(g, p), lin


def hessvec_l2(dv, lin, p):
    """Gauss-Newton Hessian in the L2 product (A17): L H_V dv."""
    return apply_L(hessvec(dv, lin, p), p)


@dataclass
class IterLog:
    E: float
    E_reg: float
    E_data: float
    mse_rel: float
    g_norm: float  # norm of the gradient in the solve's space (V, or L2 for "GN, L2")
    g_inf_rel: float
    cg_iters: int
    eta: float
    tau: float


def gn_solve(I0, I1, p, gn_iters=10, cg_iters=20, c1=1e-4, max_halvings=10, gtol=1e-3, v0=None, space="V",
             hessian="gn"):
    """Inexact Gauss-Newton-Krylov (Section 3): per iteration linearize, gradient,
    a Krylov solve of H p = -g with forcing eta = min(0.5, sqrt(||g|| / ||g_0||)),
    then Armijo backtracking v0 <- v0 + tau p (A1).  space="V": CG in V (the primary
    method); space="L2": gradient and Hessian in L2 and PCG with preconditioner K
    (A17).  hessian="newton" (with space="V") uses the full Newton Hessian (A19).
    Returns (v0, log, final Linearization)."""
    if space not in ("V", "L2"):
        raise ValueError("space must be 'V' or 'L2'")
    if hessian not in ("gn", "newton") or (hessian == "newton" and space != "V"):
        raise ValueError("hessian must be 'gn', or 'newton' with space 'V'")
    hv = hessvec_newton if hessian == "newton" else hessvec
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    v = np.zeros((3,) + tuple(p.n)) if v0 is None else np.array(v0, dtype=np.float64)
    base = inner(I0 - I1, I0 - I1, p)
    log = []
    g0 = ginf0 = None
    lin = None
    for _ in range(gn_iters):
        if space == "V":
            g, lin = gradient(v, I0, I1, p)
            gn = math.sqrt(inner_V(g, g, p))
        else:
            g, lin = gradient_l2(v, I0, I1, p)
            gn = math.sqrt(inner(g, g, p))
        ginf = float(np.max(np.abs(g)))
        if g0 is None:
            g0, ginf0 = gn, ginf
        if g0 == 0.0 or gn / g0 <= gtol:
            break
        eta = min(0.5, math.sqrt(gn / g0))
        if space == "V":
            step, its = cg_v(lambda d: hv(d, lin, p), g, p, eta, cg_iters)
            gp = inner_V(g, step, p)
        else:
            step, its = pcg_l2(lambda d: hessvec_l2(d, lin, p), g, p, eta, cg_iters, lambda r: apply_K(r, p))
            gp = inner(g, step, p)
        tau, accepted = 1.0, False
        for _ in range(max_halvings + 1):
            if energy(v + tau * step, I0, I1, p) <= lin.E + c1 * tau * gp:
                accepted = True
                break
            tau *= 0.5
        log.append(IterLog(lin.E, lin.E_reg, lin.E_data, 100.0 * inner(lin.residual, lin.residual, p) / base,
                           gn, ginf / ginf0, its, eta, tau if accepted else 0.0))
        if not accepted:
            break
        v = v + tau * step
    lin = linearize(v, I0, I1, p)
    return v, log, lin


def gd_solve(I0, I1, p, iters=50, c1=1e-4, max_halvings=10, gtol=1e-3, tau0=0.5, v0=None):
    """Gradient descent in V (Section 2.2, the EPDiff-LDDMM baseline): per iteration
    the V-gradient from the adjoint Jacobi sweep, then v0 <- v0 - tau g with tau
    from tau0 by Armijo halving (A18).  Same stop rules and log as gn_solve (no CG:
    cg_iters = 0, eta = 0).  Returns (v0, log, final Linearization)."""
    I0 = np.asarray(I0, dtype=np.float64)
    I1 = np.asarray(I1, dtype=np.float64)
    v = np.zeros((3,) + tuple(p.n)) if v0 is None else np.array(v0, dtype=np.float64)
    base = inner(I0 - I1, I0 - I1, p)
    log = []
    g0 = ginf0 = None
    for _ in range(iters):
        g, lin = gradient(v, I0, I1, p)
        gg = inner_V(g, g, p)
        gn = math.sqrt(gg)
        ginf = float(np.max(np.abs(g)))
        if g0 is None:
            g0, ginf0 = gn, ginf
        if g0 == 0.0 or gn / g0 <= gtol:
            break
        tau, accepted = tau0, False
        for _ in range(max_halvings + 1):
            if energy(v - tau * g, I0, I1, p) <= lin.E - c1 * tau * gg:
                accepted = True
                break
            tau *= 0.5
        log.append(IterLog(lin.E, lin.E_reg, lin.E_data, 100.0 * inner(lin.residual, lin.residual, p) / base,
                           gn, ginf / ginf0, 0, 0.0, tau if accepted else 0.0))
        if not accepted:
            break
        v = v - tau * g
    lin = linearize(v, I0, I1, p)
    return v, log, lin


# ---------------------------------------------------------------------------
# O12: reporting metrics (Section 4)
# ---------------------------------------------------------------------------


def mse_rel(J1, I0, I1, p):
    """||J_1 - I_1||^2 / ||I_0 - I_1||^2, in percent."""
    return 100.0 * inner(J1 - I1, J1 - I1, p) / inner(I0 - I1, I0 - I1, p)


def jacobian_det(u, p):
    """det(I + D_h u) of the inverse map id + u (central differences)."""
    J = np.empty((3, 3) + u.shape[1:])
    for c in range(3):
        for d in range(3):
            J[c, d] = ddx(u[c], d, p) + (1.0 if c == d else 0.0)
    return (
        J[0, 0] * (J[1, 1] * J[2, 2] - J[1, 2] * J[2, 1])
        - J[0, 1] * (J[1, 0] * J[2, 2] - J[1, 2] * J[2, 0])
        + J[0, 2] * (J[1, 0] * J[2, 1] - J[1, 1] * J[2, 0])
    )


# ---------------------------------------------------------------------------
# Cross-check only: the literal semi-Lagrangian discretisation of the paper's
# incremental state equation (Section 3), d(dm)/dt + grad(dm).v + grad(m).dv = 0.
# ---------------------------------------------------------------------------


def incremental_image_literal(dv, lin, I0, p):
    """delta m_1 by semi-Lagrangian transport of delta m with a trapezoidal source
    -grad(J_t) . delta v_t along the same characteristics as the state equation."""
    dt = p.dt
    _, _, hist = tangent(dv, lin.tr, p, keep_history=True)
    x = grid_coords(p)
    u = np.zeros_like(x)
    dm = np.zeros(p.n)
    I0 = np.asarray(I0, dtype=np.float64)
    J = interp(I0, x, p)
    src = -np.sum(grad(J, p) * apply_K(hist[0], p), axis=0)
    for n in range(p.nt):
        vo, vn = lin.tr.v[n], lin.tr.v[n + 1]
        X = x - 0.5 * dt * (vn + interp(vo, x - dt * vn, p))
        u = interp(u, X, p) + (X - x)
        J = interp(I0, x + u, p)
        src_new = -np.sum(grad(J, p) * apply_K(hist[n + 1], p), axis=0)
        dm = interp(dm, X, p) + 0.5 * dt * (interp(src, X, p) + src_new)
        src = src_new
    return dm
