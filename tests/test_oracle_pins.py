"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check compares the oracle with something other than itself: closed forms
(single Fourier modes, the v0 = 0 special case), exact identities of the
discretisation (adjointness, antisymmetry, symmetry of the Gauss-Newton
Hessian), library routines (scipy's periodic linear interpolation, numpy's
roll, a dense eigen-solve) and finite differences.  ``test_planted_mistakes``
checks that plausible implementation slips make at least one pin fail.
"""

import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle as O
from synth import phantom, random_field, random_velocity


def P(n=(8, 8, 8), alpha=0.01, s=2, nt=10, sigma2=1.0):
    return O.Params(tuple(n), alpha, s, nt, sigma2)


def smooth_case(n, nt=10, alpha=0.05, amp=0.1, seed=0):
    """Analytic smooth images, velocity and direction sampled on an n-grid."""
    p = P(n, alpha=alpha, nt=nt)
    x = O.grid_coords(p)
    I0 = 0.5 + 0.3 * np.sin(x[0]) * np.cos(2 * x[1]) + 0.2 * np.cos(x[2] + x[0])
    I1 = 0.5 + 0.3 * np.sin(x[0] + 0.2) * np.cos(2 * x[1] - 0.1) + 0.2 * np.cos(x[2] + x[0] + 0.15)
    v0 = amp * np.stack([np.sin(x[1]), np.cos(x[2] + x[0]), np.sin(x[0] - x[1])])
    d = np.stack([np.cos(x[2]), np.sin(x[0] + 2 * x[1]), np.cos(x[1])])
    return p, I0, I1, v0, d


def phantom_case(n=(12, 10, 14), nt=6, seed=0, amp=1.5):
    p = P(n, alpha=0.01, nt=nt)
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000 + seed)
    I1 = phantom(n, 4, (1.5, 3.0), False, 1100 + seed)
    v0 = random_velocity(n, 2000 + seed, amp, kc=2.0)
    return p, I0, I1, v0


# --------------------------------------------------------------------------- P-1
@pytest.mark.parametrize("n", [(8, 8, 8), (6, 10, 12)])
def test_L_K_single_modes(n):
    p = P(n, alpha=0.03, s=2)
    x = O.grid_coords(p)
    for k in [(0, 0, 0), (1, 0, 0), (0, 2, 0), (0, 0, 3), (1, -2, 2), (n[0] // 2, 1, n[2] // 2)]:
        f = np.cos(k[0] * x[0] + k[1] * x[1] + k[2] * x[2] + 0.3)
        lam = (1.0 + p.alpha * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2)) ** p.s
        np.testing.assert_allclose(O.apply_L(f, p), lam * f, rtol=0, atol=1e-12 * lam)
        np.testing.assert_allclose(O.apply_K(f, p), f / lam, rtol=0, atol=1e-13)


def test_L_K_inverse_random_and_power():
    p = P((8, 6, 10), alpha=0.02, s=3)
    f = random_field(p.n, 1, kc=3.0)
    np.testing.assert_allclose(O.apply_K(O.apply_L(f, p), p), f, atol=1e-12)
    # s = 1 squared equals s = 2 (integer power of the symbol)
    p1 = P(p.n, alpha=0.02, s=1)
    p2 = P(p.n, alpha=0.02, s=2)
    np.testing.assert_allclose(O.apply_L(O.apply_L(f, p1), p1), O.apply_L(f, p2), atol=1e-11)


# --------------------------------------------------------------------------- P-2
def test_central_difference_modes():
    p = P((8, 12, 10))
    x = O.grid_coords(p)
    k = (2, 3, 1)
    phase = k[0] * x[0] + k[1] * x[1] + k[2] * x[2]
    f = np.cos(phase)
    for d in range(3):
        expect = -np.sin(k[d] * p.h[d]) / p.h[d] * np.sin(phase)
        np.testing.assert_allclose(O.ddx(f, d, p), expect, atol=1e-13)
    # one-sided index check: delta_0 f[i] uses f[i+1] - f[i-1] in the first array axis
    g = np.zeros(p.n)
    g[3, 4, 5] = 1.0
    dg = O.ddx(g, 0, p)
    assert dg[2, 4, 5] == pytest.approx(1.0 / (2 * p.h[0]))
    assert dg[4, 4, 5] == pytest.approx(-1.0 / (2 * p.h[0]))


# --------------------------------------------------------------------------- P-3
def test_ad_identities():
    p = P((8, 6, 10))
    v, w, mu = random_field(p.n, 1, 2.0), random_field(p.n, 2, 2.0), random_field(p.n, 3, 2.0)
    a = O.inner(O.ad_star(v, mu, p), w, p)
    b = O.inner(mu, O.ad(v, w, p), p)
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b) + 1e-30) * 10
    np.testing.assert_allclose(O.ad(v, v, p), 0.0, atol=1e-12)
    np.testing.assert_allclose(O.ad(v, w, p), -O.ad(w, v, p), atol=1e-12)


def test_ad_constant_velocity_closed_form():
    p = P((8, 6, 10))
    c = np.array([0.7, -1.3, 0.4])
    vc = c[:, None, None, None] * np.ones((3,) + p.n)
    w = random_field(p.n, 4, 2.0)
    # ad_c w = -(Dw) c = -sum_d c_d delta_d w ; ad*_c mu = sum_d c_d delta_d mu
    dir_deriv = sum(c[d] * np.stack([O.ddx(w[k], d, p) for k in range(3)]) for d in range(3))
    np.testing.assert_allclose(O.ad(vc, w, p), -dir_deriv, atol=1e-12)
    np.testing.assert_allclose(O.ad_star(vc, w, p), dir_deriv, atol=1e-12)
    # ad*_w c for constant momentum c: (Dw)^T c + c div w
    div = sum(O.ddx(w[d], d, p) for d in range(3))
    expect = np.stack([sum(O.ddx(w[d], k, p) * c[d] for d in range(3)) + c[k] * div for k in range(3)])
    np.testing.assert_allclose(O.ad_star(w, vc, p), expect, atol=1e-12)


def test_ad_star_matches_printed_expanded_form_in_the_continuum():
    """Conservative ad* equals (Dv)^T mu + D(mu) v + mu div v up to O(h^2) (product rule)."""
    errs = []
    for N in (16, 32):
        p = P((N, N, N))
        x = O.grid_coords(p)
        v = np.stack([np.sin(x[0] + x[1]), np.cos(x[1] + x[2]), np.sin(x[2] + x[0])])
        mu = np.stack([np.cos(x[0] + 2 * x[2]), np.sin(x[1] + x[0]), np.cos(x[2] + x[1])])
        div = sum(O.ddx(v[d], d, p) for d in range(3))
        expanded = np.stack([
            sum(O.ddx(v[d], c, p) * mu[d] + O.ddx(mu[c], d, p) * v[d] for d in range(3)) + mu[c] * div
            for c in range(3)
        ])
        errs.append(np.abs(O.ad_star(v, mu, p) - expanded).max())
    assert errs[0] < 0.5 and errs[1] < errs[0] / 3.5, errs


# --------------------------------------------------------------------------- P-4
def test_interp_matches_scipy_grid_wrap():
    p = P((8, 6, 10))
    rng = np.random.default_rng(5)
    f = rng.standard_normal(p.n)
    y = rng.uniform(-7.0, 14.0, size=(3, 5, 4, 3))
    got = O.interp(f, y, p)
    coords = np.stack([y[d] / p.h[d] for d in range(3)]).reshape(3, -1)
    ref = ndi.map_coordinates(f, coords, order=1, mode="grid-wrap").reshape(y.shape[1:])
    np.testing.assert_allclose(got, ref, atol=1e-13)


def test_interp_integer_shift_is_roll():
    p = P((8, 6, 10))
    f = np.random.default_rng(6).standard_normal((3,) + p.n)
    x = O.grid_coords(p)
    shift = np.array([2, -1, 3])
    y = x + (shift * np.array(p.h))[:, None, None, None]
    np.testing.assert_allclose(O.interp(f, y, p), np.roll(f, tuple(-shift), axis=(1, 2, 3)), atol=1e-14)


# --------------------------------------------------------------------------- P-5
def test_shoot_zero_velocity_is_identity():
    p, I0, _, _ = phantom_case()
    tr = O.shoot(np.zeros((3,) + p.n), p, I0)
    assert np.all(tr.v[-1] == 0.0) and np.all(tr.u == 0.0)
    np.testing.assert_array_equal(tr.J1, I0)


def test_shoot_constant_velocity_translates():
    p, I0, _, _ = phantom_case(n=(8, 10, 12), nt=4)
    shift = np.array([1, -2, 3])
    c = shift * np.array(p.h)
    v0 = c[:, None, None, None] * np.ones((3,) + p.n)
    tr = O.shoot(v0, p, I0)
    np.testing.assert_allclose(tr.v[-1], v0, atol=1e-13)
    np.testing.assert_allclose(tr.u, -v0, atol=1e-13)
    np.testing.assert_allclose(tr.J1, np.roll(I0, tuple(shift), axis=(0, 1, 2)), atol=1e-12)


def test_sl_stationary_shear_exact():
    p = P((8, 6, 10), nt=5)
    x = O.grid_coords(p)
    v = np.stack([np.zeros(p.n), np.zeros(p.n), 0.8 * np.sin(x[0])])
    u = O.sl_transport([v] * (p.nt + 1), p)
    np.testing.assert_allclose(u, -v, atol=1e-14)


# --------------------------------------------------------------------------- P-6
def test_dot_product_tangent_vs_backward():
    p, I0, I1, v0 = phantom_case()
    lin = O.linearize(v0, I0, I1, p)
    UT = random_field(p.n, 11, 2.0)
    dv = random_field(p.n, 12, 2.0)
    X, _ = O.tangent(dv, lin.tr, p)
    _, w0 = O.backward_sweep(UT, lin.tr, p)
    a = O.inner(UT, X, p)
    b = O.inner_V(w0, dv, p)
    assert abs(a - b) <= 1e-12 * abs(a)


# --------------------------------------------------------------------------- P-7 / P-8
def test_gradient_at_zero_closed_form():
    p, I0, I1, _ = phantom_case()
    g, _ = O.gradient(np.zeros((3,) + p.n), I0, I1, p)
    gI0 = O.grad(I0, p)
    expect = -(2.0 / p.sigma2) * O.apply_K((I0 - I1)[None] * gI0, p)
    np.testing.assert_allclose(g, expect, atol=1e-13 * np.abs(expect).max() + 1e-15)


def test_hessvec_at_zero_closed_form():
    p, I0, I1, _ = phantom_case()
    p.sigma2 = 0.5
    lin = O.linearize(np.zeros((3,) + p.n), I0, I1, p)
    dv = random_field(p.n, 13, 2.0)
    gI0 = O.grad(I0, p)
    expect = 2 * dv + (2.0 / p.sigma2) * O.apply_K(np.sum(gI0 * dv, axis=0)[None] * gI0, p)
    np.testing.assert_allclose(O.hessvec(dv, lin, p), expect, atol=1e-12 * np.abs(expect).max())


# --------------------------------------------------------------------------- P-9
def _dense_hessian(lin, p):
    m = 3 * int(np.prod(p.n))
    H = np.empty((m, m))
    e = np.zeros(m)
    for j in range(m):
        e[:] = 0.0
        e[j] = 1.0
        H[:, j] = O.hessvec(e.reshape((3,) + p.n), lin, p).ravel()
    return H


def _dense_L(p):
    m = 3 * int(np.prod(p.n))
    Lm = np.empty((m, m))
    e = np.zeros(m)
    for j in range(m):
        e[:] = 0.0
        e[j] = 1.0
        Lm[:, j] = O.apply_L(e.reshape((3,) + p.n), p).ravel()
    return Lm


def test_brute_force_hessian_and_cg():
    n = (4, 4, 6)
    p = P(n, alpha=0.05, nt=4, sigma2=0.002)
    I0 = phantom(n, 3, (1.0, 2.0), False, 1000)
    I1 = phantom(n, 3, (1.0, 2.0), False, 1001)
    v0 = random_velocity(n, 2000, 0.5, kc=1.5)
    lin = O.linearize(v0, I0, I1, p)
    H = _dense_hessian(lin, p)
    Lm = _dense_L(p)
    LH = Lm @ H
    assert np.abs(LH - LH.T).max() <= 1e-10 * np.abs(LH).max()
    # generalized eigenvalues of the pencil (L H, L): the V-spectrum of H is >= 2
    Lc = np.linalg.cholesky(0.5 * (Lm + Lm.T))
    Li = np.linalg.inv(Lc)
    S = Li @ (0.5 * (LH + LH.T)) @ Li.T
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= 2.0 * (1 - 1e-10)
    assert ev.max() > 2.5  # the data term is not negligible in this case
    # CG in V converges to the dense solution of H x = -g
    g, _ = O.gradient(v0, I0, I1, p, lin)
    x_dense = np.linalg.solve(H, -g.ravel())
    x_cg, its = O.cg_v(lambda d: O.hessvec(d, lin, p), g, p, 1e-12, 400)
    np.testing.assert_allclose(x_cg.ravel(), x_dense, atol=1e-8 * np.abs(x_dense).max())


def test_first_gn_step_from_zero_matches_dense_solve():
    n = (4, 6, 4)
    p = P(n, alpha=0.05, nt=3, sigma2=0.3)
    I0 = phantom(n, 3, (1.0, 2.0), False, 1002)
    I1 = phantom(n, 3, (1.0, 2.0), False, 1003)
    zero = np.zeros((3,) + n)
    lin = O.linearize(zero, I0, I1, p)
    H = _dense_hessian(lin, p)
    # closed form at v0 = 0: H = 2 I + (2/sigma2) K [(grad I0 . dv) grad I0], g from P-7
    gI0 = O.grad(I0, p)
    g = -(2.0 / p.sigma2) * O.apply_K((I0 - I1)[None] * gI0, p)
    step = np.linalg.solve(H, -g.ravel()).reshape(g.shape)
    x_cg, _ = O.cg_v(lambda d: O.hessvec(d, lin, p), g, p, 1e-13, 400)
    np.testing.assert_allclose(x_cg, step, atol=1e-9 * np.abs(step).max())


# --------------------------------------------------------------------------- P-10 / P-11
def test_hessian_symmetric_and_bounded_below():
    p, I0, I1, v0 = phantom_case(n=(10, 12, 8))
    p.sigma2 = 0.1
    lin = O.linearize(v0, I0, I1, p)
    a, b = random_field(p.n, 21, 2.0), random_field(p.n, 22, 2.0)
    Ha, Hb = O.hessvec(a, lin, p), O.hessvec(b, lin, p)
    x1, x2 = O.inner_V(a, Hb, p), O.inner_V(Ha, b, p)
    assert abs(x1 - x2) <= 1e-12 * max(abs(x1), abs(x2))
    for f, Hf in ((a, Ha), (b, Hb)):
        assert O.inner_V(f, Hf, p) >= 2.0 * O.inner_V(f, f, p) * (1 - 1e-12)


# --------------------------------------------------------------------------- P-12
def test_tangent_momentum_is_linearised_shooting():
    p, I0, I1, v0 = phantom_case(n=(10, 8, 12), nt=5, amp=2.0)
    d = random_field(p.n, 31, 2.0)
    lin = O.linearize(v0, I0, I1, p)
    _, dmu = O.tangent(d, lin.tr, p)
    eps = 1e-4 * np.abs(v0).max()
    vp = O.shoot(v0 + eps * d, p).v[-1]
    vm = O.shoot(v0 - eps * d, p).v[-1]
    fd = (vp - vm) / (2 * eps)
    an = O.apply_K(dmu, p)
    assert np.linalg.norm(an - fd) <= 1e-7 * np.linalg.norm(fd)


# --------------------------------------------------------------------------- P-13
def test_time_convergence_orders():
    """Heun is second order in the state; on the quadratic invariant <mu, v> its
    dt^2 error term cancels, so the drift falls as dt^3 (ratio ~8 per halving)."""
    n = (16, 16, 16)
    drifts, v1 = [], []
    for nt in (10, 20, 40, 80):
        p = P(n, alpha=0.01, nt=nt)
        v0 = random_velocity(n, 2001, 3.0, kc=2.0)
        tr = O.shoot(v0, p)
        drifts.append(abs(tr.drift[-1]))
        v1.append(tr.v[-1])
    r1, r2 = drifts[0] / drifts[1], drifts[1] / drifts[2]
    assert 6.5 <= r1 <= 10.0 and 6.5 <= r2 <= 10.0, drifts
    e = [np.abs(v1[k] - v1[k + 1]).max() for k in range(3)]
    assert 3.5 <= e[0] / e[1] <= 5.5 and 3.5 <= e[1] / e[2] <= 5.5, e


# --------------------------------------------------------------------------- P-14
def test_gradient_vs_finite_differences_converges():
    gaps = []
    for N in (16, 32):
        p, I0, I1, v0, _ = smooth_case((N, N, N))
        g, lin = O.gradient(v0, I0, I1, p)
        # data-term part of the gradient as direction, so the check is not the quadratic E_reg
        d = g - 2 * v0
        d = d / math.sqrt(O.inner_V(d, d, p))
        eps = 1e-4
        fd = (O.energy(v0 + eps * d, I0, I1, p) - O.energy(v0 - eps * d, I0, I1, p)) / (2 * eps)
        an = O.inner_V(g, d, p)
        gaps.append(abs(fd - an) / abs(fd))
    assert gaps[0] <= 5e-2 and gaps[1] <= gaps[0] / 1.7, gaps


def test_regularisation_gradient_exact():
    p, I0, I1, v0 = phantom_case()
    d = random_field(p.n, 41, 2.0)
    eps = 1e-3
    ep = O.energy_terms(v0 + eps * d, I0, I1, p)[1]
    em = O.energy_terms(v0 - eps * d, I0, I1, p)[1]
    assert (ep - em) / (2 * eps) == pytest.approx(2 * O.inner_V(v0, d, p), rel=1e-10)


# --------------------------------------------------------------------------- SL in time
def _sl_flow(y, t):
    """Velocity along one axis varying in space and time (periodic in y)."""
    return 0.35 * (1.0 + 1.5 * t) * np.sin(y) + 0.25 * t * t * np.cos(2.0 * y) + 0.1


def _sl_line_case(nt, axis=2, N=4096):
    """SL transport (R7) of a flow along `axis` that depends on that coordinate and
    on time: returns the grid points of that axis and the transported displacement
    u_1 along it.  Along the axis the grid is fine, so interpolation errors stay
    far below the time-stepping errors examined."""
    n = [4, 4, 4]
    n[axis] = N
    p = P(tuple(n), nt=nt)
    x = O.grid_coords(p)
    vs = []
    for k in range(nt + 1):
        v = np.zeros((3,) + tuple(n))
        v[axis] = _sl_flow(x[axis], k / nt)
        vs.append(v)
    u = O.sl_transport(vs, p)
    idx = [0, 0, 0]
    idx[axis] = slice(None)
    others = np.delete(u, axis, axis=0)
    return np.arange(N) * p.h[axis], u[axis][tuple(idx)], float(np.abs(others).max())


def _characteristic_foot(y, steps=400):
    """Exact foot point at t = 0 of the characteristic through y at t = 1,
    dy/dt = flow(y, t), by classical RK4 with many steps."""
    h = 1.0 / steps
    t = 1.0
    for _ in range(steps):
        k1 = _sl_flow(y, t)
        k2 = _sl_flow(y - 0.5 * h * k1, t - 0.5 * h)
        k3 = _sl_flow(y - 0.5 * h * k2, t - 0.5 * h)
        k4 = _sl_flow(y - h * k3, t - h)
        y = y - h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
        t -= h
    return y


def _heun_foot(y, nt):
    """Heun's method (explicit trapezoid: Euler predictor, average of the two slopes)
    applied to the characteristic ODE backward in time from t = 1 to 0 in nt steps."""
    dt = 1.0 / nt
    for k in range(nt, 0, -1):
        s1 = _sl_flow(y, k * dt)
        s2 = _sl_flow(y - dt * s1, (k - 1) * dt)
        y = y - 0.5 * dt * (s1 + s2)
    return y


@pytest.mark.parametrize("axis", [2, 0])
def test_sl_backtrace_is_heun_on_the_characteristics(axis):
    """State equation (Section 2.3) by R7: with a velocity varying in space and time
    the transported displacement equals Heun's method on the backward
    characteristics (textbook form, exact velocities) up to interpolation error,
    and converges to the exact characteristics at second order in dt."""
    y = None
    errs = []
    for nt in (8, 16, 32):
        y, u1, off = _sl_line_case(nt, axis)
        assert off == 0.0
        heun = _heun_foot(y.copy(), nt) - y
        assert np.abs(u1 - heun).max() <= 2e-5, (nt, np.abs(u1 - heun).max())
        errs.append(np.abs(u1 - (_characteristic_foot(y.copy()) - y)).max())
    r = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(3.5 <= q <= 4.5 for q in r), (errs, r)


# --------------------------------------------------------------------------- P-16
def test_transported_momentum_identity():
    """EPDiff (Section 2.2) transports the momentum as a one-form density along the
    flow whose inverse map the state equation (Section 2.3) carries:
    mu_1 = det(D psi) (D psi)^T mu_0 o psi with psi = id + u_1.  Shooting (R6) and
    SL transport (R7) are discretised separately, so the identity holds to
    discretisation error, which shrinks as the same smooth case is refined."""
    gaps = []
    for N in (16, 32):
        p, _, _, v0, _ = smooth_case((N, N, N), nt=16, amp=0.3)
        x = O.grid_coords(p)
        tr = O.shoot(v0, p, np.zeros(p.n))
        u = tr.u
        Dpsi = np.empty((3, 3) + p.n)
        for c in range(3):
            for d in range(3):
                Dpsi[c, d] = O.ddx(u[c], d, p) + (1.0 if c == d else 0.0)
        m0 = O.interp(tr.mu[0], x + u, p)
        rhs = O.jacobian_det(u, p)[None] * np.einsum("cd...,c...->d...", Dpsi, m0)
        gaps.append(np.linalg.norm(rhs - tr.mu[-1]) / np.linalg.norm(tr.mu[-1]))
        # the identity carries content: mu changes along the geodesic by far more
        assert np.linalg.norm(tr.mu[0] - tr.mu[-1]) >= 5 * gaps[-1] * np.linalg.norm(tr.mu[-1])
    assert gaps[0] <= 0.05 and gaps[1] <= gaps[0] / 2.0, gaps


# --------------------------------------------------------------------------- VJP
def test_vjp_matches_finite_differences_of_the_warped_image():
    """The autograd backward (adjoint Jacobi sweep as a vector-Jacobian product,
    Section 2.2) against central FD of the plain sum l(J_1) = sum gbar J_1 through
    the forward shooting and SL transport: optimise-then-discretise, so the gap is
    discretisation-level and shrinks when the same smooth case is refined."""
    gaps = []
    for N in (16, 32):
        p, I0, I1, v0, d = smooth_case((N, N, N), nt=10, amp=0.2)
        x = O.grid_coords(p)
        lin = O.linearize(v0, I0, I1, p)
        gbar = np.sin(x[0] + x[1]) * np.cos(x[2]) + 0.3
        g = O.vjp_J1(gbar, lin, p)
        d = d / np.sqrt(np.sum(d * d))
        eps = 1e-4
        fd = (np.sum(gbar * O.shoot(v0 + eps * d, p, I0).J1) - np.sum(gbar * O.shoot(v0 - eps * d, p, I0).J1)) / (2 * eps)
        gaps.append(abs(fd - np.sum(g * d)) / abs(fd))
    assert gaps[0] <= 5e-2 and gaps[1] <= gaps[0] / 2.0, gaps


# --------------------------------------------------------------------------- P-15
def test_jacobi_incremental_image_matches_literal_transport():
    errs = []
    for N in (24, 48):
        p, I0, I1, v0, d = smooth_case((N, N, N), nt=8, amp=0.2)
        lin = O.linearize(v0, I0, I1, p)
        a = O.incremental_image(d, lin, p)
        b = O.incremental_image_literal(d, lin, I0, p)
        errs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    assert errs[0] < 0.1 and errs[1] < errs[0] / 1.7, errs


# --------------------------------------------------------------------------- metrics
def test_jacobian_det_closed_form_and_mse():
    p = P((8, 6, 10))
    x = O.grid_coords(p)
    a = 0.3
    u = np.stack([a * np.sin(x[0]), np.zeros(p.n), np.zeros(p.n)])
    np.testing.assert_allclose(O.jacobian_det(u, p), 1 + a * np.cos(x[0]) * np.sin(p.h[0]) / p.h[0], atol=1e-14)
    I0 = np.cos(x[1])
    I1 = np.zeros(p.n)
    assert O.mse_rel(I0, I0, I1, p) == pytest.approx(100.0)
    assert O.mse_rel(I1, I0, I1, p) == 0.0


def test_gn_solve_decreases_energy():
    p, I0, _, _ = phantom_case(n=(12, 12, 12), nt=5)
    vt = random_velocity(p.n, 2100, 1.0, kc=2.0)
    I1 = O.shoot(vt, p, I0).J1
    v, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=10)
    # accepted Armijo steps decrease E strictly; a failed line search (tau = 0) keeps v0
    Es = [it.E for it in log] + [lin.E]
    for k, it in enumerate(log):
        assert (Es[k + 1] < Es[k]) if it.tau > 0 else (Es[k + 1] == Es[k]), Es
    assert log[0].tau > 0 and Es[-1] < 0.95 * Es[0]
    assert log[0].g_inf_rel == 1.0 and all(it.cg_iters >= 1 for it in log)


# --------------------------------------------------------------------------- "GN, L2" and gradient descent
def test_l2_gradient_at_zero_closed_form():
    """At v0 = 0 the L2-gradient is -(2/sigma2) (I0 - I1) grad I0: no K (the V-gradient's K is undone by L)."""
    p, I0, I1, _ = phantom_case()
    g, _ = O.gradient_l2(np.zeros((3,) + p.n), I0, I1, p)
    expect = -(2.0 / p.sigma2) * (I0 - I1)[None] * O.grad(I0, p)
    np.testing.assert_allclose(g, expect, atol=1e-11 * np.abs(expect).max())


def _l2_system(n=(4, 4, 6)):
    p = P(n, alpha=0.05, nt=4, sigma2=0.002)
    I0 = phantom(n, 3, (1.0, 2.0), False, 1000)
    I1 = phantom(n, 3, (1.0, 2.0), False, 1001)
    v0 = random_velocity(n, 2000, 0.5, kc=1.5)
    lin = O.linearize(v0, I0, I1, p)
    g, _ = O.gradient(v0, I0, I1, p, lin)
    return p, lin, g


def test_pcg_l2_iterates_equal_cg_v_and_dense_solve():
    """PCG in L2 with preconditioner K and CG in V produce the same iterates (exact
    arithmetic identity: r_L2 = L r_V, z = K r_L2 = r_V); with many iterations both
    reach the dense solution of L H x = -L g."""
    p, lin, g = _l2_system()
    gl2 = O.apply_L(g, p)
    hl2 = lambda d: O.hessvec_l2(d, lin, p)
    K = lambda r: O.apply_K(r, p)
    for k in range(1, 7):
        x_pcg, it_p = O.pcg_l2(hl2, gl2, p, 0.0, k, K)
        x_cg, it_c = O.cg_v(lambda d: O.hessvec(d, lin, p), g, p, 0.0, k)
        assert it_p == it_c == k
        assert np.linalg.norm(x_pcg - x_cg) <= 1e-10 * np.linalg.norm(x_cg)
    H = _dense_hessian(lin, p)
    Lm = _dense_L(p)
    x_dense = np.linalg.solve(Lm @ H, -gl2.ravel())
    x_pcg, _ = O.pcg_l2(hl2, gl2, p, 1e-13, 400, K)
    np.testing.assert_allclose(x_pcg.ravel(), x_dense, atol=1e-8 * np.abs(x_dense).max())


def test_pcg_l2_stops_on_the_l2_residual():
    """The stop is the first iterate with ||-g_L2 - H_L2 x_k||_L2 <= eta ||g_L2||_L2,
    the residual recomputed here from a dense H_L2 and the CG-in-V iterates."""
    p, lin, g = _l2_system()
    gl2 = O.apply_L(g, p)
    HL2 = _dense_L(p) @ _dense_hessian(lin, p)
    cell = float(np.prod(p.h))
    gnorm = np.sqrt(cell * np.sum(gl2 * gl2))
    for eta in (0.3, 0.05, 0.01):
        _, m = O.pcg_l2(lambda d: O.hessvec_l2(d, lin, p), gl2, p, eta, 200, lambda r: O.apply_K(r, p))
        res = []
        for k in (m - 1, m):
            xk = O.cg_v(lambda d: O.hessvec(d, lin, p), g, p, 0.0, k)[0] if k > 0 else np.zeros_like(g)
            r = -gl2.ravel() - HL2 @ xk.ravel()
            res.append(np.sqrt(cell * np.sum(r * r)))
        assert res[1] <= eta * gnorm * (1 + 1e-9) and res[0] > eta * gnorm, (eta, m, res, gnorm)


def test_gn_l2_solve_decreases_energy():
    p, I0, _, _ = phantom_case(n=(12, 12, 12), nt=5)
    I1 = O.shoot(random_velocity(p.n, 2100, 1.0, kc=2.0), p, I0).J1
    v, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=10, space="L2")
    Es = [it.E for it in log] + [lin.E]
    for k, it in enumerate(log):
        assert (Es[k + 1] < Es[k]) if it.tau > 0 else (Es[k + 1] == Es[k]), Es
    assert log[0].tau > 0 and Es[-1] < 0.95 * Es[0]
    g0, _ = O.gradient_l2(np.zeros((3,) + p.n), I0, I1, p)
    assert log[0].g_norm == pytest.approx(np.sqrt(O.inner(g0, g0, p)), rel=1e-12)


def test_gd_step_minimises_the_regulariser():
    """With a negligible data term E ~ <L v0, v0>, whose V-gradient is 2 v0: the
    first trial step tau0 = 1/2 lands on v0 = 0 and is accepted."""
    p, I0, I1, _ = phantom_case()
    p.sigma2 = 1e12
    v0 = random_velocity(p.n, 2200, 1.0, kc=2.0)
    v, log, _ = O.gd_solve(I0, I1, p, iters=1, v0=v0)
    assert log[0].tau == 0.5 and log[0].cg_iters == 0
    assert np.abs(v).max() <= 1e-9 * np.abs(v0).max()


def test_gd_first_step_from_zero_and_monotone():
    p, I0, _, _ = phantom_case(n=(12, 12, 12), nt=5)
    I1 = O.shoot(random_velocity(p.n, 2100, 1.0, kc=2.0), p, I0).J1
    v1, log1, _ = O.gd_solve(I0, I1, p, iters=1)
    g0 = -(2.0 / p.sigma2) * O.apply_K((I0 - I1)[None] * O.grad(I0, p), p)  # P-7 closed form
    np.testing.assert_allclose(v1, -log1[0].tau * g0, atol=1e-12 * np.abs(v1).max())
    # accepted steps decrease E strictly; near a minimum the adjoint gradient need not
    # be a descent direction of the discrete energy (optimise-then-discretise), so a
    # failed line search (tau = 0) keeping E is allowed, as for Gauss-Newton
    _, log, lin = O.gd_solve(I0, I1, p, iters=4)
    Es = [it.E for it in log] + [lin.E]
    for k, it in enumerate(log):
        assert (Es[k + 1] < Es[k]) if it.tau > 0 else (Es[k + 1] == Es[k]), Es
    assert log[0].tau > 0 and Es[-1] < 0.95 * Es[0]


# --------------------------------------------------------------------------- full Newton Hessian
def test_newton_equals_gauss_newton_at_zero_residual():
    """With I1 = J1(v0) the multiplier lambda_1 and the first-order adjoint vanish, so
    every term Gauss-Newton drops is zero."""
    p, I0, _, v0 = phantom_case(n=(10, 12, 8), nt=5)
    I1 = O.shoot(v0, p, I0).J1
    lin = O.linearize(v0, I0, I1, p)
    dv = random_field(p.n, 21, 2.0)
    hn, hg = O.hessvec_newton(dv, lin, p), O.hessvec(dv, lin, p)
    assert np.linalg.norm(hn - hg) <= 1e-13 * np.linalg.norm(hg)


def test_newton_sweep_is_the_exact_linearisation():
    """With the final condition held, the Newton sweep is the derivative of
    v0 -> backward_sweep(U_T, shoot(v0)): central FD errors fall as eps^2."""
    p, I0, I1, v0 = phantom_case(n=(12, 10, 14), nt=5)
    lin = O.linearize(v0, I0, I1, p)
    d = random_field(p.n, 5, 2.0)
    U_T = random_field(p.n, 9, 2.0)
    _, stages = O.tangent_stages(d, lin.tr, p)
    an = O.newton_sweep(U_T, np.zeros_like(U_T), stages, lin.tr, p)
    phi = lambda v: O.backward_sweep(U_T, O.shoot(v, p), p)[1]
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (phi(v0 + eps * d) - phi(v0 - eps * d)) / (2 * eps)
        errs.append(np.linalg.norm(an - fd) / np.linalg.norm(fd))
    assert errs[1] <= 1e-7 and errs[0] / errs[1] >= 50, errs


def _smooth_newton_gaps(N):
    n = (N, N, N)
    p = P(n, alpha=0.05, nt=8, sigma2=0.5)
    x = O.grid_coords(p)
    I0 = 0.5 + 0.3 * np.sin(x[0]) * np.cos(2 * x[1]) + 0.2 * np.cos(x[2] + x[0])
    I1 = 0.5 + 0.3 * np.sin(x[0] + 0.3) * np.cos(2 * x[1] - 0.2) + 0.2 * np.cos(x[2] + x[0] + 0.25)
    v0 = 0.2 * np.stack([np.sin(x[1]), np.cos(x[2] + x[0]), np.sin(x[0] - x[1])])
    d = np.stack([np.cos(x[2]), np.sin(x[0] + x[1]), np.cos(x[1])])
    lin = O.linearize(v0, I0, I1, p)
    g = lambda v: O.gradient(v, I0, I1, p)[0]
    eps = 1e-4
    fd = (g(v0 + eps * d) - g(v0 - eps * d)) / (2 * eps)
    gap = lambda h: np.linalg.norm(h - fd) / np.linalg.norm(fd)
    return gap(O.hessvec_newton(d, lin, p)), gap(O.hessvec(d, lin, p))


def test_newton_hessian_is_the_derivative_of_the_gradient():
    """Against central FD of the gradient map, the Newton Hv differs only by the
    Jacobi-form incremental image (R8), a first-order discretisation gap that halves
    from 16^3 to 32^3; the Gauss-Newton Hv keeps an O(residual) gap that does not."""
    n16, g16 = _smooth_newton_gaps(16)
    n32, g32 = _smooth_newton_gaps(32)
    assert n16 <= 0.015 and n16 / n32 >= 1.6, (n16, n32)
    assert g32 >= 4 * n32 and g32 >= 0.7 * g16, (g16, g32, n32)


def test_cg_negative_curvature():
    """Non-positive curvature on the first direction gives the steepest-descent
    direction -g; met later, CG stops at its current iterate."""
    p = P((4, 4, 6))
    g = random_field(p.n, 3, 1.5)
    x, it = O.cg_v(lambda d: -d, g, p, 1e-12, 10)
    assert it == 0 and np.array_equal(x, -g)
    # H = identity on the span of g's first mode, -identity beyond: the second direction is negative
    e = g / math.sqrt(O.inner_V(g, g, p))
    hess = lambda d: 2 * O.inner_V(e, d, p) * e - (d - O.inner_V(e, d, p) * e)
    x2, it2 = O.cg_v(hess, g + 0.3 * random_field(p.n, 4, 1.5), p, 1e-12, 10)
    assert it2 >= 1 and np.isfinite(x2).all() and np.abs(x2).max() > 0


def test_newton_solve_decreases_energy():
    p, I0, _, _ = phantom_case(n=(12, 12, 12), nt=5)
    I1 = O.shoot(random_velocity(p.n, 2100, 1.0, kc=2.0), p, I0).J1
    v, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=10, hessian="newton")
    Es = [it.E for it in log] + [lin.E]
    for k, it in enumerate(log):
        assert (Es[k + 1] < Es[k]) if it.tau > 0 else (Es[k + 1] == Es[k]), Es
    assert log[0].tau > 0 and Es[-1] < 0.95 * Es[0]


# --------------------------------------------------------------------------- planted mistakes
def _fails(check):
    try:
        check()
    except AssertionError:
        return True
    return False


def test_planted_mistakes(monkeypatch):
    """Each plausible slip, planted in the oracle on the CPU, is caught by some pin."""
    import oracle.lddmm_oracle as OM

    def plant(name, fn):
        monkeypatch.setattr(OM, name, fn)
        monkeypatch.setattr(O, name, fn, raising=False)  # private helpers are not re-exported

    orig = {k: getattr(OM, k) for k in ("ad", "ad_star", "backward_sweep", "symbol_L", "sl_step")}

    def ad_transposed(v, w, p):  # (Dv)^T w - (Dw)^T v: antisymmetric, but wrong
        out = np.zeros_like(w)
        for c in range(3):
            for d in range(3):
                out[c] += OM.ddx(v[d], c, p) * w[d] - OM.ddx(w[d], c, p) * v[d]
        return out

    def ad_star_sign(v, mu, p):  # wrong sign on the divergence part
        out = np.zeros_like(mu)
        for c in range(3):
            for d in range(3):
                out[c] += OM.ddx(v[d], c, p) * mu[d] - OM.ddx(mu[c] * v[d], d, p)
        return out

    def bw_wrong_order(U_T, tr, p):  # forward stage order instead of the transposed one
        swapped = OM.Trajectory(tr.mu_star + [tr.mu[-1]], tr.v_star + [tr.v[-1]], tr.mu[:-1], tr.v[:-1])
        return orig["backward_sweep"](U_T, swapped, p)

    def symbol_wrong_power(p):
        return orig["symbol_L"](p) * orig["symbol_L"](OM.Params(p.n, p.alpha, 1, p.nt))

    def sl_forward_foot(u, v_old, v_new, p, x=None):  # foot point traced forward, not back
        if x is None:
            x = OM.grid_coords(p)
        X = x + 0.5 * p.dt * (v_new + OM.interp(v_old, x + p.dt * v_new, p))
        return OM.interp(u, X, p) + (X - x)

    def pcg_unpreconditioned_beta(hess, g, p, eta, maxit, precond):  # beta from <r, r>, not <r, K r>
        x = np.zeros_like(g)
        r = -g
        z = precond(r)
        d = z.copy()
        rz = OM.inner(r, z, p)
        for _ in range(maxit):
            q = hess(d)
            a = rz / OM.inner(d, q, p)
            x = x + a * d
            rr_old = OM.inner(r, r, p)
            r = r - a * q
            z = precond(r)
            d = z + (OM.inner(r, r, p) / rr_old) * d
            rz = OM.inner(r, z, p)
        return x, maxit

    def variation_wrong_sign(U, w, dv, dmu, mu, p):  # +ad_{dv} w instead of -ad_{dv} w
        a, b = orig["_adjoint_rhs_variation"](U, w, dv, dmu, mu, p)
        return a, b + 2 * OM.ad(dv, w, p)

    def sl_swapped_times(u, v_old, v_new, p, x=None):  # the two velocity times exchanged in the backtrace
        if x is None:
            x = OM.grid_coords(p)
        X = x - 0.5 * p.dt * (v_old + OM.interp(v_new, x - p.dt * v_old, p))
        return OM.interp(u, X, p) + (X - x)

    def sl_frozen_time(u, v_old, v_new, p, x=None):  # v_n at both evaluations: no time variation
        if x is None:
            x = OM.grid_coords(p)
        X = x - 0.5 * p.dt * (v_old + OM.interp(v_old, x - p.dt * v_old, p))
        return OM.interp(u, X, p) + (X - x)

    def vjp_without_L(gbar, lin, p):  # returns w_0 instead of L w_0
        _, w0 = OM.backward_sweep(-np.asarray(gbar)[None] * lin.G, lin.tr, p)
        return w0

    def vjp_gbar_sign(gbar, lin, p):  # U^(1) = +gbar grad J_1
        return orig["vjp_J1"](-np.asarray(gbar), lin, p)

    orig["pcg_l2"] = OM.pcg_l2
    orig["_adjoint_rhs_variation"] = OM._adjoint_rhs_variation
    orig["vjp_J1"] = OM.vjp_J1
    sl_pin = lambda: test_sl_backtrace_is_heun_on_the_characteristics(2)
    cases = [
        ("sl_step", sl_swapped_times, [sl_pin]),
        ("sl_step", sl_frozen_time, [sl_pin]),
        ("vjp_J1", vjp_without_L, [test_vjp_matches_finite_differences_of_the_warped_image]),
        ("vjp_J1", vjp_gbar_sign, [test_vjp_matches_finite_differences_of_the_warped_image]),
        ("_adjoint_rhs_variation", variation_wrong_sign, [test_newton_sweep_is_the_exact_linearisation]),
        ("pcg_l2", pcg_unpreconditioned_beta, [test_pcg_l2_iterates_equal_cg_v_and_dense_solve]),
        ("ad", ad_transposed, [test_ad_constant_velocity_closed_form]),
        ("ad_star", ad_star_sign, [test_ad_identities, test_dot_product_tangent_vs_backward,
                                   test_transported_momentum_identity]),
        ("backward_sweep", bw_wrong_order, [test_dot_product_tangent_vs_backward]),
        ("symbol_L", symbol_wrong_power, [lambda: test_L_K_single_modes((8, 8, 8))]),
        ("sl_step", sl_forward_foot, [test_shoot_constant_velocity_translates, test_sl_stationary_shear_exact,
                                      test_transported_momentum_identity]),
    ]
    for name, bad, checks in cases:
        plant(name, bad)
        for check in checks:
            assert _fails(check), (name, check)
        plant(name, orig[name])
