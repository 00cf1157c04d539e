"""Pins of the FP64 oracle of PDE-constrained LDDMM (the comparison method of
Section 2.3): closed forms at v = 0, exact translations, a compressible 1D flow
against the exact solution of the continuity equation, finite differences of the
energy converging with the grid, near-symmetry of the Gauss-Newton Hessian, and
planted slips that one of these pins must catch."""

import math

import numpy as np
import pytest

import oracle as O
from oracle import pde_lddmm as PL
from synth import phantom, random_field, random_velocity


def P(n, alpha=0.02, s=2, nt=6, sigma2=0.05):
    return O.Params(tuple(n), alpha, s, nt, sigma2)


def stack(fn, p):
    return np.stack([fn(k) for k in range(p.nt + 1)])


def smooth_case(N, nt=8, amp=0.15, stationary=True):
    p = P((N, N, N), alpha=0.05, nt=nt, sigma2=1.0)
    x = O.grid_coords(p)
    I0 = 0.5 + 0.3 * np.sin(x[0]) * np.cos(2 * x[1]) + 0.2 * np.cos(x[2] + x[0])
    I1 = 0.5 + 0.3 * np.sin(x[0] + 0.2) * np.cos(2 * x[1] - 0.1) + 0.2 * np.cos(x[2] + x[0] + 0.15)
    base = np.stack([np.sin(x[1]), np.cos(x[2] + x[0]), np.sin(x[0] - x[1])])
    d = np.stack([np.cos(x[2]), np.sin(x[0] + 2 * x[1]), np.cos(x[1])])
    if stationary:
        return p, I0, I1, amp * base, d
    t = np.linspace(0.0, 1.0, nt + 1)
    v = np.stack([amp * (1.0 + 0.5 * tk) * base for tk in t])
    dd = np.stack([(1.0 - 0.3 * tk) * d for tk in t])
    return p, I0, I1, v, dd


@pytest.mark.parametrize("stationary", [True, False])
def test_zero_velocity_closed_forms(stationary):
    """v = 0: m_t = I_0, lambda_t = -(2/s2)(I_0 - I_1); the L2 gradient is
    -(2/s2)(I_0 - I_1) grad I_0 at every time point (its time integral for a
    stationary v), and the Gauss-Newton Hessian is
    2 L dv_n + (2/s2) (grad I_0 . int dv dt) grad I_0."""
    n = (8, 6, 10)
    p = P(n)
    I0 = phantom(n, 3, (1.0, 2.0), False, 1000)
    I1 = phantom(n, 3, (1.0, 2.0), False, 1001)
    gI0 = O.grad(I0, p)
    ref = -(2.0 / p.sigma2) * (I0 - I1)[None] * gI0
    if stationary:
        v = np.zeros((3,) + n)
        dv = random_field(n, 5, 2.0)
        g, lin = PL.gradient(v, I0, I1, p, True)
        np.testing.assert_allclose(g, ref, atol=1e-12)
        hv = PL.hessvec(dv, lin, p)
        href = 2 * O.apply_L(dv, p) + (2.0 / p.sigma2) * np.sum(gI0 * dv, axis=0)[None] * gI0
        np.testing.assert_allclose(hv, href, atol=1e-10 * np.abs(href).max())
    else:
        v = np.zeros((p.nt + 1, 3) + n)
        dv = np.stack([random_field(n, 10 + k, 2.0) for k in range(p.nt + 1)])
        g, lin = PL.gradient(v, I0, I1, p, False)
        for k in range(p.nt + 1):
            np.testing.assert_allclose(g[k], ref, atol=1e-12)
        hv = PL.hessvec(dv, lin, p)
        w = PL.weights(p, False)
        mean_dv = sum(w[k] * dv[k] for k in range(p.nt + 1))
        src = (2.0 / p.sigma2) * np.sum(gI0 * mean_dv, axis=0)[None] * gI0
        for k in range(p.nt + 1):
            href = 2 * O.apply_L(dv[k], p) + src
            np.testing.assert_allclose(hv[k], href, atol=1e-10 * np.abs(href).max())


def test_constant_velocity_translates_state_and_adjoint():
    """A constant velocity that moves a whole number of cells per step: the state
    is I_0 shifted by -c and the adjoint (divergence-free) lambda_1 shifted by +c,
    exactly (numpy roll)."""
    n = (8, 10, 12)
    p = P(n, nt=4)
    h = p.h
    c = np.array([1, -2, 1]) * np.array(h) * p.nt  # one, two, one cells per step
    v = np.broadcast_to(c[:, None, None, None], (3,) + n).copy()
    I0 = phantom(n, 3, (1.0, 2.0), False, 1002)
    vs = PL.velocities(v, p, True)
    m = PL.state(vs, I0, p)
    expect = np.roll(I0, (p.nt * 1, p.nt * -2, p.nt * 1), axis=(0, 1, 2))
    np.testing.assert_allclose(m[-1], expect, atol=1e-13)
    lam1 = phantom(n, 3, (1.0, 2.0), False, 1003)
    lam = PL.adjoint(vs, lam1, p)
    np.testing.assert_allclose(lam[0], np.roll(lam1, (-p.nt, 2 * p.nt, -p.nt), axis=(0, 1, 2)), atol=1e-13)
    # the inverse map of a translation by c over unit time is x - c
    u = PL.displacement(vs, p)
    np.testing.assert_allclose(u, np.broadcast_to(-c[:, None, None, None], u.shape), atol=1e-13)


def _flow(y, t):
    return 0.3 * (1.0 + t) * np.sin(y) + 0.15 * np.cos(2.0 * y) * t + 0.05


def _dflow(y, t):
    return 0.3 * (1.0 + t) * np.cos(y) - 0.3 * np.sin(2.0 * y) * t


def _exact_adjoint_1d(lam1, y0, steps=400):
    """Continuity equation d_t lam + d_y(lam f) = 0 backward from t = 1: lam(0, y) =
    lam(1, phi(y)) phi'(y), phi the flow map from 0 to 1 (RK4 on the trajectory and
    its variational equation)."""
    y = y0.copy()
    J = np.ones_like(y)
    h = 1.0 / steps
    t = 0.0
    for _ in range(steps):
        def rhs(yy, jj, tt):
            return _flow(yy, tt), _dflow(yy, tt) * jj
        k1 = rhs(y, J, t)
        k2 = rhs(y + 0.5 * h * k1[0], J + 0.5 * h * k1[1], t + 0.5 * h)
        k3 = rhs(y + 0.5 * h * k2[0], J + 0.5 * h * k2[1], t + 0.5 * h)
        k4 = rhs(y + h * k3[0], J + h * k3[1], t + h)
        y = y + h / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        J = J + h / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
        t += h
    return lam1(y) * J


def _adjoint_1d_error(nt, N=4096):
    n = (4, 4, N)
    p = P(n, nt=nt)
    x = O.grid_coords(p)
    vs = []
    for k in range(nt + 1):
        v = np.zeros((3,) + n)
        v[2] = _flow(x[2], k / nt)
        vs.append(v)
    lam1 = lambda y: 1.0 + 0.5 * np.cos(y) + 0.2 * np.sin(3.0 * y)
    lam = PL.adjoint(vs, lam1(x[2]), p)
    line = np.arange(N) * p.h[2]
    return np.abs(lam[0][0, 0, :] - _exact_adjoint_1d(lam1, line)).max()


def _exact_foot_1d(x1, steps=400):
    """Foot at t = 0 of the characteristic dy/dt = f(y, t) through x1 at t = 1 (RK4 backward)."""
    y = x1.copy()
    h = 1.0 / steps
    t = 1.0
    for _ in range(steps):
        k1 = _flow(y, t)
        k2 = _flow(y - 0.5 * h * k1, t - 0.5 * h)
        k3 = _flow(y - 0.5 * h * k2, t - 0.5 * h)
        k4 = _flow(y - h * k3, t - h)
        y = y - h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t -= h
    return y


def _displacement_1d_error(nt, N=4096):
    n = (4, 4, N)
    p = P(n, nt=nt)
    x = O.grid_coords(p)
    vs = []
    for k in range(nt + 1):
        v = np.zeros((3,) + n)
        v[2] = _flow(x[2], k / nt)
        vs.append(v)
    u = PL.displacement(vs, p)
    line = np.arange(N) * p.h[2]
    return np.abs(u[2, 0, 0, :] - (_exact_foot_1d(line) - line)).max(), np.abs(u[:2]).max()


def test_displacement_is_the_inverse_flow_map():
    """The inverse-map displacement of a 1D flow that varies in space and time:
    u_1(x) converges to (foot of the exact characteristic through x) - x at second
    order in dt; the components across the flow stay zero."""
    res = [_displacement_1d_error(nt) for nt in (8, 16, 32)]
    errs = [e for e, _ in res]
    r = [errs[k] / errs[k + 1] for k in range(2)]
    assert errs[0] < 0.05 and all(3.3 <= q <= 4.7 for q in r), (errs, r)
    assert all(z == 0.0 for _, z in res)


def test_displacement_warps_the_template_like_the_state():
    """I_0 o (id + u_1) and the transported image m(1) are two discretisations of
    the same deformed template: their gap shrinks as the grid is refined."""
    gaps = []
    for N in (32, 64):  # at 16^3 the two first-order errors still partly cancel
        p, I0, _, v, _ = smooth_case(N, stationary=False)
        vs = PL.velocities(v, p, False)
        m1 = PL.state(vs, I0, p)[-1]
        u = PL.displacement(vs, p)
        warped = O.interp(I0, O.grid_coords(p) + u, p)
        gaps.append(np.linalg.norm(warped - m1) / np.linalg.norm(m1 - I0))
    assert gaps[0] < 0.2 and gaps[1] <= gaps[0] / 1.5, gaps


def test_adjoint_transport_of_a_compressible_flow():
    """The adjoint (continuity) equation of Section 2.3 along a 1D flow that varies
    in space and time (so div v != 0): lambda_0 converges to the exact solution
    lambda(1, phi(y)) phi'(y) at second order in dt."""
    errs = [_adjoint_1d_error(nt) for nt in (8, 16, 32)]
    r = [errs[k] / errs[k + 1] for k in range(2)]
    assert errs[0] < 0.05 and all(3.3 <= q <= 4.7 for q in r), (errs, r)


def test_mass_is_conserved_by_the_adjoint():
    """int lambda is invariant under -d_t lambda - div(lambda v) = 0; the SL scheme
    keeps it to discretisation error."""
    n = (24, 24, 24)
    p = P(n, nt=8)
    v = random_velocity(n, 2010, 1.5, kc=2.0)
    lam1 = 1.0 + phantom(n, 3, (2.0, 4.0), False, 1004)
    lam = PL.adjoint(PL.velocities(v, p, True), lam1, p)
    assert abs(lam[0].sum() / lam1.sum() - 1.0) < 2e-3


@pytest.mark.parametrize("stationary", [True, False])
def test_gradient_vs_finite_differences_converges(stationary):
    """Optimise-then-discretise: the L2 gradient agrees with central FD of the
    energy to discretisation error, which shrinks when the same smooth case is
    sampled on a finer grid."""
    gaps = []
    for N in (16, 32):
        p, I0, I1, v, d = smooth_case(N, stationary=stationary)
        g, _ = PL.gradient(v, I0, I1, p, stationary)
        # the data-term part of the gradient as the direction (the regulariser is exact)
        gd = g - 2 * (O.apply_L(v, p) if stationary else np.stack([O.apply_L(v[k], p) for k in range(p.nt + 1)]))
        d = gd / math.sqrt(PL.inner_t(gd, gd, p, stationary))
        eps = 1e-4
        fd = (PL.energy(v + eps * d, I0, I1, p, stationary) - PL.energy(v - eps * d, I0, I1, p, stationary)) / (2 * eps)
        an = PL.inner_t(g, d, p, stationary)
        gaps.append(abs(fd - an) / abs(fd))
    assert gaps[0] <= 0.1 and gaps[1] <= gaps[0] / 1.6, gaps


@pytest.mark.parametrize("stationary", [True, False])
def test_regularisation_gradient_exact(stationary):
    """Zero residual (I_1 = m(1) of v): lambda = 0 and the gradient is the
    regulariser's alone, whose quadratic energy central FD differentiates exactly."""
    p, I0, _, v, d = smooth_case(8, nt=4, stationary=stationary)
    d = d + v / np.abs(v).max()  # not orthogonal to L v
    I1 = PL.state(PL.velocities(v, p, stationary), I0, p)[-1]
    g, lin = PL.gradient(v, I0, I1, p, stationary)
    L = (lambda f: O.apply_L(f, p)) if stationary else (lambda f: np.stack([O.apply_L(f[k], p) for k in range(p.nt + 1)]))
    eps = 1e-3
    ereg = lambda vv: PL.inner_t(L(vv), vv, p, stationary)
    fd = (ereg(v + eps * d) - ereg(v - eps * d)) / (2 * eps)
    assert PL.inner_t(g, d, p, stationary) == pytest.approx(fd, rel=1e-10)


@pytest.mark.parametrize("stationary", [True, False])
def test_gauss_newton_hessian_near_symmetric_and_positive(stationary):
    """The discretised continuous Gauss-Newton Hessian is symmetric up to
    discretisation error (shrinking with N) and keeps <a, H a> above its
    regulariser part 2 <L a, a>."""
    gaps = []
    for N in (12, 24):
        p, I0, I1, v, d = smooth_case(N, nt=6, stationary=stationary)
        _, lin = PL.gradient(v, I0, I1, p, stationary)
        a = d
        b = (np.stack([O.apply_K(d[k][::-1].copy(), p) for k in range(p.nt + 1)]) if not stationary
             else O.apply_K(d[::-1].copy(), p))
        Ha, Hb = PL.hessvec(a, lin, p), PL.hessvec(b, lin, p)
        aHb, Hab = PL.inner_t(a, Hb, p, stationary), PL.inner_t(Ha, b, p, stationary)
        gaps.append(abs(aHb - Hab) / abs(aHb))
        L = (lambda f: O.apply_L(f, p)) if stationary else (lambda f: np.stack([O.apply_L(f[k], p) for k in range(p.nt + 1)]))
        assert PL.inner_t(a, Ha, p, stationary) >= 2 * PL.inner_t(L(a), a, p, stationary) * (1 - 1e-3)
    assert gaps[0] < 0.05 and gaps[1] <= gaps[0] / 1.5, gaps


@pytest.mark.parametrize("stationary", [True, False])
def test_gn_solve_decreases_energy(stationary):
    n = (12, 12, 12)
    p = P(n, nt=4)
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000)
    I1 = O.shoot(random_velocity(n, 2100, 1.0, kc=2.0), p, I0).J1
    v, log, lin = PL.gn_solve(I0, I1, p, stationary, gn_iters=3, cg_iters=8)
    Es = [it["E"] for it in log] + [lin.E]
    assert log and log[0]["tau"] > 0 and Es[-1] < 0.9 * Es[0], Es
    for k, it in enumerate(log):
        assert (Es[k + 1] < Es[k]) if it["tau"] > 0 else (Es[k + 1] == Es[k]), Es


def _fails(check):
    try:
        check()
    except AssertionError:
        return True
    return False


def test_planted_mistakes(monkeypatch):
    """Plausible slips planted in this oracle on the CPU: each fails some pin."""
    import oracle.pde_lddmm as M

    orig_adjoint = M.adjoint
    orig_weights = M.weights
    orig_gradient = M.gradient

    def adjoint_no_divergence(vs, lam1, p):  # plain transport, no div factor
        x = O.grid_coords(p)
        lam = [None] * (p.nt + 1)
        lam[p.nt] = np.asarray(lam1, dtype=np.float64)
        for n in reversed(range(p.nt)):
            lam[n] = O.interp(lam[n + 1], M.forward_trace(vs[n], vs[n + 1], p, x), p)
        return lam

    def adjoint_backtrace(vs, lam1, p):  # traced along the backward foot instead of forward
        x = O.grid_coords(p)
        lam = [None] * (p.nt + 1)
        lam[p.nt] = np.asarray(lam1, dtype=np.float64)
        for n in reversed(range(p.nt)):
            Y = M.backtrace(vs[n], vs[n + 1], p, x)
            lam[n] = O.interp(lam[n + 1], Y, p) * np.exp(0.5 * p.dt * (M.div(vs[n], p) + O.interp(M.div(vs[n + 1], p), Y, p)))
        return lam

    def weights_rectangle(p, stationary):  # rectangle rule instead of the trapezoid
        return np.array([1.0]) if stationary else np.full(p.nt + 1, 1.0 / (p.nt + 1))

    def gradient_half_regulariser(v, I0, I1, p, stationary, lin=None):  # the printed L v_t without the 2
        g, lin = orig_gradient(v, I0, I1, p, stationary, lin)
        L = (lambda f: O.apply_L(f, p)) if stationary else (lambda f: np.stack([O.apply_L(f[k], p) for k in range(p.nt + 1)]))
        return g - L(lin.v), lin

    orig_displacement = M.displacement

    def displacement_forward(vs, p):  # foot traced forward along the flow instead of backward
        x = O.grid_coords(p)
        u = np.zeros((3,) + tuple(p.n))
        for n in range(p.nt):
            X = M.forward_trace(vs[n], vs[n + 1], p, x)
            u = O.interp(u, X, p) + (X - x)
        return u

    cases = [
        ("displacement", displacement_forward, [test_displacement_is_the_inverse_flow_map,
                                                test_constant_velocity_translates_state_and_adjoint]),
        ("adjoint", adjoint_no_divergence, [test_adjoint_transport_of_a_compressible_flow]),
        ("adjoint", adjoint_backtrace, [test_adjoint_transport_of_a_compressible_flow,
                                        test_constant_velocity_translates_state_and_adjoint]),
        ("weights", weights_rectangle, [lambda: test_zero_velocity_closed_forms(False)]),
        ("gradient", gradient_half_regulariser, [lambda: test_regularisation_gradient_exact(True)]),
    ]
    originals = {"adjoint": orig_adjoint, "weights": orig_weights, "gradient": orig_gradient,
                 "displacement": orig_displacement}
    for name, bad, checks in cases:
        monkeypatch.setattr(M, name, bad)
        monkeypatch.setattr(PL, name, bad)
        for check in checks:
            assert _fails(check), (name, bad.__name__, check)
        monkeypatch.setattr(M, name, originals[name])
        monkeypatch.setattr(PL, name, originals[name])
