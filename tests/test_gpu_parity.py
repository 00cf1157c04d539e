"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Inputs are seeded synthetic phantoms / band-limited fields from ``synth``; the
same arrays feed both sides.  Tolerances (relative L2):
  FP64 fields: 1e-11 (operators 1e-12) - both sides are FP64 with different
                summation orders;
  FP32 fields: shooting outputs 1e-5, gradient and Hessian-vector product 1e-4
                (the stated FP32 targets), operators 2e-6.
Sizes span several FFT stages, mixed radices (2, 3, 5, 8) and non-cubic grids,
including one that takes the split (non-fused) transform path.
"""

import math

import numpy as np
import pytest
import torch

import oracle as O
from synth import phantom, random_field, random_velocity

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a.detach().cpu() if torch.is_tensor(a) else a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def T(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


TOL = {
    torch.float64: dict(op=1e-12, shoot=1e-11, grad=1e-11, hv=1e-11),
    torch.float32: dict(op=2e-6, shoot=1e-5, grad=1e-4, hv=1e-4),
}


def l_tol(p, f, Lf, dtype):
    """Bound for applying L: transform roundoff (relative eps per mode) is
    multiplied by the symbol, so the relative error of L f is about
    eps * rms(L^) * ||f|| / ||L f||; K^ <= 1 has no such growth."""
    eps = 1.1e-16 if dtype == torch.float64 else 6e-8
    lam = O.symbol_L(p)
    amp = math.sqrt(float(np.mean(lam * lam))) * np.linalg.norm(f) / np.linalg.norm(Lf)
    return max(TOL[dtype]["op"], 16 * eps * amp)


def rounded(x, dtype):
    """The values the device actually receives for x."""
    return T(x, dtype).double().cpu().numpy()


def make(n, dtype, nt=6, alpha=0.01, s=2, sigma2=1.0):
    from paper_1807_04638_amd import Registration

    say(f"[case] n={n} dtype={dtype} nt={nt} alpha={alpha} s={s} sigma2={sigma2}")
    return Registration(n, nt, alpha, s, sigma2, dtype=dtype), O.Params(tuple(n), alpha, s, nt, sigma2)


def images(n, seed=0):
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000 + seed)
    I1 = phantom(n, 4, (1.5, 3.0), False, 1100 + seed)
    return I0, I1


DTYPES = [torch.float64, torch.float32]
SMALL = [(16, 12, 20), (32, 32, 32), (24, 20, 30)]


# ------------------------------------------------------------------ a1: K / L
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SMALL + [(8, 10, 6)])
def test_operator_parity(n, dtype):
    R, p = make(n, dtype)
    f = rounded(random_field(n, 1, kc=max(n) / 4), dtype)
    Lf = O.apply_L(f, p)
    for op, ref, tol in (("K", O.apply_K(f, p), TOL[dtype]["op"]), ("L", Lf, l_tol(p, f, Lf, dtype))):
        got = R.apply_K(T(f, dtype)) if op == "K" else R.apply_L(T(f, dtype))
        e = rel(got, ref)
        say(f"  {op} rel {e:.3e} (tol {tol:.1e})")
        assert e <= tol
    # scalar fields, and in-place use
    s = T(f[0], dtype)
    R.apply_K(s, out=s)
    assert rel(s, O.apply_K(f[0], p)) <= TOL[dtype]["op"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(32, 32, 32), (64, 64, 64), (16, 32, 64), (80, 80, 80), (112, 112, 112)])
@pytest.mark.parametrize("opts", [{"fft.static": 0}, {"fft.static": 1}, {"fft.force_split": 1},
                                  {"fft.force_split": 1, "fft.static": 0}, {"fft.plane_threads": 256, "fft.pencil_tb": 32},
                                  {"fft.plane_grid": 7}, {"fft.plane_grid": 2, "fft.plane_threads": 512},
                                  {"fft.plane_halves": 0}, {"fft.plane_threads": 512, "fft.pencil_tb": 8}])
def test_operator_transform_variants(n, dtype, opts):
    """Every transform path (compile-time / generic kernels, fused / split passes,
    launch shapes, plane walks with a ragged last round) against the oracle on
    the same input."""
    R, p = make(n, dtype, alpha=0.005)
    for k, v in opts.items():
        R.set_option(k, v)
    say(f"  options {opts} fused={R.get_option('fft.fused')} static_kernels={R.get_option('fft.static_kernels')} "
        f"plane_walk={R.get_option('fft.plane_walk')} halves={R.get_option('fft.plane_halves_used')}")
    f = rounded(random_field(n, 3, kc=max(n) / 3), dtype)
    Lf = O.apply_L(f, p)
    assert rel(R.apply_K(T(f, dtype)), O.apply_K(f, p)) <= TOL[dtype]["op"]
    assert rel(R.apply_L(T(f, dtype)), Lf) <= l_tol(p, f, Lf, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("grid", [256, 192, 100, 1])
def test_plane_walk_matches_one_plane_per_workgroup(dtype, grid):
    """128^3: workgroups walking several (x1, x2) planes (next plane's inputs in
    registers) give the transform of one plane per workgroup, for vector and
    scalar fields, and stay within the oracle's tolerance."""
    n = (128, 128, 128)
    R, p = make(n, dtype, alpha=0.0025)
    f = rounded(random_field(n, 21, kc=20.0), dtype)
    ft = T(f, dtype)
    R.set_option("fft.plane_halves", 0)
    R.set_option("fft.plane_grid", 0)
    assert R.get_option("fft.plane_halves_used") == 0
    ref_K, ref_L = R.apply_K(ft).clone(), R.apply_L(ft).clone()
    ref_s = R.apply_K(ft[1].contiguous()).clone()
    threads = 1024 if dtype == torch.float32 else 512
    R.set_option("fft.plane_threads", threads)
    R.set_option("fft.plane_grid", grid)
    walk = R.get_option("fft.plane_walk")
    say(f"  plane_grid {grid} threads {threads}: walk {walk}")
    assert walk == grid
    for got, ref in ((R.apply_K(ft), ref_K), (R.apply_L(ft), ref_L), (R.apply_K(ft[1].contiguous()), ref_s)):
        e = rel(got, ref.cpu())
        say(f"  walk vs one plane per workgroup: rel {e:.2e}")
        assert e <= (1e-6 if dtype == torch.float32 else 1e-14)
    assert rel(R.apply_K(ft), O.apply_K(f, p)) <= TOL[dtype]["op"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("opts", [{}, {"fft.static": 0}, {"fft.force_split": 1}, {"fft.plane_grid": 7},
                                  {"fft.plane_halves": 0}])
def test_sweeps_under_transform_paths(dtype, opts):
    """The adjoint and Newton stages hand K's addend to the transform: the inverse
    plane pass adds it on the compile-time path (one plane per workgroup or a
    plane walk), an axpy after the transform does on the generic and split paths.
    Gradient, GN Hv and Newton Hv against the oracle on each path."""
    n = (32, 32, 32)
    R, p = make(n, dtype, sigma2=0.05)
    for k, v in opts.items():
        R.set_option(k, v)
    say(f"  options {opts} fused={R.get_option('fft.fused')} static_kernels={R.get_option('fft.static_kernels')} "
        f"plane_walk={R.get_option('fft.plane_walk')} halves={R.get_option('fft.plane_halves_used')}")
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2004, 1.5, kc=2.0)
    dv = random_field(n, 7, kc=3.0)
    go, lin = O.gradient(v0, I0, I1, p)
    g, _ = R.gradient(T(v0, dtype))
    errs = dict(grad=rel(g, go), hv=rel(R.hessvec(T(dv, dtype)), O.hessvec(dv, lin, p)),
                hv_newton=rel(R.hessvec(T(dv, dtype), newton=True), O.hessvec_newton(dv, lin, p)))
    say("  ", errs)
    assert errs["grad"] <= TOL[dtype]["grad"]
    assert errs["hv"] <= TOL[dtype]["hv"] and errs["hv_newton"] <= TOL[dtype]["hv"]


@pytest.mark.parametrize("n, dtype", [((128, 128, 128), torch.float32), ((128, 128, 128), torch.float64),
                                      ((256, 256, 256), torch.float32), ((96, 80, 80), torch.float64)])
def test_half_planes_match_whole_planes(n, dtype):
    """Half planes (even and odd x1 rows as separate units, merged by the x0
    pencil pass) give the transform of whole planes (or, where a whole plane
    exceeds the LDS, of the split passes), for vector and scalar fields, K and L;
    and K stays within the oracle's tolerance at 128^3.  (The inverse pass that
    adds K's addend is covered by the sweeps under the default transform path.)"""
    R, p = make(n, dtype, alpha=0.0025)
    f = rounded(random_field(n, 23, kc=20.0), dtype)
    ft = T(f, dtype)
    assert R.get_option("fft.plane_halves_used") == 1
    got = [R.apply_K(ft).clone(), R.apply_L(ft).clone(), R.apply_K(ft[2].contiguous()).clone()]
    R.set_option("fft.plane_halves", 0)
    assert R.get_option("fft.plane_halves_used") == 0
    say(f"  reference path: fused={R.get_option('fft.fused')}")
    ref = [R.apply_K(ft), R.apply_L(ft), R.apply_K(ft[2].contiguous())]
    # two roundings of L's transforms, each within the bound against the exact result
    tol_l = 2 * l_tol(p, f, ref[1].double().cpu().numpy(), dtype)
    for a, b, tol in zip(got, ref, (TOL[dtype]["op"], tol_l, TOL[dtype]["op"])):
        e = rel(a, b.cpu())
        say(f"  halves vs whole: rel {e:.2e} (tol {tol:.1e})")
        assert e <= tol
    if n == (128, 128, 128):
        assert rel(got[0], O.apply_K(f, p)) <= TOL[dtype]["op"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("halves", [1, 0])
def test_operator_head_grid_180x216x180(dtype, halves):
    """Brain-shaped grid (radices 2, 3, 4, 5, 8): half planes (fused in both
    precisions), or whole planes: fused compile-time planes in FP32, the split
    path in FP64 (a whole plane exceeds the LDS)."""
    n = (180, 216, 180)
    R, p = make(n, dtype, alpha=0.0025)
    R.set_option("fft.plane_halves", halves)
    say(f"  fused={R.get_option('fft.fused')} static_kernels={R.get_option('fft.static_kernels')} "
        f"halves={R.get_option('fft.plane_halves_used')}")
    assert R.get_option("fft.plane_halves_used") == halves
    assert R.get_option("fft.fused") == (1 if halves or dtype == torch.float32 else 0)
    assert R.get_option("fft.static_kernels") >= 2
    f = rounded(random_field(n, 14, kc=10.0), dtype)
    Lf = O.apply_L(f, p)
    assert rel(R.apply_K(T(f, dtype)), O.apply_K(f, p)) <= TOL[dtype]["op"]
    assert rel(R.apply_L(T(f, dtype)), Lf) <= l_tol(p, f, Lf, dtype)


def test_operator_split_path_fp64():
    """(x1, x2) half-plane of 256 x 129 complex doubles exceeds LDS: split passes."""
    n = (6, 256, 256)
    R, p = make(n, torch.float64, alpha=0.002)
    f = random_field(n, 2, kc=20.0)
    assert rel(R.apply_K(T(f, torch.float64)), O.apply_K(f, p)) <= 1e-12
    assert rel(R.apply_L(T(f, torch.float64)), O.apply_L(f, p)) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
def test_operator_single_modes_closed_form(dtype):
    n = (16, 24, 20)
    R, p = make(n, dtype, alpha=0.03, s=3)
    x = O.grid_coords(p)
    # L amplifies the rounding of the input in the highest modes by up to
    # max(L^) / L^(k) relative to the mode itself
    lam_max = (1.0 + p.alpha * sum((N // 2) ** 2 for N in n)) ** p.s
    eps = 1e-16 if dtype == torch.float64 else 6e-8
    for k in [(0, 0, 0), (1, 2, 3), (8, -5, 10), (3, 12, 1)]:
        f = np.cos(k[0] * x[0] + k[1] * x[1] + k[2] * x[2] + 0.4)
        lam = (1.0 + p.alpha * (k[0] ** 2 + k[1] ** 2 + k[2] ** 2)) ** p.s
        assert rel(R.apply_L(T(f, dtype)), lam * f) <= TOL[dtype]["op"] + 2 * eps * lam_max / lam
        assert rel(R.apply_K(T(f, dtype)), f / lam) <= TOL[dtype]["op"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("s", [1, 3])
def test_symbol_exponents_on_compile_time_kernels(dtype, s):
    """Exponents other than the usual s = 2 (the symbol's power loop instead of
    one square) on a grid whose transforms take the compile-time kernels: K, L,
    the gradient and the Gauss-Newton product against the oracle."""
    n = (32, 32, 32)
    R, p = make(n, dtype, alpha=0.02, s=s, sigma2=0.05)
    f = rounded(random_field(n, 1, kc=8.0), dtype)
    Lf = O.apply_L(f, p)
    eK = rel(R.apply_K(T(f, dtype)), O.apply_K(f, p))
    eL = rel(R.apply_L(T(f, dtype)), Lf)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2002, 1.0, kc=2.0)
    dv = random_field(n, 5, kc=3.0)
    g, _ = R.gradient(T(v0, dtype))
    hv = R.hessvec(T(dv, dtype))
    go, lin = O.gradient(v0, I0, I1, p)
    errs = dict(K=eK, L=eL, grad=rel(g, go), hv=rel(hv, O.hessvec(dv, lin, p)))
    say(f"  s={s} static={R.get_option('fft.static_kernels')}", {k: f"{e:.2e}" for k, e in errs.items()})
    assert R.get_option("fft.static_kernels") > 0
    assert eK <= TOL[dtype]["op"] and eL <= l_tol(p, f, Lf, dtype)
    assert errs["grad"] <= TOL[dtype]["grad"] and errs["hv"] <= TOL[dtype]["hv"]
    R.close()


# ------------------------------------------------------------------ FP64 dots
@pytest.mark.parametrize("dtype", DTYPES)
def test_dot_parity(dtype):
    n = (16, 12, 20)
    R, p = make(n, dtype)
    a, b = random_field(n, 3), random_field(n, 4)
    ta, tb = T(a, dtype), T(b, dtype)
    ref = O.inner(ta.double().cpu().numpy(), tb.double().cpu().numpy(), p)
    assert R.dot(ta, tb) == pytest.approx(ref, rel=1e-13)
    assert R.dot(ta[0].contiguous(), tb[0].contiguous()) == pytest.approx(
        O.inner(ta[0].double().cpu().numpy(), tb[0].double().cpu().numpy(), p), rel=1e-13
    )


# ------------------------------------------------------------------ a2, a3: shooting
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SMALL)
def test_shoot_parity(n, dtype):
    R, p = make(n, dtype)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2000, 1.5, kc=2.0)
    out = R.shoot(T(v0, dtype), energy=True)
    tr = O.shoot(v0, p, I0)
    errs = dict(v1=rel(out["v1"], tr.v[-1]), u1=rel(out["u1"], tr.u), J1=rel(out["J1"], tr.J1))
    say("  shoot", errs)
    for k, e in errs.items():
        assert e <= TOL[dtype]["shoot"], k
    assert out["energy"] == pytest.approx(O.energy(v0, I0, I1, p), rel=TOL[dtype]["shoot"])


@pytest.mark.parametrize("dtype", DTYPES)
def test_shoot_zero_velocity_is_identity(dtype):
    n = (16, 12, 20)
    R, p = make(n, dtype)
    I0, I1 = images(n)
    tI0 = T(I0, dtype)
    R.set_images(tI0, T(I1, dtype))
    out = R.shoot(torch.zeros((3,) + n, dtype=dtype, device=DEV))
    assert torch.equal(out["J1"], tI0)
    assert torch.count_nonzero(out["u1"]) == 0 and torch.count_nonzero(out["v1"]) == 0


# ------------------------------------------------------------------ a4, a5: gradient
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SMALL)
def test_gradient_parity(n, dtype):
    R, p = make(n, dtype, sigma2=0.05)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2001, 1.5, kc=2.0)
    g, E = R.gradient(T(v0, dtype))
    go, lin = O.gradient(v0, I0, I1, p)
    e = rel(g, go)
    say(f"  gradient rel {e:.3e}  E {E} vs {lin.E}")
    assert e <= TOL[dtype]["grad"]
    assert E == pytest.approx(lin.E, rel=TOL[dtype]["shoot"])


# ------------------------------------------------------------------ a6, a7: Hv
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SMALL)
def test_hessvec_parity(n, dtype):
    R, p = make(n, dtype, sigma2=0.05)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2002, 1.5, kc=2.0)
    dv = random_field(n, 5, kc=3.0)
    hv = R.hessvec(T(dv, dtype), v0=T(v0, dtype))
    lin = O.linearize(v0, I0, I1, p)
    ho = O.hessvec(dv, lin, p)
    e = rel(hv, ho)
    say(f"  hessvec rel {e:.3e}")
    assert e <= TOL[dtype]["hv"]
    # the current linearization is reused when v0 is omitted, bit for bit
    hv2 = R.hessvec(T(dv, dtype))
    assert torch.equal(hv, hv2)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(10, 6, 64), (8, 12, 128), (6, 8, 256), (6, 7, 128), (6, 8, 180), (8, 6, 80),
                               (6, 8, 112), (6, 8, 216), (6, 8, 96), (6, 7, 96), (6, 8, 192), (6, 60, 180),
                               (6, 112, 112)])
def test_row_vectorised_stencils(n, dtype):
    """Every stencil width a row of N2 voxels allows: one voxel per thread
    (stencil.rowvec = 0) and VW = 1, 2, 3, 4 voxels per lane with x2 neighbours
    across lanes (rows of 32 to 64 lanes: N2 = 180 takes 60 lanes at VW = 3 and
    45 at VW = 4, N2 = 216 54 lanes at VW = 4, N2 = 80 and 112 40 and 56 lanes at
    VW = 2, N2 = 96 32 lanes at VW = 3 and 48 at VW = 2, N2 = 192 64 and 48 lanes
    at VW = 3 and 4; N1 = 60 and 112 give 15 and 28 tile rows of 4 x1 rows, split
    over the 8 XCDs in slabs of 1 or 2 and 3 or 4 rows); with
    32-lane rows both with and without the x1 row shared by the two halves of a
    wave (N1 odd: the pairing stays off).  Each against the oracle on shooting,
    the gradient and the Hessian-vector product."""
    I0, I1 = images(n)
    v0 = random_velocity(n, 2003, 0.5, kc=2.0)  # coarse x0/x1 axes: keep the flow well resolved
    dv = random_field(n, 6, kc=3.0)
    p = O.Params(tuple(n), 0.01, 2, 6, 0.05)
    tr = O.shoot(v0, p, I0)
    go, lin = O.gradient(v0, I0, I1, p)
    ho = O.hessvec(dv, lin, p)
    hn = O.hessvec_newton(dv, lin, p)
    widths = [0] + [vw for vw in (1, 2, 3, 4) if n[2] % vw == 0 and 32 <= n[2] // vw <= 64]
    shapes = [(vw, pr) for vw in widths for pr in ((0, 1) if vw and n[2] // vw == 32 else (1,))]
    for rowvec, pair in shapes:
        R, _ = make(n, dtype, sigma2=0.05)
        R.set_option("stencil.rowvec", rowvec)
        R.set_option("stencil.pair_rows", pair)
        assert R.get_option("stencil.rowvec") == rowvec and R.get_option("stencil.pair_rows") == pair
        R.set_images(T(I0, dtype), T(I1, dtype))
        out = R.shoot(T(v0, dtype))
        g, E = R.gradient(T(v0, dtype))
        hv = R.hessvec(T(dv, dtype))
        hvn = R.hessvec(T(dv, dtype), newton=True)
        errs = dict(v1=rel(out["v1"], tr.v[-1]), J1=rel(out["J1"], tr.J1), grad=rel(g, go), hv=rel(hv, ho),
                    hv_newton=rel(hvn, hn))
        say(f"  rowvec={rowvec} pair_rows={pair}", errs)
        assert errs["v1"] <= TOL[dtype]["shoot"] and errs["J1"] <= TOL[dtype]["shoot"]
        assert errs["grad"] <= TOL[dtype]["grad"] and errs["hv"] <= TOL[dtype]["hv"]
        assert errs["hv_newton"] <= TOL[dtype]["hv"]
        assert E == pytest.approx(lin.E, rel=TOL[dtype]["shoot"])


# ------------------------------------------------------------------ full Newton Hessian
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", SMALL)
def test_hessvec_newton_parity(n, dtype):
    R, p = make(n, dtype, sigma2=0.05)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2002, 1.5, kc=2.0)
    dv = random_field(n, 5, kc=3.0)
    hv = R.hessvec(T(dv, dtype), v0=T(v0, dtype), newton=True)
    lin = O.linearize(v0, I0, I1, p)
    ho = O.hessvec_newton(dv, lin, p)
    e = rel(hv, ho)
    say(f"  newton hessvec rel {e:.3e}; differs from Gauss-Newton by {rel(ho, O.hessvec(dv, lin, p)):.3f}")
    assert e <= TOL[dtype]["hv"]
    # the recorded first-order adjoint is reused at the same linearization, bit for bit,
    # and the Gauss-Newton product is unaffected
    assert torch.equal(hv, R.hessvec(T(dv, dtype), newton=True))
    assert rel(R.hessvec(T(dv, dtype)), O.hessvec(dv, lin, p)) <= TOL[dtype]["hv"]


def test_hessvec_newton_zero_residual_is_gauss_newton():
    """I1 = J1(v0) on the device: lambda_1 and the first-order adjoint vanish."""
    n = (16, 12, 20)
    R, p = make(n, torch.float64, sigma2=0.05)
    I0, _ = images(n)
    v0 = T(random_velocity(n, 2002, 1.5, kc=2.0), torch.float64)
    dv = T(random_field(n, 5, kc=3.0), torch.float64)
    R.set_images(T(I0, torch.float64), T(I0, torch.float64))
    J1 = R.shoot(v0, want=("J1",))["J1"]
    R.set_images(T(I0, torch.float64), J1)
    hn = R.hessvec(dv, v0=v0, newton=True)
    hg = R.hessvec(dv)
    assert rel(hn, hg.cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("dtype", DTYPES)
def test_vjp_parity(dtype):
    n = (16, 12, 20)
    R, p = make(n, dtype)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2003, 1.5, kc=2.0)
    gbar = random_field(n, 6, components=1)[0]
    R.linearize(T(v0, dtype))
    got = R.vjp(T(gbar, dtype))
    lin = O.linearize(v0, I0, I1, p)
    assert rel(got, O.vjp_J1(gbar, lin, p)) <= TOL[dtype]["grad"]


# ------------------------------------------------------------------ a10: trajectory memory
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("every", [1, 2, 3, 5, -1])
def test_trajectory_policies_are_bitwise_store_all(dtype, every):
    """Checkpointing (c = 1, 2, 3, nt) and full recompute give bitwise the
    gradient, Hessian-vector product and vjp of the store-all run."""
    from paper_1807_04638_amd import Registration

    n, nt = (16, 12, 20), 5
    I0, I1 = images(n)
    v0 = T(random_velocity(n, 2005, 1.5, kc=2.0), dtype)
    dv = T(random_field(n, 9, kc=3.0), dtype)
    gbar = T(random_field(n, 10, components=1)[0], dtype)
    out = {}
    for ce in (0, every):
        say(f"[case] checkpoint_every={ce} dtype={dtype}")
        R = Registration(n, nt, 0.01, 2, 0.05, dtype=dtype, checkpoint_every=ce)
        R.set_images(T(I0, dtype), T(I1, dtype))
        expect = 0 if ce == 0 else (2 if ce < 0 else 1)
        assert R.get_option("traj.policy") == expect
        g, E = R.gradient(v0)
        hv = R.hessvec(dv)
        hv2 = R.hessvec(dv)
        vj = R.vjp(gbar)
        hn = R.hessvec(dv, newton=True)
        out[ce] = (g, E, hv, hv2, vj, R.get_option("traj.bytes"), hn)
    a, b = out[0], out[every]
    assert torch.equal(a[0], b[0]) and a[1] == b[1]
    assert torch.equal(a[2], b[2]) and torch.equal(b[2], b[3])
    assert torch.equal(a[4], b[4])
    assert torch.equal(a[6], b[6])
    assert b[5] < a[5]


def test_trajectory_policy_from_memory_budget():
    from paper_1807_04638_amd import Registration

    n, nt = (32, 32, 32), 8
    full = Registration(n, nt, 0.01, dtype=torch.float32)
    V = 3 * 32**3 * 4
    need = full.memory_bytes()
    assert full.get_option("traj.policy") == 0 and full.get_option("traj.bytes") == (4 * nt + 2) * V
    tight = Registration(n, nt, 0.01, dtype=torch.float32, mem_budget_bytes=need - 10 * V)
    assert tight.get_option("traj.policy") == 1
    c = tight.get_option("traj.every")
    assert tight.memory_bytes() <= need - 10 * V and 1 <= c < nt
    tiny = Registration(n, nt, 0.01, dtype=torch.float32, mem_budget_bytes=1)
    assert tiny.get_option("traj.policy") == 2 and tiny.get_option("traj.bytes") == 7 * V


# ------------------------------------------------------------------ a8: CG in V
@pytest.mark.parametrize("dtype", DTYPES)
def test_cg_parity(dtype):
    n = (16, 12, 20)
    R, p = make(n, dtype, sigma2=0.05)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2004, 1.0, kc=2.0)
    g, _ = R.gradient(T(v0, dtype))
    go, lin = O.gradient(v0, I0, I1, p)
    x, its = R.cg_solve(g, 0.05, 6)
    xo, its_o = O.cg_v(lambda d: O.hessvec(d, lin, p), g.double().cpu().numpy(), p, 0.05, 6)
    say(f"  cg its {its} vs {its_o}  rel {rel(x, xo):.3e}")
    assert its == its_o
    assert rel(x, xo) <= (1e-10 if dtype == torch.float64 else 1e-4)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [(32, 32, 32), (16, 12, 20)])
@pytest.mark.parametrize("nt", [1, 2])
def test_short_horizons(nt, n, dtype):
    """nt = 1 and 2: the adjoint sweep's first stage (w = 0, taken as the EPDiff
    operator with -dt and dt K U) is also its last (the one that writes 2 v + w_0
    or 2 dv + w_0); the tangent sweep's first stage is also the one that writes
    the GN final condition.  Gradient, Hv and CG (which hands its tracked L d to
    the Hv) against the oracle, on the row-vectorised (32^3) and one-voxel (N2 =
    20) stencil paths."""
    R, p = make(n, dtype, nt=nt, sigma2=0.05)
    I0, I1 = images(n)
    R.set_images(T(I0, dtype), T(I1, dtype))
    v0 = random_velocity(n, 2005, 1.0, kc=2.0)
    g, _ = R.gradient(T(v0, dtype))
    go, lin = O.gradient(v0, I0, I1, p)
    dv = random_field(n, 6, kc=3.0)
    hv = R.hessvec(T(dv, dtype))
    x, its = R.cg_solve(g, 0.05, 5)
    xo, its_o = O.cg_v(lambda d: O.hessvec(d, lin, p), g.double().cpu().numpy(), p, 0.05, 5)
    errs = dict(grad=rel(g, go), hv=rel(hv, O.hessvec(dv, lin, p)), cg=rel(x, xo))
    say(f"  nt={nt} rowvec={R.get_option('stencil.rowvec')} its {its} vs {its_o}", errs)
    assert errs["grad"] <= TOL[dtype]["grad"] and errs["hv"] <= TOL[dtype]["hv"]
    assert its == its_o
    assert errs["cg"] <= (1e-10 if dtype == torch.float64 else 1e-4)


# ------------------------------------------------------------------ a9: GN loop
def test_gn_solve_parity_fp64():
    n = (16, 16, 16)
    R, p = make(n, torch.float64, nt=5, sigma2=0.02)
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000)
    vt = random_velocity(n, 2100, 1.0, kc=2.0)
    I1 = O.shoot(vt, p, I0).J1
    R.set_images(T(I0, torch.float64), T(I1, torch.float64))
    v = torch.zeros((3,) + n, dtype=torch.float64, device=DEV)
    tr = R.gn_solve(v, gn_iters=3, cg_iters=6)
    vo, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=6)
    say("  gpu", tr.report, "\n  oracle", [(it.E, it.cg_iters, it.tau) for it in log])
    assert len(tr.log) == len(log)
    for a, b in zip(tr.log, log):
        assert a["cg_iters"] == b.cg_iters and a["tau"] == b.tau
        assert a["E"] == pytest.approx(b.E, rel=1e-10)
        assert a["mse_rel"] == pytest.approx(b.mse_rel, rel=1e-9)
        assert a["g_inf_rel"] == pytest.approx(b.g_inf_rel, rel=1e-9)
        assert a["g_norm"] == pytest.approx(b.g_norm, rel=1e-9)
    assert tr.report["E_final"] == pytest.approx(lin.E, rel=1e-10)
    assert rel(v, vo) <= 1e-9


def _variant_case():
    n = (16, 16, 16)
    p = O.Params(n, 0.01, 2, 5, 0.02)
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000)
    I1 = O.shoot(random_velocity(n, 2100, 1.0, kc=2.0), p, I0).J1
    return n, p, I0, I1


@pytest.mark.parametrize("method", ["gn_l2", "gd", "newton"])
def test_solver_variants_parity_fp64(method):
    """Gauss-Newton with PCG in L2 (preconditioner K, L2 norms) and gradient descent
    in V against the oracle's literal implementations, iteration by iteration."""
    n, p, I0, I1 = _variant_case()
    R, _ = make(n, torch.float64, nt=5, sigma2=0.02)
    R.set_images(T(I0, torch.float64), T(I1, torch.float64))
    v = torch.zeros((3,) + n, dtype=torch.float64, device=DEV)
    if method == "gn_l2":
        tr = R.gn_solve(v, gn_iters=3, cg_iters=6, method="gn_l2")
        vo, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=6, space="L2")
    elif method == "newton":
        tr = R.gn_solve(v, gn_iters=3, cg_iters=6, method="newton")
        vo, log, lin = O.gn_solve(I0, I1, p, gn_iters=3, cg_iters=6, hessian="newton")
    else:
        tr = R.gn_solve(v, gn_iters=6, method="gd")
        vo, log, lin = O.gd_solve(I0, I1, p, iters=6)
    say(f"  {method} gpu", tr.report, "\n  oracle", [(it.E, it.cg_iters, it.tau) for it in log])
    assert len(tr.log) == len(log) >= 2
    for a, b in zip(tr.log, log):
        assert a["cg_iters"] == b.cg_iters and a["tau"] == b.tau
        assert a["E"] == pytest.approx(b.E, rel=1e-10)
        assert a["mse_rel"] == pytest.approx(b.mse_rel, rel=1e-9)
        assert a["g_norm"] == pytest.approx(b.g_norm, rel=1e-9)
        assert a["g_inf_rel"] == pytest.approx(b.g_inf_rel, rel=1e-9)
    assert tr.report["E_final"] == pytest.approx(lin.E, rel=1e-10)
    assert rel(v, vo) <= 1e-9
    if method == "gd":
        assert tr.report["cg_total"] == 0 and tr.report["hessvecs"] == 0


@pytest.mark.parametrize("method", ["gn_v", "gn_l2", "gd", "newton"])
def test_solver_variants_fp32(method):
    """FP32 fields with FP64 reductions: each method decreases the energy and ends
    within 1e-3 of its FP64 run."""
    n, p, I0, I1 = _variant_case()
    out = {}
    for dtype in DTYPES:
        R, _ = make(n, dtype, nt=5, sigma2=0.02)
        R.set_images(T(I0, dtype), T(I1, dtype))
        v = torch.zeros((3,) + n, dtype=dtype, device=DEV)
        out[dtype] = R.gn_solve(v, gn_iters=4 if method != "gd" else 8, cg_iters=6, method=method).report
    a, b = out[torch.float32], out[torch.float64]
    say(f"  {method}", a, b)
    assert a["E_final"] < a["E_first"]
    assert a["E_final"] == pytest.approx(b["E_final"], rel=1e-3)


def test_gn_solve_fp32_reaches_fp64_energy():
    n = (16, 16, 16)
    I0 = phantom(n, 4, (1.5, 3.0), False, 1000)
    p = O.Params(n, 0.01, 2, 5, 0.02)
    I1 = O.shoot(random_velocity(n, 2100, 1.0, kc=2.0), p, I0).J1
    out = {}
    for dtype in DTYPES:
        R, _ = make(n, dtype, nt=5, sigma2=0.02)
        R.set_images(T(I0, dtype), T(I1, dtype))
        v = torch.zeros((3,) + n, dtype=dtype, device=DEV)
        out[dtype] = R.gn_solve(v, gn_iters=4, cg_iters=6).report
    a, b = out[torch.float32], out[torch.float64]
    assert a["E_final"] == pytest.approx(b["E_final"], rel=1e-3)
    assert a["E_final"] < a["E_first"]


# ------------------------------------------------------------------ metrics / errors
@pytest.mark.parametrize("dtype", DTYPES)
def test_jacobian_det_parity(dtype):
    n = (16, 12, 20)
    R, p = make(n, dtype)
    u = 0.1 * random_field(n, 7, kc=2.0)
    det, mn, mx = R.jacobian_det(T(u, dtype))
    ref = O.jacobian_det(u, p)
    assert rel(det, ref) <= (1e-13 if dtype == torch.float64 else 1e-6)
    assert mn == pytest.approx(ref.min(), rel=1e-5) and mx == pytest.approx(ref.max(), rel=1e-5)


def test_error_paths():
    from paper_1807_04638_amd import LddmmError, Registration

    n = (16, 12, 20)
    R, p = make(n, torch.float32)
    v = torch.zeros((3,) + n, device=DEV)
    with pytest.raises(LddmmError) as e:
        R.hessvec(v)  # no linearization yet
    assert e.value.status == -6
    I0, I1 = images(n)
    R.set_images(T(I0, torch.float32), T(I1, torch.float32))
    bad = v.clone()
    bad[1, 3, 4, 5] = float("nan")
    with pytest.raises(LddmmError) as e:
        R.gradient(bad)
    assert e.value.status == -5
    with pytest.raises(LddmmError) as e:
        Registration((16, 22, 20), 4, 0.01)
    assert e.value.status == -2
    with pytest.raises(ValueError):
        R.gradient(torch.zeros((3, 16, 12, 21), device=DEV))
    from paper_1807_04638_amd.lddmm import SolveOpts

    import ctypes

    bad_opts = SolveOpts(2, 2, 2, 7, 1e-4, 1e-3, 0.5)  # unknown method
    rc = R.lib.lddmm_gn_solve(R._ctx, ctypes.c_void_p(v.data_ptr()), ctypes.byref(bad_opts), None, None, 0)
    assert rc == -1
    for width in (1, 3, 5):  # N2 = 20: no row-vectorised width; 5 is never one
        with pytest.raises(LddmmError) as e:
            R.set_option("stencil.rowvec", width)
        assert e.value.status == -1
    assert R.get_option("stencil.rowvec") == 0
    for bad in (-1, 2):
        with pytest.raises(LddmmError) as e:
            R.set_option("stencil.pair_rows", bad)
        assert e.value.status == -1
    for bad in (-1, 70000):
        with pytest.raises(LddmmError) as e:
            R.set_option("fft.plane_grid", bad)
        assert e.value.status == -1


# ------------------------------------------------------------------ full size (128^3, nt = 10)
FULL = (128, 128, 128)


def full_case(dtype):
    """The benchmark's workload size and launch configuration: the context is
    autotuned as bench.py does before it times the solve."""
    R, p = make(FULL, dtype, nt=10, alpha=0.0025, s=2, sigma2=1.0)
    I0 = phantom(FULL, 24, (4.0, 12.0), True, 1000)
    I1 = phantom(FULL, 24, (4.0, 12.0), True, 1001)
    R.set_images(T(I0, dtype), T(I1, dtype))
    R.autotune(reps=5)
    keys = ("fft.plane_threads", "fft.pencil_tb", "fft.plane_halves_used", "fft.plane_walk", "stencil.rowvec",
            "stencil.pair_rows")
    say(f"  launch shape after autotune: { {k: R.get_option(k) for k in keys} }")
    return R, p, I0, I1


def test_full_size_operator_parity():
    R, p, _, _ = full_case(torch.float32)
    f = rounded(random_field(FULL, 8), torch.float32)
    Lf = O.apply_L(f, p)
    eK, eL = rel(R.apply_K(T(f, torch.float32)), O.apply_K(f, p)), rel(R.apply_L(T(f, torch.float32)), Lf)
    say(f"  K rel {eK:.3e}  L rel {eL:.3e} (tol {l_tol(p, f, Lf, torch.float32):.1e})")
    assert eK <= 2e-6
    assert eL <= l_tol(p, f, Lf, torch.float32)


def test_full_size_v0_zero_closed_forms():
    """At v0 = 0: g = -(2/s2) K((I0 - I1) grad I0), H dv = 2 dv + (2/s2) K[(grad I0 . dv) grad I0]."""
    R, p, I0, I1 = full_case(torch.float32)
    z = torch.zeros((3,) + FULL, device=DEV)
    g, _ = R.gradient(z)
    gI0 = O.grad(I0, p)
    ref_g = -(2.0 / p.sigma2) * O.apply_K((I0 - I1)[None] * gI0, p)
    assert rel(g, ref_g) <= 1e-4
    dv = random_field(FULL, 9)
    hv = R.hessvec(T(dv, torch.float32))
    ref_h = 2 * dv + (2.0 / p.sigma2) * O.apply_K(np.sum(gI0 * dv, axis=0)[None] * gI0, p)
    assert rel(hv, ref_h) <= 1e-4


def test_full_size_fp32_vs_fp64_and_hessian_properties():
    v0 = random_velocity(FULL, 2000, 6.0)
    a, b = random_field(FULL, 10), random_field(FULL, 11)
    res = {}
    for dtype in DTYPES:
        R, p, _, _ = full_case(dtype)
        tv = T(v0, dtype)
        sh = R.shoot(tv)
        g, E = R.gradient(tv)
        ta, tb = T(a, dtype), T(b, dtype)
        Ha, Hb = R.hessvec(ta), R.hessvec(tb)
        La, Lb = R.apply_L(ta), R.apply_L(tb)
        res[dtype] = dict(J1=sh["J1"].double().cpu(), v1=sh["v1"].double().cpu(), g=g.double().cpu(),
                          Ha=Ha.double().cpu(), E=E, aHb=R.dot(La, Hb), Hab=R.dot(Ha, Lb),
                          aHa=R.dot(La, Ha), aa=R.dot(La, ta))
        say(f"  {dtype} symmetry {res[dtype]['aHb']} {res[dtype]['Hab']} rayleigh {res[dtype]['aHa'] / res[dtype]['aa']}")
        sym_tol = 1e-11 if dtype == torch.float64 else 1e-4
        assert abs(res[dtype]["aHb"] - res[dtype]["Hab"]) <= sym_tol * abs(res[dtype]["aHb"])
        assert res[dtype]["aHa"] >= 2.0 * res[dtype]["aa"] * (1 - sym_tol)
        del R
        torch.cuda.empty_cache()
    f32, f64 = res[torch.float32], res[torch.float64]
    errs = {k: rel(f32[k].numpy(), f64[k].numpy()) for k in ("J1", "v1", "g", "Ha")}
    say("  fp32 vs fp64", errs)
    assert errs["J1"] <= 1e-5 and errs["v1"] <= 1e-5
    assert errs["g"] <= 1e-4 and errs["Ha"] <= 1e-4
    assert f32["E"] == pytest.approx(f64["E"], rel=1e-5)


def test_deterministic_repeat():
    R, p, _, _ = full_case(torch.float32)
    dv = T(random_field(FULL, 12), torch.float32)
    R.linearize(T(random_velocity(FULL, 2000, 6.0), torch.float32))
    assert torch.equal(R.hessvec(dv), R.hessvec(dv))
