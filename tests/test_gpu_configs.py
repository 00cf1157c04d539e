"""GPU against the FP64 oracle on the benchmark workloads themselves.

* 32^3 plain-method workload (6-blob phantom in an ellipsoidal shell, target shot
  by a band-limited v0 of ~2 voxels plus N(0, 0.01^2) noise, alpha = 0.01, s = 2,
  nt = 10, sigma^2 = 1, GN <= 10, CG <= 20): the whole Gauss-Newton solve in FP64,
  iteration by iteration, in V and in L2.
* 128^3 workload (24 tissue-class blobs, alpha = 0.0025, s = 2, nt = 10): shoot,
  gradient and Gauss-Newton Hv at a nonzero v0 (max 6 voxels) in both precisions,
  in the autotuned launch configuration the benchmark times; the relative L2
  error of each result against the oracle is printed and bounded by 1e-5
  (shooting outputs) and 1e-4 (gradient, Hv) in FP32, 1e-11 in FP64.
* 180x216x180 head workload (three shells, 40 tissue-class blobs, alpha =
  0.0025, s = 2) at its full grid in its autotuned launch configuration, with
  nt = 2 and a v0 of 2 voxels (one voxel per step, as the workload's 8 voxels
  over nt = 16 take half a voxel; nt = 2 still runs the first-stage and the
  regular kernel variants of both sweeps and keeps the host oracle near a
  minute): the same results and bounds.
* 256^3 memory workload (48 tissue-class blobs, alpha = 0.0025, s = 2) at its
  full grid in the launch configuration its benchmark times (the default shape:
  half-plane units in FP32, the split transform in FP64), with nt = 3 and a v0
  of 3 voxels: the same results and bounds, in FP32 under each trajectory
  policy (store-all, checkpoints every 2 steps with a ragged last segment, full
  recompute; bitwise the same Hv and gradient) and in FP64.
"""

import numpy as np
import pytest
import torch

import oracle as O
import synth
from synth import phantom, random_field, random_velocity

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a = np.asarray(a.detach().double().cpu() if torch.is_tensor(a) else a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def T(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


# ------------------------------------------------------------------ 32^3, FP64, whole solve
def pair32():
    spec = synth.WORKLOADS["pair32"]
    p = O.Params(spec.n, spec.alpha, spec.s, spec.nt, spec.sigma2)
    I0 = phantom(spec.n, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    vt = random_velocity(spec.n, 2000, spec.disp_vox)
    I1 = O.shoot(vt, p, I0).J1 + synth.noise(spec.n, 3000, spec.noise_sd)
    return spec, p, I0, I1


@pytest.mark.parametrize("method", ["gn_v", "gn_l2"])
def test_pair32_gn_solve_fp64_iteration_by_iteration(method):
    from paper_1807_04638_amd import Registration

    spec, p, I0, I1 = pair32()
    say(f"[case] pair32 {method} FP64, GN <= {spec.gn_iters}, CG <= {spec.cg_iters}")
    R = Registration(spec.n, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=torch.float64)
    R.set_images(T(I0, torch.float64), T(I1, torch.float64))
    v = torch.zeros((3,) + spec.n, dtype=torch.float64, device=DEV)
    tr = R.gn_solve(v, gn_iters=spec.gn_iters, cg_iters=spec.cg_iters, method=method)
    vo, log, lin = O.gn_solve(I0, I1, p, gn_iters=spec.gn_iters, cg_iters=spec.cg_iters,
                              space="V" if method == "gn_v" else "L2")
    say("  gpu   ", [(round(a["E"], 12), a["cg_iters"], a["tau"]) for a in tr.log], tr.report["stop_reason"])
    say("  oracle", [(round(b.E, 12), b.cg_iters, b.tau) for b in log])
    assert len(tr.log) == len(log) >= 3
    for a, b in zip(tr.log, log):
        assert a["cg_iters"] == b.cg_iters and a["tau"] == b.tau
        for key in ("E", "E_reg", "E_data"):
            assert a[key] == pytest.approx(getattr(b, key), rel=1e-10, abs=1e-15)
        assert a["mse_rel"] == pytest.approx(b.mse_rel, rel=1e-9)
        assert a["g_norm"] == pytest.approx(b.g_norm, rel=1e-9)
        assert a["g_inf_rel"] == pytest.approx(b.g_inf_rel, rel=1e-9)
        assert a["eta"] == pytest.approx(b.eta, rel=1e-9)
    assert tr.report["E_final"] == pytest.approx(lin.E, rel=1e-10)
    assert tr.report["mse_rel_final"] == pytest.approx(O.mse_rel(lin.tr.J1, I0, I1, p), rel=1e-9)
    err = rel(v, vo)
    say(f"  final v0 rel-L2 vs oracle {err:.2e}")
    assert err <= 1e-9


# ------------------------------------------------------------------ 128^3, nt = 10, nonzero v0
FULL = (128, 128, 128)


@pytest.fixture(scope="module")
def full_oracle():
    spec = synth.WORKLOADS["pair128"]
    p = O.Params(FULL, spec.alpha, spec.s, spec.nt, spec.sigma2)
    I0 = phantom(FULL, spec.n_blobs, spec.sigma_range, spec.classes, 1000)
    I1 = phantom(FULL, spec.n_blobs, spec.sigma_range, spec.classes, 1001)
    v0 = random_velocity(FULL, 2000, spec.disp_vox)
    dv = random_field(FULL, 12)
    say("[case] oracle at 128^3, nt=10: linearization, gradient, Hv")
    lin = O.linearize(v0, I0, I1, p)
    g, _ = O.gradient(v0, I0, I1, p, lin)
    hv = O.hessvec(dv, lin, p)
    return dict(spec=spec, p=p, I0=I0, I1=I1, v0=v0, dv=dv, J1=lin.tr.J1, u1=lin.tr.u, v1=lin.tr.v[-1], E=lin.E,
                g=g, hv=hv)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_full_size_nonzero_v0_vs_oracle(full_oracle, dtype):
    from paper_1807_04638_amd import Registration

    o = full_oracle
    spec = o["spec"]
    say(f"[case] 128^3 nt=10 nonzero v0, {dtype}")
    R = Registration(FULL, spec.nt, spec.alpha, spec.s, spec.sigma2, dtype=dtype)
    R.set_images(T(o["I0"], dtype), T(o["I1"], dtype))
    R.autotune(reps=5)
    R.set_option("exec.graph", 0)
    tv = T(o["v0"], dtype)
    sh = R.shoot(tv, energy=True)
    g, E = R.gradient(tv)
    hv = R.hessvec(T(o["dv"], dtype))
    errs = dict(J1=rel(sh["J1"], o["J1"]), u1=rel(sh["u1"], o["u1"]), v1=rel(sh["v1"], o["v1"]),
                gradient=rel(g, o["g"]), hessvec=rel(hv, o["hv"]), energy=abs(E - o["E"]) / abs(o["E"]))
    say("  rel-L2 vs FP64 oracle:", {k: f"{v:.2e}" for k, v in errs.items()})
    if dtype == torch.float32:
        tol = dict(J1=1e-5, u1=1e-5, v1=1e-5, gradient=1e-4, hessvec=1e-4, energy=1e-5)
    else:
        tol = dict(J1=1e-11, u1=1e-11, v1=1e-11, gradient=1e-11, hessvec=1e-11, energy=1e-12)
    for k, e in errs.items():
        assert e <= tol[k], (k, e, tol[k])
    R.close()


# ------------------------------------------------------------------ 180x216x180, nt = 2, nonzero v0
HEAD = (180, 216, 180)


@pytest.fixture(scope="module")
def head_oracle():
    spec = synth.WORKLOADS["head180x216x180"]
    p = O.Params(HEAD, spec.alpha, spec.s, 2, spec.sigma2)
    I0 = phantom(HEAD, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    I1 = phantom(HEAD, spec.n_blobs, spec.sigma_range, spec.classes, 1001, shells=spec.shells)
    v0 = random_velocity(HEAD, 2000, 2.0)
    dv = random_field(HEAD, 12)
    say("[case] oracle at 180x216x180, nt=2: linearization")
    lin = O.linearize(v0, I0, I1, p)
    say("[case] oracle at 180x216x180, nt=2: gradient")
    g, _ = O.gradient(v0, I0, I1, p, lin)
    say("[case] oracle at 180x216x180, nt=2: Hv")
    hv = O.hessvec(dv, lin, p)
    return dict(spec=spec, p=p, I0=I0, I1=I1, v0=v0, dv=dv, J1=lin.tr.J1, u1=lin.tr.u, v1=lin.tr.v[-1], E=lin.E,
                g=g, hv=hv)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_head_grid_nonzero_v0_vs_oracle(head_oracle, dtype):
    from paper_1807_04638_amd import Registration

    o = head_oracle
    p = o["p"]
    say(f"[case] 180x216x180 nt=2 nonzero v0, {dtype}")
    R = Registration(HEAD, p.nt, p.alpha, p.s, p.sigma2, dtype=dtype)
    R.set_images(T(o["I0"], dtype), T(o["I1"], dtype))
    R.autotune(reps=3)
    say("  shape", {k: R.get_option(k) for k in ("fft.plane_threads", "fft.plane_halves_used", "fft.pencil_tb",
                                                  "stencil.rowvec", "stencil.pair_rows")})
    R.set_option("exec.graph", 0)
    tv = T(o["v0"], dtype)
    sh = R.shoot(tv, energy=True)
    g, E = R.gradient(tv)
    hv = R.hessvec(T(o["dv"], dtype))
    errs = dict(J1=rel(sh["J1"], o["J1"]), u1=rel(sh["u1"], o["u1"]), v1=rel(sh["v1"], o["v1"]),
                gradient=rel(g, o["g"]), hessvec=rel(hv, o["hv"]), energy=abs(E - o["E"]) / abs(o["E"]))
    say("  rel-L2 vs FP64 oracle:", {k: f"{v:.2e}" for k, v in errs.items()})
    if dtype == torch.float32:
        tol = dict(J1=1e-5, u1=1e-5, v1=1e-5, gradient=1e-4, hessvec=1e-4, energy=1e-5)
    else:
        tol = dict(J1=1e-11, u1=1e-11, v1=1e-11, gradient=1e-11, hessvec=1e-11, energy=1e-12)
    for k, e in errs.items():
        assert e <= tol[k], (k, e, tol[k])
    R.close()


# ------------------------------------------------------------------ 256^3, nt = 3, trajectory policies
BIG = (256, 256, 256)


@pytest.fixture(scope="module")
def big_oracle():
    spec = synth.WORKLOADS["pair256"]
    p = O.Params(BIG, spec.alpha, spec.s, 3, spec.sigma2)
    I0 = phantom(BIG, spec.n_blobs, spec.sigma_range, spec.classes, 1000, shells=spec.shells)
    I1 = phantom(BIG, spec.n_blobs, spec.sigma_range, spec.classes, 1001, shells=spec.shells)
    v0 = random_velocity(BIG, 2000, 3.0)
    dv = random_field(BIG, 12)
    say("[case] oracle at 256^3, nt=3: linearization")
    lin = O.linearize(v0, I0, I1, p)
    say("[case] oracle at 256^3, nt=3: gradient")
    g, _ = O.gradient(v0, I0, I1, p, lin)
    say("[case] oracle at 256^3, nt=3: Hv")
    hv = O.hessvec(dv, lin, p)
    return dict(p=p, I0=I0, I1=I1, v0=v0, dv=dv, J1=lin.tr.J1, u1=lin.tr.u, v1=lin.tr.v[-1], E=lin.E, g=g, hv=hv)


def test_pair256_policies_vs_oracle(big_oracle):
    from paper_1807_04638_amd import Registration

    o = big_oracle
    p = o["p"]
    tol32 = dict(J1=1e-5, u1=1e-5, v1=1e-5, gradient=1e-4, hessvec=1e-4, energy=1e-5)
    tol64 = dict(J1=1e-11, u1=1e-11, v1=1e-11, gradient=1e-11, hessvec=1e-11, energy=1e-12)
    first = None
    for dtype, every in ((torch.float32, 0), (torch.float32, 2), (torch.float32, -1), (torch.float64, 0)):
        say(f"[case] 256^3 nt=3 nonzero v0, {dtype}, checkpoint_every={every}")
        R = Registration(BIG, p.nt, p.alpha, p.s, p.sigma2, dtype=dtype, checkpoint_every=every)
        R.set_images(T(o["I0"], dtype), T(o["I1"], dtype))
        say("  shape", {k: R.get_option(k) for k in ("fft.fused", "fft.plane_halves_used", "stencil.rowvec",
                                                      "stencil.pair_rows")}, "traj bytes", R.get_option("traj.bytes"))
        tv = T(o["v0"], dtype)
        sh = R.shoot(tv, energy=True)
        g, E = R.gradient(tv)
        hv = R.hessvec(T(o["dv"], dtype))
        errs = dict(J1=rel(sh["J1"], o["J1"]), u1=rel(sh["u1"], o["u1"]), v1=rel(sh["v1"], o["v1"]),
                    gradient=rel(g, o["g"]), hessvec=rel(hv, o["hv"]), energy=abs(E - o["E"]) / abs(o["E"]))
        say("  rel-L2 vs FP64 oracle:", {k: f"{v:.2e}" for k, v in errs.items()})
        tol = tol32 if dtype == torch.float32 else tol64
        for k, e in errs.items():
            assert e <= tol[k], (k, e, tol[k])
        if dtype == torch.float32:
            if first is None:
                first = (g.clone(), hv.clone())
            else:  # the trajectory policy changes what is stored, not what is computed
                assert torch.equal(g, first[0]) and torch.equal(hv, first[1])
        R.close()
        del R, sh, g, hv, tv
        torch.cuda.empty_cache()
