"""The context-free, allocation-free K / L application
(lddmm_apply_operator_noalloc, for callers that cannot allocate device memory)
against the context entry point lddmm_apply_operator, through the C ABI.

Both run the same kernels with the same default launch shapes, so the results
are compared bitwise; the oracle bounds both.  Two calls in a row, the second
on a smaller input; then a grid too large for the static workspace is refused
with a message and no launch."""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from synth import random_field

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def T(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def noalloc(lib, B, n, dtype, alpha, s, op, f, out, stream):
    nn = (ctypes.c_int32 * 3)(*n)
    ncomp = 3 if f.dim() == 4 else 1
    return lib.lddmm_apply_operator_noalloc(
        nn, B.F32 if dtype == torch.float32 else B.F64, alpha, s, op, ncomp, ctypes.c_void_p(f.data_ptr()),
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream.cuda_stream))


def context_apply(lib, B, n, dtype, alpha, s, op, f, out, stream):
    p = B.Params()
    p.n = (ctypes.c_int32 * 3)(*n)
    p.nt, p.s, p.dtype, p.alpha, p.sigma2 = 1, s, (B.F32 if dtype == torch.float32 else B.F64), alpha, 1.0
    ctx = ctypes.c_void_p()
    assert lib.lddmm_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx)) == 0
    ncomp = 3 if f.dim() == 4 else 1
    rc = lib.lddmm_apply_operator(ctx, op, ncomp, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert lib.lddmm_sync(ctx) == 0
    lib.lddmm_destroy(ctx)
    return rc


CASES = [
    # (grid, components, alpha, op): the second of each dtype's pair is smaller
    ((128, 128, 128), 3, 0.0025, 0),
    ((24, 20, 30), 1, 0.01, 1),
]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_context_entry_point(dtype):
    from paper_1807_04638_amd import lddmm as B

    lib = B.load_library()
    st = torch.cuda.Stream(device=DEV)
    for i, (n, ncomp, alpha, op) in enumerate(CASES):
        say(f"[case] noalloc {dtype} call {i}: n={n} ncomp={ncomp} op={'KL'[op]}")
        shape = (3,) + n if ncomp == 3 else n
        f64 = random_field(n, 40 + i, kc=max(n) / 4)
        f = T(f64 if ncomp == 3 else f64[0], dtype)
        assert f.shape == shape
        torch.cuda.synchronize()
        a = torch.full_like(f, float("nan"))
        b = torch.full_like(f, float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            assert noalloc(lib, B, n, dtype, alpha, 2, op, f, a, st) == 0, lib.lddmm_last_error(None)
        st.synchronize()
        assert context_apply(lib, B, n, dtype, alpha, 2, op, f, b, st) == 0
        st.synchronize()
        assert torch.equal(a, b), float((a - b).abs().max())
        p = O.Params(tuple(n), alpha, 2, 1)
        ref = (O.apply_K if op == 0 else O.apply_L)(f.double().cpu().numpy(), p)
        err = float(np.linalg.norm(a.double().cpu().numpy() - ref) / np.linalg.norm(ref))
        tol = (1e-12 if dtype == torch.float64 else 2e-6) if op == 0 else (1e-10 if dtype == torch.float64 else 5e-5)
        say(f"  bitwise equal to the context entry point; rel-L2 vs oracle {err:.2e} (tol {tol:g})")
        assert err <= tol
    # in place (in == out) on the smaller grid, after the larger one
    n, ncomp, alpha, op = CASES[1]
    f = T(random_field(n, 50, kc=4.0)[0], dtype)
    ref = (O.apply_K if op == 0 else O.apply_L)(f.double().cpu().numpy(), O.Params(tuple(n), alpha, 2, 1))
    g = f.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        assert noalloc(lib, B, n, dtype, alpha, 2, op, g, g, st) == 0
    st.synchronize()
    assert np.linalg.norm(g.double().cpu().numpy() - ref) / np.linalg.norm(ref) <= (1e-10 if dtype == torch.float64 else 5e-5)


def test_noalloc_rejects_grids_beyond_the_workspace():
    from paper_1807_04638_amd import lddmm as B

    lib = B.load_library()
    n = (256, 256, 256)
    st = torch.cuda.Stream(device=DEV)
    f = torch.zeros((3,) + n, dtype=torch.float32, device=DEV)
    say("[case] noalloc refuses 256^3 vector FP32")
    rc = noalloc(lib, B, n, torch.float32, 0.0025, 2, 0, f, f, st)
    msg = lib.lddmm_last_error(None).decode()
    say(f"  status {rc}: {msg}")
    assert rc == B.EUNSUPPORTED and "static workspace" in msg
    st.synchronize()
    assert int(torch.count_nonzero(f)) == 0
    # the binding raises with the same message
    with pytest.raises(B.LddmmError, match="static workspace"):
        B.apply_operator_noalloc(B.OP_K, f, 0.0025)
