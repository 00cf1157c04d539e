"""CPU checks of the C ABI: the built library exports every function that
include/lddmm.h declares, the ctypes mirror of the structs has the C layout,
and argument validation of lddmm_create rejects bad parameters before any
device call (so these run without a GPU)."""

import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lddmm.h")
LIB = os.path.join(ROOT, "paper_1807_04638_amd", "liblddmm.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lddmm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblddmm.so is not built: run __graft_entry__.build()")
    from paper_1807_04638_amd import lddmm as B

    return B.load_library()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("lddmm_create", "lddmm_shoot", "lddmm_gradient", "lddmm_hessvec", "lddmm_gn_solve"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    nm = shutil.which("nm")
    if nm:
        out = subprocess.run([nm, "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
        exported = set(re.findall(r"\sT\s(lddmm_\w+)", out))
        assert set(declared_functions()) <= exported, set(declared_functions()) - exported
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1807_04638_amd import lddmm as B

    assert set(declared_functions()) == set(B.SIGNATURES)


def test_struct_layouts_match_c(tmp_path):
    cc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cc):
        pytest.skip("hipcc not available")
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lddmm.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %d %d %d %d\\n\", sizeof(lddmm_params),"
        " sizeof(lddmm_solve_opts), sizeof(lddmm_iter_log), sizeof(lddmm_solve_report), offsetof(lddmm_params, alpha),"
        " offsetof(lddmm_params, mem_budget_bytes), offsetof(lddmm_solve_report, E_first),"
        " offsetof(lddmm_solve_opts, method), offsetof(lddmm_iter_log, g_norm), LDDMM_GN_V, LDDMM_GN_L2, LDDMM_GD_V,"
        " LDDMM_NEWTON_V);"
        " return 0;}\n"
    )
    exe = tmp_path / "sizes"
    gcc = shutil.which("gcc") or shutil.which("cc")
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    from paper_1807_04638_amd import lddmm as B

    expect = [
        ctypes.sizeof(B.Params),
        ctypes.sizeof(B.SolveOpts),
        ctypes.sizeof(B.IterLog),
        ctypes.sizeof(B.SolveReport),
        B.Params.alpha.offset,
        B.Params.mem_budget_bytes.offset,
        B.SolveReport.E_first.offset,
        B.SolveOpts.method.offset,
        B.IterLog.g_norm.offset,
        B.METHODS["gn_v"],
        B.METHODS["gn_l2"],
        B.METHODS["gd"],
        B.METHODS["newton"],
    ]
    assert got == expect


def _create(lib, n=(32, 32, 32), nt=10, s=2, alpha=0.01, sigma2=1.0, dtype=0):
    from paper_1807_04638_amd import lddmm as B

    p = B.Params()
    p.n = (ctypes.c_int32 * 3)(*n)
    p.nt, p.s, p.dtype, p.alpha, p.sigma2 = nt, s, dtype, alpha, sigma2
    ctx = ctypes.c_void_p()
    return lib.lddmm_create(ctypes.byref(p), None, ctypes.byref(ctx)), ctx


@pytest.mark.parametrize(
    "kw, status",
    [
        (dict(n=(11, 32, 32)), -2),  # prime factor 11
        (dict(n=(32, 32, 33)), -2),  # odd N2
        (dict(n=(2, 32, 32)), -2),  # below the minimum size
        (dict(n=(0, 32, 32)), -2),  # empty grid
        (dict(n=(32, -8, 32)), -2),  # negative extent
        (dict(n=(1024, 1024, 1024)), -2),  # 3 N beyond a 32-bit index
        (dict(n=(32, 26, 32)), -2),  # 26 = 2 * 13
        (dict(nt=0), -1),
        (dict(s=0), -1),
        (dict(alpha=0.0), -1),
        (dict(sigma2=-1.0), -1),
        (dict(dtype=7), -1),
    ],
)
def test_create_rejects_bad_params_without_touching_the_device(lib, kw, status):
    rc, ctx = _create(lib, **kw)
    assert rc == status and not ctx.value


def test_null_arguments_are_rejected(lib):
    assert lib.lddmm_create(None, None, None) == -1
    assert lib.lddmm_destroy(None) == -1
    assert lib.lddmm_shoot(None, None, None, None, None, None) == -1
    assert lib.lddmm_hessvec(None, None, None, None) == -1
    assert lib.lddmm_hessvec_newton(None, None, None, None) == -1
    assert lib.lddmm_gn_solve(None, None, None, None, None, 0) == -1
    assert lib.lddmm_vjp(None, None, None) == -1
    assert lib.lddmm_apply_operator(None, 0, 3, None, None) == -1
    for st in (0, 1):
        assert lib.lddmm_pde_energy(None, st, None, None, None) == -1
        assert lib.lddmm_pde_gradient(None, st, None, None, None) == -1
        assert lib.lddmm_pde_hessvec(None, st, None, None, None) == -1
        assert lib.lddmm_pde_gn_solve(None, st, None, None, None, None, 0) == -1
        assert lib.lddmm_pde_displacement(None, st, None, None) == -1
    assert lib.lddmm_batch_create(None, 0, None) == -1
    assert lib.lddmm_batch_gn_solve(None, None, None, None, 0) == -1
    assert lib.lddmm_batch_hessvec(None, None, None, 1, 0) == -1


def test_strerror(lib):
    assert lib.lddmm_strerror(0) == b"ok"
    assert lib.lddmm_strerror(-5) == b"non-finite input"
    assert lib.lddmm_strerror(-99) == b"unknown status"
    assert lib.lddmm_last_error(None) == b"null context"
