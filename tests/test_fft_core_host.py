"""CPU check of the FFT butterfly/twiddle/digit-reversal code shared with the GPU
kernels (compiled for the host from the same header), against numpy.fft."""

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SIZES = [2, 3, 4, 5, 7, 8, 9, 16, 18, 27, 30, 32, 40, 45, 48, 56, 60, 63, 64, 72, 80, 81, 84, 90, 96, 105, 108, 112,
         120, 128, 135, 160, 180, 192, 216, 240, 243, 256, 336, 384, 512, 648, 1024, 2048]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    cc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("fftcore") / "libfftcore_host.so")
    src = os.path.join(HERE, "native", "fft_core_host.cpp")
    inc = os.path.join(ROOT, "paper_1807_04638_amd", "csrc")
    subprocess.run([cc, "-O2", "-std=c++17", "-fPIC", "-shared", "-I", inc, src, "-o", out], check=True)
    L = ctypes.CDLL(out)
    L.fftcore_transform.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.fftcore_digit_reverse.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.fftcore_transform_static.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    return L


def _perm(lib, n):
    perm = np.zeros(n, dtype=np.int32)
    assert lib.fftcore_digit_reverse(n, perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int))) == 0
    return perm


@pytest.mark.parametrize("n", SIZES)
def test_dif_matches_numpy_in_digit_reversed_order(lib, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    buf = x.astype(np.complex128).copy()
    assert lib.fftcore_transform(n, buf.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0) >= 1
    perm = _perm(lib, n)
    assert sorted(perm.tolist()) == list(range(n))
    np.testing.assert_allclose(buf, np.fft.fft(x)[perm], atol=1e-12 * n)


@pytest.mark.parametrize("n", SIZES)
def test_dit_inverts_dif(lib, n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    buf = x.copy()
    p = buf.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    lib.fftcore_transform(n, p, 0)
    lib.fftcore_transform(n, p, 1)
    np.testing.assert_allclose(buf / n, x, atol=1e-13 * n)


def test_unsupported_length(lib):
    buf = np.zeros(22, dtype=np.complex128)
    assert lib.fftcore_transform(11, buf.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0) == -1


STATIC = [16, 32, 64, 128, 256, 40, 48, 56, 80, 90, 96, 112, 180, 216]


@pytest.mark.parametrize("n", STATIC)
def test_compile_time_plans_match_runtime_and_numpy(lib, n):
    """The compile-time plans used by the specialised GPU kernels have the
    runtime plan's radices and transform the same way."""
    rng = np.random.default_rng(300 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    buf = x.copy()
    p = buf.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.fftcore_transform_static(n, p, 0) >= 1
    np.testing.assert_allclose(buf, np.fft.fft(x)[_perm(lib, n)], atol=1e-12 * n)
    lib.fftcore_transform_static(n, p, 1)
    np.testing.assert_allclose(buf / n, x, atol=1e-13 * n)


@pytest.mark.parametrize("n, stages", [(16, 2), (32, 2), (64, 2), (128, 2), (256, 2), (384, 3), (512, 3), (1024, 3),
                                       (2048, 3), (80, 3), (96, 3)])
def test_radix16_regrouping_stage_counts(lib, n, stages):
    """With two or more radix-8 stages, a trailing 8 x 2 is one radix-16 stage and a
    trailing 8 x 8 x 4 two radix-16 stages; short lengths keep their two stages."""
    x = np.zeros(2 * n)
    assert lib.fftcore_transform(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0) == stages
