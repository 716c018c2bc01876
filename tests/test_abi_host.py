"""Host-side checks of the C-ABI library (no GPU): it loads, exports every declared symbol,
and its host-only helpers agree with the oracle; invalid arguments are rejected before any
device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "s2let_mi355x.h")

s2 = pytest.importorskip("paper_1211_1680_amd")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([A-Za-z_][A-Za-z0-9_]*)\s*\(", text)
    kw = {"if", "while", "for", "return", "sizeof", "defined"}
    return sorted({n for n in names if n not in kw and not n.isupper()})


def test_every_declared_symbol_is_exported():
    names = _declared_functions()
    assert "mw_forward" in names and "s2let_axisym_analysis" in names
    lib = ctypes.CDLL(s2.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_strerror():
    assert b"gfx950" in s2.lib.s2let_version()
    for st in (0, -1, -2, -3, -4, -5, -6):
        assert len(s2.lib.s2let_strerror(st)) > 0
        assert s2.lib.s2let_strerror(st) != b"unknown status"


@pytest.mark.parametrize("L,B", [(3, 2), (4, 2), (5, 2), (64, 2), (65, 2), (66, 2), (128, 3), (2048, 2),
                                 (1025, 2), (10, 3), (82, 3), (83, 3)])
def test_j_max_matches_oracle(L, B):
    assert s2.j_max(L, B) == oracle.j_max(L, B)


def test_bandlimits_and_sizes():
    for (L, B, J_min, mr) in [(64, 2, 0, False), (512, 2, 2, True), (2048, 2, 3, True), (128, 3, 2, True),
                              (100, 3, 1, True)]:
        J = oracle.j_max(L, B)
        tot = 0
        for j in range(J_min, J + 1):
            k = oracle.bandlimit_wav(j, L, B, mr)
            assert s2.bandlimit_wav(j, L, B, mr) == k
            tot += k * (2 * k - 1)
        assert s2.wav_size(L, B, J_min, mr) == tot
        assert s2.bandlimit_scal(J_min, L, B, mr) == oracle.bandlimit_scal(J_min, L, B, mr)
    assert s2.mw_size(1) == 1 and s2.mw_size(2048) == 2048 * 4095


def test_config_band_limits():
    # L=512, B=2, J_min=2, multiresolution: k_Phi = 4, k_j = 8, 16, ..., 512, 512
    assert s2.bandlimit_scal(2, 512, 2, True) == 4
    assert [s2.bandlimit_wav(j, 512, 2, True) for j in range(2, 10)] == [8, 16, 32, 64, 128, 256, 512, 512]
    # L=2048, B=2, J_min=3: k_Phi = 8, k_j = 16 ... 2048, 2048
    assert s2.bandlimit_scal(3, 2048, 2, True) == 8
    assert [s2.bandlimit_wav(j, 2048, 2, True) for j in range(3, 12)] == [16, 32, 64, 128, 256, 512, 1024,
                                                                         2048, 2048]


@pytest.mark.parametrize("L,B,J_min", [(64, 2, 0), (128, 3, 2), (300, 3, 1), (512, 2, 2)])
def test_tiling_matches_oracle(L, B, J_min):
    """The library's Gauss-Legendre evaluation of Eq. (12) against the oracle's adaptive
    Gauss-Kronrod (two independent quadratures)."""
    kappa, eta = s2.tiling_axisym(L, B, J_min)
    ok, oe = oracle.tiling(L, B, J_min)
    assert np.max(np.abs(kappa - ok)) < 1e-15
    assert np.max(np.abs(eta - oe)) < 1e-15
    assert np.max(np.abs(eta ** 2 + np.sum(kappa ** 2, axis=0) - 1.0)) < 4e-15


def test_invalid_arguments_rejected_without_device():
    lib = s2.lib
    ws = ctypes.c_void_p(4096)
    buf = ctypes.c_void_p(4096)
    # L < 1, bad reality, bad precision, nmaps < 1, null pointers, misaligned pointers
    assert lib.mw_forward(buf, buf, 0, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert lib.mw_forward(buf, buf, 8, 2, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert lib.mw_forward(buf, buf, 8, 0, 7, 1, ws, 1 << 40, None) == s2.EINVAL
    assert lib.mw_forward(buf, buf, 8, 0, 0, 0, ws, 1 << 40, None) == s2.EINVAL
    assert lib.mw_forward(None, buf, 8, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert lib.mw_inverse(ctypes.c_void_p(4097), buf, 8, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    # too large, too little workspace
    assert lib.mw_forward(buf, buf, 4096, 0, 0, 1, ws, 1 << 40, None) == s2.EUNSUPPORTED
    assert lib.mw_forward(buf, buf, 64, 0, 0, 1, ws, 16, None) == s2.ENOMEM
    # wavelet parameters: J_min >= J, B < 2, L < 3
    a = lib.s2let_axisym_analysis
    assert a(buf, buf, buf, 64, 2, 6, 1, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert a(buf, buf, buf, 64, 1, 0, 1, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert a(buf, buf, buf, 2, 2, 0, 1, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert a(buf, buf, buf, 64, 2, -1, 1, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    assert lib.s2let_j_max(2, 2) == s2.EINVAL and lib.s2let_j_max(10, 1) == s2.EINVAL
    assert lib.s2let_workspace_size(64, 2, 6, 1, 0, 0, 1, 1) == 0
    # the allocation-free analysis validates the same way, then refuses inputs whose workspace
    # exceeds its static scratch (16 real maps at L = 512), all before any device call
    n = lib.s2let_axisym_analysis_noalloc
    assert n(buf, buf, buf, 64, 2, 6, 1, 0, 0, 1, None) == s2.EINVAL
    assert n(buf, buf, buf, 64, 2, 0, 1, 0, 9, 1, None) == s2.EINVAL
    assert n(buf, buf, buf, 4096, 2, 3, 1, 0, 0, 1, None) == s2.EUNSUPPORTED
    assert s2.workspace_size(512, 2, 2, True, s2.REAL, s2.FP64, 16, True) > s2.NOALLOC_SCRATCH_BYTES
    assert n(buf, buf, buf, 512, 2, 2, 1, 0, 0, 16, None) == s2.ESCRATCH


def test_workspace_size_monotone():
    a = s2.workspace_size(64, nmaps=1)
    b = s2.workspace_size(64, nmaps=16)
    c = s2.workspace_size(128, nmaps=16)
    assert 0 < a < b < c
    assert s2.workspace_size(2048, 2, 3, True, s2.REAL, s2.FP64, 16, True) < 8 * 2 ** 30


# ---------------------------------------------------------------- generating functions, noise model
@pytest.mark.parametrize("L,B,J_min", [(16, 2, 0), (50, 3, 2), (128, 2, 0), (128, 3, 2), (300, 3, 1), (2048, 2, 3)])
def test_bspline_tiling_and_bandlimits_match_oracle(L, B, J_min):
    """Host B-spline tiling (long double) against the oracle's exact rationals; band-limits and
    sizes for both kernels."""
    kappa, eta = s2.tiling_axisym(L, B, J_min, s2.KERNEL_BSPLINE)
    ok, oe = oracle.tiling(L, B, J_min, "bspline")
    assert np.max(np.abs(kappa - ok)) < 1e-15 and np.max(np.abs(eta - oe)) < 1e-15
    for kernel, name in ((s2.KERNEL_SD, "sd"), (s2.KERNEL_BSPLINE, "bspline")):
        for mr in (False, True):
            tot = 0
            for j in range(J_min, oracle.j_max(L, B) + 1):
                k = oracle.bandlimit_wav(j, L, B, mr, name)
                assert s2.bandlimit_wav(j, L, B, mr, kernel) == k
                tot += k * (2 * k - 1)
            assert s2.wav_size(L, B, J_min, mr, kernel) == tot
            assert s2.bandlimit_scal(J_min, L, B, mr, kernel) == oracle.bandlimit_scal(J_min, L, B, mr, name)


def test_sd_kernel_calls_equal_default_calls():
    k1, e1 = s2.tiling_axisym(128, 3, 2)
    k2, e2 = s2.tiling_axisym(128, 3, 2, s2.KERNEL_SD)
    assert np.array_equal(k1, k2) and np.array_equal(e1, e2)
    assert s2.lib.s2let_wav_size(512, 2, 2, 1) == s2.lib.s2let_wav_size_kernel(512, 2, 2, 1, s2.KERNEL_SD)


@pytest.mark.parametrize("kernel,name", [(0, "sd"), (1, "bspline")])
def test_noise_std_matches_oracle(kernel, name):
    for (L, B, J_min, sigma) in [(64, 2, 0, 1.0), (128, 2, 0, 0.05), (300, 3, 1, 2.5)]:
        got = s2.noise_std(L, B, J_min, sigma, kernel)
        ref = oracle.noise_std(L, B, J_min, sigma, name)
        assert np.max(np.abs(got - ref) / ref) < 1e-14


def test_kernel_arguments_rejected_without_device():
    lib = s2.lib
    ws, buf = ctypes.c_void_p(4096), ctypes.c_void_p(4096)
    dp = ctypes.POINTER(ctypes.c_double)
    k = np.zeros(64 * 8)
    e = np.zeros(64)
    assert lib.s2let_tiling_axisym_kernel(k.ctypes.data_as(dp), e.ctypes.data_as(dp), 64, 2, 0, 2) == s2.EUNSUPPORTED
    assert lib.s2let_tiling_axisym_kernel(k.ctypes.data_as(dp), e.ctypes.data_as(dp), 64, 2, 0, 7) == s2.EINVAL
    assert lib.s2let_bandlimit_wav_kernel(3, 64, 2, 1, 2) == s2.EUNSUPPORTED
    assert lib.s2let_bandlimit_scal_kernel(1, 64, 2, 1, 9) == s2.EINVAL
    assert lib.s2let_wav_size_kernel(64, 2, 0, 1, 5) == -1
    a = lib.s2let_axisym_analysis_kernel
    assert a(buf, buf, buf, 64, 2, 0, 1, 2, 0, 0, 1, ws, 1 << 40, None) == s2.EUNSUPPORTED
    assert a(buf, buf, buf, 64, 2, 0, 1, -1, 0, 0, 1, ws, 1 << 40, None) == s2.EINVAL
    sy = lib.s2let_axisym_synthesis_kernel
    assert sy(buf, buf, buf, 64, 2, 0, 1, 2, 0, 0, 1, ws, 1 << 40, None) == s2.EUNSUPPORTED
    sig = np.zeros(8)
    assert lib.s2let_noise_std_axisym(sig.ctypes.data_as(dp), 64, 2, 0, 0, -1.0) == s2.EINVAL
    assert lib.s2let_noise_std_axisym(sig.ctypes.data_as(dp), 64, 2, 0, 2, 1.0) == s2.EUNSUPPORTED
    thr = np.ones(8)
    h = lib.s2let_hard_threshold
    assert h(None, thr.ctypes.data_as(dp), 64, 2, 0, 1, 0, 0, 1, None) == s2.EINVAL
    assert h(buf, None, 64, 2, 0, 1, 0, 0, 1, None) == s2.EINVAL
    assert h(buf, thr.ctypes.data_as(dp), 64, 2, 0, 1, 0, 3, 1, None) == s2.EINVAL
    assert h(buf, thr.ctypes.data_as(dp), 64, 2, 0, 1, 2, 0, 1, None) == s2.EUNSUPPORTED
    assert h(buf, thr.ctypes.data_as(dp), 64, 2, 0, 1, 0, 0, 0, None) == s2.EINVAL


def test_one_hip_runtime_whatever_the_import_order():
    """Importing the binding before torch must not map a second HIP/HSA runtime into the process
    (two HSA runtimes cannot both open the device)."""
    import subprocess
    import sys
    code = ("import paper_1211_1680_amd, torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
            "print(len([x for x in libs if 'amdhip64' in x]), len([x for x in libs if 'hsa-runtime64' in x]))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout
