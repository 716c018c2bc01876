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
    for st in (0, -1, -2, -3, -4):
        assert len(s2.lib.s2let_strerror(st)) > 0


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


def test_workspace_size_monotone():
    a = s2.workspace_size(64, nmaps=1)
    b = s2.workspace_size(64, nmaps=16)
    c = s2.workspace_size(128, nmaps=16)
    assert 0 < a < b < c
    assert s2.workspace_size(2048, 2, 3, True, s2.REAL, s2.FP64, 16, True) < 8 * 2 ** 30
