"""Pins for the oracle's adjoint transforms (used to check the library's adjoint kernels).
Each adjoint is checked against something other than itself: the defining identity
<M x, y> = <x, M^H y> with the oracle's forward maps (themselves pinned in
test_oracle_pins.py), the plain definition sum conj(Y_lm) f with scipy's Y_lm, and the identity
S^H A^H = I that follows from A S = I (the quadrature is exact for band-limited maps)."""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(1211)


def _ip(a, b):
    return float(np.real(np.vdot(a, b)))


def _rand_maps(k, nmaps=2, real=False):
    n = 2 * k - 1
    x = RNG.standard_normal((nmaps, k, n))
    return x if real else x + 1j * RNG.standard_normal((nmaps, k, n))


def _rand_coefs(k, nmaps=2):
    return RNG.standard_normal((nmaps, k * k)) + 1j * RNG.standard_normal((nmaps, k * k))


@pytest.mark.parametrize("k", [1, 2, 3, 8, 17])
def test_inverse_adjoint_dot_product(k):
    x, y = _rand_coefs(k), _rand_maps(k)
    lhs = _ip(oracle.inverse_sht(x, k), y)
    rhs = _ip(x, oracle.inverse_sht_adjoint(y, k))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("k", [1, 2, 3, 8, 17])
@pytest.mark.parametrize("real", [False, True])
def test_forward_adjoint_dot_product(k, real):
    x, y = _rand_maps(k, real=real), _rand_coefs(k)
    lhs = _ip(oracle.forward_sht(x, k), y)
    rhs = _ip(x, oracle.forward_sht_adjoint(y, k, reality=real))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("k", [3, 6])
def test_inverse_adjoint_direct_definition(k):
    from scipy.special import sph_harm_y
    f = _rand_maps(k, nmaps=1)[0]
    theta, phi = oracle.mw_nodes(k)
    TT, PP = np.meshgrid(theta, phi, indexing="ij")
    ref = np.zeros(k * k, dtype=np.complex128)
    for ell in range(k):
        for m in range(-ell, ell + 1):
            ref[ell * ell + ell + m] = np.sum(np.conj(sph_harm_y(ell, m, TT, PP)) * f)
    got = oracle.inverse_sht_adjoint(f, k)[0]
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("k", [4, 9, 16])
def test_adjoints_compose_to_identity(k):
    """A S = I on band-limited coefficients, hence S^H A^H = I."""
    y = _rand_coefs(k)
    back = oracle.inverse_sht_adjoint(oracle.forward_sht_adjoint(y, k), k)
    assert np.max(np.abs(back - y)) < 1e-13 * k


@pytest.mark.parametrize("L,B,J_min,multires,real", [(16, 2, 1, True, True), (16, 2, 0, False, False),
                                                      (27, 3, 1, True, True)])
def test_wavelet_adjoints_dot_product(L, B, J_min, multires, real):
    f = _rand_maps(L, real=real)
    wav, scal = oracle.analysis(f, L, B, J_min, multires, real)
    # random wavelet-side vector of the same shapes
    wr = [_rand_maps(w.shape[1], real=real) for w in wav]
    sr = _rand_maps(scal.shape[1], real=real)
    lhs = sum(_ip(w, v) for w, v in zip(wav, wr)) + _ip(scal, sr)
    rhs = _ip(f, oracle.analysis_adjoint(wr, sr, L, B, J_min, multires, real))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # synthesis and its adjoint
    rec = oracle.synthesis(wr, sr, L, B, J_min, multires, real)
    wa, sa = oracle.synthesis_adjoint(f, L, B, J_min, multires, real)
    lhs = _ip(rec, f)
    rhs = sum(_ip(w, v) for w, v in zip(wr, wa)) + _ip(sr, sa)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_planted_fold_sign_mistake_is_caught(monkeypatch):
    """An oracle forward adjoint whose fold and extension lose the parity (-1)^m (planted by
    making its parity vector all ones) fails the dot-product identity."""
    k = 6
    x, y = _rand_maps(k), _rand_coefs(k)
    lhs = _ip(oracle.forward_sht(x, k), y)
    real_where = np.where

    def no_parity(cond, a, b):
        out = real_where(cond, a, b)
        if np.shape(out) == (2 * k - 1,) and set(np.unique(out)) <= {1.0, -1.0}:
            return np.ones_like(out)
        return out

    monkeypatch.setattr(oracle.np, "where", no_parity)
    wrong = _ip(x, oracle.forward_sht_adjoint(y, k))
    monkeypatch.setattr(oracle.np, "where", real_where)
    right = _ip(x, oracle.forward_sht_adjoint(y, k))
    assert abs(lhs - right) <= 1e-13 * abs(lhs)
    assert abs(lhs - wrong) > 1e-6 * abs(lhs)
