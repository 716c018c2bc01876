"""The reformulation behind the band-limit 1024/2048 kernels, checked on the CPU: the theta
quadrature of the MW transform evaluated on the half-shifted grid psi_s = pi (2s+1) / (2k),
s < 2k (symmetric about the equator), with the north/south parity split of the Legendre sums,
and the inverse transform computed on that grid and resampled to the MW nodes.  The steps are
written out plainly in numpy with scipy's Y_lm (independent of the GPU code and of the oracle's
own quadrature) and compared with the oracle's forward and inverse transforms, on band-limited
maps and on arbitrary samples, for even and odd k.  Also checked: the packed form the kernels
use (an even and an odd m in one complex sequence, the even part of the weight only, plus the
odd-m pole column on the psi grid) equals the full-weight evaluation."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

import oracle
import s2let_inputs as si


def _w(p, odd_terms=True):
    p = np.asarray(p)
    out = np.zeros(p.shape, complex)
    ev = p % 2 == 0
    out[ev] = 2.0 / (1.0 - p[ev].astype(float) ** 2)
    if odd_terms:
        out[p == 1] = 1j * np.pi / 2
        out[p == -1] = -1j * np.pi / 2
    return out


def _grids(k):
    n, N = 2 * k - 1, 2 * k
    th = np.pi * (2 * np.arange(n) + 1) / n
    psi = np.pi * (2 * np.arange(N) + 1) / N
    return n, N, th, psi, np.arange(-(k - 1), k)


def _lam(l, m, x):
    v = np.real(sph_harm_y(l, abs(m), x, 0.0))
    return v * (-1) ** abs(m) if m < 0 else v


def _H_psi(g, k, odd_terms=True):
    """theta quadrature of the extended samples g (MW circle) evaluated on the psi circle"""
    n, N, th, psi, js = _grids(k)
    Gh = np.exp(-1j * np.outer(js, th)) @ g / n
    I = np.array([np.sum(Gh * _w(js + jp, odd_terms)) for jp in js])
    return np.exp(-1j * np.outer(psi, js)) @ I / N


def forward_psi(f, k):
    n, N, th, psi, js = _grids(k)
    ph = 2 * np.pi * np.arange(n) / n
    flm = np.zeros(k * k, complex)
    hs = k // 2
    for m in range(-(k - 1), k):
        G = (2 * np.pi / n) * (f @ np.exp(-1j * m * ph))
        g = np.concatenate([G, (-1) ** (m % 2) * G[n - 1 - np.arange(k, n)]])
        H = _H_psi(g, k)
        Hf = H[:k] + (-1) ** (m % 2) * H[N - 1 - np.arange(k)]
        for l in range(abs(m), k):
            lv = _lam(l, m, psi[:hs])
            val = np.sum(lv * (Hf[:hs] + (-1) ** ((l + m) % 2) * Hf[k - 1 - np.arange(hs)]))
            if k % 2:
                val += _lam(l, m, psi[hs]) * Hf[hs]
            flm[l * l + l + m] = val
    return flm


def inverse_psi(flm, k):
    n, N, th, psi, js = _grids(k)
    ph = 2 * np.pi * np.arange(n) / n
    out = np.zeros((k, n), complex)
    hs = k // 2
    for m in range(-(k - 1), k):
        E = np.zeros(hs + k % 2, complex)
        O = np.zeros(hs + k % 2, complex)
        for l in range(abs(m), k):
            v = flm[l * l + l + m] * _lam(l, m, psi[:hs + k % 2])
            if (l + m) % 2 == 0:
                E += v
            else:
                O += v
        F = np.zeros(k, complex)
        F[:hs] = E[:hs] + O[:hs]
        F[k - 1 - np.arange(hs)] = E[:hs] - O[:hs]
        if k % 2:
            F[hs] = E[hs]
        ext = np.concatenate([F, (-1) ** (m % 2) * F[N - 1 - np.arange(k, N)]])
        Fh = np.exp(-1j * np.outer(js, psi)) @ ext / N
        out += np.outer(np.exp(1j * np.outer(th[:k], js)) @ Fh, np.exp(1j * m * ph))
    return out


@pytest.mark.parametrize("k", [4, 5, 8])
def test_forward_and_inverse_on_the_symmetric_grid(k):
    flm = si.random_flm(k, 1, reality=False, seed=k)[0]
    f = oracle.inverse_sht(flm[None], k, False)[0]
    assert oracle.rel_max_err(forward_psi(f, k), flm) < 1e-13
    assert oracle.rel_max_err(inverse_psi(flm, k), f) < 1e-13
    rng = np.random.default_rng(k)
    x = rng.standard_normal((k, 2 * k - 1)) + 1j * rng.standard_normal((k, 2 * k - 1))
    assert oracle.rel_max_err(forward_psi(x, k), oracle.forward_sht(x[None], k)[0]) < 1e-13


def test_packed_even_weight_with_pole_column():
    k = 8
    n, N, th, psi, js = _grids(k)
    rng = np.random.default_rng(1)
    GE = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    GO = rng.standard_normal(k) + 1j * rng.standard_normal(k)

    def full(G, m):
        g = np.concatenate([G, (-1) ** m * G[n - 1 - np.arange(k, n)]])
        H = _H_psi(g, k)
        return H[:k] + (-1) ** m * H[N - 1 - np.arange(k)]

    g = np.zeros(n, complex)
    for t in range(n):
        tt = t if t < k else n - 1 - t
        g[t] = GE[tt] + ((1.0 if t < k else -1.0) * GO[tt] if tt < k - 1 else 0.0)
    H = _H_psi(g, k, odd_terms=False)
    he = H[:k] + H[N - 1 - np.arange(k)]
    ho = H[:k] - H[N - 1 - np.arange(k)]
    d = np.zeros(n, complex)
    d[k - 1] = 1.0
    Hd = _H_psi(d, k)
    pole = Hd[:k] - Hd[N - 1 - np.arange(k)]
    assert np.max(np.abs(pole.imag)) < 1e-15
    assert np.max(np.abs(he - full(GE, 0))) < 1e-14
    assert np.max(np.abs(ho + pole * GO[k - 1] - full(GO, 1))) < 1e-14


@pytest.mark.parametrize("k", [32, 64, 2048])
def test_parity_class_kernels_share_one_real_spectrum(k):
    """The theta correlation of each frequency-parity class Q uses the kernel Kt_Q(c) = w(2Q - 2c),
    c in [Q - (k-1), Q + (k-1)], wrapped to Nc = 2k slots (the even part of w, Sect. 2.1).  The
    kernels use one real table for both: Kt_0 is real and even, so its spectrum is real; Kt_1 is
    Kt_0 shifted by one slot, so class 1 equals the class-0 convolution read one slot lower.  Also
    checked: after that shift every class reads its output on [0, Nc/4) and [3Nc/4, Nc) only."""
    Nc = 2 * k
    kt = []
    for Q in (0, 1):
        v = np.zeros(Nc, complex)
        c = np.arange(Q - (k - 1), Q + k)
        v[c % Nc] = _w(2 * Q - 2 * c, odd_terms=False)
        kt.append(v)
    np.testing.assert_array_equal(kt[1], np.roll(kt[0], 1))
    spec = np.fft.fft(kt[0])
    assert np.max(np.abs(spec.imag)) <= 1e-13 * np.max(np.abs(spec.real))
    np.testing.assert_allclose(spec.real, spec.real[(-np.arange(Nc)) % Nc], rtol=0, atol=1e-13 * np.max(np.abs(spec)))

    rng = np.random.default_rng(7)
    j = np.arange(-(k - 1), k)
    for P in (0, 1):
        cls = j[(j - P) % 2 == 0]
        x = np.zeros(Nc, complex)
        x[((cls - P) // 2) % Nc] = rng.standard_normal(cls.size) + 1j * rng.standard_normal(cls.size)
        direct = np.fft.ifft(np.fft.fft(x) * np.fft.fft(kt[P]))
        shared = np.fft.ifft(np.fft.fft(x) * spec.real)
        rd = (-(cls - P) // 2) % Nc
        np.testing.assert_allclose(shared[(rd - P) % Nc], direct[rd], rtol=0, atol=1e-12 * np.max(np.abs(direct)))
        slot = (rd - P) % Nc
        assert np.all((slot < Nc // 4) | (slot >= 3 * Nc // 4))
