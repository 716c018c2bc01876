"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and arranges them; it holds none of the transform's
arithmetic.  Harmonic coefficients are returned in the flat layout used throughout the
project: for one map, a complex array of length L*L with f_{l,m} at index l*l + l + m.

Recipe (band-limited Gaussian signals, as in the accuracy/timing protocol of Sect. 3.3):
  * the generator is numpy's PCG64 (``numpy.random.default_rng(seed)``);
  * draws are taken map by map, then l ascending, then m ascending, real part before
    imaginary part;
  * real maps: f_{l0} = sqrt(C_l) x and, for m > 0, f_{lm} = sqrt(C_l / 2) (x + i y),
    with f_{l,-m} = (-1)^m conj(f_{lm}) so that the map is real;
  * complex maps: f_{lm} = sqrt(C_l / 2) (x + i y) for every m;
  * the paper's accuracy sweep uses complex f_{lm} ~ N(0, 1) (C_l = 2, i.e. unit
    variance per real component).
"""
from __future__ import annotations

import numpy as np


def spectrum_inverse_ll1(L: int) -> np.ndarray:
    """C_l = 1 / (l (l + 1)) for l >= 1 and C_0 = 0 (monopole removed)."""
    ell = np.arange(L, dtype=np.float64)
    c = np.zeros(L)
    c[1:] = 1.0 / (ell[1:] * (ell[1:] + 1.0))
    return c


def spectrum_power(L: int, alpha: float) -> np.ndarray:
    """C_l = (l + 1)^(-alpha), including l = 0."""
    return (np.arange(L, dtype=np.float64) + 1.0) ** (-alpha)


def _real_map(rng: np.random.Generator, L: int, cl: np.ndarray) -> np.ndarray:
    # Per l: one draw for m = 0, then (re, im) for m = 1..l  -> 2l + 1 draws, L*L in total.
    z = rng.standard_normal(L * L)
    out = np.zeros(L * L, dtype=np.complex128)
    for ell in range(L):
        base = ell * ell
        sc = np.sqrt(cl[ell])
        out[ell * ell + ell] = sc * z[base]
        if ell == 0:
            continue
        m = np.arange(1, ell + 1)
        re = z[base + 1 + 2 * (m - 1)]
        im = z[base + 2 + 2 * (m - 1)]
        v = np.sqrt(cl[ell] / 2.0) * (re + 1j * im)
        out[ell * ell + ell + m] = v
        out[ell * ell + ell - m] = ((-1.0) ** m) * np.conj(v)
    return out


def _complex_map(rng: np.random.Generator, L: int, cl: np.ndarray) -> np.ndarray:
    # Per l: (re, im) for m = -l..l -> 2(2l + 1) draws.
    z = rng.standard_normal(2 * L * L)
    out = np.zeros(L * L, dtype=np.complex128)
    for ell in range(L):
        base = 2 * ell * ell
        cnt = 2 * ell + 1
        re = z[base: base + 2 * cnt: 2]
        im = z[base + 1: base + 2 * cnt: 2]
        out[ell * ell: ell * ell + cnt] = np.sqrt(cl[ell] / 2.0) * (re + 1j * im)
    return out


def random_flm(L: int, nmaps: int = 1, reality: bool = True, seed: int = 0,
               cl: np.ndarray | None = None) -> np.ndarray:
    """Seeded band-limited harmonic coefficients, shape [nmaps, L*L] complex128."""
    if cl is None:
        cl = spectrum_inverse_ll1(L)
    cl = np.asarray(cl, dtype=np.float64)
    if cl.shape != (L,):
        raise ValueError("cl must have length L")
    rng = np.random.default_rng(seed)
    maps = [(_real_map if reality else _complex_map)(rng, L, cl) for _ in range(nmaps)]
    return np.stack(maps)


def random_flm_unit(L: int, nmaps: int = 1, seed: int = 0) -> np.ndarray:
    """Complex f_lm ~ N(0,1) per real component: the paper's accuracy/timing sweep."""
    return random_flm(L, nmaps, reality=False, seed=seed, cl=np.full(L, 2.0))


def uniform_batch_params(seed: int, nmaps: int, Ls=(64, 128, 256, 512), Bs=(2, 3),
                         alpha_range=(1.0, 3.0)):
    """Per-map (L, B, alpha) draws for the uneven batching workload."""
    rng = np.random.default_rng(seed)
    L = rng.choice(np.asarray(Ls), size=nmaps)
    B = rng.choice(np.asarray(Bs), size=nmaps)
    alpha = rng.uniform(alpha_range[0], alpha_range[1], size=nmaps)
    return [(int(a), int(b), float(c)) for a, b, c in zip(L, B, alpha)]


def random_unit_flm_basis(L: int, ell: int, m: int) -> np.ndarray:
    """Indicator coefficient vector e_{l m} (one map)."""
    out = np.zeros((1, L * L), dtype=np.complex128)
    out[0, ell * ell + ell + m] = 1.0
    return out


def denoise_workload(L: int, nmaps: int = 1, seed: int = 9, snr_db: float = 11.78, alpha: float = 3.0):
    """Signal-plus-white-noise maps for the hard-thresholding denoising example of Sect. 4.3:
    s with spectrum C_l = (l + 1)^(-alpha) (most power on large scales), and real white noise
    n with E|n_lm|^2 = sigma^2 for every (l, m), sigma chosen so that the expected noise energy
    sigma^2 L^2 sets SNR(y) to snr_db against the mean energy of the drawn signals (11.78 dB is
    the noisy map of that example).  Returns (s_lm, n_lm, sigma), both [nmaps, L*L]."""
    s = random_flm(L, nmaps, reality=True, seed=seed, cl=spectrum_power(L, alpha))
    energy = float(np.mean(np.sum(np.abs(s) ** 2, axis=1)))
    sigma = float(np.sqrt(energy / (L * L * 10.0 ** (snr_db / 10.0))))
    n = random_flm(L, nmaps, reality=True, seed=seed + 5000, cl=np.full(L, sigma * sigma))
    return s, n, sigma
