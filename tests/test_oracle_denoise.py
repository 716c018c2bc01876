"""Pins for the oracle's B-spline generating function (footnote to Sect. 2.2, Eqs. (17)-(18)),
its multiresolution band-limits (Sect. 3.1), the wavelet-space noise model and the hard
thresholding of Sect. 4.3 (Eqs. (19)-(23)).  Each test checks the oracle against something
other than itself: textbook values and a library B-spline, exact rational identities, the
supports and band-limits the paper states, Monte Carlo statistics, closed forms, and planted
mistakes that must be caught."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
import s2let_inputs as si


# ---------------------------------------------------------------- B_3 (Eq. (18))
def test_b3_textbook_values():
    b3 = oracle.bspline_b3
    assert b3(0) == F(2, 3)
    assert b3(1) == b3(-1) == F(1, 6)
    assert b3(2) == b3(-2) == b3(3) == b3(F(-7, 3)) == 0
    assert b3(F(1, 2)) == F(23, 48)          # (2/3) - x^2 + |x|^3 / 2 at x = 1/2
    assert b3(F(3, 2)) == F(1, 48)           # (2 - x)^3 / 6 at x = 3/2
    for x in (F(1, 7), F(5, 4), F(19, 10)):
        assert b3(x) == b3(-x)


def test_b3_partition_of_unity_exact():
    for x in (F(0), F(1, 3), F(2, 7), F(9, 10), F(-5, 11)):
        assert sum(oracle.bspline_b3(x - n) for n in range(-4, 5)) == 1


def test_b3_matches_scipy_bspline():
    from scipy.interpolate import BSpline
    ref = BSpline.basis_element([-2.0, -1.0, 0.0, 1.0, 2.0], extrapolate=False)
    for x in np.linspace(-1.99, 1.99, 41):
        assert abs(float(oracle.bspline_b3(F(x))) - float(ref(x))) < 1e-15


def test_b3_unit_integral():
    from scipy.integrate import quad
    val = quad(lambda x: float(oracle.bspline_b3(F(x))), -2.0, 2.0, points=[-1.0, 0.0, 1.0])[0]
    assert abs(val - 1.0) < 1e-12


# ---------------------------------------------------------------- k_lambda and the tiling
def test_k_bspline_endpoints_and_monotone():
    L, B = 128, 2
    J = oracle.j_max(L, B)
    assert oracle.k_bspline(0, B, L, J) == 1                       # (3/2) B_3(0) = 1
    edge = F(L, B ** (J - 1))                                      # 2 t B^(J-1) / L = 2
    assert oracle.k_bspline(edge, B, L, J) == 0
    assert oracle.k_bspline(edge * F(999, 1000), B, L, J) > 0
    ts = [F(i, 16) for i in range(0, 40)]
    vals = [oracle.k_bspline(t, B, L, J) for t in ts]
    assert all(a >= b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("L,B,J_min", [(16, 2, 0), (32, 3, 1), (50, 3, 2), (128, 2, 0), (128, 3, 2), (100, 2, 3)])
def test_bspline_tiling_identity_exact(L, B, J_min):
    """eta^2 + sum_j kappa_j^2 = 1 for every l < L (Eq. (9)), exactly in rationals; every term
    is non-negative (k is non-increasing)."""
    kap2, eta2 = oracle.tiling_bspline_sq(L, B, J_min)
    for ell in range(L):
        assert eta2[ell] + sum(row[ell] for row in kap2) == 1
        assert eta2[ell] >= 0 and all(row[ell] >= 0 for row in kap2)
    kappa, eta = oracle.tiling(L, B, J_min, "bspline")
    assert np.max(np.abs(eta ** 2 + np.sum(kappa ** 2, axis=0) - 1.0)) < 4e-16 * (kappa.shape[0] + 1)


@pytest.mark.parametrize("L,B", [(128, 2), (128, 3), (100, 2), (243, 3), (2048, 2)])
def test_bspline_supports_and_bandlimits_from_paper(L, B):
    """Scale j is supported on [0, L / B^(J-j-2)] (footnote to Sect. 2.2); the multiresolution
    band-limit is that end point (Sect. 3.1), rounded up and capped at L."""
    J = oracle.j_max(L, B)
    J_min = 0
    kap2, eta2 = oracle.tiling_bspline_sq(L, B, J_min)
    for j in range(J_min, J + 1):
        end = F(L, B ** (J - j - 2)) if J - j - 2 >= 0 else F(L * B ** (j + 2 - J))
        row = kap2[j - J_min]
        nz = [ell for ell in range(L) if row[ell] != 0]
        assert all(F(ell) < end for ell in nz)
        k = oracle.bandlimit_wav(j, L, B, True, "bspline")
        assert k == min(L, math.ceil(end))
        assert max(nz) == k - 1           # the band-limit is tight
        assert oracle.bandlimit_wav(j, L, B, False, "bspline") == L
    endP = F(L, B ** (J - J_min - 1))
    kP = oracle.bandlimit_scal(J_min, L, B, True, "bspline")
    assert kP == min(L, math.ceil(endP))
    assert max(ell for ell in range(L) if eta2[ell] != 0) == kP - 1


def test_bspline_bandlimits_worked_example():
    """Fig. 1 parameters (lambda = 3, J_0 = 2, L = 128, J = 5) and the denoising example's
    (lambda = 2, J_0 = 0, L = 128, J = 7)."""
    assert [oracle.bandlimit_wav(j, 128, 3, True, "bspline") for j in range(2, 6)] == [43, 128, 128, 128]
    assert oracle.bandlimit_scal(2, 128, 3, True, "bspline") == 15
    assert [oracle.bandlimit_wav(j, 128, 2, True, "bspline") for j in range(0, 8)] == \
        [4, 8, 16, 32, 64, 128, 128, 128]
    assert oracle.bandlimit_scal(0, 128, 2, True, "bspline") == 2


@pytest.mark.parametrize("L,B", [(128, 2), (128, 3), (512, 2)])
def test_bspline_peaks_track_sd_peaks(L, B):
    """The B-spline filters peak at about the scales of the scale-discretised ones (footnote
    to Sect. 2.2): peak positions agree within a factor sqrt(2) (a dropped factor 2 or B in
    the argument of Eq. (17) moves them by B or more)."""
    J_min = 1
    ks, _ = oracle.tiling(L, B, J_min, "sd")
    kb, _ = oracle.tiling(L, B, J_min, "bspline")
    for j in range(J_min, oracle.j_max(L, B)):
        ps, pb = int(np.argmax(ks[j - J_min])), int(np.argmax(kb[j - J_min]))
        assert 1 / math.sqrt(2) <= max(pb, 1) / max(ps, 1) <= math.sqrt(2), (j, ps, pb)


@pytest.mark.parametrize("L,B,J_min,multires,reality", [(16, 2, 0, True, True), (16, 2, 1, False, True),
                                                         (21, 3, 1, True, False), (32, 2, 2, True, True)])
def test_bspline_exact_reconstruction(L, B, J_min, multires, reality):
    flm = si.random_flm(L, 2, reality=reality, seed=31)
    f = oracle.inverse_sht(flm, L, reality)
    wav, scal = oracle.analysis(f, L, B, J_min, multires, reality, "bspline")
    rec = oracle.synthesis(wav, scal, L, B, J_min, multires, reality, "bspline")
    assert oracle.rel_max_err(rec, f) < 1e-12


def test_bspline_multires_equals_fullres():
    """Full-resolution scale maps carry no harmonic content at or above the multiresolution
    band-limit, and agree with the multiresolution maps on the coefficients below it."""
    L, B, J_min = 32, 2, 1
    flm = si.random_flm(L, 1, reality=True, seed=32)
    wf, sf = oracle.analysis_harmonic(flm, L, B, J_min, False, "bspline")
    wm, sm = oracle.analysis_harmonic(flm, L, B, J_min, True, "bspline")
    for j, a, b in zip(range(J_min, oracle.j_max(L, B) + 1), wf, wm):
        k = oracle.bandlimit_wav(j, L, B, True, "bspline")
        assert np.all(a[:, k * k:] == 0)
        assert np.array_equal(a[:, :k * k], b)
    kP = oracle.bandlimit_scal(J_min, L, B, True, "bspline")
    assert np.all(sf[:, kP * kP:] == 0) and np.array_equal(sf[:, :kP * kP], sm)


# ---------------------------------------------------------------- noise model (Sect. 4.3)
def test_noise_std_closed_form_sum():
    """With the tiling identity, sigma^2 sum_l (2l+1)/4pi (eta^2 + sum_j kappa_j^2) = sigma^2 L^2 / 4pi:
    the scale variances plus the scaling part's give the total."""
    for kernel in oracle.KERNELS:
        L, B, J_min, sigma = 64, 2, 1, 0.7
        sj = oracle.noise_std(L, B, J_min, sigma, kernel)
        _, eta = oracle.tiling(L, B, J_min, kernel)
        ell = np.arange(L)
        s_phi2 = sigma ** 2 * np.sum((2 * ell + 1) / (4 * math.pi) * eta ** 2)
        assert abs(np.sum(sj ** 2) + s_phi2 - sigma ** 2 * L * L / (4 * math.pi)) < 1e-12 * L * L


@pytest.mark.parametrize("kernel", ["sd", "bspline"])
def test_noise_std_monte_carlo(kernel):
    """E|N^j(omega)|^2 = sigma_j^2 at every sample: white noise with E|n_lm|^2 = sigma^2
    (Eq. (19)) run through the oracle's analysis; empirical second moments over 200 maps and
    all samples agree with sigma_j^2 within 5 standard errors."""
    L, B, J_min, sigma, nm = 16, 2, 0, 0.3, 200
    n_lm = si.random_flm(L, nm, reality=True, seed=77, cl=np.full(L, sigma ** 2))
    f = oracle.inverse_sht(n_lm, L, True)
    wav, _ = oracle.analysis(f, L, B, J_min, False, True, kernel)
    sj = oracle.noise_std(L, B, J_min, sigma, kernel)
    for w, s in zip(wav, sj):
        per_map = np.mean(np.abs(w) ** 2, axis=(1, 2))     # maps are independent draws
        se = np.std(per_map) / math.sqrt(nm)
        assert abs(np.mean(per_map) - s * s) < 5 * se + 1e-15, (np.mean(per_map), s * s, se)


# ---------------------------------------------------------------- thresholding and SNR
def test_hard_threshold_cases():
    w = [np.array([-5.0, -2.9, 0.0, 2.9, 3.0, 7.0]), np.array([1 + 1j, 3 + 4j, -0.5j])]
    d = oracle.hard_threshold(w, [3.0, 5.0])
    assert np.array_equal(d[0], [-5.0, 0.0, 0.0, 0.0, 3.0, 7.0])   # magnitude, |Y| = T kept
    assert np.array_equal(d[1], [0, 3 + 4j, 0])                     # |3+4i| = 5 kept
    assert np.array_equal(oracle.hard_threshold(w, [0.0, 0.0])[0], w[0])
    assert not np.any(oracle.hard_threshold(w, [np.inf, np.inf])[1])
    assert np.array_equal(w[0], [-5.0, -2.9, 0.0, 2.9, 3.0, 7.0])   # input untouched


def test_planted_signed_threshold_is_caught(monkeypatch):
    """Reading Eq. (23) without the magnitude would zero large negative coefficients."""
    def signed(wav, thresholds):
        return [np.where(np.real(w) < t, 0, w) for w, t in zip(wav, thresholds)]
    monkeypatch.setattr(oracle, "hard_threshold", signed)
    d = oracle.hard_threshold([np.array([-5.0, 7.0])], [3.0])
    assert d[0][0] != -5.0


def test_snr_closed_form():
    s = si.random_flm(16, 1, reality=True, seed=5)
    for c in (0.1, 0.5, 2.0):
        assert abs(oracle.snr(s, s + c * s) + 20 * math.log10(c)) < 1e-12
    n = si.random_flm(16, 1, reality=True, seed=6)
    e_s, e_n = np.sum(np.abs(s) ** 2), np.sum(np.abs(n) ** 2)
    assert abs(oracle.snr(s, s + n) - 10 * math.log10(e_s / e_n)) < 1e-12


@pytest.mark.parametrize("kernel", ["sd", "bspline"])
def test_denoise_identity_and_gain(kernel):
    """nsigma = 0 keeps every coefficient, so denoising returns y (exact reconstruction); at
    nsigma = 3 the denoised map is closer to s than y is."""
    L, B, J_min = 32, 2, 0
    s_lm, n_lm, sigma = si.denoise_workload(L, 1, seed=9)
    y = oracle.inverse_sht(s_lm + n_lm, L, True)
    d0 = oracle.denoise(y, L, B, J_min, sigma, True, True, kernel, nsigma=0.0)
    assert oracle.rel_max_err(d0, y) < 1e-12
    d = oracle.denoise(y, L, B, J_min, sigma, True, True, kernel)
    d_lm = oracle.forward_sht(d, L)
    snr_y, snr_d = oracle.snr(s_lm, s_lm + n_lm), oracle.snr(s_lm, d_lm)
    assert abs(snr_y - 11.78) < 1.5
    assert snr_d > snr_y + 0.5, (snr_y, snr_d)
