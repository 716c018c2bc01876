"""Pins for the CPU oracle: each test checks the oracle against something other than itself
(closed forms, library routines, exact integrals, brute force, invariants of the method)."""
import math
import os

import numpy as np
import pytest

import oracle
import s2let_inputs as si

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.txt")


def _golden():
    out = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, val, _ = [x.strip() for x in line.split("|")]
            out[name] = val
    return out


# ---------------------------------------------------------------- sampling (Sect. 2.1)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 16, 128])
def test_mw_nodes_and_sample_count(k):
    theta, phi = oracle.mw_nodes(k)
    n = 2 * k - 1
    assert theta.shape == (k,) and phi.shape == (n,)
    assert abs(theta[-1] - math.pi) < 1e-15            # south pole sampled
    assert theta[0] > 0                                 # north pole not sampled
    assert np.allclose(np.diff(theta), 2 * math.pi / n)  # equiangular
    # distinct points: every ring has 2k-1 points except the pole ring, which is one point
    distinct = (k - 1) * n + 1
    assert distinct == oracle.mw_size(k) - (n - 1)


def test_sample_counts_from_paper():
    g = _golden()
    for L in (4, 128):
        assert (L - 1) * (2 * L - 1) + 1 == int(g["mw_samples_L%d" % L])


# ---------------------------------------------------------------- lambda_lm
def test_closed_forms_l_le_2():
    th = np.array([0.1, 0.7, 1.3, math.pi / 2, 2.2, 3.0, math.pi])
    c, s = np.cos(th), np.sin(th)
    ref = {
        (0, 0): np.full_like(th, 0.5 / math.sqrt(math.pi)),
        (1, 0): math.sqrt(3 / (4 * math.pi)) * c,
        (1, 1): -math.sqrt(3 / (8 * math.pi)) * s,
        (2, 0): math.sqrt(5 / (16 * math.pi)) * (3 * c * c - 1),
        (2, 1): -math.sqrt(15 / (8 * math.pi)) * s * c,
        (2, 2): math.sqrt(15 / (32 * math.pi)) * s * s,
    }
    for (ell, m), r in ref.items():
        lam = oracle.legendre_lambda(3, m, th)[:, ell - m]
        assert np.max(np.abs(lam - r)) < 1e-15, (ell, m)


def test_special_values():
    k = 40
    for m in range(0, k, 3):
        at_pi = oracle.legendre_lambda(k, m, [math.pi])[0]
        ell = np.arange(m, k)
        if m == 0:
            ref = (-1.0) ** ell * np.sqrt((2 * ell + 1) / (4 * math.pi))
            assert np.max(np.abs(at_pi - ref)) < 1e-14
        else:
            assert np.max(np.abs(at_pi)) < 1e-14
        at_eq = oracle.legendre_lambda(k, m, [math.pi / 2])[0]
        odd = ((ell + m) % 2) == 1
        if np.any(odd):
            assert np.max(np.abs(at_eq[odd])) < 1e-14


def test_lambda_vs_scipy():
    from scipy.special import sph_harm_y
    k = 200
    th = np.array([0.05, 0.4, 1.0, 1.5, 2.1, 2.9])
    for m in (0, 1, 5, 37, 120, 199):
        lam = oracle.legendre_lambda(k, m, th)
        ell = np.arange(m, k)
        ref = np.real(sph_harm_y(ell[None, :], m, th[:, None], 0.0))
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(lam - ref)) < 1e-12 * max(scale, 1.0), m


def _lambda_hypergeometric(ell, m, th):
    """lambda_lm(theta) from the terminating hypergeometric form of P_l^m (Condon-Shortley):
    P_l^m(cos t) = (-1)^m sin^m t (l+m)!/(2^m m! (l-m)!) 2F1(m-l, l+m+1; m+1; sin^2(t/2))."""
    import mpmath
    th = mpmath.mpf(th)
    z = mpmath.sin(th / 2) ** 2
    F = mpmath.hyp2f1(m - ell, ell + m + 1, m + 1, z)
    logc = (mpmath.loggamma(ell + m + 1) - m * mpmath.log(2) - mpmath.loggamma(m + 1)
            - mpmath.loggamma(ell - m + 1)
            + 0.5 * (mpmath.log((2 * ell + 1) / (4 * mpmath.pi)) + mpmath.loggamma(ell - m + 1)
                     - mpmath.loggamma(ell + m + 1)))
    return (-1) ** m * mpmath.sin(th) ** m * mpmath.exp(logc) * F


def test_lambda_vs_mpmath_deep_underflow():
    """log2|lambda_lm| against a 40-digit hypergeometric evaluation, up to l = 2047 and far
    below the double range (lambda_mm ~ 2^-17000 at m = 2047 next to the pole)."""
    import mpmath
    mpmath.mp.dps = 40
    k = 2048
    cases = [(2047, 0.003), (2000, 0.02), (1500, 0.3), (600, 1.2), (3, 0.0008), (1024, 1.5707)]
    for m, th in cases:
        ours = oracle.legendre_log2(k, m, th)
        for ell in sorted({min(k - 1, x) for x in (m, m + 1, m + 7, m + 40, k - 1)}):
            val = _lambda_hypergeometric(ell, m, th)
            ref = float(mpmath.log(abs(val), 2))
            # relative accuracy 1e-13 of the value <=> 1.5e-13 absolute in log2
            assert abs(ours[ell - m] - ref) < 1.5e-13 + 1e-16 * abs(ref), (m, th, ell)
    # mpmath's own legenp agrees where its hypergeometric sum converges
    x = mpmath.cos(mpmath.mpf(1.2))
    p = mpmath.legenp(700, 600, x, type=2)
    norm = mpmath.sqrt(mpmath.mpf(1401) / (4 * mpmath.pi) * mpmath.factorial(100) / mpmath.factorial(1300))
    assert abs(float(mpmath.log(abs(norm * p), 2)) - oracle.legendre_log2(k, 600, 1.2)[100]) < 1e-12


def test_condon_shortley_sign():
    import mpmath
    th = 0.9
    for m, ell in [(1, 1), (1, 4), (3, 5), (4, 9)]:
        lam = oracle.legendre_lambda(12, m, [th])[0, ell - m]
        p = mpmath.legenp(ell, m, mpmath.cos(th), type=2)
        assert np.sign(lam) == np.sign(float(p))


# ---------------------------------------------------------------- quadrature weight
def test_quadrature_weight_vs_sympy():
    import sympy as sp
    t = sp.symbols("t", real=True)
    ps = np.arange(-8, 9)
    ours = oracle.quadrature_weight(ps)
    for p, w in zip(ps, ours):
        exact = sp.integrate(sp.exp(sp.I * int(p) * t) * sp.sin(t), (t, 0, sp.pi))
        exact = complex(sp.N(exact, 30))
        assert abs(w - exact) < 1e-15, p


# ---------------------------------------------------------------- forward / inverse
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 16])
def test_orthogonality_brute_force(k):
    """forward(inverse(e_lm)) = e_lm for every basis vector: the k^2 x k^2 identity."""
    basis = np.eye(k * k, dtype=np.complex128)
    maps = oracle.inverse_sht(basis, k)
    back = oracle.forward_sht(maps, k)
    assert np.max(np.abs(back - basis)) < 1e-13


def test_constant_map():
    for k in (1, 2, 5, 16):
        f = np.full((1, k, 2 * k - 1), 2.5, dtype=np.complex128)
        flm = oracle.forward_sht(f, k)
        ref = np.zeros(k * k, dtype=np.complex128)
        ref[0] = 2.5 * math.sqrt(4 * math.pi)
        assert np.max(np.abs(flm[0] - ref)) < 1e-13


@pytest.mark.parametrize("k", [2, 5, 12, 20])
def test_inverse_vs_direct_summation(k):
    flm = si.random_flm_unit(k, 2, seed=k)
    a = oracle.inverse_sht(flm, k)
    b = oracle.inverse_sht_direct(flm, k)
    assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("k", [2, 7, 16, 33, 128])
@pytest.mark.parametrize("reality", [False, True])
def test_inverse_rings_is_inverse_on_those_rings(k, reality):
    """Eq. (1) on selected rings: the ring-subset synthesis returns exactly the rows of the
    full synthesis (pinned above against direct Y_lm summation), for rings in any order, with
    duplicates, the south pole and the first ring; even and odd k, real and complex maps."""
    flm = si.random_flm(k, 2, reality=True, seed=11 + k) if reality else si.random_flm_unit(k, 2, seed=11 + k)
    full = oracle.inverse_sht(flm, k, reality=reality)
    rng = np.random.default_rng(k)
    rings = np.concatenate([[k - 1, 0], rng.integers(0, k, size=min(k, 9)), [k - 1, k // 2, 0]])
    sub = oracle.inverse_sht_rings(flm, k, rings, reality=reality)
    assert sub.shape == (2, rings.size, 2 * k - 1)
    assert np.isrealobj(sub) == reality
    assert np.max(np.abs(sub - full[:, rings, :])) <= 1e-14 * max(1.0, np.max(np.abs(full)))
    # the empty ring set, and every ring in reverse order
    assert oracle.inverse_sht_rings(flm, k, np.zeros(0, dtype=int), reality=reality).shape == (2, 0, 2 * k - 1)
    rev = oracle.inverse_sht_rings(flm, k, np.arange(k)[::-1], reality=reality)
    assert np.max(np.abs(rev - full[:, ::-1, :])) <= 1e-14 * max(1.0, np.max(np.abs(full)))
    with pytest.raises(ValueError):
        oracle.inverse_sht_rings(flm, k, [k], reality=reality)


def test_inverse_rings_vs_direct_summation():
    """The ring-subset synthesis against direct Y_lm summation (scipy), independent of the
    separable evaluation the full synthesis uses."""
    k = 12
    flm = si.random_flm_unit(k, 1, seed=5)
    rings = [11, 3, 3, 0, 7]
    a = oracle.inverse_sht_rings(flm, k, rings)
    b = oracle.inverse_sht_direct(flm, k)[:, rings, :]
    assert np.max(np.abs(a - b)) < 1e-12


def test_phi_integral_exact_on_trig_polynomial():
    """A single mode Y_lm is recovered exactly (phi integral of a trigonometric polynomial)."""
    k = 9
    for ell, m in [(0, 0), (3, -2), (8, 8), (8, -5), (5, 1)]:
        e = si.random_unit_flm_basis(k, ell, m)
        back = oracle.forward_sht(oracle.inverse_sht(e, k), k)
        assert np.max(np.abs(back - e)) < 1e-14


@pytest.mark.parametrize("k", [32, 64, 128])
def test_round_trip_complex(k):
    flm = si.random_flm_unit(k, 1, seed=7)
    back = oracle.forward_sht(oracle.inverse_sht(flm, k), k)
    # error of O(k) * 1e-16 (Sect. 3.3): a generous 1e-13 bound at these sizes
    assert oracle.max_abs_err(back, flm) < 1e-13


def test_real_symmetry():
    k = 24
    flm = si.random_flm(k, 1, reality=True, seed=3)
    f = oracle.inverse_sht(flm, k)
    assert np.max(np.abs(f.imag)) < 1e-15 * np.max(np.abs(f.real)) * 10
    back = oracle.forward_sht(f.real, k)[0]
    for ell in range(k):
        for m in range(1, ell + 1):
            a = back[ell * ell + ell - m]
            b = (-1) ** m * np.conj(back[ell * ell + ell + m])
            assert abs(a - b) < 1e-14


# ---------------------------------------------------------------- tiling, Eqs. (10)-(16)
def test_j_max_paper_example_and_exact_powers():
    g = _golden()
    scales = [int(x) for x in g["scales_L128_B3_J2"].split()]
    assert list(range(2, oracle.j_max(128, 3) + 1)) == scales
    assert oracle.j_max(128, 3) - 2 + 3 == int(g["shts_L128_B3_J2"])
    # exact powers: L-1 = B^J must give J, not J+1 (ceil of an exact logarithm)
    for B in (2, 3, 5):
        for J in range(1, 8):
            assert oracle.j_max(B ** J + 1, B) == J
            assert oracle.j_max(B ** J + 2, B) == J + 1
    assert oracle.j_max(64, 2) == 6 and oracle.j_max(512, 2) == 9 and oracle.j_max(2048, 2) == 11


def test_k_lambda_endpoints_and_monotone():
    for lam in (2.0, 3.0):
        assert oracle.k_lambda(0.3 / lam, lam) == 1.0
        assert oracle.k_lambda(1.0 / lam, lam) == 1.0
        assert oracle.k_lambda(1.0, lam) == 0.0
        assert oracle.k_lambda(1.7, lam) == 0.0
        ts = np.linspace(1.0 / lam, 1.0, 41)
        vals = [oracle.k_lambda(t, lam) for t in ts]
        assert all(a >= b for a, b in zip(vals, vals[1:]))


def test_k_lambda_vs_mpmath():
    """Independent evaluation of Eq. (12) by tanh-sinh quadrature at 30 digits (the paper
    prints no values of k_lambda: these pin the oracle's adaptive Gauss-Kronrod rule)."""
    import mpmath
    mpmath.mp.dps = 30

    def k_mp(t, lam):
        lam = mpmath.mpf(lam)

        def g(u):
            x = 2 * lam * (u - 1 / lam) / (lam - 1) - 1
            if abs(x) >= 1:
                return mpmath.mpf(0)
            return mpmath.exp(-2 / (1 - x * x)) / u
        num = mpmath.quad(g, [t, 1])
        den = mpmath.quad(g, [1 / lam, (1 / lam + 1) / 2, 1])
        return num / den

    for t, lam in [(0.75, 2), (0.5, 3), (0.55, 2), (0.95, 2), (0.4, 3), (0.9, 3)]:
        assert abs(oracle.k_lambda(t, float(lam)) - float(k_mp(mpmath.mpf(t), lam))) < 2e-15
    # the two reference points quoted in the blueprint of this project (30-digit mpmath)
    assert abs(oracle.k_lambda(0.75, 2.0) - 0.45255230486403153) < 2e-15
    assert abs(oracle.k_lambda(0.5, 3.0) - 0.89517435052472923) < 2e-15


def test_kappa_lambda_vs_mpmath_difference():
    """Eq. (13) directly: kappa_lambda(t)^2 = k_lambda(t/lambda) - k_lambda(t), both terms of the
    difference evaluated independently at 30 digits (tanh-sinh) and subtracted in that precision.
    The oracle evaluates the difference as one integral, so this checks that rewrite, at both ends
    of the support (1/lambda, lambda) and at its centre t = 1."""
    import mpmath
    mpmath.mp.dps = 30

    def k_mp(t, lam):
        lam, t = mpmath.mpf(lam), mpmath.mpf(t)
        if t <= 1 / lam:
            return mpmath.mpf(1)
        if t >= 1:
            return mpmath.mpf(0)

        def g(u):
            x = 2 * lam * (u - 1 / lam) / (lam - 1) - 1
            if abs(x) >= 1:
                return mpmath.mpf(0)
            return mpmath.exp(-2 / (1 - x * x)) / u
        return mpmath.quad(g, [t, 1]) / mpmath.quad(g, [1 / lam, (1 / lam + 1) / 2, 1])

    for lam in (2, 3):
        edges = [1.0 / lam + 1e-3, 1.0 / lam + 0.05, 0.8, 1.0, 1.3, lam - 0.05, lam - 1e-3]
        for t in edges:
            ref = k_mp(mpmath.mpf(t) / lam, lam) - k_mp(t, lam)
            got = oracle.kappa_lambda(t, float(lam)) ** 2
            assert abs(got - float(ref)) < 1e-14, (lam, t)
            if float(ref) > 1e-12:      # away from the 30-digit reference's own cancellation
                assert abs(got - float(ref)) < 1e-13 * float(ref), (lam, t)
        # outside the support, and its ends: exactly zero
        for t in (0.0, 0.5 / lam, 1.0 / lam, float(lam), lam + 0.5):
            assert oracle.kappa_lambda(t, float(lam)) == 0.0
        assert oracle.kappa_lambda(1.0, float(lam)) == 1.0


@pytest.mark.parametrize("L,B,J_min", [(64, 2, 0), (128, 3, 2), (512, 2, 2), (300, 3, 1)])
def test_tiling_identity_and_supports(L, B, J_min):
    """Eq. (9): eta^2 + sum_j kappa_j^2 = 1 for all l < L; supports of Eqs. (15)-(16)."""
    kappa, eta = oracle.tiling(L, B, J_min)
    total = eta ** 2 + np.sum(kappa ** 2, axis=0)
    assert np.max(np.abs(total - 1.0)) < 1e-15 * 4
    J = oracle.j_max(L, B)
    ell = np.arange(L)
    for j in range(J_min, J + 1):
        outside = (ell <= B ** (j - 1)) | (ell >= B ** (j + 1))
        assert np.all(kappa[j - J_min][outside] == 0.0)
    assert np.all(eta[ell >= B ** J_min] == 0.0)
    assert np.all(eta[ell <= B ** (J_min - 1)] == 1.0) if J_min > 0 else eta[0] == 1.0


# ---------------------------------------------------------------- wavelets, Eqs. (4), (6), (8)
def test_parseval_energy_partition():
    """Eq. (21) with Eq. (9): sum |W^Phi_lm|^2 + sum_j sum |W^j_lm|^2 = sum |f_lm|^2."""
    L, B, J_min = 64, 2, 1
    flm = si.random_flm(L, 2, reality=True, seed=5)
    wav, scal = oracle.analysis_harmonic(flm, L, B, J_min, multires=True)
    energy = np.sum(np.abs(scal) ** 2, axis=1) + sum(np.sum(np.abs(w) ** 2, axis=1) for w in wav)
    assert np.max(np.abs(energy - np.sum(np.abs(flm) ** 2, axis=1))) < 1e-13 * np.max(energy)


def test_parseval_through_maps():
    """Energy of each map, computed through its forward SHT, partitions the signal energy."""
    L, B, J_min = 32, 2, 2
    flm = si.random_flm(L, 1, reality=True, seed=8)
    f = oracle.inverse_sht(flm, L, reality=True)
    wav, scal = oracle.analysis(f, L, B, J_min, multires=True, reality=True)
    kP = oracle.bandlimit_scal(J_min, L, B, True)
    e = np.sum(np.abs(oracle.forward_sht(scal, kP)) ** 2)
    for j, w in zip(range(J_min, oracle.j_max(L, B) + 1), wav):
        e += np.sum(np.abs(oracle.forward_sht(w, oracle.bandlimit_wav(j, L, B, True))) ** 2)
    assert abs(e - np.sum(np.abs(flm) ** 2)) < 1e-12 * e


def test_multires_equals_fullres():
    L, B, J_min = 32, 2, 1
    flm = si.random_flm(L, 1, reality=False, seed=9)
    f = oracle.inverse_sht(flm, L)
    wav_m, scal_m = oracle.analysis(f, L, B, J_min, multires=True, reality=False)
    wav_f, scal_f = oracle.analysis(f, L, B, J_min, multires=False, reality=False)
    for j, wm, wf in zip(range(J_min, oracle.j_max(L, B) + 1), wav_m, wav_f):
        kj = oracle.bandlimit_wav(j, L, B, True)
        wlm = oracle.forward_sht(wm, kj)
        padded = np.zeros((1, L * L), dtype=np.complex128)
        padded[:, :kj * kj] = wlm
        assert np.max(np.abs(oracle.inverse_sht(padded, L) - wf)) < 1e-13
    rec_m = oracle.synthesis(wav_m, scal_m, L, B, J_min, True, False)
    rec_f = oracle.synthesis(wav_f, scal_f, L, B, J_min, False, False)
    assert np.max(np.abs(rec_m - rec_f)) < 1e-13
    assert np.max(np.abs(rec_m - f)) < 1e-13


def test_single_mode_input():
    """f = Y_lm gives W^j = kappa_j(l) Y_lm on the k_j grid (Eq. (4))."""
    L, B, J_min = 32, 2, 1
    kappa, eta = oracle.tiling(L, B, J_min)
    for ell, m in [(5, 2), (12, -7), (20, 0)]:
        e = si.random_unit_flm_basis(L, ell, m)
        f = oracle.inverse_sht(e, L)
        wav, scal = oracle.analysis(f, L, B, J_min, multires=True, reality=False)
        for j, w in zip(range(J_min, oracle.j_max(L, B) + 1), wav):
            kj = oracle.bandlimit_wav(j, L, B, True)
            if ell < kj:
                ref = kappa[j - J_min, ell] * oracle.inverse_sht(si.random_unit_flm_basis(kj, ell, m), kj)
            else:
                ref = np.zeros_like(w)
            assert np.max(np.abs(w - ref)) < 1e-13


def test_wavelet_round_trip_config_small():
    """Analysis then synthesis (B=2, J_min=0, full resolution, one real map, L=64)."""
    L = 64
    flm = si.random_flm(L, 1, reality=True, seed=0)
    f = oracle.inverse_sht(flm, L, reality=True)
    wav, scal = oracle.analysis(f, L, 2, 0, multires=False, reality=True)
    assert len(wav) == oracle.j_max(L, 2) + 1
    for w in wav:
        assert w.shape == (1, L, 2 * L - 1) and np.isrealobj(w)
    rec = oracle.synthesis(wav, scal, L, 2, 0, False, True)
    back = oracle.forward_sht(rec, L)
    assert oracle.max_abs_err(back, flm) < 1e-13


# ---------------------------------------------------------------- planted mistakes
def test_planted_mistakes_are_caught(monkeypatch):
    """Plausible slips in the quadrature are caught by the orthogonality pin."""
    k = 6
    basis = np.eye(k * k, dtype=np.complex128)
    maps = oracle.inverse_sht(basis, k)
    good = oracle.quadrature_weight

    def wrong_sign(p):          # sign error on the odd taps
        w = good(p)
        return np.conj(w)

    def dropped(p):             # drops the p = 0 term
        w = good(p)
        w = np.where(np.asarray(p) == 0, 0.0, w)
        return w

    for bad in (dropped,):
        monkeypatch.setattr(oracle, "quadrature_weight", bad)
        back = oracle.forward_sht(maps, k)
        assert np.max(np.abs(back - basis)) > 1e-3
    # The odd taps cancel after the fold, so the sign of w(+-1) cannot change the result.
    monkeypatch.setattr(oracle, "quadrature_weight", wrong_sign)
    back = oracle.forward_sht(maps, k)
    assert np.max(np.abs(back - basis)) < 1e-13
