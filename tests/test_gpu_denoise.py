"""B-spline wavelets (footnote to Sect. 2.2, Eqs. (17)-(18)) and hard-threshold denoising
(Sect. 4.3, Eqs. (19)-(23)) on the GPU, through the C ABI, against the oracle.

  - B-spline analysis and synthesis parity (relative max error <= 1e-10) over band-limits that
    span several tiles with ragged tails, real and complex maps, full and multi resolution;
  - B-spline transform at L = 1024 (2 real maps): reconstruction, and scale maps on rings the
    oracle evaluates one by one;
  - the threshold kernel bit for bit against the oracle's Eq. (23) on the same input;
  - the denoising workload: 4 real maps, L = 128, lambda = 2, J_0 = 0, multiresolution, signal
    C_l = (l+1)^-3, white noise with SNR(y) = 11.78 dB, seed 9 (synthetic stand-in for the
    Earth topography map of Sect. 4.3).  Every threshold decision is first shown to be unique
    (no coefficient within 1e-9 of its threshold in the oracle), then the GPU's denoised maps
    are compared with the oracle's (1e-10) and the SNR gain is checked."""
import sys

import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")

TOL = 1e-10
NAME = {s2.KERNEL_SD: "sd", s2.KERNEL_BSPLINE: "bspline"}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref, floor=0.0):
    got, ref = np.asarray(got), np.asarray(ref)
    den = max(float(np.max(np.abs(ref))) if ref.size else 0.0, floor)
    r = float(np.max(np.abs(got - ref))) / den if den > 0 else float(np.max(np.abs(got - ref)))
    _log("  rel err %.3e" % r)
    return r


def _to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("L,B,J_min,multires,reality", [
    (16, 2, 0, True, s2.REAL), (32, 3, 1, True, s2.COMPLEX), (50, 3, 2, True, s2.REAL),
    (64, 2, 1, False, s2.REAL), (128, 2, 0, True, s2.REAL), (130, 2, 3, True, s2.COMPLEX),
    (257, 3, 2, True, s2.REAL)])
def test_bspline_parity(dev, L, B, J_min, multires, reality):
    _log("bspline parity L=%d B=%d J_min=%d multires=%d reality=%d" % (L, B, J_min, multires, reality))
    real = reality == s2.REAL
    K = s2.KERNEL_BSPLINE
    flm = si.random_flm(L, 3, reality=real, seed=60 + L)
    f = oracle.inverse_sht(flm, L, real)
    wav_ref, scal_ref = oracle.analysis(f, L, B, J_min, multires, real, "bspline")
    f_wav, f_scal = s2.analysis(_to_dev(f, dev), L, B, J_min, multires, reality, kernel=K)
    floor = 1e-6 * float(np.max(np.abs(f)))
    for g, r in zip(s2.split_wav(f_wav, L, B, J_min, multires, K), wav_ref):
        assert _rel(g.cpu().numpy(), r, floor) < TOL
    assert _rel(f_scal.cpu().numpy().reshape(scal_ref.shape), scal_ref, floor) < TOL
    rec = s2.synthesis(f_wav, f_scal, L, B, J_min, multires, reality, kernel=K)
    assert _rel(rec.cpu().numpy(), f) < TOL
    # synthesis of arbitrary (inconsistent) scale maps
    rng = np.random.default_rng(L)

    def rmap(k):
        x = rng.standard_normal((3, k, 2 * k - 1))
        return x if real else x + 1j * rng.standard_normal((3, k, 2 * k - 1))

    J = oracle.j_max(L, B)
    wav = [rmap(oracle.bandlimit_wav(j, L, B, multires, "bspline")) for j in range(J_min, J + 1)]
    scal = rmap(oracle.bandlimit_scal(J_min, L, B, multires, "bspline"))
    got = s2.synthesis(_to_dev(np.concatenate([w.reshape(3, -1) for w in wav], axis=1), dev),
                       _to_dev(scal.reshape(3, -1), dev), L, B, J_min, multires, reality, kernel=K)
    assert _rel(got.cpu().numpy(), oracle.synthesis(wav, scal, L, B, J_min, multires, real, "bspline")) < TOL


def test_bspline_L1024(dev):
    L, B, J_min = 1024, 2, 2
    K = s2.KERNEL_BSPLINE
    _log("bspline L=1024: oracle synthesis of 2 maps")
    flm = si.random_flm(L, 2, reality=True, seed=61)
    f = oracle.inverse_sht(flm, L, reality=True)
    f_wav, f_scal = s2.analysis(_to_dev(f, dev), L, B, J_min, True, s2.REAL, kernel=K)
    rec = s2.synthesis(f_wav, f_scal, L, B, J_min, True, s2.REAL, kernel=K)
    assert _rel(rec.cpu().numpy(), f) < TOL
    wav_lm, scal_lm = oracle.analysis_harmonic(flm, L, B, J_min, True, "bspline")
    floor = 1e-6 * float(np.max(np.abs(f)))
    J = oracle.j_max(L, B)
    for j, g, wlm in zip(range(J_min, J + 1), s2.split_wav(f_wav, L, B, J_min, True, K), wav_lm):
        k = g.shape[1]
        rings = sorted({0, 1, k // 2, k - 2, k - 1}) if k > 64 else list(range(k))
        _log("  scale j=%d k=%d rings %s" % (j, k, rings if len(rings) < 8 else "all"))
        ref = oracle.inverse_sht_rings(wlm, k, rings, reality=True)
        assert _rel(g.cpu().numpy()[:, rings, :], ref, floor) < TOL
    kP = oracle.bandlimit_scal(J_min, L, B, True, "bspline")
    ref = oracle.inverse_sht(scal_lm, kP, reality=True)
    assert _rel(f_scal.cpu().numpy().reshape(ref.shape), ref, floor) < TOL


@pytest.mark.parametrize("reality", [s2.REAL, s2.COMPLEX])
@pytest.mark.parametrize("kernel", [s2.KERNEL_SD, s2.KERNEL_BSPLINE])
def test_hard_threshold_bit_exact(dev, reality, kernel):
    L, B, J_min, nm = 64, 2, 1, 3
    real = reality == s2.REAL
    rng = np.random.default_rng(62)
    n = s2.wav_size(L, B, J_min, True, kernel)
    x = rng.standard_normal((nm, n))
    if not real:
        x = x + 1j * rng.standard_normal((nm, n))
    ns = oracle.j_max(L, B) - J_min + 1
    thr = np.linspace(0.5, 1.5, ns)
    thr[0], thr[-1] = 0.0, np.inf                  # keep everything / drop everything
    ks = [oracle.bandlimit_wav(j, L, B, True, NAME[kernel]) for j in range(J_min, J_min + ns)]
    splits = np.cumsum([k * (2 * k - 1) for k in ks])[:-1]
    ref = np.concatenate(oracle.hard_threshold(np.split(x, splits, axis=1), thr), axis=1)
    # decisions are unique: no magnitude within 1e-13 of a finite threshold
    for part, t in zip(np.split(x, splits, axis=1), thr):
        if np.isfinite(t) and t > 0:
            assert np.min(np.abs(np.abs(part) - t)) > 1e-13 * t
    g = _to_dev(x, dev)
    s2.hard_threshold(g, thr, L, B, J_min, True, reality, kernel)
    got = g.cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.count_nonzero(ref) not in (0, ref.size)


@pytest.mark.parametrize("kernel", [s2.KERNEL_SD, s2.KERNEL_BSPLINE])
def test_denoising_workload(dev, kernel):
    L, B, J_min, nm = 128, 2, 0, 4
    name = NAME[kernel]
    _log("denoising workload kernel=%s" % name)
    s_lm, n_lm, sigma = si.denoise_workload(L, nm, seed=9)
    y = oracle.inverse_sht(s_lm + n_lm, L, True)
    # unique decisions in the oracle
    wav, _ = oracle.analysis(y, L, B, J_min, True, True, name)
    T = 3.0 * oracle.noise_std(L, B, J_min, sigma, name)
    margin = min(float(np.min(np.abs(np.abs(w) - t) / t)) for w, t in zip(wav, T))
    _log("  closest coefficient to its threshold: %.3e (relative)" % margin)
    assert margin > 1e-9
    assert np.max(np.abs(s2.noise_std(L, B, J_min, sigma, kernel) * 3.0 - T) / T) < 1e-14
    d_ref = oracle.denoise(y, L, B, J_min, sigma, True, True, name)
    d = s2.denoise(_to_dev(y, dev), L, B, J_min, sigma, True, s2.REAL, kernel)
    assert _rel(d.cpu().numpy(), d_ref) < TOL
    d_lm = s2.mw_forward(d, L, s2.REAL).cpu().numpy()
    for i in range(nm):
        snr_y = oracle.snr(s_lm[i], s_lm[i] + n_lm[i])
        snr_d = oracle.snr(s_lm[i], d_lm[i])     # the energies of the GPU's result (Eqs. (20)-(21))
        snr_d_ref = oracle.snr(s_lm[i], oracle.forward_sht(d_ref[i:i + 1], L)[0])
        _log("  map %d: SNR(y) %.3f dB  SNR(d) %.3f dB (oracle %.3f dB)" % (i, snr_y, snr_d, snr_d_ref))
        assert abs(snr_d - snr_d_ref) < 1e-8
        assert snr_d > snr_y + 2.0
