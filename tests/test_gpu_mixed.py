"""Mixed precision: the Legendre contraction on the FP32 matrix cores (FP32 operands, FP32
accumulation over runs of at most 64 terms, then FP64), the recursion and everything else in
FP64.  Checked against the FP64 oracle on the same seeded inputs.

Stated bound (relative max error, max|gpu - oracle| / max|oracle|): 2e-6 for the harmonic
transforms and wavelet maps up to L = 512.  Each product carries the FP32 rounding of both
operands (2 x 2^-24) and each 64-term FP32 run adds at most 64 x 2^-24 relative to the sum of
the magnitudes it accumulates; the measured errors stay near 1e-7 to 1e-6 and the bound leaves
headroom for the growth with L.  Batches below 16 columns (fewer than 8 real maps) run the
synthesis contraction in FP64 on the vector units, so there the bound is met with room."""
import sys

import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")

TOL_FP32 = 2e-6


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _errs(got, ref, floor=0.0):
    got, ref = np.asarray(got), np.asarray(ref)
    den = max(float(np.max(np.abs(ref))), floor)
    d = np.abs(got - ref)
    mx = float(np.max(d)) / den
    rms = float(np.sqrt(np.mean(d * d))) / den
    _log("  rel max err %.3e  rel rms err %.3e" % (mx, rms))
    return mx, rms


def _to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("nmaps,reality", [(16, s2.REAL), (8, s2.COMPLEX), (8, s2.REAL), (2, s2.REAL)])
@pytest.mark.parametrize("L", [16, 64, 257])
def test_fp32_harmonic_transforms(dev, L, nmaps, reality):
    _log("fp32 inverse/forward L=%d nmaps=%d reality=%d" % (L, nmaps, reality))
    real = reality == s2.REAL
    flm = si.random_flm(L, nmaps, reality=real, seed=500 + L + nmaps)
    ref = oracle.inverse_sht(flm, L, reality=real)
    f32 = s2.mw_inverse(_to_dev(flm, dev), L, reality, precision=s2.MIXED_FP32)
    assert _errs(f32.cpu().numpy(), ref)[0] < TOL_FP32
    back = s2.mw_forward(_to_dev(ref, dev), L, reality, precision=s2.MIXED_FP32).cpu().numpy()
    assert _errs(back, flm)[0] < TOL_FP32
    # the FP64 path is unaffected by the mode of earlier calls
    f64 = s2.mw_inverse(_to_dev(flm, dev), L, reality).cpu().numpy()
    assert oracle.rel_max_err(f64, ref) < 1e-10


def test_fp32_wavelets_per_scale(dev):
    """16 real maps, L=128, B=2, J_min=2, multiresolution: FP32 analysis and synthesis, max and RMS
    error against the FP64 oracle for every scale."""
    L, B, J_min, nm = 128, 2, 2, 16
    flm = si.random_flm(L, 2, reality=True, seed=7)
    f2 = oracle.inverse_sht(flm, L, reality=True)
    f = np.concatenate([f2] * (nm // 2))
    wav_ref, scal_ref = oracle.analysis(f2, L, B, J_min, True, True)
    fd = _to_dev(f, dev)
    f_wav, f_scal = s2.analysis(fd, L, B, J_min, True, s2.REAL, precision=s2.MIXED_FP32)
    got = [w.cpu().numpy() for w in s2.split_wav(f_wav, L, B, J_min, True)]
    kP = oracle.bandlimit_scal(J_min, L, B, True)
    floor = 1e-6 * float(np.max(np.abs(f)))
    _log("scaling map k=%d" % kP)
    assert _errs(f_scal.cpu().numpy()[:2].reshape(2, kP, 2 * kP - 1), scal_ref, floor)[0] < TOL_FP32
    for j, (g, r) in enumerate(zip(got, wav_ref)):
        _log("scale j=%d" % (J_min + j))
        assert _errs(g[:2], r, floor)[0] < TOL_FP32
    rec = s2.synthesis(f_wav, f_scal, L, B, J_min, True, s2.REAL, precision=s2.MIXED_FP32)
    _log("reconstruction")
    assert _errs(rec.cpu().numpy()[:2], f2)[0] < TOL_FP32


def test_fp32_config_512_complex_side_by_side(dev):
    """One complex map, L=512, B=2, J_min=2, multiresolution, FP64 and FP32 side by side."""
    L, B, J_min = 512, 2, 2
    flm = si.random_flm(L, 1, reality=False, seed=1)
    f = oracle.inverse_sht(flm, L)
    fd = _to_dev(f, dev)
    out = {}
    for name, prec in (("fp64", s2.FP64), ("fp32", s2.MIXED_FP32)):
        _log(name)
        got_flm = s2.mw_forward(fd, L, s2.COMPLEX, precision=prec).cpu().numpy()
        out[name] = _errs(got_flm, flm)[0]
        f_wav, f_scal = s2.analysis(fd, L, B, J_min, True, s2.COMPLEX, precision=prec)
        rec = s2.synthesis(f_wav, f_scal, L, B, J_min, True, s2.COMPLEX, precision=prec)
        out[name + "_rec"] = _errs(rec.cpu().numpy(), f)[0]
    assert out["fp64"] < 1e-10 and out["fp64_rec"] < 1e-10
    assert out["fp32"] < TOL_FP32 and out["fp32_rec"] < TOL_FP32
