"""Mixed precision: the Legendre contraction on lower-precision matrix cores, the recursion and
everything else in FP64, checked against the FP64 oracle on the same seeded inputs.

  MIXED_FP32:   FP32 operands, FP32 accumulation over runs of at most 64 terms, then FP64.
  MIXED_BF16X3: operands split x = x_hi + x_lo into two bfloat16 parts, three products
                (hi hi + hi lo + lo hi) in FP32 on the BF16 matrix cores, FP64 every 64 terms.

Stated bounds (relative max error, max|gpu - oracle| / max|oracle|), up to L = 512:
  FP32: 2e-6.  Each product carries the FP32 rounding of both operands (2 x 2^-24) and each
        64-term FP32 run adds at most 64 x 2^-24 of the magnitudes it sums; measured 1e-7..3e-7.
  BF16x3: 1e-4.  The split leaves about 2^-17 of each operand and the dropped lo x lo term is
        about 2^-18 of the product, so each product is good to about 2^-16 (1.5e-5); the
        accumulation adds the FP32 terms above.
Batches below 16 columns (fewer than 8 real maps) run the synthesis contraction in FP64 on the
vector units, so there the bounds are met with room."""
import sys

import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")

TOL_FP32 = 2e-6
TOL = {"fp32": TOL_FP32, "bf16x3": 1e-4}
PREC = {"fp32": s2.MIXED_FP32, "bf16x3": s2.MIXED_BF16X3}


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


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nmaps,reality", [(16, s2.REAL), (8, s2.COMPLEX), (8, s2.REAL), (2, s2.REAL)])
@pytest.mark.parametrize("L", [16, 64, 257])
def test_mixed_harmonic_transforms(dev, L, nmaps, reality, mode):
    _log("%s inverse/forward L=%d nmaps=%d reality=%d" % (mode, L, nmaps, reality))
    real = reality == s2.REAL
    flm = si.random_flm(L, nmaps, reality=real, seed=500 + L + nmaps)
    ref = oracle.inverse_sht(flm, L, reality=real)
    fm = s2.mw_inverse(_to_dev(flm, dev), L, reality, precision=PREC[mode])
    assert _errs(fm.cpu().numpy(), ref)[0] < TOL[mode]
    back = s2.mw_forward(_to_dev(ref, dev), L, reality, precision=PREC[mode]).cpu().numpy()
    assert _errs(back, flm)[0] < TOL[mode]
    # the FP64 path is unaffected by the mode of earlier calls
    f64 = s2.mw_inverse(_to_dev(flm, dev), L, reality).cpu().numpy()
    assert oracle.rel_max_err(f64, ref) < 1e-10


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_mixed_wavelets_per_scale(dev, mode):
    """16 real maps, L=128, B=2, J_min=2, multiresolution: mixed-precision analysis and synthesis,
    max and RMS error against the FP64 oracle for every scale."""
    L, B, J_min, nm = 128, 2, 2, 16
    flm = si.random_flm(L, 2, reality=True, seed=7)
    f2 = oracle.inverse_sht(flm, L, reality=True)
    f = np.concatenate([f2] * (nm // 2))
    wav_ref, scal_ref = oracle.analysis(f2, L, B, J_min, True, True)
    fd = _to_dev(f, dev)
    f_wav, f_scal = s2.analysis(fd, L, B, J_min, True, s2.REAL, precision=PREC[mode])
    got = [w.cpu().numpy() for w in s2.split_wav(f_wav, L, B, J_min, True)]
    kP = oracle.bandlimit_scal(J_min, L, B, True)
    floor = 1e-6 * float(np.max(np.abs(f)))
    _log("%s scaling map k=%d" % (mode, kP))
    assert _errs(f_scal.cpu().numpy()[:2].reshape(2, kP, 2 * kP - 1), scal_ref, floor)[0] < TOL[mode]
    for j, (g, r) in enumerate(zip(got, wav_ref)):
        _log("scale j=%d" % (J_min + j))
        assert _errs(g[:2], r, floor)[0] < TOL[mode]
    rec = s2.synthesis(f_wav, f_scal, L, B, J_min, True, s2.REAL, precision=PREC[mode])
    _log("reconstruction")
    assert _errs(rec.cpu().numpy()[:2], f2)[0] < TOL[mode]


@pytest.mark.parametrize("mode,nm,reality", [("fp32", 16, s2.REAL), ("bf16x3", 16, s2.REAL),
                                             ("bf16x3", 8, s2.COMPLEX), ("bf16x3", 8, s2.REAL),
                                             ("bf16x3", 7, s2.REAL)])
def test_mixed_wavelets_per_scale_L2048(dev, mode, nm, reality):
    """The full-size workload (16 real maps, L = 2048, B = 2, J_min = 3, multiresolution, spectrum
    C_l = 1/(l(l+1)), seed 3), and in BF16x3 also 8 complex maps (32 columns) and 8 real maps
    (16 columns), which take the other instantiations of the FP32 stage kernels, and 7 real maps
    (14 of 16 columns used: the last phi unit holds one map): every scale of the
    mixed analysis against the FP64 run (itself checked against the oracle in
    test_gpu_fullsize.py), relative to that scale's own max |FP64|, and the reconstruction.  The
    spectrum puts the finest scales near 1e-3 of the map, so rounding relative to the whole map in a
    forward stage would show there amplified (it did, at 1.5e-4 of the finest scale, with FP32
    forward phi and theta stages in the analysis)."""
    L, B, J_min = 2048, 2, 3
    real = reality == s2.REAL
    flm = torch.from_numpy(si.random_flm(L, nm, reality=real, seed=3)).to(dev)
    f = s2.mw_inverse(flm, L, reality)
    del flm
    w64, s64 = s2.analysis(f, L, B, J_min, True, reality)
    w, sc = s2.analysis(f, L, B, J_min, True, reality, precision=PREC[mode])
    torch.cuda.synchronize()

    def rel(a, b):
        return ((a - b).abs().max() / b.abs().max()).item()

    e = rel(sc, s64)
    _log("  %s scaling: %.2e" % (mode, e))
    assert e < TOL[mode]
    for j, (g, r) in enumerate(zip(s2.split_wav(w, L, B, J_min, True), s2.split_wav(w64, L, B, J_min, True))):
        e = rel(g, r)
        _log("  %s scale j=%d: %.2e" % (mode, J_min + j, e))
        assert e < TOL[mode]
    del w64, s64
    rec = s2.synthesis(w, sc, L, B, J_min, True, reality, precision=PREC[mode])
    e = rel(rec, f)
    _log("  %s reconstruction: %.2e" % (mode, e))
    assert e < TOL[mode]


def test_config_512_complex_side_by_side(dev):
    """One complex map, L=512, B=2, J_min=2, multiresolution, FP64, FP32 and BF16x3 side by side."""
    L, B, J_min = 512, 2, 2
    flm = si.random_flm(L, 1, reality=False, seed=1)
    f = oracle.inverse_sht(flm, L)
    fd = _to_dev(f, dev)
    out = {}
    for name, prec in (("fp64", s2.FP64), ("fp32", s2.MIXED_FP32), ("bf16x3", s2.MIXED_BF16X3)):
        _log(name)
        got_flm = s2.mw_forward(fd, L, s2.COMPLEX, precision=prec).cpu().numpy()
        out[name] = _errs(got_flm, flm)[0]
        f_wav, f_scal = s2.analysis(fd, L, B, J_min, True, s2.COMPLEX, precision=prec)
        rec = s2.synthesis(f_wav, f_scal, L, B, J_min, True, s2.COMPLEX, precision=prec)
        out[name + "_rec"] = _errs(rec.cpu().numpy(), f)[0]
    assert out["fp64"] < 1e-10 and out["fp64_rec"] < 1e-10
    assert out["fp32"] < TOL_FP32 and out["fp32_rec"] < TOL_FP32
    assert out["bf16x3"] < TOL["bf16x3"] and out["bf16x3_rec"] < TOL["bf16x3"]
