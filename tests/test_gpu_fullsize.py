"""Parity at the full benchmark size, in the launch configuration bench.py times: wavelet
analysis + synthesis of 16 real maps at L = 2048, B = 2, J_min = 3, multiresolution, FP64.

The oracle synthesises two of the maps (seeded, C_l = 1/(l(l+1))); the batch is eight copies of
the pair.  Checked against the oracle: every wavelet scale (k = 16 ... 2048), the scaling map and
the reconstruction on every ring, in FP64 and, with their per-scale max and RMS errors, in the
FP32 and BF16x3 contraction modes; the forward transform against the seeded coefficients; the
transforms and adjoints of small batches (MW-node Legendre steps) and the forward adjoint of the
full batch; the round-trip error of unit coefficients; and that copies in the batch agree."""
import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")

TOL = 1e-10
L, B, J_MIN, NMAPS = 2048, 2, 3, 16


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel(got, ref, floor):
    den = max(float(np.max(np.abs(ref))), floor)
    r = float(np.max(np.abs(np.asarray(got) - np.asarray(ref)))) / den
    print("  rel err %.3e" % r, flush=True)
    return r


@pytest.fixture(scope="module")
def data(dev):
    print("full size: oracle synthesis of 2 maps at L=%d" % L, flush=True)
    flm = si.random_flm(L, 2, reality=True, seed=3)
    f2 = oracle.inverse_sht(flm, L, reality=True)
    f = np.concatenate([f2] * (NMAPS // 2))
    fd = torch.from_numpy(f).to(dev)
    print("full size: GPU analysis + synthesis, 16 maps", flush=True)
    f_wav, f_scal = s2.analysis(fd, L, B, J_MIN, True, s2.REAL)
    rec = s2.synthesis(f_wav, f_scal, L, B, J_MIN, True, s2.REAL)
    flm_gpu = s2.mw_forward(fd, L, s2.REAL)
    torch.cuda.synchronize()
    return dict(flm=flm, f=f, fd=fd, f_wav=f_wav.cpu().numpy(), f_scal=f_scal.cpu().numpy(),
                rec=rec.cpu().numpy(), flm_gpu=flm_gpu.cpu().numpy())


def test_forward_full_size(data):
    got = data["flm_gpu"]
    for i in range(NMAPS):
        assert _rel(got[i], data["flm"][i % 2], 0.0) < TOL


def test_batch_copies_agree(data):
    w, p, r = data["f_wav"], data["f_scal"], data["rec"]
    for i in range(2, NMAPS):
        assert np.array_equal(w[i], w[i % 2])
        assert np.array_equal(p[i], p[i % 2])
        assert np.array_equal(r[i], r[i % 2])


def test_reconstruction_full_size(data):
    floor = 1e-6 * float(np.max(np.abs(data["f"])))
    assert _rel(data["rec"], data["f"], floor) < TOL


@pytest.fixture(scope="module")
def oracle_scales(data):
    """The oracle's wavelet maps of the two distinct maps, every scale on every ring (Eqs. (4),
    (6), then Eq. (1) at each scale's band-limit), and its scaling map.  The harmonic input is the
    seeded f_lm, which the oracle's forward transform of the band-limited map returns."""
    flm = data["flm"]
    wav_lm, scal_lm = oracle.analysis_harmonic(flm, L, B, J_MIN, True)
    wav = []
    for j, w in zip(range(J_MIN, oracle.j_max(L, B) + 1), wav_lm):
        k = oracle.bandlimit_wav(j, L, B, True)
        print("oracle scale j=%d k=%d (every ring)" % (j, k), flush=True)
        wav.append(oracle.inverse_sht(w, k, reality=True))
    kP = oracle.bandlimit_scal(J_MIN, L, B, True)
    return wav, oracle.inverse_sht(scal_lm, kP, reality=True)


def _split(f_wav, nm):
    out, off = [], 0
    for j in range(J_MIN, oracle.j_max(L, B) + 1):
        k = oracle.bandlimit_wav(j, L, B, True)
        out.append(f_wav[:, off:off + k * (2 * k - 1)].reshape(nm, k, 2 * k - 1))
        off += k * (2 * k - 1)
    return out


def _scale_errors(label, got_wav, got_scal, got_rec, ref_wav, ref_scal, f):
    """Per-scale max and RMS error of GPU outputs [16 maps] against the oracle's [2 maps],
    absolute and relative to that scale's max |oracle| (RMS relative to the oracle's RMS)."""
    rows = []
    ks = [oracle.bandlimit_wav(j, L, B, True) for j in range(J_MIN, oracle.j_max(L, B) + 1)]
    kP = oracle.bandlimit_scal(J_MIN, L, B, True)
    items = [("scal", kP, got_scal, ref_scal)] + \
        [("j=%d" % j, k, g, r) for j, k, g, r in zip(range(J_MIN, J_MIN + len(ks)), ks, got_wav, ref_wav)] + \
        [("rec", L, got_rec, f)]
    for name, k, g, r in items:
        d = g - np.concatenate([r] * (NMAPS // 2))
        mx, rms = float(np.max(np.abs(d))), float(np.sqrt(np.mean(d * d)))
        rmax, rrms = float(np.max(np.abs(r))), float(np.sqrt(np.mean(r * r)))
        rows.append((name, k, mx, mx / rmax, rms, rms / rrms))
        print("%-7s %-5s k=%4d  max %.3e (rel %.3e)  rms %.3e (rel %.3e)" % ((label, name, k) + rows[-1][2:]),
              flush=True)
    return rows


def test_scales_every_ring(data, oracle_scales):
    """FP64: every wavelet scale (k = 16 ... 2048), the scaling map and the reconstruction,
    on every ring, against the oracle."""
    ref_wav, ref_scal = oracle_scales
    kP = oracle.bandlimit_scal(J_MIN, L, B, True)
    got_wav = _split(data["f_wav"], NMAPS)
    rows = _scale_errors("fp64", got_wav, data["f_scal"].reshape(NMAPS, kP, 2 * kP - 1), data["rec"],
                         ref_wav, ref_scal, data["f"][:2])
    floor = 1e-6 * float(np.max(np.abs(data["f"])))
    for (name, k, mx, rel, rms, rrms), r in zip(rows, [ref_scal] + list(ref_wav) + [data["f"][:2]]):
        assert mx / max(float(np.max(np.abs(r))), floor) < TOL, name


# Stated bounds of the mixed-precision contraction (relative max error against the FP64
# oracle), the same as up to L = 512 (test_gpu_mixed.py).
MIXED_BOUNDS = {"fp32": 2e-6, "bf16x3": 1e-4}


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_mixed_per_scale_errors_full_size(data, oracle_scales, mode):
    """The precision workload (16 real maps, L = 2048, B = 2, J_min = 3, multiresolution): the
    Legendre contraction in FP32 or BF16x3 with the FP64 recursion.  Max and RMS error of every
    scale, the scaling map and the reconstruction against the FP64 oracle, every ring."""
    prec = {"fp32": s2.MIXED_FP32, "bf16x3": s2.MIXED_BF16X3}[mode]
    fd = data["fd"]
    f_wav, f_scal = s2.analysis(fd, L, B, J_MIN, True, s2.REAL, prec)
    rec = s2.synthesis(f_wav, f_scal, L, B, J_MIN, True, s2.REAL, prec)
    torch.cuda.synchronize()
    kP = oracle.bandlimit_scal(J_MIN, L, B, True)
    ref_wav, ref_scal = oracle_scales
    rows = _scale_errors(mode, _split(f_wav.cpu().numpy(), NMAPS),
                         f_scal.cpu().numpy().reshape(NMAPS, kP, 2 * kP - 1), rec.cpu().numpy(),
                         ref_wav, ref_scal, data["f"][:2])
    floor = 1e-6 * float(np.max(np.abs(data["f"])))
    for (name, k, mx, rel, rms, rrms), r in zip(rows, [ref_scal] + list(ref_wav) + [data["f"][:2]]):
        assert mx / max(float(np.max(np.abs(r))), floor) < MIXED_BOUNDS[mode], (mode, name)


def test_mw_node_path_full_size(data):
    """At L = 2048 a batch of 2 real maps (4 columns) runs the Legendre steps on the MW nodes:
    the inverse on every ring, and the adjoint of the inverse, against the oracle."""
    flm2 = torch.from_numpy(data["flm"]).to(data["fd"].device)
    got = s2.mw_inverse(flm2, L, s2.REAL).cpu().numpy()
    print("MW-node inverse, 2 real maps", flush=True)
    assert _rel(got, data["f"][:2], 0.0) < TOL
    rng = np.random.default_rng(77)
    x = rng.standard_normal((2, L, 2 * L - 1))
    print("MW-node inverse adjoint, 2 arbitrary real maps (oracle)", flush=True)
    ref = oracle.inverse_sht_adjoint(x, L, True)
    got = s2.mw_inverse_adjoint(torch.from_numpy(x).to(data["fd"].device), L, s2.REAL).cpu().numpy()
    assert _rel(got, ref, 0.0) < TOL


def test_forward_adjoint_full_size(data):
    """The adjoint of the forward transform at L = 2048, for 2 real maps (MW-node Legendre
    synthesis) and for 16 (symmetric-grid synthesis and resampling, then the quadrature's
    transpose), against the oracle's adjoint."""
    rng = np.random.default_rng(78)
    y = rng.standard_normal((2, L * L)) + 1j * rng.standard_normal((2, L * L))
    print("forward adjoint: oracle, 2 coefficient sets", flush=True)
    ref = oracle.forward_sht_adjoint(y, L, True)
    dev = data["fd"].device
    got2 = s2.mw_forward_adjoint(torch.from_numpy(y).to(dev), L, s2.REAL).cpu().numpy()
    assert _rel(got2, ref, 0.0) < TOL
    got16 = s2.mw_forward_adjoint(torch.from_numpy(np.concatenate([y] * (NMAPS // 2))).to(dev), L,
                                  s2.REAL).cpu().numpy()
    for i in range(NMAPS):
        assert _rel(got16[i], ref[i % 2], 0.0) < TOL


def test_round_trip_unit_coefficients_full_size(dev):
    """The paper's accuracy measure (Sect. 3.3): epsilon = max |f_lm - f_lm^rec| for complex
    f_lm ~ N(0, 1) through the inverse and forward transforms, at L = 2048 (8 complex maps,
    symmetric grid; 1 map, MW nodes).  Floating-point level, growing like O(L): <= 1e-12."""
    for nm in (8, 1):
        flm = torch.from_numpy(si.random_flm_unit(L, nm, seed=2048 + nm)).to(dev)
        back = s2.mw_forward(s2.mw_inverse(flm, L, s2.COMPLEX), L, s2.COMPLEX)
        eps = float((back - flm).abs().max().item())
        print("  round trip L=%d, %d complex maps: epsilon %.3e" % (L, nm, eps), flush=True)
        assert eps <= 1e-12


def test_forward_arbitrary_samples_full_size(dev):
    """Forward transform at L = 2048 of samples that are not band-limited (two real maps of
    independent unit normals, so the south-pole ring is not constant), against the oracle."""
    rng = np.random.default_rng(2048)
    f = rng.standard_normal((2, L, 2 * L - 1))
    print("full size: oracle forward of 2 arbitrary maps", flush=True)
    ref = oracle.forward_sht(f, L)
    got = s2.mw_forward(torch.from_numpy(f).to(dev), L, s2.REAL).cpu().numpy()
    assert _rel(got, ref, 0.0) < TOL


@pytest.mark.parametrize("k,reality,nmaps,ndistinct", [
    (2048, s2.REAL, 8, 2), (2048, s2.REAL, 16, 2), (2048, s2.COMPLEX, 4, 1),
    (1024, s2.REAL, 16, 2), (1024, s2.COMPLEX, 8, 1), (1024, s2.REAL, 2, 2), (1024, s2.COMPLEX, 1, 1),
    (512, s2.REAL, 16, 2), (512, s2.COMPLEX, 8, 1), (512, s2.REAL, 2, 2), (512, s2.COMPLEX, 1, 1),
    (256, s2.REAL, 16, 2), (256, s2.COMPLEX, 8, 1), (256, s2.REAL, 2, 2),
    (128, s2.REAL, 16, 2), (128, s2.COMPLEX, 8, 1), (64, s2.REAL, 16, 2), (64, s2.COMPLEX, 8, 1)])
def test_symmetric_grid_batches_full_size(dev, k, reality, nmaps, ndistinct):
    """At band-limits 2048 to 64 (compiled transforms) the FP64 transforms of batches of 16 or
    32 columns (8 or 16 real maps, 4 or 8 complex maps) run their Legendre steps on the symmetric
    grid; smaller batches (2 real maps, 1 complex map) take the compiled phi stages with the MW-node
    theta stage.  Samples that are not band-limited (independent unit normals, so the odd-m pole
    terms matter) go forward; seeded coefficients go inverse.  The batch repeats ndistinct maps,
    which the oracle evaluates."""
    real = reality == s2.REAL
    rng = np.random.default_rng(4096 + nmaps + k)
    base = rng.standard_normal((ndistinct, k, 2 * k - 1))
    if not real:
        base = base + 1j * rng.standard_normal((ndistinct, k, 2 * k - 1))
    print("k=%d: oracle forward of %d map(s), reality=%d, batch %d" % (k, ndistinct, reality, nmaps), flush=True)
    ref = oracle.forward_sht(base, k)
    f = np.concatenate([base] * (nmaps // ndistinct))
    got = s2.mw_forward(torch.from_numpy(f).to(dev), k, reality).cpu().numpy()
    for i in range(nmaps):
        assert _rel(got[i], ref[i % ndistinct], 0.0) < TOL
    flm = si.random_flm(k, ndistinct, reality=real, seed=77)
    rings = sorted({0, 1, k // 4 - 1, k // 2 - 1, k // 2, k - 2, k - 1})
    refm = oracle.inverse_sht_rings(flm, k, rings, reality=real)
    gotm = s2.mw_inverse(torch.from_numpy(np.concatenate([flm] * (nmaps // ndistinct))).to(dev), k,
                         reality).cpu().numpy()
    for i in range(nmaps):
        assert _rel(gotm[i][rings, :], refm[i % ndistinct], 0.0) < TOL


TOL_FP32_2048 = 2e-6   # the bound stated up to L = 512 (test_gpu_mixed.py) also holds at L = 2048


def test_fp32_symmetric_grid_full_size(data):
    """FP32 contraction on the symmetric grid (16 real maps, L = 2048): forward against the seeded
    coefficients, inverse on oracle rings."""
    dev = data["fd"].device
    got = s2.mw_forward(data["fd"], L, s2.REAL, s2.MIXED_FP32).cpu().numpy()
    worst = max(_rel(got[i], data["flm"][i % 2], 0.0) for i in range(NMAPS))
    print("  fp32 forward worst rel err %.3e" % worst, flush=True)
    assert worst < TOL_FP32_2048
    rings = [0, 1, 1023, 1024, 2047]
    ref = oracle.inverse_sht_rings(data["flm"], L, rings, reality=True)
    flm = torch.from_numpy(np.concatenate([data["flm"]] * (NMAPS // 2))).to(dev)
    inv = s2.mw_inverse(flm, L, s2.REAL, s2.MIXED_FP32).cpu().numpy()
    worst = max(_rel(inv[i][rings, :], ref[i % 2], 0.0) for i in range(NMAPS))
    print("  fp32 inverse worst rel err %.3e" % worst, flush=True)
    assert worst < TOL_FP32_2048


def test_bf16x3_symmetric_grid_full_size(data):
    """BF16x3 contraction on the symmetric grid (16 real maps, L = 2048), against the bound stated
    for that mode (1e-4, test_gpu_mixed.py)."""
    dev = data["fd"].device
    got = s2.mw_forward(data["fd"], L, s2.REAL, s2.MIXED_BF16X3).cpu().numpy()
    worst = max(_rel(got[i], data["flm"][i % 2], 0.0) for i in range(NMAPS))
    print("  bf16x3 forward worst rel err %.3e" % worst, flush=True)
    assert worst < 1e-4
    rings = [0, 1, 1023, 1024, 2047]
    ref = oracle.inverse_sht_rings(data["flm"], L, rings, reality=True)
    flm = torch.from_numpy(np.concatenate([data["flm"]] * (NMAPS // 2))).to(dev)
    inv = s2.mw_inverse(flm, L, s2.REAL, s2.MIXED_BF16X3).cpu().numpy()
    worst = max(_rel(inv[i][rings, :], ref[i % 2], 0.0) for i in range(NMAPS))
    print("  bf16x3 inverse worst rel err %.3e" % worst, flush=True)
    assert worst < 1e-4
