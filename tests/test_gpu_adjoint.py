"""Adjoint transforms and gradients on the GPU (through the C ABI and the autograd wrappers).

  - parity: mw_inverse_adjoint / mw_forward_adjoint and the wavelet adjoints against the
    oracle's adjoints (pinned in test_oracle_adjoint.py), relative max error <= 1e-10;
  - the dot-product identity <M x, y> = <x, M^H y> at sizes the oracle does not reach;
  - the gradient of the regularised deconvolution loss of the differentiation workload
    (8 real maps, L = 1024, B = 2, J_min = 2, multiresolution):
        loss(f) = || b_l f_lm - d_lm ||^2 + lam sum_j || W^j(f) ||^2,
    b_l = exp(-l(l+1) sigma^2 / 2), sigma = 0.005, d = b s + n with s drawn from
    C_l = 1/(l(l+1)) and n white (variance 1e-4 per coefficient), lam = 0.1, seed 4,
    checked against the explicit adjoint formula and against central finite differences (the
    loss is quadratic, so the central difference is exact up to rounding), and against the
    oracle's gradient at L = 32 and at the workload's own size, in FP64 and with the FP32
    contraction (stated bound 1e-5)."""
import sys

import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")
ad = pytest.importorskip("paper_1211_1680_amd.autograd")

TOL = 1e-10


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    r = float(np.max(np.abs(got - ref))) / den if den > 0 else float(np.max(np.abs(got - ref)))
    _log("  rel err %.3e" % r)
    return r


def _to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _ipt(a, b):
    return float(torch.real(torch.vdot(a.reshape(-1), b.reshape(-1))).item())


RNG = np.random.default_rng(4)


@pytest.mark.parametrize("nmaps,reality", [(3, s2.REAL), (2, s2.COMPLEX), (17, s2.REAL)])
@pytest.mark.parametrize("L", [1, 2, 3, 8, 16, 33, 64])
def test_sht_adjoint_parity(dev, L, nmaps, reality):
    _log("sht adjoints L=%d nmaps=%d reality=%d" % (L, nmaps, reality))
    real = reality == s2.REAL
    n = 2 * L - 1
    f = RNG.standard_normal((nmaps, L, n))
    if not real:
        f = f + 1j * RNG.standard_normal((nmaps, L, n))
    y = RNG.standard_normal((nmaps, L * L)) + 1j * RNG.standard_normal((nmaps, L * L))
    got = s2.mw_inverse_adjoint(_to_dev(f, dev), L, reality).cpu().numpy()
    assert _rel(got, oracle.inverse_sht_adjoint(f, L, real)) < TOL
    # y is not Hermitian: for real maps the adjoint uses its Hermitian part
    got = s2.mw_forward_adjoint(_to_dev(y, dev), L, reality).cpu().numpy()
    assert _rel(got, oracle.forward_sht_adjoint(y, L, real)) < TOL


@pytest.mark.parametrize("L,B,J_min,multires,reality", [(16, 2, 1, True, s2.REAL), (32, 3, 1, True, s2.COMPLEX),
                                                         (64, 2, 0, False, s2.REAL), (50, 3, 2, True, s2.REAL)])
def test_wavelet_adjoint_parity(dev, L, B, J_min, multires, reality):
    _log("wavelet adjoints", L, B, J_min, multires, reality)
    real = reality == s2.REAL
    nm = 2

    def rmap(k):
        x = RNG.standard_normal((nm, k, 2 * k - 1))
        return x if real else x + 1j * RNG.standard_normal((nm, k, 2 * k - 1))

    ks = [oracle.bandlimit_wav(j, L, B, multires) for j in range(J_min, oracle.j_max(L, B) + 1)]
    kP = oracle.bandlimit_scal(J_min, L, B, multires)
    wav = [rmap(k) for k in ks]
    scal = rmap(kP)
    f_wav = np.concatenate([w.reshape(nm, -1) for w in wav], axis=1)
    got = s2.analysis_adjoint(_to_dev(f_wav, dev), _to_dev(scal.reshape(nm, -1), dev), L, B, J_min, multires,
                              reality).cpu().numpy()
    assert _rel(got, oracle.analysis_adjoint(wav, scal, L, B, J_min, multires, real)) < TOL
    f = rmap(L)
    gw, gs = s2.synthesis_adjoint(_to_dev(f, dev), L, B, J_min, multires, reality)
    rw, rs = oracle.synthesis_adjoint(f, L, B, J_min, multires, real)
    assert _rel(gs.cpu().numpy().reshape(rs.shape), rs) < TOL
    for g, r in zip(s2.split_wav(gw, L, B, J_min, multires), rw):
        assert _rel(g.cpu().numpy(), r) < TOL


@pytest.mark.parametrize("reality", [s2.REAL, s2.COMPLEX])
@pytest.mark.parametrize("L", [256, 2048])
def test_dot_product_identities(dev, reality, L):
    """<A x, y> = <x, A^H y> for the forward and inverse transforms.  At L = 256 with 4 maps the
    transforms run on the MW nodes; at L = 2048 with 8 real (4 complex) maps, 16 columns, the
    forward and inverse transforms take the symmetric grid with the column-quad stage layout and
    their adjoints the row layout, so each identity ties the two."""
    nm = 4 if L == 256 or reality == s2.COMPLEX else 8
    _log("  dot products L=%d nmaps=%d reality=%d" % (L, nm, reality))
    real = reality == s2.REAL
    n = 2 * L - 1
    g = torch.Generator(device="cpu").manual_seed(7)
    dt = torch.float64 if real else torch.complex128
    x = torch.randn((nm, L, n), generator=g, dtype=dt).to(dev)
    y = torch.randn((nm, L * L), generator=g, dtype=torch.complex128).to(dev)
    lhs, rhs = _ipt(s2.mw_forward(x, L, reality), y), _ipt(x, s2.mw_forward_adjoint(y, L, reality))
    _log("  forward: %.6e %.6e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    if real:   # the real inverse reads only m >= 0: compare on Hermitian coefficients
        y = s2.mw_forward(torch.randn((nm, L, n), generator=g, dtype=dt).to(dev), L, reality)
    lhs, rhs = _ipt(s2.mw_inverse(y, L, reality), x), _ipt(y, s2.mw_inverse_adjoint(x, L, reality))
    _log("  inverse: %.6e %.6e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ the differentiation workload
def _workload(L, nm, seed=4, sigma=0.005):
    ell = np.arange(L)
    b = np.exp(-ell * (ell + 1) * sigma * sigma / 2.0)
    s = si.random_flm(L, nm, reality=True, seed=seed)
    noise = si.random_flm(L, nm, reality=True, seed=seed + 100, cl=np.full(L, 1e-4))
    bl = np.repeat(b, 2 * ell + 1)
    d = bl[None, :] * s + noise
    f0 = oracle.inverse_sht(si.random_flm(L, nm, reality=True, seed=seed + 200), L, reality=True)
    return bl, d, f0


def _loss_gpu(f, bl_t, d_t, L, B, J_min, lam, precision=s2.FP64):
    flm = ad.mw_forward_ad(f, L, s2.REAL, precision)
    r = bl_t[None, :] * flm - d_t
    f_wav, _ = ad.analysis_ad(f, L, B, J_min, True, s2.REAL, precision)
    return torch.sum(torch.abs(r) ** 2) + lam * torch.sum(f_wav * f_wav)


def _grad_gpu(f0, bl, d, L, B, J_min, lam, precision, dev):
    f = _to_dev(f0, dev).requires_grad_(True)
    loss = _loss_gpu(f, _to_dev(bl, dev), _to_dev(d, dev), L, B, J_min, lam, precision)
    loss.backward()
    return f.grad.detach()


def _grad_oracle(f0, bl, d, L, B, J_min, lam):
    """The loss gradient from the oracle's transforms and adjoints:
    2 A^H (b (b f_lm - d)) + 2 lam W^H (W^j(f), 0), A the forward transform, W the analysis."""
    r = bl[None, :] * oracle.forward_sht(f0, L) - d
    wav, scal = oracle.analysis(f0, L, B, J_min, True, True)
    return 2.0 * oracle.forward_sht_adjoint(bl[None, :] * r, L, True) + \
        2.0 * lam * oracle.analysis_adjoint(wav, np.zeros_like(scal), L, B, J_min, True, True)


@pytest.mark.parametrize("L,nm", [(64, 2), (1024, 8)])
def test_loss_gradient(dev, L, nm):
    B, J_min, lam = 2, 2, 0.1
    _log("loss gradient L=%d nmaps=%d" % (L, nm))
    bl, d, f0 = _workload(L, nm)
    bl_t, d_t = _to_dev(bl, dev), _to_dev(d, dev)
    f = _to_dev(f0, dev).requires_grad_(True)
    loss = _loss_gpu(f, bl_t, d_t, L, B, J_min, lam)
    loss.backward()
    grad = f.grad.detach()
    # explicit formula with the adjoint calls
    with torch.no_grad():
        fd = f.detach()
        r = bl_t[None, :] * s2.mw_forward(fd, L) - d_t
        f_wav, f_scal = s2.analysis(fd, L, B, J_min, True)
        g2 = 2.0 * s2.mw_forward_adjoint((bl_t[None, :] * r).contiguous(), L) + \
            2.0 * lam * s2.analysis_adjoint(f_wav, torch.zeros_like(f_scal), L, B, J_min, True)
    assert _rel(grad.cpu().numpy(), g2.cpu().numpy()) < 1e-12
    # central differences along random directions (exact for a quadratic up to rounding)
    gen = torch.Generator(device="cpu").manual_seed(11)
    for _ in range(3):
        v = torch.randn(fd.shape, generator=gen, dtype=torch.float64).to(dev)
        h = 1e-2 * float(fd.norm() / v.norm())
        with torch.no_grad():
            lp = _loss_gpu(fd + h * v, bl_t, d_t, L, B, J_min, lam).item()
            lm = _loss_gpu(fd - h * v, bl_t, d_t, L, B, J_min, lam).item()
        fdv = (lp - lm) / (2 * h)
        gv = float(torch.sum(grad * v).item())
        _log("  directional: finite difference %.12e  gradient %.12e" % (fdv, gv))
        assert abs(fdv - gv) <= 1e-8 * max(abs(gv), 1e-30) + 1e-12 * abs(lp) / h


# Stated bound of the FP32-contraction gradient against the FP64 oracle's (relative max error):
# each transform in the chain carries the FP32 contraction's <= 2e-6 (test_gpu_mixed.py).
TOL_GRAD_FP32 = 1e-5


@pytest.mark.parametrize("precision", [s2.FP64, s2.MIXED_FP32])
def test_loss_gradient_against_oracle(dev, precision):
    L, nm, B, J_min, lam = 32, 2, 2, 2, 0.1
    bl, d, f0 = _workload(L, nm)
    got = _grad_gpu(f0, bl, d, L, B, J_min, lam, precision, dev)
    ref = _grad_oracle(f0, bl, d, L, B, J_min, lam)
    assert _rel(got.cpu().numpy(), ref) < (TOL if precision == s2.FP64 else TOL_GRAD_FP32)


@pytest.fixture(scope="module")
def grad_ref_1024():
    L, nm, B, J_min, lam = 1024, 8, 2, 2, 0.1
    bl, d, f0 = _workload(L, nm)
    _log("oracle gradient of maps 0, 1 at L=%d" % L)
    return _grad_oracle(f0[:2], bl, d[:2], L, B, J_min, lam)


@pytest.mark.parametrize("precision", [s2.FP64, s2.MIXED_FP32])
def test_loss_gradient_full_size_against_oracle(dev, grad_ref_1024, precision):
    """The differentiation workload at its size (8 real maps, L = 1024, B = 2, J_min = 2,
    multiresolution) in FP64 and FP32: the gradient of every map from the GPU's adjoints against
    the oracle's gradient of the first two maps (the loss is a sum over maps, so each map's
    gradient depends on that map alone), and in FP32 also against the FP64 GPU gradient."""
    L, nm, B, J_min, lam = 1024, 8, 2, 2, 0.1
    bl, d, f0 = _workload(L, nm)
    _log("loss gradient L=%d nmaps=%d precision=%d: GPU" % (L, nm, precision))
    got = _grad_gpu(f0, bl, d, L, B, J_min, lam, precision, dev).cpu().numpy()
    ref = grad_ref_1024
    tol = TOL if precision == s2.FP64 else TOL_GRAD_FP32
    assert _rel(got[:2], ref) < tol
    if precision != s2.FP64:
        g64 = _grad_gpu(f0, bl, d, L, B, J_min, lam, s2.FP64, dev).cpu().numpy()
        assert _rel(got, g64) < tol
