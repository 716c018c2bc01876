"""ORACLE -- test infrastructure only.

A plain, slow, obviously-correct CPU FP64 reference for the axisymmetric scale-discretised
wavelet transform on the sphere (Leistedt, McEwen, Vandergheynst & Wiaux, S2LET), written
from the paper.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library: the C part in
``orc_legendre.c`` is built with gcc into ``oracle/_orc.so``.

Functions and the passages they follow:
  mw_nodes ................ Sect. 2.1 (MW sampling: (L-1)(2L-1)+1 equiangular samples)
  inverse_sht ............. Eq. (1), truncated at the band-limit (Sect. 2.1)
  inverse_sht_rings ....... Eq. (1) on a chosen set of rings (checks of large outputs)
  inverse_sht_direct ...... Eq. (1) by direct Y_lm summation (small L only)
  forward_sht ............. Eq. (2), evaluated exactly by the MW quadrature (Sect. 2.1)
  quadrature_weight ....... the sin(theta) integral weights used by that quadrature
  tiling .................. Eqs. (10)-(16) and J = ceil(log_lambda(L-1)) (Sect. 2.2)
  analysis / synthesis .... Eqs. (4), (6), (8); multiresolution band-limits (Sect. 3.1)
  *_adjoint ............... adjoints of the four transforms above (their steps transposed)
  bspline_b3, k_bspline ... the B-spline generating function, Eqs. (17)-(18) (exact rationals)
  noise_std ............... wavelet-space noise level of Sect. 4.3 (Eq. (19) and Eq. (15))
  hard_threshold .......... Eq. (23); snr: Eqs. (20)-(21); denoise: Sect. 4.3

Parity status: every function above is pinned by tests/test_oracle_pins.py (the adjoints by
tests/test_oracle_adjoint.py, the B-spline and denoising functions by
tests/test_oracle_denoise.py); inverse_sht_rings against the full synthesis and direct Y_lm
summation, kappa_lambda against the two 30-digit terms of Eq. (13).  Not pinned: the
absolute values of k_lambda (Eq. (12)), which the paper does not print: they are checked
against an independent high-precision quadrature only ("parity unpinned" for the absolute
kernel values).
"""
from __future__ import annotations

import ctypes
import math
from fractions import Fraction
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_orc.so")
_SRC = os.path.join(_HERE, "orc_legendre.c")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C part with gcc (OpenMP); returns the path of the shared object."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_SO)
            dp = ctypes.POINTER(ctypes.c_double)
            lib.orc_lambda.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp]
            lib.orc_lambda_log2.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
            lib.orc_legendre_inverse.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
            lib.orc_legendre_forward.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
            lib.orc_legendre_inverse_rings.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                                       ctypes.POINTER(ctypes.c_int), dp]
            _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------------------
# Sampling (Sect. 2.1)
# ----------------------------------------------------------------------------------------
def mw_nodes(k: int):
    """MW nodes: theta_t = pi(2t+1)/(2k-1), t<k (south pole sampled, north pole not);
    phi_p = 2 pi p/(2k-1), p < 2k-1.  (L-1)(2L-1)+1 distinct points (Sect. 2.1)."""
    n = 2 * k - 1
    theta = np.pi * (2.0 * np.arange(k) + 1.0) / n
    phi = 2.0 * np.pi * np.arange(n) / n
    return theta, phi


def mw_size(k: int) -> int:
    return k * (2 * k - 1)


# ----------------------------------------------------------------------------------------
# Associated Legendre values lambda_lm (Condon-Shortley, orthonormal)
# ----------------------------------------------------------------------------------------
def legendre_lambda(k: int, m: int, theta) -> np.ndarray:
    """lambda_lm(theta_j) for l = m..k-1: array [len(theta), k-m]."""
    theta = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
    out = np.zeros((theta.size, k - m))
    _load().orc_lambda(k, m, _dp(theta), theta.size, _dp(out))
    return out


def legendre_log2(k: int, m: int, theta: float) -> np.ndarray:
    """log2 |lambda_lm(theta)| for l = m..k-1 (representable even in deep underflow)."""
    out = np.zeros(k - m)
    _load().orc_lambda_log2(k, m, float(theta), _dp(out))
    return out


# ----------------------------------------------------------------------------------------
# Inverse transform, Eq. (1)
# ----------------------------------------------------------------------------------------
def _as_maps(flm: np.ndarray, k: int) -> np.ndarray:
    flm = np.asarray(flm, dtype=np.complex128)
    if flm.ndim == 1:
        flm = flm[None, :]
    if flm.shape[1] != k * k:
        raise ValueError("flm must have k*k coefficients per map")
    return np.ascontiguousarray(flm)


def inverse_sht(flm: np.ndarray, k: int, reality: bool = False) -> np.ndarray:
    """f(theta_t, phi_p) = sum_{l<k} sum_{|m|<=l} f_lm Y_lm(theta_t, phi_p)  (Eq. (1)).

    Evaluated in the separable order sum_m e^{i m phi_p} sum_l f_lm lambda_lm(theta_t):
    the Legendre sums are plain sums (C, long double); the sum over m is a library
    inverse FFT of length 2k-1.  Returns [nmaps, k, 2k-1] (real if ``reality``)."""
    flm = _as_maps(flm, k)
    nmaps = flm.shape[0]
    n = 2 * k - 1
    F = np.zeros((nmaps, k, n), dtype=np.complex128)
    _load().orc_legendre_inverse(k, nmaps, _dp(flm.view(np.float64)), _dp(F.view(np.float64)))
    # F[..., m + k - 1] = F_m(theta_t); sum_m F_m e^{i m phi_p} with phi_p = 2 pi p / n.
    spec = np.zeros_like(F)
    ms = np.arange(-(k - 1), k)
    spec[..., ms % n] = F
    f = np.fft.ifft(spec, axis=-1) * n
    if reality:
        return f.real.copy()
    return f


def inverse_sht_rings(flm: np.ndarray, k: int, rings, reality: bool = False) -> np.ndarray:
    """Eq. (1) evaluated on selected rings only: [nmaps, len(rings), 2k-1].  Same sums as
    inverse_sht (for checking outputs too large to synthesise whole on the CPU)."""
    flm = _as_maps(flm, k)
    nmaps = flm.shape[0]
    n = 2 * k - 1
    rings = np.ascontiguousarray(np.asarray(rings, dtype=np.int32))
    if rings.size and (rings.min() < 0 or rings.max() >= k):
        raise ValueError("ring index out of range")
    F = np.zeros((nmaps, rings.size, n), dtype=np.complex128)
    _load().orc_legendre_inverse_rings(k, nmaps, _dp(flm.view(np.float64)), rings.size,
                                       rings.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                       _dp(F.view(np.float64)))
    spec = np.zeros_like(F)
    ms = np.arange(-(k - 1), k)
    spec[..., ms % n] = F
    f = np.fft.ifft(spec, axis=-1) * n
    return f.real.copy() if reality else f


def inverse_sht_direct(flm: np.ndarray, k: int) -> np.ndarray:
    """Eq. (1) by direct summation of Y_lm from scipy (O(k^4); for small k only)."""
    from scipy.special import sph_harm_y
    flm = _as_maps(flm, k)
    theta, phi = mw_nodes(k)
    TT, PP = np.meshgrid(theta, phi, indexing="ij")
    out = np.zeros((flm.shape[0], k, 2 * k - 1), dtype=np.complex128)
    for ell in range(k):
        for m in range(-ell, ell + 1):
            y = sph_harm_y(ell, m, TT, PP)
            out += flm[:, ell * ell + ell + m][:, None, None] * y[None]
    return out


# ----------------------------------------------------------------------------------------
# Forward transform, Eq. (2), by the MW quadrature
# ----------------------------------------------------------------------------------------
def quadrature_weight(p: np.ndarray) -> np.ndarray:
    """w(p) = int_0^pi e^{i p theta} sin(theta) d theta:
    2/(1-p^2) for even p, +i pi/2 for p = 1, -i pi/2 for p = -1, 0 for other odd p."""
    p = np.asarray(p)
    w = np.zeros(p.shape, dtype=np.complex128)
    even = (p % 2) == 0
    w[even] = 2.0 / (1.0 - p[even].astype(np.float64) ** 2)
    w[p == 1] = 0.5j * np.pi
    w[p == -1] = -0.5j * np.pi
    return w


def forward_sht(f: np.ndarray, k: int) -> np.ndarray:
    """f_lm = int f Y*_lm dOmega  (Eq. (2)), exact for band-limit k on the MW grid.

    Steps (the integral of the band-limited product, evaluated from the samples):
      1. G_m(theta_t) = (2 pi / n) sum_p f(theta_t, phi_p) e^{-i m phi_p}      (phi integral)
      2. extend theta to [0, 2 pi): g_t = G_m(theta_t) for t < k and
         g_t = (-1)^m G_m(theta_{2k-2-t}) for k <= t <= 2k-2
      3. Fourier coefficients  Ghat_j = (1/n) sum_t g_t e^{-i j theta_t},  |j| <= k-1
      4. I_j' = sum_j Ghat_j w(j + j')                                         (sin(theta) weight)
      5. H(theta_t) = (1/n) sum_j' I_j' e^{-i j' theta_t},  t = 0..n-1
      6. fold: H'(theta_t) = H(theta_t) + (-1)^m H(theta_{2k-2-t}) for t < k-1,
         H'(theta_{k-1}) = H(theta_{k-1})
      7. f_lm = sum_{t<k} lambda_lm(theta_t) H'_m(theta_t)
    with n = 2k-1 and theta_t = pi(2t+1)/n on the extended grid.
    Returns [nmaps, k*k] complex."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    nmaps = f.shape[0]
    n = 2 * k - 1
    if f.shape[1:] != (k, n):
        raise ValueError("map must be [k, 2k-1]")
    ms = np.arange(-(k - 1), k)                       # column index c <-> m = c - (k-1)
    eps = np.where(ms % 2 == 0, 1.0, -1.0)
    # 1. phi integral (library FFT over the ring)
    G = (2.0 * np.pi / n) * np.fft.fft(f.astype(np.complex128), axis=-1)[..., ms % n]  # [map, t, m]
    # 2. extension to t = 0..n-1
    g = np.zeros((nmaps, n, n), dtype=np.complex128)
    g[:, :k, :] = G
    if k > 1:
        g[:, k:, :] = eps[None, None, :] * G[:, k - 2::-1, :]
    # 3. Fourier coefficients in theta (half-sample phase from theta_0 = pi/n)
    js = np.arange(-(k - 1), k)
    D = np.fft.fft(g, axis=1)[:, js % n, :]            # sum_t g_t e^{-2 pi i j t/n}
    Ghat = (np.exp(-1j * np.pi * js / n)[None, :, None] * D) / n
    # 4. weight correlation: real even part of w by library matmul, plus the p = +-1 terms
    P = js[:, None] + js[None, :]                      # P[j', j] = j + j'
    Wfull = quadrature_weight(P)
    We = np.ascontiguousarray(Wfull.real)              # w(p) for even p (real)
    Iw = np.empty_like(Ghat)
    for x in range(nmaps):
        Iw[x] = (We @ np.ascontiguousarray(Ghat[x].real)
                 + 1j * (We @ np.ascontiguousarray(Ghat[x].imag)))
    # odd part: w(+1) = i pi/2 at j = 1 - j', w(-1) = -i pi/2 at j = -1 - j'
    for jp_idx, jp in enumerate(js):
        for p in (1, -1):
            j = p - jp
            if -(k - 1) <= j <= k - 1:
                Iw[:, jp_idx, :] += Wfull[jp_idx, j + k - 1] * Ghat[:, j + k - 1, :]
    # 5. back to theta on the extended grid
    spec = np.zeros((nmaps, n, n), dtype=np.complex128)
    spec[:, js % n, :] = np.exp(-1j * np.pi * js / n)[None, :, None] * Iw
    H = np.fft.fft(spec, axis=1) / n                  # sum_j' (.) e^{-2 pi i j' t/n}
    # 6. fold onto t < k
    Hp = np.zeros((nmaps, k, n), dtype=np.complex128)
    Hp[:, k - 1, :] = H[:, k - 1, :]
    if k > 1:
        t = np.arange(k - 1)
        Hp[:, :k - 1, :] = H[:, t, :] + eps[None, None, :] * H[:, n - 1 - t, :]
    # 7. Legendre contraction (C, long double)
    Hp = np.ascontiguousarray(Hp)
    flm = np.zeros((nmaps, k * k), dtype=np.complex128)
    _load().orc_legendre_forward(k, nmaps, _dp(Hp.view(np.float64)), _dp(flm.view(np.float64)))
    return flm


# ----------------------------------------------------------------------------------------
# Adjoints of the two transforms (for gradients through them).  Inner products: the plain sum
# over every stored sample for maps (Re sum conj(a) b for complex maps), Re sum conj(a) b over
# the full [k*k] array for coefficients.
# ----------------------------------------------------------------------------------------
def inverse_sht_adjoint(f: np.ndarray, k: int, reality: bool = False) -> np.ndarray:
    """S^H f with S the inverse transform of Eq. (1) on the MW grid:
    g_lm = sum_{t,p} conj(Y_lm(theta_t, phi_p)) f(theta_t, phi_p)
         = sum_t lambda_lm(theta_t) sum_p f(theta_t, phi_p) e^{-i m phi_p}.
    The sum over p by library FFT (no weight), the Legendre sum in C.  [nmaps, k*k]."""
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None]
    n = 2 * k - 1
    if f.shape[1:] != (k, n):
        raise ValueError("map must be [k, 2k-1]")
    ms = np.arange(-(k - 1), k)
    Gu = np.ascontiguousarray(np.fft.fft(f.astype(np.complex128), axis=-1)[..., ms % n])
    flm = np.zeros((f.shape[0], k * k), dtype=np.complex128)
    _load().orc_legendre_forward(k, f.shape[0], _dp(Gu.view(np.float64)), _dp(flm.view(np.float64)))
    return flm


def forward_sht_adjoint(flm: np.ndarray, k: int, reality: bool = False) -> np.ndarray:
    """A^H y with A the MW quadrature (forward_sht): the transposes of its steps 7..1 in reverse
    order (real part for real maps).  [nmaps, k, 2k-1]."""
    y = _as_maps(flm, k)
    nmaps = y.shape[0]
    n = 2 * k - 1
    ms = np.arange(-(k - 1), k)
    eps = np.where(ms % 2 == 0, 1.0, -1.0)
    js = np.arange(-(k - 1), k)
    # 7^H: F_m(theta_t) = sum_l lambda_lm(theta_t) y_lm   (t < k)
    F = np.zeros((nmaps, k, n), dtype=np.complex128)
    _load().orc_legendre_inverse(k, nmaps, _dp(y.view(np.float64)), _dp(F.view(np.float64)))
    # 6^H: the fold's transpose puts F[t] at t and eps F[t] at n-1-t (t < k-1)
    Hb = np.zeros((nmaps, n, n), dtype=np.complex128)
    Hb[:, :k, :] = F
    if k > 1:
        t = np.arange(k - 1)
        Hb[:, n - 1 - t, :] = eps[None, None, :] * F[:, t, :]
    # 5^H: H = fft(spec)/n  ->  spec_bar = ifft(H_bar); I_bar = conj(phase) spec_bar
    spec_b = np.fft.ifft(Hb, axis=1)
    Ib = np.exp(1j * np.pi * js / n)[None, :, None] * spec_b[:, js % n, :]
    # 4^H: Ghat_bar = W^H I_bar with W[j', j] = w(j + j')
    P = js[:, None] + js[None, :]
    W = quadrature_weight(P)
    WH = np.ascontiguousarray(W.conj().T)
    Gb_hat = np.matmul(WH[None], Ib)                  # sum_b WH[a, b] I_bar[x, b, m]
    # 3^H: Ghat = phase D / n, D = fft(g) at js  ->  g_bar = n ifft(conj(phase) Ghat_bar / n)
    Db = np.zeros((nmaps, n, n), dtype=np.complex128)
    Db[:, js % n, :] = np.exp(1j * np.pi * js / n)[None, :, None] * Gb_hat / n
    gb = np.fft.ifft(Db, axis=1) * n
    # 2^H: the extension's transpose folds g_bar back onto t < k
    Gb = gb[:, :k, :].copy()
    if k > 1:
        t = np.arange(k - 1)
        Gb[:, t, :] += eps[None, None, :] * gb[:, n - 1 - t, :]
    # 1^H: f(theta_t, phi_p) = (2 pi / n) sum_m G_bar_m e^{i m phi_p}
    spec = np.zeros((nmaps, k, n), dtype=np.complex128)
    spec[..., ms % n] = Gb
    f = (2.0 * np.pi / n) * np.fft.ifft(spec, axis=-1) * n
    return f.real.copy() if reality else f


# ----------------------------------------------------------------------------------------
# Scale-discretised tiling, Eqs. (10)-(16)
# ----------------------------------------------------------------------------------------
def j_max(L: int, B: int) -> int:
    """J = ceil(log_B(L-1)): the smallest integer J with B^J >= L-1 (integer-exact)."""
    if L < 3 or B < 2:
        raise ValueError("need L >= 3 and B >= 2")
    J, p = 0, 1
    while p < L - 1:
        p *= B
        J += 1
    return J


KERNELS = ("sd", "bspline")


def _ceil_frac(a: int, b: int) -> int:
    return -(-a // b)


def bandlimit_wav(j: int, L: int, B: int, multires: bool, kernel: str = "sd") -> int:
    """Band-limit of wavelet scale j (Sect. 3.1): without multiresolution L; with it
    min(B^{j+1}, L) for the scale-discretised kernels, and for the B-spline kernels the end of
    their support [0, L/B^{J-j-2}] rounded up, capped at L (L itself when J-j-2 <= 0)."""
    if not multires:
        return L
    if kernel == "bspline":
        e = j_max(L, B) - j - 2
        return L if e <= 0 else min(L, _ceil_frac(L, B ** e))
    return min(B ** (j + 1), L)


def bandlimit_scal(J_min: int, L: int, B: int, multires: bool, kernel: str = "sd") -> int:
    """Band-limit of the scaling part: supp eta = [0, B^{J_min}) for the scale-discretised
    kernels, so min(B^{J_min}, L); for the B-spline kernels eta^2 = k(l/B^{J_min}) vanishes from
    l = L/B^{J-J_min-1} on, so that value rounded up (capped at L)."""
    if not multires:
        return L
    if kernel == "bspline":
        e = j_max(L, B) - J_min - 1
        return L if e <= 0 else min(L, _ceil_frac(L, B ** e))
    return min(B ** J_min, L)


def schwartz(x: float) -> float:
    """s(t) = exp(-1/(1-t^2)) on (-1, 1), 0 elsewhere (Eq. (10))."""
    return math.exp(-1.0 / (1.0 - x * x)) if -1.0 < x < 1.0 else 0.0


def s_lambda(t: float, lam: float) -> float:
    """s_lambda(t) = s(2 lambda (t - 1/lambda)/(lambda - 1) - 1), support [1/lambda, 1] (Eq. (11))."""
    return schwartz(2.0 * lam * (t - 1.0 / lam) / (lam - 1.0) - 1.0)


_k_cache: dict = {}


def k_lambda(t: float, lam: float) -> float:
    """k_lambda(t) = int_t^1 s_lambda^2(u)/u du / int_{1/lambda}^1 s_lambda^2(u)/u du (Eq. (12));
    1 for t <= 1/lambda, 0 for t >= 1.  Adaptive Gauss-Kronrod (scipy.integrate.quad)."""
    from scipy.integrate import quad
    if t <= 1.0 / lam:
        return 1.0
    if t >= 1.0:
        return 0.0
    key = (float(t), float(lam))
    if key in _k_cache:
        return _k_cache[key]
    import warnings
    g = lambda u: s_lambda(u, lam) ** 2 / u
    den_key = ("den", float(lam))
    with warnings.catch_warnings():
        # QUADPACK cannot certify 1e-14 and says so; the values are checked against a
        # 30-digit tanh-sinh evaluation in the pin tests.
        warnings.simplefilter("ignore")
        if den_key not in _k_cache:
            _k_cache[den_key] = quad(g, 1.0 / lam, 1.0, epsabs=0.0, epsrel=1.2e-14, limit=400)[0]
        num = quad(g, t, 1.0, epsabs=0.0, epsrel=1.2e-14, limit=400)[0]
    val = num / _k_cache[den_key]
    _k_cache[key] = val
    return val


def kappa_lambda(t: float, lam: float) -> float:
    """kappa_lambda(t) = sqrt(k_lambda(t/lambda) - k_lambda(t))  (Eq. (13)).

    Both terms of the difference are integrals of the same integrand s_lambda^2(u)/u over
    [t/lambda, 1] and [t, 1] (each clamped to the support [1/lambda, 1]), so the difference is
    that integrand integrated over [max(t/lambda, 1/lambda), min(t, 1)], divided by the
    normalisation of Eq. (12); evaluating it as one integral avoids the cancellation of two
    values close to 1."""
    import warnings
    from scipy.integrate import quad
    lo, hi = max(t / lam, 1.0 / lam), min(t, 1.0)
    if hi <= lo:
        return 0.0
    g = lambda u: s_lambda(u, lam) ** 2 / u
    den_key = ("den", float(lam))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        if den_key not in _k_cache:
            _k_cache[den_key] = quad(g, 1.0 / lam, 1.0, epsabs=0.0, epsrel=1.2e-14, limit=400)[0]
        num = quad(g, lo, hi, epsabs=0.0, epsrel=1.2e-14, limit=400)[0]
    return math.sqrt(max(0.0, num / _k_cache[den_key]))


def eta_lambda(t: float, lam: float) -> float:
    """eta_lambda(t) = sqrt(k_lambda(t))  (Eq. (14))."""
    return math.sqrt(max(0.0, k_lambda(t, lam)))


# ----------------------------------------------------------------------------------------
# B-spline generating function (footnote to Sect. 2.2, Eqs. (17)-(18)), in exact rationals
# ----------------------------------------------------------------------------------------
def bspline_b3(x) -> Fraction:
    """B_3(x) = (|x-2|^3 - 4|x-1|^3 + 6|x|^3 - 4|x+1|^3 + |x+2|^3) / 12  (Eq. (18)), evaluated
    exactly on rationals.  The combination is the fourth central difference of |x|^3/12, which
    is zero for |x| >= 2 (it is then a fourth difference of a cubic); outside (-2, 2) the value
    0 is returned directly."""
    x = Fraction(x)
    if abs(x) >= 2:
        return Fraction(0)
    c = lambda u: abs(u) ** 3
    return (c(x - 2) - 4 * c(x - 1) + 6 * c(x) - 4 * c(x + 1) + c(x + 2)) / 12


def k_bspline(t, lam: int, L: int, J: int) -> Fraction:
    """k_lambda(t) = (3/2) B_3(2 t lambda^{J-1} / L)  (Eq. (17)); t rational."""
    return Fraction(3, 2) * bspline_b3(2 * Fraction(t) * Fraction(lam) ** (J - 1) / L)


def tiling_bspline_sq(L: int, B: int, J_min: int):
    """Squared B-spline kernels as exact rationals: (kappa2 [scale][l], eta2 [l]) with
    eta^2(l) = k(l/B^{J_min}), kappa_j^2(l) = k(l/B^{j+1}) - k(l/B^j) for j < J, and the top
    scale kappa_J^2(l) = 1 - k(l/B^J), which makes eta^2 + sum_j kappa_j^2 = 1 (Eq. (9)) hold for
    every l < L.  (For the scale-discretised kernels the same top-scale form coincides with
    Eq. (13), since there k(l/B^{J+1}) = 1 for l < L.)"""
    J = j_max(L, B)
    if not (0 <= J_min < J):
        raise ValueError("need 0 <= J_min < J")
    eta2 = [k_bspline(Fraction(l, B ** J_min), B, L, J) for l in range(L)]
    kap2 = []
    for j in range(J_min, J + 1):
        row = []
        for l in range(L):
            lo = k_bspline(Fraction(l, B ** j), B, L, J)
            hi = k_bspline(Fraction(l, B ** (j + 1)), B, L, J) if j < J else Fraction(1)
            row.append(hi - lo)
        kap2.append(row)
    return kap2, eta2


def tiling(L: int, B: int, J_min: int, kernel: str = "sd"):
    """Harmonic kernels of Eqs. (15)-(16) without the sqrt((2l+1)/4pi) factor, which cancels
    against the sqrt(4pi/(2l+1)) of Eqs. (4), (6) and (8):
      kappa[j - J_min, l] = kappa_B(l / B^j),  j = J_min..J
      eta[l]              = eta_B(l / B^J_min).
    kernel "sd": the scale-discretised functions of Eqs. (10)-(14); "bspline": Eqs. (17)-(18)."""
    if kernel == "bspline":
        kap2, eta2 = tiling_bspline_sq(L, B, J_min)
        return (np.array([[math.sqrt(v) for v in row] for row in kap2]),
                np.array([math.sqrt(v) for v in eta2]))
    if kernel != "sd":
        raise ValueError("kernel must be 'sd' or 'bspline'")
    J = j_max(L, B)
    if not (0 <= J_min < J):
        raise ValueError("need 0 <= J_min < J")
    kappa = np.zeros((J - J_min + 1, L))
    eta = np.zeros(L)
    for ell in range(L):
        eta[ell] = eta_lambda(ell / float(B) ** J_min, float(B))
        for j in range(J_min, J + 1):
            kappa[j - J_min, ell] = kappa_lambda(ell / float(B) ** j, float(B))
    return kappa, eta


# ----------------------------------------------------------------------------------------
# Wavelet analysis and synthesis, Eqs. (4), (6), (8)
# ----------------------------------------------------------------------------------------
def _truncate(flm: np.ndarray, L: int, k: int) -> np.ndarray:
    """Keep l < k of an [nmaps, L*L] array -> [nmaps, k*k] (index l*l+l+m is prefix-stable)."""
    return flm[:, :k * k].copy()


def _extend(flm: np.ndarray, k: int, L: int) -> np.ndarray:
    out = np.zeros((flm.shape[0], L * L), dtype=np.complex128)
    out[:, :k * k] = flm
    return out


def _ell_of_index(L: int) -> np.ndarray:
    return np.repeat(np.arange(L), 2 * np.arange(L) + 1)


def analysis_harmonic(flm: np.ndarray, L: int, B: int, J_min: int, multires: bool, kernel: str = "sd"):
    """Scaling and wavelet coefficients in harmonic space (Eqs. (4), (6)):
    W^Phi_lm = eta(l) f_lm for l < k_Phi;  W^j_lm = kappa_j(l) f_lm for l < k_j."""
    flm = _as_maps(flm, L)
    kappa, eta = tiling(L, B, J_min, kernel)
    ell = _ell_of_index(L)
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires, kernel)
    scal = _truncate(flm * eta[ell][None, :], L, kP)
    wav = []
    for j in range(J_min, J + 1):
        kj = bandlimit_wav(j, L, B, multires, kernel)
        wav.append(_truncate(flm * kappa[j - J_min][ell][None, :], L, kj))
    return wav, scal


def analysis(f: np.ndarray, L: int, B: int, J_min: int, multires: bool, reality: bool, kernel: str = "sd"):
    """Wavelet analysis of maps f [nmaps, L, 2L-1]: forward SHT at L, Eqs. (4)/(6), then an
    inverse SHT per scale at its band-limit.  Returns (list of wavelet maps per j, scaling map)."""
    flm = forward_sht(f, L)
    wav_lm, scal_lm = analysis_harmonic(flm, L, B, J_min, multires, kernel)
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires, kernel)
    scal = inverse_sht(scal_lm, kP, reality)
    wav = [inverse_sht(w, bandlimit_wav(j, L, B, multires, kernel), reality)
           for j, w in zip(range(J_min, J + 1), wav_lm)]
    return wav, scal


def synthesis_harmonic(wav_lm, scal_lm, L: int, B: int, J_min: int, multires: bool,
                       kernel: str = "sd") -> np.ndarray:
    """Eq. (8): f_lm = eta(l) W^Phi_lm + sum_j kappa_j(l) W^j_lm (scales zero-extended to L)."""
    kappa, eta = tiling(L, B, J_min, kernel)
    ell = _ell_of_index(L)
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires, kernel)
    out = _extend(_as_maps(scal_lm, kP), kP, L) * eta[ell][None, :]
    for j, w in zip(range(J_min, J + 1), wav_lm):
        kj = bandlimit_wav(j, L, B, multires, kernel)
        out = out + _extend(_as_maps(w, kj), kj, L) * kappa[j - J_min][ell][None, :]
    return out


def synthesis(wav, scal, L: int, B: int, J_min: int, multires: bool, reality: bool,
              kernel: str = "sd") -> np.ndarray:
    """Wavelet synthesis: forward SHT of each scale at its band-limit, Eq. (8), inverse SHT at L."""
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires, kernel)
    scal_lm = forward_sht(scal, kP)
    wav_lm = [forward_sht(w, bandlimit_wav(j, L, B, multires, kernel))
              for j, w in zip(range(J_min, J + 1), wav)]
    flm = synthesis_harmonic(wav_lm, scal_lm, L, B, J_min, multires, kernel)
    return inverse_sht(flm, L, reality)


def analysis_adjoint(wav, scal, L: int, B: int, J_min: int, multires: bool, reality: bool) -> np.ndarray:
    """Adjoint of analysis: A^H ( eta ext(S_Phi^H scal) + sum_j kappa_j ext(S_j^H wav_j) )."""
    kappa, eta = tiling(L, B, J_min)
    ell = _ell_of_index(L)
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires)
    acc = _extend(inverse_sht_adjoint(scal, kP, reality), kP, L) * eta[ell][None, :]
    for j, w in zip(range(J_min, J + 1), wav):
        kj = bandlimit_wav(j, L, B, multires)
        acc = acc + _extend(inverse_sht_adjoint(w, kj, reality), kj, L) * kappa[j - J_min][ell][None, :]
    return forward_sht_adjoint(acc, L, reality)


def synthesis_adjoint(f: np.ndarray, L: int, B: int, J_min: int, multires: bool, reality: bool):
    """Adjoint of synthesis: g = S_L^H f, then A_Phi^H trunc(eta g) and A_j^H trunc(kappa_j g)."""
    kappa, eta = tiling(L, B, J_min)
    ell = _ell_of_index(L)
    J = j_max(L, B)
    kP = bandlimit_scal(J_min, L, B, multires)
    g = inverse_sht_adjoint(f, L, reality)
    scal = forward_sht_adjoint(_truncate(g * eta[ell][None, :], L, kP), kP, reality)
    wav = []
    for j in range(J_min, J + 1):
        kj = bandlimit_wav(j, L, B, multires)
        wav.append(forward_sht_adjoint(_truncate(g * kappa[j - J_min][ell][None, :], L, kj), kj, reality))
    return wav, scal


# ----------------------------------------------------------------------------------------
# Denoising by hard thresholding (Sect. 4.3, Eqs. (19)-(23))
# ----------------------------------------------------------------------------------------
def noise_std(L: int, B: int, J_min: int, sigma: float, kernel: str = "sd") -> np.ndarray:
    """sigma_j (j = J_min..J) for white noise with E|n_lm|^2 = sigma^2 (Eq. (19)):
    (sigma_j)^2 = sigma^2 sum_l |Psi^j_l0|^2 with Psi^j_l0 = sqrt((2l+1)/4pi) kappa_j(l)
    (Eq. (15))."""
    kappa, _ = tiling(L, B, J_min, kernel)
    ell = np.arange(L)
    psi2 = (2.0 * ell + 1.0) / (4.0 * math.pi) * kappa ** 2
    return sigma * np.sqrt(np.sum(psi2, axis=1))


def hard_threshold(wav, thresholds):
    """Eq. (23), read with the magnitude: D^j = 0 where |Y^j| < T^j, Y^j elsewhere.  wav: list
    over scales of arrays; thresholds: one value per scale.  Returns new arrays."""
    out = []
    for w, t in zip(wav, thresholds):
        d = np.array(w, copy=True)
        d[np.abs(d) < t] = 0
        out.append(d)
    return out


def snr(s_lm, y_lm) -> float:
    """SNR(y) = 10 log10(||s||^2 / ||y - s||^2) (Eq. (20)) with the energies summed over
    harmonic coefficients (Eq. (21))."""
    s_lm, y_lm = np.asarray(s_lm), np.asarray(y_lm)
    return 10.0 * math.log10(float(np.sum(np.abs(s_lm) ** 2)) / float(np.sum(np.abs(y_lm - s_lm) ** 2)))


def denoise(y, L: int, B: int, J_min: int, sigma: float, multires: bool, reality: bool,
            kernel: str = "sd", nsigma: float = 3.0):
    """Wavelet analysis of y, hard thresholding of every wavelet scale at T_j = nsigma sigma_j,
    and synthesis from the thresholded scales and the untouched scaling part (Sect. 4.3)."""
    wav, scal = analysis(y, L, B, J_min, multires, reality, kernel)
    wav = hard_threshold(wav, nsigma * noise_std(L, B, J_min, sigma, kernel))
    return synthesis(wav, scal, L, B, J_min, multires, reality, kernel)


# ----------------------------------------------------------------------------------------
# Error metrics (Sect. 3.3)
# ----------------------------------------------------------------------------------------
def max_abs_err(x, y) -> float:
    """epsilon = max |x - y| (the paper's metric)."""
    return float(np.max(np.abs(np.asarray(x) - np.asarray(y)))) if np.size(x) else 0.0


def rel_max_err(x, y) -> float:
    """max |x - y| / max |y|."""
    y = np.asarray(y)
    den = float(np.max(np.abs(y))) if y.size else 0.0
    return max_abs_err(x, y) / den if den > 0 else max_abs_err(x, y)
