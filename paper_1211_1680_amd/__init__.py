"""Python binding of libs2let_mi355x: the exact MW spherical harmonic transform and the
axisymmetric scale-discretised wavelet transform on one MI355X (gfx950).

Argument marshalling only: every step of the transforms runs in the HIP kernels behind the
C ABI declared in include/s2let_mi355x.h.  torch supplies device memory (inputs, outputs and
the workspace, all caller-owned) and the current stream.  There is no CPU fallback: if the
library or a GPU is missing the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "REAL", "COMPLEX", "FP64", "MIXED_FP32", "MIXED_BF16X3", "MAX_L", "S2letError", "lib",
    "j_max", "bandlimit_wav", "bandlimit_scal", "mw_size", "wav_size", "tiling_axisym",
    "workspace_size", "mw_forward", "mw_inverse", "analysis", "synthesis", "split_wav", "sync",
    "analysis_noalloc", "NOALLOC_SCRATCH_BYTES", "BATCH_STREAMS", "BATCH_PERSISTENT",
    "mw_forward_adjoint", "mw_inverse_adjoint", "analysis_adjoint", "synthesis_adjoint",
    "BatchPlan", "profile_enable", "profile_query", "STAGES",
    "KERNEL_SD", "KERNEL_BSPLINE", "KERNEL_NEEDLET", "noise_std", "hard_threshold", "denoise",
]

REAL, COMPLEX = 0, 1
FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
KERNEL_SD, KERNEL_BSPLINE, KERNEL_NEEDLET = 0, 1, 2
MAX_L = 2048
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, ENOTREADY, ESCRATCH = 0, -1, -2, -3, -4, -5, -6
BATCH_STREAMS, BATCH_PERSISTENT = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20   # S2LET_NOALLOC_SCRATCH_BYTES

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libs2let_mi355x.so")


class S2letError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.s2let_strerror(status).decode() if _lib is not None else str(status)
        if status == EHIP and _lib is not None:
            msg += ": %s" % _lib.s2let_last_hip_error_name().decode()
        super().__init__("%s failed: %s (status %d)" % (where, msg, status))
        self.status = status


def _load():
    # torch ships its own HIP and HSA runtimes under the same sonames as /opt/rocm's.  Loaded
    # first, they satisfy this library's dependencies and the process holds one runtime; loaded
    # after this library, torch would map a second pair, and the second HSA runtime to open the
    # device reports that there is none.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libs2let_mi355x.so is not built (run __graft_entry__.build() or "
                          "python paper_1211_1680_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    i, i64, sz, vp, dp = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, \
        ctypes.POINTER(ctypes.c_double)
    sig = {
        "s2let_j_max": (i, [i, i]),
        "s2let_bandlimit_wav": (i, [i, i, i, i]),
        "s2let_bandlimit_scal": (i, [i, i, i, i]),
        "s2let_mw_size": (i64, [i]),
        "s2let_wav_size": (i64, [i, i, i, i]),
        "s2let_tiling_axisym": (i, [dp, dp, i, i, i]),
        "s2let_workspace_size": (sz, [i, i, i, i, i, i, i, i]),
        "mw_forward": (i, [vp, vp, i, i, i, i, vp, sz, vp]),
        "mw_inverse": (i, [vp, vp, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_analysis": (i, [vp, vp, vp, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_synthesis": (i, [vp, vp, vp, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_analysis_noalloc": (i, [vp, vp, vp, i, i, i, i, i, i, i, vp]),
        "mw_forward_adjoint": (i, [vp, vp, i, i, i, i, vp, sz, vp]),
        "mw_inverse_adjoint": (i, [vp, vp, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_analysis_adjoint": (i, [vp, vp, vp, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_synthesis_adjoint": (i, [vp, vp, vp, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_batch_create": (i, [ctypes.POINTER(vp), i, ctypes.POINTER(i), ctypes.POINTER(i), i, i, i, i]),
        "s2let_batch_destroy": (i, [vp]),
        "s2let_batch_layout": (i, [vp] + [ctypes.POINTER(ctypes.c_int64)] * 4),
        "s2let_batch_workspace_size": (sz, [vp]),
        "s2let_batch_analysis": (i, [vp, vp, vp, vp, vp, sz, vp]),
        "s2let_batch_run": (i, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "s2let_batch_autotune": (i, [vp, vp, vp, vp, vp, vp, sz, vp, ctypes.POINTER(i), ctypes.POINTER(i),
                                     ctypes.POINTER(ctypes.c_float)]),
        "s2let_batch_graph_capture": (i, [vp, vp, vp, vp, vp, vp, sz, vp]),
        "s2let_batch_graph_launch": (i, [vp, vp]),
        "s2let_batch_set_execution": (i, [vp, i, ctypes.POINTER(i), ctypes.POINTER(i)]),
        "s2let_batch_get_execution": (i, [vp] + [ctypes.POINTER(i)] * 5),
        "s2let_bandlimit_wav_kernel": (i, [i, i, i, i, i]),
        "s2let_bandlimit_scal_kernel": (i, [i, i, i, i, i]),
        "s2let_wav_size_kernel": (i64, [i, i, i, i, i]),
        "s2let_tiling_axisym_kernel": (i, [dp, dp, i, i, i, i]),
        "s2let_axisym_analysis_kernel": (i, [vp, vp, vp, i, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_axisym_synthesis_kernel": (i, [vp, vp, vp, i, i, i, i, i, i, i, i, vp, sz, vp]),
        "s2let_noise_std_axisym": (i, [dp, i, i, i, i, ctypes.c_double]),
        "s2let_hard_threshold": (i, [vp, dp, i, i, i, i, i, i, i, vp]),
        "s2let_sync": (i, [vp]),
        "s2let_profile_enable": (i, [i]),
        "s2let_profile_query": (i, [i, dp, ctypes.POINTER(ctypes.c_int64), dp, dp, dp]),
        "s2let_profile_query_k": (i, [i, i, dp, ctypes.POINTER(ctypes.c_int64), dp, dp, dp]),
        "s2let_finalize": (None, []),
        "s2let_strerror": (ctypes.c_char_p, [i]),
        "s2let_last_hip_error": (i, []),
        "s2let_last_hip_error_name": (ctypes.c_char_p, []),
        "s2let_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
lib = _lib


def _check(status: int, where: str):
    if status != OK:
        raise S2letError(status, where)


# ---------------------------------------------------------------- host helpers
def j_max(L: int, B: int) -> int:
    r = _lib.s2let_j_max(L, B)
    _check(min(r, 0), "s2let_j_max")
    return r


def bandlimit_wav(j: int, L: int, B: int, multires: bool, kernel: int = KERNEL_SD) -> int:
    r = _lib.s2let_bandlimit_wav_kernel(j, L, B, int(multires), kernel)
    _check(min(r, 0), "s2let_bandlimit_wav_kernel")
    return r


def bandlimit_scal(J_min: int, L: int, B: int, multires: bool, kernel: int = KERNEL_SD) -> int:
    r = _lib.s2let_bandlimit_scal_kernel(J_min, L, B, int(multires), kernel)
    _check(min(r, 0), "s2let_bandlimit_scal_kernel")
    return r


def mw_size(k: int) -> int:
    r = _lib.s2let_mw_size(k)
    if r < 0:
        raise S2letError(EINVAL, "s2let_mw_size")
    return r


def wav_size(L: int, B: int, J_min: int, multires: bool, kernel: int = KERNEL_SD) -> int:
    r = _lib.s2let_wav_size_kernel(L, B, J_min, int(multires), kernel)
    if r < 0:
        raise S2letError(EINVAL, "s2let_wav_size_kernel")
    return r


def tiling_axisym(L: int, B: int, J_min: int, kernel: int = KERNEL_SD):
    """(kappa [J-J_min+1, L], eta [L]) as numpy arrays (host computation in the library)."""
    J = j_max(L, B)
    kappa = np.zeros((J - J_min + 1, L))
    eta = np.zeros(L)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(_lib.s2let_tiling_axisym_kernel(kappa.ctypes.data_as(dp), eta.ctypes.data_as(dp), L, B, J_min,
                                           kernel), "s2let_tiling_axisym_kernel")
    return kappa, eta


def noise_std(L: int, B: int, J_min: int, sigma: float, kernel: int = KERNEL_SD):
    """sigma_j, j = J_min..J: standard deviation of white harmonic noise of variance sigma^2
    seen through wavelet scale j (host computation in the library)."""
    out = np.zeros(j_max(L, B) - J_min + 1)
    _check(_lib.s2let_noise_std_axisym(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), L, B, J_min,
                                       kernel, float(sigma)), "s2let_noise_std_axisym")
    return out


def workspace_size(L, B=2, J_min=0, multires=False, reality=REAL, precision=FP64, nmaps=1,
                   wavelet=False) -> int:
    return int(_lib.s2let_workspace_size(L, B, J_min, int(multires), reality, precision, nmaps,
                                         int(wavelet)))


# ---------------------------------------------------------------- device calls
def _torch():
    import torch
    return torch


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(nbytes: int, device, workspace=None):
    torch = _torch()
    if nbytes == 0:
        raise S2letError(EINVAL, "s2let_workspace_size")
    if workspace is not None:
        _need_cuda(workspace, "workspace", torch.uint8, device=device)
        if workspace.numel() < nbytes:
            raise S2letError(ENOMEM, "workspace")
        return workspace
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _need_cuda(t, name, dtype, numel=None, device=None):
    """Checks a tensor handed to the C ABI: the library sees only its address, so the dtype,
    device, layout and (when given) element count are checked here."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if device is not None and t.device != torch.device(device):
        raise ValueError("%s must be on %s (it is on %s)" % (name, device, t.device))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must hold %d elements (it holds %d)" % (name, numel, t.numel()))
    return t


def _map_dtype(reality):
    torch = _torch()
    return torch.float64 if reality == REAL else torch.complex128


def mw_forward(f, L: int, reality: int = REAL, precision: int = FP64, workspace=None):
    """f: [nmaps, L, 2L-1] (float64 for REAL, complex128 for COMPLEX) -> flm [nmaps, L*L]."""
    torch = _torch()
    _need_cuda(f, "f", _map_dtype(reality))
    nmaps = f.shape[0] if f.dim() == 3 else 1
    if f.numel() != nmaps * mw_size(L):
        raise ValueError("f must hold nmaps * L * (2L-1) samples")
    flm = torch.empty((nmaps, L * L), dtype=torch.complex128, device=f.device)
    ws = _workspace(workspace_size(L, reality=reality, precision=precision, nmaps=nmaps), f.device,
                    workspace)
    _check(_lib.mw_forward(flm.data_ptr(), f.data_ptr(), L, reality, precision, nmaps,
                           ws.data_ptr(), ws.numel() * ws.element_size(), _stream(f.device)),
           "mw_forward")
    return flm


def mw_inverse(flm, L: int, reality: int = REAL, precision: int = FP64, workspace=None):
    """flm: [nmaps, L*L] complex128 -> f [nmaps, L, 2L-1]."""
    torch = _torch()
    _need_cuda(flm, "flm", torch.complex128)
    nmaps = flm.shape[0] if flm.dim() == 2 else 1
    if flm.numel() != nmaps * L * L:
        raise ValueError("flm must hold nmaps * L * L coefficients")
    f = torch.empty((nmaps, L, 2 * L - 1), dtype=_map_dtype(reality), device=flm.device)
    ws = _workspace(workspace_size(L, reality=reality, precision=precision, nmaps=nmaps),
                    flm.device, workspace)
    _check(_lib.mw_inverse(f.data_ptr(), flm.data_ptr(), L, reality, precision, nmaps,
                           ws.data_ptr(), ws.numel() * ws.element_size(), _stream(flm.device)),
           "mw_inverse")
    return f


def analysis(f, L: int, B: int, J_min: int, multires: bool = True, reality: int = REAL,
             precision: int = FP64, workspace=None, out=None, kernel: int = KERNEL_SD):
    """Wavelet analysis.  Returns (f_wav [nmaps, wav_size], f_scal [nmaps, mw_size(k_Phi)])."""
    torch = _torch()
    dt = _map_dtype(reality)
    _need_cuda(f, "f", dt)
    nmaps = f.shape[0] if f.dim() == 3 else 1
    if f.numel() != nmaps * mw_size(L):
        raise ValueError("f must hold nmaps * L * (2L-1) samples")
    kP = bandlimit_scal(J_min, L, B, multires, kernel)
    nw, ns = nmaps * wav_size(L, B, J_min, multires, kernel), nmaps * mw_size(kP)
    if out is None:
        f_wav = torch.empty((nmaps, nw // nmaps), dtype=dt, device=f.device)
        f_scal = torch.empty((nmaps, ns // nmaps), dtype=dt, device=f.device)
    else:
        f_wav, f_scal = out
        _need_cuda(f_wav, "out[0] (f_wav)", dt, nw, f.device)
        _need_cuda(f_scal, "out[1] (f_scal)", dt, ns, f.device)
    ws = _workspace(workspace_size(L, B, J_min, multires, reality, precision, nmaps, True),
                    f.device, workspace)
    _check(_lib.s2let_axisym_analysis_kernel(f_wav.data_ptr(), f_scal.data_ptr(), f.data_ptr(), L, B, J_min,
                                             int(multires), kernel, reality, precision, nmaps, ws.data_ptr(),
                                             ws.numel() * ws.element_size(), _stream(f.device)),
           "s2let_axisym_analysis_kernel")
    return f_wav, f_scal


def analysis_noalloc(f, L: int, B: int, J_min: int, multires: bool, reality: int, precision: int, out):
    """Wavelet analysis through the allocation-free entry point s2let_axisym_analysis_noalloc:
    the library's static device scratch replaces the workspace, and the caller passes the outputs
    out = (f_wav [nmaps, wav_size], f_scal [nmaps, mw_size(k_Phi)]).  The plan tables must exist
    on the device (one earlier `analysis` call with the same L, B, J_min, multires); calls that
    overlap on one device race.  Returns out."""
    dt = _map_dtype(reality)
    _need_cuda(f, "f", dt)
    nmaps = f.shape[0] if f.dim() == 3 else 1
    if f.numel() != nmaps * mw_size(L):
        raise ValueError("f must hold nmaps * L * (2L-1) samples")
    kP = bandlimit_scal(J_min, L, B, multires)
    f_wav, f_scal = out
    _need_cuda(f_wav, "out[0] (f_wav)", dt, nmaps * wav_size(L, B, J_min, multires), f.device)
    _need_cuda(f_scal, "out[1] (f_scal)", dt, nmaps * mw_size(kP), f.device)
    _check(_lib.s2let_axisym_analysis_noalloc(f_wav.data_ptr(), f_scal.data_ptr(), f.data_ptr(), L, B, J_min,
                                              int(multires), reality, precision, nmaps, _stream(f.device)),
           "s2let_axisym_analysis_noalloc")
    return f_wav, f_scal


def synthesis(f_wav, f_scal, L: int, B: int, J_min: int, multires: bool = True,
              reality: int = REAL, precision: int = FP64, workspace=None, out=None, kernel: int = KERNEL_SD):
    """Wavelet synthesis (Eq. (8)).  Returns f [nmaps, L, 2L-1]."""
    torch = _torch()
    dt = _map_dtype(reality)
    _need_cuda(f_wav, "f_wav", dt)
    nmaps = f_wav.shape[0] if f_wav.dim() == 2 else 1
    if f_wav.numel() != nmaps * wav_size(L, B, J_min, multires, kernel):
        raise ValueError("f_wav has the wrong size")
    _need_cuda(f_scal, "f_scal", dt, nmaps * mw_size(bandlimit_scal(J_min, L, B, multires, kernel)), f_wav.device)
    if out is not None:
        _need_cuda(out, "out", dt, nmaps * mw_size(L), f_wav.device)
    f = out if out is not None else torch.empty((nmaps, L, 2 * L - 1), dtype=dt, device=f_wav.device)
    ws = _workspace(workspace_size(L, B, J_min, multires, reality, precision, nmaps, True),
                    f_wav.device, workspace)
    _check(_lib.s2let_axisym_synthesis_kernel(f.data_ptr(), f_wav.data_ptr(), f_scal.data_ptr(), L, B, J_min,
                                              int(multires), kernel, reality, precision, nmaps, ws.data_ptr(),
                                              ws.numel() * ws.element_size(), _stream(f_wav.device)),
           "s2let_axisym_synthesis_kernel")
    return f


def hard_threshold(f_wav, thresholds, L: int, B: int, J_min: int, multires: bool = True,
                   reality: int = REAL, kernel: int = KERNEL_SD):
    """In place on the device: wavelet samples of scale j with magnitude below thresholds[j - J_min]
    are set to zero (Eq. (23)).  Returns f_wav."""
    dt = _map_dtype(reality)
    _need_cuda(f_wav, "f_wav", dt)
    nmaps = f_wav.shape[0] if f_wav.dim() == 2 else 1
    if f_wav.numel() != nmaps * wav_size(L, B, J_min, multires, kernel):
        raise ValueError("f_wav has the wrong size")
    thr = np.ascontiguousarray(thresholds, dtype=np.float64)
    if thr.shape != (j_max(L, B) - J_min + 1,):
        raise ValueError("one threshold per wavelet scale is needed")
    _check(_lib.s2let_hard_threshold(f_wav.data_ptr(), thr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), L, B,
                                     J_min, int(multires), kernel, reality, nmaps, _stream(f_wav.device)),
           "s2let_hard_threshold")
    return f_wav


def denoise(y, L: int, B: int, J_min: int, sigma: float, multires: bool = True, reality: int = REAL,
            kernel: int = KERNEL_SD, nsigma: float = 3.0, precision: int = FP64):
    """Wavelet hard-threshold denoising of maps y: analysis, thresholds T_j = nsigma * sigma_j on
    the wavelet scales (the scaling part is kept), synthesis.  sigma is the standard deviation of
    the white noise's harmonic coefficients.  Returns the denoised maps."""
    f_wav, f_scal = analysis(y, L, B, J_min, multires, reality, precision, kernel=kernel)
    hard_threshold(f_wav, nsigma * noise_std(L, B, J_min, sigma, kernel), L, B, J_min, multires, reality, kernel)
    return synthesis(f_wav, f_scal, L, B, J_min, multires, reality, precision, kernel=kernel)


def mw_inverse_adjoint(f, L: int, reality: int = REAL, precision: int = FP64, workspace=None):
    """Adjoint of mw_inverse: f [nmaps, L, 2L-1] -> flm [nmaps, L*L], flm = S^H f."""
    torch = _torch()
    _need_cuda(f, "f", _map_dtype(reality))
    nmaps = f.shape[0] if f.dim() == 3 else 1
    if f.numel() != nmaps * mw_size(L):
        raise ValueError("f must hold nmaps * L * (2L-1) samples")
    flm = torch.empty((nmaps, L * L), dtype=torch.complex128, device=f.device)
    ws = _workspace(workspace_size(L, reality=reality, precision=precision, nmaps=nmaps), f.device,
                    workspace)
    _check(_lib.mw_inverse_adjoint(flm.data_ptr(), f.data_ptr(), L, reality, precision, nmaps,
                                   ws.data_ptr(), ws.numel() * ws.element_size(), _stream(f.device)),
           "mw_inverse_adjoint")
    return flm


def mw_forward_adjoint(flm, L: int, reality: int = REAL, precision: int = FP64, workspace=None):
    """Adjoint of mw_forward: flm [nmaps, L*L] complex128 -> f [nmaps, L, 2L-1], f = A^H flm
    (its real part for REAL maps)."""
    torch = _torch()
    _need_cuda(flm, "flm", torch.complex128)
    nmaps = flm.shape[0] if flm.dim() == 2 else 1
    if flm.numel() != nmaps * L * L:
        raise ValueError("flm must hold nmaps * L * L coefficients")
    f = torch.empty((nmaps, L, 2 * L - 1), dtype=_map_dtype(reality), device=flm.device)
    ws = _workspace(workspace_size(L, reality=reality, precision=precision, nmaps=nmaps),
                    flm.device, workspace)
    _check(_lib.mw_forward_adjoint(f.data_ptr(), flm.data_ptr(), L, reality, precision, nmaps,
                                   ws.data_ptr(), ws.numel() * ws.element_size(), _stream(flm.device)),
           "mw_forward_adjoint")
    return f


def analysis_adjoint(f_wav, f_scal, L: int, B: int, J_min: int, multires: bool = True,
                     reality: int = REAL, precision: int = FP64, workspace=None, out=None):
    """Adjoint of analysis: (f_wav, f_scal) -> f [nmaps, L, 2L-1]."""
    torch = _torch()
    dt = _map_dtype(reality)
    _need_cuda(f_wav, "f_wav", dt)
    nmaps = f_wav.shape[0] if f_wav.dim() == 2 else 1
    if f_wav.numel() != nmaps * wav_size(L, B, J_min, multires):
        raise ValueError("f_wav has the wrong size")
    _need_cuda(f_scal, "f_scal", dt, nmaps * mw_size(bandlimit_scal(J_min, L, B, multires)), f_wav.device)
    if out is not None:
        _need_cuda(out, "out", dt, nmaps * mw_size(L), f_wav.device)
    f = out if out is not None else torch.empty((nmaps, L, 2 * L - 1), dtype=dt, device=f_wav.device)
    ws = _workspace(workspace_size(L, B, J_min, multires, reality, precision, nmaps, True),
                    f_wav.device, workspace)
    _check(_lib.s2let_axisym_analysis_adjoint(f.data_ptr(), f_wav.data_ptr(), f_scal.data_ptr(), L, B,
                                              J_min, int(multires), reality, precision, nmaps,
                                              ws.data_ptr(), ws.numel() * ws.element_size(),
                                              _stream(f_wav.device)),
           "s2let_axisym_analysis_adjoint")
    return f


def synthesis_adjoint(f, L: int, B: int, J_min: int, multires: bool = True, reality: int = REAL,
                      precision: int = FP64, workspace=None, out=None):
    """Adjoint of synthesis: f [nmaps, L, 2L-1] -> (f_wav, f_scal)."""
    torch = _torch()
    dt = _map_dtype(reality)
    _need_cuda(f, "f", dt)
    nmaps = f.shape[0] if f.dim() == 3 else 1
    if f.numel() != nmaps * mw_size(L):
        raise ValueError("f must hold nmaps * L * (2L-1) samples")
    kP = bandlimit_scal(J_min, L, B, multires)
    nw, ns = nmaps * wav_size(L, B, J_min, multires), nmaps * mw_size(kP)
    if out is None:
        f_wav = torch.empty((nmaps, nw // nmaps), dtype=dt, device=f.device)
        f_scal = torch.empty((nmaps, ns // nmaps), dtype=dt, device=f.device)
    else:
        f_wav, f_scal = out
        _need_cuda(f_wav, "out[0] (f_wav)", dt, nw, f.device)
        _need_cuda(f_scal, "out[1] (f_scal)", dt, ns, f.device)
    ws = _workspace(workspace_size(L, B, J_min, multires, reality, precision, nmaps, True),
                    f.device, workspace)
    _check(_lib.s2let_axisym_synthesis_adjoint(f_wav.data_ptr(), f_scal.data_ptr(), f.data_ptr(), L, B,
                                               J_min, int(multires), reality, precision, nmaps,
                                               ws.data_ptr(), ws.numel() * ws.element_size(),
                                               _stream(f.device)),
           "s2let_axisym_synthesis_adjoint")
    return f_wav, f_scal


def split_wav(f_wav, L: int, B: int, J_min: int, multires: bool = True, kernel: int = KERNEL_SD):
    """Views of the concatenated wavelet maps: list over j = J_min..J of [nmaps, k_j, 2k_j-1]."""
    out, off = [], 0
    nmaps = f_wav.shape[0]
    for j in range(J_min, j_max(L, B) + 1):
        k = bandlimit_wav(j, L, B, multires, kernel)
        n = mw_size(k)
        out.append(f_wav[:, off:off + n].reshape(nmaps, k, 2 * k - 1))
        off += n
    return out


class BatchPlan:
    """Wavelet analysis + synthesis of many maps with uneven (L, B) (s2let_batch_* in the C ABI).

    Maps are concatenated in the given order in one flat tensor (float64 for REAL, complex128
    for COMPLEX); wavelet and scaling maps likewise (offsets from ``map_off``, ``wav_off``,
    ``scal_off``).  The plan owns worker streams and a few device tables; call ``close()``."""

    def __init__(self, Ls, Bs, J_min: int, multires: bool = True, reality: int = REAL,
                 precision: int = FP64, device=None):
        torch = _torch()
        self.Ls, self.Bs = [int(x) for x in Ls], [int(x) for x in Bs]
        if len(self.Ls) != len(self.Bs) or not self.Ls:
            raise ValueError("Ls and Bs must have the same nonzero length")
        self.J_min, self.multires, self.reality, self.precision = J_min, multires, reality, precision
        self.device = torch.device("cuda:0") if device is None else torch.device(device)
        n = len(self.Ls)
        arrL = (ctypes.c_int * n)(*self.Ls)
        arrB = (ctypes.c_int * n)(*self.Bs)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.s2let_batch_create(ctypes.byref(h), n, arrL, arrB, J_min, int(multires), reality,
                                           precision), "s2let_batch_create")
        self._h = h
        tot = (ctypes.c_int64 * 3)()
        mo, wo, so = (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)(), (ctypes.c_int64 * n)()
        _check(_lib.s2let_batch_layout(h, tot, mo, wo, so), "s2let_batch_layout")
        cm = 1 if reality == REAL else 2
        self.totals = [int(t) // cm for t in tot]          # in elements of the map dtype
        self.map_off = [int(x) // cm for x in mo]
        self.wav_off = [int(x) // cm for x in wo]
        self.scal_off = [int(x) // cm for x in so]
        self.ws = torch.empty(int(_lib.s2let_batch_workspace_size(h)), dtype=torch.uint8, device=self.device)
        self._captured = None

    def _dtype(self):
        return _map_dtype(self.reality)

    def outputs(self):
        torch = _torch()
        dt = self._dtype()
        return (torch.empty(self.totals[1], dtype=dt, device=self.device),
                torch.empty(self.totals[2], dtype=dt, device=self.device),
                torch.empty(self.totals[0], dtype=dt, device=self.device))

    def _ws(self):
        return self.ws.data_ptr(), self.ws.numel()

    def _check_bufs(self, f, f_wav=None, f_scal=None, rec=None):
        dt = self._dtype()
        _need_cuda(f, "f", dt, self.totals[0], self.device)
        if f_wav is not None:
            _need_cuda(f_wav, "f_wav", dt, self.totals[1], self.device)
        if f_scal is not None:
            _need_cuda(f_scal, "f_scal", dt, self.totals[2], self.device)
        if rec is not None:
            _need_cuda(rec, "rec", dt, self.totals[0], self.device)

    def analysis(self, f, out=None):
        f_wav, f_scal, _ = self.outputs() if out is None else (out[0], out[1], None)
        self._check_bufs(f, f_wav, f_scal)
        _check(_lib.s2let_batch_analysis(self._h, f_wav.data_ptr(), f_scal.data_ptr(), f.data_ptr(), *self._ws(),
                                         _stream(self.device)), "s2let_batch_analysis")
        return f_wav, f_scal

    def run(self, f, out=None):
        """Analysis then synthesis: returns (f_wav, f_scal, reconstruction)."""
        f_wav, f_scal, rec = self.outputs() if out is None else out
        self._check_bufs(f, f_wav, f_scal, rec)
        _check(_lib.s2let_batch_run(self._h, f_wav.data_ptr(), f_scal.data_ptr(), rec.data_ptr(), f.data_ptr(),
                                    *self._ws(), _stream(self.device)), "s2let_batch_run")
        return f_wav, f_scal, rec

    def autotune(self, f, out):
        s_, c_, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
        f_wav, f_scal, rec = out
        self._check_bufs(f, f_wav, f_scal, rec)
        # a new configuration discards any captured graph (and the buffers it was bound to)
        self._captured = None
        _check(_lib.s2let_batch_autotune(self._h, f_wav.data_ptr(), f_scal.data_ptr(), rec.data_ptr(),
                                         f.data_ptr(), *self._ws(), _stream(self.device), ctypes.byref(s_),
                                         ctypes.byref(c_), ctypes.byref(ms)), "s2let_batch_autotune")
        return s_.value, c_.value, ms.value

    def set_execution(self, mode: int, nw_analysis=None, nw_synthesis=None):
        """Streams or persistent mode; tile shapes (waves per block) for the band-limit buckets
        64, 128, ..., 2048 (6 entries each, None keeps the current ones)."""
        def arr(v):
            if v is None:
                return None
            v = [int(x) for x in v]
            if len(v) != 6:
                raise ValueError("one tile shape per band-limit bucket (6) is needed")
            return (ctypes.c_int * 6)(*v)
        self._captured = None
        _check(_lib.s2let_batch_set_execution(self._h, int(mode), arr(nw_analysis), arr(nw_synthesis)),
               "s2let_batch_set_execution")

    def execution(self):
        """{'mode', 'streams', 'maps_per_batch', 'nw_analysis', 'nw_synthesis'} of the current plan."""
        mo, ns, mp = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        fa, sy = (ctypes.c_int * 6)(), (ctypes.c_int * 6)()
        _check(_lib.s2let_batch_get_execution(self._h, ctypes.byref(mo), ctypes.byref(ns), ctypes.byref(mp), fa, sy),
               "s2let_batch_get_execution")
        return {"mode": "persistent" if mo.value == BATCH_PERSISTENT else "streams", "streams": ns.value,
                "maps_per_batch": mp.value, "nw_analysis": list(fa), "nw_synthesis": list(sy)}

    def capture(self, f, out):
        """Capture run(f, out) into a HIP graph on the current (non-default) stream.  The graph
        writes through the addresses of f and out, so the plan keeps both alive until the next
        capture, autotune or close."""
        f_wav, f_scal, rec = out
        self._check_bufs(f, f_wav, f_scal, rec)
        _check(_lib.s2let_batch_graph_capture(self._h, f_wav.data_ptr(), f_scal.data_ptr(), rec.data_ptr(),
                                              f.data_ptr(), *self._ws(), _stream(self.device)),
               "s2let_batch_graph_capture")
        self._captured = (f, f_wav, f_scal, rec)

    def replay(self):
        if getattr(self, "_captured", None) is None:
            raise RuntimeError("BatchPlan.replay: no captured graph (call capture() first)")
        _check(_lib.s2let_batch_graph_launch(self._h, _stream(self.device)), "s2let_batch_graph_launch")

    def map_view(self, flat, i, kind="map"):
        """Map i of a flat buffer: kind 'map' -> [L, 2L-1]; 'wav' -> list of scale maps; 'scal'."""
        L, B = self.Ls[i], self.Bs[i]
        if kind == "map":
            return flat[self.map_off[i]:self.map_off[i] + mw_size(L)].view(L, 2 * L - 1)
        if kind == "scal":
            k = bandlimit_scal(self.J_min, L, B, self.multires)
            return flat[self.scal_off[i]:self.scal_off[i] + mw_size(k)].view(k, 2 * k - 1)
        out, off = [], self.wav_off[i]
        for j in range(self.J_min, j_max(L, B) + 1):
            k = bandlimit_wav(j, L, B, self.multires)
            out.append(flat[off:off + mw_size(k)].view(k, 2 * k - 1))
            off += mw_size(k)
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.s2let_batch_destroy(self._h)
            self._h = None
        self._captured = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STAGES = {"phi_forward": 0, "theta": 1, "legendre_analysis": 2, "legendre_synthesis": 3,
          "phi_inverse": 4, "tiling": 5, "resample": 6}


def profile_enable(on: bool = True):
    """Start (clearing old records) or stop per-kernel event timing inside the library."""
    _check(_lib.s2let_profile_enable(int(on)), "s2let_profile_enable")


def profile_query(stage: str, k: int = 0) -> dict:
    """Summed kernel time and algorithmic work of one stage since profile_enable(True), over the
    launches at band-limit k (all launches for k <= 0)."""
    ms, fl, fr, by = (ctypes.c_double() for _ in range(4))
    n = ctypes.c_int64()
    _check(_lib.s2let_profile_query_k(STAGES[stage], int(k), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl),
                                      ctypes.byref(fr), ctypes.byref(by)), "s2let_profile_query_k")
    return {"ms": ms.value, "launches": n.value, "flops_full": fl.value, "flops_retained": fr.value,
            "bytes": by.value}


def sync(device=None):
    _check(_lib.s2let_sync(_stream(device)), "s2let_sync")
