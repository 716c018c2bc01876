"""The allocation-free wavelet analysis (s2let_axisym_analysis_noalloc, static device scratch)
against the allocating entry point s2let_axisym_analysis, through the C ABI: two calls in a row,
the second on a smaller input, real and complex maps; plus its two refusals (plans not built,
input too large for the scratch)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import s2let_inputs as si

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
s2 = pytest.importorskip("paper_1211_1680_amd")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _maps(L, nmaps, real, seed, dev):
    flm = si.random_flm(L, nmaps, reality=real, seed=seed)
    return torch.from_numpy(oracle.inverse_sht(flm, L, reality=real)).to(dev)


def _outputs(L, B, J_min, mr, reality, nmaps, dev):
    dt = torch.float64 if reality == s2.REAL else torch.complex128
    kP = s2.bandlimit_scal(J_min, L, B, mr)
    # filled with NaN so that any sample the call fails to write shows up
    return (torch.full((nmaps, s2.wav_size(L, B, J_min, mr)), float("nan"), dtype=dt, device=dev),
            torch.full((nmaps, s2.mw_size(kP)), float("nan"), dtype=dt, device=dev))


# (L, B, J_min, multires, nmaps): the second case of each pair is smaller than the first
CASES = {
    s2.REAL: [(128, 2, 2, True, 16), (64, 3, 1, False, 5)],
    s2.COMPLEX: [(96, 2, 1, True, 8), (33, 2, 0, True, 3)],
}


@pytest.mark.parametrize("reality", [s2.REAL, s2.COMPLEX])
def test_noalloc_matches_allocating_entry_point(dev, reality):
    real = reality == s2.REAL
    for i, (L, B, J_min, mr, nmaps) in enumerate(CASES[reality]):
        _log("noalloc analysis: reality", reality, "call", i, "L", L, "B", B, "J_min", J_min, "multires", mr,
             "nmaps", nmaps)
        assert s2.workspace_size(L, B, J_min, mr, reality, s2.FP64, nmaps, True) <= s2.NOALLOC_SCRATCH_BYTES
        f = _maps(L, nmaps, real, 300 + 10 * i + reality, dev)
        # the allocating call (also builds the plan tables on this device)
        ref_wav, ref_scal = s2.analysis(f, L, B, J_min, mr, reality)
        got = _outputs(L, B, J_min, mr, reality, nmaps, dev)
        s2.analysis_noalloc(f, L, B, J_min, mr, reality, s2.FP64, got)
        torch.cuda.synchronize()
        for g, r in zip(got, (ref_wav, ref_scal)):
            assert not torch.isnan(g).any()
            den = r.abs().max().item()
            rel = (g - r).abs().max().item() / (den if den > 0 else 1.0)
            _log("  rel err against s2let_axisym_analysis %.3e, identical: %s" % (rel, bool(torch.equal(g, r))))
            assert rel <= 1e-10
            # same kernels, same order of operations: the results are bit for bit the same
            assert torch.equal(g, r)


def test_noalloc_refusals(dev):
    # plan tables never built for (L, B, J_min) = (97, 5, 1) in this process: nothing runs
    L, B, J_min = 97, 5, 1
    f = _maps(L, 1, True, 7, dev)
    out = _outputs(L, B, J_min, True, s2.REAL, 1, dev)
    st = s2.lib.s2let_axisym_analysis_noalloc(out[0].data_ptr(), out[1].data_ptr(), f.data_ptr(), L, B, J_min, 1,
                                              s2.REAL, s2.FP64, 1, ctypes.c_void_p(0))
    assert st == s2.ENOTREADY
    torch.cuda.synchronize()
    assert torch.isnan(out[0]).all() and torch.isnan(out[1]).all()
    assert b"not built" in s2.lib.s2let_strerror(st)
    # 16 real maps at L = 512 need more than the static scratch: refused before any launch
    assert s2.workspace_size(512, 2, 2, True, s2.REAL, s2.FP64, 16, True) > s2.NOALLOC_SCRATCH_BYTES
    st = s2.lib.s2let_axisym_analysis_noalloc(out[0].data_ptr(), out[1].data_ptr(), f.data_ptr(), 512, 2, 2, 1,
                                              s2.REAL, s2.FP64, 16, ctypes.c_void_p(0))
    assert st == s2.ESCRATCH
    assert torch.isnan(out[0]).all()
