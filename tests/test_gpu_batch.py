"""Uneven batches (s2let_batch_*): many maps with different band-limits L and wavelet parameters
B in one job, grouped by (L, B), run on worker streams, optionally autotuned and captured into a
HIP graph.

  - every map's outputs equal the single-map wavelet calls (within 1e-12) and, for sampled maps,
    the oracle (within 1e-10);
  - autotuning keeps the outputs correct;
  - graph replays (with other GPU work between them) reproduce the eager run bit for bit;
  - the uneven-batching workload: 256 real maps, L uniform in {64, 128, 256, 512}, B in {2, 3},
    J_min = 1, multiresolution, spectra C_l = (l+1)^-alpha with alpha uniform in [1, 3], seed 2:
    reconstruction of every map, oracle parity of one map per (L, B) group on every ring."""
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


def _rel(got, ref, floor=0.0):
    got, ref = np.asarray(got), np.asarray(ref)
    den = max(float(np.max(np.abs(ref))), floor)
    return float(np.max(np.abs(got - ref))) / den


def _maps(params, seed, on_gpu_for_large, dev, oracle_maps_upto=0, oracle_idx=()):
    """Seeded maps for (L, B, alpha) params; maps with L <= oracle_maps_upto or an index in
    oracle_idx are synthesised by the oracle (so they can be compared with it), the rest by the
    library's inverse transform."""
    flat, oracle_in = [], {}
    for i, (L, B, alpha) in enumerate(params):
        flm = si.random_flm(L, 1, reality=True, seed=seed + i, cl=si.spectrum_power(L, alpha))
        if L <= oracle_maps_upto or i in oracle_idx:
            f = oracle.inverse_sht(flm, L, reality=True)[0]
            oracle_in[i] = f
            flat.append(torch.from_numpy(f.reshape(-1)).to(dev))
        else:
            flat.append(s2.mw_inverse(torch.from_numpy(flm).to(dev), L, s2.REAL).reshape(-1))
    return torch.cat(flat), oracle_in


def test_small_uneven_batch_matches_single_calls(dev):
    rng = np.random.default_rng(5)
    params = [(int(rng.choice([8, 16, 32])), int(rng.choice([2, 3])), 2.0) for _ in range(24)]
    J_min = 1
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min)
    f, oin = _maps(params, 40, False, dev, oracle_maps_upto=32)
    f_wav, f_scal, rec = plan.run(f)
    torch.cuda.synchronize()
    for i, (L, B, _) in enumerate(params):
        fi = plan.map_view(f, i).unsqueeze(0).contiguous()
        w1, s1 = s2.analysis(fi, L, B, J_min, True, s2.REAL)
        r1 = s2.synthesis(w1, s1, L, B, J_min, True, s2.REAL)
        got_w = torch.cat([w.reshape(-1) for w in plan.map_view(f_wav, i, "wav")])
        assert _rel(got_w.cpu().numpy(), w1.reshape(-1).cpu().numpy()) < 1e-12
        assert _rel(plan.map_view(f_scal, i, "scal").cpu().numpy(), s1.reshape(plan.map_view(f_scal, i, "scal").shape).cpu().numpy(), 1e-6) < 1e-12
        assert _rel(plan.map_view(rec, i).cpu().numpy(), r1[0].cpu().numpy()) < 1e-12
        if i < 4:
            wav_ref, scal_ref = oracle.analysis(oin[i], L, B, J_min, True, True)
            for g, r in zip(plan.map_view(f_wav, i, "wav"), wav_ref):
                assert _rel(g.cpu().numpy(), r[0], 1e-6 * float(np.max(np.abs(oin[i])))) < 1e-10
            assert _rel(plan.map_view(rec, i).cpu().numpy(), oin[i]) < 1e-10
    plan.close()


def test_batch_with_band_limit_2048(dev):
    """A batch holding an L = 2048 map (its top scales run the band-limit 2048 stages, in the
    column-quad layout of the symmetric path) beside small ones: the L = 2048 map's outputs equal
    the single-call transforms of a stack of eight copies of it (16 columns, the same path), and
    every map is reconstructed."""
    params = [(2048, 2, 2.0), (64, 3, 2.0), (512, 2, 1.5)]
    J_min = 3
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min)
    f, _ = _maps(params, 120, False, dev)
    f_wav, f_scal, rec = plan.run(f)
    torch.cuda.synchronize()
    L, B, _ = params[0]
    f0 = plan.map_view(f, 0).unsqueeze(0).contiguous()
    w8, s8 = s2.analysis(f0.expand(8, -1, -1).contiguous(), L, B, J_min, True, s2.REAL)
    torch.cuda.synchronize()
    got_w = torch.cat([w.reshape(-1) for w in plan.map_view(f_wav, 0, "wav")])
    e_w = _rel(got_w.cpu().numpy(), w8[0].reshape(-1).cpu().numpy())
    sc = plan.map_view(f_scal, 0, "scal")
    e_s = _rel(sc.cpu().numpy(), s8[0].reshape(sc.shape).cpu().numpy(), 1e-6)
    _log("  L=2048 map against eight-map single calls: wavelets %.2e, scaling %.2e" % (e_w, e_s))
    assert e_w < 1e-12 and e_s < 1e-12
    for i, (Li, Bi, _) in enumerate(params):
        e = _rel(plan.map_view(rec, i).cpu().numpy(), plan.map_view(f, i).cpu().numpy())
        _log("  map %d (L=%d): reconstruction %.2e" % (i, Li, e))
        assert e < 1e-12
    plan.close()


def test_autotune_and_graph_replay(dev):
    rng = np.random.default_rng(6)
    params = [(int(rng.choice([16, 32, 64])), int(rng.choice([2, 3])), 1.5) for _ in range(20)]
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], 1)
    f, _ = _maps(params, 80, False, dev)
    out = plan.outputs()
    ref = [t.clone() for t in plan.run(f, out)]
    streams, cap, ms = plan.autotune(f, out)
    _log("  autotune: %d streams, %d maps per batch, %.3f ms" % (streams, cap, ms))
    torch.cuda.synchronize()
    for a, b in zip(out, ref):
        assert _rel(a.cpu().numpy(), b.cpu().numpy(), 1e-300) < 1e-12
    eager = [t.clone() for t in plan.run(f, out)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(f, out)
        for rep in range(3):
            for t in out:
                t.zero_()
            plan.replay()
            s.synchronize()
            for a, b in zip(out, eager):
                assert torch.equal(a, b), "graph replay %d differs from the eager run" % rep
            # other eager work between replays
            _ = s2.mw_forward(plan.map_view(f, 0).unsqueeze(0).contiguous(), params[0][0], s2.REAL)
            s.synchronize()
    plan.close()


def test_uneven_batching_workload(dev):
    """The workload itself: every map reconstructed, and the first map of every (L, B) group
    (L in {64, 128, 256, 512}, B in {2, 3}) against the oracle on every ring."""
    params = si.uniform_batch_params(seed=2, nmaps=256)
    J_min = 1
    firsts = {}
    for i, (L, B, _) in enumerate(params):
        firsts.setdefault((L, B), i)
    assert len(firsts) == 8
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min)
    _log("  oracle synthesis of one map per (L, B) group: %s" % sorted(firsts.items()))
    f, oin = _maps(params, 1000, True, dev, oracle_idx=set(firsts.values()))
    f_wav, f_scal, rec = plan.run(f)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (L, B, _) in enumerate(params):
        e = _rel(plan.map_view(rec, i).cpu().numpy(), plan.map_view(f, i).cpu().numpy())
        worst = max(worst, e)
        assert e < 1e-12, (i, L, B, e)
    _log("  worst relative reconstruction error: %.3e" % worst)
    for (L, B), i in sorted(firsts.items()):
        _log("  map %d (L=%d, B=%d): oracle analysis" % (i, L, B))
        wav_ref, scal_ref = oracle.analysis(oin[i], L, B, J_min, True, True)
        floor = 1e-6 * float(np.max(np.abs(oin[i])))
        got = plan.map_view(f_wav, i, "wav")
        assert len(got) == len(wav_ref)
        for g, r in zip(got, wav_ref):
            assert _rel(g.cpu().numpy(), r[0], floor) < 1e-10
        assert _rel(plan.map_view(f_scal, i, "scal").cpu().numpy(), scal_ref[0], floor) < 1e-10
        assert _rel(plan.map_view(rec, i).cpu().numpy(), oin[i]) < 1e-10
    plan.close()


# ------------------------------------------------------------------ persistent (level) execution
def _run_both(plan, f):
    """(streams outputs, persistent outputs) of one plan on the same input."""
    plan.set_execution(s2.BATCH_STREAMS)
    ref = [t.clone() for t in plan.run(f)]
    plan.set_execution(s2.BATCH_PERSISTENT)
    got = plan.run(f)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("shapes", [None, (1, 1, 1, 1, 2, 4), (1, 1, 2, 4, 4, 4)])
def test_persistent_matches_streams_and_oracle(dev, shapes):
    """Band-limits on the symmetric grid (64, 128, 256: persistent items) and off it (16, 48, 96;
    scales 2..32 and the B = 3 scales 9, 27, 81: per-transform kernels), real maps, in the
    persistent mode with the default and forced tile shapes: every output equals the streams mode
    (1e-12) and sampled maps the oracle (1e-10)."""
    rng = np.random.default_rng(7)
    params = [(int(rng.choice([16, 48, 64, 96, 128, 256])), int(rng.choice([2, 3])), 2.0) for _ in range(22)]
    params[0] = (64, 2, 2.0)
    params[1] = (128, 3, 2.0)
    J_min = 1
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min)
    f, oin = _maps(params, 300, False, dev, oracle_idx={0, 1, 2})
    if shapes is not None:
        plan.set_execution(s2.BATCH_PERSISTENT, shapes, [min(x, 4) for x in shapes])
        cfg = plan.execution()
        assert cfg["nw_analysis"] == list(shapes)
    ref, got = _run_both(plan, f)
    _log("  execution: %s" % plan.execution())
    for a, b in zip(got, ref):
        assert _rel(a.cpu().numpy(), b.cpu().numpy(), 1e-300) < 1e-12
    for i in (0, 1, 2):
        L, B, _ = params[i]
        wav_ref, scal_ref = oracle.analysis(oin[i], L, B, J_min, True, True)
        floor = 1e-6 * float(np.max(np.abs(oin[i])))
        for g, r in zip(plan.map_view(got[0], i, "wav"), wav_ref):
            assert _rel(g.cpu().numpy(), r[0], floor) < 1e-10
        assert _rel(plan.map_view(got[1], i, "scal").cpu().numpy(), scal_ref[0], floor) < 1e-10
        assert _rel(plan.map_view(got[2], i).cpu().numpy(), oin[i]) < 1e-10
    plan.close()


def test_persistent_complex_maps(dev):
    params = [(64, 2), (128, 2), (33, 3), (64, 3), (128, 2)]
    J_min = 1
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min, reality=s2.COMPLEX)
    flat, oin = [], {}
    for i, (L, B) in enumerate(params):
        flm = si.random_flm(L, 1, reality=False, seed=500 + i)
        fi = oracle.inverse_sht(flm, L, reality=False)[0]
        oin[i] = fi
        flat.append(torch.from_numpy(fi.reshape(-1)).to(dev))
    f = torch.cat(flat)
    ref, got = _run_both(plan, f)
    for a, b in zip(got, ref):
        assert _rel(a.cpu().numpy(), b.cpu().numpy(), 1e-300) < 1e-12
    L, B = params[1]
    wav_ref, _ = oracle.analysis(oin[1], L, B, J_min, True, False)
    for g, r in zip(plan.map_view(got[0], 1, "wav"), wav_ref):
        assert _rel(g.cpu().numpy(), r[0]) < 1e-10
    plan.close()


def test_persistent_graph_replay_and_errors(dev):
    rng = np.random.default_rng(8)
    params = [(int(rng.choice([32, 64, 128])), int(rng.choice([2, 3])), 1.5) for _ in range(12)]
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], 1)
    f, _ = _maps(params, 90, False, dev)
    # invalid tile shapes: 4 waves at band-limit 64 (k/2 = 32 nodes), 3 waves anywhere
    with pytest.raises(s2.S2letError):
        plan.set_execution(s2.BATCH_PERSISTENT, [4, 1, 1, 1, 1, 1], None)
    with pytest.raises(s2.S2letError):
        plan.set_execution(s2.BATCH_PERSISTENT, None, [1, 1, 3, 1, 1, 1])
    plan.set_execution(s2.BATCH_PERSISTENT)
    out = plan.outputs()
    eager = [t.clone() for t in plan.run(f, out)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.capture(f, out)
        for rep in range(3):
            for t in out:
                t.zero_()
            plan.replay()
            s.synchronize()
            for a, b in zip(out, eager):
                assert torch.equal(a, b), "graph replay %d differs from the eager run" % rep
            _ = s2.mw_forward(plan.map_view(f, 0).unsqueeze(0).contiguous(), params[0][0], s2.REAL)
            s.synchronize()
    plan.close()
    # the persistent mode is FP64 only
    mixed = s2.BatchPlan([64, 64], [2, 2], 1, precision=s2.MIXED_FP32)
    with pytest.raises(s2.S2letError):
        mixed.set_execution(s2.BATCH_PERSISTENT)
    mixed.close()


def test_uneven_batching_workload_persistent(dev):
    """The uneven-batching workload in the persistent mode (autotuned tile shapes): every map
    reconstructed; one map per (L, B) group against the oracle on every ring."""
    params = si.uniform_batch_params(seed=2, nmaps=256)
    J_min = 1
    firsts = {}
    for i, (L, B, _) in enumerate(params):
        firsts.setdefault((L, B), i)
    plan = s2.BatchPlan([p[0] for p in params], [p[1] for p in params], J_min)
    f, oin = _maps(params, 1000, True, dev, oracle_idx=set(firsts.values()))
    out = plan.outputs()
    plan.autotune(f, out)
    plan.set_execution(s2.BATCH_PERSISTENT)   # keeps the tuned shapes
    _log("  execution: %s" % plan.execution())
    f_wav, f_scal, rec = plan.run(f, out)
    torch.cuda.synchronize()
    for i, (L, B, _) in enumerate(params):
        e = _rel(plan.map_view(rec, i).cpu().numpy(), plan.map_view(f, i).cpu().numpy())
        assert e < 1e-12, (i, L, B, e)
    for (L, B), i in sorted(firsts.items()):
        _log("  map %d (L=%d, B=%d): oracle analysis" % (i, L, B))
        wav_ref, scal_ref = oracle.analysis(oin[i], L, B, J_min, True, True)
        floor = 1e-6 * float(np.max(np.abs(oin[i])))
        for g, r in zip(plan.map_view(f_wav, i, "wav"), wav_ref):
            assert _rel(g.cpu().numpy(), r[0], floor) < 1e-10
        assert _rel(plan.map_view(f_scal, i, "scal").cpu().numpy(), scal_ref[0], floor) < 1e-10
        assert _rel(plan.map_view(rec, i).cpu().numpy(), oin[i]) < 1e-10
    plan.close()
