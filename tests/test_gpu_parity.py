"""GPU parity: the HIP path through the C ABI against the oracle on the same
seeded events (bars in tests/parity.py)."""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


def _run(ctx, oracle, n, seed, ecm, tcut, cap, first=0, persistent=False, ecm_arr=None, tcut_arr=None):
    print(f"case n={n} seed={seed} ecm={ecm} tcut={tcut} cap={cap} first={first} persistent={persistent}", flush=True)
    g = ctx.generate(n, seed=seed, first_event=first, ecm=ecm, t_cut=tcut, max_partons=cap, summary=True,
                     records=True, persistent=persistent, ecm_per_event=ecm_arr, tcut_per_event=tcut_arr)
    o = oracle.generate(seed, first, n, ecm, tcut, cap, records=True, ecm_arr=ecm_arr, tcut_arr=tcut_arr)
    rep, same = parity.compare(g, o, ecm if ecm_arr is None else ecm_arr, n)
    print(rep, flush=True)
    return g, o, rep


def test_lep_small_plain(ctx, oracle):
    g, o, rep = _run(ctx, oracle, 1000, 1, 91.2, 1.0, 64)
    parity.assert_parity(rep)
    assert rep["frac"] == 1.0
    assert g["n_done"] == 1000


def test_ragged_sizes_and_offsets(ctx, oracle):
    # sizes that are not multiples of the wave or block, and a non-zero first id
    for n, first in ((1, 0), (63, 5), (257, 1 << 33), (1111, 77)):
        g, o, rep = _run(ctx, oracle, n, 3, 91.2, 1.0, 64, first=first)
        parity.assert_parity(rep)


@pytest.mark.parametrize("ecm,tcut,cap", [(10.0, 1.0, 64), (500.0, 0.25, 256), (200.0, 0.5, 128)])
def test_energies_and_caps(ctx, oracle, ecm, tcut, cap):
    g, o, rep = _run(ctx, oracle, 600, 9, ecm, tcut, cap)
    parity.assert_parity(rep)


@pytest.mark.parametrize("persistent", [False, True])
def test_large_events_both_observable_passes(ctx, oracle, persistent):
    # 500 GeV with t_C = 0.03: sizes from about 10 to 80 partons, so both
    # lane-group widths of the observables (16 lanes up to 31 partons, a
    # wave from 32) and their split of the sorted events are exercised
    g, o, rep = _run(ctx, oracle, 500, 5, 500.0, 0.03, 256, persistent=persistent)
    parity.assert_parity(rep)
    n = o["sum_i"][:, 0]
    assert (n < 32).any() and (n >= 32).any()


def test_overflow_wave_pass(ctx, oracle):
    # cap 40: overflowing events stop at 40 partons, on the 64-lane groups
    g, o, rep = _run(ctx, oracle, 300, 6, 500.0, 0.03, 40)
    parity.assert_parity(rep)
    assert g["n_overflow"] > 0


def test_overflow_small_cap(ctx, oracle):
    g, o, rep = _run(ctx, oracle, 800, 2, 91.2, 1.0, 4)
    assert rep["frac"] == 1.0
    assert g["n_overflow"] > 0
    assert g["n_overflow"] == int((o["sum_i"][:, 1] == 2).sum())
    assert g["n_done"] + g["n_overflow"] == 800


@pytest.mark.parametrize("persistent", [False, True])
def test_limits_and_degenerate_requests(ctx, oracle, persistent):
    import paper_2403_08692_amd as P

    # empty requests and record capacities outside 2..1024 are refused before any launch
    for n, cap in ((0, 64), (10, 1), (10, 1025)):
        print(f"case refused n={n} cap={cap} persistent={persistent}", flush=True)
        with pytest.raises(P.VshError) as ei:
            ctx.generate(n, seed=1, max_partons=cap, persistent=persistent)
        assert ei.value.code == -1
    # no phase space above the cutoff (4 t_C > s): every event ends on its
    # first cycle with its two partons, thrust exactly 1
    g, o, rep = _run(ctx, oracle, 300, 4, 10.0, 30.0, 64, persistent=persistent)
    parity.assert_parity(rep)
    assert rep["frac"] == 1.0 and (g["sum_i"][0] == 2).all() and (g["sum_i"][2] == 1).all()
    assert (g["sum_d"][4] <= 1e-15).all()  # tau = 1 - T
    # the largest record capacity, on a ragged batch
    g, o, rep = _run(ctx, oracle, 70, 8, 500.0, 0.25, 1024, persistent=persistent)
    parity.assert_parity(rep)


@pytest.mark.parametrize("form,mapping", [("plain", 1), ("plain", 0), ("persistent", 1), ("persistent", 0)])
def test_tail_cut(ctx, oracle, form, mapping):
    # events still above the cutoff after 30 veto cycles are vetoed (status 5,
    # no observables, not histogrammed); the others are those of the uncut run
    n, C = 3000, 30
    persistent = form == "persistent"
    key = "mapping" if persistent else "plain_mapping"
    before = ctx.get_tuning()[key]
    ctx.set_tuning(**{key: mapping})
    try:
        print(f"case tail cut n={n} C={C} form={form} mapping={mapping}", flush=True)
        g = ctx.generate(n, seed=4, ecm=91.2, t_cut=1.0, max_partons=64, summary=True, records=True,
                         persistent=persistent, cycle_limit=C)
    finally:
        ctx.set_tuning(**{key: before})
    o = oracle.generate(4, 0, n, 91.2, 1.0, 64, records=True, max_cycles=C)
    rep, same = parity.compare(g, o, 91.2, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
    cut = o["sum_i"][:, 1] == 5
    assert 0.05 < cut.mean() < 0.6
    assert g["n_cycle_limit"] == int(cut.sum()) and g["n_done"] == n - int(cut.sum())
    assert (g["sum_i"][2][cut] == C).all()
    assert g["hist"][7, :, 2].sum() == n - cut.sum()


@pytest.mark.parametrize("form,mapping", [("plain", 1), ("plain", 0), ("persistent", 1), ("persistent", 0)])
def test_weighted_veto(ctx, oracle, form, mapping):
    # alpha_s(10 GeV^2) in the trial density: fewer trials, and event weights
    # +-(2r - 1) where the true density exceeds the trial density
    n, t_over = 3000, 10.0
    persistent = form == "persistent"
    key = "mapping" if persistent else "plain_mapping"
    before = ctx.get_tuning()[key]
    ctx.set_tuning(**{key: mapping})
    try:
        print(f"case weighted veto n={n} t_over={t_over} form={form} mapping={mapping}", flush=True)
        g = ctx.generate(n, seed=6, ecm=91.2, t_cut=1.0, max_partons=64, summary=True, records=True,
                         persistent=persistent, t_over=t_over)
    finally:
        ctx.set_tuning(**{key: before})
    o = oracle.generate(6, 0, n, 91.2, 1.0, 64, records=True, t_over=t_over)
    rep, same = parity.compare(g, o, 91.2, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
    w = o["sum_d"][:, 0]
    me = np.array([oracle.me_event(6, e, 91.2)[3] for e in range(n)])
    assert (w < 0).any() and (np.abs(w / me - 1) > 1e-12).mean() > 0.1  # the weights are in play
    assert g["sum_w"] == pytest.approx(w.sum(), rel=1e-9)


def test_mixed_energies_per_event(ctx, oracle):
    from paper_2403_08692_amd.workloads import mixed_energies

    e, t = mixed_energies(1, 2000)
    g, o, rep = _run(ctx, oracle, 2000, 1, 91.2, 1.0, 128, ecm_arr=e, tcut_arr=t)
    parity.assert_parity(rep)


def test_lep_slice_of_1e6_sampled(ctx, oracle):
    # the full 10^6-event workload on the GPU; the oracle recomputes a sample
    # of event ids one by one and the histograms are checked statistically
    n = 1_000_000
    g = ctx.generate(n, seed=1, ecm=91.2, t_cut=1.0, max_partons=64, summary=True)
    assert g["n_done"] == n and g["n_conservation"] == 0 and g["n_nonfinite"] == 0
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(n, 2000, replace=False))
    bad = 0
    for e in ids:
        o = oracle.generate(1, int(e), 1, 91.2, 1.0, 64)
        same = all(g["sum_i"][f, e] == o["sum_i"][0, f] for f in range(7)) and g["hash"][e] == o["hash"][0]
        if same:
            np.testing.assert_allclose(g["sum_d"][2:9, e], o["sum_d"][0, 2:9], rtol=1e-9, atol=1e-12)
        bad += not same
    assert bad <= 2
    # sigma estimate against the closed form
    sig = oracle.sigma_lo(91.2 ** 2)
    w = g["sum_d"][0]
    assert abs(w.mean() - sig) < 4 * w.std() / np.sqrt(n)


# ---------------------------------------------------------------------------
# persistent (batched) form
# ---------------------------------------------------------------------------
def test_persistent_lep_small(ctx, oracle):
    g, o, rep = _run(ctx, oracle, 1000, 1, 91.2, 1.0, 64, persistent=True)
    parity.assert_parity(rep)
    assert rep["frac"] == 1.0


@pytest.mark.parametrize("n", [1, 63, 65, 4097])
def test_persistent_ragged(ctx, oracle, n):
    g, o, rep = _run(ctx, oracle, n, 5, 91.2, 1.0, 64, first=11, persistent=True)
    parity.assert_parity(rep)


def test_persistent_mixed_and_stress(ctx, oracle):
    from paper_2403_08692_amd.workloads import mixed_energies

    e, t = mixed_energies(1, 3000)
    g, o, rep = _run(ctx, oracle, 3000, 1, 91.2, 1.0, 128, ecm_arr=e, tcut_arr=t, persistent=True)
    parity.assert_parity(rep)
    g, o, rep = _run(ctx, oracle, 500, 4, 500.0, 0.25, 256, persistent=True)
    parity.assert_parity(rep)


def test_persistent_equals_plain(ctx):
    from paper_2403_08692_amd.workloads import mixed_energies

    n = 200_000
    e, t = mixed_energies(7, n)
    a = ctx.generate(n, seed=7, max_partons=128, summary=True, ecm_per_event=e, tcut_per_event=t)
    b = ctx.generate(n, seed=7, max_partons=128, summary=True, ecm_per_event=e, tcut_per_event=t, persistent=True)
    np.testing.assert_array_equal(a["sum_i"], b["sum_i"])
    np.testing.assert_array_equal(a["hash"], b["hash"])
    np.testing.assert_allclose(a["sum_d"], b["sum_d"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(a["hist"], b["hist"], rtol=1e-11, atol=1e-9)
    print("plain shower ms", a["t_shower_ms"], "persistent", b["t_shower_ms"], flush=True)


def test_persistent_graph_replays_match_eager(ctx):
    """vsh_generate_into (persistent form, replayed hipGraph) on PyTorch
    buffers, several replays with host work between them, each checked
    against the eager vsh_generate result."""
    import torch

    import paper_2403_08692_amd as P
    from paper_2403_08692_amd._native import make_request

    n = 50_000
    ref = ctx.generate(n, seed=3, ecm=200.0, t_cut=0.5, max_partons=128, summary=True, persistent=True)
    req, keep = make_request(n, 3, 0, 200.0, 0.5, 128, P.VSH_FORM_PERSISTENT)
    ws_bytes = ctx.workspace_size(req)
    dev = torch.device("cuda:0")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    hist = torch.zeros(P.HIST_DOUBLES, dtype=torch.float64, device=dev)
    sd = torch.empty((P.NSUM_D, n), dtype=torch.float64, device=dev)
    si = torch.empty((P.NSUM_I, n), dtype=torch.int32, device=dev)
    hs = torch.empty(n, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    for rep in range(4):
        hist.zero_()
        si.fill_(-1)
        ctx.generate_into(req, stream.cuda_stream, ws.data_ptr(), ws_bytes, hist.data_ptr(), sd.data_ptr(),
                          si.data_ptr(), hs.data_ptr())
        torch.cuda.synchronize()
        np.testing.assert_array_equal(si.cpu().numpy(), ref["sum_i"])
        np.testing.assert_array_equal(hs.cpu().numpy().view(np.uint64), ref["hash"])
        np.testing.assert_allclose(sd.cpu().numpy(), ref["sum_d"], rtol=1e-13, atol=0)
        np.testing.assert_allclose(hist.cpu().numpy().reshape(P.NOBS, P.NHCOL, 3), ref["hist"], rtol=1e-11,
                                   atol=1e-9)
        _ = ctx.generate(100, seed=rep, summary=False)  # unrelated eager work between replays


def test_plain_generate_into_matches_generate(ctx):
    import torch

    import paper_2403_08692_amd as P
    from paper_2403_08692_amd._native import make_request

    n = 20_000
    ref = ctx.generate(n, seed=2, summary=True)
    req, keep = make_request(n, 2, 0, 91.2, 1.0, 64, P.VSH_FORM_PLAIN)
    ws_bytes = ctx.workspace_size(req)
    dev = torch.device("cuda:0")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    hist = torch.zeros(P.HIST_DOUBLES, dtype=torch.float64, device=dev)
    si = torch.empty((P.NSUM_I, n), dtype=torch.int32, device=dev)
    ctx.timing_start()
    for _ in range(2):
        hist.zero_()
        ctx.generate_into(req, torch.cuda.current_stream(dev).cuda_stream, ws.data_ptr(), ws_bytes,
                          hist.data_ptr(), None, si.data_ptr(), None)
    torch.cuda.synchronize()
    t = ctx.timing_read()
    assert t.shape == (2, 3) and (t > 0).all()
    np.testing.assert_array_equal(si.cpu().numpy(), ref["sum_i"])
    np.testing.assert_allclose(hist.cpu().numpy().reshape(P.NOBS, P.NHCOL, 3), ref["hist"], rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("tuning", [
    dict(mapping=1, waves_per_cu=8, refill_threshold=1, refill_period=1),
    dict(mapping=1, waves_per_cu=4, refill_threshold=16, refill_period=4),
    dict(mapping=0, waves_per_cu=8, block=256, refill_threshold=1, refill_period=1),
    dict(mapping=0, waves_per_cu=16, block=64, refill_threshold=32, refill_period=3),
])
def test_persistent_settings_do_not_change_events(ctx, oracle, tuning):
    old = ctx.get_tuning()
    try:
        ctx.set_tuning(**tuning)
        g, o, rep = _run(ctx, oracle, 2500, 12, 200.0, 0.5, 128, persistent=True)
        parity.assert_parity(rep)
        assert rep["frac"] == 1.0
    finally:
        ctx.set_tuning(**old)


def test_autotune_keeps_events(ctx):
    from paper_2403_08692_amd.workloads import mixed_energies

    e, t = mixed_energies(3, 100_000)
    before = ctx.generate(100_000, seed=3, max_partons=128, ecm_per_event=e, tcut_per_event=t, persistent=True)
    chosen = ctx.autotune(100_000, seed=3, max_partons=128, ecm_per_event=e, tcut_per_event=t)
    print("autotune chose", chosen, flush=True)
    after = ctx.generate(100_000, seed=3, max_partons=128, ecm_per_event=e, tcut_per_event=t, persistent=True)
    np.testing.assert_array_equal(before["sum_i"], after["sum_i"])
    np.testing.assert_array_equal(before["hash"], after["hash"])
    plain = ctx.autotune(100_000, seed=3, max_partons=128, ecm_per_event=e, tcut_per_event=t, persistent=False)
    assert plain["plain_block"] in (64, 128, 256)


@pytest.mark.parametrize("tuning", [
    dict(plain_mapping=1),
    dict(plain_mapping=0, plain_block=256, plain_waves=2),
    dict(plain_mapping=0, plain_block=64, plain_waves=4),
])
def test_plain_settings_do_not_change_events(ctx, oracle, tuning):
    old = ctx.get_tuning()
    try:
        ctx.set_tuning(**tuning)
        g, o, rep = _run(ctx, oracle, 1500, 21, 200.0, 0.5, 128)
        parity.assert_parity(rep)
        assert rep["frac"] == 1.0
        g, o, rep = _run(ctx, oracle, 300, 22, 500.0, 0.25, 256)
        parity.assert_parity(rep)
    finally:
        ctx.set_tuning(**old)


@pytest.mark.parametrize("persistent", [True, False])
def test_tuner_cache_is_reused_across_contexts(tmp_path, persistent):
    """A context given a tuner cache file records its tuning there; a second
    context (as another process would) takes the same settings from the file
    without timing anything, and a different sample is tuned afresh."""
    import time

    import paper_2403_08692_amd as P

    path = str(tmp_path / "tuning.txt")
    kw = dict(n_events=1 << 16, seed=4, ecm=91.2, t_cut=1.0, max_partons=64, persistent=persistent)
    with P.Context(tuner_cache_path=path) as c1:
        t0 = time.perf_counter()
        a = c1.autotune(**kw)
        t_tune = time.perf_counter() - t0
    assert a["from_cache"] == 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and ("persistent" if persistent else "plain") in lines[0]
    with P.Context(tuner_cache_path=path) as c2:
        t0 = time.perf_counter()
        b = c2.autotune(**kw)
        t_hit = time.perf_counter() - t0
        assert b["from_cache"] == 1
        keys = ("mapping", "waves_per_cu", "refill_threshold", "refill_period") if persistent else \
            ("plain_block", "plain_waves", "plain_mapping")
        assert all(a[k] == b[k] for k in keys), (a, b)
        assert c2.get_tuning()[keys[0]] == a[keys[0]]
        c = c2.autotune(**dict(kw, ecm=200.0))
        assert c["from_cache"] == 0
    assert len(open(path).read().splitlines()) == 2
    print(f"tuning {t_tune:.2f} s, from the cache {t_hit * 1e3:.2f} ms", flush=True)
    assert t_hit < 0.1 * t_tune


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("ecm,tcut,cap,limit,t_over", [(91.2, 1.0, 64, 0, 0.0), (91.2, 1.0, 64, 25, 10.0),
                                                        (500.0, 0.25, 12, 0, 0.0), (500.0, 0.25, 256, 90, 20.0)])
def test_cycles_ahead_sparse_waves(ctx, oracle, persistent, ecm, tcut, cap, limit, t_over):
    # waves of a few events evaluate up to eight veto cycles per pass: the
    # events, counts, cycle limits, overflows and weights stay the oracle's
    for n, first in ((3, 0), (9, 1000), (40, 77)):
        print(f"case cycles ahead n={n} first={first} ecm={ecm} tcut={tcut} cap={cap} limit={limit} "
              f"t_over={t_over} persistent={persistent}", flush=True)
        g = ctx.generate(n, seed=12, first_event=first, ecm=ecm, t_cut=tcut, max_partons=cap, summary=True,
                         records=True, persistent=persistent, cycle_limit=limit, t_over=t_over)
        o = oracle.generate(12, first, n, ecm, tcut, cap, records=True, max_cycles=limit, t_over=t_over)
        rep, same = parity.compare(g, o, ecm, n)
        print(rep, flush=True)
        parity.assert_parity(rep)
        assert rep["frac"] == 1.0  # cycles, trials, ends, statuses and emission hashes all equal


@pytest.mark.parametrize("persistent", [False, True])
def test_cycles_ahead_same_bits_as_full_waves(ctx, persistent):
    # the first events of a full batch (waves of 64 busy events: mostly one
    # cycle per pass) against the same events alone (a few events per wave:
    # several cycles per pass): identical summaries and weights, bit for bit
    kw = dict(seed=31, ecm=200.0, t_cut=0.5, max_partons=128, summary=True, persistent=persistent, t_over=20.0)
    full = ctx.generate(6400, **kw)
    for n in (2, 5, 33):
        alone = ctx.generate(n, **kw)
        np.testing.assert_array_equal(alone["sum_i"], full["sum_i"][:, :n])
        np.testing.assert_array_equal(alone["hash"], full["hash"][:n])
        np.testing.assert_array_equal(alone["sum_d"], full["sum_d"][:, :n])


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("cap", [64, 65, 128, 129])
def test_layout_boundaries(ctx, oracle, persistent, cap):
    # record capacities on either side of the kernels' layout choices (the
    # per-event layout with quark masses up to 64 partons, the four-wave
    # builds up to 128): the same events in every build
    n = 400
    print(f"case layout boundary cap={cap} persistent={persistent}", flush=True)
    g = ctx.generate(n, seed=17, ecm=200.0, t_cut=0.5, max_partons=cap, summary=True, records=True,
                     persistent=persistent, t_over=20.0, cycle_limit=60)
    o = oracle.generate(17, 0, n, 200.0, 0.5, cap, records=True, t_over=20.0, max_cycles=60)
    rep, same = parity.compare(g, o, 200.0, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
    assert rep["frac"] == 1.0
