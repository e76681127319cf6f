"""Serving (continuous batching) through the C ABI: every request's result is
the same served alone, served in a mix, and generated in one blocking call;
cancellation and error paths."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


def _same(a, b, tag):
    np.testing.assert_array_equal(a["sum_i"], b["sum_i"], err_msg=tag)
    np.testing.assert_array_equal(a["hash"], b["hash"], err_msg=tag)
    np.testing.assert_allclose(a["sum_d"], b["sum_d"], rtol=1e-12, atol=1e-15, err_msg=tag)
    # FP64 histogram sums may differ in summation order only
    np.testing.assert_allclose(a["hist"], b["hist"], rtol=1e-11, atol=1e-9, err_msg=tag)
    for k in ("n_done", "n_overflow", "n_nonfinite", "n_conservation", "n_cycle_limit", "total_cycles",
              "total_trials"):
        assert a[k] == b[k], (tag, k)


def test_served_alone_equals_generate(ctx):
    kw = dict(seed=1001, ecm=91.2, t_cut=1.0, max_partons=128)
    ref = ctx.generate(5000, summary=True, persistent=True, **kw)
    t = ctx.submit(5000, summary=True, **kw)
    got = ctx.wait(t)
    _same(got, ref, "alone")
    assert got["t_total_ms"] > 0


def test_served_tail_cut_equals_generate(ctx):
    # a request with a tail cut served beside uncut ones: each its own limit
    kw = dict(seed=1002, ecm=91.2, t_cut=1.0, max_partons=64)
    ref = ctx.generate(4000, summary=True, cycle_limit=25, **kw)
    assert ref["n_cycle_limit"] > 0
    full = ctx.submit(4000, summary=True, **kw)
    cut = ctx.submit(4000, summary=True, cycle_limit=25, **kw)
    _same(ctx.wait(cut), ref, "cut")
    assert ctx.wait(full)["n_cycle_limit"] == 0


def test_served_weighted_veto_equals_generate(ctx):
    kw = dict(seed=1003, ecm=200.0, t_cut=0.5, max_partons=128, t_over=20.0)
    ref = ctx.generate(3000, summary=True, **kw)
    plain = ctx.submit(3000, summary=True, **dict(kw, t_over=0.0))
    t = ctx.submit(3000, summary=True, **kw)
    _same(ctx.wait(t), ref, "weighted veto")
    assert (ref["sum_d"][0] < 0).any()
    assert ctx.wait(plain)["sum_d"][0].min() > 0


def test_mix_equals_alone(ctx):
    from paper_2403_08692_amd.workloads import serving_trace

    trace = serving_trace(40, min_log10_n=2.0, max_log10_n=4.3)
    alone = {}
    for r in trace.requests[:12]:
        t = ctx.submit(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap, summary=True)
        alone[r.index] = ctx.wait(t)
    tickets = [(r, ctx.submit(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap, summary=True))
               for r in trace.requests]
    for r, t in tickets:
        res = ctx.wait(t)
        if r.index in alone:
            _same(res, alone[r.index], f"request {r.index}")
        else:
            assert res["n_events"] == r.n_events and res["n_done"] + res["n_overflow"] == r.n_events
    # a served request equals the blocking plain form too
    r = trace.requests[3]
    ref = ctx.generate(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap, summary=True)
    _same(alone[3], ref, "plain")


def test_mix_with_per_event_energies(ctx):
    from paper_2403_08692_amd.workloads import mixed_energies

    e, tc = mixed_energies(5, 3000)
    ref = ctx.generate(3000, seed=5, max_partons=128, summary=True, ecm_per_event=e, tcut_per_event=tc)
    ts = [ctx.submit(3000, seed=5, max_partons=128, summary=True, ecm_per_event=e, tcut_per_event=tc)
          for _ in range(3)]
    others = [ctx.submit(2000, seed=77 + k, ecm=500.0, t_cut=0.5, max_partons=256) for k in range(3)]
    for t in ts:
        _same(ctx.wait(t), ref, "per-event energies")
    for t in others:
        assert ctx.wait(t)["n_events"] == 2000


def test_cancel_and_errors(ctx):
    import paper_2403_08692_amd as P

    big = ctx.submit(100_000, seed=9, ecm=500.0, t_cut=0.25, max_partons=256)
    ctx.cancel(big)
    try:
        ctx.wait(big)
        cancelled = False
    except P.VshError as e:
        assert e.code == -6
        cancelled = True
    # the request either was cancelled or had already finished; either way its ticket is gone
    with pytest.raises(P.VshError) as ei:
        ctx.poll(big)
    assert ei.value.code == -5
    with pytest.raises(P.VshError) as ei:
        ctx.wait(123456789)
    assert ei.value.code == -5
    with pytest.raises(P.VshError) as ei:
        ctx.submit(10, t_cut=0.001)
    assert ei.value.code == -1
    for bad in (-1.0, 0.005, float("nan"), float("inf")):  # t_over: 0 or a finite scale above 0.01
        with pytest.raises(P.VshError) as ei:
            ctx.submit(10, t_over=bad)
        assert ei.value.code == -1 and "t_over" in str(ei.value)
    # the service keeps working after a cancel
    t = ctx.submit(1000, seed=3)
    assert ctx.wait(t)["n_done"] == 1000
    print("cancelled:", cancelled)


def test_device_error_fails_only_its_request(ctx):
    # forced from the host: the next serving launch reports a HIP launch
    # failure instead of launching, so the GPU itself stays healthy
    import paper_2403_08692_amd as P

    ref = ctx.generate(2000, seed=41, summary=True)
    ctx.test_fail_epochs(1)
    t = ctx.submit(2000, seed=41, summary=True)
    with pytest.raises(P.VshError) as ei:
        ctx.wait(t)
    assert ei.value.code == -3 and "launch" in str(ei.value)
    # the loop goes on: the same request again gives the events generate gives
    t = ctx.submit(2000, seed=41, summary=True)
    got = ctx.wait(t)
    np.testing.assert_array_equal(got["sum_i"], ref["sum_i"])
    np.testing.assert_array_equal(got["hash"], ref["hash"])


def test_poll_reports_completion(ctx):
    import time

    t = ctx.submit(20_000, seed=11)
    t0 = time.time()
    while not ctx.poll(t):
        assert time.time() - t0 < 60
        time.sleep(0.001)
    assert ctx.wait(t)["n_done"] == 20_000


def test_served_in_mix_equal_the_oracle(ctx, oracle):
    """Requests served in a mix, each compared with the oracle directly:
    every per-event field (parity bar of tests/parity.py, histogram entry
    counts included) with summaries; without summaries (the drain that copies
    only the weight and the counted fields, as the benchmark's trace runs)
    the histogram, sum_w and the totals, against the same request with
    summaries and against the oracle."""
    from paper_2403_08692_amd.workloads import serving_trace
    from tests import parity

    trace = serving_trace(30, min_log10_n=2.0, max_log10_n=3.4, master_seed=77)
    picked = trace.requests[:8]
    filler = [ctx.submit(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap)
              for r in trace.requests[8:]]
    with_sum = {r.index: ctx.submit(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap,
                                    summary=True) for r in picked}
    without = {r.index: ctx.submit(r.n_events, seed=r.seed, ecm=r.ecm, t_cut=r.tcut, max_partons=r.cap,
                                   summary=False) for r in picked}
    for r in picked:
        print(f"case served request {r.index} n={r.n_events} ecm={r.ecm} tcut={r.tcut}", flush=True)
        a, b = ctx.wait(with_sum[r.index]), ctx.wait(without[r.index])
        o = oracle.generate(r.seed, 0, r.n_events, r.ecm, r.tcut, r.cap)
        rep, same = parity.compare(a, o, r.ecm, r.n_events, records=False)
        parity.assert_parity(rep)
        assert same.all(), rep
        oi, od = o["sum_i"], o["sum_d"]
        for res in (a, b):
            assert res["n_done"] == int((oi[:, 1] == 1).sum())
            assert res["n_overflow"] == int((oi[:, 1] == 2).sum())
            assert res["total_cycles"] == int(oi[:, 2].sum())
            assert res["total_emissions"] == int(oi[:, 3].sum())
            assert res["total_trials"] == int(oi[:, 5].sum())
            assert res["total_ends"] == int(oi[:, 6].sum())
            assert res["max_cycles"] == int(oi[:, 2].max())
            assert res["sum_w"] == pytest.approx(od[:, 0].sum(), rel=1e-12)
            assert res["sum_w2"] == pytest.approx((od[:, 0] ** 2).sum(), rel=1e-12)
        # without summaries: the same histogram (entry counts exactly) as with them
        np.testing.assert_array_equal(b["hist"][..., 2], a["hist"][..., 2])
        np.testing.assert_allclose(b["hist"], a["hist"], rtol=1e-11, atol=1e-9)
        assert "sum_d" not in b
    for t in filler:
        ctx.wait(t)


@pytest.mark.parametrize("ecm,tcut,cap,n", [(91.2, 1.0, 128, 20_000), (500.0, 0.25, 256, 4_000)])
def test_fixed_point_histograms_are_the_same_bits_everywhere(ctx, oracle, ecm, tcut, cap, n):
    """VSH_HIST_FIXEDPOINT: the histogram of a request is the same bits from
    vsh_generate in both forms, from vsh_generate_into in both forms, served
    alone and served in a mix; it equals the FP64 one to rounding (entry
    counts exactly), and passes the parity bar against the oracle."""
    import torch

    import paper_2403_08692_amd as P
    from paper_2403_08692_amd._native import make_request

    kw = dict(seed=555, ecm=ecm, t_cut=tcut, max_partons=cap)
    print(f"case fixed-point histograms ecm={ecm} n={n}", flush=True)
    ref = ctx.generate(n, summary=True, fixed_hist=True, **kw)
    hists = {"generate plain": ref["hist"],
             "generate persistent": ctx.generate(n, summary=False, persistent=True, fixed_hist=True, **kw)["hist"]}
    alone = ctx.wait(ctx.submit(n, fixed_hist=True, **kw))
    hists["served alone"] = alone["hist"]
    others = [ctx.submit(3000 + 500 * k, seed=900 + k, ecm=[10.0, 200.0, 500.0][k % 3], t_cut=0.5, max_partons=256)
              for k in range(6)]
    mixed = ctx.submit(n, fixed_hist=True, summary=True, **kw)
    more = [ctx.submit(2000, seed=950 + k, ecm=35.0, t_cut=1.0, max_partons=128) for k in range(6)]
    hists["served in a mix"] = ctx.wait(mixed)["hist"]
    for t in others + more:
        ctx.wait(t)
    dev = torch.device("cuda:0")
    for form in (P.VSH_FORM_PLAIN, P.VSH_FORM_PERSISTENT):
        req, keep = make_request(n, 555, 0, ecm, tcut, cap, form | P.VSH_HIST_FIXEDPOINT)
        ws_bytes = ctx.workspace_size(req)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        h = torch.zeros(P.HIST_DOUBLES, dtype=torch.float64, device=dev)
        ctx.generate_into(req, torch.cuda.current_stream(dev).cuda_stream, ws.data_ptr(), ws_bytes, h.data_ptr())
        torch.cuda.synchronize()
        hists[f"generate_into form {form}"] = h.cpu().numpy().reshape(P.NOBS, P.NHCOL, 3)
        del ws
    for name, h in hists.items():
        assert np.array_equal(h, ref["hist"]), name
    fp = ctx.generate(n, summary=False, **kw)["hist"]
    np.testing.assert_array_equal(fp[..., 2], ref["hist"][..., 2])
    np.testing.assert_allclose(fp, ref["hist"], rtol=1e-11, atol=1e-9)
    from tests import parity

    o = oracle.generate(555, 0, n, ecm, tcut, cap)
    rep, same = parity.compare(ref, o, ecm, n, records=False)
    parity.assert_parity(rep)
