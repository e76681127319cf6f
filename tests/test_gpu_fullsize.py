"""Parity at the full sizes the benchmark runs: the batching workload (10^7
events of mixed sqrt(s) and t_C, cap 128, batched form), the stress
workload (10^6 events at 500 GeV, t_C = 0.25, cap 256, both forms) and the
LEP workload with the extensions it times (quark masses; the weighted veto
with a cycle limit).  The GPU shows every event; the oracle recomputes a
seeded sample of event ids one by one."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


def _sampled(g, oracle, seed, ids, ecm, tcut, cap, w_rtol=1e-12, **okw):
    bad = 0
    for e in ids:
        o = oracle.generate(seed, int(e), 1, float(ecm[e]), float(tcut[e]), cap, **okw)
        same = all(g["sum_i"][f, e] == o["sum_i"][0, f] for f in range(7)) and g["hash"][e] == o["hash"][0]
        if same:
            np.testing.assert_allclose(g["sum_d"][2:9, e], o["sum_d"][0, 2:9], rtol=1e-9, atol=1e-12)
            assert g["sum_d"][0, e] == pytest.approx(o["sum_d"][0, 0], rel=w_rtol)
        bad += not same
    return bad


def test_batching_workload_1e7_sampled(ctx, oracle):
    from paper_2403_08692_amd import workloads

    w = workloads.MIXED
    e, t = w.per_event()
    print(f"case {w.name} persistent", flush=True)
    g = ctx.generate(w.n_events, seed=w.seed, max_partons=w.cap, summary=True, persistent=True,
                     ecm_per_event=e, tcut_per_event=t)
    assert g["n_done"] + g["n_overflow"] == w.n_events and g["n_conservation"] == 0 and g["n_nonfinite"] == 0
    ids = np.sort(np.random.default_rng(1).choice(w.n_events, 1500, replace=False))
    assert _sampled(g, oracle, w.seed, ids, e, t, w.cap) <= 2


@pytest.mark.parametrize("persistent", [False, True])
def test_stress_workload_1e6_sampled(ctx, oracle, persistent):
    from paper_2403_08692_amd import workloads

    w = workloads.STRESS
    print(f"case {w.name} persistent={persistent}", flush=True)
    g = ctx.generate(w.n_events, seed=w.seed, ecm=w.ecm, t_cut=w.tcut, max_partons=w.cap, summary=True,
                     persistent=persistent)
    assert g["n_done"] + g["n_overflow"] == w.n_events and g["n_conservation"] == 0
    ids = np.sort(np.random.default_rng(2).choice(w.n_events, 400, replace=False))
    n = w.n_events
    assert _sampled(g, oracle, w.seed, ids, np.full(n, w.ecm), np.full(n, w.tcut), w.cap) <= 1


@pytest.mark.parametrize("persistent", [False, True])
def test_lep_extensions_1e6_sampled(ctx, oracle, persistent):
    from tests import parity

    n = 1_000_000
    ecm, tcut = np.full(n, 91.2), np.full(n, 1.0)
    cases = (("masses", dict(mass_c=1.5, mass_b=4.8), dict(mass=[0.0, 0.0, 0.0, 0.0, 1.5, 4.8]), 1e-12),
             ("weighted veto, cycle limit", dict(t_over=10.0, cycle_limit=43), dict(t_over=10.0, max_cycles=43),
              parity.W_RTOL))
    for k, (name, kw, okw, w_rtol) in enumerate(cases):
        print(f"case lep 1e6 {name} persistent={persistent}", flush=True)
        g = ctx.generate(n, seed=1, ecm=91.2, t_cut=1.0, max_partons=64, summary=True, persistent=persistent, **kw)
        assert g["n_conservation"] == 0 and g["n_nonfinite"] == 0
        ids = np.sort(np.random.default_rng(3 + k).choice(n, 300, replace=False))
        assert _sampled(g, oracle, 1, ids, ecm, tcut, 64, w_rtol=w_rtol, **okw) <= 1
