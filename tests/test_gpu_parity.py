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


def test_overflow_small_cap(ctx, oracle):
    g, o, rep = _run(ctx, oracle, 800, 2, 91.2, 1.0, 4)
    assert rep["frac"] == 1.0
    assert g["n_overflow"] > 0
    assert g["n_overflow"] == int((o["sum_i"][:, 1] == 2).sum())
    assert g["n_done"] + g["n_overflow"] == 800


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
