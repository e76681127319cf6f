"""GPU parity of the initial-state shower (vsh_generate_isr: Drell-Yan
q qbar -> V with backward evolution and the stand-in parton density),
event by event against the oracle's or_isr_generate on the same seeds:
parton counts, statuses, cycles, emissions, flavours, trials, the emission
hash, every momentum, weights, observables and histograms (bars in
tests/parity.py); ragged sizes, energies, cutoffs, overflow and refused
requests."""
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


@pytest.mark.parametrize("n,sqs,q,tc,cap,seed", [
    (3000, 1960.0, 91.2, 1.0, 64, 7),
    (1, 1960.0, 91.2, 1.0, 64, 8),
    (65, 500.0, 91.2, 0.5, 64, 9),
    (4097, 14000.0, 91.2, 1.0, 128, 10),
    (2000, 1960.0, 30.0, 2.0, 64, 11),
    (1500, 1960.0, 91.2, 1.0, 4, 12),  # small records: some events overflow
])
def test_isr_equals_oracle(ctx, oracle, n, sqs, q, tc, cap, seed):
    print(f"case isr n={n} sqrt_s={sqs} q={q} tcut={tc} cap={cap} seed={seed}", flush=True)
    g = ctx.generate_isr(n, sqrt_s_hadron=sqs, q=q, t_cut=tc, seed=seed, max_partons=cap, summary=True, records=True)
    o = oracle.isr_generate(seed, 0, n, sqs, q, tc, cap, records=True)
    rep, same = parity.compare(g, o, q, n, isr=True)
    print(rep, flush=True)
    parity.assert_parity(rep)
    assert np.allclose(g["hist_lo"], parity.ISR_LO) and np.allclose(g["hist_hi"], parity.ISR_HI)
    st = o["sum_i"][:, 1]
    assert g["n_done"] == int((st == 1).sum()) and g["n_overflow"] == int((st == 2).sum())
    assert g["total_emissions"] == int(o["sum_i"][:, 3].sum())
    if cap == 4:
        assert g["n_overflow"] > 0
    elif n > 100:
        assert g["n_done"] == n and g["total_emissions"] > n / 2


def test_isr_refuses_bad_requests(ctx):
    import paper_2403_08692_amd as P

    for kw in (dict(sqrt_s_hadron=80.0, q=91.2), dict(max_partons=2), dict(t_cut=3000.0)):
        with pytest.raises(P.VshError) as ei:
            ctx.generate_isr(10, **kw)
        assert ei.value.code == -1
