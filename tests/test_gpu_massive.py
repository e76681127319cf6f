"""GPU parity of massive charm and bottom quarks (the extension the
conclusions name) against the oracle's massive shower, event by event, in
both forms and through serving."""
import numpy as np
import pytest

from tests import parity

pytestmark = pytest.mark.gpu

MC, MB = 1.5, 4.8
TABLE = [0.0, 0.0, 0.0, 0.0, MC, MB]


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


@pytest.mark.parametrize("mapping", [1, 0])
@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("ecm,tcut,cap,n", [(91.2, 1.0, 64, 2000), (12.0, 0.5, 64, 1500), (500.0, 0.25, 256, 400)])
def test_massive_parity(ctx, oracle, mapping, persistent, ecm, tcut, cap, n):
    # mapping 1: the trials of a wave's events spread over its lanes; 0: one lane per event
    key = "mapping" if persistent else "plain_mapping"
    before = ctx.get_tuning()[key]
    ctx.set_tuning(**{key: mapping})
    try:
        print(f"case massive ecm={ecm} tcut={tcut} cap={cap} n={n} persistent={persistent} mapping={mapping}",
              flush=True)
        g = ctx.generate(n, seed=21, ecm=ecm, t_cut=tcut, max_partons=cap, summary=True, records=True,
                         persistent=persistent, mass_c=MC, mass_b=MB)
    finally:
        ctx.set_tuning(**{key: before})
    o = oracle.generate(21, 0, n, ecm, tcut, cap, records=True, mass=TABLE)
    rep, same = parity.compare(g, o, ecm, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
    fl = o["sum_i"][:, 4]
    assert (fl == 5).sum() > 0.1 * n and g["n_done"] == int((o["sum_i"][:, 1] == 1).sum())
    # heavy quarks on their mass shells in the GPU records
    off = g["rec_offsets"].astype(np.int64)
    for e in np.flatnonzero(fl >= 4)[:50]:
        p, pid = g["rec_p"][off[e]:off[e + 1]], g["rec_pid"][off[e]:off[e + 1]]
        m2 = p[:, 0] ** 2 - (p[:, 1:] ** 2).sum(1)
        want = np.array([0.0 if f == 21 else TABLE[abs(f)] ** 2 for f in pid])
        np.testing.assert_allclose(m2, want, atol=1e-9 * ecm * ecm)


@pytest.mark.parametrize("mapping", [1, 0])
def test_massive_and_massless_requests_served_together(ctx, mapping):
    # an epoch with a massive request runs the massive kernel for every event
    # of it; massless events must come out as they do alone
    before = ctx.get_tuning()
    ctx.set_tuning(plain_mapping=mapping, mapping=mapping)
    try:
        print(f"case served together mapping={mapping}", flush=True)
        heavy = dict(seed=31, ecm=91.2, t_cut=1.0, max_partons=64, mass_c=MC, mass_b=MB)
        light = dict(seed=32, ecm=91.2, t_cut=1.0, max_partons=64)
        ref_h = ctx.generate(3000, summary=True, **heavy)
        ref_l = ctx.generate(3000, summary=True, **light)
        th, tl = ctx.submit(3000, summary=True, **heavy), ctx.submit(3000, summary=True, **light)
        for t, ref in ((th, ref_h), (tl, ref_l)):
            got = ctx.wait(t)
            np.testing.assert_array_equal(got["sum_i"], ref["sum_i"])
            np.testing.assert_array_equal(got["hash"], ref["hash"])
            np.testing.assert_allclose(got["sum_d"], ref["sum_d"], rtol=1e-12, atol=1e-15)
    finally:
        ctx.set_tuning(plain_mapping=before["plain_mapping"], mapping=before["mapping"])


def test_invalid_masses_rejected(ctx):
    import paper_2403_08692_amd as P

    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(P.VshError) as ei:
            ctx.generate(10, mass_b=bad)
        assert ei.value.code == -1


@pytest.mark.parametrize("persistent,masses", [(False, True), (True, True), (False, False), (True, False)])
def test_options_together(ctx, oracle, persistent, masses):
    # tail cut, weighted veto and (optionally) quark masses in one request
    n, C, t_over = 2000, 40, 20.0
    mc, mb = (MC, MB) if masses else (0.0, 0.0)
    print(f"case options n={n} C={C} t_over={t_over} masses={masses} persistent={persistent}", flush=True)
    g = ctx.generate(n, seed=23, ecm=200.0, t_cut=0.5, max_partons=128, summary=True, records=True,
                     persistent=persistent, cycle_limit=C, t_over=t_over, mass_c=mc, mass_b=mb)
    o = oracle.generate(23, 0, n, 200.0, 0.5, 128, records=True, max_cycles=C, t_over=t_over,
                        mass=TABLE if masses else None)
    rep, same = parity.compare(g, o, 200.0, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
    st = o["sum_i"][:, 1]
    assert (st == 5).any() and (o["sum_d"][:, 0] < 0).any()
    assert g["n_cycle_limit"] == int((st == 5).sum())


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("cap", [64, 65])
def test_massive_layout_boundary(ctx, oracle, persistent, cap):
    # with quark masses the kernels keep the per-event layout up to 64
    # partons and take the single-request one above: the same events in both
    n = 600
    print(f"case massive layout boundary cap={cap} persistent={persistent}", flush=True)
    g = ctx.generate(n, seed=29, ecm=91.2, t_cut=1.0, max_partons=cap, summary=True, records=True,
                     persistent=persistent, mass_c=MC, mass_b=MB, t_over=20.0, cycle_limit=40)
    o = oracle.generate(29, 0, n, 91.2, 1.0, cap, records=True, mass=TABLE, t_over=20.0, max_cycles=40)
    rep, same = parity.compare(g, o, 91.2, n)
    print(rep, flush=True)
    parity.assert_parity(rep)
