"""GPU parity of vsh_shower_records: caller-given initial states (q qbar,
q g qbar, q g g qbar chains, closed two-gluon loops) showered through both
plain mappings, event by event against the oracle's shower of the same
partons with the same event ids."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 11
TC = 1.0
CAP = 64


@pytest.fixture(scope="module")
def ctx():
    import paper_2403_08692_amd as P

    c = P.Context()
    yield c
    c.close()


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _rambo(rng, n, ecm):
    """n massless momenta with total (ecm, 0, 0, 0), flat in phase space
    (Kleiss, Stirling and Ellis)."""
    c = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * np.pi, n)
    q0 = -np.log(rng.uniform(0, 1, n) * rng.uniform(0, 1, n))
    s = np.sqrt(1 - c * c)
    q = np.stack([q0, q0 * s * np.cos(phi), q0 * s * np.sin(phi), q0 * c], axis=1)
    Q = q.sum(axis=0)
    M = np.sqrt(Q[0] ** 2 - Q[1:] @ Q[1:])
    b = -Q[1:] / M
    x = ecm / M
    gam = Q[0] / M
    a = 1 / (1 + gam)
    bq = q[:, 1:] @ b
    p = np.empty_like(q)
    p[:, 0] = x * (gam * q[:, 0] + bq)
    p[:, 1:] = x * (q[:, 1:] + b[None, :] * q[:, :1] + a * bq[:, None] * b[None, :])
    return p


def _events(oracle):
    """List of (p[n][4], pid, col, acol) initial states."""
    rng = np.random.default_rng(2024)
    ev = []
    for e in range(60):  # LO q qbar
        f, c, ph, w, p = oracle.me_event(SEED, 10_000 + e, 91.2)
        ev.append((p, [f, -f], [1, 0], [0, 1]))
    while len(ev) < 120:  # q g qbar, random Dalitz point and orientation
        x1, x3 = rng.uniform(0.05, 1, 2)
        x2 = 2 - x1 - x3
        if not (0 < x2 < 1 and x1 + x3 > 1):
            continue
        ecm = rng.choice([35.0, 91.2, 200.0])
        E = np.array([x1, x2, x3]) * ecm / 2
        c13 = 1 - 2 * (1 - x2) / (x1 * x3)
        s13 = np.sqrt(max(0.0, 1 - c13 * c13))
        p1 = np.array([0, 0, E[0]])
        p3 = np.array([E[2] * s13, 0, E[2] * c13])
        R = _rotation(rng)
        P = np.array([[E[0], *(R @ p1)], [E[1], *(R @ (-p1 - p3))], [E[2], *(R @ p3)]])
        f = int(rng.integers(1, 6))
        ev.append((P, [f, 21, -f], [1, 2, 0], [0, 1, 2]))
    for _ in range(60):  # q g g qbar chains
        P = _rambo(rng, 4, 91.2)
        f = int(rng.integers(1, 6))
        ev.append((P, [-f, 21, 21, f], [0, 1, 2, 3], [1, 2, 3, 0]))
    for _ in range(40):  # closed two-gluon colour loops
        P = _rambo(rng, 2, 91.2)
        ev.append((P, [21, 21], [1, 2], [2, 1]))
    return ev


@pytest.mark.parametrize("mapping", [1, 0])
def test_shower_records_equal_oracle(ctx, oracle, mapping):
    ev = _events(oracle)
    n = len(ev)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(x[1]) for x in ev])
    p = np.concatenate([np.asarray(x[0], np.float64) for x in ev])
    pid = np.concatenate([np.asarray(x[1]) for x in ev]).astype(np.int8)
    col = np.concatenate([np.asarray(x[2]) for x in ev]).astype(np.uint16)
    acol = np.concatenate([np.asarray(x[3]) for x in ev]).astype(np.uint16)
    ctx.set_tuning(plain_mapping=mapping)
    print(f"case shower_records n={n} mapping={mapping}", flush=True)
    g = ctx.shower_records(off, p, pid, col, acol, seed=SEED, first_event=0, t_cut=TC, max_partons=CAP)
    assert g["n_events"] == n
    gi, gd = g["sum_i"], g["sum_d"]
    go = g["rec_offsets"].astype(np.int64)
    mom_err, obs_bad, identical = 0.0, 0, 0
    for e, (P, fl, c, a) in enumerate(ev):
        ecm = float(np.asarray(P)[:, 0].sum())
        o = oracle.shower(SEED, e, ecm, TC, np.asarray(P, np.float64), fl, c, a, cap=CAP)
        same = (gi[0, e] == o["n"] and gi[1, e] == o["status"] and gi[2, e] == o["cycles"]
                and gi[3, e] == o["n_emit"] and g["hash"][e] == o["hash"])
        lo, hi = go[e], go[e + 1]
        same = same and hi - lo == o["n"] and np.array_equal(g["rec_pid"][lo:hi], o["pid"]) \
            and np.array_equal(g["rec_col"][lo:hi], o["col"]) and np.array_equal(g["rec_acol"][lo:hi], o["acol"])
        if not same:
            continue
        identical += 1
        mom_err = max(mom_err, float(np.abs(g["rec_p"][lo:hi] - o["p"]).max() / ecm))
        assert gd[0, e] == 1.0  # weights are 1
        if o["status"] == 1:
            ref = oracle.observables(o["p"], ecm)
            ok = np.isclose(gd[2:9, e], ref, rtol=1e-9, atol=1e-12)
            obs_bad += int((~ok).sum())
    print(f"identical {identical}/{n} mom_err {mom_err:.2e} obs_bad {obs_bad}", flush=True)
    assert identical >= 0.999 * n
    assert mom_err <= 1e-9
    assert obs_bad == 0
    # the starts differ in kind: some events emitted, gluon loops split
    assert (gi[3] > 0).mean() > 0.5


def _chain(n, f):
    """Colour chain q g ... g qbar of n partons: line m runs from parton m-1
    to parton m."""
    pid = [f] + [21] * (n - 2) + [-f]
    col = [a + 1 for a in range(n - 1)] + [0]
    acol = [0] + [a for a in range(1, n)]
    return pid, col, acol


def _pack(ev):
    n = len(ev)
    off = np.zeros(n + 1, np.uint64)
    off[1:] = np.cumsum([len(x[1]) for x in ev])
    p = np.concatenate([np.asarray(x[0], np.float64) for x in ev])
    pid = np.concatenate([np.asarray(x[1]) for x in ev]).astype(np.int8)
    col = np.concatenate([np.asarray(x[2]) for x in ev]).astype(np.uint16)
    acol = np.concatenate([np.asarray(x[3]) for x in ev]).astype(np.uint16)
    return off, p, pid, col, acol


def _oracle_event(oracle, seed, e, P, fl, c, a, tc, cap):
    """The oracle's shower of one start, then its validation (the status the
    library reports)."""
    P = np.asarray(P, np.float64)
    ecm = float(P[:, 0].sum())
    o = oracle.shower(seed, e, ecm, tc, P, fl, c, a, cap=cap)
    if o["status"] == 1:
        o["status"] = oracle.validate(o["p"], ecm)
    return o, ecm


def _compare(g, oracle, ev, seed, tc, cap):
    gi, gd, go = g["sum_i"], g["sum_d"], g["rec_offsets"].astype(np.int64)
    identical, mom_err, obs_bad, statuses = 0, 0.0, 0, []
    for e, (P, fl, c, a) in enumerate(ev):
        o, ecm = _oracle_event(oracle, seed, e, P, fl, c, a, tc, cap)
        statuses.append(o["status"])
        lo, hi = go[e], go[e + 1]
        same = (gi[0, e] == o["n"] and gi[1, e] == o["status"] and gi[2, e] == o["cycles"]
                and gi[3, e] == o["n_emit"] and g["hash"][e] == o["hash"] and hi - lo == o["n"]
                and np.array_equal(g["rec_pid"][lo:hi], o["pid"]) and np.array_equal(g["rec_col"][lo:hi], o["col"])
                and np.array_equal(g["rec_acol"][lo:hi], o["acol"]))
        if not same:
            print(f"event {e}: gpu n={gi[0, e]} status={gi[1, e]} cycles={gi[2, e]}; oracle n={o['n']} "
                  f"status={o['status']} cycles={o['cycles']}", flush=True)
            continue
        identical += 1
        fin = np.isfinite(o["p"])
        assert np.array_equal(np.isfinite(g["rec_p"][lo:hi]), fin)
        mom_err = max(mom_err, float(np.abs(g["rec_p"][lo:hi][fin] - o["p"][fin]).max() / ecm))
        if o["status"] == 1:
            ref = oracle.observables(o["p"], ecm)
            obs_bad += int((~np.isclose(gd[2:9, e], ref, rtol=1e-9, atol=1e-12)).sum())
    return identical, mom_err, obs_bad, np.array(statuses)


@pytest.mark.parametrize("mapping", [1, 0])
def test_long_chains_overflow_the_cycle_lists(ctx, oracle, mapping):
    """128 colour chains of 40 to 48 partons at 500 GeV (RAMBO momenta): a
    wave's first cycle has more than 2048 trial items and more than 512 stale
    partons, past the flattened kernel's LDS lists (items are then found by
    searching the per-owner offsets and gluon masks), and the group
    observables take events of 32 partons and more."""
    rng = np.random.default_rng(99)
    ev = []
    for k in range(128):
        n = int(rng.integers(40, 49))
        pid, col, acol = _chain(n, int(rng.integers(1, 6)))
        ev.append((_rambo(rng, n, 500.0), pid, col, acol))
    assert sum(len(x[1]) for x in ev[:64]) > 2048
    ctx.set_tuning(plain_mapping=mapping)
    print(f"case long chains n=128 mapping={mapping}", flush=True)
    g = ctx.shower_records(*_pack(ev), seed=SEED, first_event=0, t_cut=TC, max_partons=256)
    identical, mom_err, obs_bad, st = _compare(g, oracle, ev, SEED, TC, 256)
    print(f"identical {identical}/128 mom_err {mom_err:.2e} obs_bad {obs_bad} statuses {np.bincount(st)}", flush=True)
    assert identical == 128
    assert mom_err <= 1e-9 and obs_bad == 0
    assert (g["sum_i"][3] > 0).all()  # every chain radiated


def _moved(P, kind, ecm, rng):
    """A copy of the start P with one planted defect (or none)."""
    q = np.array(P, np.float64)
    s = ecm * ecm
    if kind == "px_big":
        q[0, 1] += 2e-10 * ecm
    elif kind == "px_small":
        q[0, 1] += 0.5e-10 * ecm
    elif kind == "two_off_shell":  # energy moved between two partons: total kept
        eps = 3e-10 * s / (2 * max(q[0, 0], q[1, 0]))
        q[0, 0] += eps
        q[1, 0] -= eps
    elif kind == "nan":
        q[int(rng.integers(len(q))), 2] = np.nan
    return q


@pytest.mark.parametrize("mapping", [1, 0])
def test_rejected_starts_match_the_oracle(ctx, oracle, mapping):
    """Starts that are finite but do not conserve momentum, have two partons
    off their mass shells, or carry a NaN, at sizes that take each
    observables path (3 and 8 partons in registers, 12 in 16-lane groups, 40
    in 64-lane groups), with the cutoff above every dipole (no emission: the
    validation sees the start as given) and with a real cutoff (the shower
    runs first).  Statuses and everything else equal the oracle's."""
    rng = np.random.default_rng(5)
    kinds = ["none", "px_big", "px_small", "two_off_shell", "nan"]
    want = {"none": 1, "px_big": 4, "px_small": 1, "two_off_shell": 4, "nan": 3}
    for tc, kinds_here in ((1.0e6, kinds), (TC, ["none", "px_big", "two_off_shell"])):
        ev, expect = [], []
        for n in (3, 8, 12, 40):
            for kind in kinds_here:
                for _ in range(4):
                    ecm = float(rng.choice([35.0, 91.2, 500.0]))
                    pid, col, acol = _chain(n, int(rng.integers(1, 6)))
                    ev.append((_moved(_rambo(rng, n, ecm), kind, ecm, rng), pid, col, acol))
                    expect.append(want[kind])
        ctx.set_tuning(plain_mapping=mapping)
        print(f"case rejected starts t_cut={tc} n={len(ev)} mapping={mapping}", flush=True)
        g = ctx.shower_records(*_pack(ev), seed=SEED, first_event=0, t_cut=tc, max_partons=256)
        identical, mom_err, obs_bad, st = _compare(g, oracle, ev, SEED, tc, 256)
        print(f"identical {identical}/{len(ev)} statuses {np.bincount(st)}", flush=True)
        assert identical == len(ev)
        assert mom_err <= 1e-9 and obs_bad == 0
        if tc > 1e5:  # no emission: the status is the planted one's
            np.testing.assert_array_equal(st, expect)
            np.testing.assert_array_equal(g["sum_i"][1], expect)
        else:
            assert set(st) <= {1, 2, 4} and (st == 4).sum() >= len(ev) // 2
        assert g["n_nonfinite"] == int((st == 3).sum()) and g["n_conservation"] == int((st == 4).sum())
