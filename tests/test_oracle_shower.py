"""Pins of the oracle's shower: the Catani-Seymour map's invariants, the colour
and flavour bookkeeping, and the veto algorithm against the Sudakov factor
computed by direct quadrature (Appendix A: the veto algorithm must reproduce
the no-emission probability of the Sudakov equation)."""
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "derived_physics.txt")
CF, CA, TR = 4 / 3, 3.0, 0.5


def _massless(rng, e):
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    return np.array([e, *(e * v)])


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def test_cs_map_invariants(oracle):
    rng = np.random.default_rng(5)
    for trial in range(2000):
        pi = _massless(rng, rng.uniform(1, 50))
        pk = _massless(rng, rng.uniform(1, 50))
        q2 = 2 * mdot(pi, pk)
        if q2 < 1e-3:
            continue
        z = rng.uniform(0.01, 0.99)
        y = rng.uniform(1e-6, 0.999)
        t = y * z * (1 - z) * q2
        phi = rng.uniform(0, 2 * np.pi)
        a, j, k = oracle.split_kinematics(pi, pk, t, z, phi)
        scale = max(pi[0], pk[0])
        np.testing.assert_allclose(a + j + k, pi + pk, atol=1e-12 * scale)
        for v in (a, j, k):
            assert abs(mdot(v, v)) < 1e-11 * scale ** 2
            assert v[0] > 0
        pij, pik, pjk = mdot(a, j), mdot(a, k), mdot(j, k)
        assert pij / (pij + pik + pjk) == pytest.approx(y, rel=1e-9, abs=1e-14)
        assert pik / (pik + pjk) == pytest.approx(z, rel=1e-9)
        # k_T^2 = t: the transverse momentum of the splitting products
        kt = a - z * pi - (1 - z) * y * pk
        assert -mdot(kt, kt) == pytest.approx(t, rel=1e-8)


def test_cs_map_azimuth_is_a_rotation(oracle):
    # varying phi rotates k_T around the dipole axis: p_i.p_k fixed, and the
    # transverse part at phi and phi + pi is opposite
    rng = np.random.default_rng(6)
    pi = _massless(rng, 30.0)
    pk = _massless(rng, 20.0)
    q2 = 2 * mdot(pi, pk)
    z, y = 0.3, 0.2
    t = y * z * (1 - z) * q2
    a0, _, _ = oracle.split_kinematics(pi, pk, t, z, 0.4)
    a1, _, _ = oracle.split_kinematics(pi, pk, t, z, 0.4 + np.pi)
    base = z * pi + (1 - z) * y * pk
    np.testing.assert_allclose(a0 - base, -(a1 - base), atol=1e-12 * 30)


def _check_colour_and_flavour(pid, col, acol):
    n = len(pid)
    cols = [c for c in col if c != 0]
    acols = [a for a in acol if a != 0]
    assert sorted(cols) == sorted(acols)
    assert len(set(cols)) == len(cols)
    for p, c, a in zip(pid, col, acol):
        if 1 <= p <= 5:
            assert c != 0 and a == 0
        elif -5 <= p <= -1:
            assert c == 0 and a != 0
        else:
            assert p == 21 and c != 0 and a != 0
    for f in range(1, 6):
        assert (pid == f).sum() == (pid == -f).sum()
    # every chain runs from a quark through gluons to an antiquark
    by_acol = {a: i for i, a in enumerate(acol) if a != 0}
    visited = 0
    for i in range(n):
        if 1 <= pid[i] <= 5:
            cur = i
            while True:
                visited += 1
                nxt = by_acol[col[cur]]
                cur = nxt
                if pid[cur] < 0:
                    visited += 1
                    break
    assert visited == n


def test_showered_events_colour_flavour_conservation(oracle):
    r = oracle.generate(1, 0, 3000, 91.2, 0.5, 64, records=True)
    rec = r["rec"]
    st = r["sum_i"][:, 1]
    assert (st == 1).all()
    for e in range(3000):
        n = rec["n"][e]
        _check_colour_and_flavour(rec["pid"][e, :n], rec["col"][e, :n], rec["acol"][e, :n])
        p = rec["p"][e, :n]
        np.testing.assert_allclose(p.sum(0), [91.2, 0, 0, 0], atol=1e-10 * 91.2)


def test_overflow_status_at_small_cap(oracle):
    r = oracle.generate(1, 0, 500, 91.2, 1.0, 3)
    st = r["sum_i"][:, 1]
    n = r["sum_i"][:, 0]
    assert set(np.unique(st)) <= {1, 2}
    assert (st == 2).any() and (st == 1).any()
    assert (n[st == 2] == 3).all()
    # overflowed events are not histogrammed
    assert r["hist"][7, :, 2].sum() == (st == 1).sum()


# ---------------------------------------------------------------------------
# Tail cut (the study that the caption of Fig. 7 suggests): an event still
# above the cutoff after C veto cycles is given up and vetoed.  With the same
# random numbers the cut run is the first C cycles of the full run.
# ---------------------------------------------------------------------------
def test_tail_cut_is_a_prefix_of_the_full_shower(oracle):
    truncated = 0
    for e in range(150):
        f, _, _, _, p = oracle.me_event(2, e, 91.2)
        args = (2, e, 91.2, 1.0, p, [f, -f], [1, 0], [0, 1])
        full = oracle.shower(*args)
        assert full["status"] == 1
        for C in (1, 3, full["cycles"] // 2, full["cycles"] - 1, full["cycles"], full["cycles"] + 5):
            if C < 1:
                continue
            cut = oracle.shower(*args, max_cycles=C)
            if C >= full["cycles"]:  # the event reaches the cutoff in time: nothing changes
                for k in ("status", "n", "cycles", "hash", "n_emit"):
                    assert cut[k] == full[k], (e, C, k)
                np.testing.assert_array_equal(cut["p"], full["p"])
                continue
            truncated += 1
            assert cut["status"] == 5 and cut["cycles"] == C, (e, C)
            m = cut["n_emit"]
            assert m <= full["n_emit"] and cut["n"] == 2 + m
            # its emissions are the first m of the full shower ...
            np.testing.assert_array_equal(cut["log"], full["log"][:m])
            # ... and its partons those after the m-th emission of the full shower
            ref = oracle.shower(*args, max_emit=m) if m > 0 else dict(p=p, pid=[f, -f], col=[1, 0], acol=[0, 1])
            np.testing.assert_array_equal(cut["p"], ref["p"])
            for k in ("pid", "col", "acol"):
                np.testing.assert_array_equal(cut[k], ref[k])
    assert truncated > 300


def _fill(h, x, w, lo, hi):
    if not x >= lo:
        b = 0
    elif x >= hi:
        b = 51
    else:
        b = min(1 + int((x - lo) / (hi - lo) * 50), 50)
    h[b] += (w, w * w, 1.0)


def test_tail_cut_vetoes_exactly_the_long_events(oracle):
    n, C = 1500, 35
    full = oracle.generate(9, 0, n, 91.2, 1.0, 64)
    cut = oracle.generate(9, 0, n, 91.2, 1.0, 64, max_cycles=C)
    long = full["sum_i"][:, 2] > C
    assert 0.05 < long.mean() < 0.5
    # events that end within C cycles are untouched
    np.testing.assert_array_equal(cut["sum_i"][~long], full["sum_i"][~long])
    np.testing.assert_array_equal(cut["sum_d"][~long], full["sum_d"][~long])
    np.testing.assert_array_equal(cut["hash"][~long], full["hash"][~long])
    # the others are given up after exactly C cycles, with no observables
    assert (cut["sum_i"][long, 1] == 5).all() and (cut["sum_i"][long, 2] == C).all()
    assert (cut["sum_d"][long, 2:9] == 0).all()
    # the histograms hold the kept events only, filled as in the full run
    lo, hi = oracle.hist_ranges()
    ref = np.zeros_like(cut["hist"])
    for e in np.flatnonzero(~long):
        d = full["sum_d"][e]
        xs = [np.log10(d[2]) if d[2] > 0 else -np.inf, np.log10(d[3]) if d[3] > 0 else -np.inf, *d[4:9], d[1]]
        for h, x in enumerate(xs):
            _fill(ref[h], x, d[0], lo[h], hi[h])
    np.testing.assert_allclose(cut["hist"], ref, rtol=1e-12, atol=0)


# ---------------------------------------------------------------------------
# Veto algorithm against the Sudakov factor
# ---------------------------------------------------------------------------
def _alpha_s(t):
    b0 = 23.0 / (12 * np.pi)
    return 0.118 / (1 + 0.118 * b0 * np.log(t / 91.1876 ** 2))


def _rho_qg(t, q2):
    """Emission density dP/dt of one quark dipole end at scale t: the
    integrand of the Sudakov exponent, alpha_s(t)/(2 pi t) * int dz V (1-y)
    over the z range where y = t/(Q^2 z (1-z)) < 1."""
    if 4 * t >= q2:
        return 0.0
    r = np.sqrt(1 - 4 * t / q2)
    zm, zp = 0.5 * (1 - r), 0.5 * (1 + r)

    def f(z):
        y = t / (q2 * z * (1 - z))
        return CF * (2 / (1 - z * (1 - y)) - (1 + z)) * (1 - y)

    val, _ = integrate.quad(f, zm, zp, epsabs=0, epsrel=1e-10, limit=200)
    return _alpha_s(t) / (2 * np.pi * t) * val


def _sudakov_qqbar(tlo, s):
    """Delta(tlo, s) for the q qbar start: two quark ends, Q^2 = s."""
    val, _ = integrate.quad(lambda lt: np.exp(lt) * _rho_qg(np.exp(lt), s), np.log(tlo), np.log(s / 4),
                            epsabs=0, epsrel=1e-9, limit=200)
    return np.exp(-2 * val)


def test_sudakov_quadrature_matches_derived_values():
    for ecm, tc, ref in [(row[0], row[1], row[2]) for row in _golden_sudakov()]:
        assert _sudakov_qqbar(tc, ecm * ecm) == pytest.approx(ref, rel=2e-4)


def _golden_sudakov():
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            w = line.split()
            if w and w[0] == "sudakov":
                out.append([float(x) for x in w[1:]])
    return out


def _first_emissions(oracle, ecm, tc, n, seed):
    L = oracle
    ts = np.zeros(n)
    for e in range(n):
        f, c, ph, w, p = L.me_event(seed, e, ecm)
        r = L.shower(seed, e, ecm, tc, p, [f, -f], [1, 0], [0, 1], cap=4, max_emit=1, max_log=1)
        ts[e] = r["log"][0, 0] if r["n_emit"] else 0.0
    return ts


@pytest.mark.parametrize("ecm,tc", [(91.2, 1.0), (10.0, 1.0)])
def test_first_emission_follows_sudakov(oracle, ecm, tc):
    n = 40_000
    ts = _first_emissions(oracle, ecm, tc, n, seed=21)
    s = ecm * ecm
    edges = np.exp(np.linspace(np.log(tc), np.log(s / 4), 16))
    cdf = np.array([_sudakov_qqbar(x, s) for x in edges])  # P(t1 < x) for x >= tc
    probs = np.diff(cdf)
    p_none = cdf[0]
    counts, _ = np.histogram(ts[ts > 0], bins=edges)
    exp = n * probs
    chi2 = ((counts - exp) ** 2 / exp).sum() + ((ts == 0).sum() - n * p_none) ** 2 / (n * p_none)
    ndf = len(probs)
    assert chi2 < ndf + 5 * np.sqrt(2 * ndf), chi2
    assert ts.max() <= s / 4


@pytest.mark.parametrize("t_over", [10.0, 300.0])
def test_weighted_veto_follows_sudakov(oracle, t_over):
    # alpha_s(t_over) in the trial density undershoots the true density below
    # t_over; with the weighted veto the weighted first-emission distribution
    # and the weighted no-emission probability are still the Sudakov ones
    ecm, tc, n = 91.2, 1.0, 40_000
    s = ecm * ecm
    ts, ws = np.zeros(n), np.zeros(n)
    for e in range(n):
        f, c, ph, w, p = oracle.me_event(23, e, ecm)
        r = oracle.shower(23, e, ecm, tc, p, [f, -f], [1, 0], [0, 1], cap=4, max_emit=1, max_log=1, t_over=t_over)
        ts[e] = r["log"][0, 0] if r["n_emit"] else 0.0
        ws[e] = r["weight"]
    assert (ws < 0).any() and (ws > 1).any()  # the weights are in play
    edges = np.exp(np.linspace(np.log(tc), np.log(s / 4), 16))
    cdf = np.array([_sudakov_qqbar(x, s) for x in edges])
    exp = np.concatenate([[cdf[0]], np.diff(cdf)]) * n
    idx = np.where(ts > 0, np.searchsorted(edges, ts) , 0)  # 0 = no emission, b = bin b
    W = np.bincount(idx, weights=ws, minlength=len(edges))
    V = np.bincount(idx, weights=ws * ws, minlength=len(edges))
    chi2 = ((W - exp) ** 2 / V).sum()
    ndf = len(edges)
    assert chi2 < ndf + 5 * np.sqrt(2 * ndf), chi2
    # the same events unweighted fail that bar: the weights carry the correction
    cnt = np.bincount(idx, minlength=len(edges))
    assert ((cnt - exp) ** 2 / np.maximum(cnt, 1)).sum() > ndf + 5 * np.sqrt(2 * ndf)


def test_weighted_veto_is_inert_when_the_trial_density_bounds(oracle):
    # t_over at or below t_C keeps an overestimate: weights stay 1 and the
    # events are those of the plain veto (t_over below t_C only wastes trials)
    base = oracle.generate(31, 0, 300, 91.2, 1.0, 64)
    same = oracle.generate(31, 0, 300, 91.2, 1.0, 64, t_over=1.0)
    np.testing.assert_array_equal(same["sum_i"], base["sum_i"])
    np.testing.assert_array_equal(same["sum_d"], base["sum_d"])
    loose = oracle.generate(31, 0, 300, 91.2, 1.0, 64, t_over=0.5)
    np.testing.assert_array_equal(loose["sum_d"][:, 0], base["sum_d"][:, 0])
    assert (loose["sum_i"][:, 2] >= base["sum_i"][:, 2]).mean() > 0.5


def test_no_emission_fraction_is_sudakov(oracle):
    n = 100_000
    r = oracle.generate(17, 0, n, 91.2, 1.0, 64)
    frac = (r["sum_i"][:, 0] == 2).mean()
    ref = 0.066353
    assert abs(frac - ref) < 4 * np.sqrt(ref * (1 - ref) / n)
    # two-parton events are pencil-like: T = 1, and every shape vanishes
    two = r["sum_i"][:, 0] == 2
    d = r["sum_d"][two]
    assert np.all(d[:, 2:9] < 1e-12)


@pytest.mark.parametrize("ecm,tc", [(10.0, 4.0), (6.0, 4.0)])
def test_emission_probability_near_the_kinematic_limit(oracle, ecm, tc):
    # t_C close to s/4: most of the phase space lies near the cutoff, where
    # the z range of the overestimate meets the physical limit
    # z(1 - z) = t_C / Q^2.  With room for no third parton, the first
    # accepted emission overflows the record, so the overflow fraction is
    # 1 - Delta(t_C, s) of the q qbar start.
    n = 1_000_000
    r = oracle.generate(29, 0, n, ecm, tc, 2)
    frac = (r["sum_i"][:, 1] == 2).mean()
    ref = 1.0 - _sudakov_qqbar(tc, ecm * ecm)
    assert abs(frac - ref) < 4.5 * np.sqrt(ref * (1 - ref) / n), (frac, ref)


def _qgq_start():
    # a fixed q g qbar configuration at sqrt(s) = 91.2 GeV: x_q = 0.8, x_qbar = 0.7
    ecm = 91.2
    x1, x3 = 0.8, 0.7
    x2 = 2 - x1 - x3
    E = np.array([x1, x2, x3]) * ecm / 2
    c13 = 1 - 2 * (1 - x2) / (x1 * x3)
    s13 = np.sqrt(1 - c13 * c13)
    p1 = np.array([E[0], 0, 0, E[0]])
    p3 = np.array([E[2], E[2] * s13, 0, E[2] * c13])
    p2 = np.array([ecm, 0, 0, 0]) - p1 - p3
    return ecm, np.array([p1, p2, p3]), [1, 21, -1], [1, 2, 0], [0, 1, 2]


def test_qgq_first_emission_channels(oracle):
    """From a fixed q g qbar start, the share of first emissions per channel
    (q end, gluon ends by kernel, qbar end) equals the integral of that
    channel's density times the total no-emission probability."""
    ecm, p, pid, col, acol = _qgq_start()
    tc = 1.0
    s = ecm * ecm
    q2_qg = 2 * mdot(p[0], p[1])
    q2_gq = 2 * mdot(p[1], p[2])

    def rho(t, q2, kind):
        if 4 * t >= q2:
            return 0.0
        r = np.sqrt(1 - 4 * t / q2)
        zm, zp = 0.5 * (1 - r), 0.5 * (1 + r)

        def f(z):
            y = t / (q2 * z * (1 - z))
            if kind == "qg":
                v = CF * (2 / (1 - z * (1 - y)) - (1 + z))
            elif kind == "gg":
                v = 0.5 * CA * (2 / (1 - z * (1 - y)) - 2 + z * (1 - z))
            else:
                v = 0.5 * TR * (1 - 2 * z * (1 - z))
            return v * (1 - y)

        val, _ = integrate.quad(f, zm, zp, epsabs=0, epsrel=1e-9, limit=200)
        return _alpha_s(t) / (2 * np.pi * t) * val

    # channels: (label, Q^2, kind, multiplicity)
    chans = [("q", q2_qg, "qg", 1), ("g->gg", q2_qg, "gg", 1), ("g->gg", q2_gq, "gg", 1),
             ("g->qq", q2_qg, "qq", 5), ("g->qq", q2_gq, "qq", 5), ("qbar", q2_gq, "qg", 1)]

    def total(t):
        return sum(m * rho(t, q2, kind) for _, q2, kind, m in chans)

    grid = np.exp(np.linspace(np.log(tc), np.log(s), 400))
    tot = np.array([total(t) for t in grid])
    # cumulative integral from t to s of the total density
    lg = np.log(grid)
    dens = tot * grid
    cum = np.concatenate([[0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(lg))])
    expo = cum[-1] - cum  # int_t^s
    delta = np.exp(-expo)
    pred = {}
    for label, q2, kind, m in chans:
        d = np.array([m * rho(t, q2, kind) for t in grid]) * grid * delta
        pred[label] = pred.get(label, 0.0) + np.sum(0.5 * (d[1:] + d[:-1]) * np.diff(lg))
    n = 30_000
    counts = {"q": 0, "g->gg": 0, "g->qq": 0, "qbar": 0, "none": 0}
    flav = np.zeros(6)
    for e in range(n):
        r = oracle.shower(33, e, ecm, tc, p, pid, col, acol, cap=6, max_emit=1, max_log=1)
        if r["n_emit"] == 0:
            counts["none"] += 1
            continue
        K, i = int(r["log"][0, 3]), int(r["log"][0, 4])
        if i == 0:
            counts["q"] += 1
        elif i == 2:
            counts["qbar"] += 1
        elif K == 10:
            counts["g->gg"] += 1
        else:
            counts["g->qq"] += 1
            flav[K - 10] += 1
    pnone = float(delta[0])
    assert counts["none"] == pytest.approx(n * pnone, abs=5 * np.sqrt(n * pnone) + 2)
    for label in ("q", "g->gg", "g->qq", "qbar"):
        mu = n * pred[label]
        assert abs(counts[label] - mu) < 5 * np.sqrt(mu) + 0.01 * mu, (label, counts[label], mu)
    # the five g -> f fbar kernels are equally likely
    f = flav[1:]
    assert ((f - f.mean()) ** 2 / f.mean()).sum() < 4 + 5 * np.sqrt(8)
