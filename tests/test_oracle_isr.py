"""Pins of the oracle's initial-state shower (Drell-Yan q qbar -> V with a
closed-form stand-in parton density; no PDF set is available here, so
agreement with real densities is parity unpinned).

Each part is checked against something it does not share code with: the
density's momentum sum rule by quadrature; the Drell-Yan start's
kinematics and its mean weight against the luminosity integral; the
initial-initial map's invariants (momentum conservation, mass shells, the
emitter's new fraction x/z, the gluon's transverse momentum, the dipole
variables recovered from the momenta); the first emission against the
Sudakov factor of backward evolution, PDF ratio included, by quadrature;
the validation's rejections; colour lines."""
import numpy as np
import pytest
from scipy import integrate

CF = 4 / 3
SQS, Q, TC = 1960.0, 91.2, 1.0


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def _f(x):
    # the stand-in density, written out here from its definition
    return (63 / 128) * x ** -0.5 * (1 - x) ** 3


def _alpha_s(t):
    b0 = 23.0 / (12 * np.pi)
    return 0.118 / (1 + 0.118 * b0 * np.log(t / 91.1876 ** 2))


def test_density_obeys_the_momentum_sum_rule(oracle):
    q, _ = integrate.quad(lambda x: x * oracle.pdf_q(x), 0, 1, epsabs=0, epsrel=1e-12, limit=200)
    g, _ = integrate.quad(lambda x: x * oracle.pdf_g(x), 0, 1, epsabs=0, epsrel=1e-12, limit=200)
    assert 10 * q + g == pytest.approx(1.0, rel=1e-10)  # ten quark and antiquark flavours and the gluon
    assert 10 * q == pytest.approx(0.5, rel=1e-10)
    for x in (1e-4, 0.01, 0.3, 0.9):
        assert oracle.pdf_q(x) == pytest.approx(_f(x), rel=1e-14)
    assert oracle.pdf_q(1.0) == 0.0 and oracle.pdf_q(0.0) == 0.0


def test_drell_yan_start(oracle):
    tau = (Q / SQS) ** 2
    Y = np.log(SQS / Q)
    n = 60_000
    ys, ws, fl, qa = np.zeros(n), np.zeros(n), np.zeros(n, int), np.zeros(n, bool)
    for e in range(n):
        m = oracle.isr_me(3, e, SQS, Q)
        p = m["p"]
        assert m["xa"] * m["xb"] == pytest.approx(tau, rel=1e-14)
        np.testing.assert_allclose(p[2], p[0] + p[1], rtol=0, atol=1e-12 * SQS)
        assert mdot(p[2], p[2]) == pytest.approx(Q * Q, rel=1e-12)
        assert p[0][3] > 0 > p[1][3] and abs(mdot(p[0], p[0])) < 1e-9 and abs(mdot(p[1], p[1])) < 1e-9
        ys[e], ws[e], fl[e], qa[e] = m["y"], m["weight"], m["flavour"], m["quark_from_a"]
    assert np.abs(ys).max() < Y
    assert np.histogram(ys, bins=10, range=(-Y, Y))[0].min() > 0.9 * n / 10
    assert set(fl) == {1, 2, 3, 4, 5} and abs(qa.mean() - 0.5) < 4 * 0.5 / np.sqrt(n)
    # mean weight = luminosity integral over the rapidity
    lum, _ = integrate.quad(lambda y: 10 * tau * _f(np.sqrt(tau) * np.exp(y)) * _f(np.sqrt(tau) * np.exp(-y)),
                            -Y, Y, epsabs=0, epsrel=1e-10, limit=200)
    assert abs(ws.mean() - lum) < 4 * ws.std() / np.sqrt(n)


def _start(oracle, y, f=2):
    """A Drell-Yan start at rapidity y: incoming quark from A, antiquark from B."""
    tau = (Q / SQS) ** 2
    xa, xb = np.sqrt(tau) * np.exp(y), np.sqrt(tau) * np.exp(-y)
    e = SQS / 2
    pa, pb = np.array([xa * e, 0, 0, xa * e]), np.array([xb * e, 0, 0, -xb * e])
    return np.array([pa, pb, pa + pb]), [f, -f, 23], [1, 0, 0], [0, 1, 0], xa, xb


def test_initial_initial_map_invariants(oracle):
    checked = 0
    for e in range(3000):
        p, pid, col, acol, xa, xb = _start(oracle, -1.2 + 2.4 * (e % 7) / 6)
        st = 2 * mdot(p[0], p[1])
        r = oracle.isr_shower(5, e, Q, TC, p, pid, col, acol, xa, xb, cap=8, max_emit=1)
        if r["n_emit"] != 1:
            continue
        t, z, xnew, K, line = r["log"][0][:5]
        line = int(line)
        P = r["p"]
        pa, pb, pj = P[line], P[1 - line], P[3]
        x_old = (xa, xb)[line]
        assert xnew == pytest.approx(x_old / z, rel=1e-13)
        assert (r["xa"], r["xb"])[line] == pytest.approx(x_old / z, rel=1e-13)
        assert pa[0] == pytest.approx(p[line][0] / z, rel=1e-13) and abs(pa[1]) + abs(pa[2]) == 0
        np.testing.assert_allclose(P[2] + P[3], P[0] + P[1], rtol=0, atol=1e-11 * SQS)
        assert mdot(P[2], P[2]) == pytest.approx(Q * Q, rel=1e-10)
        assert abs(mdot(pj, pj)) < 1e-9 * Q * Q
        assert pj[1] ** 2 + pj[2] ** 2 == pytest.approx(t, rel=1e-10)  # both beams along z: kT is the gluon's pT
        # the dipole variables from the momenta: z = 1 - (pj.pa + pj.pb)/pa.pb, v = pj.pa/pa.pb
        ab = mdot(pa, pb)
        zr = 1 - (mdot(pj, pa) + mdot(pj, pb)) / ab
        vr = mdot(pj, pa) / ab
        assert zr == pytest.approx(z, rel=1e-10)
        assert vr * (1 - zr - vr) == pytest.approx(t * z / st, rel=1e-9)
        assert vr <= 0.5 * (1 - zr)  # the collinear root
        assert 2 * ab == pytest.approx(st / z, rel=1e-12)
        checked += 1
    assert checked > 1000


def _rho(t, x, st):
    """Backward-evolution density of one line per ln t: alpha_s/(2 pi) int dz
    P_qq(z)/z f(x/z)/f(x) over x < z with (1 - z)^2 >= 4 t z / st."""
    a = t / st
    zmax = 1 + 2 * a - 2 * np.sqrt(a + a * a)
    if zmax <= x:
        return 0.0
    val, _ = integrate.quad(lambda z: CF * (1 + z * z) / (1 - z) / z * _f(x / z) / _f(x), x, zmax,
                            epsabs=0, epsrel=1e-10, limit=400)
    return _alpha_s(t) / (2 * np.pi) * val


def _cum(lt_lo, lt_hi, x, st):
    if lt_lo >= lt_hi:
        return 0.0
    return integrate.quad(lambda lt: _rho(np.exp(lt), x, st), lt_lo, lt_hi, epsabs=0, epsrel=1e-9, limit=400)[0]


@pytest.mark.parametrize("y", [0.0, 1.5])
def test_first_emission_follows_the_backward_sudakov(oracle, y):
    """The veto algorithm with the PDF ratio reproduces the Sudakov factor of
    backward evolution: the first emission's scale and the line it comes
    from, against quadrature."""
    p, pid, col, acol, xa, xb = _start(oracle, y)
    st = 2 * mdot(p[0], p[1])
    n = 30_000
    ts, lines = np.zeros(n), np.full(n, -1)
    for e in range(n):
        r = oracle.isr_shower(17, e, Q, TC, p, pid, col, acol, xa, xb, cap=8, max_emit=1, max_log=1)
        if r["n_emit"]:
            ts[e], lines[e] = r["log"][0][0], int(r["log"][0][4])
    lq = np.log(Q * Q)
    edges = np.linspace(np.log(TC), lq, 13)
    # Delta(t) = exp(-sum over lines of the integral from t up to Q^2)
    cum = np.array([_cum(le, lq, xa, st) + _cum(le, lq, xb, st) for le in edges])
    delta = np.exp(-cum)
    probs = np.diff(delta)
    counts, _ = np.histogram(np.log(ts[ts > 0]), bins=edges)
    expct = n * probs
    ok = expct > 5
    chi2 = ((counts[ok] - expct[ok]) ** 2 / expct[ok]).sum() + ((ts == 0).sum() - n * delta[0]) ** 2 / (n * delta[0])
    ndf = int(ok.sum())
    assert chi2 < ndf + 5 * np.sqrt(2 * ndf), (chi2, ndf)
    # share of line A among first emissions: int rho_A Delta / (1 - Delta(t_C))
    share_a = integrate.quad(lambda lt: _rho(np.exp(lt), xa, st) * np.exp(-(_cum(lt, lq, xa, st) + _cum(lt, lq, xb, st))),
                             np.log(TC), lq, epsabs=0, epsrel=1e-6, limit=100)[0] / (1 - delta[0])
    em = lines >= 0
    frac_a = (lines[em] == 0).mean()
    assert abs(frac_a - share_a) < 4 * np.sqrt(share_a * (1 - share_a) / em.sum()), (frac_a, share_a)
    if y > 0:  # the line with the larger fraction radiates less (the density falls towards x = 1)
        assert share_a < 0.5


def test_showered_events_are_valid_and_coloured(oracle):
    g = oracle.isr_generate(9, 0, 3000, SQS, Q, TC, 64, records=True)
    assert (g["sum_i"][:, 1] == 1).all()
    for e in range(3000):
        k = g["rec"]["n"][e]
        pid, col, acol = g["rec"]["pid"][e, :k], g["rec"]["col"][e, :k], g["rec"]["acol"][e, :k]
        assert list(pid[3:]) == [21] * (k - 3) and pid[2] == 23
        idx = [c for c in col if c] + [a for a in acol if a]
        for c in set(idx):
            assert list(col).count(c) == 1 and list(acol).count(c) == 1
        P = g["rec"]["p"][e, :k]
        assert oracle.isr_validate(P, Q) == 1
        xa, xb = g["sum_d"][e, 3], g["sum_d"][e, 4]
        assert 0 < xa < 1 and 0 < xb < 1
        assert P[0][0] == pytest.approx(xa * SQS / 2, rel=1e-12) and P[1][0] == pytest.approx(xb * SQS / 2, rel=1e-12)
    assert g["sum_i"][:, 3].mean() > 0.5


def test_validation_rejects(oracle):
    g = oracle.isr_generate(9, 0, 50, SQS, Q, TC, 64, records=True)
    for e in range(20):
        k = g["rec"]["n"][e]
        P = g["rec"]["p"][e, :k].copy()
        E = P[0][0] + P[1][0]
        for frac, want in ((2e-10, 4), (0.5e-10, 1)):
            R = P.copy()
            R[2, 1] += frac * E
            assert oracle.isr_validate(R, Q) == want
        R = P.copy()
        R[2, 3] = np.nan
        assert oracle.isr_validate(R, Q) == 3
        assert oracle.isr_validate(P, Q * (1 + 1e-6)) == 4  # V off its mass shell
