"""Pins of the oracle's massive quarks (the next step the conclusions name:
the veto algorithm unchanged, mass terms in the splitting functions).

Each pin checks a massive formula against something it does not share code
with: textbook threshold factors of e+e- -> Q Qbar, the invariants and the
Dalitz-plot Jacobian of the massive map, the massive eikonal factor, the
massless limit, and the first emission off a heavy pair against a
quadrature of the emission density over the Dalitz plot.

Parity unpinned: the g -> Q Qbar mass term beyond its bound (it never
exceeds the massless overestimate) and its massless limit.
"""
import numpy as np
import pytest
from scipy import integrate

CF = 4 / 3
MASS = np.array([0.0, 0.0, 0.0, 0.0, 1.5, 4.8])  # d, u, s massless; c, b


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def kallen(a, b, c):
    return a * a + b * b + c * c - 2 * (a * b + a * c + b * c)


# ---------------------------------------------------------------------------
# matrix element
# ---------------------------------------------------------------------------
def test_threshold_factor_of_the_vector_current(oracle):
    # far below the Z the photon dominates: each flavour's cross-section is
    # its massless one times beta (3 - beta^2) / 2
    s = 12.0 ** 2
    for f in (4, 5):
        m = MASS[f]
        beta = np.sqrt(1 - 4 * m * m / s)
        even = lambda fn: integrate.quad(fn, -1, 1, epsabs=0, epsrel=1e-12)[0]
        massive = beta * even(lambda c: oracle.me2_massive(f, s, c, m))
        massless = even(lambda c: oracle.me2(f, s, c))
        assert massive / massless == pytest.approx(beta * (3 - beta * beta) / 2, rel=2e-3)


@pytest.mark.parametrize("f,m", [(5, 30.0), (4, 20.0)])
def test_angular_structure_with_mass(oracle, f, m):
    # |M|^2 = A_V (2 - beta^2 (1 - c^2)) + A_A beta^2 (1 + c^2) + B beta c:
    # the c^2 coefficient is beta^2 times the massless A = A_V + A_A, the
    # c-odd part beta times the massless one
    s = 91.2 ** 2
    beta = np.sqrt(1 - 4 * m * m / s)
    cs = np.linspace(-1, 1, 11)
    M = np.array([oracle.me2_massive(f, s, c, m) for c in cs])
    M0 = np.array([oracle.me2(f, s, c) for c in cs])
    even, odd = 0.5 * (M + M[::-1]), 0.5 * (M - M[::-1])
    even0, odd0 = 0.5 * (M0 + M0[::-1]), 0.5 * (M0 - M0[::-1])
    a = even[5]
    b2 = (even - a) / np.where(cs != 0, cs * cs, 1)
    A0 = even0[5]
    np.testing.assert_allclose(b2[cs != 0], beta * beta * A0, rtol=1e-12)
    np.testing.assert_allclose(odd[6:], beta * odd0[6:], rtol=1e-12)
    assert oracle.me2_massive(f, s, 0.3, 0.0) == oracle.me2(f, s, 0.3)


def _gamma():
    I2, Z2 = np.eye(2), np.zeros((2, 2))
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    g0 = np.block([[I2, Z2], [Z2, -I2]]).astype(complex)
    gs = [np.block([[Z2, s_], [-s_, Z2]]).astype(complex) for s_ in sig]
    g = [g0, *gs]
    g5 = 1j * g[0] @ g[1] @ g[2] @ g[3]
    return g, g5


def _spin_summed(k1, k2, p1, p2, m, cpl):
    """sum over spins of |M|^2 for e-(k1) e+(k2) -> Q(p1) Qbar(p2) by Dirac
    traces: currents with couplings (v, a) per exchange, propagator factors
    P; cpl = [(P, ve, ae, vf, af), ...]."""
    g, g5 = _gamma()
    metric = np.diag([1.0, -1.0, -1.0, -1.0])
    sl = lambda q: sum(metric[mu, mu] * q[mu] * g[mu] for mu in range(4))
    one = np.eye(4)
    total = 0.0
    for (P1, ve1, ae1, vf1, af1) in cpl:
        for (P2, ve2, ae2, vf2, af2) in cpl:
            L = np.empty((4, 4), complex)
            H = np.empty((4, 4), complex)
            for mu in range(4):
                for nu in range(4):
                    L[mu, nu] = np.trace(sl(k2) @ g[mu] @ (ve1 * one - ae1 * g5) @ sl(k1) @ g[nu]
                                         @ (ve2 * one - ae2 * g5))
                    H[mu, nu] = np.trace((sl(p1) + m * one) @ g[mu] @ (vf1 * one - af1 * g5)
                                         @ (sl(p2) - m * one) @ g[nu] @ (vf2 * one - af2 * g5))
            total += P1 * np.conj(P2) * np.einsum("mn,ma,nb,ab->", L, metric, metric, H)
    return total.real


def test_massive_me_against_dirac_traces(oracle):
    # the massive angular structure from an explicit spin sum over gamma and Z
    # exchange, relative to the massless one at the same angle
    s = 91.2 ** 2
    mz, gz = 91.1876, 2.4952
    sw2 = 1 - (80.385 / mz) ** 2
    kappa = 1 / (4 * sw2 * (1 - sw2))
    pz = kappa * s / (s - mz * mz + 1j * mz * gz)
    e = np.sqrt(s) / 2
    k1, k2 = np.array([e, 0, 0, e]), np.array([e, 0, 0, -e])
    for f, m in ((5, 30.0), (4, 20.0)):
        qf, t3 = (-1 / 3, -0.5) if f == 5 else (2 / 3, 0.5)
        cpl = [(-1.0 * qf, 1.0, 0.0, 1.0, 0.0), (pz, -0.5 + 2 * sw2, -0.5, t3 - 2 * qf * sw2, t3)]
        beta = np.sqrt(1 - 4 * m * m / s)
        for c in (-0.8, -0.1, 0.4, 0.95):
            st = np.sqrt(1 - c * c)
            n = np.array([st, 0, c])
            p1, p2 = np.array([e, *(beta * e * n)]), np.array([e, *(-beta * e * n)])
            q1, q2 = np.array([e, *(e * n)]), np.array([e, *(-e * n)])
            ratio = _spin_summed(k1, k2, p1, p2, m, cpl) / _spin_summed(k1, k2, q1, q2, 0.0, cpl)
            assert oracle.me2_massive(f, s, c, m) / oracle.me2(f, s, c) == pytest.approx(ratio, rel=1e-9)


def test_me_weights_and_thresholds(oracle):
    # below 2 m_b no b quarks, and the weights average to sigma over the open flavours
    for ecm, open_ in ((9.0, {1, 2, 3, 4}), (91.2, {1, 2, 3, 4, 5})):
        n = 100_000
        r = oracle.generate(3, 0, n, ecm, 1e9, 2, mass=MASS)  # t_C above s: ME only
        assert set(np.unique(r["sum_i"][:, 4])) == open_
        w = r["sum_d"][:, 0]
        sig = oracle.sigma_lo_massive(ecm * ecm, MASS)
        assert abs(w.mean() - sig) < 4 * w.std() / np.sqrt(n)
    assert oracle.sigma_lo_massive(91.2 ** 2, np.zeros(6)) == pytest.approx(oracle.sigma_lo(91.2 ** 2), rel=1e-14)


def test_me_momenta_on_shell(oracle):
    for ev in range(200):
        f, c, ph, w, p = oracle.me_event_massive(11, ev, 20.0, MASS)
        m = MASS[f]
        for q in p:
            assert mdot(q, q) == pytest.approx(m * m, abs=1e-12 * 400)
        np.testing.assert_allclose(p.sum(0), [20.0, 0, 0, 0], atol=1e-13 * 20)


# ---------------------------------------------------------------------------
# massive map
# ---------------------------------------------------------------------------
def _pair(rng, Q2, ma, mb):
    """Back-to-back momenta of masses ma, mb with (pa + pb)^2 = Q2, random
    direction, boosted along a random axis."""
    E = np.sqrt(Q2)
    pa_abs = np.sqrt(kallen(Q2, ma * ma, mb * mb)) / (2 * E)
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    pa = np.array([np.sqrt(pa_abs ** 2 + ma * ma), *(pa_abs * v)])
    pb = np.array([np.sqrt(pa_abs ** 2 + mb * mb), *(-pa_abs * v)])
    bvec = rng.normal(size=3)
    bvec *= rng.uniform(0, 0.8) / np.linalg.norm(bvec)
    g = 1 / np.sqrt(1 - bvec @ bvec)

    def boost(p):
        bp = bvec @ p[1:]
        e = g * (p[0] + bp)
        x = p[1:] + ((g - 1) * bp / (bvec @ bvec) + g * p[0]) * bvec
        return np.array([e, *x])

    return boost(pa), boost(pb)


CASES = [  # (name, mi, mj, mk, mij)
    ("Q -> Q g, massive spectator", 4.8, 0.0, 4.8, 4.8),
    ("Q -> Q g, massless spectator", 1.5, 0.0, 0.0, 1.5),
    ("q -> q g, massive spectator", 0.0, 0.0, 4.8, 0.0),
    ("g -> Q Qbar, massless spectator", 1.5, 1.5, 0.0, 0.0),
    ("g -> Q Qbar, massive spectator", 4.8, 4.8, 1.5, 0.0),
]


@pytest.mark.parametrize("name,mi,mj,mk,mij", CASES)
def test_massive_map_invariants(oracle, name, mi, mj, mk, mij):
    rng = np.random.default_rng(7)
    done = 0
    while done < 300:
        Q2 = rng.uniform(30, 60) ** 2
        pij, pk = _pair(rng, Q2, mij, mk)
        qb2 = Q2 - mi * mi - mj * mj - mk * mk
        z = rng.uniform(0.02, 0.98)
        y = rng.uniform(1e-3, 0.9)
        t = y * qb2 * z * (1 - z) - (1 - z) ** 2 * mi * mi - z * z * mj * mj
        if t <= 0 or oracle.massive_ratio(0 if mij > 0 else 11, t, z, Q2, mi, mj, mk, 1.0) < 0:
            continue  # outside the phase space
        phi = rng.uniform(0, 2 * np.pi)
        a, j, k = oracle.split_kinematics_massive(pij, pk, mi, mj, mk, mij, t, z, phi)
        sc = np.sqrt(Q2)
        np.testing.assert_allclose(a + j + k, pij + pk, atol=1e-12 * sc)
        for v, m in ((a, mi), (j, mj), (k, mk)):
            assert mdot(v, v) == pytest.approx(m * m, abs=1e-10 * Q2)
            assert v[0] > 0
        pij_, pik, pjk = mdot(a, j), mdot(a, k), mdot(j, k)
        assert pij_ / (pij_ + pik + pjk) == pytest.approx(y, rel=1e-9)
        assert pik / (pik + pjk) == pytest.approx(z, rel=1e-9)
        if mk == 0:  # then t is the transverse momentum of i relative to p_ij and p_k
            P = mdot(a + j, k)
            kt = a - (pik / P) * (a + j) - ((mdot(a, a + j) - (pik / P) * mdot(a + j, a + j)) / P) * k
            assert -mdot(kt, kt) == pytest.approx(t, rel=1e-7)
        done += 1


@pytest.mark.parametrize("name,mi,mj,mk,mij", CASES)
def test_massive_map_dalitz_jacobian(oracle, name, mi, mj, mk, mij):
    # the map covers the Dalitz plot with ds_ij ds_jk = Qb2^2 (1 - y) dy dz:
    # finite differences of the invariants of the mapped momenta
    rng = np.random.default_rng(8)
    Q2 = 45.0 ** 2
    pij, pk = _pair(rng, Q2, mij, mk)
    qb2 = Q2 - mi * mi - mj * mj - mk * mk

    def inv(y, z):
        t = y * qb2 * z * (1 - z) - (1 - z) ** 2 * mi * mi - z * z * mj * mj
        a, j, k = oracle.split_kinematics_massive(pij, pk, mi, mj, mk, mij, t, z, 0.7)
        return np.array([mdot(a + j, a + j), mdot(j + k, j + k)])

    for y, z in ((0.3, 0.4), (0.1, 0.7), (0.6, 0.5)):
        h = 1e-6
        dy = (inv(y + h, z) - inv(y - h, z)) / (2 * h)
        dz = (inv(y, z + h) - inv(y, z - h)) / (2 * h)
        jac = abs(dy[0] * dz[1] - dy[1] * dz[0])
        assert jac == pytest.approx(qb2 * qb2 * (1 - y), rel=1e-6)


@pytest.mark.parametrize("name,mi,mj,mk,mij", CASES)
def test_massive_map_at_the_phase_space_edge(oracle, name, mi, mj, mk, mij):
    """At the edges of the Dalitz region the map's transverse momentum squared
    (lower edge in t) or the Kallen function of the rescaled spectator (upper
    edge, with a massive spectator; y -> 1 without one) reaches zero, and a
    rounding can take it just below.  The reading: the map then takes it as
    zero, the value at the edge.  Just outside the edge (by one bisection step
    in t) the momenta are finite, conserve the dipole's momentum, sit on
    their mass shells and agree with those just inside."""
    rng = np.random.default_rng(10)
    K = 0 if mij > 0 else 11
    for _ in range(20):
        Q2 = rng.uniform(30, 60) ** 2
        pij, pk = _pair(rng, Q2, mij, mk)
        qb2 = Q2 - mi * mi - mj * mj - mk * mk
        z = rng.uniform(0.2, 0.8)
        t_of = lambda y: y * qb2 * z * (1 - z) - (1 - z) ** 2 * mi * mi - z * z * mj * mj
        inside = lambda t: oracle.massive_ratio(K, t, z, Q2, mi, mj, mk, 1.0) >= 0.0
        t_in = t_of(0.3)
        assert inside(t_in)
        # below the lower edge, and above the upper one where a massive
        # spectator bounds it (without a spectator mass the upper edge is
        # y = 1, where the spectator's momentum vanishes and the map's p_k
        # coefficient diverges; the (1 - y) factor gives it no weight)
        for y_out in ((-1.0, 1.5) if mk > 0 else (-1.0,)):
            lo, hi = t_in, t_of(y_out)
            assert not inside(hi)
            for _ in range(200):  # bisect to the edge: lo inside, hi outside
                mid = 0.5 * (lo + hi)
                if mid == lo or mid == hi:
                    break
                lo, hi = (mid, hi) if inside(mid) else (lo, mid)
            phi = rng.uniform(0, 2 * np.pi)
            a_in = oracle.split_kinematics_massive(pij, pk, mi, mj, mk, mij, lo, z, phi)
            a_out = oracle.split_kinematics_massive(pij, pk, mi, mj, mk, mij, hi, z, phi)
            sc = np.sqrt(Q2)
            for v_in, v_out, m in zip(a_in, a_out, (mi, mj, mk)):
                assert np.all(np.isfinite(v_out))
                assert mdot(v_out, v_out) == pytest.approx(m * m, abs=1e-9 * Q2)
                # continuous across the edge (the spectator's rescaling goes
                # as the square root of the Kallen function there)
                np.testing.assert_allclose(v_out, v_in, atol=1e-4 * sc)
            np.testing.assert_allclose(sum(a_out), pij + pk, atol=1e-12 * sc)


def test_massive_map_reduces_to_the_massless_one(oracle):
    rng = np.random.default_rng(9)
    for _ in range(200):
        pij, pk = _pair(rng, rng.uniform(20, 80) ** 2, 0.0, 0.0)
        q2 = 2 * mdot(pij, pk)
        z, y = rng.uniform(0.05, 0.95), rng.uniform(0.01, 0.9)
        t = y * q2 * z * (1 - z)
        phi = rng.uniform(0, 2 * np.pi)
        m = oracle.split_kinematics_massive(pij, pk, 0.0, 0.0, 0.0, 0.0, t, z, phi)
        o = oracle.split_kinematics(pij, pk, t, z, phi)
        for u, v in zip(m, o):
            np.testing.assert_allclose(u, v, atol=1e-11 * pij[0])


# ---------------------------------------------------------------------------
# kernels: the soft limit is the massive eikonal factor
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m", [1.5, 4.8, 12.0])
def test_soft_limit_is_the_massive_eikonal(oracle, m):
    # a soft gluon j off a Q Qbar pair: the two dipole ends (Q with spectator
    # Qbar, Qbar with spectator Q), each V / (2 p_i.p_j), add up to half the
    # eikonal factor C_F [2 p_i.p_k/(p_i.q p_k.q) - m^2/(p_i.q)^2 - m^2/(p_k.q)^2]
    rng = np.random.default_rng(10)
    ecm = 40.0
    for _ in range(50):
        pq, pqb = _pair(rng, ecm * ecm, m, m)
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        w = 1e-5 * ecm
        q = np.array([w, *(w * v)])
        total = 0.0
        for pi, pk in ((pq, pqb), (pqb, pq)):
            sig = mdot(pi, q) + mdot(pi, pk) + mdot(q, pk)
            y = mdot(pi, q) / sig
            z = mdot(pi, pk) / (mdot(pi, pk) + mdot(q, pk))
            qb2 = 2 * sig
            sij = mdot(pi + q, pi + q)
            total += oracle.kernel_value_massive(0, z, y, m, qb2, sij) / (2 * mdot(pi, q))
        eik = CF * (2 * mdot(pq, pqb) / (mdot(pq, q) * mdot(pqb, q)) - m * m / mdot(pq, q) ** 2
                    - m * m / mdot(pqb, q) ** 2)
        assert total == pytest.approx(0.5 * eik, rel=1e-3)


def test_massive_kernels_never_exceed_their_overestimates(oracle):
    rng = np.random.default_rng(11)
    for _ in range(20000):
        K = int(rng.choice([0, 4, 10, 14, 15]))
        mi = {0: 1.5, 4: 4.8, 10: 0.0, 14: 1.5, 15: 4.8}[K]
        mj = mi if K > 10 else 0.0
        mk = rng.choice([0.0, 1.5, 4.8])
        Q2 = rng.uniform(12, 100) ** 2
        z, t = rng.uniform(0, 1), np.exp(rng.uniform(np.log(0.3), np.log(Q2 / 4)))
        f = oracle.massive_flux(Q2, mi, mj, mk, mi if K < 10 else 0.0)
        r = oracle.massive_ratio(K, t, z, Q2, mi, mj, mk, max(f, 1.0))
        assert r <= 1.0 + 1e-12


def test_massive_events_are_valid(oracle):
    # every event reaches the cutoff on its mass shells, conserving momentum,
    # with consistent colour lines; heavy quarks radiate less (dead cone)
    for ecm, tc in ((91.2, 1.0), (500.0, 0.25)):
        r = oracle.generate(13, 0, 600, ecm, tc, 256, records=True, mass=MASS)
        assert (r["sum_i"][:, 1] == 1).all()
        rec = r["rec"]
        for e in range(600):
            n = rec["n"][e]
            p, pid = rec["p"][e, :n], rec["pid"][e, :n]
            np.testing.assert_allclose(p.sum(0), [ecm, 0, 0, 0], atol=1e-10 * ecm)
            for q, f in zip(p, pid):
                mm = 0.0 if f == 21 else MASS[abs(f)]
                assert mdot(q, q) == pytest.approx(mm * mm, abs=1e-10 * ecm * ecm)
            assert sorted(c for c in rec["col"][e, :n] if c) == sorted(c for c in rec["acol"][e, :n] if c)
    light = oracle.generate(14, 0, 3000, 91.2, 1.0, 64, mass=MASS)
    fl, ne = light["sum_i"][:, 4], light["sum_i"][:, 3]
    assert ne[fl == 5].mean() < ne[fl <= 3].mean() - 0.3


def test_massless_limit_of_the_shower(oracle):
    # tiny masses take the massive formulas everywhere (every kernel with a c
    # or b quark) and give the massless events
    tiny = np.array([0.0, 0.0, 0.0, 0.0, 1e-6, 1e-6])
    a = oracle.generate(12, 0, 400, 91.2, 1.0, 64, records=True)
    b = oracle.generate(12, 0, 400, 91.2, 1.0, 64, records=True, mass=tiny)
    same = (a["sum_i"][:, :5] == b["sum_i"][:, :5]).all(1) & (a["hash"] == b["hash"])
    assert same.mean() > 0.99
    heavy = a["sum_i"][:, 4] >= 4
    assert heavy.sum() > 100 and same[heavy].mean() > 0.99
    for e in np.flatnonzero(same):
        n = a["rec"]["n"][e]
        np.testing.assert_allclose(b["rec"]["p"][e, :n], a["rec"]["p"][e, :n], atol=1e-8 * 91.2)


# ---------------------------------------------------------------------------
# the veto algorithm with masses against the emission density
# ---------------------------------------------------------------------------
def _alpha_s(t):
    b0 = 23.0 / (12 * np.pi)
    return 0.118 / (1 + 0.118 * b0 * np.log(t / 91.1876 ** 2))


def _dalitz_ok(Q2, mi, mj, mk, y, z):
    """(y, z) inside the Dalitz plot of Q -> i j k (PDG limits of s_jk at fixed s_ij)."""
    qb2 = Q2 - mi * mi - mj * mj - mk * mk
    sij = mi * mi + mj * mj + y * qb2
    sjk = mj * mj + mk * mk + (1 - z) * (1 - y) * qb2
    if not (sij > (mi + mj) ** 2 and np.sqrt(sij) + mk < np.sqrt(Q2)):
        return False
    r = np.sqrt(sij)
    e2 = (sij - mi * mi + mj * mj) / (2 * r)
    e3 = (Q2 - sij - mk * mk) / (2 * r)
    a, b = np.sqrt(max(e2 * e2 - mj * mj, 0)), np.sqrt(max(e3 * e3 - mk * mk, 0))
    return (e2 + e3) ** 2 - (a + b) ** 2 <= sjk <= (e2 + e3) ** 2 - (a - b) ** 2


def _density(t, Q2, m, mk):
    """dP/dt of one Q -> Q g end from the Dalitz-plot measure:
    dPhi_3/dPhi_2 = ds_ij ds_jk / (16 pi^2 sqrt(lambda(Q2, m^2, mk^2))), the
    dipole term 8 pi alpha_s V / (2 p_i.p_j), and at fixed z
    ds_ij ds_jk = Qb2^2 (1 - y) dy dz with dy = dt / (Qb2 z (1 - z))."""
    qb2 = Q2 - m * m - mk * mk
    lam = np.sqrt(kallen(Q2, m * m, mk * mk))

    def f(z):
        y = (t + (1 - z) ** 2 * m * m) / (qb2 * z * (1 - z))
        if not (0 < y < 1) or not _dalitz_ok(Q2, m, 0.0, mk, y, z):
            return 0.0
        sij = m * m + y * qb2
        v = max(0.0, CF * (2 / (1 - z * (1 - y)) - (1 + z) - 2 * m * m / (y * qb2)))
        pipj = 0.5 * y * qb2
        return (8 * np.pi * _alpha_s(t) * v / (2 * pipj)) * qb2 * qb2 * (1 - y) / (qb2 * z * (1 - z)) \
            / (16 * np.pi ** 2 * lam)

    zs = np.linspace(1e-6, 1 - 1e-6, 4001)
    vals = np.array([f(z) for z in zs])
    return integrate.simpson(vals, x=zs)


def test_first_emission_off_a_heavy_pair(oracle):
    # b bbar at sqrt(s) = 20 GeV with m_b = 8 GeV (beta = 0.6): two Q -> Q g
    # ends with a massive spectator; the first emission's t against
    # Delta(t) = exp(-int_t^tmax 2 rho)
    mass = np.array([0.0, 0.0, 0.0, 0.0, 1.5, 8.0])
    ecm, tc, n = 20.0, 1.0, 30_000
    s = ecm * ecm
    m = 8.0
    grid = np.exp(np.linspace(np.log(tc), np.log(s / 4), 400))
    rho = np.array([2 * _density(t, s, m, m) for t in grid])
    lg = np.log(grid)
    cum = np.concatenate([[0], np.cumsum(0.5 * (rho[1:] * grid[1:] + rho[:-1] * grid[:-1]) * np.diff(lg))])
    expo = cum[-1] - cum
    edges = grid[::40]
    cdf = np.exp(-np.interp(np.log(edges), lg, expo))
    ts = np.zeros(n)
    for e in range(n):
        # every event starts from b bbar, along the direction the ME drew
        f, c, ph, w, p = oracle.me_event_massive(41, e, ecm, mass)
        beta = np.sqrt(1 - 4 * m * m / s)
        pz = 0.5 * ecm * beta
        v = p[0, 1:] / np.linalg.norm(p[0, 1:])
        pb = np.array([[0.5 * ecm, *(pz * v)], [0.5 * ecm, *(-pz * v)]])
        r = oracle.shower(41, e, ecm, tc, pb, [5, -5], [1, 0], [0, 1], cap=4, max_emit=1, max_log=1, mass=mass)
        ts[e] = r["log"][0, 0] if r["n_emit"] else 0.0
    exp = np.concatenate([[cdf[0]], np.diff(cdf)]) * n
    idx = np.where(ts > 0, np.searchsorted(edges, ts), 0)
    cnt = np.bincount(idx, minlength=len(edges))[:len(edges)]
    ok = exp > 5
    chi2 = ((cnt[ok] - exp[ok]) ** 2 / exp[ok]).sum()
    ndf = int(ok.sum())
    assert chi2 < ndf + 5 * np.sqrt(2 * ndf), (chi2, ndf)
    assert cdf[0] > 0.3  # the dead cone: a heavy slow pair radiates little
