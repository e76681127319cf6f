"""Pins of the oracle's observables: three-parton closed forms, brute-force
thrust over every hemisphere split, the C-parameter from the eigenvalues of
the linearised momentum tensor, invariances, and the histogram bookkeeping."""
import itertools

import numpy as np
import pytest


def three_partons(rng, ecm):
    """Random massless 3-body final state with random orientation."""
    while True:
        x1, x2 = rng.uniform(0, 1, 2)
        x3 = 2 - x1 - x2
        if x3 <= 0 or x3 >= 1 or x1 + x2 <= 1:
            continue
        break
    x = np.array([x1, x2, x3])
    E = x * ecm / 2
    c12 = 1 - 2 * (1 - x3) / (x1 * x2)
    s12 = np.sqrt(max(0.0, 1 - c12 * c12))
    p1 = np.array([0, 0, E[0]])
    p2 = np.array([E[1] * s12, 0, E[1] * c12])
    p3 = -p1 - p2
    R = random_rotation(rng)
    P = np.array([[E[0], *(R @ p1)], [E[1], *(R @ p2)], [E[2], *(R @ p3)]])
    return x, P


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_three_parton_closed_forms(oracle):
    rng = np.random.default_rng(2)
    ecm = 91.2
    s = ecm * ecm
    for _ in range(500):
        x, P = three_partons(rng, ecm)
        T, axis = oracle.thrust(P)
        assert T == pytest.approx(x.max(), rel=1e-12)
        o = oracle.observables(P, ecm)
        y23, y34, tau, C, rho, bt, bw = o
        assert tau == pytest.approx(1 - x.max(), abs=1e-12)
        assert rho == pytest.approx(1 - x.max(), abs=1e-12)
        assert C == pytest.approx(6 * np.prod(1 - x) / np.prod(x), rel=1e-9, abs=1e-14)
        assert y34 == 0.0
        E = x * ecm / 2
        ys = []
        for i, j in ((0, 1), (0, 2), (1, 2)):
            k = 3 - i - j
            ys.append(min(E[i], E[j]) / max(E[i], E[j]) * (1 - x[k]))
        assert y23 == pytest.approx(min(ys), rel=1e-9)
        # B_T = B_W = p_T / sqrt(s): the soft pair's transverse momentum to the thrust axis
        h = int(np.argmax(x))
        o1, o2 = [i for i in range(3) if i != h]
        c = 1 - 2 * (1 - x[o2]) / (x[h] * x[o1])
        pt = E[o1] * np.sqrt(max(0.0, 1 - c * c))
        assert bt == pytest.approx(pt / ecm, rel=1e-8, abs=1e-13)
        assert bw == pytest.approx(pt / ecm, rel=1e-8, abs=1e-13)


def brute_thrust(P):
    p = P[:, 1:]
    best = 0.0
    n = len(p)
    for signs in itertools.product((1.0, -1.0), repeat=n - 1):
        v = p[0] + np.array(signs) @ p[1:]
        best = max(best, np.linalg.norm(v))
    return best / np.linalg.norm(p, axis=1).sum()


def test_thrust_equals_brute_force_on_showered_events(oracle):
    r = oracle.generate(4, 0, 400, 500.0, 0.25, 64, records=True)
    checked = 0
    for e in range(400):
        n = r["rec"]["n"][e]
        if n < 3 or n > 13:
            continue
        P = r["rec"]["p"][e, :n]
        T, _ = oracle.thrust(P)
        assert T == pytest.approx(brute_thrust(P), rel=1e-12)
        checked += 1
    assert checked > 100


def test_thrust_equals_brute_force_random(oracle):
    rng = np.random.default_rng(9)
    for n in range(3, 11):
        for _ in range(20):
            p3 = rng.normal(size=(n, 3)) * rng.uniform(0.1, 5, size=(n, 1))
            P = np.concatenate([np.linalg.norm(p3, axis=1, keepdims=True), p3], axis=1)
            T, axis = oracle.thrust(P)
            assert T == pytest.approx(brute_thrust(P), rel=1e-12)
            # the axis realises the thrust value
            val = np.abs(P[:, 1:] @ axis).sum() / np.linalg.norm(P[:, 1:], axis=1).sum()
            assert val == pytest.approx(T, rel=1e-12)


def test_cparameter_from_eigenvalues(oracle):
    r = oracle.generate(5, 0, 300, 200.0, 0.5, 64, records=True)
    for e in range(300):
        n = r["rec"]["n"][e]
        P = r["rec"]["p"][e, :n]
        p = P[:, 1:]
        mod = np.linalg.norm(p, axis=1)
        theta = (p[:, :, None] * p[:, None, :] / mod[:, None, None]).sum(0) / mod.sum()
        lam = np.linalg.eigvalsh(theta)
        c_ref = 3 * (lam[0] * lam[1] + lam[1] * lam[2] + lam[2] * lam[0])
        assert oracle.cparameter(P) == pytest.approx(max(c_ref, 0.0), abs=1e-12)


def test_observables_rotation_and_permutation_invariant(oracle):
    r = oracle.generate(6, 0, 200, 91.2, 1.0, 64, records=True)
    rng = np.random.default_rng(3)
    for e in range(200):
        n = r["rec"]["n"][e]
        if n < 3:
            continue
        P = r["rec"]["p"][e, :n].copy()
        o = oracle.observables(P, 91.2)
        R = random_rotation(rng)
        Q = P.copy()
        Q[:, 1:] = P[:, 1:] @ R.T
        Q = Q[rng.permutation(n)]
        o2 = oracle.observables(Q, 91.2)
        np.testing.assert_allclose(o2, o, rtol=1e-9, atol=1e-13)


def test_hemisphere_masses_brute_force(oracle):
    r = oracle.generate(8, 0, 300, 91.2, 1.0, 64, records=True)
    for e in range(300):
        n = r["rec"]["n"][e]
        if n < 3:
            continue
        P = r["rec"]["p"][e, :n]
        T, axis = oracle.thrust(P)
        side = P[:, 1:] @ axis >= 0
        m2 = []
        for sel in (side, ~side):
            q = P[sel].sum(0)
            m2.append(q[0] ** 2 - q[1:] @ q[1:])
        rho, bt, bw = oracle.hemispheres(P, axis, 91.2 ** 2)
        assert rho == pytest.approx(max(max(m2) / 91.2 ** 2, 0.0), abs=1e-12)


def test_histograms_account_for_every_done_event(oracle):
    r = oracle.generate(1, 0, 2000, 91.2, 1.0, 64)
    h = r["hist"]
    done = r["sum_i"][:, 1] == 1
    w = r["sum_d"][:, 0]
    for o in range(oracle.NOBS):
        assert h[o, :, 2].sum() == done.sum()
        assert h[o, :, 0].sum() == pytest.approx(w[done].sum(), rel=1e-12)
        assert h[o, :, 1].sum() == pytest.approx((w[done] ** 2).sum(), rel=1e-12)
    # log10 y23 underflow holds exactly the events with fewer than 3 partons plus y23 < 10^-4.3
    y23 = r["sum_d"][:, 2]
    under = done & ((y23 <= 0) | (np.log10(np.where(y23 > 0, y23, 1)) < -4.3) & (y23 > 0))
    assert h[0, 0, 2] == under.sum()


def test_split_ranges_reproduce_the_serial_run(oracle):
    whole = oracle.generate(1, 0, 600, 91.2, 1.0, 64)
    parts = [oracle.generate(1, a, 200, 91.2, 1.0, 64) for a in (0, 200, 400)]
    np.testing.assert_array_equal(np.concatenate([p["sum_i"] for p in parts]), whole["sum_i"])
    np.testing.assert_array_equal(np.concatenate([p["sum_d"] for p in parts]), whole["sum_d"])
    np.testing.assert_array_equal(np.concatenate([p["hash"] for p in parts]), whole["hash"])
    np.testing.assert_allclose(sum(p["hist"] for p in parts), whole["hist"], rtol=1e-13)


def rambo(rng, n, ecm):
    """n massless momenta with total (ecm, 0, 0, 0), flat in phase space
    (Kleiss, Stirling and Ellis, the RAMBO construction)."""
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


def durham_y(pa, pb, s):
    """2 min(E_a, E_b)^2 (1 - cos theta_ab) / s, the Durham measure."""
    ua, ub = pa[1:], pb[1:]
    cos = ua @ ub / np.sqrt((ua @ ua) * (ub @ ub))
    return 2 * min(pa[0], pb[0]) ** 2 * (1 - cos) / s


@pytest.mark.parametrize("seed", range(3))
def test_durham_four_partons_brute_force(oracle, seed):
    # four partons: y34 is the smallest pair measure; merging that pair by
    # adding four-momenta (E-scheme) leaves three jets whose smallest pair
    # measure is y23
    rng = np.random.default_rng(seed)
    ecm = 91.2
    s = ecm * ecm
    for _ in range(100):
        p = rambo(rng, 4, ecm)
        assert abs(p[:, 0].sum() - ecm) < 1e-9 and np.abs(p[:, 1:].sum(axis=0)).max() < 1e-9
        pairs = list(itertools.combinations(range(4), 2))
        ys = [durham_y(p[a], p[b], s) for a, b in pairs]
        k = int(np.argmin(ys))
        a, b = pairs[k]
        rest = [p[c] for c in range(4) if c not in (a, b)]
        jets = [p[a] + p[b]] + rest
        y23 = min(durham_y(jets[u], jets[v], s) for u, v in itertools.combinations(range(3), 2))
        g23, g34 = oracle.durham(p, s)
        assert g34 == pytest.approx(ys[k], rel=1e-11)
        assert g23 == pytest.approx(y23, rel=1e-11)
