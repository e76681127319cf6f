"""Pins of the oracle's alpha_s, splitting kernels and LO matrix element
against closed forms, textbook limits and independent quadrature."""
import os

import numpy as np
import pytest
from scipy import integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "derived_physics.txt")


def golden(kind):
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = line.split()
            if w[0] == kind:
                out.append([float(x) for x in w[1:]])
    return out


MZ = 91.1876


def test_golden_file_is_the_scripts_output():
    """The committed closed-form and quadrature values are exactly what the
    script next to them writes (numpy and scipy only, no oracle)."""
    import subprocess
    import sys

    script = os.path.join(os.path.dirname(GOLDEN), "make_derived_physics.py")
    assert subprocess.run([sys.executable, script, "--check"], timeout=300).returncode == 0


def test_alpha_s_values(oracle):
    for t, ref in golden("alpha_s"):
        assert oracle.alpha_s(t) == pytest.approx(ref, abs=1.5e-6)
    assert oracle.alpha_s(MZ * MZ) == pytest.approx(0.118, abs=1e-15)


def test_alpha_s_one_loop_rge(oracle):
    # d alpha / d ln t = -b0 alpha^2 with b0 = (33 - 2 n_f)/(12 pi), n_f = 5
    b0 = 23.0 / (12 * np.pi)
    for t in (0.3, 1.0, 10.0, 1e3, 1e5):
        h = 1e-4
        d = (oracle.alpha_s(t * np.exp(h)) - oracle.alpha_s(t * np.exp(-h))) / (2 * h)
        a = oracle.alpha_s(t)
        assert d == pytest.approx(-b0 * a * a, rel=1e-7)


QG = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9]
CF, CA, TR = 4 / 3, 3.0, 0.5


def test_kernel_lists(oracle):
    for f in range(1, 6):
        assert oracle.kernel_list(f) == [f - 1]
        assert oracle.kernel_list(-f) == [4 + f]
    assert oracle.kernel_list(21) == [10, 11, 12, 13, 14, 15]


def test_kernels_collinear_limit_is_dglap(oracle):
    # y -> 0: q->qg gives the textbook C_F (1+z^2)/(1-z); the gluon's two dipole
    # ends summed and symmetrised give P_gg/2 (identical gluons) and P_qg.
    zs = np.linspace(0.01, 0.99, 37)
    for z in zs:
        for K in QG:
            assert oracle.kernel_value(K, z, 0.0) == pytest.approx(CF * (1 + z * z) / (1 - z), rel=1e-13)
        gg = lambda x: 2 * oracle.kernel_value(10, x, 0.0)
        pgg = 2 * CA * (z / (1 - z) + (1 - z) / z + z * (1 - z))
        assert 0.5 * (gg(z) + gg(1 - z)) == pytest.approx(pgg / 2, rel=1e-12)
        for K in range(11, 16):
            qq = lambda x: 2 * oracle.kernel_value(K, x, 0.0)
            assert 0.5 * (qq(z) + qq(1 - z)) == pytest.approx(TR * (z * z + (1 - z) ** 2), rel=1e-13)


def _mdot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def _null(rng, e):
    u = rng.normal(size=3)
    return np.array([e, *(e * u / np.linalg.norm(u))])


def _end_vars(pe, pj, ps):
    """(z, y) of the end with emitter pe, emission pj, spectator ps from the
    final momenta (the inverse of the dipole map): y = pe.pj / (pe.pj + pe.ps
    + pj.ps), z = pe.ps / (pe.ps + pj.ps)."""
    ej, es, js = _mdot(pe, pj), _mdot(pe, ps), _mdot(pj, ps)
    return es / (es + js), ej / (ej + es + js)


@pytest.mark.parametrize("lam", [1e-3, 1e-4, 1e-5])
def test_soft_limit_of_two_ends_is_eikonal(oracle, lam):
    """A soft gluon j radiated inside the colour dipole (i, k): the two ends'
    dipole terms V_{ij,k}/(p_i.p_j) + V_{kj,i}/(p_k.p_j) add up to the
    eikonal factor C 2 p_i.p_k / ((p_i.p_j)(p_j.p_k)), C = C_F for a quark
    dipole (two q -> q g ends) and C_A/2 for a dipole between two gluons (two
    g -> g g ends, as for a soft gluon between the gluons of a q g g qbar
    chain): the soft limit of the QCD matrix element that the kernels must
    reproduce away from y = 0, which the collinear pin does not reach.
    Corrections are of relative order lambda."""
    rng = np.random.default_rng(int(1 / lam))
    for _ in range(200):
        pi, pk = _null(rng, rng.uniform(10, 45)), _null(rng, rng.uniform(10, 45))
        pj = _null(rng, lam * 45.0)
        # the expansion parameter is p_j.p_k / p_i.p_k (and i <-> k): keep the
        # dipole wide open, 1 - cos(theta_ik) > 1/2
        if _mdot(pi, pk) < 0.5 * pi[0] * pk[0]:
            continue
        eik = 2 * _mdot(pi, pk) / (_mdot(pi, pj) * _mdot(pj, pk))
        zi, yi = _end_vars(pi, pj, pk)
        zk, yk = _end_vars(pk, pj, pi)
        for K_i, K_k, C in [(0, 5, CF), (3, 8, CF), (10, 10, CA / 2)]:
            d = oracle.kernel_value(K_i, zi, yi) / _mdot(pi, pj) + oracle.kernel_value(K_k, zk, yk) / _mdot(pk, pj)
            assert d / (C * eik) == pytest.approx(1.0, abs=60 * lam), (K_i, K_k)


def test_overestimates_bound_kernels(oracle):
    # 0 <= V(z, y) (1 - y) <= O(z) on a dense grid
    for K in (0, 7, 10, 11, 15):
        for z in np.linspace(1e-4, 1 - 1e-4, 101):
            for y in np.linspace(0.0, 1.0, 41):
                v = oracle.kernel_value(K, z, y) * (1 - y)
                assert v >= 0.0
                assert v <= oracle.kernel_over(K, z) * (1 + 1e-14)


@pytest.mark.parametrize("K", [0, 6, 10, 13])
@pytest.mark.parametrize("tq", [1e-3, 0.05, 0.2])
def test_overestimate_integral_and_inverse(oracle, K, tq):
    zp = 0.5 * (1 + np.sqrt(1 - 4 * tq))
    zm = 1 - zp
    I_num, _ = integrate.quad(lambda z: oracle.kernel_over(K, z), zm, zp, epsabs=0, epsrel=1e-12, limit=200)
    assert oracle.kernel_integral(K, zm, zp) == pytest.approx(I_num, rel=1e-10)
    for u in (1e-9, 0.1, 0.37, 0.5, 0.9, 1 - 1e-9):
        z = oracle.kernel_zgen(K, zm, zp, u)
        assert zm <= z <= zp
        part, _ = integrate.quad(lambda x: oracle.kernel_over(K, x), zm, z, epsabs=0, epsrel=1e-12, limit=200)
        assert part == pytest.approx(u * I_num, rel=1e-8, abs=1e-12)


def test_sigma_lo_values(oracle):
    for ecm, ref in golden("sigma"):
        assert oracle.sigma_lo(ecm * ecm) == pytest.approx(ref, rel=2e-6)


def test_sigma_lo_low_energy_r_ratio(oracle):
    # far below the Z the photon dominates: sigma = N_c sum Q_f^2 * 4 pi alpha^2/(3 s)
    alpha = 1 / 128.802
    for ecm in (2.0, 5.0):
        s = ecm * ecm
        qed = 4 * np.pi * alpha ** 2 / (3 * s) * 0.389379656e9
        r = oracle.sigma_lo(s) / qed
        assert r == pytest.approx(3 * (3 / 9 + 2 * 4 / 9), rel=3e-3)


def test_me_angular_shape(oracle):
    # |M|^2 = A (1 + c^2) + B c: the c-even part is exactly proportional to 1 + c^2
    for f, ratio in ((1, golden("ba_down")[0][1]), (3, golden("ba_down")[0][1]), (5, golden("ba_down")[0][1]),
                     (2, golden("ba_up")[0][1]), (4, golden("ba_up")[0][1])):
        s = 91.2 ** 2
        cs = np.linspace(-1, 1, 21)
        m = np.array([oracle.me2(f, s, c) for c in cs])
        even = 0.5 * (m + m[::-1])
        odd = 0.5 * (m - m[::-1])
        A = even[len(cs) // 2]
        np.testing.assert_allclose(even, A * (1 + cs * cs), rtol=1e-13)
        B = odd[-1]
        np.testing.assert_allclose(odd, B * cs, rtol=1e-12, atol=1e-12 * A)
        assert B / A == pytest.approx(ratio, abs=2e-5)


@pytest.mark.parametrize("ecm", [10.0, 91.2, 500.0])
def test_me_weight_mean_is_sigma(oracle, ecm):
    n = 200_000
    r = oracle.generate(3, 0, n, ecm, 1e9, 2)  # t_C above s: no shower, ME only
    w = r["sum_d"][:, 0]
    sig = oracle.sigma_lo(ecm * ecm)
    assert abs(w.mean() - sig) < 4 * w.std() / np.sqrt(n)
    # flavour fractions proportional to the per-flavour cross-sections
    fl = r["sum_i"][:, 4]
    assert set(np.unique(fl)) == {1, 2, 3, 4, 5}
    for f in range(1, 6):
        frac = (w * (fl == f)).sum() / w.sum()
        ref = oracle.me2(f, ecm * ecm, 0.0) / sum(oracle.me2(g, ecm * ecm, 0.0) for g in range(1, 6))
        assert frac == pytest.approx(ref, abs=6e-3)


def test_me_event_kinematics(oracle):
    for ev in range(200):
        f, c, ph, w, p = oracle.me_event(11, ev, 91.2)
        assert 1 <= f <= 5 and -1 < c < 1 and 0 < ph < 2 * np.pi and w > 0
        assert p[0, 0] == 45.6 and p[1, 0] == 45.6
        np.testing.assert_array_equal(p[0, 1:], -p[1, 1:])
        assert abs(p[0, 0] ** 2 - (p[0, 1:] ** 2).sum()) < 1e-12 * 45.6 ** 2
        assert p[0, 3] / 45.6 == pytest.approx(c, abs=1e-15)
