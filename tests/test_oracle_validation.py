"""Pins of the oracle's event validation (Table 1, "Validate Events"; the
paper names the step but prints no criterion, so the reading is: every
component finite, the total four-momentum (sqrt s, 0) within 1e-10 sqrt s per
component, every parton on its mass shell within 1e-10 s).

The accepted side is pinned by real showered events; these tests pin the
rejection side, which showered events never reach: momenta moved by known
amounts just above and just below each tolerance, at several energies so
that a tolerance not scaled by sqrt(s) (or scaled by s) fails one of them,
and the order of the checks (a non-finite component wins over everything
else)."""
import math

import numpy as np
import pytest

DONE, NONFINITE, CONSERVATION = 1, 3, 4
MASS = np.array([0.0, 0.0, 0.0, 0.0, 1.5, 4.8])


def _showered(oracle, ecm, n=40, seed=7, tcut=1.0, mass=None):
    """Finished events (records and flavours) that the oracle showered."""
    g = oracle.generate(seed, 0, n, ecm, tcut, 64, records=True, mass=mass)
    out = []
    for e in range(n):
        if g["sum_i"][e, 1] != DONE:
            continue
        k = g["rec"]["n"][e]
        out.append((g["rec"]["p"][e, :k].copy(), g["rec"]["pid"][e, :k].copy()))
    assert len(out) > n // 2
    return out


@pytest.mark.parametrize("ecm", [10.0, 91.2, 500.0])
def test_showered_events_validate(oracle, ecm):
    for p, pid in _showered(oracle, ecm):
        assert oracle.validate(p, ecm) == DONE


@pytest.mark.parametrize("ecm", [10.0, 91.2, 500.0])
@pytest.mark.parametrize("comp", [0, 1, 2, 3])
def test_conservation_tolerance_scales_with_sqrt_s(oracle, ecm, comp):
    """A component of the total moved by 2e-10 sqrt(s) is rejected, one moved
    by 0.5e-10 sqrt(s) is not (the mass shells move by at most 0.5e-10 s)."""
    for p, _ in _showered(oracle, ecm)[:10]:
        big, small = p.copy(), p.copy()
        big[0, comp] += 2e-10 * ecm
        small[0, comp] += 0.5e-10 * ecm
        assert oracle.validate(big, ecm) == CONSERVATION
        assert oracle.validate(small, ecm) == DONE


@pytest.mark.parametrize("ecm", [10.0, 91.2, 500.0])
def test_mass_shell_tolerance_scales_with_s(oracle, ecm):
    """Energy moved from one parton to another keeps the total but takes both
    off their shells: p_0^2 = 2 E_0 eps + eps^2, p_1^2 = -2 E_1 eps + eps^2."""
    s = ecm * ecm
    for p, _ in _showered(oracle, ecm)[:10]:
        emax = max(p[0, 0], p[1, 0])
        for frac, want in [(2.5e-10, CONSERVATION), (0.4e-10, DONE)]:
            eps = frac * s / (2.0 * emax)
            q = p.copy()
            q[0, 0] += eps
            q[1, 0] -= eps
            assert oracle.validate(q, ecm) == want, (frac, want)


def test_non_finite_is_checked_first(oracle):
    ecm = 91.2
    p, _ = _showered(oracle, ecm)[0]
    for bad in (math.nan, math.inf, -math.inf):
        for a in range(len(p)):
            for c in range(4):
                q = p.copy()
                q[a, c] = bad
                assert oracle.validate(q, ecm) == NONFINITE
    # two finite partons off their shells: conservation, not non-finite
    q = p.copy()
    q[0, 0] += 0.01
    q[1, 0] -= 0.01
    assert oracle.validate(q, ecm) == CONSERVATION
    q[2, 3] = math.nan
    assert oracle.validate(q, ecm) == NONFINITE


def test_massive_validation_uses_each_flavours_shell(oracle):
    ecm, s = 91.2, 91.2 ** 2
    evs = [(p, pid) for p, pid in _showered(oracle, ecm, n=200, seed=3, mass=MASS) if 5 in np.abs(pid)]
    assert len(evs) >= 5
    for p, pid in evs[:10]:
        assert oracle.validate_massive(p, pid, ecm, MASS) == DONE
        # the b quarks are 4.8 GeV off the massless shell: m^2 = 23 >> 1e-10 s
        assert oracle.validate(p, ecm) == CONSERVATION
        a = int(np.flatnonzero(np.abs(pid) == 5)[0])
        b = (a + 1) % len(pid)
        emax = max(p[a, 0], p[b, 0])
        for frac, want in [(2.5e-10, CONSERVATION), (0.4e-10, DONE)]:
            eps = frac * s / (2.0 * emax)
            q = p.copy()
            q[a, 0] += eps
            q[b, 0] -= eps
            assert oracle.validate_massive(q, pid, ecm, MASS) == want, (frac, want)
        # a massless parton given the b mass's shell by a wrong table
        wrong = MASS.copy()
        wrong[5] = 4.9
        assert oracle.validate_massive(p, pid, ecm, wrong) == CONSERVATION
