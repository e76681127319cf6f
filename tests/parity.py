"""Comparison of the HIP path with the oracle, event by event.

Bars (written here, used by every GPU parity test):
  * integer and index outputs -- parton count, status, veto cycles, accepted
    emissions, flavour, emission-sequence hash, final flavours and colour
    lines -- are compared exactly ("identical events");
  * at least 99.9% of events must be identical;
  * on identical events every momentum component agrees to 1e-9 sqrt(s);
  * weights (on identical events) to 1e-9 relative: with the weighted veto an
    event weight carries one factor +-(2r - 1) per veto above the trial
    density, each from the same kinematics as the momenta, so it gets the
    momenta's bar; observables to 1e-9 relative or 1e-12
    absolute (they are computed from momenta that agree to ~1e-15);
  * histograms: chi^2/ndf < 1.5 over filled bins, with the entry counts
    per bin allowed to differ only by events that differ.
Where the shower compares floating-point trial scales (the winner, the veto),
both sides decide in FP64; the GPU compares ln t, the oracle t, so a decision
can flip only when two values agree to the last few bits.
"""
from __future__ import annotations

import numpy as np

MOM_TOL = 1e-9
OBS_RTOL = 1e-9
OBS_ATOL = 1e-12
W_RTOL = 1e-9
MIN_IDENTICAL = 0.999


def oracle_records(orc, n):
    """Oracle records as a CSR triple aligned with the GPU's."""
    rn = orc["rec"]["n"]
    parts = []
    for e in range(n):
        k = rn[e]
        parts.append((orc["rec"]["p"][e, :k], orc["rec"]["pid"][e, :k], orc["rec"]["col"][e, :k],
                      orc["rec"]["acol"][e, :k]))
    return parts


def compare(gpu: dict, orc: dict, ecm, n: int, records: bool = True):
    """Returns a report dict; raises AssertionError when a bar is missed."""
    gi = gpu["sum_i"]          # [6][n]
    oi = orc["sum_i"].T        # [7][n]
    same = np.ones(n, bool)
    for f in range(7):
        same &= gi[f] == oi[f]
    same &= gpu["hash"] == orc["hash"]
    ecm = np.broadcast_to(np.asarray(ecm, np.float64), (n,))
    mom_err = 0.0
    if records:
        off = gpu["rec_offsets"].astype(np.int64)
        op = oracle_records(orc, n)
        for e in np.nonzero(same)[0]:
            a, b = off[e], off[e + 1]
            p, pid, col, acol = op[e]
            if b - a != len(pid) or not (np.array_equal(gpu["rec_pid"][a:b], pid)
                                         and np.array_equal(gpu["rec_col"][a:b], col)
                                         and np.array_equal(gpu["rec_acol"][a:b], acol)):
                same[e] = False
                continue
            d = np.abs(gpu["rec_p"][a:b] - p).max() / ecm[e]
            mom_err = max(mom_err, d)
    frac = same.mean()
    gd = gpu["sum_d"]          # [10][n]
    od = orc["sum_d"].T        # [10][n]
    # event weights (matrix element x weighted-veto factors) on identical events
    w_err = float(np.max(np.abs(gd[0][same] - od[0][same]) / np.abs(od[0][same]))) if same.any() else 0.0
    obs_bad = 0
    for f in range(2, 9):
        g, o = gd[f][same], od[f][same]
        ok = np.isclose(g, o, rtol=OBS_RTOL, atol=OBS_ATOL)
        obs_bad += int((~ok).sum())
    rep = dict(n=n, identical=int(same.sum()), frac=float(frac), mom_err=float(mom_err), w_err=float(w_err),
               obs_bad=obs_bad)
    rep.update(hist_chi2(gpu["hist"], orc["hist"]))
    return rep, same


def hist_chi2(hg, ho):
    """chi^2 between two weighted histograms [nobs][nbins+2][3] (sum w,
    sum w^2, entries), bins with entries on either side."""
    num = (hg[..., 0] - ho[..., 0]) ** 2
    den = hg[..., 1] + ho[..., 1]
    m = den > 0
    chi2 = float((num[m] / den[m]).sum())
    ndf = int(m.sum())
    return dict(chi2=chi2, ndf=ndf, chi2_ndf=chi2 / max(ndf, 1),
                max_entry_diff=float(np.abs(hg[..., 2] - ho[..., 2]).max()))


def assert_parity(rep):
    assert rep["frac"] >= MIN_IDENTICAL, rep
    assert rep["mom_err"] <= MOM_TOL, rep
    assert rep["w_err"] <= W_RTOL, rep
    assert rep["obs_bad"] == 0, rep
    assert rep["chi2_ndf"] < 1.5, rep
