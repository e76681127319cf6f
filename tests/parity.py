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
  * histograms: per observable and bin, the entry counts are equal except
    for events that differ or whose observable lies within 1e-9 (in units of
    the histogram's range) of a bin edge, where the two sides' roundings may
    bin it differently: each such event may move one entry between its two
    bins.  The GPU's entry counts are also exactly those of binning its own
    per-event observables (the same edge allowance).  Weighted sums: chi^2/ndf
    < 1.5 over filled bins.
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


def compare(gpu: dict, orc: dict, ecm, n: int, records: bool = True, isr: bool = False):
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
    rep.update(entry_check(gpu, orc, same, isr=isr))
    return rep, same


# histogram ranges (reading R24): log10 y23, log10 y34, tau, C, rho_H, B_T,
# B_W, cos(theta); 50 uniform bins [lo, hi) plus underflow and overflow
HIST_LO = np.array([-4.3, -4.3, 0.0, 0.0, 0.0, 0.0, 0.0, -1.0])
HIST_HI = np.array([-0.3, -0.3, 0.5, 1.0, 0.5, 0.5, 0.35, 1.0])
NBINS = 50
EDGE_TOL = 1e-9


def binned_values(sd):
    """The eight histogrammed values per event from summaries [10][n]."""
    with np.errstate(divide="ignore", invalid="ignore"):
        l23 = np.where(sd[2] > 0, np.log10(np.where(sd[2] > 0, sd[2], 1.0)), -np.inf)
        l34 = np.where(sd[3] > 0, np.log10(np.where(sd[3] > 0, sd[3], 1.0)), -np.inf)
    return np.stack([l23, l34, sd[4], sd[5], sd[6], sd[7], sd[8], sd[1]])


def bin_index(x, h, lo=HIST_LO, hi=HIST_HI):
    """Bin of each value of observable h: 0 underflow, 1..50, 51 overflow
    (NaN to overflow)."""
    lo, hi = lo[h], hi[h]
    with np.errstate(invalid="ignore"):
        inner = np.minimum(1 + np.floor((x - lo) / (hi - lo) * NBINS), NBINS)
        b = np.where(x < lo, 0, np.where(x >= hi, NBINS + 1, inner))
    return np.where(np.isnan(x), NBINS + 1, b).astype(np.int64)


def near_edge(x, h, lo=HIST_LO, hi=HIST_HI):
    lo, hi = lo[h], hi[h]
    u = (x - lo) / (hi - lo) * NBINS
    with np.errstate(invalid="ignore"):
        return np.isfinite(u) & (np.abs(u - np.round(u)) < EDGE_TOL * NBINS) & (u > -0.5) & (u < NBINS + 0.5)


# the initial-state branch's histograms: log10(p_T,V), y_V, emitted gluons,
# log10(p_T) of the hardest gluon (rows 4-7 unused)
ISR_LO = np.array([-1.0, -5.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0])
ISR_HI = np.array([3.0, 5.0, 50.0, 3.0, 1.0, 1.0, 1.0, 1.0])


def isr_binned_values(sd, si):
    with np.errstate(divide="ignore", invalid="ignore"):
        lpt = np.where(sd[2] > 0, np.log10(np.where(sd[2] > 0, sd[2], 1.0)), -np.inf)
        lg = np.where(sd[5] > 0, np.log10(np.where(sd[5] > 0, sd[5], 1.0)), -np.inf)
    return np.stack([lpt, sd[1], si[3].astype(np.float64), lg])


def entry_check(gpu, orc, same, isr=False):
    """Largest excess of a per-bin entry-count difference over what differing
    and edge events allow: GPU against oracle, and GPU against binning its own
    summaries.  Both must be <= 0.  isr: the initial-state branch's rows."""
    gd, od = gpu["sum_d"], orc["sum_d"].T
    g_done = gpu["sum_i"][1] == 1
    o_done = orc["sum_i"][:, 1] == 1
    if isr:
        gv, ov = isr_binned_values(gd, gpu["sum_i"]), isr_binned_values(od, orc["sum_i"].T)
        lo, hi = ISR_LO, ISR_HI
        gf = [gd[2], gd[1], gpu["sum_i"][3], gd[5]]  # the summary value behind each row
        of = [od[2], od[1], orc["sum_i"][:, 3], od[5]]
        logged = (0, 3)
    else:
        gv, ov = binned_values(gd), binned_values(od)
        lo, hi = HIST_LO, HIST_HI
        gf = [gd[k] for k in (2, 3, 4, 5, 6, 7, 8, 1)]
        of = [od[k] for k in (2, 3, 4, 5, 6, 7, 8, 1)]
        logged = (0, 1)
    worst_o, worst_self = -np.inf, -np.inf

    def counts(b, sel, spread):
        c = np.bincount(b[sel], minlength=NBINS + 2).astype(np.float64)
        if spread:  # an edge value may land in either neighbour
            c = c + np.concatenate([[0.0], c[:-1]]) + np.concatenate([c[1:], [0.0]])
        return c

    for h in range(len(gv)):
        gb, ob = bin_index(gv[h], h, lo, hi), bin_index(ov[h], h, lo, hi)
        # equal values are binned identically by the same arithmetic on both
        # sides; values that differ in their last bits may not be, near an edge
        edge = (near_edge(gv[h], h, lo, hi) | near_edge(ov[h], h, lo, hi)) & (gf[h] != of[h])
        differ = ~same
        slack = (counts(gb, differ & g_done, False) + counts(ob, differ & o_done, False)
                 + counts(gb, edge & same & g_done, True) + counts(ob, edge & same & o_done, True))
        diff = np.abs(gpu["hist"][h, :, 2] - orc["hist"][h, :, 2])
        worst_o = max(worst_o, float((diff - slack).max()))
        own = counts(gb, g_done, False)
        # the device's log10 and numpy's may round differently: only logged
        # values next to an edge may bin differently from the GPU's own fill
        own_edge = near_edge(gv[h], h, lo, hi) if h in logged else np.zeros_like(g_done)
        own_slack = counts(gb, g_done & own_edge, True)
        worst_self = max(worst_self, float((np.abs(gpu["hist"][h, :, 2] - own) - own_slack).max()))
    return dict(entry_excess=worst_o, entry_self_excess=worst_self)


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
    assert rep["entry_excess"] <= 0, rep
    assert rep["entry_self_excess"] <= 0, rep
