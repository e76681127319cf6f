"""ctypes binding of the serial FP64 oracle (``vsh_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product package never does.
The oracle is an independent, plain, serial C implementation of the shower of
Seymour & Sule (arXiv:2403.08692, Appendices A and B, Section 3.1); see the
header comment of ``vsh_oracle.c`` for what each part follows.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VSH_ORACLE_LIB points at another build of the same source (an -O3
# -march=native build for timing, or a deliberately broken copy in a test
# that checks the pins catch it).
LIB_PATH = os.environ.get("VSH_ORACLE_LIB") or os.path.join(HERE, "libvsh_oracle.so")

NOBS = 8
NBINS = 50
NHCOL = NBINS + 2
NSUM_D = 10
NSUM_I = 7
NLOG = 7
NWORK = 6

STATUS = {"RUNNING": 0, "DONE": 1, "OVERFLOW": 2, "NONFINITE": 3, "CONSERVATION": 4, "TRUNCATED": 5, "STOPPED": 6}
P_ME, P_TRIAL, P_ACCEPT, P_SPLIT = 1, 2, 3, 4
OBS_NAMES = ["log10_y23", "log10_y34", "tau", "C", "rho_H", "B_T", "B_W", "cos_theta"]
WORK_NAMES = ["cycles", "connected_ends", "active_ends", "trials", "accepted", "veto_evals"]

_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)
_u64p = C.POINTER(C.c_uint64)


def lib():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is not None:
        return _lib
    src = os.path.join(HERE, "vsh_oracle.c")
    if not os.environ.get("VSH_ORACLE_LIB") and (
            not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src)):
        from . import build as _build

        _build.build()
    L = C.CDLL(LIB_PATH)
    L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.or_uniform.argtypes = [C.c_uint32, C.c_uint32]
    L.or_uniform.restype = C.c_double
    L.or_draw.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _u32p]
    L.or_alpha_s.argtypes = [C.c_double]
    L.or_alpha_s.restype = C.c_double
    L.or_kernel_list.argtypes = [C.c_int, _ip]
    L.or_kernel_list.restype = C.c_int
    for name in ("or_kernel_value",):
        getattr(L, name).argtypes = [C.c_int, C.c_double, C.c_double]
        getattr(L, name).restype = C.c_double
    L.or_kernel_over.argtypes = [C.c_int, C.c_double]
    L.or_kernel_over.restype = C.c_double
    L.or_kernel_integral.argtypes = [C.c_int, C.c_double, C.c_double]
    L.or_kernel_integral.restype = C.c_double
    L.or_kernel_zgen.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
    L.or_kernel_zgen.restype = C.c_double
    L.or_me2.argtypes = [C.c_int, C.c_double, C.c_double]
    L.or_me2.restype = C.c_double
    L.or_sigma_lo.argtypes = [C.c_double]
    L.or_sigma_lo.restype = C.c_double
    L.or_me_event.argtypes = [C.c_uint64, C.c_uint64, C.c_double, _ip, _dp, _dp, _dp, _dp]
    L.or_split_kinematics.argtypes = [_dp, _dp, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
    L.or_shower.argtypes = [C.c_uint64, C.c_uint64, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double,
                            _dp, C.c_int, _ip, _dp, _ip, _ip, _ip, _ip, _u64p, _ip, _dp, _dp, C.c_int, _u64p]
    L.or_shower.restype = C.c_int
    L.or_thrust.argtypes = [C.c_int, _dp, _dp]
    L.or_thrust.restype = C.c_double
    L.or_durham.argtypes = [C.c_int, _dp, C.c_double, _dp, _dp]
    L.or_cparameter.argtypes = [C.c_int, _dp]
    L.or_cparameter.restype = C.c_double
    L.or_hemispheres.argtypes = [C.c_int, _dp, _dp, C.c_double, _dp, _dp, _dp]
    L.or_validate.argtypes = [C.c_int, _dp, C.c_double]
    L.or_validate.restype = C.c_int
    L.or_observables.argtypes = [C.c_int, _dp, C.c_double, _dp]
    L.or_hist_ranges.argtypes = [_dp, _dp]
    L.or_me2_massive.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
    L.or_me2_massive.restype = C.c_double
    L.or_sigma_lo_massive.argtypes = [C.c_double, _dp]
    L.or_sigma_lo_massive.restype = C.c_double
    L.or_me_event_massive.argtypes = [C.c_uint64, C.c_uint64, C.c_double, _dp, _ip, _dp, _dp, _dp, _dp]
    L.or_massive_limits.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp]
    L.or_massive_limits.restype = C.c_int
    L.or_massive_flux.argtypes = [C.c_double] * 5
    L.or_massive_flux.restype = C.c_double
    L.or_kernel_value_massive.argtypes = [C.c_int] + [C.c_double] * 5
    L.or_kernel_value_massive.restype = C.c_double
    L.or_massive_ratio.argtypes = [C.c_int] + [C.c_double] * 7
    L.or_massive_ratio.restype = C.c_double
    L.or_split_kinematics_massive.argtypes = [_dp, _dp] + [C.c_double] * 7 + [_dp, _dp, _dp]
    L.or_validate_massive.argtypes = [C.c_int, _dp, _ip, C.c_double, _dp]
    L.or_validate_massive.restype = C.c_int
    L.or_generate.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, _dp, C.c_double, _dp, C.c_double,
                              C.c_int, C.c_int, C.c_double, _dp, _dp, _i32p, _u64p, _dp, _i32p, _dp, _i32p, _i32p, _i32p, _u64p]
    L.or_generate.restype = C.c_int
    L.or_pdf_q.argtypes = [C.c_double]
    L.or_pdf_q.restype = C.c_double
    L.or_pdf_g.argtypes = [C.c_double]
    L.or_pdf_g.restype = C.c_double
    L.or_isr_zlimits.argtypes = [C.c_double] * 3 + [_dp, _dp]
    L.or_isr_zlimits.restype = C.c_int
    L.or_isr_ratio.argtypes = [C.c_double] * 4
    L.or_isr_ratio.restype = C.c_double
    L.or_isr_me.argtypes = [C.c_uint64, C.c_uint64, C.c_double, C.c_double, _ip, _ip, _dp, _dp, _dp, _dp, _dp]
    L.or_isr_shower.argtypes = [C.c_uint64, C.c_uint64, C.c_double, C.c_double, C.c_int, C.c_int, _ip, _dp, _ip, _ip,
                                _ip, _dp, _dp, _ip, _u64p, _ip, _dp, C.c_int, _u64p]
    L.or_isr_shower.restype = C.c_int
    L.or_isr_validate.argtypes = [C.c_int, _dp, C.c_double]
    L.or_isr_validate.restype = C.c_int
    L.or_isr_hist_ranges.argtypes = [_dp, _dp]
    L.or_isr_generate.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_double, C.c_double, C.c_double, C.c_int,
                                  _dp, _i32p, _u64p, _dp, _i32p, _dp, _i32p, _i32p, _i32p, _u64p]
    L.or_isr_generate.restype = C.c_int
    _lib = L
    return L


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _mass_table(mass):
    """Six doubles indexed by flavour (0 unused, 1..5 = d, u, s, c, b), or None."""
    if mass is None:
        return None
    m = np.ascontiguousarray(mass, np.float64)
    assert m.shape == (6,)
    return m


def me2_massive(flavour, s, cos_theta, m):
    return lib().or_me2_massive(int(flavour), float(s), float(cos_theta), float(m))


def sigma_lo_massive(s, mass):
    return lib().or_sigma_lo_massive(float(s), _ptr(_mass_table(mass), _dp))


def me_event_massive(seed, event, ecm, mass):
    f = C.c_int()
    c, ph, w = C.c_double(), C.c_double(), C.c_double()
    p = np.zeros(8)
    lib().or_me_event_massive(seed, event, ecm, _ptr(_mass_table(mass), _dp), C.byref(f), C.byref(c), C.byref(ph),
                              C.byref(w), _ptr(p, _dp))
    return f.value, c.value, ph.value, w.value, p.reshape(2, 4)


def massive_limits(Q2, mi, mj, mk, tcut):
    zm, zp = C.c_double(), C.c_double()
    ok = lib().or_massive_limits(float(Q2), float(mi), float(mj), float(mk), float(tcut), C.byref(zm), C.byref(zp))
    return (zm.value, zp.value) if ok else None


def massive_flux(Q2, mi, mj, mk, mij):
    return lib().or_massive_flux(float(Q2), float(mi), float(mj), float(mk), float(mij))


def kernel_value_massive(K, z, y, mi, qb2, sij):
    return lib().or_kernel_value_massive(int(K), float(z), float(y), float(mi), float(qb2), float(sij))


def massive_ratio(K, t, z, Q2, mi, mj, mk, fover):
    return lib().or_massive_ratio(int(K), float(t), float(z), float(Q2), float(mi), float(mj), float(mk),
                                  float(fover))


def split_kinematics_massive(pij, pk, mi, mj, mk, mij, t, z, phi):
    pij = np.ascontiguousarray(pij, np.float64)
    pk = np.ascontiguousarray(pk, np.float64)
    oi, oj, ok = np.zeros(4), np.zeros(4), np.zeros(4)
    lib().or_split_kinematics_massive(_ptr(pij, _dp), _ptr(pk, _dp), mi, mj, mk, mij, t, z, phi, _ptr(oi, _dp),
                                      _ptr(oj, _dp), _ptr(ok, _dp))
    return oi, oj, ok


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    lib().or_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(out, _u32p))
    return out


def draw(seed, event, cycle, purpose, slot):
    out = np.zeros(4, np.uint32)
    lib().or_draw(seed, event, cycle, purpose, slot, _ptr(out, _u32p))
    return out


def uniform(hi, lo):
    return lib().or_uniform(int(hi), int(lo))


def alpha_s(t):
    return lib().or_alpha_s(float(t))


def kernel_list(pid):
    out = (C.c_int * 6)()
    n = lib().or_kernel_list(int(pid), out)
    return [out[i] for i in range(n)]


def kernel_value(K, z, y):
    return lib().or_kernel_value(int(K), float(z), float(y))


def kernel_over(K, z):
    return lib().or_kernel_over(int(K), float(z))


def kernel_integral(K, zm, zp):
    return lib().or_kernel_integral(int(K), float(zm), float(zp))


def kernel_zgen(K, zm, zp, u):
    return lib().or_kernel_zgen(int(K), float(zm), float(zp), float(u))


def me2(flavour, s, cos_theta):
    return lib().or_me2(int(flavour), float(s), float(cos_theta))


def sigma_lo(s):
    return lib().or_sigma_lo(float(s))


def me_event(seed, event, ecm):
    f = C.c_int()
    c, ph, w = C.c_double(), C.c_double(), C.c_double()
    p = np.zeros(8)
    lib().or_me_event(seed, event, ecm, C.byref(f), C.byref(c), C.byref(ph), C.byref(w), _ptr(p, _dp))
    return f.value, c.value, ph.value, w.value, p.reshape(2, 4)


def split_kinematics(pi, pk, t, z, phi):
    pi = np.ascontiguousarray(pi, np.float64)
    pk = np.ascontiguousarray(pk, np.float64)
    oi, oj, ok = np.zeros(4), np.zeros(4), np.zeros(4)
    lib().or_split_kinematics(_ptr(pi, _dp), _ptr(pk, _dp), t, z, phi, _ptr(oi, _dp), _ptr(oj, _dp), _ptr(ok, _dp))
    return oi, oj, ok


def shower(seed, event, ecm, tcut, p, pid, col, acol, cap=64, max_emit=-1, max_log=64, max_cycles=0, t_over=0.0,
           mass=None):
    """Shower one event from the given partons.  Returns a dict.  max_cycles > 0
    gives up (status TRUNCATED) an event still above the cutoff after that many
    veto cycles; t_over > 0 takes alpha_s(t_over) for the trial density (the
    weighted veto; the returned ``weight`` is the event's shower weight); mass
    is a table of six quark masses indexed by flavour (None: massless)."""
    n0 = len(pid)
    P = np.zeros((cap, 4))
    P[:n0] = np.asarray(p, np.float64).reshape(n0, 4)
    PID = np.zeros(cap, np.intc)
    COL = np.zeros(cap, np.intc)
    ACOL = np.zeros(cap, np.intc)
    PID[:n0], COL[:n0], ACOL[:n0] = pid, col, acol
    n = C.c_int(n0)
    cyc, nemit = C.c_int(), C.c_int()
    h = C.c_uint64()
    log = np.zeros((max_log, NLOG))
    work = np.zeros(NWORK, np.uint64)
    wgt = C.c_double()
    mt = _mass_table(mass)
    st = lib().or_shower(seed, event, ecm, tcut, cap, int(max_cycles), float(t_over), _ptr(mt, _dp), max_emit,
                         C.byref(n),
                         _ptr(P, _dp), _ptr(PID, _ip), _ptr(COL, _ip), _ptr(ACOL, _ip), C.byref(cyc), C.byref(h),
                         C.byref(nemit), C.byref(wgt), _ptr(log, _dp), max_log, _ptr(work, _u64p))
    m = n.value
    return dict(status=st, n=m, p=P[:m].copy(), pid=PID[:m].copy(), col=COL[:m].copy(), acol=ACOL[:m].copy(),
                cycles=cyc.value, hash=h.value, n_emit=nemit.value, weight=wgt.value, log=log[:min(nemit.value, max_log)].copy(),
                work=work)


def _as_p(p):
    p = np.ascontiguousarray(p, np.float64).reshape(-1, 4)
    return p, len(p)


def thrust(p):
    p, n = _as_p(p)
    ax = np.zeros(3)
    T = lib().or_thrust(n, _ptr(p, _dp), _ptr(ax, _dp))
    return T, ax


def durham(p, s):
    p, n = _as_p(p)
    a, b = C.c_double(), C.c_double()
    lib().or_durham(n, _ptr(p, _dp), float(s), C.byref(a), C.byref(b))
    return a.value, b.value


def cparameter(p):
    p, n = _as_p(p)
    return lib().or_cparameter(n, _ptr(p, _dp))


def hemispheres(p, axis, s):
    p, n = _as_p(p)
    ax = np.ascontiguousarray(axis, np.float64)
    r, bt, bw = C.c_double(), C.c_double(), C.c_double()
    lib().or_hemispheres(n, _ptr(p, _dp), _ptr(ax, _dp), float(s), C.byref(r), C.byref(bt), C.byref(bw))
    return r.value, bt.value, bw.value


def validate(p, ecm):
    p, n = _as_p(p)
    return lib().or_validate(n, _ptr(p, _dp), float(ecm))


def validate_massive(p, pid, ecm, mass):
    """Status of a finished event whose partons may carry quark masses
    (mass: six doubles indexed by flavour, or None for massless)."""
    p, n = _as_p(p)
    f = np.ascontiguousarray(pid, np.intc)
    assert len(f) == n
    return lib().or_validate_massive(n, _ptr(p, _dp), _ptr(f, _ip), float(ecm), _ptr(_mass_table(mass), _dp))


def observables(p, ecm):
    p, n = _as_p(p)
    o = np.zeros(7)
    lib().or_observables(n, _ptr(p, _dp), float(ecm), _ptr(o, _dp))
    return o


def hist_ranges():
    lo, hi = np.zeros(NOBS), np.zeros(NOBS)
    lib().or_hist_ranges(_ptr(lo, _dp), _ptr(hi, _dp))
    return lo, hi


def generate(seed, first, n_events, ecm=91.2, tcut=1.0, cap=64, records=False, ecm_arr=None, tcut_arr=None,
             max_cycles=0, t_over=0.0, mass=None):
    """Run ME + shower + observables + histograms for events first..first+n-1.

    Returns a dict with per-event summaries (``sum_d`` [n, 10]: w, cos_theta,
    y23, y34, tau, C, rho_H, B_T, B_W, phi; ``sum_i`` [n, 7]: n, status,
    cycles, n_emit, flavour, trials, active dipole ends; ``hash`` [n]), histograms [8, 52, 3] and the
    work counters; with ``records`` also the final partons.  ``max_cycles`` > 0
    vetoes events still above the cutoff after that many veto cycles (status
    TRUNCATED, left out of the histograms); ``t_over`` > 0 runs the weighted
    veto with alpha_s(t_over) in the trial density (event weights in ``sum_d``
    field 0 and the histograms include the shower weight).
    """
    n_events = int(n_events)
    sum_d = np.zeros((n_events, NSUM_D))
    sum_i = np.zeros((n_events, NSUM_I), np.int32)
    hsh = np.zeros(n_events, np.uint64)
    hist = np.zeros((NOBS, NHCOL, 3))
    work = np.zeros(NWORK, np.uint64)
    rec = {}
    if records:
        rec = dict(n=np.zeros(n_events, np.int32), p=np.zeros((n_events, cap, 4)),
                   pid=np.zeros((n_events, cap), np.int32), col=np.zeros((n_events, cap), np.int32),
                   acol=np.zeros((n_events, cap), np.int32))
    e_arr = None if ecm_arr is None else np.ascontiguousarray(ecm_arr, np.float64)
    t_arr = None if tcut_arr is None else np.ascontiguousarray(tcut_arr, np.float64)
    rc = lib().or_generate(seed, first, n_events, _ptr(e_arr, _dp), float(ecm), _ptr(t_arr, _dp), float(tcut),
                           int(cap), int(max_cycles), float(t_over), _ptr(_mass_table(mass), _dp), _ptr(sum_d, _dp), _ptr(sum_i, _i32p), _ptr(hsh, _u64p), _ptr(hist, _dp),
                           _ptr(rec.get("n"), _i32p), _ptr(rec.get("p"), _dp), _ptr(rec.get("pid"), _i32p),
                           _ptr(rec.get("col"), _i32p), _ptr(rec.get("acol"), _i32p), _ptr(work, _u64p))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    out = dict(sum_d=sum_d, sum_i=sum_i, hash=hsh, hist=hist, work=work)
    if records:
        out["rec"] = rec
    return out


# ---------------------------------------------------------------------------
# Initial-state shower of Drell-Yan events (closed-form stand-in density)
# ---------------------------------------------------------------------------
def pdf_q(x):
    return lib().or_pdf_q(float(x))


def pdf_g(x):
    return lib().or_pdf_g(float(x))


def isr_zlimits(x, st, tcut):
    lo, hi = C.c_double(), C.c_double()
    ok = lib().or_isr_zlimits(float(x), float(st), float(tcut), C.byref(lo), C.byref(hi))
    return (lo.value, hi.value) if ok else None


def isr_ratio(t, z, x, st):
    return lib().or_isr_ratio(float(t), float(z), float(x), float(st))


def isr_me(seed, event, sqrt_s_had, q):
    f, qa = C.c_int(), C.c_int()
    y, w, xa, xb = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    p = np.zeros(12)
    lib().or_isr_me(seed, event, float(sqrt_s_had), float(q), C.byref(f), C.byref(qa), C.byref(y), C.byref(w),
                    C.byref(xa), C.byref(xb), _ptr(p, _dp))
    return dict(flavour=f.value, quark_from_a=bool(qa.value), y=y.value, weight=w.value, xa=xa.value, xb=xb.value,
                p=p.reshape(3, 4))


def isr_shower(seed, event, q, tcut, p, pid, col, acol, xa, xb, cap=64, max_emit=-1, max_log=64):
    """Backward evolution of one Drell-Yan event from the partons given
    (incoming from A, incoming from B, then the final state)."""
    n0 = len(pid)
    P = np.zeros((cap, 4))
    P[:n0] = np.asarray(p, np.float64).reshape(n0, 4)
    PID = np.zeros(cap, np.intc)
    COL = np.zeros(cap, np.intc)
    ACOL = np.zeros(cap, np.intc)
    PID[:n0], COL[:n0], ACOL[:n0] = pid, col, acol
    n = C.c_int(n0)
    XA, XB = C.c_double(xa), C.c_double(xb)
    cyc, nemit = C.c_int(), C.c_int()
    h = C.c_uint64()
    log = np.zeros((max_log, NLOG))
    work = np.zeros(NWORK, np.uint64)
    st = lib().or_isr_shower(seed, event, float(q), float(tcut), cap, max_emit, C.byref(n), _ptr(P, _dp),
                             _ptr(PID, _ip), _ptr(COL, _ip), _ptr(ACOL, _ip), C.byref(XA), C.byref(XB),
                             C.byref(cyc), C.byref(h), C.byref(nemit), _ptr(log, _dp), max_log, _ptr(work, _u64p))
    m = n.value
    return dict(status=st, n=m, p=P[:m].copy(), pid=PID[:m].copy(), col=COL[:m].copy(), acol=ACOL[:m].copy(),
                xa=XA.value, xb=XB.value, cycles=cyc.value, hash=h.value, n_emit=nemit.value,
                log=log[:min(nemit.value, max_log)].copy(), work=work)


def isr_validate(p, q):
    p, n = _as_p(p)
    return lib().or_isr_validate(n, _ptr(p, _dp), float(q))


def isr_hist_ranges():
    lo, hi = np.zeros(NOBS), np.zeros(NOBS)
    lib().or_isr_hist_ranges(_ptr(lo, _dp), _ptr(hi, _dp))
    return lo, hi


def isr_generate(seed, first, n_events, sqrt_s_had, q, tcut, cap=64, records=False):
    """Drell-Yan events through start, backward shower, validation,
    observables and histograms; the layout of generate()'s outputs (sum_d
    per event: w, y_V, p_T,V, x_A, x_B, hardest gluon p_T, 0...)."""
    n_events = int(n_events)
    sum_d = np.zeros((n_events, NSUM_D))
    sum_i = np.zeros((n_events, NSUM_I), np.int32)
    hsh = np.zeros(n_events, np.uint64)
    hist = np.zeros((NOBS, NHCOL, 3))
    work = np.zeros(NWORK, np.uint64)
    rec = {}
    if records:
        rec = dict(n=np.zeros(n_events, np.int32), p=np.zeros((n_events, cap, 4)),
                   pid=np.zeros((n_events, cap), np.int32), col=np.zeros((n_events, cap), np.int32),
                   acol=np.zeros((n_events, cap), np.int32))
    rc = lib().or_isr_generate(seed, first, n_events, float(sqrt_s_had), float(q), float(tcut), int(cap),
                               _ptr(sum_d, _dp), _ptr(sum_i, _i32p), _ptr(hsh, _u64p), _ptr(hist, _dp),
                               _ptr(rec.get("n"), _i32p), _ptr(rec.get("p"), _dp), _ptr(rec.get("pid"), _i32p),
                               _ptr(rec.get("col"), _i32p), _ptr(rec.get("acol"), _i32p), _ptr(work, _u64p))
    if rc != 0:
        raise ValueError("oracle: bad arguments")
    out = dict(sum_d=sum_d, sum_i=sum_i, hash=hsh, hist=hist, work=work)
    if records:
        out["rec"] = rec
    return out
