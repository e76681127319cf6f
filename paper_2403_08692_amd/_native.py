"""ctypes binding of libvsh (include/vsh.h).

Argument marshalling only: every step of the matrix element, shower,
observables and histogramming runs in the HIP kernels of libvsh.so.  There is
no CPU fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvsh.so")

VSH_OK = 0
STATUS_NAMES = {0: "VSH_OK", -1: "VSH_E_INVALID", -2: "VSH_E_NOMEM", -3: "VSH_E_DEVICE", -4: "VSH_E_BUSY",
                -5: "VSH_E_NOTFOUND", -6: "VSH_E_CANCELLED", -7: "VSH_E_INTERNAL"}
VSH_SUMMARY = 0x1
VSH_RECORDS = 0x2
VSH_FORM_PLAIN = 0x0
VSH_FORM_PERSISTENT = 0x4
VSH_INPUTS_ON_DEVICE = 0x8
VSH_HIST_FIXEDPOINT = 0x10
NOBS, NBINS = 8, 50
NHCOL = NBINS + 2
HIST_DOUBLES = NOBS * NHCOL * 3
NSUM_D, NSUM_I = 10, 7
STATIC_SCRATCH_BYTES = 64 * 1024 * 1024  # VSH_STATIC_SCRATCH_BYTES
EV_DONE, EV_OVERFLOW, EV_NONFINITE, EV_CONSERVATION = 1, 2, 3, 4


class vsh_ctx_opts(C.Structure):
    _fields_ = [("device", C.c_int), ("mem_budget_bytes", C.c_uint64), ("flags", C.c_uint32),
                ("tuner_cache_path", C.c_char_p)]


class vsh_request(C.Structure):
    _fields_ = [("n_events", C.c_uint64), ("seed", C.c_uint64), ("first_event", C.c_uint64),
                ("ecm", C.c_double), ("t_cut", C.c_double),
                ("ecm_per_event", C.c_void_p), ("tcut_per_event", C.c_void_p),
                ("max_partons", C.c_uint32), ("flags", C.c_uint32), ("cycle_limit", C.c_uint32),
                ("t_over", C.c_double), ("mass_c", C.c_double), ("mass_b", C.c_double)]


class vsh_tuning(C.Structure):
    _fields_ = [("plain_block", C.c_uint32), ("mapping", C.c_uint32), ("waves_per_cu", C.c_uint32),
                ("block", C.c_uint32), ("refill_threshold", C.c_uint32), ("refill_period", C.c_uint32),
                ("plain_waves", C.c_uint32), ("plain_mapping", C.c_uint32), ("from_cache", C.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class vsh_result(C.Structure):
    _fields_ = [("n_events", C.c_uint64), ("n_done", C.c_uint64), ("n_overflow", C.c_uint64),
                ("n_nonfinite", C.c_uint64), ("n_conservation", C.c_uint64),
                ("sum_w", C.c_double), ("sum_w2", C.c_double),
                ("n_obs", C.c_uint32), ("n_bins", C.c_uint32),
                ("hist_lo", C.POINTER(C.c_double)), ("hist_hi", C.POINTER(C.c_double)),
                ("hist", C.POINTER(C.c_double)),
                ("sum_d", C.POINTER(C.c_double)), ("sum_i", C.POINTER(C.c_int32)),
                ("sum_hash", C.POINTER(C.c_uint64)),
                ("rec_offsets", C.POINTER(C.c_uint64)), ("rec_p", C.POINTER(C.c_double)),
                ("rec_pid", C.POINTER(C.c_int8)), ("rec_col", C.POINTER(C.c_uint16)),
                ("rec_acol", C.POINTER(C.c_uint16)),
                ("total_cycles", C.c_uint64), ("total_trials", C.c_uint64), ("total_ends", C.c_uint64),
                ("total_emissions", C.c_uint64), ("max_cycles", C.c_uint32),
                ("t_me_ms", C.c_double), ("t_shower_ms", C.c_double), ("t_obs_ms", C.c_double),
                ("t_total_ms", C.c_double), ("n_cycle_limit", C.c_uint64), ("queue_ahead", C.c_uint32),
                ("t_queue_ms", C.c_double)]


_lib = None


def load():
    """Load libvsh.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libvsh.so is not built ({LIB_PATH}); run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime under the same soname; whichever is
    # loaded first serves the whole process.  Load PyTorch's first when it is
    # installed, so that device buffers and streams from PyTorch and the
    # library's launches share one runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.vsh_create.argtypes = [C.POINTER(vsh_ctx_opts), C.POINTER(P)]
    L.vsh_create.restype = C.c_int
    L.vsh_destroy.argtypes = [P]
    L.vsh_destroy.restype = None
    L.vsh_last_error.argtypes = [P]
    L.vsh_last_error.restype = C.c_char_p
    L.vsh_generate.argtypes = [P, C.POINTER(vsh_request), C.POINTER(C.POINTER(vsh_result))]
    L.vsh_generate.restype = C.c_int
    L.vsh_result_free.argtypes = [C.POINTER(vsh_result)]
    L.vsh_result_free.restype = None
    L.vsh_shower_records.argtypes = [P, C.POINTER(vsh_request), P, P, P, P, P, C.POINTER(C.POINTER(vsh_result))]
    L.vsh_shower_records.restype = C.c_int
    L.vsh_generate_into.argtypes = [P, C.POINTER(vsh_request), P, P, C.c_uint64, P, P, P, P]
    L.vsh_generate_into.restype = C.c_int
    L.vsh_generate_into_static.argtypes = [P, C.POINTER(vsh_request), P, P, P, P, P]
    L.vsh_generate_into_static.restype = C.c_int
    L.vsh_generate_isr.argtypes = [P, C.POINTER(vsh_request), C.c_double, C.POINTER(C.POINTER(vsh_result))]
    L.vsh_generate_isr.restype = C.c_int
    L.vsh_workspace_size.argtypes = [C.POINTER(vsh_request)]
    L.vsh_workspace_size.restype = C.c_uint64
    L.vsh_submit.argtypes = [P, C.POINTER(vsh_request), C.POINTER(C.c_uint64)]
    L.vsh_submit.restype = C.c_int
    L.vsh_poll.argtypes = [P, C.c_uint64, C.POINTER(C.c_int)]
    L.vsh_poll.restype = C.c_int
    L.vsh_wait.argtypes = [P, C.c_uint64, C.POINTER(C.POINTER(vsh_result))]
    L.vsh_wait.restype = C.c_int
    L.vsh_cancel.argtypes = [P, C.c_uint64]
    L.vsh_cancel.restype = C.c_int
    L.vsh_test_fail_epochs.argtypes = [P, C.c_uint32]
    L.vsh_test_fail_epochs.restype = C.c_int
    L.vsh_timing_start.argtypes = [P]
    L.vsh_timing_start.restype = C.c_int
    L.vsh_timing_read.argtypes = [P, C.POINTER(C.c_float), C.c_uint32, C.POINTER(C.c_uint32)]
    L.vsh_timing_read.restype = C.c_int
    L.vsh_get_tuning.argtypes = [P, C.POINTER(vsh_tuning)]
    L.vsh_get_tuning.restype = C.c_int
    L.vsh_set_tuning.argtypes = [P, C.POINTER(vsh_tuning)]
    L.vsh_set_tuning.restype = C.c_int
    L.vsh_autotune.argtypes = [P, C.POINTER(vsh_request), C.POINTER(vsh_tuning)]
    L.vsh_autotune.restype = C.c_int
    _lib = L
    return L


EXPORTS = ["vsh_create", "vsh_destroy", "vsh_last_error", "vsh_generate", "vsh_result_free",
           "vsh_shower_records", "vsh_generate_into", "vsh_workspace_size", "vsh_submit", "vsh_poll",
           "vsh_wait", "vsh_cancel", "vsh_timing_start", "vsh_timing_read", "vsh_get_tuning", "vsh_set_tuning",
           "vsh_autotune", "vsh_test_fail_epochs", "vsh_generate_into_static", "vsh_generate_isr"]


class VshError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(code, ctx_ptr=None):
    if code != VSH_OK:
        msg = load().vsh_last_error(ctx_ptr)
        raise VshError(code, msg.decode() if msg else "")


def _arr(ptr, count, dtype):
    if not ptr or count == 0:
        return None
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


def result_to_dict(res: vsh_result) -> dict:
    n = res.n_events
    out = dict(n_events=n, n_done=res.n_done, n_overflow=res.n_overflow, n_nonfinite=res.n_nonfinite,
               n_conservation=res.n_conservation, n_cycle_limit=res.n_cycle_limit, sum_w=res.sum_w, sum_w2=res.sum_w2,
               total_cycles=res.total_cycles, total_trials=res.total_trials, total_ends=res.total_ends,
               total_emissions=res.total_emissions, max_cycles=res.max_cycles,
               t_me_ms=res.t_me_ms, t_shower_ms=res.t_shower_ms, t_obs_ms=res.t_obs_ms,
               t_total_ms=res.t_total_ms, queue_ahead=res.queue_ahead, t_queue_ms=res.t_queue_ms)
    out["hist"] = _arr(res.hist, HIST_DOUBLES, np.float64).reshape(NOBS, NHCOL, 3)
    out["hist_lo"] = _arr(res.hist_lo, NOBS, np.float64)
    out["hist_hi"] = _arr(res.hist_hi, NOBS, np.float64)
    if res.sum_d:
        out["sum_d"] = _arr(res.sum_d, NSUM_D * n, np.float64).reshape(NSUM_D, n)
        out["sum_i"] = _arr(res.sum_i, NSUM_I * n, np.int32).reshape(NSUM_I, n)
        out["hash"] = _arr(res.sum_hash, n, np.uint64)
    if res.rec_offsets:
        off = _arr(res.rec_offsets, n + 1, np.uint64)
        tot = int(off[-1])
        out["rec_offsets"] = off
        out["rec_p"] = _arr(res.rec_p, 4 * tot, np.float64).reshape(tot, 4) if tot else np.zeros((0, 4))
        out["rec_pid"] = _arr(res.rec_pid, tot, np.int8) if tot else np.zeros(0, np.int8)
        out["rec_col"] = _arr(res.rec_col, tot, np.uint16) if tot else np.zeros(0, np.uint16)
        out["rec_acol"] = _arr(res.rec_acol, tot, np.uint16) if tot else np.zeros(0, np.uint16)
    return out


def make_request(n_events, seed=1, first_event=0, ecm=91.2, t_cut=1.0, max_partons=64, flags=0,
                 ecm_per_event=None, tcut_per_event=None, cycle_limit=0, t_over=0.0, mass_c=0.0, mass_b=0.0):
    """Build a vsh_request; per-event arrays are numpy float64 (host) or
    integer device addresses (with VSH_INPUTS_ON_DEVICE).  cycle_limit > 0
    vetoes events still above the cutoff after that many veto cycles; t_over
    > 0 is the alpha_s scale of the trial density (weighted veto); mass_c,
    mass_b > 0 make charm and bottom quarks massive.
    Returns (req, keepalive)."""
    keep = []

    def addr(a):
        if a is None:
            return None
        if isinstance(a, int):
            return a
        a = np.ascontiguousarray(a, np.float64)
        keep.append(a)
        return a.ctypes.data

    req = vsh_request(int(n_events), int(seed), int(first_event), float(ecm), float(t_cut),
                      addr(ecm_per_event), addr(tcut_per_event), int(max_partons), int(flags), int(cycle_limit),
                      float(t_over), float(mass_c), float(mass_b))
    return req, keep


class Context:
    """One libvsh context on one device."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0, tuner_cache_path: str | None = None):
        L = load()
        self._ptr = C.c_void_p()
        opts = vsh_ctx_opts(device, mem_budget_bytes, 0,
                            tuner_cache_path.encode() if tuner_cache_path else None)
        _check(L.vsh_create(C.byref(opts), C.byref(self._ptr)), None)

    @property
    def ptr(self):
        return self._ptr

    def close(self):
        if self._ptr:
            load().vsh_destroy(self._ptr)
            self._ptr = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return load().vsh_last_error(self._ptr).decode()

    def generate(self, n_events, seed=1, first_event=0, ecm=91.2, t_cut=1.0, max_partons=64,
                 summary=True, records=False, persistent=False, ecm_per_event=None, tcut_per_event=None,
                 cycle_limit=0, t_over=0.0, mass_c=0.0, mass_b=0.0, fixed_hist=False):
        flags = (VSH_SUMMARY if summary else 0) | (VSH_RECORDS if records else 0) | \
                (VSH_FORM_PERSISTENT if persistent else 0) | (VSH_HIST_FIXEDPOINT if fixed_hist else 0)
        req, keep = make_request(n_events, seed, first_event, ecm, t_cut, max_partons, flags,
                                 ecm_per_event, tcut_per_event, cycle_limit, t_over, mass_c, mass_b)
        res = C.POINTER(vsh_result)()
        _check(load().vsh_generate(self._ptr, C.byref(req), C.byref(res)), self._ptr)
        try:
            return result_to_dict(res.contents)
        finally:
            load().vsh_result_free(res)

    def generate_isr(self, n_events, sqrt_s_hadron=1960.0, q=91.2, t_cut=1.0, seed=1, first_event=0, max_partons=64,
                     summary=True, records=False):
        """vsh_generate_isr: Drell-Yan events with the initial-state shower
        (closed-form stand-in parton density)."""
        flags = (VSH_SUMMARY if summary else 0) | (VSH_RECORDS if records else 0)
        req, keep = make_request(n_events, seed, first_event, q, t_cut, max_partons, flags)
        res = C.POINTER(vsh_result)()
        _check(load().vsh_generate_isr(self._ptr, C.byref(req), float(sqrt_s_hadron), C.byref(res)), self._ptr)
        try:
            return result_to_dict(res.contents)
        finally:
            load().vsh_result_free(res)

    def shower_records(self, offsets, p, pid, col, acol, seed=1, first_event=0, t_cut=1.0, max_partons=64,
                       summary=True, records=True, mass_c=0.0, mass_b=0.0):
        offsets = np.ascontiguousarray(offsets, np.uint64)
        p = np.ascontiguousarray(p, np.float64)
        pid = np.ascontiguousarray(pid, np.int8)
        col = np.ascontiguousarray(col, np.uint16)
        acol = np.ascontiguousarray(acol, np.uint16)
        flags = (VSH_SUMMARY if summary else 0) | (VSH_RECORDS if records else 0)
        req, keep = make_request(len(offsets) - 1, seed, first_event, 0.0, t_cut, max_partons, flags,
                                 mass_c=mass_c, mass_b=mass_b)
        res = C.POINTER(vsh_result)()
        _check(load().vsh_shower_records(self._ptr, C.byref(req), offsets.ctypes.data, p.ctypes.data,
                                         pid.ctypes.data, col.ctypes.data, acol.ctypes.data, C.byref(res)),
               self._ptr)
        try:
            return result_to_dict(res.contents)
        finally:
            load().vsh_result_free(res)

    def workspace_size(self, req):
        return int(load().vsh_workspace_size(C.byref(req)))

    def generate_into(self, req, stream, workspace, workspace_bytes, dev_hist, dev_sum_d=None, dev_sum_i=None,
                      dev_hash=None):
        """All buffer arguments are integer device addresses; stream a hipStream_t address."""
        _check(load().vsh_generate_into(self._ptr, C.byref(req), stream, workspace, int(workspace_bytes),
                                        dev_hist, dev_sum_d, dev_sum_i, dev_hash), self._ptr)

    def generate_into_static(self, req, stream, dev_hist, dev_sum_d=None, dev_sum_i=None, dev_hash=None):
        """vsh_generate_into_static: the plain form with the library's own
        static device workspace (no allocation).  Buffer arguments are
        integer device addresses; stream a hipStream_t address."""
        _check(load().vsh_generate_into_static(self._ptr, C.byref(req), stream, dev_hist, dev_sum_d, dev_sum_i,
                                               dev_hash), self._ptr)

    def get_tuning(self):
        t = vsh_tuning()
        _check(load().vsh_get_tuning(self._ptr, C.byref(t)), self._ptr)
        return t.as_dict()

    def set_tuning(self, **kw):
        t = vsh_tuning()
        _check(load().vsh_get_tuning(self._ptr, C.byref(t)), self._ptr)
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(load().vsh_set_tuning(self._ptr, C.byref(t)), self._ptr)
        return self.get_tuning()

    def autotune(self, n_events=1 << 18, seed=1, ecm=91.2, t_cut=1.0, max_partons=64, persistent=True,
                 ecm_per_event=None, tcut_per_event=None):
        flags = VSH_FORM_PERSISTENT if persistent else VSH_FORM_PLAIN
        req, keep = make_request(n_events, seed, 0, ecm, t_cut, max_partons, flags, ecm_per_event, tcut_per_event)
        t = vsh_tuning()
        _check(load().vsh_autotune(self._ptr, C.byref(req), C.byref(t)), self._ptr)
        return t.as_dict()

    def timing_start(self):
        _check(load().vsh_timing_start(self._ptr), self._ptr)

    def timing_read(self, max_calls=1024):
        """Per-call stage times [n_calls, 3] in ms (ME, shower, observables)."""
        buf = (C.c_float * (3 * max_calls))()
        n = C.c_uint32()
        _check(load().vsh_timing_read(self._ptr, buf, max_calls, C.byref(n)), self._ptr)
        return np.array(buf[:3 * n.value], np.float64).reshape(n.value, 3)

    def submit(self, n_events, seed=1, first_event=0, ecm=91.2, t_cut=1.0, max_partons=128, summary=False,
               ecm_per_event=None, tcut_per_event=None, cycle_limit=0, t_over=0.0, mass_c=0.0, mass_b=0.0,
               fixed_hist=False):
        flags = (VSH_SUMMARY if summary else 0) | (VSH_HIST_FIXEDPOINT if fixed_hist else 0)
        req, keep = make_request(n_events, seed, first_event, ecm, t_cut, max_partons, flags,
                                 ecm_per_event, tcut_per_event, cycle_limit, t_over, mass_c, mass_b)
        t = C.c_uint64()
        _check(load().vsh_submit(self._ptr, C.byref(req), C.byref(t)), self._ptr)
        return t.value

    def poll(self, ticket):
        d = C.c_int()
        _check(load().vsh_poll(self._ptr, ticket, C.byref(d)), self._ptr)
        return bool(d.value)

    def wait(self, ticket):
        res = C.POINTER(vsh_result)()
        _check(load().vsh_wait(self._ptr, ticket, C.byref(res)), self._ptr)
        try:
            return result_to_dict(res.contents)
        finally:
            load().vsh_result_free(res)

    def cancel(self, ticket):
        _check(load().vsh_cancel(self._ptr, ticket), self._ptr)

    def test_fail_epochs(self, count):
        """Testing hook: the next `count` serving launches report a HIP launch failure."""
        _check(load().vsh_test_fail_epochs(self._ptr, int(count)), self._ptr)
