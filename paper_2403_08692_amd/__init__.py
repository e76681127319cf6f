"""MI355X-native parallel Sudakov-veto parton shower (Seymour & Sule,
arXiv:2403.08692): HIP kernels for gfx950 behind the C ABI of include/vsh.h,
with a thin ctypes binding of the same names.
"""
from ._native import (  # noqa: F401
    EXPORTS,
    Context,
    VshError,
    load,
    make_request,
    vsh_request,
    vsh_result,
    VSH_SUMMARY,
    VSH_RECORDS,
    VSH_FORM_PLAIN,
    VSH_FORM_PERSISTENT,
    VSH_INPUTS_ON_DEVICE,
    NOBS,
    NBINS,
    NHCOL,
    HIST_DOUBLES,
    NSUM_D,
    NSUM_I,
)
