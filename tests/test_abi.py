"""The C ABI without a GPU: the library loads, exports every function that
include/vsh.h declares (and nothing else under the vsh_ prefix), and the
binding's export list and the header agree.  No compute call is made."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vsh.h")
LIB = os.path.join(ROOT, "paper_2403_08692_amd", "libvsh.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vsh_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libvsh.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_calls():
    names = declared()
    for must in ("vsh_create", "vsh_destroy", "vsh_generate", "vsh_generate_into", "vsh_generate_into_static",
                 "vsh_shower_records", "vsh_submit", "vsh_wait", "vsh_autotune"):
        assert must in names


def test_library_exports_every_declared_call(lib):
    for name in declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = sorted({w.split()[-1] for w in out.splitlines() if re.search(r" T vsh_", w)})
    assert exported == declared()


def test_binding_export_list_matches_the_header():
    from paper_2403_08692_amd import _native

    assert sorted(_native.EXPORTS) == declared()
