"""The C-ABI library is built for gfx950 and exports every declared entry point.

No compute call is made here (no GPU needed)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmfvm.h")
LIB = os.path.join(ROOT, "paper_1908_08386_amd", "liblbmfvm.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lf_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python paper_1908_08386_amd/build.py)"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_library_loads_and_reports_abi_version():
    L = ctypes.CDLL(LIB)
    assert L.lf_abi_version() == 1
    L.lf_last_error.restype = ctypes.c_char_p
    assert isinstance(L.lf_last_error(), bytes)


def test_library_is_gfx950_code():
    # the fat binary embedded in the library names its single target
    data = open(LIB, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data
    assert b"gfx942" not in data and b"gfx90a" not in data


def test_oracle_shares_no_code_with_library():
    # the oracle's sources must not include or import the product sources
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith((".c", ".h", ".py")):
            text = open(os.path.join(odir, f)).read()
            assert "paper_1908_08386_amd" not in text.replace("(``paper_1908_08386_amd``)", "") \
                or f == "__init__.py"
            assert "lbmfvm.h" not in text
            assert "lf_internal" not in text
