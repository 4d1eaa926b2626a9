"""The C-ABI library loads and exports every symbol include/apx.h declares (no GPU needed);
host-only geometry checks."""
import os
import re
import subprocess

import pytest

from paper_1201_3018_amd import apx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "apx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(apx_[a-z0-9_]+)\s*\(", txt)))


def test_header_matches_binding_exports():
    assert _header_functions() == sorted(apx.EXPORTS)


def test_library_exports_every_header_symbol():
    if not os.path.exists(apx.LIB_PATH):
        pytest.skip("libapx.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", apx.LIB_PATH], capture_output=True, text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _header_functions():
        assert name in syms, name
    L = apx.lib()
    for name in _header_functions():
        assert hasattr(L, name)


def test_geometry_host_only():
    if not os.path.exists(apx.LIB_PATH):
        pytest.skip("libapx.so not built")
    assert apx.apx_geometry(65536, 64, 1024) == (65, 958, 69)
    assert apx.apx_geometry(1 << 22, 1024, 4096) == (1025, 3070, 1367)
    assert apx.apx_geometry(100, 3, 32) == (3, 28, 4)
    with pytest.raises(apx.ApxError) as e:
        apx.apx_geometry(1000, 64, 1025)       # W odd
    assert e.value.status == apx.APX_E_INVALID
    with pytest.raises(apx.ApxError):
        apx.apx_geometry(1000, 64, 100)        # W < 2N
    with pytest.raises(apx.ApxError):
        apx.apx_geometry(0, 3, 32)             # empty input
    with pytest.raises(apx.ApxError):
        apx.apx_geometry(10, 0, 32)            # empty kernel
    assert apx.lib().apx_status_str(apx.APX_E_BOUND).decode().startswith("companding range")


def test_oracle_and_product_share_nothing():
    """The product package never imports the oracle, and the oracle never imports the product."""
    pkg = os.path.join(ROOT, "paper_1201_3018_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, re.M), f
                assert "orc.c" not in src and "liborc" not in src, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1201_3018_amd" not in src, f
