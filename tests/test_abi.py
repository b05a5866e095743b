"""The C-ABI library loads and exports every function include/dust.h
declares (no GPU calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dust.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(dust_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ("dust_bin", "dust_gather", "dust_push_expmid", "dust_deposit", "dust_step",
              "dust_ctx_create", "dust_ctx_destroy", "dust_ctx_status", "dust_last_error"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1908_10793_amd import dust
    if not os.path.exists(dust.LIB_PATH):
        from paper_1908_10793_amd import build
        build.build()
    L = dust.load_library()
    for n in declared_functions():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", dust.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r" T (dust_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(dust.EXPORTS) <= exported


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_1908_10793_amd import dust
    with pytest.raises(ValueError):
        dust._ptr(torch.zeros(3), torch.float32, "x")
