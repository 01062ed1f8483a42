"""The C-ABI library loads and exports every symbol its header declares.

No compute calls: this runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddst.h")
LIB = os.path.join(ROOT, "paper_2510_25991_amd", "libddst.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ddst_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ddst_build_transfer", "ddst_compress", "ddst_solve", "ddst_adjoint"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libddst.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libddst.so not built")
def test_binding_declares_every_export():
    from paper_2510_25991_amd import ddst
    assert sorted(ddst.EXPORTS) == declared_functions()
    ddst.load_library()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libddst.so not built")
def test_struct_layouts_match_header():
    """The ctypes mirrors have the sizes the C compiler gives the structs."""
    from paper_2510_25991_amd import ddst
    assert ctypes.sizeof(ddst.ProblemC) == 56
    assert ctypes.sizeof(ddst.BuildOptsC) == 16
    assert ctypes.sizeof(ddst.CompressOptsC) == 40
    assert ctypes.sizeof(ddst.SolveOptsC) == 32
    assert ctypes.sizeof(ddst.StatsC) == 104


def test_no_cpu_fallback_without_gpu():
    import torch
    from paper_2510_25991_amd import ddst
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        ddst.Operator(2, 15, 4)
