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


def _c_sizes(names):
    """sizeof of the header's structs as the C compiler lays them out."""
    import subprocess
    import tempfile
    src = "#include <stdio.h>\n#include \"ddst.h\"\nint main(void) {\n"
    src += "".join(f'  printf("%zu\\n", sizeof({n}));\n' for n in names) + "  return 0;\n}\n"
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "sizes.c"), os.path.join(d, "sizes")
        open(c, "w").write(src)
        inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
        r = subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", inc, "-I", "/opt/rocm/include",
                            c, "-o", exe], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("cannot compile against the header: " + r.stderr[:200])
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    return [int(v) for v in out.split()]


@pytest.mark.skipif(not os.path.exists(LIB), reason="libddst.so not built")
def test_struct_layouts_match_header():
    """The ctypes mirrors have the sizes the C compiler gives the structs."""
    from paper_2510_25991_amd import ddst
    pairs = [("ddst_problem_t", ddst.ProblemC), ("ddst_build_opts_t", ddst.BuildOptsC),
             ("ddst_compress_opts_t", ddst.CompressOptsC), ("ddst_solve_opts_t", ddst.SolveOptsC),
             ("ddst_stats_t", ddst.StatsC)]
    sizes = _c_sizes([n for n, _ in pairs])
    for (name, cls), size in zip(pairs, sizes):
        assert ctypes.sizeof(cls) == size, name


def test_no_cpu_fallback_without_gpu():
    import torch
    from paper_2510_25991_amd import ddst
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        ddst.Operator(2, 15, 4)
