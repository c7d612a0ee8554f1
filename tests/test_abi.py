"""CPU checks of the C ABI boundary: the built library loads without a GPU,
exports every entry point include/nks.h declares, and the ctypes structures
have the C layout (checked against a gcc-compiled probe of the header)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nks.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(nks_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def built():
    import paper_2007_13966_amd._lib as L
    if not os.path.exists(L.LIBPATH):
        from paper_2007_13966_amd import build
        build.build()
    return L


def test_library_exports_every_declared_symbol(built):
    lib = built.load()
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(built.PROTOTYPES), set(names) ^ set(built.PROTOTYPES)
    assert lib.nks_version().startswith(b"libnks")


def test_struct_layouts_match_c(built, tmp_path):
    structs = ["nks_fluid", "nks_reservoir_desc", "nks_grid_desc", "nks_ras_desc",
               "nks_gmres_desc", "nks_gmres_stats", "nks_newton_desc", "nks_newton_stats",
               "nks_adjoint_stats", "nks_autotune_entry"]
    src = tmp_path / "probe.c"
    body = "\n".join(f'printf("{s} %zu\\n", sizeof({s}));' for s in structs)
    src.write_text(f'#include <stdio.h>\n#include "nks.h"\nint main(void){{{body} return 0;}}\n')
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sizes = dict(zip(out[0::2], map(int, out[1::2])))
    for s in structs:
        assert C.sizeof(getattr(built, s)) == sizes[s], s


def test_error_path_without_gpu_work(built):
    # argument validation happens before any device call
    lib = built.load()
    h = C.c_void_p()
    assert lib.nks_setup_grid(None, C.byref(h)) == -1
    assert b"descriptor" in lib.nks_last_error()
    assert lib.nks_ras_apply(None, None, None) == -1
    assert lib.nks_destroy_grid(None) == 0


def test_adjoint_argument_checks_without_gpu_work(built):
    lib = built.load()
    assert lib.nks_adjoint(None, 1, None, None, 1.0, None, None, None, None, None, None) == -1
    assert lib.nks_matrix_transpose(None, None) == -1
    assert lib.nks_ras_apply_transpose(None, None, None) == -1
