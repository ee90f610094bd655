"""The C ABI: every symbol include/dd.h declares is exported; host-only error paths."""

import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "dd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1708_02845_amd import _lib
    return _lib.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("dd_create", "dd_destroy", "dd_load_kernel_dense", "dd_load_kernel_csr",
              "dd_distance_field", "dd_batch_distance_fields", "dd_trace_paths", "dd_plan_path",
              "dd_free_kernel", "dd_last_error", "dd_kernel_get_info", "dd_dense_footprint"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_1708_02845_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_null_handles_are_rejected_without_touching_the_device(lib):
    from paper_1708_02845_amd import _lib as L
    b = L.dd_error_bound()
    assert lib.dd_distance_field(None, 0, 0, None, C.byref(b), None) == L.DD_ESTATE
    assert b"not a live kernel" in lib.dd_last_error()
    assert lib.dd_free_kernel(None) == L.DD_ESTATE
    assert lib.dd_grid_poisson_kernel(None, 9, None, 0, 1, None, 0, None, 0, 1e-12, 10, 0, None,
                                      None) == L.DD_ESTATE
    assert lib.dd_destroy(None) == L.DD_ESTATE
    assert lib.dd_path_level1(None, -1, None, None) == L.DD_ESTATE
    n = C.c_int32()
    assert lib.dd_plan_path(None, 0, 1, 0, 10, None, C.byref(n), C.byref(n), None, None) \
        == L.DD_ESTATE


def test_footprint_is_host_arithmetic(lib):
    from paper_1708_02845_amd import Kernel
    N, B = 1000, 257
    ld = 260
    assert Kernel.dense_footprint(N, B) == N * ld * 4 + N * 8
    assert Kernel.dense_footprint(N, B, f64=True) == N * ld * 4 + N * 8 + N * B * 8
    lda = 320    # operand columns padded to a multiple of 64
    npad = 1024  # operand rows padded to a multiple of 128 (tile-major layout)
    assert Kernel.dense_footprint(N, B, gemm_form="f32") == N * ld * 4 + npad * lda * 4 + N * 8 + N * 4
    assert Kernel.dense_footprint(N, B, gemm_form="f16x3") == Kernel.dense_footprint(N, B, gemm_form="f32")
    from paper_1708_02845_amd import _lib as L
    out = C.c_size_t()
    assert lib.dd_dense_footprint(0, 5, 0, None, C.byref(out)) == L.DD_EINVAL


def test_python_layer_refuses_without_library(monkeypatch, tmp_path):
    from paper_1708_02845_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and offsetof of every struct the binding mirrors, from a C program
    compiled against include/dd.h, equal the ctypes layouts."""
    import shutil
    import subprocess
    from paper_1708_02845_amd import _lib as L
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"dd_load_opts": L.dd_load_opts, "dd_error_bound": L.dd_error_bound,
               "dd_kernel_info": L.dd_kernel_info, "dd_adjacency": L.dd_adjacency,
               "dd_grid_solve_stats": L.dd_grid_solve_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dd.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(x.split()[:2]): int(x.split()[2]) for x in out if x.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
