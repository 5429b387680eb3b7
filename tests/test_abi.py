"""CPU checks of the boundary: the built HIP library loads and exports every
function that include/kfmi.h declares; the binding refuses to run without it."""
import ctypes
import os

import pytest

from paper_1705_02876_amd import kfmi


def test_header_declares_the_core_calls():
    syms = kfmi.header_symbols()
    for s in ("kf_ctx_create", "kf_ctx_destroy", "kf_last_error", "kf_set_geometry", "kf_propagate_to_r",
              "kf_update", "kf_fit", "kf_smooth"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    if not os.path.exists(kfmi.LIB_PATH):
        pytest.fail("libkfmi.so not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(kfmi.LIB_PATH)
    missing = [s for s in kfmi.header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(kfmi, "_lib", None)
    with pytest.raises(RuntimeError, match="must be built"):
        kfmi.load_library(str(tmp_path / "nope.so"))


def test_geometry_struct_layout_matches_header():
    # n_layers + 3 x 32 floats + bz + eloss + mass
    assert ctypes.sizeof(kfmi.kf_geometry) == 4 + 3 * 32 * 4 + 3 * 4
    assert ctypes.sizeof(kfmi.kf_fit_args) == 19 * 8


def test_last_error_is_a_string_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("exercises the no-device error path")
    lib = kfmi.load_library()
    h = ctypes.c_void_p()
    rc = lib.kf_ctx_create(ctypes.byref(h), 0)
    assert rc != 0 and not h.value
    assert isinstance(lib.kf_last_error(), bytes)


def test_struct_layouts_match_the_c_header(tmp_path):
    """The ctypes structures have the sizes and field offsets the C compiler gives the header's structs."""
    import shutil
    import subprocess
    from paper_1705_02876_amd import kfmi_build as KB
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"kf_geometry": kfmi.kf_geometry, "kf_fit_args": kfmi.kf_fit_args,
               "kf_smooth_args": kfmi.kf_smooth_args, "kf_bin_args": KB.kf_bin_args,
               "kf_build_cfg": KB.kf_build_cfg, "kf_build_args": KB.kf_build_args}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{kfmi.HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[f"{name}.{fname}"]) == getattr(cls, fname).offset, f"{name}.{fname}"
