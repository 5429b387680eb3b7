"""CPU checks of the boundary: the built HIP library loads and exports every
function that include/kfmi.h declares; the binding refuses to run without it."""
import ctypes
import os

import pytest

from paper_1705_02876_amd import kfmi


def test_header_declares_the_core_calls():
    syms = kfmi.header_symbols()
    for s in ("kf_ctx_create", "kf_ctx_destroy", "kf_last_error", "kf_set_geometry", "kf_propagate_to_r",
              "kf_update", "kf_fit"):
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
