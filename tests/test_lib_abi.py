"""CPU-side checks of the C ABI: the library builds for gfx950, loads, and
exports every function declared in include/muoncave.h.  No compute calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "muoncave.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("load_geometry_grid", "set_sensors", "set_counts", "logpost_batch",
                     "logpost_grad_batch", "mcmc_run", "mc_create", "mc_destroy", "mc_last_error"):
        assert required in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2603_28907_amd import binding
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.mc_version()
    for name in binding.EXPORTED_SYMBOLS:
        assert name in declared_functions()


def test_create_without_gpu_reports_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2603_28907_amd import binding
    lib = binding.load_library()
    h = ctypes.c_void_p()
    st = lib.mc_create(0, 0, ctypes.byref(h))
    assert st != 0
    assert lib.mc_last_error(None)


def test_server_create_without_gpu_reports_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2603_28907_amd import binding
    lib = binding.load_library()
    h = ctypes.c_void_p()
    cfg = binding.ServerConfig(0, 0, 0, 0, 4, 10)
    assert lib.mc_server_create(ctypes.byref(cfg), ctypes.byref(h)) != 0
    assert lib.mc_server_last_error(None)
    bad = binding.ServerConfig(0, 0, 0, 0, 0, 10)
    assert lib.mc_server_create(ctypes.byref(bad), ctypes.byref(h)) == -1   # MC_ERR_ARG before any device call


def test_every_declared_symbol_has_a_binding():
    from paper_2603_28907_amd import binding
    missing = [n for n in declared_functions() if n not in binding.EXPORTED_SYMBOLS]
    assert missing == []
