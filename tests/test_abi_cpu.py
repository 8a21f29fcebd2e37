"""The C-ABI library builds, loads and exports every entry point that
include/ba.h declares.  Host-side argument checks that touch no device run
here too; no compute call is made (no GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ba.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ba_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2608_14266_amd import build as hb
    if not os.path.exists(hb.LIB):
        hb.build()
    return ct.CDLL(hb.LIB)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("ba_build_clusters", "ba_eval_residual_grad_hessian", "ba_solve_increment", "ba_iterate"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_status_strings(lib):
    lib.ba_status_str.restype = ct.c_char_p
    lib.ba_status_str.argtypes = [ct.c_int32]
    assert lib.ba_status_str(0) == b"ok"
    assert lib.ba_status_str(-1) == b"invalid argument"
    assert lib.ba_status_str(-4) == b"matrix not positive definite"


def test_null_arguments_rejected_without_device(lib):
    P = ct.c_void_p
    lib.ba_build_clusters.restype = ct.c_int32
    lib.ba_build_clusters.argtypes = [P, P, P, P]
    out = ct.c_void_p()
    assert lib.ba_build_clusters(None, None, ct.byref(out), None) == -1
    lib.ba_iterate.restype = ct.c_int32
    lib.ba_iterate.argtypes = [P, P, P, P, P, P]
    assert lib.ba_iterate(None, None, None, None, None, None) == -1
    lib.ba_eval_residual_grad_hessian.restype = ct.c_int32
    lib.ba_eval_residual_grad_hessian.argtypes = [P, P, ct.c_int32, P, P, P, P, P]
    assert lib.ba_eval_residual_grad_hessian(None, None, 0, None, None, None, None, None) == -1
    lib.ba_last_error.restype = ct.c_char_p
    assert len(lib.ba_last_error()) > 0


def test_solve_workspace_query(lib):
    lib.ba_solve_increment_workspace.restype = ct.c_size_t
    lib.ba_solve_increment_workspace.argtypes = [ct.c_int32, ct.c_int32]
    assert lib.ba_solve_increment_workspace(0, 10) > 0
    assert lib.ba_solve_increment_workspace(0, 0) == 0
    assert lib.ba_solve_increment_workspace(7, 10) == 0


def test_binding_checks_solve_shapes():
    """The Python binding derives the scan count from grad and rejects a hess
    whose size does not match it (no silent truncation to whole scans)."""
    import torch
    from paper_2608_14266_amd import _lib
    g = torch.zeros(12, dtype=torch.float64)
    assert _lib._solve_scans(_lib.MODE_MM, torch.zeros(72, dtype=torch.float64), g) == 2
    assert _lib._solve_scans(_lib.MODE_COUPLED, torch.zeros(144, dtype=torch.float64), g) == 2
    with pytest.raises(ValueError):
        _lib._solve_scans(_lib.MODE_COUPLED, torch.zeros(72, dtype=torch.float64), g)
    with pytest.raises(ValueError):
        _lib._solve_scans(_lib.MODE_COUPLED, torch.zeros(200 * 200, dtype=torch.float64),
                          torch.zeros(200, dtype=torch.float64))
    with pytest.raises(ValueError):
        _lib._solve_scans(_lib.MODE_MM, torch.zeros(0, dtype=torch.float64), torch.zeros(0, dtype=torch.float64))
