"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, and rejects invalid graphs and
arguments before touching the device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nvd.h")


def _lib():
    from paper_2310_11222_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libnvd.so not built (run __graft_entry__.build())")
    return _abi.load(), _abi


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nvd_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for must in ["nvd_graph_create", "nvd_distances", "nvd_laplacian_apply", "nvd_project",
                 "nvd_grad_weights", "nvd_batch_create", "nvd_batch_distances"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib, abi = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(nvd_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # and the binding declares the same set
    assert set(abi.SIGNATURES) == set(_declared())


def test_version_and_strings():
    lib, abi = _lib()
    assert lib.nvd_abi_version() == 1
    assert lib.nvd_status_string(abi.NVD_E_GRAPH) == b"invalid graph"
    o = abi.NvdOpts()
    assert lib.nvd_opts_default(C.byref(o)) == 0
    assert o.precision == abi.NVD_FP64 and o.rtol == 1e-10 and o.tile_k == 0


def _create(lib, n, rp, ci, w=None):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    wp = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    h = C.c_void_p()
    st = lib.nvd_graph_create(n, ci.size, rp.ctypes.data_as(C.c_void_p),
                              ci.ctypes.data_as(C.c_void_p),
                              None if wp is None else wp.ctypes.data_as(C.c_void_p), None,
                              C.byref(h))
    return st, lib.nvd_last_error().decode()


@pytest.mark.parametrize("case", ["asym", "col_range", "neg_weight", "nan_weight", "dup",
                                  "rp_monotone", "rp_end", "weight_mismatch"])
def test_graph_validation_rejects(case):
    lib, abi = _lib()
    n = 3
    rp = [0, 2, 4, 6]
    ci = [1, 2, 0, 2, 0, 1]
    w = [1.0] * 6
    if case == "asym":
        rp, ci = [0, 1, 1, 1], [1]
        w = None
    elif case == "col_range":
        ci = [1, 3, 0, 2, 0, 1]
    elif case == "neg_weight":
        w = [1.0, -1.0, 1.0, 1.0, -1.0, 1.0]
    elif case == "nan_weight":
        w = [1.0, float("nan"), 1.0, 1.0, float("nan"), 1.0]
    elif case == "dup":
        rp, ci, w = [0, 2, 4, 4], [1, 1, 0, 0], None
    elif case == "rp_monotone":
        rp = [0, 3, 2, 6]
    elif case == "rp_end":
        rp = [0, 2, 4, 5]
    elif case == "weight_mismatch":
        w = [1.0, 2.0, 1.0, 1.0, 3.0, 1.0]
    st, msg = _create(lib, n, rp, ci, w)
    assert st == abi.NVD_E_GRAPH, (st, msg)
    assert msg


def test_argument_errors():
    lib, abi = _lib()
    h = C.c_void_p()
    assert lib.nvd_graph_create(0, 0, None, None, None, None, C.byref(h)) == abi.NVD_E_ARG
    assert lib.nvd_graph_create(5, 0, None, None, None, None, None) == abi.NVD_E_ARG
    big = np.zeros(2, dtype=np.int64)
    assert lib.nvd_graph_create(2 ** 31, 0, big.ctypes.data_as(C.c_void_p), None, None, None,
                                C.byref(h)) == abi.NVD_E_UNSUPPORTED
    assert lib.nvd_distances(None, 1, None, None, 1, None, None, None, 0, None, None) == abi.NVD_E_ARG
    assert lib.nvd_laplacian_apply(None, 0, 1, None, 1, None, 1, None) == abi.NVD_E_ARG
    assert lib.nvd_opts_default(None) == abi.NVD_E_ARG
    assert lib.nvd_pairwise(None, 4, None, 4, None, None, 4, None, 0, None, None) == abi.NVD_E_ARG
    # graph from device arrays: flag and argument checks come first
    assert lib.nvd_graph_create_ex(3, 0, None, None, None, 4, None, C.byref(h)) == abi.NVD_E_ARG
    assert lib.nvd_graph_create_ex(3, 6, None, None, None, abi.NVD_PTR_DEVICE, None,
                                   C.byref(h)) == abi.NVD_E_ARG
    assert lib.nvd_graph_create_ex(2 ** 31, 0, big.ctypes.data_as(C.c_void_p), None, None,
                                   abi.NVD_PTR_DEVICE, None, C.byref(h)) == abi.NVD_E_ARG
    # adjoint entry points
    assert lib.nvd_grad_vectors(None, 1, None, 1, None, None, 1, None, 1, None) == abi.NVD_E_ARG
    assert lib.nvd_grad_scale_from_d(0, None, None, None, None) == abi.NVD_E_ARG
    assert lib.nvd_grad_weights(None, 1, None, 1, None, None, None) == abi.NVD_E_ARG


def test_host_graph_create_ex_matches_create():
    """nvd_graph_create_ex with NVD_PTR_HOST validates like nvd_graph_create
    (the invalid graph is rejected before any device work)."""
    lib, abi = _lib()
    rp = np.array([0, 1, 1, 1], dtype=np.int64)
    ci = np.array([1], dtype=np.int32)
    h = C.c_void_p()
    st = lib.nvd_graph_create_ex(3, 1, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
                                 None, abi.NVD_PTR_HOST, None, C.byref(h))
    assert st == abi.NVD_E_GRAPH
    assert b"mirror" in lib.nvd_last_error()


def test_binding_output_checks_on_host_tensors():
    """The binding refuses an output buffer that is not a CUDA tensor before
    the library is called (the check needs no GPU)."""
    torch = pytest.importorskip("torch")
    from paper_2310_11222_amd import _check_out
    with pytest.raises(ValueError):
        _check_out(torch.empty(4, dtype=torch.float64), "out", (4,), torch.float64)
    with pytest.raises(ValueError):
        _check_out(np.empty(4), "out", (4,), torch.float64)
