"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")
PKG = os.path.join(ROOT, "paper_2607_27644_amd")


def declared_symbols():
    """Every function declared in include/*.h."""
    txt = "".join(open(os.path.join(INCLUDE, f)).read() for f in sorted(os.listdir(INCLUDE)) if f.endswith(".h"))
    return sorted(set(re.findall(r"\b(rbp_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for must in ("rbp_code_create", "rbp_sample", "rbp_decode", "rbp_decode_multi", "rbp_trace",
                 "rbp_mlp_forward", "rbp_mlp_train_step", "rbp_mlp_save", "rbp_mlp_load", "rbp_last_error"):
        assert must in syms


def test_library_exports_every_declared_symbol():
    lib_path = os.path.join(PKG, "librbp.so")
    if not os.path.exists(lib_path):
        pytest.fail("librbp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(lib_path)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    lib.rbp_last_error.restype = ctypes.c_char_p
    assert lib.rbp_last_error() is not None


def test_fp32_network_test_build_exports_the_network_entry_points():
    """librbp_mlp_f32.so, the FP32 test build of the network kernels, exports
    the same rbp_mlp_* entry points (and nothing of the decoder)."""
    path = os.path.join(PKG, "librbp_mlp_f32.so")
    if not os.path.exists(path):
        pytest.fail("librbp_mlp_f32.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    mlp = [s for s in declared_symbols() if s.startswith("rbp_mlp_")]
    assert len(mlp) >= 8
    assert all(hasattr(lib, s) for s in mlp + ["rbp_last_error"])
    assert not hasattr(lib, "rbp_decode")


def test_host_validation_without_gpu():
    """Argument checks run before any device call."""
    lib = ctypes.CDLL(os.path.join(PKG, "librbp.so"))
    lib.rbp_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    i32 = ctypes.c_int32
    # row with degree 1 -> UNSUPPORTED
    cp = (i32 * 3)(0, 1, 2)
    ri = (i32 * 2)(0, 1)
    assert lib.rbp_code_create(2, 2, cp, ri, 0, None, None, ctypes.byref(out)) == -3
    # unsorted rows inside a column -> SHAPE
    cp = (i32 * 2)(0, 2)
    ri = (i32 * 2)(1, 0)
    assert lib.rbp_code_create(2, 1, cp, ri, 0, None, None, ctypes.byref(out)) == -2
    assert b"ascending" in lib.rbp_last_error()
    # row index out of range -> SHAPE
    ri = (i32 * 2)(0, 5)
    assert lib.rbp_code_create(2, 1, cp, ri, 0, None, None, ctypes.byref(out)) == -2
    # NULL handle -> INVALID_ARG
    assert lib.rbp_decode(None, None, None, 0, None, None, None, None, None, None) == -1


def test_product_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b|orc_|liboracle", txt, re.M), f


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_2607_27644_amd import rbp
    monkeypatch.setattr(rbp, "_lib", None)
    monkeypatch.setattr(rbp, "LIB_PATH", os.path.join(PKG, "does_not_exist.so"))
    with pytest.raises(RuntimeError, match="not built"):
        rbp.lib()


def test_resident_and_each_validation_without_gpu():
    """The resident decoder's and rbp_decode_each's argument checks return
    INVALID_ARG before any device call; stopping a NULL handle is a no-op."""
    lib = ctypes.CDLL(os.path.join(PKG, "librbp.so"))
    lib.rbp_last_error.restype = ctypes.c_char_p
    vp = ctypes.c_void_p
    out = vp()
    assert lib.rbp_resident_start(None, None, None, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.rbp_resident_decode(None, None, None, None, None) == -1
    assert b"NULL" in lib.rbp_last_error()
    assert lib.rbp_resident_info(None, None, None, None, None) == -1
    assert lib.rbp_resident_stop(None) == 0
    # rbp_decode_each: model count out of range, NULL arrays, NULL handle
    assert lib.rbp_decode_each(0, None, None, None, None, None, None, None, None, None) == -1
    assert lib.rbp_decode_each(9, None, None, None, None, None, None, None, None, None) == -1
    assert lib.rbp_decode_each(1, None, None, None, None, None, None, None, None, None) == -1
    codes = (vp * 1)(None)
    shots = (ctypes.c_uint64 * 1)(0)
    arr = (vp * 1)(None)

    class Params(ctypes.Structure):
        _fields_ = [("gamma0", ctypes.c_float), ("gamma_min", ctypes.c_float), ("gamma_max", ctypes.c_float),
                    ("pre_iter", ctypes.c_int32), ("max_iterations", ctypes.c_int32), ("num_sets", ctypes.c_int32),
                    ("stop_nconv", ctypes.c_int32), ("stopping_criterion", ctypes.c_int32),
                    ("gamma_seed", ctypes.c_uint64)]
    prm = Params(0.125, -0.24, 0.66, 80, 60, 100, 5, 0, 0)
    assert lib.rbp_decode_each(1, codes, arr, shots, arr, ctypes.byref(prm), arr, arr, None, None) == -1
    assert b"code is NULL" in lib.rbp_last_error()


def test_position_order_validation_without_gpu():
    """rbp_code_positions, rbp_decode_proposal_pos and rbp_mlp_set_output_order
    reject NULL handles before any device call."""
    lib = ctypes.CDLL(os.path.join(PKG, "librbp.so"))
    lib.rbp_last_error.restype = ctypes.c_char_p
    n = ctypes.c_int32()
    assert lib.rbp_code_positions(None, ctypes.byref(n), None) == -1
    assert lib.rbp_decode_proposal_pos(None, None, None, 0, None, None, None, None, None, None) == -1
    assert lib.rbp_mlp_set_output_order(None, None, 0) == -1
