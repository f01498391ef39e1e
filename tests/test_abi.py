"""The C-ABI library loads and exports every symbol include/ecc.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1806_02637_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    with open(os.path.join(ROOT, "include", "ecc.h")) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecc_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert sorted(binding.SYMBOLS) == declared


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libecc.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_codes_and_eval_params_layout():
    assert ctypes.sizeof(binding.EvalParams) == 24
    assert (binding.ECC_OK, binding.ECC_E_ARG, binding.ECC_E_BUDGET, binding.ECC_E_HIP, binding.ECC_E_STATE,
            binding.ECC_E_NOSCAN) == (0, -1, -2, -3, -4, -5)


def test_null_context_is_an_argument_error_not_a_crash():
    # host-side argument checks run before any device call
    lib = binding.load_library()
    assert lib.ecc_destroy(None) == binding.ECC_E_ARG
    assert "null" in binding.ecc_last_error()
    assert lib.ecc_scan_free(None, 1) == binding.ECC_E_ARG
    params = binding.EvalParams(64, 0, 90.0, 0.0)
    assert lib.ecc_cost(None, 1, 1, None, ctypes.byref(params), None, None, None, 0, None) == binding.ECC_E_ARG
