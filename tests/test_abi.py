"""The C-ABI library loads and exports every symbol include/ecc.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1806_02637_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions(header="ecc.h"):
    with open(os.path.join(ROOT, "include", header)) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecc_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    declared = _declared_functions()
    assert declared, "no declarations parsed"
    assert sorted(binding.SYMBOLS) == declared
    assert sorted(binding.PROBE_SYMBOLS) == _declared_functions("ecc_probe.h")


def test_library_exports_every_declared_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libecc.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in _declared_functions() + _declared_functions("ecc_probe.h"):
        assert hasattr(lib, name), name


def test_status_codes_and_eval_params_layout(tmp_path):
    # the ctypes mirror must match the C header's struct, field by field
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "ecc.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ecc_eval_params),'
        ' offsetof(ecc_eval_params, K), offsetof(ecc_eval_params, geom), offsetof(ecc_eval_params, R_mm),'
        ' offsetof(ecc_eval_params, c), offsetof(ecc_eval_params, kappa_range),'
        ' offsetof(ecc_eval_params, reserved)); return 0; }\n')
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    c_layout = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    E = binding.EvalParams
    py_layout = [ctypes.sizeof(E)] + [getattr(E, f).offset for f in ("K", "geom", "R_mm", "c", "kappa_range", "reserved")]
    assert c_layout == py_layout
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "ecc.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(ecc_volume), offsetof(ecc_volume, nx),'
        ' offsetof(ecc_volume, ny), offsetof(ecc_volume, nz), offsetof(ecc_volume, reserved),'
        ' offsetof(ecc_volume, voxel_mm)); return 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    c_layout = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    V = binding.EccVolume
    assert c_layout == [ctypes.sizeof(V)] + [getattr(V, f).offset for f in ("nx", "ny", "nz", "reserved", "voxel_mm")]
    assert (binding.ECC_KAPPA_OBJECT, binding.ECC_KAPPA_DETECTOR) == (0, 1)
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
