"""Each plausible mistake in the oracle must fail one of the pins that tie
it to the mathematics (``pins.py``), not only its own golden record: a copy
of ``oracle/`` gets one planted change, and the pin named for it must raise.
The unchanged copy passes every pin (the harness itself changes nothing)."""
import importlib
import os
import shutil
import sys

import pytest

import pins

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

LOOKUP, HIT, KAPPA, COSINE = (pins.check_lookup_closed_form, pins.check_hit_test, pins.check_kappa_max,
                              pins.check_cosine_weight)

# (name, file, text as written, planted text, checks that must fail)
MUTATIONS = [
    ("no Grangeat weight", "ecc.py", "weight = 1.0 + t * t / (f * f)", "weight = 1.0 + 0.0 * t", [LOOKUP]),
    ("half the Grangeat weight", "ecc.py", "weight = 1.0 + t * t / (f * f)", "weight = 1.0 + 0.5 * t * t / (f * f)",
     [LOOKUP]),
    ("no fold sign", "ecc.py", "sign = np.where(flip, -1.0, 1.0)", "sign = np.where(flip, 1.0, 1.0)", [LOOKUP]),
    ("no hit test", "ecc.py", "hit = ok & (np.abs(tv) <=", "hit = ok | (np.abs(tv) <=", [HIT]),
    ("hit rectangle twice the detector", "ecc.py", "0.5 * grid.W * np.abs(np.cos(av))", "grid.W * np.abs(np.cos(av))",
     [HIT]),
    ("no cosine weight", "sinogram.py", "return img * (f / np.sqrt(f * f + x[None, :] ** 2 + y[:, None] ** 2))",
     "return img * 1.0", [COSINE, LOOKUP]),
    ("kappa_max = asin(R / 2h)", "geometry.py", "ratio = R_mm / h", "ratio = R_mm / (2.0 * h)", [KAPPA]),
    ("t offset by half a cell", "ecc.py", "tau = (t + grid.t_max) / grid.dt", "tau = (t + grid.t_max) / grid.dt + 0.5",
     [LOOKUP]),
    ("alpha and t fractions swapped", "ecc.py",
     "interp = (1.0 - fa) * ((1.0 - ft) * s00 + ft * s01) + fa * ((1.0 - ft) * s10 + ft * s11)",
     "interp = (1.0 - ft) * ((1.0 - fa) * s00 + fa * s01) + ft * ((1.0 - fa) * s10 + fa * s11)", [LOOKUP]),
    ("cell derivative reversed", "sinogram.py", "d = (g_hi - g_lo) / (2.0 * grid.dt)",
     "d = (g_lo - g_hi) / (2.0 * grid.dt)", [LOOKUP]),
    ("row derivative reversed", "sinogram.py", "d = (Gp[:, 2:] - Gp[:, :-2]) / (2.0 * grid.dt)",
     "d = (Gp[:, :-2] - Gp[:, 2:]) / (2.0 * grid.dt)", [COSINE]),
    ("h from the source instead of the baseline", "geometry.py", "h = ops.sqrt(dot3(w, w))",
     "h = ops.sqrt(dot3(C_a, C_a))", [KAPPA]),
]


def _mutant(tmp_path, tag, fname=None, old=None, new=None):
    pkg = f"oracle_mutant_{tag}"
    dst = tmp_path / pkg
    shutil.copytree(ORACLE_DIR, dst, ignore=shutil.ignore_patterns("__pycache__", "*.tmp*"))
    if fname is not None:
        path = dst / fname
        src = path.read_text()
        assert src.count(old) == 1, f"{fname}: the text to change occurs {src.count(old)} times"
        path.write_text(src.replace(old, new))
    sys.path.insert(0, str(tmp_path))
    try:
        return importlib.import_module(pkg)
    finally:
        sys.path.remove(str(tmp_path))


def test_unchanged_copy_passes_every_pin(tmp_path):
    mod = _mutant(tmp_path, "identity")
    for check in (LOOKUP, HIT, KAPPA, COSINE):
        check(mod)


@pytest.mark.parametrize("name,fname,old,new,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_its_pin(tmp_path, name, fname, old, new, checks):
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    mod = _mutant(tmp_path, tag, fname, old, new)
    for check in checks:
        with pytest.raises(AssertionError):
            check(mod)
