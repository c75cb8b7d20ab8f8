"""The C-ABI library loads and exports every entry point include/tw.h declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2310_07119_amd import twa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|int64_t|const char\*)\s+(tw_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    assert set(_declared()) == set(twa.EXPORTS)


@pytest.mark.skipif(not os.path.exists(twa.LIB_PATH), reason="libtw.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(twa.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", twa.LIB_PATH], capture_output=True, text=True).stdout
    for name in _declared():
        assert re.search(r"\bT " + name + r"\b", out), name


@pytest.mark.skipif(not os.path.exists(twa.LIB_PATH), reason="libtw.so not built")
def test_argument_validation_without_gpu():
    """tw_plan_create rejects bad problems before touching the device."""
    lib = twa.load_library()
    bad = [dict(dim=4), dict(n=(100, 1, 1)), dict(hbar_m=-1.0), dict(n_real=0), dict(precision=7),
           dict(n=(64, 2, 1), dim=1), dict(G=float("nan")), dict(n_tot=0.0), dict(n=(4, 64, 1), dim=2)]
    for over in bad:
        pr = twa.TwProblem()
        pr.dim = over.get("dim", 1)
        n = over.get("n", (64, 1, 1))
        for d in range(3):
            pr.n[d] = n[d]
            pr.box[d] = 1.0
        pr.hbar_m = over.get("hbar_m", 1.0)
        pr.G = over.get("G", 1.0)
        pr.m_tot = 1.0
        pr.n_tot = over.get("n_tot", 100.0)
        pr.n_real = over.get("n_real", 4)
        pr.precision = over.get("precision", 0)
        h = ctypes.c_void_p()
        rc = lib.tw_plan_create(ctypes.byref(pr), ctypes.byref(h))
        assert rc in (-1, -2), (over, rc)
        assert lib.tw_last_error().decode()
    assert lib.tw_sample(None, None, 0, 0, None, None) == -1
    assert lib.tw_step(None, None, None, 1, 0.1, None) == -1
    assert lib.tw_moments(None, None, None, None, None) == -1
    assert lib.tw_plan_destroy(None) == 0
