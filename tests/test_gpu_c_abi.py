"""The C ABI used from a plain host program (tests/c_abi_example.cpp, built
next to libtw.so): sampling, stepping with the classical field, and the
moment scalars, compared with the oracle on the same seeded input."""
import os
import subprocess

import numpy as np
import pytest

from oracle import twa_oracle as tw
from tests.gpu_util import TOL, rel

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_2310_07119_amd", "tw_c_example")

NX, NY, NREAL, NSTEPS, DT, SEED = 64, 32, 3, 6, 2e-4, 7
BOX = (1.0, 0.5)
HBAR_M, G, M_TOT, N_TOT = 1.0, 1.0, 20.0, 1e5


def _initial_field():
    """The program's coherent field: sqrt of 1 + 0.3 cos(2 pi x/nx) + 0.2 sin(2 pi y/ny), unit norm."""
    x = np.arange(NX)[None, :]
    y = np.arange(NY)[:, None]
    rho = 1.0 + 0.3 * np.cos(2.0 * np.pi * x / NX) + 0.2 * np.sin(2.0 * np.pi * y / NY)
    dv = (BOX[0] / NX) * (BOX[1] / NY)
    psi = np.sqrt(rho).astype(np.complex128)
    return psi / np.sqrt(np.sum(rho) * dv)


def test_c_program_matches_oracle(tmp_path):
    if not os.path.exists(EXAMPLE):
        raise RuntimeError(f"{EXAMPLE} is missing: build the library first")
    out = tmp_path / "tw_c_example.bin"
    print(f"running {EXAMPLE}", flush=True)
    r = subprocess.run([EXAMPLE, str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = np.fromfile(out, dtype=np.float64)
    ncell = NX * NY
    assert raw.size == 2 * ncell * (NREAL + 2) + 8
    c = raw[: 2 * ncell].view(np.complex128).reshape(NY, NX)
    psi = raw[2 * ncell: 2 * ncell * (NREAL + 1)].view(np.complex128).reshape(NREAL, NY, NX)
    clt = raw[2 * ncell * (NREAL + 1): 2 * ncell * (NREAL + 2)].view(np.complex128).reshape(NY, NX)
    scal = raw[-8:]

    psi_cl = _initial_field()
    assert rel(c, psi_cl) < 1e-14
    prob = tw.Problem(tw.Grid((NX, NY), BOX), HBAR_M, G, M_TOT)
    opsi, ocl, om = tw.run(prob, psi_cl, NREAL, N_TOT, SEED, NSTEPS, DT)
    assert rel(psi, opsi) < TOL["fp64"]
    assert rel(clt, ocl) < TOL["fp64"]
    assert abs(scal[0] - om["Q_raw"]) < TOL["fp64"] * abs(om["Q_raw"])
    assert abs(scal[5] - np.mean(om["norm"])) < TOL["fp64"]
    assert scal[6] == 0.0
