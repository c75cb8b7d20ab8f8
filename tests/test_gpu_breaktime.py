"""Q(t) recorded on the GPU over a collapse (the 2D momentum-space Gaussian
regenerated at 64^2) against the oracle's Q at the same times, and the
breaktime fits on both series."""
import numpy as np
import pytest
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Plan, Problem, breaktime as bt, inputs
from tests.gpu_util import oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_q_series_and_fits_vs_oracle():
    w = inputs.WORKLOADS["2d_n512_kgauss"]
    n, nreal, nsteps, every, seed = (64, 64), 32, 30, 5, 21
    n_tot = 1e3 * 64 * 64
    p = Problem(n=n, box=w["box"], hbar_m=w["hbar_m"], G=w["G"], m_tot=w["m_tot"], n_tot=n_tot, n_real=nreal,
                precision="fp64")
    psi_cl = inputs.initial_field("2d_n512_kgauss", n=n)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.clone()
    rec = bt.record(plan, psi, clt, nsteps, w["dt"], every, modes=True)
    plan.close()

    prob = oracle_problem(p)
    opsi = tw.sample(prob.grid, psi_cl, nreal, n_tot, seed)
    ocl = psi_cl.copy()
    ref = {k: [] for k in ("Q_raw", "Q_sym", "dev_rho_L1", "mode_occ")}
    for i in range(nsteps // every + 1):
        if i:
            opsi = tw.evolve(prob, opsi, every, w["dt"])
            ocl = tw.evolve(prob, ocl, every, w["dt"])
        m = tw.moments(prob, opsi, n_tot, ocl, modes=True)
        for k in ref:
            ref[k].append(m[k])
    assert np.allclose(rec["t"], w["dt"] * every * np.arange(nsteps // every + 1))
    for k in ("Q_raw", "dev_rho_L1"):
        assert np.allclose(rec[k], ref[k], rtol=1e-10, atol=0), k
    assert np.allclose(rec["Q_sym"], ref["Q_sym"], rtol=0, atol=1e-10 * max(ref["Q_raw"]))
    # the series the paper analyses: the sampled initial value subtracted
    ref_d = np.asarray(ref["Q_raw"]) - ref["Q_raw"][0]
    assert rec["Q_minus_Q0"][0] == 0.0
    assert np.allclose(rec["Q_minus_Q0"], ref_d, rtol=0, atol=1e-10 * max(ref["Q_raw"]))
    for got, want in zip(rec["mode_occ"], ref["mode_occ"]):
        assert np.linalg.norm(got - want) < 1e-10 * np.linalg.norm(want)
    # Q grows during the collapse; fits on both series agree
    assert rec["Q_minus_Q0"][-1] > 10 * abs(rec["Q_minus_Q0"][1])
    t, q = rec["t"][1:], rec["Q_minus_Q0"][1:]
    la, lam = bt.fit_exponential(t, q)
    la_o, lam_o = bt.fit_exponential(t, ref_d[1:])
    assert abs(lam - lam_o) < 1e-7 * abs(lam_o) and abs(la - la_o) < 1e-7 * abs(la_o)
    k, spec, cnt = bt.shell_spectrum(rec["mode_occ"][-1], w["box"])
    assert cnt.sum() == 64 * 64 and np.all(spec > 0)
