"""Parity at the workloads' own shapes, in the launch configuration the
benchmark times (all realizations of the workload in one plan).

Where the oracle can run the whole workload it does (1D: 64 realizations x
1000 steps). At full 2D/3D size it recomputes sampled realizations one by one
from the same seed, and the moment reductions are checked against the oracle's
moments of the very state the GPU produced."""
import numpy as np
import pytest
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Plan, Problem, inputs
from tests.gpu_util import TOL, oracle_problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem(name, precision, **over):
    w = dict(inputs.WORKLOADS[name])
    w.update(over)
    return Problem(n=w["n"], box=w["box"], hbar_m=w["hbar_m"], G=w["G"], m_tot=w["m_tot"], n_tot=w["n_tot"],
                   n_real=w["n_real"], precision=precision), w


def test_1d_workload_complete_run_fp64():
    """64 realizations of the 256-point 1D field, all 1000 steps, every output."""
    p, w = _problem("1d_n256", "fp64")
    psi_cl = inputs.initial_field("1d_n256")
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 0)
    clt = cl.clone()
    plan.step(psi, w["nsteps"], w["dt"], clt)
    m = plan.moments(psi, clt, modes=True)
    prob = oracle_problem(p)
    opsi, ocl, om = tw.run(prob, psi_cl, p.n_real, p.n_tot, 0, w["nsteps"], w["dt"])
    tol = TOL["fp64"]
    assert rel(psi.cpu().numpy(), opsi) < tol
    assert rel(clt.cpu().numpy(), ocl) < tol
    assert rel(m["mode_occ"].cpu().numpy(), tw.moments(prob, opsi, p.n_tot, modes=True)["mode_occ"]) < tol
    for k in ("mean_psi", "mean_rho", "var_rho", "norm", "energy"):
        assert rel(m[k].cpu().numpy(), om[k]) < tol, k
    for k in ("Q_raw", "dev_rho_L1", "dev_psi_L2"):
        assert abs(m[k] - om[k]) < tol * abs(om[k]), k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_2d_workload_full_size_sampled(precision):
    """512^2, 256 realizations + classical, 5 steps; realizations 0, 131, 255
    recomputed by the oracle; moments vs the oracle's moments of the GPU state."""
    p, w = _problem("2d_n512_pair", precision)
    psi_cl = inputs.initial_field("2d_n512_pair")
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    seed, nsteps = 77, 5
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    plan.step(psi, nsteps, w["dt"], clt)
    m = plan.moments(psi, clt, modes=True, decoherence=True)
    host = psi.cpu().numpy()
    prob = oracle_problem(p)
    tol = TOL[precision]
    for r in (0, 131, 255):
        x0 = tw.sample(prob.grid, psi_cl, 1, p.n_tot, seed, real_offset=r)
        if precision == "fp32":
            x0 = x0.astype(np.complex64).astype(np.complex128)
        ref = tw.evolve(prob, x0, nsteps, w["dt"])[0]
        assert rel(host[r], ref) < tol, r
    om = tw.moments(prob, host.astype(np.complex128), p.n_tot, clt.cpu().numpy().astype(np.complex128), modes=True,
                    decoherence_=True)
    for k in ("mean_psi", "mean_rho", "var_rho", "norm", "var_amp", "var_phase"):
        assert rel(m[k].cpu().numpy(), om[k]) < 1e-12, k
    # mode occupations: the GPU transforms in the plan's precision
    assert rel(m["mode_occ"].cpu().numpy(), om["mode_occ"]) < (1e-12 if precision == "fp64" else 1e-5)
    for k in ("Q_raw", "dev_rho_L1", "dev_psi_L2", "Var_A", "Var_phi"):
        assert abs(m[k] - om[k]) < 1e-11 * abs(om[k]), k
    del psi, host
    plan.close()
    torch.cuda.empty_cache()


def test_3d_workload_full_size_sampled_fp32():
    """128^3 FP32-split, 64 realizations, 4 steps; two realizations recomputed by the oracle."""
    p, w = _problem("3d_n128_grf", "fp32")
    psi_cl = inputs.initial_field("3d_n128_grf")
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    seed, nsteps = 5, 4
    psi = plan.sample(cl, seed)
    plan.step(psi, nsteps, w["dt"])
    prob = oracle_problem(p)
    for r in (0, 63):
        x0 = tw.sample(prob.grid, psi_cl, 1, p.n_tot, seed, real_offset=r).astype(np.complex64)
        ref = tw.evolve(prob, x0.astype(np.complex128), nsteps, w["dt"])[0]
        assert rel(psi[r].cpu().numpy(), ref) < TOL["fp32"], r
    plan.close()


def test_3d_subset_32cube_fp32_vs_oracle():
    """The 3D Gaussian-random-field workload regenerated at 32^3 (cut at the
    Nyquist index), FP32-split vs the FP64 oracle over 300 steps, 16 realizations."""
    p, w = _problem("3d_n128_grf", "fp32", n=(32, 32, 32), n_real=16, n_tot=1e3 * 32 ** 3)
    psi_cl = inputs.initial_field("3d_n128_grf", n=(32, 32, 32))
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 11)
    clt = cl.to(torch.complex64).clone()
    nsteps = 300
    plan.step(psi, nsteps, w["dt"], clt)
    m = plan.moments(psi, clt)
    prob = oracle_problem(p)
    x0 = psi.new_empty(0)  # placeholder to keep names short
    x0 = tw.sample(prob.grid, psi_cl, p.n_real, p.n_tot, 11).astype(np.complex64).astype(np.complex128)
    opsi = tw.evolve(prob, x0, nsteps, w["dt"])
    ocl = tw.evolve(prob, psi_cl.astype(np.complex64).astype(np.complex128), nsteps, w["dt"])
    om = tw.moments(prob, opsi, p.n_tot, ocl)
    for k in ("mean_rho", "var_rho", "mean_psi", "norm", "energy"):
        assert rel(m[k].cpu().numpy(), om[k]) < TOL["fp32"], k


def test_3d_subset_32cube_fp64_full_horizon_vs_oracle():
    """The same 32^3 regeneration over the workload's full horizon (2000 steps)
    in FP64: three realizations and the classical field against the oracle at
    1e-10 (a 1e-15 perturbation of the initial ensemble moves the oracle's
    final state by 2e-14 over this horizon, so rounding is not amplified)."""
    p, w = _problem("3d_n128_grf", "fp64", n=(32, 32, 32), n_real=3, n_tot=1e3 * 32 ** 3)
    psi_cl = inputs.initial_field("3d_n128_grf", n=(32, 32, 32))
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 11)
    clt = cl.clone()
    plan.step(psi, w["nsteps"], w["dt"], clt)
    m = plan.moments(psi, clt)
    prob = oracle_problem(p)
    opsi, ocl, om = tw.run(prob, psi_cl, p.n_real, p.n_tot, 11, w["nsteps"], w["dt"])
    tol = TOL["fp64"]
    assert rel(psi.cpu().numpy(), opsi) < tol
    assert rel(clt.cpu().numpy(), ocl) < tol
    for k in ("mean_psi", "mean_rho", "var_rho", "norm", "energy"):
        assert rel(m[k].cpu().numpy(), om[k]) < 10 * tol, k
    for k in ("Q_raw", "dev_rho_L1", "dev_psi_L2"):
        assert abs(m[k] - om[k]) < 10 * tol * abs(om[k]), k
    plan.close()
