"""D = 3 steps on the xy-plane schedule (three HBM passes per step: plane
passes along x and y with the plane in LDS, pencil passes along z) against
the oracle and against the pencil schedule on the same draws. Bars: 1e-10
(FP64) and 1e-4 (FP32) normwise, per realization and for the classical field;
odd and even step counts (the schedule alternates two kinds of step), odd
ensembles (a pair slot without partner), 3 * 2^k lengths."""
import numpy as np
import pytest
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Plan, Problem, inputs
from tests.gpu_util import TOL, oracle_problem, rel

pytestmark = pytest.mark.gpu

CASES = [
    # (n, precision, n_real)
    ((16, 16, 32), "fp64", 3),
    ((32, 32, 16), "fp64", 4),
    ((64, 64, 24), "fp64", 3),
    ((16, 16, 32), "fp32", 3),
    ((32, 32, 48), "fp32", 2),
    ((64, 64, 16), "fp32", 5),
    ((96, 96, 16), "fp32", 3),
    ((128, 128, 16), "fp32", 3),
]


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem(n, precision, nr):
    box = (1.0, 1.0, n[2] / n[0])
    return Problem(n=n, box=box, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=1e3 * int(np.prod(n)), n_real=nr,
                   precision=precision)


def _run(p, psi_cl, seed, nsteps, dt, slab, monkeypatch):
    monkeypatch.setenv("TW_SLAB", "1" if slab else "0")
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, seed)
    psi0 = psi.cpu().numpy()
    clt = cl.to(p.cdtype).clone()
    plan.step(psi, nsteps, dt, clt)
    m = plan.moments(psi, clt)
    torch.cuda.synchronize()
    out = psi0, psi.cpu().numpy(), clt.cpu().numpy(), m
    plan.close()
    return out


@pytest.mark.parametrize("nsteps", [5, 6])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])) + "_" + c[1])
def test_plane_schedule_vs_oracle_and_pencils(case, nsteps, monkeypatch):
    n, precision, nr = case
    p = _problem(n, precision, nr)
    psi_cl = inputs.lognormal_field(n, p.box, kcut=min(n) // 4, seed=4)
    dt = 2e-4
    print(f"plane schedule {n} {precision} nsteps={nsteps}", flush=True)
    psi0, psi, cl, m = _run(p, psi_cl, 31, nsteps, dt, True, monkeypatch)
    _, psi_p, cl_p, m_p = _run(p, psi_cl, 31, nsteps, dt, False, monkeypatch)
    prob = oracle_problem(p)
    ref = tw.evolve(prob, psi0.astype(np.complex128), nsteps, dt)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    ref_cl = tw.evolve(prob, cl0, nsteps, dt)
    tol = TOL[precision]
    for r in range(nr):
        assert rel(psi[r], ref[r]) < tol, r
        assert rel(psi[r], psi_p[r]) < tol, r
    assert rel(cl, ref_cl) < tol and rel(cl, cl_p) < tol
    mo = tw.moments(prob, ref, p.n_tot, ref_cl)
    for k in ("mean_psi", "mean_rho", "var_rho", "norm", "energy"):
        assert rel(m[k].cpu().numpy(), mo[k]) < tol, k
    assert abs(m["Q_raw"] - mo["Q_raw"]) < tol * abs(mo["Q_raw"])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plane_schedule_adaptive_steps(precision, monkeypatch):
    """Device-chosen step sizes on the plane schedule (the kick pass of either
    kind records max|V|) against the oracle's adaptive evolution."""
    monkeypatch.setenv("TW_SLAB", "1")
    n = (32, 32, 16)
    p = Problem(n=n, box=(1.0, 1.0, 0.5), hbar_m=0.05, G=1.0, m_tot=400.0, n_tot=1e6, n_real=3,
                precision=precision)
    psi_cl = inputs.lognormal_field(n, p.box, kcut=6, seed=2)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 8)
    psi0 = psi.cpu().numpy().astype(np.complex128)
    clt = cl.to(p.cdtype).clone()
    nsteps = 7
    dts = plan.step_adaptive(psi, nsteps, 2e-2, 0.5, clt).cpu().numpy()
    torch.cuda.synchronize()
    prob = oracle_problem(p)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    ref, ref_dts = tw.evolve_adaptive(prob, np.concatenate([psi0, cl0[None]]), nsteps, 2e-2, 0.5)
    tol = TOL[precision]
    assert np.max(np.abs(dts / ref_dts - 1)) < tol
    assert len(set(ref_dts.tolist())) > 2       # the potential bound varies the step
    assert rel(psi.cpu().numpy(), ref[:3]) < tol
    assert rel(clt.cpu().numpy(), ref[3]) < tol
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_plane_schedule_tracers(precision, monkeypatch):
    """Test particles pushed in each field's potential, written back by either
    kind of kick pass, against the oracle's step_tracers."""
    monkeypatch.setenv("TW_SLAB", "1")
    n = (32, 32, 16)
    box = (1.0, 1.0, 0.5)
    p = Problem(n=n, box=box, hbar_m=0.5, G=1.0, m_tot=30.0, n_tot=1e5, n_real=3, precision=precision)
    psi_cl = inputs.lognormal_field(n, box, kcut=8, seed=6)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 5)
    clt = cl.to(p.cdtype).clone()
    rng = np.random.default_rng(1)
    tr0 = np.zeros((4, 5, 6))
    tr0[:, :, :3] = rng.uniform(0, 1, (4, 5, 3)) * np.array(box)
    tr0[:, :, 3:] = rng.normal(0, 0.5, (4, 5, 3))
    tr = torch.from_numpy(tr0.copy()).cuda()
    psi0 = psi.cpu().numpy().astype(np.complex128)
    plan.step_tracers(psi, 5, 2e-3, tr, psi_classical=clt)
    torch.cuda.synchronize()
    prob = oracle_problem(p)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    ref_psi, ref_tr = tw.evolve_tracers(prob, np.concatenate([psi0, cl0[None]]), tr0, 5, 2e-3)
    tol = TOL[precision]
    got = tr.cpu().numpy()
    assert rel(psi.cpu().numpy(), ref_psi[:3]) < tol
    assert np.abs(ref_tr[:, :, 3:] - tr0[:, :, 3:]).max() > 1e-3
    assert rel(got, ref_tr) < tol
    assert rel(got[:, :, 3:] - tr0[:, :, 3:], ref_tr[:, :, 3:] - tr0[:, :, 3:]) < tol
    plan.close()
