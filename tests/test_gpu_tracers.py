"""Test particles advanced with the fields (tw_step_tracers) against the
oracle's step_tracers: every field's particles in that field's own potential."""
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


def _tracers(nfield, ntr, box, seed):
    rng = np.random.default_rng(seed)
    D = len(box)
    t = np.zeros((nfield, ntr, 2 * D))
    t[:, :, :D] = rng.uniform(0, 1, (nfield, ntr, D)) * np.array(box)
    t[:, :, D:] = rng.normal(0, 0.5, (nfield, ntr, D))
    return t


CASES = [
    # (n, box, n_real, nsteps, ntracer)
    ((64, 32), (1.0, 0.5), 5, 7, 4),
    ((128, 128), (1.0, 1.0), 17, 5, 3),
    ((32, 16, 16), (1.0, 0.5, 0.5), 3, 4, 5),
]


@pytest.mark.parametrize("transpose", ["0", "1"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[0])))
def test_tracers_vs_oracle(case, precision, transpose, monkeypatch):
    n, box, nr, nsteps, ntr = case
    if len(n) == 3 and transpose == "1":
        pytest.skip("the alternating schedule is the 2D one")
    monkeypatch.setenv("TW_TRANSPOSE", transpose)
    p = Problem(n=n, box=box, hbar_m=0.5, G=1.0, m_tot=30.0, n_tot=1e5, n_real=nr, precision=precision)
    psi_cl = inputs.lognormal_field(n, box, kcut=min(n) // 4, seed=6)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 5)
    clt = cl.to(p.cdtype).clone()
    tr0 = _tracers(nr + 1, ntr, box, 1)
    tr = torch.from_numpy(tr0.copy()).cuda()
    psi0 = psi.cpu().numpy().astype(np.complex128)
    dt = 2e-3
    print(f"tracers {n} {precision} transpose={transpose}", flush=True)
    plan.step_tracers(psi, nsteps, dt, tr, psi_classical=clt)
    torch.cuda.synchronize()
    prob = oracle_problem(p)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    ref_psi, ref_tr = tw.evolve_tracers(prob, np.concatenate([psi0, cl0[None]]), tr0, nsteps, dt)
    tol = TOL[precision]
    got = tr.cpu().numpy()
    assert rel(psi.cpu().numpy(), ref_psi[:nr]) < tol
    D = len(n)
    moved = np.abs(ref_tr[:, :, D:] - tr0[:, :, D:]).max()
    assert moved > 1e-3, "gravity should change the velocities"
    assert rel(got[:, :, :D], ref_tr[:, :, :D]) < tol
    assert rel(got[:, :, D:], ref_tr[:, :, D:]) < tol
    # the velocity change alone (what gravity did) at the same bar
    assert rel(got[:, :, D:] - tr0[:, :, D:], ref_tr[:, :, D:] - tr0[:, :, D:]) < tol
    spread = plan.tracer_spread(tr).cpu().numpy()
    assert rel(spread, tw.tracer_spread(got, nr)) < 1e-12
    plan.close()


def test_tracers_without_gravity_move_straight():
    p = Problem(n=(32, 32), G=0.0, n_tot=1e4, n_real=2)
    plan = Plan(p)
    cl = torch.from_numpy(inputs.lognormal_field(p.n, p.box, seed=1)).cuda()
    psi = plan.sample(cl, 1)
    tr0 = _tracers(2, 6, p.box, 3)
    tr = torch.from_numpy(tr0.copy()).cuda()
    plan.step_tracers(psi, 10, 1e-2, tr)
    got = tr.cpu().numpy()
    assert np.allclose(got[:, :, :2], tr0[:, :, :2] + 0.1 * tr0[:, :, 2:], rtol=0, atol=1e-14)
    assert np.array_equal(got[:, :, 2:], tr0[:, :, 2:])
