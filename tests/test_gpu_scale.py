"""The paper's momentum-space Gaussian test problem at 512^3 (FP32 split, the
largest grid the passes support), and the same family regenerated at 32^3 for
a complete comparison with the oracle. At full size the oracle recomputes
sampled cells one by one; the evolution is checked through properties that
hold at any size (norm of every realization, step sizes within the rule)."""
import numpy as np
import pytest
import torch

from oracle import philox
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


def test_kgauss_512cube_fp32():
    p, w = _problem("3d_n512_kgauss", "fp32", n_real=8)
    print("512^3 momentum-space Gaussian, 8 realizations, fp32", flush=True)
    psi_cl = inputs.initial_field("3d_n512_kgauss")
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    seed = 31
    psi = plan.sample(cl, seed)
    torch.cuda.synchronize()
    # sampled cells recomputed by the oracle's generator, one by one
    rng = np.random.default_rng(0)
    g = rng.integers(0, p.ncell, 64).astype(np.uint64)
    r = rng.integers(0, p.n_real, 64).astype(np.uint64)
    words = philox.philox4x64([g, r, np.zeros_like(g), np.zeros_like(g)], (seed, tw.SAMPLE_KEY_TAG))
    z1, z2 = philox.box_muller(words[0], words[1])
    grid = tw.Grid(p.n, p.box)
    sc = tw.noise_scale(grid, p.n_tot)
    flat_cl = psi_cl.reshape(-1)
    expect = (flat_cl.real[g.astype(np.int64)] + z1 * sc) + 1j * (flat_cl.imag[g.astype(np.int64)] + z2 * sc)
    got = psi.reshape(p.n_real, -1)[torch.from_numpy(r.astype(np.int64)).cuda(),
                                     torch.from_numpy(g.astype(np.int64)).cuda()].cpu().numpy()
    assert np.array_equal(got, expect.astype(np.complex64))
    n0 = plan.moments(psi, energy=False, per_cell=False)["norm"].cpu().numpy()
    clt = cl.to(torch.complex64).clone()
    dts = plan.step_adaptive(psi, 3, w["dt"], courant=0.5, psi_classical=clt).cpu().numpy()
    n1 = plan.moments(psi, energy=False, per_cell=False)["norm"].cpu().numpy()
    assert np.all(np.abs(n1 / n0 - 1.0) < 1e-5)
    kin = tw.kinetic_dt_bound(tw.Problem(grid, p.hbar_m, p.G, p.m_tot))
    assert np.all(dts > 0) and np.all(dts <= w["dt"]) and np.all(dts <= 0.5 * kin * (1 + 1e-12))
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()


def test_kgauss_32cube_subset_vs_oracle():
    """The same problem family regenerated at 32^3, FP32 split with adaptive
    steps, against the oracle's adaptive evolution (every realization)."""
    p, w = _problem("3d_n512_kgauss", "fp32", n=(32, 32, 32), n_real=6, n_tot=1e3 * 32 ** 3)
    psi_cl = inputs.initial_field("3d_n512_kgauss", n=(32, 32, 32))
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 3)
    clt = cl.to(torch.complex64).clone()
    psi0 = psi.cpu().numpy().astype(np.complex128)
    nsteps = 12
    dts = plan.step_adaptive(psi, nsteps, w["dt"], courant=0.5, psi_classical=clt).cpu().numpy()
    prob = oracle_problem(p)
    cl0 = psi_cl.astype(np.complex64).astype(np.complex128)
    ref, rdts = tw.evolve_adaptive(prob, np.concatenate([psi0, cl0[None]]), nsteps, w["dt"], 0.5)
    assert rel(dts, rdts) < 1e-6
    assert rel(psi.cpu().numpy(), ref[:p.n_real]) < TOL["fp32"]
    assert rel(clt.cpu().numpy(), ref[p.n_real]) < TOL["fp32"]
    plan.close()


def test_largest_ensemble_per_sample_call():
    """65535 realizations (the most one tw_sample call draws) of a 16 x 16 field
    with the classical field: the last realization's draw bit for bit and its
    evolution against the oracle, the moments against the oracle's moments of
    the GPU state; one realization more is refused before any launch."""
    n, nreal, seed, nsteps, dt = (16, 16), 65535, 4, 3, 2e-4
    p = Problem(n=n, hbar_m=1.0, G=1.0, m_tot=10.0, n_tot=1e4, n_real=nreal, precision="fp64")
    psi_cl = inputs.lognormal_field(n, p.box, kcut=4, seed=3)
    print(f"largest ensemble: {nreal} realizations of {n}", flush=True)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, seed)
    last0 = psi[nreal - 1].cpu().numpy()
    clt = cl.clone()
    plan.step(psi, nsteps, dt, clt)
    m = plan.moments(psi, clt)
    host = psi.cpu().numpy()
    prob = oracle_problem(p)
    x0 = tw.sample(prob.grid, psi_cl, 1, p.n_tot, seed, real_offset=nreal - 1)
    assert np.array_equal(last0, x0[0])
    assert rel(host[nreal - 1], tw.evolve(prob, x0, nsteps, dt)[0]) < TOL["fp64"]
    om = tw.moments(prob, host, p.n_tot, clt.cpu().numpy())
    for k in ("mean_psi", "mean_rho", "var_rho", "norm"):
        assert rel(m[k].cpu().numpy(), om[k]) < 1e-12, k
    for k in ("Q_raw", "dev_rho_L1", "dev_psi_L2"):
        assert abs(m[k] - om[k]) < 1e-11 * abs(om[k]), k
    plan.close()
    del psi, host
    torch.cuda.empty_cache()
    from paper_2310_07119_amd.twa import TwError
    p2 = Problem(n=n, hbar_m=1.0, G=1.0, m_tot=10.0, n_tot=1e4, n_real=nreal + 1, precision="fp64")
    plan2 = Plan(p2)
    with pytest.raises(TwError):
        plan2.sample(cl, seed)
    plan2.close()


def test_kgauss_512sq_full_grid_vs_oracle():
    """The paper's 2D momentum-space Gaussian (Sec. "Momentum space gaussian",
    Eq. (kspaceGauss)) on its full 512^2 grid in physical units (L = 60 kpc,
    M_tot = 6e9 M_sun, hbar/m = 0.02 kpc^2/Myr), FP64, 8 realizations + the
    classical field, 10 device-chosen steps against the oracle's adaptive
    evolution of the same draws: step sizes, fields and moments at 1e-10."""
    p, w = _problem("2d_n512_kgauss", "fp64", n_real=8)
    psi_cl = inputs.initial_field("2d_n512_kgauss")
    print("512^2 momentum-space Gaussian, 8 realizations, fp64, 10 adaptive steps", flush=True)
    plan = Plan(p)
    cl = torch.from_numpy(psi_cl).cuda()
    psi = plan.sample(cl, 17)
    clt = cl.clone()
    psi0 = psi.cpu().numpy()
    nsteps = 10
    dts = plan.step_adaptive(psi, nsteps, w["dt"], courant=0.5, psi_classical=clt).cpu().numpy()
    m = plan.moments(psi, clt)
    torch.cuda.synchronize()
    prob = oracle_problem(p)
    ref, rdts = tw.evolve_adaptive(prob, np.concatenate([psi0, psi_cl[None]]), nsteps, w["dt"], 0.5)
    assert rel(dts, rdts) < 1e-12
    assert rel(psi.cpu().numpy(), ref[:-1]) < TOL["fp64"]
    assert rel(clt.cpu().numpy(), ref[-1]) < TOL["fp64"]
    mo = tw.moments(prob, ref[:-1], p.n_tot, ref[-1])
    for k in ("mean_psi", "mean_rho", "var_rho", "norm", "energy"):
        assert rel(m[k].cpu().numpy(), mo[k]) < TOL["fp64"], k
    assert abs(m["Q_raw"] - mo["Q_raw"]) < TOL["fp64"] * abs(mo["Q_raw"])
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()
