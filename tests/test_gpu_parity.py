"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs. Bars: sampled states bit-exact; FP64 results within
1e-10 and FP32-split results within 1e-4 normwise relative error."""
import numpy as np
import pytest
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Plan, Problem, inputs
from tests.gpu_util import TOL, gpu_run, oracle_problem, rel

pytestmark = pytest.mark.gpu

CASES = [
    # (n, n_real, nsteps, dt, hbar, G, m_tot, n_tot)
    ((256,), 64, 40, 1e-4, 1.0, 1.0, 1.0, 1e4),            # 1D workload shape, fewer steps
    ((16,), 3, 25, 1e-3, 0.3, 2.0, 5.0, 50.0),              # 1D tiny, odd ensemble
    ((96,), 5, 30, 1e-3, 0.5, 1.0, 3.0, 100.0),             # 1D, 3*2^k length (radix-4/2/6 stages)
    ((1024,), 4, 20, 1e-4, 1.0, 1.0, 1.0, 1e5),             # 1D, longest axis (sixteen points per thread)
    ((64, 32), 5, 12, 2e-4, 1.0, 1.0, 30.0, 1e5),           # 2D, several tiles, odd ensemble
    ((32, 128), 2, 10, 2e-4, 0.5, 3.0, 10.0, 1e5),          # 2D, long y axis
    ((16, 16, 32), 3, 6, 2e-4, 1.0, 1.0, 20.0, 1e6),        # 3D
    ((32, 16, 16), 4, 5, 1e-4, 1.0, 2.0, 10.0, 1e6),        # 3D, x longest
    ((48, 24), 1, 8, 2e-4, 0.7, 0.0, 1.0, 1e3),             # 2D, one realization, G = 0 (free field), 3*2^k axes
    ((16, 24, 16), 1, 4, 2e-4, 1.0, 1.5, 8.0, 1e4),         # 3D, one realization, mixed radix y
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"_r{c[1]}"


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("variant", ["0", "1"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_sample_step_moments_vs_oracle(case, precision, variant, monkeypatch):
    n, nr, nsteps, dt, hbar, G, m_tot, n_tot = case
    if len(n) == 1 and variant == "1":
        pytest.skip("1D has no strided passes")
    monkeypatch.setenv("TW_COLS_VARIANT", variant)
    p = Problem(n=n, hbar_m=hbar, G=G, m_tot=m_tot, n_tot=n_tot, n_real=nr, precision=precision)
    psi_cl = inputs.lognormal_field(n, p.box, kcut=min(n) // 4, seed=1)
    seed = 1234567
    print(f"case n={n} n_real={nr} {precision}", flush=True)
    g = gpu_run(p, psi_cl, seed, nsteps, dt, real_offset=7, modes=True, decoherence=True)
    prob = oracle_problem(p)
    psi0 = tw.sample(prob.grid, psi_cl, nr, n_tot, seed, real_offset=7)
    # sampled initial state: bit-exact (FP32 = the FP64 draw rounded to nearest)
    if precision == "fp64":
        assert np.array_equal(g["psi0"], psi0)
    else:
        assert np.array_equal(g["psi0"], psi0.astype(np.complex64))
        psi0 = g["psi0"].astype(np.complex128)      # oracle continues from the stored FP32 state
    psi = tw.evolve(prob, psi0, nsteps, dt)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    cl = tw.evolve(prob, cl0, nsteps, dt)
    tol = TOL[precision]
    assert rel(g["psi"], psi) < tol
    assert rel(g["cl"], cl) < tol
    ref = tw.moments(prob, psi, n_tot, cl, modes=True, decoherence_=True)
    # the reductions alone: the oracle's moments of the GPU's own final fields
    own = tw.moments(prob, g["psi"].astype(np.complex128), n_tot, g["cl"].astype(np.complex128), modes=True,
                     decoherence_=True)
    m = g["mom"]
    for k in ("mean_psi", "mean_abs2", "mean_rho", "var_rho", "mode_occ", "var_amp", "var_phase", "norm", "energy"):
        if nr == 1 and k in ("var_rho", "var_amp", "var_phase"):
            # one realization: spreads are zero up to rounding on both sides
            assert np.max(np.abs(m[k])) < 1e-12 and np.max(np.abs(ref[k])) < 1e-12, k
            continue
        assert rel(m[k], ref[k]) < tol, k
        assert rel(m[k], own[k]) < tol, k
    for k in ("Q_raw", "Q_sym", "dev_rho_L1", "dev_psi_L2", "Var_A", "Var_phi"):
        if nr == 1 and k in ("Q_raw", "Var_A", "Var_phi"):
            # one realization: these are differences of equal quantities, zero up to rounding
            assert abs(m[k]) < 1e-12 and abs(ref[k]) < 1e-12, k
            continue
        # Q_sym = Q_raw - N / (2 n_tot) nearly cancels (E Q_raw(0) = (1 - 1/N_s) N / (2 n_tot)), so its
        # error is Q_raw's and is bounded relative to Q_raw
        scale = abs(ref["Q_raw"]) if k == "Q_sym" else abs(ref[k])
        assert abs(m[k] - ref[k]) <= tol * scale, k
        assert abs(m[k] - own[k]) <= tol * scale, k
    assert abs(m["energy_mean"] - ref["energy"].mean()) < tol * abs(ref["energy"].mean())
    assert abs(m["energy_classical"] - tw.energy(prob, cl)) < tol * abs(tw.energy(prob, cl))
    assert m["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_steps_and_no_classical(precision):
    p = Problem(n=(32, 32), n_real=3, n_tot=1e3, precision=precision)
    psi_cl = inputs.lognormal_field(p.n, p.box, seed=2)
    g = gpu_run(p, psi_cl, 5, 0, 1e-3, with_classical=False)
    assert np.array_equal(g["psi"], g["psi0"])
    prob = oracle_problem(p)
    ref = tw.moments(prob, g["psi0"].astype(np.complex128), p.n_tot)
    assert abs(g["mom"]["Q_raw"] - ref["Q_raw"]) < 1e-10 * ref["Q_raw"]
    assert g["mom"]["dev_rho_L1"] == 0.0


def test_autotune_picks_a_variant_and_caches_it(tmp_path, monkeypatch):
    from paper_2310_07119_amd import Plan
    monkeypatch.setenv("TW_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.delenv("TW_COLS_VARIANT", raising=False)
    p = Problem(n=(64, 128), n_real=9, n_tot=1e4, precision="fp32")
    v = Plan(p).autotune()
    assert v in (0, 1)
    text = (tmp_path / "tune.json").read_text()
    import json
    entry = list(json.loads(text).values())[0]
    assert entry["cols_variant"] == v and len(entry["us"]) == 2
    # a second plan of the same shape reads the cache (same choice, no new entry)
    Plan(Problem(n=(64, 128), n_real=9, n_tot=1e4, precision="fp32")).autotune()
    assert len(json.loads((tmp_path / "tune.json").read_text())) == 1


def test_nonfinite_realization_is_counted():
    p = Problem(n=(32, 16), n_real=4, n_tot=1e3)
    from paper_2310_07119_amd import Plan
    plan = Plan(p)
    psi = torch.ones((4, 16, 32), dtype=torch.complex128, device="cuda")
    psi[2, 3, 4] = float("nan")
    m = plan.moments(psi, energy=False)
    assert m["nonfinite"] == 1


@pytest.mark.parametrize("transpose", ["0", "1"])
@pytest.mark.parametrize("nsteps", [5, 6])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_2d_schedules_vs_oracle(precision, nsteps, transpose, monkeypatch):
    """Both 2D step schedules (strided passes in place / alternating storage with
    transposed stores into a second buffer) on a grid with many workgroups per
    pass, odd and even step counts (the alternating schedule ends in the
    caller's buffer either way)."""
    monkeypatch.setenv("TW_TRANSPOSE", transpose)
    n, nr, n_tot = (256, 96), 41, 1e5
    p = Problem(n=n, box=(1.0, 0.375), hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=n_tot, n_real=nr, precision=precision)
    psi_cl = inputs.lognormal_field(n, p.box, kcut=16, seed=3)
    seed, dt = 4242, 2e-4
    print(f"2d schedule transpose={transpose} nsteps={nsteps} {precision}", flush=True)
    g = gpu_run(p, psi_cl, seed, nsteps, dt)
    prob = oracle_problem(p)
    psi0 = g["psi0"].astype(np.complex128)
    psi = tw.evolve(prob, psi0, nsteps, dt)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    cl = tw.evolve(prob, cl0, nsteps, dt)
    tol = TOL[precision]
    assert rel(g["psi"], psi) < tol
    assert rel(g["cl"], cl) < tol
    for r in (0, 17, 40):
        assert rel(g["psi"][r], psi[r]) < tol, r


@pytest.mark.parametrize("transpose", ["0", "1"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [(96, 48), (48, 192), (1024, 32), (24, 384)], ids=lambda n: "x".join(map(str, n)))
def test_2d_mixed_radix_and_long_axes(n, precision, transpose, monkeypatch):
    """Lengths 3 * 2^k and the longest supported axis (1024, sixteen points per
    thread) in both 2D schedules, on non-square grids (the alternating schedule
    swaps the roles of the axes every step)."""
    monkeypatch.setenv("TW_TRANSPOSE", transpose)
    box = (1.0, n[1] / n[0])
    p = Problem(n=n, box=box, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=1e5, n_real=5, precision=precision)
    psi_cl = inputs.lognormal_field(n, box, kcut=min(n) // 4, seed=8)
    nsteps, dt = 5, 1e-4
    print(f"2d mixed radix {n} {precision} transpose={transpose}", flush=True)
    g = gpu_run(p, psi_cl, 99, nsteps, dt)
    prob = oracle_problem(p)
    psi = tw.evolve(prob, g["psi0"].astype(np.complex128), nsteps, dt)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64).astype(np.complex128)
    tol = TOL[precision]
    assert rel(g["psi"], psi) < tol
    assert rel(g["cl"], tw.evolve(prob, cl0, nsteps, dt)) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_classical_limit_infinite_particle_number(precision):
    """n_tot = infinity (Sec. "Estimating the breaktime": the classical field is
    the limit of vanishing noise): every sampled realization is the coherent
    field bit for bit, and after the steps every realization still equals the
    classical field run alongside, so Q and Var rho vanish to rounding."""
    n = (64, 32)
    p = Problem(n=n, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=float("inf"), n_real=5, precision=precision)
    psi_cl = inputs.lognormal_field(n, p.box, kcut=8, seed=2)
    print(f"classical limit {precision}", flush=True)
    g = gpu_run(p, psi_cl, 9, 10, 2e-4)
    cl0 = psi_cl if precision == "fp64" else psi_cl.astype(np.complex64)
    assert all(np.array_equal(g["psi0"][r], cl0) for r in range(p.n_real))
    tol = 1e-12 if precision == "fp64" else 1e-5
    for r in range(p.n_real):
        assert rel(g["psi"][r], g["cl"]) < tol, r
    m = g["mom"]
    assert abs(m["Q_raw"]) < tol * np.mean(m["norm"])
    assert np.max(m["var_rho"]) < tol * np.max(m["mean_rho"]) ** 2
    assert m["nonfinite"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,slab", [((64, 32), "0"), ((16, 16, 32), "0"), ((16, 16, 32), "1")],
                         ids=["2d", "3d-pencils", "3d-planes"])
def test_pass_order_leaves_results_bit_identical(n, slab, precision, monkeypatch):
    """Consecutive passes walk the pairs in alternating directions, continuing
    from whatever the plan launched before. Every workgroup's arithmetic is
    independent of that order, so a plan that has already run an odd number
    of passes (one step of a scratch ensemble: five passes in the 2D and the
    3D plane schedules, nine in the 3D pencil schedule) must give
    bit-identical results to a fresh plan, whose passes all run the other way."""
    monkeypatch.setenv("TW_SLAB", slab)
    dev = torch.device("cuda:0")
    p = Problem(n=n, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=1e5, n_real=5, precision=precision)
    psi_cl = torch.from_numpy(inputs.lognormal_field(n, p.box, kcut=4, seed=3)).to(dev)
    print(f"pass order {n} slab={slab} {precision}", flush=True)
    fresh, used = Plan(p), Plan(p)
    scratch = used.sample(psi_cl, 5)
    used.step(scratch, 1, 2e-4)
    out = []
    for plan in (fresh, used):
        psi = plan.sample(psi_cl, 11)
        cl = psi_cl.to(p.cdtype).clone()
        plan.step(psi, 7, 2e-4, cl)
        torch.cuda.synchronize()
        out.append((psi.cpu(), cl.cpu()))
    fresh.close()
    used.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [(64, 32), (16, 16, 32)], ids=["2d", "3d"])
@pytest.mark.parametrize("env", [{"TW_CHUNK_PAIRS": "1"}, {"TW_STREAMS": "2"},
                                 {"TW_CHUNK_PAIRS": "2", "TW_STREAMS": "2"}],
                         ids=["chunks", "two_streams", "both"])
def test_pair_chunks_and_streams_leave_results_bit_identical(env, n, precision, monkeypatch):
    """Realizations are independent, so advancing the pairs in chunks through
    all steps (TW_CHUNK_PAIRS) or splitting them over two streams (TW_STREAMS)
    changes only the order of the work: the results must equal the default
    schedule's bit for bit."""
    dev = torch.device("cuda:0")
    p = Problem(n=n, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=1e5, n_real=5, precision=precision)
    psi_cl = torch.from_numpy(inputs.lognormal_field(n, p.box, kcut=4, seed=4)).to(dev)
    print(f"pair schedule {env} {n} {precision}", flush=True)
    out = []
    for use_env in (False, True):
        if use_env:
            for k, v in env.items():
                monkeypatch.setenv(k, v)
        plan = Plan(p)
        psi = plan.sample(psi_cl, 21)
        cl = psi_cl.to(p.cdtype).clone()
        plan.step(psi, 6, 2e-4, cl)
        torch.cuda.synchronize()
        out.append((psi.cpu(), cl.cpu()))
        plan.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
