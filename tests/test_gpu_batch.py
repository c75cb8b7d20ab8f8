"""Batched uneven ensembles: grouped launches replayed from one HIP graph.

Bars: every class of a batch equals the same class advanced alone by tw_step
with the same strided-pass organisation (bit for bit: the same kernels run in
the same order), and matches the CPU oracle (1e-4 FP32, 1e-10 FP64)."""
import numpy as np
import pytest
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Batch, Plan, Problem, inputs
from tests.gpu_util import TOL, oracle_problem, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _classes(precision, sizes, n_real):
    return [Problem(n=n, hbar_m=1.0, G=1.0, m_tot=20.0, n_tot=1e3 * int(np.prod(n)), n_real=r,
                    precision=precision) for n, r in zip(sizes, n_real)]


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("variant", ["0", "1"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_equals_single_plans_and_oracle(precision, variant, mode, monkeypatch):
    monkeypatch.setenv("TW_COLS_VARIANT", variant)
    monkeypatch.setenv("TW_BATCH_MODE", mode)
    # grouped launches (mode 0) run the pencil schedule; single plans compared
    # bit for bit with them must too (mode 1 runs each class's own plan)
    monkeypatch.setenv("TW_SLAB", "0" if mode == "0" else "1")
    sizes = [(16, 16, 16), (24, 24, 24), (32, 16, 32)]
    probs = _classes(precision, sizes, [3, 4, 2])
    batch = Batch(probs)
    seed, nsteps, dt = 9, 6, 2e-4
    cls, psis, clt = [], [], []
    for p, plan in zip(probs, batch.plans):
        c = torch.from_numpy(inputs.soliton_3d(p.n, p.box, core=0.15)).cuda()
        cls.append(c)
        psis.append(plan.sample(c, seed))
        clt.append(c.to(p.cdtype).clone())
    ref = [x.clone() for x in psis]
    ref_cl = [x.clone() for x in clt]
    batch.step(psis, nsteps, dt, clt)
    batch.step(psis, nsteps, dt, clt)          # second call replays the captured graph
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        single = Plan(p)
        single.step(ref[i], nsteps, dt, ref_cl[i])
        single.step(ref[i], nsteps, dt, ref_cl[i])
        torch.cuda.synchronize()
        assert torch.equal(psis[i], ref[i]), f"class {i} differs from the single-plan run"
        assert torch.equal(clt[i], ref_cl[i])
        prob = oracle_problem(p)
        x0 = batch.plans[i].sample(cls[i], seed).cpu().numpy().astype(np.complex128)
        o = tw.evolve(prob, x0, 2 * nsteps, dt)
        assert rel(psis[i].cpu().numpy(), o) < TOL[precision]
    batch.close()


def test_batch_autotune_and_moments(tmp_path, monkeypatch):
    monkeypatch.setenv("TW_TUNE_CACHE", str(tmp_path / "tune.json"))
    monkeypatch.delenv("TW_COLS_VARIANT", raising=False)
    monkeypatch.delenv("TW_BATCH_MODE", raising=False)
    probs = _classes("fp32", [(32, 32, 32), (48, 48, 48)], [5, 3])
    batch = Batch(probs)
    v, m = batch.autotune()
    assert v in (0, 1) and m in (0, 1)
    text = (tmp_path / "tune.json").read_text()
    assert "batch" in text and "|mode" in text
    psis = []
    for p, plan in zip(probs, batch.plans):
        c = torch.from_numpy(inputs.soliton_3d(p.n, p.box)).cuda()
        psis.append(plan.sample(c, 1))
    batch.step(psis, 4, 1e-4)
    for p, plan, x in zip(probs, batch.plans, psis):
        m = plan.moments(x, energy=True)
        ref = tw.moments(oracle_problem(p), x.cpu().numpy().astype(np.complex128), p.n_tot)
        assert rel(m["mean_rho"].cpu().numpy(), ref["mean_rho"]) < 1e-12
        assert rel(m["energy"].cpu().numpy(), ref["energy"]) < 1e-4
    batch.close()


def test_batch_rejects_mixed_or_unsupported():
    from paper_2310_07119_amd.twa import TwError
    with pytest.raises(TwError):
        Batch([Problem(n=(32, 32), n_real=2), Problem(n=(32, 32, 32), n_real=2)])
    with pytest.raises(TwError):
        Batch([Problem(n=(256, 256), n_real=2)])
    with pytest.raises(TwError):
        Batch([Problem(n=(32, 32), n_real=2, precision="fp32"), Problem(n=(32, 32), n_real=2)])


_C4_ORACLE = {}


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("variant", ["0", "1"])
def test_batch_workload_classes(variant, mode, monkeypatch):
    """The batched workload's own size classes (64^3, 96^3, 128^3; FP32 split,
    stable soliton core of radius 0.1 L, 10^3 particles per cell) with a few
    realizations each: every class equals its single plan bit for bit and the
    oracle within 1e-4; the grouped kernels for lengths 64, 96 and 128 run
    here in both strided organisations."""
    monkeypatch.setenv("TW_COLS_VARIANT", variant)
    monkeypatch.setenv("TW_BATCH_MODE", mode)
    monkeypatch.setenv("TW_SLAB", "0" if mode == "0" else "1")
    w = inputs.WORKLOADS["3d_batched_soliton"]
    sizes, n_real = w["classes"], [3, 2, 2]
    probs = [Problem(n=n, box=w["box"], hbar_m=w["hbar_m"], G=w["G"], m_tot=w["m_tot"],
                     n_tot=w["occupation"] * int(np.prod(n)), n_real=r, precision="fp32")
             for n, r in zip(sizes, n_real)]
    print(f"batch workload classes variant={variant} mode={mode}", flush=True)
    batch = Batch(probs)
    seed, nsteps, dt = 13, 4, w["dt"]
    cls, psis, clt = [], [], []
    for p, plan in zip(probs, batch.plans):
        c = torch.from_numpy(inputs.soliton_3d(p.n, p.box, core=0.1)).cuda()
        cls.append(c)
        psis.append(plan.sample(c, seed))
        clt.append(c.to(p.cdtype).clone())
    x0 = [x.cpu().numpy() for x in psis]
    ref = [x.clone() for x in psis]
    ref_cl = [x.clone() for x in clt]
    batch.step(psis, nsteps, dt, clt)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        single = Plan(p)
        single.step(ref[i], nsteps, dt, ref_cl[i])
        torch.cuda.synchronize()
        assert torch.equal(psis[i], ref[i]), f"class {p.n} differs from the single-plan run"
        assert torch.equal(clt[i], ref_cl[i])
        single.close()
        key = tuple(p.n)
        if key not in _C4_ORACLE:
            prob = oracle_problem(p)
            o = tw.evolve(prob, x0[i].astype(np.complex128), nsteps, dt)
            ocl = tw.evolve(prob, cls[i].cpu().numpy().astype(np.complex64).astype(np.complex128), nsteps, dt)
            _C4_ORACLE[key] = (o, ocl)
        o, ocl = _C4_ORACLE[key]
        assert rel(psis[i].cpu().numpy(), o) < TOL["fp32"], p.n
        assert rel(clt[i].cpu().numpy(), ocl) < TOL["fp32"], p.n
    batch.close()
