"""tw_moments_static (the allocation-free moment reductions, partial sums in
the library's fixed device array) against tw_moments of a plan on the same
ensembles: two calls in a row, the second on a smaller input, both equal bit
for bit (same kernels, same fixed summation order); sizes beyond the fixed
array are refused before any launch."""
import numpy as np
import pytest
import torch

from paper_2310_07119_amd import Plan, Problem, inputs
from paper_2310_07119_amd.twa import TwError, moments_static

pytestmark = pytest.mark.gpu

KEYS = ("mean_psi", "mean_abs2", "mean_rho", "var_rho", "norm")


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _ensemble(p, seed):
    plan = Plan(p)
    cl = torch.from_numpy(inputs.lognormal_field(p.n, p.box, kcut=min(p.n) // 4, seed=seed)).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    plan.step(psi, 3, 2e-4, clt)
    return plan, psi, clt


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_moments_equal_plan_moments_twice(precision):
    # the first call fills more of the fixed array than the second reads
    cases = [Problem(n=(256, 96), box=(1.0, 0.375), m_tot=20.0, n_tot=1e5, n_real=37, precision=precision),
             Problem(n=(16, 24, 16), box=(1.0, 1.5, 1.0), m_tot=5.0, n_tot=1e4, n_real=3, precision=precision)]
    for i, p in enumerate(cases):
        print(f"moments_static {precision} call {i}: n={p.n} n_real={p.n_real}", flush=True)
        plan, psi, clt = _ensemble(p, 11 + i)
        ref = plan.moments(psi, clt, energy=False)
        got = moments_static(p, psi, clt)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(got[k], ref[k]), k
        scal = got["scalars"].cpu().numpy()
        for j, name in enumerate(("Q_raw", "Q_sym", "dev_rho_L1", "dev_psi_L2", "energy_mean", "norm_mean",
                                  "nonfinite", "energy_classical")):
            assert scal[j] == ref[name], name
        # without the classical field the deviations are 0, as in tw_moments
        got2 = moments_static(p, psi)
        ref2 = plan.moments(psi, energy=False)
        assert got2["scalars"][2].item() == 0.0 == ref2["dev_rho_L1"]
        assert torch.equal(got2["var_rho"], ref2["var_rho"])
        plan.close()


def test_static_moments_refuses_oversize_and_plan_outputs():
    # 512^3 with 32 realizations needs 32 * 2^21 partial sums > 2^22
    big = Problem(n=(512, 512, 512), n_real=32, precision="fp32")
    psi = torch.empty(8, dtype=torch.complex64, device="cuda")
    with pytest.raises(TwError, match="fixed scratch"):
        moments_static(big, psi, out={"norm": None})
    # the largest workloads of this library fit
    for p in (Problem(n=(512, 512), n_real=256), Problem(n=(128, 128, 128), n_real=64, precision="fp32")):
        nw = -(-p.ncell // 64)
        assert p.n_real * nw + 3 * nw + p.n_real + 3 <= 1 << 22
