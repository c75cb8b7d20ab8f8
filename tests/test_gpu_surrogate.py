"""The learned surrogate: trained on ensembles the method generates (tw_sample /
tw_step / tw_moments) by the library's own FNO forward, backward and Adam
kernels, it must beat the classical field (the method without quantum
corrections: <rho> = rho_cl, Var rho = 0) on held-out coherent fields, judged
against a large reference ensemble, and answer faster than running an ensemble.
Surrogate accuracy itself has no analytic pin (parity unpinned): it is judged
statistically against the plain ensemble."""
import pytest
import torch

from paper_2310_07119_amd import surrogate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_surrogate_gains_over_classical_field():
    spec = surrogate.DatasetSpec(n=(64, 64), n_real=64, steps=100, dt=1e-4, n_tot=1e4, G=1.0, m_tot=20.0)
    res = surrogate.gain_study(spec, n_train=160, n_test=12, epochs=40, batch=8, ref_real=512,
                               net_kw=dict(width=16, modes_x=8, modes_y=8, layers=3, proj=32), seed=11,
                               log=lambda s: print(s, flush=True))
    print(res, flush=True)
    assert res["loss_last"] < 0.5 * res["loss_first"]
    s, c = res["surrogate"], res["classical"]
    assert s["var_err"] < 0.5 * c["var_err"]
    assert s["rho_err"] < c["rho_err"]
    assert res["inference_seconds_per_field"] < res["twa_64_seconds_per_field"]
