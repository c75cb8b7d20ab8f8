"""Error paths of the C ABI on a live plan: every rejected call returns its
status before any kernel is launched, leaves a message, and leaves the plan
and the fields untouched (the next valid calls give the same results as a
fresh plan)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2310_07119_amd import Plan, Problem, inputs, twa

pytestmark = pytest.mark.gpu

EINVAL, ELAYOUT = -1, -3


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _problem():
    w = inputs.WORKLOADS["2d_n512_pair"]
    return Problem(n=(64, 32), box=(1.0, 0.5), hbar_m=w["hbar_m"], G=w["G"], m_tot=w["m_tot"], n_tot=1e5, n_real=4,
                   precision="fp64")


def _field(p):
    x = np.arange(64)[None, :]
    y = np.arange(32)[:, None]
    rho = 1.0 + 0.3 * np.cos(2 * np.pi * x / 64) + 0.2 * np.sin(2 * np.pi * y / 32)
    psi = np.sqrt(rho).astype(np.complex128)
    return psi / np.sqrt(np.sum(rho) * (1.0 / 64) * (0.5 / 32))


def test_rejected_calls_leave_plan_usable():
    p = _problem()
    lib = twa.load_library()
    cl = torch.from_numpy(_field(p)).cuda()
    plan = Plan(p)
    psi = plan.sample(cl, 3)
    before = psi.clone()
    h = plan.handle
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    vp = ctypes.c_void_p
    a, c = psi.data_ptr(), cl.data_ptr()
    tr = torch.zeros(5 * 4 * 4 + 1, dtype=torch.float64, device="cuda")
    out = torch.zeros(4 * 4 + 1, dtype=torch.float64, device="cuda")
    dts = torch.zeros(3, dtype=torch.float64, device="cuda")
    cases = [
        ("step misaligned", lambda: lib.tw_step(h, vp(a + 8), None, 1, 1e-4, s), ELAYOUT),
        ("step classical misaligned", lambda: lib.tw_step(h, vp(a), vp(c + 4), 1, 1e-4, s), ELAYOUT),
        ("step NULL psi", lambda: lib.tw_step(h, None, None, 1, 1e-4, s), EINVAL),
        ("step nsteps < 0", lambda: lib.tw_step(h, vp(a), None, -1, 1e-4, s), EINVAL),
        ("step dt NaN", lambda: lib.tw_step(h, vp(a), None, 1, float("nan"), s), EINVAL),
        ("sample psi_cl misaligned", lambda: lib.tw_sample(h, vp(c + 8), 0, 0, vp(a), s), ELAYOUT),
        ("sample offset < 0", lambda: lib.tw_sample(h, vp(c), 0, -1, vp(a), s), EINVAL),
        ("moments NULL out", lambda: lib.tw_moments(h, vp(a), None, None, s), EINVAL),
        ("adaptive dt_max 0", lambda: lib.tw_step_adaptive(h, vp(a), None, 1, 0.0, 0.5, None, s), EINVAL),
        ("adaptive courant > 1", lambda: lib.tw_step_adaptive(h, vp(a), None, 1, 1e-3, 1.5, None, s), EINVAL),
        ("adaptive dt_out misaligned",
         lambda: lib.tw_step_adaptive(h, vp(a), None, 1, 1e-3, 0.5, vp(dts.data_ptr() + 4), s), ELAYOUT),
        ("tracers misaligned", lambda: lib.tw_step_tracers(h, vp(a), None, 1, 1e-4, vp(tr.data_ptr() + 4), 4, s),
         ELAYOUT),
        ("tracers none", lambda: lib.tw_step_tracers(h, vp(a), None, 1, 1e-4, vp(tr.data_ptr()), 0, s), EINVAL),
        ("spread misaligned", lambda: lib.tw_tracer_spread(h, vp(tr.data_ptr()), 4, vp(out.data_ptr() + 4), s),
         ELAYOUT),
        ("spread NULL", lambda: lib.tw_tracer_spread(h, None, 4, vp(out.data_ptr()), s), EINVAL),
    ]
    for name, call, want in cases:
        print(name, flush=True)
        assert call() == want, name
        assert lib.tw_last_error().decode(), name
    torch.cuda.synchronize()
    assert torch.equal(psi, before)
    # the plan still works, and gives what a fresh plan gives
    clt = cl.clone()
    plan.step(psi, 3, 1e-4, clt)
    m = plan.moments(psi, clt)
    plan2 = Plan(p)
    psi2 = plan2.sample(cl, 3)
    clt2 = cl.clone()
    plan2.step(psi2, 3, 1e-4, clt2)
    m2 = plan2.moments(psi2, clt2)
    assert torch.equal(psi, psi2) and torch.equal(clt, clt2)
    assert m["Q_raw"] == m2["Q_raw"]
    plan.close()
    plan2.close()
