"""Breaktime analysis (host logic): the paper's printed worked examples,
closed forms of the growth fits, and the shell spectrum's bookkeeping."""
import json
import math
import os

import numpy as np
import pytest

from paper_2310_07119_amd import breaktime as bt
from paper_2310_07119_amd.inputs import G_KPC_MYR_MSUN

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "breaktime_examples.json")))


def test_q_relation_worked_example():
    """Sec. 'Estimating the breaktime': Q_s ~ 1e-8 t^2 sampled with n_s = 1e8
    predicts Q_p ~ 1e-98 t^2 for n_p = 1e98 and a breaktime of 1e49 Myr."""
    g = GOLDEN["q_relation_example"]
    t = np.linspace(0.0, 500.0, 51)
    q_s = g["q_sim_coefficient_per_myr2"] * t ** 2
    q_p = bt.q_physical(q_s, g["n_sim"], g["n_phys"])
    a_p = bt.fit_quadratic(t, q_p)
    assert a_p == pytest.approx(g["q_phys_coefficient_per_myr2"], rel=1e-12)
    assert bt.breaktime_quadratic(a_p) == pytest.approx(g["t_break_myr"], rel=1e-12)


def test_collapse_estimate_and_dynamical_time():
    """Eq. (TbreakEstimate): ln(1e100)/7 collapse times of about 2 Gyr is about
    65 Gyr; the 3D collapse time 1/sqrt(G M/L^3) for 1e10 Msun in 60 kpc is about 2 Gyr."""
    g = GOLDEN["collapse_estimate"]
    t_br = bt.breaktime_collapse_estimate(g["n_tot"], g["t_c_myr"], g["rate"])
    assert t_br == pytest.approx(g["t_break_myr_approx"], rel=0.02)
    c = GOLDEN["collapse_time"]
    t_c = bt.dynamical_time((c["box_kpc"],) * 3, G_KPC_MYR_MSUN, c["m_tot_msun"])
    assert 0.75 * c["t_c_myr_approx"] < t_c < 1.25 * c["t_c_myr_approx"]


def test_exponential_fit_closed_form():
    """Q = A e^(lambda t) exactly: the fit returns ln A and lambda, and the
    breaktime solves A_p e^(lambda t) = 1; points with Q <= 0 are ignored."""
    t = np.linspace(0.0, 10.0, 41)
    log_a, lam = math.log(3e-9), 1.7
    q = np.exp(log_a + lam * t)
    q[:3] = [-1e-12, 0.0, -5e-13]          # early noise of the symmetric estimator
    la, l = bt.fit_exponential(t, q)
    assert la == pytest.approx(log_a, rel=1e-12) and l == pytest.approx(lam, rel=1e-12)
    n_s, n_p = 1e6, 1e20
    la_p, l_p = bt.fit_exponential(t, bt.q_physical(q, n_s, n_p))
    t_br = bt.breaktime_exponential(la_p, l_p)
    assert math.exp(la_p + l_p * t_br) == pytest.approx(1.0, rel=1e-10)
    assert t_br == pytest.approx((math.log(n_p / n_s) - log_a) / lam, rel=1e-12)


def test_quadratic_fit_least_squares():
    """The quadratic fit is the least-squares slope against t^2 (normal equation)."""
    rng = np.random.default_rng(3)
    t = np.linspace(0.1, 4.0, 30)
    q = 2.5e-3 * t ** 2 * (1.0 + 0.05 * rng.standard_normal(t.size))
    a = bt.fit_quadratic(t, q)
    grid = a + np.linspace(-1e-5, 1e-5, 21)
    res = [np.sum((q - x * t ** 2) ** 2) for x in grid]
    assert int(np.argmin(res)) == 10


def test_fit_errors():
    with pytest.raises(ValueError):
        bt.fit_exponential([0.0, 1.0], [1.0, -1.0])
    with pytest.raises(ValueError):
        bt.breaktime_exponential(-3.0, 0.0)
    with pytest.raises(ValueError):
        bt.breaktime_quadratic(0.0)
    with pytest.raises(ValueError):
        bt.q_physical([1.0], 0.0, 1.0)


def test_shell_spectrum_bookkeeping():
    """On a 2D 8x6 grid with a non-square box: every mode lands in exactly one
    shell, a constant occupation averages to itself, and an occupation equal to
    the shell index averages to that index."""
    nx, ny, box = 8, 6, (2.0, 1.5)
    occ = np.ones((ny, nx))
    k, mean, cnt = bt.shell_spectrum(occ, box)
    assert cnt.sum() == nx * ny and np.allclose(mean, 1.0)
    kx = 2 * np.pi * np.fft.fftfreq(nx, d=1.0 / nx) / box[0]
    ky = 2 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny) / box[1]
    dk = min(2 * np.pi / box[0], 2 * np.pi / box[1])
    shell = np.rint(np.sqrt(kx[None, :] ** 2 + ky[:, None] ** 2) / dk)
    k2, mean2, _ = bt.shell_spectrum(shell, box)
    assert np.allclose(mean2, k2 / dk)
    assert k[0] == 0.0 and mean2[0] == 0.0


class _StubPlan:
    """Host stand-in for a plan: Q_raw grows by a known amount per step."""

    def __init__(self, q0):
        self.q = q0
        self.steps = []

    def moments(self, psi, psi_cl, energy=False, per_cell=False, modes=False):
        return {"Q_raw": self.q, "Q_sym": self.q - 0.5, "dev_rho_L1": 0.0, "dev_psi_L2": 0.0}

    def step(self, psi, k, dt, psi_cl):
        self.steps.append(k)
        self.q += 0.25 * k


def test_record_subtracts_the_sampled_initial_q():
    """Sec. 'Estimating the breaktime': the sampled Q(0) is not zero and is
    subtracted; outputs every `every` steps, the last one at nsteps."""
    plan = _StubPlan(q0=3.0)
    rec = bt.record(plan, None, None, nsteps=7, dt=0.1, every=3)
    assert plan.steps == [3, 3, 1]
    assert np.allclose(rec["t"], [0.0, 0.3, 0.6, 0.7])
    assert np.array_equal(rec["Q_raw"], [3.0, 3.75, 4.5, 4.75])
    assert np.array_equal(rec["Q_minus_Q0"], [0.0, 0.75, 1.5, 1.75])
