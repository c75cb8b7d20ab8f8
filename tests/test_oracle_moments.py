"""Pins for the oracle's ensemble moments (Sec. "Evaluating operators", Eq. (Q)).

Closed forms at t=0 follow from the Gaussian vacuum noise of a coherent state:
with sigma^2 = E|d psi'|^2 = 1/(2 n_tot dV) per cell,
  E <|psi'|^2>_g = |psi_cl|^2 + sigma^2,
  E Var rho_g   = (1 - 1/N_s) M^2 (2 |psi_cl|^2 sigma^2 + sigma^4),
  E Q_raw(0)    = (1 - 1/N_s) N / (2 n_tot),
the (1 - 1/N_s) being the bias of the plug-in estimator. The scaling
Q ~ 1/n_tot in the linear regime is the invariant of Eq. (Q_relation).
"""
import numpy as np

from oracle import twa_oracle as tw
from paper_2310_07119_amd import inputs


def test_moments_brute_force_tiny():
    grid = tw.Grid((8,), (1.0,))
    prob = tw.Problem(grid, m_tot=2.0)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((3, 8)) + 1j * rng.standard_normal((3, 8))
    psi_cl = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    m = tw.moments(prob, psi, 50.0, psi_cl)
    dV = 1.0 / 8
    q = 0.0
    dev_r = 0.0
    dev_p = 0.0
    for g in range(8):
        vals = [complex(psi[r, g]) for r in range(3)]
        mean = sum(vals) / 3
        m2 = sum(abs(v) ** 2 for v in vals) / 3
        rhos = [2.0 * abs(v) ** 2 for v in vals]
        mr = sum(rhos) / 3
        vr = sum((x - mr) ** 2 for x in rhos) / 3
        assert abs(m["mean_psi"][g] - mean) < 1e-14
        assert abs(m["mean_abs2"][g] - m2) < 1e-14
        assert abs(m["mean_rho"][g] - mr) < 1e-14
        assert abs(m["var_rho"][g] - vr) < 1e-13
        q += (m2 - abs(mean) ** 2) * dV
        dev_r += abs(mr - 2.0 * abs(psi_cl[g]) ** 2) * dV / 2.0
        dev_p += abs(mean - psi_cl[g]) ** 2 * dV
    assert abs(m["Q_raw"] - q) < 1e-14
    assert abs(m["Q_sym"] - (q - 8 / 100.0)) < 1e-14
    assert abs(m["dev_rho_L1"] - dev_r) < 1e-14
    assert abs(m["dev_psi_L2"] - dev_p) < 1e-14
    for r in range(3):
        assert abs(m["norm"][r] - sum(abs(psi[r, g]) ** 2 for g in range(8)) * dV) < 1e-14


def test_moments_closed_forms_at_t0():
    n = (16, 8)
    grid = tw.Grid(n, (1.0, 0.5))
    prob = tw.Problem(grid, m_tot=3.0)
    psi_cl = inputs.lognormal_field(n, (1.0, 0.5), seed=2)
    n_tot, ns = 40.0, 3000
    psi = tw.sample(grid, psi_cl, ns, n_tot, seed=17)
    m = tw.moments(prob, psi, n_tot, psi_cl)
    sig2 = 1.0 / (2 * n_tot * grid.dV)
    a2 = np.abs(psi_cl) ** 2
    e_m2 = a2 + sig2
    se_m2 = np.sqrt((2 * a2 * sig2 + sig2 ** 2) / ns)
    assert np.all(np.abs(m["mean_abs2"] - e_m2) < 5 * se_m2)
    e_var = (1 - 1 / ns) * prob.m_tot ** 2 * (2 * a2 * sig2 + sig2 ** 2)
    ratio = (m["var_rho"] / e_var).mean()
    assert abs(ratio - 1.0) < 0.02
    e_q = (1 - 1 / ns) * grid.ncell / (2 * n_tot)
    assert abs(m["Q_raw"] / e_q - 1.0) < 5 * np.sqrt(1.0 / (ns * grid.ncell)) * 2
    assert abs(m["Q_sym"]) < 0.01 * e_q + grid.ncell / (2 * n_tot) / ns * 2
    e_norm = 1 + grid.ncell / (2 * n_tot)
    assert abs(m["norm"].mean() - e_norm) < 5 * m["norm"].std() / np.sqrt(ns)


def test_zero_noise_limit():
    grid = tw.Grid((32,), (1.0,))
    prob = tw.Problem(grid)
    psi_cl = inputs.lognormal_field((32,), (1.0,), seed=1)
    psi = tw.sample(grid, psi_cl, 4, np.inf, seed=3)
    assert np.array_equal(psi, np.broadcast_to(psi_cl, psi.shape))
    psi = tw.evolve(prob, psi, 10, 1e-3)
    m = tw.moments(prob, psi, np.inf, tw.evolve(prob, psi_cl, 10, 1e-3))
    assert np.max(m["var_rho"]) == 0.0 and abs(m["Q_raw"]) < 1e-15
    assert m["dev_rho_L1"] == 0.0 and m["dev_psi_L2"] == 0.0


def test_q_scales_inversely_with_n_tot():
    """Eq. (Q_relation): Q(t) - Q(0) ~ 1/n_tot while it is small; same seed, n and 4n."""
    grid = tw.Grid((64,), (1.0,))
    prob = tw.Problem(grid, hbar_m=0.02, G=1.0, m_tot=5.0)
    psi_cl = inputs.lognormal_field((64,), (1.0,), kcut=4, seed=3)
    out = []
    for n_tot in (1e8, 4e8):
        psi = tw.sample(grid, psi_cl, 64, n_tot, seed=5)
        q0 = tw.moments(prob, psi, n_tot)["Q_raw"]
        psi = tw.evolve(prob, psi, 200, 2e-3)
        q1 = tw.moments(prob, psi, n_tot)["Q_raw"]
        out.append((q1 - q0) * n_tot)
    assert abs(out[0]) > 1e-3
    assert abs(out[0] / out[1] - 1.0) < 1e-3


def test_nonfinite_flag():
    grid = tw.Grid((8,), (1.0,))
    prob = tw.Problem(grid)
    psi = np.ones((4, 8), complex)
    psi[2, 5] = np.nan
    assert tw.moments(prob, psi, 10.0)["nonfinite"] == 1


def test_mode_occupation_brute_force_and_parseval():
    """<|a_j|^2> summed from the DFT's definition on a non-square grid (a swapped
    axis or a missing 1/sqrt(N) fails it), and Parseval: sum_j <|a_j|^2> equals
    n_tot dV sum_g <|psi'|^2>_g."""
    n = (4, 3)
    grid = tw.Grid(n, (1.0, 0.6))
    prob = tw.Problem(grid)
    rng = np.random.default_rng(3)
    ns, n_tot = 3, 7.0
    psi = rng.standard_normal((ns, 3, 4)) + 1j * rng.standard_normal((ns, 3, 4))
    m = tw.moments(prob, psi, n_tot, modes=True)
    N = 12
    for jy in range(3):
        for jx in range(4):
            acc = 0.0
            for r in range(ns):
                s = 0j
                for y in range(3):
                    for x in range(4):
                        s += np.sqrt(n_tot * grid.dV) * psi[r, y, x] * np.exp(-2j * np.pi * (jx * x / 4 + jy * y / 3))
                acc += abs(s / np.sqrt(N)) ** 2
            assert abs(m["mode_occ"][jy, jx] - acc / ns) < 1e-12 * max(1.0, acc / ns)
    assert abs(m["mode_occ"].sum() - n_tot * grid.dV * m["mean_abs2"].sum()) < 1e-12 * m["mode_occ"].sum()


def test_mode_occupation_half_quantum_at_t0():
    """Right after sampling every mode holds its classical occupation plus the
    Weyl vacuum half quantum: E<|a_j|^2> = |a_cl,j|^2 + 1/2."""
    n = (16, 8)
    grid = tw.Grid(n, (1.0, 0.5))
    prob = tw.Problem(grid)
    psi_cl = inputs.lognormal_field(n, (1.0, 0.5), seed=4)
    n_tot, ns = 200.0, 2000
    psi = tw.sample(grid, psi_cl, ns, n_tot, seed=23)
    m = tw.moments(prob, psi, n_tot, modes=True)
    occ_cl = np.abs(tw.mode_amplitudes(prob, psi_cl, n_tot)) ** 2
    sigma = np.sqrt((2 * occ_cl + 0.5) * 0.5 / ns)
    assert np.all(np.abs(m["mode_occ"] - occ_cl - 0.5) < 6 * sigma)


def test_decoherence_brute_force_tiny():
    """Amplitude/phase spread summed by hand on 3 realizations of 6 cells,
    including a phase deviation beyond pi/2 and the normal-ordering shift."""
    grid = tw.Grid((6,), (1.5,))
    prob = tw.Problem(grid)
    rng = np.random.default_rng(8)
    psi = rng.standard_normal((3, 6)) + 1j * rng.standard_normal((3, 6))
    n_tot = 4.0
    va, vp, VA, VP = tw.decoherence(prob, psi, n_tot)
    dV = 0.25
    ta = tp = 0.0
    import cmath
    import math
    for g in range(6):
        vals = [complex(psi[r, g]) for r in range(3)]
        m1 = sum(vals) / 3
        amps = [abs(v) for v in vals]
        ma = sum(amps) / 3
        a_var = sum((x - ma) ** 2 for x in amps) / 3
        dev = [cmath.phase(v / m1) for v in vals]       # same angle as v conj(m1)
        p_var = sum(d * d for d in dev) / 3
        assert abs(va[g] - a_var) < 1e-13 and abs(vp[g] - p_var) < 1e-13
        occ = sum(abs(v) ** 2 for v in vals) / 3 - 1 / (2 * n_tot * dV)
        ta += dV * occ * a_var / ma
        tp += dV * occ * p_var / (math.pi / math.sqrt(3))
    assert abs(VA - ta) < 1e-13 and abs(VP - tp) < 1e-13


def test_decoherence_limits():
    """A coherent ensemble (identical realizations) has no spread at all; with
    uniformly random phases at fixed amplitude the amplitude spread vanishes
    and <dphi^2> tends to pi^2/3, the variance of a uniform angle."""
    grid = tw.Grid((16,), (1.0,))
    prob = tw.Problem(grid)
    base = inputs.lognormal_field((16,), (1.0,), seed=1)
    same = np.repeat(base[None], 5, axis=0)
    va, vp, VA, VP = tw.decoherence(prob, same, 1e30)
    assert np.all(va < 1e-28) and np.all(vp == 0.0) and abs(VA) < 1e-25 and VP == 0.0
    rng = np.random.default_rng(2)
    ns = 20000
    phases = rng.uniform(-np.pi, np.pi, (ns, 16))
    psi = np.abs(base)[None] * np.exp(1j * phases)
    va, vp, VA, VP = tw.decoherence(prob, psi, 1e30)
    assert np.all(va < 1e-20)   # rounding only: amplitudes are equal
    # the deviation is taken from the (nearly random) phase of the mean field: still uniform on the circle
    assert np.all(np.abs(vp - np.pi ** 2 / 3) < 0.1)
    norm = (np.abs(base) ** 2).sum() * grid.dV
    assert abs(VP - norm * (np.pi ** 2 / 3) / (np.pi / np.sqrt(3))) < 0.05 * VP
