"""Breaktime analysis of a truncated-Wigner run (Sec. "Estimating the
breaktime", Eq. (Q_relation); Sec. "Breaktimes").

The GPU path reduces the ensemble to the scalar Q_s(t) at each output time
(tw_moments); this module records that series and does the analysis the
paper does on it, on the host, over a few hundred scalars:

* Q_p(t) = (n_s / n_p) Q_s(t): the sampling particle number n_s only sets the
  noise amplitude, so Q measured with n_s predicts the physical Q for the
  physical occupation n_p while Q << 1 (Eq. (Q_relation));
* growth fits: quadratic Q = a t^2 (stable, virialised systems and early
  times) and exponential Q = A e^(lambda t) (nonlinear collapse and mergers);
* breaktimes: the time at which the fitted physical Q reaches 1, and the
  paper's estimate for collapsing systems t_br ~ ln(n_tot) t_c / 7 with the
  dynamical time t_c ~ sqrt(L^D / (G M_tot));
* spectra over time: per-mode occupations <|a_k|^2> averaged over shells of
  |k| (the mode_occ output of tw_moments).

The sampled ensemble only estimates the initial Wigner function, so the
simulated Q at t = 0 is not exactly zero; the paper therefore subtracts the
sampled initial value and analyses Q_s(t) - Q_s(0) (Sec. "Estimating the
breaktime"). `record` returns that series as Q_minus_Q0 (Q_raw minus its value
at the first output, which `record` takes at the start of the run). Q_sym of
tw_moments (Q_raw with the Weyl half quantum per cell mode, N / (2 n_tot),
removed) is not a substitute at t = 0: with the plug-in estimator
E Q_raw(0) = (1 - 1/N_s) N / (2 n_tot), so E Q_sym(0) = -N / (2 n_tot N_s),
a bias that shrinks only as 1/N_s.
"""
from __future__ import annotations

import math

import numpy as np


def q_physical(q_sim, n_sim: float, n_phys: float):
    """Q_p = (n_s / n_p) Q_s (Eq. (Q_relation)); valid while Q_s << 1."""
    if not (n_sim > 0 and n_phys > 0):
        raise ValueError("particle numbers must be positive")
    return np.asarray(q_sim, dtype=np.float64) * (n_sim / n_phys)


def fit_quadratic(t, q) -> float:
    """Least-squares a of Q = a t^2 (no constant or linear term: Q(0) = 0)."""
    t = np.asarray(t, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if t.shape != q.shape or t.size == 0:
        raise ValueError("t and q must be non-empty arrays of one shape")
    den = np.sum(t ** 4)
    if den == 0.0:
        raise ValueError("all times are zero")
    return float(np.sum(t ** 2 * q) / den)


def fit_exponential(t, q):
    """Least-squares (ln A, lambda) of ln Q = ln A + lambda t over the points
    with Q > 0 (at least two are needed)."""
    t = np.asarray(t, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if t.shape != q.shape:
        raise ValueError("t and q must have one shape")
    keep = q > 0
    if np.count_nonzero(keep) < 2:
        raise ValueError("an exponential fit needs two points with Q > 0")
    tt, lq = t[keep], np.log(q[keep])
    tm, lm = tt.mean(), lq.mean()
    var = np.sum((tt - tm) ** 2)
    if var == 0.0:
        raise ValueError("an exponential fit needs two distinct times")
    lam = float(np.sum((tt - tm) * (lq - lm)) / var)
    return float(lm - lam * tm), lam


def breaktime_quadratic(a_phys: float) -> float:
    """t with a_p t^2 = 1, from the quadratic growth of the physical Q."""
    if a_phys <= 0:
        raise ValueError("quadratic coefficient must be positive")
    return 1.0 / math.sqrt(a_phys)


def breaktime_exponential(log_a_phys: float, lam: float) -> float:
    """t with A_p e^(lambda t) = 1, from the exponential growth of the physical Q."""
    if lam <= 0:
        raise ValueError("growth rate must be positive")
    return -log_a_phys / lam


def dynamical_time(box, G: float, m_tot: float) -> float:
    """t_c ~ sqrt(L^D / (G M_tot)) for a box of side lengths `box` (Sec. "Breaktimes")."""
    vol = float(np.prod(np.asarray(box, dtype=np.float64)))
    if G <= 0 or m_tot <= 0:
        raise ValueError("G and M_tot must be positive")
    return math.sqrt(vol / (G * m_tot))


def breaktime_collapse_estimate(n_tot: float, t_c: float, rate: float = 7.0) -> float:
    """The paper's estimate for collapsing systems, Q ~ e^(rate t / t_c) / n_tot
    with rate about 7: t_br ~ ln(n_tot) t_c / rate."""
    return math.log(n_tot) * t_c / rate


def shell_spectrum(mode_occ, box):
    """Shell average of per-mode occupations: returns (k_centres, mean <|a_k|^2>
    per shell, modes per shell). mode_occ has the field's array shape (x last,
    FFT order); shells are |k| in units of the smallest 2 pi / L_d, rounded."""
    occ = np.asarray(mode_occ, dtype=np.float64)
    dim = occ.ndim
    box = tuple(float(b) for b in box)[:dim]
    kmag2 = np.zeros(occ.shape)
    for d in range(dim):                         # grid axis d is array axis dim-1-d
        n = occ.shape[dim - 1 - d]
        kd = 2.0 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / box[d]
        shape = [1] * dim
        shape[dim - 1 - d] = n
        kmag2 = kmag2 + (kd ** 2).reshape(shape)
    dk = min(2.0 * np.pi / b for b in box)
    shell = np.rint(np.sqrt(kmag2) / dk).astype(np.int64).ravel()
    counts = np.bincount(shell)
    sums = np.bincount(shell, weights=occ.ravel())
    used = counts > 0
    return np.nonzero(used)[0] * dk, sums[used] / counts[used], counts[used]


def record(plan, psi, psi_classical, nsteps: int, dt: float, every: int, modes: bool = False):
    """Advance the ensemble `nsteps` steps of size dt on the GPU, taking the
    moments every `every` steps (and at t = 0). Returns a dict of host arrays:
    t, Q_raw, Q_sym, Q_minus_Q0 (Q_raw minus its sampled value at the first
    output: the series the paper fits), dev_rho_L1, dev_psi_L2 (and mode_occ,
    one field-shaped array per output, if modes)."""
    if every <= 0 or nsteps < 0:
        raise ValueError("every must be positive and nsteps non-negative")
    keys = ("Q_raw", "Q_sym", "dev_rho_L1", "dev_psi_L2")
    out = {k: [] for k in ("t",) + keys}
    if modes:
        out["mode_occ"] = []
    done = 0
    while True:
        m = plan.moments(psi, psi_classical, energy=False, per_cell=False, modes=modes)
        out["t"].append(done * dt)
        for k in keys:
            out[k].append(m[k])
        if modes:
            out["mode_occ"].append(m["mode_occ"].cpu().numpy())
        if done >= nsteps:
            break
        k = min(every, nsteps - done)
        plan.step(psi, k, dt, psi_classical)
        done += k
    res = {k: (np.asarray(v) if k != "mode_occ" else v) for k, v in out.items()}
    res["Q_minus_Q0"] = res["Q_raw"] - res["Q_raw"][0]
    return res
