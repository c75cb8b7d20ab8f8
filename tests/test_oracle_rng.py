"""Pins for the oracle's counter-based generator and Wigner sampler.

Philox4x64-10 is pinned against numpy's independent implementation
(numpy.random.Philox); the project-written log and sin/cos against numpy's
libm-backed routines; the sampler against the statistics the paper fixes for
a coherent state's Wigner function (Sec. "Initial conditions generation").
"""
import numpy as np
import pytest

from oracle import philox
from oracle import twa_oracle as tw


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 3, 9, 0), (123, 456)),
    ((7, 0, 1, 2 ** 63), (2 ** 64 - 1, 0x5457)),
    ((2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1), (2 ** 64 - 1, 2 ** 64 - 1)),
    ((12345, 678, 0, 0), (0, 0x5457)),
])
def test_philox_matches_numpy_bitgenerator(ctr, key):
    # numpy's Philox increments the counter before producing a block.
    c = list(ctr)
    c[0] -= 1
    carry = 0
    if c[0] < 0:
        c[0] += 2 ** 64
        carry = 1
    for i in range(1, 4):
        if not carry:
            break
        c[i] -= 1
        carry = 0
        if c[i] < 0:
            c[i] += 2 ** 64
            carry = 1
    ref = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                           key=np.array(key, dtype=np.uint64)).random_raw(4)
    got = philox.philox4x64([[v] for v in ctr], key)[:, 0]
    assert [int(v) for v in got] == [int(v) for v in ref]


def test_uniform52_range_and_exactness():
    x = np.array([0, 1, 2 ** 12 - 1, 2 ** 12, 2 ** 64 - 1], dtype=np.uint64)
    u = philox.uniform52(x)
    assert u[0] == 2.0 ** -53 and u[1] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[3] == 1.5 * 2.0 ** -52
    assert u[4] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_log_series_vs_libm():
    rng = np.random.default_rng(3)
    u = np.concatenate([rng.random(200000), 2.0 ** -rng.uniform(0, 53, 20000),
                        [2.0 ** -53, 1.0 - 2.0 ** -53, 0.5, 0.70710678118654746,
                         0.70710678118654757]])
    u = u[u > 0]
    ref = np.log(u)
    got = philox.log_series(u)
    # within 3 units in the last place of the correctly rounded value
    assert np.max(np.abs(got - ref) / np.spacing(np.abs(ref))) <= 3.0


def test_cos_sin_turn_vs_libm():
    rng = np.random.default_rng(4)
    u = np.concatenate([rng.random(200000), np.arange(1, 16) / 16.0,
                        [2.0 ** -53, 1.0 - 2.0 ** -53]])
    c, s = philox.cos_sin_turn(u)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 1e-15
    assert np.max(np.abs(s - np.sin(2 * np.pi * u))) < 1e-15
    assert np.max(np.abs(c * c + s * s - 1.0)) < 5e-16


def test_box_muller_is_standard_normal():
    from scipy import stats
    words = philox.philox4x64([np.arange(200000, dtype=np.uint64), np.zeros(200000, np.uint64),
                               np.zeros(200000, np.uint64), np.zeros(200000, np.uint64)], (7, 0x5457))
    z1, z2 = philox.box_muller(words[0], words[1])
    n = z1.size
    for z in (z1, z2):
        assert abs(z.mean()) < 5 / np.sqrt(n)
        assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(z, "norm").pvalue > 1e-4
    assert abs(np.mean(z1 * z2)) < 5 / np.sqrt(n)


def test_sample_vacuum_noise_per_cell_mode():
    """E d alpha = 0, E|d alpha|^2 = 1/2, E d alpha^2 = 0 per cell mode (coherent-state Wigner)."""
    grid = tw.Grid((64, 32), (1.0, 2.0))
    n_tot = 1e4
    psi_cl = np.full(grid.shape, 0.3 + 0.1j)
    psi = tw.sample(grid, psi_cl, 64, n_tot, seed=11)
    alpha = (psi - psi_cl[None]) * np.sqrt(n_tot * grid.dV)
    m = alpha.size
    assert abs(alpha.mean()) < 5 * np.sqrt(0.5 / m)
    a2 = np.abs(alpha) ** 2
    assert abs(a2.mean() - 0.5) < 5 * 0.5 / np.sqrt(m)
    sq = (alpha ** 2).mean()
    assert abs(sq) < 5 * 0.5 / np.sqrt(m)
    assert abs((alpha.real ** 2).mean() - 0.25) < 5 * 0.25 * np.sqrt(2.0 / m)


def test_sample_mode_occupation_is_n_plus_half():
    """Under the unitary DFT, E|a_j|^2 = |z_j|^2 + 1/2 per Fourier mode."""
    grid = tw.Grid((32,), (1.0,))
    prob = tw.Problem(grid)
    n_tot = 200.0
    x = np.arange(32) / 32.0
    psi_cl = (1.0 + 0.5 * np.cos(2 * np.pi * 3 * x)).astype(complex)
    psi_cl /= np.sqrt((np.abs(psi_cl) ** 2).sum() * grid.dV)
    ns = 4000
    psi = tw.sample(grid, psi_cl, ns, n_tot, seed=5)
    occ = (np.abs(tw.mode_amplitudes(prob, psi, n_tot)) ** 2).mean(axis=0)
    occ_cl = np.abs(tw.mode_amplitudes(prob, psi_cl, n_tot)) ** 2
    assert abs(occ_cl.sum() - n_tot) < 1e-9 * n_tot
    sigma = np.sqrt((2 * occ_cl + 0.5) * 0.5 / ns) + 0.5 / np.sqrt(ns)
    assert np.all(np.abs(occ - occ_cl - 0.5) < 6 * sigma)


def test_sample_offset_and_independence():
    grid = tw.Grid((8, 8), (1.0, 1.0))
    psi_cl = np.zeros(grid.shape, complex)
    full = tw.sample(grid, psi_cl, 6, 10.0, seed=99)
    part = tw.sample(grid, psi_cl, 2, 10.0, seed=99, real_offset=3)
    assert np.array_equal(full[3:5], part)
    other = tw.sample(grid, psi_cl, 6, 10.0, seed=100)
    assert not np.any(full == other)
