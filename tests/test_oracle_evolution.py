"""Pins for the oracle's transforms and split-step evolution.

Each check is fixed by mathematics independent of the oracle's own code:
the DFT summed from its definition, exact solutions of the free Schrodinger
equation, the closed-form potential of a cosine density, the linear Jeans
dispersion of the Schrodinger-Poisson system, and the conservation laws and
time-reversal symmetry of the symplectic Strang splitting (Sec. "Integrating
the equations of motion").
"""
import numpy as np
import pytest

from oracle import twa_oracle as tw
from paper_2310_07119_amd import inputs


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(np.asarray(b).ravel())


# ----------------------------------------------------------------- transforms
@pytest.mark.parametrize("n", [(8,), (16,), (8, 16), (16, 8), (8, 8, 8), (4, 8, 16)])
def test_fft_equals_naive_dft(n):
    grid = tw.Grid(n, (1.0,) * len(n))
    rng = np.random.default_rng(1)
    f = rng.standard_normal((3,) + grid.shape) + 1j * rng.standard_normal((3,) + grid.shape)
    fast, slow = tw.Transform(grid, "fft"), tw.Transform(grid, "naive")
    assert rel(fast.fwd(f), slow.fwd(f)) < 1e-13
    assert rel(fast.inv(f), slow.inv(f)) < 1e-13
    assert rel(fast.inv(fast.fwd(f)), f) < 1e-14


def test_dft_delta_constant_and_parseval():
    grid = tw.Grid((8, 16), (1.0, 1.0))
    T = tw.Transform(grid, "naive")
    delta = np.zeros(grid.shape, complex)
    delta[0, 0] = 1.0
    assert np.allclose(T.fwd(delta), 1.0, atol=1e-14)
    const = np.ones(grid.shape, complex)
    F = T.fwd(const)
    assert abs(F[0, 0] - grid.ncell) < 1e-12 and np.abs(F).sum() - grid.ncell < 1e-9
    rng = np.random.default_rng(2)
    f = rng.standard_normal(grid.shape) + 1j * rng.standard_normal(grid.shape)
    assert abs((np.abs(f) ** 2).sum() - (np.abs(T.fwd(f)) ** 2).sum() / grid.ncell) < 1e-12 * grid.ncell


def test_wavenumbers_fft_order():
    grid = tw.Grid((8,), (2.0,))
    k = grid.k_axis(0)
    assert np.allclose(k, np.pi * np.array([0, 1, 2, 3, -4, -3, -2, -1]))


@pytest.mark.parametrize("n", [(16,), (8, 8), (4, 8, 8)])
def test_step_naive_equals_fft(n):
    grid = tw.Grid(n, (1.0,) * len(n))
    psi = inputs.random_field(n, seed=4)[None] * 0.3
    a = tw.evolve(tw.Problem(grid, 1.0, 3.0, 2.0, "fft"), psi, 5, 1e-3)
    b = tw.evolve(tw.Problem(grid, 1.0, 3.0, 2.0, "naive"), psi, 5, 1e-3)
    assert rel(a, b) < 1e-12


# --------------------------------------------------------- exact solutions
def test_plane_wave_phase_is_exact():
    grid = tw.Grid((32, 16), (1.0, 2.0))
    prob = tw.Problem(grid, hbar_m=0.7, G=5.0, m_tot=3.0)
    X = np.arange(32)[None, :] / 32.0
    Y = np.arange(16)[:, None] * (2.0 / 16)
    kx, ky = 2 * np.pi * 3, 2 * np.pi * (-2) / 2.0
    psi0 = np.exp(1j * (kx * X + ky * Y)) / np.sqrt(grid.volume)
    nsteps, dt = 40, 1e-3
    psi = tw.evolve(prob, psi0, nsteps, dt)
    expect = psi0 * np.exp(-1j * prob.hbar * (kx ** 2 + ky ** 2) * nsteps * dt / 2.0)
    assert np.max(np.abs(psi - expect)) < 1e-13 * np.max(np.abs(psi0)) * 10


def _free_packet_1d(x, t, L, sigma, x0, k0, hbar, images=6):
    """Periodised exact free evolution of a Gaussian packet."""
    a = 1.0 + 1j * hbar * t / (2 * sigma ** 2)
    out = np.zeros_like(x, dtype=complex)
    for m in range(-images, images + 1):
        xm = x + m * L
        out += (np.exp(-(xm - x0 - hbar * k0 * t) ** 2 / (4 * sigma ** 2 * a)
                       + 1j * k0 * (xm - x0) - 1j * hbar * k0 ** 2 * t / 2) / np.sqrt(a))
    return out * (2 * np.pi * sigma ** 2) ** -0.25


def test_free_gaussian_packet_1d():
    L, n = 1.0, 256
    grid = tw.Grid((n,), (L,))
    prob = tw.Problem(grid, hbar_m=0.5, G=0.0)
    x = np.arange(n) * L / n
    sig, x0, k0 = 0.05, 0.4, 2 * np.pi * 4.3
    psi0 = _free_packet_1d(x, 0.0, L, sig, x0, k0, prob.hbar)
    nsteps, dt = 50, 2e-4
    psi = tw.evolve(prob, psi0, nsteps, dt)
    exact = _free_packet_1d(x, nsteps * dt, L, sig, x0, k0, prob.hbar)
    assert rel(psi, exact) < 1e-12


def test_free_gaussian_packet_2d_product():
    L, n = 1.0, (64, 32)
    grid = tw.Grid(n, (L, L))
    prob = tw.Problem(grid, hbar_m=1.0, G=0.0)
    x = np.arange(64) / 64.0
    y = np.arange(32) / 32.0
    sx, sy = 0.06, 0.08
    f = lambda t: (_free_packet_1d(y, t, L, sy, 0.5, -2 * np.pi, 1.0)[:, None]
                   * _free_packet_1d(x, t, L, sx, 0.3, 2 * np.pi * 2, 1.0)[None, :])
    psi = tw.evolve(prob, f(0.0), 20, 5e-4)
    assert rel(psi, f(20 * 5e-4)) < 1e-12


# ---------------------------------------------------------------- Poisson
def test_poisson_cosine_closed_form():
    grid = tw.Grid((32, 16, 8), (1.0, 2.0, 0.5))
    prob = tw.Problem(grid, G=2.5)
    Z, Y, X = np.meshgrid(np.arange(8) * 0.5 / 8, np.arange(16) * 2.0 / 16,
                          np.arange(32) / 32.0, indexing="ij")
    kvec = (2 * np.pi * 3, 2 * np.pi * 1 / 2.0, 2 * np.pi * 2 / 0.5)
    arg = kvec[0] * X + kvec[1] * Y + kvec[2] * Z
    rho = 7.0 + 0.3 * np.cos(arg)
    V = tw.potential(prob, rho)
    k2 = sum(k * k for k in kvec)
    assert np.max(np.abs(V - (-4 * np.pi * prob.G * 0.3 * np.cos(arg) / k2))) < 1e-13
    assert abs(V.mean()) < 1e-15


def test_uniform_density_no_force_and_kick_preserves_modulus():
    grid = tw.Grid((16, 16), (1.0, 1.0))
    prob = tw.Problem(grid, G=10.0)
    assert np.max(np.abs(tw.potential(prob, np.full(grid.shape, 3.3)))) < 1e-14
    psi = inputs.random_field((16, 16), seed=8)
    V = np.random.default_rng(0).standard_normal(grid.shape) * 50
    out = tw.kick(prob, psi, V, 1e-2)
    assert np.max(np.abs(np.abs(out) - np.abs(psi))) < 1e-14 * np.max(np.abs(psi)) * 10


@pytest.mark.parametrize("m_tot,kind", [(20.0, "oscillate"), (40.0, "grow")])
def test_linear_jeans_dispersion(m_tot, kind):
    """Small density mode on a uniform background: omega^2 = (hbar k^2/2)^2 - 4 pi G rho_bar."""
    L, n = 1.0, 64
    grid = tw.Grid((n,), (L,))
    prob = tw.Problem(grid, hbar_m=1.0, G=1.0, m_tot=m_tot)
    x = np.arange(n) / n
    k = 2 * np.pi / L
    eps = 1e-6
    psi0 = (1 + eps * np.cos(k * x)).astype(complex) / np.sqrt(L)
    rho_bar = m_tot / L
    w2 = (prob.hbar * k * k / 2) ** 2 - 4 * np.pi * prob.G * rho_bar
    dt, nsteps = 1e-4, 1500
    psi = tw.evolve(prob, psi0, nsteps, dt)
    t = nsteps * dt
    contrast = (np.abs(psi) ** 2) * L - 1.0
    amp = 2 * np.sum(contrast * np.cos(k * x)) / n        # coefficient of cos(kx)
    expect = 2 * eps * (np.cos(np.sqrt(w2) * t) if w2 > 0 else np.cosh(np.sqrt(-w2) * t))
    assert (w2 > 0) == (kind == "oscillate")
    assert abs(amp - expect) < 2e-3 * abs(2 * eps) * max(1.0, abs(expect / (2 * eps)))
    # and it is NOT the free (G=0) answer
    free = 2 * eps * np.cos(prob.hbar * k * k / 2 * t)
    assert abs(free - expect) > 50 * abs(amp - expect)


# --------------------------------------------------- conservation / symmetry
def _nonlinear_1d():
    grid = tw.Grid((128,), (1.0,))
    prob = tw.Problem(grid, hbar_m=0.05, G=1.0, m_tot=5.0)
    psi0 = inputs.lognormal_field((128,), (1.0,), seed=3)
    return prob, psi0


def test_norm_conserved():
    prob, psi0 = _nonlinear_1d()
    psi = tw.evolve(prob, psi0, 1000, 1e-3)
    assert abs(tw.norm(prob, psi) - tw.norm(prob, psi0)) < 1e-12


def test_energy_error_second_order():
    grid = tw.Grid((128,), (1.0,))
    prob = tw.Problem(grid, hbar_m=0.05, G=1.0, m_tot=5.0)
    psi0 = inputs.lognormal_field((128,), (1.0,), kcut=6, seed=3)
    T = 0.4
    errs = []
    for nst in (100, 200, 400):
        psi = tw.evolve(prob, psi0, nst, T / nst)
        errs.append(abs(tw.energy(prob, psi) - tw.energy(prob, psi0)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, errs


def test_time_reversal():
    prob, psi0 = _nonlinear_1d()
    fwd = tw.evolve(prob, psi0, 300, 1e-3)
    back = tw.evolve(prob, fwd, 300, -1e-3)
    assert rel(back, psi0) < 1e-11
    assert rel(fwd, psi0) > 1e-2


# ------------------------------------------------------------- adaptive step
def test_adaptive_free_field_equals_fixed_step():
    """With G = 0 the potential bound never binds, so the adaptive evolution is
    the fixed-step one at min(dt_max, c_f * kinetic bound), exactly."""
    grid = tw.Grid((32, 16), (1.0, 0.5))
    prob = tw.Problem(grid, hbar_m=0.8, G=0.0)
    psi = inputs.lognormal_field((32, 16), (1.0, 0.5), seed=3)[None]
    got, dts = tw.evolve_adaptive(prob, psi, 4, 1e-3, 0.5)
    assert np.all(dts == 1e-3)
    assert np.array_equal(got, tw.evolve(prob, psi, 4, 1e-3))
    big, dts = tw.evolve_adaptive(prob, psi, 2, 10.0, 0.5)
    # kinetic bound: dt < 4 pi / (hbar k_max dk), k_max = pi / dx, dk = 2 pi / L, worst axis
    kin = min(4 * np.pi / (0.8 * (np.pi * n / L) * (2 * np.pi / L)) for n, L in ((32, 1.0), (16, 0.5)))
    assert abs(kin - 2 * 0.5 ** 2 / (np.pi * 16 * 0.8)) < 1e-15
    assert np.allclose(dts, 0.5 * kin, rtol=1e-15, atol=0)


def test_adaptive_potential_bound_closed_form():
    """Uniform density plus a cosine: V = -4 pi G eps cos(k0 x) / k0^2 exactly
    (the mean is removed), so the first step is c_f 2 pi hbar / max|V| with
    max|V| from that closed form, when it is the tighter bound."""
    n, L = 64, 1.0
    grid = tw.Grid((n,), (L,))
    hbar, G, m_tot, c = 0.02, 30.0, 1.0, 0.7
    prob = tw.Problem(grid, hbar_m=hbar, G=G, m_tot=m_tot)
    x = np.arange(n) * L / n
    eps, k0 = 0.2, 2 * np.pi * 2 / L
    rho = m_tot / L * (1 + eps * np.cos(k0 * x))
    psi = np.sqrt(rho / m_tot).astype(complex)[None]
    vmax = 4 * np.pi * G * (m_tot / L) * eps / k0 ** 2
    _, dts = tw.evolve_adaptive(prob, psi, 1, 1.0, c)
    expect = c * 2 * np.pi * hbar / vmax
    assert expect < c * 2 * L * (L / n) / (np.pi * hbar)
    assert abs(dts[0] - expect) < 1e-12 * expect


def test_adaptive_lag_rule():
    """Steps 0 and 1 share the size set by the initial potential; the size of
    step n + 2 comes from the potential evaluated inside step n (recomputed
    here with the fixed-step pieces at the returned sizes)."""
    grid = tw.Grid((32,), (1.0,))
    prob = tw.Problem(grid, hbar_m=0.05, G=1.0, m_tot=30.0)
    psi0 = np.stack([inputs.lognormal_field((32,), (1.0,), seed=s) for s in (1, 2)])
    _, dts = tw.evolve_adaptive(prob, psi0, 5, 1.0, 0.5)
    assert dts[0] == dts[1]
    assert len(set(dts.tolist())) > 2   # the potential bound binds and varies
    psi = psi0
    for n in range(3):
        half = tw.drift(prob, psi, dts[n] / 2)
        V = tw.potential(prob, tw.density(prob, half))
        assert dts[n + 2] == min(1.0, 0.5 * tw.kinetic_dt_bound(prob), 0.5 * 2 * np.pi * 0.05 / np.abs(V).max())
        psi = tw.step(prob, psi, dts[n])


# ----------------------------------------------------------- tracer particles
def test_tracers_move_straight_without_gravity():
    grid = tw.Grid((16, 8), (1.0, 0.5))
    prob = tw.Problem(grid, G=0.0)
    psi = inputs.lognormal_field((16, 8), (1.0, 0.5), seed=2)[None]
    tr = np.array([[[0.1, 0.2, 3.0, -1.5], [0.9, 0.45, -0.2, 0.7]]])
    _, got = tw.evolve_tracers(prob, psi, tr, 5, 1e-2)
    expect = tr.copy()
    expect[:, :, :2] += 5 * 1e-2 * tr[:, :, 2:]
    assert np.allclose(got, expect, rtol=0, atol=1e-15)


def test_fourth_order_gradient_of_a_cosine():
    """The fourth-order difference of cos(kx) is -sin(kx) (8 sin(k dx) - sin(2 k dx)) / (6 dx)."""
    n, L = 32, 2.0
    grid = tw.Grid((n,), (L,))
    prob = tw.Problem(grid)
    x = np.arange(n) * L / n
    k, dx = 2 * np.pi * 3 / L, L / n
    (gx,) = tw.grid_gradient(prob, np.cos(k * x)[None])
    expect = -np.sin(k * x) * (8 * np.sin(k * dx) - np.sin(2 * k * dx)) / (6 * dx)
    assert np.allclose(gx[0], expect, rtol=0, atol=1e-13)
    assert np.max(np.abs(gx[0] + k * np.sin(k * x))) < 1e-2 * k   # and it approximates the derivative


def test_cic_interpolation_is_exact_for_linear_fields():
    """Between grid points a bilinear field is reproduced exactly (away from the
    periodic seam), and positions outside the box wrap."""
    grid = tw.Grid((8, 4), (2.0, 1.0))
    prob = tw.Problem(grid)
    y, x = np.meshgrid(np.arange(4) * 0.25, np.arange(8) * 0.25, indexing="ij")
    F = (1.0 + 2.0 * x - 3.0 * y + 0.5 * x * y)[None]
    pos = np.array([[[0.3, 0.1], [1.6, 0.7], [0.3 + 2.0, 0.1 - 1.0]]])
    got = tw.interpolate(prob, F, pos)
    for i, (px, py) in enumerate([(0.3, 0.1), (1.6, 0.7), (0.3, 0.1)]):
        assert abs(got[0, i] - (1.0 + 2.0 * px - 3.0 * py + 0.5 * px * py)) < 1e-14


def _cosine_background(n, box, axis, mode, eps, m_tot):
    """Real field psi' = sqrt((1 + eps cos k0 u) / volume), u the coordinate
    along `axis`, k0 = 2 pi mode / L_axis: density rho = rho_bar (1 + eps cos k0 u)."""
    grid = tw.Grid(n, box)
    coords = np.meshgrid(*[np.arange(m) * L / m for m, L in zip(reversed(n), reversed(box))], indexing="ij")
    u = coords[grid.dim - 1 - axis]
    k0 = 2 * np.pi * mode / box[axis]
    psi = np.sqrt((1 + eps * np.cos(k0 * u)) / grid.volume).astype(complex)
    return grid, psi, k0, m_tot / grid.volume


@pytest.mark.parametrize("axis", [0, 1])
def test_tracer_push_is_the_cosine_density_force(axis):
    """One step of a particle at rest in the field of rho = rho_bar (1 + eps cos k0 u):
    Poisson gives V = -4 pi G rho_bar eps cos(k0 u) / k0^2, so the kick is
    dv_u = -dt dV/du = -dt 4 pi G rho_bar eps sin(k0 u0) / k0 and the other
    component stays 0 (Sec. "Modeling decoherence": dv/dt = -grad V). The
    field's own motion over dt/2 and the fourth-order difference change this
    by O(dt^2) and O((k0 du)^4); a flipped sign, a wrong factor or a swapped
    axis miss it by far more than the tolerance."""
    n, box = (32, 48), (1.5, 2.0)
    G, m_tot, eps, dt = 3.0, 2.0, 0.3, 1e-4
    grid, psi, k0, rho_bar = _cosine_background(n, box, axis, 1, eps, m_tot)
    prob = tw.Problem(grid, hbar_m=0.5, G=G, m_tot=m_tot)
    du = box[axis] / n[axis]
    # on grid points (interpolation exact) and between them (linear weights)
    starts = [(5 * box[0] / n[0], 7 * box[1] / n[1]), (0.37 * box[0], 0.61 * box[1])]
    tr = np.zeros((1, len(starts), 4))
    tr[0, :, :2] = starts
    _, got = tw.step_tracers(prob, psi[None], tr, dt)
    amp = 4 * np.pi * G * rho_bar * eps / k0
    other = 1 - axis
    for i, (tol, p) in enumerate([(1e-4, starts[0]), (5e-3, starts[1])]):
        expect = -dt * amp * np.sin(k0 * p[axis])
        assert abs(got[0, i, 2 + axis] - expect) < tol * abs(expect), (i, got[0, i], expect)
        assert abs(got[0, i, 2 + other]) < 1e-12 * abs(expect)
        # positions: the second half drift moves by v dt / 2
        assert abs(got[0, i, axis] - (p[axis] + 0.5 * dt * got[0, i, 2 + axis])) < 1e-15
        assert got[0, i, other] == p[other]


def test_energy_of_a_plane_wave_is_kinetic_only():
    """psi' = exp(i k.x) / sqrt(volume): uniform density, so V = 0 whatever G,
    and E = M_tot hbar^2 |k|^2 / 2 exactly (Eq. (mft_normed) energy)."""
    n, box = (16, 24), (1.5, 2.0)
    grid = tw.Grid(n, box)
    prob = tw.Problem(grid, hbar_m=0.7, G=5.0, m_tot=3.0)
    y, x = np.meshgrid(np.arange(24) * 2.0 / 24, np.arange(16) * 1.5 / 16, indexing="ij")
    kx, ky = 2 * np.pi * 3 / 1.5, 2 * np.pi * (-2) / 2.0
    psi = np.exp(1j * (kx * x + ky * y)) / np.sqrt(grid.volume)
    expect = 3.0 * 0.7 ** 2 * (kx * kx + ky * ky) / 2
    assert abs(tw.energy(prob, psi[None])[0] - expect) < 1e-13 * expect


@pytest.mark.parametrize("dim", [1, 2])
def test_energy_of_a_cosine_density_closed_form(dim):
    """psi' = sqrt((1 + eps cos k0 u) / volume):
    int |grad psi'|^2 = k0^2 (1 - sqrt(1 - eps^2)) / 4 (from the integral of
    sin^2/(1 + eps cos) over a period), and (1/2) int V |psi'|^2 =
    -pi G rho_bar eps^2 / k0^2 with the closed-form potential, so
    E = M_tot [hbar^2 k0^2 (1 - sqrt(1 - eps^2)) / 8 - pi G rho_bar eps^2 / k0^2].
    A dropped or doubled M_tot, a missing cell volume or a wrong weight between
    the two terms all change E by far more than the tolerance."""
    n, box = ((64,), (2.0,)) if dim == 1 else ((16, 48), (1.5, 2.0))
    axis = dim - 1
    hbar, G, m_tot, eps = 0.8, 1.0, 3.0, 0.5
    grid, psi, k0, rho_bar = _cosine_background(n, box, axis, 1, eps, m_tot)
    prob = tw.Problem(grid, hbar_m=hbar, G=G, m_tot=m_tot)
    kin = hbar ** 2 * k0 ** 2 * (1 - np.sqrt(1 - eps ** 2)) / 8
    pot = -np.pi * G * rho_bar * eps ** 2 / k0 ** 2
    expect = m_tot * (kin + pot)
    assert abs(kin) > 0.1 * abs(pot) and abs(pot) > 0.1 * abs(kin)   # both terms matter
    got = tw.energy(prob, psi[None])[0]
    assert abs(got - expect) < 1e-12 * abs(m_tot * kin), (got, expect)


def test_tracer_spread_brute_force():
    """Plug-in variance over realizations, written out for three realizations
    and one particle (the extra classical slot beyond n_real is ignored)."""
    t = np.array([[[0.0, 1.0, 2.0, -1.0]], [[0.3, 1.0, 2.5, -1.0]], [[0.9, 0.7, 1.0, 0.5]],
                  [[50.0, 50.0, 50.0, 50.0]]])
    got = tw.tracer_spread(t, 3)
    for d in range(4):
        vals = [t[0, 0, d], t[1, 0, d], t[2, 0, d]]
        m = (vals[0] + vals[1] + vals[2]) / 3
        var = ((vals[0] - m) ** 2 + (vals[1] - m) ** 2 + (vals[2] - m) ** 2) / 3
        assert abs(got[0, d] - var) < 1e-15
