"""Seeded synthetic initial fields for the workloads (host side, numpy FP64).

This module builds input data only. It holds none of the method's arithmetic
(no sampling noise, no evolution, no moments); both the GPU path and the CPU
oracle are fed from it. Every field is returned as a complex128 array in
numpy order (x fastest, shape (n2, n1, n0) / (n1, n0) / (n0,)) normalised to
sum_g |psi|^2 dV = 1, the normalisation of the paper's psi'.
"""
import numpy as np


def _grid_coords(n, box):
    """Cell-corner coordinates x_g = g dx per axis, broadcast in numpy order."""
    dim = len(n)
    out = []
    for d in range(dim):
        x = np.arange(n[d]) * (box[d] / n[d])
        shape = [1] * dim
        shape[dim - 1 - d] = n[d]
        out.append(x.reshape(shape))
    return out


def normalise(psi, n, box):
    dv = float(np.prod([box[d] / n[d] for d in range(len(n))]))
    return psi / np.sqrt((np.abs(psi) ** 2).sum() * dv)


def lognormal_field(n, box, kcut=None, amp=0.5, seed=0):
    """sqrt of a positive Gaussian-random density with spectrum P(k) ~ k^-2.

    delta_j = (a + i b)/|j| for 1 <= |j| <= kcut (integer wavevector j,
    a, b ~ N(0,1) from numpy default_rng(seed)), delta = Re IDFT, scaled to unit
    rms; rho ~ exp(amp*delta - amp^2/2); psi = sqrt(rho), normalised.
    """
    n = tuple(int(v) for v in n)
    dim = len(n)
    shape = tuple(reversed(n))
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    jj = np.zeros(shape)
    for d in range(dim):
        j = np.fft.fftfreq(n[d], d=1.0 / n[d])
        bs = [1] * dim
        bs[dim - 1 - d] = n[d]
        jj = jj + (j ** 2).reshape(bs)
    jabs = np.sqrt(jj)
    if kcut is None:
        kcut = min(n) // 2
    keep = (jabs >= 1) & (jabs <= kcut)
    dk = np.where(keep, (a + 1j * b) / np.where(jabs == 0, 1.0, jabs), 0.0)
    delta = np.fft.ifftn(dk).real
    delta = delta / np.sqrt((delta ** 2).mean())
    rho = np.exp(amp * delta - 0.5 * amp * amp)
    return normalise(np.sqrt(rho).astype(np.complex128), n, box)


def _min_image(x, c, L):
    d = x - c
    return d - L * np.round(d / L)


def gaussian_pair_2d(n=(512, 512), box=(1.0, 1.0), width=0.05, sep=0.3, vel=5.0,
                     hbar_m=1.0, phase=0.0):
    """Two Gaussian-profile cores moving towards each other along x.

    Density std `width`*L, centres (0.5 -+ sep/2, 0.5) L, phase gradient
    +-vel/hbar_m along x (velocity in hbar/m units), relative phase `phase`.
    """
    X, Y = _grid_coords(n, box)
    out = np.zeros(tuple(reversed(n)), dtype=np.complex128)
    w = width * box[0]
    for sgn, ph in ((+1.0, 0.0), (-1.0, phase)):
        cx = (0.5 - sgn * sep / 2.0) * box[0]
        cy = 0.5 * box[1]
        dx = _min_image(X, cx, box[0])
        dy = _min_image(Y, cy, box[1])
        env = np.exp(-(dx ** 2 + dy ** 2) / (4.0 * w * w))
        out = out + env * np.exp(1j * (sgn * vel * dx / hbar_m + ph))
    return normalise(out, n, box)


def random_gaussian_pair_2d(n, box, rng, hbar_m=1.0):
    """Random soliton pair for surrogate training: widths in [0.03, 0.07] L,
    separation in [0.15, 0.4] L along a random direction, speeds in [0, 5]
    towards each other, random relative phase. `rng` is a numpy Generator."""
    X, Y = _grid_coords(n, box)
    out = np.zeros(tuple(reversed(n)), dtype=np.complex128)
    ang = rng.uniform(0, 2 * np.pi)
    ex, ey = np.cos(ang), np.sin(ang)
    sep = rng.uniform(0.15, 0.4)
    cx0, cy0 = rng.uniform(0.3, 0.7, size=2)
    for sgn in (+1.0, -1.0):
        w = rng.uniform(0.03, 0.07) * box[0]
        v = rng.uniform(0.0, 5.0)
        ph = rng.uniform(0, 2 * np.pi) if sgn < 0 else 0.0
        amp = rng.uniform(0.5, 1.5)
        cx = (cx0 + sgn * 0.5 * sep * ex) * box[0]
        cy = (cy0 + sgn * 0.5 * sep * ey) * box[1]
        dx = _min_image(X, cx, box[0])
        dy = _min_image(Y, cy, box[1])
        env = amp * np.exp(-(dx ** 2 + dy ** 2) / (4.0 * w * w))
        out = out + env * np.exp(1j * (-sgn * v * (ex * dx + ey * dy) / hbar_m + ph))
    return normalise(out, n, box)


def soliton_3d(n=(64, 64, 64), box=(1.0, 1.0, 1.0), core=0.1):
    """Ground-state-like core profile rho ~ [1 + 0.091 (r/r_c)^2]^-8, r_c = core*L."""
    X, Y, Z = _grid_coords(n, box)
    r2 = (_min_image(X, 0.5 * box[0], box[0]) ** 2 + _min_image(Y, 0.5 * box[1], box[1]) ** 2
          + _min_image(Z, 0.5 * box[2], box[2]) ** 2)
    rc = core * box[0]
    rho = (1.0 + 0.091 * r2 / (rc * rc)) ** -8
    return normalise(np.sqrt(rho).astype(np.complex128), n, box)


def random_field(n, seed=0):
    """Generic smooth-plus-rough complex test field (for parity on small grids)."""
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(tuple(int(v) for v in n)))
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape) + 2.0
    return psi


def sinusoid(n, box, delta=0.1):
    """The sinusoidal overdensity test problem (Sec. "Sinusoidal overdensity"):
    psi_cl = sqrt(1 + delta cos(2 pi x / L_x)), normalised; constant along
    the other axes."""
    x = _grid_coords(n, box)[0]
    shape = tuple(reversed(tuple(int(v) for v in n)))
    psi = np.broadcast_to(np.sqrt(1.0 + delta * np.cos(2.0 * np.pi * x / box[0])), shape).astype(np.complex128)
    return normalise(psi, n, box)


def kspace_gaussian(n, box, kd, seed=0):
    """The momentum-space Gaussian test problem (Sec. "Momentum space
    gaussian", Eq. (kspaceGauss)): Fourier amplitudes exp(-|k|^2 / (2 kd^2))
    with independent uniform phases on every mode, transformed to position
    space and normalised. The printed phase distribution U[0, 1] is read as a
    full turn, U[0, 2 pi)."""
    dim = len(n)
    shape = tuple(reversed(tuple(int(v) for v in n)))
    k2 = np.zeros(shape)
    for d in range(dim):
        k = 2.0 * np.pi * np.fft.fftfreq(n[d], d=box[d] / n[d])
        sh = [1] * dim
        sh[dim - 1 - d] = n[d]
        k2 = k2 + (k ** 2).reshape(sh)
    rng = np.random.default_rng(seed)
    phase = rng.uniform(0.0, 2.0 * np.pi, shape)
    psi = np.fft.ifftn(np.exp(-k2 / (2.0 * kd ** 2) + 1j * phase))
    return normalise(psi, n, box)


# Gravitational constant in kpc^3 / (M_sun Myr^2) (GM_sun = 1.32712440018e20
# m^3/s^2, 1 kpc = 3.0856775814913673e19 m, 1 Myr = 3.15576e13 s).
G_KPC_MYR_MSUN = 4.4985021520796915e-12

# Named workloads --------------------------------------------------------------
WORKLOADS = {
    "1d_n256": dict(n=(256,), box=(1.0,), n_real=64, n_tot=1e4, dt=1e-4, nsteps=1000,
                    hbar_m=1.0, G=1.0, m_tot=1.0),
    "2d_n512_pair": dict(n=(512, 512), box=(1.0, 1.0), n_real=256, n_tot=1e6, dt=1e-4,
                         nsteps=5000, hbar_m=1.0, G=1.0, m_tot=1.0),
    "3d_n128_grf": dict(n=(128, 128, 128), box=(1.0, 1.0, 1.0), n_real=64,
                        n_tot=1e3 * 128 ** 3, dt=1e-4, nsteps=2000, hbar_m=1.0, G=1.0, m_tot=1.0),
    # three size classes advanced together (FP32 split): 64 realizations each
    "3d_batched_soliton": dict(classes=((64, 64, 64), (96, 96, 96), (128, 128, 128)), box=(1.0, 1.0, 1.0),
                               n_real=64, occupation=1e3, dt=1e-4, nsteps=1000, hbar_m=1.0, G=1.0, m_tot=1.0),
    # the paper's own test problems in its physical units (kpc, Myr, M_sun), run
    # with device-chosen steps (dt is the upper bound dt_max)
    "1d_sinusoid": dict(n=(512,), box=(60.0,), n_real=64, n_tot=1e6, dt=10.0, nsteps=1000, hbar_m=0.01,
                        G=G_KPC_MYR_MSUN, m_tot=1e8, delta=0.1),
    "2d_n512_kgauss": dict(n=(512, 512), box=(60.0, 60.0), n_real=64, n_tot=1e3 * 512 ** 2, dt=10.0, nsteps=1000,
                           hbar_m=0.02, G=G_KPC_MYR_MSUN, m_tot=6e9, kd=0.158113883008419),
    "3d_n512_kgauss": dict(n=(512, 512, 512), box=(60.0, 60.0, 60.0), n_real=32, n_tot=1e3 * 512 ** 3, dt=10.0,
                           nsteps=1000, hbar_m=0.02, G=G_KPC_MYR_MSUN, m_tot=1e10, kd=0.158113883008419),
}


def initial_field(name, n=None):
    """The coherent (classical) field of a named workload, optionally regenerated at grid n."""
    w = WORKLOADS[name]
    n = tuple(n) if n is not None else w["n"]
    box = w["box"][: len(n)]
    if name == "1d_n256":
        return lognormal_field(n, box, seed=0)
    if name == "2d_n512_pair":
        return gaussian_pair_2d(n, box, hbar_m=w["hbar_m"])
    if name == "3d_n128_grf":
        return lognormal_field(n, box, kcut=min(32, min(n) // 2), seed=0)
    if name == "3d_batched_soliton":
        return soliton_3d(n, box, core=0.1)
    if name == "1d_sinusoid":
        return sinusoid(n, box, w["delta"])
    if name in ("2d_n512_kgauss", "3d_n512_kgauss"):
        return kspace_gaussian(n, box, w["kd"], seed=1)
    raise KeyError(name)
