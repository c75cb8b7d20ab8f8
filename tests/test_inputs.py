"""The paper's own test-problem generators (Sec. "Sinusoidal overdensity",
Sec. "Momentum space gaussian"), checked against their defining formulas."""
import numpy as np

from paper_2310_07119_amd import inputs


def test_sinusoid_profile_and_norm():
    n, box = (64, 8), (60.0, 7.5)
    psi = inputs.sinusoid(n, box, delta=0.3)
    dv = (60.0 / 64) * (7.5 / 8)
    assert abs((np.abs(psi) ** 2).sum() * dv - 1.0) < 1e-13
    rho = np.abs(psi[0]) ** 2
    x = np.arange(64) * 60.0 / 64
    ratio = rho / rho[0]
    assert np.allclose(ratio, (1 + 0.3 * np.cos(2 * np.pi * x / 60.0)) / 1.3, rtol=1e-13, atol=0)
    assert np.all(psi == psi[0][None])                    # constant along y
    assert np.all(psi.imag == 0)


def test_kspace_gaussian_spectrum_and_phases():
    n, box, kd = (32, 16), (60.0, 30.0), 0.3
    psi = inputs.kspace_gaussian(n, box, kd, seed=4)
    dv = (60.0 / 32) * (30.0 / 16)
    assert abs((np.abs(psi) ** 2).sum() * dv - 1.0) < 1e-13
    f = np.fft.fftn(psi)
    kx = 2 * np.pi * np.fft.fftfreq(32, d=60.0 / 32)
    ky = 2 * np.pi * np.fft.fftfreq(16, d=30.0 / 16)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    amp = np.abs(f) / np.abs(f[0, 0])
    assert np.allclose(amp, np.exp(-k2 / (2 * kd ** 2)), rtol=1e-10, atol=1e-14)
    ph = np.angle(f[np.exp(-k2 / (2 * kd ** 2)) > 1e-3])
    assert ph.std() > 1.0                                  # phases spread over the circle
    other = inputs.kspace_gaussian(n, box, kd, seed=5)
    assert not np.allclose(psi, other)
