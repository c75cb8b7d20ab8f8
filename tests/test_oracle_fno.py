"""Pins for the FNO surrogate oracle.

The spectral layer with an identity mode-mixer must equal a low-pass filter
computed with numpy's real FFT (an independent route to the same DFTs); the
hand-written backward must match central finite differences; BF16 rounding
must be round-to-nearest-even; Adam must match its closed form on a quadratic.
"""
import numpy as np

from oracle import fno_oracle as fo


def tiny():
    return fo.Config(H=8, W=8, c_in=3, width=4, mx=2, my=2, layers=2, proj=6, c_out=2)


def test_bf16_rounding_rne():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, -2.5, 3.0e38, 1e-40])
    r = fo.bf16(vals)
    # BF16 keeps 7 fraction bits: one unit in the last place at 1.0 is 2^-7
    assert r[0] == 1.0
    assert r[1] == 1.0                    # exactly half a unit: tie goes to the even neighbour
    assert r[2] == 1.0 + 2 ** -7          # three quarters of a unit rounds up
    assert r[3] == 1.0                    # a quarter of a unit rounds down
    assert r[4] == -2.5
    # every result is exactly representable with 8 significant bits
    f = r.astype(np.float32).view(np.uint32)
    assert np.all((f & 0xFFFF) == 0)
    assert fo.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6   # tie between odd and even: even


def test_spectral_identity_mixer_is_fft_lowpass():
    cfg = fo.Config(H=16, W=12, c_in=1, width=3, mx=4, my=3, layers=1, proj=2, c_out=1)
    rng = np.random.default_rng(0)
    v = rng.standard_normal((2, cfg.H, cfg.W, cfg.width))
    eye = np.zeros((2 * cfg.my, cfg.mx, cfg.width, cfg.width))
    for c in range(cfg.width):
        eye[:, :, c, c] = 1.0
    s, _ = fo.spectral_forward(cfg, fo.Ops(False), fo.dft_mats(cfg), v, eye, np.zeros_like(eye))
    F = np.fft.rfft2(v, axes=(1, 2))                 # [B,H,W//2+1,C]
    keep = np.zeros(F.shape[1:3], bool)
    keep[np.ix_(cfg.ky_list(), np.arange(cfg.mx))] = True
    ref = np.fft.irfft2(np.where(keep[None, :, :, None], F, 0), s=(cfg.H, cfg.W), axes=(1, 2))
    assert np.max(np.abs(s - ref)) < 1e-12


def test_backward_matches_finite_differences():
    cfg = tiny()
    rng = np.random.default_rng(1)
    p = fo.init_params(cfg, 3)
    for k in p:                                     # non-zero biases for a generic point
        p[k] = p[k] + 0.05 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((2, cfg.H, cfg.W, cfg.c_in))
    dy = rng.standard_normal((2, cfg.H, cfg.W, cfg.c_out))
    g = fo.flatten(cfg, fo.backward(cfg, p, x, dy, bf16_on=False))
    flat = fo.flatten(cfg, p)
    h = 1e-6
    idx = rng.choice(flat.size, 120, replace=False)
    num = []
    for i in idx:
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        lp = (dy * fo.forward(cfg, fp, x, bf16_on=False)).sum()
        lm = (dy * fo.forward(cfg, fm, x, bf16_on=False)).sum()
        num.append((lp - lm) / (2 * h))
    num = np.array(num)
    assert np.linalg.norm(g[idx] - num) / np.linalg.norm(num) < 1e-6


def test_bf16_forward_close_to_fp64():
    cfg = tiny()
    p = fo.init_params(cfg, 4)
    x = np.random.default_rng(2).standard_normal((1, cfg.H, cfg.W, cfg.c_in))
    a = fo.forward(cfg, p, x, bf16_on=True)
    b = fo.forward(cfg, p, x, bf16_on=False)
    e = np.linalg.norm(a - b) / np.linalg.norm(b)
    assert 1e-5 < e < 3e-2           # BF16 operands: visible but small differences


def test_adam_closed_form_quadratic():
    theta = np.array([3.0, -2.0])
    m, v = np.zeros(2), np.zeros(2)
    for t in range(1, 2001):
        fo.adam(theta, 2 * theta, m, v, t, lr=1e-2)
    assert np.max(np.abs(theta)) < 1e-2
    # first step moves every coordinate by lr (bias-corrected m/sqrt(v) = sign(g))
    th = np.array([5.0, -7.0]); m1, v1 = np.zeros(2), np.zeros(2)
    fo.adam(th, np.array([0.3, -4.0]), m1, v1, 1, lr=0.1)
    assert np.allclose(th, [4.9, -6.9], atol=1e-7)


def test_mse_gradient():
    rng = np.random.default_rng(3)
    y, t = rng.standard_normal((2, 3)), rng.standard_normal((2, 3))
    loss, g = fo.mse(y, t)
    assert abs(loss - ((y - t) ** 2).mean()) < 1e-15
    h = 1e-7
    y2 = y.copy(); y2[1, 2] += h
    assert abs((fo.mse(y2, t)[0] - loss) / h - g[1, 2]) < 1e-6
