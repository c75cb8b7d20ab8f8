"""CPU FP64 oracle of the Fourier-neural-operator surrogate (forward, hand-written
backward, loss, Adam).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU leg
use it. The surrogate is not part of the paper; its architecture is the
published Fourier neural operator (Li et al., 2020): a pointwise lift, L
Fourier layers v <- act(W v + b + F^-1(R . F(v) restricted to low modes)), and
a two-layer pointwise projection.

Precision emulation: the GPU computes every dense contraction with BF16
operands and FP32 accumulation. With `bf16=True` this oracle rounds both
operands of the same contractions to BF16 (round to nearest even) and
accumulates in FP64; everything else (bias, GELU, mode mixing, loss) is FP64.
With `bf16=False` it is a plain FP64 implementation, used to pin the
hand-written backward against finite differences.

Layouts (row-major, channel last):
  activations  [B, H, W, C]
  spectral weights R_l: complex [2*my, mx, C, C] over modes ky in
  {0..my-1, H-my..H-1} (index order) and kx in {0..mx-1}.
"""
import numpy as np


class Config:
    def __init__(self, H=256, W=256, c_in=4, width=32, mx=16, my=16, layers=4, proj=128, c_out=2):
        self.H, self.W, self.c_in, self.width = H, W, c_in, width
        self.mx, self.my, self.layers, self.proj, self.c_out = mx, my, layers, proj, c_out
        if not (mx < W // 2 + 1 and 2 * my <= H):
            raise ValueError("too many modes for the grid")

    def shapes(self):
        """Parameter tensors in their flat-buffer order: (name, shape, is_complex_plane)."""
        C, out = self.width, []
        out.append(("lift_w", (self.c_in, C)))
        out.append(("lift_b", (C,)))
        for l in range(self.layers):
            out.append((f"R{l}_re", (2 * self.my, self.mx, C, C)))
            out.append((f"R{l}_im", (2 * self.my, self.mx, C, C)))
            out.append((f"W{l}", (C, C)))
            out.append((f"b{l}", (C,)))
        out.append(("q1_w", (C, self.proj)))
        out.append(("q1_b", (self.proj,)))
        out.append(("q2_w", (self.proj, self.c_out)))
        out.append(("q2_b", (self.c_out,)))
        return out

    def n_params(self):
        return int(sum(np.prod(s) for _, s in self.shapes()))

    def ky_list(self):
        return np.concatenate([np.arange(self.my), np.arange(self.H - self.my, self.H)])


def unflatten(cfg, flat):
    out, o = {}, 0
    for name, shp in cfg.shapes():
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def flatten(cfg, d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in cfg.shapes()])


# ------------------------------------------------------------------- rounding
def bf16(a):
    """Round to the nearest BF16 value (ties to even), via FP32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


class Ops:
    """Contractions with optional BF16 operand rounding."""

    def __init__(self, bf16_on=True):
        self.on = bf16_on

    def r(self, a):
        return bf16(a) if self.on else np.asarray(a, dtype=np.float64)

    def mm(self, a, b):
        """sum over the last axis of a and the first axis of b."""
        return np.tensordot(self.r(a), self.r(b), axes=([a.ndim - 1], [0]))


# ------------------------------------------------------------- DFT matrices
def dft_mats(cfg):
    """Real DFT matrices of the five spectral stages (FP64)."""
    H, W, mx = cfg.H, cfg.W, cfg.mx
    x = np.arange(W)
    kx = np.arange(mx)
    ang_x = 2 * np.pi * np.outer(x, kx) / W                # [W, mx]
    ky = cfg.ky_list()
    y = np.arange(H)
    ang_y = 2 * np.pi * np.outer(ky, y) / H                # [2my, H]
    wk = np.where(kx == 0, 1.0, 2.0) / (H * W)             # Hermitian completion and 1/(HW)
    return dict(
        # stage 1: A = sum_x v e^{-i kx x}:   A_re = v @ cos, A_im = v @ (-sin)
        f1_re=np.cos(ang_x), f1_im=-np.sin(ang_x),
        # stage 2: Bm = sum_y e^{-i ky y} A:  E2 = cos - i sin  [2my, H]
        e2_re=np.cos(ang_y), e2_im=-np.sin(ang_y),
        # stage 4: D = sum_ky e^{+i ky y} Cm: E4 [H, 2my]
        e4_re=np.cos(ang_y).T, e4_im=np.sin(ang_y).T,
        # stage 5: s = sum_kx wk Re(D e^{+i kx x}) = D_re @ (wk cos)^T - D_im @ (wk sin)^T   [mx, W]
        g5_re=(wk[:, None] * np.cos(ang_x).T), g5_im=-(wk[:, None] * np.sin(ang_x).T),
    )


# ------------------------------------------------------------------ pieces
SQRT2 = np.sqrt(2.0)


def gelu(z):
    from scipy.special import erf
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)


def spectral_forward(cfg, ops, M, v, Rre, Rim):
    """v [B,H,W,C] -> s [B,H,W,C]; returns s and the cache for the backward."""
    # stage 1 along x: [B,H,W,C] -> [B,H,mx,C]
    vt = np.moveaxis(v, 2, 3)                                   # [B,H,C,W]
    a_re = np.moveaxis(ops.mm(vt, M["f1_re"]), 3, 2)            # [B,H,mx,C]
    a_im = np.moveaxis(ops.mm(vt, M["f1_im"]), 3, 2)
    # stage 2 along y: [B,H,mx,C] -> [B,2my,mx,C]
    def ymix(e, a):                                             # e [K,H], a [B,H,mx,C] -> [B,K,mx,C]
        return np.moveaxis(ops.mm(e, np.moveaxis(a, 1, 0)), 0, 1)
    b_re = ymix(M["e2_re"], a_re) - ymix(M["e2_im"], a_im)
    b_im = ymix(M["e2_re"], a_im) + ymix(M["e2_im"], a_re)
    # stage 3 mode mixing (FP64, no rounding): C[b,k,x,o] = sum_c B[b,k,x,c] R[k,x,c,o]
    c_re = np.einsum("bkxc,kxco->bkxo", b_re, Rre) - np.einsum("bkxc,kxco->bkxo", b_im, Rim)
    c_im = np.einsum("bkxc,kxco->bkxo", b_re, Rim) + np.einsum("bkxc,kxco->bkxo", b_im, Rre)
    # stage 4 inverse along y: [B,2my,mx,C] -> [B,H,mx,C]
    d_re = ymix(M["e4_re"], c_re) - ymix(M["e4_im"], c_im)
    d_im = ymix(M["e4_re"], c_im) + ymix(M["e4_im"], c_re)
    # stage 5 inverse along x: [B,H,mx,C] -> [B,H,W,C]
    dt_re = np.moveaxis(d_re, 2, 3)                             # [B,H,C,mx]
    dt_im = np.moveaxis(d_im, 2, 3)
    s = np.moveaxis(ops.mm(dt_re, M["g5_re"]) + ops.mm(dt_im, M["g5_im"]), 3, 2)
    return s, (v, b_re, b_im, dt_re, dt_im)


def spectral_backward(cfg, ops, M, ds, cache, Rre, Rim):
    v, b_re, b_im, _, _ = cache
    # stage 5 adjoint: dD_re = ds @ g5_re^T (over x), dD_im = ds @ g5_im^T
    dst = np.moveaxis(ds, 2, 3)                                 # [B,H,C,W]
    dd_re = np.moveaxis(ops.mm(dst, M["g5_re"].T), 3, 2)        # [B,H,mx,C]
    dd_im = np.moveaxis(ops.mm(dst, M["g5_im"].T), 3, 2)
    # stage 4 adjoint: dC = sum_y conj(E4) dD  -> E4^H [2my,H]
    def ymix(e, a):
        return np.moveaxis(ops.mm(e, np.moveaxis(a, 1, 0)), 0, 1)
    e4h_re, e4h_im = M["e4_re"].T, -M["e4_im"].T
    dc_re = ymix(e4h_re, dd_re) - ymix(e4h_im, dd_im)
    dc_im = ymix(e4h_re, dd_im) + ymix(e4h_im, dd_re)
    # stage 3 adjoint (FP64)
    db_re = np.einsum("bkxo,kxco->bkxc", dc_re, Rre) + np.einsum("bkxo,kxco->bkxc", dc_im, Rim)
    db_im = np.einsum("bkxo,kxco->bkxc", dc_im, Rre) - np.einsum("bkxo,kxco->bkxc", dc_re, Rim)
    dR_re = np.einsum("bkxc,bkxo->kxco", b_re, dc_re) + np.einsum("bkxc,bkxo->kxco", b_im, dc_im)
    dR_im = np.einsum("bkxc,bkxo->kxco", b_re, dc_im) - np.einsum("bkxc,bkxo->kxco", b_im, dc_re)
    # stage 2 adjoint: dA = E2^H dB  [H, 2my]
    e2h_re, e2h_im = M["e2_re"].T, -M["e2_im"].T
    da_re = ymix(e2h_re, db_re) - ymix(e2h_im, db_im)
    da_im = ymix(e2h_re, db_im) + ymix(e2h_im, db_re)
    # stage 1 adjoint: dv = Re(dA conj(F1)) over kx = dA_re f1_re^T + dA_im f1_im^T
    dat_re = np.moveaxis(da_re, 2, 3)                           # [B,H,C,mx]
    dat_im = np.moveaxis(da_im, 2, 3)
    dv = np.moveaxis(ops.mm(dat_re, M["f1_re"].T) + ops.mm(dat_im, M["f1_im"].T), 3, 2)
    return dv, dR_re, dR_im


def forward(cfg, params, x, bf16_on=True, keep=False):
    """x [B,H,W,c_in] -> y [B,H,W,c_out] (and the activations if keep)."""
    ops = Ops(bf16_on)
    M = dft_mats(cfg)
    p = params if isinstance(params, dict) else unflatten(cfg, params)
    v = ops.mm(x, p["lift_w"]) + p["lift_b"]
    acts = dict(x=x, v=[v], u=[], sc=[])
    for l in range(cfg.layers):
        s, sc = spectral_forward(cfg, ops, M, v, p[f"R{l}_re"], p[f"R{l}_im"])
        u = s + ops.mm(v, p[f"W{l}"]) + p[f"b{l}"]
        acts["u"].append(u)
        acts["sc"].append(sc)
        v = gelu(u) if l < cfg.layers - 1 else u
        acts["v"].append(v)
    z1 = ops.mm(v, p["q1_w"]) + p["q1_b"]
    h = gelu(z1)
    y = ops.mm(h, p["q2_w"]) + p["q2_b"]
    acts.update(z1=z1, h=h)
    return (y, acts) if keep else y


def backward(cfg, params, x, dy, bf16_on=True):
    """Gradient of sum(dy * y) with respect to every parameter (dict of arrays)."""
    ops = Ops(bf16_on)
    M = dft_mats(cfg)
    p = params if isinstance(params, dict) else unflatten(cfg, params)
    y, A = forward(cfg, p, x, bf16_on, keep=True)
    g = {}
    red = tuple(range(dy.ndim - 1))

    def wgrad(a, d):          # sum over all positions of a^T d
        C1, C2 = a.shape[-1], d.shape[-1]
        return ops.mm(a.reshape(-1, C1).T, d.reshape(-1, C2))

    g["q2_w"] = wgrad(A["h"], dy)
    g["q2_b"] = dy.sum(axis=red)
    dh = ops.mm(dy, p["q2_w"].T)
    dz1 = dh * gelu_grad(A["z1"])
    g["q1_w"] = wgrad(A["v"][-1], dz1)
    g["q1_b"] = dz1.sum(axis=red)
    dv = ops.mm(dz1, p["q1_w"].T)
    for l in range(cfg.layers - 1, -1, -1):
        du = dv * gelu_grad(A["u"][l]) if l < cfg.layers - 1 else dv
        g[f"W{l}"] = wgrad(A["v"][l], du)
        g[f"b{l}"] = du.sum(axis=red)
        dvs, g[f"R{l}_re"], g[f"R{l}_im"] = spectral_backward(cfg, ops, M, du, A["sc"][l],
                                                              p[f"R{l}_re"], p[f"R{l}_im"])
        dv = ops.mm(du, p[f"W{l}"].T) + dvs
    g["lift_w"] = wgrad(x, dv)
    g["lift_b"] = dv.sum(axis=red)
    return g


def mse(y, t):
    """Loss (1/count) sum (y - t)^2 and its gradient with respect to y."""
    d = y - t
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


def adam(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015), bias-corrected, in place; returns theta."""
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta -= lr * mh / (np.sqrt(vh) + eps)
    return theta


def init_params(cfg, seed):
    """Reference initialisation scheme (the GPU library has its own generator):
    uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases, spectral
    weights uniform(0, 1)/(C*C)."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in cfg.shapes():
        if name.endswith("_b") or (name.startswith("b") and name[1:].isdigit()):
            d[name] = np.zeros(shp)
        elif name.startswith("R"):
            d[name] = rng.uniform(0, 1, shp) / (cfg.width * cfg.width)
        else:
            d[name] = rng.uniform(-1, 1, shp) / np.sqrt(shp[0])
    return d
