"""Learned surrogate for the ensemble moments (the GPU FNO of tw_fno_*).

Task: from the coherent field psi_cl(0) of a random soliton pair (2D) and its
classical evolution psi_cl(T), predict the truncated-Wigner moments <rho>(T)
and Var rho(T) that an ensemble of n_real realizations gives at T = steps*dt.
Training data are produced by the method itself (tw_sample / tw_step /
tw_moments); the network is trained by the library's own forward, backward and
Adam kernels. The plain ensemble is the fallback and the judge of its error.

Channels (all scaled by the box-mean density rho_bar = m_tot / volume):
  inputs   rho_cl(T), rho_cl(0), Re psi_cl(0) / sqrt(rho_bar / m_tot), Im ...
  targets  <rho>(T) / rho_bar - 1 - (rho_cl(T) / rho_bar - 1)   (quantum correction)
           Var rho(T) / rho_bar^2 * var_scale
"""
import time

import numpy as np
import torch

from . import inputs
from .twa import Fno, Plan, Problem


def _fields(plan, cl, n_real, steps, dt, seed):
    """Run the method on one coherent field: returns (rho_cl(T), mean_rho, var_rho) on the device."""
    psi = plan.sample(cl, seed)
    clt = cl.to(plan.problem.cdtype).clone()
    plan.step(psi, steps, dt, clt)
    m = plan.moments(psi, clt, energy=False)
    rho_cl_t = plan.problem.m_tot * (clt.real.double() ** 2 + clt.imag.double() ** 2)
    return rho_cl_t, m["mean_rho"], m["var_rho"]


class DatasetSpec:
    def __init__(self, n=(256, 256), n_real=128, steps=100, dt=1e-4, n_tot=1e6, hbar_m=1.0, G=1.0, m_tot=1.0,
                 precision="fp32", var_scale=None):
        self.n, self.n_real, self.steps, self.dt = tuple(n), n_real, steps, dt
        self.n_tot, self.hbar_m, self.G, self.m_tot, self.precision = n_tot, hbar_m, G, m_tot, precision
        self.box = (1.0,) * len(self.n)
        cells = int(np.prod(self.n))
        self.rho_bar = m_tot / float(np.prod(self.box))
        # vacuum-noise density variance of a uniform field sets the target scale
        sigma2 = cells / (2.0 * n_tot)          # <|d psi'|^2> * volume
        self.var_scale = var_scale if var_scale is not None else 1.0 / (2.0 * sigma2 + sigma2 ** 2)

    def problem(self, n_real):
        return Problem(n=self.n, box=self.box, hbar_m=self.hbar_m, G=self.G, m_tot=self.m_tot, n_tot=self.n_tot,
                       n_real=n_real, precision=self.precision)


def make_dataset(spec, count, seed, n_real=None, device="cuda", noise_offset=0, log=None):
    """count samples: x [count,H,W,4], t [count,H,W,2] (FP32, device). The
    coherent fields depend on `seed` only; `noise_offset` shifts the sampling
    seeds so two datasets of the same fields have independent noise."""
    n_real = spec.n_real if n_real is None else n_real
    plan = Plan(spec.problem(n_real))
    plan.autotune()
    rng = np.random.default_rng(seed)
    H, W = spec.n[1], spec.n[0]
    x = torch.empty((count, H, W, 4), dtype=torch.float32, device=device)
    t = torch.empty((count, H, W, 2), dtype=torch.float32, device=device)
    amp = np.sqrt(spec.rho_bar / spec.m_tot)
    for i in range(count):
        psi0 = inputs.random_gaussian_pair_2d(spec.n, spec.box, rng, spec.hbar_m)
        cl = torch.from_numpy(psi0).to(device)
        rho_cl_t, mean_rho, var_rho = _fields(plan, cl, n_real, spec.steps, spec.dt,
                                              seed=int(rng.integers(2**62)) + noise_offset)
        rho0 = spec.m_tot * (cl.real ** 2 + cl.imag ** 2)
        x[i, ..., 0] = (rho_cl_t / spec.rho_bar - 1.0).float()
        x[i, ..., 1] = (rho0 / spec.rho_bar - 1.0).float()
        x[i, ..., 2] = (cl.real / amp).float()
        x[i, ..., 3] = (cl.imag / amp).float()
        t[i, ..., 0] = ((mean_rho - rho_cl_t) / spec.rho_bar).float()
        t[i, ..., 1] = (var_rho / spec.rho_bar ** 2 * spec.var_scale).float()
        if log and (i + 1) % 200 == 0:
            log(f"generated {i + 1}/{count} ensembles")
    plan.close()
    return x.contiguous(), t.contiguous()


def relative_errors(pred, ref):
    """Normwise relative L2 error per target channel (mean density, variance),
    with the mean density measured as the full <rho> (classical part added back)."""
    out = []
    for c in range(ref.shape[-1]):
        d = (pred[..., c] - ref[..., c]).double()
        out.append(float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref[..., c].double())))
    return out


def density_error(pred, ref, x):
    """Relative L2 error of <rho>/rho_bar = 1 + rho_cl(T)/rho_bar - 1 + correction."""
    full_p = 1.0 + x[..., 0].double() + pred[..., 0].double()
    full_r = 1.0 + x[..., 0].double() + ref[..., 0].double()
    return float(torch.linalg.vector_norm(full_p - full_r) / torch.linalg.vector_norm(full_r))


def train(net, x, t, epochs, batch, lr=1e-3, seed=0, log=None):
    n = x.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g)
        tot = 0.0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch].to(x.device)
            xb, tb = x[idx].contiguous(), t[idx].contiguous()
            tot += float(net.train_step(xb, tb, lr=lr).item())
        hist.append(tot / max(1, n // batch))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def predict(net, x, batch):
    out = torch.empty(x.shape[:3] + (2,), dtype=torch.float32, device=x.device)
    for i in range(0, x.shape[0], batch):
        out[i:i + batch] = net.forward(x[i:i + batch].contiguous())
    return out


def gain_study(spec, n_train, n_test, epochs, batch, ref_real, net_kw=None, seed=0, log=None):
    """Train on `n_train` ensembles, evaluate on `n_test` held-out coherent fields
    against a reference ensemble of `ref_real` realizations. Reports the
    surrogate, the classical field (no correction, no variance) and the plain
    method with the training ensemble size."""
    t0 = time.perf_counter()
    xtr, ttr = make_dataset(spec, n_train, seed, log=log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    xte, tte_ref = make_dataset(spec, n_test, seed + 1, n_real=ref_real)
    t0 = time.perf_counter()
    _, tte_small = make_dataset(spec, n_test, seed + 1, n_real=spec.n_real, noise_offset=7919)  # same fields
    torch.cuda.synchronize()
    t_twa = (time.perf_counter() - t0) / n_test
    kw = dict(H=spec.n[1], W=spec.n[0], c_in=4, width=32, modes_x=16, modes_y=16, layers=4, proj=128, c_out=2)
    kw.update(net_kw or {})
    net = Fno(**kw, max_batch=batch, seed=seed)
    t0 = time.perf_counter()
    hist = train(net, xtr, ttr, epochs, batch, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    pred = predict(net, xte, batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        predict(net, xte, batch)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / (3 * n_test)
    zero = torch.zeros_like(tte_ref)
    res = {
        "surrogate": {"rho_err": density_error(pred, tte_ref, xte), "var_err": relative_errors(pred, tte_ref)[1]},
        "classical": {"rho_err": density_error(zero, tte_ref, xte), "var_err": 1.0},
        f"twa_{spec.n_real}": {"rho_err": density_error(tte_small, tte_ref, xte),
                               "var_err": relative_errors(tte_small, tte_ref)[1]},
        "loss_first": hist[0], "loss_last": hist[-1], "epochs": epochs,
        "n_train": n_train, "n_test": n_test, "ref_real": ref_real,
        "data_seconds": t_data, "train_seconds": t_train, "inference_seconds_per_field": t_inf,
        f"twa_{spec.n_real}_seconds_per_field": t_twa,
    }
    net.close()
    return res


def main(argv=None):
    """Surrogate study on the 2D soliton-pair workload:
    --full : 256^2 fields, 2000 training ensembles of 128 realizations, 100 steps
             ahead, 4-layer FNO (16 modes, width 32), held-out fields judged
             against 1024-realization ensembles.
    default: a reduced study (fewer ensembles and epochs) for quick checks."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--full", action="store_true")
    ap.add_argument("--train", type=int, default=None)
    ap.add_argument("--epochs", type=int, default=None)
    a = ap.parse_args(argv)
    spec = DatasetSpec(n=(256, 256), n_real=128, steps=100, dt=1e-4, n_tot=1e6, G=1.0, m_tot=1.0)
    n_train = a.train or (2000 if a.full else 200)
    epochs = a.epochs or (20 if a.full else 6)
    res = gain_study(spec, n_train=n_train, n_test=16 if a.full else 8, epochs=epochs, batch=8,
                     ref_real=1024, seed=2023, log=lambda s: print(s, file=sys.stderr, flush=True))
    res["workload"] = "2d_n256_soliton_pairs"
    res["spec"] = dict(grid=list(spec.n), n_real=spec.n_real, steps=spec.steps, dt=spec.dt, n_tot=spec.n_tot)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
