"""Helpers for GPU parity tests: run the HIP path through the C ABI binding and
the oracle on the same seeded inputs, compare normwise."""
import numpy as np
import torch

from oracle import twa_oracle as tw
from paper_2310_07119_amd import Plan, Problem

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def oracle_problem(p: Problem):
    grid = tw.Grid(p.n, p.box)
    return tw.Problem(grid, p.hbar_m, p.G, p.m_tot)


def gpu_run(p: Problem, psi_cl_np, seed, nsteps, dt, real_offset=0, with_classical=True, energy=True, modes=False,
            decoherence=False):
    """Sample, step and take moments on the GPU; returns host numpy results."""
    dev = torch.device("cuda:0")
    plan = Plan(p)
    cl = torch.from_numpy(np.ascontiguousarray(psi_cl_np)).to(dev)
    psi = plan.sample(cl, seed, real_offset)
    psi0 = psi.cpu().numpy()
    clt = cl.to(p.cdtype).clone() if with_classical else None
    plan.step(psi, nsteps, dt, clt)
    mom = plan.moments(psi, clt, energy=energy, modes=modes, decoherence=decoherence)
    torch.cuda.synchronize()
    out = dict(psi0=psi0, psi=psi.cpu().numpy(), cl=None if clt is None else clt.cpu().numpy())
    out["mom"] = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in mom.items()}
    plan.close()
    return out
