"""ctypes binding of the C ABI in include/tw.h (argument marshalling only).

Every computation happens in the HIP library ``libtw.so``; this module only
converts torch device tensors to pointers, passes the current HIP stream and
raises on a non-zero status. There is no CPU fallback: importing works without
the library, but creating a Plan raises if it is missing.
"""
import ctypes
import math
import os
from dataclasses import dataclass, field

import torch

_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtw.so")

TW_FP64 = 0
TW_FP32_SPLIT = 1
STATUS = {0: "TW_OK", -1: "TW_EINVAL", -2: "TW_EUNSUPPORTED", -3: "TW_ELAYOUT", -4: "TW_EHIP", -5: "TW_ENOMEM"}
SCALAR_NAMES = ("Q_raw", "Q_sym", "dev_rho_L1", "dev_psi_L2", "energy_mean", "norm_mean",
                "nonfinite", "energy_classical")

# Exported entry points and their argument types (mirrors include/tw.h).
EXPORTS = ("tw_plan_create", "tw_plan_destroy", "tw_sample", "tw_step", "tw_step_adaptive", "tw_step_tracers",
           "tw_tracer_spread", "tw_moments", "tw_moments_static",
           "tw_plan_autotune", "tw_batch_create", "tw_batch_plan", "tw_batch_autotune", "tw_batch_step",
           "tw_batch_destroy", "tw_fno_param_count", "tw_fno_create", "tw_fno_destroy", "tw_fno_init_params",
           "tw_fno_forward", "tw_fno_backward", "tw_fno_mse", "tw_fno_adam", "tw_fno_last_error",
           "tw_plan_set_profiling", "tw_plan_get_profile", "tw_kernel_kind_name", "tw_last_error")
NUM_KERNEL_KINDS = 20


class TwProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("box", ctypes.c_double * 3),
                ("hbar_m", ctypes.c_double), ("G", ctypes.c_double), ("m_tot", ctypes.c_double),
                ("n_tot", ctypes.c_double), ("n_real", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class TwMomentsOut(ctypes.Structure):
    _fields_ = [("mean_psi", ctypes.c_void_p), ("mean_abs2", ctypes.c_void_p), ("mean_rho", ctypes.c_void_p),
                ("var_rho", ctypes.c_void_p), ("mode_occ", ctypes.c_void_p), ("var_amp", ctypes.c_void_p),
                ("var_phase", ctypes.c_void_p), ("decoherence", ctypes.c_void_p), ("norm", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("scalars", ctypes.c_void_p)]


class TwFnoConfig(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("H", "W", "c_in", "width", "modes_x", "modes_y", "layers", "proj",
                                                "c_out")]


class TwError(RuntimeError):
    pass


def load_library(path=LIB_PATH):
    """Load libtw.so (built by paper_2310_07119_amd.build). Raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise TwError(f"HIP library not built: {path} is missing (run `python -m paper_2310_07119_amd.build`)")
    lib = ctypes.CDLL(path)
    vp, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.tw_plan_create.argtypes = [ctypes.POINTER(TwProblem), ctypes.POINTER(vp)]
    lib.tw_plan_destroy.argtypes = [vp]
    lib.tw_sample.argtypes = [vp, vp, u64, i64, vp, vp]
    lib.tw_step.argtypes = [vp, vp, vp, i64, dbl, vp]
    lib.tw_step_adaptive.argtypes = [vp, vp, vp, i64, dbl, dbl, vp, vp]
    lib.tw_step_tracers.argtypes = [vp, vp, vp, i64, dbl, vp, i64, vp]
    lib.tw_tracer_spread.argtypes = [vp, vp, i64, vp, vp]
    lib.tw_moments.argtypes = [vp, vp, vp, ctypes.POINTER(TwMomentsOut), vp]
    lib.tw_moments_static.argtypes = [ctypes.POINTER(TwProblem), vp, vp, ctypes.POINTER(TwMomentsOut), vp]
    lib.tw_plan_autotune.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), vp]
    lib.tw_batch_create.argtypes = [ctypes.POINTER(TwProblem), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.tw_batch_plan.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.tw_batch_autotune.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), vp]
    lib.tw_batch_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i64, dbl, vp]
    lib.tw_batch_destroy.argtypes = [vp]
    pf = ctypes.POINTER(ctypes.c_float)
    lib.tw_fno_param_count.argtypes = [ctypes.POINTER(TwFnoConfig)]
    lib.tw_fno_param_count.restype = ctypes.c_int64
    lib.tw_fno_create.argtypes = [ctypes.POINTER(TwFnoConfig), ctypes.c_int32, ctypes.POINTER(vp)]
    lib.tw_fno_destroy.argtypes = [vp]
    lib.tw_fno_init_params.argtypes = [vp, u64, vp, vp]
    lib.tw_fno_forward.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp]
    lib.tw_fno_backward.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    lib.tw_fno_mse.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.tw_fno_adam.argtypes = [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i64, vp]
    lib.tw_fno_last_error.restype = ctypes.c_char_p
    lib.tw_plan_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.tw_plan_get_profile.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.tw_kernel_kind_name.argtypes = [ctypes.c_int32]
    lib.tw_kernel_kind_name.restype = ctypes.c_char_p
    lib.tw_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("tw_last_error", "tw_kernel_kind_name", "tw_fno_last_error", "tw_fno_param_count"):
            getattr(lib, name).restype = ctypes.c_int
    _LIB = lib
    return lib


def _check(rc, what):
    if rc != 0:
        msg = _LIB.tw_last_error().decode()
        raise TwError(f"{what} failed: {STATUS.get(rc, rc)}: {msg}")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


@dataclass
class Problem:
    """Problem statement of Eq. (mft_normed) on a periodic grid (x first)."""
    n: tuple
    box: tuple = None
    hbar_m: float = 1.0
    G: float = 1.0
    m_tot: float = 1.0
    n_tot: float = 1e4
    n_real: int = 64
    precision: str = "fp64"      # "fp64" or "fp32"
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        if self.box is None:
            self.box = (1.0,) * len(self.n)
        self.box = tuple(float(v) for v in self.box)

    @property
    def dim(self):
        return len(self.n)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def ncell(self):
        return int(math.prod(self.n))

    @property
    def dV(self):
        dv = 1.0
        for d in range(self.dim):
            dv = dv * (self.box[d] / self.n[d])
        return dv

    @property
    def cdtype(self):
        return torch.complex128 if self.precision == "fp64" else torch.complex64


def _problem_struct(problem):
    pr = TwProblem()
    pr.dim = problem.dim
    for d in range(3):
        pr.n[d] = problem.n[d] if d < problem.dim else 1
        pr.box[d] = problem.box[d] if d < problem.dim else 1.0
    pr.hbar_m, pr.G, pr.m_tot, pr.n_tot = problem.hbar_m, problem.G, problem.m_tot, problem.n_tot
    pr.n_real = problem.n_real
    pr.precision = TW_FP64 if problem.precision == "fp64" else TW_FP32_SPLIT
    pr.reserved = 0
    return pr


class Plan:
    """Owns a tw_plan (tables + device workspace) for one Problem on the current device."""

    def __init__(self, problem: Problem, _borrowed=None):
        lib = load_library()
        self.problem = problem
        self._lib = lib
        if _borrowed is not None:      # a batch's class plan: owned by the batch
            self._h = None
            self._borrowed = _borrowed
            return
        self._borrowed = None
        pr = _problem_struct(problem)
        h = ctypes.c_void_p()
        _check(lib.tw_plan_create(ctypes.byref(pr), ctypes.byref(h)), "tw_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._borrowed if self._borrowed is not None else self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tw_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- calls
    def empty_ensemble(self, device="cuda"):
        p = self.problem
        return torch.empty((p.n_real,) + p.shape, dtype=p.cdtype, device=device)

    def sample(self, psi_cl, seed, real_offset=0, out=None):
        """Draw the ensemble (tw_sample). psi_cl: complex128 device tensor of the grid shape."""
        assert psi_cl.dtype == torch.complex128 and psi_cl.is_cuda and psi_cl.is_contiguous()
        out = self.empty_ensemble(psi_cl.device) if out is None else out
        assert out.dtype == self.problem.cdtype and out.is_contiguous()
        _check(self._lib.tw_sample(self.handle, _ptr(psi_cl), ctypes.c_uint64(int(seed) & (2 ** 64 - 1)),
                                   int(real_offset), _ptr(out), _stream()), "tw_sample")
        return out

    def step(self, psi, nsteps, dt, psi_classical=None):
        """Advance psi (and psi_classical) in place by nsteps leapfrog steps (tw_step)."""
        assert psi.dtype == self.problem.cdtype and psi.is_contiguous()
        if psi_classical is not None:
            assert psi_classical.dtype == self.problem.cdtype and psi_classical.is_contiguous()
        _check(self._lib.tw_step(self.handle, _ptr(psi), _ptr(psi_classical), int(nsteps), float(dt), _stream()),
               "tw_step")
        return psi

    def step_tracers(self, psi, nsteps, dt, tracers, psi_classical=None):
        """tw_step with test particles: tracers is a float64 device tensor
        [nfield][ntracer][2 D] (positions, then velocities), updated in place."""
        assert psi.dtype == self.problem.cdtype and psi.is_contiguous()
        if psi_classical is not None:
            assert psi_classical.dtype == self.problem.cdtype and psi_classical.is_contiguous()
        nfield = self.problem.n_real + (1 if psi_classical is not None else 0)
        assert tracers.dtype == torch.float64 and tracers.is_contiguous()
        assert tracers.dim() == 3 and tracers.shape[0] == nfield and tracers.shape[2] == 2 * len(self.problem.n)
        _check(self._lib.tw_step_tracers(self.handle, _ptr(psi), _ptr(psi_classical), int(nsteps), float(dt),
                                         _ptr(tracers), int(tracers.shape[1]), _stream()), "tw_step_tracers")
        return tracers

    def tracer_spread(self, tracers):
        """Variances over the realizations of every particle coordinate [ntracer][2 D] (tw_tracer_spread)."""
        assert tracers.dtype == torch.float64 and tracers.is_contiguous()
        out = torch.empty((tracers.shape[1], tracers.shape[2]), dtype=torch.float64, device=tracers.device)
        _check(self._lib.tw_tracer_spread(self.handle, _ptr(tracers), int(tracers.shape[1]), _ptr(out), _stream()),
               "tw_tracer_spread")
        return out

    def step_adaptive(self, psi, nsteps, dt_max, courant=1.0, psi_classical=None):
        """Advance psi (and psi_classical) in place by nsteps steps whose sizes the
        device chooses (tw_step_adaptive). Returns the step sizes as a float64
        device tensor [nsteps]."""
        assert psi.dtype == self.problem.cdtype and psi.is_contiguous()
        if psi_classical is not None:
            assert psi_classical.dtype == self.problem.cdtype and psi_classical.is_contiguous()
        dts = torch.zeros(max(int(nsteps), 1), dtype=torch.float64, device=psi.device)
        _check(self._lib.tw_step_adaptive(self.handle, _ptr(psi), _ptr(psi_classical), int(nsteps), float(dt_max),
                                          float(courant), _ptr(dts), _stream()), "tw_step_adaptive")
        return dts[: int(nsteps)]

    def autotune(self):
        """Measure both strided-pass organisations and keep the faster (tw_plan_autotune)."""
        v = ctypes.c_int32(-1)
        _check(self._lib.tw_plan_autotune(self.handle, ctypes.byref(v), _stream()), "tw_plan_autotune")
        return int(v.value)

    def set_profiling(self, enable=True):
        """Bracket every kernel launch with HIP events on its stream (tw_plan_set_profiling)."""
        _check(self._lib.tw_plan_set_profiling(self.handle, 1 if enable else 0), "tw_plan_set_profiling")

    def profile(self):
        """{kernel kind: (launches, total device ms)} since the last call (tw_plan_get_profile)."""
        n = NUM_KERNEL_KINDS
        launches = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        _check(self._lib.tw_plan_get_profile(self.handle, n, launches, ms), "tw_plan_get_profile")
        out = {}
        for k in range(n):
            if launches[k]:
                out[self._lib.tw_kernel_kind_name(k).decode()] = (int(launches[k]), float(ms[k]))
        return out

    def moments(self, psi, psi_classical=None, energy=True, per_cell=True, modes=False, decoherence=False):
        """Ensemble moments (tw_moments) as a dict of device tensors (scalars on the host).
        modes=True adds mode_occ, the per-mode occupation <|a_j|^2>; decoherence=True
        adds the per-cell amplitude and phase variances var_amp, var_phase and the
        weighted integrals Var_A, Var_phi."""
        p = self.problem
        dev = psi.device
        f64 = dict(dtype=torch.float64, device=dev)
        out = {}
        if per_cell:
            out["mean_psi"] = torch.empty(p.shape, dtype=torch.complex128, device=dev)
            for k in ("mean_abs2", "mean_rho", "var_rho"):
                out[k] = torch.empty(p.shape, **f64)
        out["norm"] = torch.empty(p.n_real, **f64)
        if energy:
            out["energy"] = torch.empty(p.n_real, **f64)
        if modes:
            out["mode_occ"] = torch.empty(p.shape, **f64)
        deco = None
        if decoherence:
            out["var_amp"] = torch.empty(p.shape, **f64)
            out["var_phase"] = torch.empty(p.shape, **f64)
            deco = torch.empty(2, **f64)
        scal = torch.empty(8, **f64)
        mo = TwMomentsOut()
        for k in ("mean_psi", "mean_abs2", "mean_rho", "var_rho", "mode_occ", "var_amp", "var_phase", "norm",
                  "energy"):
            setattr(mo, k, out[k].data_ptr() if k in out else None)
        mo.decoherence = deco.data_ptr() if deco is not None else None
        mo.scalars = scal.data_ptr()
        _check(self._lib.tw_moments(self.handle, _ptr(psi), _ptr(psi_classical), ctypes.byref(mo), _stream()),
               "tw_moments")
        vals = scal.cpu().tolist()
        for name, v in zip(SCALAR_NAMES, vals):
            out[name] = v
        out["nonfinite"] = int(out["nonfinite"])
        if deco is not None:
            out["Var_A"], out["Var_phi"] = deco.cpu().tolist()
        return out


def moments_static(problem: Problem, psi, psi_classical=None, out=None):
    """Moment reductions without a plan (tw_moments_static): mean_psi,
    mean_abs2, mean_rho, var_rho, norm and the scalars, into the caller's
    device tensors `out` (a dict with those keys plus "scalars" [8]; allocated
    here if None). The library call itself allocates nothing."""
    lib = load_library()
    p = problem
    assert psi.dtype == p.cdtype and psi.is_contiguous()
    if psi_classical is not None:
        assert psi_classical.dtype == p.cdtype and psi_classical.is_contiguous()
    if out is None:
        dev = psi.device
        f64 = dict(dtype=torch.float64, device=dev)
        out = {"mean_psi": torch.empty(p.shape, dtype=torch.complex128, device=dev),
               "mean_abs2": torch.empty(p.shape, **f64), "mean_rho": torch.empty(p.shape, **f64),
               "var_rho": torch.empty(p.shape, **f64), "norm": torch.empty(p.n_real, **f64),
               "scalars": torch.empty(8, **f64)}
    mo = TwMomentsOut()
    for k in ("mean_psi", "mean_abs2", "mean_rho", "var_rho", "norm", "scalars"):
        setattr(mo, k, out[k].data_ptr() if out.get(k) is not None else None)
    pr = _problem_struct(p)
    _check(lib.tw_moments_static(ctypes.byref(pr), _ptr(psi), _ptr(psi_classical), ctypes.byref(mo), _stream()),
           "tw_moments_static")
    return out


class Batch:
    """Owns a tw_batch: several size classes advanced by grouped launches from one HIP graph."""

    def __init__(self, problems):
        lib = load_library()
        self._lib = lib
        self.problems = list(problems)
        arr = (TwProblem * len(self.problems))(*[_problem_struct(p) for p in self.problems])
        h = ctypes.c_void_p()
        _check(lib.tw_batch_create(arr, len(self.problems), ctypes.byref(h)), "tw_batch_create")
        self._h = h
        self.plans = []
        for i, p in enumerate(self.problems):
            ph = ctypes.c_void_p()
            _check(lib.tw_batch_plan(h, i, ctypes.byref(ph)), "tw_batch_plan")
            self.plans.append(Plan(p, _borrowed=ph))

    def autotune(self):
        """Tune the batch (tw_batch_autotune); returns (strided-pass variant, batching mode)."""
        v = ctypes.c_int32(-1)
        m = ctypes.c_int32(-1)
        _check(self._lib.tw_batch_autotune(self._h, ctypes.byref(v), ctypes.byref(m), _stream()), "tw_batch_autotune")
        return int(v.value), int(m.value)

    def step(self, psis, nsteps, dt, classical=None):
        n = len(self.problems)
        assert len(psis) == n
        for p, x in zip(self.problems, psis):
            assert x.dtype == p.cdtype and x.is_contiguous()
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in psis])
        cls = None
        if classical is not None:
            cls = (ctypes.c_void_p * n)(*[(x.data_ptr() if x is not None else None) for x in classical])
        _check(self._lib.tw_batch_step(self._h, ptrs, cls, int(nsteps), float(dt), _stream()), "tw_batch_step")
        return psis

    def close(self):
        if getattr(self, "_h", None):
            for p in self.plans:
                p._borrowed = None
            self._lib.tw_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Fno:
    """Fourier-neural-operator surrogate on the GPU (tw_fno_*): parameters, Adam
    state and data are torch FP32 device tensors owned here / by the caller."""

    def __init__(self, H=256, W=256, c_in=4, width=32, modes_x=16, modes_y=16, layers=4, proj=128, c_out=2,
                 max_batch=8, seed=0, device="cuda"):
        lib = load_library()
        self._lib = lib
        self.cfg = TwFnoConfig(H, W, c_in, width, modes_x, modes_y, layers, proj, c_out)
        self.max_batch = max_batch
        n = lib.tw_fno_param_count(ctypes.byref(self.cfg))
        h = ctypes.c_void_p()
        rc = lib.tw_fno_create(ctypes.byref(self.cfg), max_batch, ctypes.byref(h))
        if rc != 0:
            raise TwError(f"tw_fno_create failed: {STATUS.get(rc, rc)}: {lib.tw_fno_last_error().decode()}")
        self._h = h
        self.params = torch.empty(n, dtype=torch.float32, device=device)
        self.grads = torch.zeros(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.step_count = 0
        self._call(lib.tw_fno_init_params(h, ctypes.c_uint64(seed), _ptr(self.params), _stream()), "init")

    def _call(self, rc, what):
        if rc != 0:
            raise TwError(f"tw_fno_{what} failed: {STATUS.get(rc, rc)}: {self._lib.tw_fno_last_error().decode()}")

    def forward(self, x, out=None):
        b = x.shape[0]
        assert x.dtype == torch.float32 and x.is_contiguous() and b <= self.max_batch
        out = torch.empty(x.shape[:3] + (self.cfg.c_out,), dtype=torch.float32, device=x.device) if out is None else out
        self._call(self._lib.tw_fno_forward(self._h, _ptr(self.params), _ptr(x), b, _ptr(out), _stream()), "forward")
        return out

    def backward(self, x, dy):
        self._call(self._lib.tw_fno_backward(self._h, _ptr(self.params), _ptr(x), x.shape[0], _ptr(dy),
                                             _ptr(self.grads), _stream()), "backward")
        return self.grads

    def mse(self, y, t, want_grad=True):
        loss = torch.empty(1, dtype=torch.float32, device=y.device)
        dy = torch.empty_like(y) if want_grad else None
        self._call(self._lib.tw_fno_mse(_ptr(y), _ptr(t), y.numel(), _ptr(dy), _ptr(loss), _stream()), "mse")
        return loss, dy

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        self._call(self._lib.tw_fno_adam(_ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v),
                                         self.params.numel(), lr, b1, b2, eps, self.step_count, _stream()), "adam")

    def train_step(self, x, t, lr=1e-3):
        y = self.forward(x)
        loss, dy = self.mse(y, t)
        self.backward(x, dy)
        self.adam(lr)
        return loss

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tw_fno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
