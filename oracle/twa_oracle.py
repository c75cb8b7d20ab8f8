"""CPU FP64 oracle: truncated-Wigner ensemble of Schrodinger-Poisson fields.

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module. It is deliberately plain and slow: every
step of the method is written out in the order the paper gives it, in FP64,
with numpy's FFT (or, for tiny grids, the DFT summed from its definition) as
the only library primitive.

Array conventions
-----------------
A field on a D-dimensional grid with points-per-axis (n0, n1, n2) (x first) is
a numpy array of shape (n2, n1, n0) for D=3, (n1, n0) for D=2, (n0,) for D=1:
x is the fastest index, so the flat cell index is g = x + n0*(y + n1*z). An
ensemble carries a leading realization axis. Fields are the normalised psi'
of the paper (Sec. "Estimating the breaktime", Eq. (mft_normed)):
sum_g |psi'_g|^2 dV = 1, with rho = M_tot |psi'|^2.

Fourier convention (the paper states none): forward DFT
F[f]_j = sum_g f_g exp(-2 pi i j.g / n), inverse with +i and 1/N;
k_j = 2 pi j / L with j in FFT order. Only |k|^2 enters the method, so the
sign convention does not change any result.
"""
import numpy as np

from . import philox

FOUR_PI = 4.0 * np.pi
SAMPLE_KEY_TAG = 0x5457          # second Philox key word for Wigner sampling


# --------------------------------------------------------------------------- grid
class Grid:
    """Periodic grid: D in {1,2,3}, points n[d] and box length L[d] per axis (x first)."""

    def __init__(self, n, box):
        self.n = tuple(int(v) for v in n)
        self.box = tuple(float(v) for v in box)
        if len(self.n) != len(self.box) or not 1 <= len(self.n) <= 3:
            raise ValueError("n and box must have the same length 1..3")
        self.dim = len(self.n)
        self.shape = tuple(reversed(self.n))          # numpy shape, x last
        self.ncell = int(np.prod(self.n))
        dv = 1.0
        for d in range(self.dim):
            dv = dv * (self.box[d] / self.n[d])
        self.dV = dv
        self.volume = float(np.prod(self.box))

    def k_axis(self, d):
        """Wavenumbers 2 pi j / L_d along axis d, j in FFT order."""
        n = self.n[d]
        j = np.fft.fftfreq(n, d=1.0 / n)
        return 2.0 * np.pi * j / self.box[d]

    def k2(self):
        """|k|^2 on the full grid (numpy shape)."""
        out = np.zeros(self.shape)
        for d in range(self.dim):
            kd = self.k_axis(d)
            ax = self.dim - 1 - d                       # numpy axis of grid axis d
            bshape = [1] * self.dim
            bshape[ax] = self.n[d]
            out = out + (kd ** 2).reshape(bshape)
        return out


# ---------------------------------------------------------------- transforms
def _spatial_axes(grid, arr):
    return tuple(range(arr.ndim - grid.dim, arr.ndim))


def dft_naive(grid, f, inverse=False):
    """D-dimensional DFT summed from its definition, O(N^2); tiny grids only."""
    if grid.ncell > 4096:
        raise ValueError("naive DFT is for grids of at most 4096 cells")
    idx = np.indices(grid.shape).reshape(grid.dim, -1)    # numpy-axis order
    phase = np.zeros((grid.ncell, grid.ncell))
    for ax in range(grid.dim):
        n = grid.shape[ax]
        phase = phase + np.outer(idx[ax], idx[ax]) / n
    sign = 1.0 if inverse else -1.0
    mat = np.exp(sign * 2j * np.pi * phase)
    lead = f.shape[: f.ndim - grid.dim]
    flat = f.reshape(lead + (grid.ncell,))
    out = flat @ mat.T
    if inverse:
        out = out / grid.ncell
    return out.reshape(f.shape)


class Transform:
    """Forward/inverse D-dim DFT, by numpy FFT ('fft') or by definition ('naive')."""

    def __init__(self, grid, mode="fft"):
        if mode not in ("fft", "naive"):
            raise ValueError(mode)
        self.grid = grid
        self.mode = mode

    def fwd(self, f):
        if self.mode == "naive":
            return dft_naive(self.grid, f)
        return np.fft.fftn(f, axes=_spatial_axes(self.grid, f))

    def inv(self, f):
        if self.mode == "naive":
            return dft_naive(self.grid, f, inverse=True)
        return np.fft.ifftn(f, axes=_spatial_axes(self.grid, f))


# ------------------------------------------------------------------ sampling
def sample_noise(grid, n_real, seed, real_offset=0):
    """Standard-normal pairs (z1, z2) for every (realization, cell).

    Counter = (cell g, global realization index, 0, 0), key = (seed, 0x5457);
    words 0 and 1 of the Philox block feed Box-Muller. Shapes (n_real,)+grid.shape.
    """
    g = np.arange(grid.ncell, dtype=np.uint64)
    z1 = np.empty((n_real, grid.ncell))
    z2 = np.empty((n_real, grid.ncell))
    zeros = np.zeros(grid.ncell, dtype=np.uint64)
    for r in range(n_real):
        rr = np.full(grid.ncell, real_offset + r, dtype=np.uint64)
        words = philox.philox4x64([g, rr, zeros, zeros], (seed, SAMPLE_KEY_TAG))
        z1[r], z2[r] = philox.box_muller(words[0], words[1])
    shape = (n_real,) + grid.shape
    return z1.reshape(shape), z2.reshape(shape)


def noise_scale(grid, n_tot):
    """Amplitude factor 0.5 / sqrt(n_tot dV) applied to a unit-normal pair.

    Eq. (sample) adds independent Gaussians to the real and imaginary parts of
    the normalised field at each grid point. Reading: each cell is one mode
    alpha_g = sqrt(n_tot dV) psi'_g whose vacuum noise has E|d alpha|^2 = 1/2
    (quadrature variance 1/4, the Wigner function of a coherent state), so
    d psi' = (z1 + i z2) / 2 / sqrt(n_tot dV).
    """
    return 0.5 / np.sqrt(n_tot * grid.dV)


def sample(grid, psi_cl, n_real, n_tot, seed, real_offset=0):
    """Draw n_real fields from the coherent state's Wigner function (Sec.
    "Initial conditions generation", Eq. (sample)): psi_i = psi_cl + noise."""
    z1, z2 = sample_noise(grid, n_real, seed, real_offset)
    sc = noise_scale(grid, n_tot)
    re = psi_cl.real[None] + z1 * sc
    im = psi_cl.imag[None] + z2 * sc
    return re + 1j * im


# ---------------------------------------------------------------- evolution
class Problem:
    """Physical parameters of Eq. (mft_normed): hbar/m, G, M_tot on a Grid."""

    def __init__(self, grid, hbar_m=1.0, G=1.0, m_tot=1.0, transform="fft"):
        self.grid = grid
        self.hbar = float(hbar_m)
        self.G = float(G)
        self.m_tot = float(m_tot)
        self.T = Transform(grid, transform)
        self.k2 = grid.k2()


def density(prob, psi):
    """rho = M_tot |psi'|^2 (Eq. (mft_normed))."""
    return prob.m_tot * (psi.real ** 2 + psi.imag ** 2)


def potential(prob, rho):
    """Solve lap V = 4 pi G rho spectrally: V_k = -4 pi G rho_k / |k|^2, V_0 = 0."""
    rho_k = prob.T.fwd(rho)
    k2 = prob.k2
    safe = np.where(k2 == 0.0, 1.0, k2)
    v_k = np.where(k2 == 0.0, 0.0, -FOUR_PI * prob.G * rho_k / safe)
    return prob.T.inv(v_k).real


def drift(prob, psi, tau):
    """Kinetic update U^T(tau) in Fourier space: psi_k *= exp(-i hbar |k|^2 tau / 2).

    Sign: Eq. (mft_normed) has i d_t psi = (-hbar lap / 2 + V/hbar) psi, whose
    kinetic propagator carries exp(-i hbar k^2 tau / 2); the opposite sign
    printed for U^T in "Integrating the equations of motion" is read as a typo.
    """
    psi_k = prob.T.fwd(psi)
    psi_k = psi_k * np.exp(-1j * (prob.hbar * prob.k2 * tau / 2.0))
    return prob.T.inv(psi_k)


def kick(prob, psi, V, dt):
    """Potential update U^V(dt) in real space: psi *= exp(-i dt V / hbar)."""
    return psi * np.exp(-1j * (dt * V / prob.hbar))


def step(prob, psi, dt):
    """One symplectic pseudo-spectral leapfrog step (Sec. "Integrating the
    equations of motion"): half drift, potential from the drifted field, full
    kick, half drift. Each realization sees only its own potential (Sec.
    "Approximation scheme": V_i depends on psi_i alone)."""
    psi = drift(prob, psi, dt / 2.0)
    V = potential(prob, density(prob, psi))
    psi = kick(prob, psi, V, dt)
    return drift(prob, psi, dt / 2.0)


def evolve(prob, psi, nsteps, dt):
    """Apply `step` nsteps times; no merging of adjacent half drifts."""
    for _ in range(int(nsteps)):
        psi = step(prob, psi, dt)
    return psi


# ------------------------------------------------------------ adaptive step
def kinetic_dt_bound(prob):
    """Kinetic step bound of the time-step footnote (Sec. "Numerical
    implementation"): the phase gradient must not alias, dt < 4 pi / (hbar
    k_max dk), with k_max = pi / dx (the largest wavenumber on the grid; the
    printed hbar/2/dx is read as garbled) and dk = 2 pi / L; the smallest over
    the axes."""
    g = prob.grid
    out = np.inf
    for n, L in zip(g.n, g.box):
        dx = L / n
        out = min(out, 4.0 * np.pi / (prob.hbar * (np.pi / dx) * (2.0 * np.pi / L)))
    return out


def adaptive_dt(prob, vmax, dt_max, courant):
    """Step size from the rule of Sec. "Integrating the equations of motion":
    c_f times the smaller of the potential bound 2 pi hbar / max|V| (the kick
    phase stays below 2 pi c_f) and the kinetic bound, never above dt_max."""
    dt = min(dt_max, courant * kinetic_dt_bound(prob))
    if vmax > 0.0:
        dt = min(dt, courant * 2.0 * np.pi * prob.hbar / vmax)
    return dt


def evolve_adaptive(prob, psi, nsteps, dt_max, courant):
    """Leapfrog steps whose sizes follow `adaptive_dt`, one size for all fields
    (psi holds every field, classical one included, on its leading axis).
    Steps 0 and 1 take their size from the potential of the initial fields;
    step n + 2 from the potential evaluated inside step n (the one the kick of
    step n uses). Returns (psi, step sizes)."""
    vm0 = float(np.abs(potential(prob, density(prob, psi))).max())
    dts = [adaptive_dt(prob, vm0, dt_max, courant)] * 2
    for n in range(int(nsteps)):
        dt = dts[n]
        psi = drift(prob, psi, dt / 2.0)
        V = potential(prob, density(prob, psi))
        dts.append(adaptive_dt(prob, float(np.abs(V).max()), dt_max, courant))
        psi = kick(prob, psi, V, dt)
        psi = drift(prob, psi, dt / 2.0)
    return psi, np.array(dts[: int(nsteps)])


# ---------------------------------------------------------- tracer particles
def grid_gradient(prob, V):
    """Gradient of V on the grid by fourth-order central differences along
    each axis: (-V[g+2] + 8 V[g+1] - 8 V[g-1] + V[g-2]) / (12 dx), periodic.
    V carries a leading field axis; returns one array per spatial axis (x first)."""
    g = prob.grid
    out = []
    for d in range(g.dim):
        ax = V.ndim - 1 - d
        dx = g.box[d] / g.n[d]
        f = lambda s: np.roll(V, -s, axis=ax)
        out.append((-f(2) + 8.0 * f(1) - 8.0 * f(-1) + f(-2)) / (12.0 * dx))
    return out


def interpolate(prob, F, pos):
    """Linear (cloud-in-cell) interpolation of the grid field F (leading
    field axis) at positions pos[f][i][d] (any real coordinates: wrapped into
    the periodic box). Returns [field][particle]."""
    g = prob.grid
    nf, npart = pos.shape[0], pos.shape[1]
    out = np.zeros((nf, npart))
    for f in range(nf):
        flat = F[f].reshape(-1)
        for i in range(npart):
            base = []
            frac = []
            for d in range(g.dim):
                s = (pos[f, i, d] % g.box[d]) / (g.box[d] / g.n[d])
                i0 = int(np.floor(s))
                base.append(i0)
                frac.append(s - i0)
            acc = 0.0
            for corner in range(1 << g.dim):
                w = 1.0
                idx = 0
                stride = 1
                for d in range(g.dim):
                    bit = (corner >> d) & 1
                    w *= frac[d] if bit else 1.0 - frac[d]
                    idx += ((base[d] + bit) % g.n[d]) * stride
                    stride *= g.n[d]
                acc += w * flat[idx]
            out[f, i] = acc
    return out


def step_tracers(prob, psi, tracers, dt):
    """One step of fields and test particles (Sec. "Modeling decoherence":
    each realization's particles move in that realization's own potential,
    dr/dt = v, dv/dt = -grad V_s(r)). The particles follow the same splitting
    as the fields: half drift r += v dt/2, kick v -= dt grad V(r) with the
    potential the field kick uses, half drift. tracers[f][i] = (r_0..r_{D-1},
    v_0..v_{D-1}); positions are not wrapped (spreads need unwrapped paths)."""
    D = prob.grid.dim
    psi = drift(prob, psi, dt / 2.0)
    V = potential(prob, density(prob, psi))
    tr = tracers.copy()
    tr[:, :, :D] += 0.5 * dt * tr[:, :, D:]
    grads = grid_gradient(prob, V)
    for d in range(D):
        tr[:, :, D + d] -= dt * interpolate(prob, grads[d], tr[:, :, :D])
    tr[:, :, :D] += 0.5 * dt * tr[:, :, D:]
    psi = kick(prob, psi, V, dt)
    return drift(prob, psi, dt / 2.0), tr


def evolve_tracers(prob, psi, tracers, nsteps, dt):
    for _ in range(int(nsteps)):
        psi, tracers = step_tracers(prob, psi, tracers, dt)
    return psi, tracers


def tracer_spread(tracers, n_real):
    """Plug-in variances over the realizations (the first n_real entries) of
    every particle's position and velocity components: [particle][2D]."""
    t = tracers[:n_real]
    return ((t - t.mean(axis=0)[None]) ** 2).mean(axis=0)


# ------------------------------------------------------------- diagnostics
def norm(prob, psi):
    """sum_g |psi'_g|^2 dV per realization (1 for a normalised field)."""
    g = prob.grid
    a2 = psi.real ** 2 + psi.imag ** 2
    return a2.reshape(a2.shape[: a2.ndim - g.dim] + (-1,)).sum(axis=-1) * g.dV


def energy(prob, psi):
    """E = M_tot [ (hbar^2/2) int |grad psi'|^2 + (1/2) int V |psi'|^2 ] per realization.

    The functional whose variation gives Eq. (mft_normed); the gradient term is
    evaluated spectrally: int |grad psi|^2 dV = (dV/N) sum_k |k|^2 |F[psi]_k|^2.
    """
    g = prob.grid
    lead = psi.shape[: psi.ndim - g.dim]
    psi_k = prob.T.fwd(psi)
    kin = (prob.k2 * (psi_k.real ** 2 + psi_k.imag ** 2))
    kin = kin.reshape(lead + (-1,)).sum(axis=-1) * (g.dV / g.ncell)
    rho = density(prob, psi)
    V = potential(prob, rho)
    pot = (V * (psi.real ** 2 + psi.imag ** 2)).reshape(lead + (-1,)).sum(axis=-1) * g.dV
    return prob.m_tot * (0.5 * prob.hbar ** 2 * kin + 0.5 * pot)


def mode_amplitudes(prob, psi, n_tot):
    """Unitary mode amplitudes a_j = F[alpha]_j / sqrt(N), alpha_g = sqrt(n_tot dV) psi'_g
    (Sec. "Quantum description", Eq. (psi2a): the field is a sum of mode operators)."""
    g = prob.grid
    alpha = np.sqrt(n_tot * g.dV) * psi
    return prob.T.fwd(alpha) / np.sqrt(g.ncell)


def decoherence(prob, psi, n_tot):
    """Amplitude and phase spread of the ensemble (Sec. "Large quantum
    corrections", Eqs. (varA) and (varPhi)). Per cell: the plug-in variance of
    the amplitude A = |psi'| and of the phase deviation dphi = arg(psi'
    conj<psi'>) in (-pi, pi] from the phase of the ensemble-mean field; the
    integrals weight them with the normal-ordered density <psi^dag psi> =
    <|psi'|^2> - 1/(2 n_tot dV) (the Weyl average minus the vacuum half quantum
    per cell mode):
        Var A~   = sum_g dV <psi^dag psi> <dA^2> / <A>
        Var phi~ = sum_g dV <psi^dag psi> <dphi^2> / (pi / sqrt 3)
    (the constant as printed; a uniformly random phase has <dphi^2> = pi^2/3).
    Returns (var_amp, var_phase, Var_A, Var_phi)."""
    g = prob.grid
    ns = psi.shape[0]
    amp = np.abs(psi)
    mean_amp = amp.sum(axis=0) / ns
    var_amp = ((amp - mean_amp[None]) ** 2).sum(axis=0) / ns
    m1 = psi.sum(axis=0) / ns
    dphi = np.angle(psi * np.conj(m1)[None])
    var_phase = (dphi ** 2).sum(axis=0) / ns
    occ = (psi.real ** 2 + psi.imag ** 2).sum(axis=0) / ns - 1.0 / (2.0 * n_tot * g.dV)
    safe = np.where(mean_amp > 0, mean_amp, 1.0)
    var_a = (g.dV * occ * np.where(mean_amp > 0, var_amp / safe, 0.0)).sum()
    var_p = (g.dV * occ * var_phase).sum() / (np.pi / np.sqrt(3.0))
    return var_amp, var_phase, float(var_a), float(var_p)


def moments(prob, psi, n_tot, psi_cl=None, modes=False, decoherence_=False):
    """Ensemble moments by the plug-in estimator (1/N_s) sum_i (Sec. "Evaluating
    operators"); every Weyl symbol is evaluated per realization and averaged.

    Returns a dict:
      mean_psi   <psi'>_g                       (complex, grid shape)
      mean_abs2  <|psi'|^2>_g (Weyl, symmetric ordering)
      mean_rho   <rho>_g = M_tot <|psi'|^2>_g
      var_rho    <(rho - <rho>)^2>_g
      norm, energy            per realization
      Q_raw      sum_g dV (<|psi'|^2> - |<psi'>|^2)   (Eq. (Q) with psi' = psi/sqrt(n_tot))
      Q_sym      Q_raw - N / (2 n_tot): the Weyl vacuum half-quantum per cell mode removed
      dev_rho_L1 sum_g dV |<rho> - rho_cl| / M_tot          (if psi_cl given)
      dev_psi_L2 sum_g dV |<psi'> - psi'_cl|^2               (if psi_cl given)
      nonfinite  count of realizations holding a non-finite value
      mode_occ   <|a_j|^2> per Fourier mode, a_j from mode_amplitudes (if modes=True)
      var_amp, var_phase, Var_A, Var_phi   from `decoherence` (if decoherence_=True)
    """
    g = prob.grid
    ns = psi.shape[0]
    a2 = psi.real ** 2 + psi.imag ** 2
    mean_psi = psi.sum(axis=0) / ns
    mean_abs2 = a2.sum(axis=0) / ns
    rho = prob.m_tot * a2
    mean_rho = rho.sum(axis=0) / ns
    var_rho = ((rho - mean_rho[None]) ** 2).sum(axis=0) / ns
    var_psi = mean_abs2 - (mean_psi.real ** 2 + mean_psi.imag ** 2)
    q_raw = var_psi.sum() * g.dV
    out = dict(mean_psi=mean_psi, mean_abs2=mean_abs2, mean_rho=mean_rho,
               var_rho=var_rho, norm=norm(prob, psi), energy=energy(prob, psi),
               Q_raw=q_raw, Q_sym=q_raw - g.ncell / (2.0 * n_tot))
    flat = psi.reshape(ns, -1)
    out["nonfinite"] = int((~np.isfinite(flat)).any(axis=1).sum())
    if decoherence_:
        out["var_amp"], out["var_phase"], out["Var_A"], out["Var_phi"] = decoherence(prob, psi, n_tot)
    if modes:
        a = mode_amplitudes(prob, psi, n_tot)
        out["mode_occ"] = (a.real ** 2 + a.imag ** 2).sum(axis=0) / ns
    if psi_cl is not None:
        rho_cl = density(prob, psi_cl)
        out["dev_rho_L1"] = np.abs(mean_rho - rho_cl).sum() * g.dV / prob.m_tot
        d = mean_psi - psi_cl
        out["dev_psi_L2"] = (d.real ** 2 + d.imag ** 2).sum() * g.dV
    return out


def run(prob, psi_cl, n_real, n_tot, seed, nsteps, dt, real_offset=0):
    """Sample an ensemble, evolve it and the classical field, return
    (psi, psi_cl_t, moments): the whole method end to end."""
    psi = sample(prob.grid, psi_cl, n_real, n_tot, seed, real_offset)
    psi = evolve(prob, psi, nsteps, dt)
    cl = evolve(prob, psi_cl, nsteps, dt)
    return psi, cl, moments(prob, psi, n_tot, cl)
