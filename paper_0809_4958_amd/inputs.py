"""Seeded synthetic inputs for the fine-box lattice-Boltzmann run.

This module holds none of the lattice-Boltzmann arithmetic: it only draws
random numbers and evaluates the input fields they define, so that the FP64
oracle and the GPU library are fed the very same numbers.

What it produces (all FP64 numpy arrays):

* ``ou_strain``      -- a traceless 3x3 velocity-gradient history A(t_n) that
                        follows an Ornstein-Uhlenbeck process; it drives the
                        affine boundary u_b = A (y - x_c).
* ``KSField``        -- a kinematic-simulation (KS) velocity field: a finite
                        sum of divergence-free Fourier modes with a
                        k^-5/3 exp(-k eta) spectrum in Kolmogorov units.  It
                        stands in for the DNS of homogeneous isotropic
                        turbulence the paper samples (Sec. 3, run 4 of the
                        DNS study), whose data are not available.
* ``Tracer``         -- a Lagrangian tracer advected through the KS field
                        (RK4); the box comoves with it (Sec. 2).
* ``UnitMap``        -- the reduced-unit matching of Eq. (1): Kolmogorov
                        units of the KS field to lattice units of a box of N
                        nodes that spans a given number of Kolmogorov lengths.
* ``face_samples`` / ``initial_field`` -- the Galilei-transformed field
                        w = u - v(t) (Sec. 2) evaluated on corner-aligned
                        face sample grids at sample times, and on every node
                        at t = 0, in lattice units.
* ``chain_init``     -- a bead-spring chain as a random walk of unit bonds,
                        shifted so its centre of mass sits on the anchor.
* ``box_sizes``, ``anchors`` -- batch and multi-chain layouts.
* ``upsampler_samples`` -- training / evaluation samples of the learned
                        boundary upsampler: coarse face samples every dt
                        steps and the dense per-step face field they should
                        be mapped to, both from the KS field.

Seeds follow ``np.random.SeedSequence(entropy=0x08094958,
spawn_key=(config_idx, stream_idx))`` with streams 0 = OU / KS modes,
1 = tracer start, 2 = chain init, 3 = box sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

ENTROPY = 0x08094958

# Face order used for boundary samples: -x, +x, -y, +y, -z, +z.  On each face
# the two tangential axes are (u, v) = the lower-index axis first.
FACE_AXES = ((1, 2), (1, 2), (0, 2), (0, 2), (0, 1), (0, 1))


def rng(config_idx: int, stream_idx: int) -> np.random.Generator:
    """Independent generator for (configuration, stream)."""
    ss = np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config_idx, stream_idx))
    return np.random.Generator(np.random.PCG64(ss))


# --------------------------------------------------------------------------
# Ornstein-Uhlenbeck strain history (affine boundary)
# --------------------------------------------------------------------------
def _traceless(m: np.ndarray) -> np.ndarray:
    return m - np.trace(m) / 3.0 * np.eye(3)


def ou_strain(n_samples: int, gen: np.random.Generator, corr_steps: float = 500.0,
              rms: float = 1e-3) -> np.ndarray:
    """Traceless OU matrix history, shape [n_samples, 9] (row-major A).

    Exact OU update with correlation time ``corr_steps`` (in LB steps):
    A_{n+1} = e^{-1/T} A_n + sigma sqrt(1 - e^{-2/T}) P(xi_n), with P the
    traceless projection of a 3x3 standard-normal matrix.  The projection
    leaves variance sigma^2 on the 6 off-diagonal and (2/3) sigma^2 on the 3
    diagonal entries, so sigma = rms * sqrt(9/8) makes the rms over all nine
    entries equal ``rms``.  A_0 is drawn from the stationary law.
    """
    sigma = rms * math.sqrt(9.0 / 8.0)
    decay = math.exp(-1.0 / corr_steps)
    kick = sigma * math.sqrt(1.0 - math.exp(-2.0 / corr_steps))
    out = np.empty((n_samples, 3, 3))
    out[0] = sigma * _traceless(gen.standard_normal((3, 3)))
    for n in range(1, n_samples):
        out[n] = decay * out[n - 1] + kick * _traceless(gen.standard_normal((3, 3)))
    return out.reshape(n_samples, 9)


# --------------------------------------------------------------------------
# Kinematic simulation field (stand-in for the DNS)
# --------------------------------------------------------------------------
class KSField:
    """u(x, t) = sum_n A_n cos(k_n.x + w_n t) + B_n sin(k_n.x + w_n t).

    Kolmogorov units (eta = tau_eta = u_eta = 1, nu = 1).  Wavenumbers are
    log-spaced in [k_min, k_max], directions uniform on the sphere, A_n and
    B_n are perpendicular to k_n (so div u = 0 exactly) with
    |A_n|^2 = |B_n|^2 = E(k_n) dk_n, E(k) = C k^-5/3 exp(-k), and
    w_n = 0.5 sqrt(k_n^3 E(k_n)).  C is fixed so that the mean squared
    velocity gradient <du_i/dx_j du_i/dx_j> = sum_n k_n^2 E_n dk_n equals 1,
    i.e. the dissipation rate nu <|grad u|^2> is 1 in Kolmogorov units.
    """

    def __init__(self, gen: np.random.Generator, n_modes: int = 200,
                 k_min: float = 0.02, k_max: float = 3.0):
        k = np.geomspace(k_min, k_max, n_modes)
        # widths of the log-spaced bins (geometric midpoints)
        r = (k_max / k_min) ** (1.0 / max(n_modes - 1, 1))
        dk = k * (math.sqrt(r) - 1.0 / math.sqrt(r)) if n_modes > 1 else np.ones(1)
        e = k ** (-5.0 / 3.0) * np.exp(-k)
        e *= 1.0 / np.sum(k * k * e * dk)
        d = gen.standard_normal((n_modes, 3))
        khat = d / np.linalg.norm(d, axis=1, keepdims=True)
        amp = np.sqrt(e * dk)

        def perp(v):
            v = v - np.sum(v * khat, axis=1, keepdims=True) * khat
            return v / np.linalg.norm(v, axis=1, keepdims=True)

        self.A = perp(gen.standard_normal((n_modes, 3))) * amp[:, None]
        self.B = perp(gen.standard_normal((n_modes, 3))) * amp[:, None]
        self.k = k[:, None] * khat           # [n, 3]
        self.kmag = k
        self.omega = 0.5 * np.sqrt(k ** 3 * e)
        self.E = e
        self.dk = dk

    def velocity(self, x: np.ndarray, t: float) -> np.ndarray:
        """u at points x[..., 3] and time t (Kolmogorov units)."""
        ph = x @ self.k.T + self.omega * t
        return np.cos(ph) @ self.A + np.sin(ph) @ self.B

    def time_derivative(self, x: np.ndarray, t: float) -> np.ndarray:
        """du/dt at fixed points x[..., 3]."""
        ph = x @ self.k.T + self.omega * t
        return (-np.sin(ph) * self.omega) @ self.A + (np.cos(ph) * self.omega) @ self.B

    def gradient(self, x: np.ndarray, t: float) -> np.ndarray:
        """du_i/dx_j at points x[..., 3]: shape [..., 3 (i), 3 (j)]."""
        ph = x @ self.k.T + self.omega * t
        c, s = np.cos(ph), np.sin(ph)
        # d/dx_j [A_i cos + B_i sin] = (-A_i sin + B_i cos) k_j
        return (np.einsum('...n,ni,nj->...ij', -s, self.A, self.k)
                + np.einsum('...n,ni,nj->...ij', c, self.B, self.k))

    def _coef(self, x0: np.ndarray, t: float) -> np.ndarray:
        """Complex mode coefficients (A - iB) e^{i(k.x0 + w t)}, shape [n, 3]."""
        ph = self.k @ x0 + self.omega * t
        return (self.A - 1j * self.B) * np.exp(1j * ph)[:, None]

    def grid_velocity(self, x0: np.ndarray, t: float, axes: list[np.ndarray]) -> np.ndarray:
        """u on the tensor grid x0 + sum_d offs_d e_d, for the listed 3 axes.

        ``axes`` holds three 1-D arrays of offsets along x, y, z.  Returns
        [len(z), len(y), len(x), 3].  Uses e^{ik.(x0+r)} = e^{ik.x0} prod_d
        e^{ik_d r_d}, which is exact; only the evaluation order differs from
        ``velocity``.
        """
        return self._grid_eval(self._coef(x0, t), axes)

    def grid_vorticity(self, x0: np.ndarray, t: float, axes: list[np.ndarray]) -> np.ndarray:
        """Analytic vorticity curl u on the same tensor grid, [nz][ny][nx][3]:
        the curl of Re[c e^{ik.x}] is Re[(i k x c) e^{ik.x}] mode by mode."""
        c = self._coef(x0, t)
        return self._grid_eval(1j * np.cross(self.k, c), axes)

    def _grid_eval(self, c: np.ndarray, axes: list[np.ndarray]) -> np.ndarray:
        ex = np.exp(1j * np.outer(axes[0], self.k[:, 0]))  # [nx, n]
        ey = np.exp(1j * np.outer(axes[1], self.k[:, 1]))
        ez = np.exp(1j * np.outer(axes[2], self.k[:, 2]))
        out = np.empty((len(axes[2]), len(axes[1]), len(axes[0]), 3))
        for iz in range(len(axes[2])):
            m = ey * ez[iz][None, :]                        # [ny, n]
            for comp in range(3):
                out[iz, :, :, comp] = np.real((m * c[:, comp][None, :]) @ ex.T)
        return out


@dataclass
class Tracer:
    """Trajectory X(t), v(t) = u(X(t), t) of a passive tracer (Sec. 2)."""
    times: np.ndarray   # [T] Kolmogorov times
    pos: np.ndarray     # [T, 3]
    vel: np.ndarray     # [T, 3]


def tracer_path(ks: KSField, x0: np.ndarray, times: np.ndarray, h_max: float = 0.02) -> Tracer:
    """Integrate dX/dt = u(X, t) with classical RK4 to each listed time."""
    times = np.asarray(times, dtype=np.float64)
    pos = np.empty((len(times), 3))
    x = np.array(x0, dtype=np.float64)
    t = 0.0
    for i, tt in enumerate(times):
        span = tt - t
        if span < 0:
            raise ValueError("tracer times must be non-decreasing and >= 0")
        n = max(1, int(math.ceil(span / h_max))) if span > 0 else 0
        if n:
            h = span / n
            for _ in range(n):
                k1 = ks.velocity(x, t)
                k2 = ks.velocity(x + 0.5 * h * k1, t + 0.5 * h)
                k3 = ks.velocity(x + 0.5 * h * k2, t + 0.5 * h)
                k4 = ks.velocity(x + h * k3, t + h)
                x = x + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
                t = t + h
        t = tt
        pos[i] = x
    vel = np.stack([ks.velocity(p, tt) for p, tt in zip(pos, times)])
    return Tracer(times, pos, vel)


# --------------------------------------------------------------------------
# Eq. (1): reduced-unit matching between the KS (Kolmogorov units) and LB
# --------------------------------------------------------------------------
@dataclass
class UnitMap:
    """Lattice box of ``n`` nodes per edge spanning ``width_eta`` Kolmogorov lengths.

    eta~ = (n-1)/width_eta lattice spacings, nu~ = (tau-1/2)/3,
    tau~_eta = eta~^2/nu~ steps (Sec. 3), and by Eq. (1) a velocity w in
    Kolmogorov units maps to w~ = w eta~/tau~_eta = w nu~/eta~.
    """
    n: int
    tau: float
    width_eta: float = 2.0

    @property
    def eta(self) -> float:
        return (self.n - 1) / self.width_eta

    @property
    def nu(self) -> float:
        return (self.tau - 0.5) / 3.0

    @property
    def tau_eta(self) -> float:
        return self.eta ** 2 / self.nu

    @property
    def u_scale(self) -> float:
        return self.eta / self.tau_eta

    def mach(self) -> float:
        """Ma = eta~ / (tau~_eta c_s) with c_s = 1/sqrt(3) (Sec. 3)."""
        return self.eta / (self.tau_eta * math.sqrt(1.0 / 3.0))


def paper_mach(zoom: float, eta_over_delta: float, nu_lb: float) -> float:
    """Mach number of Sec. 3 for zoom z, eta/Delta and LB viscosity nu~."""
    eta_lb = eta_over_delta * zoom
    tau_eta_lb = eta_lb ** 2 / nu_lb
    return eta_lb / (tau_eta_lb * math.sqrt(1.0 / 3.0))


def _sample_offsets(n_nodes: int, res: int, centre: float) -> np.ndarray:
    """Corner-aligned sample grid: point p sits at node coordinate p (n-1)/(res-1)."""
    return np.arange(res) * ((n_nodes - 1) / (res - 1)) - centre


def face_samples(ks: KSField, tracer: Tracer, dims: tuple[int, int, int], units: UnitMap,
                 res: int, step_times: np.ndarray) -> np.ndarray:
    """Tracer-frame samples w~ on the six faces, [len(step_times), 6, res, res, 3].

    ``dims`` = (nx, ny, nz) nodes; ``step_times`` are LB step indices; the
    tracer must have been integrated to the matching Kolmogorov times
    step/tau~_eta.  Face f lies at node coordinate 0 (even f) or n-1 (odd f)
    along axis f//2; entry [v][u] holds grid point (u, v) along the face's
    tangential axes (lower-index axis = u).  Evaluated for all sample times at
    once: u = Re sum_n (A_n - i B_n) e^{i(k_n.X(t) + w_n t)} e^{i k_n.r}, with
    e^{i k_n.r} tabulated once per face.
    """
    dims = tuple(int(d) for d in dims)
    centre = [(d - 1) / 2.0 for d in dims]
    T = len(step_times)
    tk = np.asarray(step_times, dtype=np.float64) / units.tau_eta
    # per-time mode coefficients C[t, n, c] = (A - iB)_{n,c} e^{i(k_n . X(t) + w_n t)}
    ph = tracer.pos[:T] @ ks.k.T + ks.omega[None, :] * tk[:, None]          # [T, n]
    amp = ks.A - 1j * ks.B                                                 # [n, 3]
    coef = np.exp(1j * ph)[:, :, None] * amp[None, :, :]                   # [T, n, 3]
    cflat = np.ascontiguousarray(coef.transpose(0, 2, 1)).reshape(T * 3, -1)  # [(t,c), n]
    out = np.empty((T, 6, res, res, 3))
    for f in range(6):
        a = f // 2
        au, av = FACE_AXES[f]
        r_a = ((0.0 if f % 2 == 0 else dims[a] - 1.0) - centre[a]) / units.eta
        ou = _sample_offsets(dims[au], res, centre[au]) / units.eta
        ov = _sample_offsets(dims[av], res, centre[av]) / units.eta
        e_a = np.exp(1j * ks.k[:, a] * r_a)                                   # [n]
        eu = np.exp(1j * np.outer(ou, ks.k[:, au]))                           # [res(u), n]
        ev = np.exp(1j * np.outer(ov, ks.k[:, av]))                           # [res(v), n]
        m = (ev[:, None, :] * eu[None, :, :]) * e_a[None, None, :]            # [v, u, n]
        vals = np.real(cflat @ m.reshape(res * res, -1).T)                   # [(t,c), v*u]
        vals = vals.reshape(T, 3, res, res).transpose(0, 2, 3, 1)            # [t, v, u, c]
        out[:, f] = (vals - tracer.vel[:T, None, None, :]) * units.u_scale
    return out


def initial_field(ks: KSField, tracer: Tracer, dims: tuple[int, int, int], units: UnitMap,
                  index: int = 0) -> np.ndarray:
    """Tracer-frame field w~ on every node at tracer sample ``index``: [nz, ny, nx, 3]."""
    nx, ny, nz = dims
    axes = [(np.arange(d) - (d - 1) / 2.0) / units.eta for d in (nx, ny, nz)]
    tk = float(tracer.times[index])
    g = ks.grid_velocity(tracer.pos[index], tk, axes)
    return (g - tracer.vel[index]) * units.u_scale


# --------------------------------------------------------------------------
# Chains and batch layout
# --------------------------------------------------------------------------
def chain_init(n_beads: int, anchor, gen: np.random.Generator, bond: float = 1.0):
    """Random walk of ``n_beads`` with bond length ``bond`` and uniform directions,
    shifted so that its centre of mass is ``anchor``; velocities zero."""
    steps = gen.standard_normal((max(n_beads - 1, 0), 3))
    steps = bond * steps / np.linalg.norm(steps, axis=1, keepdims=True)
    pos = np.zeros((n_beads, 3))
    if n_beads > 1:
        pos[1:] = np.cumsum(steps, axis=0)
    pos += np.asarray(anchor, dtype=np.float64) - pos.mean(axis=0)
    return pos, np.zeros((n_beads, 3))


def box_sizes(n_boxes: int, gen: np.random.Generator, choices=(32, 48, 64, 96)) -> np.ndarray:
    """Edge lengths drawn uniformly from ``choices``."""
    return np.asarray(gen.choice(np.asarray(choices), size=n_boxes), dtype=np.int64)


def anchors(n: int, box_n: int, gen: np.random.Generator) -> np.ndarray:
    """Chain anchors uniform in [N/4, 3N/4]^3."""
    return gen.uniform(box_n / 4.0, 3.0 * box_n / 4.0, size=(n, 3))


def ks_tracer(config_idx: int, box_idx: int, n_modes: int = 200):
    """The KS field of a box (modes from stream 0) and its tracer's start
    (stream 1, uniform in [-50, 50]^3 Kolmogorov lengths), both spawned per box."""
    base = np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config_idx, 0, box_idx))
    ks = KSField(np.random.Generator(np.random.PCG64(base)), n_modes=n_modes)
    g1 = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config_idx, 1, box_idx))))
    return ks, g1.uniform(-50.0, 50.0, size=3)


def ks_box_inputs(config_idx: int, box_idx: int, n: int, tau: float, n_steps: int,
                  dt: int, res: int, width_eta: float = 2.0, n_modes: int = 200):
    """Everything one KS-driven box needs: (units, initial field, face samples).

    The KS modes of box ``box_idx`` come from stream 0 spawned per box, the
    tracer start from stream 1.  Samples are taken at steps 0, dt, 2 dt, ...
    covering ``n_steps`` (the last sample lies at or beyond n_steps).
    """
    ks, x0 = ks_tracer(config_idx, box_idx, n_modes)
    units = UnitMap(n, tau, width_eta)
    n_samples = -(-n_steps // dt) + 1
    steps = np.arange(n_samples) * dt
    tr = tracer_path(ks, x0, steps / units.tau_eta)
    u0 = initial_field(ks, tr, (n, n, n), units, 0)
    faces = face_samples(ks, tr, (n, n, n), units, res, steps)
    return units, u0, faces


def upsampler_samples(config_idx: int, traj_ids, n: int = 64, tau: float = 0.6, R: int = 8,
                      dt: int = 20, windows=(0, 1), phases=(0, 5, 10, 15), width_eta: float = 2.0,
                      n_modes: int = 200):
    """Samples (face, window k, phase j) of KS tracer trajectories for the upsampler.

    Trajectory ``i`` draws its KS modes from stream 0 and its tracer start from
    stream 1, both spawned per trajectory.  For every listed window k and phase
    j and every face f it returns

      coarse [4][3][R][R]   samples S_{k-1..k+2} of face f on the R x R
                            corner-aligned grid (times clamped at 0),
                            indexed [time][component][v][u]
      theta                 j / dt
      truth  [n][n][3]      the face field at step k dt + j on every face node

    as float32 arrays (coarse [S][4][3][R][R], theta [S], truth [S][n][n][3]),
    samples ordered (trajectory, window, phase, face).
    """
    windows = [int(k) for k in windows]
    phases = [int(j) for j in phases]
    co_list, th_list, tr_list = [], [], []
    for i in traj_ids:
        ks = KSField(np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config_idx, 0, int(i))))), n_modes=n_modes)
        g1 = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence(entropy=ENTROPY, spawn_key=(config_idx, 1, int(i)))))
        x0 = g1.uniform(-50.0, 50.0, size=3)
        units = UnitMap(n, tau, width_eta)
        k_hi = max(windows) + 2
        c_steps = np.arange(k_hi + 1) * dt
        d_steps = np.array([k * dt + j for k in windows for j in phases])
        all_steps = np.unique(np.concatenate([c_steps, d_steps]))
        tr = tracer_path(ks, x0, all_steps / units.tau_eta)

        def sub(steps):
            idx = np.searchsorted(all_steps, steps)
            return Tracer(tr.times[idx], tr.pos[idx], tr.vel[idx])
        coarse = face_samples(ks, sub(c_steps), (n, n, n), units, R, c_steps)      # [K][6][R][R][3]
        dense = face_samples(ks, sub(d_steps), (n, n, n), units, n, d_steps)       # [D][6][n][n][3]
        d = 0
        for k in windows:
            ks_idx = [min(max(k - 1 + tau_i, 0), k_hi) for tau_i in range(4)]
            cw = coarse[ks_idx].transpose(1, 0, 4, 2, 3)                           # [6][4][3][R][R]
            for j in phases:
                for f in range(6):
                    co_list.append(cw[f])
                    th_list.append(j / dt)
                    tr_list.append(dense[d, f])
                d += 1
    return (np.asarray(co_list, dtype=np.float32), np.asarray(th_list, dtype=np.float32),
            np.asarray(tr_list, dtype=np.float32))



# --------------------------------------------------------------------------
# Sub-volume history files (the data-on-disk coupling of the two scales)
# --------------------------------------------------------------------------
def tracer_acceleration(ks: KSField, tracer: Tracer) -> np.ndarray:
    """dv/dt of the tracer, the Lagrangian acceleration du/dt + (u . grad) u of
    the field at its position: [T, 3] in Kolmogorov units."""
    out = np.empty((len(tracer.times), 3))
    for i, (p, t) in enumerate(zip(tracer.pos, tracer.times)):
        g = ks.gradient(p, float(t))
        out[i] = ks.time_derivative(p, float(t)) + g @ ks.velocity(p, float(t))
    return out


def ks_subvolume_history(config_idx: int, box_idx: int, n: int, tau: float, n_steps: int,
                         dt: int, grid: int, width_eta: float = 2.0, n_modes: int = 200):
    """A sub-volume history of a KS tracer box: the tracer-frame velocity on a
    corner-aligned grid of ``grid`` points per edge at steps 0, dt, ... covering
    n_steps, [S][grid][grid][grid][3] as [z][y][x][c] in lattice units, and the
    tracer accelerations [S][3] in lattice units per step."""
    ks, x0 = ks_tracer(config_idx, box_idx, n_modes)
    units = UnitMap(n, tau, width_eta)
    n_samples = -(-n_steps // dt) + 1
    steps = np.arange(n_samples) * dt
    tr = tracer_path(ks, x0, steps / units.tau_eta)
    offs = _sample_offsets(n, grid, (n - 1) / 2.0) / units.eta
    w = np.empty((n_samples, grid, grid, grid, 3))
    for k in range(n_samples):
        g = ks.grid_velocity(tr.pos[k], float(tr.times[k]), [offs, offs, offs])
        w[k] = (g - tr.vel[k]) * units.u_scale
    acc = tracer_acceleration(ks, tr) * units.u_scale / units.tau_eta
    return w, acc


def write_subvolume(path: str, w: np.ndarray, dt: int, t0: int = 0, accel=None) -> None:
    """Writes a sub-volume history file (format version 1, little endian):
    magic "LBSUBVOL", int32 version, grid R, n_samples, dt, int64 t0, int32
    flags (bit 0: accelerations follow), int32 0, float32 w[S][R][R][R][3],
    then float64 accel[S][3] if given."""
    w = np.ascontiguousarray(w, dtype="<f4")
    S, R = w.shape[0], w.shape[1]
    if w.shape != (S, R, R, R, 3):
        raise ValueError("w must be [samples][R][R][R][3]")
    flags = 1 if accel is not None else 0
    with open(path, "wb") as fh:
        fh.write(b"LBSUBVOL")
        fh.write(np.array([1, R, S, dt], dtype="<i4").tobytes())
        fh.write(np.array([t0], dtype="<i8").tobytes())
        fh.write(np.array([flags, 0], dtype="<i4").tobytes())
        fh.write(w.tobytes())
        if accel is not None:
            a = np.ascontiguousarray(accel, dtype="<f8")
            if a.shape != (S, 3):
                raise ValueError("accel must be [samples][3]")
            fh.write(a.tobytes())
