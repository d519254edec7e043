"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

:func:`build` compiles ``lb_oracle.c`` with gcc (``-O2 -fopenmp``, no fast-math)
into ``liblboracle.so`` next to this file.  :class:`OracleBox` wraps one box.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "liblboracle.so")

OK, ERR_ARG, ERR_OOM, ERR_FENE, ERR_BEAD_OUT, ERR_UNSTABLE, ERR_STATE = 0, -1, -2, -4, -5, -6, -7
BGK, MRT = 0, 1
BC_AFFINE, BC_SAMPLED = 0, 1
Q = 19


def build(force: bool = True) -> str:
    """Compile the oracle shared library; returns its path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("periodic_mask", ct.c_uint), ("collision", ct.c_int),
                ("tau", ct.c_double), ("tau_bulk", ct.c_double), ("ghost_rate", ct.c_double),
                ("rho0", ct.c_double), ("reduce_every", ct.c_int)]


_lib = None
_dp = ct.POINTER(ct.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ct.CDLL(LIB)
        lib.or_create.restype = ct.c_void_p
        lib.or_create.argtypes = [ct.POINTER(_Params)]
        lib.or_destroy.argtypes = [ct.c_void_p]
        lib.or_set_initial.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_set_populations.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_set_boundary.argtypes = [ct.c_void_p, ct.c_int, ct.c_long, ct.c_int, ct.c_int,
                                        ct.c_int, ct.c_void_p]
        lib.or_add_chain.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_double,
                                     ct.c_double, ct.c_double, ct.c_double, ct.c_void_p,
                                     ct.c_void_p, ct.c_void_p]
        lib.or_step.argtypes = [ct.c_void_p, ct.c_int]
        lib.or_get_step.restype = ct.c_long
        lib.or_get_step.argtypes = [ct.c_void_p]
        lib.or_get_error.argtypes = [ct.c_void_p, ct.POINTER(ct.c_int), ct.POINTER(ct.c_long)]
        lib.or_boundary_velocity.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_long,
                                             ct.c_void_p]
        lib.or_read_pop.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_read_rho_u.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.or_n_beads.argtypes = [ct.c_void_p]
        lib.or_read_beads.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.or_read_mass_mom.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_read_last_force.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_set_body_force.argtypes = [ct.c_void_p, ct.c_long, ct.c_int, ct.c_int, ct.c_void_p]
        lib.or_set_thermal.argtypes = [ct.c_void_p, ct.c_double, ct.c_ulonglong, ct.c_uint]
        lib.or_philox4x32.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.or_unit_uniform.argtypes = [ct.c_uint]
        lib.or_unit_uniform.restype = ct.c_double
        lib.or_collide_noise.argtypes = [ct.POINTER(_Params), ct.c_void_p, ct.c_void_p, ct.c_double,
                                         ct.c_void_p, ct.c_void_p]
        lib.or_chain_md_noise.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double,
                                          ct.c_double, ct.c_double, ct.c_void_p, ct.c_void_p,
                                          ct.c_void_p, ct.c_void_p, ct.c_double, ct.c_void_p,
                                          ct.c_void_p]
        lib.or_vorticity.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_vorticity_mean.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.or_lattice.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_threads.restype = ct.c_int
        lib.or_mrt_basis.argtypes = [ct.c_void_p, ct.c_void_p]
        lib.or_equilibrium.argtypes = [ct.c_double, ct.c_void_p, ct.c_void_p]
        lib.or_collide.argtypes = [ct.POINTER(_Params), ct.c_void_p, ct.c_void_p, ct.c_void_p]
        lib.or_chain_md.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_double, ct.c_double,
                                    ct.c_double, ct.c_double, ct.c_void_p, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p, ct.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def threads() -> int:
    """OpenMP threads the oracle's steps use."""
    return int(_load().or_threads())


def lattice():
    """(c[19,3] int, w[19]) in the library's direction order."""
    lib = _load()
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    lib.or_lattice(_ptr(c), _ptr(w))
    return c.astype(np.int64), w


def mrt_basis():
    """(E[19,19] with E[k,i] = e_k(c_i), b[19] norms)."""
    lib = _load()
    e = np.zeros((Q, Q))
    b = np.zeros(Q)
    lib.or_mrt_basis(_ptr(e), _ptr(b))
    return e, b


def _params(nx=1, ny=1, nz=1, periodic_mask=7, collision=BGK, tau=0.8, tau_bulk=None,
            ghost_rate=1.0, rho0=1.0, reduce_every=0) -> _Params:
    return _Params(nx, ny, nz, periodic_mask, collision, tau,
                   tau if tau_bulk is None else tau_bulk, ghost_rate, rho0, reduce_every)


def equilibrium(rho: float, u) -> np.ndarray:
    lib = _load()
    out = np.zeros(Q)
    lib.or_equilibrium(float(rho), _ptr(_f64(u)), _ptr(out))
    return out


def collide(f, g=(0.0, 0.0, 0.0), **kw) -> np.ndarray:
    """Post-collision populations of one node (kwargs: collision, tau, tau_bulk, ghost_rate)."""
    lib = _load()
    p = _params(**kw)
    out = np.zeros(Q)
    lib.or_collide(ct.byref(p), _ptr(_f64(f)), _ptr(_f64(g)), _ptr(out))
    return out


def chain_md(pos, vel, ubead, substeps=10, fix_com=False, zeta=5.0, mass=1.0, fene_k=1.0,
             fene_r0=2.0, anchor=(0.0, 0.0, 0.0)):
    """One LB step of chain dynamics; returns (status, pos, vel, dp)."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    ub = _f64(ubead)
    nb = pos.shape[0]
    dp = np.zeros((nb, 3))
    st = lib.or_chain_md(nb, substeps, int(fix_com), zeta, mass, fene_k, fene_r0,
                         _ptr(_f64(anchor)), _ptr(pos), _ptr(vel), _ptr(ub), _ptr(dp))
    return st, pos, vel, dp


def philox(ctr, key):
    """Philox4x32-10 of a 128-bit counter under a 64-bit key: four uint32."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32(_ptr(c), _ptr(k), _ptr(out))
    return out


def unit_uniform(u) -> float:
    """32 random bits -> uniform on (-sqrt 3, sqrt 3) (mean 0, variance 1)."""
    return float(_load().or_unit_uniform(int(u)))


def collide_noise(f, g, mu, r, **kw) -> np.ndarray:
    """Fluctuating MRT collision of one node: mu = 3 kT, r[19] (modes k >= 4 used)."""
    lib = _load()
    p = _params(**kw)
    out = np.zeros(Q)
    lib.or_collide_noise(ct.byref(p), _ptr(_f64(f)), _ptr(_f64(g)), float(mu), _ptr(_f64(r)),
                         _ptr(out))
    return out


def chain_md_noise(pos, vel, ubead, kT, rnd, substeps=10, fix_com=False, zeta=5.0, mass=1.0,
                   fene_k=1.0, fene_r0=2.0, anchor=(0.0, 0.0, 0.0)):
    """chain_md with Langevin noise: rnd[substeps][nb][3] unit-variance numbers."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    nb = pos.shape[0]
    dp = np.zeros((nb, 3))
    st = lib.or_chain_md_noise(nb, substeps, int(fix_com), zeta, mass, fene_k, fene_r0,
                               _ptr(_f64(anchor)), _ptr(pos), _ptr(vel), _ptr(_f64(ubead)),
                               float(kT), _ptr(_f64(rnd)), _ptr(dp))
    return st, pos, vel, dp


class OracleBox:
    """One lattice box: ``dims`` = (nx, ny, nz) nodes including the boundary layer."""

    def __init__(self, dims, collision=BGK, tau=0.8, tau_bulk=None, ghost_rate=1.0, rho0=1.0,
                 periodic_mask=0, reduce_every=0):
        self._lib = _load()
        self.dims = tuple(int(d) for d in dims)
        nx, ny, nz = self.dims
        self.params = _params(nx, ny, nz, periodic_mask, collision, tau, tau_bulk, ghost_rate,
                              rho0, reduce_every)
        self._h = self._lib.or_create(ct.byref(self.params))
        if not self._h:
            raise ValueError("oracle: invalid box parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    @property
    def shape(self):
        nx, ny, nz = self.dims
        return (nz, ny, nx)

    def set_initial(self, u=None):
        if u is None:
            return self._lib.or_set_initial(self._h, None)
        return self._lib.or_set_initial(self._h, _ptr(_f64(u, self.shape + (3,))))

    def set_populations(self, f):
        return self._lib.or_set_populations(self._h, _ptr(_f64(f, (Q,) + self.shape)))

    def set_boundary(self, mode, data, t0=0, dt=1, res=0):
        data = _f64(data)
        ns = data.shape[0]
        return self._lib.or_set_boundary(self._h, mode, t0, dt, ns, res, _ptr(data))

    def add_chain(self, pos, vel=None, substeps=10, fix_com=True, zeta=5.0, mass=1.0,
                  fene_k=1.0, fene_r0=2.0, anchor=None):
        pos = _f64(pos)
        if anchor is None:
            anchor = pos.mean(axis=0)
        v = None if vel is None else _ptr(_f64(vel))
        return self._lib.or_add_chain(self._h, pos.shape[0], substeps, int(fix_com), zeta, mass,
                                      fene_k, fene_r0, _ptr(_f64(anchor)), _ptr(pos), v)

    def set_body_force(self, accel, t0=0, dt=1):
        """Tracer acceleration samples [n][3] (lattice units); None clears."""
        if accel is None:
            return self._lib.or_set_body_force(self._h, 0, 1, 0, None)
        a = _f64(accel).reshape(-1, 3)
        return self._lib.or_set_body_force(self._h, t0, dt, a.shape[0], _ptr(a))

    def set_thermal(self, kT, seed=0, box_index=0):
        return self._lib.or_set_thermal(self._h, float(kT), int(seed), int(box_index))

    def step(self, n=1) -> int:
        return self._lib.or_step(self._h, int(n))

    @property
    def step_index(self) -> int:
        return int(self._lib.or_get_step(self._h))

    def error(self):
        code = ct.c_int()
        st = ct.c_long()
        self._lib.or_get_error(self._h, ct.byref(code), ct.byref(st))
        return code.value, st.value

    def boundary_velocity(self, x, y, z, n):
        out = np.zeros(3)
        st = self._lib.or_boundary_velocity(self._h, x, y, z, n, _ptr(out))
        return st, out

    def pop(self) -> np.ndarray:
        out = np.zeros((Q,) + self.shape)
        self._lib.or_read_pop(self._h, _ptr(out))
        return out

    def rho_u(self):
        rho = np.zeros(self.shape)
        u = np.zeros(self.shape + (3,))
        self._lib.or_read_rho_u(self._h, _ptr(rho), _ptr(u))
        return rho, u

    def beads(self):
        n = self._lib.or_n_beads(self._h)
        pos = np.zeros((n, 3))
        vel = np.zeros((n, 3))
        self._lib.or_read_beads(self._h, _ptr(pos), _ptr(vel))
        return pos, vel

    def mass_mom(self) -> np.ndarray:
        out = np.zeros(5)
        self._lib.or_read_mass_mom(self._h, _ptr(out))
        return out

    def last_force(self) -> np.ndarray:
        out = np.zeros(self.shape + (3,))
        self._lib.or_read_last_force(self._h, _ptr(out))
        return out

    def vorticity(self):
        """(|curl u| [nz, ny, nx] by central differences, 0 where undefined;
        number of nodes where it is defined)."""
        out = np.zeros(self.shape)
        n = self._lib.or_vorticity(self._h, _ptr(out))
        return out, int(n)

    def vorticity_mean(self, lo, hi) -> float:
        """Mean |curl u| over the node range lo..hi (inclusive, x y z)."""
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        hi = np.ascontiguousarray(hi, dtype=np.int32)
        out = ct.c_double()
        st = self._lib.or_vorticity_mean(self._h, _ptr(lo), _ptr(hi), ct.byref(out))
        if st != OK:
            raise ValueError("vorticity is not defined on every node of the range")
        return out.value

    def interior_mask(self) -> np.ndarray:
        """Boolean [nz, ny, nx] mask of evolved (interior) nodes."""
        nx, ny, nz = self.dims
        m = np.ones(self.shape, dtype=bool)
        pm = self.params.periodic_mask
        for a, n in enumerate((nx, ny, nz)):
            if (pm >> a) & 1:
                continue
            sl = [slice(None)] * 3
            ax = 2 - a
            sl[ax] = 0
            m[tuple(sl)] = False
            sl[ax] = n - 1
            m[tuple(sl)] = False
        return m
