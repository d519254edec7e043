"""Thin Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice-Boltzmann path runs in the HIP library
``liblbm.so``; this module only converts numpy arrays to pointers and status
codes to exceptions.  PyTorch is optional and used only for device memory
(its caching allocator) and streams.  There is no CPU fallback: if the library
is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

from .build import LIB

Q = 19

OK, ERR_ARG, ERR_OOM, ERR_HIP, ERR_FENE, ERR_BEAD_OUT, ERR_UNSTABLE, ERR_STATE, ERR_BUFSIZE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "LB_OK", -1: "LB_ERR_ARG", -2: "LB_ERR_OOM", -3: "LB_ERR_HIP", -4: "LB_ERR_FENE",
                -5: "LB_ERR_BEAD_OUT", -6: "LB_ERR_UNSTABLE", -7: "LB_ERR_STATE",
                -8: "LB_ERR_BUFSIZE"}
BGK, MRT = 0, 1
STORE_F64, STORE_F32, STORE_F16DEV = 0, 1, 2
BC_AFFINE, BC_SAMPLED, BC_LEARNED = 0, 1, 2
STREAM_AB, STREAM_AA = 0, 1
F_RHO, F_U, F_POP, F_BEAD_POS, F_BEAD_VEL, F_MASS_MOM, F_STEP, F_POP_DEV, F_BEAD_REL, F_VORT = \
    range(10)

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class LbBox(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("periodic_mask", ct.c_uint32)]


class LbConfig(ct.Structure):
    _fields_ = [("n_boxes", ct.c_int32), ("boxes", ct.POINTER(LbBox)), ("collision", ct.c_int),
                ("tau", ct.c_double), ("tau_bulk", ct.c_double), ("ghost_rate", ct.c_double),
                ("storage", ct.c_int), ("rho0", ct.c_double), ("reduce_every", ct.c_int32),
                ("fp16_exp", ct.c_int32), ("stream", ct.c_void_p), ("dev_alloc", ALLOC_FN),
                ("dev_free", FREE_FN), ("alloc_user", ct.c_void_p), ("tune_cache", ct.c_char_p),
                ("graph_steps", ct.c_int32), ("streaming", ct.c_int32)]


class LbBoundary(ct.Structure):
    _fields_ = [("mode", ct.c_int), ("t0", ct.c_int64), ("dt", ct.c_int32),
                ("n_samples", ct.c_int32), ("res", ct.c_int32), ("data", ct.c_void_p),
                ("data_is_f64", ct.c_int32)]


class LbChain(ct.Structure):
    _fields_ = [("n_beads", ct.c_int32), ("md_substeps", ct.c_int32), ("fix_com", ct.c_int32),
                ("zeta", ct.c_double), ("mass", ct.c_double), ("fene_k", ct.c_double),
                ("fene_r0", ct.c_double), ("anchor", ct.c_double * 3)]


EXPORTS = ["lb_init", "lb_set_initial", "lb_set_boundary", "lb_couple_chain", "lb_step",
           "lb_read_fields", "lb_read_sites", "lb_write_state", "lb_sync", "lb_autotune",
           "lb_set_timing", "lb_get_timing", "lb_describe", "lb_last_error", "lb_free",
           "lb_copy_probe", "lb_memcpy_probe", "lb_read_sites_noalloc", "lb_vorticity",
           "lb_set_body_force", "lb_set_thermal", "lb_load_subvolume"]
SUBVOL_INITIAL, SUBVOL_BOUNDARY, SUBVOL_BODY = 1, 2, 4

_lib = None


def load(path: str = LIB):
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ct.CDLL(path)
    vp = ct.c_void_p
    lib.lb_init.argtypes = [ct.POINTER(LbConfig), ct.POINTER(vp)]
    lib.lb_set_initial.argtypes = [vp, ct.c_int32, vp]
    lib.lb_set_boundary.argtypes = [vp, ct.c_int32, ct.POINTER(LbBoundary)]
    lib.lb_couple_chain.argtypes = [vp, ct.c_int32, ct.POINTER(LbChain), vp, vp]
    lib.lb_step.argtypes = [vp, ct.c_int32]
    lib.lb_read_fields.argtypes = [vp, ct.c_int32, ct.c_int, vp, ct.c_size_t, ct.c_int32]
    lib.lb_read_sites.argtypes = [vp, ct.c_int32, ct.c_int32, vp, vp]
    lib.lb_read_sites_noalloc.argtypes = [vp, ct.c_int32, ct.c_int32, vp, vp]
    lib.lb_vorticity.argtypes = [vp, ct.c_int32, ct.c_int32, vp, vp]
    lib.lb_set_body_force.argtypes = [vp, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32, vp]
    lib.lb_set_thermal.argtypes = [vp, ct.c_double, ct.c_uint64]
    lib.lb_load_subvolume.argtypes = [vp, ct.c_int32, ct.c_char_p, ct.c_int32]
    lib.lb_write_state.argtypes = [vp, ct.c_int32, ct.c_int, vp, ct.c_size_t]
    lib.lb_sync.argtypes = [vp]
    lib.lb_autotune.argtypes = [vp, ct.c_int32]
    lib.lb_set_timing.argtypes = [vp, ct.c_int32]
    lib.lb_get_timing.argtypes = [vp, vp]
    lib.lb_describe.argtypes = [vp]
    lib.lb_describe.restype = ct.c_char_p
    lib.lb_last_error.argtypes = [vp]
    lib.lb_last_error.restype = ct.c_char_p
    lib.lb_free.argtypes = [vp]
    lib.lb_free.restype = None
    lib.lb_copy_probe.argtypes = [ct.c_size_t, ct.c_int32, vp]
    lib.lb_memcpy_probe.argtypes = [ct.c_size_t, ct.c_int32, vp]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or ct.c_int
    _lib = lib
    return lib


def copy_probe(nbytes=1 << 30, iters=20) -> float:
    """Measured HBM copy bandwidth (read + write) in GB/s."""
    lib = load()
    out = ct.c_double()
    st = lib.lb_copy_probe(int(nbytes), int(iters), ct.byref(out))
    if st != OK:
        raise LBError(st, "lb_copy_probe failed")
    return out.value


def memcpy_probe(nbytes=1 << 32, iters=10) -> float:
    """The runtime's device-to-device copy (hipMemcpyAsync): (read + write) GB/s."""
    lib = load()
    out = ct.c_double()
    st = lib.lb_memcpy_probe(int(nbytes), int(iters), ct.byref(out))
    if st != OK:
        raise LBError(st, "lb_memcpy_probe failed")
    return out.value


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


class Context:
    """One library context (one or many boxes advanced together)."""

    def __init__(self, boxes, collision=BGK, tau=0.8, tau_bulk=None, ghost_rate=1.0,
                 storage=STORE_F64, rho0=1.0, reduce_every=0, fp16_exp=0, stream=None,
                 torch_alloc=False, tune_cache=None, graph_steps=0, streaming=STREAM_AB):
        self._lib = load()
        self.boxes = [tuple(int(v) for v in b) + ((0,) if len(b) == 3 else ()) for b in boxes]
        arr = (LbBox * len(self.boxes))(*[LbBox(*b) for b in self.boxes])
        self._keep = [arr]
        cfg = LbConfig()
        cfg.n_boxes = len(self.boxes)
        cfg.boxes = ct.cast(arr, ct.POINTER(LbBox))
        cfg.collision = collision
        cfg.tau = tau
        cfg.tau_bulk = tau if tau_bulk is None else tau_bulk
        cfg.ghost_rate = ghost_rate
        cfg.storage = storage
        cfg.rho0 = rho0
        cfg.reduce_every = reduce_every
        cfg.fp16_exp = fp16_exp
        cfg.stream = stream
        cfg.graph_steps = graph_steps
        cfg.streaming = streaming
        if tune_cache:
            self._tc = tune_cache.encode()
            cfg.tune_cache = self._tc
        if torch_alloc:
            import torch
            dev = torch.cuda.current_device()

            alloc, delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

            def _alloc(n, user):
                return alloc(int(n), dev)

            def _free(ptr, user):
                try:
                    delete(ptr)
                except Exception:  # interpreter shutdown: the process frees everything
                    pass
            self._cb = (ALLOC_FN(_alloc), FREE_FN(_free))
            cfg.dev_alloc, cfg.dev_free = self._cb
        h = ct.c_void_p()
        st = self._lib.lb_init(ct.byref(cfg), ct.byref(h))
        if st != OK:
            raise LBError(st, "lb_init failed")
        self._h = h
        self.storage = storage

    # -- lifecycle ----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.lb_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != OK:
            raise LBError(st, self._lib.lb_last_error(self._h).decode())
        return st

    def shape(self, box):
        nx, ny, nz, _ = self.boxes[box]
        return (nz, ny, nx)

    # -- inputs -------------------------------------------------------------
    def set_initial(self, box, u=None):
        if u is None:
            return self._check(self._lib.lb_set_initial(self._h, box, None))
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape(box) + (3,))
        return self._check(self._lib.lb_set_initial(self._h, box, _p(u)))

    def set_boundary(self, box, mode, data, t0=0, dt=1, res=0):
        if mode == BC_LEARNED:
            # a float32 CUDA tensor [n_slots][6][res][res][3], read in place by
            # the library: the caller keeps it alive and refills it
            import torch
            if not (isinstance(data, torch.Tensor) and data.is_cuda and data.dtype == torch.float32
                    and data.is_contiguous() and data.dim() == 5):
                raise TypeError("a learned boundary ring is a contiguous float32 CUDA tensor "
                                "[n_slots][6][res][res][3]")
            bc = LbBoundary(mode, t0, dt, data.shape[0], res or data.shape[2],
                            ct.c_void_p(data.data_ptr()), 0)
            self._ring = data
            return self._check(self._lib.lb_set_boundary(self._h, box, ct.byref(bc)))
        f64 = mode == BC_AFFINE or np.asarray(data).dtype == np.float64
        data = np.ascontiguousarray(data, dtype=np.float64 if f64 else np.float32)
        bc = LbBoundary(mode, t0, dt, data.shape[0], res, _p(data), 1 if f64 else 0)
        return self._check(self._lib.lb_set_boundary(self._h, box, ct.byref(bc)))

    def couple_chain(self, box, pos, vel=None, substeps=10, fix_com=True, zeta=5.0, mass=1.0,
                     fene_k=1.0, fene_r0=2.0, anchor=None):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        if anchor is None:
            anchor = pos.mean(axis=0)
        ch = LbChain(pos.shape[0], substeps, int(fix_com), zeta, mass, fene_k, fene_r0,
                     (ct.c_double * 3)(*[float(a) for a in anchor]))
        v = None
        if vel is not None:
            vel = np.ascontiguousarray(vel, dtype=np.float64)
            v = _p(vel)
        return self._check(self._lib.lb_couple_chain(self._h, box, ct.byref(ch), _p(pos), v))

    def set_body_force(self, box, accel, t0=0, dt=1):
        """Tracer acceleration samples [n][3] (lattice units); None removes it."""
        if accel is None:
            return self._check(self._lib.lb_set_body_force(self._h, box, 0, 1, 0, None))
        a = np.ascontiguousarray(accel, dtype=np.float64).reshape(-1, 3)
        return self._check(self._lib.lb_set_body_force(self._h, box, int(t0), int(dt), a.shape[0],
                                                       _p(a)))

    def load_subvolume(self, box, path, what=SUBVOL_INITIAL | SUBVOL_BOUNDARY):
        """Apply a sub-volume history file (format in include/lbm.h) to a box."""
        return self._check(self._lib.lb_load_subvolume(self._h, box, str(path).encode(), int(what)))

    def set_thermal(self, kT, seed=0):
        return self._check(self._lib.lb_set_thermal(self._h, float(kT), int(seed)))

    # -- stepping -----------------------------------------------------------
    def step(self, n=1):
        return self._check(self._lib.lb_step(self._h, int(n)))

    def step_status(self, n=1) -> int:
        return self._lib.lb_step(self._h, int(n))

    def sync(self):
        return self._check(self._lib.lb_sync(self._h))

    def sync_status(self) -> int:
        return self._lib.lb_sync(self._h)

    def autotune(self, trials=3):
        return self._check(self._lib.lb_autotune(self._h, trials))

    def set_timing(self, on=True):
        return self._check(self._lib.lb_set_timing(self._h, 1 if on else 0))

    def timing(self):
        out = np.zeros(4)
        self._check(self._lib.lb_get_timing(self._h, _p(out)))
        return out

    def describe(self) -> str:
        return self._lib.lb_describe(self._h).decode()

    def last_error(self) -> str:
        return self._lib.lb_last_error(self._h).decode()

    # -- readout ------------------------------------------------------------
    def _read(self, box, field, shape, dtype=np.float64, strict=True):
        out = np.zeros(shape, dtype=dtype)
        st = self._lib.lb_read_fields(self._h, box, field, _p(out), out.nbytes, 0)
        if strict:
            self._check(st)
        return out, st

    def n_beads(self, box):
        return self._nbeads.get(box, 0) if hasattr(self, "_nbeads") else 0

    def read(self, box, field, n_beads=0, strict=True):
        if field in (F_POP, F_POP_DEV):
            shp = (Q,) + self.shape(box)
        elif field in (F_RHO, F_VORT):
            shp = self.shape(box)
        elif field == F_U:
            shp = self.shape(box) + (3,)
        elif field in (F_BEAD_POS, F_BEAD_VEL, F_BEAD_REL):
            shp = (n_beads, 3)
        elif field == F_MASS_MOM:
            shp = (5,)
        elif field == F_STEP:
            out, st = self._read(0, F_STEP, (1,), np.int64, strict)
            return int(out[0]) if strict else (int(out[0]), st)
        else:
            raise ValueError(field)
        out, st = self._read(box, field, shp, strict=strict)
        return out if strict else (out, st)

    def read_sites(self, box, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        out = np.zeros((xyz.shape[0], Q))
        self._check(self._lib.lb_read_sites(self._h, box, xyz.shape[0], _p(xyz), _p(out)))
        return out

    def vorticity(self, box, volumes):
        """Mean |curl u| over control volumes [(lo_xyz, hi_xyz), ...] (inclusive)."""
        vol = np.ascontiguousarray([list(lo) + list(hi) for lo, hi in volumes],
                                   dtype=np.int32).reshape(-1, 6)
        out = np.zeros(vol.shape[0])
        self._check(self._lib.lb_vorticity(self._h, box, vol.shape[0], _p(vol), _p(out)))
        return out

    def read_sites_noalloc(self, box, xyz, strict=True):
        """lb_read_sites_noalloc: the same readout staged in the library's
        static device array (no device allocation; at most 32768 sites)."""
        xyz = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
        out = np.zeros((xyz.shape[0], Q))
        st = self._lib.lb_read_sites_noalloc(self._h, box, xyz.shape[0], _p(xyz), _p(out))
        if strict:
            self._check(st)
            return out
        return out, st

    def write_state(self, box, field, data):
        if field == F_STEP:
            arr = np.asarray([int(data)], dtype=np.int64)
        else:
            arr = np.ascontiguousarray(data, dtype=np.float64)
        return self._check(self._lib.lb_write_state(self._h, box, field, _p(arr), arr.nbytes))
