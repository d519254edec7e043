"""Thin Python binding of the learned-boundary upsampler ABI (include/lbnet.h).

Argument marshalling only: every step of the network (lift, convolutions,
loss, backward passes, Adam) runs in the HIP kernels of ``liblbm.so``.  Device
tensors are passed as torch CUDA tensors (float32, contiguous) whose pointers
go to the library unchanged; host parameter vectors are numpy float32 arrays.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import lbm

IMG = 64
PARAM_COUNT = 47363
IN_CH, HIDDEN, OUT_CH = 15, 64, 3
(BUF_LIFT, BUF_A1, BUF_A2, BUF_R, BUF_BASE, BUF_SCALE) = range(6)

EXPORTS = ["lbn_init", "lbn_set_params", "lbn_get_params", "lbn_forward", "lbn_window_forward",
           "lbn_loss_grad", "lbn_adam_step", "lbn_read_buffer", "lbn_sync", "lbn_last_error",
           "lbn_free"]


class LbnConfig(ct.Structure):
    _fields_ = [("coarse", ct.c_int32), ("max_batch", ct.c_int32), ("stream", ct.c_void_p),
                ("dev_alloc", lbm.ALLOC_FN), ("dev_free", lbm.FREE_FN), ("alloc_user", ct.c_void_p)]


_bound = False


def _lib():
    global _bound
    lib = lbm.load()
    if not _bound:
        vp = ct.c_void_p
        lib.lbn_init.argtypes = [ct.POINTER(LbnConfig), ct.POINTER(vp)]
        lib.lbn_set_params.argtypes = [vp, vp, ct.c_size_t]
        lib.lbn_get_params.argtypes = [vp, vp, ct.c_size_t]
        lib.lbn_forward.argtypes = [vp, vp, vp, ct.c_int32, vp]
        lib.lbn_window_forward.argtypes = [vp, vp, ct.c_int32, ct.c_int32, ct.c_int32, vp]
        lib.lbn_loss_grad.argtypes = [vp, vp, vp, vp, ct.c_int32, ct.POINTER(ct.c_double), vp]
        lib.lbn_adam_step.argtypes = [vp, ct.c_float, ct.c_float, ct.c_float, ct.c_float]
        lib.lbn_read_buffer.argtypes = [vp, ct.c_int32, ct.c_int32, vp, ct.c_size_t]
        lib.lbn_sync.argtypes = [vp]
        lib.lbn_last_error.argtypes = [vp]
        lib.lbn_last_error.restype = ct.c_char_p
        lib.lbn_free.argtypes = [vp]
        lib.lbn_free.restype = None
        for name in EXPORTS:
            if name not in ("lbn_last_error", "lbn_free"):
                getattr(lib, name).restype = ct.c_int
        _bound = True
    return lib


def _dev(t, shape=None, name="tensor"):
    """Pointer of a contiguous float32 CUDA tensor (shape checked)."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ct.c_void_p(t.data_ptr())


class Upsampler:
    """One network context: parameters, optimiser state and work buffers."""

    def __init__(self, coarse=8, max_batch=128, stream=None, torch_alloc=True):
        """``stream`` defaults to torch's current stream, so the device tensors
        passed to the calls are ordered with the network's kernels."""
        self._lib = _lib()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.coarse = int(coarse)
        self.max_batch = int(max_batch)
        cfg = LbnConfig()
        cfg.coarse = self.coarse
        cfg.max_batch = self.max_batch
        cfg.stream = stream
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
            self._cb = (lbm.ALLOC_FN(_alloc), lbm.FREE_FN(_free))
            cfg.dev_alloc, cfg.dev_free = self._cb
        h = ct.c_void_p()
        st = self._lib.lbn_init(ct.byref(cfg), ct.byref(h))
        if st != lbm.OK:
            raise lbm.LBError(st, "lbn_init failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != lbm.OK:
            raise lbm.LBError(st, self._lib.lbn_last_error(self._h).decode())

    # -- parameters -----------------------------------------------------------
    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        self._check(self._lib.lbn_set_params(self._h, lbm._p(p), p.size))

    def params(self) -> np.ndarray:
        out = np.zeros(PARAM_COUNT, np.float32)
        self._check(self._lib.lbn_get_params(self._h, lbm._p(out), out.size))
        return out

    # -- compute ----------------------------------------------------------------
    def forward(self, coarse, theta, out):
        b = coarse.shape[0]
        R = self.coarse
        self._check(self._lib.lbn_forward(self._h, _dev(coarse, (b, 4, 3, R, R), "coarse"),
                                          _dev(theta, (b,), "theta"), b,
                                          _dev(out, (b, IMG, IMG, 3), "out")))

    def window_forward(self, samples, k, dt, ring):
        ns = samples.shape[0]
        R = self.coarse
        self._check(self._lib.lbn_window_forward(self._h, _dev(samples, (ns, 6, R, R, 3), "samples"),
                                                 ns, int(k), int(dt),
                                                 _dev(ring, (dt, 6, IMG, IMG, 3), "ring")))

    def loss_grad(self, coarse, theta, truth, want_loss=True, want_grad=False):
        b = coarse.shape[0]
        R = self.coarse
        loss = ct.c_double(np.nan)
        grad = np.zeros(PARAM_COUNT, np.float32) if want_grad else None
        self._check(self._lib.lbn_loss_grad(
            self._h, _dev(coarse, (b, 4, 3, R, R), "coarse"), _dev(theta, (b,), "theta"),
            _dev(truth, (b, IMG, IMG, 3), "truth"), b, ct.byref(loss) if want_loss else None,
            lbm._p(grad) if want_grad else None))
        return (loss.value if want_loss else None), grad

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self._lib.lbn_adam_step(self._h, lr, beta1, beta2, eps))

    def train_step(self, coarse, theta, truth, lr=1e-3, want_loss=False, **adam):
        loss, _ = self.loss_grad(coarse, theta, truth, want_loss=want_loss)
        self.adam_step(lr, **adam)
        return loss

    def read_buffer(self, which, batch) -> np.ndarray:
        shapes = {BUF_LIFT: (batch, IMG, IMG, 16), BUF_A1: (batch, IMG, IMG, HIDDEN),
                  BUF_A2: (batch, IMG, IMG, HIDDEN), BUF_R: (batch, IMG, IMG, 16),
                  BUF_BASE: (batch, IMG, IMG, 3), BUF_SCALE: (batch,)}
        out = np.zeros(shapes[which], np.float32)
        self._check(self._lib.lbn_read_buffer(self._h, which, batch, lbm._p(out), out.size))
        return out

    def sync(self):
        self._check(self._lib.lbn_sync(self._h))


def split_params(p):
    """Views of the parameter vector: (W1, b1, W2, b2, W3, b3), W as [co][ci][3][3]."""
    p = np.asarray(p)
    out, o = [], 0
    for co, ci in ((HIDDEN, IN_CH), (HIDDEN, HIDDEN), (OUT_CH, HIDDEN)):
        n = co * ci * 9
        out.append(p[o:o + n].reshape(co, ci, 3, 3))
        o += n
        out.append(p[o:o + co])
        o += co
    assert o == PARAM_COUNT
    return tuple(out)


def init_params(seed=0):
    """He-normal weights for the two ReLU layers, zero biases and a zero last
    layer, so that the untrained network returns the plain interpolation
    (seeded; the host side of the parameter initialisation)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=0x08094958, spawn_key=(9, seed))))
    parts = []
    for co, ci, gain in ((HIDDEN, IN_CH, np.sqrt(2.0)), (HIDDEN, HIDDEN, np.sqrt(2.0)), (OUT_CH, HIDDEN, 0.0)):
        parts.append((rng.standard_normal((co, ci, 3, 3)) * gain / np.sqrt(ci * 9)).reshape(-1))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
