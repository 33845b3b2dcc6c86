"""Batched reconstructions: many independent problems of uneven size in one
persistent launch per window size, and one full-batch gradient-descent
iteration recorded in a hipGraph (include/ptycho.h, ``ptycho_batch_*``).

The caller owns the tensors; the batch keeps raw pointers to them, so the
tensors must stay alive (the ``Batch`` object holds references).
"""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np

from . import _binding as B


class ReconDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("S", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
        ("n", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("slice_stride", ctypes.c_int64), ("ld", ctypes.c_int64),
        ("obj", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("probe", ctypes.c_void_p),
        ("pos", ctypes.c_void_p), ("meas", ctypes.c_void_p),
        ("wavelength_A", ctypes.c_double), ("dz_A", ctypes.c_double), ("pixel_A", ctypes.c_double),
        ("alpha", ctypes.c_double),
    ]


_SIGS = {
    "ptycho_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ReconDesc), ctypes.c_int32,
                                           ctypes.c_int32]),
    "ptycho_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_set_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "ptycho_batch_get_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "ptycho_batch_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "ptycho_batch_update": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_step": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_capture": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_replay": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_history": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "ptycho_batch_reset_history": (ctypes.c_int, [ctypes.c_void_p]),
    "ptycho_batch_stream": (ctypes.c_void_p, [ctypes.c_void_p]),
}


def _lib():
    L = B.lib()
    if not getattr(L, "_batch_sigs", False):
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        L._batch_sigs = True
    return L


class Recon:
    """One reconstruction: device tensors plus physics and step size."""

    def __init__(self, obj, probe, pos, meas, wavelength_A: float, dz_A: float, pixel_A: float, alpha: float,
                 grad=None):
        import torch
        S, H, W, ss, ld = B._obj_geometry(obj)
        M = probe.shape[0]
        B._need(probe, torch.complex64, (M, M), "probe")
        n = B._need_pos(pos)
        B._need(meas, torch.float32, (n, M, M), "meas")
        if grad is None:
            grad = torch.empty_strided(obj.shape, obj.stride(), dtype=torch.complex64, device=obj.device)
        B._on_device(grad, "grad")
        if grad.shape != obj.shape or grad.stride() != obj.stride() or grad.dtype != torch.complex64:
            raise ValueError("grad must have the object's shape and strides")
        self.obj, self.probe, self.pos, self.meas, self.grad = obj, probe, pos, meas, grad
        self.physics = (float(wavelength_A), float(dz_A), float(pixel_A))
        self.alpha = float(alpha)

    def desc(self) -> ReconDesc:
        S, H, W, ss, ld = B._obj_geometry(self.obj)
        d = ReconDesc()
        d.M, d.S, d.H, d.W = self.probe.shape[0], S, H, W
        d.n, d.reserved = self.pos.shape[0], 0
        d.slice_stride, d.ld = ss, ld
        d.obj, d.grad = self.obj.data_ptr(), self.grad.data_ptr()
        d.probe, d.pos, d.meas = self.probe.data_ptr(), self.pos.data_ptr(), self.meas.data_ptr()
        d.wavelength_A, d.dz_A, d.pixel_A = self.physics
        d.alpha = self.alpha
        return d


class Batch:
    def __init__(self, recons: Sequence[Recon], history_rows: int = 64):
        import torch
        self.recons: List[Recon] = list(recons)
        arr = (ReconDesc * max(len(self.recons), 1))(*[r.desc() for r in self.recons])
        torch.cuda.synchronize()  # the tensors were written on torch's streams
        self._h = ctypes.c_void_p()
        B._check(_lib().ptycho_batch_create(ctypes.byref(self._h), arr, len(self.recons), int(history_rows)))
        self.history_rows = int(history_rows)

    def close(self):
        if self._h:
            _lib().ptycho_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream_ptr(self) -> int:
        return int(_lib().ptycho_batch_stream(self._h) or 0)

    def set_grid(self, M: int, grid: int) -> None:
        B._check(_lib().ptycho_batch_set_grid(self._h, int(M), int(grid)))

    def grid(self, M: int) -> int:
        return int(_lib().ptycho_batch_get_grid(self._h, int(M)))

    def _ordered(self, call) -> None:
        """Enqueue a batch call on the batch stream after the work already on the caller's current
        stream (which may have written the tensors the batch reads), and make the caller's stream
        wait for it, so that the caller sees its results in stream order."""
        import torch
        cur = torch.cuda.current_stream()
        bs = torch.cuda.ExternalStream(self.stream_ptr)
        bs.wait_stream(cur)
        B._check(call())
        cur.wait_stream(bs)

    def loss_grad(self, losses=None) -> None:
        """One batched gradient launch; losses (optional float64 [nrecon] device tensor) receives the losses."""
        if losses is not None:
            import torch
            B._need(losses, torch.float64, (len(self.recons),), "losses")
        ptr = ctypes.c_void_p(losses.data_ptr()) if losses is not None else ctypes.c_void_p(0)
        self._ordered(lambda: _lib().ptycho_batch_loss_grad(self._h, ptr))

    def update(self) -> None:
        self._ordered(lambda: _lib().ptycho_batch_update(self._h))

    def step(self) -> None:
        self._ordered(lambda: _lib().ptycho_batch_step(self._h))

    def capture(self) -> None:
        B._check(_lib().ptycho_batch_capture(self._h))

    def replay(self) -> None:
        self._ordered(lambda: _lib().ptycho_batch_replay(self._h))

    def sync(self) -> None:
        B._check(_lib().ptycho_batch_sync(self._h))

    def reset_history(self) -> None:
        B._check(_lib().ptycho_batch_reset_history(self._h))

    def history(self) -> np.ndarray:
        out = np.zeros((self.history_rows, max(len(self.recons), 1)), dtype=np.float64)
        rows = ctypes.c_int32()
        B._check(_lib().ptycho_batch_history(self._h, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rows)))
        return out[: rows.value, : len(self.recons)].copy()
