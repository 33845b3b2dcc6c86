"""Thin ctypes binding of libptycho.so (include/ptycho.h).

Only argument marshalling lives here: tensors are turned into raw device
pointers and strides, and every computation runs in the HIP library.  The
library must be built (``python -m paper_2205_06327_amd.build``); if it is
missing, every call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptycho.so")

PTYCHO_OK = 0
PTYCHO_ACCUMULATE = 1
ERRORS = {
    -1: "PTYCHO_E_ARG",
    -2: "PTYCHO_E_SHAPE",
    -3: "PTYCHO_E_BOUNDS",
    -4: "PTYCHO_E_HALO",
    -5: "PTYCHO_E_ASSIGN",
    -6: "PTYCHO_E_UNSUPPORTED",
    -7: "PTYCHO_E_HIP",
    -8: "PTYCHO_E_NOMEM",
    -9: "PTYCHO_E_CAPACITY",
}
class TileDesc(ctypes.Structure):
    """ptycho_tile_desc: a tile, its extended box and its gradient buffer."""
    _fields_ = [("ty0", ctypes.c_int32), ("ty1", ctypes.c_int32), ("tx0", ctypes.c_int32), ("tx1", ctypes.c_int32),
                ("ey0", ctypes.c_int32), ("ex0", ctypes.c_int32), ("eh", ctypes.c_int32), ("ew", ctypes.c_int32),
                ("grad", ctypes.c_void_p)]


EXPORTED = (
    "ptycho_create", "ptycho_destroy", "ptycho_set_stream", "ptycho_reserve", "ptycho_workspace_bytes",
    "ptycho_forward", "ptycho_loss_grad", "ptycho_tile_grad", "ptycho_bin_positions",
    "ptycho_validate_positions", "ptycho_tile_box", "ptycho_check", "ptycho_last_error", "ptycho_version",
    "ptycho_tile_accumulate", "ptycho_profile_enable", "ptycho_profile_read", "ptycho_zero_gradient",
    "ptycho_loss", "ptycho_batch_create", "ptycho_batch_destroy", "ptycho_batch_set_grid", "ptycho_batch_get_grid",
    "ptycho_batch_loss_grad", "ptycho_batch_update", "ptycho_batch_step", "ptycho_batch_capture",
    "ptycho_batch_replay", "ptycho_batch_sync", "ptycho_batch_history", "ptycho_batch_reset_history",
    "ptycho_batch_stream", "ptycho_box_exchange", "ptycho_set_checkpoint",
    "ptycho_box_axpy", "ptycho_potential_transmission", "ptycho_potential_gradient", "ptycho_loss_grad_probe",
    "ptycho_copy_box", "ptycho_tiles_grad", "ptycho_shift_probes", "ptycho_forward_stack",
    "ptycho_loss_grad_stack", "ptycho_loss_stack", "ptycho_tiles_grad_stack", "ptycho_gd_step_size",
    "ptycho_loss_grad_static",
)


class PtychoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


_lib = None

c_i32, c_i64, c_u32, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p
P_i32 = ctypes.POINTER(ctypes.c_int32)


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2205_06327_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "ptycho_create": (ctypes.c_int, [ctypes.POINTER(c_vp), c_i32, c_i32, c_dbl, c_dbl, c_dbl, c_i32, c_vp]),
            "ptycho_destroy": (ctypes.c_int, [c_vp]),
            "ptycho_set_stream": (ctypes.c_int, [c_vp, c_vp]),
            "ptycho_reserve": (ctypes.c_int, [c_vp, c_i32]),
            "ptycho_workspace_bytes": (c_i64, [c_vp]),
            "ptycho_forward": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_i32, c_vp]),
            "ptycho_loss_grad_static": (ctypes.c_int, [c_i32, c_i32, c_dbl, c_dbl, c_dbl, c_vp, c_vp, c_i32, c_i32,
                                                         c_i64, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                                                         c_i64, c_i32, c_u32, c_vp]),
            "ptycho_loss_grad": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_i32, c_vp,
                                                c_vp, c_vp, c_vp, c_i64, c_i32, c_u32, c_vp]),
            "ptycho_loss_grad_probe": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_i32,
                                                      c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_vp, c_u32, c_vp]),
            "ptycho_loss": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_vp, c_i32, c_vp,
                                           c_vp, c_vp, c_u32]),
            "ptycho_tile_grad": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i64, c_i32, c_i32, c_i32,
                                                c_i32, c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp,
                                                c_vp, c_vp, c_u32]),
            "ptycho_bin_positions": (ctypes.c_int, [P_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, P_i32]),
            "ptycho_validate_positions": (ctypes.c_int, [P_i32, c_i32, c_i32, c_i32, c_i32]),
            "ptycho_tile_box": (ctypes.c_int, [c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32] + [P_i32] * 8),
            "ptycho_gd_step_size": (ctypes.c_int, [c_vp, c_i32, P_i32, c_i32, c_i32, c_i32, c_i32,
                                                   ctypes.POINTER(c_dbl)]),
            "ptycho_check": (ctypes.c_int, [c_vp, ctypes.POINTER(c_u32)]),
            "ptycho_tile_accumulate": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i32, c_i32, c_i32, c_i32, c_vp,
                                                      c_i64, c_i32]),
            "ptycho_profile_enable": (ctypes.c_int, [c_vp, c_i32]),
            "ptycho_zero_gradient": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32]),
            "ptycho_set_checkpoint": (ctypes.c_int, [c_vp, c_i32]),
            "ptycho_shift_probes": (ctypes.c_int, [c_vp, c_vp, c_vp, c_i32, c_vp]),
            "ptycho_forward_stack": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_i64, c_vp, c_i32,
                                                    c_vp]),
            "ptycho_tiles_grad_stack": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, ctypes.POINTER(TileDesc),
                                                       c_i32, c_i32, c_vp, c_vp, c_i64, c_vp, c_i32, c_vp, c_vp, c_vp,
                                                       c_u32]),
            "ptycho_loss_stack": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_i64, c_vp, c_i32,
                                                 c_vp, c_vp, c_vp, c_u32]),
            "ptycho_loss_grad_stack": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, c_vp, c_i64, c_vp,
                                                      c_i32, c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_u32, c_vp]),
            "ptycho_copy_box": (ctypes.c_int, [c_vp, c_i32, c_i32, c_i32, c_vp, c_i64, c_i32, c_vp, c_i64, c_i32]),
            "ptycho_tiles_grad": (ctypes.c_int, [c_vp, c_vp, c_i32, c_i32, c_i64, c_i32, ctypes.POINTER(TileDesc),
                                                 c_i32, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_u32]),
            "ptycho_potential_transmission": (ctypes.c_int, [c_vp, c_i32, c_i32, ctypes.c_float, c_vp, c_i64, c_i32,
                                                             c_vp, c_i64, c_i32]),
            "ptycho_potential_gradient": (ctypes.c_int, [c_vp, c_i32, c_i32, ctypes.c_float, c_vp, c_i64, c_i32,
                                                         c_vp, c_i64, c_i32, c_vp, c_i64, c_i32]),
            "ptycho_box_axpy": (ctypes.c_int, [c_vp, c_i32, ctypes.c_float, c_vp, c_i32, c_i32, c_i32, c_i32, c_i64,
                                               c_i32, c_vp, c_i32, c_i32, c_i32, c_i32, c_i64, c_i32]),
            "ptycho_box_exchange": (ctypes.c_int, [c_vp, c_i32, c_vp, c_i32, c_i32, c_i32, c_i32, c_i64, c_i32,
                                                   c_vp, c_i32, c_i32, c_i32, c_i32, c_i64, c_i32, c_u32]),
            "ptycho_profile_read": (ctypes.c_int, [c_vp, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64),
                                                   ctypes.POINTER(c_i64)]),
            "ptycho_last_error": (ctypes.c_char_p, []),
            "ptycho_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != PTYCHO_OK:
        raise PtychoError(rc, lib().ptycho_last_error().decode())


def version() -> str:
    return lib().ptycho_version().decode()


# ---------------------------------------------------------------------------
# host helpers (numpy int32 [n, 2])
# ---------------------------------------------------------------------------
def _pos_np(pos) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(pos, dtype=np.int32).reshape(-1, 2))
    return a


def validate_positions(pos, H: int, W: int, M: int) -> None:
    a = _pos_np(pos)
    _check(lib().ptycho_validate_positions(a.ctypes.data_as(P_i32), len(a), H, W, M))


def bin_positions(pos, H: int, W: int, M: int, tiles_y: int, tiles_x: int) -> np.ndarray:
    a = _pos_np(pos)
    out = np.empty(len(a), dtype=np.int32)
    _check(lib().ptycho_bin_positions(a.ctypes.data_as(P_i32), len(a), H, W, M, tiles_y, tiles_x,
                                      out.ctypes.data_as(P_i32)))
    return out


def tile_box(H: int, W: int, tiles_y: int, tiles_x: int, ty: int, tx: int, halo: int):
    """((ty0, ty1, tx0, tx1), (ey0, ey1, ex0, ex1)) of tile (ty, tx)."""
    v = [ctypes.c_int32() for _ in range(8)]
    _check(lib().ptycho_tile_box(H, W, tiles_y, tiles_x, ty, tx, halo, *[ctypes.byref(x) for x in v]))
    vals = [x.value for x in v]
    return tuple(vals[:4]), tuple(vals[4:])


def gd_step_size(probe, pos, H: int, W: int, S: int) -> float:
    """The library's gradient-descent step length for a probe (complex64 [M, M], host or device) and
    window corners over an H x W object with S slices (ptycho_gd_step_size)."""
    if hasattr(probe, "detach"):
        probe = probe.detach().cpu().numpy()
    p = np.ascontiguousarray(np.asarray(probe), dtype=np.complex64)
    if p.ndim != 2 or p.shape[0] != p.shape[1]:
        raise ValueError("probe must be square [M, M]")
    a = _pos_np(pos.detach().cpu().numpy() if hasattr(pos, "detach") else pos)
    out = ctypes.c_double()
    _check(lib().ptycho_gd_step_size(p.ctypes.data_as(c_vp), p.shape[0], a.ctypes.data_as(P_i32), len(a), int(H),
                                     int(W), int(S), ctypes.byref(out)))
    return out.value


# ---------------------------------------------------------------------------
# device calls (torch tensors on the GPU)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream_ptr() -> int:
    torch = _torch()
    return int(torch.cuda.current_stream().cuda_stream)


def _on_device(t, name: str) -> None:
    """Every pointer handed to the library must be device memory of the current device: a host
    pointer or another device's memory would reach the kernels as an invalid address."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.device.index is not None and t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name} is on {t.device}, the current device is cuda:{torch.cuda.current_device()}")


def _obj_geometry(obj) -> Tuple[int, int, int, int, int]:
    """(S, H, W, slice_stride, ld) of a complex64 [S, H, W] device tensor with unit column stride."""
    torch = _torch()
    _on_device(obj, "object")
    if obj.dtype != torch.complex64 or obj.dim() != 3 or obj.stride(2) != 1:
        raise ValueError("object must be complex64 [S, H, W] with unit stride along W")
    S, H, W = obj.shape
    return S, H, W, obj.stride(0), obj.stride(1)


def _need_pos(pos) -> int:
    """Positions: int32 [n, 2] contiguous device tensor; returns n."""
    torch = _torch()
    _need(pos, torch.int32, None, "pos")
    if pos.dim() != 2 or pos.shape[1] != 2:
        raise ValueError(f"pos must have shape [n, 2], got {tuple(pos.shape)}")
    return int(pos.shape[0])


def _need_probe(probe, M: int, n: int) -> int:
    """One probe complex64 [M, M] (returns stride 0) or one per position [n, M, M] (returns M*M)."""
    torch = _torch()
    if isinstance(probe, torch.Tensor) and probe.dim() == 3:
        _need(probe, torch.complex64, (n, M, M), "probe stack")
        return M * M
    _need(probe, torch.complex64, (M, M), "probe")
    return 0


def _need(t, dtype, shape=None, name="tensor"):
    torch = _torch()
    _on_device(t, name)
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """A library context for M x M windows and S slices (one per stream of work)."""

    def __init__(self, M: int, S: int, wavelength_A: float, dz_A: float, pixel_A: float,
                 max_positions: int = 0):
        self._h = c_vp()
        self.M, self.S = int(M), int(S)
        self.physics = (float(wavelength_A), float(dz_A), float(pixel_A))
        self.checkpoint = 1
        _check(lib().ptycho_create(ctypes.byref(self._h), self.M, self.S, float(wavelength_A), float(dz_A),
                                   float(pixel_A), int(max_positions), c_vp(_stream_ptr())))

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("context destroyed")
        return self._h

    def close(self) -> None:
        if self._h:
            lib().ptycho_destroy(self._h)
            self._h = c_vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self) -> None:
        _check(lib().ptycho_set_stream(self.handle, c_vp(_stream_ptr())))

    def reserve(self, max_positions: int) -> None:
        _check(lib().ptycho_reserve(self.handle, int(max_positions)))

    def set_checkpoint(self, interval: int) -> None:
        """Keep the incident wave of every interval-th slice and recompute the others in the adjoint sweep."""
        _check(lib().ptycho_set_checkpoint(self.handle, int(interval)))
        self.checkpoint = int(interval)

    def workspace_bytes(self) -> int:
        return int(lib().ptycho_workspace_bytes(self.handle))

    def check(self) -> int:
        st = c_u32()
        _check(lib().ptycho_check(self.handle, ctypes.byref(st)))
        return st.value

    def profile(self, enable: bool = True) -> None:
        _check(lib().ptycho_profile_enable(self.handle, 1 if enable else 0))

    def profile_read(self):
        """(kernel ms summed, launches, positions) since the last read."""
        ms, nl, npos = c_dbl(), c_i64(), c_i64()
        _check(lib().ptycho_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(npos)))
        return ms.value, nl.value, npos.value


def ptycho_forward(ctx: Context, obj, probe, pos, intens=None):
    """I_i = |G(p_i, V)|^2 for every position; returns float32 [n, M, M].

    probe: complex64 [M, M], or [n, M, M] with one probe per position (ptycho_forward_stack, e.g. the
    sub-pixel probes of ptycho_shift_probes)."""
    torch = _torch()
    S, H, W, ss, ld = _obj_geometry(obj)
    if S != ctx.S:
        raise ValueError(f"object has {S} slices, context {ctx.S}")
    M = ctx.M
    n = _need_pos(pos)
    pstride = _need_probe(probe, M, n)
    if intens is None:
        intens = torch.empty((n, M, M), dtype=torch.float32, device=obj.device)
    _need(intens, torch.float32, (n, M, M), "intens")
    ctx._bind_stream()
    if pstride:
        _check(lib().ptycho_forward_stack(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                          pstride, c_vp(pos.data_ptr()), n, c_vp(intens.data_ptr())))
    else:
        _check(lib().ptycho_forward(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                    c_vp(pos.data_ptr()), n, c_vp(intens.data_ptr())))
    return intens


def ptycho_loss(ctx: Context, obj, probe, pos, meas, loss=None, loss_per_pos=None, accumulate: bool = False):
    """Amplitude cost F as a float64 [1] device tensor (forward sweep only); probe [M, M] or one per
    position [n, M, M] (ptycho_loss_stack)."""
    torch = _torch()
    S, H, W, ss, ld = _obj_geometry(obj)
    if S != ctx.S:
        raise ValueError(f"object has {S} slices, context {ctx.S}")
    M = ctx.M
    n = _need_pos(pos)
    pstride = _need_probe(probe, M, n)
    _need(meas, torch.float32, (n, M, M), "meas")
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
    _need(loss, torch.float64, (1,), "loss")
    lpp = c_vp(0)
    if loss_per_pos is not None:
        _need(loss_per_pos, torch.float64, (n,), "loss_per_pos")
        lpp = c_vp(loss_per_pos.data_ptr())
    ctx._bind_stream()
    flags = PTYCHO_ACCUMULATE if accumulate else 0
    if pstride:
        _check(lib().ptycho_loss_stack(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                       pstride, c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()),
                                       c_vp(loss.data_ptr()), lpp, flags))
    else:
        _check(lib().ptycho_loss(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                 c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()), c_vp(loss.data_ptr()), lpp, flags))
    return loss


def ptycho_loss_grad(ctx: Context, obj, probe, pos, meas, grad=None, loss=None, loss_per_pos=None,
                     accumulate: bool = False, grad_scale=None, probe_grad=None):
    """(loss float64 [1], grad complex64 [S, H, W]) of the amplitude cost.

    grad_scale: optional float64 [1] device tensor multiplying the gradient.
    probe_grad: optional complex64 [M, M] device tensor that receives dF/dP
    (ptycho_loss_grad_probe).
    probe: complex64 [M, M], or [n, M, M] with one probe per position (ptycho_loss_grad_stack; no
    probe gradient then).
    """
    torch = _torch()
    S, H, W, ss, ld = _obj_geometry(obj)
    if S != ctx.S:
        raise ValueError(f"object has {S} slices, context {ctx.S}")
    M = ctx.M
    n = _need_pos(pos)
    pstride = _need_probe(probe, M, n)
    if pstride and probe_grad is not None:
        raise ValueError("the probe gradient needs one probe shared by all positions")
    _need(meas, torch.float32, (n, M, M), "meas")
    if grad is None:
        grad = torch.empty((S, H, W), dtype=torch.complex64, device=obj.device)
    if grad.dtype != torch.complex64 or grad.dim() != 3 or tuple(grad.shape) != (S, H, W) or grad.stride(2) != 1:
        raise ValueError("grad must be complex64 [S, H, W] with unit stride along W")
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
    _need(loss, torch.float64, (1,), "loss")
    lpp = c_vp(0)
    if loss_per_pos is not None:
        _need(loss_per_pos, torch.float64, (n,), "loss_per_pos")
        lpp = c_vp(loss_per_pos.data_ptr())
    gs = c_vp(0)
    if grad_scale is not None:
        _need(grad_scale, torch.float64, (1,), "grad_scale")
        gs = c_vp(grad_scale.data_ptr())
    ctx._bind_stream()
    flags = PTYCHO_ACCUMULATE if accumulate else 0
    if pstride:
        _check(lib().ptycho_loss_grad_stack(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                            pstride, c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()),
                                            c_vp(loss.data_ptr()), lpp, c_vp(grad.data_ptr()), grad.stride(0),
                                            grad.stride(1), flags, gs))
    elif probe_grad is None:
        _check(lib().ptycho_loss_grad(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                      c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()), c_vp(loss.data_ptr()), lpp,
                                      c_vp(grad.data_ptr()), grad.stride(0), grad.stride(1), flags, gs))
    else:
        _need(probe_grad, torch.complex64, (M, M), "probe_grad")
        _check(lib().ptycho_loss_grad_probe(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, c_vp(probe.data_ptr()),
                                            c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()), c_vp(loss.data_ptr()),
                                            lpp, c_vp(grad.data_ptr()), grad.stride(0), grad.stride(1),
                                            c_vp(probe_grad.data_ptr()), flags, gs))
    return loss, grad


def ptycho_loss_grad_static(M: int, wavelength_A: float, dz_A: float, pixel_A: float, obj, probe, pos, meas,
                            grad=None, loss=None, loss_per_pos=None, accumulate: bool = False, grad_scale=None):
    """ptycho_loss_grad without a context (ptycho_loss_grad_static): the library's own static device
    workspace instead of a context's allocations; on torch's current stream.  S comes from obj."""
    torch = _torch()
    S, H, W, ss, ld = _obj_geometry(obj)
    n = _need_pos(pos)
    _need(probe, torch.complex64, (M, M), "probe")
    _need(meas, torch.float32, (n, M, M), "meas")
    if grad is None:
        grad = torch.empty((S, H, W), dtype=torch.complex64, device=obj.device)
    if grad.dtype != torch.complex64 or grad.dim() != 3 or tuple(grad.shape) != (S, H, W) or grad.stride(2) != 1:
        raise ValueError("grad must be complex64 [S, H, W] with unit stride along W")
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
    _need(loss, torch.float64, (1,), "loss")
    lpp = c_vp(0)
    if loss_per_pos is not None:
        _need(loss_per_pos, torch.float64, (n,), "loss_per_pos")
        lpp = c_vp(loss_per_pos.data_ptr())
    gs = c_vp(0)
    if grad_scale is not None:
        _need(grad_scale, torch.float64, (1,), "grad_scale")
        gs = c_vp(grad_scale.data_ptr())
    flags = PTYCHO_ACCUMULATE if accumulate else 0
    _check(lib().ptycho_loss_grad_static(int(M), S, float(wavelength_A), float(dz_A), float(pixel_A),
                                         c_vp(_stream_ptr()), c_vp(obj.data_ptr()), H, W, ss, ld,
                                         c_vp(probe.data_ptr()), c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()),
                                         c_vp(loss.data_ptr()), lpp, c_vp(grad.data_ptr()), grad.stride(0),
                                         grad.stride(1), flags, gs))
    return loss, grad


def ptycho_shift_probes(ctx: Context, probe, shifts, out=None):
    """The probe translated by shifts[i] = (dy, dx) pixels for every i (Fourier shift theorem on the
    window grid); probe complex64 [M, M], shifts float32 [n, 2] on the device; returns [n, M, M]."""
    torch = _torch()
    M = ctx.M
    _need(probe, torch.complex64, (M, M), "probe")
    _need(shifts, torch.float32, None, "shifts")
    if shifts.dim() != 2 or shifts.shape[1] != 2:
        raise ValueError(f"shifts must have shape [n, 2], got {tuple(shifts.shape)}")
    n = int(shifts.shape[0])
    if out is None:
        out = torch.empty((n, M, M), dtype=torch.complex64, device=probe.device)
    _need(out, torch.complex64, (n, M, M), "out")
    ctx._bind_stream()
    _check(lib().ptycho_shift_probes(ctx.handle, c_vp(probe.data_ptr()), c_vp(shifts.data_ptr()), n,
                                     c_vp(out.data_ptr())))
    return out


def split_positions(pos):
    """Real-valued positions [n, 2] (host array) -> (integer window corners int32 [n, 2], fractions
    float32 [n, 2] in [0, 1)), the split of a sub-pixel position into window and probe translation."""
    import numpy as np
    p = np.asarray(pos, dtype=np.float64).reshape(-1, 2)
    corner = np.floor(p)
    return corner.astype(np.int32), (p - corner).astype(np.float32)


def ptycho_tile_grad(ctx: Context, obj_ext, box, tile, halo: int, H: int, W: int, probe, pos, meas,
                     tile_grad=None, loss=None, loss_per_pos=None, accumulate: bool = False):
    """Gradient of one tile's positions on its extended box.

    box = (ey0, ex0, eh, ew); tile = (ty0, ty1, tx0, tx1) in global pixels;
    obj_ext is the [S, eh, ew] box of the object (may be a view of the full object).
    """
    torch = _torch()
    S, eh, ew, ss, ld = _obj_geometry(obj_ext)
    ey0, ex0, beh, bew = box
    if (beh, bew) != (eh, ew) or S != ctx.S:
        raise ValueError("obj_ext shape does not match the box or the context")
    M = ctx.M
    _need(probe, torch.complex64, (M, M), "probe")
    _need_pos(pos)
    n = pos.shape[0]
    _need(meas, torch.float32, (n, M, M), "meas")
    if tile_grad is None:
        tile_grad = torch.empty((S, eh, ew), dtype=torch.complex64, device=obj_ext.device)
    _need(tile_grad, torch.complex64, (S, eh, ew), "tile_grad")
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=obj_ext.device)
    _need(loss, torch.float64, (1,), "loss")
    lpp = c_vp(0)
    if loss_per_pos is not None:
        _need(loss_per_pos, torch.float64, (n,), "loss_per_pos")
        lpp = c_vp(loss_per_pos.data_ptr())
    ty0, ty1, tx0, tx1 = tile
    ctx._bind_stream()
    _check(lib().ptycho_tile_grad(ctx.handle, c_vp(obj_ext.data_ptr()), ey0, ex0, eh, ew, ss, ld, ty0, ty1, tx0,
                                  tx1, halo, H, W, c_vp(probe.data_ptr()), c_vp(pos.data_ptr()), n,
                                  c_vp(meas.data_ptr()), c_vp(loss.data_ptr()), lpp, c_vp(tile_grad.data_ptr()),
                                  PTYCHO_ACCUMULATE if accumulate else 0))
    return loss, tile_grad


def ptycho_tile_accumulate(ctx: Context, tile_grad, box, grad) -> None:
    """grad[:, ey0:ey0+eh, ex0:ex0+ew] += tile_grad (the stitch of the tile walk)."""
    torch = _torch()
    ey0, ex0, eh, ew = box
    if grad.dim() != 3:
        raise ValueError("grad must be complex64 [S, H, W] with unit stride along W")
    S, H, W = grad.shape
    _need(tile_grad, torch.complex64, (ctx.S, eh, ew), "tile_grad")
    _on_device(grad, "grad")
    if grad.dtype != torch.complex64 or grad.dim() != 3 or grad.stride(2) != 1 or S != ctx.S:
        raise ValueError("grad must be complex64 [S, H, W] with unit stride along W")
    ctx._bind_stream()
    _check(lib().ptycho_tile_accumulate(ctx.handle, c_vp(tile_grad.data_ptr()), ey0, ex0, eh, ew, H, W,
                                        c_vp(grad.data_ptr()), grad.stride(0), grad.stride(1)))


EXCHANGE_ADD, EXCHANGE_REPLACE = 0, 1


def ptycho_box_exchange(ctx: Context, src, src_origin, dst, dst_origin, replace: bool = False) -> None:
    """On the overlap of two boxes (global origins (y0, x0), sizes from the
    tensors' shapes): dst += src, or dst = src with replace=True.  src and dst
    are complex64 [S, h, w] views with unit stride along w, in separate memory."""
    torch = _torch()
    for t, name in ((src, "src"), (dst, "dst")):
        _on_device(t, name)
        if t.dtype != torch.complex64:
            raise ValueError(f"{name} must be a complex64 CUDA tensor")
        if t.dim() != 3 or t.stride(2) != 1 or t.shape[0] != ctx.S:
            raise ValueError(f"{name} must be [S, h, w] with unit stride along w")
    ctx._bind_stream()
    _check(lib().ptycho_box_exchange(ctx.handle, ctx.S, c_vp(src.data_ptr()), int(src_origin[0]),
                                     int(src_origin[1]), src.shape[1], src.shape[2], src.stride(0), src.stride(1),
                                     c_vp(dst.data_ptr()), int(dst_origin[0]), int(dst_origin[1]), dst.shape[1],
                                     dst.shape[2], dst.stride(0), dst.stride(1),
                                     EXCHANGE_REPLACE if replace else EXCHANGE_ADD))


def ptycho_box_axpy(ctx: Context, alpha: float, src, src_origin, dst, dst_origin) -> None:
    """dst += alpha * src on the overlap of two boxes (same conventions as ptycho_box_exchange)."""
    torch = _torch()
    for t, name in ((src, "src"), (dst, "dst")):
        _on_device(t, name)
        if t.dtype != torch.complex64:
            raise ValueError(f"{name} must be a complex64 CUDA tensor")
        if t.dim() != 3 or t.stride(2) != 1 or t.shape[0] != ctx.S:
            raise ValueError(f"{name} must be [S, h, w] with unit stride along w")
    ctx._bind_stream()
    _check(lib().ptycho_box_axpy(ctx.handle, ctx.S, float(alpha), c_vp(src.data_ptr()), int(src_origin[0]),
                                 int(src_origin[1]), src.shape[1], src.shape[2], src.stride(0), src.stride(1),
                                 c_vp(dst.data_ptr()), int(dst_origin[0]), int(dst_origin[1]), dst.shape[1],
                                 dst.shape[2], dst.stride(0), dst.stride(1)))


def _plane(t, dtype, S, name):
    torch = _torch()
    _on_device(t, name)
    if t.dtype != dtype:
        raise ValueError(f"{name} must be a {dtype} CUDA tensor")
    if t.dim() != 3 or t.stride(2) != 1 or t.shape[0] != S:
        raise ValueError(f"{name} must be [S, H, W] with unit stride along W")


def ptycho_potential_transmission(ctx: Context, V, sigma: float, t=None):
    """t = exp(i sigma V) for a float32 [S, H, W] potential; returns complex64 [S, H, W]."""
    torch = _torch()
    _plane(V, torch.float32, ctx.S, "V")
    if t is None:
        t = torch.empty(tuple(V.shape), dtype=torch.complex64, device=V.device)
    _plane(t, torch.complex64, ctx.S, "t")
    if tuple(t.shape) != tuple(V.shape):
        raise ValueError("t must have V's shape")
    ctx._bind_stream()
    _check(lib().ptycho_potential_transmission(ctx.handle, V.shape[1], V.shape[2], float(sigma), c_vp(V.data_ptr()),
                                               V.stride(0), V.stride(1), c_vp(t.data_ptr()), t.stride(0),
                                               t.stride(1)))
    return t


def ptycho_potential_gradient(ctx: Context, t, grad_t, sigma: float, grad_V=None):
    """dF/dV = sigma Im(conj(t) grad_t) for t = exp(i sigma V); returns float32 [S, H, W]."""
    torch = _torch()
    _plane(t, torch.complex64, ctx.S, "t")
    _plane(grad_t, torch.complex64, ctx.S, "grad_t")
    if grad_V is None:
        grad_V = torch.empty(tuple(t.shape), dtype=torch.float32, device=t.device)
    _plane(grad_V, torch.float32, ctx.S, "grad_V")
    if tuple(grad_t.shape) != tuple(t.shape) or tuple(grad_V.shape) != tuple(t.shape):
        raise ValueError("t, grad_t and grad_V must have one shape")
    ctx._bind_stream()
    _check(lib().ptycho_potential_gradient(ctx.handle, t.shape[1], t.shape[2], float(sigma), c_vp(t.data_ptr()),
                                           t.stride(0), t.stride(1), c_vp(grad_t.data_ptr()), grad_t.stride(0),
                                           grad_t.stride(1), c_vp(grad_V.data_ptr()), grad_V.stride(0),
                                           grad_V.stride(1)))
    return grad_V


def ptycho_tiles_grad(ctx: Context, obj, tiles, halo: int, tile_of_pos, probe, pos, meas, loss=None,
                      loss_per_pos=None, accumulate: bool = False):
    """All tiles' gradients in one launch.  tiles: sequence of (tile (ty0, ty1, tx0, tx1),
    box (ey0, ex0, eh, ew), grad complex64 [S, eh, ew] contiguous); tile_of_pos int32 [n] and pos
    int32 [n, 2] (global) on the device; probe [M, M] or one per position [n, M, M] in the order of
    pos (ptycho_tiles_grad_stack).  Returns the total loss (float64 [1])."""
    torch = _torch()
    S, H, W, ss, ld = _obj_geometry(obj)
    if S != ctx.S:
        raise ValueError(f"object has {S} slices, context {ctx.S}")
    M = ctx.M
    n = _need_pos(pos)
    pstride = _need_probe(probe, M, n)
    _need(tile_of_pos, torch.int32, (n,), "tile_of_pos")
    _need(meas, torch.float32, (n, M, M), "meas")
    arr = (TileDesc * len(tiles))()
    for k, (tile, box, g) in enumerate(tiles):
        _need(g, torch.complex64, (S, box[2], box[3]), f"tile gradient {k}")
        arr[k] = TileDesc(tile[0], tile[1], tile[2], tile[3], box[0], box[1], box[2], box[3], g.data_ptr())
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
    _need(loss, torch.float64, (1,), "loss")
    lpp = c_vp(0)
    if loss_per_pos is not None:
        _need(loss_per_pos, torch.float64, (n,), "loss_per_pos")
        lpp = c_vp(loss_per_pos.data_ptr())
    ctx._bind_stream()
    flags = PTYCHO_ACCUMULATE if accumulate else 0
    if pstride:
        _check(lib().ptycho_tiles_grad_stack(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, arr, len(tiles),
                                             int(halo), c_vp(tile_of_pos.data_ptr()), c_vp(probe.data_ptr()), pstride,
                                             c_vp(pos.data_ptr()), n, c_vp(meas.data_ptr()), c_vp(loss.data_ptr()),
                                             lpp, flags))
    else:
        _check(lib().ptycho_tiles_grad(ctx.handle, c_vp(obj.data_ptr()), H, W, ss, ld, arr, len(tiles), int(halo),
                                       c_vp(tile_of_pos.data_ptr()), c_vp(probe.data_ptr()), c_vp(pos.data_ptr()), n,
                                       c_vp(meas.data_ptr()), c_vp(loss.data_ptr()), lpp, flags))
    return loss


def ptycho_copy_box(ctx: Context, src, dst) -> None:
    """dst[...] = src[...] for complex64 [S, h, w] views (host or device, unit stride along w), one
    pitched copy per slice on the context stream; pinned host memory makes it asynchronous."""
    torch = _torch()
    for t, name in ((src, "src"), (dst, "dst")):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex64 or t.dim() != 3 or t.stride(2) != 1:
            raise ValueError(f"{name} must be complex64 [S, h, w] with unit stride along w")
    if tuple(src.shape) != tuple(dst.shape):
        raise ValueError("src and dst must have one shape")
    S, h, w = src.shape
    ctx._bind_stream()
    _check(lib().ptycho_copy_box(ctx.handle, S, h, w, c_vp(src.data_ptr()), src.stride(0), src.stride(1),
                                 c_vp(dst.data_ptr()), dst.stride(0), dst.stride(1)))


def ptycho_zero_gradient(ctx: Context, grad) -> None:
    """grad[...] = 0 with the library's fill kernel."""
    torch = _torch()
    _on_device(grad, "grad")
    if grad.dtype != torch.complex64 or grad.dim() != 3 or grad.stride(2) != 1 or grad.shape[0] != ctx.S:
        raise ValueError("grad must be complex64 [S, H, W] with unit stride along W")
    ctx._bind_stream()
    _check(lib().ptycho_zero_gradient(ctx.handle, c_vp(grad.data_ptr()), grad.shape[1], grad.shape[2],
                                      grad.stride(0), grad.stride(1)))
