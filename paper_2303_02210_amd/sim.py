"""Python face of the C ABI: one simulation (``Sim``) per handle.

PyTorch provides the device workspace (a uint8 tensor) and the stream; every
computation happens in ``liblbmgrow.so``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _ffi


def _torch():
    import torch
    return torch


class Sim:
    """A growing-tissue simulation (D2Q9, or the paper's D2Q7 lattice)
    resident on one GPU.

    ``cfg`` is a workload dict (keys of ``lbm_params``; see ``synth_inputs``).
    """

    def __init__(self, cfg: dict, device: str = "cuda:0", stream=None,
                 static_scratch: bool = False):
        """static_scratch: create through lbm_create_static, so that the
        library keeps everything but the populations in its static device
        array (at most one such Sim per device at a time)."""
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("Sim needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.cfg = dict(cfg)
        self.L = int(cfg["L"])
        self.H = int(cfg["H"])
        self.Q = _ffi.Q[cfg.get("lattice", "d2q9")]
        self.device = torch.device(device)
        self._lib = _ffi.lib()
        self._p = _ffi.make_params(cfg)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if static_scratch:
            size = ctypes.c_size_t(0)
            rc = self._lib.lbm_create_static(ctypes.byref(self._p), None, ctypes.byref(size),
                                             None, None)
            if rc != 0:
                raise _ffi.LbmError(rc, "lbm_create_static (size query)")
            nbytes = int(size.value)
            with torch.cuda.device(self.device):
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            rc = self._lib.lbm_create_static(ctypes.byref(self._p),
                                             ctypes.c_void_p(self._ws.data_ptr()),
                                             ctypes.byref(size),
                                             ctypes.c_void_p(self.stream.cuda_stream),
                                             ctypes.byref(h))
            where = "lbm_create_static"
        else:
            nbytes = int(self._lib.lbm_workspace_bytes(ctypes.byref(self._p)))
            if nbytes == 0:
                raise ValueError(f"invalid parameters: {cfg}")
            with torch.cuda.device(self.device):
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            rc = self._lib.lbm_create(ctypes.byref(self._p), ctypes.c_void_p(self._ws.data_ptr()),
                                      nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(h))
            where = "lbm_create"
        self.workspace_bytes = nbytes
        if rc != 0:
            raise _ffi.LbmError(rc, where)
        self._h = h

    # -- life cycle ------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _check(self, rc: int, where: str):
        if rc != 0:
            detail = self._lib.lbm_last_error(self._h).decode() if self._h else ""
            raise _ffi.LbmError(rc, where, detail)

    # -- stepping --------------------------------------------------------
    def step(self, n: int = 1) -> None:
        self._check(self._lib.lbm_step(self._h, int(n)), "lbm_step")

    def front_heights(self) -> np.ndarray:
        out = np.zeros(self.L, np.int32)
        step = ctypes.c_int64()
        self._check(self._lib.lbm_front_heights(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.byref(step)), "lbm_front_heights")
        self.last_step = step.value
        return out

    def front_heights_async(self, dst) -> None:
        """Enqueue h(x) into ``dst`` (an int32 tensor of L elements, on the
        device or in pinned host memory)."""
        assert dst.dtype == _torch().int32 and dst.numel() == self.L and dst.is_contiguous()
        self._check(self._lib.lbm_front_heights_async(self._h, ctypes.c_void_p(dst.data_ptr())),
                    "lbm_front_heights_async")

    def diagnostics(self) -> dict:
        d = _ffi.Diag()
        self._check(self._lib.lbm_diagnostics(self._h, ctypes.byref(d)), "lbm_diagnostics")
        return {k: getattr(d, k) for k, _ in _ffi.Diag._fields_ if k != "reserved"}

    # -- state access ----------------------------------------------------
    def populations(self) -> np.ndarray:
        out = np.zeros((self.Q, self.H, self.L), np.float64)
        self._check(self._lib.lbm_get_populations(self._h, out.ctypes.data_as(ctypes.c_void_p)),
                    "lbm_get_populations")
        return out

    def set_populations(self, f) -> None:
        a = np.ascontiguousarray(f, dtype=np.float64)
        assert a.shape == (self.Q, self.H, self.L)
        self._check(self._lib.lbm_set_populations(self._h, a.ctypes.data_as(ctypes.c_void_p)),
                    "lbm_set_populations")

    def division_map(self, clear: bool = False) -> np.ndarray:
        """Divisions per site of the window since creation or the last clear,
        [H][L] (row j = absolute row y_wall + j); needs cfg["division_map"]."""
        out = np.zeros((self.H, self.L), np.int32)
        self._check(self._lib.lbm_division_map(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                               1 if clear else 0), "lbm_division_map")
        return out

    def set_front_heights(self, h) -> None:
        a = np.ascontiguousarray(h, dtype=np.int32)
        assert a.shape == (self.L,)
        self._check(self._lib.lbm_set_front_heights(self._h, a.ctypes.data_as(ctypes.c_void_p)),
                    "lbm_set_front_heights")

    def get_state(self) -> bytes:
        n = int(self._lib.lbm_state_bytes(self._h))
        buf = ctypes.create_string_buffer(n)
        self._check(self._lib.lbm_get_state(self._h, buf, n), "lbm_get_state")
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self._lib.lbm_set_state(self._h, buf, len(blob)), "lbm_set_state")

    def last_error(self) -> str:
        return self._lib.lbm_last_error(self._h).decode()
