"""Python binding of the HIP stepper: torch tensors in, device pointers out.

PyTorch provides device memory and streams only; every step of the method
runs in the HIP kernels of libabc_dtn.so.  There is no CPU fallback: if the
library is missing or the tensors are not on a GPU the calls raise.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Solver:
    """One context of the C ABI (operators + scratch) for a fixed box.

    shape: (nz, ny, nx).  order: "dirichlet" | "periodic" | "zeroth" | "first".
    form: "faces" | "box".  dtype: "c128" | "c64".  meanfield: (t0, t3) or None.
    """

    def __init__(self, shape: Sequence[int], h: float, dt: float, *, radius: int = 1,
                 order: str = "first", form: str = "faces", s0: float = 1.0, s1: float = 1.0,
                 s2: float = 0.0, window: int = 0, fejer: bool = True, dtype: str = "c128",
                 batch: int = 1, meanfield=None, path: str = "auto", device=None):
        lib = _lib.load()
        p = _lib.AbcParams()
        lib.abc_params_default(ctypes.byref(p))
        nz, ny, nx = (int(v) for v in shape)
        p.nx, p.ny, p.nz = nx, ny, nz
        p.h, p.dt = float(h), float(dt)
        p.radius = int(radius)
        p.order = _lib.ORDERS[order]
        p.form = _lib.FORMS[form]
        p.s0, p.s1 = float(s0), float(s1)
        p.s2 = 0.0 if (s2 is None or (isinstance(s2, float) and math.isinf(s2))) else float(s2)
        p.window = int(window)
        p.fejer = 1 if fejer else 0
        p.dtype = _lib.DTYPES[dtype]
        p.batch = int(batch)
        if meanfield is not None:
            p.meanfield = 1
            p.t0, p.t3 = float(meanfield[0]), float(meanfield[1])
        p.path = _lib.PATHS[path]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.params = p
        self.shape = (nz, ny, nx)
        self.batch = p.batch
        self.order, self.form, self.dtype = order, form, dtype
        self.cdtype = torch.complex128 if dtype == "c128" else torch.complex64
        self.rdtype = torch.float64 if dtype == "c128" else torch.float32
        ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.abc_setup(ctypes.byref(p), ctypes.byref(ctx)))
        self._ctx = ctx
        self._lib = lib
        self.aux_elems = int(lib.abc_aux_elems(ctx))
        self.use_fused = int(lib.abc_path(ctx)) == _lib.PATHS["fused"]

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.abc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def psi_shape(self):
        return self.shape if self.batch == 1 else self.shape + (self.batch,)

    def new_aux(self) -> torch.Tensor:
        return torch.zeros(max(self.aux_elems, 1), dtype=torch.complex128, device=self.device)

    def _check_psi(self, psi):
        if not isinstance(psi, torch.Tensor) or psi.device.type != "cuda":
            raise ValueError("psi must be a CUDA/HIP tensor")
        if psi.dtype != self.cdtype or not psi.is_contiguous():
            raise ValueError("psi must be contiguous %s" % self.cdtype)
        if tuple(psi.shape) not in (self.psi_shape(), self.shape + (self.batch,)):
            raise ValueError("psi has shape %s, expected %s" % (tuple(psi.shape), self.psi_shape()))

    def _check_V(self, V):
        if V is None:
            return None
        if V.dtype != self.rdtype or not V.is_contiguous() or tuple(V.shape) != self.shape or V.device.type != "cuda":
            raise ValueError("V must be a contiguous %s CUDA tensor of shape %s" % (self.rdtype, self.shape))
        return V.data_ptr()

    def _check_aux(self, aux):
        if self.order != "first":
            return None if aux is None else aux.data_ptr()
        if aux is None or aux.dtype != torch.complex128 or aux.numel() < self.aux_elems or not aux.is_contiguous():
            raise ValueError("aux must be a contiguous complex128 tensor of %d elements" % self.aux_elems)
        return aux.data_ptr()

    def step(self, psi, aux=None, V=None, n_steps: int = 1, stream=None):
        """Advance psi (and aux) in place by n_steps on ``stream``."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux)
        _lib.check(self._lib.abc_step(self._ctx, psi.data_ptr(), ap, vp, int(n_steps), _stream_handle(stream)))
        return psi

    def step_timed(self, psi, aux=None, V=None, n_steps: int = 1, stream=None, cap: int = 64):
        """Advance like step() and return [(launch label, mean ms per step)] for
        the kernel launches of one step (HIP events around each launch)."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux)
        ms = (ctypes.c_double * cap)()
        k = ctypes.c_int(0)
        _lib.check(self._lib.abc_step_timed(self._ctx, psi.data_ptr(), ap, vp, int(n_steps), _stream_handle(stream),
                                            ctypes.cast(ms, ctypes.c_void_p), cap, ctypes.byref(k)))
        return [(self._lib.abc_launch_label(self._ctx, j).decode(), ms[j]) for j in range(min(k.value, cap))]

    def adjoint(self, psi0, V=None, n_steps: int = 1, objective: str = "prob", ckpt_stride: int = 0,
                stream=None):
        """Reverse-mode gradient of J(psi_N) after n_steps from (psi0, f = 0).

        Returns (J, grad_psi0, grad_V) with grad_psi0 = dJ/dRe psi0 + i dJ/dIm psi0
        (complex128, psi0's shape) and grad_V = dJ/dV (float64, the box shape).
        objective: "prob" (h^3 sum |psi_N|^2) or "energy" (h^3 Re <psi_N, H psi_N>)."""
        self._check_psi(psi0)
        vp = self._check_V(V)
        gpsi = torch.empty_like(psi0)
        gV = torch.empty(self.shape, dtype=torch.float64, device=psi0.device)
        J = ctypes.c_double(0.0)
        _lib.check(self._lib.abc_adjoint(self._ctx, psi0.data_ptr(), vp, int(n_steps), int(ckpt_stride),
                                         _lib.OBJECTIVES[objective], gpsi.data_ptr(), gV.data_ptr(),
                                         ctypes.byref(J), _stream_handle(stream)))
        return J.value, gpsi, gV

    def diagnostics(self, psi, aux=None, V=None, out: Optional[torch.Tensor] = None, stream=None):
        """Tensor of 3*batch+1 float64: norm, Lyapunov W, energy per orbital, interaction energy."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux) if self.order == "first" else None
        if out is None:
            out = torch.empty(3 * self.batch + 1, dtype=torch.float64, device=self.device)
        _lib.check(self._lib.abc_diagnostics(self._ctx, psi.data_ptr(), ap, vp, out.data_ptr(),
                                             _stream_handle(stream)))
        return out

    def export(self, which: int, count: int) -> np.ndarray:
        buf = np.zeros(count, dtype=np.complex128)
        _lib.check(self._lib.abc_export(self._ctx, which, buf.ctypes.data, count))
        return buf

    def face_kernel(self) -> np.ndarray:
        R, w = self.params.radius, self.params.window
        K = 2 * w + 1
        return self.export(0, R * R * K * K).reshape(R, R, K, K)

    def device_bytes(self) -> int:
        return int(self._lib.abc_device_bytes(self._ctx))
