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


SECOND_ORDER_POINTS = (1.0, 2.0, 3.0, 10.0)


def make_params(shape, h, dt, *, radius=1, order="first", form="faces", s0=1.0, s1=1.0, s2=0.0, window=0,
                fejer=True, dtype="c128", batch=1, meanfield=None, path="auto",
                s_points=None, diag_every=0) -> _lib.AbcParams:
    """abc_params for a box of shape (nz, ny, nx) (see include/abc_dtn.h).
    s_points: the four interpolation points of the second order (default
    SECOND_ORDER_POINTS); s1, s2 are the first order's."""
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
    if order == "second":
        pts = SECOND_ORDER_POINTS if s_points is None else tuple(float(v) for v in s_points)
        if len(pts) != 4:
            raise ValueError("the second order takes four interpolation points")
        p.s1, p.s2, p.s3, p.s4 = pts
    p.window = int(window)
    p.fejer = 1 if fejer else 0
    p.dtype = _lib.DTYPES[dtype]
    p.batch = int(batch)
    if isinstance(meanfield, dict):
        # Sec. 4.3 with the long-range terms: t0, t3, v0, a (Yukawa), e2
        # (Coulomb), tol and maxit of the conjugate-gradient solves
        mf = dict(meanfield)
        p.meanfield = 2
        p.t0, p.t3 = float(mf.pop("t0", 0.0)), float(mf.pop("t3", 0.0))
        p.v0, p.a_yukawa, p.e2 = float(mf.pop("v0", 0.0)), float(mf.pop("a", 1.0)), float(mf.pop("e2", 0.0))
        p.pcg_tol, p.pcg_maxit = float(mf.pop("tol", 1e-12)), int(mf.pop("maxit", 1000))
        p.pcg_fixed = int(mf.pop("fixed_iters", 0))
        if mf:
            raise ValueError("unknown mean-field keys %s" % sorted(mf))
    elif meanfield is not None:
        p.meanfield = 1
        p.t0, p.t3 = float(meanfield[0]), float(meanfield[1])
    p.path = _lib.PATHS[path]
    p.diag_every = int(diag_every)
    return p


class Solver:
    """One context of the C ABI (operators + scratch) for a fixed box.

    shape: (nz, ny, nx).  order: "dirichlet" | "periodic" | "zeroth" | "first"
    | "second" (box form; s_points = its four interpolation points).
    form: "faces" | "box".  dtype: "c128" | "c64".  meanfield: (t0, t3), a dict with
    t0, t3, v0, a, e2, tol, maxit (the Skyrme mean field with Yukawa and Coulomb
    terms), or None.  path: "auto" | "staged" | "fused" (two launches of two
    stages per step) | "onepass" (one launch per step); after setup,
    ``self.path`` names the one chosen.  diag_every: steps between the
    records of step_monitored (0: no monitoring).
    """

    def __init__(self, shape: Sequence[int], h: float, dt: float, *, radius: int = 1,
                 order: str = "first", form: str = "faces", s0: float = 1.0, s1: float = 1.0,
                 s2: float = 0.0, window: int = 0, fejer: bool = True, dtype: str = "c128",
                 batch: int = 1, meanfield=None, path: str = "auto", device=None, s_points=None,
                 diag_every: int = 0):
        lib = _lib.load()
        p = make_params(shape, h, dt, radius=radius, order=order, form=form, s0=s0, s1=s1, s2=s2,
                        window=window, fejer=fejer, dtype=dtype, batch=batch, meanfield=meanfield, path=path,
                        s_points=s_points, diag_every=diag_every)
        nz, ny, nx = (int(v) for v in shape)
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
        code = int(lib.abc_path(ctx))
        self.path = {v: k for k, v in _lib.PATHS.items()}[code]
        self.use_fused = self.path in ("fused", "onepass")

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
        if self.aux_elems == 0:
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

    def new_monitor(self, ring_len: int = 16):
        """(ring, flags) for step_monitored: ring_len records of 3*batch+2
        float64 (step count, then the diagnostics), and a zeroed int32 flag word."""
        ring = torch.zeros((int(ring_len), 3 * self.batch + 2), dtype=torch.float64, device=self.device)
        return ring, torch.zeros(1, dtype=torch.int32, device=self.device)

    def step_monitored(self, psi, ring, flags, aux=None, V=None, n_steps: int = 1, stream=None):
        """step() with a diagnostics record every diag_every steps into ``ring``
        and the _lib.ABC_FLAG_* failure flags or-ed into ``flags`` (both on the
        device; read them after synchronising)."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux)
        if ring.dtype != torch.float64 or ring.dim() != 2 or ring.shape[1] != 3 * self.batch + 2 \
                or not ring.is_contiguous() or ring.device.type != "cuda":
            raise ValueError("ring must be a contiguous float64 CUDA tensor of shape (n, %d)" % (3 * self.batch + 2))
        if flags.dtype != torch.int32 or flags.numel() < 1 or flags.device.type != "cuda":
            raise ValueError("flags must be an int32 CUDA tensor")
        _lib.check(self._lib.abc_step_monitored(self._ctx, psi.data_ptr(), ap, vp, int(n_steps),
                                                _stream_handle(stream), ring.data_ptr(), int(ring.shape[0]),
                                                flags.data_ptr()))
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

    def objective(self, psi0, V=None, n_steps: int = 1, objective: str = "prob", stream=None) -> float:
        """J(psi_N) after n_steps from (psi0, f = 0), forward only: h^3 sum
        |psi_N|^2 ("prob") or h^3 Re <psi_N, H psi_N> ("energy"), from the
        device diagnostics of a stepped copy of psi0 (one orbital)."""
        if self.batch != 1:
            raise ValueError("objective: one orbital")
        if objective not in _lib.OBJECTIVES:
            raise ValueError("objective must be one of %s" % sorted(_lib.OBJECTIVES))
        psi = psi0.detach().clone().contiguous()
        aux = self.new_aux()
        self.step(psi, aux, V, n_steps, stream=stream)
        d = self.diagnostics(psi, aux if self.aux_elems else None, V, stream=stream)
        return float(d[0 if objective == "prob" else 2].item())

    def tune(self, psi, aux=None, V=None, stream=None) -> int:
        """Pick the fused path's tile depth by timing (state restored); returns it."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux)
        tz = ctypes.c_int(0)
        _lib.check(self._lib.abc_tune(self._ctx, psi.data_ptr(), ap, vp, _stream_handle(stream), ctypes.byref(tz)))
        return tz.value

    def diagnostics(self, psi, aux=None, V=None, out: Optional[torch.Tensor] = None, stream=None):
        """Tensor of 3*batch+1 float64: norm, Lyapunov W, energy per orbital, interaction energy."""
        self._check_psi(psi)
        vp = self._check_V(V)
        ap = self._check_aux(aux) if self.aux_elems else None
        if out is None:
            out = torch.empty(3 * self.batch + 1, dtype=torch.float64, device=self.device)
        _lib.check(self._lib.abc_diagnostics(self._ctx, psi.data_ptr(), ap, vp, out.data_ptr(),
                                             _stream_handle(stream)))
        return out

    def effective_potential(self, psi, V=None, out: Optional[torch.Tensor] = None, stream=None):
        """V + t0 rho + t3 rho^2 + W_Y + W_C of psi (Skyrme mean field only)."""
        self._check_psi(psi)
        vp = self._check_V(V)
        if out is None:
            out = torch.empty(self.shape, dtype=self.rdtype, device=self.device)
        _lib.check(self._lib.abc_effective_potential(self._ctx, psi.data_ptr(), vp, out.data_ptr(),
                                                     _stream_handle(stream)))
        return out

    def potential_iterations(self):
        """(mean-field evaluations, Yukawa CG iterations, Coulomb CG iterations)."""
        buf = (ctypes.c_longlong * 3)()
        _lib.check(self._lib.abc_potential_iterations(self._ctx, buf))
        return tuple(int(v) for v in buf)

    def potential_unconverged(self) -> int:
        """Mean-field solves so far that ended without reaching their tolerance
        (counted on the device; synchronises it)."""
        v = ctypes.c_longlong()
        _lib.check(self._lib.abc_potential_unconverged(self._ctx, ctypes.byref(v)))
        return int(v.value)

    def save_state(self, path: str, psi, aux=None, step: int = 0, stream=None):
        """Checkpoint (psi, aux) and a step counter to a file (abc_state_save)."""
        self._check_psi(psi)
        ap = self._check_aux(aux) if self.aux_elems else None
        _lib.check(self._lib.abc_state_save(self._ctx, psi.data_ptr(), ap, int(step), str(path).encode(),
                                            _stream_handle(stream)))

    def load_state(self, path: str, psi, aux=None, stream=None) -> int:
        """Restore (psi, aux) from a checkpoint of a matching context; returns its step."""
        self._check_psi(psi)
        ap = self._check_aux(aux) if self.aux_elems else None
        step = ctypes.c_longlong(0)
        _lib.check(self._lib.abc_state_load(self._ctx, psi.data_ptr(), ap, ctypes.byref(step), str(path).encode(),
                                            _stream_handle(stream)))
        return int(step.value)

    def export(self, which: int, count: int) -> np.ndarray:
        buf = np.zeros(count, dtype=np.complex128)
        _lib.check(self._lib.abc_export(self._ctx, which, buf.ctypes.data, count))
        return buf

    def box_info(self) -> dict:
        """Box form: n_Gamma, the dimension the second order interpolates in,
        and the spectral bound of the boundary block."""
        v = self.export(3, 2)
        return {"n_gamma": int(v[0].real), "subspace_dim": int(v[0].imag), "bound": float(v[1].real)}

    def face_kernel(self) -> np.ndarray:
        R, w = self.params.radius, self.params.window
        K = 2 * w + 1
        return self.export(0, R * R * K * K).reshape(R, R, K, K)

    def device_bytes(self) -> int:
        return int(self._lib.abc_device_bytes(self._ctx))


def h2_objective(h: float, s1, *, window: int = 0, fejer: bool = True, modes: int = 64, nodes: int = 4096,
                 stream=None) -> np.ndarray:
    """H2 objective J(s1) of the first-order face-form condition (R = 1) for
    each candidate point, evaluated on the device (abc_h2_objective)."""
    lib = _lib.load()
    pts = np.ascontiguousarray(np.atleast_1d(np.asarray(s1, dtype=np.float64)))
    p = make_params((8, 8, 8), h, 1e-3, order="first", form="faces", window=window, fejer=fejer)
    out = np.zeros(pts.size, dtype=np.float64)
    _lib.check(lib.abc_h2_objective(ctypes.byref(p), pts.ctypes.data, int(pts.size), int(modes), int(nodes),
                                    out.ctypes.data, _stream_handle(stream)))
    return out


def optimal_point(h: float, *, window: int = 0, fejer: bool = True, modes: int = 64, nodes: int = 4096,
                  lo: float = 1e-2, hi: float = 1e4, grid: int = 25, iters: int = 30):
    """The H2-optimal first-order point: the smallest J on a log-spaced grid
    over [lo, hi], refined by golden-section search in log s1 between the
    grid neighbours of that point.  Returns (s1, J(s1))."""
    xs = np.exp(np.linspace(math.log(lo), math.log(hi), grid))
    js = h2_objective(h, xs, window=window, fejer=fejer, modes=modes, nodes=nodes)
    k = int(np.argmin(js))
    a = math.log(xs[max(k - 1, 0)])
    b = math.log(xs[min(k + 1, grid - 1)])
    f = lambda t: float(h2_objective(h, math.exp(t), window=window, fejer=fejer, modes=modes, nodes=nodes)[0])
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    best = min([(fc, c), (fd, d), (float(js[k]), math.log(xs[k]))])
    return math.exp(best[1]), best[0]


class Batch:
    """Independent boxes stepped together (abc_setup_batch / abc_step_batch).

    configs: list of dicts with the Solver keyword arguments plus "shape", "h", "dt".
    """

    def __init__(self, configs, device=None):
        lib = _lib.load()
        n = len(configs)
        arr = (_lib.AbcParams * n)()
        self.configs = []
        for i, cfg in enumerate(configs):
            cfg = dict(cfg)
            shape, h, dt = cfg.pop("shape"), cfg.pop("h"), cfg.pop("dt")
            arr[i] = make_params(shape, h, dt, **cfg)
            self.configs.append(dict(shape=tuple(int(v) for v in shape), dtype=cfg.get("dtype", "c128"),
                                     order=cfg.get("order", "first")))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.abc_setup_batch(arr, n, ctypes.byref(b)))
        self._b = b
        self._lib = lib
        self.n = n
        self.aux_elems = [int(lib.abc_batch_aux_elems(b, i)) for i in range(n)]

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.abc_destroy_batch(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_aux(self, i):
        return torch.zeros(max(self.aux_elems[i], 1), dtype=torch.complex128, device=self.device)

    def groups(self):
        g = int(self._lib.abc_batch_launch_groups(self._b))
        return [int(self._lib.abc_batch_tile_depth(self._b, k)) for k in range(g)]

    def _ptrs(self, psis, auxs, Vs):
        if len(psis) != self.n:
            raise ValueError("expected %d psi tensors" % self.n)
        for i, (p, cfg) in enumerate(zip(psis, self.configs)):
            cdt = torch.complex128 if cfg["dtype"] == "c128" else torch.complex64
            if p.dtype != cdt or tuple(p.shape) != cfg["shape"] or not p.is_contiguous() or p.device.type != "cuda":
                raise ValueError("psi %d must be a contiguous %s tensor of shape %s" % (i, cdt, cfg["shape"]))
        P = (ctypes.c_void_p * self.n)(*[p.data_ptr() for p in psis])
        A = None
        if auxs is not None:
            for i, a in enumerate(auxs):
                if a is not None and (a.dtype != torch.complex128 or a.numel() < self.aux_elems[i]):
                    raise ValueError("aux %d must hold %d complex128 elements" % (i, self.aux_elems[i]))
            A = (ctypes.c_void_p * self.n)(*[0 if a is None else a.data_ptr() for a in auxs])
        Vp = None
        if Vs is not None:
            Vp = (ctypes.c_void_p * self.n)(*[0 if v is None else v.data_ptr() for v in Vs])
        return P, A, Vp

    def step(self, psis, auxs=None, Vs=None, n_steps=1, graph=False, stream=None):
        P, A, Vp = self._ptrs(psis, auxs, Vs)
        flags = _lib.ABC_BATCH_GRAPH if graph else 0
        _lib.check(self._lib.abc_step_batch(self._b, P, A, Vp, int(n_steps), flags, _stream_handle(stream)))

    def tune(self, psis, auxs=None, Vs=None, stream=None):
        P, A, Vp = self._ptrs(psis, auxs, Vs)
        _lib.check(self._lib.abc_tune_batch(self._b, P, A, Vp, _stream_handle(stream)))
        return self.groups()
