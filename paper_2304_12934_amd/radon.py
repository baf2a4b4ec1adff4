"""Python front end: plans, operators, autograd functions and the MBIR driver.

Thin wrappers over libnufftradon: tensors are validated and their device
pointers handed to the C ABI together with the current HIP stream.  No
arithmetic of the method runs here.
"""

from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (NR_FBP_BUTTERWORTH, NR_FBP_RAMP, NR_MBIR_STATE_DOUBLES, NR_STREAM_ADJ, NR_STREAM_FBP,
                   NR_STREAM_FWD, NR_WEIGHTS_GAUSSIAN, NR_WEIGHTS_INV_DISTANCE, NrFbp, NrMbir, NrNufft, NrPrior,
                   NrSlice, check, lib)

# Plans and graphs still open, closed at interpreter exit while the HIP
# runtime is alive (their streams and graphs are HIP objects); a handle whose
# owner is collected during interpreter finalisation is left to the process
# exit instead of being destroyed then.
_LIVE: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_live() -> None:
    for obj in sorted(list(_LIVE), key=lambda o: 0 if isinstance(o, Graph) else 1):
        try:
            obj.close()
        except Exception:
            pass


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, numel: int, device: torch.device, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, plan is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


@dataclass
class SliceGeometry:
    """One slice of a stack: width ``n``, detector bins ``n_det``, angles (radians)
    and ``center``, the offset in bins of the rotation axis from the detector
    centre (the axis projects to bin ``n_det/2 + center``)."""
    n: int
    n_det: int
    angles: np.ndarray
    center: float = 0.0


class Plan:
    """NUFFT Radon plan for a slice stack, bound to device workspace.

    ``Plan.uniform(n, n_det, angles, n_slices)`` describes ``n_slices`` slices
    sharing one geometry, with volume ``[Z, n, n]`` and sinogram
    ``[Z, n_angles, n_det]``.  ``Plan(geoms)`` describes an uneven stack whose
    volumes and sinograms are packed back to back in flat buffers.
    """

    def __init__(self, geoms: Sequence[SliceGeometry], width: int = 7, beta: float = 0.0,
                 device: torch.device | str | None = None, share_angles: bool = True,
                 tuning: dict | None = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the projector runs on a GPU device only")
        self.geoms = list(geoms)
        slices = (NrSlice * len(self.geoms))()
        angle_chunks: list[np.ndarray] = []
        angle_index: dict[bytes, int] = {}
        vol_off = sino_off = angle_off = 0
        self.vol_offsets, self.sino_offsets = [], []
        for i, g in enumerate(self.geoms):
            ang = np.ascontiguousarray(np.asarray(g.angles, dtype=np.float64))
            key = ang.tobytes()
            if share_angles and key in angle_index:
                a_off = angle_index[key]
            else:
                a_off = angle_off
                angle_index[key] = a_off
                angle_chunks.append(ang)
                angle_off += len(ang)
            slices[i] = NrSlice(int(g.n), int(g.n_det), len(ang), vol_off, sino_off, a_off, float(g.center))
            self.vol_offsets.append(vol_off)
            self.sino_offsets.append(sino_off)
            vol_off += int(g.n) * int(g.n)
            sino_off += len(ang) * int(g.n_det)
        self.vol_numel, self.sino_numel = vol_off, sino_off
        self._angles = np.ascontiguousarray(np.concatenate(angle_chunks)) if angle_chunks else np.zeros(1)
        params = NrNufft(2.0, int(width), float(beta))
        handle = ctypes.c_void_p()
        L = lib()
        check(L.nr_plan_create(slices, len(self.geoms),
                               self._angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(params), ctypes.byref(handle)), "nr_plan_create")
        self._h = handle
        _LIVE.add(self)
        self.tuning = {}
        self._ws = None
        self.retune(**(tuning or {}))
        u = self.geoms[0]
        self.uniform = all(g.n == u.n and g.n_det == u.n_det and len(g.angles) == len(u.angles)
                           for g in self.geoms)

    def retune(self, **kw) -> None:
        """Apply execution parameters (tile_w, tile_h, chunk, batch, spread_mode)
        and (re)bind a workspace of the size the new layout needs."""
        L = lib()
        for k, v in kw.items():
            check(L.nr_plan_tune(self._h, k.encode(), int(v)), f"nr_plan_tune({k})")
            self.tuning[k] = int(v)
        if self._ws is not None and set(kw) <= {"spread_mode"}:
            return
        self._bind()

    def _bind(self) -> None:
        """Allocate a workspace of the size the current layout needs and bind it."""
        L = lib()
        nbytes = ctypes.c_size_t()
        check(L.nr_plan_workspace_bytes(self._h, ctypes.byref(nbytes)), "nr_plan_workspace_bytes")
        self.workspace_bytes = int(nbytes.value)
        self._ws = None
        self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws.data_ptr()) % 256
        ws_ptr = ctypes.c_void_p(self._ws.data_ptr() + off)
        with torch.cuda.device(self.device):
            check(L.nr_plan_bind(self._h, ws_ptr, self.workspace_bytes, _stream(self.device)), "nr_plan_bind")

    def autotune(self, cache_path: str | None = None) -> dict:
        """Pick the execution parameters by timing candidates on the device
        (``nr_autotune``: batch budget, streams, spreading tile and item size,
        one at a time), cached per geometry and device in ``cache_path``
        (JSON; None: no cache), then rebind.  Returns the chosen tuning."""
        L = lib()
        need = ctypes.c_size_t()
        check(L.nr_autotune_scratch_bytes(self._h, ctypes.byref(need)), "nr_autotune_scratch_bytes")
        self._ws = None                      # the tuner lays out and binds its own candidates
        torch.cuda.empty_cache()
        try:
            scratch = torch.empty(int(need.value) + 256, dtype=torch.uint8, device=self.device)
            ptr = ctypes.c_void_p(scratch.data_ptr() + (-scratch.data_ptr()) % 256)
            with torch.cuda.device(self.device):
                check(L.nr_autotune(self._h, ptr, int(need.value), cache_path.encode() if cache_path else None,
                                    _stream(self.device)), "nr_autotune")
            del scratch
            torch.cuda.empty_cache()
        finally:
            # whatever happened, the plan gets a workspace of its current layout back
            self._bind()
        self.tuning = {k: self.get_tune(k) for k in ("tile_w", "tile_h", "chunk", "batch_mb", "streams")}
        return dict(self.tuning)

    def get_tune(self, key: str) -> int:
        v = ctypes.c_int64()
        check(lib().nr_plan_get_tune(self._h, key.encode(), ctypes.byref(v)), "nr_plan_get_tune")
        return int(v.value)

    def capture(self, what: str, vol_in: torch.Tensor | None = None, sino: torch.Tensor | None = None,
                vol_out: torch.Tensor | None = None) -> "Graph":
        """Capture 'fwd', 'adj' or 'fwd+adj' over these buffers into one HIP graph."""
        code = {"fwd": 1, "adj": 2, "fwd+adj": 3}[what]
        if code & 1:
            _require(vol_in, self.vol_numel, self.device, "vol_in")
        _require(sino, self.sino_numel, self.device, "sino")
        if code & 2:
            _require(vol_out, self.vol_numel, self.device, "vol_out")
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().nr_graph_capture_radon(self._h, code, _ptr(vol_in) if code & 1 else None, _ptr(sino),
                                               _ptr(vol_out) if code & 2 else None, ctypes.byref(h)),
                  "nr_graph_capture_radon")
        return Graph(h, self, (vol_in, sino, vol_out))

    @classmethod
    def uniform_stack(cls, n: int, n_det: int, angles, n_slices: int = 1, center: float = 0.0, **kw) -> "Plan":
        ang = np.asarray(angles, dtype=np.float64)
        return cls([SliceGeometry(n, n_det, ang, center) for _ in range(n_slices)], **kw)

    # --------------------------------------------------------------- shapes
    @property
    def n_slices(self) -> int:
        return len(self.geoms)

    def vol_shape(self):
        g = self.geoms[0]
        return (self.n_slices, g.n, g.n) if self.uniform else (self.vol_numel,)

    def sino_shape(self):
        g = self.geoms[0]
        return (self.n_slices, len(g.angles), g.n_det) if self.uniform else (self.sino_numel,)

    # ------------------------------------------------------------ operators
    def fwd(self, vol: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Sinograms ``R f`` of every slice (float32)."""
        _require(vol, self.vol_numel, self.device, "vol")
        if out is None:
            out = torch.empty(self.sino_shape(), dtype=torch.float32, device=self.device)
        _require(out, self.sino_numel, self.device, "out")
        with torch.cuda.device(self.device):
            check(lib().radon_fwd(self._h, _ptr(vol), _ptr(out), _stream(self.device)), "radon_fwd")
        return out

    def adj(self, sino: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Back-projections ``R^T y`` of every slice (float32)."""
        _require(sino, self.sino_numel, self.device, "sino")
        if out is None:
            out = torch.empty(self.vol_shape(), dtype=torch.float32, device=self.device)
        _require(out, self.vol_numel, self.device, "out")
        with torch.cuda.device(self.device):
            check(lib().radon_adj(self._h, _ptr(sino), _ptr(out), _stream(self.device)), "radon_adj")
        return out

    def fbp(self, sino: torch.Tensor, out: torch.Tensor | None = None, filter: str = "ramp", order: int = 2,
            cutoff: float = 0.25) -> torch.Tensor:
        """Filtered back-projections of every slice (float32): ``filter`` is
        ``"ramp"`` (|k|) or ``"butterworth"`` (|k| / (1 + (|k|/cutoff)^(2 order)),
        cutoff in cycles per pixel)."""
        codes = {"ramp": NR_FBP_RAMP, "butterworth": NR_FBP_BUTTERWORTH}
        if filter not in codes:
            raise ValueError(f"filter must be one of {sorted(codes)}")
        _require(sino, self.sino_numel, self.device, "sino")
        if out is None:
            out = torch.empty(self.vol_shape(), dtype=torch.float32, device=self.device)
        _require(out, self.vol_numel, self.device, "out")
        params = NrFbp(codes[filter], int(order), float(cutoff))
        with torch.cuda.device(self.device):
            check(lib().radon_fbp(self._h, ctypes.byref(params), _ptr(sino), _ptr(out), _stream(self.device)),
                  "radon_fbp")
        return out

    def stream(self, what: str, host_in: torch.Tensor, host_out: torch.Tensor | None = None,
               filter: str = "ramp", order: int = 2, cutoff: float = 0.25, sync: bool = True) -> torch.Tensor:
        """``what`` = 'fwd', 'adj' or 'fbp' over a host-resident stack of whole
        chunks, the plan describing one chunk: chunk i is copied to the device
        while chunk i-1 is computed and chunk i-2 copied back.  ``host_in`` is a
        float32 CPU tensor holding n_chunks chunks (pinned memory for the copies
        to overlap); ``host_out`` (allocated pinned when None) receives the
        results.  With ``sync`` the call waits until ``host_out`` is complete."""
        codes = {"fwd": NR_STREAM_FWD, "adj": NR_STREAM_ADJ, "fbp": NR_STREAM_FBP}
        if what not in codes:
            raise ValueError(f"what must be one of {sorted(codes)}")
        fcodes = {"ramp": NR_FBP_RAMP, "butterworth": NR_FBP_BUTTERWORTH}
        if filter not in fcodes:
            raise ValueError(f"filter must be one of {sorted(fcodes)}")
        n_in, n_out = (self.vol_numel, self.sino_numel) if what == "fwd" else (self.sino_numel, self.vol_numel)
        if host_in.device.type != "cpu" or host_in.dtype != torch.float32 or not host_in.is_contiguous():
            raise ValueError("host_in must be a contiguous float32 CPU tensor")
        if host_in.numel() % n_in:
            raise ValueError(f"host_in has {host_in.numel()} elements, not a multiple of the chunk's {n_in}")
        n_chunks = host_in.numel() // n_in
        if host_out is None:
            host_out = torch.empty(n_chunks * n_out, dtype=torch.float32, pin_memory=True)
        if (host_out.device.type != "cpu" or host_out.dtype != torch.float32 or not host_out.is_contiguous()
                or host_out.numel() != n_chunks * n_out):
            raise ValueError(f"host_out must be a contiguous float32 CPU tensor of {n_chunks * n_out} elements")
        key = (n_in, n_out)
        if getattr(self, "_stream_key", None) != key:
            self._stream_bufs = [torch.empty(n, dtype=torch.float32, device=self.device)
                                 for n in (n_in, n_in, n_out, n_out)]
            self._stream_key = key
        bufs = self._stream_bufs
        d_in = (ctypes.c_void_p * 2)(bufs[0].data_ptr(), bufs[1].data_ptr())
        d_out = (ctypes.c_void_p * 2)(bufs[2].data_ptr(), bufs[3].data_ptr())
        params = NrFbp(fcodes[filter], int(order), float(cutoff))
        with torch.cuda.device(self.device):
            check(lib().radon_stream(self._h, codes[what], ctypes.byref(params), ctypes.c_void_p(host_in.data_ptr()),
                                     ctypes.c_void_p(host_out.data_ptr()), n_chunks, d_in, d_out,
                                     _stream(self.device)), "radon_stream")
            if sync:
                torch.cuda.current_stream(self.device).synchronize()
        return host_out

    def normal(self, vol: torch.Tensor, b: torch.Tensor | None = None, sino: torch.Tensor | None = None,
               out: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
        """``sino = R vol - b`` (``R vol`` without b) and ``out = R^T sino`` in one call.

        Each batch of slices runs its forward, residual and adjoint back to
        back on one of the plan's streams (no join between the two chains).
        """
        _require(vol, self.vol_numel, self.device, "vol")
        if b is not None:
            _require(b, self.sino_numel, self.device, "b")
        if sino is None:
            sino = torch.empty(self.sino_shape(), dtype=torch.float32, device=self.device)
        if out is None:
            out = torch.empty(self.vol_shape(), dtype=torch.float32, device=self.device)
        _require(sino, self.sino_numel, self.device, "sino")
        _require(out, self.vol_numel, self.device, "out")
        if out.data_ptr() == vol.data_ptr():
            raise ValueError("out must not alias vol")
        with torch.cuda.device(self.device):
            check(lib().radon_normal(self._h, _ptr(vol), _ptr(b) if b is not None else None, _ptr(sino), _ptr(out),
                                     _stream(self.device)), "radon_normal")
        return sino, out

    STAGES = ("fwd_rows", "fwd_cols", "fwd_interp", "adj_radial", "spread", "adj_cols", "adj_rows",
              "residual", "prior", "mbir_update", "spread_clear")

    def profile(self, enable: bool = True) -> None:
        """Bracket every stage launch with HIP events on the launch stream."""
        check(lib().nr_plan_profile(self._h, 1 if enable else 0), "nr_plan_profile")

    def profile_read(self) -> dict:
        """Per stage: (total ms, launches) since the last read; waits for the recorded events."""
        n = len(self.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        with torch.cuda.device(self.device):
            check(lib().nr_plan_profile_read(self._h, ms, cnt, n), "nr_plan_profile_read")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(self.STAGES) if cnt[i]}

    def tune(self, key: str, value: int) -> None:
        check(lib().nr_plan_tune(self._h, key.encode(), int(value)), "nr_plan_tune")

    def check(self) -> None:
        """Synchronise the current stream and raise if a persistent launch of
        this plan gave up waiting for a stage (``nr_plan_check``)."""
        with torch.cuda.device(self.device):
            check(lib().nr_plan_check(self._h, _stream(self.device)), "nr_plan_check")

    def info(self, index: int = 0) -> dict:
        buf = (ctypes.c_int64 * 8)()
        check(lib().nr_plan_info(self._h, index, buf, 8), "nr_plan_info")
        keys = ("G", "tiles", "tile_entries", "spread_items", "poly_degree", "slots", "batches", "launches")
        return dict(zip(keys, list(buf)))

    def close(self) -> None:
        """Destroy the plan (its streams and events) now; the workspace is
        released with the Python object."""
        h = getattr(self, "_h", None)
        self._h = None
        _LIVE.discard(self)
        if h is not None and h.value:
            lib().nr_plan_destroy(h)

    def __enter__(self) -> "Plan":
        return self

    def __exit__(self, *exc) -> None:
        self.close()

    def __del__(self):
        # at interpreter shutdown the process exit releases the handle
        if not sys.is_finalizing():
            try:
                self.close()
            except Exception:
                pass


class Graph:
    """A captured HIP graph (keeps its plan and buffers alive)."""

    def __init__(self, handle: ctypes.c_void_p, plan: Plan, keep: tuple):
        self._h, self.plan, self._keep = handle, plan, keep
        _LIVE.add(self)

    def launch(self) -> None:
        with torch.cuda.device(self.plan.device):
            check(lib().nr_graph_launch(self._h, _stream(self.plan.device)), "nr_graph_launch")

    def close(self) -> None:
        h = getattr(self, "_h", None)
        self._h = None
        _LIVE.discard(self)
        if h is not None and h.value:
            lib().nr_graph_destroy(h)

    def __enter__(self) -> "Graph":
        return self

    def __exit__(self, *exc) -> None:
        self.close()

    def __del__(self):
        if not sys.is_finalizing():
            try:
                self.close()
            except Exception:
                pass


# --------------------------------------------------------------------------
# prior
# --------------------------------------------------------------------------

_WEIGHT_KINDS = {"inv_distance": NR_WEIGHTS_INV_DISTANCE, "gaussian": NR_WEIGHTS_GAUSSIAN}


@dataclass
class Prior:
    """qGGMRF hyper-parameters (defaults: the paper's p = 1.2, sigma = 1/0.7, c = 1e-4).

    ``weights``: ``"inv_distance"`` (w proportional to 1/distance, the
    default), ``"gaussian"``, or an explicit (face, edge, corner) tuple; the
    library fills in the named kinds (``nr_prior_init``)."""
    p: float = 1.2
    sigma: float = 1.0 / 0.7
    c: float = 1e-4
    lam: float = 1.0
    weights: object = "inv_distance"

    def as_c(self) -> NrPrior:
        if isinstance(self.weights, str):
            if self.weights not in _WEIGHT_KINDS:
                raise ValueError(f"weights must be one of {sorted(_WEIGHT_KINDS)} or a (face, edge, corner) tuple")
            out = NrPrior()
            check(lib().nr_prior_init(ctypes.byref(out), self.p, self.sigma, self.c, self.lam,
                                      _WEIGHT_KINDS[self.weights]), "nr_prior_init")
            return out
        wf, we, wc = self.weights
        return NrPrior(self.p, self.sigma, self.c, self.lam, wf, we, wc)

    def lipschitz(self) -> float:
        """A Lipschitz constant of the prior's gradient (``nr_prior_lipschitz``)."""
        out = ctypes.c_double()
        check(lib().nr_prior_lipschitz(ctypes.byref(self.as_c()), ctypes.byref(out)), "nr_prior_lipschitz")
        return float(out.value)


def qggmrf_grad(vol: torch.Tensor, prior: Prior, scale: float = 1.0, grad: torch.Tensor | None = None,
                value: bool = False):
    """``grad += scale * dH/dvol`` for a ``[Z, N, N]`` volume; returns ``(grad, H or None)``."""
    if vol.dim() != 3 or vol.shape[1] != vol.shape[2]:
        raise ValueError("vol must be [Z, N, N]")
    _require(vol, vol.numel(), vol.device, "vol")
    if grad is None:
        grad = torch.zeros_like(vol)
    _require(grad, vol.numel(), vol.device, "grad")
    val = torch.zeros(1, dtype=torch.float64, device=vol.device) if value else None
    pr = prior.as_c()
    with torch.cuda.device(vol.device):
        check(lib().qggmrf_grad(_ptr(vol), vol.shape[0], vol.shape[1], ctypes.byref(pr), float(scale),
                                _ptr(grad), _ptr(val) if value else None, _stream(vol.device)), "qggmrf_grad")
    return grad, (val if value else None)


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------

class RadonFn(torch.autograd.Function):
    """``s = R x`` whose backward is the hand-written adjoint ``R^T g``."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.fwd(x.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.adj(g.contiguous()), None


class DataFidelityFn(torch.autograd.Function):
    """``1/2 ||R x - b||^2`` (float64 scalar); the residual and the half-norm run
    in the library, the backward is the hand-written adjoint of the residual."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan, b: torch.Tensor) -> torch.Tensor:
        _require(b, plan.sino_numel, plan.device, "b")
        xc = x.contiguous()
        _require(xc, plan.vol_numel, plan.device, "x")
        r = torch.empty(plan.sino_shape(), dtype=torch.float32, device=plan.device)
        val = torch.empty(1, dtype=torch.float64, device=plan.device)
        with torch.cuda.device(plan.device):
            check(lib().radon_residual(plan._h, _ptr(xc), _ptr(b), _ptr(r), _ptr(val), _stream(plan.device)),
                  "radon_residual")
        ctx.plan = plan
        ctx.save_for_backward(r)
        return val[0]

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (r,) = ctx.saved_tensors
        grad = ctx.plan.adj(r)
        # scaled on the device whatever g is: testing g == 1 would stall the
        # host until the forward has finished
        return grad.mul_(g.to(grad.dtype)), None, None


class QGGMRFFn(torch.autograd.Function):
    """``H(x)`` (float64 scalar) whose backward is the hand-written prior gradient."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, prior: Prior) -> torch.Tensor:
        grad, val = qggmrf_grad(x.contiguous(), prior, 1.0, None, value=True)
        ctx.save_for_backward(grad)
        return val[0]

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.dtype), None


# --------------------------------------------------------------------------
# MBIR driver
# --------------------------------------------------------------------------

class MBIR:
    """Accelerated-gradient MBIR on the device: one ``mbir_step`` per iteration.

    State ``{x, x_prev, y, grad, t, ...}`` lives on the device; ``step()``
    enqueues one iteration without synchronising the host.  The step size
    is ``1/L``: ``L`` given whole, or ``L_data`` (the largest eigenvalue of
    ``R^T R``) to which the library adds the prior's constant, or neither
    (the library's power iteration).  ``restart``: the gradient restart test;
    ``monotone``: reject a step that raises the objective (one more forward
    projection per iteration).
    """

    def __init__(self, plan: Plan, b: torch.Tensor, prior: Prior, L: float | None = None,
                 nonneg: bool = False, x0: torch.Tensor | None = None, L_data: float | None = None,
                 restart: bool = True, monotone: bool = False):
        if not plan.uniform:
            raise ValueError("MBIR needs a uniform stack (one N for every slice)")
        self.plan, self.b, self.prior = plan, b.contiguous(), prior
        _require(self.b, plan.sino_numel, plan.device, "b")
        shape = plan.vol_shape()
        dev = plan.device
        self.x = torch.zeros(shape, dtype=torch.float32, device=dev) if x0 is None else x0.clone().contiguous()
        self.y = self.x.clone()
        self.x_prev = self.x.clone()
        self.grad = torch.zeros_like(self.x)
        self.scratch = torch.empty(plan.sino_shape(), dtype=torch.float32, device=dev)
        self.state = torch.empty(NR_MBIR_STATE_DOUBLES, dtype=torch.float64, device=dev)
        with torch.cuda.device(dev):
            check(lib().mbir_state_init(_ptr(self.state), _stream(dev)), "mbir_state_init")
        self._prior_c = prior.as_c()
        self.params = NrMbir()
        flags = (1 if restart else 0, 1 if nonneg else 0, 1 if monotone else 0)
        if L is not None:
            check(lib().nr_mbir_params(float(L), None, *flags, ctypes.byref(self.params)), "nr_mbir_params")
        else:
            ld = power_lipschitz(plan) if L_data is None else float(L_data)
            check(lib().nr_mbir_params(ld, ctypes.byref(self._prior_c), *flags, ctypes.byref(self.params)),
                  "nr_mbir_params")
        self.k = 0

    def step(self) -> None:
        with torch.cuda.device(self.plan.device):
            check(lib().mbir_step(self.plan._h, ctypes.byref(self._prior_c), ctypes.byref(self.params),
                                  _ptr(self.b), _ptr(self.x), _ptr(self.x_prev), _ptr(self.y), _ptr(self.grad),
                                  _ptr(self.scratch), _ptr(self.state), _stream(self.plan.device)), "mbir_step")
        self.k += 1

    def run(self, iters: int) -> torch.Tensor:
        for _ in range(iters):
            self.step()
        return self.x

    def capture(self, iters: int = 1) -> Graph:
        """Capture `iters` consecutive mbir_step calls on this state into one HIP graph."""
        h = ctypes.c_void_p()
        with torch.cuda.device(self.plan.device):
            check(lib().nr_graph_capture_mbir(self.plan._h, ctypes.byref(self._prior_c), ctypes.byref(self.params),
                                              _ptr(self.b), _ptr(self.x), _ptr(self.x_prev), _ptr(self.y),
                                              _ptr(self.grad), _ptr(self.scratch), _ptr(self.state), int(iters),
                                              ctypes.byref(h)), "nr_graph_capture_mbir")
        return Graph(h, self.plan, (self.b, self.x, self.x_prev, self.y, self.grad, self.scratch, self.state))

    def step_autograd(self) -> None:
        """Same iteration with the gradient from autograd: ``DataFidelityFn``
        (backward = the hand-written adjoint of the residual) and ``QGGMRFFn``
        (backward = the prior kernel), then the update kernel."""
        y = self.y.detach().requires_grad_(True)
        loss = DataFidelityFn.apply(y, self.plan, self.b)
        if self.prior.lam > 0:
            loss = loss + QGGMRFFn.apply(y, self.prior)
        loss.backward()
        g = y.grad if y.grad.is_contiguous() else y.grad.contiguous()
        with torch.cuda.device(self.plan.device):
            check(lib().mbir_update(ctypes.byref(self.params), _ptr(self.x), _ptr(self.x_prev), _ptr(self.y),
                                    _ptr(g), self.x.numel(), _ptr(self.state), _stream(self.plan.device)),
                  "mbir_update")
        self.grad = g
        self.k += 1

    @property
    def restarts(self) -> int:
        return int(self.state[3].item())

    @property
    def nonfinite(self) -> bool:
        return bool(self.state[2].item() != 0.0)

    @property
    def rejected(self) -> int:
        """Steps the monotone test rejected so far."""
        return int(self.state[10].item())

    @property
    def objective(self) -> float:
        """Objective at x recorded by the last monotone step (NaN before one ran)."""
        st = self.state[5:7].cpu()
        return float(st[0]) if float(st[1]) != 0.0 else float("nan")


class HostMBIR:
    """Accelerated-gradient MBIR over a volume in host memory (Sec. 4.1: the
    partition along the rotation axis streamed through the GPU): one
    ``mbir_stream_iterate`` per iteration.  ``plan`` describes one chunk of
    slices; the volume is ``n_chunks`` chunks stacked in order, and ``b_host``
    their data back to back.  The iterates x_k, x_{k-1} and x_{k+1} live in
    three pinned host buffers that rotate each step; the device holds two
    chunks in flight.  Steps match ``MBIR.step`` (non-monotone) up to float32
    rounding.  ``L``/``L_data`` as for ``MBIR`` (a chunk's power iteration
    gives the volume's ``L_data``: ``R^T R`` acts slice by slice)."""

    def __init__(self, plan: Plan, b_host: torch.Tensor, n_chunks: int, prior: Prior, L: float | None = None,
                 nonneg: bool = False, x0: torch.Tensor | None = None, L_data: float | None = None,
                 restart: bool = True):
        if not plan.uniform:
            raise ValueError("HostMBIR needs a uniform stack (one N for every slice)")
        if n_chunks < 1:
            raise ValueError("n_chunks must be >= 1")
        if (b_host.device.type != "cpu" or b_host.dtype != torch.float32 or not b_host.is_contiguous()
                or b_host.numel() != n_chunks * plan.sino_numel):
            raise ValueError(f"b_host must be a contiguous float32 CPU tensor of {n_chunks * plan.sino_numel} "
                             "elements")
        self.plan, self.prior, self.n_chunks = plan, prior, int(n_chunks)
        self.b = b_host
        nz, n = plan.vol_shape()[0], plan.vol_shape()[1]
        shape = (self.n_chunks * nz, n, n)
        bufs = [torch.zeros(shape, dtype=torch.float32, pin_memory=True) for _ in range(3)]
        if x0 is not None:
            bufs[0].copy_(x0.reshape(shape))
        bufs[1].copy_(bufs[0])
        self._x, self._x_prev, self._x_next = bufs
        size = ctypes.c_size_t()
        check(lib().mbir_stream_work_bytes(plan._h, ctypes.byref(size)), "mbir_stream_work_bytes")
        dev = plan.device
        self.work = torch.empty(max(1, size.value), dtype=torch.uint8, device=dev)
        self.state = torch.empty(NR_MBIR_STATE_DOUBLES, dtype=torch.float64, device=dev)
        with torch.cuda.device(dev):
            check(lib().mbir_state_init(_ptr(self.state), _stream(dev)), "mbir_state_init")
        self._prior_c = prior.as_c()
        self.params = NrMbir()
        flags = (1 if restart else 0, 1 if nonneg else 0, 0)
        if L is not None:
            check(lib().nr_mbir_params(float(L), None, *flags, ctypes.byref(self.params)), "nr_mbir_params")
        else:
            ld = power_lipschitz(plan) if L_data is None else float(L_data)
            check(lib().nr_mbir_params(ld, ctypes.byref(self._prior_c), *flags, ctypes.byref(self.params)),
                  "nr_mbir_params")
        self.k = 0

    def step(self) -> None:
        """Enqueue one iteration; the host buffers must not be touched until
        the plan's device stream is synchronised (``x`` does that)."""
        dev = self.plan.device
        with torch.cuda.device(dev):
            check(lib().mbir_stream_iterate(self.plan._h, ctypes.byref(self._prior_c), ctypes.byref(self.params),
                                            self.n_chunks, _ptr(self.b), _ptr(self._x), _ptr(self._x_prev),
                                            _ptr(self._x_next), _ptr(self.work), self.work.numel(),
                                            _ptr(self.state), _stream(dev)), "mbir_stream_iterate")
        self._x_prev, self._x, self._x_next = self._x, self._x_next, self._x_prev
        self.k += 1

    def run(self, iters: int) -> torch.Tensor:
        for _ in range(iters):
            self.step()
        return self.x

    def reset(self, x0: torch.Tensor | None = None) -> None:
        """Start again from ``x0`` (zeros when None) with a fresh state."""
        dev = self.plan.device
        torch.cuda.current_stream(dev).synchronize()
        if x0 is None:
            self._x.zero_()
        else:
            self._x.copy_(x0.reshape(self._x.shape))
        self._x_prev.copy_(self._x)
        with torch.cuda.device(dev):
            check(lib().mbir_state_init(_ptr(self.state), _stream(dev)), "mbir_state_init")
        self.k = 0

    @property
    def x(self) -> torch.Tensor:
        """The current iterate (host, pinned), after synchronising the stream."""
        torch.cuda.current_stream(self.plan.device).synchronize()
        return self._x

    @property
    def restarts(self) -> int:
        return int(self.state[3].item())

    @property
    def nonfinite(self) -> bool:
        return bool(self.state[2].item() != 0.0)


def stream_stack(what: str, host_in: torch.Tensor, n: int, n_det: int, angles, chunk: int, center: float = 0.0,
                 device: torch.device | str | None = None, filter: str = "ramp", order: int = 2,
                 cutoff: float = 0.25, tuning: dict | None = None) -> torch.Tensor:
    """``what`` = 'fwd', 'adj' or 'fbp' over a host-resident uniform stack of Z
    slices, streamed through the GPU ``chunk`` slices at a time (``Plan.stream``);
    a last, shorter chunk runs on a plan of its own.  Returns a pinned CPU
    tensor ``[Z, n_angles, n_det]`` (fwd) or ``[Z, n, n]``."""
    ang = np.asarray(angles, dtype=np.float64)
    na = len(ang)
    fwd = what == "fwd"
    per_in, per_out = (n * n, na * n_det) if fwd else (na * n_det, n * n)
    if chunk < 1:
        raise ValueError("chunk must be >= 1")
    if host_in.numel() % per_in:
        raise ValueError(f"host_in has {host_in.numel()} elements, not a whole number of slices of {per_in}")
    Z = host_in.numel() // per_in
    host_out = torch.empty((Z, na, n_det) if fwd else (Z, n, n), dtype=torch.float32, pin_memory=True)
    flat_in, flat_out = host_in.reshape(-1), host_out.view(-1)
    full, tail = divmod(Z, chunk)
    kw = dict(filter=filter, order=order, cutoff=cutoff)
    for count, z0, k in ((chunk, 0, full), (tail, full * chunk, 1 if tail else 0)):
        if k == 0:
            continue
        plan = Plan.uniform_stack(n, n_det, ang, count, center=center, device=device, tuning=tuning)
        plan.stream(what, flat_in[z0 * per_in:(z0 + k * count) * per_in],
                    flat_out[z0 * per_out:(z0 + k * count) * per_out], **kw)
    return host_out


def power_lipschitz(plan: Plan, iters: int = 30, seed: int = 0, safety: float = 1.01) -> float:
    """Largest eigenvalue of ``R^T R`` for the plan, times ``safety``
    (``nr_power_lipschitz``: power iteration on the device, float64 norms)."""
    dev = plan.device
    v = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    w = torch.empty_like(v)
    s = torch.empty(plan.sino_numel, dtype=torch.float32, device=dev)
    work = torch.empty(1, dtype=torch.float64, device=dev)
    out = ctypes.c_double()
    with torch.cuda.device(dev):
        check(lib().nr_power_lipschitz(plan._h, int(iters), int(seed) & (2 ** 64 - 1), float(safety), _ptr(v), _ptr(w),
                                       _ptr(s), _ptr(work), ctypes.byref(out), _stream(dev)), "nr_power_lipschitz")
    return float(out.value)


def kb_eval(width: int, beta: float, u: np.ndarray, xi: np.ndarray):
    """Host evaluation of the plan's Kaiser-Bessel tables: (phi(u), phihat(xi), polynomial phi(u))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = max(len(u), len(xi))
    phi, ph, poly = np.zeros(n), np.zeros(n), np.zeros(n)
    P = ctypes.POINTER(ctypes.c_double)
    uu = np.resize(u, n) if len(u) else np.zeros(n)
    xx = np.resize(xi, n) if len(xi) else np.zeros(n)
    check(lib().nr_kb_eval(width, beta, n, uu.ctypes.data_as(P), xx.ctypes.data_as(P), phi.ctypes.data_as(P),
                           ph.ctypes.data_as(P), poly.ctypes.data_as(P)), "nr_kb_eval")
    return phi[:len(u)], ph[:len(xi)], poly[:len(u)]
