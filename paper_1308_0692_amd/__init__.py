"""fdlb on MI355X: the finite-difference lattice Boltzmann method with half-range
Gauss-Hermite velocities (Ghiroldi & Gibelli, arXiv 1308.0692), as hand-written
HIP kernels for gfx950 behind the C ABI of include/fdlb.h.

Python layer: argument marshalling over ctypes; PyTorch provides device memory
and the stream.  Importing this package requires the built libfdlb.so.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (BOTTOM, LEFT, RIGHT, TOP, FdlbError, check, desc_from_case, make_desc,
                   quad_full_range, quad_half_range, tile_count, tile_describe)

__all__ = ["Problem", "Batch", "Mlp", "Hybrid", "FdlbError", "quad_half_range", "quad_full_range", "BOTTOM", "TOP", "LEFT",
           "RIGHT", "tile_count", "tile_describe", "stream_copy", "stream_probe", "set_tune_cache",
           "default_tune_cache"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libfdlb needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _alloc(nbytes: int, device, poison: bool = False):
    """A 256-byte aligned device buffer; poison fills it with 0xFF bytes (NaN as float or double),
    so that a read of memory the library never wrote shows up in the results."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 256) + 256, dtype=torch.uint8, device=device)
    if poison:
        t.fill_(255)
        torch.cuda.current_stream(device).synchronize()
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


class Problem:
    """One boundary-value problem bound to device memory on `device` (default cuda:0)."""

    def __init__(self, case=None, *, precision: Optional[str] = None, allow_unstable: bool = False,
                 device="cuda:0", stream=None, bind: bool = True, desc: Optional[_lib.ProblemDesc] = None,
                 poison: bool = False):
        self.desc = desc if desc is not None else desc_from_case(case, precision, allow_unstable)
        self.precision = _lib.PRECISION_NAMES[self.desc.precision]
        h = C.c_void_p()
        check(_lib.lib.fdlb_problem_create(C.byref(self.desc), C.byref(h)))
        self._h = h
        self.nx, self.ny = self.desc.nx, self.desc.ny
        self.q = _lib.lib.fdlb_problem_q(h)
        self.dt = _lib.lib.fdlb_problem_dt(h)
        self.omega = _lib.lib.fdlb_problem_omega(h)
        self.state_bytes = _lib.lib.fdlb_state_bytes(h)
        self.workspace_bytes = _lib.lib.fdlb_workspace_bytes(h)
        self.device = device
        self._stream = stream
        if bind:
            self.bind(poison=poison)

    # -- memory ----------------------------------------------------------------
    def bind(self, poison: bool = False):
        torch = _torch()
        # A stream of its own (default priority) so that step chunks can be graph-captured.
        s = self._stream if self._stream is not None else torch.cuda.Stream(device=self.device)
        self._stream = s
        self._state_t, self._state = _alloc(self.state_bytes, self.device, poison)
        self._work_t, self._work = _alloc(self.workspace_bytes, self.device, poison)
        check(_lib.lib.fdlb_bind(self._h, C.c_void_p(self._state), C.c_void_p(self._work),
                                 C.c_void_p(s.cuda_stream)))

    @property
    def stream(self):
        return self._stream

    def velocities(self):
        x, y, w = np.empty(self.q), np.empty(self.q), np.empty(self.q)
        check(_lib.lib.fdlb_problem_velocities(self._h, _lib._dp(x), _lib._dp(y), _lib._dp(w)))
        return x, y, w

    # -- initial state -----------------------------------------------------------
    def init_equilibrium(self, rho=None, ux=None, uy=None, renormalize: bool = False):
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
               for a in (rho, ux, uy)]
        check(_lib.lib.fdlb_init_equilibrium(self._h, *[_lib._dp(a) for a in arr], int(renormalize)))

    def init_equilibrium_dev(self, rho, ux, uy, renormalize: bool = True):
        """Seed from device float32 tensors of shape (ny, nx) (e.g. a network's prediction)."""
        torch = _torch()
        ts = [t.contiguous().to(torch.float32) for t in (rho, ux, uy)]
        for t in ts:
            assert t.numel() == self.nx * self.ny and t.is_cuda
        self._stream.wait_stream(torch.cuda.current_stream(self.device))
        ptrs = [C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_float)) for t in ts]
        check(_lib.lib.fdlb_init_equilibrium_dev(self._h, *ptrs, int(renormalize)))
        self._keep = ts

    def upload(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.q, self.ny, self.nx)
        check(_lib.lib.fdlb_state_upload(self._h, _lib._dp(f)))

    def download(self) -> np.ndarray:
        f = np.empty((self.q, self.ny, self.nx))
        check(_lib.lib.fdlb_state_download(self._h, _lib._dp(f)))
        return f

    def checkpoint(self) -> bytes:
        """Exact copy of the carried device state (see fdlb_checkpoint_save)."""
        n = _lib.lib.fdlb_checkpoint_bytes(self._h)
        buf = C.create_string_buffer(n)
        check(_lib.lib.fdlb_checkpoint_save(self._h, C.cast(buf, C.c_void_p)))
        return buf.raw

    def restore(self, data: bytes):
        n = _lib.lib.fdlb_checkpoint_bytes(self._h)
        if len(data) != n:
            raise ValueError(f"checkpoint has {len(data)} bytes, this problem needs {n}")
        buf = C.create_string_buffer(data, n)
        check(_lib.lib.fdlb_checkpoint_load(self._h, C.cast(buf, C.c_void_p)))

    # -- marching ------------------------------------------------------------------
    def step(self, n: int = 1):
        check(_lib.lib.fdlb_step(self._h, int(n)))

    def step_timed(self, n: int):
        """Advance n steps; returns (ms in fused step kernels, ms in reduction kernels) from HIP events."""
        a, b = C.c_double(), C.c_double()
        check(_lib.lib.fdlb_step_timed(self._h, int(n), C.byref(a), C.byref(b)))
        return a.value, b.value

    def last_residual(self):
        r, s = C.c_double(), C.c_int64()
        check(_lib.lib.fdlb_last_residual(self._h, C.byref(r), C.byref(s)))
        return r.value, s.value

    def solve(self, tol: float, max_steps: int, check_every: int = 100, use_graph: bool = True,
              history_cap: int = 0, raise_on_diverge: bool = True) -> dict:
        rep = _lib.Report()
        hist = np.zeros(max(history_cap, 1))
        rep.history_cap = history_cap
        rep.history = _lib._dp(hist) if history_cap else None
        code = _lib.lib.fdlb_solve_steady(self._h, float(tol), int(max_steps), int(check_every),
                                          int(use_graph), C.byref(rep))
        if code == _lib.EDIVERGED and not raise_on_diverge:
            pass
        else:
            check(code, allow=(_lib.OK, _lib.ENOTCONVERGED))
        return dict(status=code, steps=rep.steps, first_below=rep.first_below, residual=rep.residual,
                    wall_s=rep.wall_s, updates_per_s=rep.updates_per_s, bytes_per_s=rep.bytes_per_s,
                    steps_fp32=rep.steps_fp32, history=hist[:rep.history_len].copy())

    # -- outputs ----------------------------------------------------------------------
    def moments(self):
        """(rho, ux, uy, pxy), float64 arrays of shape (ny, nx)."""
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        check(_lib.lib.fdlb_moments(self._h, *[_lib._dp(a) for a in out]))
        return tuple(out)

    def wall_profile(self, wall: int):
        n = self.nx if wall in (BOTTOM, TOP) else self.ny
        out = [np.empty(n) for _ in range(3)]
        check(_lib.lib.fdlb_wall_profile(self._h, int(wall), *[_lib._dp(a) for a in out]))
        return tuple(out)

    def field_samples(self):
        """(inputs, targets) of the warm-start network from the current state: device float32
        tensors of shape (ny * nx, 3) each (fdlb_field_samples)."""
        torch = _torch()
        n = self.nx * self.ny
        a = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        t = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        self._stream.wait_stream(torch.cuda.current_stream(self.device))
        check(_lib.lib.fdlb_field_samples(self._h, C.c_void_p(a.data_ptr()), C.c_void_p(t.data_ptr())))
        torch.cuda.current_stream(self.device).wait_stream(self._stream)
        return a, t

    # -- precision ----------------------------------------------------------------------
    @property
    def active_precision(self) -> str:
        """'fp32' or 'fp64': the kernels the state is marched with now."""
        return _lib.PRECISION_NAMES[check(_lib.lib.fdlb_problem_active_precision(self._h), allow=(0, 1))]

    def promote(self):
        """Mixed precision: widen the float state to double now (fdlb_promote)."""
        check(_lib.lib.fdlb_promote(self._h))

    # -- steady iteration ------------------------------------------------------------------
    def set_pseudo_time(self, on: bool = True):
        """Velocity-local pseudo-time steps for later steps and solves (fdlb_set_pseudo_time)."""
        check(_lib.lib.fdlb_set_pseudo_time(self._h, int(bool(on))))

    def pseudo_weights(self) -> np.ndarray:
        out = np.empty(self.q)
        check(_lib.lib.fdlb_problem_pseudo_weights(self._h, _lib._dp(out)))
        return out

    # -- tiles ------------------------------------------------------------------------
    @property
    def tile(self) -> int:
        return _lib.lib.fdlb_problem_get_tile(self._h)

    def set_tile(self, tile: int):
        check(_lib.lib.fdlb_problem_set_tile(self._h, int(tile)))

    def autotune(self, steps: int = 10) -> float:
        ms = C.c_double()
        check(_lib.lib.fdlb_autotune(self._h, int(steps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            # Work queued on the library's stream must finish before torch may recycle the buffers.
            if getattr(self, "_state_t", None) is not None and self._stream is not None:
                self._stream.synchronize()
            _lib.lib.fdlb_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_copy(dst, src, nbytes: int, stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    check(_lib.lib.fdlb_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                    int(nbytes), C.c_void_p(s.cuda_stream)))


def default_tune_cache() -> str:
    """$FDLB_TUNE_CACHE if set (empty: no cache), else <user cache dir>/fdlb/tiles.txt."""
    import os
    if "FDLB_TUNE_CACHE" in os.environ:
        return os.environ["FDLB_TUNE_CACHE"]
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "fdlb", "tiles.txt")


def set_tune_cache(path: Optional[str]):
    """Cache autotuned tile choices in this text file (fdlb_set_tune_cache); None or "" disables."""
    import os
    if path:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        except OSError:
            pass
    check(_lib.lib.fdlb_set_tune_cache(path.encode() if path else None))


PROBE_MODES = {"plain": 0, "nt_load": 1, "nt_store": 2, "nt": 3, "read": 4, "write": 5}


def stream_probe(dst, src, nbytes: int, mode: str, stream=None):
    """One streaming probe kernel (fdlb_stream_probe) over nbytes; mode is a key of PROBE_MODES."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    check(_lib.lib.fdlb_stream_probe(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr() if src is not None else 0),
                                     int(nbytes), int(PROBE_MODES[mode]), C.c_void_p(s.cuda_stream)))


class Batch:
    """Many independent problems solved together (one launch per step for all of them)."""

    def __init__(self, cases, *, precision: Optional[str] = None, allow_unstable=False, device="cuda:0",
                 stream=None, descs=None, poison: bool = False):
        torch = _torch()
        if descs is None:
            descs = [desc_from_case(c, precision, allow_unstable) for c in cases]
        self.n = len(descs)
        arr = (_lib.ProblemDesc * self.n)(*descs)
        h = C.c_void_p()
        check(_lib.lib.fdlb_batch_create(arr, self.n, C.byref(h)))
        self._h = h
        self.shapes = [(d.nx, d.ny) for d in descs]
        self.qs = [_lib.lib.fdlb_batch_problem_q(h, i) for i in range(self.n)]
        self.precision = _lib.PRECISION_NAMES[descs[0].precision]
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._state_t, self._state = _alloc(_lib.lib.fdlb_batch_state_bytes(h), device, poison)
        self._work_t, self._work = _alloc(_lib.lib.fdlb_batch_workspace_bytes(h), device, poison)
        check(_lib.lib.fdlb_batch_bind(h, C.c_void_p(self._state), C.c_void_p(self._work),
                                       C.c_void_p(self._stream.cuda_stream)))

    @property
    def stream(self):
        return self._stream

    def init_equilibrium(self, i: int, rho=None, ux=None, uy=None, renormalize: bool = False):
        nx, ny = self.shapes[i]
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx)
               for a in (rho, ux, uy)]
        check(_lib.lib.fdlb_batch_init_equilibrium(self._h, int(i), *[_lib._dp(a) for a in arr],
                                                   int(renormalize)))

    def init_equilibrium_dev(self, i: int, rho, ux, uy, renormalize: bool = True):
        torch = _torch()
        ts = [t.contiguous().to(torch.float32) for t in (rho, ux, uy)]
        self._stream.wait_stream(torch.cuda.current_stream(self.device))
        ptrs = [C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_float)) for t in ts]
        check(_lib.lib.fdlb_batch_init_equilibrium_dev(self._h, int(i), *ptrs, int(renormalize)))
        self._stream.synchronize()

    def solve(self, tol: float, max_steps: int, check_every: int = 100, use_graph: bool = True,
              history_cap: int = 0):
        """Returns (status, [report dict per problem])."""
        reps = (_lib.Report * self.n)()
        hists = [np.zeros(max(history_cap, 1)) for _ in range(self.n)]
        for r, h in zip(reps, hists):
            r.history_cap = history_cap
            r.history = _lib._dp(h) if history_cap else None
        code = _lib.lib.fdlb_batch_solve(self._h, float(tol), int(max_steps), int(check_every),
                                         int(use_graph), reps)
        check(code, allow=(_lib.OK, _lib.ENOTCONVERGED, _lib.EDIVERGED))
        out = [dict(status=r.status, steps=r.steps, first_below=r.first_below, residual=r.residual,
                    wall_s=r.wall_s, updates_per_s=r.updates_per_s, steps_fp32=r.steps_fp32,
                    history=h[:r.history_len].copy())
               for r, h in zip(reps, hists)]
        return code, out

    def moments(self, i: int):
        nx, ny = self.shapes[i]
        out = [np.empty((ny, nx)) for _ in range(4)]
        check(_lib.lib.fdlb_batch_moments(self._h, int(i), *[_lib._dp(a) for a in out]))
        return tuple(out)

    def wall_profile(self, i: int, wall: int):
        """(rho, u_t, p_xy) of the face state along one wall of instance i."""
        nx, ny = self.shapes[i]
        n = nx if wall in (BOTTOM, TOP) else ny
        out = [np.empty(n) for _ in range(3)]
        check(_lib.lib.fdlb_batch_wall_profile(self._h, int(i), int(wall), *[_lib._dp(a) for a in out]))
        return tuple(out)

    def upload(self, i: int, f: np.ndarray):
        nx, ny = self.shapes[i]
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (self.qs[i], ny, nx)
        check(_lib.lib.fdlb_batch_state_upload(self._h, int(i), _lib._dp(f)))

    def download(self, i: int, q: Optional[int] = None) -> np.ndarray:
        nx, ny = self.shapes[i]
        if q is not None and q != self.qs[i]:
            raise ValueError(f"instance {i} has {self.qs[i]} velocities, not {q}")
        f = np.empty((self.qs[i], ny, nx))
        check(_lib.lib.fdlb_batch_state_download(self._h, int(i), _lib._dp(f)))
        return f

    def field_samples(self, i: int, out_in=None, out_target=None):
        """Warm-start samples of instance i (see Problem.field_samples); optionally into given
        contiguous float32 device tensors of shape (ny * nx, 3)."""
        torch = _torch()
        nx, ny = self.shapes[i]
        a = out_in if out_in is not None else torch.empty((nx * ny, 3), dtype=torch.float32, device=self.device)
        t = out_target if out_target is not None else torch.empty_like(a)
        assert a.is_contiguous() and t.is_contiguous() and a.numel() == t.numel() == 3 * nx * ny
        self._stream.wait_stream(torch.cuda.current_stream(self.device))
        check(_lib.lib.fdlb_batch_field_samples(self._h, int(i), C.c_void_p(a.data_ptr()), C.c_void_p(t.data_ptr())))
        torch.cuda.current_stream(self.device).wait_stream(self._stream)
        return a, t

    def active_precision(self, i: int) -> str:
        return _lib.PRECISION_NAMES[check(_lib.lib.fdlb_batch_active_precision(self._h, int(i)), allow=(0, 1))]

    def set_pseudo_time(self, on: bool = True):
        """Velocity-local pseudo-time steps for every instance (fdlb_batch_set_pseudo_time)."""
        check(_lib.lib.fdlb_batch_set_pseudo_time(self._h, int(bool(on))))

    def set_retile(self, max_members: int):
        """Tail re-tiling threshold of the solves (fdlb_batch_set_retile); 0 disables."""
        check(_lib.lib.fdlb_batch_set_retile(self._h, int(max_members)))

    @property
    def tile(self) -> int:
        return _lib.lib.fdlb_batch_get_tile(self._h)

    def set_tile(self, tile: int):
        check(_lib.lib.fdlb_batch_set_tile(self._h, int(tile)))

    def autotune(self, steps: int = 5) -> float:
        ms = C.c_double()
        check(_lib.lib.fdlb_batch_autotune(self._h, int(steps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None):
            self._stream.synchronize()
            _lib.lib.fdlb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hybrid:
    """Couette channels with half-range layers at the plates and a full-range bulk (one
    workgroup per channel, state resident in LDS).  ``channels`` is a list of dicts with the
    keys of ``_lib.make_hybrid_desc`` (ny, layer, kn, u_w, n_half, n_full, qx, cfl)."""

    def __init__(self, channels, *, device="cuda:0", stream=None, poison: bool = False):
        torch = _torch()
        descs = [_lib.make_hybrid_desc(**c) for c in channels]
        self.n = len(descs)
        arr = (_lib.HybridDesc * self.n)(*descs)
        h = C.c_void_p()
        check(_lib.lib.fdlb_hybrid_create(arr, self.n, C.byref(h)))
        self._h = h
        self.ny = [d.ny for d in descs]
        self.info = []
        for i in range(self.n):
            ql, qb, sd = C.c_int32(), C.c_int32(), C.c_int64()
            dt, om = C.c_double(), C.c_double()
            check(_lib.lib.fdlb_hybrid_info(h, i, C.byref(ql), C.byref(qb), C.byref(sd), C.byref(dt), C.byref(om)))
            self.info.append(dict(q_layer=ql.value, q_bulk=qb.value, state_doubles=sd.value, dt=dt.value,
                                  omega=om.value))
        self.device = device
        self._stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self._state_t, self._state = _alloc(_lib.lib.fdlb_hybrid_state_bytes(h), device, poison)
        self._work_t, self._work = _alloc(_lib.lib.fdlb_hybrid_workspace_bytes(h), device, poison)
        check(_lib.lib.fdlb_hybrid_bind(h, C.c_void_p(self._state), C.c_void_p(self._work),
                                        C.c_void_p(self._stream.cuda_stream)))

    @property
    def stream(self):
        return self._stream

    def init_equilibrium(self, i: int, rho=None, ux=None, uy=None):
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny[i])
               for a in (rho, ux, uy)]
        check(_lib.lib.fdlb_hybrid_init_equilibrium(self._h, int(i), *[_lib._dp(a) for a in arr]))

    def init_all(self):
        for i in range(self.n):
            self.init_equilibrium(i)

    def set_state(self, i: int, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        assert flat.shape == (self.info[i]["state_doubles"],)
        check(_lib.lib.fdlb_hybrid_set_state(self._h, int(i), _lib._dp(flat)))

    def state(self, i: int) -> np.ndarray:
        out = np.empty(self.info[i]["state_doubles"])
        check(_lib.lib.fdlb_hybrid_get_state(self._h, int(i), _lib._dp(out)))
        return out

    def step(self, n: int):
        check(_lib.lib.fdlb_hybrid_step(self._h, int(n)))

    def solve(self, tol: float, max_steps: int, chunk: int = 0, history_cap: int = 0):
        """Returns (status, [report dict per channel])."""
        reps = (_lib.Report * self.n)()
        hists = [np.zeros(max(history_cap, 1)) for _ in range(self.n)]
        for r, h in zip(reps, hists):
            r.history_cap = history_cap
            r.history = _lib._dp(h) if history_cap else None
        code = _lib.lib.fdlb_hybrid_solve(self._h, float(tol), int(max_steps), int(chunk), reps)
        check(code, allow=(_lib.OK, _lib.ENOTCONVERGED, _lib.EDIVERGED))
        out = [dict(status=r.status, steps=r.steps, first_below=r.first_below, residual=r.residual,
                    wall_s=r.wall_s, updates_per_s=r.updates_per_s, history=h[:r.history_len].copy())
               for r, h in zip(reps, hists)]
        return code, out

    def moments(self, i: int):
        """(rho, u_x, u_y, p_xy) per cell, bottom to top."""
        out = [np.empty(self.ny[i]) for _ in range(4)]
        check(_lib.lib.fdlb_hybrid_moments(self._h, int(i), *[_lib._dp(a) for a in out]))
        return tuple(out)

    def faces(self, i: int) -> np.ndarray:
        """[u_x, p_xy at the bottom plate, u_x, p_xy at the top plate, lower interface flux from
        the layer / bulk cell, upper interface flux from the bulk / layer cell]."""
        out = np.empty(8)
        check(_lib.lib.fdlb_hybrid_faces(self._h, int(i), _lib._dp(out)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._stream.synchronize()
            _lib.lib.fdlb_hybrid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The warm-start network (fdlb_mlp_*): parameters, gradient and Adam moments in device
    float32 tensors owned here, all arithmetic in the library's kernels."""

    def __init__(self, hidden: int = 4, max_batch: int = 8192, seed: int = 0, device="cuda:0", stream=None,
                 params=None, poison: bool = False):
        torch = _torch()
        h = C.c_void_p()
        check(_lib.lib.fdlb_mlp_create(int(hidden), int(max_batch), C.byref(h)))
        self._h = h
        self.hidden, self.max_batch, self.device = hidden, max_batch, device
        self.param_count = int(_lib.lib.fdlb_mlp_param_count(h))
        if params is None:
            host = np.empty(self.param_count, dtype=np.float32)
            check(_lib.lib.fdlb_mlp_init_params(h, C.c_uint64(seed),
                                                host.ctypes.data_as(C.POINTER(C.c_float))))
            params = host
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        assert self.params.numel() == self.param_count
        self.grad = torch.zeros_like(self.params)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self._work_t, self._work = _alloc(_lib.lib.fdlb_mlp_workspace_bytes(h), device, poison)
        self._stream = stream if stream is not None else torch.cuda.Stream(device=device)
        torch.cuda.current_stream(device).synchronize()   # parameter upload and zeroed moments
        check(_lib.lib.fdlb_mlp_bind(h, *[C.c_void_p(t.data_ptr()) for t in
                                          (self.params, self.grad, self.adam_m, self.adam_v)],
                                     C.c_void_p(self._work), C.c_void_p(self._stream.cuda_stream)))
        self.step_count = 0

    @property
    def stream(self):
        return self._stream

    def _enter(self, *tensors):
        torch = _torch()
        for t in tensors:
            if t is not None:
                assert t.is_cuda and t.is_contiguous() and t.dtype in (torch.float32, torch.int32)
        self._stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch = _torch()
        torch.cuda.current_stream(self.device).wait_stream(self._stream)

    def forward(self, x):
        torch = _torch()
        self._enter(x)
        y = torch.empty((x.shape[0], 3), dtype=torch.float32, device=self.device)
        check(_lib.lib.fdlb_mlp_forward(self._h, C.c_void_p(x.data_ptr()), int(x.shape[0]), C.c_void_p(y.data_ptr())))
        self._leave()
        return y

    def backward(self, x, t, rows=None, n: Optional[int] = None):
        """Gradient of the mean squared error into self.grad (asynchronous).  rows: optional
        int32 device tensor selecting the samples (n of them, default all rows)."""
        self._enter(x, t, rows)
        n = int(n if n is not None else (rows.numel() if rows is not None else x.shape[0]))
        rp = C.c_void_p(rows.data_ptr()) if rows is not None else None
        check(_lib.lib.fdlb_mlp_backward(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), rp, n))
        self._leave()

    def last_loss(self) -> float:
        v = C.c_double()
        check(_lib.lib.fdlb_mlp_last_loss(self._h, C.byref(v)))
        return v.value

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._enter()
        self.step_count += 1
        check(_lib.lib.fdlb_mlp_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                          int(self.step_count)))
        self._leave()

    def train_steps(self, x, t, rows, batch: int, lrs, beta1: float = 0.9, beta2: float = 0.999,
                    eps: float = 1e-8):
        """len(lrs) minibatch steps (backward, then Adam) enqueued in one call: step s takes the
        samples rows[s batch : (s + 1) batch] (int32 device tensor) and learning rate lrs[s];
        the same parameters, to the bit, as that many backward / adam_step calls."""
        lr = np.ascontiguousarray(lrs, dtype=np.float64)
        self._enter(x, t, rows)
        check(_lib.lib.fdlb_mlp_train(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                      C.c_void_p(rows.data_ptr()), int(rows.numel()), int(batch), int(lr.size),
                                      _lib._dp(lr), float(beta1), float(beta2), float(eps), int(self.step_count + 1)))
        self.step_count += int(lr.size)
        self._leave()

    def predict_fields(self, kn: float, nx: int, ny: int, u_w: float):
        """Device float32 (rho, ux, uy), each of shape (ny, nx)."""
        torch = _torch()
        out = [torch.empty((ny, nx), dtype=torch.float32, device=self.device) for _ in range(3)]
        self._enter()
        check(_lib.lib.fdlb_mlp_predict_fields(self._h, float(kn), int(nx), int(ny), float(u_w),
                                               *[C.c_void_p(o.data_ptr()) for o in out]))
        self._leave()
        return tuple(out)

    def close(self):
        if getattr(self, "_h", None):
            self._stream.synchronize()
            _lib.lib.fdlb_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
