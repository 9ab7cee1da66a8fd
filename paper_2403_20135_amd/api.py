"""Python binding of the dSDC library: torch device tensors in, the C ABI underneath.

Every numerical step runs in the HIP library; this module only checks tensor shapes and passes
device pointers and the HIP stream.  There is no CPU path: without the built library or a GPU
the constructor raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import SDCError, check  # noqa: F401  (re-exported)


def _ptr(t) -> int:
    return t.data_ptr()


class SDC:
    """One truncation (and `batch` ensemble members) on the current CUDA/HIP stream of torch."""

    def __init__(self, T: int, nlat: int, nlon: int, M: int, K: int, batch: int = 1,
                 precision: str = "fp64", radius: float = 6.371e6, gravity: float = 9.81,
                 omega: float = 7.292e-5, mean_depth: float = 1.0e4, stream: Optional[int] = None,
                 qdelta: str = "flex", implicit_coriolis: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the dSDC library needs a GPU (no CPU fallback)")
        lib = _lib.load()
        self._torch = torch
        self.cfg = _lib.SdcConfig(T=T, nlat=nlat, nlon=nlon, radius=radius, gravity=gravity,
                                  omega=omega, mean_depth=mean_depth, M=M, K=K, nodes=0,
                                  qdelta=_lib.QDELTAS[qdelta],
                                  precision=_lib.PRECISIONS[precision], batch=batch,
                                  implicit_coriolis=int(bool(implicit_coriolis)))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        check(lib.sdc_init(ctypes.byref(self.cfg), ctypes.c_void_p(stream), ctypes.byref(h)))
        self.h = h
        self.lib = lib
        self.T, self.nlat, self.nlon, self.M, self.K, self.batch = T, nlat, nlon, M, K, batch
        self.ncoef = (T + 1) * (T + 2) // 2

    # ------------------------------------------------------------------ helpers
    def _check(self, t, shape, name):
        torch = self._torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA/HIP tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    @property
    def state_shape(self):
        return (self.batch, 3, self.ncoef, 2)

    @property
    def spec_shape(self):
        return (self.batch, self.ncoef, 2)

    @property
    def grid_shape(self):
        return (self.batch, self.nlat, self.nlon)

    # ------------------------------------------------------------------ C ABI calls
    def step(self, state, dt: float, M: Optional[int] = None, K: Optional[int] = None):
        """One dSDC step in place."""
        self._check(state, self.state_shape, "state")
        check(self.lib.sdc_step(self.h, _ptr(state), float(dt), M or self.M, K or self.K))
        return state

    def step_graph(self, state, dt: float, M: Optional[int] = None, K: Optional[int] = None):
        """One dSDC step in place as a replayed hipGraph (captured on first use per key)."""
        self._check(state, self.state_shape, "state")
        check(self.lib.sdc_step_graph(self.h, _ptr(state), float(dt), M or self.M, K or self.K))
        return state

    def step_sequential(self, state, dt: float, M: Optional[int] = None, K: Optional[int] = None):
        """One sequential IMEX SDC step (Algorithm 1) in place."""
        self._check(state, self.state_shape, "state")
        check(self.lib.sdc_step_sequential(self.h, _ptr(state), float(dt), M or self.M, K or self.K))
        return state

    def step_sequential_graph(self, state, dt: float, M: Optional[int] = None, K: Optional[int] = None):
        self._check(state, self.state_shape, "state")
        check(self.lib.sdc_step_sequential_graph(self.h, _ptr(state), float(dt), M or self.M, K or self.K))
        return state

    def tape_size(self, M: Optional[int] = None, K: Optional[int] = None) -> int:
        """Bytes of the tape of one step (sdc_step_taped)."""
        n = ctypes.c_longlong()
        check(self.lib.sdc_tape_size(self.h, M or self.M, K or self.K, ctypes.byref(n)))
        return n.value

    def new_tape(self, M: Optional[int] = None, K: Optional[int] = None):
        """A device buffer for one step's tape (uint8 tensor)."""
        return self._torch.empty(self.tape_size(M, K), dtype=self._torch.uint8, device="cuda")

    def step_taped(self, state, dt: float, tape, M: Optional[int] = None, K: Optional[int] = None):
        """One dSDC step in place that also records its stages in `tape`."""
        self._check(state, self.state_shape, "state")
        if tape.numel() * tape.element_size() < self.tape_size(M, K):
            raise ValueError("tape too small")
        check(self.lib.sdc_step_taped(self.h, _ptr(state), float(dt), M or self.M, K or self.K, _ptr(tape)))
        return state

    def step_adjoint_taped(self, tape, lam_np1, lam_n, dt: float, M: Optional[int] = None,
                           K: Optional[int] = None):
        """Adjoint of a taped step from its tape (no recomputation)."""
        self._check(lam_np1, self.state_shape, "lam_np1")
        self._check(lam_n, self.state_shape, "lam_n")
        if tape.numel() * tape.element_size() < self.tape_size(M, K):
            raise ValueError("tape too small")
        check(self.lib.sdc_step_adjoint_taped(self.h, _ptr(tape), _ptr(lam_np1), _ptr(lam_n), float(dt),
                                              M or self.M, K or self.K))
        return lam_n

    def imex2_step(self, state, dt: float):
        """One IMEX-o2 step (the paper's reference integrator) in place."""
        self._check(state, self.state_shape, "state")
        check(self.lib.imex2_step(self.h, _ptr(state), float(dt)))
        return state

    def imex2_step_graph(self, state, dt: float):
        """One IMEX-o2 step in place as a replayed hipGraph."""
        self._check(state, self.state_shape, "state")
        check(self.lib.imex2_step_graph(self.h, _ptr(state), float(dt)))
        return state

    def imex2_step_noalloc(self, state, dt: float):
        """One IMEX-o2 step in place with the library's fixed device scratch (no allocation)."""
        self._check(state, self.state_shape, "state")
        check(self.lib.imex2_step_noalloc(self.h, _ptr(state), float(dt)))
        return state

    def step_adjoint(self, state_n, lam_np1, lam_n, dt: float, M: Optional[int] = None,
                     K: Optional[int] = None):
        self._check(state_n, self.state_shape, "state_n")
        self._check(lam_np1, self.state_shape, "lam_np1")
        self._check(lam_n, self.state_shape, "lam_n")
        check(self.lib.sdc_step_adjoint(self.h, _ptr(state_n), _ptr(lam_np1), _ptr(lam_n), float(dt),
                                        M or self.M, K or self.K))
        return lam_n

    def sht_forward(self, grid, spec):
        self._check(grid, self.grid_shape, "grid")
        self._check(spec, self.spec_shape, "spec")
        check(self.lib.sht_forward(self.h, _ptr(grid), _ptr(spec)))
        return spec

    def sht_inverse(self, spec, grid):
        self._check(spec, self.spec_shape, "spec")
        self._check(grid, self.grid_shape, "grid")
        check(self.lib.sht_inverse(self.h, _ptr(spec), _ptr(grid)))
        return grid

    def sht_inverse_adjoint(self, grid, spec):
        self._check(grid, self.grid_shape, "grid")
        self._check(spec, self.spec_shape, "spec")
        check(self.lib.sht_inverse_adjoint(self.h, _ptr(grid), _ptr(spec)))
        return spec

    def imex_solve(self, alpha: float, beta, u):
        self._check(beta, self.state_shape, "beta")
        self._check(u, self.state_shape, "u")
        check(self.lib.imex_solve(self.h, float(alpha), _ptr(beta), _ptr(u)))
        return u

    def eval_explicit(self, u, fE):
        self._check(u, self.state_shape, "u")
        self._check(fE, self.state_shape, "fE")
        check(self.lib.eval_explicit(self.h, _ptr(u), _ptr(fE)))
        return fE

    def eval_implicit(self, u, fI):
        self._check(u, self.state_shape, "u")
        self._check(fI, self.state_shape, "fI")
        check(self.lib.eval_implicit(self.h, _ptr(u), _ptr(fI)))
        return fI

    def sync(self):
        check(self.lib.sdc_sync(self.h))

    def debug_poison(self, on: bool):
        """NaN-fill every step workspace before the launch that writes it (read-before-write check)."""
        check(self.lib.sdc_debug_poison(self.h, int(bool(on))))

    def timing(self, on: bool):
        """Enable/disable per-kernel HIP-event timing on this handle's stream (clears figures)."""
        check(self.lib.sdc_timing_enable(self.h, 1 if on else 0))

    def timing_read(self) -> dict:
        """{class: (total_ms, launches)} accumulated since timing was enabled."""
        out = {}
        for name, k in _lib.KERNEL_CLASSES.items():
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            check(self.lib.sdc_timing_read(self.h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def plan(self) -> dict:
        """The Legendre launch variants in use (see sdc_plan)."""
        pl = _lib.SdcPlan()
        check(self.lib.sdc_get_plan(self.h, ctypes.byref(pl)))
        return {k: getattr(pl, k) for k, _ in pl._fields_}

    def set_plan(self, syn_lat_tiles: int, syn_depth: int, ana_depth: int, ana_interleave: int,
                 fuse_update: int = 1, syn_recur: int = 0, ana_recur: int = 0, node_launch: int = 0):
        """Select the launch variants (see sdc_plan in include/sdc.h); every variant gives bitwise
        the same results."""
        pl = _lib.SdcPlan(syn_lat_tiles, syn_depth, ana_depth, ana_interleave, fuse_update, syn_recur,
                          ana_recur, node_launch)
        check(self.lib.sdc_set_plan(self.h, ctypes.byref(pl)))

    def plan_for(self, states: int) -> dict:
        """The launch variants of the launches over `states` states per member (1 or M)."""
        pl = _lib.SdcPlan()
        check(self.lib.sdc_get_plan_for(self.h, int(states), ctypes.byref(pl)))
        return {k: getattr(pl, k) for k, _ in pl._fields_}

    def set_plan_for(self, states: int, syn_lat_tiles: int, syn_depth: int, ana_depth: int,
                     ana_interleave: int, fuse_update: int = 1, syn_recur: int = 0, ana_recur: int = 0,
                     node_launch: int = 0):
        """Select the variants of the launches over `states` states per member (1 or M)."""
        pl = _lib.SdcPlan(syn_lat_tiles, syn_depth, ana_depth, ana_interleave, fuse_update, syn_recur,
                          ana_recur, node_launch)
        check(self.lib.sdc_set_plan_for(self.h, int(states), ctypes.byref(pl)))

    def autotune(self, reps: int = 10) -> dict:
        """Time every built variant at this handle's step shape and keep the fastest."""
        pl = _lib.SdcPlan()
        check(self.lib.sdc_autotune(self.h, int(reps), ctypes.byref(pl)))
        return {k: getattr(pl, k) for k, _ in pl._fields_}

    def info(self) -> dict:
        inf = _lib.SdcInfo()
        check(self.lib.sdc_get_info(self.h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in inf._fields_}

    def grid(self):
        mu = np.zeros(self.nlat)
        w = np.zeros(self.nlat)
        check(self.lib.sdc_copy_grid(self.h, mu.ctypes.data_as(_lib.P_DOUBLE), w.ctypes.data_as(_lib.P_DOUBLE)))
        return mu, w

    def coefficients(self, M: int):
        tau = np.zeros(M)
        Q = np.zeros(M * M)
        check(self.lib.sdc_copy_coefficients(self.h, M, tau.ctypes.data_as(_lib.P_DOUBLE),
                                             Q.ctypes.data_as(_lib.P_DOUBLE)))
        return tau, Q.reshape(M, M)

    def legendre(self, m: int):
        rows = self.T - m + 1
        P = np.zeros(rows * (self.nlat // 2))
        H = np.zeros_like(P)
        check(self.lib.sdc_copy_legendre(self.h, m, P.ctypes.data_as(_lib.P_DOUBLE),
                                         H.ctypes.data_as(_lib.P_DOUBLE)))
        return P.reshape(rows, -1), H.reshape(rows, -1)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.sdc_free(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SDCGroup:
    """Members of different truncations advanced together: one graph launch per step."""

    def __init__(self, members, stream: Optional[int] = None):
        import torch
        self.members = list(members)
        self.lib = _lib.load()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        arr = (ctypes.c_void_p * len(self.members))(*[m.h.value for m in self.members])
        g = ctypes.c_void_p()
        check(self.lib.sdc_group_create(arr, len(self.members), ctypes.c_void_p(stream), ctypes.byref(g)))
        self.g = g

    @property
    def mode(self) -> int:
        """1: one launch per kernel class and phase over all members; 0: one graph branch each."""
        v = ctypes.c_int()
        check(self.lib.sdc_group_get_mode(self.g, ctypes.byref(v)))
        return v.value

    def set_mode(self, mode: int):
        check(self.lib.sdc_group_set_mode(self.g, int(mode)))

    def step(self, states, dts, M: int, K: int):
        if len(states) != len(self.members) or len(dts) != len(self.members):
            raise ValueError("one state tensor and one dt per member handle")
        for m, s in zip(self.members, states):
            m._check(s, m.state_shape, "state")
        ptrs = (ctypes.c_void_p * len(states))(*[s.data_ptr() for s in states])
        dd = (ctypes.c_double * len(dts))(*[float(d) for d in dts])
        check(self.lib.sdc_group_step(self.g, ptrs, dd, int(M), int(K)))
        return states

    def autotune(self, states, dts, M: int, K: int, reps: int = 5) -> int:
        """Tune the merged launches' variants, time both modes on these states (restored) and keep
        the faster; returns the mode."""
        if len(states) != len(self.members) or len(dts) != len(self.members):
            raise ValueError("one state tensor and one dt per member handle")
        for m, s in zip(self.members, states):
            m._check(s, m.state_shape, "state")
        ptrs = (ctypes.c_void_p * len(states))(*[s.data_ptr() for s in states])
        dd = (ctypes.c_double * len(dts))(*[float(d) for d in dts])
        mode = ctypes.c_int()
        check(self.lib.sdc_group_autotune(self.g, ptrs, dd, int(M), int(K), int(reps), ctypes.byref(mode)))
        return mode.value

    def sync(self):
        check(self.lib.sdc_group_sync(self.g))

    def close(self):
        if getattr(self, "g", None) is not None and self.g.value:
            self.lib.sdc_group_free(self.g)
            self.g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
