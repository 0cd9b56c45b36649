"""Thin Python binding of the gqd C ABI (include/gqd.h).

Argument marshalling only: every step of the propagation runs in the HIP library
libgqd.so.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Union

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgqd.so")

TRAP, MIDP = 0, 1
# the paper's elementary, non-geometric methods (Eqs. 13, 14, 16): order 1, 1 and 2,
# not composed, 1D only
EULER_EXPLICIT, EULER_IMPLICIT, SOD = 2, 3, 4
# the diabatic split-operator method (Table I): the surfaces are read as W11, W22, W12
SPLIT_OPERATOR = 5
TRIPLE_JUMP, SUZUKI, OPTIMAL = 0, 1, 2
_METHODS = {"trap": TRAP, "midp": MIDP, "euler_explicit": EULER_EXPLICIT,
            "euler_implicit": EULER_IMPLICIT, "sod": SOD, "split_operator": SPLIT_OPERATOR}
_METHODS.update({v: v for v in list(_METHODS.values())})
_SCHEMES = {"triple_jump": TRIPLE_JUMP, "suzuki": SUZUKI, "optimal": OPTIMAL,
            TRIPLE_JUMP: TRIPLE_JUMP, SUZUKI: SUZUKI, OPTIMAL: OPTIMAL}
SIZES = (256, 512, 1024, 2048, 4096)

STATUS = {0: "OK", -1: "INVALID", -2: "HIP", -3: "NOMEM", -4: "NOT_CONVERGED",
          -5: "UNSUPPORTED", -6: "NONFINITE", -7: "STATE"}


class GqdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gqd {STATUS.get(code, code)}: {msg}")
        self.code = code


class NotConverged(GqdError):
    pass


class _GridDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int), ("surfaces", ctypes.c_int), ("batch", ctypes.c_int),
                ("n", ctypes.POINTER(ctypes.c_int)), ("qmin", ctypes.POINTER(ctypes.c_double)),
                ("qmax", ctypes.POINTER(ctypes.c_double)), ("mass", ctypes.POINTER(ctypes.c_double))]


class _SolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("literal", ctypes.c_int), ("verify", ctypes.c_int), ("precond", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("h_applies", ctypes.c_longlong), ("iterations", ctypes.c_longlong),
                ("iterations_sq", ctypes.c_longlong),
                ("solves", ctypes.c_longlong), ("max_iters", ctypes.c_int),
                ("failures", ctypes.c_int), ("failed_item", ctypes.c_int),
                ("nonfinite", ctypes.c_int), ("alg_bytes", ctypes.c_double),
                ("max_true_resid", ctypes.c_double), ("impl_bytes", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgqd.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run python -m paper_1902_04661_amd.build "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "gqd_create": ([ctypes.POINTER(vp), ctypes.POINTER(_GridDesc)], i),
        "gqd_destroy": ([vp], None),
        "gqd_state_size": ([vp, ctypes.POINTER(ll)], i),
        "gqd_state_offset": ([vp, i, ctypes.POINTER(ll)], i),
        "gqd_workspace_size": ([vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(ctypes.c_size_t)], i),
        "gqd_set_workspace": ([vp, vp, ctypes.c_size_t], i),
        "gqd_set_surfaces": ([vp, vp, vp], i),
        "gqd_apply_H": ([vp, vp, vp, vp], i),
        "gqd_implicit_step": ([vp, i, d, vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(_Stats), vp], i),
        "gqd_propagate": ([vp, i, i, i, d, ll, vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(_Stats), vp], i),
        "gqd_propagate_items": ([vp, i, i, i, vp, vp, vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(_Stats), vp], i),
        "gqd_propagate_noalloc": ([vp, i, i, i, d, ll, vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(_Stats), vp], i),
        "gqd_adjoint": ([vp, i, i, d, ll, vp, vp, vp, ctypes.POINTER(_SolverOpts), ctypes.POINTER(_Stats), vp], i),
        "gqd_autotune": ([vp, i, i, i, d, ll, vp, ctypes.POINTER(_SolverOpts), vp, vp], i),
        "gqd_list_plans": ([i, vp, i, ctypes.POINTER(i)], i),
        "gqd_set_plan": ([vp, i, vp], i),
        "gqd_set_wait_limit": ([vp, i], i),
        "gqd_set_solve_log": ([vp, vp, ll], i),
        "gqd_composition": ([i, i, vp, i, ctypes.POINTER(i)], i),
        "gqd_diag": ([vp, vp, vp, vp], i),
        "gqd_inner": ([vp, vp, vp, vp, vp], i),
        "gqd_last_error": ([], ctypes.c_char_p),
    }
    for name, (argtypes, restype) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    _lib = lib
    return lib


def exported_symbols() -> List[str]:
    return ["gqd_create", "gqd_destroy", "gqd_state_size", "gqd_state_offset",
            "gqd_workspace_size", "gqd_set_workspace", "gqd_set_surfaces", "gqd_apply_H",
            "gqd_implicit_step", "gqd_propagate", "gqd_propagate_items", "gqd_propagate_noalloc", "gqd_adjoint", "gqd_autotune",
            "gqd_list_plans", "gqd_set_plan", "gqd_set_wait_limit", "gqd_set_solve_log", "gqd_composition",
            "gqd_diag", "gqd_inner",
            "gqd_last_error"]


def _check(code: int):
    if code != 0:
        msg = _lib.gqd_last_error().decode()
        if code == -4:
            raise NotConverged(code, msg)
        raise GqdError(code, msg)


@dataclass
class SolverOpts:
    tol: float = 1e-13
    restart: int = 32
    maxit: int = 1000
    literal: bool = False
    verify: bool = False  # end a solve only on a true residual within tol (restart otherwise)
    # right-precondition GMRES by (1 + i a p^2 / 2m)^-1 (1D); "auto": per size class,
    # where the kinetic stiffness a T_max of the call exceeds 1.25
    precond: Union[bool, str] = False

    def c(self) -> _SolverOpts:
        if isinstance(self.precond, str):
            if self.precond != "auto":
                raise ValueError(f"precond must be a bool or 'auto', not {self.precond!r}")
            pc = 2
        else:
            pc = int(bool(self.precond))
        return _SolverOpts(float(self.tol), int(self.restart), int(self.maxit), int(bool(self.literal)),
                           int(bool(self.verify)), pc)


@dataclass
class Stats:
    h_applies: int
    iterations: int
    iterations_sq: int
    solves: int
    max_iters: int
    failures: int
    failed_item: int
    nonfinite: int
    alg_bytes: float
    max_true_resid: float
    impl_bytes: float


def _stats(st) -> Optional[Stats]:
    if st is None:
        return None
    return Stats(st.h_applies, st.iterations, st.iterations_sq, st.solves, st.max_iters,
                 st.failures, st.failed_item, st.nonfinite, st.alg_bytes, st.max_true_resid, st.impl_bytes)


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def list_plans(n: int) -> List[tuple]:
    """Radices (R0, R1, R2, R3) of every transform plan of 1D size n, default first."""
    load_library()
    buf = (ctypes.c_int * 64)()
    cnt = ctypes.c_int()
    _check(_lib.gqd_list_plans(int(n), buf, 16, ctypes.byref(cnt)))
    return [tuple(buf[4 * k + i] for i in range(4)) for k in range(cnt.value)]


def composition(scheme, order: int) -> np.ndarray:
    """Substep fractions tau_c of one composed step, in order of application."""
    load_library()
    cnt = ctypes.c_int()
    _check(_lib.gqd_composition(_SCHEMES[scheme], int(order), None, 0, ctypes.byref(cnt)))
    buf = (ctypes.c_double * cnt.value)()
    _check(_lib.gqd_composition(_SCHEMES[scheme], int(order), buf, cnt.value, ctypes.byref(cnt)))
    return np.array(buf[:], dtype=np.float64)


class Propagator:
    """A batch of 1D two-surface wavepackets on one GPU.

    n, qmin, qmax: per item; mass: nuclear mass.  V (batch of [2][n]) and F ([n])
    are given as numpy arrays or device tensors and kept on the device.
    """

    dims = 1

    def __init__(self, n: Sequence[int], qmin: Sequence[float], qmax: Sequence[float],
                 mass: float, V=None, F=None, device: str = "cuda"):
        lib = load_library()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n = np.asarray(n, dtype=np.int32).ravel()
        self.batch = int(self.n.size)
        self.qmin = np.broadcast_to(np.asarray(qmin, dtype=np.float64), (self.batch,)).copy()
        self.qmax = np.broadcast_to(np.asarray(qmax, dtype=np.float64), (self.batch,)).copy()
        self.mass = float(mass)
        self._mass = np.array([self.mass], dtype=np.float64)
        desc = _GridDesc(1, 2, self.batch,
                         self.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                         self.qmin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self.qmax.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self._mass.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._create(desc, np.concatenate([[0], np.cumsum(2 * self.n.astype(np.int64))]),
                     [(2, int(k)) for k in self.n], V, F)
        self.f_size = self.state_size // 2
        self._finish_init()

    def _create(self, desc, offsets, shapes, V, F):
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)))
        self._h = h
        total = ctypes.c_longlong()
        _check(_lib.gqd_state_size(h, ctypes.byref(total)))
        self.state_size = int(total.value)
        self.offsets = offsets
        self.shapes = shapes
        self._work = None
        self._work_m = -1
        self._log = None
        self.V = None
        self.F = None
        self._pending_surfaces = (V, F)

    def _finish_init(self):
        V, F = self._pending_surfaces
        del self._pending_surfaces
        if V is not None and F is not None:
            self.set_surfaces(V, F)

    def close(self) -> None:
        """Destroy the handle now (device tables, side streams and events), with the HIP
        runtime still up.  Waits for the device first.  Later calls raise."""
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            torch.cuda.synchronize(self.device)
            _lib.gqd_destroy(h)
        self._h = None
        self._work = None
        self._log = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        # a handle that was never closed is freed here; at interpreter exit the library
        # may already be gone, so close() is the dependable way
        try:
            if getattr(self, "_h", None) is not None and _lib is not None:
                _lib.gqd_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # -------------------------------------------------------------- data layout
    def pack(self, arrays) -> torch.Tensor:
        """Concatenate per-item complex arrays of shape (2, n_b) into one device state."""
        flat = np.concatenate([np.asarray(a, dtype=np.complex128).reshape(-1) for a in arrays])
        assert flat.size == self.state_size
        return torch.from_numpy(flat).to(self.device)

    def unpack(self, psi: torch.Tensor) -> List[np.ndarray]:
        host = psi.detach().cpu().numpy()
        return [host[self.offsets[b]:self.offsets[b + 1]].reshape(self.shapes[b]) for b in range(self.batch)]

    def set_surfaces(self, V, F):
        """V: per-item (2, *grid) float64 (or a flat device tensor); F: per-item F12 along
        each dimension, (D, *grid) (1D also (n_b,))."""
        if isinstance(V, torch.Tensor):
            Vt = V.to(self.device, torch.float64).contiguous().reshape(-1)
        else:
            Vt = torch.from_numpy(np.concatenate([np.asarray(v, np.float64).reshape(-1) for v in V])).to(self.device)
        if isinstance(F, torch.Tensor):
            Ft = F.to(self.device, torch.float64).contiguous().reshape(-1)
        else:
            Ft = torch.from_numpy(np.concatenate([np.asarray(f, np.float64).reshape(-1) for f in F])).to(self.device)
        if Vt.numel() != self.state_size or Ft.numel() != self.f_size:
            raise ValueError("V or F has the wrong size for this grid")
        self.V, self.F = Vt, Ft
        _check(_lib.gqd_set_surfaces(self._h, ctypes.c_void_p(Vt.data_ptr()), ctypes.c_void_p(Ft.data_ptr())))

    def _ensure_workspace(self, opts: SolverOpts):
        if self._work is not None and self._work_m >= opts.restart:
            return
        nbytes = ctypes.c_size_t()
        co = opts.c()
        _check(_lib.gqd_workspace_size(self._h, ctypes.byref(co), ctypes.byref(nbytes)))
        self._work = torch.empty(int(nbytes.value) // 16 + 1, dtype=torch.complex128, device=self.device)
        self._work_m = opts.restart
        _check(_lib.gqd_set_workspace(self._h, ctypes.c_void_p(self._work.data_ptr()), self._work.numel() * 16))

    def _state(self, psi: torch.Tensor) -> ctypes.c_void_p:
        if psi.dtype != torch.complex128 or not psi.is_contiguous() or psi.numel() != self.state_size \
                or psi.device != self.device:
            raise ValueError("state must be a contiguous complex128 device tensor of state_size elements")
        return ctypes.c_void_p(psi.data_ptr())

    # ------------------------------------------------------------------- calls
    def apply_H(self, psi: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        out = torch.empty_like(psi) if out is None else out
        if self.dims == 2:
            self._ensure_workspace(SolverOpts(restart=max(self._work_m, 1)))
        _check(_lib.gqd_apply_H(self._h, self._state(psi), self._state(out), _stream_ptr(stream)))
        return out

    def propagate(self, psi: torch.Tensor, method="midp", scheme="suzuki", order: int = 2,
                  dt: float = 1.0, nsteps: int = 1, opts: Optional[SolverOpts] = None,
                  stats: bool = True, stream=None) -> Optional[Stats]:
        """In place: nsteps composed steps.  With stats=True the call waits and returns
        solver counters (and raises NotConverged if any solve hit maxit)."""
        opts = opts or SolverOpts()
        self._ensure_workspace(opts)
        co = opts.c()
        st = _Stats() if stats else None
        _check(_lib.gqd_propagate(self._h, _METHODS[method], _SCHEMES[scheme], int(order), float(dt),
                                  int(nsteps), self._state(psi), ctypes.byref(co),
                                  ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
        return _stats(st)

    def propagate_noalloc(self, psi: torch.Tensor, method="midp", scheme="suzuki", order: int = 2,
                          dt: float = 1.0, nsteps: int = 1, opts: Optional[SolverOpts] = None,
                          stats: bool = True, stream=None) -> Optional[Stats]:
        """As propagate, in the library's static workspace: no device allocation (neither
        here nor in the library); calls on one GPU must not overlap."""
        opts = opts or SolverOpts()
        co = opts.c()
        st = _Stats() if stats else None
        _check(_lib.gqd_propagate_noalloc(self._h, _METHODS[method], _SCHEMES[scheme], int(order), float(dt),
                                          int(nsteps), self._state(psi), ctypes.byref(co),
                                          ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
        return _stats(st)

    def propagate_items(self, psi: torch.Tensor, method="midp", scheme="suzuki", order: int = 2,
                        dt=None, nsteps=None, opts: Optional[SolverOpts] = None,
                        stats: bool = True, stream=None) -> Optional[Stats]:
        """In place, item b takes nsteps[b] composed steps of dt[b] (one launch)."""
        opts = opts or SolverOpts()
        self._ensure_workspace(opts)
        dt_t = torch.as_tensor(np.asarray(dt, dtype=np.float64).reshape(self.batch)).to(self.device)
        ns_t = torch.as_tensor(np.asarray(nsteps, dtype=np.int64).reshape(self.batch)).to(self.device)
        co = opts.c()
        st = _Stats() if stats else None
        _check(_lib.gqd_propagate_items(self._h, _METHODS[method], _SCHEMES[scheme], int(order),
                                        ctypes.c_void_p(dt_t.data_ptr()), ctypes.c_void_p(ns_t.data_ptr()),
                                        self._state(psi), ctypes.byref(co),
                                        ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
        if st is None:
            self._keep = (dt_t, ns_t)  # alive until the caller synchronises
        return _stats(st)

    def set_plan(self, n: int, radices) -> None:
        """Use the transform plan with these radices for items of size n."""
        r = (ctypes.c_int * 4)(*[int(x) for x in radices])
        _check(_lib.gqd_set_plan(self._h, int(n), r))

    def set_solve_log(self, per_item: int) -> None:
        """Record the Arnoldi iteration count of each of the first per_item solves of
        every item in later calls (0 switches the record off); read it with solve_log()."""
        if per_item > 0:
            self._log = torch.full((self.batch, int(per_item)), -1, dtype=torch.int32, device=self.device)
            _check(_lib.gqd_set_solve_log(self._h, ctypes.c_void_p(self._log.data_ptr()), int(per_item)))
        else:
            _check(_lib.gqd_set_solve_log(self._h, None, 0))
            self._log = None

    def solve_log(self, clear: bool = True) -> np.ndarray:
        """(batch, per_item) iteration counts of the last calls' solves (-1: no solve)."""
        if self._log is None:
            raise ValueError("no solve log set (set_solve_log)")
        out = self._log.cpu().numpy().copy()
        if clear:
            self._log.fill_(-1)
        return out

    def set_wait_limit(self, polls: int) -> None:
        """Polls a 2D grid wait makes before the item gives up (0: the default)."""
        _check(_lib.gqd_set_wait_limit(self._h, int(polls)))

    def autotune(self, psi: torch.Tensor, method="midp", scheme="suzuki", order: int = 2,
                 dt: float = 1.0, nsteps: int = 1, opts: Optional[SolverOpts] = None, stream=None):
        """Pick the fastest transform plan per grid size on a copy of psi (psi itself is
        left alone); returns {N: radices} for the sizes present."""
        opts = opts or SolverOpts()
        self._ensure_workspace(opts)
        scratch = psi.detach().clone()
        co = opts.c()
        rad = (ctypes.c_int * 20)()
        _check(_lib.gqd_autotune(self._h, _METHODS[method], _SCHEMES[scheme], int(order), float(dt),
                                 int(nsteps), self._state(scratch), ctypes.byref(co), rad, _stream_ptr(stream)))
        out = {}
        for c, n in enumerate(SIZES):
            r = tuple(rad[4 * c + k] for k in range(4))
            if any(r):
                out[n] = r
        return out

    def implicit_step(self, psi: torch.Tensor, method="midp", dt: float = 1.0,
                      opts: Optional[SolverOpts] = None, stats: bool = True, stream=None):
        opts = opts or SolverOpts()
        self._ensure_workspace(opts)
        co = opts.c()
        st = _Stats() if stats else None
        _check(_lib.gqd_implicit_step(self._h, _METHODS[method], float(dt), self._state(psi), ctypes.byref(co),
                                      ctypes.byref(st) if st is not None else None, _stream_ptr(stream)))
        return _stats(st)

    def adjoint(self, psi: torch.Tensor, lam: torch.Tensor, gF: torch.Tensor, scheme="suzuki",
                order: int = 2, dt: float = 1.0, nsteps: int = 1, opts: Optional[SolverOpts] = None,
                stats: bool = True, stream=None):
        """In place reverse sweep: psi(T) -> psi(0), lam = dL/dpsi*(T) -> (0); gF += dL/dF12."""
        opts = opts or SolverOpts()
        self._ensure_workspace(opts)
        if gF.dtype != torch.float64 or gF.numel() != self.f_size or not gF.is_contiguous():
            raise ValueError("gF must be a contiguous float64 tensor with one entry per grid point and dimension")
        co = opts.c()
        st = _Stats() if stats else None
        _check(_lib.gqd_adjoint(self._h, _SCHEMES[scheme], int(order), float(dt), int(nsteps),
                                self._state(psi), self._state(lam), ctypes.c_void_p(gF.data_ptr()),
                                ctypes.byref(co), ctypes.byref(st) if st is not None else None,
                                _stream_ptr(stream)))
        return _stats(st)

    def diag(self, psi: torch.Tensor, stream=None) -> torch.Tensor:
        """(batch, 4): norm, energy, population of surface 1, of surface 2."""
        out = torch.empty(self.batch * 4, dtype=torch.float64, device=self.device)
        if self.dims == 2:
            self._ensure_workspace(SolverOpts(restart=max(self._work_m, 1)))
        _check(_lib.gqd_diag(self._h, self._state(psi), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out.reshape(self.batch, 4)

    def inner(self, psi: torch.Tensor, phi: torch.Tensor, stream=None) -> torch.Tensor:
        out = torch.empty(self.batch * 2, dtype=torch.float64, device=self.device)
        _check(_lib.gqd_inner(self._h, self._state(psi), self._state(phi), ctypes.c_void_p(out.data_ptr()),
                              _stream_ptr(stream)))
        o = out.reshape(self.batch, 2)
        return torch.complex(o[:, 0], o[:, 1])


class Propagator2D(Propagator):
    """A batch of two-surface wavepackets on n x n grids (n in 64, 128, 256, 512).

    State of one item: (2, n, n) complex128, q1 the slow and q2 the fast index.
    qmin, qmax: (batch, 2) or (2,) bounds per item and axis; mass: (m1, m2).
    V: per-item (2, n, n); F: per-item (2, n, n), F12 along q1 and along q2.
    A group of workgroups shares each item; every call runs as cooperative launches.
    """
    dims = 2

    def __init__(self, n: int, qmin, qmax, mass, V=None, F=None, batch: Optional[int] = None,
                 device: str = "cuda"):
        load_library()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        qmin = np.asarray(qmin, dtype=np.float64).reshape(-1, 2)
        qmax = np.asarray(qmax, dtype=np.float64).reshape(-1, 2)
        self.batch = int(batch if batch is not None else max(qmin.shape[0], qmax.shape[0]))
        self.qmin = np.ascontiguousarray(np.broadcast_to(qmin, (self.batch, 2)))
        self.qmax = np.ascontiguousarray(np.broadcast_to(qmax, (self.batch, 2)))
        self.n2 = int(n)
        self.n = np.full(2 * self.batch, self.n2, dtype=np.int32)
        self._mass = np.asarray(mass, dtype=np.float64).reshape(2).copy()
        self.mass = tuple(float(x) for x in self._mass)
        desc = _GridDesc(2, 2, self.batch,
                         self.n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                         self.qmin.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self.qmax.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self._mass.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        per = 2 * self.n2 * self.n2
        self._create(desc, np.arange(self.batch + 1, dtype=np.int64) * per,
                     [(2, self.n2, self.n2)] * self.batch, V, F)
        self.f_size = self.state_size
        self._finish_init()

    def propagate_items(self, *args, **kwargs):
        raise GqdError(-5, "per-item steps are available on 1D grids")


def from_items(items, device: str = "cuda") -> Propagator:
    """Propagator for a list of input items (objects with n, qmin, qmax, mass, V, F):
    1D items give a Propagator, 2D items (n a pair) a Propagator2D."""
    if np.ndim(items[0].n) == 1:
        n = {tuple(int(k) for k in it.n) for it in items}
        masses = {tuple(float(x) for x in it.mass) for it in items}
        if len(n) != 1 or len(masses) != 1:
            raise ValueError("2D items must share one grid size and one pair of masses")
        n1, n2 = n.pop()
        if n1 != n2:
            raise GqdError(-5, "2D grids must be n x n")
        return Propagator2D(n1, [it.qmin for it in items], [it.qmax for it in items], masses.pop(),
                            [it.V for it in items], [it.F for it in items], batch=len(items), device=device)
    masses = {float(it.mass) for it in items}
    if len(masses) != 1:
        raise ValueError("all items must share one mass")
    return Propagator([it.n for it in items], [it.qmin for it in items], [it.qmax for it in items],
                      masses.pop(), [it.V for it in items], [it.F for it in items], device=device)
