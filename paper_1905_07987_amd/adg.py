"""ctypes binding of libadg (include/adg.h).

Argument marshalling only: every step of the ADER-DG path runs in the HIP
kernels of ``libadg.so``.  Device arrays are torch tensors (float64,
contiguous, on the context's GPU); their raw pointers and torch's current HIP
stream are handed to the C ABI.  There is no CPU fallback: if the library is
missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadg.so")

PDE_EULER, PDE_ELASTIC, PDE_ADVECTION = 1, 2, 3
FP64, MIXED_FP32, MIXED_BF16X3 = 0, 1, 2
GUESS_CONSTANT, GUESS_CERK = 0, 1
_GUESS_NAMES = {"constant": GUESS_CONSTANT, "cerk": GUESS_CERK}
STEP_NEXT_DT = 1
STEP_REUSE_RANGES = 2

PDE_USER = 4
_PDE_NAMES = {"euler": PDE_EULER, "elastic": PDE_ELASTIC, "advection": PDE_ADVECTION, "user": PDE_USER}
_PREC_NAMES = {"fp64": FP64, "fp32": MIXED_FP32, "mixed_fp32": MIXED_FP32, "bf16x3": MIXED_BF16X3,
               "mixed_bf16x3": MIXED_BF16X3}


class AdgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libadg status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("order", C.c_int), ("pde", C.c_int), ("precision", C.c_int),
        ("cells", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("cfl", C.c_double), ("picard_iters", C.c_int), ("initial_guess", C.c_int),
        ("gamma", C.c_double), ("adv", C.c_double * 3), ("kappa", C.c_double),
        ("bc", C.c_int * 6),
        ("bc_state", (C.c_double * 16) * 6),
    ]


BC_PERIODIC, BC_OUTFLOW, BC_WALL, BC_INFLOW, BC_USER = 0, 1, 2, 3, 4
_BC_NAMES = {"periodic": BC_PERIODIC, "outflow": BC_OUTFLOW, "wall": BC_WALL, "inflow": BC_INFLOW,
             "user": BC_USER}


class Info(C.Structure):
    _fields_ = [
        ("nvar", C.c_int), ("nparam", C.c_int), ("nodes_per_cell", C.c_int), ("face_nodes", C.c_int),
        ("ncells", C.c_longlong), ("state_elems", C.c_longlong), ("workspace_bytes", C.c_size_t),
        ("trace_elems", C.c_size_t),
    ]


class PointSource(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("weight", C.c_double * 16), ("f0", C.c_double),
                ("t0", C.c_double), ("amp", C.c_double)]


_lib = None


def lib():
    """Load libadg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.adg_last_error.restype = C.c_char_p
        L.adg_max_order.argtypes = [C.c_int, C.c_int]
        L.adg_basis_tables.argtypes = [C.c_int] + [dp] * 6
        L.adg_create.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.adg_create_user.argtypes = [C.POINTER(Config), C.c_char_p, C.POINTER(vp)]
        L.adg_destroy.argtypes = [vp]
        L.adg_query.argtypes = [vp, C.POINTER(Info)]
        L.adg_node_coords.argtypes = [vp, dp]
        L.adg_stable_dt.argtypes = [vp, vp, vp, vp, vp]
        L.adg_step.argtypes = [vp, vp, vp, vp, C.c_int, vp]
        L.adg_step_noalloc.argtypes = [vp, vp, vp, vp, C.c_int, vp]
        L.adg_read_clock_host.argtypes = [vp, dp, vp]
        L.adg_run.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp]
        L.adg_run_reserve.argtypes = [vp]
        L.adg_predict.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.adg_correct.argtypes = [vp, vp, vp, vp, C.c_int, vp]
        L.adg_check_admissible.argtypes = [vp, vp, vp, vp, vp, vp]
        L.adg_set_point_sources.argtypes = [vp, C.c_int, C.POINTER(PointSource)]
        L.adg_set_receivers.argtypes = [vp, C.c_int, dp]
        L.adg_sample_receivers.argtypes = [vp, vp, vp, vp]
        L.adg_step_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.adg_keep_size.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.adg_step_keep.argtypes = [vp, vp, vp, vp, vp, vp]
        L.adg_run_keep.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L.adg_step_adjoint_kept.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.adg_sample_receivers_adjoint.argtypes = [vp, vp, vp, vp]
        L.adg_limiter_tables.argtypes = [C.c_int, dp, dp, dp]
        L.adg_step_limited.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.c_int, vp]
        L.adg_limiter_reserve.argtypes = [vp]
        _lib = L
    return _lib


def limiter_tables(order: int):
    """Host-only: (A [m][n], B [n][m], Qf [n][m]) of the subcell limiter,
    n = order + 1, m = 2 order + 1."""
    n, m = max(order + 1, 1), max(2 * order + 1, 1)  # the library refuses a bad order
    A, B, Qf = np.zeros((m, n)), np.zeros((n, m)), np.zeros((n, m))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(lib().adg_limiter_tables(order, dp(A), dp(B), dp(Qf)))
    return A, B, Qf


EXPORTED = ("adg_last_error", "adg_max_order", "adg_basis_tables", "adg_create", "adg_create_user", "adg_destroy",
            "adg_query", "adg_node_coords", "adg_stable_dt", "adg_read_clock_host", "adg_step", "adg_step_noalloc", "adg_run",
            "adg_run_reserve",
            "adg_predict",
            "adg_correct",
            "adg_check_admissible", "adg_set_point_sources", "adg_set_receivers",
            "adg_sample_receivers", "adg_step_adjoint", "adg_sample_receivers_adjoint",
            "adg_keep_size", "adg_step_keep", "adg_run_keep", "adg_step_adjoint_kept",
            "adg_limiter_tables", "adg_limiter_reserve", "adg_step_limited")


def _check(st: int):
    if st != 0:
        raise AdgError(st, lib().adg_last_error().decode())


def max_order(pde: str | int, dim: int) -> int:
    return lib().adg_max_order(_PDE_NAMES.get(pde, pde), dim)


def basis_tables(order: int) -> dict:
    """Host-side tables of the library (no GPU needed)."""
    n = order + 1
    xi, w, l0, l1 = (np.zeros(n) for _ in range(4))
    D, Ki = np.zeros((n, n)), np.zeros((n, n))
    p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    _check(lib().adg_basis_tables(order, p(xi), p(w), p(D), p(l0), p(l1), p(Ki)))
    return dict(xi=xi, w=w, D=D, l0=l0, l1=l1, K1inv=Ki)


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One ADER-DG problem on the current GPU (a libadg context)."""

    def __init__(self, dim: int, order: int, pde="euler", cells=(16, 16, 1), lo=(0.0, 0.0, 0.0),
                 hi=(1.0, 1.0, 1.0), cfl: float = 0.9, picard_iters: int = 0, precision="fp64",
                 gamma: float = 1.4, adv=(1.0, 1.0, 1.0), kappa: float = 0.0, bc=None, bc_state=None,
                 source: str | None = None, initial_guess="constant"):
        cfg = Config()
        cfg.initial_guess = _GUESS_NAMES.get(initial_guess, initial_guess)
        for f, b in enumerate(bc or ()):
            cfg.bc[f] = _BC_NAMES.get(b, b)
        for f, q in (bc_state or {}).items():
            for v, x in enumerate(q):
                cfg.bc_state[f][v] = x
        cfg.dim, cfg.order = dim, order
        cfg.pde = _PDE_NAMES.get(pde, pde)
        cfg.precision = _PREC_NAMES.get(precision, precision)
        cells = list(cells) + [1] * (3 - len(cells))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        adv = list(adv) + [0.0] * (3 - len(adv))
        for d in range(3):
            cfg.cells[d], cfg.lo[d], cfg.hi[d], cfg.adv[d] = cells[d], lo[d], hi[d], adv[d]
        cfg.cfl, cfg.picard_iters, cfg.gamma, cfg.kappa = cfl, picard_iters, gamma, kappa
        self.cfg = cfg
        self._ctx = C.c_void_p()
        if source is not None:
            # a PDE given as HIP source text (struct AdgUserPDE), compiled now
            cfg.pde = PDE_USER
            _check(lib().adg_create_user(C.byref(cfg), source.encode(), C.byref(self._ctx)))
        else:
            _check(lib().adg_create(C.byref(cfg), C.byref(self._ctx)))
        info = Info()
        _check(lib().adg_query(self._ctx, C.byref(info)))
        self.info = info
        self.dim, self.order, self.n = dim, order, order + 1
        self.nvar, self.nparam = info.nvar, info.nparam
        self.S, self.F, self.ncells = info.nodes_per_cell, info.face_nodes, info.ncells
        self.nrec = 0
        self._limiter_ready = False
        self._run_ready = False

    def close(self):
        if self._ctx:
            lib().adg_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    @property
    def state_shape(self):
        return (self.ncells, self.nvar, self.S)

    @property
    def trace_shape(self):
        return (self.ncells, 2 * self.dim, 2, self.nvar, self.F)

    def _dev(self, t, shape=None, dtype=None, name="array"):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name} must have dtype {dtype}")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        return C.c_void_p(t.data_ptr())

    def _params(self, params):
        import torch
        if self.nparam == 0:
            return C.c_void_p()
        if params is None:
            raise ValueError("this PDE needs material parameters [ncells, nparam]")
        return self._dev(params, (self.ncells, self.nparam), torch.float64, "params")

    # ---------------------------------------------------------------- API
    def node_coords(self) -> np.ndarray:
        xyz = np.zeros((self.ncells, self.S, self.dim))
        _check(lib().adg_node_coords(self._ctx, xyz.ctypes.data_as(C.POINTER(C.c_double))))
        return xyz

    def stable_dt(self, Q, params, clock, stream=None):
        import torch
        _check(lib().adg_stable_dt(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                   self._params(params), self._dev(clock, (2,), torch.float64, "clock"),
                                   _stream(stream)))

    def step(self, Q, params, clock, next_dt: bool = True, stream=None):
        import torch
        _check(lib().adg_step(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                              self._params(params), self._dev(clock, (2,), torch.float64, "clock"),
                              STEP_NEXT_DT if next_dt else 0, _stream(stream)))

    def predict(self, Q, params, clock, Qvol, traces=None, stream=None):
        import torch
        tr = C.c_void_p() if traces is None else self._dev(traces, self.trace_shape, torch.float64,
                                                           "traces")
        _check(lib().adg_predict(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                 self._params(params), self._dev(clock, (2,), torch.float64, "clock"),
                                 self._dev(Qvol, self.state_shape, torch.float64, "Qvol"), tr,
                                 _stream(stream)))

    def correct(self, Q, params, clock, next_dt: bool = True, stream=None):
        import torch
        _check(lib().adg_correct(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                 self._params(params), self._dev(clock, (2,), torch.float64, "clock"),
                                 STEP_NEXT_DT if next_dt else 0, _stream(stream)))

    def run(self, Q, params, clock, nsteps: int, rec_out=None, stream=None):
        """nsteps steps with the step size clock[1] held fixed; rec_out
        ([nsteps, nrec, nvar] float64 or None) receives the receiver samples
        after every step.  Fused corrector/predictor kernels where built."""
        import torch
        if not self._run_ready:
            self.reserve_run()
        ro = None
        if rec_out is not None:
            ro = self._dev(rec_out, (nsteps, self.nrec, self.nvar), torch.float64, "rec_out")
        _check(lib().adg_run(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"), self._params(params),
                             self._dev(clock, (2,), torch.float64, "clock"), int(nsteps), ro, _stream(stream)))

    def reserve_run(self):
        """Allocate the second trace array of fused runs (done on the first
        run call otherwise)."""
        _check(lib().adg_run_reserve(self._ctx))
        self._run_ready = True

    def read_clock(self, clock, stream=None):
        """(t, dt) of a device clock, after the work queued on the stream."""
        import torch
        out = (C.c_double * 2)()
        _check(lib().adg_read_clock_host(self._dev(clock, (2,), torch.float64, "clock"), out, _stream(stream)))
        return out[0], out[1]

    @property
    def subcell_shape(self):
        """Shape of the FV subcell arrays of the subcell limiter."""
        return (self.ncells, self.nvar, (2 * self.order + 1) ** self.dim)

    def reserve_limiter(self):
        """Allocate the subcell limiter's workspace (done on the first
        step_limited call otherwise)."""
        _check(lib().adg_limiter_reserve(self._ctx))
        self._limiter_ready = True

    def step_limited(self, Q, clock, sub_in, sub_out, status, counts=None, next_dt: bool = True,
                     reuse_ranges: bool = False, stream=None):
        """One step with the a-posteriori subcell limiter (Euler): Q, status
        (uint8 [ncells]) in place; sub_in / sub_out (subcell_shape) the FV
        data before and after the step (distinct tensors, swapped by the
        caller each step); counts (int32 [3]) or None.  reuse_ranges: Q,
        status and sub_in are what the previous step_limited left (a run of
        limited steps); the t^n ranges of DG cells are then taken from that
        step's candidate (ADG_STEP_REUSE_RANGES), with bitwise the same
        results."""
        import torch
        if not self._limiter_ready:
            self.reserve_limiter()
        cnt = C.c_void_p() if counts is None else self._dev(counts, (3,), torch.int32, "counts")
        _check(lib().adg_step_limited(
            self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
            self._dev(clock, (2,), torch.float64, "clock"),
            self._dev(sub_in, self.subcell_shape, torch.float64, "sub_in"),
            self._dev(sub_out, self.subcell_shape, torch.float64, "sub_out"),
            self._dev(status, (self.ncells,), torch.uint8, "status"), cnt,
            (STEP_NEXT_DT if next_dt else 0) | (STEP_REUSE_RANGES if reuse_ranges else 0), _stream(stream)))

    def check_admissible(self, Q, params, troubled, count, stream=None):
        import torch
        _check(lib().adg_check_admissible(
            self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"), self._params(params),
            self._dev(troubled, (self.ncells,), torch.uint8, "troubled"),
            self._dev(count, (1,), torch.int32, "count"), _stream(stream)))

    def set_point_sources(self, sources):
        """sources: list of dicts with x (3), weight (nvar), f0, t0, amp."""
        arr = (PointSource * max(1, len(sources)))()
        for i, s in enumerate(sources):
            for d in range(3):
                arr[i].x[d] = s["x"][d] if d < len(s["x"]) else 0.0
            for v, wv in enumerate(s["weight"]):
                arr[i].weight[v] = wv
            arr[i].f0, arr[i].t0, arr[i].amp = s["f0"], s["t0"], s["amp"]
        _check(lib().adg_set_point_sources(self._ctx, len(sources), arr))

    def set_receivers(self, xyz):
        xyz = np.asarray(xyz, dtype=np.float64).reshape(len(xyz), -1)
        if xyz.shape[1] < 3:
            xyz = np.pad(xyz, ((0, 0), (0, 3 - xyz.shape[1])))
        xyz = np.ascontiguousarray(xyz)
        _check(lib().adg_set_receivers(self._ctx, len(xyz), xyz.ctypes.data_as(C.POINTER(C.c_double))))
        self.nrec = len(xyz)

    def sample_receivers(self, Q, out, stream=None):
        import torch
        _check(lib().adg_sample_receivers(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                          self._dev(out, (self.nrec, self.nvar), torch.float64, "out"),
                                          _stream(stream)))

    def step_adjoint(self, Q, params, clock, lam, gparams=None, stream=None):
        """lam <- (du^{n+1}/du^n)^T lam and gparams += (du^{n+1}/dm)^T lam for the
        FP64 step from Q = u^n with clock {t^n, dt} (dt held fixed)."""
        import torch
        gp = C.c_void_p()
        if self.nparam > 0:
            if gparams is None:
                raise ValueError("this PDE needs a parameter-gradient array [ncells, nparam]")
            gp = self._dev(gparams, (self.ncells, self.nparam), torch.float64, "gparams")
        _check(lib().adg_step_adjoint(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                      self._params(params),
                                      self._dev(clock, (2,), torch.float64, "clock"),
                                      self._dev(lam, self.state_shape, torch.float64, "lam"), gp,
                                      _stream(stream)))

    def keep_size(self) -> int:
        """Doubles of one step's keep buffer (adg_step_keep / adg_step_adjoint_kept)."""
        n = C.c_longlong(0)
        _check(lib().adg_keep_size(self._ctx, C.byref(n)))
        return int(n.value)

    def step_keep(self, Q, params, clock, keep, stream=None):
        """One FP64 step (dt held fixed) that also writes into keep [keep_size()]
        what the step's adjoint reads of its forward predictor."""
        import torch
        _check(lib().adg_step_keep(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"),
                                   self._params(params), self._dev(clock, (2,), torch.float64, "clock"),
                                   self._dev(keep, (self.keep_size(),), torch.float64, "keep"), _stream(stream)))

    def run_keep(self, Q, params, clock, nsteps: int, keeps, rec_out=None, stream=None):
        """run() of nsteps steps that also writes step n's keep buffer into
        keeps[n] (keeps: [nsteps, keep_size()] float64); rec_out as in run()."""
        import torch
        if not self._run_ready:
            self.reserve_run()
        ro = None
        if rec_out is not None:
            ro = self._dev(rec_out, (nsteps, self.nrec, self.nvar), torch.float64, "rec_out")
        _check(lib().adg_run_keep(self._ctx, self._dev(Q, self.state_shape, torch.float64, "Q"), self._params(params),
                                  self._dev(clock, (2,), torch.float64, "clock"), int(nsteps), ro,
                                  self._dev(keeps, (nsteps, self.keep_size()), torch.float64, "keeps"),
                                  _stream(stream)))

    def step_adjoint_kept(self, params, clock, keep, lam, gparams=None, stream=None):
        """step_adjoint of the step that wrote keep (step_keep), without u^n."""
        import torch
        gp = C.c_void_p()
        if self.nparam > 0:
            if gparams is None:
                raise ValueError("this PDE needs a parameter-gradient array [ncells, nparam]")
            gp = self._dev(gparams, (self.ncells, self.nparam), torch.float64, "gparams")
        _check(lib().adg_step_adjoint_kept(self._ctx, self._params(params),
                                           self._dev(clock, (2,), torch.float64, "clock"),
                                           self._dev(keep, (self.keep_size(),), torch.float64, "keep"),
                                           self._dev(lam, self.state_shape, torch.float64, "lam"), gp,
                                           _stream(stream)))

    def sample_receivers_adjoint(self, lamrec, lam, stream=None):
        """lam += transpose of receiver sampling applied to lamrec [nrec, nvar]."""
        import torch
        _check(lib().adg_sample_receivers_adjoint(
            self._ctx, self._dev(lamrec, (self.nrec, self.nvar), torch.float64, "lamrec"),
            self._dev(lam, self.state_shape, torch.float64, "lam"), _stream(stream)))
