"""Plain FP64 CPU oracle of the ADER-DG step -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library under
``paper_1905_07987_amd`` never imports it and shares no code with it.

The arithmetic lives in ``adg_oracle.c`` (built with gcc, ``-O2
-fno-fast-math -ffp-contract=off``); this module only marshals numpy arrays
through ctypes.  The C file's header lists the passages of the ExaHyPE paper
each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the same source built with the address and undefined-behaviour sanitizers
# (host code only; tests/test_oracle_sanitizers.py runs the oracle's pins on
# it in a subprocess that preloads the sanitizer runtime)
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")

EULER, ELASTIC, ADVECTION = 1, 2, 3
MAXQ, MAXSRC = 16, 8


def build(sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE binary64); with
    sanitize=True a second library instrumented with AddressSanitizer and
    UndefinedBehaviorSanitizer (aborting on the first report)."""
    out = _LIB_SAN if sanitize else _LIB
    san = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = (["gcc", "-O1" if sanitize else "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared",
            "-fPIC"] + (san if sanitize else []) + ["-o", out, _SRC, "-lm"])
    subprocess.run(cmd, check=True)
    return out


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("order", C.c_int), ("pde", C.c_int), ("nvar", C.c_int),
        ("nparam", C.c_int), ("picard_iters", C.c_int),
        ("cells", C.c_int * 3),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("cfl", C.c_double), ("gamma", C.c_double), ("adv", C.c_double * 3),
        ("kappa", C.c_double),
        ("nsrc", C.c_int), ("guess", C.c_int),
        ("src_x", (C.c_double * 3) * MAXSRC),
        ("src_w", (C.c_double * MAXQ) * MAXSRC),
        ("src_f0", C.c_double * MAXSRC), ("src_t0", C.c_double * MAXSRC),
        ("src_amp", C.c_double * MAXSRC),
        ("bc", C.c_int * 6),
        ("bc_state", (C.c_double * MAXQ) * 6),
    ]

    @property
    def n(self) -> int:
        return self.order + 1

    @property
    def S(self) -> int:
        return self.n ** self.dim

    @property
    def ncells(self) -> int:
        c = 1
        for d in range(self.dim):
            c *= self.cells[d]
        return c

    @property
    def h(self):
        return [(self.hi[d] - self.lo[d]) / self.cells[d] for d in range(self.dim)]


_NV = {EULER: None, ELASTIC: 9, ADVECTION: 1}


BC_PERIODIC, BC_OUTFLOW, BC_WALL, BC_INFLOW = 0, 1, 2, 3


GUESS_CONSTANT, GUESS_CERK = 0, 1


def problem(dim, order, pde, cells, lo=None, hi=None, cfl=0.9, picard_iters=None,
            gamma=1.4, adv=(1.0, 1.0, 1.0), kappa=0.0, sources=(), bc=None, bc_state=None,
            guess=GUESS_CONSTANT):
    """Build a Problem.  ``guess``: GUESS_CONSTANT (q^0 = u^n, default
    picard_iters N+1) or GUESS_CERK (the CERK initial guess, default
    picard_iters max(1, N-2)).  ``sources`` is a list of dicts with keys x, w, f0, t0, amp;
    ``bc`` the boundary condition of each face 2 d + side (default periodic);
    ``bc_state`` {face: outside state} for BC_INFLOW faces."""
    P = Problem()
    P.dim, P.order, P.pde = dim, order, pde
    if pde == EULER:
        P.nvar, P.nparam = dim + 2, 0
    elif pde == ELASTIC:
        if dim != 3:
            raise ValueError("the elastic PDE is three-dimensional")
        P.nvar, P.nparam = 9, 3
    elif pde == ADVECTION:
        P.nvar, P.nparam = 1, 0
    else:
        raise ValueError(pde)
    P.guess = guess
    if picard_iters is None:
        picard_iters = order + 1 if guess == GUESS_CONSTANT else max(1, order - 2)
    P.picard_iters = picard_iters
    cells = list(cells) + [1] * (3 - len(cells))
    lo = list(lo if lo is not None else [0.0] * dim) + [0.0] * (3 - dim)
    hi = list(hi if hi is not None else [1.0] * dim) + [1.0] * (3 - dim)
    for d in range(3):
        P.cells[d], P.lo[d], P.hi[d] = cells[d], lo[d], hi[d]
        P.adv[d] = adv[d] if d < len(adv) else 0.0
    P.cfl, P.gamma, P.kappa = cfl, gamma, kappa
    if len(sources) > MAXSRC:
        raise ValueError("too many point sources")
    P.nsrc = len(sources)
    for s, src in enumerate(sources):
        for d in range(3):
            P.src_x[s][d] = src["x"][d] if d < len(src["x"]) else 0.0
        for v, wv in enumerate(src["w"]):
            P.src_w[s][v] = wv
        P.src_f0[s], P.src_t0[s], P.src_amp[s] = src["f0"], src["t0"], src["amp"]
    for f, b in enumerate(bc or ()):
        P.bc[f] = b
    for f, q in (bc_state or {}).items():
        for v, x in enumerate(q):
            P.bc_state[f][v] = x
    return P


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB_SAN if os.environ.get("ADG_ORACLE_SANITIZED") == "1" else _LIB
        if not os.path.exists(path):
            raise RuntimeError(f"oracle library missing: {path} (run __graft_entry__.build())")
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        pp = C.POINTER(Problem)
        L.orc_tables.argtypes = [C.c_int] + [dp] * 7
        L.orc_basis_eval.argtypes = [C.c_int, C.c_double, dp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_node_coords.argtypes = [pp, dp]
        L.orc_pointwise.argtypes = [pp, dp, C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.orc_ncp.argtypes = [pp, dp, dp, dp]
        L.orc_rusanov.argtypes = [pp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.orc_stable_dt.argtypes = [pp, dp, dp, dp, dp]
        L.orc_predictor.argtypes = [pp, C.c_long, dp, dp, C.c_double, C.c_double, C.c_int, dp, dp, dp]
        L.orc_step.argtypes = [pp, dp, dp, C.c_double, C.c_double, dp]
        L.orc_step_cells.argtypes = [pp, dp, dp, C.c_double, C.c_double, C.c_long,
                                     C.POINTER(C.c_long), dp]
        L.orc_cell_traces.argtypes = [pp, C.c_long, dp, dp, C.c_double, C.c_double, dp, dp, dp]
        L.orc_sample_receivers.argtypes = [pp, C.c_int, dp, dp, dp]
        L.orc_check_admissible.argtypes = [pp, dp, dp, C.POINTER(C.c_ubyte), C.POINTER(C.c_int)]
        L.orc_step_adjoint.argtypes = [pp, dp, dp, C.c_double, C.c_double, dp, dp]
        L.orc_sample_receivers_T.argtypes = [pp, C.c_int, dp, dp, dp]
        L.orc_step_limited.argtypes = [pp, dp, dp, C.c_double, C.c_double, dp, C.POINTER(C.c_ubyte),
                                       C.POINTER(C.c_int)]
        L.orc_limiter_tables.argtypes = [C.c_int, dp, dp, dp]
        L.orc_fv_step.argtypes = [pp, dp, C.c_double, dp]
        L.orc_stable_dt_limited.argtypes = [pp, dp, dp, C.POINTER(C.c_ubyte), dp, dp]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def set_threads(n: int) -> int:
    return lib().orc_set_threads(n)


def tables(n: int) -> dict:
    """GL nodes/weights on [0,1], D_ij = phi_j'(xi_i), l0, l1, K1, K1^{-1}."""
    xi, w, l0, l1 = (np.zeros(n) for _ in range(4))
    D, K1, K1inv = (np.zeros((n, n)) for _ in range(3))
    _check(lib().orc_tables(n, _p(xi), _p(w), _p(D), _p(l0), _p(l1), _p(K1), _p(K1inv)), "tables")
    return dict(xi=xi, w=w, D=D, l0=l0, l1=l1, K1=K1, K1inv=K1inv)


def basis_eval(n: int, x: float) -> np.ndarray:
    phi = np.zeros(n)
    _check(lib().orc_basis_eval(n, float(x), _p(phi)), "basis_eval")
    return phi


def node_coords(P: Problem) -> np.ndarray:
    """[C][S][dim] physical node coordinates."""
    out = np.zeros((P.ncells, P.S, P.dim))
    _check(lib().orc_node_coords(C.byref(P), _p(out)), "node_coords")
    return out


def pointwise(P: Problem, Q, d: int):
    Q = _arr(Q)
    F = np.zeros(P.nvar)
    lam = C.c_double()
    adm = C.c_int()
    _check(lib().orc_pointwise(C.byref(P), _p(Q), d, _p(F), C.byref(lam), C.byref(adm)), "pointwise")
    return F, lam.value, bool(adm.value)


def ncp(P: Problem, Q, gradQ):
    Q, gradQ = _arr(Q), _arr(gradQ)
    out = np.zeros(P.nvar)
    _check(lib().orc_ncp(C.byref(P), _p(Q), _p(gradQ), _p(out)), "ncp")
    return out


def rusanov(P: Problem, d: int, qL, FL, qR, FR):
    qL, FL, qR, FR = map(_arr, (qL, FL, qR, FR))
    flL, flR = np.zeros(P.nvar), np.zeros(P.nvar)
    _check(lib().orc_rusanov(C.byref(P), d, _p(qL), _p(FL), _p(qR), _p(FR), _p(flL), _p(flR)),
           "rusanov")
    return flL, flR


def _params(P, params):
    if P.nparam == 0:
        return None
    return _arr(params)


def stable_dt(P: Problem, Q, params=None):
    dt, lam = C.c_double(), C.c_double()
    Q = _arr(Q)
    _check(lib().orc_stable_dt(C.byref(P), _p(Q), _p(_params(P, params)), C.byref(dt),
                               C.byref(lam)), "stable_dt")
    return dt.value, lam.value


def predictor(P: Problem, cell: int, Q, params, dt: float, t: float = 0.0, iters=None):
    iters = P.picard_iters if iters is None else iters
    nq = P.nvar + P.nparam
    Q = _arr(Q)
    qst = np.zeros((P.n, P.S, nq))
    qbar = np.zeros((P.S, P.nvar))
    Fbar = np.zeros((P.dim, P.S, P.nvar))
    _check(lib().orc_predictor(C.byref(P), cell, _p(Q), _p(_params(P, params)), dt, t, iters,
                               _p(qst), _p(qbar), _p(Fbar)), "predictor")
    return qst, qbar, Fbar


def cell_traces(P: Problem, cell: int, Q, params, dt: float, t: float = 0.0):
    nf = P.n ** (P.dim - 1)
    Q = _arr(Q)
    qh = np.zeros((2 * P.dim, nf, P.nvar))
    Fh = np.zeros((2 * P.dim, nf, P.nvar))
    vol = np.zeros((P.S, P.nvar))
    _check(lib().orc_cell_traces(C.byref(P), cell, _p(Q), _p(_params(P, params)), dt, t, _p(qh),
                                 _p(Fh), _p(vol)), "cell_traces")
    return qh, Fh, vol


def step(P: Problem, Q, params, dt: float, t: float = 0.0, weak: bool = False):
    """Return u^{n+1} (a new array); with weak=True also the weak-form result."""
    Qn = _arr(Q).copy()
    w = np.zeros_like(Qn) if weak else None
    _check(lib().orc_step(C.byref(P), _p(Qn), _p(_params(P, params)), dt, t, _p(w)), "step")
    return (Qn, w) if weak else Qn


def step_cells(P: Problem, Q, params, dt: float, t: float, cells) -> np.ndarray:
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    Q = _arr(Q)
    out = np.zeros((len(cells), P.nvar, P.S))
    _check(lib().orc_step_cells(C.byref(P), _p(Q), _p(_params(P, params)), dt, t, len(cells),
                                cells.ctypes.data_as(C.POINTER(C.c_long)), _p(out)), "step_cells")
    return out


def sample_receivers(P: Problem, xyz, Q) -> np.ndarray:
    xyz = np.asarray(xyz, dtype=np.float64).reshape(len(xyz), -1)
    if xyz.shape[1] < 3:
        xyz = np.pad(xyz, ((0, 0), (0, 3 - xyz.shape[1])))
    xyz = _arr(xyz)
    Q = _arr(Q)
    out = np.zeros((len(xyz), P.nvar))
    _check(lib().orc_sample_receivers(C.byref(P), len(xyz), _p(xyz), _p(Q), _p(out)), "receivers")
    return out


def check_admissible(P: Problem, Q, params=None):
    Q = _arr(Q)
    flags = np.zeros(P.ncells, dtype=np.uint8)
    cnt = C.c_int()
    _check(lib().orc_check_admissible(C.byref(P), _p(Q), _p(_params(P, params)),
                                      flags.ctypes.data_as(C.POINTER(C.c_ubyte)), C.byref(cnt)),
           "check_admissible")
    return flags, cnt.value


STATUS_DG, STATUS_DG_FV_FACES, STATUS_FV, STATUS_TROUBLED = 0, 1, 2, 3


def limiter_subcells(P: Problem) -> int:
    return (2 * P.n - 1) ** P.dim


def step_limited(P: Problem, Q, dt: float, t: float = 0.0, sub=None, status=None):
    """One step with the a-posteriori subcell limiter (Euler).  ``sub``
    [C][nv][m^dim] and ``status`` [C] carry the FV cells from step to step
    (None: a first step, nothing on FV).  Returns (u^{n+1}, sub, status,
    counts (troubled, FV cells, DG cells with FV faces)), all new arrays."""
    Qn = _arr(Q).copy()
    sub = np.zeros((P.ncells, P.nvar, limiter_subcells(P))) if sub is None else _arr(sub).copy()
    status = np.zeros(P.ncells, dtype=np.uint8) if status is None else np.array(status, dtype=np.uint8)
    counts = (C.c_int * 3)()
    _check(lib().orc_step_limited(C.byref(P), _p(Qn), None, dt, t, _p(sub),
                                  status.ctypes.data_as(C.POINTER(C.c_ubyte)), counts), "step_limited")
    return Qn, sub, status, tuple(counts)


def stable_dt_limited(P: Problem, Q, sub, status):
    """Eq. (7) in a limited run: FV cells (status >= 2) by their subcell
    averages, the others by their nodes.  Returns (dt, lambda_max)."""
    dt, lam = C.c_double(), C.c_double()
    st = np.ascontiguousarray(status, dtype=np.uint8)
    _check(lib().orc_stable_dt_limited(C.byref(P), _p(_arr(Q)), _p(_arr(sub)),
                                       st.ctypes.data_as(C.POINTER(C.c_ubyte)), C.byref(dt), C.byref(lam)),
           "stable_dt_limited")
    return dt.value, lam.value


def limiter_tables(n: int):
    """(A [m][n] subcell averages of the basis, B [n][m] its least-squares
    inverse, Qf [n][m] subface data to face nodes), m = 2n - 1."""
    m = 2 * n - 1
    A, B, Qf = np.zeros((m, n)), np.zeros((n, m)), np.zeros((n, m))
    _check(lib().orc_limiter_tables(n, _p(A), _p(B), _p(Qf)), "limiter_tables")
    return A, B, Qf


def fv_step(P: Problem, Q, dt: float):
    """The FV scheme alone on every cell: (u^{n+1} projected back to DG,
    subcell averages [C][nv][m^dim] after the FV step)."""
    Qn = _arr(Q).copy()
    m = 2 * P.n - 1
    sub = np.zeros((P.ncells, P.nvar, m ** P.dim))
    _check(lib().orc_fv_step(C.byref(P), _p(Qn), dt, _p(sub)), "fv_step")
    return Qn, sub


def run(P: Problem, Q, params=None, steps: int = 1, t0: float = 0.0, dt_fixed=None):
    """Advance ``steps`` steps with Eq. (7) recomputed each step (or a fixed dt)."""
    Q = _arr(Q).copy()
    t = t0
    for _ in range(steps):
        dt = dt_fixed if dt_fixed is not None else stable_dt(P, Q, params)[0]
        Q = step(P, Q, params, dt, t)
        t += dt
    return Q, t


def _xyz3(xyz):
    xyz = np.asarray(xyz, dtype=np.float64).reshape(len(xyz), -1)
    if xyz.shape[1] < 3:
        xyz = np.pad(xyz, ((0, 0), (0, 3 - xyz.shape[1])))
    return np.ascontiguousarray(xyz)


def step_adjoint(P: Problem, Q, params, dt: float, t: float, lam):
    """Discrete adjoint of one step (linear PDEs, dt frozen): returns
    (dJ/du^n, dJ/dm of this step) for lam = dJ/du^{n+1}."""
    Q = _arr(Q)
    lam_n = _arr(lam).copy()
    g = np.zeros((P.ncells, max(P.nparam, 1)))
    _check(lib().orc_step_adjoint(C.byref(P), _p(Q), _p(_params(P, params)), dt, t, _p(lam_n),
                                  _p(g) if P.nparam else None), "step_adjoint")
    return lam_n, (g if P.nparam else None)


def sample_receivers_T(P: Problem, xyz, lamrec, lam):
    """lam += transpose of receiver sampling applied to lamrec [nrec][nvar]."""
    xyz = _xyz3(xyz)
    lamrec = _arr(lamrec)
    _check(lib().orc_sample_receivers_T(C.byref(P), len(xyz), _p(xyz), _p(lamrec), _p(lam)), "receivers_T")
    return lam


def seismogram_misfit(P: Problem, u0, params, dt: float, steps: int, rec_xyz, data=None):
    """J = 1/2 sum_{n=1..steps} dt sum_r sum_c (v^n_rc - d^n_rc)^2 with v the
    particle velocity (rho v)/rho of the receiver's cell, sampled after every
    step with a frozen dt.  Returns (J, seismograms [steps][R][3], states)."""
    rec_xyz = _xyz3(rec_xyz)
    cells = _receiver_cells(P, rec_xyz)
    Q = _arr(u0).copy()
    states = [Q.copy()]
    seis = []
    t = 0.0
    for n in range(steps):
        Q = step(P, Q, params, dt, t)
        t += dt
        states.append(Q.copy())
        samp = sample_receivers(P, rec_xyz, Q)
        seis.append(samp[:, 6:9] / params[cells, 0:1])
    seis = np.array(seis)
    J = 0.0 if data is None else 0.5 * dt * float(((seis - data) ** 2).sum())
    return J, seis, states


def _receiver_cells(P, rec_xyz):
    h = P.h
    out = []
    for x in rec_xyz:
        cc = [int(np.floor((x[d] - P.lo[d]) / h[d])) for d in range(P.dim)]
        c = cc[0] + P.cells[0] * (cc[1] + P.cells[1] * (cc[2] if P.dim == 3 else 0))
        out.append(c)
    return np.array(out)


def misfit_gradient(P: Problem, u0, params, dt: float, steps: int, rec_xyz, data):
    """J and its gradients with respect to u0 and the per-cell parameters by
    the discrete adjoint (every state kept in memory: small problems only)."""
    rec_xyz = _xyz3(rec_xyz)
    cells = _receiver_cells(P, rec_xyz)
    J, seis, states = seismogram_misfit(P, u0, params, dt, steps, rec_xyz, data)
    lam = np.zeros_like(states[0])
    g = np.zeros_like(np.asarray(params, dtype=np.float64))
    rho = params[cells, 0]
    for n in range(steps, 0, -1):
        r = dt * (seis[n - 1] - data[n - 1])          # dJ/dv^n  [R][3]
        lamrec = np.zeros((len(rec_xyz), P.nvar))
        lamrec[:, 6:9] = r / rho[:, None]
        sample_receivers_T(P, rec_xyz, lamrec, lam)
        np.add.at(g[:, 0], cells, -(r * seis[n - 1]).sum(axis=1) / rho)
        lam, gs = step_adjoint(P, states[n - 1], params, dt, (n - 1) * dt, lam)
        g += gs
    return J, lam, g
