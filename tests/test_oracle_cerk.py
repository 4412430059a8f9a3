"""The CERK initial guess of the Picard iteration in the oracle (the
alternative guess the paper names for its optimised kernels, Sec. 5.2; the
reading is stated in adg_oracle.c: classical four-stage Runge-Kutta with its
uniform third-order continuous extension, evaluated at the time nodes).

Pins, none of which re-types the oracle's formulas:
  * the guess on polynomial advection data against the exact translate
    p(x - a tau dt) (the space holds it, so only the time error is left):
    O(dt^4) at every time node, O(dt) for the constant guess;
  * CERK followed by dN + 1 Picard passes equals the dense solve of the
    element system (the linear Picard map is nilpotent: the guess is
    forgotten after dN + 1 passes);
  * the full step with the CERK guess and N - 2 passes keeps the order N + 1
    on the 2-D density wave of Eqs. (8), (10).
"""
import numpy as np
import pytest

import oracle as O
from test_oracle_pins import _c1_state, _dense_predictor, _rel_l2, _run_to


def _poly_case(N):
    a = np.array([0.6, -0.4])
    P = O.problem(2, N, O.ADVECTION, [2, 2], adv=tuple(a), guess=O.GUESS_CERK)
    X = O.node_coords(P)

    def p(x, y):
        return (1.0 + 0.3 * x - 0.2 * y + 0.5 * x * x * y - 0.7 * x ** 3 * y ** 2 + 0.1 * y ** 3
                + 0.4 * x ** N - 0.3 * y ** N + 0.2 * x ** (N - 1) * y)

    return P, X, p, a


@pytest.mark.parametrize("N", [3, 5])
def test_cerk_guess_is_third_order_in_time(N):
    P, X, p, a = _poly_case(N)
    Q = p(X[..., 0], X[..., 1])[:, None, :]
    tau = O.tables(N + 1)["xi"]
    errs, errs_const = [], []
    for dt in (0.4, 0.2, 0.1, 0.05):
        q0, _, _ = O.predictor(P, 1, Q, None, dt, iters=0)
        e = 0.0
        for j in range(N + 1):
            s = tau[j] * dt
            exact = p(X[1, :, 0] - a[0] * s, X[1, :, 1] - a[1] * s)
            e = max(e, np.abs(q0[j, :, 0] - exact).max())
        errs.append(e)
        P.guess = O.GUESS_CONSTANT
        qc, _, _ = O.predictor(P, 1, Q, None, dt, iters=0)
        P.guess = O.GUESS_CERK
        errs_const.append(max(np.abs(qc[j, :, 0] - p(X[1, :, 0] - a[0] * tau[j] * dt,
                                                    X[1, :, 1] - a[1] * tau[j] * dt)).max()
                              for j in range(N + 1)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    rates_c = np.log2(np.array(errs_const[:-1]) / np.array(errs_const[1:]))
    assert rates.min() >= 3.8, (errs, rates)
    assert abs(rates_c[-1] - 1.0) < 0.1, rates_c
    assert errs[-1] < 1e-4 * errs_const[-1]


@pytest.mark.parametrize("dim,N", [(2, 2), (2, 3), (3, 2)])
def test_cerk_then_dN_plus_one_passes_equal_the_dense_solve(dim, N):
    a = (0.8, -0.5, 0.3)[:dim]
    P = O.problem(dim, N, O.ADVECTION, [3] * dim, adv=a, hi=[1.0, 0.7, 1.3][:dim], guess=O.GUESS_CERK)
    rng = np.random.default_rng(30 + dim + N)
    Q = rng.normal(size=(P.ncells, 1, P.S))
    c, dt = 4, 0.05
    qst, _, _ = O.predictor(P, c, Q, None, dt, iters=dim * N + 1)
    ref = _dense_predictor(P, Q[c].T, dt, [np.array([[ad]]) for ad in a])
    np.testing.assert_allclose(qst[..., 0], ref[..., 0], atol=2e-13 * np.abs(ref).max())
    # fewer passes do not reach it (the guess is not the fixed point)
    q1, _, _ = O.predictor(P, c, Q, None, dt, iters=1)
    assert np.abs(q1[..., 0] - ref[..., 0]).max() > 1e-9 * np.abs(ref).max()


def test_cerk_full_step_keeps_the_order():
    # CFL_N 0.5: inside the linear stability limit of both guesses for N <= 5
    # (0.9 is beyond it for N >= 4, where runs over many steps grow)
    for N in (3, 4, 5):
        errs, errs_const = [], []
        for m in (4, 8, 16):
            P = O.problem(2, N, O.EULER, [m, m], guess=O.GUESS_CERK, cfl=0.5)
            assert P.picard_iters == max(1, N - 2)
            errs.append(_rel_l2(P, _run_to(P, _c1_state(P, 0.0), 0.05), _c1_state(P, 0.05)))
            Pc = O.problem(2, N, O.EULER, [m, m], cfl=0.5)
            errs_const.append(_rel_l2(Pc, _run_to(Pc, _c1_state(Pc, 0.0), 0.05), _c1_state(Pc, 0.05)))
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates[-1] >= N + 1 - 0.3, (N, errs, rates)
        # same accuracy class as the constant guess with N + 1 passes
        assert errs[-1] < 3.0 * errs_const[-1], (errs, errs_const)
