"""The identity behind the predictor for PDEs linear in Q, checked on the
oracle alone (CPU).

With R(q) = L q (L the element's spatial operator), the Picard iteration of
Eq. 5 started from q^0 = u has the time average
    qbar = sum_{k=0..I} c_k (dt L)^k u,   c_k = w^T (K1^{-1} W)^k 1,
and c_k = 1/(k+1)! for k <= N (K1^{-1} W integrates polynomials of degree
below n exactly).  The GPU's linear predictor evaluates this polynomial; the
oracle iterates.  Here the oracle's Picard average of the advection-decay
PDE is compared with the polynomial built from the oracle's own tables and
a plain numpy L.
"""
import math

import numpy as np
import pytest

import oracle as O


def lin_coeffs(n, kmax):
    T = O.tables(n)
    KW = T["K1inv"] * T["w"][None, :]
    v = np.ones(n)
    out = []
    for k in range(kmax + 1):
        if k:
            v = KW @ v
        out.append(float(T["w"] @ v))
    return out


@pytest.mark.parametrize("n", range(2, 9))
def test_average_weights_are_taylor_weights_up_to_N(n):
    c = lin_coeffs(n, n - 1)
    for k in range(n):
        assert abs(c[k] * math.factorial(k + 1) - 1.0) <= 1e-13, (n, k, c[k])


@pytest.mark.parametrize("N,iters", [(1, 1), (2, 3), (3, 1), (3, 2), (3, 4), (4, 5), (3, 9)])
def test_picard_average_is_the_polynomial_in_dt_L(N, iters):
    n = N + 1
    cells, lo, hi = [3, 2], [0.0, 0.0], [1.5, 0.8]
    adv, kappa = (0.7, -0.4), 0.3
    P = O.problem(2, N, O.ADVECTION, cells, lo, hi, adv=adv + (0.0,), kappa=kappa, picard_iters=iters)
    rng = np.random.default_rng(100 + 10 * N + iters)
    Q = rng.normal(size=(P.ncells, 1, P.S))
    dt = 0.5 * O.stable_dt(P, Q)[0]
    cell = 4
    _, qbar, _ = O.predictor(P, cell, Q, None, dt, 0.0, iters)

    D = O.tables(n)["D"]
    h = [(hi[d] - lo[d]) / cells[d] for d in range(2)]

    def L(u):  # u[ky, kx]
        ux = u @ D.T / h[0]            # derivative along x (last axis)
        uy = D @ u / h[1]              # derivative along y
        return -(adv[0] * ux + adv[1] * uy) - kappa * u

    u = Q[cell, 0].reshape(n, n)
    c = lin_coeffs(n, iters)
    term, poly = u.copy(), c[0] * u
    for k in range(1, iters + 1):
        term = dt * L(term)
        poly = poly + c[k] * term
    ref = qbar[:, 0].reshape(n, n)
    assert np.linalg.norm(poly - ref) <= 1e-13 * np.linalg.norm(ref)
