"""Pins of the oracle's discrete adjoint (linear PDEs, frozen dt).

The adjoint is checked against the forward oracle only through identities
that any correct transpose satisfies: the dot-product test of the (linear in
u) step map, central finite differences for the parameters, finite
differences and a Taylor test of the multi-step seismogram misfit.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import inputs


def _elastic_case(cells=(3, 3, 2), N=2, seed=1):
    P = O.problem(3, N, O.ELASTIC, list(cells), hi=[500.0 * c for c in cells])
    rng = np.random.default_rng(seed)
    params = np.column_stack([rng.uniform(2000, 3000, P.ncells), rng.uniform(5000, 7000, P.ncells),
                              rng.uniform(2500, 3400, P.ncells)])
    u = rng.normal(size=(P.ncells, 9, P.S)) * np.array([6000.0] * 6 + [1.0] * 3)[None, :, None]
    dt = 0.5 * O.stable_dt(P, u, params)[0]
    return P, params, u, dt, rng


def test_adjoint_dot_product_elastic():
    """<lam, A u> = <A^T lam, u> for the (linear, source-free) step map A."""
    P, params, u, dt, rng = _elastic_case()
    lam = rng.normal(size=u.shape)
    Au = O.step(P, u, params, dt, 0.0)
    lam_n, _ = O.step_adjoint(P, u, params, dt, 0.0, lam)
    a, b = (lam * Au).sum(), (lam_n * u).sum()
    assert abs(a - b) <= 1e-13 * abs(a)


def test_adjoint_dot_product_advection_decay():
    P = O.problem(2, 3, O.ADVECTION, [4, 3], adv=(0.7, -0.4), kappa=1.3)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(P.ncells, 1, P.S))
    lam = rng.normal(size=u.shape)
    dt = O.stable_dt(P, u)[0]
    Au = O.step(P, u, None, dt, 0.0)
    lam_n, _ = O.step_adjoint(P, u, None, dt, 0.0, lam)
    a, b = (lam * Au).sum(), (lam_n * u).sum()
    assert abs(a - b) <= 1e-13 * abs(a)


def test_adjoint_parameters_central_differences():
    """d/de <lam, step(u, m + e dm)> at e = 0 against the adjoint's dJ/dm."""
    P, params, u, dt, rng = _elastic_case(seed=3)
    lam = rng.normal(size=u.shape)
    _, g = O.step_adjoint(P, u, params, dt, 0.0, lam)
    for trial in range(3):
        dm = rng.normal(size=params.shape) * params * 1e-3
        eps = 1e-2
        fp = (lam * O.step(P, u, params + eps * dm, dt, 0.0)).sum()
        fm = (lam * O.step(P, u, params - eps * dm, dt, 0.0)).sum()
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - (g * dm).sum()) <= 1e-7 * abs(fd), (trial, fd, (g * dm).sum())


def test_adjoint_parameters_with_material_jumps_per_parameter():
    """Each of rho, cp, cs separately (rho enters only through the midpoint
    of the face non-conservative product and cancels in the volume term)."""
    P, params, u, dt, rng = _elastic_case(cells=(2, 2, 2), seed=4)
    lam = rng.normal(size=u.shape)
    _, g = O.step_adjoint(P, u, params, dt, 0.0, lam)
    for p in range(3):
        dm = np.zeros_like(params)
        dm[:, p] = rng.normal(size=P.ncells) * params[:, p] * 1e-3
        eps = 1e-2
        fd = ((lam * O.step(P, u, params + eps * dm, dt, 0.0)).sum()
              - (lam * O.step(P, u, params - eps * dm, dt, 0.0)).sum()) / (2 * eps)
        scale = (np.abs(g) * np.abs(params) * 1e-3).sum()  # size of a typical directional derivative
        assert abs(fd - (g * dm).sum()) <= 1e-7 * scale, (p, fd, (g * dm).sum())
    # rho cancels from E(lambda, mu) grad v = E(cp^2 - 2 cs^2, cs^2) grad(rho v): no sensitivity
    assert np.abs(g[:, 0]).max() <= 1e-12 * np.abs(g).max()


def _misfit_case(seed=5, steps=6):
    """A small layered elastic problem with a point source, receivers and
    'observed' data from a perturbed material."""
    cells = (4, 3, 3)
    lo, hi = [0.0] * 3, [2000.0, 1500.0, 1500.0]
    src = dict(x=(1250.0, 750.0, 600.0), w=[0.0] * 8 + [1.0], f0=5.0, t0=0.0, amp=1e6)
    P = O.problem(3, 2, O.ELASTIC, list(cells), lo, hi, sources=[src])
    cen = inputs.cell_centres(cells, lo, hi)
    params = inputs.layered_material(cen[:, 2] * 4.0, seed)
    params_obs = params * (1.0 + 0.05 * np.random.default_rng(seed + 1).uniform(-1, 1, params.shape))
    rec = np.array([[300.0, 400.0, 200.0], [1700.0, 1100.0, 900.0], [1000.0, 700.0, 1400.0]])
    u0 = np.zeros((P.ncells, 9, P.S))
    dt = 0.5 * min(O.stable_dt(P, u0, params)[0], O.stable_dt(P, u0, params_obs)[0])
    _, data, _ = O.seismogram_misfit(P, u0, params_obs, dt, steps, rec)
    return P, params, u0, dt, steps, rec, data


def test_misfit_gradient_parameters_finite_differences():
    P, params, u0, dt, steps, rec, data = _misfit_case()
    J, gu, gm = O.misfit_gradient(P, u0, params, dt, steps, rec, data)
    assert J > 0
    rng = np.random.default_rng(9)
    flat = np.abs(gm).ravel()
    cand = np.nonzero(flat >= 1e-2 * flat.max())[0]
    for idx in rng.choice(cand, size=min(6, len(cand)), replace=False):
        c, p = divmod(int(idx), 3)
        h = 1e-4 * params[c, p]
        pp, pm = params.copy(), params.copy()
        pp[c, p] += h
        pm[c, p] -= h
        Jp = O.seismogram_misfit(P, u0, pp, dt, steps, rec, data)[0]
        Jm = O.seismogram_misfit(P, u0, pm, dt, steps, rec, data)[0]
        fd = (Jp - Jm) / (2 * h)
        assert abs(fd - gm[c, p]) <= 1e-6 * abs(fd), (c, p, fd, gm[c, p])


def test_misfit_gradient_initial_state_taylor():
    """J is quadratic in u0 at fixed material: the Taylor remainder
    J(u0 + e du) - J(u0) - e <g, du> shrinks exactly like e^2."""
    P, params, u0, dt, steps, rec, data = _misfit_case(seed=6, steps=5)
    rng = np.random.default_rng(10)
    u0 = rng.normal(size=u0.shape) * 1e-3 * np.array([6000.0] * 6 + [2700.0] * 3)[None, :, None]
    J, gu, _ = O.misfit_gradient(P, u0, params, dt, steps, rec, data)
    du = rng.normal(size=u0.shape) * np.array([6000.0] * 6 + [2700.0] * 3)[None, :, None] * 1e-3
    rem = []
    for e in (1e-1, 5e-2, 2.5e-2):
        Je = O.seismogram_misfit(P, u0 + e * du, params, dt, steps, rec, data)[0]
        rem.append(Je - J - e * (gu * du).sum())
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    np.testing.assert_allclose(rates, 2.0, atol=1e-3)
