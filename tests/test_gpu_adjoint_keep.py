"""The adjoint step from a kept forward step (adg_step_keep + adg_step_adjoint_kept).

The kept path must give what adg_step_adjoint gives from u^n, and the
oracle's discrete adjoint to 1e-12; adg_step_keep must leave the forward
step itself unchanged (bitwise the state of adg_step).  lam is compared
bitwise (the same arithmetic on the same values).  The parameter gradient
is compared to rounding: the kept path takes the Rusanov flux's two
transposes in one kernel, whose compiled products may round differently
from those of the two separate kernels (measured: at most 1.8e-15 against
entries of order 1).  Cases: elasticity with
per-cell material at N = 1..4 (ragged last blocks), fewer Picard iterations
than N + 1, a point source, advection in 2-D and 3-D; error paths.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import adg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
GRAD_ROUNDING = 1e-14  # kept vs state path, relative to the largest entry


def same_gradient(ga, gb):
    return ga is None and gb is None or np.abs(ga - gb).max() <= GRAD_ROUNDING * np.abs(ga).max()


def say(*a):
    print("[gpu-test]", *a, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def elastic(cells, N, seed, picard_iters=0, sources=()):
    hi = [500.0 * c for c in cells]
    kw = dict(picard_iters=picard_iters) if picard_iters else {}
    P = O.problem(3, N, O.ELASTIC, list(cells), hi=hi, sources=sources, **kw)
    s = adg.Solver(3, N, "elastic", list(cells), [0.0] * 3, hi, picard_iters=picard_iters)
    if sources:
        s.set_point_sources([dict(x=src["x"], weight=src["w"], f0=src["f0"], t0=src["t0"],
                                  amp=src["amp"]) for src in sources])
    rng = np.random.default_rng(seed)
    params = np.column_stack([rng.uniform(2000, 3000, P.ncells), rng.uniform(5000, 7000, P.ncells),
                              rng.uniform(2500, 3400, P.ncells)])
    u = rng.normal(size=(P.ncells, 9, P.S)) * np.array([6000.0] * 6 + [1.0] * 3)[None, :, None]
    lam = rng.normal(size=u.shape)
    dt = 0.5 * O.stable_dt(P, u, params)[0]
    return s, P, params, u, lam, dt


def both_paths(s, u, params, lam, dt, t=0.0):
    """(state after adg_step, after adg_step_keep; lam and gparams of the
    state-based adjoint and of the kept one)."""
    prm = dev(params) if params is not None else None
    # forward: plain step and kept step from the same u^n and clock
    Q1, Q2 = dev(u), dev(u)
    c1, c2 = dev([t, dt]), dev([t, dt])
    s.step(Q1, prm, c1, next_dt=False)
    keep = torch.full((s.keep_size(),), float("nan"), dtype=torch.float64, device="cuda")
    s.step_keep(Q2, prm, c2, keep)
    # adjoints of the step t -> t + dt
    gz = lambda: torch.zeros((s.ncells, s.nparam), dtype=torch.float64, device="cuda") if s.nparam else None
    la, ga = dev(lam), gz()
    s.step_adjoint(dev(u), prm, dev([t, dt]), la, ga)
    lb, gb = dev(lam), gz()
    s.step_adjoint_kept(prm, dev([t, dt]), keep, lb, gb)
    torch.cuda.synchronize()
    cpu = lambda x: x.cpu().numpy() if x is not None else None
    return cpu(Q1), cpu(Q2), cpu(c1), cpu(c2), cpu(la), cpu(ga), cpu(lb), cpu(gb)


@pytest.mark.parametrize("N,cells", [(1, (7, 3, 2)), (2, (4, 3, 5)), (3, (7, 6, 5)), (3, (1, 1, 2)),
                                     (4, (3, 3, 1))])
def test_kept_adjoint_elastic(N, cells):
    say(f"kept adjoint elastic N={N} cells={cells}")
    s, P, params, u, lam, dt = elastic(cells, N, seed=40 + N)
    Q1, Q2, c1, c2, la, ga, lb, gb = both_paths(s, u, params, lam, dt)
    assert np.array_equal(Q1, Q2) and np.array_equal(c1, c2)
    say(f"  kept vs state path: lam max |diff| {np.abs(la - lb).max():.1e}, grad {np.abs(ga - gb).max():.1e}"
        f" (max |grad| {np.abs(ga).max():.2e})")
    assert np.array_equal(la, lb) and same_gradient(ga, gb)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.0, lam)
    e_l, e_g = rel_l2(lb, lam_o), rel_l2(gb[:, 1:], g_o[:, 1:])
    say(f"  vs oracle: rel L2 lam {e_l:.2e}, grad(cp, cs) {e_g:.2e}")
    assert e_l <= TOL and e_g <= TOL


def test_kept_adjoint_fewer_picard_iterations():
    s, P, params, u, lam, dt = elastic((3, 2, 2), 3, seed=47, picard_iters=2)
    Q1, Q2, c1, c2, la, ga, lb, gb = both_paths(s, u, params, lam, dt)
    assert np.array_equal(Q1, Q2)
    assert np.array_equal(la, lb) and same_gradient(ga, gb)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.0, lam)
    assert rel_l2(lb, lam_o) <= TOL and rel_l2(gb[:, 1:], g_o[:, 1:]) <= TOL


def test_kept_adjoint_point_source():
    src = [dict(x=(700.0, 900.0, 400.0), w=[0.0] * 6 + [0.3, -0.2, 1.0], f0=5.0, t0=0.1, amp=1e7)]
    s, P, params, u, lam, dt = elastic((3, 3, 2), 3, seed=48, sources=src)
    u *= 1e-3
    Q1, Q2, c1, c2, la, ga, lb, gb = both_paths(s, u, params, lam, dt, t=0.05)
    assert np.array_equal(Q1, Q2)
    assert np.array_equal(la, lb) and same_gradient(ga, gb)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.05, lam)
    e_l, e_g = rel_l2(lb, lam_o), rel_l2(gb[:, 1:], g_o[:, 1:])
    say(f"point source, kept: rel L2 lam {e_l:.2e}, grad {e_g:.2e}")
    assert e_l <= TOL and e_g <= TOL


@pytest.mark.parametrize("dim,N,cells", [(2, 3, (6, 9)), (3, 2, (4, 3, 5)), (3, 5, (2, 3, 2))])
def test_kept_adjoint_advection(dim, N, cells):
    adv = (0.7, -0.4, 0.3)[:dim]
    P = O.problem(dim, N, O.ADVECTION, list(cells), adv=adv, kappa=1.3)
    s = adg.Solver(dim, N, "advection", list(cells), adv=adv, kappa=1.3)
    rng = np.random.default_rng(50 + dim * 10 + N)
    u = rng.normal(size=(P.ncells, 1, P.S))
    lam = rng.normal(size=u.shape)
    dt = O.stable_dt(P, u)[0]
    Q1, Q2, c1, c2, la, _, lb, _ = both_paths(s, u, None, lam, dt)
    assert np.array_equal(Q1, Q2) and np.array_equal(la, lb)
    lam_o, _ = O.step_adjoint(P, u, None, dt, 0.0, lam)
    e = rel_l2(lb, lam_o)
    say(f"advection dim={dim} N={N} kept: rel L2 {e:.2e}")
    assert e <= TOL


def test_keep_error_paths():
    e = adg.Solver(3, 2, "euler", [2, 2, 2])
    with pytest.raises(adg.AdgError) as ei:
        e.keep_size()
    assert ei.value.status == -4
    s = adg.Solver(3, 2, "elastic", [2, 2, 2], precision="fp32")
    with pytest.raises(adg.AdgError) as ei:
        Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
        prm = torch.ones((s.ncells, 3), dtype=torch.float64, device="cuda")
        s.step_keep(Q, prm, dev([0.0, 1e-3]), torch.zeros(s.keep_size(), dtype=torch.float64, device="cuda"))
    assert ei.value.status == -4
    s = adg.Solver(3, 2, "elastic", [2, 2, 2])
    Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
    prm = torch.ones((s.ncells, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        s.step_keep(Q, prm, dev([0.0, 1e-3]), torch.zeros(s.keep_size() + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        s.step_adjoint_kept(prm, dev([0.0, 1e-3]), torch.zeros(s.keep_size(), dtype=torch.float64, device="cuda"),
                            Q.clone(), None)


@pytest.mark.parametrize("nsteps", [1, 4])
def test_run_keep_equals_step_keep(nsteps):
    """adg_run_keep (fused corrector/predictor kernels for nsteps > 1) writes
    the same keep buffers and reaches the same state as nsteps adg_step_keep,
    and its receiver samples are adg_run's (two receivers share a cell)."""
    src = [dict(x=(700.0, 900.0, 400.0), w=[0.0] * 6 + [0.3, -0.2, 1.0], f0=5.0, t0=0.1, amp=1e7)]
    s, P, params, u, lam, dt = elastic((4, 3, 3), 3, seed=49, sources=src)
    s.set_receivers(np.array([[300.0, 400.0, 200.0], [1700.0, 1100.0, 900.0], [320.0, 410.0, 260.0]]))
    u *= 1e-3
    prm = dev(params)
    kn = s.keep_size()
    Qa, ca = dev(u), dev([0.02, dt])
    ka = torch.full((nsteps, kn), float("nan"), dtype=torch.float64, device="cuda")
    for n in range(nsteps):
        s.step_keep(Qa, prm, ca, ka[n])
    Qb, cb = dev(u), dev([0.02, dt])
    kb = torch.full((nsteps, kn), float("nan"), dtype=torch.float64, device="cuda")
    rb = torch.full((nsteps, 3, 9), float("nan"), dtype=torch.float64, device="cuda")
    s.run_keep(Qb, prm, cb, nsteps, kb, rb)
    # the samples are those of run()
    Qc, cc = dev(u), dev([0.02, dt])
    rc = torch.full((nsteps, 3, 9), float("nan"), dtype=torch.float64, device="cuda")
    s.run(Qc, prm, cc, nsteps, rc)
    torch.cuda.synchronize()
    say(f"run_keep nsteps={nsteps}: state max |diff| {float((Qa - Qb).abs().max()):.1e}")
    assert torch.equal(Qa, Qb) and torch.equal(ca, cb) and torch.equal(Qb, Qc)
    assert torch.equal(rb, rc)
    assert torch.equal(torch.nan_to_num(ka, nan=1.5), torch.nan_to_num(kb, nan=1.5))
    # every node slot is written at picard_iters = N + 1, and every state
    # trace behind them (the linear step leaves the flux traces unwritten)
    F = 4 * 4  # face nodes at N = 3
    nodes = kn - s.ncells * 6 * 2 * 9 * F
    assert nodes > 0 and nodes % (s.ncells * P.S) == 0
    assert not torch.isnan(kb[:, :nodes]).any()
    tr = kb[:, nodes:].reshape(nsteps, s.ncells, 6, 2, 9, F)
    assert not torch.isnan(tr[:, :, :, 0]).any() and torch.isnan(tr[:, :, :, 1]).all()
