"""Parity of the HIP discrete adjoint (through the C ABI) with the oracle's.

Bar: relative L2 <= 1e-12 for dJ/du^n and dJ/dm of one adjoint step and of
the checkpointed multi-step misfit gradient, on the same seeded inputs; the
adjoint identity <lam, A u> = <A^T lam, u> on the GPU's own step; central
finite differences of the GPU misfit against the GPU gradient to 1e-6.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import adg, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print("[gpu-test]", *a, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def elastic_case(cells, N, seed, sources=None):
    hi = [500.0 * c for c in cells]
    P = O.problem(3, N, O.ELASTIC, list(cells), hi=hi, sources=sources or ())
    s = adg.Solver(3, N, "elastic", list(cells), [0.0] * 3, hi)
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


def gpu_adjoint(s, u, params, lam, dt, t=0.0):
    lam_d = dev(lam)
    g_d = torch.zeros((s.ncells, s.nparam), dtype=torch.float64, device="cuda") if s.nparam else None
    s.step_adjoint(dev(u), dev(params) if params is not None else None, dev([t, dt]), lam_d, g_d)
    torch.cuda.synchronize()
    return lam_d.cpu().numpy(), (g_d.cpu().numpy() if g_d is not None else None)


# ragged last blocks of the predictor adjoint (30, 8, 4 and 2 cells per block
# at N = 1..4): (7, 3, 2), (4, 3, 5), (5, 2, 2), (7, 6, 5), (3, 3, 1); fewer
# cells than one block: (1, 1, 2)
@pytest.mark.parametrize("N,cells", [(1, (5, 4, 3)), (1, (7, 3, 2)), (2, (4, 3, 5)), (2, (5, 2, 2)),
                                     (3, (3, 4, 3)), (3, (7, 6, 5)), (3, (1, 1, 2)), (4, (3, 3, 1)),
                                     (4, (2, 2, 2))])
def test_step_adjoint_elastic_vs_oracle(N, cells):
    say(f"elastic adjoint N={N} cells={cells}")
    s, P, params, u, lam, dt = elastic_case(cells, N, seed=10 + N)
    lam_g, g_g = gpu_adjoint(s, u, params, lam, dt)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.0, lam)
    e_l, e_g = rel_l2(lam_g, lam_o), rel_l2(g_g[:, 1:], g_o[:, 1:])
    say(f"  rel L2 lam {e_l:.2e}, grad(cp, cs) {e_g:.2e}")
    assert e_l <= TOL and e_g <= TOL
    # rho: analytically zero (rho cancels); both sides at rounding level
    assert np.abs(g_g[:, 0]).max() <= 1e-10 * np.abs(g_o[:, 1:]).max()


def test_step_adjoint_fewer_picard_iterations_vs_oracle():
    """picard_iters = 2 < N + 1 at N = 3 (the adjoint unrolls up to N + 1)."""
    cells = (3, 2, 2)
    hi = [500.0 * c for c in cells]
    P = O.problem(3, 3, O.ELASTIC, list(cells), hi=hi, picard_iters=2)
    s = adg.Solver(3, 3, "elastic", list(cells), [0.0] * 3, hi, picard_iters=2)
    rng = np.random.default_rng(17)
    params = np.column_stack([rng.uniform(2000, 3000, P.ncells), rng.uniform(5000, 7000, P.ncells),
                              rng.uniform(2500, 3400, P.ncells)])
    u = rng.normal(size=(P.ncells, 9, P.S))
    lam = rng.normal(size=u.shape)
    dt = 0.5 * O.stable_dt(P, u, params)[0]
    lam_g, g_g = gpu_adjoint(s, u, params, lam, dt)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.0, lam)
    e_l, e_g = rel_l2(lam_g, lam_o), rel_l2(g_g[:, 1:], g_o[:, 1:])
    say(f"picard_iters=2: rel L2 lam {e_l:.2e}, grad {e_g:.2e}")
    assert e_l <= TOL and e_g <= TOL


def test_step_adjoint_elastic_point_source_vs_oracle():
    """A point source changes the forward iterates and so dJ/dm."""
    src = [dict(x=(700.0, 900.0, 400.0), w=[0.0] * 6 + [0.3, -0.2, 1.0], f0=5.0, t0=0.1, amp=1e7)]
    s, P, params, u, lam, dt = elastic_case((3, 3, 2), 3, seed=21, sources=src)
    u *= 1e-3
    lam_g, g_g = gpu_adjoint(s, u, params, lam, dt, t=0.05)
    lam_o, g_o = O.step_adjoint(P, u, params, dt, 0.05, lam)
    e_l, e_g = rel_l2(lam_g, lam_o), rel_l2(g_g[:, 1:], g_o[:, 1:])
    say(f"point source: rel L2 lam {e_l:.2e}, grad {e_g:.2e}")
    assert e_l <= TOL and e_g <= TOL


@pytest.mark.parametrize("dim,N,cells", [(2, 1, (7, 5)), (2, 3, (6, 9)), (2, 7, (3, 4)),
                                         (3, 2, (4, 3, 5)), (3, 3, (3, 3, 4)), (3, 5, (2, 3, 2)),
                                         (3, 6, (2, 2, 1))])
def test_step_adjoint_advection_vs_oracle(dim, N, cells):
    say(f"advection adjoint dim={dim} N={N} cells={cells}")
    adv = (0.7, -0.4, 0.3)[:dim]
    P = O.problem(dim, N, O.ADVECTION, list(cells), adv=adv, kappa=1.3)
    s = adg.Solver(dim, N, "advection", list(cells), adv=adv, kappa=1.3)
    rng = np.random.default_rng(dim * 10 + N)
    u = rng.normal(size=(P.ncells, 1, P.S))
    lam = rng.normal(size=u.shape)
    dt = O.stable_dt(P, u)[0]
    lam_g, _ = gpu_adjoint(s, u, None, lam, dt)
    lam_o, _ = O.step_adjoint(P, u, None, dt, 0.0, lam)
    e = rel_l2(lam_g, lam_o)
    say(f"  rel L2 {e:.2e}")
    assert e <= TOL


def test_step_adjoint_is_deterministic():
    """No atomics: two adjoint steps on the same inputs agree bitwise."""
    s, P, params, u, lam, dt = elastic_case((5, 4, 3), 3, seed=33)
    a = gpu_adjoint(s, u, params, lam, dt)
    b = gpu_adjoint(s, u, params, lam, dt)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_step_adjoint_dot_product_on_gpu_step():
    """<lam, A u> (GPU forward) = <A^T lam, u> (GPU adjoint), source-free."""
    s, P, params, u, lam, dt = elastic_case((6, 5, 4), 3, seed=31)
    Q = dev(u)
    s.step(Q, dev(params), dev([0.0, dt]), next_dt=False)
    lam_n, _ = gpu_adjoint(s, u, params, lam, dt)
    a = float((lam * Q.cpu().numpy()).sum())
    b = float((lam_n * u).sum())
    say(f"dot product: {a:.16e} vs {b:.16e}")
    assert abs(a - b) <= 1e-12 * abs(a)


def test_sample_receivers_adjoint_vs_oracle():
    s, P, params, u, lam, dt = elastic_case((4, 3, 3), 2, seed=41)
    rec = np.array([[300.0, 400.0, 200.0], [1700.0, 1100.0, 900.0], [320.0, 410.0, 260.0]])
    s.set_receivers(rec)
    rng = np.random.default_rng(42)
    lamrec = rng.normal(size=(3, 9))
    lam_d = dev(lam)
    s.sample_receivers_adjoint(dev(lamrec), lam_d)
    torch.cuda.synchronize()
    ref = lam.copy()
    O.sample_receivers_T(P, rec, lamrec, ref)
    e = rel_l2(lam_d.cpu().numpy() - lam, ref - lam)
    say(f"receiver transpose rel L2 {e:.2e}")
    assert e <= TOL


def misfit_case(seed=5, steps=6):
    cells = (4, 3, 3)
    lo, hi = [0.0] * 3, [2000.0, 1500.0, 1500.0]
    src = dict(x=(1250.0, 750.0, 600.0), w=[0.0] * 8 + [1.0], f0=5.0, t0=0.0, amp=1e6)
    P = O.problem(3, 2, O.ELASTIC, list(cells), lo, hi, sources=[src])
    s = adg.Solver(3, 2, "elastic", list(cells), lo, hi)
    s.set_point_sources([dict(x=src["x"], weight=src["w"], f0=src["f0"], t0=src["t0"], amp=src["amp"])])
    cen = inputs.cell_centres(cells, lo, hi)
    params = inputs.layered_material(cen[:, 2] * 4.0, seed)
    params_obs = params * (1.0 + 0.05 * np.random.default_rng(seed + 1).uniform(-1, 1, params.shape))
    rec = np.array([[300.0, 400.0, 200.0], [1700.0, 1100.0, 900.0], [1000.0, 700.0, 1400.0]])
    s.set_receivers(rec)
    u0 = np.zeros((P.ncells, 9, P.S))
    dt = 0.5 * min(O.stable_dt(P, u0, params)[0], O.stable_dt(P, u0, params_obs)[0])
    _, data, _ = O.seismogram_misfit(P, u0, params_obs, dt, steps, rec)
    cellsr = np.array([int(x[0] // 500) + 4 * (int(x[1] // 500) + 3 * int(x[2] // 500)) for x in rec])
    return s, P, params, u0, dt, steps, rec, data, cellsr


def gpu_misfit(s, u0, params, dt, steps, data, cellsr, every):
    from paper_1905_07987_amd.autograd import seismograms
    u = dev(u0).requires_grad_(True)
    m = dev(params).requires_grad_(True)
    samp = seismograms(s, u, m, dt, steps, every=every)
    rho = m[torch.as_tensor(cellsr, device="cuda"), 0]
    v = samp[:, :, 6:9] / rho[None, :, None]
    J = 0.5 * dt * ((v - dev(data)) ** 2).sum()
    return J, u, m


@pytest.mark.parametrize("every", [1, 2, 4, 6])
def test_misfit_gradient_vs_oracle(every):
    s, P, params, u0, dt, steps, rec, data, cellsr = misfit_case()
    J, u, m = gpu_misfit(s, u0, params, dt, steps, data, cellsr, every)
    J.backward()
    Jo, gu_o, gm_o = O.misfit_gradient(P, u0, params, dt, steps, rec, data)
    e_J = abs(float(J.detach()) - Jo) / Jo
    e_u = rel_l2(u.grad.cpu().numpy(), gu_o)
    e_m = rel_l2(m.grad.cpu().numpy(), gm_o)
    say(f"misfit every={every}: J {e_J:.2e}, dJ/du0 {e_u:.2e}, dJ/dm {e_m:.2e}")
    assert e_J <= TOL and e_u <= TOL and e_m <= TOL


def test_misfit_gradient_is_the_same_for_every_checkpoint_interval():
    """The checkpoint interval changes which kernels run (fused multi-step
    runs forward, single steps when a segment is recomputed), not the
    arithmetic: the fused step equals the single step bit for bit and both
    sample the receivers with the same ordered sum, so J and the gradients
    are bitwise the same for every interval, K = 1 (every state kept)
    included."""
    s, P, params, u0, dt, steps, rec, data, cellsr = misfit_case()
    res = []
    for every in (1, 3, 6):
        J, u, m = gpu_misfit(s, u0, params, dt, steps, data, cellsr, every)
        J.backward()
        res.append((float(J.detach()), u.grad.clone(), m.grad.clone()))
    for J1, gu, gm in res[1:]:
        assert J1 == res[0][0] and torch.equal(gu, res[0][1]) and torch.equal(gm, res[0][2])


def test_checkpointed_adjoint_runs_once():
    """The backward pass consumes its checkpoints and the forward pass's kept
    last segment: a second backward through the same graph is an error, not
    a wrong gradient."""
    s, P, params, u0, dt, steps, rec, data, cellsr = misfit_case()
    J, u, m = gpu_misfit(s, u0, params, dt, steps, data, cellsr, every=4)
    J.backward(retain_graph=True)
    with pytest.raises(RuntimeError, match="once per forward"):
        J.backward()


def test_misfit_gradient_finite_differences_on_gpu():
    """Central differences of the GPU misfit at the largest-gradient entries."""
    s, P, params, u0, dt, steps, rec, data, cellsr = misfit_case(seed=7)
    J, u, m = gpu_misfit(s, u0, params, dt, steps, data, cellsr, every=3)
    J.backward()
    g = m.grad.cpu().numpy()
    flat = np.abs(g).ravel()
    cand = np.nonzero(flat >= 1e-2 * flat.max())[0]
    rng = np.random.default_rng(11)
    for idx in rng.choice(cand, size=min(6, len(cand)), replace=False):
        c, p = divmod(int(idx), 3)
        h = 1e-4 * params[c, p]
        vals = []
        for sgn in (1, -1):
            pp = params.copy()
            pp[c, p] += sgn * h
            with torch.no_grad():
                Jx, _, _ = gpu_misfit(s, u0, pp, dt, steps, data, cellsr, every=3)
            vals.append(float(Jx))
        fd = (vals[0] - vals[1]) / (2 * h)
        say(f"cell {c} param {p}: fd {fd:.10e} adjoint {g[c, p]:.10e}")
        assert abs(fd - g[c, p]) <= 1e-6 * abs(fd)


def test_adjoint_error_paths():
    e = adg.Solver(3, 2, "euler", [2, 2, 2])
    Q = torch.zeros(e.state_shape, dtype=torch.float64, device="cuda")
    with pytest.raises(adg.AdgError) as ei:
        e.step_adjoint(Q, None, dev([0.0, 1e-3]), Q.clone())
    assert ei.value.status == -4
    s = adg.Solver(3, 2, "elastic", [2, 2, 2], picard_iters=5)
    Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
    prm = torch.ones((s.ncells, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(adg.AdgError) as ei:
        s.step_adjoint(Q, prm, dev([0.0, 1e-3]), Q.clone(), prm.clone())
    assert ei.value.status == -4
    s = adg.Solver(3, 2, "elastic", [2, 2, 2])
    with pytest.raises(ValueError):
        s.step_adjoint(Q, prm, dev([0.0, 1e-3]), Q.clone(), None)
    with pytest.raises(adg.AdgError) as ei:
        s.sample_receivers_adjoint(torch.zeros((0, 9), dtype=torch.float64, device="cuda"), Q)
    assert ei.value.status == -6


def test_c4_full_size_dot_product():
    """32^3 cells, N=3: the adjoint step in the benchmark's launch
    configuration against the GPU's own forward step (<lam, A u> = <A^T lam, u>
    for the source-free step)."""
    cfg = inputs.elastic_config("c4")
    s = adg.Solver(3, 3, "elastic", list(cfg["cells"]), cfg["lo"], cfg["hi"])
    prm = dev(cfg["params"])
    g = torch.Generator(device="cuda").manual_seed(71)
    u = torch.randn(s.state_shape, dtype=torch.float64, device="cuda", generator=g)
    lam = torch.randn(s.state_shape, dtype=torch.float64, device="cuda", generator=g)
    clock = dev([0.0, 0.0])
    s.stable_dt(u, prm, clock)
    Au = u.clone()
    s.step(Au, prm, clock.clone(), next_dt=False)
    lam_n = lam.clone()
    gp = torch.zeros_like(prm)
    s.step_adjoint(u, prm, clock, lam_n, gp)
    a = float((lam * Au).sum())
    b = float((lam_n * u).sum())
    say(f"c4 dot product: {a:.16e} vs {b:.16e}")
    assert abs(a - b) <= 1e-12 * abs(a)


def test_c4_gradient_finite_differences():
    """The C4 gradient (200 steps, 16 receivers, checkpoints every 15 steps)
    against central differences of the GPU misfit on 20 seeded (cell,
    parameter) samples: 4 rho samples among the receivers' cells (the only
    cells where J depends on rho) and 16 cp / cs samples among those with
    |g| >= 1e-2 max |g|, leaving out cp samples at a Rusanov-speed tie.  The
    misfit bends on the scale of a
    travel-time shift: a plain central difference at h = 1e-4 of the
    parameter still carries an O(h^2) error of up to 2e-6, and below 3e-5 the
    forward solution's rounding noise takes over (1e-6 at h = 1e-5).  The
    check therefore extrapolates central differences at h and 2h
    (Richardson, error O(h^4)), h = 1e-4 of the parameter."""
    from paper_1905_07987_amd.autograd import seismograms
    cfg = inputs.elastic_config("c4")
    steps = cfg["steps"]
    s = adg.Solver(3, 3, "elastic", list(cfg["cells"]), cfg["lo"], cfg["hi"])
    s.set_point_sources([cfg["source"]])
    s.set_receivers(cfg["receivers"])
    params = cfg["params"]
    pert = np.random.default_rng(cfg["seed"] + 1).uniform(-1.0, 1.0, params.shape)
    params_obs = params * (1.0 + 0.05 * pert)
    u0 = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
    clock = dev([0.0, 0.0])
    s.stable_dt(u0, dev(params), clock)
    dt1 = float(clock[1])
    s.stable_dt(u0, dev(params_obs), clock)
    dt = min(dt1, float(clock[1]))
    h = np.array([(cfg["hi"][d] - cfg["lo"][d]) / cfg["cells"][d] for d in range(3)])
    rc = np.floor((cfg["receivers"] - np.array(cfg["lo"])) / h).astype(np.int64)
    cellsr = torch.as_tensor(rc[:, 0] + cfg["cells"][0] * (rc[:, 1] + cfg["cells"][1] * rc[:, 2]),
                             device="cuda")
    with torch.no_grad():
        sm = seismograms(s, u0, dev(params_obs), dt, steps)
        data = sm[:, :, 6:9] / dev(params_obs)[cellsr, 0][None, :, None]

    def misfit(m):
        sm = seismograms(s, u0, m, dt, steps, every=15)
        v = sm[:, :, 6:9] / m[cellsr, 0][None, :, None]
        return 0.5 * dt * ((v - data) ** 2).sum()

    say("c4: gradient")
    m = dev(params).requires_grad_(True)
    J = misfit(m)
    J.backward()
    g = m.grad.cpu().numpy()
    # cp and cs: cells with |g| >= 1e-2 max|g|; rho: it enters J only through
    # v = (rho v) / rho at the receivers' cells (the stress rows see lambda / rho
    # and mu / rho, which do not depend on rho), so its candidates are those
    # cells, with the threshold relative to the largest rho derivative
    flat = np.abs(g[:, 1:]).ravel()
    cand = [divmod(int(i), 2) for i in np.nonzero(flat >= 1e-2 * flat.max())[0]]
    cand = [(c, p + 1) for c, p in cand]
    # cp is the Rusanov speed of its faces, max(cp_L, cp_R): J has a kink where
    # a face neighbour's cp is equal.  The difference stencil below reaches
    # +-2e-4 cp, so cp samples whose nearest neighbour cp is closer than 4e-4
    # (relative) are not differentiable over the stencil and are left out.
    n3 = 32
    cc = np.arange(params.shape[0])
    cx, cy, cz = cc % n3, (cc // n3) % n3, cc // (n3 * n3)
    gap = np.full(params.shape[0], np.inf)
    for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        o = (cx + dx) % n3 + n3 * ((cy + dy) % n3 + n3 * ((cz + dz) % n3))
        gap = np.minimum(gap, np.abs(params[o, 1] - params[:, 1]) / params[:, 1])
    cand = [(c, p) for c, p in cand if p == 2 or gap[c] > 4e-4]
    grho = np.abs(g[:, 0])
    cand_rho = [(int(c), 0) for c in np.nonzero(grho >= 1e-2 * grho.max())[0]]
    rng = np.random.default_rng(7989)
    pick_rho = [cand_rho[i] for i in rng.choice(len(cand_rho), size=min(4, len(cand_rho)), replace=False)]
    pick_cs = [cand[i] for i in rng.choice(len(cand), size=20 - len(pick_rho), replace=False)]
    picks = pick_rho + pick_cs
    assert len(pick_rho) >= 3 and len(picks) == 20
    worst = 0.0
    for c, p in picks:
        hstep = 1e-4 * params[c, p]
        cd = []
        for hh in (hstep, 2 * hstep):
            vals = []
            for sgn in (1, -1):
                pp = params.copy()
                pp[c, p] += sgn * hh
                with torch.no_grad():
                    vals.append(float(misfit(dev(pp))))
            cd.append((vals[0] - vals[1]) / (2 * hh))
        fd = (4.0 * cd[0] - cd[1]) / 3.0
        err = abs(fd - g[c, p]) / abs(fd)
        worst = max(worst, err)
        assert err <= 1e-6, (c, p, fd, g[c, p])
    say(f"c4: 20 cells ({len(pick_rho)} rho), worst relative difference {worst:.2e}")
