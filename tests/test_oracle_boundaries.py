"""Pins of the oracle's non-periodic boundary conditions (CPU).

The outside state and normal flux of a boundary face are built from the
cell's own time-averaged traces (the paper's boundaryValues user function,
Table 2; walls in its Euler explosion problem): OUTFLOW copies them, WALL
takes their mirror image (Euler: normal momentum reversed; elasticity:
traction reversed).  Pins:
  - mirror image: Euler with walls at both ends of x on [0, 1] equals the
    periodic run on [-1, 1] started from the even mirror image of the data
    (rho, E, j_y even in x, j_x odd): at x = 0 and x = +-1 the periodic
    neighbour's trace is exactly the mirrored own trace;
  - a reflecting box conserves mass and energy (the outside flux is the
    mirror image of the inside one, so no mass or energy crosses a wall;
    momentum is not conserved: the wall pushes back);
  - outflow keeps a uniform moving state (free stream);
  - a uniform traction-free elastic state stays as it is with free surfaces;
  - invalid combinations are refused.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import inputs

W, OUT, PER = O.BC_WALL, O.BC_OUTFLOW, O.BC_PERIODIC


def mirror_x(P_half, Q_half):
    """[cells_y][cells_x] half-domain data -> the even mirror image on twice
    the cells in x: mirrored cells first, node order reversed along x, j_x
    negated (Euler 2-D)."""
    n, cx, cy = P_half.n, P_half.cells[0], P_half.cells[1]
    nv = P_half.nvar
    q = Q_half.reshape(cy, cx, nv, n, n)           # [cy][cx][v][ky][kx]
    m = q[:, ::-1, :, :, ::-1].copy()               # reflected cells and nodes
    m[:, :, 1] *= -1.0                               # j_x
    full = np.concatenate([m, q], axis=1)            # x from -1 to 1
    return full.reshape(cy * 2 * cx, nv, n * n)


@pytest.mark.parametrize("N", [2, 3])
def test_euler_wall_is_the_mirror_image_of_a_periodic_run(N):
    cells = [4, 3]
    Pw = O.problem(2, N, O.EULER, cells, [0.0, 0.0], [1.0, 1.0], bc=[W, W, PER, PER])
    Pp = O.problem(2, N, O.EULER, [8, 3], [-1.0, 0.0], [1.0, 1.0])
    Q0 = inputs.smooth_euler_state(O.node_coords(Pw), 61)
    Qp0 = mirror_x(Pw, Q0)
    dt = 0.5 * O.stable_dt(Pw, Q0)[0]
    Qw, _ = O.run(Pw, Q0, steps=4, dt_fixed=dt)
    Qp, _ = O.run(Pp, Qp0, steps=4, dt_fixed=dt)
    right = Qp.reshape(3, 8, Pw.nvar, -1)[:, 4:].reshape(Qw.shape)
    assert np.linalg.norm(right - Qw) <= 1e-12 * np.linalg.norm(Qw)
    assert np.linalg.norm(Qw - Q0) > 1e-4 * np.linalg.norm(Q0)  # the run did something


def cell_integrals(P, Q):
    T = O.tables(P.n)
    w = T["w"]
    wk = w
    for _ in range(P.dim - 1):
        wk = np.multiply.outer(w, wk).ravel()  # x fastest
    vol = np.prod(P.h)
    return (Q * wk[None, None, :]).sum(axis=(0, 2)) * vol


@pytest.mark.parametrize("dim,cells", [(2, [5, 4]), (3, [3, 2, 2])])
def test_reflecting_box_conserves_mass_and_energy(dim, cells):
    P = O.problem(dim, 3, O.EULER, cells, bc=[W] * (2 * dim))
    Q0 = inputs.smooth_euler_state(O.node_coords(P), 62)
    Q, _ = O.run(P, Q0, steps=5)
    m0, m1 = cell_integrals(P, Q0), cell_integrals(P, Q)
    for v in (0, dim + 1):
        assert abs(m1[v] - m0[v]) <= 1e-13 * abs(m0[v]), (v, m0[v], m1[v])
    # the walls exchange momentum with the fluid
    assert max(abs(m1[1 + a] - m0[1 + a]) for a in range(dim)) > 1e-8


def test_outflow_keeps_a_uniform_moving_state():
    P = O.problem(2, 3, O.EULER, [4, 3], bc=[OUT, OUT, OUT, OUT])
    rho, u, v, p = 1.3, 0.4, -0.25, 0.9
    q = np.array([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    Q0 = np.broadcast_to(q[None, :, None], (P.ncells, 4, P.S)).copy()
    Q, _ = O.run(P, Q0, steps=3)
    assert np.abs(Q - Q0).max() <= 1e-14 * np.abs(Q0).max()


def test_traction_free_uniform_elastic_state_stays():
    P = O.problem(3, 2, O.ELASTIC, [3, 2, 2], hi=[1500.0, 1000.0, 1000.0], bc=[W] * 6)
    prm = np.tile([2700.0, 6000.0, 3464.0], (P.ncells, 1))
    q = np.array([0.0] * 6 + [1.2, -0.7, 0.4])
    Q0 = np.broadcast_to(q[None, :, None], (P.ncells, 9, P.S)).copy()
    Q, _ = O.run(P, Q0, prm, steps=3)
    # velocities to rounding; stresses to rounding of the impedance scale
    assert np.abs(Q[:, 6:] - Q0[:, 6:]).max() <= 1e-14 * np.abs(Q0).max()
    assert np.abs(Q[:, :6]).max() <= 1e-14 * 2700.0 * 6000.0 * np.abs(Q0).max()
    # a uniform stress is not traction free: the surfaces respond
    Q1 = Q0.copy()
    Q1[:, 0] = 1e6
    Q2, _ = O.run(P, Q1, prm, steps=1)
    assert np.abs(Q2[:, 6]).max() > 1.2 + 1e-3


@pytest.mark.parametrize("pde,dim,bc", [(O.EULER, 2, [W, PER, PER, PER]),
                                         (O.ADVECTION, 2, [W, W, PER, PER]),
                                         (O.EULER, 2, [PER, PER, PER, PER, W, W])])
def test_invalid_boundary_combinations_are_refused(pde, dim, bc):
    P = O.problem(dim, 2, pde, [3, 3], bc=bc)
    Q = np.ones((P.ncells, P.nvar, P.S))
    with pytest.raises(Exception):
        O.step(P, Q, None, 1e-3)


IN = O.BC_INFLOW


@pytest.mark.parametrize("side", [0, 1])
def test_inflow_face_is_upwind_for_advection(side):
    # a = +-e_x, uniform q = 2, inflow 3 on the upstream face: the Rusanov
    # flux there is the upwind a q_in, so one step changes only the cells on
    # that face, by dt l(xi_k) / (h w_k) at their nodes (l = l0 at x = 0,
    # l1 at x = 1), and leaves every other cell at exactly 2
    N, cells = 3, [5, 3]
    a = 1.0 if side == 0 else -1.0
    bc = [IN, OUT, PER, PER] if side == 0 else [OUT, IN, PER, PER]
    P = O.problem(2, N, O.ADVECTION, cells, adv=(a, 0.0), kappa=0.0, bc=bc, bc_state={side: [3.0]})
    Q = np.full((P.ncells, 1, P.S), 2.0)
    dt = 0.01
    Q1 = O.step(P, Q, None, dt)
    T = O.tables(P.n)
    h = 1.0 / cells[0]
    kx = np.arange(P.S) % P.n
    lb = T["l0"] if side == 0 else T["l1"]
    bump = dt * lb[kx] / (h * T["w"][kx])
    for c in range(P.ncells):
        cx = c % cells[0]
        if cx == (0 if side == 0 else cells[0] - 1):
            np.testing.assert_allclose(Q1[c, 0], 2.0 + bump, rtol=0, atol=1e-14)
        else:
            assert np.array_equal(Q1[c, 0], Q[c, 0])


def test_inflow_of_the_interior_state_keeps_a_uniform_euler_flow():
    q = [1.2, 0.6, -0.3, 3.1]
    P = O.problem(2, 3, O.EULER, [4, 3], bc=[IN, OUT, IN, IN], bc_state={0: q, 2: q, 3: q})
    Q = np.tile(np.array(q)[None, :, None], (P.ncells, 1, P.S))
    Q1 = O.step(P, Q, None, 0.5 * O.stable_dt(P, Q)[0])
    assert np.abs(Q1 - Q).max() < 1e-14
