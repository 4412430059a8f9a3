"""adg_step_noalloc (the step with its face traces and reduction slots in the
library's static device scratch array) against adg_step, through the C ABI.

Bar: the same kernels on the same inputs, so the state and the clock equal
adg_step's bit for bit; two calls in a row on one GPU, the second on a
smaller mesh (the array keeps the first call's contents); a mesh whose face
traces exceed the scratch array is refused.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import adg, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

UNSUPPORTED = -4


def say(*a):
    print("[gpu-test]", *a, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def both_paths(s, Q0, params, steps):
    """(state, clock) after `steps` steps with adg_step and with adg_step_noalloc."""
    L = adg.lib()
    prm = dev(params) if params is not None else None
    out = []
    for noalloc in (False, True):
        Q = dev(Q0)
        clock = dev([0.0, 0.0])
        s.stable_dt(Q, prm, clock)
        for _ in range(steps):
            if noalloc:
                st = L.adg_step_noalloc(s._ctx, Q.data_ptr(), prm.data_ptr() if prm is not None else None,
                                        clock.data_ptr(), adg.STEP_NEXT_DT, None)
                assert st == 0, L.adg_last_error()
            else:
                s.step(Q, prm, clock, next_dt=True)
        torch.cuda.synchronize()
        out.append((Q.cpu().numpy(), clock.cpu().numpy()))
    return out


def test_noalloc_step_equals_step_on_two_meshes():
    # first call: 3-D Euler N = 3 on 6 x 5 x 4 cells (1.2 MB of traces);
    # second call: the 2-D Euler wave of Eq. (8) on 5 x 4 cells (smaller)
    say("noalloc step, 3-D Euler N=3 6x5x4")
    P = O.problem(3, 3, O.EULER, [6, 5, 4])
    s = adg.Solver(3, 3, "euler", [6, 5, 4])
    Q0 = inputs.smooth_euler_state(O.node_coords(P), 71)
    (Qa, ca), (Qb, cb) = both_paths(s, Q0, None, 3)
    assert np.array_equal(Qa, Qb) and np.array_equal(ca, cb)
    s.close()
    say("noalloc step, 2-D Euler N=3 5x4 (smaller, after the larger call)")
    P2 = O.problem(2, 3, O.EULER, [5, 4])
    s2 = adg.Solver(2, 3, "euler", [5, 4])
    Q2 = inputs.c1_state(O.node_coords(P2))
    (Qa, ca), (Qb, cb) = both_paths(s2, Q2, None, 2)
    assert np.array_equal(Qa, Qb) and np.array_equal(ca, cb)
    Qo, to = O.run(P2, Q2, steps=2)
    assert np.linalg.norm(Qb - Qo) <= 1e-12 * np.linalg.norm(Qo)
    s2.close()


def test_noalloc_step_elastic_with_source():
    say("noalloc step, elastic N=2 with a point source")
    cfg = inputs.elastic_config("c3")
    cells = [3, 3, 2]
    s = adg.Solver(3, 2, "elastic", cells, [0.0] * 3, [1500.0, 1500.0, 1000.0])
    P = O.problem(3, 2, O.ELASTIC, cells, [0.0] * 3, [1500.0, 1500.0, 1000.0])
    src = dict(x=[700.0, 800.0, 300.0], weight=[0, 0, 0, 0, 0, 0, 0, 0, 1.0], f0=5.0, t0=0.1, amp=1e3)
    s.set_point_sources([src])
    prm = cfg["params"][:P.ncells]
    Q0 = inputs.elastic_smooth_state(O.node_coords(P), 72)
    (Qa, ca), (Qb, cb) = both_paths(s, Q0, prm, 2)
    assert np.array_equal(Qa, Qb) and np.array_equal(ca, cb)
    s.close()


def test_noalloc_step_refuses_meshes_beyond_the_scratch():
    say("noalloc step, too large")
    # 3-D Euler N = 5: 17,280 bytes of face traces per cell; 14^3 cells need 47 MB
    s = adg.Solver(3, 5, "euler", [14, 14, 14])
    Q = torch.zeros(s.state_shape, dtype=torch.float64, device="cuda")
    clock = dev([0.0, 1e-3])
    L = adg.lib()
    st = L.adg_step_noalloc(s._ctx, Q.data_ptr(), None, clock.data_ptr(), 0, None)
    assert st == UNSUPPORTED and b"static scratch" in L.adg_last_error()
    torch.cuda.synchronize()
    assert float(clock[1]) == 1e-3  # nothing enqueued
    s.close()
