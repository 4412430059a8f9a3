"""The split-BF16 predictor (ADG_MIXED_BF16X3: derivative contractions on
the matrix cores with three-term BF16 splits and FP32 accumulation, the
rest of the predictor in FP32, dt, faces and update in FP64) against the
FP64 oracle.

Not a parity pin (mixed precision): the bar is the error statement.  Each
derivative keeps the partial products down to 2^-16 of the product, so the
result carries FP32-sized errors, ~1e-7 relative after a few steps (the
FP32 predictor's); bound 1e-6, and on the paper's density wave the error
against the closed form is no larger than the FP32 predictor's (both sit
above the FP64 discretisation error at this resolution: 5.8e-7 and 6.8e-7
against the oracle, 2.5e-7 for FP64 against the closed form, 16^2 cells
N = 3, 10 steps).
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import adg, inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, flush=True)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def run(s, Q0, steps):
    Q, clock = dev(Q0), dev([0.0, 0.0])
    s.stable_dt(Q, None, clock)
    for _ in range(steps):
        s.step(Q, None, clock, next_dt=True)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), float(clock[0])


def test_bf16x3_c1_against_oracle_and_closed_form():
    say("bf16x3 c1")
    P = O.problem(2, 3, O.EULER, [16, 16], cfl=0.9)
    Q0 = inputs.c1_state(O.node_coords(P))
    Qo, t = O.run(P, Q0, steps=10)
    exact = inputs.c1_state(O.node_coords(P), t)
    res = {}
    for prec in ("bf16x3", "fp32", "fp64"):
        s = adg.Solver(2, 3, "euler", [16, 16], cfl=0.9, precision=prec)
        Q, tg = run(s, Q0, 10)
        res[prec] = (rel_l2(Q, Qo), rel_l2(Q, exact))
        s.close()
    say("  vs oracle / vs closed form: " + ", ".join(f"{k} {v[0]:.1e} / {v[1]:.2e}" for k, v in res.items()))
    assert res["bf16x3"][0] <= 1e-6
    assert res["bf16x3"][1] <= 1.05 * res["fp32"][1]


@pytest.mark.parametrize("cells", [[4, 3, 3], [3, 2, 2]])
def test_bf16x3_c2_shape_against_oracle(cells):
    say("bf16x3 3-D Euler N=5", cells)
    P = O.problem(3, 5, O.EULER, cells, cfl=0.5)
    Q0 = inputs.c2_state(O.node_coords(P))
    Q0[:, 1:4] += 0.1 * inputs.smooth_euler_state(O.node_coords(P), 63)[:, 1:4]
    Qo, _ = O.run(P, Q0, steps=3)
    s = adg.Solver(3, 5, "euler", cells, cfl=0.5, precision="bf16x3")
    Q, _ = run(s, Q0, 3)
    s32 = adg.Solver(3, 5, "euler", cells, cfl=0.5, precision="fp32")
    Q32, _ = run(s32, Q0, 3)
    e, e32 = rel_l2(Q, Qo), rel_l2(Q32, Qo)
    say(f"  rel L2 vs oracle: bf16x3 {e:.2e}, fp32 {e32:.2e}")
    assert e <= 1e-6 and np.isfinite(Q).all()
    s.close()
    s32.close()


def test_bf16x3_errors():
    for pde, dim in (("elastic", 3), ("advection", 2)):
        with pytest.raises(adg.AdgError) as e:
            adg.Solver(dim, 2, pde, [2] * dim, precision="bf16x3")
        assert e.value.status == -4
