"""Host-side checks of libadg that need no GPU: the library loads, exports
every symbol include/adg.h declares, and its own basis tables (built by code
that shares nothing with the oracle) agree with the oracle's."""
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1905_07987_amd import adg

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "adg.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(adg_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = adg.lib()
    names = _declared()
    assert "adg_step" in names and "adg_stable_dt" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(adg.EXPORTED)


@pytest.mark.parametrize("order", range(0, 8))
def test_library_tables_match_oracle(order):
    n = order + 1
    A = adg.basis_tables(order)
    B = O.tables(n)
    ulp = np.finfo(np.float64).eps
    np.testing.assert_allclose(A["xi"], B["xi"], rtol=0, atol=2 * ulp)
    np.testing.assert_allclose(A["w"], B["w"], rtol=0, atol=2 * ulp)
    np.testing.assert_allclose(A["l0"], B["l0"], rtol=0, atol=8 * ulp * max(1, np.abs(B["l0"]).max()))
    np.testing.assert_allclose(A["l1"], B["l1"], rtol=0, atol=8 * ulp * max(1, np.abs(B["l1"]).max()))
    np.testing.assert_allclose(A["D"], B["D"], rtol=0, atol=16 * ulp * max(1, np.abs(B["D"]).max()))
    np.testing.assert_allclose(A["K1inv"], B["K1inv"], rtol=0,
                               atol=16 * ulp * max(1, np.abs(B["K1inv"]).max()))


def test_built_orders():
    assert adg.max_order("euler", 2) >= 3
    assert adg.max_order("euler", 3) >= 5
    assert adg.max_order("elastic", 3) >= 4
    assert adg.max_order("elastic", 2) == 0
    assert adg.max_order(99, 3) == 0


def test_bad_order_is_an_error_not_a_crash():
    with pytest.raises(adg.AdgError) as e:
        adg.basis_tables(8)
    assert e.value.status == -1


@pytest.mark.parametrize("order", range(0, 8))
def test_library_limiter_tables_match_oracle(order):
    # two constructions that share nothing: exact antiderivatives of the
    # monomial expansion and Cholesky (library) against subinterval Gauss
    # quadrature and Gauss-Jordan on the normal equations (oracle)
    A, B, Qf = adg.limiter_tables(order)
    Ao, Bo, Qfo = O.limiter_tables(order + 1)
    np.testing.assert_allclose(A, Ao, rtol=0, atol=1e-14)
    np.testing.assert_allclose(B, Bo, rtol=0, atol=1e-13 * max(1.0, np.abs(Bo).max()))
    np.testing.assert_allclose(Qf, Qfo, rtol=0, atol=1e-14 * max(1.0, np.abs(Qfo).max()))
    assert np.abs(B @ A - np.eye(order + 1)).max() < 1e-13


def test_bad_limiter_order_is_an_error():
    with pytest.raises(adg.AdgError) as e:
        adg.limiter_tables(8)
    assert e.value.status == -1
    with pytest.raises(adg.AdgError):
        adg.limiter_tables(-1)


def test_checkpoint_segments():
    """The checkpointed adjoint's segments: whole segments of `every` steps
    counted from the end (the forward pass keeps the last one), the first
    one the remainder; they tile 0..steps."""
    from paper_1905_07987_amd.autograd import _segments
    for steps, every in [(200, 15), (6, 4), (6, 6), (6, 1), (7, 3), (1, 1), (5, 10), (30, 15)]:
        b = _segments(steps, every)
        lens = [b[i + 1] - b[i] for i in range(len(b) - 1)]
        assert b[0] == 0 and b[-1] == steps and len(lens) == -(-steps // every)
        assert all(0 < n <= every for n in lens) and all(n == every for n in lens[1:])
    assert _segments(200, 15)[:3] == [0, 5, 20]
    assert _segments(0, 4) == [0]  # no steps: no segment
