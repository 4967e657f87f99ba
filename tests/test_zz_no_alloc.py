"""The entry point that allocates nothing (sq_stress_static): its sums live
in the library's static device scratch.  Checked through the C ABI against
sq_stress, bit for bit, on two calls in a row, the second with a smaller
input (a cell with fewer nodes), in both orders of the two entry points."""

import numpy as np
import pytest

from paper_2006_03697_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sq():
    import torch
    from paper_2006_03697_amd import sq as sqmod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    sqmod.load()
    return sqmod


def _cells():
    big = W.random_cell(seed=21, L=8.0, h=0.4, n_atoms=10, d_min=1.5, rcut=2.0, npl=30, kT=0.1)
    small = W.tiny_cell(npl=20)
    return [big, small]   # 8000 and 1728 nodes


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_static_scratch_stress_matches_sq_stress(sq, precision):
    cells = _cells()
    with sq.Plan(cells, precision=precision) as P:
        P.density(-1)
        # the static entry point first: cell 0, then the smaller cell 1
        s0, p0 = P.stress_static(0)
        s1, p1 = P.stress_static(1)
        r0, q0 = P.stress(0)
        r1, q1 = P.stress(1)
        assert np.array_equal(s0, r0) and np.array_equal(p0, q0)
        assert np.array_equal(s1, r1) and np.array_equal(p1, q1)
        # again after sq_stress, and over both cells at once
        t, u = P.stress_static(-1)
        assert np.array_equal(t[0], r0[0]) and np.array_equal(t[1], r1[0])
        assert np.array_equal(u[0], q0[0]) and np.array_equal(u[1], q1[0])
        # a second plan on the same GPU shares the array: its results are
        # its own (the rows are rewritten before they are read)
        with sq.Plan([cells[1]], precision=precision) as Q:
            Q.density(0)
            a, b = Q.stress_static(0)
            c, d = Q.stress(0)
            assert np.array_equal(a, c) and np.array_equal(b, d)
        s0b, _ = P.stress_static(0)
        assert np.array_equal(s0b, r0)


def test_static_scratch_stress_state_checks(sq):
    with sq.Plan([W.tiny_cell()], precision="fp64") as P:
        with pytest.raises(sq.SqError) as e:
            P.stress_static(0)
        assert e.value.status == sq.SQ_E_STATE
        P.density(0)
        with pytest.raises(sq.SqError) as e:
            P.stress_static(3)
        assert e.value.status == sq.SQ_E_ARG
        # sq_pressure still runs its own stress pass after the static call
        s, _ = P.stress_static(0)
        pd, pt = P.pressure(0)
        r, _ = P.stress(0)
        assert np.array_equal(s, r)
        assert abs(pt[0] + (r[0][0] + r[0][1] + r[0][2]) / 3) < 1e-12 * abs(pt[0])
