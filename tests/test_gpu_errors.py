"""Error paths of the C-ABI that need a device context: each misuse returns
its documented code, leaves the context usable, and a later step gives the
same state as a context that never saw the error."""
import numpy as np
import pytest

from paper_1410_0753_amd import synth

pytestmark = pytest.mark.gpu

EINVAL, ECFL, EHIP, ENONFINITE, ESTATE, ENOSPACE = -1, -2, -3, -4, -5, -6


@pytest.fixture(scope="module")
def clf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0753_amd import clf as m
    m.load()
    return m


def code(clf, fn, *a, **k):
    with pytest.raises(clf.ClfError) as e:
        fn(*a, **k)
    return e.value.code


@pytest.fixture
def case():
    return synth.random_small(21, 40, 30, land=True, amp=0.2)


def still_works(clf, s, case):
    # the context steps on and matches a fresh one
    ref = clf.Solver.from_case(case)
    for obj in (s, ref):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.step(5)
    for a, b in zip(s.raw_state(), ref.raw_state()):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_gauge_errors(clf, case):
    s = clf.Solver.from_case(case, max_gauges=2, gauge_capacity=3, gout=1)
    assert code(clf, s.set_gauges, [1, 50], [1, 1]) == EINVAL        # outside the grid
    assert code(clf, s.set_gauges, [1, 2, 3], [1, 1, 1]) == ENOSPACE  # more than max_gauges
    s.set_gauges([1, 2], [3, 4])
    s.set_initial(case.eta0)
    # records at n = 0, 1, 2 fit; a step past the capacity is refused up front
    s.step(2)
    assert code(clf, s.step, 5) == ENOSPACE
    assert s.query(clf.Q_STEP) == 2
    s.clear_records()
    s.step(1)
    assert s.query(clf.Q_STEP) == 3


def test_enclosed_grid_errors(clf, case):
    s = clf.Solver.from_case(case, max_enclosed=1, bndout=1)
    x, y = case.x.astype(np.float64), case.y.astype(np.float64)
    inside_x = np.linspace(x[3], x[10], 8)
    inside_y = np.linspace(y[3], y[10], 8)
    assert code(clf, s.add_enclosed_grid, inside_x + 1e7, inside_y) == EINVAL   # outside
    assert s.add_enclosed_grid(inside_x, inside_y) == 0
    assert code(clf, s.add_enclosed_grid, inside_x, inside_y) == ENOSPACE       # max_enclosed
    lib = clf.load()
    assert lib.clf_read_boundary_series(s._h, 5, 0, None, None, None, 0) == EINVAL  # bad id
    assert lib.clf_read_boundary_series(s._h, 0, 9, None, None, None, 0) == EINVAL  # bad side
    still_works(clf, s, case)


def test_forcing_errors(clf, case):
    s = clf.Solver.from_case(case, forcing_capacity=4)
    vals = np.zeros((2, 3, case.ny))
    assert code(clf, s.set_boundary_forcing, 7, [0.0, 1.0], vals) == EINVAL      # bad side
    assert code(clf, s.set_boundary_forcing, clf.WEST, [1.0, 0.0], vals) == EINVAL   # times
    big = np.zeros((5, 3, case.ny))
    assert code(clf, s.set_boundary_forcing, clf.WEST, np.arange(5.0), big) == ENOSPACE
    one_d = synth.random_small(22, 60, 1, land=False)
    t = clf.Solver.from_case(one_d, forcing_capacity=4)
    assert code(clf, t.set_boundary_forcing, clf.SOUTH, [0.0, 1.0], np.zeros((2, 3, 60))) == EINVAL
    assert code(clf, t.sweep, 1) == EINVAL          # no sweep along a dimension of length 1
    still_works(clf, s, case)


def test_misc_errors(clf, case):
    s = clf.Solver.from_case(case)
    assert code(clf, s.sweep, 2) == EINVAL
    assert code(clf, s.query, 999) == EINVAL
    assert code(clf, s.set_raw_state, case.depth, case.u0, case.v0, -1) == EINVAL
    bad = case.depth.astype(np.float64).copy()
    bad[3, 4] = np.nan
    assert code(clf, clf.Solver, case.x, case.y, bad, case.dt) == EINVAL        # non-finite depth
    assert code(clf, clf.Solver, case.x, case.y, case.depth, -1.0) == EINVAL    # dt <= 0
    still_works(clf, s, case)


def test_adjoint_errors(clf, case):
    f32 = clf.Solver.from_case(case, precision=clf.FP32)
    f32.set_initial(case.eta0)
    assert code(clf, f32.adjoint_forward, 10) == EINVAL                # FP64 only
    alt = clf.Solver.from_case(case, sweep_order=clf.ORDER_ALTERNATE)
    alt.set_initial(case.eta0)
    assert code(clf, alt.adjoint_forward, 10) == EINVAL                # x-y order only
    s = clf.Solver.from_case(case, gout=2)
    s.set_gauges([5, 20], [5, 20])
    s.set_initial(case.eta0)
    assert code(clf, s.adjoint_backward, np.zeros((6, 2, 3))) == ESTATE  # no forward run
    s.step(3)
    assert code(clf, s.adjoint_forward, 10) == ESTATE                  # not from set_initial
    s.set_initial(case.eta0)
    s.adjoint_forward(10)
    assert code(clf, s.adjoint_backward, np.zeros((4, 2, 3))) == EINVAL  # 6 records expected
    g = s.adjoint_backward(np.zeros((6, 2, 3)))[0]
    assert float(g.abs().max()) == 0.0
