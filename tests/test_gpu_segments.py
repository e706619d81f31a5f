"""FP64 parity of the march kernel under forced tile shapes: the shortest
segments allowed (8 rows) and odd lengths, so that many segments start
inside the grid (at a segment start the update of the rows above it is
skipped and only the interface below the row above it is carried), one
segment spanning the grid, persistent launches, and grid widths at and
around multiples of the 58 output columns of a strip.  Each case is
bitwise against the oracle."""
import numpy as np
import pytest

from paper_1410_0753_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0753_amd import clf as m
    m.load()
    return m


def _bitwise(g, o, what):
    e_g, u_g, v_g, w_g = (t.cpu().numpy() for t in g.state())
    e_o, u_o, v_o, w_o = o.state()
    assert np.array_equal(w_g.astype(bool), w_o.astype(bool)), what + ": wet mask"
    for name, a, b in (("eta", e_g, e_o), ("u", u_g, u_o), ("v", v_g, v_o)):
        assert np.array_equal(a, b), "%s: %s max diff %.3e" % (what, name, np.abs(a - b).max())


@pytest.mark.parametrize("order", [0, 1], ids=["xy", "alternate"])
@pytest.mark.parametrize("segment", [8, 9, 11, 13, 45, 64])
def test_short_segments(clf, oracle_mod, segment, order):
    case = synth.random_small(13, 130, 45, land=True)
    print("segment", segment, "order", order, flush=True)
    g = clf.Solver.from_case(case, segment=segment, sweep_order=order)
    o = oracle_mod.Oracle.from_case(case, sweep_order=order)
    assert g.query(clf.Q_SEGMENT) == segment
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
    for k in range(3):
        g.step(3)
        o.step(3)
        _bitwise(g, o, "segment %d, %d steps" % (segment, 3 * (k + 1)))


@pytest.mark.parametrize("nx", [57, 58, 59, 116, 117, 175])
def test_strip_widths(clf, oracle_mod, nx):
    case = synth.random_small(14, nx, 23, land=True)
    print("nx", nx, flush=True)
    g = clf.Solver.from_case(case)
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(8)
    _bitwise(g, o, "nx %d" % nx)


@pytest.mark.parametrize("blocks", [8, 16])
def test_persistent_short_segments(clf, oracle_mod, blocks):
    # a few workgroups walk the whole tile list of 8-row segments
    case = synth.random_small(15, 100, 40, land=True)
    g = clf.Solver.from_case(case, segment=8, persistent_blocks=blocks)
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(6)
    _bitwise(g, o, "persistent %d" % blocks)
