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


@pytest.mark.parametrize("segment", [8, 9, 10, 11])
def test_runup_across_segment_edges(clf, oracle_mod, segment):
    # A wave runs up a beach that slopes along y. The shoreline advances one
    # row at a time from row 20 to row 30, so nodes flood in step (b) of the
    # y-sweep on the first and last rows of segments (both march
    # directions). Their limiter (e) reads the rows just outside the segment,
    # whose update the FP64 kernel runs only in that case.
    nx, ny = 70, 48
    x = np.arange(nx) * 100.0
    y = np.arange(ny) * 100.0
    j = np.arange(ny)[:, None] * np.ones((1, nx))
    d = 6.0 - 0.3 * j
    eta = 1.5 * np.exp(-0.5 * ((j - 8) / 3.0) ** 2)
    v = np.sqrt(9.81 / np.maximum(d, 1.0)) * eta
    u = np.zeros_like(eta)
    dt = 0.4 * 100.0 / np.sqrt(9.81 * 8.0)
    print("segment", segment, flush=True)
    g = clf.Solver(x, y, d, dt, ssl_alpha=0.0, h_min=0.01, segment=segment)
    o = oracle_mod.Oracle(x, y, d, dt, ssl_alpha=0.0, h_min=0.01)
    assert g.query(clf.Q_SEGMENT) == segment
    for obj in (g, o):
        obj.set_initial(eta, u, v)
    for k in range(10):
        g.step(10)
        o.step(10)
        _bitwise(g, o, "runup, segment %d, %d steps" % (segment, 10 * (k + 1)))
    # the front crossed the edge rows of every segment length above
    assert np.where(o.state()[3].astype(bool).any(axis=1))[0].max() >= 29


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
