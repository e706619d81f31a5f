"""The FP32 march staging its rows in LDS (direct global-to-LDS loads, taken
by FP32 grids whose fields exceed the last-level cache) against the same
kernel with rows prefetched into registers: the same bits for state, wet
mask, maxwave and gauge records, across segment lengths, both sweep
orders, flooding, friction, and the variants that stage in registers
only.  CLF_LDS_ROWS=1 or 0 forces either mode on small grids."""
import os

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


def _make(clf, case, mode, **kw):
    old = os.environ.get("CLF_LDS_ROWS")
    os.environ["CLF_LDS_ROWS"] = mode
    try:
        return clf.Solver.from_case(case, precision=clf.FP32, **kw)
    finally:
        if old is None:
            del os.environ["CLF_LDS_ROWS"]
        else:
            os.environ["CLF_LDS_ROWS"] = old


def _fields(s):
    return [t.cpu().numpy() for t in s.state()] + [t.cpu().numpy() for t in s.read_maxwave()]


def _same(a, b, what):
    for name, x, y in zip(("eta", "u", "v", "wet", "eta_max", "speed_max"), _fields(a), _fields(b)):
        assert np.array_equal(x, y), "%s: %s differs at %d nodes" % (what, name, int((x != y).sum()))


@pytest.mark.parametrize("fric", [0.0, 0.0009], ids=["fast", "friction"])
@pytest.mark.parametrize("order", [0, 1], ids=["xy", "alternate"])
@pytest.mark.parametrize("segment", [8, 13, 45, 0])
def test_lds_rows_equal_register_rows(clf, fric, order, segment):
    # runup onto land (flooding in both sweeps), spherical source terms on
    case = synth.random_small(31, 150, 77, land=True, coord=synth.SPHERICAL)
    kw = dict(sweep_order=order, manning_n2=fric, graph_steps=0)
    if segment:
        kw["segment"] = segment
    print("lds rows", fric, order, segment, flush=True)
    a = _make(clf, case, "1", **kw)
    b = _make(clf, case, "0", **kw)
    assert a.query(clf.Q_LDS_ROWS) == 1 and b.query(clf.Q_LDS_ROWS) == 0
    assert a.query(clf.Q_SEGMENT) == b.query(clf.Q_SEGMENT)
    gx = np.array([3, 40, 77, 149, 0]); gy = np.array([0, 20, 76, 38, 50])
    for s in (a, b):
        s.set_gauges(gx, gy)
        s.set_initial(3.0 * case.eta0, case.u0, case.v0)
    dry0 = a.state()[3].cpu().numpy() == 0
    for k in range(3):
        a.step(7)
        b.step(7)
        _same(a, b, "order %d segment %d after %d steps" % (order, segment, 7 * (k + 1)))
    ra, _ = a.read_gauges()
    rb, _ = b.read_gauges()
    assert np.array_equal(ra, rb)
    # the case floods: initially dry nodes reached the maxwave
    assert ((a.read_maxwave()[0].cpu().numpy() > 0) & dry0).any()


def test_lds_rows_other_variants_and_fp64(clf):
    # forced on, the variants that stage in registers only (wall mode,
    # FP64) still run and report it
    case = synth.random_small(32, 90, 60, land=True)
    a = _make(clf, case, "1", itopo=0, dwall=5.0)
    b = _make(clf, case, "0", itopo=0, dwall=5.0)
    for s in (a, b):
        s.set_initial(2.0 * case.eta0, case.u0, case.v0)
        s.step(15)
    _same(a, b, "wall mode")
    old = os.environ.get("CLF_LDS_ROWS")
    os.environ["CLF_LDS_ROWS"] = "1"
    try:
        d = clf.Solver.from_case(case)
    finally:
        if old is None:
            del os.environ["CLF_LDS_ROWS"]
        else:
            os.environ["CLF_LDS_ROWS"] = old
    assert d.query(clf.Q_LDS_ROWS) == 0


def test_lds_rows_by_footprint(clf):
    # 9 FP32 arrays of the grid against 256 MiB: 2400 x 1800 stays in
    # registers, 3000 x 2600 stages in LDS
    assert "CLF_LDS_ROWS" not in os.environ
    for nx, ny, want in ((2400, 1800, 0), (3000, 2600, 1)):
        x = np.arange(nx) * 100.0
        y = np.arange(ny) * 100.0
        depth = np.full((ny, nx), 50.0)
        z = np.zeros((ny, nx))
        case = synth.Case("flat", synth.CARTESIAN, x, y, depth, z, z, z, 1.0, 1)
        s = clf.Solver.from_case(case, precision=clf.FP32, graph_steps=0)
        assert s.query(clf.Q_LDS_ROWS) == want, (nx, ny)
        s.set_initial(None)
        s.step(2)
        e = s.state()[0].cpu().numpy()
        assert np.array_equal(e, np.zeros_like(e))   # a lake at rest stays at rest
        del s


class _Env:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        self.old = os.environ.get("CLF_LDS_ROWS")
        os.environ["CLF_LDS_ROWS"] = self.value

    def __exit__(self, *a):
        if self.old is None:
            del os.environ["CLF_LDS_ROWS"]
        else:
            os.environ["CLF_LDS_ROWS"] = self.old


def test_lds_rows_in_ensembles_and_bands(clf):
    # members of uneven size (strips not a multiple of four, ragged last
    # segments) in one launch, and y-bands with their halo exchange
    cases = [synth.random_small(40 + k, 70 + 23 * k, 45 + 11 * k, land=True) for k in range(3)]
    out = {}
    for mode in ("1", "0"):
        with _Env(mode):
            ens = clf.Ensemble(cases, precision=clf.FP32, graph_steps=0)
            assert ens.query(clf.Q_LDS_ROWS) == int(mode)
            for i, c in enumerate(cases):
                ens.set_initial(i, 3.0 * c.eta0, c.u0, c.v0)
            ens.step(13)
            st = [[t.cpu().numpy() for t in ens.state(i)] for i in range(len(cases))]
            bands = clf.Bands.from_case(cases[2], 3, precision=clf.FP32)
            assert bands.query(clf.Q_LDS_ROWS) == int(mode)
            bands.set_initial(3.0 * cases[2].eta0, cases[2].u0, cases[2].v0)
            bands.step(13)
            out[mode] = (st, _fields(bands))
            del ens, bands
    for i in range(len(cases)):
        for a, b in zip(out["1"][0][i], out["0"][0][i]):
            assert np.array_equal(a, b), "ensemble member %d" % i
    for a, b in zip(out["1"][1], out["0"][1]):
        assert np.array_equal(a, b), "bands"


def test_lds_rows_in_the_static_entry_point(clf):
    import torch
    case = synth.random_small(44, 97, 52, land=True, coord=synth.SPHERICAL)
    ctx = clf.Solver.from_case(case, precision=clf.FP32)
    ctx.set_initial(3.0 * case.eta0, case.u0, case.v0)
    e, u, v, w = (t.cpu().numpy() for t in ctx.state())
    d = ctx.depth().cpu().numpy()
    eta = np.where(w.astype(bool), e, -d)
    res = {}
    for mode in ("1", "0"):
        D, H, U, V = (torch.tensor(a.astype(np.float32), device="cuda") for a in (d, eta, u, v))
        b = [torch.empty_like(H) for _ in range(3)]
        em, sm = torch.zeros_like(H), torch.zeros_like(H)
        with _Env(mode):
            which, bad = clf.step_static(case.x, case.y, case.coord, D, (H, U, V), tuple(b), 9,
                                         case.dt, eta_max=em, speed2_max=sm,
                                         precision=clf.FP32, h_min=case.h_min)
        assert not bad
        fin = (H, U, V) if which == 0 else tuple(b)
        res[mode] = [t.cpu().numpy() for t in fin] + [em.cpu().numpy(), sm.cpu().numpy()]
    for a, b in zip(res["1"], res["0"]):
        assert np.array_equal(a, b)
