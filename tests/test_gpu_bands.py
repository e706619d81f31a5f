"""y-band decomposition of one grid on one device: every band holds 3 halo
rows beyond each inner edge and the halo rows are exchanged after each step
(the splitting into independent row and column problems, section Numerics).
The result must be bit for bit the whole-grid run's (state, wet mask and
maxwave), in FP64 and FP32, with the shoreline crossing band edges."""
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


def _equal(a, b, what):
    sa = [t.cpu().numpy() for t in a.state()] + [t.cpu().numpy() for t in a.read_maxwave()]
    sb = [t.cpu().numpy() for t in b.state()] + [t.cpu().numpy() for t in b.read_maxwave()]
    for name, x, y in zip(("eta", "u", "v", "wet", "eta_max", "speed_max"), sa, sb):
        assert np.array_equal(x, y), "%s: %s differs at %d nodes" % (what, name,
                                                                    int((x != y).sum()))


CASES = [
    ("c1-island-120x90", lambda: synth.config1(nx=120, ny=90, steps=10), {}),
    ("random-land-130x75", lambda: synth.random_small(1, 130, 75, land=True), {}),
    ("spherical-c2-scale8", lambda: synth.config2(steps=10, scale=8), {}),
    ("friction-130x75", lambda: synth.random_small(1, 130, 75, land=True),
     dict(manning_n2=0.0009)),
    ("open-edges-96x80", lambda: synth.random_small(6, 96, 80, land=False), dict(open_sides=15)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nbands", [2, 3, 7])
@pytest.mark.parametrize("label,gen,kw", CASES, ids=[c[0] for c in CASES])
def test_bands_equal_whole_grid(clf, label, gen, kw, nbands, prec):
    case = gen()
    p = clf.FP64 if prec == "fp64" else clf.FP32
    print("bands", label, nbands, prec, flush=True)
    whole = clf.Solver.from_case(case, precision=p, graph_steps=0, **kw)
    bands = clf.Bands.from_case(case, nbands, precision=p, **kw)
    for obj in (whole, bands):
        obj.set_initial(3.0 * case.eta0, case.u0, case.v0)
    for k in range(3):
        whole.step(11)
        bands.step(11)
        _equal(bands, whole, "%s %d bands %s after %d steps" % (label, nbands, prec, 11 * (k + 1)))


def test_bands_flooding_across_band_edges(clf):
    # runup floods initially dry nodes in the halo rows of every inner edge
    # of 7 bands (rows 11, 22, 33, 44, 55, 65 of 75): the exchanged rows carry
    # the flooding (b) and the caps (e) of the owning band
    case = synth.random_small(1, 130, 75, land=True)
    whole = clf.Solver.from_case(case, graph_steps=0)
    bands = clf.Bands.from_case(case, 7)
    for obj in (whole, bands):
        obj.set_initial(3.0 * case.eta0, case.u0, case.v0)
    dry0 = whole.state()[3].cpu().numpy() == 0
    for _ in range(33):
        whole.step(1)
        bands.step(1)
    _equal(bands, whole, "runup 33 steps")
    flooded = (whole.read_maxwave()[0].cpu().numpy() > 0) & dry0
    rows = set(np.nonzero(flooded.any(axis=1))[0].tolist())
    for edge in (11, 22, 33, 44, 55, 65):
        assert rows & set(range(edge - 3, edge + 3)), "no flooding next to band edge %d" % edge


def test_bands_deform_bottom_and_queries(clf):
    case = synth.random_small(4, 90, 64, land=True)
    whole = clf.Solver.from_case(case, graph_steps=0)
    bands = clf.Bands.from_case(case, 4)
    for obj in (whole, bands):
        obj.set_initial(case.eta0, None, None, deform_bottom=True)
        obj.step(20)
    _equal(bands, whole, "deform_bottom")
    assert bands.query(clf.Q_STEP) == 20
    assert abs(bands.query(clf.Q_MAX_CFL) - whole.query(clf.Q_MAX_CFL)) == 0.0
    assert bands.query(clf.Q_SSL_PASSES) == whole.query(clf.Q_SSL_PASSES)


def test_bands_reject_bad_layouts(clf):
    case = synth.random_small(4, 90, 20, land=True)
    with pytest.raises(clf.ClfError):
        clf.Bands.from_case(case, 7)          # 20 rows in 7 bands: fewer than 3 rows each
    with pytest.raises(clf.ClfError):
        clf.Bands.from_case(case, 2, sweep_order=1)
    line = synth.random_small(4, 90, 1, land=False)
    with pytest.raises(clf.ClfError):
        clf.Bands.from_case(line, 1)
