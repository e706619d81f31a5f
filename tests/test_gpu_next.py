"""GPU parity of the NEXT workloads: the 1-D graded-beach runup and the
nested-grid chain (parent series driving a finer child grid)."""
import math

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


def test_beach_runup_bitwise(clf, oracle_mod):
    from tests.golden import load
    gb = load("sloping_beach.txt")
    c = synth.beach_1d(H_over_d=gb["H_over_d"], cot_beta=gb["cot_beta"], steps=1200)
    g = clf.Solver.from_case(c, ssl_alpha=0.0, maxout=1)
    o = oracle_mod.Oracle.from_case(c, ssl_alpha=0.0, maxout=1)
    for obj in (g, o):
        obj.set_initial(c.eta0, c.u0, None)
        obj.step(c.steps)
    mg = g.read_maxwave()[0].cpu().numpy()
    mo = o.read_maxwave()[0]
    assert np.array_equal(mg, mo)
    for a, b in zip((t.cpu().numpy() for t in g.raw_state()), o.raw_state()):
        assert np.array_equal(a, b)
    land = c.depth[0] < 0
    law = gb["runup_law_coefficient"] * math.sqrt(gb["cot_beta"]) * gb["H_over_d"] ** 1.25
    assert abs(mg[0][land].max() / law - 1.0) <= 0.1


def test_nested_chain_bitwise(clf, oracle_mod):
    from tests.test_oracle_pins import nested_setup
    S = nested_setup()
    Np = 60
    res = {}
    for name, make in (("gpu", lambda *a, **k: clf.Solver(*a, forcing_capacity=Np + 2, **k)),
                       ("ora", lambda *a, **k: oracle_mod.Oracle(*a, **k))):
        par = make(S["xp"], S["yp"], S["dp"], S["dt_p"], ssl_alpha=0.0, bndout=1)
        par.set_initial(S["eta"])
        gid = par.add_enclosed_grid(S["xc"], S["yc"])
        par.step(Np)
        child = make(S["xc"], S["yc"], S["dc"], S["dt_p"] / 2, ssl_alpha=0.0)
        child.set_initial(None)
        series = []
        for side in range(4):
            vals, t = par.read_boundary_series(gid, side)
            series.append(vals)
            child.set_boundary_forcing(side, t, vals)
        child.step(2 * Np)
        st = child.raw_state()
        res[name] = ([np.asarray(s.cpu().numpy() if hasattr(s, "cpu") else s) for s in st], series)
    for a, b in zip(res["gpu"][1], res["ora"][1]):
        assert np.array_equal(a, b)
    for a, b in zip(res["gpu"][0], res["ora"][0]):
        assert np.array_equal(a, b)
