"""The step kernel's 64-bit-address variant (taken by grids whose field
arrays exceed 4 GiB), forced on small grids by CLF_WIDE_OFFSETS=1: FP64
results bitwise equal to the oracle across the options it carries, FP32
close to it, ensemble members equal to their single-grid runs."""
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


@pytest.fixture
def wide():
    old = os.environ.get("CLF_WIDE_OFFSETS")
    os.environ["CLF_WIDE_OFFSETS"] = "1"
    yield
    if old is None:
        del os.environ["CLF_WIDE_OFFSETS"]
    else:
        os.environ["CLF_WIDE_OFFSETS"] = old


def _bitwise(g, o, what):
    e_g, u_g, v_g, w_g = (t.cpu().numpy() for t in g.state())
    e_o, u_o, v_o, w_o = o.state()
    assert np.array_equal(w_g.astype(bool), w_o.astype(bool)), what + ": wet mask"
    for name, a, b in (("eta", e_g, e_o), ("u", u_g, u_o), ("v", v_g, v_o)):
        assert np.array_equal(a, b), "%s: %s max diff %.3e" % (what, name, np.abs(a - b).max())


@pytest.mark.parametrize("opts", [dict(), dict(sweep_order=1), dict(solver=1),
                                  dict(itopo=0, dwall=5.0)],
                         ids=["xy", "alternate", "solver1", "wallmode"])
@pytest.mark.parametrize("coord", [synth.CARTESIAN, synth.SPHERICAL], ids=["cartesian", "spherical"])
def test_wide_parity(clf, oracle_mod, wide, opts, coord):
    case = synth.random_small(17, 123, 58, land=True, coord=coord)
    g = clf.Solver.from_case(case, **opts)
    assert g.query(clf.Q_WIDE) == 1
    o = oracle_mod.Oracle.from_case(case, **opts)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(11)
    _bitwise(g, o, "wide %s" % opts)


def test_wide_friction_and_sampling(clf, oracle_mod, wide):
    case = synth.config1(nx=120, ny=100, steps=10)
    g = clf.Solver.from_case(case, manning_n2=0.0009, gout=3, maxout=2)
    o = oracle_mod.Oracle.from_case(case, manning_n2=0.0009, gout=3, maxout=2)
    ix = np.array([3, 50, 100, 119]); iy = np.array([5, 50, 20, 99])
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0)
        obj.set_gauges(ix, iy)
        obj.step(12)
    e_g = g.state()[0].cpu().numpy()
    e_o = o.state()[0]
    assert np.abs(e_g - e_o).max() <= 1e-10 * np.abs(e_o).max()
    rg, _ = g.read_gauges()
    ro, _ = o.read_gauges()
    assert np.abs(rg - ro).max() <= 1e-10 * max(np.abs(ro).max(), 1e-300)
    mg = g.read_maxwave()[0].cpu().numpy()
    assert np.abs(mg - o.read_maxwave()[0]).max() <= 1e-10 * max(np.abs(mg).max(), 1e-300)


def test_wide_sweeps_and_one_d(clf, oracle_mod, wide):
    case = synth.random_small(18, 140, 97, land=True)
    g = clf.Solver.from_case(case)
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 3.0, case.u0, case.v0)
        for axis in (0, 1, 1, 0):
            obj.sweep(axis)
    _bitwise(g, o, "wide sweeps")
    n = 150
    s = np.arange(n) * 10.0
    d = synth.f32((1000.0 - s) / 20.0).reshape(1, n)
    eta = synth.f32(0.8 * np.exp(-0.5 * ((np.arange(n) - 30) / 6.0) ** 2)).reshape(1, n)
    dt = 0.4 * 10.0 / np.sqrt(9.81 * 50.0)
    g = clf.Solver(s, np.array([0.0]), d, dt, h_min=0.01)
    o = oracle_mod.Oracle(s, np.array([0.0]), d, dt, h_min=0.01)
    for obj in (g, o):
        obj.set_initial(eta)
        obj.step(120)
    _bitwise(g, o, "wide 1-D")


def test_wide_fp32_and_ensemble(clf, oracle_mod, wide):
    case = synth.random_small(19, 90, 70, land=True)
    g = clf.Solver.from_case(case, precision=clf.FP32)
    assert g.query(clf.Q_WIDE) == 1
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(2.0 * case.eta0, case.u0, case.v0)
        obj.step(20)
    e_g = g.state()[0].cpu().numpy()
    e_o = o.state()[0]
    assert np.abs(e_g - e_o).max() <= 2e-3 * np.abs(e_o).max()
    cases = [synth.random_small(60 + k, 50 + 17 * k, 40 + 7 * k, land=True) for k in range(3)]
    ref = []
    for c in cases:
        s = clf.Solver.from_case(c, graph_steps=0)
        s.set_initial(c.eta0, c.u0, c.v0)
        s.step(7)
        ref.append([t.cpu().numpy() for t in s.state()])
    ens = clf.Ensemble(cases, graph_steps=4)
    assert ens.query(clf.Q_WIDE) == 1
    for i, c in enumerate(cases):
        ens.set_initial(i, c.eta0, c.u0, c.v0)
    ens.step(7)
    for i in range(len(cases)):
        for a, b in zip((t.cpu().numpy() for t in ens.state(i)), ref[i]):
            assert np.array_equal(a, b), "member %d" % i


def test_wide_adjoint_equals_narrow(clf):
    # the adjoint's recomputed sweeps run the same arithmetic either way
    c = synth.random_small(61, 70, 52, land=True, amp=0.3)
    gx = np.array([5, 30, 60, 44]); gy = np.array([10, 25, 40, 7])
    nsteps = 30
    obs = 0.05 * np.random.default_rng(4).standard_normal((nsteps // 2 + 1, len(gx)))
    grads = []
    for flag in ("0", "1"):
        os.environ["CLF_WIDE_OFFSETS"] = flag
        try:
            s = clf.Solver.from_case(c, gout=2)
            assert s.query(clf.Q_WIDE) == int(flag)
            s.set_gauges(gx, gy)
            s.set_initial(c.eta0)
            s.adjoint_forward(nsteps, 0)
            rec, _ = s.read_gauges()
            adj = np.zeros_like(rec)
            adj[:, :, 0] = rec[:, :, 0] - obs
            grads.append(s.adjoint_backward(adj)[0].cpu().numpy())
        finally:
            del os.environ["CLF_WIDE_OFFSETS"]
    assert np.array_equal(grads[0], grads[1])


def test_narrow_by_default(clf):
    assert "CLF_WIDE_OFFSETS" not in os.environ or os.environ["CLF_WIDE_OFFSETS"] != "1"
    case = synth.random_small(20, 40, 30, land=True)
    g = clf.Solver.from_case(case)
    assert g.query(clf.Q_WIDE) == 0
