"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bar (FP64): the wet/dry mask is identical and eta, u, v agree within 1e-10
relative to the field's max magnitude; the formulation note makes bitwise
equality the expected outcome, which is also reported.  Friction uses
cbrt, whose last bit may differ between libm and the device, so it is
held to the 1e-10 bar only.
"""
import numpy as np
import pytest

from paper_1410_0753_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def clf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1410_0753_amd import clf as m
    m.load()
    return m


def _cmp_state(gpu, ora, tol=TOL, bitwise=False, what=""):
    e_g, u_g, v_g, w_g = (t.cpu().numpy() for t in gpu.state())
    e_o, u_o, v_o, w_o = ora.state()
    assert np.array_equal(w_g.astype(bool), w_o.astype(bool)), "%s: wet mask differs at %d nodes" % (
        what, int((w_g.astype(bool) != w_o.astype(bool)).sum()))
    for name, a, b in (("eta", e_g, e_o), ("u", u_g, u_o), ("v", v_g, v_o)):
        scale = max(np.abs(b).max(), 1e-300)
        err = np.abs(a - b).max() / scale
        assert err <= tol, "%s: %s rel err %.3e" % (what, name, err)
        if bitwise:
            assert np.array_equal(a, b), "%s: %s not bitwise (rel %.3e)" % (what, name, err)
    return True


def _pair(clf, case, oracle_mod, **kw):
    g = clf.Solver.from_case(case, **kw)
    o = oracle_mod.Oracle.from_case(case, **kw)
    return g, o


CASES = [
    # (label, generator) -- sizes span several 58-column strips and ragged tails
    ("random-land-130x75", lambda: synth.random_small(1, 130, 75, land=True)),
    ("random-wet-61x200", lambda: synth.random_small(2, 61, 200, land=False)),
    ("random-land-3x3", lambda: synth.random_small(3, 3, 3, land=True)),
    ("random-land-59x5", lambda: synth.random_small(4, 59, 5, land=True)),
    ("c1-small-120x90", lambda: synth.config1(nx=120, ny=90, steps=10)),
]


@pytest.mark.parametrize("label,gen", CASES, ids=[c[0] for c in CASES])
def test_step_parity(clf, oracle_mod, label, gen):
    case = gen()
    print("case", label, flush=True)
    g, o = _pair(clf, case, oracle_mod)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
    for k in range(3):
        g.step(7)
        o.step(7)
        _cmp_state(g, o, bitwise=True, what="%s after %d steps" % (label, 7 * (k + 1)))


@pytest.mark.parametrize("axis", [0, 1])
def test_single_sweep_parity(clf, oracle_mod, axis):
    case = synth.random_small(5, 140, 97, land=True)
    g, o = _pair(clf, case, oracle_mod)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 3.0, case.u0, case.v0)
    for _ in range(5):
        g.sweep(axis)
        o.sweep(axis)
    _cmp_state(g, o, bitwise=True, what="sweep %d" % axis)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_edge_interfaces(clf, oracle_mod, axis, prec):
    # A flow normal to every edge of a wet spherical basin with uneven
    # spacing: the wall interface of the first row or column is evaluated
    # from outside the grid (by the lane or pipeline row before it), so its
    # inverse spacing must be that of the edge and not a default.
    rng = np.random.default_rng(21)
    nx, ny = 131, 77
    x = 140.0 + np.cumsum(np.r_[0.0, 0.01 + 0.02 * rng.random(nx - 1)])
    y = 20.0 + np.cumsum(np.r_[0.0, 0.01 + 0.02 * rng.random(ny - 1)])
    d = synth.f32(1000.0 + 500.0 * rng.random((ny, nx)))
    eta = synth.f32(0.3 * rng.standard_normal((ny, nx)))
    u = synth.f32(np.where(np.arange(nx)[None, :] < nx // 2, -0.5, 0.5) * np.ones((ny, 1)))
    v = synth.f32(np.where(np.arange(ny)[:, None] < ny // 2, -0.4, 0.4) * np.ones((1, nx)))
    dt = 2.0
    p = clf.FP64 if prec == "fp64" else clf.FP32
    g = clf.Solver(x, y, d, dt, coord=synth.SPHERICAL, precision=p, ssl_alpha=0.0)
    o = oracle_mod.Oracle(x, y, d, dt, coord=synth.SPHERICAL, ssl_alpha=0.0)
    for obj in (g, o):
        obj.set_initial(eta, u, v)
        for _ in range(3):
            obj.sweep(axis)
    if prec == "fp64":
        _cmp_state(g, o, bitwise=True, what="edge interfaces, sweep %d" % axis)
    else:
        e_g, u_g, v_g, _ = (t.cpu().numpy() for t in g.state())
        e_o, u_o, v_o, _ = o.state()
        for name, a, b in (("eta", e_g, e_o), ("u", u_g, u_o), ("v", v_g, v_o)):
            err = np.abs(a - b).max() / np.abs(b).max()
            assert err < 1e-5, "%s rel err %.2e" % (name, err)


def test_raw_state_bitwise(clf, oracle_mod):
    case = synth.random_small(6, 100, 64, land=True)
    g, o = _pair(clf, case, oracle_mod)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(20)
    Hg, ug, vg = (t.cpu().numpy() for t in g.raw_state())
    Ho, uo, vo = o.raw_state()
    assert np.array_equal(Hg, Ho) and np.array_equal(ug, uo) and np.array_equal(vg, vo)


@pytest.mark.parametrize("opts", [
    dict(sweep_order=1),
    dict(solver=1),
    dict(itopo=0, dwall=5.0),
    dict(ssl_alpha=0.0),
    dict(ssl_alpha=2.5, h_min=0.05),
], ids=["alternate", "solver1", "wallmode", "no-ssl", "ssl2.5"])
def test_option_parity(clf, oracle_mod, opts):
    case = synth.random_small(7, 90, 70, land=True)
    g, o = _pair(clf, case, oracle_mod, **opts)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(15)
    _cmp_state(g, o, bitwise=True, what=str(opts))


@pytest.mark.parametrize("coord", [synth.CARTESIAN, synth.SPHERICAL], ids=["cartesian", "spherical"])
def test_friction_parity(clf, oracle_mod, coord):
    case = synth.random_small(8, 80, 60, land=True, coord=coord)
    g, o = _pair(clf, case, oracle_mod, manning_n2=0.0009)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(15)
    _cmp_state(g, o, tol=TOL, what="friction")


@pytest.mark.parametrize("opts", [
    dict(sweep_order=1),
    dict(solver=1),
    dict(itopo=0, dwall=5.0),
    dict(sweep_order=1, solver=1, itopo=0, dwall=5.0),
], ids=["alternate", "solver1", "wallmode", "all"])
@pytest.mark.parametrize("coord", [synth.CARTESIAN, synth.SPHERICAL], ids=["cartesian", "spherical"])
def test_friction_with_options(clf, oracle_mod, opts, coord):
    # friction selects its own kernel variants (the y update per node in
    # FP64, and the general variant with solver1 or wall mode)
    case = synth.random_small(16, 85, 64, land=True, coord=coord)
    g, o = _pair(clf, case, oracle_mod, manning_n2=0.0009, **opts)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0, case.u0, case.v0)
        obj.step(13)
    _cmp_state(g, o, tol=TOL, what="friction %s" % opts)


@pytest.mark.parametrize("shape", [(1, 150), (150, 1)], ids=["1d-x", "1d-y"])
def test_one_d_parity(clf, oracle_mod, shape):
    ny, nx = shape
    n = max(nx, ny)
    s = np.arange(n) * 10.0
    d = synth.f32((1000.0 - s) / 20.0)
    eta = synth.f32(0.8 * np.exp(-0.5 * ((np.arange(n) - 30) / 6.0) ** 2))
    d, eta = d.reshape(ny, nx), eta.reshape(ny, nx)
    x = s if nx > 1 else np.array([0.0])
    y = s if ny > 1 else np.array([0.0])
    dt = 0.4 * 10.0 / np.sqrt(9.81 * 50.0)
    g = clf.Solver(x, y, d, dt, h_min=0.01)
    o = oracle_mod.Oracle(x, y, d, dt, h_min=0.01)
    for obj in (g, o):
        obj.set_initial(eta)
    for _ in range(4):
        g.step(50)
        o.step(50)
        _cmp_state(g, o, bitwise=True, what="1-D %s" % (shape,))


def test_spherical_parity(clf, oracle_mod):
    case = synth.config2(steps=10, scale=12)
    g, o = _pair(clf, case, oracle_mod)
    for obj in (g, o):
        obj.set_initial(case.eta0)
        obj.step(12)
    _cmp_state(g, o, bitwise=True, what="spherical")


def test_deform_bottom_parity(clf, oracle_mod):
    case = synth.random_small(9, 70, 50, land=True)
    g, o = _pair(clf, case, oracle_mod)
    for obj in (g, o):
        obj.set_initial(case.eta0, None, None, deform_bottom=True)
    assert np.array_equal(g.depth().cpu().numpy(), o.depth())
    g.step(10)
    o.step(10)
    _cmp_state(g, o, bitwise=True, what="deformed bottom")


def test_sampling_parity(clf, oracle_mod):
    case = synth.config1(nx=120, ny=100, steps=10)
    g, o = _pair(clf, case, oracle_mod, gout=3, maxout=2)
    ix = np.array([3, 50, 100, 119, 60]); iy = np.array([5, 50, 20, 99, 0])
    xe = np.linspace(case.x[20] + 123.0, case.x[60] + 7.0, 17)
    ye = np.linspace(case.y[30] + 11.0, case.y[70] - 3.0, 13)
    for obj in (g, o):
        obj.set_initial(case.eta0 * 2.0)
        obj.set_gauges(ix, iy)
        obj.add_enclosed_grid(xe, ye)
        obj.step(10)
        obj.step(7)
    rg, tg = g.read_gauges()
    ro, to = o.read_gauges()
    assert rg.shape == ro.shape and np.array_equal(tg, to)
    assert np.array_equal(rg, ro)
    mg = [t.cpu().numpy() for t in g.read_maxwave()]
    mo = o.read_maxwave()
    assert np.array_equal(mg[0], mo[0]) and np.array_equal(mg[1], mo[1])
    for side in range(4):
        sg, stg = g.read_boundary_series(0, side)
        so, sto = o.read_boundary_series(0, side)
        assert sg.shape == so.shape and np.array_equal(stg, sto)
        assert np.array_equal(sg, so)


@pytest.mark.parametrize("n2", [0.0, 0.0009], ids=["plain", "friction"])
def test_forcing_parity(clf, oracle_mod, n2):
    case = synth.random_small(10, 64, 48, land=False)
    t = np.array([0.0, 3 * case.dt, 11 * case.dt])
    rng = np.random.default_rng(0)
    g = clf.Solver.from_case(case, forcing_capacity=8, manning_n2=n2)
    o = oracle_mod.Oracle.from_case(case, manning_n2=n2)
    for obj in (g, o):
        obj.set_initial(case.eta0)
    for side in range(4):
        np_ = case.ny if side < 2 else case.nx
        vals = synth.f32(0.05 * rng.standard_normal((len(t), 3, np_)))
        g.set_boundary_forcing(side, t, vals)
        o.set_boundary_forcing(side, t, vals)
    g.step(15)
    o.step(15)
    # friction uses cbrt, held to the 1e-10 bar only
    _cmp_state(g, o, bitwise=(n2 == 0.0), what="forcing")


def test_restart_parity(clf, oracle_mod):
    case = synth.random_small(11, 75, 66, land=True)
    a = clf.Solver.from_case(case)
    a.set_initial(case.eta0 * 2.0, case.u0, case.v0)
    a.step(12)
    h, u, v = a.raw_state()
    a.step(9)
    b = clf.Solver.from_case(case)
    b.set_raw_state(h, u, v, 12)
    b.step(9)
    for p, q in zip(a.raw_state(), b.raw_state()):
        assert bool((p == q).all())


def test_errors(clf):
    case = synth.random_small(12, 20, 20, land=True)
    with pytest.raises(clf.ClfError) as ei:
        clf.Solver.from_case(case.__class__(**{**case.__dict__, "dt": case.dt * 10}))
    assert ei.value.code == -2
    s = clf.Solver.from_case(case, max_gauges=2)
    with pytest.raises(clf.ClfError) as ei:
        s.set_gauges([0, 1, 2], [0, 1, 2])
    assert ei.value.code == -6
    with pytest.raises(clf.ClfError) as ei:
        s.set_gauges([0], [25])
    assert ei.value.code == -1
    with pytest.raises(clf.ClfError) as ei:
        s.set_boundary_forcing(0, [0.0], np.zeros((1, 3, 20)))
    assert ei.value.code == -6


def test_tiny_h_min_thin_film(clf, oracle_mod):
    # wet films of 1e-245 m put sqrt(g h) arguments below 2^-767, which only
    # the general kernel's square root rescales; an h_min below 1e-200 routes
    # the grid there, and the state stays bitwise equal to the oracle's
    n = 48
    x = np.arange(n) * 10.0
    d = np.full((n, n), 20.0)
    d[:, :8] = 1e-245 * (1.0 + np.arange(8))[None, :]
    ii = np.arange(n)
    eta = 0.3 * np.exp(-0.5 * (((ii[None, :] - 34) / 5.0) ** 2 + ((ii[:, None] - 24) / 5.0) ** 2))
    eta[:, :12] = 0.0
    dt = 0.4 * 10.0 / np.sqrt(9.81 * 20.0)
    g = clf.Solver(x, x, d, dt, ssl_alpha=0.0, h_min=1e-250)
    o = oracle_mod.Oracle(x, x, d, dt, ssl_alpha=0.0, h_min=1e-250)
    for obj in (g, o):
        obj.set_initial(eta)
    w = g.state()[3].cpu().numpy().astype(bool)
    assert w[:, :8].all()
    for k in range(3):
        g.step(20)
        o.step(20)
        _cmp_state(g, o, bitwise=True, what="thin film, %d steps" % (20 * (k + 1)))


def test_nonfinite_detected(clf, oracle_mod):
    # six times the Courant limit (allowed by raising cfl_limit) overflows
    # within a few steps; the device flag surfaces as CLF_ENONFINITE at sync
    n = 64
    d = np.full((n, n), 100.0)
    x = np.arange(n) * 100.0
    dt = 6.0 * 100.0 / np.sqrt(9.81 * 100.0)
    eta = 1e-3 * np.random.default_rng(1).standard_normal((n, n))
    o = oracle_mod.Oracle(x, x, d, dt, ssl_alpha=0.0, h_min=1e-3)
    o.set_initial(eta)
    o.step(5)
    assert not np.isfinite(o.raw_state()[0]).all()
    s = clf.Solver(x, x, d, dt, ssl_alpha=0.0, h_min=1e-3, cfl_limit=100.0)
    s.set_initial(eta)
    s.step(5)
    with pytest.raises(clf.ClfError) as ei:
        s.sync()
    assert ei.value.code == -4
