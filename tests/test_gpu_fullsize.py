"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (autotuned segment, gauges, maxwave every step), plus randomised tiny
grids (edge cases: 3-node lines, ragged strips and segments)."""
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


def test_full_size_2400x1800_fp64_bitwise(clf, oracle_mod):
    case = synth.config2(steps=20)
    print("full-size 2400x1800 FP64, 20 steps", flush=True)
    g = clf.Solver.from_case(case, gout=10, maxout=1, autotune=1)
    o = oracle_mod.Oracle.from_case(case, gout=10, maxout=1)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
        obj.step(20)
    for a, b in zip((t.cpu().numpy() for t in g.raw_state()), o.raw_state()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.read_gauges()[0], o.read_gauges()[0])
    mg = [t.cpu().numpy() for t in g.read_maxwave()]
    mo = o.read_maxwave()
    assert np.array_equal(mg[0], mo[0]) and np.array_equal(mg[1], mo[1])


def test_reduced_2400x1800_flooding_1500_steps_bitwise(clf, oracle_mod):
    # the 2400x1800 workload at half resolution (1200x900, 2 arc-minutes),
    # 1500 steps: the dipole's waves reach the coast and flood initially dry
    # nodes of the land band; state, gauges and maxwave bit for bit
    case = synth.config2(steps=1500, scale=2)
    print("reduced 1200x900 FP64, 1500 steps", flush=True)
    g = clf.Solver.from_case(case, gout=10, maxout=1, autotune=1)
    o = oracle_mod.Oracle.from_case(case, gout=10, maxout=1)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
    dry0 = o.state()[3] == 0
    for k in range(3):
        g.step(500)
        o.step(500)
        print("  step", 500 * (k + 1), flush=True)
    for a, b in zip((t.cpu().numpy() for t in g.raw_state()), o.raw_state()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.read_gauges()[0], o.read_gauges()[0])
    mg = [t.cpu().numpy() for t in g.read_maxwave()]
    mo = o.read_maxwave()
    assert np.array_equal(mg[0], mo[0]) and np.array_equal(mg[1], mo[1])
    flooded = dry0 & (mo[0] > 0)
    print("  initially dry nodes ever wet:", int(flooded.sum()), flush=True)
    assert flooded.sum() >= 20


def test_reduced_8000x6000_runup_floods_plane_beaches(clf, oracle_mod):
    # the 8000x6000 runup workload at quarter resolution (2000x1500, 2 arc-
    # minutes) with a 6 m dipole: within 800 steps the waves flood more than
    # a hundred initially dry nodes.  Friction (explicit form) goes through
    # cbrt in the oracle, so the bar is the same wet mask and 1e-10 of each
    # field's magnitude, for the state, the gauges, maxwave and the boundary
    # series of the 4 enclosed grids
    case = synth.config5(steps=800, scale=4, amp=6.0)
    print("reduced 2000x1500 runup FP64, 800 steps", flush=True)
    kw = dict(gout=10, maxout=1, bndout=5, max_enclosed=4)
    g = clf.Solver.from_case(case, autotune=1, series_capacity=200, **kw)
    o = oracle_mod.Oracle.from_case(case, **kw)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
        for ex, ey in case.enclosed:
            obj.add_enclosed_grid(ex, ey)
    dry0 = o.state()[3] == 0
    for k in range(4):
        g.step(200)
        o.step(200)
        print("  step", 200 * (k + 1), flush=True)

    def close(a, b, what):
        assert np.abs(a - b).max() <= 1e-10 * max(np.abs(b).max(), 1e-300), what

    eg, ug, vg, wg = (t.cpu().numpy() for t in g.state())
    eo, uo, vo, wo = o.state()
    assert np.array_equal(wg, wo), "wet mask differs"
    for a, b, n in ((eg, eo, "eta"), (ug, uo, "u"), (vg, vo, "v")):
        close(a, b, n)
    close(g.read_gauges()[0], o.read_gauges()[0], "gauges")
    mg = [t.cpu().numpy() for t in g.read_maxwave()]
    mo = o.read_maxwave()
    close(mg[0], mo[0], "eta max")
    close(mg[1], mo[1], "speed max")
    for gid in range(4):
        for side in range(4):
            close(g.read_boundary_series(gid, side)[0], o.read_boundary_series(gid, side)[0],
                  "series %d/%d" % (gid, side))
    flooded = dry0 & (mo[0] > 0)
    print("  initially dry nodes ever wet:", int(flooded.sum()), flush=True)
    assert np.array_equal(flooded, dry0 & (mg[0] > 0))
    assert flooded.sum() >= 50


def test_full_size_2400x1800_fp64_long_bitwise(clf, oracle_mod):
    # 2000 steps: the waves reach the coast after about 1000, and a few
    # hundred initially dry nodes flood and dry again; state, gauges and
    # maxwave bit for bit
    case = synth.config2(steps=2000)
    print("full-size 2400x1800 FP64, 2000 steps", flush=True)
    g = clf.Solver.from_case(case, gout=10, maxout=1, autotune=1)
    o = oracle_mod.Oracle.from_case(case, gout=10, maxout=1)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
    for k in range(4):
        g.step(500)
        o.step(500)
        print("  step", 500 * (k + 1), flush=True)
    for a, b in zip((t.cpu().numpy() for t in g.raw_state()), o.raw_state()):
        assert np.array_equal(a, b)
    assert np.array_equal(g.read_gauges()[0], o.read_gauges()[0])
    mg = [t.cpu().numpy() for t in g.read_maxwave()]
    mo = o.read_maxwave()
    assert np.array_equal(mg[0], mo[0]) and np.array_equal(mg[1], mo[1])
    # nodes dry at the start that were wet at some step (maxwave is kept
    # on wet nodes only), so the run did exercise inundation
    ever = (case.depth <= 0) & ((mg[0] != 0) | (mg[1] != 0))
    print("  initially dry nodes ever wet:", int(ever.sum()), flush=True)
    assert ever.sum() > 0


def test_full_size_8000x6000_fp32_whole_grid(clf, oracle_mod):
    # FP32 on the large grid: error against the FP64 oracle on every node
    # (eta relative to the amplitude, u and v relative to the largest speed),
    # and the same wet set
    case = synth.config5(steps=4)
    print("full-size 8000x6000 FP32, 4 steps", flush=True)
    g = clf.Solver.from_case(case, precision=clf.FP32, autotune=1)
    g.set_initial(case.eta0)
    g.step(4)
    eg, ug, vg, wg = (t.cpu().numpy() for t in g.state())
    del g
    o = oracle_mod.Oracle.from_case(case)
    o.set_initial(case.eta0)
    o.step(4)
    eo, uo, vo, wo = o.state()
    amp = np.abs(eo).max()
    spd = max(np.abs(uo).max(), np.abs(vo).max())
    err = np.abs(eg - eo).max() / amp
    erru = max(np.abs(ug - uo).max(), np.abs(vg - vo).max()) / spd
    print("max eta err %.3e, max u/v err %.3e" % (err, erru), flush=True)
    assert np.array_equal(wg.astype(bool), wo.astype(bool))
    assert err <= 1e-4 and erru <= 1e-4


def test_full_size_8000x6000_fp32_against_fp64_200_steps(clf):
    # 200 steps of the benchmark configuration (gauges, enclosed-grid series,
    # maxwave every step) in FP32 against the FP64 path, which equals the
    # oracle bit for bit in the parity tests: state, wet set and maxwave
    case = synth.config5(steps=200)
    out = {}
    for prec in (clf.FP64, clf.FP32):
        print("full-size 8000x6000", "fp32" if prec == clf.FP32 else "fp64", "200 steps", flush=True)
        g = clf.Solver.from_case(
            case, precision=prec, autotune=1, maxout=1, gout=10, gauge_capacity=40, bndout=1,
            max_enclosed=len(case.enclosed),
            max_enclosed_points=sum(2 * (len(x) + len(y)) for x, y in case.enclosed),
            series_capacity=210)
        g.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
        for ex, ey in case.enclosed:
            g.add_enclosed_grid(ex, ey)
        g.set_initial(case.eta0)
        g.step(200)
        out[prec] = ([t.cpu().numpy() for t in g.state()] + [t.cpu().numpy() for t in g.read_maxwave()]
                     + [g.read_gauges()[0], g.read_boundary_series(0, 0)[0]])
        del g
    e64, u64, v64, w64, m64, s64, g64, b64 = out[clf.FP64]
    e32, u32, v32, w32, m32, s32, g32, b32 = out[clf.FP32]
    assert g64.shape == g32.shape and b64.shape == b32.shape
    amp = np.abs(e64).max()
    spd = max(np.abs(u64).max(), np.abs(v64).max())
    err = np.abs(e32 - e64).max() / amp
    erru = max(np.abs(u32 - u64).max(), np.abs(v32 - v64).max()) / spd
    errm = np.abs(m32 - m64).max() / np.abs(m64).max()
    errs = np.abs(s32 - s64).max() / np.abs(s64).max()
    flips = (w32.astype(bool) != w64.astype(bool)).mean()
    print("eta %.3e u/v %.3e eta_max %.3e speed_max %.3e flips %.3e" % (err, erru, errm, errs, flips),
          flush=True)
    assert err <= 1e-4 and erru <= 1e-4 and errm <= 1e-4 and errs <= 1e-4
    assert flips <= 1e-6
    # gauge and series records hold eta, u and v (at 200 steps the waves
    # have not reached most of them): within the same bound of the wave's
    # amplitude and largest speed
    for r32, r64 in ((g32, g64), (b32, b64)):
        assert np.abs(r32 - r64).max() <= 1e-4 * max(amp, spd)


@pytest.mark.parametrize("seed", range(12))
def test_random_tiny_grids_bitwise(clf, oracle_mod, seed):
    rng = np.random.default_rng(1000 + seed)
    nx = int(rng.integers(3, 140))
    ny = int(rng.integers(3, 90))
    land = bool(rng.integers(0, 2))
    case = synth.random_small(seed + 100, nx, ny, land=land, amp=float(rng.uniform(0.05, 1.5)))
    seg = int(rng.choice([8, 12, 16, 32]))
    print("seed", seed, nx, ny, land, seg, flush=True)
    nsteps = int(rng.integers(1, 12))
    g = clf.Solver.from_case(case, segment=seg)
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.step(nsteps)
    for a, b in zip((t.cpu().numpy() for t in g.raw_state()), o.raw_state()):
        assert np.array_equal(a, b)


def test_zero_steps_and_errors(clf):
    case = synth.random_small(3, 30, 20)
    g = clf.Solver.from_case(case)
    g.set_initial(case.eta0)
    h0 = g.raw_state()[0].cpu().numpy()
    g.step(0)
    assert np.array_equal(g.raw_state()[0].cpu().numpy(), h0)
    with pytest.raises(clf.ClfError):
        g.step(-1)
    with pytest.raises(clf.ClfError):
        clf.Solver.from_case(case, segment=3)


@pytest.mark.parametrize("wl", ["2400x1800", "8000x6000"])
def test_full_length_runs_stay_finite(clf, wl):
    # the configured run lengths of the two spherical workloads (10000 and
    # 20000 steps) stay finite with bounded speeds: the beach between land
    # and shelf, and friction on the runup grid
    import torch
    case = synth.config2(steps=10000) if wl == "2400x1800" else synth.config5(steps=20000)
    precs = [clf.FP64, clf.FP32] if wl == "2400x1800" else [clf.FP32]
    for prec in precs:
        print("full length", wl, "fp32" if prec == clf.FP32 else "fp64", case.steps, flush=True)
        g = clf.Solver.from_case(case, precision=prec, maxout=1, autotune=1)
        g.set_initial(case.eta0, case.u0, case.v0)
        g.step(case.steps)
        g.sync()
        e, u, v, _ = g.state()
        smax = float(torch.sqrt(u * u + v * v).max())
        emax = float(e.abs().max())
        print("  max speed %.3f max |eta| %.3f" % (smax, emax), flush=True)
        assert smax < 50.0 and emax < 50.0
        del g


def test_full_size_8000x6000_fp64_with_friction(clf, oracle_mod):
    # the FP64 runup grid as bench.py runs it (friction, autotuned segment,
    # gauges, maxwave) against the oracle: friction is held to 1e-10
    case = synth.config5(steps=3)
    print("full-size 8000x6000 FP64, 3 steps", flush=True)
    g = clf.Solver.from_case(case, gout=10, maxout=1, autotune=1)
    g.set_initial(case.eta0, case.u0, case.v0)
    g.step(3)
    hg, ug, vg = (t.cpu().numpy() for t in g.raw_state())
    del g
    o = oracle_mod.Oracle.from_case(case, gout=10, maxout=1)
    o.set_initial(case.eta0, case.u0, case.v0)
    o.step(3)
    ho, uo, vo = o.raw_state()
    for a, b, name in ((hg, ho, "h"), (ug, uo, "u"), (vg, vo, "v")):
        scale = max(np.abs(b).max(), 1e-300)
        err = np.abs(a - b).max() / scale
        print(name, "max rel", err)
        assert err <= 1e-10
    assert np.array_equal(hg > case.h_min, ho > case.h_min)


def test_full_size_ensemble_64_members(clf, oracle_mod):
    # the 64-member FP32 ensemble in bench.py's launch configuration: every
    # member equals its single-grid run bit for bit; three members of the
    # FP64 ensemble equal the oracle bit for bit
    cases = synth.config3(n=64, steps=12)
    print("full-size ensemble, 64 members, 12 steps", flush=True)
    ens = clf.Ensemble(cases, precision=clf.FP32, maxout=1, autotune=1)
    for i, c in enumerate(cases):
        ens.set_initial(i, c.eta0, c.u0, c.v0)
    ens.step(12)
    for i, c in enumerate(cases):
        s = clf.Solver.from_case(c, precision=clf.FP32, maxout=1)
        s.set_initial(c.eta0, c.u0, c.v0)
        s.step(12)
        for a, b in zip(ens.state(i), s.state()):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()), "member %d" % i
        del s
    del ens
    e64 = clf.Ensemble(cases, precision=clf.FP64, maxout=1, autotune=1)
    for i, c in enumerate(cases):
        e64.set_initial(i, c.eta0, c.u0, c.v0)
    e64.step(12)
    for i in (0, 31, 63):
        o = oracle_mod.Oracle.from_case(cases[i], maxout=1)
        o.set_initial(cases[i].eta0, cases[i].u0, cases[i].v0)
        o.step(12)
        eo, uo, vo, wo = o.state()
        eg, ug, vg, wg = (t.cpu().numpy() for t in e64.state(i))
        assert np.array_equal(eg, eo) and np.array_equal(ug, uo) and np.array_equal(vg, vo)
        assert np.array_equal(wg, wo)
