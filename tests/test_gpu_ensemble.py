"""Batched ensemble: every member equals its single-grid run bit for bit,
with and without hipGraph replays and persistent launches; graph replays are
interleaved with eager work and synchronisation and each one is checked."""
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


def members():
    return [synth.config3_member(s, steps=10, size_scale=0.08) for s in range(5)] + \
           [synth.random_small(40, 130, 61, land=True), synth.random_small(41, 59, 123, land=True)]


def single_states(clf, cases, prec, nsteps):
    out = []
    for c in cases:
        s = clf.Solver.from_case(c, precision=prec, graph_steps=0)
        s.set_initial(c.eta0, c.u0, c.v0)
        s.step(nsteps)
        out.append([t.cpu().numpy() for t in s.state()] + [t.cpu().numpy() for t in s.read_maxwave()])
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("opts", [dict(graph_steps=0), dict(graph_steps=4),
                                  dict(graph_steps=0, persistent_blocks=8)],
                         ids=["eager", "graph", "persistent"])
def test_members_equal_single_runs(clf, prec, opts):
    p = clf.FP64 if prec == "fp64" else clf.FP32
    cases = members()
    ref = single_states(clf, cases, p, 12)
    ens = clf.Ensemble(cases, precision=p, **opts)
    for i, c in enumerate(cases):
        ens.set_initial(i, c.eta0, c.u0, c.v0)
    ens.step(12)
    for i in range(len(cases)):
        got = [t.cpu().numpy() for t in ens.state(i)] + [t.cpu().numpy() for t in ens.read_maxwave(i)]
        for a, b in zip(got, ref[i]):
            assert np.array_equal(a, b), "member %d differs" % i
    if opts.get("graph_steps"):
        assert ens.query(clf.Q_GRAPH_REPLAYS) == 3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_members_equal_single_runs_with_friction(clf, prec):
    # the friction variants over the combined tile list, spherical members too
    p = clf.FP64 if prec == "fp64" else clf.FP32
    cases = [synth.random_small(50 + k, 70 + 13 * k, 40 + 9 * k, land=True,
                                coord=synth.SPHERICAL if k % 2 else synth.CARTESIAN)
             for k in range(4)]
    ref = []
    for c in cases:
        s = clf.Solver.from_case(c, precision=p, graph_steps=0, manning_n2=0.0009)
        s.set_initial(c.eta0, c.u0, c.v0)
        s.step(9)
        ref.append([t.cpu().numpy() for t in s.state()])
    ens = clf.Ensemble(cases, precision=p, graph_steps=0, manning_n2=0.0009)
    for i, c in enumerate(cases):
        ens.set_initial(i, c.eta0, c.u0, c.v0)
    ens.step(9)
    for i in range(len(cases)):
        for a, b in zip((t.cpu().numpy() for t in ens.state(i)), ref[i]):
            assert np.array_equal(a, b), "member %d differs" % i


def test_graph_replays_match_eager_each_time(clf):
    cases = members()[:4]
    g = clf.Ensemble(cases, precision=clf.FP32, graph_steps=2)
    e = clf.Ensemble(cases, precision=clf.FP32, graph_steps=0)
    for ens in (g, e):
        for i, c in enumerate(cases):
            ens.set_initial(i, c.eta0, c.u0, c.v0)
    import torch
    for rep in range(5):
        g.step(2)
        e.step(2)
        # eager work on the same stream between replays, then a full sync
        junk = torch.ones(1 << 20, device="cuda") * float(rep)
        torch.cuda.synchronize()
        for i in range(len(cases)):
            a = [t.cpu().numpy() for t in g.state(i)]
            b = [t.cpu().numpy() for t in e.state(i)]
            for x, y in zip(a, b):
                assert np.array_equal(x, y), "replay %d member %d" % (rep, i)
        del junk
    assert g.query(clf.Q_GRAPH_REPLAYS) == 5


def test_single_grid_graph_matches_eager(clf, oracle_mod):
    case = synth.config1(nx=120, ny=90, steps=10)
    g = clf.Solver.from_case(case, graph_steps=4)
    o = oracle_mod.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(2.0 * case.eta0)
    for rep in range(3):
        g.step(5)
        o.step(5)
        e_g = g.state()[0].cpu().numpy()
        assert np.array_equal(e_g, o.state()[0])
    assert g.query(clf.Q_GRAPH_REPLAYS) >= 2
