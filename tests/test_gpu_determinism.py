"""Run-to-run determinism and tiling independence of the FP32 path, which
has no bitwise reference (the FP64 path is pinned bit for bit to the
oracle): no atomics, and every node's arithmetic is the same whatever the
segment length, the launch shape or the graph replay."""
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


def run(clf, case, nsteps, **kw):
    s = clf.Solver.from_case(case, precision=clf.FP32, maxout=1, **kw)
    s.set_initial(case.eta0, case.u0, case.v0)
    s.step(nsteps)
    out = [t.cpu().numpy() for t in s.state()] + [t.cpu().numpy() for t in s.read_maxwave()]
    del s
    return out


@pytest.mark.parametrize("gen", ["coast", "spherical"])
def test_fp32_independent_of_tiling_and_runs(clf, gen):
    if gen == "coast":
        case = synth.random_small(80, 300, 260, land=True, amp=1.0)
    else:
        case = synth.config2(steps=10, scale=4)
    print("determinism", gen, case.nx, case.ny, flush=True)
    ref = run(clf, case, 40, segment=16, graph_steps=0)
    variants = [dict(segment=16, graph_steps=0),            # the same again
                dict(segment=8, graph_steps=0), dict(segment=37, graph_steps=0),
                dict(segment=256, graph_steps=0), dict(segment=16, graph_steps=8),
                dict(segment=16, graph_steps=0, persistent_blocks=16), dict(autotune=1)]
    for kw in variants:
        got = run(clf, case, 40, **kw)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), str(kw)
