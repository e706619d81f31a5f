"""The no-allocation entry point clf_step_static against clf_step on a
context (the existing entry point), through the C-ABI: same grid, depth,
parameters and initial state, bit-identical state and maxwave, on two calls
in a row, the second on a smaller grid, in FP64 and FP32."""
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


def _storage(ctx, prec):
    """The context's state and depth in the storage form (exact)."""
    import torch
    e, u, v, w = (t.cpu().numpy() for t in ctx.state())
    d = ctx.depth().cpu().numpy()
    if prec == "fp64":
        h = ctx.raw_state()[0].cpu().numpy()
        arrs = (d, h, u, v)
        dtype = torch.float64
    else:
        # FP32 stores eta on wet nodes and -d on dry ones (h = 0 exactly)
        eta = np.where(w.astype(bool), e, -d)
        arrs = tuple(a.astype(np.float32) for a in (d, eta, u, v))
        dtype = torch.float32
    return [torch.tensor(a, dtype=dtype, device="cuda") for a in arrs]


def _observe(H, U, V, D, hmin, prec):
    """eta, u, v (zero on dry nodes) and the wet flag, as clf_get_state gives them."""
    H, U, V, D = (t.cpu().numpy() for t in (H, U, V, D))
    if prec == "fp64":
        wet = H > hmin
        eta = H - D
    else:
        wet = (D + H) > np.float32(hmin)
        eta = H
    z = lambda a: np.where(wet, a.astype(np.float64), 0.0)
    return z(eta), z(U), z(V), wet


def _run_pair(clf, case, prec, nsteps, with_max, **kw):
    import torch
    p = clf.FP64 if prec == "fp64" else clf.FP32
    ctx = clf.Solver.from_case(case, precision=p, **kw)
    ctx.set_initial(2.0 * case.eta0, case.u0, case.v0)
    D, H, U, V = _storage(ctx, prec)
    b = [torch.empty_like(H) for _ in range(3)]
    emax = torch.zeros_like(H) if with_max else None
    s2max = torch.zeros_like(H) if with_max else None
    print("static", prec, case.nx, case.ny, nsteps, flush=True)
    which, bad = clf.step_static(case.x, case.y, case.coord, D, (H, U, V), tuple(b), nsteps,
                                 case.dt, eta_max=emax, speed2_max=s2max, precision=p,
                                 h_min=case.h_min, manning_n2=case.manning_n2, **kw)
    assert not bad
    fin = (H, U, V) if which == 0 else tuple(b)
    got = _observe(*fin, D, case.h_min, prec)
    ctx.step(nsteps)
    ref = [t.cpu().numpy() for t in ctx.state()]
    assert np.array_equal(got[3], ref[3].astype(bool)), "wet mask differs"
    for name, a, r in zip(("eta", "u", "v"), got[:3], ref[:3]):
        assert np.array_equal(a, r), "%s differs (max %.3e)" % (name, np.abs(a - r).max())
    if with_max:
        em, sm = (t.cpu().numpy() for t in ctx.read_maxwave())
        assert np.array_equal(emax.cpu().numpy().astype(np.float64), em)
        assert np.array_equal(np.sqrt(s2max.cpu().numpy().astype(np.float64)), sm)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_static_step_matches_context_twice(clf, prec):
    # first call: a larger grid with land, friction and maxwave, odd step
    # count (result in buffer B); second call on the same GPU scratch: a
    # smaller grid, even step count (result in buffer A), no maxwave
    big = synth.random_small(1, 130, 75, land=True)
    big.manning_n2 = 0.0009
    _run_pair(clf, big, prec, 7, True)
    small = synth.random_small(2, 61, 40, land=True, coord=synth.SPHERICAL)
    _run_pair(clf, small, prec, 4, False)


def test_static_step_repeats_after_another_grid(clf):
    # back to the first grid: the scratch is rebuilt for it
    c = synth.config1(nx=120, ny=90, steps=10)
    _run_pair(clf, c, "fp64", 5, True)
    _run_pair(clf, synth.random_small(3, 64, 33, land=True), "fp64", 2, False)
    _run_pair(clf, c, "fp64", 6, True)


def test_static_step_rejects_oversize_and_bad_arguments(clf):
    import torch
    t = torch.zeros(4, dtype=torch.float64, device="cuda")
    # metric arrays of a 300000-node-long grid exceed the 4 MiB scratch
    nx = 300000
    x = np.arange(nx, dtype=np.float64)
    y = np.arange(3, dtype=np.float64)
    depth = torch.zeros((3, nx), dtype=torch.float64, device="cuda")
    with pytest.raises(clf.ClfError) as ei:
        clf.step_static(x, y, clf.CARTESIAN, depth, (t, t, t), (t, t, t), 1, 1.0)
    assert ei.value.code == -6
    # alternate sweep order and mismatched maxwave arrays are refused
    small = torch.zeros((5, 5), dtype=torch.float64, device="cuda")
    s5 = np.arange(5.0)
    with pytest.raises(clf.ClfError) as ei:
        clf.step_static(s5, s5, clf.CARTESIAN, small, (t, t, t), (t, t, t), 1, 1.0, sweep_order=1)
    assert ei.value.code == -1
    with pytest.raises(clf.ClfError) as ei:
        clf.step_static(s5, s5, clf.CARTESIAN, small, (t, t, t), (t, t, t), 1, 1.0, eta_max=small)
    assert ei.value.code == -1
