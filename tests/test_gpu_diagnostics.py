"""Set-up diagnostics of the library (section Numerical stability and the
CFL remark after solver2): the preprocessed depth, its pass count, the
still-water Courant number and the stability factor f_j (eq:f), against the
oracle and a closed form."""
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


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_preprocessing_and_courant_match_oracle(clf, oracle_mod, seed):
    case = synth.random_small(seed, 70, 50, land=True, amp=0.3)
    print("diagnostics seed", seed, flush=True)
    g = clf.Solver.from_case(case)
    o = oracle_mod.Oracle.from_case(case)
    assert np.array_equal(g.depth().cpu().numpy(), o.depth())
    assert g.query(clf.Q_SSL_PASSES) == o.ssl_passes
    assert abs(g.query(clf.Q_MAX_CFL) - o.max_cfl()) <= 1e-12 * o.max_cfl()


def test_min_f_closed_form(clf):
    # one node of depth 1 between neighbours of depth 49 on both axes:
    # f = (6*1 - 7 - 7) / (4*1) = -2 there (eq:f), and larger elsewhere
    x = np.arange(5) * 100.0
    y = np.arange(5) * 100.0
    d = np.full((5, 5), 49.0)
    d[2, 2] = 1.0
    s = clf.Solver(x, y, d, 0.5, ssl_alpha=0.0)
    assert s.query(clf.Q_MIN_F) == -2.0
    # with the preprocessing the spike is deepened and f becomes positive
    t = clf.Solver(x, y, d, 0.5)
    assert t.query(clf.Q_MIN_F) > 0.0
    assert t.query(clf.Q_SSL_PASSES) >= 1


def test_courant_limit_rejected(clf):
    x = np.arange(20) * 100.0
    d = np.full((20, 20), 100.0)
    dt_ok = 0.99 * 100.0 / np.sqrt(9.81 * 100.0)
    s = clf.Solver(x, x, d, dt_ok, ssl_alpha=0.0)
    assert abs(s.query(clf.Q_MAX_CFL) - 0.99) < 1e-12
    with pytest.raises(clf.ClfError) as e:
        clf.Solver(x, x, d, 1.2 * dt_ok, ssl_alpha=0.0)
    assert e.value.code == -2
