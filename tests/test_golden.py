"""The synthetic workloads and the defaults of the library and the oracle
use the values the paper prints (tests/golden/)."""
import ctypes
import inspect

import numpy as np

from paper_1410_0753_amd import synth
from tests.golden import load


def test_beach_workload_uses_the_paper_table():
    g = load("sloping_beach.txt")
    c = synth.beach_1d()
    assert c.coord == synth.CARTESIAN and g["cartesian"] == 1
    assert c.h_min == g["h_min"] and c.dt == g["dt"] and c.steps == g["steps"]
    assert c.extra["cot_beta"] == g["cot_beta"]
    assert abs(c.extra["H"] / c.extra["d"] - g["H_over_d"]) < 1e-15
    # graded spacing: d on the deep end, 0.1 d at the still shoreline
    dx = np.diff(c.x.astype(np.float64)) / c.extra["d"]
    # (coordinates are rounded to float32)
    assert abs(dx.max() - g["spacing_deep"]) < 1e-5
    assert abs(dx[c.x[:-1] >= 0].min() - g["spacing_shore"]) < 1e-5
    # the depth is the 1:cot_beta plane up to d
    x = c.x.astype(np.float64)
    d = c.depth[0].astype(np.float64)
    ref = np.minimum(c.extra["d"], x / g["cot_beta"])
    assert np.allclose(d, ref, rtol=1e-6, atol=1e-7)


def test_preprocessing_defaults_match_the_paper():
    g = load("depth_preprocessing.txt")
    from paper_1410_0753_amd import build, clf
    lib = ctypes.CDLL(build.LIB)
    p = clf.Params()
    lib.clf_default_params(ctypes.byref(p))
    assert p.ssl_alpha == g["alpha_default"]
    assert p.ssl_min_depth == g["min_depth_default"]
    assert g["alpha_lower"] < p.ssl_alpha < g["alpha_upper"]
    assert p.h_min == g["h_min_2d_examples"]
    import oracle
    sig = inspect.signature(oracle.ssl)
    assert sig.parameters["alpha"].default == g["alpha_default"]
    assert sig.parameters["min_depth"].default == g["min_depth_default"]
    ora = inspect.signature(oracle.Oracle.__init__)
    assert ora.parameters["h_min"].default == g["h_min_2d_examples"]
