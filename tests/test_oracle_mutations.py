"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's source (a dropped
term, a wrong sign, index or side, a swapped reading), compiles the copy on
the CPU and runs the pins that must notice it, in a child process that loads
the mutated library (``CLF_ORACLE_LIB``).  The case passes when those pins
fail.  The real oracle is not touched.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "cliffs_oracle.cpp")
PINS = "tests/test_oracle_pins.py::"

# (name, original text, planted text, pins that must fail)
MUTATIONS = [
    ("spherical x spacing without cos(lat)",
     "m.xfac[j] = 1.0 / (Rd * std::cos(m.y[j] * deg));", "m.xfac[j] = 1.0 / Rd;",
     ["test_spherical_zonal_wave_speed_at_45N"]),
    ("cos(lat) of the latitude taken in radians",
     "m.xfac[j] = 1.0 / (Rd * std::cos(m.y[j] * deg));",
     "m.xfac[j] = 1.0 / (Rd * std::cos(m.y[j]));",
     ["test_spherical_zonal_wave_speed_at_45N"]),
    ("sea-floor deformation with the wrong sign",
     "m.d[k] = m.d[k] - re(e);", "m.d[k] = m.d[k] + re(e);",
     ["test_deform_bottom_definition"]),
    ("flooding tie resolved to the left neighbour",
     "if (re(fL) > re(fR)) s = -1;", "if (re(fL) >= re(fR)) s = -1;",
     ["test_flood_tie_on_symmetric_sill"]),
    ("tie velocity taken from one side",
     "w1[k] = 0.5 * (w[k - 1] + w[k + 1]);", "w1[k] = w[k - 1];",
     ["test_flood_tie_on_symmetric_sill"]),
    ("semi-implicit friction in place of the explicit -alpha dt",
     "if (p.n2 > 0.0 && p.fric_form == 0) {", "if (p.n2 > 0.0 && p.fric_form == 7) {",
     ["test_friction_explicit_one_step"]),
    ("explicit friction without the no-reversal cap",
     "if (re(f) > 1.0) f = T(1.0);", "",
     ["test_friction_explicit_does_not_reverse_the_flow"]),
    ("friction on p only",
     "      Pn = Pn - a;\n      Mn = Mn - a;", "      Pn = Pn - a;",
     ["test_friction_explicit_one_step"]),
    ("friction speed without the tangential velocity",
     "T sp = sqrt_t(C.w * C.w + C.t * C.t);\n      T den = C.H * cbrt_t(C.H);\n      T f =",
     "T sp = sqrt_t(C.w * C.w);\n      T den = C.H * cbrt_t(C.H);\n      T f =",
     ["test_friction_explicit_one_step"]),
    ("open edge: incoming invariant taken from the node",
     "    pp = w + 2.0 * c;\n    qq = T(-2.0 * c0);", "    pp = w + 2.0 * c;\n    qq = w - 2.0 * c;",
     ["test_open_edge_drains_a_raised_lake_to_still_water"]),
    ("open edge on the wrong side",
     "m.xfac[j], nullptr, (m.p.open_mask & 1) != 0,",
     "m.xfac[j], nullptr, (m.p.open_mask & 2) != 0,",
     ["test_open_edge_lets_a_linear_pulse_leave"]),
    ("left interface with the right spacing",
     "const double iL = fac * ib[k];", "const double iL = fac * ib[k + 1];",
     ["test_single_node_pulse_graded_grid"]),
    ("mirror ghost keeps the normal velocity",
     "L.H = C.H; L.w = -C.w; L.t = C.t; L.D = C.D;  // mirror ghost",
     "L.H = C.H; L.w = C.w; L.t = C.t; L.D = C.D;  // mirror ghost",
     ["test_mirror_symmetry_bitwise", "test_lake_at_rest"]),
    ("second-order term with dt instead of dt^2",
     "T b2 = lam * p.dt2;", "T b2 = lam * p.dt;",
     ["test_single_node_pulse_closed_form", "test_lax_wendroff_standing_mode"]),
    ("height cap of a newly wet node at the full source height",
     "    T cap = 0.5 * Hn[j];", "    T cap = Hn[j];",
     ["test_wet_front_one_cell_per_sweep"]),
    ("flooding test without the neighbour's depth",
     "fL = (H[k - 1] - D[k - 1]) + D[k];", "fL = H[k - 1] + D[k];",
     ["test_wet_front_one_cell_per_sweep", "test_mirror_symmetry_bitwise"]),
    ("spherical source with the wrong sign",
     "      Pn = Pn + s3;\n      Mn = Mn - s3;", "      Pn = Pn - s3;\n      Mn = Mn + s3;",
     ["test_spherical_source_conserves_area_weighted_volume"]),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found exactly once: %r" % old
    mutated = tmp_path / "mutant.cpp"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-std=c++17", "-shared", "-fPIC", "-o", str(lib), str(mutated)], check=True)
    env = dict(os.environ, CLF_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
                         + [PINS + p for p in pins], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=600)
    # exit code 1: tests ran and at least one failed (not a crash or a collection error)
    assert res.returncode == 1, "mutation '%s' not caught:\n%s" % (name, res.stdout[-2000:])
