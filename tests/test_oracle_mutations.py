"""Each plausible mistake planted in a copy of the oracle's C source (a dropped
term, a wrong sign, a wrong index or comparison) must make at least one pin of
tests/test_oracle_pins.py fail. The oracle itself is never modified."""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "csc_oracle.c")

MUTATIONS = {
    "sign_rule_flipped": ("*s = vdot(pq, N) >= 0 ? 1.0 : -1.0;", "*s = vdot(pq, N) <= 0 ? 1.0 : -1.0;"),
    "pseudonormal_unweighted": ("vn[3 * v] += al * n.x; vn[3 * v + 1] += al * n.y; vn[3 * v + 2] += al * n.z;",
                                "vn[3 * v] += n.x; vn[3 * v + 1] += n.y; vn[3 * v + 2] += n.z;"),
    "edge_normal_one_face": ("en[3 * e + c] = fn[3 * fl + c] + fn[3 * fr + c];",
                             "en[3 * e + c] = 2.0 * fn[3 * fl + c];"),
    "closest_region_wrong": ("if (d6 >= 0 && d5 <= d6)", "if (d6 >= 0 && d5 >= d6)"),
    "edge_param_wrong": ("double t = d2 / (d2 - d6);", "double t = d6 / (d2 - d6);"),
    "cull_too_tight": ("const double r = wh + 2 * tol;", "const double r = 0.7 * wh;"),
    "edge_owner_flipped": ("        if (u < w) {\n            face_edges[h] = (int32_t)ne;",
                           "        if (u > w) {\n            face_edges[h] = (int32_t)ne;"),
    "gradient_sign": ("double f = -up[c] * w[k];", "double f = up[c] * w[k];"),
    "winding_term_dropped": ("+ vdot(a, cc) * lb + vdot(b, cc) * la;", "+ vdot(a, cc) * lb;"),
}

# quick pins (whole-function calls; fixtures replaced by direct generation)
import meshgen  # noqa: E402

_cfg = {}


def _configs(k):
    if k not in _cfg:
        _cfg[k] = meshgen.make_config(k)
    return _cfg[k]


PIN_CALLS = [
    ("cube_closed_form", lambda: pins.test_cube_matches_closed_form()),
    ("cube_pseudonormals", lambda: pins.test_cube_features_and_pseudonormals()),
    ("tetra_numbering", lambda: pins.test_feature_numbering_tetrahedron()),
    ("feature_regions", lambda: pins.test_feature_distance_every_region()),
    ("allpairs_torus", lambda: pins.test_allpairs_matches_culled_oracle("torus", 28)),
    ("icosphere_bracket", lambda: pins.test_icosphere_brackets_sphere(2)),
    ("winding_sign", lambda: pins.test_sign_matches_winding_number(_configs, 2)),
    ("gradient_fd", lambda: pins.test_gradient_matches_finite_differences()),
    ("translation", lambda: pins.test_gradient_translation_invariant()),
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    mutated = tmp_path / "csc_oracle_mut.c"
    mutated.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", str(so),
                    str(mutated), "-lm"], check=True)
    caught = []
    with oracle.library(str(so)):
        for pin, call in PIN_CALLS:
            try:
                call()
            except (AssertionError, ValueError):
                caught.append(pin)
                break
    assert caught, f"no pin catches the planted mistake {name}"
