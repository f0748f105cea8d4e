"""The workload descriptions in paper_2412_19207_amd/configs/*.json against the
seeded generator that builds them: names, layout, widths (and the seed that
draws uneven ones), points, boundary rows, right-hand sides, probes and the
solver settings."""
import glob
import json
import os

import numpy as np
import pytest

from paper_2412_19207_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted(glob.glob(os.path.join(ROOT, "paper_2412_19207_amd", "configs", "*.json")))


def test_every_benchmark_configuration_has_a_file():
    names = {os.path.splitext(os.path.basename(f))[0] for f in FILES}
    assert {"cfg1", "cfg2", "cfg3", "cfg4", "cfg5"} <= names


@pytest.mark.parametrize("path", FILES, ids=lambda p: os.path.basename(p))
def test_config_matches_the_generator(path):
    cfg = json.load(open(path))
    prob = wl.make(cfg["builder"])
    assert prob.name == cfg["workload"]
    assert prob.d == cfg["d"]
    assert list(prob.l) == cfg["subdomains"]
    J = int(np.prod(cfg["subdomains"]))
    w = cfg["hidden_width"]
    if isinstance(w, dict):
        lo, hi = w["uniform_int"]
        expect = np.random.default_rng(w["seed"]).integers(lo, hi + 1, size=J)
        assert np.array_equal(prob.m, expect)
    else:
        assert np.all(prob.m == w)
    # weights drawn as scale * U[-1, 1]
    rmax = max(float(np.abs(r).max()) for r in prob.R)
    assert 0.5 * cfg["weight_scale"] < rmax <= cfg["weight_scale"]
    assert prob.X_int.shape[0] == int(np.prod(np.array(cfg["points_per_subdomain"]) * np.array(cfg["subdomains"])))
    assert prob.X_bnd.shape[0] == cfg["boundary_points"]
    assert prob.F.shape[1] == cfg["right_hand_sides"]
    assert prob.probes.shape[0] == int(np.prod(cfg["probes_per_dim"]))
    assert prob.lambda_B == cfg["lambda_B"]
    meta = dict(prob.meta)
    meta.setdefault("precision", "fp64")
    for key, val in cfg["solver"].items():
        assert meta[key] == val, key
