"""Values the paper prints (tests/golden/, each with its citation) against
the defaults and workloads of this implementation."""
import json
import os

import pytest

import z4c_inputs as zi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_default_parameters_are_the_papers():
    g = load("paper_parameters.json")
    p = zi.params_default(g["fd_order"])
    assert p["fd_order"] == g["fd_order"]
    assert p["ko_sigma"] == g["ko_sigma"]
    assert p["kappa1"] == g["kappa1"]
    assert p["kappa2"] == g["kappa2"]


@pytest.mark.parametrize("name", ["periodic16", "bl64x32", "bbh512mixed"])
def test_workload_time_steps_use_the_papers_cfl(name):
    g = load("paper_parameters.json")
    mesh, p, _, dt, _ = zi.workload(name)
    assert dt == pytest.approx(g["cfl"] * mesh.dx_min(), rel=1e-15)
    assert p["ko_sigma"] == g["ko_sigma"] and p["kappa1"] == g["kappa1"]
