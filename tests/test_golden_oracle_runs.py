"""The stored oracle runs under tests/golden/oracle_runs (written by
tests/golden/make_oracle_runs.py, which calls only the oracle and the input generators)
belong to the sources in the tree, and their start and end satisfy what the method
fixes: sum(phi) is conserved by the FP64 oracle to rounding in a closed box."""
import importlib.util
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _G():
    spec = importlib.util.spec_from_file_location(
        "make_oracle_runs", os.path.join(HERE, "golden", "make_oracle_runs.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


G = _G()


@pytest.mark.parametrize("name", sorted(G.CASES))
def test_oracle_run_fixture_is_current(name):
    cfg, steps, d = G.load(name)
    assert str(d["source_sha1"]) == G.source_sha1(), (
        "the oracle or the inputs changed since the fixture was written: "
        "run python tests/golden/make_oracle_runs.py " + name)
    assert str(d["cfg"]) == G.cfg_json(cfg)
    assert str(d["input_sha1"]) == G.input_sha1(cfg), "the seeded start changed"
    assert int(d["steps"]) == steps
    nx, ny, nz = cfg["shape"]
    assert d["phi"].shape == (nz, ny, nx) and d["J"].shape == (3, nz, ny, nx)
    if cfg.get("open_P") is None:
        # sum(phi) exact under the oracle's streaming with walls (bounce-back) and BGK
        assert abs(float(d["mass1"]) - float(d["mass0"])) <= 1e-12 * float(d["mass0"])
    else:
        # through an open face over light fluid (phi ~ 0 there) sum(phi) changes little
        assert abs(float(d["mass1"]) - float(d["mass0"])) <= 1e-4 * float(d["mass0"])
    # the stored phi (float32) sums to the stored mass
    assert abs(d["phi"].astype(np.float64).sum() - float(d["mass1"])) <= 1e-6 * float(d["mass1"])
    assert np.isfinite(d["J"]).all() and np.isfinite(d["P"]).all()
