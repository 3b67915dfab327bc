"""The oracle against its stored 10-atom trajectory (tests/golden/), written
by tests/golden/make_golden.py from the oracle alone.  A regression anchor:
a change to the oracle's arithmetic moves these values and has to be made on
purpose, with the file rewritten by that script."""

import json
import os
import sys

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load():
    with open(os.path.join(GOLDEN, "c10_oracle_trajectory.json")) as f:
        return json.load(f)


def test_oracle_reproduces_stored_trajectory():
    sys.path.insert(0, GOLDEN)
    try:
        import make_golden
    finally:
        sys.path.remove(GOLDEN)
    ref = _load()
    got = make_golden.trajectory()
    assert np.abs(np.array(got["X_min"]) - np.array(ref["X_min"])).max() <= 1e-12
    assert got["init"]["U"] == pytest.approx(ref["init"]["U"], rel=1e-11)
    assert got["init"]["mu"] == pytest.approx(ref["init"]["mu"], abs=1e-10)
    assert len(got["steps"]) == len(ref["steps"])
    for g, r in zip(got["steps"], ref["steps"]):
        for k in ("E_tot", "KE", "U", "mu"):
            assert g[k] == pytest.approx(r[k], rel=1e-11, abs=1e-10), k
        assert g["TS"] == pytest.approx(r["TS"], rel=1e-9, abs=1e-11)
        assert g["W0"] == pytest.approx(r["W0"], rel=1e-8, abs=1e-12)
        assert g["rank"] == r["rank"]
        assert np.abs(np.array(g["R"]) - np.array(r["R"])).max() <= 1e-12
