"""The stored expected values under tests/golden/ still agree with the oracle
that wrote them (tests/golden/make_golden.py)."""
import json
import os

import numpy as np

import workloads as wl
from oracle import dense, models


def test_xxz_l12_golden_matches_oracle(golden_dir):
    with open(os.path.join(golden_dir, "xxz_L12_eps05.json")) as f:
        g = json.load(f)
    h = wl.xxz_fields(12, 1.0, 0)
    assert np.array_equal(h, np.array(g["fields"]))
    H, _ = models.xxz(12, 6, 1.0, 1.0, h)
    E, _ = dense.nearest_eigenpairs(H, g["lambda"], g["n_ev"])
    assert np.max(np.abs(E - np.array(g["eigenvalues_nearest"]))) < 1e-12
