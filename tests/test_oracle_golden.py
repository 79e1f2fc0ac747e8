"""The oracle against its stored results on the small workload
(tests/golden/oracle_small.json, written by tests/golden/make_oracle_golden.py
from the oracle alone). Guards the oracle against unintended changes; its
correctness pins are the closed-form, brute-force and invariant tests."""
import json
import os

import numpy as np

from tests.golden import make_oracle_golden as G


def test_oracle_matches_stored_small_workload():
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_small.json")) as f:
        ref = json.load(f)
    now = G.compute()
    assert now["n_records"] == ref["n_records"]
    assert now["offsets_sha256"] == ref["offsets_sha256"]
    assert now["records_sha256"] == ref["records_sha256"]
    assert now["covered_pixels"] == ref["covered_pixels"]
    assert now["counters"] == ref["counters"]
    assert abs(now["rho_sum"] - ref["rho_sum"]) <= 1e-9 * abs(ref["rho_sum"])
    assert np.allclose(now["image_channel_sums"], ref["image_channel_sums"], rtol=0, atol=1e-6)
    assert np.allclose(now["sample_values"], ref["sample_values"], rtol=0, atol=1e-9)
