"""The stored oracle solves (tests/golden/oracle_*.npz) were written by the current oracle on the
current inputs: each records a hash of the oracle's sources and a fingerprint of the generated
workload, which must match."""
import os
import sys

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLDEN)
import make_oracle_solves as mk  # noqa: E402


@pytest.mark.parametrize("name", sorted(mk.SOLVES))
def test_stored_oracle_solve_is_current(name):
    g = np.load(mk.golden_path(name), allow_pickle=False)
    assert str(g["oracle_hash"]) == mk.oracle_hash(), f"rerun: python tests/golden/make_oracle_solves.py {name}"
    assert str(g["input_hash"]) == mk.input_hash(mk.SOLVES[name][0]()), "the workload generator changed"
    assert int(np.sum(g["stages"])) == sum(mk.SOLVES[name][1])
    assert np.all(np.isfinite(g["S"])) and g["S"].shape[1] == 4
