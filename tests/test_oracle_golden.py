"""The oracle reproduces its committed regression fixtures (tests/golden/) bit for bit. The
fixtures come from the oracle alone (tests/golden/make_golden.py); a change of the oracle's
arithmetic shows here and is made deliberately, with the fixtures regenerated."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, HERE)
import make_golden  # noqa: E402


@pytest.mark.parametrize("name,desc,vals", make_golden.cases(), ids=lambda x: x if isinstance(x, str) and " " not in x else "")
def test_oracle_matches_fixture(name, desc, vals):
    lines = [l.strip() for l in open(os.path.join(HERE, name + ".txt")) if not l.startswith("#")]
    stored = np.array([float.fromhex(l) for l in lines if l])
    assert stored.shape == vals.shape
    assert np.array_equal(stored, vals), name
