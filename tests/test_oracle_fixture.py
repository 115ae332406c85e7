"""Regression check of the oracle against its stored fixture
(``tests/golden/oracle_m8_q32.json``, written by
``tests/golden/make_oracle_fixture.py`` from the oracle only).  Not a pin to
the paper: it makes any change of the oracle's arithmetic visible."""
import json
import os

import numpy as np

from tests.golden.make_oracle_fixture import OUT, compute


def test_oracle_reproduces_fixture(orc):
    ref = json.load(open(OUT))
    cur = compute()
    assert cur["iters"] == ref["iters"]
    for key in ("Pbar", "Cbar", "sigma", "dsdD"):
        a, b = np.asarray(cur[key]), np.asarray(ref[key])
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max(), key
