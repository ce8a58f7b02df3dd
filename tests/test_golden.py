"""The oracle still produces its stored regression values (tests/golden)."""
import json
import os

import numpy as np

from oracle import oracle as O
from tests.golden.make_golden import cases

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_regression_values():
    with open(os.path.join(HERE, "golden", "oracle_regression.json")) as fh:
        rec = json.load(fh)
    for name, vol, sp in cases():
        r = O.shape3d(vol, sp)
        e = rec[name]
        assert (r["V"], r["T"]) == (e["V"], e["T"]), name
        np.testing.assert_allclose(r["features"], e["features"], rtol=1e-13, err_msg=name)
        np.testing.assert_array_equal(r["pair_ids"], np.array(e["pair_ids"]))
