"""The stored oracle results under tests/golden/ (written by
tests/golden/make_golden.py from oracle/ and synth/ only): they load
without pickles, name their recipe, and the w = 0.2 trace shows what the
method does on that workload."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAMES = ["affine4000", "surface10k", "surface50k", "surface20k_w02"]


def _load(name):
    z = np.load(os.path.join(GOLD, name + ".npz"), allow_pickle=False)
    return z, json.loads(str(z["meta"]))


@pytest.mark.parametrize("name", NAMES)
def test_fixture_loads_and_names_its_recipe(name):
    z, meta = _load(name)
    assert meta["M"] > 0 and "workload" in meta and "oracle" in meta
    for k in z.files:
        assert np.all(np.isfinite(z[k])) if z[k].dtype.kind == "f" else True


def test_surface20k_w02_stalls_and_drifts():
    """Section IV uses w = 0.7; with w = 0.2 and 20% uniform outliers the
    oracle's run does not converge to the registration: the RMSE against
    the true positions (eq. 22) falls to its minimum within the first 50
    iterations (0.14 at iteration 30) and then grows (0.62 at 250), while
    sigma^2 plateaus near 0.06 and stays two orders of magnitude above the
    scene noise (0.02^2)."""
    z, meta = _load("surface20k_w02")
    s2, rm = z["sigma2"], z["rmse"]
    assert len(s2) == meta["iters"] == 250
    assert s2.min() > 75 * 0.02 ** 2
    k = int(np.argmin(rm))
    assert k < 50 and rm[-1] > 4 * rm[k]
    assert np.all(np.diff(rm[k:]) > 0)
