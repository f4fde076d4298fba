"""The autotuner: every candidate it may choose matched the default schedule's
result, the chosen factorisation is what later plans of that extent use, solves
with the tuned plans match the FP64 loop oracle, and the database survives a
save / clear / load round trip."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import TOL, assert_close, gpu_periodic, rounded_input

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,dtype", [((1024, 768), "f32"), ((600, 640), "f64"), ((64, 192, 96), "f32")])
def test_tuned_plans_match_oracle(dims, dtype, tmp_path):
    import paper_2105_06676_amd as sfft
    sfft.tune_clear()
    rep = sfft.tune(dims, dtype, reps=3)
    assert len(rep["axes"]) >= 1
    for ax in rep["axes"]:
        n = ax["n"]
        assert any(c.get("eligible") for c in ax["candidates"]), ax
        for c in ax["candidates"]:
            if c.get("eligible"):
                assert c["rel_l2_vs_default"] <= TOL[dtype]
        chosen = ax["chosen"]
        desc = sfft.plan_describe(dims, dtype)
        if chosen != "default":
            assert int(np.prod(chosen)) == n
            axis = list(dims).index(n)
            assert desc["levels"][axis] == chosen, (desc["levels"], chosen)
    # the tuned plans against the oracle (every mode visible at small T)
    c = wl.box_random_coeffs(77, len(dims), 1)
    a0 = wl.uniform(77, "grid", int(np.prod(dims))).reshape(dims)
    ref = oracle.periodic(rounded_input(a0, dtype), c, 5)
    assert_close(gpu_periodic(a0, c, 5, dtype), ref, TOL[dtype], (dims, dtype))
    # persistence
    path = str(tmp_path / "tune.json")
    sfft.tune_save(path)
    saved = json.load(open(path))
    before = sfft.plan_describe(dims, dtype)
    sfft.tune_clear()
    sfft.tune_load(path)
    after = sfft.plan_describe(dims, dtype)
    assert after["levels"] == before["levels"]
    assert saved["version"] == 1
    sfft.tune_clear()


def test_tune_load_rejects_bad_levels(tmp_path):
    import paper_2105_06676_amd as sfft
    path = str(tmp_path / "bad.json")
    with open(path, "w") as f:
        f.write('{"version": 1, "splits": [{"n": 1000, "f64": 0, "levels": [10, 10]}]}')
    with pytest.raises(sfft.SfftError):
        sfft.tune_load(path)
