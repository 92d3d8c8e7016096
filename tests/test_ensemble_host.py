"""Host-side logic of the checkpointed ensemble runner (no GPU needed)."""
import json

import numpy as np
import pytest


def test_checkpoint_of_another_run_is_refused(tmp_path):
    from paper_1903_12227_amd import ensemble
    ck = str(tmp_path / "run.npz")
    other = {"L": 8, "m0": 8, "contrast": 10.0, "a_bg": 1.0, "N": 99, "seed": 1, "prec": 2, "tol": 1e-10,
             "occ_threshold": 1}
    np.savez(ck, params=np.array(json.dumps(other, sort_keys=True)), done=np.array(0),
             ahom=np.zeros((0, 2, 2)), iters=np.zeros((0, 2), dtype=np.int32))
    with pytest.raises(ValueError):
        ensemble.run_ensemble(8, 8, 10.0, 10, checkpoint=ck)


def test_checkpoint_round_trip(tmp_path):
    from paper_1903_12227_amd import ensemble
    ck = str(tmp_path / "run.npz")
    params = ensemble._params(8, 8, 10.0, 1.0, 5, 3, 2, 1e-10, 1234)
    ah = np.arange(20, dtype=np.float64).reshape(5, 2, 2)
    it = np.arange(10, dtype=np.int32).reshape(5, 2)
    ensemble._save(ck, params, 3, ah, it)
    done, a2, i2 = ensemble._load(ck, params)
    assert done == 3 and np.array_equal(a2, ah[:3]) and np.array_equal(i2, it[:3])
