"""Training checkpoints on the host: the .npz round trip, and refusal of files that are not
checkpoints (read with allow_pickle=False only)."""
import numpy as np
import pytest

from paper_1311_5029_amd import train as TR


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(5)
    p, m, v = (rng.standard_normal(27 * 32 * 2).astype(np.float32) for _ in range(3))
    path = str(tmp_path / "ck.npz")
    TR.save_checkpoint(path, p, m, v, 37, 2, 400, 16, 3e-3, [(1, 0.9), (37, 0.25)])
    st = TR.load_checkpoint(path)
    assert st["step"] == 37 and st["n_layers"] == 2 and st["steps"] == 400 and st["batch"] == 16
    assert st["lr"] == 3e-3 and st["history"] == [(1, 0.9), (37, 0.25)]
    for k, a in (("params", p), ("adam_m", m), ("adam_v", v)):
        assert st[k].dtype == np.float32 and np.array_equal(st[k], a)
    # a second save replaces the file whole
    TR.save_checkpoint(path, p, m, v, 38, 2, 400, 16, 3e-3, [])
    assert TR.load_checkpoint(path)["step"] == 38


def test_not_a_checkpoint(tmp_path):
    path = str(tmp_path / "other.npz")
    np.savez(path, params=np.zeros(4, np.float32))
    with pytest.raises(ValueError):
        TR.load_checkpoint(path)
    obj = str(tmp_path / "obj.npz")
    np.savez(obj, **{k: np.array([{"a": 1}], dtype=object) for k in TR.CHECKPOINT_KEYS})
    with pytest.raises(ValueError):   # object arrays need pickle, which the loader refuses
        TR.load_checkpoint(obj)
