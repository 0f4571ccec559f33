"""Observation stream and checkpoint files (host side): rows carry absolute
steps and t = step * dt, and a checkpoint round-trips the field, the step
and the metadata through torch.load(weights_only=True)."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1309_2451_amd import runlog  # noqa: E402
from paper_1309_2451_amd._ssf import OBS_DTYPE  # noqa: E402


def _records(steps):
    r = np.zeros(len(steps), dtype=OBS_DTYPE)
    for k, s in enumerate(steps):
        r[k]["step"] = s
        r[k]["norm"] = 1.0 - 1e-9 * k
        r[k]["mean"] = (0.5 * k, -0.25, 3.0)
        r[k]["pop"] = (0.9, 0.1 - 0.01 * k, 0.01 * k)
        r[k]["energy"] = 2.5
        r[k]["epot"] = -1.5
    return r


def test_obs_rows_use_absolute_steps_and_integer_time(tmp_path):
    dt = 0.002
    path = tmp_path / "obs.jsonl"
    with runlog.ObsLog(path, "w") as log:
        log.write(_records([100, 200]), dt, step0=0)
        log.write(_records([100, 200]), dt, step0=200)
    rows = runlog.read_log(path)
    assert [r["step"] for r in rows] == [100, 200, 300, 400]
    # t is step * dt, not a running sum of dt
    assert [r["t"] for r in rows] == [s * dt for s in (100, 200, 300, 400)]
    assert rows[1]["pop"] == [0.9, 0.1 - 0.01, 0.01]
    assert rows[0]["mean"] == [0.0, -0.25, 3.0] and rows[0]["energy"] == 2.5 and rows[0]["flags"] == 0
    for line in open(path):
        json.loads(line)                                # one object per line


def test_checkpoint_round_trip_is_exact(tmp_path):
    rng = np.random.default_rng(1)
    for dtype in (torch.complex64, torch.complex128):
        psi = torch.from_numpy(rng.standard_normal((4, 6, 8)) + 1j * rng.standard_normal((4, 6, 8))).to(dtype)
        path = tmp_path / ("c%d.pt" % psi.element_size())
        runlog.save_checkpoint(torch, path, psi, 1234, 0.004, {"grid": [8, 6, 4], "config": "test"})
        got, step, dt, meta = runlog.load_checkpoint(torch, path, "cpu")
        assert torch.equal(got, psi) and got.dtype == dtype
        assert step == 1234 and dt == 0.004
        assert meta == {"grid": [8, 6, 4], "config": "test"}


def test_run_rejects_segments_that_split_observations():
    with pytest.raises(ValueError):
        runlog.run(None, None, 10, 0.01, obs_every=4, segment=6)
