"""Deterministic kernels on the GPU: the same steps twice give the same bits
(every tile variant; a race in an LDS exchange would show here), and a run
stopped at a checkpoint and resumed on a fresh handle reproduces the
uninterrupted run bit for bit, observations included."""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
ssf = pytest.importorskip("paper_1309_2451_amd")
from paper_1309_2451_amd import runlog  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n):
    g = synth.Grid(n, (-8.0, -8.0, -20.0), (8.0, 8.0, 20.0))
    gd = synth.ctap_guides(g, z1=4.0, z3=-4.0, wg=4.0)
    psi0 = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, -10.0), width=(0.5, 0.5, 3.0), k=(0.0, 0.0, 3.0))
    return g, gd, psi0


def _solver(g, gd, dtype, tiles=None):
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=DEV)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    if tiles is not None:
        s.set_tiles(tiles)
    return s


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("tiles", [[0, 0, 0], [0, 1, 1], [0, 2, 2]])
def test_repeated_runs_are_bitwise(dtype, tiles):
    say("repeat", dtype, tiles)
    g, gd, psi0 = _case((40, 24, 48))
    s = _solver(g, gd, dtype, tiles)
    outs = []
    for _ in range(2):
        t = torch.from_numpy(psi0).to(s.tdtype).to(DEV).contiguous()
        rec = s.step(t, 30, 0.004, obs_every=10)
        outs.append((t, rec))
    s.close()
    assert torch.equal(outs[0][0], outs[1][0])
    assert outs[0][1].tobytes() == outs[1][1].tobytes()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_resume_from_checkpoint_is_bitwise(dtype, tmp_path):
    say("resume", dtype)
    g, gd, psi0 = _case((32, 24, 40))
    dt, every, seg = 0.004, 10, 20
    # uninterrupted: 60 steps in segments of 20
    s = _solver(g, gd, dtype)
    a = torch.from_numpy(psi0).to(s.tdtype).to(DEV).contiguous()
    with runlog.ObsLog(tmp_path / "a.jsonl", "w") as log:
        end = runlog.run(s, a, 60, dt, every, seg, log=log)
    s.close()
    assert end == 60
    # interrupted after 40 steps, resumed from the checkpoint on a new handle
    s = _solver(g, gd, dtype)
    b = torch.from_numpy(psi0).to(s.tdtype).to(DEV).contiguous()
    ck = tmp_path / "ck.pt"
    with runlog.ObsLog(tmp_path / "b.jsonl", "w") as log:
        runlog.run(s, b, 40, dt, every, seg, log=log, ckpt_path=ck, meta={"grid": list(g.n)})
    s.close()
    del b
    c, step, dt2, meta = runlog.load_checkpoint(torch, ck, DEV)
    assert step == 40 and dt2 == dt and meta == {"grid": list(g.n)}
    s = _solver(g, gd, dtype)
    with runlog.ObsLog(tmp_path / "b.jsonl", "a") as log:
        end = runlog.run(s, c, 60 - step, dt, every, seg, step0=step, log=log)
    s.close()
    assert end == 60
    assert torch.equal(a, c)
    ra, rb = runlog.read_log(tmp_path / "a.jsonl"), runlog.read_log(tmp_path / "b.jsonl")
    assert [r["step"] for r in ra] == list(range(10, 61, 10))
    assert ra == rb
