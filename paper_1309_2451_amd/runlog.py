"""Long runs: a JSON-lines stream of the observations and torch checkpoints of
the field, so that a run can stop and resume (the populations-against-time
records of Sec. V, Fig. 4, written as they are produced).

Time is the integer step counter times dt, never a running sum, and the pass
kernels are deterministic, so a run resumed from a checkpoint reproduces the
uninterrupted run with the same segment length bit for bit.  (A different
segment length moves the boundaries of the fused step chains: the result
then agrees to rounding, not bitwise.)

Checkpoints hold only tensors, numbers and a JSON string, and are read with
torch.load(weights_only=True).
"""
from __future__ import annotations

import json
import os

import numpy as np


def obs_rows(records, dt, step0=0):
    """JSON-ready dicts of the library's observation records (Solver.step /
    read_obs).  Record steps count from the start of their call; step0 is the
    absolute step at that start, and t = step * dt."""
    rows = []
    for r in records:
        step = int(step0) + int(r["step"])
        rows.append({"step": step, "t": step * float(dt), "norm": float(r["norm"]),
                     "mean": [float(v) for v in r["mean"]], "pop": [float(v) for v in r["pop"]],
                     "epot": float(r["epot"]), "energy": float(r["energy"]), "flags": int(r["flags"])})
    return rows


class ObsLog:
    """Appends observation rows to a JSON-lines file, one object per line,
    flushed after every write."""

    def __init__(self, path, mode="a"):
        self.path = str(path)
        self.f = open(self.path, mode)

    def write(self, records, dt, step0=0):
        for row in obs_rows(records, dt, step0):
            self.f.write(json.dumps(row) + "\n")
        self.f.flush()

    def close(self):
        if self.f:
            self.f.close()
            self.f = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def read_log(path):
    """The rows of a JSON-lines observation file."""
    with open(path) as f:
        return [json.loads(line) for line in f if line.strip()]


def save_checkpoint(torch, path, psi, step, dt, meta=None):
    """The field (copied to the host), the absolute step, dt and a metadata
    dict (JSON-serialisable) into `path`, written to a temporary file first
    and then renamed, so an interrupted write leaves the previous checkpoint
    intact."""
    tmp = str(path) + ".tmp"
    torch.save({"psi": psi.detach().cpu().contiguous(), "step": int(step), "dt": float(dt),
                "meta": json.dumps(meta or {}, sort_keys=True)}, tmp)
    os.replace(tmp, str(path))


def load_checkpoint(torch, path, device):
    """(psi on `device`, step, dt, meta) from a checkpoint of save_checkpoint."""
    d = torch.load(str(path), map_location="cpu", weights_only=True)
    return d["psi"].to(device).contiguous(), int(d["step"]), float(d["dt"]), json.loads(d["meta"])


def run(solver, psi, nsteps, dt, obs_every, segment, step0=0, log=None, ckpt_path=None, meta=None):
    """Advance `psi` in place from absolute step `step0` by `nsteps` real-time
    steps, in segments of `segment` steps (a multiple of obs_every when
    observations are taken); after each segment the observations go to `log`
    (an ObsLog) and, with `ckpt_path`, the field to a checkpoint.  Returns the
    absolute step reached."""
    if segment < 1 or (obs_every and segment % obs_every):
        raise ValueError("segment must be a positive multiple of obs_every")
    step = int(step0)
    end = step + int(nsteps)
    while step < end:
        n = min(segment, end - step)
        rec = solver.step(psi, n, dt, obs_every=obs_every)
        if log is not None and rec is not None and len(rec):
            log.write(rec, dt, step)
        step += n
        if ckpt_path is not None:
            save_checkpoint(solver.torch, ckpt_path, psi, step, dt, meta)
    return step
