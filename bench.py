#!/usr/bin/env python
"""Benchmark: split-step Fourier propagation of the three-guide workload.

Workload (default): 256 x 256 x 512 grid on [-8,8)^2 x [-64,64), three
Gaussian guides (v0 = 40, sigma = 0.6, d0 = 3, delta = 1.2), initial state =
transverse ground state of guide 1 (2000 imaginary-time steps at dtau = 0.002
on the 256 x 256 plane) x a z Gaussian of width 4 at z0 = -30 moving with
k_z = 3; real-time Strang steps at dt = 0.002 with an observation (norm,
moments, guide populations) every 100 steps.  Storage complex64 with FP64
arithmetic (the fast mode); the complex128 mode is timed on the same input
for the c64-vs-c128 comparison and the accuracy of c64 is stated against it.

One "step" = one Strang step of the whole hot path.  The timed region covers
exactly --steps steps, bracketed by device synchronisation; the field is
resident in HBM before it starts.  Per-pass kernel times come from HIP
events that the library records around each pass launch on its own stream
during the timed region (ssf_set_timing); the dominant pass gives the
roofline entry.  The CPU baseline is the FP64 oracle on a bounded sample of
the same workload (a few full-grid steps).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid-point split-step updates/s + HBM GB/s vs roofline, c64 vs c128 at ≤1e-4 L2"


def initial_state(torch, ssf, cfg, dtype, device):
    """phi_1(x, y) (imaginary-time ground state of guide 1 alone at z0) times a
    moving z Gaussian, normalised on the grid."""
    import numpy as np
    g = cfg["grid"]
    gd = cfg["guides"]
    z0 = cfg["z0"]
    iz0 = int(round((z0 - g.lo[2]) / g.spacing(2)))
    s2 = ssf.Solver((g.n[0], g.n[1], 1), (g.lo[0], g.lo[1], 0.0), (g.hi[0], g.hi[1], 1.0), "c128", device=device)
    s2.set_guides(gd.v0[:1], gd.sigma[:1], gd.xc[0:1, iz0:iz0 + 1])
    x = torch.tensor(g.axis(0), dtype=torch.float64, device=device)
    y = torch.tensor(g.axis(1), dtype=torch.float64, device=device)
    xc = float(gd.xc[0, iz0])
    phi = torch.exp(-((x[None, :] - xc) ** 2 + y[:, None] ** 2) / (2 * 0.36)).to(torch.complex128)
    phi = phi.reshape(1, g.n[1], g.n[0]).contiguous()
    s2.step(phi, cfg["imag_steps"], cfg["dt"], imag=True)
    z = torch.tensor(g.axis(2), dtype=torch.float64, device=device)
    fz = torch.exp(-((z - z0) ** 2) / (2 * cfg["zwidth"] ** 2)).to(torch.complex128) * torch.exp(1j * cfg["kz"] * z)
    psi = (fz[:, None, None] * phi).contiguous()
    nrm = torch.sqrt(torch.sum(torch.abs(psi) ** 2) * g.dv)
    psi = (psi / nrm).to(dtype).contiguous()
    s2.close()
    return psi


def run_mode(torch, ssf, cfg, psi0, dtype, steps, warmup, obs_every, device):
    g = cfg["grid"]
    gd = cfg["guides"]
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=device)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    tiles, tune_us = s.tune(reps=10)          # tile autotuner (outside the timed region)
    s.tune_result = {"choice": tiles, "us": {"axis%d_variant%d" % k: v for k, v in tune_us.items()}}
    psi = psi0.to(s.tdtype).contiguous().clone()
    obs = s.obs_buffer(max(1, (steps + warmup) // obs_every))
    if warmup:
        s.step(psi, warmup, cfg["dt"], obs_every=obs_every, obs_buf=obs)
    torch.cuda.synchronize()
    s.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    s.step(psi, steps, cfg["dt"], obs_every=obs_every, obs_buf=obs)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    passes = s.timing_read()
    s.set_timing(False)
    nobs = steps // obs_every
    rec = s.read_obs(obs, nobs) if nobs else None
    return s, psi, ms, passes, rec


def cpu_baseline(cfg, sample_steps):
    """FP64 oracle on the host: `sample_steps` full-grid steps of the same workload."""
    import numpy as np
    import oracle
    import synth
    g = cfg["grid"]
    gd = cfg["guides"]
    rng = np.random.default_rng(0)
    psi = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, cfg["z0"]), width=(0.3, 0.3, cfg["zwidth"]),
                                k=(0.0, 0.0, cfg["kz"]))
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    oracle.step(psi, V, g.lo, g.hi, cfg["dt"], 1)          # warm-up (page-in, thread pool)
    t0 = time.perf_counter()
    oracle.step(psi, V, g.lo, g.hi, cfg["dt"], sample_steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores)
    del rng
    return {"value": g.points * sample_steps / dt, "unit": "updates/s", "cores": cores, "kind": "oracle",
            "sample": "%d Strang steps of the full %dx%dx%d grid (FP64, OpenMP over pencils), %.1f s"
                      % (sample_steps, g.n[0], g.n[1], g.n[2], dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--obs-every", type=int, default=100)
    ap.add_argument("--grid", type=str, default="256,256,512", help="Nx,Ny,Nz of the guide workload")
    ap.add_argument("--no-c128", action="store_true", help="skip the complex128 comparison run")
    ap.add_argument("--cpu-steps", type=int, default=3, help="oracle steps for the CPU baseline (0: skip)")
    ap.add_argument("--imag-steps", type=int, default=None,
                    help="imaginary-time steps of the transverse ground state (default: the workload's 2000)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain device copy of one field (for scaling profiler byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1309_2451_amd as ssf

    device = "cuda:0"
    n = tuple(int(v) for v in a.grid.split(","))
    cfg = synth.config2(n)
    if a.imag_steps is not None:
        cfg["imag_steps"] = a.imag_steps
    g = cfg["grid"]
    print("bench: building initial state on %s" % (g.n,), file=sys.stderr, flush=True)
    psi0 = initial_state(torch, ssf, cfg, torch.complex128, device)

    print("bench: c64 run, %d warmup + %d timed steps" % (a.warmup, a.steps), file=sys.stderr, flush=True)
    s64, psi64, ms64, pass64, rec64 = run_mode(torch, ssf, cfg, psi0, "c64", a.steps, a.warmup, a.obs_every, device)
    ups64 = g.points * a.steps / (ms64 * 1e-3)

    # roofline entry: dominant pass kind of the timed region
    esize = 8
    dom = max(pass64.items(), key=lambda kv: kv[1][0])
    dom_name, (dom_ms, dom_n) = dom
    avg_s = dom_ms * 1e-3 / max(dom_n, 1)
    bytes_per_launch = 2.0 * esize * g.points            # read + write psi once
    achieved = bytes_per_launch / avg_s / 1e9
    # whole-step algorithmic bandwidth: passes per step x 2 x esize x points
    launches = sum(c for _, c in pass64.values())
    step_gbs = launches * 2.0 * esize * g.points / (ms64 * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": ups64,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms64 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "three-guide CTAP %dx%dx%d, complex64 storage, FP64 arithmetic, dt=0.002, "
                               "observables every %d steps" % (g.n[0], g.n[1], g.n[2], a.obs_every),
                   "grid": list(g.n), "storage": "complex64", "arithmetic": "f64", "obs_every": a.obs_every},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dom_name,
                     "kernel_avg_us": avg_s * 1e6, "bytes_per_launch": bytes_per_launch},
        "step_algorithmic_gbs": step_gbs,
        "passes_per_step": launches / a.steps,
        "pass_times_ms": {k: {"total_ms": v[0], "launches": v[1]} for k, v in pass64.items()},
        "tiles": s64.tune_result,
    }
    if rec64 is not None and len(rec64):
        out["final_populations"] = [float(v) for v in rec64[-1]["pop"]]
        out["norm_drift"] = float(rec64[-1]["norm"] - 1.0)

    if not a.no_c128:
        print("bench: c128 run", file=sys.stderr, flush=True)
        s128, psi128, ms128, pass128, rec128 = run_mode(torch, ssf, cfg, psi0, "c128", a.steps, a.warmup,
                                                        a.obs_every, device)
        ups128 = g.points * a.steps / (ms128 * 1e-3)
        d = (psi64.to(torch.complex128) - psi128)
        relL2 = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(psi128))
        dom128 = max(pass128.items(), key=lambda kv: kv[1][0])
        avg128 = dom128[1][0] * 1e-3 / max(dom128[1][1], 1)
        out["c128"] = {"value": ups128, "ms_per_step": ms128 / a.steps,
                       "kernel": dom128[0], "kernel_avg_us": avg128 * 1e6,
                       "achieved_gbs": 2.0 * 16 * g.points / avg128 / 1e9}
        out["c64_speedup_vs_c128"] = ups64 / ups128
        out["c64_vs_c128_rel_l2"] = relL2
        out["c64_vs_c128_steps"] = a.steps + a.warmup
        s128.close()
    if a.calibrate_copy:
        # a plain copy of one complex64 field: 2 * 8 * points bytes of HBM traffic per launch
        src = psi64.contiguous()
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 2 * src.numel() * src.element_size()
    s64.close()

    if a.cpu_steps > 0:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
