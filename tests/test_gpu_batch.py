"""GPU parity of the batched path (many instances, grouped by grid, graph replay).

Each instance of a batch must evolve exactly as the same instance stepped
alone by a single handle whose chain is broken at the same steps (the batch
breaks it at every chunk boundary, a single handle at every observation), so
fields are compared bitwise; the batch observations come from a separate
reduction and are compared to the single-handle ones at FP64 rounding level.
One small instance is also checked against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ssf = pytest.importorskip("paper_1309_2451_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _instances():
    """Five instances on two grids with different guide geometries and partitions."""
    out = []
    specs = [((32, 24, 40), 2.0, 0.6, 2.0), ((32, 24, 40), 2.4, 0.8, 2.5), ((48, 32, 64), 2.2, 0.5, 1.5),
             ((32, 24, 40), 1.8, 0.7, 3.0), ((48, 32, 64), 2.6, 0.9, 2.0)]
    for i, (n, d0, de, kz) in enumerate(specs):
        g = synth.Grid(n, (-5.0, -4.0, -12.0), (5.0, 4.0, 12.0))
        gd = synth.ctap_guides(g, d0=d0, delta=de, v0=10.0 + i, sigma=0.55 + 0.05 * i, z1=2.0, z3=-2.0, wg=3.0)
        psi = synth.gaussian_packet(g, centre=(-d0 / 2 - 0.2, 0.0, -5.0), width=(0.5, 0.5, 2.0), k=(0.0, 0.0, kz))
        out.append((g, gd, psi))
    return out


def _batch(inst, dtype):
    return ssf.Batch([(g.n, g.lo, g.hi) for g, _, _ in inst], [(gd.v0, gd.sigma, gd.xc) for _, gd, _ in inst],
                     [gd.x_lo for _, gd, _ in inst], [gd.x_hi for _, gd, _ in inst], dtype=dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_matches_single_handles(dtype):
    inst = _instances()
    b = _batch(inst, dtype)
    ng, gof = b.groups()
    assert ng == 2 and list(gof) == [0, 0, 1, 0, 1]
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    dt, chunk = 0.01, 4
    for rnd, nsteps in enumerate((12, 8)):            # second call: new fields, fewer steps, graph reused
        say("batch vs single", dtype, "call", rnd, "nsteps", nsteps)
        fields = [torch.from_numpy(p).to(tdt).to(DEV).contiguous() for _, _, p in inst]
        refs = [f.clone() for f in fields]
        obs = b.obs_buffer()
        b.run(fields, nsteps, dt, chunk=chunk, obs_buf=obs)
        rec = b.read_obs(obs)
        for i, (g, gd, _) in enumerate(inst):
            s = ssf.Solver(g.n, g.lo, g.hi, dtype)
            s.set_guides(gd.v0, gd.sigma, gd.xc)
            s.set_partition(gd.x_lo, gd.x_hi)
            o = s.step(refs[i], nsteps, dt, obs_every=chunk)
            torch.cuda.synchronize()
            assert torch.equal(fields[i], refs[i]), "instance %d differs from its single-handle run" % i
            r = rec[i]
            assert r["step"] == nsteps and r["flags"] == 0
            for key in ("norm", "epot"):
                assert abs(r[key] - o[-1][key]) < 1e-12 * max(1.0, abs(o[-1][key])), (i, key)
            assert np.allclose(r["pop"], o[-1]["pop"], rtol=0, atol=1e-12), i
            assert np.allclose(r["mean"], o[-1]["mean"], rtol=0, atol=1e-11), i
            s.close()
    b.close()


def test_batch_vs_oracle_and_remainder():
    """nsteps not a multiple of the chunk (eager remainder, then replays), c128
    against the oracle; a second dt rebuilds the graph."""
    inst = _instances()[:3]
    b = _batch(inst, "c128")
    for dt, nsteps, chunk in ((0.01, 11, 4), (0.005, 9, 3)):
        say("batch vs oracle dt", dt, "nsteps", nsteps, "chunk", chunk)
        fields = [torch.from_numpy(p).to(DEV).contiguous() for _, _, p in inst]
        obs = b.obs_buffer()
        b.run(fields, nsteps, dt, chunk=chunk, obs_buf=obs)
        rec = b.read_obs(obs)
        for i, (g, gd, psi) in enumerate(inst):
            V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
            ref, _ = oracle.step(psi, V, g.lo, g.hi, dt, nsteps)
            got = fields[i].cpu().numpy()
            assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12, i
            o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
            assert abs(rec[i]["norm"] - o["norm"]) < 1e-12
            for a, key in enumerate(("p1", "p2", "p3")):
                assert abs(rec[i]["pop"][a] - o[key]) < 1e-12, (i, key)
    b.close()


def test_batch_tuned_and_zero_steps():
    inst = _instances()
    b = _batch(inst, "c64")
    b.tune(reps=2)
    fields = [torch.from_numpy(p).to(torch.complex64).to(DEV).contiguous() for _, _, p in inst]
    before = [f.clone() for f in fields]
    obs = b.obs_buffer()
    b.run(fields, 0, 0.01, chunk=5, obs_buf=obs)          # observation only
    rec = b.read_obs(obs)
    for i in range(len(inst)):
        assert torch.equal(fields[i], before[i])
        g = inst[i][0]
        nrm = float(torch.sum(torch.abs(before[i].to(torch.complex128)) ** 2).item() * g.dv)
        assert abs(rec[i]["norm"] - nrm) < 1e-12
    b.run(fields, 10, 0.01, chunk=5, obs_buf=obs)
    rec = b.read_obs(obs)
    assert all(abs(r["norm"] - 1.0) < 1e-5 for r in rec)
    with pytest.raises(ssf.SSFError):
        b.run(fields, 10, 0.0, chunk=5)
    b.close()


def test_batch_single_instance_ragged_grid_and_errors():
    """One instance on a grid whose lengths need radix-3/5 plans and ragged
    tiles, c128 against the oracle; invalid descriptions are rejected."""
    g = synth.Grid((24, 20, 40), (-4.0, -3.0, -8.0), (4.0, 3.0, 8.0))
    gd = synth.ctap_guides(g, d0=2.0, delta=0.6, v0=12.0, sigma=0.6, z1=2.0, z3=-2.0, wg=3.0)
    psi = synth.gaussian_packet(g, centre=(-2.0, 0.0, -3.0), width=(0.5, 0.5, 1.5), k=(0.0, 0.0, 2.0))
    b = ssf.Batch([(g.n, g.lo, g.hi)], [(gd.v0, gd.sigma, gd.xc)], [gd.x_lo], [gd.x_hi], dtype="c128")
    assert b.groups()[0] == 1
    f = [torch.from_numpy(psi).to(DEV).contiguous()]
    obs = b.obs_buffer()
    b.run(f, 13, 0.01, chunk=5, obs_buf=obs)
    rec = b.read_obs(obs)
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref, _ = oracle.step(psi, V, g.lo, g.hi, 0.01, 13)
    assert np.linalg.norm(f[0].cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-12
    o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
    assert abs(rec[0]["pop"][2] - o["p3"]) < 1e-12 and abs(rec[0]["norm"] - o["norm"]) < 1e-12
    b.close()
    with pytest.raises(ssf.SSFError):
        ssf.Batch([(g.n, g.lo, g.hi)], [(gd.v0, gd.sigma, gd.xc)], [1.0], [-1.0], dtype="c64")
    with pytest.raises(ssf.SSFError):
        ssf.Batch([(g.n, g.lo, g.hi)], [(gd.v0, (0.6, -1.0, 0.6), gd.xc)], [gd.x_lo], [gd.x_hi], dtype="c64")
    with pytest.raises(ssf.SSFError):
        ssf.Batch([((24, 20, 7), g.lo, g.hi)], [(gd.v0, gd.sigma, np.zeros((3, 7)))], [0.0], [0.0], dtype="c64")


def test_batch_sweep_full_size_instances_vs_oracle():
    """One instance of each grid size of the 96-instance sweep (seeded) at its
    full size, run as one batch in complex128 for 6 steps in chunks of 4
    (a remainder of 2 run eagerly, then one graph replay), against
    the oracle instance by instance."""
    cfg = synth.config4()
    picked, seen = [], set()
    for it in cfg["instances"]:
        if it["grid"].n not in seen:
            seen.add(it["grid"].n)
            picked.append(it)
    inst = []
    for it in picked:
        g, gd = it["grid"], it["guides"]
        psi = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, it["z0"]), width=(0.5, 0.5, it["zwidth"]),
                                    k=(0.0, 0.0, it["kz"]))
        inst.append((g, gd, psi))
    b = _batch(inst, "c128")
    assert b.groups()[0] == len(inst)
    fields = [torch.from_numpy(p).to(DEV).contiguous() for _, _, p in inst]
    obs = b.obs_buffer()
    dt = cfg["dt"]
    b.run(fields, 6, dt, chunk=4, obs_buf=obs)
    rec = b.read_obs(obs)
    for i, (g, gd, psi) in enumerate(inst):
        say("sweep instance", g.n)
        V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
        ref, _ = oracle.step(psi, V, g.lo, g.hi, dt, 6)
        assert np.linalg.norm(fields[i].cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-12, g.n
        o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
        assert abs(rec[i]["norm"] - o["norm"]) < 1e-12
        assert abs(rec[i]["pop"][0] - o["p1"]) < 1e-12
    b.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_two_runs_on_a_side_stream_without_host_sync(dtype):
    """Two runs with different field lists enqueued back to back on a side
    stream, no host synchronisation between them: the second run's
    descriptor upload must wait for the first run's graph replays, so each
    field list evolves exactly as on single handles."""
    inst = _instances()
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    dt, chunk = 0.01, 4
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b = _batch(inst, dtype)
        fa = [torch.from_numpy(p).to(tdt).to(DEV).contiguous() for _, _, p in inst]
        fb = [torch.from_numpy(p).to(tdt).to(DEV).contiguous() * 0.5 for _, _, p in inst]
        ra = [f.clone() for f in fa]
        rb = [f.clone() for f in fb]
        say("side stream: run A (40 steps), run B (12 steps)", dtype)
        b.run(fa, 40, dt, chunk=chunk)
        b.run(fb, 12, dt, chunk=chunk)
    side.synchronize()
    for i, (g, gd, _) in enumerate(inst):
        s = ssf.Solver(g.n, g.lo, g.hi, dtype)
        s.set_guides(gd.v0, gd.sigma, gd.xc)
        s.set_partition(gd.x_lo, gd.x_hi)
        s.step(ra[i], 40, dt, obs_every=chunk)
        s.step(rb[i], 12, dt, obs_every=chunk)
        torch.cuda.synchronize()
        assert torch.equal(fa[i], ra[i]), "run A, instance %d" % i
        assert torch.equal(fb[i], rb[i]), "run B, instance %d" % i
        s.close()
    b.close()
