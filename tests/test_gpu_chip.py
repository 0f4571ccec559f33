"""GPU parity of the atom-chip potential (Sec. III) and of steps and batches
that use it.

  * ssf_chip_potential on the paper's 256 x 64 x 1024 points (I_M = 0.07 A)
    against the oracle's Biot-Savart sum at 4096 seeded grid points; with no
    currents and no bias field it must reduce to the bare longitudinal trap
    everywhere (closed form).
  * Real-time steps with the chip table (fused chain, observations) against
    the oracle stepping its own chip potential, on a 80 x 24 x 96 cut of the
    chip (ragged tiles) in complex128 and complex64, and at the full paper
    grid in the launch configuration the benchmark uses.
  * A batch of chip instances (different middle-wire currents, two grids)
    against single-handle runs (bitwise) and, in complex128, the oracle.
Oracle inputs are synth's seeded packets and wire geometry, never GPU output.
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _chip_args(cfg):
    return (cfg["paths"], cfg["currents"], cfg["b_bias"], cfg["b_ip"], cfg["length_unit"], cfg["mu_over_e0"],
            cfg["omega_z"], cfg["z_c"])


def _oracle_V(cfg, g):
    return oracle.chip_potential(g.shape, g.lo, g.hi, *_chip_args(cfg))


def _cut(cfg, n=(80, 24, 96), zlo=440.0, zhi=560.0):
    """A smaller grid over the coupling region of the chip, same x and y box."""
    g0 = cfg["grid"]
    height = g0.hi[1] - g0.lo[1]
    dy = height / n[1]
    return synth.Grid(n, (g0.lo[0], 0.5 * dy, zlo), (g0.hi[0], height + 0.5 * dy, zhi))


def test_chip_potential_vs_oracle_at_sampled_points():
    cfg = synth.config_chip(i_mid=0.07)
    g = cfg["grid"]
    say("chip potential on", g.n)
    s = ssf.Solver(g.n, g.lo, g.hi, "c64", device=DEV)
    V = s.chip_potential(*_chip_args(cfg))
    torch.cuda.synchronize()
    Vh = V.cpu().numpy()
    s.close()
    rng = np.random.default_rng(31)
    idx = np.stack([rng.integers(0, g.n[2], 4096), rng.integers(0, g.n[1], 4096), rng.integers(0, g.n[0], 4096)], 1)
    # every corner and the planes of closest approach too
    idx = np.concatenate([idx, [[0, 0, 0], [g.n[2] - 1, g.n[1] - 1, g.n[0] - 1], [512, 20, 100], [512, 21, 128]]])
    x, y, z = g.axis(0), g.axis(1), g.axis(2)
    pts = np.stack([x[idx[:, 2]], y[idx[:, 1]], z[idx[:, 0]]], 1)
    ref = oracle.chip_potential_points(pts, *_chip_args(cfg))
    got = Vh[idx[:, 0], idx[:, 1], idx[:, 2]]
    err = np.abs(got - ref)
    say("max |dV| %.3e, max |V| %.3e" % (err.max(), np.abs(ref).max()))
    assert np.all(err <= 2e-12 + 2e-13 * np.abs(ref))
    assert np.all(np.isfinite(Vh))


def test_chip_potential_without_wires_is_the_bare_trap():
    cfg = synth.config_chip()
    g = _cut(cfg, (64, 16, 128), 0.0, 1000.0)
    s = ssf.Solver(g.n, g.lo, g.hi, "c128", device=DEV)
    V = s.chip_potential(cfg["paths"], [0.0, 0.0, 0.0], 0.0, cfg["b_ip"], cfg["length_unit"], cfg["mu_over_e0"],
                         cfg["omega_z"], cfg["z_c"]).cpu().numpy()
    s.close()
    zz = g.axis(2)[:, None, None]
    expect = np.broadcast_to(0.5 * cfg["omega_z"] ** 2 * (zz - cfg["z_c"]) ** 2, g.shape)
    assert np.max(np.abs(V - expect)) <= 1e-15 * np.max(expect)


def _packet(cfg, g, kz=1.0):
    # centred on the left guide's minimum near the chip (x ~ -3.8, y ~ 1.3)
    return synth.gaussian_packet(g, centre=(-3.8, 1.3, 0.5 * (g.lo[2] + g.hi[2]) - 20.0), width=(0.5, 0.5, 6.0),
                                 k=(0.0, 0.0, kz))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_chip_steps_vs_oracle(dtype):
    cfg = synth.config_chip(i_mid=0.07)
    g = _cut(cfg)
    say("chip steps", dtype, g.n)
    psi0 = _packet(cfg, g)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=DEV)
    V = s.chip_potential(*_chip_args(cfg))
    s.set_potential_table(V)
    s.set_partition(-1.8, 1.8)
    t = torch.from_numpy(psi0).to(s.tdtype).to(DEV).contiguous()
    steps, every, dt = 24, 8, cfg["dt"]
    rec = s.step(t, steps, dt, obs_every=every)
    got = t.cpu().numpy().astype(np.complex128)
    s.close()
    Vo = _oracle_V(cfg, g)
    ref = psi0
    for k in range(steps // every):
        ref, _ = oracle.step(ref, Vo, g.lo, g.hi, dt, every)
        o = oracle.observables(ref, Vo, g.lo, g.hi, -1.8, 1.8)
        tol = 1e-12 if dtype == "c128" else 1e-6
        assert abs(rec[k]["norm"] - o["norm"]) < tol
        assert np.max(np.abs(rec[k]["pop"] - [o["p1"], o["p2"], o["p3"]])) < tol
        assert np.max(np.abs(rec[k]["mean"] - [o["mx"], o["my"], o["mz"]])) < tol * 600
    err = rel(got, ref)
    say("rel L2", err)
    passes = 4 * steps + steps // every
    assert err < (1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(passes))


def test_chip_full_grid_c128_vs_oracle():
    """The paper's 256 x 64 x 1024 points in the benchmark's launch
    configuration (tuned tiles, fused chain), 3 steps with one observation."""
    cfg = synth.config_chip(i_mid=0.07)
    g = cfg["grid"]
    psi0 = synth.gaussian_packet(g, centre=(-6.64, 1.41, 60.0), width=(0.6, 0.6, 4.0), k=(0.0, 0.0, 1.0))
    say("chip full grid: GPU")
    s = ssf.Solver(g.n, g.lo, g.hi, "c128", device=DEV)
    V = s.chip_potential(*_chip_args(cfg))
    s.set_potential_table(V)
    s.set_partition(-3.5, 3.5)
    s.tune(reps=2)
    t = torch.from_numpy(psi0).to(DEV).contiguous()
    rec = s.step(t, 3, cfg["dt"], obs_every=3)
    got = t.cpu().numpy()
    del t, V
    s.close()
    say("chip full grid: oracle potential and steps")
    Vo = _oracle_V(cfg, g)
    ref, _ = oracle.step(psi0, Vo, g.lo, g.hi, cfg["dt"], 3)
    o = oracle.observables(ref, Vo, g.lo, g.hi, -3.5, 3.5)
    err = rel(got, ref)
    say("rel L2", err)
    assert err < 1e-12
    assert abs(rec[0]["norm"] - o["norm"]) < 1e-12
    assert np.max(np.abs(rec[0]["pop"] - [o["p1"], o["p2"], o["p3"]])) < 1e-12


def _chip_instances(cfg):
    out = []
    for n, i_mid in (((80, 24, 96), 0.0672), ((80, 24, 96), 0.0722), ((64, 16, 128), 0.0762)):
        c = dict(cfg)
        c["currents"] = np.array([cfg["currents"][0], i_mid, cfg["currents"][2]])
        g = _cut(cfg, n)
        out.append((g, c, _packet(cfg, g, kz=0.8 + 10 * (i_mid - 0.07))))
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_chip_batch_matches_single_handles(dtype):
    cfg = synth.config_chip()
    inst = _chip_instances(cfg)
    tabs = []
    for g, c, _ in inst:
        s = ssf.Solver(g.n, g.lo, g.hi, "c128", device=DEV)
        tabs.append(s.chip_potential(*_chip_args(c)))
        s.close()
    torch.cuda.synchronize()
    b = ssf.Batch([(g.n, g.lo, g.hi) for g, _, _ in inst], None, [-1.8] * 3, [1.8] * 3, dtype=dtype, tables=tabs)
    ng, gof = b.groups()
    assert ng == 2 and list(gof) == [0, 0, 1]
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    dt, chunk = cfg["dt"], 4
    for rnd, nsteps in enumerate((12, 6)):
        say("chip batch vs single", dtype, "call", rnd)
        fields = [torch.from_numpy(p).to(tdt).to(DEV).contiguous() for _, _, p in inst]
        refs = [f.clone() for f in fields]
        obs = b.obs_buffer()
        b.run(fields, nsteps, dt, chunk=chunk, obs_buf=obs)
        rec = b.read_obs(obs)
        for i, (g, c, _) in enumerate(inst):
            s = ssf.Solver(g.n, g.lo, g.hi, dtype)
            s.set_potential_table(tabs[i])
            s.set_partition(-1.8, 1.8)
            o = s.step(refs[i], nsteps, dt, obs_every=chunk if nsteps % chunk == 0 else nsteps)
            torch.cuda.synchronize()
            if nsteps % chunk == 0:
                assert torch.equal(fields[i], refs[i]), "instance %d differs from its single-handle run" % i
            else:
                d = (fields[i].to(torch.complex128) - refs[i].to(torch.complex128)).abs().max().item()
                assert d < (1e-13 if dtype == "c128" else 1e-6), (i, d)
            r = rec[i]
            assert r["step"] == nsteps and r["flags"] == 0
            for key in ("norm", "epot"):
                assert abs(r[key] - o[-1][key]) < (1e-12 if dtype == "c128" else 1e-6) * max(1.0, abs(o[-1][key]))
            assert np.allclose(r["pop"], o[-1]["pop"], rtol=0, atol=1e-12 if dtype == "c128" else 1e-6), i
            s.close()
    if dtype == "c128":
        say("chip batch vs oracle")
        fields = [torch.from_numpy(p).to(DEV).contiguous() for _, _, p in inst]
        b.run(fields, 10, dt, chunk=4)
        torch.cuda.synchronize()
        for i, (g, c, p) in enumerate(inst):
            ref, _ = oracle.step(p, _oracle_V(c, g), g.lo, g.hi, dt, 10)
            assert rel(fields[i].cpu().numpy(), ref) < 1e-12, i
    b.close()
