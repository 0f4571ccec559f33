"""GPU accuracy targets at the workloads that define them, and error paths.

  * 256 x 256 x 512 guide transfer, 10^4 real-time steps (dt = 0.002,
    observations every 100 steps, tuned tiles, fused chain) from the workload's
    own initial state in complex64 and complex128 storage: complex64 within
    1e-4 relative L2 of complex128 and its norm within 1e-5 of 1.
  * The same grid in complex128 against the FP64 oracle for the first 200
    steps (observations at 100 and 200): 1e-12 relative L2.
  * 512^3 (seeded +-5 % guides) in complex128 against the oracle, 2 steps.
  * A non-finite field is reported as SSF_E_NONFINITE when its observation is
    read; misaligned field pointers are rejected with SSF_E_INVALID before
    anything is launched.

Oracle inputs are synth's seeded Gaussian packets, never GPU output.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ssf = pytest.importorskip("paper_1309_2451_amd")
from paper_1309_2451_amd import _ssf  # noqa: E402
from paper_1309_2451_amd.states import guide_transfer_state  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_dev(a, b):
    d = a.to(torch.complex128) - b.to(torch.complex128)
    return float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(b.to(torch.complex128)))


def _solver(cfg, dtype):
    g, gd = cfg["grid"], cfg["guides"]
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=DEV)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    return s


@pytest.mark.timeout(900)
def test_guide_transfer_ten_thousand_steps_c64_vs_c128():
    cfg = synth.config2()
    steps, every = 10000, 100
    say("256x256x512: initial state (%d imaginary-time steps on the transverse plane)" % cfg["imag_steps"])
    psi0 = guide_transfer_state(torch, cfg, DEV)
    out = {}
    for dtype in ("c128", "c64"):
        say("256x256x512 %s: %d steps, observations every %d" % (dtype, steps, every))
        s = _solver(cfg, dtype)
        s.tune(reps=3)
        psi = psi0.to(s.tdtype).contiguous().clone()
        rec = s.step(psi, steps, cfg["dt"], obs_every=every)
        out[dtype] = (psi, rec)
        s.close()
    l2 = rel_dev(out["c64"][0], out["c128"][0])
    r64, r128 = out["c64"][1], out["c128"][1]
    drift64 = float(r64[-1]["norm"] - 1.0)
    drift128 = float(r128[-1]["norm"] - 1.0)
    dp3 = abs(float(r64[-1]["pop"][2] - r128[-1]["pop"][2]))
    say("c64 vs c128 rel L2 %.3e, c64 norm drift %.3e, c128 norm drift %.3e, |dP3| %.3e"
        % (l2, drift64, drift128, dp3))
    assert len(r64) == len(r128) == steps // every
    assert l2 <= 1e-4
    assert abs(drift64) <= 1e-5
    assert abs(drift128) <= 1e-10
    assert dp3 <= 1e-6
    # every observation along the way: the two storage types track each other
    for a, b in zip(r64, r128):
        assert abs(a["norm"] - b["norm"]) <= 1e-5
        assert np.max(np.abs(a["pop"] - b["pop"])) <= 1e-5


@pytest.mark.timeout(1200)
def test_guide_transfer_first_200_steps_c128_vs_oracle():
    cfg = synth.config2()
    g, gd = cfg["grid"], cfg["guides"]
    psi0 = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, cfg["z0"]), width=(0.4, 0.4, cfg["zwidth"]),
                                 k=(0.0, 0.0, cfg["kz"]))
    say("256x256x512 c128: 200 steps on the GPU (observations every 100)")
    s = _solver(cfg, "c128")
    s.tune(reps=3)
    t = torch.from_numpy(psi0).to(DEV).contiguous()
    rec = s.step(t, 200, cfg["dt"], obs_every=100)
    got = t.cpu().numpy()
    del t
    s.close()
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref = psi0
    for k in range(2):
        say("oracle: steps %d..%d" % (100 * k + 1, 100 * (k + 1)))
        ref, _ = oracle.step(ref, V, g.lo, g.hi, cfg["dt"], 100)
        o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
        assert rec[k]["step"] == 100 * (k + 1)
        assert abs(rec[k]["norm"] - o["norm"]) < 1e-12
        for a, key in enumerate(("p1", "p2", "p3")):
            assert abs(rec[k]["pop"][a] - o[key]) < 1e-12, (k, key)
        for a, key in enumerate(("mx", "my", "mz")):
            assert abs(rec[k]["mean"][a] - o[key]) < 1e-11, (k, key)
    err = rel(got, ref)
    say("rel L2 after 200 steps", err)
    assert err < 1e-12
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.timeout(900)
def test_512_cube_c128_vs_oracle():
    cfg = synth.config3()
    g, gd = cfg["grid"], cfg["guides"]
    say("512^3 c128: building the packet")
    psi0 = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, cfg["z0"]), width=(0.4, 0.4, cfg["zwidth"]),
                                 k=(0.0, 0.0, cfg["kz"]))
    say("512^3 c128: 2 steps on the GPU")
    s = _solver(cfg, "c128")
    s.tune(reps=2)
    t = torch.from_numpy(psi0).to(DEV).contiguous()
    s.step(t, 2, cfg["dt"])
    got = t.cpu().numpy()
    del t
    s.close()
    torch.cuda.empty_cache()
    say("512^3: oracle, 2 steps")
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, cfg["dt"], 2)
    del V, psi0
    err = rel(got, ref)
    say("rel L2", err)
    assert err < 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_nonfinite_field_is_reported_at_read(dtype):
    say("non-finite field", dtype)
    g = synth.Grid((16, 12, 20), (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=DEV)
    s.set_potential_table(torch.from_numpy(synth.harmonic_table(g)).to(DEV))
    psi = torch.from_numpy(synth.gaussian_packet(g)).to(s.tdtype).to(DEV).contiguous()
    psi[3, 4, 5] = complex(float("nan"), 0.0)
    with pytest.raises(ssf.SSFError) as e:
        s.step(psi, 4, 0.01, obs_every=2)
    assert e.value.status == _ssf.SSF_E_NONFINITE
    with pytest.raises(ssf.SSFError) as e:
        s.observables(psi)
    assert e.value.status == _ssf.SSF_E_NONFINITE
    # a finite field on the same handle reads normally afterwards
    psi = torch.from_numpy(synth.gaussian_packet(g)).to(s.tdtype).to(DEV).contiguous()
    rec = s.step(psi, 4, 0.01, obs_every=2)
    assert rec[-1]["flags"] == 0 and abs(rec[-1]["norm"] - 1.0) < 1e-5
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_misaligned_field_pointer_is_rejected(dtype):
    """Field pointers must be aligned to the scalar size (8 B for complex128,
    4 B for complex64); the library checks before it launches anything."""
    say("misaligned pointers", dtype)
    g = synth.Grid((16, 12, 20), (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = ssf.Solver(g.n, g.lo, g.hi, dtype, device=DEV)
    buf = torch.zeros(2 * g.points + 64, dtype=torch.complex128, device=DEV)
    bad = ctypes.c_void_p(buf.data_ptr() + (4 if dtype == "c128" else 2))
    good = ctypes.c_void_p(buf.data_ptr() + 8 * g.points)
    lib = _ssf.load()
    obs = s.obs_buffer(1)
    ob = ctypes.c_void_p(obs.data_ptr())
    calls = [("ssf_step", (s.h, bad, 1, 0.01, 0, 0, None)),
             ("ssf_fft", (s.h, bad, 7, 0)),
             ("ssf_observables", (s.h, bad, ob)),
             ("ssf_copy", (s.h, bad, good)),
             ("ssf_copy", (s.h, good, bad)),
             ("ssf_density_xz", (s.h, bad, ob)),
             ("ssf_adjoint_init", (s.h, good, bad))]
    for name, args in calls:
        assert getattr(lib, name)(*args) == _ssf.SSF_E_INVALID, name
        assert b"aligned" in lib.ssf_last_error(), name
    torch.cuda.synchronize()
    assert torch.count_nonzero(buf) == 0           # nothing was written
    s.close()
