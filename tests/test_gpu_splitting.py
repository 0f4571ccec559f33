"""GPU parity of the T/2 - V - T/2 ordering (ssf_set_splitting) against the
oracle's ordering of the same name, through the C ABI.  Tolerances as in
test_gpu_parity: c128 1e-12 relative L2; c64 3 x 6e-8 sqrt(passes)."""
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


def to_dev(a, solver):
    return torch.from_numpy(np.ascontiguousarray(a)).to(solver.tdtype).to(DEV).contiguous()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tvt_random_field_table_potential(dtype, fuse):
    say("tvt table", dtype, "fuse", fuse)
    g = synth.Grid((40, 12, 20), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    rng = np.random.default_rng(21)
    psi0 = synth.random_field(g, 21, smooth=2.0)
    V = rng.uniform(-10, 10, g.shape)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_splitting("tvt")
    s.set_fusion(fuse)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    s.set_partition(-1.0, 0.5)
    t = to_dev(psi0, s)
    dt, n = 0.013, 23
    obs = s.step(t, n, dt, obs_every=5)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n, order="tvt")
    tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(8 * n)
    assert rel(host(t), ref) < tol
    ref_psi = psi0
    for k in range(len(obs)):
        ref_psi, _ = oracle.step(ref_psi, V, g.lo, g.hi, dt, 5, order="tvt")
        o = oracle.observables(ref_psi, V, g.lo, g.hi, -1.0, 0.5)
        assert obs[k]["step"] == 5 * (k + 1)
        for a, key in enumerate(("p1", "p2", "p3")):
            assert abs(obs[k]["pop"][a] - o[key]) < (1e-12 if dtype == "c128" else 1e-6)
    # the orderings agree to second order, not exactly
    vtv, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    assert rel(ref, vtv) > 1e-6
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tvt_guide_potential(dtype):
    """Guide potential (the lean fused x pass with the short phase series)."""
    say("tvt guides", dtype)
    g = synth.Grid((32, 24, 64), (-5.0, -4.0, -16.0), (5.0, 4.0, 16.0))
    gd = synth.ctap_guides(g, d0=2.0, delta=0.6, v0=12.0, sigma=0.6, z1=2.0, z3=-2.0, wg=3.0)
    psi0 = synth.gaussian_packet(g, centre=(-2.0, 0.0, -6.0), width=(0.5, 0.5, 2.0), k=(0.0, 0.0, 2.0))
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_splitting("tvt")
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    t = to_dev(psi0, s)
    for dt in (0.005, 0.02):                      # |V dt| below 0.1, then above
        t.copy_(to_dev(psi0, s))
        n = 30
        obs = s.step(t, n, dt, obs_every=15)
        V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
        ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n, order="tvt")
        tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(5 * n)
        assert rel(host(t), ref) < tol, dt
        o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
        assert abs(obs[-1]["pop"][2] - o["p3"]) < (1e-12 if dtype == "c128" else 1e-6)
    s.close()


def test_tvt_restrictions_and_switch_back():
    g = synth.Grid((16, 12, 20), (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    V = synth.harmonic_table(g)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    psi0 = synth.gaussian_packet(g, centre=(0.5, 0.0, 0.0))
    t = to_dev(psi0, s)
    s.set_splitting("tvt")
    with pytest.raises(ssf.SSFError):
        s.step(t, 3, 0.01, imag=True)
    with pytest.raises(ssf.SSFError):
        s.step_ckpt(t, 4, 0.01, 2, s.empty(2))
    s.set_splitting("vtv")
    s.step(t, 7, 0.01)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, 0.01, 7)
    assert rel(host(t), ref) < 1e-12
    s.close()
