"""GPU parity of the plane-dependent guide populations and the y-integrated
x-z density (Sec. V, Figs. 4 and 5) against the oracle, through the C ABI."""
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


def _case(intuitive=False):
    g = synth.Grid((32, 24, 64), (-5.0, -4.0, -16.0), (5.0, 4.0, 16.0))
    z1, z3 = (-2.0, 2.0) if intuitive else (2.0, -2.0)
    gd = synth.ctap_guides(g, d0=1.6, delta=0.6, v0=12.0, sigma=0.7, z1=z1, z3=z3, wg=3.0)
    psi0 = synth.gaussian_packet(g, centre=(-1.6, 0.0, -6.0), width=(0.7, 0.6, 2.0), k=(0.0, 0.0, 3.0))
    return g, gd, psi0


@pytest.mark.parametrize("intuitive", [False, True])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_time_resolved_midline_populations(dtype, intuitive):
    """P1..P3(t) with the midlines between the moving guides as boundaries,
    recorded every 10 steps during a fused run, against the oracle."""
    say("midline populations", dtype, "intuitive", intuitive)
    g, gd, psi0 = _case(intuitive)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    xl, xh = synth.midlines(gd.xc)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition_z(xl, xh)
    t = to_dev(psi0, s)
    dt, every, n = 0.01, 10, 60
    obs = s.step(t, n, dt, obs_every=every)
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref = psi0
    tol = 1e-12 if dtype == "c128" else 2e-6
    for k in range(n // every):
        ref, _ = oracle.step(ref, V, g.lo, g.hi, dt, every)
        p = oracle.populations_z(ref, g.lo, g.hi, xl, xh)
        assert np.allclose(obs[k]["pop"], p, rtol=0, atol=tol), (k, obs[k]["pop"], p)
    # the same state through ssf_observables, and the fixed partition again
    o = s.observables(t)
    assert np.allclose(o["pop"], obs[-1]["pop"], rtol=0, atol=1e-12 if dtype == "c128" else 1e-7)
    s.set_partition(gd.x_lo, gd.x_hi)
    o2 = s.observables(t)
    ref_fixed = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
    assert abs(o2["pop"][2] - ref_fixed["p3"]) < tol
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_density_xz_vs_oracle(dtype):
    say("density xz", dtype)
    g, gd, psi0 = _case()
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    t = to_dev(psi0, s)
    s.step(t, 25, 0.01)
    rho = s.density_xz(t).cpu().numpy()
    state = t.cpu().numpy().astype(np.complex128)
    ref = oracle.density_xz(state, g.lo, g.hi)
    assert rho.shape == (g.n[2], g.n[0])
    assert np.max(np.abs(rho - ref)) < 1e-13 * np.max(ref)
    # and against the oracle's own propagation
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    prop, _ = oracle.step(psi0.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi0,
                          V, g.lo, g.hi, 0.01, 25)
    assert rel(rho, oracle.density_xz(prop, g.lo, g.hi)) < (1e-12 if dtype == "c128" else 1e-5)
    s.close()


def test_adjoint_mask_uses_plane_boundaries():
    g, gd, psi0 = _case()
    xl, xh = synth.midlines(gd.xc)
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition_z(xl, xh)
    t = to_dev(psi0, s)
    lam = s.empty()
    s.adjoint_init(t, lam)
    x = g.axis(0)
    keep = x[None, :] > xh[:, None]                      # (Nz, Nx): x_i > x_hi(z)
    ref = psi0 * keep[:, None, :]
    assert np.array_equal(lam.cpu().numpy(), ref)
    with pytest.raises(ssf.SSFError):
        s.set_partition_z(xh, xl)                       # x_lo > x_hi somewhere
    s.close()
