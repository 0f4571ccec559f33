"""Pins of the oracle's observables, guide potential, B-splines and adjoint.

- observables: closed-form moments and energies of resolved Gaussians and of
  harmonic-oscillator eigenstates; populations of states confined to a region;
- guide potential: an isolated guide has its minimum -v0 at its centre and the
  value -v0 exp(-1/2) one sigma away, symmetric in y;
- B-splines: partition of unity, exact reproduction of linear functions from
  Greville coefficients, local support;
- adjoint: central finite differences of the forward oracle (whose step is
  pinned in test_oracle_step.py), at two step sizes to see the O(h^2) error.
"""
import numpy as np
import pytest

import oracle
import synth


def test_observables_gaussian_moments_and_populations():
    g = synth.Grid((48, 40, 56), (-6.0, -5.0, -7.0), (6.0, 5.0, 7.0))
    psi = synth.gaussian_packet(g, centre=(1.0, -0.5, 2.0), width=(0.7, 0.8, 0.9), k=(1.0, 0, 0))
    o = oracle.observables(psi, None, g.lo, g.hi, -100.0, 100.0)
    assert abs(o["norm"] - 1.0) < 1e-13
    assert abs(o["mx"] - 1.0) < 1e-12 and abs(o["my"] + 0.5) < 1e-12 and abs(o["mz"] - 2.0) < 1e-12
    assert o["p1"] == 0.0 and o["p3"] == 0.0 and abs(o["p2"] - 1.0) < 1e-13
    # kinetic energy of this packet: sum_a (1/(4 w_a^2)) + k0^2/2
    ek = 1 / (4 * 0.49) + 1 / (4 * 0.64) + 1 / (4 * 0.81) + 0.5
    assert abs(o["energy"] - ek) < 1e-11
    # confined to x > 3: all population in P3; strict inequality at a grid point
    psi3 = synth.gaussian_packet(g, centre=(4.5, 0, 0), width=(0.25, 1, 1))
    o3 = oracle.observables(psi3, None, g.lo, g.hi, -1.0, 3.0)
    assert abs(o3["p3"] - 1.0) < 1e-12 and o3["p1"] < 1e-20
    # symmetric state (negligible at the unpaired edge point x = lo): P1 == P3
    psis = synth.gaussian_packet(g, centre=(0.0, 0, 0), width=(0.8, 1, 1))
    os_ = oracle.observables(psis, None, g.lo, g.hi, -1.0, 1.0)
    assert abs(os_["p1"] - os_["p3"]) < 1e-14
    assert abs(os_["p1"] + os_["p2"] + os_["p3"] - os_["norm"]) < 1e-14


def test_observables_harmonic_eigen_energies():
    g = synth.Grid((64, 64, 64), (-8.0, -8.0, -8.0), (8.0, 8.0, 8.0))
    V = synth.harmonic_table(g)
    x, y, z = g.mesh()
    g0 = np.exp(-(x * x + y * y + z * z) / 2) + 0j
    assert abs(oracle.observables(synth.normalise(g0, g), V, g.lo, g.hi, -1, 1)["energy"] - 1.5) < 1e-12
    e1 = synth.normalise(x * g0, g)
    assert abs(oracle.observables(e1, V, g.lo, g.hi, -1, 1)["energy"] - 2.5) < 1e-12
    e2 = synth.normalise(x * y * g0 * (1 + 0j), g)
    assert abs(oracle.observables(e2, V, g.lo, g.hi, -1, 1)["energy"] - 3.5) < 1e-12


def test_ctap_potential_special_cases():
    g = synth.Grid((64, 32, 4), (-16.0, -4.0, 0.0), (16.0, 4.0, 4.0))
    # guides 10 apart: each one isolated to exp(-50/0.72) ~ 1e-30
    xc = np.array([[-10.0] * 4, [0.0] * 4, [10.0] * 4])
    v0 = np.array([40.0, 30.0, 20.0])
    sig = np.array([0.6, 0.5, 1.0])
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, v0, sig, xc)
    xs = g.axis(0)
    ys = g.axis(1)
    iy0 = int(np.argmin(np.abs(ys)))
    assert ys[iy0] == 0.0
    for j, xcen in enumerate([-10.0, 0.0, 10.0]):
        ix = int(np.argmin(np.abs(xs - xcen)))
        assert xs[ix] == xcen
        assert abs(V[0, iy0, ix] + v0[j]) < 1e-12
    # one sigma away along x for guide 3 (sigma = 1, x = 11)
    ix = int(np.argmin(np.abs(xs - 11.0)))
    assert abs(V[0, iy0, ix] + 20.0 * np.exp(-0.5)) < 1e-12
    # y symmetry about the grid point y = 0 (y = -4 is the unpaired edge point)
    for iy in range(1, 16):
        assert np.allclose(V[:, iy0 + iy, :], V[:, iy0 - iy, :], rtol=0, atol=1e-13)


@pytest.mark.parametrize("M", [4, 7, 16])
def test_bspline_partition_of_unity_and_linear_precision(M):
    a, b = -48.0, 48.0
    z = np.linspace(a, b, 257)
    B = oracle.bspline_basis(M, a, b, z)
    assert np.allclose(B.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    assert np.all(B >= -1e-15)
    gv = synth.greville(M, a, b)
    assert np.allclose(B @ gv, z, rtol=0, atol=1e-12)
    # clamped ends
    assert abs(B[0, 0] - 1.0) < 1e-15 and abs(B[-1, -1] - 1.0) < 1e-15
    # local support: B_m vanishes outside [t_m, t_{m+4}]
    t = synth.bspline_knots(M, a, b)
    for m in range(M):
        out = (z < t[m]) | (z > t[m + 4])
        assert np.all(np.abs(B[out, m]) < 1e-15)


def _adjoint_case():
    g = synth.Grid((16, 12, 24), (-4.0, -3.0, -6.0), (4.0, 3.0, 6.0))
    z = g.axis(2)
    xc = np.stack([-1.3 + 0.2 * np.sin(0.7 * z), 0.05 * np.cos(z), 1.3 - 0.3 * np.exp(-z * z / 8)])
    v0 = np.array([8.0, 7.0, 9.0])
    sig = np.array([0.6, 0.55, 0.65])
    psi0 = synth.gaussian_packet(g, centre=(-1.0, 0.0, -1.0), width=(0.6, 0.6, 1.5), k=(0.5, 0, 1.0))
    return g, xc, v0, sig, psi0


def test_adjoint_matches_central_differences():
    g, xc, v0, sig, psi0 = _adjoint_case()
    dt, n, xhi = 0.02, 30, 0.6
    F, G, _ = oracle.adjoint_ctap(psi0, g.lo, g.hi, v0, sig, xc, dt, n, xhi)
    assert 1e-4 < F < 1.0

    def Fof(xcp):
        V = oracle.ctap_potential(g.shape, g.lo, g.hi, v0, sig, xcp)
        psi, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
        return oracle.observables(psi, None, g.lo, g.hi, -1e9, xhi)["p3"]

    assert abs(Fof(xc) - F) < 1e-15
    for (j, iz) in [(0, 11), (2, 9), (1, 12), (2, 15)]:
        errs = []
        for h in (2e-3, 1e-3):
            xp, xm = xc.copy(), xc.copy()
            xp[j, iz] += h
            xm[j, iz] -= h
            fd = (Fof(xp) - Fof(xm)) / (2 * h)
            errs.append(abs(fd - G[j, iz]))
        assert errs[1] < 1e-6 * max(1.0, abs(G[j, iz])) + 1e-10
        assert abs(G[j, iz]) > 1e-6
    # directional derivative along a random direction of all centres
    rng = np.random.default_rng(0)
    d = rng.standard_normal(xc.shape)
    h = 1e-4
    fd = (Fof(xc + h * d) - Fof(xc - h * d)) / (2 * h)
    assert abs(fd - np.sum(G * d)) < 1e-7 * max(1.0, abs(fd))


def test_observables_sums_are_exact_to_a_few_ulps_on_a_large_grid():
    """The observables are plain sums over every grid point; on a grid of
    2^22 points a running FP64 sum would be off by ~1e-14 relative or more.
    The oracle's sums must agree with the exactly rounded sums of the same
    products (math.fsum) to a few units in the last place."""
    import math
    g = synth.Grid((256, 128, 128), (-8.0, -8.0, -16.0), (8.0, 8.0, 16.0))
    rng = np.random.default_rng(11)
    psi = (rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)) * 1e-3
    V = rng.uniform(-40.0, 5.0, g.shape)
    x_lo, x_hi = -1.3, 2.1
    o = oracle.observables(psi, V, g.lo, g.hi, x_lo, x_hi)
    dv = np.prod([(h - l) / n for n, l, h in zip(g.n, g.lo, g.hi)])
    r = psi.real * psi.real + psi.imag * psi.imag
    x = g.axis(0)
    X = np.broadcast_to(x[None, None, :], g.shape)
    exact = {
        "norm": math.fsum(r.ravel()) * dv,
        "mx": math.fsum((X * r).ravel()) * dv,
        "p1": math.fsum(r[:, :, x < x_lo].ravel()) * dv,
        "p3": math.fsum(r[:, :, x > x_hi].ravel()) * dv,
        "p2": math.fsum(r[:, :, (x >= x_lo) & (x <= x_hi)].ravel()) * dv,
    }
    for key, val in exact.items():
        assert abs(o[key] - val) <= 4e-16 * abs(val), (key, o[key], val)
    # and the populations add up to the norm to the same accuracy
    assert abs(o["p1"] + o["p2"] + o["p3"] - o["norm"]) <= 1e-15 * o["norm"]
