"""Pins of the oracle's plane-dependent guide populations and x-z density
(Sec. V, Figs. 4 and 5).

- constant boundaries reduce to the populations of ``observables`` (pinned in
  test_oracle_misc); brute force with explicit loops on a tiny grid; the three
  populations add up to the norm;
- the density of a separable state f(x) g(y) h(z) with a Gaussian g is
  |f|^2 |h|^2 sqrt(pi) w (the y-sum of a resolved Gaussian equals its integral
  to rounding); brute force on a tiny grid; its x-z sum is the norm.
"""
import numpy as np

import oracle
import synth


def test_populations_constant_boundaries_match_observables():
    g = synth.Grid((24, 12, 16), (-3.0, -2.0, -4.0), (3.0, 2.0, 4.0))
    psi = synth.random_field(g, 31, smooth=1.5)
    o = oracle.observables(psi, None, g.lo, g.hi, -0.7, 0.4)
    p = oracle.populations_z(psi, g.lo, g.hi, np.full(16, -0.7), np.full(16, 0.4))
    assert np.allclose(p, (o["p1"], o["p2"], o["p3"]), rtol=0, atol=1e-15)
    assert abs(sum(p) - o["norm"]) < 1e-14


def test_populations_bruteforce_tiny():
    g = synth.Grid((5, 3, 4), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(7)
    psi = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    xl = rng.uniform(-1.0, 0.0, 4)
    xh = rng.uniform(0.0, 1.0, 4)
    P = [0.0, 0.0, 0.0]
    dv = g.dv
    for z in range(4):
        for y in range(3):
            for x in range(5):
                xc = -1.0 + x * 2.0 / 5
                r = abs(psi[z, y, x]) ** 2 * dv
                if xc < xl[z]:
                    P[0] += r
                elif xc > xh[z]:
                    P[2] += r
                else:
                    P[1] += r
    assert np.allclose(oracle.populations_z(psi, g.lo, g.hi, xl, xh), P, rtol=1e-14, atol=0)


def test_density_xz_separable_gaussian_closed_form():
    g = synth.Grid((20, 64, 12), (-2.0, -8.0, -3.0), (2.0, 8.0, 3.0))
    x, y, z = g.mesh()
    w = 0.9
    f = np.cos(1.3 * x) + 0.2j * x
    h = np.exp(-z ** 2 / 3.0)
    psi = f * np.exp(-y ** 2 / (2 * w * w)) * h
    rho = oracle.density_xz(psi, g.lo, g.hi)
    ref = (np.abs(f[:, 0, :]) ** 2) * (np.abs(h[:, 0, :]) ** 2) * np.sqrt(np.pi) * w
    assert np.max(np.abs(rho - ref)) < 1e-13 * np.max(ref)
    norm = np.sum(np.abs(psi) ** 2) * g.dv
    assert abs(np.sum(rho) * g.spacing(0) * g.spacing(2) - norm) < 1e-12 * norm


def test_density_xz_bruteforce_tiny():
    g = synth.Grid((3, 4, 2), (0.0, -1.0, 0.0), (1.0, 1.0, 1.0))
    rng = np.random.default_rng(8)
    psi = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    dy = 2.0 / 4
    ref = np.zeros((2, 3))
    for z in range(2):
        for x in range(3):
            for y in range(4):
                ref[z, x] += abs(psi[z, y, x]) ** 2 * dy
    assert np.allclose(oracle.density_xz(psi, g.lo, g.hi), ref, rtol=1e-14, atol=0)
