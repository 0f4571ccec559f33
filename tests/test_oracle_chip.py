"""Pins of the oracle's atom-chip potential (Sec. III): the Biot-Savart field
of thin wires made of straight segments, the bias and offset fields, and the
longitudinal harmonic trap V_z.  Each check uses a fact that does not come
from the oracle's own formula: a numerical quadrature of the Biot-Savart
integrand, the infinite-wire field, the guide height r0 = mu0 I / (2 pi B_b)
printed in Sec. III, the harmonic trap frequency of a single-wire guide,
symmetry and additivity."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth

MU0 = 1.25663706212e-6                # vacuum permeability, CODATA 2018 (T m / A)


def _field(pts, paths, currents, b_bias=0.0, b_ip=0.0, L0=1e-6):
    return oracle.chip_field_points(pts, paths, currents, b_bias, b_ip, L0)


def test_segment_matches_quadrature_of_the_biot_savart_integrand():
    """An oblique segment (x and z components, as in the bends), field at
    points off its line: the closed form against adaptive quadrature of
    mu0 I / (4 pi) * integral of dl x (P - l) / |P - l|^3."""
    A, B = np.array([0.3, 0.0, -1.2]), np.array([1.7, 0.0, 2.5])
    I, L0 = 0.08, 1e-6
    rng = np.random.default_rng(1)
    pts = np.column_stack([rng.uniform(-3, 3, 6), rng.uniform(0.2, 3, 6), rng.uniform(-3, 4, 6)])
    got = _field(pts, [np.array([[A[0], A[2]], [B[0], B[2]]])], [I], L0=L0)
    Lv = B - A
    for p, g in zip(pts, got):
        ref = np.zeros(3)
        for c in range(3):
            def f(t, c=c):
                r = p - (A + t * Lv)
                return np.cross(Lv, r)[c] / np.linalg.norm(r) ** 3
            ref[c] = integrate.quad(f, 0.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)[0]
        ref *= MU0 * I / (4 * np.pi) / L0
        assert np.max(np.abs(g - ref)) < 1e-10 * np.max(np.abs(ref)), (p, g, ref)


def test_long_straight_wire_is_the_infinite_wire():
    """|B| = mu0 I / (2 pi rho), azimuthal (z x rho_hat for current along +z)."""
    I, L0 = 0.1, 1e-6
    wire = [np.array([[0.0, -1e7], [0.0, 1e7]])]
    pts = np.array([[0.5, 1.0, 0.0], [-2.0, 0.3, 100.0], [0.0, 1.43, -50.0], [3.0, 4.0, 7.0]])
    B = _field(pts, wire, [I], L0=L0)
    for p, b in zip(pts, B):
        rho = np.hypot(p[0], p[1])
        mag = MU0 * I / (2 * np.pi * rho * L0)
        direction = np.array([-p[1], p[0], 0.0]) / rho
        assert np.max(np.abs(b - mag * direction)) < 1e-11 * mag


def test_guide_height_under_a_bias_field():
    """Sec. III: a bias field B_b across the wire puts the field zero at
    r0 = mu0 I / (2 pi B_b) above it; there |B| is the offset field, so the
    potential (without V_z) is zero, and it rises around that point."""
    I, Bb, Bip, L0 = 0.1, 0.014, 0.03, 1e-6
    r0 = MU0 * I / (2 * np.pi * Bb) / L0
    assert abs(r0 - 1.4286) < 1e-3                      # ~1.43 um for the chip's numbers
    wire = [np.array([[1.5, -1e7], [1.5, 1e7]])]
    B = _field(np.array([[1.5, r0, 3.0]]), wire, [I], Bb, Bip, L0)[0]
    assert abs(B[0]) < 1e-12 * Bb and abs(B[1]) < 1e-12 * Bb and abs(B[2] - Bip) < 1e-15
    mu = 1000.0
    h = 1e-3
    cross = np.array([[1.5, r0, 3.0], [1.5 + h, r0, 3.0], [1.5 - h, r0, 3.0], [1.5, r0 + h, 3.0], [1.5, r0 - h, 3.0]])
    V = oracle.chip_potential_points(cross, wire, [I], Bb, Bip, L0, mu, 0.0, 0.0)
    assert abs(V[0]) < 1e-12 * mu * Bip
    assert np.all(V[1:] > V[0])


def test_single_wire_guide_trap_frequency():
    """Near the field zero |B| = sqrt(B_ip^2 + G^2 r^2) with G = 2 pi B_b^2 /
    (mu0 I), so V = mu (|B| - B_ip) has curvature omega^2 = mu G^2 / B_ip in
    every transverse direction (second differences at a small step)."""
    I, Bb, Bip, L0 = 0.1, 0.014, 0.03, 1e-6
    r0 = MU0 * I / (2 * np.pi * Bb) / L0
    G = 2 * np.pi * Bb ** 2 / (MU0 * I) * L0
    mu = 2766.0
    w2 = mu * G ** 2 / Bip
    wire = [np.array([[0.0, -1e7], [0.0, 1e7]])]
    h = 2e-3
    for d in (np.array([1.0, 0.0]), np.array([0.0, 1.0]), np.array([0.6, 0.8])):
        pts = np.array([[0.0, r0, 0.0], [h * d[0], r0 + h * d[1], 0.0], [-h * d[0], r0 - h * d[1], 0.0]])
        V = oracle.chip_potential_points(pts, wire, [I], Bb, Bip, L0, mu, 0.0, 0.0)
        curv = (V[1] - 2 * V[0] + V[2]) / h ** 2
        assert abs(curv - w2) < 1e-3 * w2, (d, curv, w2)
    # the synthetic workload's moment gives exactly the stated period through this formula
    u = synth.chip_units()
    m = synth.chip_moment_for_period(u, Bb, Bip, I, 0.2e-3)
    assert abs(np.sqrt(m * G ** 2 / Bip) - 2 * np.pi * u["t0"] / 0.2e-3) < 1e-12


def test_segment_additivity_and_direction():
    """Splitting a straight run into collinear pieces changes nothing;
    reversing a path and its current changes nothing."""
    L0 = 1e-6
    one = [np.array([[-1.0, -40.0], [2.0, 35.0]])]
    t = np.linspace(0, 1, 7)[:, None]
    many = [np.array([-1.0, -40.0]) + t * np.array([3.0, 75.0])]
    pts = np.array([[0.4, 0.9, 1.0], [-3.0, 2.0, -20.0], [5.0, 0.1, 30.0]])
    B1 = _field(pts, one, [0.05], L0=L0)
    B2 = _field(pts, many, [0.05], L0=L0)
    B3 = _field(pts, [one[0][::-1].copy()], [-0.05], L0=L0)
    assert np.max(np.abs(B1 - B2)) < 1e-13 * np.max(np.abs(B1))
    assert np.max(np.abs(B1 - B3)) < 1e-15 * np.max(np.abs(B1))


def test_mirror_symmetry_of_straight_wires():
    """Three straight parallel wires, equal outer currents, mirror-placed:
    V(x, y, z) = V(-x, y, z) on a grid symmetric about x = 0, and B_z = 0."""
    g = synth.Grid((16, 6, 5), (-8.0, 0.1, 0.0), (8.0, 3.1, 50.0))
    wires = [np.array([[-3.0, -1e6], [-3.0, 1e6]]), np.array([[0.0, -1e6], [0.0, 1e6]]),
             np.array([[3.0, -1e6], [3.0, 1e6]])]
    V = oracle.chip_potential(g.shape, g.lo, g.hi, wires, [0.1, 0.07, 0.1], 0.014, 0.03, 1e-6, 2766.0,
                              0.003, 25.0)
    assert np.max(np.abs(V[:, :, 1:] - V[:, :, :0:-1])) < 1e-12 * np.max(np.abs(V))
    x, y, z = g.mesh()
    pts = np.column_stack([x.ravel(), y.ravel(), z.ravel()])
    B = _field(pts, wires, [0.1, 0.07, 0.1], 0.014, 0.03)
    assert np.max(np.abs(B[:, 2] - 0.03)) < 1e-18


def test_bare_longitudinal_trap():
    """No current, no bias: V = omega_z^2 (z - z_c)^2 / 2 exactly."""
    g = synth.Grid((4, 3, 32), (-1.0, 0.5, 0.0), (1.0, 2.0, 1000.0))
    wires = [np.array([[0.0, -1e6], [0.0, 1e6]])]
    V = oracle.chip_potential(g.shape, g.lo, g.hi, wires, [0.0], 0.0, 0.03, 1e-6, 2766.0, 0.002976, 500.0)
    z = g.axis(2)[:, None, None]
    assert np.max(np.abs(V - 0.5 * 0.002976 ** 2 * (z - 500.0) ** 2)) < 1e-13


def test_grid_and_point_forms_agree():
    c = synth.config_chip(n=(16, 8, 32))
    g = c["grid"]
    args = (c["paths"], c["currents"], c["b_bias"], c["b_ip"], c["length_unit"], c["mu_over_e0"], c["omega_z"],
            c["z_c"])
    V = oracle.chip_potential(g.shape, g.lo, g.hi, *args)
    x, y, z = g.mesh()
    Vp = oracle.chip_potential_points(np.column_stack([x.ravel(), y.ravel(), z.ravel()]), *args)
    assert np.array_equal(V.ravel(), Vp)
