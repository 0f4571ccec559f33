"""Pins of the oracle's second symmetric ordering, T/2 - V - T/2.

Sec. IV of the paper counts four Fourier transforms and three complex
multiplications per step, which is the ordering half kinetic step, full
potential step, half kinetic step taken one step at a time.  Pins (none of
them calls the oracle's FFT or step):
- brute force on 8^3 with dense DFT matrices (real and imaginary time);
- the exact discrete Gaussian recursion in a harmonic trap, the scalar maps
  applied in T/2 - V - T/2 order;
- the exact mean position and momentum of a displaced Gaussian: for a
  quadratic potential every factor of the step acts on (<x>, <p>) as a linear
  map, drift (x += p tau) and kick (p -= w^2 dt x), so
  (<x>, <p>)_n = M^n (x0, p0) with M = D(dt/2) K(dt) D(dt/2); both orderings
  share <x>_n = cos(n theta) for p0 = 0 but differ in <p>_n;
- with V = 0 both orderings are the exact free evolution (plane-wave phase);
- both orderings converge to the continuum coherent state at second order.
"""
import numpy as np
import pytest

import oracle
import synth


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def kick(A, B, C, h):
    return A + h, B, C


def drift(A, B, C, tau):
    d = 1.0 + 1j * A * tau
    return A / d, B / d, C + 1j * B * B * tau / (2.0 * d) - 0.5 * np.log(d)


def tvt_real(A, B, C, omega, dt, n):
    for _ in range(n):
        A, B, C = drift(A, B, C, dt / 2.0)
        A, B, C = kick(A, B, C, 1j * omega ** 2 * dt)
        A, B, C = drift(A, B, C, dt / 2.0)
    return A, B, C


def gauss_eval(grid, params):
    x, y, z = grid.mesh()
    r = (x, y, z)
    e = np.zeros(grid.shape, dtype=np.complex128)
    for a in range(3):
        A, B, C = params[a]
        e += -A * r[a] ** 2 / 2.0 + B * r[a] + C
    return np.exp(e)


def test_bruteforce_tvt_step_8cubed_dense_dft():
    g = synth.Grid((8, 8, 8), (-3.0, -2.0, -4.0), (3.0, 2.0, 4.0))
    rng = np.random.default_rng(12)
    psi0 = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    V = rng.uniform(-5, 5, g.shape)
    dt = 0.041

    def F(n):
        j = np.arange(n)
        return np.exp(-2j * np.pi * np.outer(j, j) / n)

    def kk(n, L):
        j = np.arange(n)
        return 2 * np.pi / L * np.where(j < n // 2, j, j - n)

    Fm = F(8)
    kx, ky, kz = (kk(8, g.hi[a] - g.lo[a]) for a in range(3))
    K2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2

    def fwd(u):
        return np.einsum("az,by,cx,zyx->abc", Fm, Fm, Fm, u)

    def inv(u):
        return np.einsum("az,by,cx,zyx->abc", Fm.conj(), Fm.conj(), Fm.conj(), u) / 512

    for imag in (False, True):
        f_t = np.exp(-K2 * dt / 4) if imag else np.exp(-1j * K2 * dt / 4)
        f_v = np.exp(-V * dt) if imag else np.exp(-1j * V * dt)
        u = inv(f_t * fwd(psi0))
        u = inv(f_t * fwd(f_v * u))
        if imag:
            u = u / np.sqrt(np.sum(np.abs(u) ** 2) * g.dv)
        got, _ = oracle.step(psi0, V, g.lo, g.hi, dt, 1, imag=imag, order="tvt")
        assert rel(got, u) < 1e-14, imag


def test_tvt_harmonic_gaussian_recursion():
    cfg = synth.config1()
    g, dt, n = cfg["grid"], cfg["dt"], cfg["steps"]
    p0 = [(1.0 + 0j, 1.0 + 0j, -0.5 + 0j), (1.0 + 0j, 0j, 0j), (1.0 + 0j, 0j, 0j)]
    pn = [tvt_real(*p, 1.0, dt, n) for p in p0]
    psi0 = gauss_eval(g, p0)
    ref = gauss_eval(g, pn)
    got, _ = oracle.step(psi0, cfg["V"], g.lo, g.hi, dt, n, order="tvt")
    assert rel(got, ref) < 1e-11


def _means(grid, psi):
    """<x> from the density and <p_x> from the momentum density (numpy FFT)."""
    x, _, _ = grid.mesh()
    rho = np.abs(psi) ** 2
    mx = np.sum(x * rho) / np.sum(rho)
    kx = 2 * np.pi * np.fft.fftfreq(grid.n[0], d=grid.spacing(0))
    ph = np.abs(np.fft.fft(psi, axis=2)) ** 2
    px = np.sum(kx[None, None, :] * ph) / np.sum(ph)
    return mx, px


def test_mean_position_and_momentum_both_orderings():
    g = synth.Grid((64, 16, 16), (-8.0, -4.0, -4.0), (8.0, 4.0, 4.0))
    omega, dt, n = 1.3, 0.05, 37
    V = synth.harmonic_table(g, omega=(omega, omega, omega))
    psi0 = synth.gaussian_packet(g, centre=(1.2, 0.0, 0.0), width=(0.8, 0.8, 0.8))

    def D(t):
        return np.array([[1.0, t], [0.0, 1.0]])

    def K(c):
        return np.array([[1.0, 0.0], [-c, 1.0]])

    w2 = omega ** 2
    maps = {"vtv": K(w2 * dt / 2) @ D(dt) @ K(w2 * dt / 2), "tvt": D(dt / 2) @ K(w2 * dt) @ D(dt / 2)}
    theta = np.arccos(1.0 - w2 * dt * dt / 2.0)
    res = {}
    for order, M in maps.items():
        psi, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n, order=order)
        mx, px = _means(g, psi)
        x_n, p_n = np.linalg.matrix_power(M, n) @ np.array([1.2, 0.0])
        assert abs(mx - x_n) < 1e-10, order
        assert abs(px - p_n) < 1e-10, order
        assert abs(x_n - 1.2 * np.cos(n * theta)) < 1e-12
        res[order] = p_n
    assert abs(res["vtv"] - res["tvt"]) > 1e-3       # the orderings are distinguishable


def test_tvt_free_plane_wave_phase():
    g = synth.Grid((16, 8, 12), (0.0, 0.0, 0.0), (2 * np.pi, 2 * np.pi, 2 * np.pi))
    x, y, z = g.mesh()
    k = (3.0, -2.0, 1.0)
    psi0 = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    dt, n = 0.013, 2000
    psi, _ = oracle.step(psi0, None, g.lo, g.hi, dt, n, order="tvt")
    ksq = sum(kk * kk for kk in k)
    assert rel(psi, np.exp(-1j * ((n * ksq * dt / 2.0) % (2 * np.pi))) * psi0) < 1e-11


@pytest.mark.parametrize("order", ["vtv", "tvt"])
def test_second_order_convergence_to_coherent_state(order):
    """Harmonic oscillator, Gaussian displaced by 1: error at t = 1 against the
    continuum coherent state falls by 4 when dt halves."""
    g = synth.Grid((64, 64, 64), (-8.0, -8.0, -8.0), (8.0, 8.0, 8.0))
    V = synth.harmonic_table(g)
    psi0 = synth.gaussian_packet(g, centre=(1.0, 0.0, 0.0))
    x, y, z = g.mesh()
    t = 1.0
    q, p = np.cos(t), -np.sin(t)
    exact = np.pi ** -0.75 * np.exp(-((x - q) ** 2 + y ** 2 + z ** 2) / 2 + 1j * p * x - 1j * p * q / 2 - 1.5j * t)
    errs = []
    for nsteps in (25, 50):
        psi, _ = oracle.step(psi0, V, g.lo, g.hi, t / nsteps, nsteps, order=order)
        errs.append(rel(psi, exact))
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4, (errs, ratio)
