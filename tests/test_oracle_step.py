"""Pins of the oracle's split-operator step (real and imaginary time).

Closed forms used (none of them calls the oracle's FFT or step):
- A Gaussian stays Gaussian under every factor of a Strang step in a harmonic
  trap: the potential half-step adds to the quadratic coefficient, the kinetic
  factor is the exact free-particle propagator for a Gaussian.  Iterating these
  scalar maps gives the exact discrete-Strang state after n steps, which a
  spectrally resolved grid reproduces to ~1e-12.
- With V = 0 the Strang step is the exact free evolution: a periodised
  spreading Gaussian (image sum) and a plane wave exp(i k.x) with phase
  exp(-i n k^2 dt / 2) after n steps.
- Imaginary time: the Strang fixed point is exp(-a x^2/2) with
  a = omega sqrt(1 + omega^2 dtau^2 / 4), and the per-step norm ratio follows
  from the same scalar recursion.
- Brute force: a whole step on 8^3 with dense DFT matrices.
"""
import numpy as np
import pytest

import oracle
import synth


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# --- exact Gaussian recursion (per axis: psi = exp(-A x^2/2 + B x + C)) -------

def kick(A, B, C, h):
    """multiply by exp(-h x^2 / 2) (h complex: i w^2 dt/2 real time, w^2 dtau/2 imaginary)."""
    return A + h, B, C


def drift(A, B, C, tau):
    """free propagation exp(-i k^2 tau / 2); tau -> -i tau gives imaginary time."""
    d = 1.0 + 1j * A * tau
    return A / d, B / d, C + 1j * B * B * tau / (2.0 * d) - 0.5 * np.log(d)


def strang_real(A, B, C, omega, dt, n):
    h = 1j * omega ** 2 * dt / 2.0
    for _ in range(n):
        A, B, C = kick(A, B, C, h)
        A, B, C = drift(A, B, C, dt)
        A, B, C = kick(A, B, C, h)
    return A, B, C


def gauss_eval(grid, params):
    x, y, z = grid.mesh()
    r = (x, y, z)
    e = np.zeros(grid.shape, dtype=np.complex128)
    for a in range(3):
        A, B, C = params[a]
        e += -A * r[a] ** 2 / 2.0 + B * r[a] + C
    return np.exp(e)


def test_config1_harmonic_strang_closed_form():
    c = synth.config1()
    g = c["grid"]
    psi0 = c["psi0"]
    # the same state as three scalar Gaussians: exp(-(x-1)^2/2) exp(-y^2/2) exp(-z^2/2)
    p0 = [(1.0 + 0j, 1.0 + 0j, -0.5 + 0j), (1.0 + 0j, 0j, 0j), (1.0 + 0j, 0j, 0j)]
    scale = psi0.flat[0] / gauss_eval(g, p0).flat[0]
    psi, _ = oracle.step(psi0, c["V"], g.lo, g.hi, c["dt"], c["steps"])
    pn = [strang_real(*p, 1.0, c["dt"], c["steps"]) for p in p0]
    ref = scale * gauss_eval(g, pn)
    assert rel(psi, ref) < 2e-11
    obs = oracle.observables(psi, c["V"], g.lo, g.hi, -1.5, 1.5)
    theta = np.arccos(1.0 - c["dt"] ** 2 / 2.0)
    # <x>_n = cos(n theta) exactly for discrete Strang; continuum would give cos(1)
    assert abs(obs["mx"] - np.cos(200 * theta)) < 1e-11
    assert abs(obs["mx"] - 0.5403014293340861) < 1e-11
    assert abs(obs["norm"] - 1.0) < 1e-13


def test_anisotropic_harmonic_closed_form_catches_axis_swaps():
    g = synth.Grid((96, 48, 40), (-8.0, -7.0, -8.0), (8.0, 7.0, 8.0))
    om = (2.0, 1.5, 1.0)  # x resolved to k_max = 18.8, y to 10.8, z to 7.9
    V = synth.harmonic_table(g, om)
    p0 = [(1.3 + 0j, 0.4 + 0.3j, 0j), (1.1 + 0j, -0.2 + 0.5j, 0j), (0.9 + 0j, 0.1 - 0.4j, 0j)]
    psi0 = gauss_eval(g, p0)
    dt, n = 0.01, 40
    psi, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    ref = gauss_eval(g, [strang_real(*p0[a], om[a], dt, n) for a in range(3)])
    assert rel(psi, ref) < 1e-11


def test_free_gaussian_periodised_image_sum():
    g = synth.Grid((64, 64, 64), (-8.0, -6.0, -10.0), (8.0, 6.0, 10.0))  # k_max 12.6, 16.8, 10
    L = [g.hi[a] - g.lo[a] for a in range(3)]
    # per axis exp(-(r-c)^2/(2 w^2) + i k0 r)
    par = [(0.5, 0.8, 1.5), (-0.3, 0.7, -1.0), (1.0, 1.0, 0.7)]
    p0 = []
    for c_, w, k0 in par:
        A = 1.0 / w ** 2
        p0.append((A + 0j, c_ * A + 1j * k0, -c_ * c_ * A / 2.0 + 0j))
    psi0 = gauss_eval(g, p0)
    dt, n = 0.02, 25
    psi, _ = oracle.step(psi0, None, g.lo, g.hi, dt, n)
    t = dt * n
    pt = [drift(*p, t) for p in p0]
    x, y, z = g.mesh()
    r = (x, y, z)
    ref = np.ones(g.shape, dtype=np.complex128)
    for a in range(3):
        A, B, C = pt[a]
        s = np.zeros(g.shape, dtype=np.complex128)
        for m in range(-4, 5):
            rr = r[a] + m * L[a]
            s += np.exp(-A * rr ** 2 / 2 + B * rr + C)
        ref *= s
    assert rel(psi, ref) < 1e-12


def test_plane_wave_phase_after_1e4_steps():
    g = synth.Grid((8, 8, 8), (0.0, 0.0, 0.0), (2.0, 3.0, 5.0))
    m = (1, -2, 3)
    k = [2 * np.pi * m[a] / (g.hi[a] - g.lo[a]) for a in range(3)]
    x, y, z = g.mesh()
    psi0 = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z))
    n, dt = 10000, 0.003
    psi, _ = oracle.step(psi0, None, g.lo, g.hi, dt, n)
    ksq = sum(kk * kk for kk in k)
    ref = np.exp(-1j * ((n * ksq * dt / 2.0) % (2 * np.pi))) * psi0
    assert rel(psi, ref) < 1e-11


def test_bruteforce_step_8cubed_dense_dft():
    g = synth.Grid((8, 8, 8), (-3.0, -2.0, -4.0), (3.0, 2.0, 4.0))
    rng = np.random.default_rng(11)
    psi0 = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    V = rng.uniform(-5, 5, g.shape)
    dt = 0.037
    # dense DFT matrices and the k^2 grid written from the definitions
    def F(n):
        j = np.arange(n)
        return np.exp(-2j * np.pi * np.outer(j, j) / n)
    Fz, Fy, Fx = F(8), F(8), F(8)
    def kk(n, L):
        j = np.arange(n)
        return 2 * np.pi / L * np.where(j < n // 2, j, j - n)
    kx, ky, kz = (kk(8, g.hi[a] - g.lo[a]) for a in range(3))
    K2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    u = np.exp(-1j * V * dt / 2) * psi0
    uh = np.einsum("az,by,cx,zyx->abc", Fz, Fy, Fx, u)
    uh *= np.exp(-1j * K2 * dt / 2)
    u = np.einsum("az,by,cx,zyx->abc", Fz.conj(), Fy.conj(), Fx.conj(), uh) / 512
    ref = np.exp(-1j * V * dt / 2) * u
    got, _ = oracle.step(psi0, V, g.lo, g.hi, dt, 1)
    assert rel(got, ref) < 1e-14
    # the same for imaginary time (real factors, then renormalisation)
    u = np.exp(-V * dt / 2) * psi0
    uh = np.einsum("az,by,cx,zyx->abc", Fz, Fy, Fx, u) * np.exp(-K2 * dt / 2)
    u = np.exp(-V * dt / 2) * np.einsum("az,by,cx,zyx->abc", Fz.conj(), Fy.conj(), Fx.conj(), uh) / 512
    ref = u / np.sqrt(np.sum(np.abs(u) ** 2) * g.dv)
    got, _ = oracle.step(psi0, V, g.lo, g.hi, dt, 1, imag=True)
    assert rel(got, ref) < 1e-14


def test_real_time_norm_conservation_and_reversibility():
    g = synth.Grid((16, 12, 20), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    rng = np.random.default_rng(3)
    psi0 = synth.random_field(g, 3)
    V = rng.uniform(-10, 10, g.shape)
    psi, _ = oracle.step(psi0, V, g.lo, g.hi, 0.01, 50)
    assert abs(np.sum(np.abs(psi) ** 2) * g.dv - 1.0) < 1e-13
    back, _ = oracle.step(psi, V, g.lo, g.hi, -0.01, 50)
    assert rel(back, psi0) < 1e-13


# --- imaginary time ------------------------------------------------------------

def strang_imag_fixed_point(omega, dtau):
    h = omega ** 2 * dtau / 2.0
    a_star = np.sqrt(h * h + 2 * h / dtau)
    u = a_star + h
    return a_star, u


@pytest.mark.parametrize("omega", [1.0, 2.0])
def test_imag_time_fixed_point_1d(omega):
    # 1-D (ny = nz = 1) long run: the state converges to exp(-a* x^2/2) and the
    # per-step norm ratio to (1 + u dtau)^(-1/2)
    g = synth.Grid((64, 1, 1), (-8.0, 0.0, 0.0), (8.0, 1.0, 1.0))
    x = g.axis(0)
    V = (0.5 * omega ** 2 * x ** 2).reshape(g.shape)
    psi0 = synth.normalise(np.exp(-0.8 * x ** 2 / 2).reshape(g.shape) + 0j, g)
    dtau = 0.01
    psi, ed = oracle.step(psi0, V, g.lo, g.hi, dtau, 3000, imag=True)
    a_star, u = strang_imag_fixed_point(omega, dtau)
    ref = synth.normalise(np.exp(-a_star * x ** 2 / 2).reshape(g.shape) + 0j, g)
    assert rel(psi, ref) < 1e-12
    e_ref = 0.5 * np.log(1 + u * dtau) / dtau
    assert abs(ed[-1] - e_ref) < 1e-11
    assert abs(a_star - omega * np.sqrt(1 + omega ** 2 * dtau ** 2 / 4)) < 1e-15


def test_imag_time_3d_recursion_and_energy():
    g = synth.Grid((64, 64, 64), (-8.0, -8.0, -8.0), (8.0, 8.0, 8.0))
    V = synth.harmonic_table(g)
    psi0 = synth.gaussian_packet(g, width=(1.2, 0.9, 1.0))
    dtau, n = 0.005, 60
    psi, ed = oracle.step(psi0, V, g.lo, g.hi, dtau, n, imag=True)
    # scalar recursion with real factors; per-axis norm^2 of exp(-A x^2/2 + C)
    # is exp(2 Re C) sqrt(pi / Re A) for a resolved Gaussian
    p = [(1 / 1.2 ** 2 + 0j, 0j, 0j), (1 / 0.9 ** 2 + 0j, 0j, 0j), (1.0 + 0j, 0j, 0j)]
    h = dtau / 2.0
    lognorm = lambda q: sum(np.real(C) + 0.25 * np.log(np.pi / np.real(A)) for A, B, C in q)
    ed_ref = []
    for _ in range(n):
        before = lognorm(p)
        nxt = []
        for A, B, C in p:
            A, B, C = kick(A, B, C, h)
            A, B, C = drift(A, B, C, -1j * dtau)
            A, B, C = kick(A, B, C, h)
            nxt.append((A, B, C))
        p = nxt
        ed_ref.append(-(lognorm(p) - before) / dtau)
    ref = synth.normalise(gauss_eval(g, p), g)
    assert rel(psi, ref) < 1e-11
    assert np.max(np.abs(ed - np.array(ed_ref))) < 1e-9
    # <H> of the Strang fixed point exp(-a* r^2/2): a*/4 + 1/(4 a*) per axis
    a_star, u = strang_imag_fixed_point(1.0, dtau)
    gs = synth.normalise(np.exp(-a_star * (sum(r * r for r in g.mesh())) / 2) + 0j, g)
    obs = oracle.observables(gs, V, g.lo, g.hi, -1, 1)
    assert abs(obs["energy"] - 3 * (a_star / 4 + 1 / (4 * a_star))) < 1e-12
