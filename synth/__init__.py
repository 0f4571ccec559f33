"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds none of the split-operator arithmetic: it only lays out the
workloads (grid boxes and sizes, initial wavepackets, trap tables, the guide
centre profiles that describe where the three waveguides run) and draws the
seeded random parameters.  Both the FP64 oracle and the HIP library take what
it produces as plain arrays and numbers and evaluate the method themselves.

Physical setting: Morgan et al., arXiv:1309.2451, Sec. III (three waveguides
whose spacing varies along the propagation direction z, outer guides
approaching the middle one in the counter-intuitive order) and Sec. V (atom
starts in the left guide in its transverse ground state times a longitudinal
Gaussian and travels along +z).  Units are dimensionless (hbar = m = 1) and
the chip's magnetic guides are replaced by Gaussian wells, so that every input
here is a closed-form function of a few parameters.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import numpy as np


@dataclass(frozen=True)
class Grid:
    """Periodic box [lo, hi) per axis with n points; arrays are (nz, ny, nx)."""
    n: tuple          # (nx, ny, nz)
    lo: tuple         # (xlo, ylo, zlo)
    hi: tuple         # (xhi, yhi, zhi)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def points(self):
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])

    def spacing(self, a):
        return (self.hi[a] - self.lo[a]) / self.n[a]

    @property
    def dv(self):
        return self.spacing(0) * self.spacing(1) * self.spacing(2)

    def axis(self, a):
        """Sample positions lo + i*(hi-lo)/n, i = 0..n-1."""
        return self.lo[a] + np.arange(self.n[a], dtype=np.float64) * self.spacing(a)

    def mesh(self):
        z, y, x = np.meshgrid(self.axis(2), self.axis(1), self.axis(0), indexing="ij")
        return x, y, z


def normalise(psi, grid: Grid):
    """Scale so that sum |psi|^2 dV = 1 on the grid."""
    s = np.sqrt(np.sum(np.abs(psi) ** 2) * grid.dv)
    return psi / s


def gaussian_packet(grid: Grid, centre=(0.0, 0.0, 0.0), width=(1.0, 1.0, 1.0),
                    k=(0.0, 0.0, 0.0), normalised=True):
    """psi = prod_a exp(-(r_a - c_a)^2 / (2 w_a^2) + i k_a r_a), complex128."""
    x, y, z = grid.mesh()
    r = (x, y, z)
    e = np.zeros(grid.shape, dtype=np.complex128)
    for a in range(3):
        e += -((r[a] - centre[a]) ** 2) / (2.0 * width[a] ** 2) + 1j * k[a] * r[a]
    psi = np.exp(e)
    return normalise(psi, grid) if normalised else psi


def harmonic_table(grid: Grid, omega=(1.0, 1.0, 1.0)):
    """V = 1/2 sum_a omega_a^2 r_a^2 as a (nz, ny, nx) FP64 table."""
    x, y, z = grid.mesh()
    return 0.5 * (omega[0] ** 2 * x * x + omega[1] ** 2 * y * y + omega[2] ** 2 * z * z)


def random_field(grid: Grid, seed: int, smooth: float = 0.0):
    """Seeded complex128 field with N(0,1) real and imaginary parts, normalised.
    smooth > 0 multiplies by a Gaussian envelope of that width (in box units)
    so the field decays towards the box edges."""
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(grid.shape) + 1j * rng.standard_normal(grid.shape)
    if smooth > 0:
        x, y, z = grid.mesh()
        psi = psi * np.exp(-(x * x + y * y + z * z) / (2 * smooth * smooth))
    return normalise(psi, grid)


@dataclass
class Guides:
    """Three Gaussian waveguides: depth v0[j], width sigma[j], centre xc[j][z]."""
    v0: np.ndarray        # (3,)
    sigma: np.ndarray     # (3,)
    xc: np.ndarray        # (3, nz)
    x_lo: float           # left/middle partition boundary
    x_hi: float           # middle/right partition boundary


def bump(z, zc, w):
    return np.exp(-((z - zc) ** 2) / (2.0 * w * w))


def ctap_profile(z, d0, delta, z1, z3, wg):
    """Guide centres along z: x1 = -(d0 - delta g1), x2 = 0, x3 = +(d0 - delta g3)
    with Gaussian bumps g_j centred at z_j.  z3 < z1 puts the right pair first
    for motion towards +z (counter-intuitive order)."""
    x1 = -(d0 - delta * bump(z, z1, wg))
    x3 = +(d0 - delta * bump(z, z3, wg))
    return np.stack([x1, np.zeros_like(z), x3])


def midlines(xc):
    """Plane-dependent guide regions: the midlines between neighbouring guide
    centres, x_lo(z) = (x1 + x2)/2 and x_hi(z) = (x2 + x3)/2 for xc of shape
    (3, Nz)."""
    xc = np.asarray(xc, dtype=np.float64)
    return 0.5 * (xc[0] + xc[1]), 0.5 * (xc[1] + xc[2])


def ctap_guides(grid: Grid, d0=3.0, delta=1.2, v0=40.0, sigma=0.6, z1=6.0, z3=-6.0, wg=8.0,
                v0s=None, sigmas=None):
    z = grid.axis(2)
    xc = ctap_profile(z, d0, delta, z1, z3, wg)
    v = np.full(3, v0) if v0s is None else np.asarray(v0s, dtype=np.float64)
    s = np.full(3, sigma) if sigmas is None else np.asarray(sigmas, dtype=np.float64)
    return Guides(v0=v, sigma=s, xc=np.ascontiguousarray(xc), x_lo=-d0 / 2.0, x_hi=d0 / 2.0)


# ---------------------------------------------------------------------------
# Clamped uniform cubic B-spline coefficients (guide-centre parameterisation).
# ---------------------------------------------------------------------------

def bspline_knots(M, a, b):
    """Clamped uniform cubic knot vector over [a, b] with M basis functions."""
    nseg = M - 3
    inner = a + (b - a) * np.arange(1, nseg) / nseg
    return np.concatenate([[a] * 4, inner, [b] * 4])


def greville(M, a, b):
    """Knot averages (t_{m+1} + t_{m+2} + t_{m+3}) / 3: sampling a smooth profile
    there gives B-spline coefficients that reproduce it to second order."""
    t = bspline_knots(M, a, b)
    return np.array([(t[m + 1] + t[m + 2] + t[m + 3]) / 3.0 for m in range(M)])


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

BOX8 = (-8.0, 8.0)


def config1():
    """Harmonic trap, 64^3 on [-8,8)^3, complex128, Gaussian displaced by 1 along
    x, 200 real-time steps at dt = 0.005."""
    g = Grid((64, 64, 64), (-8.0, -8.0, -8.0), (8.0, 8.0, 8.0))
    psi0 = gaussian_packet(g, centre=(1.0, 0.0, 0.0))
    V = harmonic_table(g)
    return dict(name="harmonic 64^3", grid=g, psi0=psi0, V=V, dt=0.005, steps=200)


def config2(n=(256, 256, 512), intuitive=False, v0=40.0, sigma=0.6, d0=3.0, delta=1.2):
    """Three-guide CTAP, 256 x 256 x 512 on [-8,8)^2 x [-64,64), 10^4 real steps
    at dt = 0.002, z packet at z0 = -30 (width 4) moving with k_z = 3.
    intuitive=True swaps the bumps (the 1-2 pair approaches first).  The guide
    parameters default to the workload's (v0 = 40, sigma = 0.6, d0 = 3,
    delta = 1.2), where the wells barely couple."""
    g = Grid(tuple(n), (-8.0, -8.0, -64.0), (8.0, 8.0, 64.0))
    kw = dict(v0=v0, sigma=sigma, d0=d0, delta=delta)
    guides = ctap_guides(g, z1=-6.0, z3=6.0, **kw) if intuitive else ctap_guides(g, **kw)
    return dict(name="ctap %dx%dx%d" % tuple(n), grid=g, guides=guides, dt=0.002,
                steps=10000, imag_steps=2000, z0=-30.0, zwidth=4.0, kz=3.0)


def config3(n=(512, 512, 512)):
    """512^3 CTAP with seeded +-5 % perturbations of v0 and sigma per guide."""
    rng = np.random.default_rng(3)
    v0s, sig = np.empty(3), np.empty(3)
    for j in range(3):
        v0s[j] = 40.0 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0))
        sig[j] = 0.6 * (1.0 + 0.05 * rng.uniform(-1.0, 1.0))
    g = Grid(tuple(n), (-8.0, -8.0, -64.0), (8.0, 8.0, 64.0))
    guides = ctap_guides(g, v0s=v0s, sigmas=sig)
    return dict(name="ctap %dx%dx%d" % tuple(n), grid=g, guides=guides, dt=0.002,
                steps=5000, imag_steps=500, z0=-30.0, zwidth=4.0, kz=3.0)


BATCH_SIZES = ((96, 96, 96), (128, 128, 128), (128, 128, 256), (160, 160, 160))


def config4(count=96):
    """Batched sweep: per instance a grid size from BATCH_SIZES and
    d0 ~ U[2.5,3.5], delta ~ U[0.8,1.6], k_z ~ U[2,4] (seed 4)."""
    rng = np.random.default_rng(4)
    inst = []
    for _ in range(count):
        si = int(rng.integers(4))
        d0 = float(rng.uniform(2.5, 3.5))
        de = float(rng.uniform(0.8, 1.6))
        kz = float(rng.uniform(2.0, 4.0))
        n = BATCH_SIZES[si]
        g = Grid(n, (-8.0, -8.0, -28.0), (8.0, 8.0, 28.0))
        guides = ctap_guides(g, d0=d0, delta=de, z1=4.0, z3=-4.0, wg=4.0)
        inst.append(dict(grid=g, guides=guides, d0=d0, delta=de, kz=kz, z0=-16.0, zwidth=4.0))
    return dict(name="batched sweep", instances=inst, dt=0.004, steps=2000)


def config5(n=(128, 128, 256), M=16):
    """Gradient workload: guide centres x1(z), x3(z) as M cubic B-splines each,
    coefficients from the nominal profile at the Greville points plus
    0.05 N(0,1) (seed 5, x1 then x3)."""
    g = Grid(tuple(n), (-8.0, -8.0, -48.0), (8.0, 8.0, 48.0))
    a, b = g.lo[2], g.hi[2]
    zg = greville(M, a, b)
    prof = ctap_profile(zg, 3.0, 1.2, 6.0, -6.0, 8.0)
    rng = np.random.default_rng(5)
    c1 = prof[0] + 0.05 * rng.standard_normal(M)
    c3 = prof[2] + 0.05 * rng.standard_normal(M)
    return dict(name="gradient %dx%dx%d" % tuple(n), grid=g, M=M, zrange=(a, b),
                coeffs=np.stack([c1, c3]), v0=np.full(3, 40.0), sigma=np.full(3, 0.6),
                x_lo=-1.5, x_hi=1.5, dt=0.004, steps=4000, ckpt_every=64,
                z0=-24.0, zwidth=4.0, kz=3.0)


# ---------------------------------------------------------------------------
# Atom chip (Sec. III): three thin wires on the chip surface, a bias field
# across them, an offset field along them, a 6Li atom and a longitudinal
# harmonic trap.  Only parameters and geometry here; the field and the
# potential are computed by the oracle and by the library.
# ---------------------------------------------------------------------------

HBAR = 1.054571817e-34           # J s (CODATA 2018)
ATOMIC_MASS = 1.66053906660e-27  # kg
MASS_LI6 = 6.0151228874 * ATOMIC_MASS
MU_B = 9.2740100783e-24          # J / T; 6Li |F=3/2, m_F=3/2>: g_F m_F = 1


def chip_units(length_unit=1e-6, mass=MASS_LI6, moment=MU_B):
    """hbar = m = 1 units with lengths in `length_unit` metres: time unit
    t0 = m L0^2 / hbar (s), energy unit e0 = hbar / t0 (J), and the magnetic
    moment in energy units per tesla."""
    t0 = mass * length_unit ** 2 / HBAR
    e0 = HBAR / t0
    return dict(length_unit=length_unit, t0=t0, e0=e0, mu_over_e0=moment / e0)


def chip_separation(z, z_close, sep0=7.0, sep_min=4.3, bend=700.0):
    """Distance of an outer wire from the middle one along z: sep0 far away,
    sep_min at z_close, a raised-cosine approach and retreat over `bend`."""
    u = (np.asarray(z, dtype=np.float64) - (z_close - 0.5 * bend)) / bend
    c = np.where((u > 0.0) & (u < 1.0), 0.5 * (1.0 - np.cos(2.0 * np.pi * u)), 0.0)
    return sep0 - (sep0 - sep_min) * c


def chip_wire_paths(sep0=7.0, sep_min=4.3, xi=50.0, z_mid=500.0, bend=700.0, ds=1.0, ext=1.0e5,
                    zlen=1000.0, intuitive=False):
    """Polylines (k, 2) of (x, z) in micrometres for the left, middle and right
    wires.  The middle wire runs straight along x = 0.  The outer wires run at
    -/+ sep0 and approach the middle one to sep_min; the left wire stays
    straight for xi longer, so the right pair comes closest first
    (counter-intuitive order for an atom moving towards +z); intuitive=True
    swaps the two.  Straight ends continue to z = -ext and z = zlen + ext, so
    both ends of the simulated box see the same straight, evenly spaced wires."""
    z_right = z_mid - 0.5 * xi
    z_left = z_mid + 0.5 * xi
    if intuitive:
        z_right, z_left = z_left, z_right
    paths = []
    for sign, zc in ((-1.0, z_left), (None, None), (+1.0, z_right)):
        if sign is None:
            paths.append(np.array([[0.0, -ext], [0.0, zlen + ext]]))
            continue
        z0, z1 = zc - 0.5 * bend, zc + 0.5 * bend
        zb = np.linspace(z0, z1, int(round(bend / ds)) + 1)
        xb = sign * chip_separation(zb, zc, sep0, sep_min, bend)
        pts = np.concatenate([[[sign * sep0, -ext]], np.stack([xb, zb], axis=1), [[sign * sep0, zlen + ext]]])
        paths.append(pts)
    return paths


def chip_wire_x(paths, z):
    """(3, len(z)) x positions of the wires in the planes z (linear along each polyline)."""
    return np.stack([np.interp(z, p[:, 1], p[:, 0]) for p in paths])


MU0 = 1.25663706212e-6           # T m / A (CODATA 2018)


def chip_moment_for_period(units, b_bias=0.014, b_ip=0.03, current=0.1, period=0.2e-3):
    """Magnetic moment over the energy unit (per tesla) that gives an isolated
    straight-wire guide the transverse trap period `period` (s) in the harmonic
    approximation: a wire with current I under a bias B_b has its field zero
    at r0 = mu0 I / (2 pi B_b), where the transverse field grows with gradient
    G = 2 pi B_b^2 / (mu0 I); with the offset field B_ip the energy rises as
    mu G^2 r^2 / (2 B_ip), so omega^2 = (mu/E0) G^2 / B_ip in units with
    hbar = m = 1."""
    G = 2.0 * np.pi * b_bias ** 2 / (MU0 * current) * units["length_unit"]   # tesla per length unit
    omega = 2.0 * np.pi * units["t0"] / period
    return omega ** 2 * b_ip / G ** 2


def config_chip(i_mid=0.07, n=(256, 64, 1024), intuitive=False, i_outer=0.1, height=8.0):
    """The three-wire 6Li atom chip of Secs. III and V: chip area 20 um x
    1000 um (x, z), wires 7 um apart approaching to 4.3 um, left wire
    straight 50 um longer, B_b = 0.014 T, B_ip = 0.03 T, currents
    I_L = I_R = 0.1 A and I_M, longitudinal trap 2 pi x 5 Hz centred at
    z = 500 um, dt = 1e-6 s for half a trap period (0.1 s, 10^5 steps), on the
    stated 256 x 64 x 1024 points.
    Grid: x in [-10, 10) um, y from half a spacing above the chip surface (so
    no grid point lies on a wire) up to `height` um, z in [0, 1000) um.  The
    stated height is 4 um; with the moment scaled to the stated transverse
    period (below) the potential above a guide rises only to ~5 energy units
    at 4 um against a ground state at ~3.2, so in a 4 um periodic box the
    state reaches the top and wraps onto the chip surface (V ~ 10^3 there),
    which pumps energy into it; 8 um keeps the guides' states inside."""
    u = chip_units()
    dy = float(height) / n[1]
    g = Grid(tuple(n), (-10.0, 0.5 * dy, 0.0), (10.0, float(height) + 0.5 * dy, 1000.0))
    paths = chip_wire_paths(intuitive=intuitive)
    omega_z = 2.0 * np.pi * 5.0 * u["t0"]
    dt = 1.0e-6 / u["t0"]
    steps = int(round(0.1 / 1.0e-6))
    xw = chip_wire_x(paths, g.axis(2))
    # the stated fields give an isolated guide a ~270 kHz trap with the bare
    # moment of 6Li, against the stated ~0.2 ms transverse period: the moment
    # is scaled to the stated period (fields, currents and geometry unchanged)
    mu = chip_moment_for_period(u, 0.014, 0.03, i_outer, 0.2e-3)
    return dict(name="atom chip %dx%dx%d I_M=%g" % (tuple(n) + (i_mid,)), grid=g, paths=paths,
                currents=np.array([i_outer, i_mid, i_outer]), b_bias=0.014, b_ip=0.03,
                length_unit=u["length_unit"], mu_over_e0=mu, mu_over_e0_bare=u["mu_over_e0"],
                omega_z=omega_z, z_c=500.0,
                units=u, dt=dt, steps=steps, z0=16.0, zwidth=4.0,
                x_lo=0.5 * (xw[0] + xw[1]), x_hi=0.5 * (xw[1] + xw[2]), wire_x=xw)


def chip_sweep_currents():
    """Middle-wire currents of the Fig. 6 sweep: 0.0672 A upwards in steps
    of 0.001 A, ten values (0.0672 ... 0.0762 A)."""
    return [round(0.0672 + 0.001 * k, 4) for k in range(10)]
