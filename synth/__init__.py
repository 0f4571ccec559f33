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


def config2(n=(256, 256, 512), intuitive=False):
    """Three-guide CTAP, 256 x 256 x 512 on [-8,8)^2 x [-64,64), 10^4 real steps
    at dt = 0.002, z packet at z0 = -30 (width 4) moving with k_z = 3.
    intuitive=True swaps the bumps (the 1-2 pair approaches first)."""
    g = Grid(tuple(n), (-8.0, -8.0, -64.0), (8.0, 8.0, 64.0))
    guides = ctap_guides(g, z1=-6.0, z3=6.0) if intuitive else ctap_guides(g)
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
