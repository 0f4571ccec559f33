"""FP64 CPU oracle for the Fourier split-operator propagation (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the HIP library and its Python binding) never imports, links or calls it, and
the two share no code: this package wraps ``ssf_oracle.c`` (plain C, FP64),
compiled with gcc into ``liboracle.so`` next to it.

Method: Morgan et al., "Coherent transport by adiabatic passage on atom chips"
(arXiv:1309.2451), Sec. IV (Fourier split-operator method, p_max = pi N / L)
and Sec. V (numerical transverse ground state, guide populations).  The C file
header lists the conventions.

Parity status of each function (what pins it is in ``tests/test_oracle_*.py``):
  fft1d / fft3d / fft_axis   pinned: brute-force DFT matrices, numpy.fft, Parseval
  step (real time)           pinned: brute-force 8^3 step with dense DFT matrices,
                             exact discrete-Strang Gaussian recursion (harmonic
                             trap), periodised free-Gaussian closed form, plane-wave
                             phase after 10^4 steps, norm conservation
  step (imaginary time)      pinned: Strang fixed-point Gaussian width and per-step
                             norm ratio (closed forms)
  step, order "tvt"          pinned: brute-force 8^3 T/2-V-T/2 step, exact discrete
                             mean position and momentum of a displaced Gaussian in a
                             harmonic trap (both orders: same <x>, different <p>),
                             free-particle identity with "vtv", second-order
                             convergence of both orders to the continuum coherent state
  observables                pinned: closed-form moments of Gaussians, <H> of
                             harmonic-oscillator eigenstates
  populations_z              pinned: constant boundaries reduce to observables'
                             populations, brute force on a tiny grid, P1+P2+P3 = norm
  density_xz                 pinned: closed-form Gaussian y-integral of a separable
                             state, brute force on a tiny grid, total = norm
  ctap_potential             pinned: special cases (isolated guide minimum -v0,
                             value one sigma off-centre, y-symmetry)
  bspline_basis              pinned: partition of unity, linear precision with
                             Greville coefficients, support and endpoint values
  adjoint_ctap               pinned: central finite differences of the forward
                             oracle (O(h^2) check at two step sizes)
  chip_field_points /        pinned: infinite straight wire mu0 I / (2 pi rho), the
  chip_potential(_points)    guide height r0 = mu0 I / (2 pi B_b) of a wire under a
                             bias field (Sec. III), segment additivity, mirror
                             symmetry of straight wires, the harmonic transverse
                             frequency of a single-wire guide, the bare V_z trap
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ssf_oracle.c with gcc (FP64, OpenMP over independent pencils)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_fft1d.argtypes = [dp, ctypes.c_int, ctypes.c_int]
        lib.orc_fft3d.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_fft_axis.argtypes = [dp] + [ctypes.c_int] * 5
        lib.orc_kgrid.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        lib.orc_step.argtypes = [dp, dp, ip, dp, dp, ctypes.c_double, ctypes.c_long,
                                 ctypes.c_int, dp]
        lib.orc_step_order.argtypes = [dp, dp, ip, dp, dp, ctypes.c_double, ctypes.c_long,
                                       ctypes.c_int, dp, ctypes.c_int]
        lib.orc_observables.argtypes = [dp, dp, ip, dp, dp, ctypes.c_double,
                                        ctypes.c_double, dp]
        lib.orc_ctap_potential.argtypes = [dp, ip, dp, dp, ctypes.c_int, dp, dp, dp]
        lib.orc_populations_z.argtypes = [dp, ip, dp, dp, dp, dp, dp]
        lib.orc_density_xz.argtypes = [dp, ip, dp, dp, dp]
        lib.orc_bspline_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                          dp, ctypes.c_int, dp]
        lib.orc_adjoint_ctap.argtypes = [dp, ip, dp, dp, ctypes.c_int, dp, dp, dp,
                                         ctypes.c_double, ctypes.c_long, ctypes.c_double,
                                         dp, dp, dp]
        chip = [ctypes.c_int, ip, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.orc_chip_potential_points.argtypes = [dp, dp, ctypes.c_long] + chip + [ctypes.c_double] * 3
        lib.orc_chip_potential.argtypes = [dp, ip, dp, dp] + chip + [ctypes.c_double] * 3
        lib.orc_chip_field_points.argtypes = [dp, dp, ctypes.c_long] + chip
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _wires(paths, currents):
    """(nwires, npts int array, concatenated (x, z) path array, currents) for the C side."""
    paths = [np.ascontiguousarray(p, dtype=np.float64).reshape(-1, 2) for p in paths]
    npts = np.array([p.shape[0] for p in paths], dtype=np.int32)
    flat = np.ascontiguousarray(np.concatenate([p.ravel() for p in paths]))
    cur = np.ascontiguousarray(currents, dtype=np.float64)
    assert cur.shape == (len(paths),) and np.all(npts >= 2)
    return len(paths), npts, flat, cur


def chip_field_points(pts, paths, currents, b_bias, b_ip, length_unit):
    """Magnetic field (tesla), shape (m, 3), of thin wires along the polylines
    `paths` (each (k, 2): x, z in the chip plane y = 0) with `currents`, plus
    b_bias along +x and b_ip along +z, at points pts (m, 3) = (x, y, z)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    nw, npts, flat, cur = _wires(paths, currents)
    out = np.zeros((pts.shape[0], 3))
    _load().orc_chip_field_points(_dp(out), _dp(pts), pts.shape[0], nw,
                                  npts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(flat), _dp(cur),
                                  float(b_bias), float(b_ip), float(length_unit))
    return out


def chip_potential_points(pts, paths, currents, b_bias, b_ip, length_unit, mu_over_e0, omega_z, z_c):
    """Atom-chip potential mu_over_e0 (|B| - b_ip) + omega_z^2 (z - z_c)^2 / 2 at points (m, 3)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    nw, npts, flat, cur = _wires(paths, currents)
    out = np.zeros(pts.shape[0])
    _load().orc_chip_potential_points(_dp(out), _dp(pts), pts.shape[0], nw,
                                      npts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(flat), _dp(cur),
                                      float(b_bias), float(b_ip), float(length_unit), float(mu_over_e0),
                                      float(omega_z), float(z_c))
    return out


def chip_potential(shape_zyx, lo, hi, paths, currents, b_bias, b_ip, length_unit, mu_over_e0, omega_z, z_c):
    """The atom-chip potential on a (nz, ny, nx) grid."""
    n, lo, hi = _grid_from(shape_zyx, lo, hi)
    nw, npts, flat, cur = _wires(paths, currents)
    V = np.zeros(tuple(shape_zyx))
    _load().orc_chip_potential(_dp(V), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(lo), _dp(hi), nw,
                               npts.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(flat), _dp(cur),
                               float(b_bias), float(b_ip), float(length_unit), float(mu_over_e0), float(omega_z),
                               float(z_c))
    return V


def threads():
    """Threads the oracle's parallel loops use (results do not depend on it)."""
    return int(_load().orc_threads())


def set_threads(n):
    _load().orc_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _grid_args(n, lo, hi):
    n = np.ascontiguousarray(n, dtype=np.int32)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    assert n.shape == (3,) and lo.shape == (3,) and hi.shape == (3,)
    return n, lo, hi


def _c128(psi, shape=None):
    a = np.ascontiguousarray(psi, dtype=np.complex128).copy()
    if shape is not None:
        assert a.shape == tuple(shape), (a.shape, shape)
    return a


def _as_dp_complex(a):
    return a.view(np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def fft1d(x, sign=-1):
    """Unnormalised 1-D DFT with kernel exp(sign 2 pi i j k / n)."""
    a = _c128(x)
    _load().orc_fft1d(_as_dp_complex(a), a.shape[0], int(sign))
    return a


def fft3d(psi, direction=-1):
    """3-D DFT of a (nz, ny, nx) array: forward unnormalised (direction -1) or
    inverse scaled by 1/N (direction +1)."""
    a = _c128(psi)
    nz, ny, nx = a.shape
    _load().orc_fft3d(_as_dp_complex(a), nx, ny, nz, int(direction))
    return a


def fft_axis(psi, axis, sign=-1):
    """Unnormalised 1-D DFT along one axis (0 = x, 1 = y, 2 = z) of (nz, ny, nx)."""
    a = _c128(psi)
    nz, ny, nx = a.shape
    _load().orc_fft_axis(_as_dp_complex(a), nx, ny, nz, int(axis), int(sign))
    return a


def kgrid(n, L):
    k = np.empty(n, dtype=np.float64)
    _load().orc_kgrid(n, float(L), _dp(k))
    return k


def _grid_from(shape_zyx, lo, hi):
    nz, ny, nx = shape_zyx
    return _grid_args([nx, ny, nz], lo, hi)


def step(psi, V, lo, hi, dt, nsteps, imag=False, order="vtv"):
    """nsteps Strang steps, order "vtv" (V/2-T-V/2) or "tvt" (T/2-V-T/2).
    Returns (psi, edecay) where edecay is the per-step -ln(norm ratio)/dt in
    imaginary time (None in real time)."""
    a = _c128(psi)
    n, lo, hi = _grid_from(a.shape, lo, hi)
    Va = None if V is None else np.ascontiguousarray(V, dtype=np.float64)
    if Va is not None:
        assert Va.shape == a.shape
    ed = np.zeros(max(int(nsteps), 1), dtype=np.float64) if imag else None
    _load().orc_step_order(_as_dp_complex(a), _dp(Va), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                           _dp(lo), _dp(hi), float(dt), int(nsteps), 1 if imag else 0, _dp(ed),
                           {"vtv": 0, "tvt": 1}[order])
    return a, (ed[:int(nsteps)] if imag else None)


OBS_FIELDS = ("norm", "mx", "my", "mz", "p1", "p2", "p3", "energy")


def observables(psi, V, lo, hi, x_lo, x_hi):
    """Dict of norm, first moments (unnormalised), guide populations and <H>."""
    a = _c128(psi)
    n, lo, hi = _grid_from(a.shape, lo, hi)
    Va = None if V is None else np.ascontiguousarray(V, dtype=np.float64)
    out = np.zeros(8, dtype=np.float64)
    _load().orc_observables(_as_dp_complex(a), _dp(Va),
                            n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(lo), _dp(hi),
                            float(x_lo), float(x_hi), _dp(out))
    return dict(zip(OBS_FIELDS, out.tolist()))


def populations_z(psi, lo, hi, x_lo, x_hi):
    """(P1, P2, P3) with plane-dependent boundaries x_lo[z], x_hi[z] (length Nz)."""
    a = _c128(psi)
    n, lo, hi = _grid_from(a.shape, lo, hi)
    xl = np.ascontiguousarray(x_lo, dtype=np.float64)
    xh = np.ascontiguousarray(x_hi, dtype=np.float64)
    assert xl.shape == (a.shape[0],) and xh.shape == (a.shape[0],)
    out = np.zeros(3, dtype=np.float64)
    _load().orc_populations_z(_as_dp_complex(a), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(lo), _dp(hi),
                              _dp(xl), _dp(xh), _dp(out))
    return tuple(out.tolist())


def density_xz(psi, lo, hi):
    """(Nz, Nx) density integrated over y: sum_y |psi|^2 dy."""
    a = _c128(psi)
    n, lo, hi = _grid_from(a.shape, lo, hi)
    out = np.zeros((a.shape[0], a.shape[2]), dtype=np.float64)
    _load().orc_density_xz(_as_dp_complex(a), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(lo), _dp(hi),
                           _dp(out))
    return out


def ctap_potential(shape_zyx, lo, hi, v0, sigma, xc):
    """Three-guide Gaussian potential on a (nz, ny, nx) grid; xc is (nguides, nz)."""
    n, lo, hi = _grid_from(shape_zyx, lo, hi)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    xc = np.ascontiguousarray(xc, dtype=np.float64)
    ng = v0.shape[0]
    assert sigma.shape == (ng,) and xc.shape == (ng, shape_zyx[0])
    V = np.empty(shape_zyx, dtype=np.float64)
    _load().orc_ctap_potential(_dp(V), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               _dp(lo), _dp(hi), ng, _dp(v0), _dp(sigma), _dp(xc))
    return V


def bspline_basis(M, a, b, z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    B = np.empty((z.shape[0], M), dtype=np.float64)
    _load().orc_bspline_basis(int(M), float(a), float(b), _dp(z), z.shape[0], _dp(B))
    return B


def adjoint_ctap(psi0, lo, hi, v0, sigma, xc, dt, nsteps, x_hi):
    """Final target population F and dF/dxc (nguides, nz); also returns psi_N."""
    a = _c128(psi0)
    n, lo, hi = _grid_from(a.shape, lo, hi)
    v0 = np.ascontiguousarray(v0, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    xc = np.ascontiguousarray(xc, dtype=np.float64)
    ng = v0.shape[0]
    G = np.zeros((ng, a.shape[0]), dtype=np.float64)
    F = np.zeros(1, dtype=np.float64)
    out = np.empty_like(a)
    _load().orc_adjoint_ctap(_as_dp_complex(a), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                             _dp(lo), _dp(hi), ng, _dp(v0), _dp(sigma), _dp(xc), float(dt),
                             int(nsteps), float(x_hi), _dp(F), _dp(G), _as_dp_complex(out))
    return float(F[0]), G, out
