"""Initial states of the guide-transfer workloads (Morgan et al.,
arXiv:1309.2451, Sec. V: the atom starts in the transverse ground state of
the left guide, found numerically, times a longitudinal Gaussian moving
along the guides).

The ground state comes from the library's imaginary-time split step on the
transverse plane (a grid with Nz = 1); torch only forms the product with the
z factor and normalises it.
"""
from __future__ import annotations

import numpy as np

from . import Solver


def transverse_ground_state(torch, n_xy, lo_xy, hi_xy, v0, sigma, xc, steps, dtau, device):
    """(1, Ny, Nx) complex128 tensor: imaginary-time ground state of one guide
    (depth v0, width sigma, centre x = xc) on the transverse plane
    n_xy = (Nx, Ny), box [lo_xy, hi_xy), from a Gaussian start (real and
    positive, which fixes sign and phase)."""
    nx, ny = int(n_xy[0]), int(n_xy[1])
    s2 = Solver((nx, ny, 1), (lo_xy[0], lo_xy[1], 0.0), (hi_xy[0], hi_xy[1], 1.0), "c128", device=device)
    try:
        s2.set_guides([v0], [sigma], np.array([[xc]], dtype=np.float64))
        x = lo_xy[0] + torch.arange(nx, dtype=torch.float64, device=device) * ((hi_xy[0] - lo_xy[0]) / nx)
        y = lo_xy[1] + torch.arange(ny, dtype=torch.float64, device=device) * ((hi_xy[1] - lo_xy[1]) / ny)
        phi = torch.exp(-((x[None, :] - xc) ** 2 + y[:, None] ** 2) / (2 * sigma ** 2)).to(torch.complex128)
        phi = phi.reshape(1, ny, nx).contiguous()
        s2.step(phi, steps, dtau, imag=True)
        torch.cuda.current_stream(device).synchronize()
    finally:
        s2.close()
    return phi


def packet(torch, grid, phi, z0, zwidth, kz, device):
    """phi(x, y) exp(-(z - z0)^2 / (2 zwidth^2) + i kz z) on `grid` (an object
    with n, lo, hi, axis(a) and dv), normalised to sum |psi|^2 dV = 1 (complex128)."""
    z = torch.tensor(grid.axis(2), dtype=torch.float64, device=device)
    fz = torch.exp(-((z - z0) ** 2) / (2 * zwidth ** 2)).to(torch.complex128) * torch.exp(1j * kz * z)
    psi = (fz[:, None, None] * phi).contiguous()
    nrm = torch.sqrt(torch.sum(torch.abs(psi) ** 2) * grid.dv)
    return (psi / nrm).contiguous()


def guide_index(grid, z0):
    """Index of the z plane nearest z0."""
    return int(round((z0 - grid.lo[2]) / grid.spacing(2)))


def guide_transfer_state(torch, cfg, device, imag_steps=None, kz=None):
    """The initial state of a guide-transfer workload description (grid,
    guides, z0, zwidth, kz, dt, imag_steps): guide 1's transverse ground
    state at z0 (imaginary time with dtau = dt) times the moving z Gaussian."""
    g, gd = cfg["grid"], cfg["guides"]
    xc = float(gd.xc[0, guide_index(g, cfg["z0"])])
    steps = cfg["imag_steps"] if imag_steps is None else imag_steps
    phi = transverse_ground_state(torch, g.n[:2], g.lo[:2], g.hi[:2], gd.v0[0], gd.sigma[0], xc, steps, cfg["dt"],
                                  device)
    return packet(torch, g, phi, cfg["z0"], cfg["zwidth"], cfg["kz"] if kz is None else kz, device)


def chip_guide_state(torch, cfg, device, steps=2000, wall=50.0):
    """The atom-chip workload's initial state (Sec. V): the transverse ground
    state of the left guide at z0, found by the library's imaginary-time step
    on the transverse plane with the chip potential of that plane (walled off
    by `wall` energy units beyond the midline between the left and the middle
    wire, so the state settles in the left guide), times a Gaussian of width
    zwidth along z at rest (the longitudinal trap sets it moving).
    cfg: synth.config_chip(...) (grid, wires, fields, dt, z0, zwidth)."""
    g = cfg["grid"]
    nx, ny = g.n[0], g.n[1]
    z0 = float(cfg["z0"])
    dz = g.spacing(2)
    s2 = Solver((nx, ny, 1), (g.lo[0], g.lo[1], z0), (g.hi[0], g.hi[1], z0 + dz), "c128", device=device)
    try:
        V = s2.chip_potential(cfg["paths"], cfg["currents"], cfg["b_bias"], cfg["b_ip"], cfg["length_unit"],
                              cfg["mu_over_e0"], cfg["omega_z"], cfg["z_c"])
        x = g.lo[0] + torch.arange(nx, dtype=torch.float64, device=device) * g.spacing(0)
        y = g.lo[1] + torch.arange(ny, dtype=torch.float64, device=device) * g.spacing(1)
        # wire positions in the plane z0 (linear along each polyline)
        xw = [float(np.interp(z0, np.asarray(p)[:, 1], np.asarray(p)[:, 0])) for p in cfg["paths"]]
        mid = 0.5 * (xw[0] + xw[1])
        V = (V + wall * (x[None, None, :] >= mid).to(torch.float64)).contiguous()
        s2.set_potential_table(V)
        # start: a Gaussian under the left wire at the single-wire guide height
        r0 = 2e-7 * float(cfg["currents"][0]) / float(cfg["b_bias"]) / float(cfg["length_unit"])
        phi = torch.exp(-((x[None, :] - xw[0]) ** 2 + (y[:, None] - r0) ** 2) / (2 * 0.6 ** 2)).to(torch.complex128)
        phi = phi.reshape(1, ny, nx).contiguous()
        s2.step(phi, steps, cfg["dt"], imag=True)
        torch.cuda.current_stream(device).synchronize()
    finally:
        s2.close()
    return packet(torch, g, phi, z0, cfg["zwidth"], 0.0, device)
