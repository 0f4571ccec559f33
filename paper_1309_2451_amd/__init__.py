"""MI355X split-step Fourier propagation of the 3-D Schroedinger equation.

Python face of libssf (include/ssf.h).  Fields are torch tensors on the GPU,
shape (Nz, Ny, Nx), dtype complex64 or complex128, contiguous; every method
forwards to the C ABI function of the same name with the tensors' device
pointers and torch's current HIP stream.  The split-step arithmetic runs in
the library's HIP kernels only.

Method: Morgan et al., "Coherent transport by adiabatic passage on atom
chips", arXiv:1309.2451 -- Sec. IV (Fourier split-operator time step,
p_max = pi N / L), Sec. V (imaginary-time transverse ground state, guide
populations and final transfer fidelity).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _ssf
from ._ssf import OBS_DTYPE, SSF_C64, SSF_C128, SSF_IMAG, SSF_REAL, SSFError

__all__ = ["Solver", "Batch", "SSFError", "OBS_DTYPE", "supported_length", "bspline_basis", "bspline_eval", "load"]


def load():
    return _ssf.load()


def supported_length(n: int) -> bool:
    return bool(_ssf.load().ssf_supported_length(int(n)))


def bspline_basis(M, a, b, z):
    """(len(z), M) clamped uniform cubic B-spline basis on [a, b] (host, FP64)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    B = np.empty((z.shape[0], int(M)), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _ssf.call("ssf_bspline_basis", int(M), float(a), float(b), z.ctypes.data_as(dp), z.shape[0],
              B.ctypes.data_as(dp))
    return B


def bspline_eval(M, a, b, coeffs, z):
    """(len(coeffs), len(z)) profiles sum_m coeffs[k, m] B_m(z) of the same basis (host, FP64)."""
    c = np.ascontiguousarray(np.atleast_2d(coeffs), dtype=np.float64)
    if c.shape[1] != int(M):
        raise ValueError("coeffs must have M = %d columns" % int(M))
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty((c.shape[0], z.shape[0]), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _ssf.call("ssf_bspline_eval", int(M), float(a), float(b), c.ctypes.data_as(dp), c.shape[0],
              z.ctypes.data_as(dp), z.shape[0], out.ctypes.data_as(dp))
    return out


def _torch():
    import torch
    return torch


class Solver:
    """One grid + storage type on one GPU (an ssf_handle).

    n = (Nx, Ny, Nz); lo, hi = box per axis; dtype "c64" or "c128".
    """

    def __init__(self, n, lo, hi, dtype="c128", device=None):
        torch = _torch()
        self.torch = torch
        self.n = tuple(int(v) for v in n)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.dtype = {"c64": SSF_C64, "c128": SSF_C128}[dtype]
        self.tdtype = torch.complex64 if self.dtype == SSF_C64 else torch.complex128
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.shape = (self.n[2], self.n[1], self.n[0])
        g = _ssf.ssf_grid_desc()
        for a in range(3):
            g.n[a], g.lo[a], g.hi[a] = self.n[a], self.lo[a], self.hi[a]
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            _ssf.call("ssf_create", ctypes.byref(g), self.dtype, ctypes.c_void_p(stream), ctypes.byref(h))
        self.h = h
        self._keep = {}

    # -- plumbing -------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            _ssf.call("ssf_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = self.torch.cuda.current_stream(self.device).cuda_stream
        _ssf.call("ssf_set_stream", self.h, ctypes.c_void_p(s))

    def _field(self, t, name="psi"):
        if t.dtype != self.tdtype or tuple(t.shape[-3:]) != self.shape or not t.is_contiguous() \
                or t.device != self.device:
            raise ValueError("%s must be a contiguous %s tensor of shape %s on %s (got %s %s %s)"
                             % (name, self.tdtype, self.shape, self.device, t.dtype, tuple(t.shape), t.device))
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, *lead):
        return self.torch.empty(*lead, *self.shape, dtype=self.tdtype, device=self.device)

    def obs_buffer(self, count):
        return self.torch.zeros(max(int(count), 1) * OBS_DTYPE.itemsize, dtype=self.torch.uint8, device=self.device)

    def read_obs(self, buf, count):
        host = np.zeros(int(count), dtype=OBS_DTYPE)
        if count:
            self._sync_stream()
            _ssf.call("ssf_obs_read", self.h, ctypes.c_void_p(buf.data_ptr()),
                      ctypes.c_void_p(host.ctypes.data), int(count))
        return host

    # -- configuration ----------------------------------------------------------
    def set_potential_table(self, V):
        torch = self.torch
        if V.dtype not in (torch.float64, torch.float32) or tuple(V.shape) != self.shape or not V.is_contiguous():
            raise ValueError("potential table must be a contiguous float32/float64 tensor of shape %s" % (self.shape,))
        self._keep["V"] = V
        _ssf.call("ssf_set_potential_table", self.h, ctypes.c_void_p(V.data_ptr()), 1 if V.dtype == torch.float64 else 0)

    def set_guides(self, v0, sigma, xc):
        xc = np.ascontiguousarray(xc, dtype=np.float64)
        d = _ssf.ssf_ctap_desc()
        d.nguides = xc.shape[0]
        for g in range(d.nguides):
            d.v0[g] = float(v0[g])
            d.sigma[g] = float(sigma[g])
        if xc.shape != (d.nguides, self.n[2]):
            raise ValueError("xc must be (nguides, Nz)")
        d.xc = xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._sync_stream()
        _ssf.call("ssf_set_potential_ctap", self.h, ctypes.byref(d))
        self.nguides = d.nguides

    def chip_potential(self, paths, currents, b_bias, b_ip, length_unit, mu_over_e0, omega_z, z_c, out=None):
        """The atom-chip potential (ssf_chip_potential) on this grid as a
        float64 (Nz, Ny, Nx) tensor on the device (into `out` if given):
        wires along the polylines `paths` (each (k, 2): x, z in length
        units, on the chip surface y = 0) with `currents` (A), bias field
        b_bias along x and offset field b_ip along z (T), length unit in
        metres, moment over energy unit (per T), longitudinal trap omega_z
        centred at z_c.  Use with set_potential_table."""
        torch = self.torch
        paths = [np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 2) for q in paths]
        npts = np.ascontiguousarray([q.shape[0] for q in paths], dtype=np.int32)
        flat = np.ascontiguousarray(np.concatenate([q.ravel() for q in paths]))
        cur = np.ascontiguousarray(currents, dtype=np.float64)
        if cur.shape != (len(paths),):
            raise ValueError("one current per wire")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        elif out.dtype != torch.float64 or tuple(out.shape) != self.shape or not out.is_contiguous() \
                or out.device != self.device:
            raise ValueError("out must be a contiguous float64 tensor of shape %s on %s" % (self.shape, self.device))
        d = _ssf.ssf_chip_desc()
        d.nwires = len(paths)
        d.npts = npts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.path = flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.current = cur.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.b_bias, d.b_ip, d.length_unit = float(b_bias), float(b_ip), float(length_unit)
        d.mu_over_e0, d.omega_z, d.z_c = float(mu_over_e0), float(omega_z), float(z_c)
        self._sync_stream()
        _ssf.call("ssf_chip_potential", self.h, ctypes.byref(d), ctypes.c_void_p(out.data_ptr()))
        return out

    def clear_potential(self):
        _ssf.call("ssf_clear_potential", self.h)

    def set_partition(self, x_lo, x_hi):
        _ssf.call("ssf_set_partition", self.h, float(x_lo), float(x_hi))

    def set_partition_z(self, x_lo, x_hi):
        """Plane-dependent guide regions: arrays of length Nz."""
        xl = np.ascontiguousarray(x_lo, dtype=np.float64)
        xh = np.ascontiguousarray(x_hi, dtype=np.float64)
        if xl.shape != (self.n[2],) or xh.shape != (self.n[2],):
            raise ValueError("x_lo and x_hi must have length Nz = %d" % self.n[2])
        dp = ctypes.POINTER(ctypes.c_double)
        self._sync_stream()
        _ssf.call("ssf_set_partition_z", self.h, xl.ctypes.data_as(dp), xh.ctypes.data_as(dp))

    def density_xz(self, psi, out=None):
        """(Nz, Nx) float64 tensor: sum over y of |psi|^2 dy."""
        torch = self.torch
        if out is None:
            out = torch.empty((self.n[2], self.n[0]), dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or tuple(out.shape) != (self.n[2], self.n[0]) or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape (Nz, Nx)")
        self._sync_stream()
        _ssf.call("ssf_density_xz", self.h, self._field(psi), ctypes.c_void_p(out.data_ptr()))
        return out

    def set_fusion(self, on: bool):
        _ssf.call("ssf_set_fusion", self.h, 1 if on else 0)

    def set_splitting(self, order: str):
        """"vtv" (default: V/2-T-V/2) or "tvt" (T/2-V-T/2) for real-time steps."""
        _ssf.call("ssf_set_splitting", self.h, {"vtv": _ssf.SSF_SPLIT_VTV, "tvt": _ssf.SSF_SPLIT_TVT}[order])

    def set_arithmetic(self, mode: str):
        """"f64" (default) or "f32" (complex64 handles: FP32 bulk arithmetic,
        FP64 phase arguments, factors and sums)."""
        _ssf.call("ssf_set_arithmetic", self.h, {"f64": _ssf.SSF_ARITH_F64, "f32": _ssf.SSF_ARITH_F32}[mode])

    def tune(self, reps=5):
        """Time every y/z tile variant on this grid and keep the fastest.
        Returns (choice[3], {(axis, variant): microseconds})."""
        self._sync_stream()
        nv = _ssf.SSF_TILE_VARIANTS
        ch = np.zeros(3, dtype=np.int32)
        us = np.zeros(3 * nv, dtype=np.float64)
        _ssf.call("ssf_tune", self.h, int(reps), ctypes.c_void_p(ch.ctypes.data), ctypes.c_void_p(us.ctypes.data))
        return ch.tolist(), {(a, v): float(us[a * nv + v]) for a in (1, 2) for v in range(nv)}

    def tune_cached(self, cache_path, reps=5):
        """The tuner through a cache file (ssf_tune_cached): (choice[3], hit)."""
        self._sync_stream()
        ch = np.zeros(3, dtype=np.int32)
        hit = np.zeros(1, dtype=np.int32)
        _ssf.call("ssf_tune_cached", self.h, int(reps), str(cache_path).encode(), ctypes.c_void_p(ch.ctypes.data),
                  ctypes.c_void_p(hit.ctypes.data))
        return ch.tolist(), bool(hit[0])

    def set_tiles(self, choice):
        ch = np.ascontiguousarray(choice, dtype=np.int32)
        _ssf.call("ssf_set_tiles", self.h, ctypes.c_void_p(ch.ctypes.data))

    def get_tiles(self):
        ch = np.zeros(3, dtype=np.int32)
        _ssf.call("ssf_get_tiles", self.h, ctypes.c_void_p(ch.ctypes.data))
        return ch.tolist()

    PASS_KINDS = ("x_fwd", "x_inv", "x_inv_phase_fwd", "yz_fwd", "yz_inv", "z_fwd_kin_inv")

    def set_timing(self, on: bool):
        _ssf.call("ssf_set_timing", self.h, 1 if on else 0)

    def timing_read(self):
        """{pass kind: (total ms, launches)} since timing was enabled or last read."""
        self._sync_stream()
        ms = np.zeros(6, dtype=np.float64)
        cnt = np.zeros(6, dtype=np.int64)
        _ssf.call("ssf_timing_read", self.h, ctypes.c_void_p(ms.ctypes.data), ctypes.c_void_p(cnt.ctypes.data))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.PASS_KINDS)}

    # -- the path ----------------------------------------------------------------
    def step(self, psi, nsteps, dt, imag=False, obs_every=0, obs_buf=None):
        """nsteps Strang steps in place.  Returns the observation records
        (numpy, OBS_DTYPE) if obs_every > 0, else None.  With obs_buf given the
        records stay on the device (no synchronisation) and None is returned."""
        self._sync_stream()
        p = self._field(psi)
        nobs = (int(nsteps) // int(obs_every)) if obs_every else 0
        buf = obs_buf if obs_buf is not None else (self.obs_buffer(nobs) if nobs else None)
        _ssf.call("ssf_step", self.h, p, int(nsteps), float(dt), SSF_IMAG if imag else SSF_REAL,
                  int(obs_every) if nobs else 0, ctypes.c_void_p(buf.data_ptr()) if buf is not None else None)
        if nobs and obs_buf is None:
            return self.read_obs(buf, nobs)
        return None

    def step_noalloc(self, psi, nsteps, dt, imag=False, obs_every=0, obs_buf=None):
        """As step(), through ssf_step_noalloc: the library allocates nothing
        (its per-call buffers live in a static per-GPU scratch array).  Pass
        obs_buf (from obs_buffer) to keep the call itself free of allocation;
        without it a records buffer is allocated here by torch."""
        self._sync_stream()
        p = self._field(psi)
        nobs = (int(nsteps) // int(obs_every)) if obs_every else 0
        buf = obs_buf if obs_buf is not None else (self.obs_buffer(nobs) if nobs else None)
        _ssf.call("ssf_step_noalloc", self.h, p, int(nsteps), float(dt), SSF_IMAG if imag else SSF_REAL,
                  int(obs_every) if nobs else 0, ctypes.c_void_p(buf.data_ptr()) if buf is not None else None)
        if nobs and obs_buf is None:
            return self.read_obs(buf, nobs)
        return None

    def fft(self, psi, axes=(0, 1, 2), inverse=False):
        self._sync_stream()
        mask = 0
        for a in axes:
            mask |= 1 << int(a)
        _ssf.call("ssf_fft", self.h, self._field(psi), mask, 1 if inverse else 0)

    def observables(self, psi):
        self._sync_stream()
        buf = self.obs_buffer(1)
        _ssf.call("ssf_observables", self.h, self._field(psi), ctypes.c_void_p(buf.data_ptr()))
        return self.read_obs(buf, 1)[0]

    def step_ckpt(self, psi, nsteps, dt, every, ckpt):
        self._sync_stream()
        nslots = -(-int(nsteps) // int(every))
        if ckpt.shape[0] < nslots:
            raise ValueError("checkpoint buffer needs %d slots" % nslots)
        self._field(ckpt[0], "ckpt")
        _ssf.call("ssf_step_ckpt", self.h, self._field(psi), int(nsteps), float(dt), int(every),
                  ctypes.c_void_p(ckpt.data_ptr()))

    def step_seq(self, psi0, nsteps, dt, seq):
        self._sync_stream()
        if seq.shape[0] < int(nsteps) + 1:
            raise ValueError("sequence buffer needs nsteps + 1 slots")
        self._field(seq[0], "seq")
        _ssf.call("ssf_step_seq", self.h, self._field(psi0, "psi0"), int(nsteps), float(dt),
                  ctypes.c_void_p(seq.data_ptr()))

    def adjoint_init(self, psi, lam):
        self._sync_stream()
        _ssf.call("ssf_adjoint_init", self.h, self._field(psi), self._field(lam, "lambda"))

    def adjoint_segment(self, lam, seq, nsteps, dt, G):
        torch = self.torch
        if G.dtype != torch.float64 or not G.is_contiguous() or G.numel() < self.nguides * self.n[2]:
            raise ValueError("G must be a contiguous float64 tensor with nguides * Nz entries")
        if seq.shape[0] < int(nsteps) + 1:
            raise ValueError("sequence buffer needs nsteps + 1 slots")
        self._field(seq[0], "seq")
        self._sync_stream()
        _ssf.call("ssf_adjoint_segment", self.h, self._field(lam, "lambda"), ctypes.c_void_p(seq.data_ptr()),
                  int(nsteps), float(dt), ctypes.c_void_p(G.data_ptr()))

    def profile_grad(self, G, B, nguides, out):
        """out[g, m] = sum_z G[g, z] B[z, m] on the device (FP64 tensors)."""
        torch = self.torch
        for t in (G, B, out):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("profile_grad needs contiguous float64 tensors on the solver's device")
        M = B.shape[1]
        self._sync_stream()
        _ssf.call("ssf_profile_grad", self.h, ctypes.c_void_p(G.data_ptr()), int(nguides),
                  ctypes.c_void_p(B.data_ptr()), int(M), ctypes.c_void_p(out.data_ptr()))

    def sync(self):
        _ssf.call("ssf_sync", self.h)

    def copy(self, src, dst):
        """dst = src by a plain copy kernel (2 x field bytes of HBM traffic)."""
        self._sync_stream()
        _ssf.call("ssf_copy", self.h, self._field(src, "src"), self._field(dst, "dst"))


class Batch:
    """Many independent instances (an ssf_batch): instance i has its own grid
    n[i], lo[i], hi[i], potential and partition (x_lo[i], x_hi[i]).  The
    potential is either guides (v0[i], sigma[i], xc[i] of shape (3, Nz_i)) or,
    with tables=..., a float64 device tensor (Nz_i, Ny_i, Nx_i) per instance
    (borrowed: kept referenced here).  Instances with equal grids share tables
    and are stepped together by one persistent launch per pass; the groups run
    concurrently.  Fields are a list of tensors (Nz_i, Ny_i, Nx_i)."""

    def __init__(self, grids, guides, x_lo, x_hi, dtype="c64", device=None, tables=None):
        torch = _torch()
        self.torch = torch
        self.count = len(grids)
        if (guides is None) == (tables is None):
            raise ValueError("give either guides or tables")
        if not (len(guides if tables is None else tables) == len(x_lo) == len(x_hi) == self.count) \
                or self.count < 1:
            raise ValueError("grids, guides or tables, x_lo, x_hi must have one entry per instance")
        self.dtype = {"c64": SSF_C64, "c128": SSF_C128}[dtype]
        self.tdtype = torch.complex64 if self.dtype == SSF_C64 else torch.complex128
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        gd = (_ssf.ssf_grid_desc * self.count)()
        cd = (_ssf.ssf_ctap_desc * self.count)()
        self._xc = []
        self.shapes = []
        for i, (n, lo, hi) in enumerate(grids):
            for a in range(3):
                gd[i].n[a], gd[i].lo[a], gd[i].hi[a] = int(n[a]), float(lo[a]), float(hi[a])
            self.shapes.append((int(n[2]), int(n[1]), int(n[0])))
        self._tables = None
        if tables is not None:
            tp = (ctypes.c_void_p * self.count)()
            for i, t in enumerate(tables):
                if t.dtype != torch.float64 or tuple(t.shape) != self.shapes[i] or not t.is_contiguous() \
                        or t.device != self.device:
                    raise ValueError("table %d must be a contiguous float64 tensor of shape %s on %s"
                                     % (i, self.shapes[i], self.device))
                tp[i] = t.data_ptr()
            self._tables = list(tables)
        for i, ((n, lo, hi), gdesc) in enumerate(zip(grids, guides if guides is not None else [])):
            v0, sigma, xc = gdesc
            xc = np.ascontiguousarray(xc, dtype=np.float64)
            if xc.ndim != 2 or xc.shape[1] != int(n[2]) or not 1 <= xc.shape[0] <= 3:
                raise ValueError("instance %d: xc must be (nguides, Nz)" % i)
            cd[i].nguides = xc.shape[0]
            for g in range(xc.shape[0]):
                cd[i].v0[g] = float(v0[g])
                cd[i].sigma[g] = float(sigma[g])
            cd[i].xc = xc.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self._xc.append(xc)
        lo_a = np.ascontiguousarray(x_lo, dtype=np.float64)
        hi_a = np.ascontiguousarray(x_hi, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            if tables is None:
                _ssf.call("ssf_batch_create", self.count, gd, cd, lo_a.ctypes.data_as(dp), hi_a.ctypes.data_as(dp),
                          self.dtype, ctypes.c_void_p(stream), ctypes.byref(h))
            else:
                _ssf.call("ssf_batch_create_tables", self.count, gd, tp, lo_a.ctypes.data_as(dp),
                          hi_a.ctypes.data_as(dp), self.dtype, ctypes.c_void_p(stream), ctypes.byref(h))
        self.h = h
        self._ptrs = (ctypes.c_void_p * self.count)()

    def close(self):
        if getattr(self, "h", None):
            _ssf.call("ssf_batch_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def groups(self):
        """(number of groups, group index of each instance)."""
        ng = ctypes.c_int32()
        gof = np.zeros(self.count, dtype=np.int32)
        _ssf.call("ssf_batch_info", self.h, ctypes.byref(ng), ctypes.c_void_p(gof.ctypes.data))
        return int(ng.value), gof

    def empty(self):
        return [self.torch.empty(s, dtype=self.tdtype, device=self.device) for s in self.shapes]

    def obs_buffer(self):
        return self.torch.zeros(self.count * OBS_DTYPE.itemsize, dtype=self.torch.uint8, device=self.device)

    def tune(self, reps=5):
        _ssf.call("ssf_batch_tune", self.h, int(reps))

    def run(self, fields, nsteps, dt, chunk=50, obs_buf=None):
        if len(fields) != self.count:
            raise ValueError("need one field per instance")
        for i, (t, s) in enumerate(zip(fields, self.shapes)):
            if t.dtype != self.tdtype or tuple(t.shape) != s or not t.is_contiguous() or t.device != self.device:
                raise ValueError("field %d must be a contiguous %s tensor of shape %s on %s"
                                 % (i, self.tdtype, s, self.device))
            self._ptrs[i] = t.data_ptr()
        ob = ctypes.c_void_p(obs_buf.data_ptr()) if obs_buf is not None else ctypes.c_void_p(0)
        stream = self.torch.cuda.current_stream(self.device).cuda_stream
        _ssf.call("ssf_batch_set_stream", self.h, ctypes.c_void_p(stream))
        _ssf.call("ssf_batch_run", self.h, self._ptrs, int(nsteps), float(dt), int(chunk), ob)

    def read_obs(self, buf):
        """Observation records of the last run (host, OBS_DTYPE)."""
        self.torch.cuda.current_stream(self.device).synchronize()
        return np.frombuffer(buf.cpu().numpy().tobytes(), dtype=OBS_DTYPE).copy()
