"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 unless stated):
  complex128 storage: 1e-12 (FP64 rounding of a few hundred passes);
  complex64 storage: the input and every pass output are rounded to FP32
  (unit roundoff 6e-8), arithmetic is FP64, so after n passes the error is a
  random walk of at most ~6e-8 sqrt(n) per value; the bounds below allow 3x.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
ssf = pytest.importorskip("paper_1309_2451_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a, solver):
    return torch.from_numpy(np.ascontiguousarray(a)).to(solver.tdtype).to(DEV).contiguous()


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def c64_round(a):
    return np.asarray(a, dtype=np.complex64).astype(np.complex128)


FFT_SHAPES = [(8, 8, 8), (12, 20, 40), (16, 32, 64), (1, 24, 160), (96, 48, 1), (4, 12, 512), (2, 4, 1024),
              (20, 12, 96), (20, 2, 256), (12, 128, 8), (192, 1, 16), (2, 384, 20), (768, 2, 1), (80, 320, 2),
              (4, 2, 640), (1, 1, 1)]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft_each_axis_vs_oracle(dtype, shape):
    nz, ny, nx = shape
    say("fft", dtype, shape)
    s = ssf.Solver((nx, ny, nz), (0, 0, 0), (1, 1, 1), dtype)
    rng = np.random.default_rng(nx * 7 + ny * 3 + nz)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    if dtype == "c64":
        x = c64_round(x)
    tol = 1e-13 if dtype == "c128" else 2e-7
    for axis in range(3):
        for inverse in (False, True):
            t = to_dev(x, s)
            s.fft(t, axes=(axis,), inverse=inverse)
            ref = oracle.fft_axis(x, axis, +1 if inverse else -1)
            assert rel(host(t), ref) < tol, (axis, inverse)
    t = to_dev(x, s)
    s.fft(t)
    assert rel(host(t), oracle.fft3d(x, -1)) < tol * 2
    s.close()


def _random_case(shape, seed, vscale=10.0):
    nz, ny, nx = shape
    g = synth.Grid((nx, ny, nz), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    rng = np.random.default_rng(seed)
    psi = synth.random_field(g, seed, smooth=2.0)
    V = rng.uniform(-vscale, vscale, g.shape)
    return g, psi, V


@pytest.mark.parametrize("fuse", [True, False])
@pytest.mark.parametrize("shape", [(20, 12, 40), (16, 24, 32), (12, 8, 96)])
def test_step_random_c128_vs_oracle(shape, fuse):
    say("step c128", shape, "fuse", fuse)
    g, psi0, V = _random_case(shape, 5)
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    s.set_fusion(fuse)
    Vt = torch.from_numpy(V).to(DEV)
    s.set_potential_table(Vt)
    s.set_partition(-1.0, 0.5)
    t = to_dev(psi0, s)
    dt, n = 0.013, 37
    obs = s.step(t, n, dt, obs_every=5)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    assert rel(host(t), ref) < 1e-12
    # observations at steps 5, 10, ..., 35
    ref_psi = psi0
    for k in range(len(obs)):
        ref_psi, _ = oracle.step(ref_psi, V, g.lo, g.hi, dt, 5)
        o = oracle.observables(ref_psi, V, g.lo, g.hi, -1.0, 0.5)
        assert obs[k]["step"] == 5 * (k + 1)
        assert abs(obs[k]["norm"] - o["norm"]) < 1e-12
        for a, key in enumerate(("mx", "my", "mz")):
            assert abs(obs[k]["mean"][a] - o[key]) < 1e-12
        for a, key in enumerate(("p1", "p2", "p3")):
            assert abs(obs[k]["pop"][a] - o[key]) < 1e-12
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("nx", [640, 768, 1024])
def test_long_x_rows_step_vs_oracle(dtype, nx):
    """The longest x lengths (fused x passes with 20-, 24- and 8-value plans,
    stage-major twiddle tables of both radix orders) in 30 steps against the
    oracle, on a box with x spacing 1/8 (kinetic phases of a few radians)."""
    say("long x rows", dtype, nx)
    g = synth.Grid((nx, 4, 4), (-nx / 16.0, -2.0, -2.0), (nx / 16.0, 2.0, 2.0))
    rng = np.random.default_rng(nx)
    psi0 = synth.random_field(g, nx + 1, smooth=nx / 32.0)
    V = rng.uniform(-10.0, 10.0, g.shape)
    if dtype == "c64":
        psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    t = to_dev(psi0, s)
    dt, n = 0.013, 30
    s.step(t, n, dt)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(n * 5)
    assert rel(host(t), ref) < tol
    s.close()


@pytest.mark.parametrize("shape", [(20, 12, 40), (12, 8, 96)])
def test_step_random_c64_vs_oracle(shape):
    say("step c64", shape)
    g, psi0, V = _random_case(shape, 6)
    psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    t = to_dev(psi0, s)
    dt, n = 0.013, 50
    s.step(t, n, dt)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    # 50 steps x 4-5 rounded passes
    assert rel(host(t), ref) < 3 * 6e-8 * np.sqrt(50 * 5)
    # float32 potential table: V itself is rounded, still close
    s.set_potential_table(torch.from_numpy(V.astype(np.float32)).to(DEV))
    t = to_dev(psi0, s)
    s.step(t, n, dt)
    ref32, _ = oracle.step(psi0, V.astype(np.float32).astype(np.float64), g.lo, g.hi, dt, n)
    assert rel(host(t), ref32) < 3 * 6e-8 * np.sqrt(50 * 5)
    s.close()


@pytest.mark.parametrize("shape", [(20, 12, 40), (12, 8, 96), (8, 16, 512)])
def test_fp32_arithmetic_mode_vs_oracle(shape):
    """Complex64 storage with FP32 bulk arithmetic (ssf_set_arithmetic):
    transforms and steps against the oracle within FP32 rounding over the
    transform depth, and different from (less exact than) the FP64-arithmetic
    mode on the same input."""
    say("fp32 arithmetic", shape)
    g, psi0, V = _random_case(shape, 8)
    psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    dt, n = 0.013, 50
    t64 = to_dev(psi0, s)
    s.step(t64, n, dt)
    s.set_arithmetic("f32")
    for axis in (0, 1, 2):
        t = to_dev(psi0, s)
        s.fft(t, axes=(axis,))
        err = rel(host(t), oracle.fft_axis(psi0, axis, -1))
        assert err < 6e-8 * 3 * np.log2(max(g.n[axis], 2)) + 1e-7, (axis, err)
    t = to_dev(psi0, s)
    s.step(t, n, dt)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    err32, err64 = rel(host(t), ref), rel(host(t64), ref)
    say("fp32 arithmetic rel L2 %.3e, fp64 arithmetic %.3e" % (err32, err64))
    # 50 steps x 4-5 passes, each with a few FP32 roundings per transform stage
    assert err32 < 2e-5
    assert rel(host(t), host(t64)) > 1e-9
    with pytest.raises(ssf.SSFError):
        ssf.Solver(g.n, g.lo, g.hi, "c128").set_arithmetic("f32")
    s.set_arithmetic("f64")
    t = to_dev(psi0, s)
    s.step(t, n, dt)
    assert torch.equal(t, t64)
    s.close()


def test_config1_harmonic_c128():
    c = synth.config1()
    g = c["grid"]
    say("config1 harmonic 64^3 c128, 200 steps")
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    s.set_potential_table(torch.from_numpy(c["V"]).to(DEV))
    s.set_partition(-1.5, 1.5)
    t = to_dev(c["psi0"], s)
    obs = s.step(t, c["steps"], c["dt"], obs_every=1)
    ref, _ = oracle.step(c["psi0"], c["V"], g.lo, g.hi, c["dt"], c["steps"])
    assert rel(host(t), ref) < 1e-12
    theta = np.arccos(1.0 - c["dt"] ** 2 / 2.0)
    n = np.arange(1, c["steps"] + 1)
    assert np.max(np.abs(obs["mean"][:, 0] - np.cos(n * theta))) < 1e-11
    assert np.max(np.abs(obs["norm"] - 1.0)) < 1e-12
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_imaginary_time_vs_oracle(dtype):
    say("imag", dtype)
    g = synth.Grid((32, 24, 40), (-6.0, -5.0, -7.0), (6.0, 5.0, 7.0))
    V = synth.harmonic_table(g, (1.0, 1.3, 0.8))
    psi0 = synth.gaussian_packet(g, centre=(0.3, -0.2, 0.5), width=(1.3, 0.7, 1.1))
    if dtype == "c64":
        psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    t = to_dev(psi0, s)
    dtau, n = 0.01, 60
    obs = s.step(t, n, dtau, imag=True, obs_every=1)
    ref, ed = oracle.step(psi0, V, g.lo, g.hi, dtau, n, imag=True)
    tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(5 * n)
    assert rel(host(t), ref) < tol
    assert np.max(np.abs(obs["energy"] - ed)) < (1e-9 if dtype == "c128" else 1e-3)
    assert abs(obs["norm"][-1] - np.exp(-2 * ed[-1] * dtau)) < (1e-12 if dtype == "c128" else 1e-6)
    o = s.observables(t)
    assert abs(o["norm"] - 1.0) < (1e-13 if dtype == "c128" else 1e-6)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("obs_every", [0, 7])
def test_imaginary_time_fused_chain_vs_oracle(dtype, obs_every):
    """Imaginary time with the step chain fused across observations: the norm
    of every step is summed inside the x pass between two steps and the scale
    rides on the next pass.  Final field against the oracle, step energies at
    the observed steps against the oracle's, and the unfused path."""
    say("imag fused", dtype, obs_every)
    g = synth.Grid((32, 24, 40), (-6.0, -5.0, -7.0), (6.0, 5.0, 7.0))
    V = synth.harmonic_table(g, (1.0, 1.3, 0.8))
    psi0 = synth.gaussian_packet(g, centre=(0.3, -0.2, 0.5), width=(1.3, 0.7, 1.1))
    if dtype == "c64":
        psi0 = c64_round(psi0)
    dtau, n = 0.01, 30
    ref, ed = oracle.step(psi0, V, g.lo, g.hi, dtau, n, imag=True)
    out = {}
    for fuse in (True, False):
        s = ssf.Solver(g.n, g.lo, g.hi, dtype)
        s.set_potential_table(torch.from_numpy(V).to(DEV))
        s.set_fusion(fuse)
        t = to_dev(psi0, s)
        obs = s.step(t, n, dtau, imag=True, obs_every=obs_every)
        out[fuse] = host(t)
        tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(5 * n)
        assert rel(out[fuse], ref) < tol, fuse
        if obs_every:
            k = np.arange(obs_every, n + 1, obs_every)
            assert np.max(np.abs(obs["energy"] - ed[k - 1])) < (1e-9 if dtype == "c128" else 1e-3)
        o = s.observables(t)
        assert abs(o["norm"] - 1.0) < (1e-13 if dtype == "c128" else 1e-6)
        s.close()
    assert rel(out[True], out[False]) < (1e-13 if dtype == "c128" else 1e-6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_observables_energy_vs_oracle(dtype):
    say("observables", dtype)
    g = synth.Grid((40, 24, 32), (-6.0, -5.0, -7.0), (6.0, 5.0, 7.0))
    V = synth.harmonic_table(g, (1.0, 1.3, 0.8))
    psi = synth.gaussian_packet(g, centre=(0.5, 0.2, -0.4), width=(0.9, 0.8, 1.2), k=(0.7, 0.0, -0.3))
    if dtype == "c64":
        psi = c64_round(psi)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    s.set_partition(-0.5, 1.0)
    o = s.observables(to_dev(psi, s))
    r = oracle.observables(psi, V, g.lo, g.hi, -0.5, 1.0)
    tol = 1e-12
    assert abs(o["norm"] - r["norm"]) < tol
    # complex64: the kinetic part is summed from a transform whose passes round to FP32
    assert abs(o["energy"] - r["energy"]) < (1e-11 if dtype == "c128" else 1e-7 * abs(r["energy"]))
    assert abs(o["pop"][0] - r["p1"]) < tol and abs(o["pop"][2] - r["p3"]) < tol
    s.close()


def _ctap_small():
    g = synth.Grid((32, 24, 64), (-5.0, -4.0, -16.0), (5.0, 4.0, 16.0))
    guides = synth.ctap_guides(g, d0=2.0, delta=0.6, v0=12.0, sigma=0.6, z1=2.0, z3=-2.0, wg=3.0)
    psi0 = synth.gaussian_packet(g, centre=(-2.0, 0.0, -6.0), width=(0.5, 0.5, 2.0), k=(0.0, 0.0, 2.0))
    return g, guides, psi0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_guide_potential_step_vs_oracle(dtype):
    say("ctap step", dtype)
    g, gd, psi0 = _ctap_small()
    if dtype == "c64":
        psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    t = to_dev(psi0, s)
    dt, n = 0.01, 80
    obs = s.step(t, n, dt, obs_every=40)
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, dt, n)
    tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(5 * n)
    assert rel(host(t), ref) < tol
    o = oracle.observables(ref, V, g.lo, g.hi, gd.x_lo, gd.x_hi)
    for a, key in enumerate(("p1", "p2", "p3")):
        assert abs(obs[-1]["pop"][a] - o[key]) < (1e-12 if dtype == "c128" else 1e-6)
    ekin = oracle.observables(ref, None, g.lo, g.hi, 0, 0)["energy"]
    assert abs(obs[-1]["epot"] - (o["energy"] - ekin)) < (1e-9 if dtype == "c128" else 1e-4)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_gradient_vs_oracle(dtype):
    say("adjoint", dtype)
    g, gd, psi0 = _ctap_small()
    if dtype == "c64":
        psi0 = c64_round(psi0)
    dt, n, seg = 0.01, 40, 16
    F_ref, G_ref, psiN_ref = oracle.adjoint_ctap(psi0, g.lo, g.hi, gd.v0, gd.sigma, gd.xc, dt, n, gd.x_hi)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    psi = to_dev(psi0, s)
    nseg = -(-n // seg)
    ck = s.empty(nseg)
    s.step_ckpt(psi, n, dt, seg, ck)
    F = s.observables(psi)["pop"][2]
    lam = s.empty()
    s.adjoint_init(psi, lam)
    G = torch.zeros(3 * g.n[2], dtype=torch.float64, device=DEV)
    seq = s.empty(seg + 1)
    for k in reversed(range(nseg)):
        steps = min(seg, n - k * seg)
        s.step_seq(ck[k], steps, dt, seq)
        s.adjoint_segment(lam, seq, steps, dt, G)
    Gh = G.cpu().numpy().reshape(3, g.n[2])
    scale = np.max(np.abs(G_ref))
    if dtype == "c128":
        assert abs(F - F_ref) < 1e-12
        assert np.max(np.abs(Gh - G_ref)) < 1e-10 * scale
    else:
        assert abs(F - F_ref) < 1e-6
        assert np.max(np.abs(Gh - G_ref)) < 1e-4 * scale
    s.close()


def test_checkpoint_recompute_is_bitwise():
    say("ckpt bitwise")
    g, gd, psi0 = _ctap_small()
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    dt, n, every = 0.01, 24, 8
    psi = to_dev(psi0, s)
    ck = s.empty(3)
    s.step_ckpt(psi, n, dt, every, ck)
    seq = s.empty(every + 1)
    s.step_seq(ck[1], every, dt, seq)
    assert torch.equal(seq[every], ck[2])
    s.step_seq(ck[2], every, dt, seq)
    assert torch.equal(seq[every], psi)
    s.close()


def test_fidelity_autograd_fd_and_oracle_chain_rule():
    say("fidelity autograd c128")
    from paper_1309_2451_amd.fidelity import FidelityFn, FidelityProblem
    g, gd, psi0 = _ctap_small()
    M = 8
    a, b = g.lo[2], g.hi[2]
    zg = synth.greville(M, a, b)
    prof = synth.ctap_profile(zg, 2.0, 0.6, 2.0, -2.0, 3.0)
    coeffs = np.stack([prof[0], prof[2]])
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    dt, n, every = 0.01, 30, 8
    prob = FidelityProblem(s, to_dev(psi0, s), gd.v0, gd.sigma, np.zeros(g.n[2]), M, (a, b), gd.x_lo, gd.x_hi,
                           dt, n, every)
    c = torch.tensor(coeffs, dtype=torch.float64, requires_grad=True)
    F = FidelityFn.apply(c, prob)
    F.backward()
    grad = c.grad.numpy()
    # oracle: F and dF/dxc on the same profile, chain rule with the oracle's own B-splines
    xc = prob.profile(coeffs)
    F_ref, G_ref, _ = oracle.adjoint_ctap(psi0, g.lo, g.hi, gd.v0, gd.sigma, xc, dt, n, gd.x_hi)
    Bo = oracle.bspline_basis(M, a, b, g.axis(2))
    grad_ref = np.stack([G_ref[0] @ Bo, G_ref[2] @ Bo])
    assert abs(float(F) - F_ref) < 1e-12
    assert np.max(np.abs(grad - grad_ref)) < 1e-10 * np.max(np.abs(grad_ref))
    # central finite differences through the GPU forward path
    for k, m in [(0, 3), (1, 4)]:
        h = 1e-4
        cp, cm = coeffs.copy(), coeffs.copy()
        cp[k, m] += h
        cm[k, m] -= h
        fd = (prob.forward(cp) - prob.forward(cm)) / (2 * h)
        assert abs(fd - grad[k, m]) < 1e-6 * max(1.0, abs(fd)), (k, m, fd, grad[k, m])
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(16, 32, 64), (12, 20, 40), (64, 24, 32), (20, 12, 96), (4, 12, 512)])
def test_tile_variants_and_tuner(dtype, shape):
    say("tile variants", dtype, shape)
    nz, ny, nx = shape
    g = synth.Grid((nx, ny, nz), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    rng = np.random.default_rng(17)
    x = rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape)
    psi0 = synth.random_field(g, 9, smooth=2.0)
    V = rng.uniform(-8, 8, g.shape)
    if dtype == "c64":
        x, psi0 = c64_round(x), c64_round(psi0)
    tol_fft = 1e-13 if dtype == "c128" else 2e-7
    tol_step = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(5 * 20)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    ref_step, _ = oracle.step(psi0, V, g.lo, g.hi, 0.01, 20)
    for choice in ([0, 1, 1], [0, 0, 1], [0, 1, 0], [0, 2, 2], [0, 2, 0], [0, 0, 2]):
        s.set_tiles(choice)
        assert s.get_tiles() == choice
        for axis in (1, 2):
            t = to_dev(x, s)
            s.fft(t, axes=(axis,))
            assert rel(host(t), oracle.fft_axis(x, axis, -1)) < tol_fft, (choice, axis)
        t = to_dev(psi0, s)
        s.step(t, 20, 0.01)
        assert rel(host(t), ref_step) < tol_step, choice
    choice, us = s.tune(reps=2)
    assert choice[0] == 0 and choice[1] in (0, 1, 2) and choice[2] in (0, 1, 2)
    assert all(v > 0 for v in us.values())
    t = to_dev(psi0, s)
    s.step(t, 20, 0.01)
    assert rel(host(t), ref_step) < tol_step
    s.close()


@pytest.mark.parametrize("n", [96, 128, 160])
def test_complex64_norm_holds_for_every_tile_variant(n):
    """A sweep-size instance (n^3, complex64, dt = 0.004) over 500 steps with
    each y/z tile variant: the norm stays within 2e-7 of its start.  Storage
    rounding alone moves it by a few 1e-8; FP32 exchanges in the 96-point
    single-transform passes lost 1e-6 in 500 steps."""
    say("complex64 norm, every tile variant", n)
    cfg = synth.config4(96)
    it = [i for i in cfg["instances"] if tuple(i["grid"].n) == (n, n, n)][0]
    g, gd = it["grid"], it["guides"]
    psi0 = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, it["z0"]), width=(0.4, 0.4, it["zwidth"]),
                                 k=(0.0, 0.0, it["kz"]))
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    for choice in ([0, 0, 0], [0, 1, 1], [0, 2, 2]):
        s.set_tiles(choice)
        t = to_dev(psi0, s)
        n0 = float(torch.sum(torch.abs(t.to(torch.complex128)) ** 2) * g.dv)
        rec = s.step(t, 500, cfg["dt"], obs_every=250)
        drift = [float(r["norm"]) - n0 for r in rec]
        say("tiles", choice, "norm drift", drift)
        assert max(abs(d) for d in drift) < 2e-7, (choice, drift)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_plain_copy_is_bitwise(dtype):
    say("copy", dtype)
    g = synth.Grid((24, 20, 40), (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    x = to_dev(synth.random_field(g, 3), s)
    y = s.empty()
    s.copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    with pytest.raises(ssf.SSFError):
        s.copy(x, x)
    s.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gradient_workload_copy_vs_oracle_adjoint(dtype):
    """The gradient workload on a 48 x 48 x 96 copy of its box (16 B-spline
    coefficients per moving guide, seeded), 200 steps with checkpoints every
    64: F and dF/dc through the autograd function against the oracle's
    stored-state adjoint, and central differences (h = 1e-3) in complex128."""
    say("gradient workload copy", dtype)
    from paper_1309_2451_amd.fidelity import FidelityFn, FidelityProblem
    cfg = synth.config5(n=(48, 48, 96))
    g = cfg["grid"]
    a, b = cfg["zrange"]
    M, dt, n = cfg["M"], cfg["dt"], 200
    nominal = synth.ctap_profile(g.axis(2), 3.0, 1.2, 6.0, -6.0, 8.0)
    z0 = -8.0
    iz = int(round((z0 - g.lo[2]) / g.spacing(2)))
    psi0 = synth.gaussian_packet(g, centre=(nominal[0, iz], 0.0, z0), width=(0.5, 0.5, 3.0), k=(0.0, 0.0, 3.0))
    if dtype == "c64":
        psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    prob = FidelityProblem(s, to_dev(psi0, s), cfg["v0"], cfg["sigma"], np.zeros(g.n[2]), M, (a, b),
                           cfg["x_lo"], cfg["x_hi"], dt, n, cfg["ckpt_every"])
    c = torch.tensor(cfg["coeffs"], dtype=torch.float64, requires_grad=True)
    F = FidelityFn.apply(c, prob)
    F.backward()
    grad = c.grad.numpy()
    xc = prob.profile(cfg["coeffs"])
    F_ref, G_ref, _ = oracle.adjoint_ctap(psi0, g.lo, g.hi, cfg["v0"], cfg["sigma"], xc, dt, n, cfg["x_hi"])
    Bo = oracle.bspline_basis(M, a, b, g.axis(2))
    grad_ref = np.stack([G_ref[0] @ Bo, G_ref[2] @ Bo])
    scale = np.max(np.abs(grad_ref))
    say("F", float(F.detach()), F_ref, "max|grad|", scale)
    assert F_ref > 5e-5                       # the packet is in the coupling region
    err = np.max(np.abs(grad - grad_ref))
    say("max |grad - oracle| / max|grad|", err / scale)

    def central(k, m, h):
        cp, cm = cfg["coeffs"].copy(), cfg["coeffs"].copy()
        cp[k, m] += h
        cm[k, m] -= h
        return (prob.forward(cp) - prob.forward(cm)) / (2 * h)

    # the two largest gradient components (a relative check needs |g| well above the rounding of F / h)
    top = np.dstack(np.unravel_index(np.argsort(-np.abs(grad_ref), axis=None)[:2], grad_ref.shape))[0]
    h = 1e-3
    if dtype == "c128":
        assert abs(float(F.detach()) - F_ref) < 1e-12
        assert err < 1e-9 * scale
        for k, m in top:
            d1, d2 = central(k, m, h), central(k, m, h / 2)
            rich = (4.0 * d2 - d1) / 3.0                # O(h^4): removes the h^2 term of both
            say("central differences (%d, %d): h %.6e, h/2 %.6e, extrapolated %.6e, adjoint %.6e"
                % (k, m, d1, d2, rich, grad[k, m]))
            assert abs(rich - grad[k, m]) <= 1e-5 * abs(grad[k, m]), (k, m, rich, grad[k, m])
            assert abs(d2 - grad[k, m]) <= 1e-3 * abs(grad[k, m]), (k, m, d2, grad[k, m])
    else:
        assert abs(float(F.detach()) - F_ref) < 1e-6 * max(F_ref, 1e-3)
        assert err < 1e-4 * scale
        for k, m in top:
            d1 = central(k, m, h)
            say("c64 central difference (%d, %d): %.6e, adjoint %.6e" % (k, m, d1, grad[k, m]))
            assert abs(d1 - grad[k, m]) <= max(2e-2 * abs(grad[k, m]), 1e-3 * scale), (k, m, d1, grad[k, m])
    s.close()


def test_gradient_where_the_guides_couple():
    """The gradient workload's box with guides that couple (v0 = 20, sigma = 0.7,
    d0 = 2, delta = 0.6; the packet crosses the coupling region and ends with
    most of its population in the third guide), 48 x 48 x 128, 4000 steps:
    the adjoint gradient against Richardson-extrapolated central differences
    in complex128, and the complex64 gradient against the complex128 one."""
    from paper_1309_2451_amd.fidelity import FidelityFn, FidelityProblem
    g = synth.Grid((48, 48, 128), (-8.0, -8.0, -48.0), (8.0, 8.0, 48.0))
    M, dt, n, every = 16, 0.004, 4000, 100
    a, b = g.lo[2], g.hi[2]
    zg = synth.greville(M, a, b)
    prof = synth.ctap_profile(zg, 2.0, 0.6, 6.0, -6.0, 8.0)
    rng = np.random.default_rng(23)
    coeffs = np.stack([prof[0], prof[2]]) + 0.05 * rng.standard_normal((2, M))
    nominal = synth.ctap_profile(g.axis(2), 2.0, 0.6, 6.0, -6.0, 8.0)
    z0 = -24.0
    iz = int(round((z0 - g.lo[2]) / g.spacing(2)))
    psi0 = synth.gaussian_packet(g, centre=(nominal[0, iz], 0.0, z0), width=(0.5, 0.5, 3.0), k=(0.0, 0.0, 3.0))
    out = {}
    for dtype in ("c128", "c64"):
        say("coupled gradient", dtype)
        s = ssf.Solver(g.n, g.lo, g.hi, dtype)
        p0 = c64_round(psi0) if dtype == "c64" else psi0
        prob = FidelityProblem(s, to_dev(p0, s), np.full(3, 20.0), np.full(3, 0.7), np.zeros(g.n[2]), M, (a, b),
                               -1.0, 1.0, dt, n, every)
        c = torch.tensor(coeffs, dtype=torch.float64, requires_grad=True)
        F = FidelityFn.apply(c, prob)
        F.backward()
        out[dtype] = (float(F.detach()), c.grad.numpy().copy(), prob, s)
    F128, g128, prob, s = out["c128"]
    F64, g64 = out["c64"][0], out["c64"][1]
    scale = np.max(np.abs(g128))
    say("F c128 %.6f c64 %.6f, max|dF/dc| %.4e, c64 gradient error %.3e" % (F128, F64, scale,
                                                                          np.max(np.abs(g64 - g128)) / scale))
    assert F128 > 0.3                                   # most of the population transferred
    assert abs(F64 - F128) < 1e-4 * F128
    assert np.max(np.abs(g64 - g128)) < 1e-3 * scale
    top = np.dstack(np.unravel_index(np.argsort(-np.abs(g128), axis=None)[:2], g128.shape))[0]

    def central(k, m, h):
        cp, cm = coeffs.copy(), coeffs.copy()
        cp[k, m] += h
        cm[k, m] -= h
        return (prob.forward(cp) - prob.forward(cm)) / (2 * h)

    h = 1e-3
    for k, m in top:
        d1, d2 = central(k, m, h), central(k, m, h / 2)
        rich = (4.0 * d2 - d1) / 3.0
        say("central differences (%d, %d): extrapolated %.8e, adjoint %.8e" % (k, m, rich, g128[k, m]))
        assert abs(rich - g128[k, m]) <= 1e-5 * abs(g128[k, m]), (k, m, rich, g128[k, m])
    for dtype in ("c128", "c64"):
        out[dtype][3].close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_workload_vs_oracle(dtype):
    """The headline workload at its full size (256 x 256 x 512, three guides) in
    the configuration the bench times (tuned tiles, fused step chain): three
    steps against the oracle's three steps, element by element."""
    say("full-size workload", dtype)
    cfg = synth.config2()
    g, gd = cfg["grid"], cfg["guides"]
    psi0 = synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, cfg["z0"]), width=(0.4, 0.4, cfg["zwidth"]),
                                 k=(0.0, 0.0, cfg["kz"]))
    if dtype == "c64":
        psi0 = c64_round(psi0)
    s = ssf.Solver(g.n, g.lo, g.hi, dtype)
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    s.tune(reps=3)
    t = to_dev(psi0, s)
    n = 3
    s.step(t, n, cfg["dt"])
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, cfg["dt"], n)
    got = host(t)
    del t
    tol = 1e-12 if dtype == "c128" else 3 * 6e-8 * np.sqrt(4 * n + 2)
    err = rel(got, ref)
    say("rel L2", err)
    assert err < tol
    # the largest pointwise deviation relative to the field's peak
    assert np.max(np.abs(got - ref)) < (1e-12 if dtype == "c128" else 1e-6) * np.max(np.abs(ref))
    s.close()


def test_zero_steps_and_sparse_observations():
    g = synth.Grid((16, 12, 20), (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    V = synth.harmonic_table(g)
    s.set_potential_table(torch.from_numpy(V).to(DEV))
    psi0 = synth.gaussian_packet(g, centre=(0.5, 0.0, 0.0))
    t = to_dev(psi0, s)
    assert s.step(t, 0, 0.01) is None
    assert np.array_equal(host(t), psi0)
    obs = s.step(t, 7, 0.01, obs_every=10)              # no observation falls due
    assert obs is None
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, 0.01, 7)
    assert rel(host(t), ref) < 1e-12
    with pytest.raises(ssf.SSFError):
        s.step(t, -1, 0.01)
    with pytest.raises(ssf.SSFError):
        s.step(t, 1, float("nan"))
    s.close()


def test_full_size_512_cube_vs_oracle():
    """The 512^3 workload (seeded +-5 % guides) in complex64 at its full size,
    tuned tiles, fused chain: two steps against the oracle."""
    say("512^3 workload c64")
    cfg = synth.config3()
    g, gd = cfg["grid"], cfg["guides"]
    psi0 = c64_round(synth.gaussian_packet(g, centre=(gd.xc[0, 0], 0.0, cfg["z0"]), width=(0.4, 0.4, cfg["zwidth"]),
                                           k=(0.0, 0.0, cfg["kz"])))
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    s.set_guides(gd.v0, gd.sigma, gd.xc)
    s.set_partition(gd.x_lo, gd.x_hi)
    s.tune(reps=2)
    t = to_dev(psi0, s)
    n = 2
    s.step(t, n, cfg["dt"])
    V = oracle.ctap_potential(g.shape, g.lo, g.hi, gd.v0, gd.sigma, gd.xc)
    ref, _ = oracle.step(psi0, V, g.lo, g.hi, cfg["dt"], n)
    del V
    err = rel(host(t), ref)
    say("rel L2", err)
    assert err < 3 * 6e-8 * np.sqrt(4 * n + 2)
    s.close()


def test_gradient_workload_full_size_vs_oracle_adjoint():
    """The gradient workload at its full size (128 x 128 x 256, 2 x 16 B-spline
    coefficients) in complex128 through the autograd function, 24 steps with
    checkpoints every 8, against the oracle's stored-state adjoint."""
    say("gradient workload full size")
    from paper_1309_2451_amd.fidelity import FidelityFn, FidelityProblem
    cfg = synth.config5()
    g = cfg["grid"]
    a, b = cfg["zrange"]
    M, dt, n = cfg["M"], cfg["dt"], 24
    # a packet straddling the target-guide boundary, so that F and its gradient are O(1e-1)
    psi0 = synth.gaussian_packet(g, centre=(0.8, 0.0, -8.0), width=(1.0, 0.8, 3.0), k=(0.0, 0.0, 3.0))
    s = ssf.Solver(g.n, g.lo, g.hi, "c128")
    prob = FidelityProblem(s, to_dev(psi0, s), cfg["v0"], cfg["sigma"], np.zeros(g.n[2]), M, (a, b),
                           cfg["x_lo"], cfg["x_hi"], dt, n, 8)
    c = torch.tensor(cfg["coeffs"], dtype=torch.float64, requires_grad=True)
    F = FidelityFn.apply(c, prob)
    F.backward()
    grad = c.grad.numpy()
    xc = prob.profile(cfg["coeffs"])
    F_ref, G_ref, _ = oracle.adjoint_ctap(psi0, g.lo, g.hi, cfg["v0"], cfg["sigma"], xc, dt, n, cfg["x_hi"])
    Bo = oracle.bspline_basis(M, a, b, g.axis(2))
    grad_ref = np.stack([G_ref[0] @ Bo, G_ref[2] @ Bo])
    scale = np.max(np.abs(grad_ref))
    say("F", float(F.detach()), F_ref, "max|grad|", scale)
    assert F_ref > 1e-2 and scale > 1e-4
    assert abs(float(F.detach()) - F_ref) < 1e-12
    assert np.max(np.abs(grad - grad_ref)) < 1e-9 * scale
    s.close()


def test_tune_cache_round_trip(tmp_path):
    """ssf_tune_cached: a miss tunes and appends one line, a hit applies the
    stored choice without tuning, other grids get their own lines, unparsable
    lines are ignored and the last matching line wins."""
    path = tmp_path / "tiles.txt"
    g = synth.Grid((32, 24, 40), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    s = ssf.Solver(g.n, g.lo, g.hi, "c64")
    ch, hit = s.tune_cached(path, reps=2)
    assert not hit and ch[0] == 0 and ch[1] in (0, 1, 2) and ch[2] in (0, 1, 2)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and " 32x24x40 c64 f64 " in lines[0]
    s2 = ssf.Solver(g.n, g.lo, g.hi, "c64")
    ch2, hit2 = s2.tune_cached(path, reps=2)
    assert hit2 and ch2 == ch and s2.get_tiles() == ch
    g3 = synth.Grid((16, 24, 40), (-4.0, -3.0, -5.0), (4.0, 3.0, 5.0))
    s3 = ssf.Solver(g3.n, g3.lo, g3.hi, "c128")
    _, hit3 = s3.tune_cached(path, reps=2)
    assert not hit3 and len(path.read_text().splitlines()) == 2
    other = [v for v in (0, 1, 2) if v != ch[2]][0]
    with open(path, "a") as f:
        f.write("garbage line\n")
        f.write(lines[0].split(" | ")[0] + " | %d %d\n" % (ch[1], other))
    s4 = ssf.Solver(g.n, g.lo, g.hi, "c64")
    ch4, hit4 = s4.tune_cached(path, reps=2)
    assert hit4 and ch4 == [0, ch[1], other]
    # the stored choice gives the oracle's transform
    rng = np.random.default_rng(3)
    x = c64_round(rng.standard_normal(g.shape) + 1j * rng.standard_normal(g.shape))
    t = to_dev(x, s4)
    s4.fft(t, axes=(2,))
    assert rel(host(t), oracle.fft_axis(x, 2, -1)) < 2e-7
    for h in (s, s2, s3, s4):
        h.close()
