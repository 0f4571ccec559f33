"""Pins of the oracle's FFT against definitions that do not use it.

- brute-force DFT matrices built from the defining sum (exp(-2 pi i j k/n)),
- numpy.fft (an independent library) at the production lengths,
- inverse(forward(x)) = x and Parseval's identity.
A transposed axis, a wrong twiddle index or sign, or a wrong radix-3/5 stage
fails one of these.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")

LENGTHS_1D = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 15, 16, 25, 27, 48, 64, 96, 128, 160, 256, 512]


def dft_matrix(n, sign=-1):
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("n", LENGTHS_1D)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft1d_vs_bruteforce(n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = dft_matrix(n, sign) @ x
    got = oracle.fft1d(x, sign)
    assert rel(got, ref) < 1e-13 * max(1.0, np.log2(max(n, 2)))


@pytest.mark.parametrize("n", [48, 96, 160, 256, 512, 1024])
def test_fft1d_vs_numpy(n):
    rng = np.random.default_rng(7 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert rel(oracle.fft1d(x, -1), np.fft.fft(x)) < 1e-14
    assert rel(oracle.fft1d(x, +1), np.fft.ifft(x) * n) < 1e-14


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 6), (5, 3, 4), (1, 8, 8), (8, 1, 1)])
def test_fft3d_vs_bruteforce(shape):
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    # defining sum, axis by axis: X[kz,ky,kx] = sum psi[z,y,x] e^{-2 pi i (kx x/nx + ky y/ny + kz z/nz)}
    ref = np.einsum("az,by,cx,zyx->abc", dft_matrix(nz), dft_matrix(ny), dft_matrix(nx), psi)
    got = oracle.fft3d(psi, -1)
    assert rel(got, ref) < 1e-13
    back = oracle.fft3d(got, +1)
    assert rel(back, psi) < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fft_axis_selects_the_right_axis(axis):
    shape = (6, 10, 12)  # (nz, ny, nx): all different so a swapped axis cannot pass
    rng = np.random.default_rng(axis)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np_axis = 2 - axis
    ref = np.fft.fft(psi, axis=np_axis)
    assert rel(oracle.fft_axis(psi, axis, -1), ref) < 1e-14


def test_fft3d_numpy_and_parseval_production_shape():
    shape = (40, 48, 32)
    rng = np.random.default_rng(1)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    X = oracle.fft3d(psi, -1)
    assert rel(X, np.fft.fftn(psi)) < 1e-14
    # Parseval: sum |X|^2 = N sum |x|^2
    N = psi.size
    assert abs(np.sum(np.abs(X) ** 2) - N * np.sum(np.abs(psi) ** 2)) / (N * np.sum(np.abs(psi) ** 2)) < 1e-14


def test_kgrid_matches_momentum_bound():
    # Sec. IV: p_max = pi N / L.  Bins 0..N/2-1 positive, N/2..N-1 negative.
    k = oracle.kgrid(64, 16.0)
    assert k[0] == 0.0
    assert np.isclose(k[1], 2 * np.pi / 16.0, rtol=0, atol=1e-15)
    assert np.isclose(-k[32], np.pi * 64 / 16.0, rtol=1e-15)
    assert np.max(np.abs(k)) <= np.pi * 64 / 16.0 + 1e-12
    assert np.allclose(k, 2 * np.pi * np.fft.fftfreq(64, d=16.0 / 64), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 5, 7, 48])
def test_kgrid_odd_and_unit_lengths(n):
    # bins 0..floor((n-1)/2) non-negative, the rest negative; a 1-point axis has k = 0
    L = 3.0
    ref = 2 * np.pi * np.fft.fftfreq(n, d=L / n)
    assert np.allclose(oracle.kgrid(n, L), ref, rtol=0, atol=1e-13)
