"""C-ABI boundary tests that need no GPU: the library loads, exports every
function include/ssf.h declares, validates arguments before touching a device,
and its host helpers agree with the oracle's independent implementation."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ssfpkg = pytest.importorskip("paper_1309_2451_amd")
from paper_1309_2451_amd import _ssf  # noqa: E402


def _lib():
    try:
        return _ssf.load()
    except ImportError as e:
        pytest.skip(str(e))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ssf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ssf_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    lib = _lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_ssf.EXPORTS)


def test_supported_lengths():
    lib = _lib()
    src = open(os.path.join(ROOT, "paper_1309_2451_amd", "csrc", "ssf_internal.hpp")).read()
    block = re.search(r"#define SSF_LENGTHS\(X\)(.*?)\n\n", src, re.S).group(1)
    lengths = [int(v) for v in re.findall(r"X\((\d+)\)", block)]
    for n in lengths:
        assert lib.ssf_supported_length(n) == 1
    for n in (0, -1, 3, 7, 11, 1000, 2048):
        assert lib.ssf_supported_length(n) == 0
    # every length of the workloads is built in
    for n in (64, 96, 128, 160, 256, 512, 48):
        assert lib.ssf_supported_length(n) == 1


def _grid(n=(8, 8, 8), lo=(0, 0, 0), hi=(1, 1, 1)):
    g = _ssf.ssf_grid_desc()
    for a in range(3):
        g.n[a], g.lo[a], g.hi[a] = n[a], lo[a], hi[a]
    return g


def test_create_validates_before_the_device():
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.ssf_create(None, 2, None, ctypes.byref(h)) == _ssf.SSF_E_INVALID
    assert lib.ssf_create(ctypes.byref(_grid()), 3, None, ctypes.byref(h)) == _ssf.SSF_E_INVALID
    assert lib.ssf_create(ctypes.byref(_grid(n=(8, 0, 8))), 2, None, ctypes.byref(h)) == _ssf.SSF_E_INVALID
    assert lib.ssf_create(ctypes.byref(_grid(hi=(1, 0, 1))), 2, None, ctypes.byref(h)) == _ssf.SSF_E_INVALID
    assert lib.ssf_create(ctypes.byref(_grid(n=(7, 8, 8))), 2, None, ctypes.byref(h)) == _ssf.SSF_E_UNSUPPORTED
    assert b"7" in lib.ssf_last_error()


def test_null_handle_is_rejected():
    lib = _lib()
    for name, args in [("ssf_step", (None, None, 1, 0.1, 0, 0, None)), ("ssf_fft", (None, None, 7, 0)),
                       ("ssf_sync", (None,)), ("ssf_set_partition", (None, -1.0, 1.0)),
                       ("ssf_observables", (None, None, None)), ("ssf_adjoint_init", (None, None, None))]:
        assert getattr(lib, name)(*args) == _ssf.SSF_E_INVALID, name
    assert lib.ssf_destroy(None) == _ssf.SSF_OK
    assert lib.ssf_status_string(_ssf.SSF_E_NONFINITE) == b"non-finite norm observed"


def test_create_without_device_reports_nodevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    lib = _lib()
    h = ctypes.c_void_p()
    assert lib.ssf_create(ctypes.byref(_grid()), 2, None, ctypes.byref(h)) == _ssf.SSF_E_NODEVICE


@pytest.mark.parametrize("M", [4, 9, 16])
def test_bspline_host_helper_matches_oracle(M):
    import oracle
    z = np.linspace(-48.0, 48.0, 301)
    B = ssfpkg.bspline_basis(M, -48.0, 48.0, z)
    Bo = oracle.bspline_basis(M, -48.0, 48.0, z)
    assert np.max(np.abs(B - Bo)) < 1e-14
    with pytest.raises(ssfpkg.SSFError):
        ssfpkg.bspline_basis(3, -1.0, 1.0, z)


@pytest.mark.parametrize("M", [4, 16])
def test_bspline_profile_helper_matches_oracle(M):
    """The guide-centre map x_k(z) = sum_m c_km B_m(z) that the gradient
    workload evaluates in the library, against the oracle's basis times the
    coefficients (the transpose of the map ssf_profile_grad applies)."""
    import oracle
    z = np.linspace(-48.0, 48.0, 257)
    c = np.random.default_rng(M).standard_normal((2, M))
    prof = ssfpkg.bspline_eval(M, -48.0, 48.0, c, z)
    Bo = oracle.bspline_basis(M, -48.0, 48.0, z)
    assert prof.shape == (2, z.size)
    assert np.max(np.abs(prof - c @ Bo.T)) < 1e-13 * np.max(np.abs(c))
    with pytest.raises(ValueError):
        ssfpkg.bspline_eval(M, -48.0, 48.0, np.zeros((2, M + 1)), z)
    lib = _lib()
    assert lib.ssf_bspline_eval(3, -1.0, 1.0, None, 1, None, 1, None) == _ssf.SSF_E_INVALID
