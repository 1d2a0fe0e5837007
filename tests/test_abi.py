"""C-ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments before any device work."""
import ctypes

import pytest

from paper_cs_0103001_amd import _binding as B

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False


def test_library_exports_header_functions():
    lib = B.lib()
    names = B.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert lib.fft_version() == 0x000100


def test_strerror_texts():
    for code in (B.FFT_OK, B.FFT_ERR_ARG, B.FFT_ERR_SIZE, B.FFT_ERR_UNSUPPORTED, B.FFT_ERR_WORKSPACE,
                 B.FFT_ERR_HIP, B.FFT_ERR_NOMEM, B.FFT_ERR_STATE, B.FFT_ERR_SCRATCH, -99):
        assert isinstance(B.strerror(code), str) and B.strerror(code)


def _plan_rc(rank, dims, batch, flags=0, null_out=False, null_dims=False):
    lib = B.lib()
    h = ctypes.c_void_p()
    arr = None if null_dims else (ctypes.c_int64 * len(dims))(*dims)
    rc = lib.fft_plan(None if null_out else ctypes.byref(h), rank, arr, batch, flags)
    return rc, h.value


@pytest.mark.parametrize("args,code", [
    (dict(rank=1, dims=[8], batch=1, null_out=True), B.FFT_ERR_ARG),
    (dict(rank=1, dims=[8], batch=1, null_dims=True), B.FFT_ERR_ARG),
    (dict(rank=3, dims=[8, 8, 8], batch=1), B.FFT_ERR_ARG),
    (dict(rank=0, dims=[8], batch=1), B.FFT_ERR_ARG),
    (dict(rank=1, dims=[8], batch=-1), B.FFT_ERR_ARG),
    (dict(rank=1, dims=[8], batch=1, flags=0x80), B.FFT_ERR_ARG),
    (dict(rank=1, dims=[12], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=1, dims=[0], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=1, dims=[-8], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=1, dims=[1 << 25], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=2, dims=[8, 6], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=2, dims=[1 << 15, 8], batch=1), B.FFT_ERR_SIZE),
    (dict(rank=2, dims=[8, 1 << 15], batch=1), B.FFT_ERR_SIZE),
])
def test_plan_argument_errors(args, code):
    rc, h = _plan_rc(**args)
    assert rc == code
    assert h is None


@pytest.mark.skipif(HAVE_GPU, reason="checks the no-device path")
def test_plan_without_device_reports_hip_error():
    rc, h = _plan_rc(1, [1024], 4)
    assert rc == B.FFT_ERR_HIP and h is None
    assert "HIP" in B.strerror(B.FFT_ERR_HIP)


def test_calls_reject_bad_plans():
    lib = B.lib()
    bogus = ctypes.c_void_p(0x1234)
    n = ctypes.c_size_t()
    assert lib.fft_plan_destroy(None) == B.FFT_OK
    assert lib.fft_plan_destroy(bogus) == B.FFT_ERR_ARG
    assert lib.fft_workspace_size(None, ctypes.byref(n)) == B.FFT_ERR_ARG
    assert lib.fft_workspace_size(bogus, ctypes.byref(n)) == B.FFT_ERR_ARG
    assert lib.fft_spectrum_size(bogus, ctypes.byref(n)) == B.FFT_ERR_ARG
    p = ctypes.c_void_p(0x10)
    assert lib.fft_exec(bogus, p, p, p, B.FFT_FORWARD, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter(bogus, p, p, None, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_noalloc(bogus, p, p, None, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_save(bogus, p, p, None, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mask_grad(bogus, p, p, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_grad(bogus, p, p, p, p, 1.0, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_grad(None, p, None, p, p, 1.0, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse(bogus, p, p, p, 1.0, p, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_spectral(bogus, p, p, p, 1.0, p, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_spectral(None, p, p, p, 1.0, p, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_spectral_grad(bogus, p, p, 1.0, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_mse_spectral_grad(None, p, p, 1.0, p, None) == B.FFT_ERR_ARG
    assert lib.fft2d_filter_ragged(bogus, p, p, None, p, None) == B.FFT_ERR_ARG


def test_mask_struct_layout_matches_header():
    # int kind; const float* data; double sigma_f, cutoff; int order; double b, c1, c2
    m = B.fft_mask
    assert m.kind.offset == 0 and m.data.offset == 8 and m.sigma_f.offset == 16
    assert m.cutoff.offset == 24 and m.order.offset == 32 and m.b.offset == 40
    assert m.c2.offset == 56 and ctypes.sizeof(m) == 64


def test_padded_plan_and_spectrum_argument_errors():
    lib = B.lib()
    h = ctypes.c_void_p()
    bad = (ctypes.c_int64 * 2)(0, 5)
    assert lib.fft_plan_padded(ctypes.byref(h), bad, 1, 0) == B.FFT_ERR_SIZE
    big = (ctypes.c_int64 * 2)(17000, 5)
    assert lib.fft_plan_padded(ctypes.byref(h), big, 1, 0) == B.FFT_ERR_SIZE
    ok = (ctypes.c_int64 * 2)(460, 506)
    assert lib.fft_plan_padded(None, ok, 1, 0) == B.FFT_ERR_ARG
    assert lib.fft_plan_padded(ctypes.byref(h), None, 1, 0) == B.FFT_ERR_ARG
    assert lib.fft_plan_padded(ctypes.byref(h), ok, -1, 0) == B.FFT_ERR_ARG
    p = ctypes.c_void_p(0x10)
    assert lib.fft2d_spectrum(ctypes.c_void_p(0x1234), p, p, p, None) == B.FFT_ERR_ARG
    assert lib.fft_plan_tune(ctypes.c_void_p(0x1234), p, p, None, p, None) == B.FFT_ERR_ARG


def test_plan_layout_rejects_bad_plans():
    lib = B.lib()
    rb = ctypes.c_int()
    assert lib.fft_plan_layout(None, ctypes.byref(rb), None, None, None) == B.FFT_ERR_ARG
    assert lib.fft_plan_layout(ctypes.c_void_p(0x1234), None, None, None, None) == B.FFT_ERR_ARG


def test_learnable_mask_wrappers_validate_before_any_launch():
    """Shape, dtype and device mismatches raise in Python before a kernel could
    read past a buffer (CPU tensors: the checks come before the device check)."""
    import torch
    from paper_cs_0103001_amd import api
    x = torch.zeros((2, 16, 16), dtype=torch.float32)
    mask = torch.ones((16, 16), dtype=torch.float32)
    with pytest.raises(ValueError):
        api.filter_mse(x, torch.zeros((1, 16, 16)), mask, 1.0)          # clean smaller than x
    with pytest.raises(ValueError):
        api.filter_mse(x, x, torch.ones((8, 16)), 1.0)                   # mask of another shape
    with pytest.raises(ValueError):
        api.filter_mse(x, x, torch.ones((16, 16), dtype=torch.float64), 1.0)
    with pytest.raises(TypeError):
        api.filter_mse(x.to(torch.complex64), x.to(torch.complex64), mask, 1.0)
    with pytest.raises(ValueError):
        api.mse_grad(x, torch.zeros((2, 16, 8)), torch.zeros(1, dtype=torch.uint8), mask, 1.0)
    with pytest.raises(ValueError):
        api.mse_grad(x, x, torch.zeros(1, dtype=torch.uint8), torch.ones((16, 8)), 1.0)
    with pytest.raises(TypeError):
        api.mse_grad(x, x.double(), torch.zeros(1, dtype=torch.uint8), mask, 1.0)
    with pytest.raises(ValueError):
        api.mask_grad(torch.zeros((16,), dtype=torch.complex64), torch.zeros(1, dtype=torch.uint8))


def test_entry_points_open_roctx_ranges():
    """The library names each entry point's device work with rocTX ranges
    (rocprofv3 --marker-trace shows them)."""
    import shutil
    import subprocess
    if not shutil.which("nm"):
        pytest.skip("nm not found")
    out = subprocess.run(["nm", "-D", B.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
