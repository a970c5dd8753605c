"""The measurement probes behind the measured roofline denominators: the
copy moves the right bytes and both rates are physically plausible (below
the datasheet peaks of 8 TB/s and 2.5 PFLOP/s dense BF16)."""
import pytest

from tests.helpers import device, hgl

pytestmark = pytest.mark.gpu


def test_measured_peaks():
    dev = device()
    pk = hgl().measure_peaks(dev, copy_bytes=1 << 29, reps=3)
    assert 1000.0 < pk["hbm_gbs"] < 8000.0 * 1.05
    assert 100.0 < pk["bf16_mfma_tflops"] < 2500.0 * 1.05


def test_peak_copy_arguments():
    import ctypes as C

    import torch
    from paper_1908_08281_amd import _lib
    dev = device()
    lib = _lib.load()
    a = torch.arange(1000, dtype=torch.int32, device=dev)
    b = torch.zeros_like(a)
    st = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    assert lib.hgl_peak_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 4000, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert lib.hgl_peak_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), 4001, st) == _lib.HGL_EINVAL
