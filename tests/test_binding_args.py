"""Argument checks of the ctypes binding, before any pointer reaches the library.

Every device buffer crosses the C ABI as a bare address whose extent the library
derives from the problem sizes, so the binding must refuse a tensor whose dtype
or element count does not match that extent.  These checks run on CPU tensors
(no GPU needed): each rule is tested on a tensor that breaks only that rule.
"""
import pytest

torch = pytest.importorskip("torch")
em = pytest.importorskip("paper_2302_05804_amd.em")


def test_image_buffers_must_be_float32():
    for dt in (torch.uint8, torch.float64, torch.float16, torch.int32):
        with pytest.raises(TypeError, match="float32"):
            em._dev_ptr(torch.zeros(12, dtype=dt), "y", 12)


def test_byte_tensor_with_the_float_count_is_refused():
    # n*Hf*Wf bytes hold a quarter of the floats the library would read
    with pytest.raises(TypeError, match="must be float32, not uint8"):
        em._dev_ptr(torch.zeros(4 * 8 * 8, dtype=torch.uint8), "y", 4 * 8 * 8)


def test_workspace_must_be_bytes():
    with pytest.raises(TypeError, match="uint8"):
        em._ws_ptr(torch.zeros(256, dtype=torch.float32))


def test_element_count_and_layout():
    with pytest.raises(ValueError, match="11 elements, 12 expected"):
        em._dev_ptr(torch.zeros(11), "v", 12)
    with pytest.raises(ValueError, match="contiguous"):
        em._dev_ptr(torch.zeros(4, 6).t(), "psf", 24)


def test_host_tensor_is_refused_after_the_other_checks():
    with pytest.raises(TypeError, match="CUDA"):
        em._dev_ptr(torch.zeros(12), "x", 12)
    with pytest.raises(TypeError, match="CUDA"):
        em._ws_ptr(torch.zeros(256, dtype=torch.uint8))
    with pytest.raises(TypeError, match="CUDA"):
        em._dev_ptr([0.0] * 12, "x", 12)


def test_absent_optional_buffer_is_null():
    assert em._dev_ptr(None, "x0", 12) is None
