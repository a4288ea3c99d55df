"""Host-side argument checks of the Python binding (no GPU): a caller's
output buffer with the wrong dtype, device, layout or size is refused before
the library could write past its end."""
import pytest
import torch

from paper_2302_00414_amd.nfft import check_out


def test_accepts_matching_buffer():
    out = torch.empty((2, 16), dtype=torch.complex64)
    check_out(out, torch.complex64, torch.device("cpu"), 32)
    check_out(out, torch.complex64, torch.device("cpu"), 20)  # larger buffers are fine


@pytest.mark.parametrize("out,why", [
    (torch.empty(32, dtype=torch.complex128), "dtype"),
    (torch.empty(32, dtype=torch.float32), "dtype"),
    (torch.empty(31, dtype=torch.complex64), "elements"),
    (torch.empty((16, 4), dtype=torch.complex64).t(), "contiguous"),
])
def test_rejects_bad_buffer(out, why):
    with pytest.raises(ValueError, match=why):
        check_out(out, torch.complex64, torch.device("cpu"), 32)


def test_rejects_other_device():
    out = torch.empty(32, dtype=torch.complex64)
    with pytest.raises(ValueError, match="device"):
        check_out(out, torch.complex64, torch.device("cuda:0"), 32)


def test_rejects_non_tensor():
    with pytest.raises(ValueError, match="Tensor"):
        check_out([0j] * 32, torch.complex64, torch.device("cpu"), 32)
