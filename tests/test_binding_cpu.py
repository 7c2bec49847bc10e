"""CPU checks of the Python binding's argument checks: caller-supplied
buffers of the wrong kind (host tensors, wrong dtype, too small,
non-contiguous) are refused with ValueError before anything reaches the
library, so no launch can read or write past a buffer.  No device is
needed: every refusal happens before the first device call."""
import pytest
import torch

import paper_cs_0607001_amd as S


def test_host_tensors_are_refused():
    with pytest.raises(ValueError, match="device"):
        S._check_buf(torch.zeros(16, dtype=torch.complex64), torch.complex64, 16, "out")
    with pytest.raises(ValueError, match="device"):
        S._check_pulses(torch.zeros((2, 16), dtype=torch.complex64), torch.complex64)
    with pytest.raises(ValueError, match="device"):
        S.lift_many("cdf97", 3, torch.zeros((2, 64), dtype=torch.complex64))
    with pytest.raises(ValueError, match="device"):
        S.synth_many("cdf97", 3, torch.zeros((2, 64), dtype=torch.complex64))


def test_non_tensors_are_refused():
    with pytest.raises(ValueError, match="tensor"):
        S._check_buf([0.0] * 16, torch.complex64, 16, "out")


def test_unknown_filters_and_levels_are_refused():
    x = torch.zeros((2, 64), dtype=torch.complex64)
    with pytest.raises(ValueError, match="filter"):
        S.lift_many("haar", 3, x)
    with pytest.raises(ValueError, match="filter"):
        S.synth_many("haar", 3, x)


@pytest.mark.gpu
def test_device_buffers_of_the_wrong_kind_are_refused():
    d = torch.device("cuda:0")
    ok = torch.zeros(64, dtype=torch.complex64, device=d)
    S._check_buf(ok, torch.complex64, 64, "out")
    with pytest.raises(ValueError, match="needs"):
        S._check_buf(ok, torch.complex64, 65, "out")
    with pytest.raises(ValueError, match="must be"):
        S._check_buf(ok.view(torch.float32), torch.complex64, 64, "out")
    with pytest.raises(ValueError, match="contiguous"):
        S._check_buf(torch.zeros((8, 16), dtype=torch.complex64, device=d)[:, ::2],
                     torch.complex64, 8, "out")
