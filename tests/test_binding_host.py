"""Host-side argument checks of the Python binding (no device needed): every
buffer handed to a kernel is a contiguous device tensor of the right type and
exactly the size the kernel indexes."""
import numpy as np
import pytest
import torch

from paper_2607_26901_amd import ccfr


class FakeDev:
    """Stands in for a device tensor: the checks read only these attributes."""

    def __init__(self, t: torch.Tensor, contiguous=True):
        self.t = t
        self.is_cuda = True
        self.dtype = t.dtype
        self._contig = contiguous

    def numel(self):
        return self.t.numel()

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        return 4096


def test_dev_accepts_exact_buffer():
    p = ccfr._dev(FakeDev(torch.zeros(12, 3)), "float32", 36, "x")
    assert p.value == 4096


@pytest.mark.parametrize("t,numel,msg", [
    (torch.zeros(12, 3), 36, "device"),                          # host tensor
    (FakeDev(torch.zeros(11, 3)), 36, "elements"),               # one vertex short
    (FakeDev(torch.zeros(12, 3, dtype=torch.float64)), 36, "dtype"),
    (FakeDev(torch.zeros(12, 3), contiguous=False), 36, "contiguous"),
    (None, 36, "required"),
])
def test_dev_refuses(t, numel, msg):
    with pytest.raises(ValueError, match=msg):
        ccfr._dev(t, "float32", numel, "x")


def test_dev_empty_and_optional():
    assert ccfr._dev(None, "float32", 0, "x") is None
    assert ccfr._dev(None, "uint8", 10, "halted", optional=True) is None
    assert ccfr._dev(FakeDev(torch.zeros(0, 3)), "float32", 0, "x") is None


def test_host_exact():
    a, p = ccfr._host_exact(np.arange(6), np.float32, 2, 3, "x")
    assert a.dtype == np.float32 and p is not None
    assert ccfr._host_exact(None, np.float32, 2, 3, "x") == (None, None)
    with pytest.raises(ValueError, match="expected 6"):
        ccfr._host_exact(np.arange(5), np.float32, 2, 3, "x")
