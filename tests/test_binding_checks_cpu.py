"""The Python binding refuses output arrays the library would misuse (wrong
element type, host memory, another device, a strided view, a capacity
beyond the array) before anything reaches the C interface.  Runs without a
GPU: torch CPU tensors and small stand-ins with the attributes the check
reads."""

import pytest
import torch

import paper_1411_2484_amd as ph


class FakeDev:
    def __init__(self, index):
        self.index = index


class FakeTensor:
    """Looks like a device tensor to the binding's check."""

    def __init__(self, dtype, n=16, device=0, contiguous=True):
        self.dtype = dtype
        self.is_cuda = True
        self.device = FakeDev(device)
        self._n = n
        self._contig = contiguous

    def is_contiguous(self):
        return self._contig

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def test_accepts_matching_device_arrays():
    p32, p64, pr, cap = ph._outputs(FakeTensor(torch.int32), FakeTensor(torch.int64, 20), FakeTensor(torch.float64),
                                    0, None)
    assert (p32, p64, pr, cap) == (0x1000, 0x1000, 0x1000, 16)
    assert ph._outputs(None, None, FakeTensor(torch.float64, 8), 0, 5)[3] == 5
    assert ph._outputs(None, None, None, 0, None)[3] == 0


@pytest.mark.parametrize("which,dtype", [(0, torch.float32), (0, torch.int64), (1, torch.int32), (1, torch.float64),
                                         (2, torch.float32), (2, torch.int64)])
def test_rejects_wrong_element_type(which, dtype):
    outs = [None, None, None]
    outs[which] = FakeTensor(dtype)
    with pytest.raises(TypeError):
        ph._outputs(*outs, 0, None)


def test_rejects_host_tensors():
    for outs in ((torch.zeros(8, dtype=torch.int32), None, None), (None, torch.zeros(8, dtype=torch.int64), None),
                 (None, None, torch.zeros(8, dtype=torch.float64))):
        with pytest.raises(ValueError):
            ph._outputs(*outs, 0, None)


def test_rejects_other_device_and_strided_views():
    with pytest.raises(ValueError):
        ph._outputs(None, None, FakeTensor(torch.float64, device=1), 0, None)
    with pytest.raises(ValueError):
        ph._outputs(None, None, FakeTensor(torch.float64, contiguous=False), 0, None)


def test_rejects_capacity_beyond_an_array():
    with pytest.raises(ValueError):
        ph._outputs(FakeTensor(torch.int32, 10), None, FakeTensor(torch.float64, 100), 0, 50)


def test_generate_checks_before_the_library():
    """Context.generate runs the checks before calling phprng_generate: a
    context object that is never created on a device still raises the
    binding's error, not a device error."""
    ctx = ph.Context.__new__(ph.Context)
    ctx._h = None
    ctx.device = 0
    reqs = ph.make_requests([0], [4], [0])
    with pytest.raises(TypeError):
        ctx.generate(reqs, None, None, FakeTensor(torch.float32))
    with pytest.raises(ValueError):
        ctx.generate(reqs, None, None, torch.zeros(4, dtype=torch.float64))
    with pytest.raises(TypeError):
        ctx.generate_noalloc(reqs, FakeTensor(torch.float64), None, None)
