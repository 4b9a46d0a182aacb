"""The measurement probes on the device: the stream probe's copy really
copies, and both probes report rates in a plausible range.  The buffers
are 1 GiB each, well beyond the 256 MB last-level cache, so the copy runs
at HBM speed (under 10 TB/s)."""
import ctypes

import pytest
import torch

import paper_2206_06079_amd as ohm
from gpu_helpers import device
from paper_2206_06079_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("read_only", [False, True])
def test_stream_probe(read_only):
    n = (1 << 30) + 4096  # not a multiple of the grid's stride: the tail loop runs
    src = torch.arange(n // 4, dtype=torch.int32, device=device()).view(torch.uint8)
    dst = torch.zeros(n, dtype=torch.uint8, device=device())
    rate = ctypes.c_double(0.0)
    st = _lib.load().ohm_probe_stream_rate(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n,
                                           _lib.PROBE_READ_ONLY if read_only else 0, ctypes.byref(rate), None)
    assert st == _lib.OHM_OK
    torch.cuda.synchronize()
    if not read_only:
        assert torch.equal(src, dst)
    assert 1e11 < rate.value < 1e13


def test_atomic_probe_rates():
    rnd = ohm.probe_atomic_rate(64 << 20)
    seq = ohm.probe_atomic_rate(64 << 20, sequential=True)
    cas = ohm.probe_atomic_rate(64 << 20, op="f32_cas")
    u64 = ohm.probe_atomic_rate(64 << 20, op="u64_add")
    assert 1e9 < rnd < seq
    assert cas > 1e8 and u64 > 1e9
