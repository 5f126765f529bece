"""The achievable-bandwidth yardsticks (include/amh_yardstick.h) read what their
header says: each output is reproduced exactly on the host (small-integer data, so
every float sum is exact) from the documented access pattern: the streaming read
touches every element once, the gathers read the 4 floats at the hashed row and bin
(both in range), the LDS kernel walks its documented index sequence."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402  (an import error fails the run)


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_2211_03193_amd import amh
    return amh, amh.lib()


def test_stream_reads_every_element_once():
    amh, L = _lib()
    n4, blocks = 100003, 37   # ragged against the grid of 37 x 256 threads
    src = (torch.arange(4 * n4, dtype=torch.int64) % 7).to(torch.float32).to(gu.DEV)
    sink = torch.full((blocks * 256,), -1.0, dtype=torch.float32, device=gu.DEV)
    amh.check(L.amh_yard_stream(amh._ptr(src), n4, blocks, amh._ptr(sink), amh._stream()))
    torch.cuda.synchronize()
    v = src.cpu().numpy().reshape(n4, 4).astype(np.float64)
    per = (v[:, 0] + v[:, 1]) + (v[:, 2] + v[:, 3])
    T = blocks * 256
    want = np.array([per[t::T].sum() for t in range(T)])
    assert np.array_equal(sink.cpu().numpy().astype(np.float64), want)


def _mix(x):
    x = x.astype(np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x7FEB352D) & 0xFFFFFFFF
    x ^= x >> 15
    x = (x * 0x846CA68B) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def test_gather_reads_the_hashed_rows_and_bins():
    amh, L = _lib()
    rows, stride, max_bin, per_thread, blocks = 4099, 40, 36, 9, 5
    tab = ((torch.arange(rows * stride, dtype=torch.int64) * 13) % 17).to(torch.float32)
    table = tab.to(gu.DEV)
    sink = torch.full((blocks * 256,), -1.0, dtype=torch.float32, device=gu.DEV)
    amh.check(L.amh_yard_gather(amh._ptr(table), rows, stride, max_bin, per_thread, blocks,
                                amh._ptr(sink), amh._stream()))
    torch.cuda.synchronize()
    t = np.arange(blocks * 256, dtype=np.uint64)
    h = _mix((t * 0x9E3779B9 + 1) & 0xFFFFFFFF)
    acc = np.zeros(t.size)
    tv = tab.numpy().astype(np.float64)
    for m in range(per_thread):
        h = _mix((h + m) & 0xFFFFFFFF)
        row = (h * rows) >> 32
        b = (h >> 3) % (max_bin + 1)
        assert row.max() < rows and b.max() <= max_bin
        base = (row * stride + b).astype(np.int64)
        acc += (tv[base] + tv[base + 1]) + (tv[base + 2] + tv[base + 3])
    assert np.array_equal(sink.cpu().numpy().astype(np.float64), acc)
    with pytest.raises(amh.AmhError):   # a stencil reaching past the row is refused
        amh.check(L.amh_yard_gather(amh._ptr(table), rows, stride, stride - 3, 1, 1, amh._ptr(sink),
                                    amh._stream()))


def test_lds_walks_its_index_sequence():
    amh, L = _lib()
    per_thread, blocks = 64, 3
    sink = torch.full((blocks * 512,), -1.0, dtype=torch.float32, device=gu.DEV)
    amh.check(L.amh_yard_lds(per_thread, blocks, amh._ptr(sink), amh._stream()))
    torch.cuda.synchronize()
    want = np.zeros(512)
    for tid in range(512):
        idx, acc = (tid * 7) & 4095, 0.0
        for m in range(per_thread):
            acc += (idx + 1.0) + (2.0 + 3.0)
            idx = (idx + 64 + (m & 7)) & 4095
        want[tid] = acc
    assert np.array_equal(sink.cpu().numpy().astype(np.float64), np.tile(want, blocks))
