"""Occupancy import and export (kmc_load_occupancy, kmc_read_occupancy) on
layouts whose size is not a multiple of 16 bytes, with device boundaries
inside a 16-byte group, through caller buffers at every alignment (needs an
MI355X).

The import reads any nonzero byte as an ion; the export writes 0 or 1 back
into the caller's buffer.  Loading bytes in {0, 5, -3} and reading the buffer
afterwards therefore shows whether every byte was exported (and only those:
guard bytes around the buffer must keep their value).  The expected values
are the input's own (x != 0)."""
import numpy as np
import pytest

from parity_util import gpu_available
from workloads import Physics

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

GEOMETRIES = [
    ([3, 5], [7, 9]),              # 66 sites, device boundary at 21 (inside a 16-byte group)
    ([1], [2]),                    # the smallest lattice
    ([150, 7, 2], [96, 33, 5]),    # three devices, ragged tail
    ([2, 1, 3], [17, 2, 31]),      # one-rail device of 2 sites between two others
    ([4096], [1023]),              # large, odd rail length
]


def _codes(n, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([0, 0, 5, -3], dtype=np.int8), size=n)


@pytest.mark.parametrize("rails,sites", GEOMETRIES)
@pytest.mark.parametrize("shift", [0, 1, 8, 15])
def test_load_then_export_at_any_alignment(rails, sites, shift):
    import torch

    import paper_2511_09413_amd as k
    n = int(sum(r * l for r, l in zip(rails, sites)))
    codes = _codes(n, 11 + shift)
    guard = 77
    buf = torch.full((n + 48,), guard, dtype=torch.int8, device="cuda:0")
    view = buf[16 + shift:16 + shift + n]
    view.copy_(torch.as_tensor(codes).to("cuda:0"))
    params, keep = k.make_params(Physics(seed=2), rails, sites)
    nbytes = k.workspace_bytes(params)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:0")
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    stream = torch.cuda.current_stream()
    ctx = k.init_device(params, view.data_ptr(), None, ws_ptr, nbytes, stream.cuda_stream)
    try:
        view.copy_(torch.as_tensor(codes).to("cuda:0"))  # init exported its own (empty) state
        k.load_occupancy(ctx)
        want = (codes != 0).astype(np.int8)
        assert np.array_equal(k.read_occupancy(ctx, n), want)
        torch.cuda.synchronize()
        host = buf.cpu().numpy()
        assert np.array_equal(host[16 + shift:16 + shift + n], want)
        assert np.all(host[:16 + shift] == guard) and np.all(host[16 + shift + n:] == guard)
    finally:
        k.destroy(ctx)
    del keep
