"""The streaming probe reads every byte of its tiles in the BS_1 lane layout and
writes one folded dword per lane: its output is checked against the same fold
on the host, and its arguments are validated."""
import numpy as np
import pytest
import torch

from helpers import flush

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu(built_lib):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("ntiles", [1, 37, 5000])
def test_probe_folds_every_tile(ntiles):
    from paper_2209_00220_amd import _lib

    flush("stream probe, %d tiles" % ntiles)
    rng = np.random.default_rng(ntiles)
    host = rng.integers(0, 2**32, size=ntiles * 512, dtype=np.uint32)
    src = torch.from_numpy(host.view(np.uint8).copy()).cuda()
    dst = torch.zeros(ntiles * 64, dtype=torch.int32, device="cuda")
    _lib.bst_stream_probe(src, ntiles * 2048, dst, 0)
    torch.cuda.synchronize()
    got = dst.cpu().numpy().view(np.uint32)
    # lane L of tile t: dwords 0-3 at t*2048 + 16L, dwords 4-7 at t*2048 + 1024 + 16L
    d = host.reshape(ntiles, 2, 64, 4)
    want = np.bitwise_xor.reduce(d.transpose(0, 2, 1, 3).reshape(ntiles, 64, 8), axis=2).reshape(-1)
    assert np.array_equal(got, want)


def test_probe_rejects_bad_arguments():
    from paper_2209_00220_amd import _lib

    src = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    dst = torch.zeros(512, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError, match="multiple of 2048"):
        _lib.bst_stream_probe(src, 3000, dst, 0)
    with pytest.raises(RuntimeError, match="aligned"):
        _lib.bst_stream_probe(src[8:], 2048, dst, 0)
    _lib.bst_stream_probe(src, 0, dst, 0)   # nothing to read
    torch.cuda.synchronize()
