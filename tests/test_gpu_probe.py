"""gf_hbm_probe, the streaming-read probe bench.py reports beside the
rooflines: a plausible rate, the buffer left unchanged, bad buffers
rejected before any launch."""
import numpy as np
import pytest

from paper_1603_09596_amd import geraf

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    geraf.load()


def test_probe_rate_and_buffer_unchanged():
    buf = torch.arange(64 << 20, dtype=torch.int32, device="cuda:0")   # 256 MiB
    before = buf[::4097].cpu().numpy().copy()
    rate = geraf.hbm_probe(buf, 3)
    assert 100.0 < rate < 12_000.0, rate
    assert np.array_equal(buf[::4097].cpu().numpy(), before)
    # a ragged size: the last bytes past a 16-byte multiple are not read
    assert geraf.hbm_probe(buf[: (1 << 20) + 3], 1) > 0.0


def test_probe_rejects_host_and_misaligned_buffers():
    with pytest.raises(geraf.GerafError):
        geraf.hbm_probe(np.zeros(1 << 20, np.uint8), 1)
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(geraf.GerafError):
        geraf.hbm_probe(buf[1:], 1)
    with pytest.raises(geraf.GerafError):
        geraf.hbm_probe(buf[:8], 1)
