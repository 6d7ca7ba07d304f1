"""GPU test of the streaming-read probe (the measured ceiling reported
beside the published HBM bandwidth): a positive rate below the published
8 TB/s, best >= median, and a 1 GiB read takes at least what the published
peak allows."""
import pytest

pytestmark = pytest.mark.gpu
M = pytest.importorskip("paper_2004_08227_amd")


def test_stream_read_probe_rate_is_plausible():
    print("CASE stream read probe 1 GiB x 3", flush=True)
    med, best = M.stream_read_probe(1 << 30, 3)
    print(f"stream read: median {med:.0f} GB/s, best {best:.0f} GB/s", flush=True)
    assert 0 < med <= best
    # (1 GiB is four times the 256 MB last-level cache: the reads come from HBM)
    assert best <= 8000.0 * 1.02
