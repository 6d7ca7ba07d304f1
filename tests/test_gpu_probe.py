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


def test_allocation_failure_is_reported_and_the_library_stays_usable():
    """A request far beyond the device's memory (1 TiB on a 288 GB device)
    fails in hipMalloc before any kernel runs: MPLPXX_ENOMEM with a message,
    and the next calls work."""
    import numpy as np
    from paper_2004_08227_amd import workloads as W
    print("CASE stream read probe 1 TiB (allocation failure)", flush=True)
    with pytest.raises(M.MplpError) as ei:
        M.stream_read_probe(1 << 40, 1)
    assert ei.value.code == M.ENOMEM
    assert M.lib().mplpxx_last_error()
    with M.Solver.from_model(W.tiny(0)) as s:
        s.iterate(3)
        assert np.isfinite(s.dual_bound())
