"""The random-read probe the benchmark quotes as the lookup's ceiling: it runs, reports a
positive time for every supported width, and rejects unsupported arguments on the host
before anything is launched."""
import pytest

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _fks():
    from paper_2508_11443_amd import fks
    return fks


@pytest.mark.parametrize("width", [16, 32, 64, 128])
def test_probe_reports_a_time(width):
    fks = _fks()
    announce(f"probe: 64 MiB buffer, 2^20 reads of {width} bytes")
    ms = fks.fks_probe_random_reads(64 << 20, 1 << 20, width)
    assert 0.0 < ms < 1000.0


def test_probe_buffer_smaller_than_one_read():
    # a buffer below one read's width still holds one whole block
    announce("probe: 8-byte buffer, 64-byte reads")
    assert _fks().fks_probe_random_reads(8, 4096, 64) > 0.0


@pytest.mark.parametrize("buffer_bytes,probes,width", [(1 << 20, 0, 16), (1 << 20, 1024, 24), (1 << 20, 1024, 256)])
def test_probe_rejects_bad_arguments(buffer_bytes, probes, width):
    fks = _fks()
    with pytest.raises(fks.FksError) as err:
        fks.fks_probe_random_reads(buffer_bytes, probes, width)
    assert err.value.code == fks.FKS_EINVAL
