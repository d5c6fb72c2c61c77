"""The streaming-bandwidth probes (mg_stream_probe) that bench.py reports as
the practical ceilings next to the datasheet peak."""
import pytest

pytestmark = pytest.mark.gpu


def test_stream_probe_rates_are_plausible():
    from paper_2402_12947_amd.binding import stream_probe
    rates = {k: stream_probe(k, 256 << 20, 3) for k in ("read", "copy", "mix7:1")}
    # a positive rate below the 8 TB/s datasheet peak for each stream kind
    assert all(0 < v < 8000 for v in rates.values()), rates
