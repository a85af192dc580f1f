"""The synthetic workloads' constants against the numbers the paper prints.

Fixture: ``tests/golden/paper_dimensions.json`` (each entry cites its section/table).
"""

import json
import os

from paper_1801_04834_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_dimensions.json")


def _g():
    with open(GOLDEN) as f:
        return json.load(f)


def test_sample_rate_matches_printed_period_and_bandwidth():
    g = _g()
    assert abs(1e6 / synth.SAMPLE_RATE_HZ - g["sample_period_us"]["value"]) < 1e-12
    assert round(synth.SAMPLE_RATE_HZ / 1e3) == g["subband_bandwidth_khz"]["value"]
    # 512 subbands of f_s tile the 100 MHz Nyquist band of a 200 MHz sampling clock
    assert synth.SAMPLE_RATE_HZ * g["station_subbands"]["value"] == 100e6


def test_block_length_matches_dimension_table():
    g = _g()
    d = g["samples_per_channel_per_second"]
    # the block is one second's worth of channel samples: N at 1 channel, N/256 at 256
    assert synth.BLOCK_SAMPLES == d["max"]
    assert synth.BLOCK_SAMPLES // g["channels_per_subband_correlator"]["max"] == d["min"]
    assert synth.BLOCK_SAMPLES % g["channels_per_subband_correlator"]["min"] == 0
    secs = synth.BLOCK_SAMPLES / synth.SAMPLE_RATE_HZ
    assert abs(secs - 1.00663296) < 1e-12
    assert abs(secs - g["block_seconds_approx"]["value"]) < 0.01


def test_workloads_within_printed_ranges():
    g = _g()
    for name in ("int16_share", "int8_full"):
        w = synth.workload(name)
        assert g["antenna_fields_correlator"]["min"] <= w.S <= 80
        assert g["channels_per_subband_correlator"]["min"] <= w.C <= g["channels_per_subband_correlator"]["max"]
        assert w.N == synth.BLOCK_SAMPLES
