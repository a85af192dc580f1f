"""FP64 CPU reference of the LOFAR correlator FX chain (Cobalt, arXiv 1801.04834).

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code, table or
helper with the HIP library in ``paper_1801_04834_amd``; neither side imports the other.

Modules
-------
``fx``     vectorised numpy reference: polyphase filter bank, fine delay + bandpass,
           8-bit requantisation, cross-correlation (X stage).
``brute``  the same defining sums written as plain Python loops, for tiny inputs only.
"""

from .fx import (  # noqa: F401
    baseline_index,
    channel_sky_freqs,
    correlate,
    correlate_int,
    delay_cycles,
    fine_delay_bandpass,
    fx_block,
    polyphase_filterbank,
    reduce_cycles,
    requantise_int8,
    stream_timeline,
    visibilities_from_full,
)
