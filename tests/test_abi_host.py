"""The C ABI on the host (no GPU): the library loads, exports every function the header
declares, and validates settings with the documented error codes before touching a GPU."""

import os
import re

import numpy as np
import pytest

from paper_1801_04834_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cobalt.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cobalt_[a-z0-9_]+)\s*\(", txt)))


def _lib():
    if not os.path.exists(binding.lib_path):
        pytest.skip("libcobalt.so not built (run __graft_entry__.build())")
    return binding.load_library()


def test_header_declares_the_binding_surface():
    assert _declared() == sorted(binding.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name
        assert getattr(lib, name) is not None


def _kw(**over):
    w = synth.workload("int16_share")
    kw = dict(n_stations=w.S, n_subbands=w.SB, samples_per_block=w.N, sample_type=w.sample_type,
              x_mode=w.x_mode, fir=w.fir(), subband_freqs=w.subband_freqs(), bandpass=w.bandpass(),
              fp16_prescale_log2=-1, requant_gain=8.0)
    kw.update(over)
    return kw


def test_estimate_bytes_of_the_16bit_share():
    _lib()
    n = binding.estimate_bytes(**_kw())
    # channelised FP16 hi/lo planes dominate: 64 SB x 64 ch x 2 x 152 x 3072 x 4 B
    chan = 64 * 64 * 2 * 152 * 3072 * 4
    hist = 2 * 64 * 152 * 960 * 4          # two FIR-history buffers of (T-1)*C ci16 samples
    cflag = 76 * 64 * (3072 // 32) * 4      # flagged-channel-sample bits per station and subband
    assert chan + hist + cflag <= n <= chan + hist + cflag + 2**20


@pytest.mark.parametrize("over,code", [
    (dict(n_stations=0), binding.EINVAL),
    (dict(n_pols=3), binding.EUNSUPPORTED),
    (dict(n_subbands=0), binding.EINVAL),
    (dict(n_channels=128), binding.EUNSUPPORTED),
    (dict(n_taps=8), binding.EUNSUPPORTED),
    (dict(samples_per_block=1000), binding.EINVAL),
    (dict(samples_per_block=-64), binding.EINVAL),
    (dict(sample_type=7), binding.EINVAL),
    (dict(x_mode=9), binding.EINVAL),
    (dict(sample_rate=0.0), binding.EINVAL),
    (dict(n_stations=81), binding.EUNSUPPORTED),
    (dict(n_stations=129, x_mode=synth.X_FP32), binding.EUNSUPPORTED),
    (dict(x_mode=synth.X_INT8, requant_gain=0.0), binding.EINVAL),
    (dict(x_mode=synth.X_INT8, samples_per_block=64 * 66592), binding.EOVERFLOW),
    (dict(fp16_prescale_log2=30), binding.EINVAL),
    (dict(fir=np.full(1024, np.nan, np.float32)), binding.EINVAL),
    (dict(subband_freqs=np.full(64, np.inf)), binding.EINVAL),
])
def test_invalid_settings_return_codes(over, code):
    _lib()
    with pytest.raises(binding.CobaltError) as ei:
        binding.estimate_bytes(**_kw(**over))
    assert ei.value.code == code
    assert binding.load_library().cobalt_last_error().decode()


def test_int8_overflow_bound_edge():
    _lib()
    ok = binding.estimate_bytes(**_kw(x_mode=synth.X_INT8, samples_per_block=64 * 66572))
    assert ok > 0
    with pytest.raises(binding.CobaltError) as ei:
        binding.estimate_bytes(**_kw(x_mode=synth.X_INT8, samples_per_block=64 * 66573))
    assert ei.value.code == binding.EOVERFLOW


def test_largest_mfma_setting_is_accepted():
    _lib()
    assert binding.estimate_bytes(**_kw(n_stations=80)) > 0
    assert binding.estimate_bytes(**_kw(n_stations=128, x_mode=synth.X_FP32)) > 0
    assert binding.estimate_bytes(**_kw(samples_per_block=0)) > 0


def test_plan_requires_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "lib_path", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        binding.load_library()


@pytest.mark.parametrize("args", [(2**30, 0, 4, 1.0), (2**30, 65, 4, 1.0), (2**30, 2, 0, 1.0), (2**30, 2, 4, 0.0)])
def test_service_rejects_bad_arguments_before_touching_a_gpu(args):
    import ctypes as ct
    lib = _lib()
    out = ct.c_void_p(None)
    rc = lib.cobalt_service_create(ct.c_size_t(args[0]), args[1], args[2], ct.c_double(args[3]), ct.byref(out))
    assert rc == binding.EINVAL and not out.value
    assert lib.cobalt_service_last_error().decode()


@pytest.mark.parametrize("mode,iters,wgs,sink", [(0, 10, 1, 256), (1, 0, 1, 256), (2, 2**19 + 1, 1, 256),
                                                 (1, 10, 0, 256), (2, 10, 1, 0), (1, 10, 1, 258)])
def test_mfma_probe_rejects_bad_arguments_before_touching_a_gpu(mode, iters, wgs, sink):
    """FP32 mode, iterations outside 1 .. 2^19, no workgroups, a NULL or misaligned sink:
    EINVAL from the argument checks (the sink pointers are never dereferenced)."""
    import ctypes as ct
    lib = _lib()
    rc = lib.cobalt_mfma_probe(mode, ct.c_int64(iters), wgs, ct.c_void_p(sink), None)
    assert rc == binding.EINVAL
    assert lib.cobalt_last_error().decode()


@pytest.mark.parametrize("ptrs,nbytes", [((0, 256, 512), 64), ((256, 256 + 8, 512), 64), ((256, 512, 768), 24)])
def test_copies_reject_bad_arguments_before_touching_a_gpu(ptrs, nbytes):
    """NULL or misaligned pointers and sizes that are not multiples of 16: EINVAL."""
    import ctypes as ct
    lib = _lib()
    d0, d1, s = (ct.c_void_p(p) for p in ptrs)
    assert lib.cobalt_device_fanout(d0, d1, s, ct.c_size_t(nbytes), None) == binding.EINVAL


def test_noalloc_refuses_settings_beyond_its_scratch_before_touching_a_gpu():
    """The 16-bit share needs a 15 GB channelised block: cobalt_correlate_noalloc refuses it
    (EUNSUPPORTED) from the sizes alone; the dummy device pointers are never dereferenced."""
    import ctypes as ct
    lib = _lib()
    cfg, keep = binding.make_config(**_kw(fp16_prescale_log2=-1))
    d = np.zeros(2 * 76)
    p = ct.c_void_p(256)
    rc = lib.cobalt_correlate_noalloc(ct.byref(cfg), p, d.ctypes.data_as(ct.POINTER(ct.c_double)), None, None, p, None)
    assert rc == binding.EUNSUPPORTED
    assert "scratch" in lib.cobalt_last_error().decode()
    del keep
