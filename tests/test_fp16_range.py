"""Dynamic range of the FP16-split channelised data (no GPU).

Fixed-point station samples are converted to float before the chain ("Processing steps",
sec. 3.2); the FP16-split mode then stores ``2^k Z`` as an FP16 hi/lo pair, so the prescale k
must keep every channel sample that valid 8/16-bit input can produce below the FP16 limit.
The library derives the largest safe k from the sample type, the taps and the bandpass
(``cobalt_fp16_prescale_max``) and refuses larger ones at plan creation (EOVERFLOW).  These
tests pin that bound against the FP64 oracle: an input matched to the signs of the taps,
with a delay that turns FFT bin 0 onto the real axis, reaches it, so the next larger k would
overflow on that input.
"""

import os

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import binding, synth

FP16_MAX = 65504.0
FP16_OVERFLOW = 65520.0            # round-to-nearest turns values from here on into infinity


def _lib():
    if not os.path.exists(binding.lib_path):
        pytest.skip("libcobalt.so not built (run __graft_entry__.build())")
    return binding.load_library()


def _kw(sample_type, x_mode=synth.X_FP16_SPLIT, k=None, C=64, ripple=0.05, **over):
    w = synth.Workload(name="range", S=4, SB=1, sample_type=sample_type, x_mode=x_mode, N=C * 64, C=C,
                       ripple=ripple, f_sb0=150e6)
    kw = binding.plan_kwargs(w)
    if k is not None:
        kw["fp16_prescale_log2"] = k
    kw.update(over)
    return kw


@pytest.mark.parametrize("st,C,expect", [(synth.CI16, 64, -1), (synth.CI8, 64, 7), (synth.CI16, 256, -1),
                                         (synth.CI8, 256, 7)])
def test_largest_safe_prescale_of_the_default_taps(st, C, expect):
    _lib()
    assert binding.fp16_prescale_max(**_kw(st, C=C)) == expect


def test_flat_bandpass_and_scaled_taps_move_the_bound():
    """The bound scales with max|b| and sum|h|: doubling the taps lowers k by one."""
    _lib()
    k_flat = binding.fp16_prescale_max(**_kw(synth.CI16, ripple=0.0))
    h2 = synth.fir_windowed_sinc() * np.float32(2.0)
    k_twice = binding.fp16_prescale_max(**_kw(synth.CI16, ripple=0.0, fir=h2))
    assert k_twice == k_flat - 1


@pytest.mark.parametrize("st", [synth.CI16, synth.CI8])
def test_plan_settings_above_the_bound_are_refused(st):
    _lib()
    kmax = binding.fp16_prescale_max(**_kw(st))
    assert binding.estimate_bytes(**_kw(st, k=kmax)) > 0
    with pytest.raises(binding.CobaltError) as ei:
        binding.estimate_bytes(**_kw(st, k=kmax + 1))
    assert ei.value.code == binding.EOVERFLOW
    assert f"largest safe value is {kmax}" in str(ei.value)
    # other modes ignore the prescale
    assert binding.estimate_bytes(**_kw(st, x_mode=synth.X_FP32, k=24)) > 0


def test_float_samples_have_no_fixed_bound():
    _lib()
    with pytest.raises(binding.CobaltError) as ei:
        binding.fp16_prescale_max(**_kw(synth.CF32))
    assert ei.value.code == binding.EINVAL
    # any k in range is accepted for float samples (the kernel saturates instead)
    assert binding.estimate_bytes(**_kw(synth.CF32, k=24)) > 0


def _worst_case_delays(S, f_sb):
    """Station 0's delay turns the phase of (1 + i) onto the real axis in the DC channel
    (c = C/2, sky frequency f_SB): a phase of -1/8 cycle."""
    d = np.zeros((S, 2))
    d[0, :] = -1.0 / (8.0 * f_sb)
    return d


@pytest.mark.parametrize("st", [synth.CI16, synth.CI8])
def test_sign_matched_input_reaches_the_bound(st):
    """Oracle on the full-scale input: station 0's DC channel reaches a component of
    A sqrt(2) sum|h| max|b| at the end of each matched window, so 2^k_max keeps it below
    the FP16 limit and 2^(k_max + 1) would overflow."""
    _lib()
    C, T, n_c = 64, 16, 64
    h = synth.fir_windowed_sinc(C, T)
    b = synth.bandpass_ripple(C, 0.05)
    x = synth.full_scale_streams(h, C, T, C * n_c, seed=3, sample_type=st)
    f_sb = np.array([150e6])
    out = oracle.fx_block(synth.to_complex(x), np.zeros((4, 2, 1, (T - 1) * C), np.complex128), h, b, f_sb,
                          synth.SAMPLE_RATE_HZ, _worst_case_delays(4, f_sb[0]), C, T, mode="fp16_split")
    Z = out["Z"]                                             # [SB, C, M, N_c]
    comp = np.maximum(np.abs(Z.real), np.abs(Z.imag))
    A = 127 if st == synth.CI8 else 32767
    expect = A * np.sqrt(2.0) * np.sum(np.abs(h.astype(np.float64))) * float(b[C // 2])
    assert comp.max() == pytest.approx(expect, rel=1e-9)
    j_max = np.unravel_index(np.argmax(comp), comp.shape)
    assert j_max[1] == C // 2 and j_max[2] in (0, 1) and j_max[3] % T == T - 1
    kmax = binding.fp16_prescale_max(**_kw(st))
    assert 2.0 ** kmax * comp.max() <= FP16_MAX
    assert 2.0 ** (kmax + 1) * comp.max() >= FP16_OVERFLOW
