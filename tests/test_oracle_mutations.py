"""Planted mistakes in the FP64 reference are caught by its pins.

Each case swaps one function of ``oracle.fx`` for a copy with a plausible mistake (dropped
tap, reversed taps, wrong delay sign or frequency, unshifted channel order, normalised FFT,
missing bandpass, conjugate on the wrong operand, interpolation at the wrong time point,
rounding half away from zero) and runs the pin that must reject it.  Everything runs on the
CPU; nothing here touches the HIP library.
"""

import numpy as np
import pytest

import oracle
import oracle.beam as obm
import oracle.flags as ofl
import oracle.fx as fx
from tests import test_oracle_beam as bpins
from tests import test_oracle_flags as fpins
from tests import test_oracle_pins as pins

_orig = {name: getattr(fx, name) for name in (
    "polyphase_filterbank", "channel_sky_freqs", "delay_cycles", "fine_delay_bandpass",
    "correlate", "requantise_int8")}


def _ppf_dropped_tap(timeline, h, C, T):
    h = np.array(h, np.float64)
    h[(T - 1) * C:] = 0.0                      # last tap row ignored
    return _orig["polyphase_filterbank"](timeline, h, C, T)


def _ppf_reversed_taps(timeline, h, C, T):
    h = np.asarray(h, np.float64).reshape(T, C)[::-1].reshape(-1)
    return _orig["polyphase_filterbank"](timeline, h, C, T)


def _ppf_no_shift(timeline, h, C, T):
    X = _orig["polyphase_filterbank"](timeline, h, C, T)
    return np.roll(X, -(C // 2), axis=-1)      # DFT bin order instead of ascending frequency


def _ppf_normalised(timeline, h, C, T):
    return _orig["polyphase_filterbank"](timeline, h, C, T) / C


def _freqs_without_offset(f_sb, C, f_s):
    c = np.arange(C, dtype=np.float64)
    return f_sb + c * (f_s / C)


def _delay_wrong_time(f_c, tau0, tau1, n_c):
    j = np.arange(n_c, dtype=np.float64) + 0.5
    tau = tau0 + (tau1 - tau0) * j / n_c
    return tau[:, None] * np.asarray(f_c, np.float64)[None, :]


def _rotate_wrong_sign(X, cyc, bandpass):
    return _orig["fine_delay_bandpass"](X, -np.asarray(cyc), bandpass)


def _rotate_no_bandpass(X, cyc, bandpass):
    return _orig["fine_delay_bandpass"](X, cyc, np.ones_like(np.asarray(bandpass, np.float64)))


def _correlate_conj_first(Z, S, P=2):
    Z = np.asarray(Z, np.complex128)
    Vfull = np.matmul(np.conj(Z), np.swapaxes(Z, -1, -2))
    return oracle.visibilities_from_full(Vfull, S, P)


def _requant_half_away(Z, gain):
    g = np.float64(np.float32(gain))
    Z = np.asarray(Z, np.complex128)
    out = np.empty(Z.shape + (2,), np.int8)
    for comp, part in ((0, Z.real), (1, Z.imag)):
        v = (g * part).astype(np.float32).astype(np.float64)
        out[..., comp] = np.clip(np.sign(v) * np.floor(np.abs(v) + 0.5), -127, 127).astype(np.int8)
    return out


_orig_fl = {name: getattr(ofl, name) for name in ("channel_flags", "visibility_weights", "coarse_window")}


def _flags_short_window(win_flags, hist_row_flags, C, T):
    return _orig_fl["channel_flags"](win_flags, hist_row_flags, C, T - 1)


def _flags_ignore_history(win_flags, hist_row_flags, C, T):
    return _orig_fl["channel_flags"](win_flags, np.zeros_like(np.asarray(hist_row_flags, bool)), C, T)


def _weights_union(chan_flags):
    S = chan_flags.shape[0]
    W = np.zeros((chan_flags.shape[1], S * (S + 1) // 2), np.int64)
    for s1 in range(S):
        for s2 in range(s1 + 1):
            W[:, oracle.baseline_index(s1, s2)] = np.sum(~chan_flags[s1] | ~chan_flags[s2], axis=-1)
    return W


def _window_reversed(rows, offsets, N):
    G = np.asarray(rows).shape[-1] - N
    return _orig_fl["coarse_window"](rows, G - np.asarray(offsets), N)


FLAG_MUTANTS = [
    ("channel_flags", _flags_short_window, fpins.test_flagged_channel_samples_are_exactly_those_reading_lost_samples, (1,)),
    ("channel_flags", _flags_ignore_history, fpins.test_flagged_channel_samples_are_exactly_those_reading_lost_samples, (2,)),
    ("visibility_weights", _weights_union, fpins.test_weights_and_visibilities_are_sums_over_common_valid_samples, ("fp32",)),
    ("coarse_window", _window_reversed, fpins.test_integer_sample_delay_is_removed_exactly_by_the_window_offset, ()),
]


@pytest.mark.parametrize("name,mutant,pin,args", FLAG_MUTANTS, ids=[f"{m[0]}:{m[1].__name__}" for m in FLAG_MUTANTS])
def test_planted_flag_mistake_is_caught(monkeypatch, name, mutant, pin, args):
    pin(*args)
    monkeypatch.setattr(ofl, name, mutant)
    with pytest.raises(AssertionError):
        pin(*args)


_orig_bm = {name: getattr(obm, name) for name in ("beam_weights", "stokes", "incoherent_stokes",
                                                  "resolution_transform")}


def _weights_conjugated(f_c, dtau):
    return np.conj(_orig_bm["beam_weights"](f_c, dtau))


def _stokes_u_v_swapped(X, Y, which="IQUV"):
    st = _orig_bm["stokes"](X, Y, "IQUV")
    st = st[..., [0, 1, 3, 2], :]
    return st if which == "IQUV" else st[..., :1, :]


def _incoherent_one_pol(Z, S, P=2, which="IQUV"):
    Z = np.asarray(Z, np.complex128)
    Zp = Z.reshape(Z.shape[0], S, P, Z.shape[-1])
    return _orig_bm["stokes"](Zp[:, :, 0], 0 * Zp[:, :, 1], which).sum(axis=1)


def _transform_forward_sign(B, C_out):
    return np.conj(_orig_bm["resolution_transform"](np.conj(B), C_out))


def _transform_unshifted(B, C_out):
    return _orig_bm["resolution_transform"](np.roll(np.asarray(B), -np.asarray(B).shape[-2] // 2, axis=-2), C_out)


def _transform_unscaled(B, C_out):
    return np.asarray(B).shape[-2] * _orig_bm["resolution_transform"](B, C_out)


BEAM_MUTANTS = [
    ("beam_weights", _weights_conjugated, bpins.test_point_source_gains, ()),
    ("stokes", _stokes_u_v_swapped, bpins.test_point_source_gains, ()),
    ("incoherent_stokes", _incoherent_one_pol,
     bpins.test_coherent_power_is_the_quadratic_form_of_the_correlation_matrix, ()),
    ("resolution_transform", _transform_forward_sign, bpins.test_transform_to_one_channel_is_the_inverse_fft, ()),
    ("resolution_transform", _transform_unshifted, bpins.test_bin_centred_channel_lands_in_its_output_channel, (16, 3)),
    ("resolution_transform", _transform_unscaled, bpins.test_transform_conserves_power, ()),
]


@pytest.mark.parametrize("name,mutant,pin,args", BEAM_MUTANTS, ids=[f"{m[0]}:{m[1].__name__}" for m in BEAM_MUTANTS])
def test_planted_beam_mistake_is_caught(monkeypatch, name, mutant, pin, args):
    pin(*args)
    monkeypatch.setattr(obm, name, mutant)
    with pytest.raises(AssertionError):
        pin(*args)


MUTANTS = [
    ("polyphase_filterbank", _ppf_dropped_tap, pins.test_bin_centred_tone_lands_in_its_channel_with_fir_gain, ()),
    ("polyphase_filterbank", _ppf_reversed_taps, pins.test_single_channel_is_plain_fir, ()),
    ("polyphase_filterbank", _ppf_no_shift, pins.test_impulse_response_closed_form, (8,)),
    ("polyphase_filterbank", _ppf_normalised, pins.test_dft_unnormalised_parseval, ()),
    ("channel_sky_freqs", _freqs_without_offset, pins.test_delay_sign_and_frequency_align_a_delayed_sky_tone, ()),
    ("delay_cycles", _delay_wrong_time, pins.test_linear_delay_drift_geometric_series, ()),
    ("fine_delay_bandpass", _rotate_wrong_sign, pins.test_delay_sign_and_frequency_align_a_delayed_sky_tone, ()),
    ("fine_delay_bandpass", _rotate_no_bandpass, pins.test_autocorrelation_closed_form, ()),
    ("correlate", _correlate_conj_first, pins.test_correlate_matches_loops, ()),
    ("requantise_int8", _requant_half_away, pins.test_requantise_rounding_and_clipping, ()),
]


@pytest.mark.parametrize("name,mutant,pin,args", MUTANTS, ids=[f"{m[0]}:{m[1].__name__}" for m in MUTANTS])
def test_planted_mistake_is_caught(monkeypatch, name, mutant, pin, args):
    pin(*args)                                  # the pin passes on the real reference
    monkeypatch.setattr(fx, name, mutant)       # used inside fx_block
    monkeypatch.setattr(oracle, name, mutant)   # used by the pins directly
    with pytest.raises(AssertionError):
        pin(*args)
