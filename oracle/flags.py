"""FP64 reference of coarse delay compensation and lost-sample flags with visibility weights.

Test infrastructure only (see the package docstring).

Paper: coarse delay compensation shifts each station's sample stream by a whole number of
samples, and only the sub-sample remainder is applied later as a phase rotation on the GPU
("Software architecture", sec. 7.1; "Signal processing with GPU kernels", sec. 7.5: the fine
delay uses the residual of the coarse compensation).  Packets that are missing after a
deadline count as lost ("Processing steps", sec. 3.2), and lost or dropped data is recorded
in metadata that travels with the data product ("Dealing with jitter and hardware failure",
sec. 7.2).  The paper gives no formula for how lost samples reach the visibilities; the
readings below are this library's:

* Coarse delay: station s reads its block from rows of ``N + G`` samples starting at sample
  ``g_s`` (``0 <= g_s <= G``), i.e. the block is ``row[g_s : g_s + N]``; both polarisations
  and all subbands of a station share ``g_s``.  The carried FIR history is the end of the
  previous block's window, so a change of ``g_s`` between blocks repeats or skips samples at
  the block edge, as shifting a circular buffer's read pointer does.  The delays handed to
  the fine stage are the residual delays.
* Flags: one bit per (station, subband, sample of the row); both polarisations share it (one
  packet carries both).  A channel sample ``j`` is flagged when any input sample inside its
  FIR window -- the ``T*C`` samples ``(j-T+1)*C .. (j+1)*C - 1`` of the block window,
  reaching into the carried history -- is flagged.  Flagged channel samples are set to zero
  in the channelised data (so they drop out of every product of the X stage), and each
  baseline gets a weight: the number of channel samples valid for both of its stations.
  History rows are unflagged after a reset.
"""

from __future__ import annotations

import numpy as np

from . import fx

__all__ = ["coarse_window", "window_flags", "channel_flags", "visibility_weights", "fx_block_flagged"]


def coarse_window(rows: np.ndarray, offsets: np.ndarray, N: int) -> np.ndarray:
    """Block window of every stream after the integer-sample shift (sec. 7.1).

    rows [S, P, SB, N + G]; offsets int [S] with 0 <= g_s <= G.  Returns [S, P, SB, N]."""
    rows = np.asarray(rows)
    S = rows.shape[0]
    G = rows.shape[-1] - N
    out = np.empty(rows.shape[:-1] + (N,), rows.dtype)
    for s in range(S):
        g = int(offsets[s])
        assert 0 <= g <= G, (s, g, G)
        out[s] = rows[s, ..., g:g + N]
    return out


def window_flags(flags: np.ndarray, offsets: np.ndarray, N: int) -> np.ndarray:
    """Sample flags of each station's block window: bool [S, SB, N + G] -> [S, SB, N]."""
    flags = np.asarray(flags, bool)
    return np.stack([flags[s, :, int(offsets[s]):int(offsets[s]) + N] for s in range(flags.shape[0])])


def channel_flags(win_flags: np.ndarray, hist_row_flags: np.ndarray, C: int, T: int):
    """Flags of the channel samples and the row flags carried to the next block.

    win_flags bool [S, SB, N] (the window's sample flags); hist_row_flags bool [S, SB, T-1]
    (whether each of the T-1 rows of C samples preceding the block held a flagged sample).
    A timeline row is flagged when any of its C samples is; channel sample j is flagged when
    any of the T rows its FIR output reads (the T-1 rows before row j of the block, and row
    j) is.  Returns (chan_flags bool [S, SB, N_c], new hist_row_flags [S, SB, T-1])."""
    S, SB, N = win_flags.shape
    n_c = N // C
    rows = win_flags.reshape(S, SB, n_c, C).any(axis=-1)
    timeline = np.concatenate([np.asarray(hist_row_flags, bool), rows], axis=-1)   # [S, SB, T-1+N_c]
    chan = np.zeros((S, SB, n_c), bool)
    for j in range(n_c):
        chan[:, :, j] = timeline[:, :, j:j + T].any(axis=-1)
    return chan, timeline[:, :, timeline.shape[-1] - (T - 1):].copy()


def visibility_weights(chan_flags: np.ndarray) -> np.ndarray:
    """Channel samples valid for both stations of each baseline: int64 [SB, B]."""
    valid = ~np.asarray(chan_flags, bool)          # [S, SB, N_c]
    S, SB, _ = valid.shape
    W = np.zeros((SB, S * (S + 1) // 2), np.int64)
    for s1 in range(S):
        for s2 in range(s1 + 1):
            W[:, fx.baseline_index(s1, s2)] = np.sum(valid[s1] & valid[s2], axis=-1)
    return W


def fx_block_flagged(rows, N, offsets, flags, history, hist_row_flags, h, bandpass, subband_freqs,
                     sample_rate, residual_delays, C, T, mode="fp32", gain=None):
    """One block of the FX chain with coarse delay and lost-sample flags.

    rows complex [S, P, SB, N + G]; N samples per block window; offsets int [S]; flags bool
    [S, SB, N + G] or None (nothing lost); history / hist_row_flags as carried from the
    previous block (zeros / False after a reset); residual_delays float64 [S, 2].  The block
    window goes through ``fx.fx_block``; flagged channel samples are then zeroed before the X
    stage (after requantisation in int8 mode; zero is exact either way).  Returns a dict with
    ``V``, ``W`` (weights [SB, B]), ``chan_flags``, ``Z`` (float modes) or ``Q`` and ``Zf``
    (int8), ``history`` and ``hist_row_flags``."""
    rows = np.asarray(rows)
    S, P, SB, _ = rows.shape
    x = coarse_window(rows, offsets, N)
    if flags is None:
        flags = np.zeros((S, SB, rows.shape[-1]), bool)
    chan, new_rows = channel_flags(window_flags(flags, offsets, N), hist_row_flags, C, T)
    res = fx.fx_block(x, history, h, bandpass, subband_freqs, sample_rate, residual_delays, C, T,
                      mode=mode, gain=gain)
    # chan [S, SB, N_c] -> per channelised row (s*P + p) of [SB, C, M, N_c]
    mask = np.repeat(chan.transpose(1, 0, 2), P, axis=1)[:, None, :, :]     # [SB, 1, M, N_c]
    out = {"history": res["history"], "hist_row_flags": new_rows, "chan_flags": chan,
           "W": visibility_weights(chan)}
    if mode == "int8":
        Q = res["Q"].copy()
        Q[np.broadcast_to(mask, Q.shape[:-1])] = 0
        out["Q"] = Q
        out["Zf"] = np.where(mask, 0, res["Zf"])        # float64 values before requantisation
        out["V"] = fx.correlate_int(Q, S, P)
    else:
        Z = np.where(mask, 0, res["Z"])
        out["Z"] = Z
        out["V"] = fx.correlate(Z, S, P)
    return out
