"""Conversions between the K-blocked channelised layout of the C ABI and row-major arrays
(test helpers; no FX arithmetic)."""

import numpy as np


def unblock(a):
    """[..., n_kb, M, 32, 2] -> [..., M, n_kb*32, 2]."""
    a = np.asarray(a)
    *lead, n_kb, M, kb, two = a.shape
    a = np.moveaxis(a, -4, -3)                      # [..., M, n_kb, 32, 2]
    return a.reshape(*lead, M, n_kb * kb, two)


def block(a, kb=32):
    """[..., M, pitch, 2] -> [..., pitch/32, M, 32, 2]."""
    a = np.asarray(a)
    *lead, M, pitch, two = a.shape
    assert pitch % kb == 0
    a = a.reshape(*lead, M, pitch // kb, kb, two)
    return np.ascontiguousarray(np.moveaxis(a, -3, -4))


def unblock_planes(a):
    """FP16-split [..., n_kb, 2, M, 32, 2] -> (hi, lo) each [..., M, pitch, 2]."""
    a = np.asarray(a)
    return unblock(a[..., 0, :, :, :]), unblock(a[..., 1, :, :, :])


def block_planes(hi, lo):
    """(hi, lo) [..., M, pitch, 2] -> [..., n_kb, 2, M, 32, 2]."""
    return np.ascontiguousarray(np.stack([block(hi), block(lo)], axis=-4))
