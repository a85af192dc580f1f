"""Seeded synthetic inputs shaped like LOFAR correlator workloads.

Nothing here computes any step of the FX chain: this module only draws samples, delays,
frequencies and filter coefficients.  Both the HIP library's tests/benchmarks and the
CPU reference consume what it produces.  It imports neither of them.

Shapes follow the paper: subbands of 195 312.5 Hz (one sample = 5.12 us, "Software
architecture", sec. 7.1; 195 kHz subbands, sec. 3), blocks of 196 608 samples (about 1 s;
Table "Dimensions to map", sec. 7.3), 64 channels, 8/16-bit complex station samples
("Processing steps", sec. 3.2; requirements in sec. 5), up to 80 antenna fields.

Every random stream is keyed by ``numpy.random.default_rng([seed, block, s, p, sb])`` so
any single input stream of a large block can be regenerated on its own.
"""

from __future__ import annotations

import concurrent.futures as _cf
import math
import os
from dataclasses import dataclass, field

import numpy as np

SAMPLE_RATE_HZ = 195312.5          # 200 MHz / 1024: one subband sample every 5.12 us
BLOCK_SAMPLES = 196608             # samples per subband per block (~1.00663296 s)

CI8, CI16, CF32 = 1, 2, 3          # sample types (complex int8 / int16 / float32)
X_FP32, X_FP16_SPLIT, X_INT8 = 0, 1, 2


def fir_windowed_sinc(C: int = 64, T: int = 16) -> np.ndarray:
    """Prototype low-pass FIR for a C-channel, T-tap polyphase filter bank (float32).

    ``h[m] = sinc((m - (L-1)/2) / C) * blackman(L)[m]``, L = T*C, scaled to sum 1 in
    float64 and rounded to float32.  (A coefficient choice: the paper gives none.)
    """
    L = T * C
    m = np.arange(L, dtype=np.float64)
    h = np.sinc((m - (L - 1) / 2.0) / C) * np.blackman(L)
    return (h / h.sum()).astype(np.float32)


def bandpass_ripple(C: int = 64, depth: float = 0.05) -> np.ndarray:
    """Deterministic per-channel bandpass correction ``1 + depth*cos(2 pi (c - C/2)/C)``."""
    c = np.arange(C, dtype=np.float64)
    return (1.0 + depth * np.cos(2 * np.pi * (c - C / 2) / C)).astype(np.float32)


def hba_subband_freqs(n_subbands: int, first: int = 256, base_hz: float = 100e6) -> np.ndarray:
    """Sky centre frequencies of consecutive subbands: ``base + (first + i) * f_s`` (Hz)."""
    i = np.arange(n_subbands, dtype=np.float64)
    return base_hz + (first + i) * SAMPLE_RATE_HZ


def station_delays(seed: int, S: int, spread_s: float = 5e-6, drift_s: float = 25e-9) -> np.ndarray:
    """Residual delays [S, 2] (block start, block end) in seconds, float64.

    start ~ U(-spread, +spread), end = start + U(-drift, +drift).
    """
    rng = np.random.default_rng([seed, 0xDE1A])
    t0 = rng.uniform(-spread_s, spread_s, S)
    t1 = t0 + rng.uniform(-drift_s, drift_s, S)
    return np.stack([t0, t1], axis=1)


def requant_gain(sigma_in: float, h: np.ndarray, target_sigma: float = 16.0) -> float:
    """Gain g for the 8-bit requantisation so that g*Z has std ``target_sigma`` per
    component for white input of std ``sigma_in`` per component (float32 value).

    Uses only the input statistics and the FIR's sum of squares (a setting, not a step
    of the chain): ``g = target / (sigma_in * sqrt(sum h^2))``.
    """
    h64 = np.asarray(h, np.float64)
    return float(np.float32(target_sigma / (sigma_in * math.sqrt(float(np.dot(h64, h64))))))


def _stream_rng(seed, block, s, p, sb):
    return np.random.default_rng([int(seed), int(block), int(s), int(p), int(sb)])


def gaussian_stream(seed, block, s, p, sb, n, sigma, sample_type):
    """One input stream of ``n`` complex samples, per-component N(0, sigma^2).

    ci16: rounded to nearest and clipped to [-32767, 32767]; ci8: clipped to [-127, 127];
    cf32: float32.  Returns the storage array [n, 2] of the sample type.
    """
    rng = _stream_rng(seed, block, s, p, sb)
    v = rng.standard_normal(2 * n, dtype=np.float32) * np.float32(sigma)
    v = v.reshape(n, 2)
    if sample_type == CF32:
        return v
    lim = 127 if sample_type == CI8 else 32767
    dt = np.int8 if sample_type == CI8 else np.int16
    return np.clip(np.rint(v), -lim, lim).astype(dt)


def add_tone(samples: np.ndarray, amplitude: float, cycles_per_sample: float, n0: int = 0,
             phase_cycles: float = 0.0) -> np.ndarray:
    """Add ``A exp(2 pi i (f0 (n0 + n) + phase))`` to a stream ([n, 2] storage array).

    Integer storage is rounded to nearest after adding (so the tone carries +-0.5 rounding
    noise); float32 storage stores the float32-rounded sum.
    """
    n = samples.shape[0]
    idx = (n0 + np.arange(n, dtype=np.float64))
    ph = 2 * np.pi * (cycles_per_sample * idx + phase_cycles)
    re = samples[:, 0].astype(np.float64) + amplitude * np.cos(ph)
    im = samples[:, 1].astype(np.float64) + amplitude * np.sin(ph)
    out = np.empty_like(samples)
    if samples.dtype == np.float32:
        out[:, 0], out[:, 1] = re, im
    else:
        lim = np.iinfo(samples.dtype).max
        out[:, 0] = np.clip(np.rint(re), -lim, lim)
        out[:, 1] = np.clip(np.rint(im), -lim, lim)
    return out


def to_complex(samples: np.ndarray) -> np.ndarray:
    """Storage array [..., 2] -> complex128 (exact for all three sample types)."""
    return samples[..., 0].astype(np.float64) + 1j * samples[..., 1].astype(np.float64)


_DTYPES = {CI8: np.int8, CI16: np.int16, CF32: np.float32}


def storage_dtype(sample_type: int):
    return _DTYPES[sample_type]


@dataclass
class Workload:
    """A complete synthetic correlator workload (one plan's settings + input recipe)."""
    name: str
    S: int
    SB: int
    sample_type: int
    x_mode: int
    N: int = BLOCK_SAMPLES
    C: int = 64
    T: int = 16
    P: int = 2
    sigma: float = 64.0
    seed: int = 1801
    tone_amplitude: float = 0.0
    tone_channel: int = 37
    delay_spread_s: float = 0.0
    delay_drift_s: float = 0.0
    ripple: float = 0.0
    f_sb0: float | None = None
    fp16_prescale_log2: int = 0
    extra: dict = field(default_factory=dict)

    # ---- derived settings (no FX arithmetic) -------------------------------------
    @property
    def M(self):
        return self.S * self.P

    @property
    def n_c(self):
        return self.N // self.C

    @property
    def n_baselines(self):
        return self.S * (self.S + 1) // 2

    def fir(self):
        return fir_windowed_sinc(self.C, self.T)

    def bandpass(self):
        if self.ripple == 0.0:
            return np.ones(self.C, np.float32)
        return bandpass_ripple(self.C, self.ripple)

    def subband_freqs(self):
        if self.f_sb0 is not None:
            return self.f_sb0 + np.arange(self.SB, dtype=np.float64) * SAMPLE_RATE_HZ
        return hba_subband_freqs(self.SB)

    def delays(self, block: int = 0):
        if self.delay_spread_s == 0.0 and self.delay_drift_s == 0.0:
            return np.zeros((self.S, 2), np.float64)
        return station_delays(self.seed + 7919 * block, self.S, self.delay_spread_s, self.delay_drift_s)

    def gain(self):
        return requant_gain(self.sigma, self.fir()) if self.x_mode == X_INT8 else 1.0

    def tone_cycles_per_sample(self):
        """Baseband frequency (cycles/sample) centred on channel ``tone_channel``."""
        return (self.tone_channel - self.C // 2) / self.C

    # ---- sample generation -------------------------------------------------------
    def stream(self, block, s, p, sb):
        x = gaussian_stream(self.seed, block, s, p, sb, self.N, self.sigma, self.sample_type)
        if self.tone_amplitude:
            x = add_tone(x, self.tone_amplitude, self.tone_cycles_per_sample(), n0=block * self.N)
        return x

    def block(self, block: int = 0, subbands=None, threads: int | None = None) -> np.ndarray:
        """Input block [S, P, SB', N, 2] in the storage dtype (SB' = len(subbands))."""
        sbs = list(range(self.SB)) if subbands is None else list(subbands)
        out = np.empty((self.S, self.P, len(sbs), self.N, 2), storage_dtype(self.sample_type))
        jobs = [(s, p, i, sb) for s in range(self.S) for p in range(self.P) for i, sb in enumerate(sbs)]

        def work(job):
            s, p, i, sb = job
            out[s, p, i] = self.stream(block, s, p, sb)

        threads = threads or min(16, len(os.sched_getaffinity(0)))
        if threads <= 1 or len(jobs) < 4:
            for jb in jobs:
                work(jb)
        else:
            with _cf.ThreadPoolExecutor(threads) as ex:
                list(ex.map(work, jobs))
        return out


def workload(name: str, **overrides) -> Workload:
    """The named synthetic workloads.

    ``plain_fx``    8 stations, 1 subband, ci16 N(0, 64^2) + tone A=256 at channel 37,
                    zero delays, flat bandpass, FP32 X stage.
    ``int16_share`` 76 stations, 64 subbands, ci16 N(0, 64^2), delays U(+-5 us) with
                    +-25 ns drift, 5 % bandpass ripple, FP16-split X stage (prescale 2^-1, the
                    largest for which no 16-bit input overflows FP16 with these taps).
    ``int8_full``   76 stations, 128 subbands, ci8 N(0, 16^2) clipped to +-127, delays and
                    bandpass as int16_share, int8 X stage.
    """
    presets = {
        "plain_fx": dict(S=8, SB=1, sample_type=CI16, x_mode=X_FP32, sigma=64.0, seed=1801,
                         tone_amplitude=256.0, tone_channel=37, f_sb0=150e6),
        "int16_share": dict(S=76, SB=64, sample_type=CI16, x_mode=X_FP16_SPLIT, sigma=64.0, seed=1802,
                            delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1),
        "int8_full": dict(S=76, SB=128, sample_type=CI8, x_mode=X_INT8, sigma=16.0, seed=1803,
                          delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05),
    }
    kw = dict(presets[name])
    kw.update(overrides)
    return Workload(name=name, **kw)


def full_scale_streams(fir: np.ndarray, C: int, T: int, n: int, seed: int, sample_type: int = CI16,
                       tone_channel: int = 37, block: int = 0) -> np.ndarray:
    """Full-scale test input of four stations [4, 2, 1, n, 2] (storage dtype, one subband):

    * station 0: in every even FIR window (rows wT .. wT+T-1 of C samples, w even) sample
      t*C + p is ``sgn(h[t*C + p]) * A (1 + i)``, A = the type's largest magnitude (32767 /
      127); polarisation 1 carries the negated pattern.  The FIR output of the window's last
      row is then ``A (1 + i) sum_t |h[t*C + p]|`` for every phase p, all in phase, so FFT
      bin 0 receives ``A (1 + i) sum |h|``: the largest value any input of the type can
      produce there.  Odd windows hold N(0, (A/32)^2) noise, so no channel is empty.
    * station 1: a complex tone of amplitude A - 4 sigma_1 centred on ``tone_channel`` over
      N(0, sigma_1^2) noise (sigma_1 = 256, 8-bit: 4; 42 dB below the tone), clipped to +-A.
    * station 2: +-A per component with random signs (full-scale white noise).
    * station 3: N(0, sigma^2) noise plus a tone of amplitude A/16 on ``tone_channel``
      (strong narrowband interference on ordinary noise).
    The windows are aligned to the block start; ``block`` keys the random draws.
    """
    h = np.asarray(fir, np.float32)
    A = 127 if sample_type == CI8 else 32767
    sig = 4.0 if sample_type == CI8 else 64.0
    dt = storage_dtype(sample_type)
    rng = np.random.default_rng([seed, block, 0xF5])
    out = np.zeros((4, 2, 1, n, 2), np.float64)
    sgn = np.sign(h.astype(np.float64)).reshape(T, C)
    sgn[sgn == 0] = 1.0
    rows = n // C
    even = ((np.arange(rows) // T) % 2 == 0)[:, None]
    for p, sign in ((0, 1.0), (1, -1.0)):
        pat = np.tile(sgn, ((rows + T - 1) // T, 1))[:rows] * (sign * A)
        noise = np.clip(np.rint(rng.standard_normal((rows, C, 2)) * (A / 32)), -A, A)
        for comp in range(2):
            out[0, p, 0, :rows * C, comp] = np.where(even, pat, noise[..., comp]).reshape(-1)
    f0 = (tone_channel - C // 2) / C
    idx = np.arange(n, dtype=np.float64) + block * n
    for p in range(2):
        ph = 2 * np.pi * (f0 * idx + 0.25 * p)
        sig1 = 4.0 if sample_type == CI8 else 256.0
        nz = rng.standard_normal((n, 2)) * sig1
        out[1, p, 0, :, 0] = np.clip(np.rint((A - 4 * sig1) * np.cos(ph) + nz[:, 0]), -A, A)
        out[1, p, 0, :, 1] = np.clip(np.rint((A - 4 * sig1) * np.sin(ph) + nz[:, 1]), -A, A)
        out[2, p, 0] = A * rng.choice(np.array([-1.0, 1.0]), size=(n, 2))
        noise = np.rint(rng.standard_normal((n, 2)) * sig)
        out[3, p, 0, :, 0] = np.clip(noise[:, 0] + np.rint(A / 16 * np.cos(ph + 1.0)), -A, A)
        out[3, p, 0, :, 1] = np.clip(noise[:, 1] + np.rint(A / 16 * np.sin(ph + 1.0)), -A, A)
    return out.astype(dt)


def int8_channelised(seed: int, n_chan: int, M: int, n_c: int, pitch: int, extreme: bool = False) -> np.ndarray:
    """Random 8-bit channelised samples [n_chan, M, pitch, 2] in [-127, 127], zero pad.

    ``extreme=True`` draws only from {-127, +127} (the largest products).
    """
    rng = np.random.default_rng([seed, 0x18])
    if extreme:
        v = rng.choice(np.array([-127, 127], np.int8), size=(n_chan, M, n_c, 2))
    else:
        v = np.clip(np.rint(rng.standard_normal((n_chan, M, n_c, 2)) * 40.0), -127, 127).astype(np.int8)
    out = np.zeros((n_chan, M, pitch, 2), np.int8)
    out[:, :, :n_c] = v
    return out


def float_channelised(seed: int, n_chan: int, M: int, n_c: int, sigma: float = 8.0) -> np.ndarray:
    """Random complex channelised samples [n_chan, M, n_c] (complex128 of float32 values)."""
    rng = np.random.default_rng([seed, 0xF1])
    v = (rng.standard_normal((n_chan, M, n_c, 2)) * sigma).astype(np.float32)
    return v[..., 0].astype(np.float64) + 1j * v[..., 1].astype(np.float64)


def guarded_rows(w: "Workload", block: int, guard: int) -> np.ndarray:
    """Input rows of ``N + guard`` samples per stream [S, P, SB, N + guard, 2] (storage dtype),
    for blocks read through per-station coarse-delay windows; drawn like ``Workload.block``
    with the guard samples appended to each stream."""
    out = np.empty((w.S, w.P, w.SB, w.N + guard, 2), storage_dtype(w.sample_type))
    for s in range(w.S):
        for p in range(w.P):
            for sb in range(w.SB):
                out[s, p, sb] = gaussian_stream(w.seed, block, s, p, sb, w.N + guard, w.sigma, w.sample_type)
    return out


def lost_sample_flags(seed: int, S: int, SB: int, n: int, packet: int = 16, p_packet: float = 0.002,
                      p_sample: float = 0.0005, clean_stations=()) -> np.ndarray:
    """Lost-sample flags bool [S, SB, n]: whole packets of ``packet`` consecutive samples lost
    with probability ``p_packet`` each (packets aligned to multiples of ``packet``, as station
    packets carry fixed runs of time samples) plus isolated lost samples with probability
    ``p_sample``; the stations in ``clean_stations`` lose nothing."""
    rng = np.random.default_rng([seed, 0xF1A6])
    n_pk = (n + packet - 1) // packet
    lost_pk = rng.random((S, SB, n_pk)) < p_packet
    flags = np.repeat(lost_pk, packet, axis=-1)[..., :n]
    flags |= rng.random((S, SB, n)) < p_sample
    for s in clean_stations:
        flags[s] = False
    return flags


def pack_flags(flags: np.ndarray) -> np.ndarray:
    """bool [..., n] -> uint32 words [..., ceil(n / 32)]: bit k of word w = sample 32 w + k."""
    f = np.asarray(flags, bool)
    n = f.shape[-1]
    words = (n + 31) // 32
    pad = np.zeros(f.shape[:-1] + (words * 32,), bool)
    pad[..., :n] = f
    bits = pad.reshape(f.shape[:-1] + (words, 32)).astype(np.uint64)
    return np.sum(bits << np.arange(32, dtype=np.uint64), axis=-1).astype(np.uint32)
