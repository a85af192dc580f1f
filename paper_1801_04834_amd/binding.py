"""ctypes binding of ``libcobalt.so`` (C ABI in ``include/cobalt.h``).

Argument marshalling only: torch tensors supply device memory and the HIP stream, every
step of the FX chain runs in the library's HIP kernels.  There is no CPU fallback; if
the library is missing or fails to load, creating a ``Plan`` raises.
"""

from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libcobalt.so")

CI8, CI16, CF32 = 1, 2, 3
X_FP32, X_FP16_SPLIT, X_INT8 = 0, 1, 2

COBALT_OK, EINVAL, EUNSUPPORTED, EOVERFLOW, ENOMEM, EBUSY, EDEVICE = 0, -1, -2, -3, -4, -5, -6
_CODES = {EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", EOVERFLOW: "EOVERFLOW", ENOMEM: "ENOMEM",
          EBUSY: "EBUSY", EDEVICE: "EDEVICE"}

EXPORTED = ["cobalt_plan_create", "cobalt_estimate_bytes", "cobalt_plan_query", "cobalt_correlate",
            "cobalt_channelize", "cobalt_correlate_channelized", "cobalt_reset_history",
            "cobalt_apply_gains", "cobalt_apply_gains_adjoint", "cobalt_device_copy", "cobalt_plan_destroy",
            "cobalt_last_error"]


class CobaltError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{_CODES.get(code, code)}: {message}")
        self.code = code


class Config(ct.Structure):
    _fields_ = [
        ("n_stations", ct.c_int32), ("n_pols", ct.c_int32), ("n_subbands", ct.c_int32),
        ("n_channels", ct.c_int32), ("n_taps", ct.c_int32), ("sample_type", ct.c_int32),
        ("x_mode", ct.c_int32), ("fp16_prescale_log2", ct.c_int32),
        ("samples_per_block", ct.c_int64), ("sample_rate_hz", ct.c_double),
        ("requant_gain", ct.c_float), ("reserved0", ct.c_int32),
        ("h_fir", ct.POINTER(ct.c_float)), ("h_bandpass", ct.POINTER(ct.c_float)),
        ("h_subband_freq_hz", ct.POINTER(ct.c_double)),
    ]


class PlanInfo(ct.Structure):
    _fields_ = [(n, ct.c_int64) for n in (
        "n_channel_samples", "chan_pitch", "n_baselines", "input_bytes", "chan_bytes",
        "vis_bytes", "workspace_bytes", "useful_cmacs")]


_LIB = None


def load_library():
    """Load libcobalt.so (once).  Raises RuntimeError when it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(lib_path):
        raise RuntimeError(f"{lib_path} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ct.CDLL(lib_path)
    vp, i32 = ct.c_void_p, ct.c_int
    lib.cobalt_plan_create.argtypes = [ct.POINTER(Config), ct.POINTER(vp)]
    lib.cobalt_estimate_bytes.argtypes = [ct.POINTER(Config), ct.POINTER(ct.c_size_t)]
    lib.cobalt_plan_query.argtypes = [vp, ct.POINTER(PlanInfo)]
    lib.cobalt_correlate.argtypes = [vp, vp, ct.POINTER(ct.c_double), vp, vp]
    lib.cobalt_channelize.argtypes = [vp, vp, ct.POINTER(ct.c_double), vp, vp]
    lib.cobalt_correlate_channelized.argtypes = [vp, vp, vp, vp]
    lib.cobalt_reset_history.argtypes = [vp, vp]
    lib.cobalt_apply_gains.argtypes = [vp, vp, vp, vp, vp]
    lib.cobalt_apply_gains_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.cobalt_device_copy.argtypes = [vp, vp, ct.c_size_t, vp]
    lib.cobalt_plan_destroy.argtypes = [vp]
    lib.cobalt_last_error.argtypes = []
    lib.cobalt_last_error.restype = ct.c_char_p
    for name in EXPORTED[:-1]:
        getattr(lib, name).restype = i32
    _LIB = lib
    return lib


def _check(rc):
    if rc != COBALT_OK:
        msg = load_library().cobalt_last_error().decode(errors="replace")
        raise CobaltError(rc, msg)


class _HostArrays:
    """Keeps the host tables referenced by a Config alive."""

    def __init__(self, fir, bandpass, freqs):
        self.fir = np.ascontiguousarray(fir, np.float32)
        self.bandpass = None if bandpass is None else np.ascontiguousarray(bandpass, np.float32)
        self.freqs = np.ascontiguousarray(freqs, np.float64)


def make_config(n_stations, n_subbands, samples_per_block, sample_type, x_mode, fir, subband_freqs,
                sample_rate=195312.5, bandpass=None, requant_gain=1.0, fp16_prescale_log2=0,
                n_channels=64, n_taps=16, n_pols=2):
    keep = _HostArrays(fir, bandpass, subband_freqs)
    cfg = Config()
    cfg.n_stations, cfg.n_pols, cfg.n_subbands = n_stations, n_pols, n_subbands
    cfg.n_channels, cfg.n_taps = n_channels, n_taps
    cfg.sample_type, cfg.x_mode, cfg.fp16_prescale_log2 = sample_type, x_mode, fp16_prescale_log2
    cfg.samples_per_block, cfg.sample_rate_hz = samples_per_block, sample_rate
    cfg.requant_gain, cfg.reserved0 = requant_gain, 0
    cfg.h_fir = keep.fir.ctypes.data_as(ct.POINTER(ct.c_float)) if keep.fir.size else None
    cfg.h_bandpass = None if keep.bandpass is None else keep.bandpass.ctypes.data_as(ct.POINTER(ct.c_float))
    cfg.h_subband_freq_hz = keep.freqs.ctypes.data_as(ct.POINTER(ct.c_double)) if keep.freqs.size else None
    return cfg, keep


def estimate_bytes(**kw) -> int:
    """Device bytes a plan with these settings would allocate (``cobalt_estimate_bytes``)."""
    cfg, keep = make_config(**kw)
    out = ct.c_size_t(0)
    _check(load_library().cobalt_estimate_bytes(ct.byref(cfg), ct.byref(out)))
    del keep
    return int(out.value)


def device_copy(dst, src, stream=None):
    """Plain 16-byte-per-lane copy between two contiguous device tensors of equal size."""
    import torch
    if dst.numel() * dst.element_size() != src.numel() * src.element_size():
        raise ValueError("size mismatch")
    _check(load_library().cobalt_device_copy(ct.c_void_p(dst.data_ptr()), ct.c_void_p(src.data_ptr()),
                                             dst.numel() * dst.element_size(),
                                             _stream_handle(torch, stream, dst.device)))
    return dst


def _stream_handle(torch, stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ct.c_void_p(s.cuda_stream)


class Plan:
    """One observation setting on one GPU (``cobalt_plan``).

    Keyword arguments follow ``cobalt_config``; ``fir`` [T*C] float32, ``subband_freqs``
    [SB] float64 (Hz), ``bandpass`` [C] or None.  Tensors passed to the methods must be
    contiguous, on the plan's device, with the shapes ``input_shape``, ``chan_shape`` and
    ``vis_shape`` and the matching dtypes.
    """

    def __init__(self, *, device=None, **kw):
        import torch
        self._torch = torch
        self._lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.kw = dict(kw)
        cfg, self._keep = make_config(**kw)
        self._ptr = ct.c_void_p(None)
        with torch.cuda.device(self.device):
            _check(self._lib.cobalt_plan_create(ct.byref(cfg), ct.byref(self._ptr)))
        info = PlanInfo()
        _check(self._lib.cobalt_plan_query(self._ptr, ct.byref(info)))
        self.info = {f: int(getattr(info, f)) for f, _ in PlanInfo._fields_}
        self.S = kw["n_stations"]
        self.SB = kw["n_subbands"]
        self.C = kw.get("n_channels", 64)
        self.N = kw["samples_per_block"]
        self.sample_type = kw["sample_type"]
        self.x_mode = kw["x_mode"]
        self.M = 2 * self.S
        self.n_c = self.info["n_channel_samples"]
        self.pitch = self.info["chan_pitch"]
        self.B = self.info["n_baselines"]

    # ---- shapes and dtypes -----------------------------------------------------------
    @property
    def input_dtype(self):
        t = self._torch
        return {CI8: t.int8, CI16: t.int16, CF32: t.float32}[self.sample_type]

    @property
    def input_shape(self):
        return (self.S, 2, self.SB, self.N, 2)

    @property
    def chan_dtype(self):
        t = self._torch
        return {X_FP32: t.float32, X_FP16_SPLIT: t.float16, X_INT8: t.int8}[self.x_mode]

    @property
    def n_kb(self):
        return self.pitch // 32

    @property
    def chan_shape(self):
        """K-blocked: [SB][C][n_kb]([2 planes])[M][32][re, im]."""
        if self.x_mode == X_FP16_SPLIT:
            return (self.SB, self.C, self.n_kb, 2, self.M, 32, 2)
        return (self.SB, self.C, self.n_kb, self.M, 32, 2)

    @property
    def vis_dtype(self):
        t = self._torch
        return t.int32 if self.x_mode == X_INT8 else t.float32

    @property
    def vis_shape(self):
        return (self.SB, self.C, self.B, 4, 2)

    def empty_vis(self):
        return self._torch.empty(self.vis_shape, dtype=self.vis_dtype, device=self.device)

    def empty_chan(self):
        return self._torch.empty(self.chan_shape, dtype=self.chan_dtype, device=self.device)

    # ---- calls -----------------------------------------------------------------------
    def _dev(self, t, shape, dtype, name):
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name}: need contiguous {dtype} {tuple(shape)} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")
        return ct.c_void_p(t.data_ptr())

    def _delays(self, delays):
        d = np.ascontiguousarray(delays, np.float64).reshape(-1)
        if d.size != 2 * self.S:
            raise ValueError(f"delays: need {self.S}x2 float64 seconds")
        return d

    def correlate(self, x, delays, out=None, stream=None):
        """Full FX chain of one block; returns the visibility tensor."""
        out = self.empty_vis() if out is None else out
        d = self._delays(delays)
        _check(self._lib.cobalt_correlate(
            self._ptr, self._dev(x, self.input_shape, self.input_dtype, "x"),
            d.ctypes.data_as(ct.POINTER(ct.c_double)), self._dev(out, self.vis_shape, self.vis_dtype, "out"),
            _stream_handle(self._torch, stream, self.device)))
        return out

    def channelize(self, x, delays, out=None, stream=None):
        """F stage only; returns the channelised tensor."""
        out = self.empty_chan() if out is None else out
        d = self._delays(delays)
        _check(self._lib.cobalt_channelize(
            self._ptr, self._dev(x, self.input_shape, self.input_dtype, "x"),
            d.ctypes.data_as(ct.POINTER(ct.c_double)), self._dev(out, self.chan_shape, self.chan_dtype, "out"),
            _stream_handle(self._torch, stream, self.device)))
        return out

    def correlate_channelized(self, chan, out=None, stream=None):
        """X stage only on a channelised tensor; returns the visibility tensor."""
        out = self.empty_vis() if out is None else out
        _check(self._lib.cobalt_correlate_channelized(
            self._ptr, self._dev(chan, self.chan_shape, self.chan_dtype, "chan"),
            self._dev(out, self.vis_shape, self.vis_dtype, "out"),
            _stream_handle(self._torch, stream, self.device)))
        return out

    @property
    def gains_shape(self):
        return (self.SB, self.C, self.M)

    def apply_gains(self, vis0, gains, out=None, stream=None):
        """V'[sb,c,bl,q] = g[a] conj(g[b]) V0[sb,c,bl,q]; complex64 tensors (vis [SB,C,B,4],
        gains [SB,C,M])."""
        t = self._torch
        out = t.empty_like(vis0) if out is None else out
        vshape = self.vis_shape[:-1]
        _check(self._lib.cobalt_apply_gains(
            self._ptr, self._dev(vis0, vshape, t.complex64, "vis0"), self._dev(gains, self.gains_shape, t.complex64, "gains"),
            self._dev(out, vshape, t.complex64, "out"), _stream_handle(t, stream, self.device)))
        return out

    def apply_gains_adjoint(self, vis0, gains, grad_vis, out=None, stream=None):
        """dL/dg (dL/dRe g + i dL/dIm g) from the upstream gradient with respect to V'."""
        t = self._torch
        out = t.empty_like(gains) if out is None else out
        vshape = self.vis_shape[:-1]
        _check(self._lib.cobalt_apply_gains_adjoint(
            self._ptr, self._dev(vis0, vshape, t.complex64, "vis0"), self._dev(gains, self.gains_shape, t.complex64, "gains"),
            self._dev(grad_vis, vshape, t.complex64, "grad_vis"), self._dev(out, self.gains_shape, t.complex64, "out"),
            _stream_handle(t, stream, self.device)))
        return out

    def reset_history(self, stream=None):
        _check(self._lib.cobalt_reset_history(self._ptr, _stream_handle(self._torch, stream, self.device)))

    def close(self):
        if self._ptr is not None and self._ptr.value:
            rc = self._lib.cobalt_plan_destroy(self._ptr)
            self._ptr = ct.c_void_p(None)
            _check(rc)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_for(workload, **overrides):
    """Plan for a ``synth.Workload`` (settings only; overrides go to the config)."""
    kw = dict(n_stations=workload.S, n_subbands=workload.SB, samples_per_block=workload.N,
              sample_type=workload.sample_type, x_mode=workload.x_mode, fir=workload.fir(),
              subband_freqs=workload.subband_freqs(), bandpass=workload.bandpass(),
              requant_gain=workload.gain(), fp16_prescale_log2=workload.fp16_prescale_log2)
    kw.update(overrides)
    return Plan(**kw)
