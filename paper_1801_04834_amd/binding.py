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

EXPORTED = ["cobalt_plan_create", "cobalt_estimate_bytes", "cobalt_fp16_prescale_max", "cobalt_plan_query", "cobalt_correlate",
            "cobalt_channelize", "cobalt_correlate_noalloc", "cobalt_correlate_ex", "cobalt_channelize_ex", "cobalt_beamform",
            "cobalt_beamform_channelized", "cobalt_beam_transform", "cobalt_correlate_channelized",
            "cobalt_reset_history",
            "cobalt_apply_gains", "cobalt_apply_gains_adjoint", "cobalt_device_copy", "cobalt_device_fanout", "cobalt_mfma_probe", "cobalt_plan_destroy",
            "cobalt_last_error", "cobalt_service_create", "cobalt_service_open", "cobalt_service_query",
            "cobalt_service_submit",
            "cobalt_service_wait", "cobalt_service_pause", "cobalt_service_get_stats", "cobalt_service_close",
            "cobalt_service_destroy", "cobalt_service_last_error"]


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


class BlockExt(ct.Structure):
    """``cobalt_block_ext``: coarse delay offsets, lost-sample flags and weights of a block."""
    _fields_ = [("row_samples", ct.c_int64), ("h_coarse_offset", ct.POINTER(ct.c_int32)),
                ("d_flags", ct.c_void_p), ("d_weights", ct.c_void_p)]


class BeamParams(ct.Structure):
    """``cobalt_beam_params``."""
    _fields_ = [("n_beams", ct.c_int32), ("n_stokes", ct.c_int32), ("n_int", ct.c_int32),
                ("voltage_stride", ct.c_int32), ("d_beam_dtau", ct.c_void_p)]


class TransformParams(ct.Structure):
    """``cobalt_transform_params``."""
    _fields_ = [("n_beams", ct.c_int32), ("c_out", ct.c_int32), ("n_stokes", ct.c_int32), ("n_int", ct.c_int32),
                ("voltage_stride", ct.c_int32)]


class ServiceStats(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("completed", ct.c_int64), ("dropped", ct.c_int64),
                ("late", ct.c_int64), ("p50_latency_s", ct.c_double), ("p99_latency_s", ct.c_double),
                ("max_latency_s", ct.c_double), ("hbm_used_bytes", ct.c_int64), ("hbm_budget_bytes", ct.c_int64),
                ("obs_admitted", ct.c_int64), ("obs_pending", ct.c_int64)]


OBS_PENDING, OBS_ADMITTED, OBS_CLOSED, OBS_FAILED = 0, 1, 2, 3


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
    lib.cobalt_fp16_prescale_max.argtypes = [ct.POINTER(Config), ct.POINTER(ct.c_int32)]
    lib.cobalt_plan_query.argtypes = [vp, ct.POINTER(PlanInfo)]
    lib.cobalt_correlate.argtypes = [vp, vp, ct.POINTER(ct.c_double), vp, vp]
    lib.cobalt_channelize.argtypes = [vp, vp, ct.POINTER(ct.c_double), vp, vp]
    lib.cobalt_correlate_noalloc.argtypes = [ct.POINTER(Config), vp, ct.POINTER(ct.c_double), vp, vp, vp, vp]
    lib.cobalt_correlate_ex.argtypes = [vp, vp, ct.POINTER(ct.c_double), ct.POINTER(BlockExt), vp, vp]
    lib.cobalt_channelize_ex.argtypes = [vp, vp, ct.POINTER(ct.c_double), ct.POINTER(BlockExt), vp, vp]
    lib.cobalt_beamform.argtypes = [vp, vp, ct.POINTER(ct.c_double), ct.POINTER(BeamParams), vp, vp, vp, vp]
    lib.cobalt_beamform_channelized.argtypes = [vp, vp, ct.POINTER(BeamParams), vp, vp, vp, vp]
    lib.cobalt_correlate_channelized.argtypes = [vp, vp, vp, vp]
    lib.cobalt_beam_transform.argtypes = [vp, vp, ct.POINTER(TransformParams), vp, vp, vp]
    lib.cobalt_reset_history.argtypes = [vp, vp]
    lib.cobalt_apply_gains.argtypes = [vp, vp, vp, vp, vp]
    lib.cobalt_apply_gains_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.cobalt_device_copy.argtypes = [vp, vp, ct.c_size_t, vp]
    lib.cobalt_mfma_probe.argtypes = [i32, ct.c_int64, i32, vp, vp]
    lib.cobalt_device_fanout.argtypes = [vp, vp, vp, ct.c_size_t, vp]
    lib.cobalt_plan_destroy.argtypes = [vp]
    lib.cobalt_last_error.argtypes = []
    lib.cobalt_last_error.restype = ct.c_char_p
    lib.cobalt_service_create.argtypes = [ct.c_size_t, i32, i32, ct.c_double, ct.POINTER(vp)]
    lib.cobalt_service_open.argtypes = [vp, ct.POINTER(Config), ct.POINTER(i32)]
    lib.cobalt_service_query.argtypes = [vp, i32, ct.POINTER(i32)]
    lib.cobalt_service_submit.argtypes = [vp, i32, vp, ct.POINTER(ct.c_double), vp, ct.POINTER(ct.c_int64)]
    lib.cobalt_service_wait.argtypes = [vp, ct.c_int64, ct.POINTER(ct.c_double)]
    lib.cobalt_service_pause.argtypes = [vp, i32]
    lib.cobalt_service_get_stats.argtypes = [vp, ct.POINTER(ServiceStats)]
    lib.cobalt_service_close.argtypes = [vp, i32]
    lib.cobalt_service_destroy.argtypes = [vp]
    lib.cobalt_service_last_error.argtypes = []
    lib.cobalt_service_last_error.restype = ct.c_char_p
    for name in EXPORTED:
        if name not in ("cobalt_last_error", "cobalt_service_last_error"):
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


def fp16_prescale_max(**kw) -> int:
    """Largest ``fp16_prescale_log2`` for which no 8/16-bit input of this setting can overflow
    FP16 (``cobalt_fp16_prescale_max``)."""
    cfg, keep = make_config(**kw)
    out = ct.c_int32(0)
    _check(load_library().cobalt_fp16_prescale_max(ct.byref(cfg), ct.byref(out)))
    del keep
    return int(out.value)


def mfma_probe(x_mode, iterations, sink, stream=None):
    """Dense MFMA rate probe (``cobalt_mfma_probe``): ``sink`` is a contiguous float32 device
    tensor of workgroups * 256 elements; returns the number of MFMA operations (flop or int8
    ops) the launch performs."""
    import torch
    if sink.dtype != torch.float32 or not sink.is_contiguous() or sink.numel() % 256:
        raise ValueError("sink: contiguous float32, a multiple of 256 elements")
    wgs = sink.numel() // 256
    _check(load_library().cobalt_mfma_probe(int(x_mode), int(iterations), wgs, ct.c_void_p(sink.data_ptr()),
                                            _stream_handle(torch, stream, sink.device)))
    per = 32768 if x_mode == 1 else 65536
    return wgs * 4 * int(iterations) * 8 * per


def device_fanout(dst0, dst1, src, stream=None):
    """``src`` copied into both ``dst0`` and ``dst1`` (contiguous device tensors of equal size)."""
    import torch
    nb = src.numel() * src.element_size()
    if any(t.numel() * t.element_size() != nb for t in (dst0, dst1)):
        raise ValueError("size mismatch")
    _check(load_library().cobalt_device_fanout(ct.c_void_p(dst0.data_ptr()), ct.c_void_p(dst1.data_ptr()),
                                               ct.c_void_p(src.data_ptr()), nb, _stream_handle(torch, stream, src.device)))
    return dst0, dst1


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

    def flag_words(self, row_samples=None):
        return ((self.N if row_samples is None else row_samples) + 31) // 32

    def weights_shape(self):
        return (self.SB, self.B)

    def _ext(self, x, coarse, flags, weights):
        """Marshal the per-block extras; returns (BlockExt, keep-alive tuple, input shape)."""
        t = self._torch
        row = x.shape[3] if x.dim() == 5 else self.N
        ext = BlockExt()
        ext.row_samples = row
        keep = []
        if coarse is not None:
            c = np.ascontiguousarray(coarse, np.int32).reshape(-1)
            if c.size != self.S:
                raise ValueError(f"coarse: need {self.S} int32 offsets")
            ext.h_coarse_offset = c.ctypes.data_as(ct.POINTER(ct.c_int32))
            keep.append(c)
        if flags is not None:
            ext.d_flags = self._dev(flags, (self.S, self.SB, self.flag_words(row)), t.int32, "flags")
        if weights is not None:
            ext.d_weights = self._dev(weights, self.weights_shape(), t.int32, "weights")
        return ext, keep, (self.S, 2, self.SB, row, 2)

    def correlate_ex(self, x, delays, coarse=None, flags=None, weights=None, out=None, stream=None):
        """Full FX chain with coarse delay offsets (int32 [S], host), lost-sample flags
        (int32 bit words [S][SB][ceil(row/32)], device) and weights (int32 [SB][B], device,
        written).  x: [S][2][SB][row_samples][2] with row_samples >= N."""
        out = self.empty_vis() if out is None else out
        d = self._delays(delays)
        ext, keep, shape = self._ext(x, coarse, flags, weights)
        _check(self._lib.cobalt_correlate_ex(
            self._ptr, self._dev(x, shape, self.input_dtype, "x"), d.ctypes.data_as(ct.POINTER(ct.c_double)),
            ct.byref(ext), self._dev(out, self.vis_shape, self.vis_dtype, "out"),
            _stream_handle(self._torch, stream, self.device)))
        del keep
        return out

    def channelize_ex(self, x, delays, coarse=None, flags=None, weights=None, out=None, stream=None):
        """F stage with the same extras as ``correlate_ex``; returns the channelised tensor."""
        out = self.empty_chan() if out is None else out
        d = self._delays(delays)
        ext, keep, shape = self._ext(x, coarse, flags, weights)
        _check(self._lib.cobalt_channelize_ex(
            self._ptr, self._dev(x, shape, self.input_dtype, "x"), d.ctypes.data_as(ct.POINTER(ct.c_double)),
            ct.byref(ext), self._dev(out, self.chan_shape, self.chan_dtype, "out"),
            _stream_handle(self._torch, stream, self.device)))
        del keep
        return out

    # ---- beamformer --------------------------------------------------------------------
    def beam_shapes(self, n_beams, n_stokes=4, n_int=1, voltage_stride=0):
        """Shapes of the coherent Stokes, voltage and incoherent Stokes outputs; voltage rows
        hold ``voltage_stride`` beams (0: n_beams; 16-beam multiples are the fast layout)."""
        n_out = self.n_c // n_int
        nbs = voltage_stride or n_beams
        return ((self.SB, self.C, n_out, n_stokes, n_beams), (self.SB, self.C, self.n_c, 2, nbs, 2),
                (self.SB, self.C, n_out, n_stokes))

    def _beam_call(self, fn, first, delays, dtau, n_stokes, n_int, coherent, voltages, incoherent, stream):
        t = self._torch
        if dtau.dtype != t.float64 or dtau.dim() != 2 or dtau.shape[1] != self.S:
            raise ValueError(f"dtau: need float64 [NB][{self.S}] on the device")
        nb = dtau.shape[0]
        # the voltage tensor's row length is the stride (rows of 16-beam multiples are faster)
        nbs = voltages.shape[4] if voltages is not None and voltages.dim() == 6 else nb
        if nbs < nb:
            raise ValueError(f"voltages: rows of {nbs} beams hold fewer than the {nb} beams")
        cs, vs, isz = self.beam_shapes(nb, n_stokes, n_int, nbs)
        bp = BeamParams(nb, n_stokes, n_int, nbs, self._dev(dtau, tuple(dtau.shape), t.float64, "dtau"))
        ptr = lambda x, shp, dt, name: None if x is None else self._dev(x, shp, dt, name)  # noqa: E731
        args = [self._ptr, first]
        if delays is not None:
            d = self._delays(delays)
            args.append(d.ctypes.data_as(ct.POINTER(ct.c_double)))
        args += [ct.byref(bp), ptr(coherent, cs, t.float32, "coherent"), ptr(voltages, vs, t.float32, "voltages"),
                 ptr(incoherent, isz, t.float32, "incoherent"), _stream_handle(t, stream, self.device)]
        _check(fn(*args))
        return coherent, voltages, incoherent

    def beamform(self, x, delays, dtau, n_stokes=4, n_int=1, coherent=None, voltages=None, incoherent=None,
                 stream=None):
        """F stage + beamformer; outputs are caller tensors (float32, ``beam_shapes``)."""
        return self._beam_call(self._lib.cobalt_beamform, self._dev(x, self.input_shape, self.input_dtype, "x"),
                               delays, dtau, n_stokes, n_int, coherent, voltages, incoherent, stream)

    def beamform_channelized(self, chan, dtau, n_stokes=4, n_int=1, coherent=None, voltages=None, incoherent=None,
                             stream=None):
        """Beamformer only on a channelised tensor of this plan."""
        return self._beam_call(self._lib.cobalt_beamform_channelized,
                               self._dev(chan, self.chan_shape, self.chan_dtype, "chan"), None, dtau, n_stokes, n_int,
                               coherent, voltages, incoherent, stream)

    def transform_shapes(self, n_beams, c_out, n_stokes=4, n_int=1, voltage_stride=0):
        """Shapes of the transformed voltages (rows of ``voltage_stride`` beams, 0: n_beams)
        and of their Stokes (``cobalt_beam_transform``)."""
        G = self.n_c * self.C // c_out
        return (self.SB, G, c_out, 2, voltage_stride or n_beams, 2), (self.SB, G // n_int, c_out, n_stokes, n_beams)

    def beam_transform(self, voltages, c_out, n_stokes=4, n_int=1, out_voltages=None, out_stokes=None, stream=None,
                       n_beams=None):
        """256 -> c_out channels of the beamformer's voltages (float32 [SB][256][N_c][2][NBs][2],
        rows of NBs beams of which the first ``n_beams`` (default NBs) are beams); outputs are
        caller tensors of ``transform_shapes`` (either may be None, not both)."""
        t = self._torch
        if voltages.dim() != 6:
            raise ValueError("voltages: need float32 [SB][C][N_c][2][NBs][2]")
        nbs = voltages.shape[4]
        nb = nbs if n_beams is None else int(n_beams)
        if not 1 <= nb <= nbs:
            raise ValueError(f"n_beams must be in [1, {nbs}] (got {nb})")
        vs = (self.SB, self.C, self.n_c, 2, nbs, 2)
        ov, osk = self.transform_shapes(nb, c_out, n_stokes, n_int, nbs)
        tp = TransformParams(nb, c_out, n_stokes, n_int, nbs)
        ptr = lambda x, shp, name: None if x is None else self._dev(x, shp, t.float32, name)  # noqa: E731
        _check(self._lib.cobalt_beam_transform(self._ptr, self._dev(voltages, vs, t.float32, "voltages"), ct.byref(tp),
                                               ptr(out_voltages, ov, "out_voltages"), ptr(out_stokes, osk, "out_stokes"),
                                               _stream_handle(t, stream, self.device)))
        return out_voltages, out_stokes

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


def correlate_noalloc(x, delays, out, hist_in=None, hist_out=None, stream=None, **kw):
    """One block of the FX chain without a plan (``cobalt_correlate_noalloc``): keywords as
    ``Plan``; ``x`` input [S][2][SB][N][2], ``out`` visibilities [SB][C][B][4][2], ``hist_in``
    / ``hist_out`` the carried FIR history [S*2*SB][(T-1)*C][2] in the input dtype (None: zeros
    / discarded); all contiguous tensors on the current device.  Returns ``out``."""
    import torch
    cfg, keep = make_config(**kw)
    S, SB, N = kw["n_stations"], kw["n_subbands"], kw["samples_per_block"]
    C, T = kw.get("n_channels", 64), kw.get("n_taps", 16)
    B = S * (S + 1) // 2
    idt = {CI8: torch.int8, CI16: torch.int16, CF32: torch.float32}[kw["sample_type"]]
    vdt = torch.int32 if kw["x_mode"] == X_INT8 else torch.float32

    def chk(t, shape, dt, name):
        if t is None:
            return None
        if not t.is_cuda or t.dtype != dt or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name}: need contiguous {dt} {tuple(shape)} on the GPU, got {t.dtype} {tuple(t.shape)}")
        return ct.c_void_p(t.data_ptr())

    d = np.ascontiguousarray(delays, np.float64).reshape(-1)
    if d.size != 2 * S:
        raise ValueError(f"delays: need {S}x2 float64 seconds")
    hshape = (S * 2 * SB, (T - 1) * C, 2)
    args = (ct.byref(cfg), chk(x, (S, 2, SB, N, 2), idt, "x"), d.ctypes.data_as(ct.POINTER(ct.c_double)),
            chk(hist_in, hshape, idt, "hist_in"), chk(hist_out, hshape, idt, "hist_out"),
            chk(out, (SB, C, B, 4, 2), vdt, "out"), _stream_handle(torch, stream, x.device))
    _check(load_library().cobalt_correlate_noalloc(*args))
    del keep
    return out


def plan_for(workload, **overrides):
    """Plan for a ``synth.Workload`` (settings only; overrides go to the config)."""
    kw = dict(n_stations=workload.S, n_subbands=workload.SB, samples_per_block=workload.N,
              sample_type=workload.sample_type, x_mode=workload.x_mode, fir=workload.fir(),
              subband_freqs=workload.subband_freqs(), bandpass=workload.bandpass(),
              requant_gain=workload.gain(), fp16_prescale_log2=workload.fp16_prescale_log2,
              n_channels=workload.C)
    kw.update(overrides)
    return Plan(**kw)


def _scheck(rc):
    if rc != COBALT_OK:
        msg = load_library().cobalt_service_last_error().decode(errors="replace")
        raise CobaltError(rc, msg)


def _host_buffer(a, nbytes, name):
    """Data pointer of a contiguous host buffer (numpy array or CPU torch tensor) holding
    exactly ``nbytes`` bytes."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError(f"{name}: host buffer must be contiguous")
        if a.nbytes != nbytes:
            raise ValueError(f"{name}: need {nbytes} bytes, got {a.nbytes}")
        return ct.c_void_p(a.ctypes.data)
    if a.is_cuda or not a.is_contiguous():
        raise ValueError(f"{name}: host buffer must be a contiguous CPU tensor")
    if a.numel() * a.element_size() != nbytes:
        raise ValueError(f"{name}: need {nbytes} bytes, got {a.numel() * a.element_size()}")
    return ct.c_void_p(a.data_ptr())


class Service:
    """Streaming service (``cobalt_service``): the HBM budget is allocated once as an arena;
    observations are admitted when their working set fits (else they wait, in arrival order,
    until closes free enough of it); blocks run on free worker streams as they arrive.  Host
    buffers passed to ``submit`` are kept referenced until ``wait`` returns for their ticket
    (use pinned tensors for asynchronous copies)."""

    def __init__(self, hbm_budget_bytes, n_slots=4, queue_depth=4, deadline_s=196608 / 195312.5):
        import torch
        self._lib = load_library()
        self._ptr = ct.c_void_p(None)
        self.device = torch.device("cuda", torch.cuda.current_device())
        _scheck(self._lib.cobalt_service_create(int(hbm_budget_bytes), int(n_slots), int(queue_depth),
                                                float(deadline_s), ct.byref(self._ptr)))
        self._obs = {}
        self._held = {}

    def open(self, **kw):
        """Open an observation (keywords as ``Plan``); returns its id.  It is admitted at once
        when its working set fits, else it waits for admission (``state``).  Raises
        CobaltError with code ENOMEM when it exceeds the whole budget."""
        cfg, keep = make_config(**kw)
        oid = ct.c_int(-1)
        _scheck(self._lib.cobalt_service_open(self._ptr, ct.byref(cfg), ct.byref(oid)))
        S, SB, C = kw["n_stations"], kw["n_subbands"], kw.get("n_channels", 64)
        B = S * (S + 1) // 2
        vis_dtype = np.int32 if kw["x_mode"] == X_INT8 else np.float32
        sample_b = {CI8: 2, CI16: 4, CF32: 8}[kw["sample_type"]]
        self._obs[oid.value] = dict(kw=kw, keep=keep, S=S, vis_shape=(SB, C, B, 4, 2), vis_dtype=vis_dtype,
                                    in_bytes=S * 2 * SB * kw["samples_per_block"] * sample_b,
                                    vis_bytes=SB * C * B * 4 * 8)
        return oid.value

    def state(self, obs_id):
        """OBS_PENDING, OBS_ADMITTED, OBS_CLOSED or OBS_FAILED."""
        st = ct.c_int(-1)
        _scheck(self._lib.cobalt_service_query(self._ptr, int(obs_id), ct.byref(st)))
        return st.value

    def vis_buffer(self, obs_id, pinned=True):
        """A host buffer for one block's visibilities of this observation."""
        import torch
        o = self._obs[obs_id]
        dt = torch.int32 if o["vis_dtype"] == np.int32 else torch.float32
        return torch.empty(o["vis_shape"], dtype=dt, pin_memory=pinned)

    def submit(self, obs_id, h_block, delays, h_vis):
        """Queue one block; returns its ticket, or None when the FIFO was full (dropped).
        ``h_block`` must hold exactly one input block of the observation and ``h_vis`` one
        visibility block (contiguous host memory)."""
        o = self._obs.get(obs_id)
        if o is None:
            raise ValueError(f"unknown observation {obs_id}")
        d = np.ascontiguousarray(delays, np.float64).reshape(-1)
        if d.size != 2 * o["S"]:
            raise ValueError("delays: need S x 2 float64 seconds")
        pin = _host_buffer(h_block, o["in_bytes"], "h_block")
        pvis = _host_buffer(h_vis, o["vis_bytes"], "h_vis")
        t = ct.c_int64(-1)
        rc = self._lib.cobalt_service_submit(self._ptr, int(obs_id), pin, d.ctypes.data_as(ct.POINTER(ct.c_double)),
                                             pvis, ct.byref(t))
        if rc == EBUSY:
            return None
        _scheck(rc)
        self._held[t.value] = (h_block, h_vis)
        return t.value

    def wait(self, ticket):
        """Block until the ticket completes; returns its latency in seconds."""
        lat = ct.c_double(0)
        rc = self._lib.cobalt_service_wait(self._ptr, ct.c_int64(ticket), ct.byref(lat))
        self._held.pop(ticket, None)
        _scheck(rc)
        return lat.value

    def pause(self, paused=True):
        _scheck(self._lib.cobalt_service_pause(self._ptr, 1 if paused else 0))

    def stats(self):
        st = ServiceStats()
        _scheck(self._lib.cobalt_service_get_stats(self._ptr, ct.byref(st)))
        return {f: getattr(st, f) for f, _ in ServiceStats._fields_}

    def close(self, obs_id):
        _scheck(self._lib.cobalt_service_close(self._ptr, int(obs_id)))
        self._obs.pop(obs_id, None)

    def destroy(self):
        if self._ptr is not None and self._ptr.value:
            rc = self._lib.cobalt_service_destroy(self._ptr)
            self._ptr = ct.c_void_p(None)
            self._held.clear()
            _scheck(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def plan_kwargs(workload, **overrides):
    """Plan keyword arguments of a ``synth.Workload``."""
    kw = dict(n_stations=workload.S, n_subbands=workload.SB, samples_per_block=workload.N,
              sample_type=workload.sample_type, x_mode=workload.x_mode, fir=workload.fir(),
              subband_freqs=workload.subband_freqs(), bandpass=workload.bandpass(),
              requant_gain=workload.gain(), fp16_prescale_log2=workload.fp16_prescale_log2,
              n_channels=workload.C)
    kw.update(overrides)
    return kw
