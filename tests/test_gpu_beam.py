"""GPU parity of the beamformer (coherent voltages and Stokes, incoherent Stokes) against the
FP64 oracle ``oracle.beam``, through the C ABI, at 256 channels.

Tolerances (FP16-split operands, FP32 accumulation; the channelised data carry at most
5e-6 rms + 2e-6 |Z| error, the weights 2^-22): voltages max |dB| <= 2e-5 rms(B); Stokes
|dS| <= 2e-5 I + 1e-6 mean(I) per element (a relative voltage error e moves I, Q, U, V by
at most about 2e I).
"""

import sys

import numpy as np
import pytest

from oracle import beam as ob
from paper_1801_04834_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C = 256


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _work(S, SB, n_c, seed, st=synth.CI16, mode=synth.X_FP16_SPLIT):
    return synth.Workload(name="beam", S=S, SB=SB, sample_type=st, x_mode=mode, N=C * n_c, C=C, sigma=64.0, seed=seed,
                          delay_spread_s=2e-6, delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1)


def _oracle(w, blocks, dtau, n_stokes, n_int):
    hist = np.zeros((w.S, 2, w.SB, 15 * C), np.complex128)
    outs = []
    for k, x in enumerate(blocks):
        o = ob.beamform_block(synth.to_complex(x), hist, w.fir(), w.bandpass(), w.subband_freqs(), synth.SAMPLE_RATE_HZ,
                              w.delays(k), dtau, C, 16, which="IQUV" if n_stokes == 4 else "I", n_int=n_int)
        hist = o["history"]
        outs.append(o)
    return outs


def _check(label, coh, volt, inc, o):
    """GPU outputs are beam-fastest; the oracle's are time-fastest."""
    coh = coh.transpose(0, 1, 4, 3, 2)
    volt = volt.transpose(0, 1, 4, 3, 2, 5)
    inc = inc.transpose(0, 1, 3, 2)
    B = o["beams"]
    Vg = volt[..., 0].astype(np.float64) + 1j * volt[..., 1]
    rms = np.sqrt(np.mean(np.abs(B) ** 2))
    ev = float(np.max(np.abs(Vg - B))) / rms
    res = {"voltages": ev}
    for name, got, want in (("coherent", coh, o["coherent"]), ("incoherent", inc, o["incoherent"])):
        I = want[..., 0:1, :]
        err = np.abs(got.astype(np.float64) - want)
        bound = 2e-5 * np.abs(I) + 1e-6 * np.mean(np.abs(I))
        res[name] = float(np.max(err / (np.abs(I) + np.mean(np.abs(I)))))
        assert np.all(err <= bound), f"{label}: {name} off, worst {res[name]:.3e}"
    _say(f"  {label}: " + "  ".join(f"{k} {v:.2e}" for k, v in res.items()))
    assert ev <= 2e-5, f"{label}: voltages off by {ev:.3e} rms"


@pytest.mark.parametrize("S,NB,n_c,n_int,n_stokes", [(6, 37, 40, 1, 4), (6, 37, 40, 8, 4), (13, 130, 64, 64, 1),
                                                     (48, 32, 96, 32, 4), (1, 1, 33, 1, 4), (56, 40, 32, 16, 1),
                                                     (48, 127, 96, 16, 1), (20, 70, 96, 8, 1), (29, 129, 64, 4, 4),
                                                     (37, 60, 50, 2, 1)])
def test_beamformer_matches_oracle(S, NB, n_c, n_int, n_stokes):
    from paper_1801_04834_amd import binding
    SB = 2
    seed = 2700 + S + NB + n_c
    w = _work(S, SB, n_c, seed)
    rng = np.random.default_rng(seed)
    dtau = rng.uniform(-4e-6, 4e-6, (NB, S))
    _say(f"CASE beam S={S} NB={NB} n_c={n_c} n_int={n_int} n_stokes={n_stokes} seed={seed}")
    blocks = [w.block(k) for k in range(2)]
    outs = _oracle(w, blocks, dtau, n_stokes, n_int)
    with binding.plan_for(w) as plan, binding.plan_for(w) as plan2:
        cs, vs, isz = plan.beam_shapes(NB, n_stokes, n_int)
        dt = torch.from_numpy(dtau).cuda()
        for k in range(2):
            x = torch.from_numpy(blocks[k]).cuda()
            coh = torch.full(cs, np.nan, dtype=torch.float32, device="cuda")
            volt = torch.full(vs, np.nan, dtype=torch.float32, device="cuda")
            inc = torch.full(isz, np.nan, dtype=torch.float32, device="cuda")
            plan.beamform(x, w.delays(k), dt, n_stokes, n_int, coherent=coh, voltages=volt, incoherent=inc)
            # the same block through the F stage + the stateless beamformer on a second plan,
            # without voltage output (a kernel built without the voltage stores): the same bits
            chan = plan2.channelize(x, w.delays(k))
            coh2 = torch.full(cs, np.nan, dtype=torch.float32, device="cuda")
            inc2 = torch.full(isz, np.nan, dtype=torch.float32, device="cuda")
            plan2.beamform_channelized(chan, dt, n_stokes, n_int, coherent=coh2, incoherent=inc2)
            torch.cuda.synchronize()
            assert torch.equal(coh, coh2)
            assert torch.equal(inc, inc2)
            _check(f"block {k}", coh.cpu().numpy(), volt.cpu().numpy(), inc.cpu().numpy(), outs[k])


@pytest.mark.parametrize("n_int", [8, 16])
def test_incoherent_only_and_coherent_only_match_the_full_call(n_int):
    """Stokes I over 8 or more samples without voltages (the interleaved kernel form): asking for
    the incoherent beam alone, or the coherent beams alone, gives the same bits as asking for
    both, and nothing is written through the output that is not asked for."""
    from paper_1801_04834_amd import binding
    S, NB, n_c = 20, 70, 64
    w = _work(S, 2, n_c, 3301 + n_int)
    dt = torch.from_numpy(np.random.default_rng(3302).uniform(-4e-6, 4e-6, (NB, S))).cuda()
    _say(f"CASE beam incoherent-only / coherent-only S={S} NB={NB} n_c={n_c} n_int={n_int}")
    with binding.plan_for(w) as plan:
        chan = plan.channelize(torch.from_numpy(w.block(0)).cuda(), w.delays(0))
        cs, _, isz = plan.beam_shapes(NB, 1, n_int)
        coh = torch.full(cs, np.nan, dtype=torch.float32, device="cuda")
        inc = torch.full(isz, np.nan, dtype=torch.float32, device="cuda")
        plan.beamform_channelized(chan, dt, 1, n_int, coherent=coh, incoherent=inc)
        inc1 = torch.full(isz, np.nan, dtype=torch.float32, device="cuda")
        plan.beamform_channelized(chan, dt, 1, n_int, incoherent=inc1)
        coh1 = torch.full(cs, np.nan, dtype=torch.float32, device="cuda")
        plan.beamform_channelized(chan, dt, 1, n_int, coherent=coh1)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(coh).all()) and bool(torch.isfinite(inc).all())
        assert torch.equal(inc1, inc) and torch.equal(coh1, coh)


def test_pointed_beam_on_a_tone():
    """A bin-centred sky tone reaching station s tau_s late: the beam with dtau = tau has
    I = 2 S^2 |z|^2 in the tone's channel (z = one station's aligned channel value), the beam
    at the centre much less, and the incoherent beam 2 S |z|^2."""
    from paper_1801_04834_amd import binding
    S, n_c, A, c0 = 8, 32, 200.0, 91
    f_s = synth.SAMPLE_RATE_HZ
    w = synth.Workload(name="beamtone", S=S, SB=1, sample_type=synth.CF32, x_mode=synth.X_FP16_SPLIT, N=C * n_c, C=C,
                       sigma=0.0, seed=3, f_sb0=768 * f_s, fp16_prescale_log2=0)
    F = 768 * f_s + (c0 - C / 2) * f_s / C
    taus = np.random.default_rng(9).uniform(-2e-6, 2e-6, S)
    _say(f"CASE beam tone c0={c0}")
    n = np.arange(2 * w.N)
    x = np.zeros((S, 2, 1, 2 * w.N, 2), np.float32)
    for s in range(S):
        v = A * np.exp(2j * np.pi * ((c0 - C // 2) / C * n - F * taus[s]))
        x[s, :, 0, :, 0] = v.real
        x[s, :, 0, :, 1] = v.imag
    with binding.plan_for(w) as plan:
        dt = torch.from_numpy(np.stack([taus, np.zeros(S)])).cuda()
        cs, vs, isz = plan.beam_shapes(2, 4, n_c)
        coh = torch.empty(cs, dtype=torch.float32, device="cuda")
        inc = torch.empty(isz, dtype=torch.float32, device="cuda")
        for k in range(2):                   # the second block is past the FIR warm-up
            xb = torch.from_numpy(np.ascontiguousarray(x[..., k * w.N:(k + 1) * w.N, :])).cuda()
            plan.beamform(xb, np.zeros((S, 2)), dt, 4, n_c, coherent=coh, incoherent=inc)
        torch.cuda.synchronize()
        one = n_c * (A * float(np.sum(w.fir().astype(np.float64)))) ** 2
        I = coh.cpu().numpy()[0, c0, 0, 0, :]
        _say(f"  pointed {I[0] / (2 * S * S * one):.6f}  centre {I[1] / (2 * S * S * one):.4f}")
        assert abs(I[0] - 2 * S * S * one) <= 2e-5 * I[0]
        assert I[1] < 0.6 * I[0]
        assert abs(inc.cpu().numpy()[0, c0, 0, 0] - 2 * S * one) <= 2e-5 * 2 * S * one


def test_beamformer_rejects_bad_parameters():
    from paper_1801_04834_amd import binding
    w = _work(4, 1, 40, 2800)
    _say("CASE beam invalid")
    dt = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    with binding.plan_for(w) as plan:
        chan = plan.empty_chan()
        coh = torch.empty(plan.beam_shapes(3, 4, 8)[0], dtype=torch.float32, device="cuda")
        for n_int in (3, 16):                # 3 is no power of two, 16 does not divide 40
            out = torch.empty(plan.beam_shapes(3, 4, n_int)[0], dtype=torch.float32, device="cuda")
            with pytest.raises(binding.CobaltError) as ei:
                plan.beamform_channelized(chan, dt, 4, n_int, coherent=out)
            assert ei.value.code == binding.EINVAL
        with pytest.raises(binding.CobaltError) as ei:
            plan.beamform_channelized(chan, dt, 4, 8)          # no output
        assert ei.value.code == binding.EINVAL
    with binding.plan_for(_work(4, 1, 40, 2801, mode=synth.X_FP32)) as plan:
        with pytest.raises(binding.CobaltError) as ei:
            plan.beamform_channelized(plan.empty_chan(), dt, 4, 8, coherent=coh)
        assert ei.value.code == binding.EUNSUPPORTED


@pytest.mark.parametrize("c_out,n_stokes,n_int", [(16, 4, 1), (16, 1, 16), (1, 4, 64), (4, 4, 8), (2, 1, 1), (8, 4, 32)])
def test_output_resolution_transform_matches_oracle(c_out, n_stokes, n_int):
    """The beamformer's 256-channel voltages transformed to c_out channels on the GPU: against
    the oracle's transform of the same GPU voltages (FP32 transform error only: <= 2e-6 of the
    rms), and against the oracle's whole chain (beams in FP64, then the transform: the voltage
    tolerance 2e-5 rms; Stokes |dS| <= 4e-5 I + 1e-6 mean(I)).  37 beams: three groups of 16,
    the last partial."""
    from paper_1801_04834_amd import binding
    S, NB, n_c, SB = 6, 37, 24, 2
    seed = 2900 + c_out + n_int
    w = _work(S, SB, n_c, seed)
    rng = np.random.default_rng(seed)
    dtau = rng.uniform(-4e-6, 4e-6, (NB, S))
    _say(f"CASE beam transform c_out={c_out} n_stokes={n_stokes} n_int={n_int} S={S} NB={NB} n_c={n_c}")
    x = w.block(0)
    o = _oracle(w, [x], dtau, 4, 1)[0]
    which = "IQUV" if n_stokes == 4 else "I"
    with binding.plan_for(w) as plan:
        _, vs, _ = plan.beam_shapes(NB, 4, 1)
        volt = torch.empty(vs, dtype=torch.float32, device="cuda")
        plan.beamform(torch.from_numpy(x).cuda(), w.delays(0), torch.from_numpy(dtau).cuda(), 4, 1, voltages=volt)
        ov, osk = plan.transform_shapes(NB, c_out, n_stokes, n_int)
        tv = torch.full(ov, np.nan, dtype=torch.float32, device="cuda")
        ts = torch.full(osk, np.nan, dtype=torch.float32, device="cuda")
        plan.beam_transform(volt, c_out, n_stokes, n_int, out_voltages=tv, out_stokes=ts)
        # Stokes only (no voltage output): the same values
        ts2 = torch.full(osk, np.nan, dtype=torch.float32, device="cuda")
        plan.beam_transform(volt, c_out, n_stokes, n_int, out_stokes=ts2)
        torch.cuda.synchronize()
        assert torch.equal(ts, ts2)
        vg = volt.cpu().numpy().astype(np.float64)               # [SB, C, n_c, P, NB, 2]
        Tg = tv.cpu().numpy().astype(np.float64)                 # [SB, G, c_out, P, NB, 2]
        Sg = ts.cpu().numpy().astype(np.float64)                 # [SB, G/n_int, c_out, n_stokes, NB]
    Tg = Tg[..., 0] + 1j * Tg[..., 1]
    # oracle transform of the GPU's own voltages: [SB, NB, P, C, n_c] -> [SB, NB, P, G, c_out]
    Bg = np.transpose(vg[..., 0] + 1j * vg[..., 1], (0, 4, 3, 1, 2))
    ref_own = ob.resolution_transform(Bg, c_out)
    got = np.transpose(Tg, (0, 4, 3, 1, 2))                     # [SB, NB, P, G, c_out]
    rms = np.sqrt(np.mean(np.abs(ref_own) ** 2))
    e_own = float(np.max(np.abs(got - ref_own))) / rms
    # the whole chain: oracle beams [SB, C, NB, P, n_c] -> [SB, NB, P, C, n_c]
    Bo = np.transpose(o["beams"], (0, 2, 3, 1, 4))
    ref = ob.resolution_transform(Bo, c_out)
    e_chain = float(np.max(np.abs(got - ref))) / np.sqrt(np.mean(np.abs(ref) ** 2))
    st = ob.transformed_stokes(Bo, c_out, which, n_int)         # [SB, NB, G/n_int, c_out, n_stokes]
    Sgt = np.transpose(Sg, (0, 4, 1, 2, 3))
    I = st[..., 0:1]
    err = np.abs(Sgt - st)
    worst = float(np.max(err / (np.abs(I) + np.mean(np.abs(I)))))
    _say(f"  voltages vs oracle transform of the same input {e_own:.2e} rms, vs oracle chain {e_chain:.2e} rms; "
         f"Stokes worst {worst:.2e}")
    assert e_own <= 2e-6
    assert e_chain <= 2e-5
    assert np.all(err <= 4e-5 * np.abs(I) + 1e-6 * np.mean(np.abs(I)))


@pytest.mark.parametrize("c_out,n_stokes,n_int", [(16, 4, 2), (4, 1, 8)])
def test_voltage_stride_matches_packed_layout(c_out, n_stokes, n_int):
    """Voltage rows padded to 48 beams (37 beams: the last group of 16 is partial and the row
    is 128-byte aligned): the beamformer's voltages and the transform's outputs equal the
    packed layout's bit for bit, and the padding beams are never read (NaN put there does not
    reach any output)."""
    from paper_1801_04834_amd import binding
    S, NB, NBS, n_c, SB = 6, 37, 48, 24, 2
    w = _work(S, SB, n_c, 3101)
    dtau = torch.from_numpy(np.random.default_rng(3102).uniform(-4e-6, 4e-6, (NB, S))).cuda()
    _say(f"CASE voltage stride NB={NB} stride={NBS} c_out={c_out} n_stokes={n_stokes} n_int={n_int}")
    with binding.plan_for(w) as plan:
        chan = plan.channelize(torch.from_numpy(w.block(0)).cuda(), w.delays(0))
        _, vs, _ = plan.beam_shapes(NB, 4, 1)
        _, vsp, _ = plan.beam_shapes(NB, 4, 1, voltage_stride=NBS)
        assert vsp[4] == NBS
        packed = torch.full(vs, np.nan, dtype=torch.float32, device="cuda")
        padded = torch.full(vsp, np.nan, dtype=torch.float32, device="cuda")
        plan.beamform_channelized(chan, dtau, 4, 1, voltages=packed)
        plan.beamform_channelized(chan, dtau, 4, 1, voltages=padded)
        torch.cuda.synchronize()
        assert torch.equal(padded[..., :NB, :], packed)
        padded[..., NB:, :] = float("nan")
        ov, osk = plan.transform_shapes(NB, c_out, n_stokes, n_int)
        ovp, _ = plan.transform_shapes(NB, c_out, n_stokes, n_int, voltage_stride=NBS)
        tv = torch.full(ov, np.nan, dtype=torch.float32, device="cuda")
        ts = torch.full(osk, np.nan, dtype=torch.float32, device="cuda")
        tvp = torch.full(ovp, np.nan, dtype=torch.float32, device="cuda")
        tsp = torch.full(osk, np.nan, dtype=torch.float32, device="cuda")
        plan.beam_transform(packed, c_out, n_stokes, n_int, out_voltages=tv, out_stokes=ts)
        plan.beam_transform(padded, c_out, n_stokes, n_int, out_voltages=tvp, out_stokes=tsp, n_beams=NB)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(tv).all()) and bool(torch.isfinite(ts).all())
        assert torch.equal(tvp[..., :NB, :], tv) and torch.equal(tsp, ts)
        # strides below the beam count are refused
        tp = binding.TransformParams(NB, c_out, n_stokes, n_int, NB - 1)
        rc = plan._lib.cobalt_beam_transform(plan._ptr, binding.ct.c_void_p(padded.data_ptr()), binding.ct.byref(tp),
                                             None, binding.ct.c_void_p(tsp.data_ptr()), None)
        assert rc == binding.EINVAL
        bp = binding.BeamParams(NB, 4, 1, NB - 1, binding.ct.c_void_p(dtau.data_ptr()))
        rc = plan._lib.cobalt_beamform_channelized(plan._ptr, binding.ct.c_void_p(chan.data_ptr()), binding.ct.byref(bp),
                                                   None, binding.ct.c_void_p(padded.data_ptr()), None, None)
        assert rc == binding.EINVAL


def test_output_resolution_transform_rejects_bad_settings():
    from paper_1801_04834_amd import binding
    w = _work(2, 1, 16, 5)
    with binding.plan_for(w) as plan:
        _, vs, _ = plan.beam_shapes(3, 4, 1)
        volt = torch.zeros(vs, dtype=torch.float32, device="cuda")
        sink = torch.empty(1 << 20, device="cuda")          # never written: every call is refused
        for c_out, n_int, code in ((3, 1, binding.EUNSUPPORTED), (32, 1, binding.EUNSUPPORTED),
                                   (16, 32, binding.EINVAL), (16, 3, binding.EINVAL)):
            tp = binding.TransformParams(3, c_out, 4, n_int, 0)
            rc = plan._lib.cobalt_beam_transform(plan._ptr, binding.ct.c_void_p(volt.data_ptr()), binding.ct.byref(tp),
                                                 None, binding.ct.c_void_p(sink.data_ptr()), None)
            assert rc == code, (c_out, n_int, rc)
    w64 = synth.Workload(name="beam64", S=2, SB=1, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, N=64 * 16,
                         fp16_prescale_log2=-1)
    with binding.plan_for(w64) as plan:
        tp = binding.TransformParams(3, 16, 4, 1, 0)
        buf = torch.empty(1 << 20, device="cuda")
        rc = plan._lib.cobalt_beam_transform(plan._ptr, binding.ct.c_void_p(buf.data_ptr()), binding.ct.byref(tp),
                                             binding.ct.c_void_p(buf.data_ptr()), None, None)
        assert rc == binding.EUNSUPPORTED
