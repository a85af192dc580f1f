"""Streaming service on the GPU: results alone equal results in the mix (bit for bit) and the
FP64 oracle's, admission by HBM budget (an observation that does not fit waits and is admitted
when a close frees the arena), drop-on-full FIFOs, latency accounting, opens and closes from
concurrent host threads.

Every block's visibilities are compared with a direct plan run of the same blocks; at the
streaming-service workload's shapes (24 / 48 / 76 stations, 32 / 64 / 128 subbands, ci16 / ci16
/ ci8, two blocks each, every block submitted before any wait) also with the oracle on sampled
subbands (16-bit: coherence error <= 1e-5; 8-bit: entries with no rounding-ambiguous input
element bit-exact, the rest within one flipped component per ambiguous element).
"""

import sys
import threading

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.metrics import coherence_error, near_rounding_boundary, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS_FP16 = 1e-5


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _workloads():
    n = 64 * 256
    return [
        synth.Workload(name="obsA", S=4, SB=2, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, N=n, seed=1805,
                       delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1),
        synth.Workload(name="obsB", S=6, SB=1, sample_type=synth.CI8, x_mode=synth.X_INT8, N=n, sigma=16.0,
                       seed=1806, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05),
        synth.Workload(name="obsC", S=3, SB=3, sample_type=synth.CI16, x_mode=synth.X_FP32, N=n, seed=1807,
                       delay_spread_s=5e-6, delay_drift_s=25e-9),
    ]


def _blocks(w, n):
    return [torch.from_numpy(w.block(k)).pin_memory() for k in range(n)]


def _direct(w, blocks):
    from paper_1801_04834_amd import binding
    out = []
    with binding.plan_for(w) as plan:
        for k, x in enumerate(blocks):
            out.append(plan.correlate(x.cuda(), w.delays(k)).cpu())
    torch.cuda.synchronize()
    return out


def test_each_result_is_the_same_alone_and_in_the_mix():
    from paper_1801_04834_amd import binding
    ws = _workloads()
    nblk = 3
    blocks = [_blocks(w, nblk) for w in ws]
    direct = [_direct(w, b) for w, b in zip(ws, blocks)]
    budget = 8 * 2**30
    # alone: one observation per service, blocks one at a time
    alone = []
    for w, bl in zip(ws, blocks):
        _say(f"CASE service alone {w.name}")
        with binding.Service(budget, n_slots=4, queue_depth=4) as svc:
            oid = svc.open(**binding.plan_kwargs(w))
            assert svc.state(oid) == binding.OBS_ADMITTED
            res = []
            for k in range(nblk):
                out = svc.vis_buffer(oid)
                t = svc.submit(oid, bl[k], w.delays(k), out)
                svc.wait(t)
                res.append(out.clone())
            alone.append(res)
    # mix: all observations open, every block submitted before any wait
    _say("CASE service mix")
    with binding.Service(budget, n_slots=3, queue_depth=nblk) as svc:
        oids = [svc.open(**binding.plan_kwargs(w)) for w in ws]
        outs = [[svc.vis_buffer(o) for _ in range(nblk)] for o in oids]
        tickets = []
        for k in range(nblk):
            for i, w in enumerate(ws):
                t = svc.submit(oids[i], blocks[i][k], w.delays(k), outs[i][k])
                assert t is not None
                tickets.append(t)
        lats = [svc.wait(t) for t in tickets]
        st = svc.stats()
        _say(f"  stats {st}")
        assert st["completed"] == len(tickets) and st["dropped"] == 0
        assert 0 < st["p50_latency_s"] <= st["p99_latency_s"] <= st["max_latency_s"]
        assert max(lats) == pytest.approx(st["max_latency_s"])
    for i in range(len(ws)):
        for k in range(nblk):
            assert torch.equal(alone[i][k], outs[i][k]), (ws[i].name, k)
            assert torch.equal(direct[i][k], outs[i][k]), (ws[i].name, k)


def _need(binding, w):
    """Arena bytes of an observation's working set: plan workspace, one input block, one
    visibility buffer, each rounded up to 256 bytes (as documented for the service)."""
    up = lambda v: (v + 255) // 256 * 256  # noqa: E731
    sb = {synth.CI8: 2, synth.CI16: 4, synth.CF32: 8}[w.sample_type]
    return (up(binding.estimate_bytes(**binding.plan_kwargs(w))) + up(w.M * w.SB * w.N * sb)
            + up(w.SB * w.C * w.n_baselines * 4 * 8))


def test_observation_waits_for_memory_and_is_admitted_when_a_close_frees_it():
    """A budget of B + max(A, C): B and A fit (B opened first, so A's range is the arena's
    tail), C waits (its block queues), closing A frees a range C fits in and admits C, C's
    block runs and equals a direct plan run; the arena accounting returns to zero."""
    from paper_1801_04834_amd import binding
    ws = _workloads()
    nA, nB, nC = (_need(binding, w) for w in ws)
    _say(f"CASE service admission needA={nA} needB={nB} needC={nC}")
    blk = [_blocks(w, 1)[0] for w in ws]
    with binding.Service(nB + max(nA, nC), n_slots=2, queue_depth=2) as svc:
        b = svc.open(**binding.plan_kwargs(ws[1]))
        a = svc.open(**binding.plan_kwargs(ws[0]))
        assert svc.state(a) == svc.state(b) == binding.OBS_ADMITTED
        c = svc.open(**binding.plan_kwargs(ws[2]))
        assert svc.state(c) == binding.OBS_PENDING
        st = svc.stats()
        assert st["hbm_used_bytes"] == nA + nB and st["obs_admitted"] == 2 and st["obs_pending"] == 1
        outs = [svc.vis_buffer(o) for o in (a, b, c)]
        tc = svc.submit(c, blk[2], ws[2].delays(0), outs[2])       # queued while C waits
        tb = svc.submit(b, blk[1], ws[1].delays(0), outs[1])
        svc.wait(tb)
        assert svc.state(c) == binding.OBS_PENDING
        svc.close(a)                                                # frees A's range: C fits
        svc.wait(tc)
        assert svc.state(c) == binding.OBS_ADMITTED and svc.state(a) == binding.OBS_CLOSED
        st = svc.stats()
        assert st["hbm_used_bytes"] == nB + nC and st["obs_pending"] == 0
        assert torch.equal(outs[2], _direct(ws[2], [blk[2]])[0])
        assert torch.equal(outs[1], _direct(ws[1], [blk[1]])[0])
        svc.close(b)
        svc.close(c)
        assert svc.stats()["hbm_used_bytes"] == 0


def test_too_large_an_observation_is_refused_and_pending_blocks_drop_on_close():
    from paper_1801_04834_amd import binding
    ws = _workloads()
    nA, nC = _need(binding, ws[0]), _need(binding, ws[2])
    _say("CASE service refusal")
    with binding.Service(max(nA, nC), n_slots=1, queue_depth=2) as svc:
        with pytest.raises(binding.CobaltError) as ei:
            svc.open(**binding.plan_kwargs(ws[0], n_stations=8))       # more than the whole budget
        assert ei.value.code == binding.ENOMEM
        a = svc.open(**binding.plan_kwargs(ws[0]))
        c = svc.open(**binding.plan_kwargs(ws[2]))
        assert svc.state(c) == binding.OBS_PENDING
        out = svc.vis_buffer(c)
        t = svc.submit(c, _blocks(ws[2], 1)[0], ws[2].delays(0), out)
        svc.close(c)                                                # closed before admission
        with pytest.raises(binding.CobaltError) as ei:
            svc.wait(t)
        assert ei.value.code == binding.EBUSY
        assert svc.stats()["dropped"] == 1
        svc.close(a)


def test_submit_checks_host_buffer_sizes():
    from paper_1801_04834_amd import binding
    ws = _workloads()
    with binding.Service(8 * 2**30, n_slots=1, queue_depth=2) as svc:
        a = svc.open(**binding.plan_kwargs(ws[0]))
        b = svc.open(**binding.plan_kwargs(ws[1]))
        blk = _blocks(ws[0], 1)[0]
        with pytest.raises(ValueError):
            svc.submit(a, blk, ws[0].delays(0), svc.vis_buffer(b))     # another observation's buffer
        with pytest.raises(ValueError):
            svc.submit(a, blk[:, :, :1].contiguous(), ws[0].delays(0), svc.vis_buffer(a))
        assert svc.stats()["submitted"] == 0


def test_opens_and_closes_from_concurrent_threads():
    """One thread keeps opening, running and closing observations while another does the same
    with a different setting: every block equals its direct plan run."""
    from paper_1801_04834_amd import binding
    ws = _workloads()
    blk = [_blocks(w, 1)[0] for w in ws[:2]]
    ref = [_direct(w, [b])[0] for w, b in zip(ws[:2], blk)]
    _say("CASE service concurrent open/close")
    errors = []
    with binding.Service(8 * 2**30, n_slots=2, queue_depth=2) as svc:
        def loop(i):
            try:
                for _ in range(6):
                    o = svc.open(**binding.plan_kwargs(ws[i]))
                    out = svc.vis_buffer(o)
                    svc.wait(svc.submit(o, blk[i], ws[i].delays(0), out))
                    if not torch.equal(out, ref[i]):
                        errors.append(f"mismatch in thread {i}")
                    svc.close(o)
            except Exception as e:  # noqa: BLE001
                errors.append(repr(e))
        ths = [threading.Thread(target=loop, args=(i,)) for i in range(2)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        assert svc.stats()["hbm_used_bytes"] == 0
    assert not errors, errors


def test_full_fifo_drops_the_new_block():
    from paper_1801_04834_amd import binding
    w = _workloads()[0]
    _say("CASE service drop")
    with binding.Service(8 * 2**30, n_slots=2, queue_depth=2) as svc:
        oid = svc.open(**binding.plan_kwargs(w))
        blk = _blocks(w, 1)[0]
        outs = [svc.vis_buffer(oid) for _ in range(3)]
        svc.pause(True)                            # hold dispatch so the FIFO fills
        t0 = svc.submit(oid, blk, w.delays(0), outs[0])
        t1 = svc.submit(oid, blk, w.delays(0), outs[1])
        t2 = svc.submit(oid, blk, w.delays(0), outs[2])
        assert t0 is not None and t1 is not None and t2 is None
        svc.pause(False)
        svc.wait(t0)
        svc.wait(t1)
        st = svc.stats()
        assert st["dropped"] == 1 and st["completed"] == 2 and st["submitted"] == 3


# ------------------------------------------------------------ streaming-service shapes ----

def service_workloads():
    """The three concurrent observations of the streaming-service workload."""
    kw = dict(delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05)
    return [synth.Workload(name="O1", S=24, SB=32, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, seed=1805,
                           fp16_prescale_log2=-1, **kw),
            synth.Workload(name="O2", S=48, SB=64, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, seed=1806,
                           fp16_prescale_log2=-1, **kw),
            synth.Workload(name="O3", S=76, SB=128, sample_type=synth.CI8, x_mode=synth.X_INT8, sigma=16.0, seed=1807,
                           **kw)]


def _host_block(w, k):
    dt = {synth.CI8: torch.int8, synth.CI16: torch.int16}[w.sample_type]
    x = torch.empty((w.S, 2, w.SB, w.N, 2), dtype=dt, pin_memory=True)
    for sb0 in range(0, w.SB, 16):
        sbs = list(range(sb0, min(w.SB, sb0 + 16)))
        x[:, :, sb0:sb0 + len(sbs)].copy_(torch.from_numpy(w.block(k, subbands=sbs)))
    return x


def _check_against_oracle(w, blocks_sb, sb, got):
    """Visibilities of subband ``sb`` over consecutive blocks (``got``: list of [C, B, 4, 2])
    against the oracle run on that subband alone (history carried)."""
    mode = {synth.X_FP16_SPLIT: "fp16_split", synth.X_INT8: "int8"}[w.x_mode]
    hist = np.zeros((w.S, 2, 1, 15 * w.C), np.complex128)
    for k, x in enumerate(blocks_sb):
        ref = oracle.fx_block(synth.to_complex(x), hist, w.fir(), w.bandpass(), w.subband_freqs()[[sb]],
                              synth.SAMPLE_RATE_HZ, w.delays(k), w.C, 16, mode=mode, gain=w.gain())
        hist = ref["history"]
        if w.x_mode == synth.X_INT8:
            g = got[k].astype(np.int64)[None]
            V = ref["V"]
            gg = np.float64(np.float32(w.gain()))
            Zf = ref["Zf"]
            pre = np.stack([(gg * Zf.real).astype(np.float32), (gg * Zf.imag).astype(np.float32)], -1)
            amb = near_rounding_boundary(pre, 1e-3).any(-1).sum(-1)     # [1, C, M]
            exact = 0
            for s1 in range(w.S):
                for s2 in range(s1 + 1):
                    bl = s1 * (s1 + 1) // 2 + s2
                    for p1 in range(2):
                        for p2 in range(2):
                            a, b = 2 * s1 + p1, 2 * s2 + p2
                            n_amb = amb[:, :, a] + (amb[:, :, b] if b != a else 0)
                            d = np.abs(g[:, :, bl, 2 * p1 + p2] - V[:, :, bl, 2 * p1 + p2]).max(-1)
                            assert np.all(d <= 2 * (2 * 127 + 1) * n_amb)
                            assert np.all(d[n_amb == 0] == 0)
                            exact += int((n_amb == 0).sum())
            _say(f"  {w.name} block {k} subband {sb}: {exact} entries bit-exact, the rest within the rounding rule")
        else:
            eps = coherence_error(vis_complex(got[k])[None], ref["V"], w.S)
            _say(f"  {w.name} block {k} subband {sb}: eps {eps:.3e}")
            assert eps <= EPS_FP16


def test_streaming_service_shapes_match_alone_and_oracle():
    """The three observations of the streaming-service workload, two blocks each, every block
    submitted before any wait on a 48 GiB service: each block's visibilities equal the
    observation's plan run alone (bit for bit) and, on two sampled subbands, the oracle's."""
    from paper_1801_04834_amd import binding
    ws = service_workloads()
    nblk = 2
    _say("CASE service workload shapes: generating inputs")
    host = [[_host_block(w, k) for k in range(nblk)] for w in ws]
    alone = []
    for w, hb in zip(ws, host):
        _say(f"CASE service alone {w.name} S={w.S} SB={w.SB}")
        alone.append([v.numpy().copy() for v in _direct(w, hb)])
        torch.cuda.empty_cache()
    _say("CASE service mix of O1, O2, O3")
    with binding.Service(48 * 2**30, n_slots=3, queue_depth=nblk) as svc:
        oids = [svc.open(**binding.plan_kwargs(w)) for w in ws]
        assert all(svc.state(o) == binding.OBS_ADMITTED for o in oids)
        outs = [[svc.vis_buffer(o) for _ in range(nblk)] for o in oids]
        tickets = []
        for k in range(nblk):
            for i, w in enumerate(ws):
                t = svc.submit(oids[i], host[i][k], w.delays(k), outs[i][k])
                assert t is not None
                tickets.append(t)
        lats = [svc.wait(t) for t in tickets]
        st = svc.stats()
        _say(f"  latencies {[round(v * 1e3, 1) for v in lats]} ms; stats {st}")
        assert st["completed"] == len(tickets) and st["dropped"] == 0
    for i, w in enumerate(ws):
        for k in range(nblk):
            assert np.array_equal(outs[i][k].numpy(), alone[i][k]), (w.name, k)
        for sb in (0, w.SB - 1):
            blocks_sb = [w.block(k, subbands=[sb]) for k in range(nblk)]
            _check_against_oracle(w, blocks_sb, sb, [outs[i][k].numpy()[sb] for k in range(nblk)])
