"""Streaming service on the GPU: results alone equal results in the mix (bit for bit),
admission by HBM budget, drop-on-full FIFOs, latency accounting.

Every block's visibilities are also compared with a direct plan run of the same blocks.
"""

import numpy as np
import pytest

from paper_1801_04834_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


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
    """Bytes the service admits an observation for: plan workspace, one input block, one
    visibility buffer (+1 KiB slack), as documented for cobalt_service_open."""
    kw = binding.plan_kwargs(w)
    sb = {synth.CI8: 2, synth.CI16: 4, synth.CF32: 8}[w.sample_type]
    io = w.M * w.SB * w.N * sb + w.SB * w.C * w.n_baselines * 4 * 8
    return binding.estimate_bytes(**kw) + io + 1024


def test_admission_by_hbm_budget():
    from paper_1801_04834_amd import binding
    ws = _workloads()
    nA, nB = _need(binding, ws[0]), _need(binding, ws[1])
    _say(f"CASE service admission needA={nA} needB={nB}")
    with binding.Service(nA + nB - 1, n_slots=2, queue_depth=2) as svc:
        a = svc.open(**binding.plan_kwargs(ws[0]))
        with pytest.raises(binding.CobaltError) as ei:
            svc.open(**binding.plan_kwargs(ws[1]))
        assert ei.value.code == binding.ENOMEM
        assert svc.stats()["hbm_used_bytes"] == nA
        svc.close(a)
        assert svc.stats()["hbm_used_bytes"] == 0
        b = svc.open(**binding.plan_kwargs(ws[1]))        # memory freed by the close is admitted
        out = svc.vis_buffer(b)
        blk = _blocks(ws[1], 1)[0]
        svc.wait(svc.submit(b, blk, ws[1].delays(0), out))
        assert torch.equal(out, _direct(ws[1], [blk])[0])


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
