"""The entry point that allocates nothing (``cobalt_correlate_noalloc``) against the plan path
(``cobalt_correlate``) on the GPU: two calls in a row, the second with a smaller input of
another setting, then a third that continues the first observation with the FIR history the
caller carried; every result equals the plan's bit for bit (same kernels on the same data), and
the continued block also matches the FP64 oracle (coherence error <= 1e-5)."""

import sys

import numpy as np
import pytest

import oracle
from paper_1801_04834_amd import synth
from tests.metrics import coherence_error, vis_complex

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def test_noalloc_equals_the_plan_path_on_consecutive_calls():
    from paper_1801_04834_amd import binding
    wA = synth.Workload(name="noallocA", S=8, SB=2, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT, N=64 * 512,
                        seed=41, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05, fp16_prescale_log2=-1)
    wB = synth.Workload(name="noallocB", S=4, SB=1, sample_type=synth.CI8, x_mode=synth.X_INT8, N=64 * 256,
                        sigma=16.0, seed=42, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05)
    xA = [torch.from_numpy(wA.block(k)).cuda() for k in range(2)]
    xB = torch.from_numpy(wB.block(0)).cuda()
    _say(f"CASE noalloc reference plans A S={wA.S} SB={wA.SB} N={wA.N}, B S={wB.S} SB={wB.SB} N={wB.N}")
    with binding.plan_for(wA) as pA:
        refA = [pA.correlate(xA[k], wA.delays(k)).clone() for k in range(2)]
    with binding.plan_for(wB) as pB:
        refB = pB.correlate(xB, wB.delays(0)).clone()
    torch.cuda.synchronize()
    kwA, kwB = binding.plan_kwargs(wA), binding.plan_kwargs(wB)
    hshape = (wA.S * 2 * wA.SB, 15 * wA.C, 2)
    H1 = torch.empty(hshape, dtype=torch.int16, device="cuda")
    H2 = torch.empty_like(H1)
    outA0 = torch.empty_like(refA[0])
    outB = torch.empty_like(refB)
    outA1 = torch.empty_like(refA[1])
    _say("CASE noalloc call 1: A block 0 (zero history in, history out)")
    binding.correlate_noalloc(xA[0], wA.delays(0), outA0, hist_out=H1, **kwA)
    _say("CASE noalloc call 2: B block 0 (smaller input, another setting)")
    binding.correlate_noalloc(xB, wB.delays(0), outB, **kwB)
    _say("CASE noalloc call 3: A block 1 (history carried by the caller)")
    binding.correlate_noalloc(xA[1], wA.delays(1), outA1, hist_in=H1, hist_out=H2, **kwA)
    torch.cuda.synchronize()
    assert torch.equal(outA0, refA[0])
    assert torch.equal(outB, refB)
    assert torch.equal(outA1, refA[1])
    # the continued block against the oracle run over both blocks
    hist = np.zeros((wA.S, 2, wA.SB, 15 * wA.C), np.complex128)
    for k in range(2):
        ref = oracle.fx_block(synth.to_complex(wA.block(k)), hist, wA.fir(), wA.bandpass(), wA.subband_freqs(),
                              synth.SAMPLE_RATE_HZ, wA.delays(k), wA.C, 16, mode="fp16_split")
        hist = ref["history"]
    eps = coherence_error(vis_complex(outA1.cpu().numpy()), ref["V"], wA.S)
    _say(f"  continued block vs oracle: eps {eps:.3e}")
    assert eps <= 1e-5
