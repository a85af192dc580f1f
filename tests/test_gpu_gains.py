"""GPU parity of the differentiable gain-applied correlator (forward, HIP adjoint, autograd).

Expected values come from ``oracle.gains`` (FP64); the adjoint is also checked against
central finite differences of the GPU forward.  Tolerances: forward and adjoint relative
error <= 2e-6 of the largest magnitude (FP32 complex products and sums of <= 4S terms).
"""

import numpy as np
import pytest

import oracle
from oracle import gains as og
from paper_1801_04834_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


def _plan(S, SB, mode=synth.X_FP16_SPLIT, n_c=64):
    from paper_1801_04834_amd import binding
    w = synth.Workload(name="gains", S=S, SB=SB, sample_type=synth.CI16, x_mode=mode, N=64 * n_c,
                       fp16_prescale_log2=-1 if mode == synth.X_FP16_SPLIT else 0)
    return w, binding.plan_for(w)


def _rand(rng, shape, scale=1.0):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * scale).astype(np.complex64)


def _gains(rng, shape):
    return (rng.uniform(0.5, 1.5, shape) * np.exp(1j * rng.uniform(-np.pi, np.pi, shape))).astype(np.complex64)


@pytest.mark.parametrize("S,SB", [(1, 1), (5, 2), (48, 1), (80, 1), (48, 16)])
def test_apply_and_adjoint_match_oracle(S, SB):
    _say(f"CASE gains S={S} SB={SB}")
    rng = np.random.default_rng(S * 10 + SB)
    w, plan = _plan(S, SB)
    with plan:
        B = S * (S + 1) // 2
        V0 = _rand(rng, (SB, 64, B, 4), 100.0)
        g = _gains(rng, (SB, 64, 2 * S))
        G = _rand(rng, (SB, 64, B, 4), 3.0)
        Vd = plan.apply_gains(torch.from_numpy(V0).cuda(), torch.from_numpy(g).cuda())
        gd = plan.apply_gains_adjoint(torch.from_numpy(V0).cuda(), torch.from_numpy(g).cuda(), torch.from_numpy(G).cuda())
        torch.cuda.synchronize()
        ref_v = og.apply_gains(V0.astype(np.complex128), g.astype(np.complex128), S)
        ref_g = og.apply_gains_adjoint(V0.astype(np.complex128), g.astype(np.complex128), G.astype(np.complex128), S)
        ev = np.abs(Vd.cpu().numpy() - ref_v).max() / np.abs(ref_v).max()
        eg = np.abs(gd.cpu().numpy() - ref_g).max() / np.abs(ref_g).max()
        _say(f"  forward rel {ev:.2e}  adjoint rel {eg:.2e}")
        assert ev <= 2e-6 and eg <= 2e-6


def test_autograd_through_correlator_matches_oracle_and_finite_differences():
    """Gains applied to correlator output of a real 16-bit block: loss sum |V' - M|^2 against
    a seeded model; torch autograd (HIP adjoint) vs the FP64 oracle gradient, and central
    finite differences of the GPU forward for a few gain components."""
    from paper_1801_04834_amd.autograd import gain_correlate
    S, SB, n_c = 48, 1, 256
    _say(f"CASE autograd S={S} SB={SB} n_c={n_c}")
    rng = np.random.default_rng(1804)
    w, plan = _plan(S, SB, n_c=n_c)
    w.sigma, w.seed = 64.0, 1804
    with plan:
        x = torch.from_numpy(w.block(0)).cuda()
        V0 = torch.view_as_complex(plan.correlate(x, w.delays(0)))
        g_true = _gains(rng, (SB, 64, 2 * S))
        V0n = V0.cpu().numpy().astype(np.complex128)
        Mdl = og.apply_gains(V0n, g_true.astype(np.complex128), S)
        Mdl = Mdl + 0.05 * np.abs(Mdl).mean() * (rng.standard_normal(Mdl.shape) + 1j * rng.standard_normal(Mdl.shape))
        g0 = _gains(rng, (SB, 64, 2 * S))
        gt = torch.from_numpy(g0).cuda().requires_grad_(True)
        Vp = gain_correlate(plan, V0, gt)
        Mt = torch.from_numpy(Mdl.astype(np.complex64)).cuda()
        loss = torch.sum(torch.abs(Vp.to(torch.complex128) - Mt.to(torch.complex128)) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        got = gt.grad.cpu().numpy()
        _, G = og.model_loss(V0n, g0.astype(np.complex128), Mdl.astype(np.complex64).astype(np.complex128), S)
        ref = og.apply_gains_adjoint(V0n, g0.astype(np.complex128), G, S)
        rel = np.abs(got - ref).max() / np.abs(ref).max()
        _say(f"  autograd vs oracle rel {rel:.2e}")
        assert rel <= 2e-5

        # central finite differences of the GPU forward (loss summed in FP64 on the device)
        def L(gn):
            v = plan.apply_gains(V0, torch.from_numpy(gn).cuda())
            return float(torch.sum(torch.abs(v.to(torch.complex128) - Mt.to(torch.complex128)) ** 2))

        # the loss is a polynomial of degree 4 in (Re g_k, Im g_k), so the five-point
        # stencil is exact up to rounding of the FP32 forward
        for _ in range(6):
            idx = (0, int(rng.integers(64)), int(rng.integers(2 * S)))
            for comp, unit in ((0, 1.0), (1, 1j)):
                h = 0.05
                vals = []
                for m in (2, 1, -1, -2):
                    gg = g0.copy()
                    gg[idx] += np.complex64(m * h * unit)
                    vals.append(L(gg))
                fd = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
                an = got[idx].real if comp == 0 else got[idx].imag
                _say(f"  fd {idx} {comp}: {fd:.6e} vs {an:.6e}")
                assert abs(fd - an) <= 2e-3 * max(abs(an), 1e-3 * np.abs(got).max())


def test_int8_plan_rejects_gains():
    from paper_1801_04834_amd import binding
    w, plan = _plan(2, 1, mode=synth.X_INT8)
    with plan:
        v = torch.zeros((1, 64, 3, 4), dtype=torch.complex64, device="cuda")
        g = torch.ones((1, 64, 4), dtype=torch.complex64, device="cuda")
        with pytest.raises(binding.CobaltError) as ei:
            plan.apply_gains(v, g)
        assert ei.value.code == binding.EUNSUPPORTED


def test_differentiable_workload_end_to_end_at_full_size():
    """The differentiable workload end to end: 48 stations x 2 pol, 16 subbands x 64 channels,
    196 608 samples of ci16 (3072 channel samples), FP16-split correlator on the GPU, gains with
    |g| ~ U(0.5, 1.5) and uniform phase, loss sum |V' - M|^2 against a seeded model (the oracle's
    gained visibilities plus 5 % noise), gradient through torch autograd (HIP adjoint).  Against
    the oracle run of the whole chain (FP64 FX, gains, loss, adjoint): the loss within 1e-5 and
    the gradient within 1e-4 of its largest magnitude (the GPU's visibilities carry the 16-bit
    mode's ~1e-6 relative error into both); central finite differences of the GPU forward on a
    few gain components."""
    from paper_1801_04834_amd import binding
    from paper_1801_04834_amd.autograd import gain_correlate
    w = synth.Workload(name="gains_full", S=48, SB=16, sample_type=synth.CI16, x_mode=synth.X_FP16_SPLIT,
                       sigma=64.0, seed=1804, delay_spread_s=5e-6, delay_drift_s=25e-9, ripple=0.05,
                       fp16_prescale_log2=-1)
    _say(f"CASE gains end to end S={w.S} SB={w.SB} N={w.N}")
    x = w.block(0)
    ref = oracle.fx_block(synth.to_complex(x), np.zeros((w.S, 2, w.SB, 960), np.complex128), w.fir(), w.bandpass(),
                          w.subband_freqs(), synth.SAMPLE_RATE_HZ, w.delays(0), 64, 16, mode="fp16_split",
                          return_channelised=False)
    V0ref = ref["V"]                                                # [SB, C, B, 4]
    rng = np.random.default_rng(1804)
    shape = (w.SB, 64, 2 * w.S)
    g_true = _gains(rng, shape).astype(np.complex128)
    Mdl = og.apply_gains(V0ref, g_true, w.S)
    Mdl = Mdl + 0.05 * np.abs(Mdl).mean() * (rng.standard_normal(Mdl.shape) + 1j * rng.standard_normal(Mdl.shape))
    Mdl = Mdl.astype(np.complex64)
    g0 = _gains(rng, shape)
    L_ref, G_ref = og.model_loss(V0ref, g0.astype(np.complex128), Mdl.astype(np.complex128), w.S)
    grad_ref = og.apply_gains_adjoint(V0ref, g0.astype(np.complex128), G_ref, w.S)
    with binding.plan_for(w) as plan:
        V0 = torch.view_as_complex(plan.correlate(torch.from_numpy(x).cuda(), w.delays(0)))
        Mt = torch.from_numpy(Mdl).cuda()
        gt = torch.from_numpy(g0).cuda().requires_grad_(True)
        Vp = gain_correlate(plan, V0, gt)
        loss = torch.sum(torch.abs(Vp.to(torch.complex128) - Mt.to(torch.complex128)) ** 2)
        loss.backward()
        torch.cuda.synchronize()
        got = gt.grad.cpu().numpy()
        rl = abs(float(loss) - L_ref) / L_ref
        rg = np.abs(got - grad_ref).max() / np.abs(grad_ref).max()
        _say(f"  loss {float(loss):.6e} vs oracle {L_ref:.6e} (rel {rl:.2e}); gradient rel {rg:.2e}")
        assert rl <= 1e-5 and rg <= 1e-4

        def L(gn):
            v = plan.apply_gains(V0, torch.from_numpy(gn).cuda())
            return float(torch.sum(torch.abs(v.to(torch.complex128) - Mt.to(torch.complex128)) ** 2))

        for _ in range(4):
            idx = (int(rng.integers(w.SB)), int(rng.integers(64)), int(rng.integers(2 * w.S)))
            for comp, unit in ((0, 1.0), (1, 1j)):
                h = 0.05
                vals = []
                for m in (2, 1, -1, -2):
                    gg = g0.copy()
                    gg[idx] += np.complex64(m * h * unit)
                    vals.append(L(gg))
                fd = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
                an = got[idx].real if comp == 0 else got[idx].imag
                _say(f"  fd {idx} {comp}: {fd:.6e} vs {an:.6e}")
                assert abs(fd - an) <= 2e-3 * max(abs(an), 1e-3 * np.abs(got).max())
