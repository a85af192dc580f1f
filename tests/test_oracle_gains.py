"""Pins of the gain-applied correlator reference and its adjoint (no GPU).

* gains applied to the channelised samples before the X stage give the same visibilities
  as ``apply_gains`` on the ungained ones (the definition vs the factorised form);
* the adjoint equals FP64 central finite differences of the loss, component by component;
* the adjoint equals torch autograd (CPU, complex128) of the definition written in torch ops;
* unit gains are the identity; pure phases rotate each baseline by the phase difference.
"""

import numpy as np
import pytest

import oracle
from oracle import gains as og


def _setup(seed=1, S=4, n_chan=3, n_c=20):
    rng = np.random.default_rng(seed)
    M = 2 * S
    Z = rng.standard_normal((n_chan, M, n_c)) + 1j * rng.standard_normal((n_chan, M, n_c))
    V0 = oracle.correlate(Z, S)
    g = rng.uniform(0.5, 1.5, (n_chan, M)) * np.exp(1j * rng.uniform(-np.pi, np.pi, (n_chan, M)))
    return rng, Z, V0, g


def test_gains_before_x_equal_factorised_form():
    rng, Z, V0, g = _setup()
    direct = oracle.correlate(g[:, :, None] * Z, 4)
    np.testing.assert_allclose(og.apply_gains(V0, g, 4), direct, rtol=0, atol=1e-12 * np.abs(direct).max())


def test_unit_and_phase_gains():
    rng, Z, V0, g = _setup(2)
    np.testing.assert_array_equal(og.apply_gains(V0, np.ones_like(g), 4), V0)
    phi = rng.uniform(-np.pi, np.pi, g.shape)
    Vp = og.apply_gains(V0, np.exp(1j * phi), 4)
    for s1 in range(4):
        for s2 in range(s1 + 1):
            bl = oracle.baseline_index(s1, s2)
            for p1 in range(2):
                for p2 in range(2):
                    rot = np.exp(1j * (phi[:, 2 * s1 + p1] - phi[:, 2 * s2 + p2]))
                    np.testing.assert_allclose(Vp[:, bl, 2 * p1 + p2], rot * V0[:, bl, 2 * p1 + p2], rtol=1e-13)


@pytest.mark.parametrize("seed", [3, 4])
def test_adjoint_matches_central_finite_differences(seed):
    rng, Z, V0, g = _setup(seed, S=3, n_chan=2, n_c=10)
    Mdl = og.apply_gains(V0, g * (1 + 0.1 * rng.standard_normal(g.shape)), 3) + rng.standard_normal(V0.shape)
    L, G = og.model_loss(V0, g, Mdl, 3)
    grad = og.apply_gains_adjoint(V0, g, G, 3)
    h = 1e-6
    for idx in np.ndindex(g.shape):
        for comp, unit in ((0, 1.0), (1, 1j)):
            gp, gm = g.copy(), g.copy()
            gp[idx] += h * unit
            gm[idx] -= h * unit
            fd = (og.model_loss(V0, gp, Mdl, 3)[0] - og.model_loss(V0, gm, Mdl, 3)[0]) / (2 * h)
            an = grad[idx].real if comp == 0 else grad[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (idx, comp, fd, an)


def test_adjoint_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng, Z, V0, g = _setup(5, S=3, n_chan=2, n_c=12)
    Mdl = rng.standard_normal(V0.shape) + 1j * rng.standard_normal(V0.shape)
    ent = og._entries(3)
    gt = torch.tensor(g, dtype=torch.complex128, requires_grad=True)
    V0t = torch.tensor(V0, dtype=torch.complex128)
    Mt = torch.tensor(Mdl, dtype=torch.complex128)
    loss = 0
    for bl, q, a, b in ent:
        v = gt[:, a] * torch.conj(gt[:, b]) * V0t[:, bl, q]
        loss = loss + torch.sum(torch.abs(v - Mt[:, bl, q]) ** 2)
    loss.backward()
    _, G = og.model_loss(V0, g, Mdl, 3)
    ours = og.apply_gains_adjoint(V0, g, G, 3)
    np.testing.assert_allclose(gt.grad.numpy(), ours, rtol=1e-12, atol=1e-12 * np.abs(ours).max())
