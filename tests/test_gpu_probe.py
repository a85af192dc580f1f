"""GPU readiness probes through the C ABI: the plain copy moves every byte, and the MFMA probe
leaves exactly iterations * K in every accumulator element (K = 16 for the FP16 MFMA, 32 for
the int8 one), so its operation count is real work, not an estimate."""

import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode,K", [(1, 16), (2, 32)])
@pytest.mark.parametrize("iters,wgs", [(1, 1), (300, 37)])
def test_mfma_probe_counts_every_product(mode, K, iters, wgs):
    from paper_1801_04834_amd import binding
    _say(f"CASE mfma probe mode={mode} iters={iters} wgs={wgs}")
    sink = torch.full((wgs * 256,), -7.0, dtype=torch.float32, device="cuda")
    ops = binding.mfma_probe(mode, iters, sink)
    torch.cuda.synchronize()
    assert torch.all(sink == float(iters * K))
    assert ops == wgs * 4 * iters * 8 * 2 * 32 * 32 * K


def test_device_copy_moves_every_byte():
    from paper_1801_04834_amd import binding
    _say("CASE device copy")
    src = torch.randint(-2**31, 2**31 - 1, (3 * 2**20 + 4,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    binding.device_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_device_fanout_writes_both_destinations():
    from paper_1801_04834_amd import binding
    _say("CASE device fan-out")
    src = torch.randint(-2**31, 2**31 - 1, (2**20 + 8,), dtype=torch.int32, device="cuda")
    d0, d1 = torch.zeros_like(src), torch.zeros_like(src)
    binding.device_fanout(d0, d1, src)
    torch.cuda.synchronize()
    assert torch.equal(d0, src) and torch.equal(d1, src)
