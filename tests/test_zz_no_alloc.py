"""The allocation-free metrics entry point (ara_risk_metrics_noalloc) through
the C ABI: two calls in a row, the second on a smaller input, each equal to
ara_risk_metrics on the same device input and to the oracle within 1e-12."""

import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def ara():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1606_04473_amd import ara as mod
    mod.lib()
    return mod


def _ylt(n, seed):
    """Year losses with zeros and ties, like a layer's YLT."""
    rng = np.random.default_rng(seed)
    y = rng.lognormal(12.0, 1.5, size=n)
    y[rng.random(n) < 0.3] = 0.0
    y[rng.integers(0, n, size=max(1, n // 50))] = y[0]
    return y


def test_noalloc_metrics_equal_allocating_call(ara):
    import torch
    cases = ((1_000_000, [0.99, 0.996, 0.5, 0.989999999999], 11), (1_234, [0.99, 1.0 / 3.0], 12))
    for n, probs, seed in cases:
        y = _ylt(n, seed)
        d = torch.from_numpy(y).cuda()
        k = len(probs)
        ref = ara.risk_metrics(d, probs, outputs=torch.empty(1 + 2 * k, dtype=torch.float64, device="cuda"))
        got = torch.full((1 + 2 * k,), math.nan, dtype=torch.float64, device="cuda")
        ara.risk_metrics_noalloc(d, probs, outputs=got)
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (n, g, r)
        mean, pml, tvar = oracle.risk_metrics(y, probs)
        want = np.array([mean, *pml, *tvar])
        assert np.all(np.abs(g - want) <= REL * np.abs(want)), (n, g, want)


def test_noalloc_metrics_limit(ara):
    import torch
    n = (4 << 20) // 4 + 1                       # 4 probabilities x n keys exceed the static scratch
    d = torch.zeros(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    with pytest.raises(ara.AraError) as e:
        ara.risk_metrics_noalloc(d, [0.9, 0.99, 0.996, 0.999], outputs=out)
    assert "UNSUPPORTED" in str(e.value)
    # the mean alone needs no candidate keys: any size
    ara.risk_metrics_noalloc(d, [], outputs=out[:1])
    one = ara.risk_metrics_noalloc(torch.full((3,), 2.0, dtype=torch.float64, device="cuda"), [0.5],
                                   outputs=torch.empty(3, dtype=torch.float64, device="cuda"))
    assert one.cpu().tolist() == [2.0, 2.0, 2.0]
    assert out[0].item() == 0.0
