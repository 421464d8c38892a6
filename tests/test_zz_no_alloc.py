"""GPU test of semipar_mlp_loss_grad_noalloc, the cost model's loss and gradient for
callers that cannot allocate: through the C ABI it must give what
semipar_mlp_loss_grad gives (the same kernels, the same summation order, so the same
bits), on two calls in a row with the second smaller, and reject more samples than its
fixed scratch holds."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1011_4046_amd import semipar
    semipar.lib()
    return semipar


def _case(seed, n):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.25, 5057).astype(np.float32)
    x = rng.normal(1.0, 2.0, (n, 12)).astype(np.float32)
    t = (0.5 * x[:, 0] - 0.2 * x[:, 4] + 0.1 * x[:, 7] ** 2).astype(np.float32)
    return p, x, t


def test_noalloc_loss_grad_equals_allocating_call(S):
    import torch
    print("case: mlp loss/grad without allocation, n = 8192 then 700, vs the allocating call",
          flush=True)
    p, _, _ = _case(3, 1)
    m = S.CostModel(p)
    for n, seed in ((8192, 4), (700, 5)):
        _, x, t = _case(seed, n)
        m.set_norm_from(x)
        want_l, want_g = m.loss_grad(x, t)
        xd = torch.from_numpy(x).cuda()
        td = torch.from_numpy(t).cuda()
        g, l = m.loss_grad_noalloc(xd, td)
        torch.cuda.synchronize()
        got_g, got_l = g.cpu().numpy(), float(l.cpu()[0])
        assert got_g.tobytes() == want_g.tobytes(), n
        assert got_l == want_l, n
        assert np.allclose(got_g, want_g, rtol=1e-6, atol=0), n


def test_noalloc_rejects_more_samples_than_its_scratch(S):
    import torch
    print("case: mlp loss/grad without allocation, n = 8193 rejected", flush=True)
    p, x, t = _case(6, 8193)
    m = S.CostModel(p)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    with pytest.raises(S.SemiparError) as e:
        m.loss_grad_noalloc(xd, td)
    assert e.value.code == -1
    assert "SEMIPAR_MLP_NOALLOC_MAX" in S.last_error()
