"""The allocation-free backward entry point (lz_mlp_backward_noalloc) against
the entry point that takes a work buffer (lz_mlp_backward): two calls in a
row, the second with a smaller batch, each compared element by element with
the buffered call on the same inputs and with the float64 reference."""
import numpy as np
import pytest

from oracle import mlp_ref
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(B, seed):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.15, mlp_ref.N_PARAMS).astype(np.float32)
    x = rng.normal(0, 1, (B, 64)).astype(np.float32)
    y = rng.integers(0, 16, B).astype(np.int32)
    return theta, x, y


def test_backward_noalloc_equals_buffered_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for B, seed in ((4096, 1), (300, 2)):
        print("noalloc backward: batch %d seed %d" % (B, seed), flush=True)
        theta, x, y = _case(B, seed)
        P, X, Y = (torch.from_numpy(a).cuda() for a in (theta, x, y))
        h1 = torch.empty(B, 128, device="cuda")
        h2 = torch.empty(B, 128, device="cuda")
        lg = torch.empty(B, 16, device="cuda")
        lz.mlp_forward(P, X, h1, h2, lg)
        g_buf = torch.zeros(P.numel(), device="cuda")
        loss_buf = torch.zeros(1, device="cuda")
        work = torch.empty(B * 272, device="cuda")
        lz.mlp_backward(P, X, h1, h2, lg, Y, g_buf, work, loss_buf)
        g_na = torch.full((P.numel(),), float("nan"), device="cuda")
        loss_na = torch.zeros(1, device="cuda")
        lz.mlp_backward_noalloc(P, X, h1, h2, lg, Y, g_na, loss_na)
        torch.cuda.synchronize()
        gb, gn = g_buf.cpu().numpy(), g_na.cpu().numpy()
        assert np.isfinite(gn).all()
        # the same kernels on the same inputs: equal gradients; the loss is
        # an atomic sum over rows, equal up to summation order
        assert np.array_equal(gb, gn)
        assert abs(loss_buf.item() - loss_na.item()) <= 1e-6 * max(1.0, abs(loss_buf.item()))
        rg = mlp_ref.grad(theta.astype(np.float64), x.astype(np.float64), y)
        assert np.abs(gn - rg).max() <= 1e-4 * np.abs(rg).max() + 1e-7


def test_backward_noalloc_rejects_batch_over_maximum():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B = 4097
    theta, x, y = _case(B, 3)
    P, X, Y = (torch.from_numpy(a).cuda() for a in (theta, x, y))
    h1 = torch.empty(B, 128, device="cuda")
    h2 = torch.empty(B, 128, device="cuda")
    lg = torch.empty(B, 16, device="cuda")
    g = torch.zeros(P.numel(), device="cuda")
    with pytest.raises(lz.LzError) as e:
        lz.mlp_backward_noalloc(P, X, h1, h2, lg, Y, g)
    assert e.value.rc == lz.LZ_E_INVAL
