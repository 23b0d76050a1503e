"""The selector network's HIP kernels against the float64 reference, and a
small end-to-end training run showing what the learned choice gains over the
fixed 12/16/24/32 setting (measured sizes and GPU decode times)."""
import numpy as np
import pytest

from oracle import mlp_ref
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(B, seed):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.15, mlp_ref.N_PARAMS).astype(np.float32)
    x = rng.normal(0, 1, (B, 64)).astype(np.float32)
    y = rng.integers(0, 16, B).astype(np.int32)
    return theta, x, y


@pytest.mark.parametrize("B", [1, 7, 256, 300])
def test_forward_backward_adam_match_reference(B):
    _dev()
    theta, x, y = _setup(B, B)
    P = torch.from_numpy(theta).cuda()
    X = torch.from_numpy(x).cuda()
    Y = torch.from_numpy(y).cuda()
    h1 = torch.empty(B, 128, device="cuda")
    h2 = torch.empty(B, 128, device="cuda")
    lg = torch.empty(B, 16, device="cuda")
    lz.mlp_forward(P, X, h1, h2, lg)
    r1, r2, rl = mlp_ref.forward(theta.astype(np.float64), x.astype(np.float64))
    assert np.allclose(lg.cpu().numpy(), rl, rtol=1e-4, atol=1e-5)
    assert np.allclose(h2.cpu().numpy(), r2, rtol=1e-4, atol=1e-5)
    g = torch.zeros(P.numel(), device="cuda")
    work = torch.empty(B * 272, device="cuda")
    loss = torch.zeros(1, device="cuda")
    lz.mlp_backward(P, X, h1, h2, lg, Y, g, work, loss)
    rg = mlp_ref.grad(theta.astype(np.float64), x.astype(np.float64), y)
    gg = g.cpu().numpy()
    scale = np.abs(rg).max()
    assert np.abs(gg - rg).max() <= 1e-4 * scale + 1e-7
    assert abs(loss.item() - mlp_ref.loss(theta.astype(np.float64), x.astype(np.float64), y)) < 1e-4
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    lz.mlp_adam(P, g, m, v, 1, lr=1e-3)
    rt, rm, rv = mlp_ref.adam(theta.astype(np.float64), gg.astype(np.float64), np.zeros(theta.size),
                              np.zeros(theta.size), 1)
    assert np.allclose(P.cpu().numpy(), rt, rtol=1e-6, atol=1e-7)


def test_selector_training_step_matches_reference():
    """lz_selector_train over one epoch whose single batch holds every row is
    one Adam step on the mean gradient of the normalised rows: equal to the
    float64 reference of the same step."""
    _dev()
    rng = np.random.default_rng(11)
    B = 200
    F = rng.uniform(0, 0.3, (B, 64)).astype(np.float32)
    y = rng.integers(0, 16, B).astype(np.int32)
    tuples = np.tile(np.array([12, 16, 24, 32], np.uint32), (16, 1))
    sel = lz.Selector(tuples, 1, 4)
    sel.set_norm(F)
    theta = sel.params().astype(np.float64)
    inf = sel.info()
    x = (F.astype(np.float64) - inf["mu"]) / inf["sd"]
    hist = sel.train(F, y, epochs=1, batch=256, lr=1e-3, seed=9)
    assert abs(hist[0] - mlp_ref.loss(theta, x, y)) < 1e-4
    g = mlp_ref.grad(theta, x, y)
    want, _, _ = mlp_ref.adam(theta, g, np.zeros(theta.size), np.zeros(theta.size), 1)
    got = sel.params().astype(np.float64)
    # Adam's first step moves every weight by lr * sign(g) where |g| >> eps
    big = np.abs(g) > 1e-5
    assert np.allclose(got[big], want[big], rtol=1e-5, atol=1e-7)
    assert np.abs(got - want).max() <= 1.01e-3


def test_learned_selector_end_to_end():
    """Train on measurements of generated files, calibrate the fallback, then
    encode held-out files in learned mode and compare, measured end to end
    (entropy-bound size and GPU decode time), with the fixed 12/16/24/32
    encode: the learned choice must cost less (J below 2 by a margin)."""
    _dev()
    from paper_2607_18541_amd import learn
    res, sel = learn.run(n_files=60, blocks_per_file=16, log2_bs=14, epochs=40, seed=3)
    info = {k: res[k] for k in ("loss_first", "loss_last", "val_accuracy", "test_mean_J", "fixed_J", "test_gain",
                                "test_size_ratio", "test_time_ratio", "test_non_fixed_blocks")}
    print("learned selector:", info, flush=True)
    assert res["loss_last"] < res["loss_first"]
    assert res["test_gain"] > 0.05, info
