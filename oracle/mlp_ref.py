"""Float64 reference of the per-block threshold selector -- TEST INFRASTRUCTURE.

Plain numpy restatement of what the GPU kernels compute; only tests, smoke and
the bench's CPU leg use it.

Network: x (64) -> ReLU(x W1 + b1) (128) -> ReLU(h1 W2 + b2) (128) -> h2 W3 + b3
(16 logits), softmax cross-entropy against the best of 16 threshold tuples,
Adam.  Parameters are one flat vector in the order W1 (64x128, row-major),
b1, W2 (128x128), b2, W3 (128x16), b3: 26,896 values.

Features follow the paper's mechanism (Sec. 3.3, Sec. 4.1: throughput follows
the match-length distribution; Sec. 4.3: short far matches cost offset
entropy): for each of the 4 distance classes and 16 length bins, the fraction
of the block's bytes covered by matches of that class and length, taken from a
cheap greedy parse.
"""
import numpy as np

SHAPES = [(64, 128), (128,), (128, 128), (128,), (128, 16), (16,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)
LEN_EDGES = np.array([0, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64, 128, 256, 1024, 4096, 16384], dtype=np.int64)


def unpack(theta):
    out, o = [], 0
    for s in SHAPES:
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def forward(theta, x):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    logits = h2 @ W3 + b3
    return h1, h2, logits


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def loss(theta, x, y):
    """Mean softmax cross-entropy."""
    _, _, logits = forward(theta, x)
    z = logits - logits.max(axis=1, keepdims=True)
    lse = np.log(np.exp(z).sum(axis=1))
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def grad(theta, x, y):
    """Gradient of the mean cross-entropy by the chain rule; the logit
    gradient is (softmax - onehot) / B."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    B = x.shape[0]
    h1, h2, logits = forward(theta, x)
    d3 = softmax(logits)
    d3[np.arange(B), y] -= 1.0
    d3 /= B
    gW3 = h2.T @ d3
    gb3 = d3.sum(axis=0)
    dh2 = (d3 @ W3.T) * (h2 > 0)
    gW2 = h1.T @ dh2
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    gW1 = x.T @ dh1
    gb1 = dh1.sum(axis=0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def block_features(tok, n, log2_bs, bounds):
    """64 features per block from an oracle token table (oracle.tokens)."""
    bs = 1 << log2_bs
    nb = (n + bs - 1) // bs
    f = np.zeros((nb, 4, 16), dtype=np.float64)
    m = tok["mlen"] > 0
    L = tok["mlen"][m].astype(np.int64)
    d = (tok["dst"][m] + tok["lit_len"][m] - tok["src"][m]).astype(np.int64)
    cls = np.where(d < bounds[0], 0, np.where(d < bounds[1], 1, np.where(d < bounds[2], 2, 3)))
    b = np.searchsorted(LEN_EDGES, L, side="right") - 1
    blk = tok["blk"][m].astype(np.int64)
    np.add.at(f, (blk, cls, b), L)
    lens = np.minimum(bs, n - np.arange(nb) * bs).astype(np.float64)
    return (f.reshape(nb, 64) / lens[:, None])
