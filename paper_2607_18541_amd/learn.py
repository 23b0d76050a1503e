"""Learned per-block distance-class thresholds.

The paper finds 12/16/24/32 the universal win on its data, with the optimum
data-dependent at the margin (Sec. 4.3: 16/24/32/48 trades ratio for
throughput; Sec. 6).  This module trains a small network on the GPU that
picks, per LZ block, one of 16 candidate threshold tuples from the block's
match-length / distance-class histogram, using labels produced by the method
itself: every training file is encoded under every tuple (sizes) and decoded
on the GPU (times).  It only chooses encoder parameters: decode stays bit-exact
and the ratio is measured, not assumed.  The fixed 12/16/24/32 setting is both
the fallback and the yardstick.

Label of block b: argmin over tuples t of
    J(b, t) = size(b, t) / size(b, fixed) + lam * time(b, t) / time(b, fixed)
size = entropy-bound bytes of the block's streams; time = a per-block decode
time from a linear model fitted to measured whole-file GPU decode times
(time = a * tokens + c * matches + d * match bytes + e * levels / blocks).

Everything numeric runs in liblz: the parse (lz_encode), features and block
statistics (host C++), the decoder, and the network's forward, backward and
Adam kernels (HIP).  This file only orchestrates.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import lz

TUPLES = [
    (6, 8, 10, 12), (12, 16, 24, 32), (16, 24, 32, 48), (4, 6, 8, 10),
    (8, 10, 12, 16), (8, 12, 16, 20), (10, 12, 16, 24), (12, 16, 20, 24),
    (16, 20, 24, 32), (20, 24, 32, 48), (24, 32, 48, 64), (6, 8, 12, 16),
    (6, 10, 16, 24), (8, 12, 20, 32), (10, 16, 24, 48), (12, 20, 32, 64),
]
FIXED = 1  # index of 12/16/24/32
CHEAP = (4, 4, 4, 4)


def log(msg):
    print("[learn] " + msg, file=sys.stderr, flush=True)


def make_files(count, blocks_per_file, log2_bs, seed, torch):
    """Seeded training files: Zipf text (s in [0.8, 1.4]), FASTQ-like reads
    (substitution rate in [0.2%, 3%]) and generated streams (mean match length
    log-uniform in [8, 512]); the stream bytes come from decoding the token
    list with the GPU decoder."""
    import synth
    n = blocks_per_file << log2_bs
    u = synth.uniform(3 * count, seed)
    files = []
    for i in range(count):
        kind = i % 3
        if kind == 0:
            x = synth.zipf_text(n, seed=seed * 7919 + i, s=0.8 + 0.6 * u[3 * i])
        elif kind == 1:
            x = synth.fastq(n, seed=seed * 7919 + i, sub_rate=0.002 + 0.028 * u[3 * i + 1])
            if x.size < (n >> 1):
                x = synth.fastq(n, seed=seed * 7919 + i)
        else:
            m = float(np.exp(np.log(8) + (np.log(512) - np.log(8)) * u[3 * i + 2]))
            ll, ml, sr, lit = synth.geo_tokens(n, m, seed=seed * 7919 + i, lit_prefix=min(4096, n), min_back=1)
            da = lz.DeviceArchive(lz.build_archive(n, log2_bs, ll, ml, sr, lit))
            x = da.decode().cpu().numpy().copy()
            da.close()
        files.append(np.ascontiguousarray(x))
    return files


def decode_ms(arc, torch, reps=3):
    da = lz.DeviceArchive(arc)
    out = torch.empty(max(da.n, 1), dtype=torch.uint8, device="cuda")
    da.decode(out)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        da.decode_async(out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    lv = da.levels
    da.close()
    return ms, lv


def measure(files, log2_bs, torch, lam=1.0):
    """Features, per-(block, tuple) sizes and modelled times, and labels."""
    feats, sizes, counts, file_ms, file_rows = [], [], [], [], []
    for fi, x in enumerate(files):
        cheap = lz.encode(x, log2_bs, CHEAP, max_chain=16)
        F = lz.block_features(cheap)
        S = np.zeros((F.shape[0], len(TUPLES)))
        C = np.zeros((F.shape[0], len(TUPLES), 3))
        for t, thr in enumerate(TUPLES):
            arc = lz.encode(x, log2_bs, thr)
            ent, nt, nm, mb = lz.block_stats(arc)
            S[:, t] = ent
            C[:, t, 0], C[:, t, 1], C[:, t, 2] = nt, nm, mb
            ms, lv = decode_ms(arc, torch)
            file_ms.append(ms)
            file_rows.append([nt.sum(), nm.sum(), mb.sum(), lv, 1.0])
        feats.append(F)
        sizes.append(S)
        counts.append(C)
        if (fi + 1) % 10 == 0 or fi + 1 == len(files):
            log("measured %d/%d files" % (fi + 1, len(files)))
    # time model fitted to whole-file decode times
    A = np.array(file_rows, dtype=np.float64)
    y = np.array(file_ms, dtype=np.float64)
    coef, *_ = np.linalg.lstsq(A, y, rcond=None)
    coef = np.maximum(coef, 0.0)
    times = []
    for fi, C in enumerate(counts):
        nb = C.shape[0]
        lv = np.array([file_rows[fi * len(TUPLES) + t][3] for t in range(len(TUPLES))])
        T = coef[0] * C[:, :, 0] + coef[1] * C[:, :, 1] + coef[2] * C[:, :, 2] + (coef[3] * lv + coef[4])[None, :] / nb
        times.append(np.maximum(T, 1e-9))
    labels, J = [], []
    for S, T in zip(sizes, times):
        j = S / S[:, FIXED:FIXED + 1] + lam * T / T[:, FIXED:FIXED + 1]
        J.append(j)
        labels.append(np.argmin(j, axis=1))
    return {"feats": feats, "sizes": sizes, "times": times, "J": J, "labels": labels, "time_model": coef.tolist()}


class Selector:
    """Network parameters (device), feature normalisation and per-tuple mean
    validation J; picks a tuple per block or falls back to 12/16/24/32."""

    def __init__(self, torch, seed=1):
        import synth
        self.torch = torch
        npar = int(lz.lib().lz_mlp_param_count())
        theta = np.zeros(npar, dtype=np.float32)
        o = 0
        for fan_in, shape in ((64, (64, 128)), (0, (128,)), (128, (128, 128)), (0, (128,)), (128, (128, 16)),
                              (0, (16,))):
            k = int(np.prod(shape))
            if fan_in:
                theta[o:o + k] = synth.normal(k, seed + o) * np.sqrt(2.0 / fan_in)
            o += k
        self.params = torch.from_numpy(theta).cuda()
        self.mu = np.zeros(64, np.float32)
        self.sd = np.ones(64, np.float32)
        self.val_J = np.ones(len(TUPLES))

    def _norm(self, F):
        return self.torch.from_numpy(((F - self.mu) / self.sd).astype(np.float32)).cuda()

    def forward(self, F):
        torch = self.torch
        x = self._norm(F)
        B = x.shape[0]
        h1 = torch.empty(B, 128, device="cuda")
        h2 = torch.empty(B, 128, device="cuda")
        lg = torch.empty(B, 16, device="cuda")
        lz.mlp_forward(self.params, x, h1, h2, lg)
        return lg

    def choose(self, F):
        """Tuple index per block, with the fallback: 12/16/24/32 when the top
        probability is below 0.5 or the tuple's validation J is not below 1."""
        lg = self.forward(F).cpu().numpy().astype(np.float64)
        p = np.exp(lg - lg.max(axis=1, keepdims=True))
        p /= p.sum(axis=1, keepdims=True)
        k = p.argmax(axis=1)
        ok = (p.max(axis=1) >= 0.5) & (self.val_J[k] < 1.0)
        return np.where(ok, k, FIXED)

    def train(self, F, y, epochs=50, batch=256, lr=1e-3, seed=0):
        torch = self.torch
        self.mu = F.mean(axis=0).astype(np.float32)
        self.sd = (F.std(axis=0) + 1e-6).astype(np.float32)
        X = self._norm(F)
        Y = torch.from_numpy(y.astype(np.int32)).cuda()
        n = X.shape[0]
        npar = self.params.numel()
        grads = torch.zeros(npar, device="cuda")
        m = torch.zeros(npar, device="cuda")
        v = torch.zeros(npar, device="cuda")
        h1 = torch.empty(batch, 128, device="cuda")
        h2 = torch.empty(batch, 128, device="cuda")
        lg = torch.empty(batch, 16, device="cuda")
        work = torch.empty(batch * 272, device="cuda")
        loss = torch.zeros(1, device="cuda")
        rng = np.random.default_rng(seed)
        step = 0
        hist = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            loss.zero_()
            nb = 0
            for s0 in range(0, n, batch):
                idx = perm[s0:s0 + batch]
                xb = X[idx].contiguous()
                yb = Y[idx].contiguous()
                B = xb.shape[0]
                lz.mlp_forward(self.params, xb, h1[:B], h2[:B], lg[:B])
                lz.mlp_backward(self.params, xb, h1[:B], h2[:B], lg[:B], yb, grads, work, loss)
                step += 1
                lz.mlp_adam(self.params, grads, m, v, step, lr=lr)
                nb += 1
            hist.append(float(loss.item()) / max(nb, 1))
        return hist

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu, sd=self.sd, val_J=self.val_J)

    def load(self, path):
        d = np.load(path, allow_pickle=False)
        self.params = self.torch.from_numpy(d["params"]).cuda()
        self.mu, self.sd, self.val_J = d["mu"], d["sd"], d["val_J"]


def encode_learned(x, sel, log2_bs=16):
    """Encodes x with the tuple the selector picks for each block (tuple ids
    are stored in the archive's per-block info bytes)."""
    cheap = lz.encode(x, log2_bs, CHEAP, max_chain=16)
    k = sel.choose(lz.block_features(cheap))
    thr = np.array([TUPLES[i] for i in k], dtype=np.uint32)
    return lz.encode_blockwise(x, thr, k.astype(np.uint8), log2_bs=log2_bs), k


def evaluate(files, sel, log2_bs, torch, lam=1.0):
    """Held-out comparison, measured end to end: entropy-bound size and GPU
    decode time of the learned archive against the fixed 12/16/24/32 one."""
    rows = []
    for x in files:
        arc_l, k = encode_learned(x, sel, log2_bs)
        arc_f = lz.encode(x, log2_bs, TUPLES[FIXED])
        sl, _ = lz.entropy_size(arc_l)
        sf, _ = lz.entropy_size(arc_f)
        tl, _ = decode_ms(arc_l, torch)
        tf, _ = decode_ms(arc_f, torch)
        da = lz.DeviceArchive(arc_l)
        assert np.array_equal(da.decode().cpu().numpy(), x)  # decode stays bit-exact
        da.close()
        rows.append({"size_learned": sl, "size_fixed": sf, "ms_learned": tl, "ms_fixed": tf,
                     "J": sl / sf + lam * tl / tf, "non_fixed_blocks": float(np.mean(k != FIXED))})
    J = float(np.mean([r["J"] for r in rows]))
    return {"mean_J": J, "gain_vs_fixed": (1.0 + lam) - J, "files": rows,
            "size_ratio": float(np.mean([r["size_learned"] / r["size_fixed"] for r in rows])),
            "time_ratio": float(np.mean([r["ms_learned"] / r["ms_fixed"] for r in rows])),
            "non_fixed_blocks": float(np.mean([r["non_fixed_blocks"] for r in rows]))}


def run(n_files=100, blocks_per_file=100, log2_bs=16, epochs=50, seed=5, lam=1.0, out=None):
    import torch
    t0 = time.time()
    files = make_files(n_files, blocks_per_file, log2_bs, seed, torch)
    log("generated %d files in %.1fs" % (len(files), time.time() - t0))
    n_tr = int(0.8 * n_files)
    n_va = int(0.1 * n_files)
    M = measure(files, log2_bs, torch, lam)
    log("measured in %.1fs; time model %s" % (time.time() - t0, M["time_model"]))
    F_tr = np.concatenate(M["feats"][:n_tr])
    y_tr = np.concatenate(M["labels"][:n_tr])
    sel = Selector(torch, seed)
    hist = sel.train(F_tr, y_tr, epochs=epochs)
    log("trained: loss %.4f -> %.4f" % (hist[0], hist[-1]))
    # validation J per predicted tuple (for the fallback rule)
    F_va = np.concatenate(M["feats"][n_tr:n_tr + n_va])
    J_va = np.concatenate(M["J"][n_tr:n_tr + n_va])
    sel.val_J = np.ones(len(TUPLES)) * 9.0
    pred = sel.forward(F_va).cpu().numpy().argmax(axis=1)
    for t in range(len(TUPLES)):
        if np.any(pred == t):
            sel.val_J[t] = float(J_va[pred == t, t].mean()) / (1.0 + lam)
    sel.val_J[FIXED] = 1.0
    acc = float(np.mean(pred == np.concatenate(M["labels"][n_tr:n_tr + n_va])))
    ev = evaluate(files[n_tr + n_va:], sel, log2_bs, torch, lam)
    res = {"files": n_files, "blocks_per_file": blocks_per_file, "log2_bs": log2_bs, "epochs": epochs,
           "loss_first": hist[0], "loss_last": hist[-1], "val_accuracy": acc, "test_mean_J": ev["mean_J"],
           "fixed_J": 1.0 + lam, "test_gain": ev["gain_vs_fixed"], "test_size_ratio": ev["size_ratio"],
           "test_time_ratio": ev["time_ratio"], "test_non_fixed_blocks": ev["non_fixed_blocks"],
           "time_model": M["time_model"],
           "label_hist": np.bincount(np.concatenate(M["labels"]), minlength=16).tolist(),
           "test_files": ev["files"], "seconds": time.time() - t0}
    if out:
        sel.save(out)
    return res, sel


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--files", type=int, default=100)
    ap.add_argument("--blocks", type=int, default=100)
    ap.add_argument("--log2-bs", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=50)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    r, _ = run(a.files, a.blocks, a.log2_bs, a.epochs, out=a.out)
    print(json.dumps({k: v for k, v in r.items() if k != "test_files"}))
