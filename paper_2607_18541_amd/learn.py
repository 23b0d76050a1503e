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
(time = a * tokens + c * matches + d * match bytes + (e * depths + f) / blocks).

The arithmetic runs in liblz: the parses (lz_encode), features and block
statistics, the time model, J and labels (lz_learn_labels), the feature
normalisation, training (lz_selector_train: the network's forward, backward
and Adam kernels on the GPU), the fallback table (lz_selector_calibrate),
inference with the fallback rule (lz_selector_choose) and the learned encode
(lz_encode_learned).  This file generates the inputs, times GPU decodes with
events and passes arrays between those calls.
"""
import argparse
import json
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
    """Mean GPU decode time (events on the launching stream) and depth count."""
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
    """Features, per-(block, tuple) sizes and counts, whole-file decode times
    and depths; the time model, J and labels come from lz_learn_labels."""
    feats, sizes, counts, blocks = [], [], [], []
    file_ms = np.zeros((len(files), len(TUPLES)))
    file_depths = np.zeros((len(files), len(TUPLES)), np.uint32)
    for fi, x in enumerate(files):
        cheap = lz.encode(x, log2_bs, CHEAP, max_chain=16, depth_passes=0)
        F = lz.block_features(cheap)
        S = np.zeros((F.shape[0], len(TUPLES)))
        C = np.zeros((F.shape[0], len(TUPLES), 3), np.uint64)
        for t, thr in enumerate(TUPLES):
            arc = lz.encode(x, log2_bs, thr)
            ent, nt, nm, mb = lz.block_stats(arc)
            S[:, t] = ent
            C[:, t, 0], C[:, t, 1], C[:, t, 2] = nt, nm, mb
            file_ms[fi, t], file_depths[fi, t] = decode_ms(arc, torch)
        feats.append(F)
        sizes.append(S)
        counts.append(C)
        blocks.append(F.shape[0])
        if (fi + 1) % 10 == 0 or fi + 1 == len(files):
            log("measured %d/%d files" % (fi + 1, len(files)))
    coef, J, labels = lz.learn_labels(blocks, np.concatenate(sizes), np.concatenate(counts), file_ms, file_depths,
                                      lam, FIXED)
    cut = np.cumsum([0] + blocks)
    return {"feats": feats, "J": [J[a:b] for a, b in zip(cut[:-1], cut[1:])],
            "labels": [labels[a:b] for a, b in zip(cut[:-1], cut[1:])], "time_model": coef.tolist()}


def evaluate(files, sel, log2_bs, torch, lam=1.0):
    """Held-out comparison, measured end to end: entropy-bound size and GPU
    decode time of the learned archive against the fixed 12/16/24/32 one."""
    rows = []
    for x in files:
        arc_l, k = lz.encode_learned(x, sel, log2_bs)
        arc_f = lz.encode(x, log2_bs, TUPLES[FIXED])
        sl, _ = lz.entropy_size(arc_l)
        sf, _ = lz.entropy_size(arc_f)
        tl, _ = decode_ms(arc_l, torch, reps=10)
        tf, _ = decode_ms(arc_f, torch, reps=10)
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
    """Generate, measure, train (80 % of the files), calibrate the fallback on
    10 %, and evaluate the learned encoder end to end on the last 10 %."""
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
    sel = lz.Selector(TUPLES, FIXED, seed)
    sel.set_norm(F_tr)
    hist = sel.train(F_tr, y_tr, epochs=epochs, seed=seed)
    log("trained: loss %.4f -> %.4f" % (hist[0], hist[-1]))
    # validation J per predicted tuple: the fallback rule's table
    F_va = np.concatenate(M["feats"][n_tr:n_tr + n_va])
    J_va = np.concatenate(M["J"][n_tr:n_tr + n_va])
    sel.calibrate(F_va, J_va, lam)
    pred, _ = sel.choose(F_va)
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
    ap.add_argument("--out", default=None, help="selector file to write (lz_selector_save format)")
    a = ap.parse_args()
    r, _ = run(a.files, a.blocks, a.log2_bs, a.epochs, out=a.out)
    print(json.dumps({k: v for k, v in r.items() if k != "test_files"}))
