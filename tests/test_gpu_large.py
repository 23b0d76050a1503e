"""Outputs above 4 GiB: the high byte plane of the sources, the 16-bit high
fields of the device match records and gathers past 2^32 are compared with
the oracle.  A 4.38 GB token stream (geometric match lengths of mean 256,
sources uniform over everything at least 64 KiB back, so most matches past
2^32 read below it) gets a few planted matches: sources whose span straddles
2^32, a period-3 self-overlapping match cut at 2^32, and matches written
above 2^32 whose sources lie inside a literal run there (copied by the parse
from the literal stream, so their records carry high destination bits).  The
whole decode,
ranges around and across 2^32 and a served request are checked byte by byte
and by FNV-1a 64 against the oracle's execution of the same tokens."""
import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B32 = 1 << 32


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _stream():
    n = B32 + (384 << 20)
    ll, ml, sr, lit = synth.geo_tokens(n, 256, seed=41)
    ml = ml.copy()
    sr = sr.copy()
    mstart = np.concatenate([[0], np.cumsum(ll.astype(np.int64) + ml)[:-1]]) + ll
    # sources straddling 2^32, for matches written well above it
    far = np.nonzero((mstart > B32 + (64 << 20)) & (ml >= 32))[0][:16:2]
    for t in far:
        sr[t] = B32 - int(ml[t]) // 2
    # a self-overlapping match (period 3) whose output crosses 2^32
    t = int(np.nonzero(mstart + ml > B32)[0][0])
    if mstart[t] >= B32 - 8:  # make it start below 2^32
        t -= 1
    assert mstart[t] < B32 < mstart[t] + ml[t] or mstart[t] + ml[t] <= B32
    sr[t] = mstart[t] - 3
    per_at = int(mstart[t])
    # literal-sourced matches above 2^32: the next short match after a literal
    # run of 8 bytes or more reads that run's first bytes
    lit_src = []
    runs = np.nonzero((mstart - ll > B32 + (96 << 20)) & (ll >= 8))[0][:8]
    for r in runs:
        run0 = int(mstart[r] - ll[r])
        for t2 in range(int(r) + 2, int(r) + 4000):
            if 1 <= ml[t2] <= ll[r] and t2 not in far:
                sr[t2] = run0
                lit_src.append(t2)
                break
    assert len(lit_src) == 8
    return n, ll, ml, sr, lit, far, per_at, lit_src


def test_decode_above_4gib_matches_oracle():
    dev = _dev()
    n, ll, ml, sr, lit, far, per_at, lit_src = _stream()
    print("building the 4.38 GB stream and its oracle output", flush=True)
    x = oracle.exec_tokens(n, ll, ml, sr, lit)
    arc = lz.build_archive(n, 16, ll, ml, sr, lit)
    assert lz.archive_info(arc)["n"] == n
    assert np.array_equal(oracle.decode(arc), x), "the oracle's reader disagrees with its token execution"
    x_fnv = oracle.fnv1a64(x)
    da = lz.DeviceArchive(arc, device=dev)
    print("device archive: %d depths, %d literal-sourced matches" % (da.levels, da.fused), flush=True)
    assert da.fused >= len(lit_src)
    exp = torch.from_numpy(x).to(dev)
    out = da.decode()
    torch.cuda.synchronize()
    assert torch.equal(out, exp), "whole decode differs from the oracle"
    host = out.cpu().numpy()
    assert lz.fnv1a64(host) == x_fnv
    del host, out
    torch.cuda.empty_cache()
    # ranges around and across 2^32, near the planted matches, and random ones
    rng = np.random.default_rng(42)
    cases = [(B32 - 1, 2), (B32 - 5000, 10000), (B32, 1), (B32 - (1 << 20), 2 << 20), (n - 1, 1), (n - (3 << 20), 3 << 20),
             (per_at - 4, 64), (B32 - 17, 33), (0, 4096)]
    for t in list(far[:4]) + lit_src[:4]:
        a = int(np.concatenate([[0], np.cumsum(ll[:t].astype(np.int64) + ml[:t])])[-1] + ll[t])
        cases.append((a - 10, int(ml[t]) + 20))
    for _ in range(30):
        L = int(np.exp(rng.uniform(np.log(16), np.log(4 << 20))))
        o = int(rng.integers(B32 - (512 << 20), n - L))
        cases.append((o, L))
    for o, L in cases:
        print("range %d +%d" % (o, L), flush=True)
        got = da.decode_range(o, L)
        torch.cuda.synchronize()
        assert torch.equal(got, exp[o:o + L]), (o, L)
    # one request through the server, across 2^32
    srv = lz.Server(da, 6 << 30, slots=4)
    o, L = B32 - (3 << 20), 5 << 20
    rid = srv.submit(o, L)
    for _ in range(100000):
        srv.tick()
        if srv.status(rid)[0] == 2:
            break
    got = srv.result(rid, L)
    assert torch.equal(got, exp[o:o + L])
    assert lz.fnv1a64(got.cpu().numpy()) == oracle.fnv1a64(x[o:o + L])
    srv.release(rid)
    srv.destroy()
    da.close()


@pytest.mark.parametrize("thr", [lz.BASE_THR, lz.TUNED_THR])
def test_fastq_1gib_full_size_matches_oracle(thr):
    """The benchmark's FASTQ-like workload at its full size (1,073,741,535
    bytes, 64 KiB blocks) in the launch configuration the bench times (G 64,
    unroll 2, schedule 1): the GPU decode equals the oracle's sequential
    decode of the same archive and the input, byte for byte and by FNV-1a 64;
    so do ranges sampled across the file."""
    dev = _dev()
    x = synth.fastq(1 << 30, seed=3)
    print("encoding %d bytes with %s" % (x.size, thr), flush=True)
    arc = lz.encode(x, 16, thr)
    ref = oracle.decode(arc)
    assert np.array_equal(ref, x)
    da = lz.DeviceArchive(arc, device=dev)
    out = da.decode(G=64, unroll=2, schedule=1)
    torch.cuda.synchronize()
    assert torch.equal(out, torch.from_numpy(ref).to(dev))
    assert lz.fnv1a64(out.cpu().numpy()) == oracle.fnv1a64(ref)
    rng = np.random.default_rng(7)
    for _ in range(12):
        L = int(np.exp(rng.uniform(np.log(16), np.log(8 << 20))))
        o = int(rng.integers(0, x.size - L))
        got = da.decode_range(o, L)
        assert bytes(got.cpu().numpy()) == bytes(ref[o:o + L]), (o, L)
    da.close()


@pytest.mark.parametrize("m", [256, 1024])
def test_sweep_stream_full_size_matches_oracle(m):
    """The granularity sweep's 256 MiB streams at the mean match lengths where
    the bandwidth target is set, 16 KiB blocks, every G: equal to the oracle's
    execution of the same tokens."""
    dev = _dev()
    n = 1 << 28
    seed = 2 + (32, 64, 128, 256, 512, 1024).index(m)
    ll, ml, sr, lit = synth.geo_tokens(n, m, seed=seed)
    exp = torch.from_numpy(oracle.exec_tokens(n, ll, ml, sr, lit)).to(dev)
    da = lz.DeviceArchive(lz.build_archive(n, 14, ll, ml, sr, lit), device=dev)
    for G in (8, 16, 32, 64):
        print("m=%d G=%d" % (m, G), flush=True)
        out = da.decode(G=G)
        torch.cuda.synchronize()
        assert torch.equal(out, exp), G
    da.close()
