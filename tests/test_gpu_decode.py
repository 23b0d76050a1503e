"""GPU parity: the HIP match-phase decoder against the CPU oracle, byte for
byte and by FNV-1a 64, through the C ABI (paper_2607_18541_amd.lz)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GS = (8, 16, 32, 64)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check(arc, expect, cfgs, label):
    dev = _dev()
    da = lz.DeviceArchive(arc, device=dev)
    exp_t = torch.from_numpy(np.ascontiguousarray(expect)).to(dev)
    h = oracle.fnv1a64(expect)
    for c in cfgs:
        G, U, S = c[:3]
        M = c[3] if len(c) > 3 else 0
        # the parse runs with the copy's G and unroll unless the case names its own
        PG = c[4] if len(c) > 4 else G
        PU = c[5] if len(c) > 5 else U
        print(f"[{label}] G={G} U={U} sched={S} mapping={M} parse {PG}/{PU} n={da.n}", flush=True)
        out = torch.full((max(da.n, 1) + 64,), 0xA5, dtype=torch.uint8, device=dev)
        got = da.decode(out, G=G, unroll=U, schedule=S, mapping=M, parse_G=PG, parse_unroll=PU)
        torch.cuda.synchronize()
        if not torch.equal(got, exp_t):
            bad = (got != exp_t).nonzero()
            i = int(bad[0].item())
            raise AssertionError(f"{label} G={G} U={U} S={S} M={M}: {bad.numel()} bytes differ, first at {i}")
        assert lz.fnv1a64(got.cpu().numpy()) == h
        # nothing written past n
        assert bool((out[da.n:] == 0xA5).all().item())
    da.close()


# (G, unroll, schedule[, mapping[, parse G, parse unroll]]); mapping 1 =
# XCD-contiguous workgroups; without parse values the parse takes G and unroll
ALL = [(G, U, S) for G in GS for U in (1, 2, 4) for S in (0, 1)] + [(64, 2, 1, 1), (32, 4, 0, 1), (8, 1, 1, 1)] + \
    [(32, 2, 1, 0, 64, 2), (8, 4, 1, 0, 64, 2), (16, 1, 0, 0, 64, 4), (64, 2, 1, 0, 32, 1)]
SOME = [(8, 2, 0), (32, 1, 0), (64, 4, 0), (16, 2, 1), (32, 4, 1), (64, 2, 1, 1), (16, 2, 0, 1), (32, 2, 1, 0, 64, 2)]


def test_zipf_1mib_all_configs():
    """1 MiB Zipf text, 64 KiB blocks, 6/8/10/12 (the small text config)."""
    x = synth.zipf_text(1 << 20, seed=1)
    arc = lz.encode(x, 16, lz.BASE_THR)
    assert np.array_equal(oracle.decode(arc), x)
    _check(arc, x, ALL, "zipf1m")


@pytest.mark.parametrize("thr", [lz.BASE_THR, lz.TUNED_THR])
def test_fastq_4mib(thr):
    x = synth.fastq(4 << 20, seed=3)
    arc = lz.encode(x, 16, thr)
    _check(arc, oracle.decode(arc), SOME, f"fastq{thr}")


@pytest.mark.parametrize("lb", [12, 14, 16, 20])
def test_geo_tokens_blocks(lb):
    """Generated streams (controlled mean match length), several block sizes."""
    n = 3 << 20
    ll, ml, sr, lit = synth.geo_tokens(n, 128, seed=2, lit_prefix=65536)
    expect = oracle.exec_tokens(n, ll, ml, sr, lit)
    arc = lz.build_archive(n, lb, ll, ml, sr, lit)
    _check(arc, expect, SOME, f"geo bs=2^{lb}")


def _tokens_to_arc(n, toks, lits, lb):
    ll = np.array([t[0] for t in toks], np.uint32)
    ml = np.array([t[1] for t in toks], np.uint32)
    sr = np.array([t[2] for t in toks], np.uint64)
    lit = np.array(lits, np.uint8)
    assert int(ll.sum() + ml.sum()) == n
    return lz.build_archive(n, lb, ll, ml, sr, lit), oracle.exec_tokens(n, ll, ml, sr, lit)


def test_adversarial_raw_chain():
    """Every match reads the bytes the previous token just wrote."""
    rng = np.random.default_rng(1)
    toks, lits, pos = [], [], 0
    while pos < 200_000:
        L = int(rng.integers(0, 3))
        lits += list(rng.integers(0, 256, L))
        pos += L
        if pos == 0:
            lits.append(7); pos += 1; toks.append((1, 0, 0)); continue
        M = int(rng.integers(1, 40))
        back = int(rng.integers(1, min(pos, 48) + 1))
        toks.append((L, M, pos - back))
        pos += M
    arc, exp = _tokens_to_arc(pos, toks, lits, 14)
    _check(arc, exp, ALL[::3], "rawchain")


def test_adversarial_overlap_distances():
    toks, lits, pos = [], [], 0
    rng = np.random.default_rng(2)
    for d in (1, 2, 3, 15, 16, 17, 63, 64, 65, 1023, 1024, 1025):
        for M in (d + 1, 2 * d + 5, 4000, 17):
            L = d + 3
            lits += list(rng.integers(0, 256, L))
            pos += L
            toks.append((L, M, pos - d))
            pos += M
    arc, exp = _tokens_to_arc(pos, toks, lits, 12)
    _check(arc, exp, ALL[::2], "overlap")


def test_adversarial_alignments():
    """Every source/destination alignment mod 16, short and long copies."""
    rng = np.random.default_rng(3)
    base = list(rng.integers(0, 256, 4096))
    toks, lits, pos = [(4096, 0, 0)], base[:], 4096
    for sa in range(16):
        for da in range(16):
            pad = (da - pos) % 16
            lits += list(rng.integers(0, 256, pad + 1))
            pos += pad + 1
            for M in (1, 5, 16, 33, 100):
                src = 1024 + sa + 16 * int(rng.integers(0, 100))
                toks.append((pad + 1 if M == 1 else 0, M, src))
                pos += M
                pad = 0
    arc, exp = _tokens_to_arc(pos, toks, lits, 13)
    _check(arc, exp, SOME + [(64, 1, 0), (8, 4, 0)], "align")


def test_adversarial_deep_chain():
    """A chain of 300 dependency levels: each block copies from the previous."""
    bs = 1 << 10
    rng = np.random.default_rng(4)
    toks, lits, pos = [(bs, 0, 0)], list(rng.integers(0, 256, bs)), bs
    for b in range(1, 300):
        toks.append((3, bs - 3, pos - bs + 5))
        lits += list(rng.integers(0, 256, 3))
        pos += bs
    arc, exp = _tokens_to_arc(pos, toks, lits, 10)
    lv, mx = lz.plan(arc)
    assert mx >= 299
    _check(arc, exp, [(8, 1, 0), (32, 2, 0), (64, 4, 0), (16, 1, 1)], "deep")


def test_adversarial_block_edges_and_long_literals():
    """Matches ending exactly at block ends; literal runs of a whole block."""
    rng = np.random.default_rng(5)
    bs = 1 << 12
    toks, lits = [], []
    lits += list(rng.integers(0, 256, 3 * bs))
    toks.append((3 * bs, 0, 0))
    pos = 3 * bs
    for b in range(3, 40):
        L = int(rng.integers(0, 200))
        lits += list(rng.integers(0, 256, L))
        toks.append((L, bs - L, int(rng.integers(0, pos - bs))))
        pos += bs
    arc, exp = _tokens_to_arc(pos, toks, lits, 12)
    _check(arc, exp, SOME, "edges")


@pytest.mark.parametrize("n", [1, 15, 16, 17, 4095, 4096, 4097, 65535, 65537])
def test_small_and_ragged_sizes(n):
    x = synth.zipf_text(n, seed=n)
    arc = lz.encode(x, 12, (4, 4, 4, 4))
    _check(arc, x, [(8, 1, 0), (64, 4, 0), (32, 2, 1)], f"n={n}")


def test_empty_archive():
    _dev()
    arc = lz.encode(np.zeros(0, np.uint8), 12)
    da = lz.DeviceArchive(arc)
    assert da.n == 0
    da.decode(torch.empty(1, dtype=torch.uint8, device="cuda"))


def test_output_capacity_rejected():
    _dev()
    x = synth.zipf_text(10000, seed=1)
    da = lz.DeviceArchive(lz.encode(x, 12))
    with pytest.raises(lz.LzError):
        da.decode(torch.empty(9999, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("m", [32, 256])
def test_purecopy_matches_reference(m):
    """Pre-decoded tokens whose matches read a pre-filled reference buffer
    (the pure-copy control): the output equals the reference."""
    dev = _dev()
    n = 4 << 20
    ll, ml, sr, lit = synth.geo_tokens(n, m, seed=10 + m)
    ref = oracle.exec_tokens(n, ll, ml, sr, lit)
    dst = np.concatenate([[0], np.cumsum(ll.astype(np.uint64) + ml)[:-1]]).astype(np.uint64)
    loff = np.concatenate([[0], np.cumsum(ll.astype(np.uint64))[:-1]]).astype(np.uint64)
    for lb in (14, 16):
        blk = dst >> lb
        us = np.searchsorted(blk, np.arange(0, (n >> lb) + 1), side="left").astype(np.uint64)
        us = np.unique(np.concatenate([us, [dst.size]])).astype(np.uint64)
        us[0] = 0
        T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        for G, U in ((8, 2), (32, 1), (64, 4)):
            print(f"[purecopy m={m} bs=2^{lb}] G={G} U={U}", flush=True)
            out = torch.zeros(n, dtype=torch.uint8, device=dev)
            lz.purecopy(T(dst), T(loff), T(ll), T(sr), T(ml), T(us), T(lit), T(ref), out, G=G, unroll=U)
            torch.cuda.synchronize()
            assert torch.equal(out, T(ref))


def test_stages_and_tail_settings_agree():
    """Parse and match passes launched apart, and every tail setting (no tail
    launch, tail of one-window depths, default, everything after the first
    depth), give the oracle's bytes."""
    dev = _dev()
    x = synth.fastq(3 << 20, seed=9)
    arc = lz.encode(x, 14, lz.BASE_THR)
    exp = torch.from_numpy(oracle.decode(arc)).to(dev)
    da = lz.DeviceArchive(arc, device=dev)
    assert da.levels >= 8
    out = torch.full((da.n + 32,), 0x3C, dtype=torch.uint8, device=dev)
    print("[stages] staged decode", flush=True)
    da.decode_stage(out, 1)
    da.decode_stage(out, 2)
    da.check()
    torch.cuda.synchronize()
    assert torch.equal(out[:da.n], exp)
    for tail in (lz.TAIL_OFF, 1, 0, 1 << 20):
        print(f"[stages] tail={tail}", flush=True)
        out.fill_(0x3C)
        got = da.decode(out, tail=tail)
        torch.cuda.synchronize()
        assert torch.equal(got, exp), tail
        assert bool((out[da.n:] == 0x3C).all().item())
    da.close()


@pytest.mark.parametrize("off", [1, 7, 8, 15])
def test_unaligned_output_address(off):
    """Output views at every class of misalignment: literal blocks are aligned
    in the address space, so the span ends move; nothing outside [off, off+n)."""
    dev = _dev()
    x = synth.fastq(300_000, seed=off)
    arc = lz.encode(x, 14, lz.TUNED_THR)
    da = lz.DeviceArchive(arc, device=dev)
    exp_t = torch.from_numpy(x).to(dev)
    for G, U, S in [(64, 2, 1), (16, 4, 0), (32, 1, 1)]:
        print(f"[unaligned off={off}] G={G} U={U} sched={S}", flush=True)
        buf = torch.full((da.n + 64,), 0x5A, dtype=torch.uint8, device=dev)
        view = buf[off:off + da.n]
        got = da.decode(view, G=G, unroll=U, schedule=S)
        torch.cuda.synchronize()
        assert torch.equal(got, exp_t)
        assert bool((buf[:off] == 0x5A).all().item()) and bool((buf[off + da.n:] == 0x5A).all().item())
    da.close()


def test_dense_short_runs_many_per_block():
    """Literal runs and matches of 1-3 bytes (literals about half the bytes):
    the whole-span parse path with up to eight runs inside one 16-byte block,
    and near sources (overlapping matches)."""
    rng = np.random.default_rng(7)
    toks, lits, pos = [(64, 0, 0)], list(rng.integers(0, 256, 64)), 64
    while pos < 300_000:
        L = int(rng.integers(1, 4))
        lits += list(rng.integers(0, 256, L))
        pos += L
        M = int(rng.integers(1, 4))
        back = int(rng.integers(1, min(pos, 300) + 1))
        toks.append((L, M, pos - back))
        pos += M
    arc, exp = _tokens_to_arc(pos, toks, lits, 14)
    _check(arc, exp, [(64, 2, 1), (64, 1, 0), (32, 4, 1), (8, 2, 1)], "dense-short")


def test_occupancy_control_decodes_exactly():
    """The occupancy control (depth passes held to k resident workgroups per
    CU by LDS padding) changes only the schedule: the bytes equal the
    oracle's; values outside [3, 8] are refused."""
    dev = _dev()
    x = synth.fastq(4 << 20, seed=3)
    arc = lz.encode(x, 16, lz.TUNED_THR)
    da = lz.DeviceArchive(arc, device=dev)
    exp_t = torch.from_numpy(oracle.decode(arc)).to(dev)
    for k in (6, 4, 3):
        print(f"[occupancy {k}]", flush=True)
        out = torch.full((da.n + 64,), 0xA5, dtype=torch.uint8, device=dev)
        got = da.decode(out, occupancy=k)
        torch.cuda.synchronize()
        assert torch.equal(got, exp_t), k
        assert bool((out[da.n:] == 0xA5).all().item())
    for bad in (2, 9):
        with pytest.raises(lz.LzError) as e:
            da.decode(occupancy=bad)
        assert e.value.rc == lz.LZ_E_INVAL
    da.close()


@pytest.mark.parametrize("cap", [1, 3, 8])
def test_depth_capped_archives(cap):
    """Archives encoded with a depth cap decode exactly, and the device plan
    has the oracle's depth count (at most the cap)."""
    x = synth.zipf_text(3 << 20, seed=2)
    arc = lz.encode(x, 14, lz.BASE_THR, depth_cap=cap)
    expect = oracle.decode(arc)
    assert np.array_equal(expect, x)
    _, d = oracle.levels(arc)
    assert d <= cap
    da = lz.DeviceArchive(arc, device=_dev())
    assert da.levels == d, (da.levels, d)
    da.close()
    _check(arc, expect, SOME, f"cap{cap}")
