"""GPU range decode (region seek): every range equals the same bytes of the
oracle's full decode, alone and merged into one multi-range plan."""
import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def horizon_by_definition(tk, first, end, log2_grain=20):
    """The decode horizon of output [first, end), straight from its definition:
    the largest multiple h of the grain (2^20 bytes) at or below `first` such
    that no match written in [h, end of the grain holding end - 1) reads a
    byte below h; searched one grain at a time from the top."""
    grain = 1 << log2_grain
    g_end = ((end - 1) // grain + 1) * grain
    m = tk["mlen"] > 0
    mdst = (tk["dst"] + tk["lit_len"])[m].astype(np.int64)
    msrc = tk["src"][m].astype(np.int64)
    h = (first // grain) * grain
    while h > 0:
        sel = (mdst >= h) & (mdst < g_end)
        if not sel.any() or msrc[sel].min() >= h:
            return h
        h -= grain
    return 0


def _ranges(n, bs, rng, k=40):
    r = [(0, 1), (0, n), (n - 1, 1), (n - 7, 7), (bs - 3, 9), (2 * bs - 1, bs + 2), (n // 2, 0)]
    for _ in range(k):
        L = int(min(n, np.exp(rng.uniform(0, np.log(max(2, n // 4))))))
        o = int(rng.integers(0, n - L + 1))
        r.append((o, L))
    return [(o, L) for o, L in r if 0 <= o and o + L <= n]


def _check_archive(arc, expect, label, log2_bs):
    dev = _dev()
    da = lz.DeviceArchive(arc, device=dev)
    n = da.n
    rng = np.random.default_rng(len(expect))
    rs = _ranges(n, 1 << log2_bs, rng)
    exp_t = torch.from_numpy(np.ascontiguousarray(expect)).to(dev)
    for o, L in rs:
        print(f"[{label}] range {o} +{L}", flush=True)
        got = da.decode_range(o, L)
        torch.cuda.synchronize()
        assert torch.equal(got, exp_t[o:o + L]), (label, o, L)
    # all ranges merged into one plan, into one arena
    offs = [o for o, L in rs]
    lens = [L for o, L in rs]
    plan = da.range_plan(offs, lens)
    oo = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64) if lens else np.zeros(0, np.uint64)
    out = torch.full((int(sum(lens)) + 8,), 0x5A, dtype=torch.uint8, device=dev)
    scratch = torch.empty(plan.scratch_bytes, dtype=torch.uint8, device=dev)
    plan.run(out, oo, scratch)
    torch.cuda.synchronize()
    for (o, L), q in zip(rs, oo):
        assert torch.equal(out[int(q):int(q) + L], exp_t[o:o + L]), (label, "merged", o, L)
    assert bool((out[int(sum(lens)):] == 0x5A).all().item())
    plan.free()
    da.close()


@pytest.mark.parametrize("thr", [lz.BASE_THR, lz.TUNED_THR])
def test_range_fastq(thr):
    x = synth.fastq(6 << 20, seed=3)
    arc = lz.encode(x, 16, thr)
    _check_archive(arc, x, f"fastq{thr}", 16)


def test_range_zipf_small_blocks():
    x = synth.zipf_text(3 << 20, seed=2)
    arc = lz.encode(x, 12, lz.BASE_THR)
    _check_archive(arc, x, "zipf", 12)


def test_range_generated_and_overlaps():
    n = 2 << 20
    ll, ml, sr, lit = synth.geo_tokens(n, 64, seed=4, lit_prefix=4096, min_back=1)
    x = oracle.exec_tokens(n, ll, ml, sr, lit)
    arc = lz.build_archive(n, 14, ll, ml, sr, lit)
    _check_archive(arc, x, "geo-overlap", 14)
    z = np.zeros(300_000, np.uint8)
    z[::1000] = 7
    _check_archive(lz.encode(z, 12, (4, 4, 4, 4)), z, "runs", 12)


def test_range_errors():
    dev = _dev()
    x = synth.zipf_text(50_000, seed=1)
    da = lz.DeviceArchive(lz.encode(x, 12), device=dev)
    with pytest.raises(lz.LzError) as e:
        da.decode_range(49_990, 11)
    assert e.value.rc == lz.LZ_E_RANGE
    with pytest.raises(lz.LzError):
        da.range_plan([10, 60_000], [5, 1])
    got = da.decode_range(49_990, 10)
    assert bytes(got.cpu().numpy()) == bytes(x[49_990:])


def test_range_plan_modes():
    """A seek whose closure is small is served from its closure; one whose
    closure would exceed max(256 KiB, (end - horizon) / 4096) decodes its prefix on the
    device instead.  Both give the input's bytes."""
    dev = _dev()
    z = synth.zipf_text(8 << 20, seed=5)
    da = lz.DeviceArchive(lz.encode(z, 16, lz.TUNED_THR), device=dev)
    p = da.range_plan([100], [4096])
    assert p.prefix_bytes == 0 and 0 < p.closure_bytes < (256 << 10)
    p.free()
    da.close()
    x = synth.fastq(8 << 20, seed=5)
    da = lz.DeviceArchive(lz.encode(x, 16, lz.TUNED_THR), device=dev)
    # a small range early in the file: a closure plan, whose bytes are the input's
    p = da.range_plan([20_000], [3000])
    assert p.prefix_bytes == 0 and 0 < p.closure_bytes < (256 << 10)
    out = torch.zeros(3000, dtype=torch.uint8, device=dev)
    scratch = torch.empty(p.scratch_bytes, dtype=torch.uint8, device=dev)
    p.run(out, np.zeros(1, np.uint64), scratch)
    torch.cuda.synchronize()
    assert bytes(out.cpu().numpy()) == bytes(x[20_000:23_000])
    p.free()
    p = da.range_plan([6 << 20, 1 << 20], [16 << 10, 1 << 20])
    assert p.closure_bytes == 0 and p.prefix_bytes == (6 << 20) + (16 << 10) - p.horizon
    assert p.horizon == horizon_by_definition(oracle.tokens(da.arc), 1 << 20, (6 << 20) + (16 << 10))
    out = torch.zeros((17 << 16) + (1 << 20), dtype=torch.uint8, device=dev)
    scratch = torch.empty(p.scratch_bytes, dtype=torch.uint8, device=dev)
    p.run(out, np.array([0, 16 << 10], np.uint64), scratch)
    torch.cuda.synchronize()
    assert bytes(out[:16 << 10].cpu().numpy()) == bytes(x[6 << 20:(6 << 20) + (16 << 10)])
    assert bytes(out[16 << 10:(16 << 10) + (1 << 20)].cpu().numpy()) == bytes(x[1 << 20:2 << 20])
    p.free()
    da.close()


@pytest.mark.parametrize("segment_mib", [0, 4])
def test_range_prefix_horizon(segment_mib):
    """Prefix plans start at the decode horizon: on an archive encoded in
    4 MiB segments that is the segment start, so a seek decodes at most the
    segment up to its range; without segments it is what the sources allow.
    The horizon equals its definition computed from the oracle's tokens, and
    every range equals the oracle's decode, alone and merged."""
    dev = _dev()
    x = synth.fastq(24 << 20, seed=11)
    arc = lz.encode(x, 16, lz.TUNED_THR, segment=segment_mib << 20)
    expect = oracle.decode(arc)
    assert np.array_equal(expect, x)
    tk = oracle.tokens(arc)
    da = lz.DeviceArchive(arc, device=dev)
    n = da.n
    exp_t = torch.from_numpy(expect).to(dev)
    rng = np.random.default_rng(7)
    cases = [((4 << 20) - 5, 10), ((4 << 20), 3 << 20), ((13 << 20) + 12345, 2 << 20), (n - (2 << 20), 2 << 20),
             ((8 << 20) + 1, 1 << 20)]
    cases += [(int(rng.integers(0, n - (3 << 20))), int(rng.integers(1 << 20, 3 << 20))) for _ in range(8)]
    prefix_plans = 0
    for o, L in cases:
        print(f"[horizon seg={segment_mib}] range {o} +{L}", flush=True)
        p = da.range_plan([o], [L])
        if p.prefix_bytes:
            prefix_plans += 1
            h = horizon_by_definition(tk, o, o + L)
            assert p.horizon == h, (o, L, p.horizon, h)
            assert p.prefix_bytes == o + L - h
            if segment_mib:
                assert h >= (o // (segment_mib << 20)) * (segment_mib << 20)
                assert p.scratch_bytes < (segment_mib << 21)
        out = torch.full((L + 16,), 0xA5, dtype=torch.uint8, device=dev)
        scratch = torch.empty(p.scratch_bytes, dtype=torch.uint8, device=dev)
        p.run(out, np.zeros(1, np.uint64), scratch)
        torch.cuda.synchronize()
        assert torch.equal(out[:L], exp_t[o:o + L]), (o, L)
        assert bool((out[L:] == 0xA5).all().item())
        p.free()
    assert prefix_plans >= 5
    # merged: the horizon of the lowest range start serves every range
    offs = [o for o, L in cases[:6]]
    lens = [L for o, L in cases[:6]]
    p = da.range_plan(offs, lens)
    oo = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.uint64)
    out = torch.empty(int(sum(lens)), dtype=torch.uint8, device=dev)
    scratch = torch.empty(p.scratch_bytes, dtype=torch.uint8, device=dev)
    p.run(out, oo, scratch)
    torch.cuda.synchronize()
    if p.prefix_bytes:
        assert p.horizon == horizon_by_definition(tk, min(offs), max(o + L for o, L in zip(offs, lens)))
    for (o, L), q in zip(zip(offs, lens), oo):
        assert torch.equal(out[int(q):int(q) + L], exp_t[o:o + L]), ("merged", o, L)
    p.free()
    da.close()
