"""Encoder depth cap: the matches that would lie deeper than the cap become
literals.  Pinned by the oracle: a capped archive decodes to the input; its
deepest match (the oracle's own level computation) is at most the cap; every
match it keeps is a match of the uncapped parse (same output position,
source and length); every match it drops would have been deeper than the cap
given the bytes before it (no match is dropped needlessly); and a cap at the
uncapped depth changes nothing."""
import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz


def _matches(arc):
    tk = oracle.tokens(arc)
    m = tk["mlen"] > 0
    pos = (tk["dst"] + tk["lit_len"])[m].astype(np.int64)
    return pos, tk["src"][m].astype(np.int64), tk["mlen"][m].astype(np.int64)


def _byte_depths(arc, n):
    """Depth of the token that writes each output byte (literals 0)."""
    lv, _ = oracle.levels(arc)
    tk = oracle.tokens(arc)
    m = tk["mlen"] > 0
    pos = (tk["dst"] + tk["lit_len"])[m].astype(np.int64)
    ln = tk["mlen"][m].astype(np.int64)
    d = np.zeros(n, np.uint32)
    idx = np.repeat(pos, ln) + (np.arange(ln.sum()) - np.repeat(np.cumsum(ln) - ln, ln))
    d[idx] = np.repeat(lv[m], ln)
    return d


CASES = [("zipf", lambda: synth.zipf_text(3 << 20, seed=2), 14, lz.BASE_THR),
         ("fastq", lambda: synth.fastq(6 << 20, seed=3), 16, lz.TUNED_THR)]


@pytest.mark.parametrize("name,make,lb,thr", CASES, ids=[c[0] for c in CASES])
def test_depth_cap(name, make, lb, thr):
    x = make()
    base = lz.encode(x, lb, thr)
    _, d0 = oracle.levels(base)
    assert d0 >= 4, d0
    p0, s0, l0 = _matches(base)
    kept0 = set(zip(p0.tolist(), s0.tolist(), l0.tolist()))
    rng = np.random.default_rng(1)
    for cap in sorted({1, 2, d0 // 2, d0 - 1}):
        arc = lz.encode(x, lb, thr, depth_cap=cap)
        assert np.array_equal(oracle.decode(arc), x), cap
        _, d = oracle.levels(arc)
        assert d <= cap, (cap, d)
        p, s, l = _matches(arc)
        kept = set(zip(p.tolist(), s.tolist(), l.tolist()))
        assert kept <= kept0, cap
        dropped = sorted(kept0 - kept)
        assert dropped, cap
        bd = _byte_depths(arc, x.size)
        for j in rng.choice(len(dropped), min(len(dropped), 1500), replace=False):
            q, sr, ln = dropped[j]
            assert bd[q:q + ln].max() == 0, (cap, q)  # its bytes are literals now
            e = min(sr + ln, q)
            assert int(bd[sr:e].max()) + 1 > cap, (cap, q, sr, ln)
    same = lz.encode(x, lb, thr, depth_cap=d0)
    assert bytes(same) == bytes(base)


def test_depth_cap_limits():
    x = synth.zipf_text(100_000, seed=1)
    with pytest.raises(lz.LzError) as e:
        lz.encode(x, 12, depth_cap=65535)
    assert e.value.rc == lz.LZ_E_INVAL
    arc = lz.encode(x, 12, lz.BASE_THR, depth_cap=65534)
    assert bytes(arc) == bytes(lz.encode(x, 12, lz.BASE_THR))
