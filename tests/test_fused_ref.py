"""CPU checks of the reference count of literal-sourced matches (the matches
the parse copies from the literal stream, `fused_ref.literal_sourced`), which
the GPU test compares with the plan: a hand-built archive with one case of
each kind, and a byte-by-byte brute force over small encoded inputs."""
import numpy as np

import oracle
import synth
from fused_ref import literal_sourced


def brute_force(arc):
    """Per match: depth 1, no overlap with its own output, and every source
    byte a literal byte of one and the same token (checked byte by byte)."""
    tk = oracle.tokens(arc)
    depth, _ = oracle.levels(arc)
    n = oracle.info(arc)["n"]
    owner = np.full(n, -1, dtype=np.int64)  # token whose literal run holds the byte, else -1
    for t in range(len(tk["dst"])):
        d, ll = int(tk["dst"][t]), int(tk["lit_len"][t])
        owner[d:d + ll] = t
    out = np.zeros(len(tk["dst"]), dtype=bool)
    for t in range(len(tk["dst"])):
        ml = int(tk["mlen"][t])
        if ml == 0 or depth[t] != 1:
            continue
        s, md = int(tk["src"][t]), int(tk["dst"][t] + tk["lit_len"][t])
        if s + ml > md:
            continue
        o = owner[s:s + ml]
        out[t] = bool(o[0] >= 0 and (o == o[0]).all())
    return out


def test_hand_built_cases():
    # 64-byte blocks; tokens (literal run, match length, source):
    #   A [0,20) lits, match 10 from 2 (inside A's run)          -> copied by the parse
    #   B [30,35) lits, match 8 from 31 (overlaps itself, d = 4)  -> not
    #   C [43,46) lits, match 6 from 21 (reads A's match: depth 2) -> not
    #   D [52,64) lits, block end
    #   E [64,74) lits, match 12 from 58 (D's run and E's run)    -> not
    #   F [86,90) lits, match 10 from 0 (inside A's run)          -> copied by the parse
    #   G [100,128) lits
    ll = [20, 5, 3, 12, 10, 4, 28]
    ml = [10, 8, 6, 0, 12, 10, 0]
    sr = [2, 31, 21, 0, 58, 0, 0]
    lit = synth.random_bytes(sum(ll), 4)
    arc = oracle.write_archive(128, 6, ll, ml, sr, lit)
    depth, mx = oracle.levels(arc)
    assert list(depth) == [1, 1, 2, 0, 1, 1, 0] and mx == 2
    mask, md, mlen = literal_sourced(arc)
    assert list(mask) == [True, False, False, False, False, True, False]
    assert list(md[mask]) == [20, 90] and int(mlen[mask].sum()) == 20
    assert np.array_equal(mask, brute_force(arc))


def test_matches_brute_force_on_encoded_inputs():
    for x, lb, thr in ((synth.fastq(40 << 10, seed=11), 12, (12, 16, 24, 32)),
                       (synth.fastq(40 << 10, seed=11), 14, (6, 8, 10, 12)),
                       (synth.zipf_text(32 << 10, seed=3), 12, (6, 8, 10, 12))):
        ll, ml, sr, lit = oracle.encode(x, lb, thr)
        arc = oracle.write_archive(x.size, lb, ll, ml, sr, lit, min_match=min(thr), thr=thr,
                                   bounds=oracle.BOUNDS_CFG)
        mask, _, _ = literal_sourced(arc)
        bf = brute_force(arc)
        assert mask.sum() > 0 and np.array_equal(mask, bf)
