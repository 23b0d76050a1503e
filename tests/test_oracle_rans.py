"""The tile-rANS oracle against what the definition fixes (CPU only): a tile
worked by hand (tests/golden/rans_tile_aab.txt), the quantisation rule's
branches on hand-counted inputs, round trips, the code length against the
ideal length under the quantised model, and the repeated and raw special
cases; then the library's coder against the oracle: byte-identical coded
containers, the oracle's decode of them, and rejection of corrupt ones."""
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rans_tile_aab.txt")


def _golden():
    freq, states, rest, size = {}, {}, None, None
    for line in open(GOLDEN):
        w = line.split()
        if not w or w[0].startswith("#"):
            continue
        if w[0] == "freq":
            freq[int(w[1])] = int(w[2])
        elif w[0] == "state":
            states[int(w[1])] = int(w[2])
        elif w[0] == "state_rest":
            rest = int(w[1])
        elif w[0] == "payload_bytes":
            size = int(w[1])
    return freq, states, rest, size


def _parse_payload(p):
    bitmap = p[:32]
    syms = [s for s in range(256) if (bitmap[s // 8] >> (s % 8)) & 1]
    o = 32
    f = {}
    for s in syms:
        f[s] = int(p[o]) | (int(p[o + 1]) << 8)
        o += 2
    st = [int.from_bytes(p[o + 4 * j:o + 4 * j + 4].tobytes(), "little") for j in range(64)]
    o += 256
    words = [int(p[o + 2 * k]) | (int(p[o + 2 * k + 1]) << 8) for k in range((p.size - o) // 2)]
    return f, st, words


def test_hand_worked_tile():
    freq, states, rest, size = _golden()
    p = oracle.rans_encode_tile(np.frombuffer(b"aab", np.uint8))
    assert p.size == size
    f, st, words = _parse_payload(p)
    assert f == freq and not words
    for j in range(64):
        assert st[j] == states.get(j, rest), j
    assert bytes(oracle.rans_decode_tile(p, 3)) == b"aab"


def test_quantisation_branches():
    # shortfall goes to the most frequent symbol
    c = np.zeros(256, np.uint64)
    c[ord("a")], c[ord("b")] = 2, 1
    f = oracle.rans_normalise(c)
    assert f[ord("a")] == 2731 and f[ord("b")] == 1365 and f.sum() == 4096
    # excess: 200 singletons raised to 1 and one symbol of 65,336:
    # floor(65336 * 4096 / 65536) = 4083; 4083 + 200 = 4283, 187 too many,
    # taken from the largest frequency above 1
    c = np.zeros(256, np.uint64)
    c[:200] = 1
    c[250] = 65336
    f = oracle.rans_normalise(c)
    assert np.all(f[:200] == 1) and f[250] == 4083 - 187 and f.sum() == 4096
    # ties in count: the lowest byte takes the correction
    c = np.zeros(256, np.uint64)
    c[[10, 20, 30]] = 1
    f = oracle.rans_normalise(c)
    assert f[10] == 1366 and f[20] == 1365 and f[30] == 1365


@pytest.mark.parametrize("seed", range(8))
def test_round_trip_and_code_length(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 65537))
    alpha = int(rng.integers(2, 257))
    p = rng.dirichlet(np.full(alpha, 0.3))
    x = rng.choice(alpha, size=N, p=p).astype(np.uint8)
    if np.all(x == x[0]):
        x[0] ^= 1
    pay = oracle.rans_encode_tile(x)
    assert np.array_equal(oracle.rans_decode_tile(pay, N), x)
    f, st, words = _parse_payload(pay)
    # ideal length under the quantised model: sum of log2(4096 / f(x_i)) bits;
    # the coded bits (words plus final states, less the 64 x 16 starting bits)
    # match it up to rounding of the integer divisions
    fx = np.array([f.get(s, 0) for s in range(256)], dtype=np.float64)[x]
    ideal = float(np.sum(np.log2(4096.0 / fx)))
    coded = 16 * len(words) + sum(np.log2(s) for s in st) - 64 * 16
    assert abs(coded - ideal) <= 0.002 * ideal + 64 * 2, (coded, ideal)


def test_entropy_container_special_cases_and_identity():
    # a literal-only archive of a constant run, random bytes, and FASTQ-like text
    for x, lb in ((np.full(200_000, 7, np.uint8), 12), (synth.random_bytes(150_000, 5), 14),
                  (synth.fastq(300_000, seed=2), 14), (np.zeros(0, np.uint8), 12), (synth.zipf_text(5, seed=1), 4)):
        arc = lz.encode(x, lb, lz.TUNED_THR)
        mine = lz.entropy_encode(arc)
        ref = oracle.entropy_encode(arc)
        assert np.array_equal(mine, ref)  # same reading of the coder, independently written
        assert np.array_equal(oracle.entropy_decode(mine), arc)
        assert np.array_equal(oracle.decode(oracle.entropy_decode(mine)), x)
    # random literals stay raw: the coded size is the raw size plus records
    arc = lz.encode(synth.random_bytes(300_000, 9), 16, lz.TUNED_THR)
    info = lz.entropy_info(lz.entropy_encode(arc))
    assert info["raw"] >= 4


def test_coded_size_near_order0_bound():
    x = synth.fastq(8 << 20, seed=3)
    arc = lz.encode(x, 16, lz.TUNED_THR)
    coded = lz.entropy_encode(arc)
    ent, _ = lz.entropy_size(arc)
    # the bound charges 1 + 2 x distinct per tile; a rANS tile carries its
    # 32-byte bitmap and 256 bytes of states: within 1.5 % of the bound
    assert ent <= coded.size <= 1.015 * ent + 4096, (coded.size, ent)


def test_corrupt_coded_containers_rejected():
    arc = lz.encode(synth.fastq(200_000, seed=4), 14, lz.TUNED_THR)
    good = lz.entropy_encode(arc)
    nt = int(np.frombuffer(good[16:20].tobytes(), np.uint32)[0])
    rec = 192
    rans = [t for t in range(nt) if int(np.frombuffer(good[rec + 32 * t + 28:rec + 32 * t + 32].tobytes(),
                                                        np.uint32)[0]) == 1]
    assert rans
    bad = []
    b = good.copy()
    b[rec + 16:rec + 20] = np.frombuffer(np.uint32(65537).tobytes(), np.uint8)  # too many symbols
    bad.append(b)
    b = good.copy()
    t = rans[0]
    po = int(np.frombuffer(good[rec + 32 * t:rec + 32 * t + 8].tobytes(), np.uint64)[0])
    p0 = 192 + 32 * nt
    fpos = p0 + po + 32  # first frequency
    b[fpos] ^= 1  # frequencies no longer sum to 4096
    bad.append(b)
    b = good.copy()
    b[rec + 32 + 8:rec + 32 + 16] = b[rec + 8:rec + 16]  # two tiles write the same bytes
    bad.append(b)
    b = good.copy()
    b[rec:rec + 8] = np.frombuffer(np.uint64(good.size).tobytes(), np.uint8)  # payload outside
    bad.append(b)
    bad.append(good[:-1].copy())
    for b in bad:
        with pytest.raises(lz.LzError) as e:
            lz.entropy_info(b)
        assert e.value.rc == lz.LZ_E_CORRUPT
        with pytest.raises(oracle.OracleError):
            oracle.entropy_decode(b)
