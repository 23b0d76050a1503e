"""Pins for the CPU oracle, checked against things other than the oracle itself:
published hash vectors, hand-worked parses, an independent brute-force
(dynamic-programming) formulation of the greedy parse on tiny inputs,
container bytes laid out by hand, closed-form entropies, and a schedule
simulation for the dependency depths."""
import os
import struct

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ FNV-1a 64

def test_fnv_published_vectors():
    n = 0
    with open(os.path.join(GOLD, "fnv1a64_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lit, h = line.rstrip("\n").split("\t")
            data = eval(lit)  # python bytes literal from the fixture
            assert oracle.fnv1a64(data) == int(h, 16), lit
            n += 1
    assert n >= 5


# ---------------------------------------------------------- greedy parse pins

def _cls(d, bounds):
    return 0 if d < bounds[0] else 1 if d < bounds[1] else 2 if d < bounds[2] else 3


def greedy_by_dp(x, bs, thr, bounds):
    """Greedy parse from a longest-common-prefix table (a different
    formulation from the oracle's forward scan): lcp[i][j] is filled from the
    end of the string, then each position takes the longest valid source,
    nearest on ties."""
    x = list(int(v) for v in x)
    n = len(x)
    lcp = np.zeros((n + 1, n + 1), dtype=np.int64)
    for i in range(n - 1, -1, -1):
        for j in range(n - 1, -1, -1):
            if x[i] == x[j]:
                lcp[i, j] = lcp[i + 1, j + 1] + 1
    toks = []
    for b0 in range(0, n, bs):
        end = min(n, b0 + bs)
        pos, run = b0, 0
        while pos < end:
            best = None
            for src in range(pos):
                L = min(int(lcp[src, pos]), end - pos)
                if L >= thr[_cls(pos - src, bounds)]:
                    if best is None or L > best[0] or (L == best[0] and src > best[1]):
                        best = (L, src)
            if best:
                toks.append((run, best[0], best[1]))
                run = 0
                pos += best[0]
            else:
                run += 1
                pos += 1
        if run:
            toks.append((run, 0, 0))
    return toks


def _otoks(x, log2_bs, thr, bounds):
    ll, ml, sr, lit = oracle.encode(np.asarray(x, dtype=np.uint8), log2_bs, thr, bounds)
    return [(int(a), int(b), int(c) if b else 0) for a, b, c in zip(ll, ml, sr)], lit


@pytest.mark.parametrize("seed", range(12))
def test_greedy_matches_dp_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 160))
    alpha = int(rng.integers(1, 5))
    x = rng.integers(0, alpha, size=n).astype(np.uint8)
    # sometimes splice in a repeat to get long matches
    if n > 40 and seed % 2:
        x[n // 2:n // 2 + 20] = x[3:23]
    log2_bs = int(rng.integers(4, 8))
    thr = tuple(sorted(int(v) for v in rng.integers(1, 7, size=4)))
    bounds = (int(rng.integers(1, 8)), int(rng.integers(8, 32)), int(rng.integers(32, 96)))
    got, lit = _otoks(x, log2_bs, thr, bounds)
    want = greedy_by_dp(x, 1 << log2_bs, thr, bounds)
    assert got == want
    # literal stream = the bytes not covered by matches, in order
    pos, lits = 0, []
    for a, b, c in want:
        lits.extend(x[pos:pos + a])
        pos += a + b
    assert np.array_equal(lit, np.array(lits, dtype=np.uint8))


def test_greedy_hand_worked():
    """Parses worked by hand from the definition."""
    B = (4096, 65536, 1 << 20)
    # period-3 text: three literals, then one overlapping match to the end
    got, _ = _otoks(np.frombuffer(b"abcabcabcabc", np.uint8), 4, (3, 3, 3, 3), B)
    assert got == [(3, 9, 0)]
    # run of one byte: a literal then a distance-1 match
    got, _ = _otoks(np.frombuffer(b"aaaaaaaa", np.uint8), 4, (2, 2, 2, 2), B)
    assert got == [(1, 7, 0)]
    # thresholds above any possible length: all literal
    got, _ = _otoks(np.frombuffer(b"aaaaaaaa", np.uint8), 4, (99, 99, 99, 99), B)
    assert got == [(8, 0, 0)]
    # block size 16 cuts the run: each block restarts; the second block can
    # reach back into the first (absolute sources, whole-prefix window)
    got, _ = _otoks(np.frombuffer(b"a" * 20, np.uint8), 4, (2, 2, 2, 2), B)
    assert got == [(1, 15, 0), (0, 4, 15)]
    # distance classes: "wxyz" repeats at distance 4 (class 0, thr 4) and
    # its second copy at distance 8 would be class 1 (thr 5): only the
    # nearest is valid and nearest wins ties anyway
    got, _ = _otoks(np.frombuffer(b"wxyzwxyzwxyz", np.uint8), 4, (4, 5, 5, 5), (5, 64, 128))
    assert got == [(4, 8, 0)]
    # raising the class-0 threshold above 8 forbids the distance-4 source,
    # and nothing else can reach 9
    got, _ = _otoks(np.frombuffer(b"wxyzwxyzwxyz", np.uint8), 4, (9, 9, 9, 9), (5, 64, 128))
    assert got == [(12, 0, 0)]
    # longest wins over nearest: "abcd" at 0, "abc" at 5, then "abcd"
    got, _ = _otoks(np.frombuffer(b"abcdXabcYabcd", np.uint8), 4, (3, 3, 3, 3), B)
    assert got == [(5, 3, 0), (1, 4, 0)]


def test_greedy_invariants_zipf():
    x = synth.zipf_text(12000, seed=11)
    thr, B = (6, 8, 10, 12), (512, 4096, 8192)
    ll, ml, sr, lit = oracle.encode(x, 11, thr, B)
    arc = oracle.write_archive(x.size, 11, ll, ml, sr, lit, min_match=6, thr=thr, bounds=B)
    T = oracle.tokens(arc)
    bs = 1 << 11
    m = T["mlen"] > 0
    mstart = T["dst"] + T["lit_len"]
    assert np.all(T["src"][m] < mstart[m])
    cls = np.array([_cls(int(d), B) for d in (mstart[m] - T["src"][m])])
    assert np.all(T["mlen"][m] >= np.array(thr)[cls])
    # tokens tile each block and never cross a block end
    ends = mstart + T["mlen"]
    assert np.all((ends - 1) // bs == T["dst"] // bs)
    assert np.array_equal(oracle.decode(arc), x)


# ------------------------------------------------------------ container pins

def _hand_archive():
    """Container bytes laid out by hand from the format statement: n = 29,
    one block of 32 bytes holding two tokens, min_match 3.
    token 0: 3 literals "xyz", match code 2 (length 3 + 2 = 5) from 0,
             an overlapping copy -> "xyz" + "xyzxy"
    token 1 (last): 17 literals via code 15 + x16 value 2, then a match of
             the implied length 29 - 8 - 17 = 4 from position 10."""
    lits = b"xyz" + b"ABCDEFGHIJKLMNOPQ"
    n = 3 + 5 + 17 + 4
    hdr = bytearray(128)
    struct.pack_into("<IIQIIII", hdr, 0, 0x314D5A4C, 1, n, 5, 1, 3, 0)
    struct.pack_into("<QQQQ", hdr, 32, 2, 1, 0, len(lits))
    table = struct.pack("<4Q", 0, 0, 0, 0) + struct.pack("<4Q", 2, len(lits), 1, 0)
    body = bytearray(hdr) + table
    def pad(b):
        b += bytes((16 - len(b) % 16) % 16)
    pad(body)
    body += bytes([0x32, 0xF0])        # cmd: (3,2) then (15,0)
    pad(body)
    body += struct.pack("<H", 2)      # x16: 15 + 2 = 17 literals
    pad(body)
    pad(body)                          # x32: empty
    body += struct.pack("<II", 0, 10)  # src_lo: token 0 from 0, token 1 from 10
    pad(body)
    body += lits
    pad(body)
    body += bytes(16)
    expect = bytearray(b"xyz")
    for i in range(5):
        expect.append(expect[0 + i])
    expect += b"ABCDEFGHIJKLMNOPQ"
    for i in range(4):
        expect.append(expect[10 + i])
    return np.frombuffer(bytes(body), np.uint8), np.frombuffer(bytes(expect), np.uint8)


def test_decode_hand_built_archive():
    arc, expect = _hand_archive()
    assert expect.size == 29
    out = oracle.decode(arc)
    assert bytes(out) == bytes(expect)
    assert bytes(out) == b"xyzxyzxyABCDEFGHIJKLMNOPQCDEF"


def test_decode_rejects_corruption():
    arc, _ = _hand_archive()
    assert oracle.decode_rc(arc) == 0
    bad = arc.copy(); bad[0] ^= 1
    assert oracle.decode_rc(bad) == oracle.OR_E_CORRUPT
    assert oracle.decode_rc(arc[:100]) == oracle.OR_E_CORRUPT
    assert oracle.decode_rc(arc[:-17]) == oracle.OR_E_CORRUPT
    # source not before its destination: token 0 from 3 (its own start)
    i = arc.size - 16 - 32 - 16  # start of src_lo
    bad = arc.copy(); bad[i] = 3
    assert oracle.decode_rc(bad) == oracle.OR_E_CORRUPT
    # last token with a non-zero match code
    j = 128 + 64
    bad = arc.copy(); bad[j + 1] = 0xF1
    assert oracle.decode_rc(bad) == oracle.OR_E_CORRUPT
    # match code that overruns the block
    bad = arc.copy(); bad[j] = 0x3E
    assert oracle.decode_rc(bad) == oracle.OR_E_CORRUPT


@pytest.mark.parametrize("log2_bs", [4, 6, 12, 16])
def test_roundtrip_sizes(log2_bs):
    bs = 1 << log2_bs
    rng = np.random.default_rng(log2_bs)
    for n in [0, 1, bs - 1, bs, bs + 1, 3 * bs]:
        if n > 3000:
            continue
        x = rng.integers(0, 3, size=n).astype(np.uint8)
        ll, ml, sr, lit = oracle.encode(x, log2_bs, (2, 3, 4, 5))
        arc = oracle.write_archive(n, log2_bs, ll, ml, sr, lit)
        assert np.array_equal(oracle.decode(arc), x)
    z = np.zeros(2000, np.uint8)
    ll, ml, sr, lit = oracle.encode(z, log2_bs, (4, 4, 4, 4))
    arc = oracle.write_archive(z.size, log2_bs, ll, ml, sr, lit)
    assert np.array_equal(oracle.decode(arc), z)
    # one literal + distance-1 matches: in each block, the first token reaches
    # back to the previous byte (or is the single literal at position 0)
    T = oracle.tokens(arc)
    m = T["mlen"] > 0
    assert int(T["lit_len"].sum()) == 1
    assert np.all(T["dst"][m] + T["lit_len"][m] - T["src"][m] == 1)


def test_split_matches_unsplit_execution():
    """Cutting a generated token stream at block ends leaves the output as
    executing the uncut stream."""
    n = 200_000
    ll, ml, sr, lit = synth.geo_tokens(n, 64, seed=5, lit_prefix=4096, min_back=4096)
    ref = oracle.exec_tokens(n, ll, ml, sr, lit)
    for lb in (10, 14, 16):
        arc = oracle.write_archive(n, lb, ll, ml, sr, lit)
        assert np.array_equal(oracle.decode(arc), ref)
    # a plain python execution of the first tokens agrees
    out = bytearray()
    lo = 0
    for t in range(40):
        out += bytes(lit[lo:lo + ll[t]]); lo += int(ll[t])
        for i in range(int(ml[t])):
            out.append(out[int(sr[t]) + i])
    assert bytes(ref[:len(out)]) == bytes(out)


# -------------------------------------------------------------- depth pins

def replay_by_depth(arc, lv):
    """Runs the decode the way the GPU schedule does: all literals first, then
    pass p = 1, 2, ... executes every depth-p match at once against a snapshot
    taken before the pass (only a match's own earlier bytes, its period, come
    from the pass itself).  Every byte a match reads from the snapshot must
    already be written, and each depth must be the smallest that allows this.
    Returns the output, which must equal the sequential decode."""
    T = oracle.tokens(arc)
    n = oracle.info(arc)["n"]
    out = np.zeros(n, dtype=np.uint8)
    wdep = np.full(n, -1, dtype=np.int64)  # pass that wrote each byte
    lit = np.frombuffer(oracle.decode(arc).tobytes(), dtype=np.uint8)  # only to fetch literal bytes
    for t in range(T["dst"].size):
        d, L = int(T["dst"][t]), int(T["lit_len"][t])
        out[d:d + L] = lit[d:d + L]
        wdep[d:d + L] = 0
    mx = int(lv.max()) if lv.size else 0
    for p in range(1, mx + 1):
        snap, wsnap = out.copy(), wdep.copy()
        for t in np.nonzero(lv == p)[0]:
            m0 = int(T["dst"][t] + T["lit_len"][t])
            M, s = int(T["mlen"][t]), int(T["src"][t])
            assert M > 0
            deepest = 0
            for i in range(M):
                q = s + i
                if q < m0:
                    assert 0 <= wsnap[q] < p, (t, q)
                    deepest = max(deepest, int(wsnap[q]))
                    out[m0 + i] = snap[q]
                else:
                    out[m0 + i] = out[q]  # own period, written earlier in this match
            assert p == deepest + 1, (t, p, deepest)
            wdep[m0:m0 + M] = p
    assert np.all(lv[T["mlen"] == 0] == 0)
    return out


def test_depth_replay_equals_decode():
    x = synth.zipf_text(6000, seed=4)
    for lb in (9, 10, 12):
        ll, ml, sr, lit = oracle.encode(x, lb, (4, 6, 8, 10), (256, 1024, 4096))
        arc = oracle.write_archive(x.size, lb, ll, ml, sr, lit)
        lv, mx = oracle.levels(arc)
        assert mx == lv.max() and mx >= 2
        assert np.array_equal(replay_by_depth(arc, lv), x)
    # generated stream with overlapping matches (sources from 1 byte back)
    n = 60_000
    ll, ml, sr, lit = synth.geo_tokens(n, 32, seed=9, lit_prefix=512, min_back=1)
    arc = oracle.write_archive(n, 12, ll, ml, sr, lit)
    lv, mx = oracle.levels(arc)
    assert np.array_equal(replay_by_depth(arc, lv), oracle.exec_tokens(n, ll, ml, sr, lit))


def test_levels_omp_decode_equals_sequential():
    """The level-parallel CPU baseline (every depth one parallel loop) gives the
    sequential decode, with self-overlapping matches and deep chains."""
    cases = []
    x = synth.zipf_text(20_000, seed=6)
    ll, ml, sr, lit = oracle.encode(x, 10, (4, 6, 8, 10), (256, 1024, 4096))
    cases.append(oracle.write_archive(x.size, 10, ll, ml, sr, lit))
    n = 200_000
    ll, ml, sr, lit = synth.geo_tokens(n, 32, seed=10, lit_prefix=512, min_back=1)
    cases.append(oracle.write_archive(n, 12, ll, ml, sr, lit))
    for arc in cases:
        prep = oracle.levels_prepare(arc)
        assert prep["max_depth"] >= 2
        out = np.zeros(prep["n"], np.uint8)
        assert oracle.decode_levels_omp(prep, out) >= 1
        assert np.array_equal(out, oracle.decode(arc))


def test_depth_hand_built():
    """Literals 'abcd'; A copies [0,4) -> depth 1; B copies A's bytes -> 2;
    C copies literals again -> 1; D reads B and C -> 3; E overlaps itself
    (period 1) over a literal -> 1.  Block boundaries do not add depth."""
    lit = np.frombuffer(b"abcdz", np.uint8)
    # tokens (lit_len, mlen, src): dst advances by lit_len + mlen
    ll = [4, 0, 0, 0, 1]
    ml = [4, 4, 4, 8, 6]
    sr = [0, 4, 0, 8, 24]  # E: literal 'z' at 24, copies from 24 (period 1)
    for lb in (4, 5, 12):  # 16-byte, 32-byte and single blocks
        n = sum(ll) + sum(ml)
        arc = oracle.write_archive(n, lb, ll, ml, sr, lit, min_match=1)
        T = oracle.tokens(arc)
        lv, mx = oracle.levels(arc)
        out = oracle.decode(arc)
        assert bytes(out) == b"abcd" + b"abcd" * 3 + b"abcdabcd" + b"z" * 7
        # depth of the match covering each output position of A..E
        m0 = T["dst"] + T["lit_len"]
        want = {4: 1, 8: 2, 12: 1, 16: 3, 25: 1}
        for pos, dep in want.items():
            k = np.nonzero((m0 <= pos) & (pos < m0 + T["mlen"]))[0]
            assert k.size == 1 and lv[k[0]] == dep, (lb, pos, lv)
        assert mx == 3


# ------------------------------------------------------------- entropy pins

def _literal_archive(data, log2_bs=16):
    n = len(data)
    return oracle.write_archive(n, log2_bs, [n], [0], [0], np.asarray(data, np.uint8))


def test_entropy_closed_forms():
    # constant bytes: H = 0 -> 0 bytes + table charge 1 + 2*1 per tile
    arc = _literal_archive(np.full(65536, 7, np.uint8))
    tot, parts = oracle.entropy_size(arc)
    assert parts[4] == 3.0
    # two symbols, equally often: exactly one bit each -> N/8 + 1 + 4
    two = np.tile(np.array([1, 2], np.uint8), 32768)
    tot, parts = oracle.entropy_size(_literal_archive(two))
    assert parts[4] == 65536 / 8 + 5
    # all 256 byte values equally often: 8 bits each -> N + 1 + 512
    allv = np.tile(np.arange(256, dtype=np.uint8), 256)
    tot, parts = oracle.entropy_size(_literal_archive(allv))
    assert parts[4] == 65536 + 513
    # two tiles are charged separately
    tot, parts = oracle.entropy_size(_literal_archive(np.full(65537, 3, np.uint8), 17))
    assert parts[4] == 3.0 + 3.0
    # header + table verbatim; one token in cmd (1 symbol) and 4 src planes
    assert parts[5] == 128 + 32 * 2
    assert parts[0] == 3.0 and parts[3] == 12.0
    assert tot == pytest.approx(parts.sum())


# --------------------------------------------------------------- pure copy

def test_purecopy_definition():
    rng = np.random.default_rng(3)
    ref = rng.integers(0, 256, 5000).astype(np.uint8)
    lit = rng.integers(0, 256, 300).astype(np.uint8)
    dst = np.array([0, 100, 2000], np.uint64)
    lo = np.array([0, 10, 20], np.uint64)
    ll = np.array([10, 10, 5], np.uint32)
    src = np.array([4000, 7, 3], np.uint64)
    ml = np.array([90, 1000, 2995], np.uint32)
    out = oracle.purecopy(5000, dst, lo, ll, src, ml, lit, ref)
    exp = np.zeros(5000, np.uint8)
    for t in range(3):
        d = int(dst[t]); a = int(ll[t]); b = int(ml[t])
        exp[d:d + a] = lit[int(lo[t]):int(lo[t]) + a]
        exp[d + a:d + a + b] = ref[int(src[t]):int(src[t]) + b]
    assert np.array_equal(out, exp)


def test_purecopy_hand_worked():
    """Three tokens laid out by hand: literals "ab" then ref[3:7], ref[0:3],
    ref[9:10] give "ab" "3456" "012" "9"."""
    ref = np.frombuffer(b"0123456789", np.uint8).copy()
    lit = np.frombuffer(b"ab", np.uint8).copy()
    dst = np.array([0, 6, 9], np.uint64)
    lo = np.array([0, 2, 2], np.uint64)
    ll = np.array([2, 0, 0], np.uint32)
    src = np.array([3, 0, 9], np.uint64)
    ml = np.array([4, 3, 1], np.uint32)
    out = oracle.purecopy(10, dst, lo, ll, src, ml, lit, ref)
    assert bytes(out) == b"ab34560129"


def test_purecopy_from_decoded_output_reproduces_decode():
    """The Table II control: executing every token against a copy of the
    decoded output (sources no longer wait for each other) reproduces the
    sequential decode, overlapping matches included."""
    n = 1 << 16
    ll, ml, sr, lit = synth.geo_tokens(n, 24, seed=9, lit_prefix=256, min_back=1)
    dec = oracle.exec_tokens(n, ll, ml, sr, lit)
    llv = np.asarray(ll, np.int64)
    mlv = np.asarray(ml, np.int64)
    dst = np.concatenate([[0], np.cumsum(llv + mlv)[:-1]]).astype(np.uint64)
    lo = np.concatenate([[0], np.cumsum(llv)[:-1]]).astype(np.uint64)
    assert (np.asarray(sr, np.int64)[mlv > 0] + mlv[mlv > 0] > (dst + llv.astype(np.uint64))[mlv > 0]).any()
    out = oracle.purecopy(n, dst, lo, ll, sr, ml, lit, dec)
    assert np.array_equal(out, dec)
