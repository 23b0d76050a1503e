"""Host side of liblz against the oracle (CPU only): encoder, container writer,
validation, statistics, planner, entropy bound, and that the C-ABI library
loads and exports every symbol include/lz.h declares."""
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    import ctypes
    hdrs = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]
    names = set()
    for h in hdrs:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(lz_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    assert len(names) >= 15
    L = ctypes.CDLL(lz.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("thr", [(6, 8, 10, 12), (12, 16, 24, 32), (4, 6, 8, 10)])
def test_exact_encoder_equals_oracle(thr):
    """With whole hash chains the library parse is the exhaustive greedy
    parse: the archive is byte-identical to the oracle's."""
    x = synth.zipf_text(24000, seed=21)
    bounds = (512, 4096, 16384)
    a = lz.encode(x, 12, thr, bounds, max_chain=0, depth_passes=0)
    ll, ml, sr, lit = oracle.encode(x, 12, thr, bounds)
    b = oracle.write_archive(x.size, 12, ll, ml, sr, lit, min_match=min(thr), thr=thr, bounds=bounds)
    assert np.array_equal(a, b)


def test_exact_encoder_fastq_and_binary():
    for x in (synth.fastq(30000, seed=7), synth.random_bytes(5000, 3),
              np.zeros(7000, np.uint8), np.tile(np.arange(7, dtype=np.uint8), 900)):
        for lb in (8, 12):
            a = lz.encode(x, lb, (4, 5, 6, 7), (64, 1024, 4096), max_chain=0, depth_passes=0)
            ll, ml, sr, lit = oracle.encode(x, lb, (4, 5, 6, 7), (64, 1024, 4096))
            b = oracle.write_archive(x.size, lb, ll, ml, sr, lit, min_match=4, thr=(4, 5, 6, 7),
                                     bounds=(64, 1024, 4096))
            assert np.array_equal(a, b)


def _lcp_table(x):
    """lcp[i, j] = length of the longest common prefix of x[i:] and x[j:]."""
    n = x.size
    L = np.zeros((n + 1, n + 1), dtype=np.int32)
    for i in range(n - 1, -1, -1):
        L[i, :n] = np.where(x[i] == x, L[i + 1, 1:n + 1] + 1, 0)
    return L


def _byte_depths(arc):
    """Dependency depth of every output byte from the oracle: literal bytes
    0, match bytes their match's depth."""
    T = oracle.tokens(arc)
    lv, _ = oracle.levels(arc)
    n = int(oracle.info(arc)["n"])
    d = np.zeros(n, dtype=np.int64)
    for t in range(T["dst"].size):
        m0 = int(T["dst"][t] + T["lit_len"][t])
        d[m0:m0 + int(T["mlen"][t])] = int(lv[t])
    return T, d


@pytest.mark.parametrize("kind", ["fastq", "zipf", "runs"])
def test_depth_aware_ties_choose_shallowest_then_nearest(kind):
    """One block, exhaustive chains: match lengths equal the oracle's
    exhaustive greedy parse, and every match's source is, among all valid
    candidates of its length (brute force over every earlier position), one
    of lowest resulting depth (1 + the deepest byte it reads, its own output
    excluded), and the nearest of those."""
    if kind == "fastq":
        x = synth.fastq(4096, seed=31)
    elif kind == "zipf":
        x = synth.zipf_text(4096, seed=32, vocab=64)
    else:
        x = np.frombuffer(b"".join(b"@R.%d %d/1\nACGTTGCAAC\n+\nIIIIIIII\n" % (i, i) for i in range(90)),
                          np.uint8)[:4096].copy()
    n = x.size
    thr, bounds = (4, 5, 6, 8), (64, 512, 2048)
    arc = lz.encode(x, 12, thr, bounds, max_chain=0, depth_passes=1)
    assert np.array_equal(oracle.decode(arc), x)
    ll, ml, sr, lit = oracle.encode(x, 12, thr, bounds)
    T, dep = _byte_depths(arc)
    assert T["lit_len"].tolist() == [int(v) for v in ll] and T["mlen"].tolist() == [int(v) for v in ml]
    lcp = _lcp_table(x)
    ties = 0
    for t in range(T["dst"].size):
        L = int(T["mlen"][t])
        if L == 0:
            continue
        pos = int(T["dst"][t] + T["lit_len"][t])
        s = np.arange(pos)
        cap = np.minimum(lcp[s, pos], n - pos)
        d = pos - s
        cls = np.where(d < bounds[0], 0, np.where(d < bounds[1], 1, np.where(d < bounds[2], 2, 3)))
        valid = cap >= np.array(thr)[cls]
        assert cap[valid].max() == L
        cands = s[valid & (cap == L)]
        cdep = np.array([1 + dep[c:min(c + L, pos)].max() for c in cands])
        best = cands[cdep == cdep.min()].max()
        ties += int(cands.size > 1)
        assert int(T["src"][t]) == best, (t, pos, L, int(T["src"][t]), best)
    assert ties > 5


def test_depth_aware_passes_keep_lengths_and_cut_depth():
    """Several blocks, exhaustive chains: 1 and 2 depth-aware passes keep the
    exhaustive parse's lengths (equal to the oracle's), round-trip, and do not
    deepen the plan of header-heavy records."""
    x = synth.fastq(64_000, seed=33)
    thr, bounds = (5, 6, 8, 10), (4096, 65536, 1 << 20)
    ll, ml, sr, lit = oracle.encode(x, 12, thr, bounds)
    depths = []
    for dp in (0, 1, 2):
        arc = lz.encode(x, 12, thr, bounds, max_chain=0, depth_passes=dp)
        assert np.array_equal(oracle.decode(arc), x)
        T = oracle.tokens(arc)
        assert T["lit_len"].tolist() == [int(v) for v in ll] and T["mlen"].tolist() == [int(v) for v in ml]
        depths.append(oracle.levels(arc)[1])
    assert depths[1] <= depths[0] and depths[2] <= depths[0]
    assert depths[1] < depths[0]


def test_chain_limited_encoder_roundtrips_and_keeps_invariants():
    x = synth.fastq(1 << 20, seed=3)
    for thr in (lz.BASE_THR, lz.TUNED_THR):
        arc = lz.encode(x, 16, thr, max_chain=16)
        assert np.array_equal(oracle.decode(arc), x)
        T = oracle.tokens(arc)
        m = T["mlen"] > 0
        ms = T["dst"] + T["lit_len"]
        d = ms[m] - T["src"][m]
        B = lz.BOUNDS_CFG
        cls = np.where(d < B[0], 0, np.where(d < B[1], 1, np.where(d < B[2], 2, 3)))
        assert np.all(T["mlen"][m] >= np.array(thr)[cls])


def test_segmented_encoder():
    x = synth.zipf_text(300_000, seed=5)
    arc = lz.encode(x, 14, segment=1 << 16)
    assert np.array_equal(oracle.decode(arc), x)
    T = oracle.tokens(arc)
    m = T["mlen"] > 0
    ms = T["dst"] + T["lit_len"]
    assert np.all(T["src"][m] // (1 << 16) == ms[m] // (1 << 16))


def test_build_archive_equals_oracle_writer():
    n = 1 << 21
    ll, ml, sr, lit = synth.geo_tokens(n, 128, seed=2)
    for lb in (12, 14, 16, 20):
        a = lz.build_archive(n, lb, ll, ml, sr, lit)
        b = oracle.write_archive(n, lb, ll, ml, sr, lit)
        assert np.array_equal(a, b)


def test_oracle_archives_validate_in_library():
    x = synth.zipf_text(50000, seed=9)
    ll, ml, sr, lit = oracle.encode(x[:8000], 10, (4, 4, 4, 4))
    arc = oracle.write_archive(8000, 10, ll, ml, sr, lit)
    inf = lz.archive_info(arc)
    assert inf["n"] == 8000 and inf["n_tok"] == len(ll)


def test_corrupt_archives_rejected():
    x = synth.zipf_text(40000, seed=2)
    arc = lz.encode(x, 12)
    rng = np.random.default_rng(0)
    with pytest.raises(lz.LzError):
        lz.archive_info(arc[:100])
    with pytest.raises(lz.LzError):
        lz.archive_info(arc[:-32])
    n_bad = 0
    for trial in range(200):
        b = arc.copy()
        i = int(rng.integers(0, b.size))
        b[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        o = oracle.decode_rc(b)
        try:
            lz.archive_info(b)
            lib_ok = True
        except lz.LzError:
            lib_ok = False
        # both readers agree on validity; a flipped literal byte stays valid
        assert lib_ok == (o == 0), (trial, i)
        n_bad += (not lib_ok)
    assert n_bad > 10


def test_stats_match_oracle_tokens():
    x = synth.fastq(500_000, seed=4)
    arc = lz.encode(x, 16, lz.TUNED_THR)
    inf = lz.archive_info(arc)
    T = oracle.tokens(arc)
    m = T["mlen"] > 0
    assert inf["n_match"] == int(m.sum())
    assert inf["match_bytes"] == int(T["mlen"].sum())
    assert inf["mean_match"] == pytest.approx(T["mlen"][m].mean())
    assert inf["frac_lt32"] == pytest.approx((T["mlen"][m] < 32).mean())
    assert int(inf["hist"].sum()) == inf["n_match"]


def test_plan_equals_oracle_levels():
    x = synth.zipf_text(400_000, seed=6)
    for lb in (12, 14):
        arc = lz.encode(x, lb)
        a, amx = lz.plan(arc)
        b, bmx = oracle.levels(arc)
        assert amx == bmx and np.array_equal(a, b)
    n = 1 << 21
    ll, ml, sr, lit = synth.geo_tokens(n, 64, seed=8)
    arc = lz.build_archive(n, 14, ll, ml, sr, lit)
    a, amx = lz.plan(arc)
    b, bmx = oracle.levels(arc)
    assert amx == bmx and np.array_equal(a, b)


def test_entropy_equals_oracle():
    for x in (synth.zipf_text(300_000, seed=1), synth.fastq(300_000, seed=2)):
        arc = lz.encode(x, 16)
        a, pa = lz.entropy_size(arc)
        b, pb = oracle.entropy_size(arc)
        assert a == pytest.approx(b, abs=8)
        assert np.allclose(pa, pb, atol=2)


def test_fnv_agrees_with_oracle():
    for n in (0, 1, 7, 1000, 65537):
        x = synth.random_bytes(n, n + 1)
        assert lz.fnv1a64(x) == oracle.fnv1a64(x)


def test_params_rejected():
    x = synth.zipf_text(1000, seed=1)
    with pytest.raises(lz.LzError):
        lz.encode(x, 3)
    with pytest.raises(lz.LzError):
        lz.encode(x, 12, thr=(0, 1, 1, 1))
    with pytest.raises(lz.LzError):
        lz.encode(x, 12, bounds=(100, 50, 200))
    with pytest.raises(lz.LzError):
        lz.encode(x, 12, segment=1000)


def test_block_features_equal_oracle():
    from oracle import mlp_ref
    for x in (synth.zipf_text(700_000, seed=3), synth.fastq(600_000, seed=4)):
        arc = lz.encode(x, 16, (4, 4, 4, 4), max_chain=16)
        F = lz.block_features(arc, lz.BOUNDS_CFG)
        R = mlp_ref.block_features(oracle.tokens(arc), x.size, 16, lz.BOUNDS_CFG)
        assert np.allclose(F, R, rtol=1e-6, atol=1e-7)


def test_block_stats_single_block_equal_oracle_entropy():
    for x in (synth.zipf_text(60_000, seed=5), synth.fastq(50_000, seed=6)):
        arc = lz.encode(x, 16, lz.BASE_THR)
        ent, nt, nm, mb = lz.block_stats(arc)
        tot, parts = oracle.entropy_size(arc)
        assert ent.size == 1
        assert ent[0] == pytest.approx(parts[0] + parts[1] + parts[2] + parts[3] + parts[4] + parts[6], abs=1e-6)
        T = oracle.tokens(arc)
        assert nt[0] == T["dst"].size and nm[0] == int((T["mlen"] > 0).sum()) and mb[0] == int(T["mlen"].sum())


def test_blockwise_encoder_uniform_equals_plain():
    """Per-block thresholds that are all equal give the plain parse (same
    tokens; only the per-block info bytes are added)."""
    x = synth.fastq(300_000, seed=8)
    nb = (x.size + (1 << 14) - 1) >> 14
    for thr in (lz.BASE_THR, lz.TUNED_THR):
        a = lz.encode_blockwise(x, np.array([thr] * nb, np.uint32), np.full(nb, 1, np.uint8), log2_bs=14)
        b = lz.encode(x, 14, thr)
        ta, tb = oracle.tokens(a), oracle.tokens(b)
        for k in ta:
            assert np.array_equal(ta[k], tb[k])
        assert np.array_equal(oracle.decode(a), x)


def test_device_buffer_alignment_rejected_before_any_device_call():
    """lz_device_open refuses a device buffer that is not 256-byte aligned
    (kernels update words in it atomically); the check runs before the
    archive is validated or any HIP call is made."""
    import ctypes
    x = synth.zipf_text(4096, seed=2)
    arc = lz.encode(x, 12, (4, 4, 4, 4))
    h = ctypes.c_void_p()
    rc = lz.lib().lz_device_open(arc.ctypes.data, arc.size, ctypes.c_void_p(0x10001), 1 << 30, None,
                                 ctypes.byref(h))
    assert rc == lz.LZ_E_INVAL and not h.value
    assert b"256-byte aligned" in lz.lib().lz_last_error()
