"""Host side of the learned threshold selector (CPU only): labels and the
decode-time model against a numpy least-squares restatement, inference and
the fallback rule against the float64 reference network, the validation
table, feature normalisation, the selector file, and the learned encoder
(per-block tuples stored and obeyed, decode equal to the input)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp_ref
from paper_2607_18541_amd import lz

TUPLES = np.array([(6, 8, 10, 12), (12, 16, 24, 32), (16, 24, 32, 48), (4, 6, 8, 10), (8, 10, 12, 16),
                   (8, 12, 16, 20), (10, 12, 16, 24), (12, 16, 20, 24), (16, 20, 24, 32), (20, 24, 32, 48),
                   (24, 32, 48, 64), (6, 8, 12, 16), (6, 10, 16, 24), (8, 12, 20, 32), (10, 16, 24, 48),
                   (12, 20, 32, 64)], np.uint32)


def test_labels_follow_the_least_squares_time_model():
    rng = np.random.default_rng(4)
    blocks = np.array([3, 5, 2, 4, 6, 3, 2, 5], np.uint32)
    K, F, T = int(blocks.sum()), blocks.size, 16
    size = rng.uniform(1000, 5000, (K, T))
    counts = rng.integers(10, 4000, (K, T, 3)).astype(np.uint64)
    depths = rng.integers(2, 90, (F, T)).astype(np.uint32)
    true = np.array([2e-5, 5e-5, 1e-7, 4e-3, 2e-2])
    cut = np.concatenate([[0], np.cumsum(blocks)]).astype(np.int64)
    rows, ms = [], []
    for f in range(F):
        for t in range(T):
            c = counts[cut[f]:cut[f + 1], t].sum(axis=0).astype(np.float64)
            r = np.array([c[0], c[1], c[2], depths[f, t], 1.0])
            rows.append(r)
            ms.append(r @ true * (1 + 0.01 * rng.standard_normal()))
    ms = np.array(ms).reshape(F, T)
    coef, J, lab = lz.learn_labels(blocks, size, counts, ms, depths, lam=1.0, fixed=1)
    want = np.maximum(np.linalg.lstsq(np.array(rows), ms.reshape(-1), rcond=None)[0], 0.0)
    assert np.allclose(coef, want, rtol=1e-6, atol=1e-12)
    # J and labels from the fitted model
    for f in range(F):
        for k in range(cut[f], cut[f + 1]):
            tm = np.maximum(coef[0] * counts[k, :, 0] + coef[1] * counts[k, :, 1] + coef[2] * counts[k, :, 2]
                            + (coef[3] * depths[f] + coef[4]) / blocks[f], 1e-12)
            j = size[k] / size[k, 1] + tm / tm[1]
            assert np.allclose(J[k], j, rtol=1e-12)
            assert lab[k] == int(np.argmin(j))
    assert np.allclose(J[:, 1], 2.0)


def _selector(seed=3, confident=None):
    sel = lz.Selector(TUPLES, 1, seed)
    if confident is not None:
        p = sel.params()
        p[-16:] = 0
        p[-16 + confident] = 60.0  # the last-layer bias decides
        sel.params(p)
    return sel


def _reference_choice(sel, F):
    inf = sel.info()
    x = (F.astype(np.float64) - inf["mu"]) / inf["sd"]
    _, _, logits = mlp_ref.forward(sel.params().astype(np.float64), x)
    p = mlp_ref.softmax(logits)
    k = p.argmax(axis=1)
    ok = (p.max(axis=1) >= 0.5) & (inf["val_J"][k] < 1.0)
    return np.where(ok, k, inf["fixed"]), p.max(axis=1), k


def test_choose_matches_reference_network_and_fallback():
    rng = np.random.default_rng(5)
    F = rng.uniform(0, 0.2, (300, 64)).astype(np.float32)
    sel = _selector(7)
    sel.set_norm(F)
    inf = sel.info()
    assert np.allclose(inf["mu"], F.astype(np.float64).mean(axis=0), rtol=1e-5, atol=1e-7)
    assert np.allclose(inf["sd"], F.astype(np.float64).std(axis=0) + 1e-6, rtol=1e-5, atol=1e-7)
    # validation table: mean J of the rows each tuple is predicted for, / (1 + lam)
    J = rng.uniform(1.2, 2.4, (300, 16))
    sel.calibrate(F, J, lam=1.0)
    _, _, k = _reference_choice(sel, F)
    vj = sel.info()["val_J"]
    for t in range(16):
        want = 1.0 if t == 1 else (J[k == t, t].mean() / 2.0 if np.any(k == t) else 9.0)
        assert abs(vj[t] - want) < 1e-5, t
    got, top = sel.choose(F)
    want, wtop, _ = _reference_choice(sel, F)
    assert np.array_equal(got, want)
    assert np.allclose(top, wtop, rtol=1e-5, atol=1e-6)
    # a confident network whose tuple beat the fixed one is followed ...
    sel = _selector(1, confident=5)
    sel.calibrate(F, np.where(np.arange(16) == 5, 1.0, 2.0)[None, :].repeat(300, 0), lam=1.0)
    assert np.all(sel.choose(F)[0] == 5)
    # ... and falls back when its tuple did not beat the fixed one
    sel.calibrate(F, np.full((300, 16), 2.5), lam=1.0)
    assert np.all(sel.choose(F)[0] == 1)


def test_selector_file_round_trip_and_rejection(tmp_path):
    sel = _selector(9)
    rng = np.random.default_rng(1)
    F = rng.uniform(0, 1, (50, 64)).astype(np.float32)
    sel.set_norm(F)
    sel.calibrate(F, rng.uniform(1, 3, (50, 16)))
    path = str(tmp_path / "sel.bin")
    sel.save(path)
    back = lz.Selector(path=path)
    a, b = sel.info(), back.info()
    for key in ("tuples", "mu", "sd", "val_J"):
        assert np.array_equal(a[key], b[key])
    assert a["fixed"] == b["fixed"] and np.array_equal(sel.params(), back.params())
    assert np.array_equal(sel.choose(F)[0], back.choose(F)[0])
    bad = tmp_path / "bad.bin"
    bad.write_bytes(open(path, "rb").read()[:100])
    with pytest.raises(lz.LzError) as e:
        lz.Selector(path=str(bad))
    assert e.value.rc == lz.LZ_E_CORRUPT


@pytest.mark.parametrize("pick", [2, 10])
def test_learned_encode_stores_and_obeys_the_chosen_tuples(pick):
    x = synth.fastq(300_000, seed=12)
    sel = _selector(2, confident=pick)
    sel.calibrate(np.zeros((4, 64), np.float32), np.where(np.arange(16) == pick, 0.5, 2.0)[None, :].repeat(4, 0))
    arc, choice = lz.encode_learned(x, sel, log2_bs=14)
    nb = (x.size + (1 << 14) - 1) >> 14
    assert choice.size == nb and np.all(choice == pick)
    assert np.array_equal(oracle.decode(arc), x)
    # the per-block info bytes hold the tuple index
    a = np.asarray(arc)
    flags = int.from_bytes(a[28:32].tobytes(), "little")
    assert flags & 2
    assert np.all(a[-16 - ((nb + 15) // 16) * 16:][:nb] == pick)
    # every match meets the chosen tuple's threshold for its distance class
    T = oracle.tokens(arc)
    m = T["mlen"] > 0
    d = (T["dst"] + T["lit_len"])[m] - T["src"][m]
    B = lz.BOUNDS_CFG
    cls = np.where(d < B[0], 0, np.where(d < B[1], 1, np.where(d < B[2], 2, 3)))
    last = np.r_[T["blk"][1:] != T["blk"][:-1], True][m]  # a block's last token has an implied length
    assert np.all((T["mlen"][m] >= TUPLES[pick][cls]) | last)


def test_encode_learned_mode_through_params(tmp_path):
    """lz_params.mode = 1 with a selector file gives the archive of
    lz_encode_learned with the same selector, byte for byte; mode 1 without a
    file and modes above 1 are refused."""
    x = synth.fastq(200_000, seed=13)
    sel = _selector(4, confident=10)
    sel.calibrate(np.zeros((4, 64), np.float32), np.where(np.arange(16) == 10, 0.5, 2.0)[None, :].repeat(4, 0))
    path = str(tmp_path / "sel.bin")
    sel.save(path)
    direct, _ = lz.encode_learned(x, sel, log2_bs=14)
    via_params = lz.encode(x, 14, lz.TUNED_THR, mlp_path=path)  # header thresholds: informational
    assert bytes(np.asarray(via_params)) == bytes(np.asarray(direct))
    assert np.array_equal(oracle.decode(via_params), x)
    p = lz.params(14)
    for mode, fname in ((1, None), (2, path.encode())):
        p.mode = mode
        p.mlp_path = fname
        pa, sz = lz.ctypes.c_void_p(), lz.ctypes.c_uint64()
        rc = lz.lib().lz_encode(lz._u8(x).ctypes.data, x.size, lz.ctypes.byref(p), lz.ctypes.byref(pa),
                                lz.ctypes.byref(sz))
        assert rc == lz.LZ_E_INVAL
