"""Read index (CPU only): per block, the id and offset of the first record
starting in it or later, against a plain split of the input into records of
`lines` lines; file round trip and rejection."""
import numpy as np
import pytest

import synth
from paper_2607_18541_amd import lz


def record_starts(x, lines):
    """Offsets of every record start: 0, then just after every lines-th newline."""
    nl = np.nonzero(np.asarray(x) == ord("\n"))[0] + 1
    starts = [0] + [int(p) for p in nl[lines - 1::lines] if p < x.size]
    return starts if x.size else []


def expected_blocks(x, log2_bs, lines):
    starts = record_starts(x, lines)
    n = x.size
    nb = (n + (1 << log2_bs) - 1) >> log2_bs
    out = []
    for b in range(nb):
        i = int(np.searchsorted(starts, b << log2_bs))
        out.append((i, starts[i]) if i < len(starts) else (len(starts), n))
    return out, len(starts)


CASES = [("fastq", 14, 4), ("fastq", 4, 4), ("zipf", 12, 1), ("no-final-newline", 6, 2), ("empty", 8, 4),
         ("one-line", 8, 3)]


def _input(kind):
    if kind == "fastq":
        return synth.fastq(200_000, seed=4)
    if kind == "zipf":
        return synth.zipf_text(100_000, seed=2)
    if kind == "no-final-newline":
        return np.frombuffer(b"a\nbb\nccc\ndddd\neeeee\nf", np.uint8).copy()
    if kind == "empty":
        return np.zeros(0, np.uint8)
    return np.frombuffer(b"no newline at all in this one", np.uint8).copy()


@pytest.mark.parametrize("kind,log2_bs,lines", CASES)
def test_index_matches_plain_record_split(kind, log2_bs, lines):
    x = _input(kind)
    idx = lz.ReadIndex(x, log2_bs, lines)
    want, records = expected_blocks(x, log2_bs, lines)
    assert idx.records == records
    for b, (fid, foff) in enumerate(want):
        assert idx.block(b) == (fid, foff), b


def test_index_file_round_trip(tmp_path):
    x = synth.fastq(50_000, seed=6)
    idx = lz.ReadIndex(x, 10, 4)
    p = str(tmp_path / "i.bin")
    idx.save(p)
    back = lz.ReadIndex(path=p)
    assert back.records == idx.records
    nb = (x.size + 1023) >> 10
    assert [back.block(b) for b in range(nb)] == [idx.block(b) for b in range(nb)]
    bad = tmp_path / "bad.bin"
    good = open(p, "rb").read()
    bad.write_bytes(good[:40])
    with pytest.raises(lz.LzError) as e:
        lz.ReadIndex(path=str(bad))
    assert e.value.rc == lz.LZ_E_CORRUPT
    # a size field that claims a huge input (and so a huge table) is refused
    # before anything is allocated for it
    huge = bytearray(good)
    huge[8:16] = (1 << 62).to_bytes(8, "little")
    huge[32:40] = ((1 << 62) >> 10).to_bytes(8, "little")
    bad.write_bytes(bytes(huge))
    with pytest.raises(lz.LzError) as e:
        lz.ReadIndex(path=str(bad))
    assert e.value.rc == lz.LZ_E_CORRUPT
    # record offsets that go backwards are refused
    nbk = int.from_bytes(good[32:40], "little")
    offs = np.frombuffer(good[40 + 8 * nbk:], np.uint64).copy()
    if nbk > 2:
        offs[2] = 0 if offs[1] > 0 else offs[2]
        if offs[1] > 0:
            bad.write_bytes(good[:40 + 8 * nbk] + offs.tobytes())
            with pytest.raises(lz.LzError) as e:
                lz.ReadIndex(path=str(bad))
            assert e.value.rc == lz.LZ_E_CORRUPT
