"""Read-level seek on the GPU: record id -> block -> the record's bytes,
equal to the record taken from the input (a plain split into records of
`lines` lines), for first, last, random and block-straddling records, with
blocks smaller than a record, and on an archive encoded in segments."""
import numpy as np
import pytest

import synth
from paper_2607_18541_amd import lz

from test_records_host import record_starts

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("kind,log2_bs,lines,segment", [("fastq", 14, 4, 0), ("fastq", 6, 4, 0),
                                                        ("fastq", 16, 4, 1 << 20), ("zipf", 12, 1, 0)])
def test_seek_records_equal_input(kind, log2_bs, lines, segment):
    dev = _dev()
    x = synth.fastq(3 << 20, seed=8) if kind == "fastq" else synth.zipf_text(1 << 20, seed=9)
    if log2_bs < 10:
        x = x[:200_000].copy()
    arc = lz.encode(x, log2_bs, lz.TUNED_THR, segment=segment)
    da = lz.DeviceArchive(arc, device=dev)
    idx = lz.ReadIndex(x, log2_bs, lines)
    starts = record_starts(x, lines) + [x.size]
    R = idx.records
    assert R == len(starts) - 1
    rng = np.random.default_rng(5)
    ids = [0, 1, R - 2, R - 1] + [int(v) for v in rng.integers(0, R, 60)]
    # records that cross a block boundary
    bs = 1 << log2_bs
    cross = [r for r in range(R) if starts[r] // bs != (starts[r + 1] - 1) // bs]
    ids += cross[:10] + cross[-5:]
    out = torch.empty(1 << 16, dtype=torch.uint8, device=dev)
    for r in ids:
        print("[%s bs=2^%d seg=%d] record %d" % (kind, log2_bs, segment, r), flush=True)
        got = idx.seek(da, r, out=out)
        assert bytes(got.cpu().numpy()) == bytes(x[starts[r]:starts[r + 1]]), r
    with pytest.raises(lz.LzError) as e:
        idx.seek(da, R)
    assert e.value.rc == lz.LZ_E_RANGE
    small = torch.empty(4, dtype=torch.uint8, device=dev)
    with pytest.raises(lz.LzError) as e:
        idx.seek(da, 0, out=small)
    assert e.value.rc == lz.LZ_E_NOMEM
    da.close()
