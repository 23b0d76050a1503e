"""GPU parity for the literal-sourced matches the parse copies itself: the
plan's choice is pinned by a count derived from the oracle's tokens
and dependency depths, and the bytes those matches write after the parse
launch alone are compared with the input."""
import numpy as np
import pytest

import oracle
import synth
from fused_ref import literal_sourced
from paper_2607_18541_amd import lz

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


CASES = [
    ("fastq 4 MiB 12/16/24/32", lambda: synth.fastq(4 << 20, seed=7), lz.TUNED_THR, 16),
    ("fastq 4 MiB 6/8/10/12", lambda: synth.fastq(4 << 20, seed=7), lz.BASE_THR, 16),
    ("zipf 1 MiB 6/8/10/12, 16 KiB blocks", lambda: synth.zipf_text(1 << 20, seed=1), lz.BASE_THR, 14),
]


@pytest.mark.parametrize("label,gen,thr,lb", CASES, ids=[c[0] for c in CASES])
def test_parse_copies_literal_sourced_matches(label, gen, thr, lb):
    dev = _dev()
    x = gen()
    arc = lz.encode(x, lb, thr)
    mask, md, ml = literal_sourced(arc)
    da = lz.DeviceArchive(arc, device=dev)
    print(f"[{label}] fused {da.fused} matches, {da.fused_bytes} bytes; oracle count {int(mask.sum())}", flush=True)
    assert da.fused == int(mask.sum()) and da.fused > 0
    assert da.fused_bytes == int(ml[mask].sum())
    exp = torch.from_numpy(x).to(dev)
    for pg, pu in ((64, 2), (32, 1), (16, 4), (8, 2)):
        # the parse launch alone: every literal and every literal-sourced match is final
        out = torch.zeros(da.n, dtype=torch.uint8, device=dev)
        da.decode_stage(out, 1, parse_G=pg, parse_unroll=pu)
        da.check()
        got = out.cpu().numpy()
        idx = np.concatenate([np.arange(a, a + b) for a, b in zip(md[mask], ml[mask])])
        assert np.array_equal(got[idx], x[idx]), f"{label} parse {pg}/{pu}: literal-sourced match bytes differ"
        # then the depth passes complete the output
        da.decode_stage(out, 2, parse_G=pg, parse_unroll=pu)
        da.check()
        assert torch.equal(out, exp), f"{label} parse {pg}/{pu}: decode differs"
    # a full decode, and the oracle's own decode of the same archive
    got = da.decode(torch.empty(da.n, dtype=torch.uint8, device=dev))
    assert torch.equal(got, exp)
    assert np.array_equal(oracle.decode(arc), x)
    da.close()


def test_generated_stream_literal_sourced_count():
    """Generated tokens read sources at least 64 KiB back from a stream whose
    first 64 KiB is literal, so its depth-1 matches mostly read that prefix:
    the plan's count equals the oracle-derived one and the decode is exact."""
    dev = _dev()
    n = 1 << 22
    ll, mlen, src, lit = synth.geo_tokens(n, 64, seed=9)
    arc = lz.build_archive(n, 14, ll, mlen, src, lit)
    mask, _, _ = literal_sourced(arc)
    da = lz.DeviceArchive(arc, device=dev)
    print(f"[geo m=64] fused {da.fused}, oracle count {int(mask.sum())}", flush=True)
    assert da.fused == int(mask.sum())
    exp = torch.from_numpy(oracle.exec_tokens(n, ll, mlen, src, lit)).to(dev)
    got = da.decode(torch.empty(n, dtype=torch.uint8, device=dev))
    assert torch.equal(got, exp)
    da.close()
