"""The tile-rANS entropy stage on the GPU: a coded container opened on the
device is entropy-decoded (one wave per tile) into exactly the container the
oracle's decoder gives, byte for byte; the full pipeline (entropy stage, then
the match phase) reproduces the input, also when the stage is re-run; a
stream corrupted past the host checks is reported, not decoded."""
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


def _inputs():
    n = 1 << 21
    ll, ml, sr, lit = synth.geo_tokens(n, 64, seed=7, lit_prefix=4096, min_back=1)
    geo_arc = lz.build_archive(n, 14, ll, ml, sr, lit)
    return [("fastq", synth.fastq(8 << 20, seed=3), None, 16), ("zipf", synth.zipf_text(3 << 20, seed=1), None, 12),
            ("geo", oracle.exec_tokens(n, ll, ml, sr, lit), geo_arc, 14),
            ("random", synth.random_bytes(700_000, 2), None, 16), ("constant", np.full(500_000, 65, np.uint8), None, 16),
            ("tiny", np.frombuffer(b"abcab", np.uint8).copy(), None, 4)]


@pytest.mark.parametrize("case", range(6))
def test_entropy_stage_matches_oracle_and_pipeline_decodes(case):
    dev = _dev()
    name, x, arc, lb = _inputs()[case]
    if arc is None:
        arc = lz.encode(x, lb, lz.TUNED_THR)
    coded = lz.entropy_encode(arc)
    expect_arc = oracle.entropy_decode(coded)
    assert np.array_equal(expect_arc, arc)
    print("[%s] %d B container, %d B coded, %s" % (name, arc.size, coded.size, lz.entropy_info(coded)), flush=True)
    da = lz.DeviceArchive(coded, device=dev, coded=True)
    creg = (coded.size + 16 + 255) & ~255
    region = da.buf[creg:creg + arc.size]
    assert torch.equal(region, torch.from_numpy(expect_arc).to(dev)), "entropy stage differs from the oracle"
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = da.decode()
    assert torch.equal(out[:x.size], xt)
    # full pipeline again: wipe the archive region, re-run the stage, decode
    region.fill_(0xCC)
    da.entropy_decode_async()
    out2 = torch.empty(max(x.size, 1), dtype=torch.uint8, device=dev)
    da.decode(out2)
    da.check()
    assert torch.equal(out2[:x.size], xt)
    assert torch.equal(region, torch.from_numpy(expect_arc).to(dev))
    assert lz.fnv1a64(out2[:x.size].cpu().numpy()) == oracle.fnv1a64(x)
    da.close()


def test_corrupt_word_stream_is_reported():
    dev = _dev()
    x = synth.fastq(2 << 20, seed=5)
    coded = lz.entropy_encode(lz.encode(x, 16, lz.TUNED_THR))
    nt = int(np.frombuffer(coded[16:20].tobytes(), np.uint32)[0])
    p0 = 192 + 32 * nt
    hit = 0
    for t in range(nt):
        r = 192 + 32 * t
        mode = int(np.frombuffer(coded[r + 28:r + 32].tobytes(), np.uint32)[0])
        pb = int(np.frombuffer(coded[r + 20:r + 24].tobytes(), np.uint32)[0])
        if mode == 1 and pb > 4000:
            po = int(np.frombuffer(coded[r:r + 8].tobytes(), np.uint64)[0])
            coded[p0 + po + pb - 1000] ^= 0x5A  # a word deep in the stream: tables and states stay valid
            hit += 1
            break
    assert hit
    lz.entropy_info(coded)  # passes the host checks
    with pytest.raises(lz.LzError) as e:
        lz.DeviceArchive(coded, device=dev, coded=True)
    assert e.value.rc == lz.LZ_E_CORRUPT
