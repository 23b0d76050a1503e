"""Batched decode of many uneven archives in one graph launch: every archive's
bytes equal its solo decode and the oracle; the autotuner's choices decode
bit-exactly too."""
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


def _mixed_archives(k, seed):
    sizes = synth.loguniform(k, 4096, 2 << 20, seed)
    arcs, inputs = [], []
    for i, n in enumerate(sizes):
        n = int(n)
        if i % 3 == 0:
            x = synth.zipf_text(n, seed=seed * 1000 + i)
        elif i % 3 == 1:
            x = synth.fastq(n, seed=seed * 1000 + i)
        else:
            ll, ml, sr, lit = synth.geo_tokens(n, 64, seed=seed * 1000 + i, lit_prefix=min(4096, n), min_back=1)
            x = oracle.exec_tokens(n, ll, ml, sr, lit)
        thr = (lz.BASE_THR, lz.TUNED_THR)[i % 2]
        lb = (12, 14, 16)[i % 3]
        if i % 3 == 2:
            arc = lz.build_archive(x.size, lb, ll, ml, sr, lit)
        else:
            arc = lz.encode(x, lb, thr)
        arcs.append(arc)
        inputs.append(x)
    return arcs, inputs


@pytest.mark.parametrize("mix", ["default", "mixed", "flow"])
def test_batch_equals_solo(mix):
    dev = _dev()
    arcs, inputs = _mixed_archives(60, 7)
    das = [lz.DeviceArchive(a, device=dev) for a in arcs]
    outs = [torch.full((max(d.n, 1) + 16,), 0xEE, dtype=torch.uint8, device=dev) for d in das]
    if mix == "default":
        cfgs = None
    elif mix == "mixed":
        # G, unroll, schedule, tail (default), mapping (XCD-contiguous on every
        # other pair), occupancy (default), parse G and unroll (the copy's, or
        # the default wave)
        cfgs = [((16, 32, 64)[i % 3], (1, 2, 4)[i % 3], i % 2, 0, (i // 2) % 2, 0, ((16, 32, 64)[i % 3], 0)[i % 5 == 0],
                 ((1, 2, 4)[i % 3], 0)[i % 5 == 0]) for i in range(len(das))]
    else:
        cfgs = [(32, 2, 0)] * len(das)
    print(f"[batch {mix}] {len(das)} archives", flush=True)
    b = lz.Batch(das, outs, cfgs)
    for rep in range(2):
        b.launch()
        torch.cuda.synchronize()
        for i, (d, x) in enumerate(zip(das, inputs)):
            got = outs[i][:d.n].cpu().numpy()
            assert np.array_equal(got, x), (mix, rep, i, d.n)
            assert bool((outs[i][d.n:] == 0xEE).all().item())
    # equal to the solo decode of the same archive
    for i in (0, 1, 2, len(das) - 1):
        solo = das[i].decode()
        assert torch.equal(solo, outs[i][:das[i].n])
    b.destroy()


def test_batch_packed_unaligned_outputs():
    """Outputs packed back to back in one buffer at odd offsets, 3 guard bytes
    between them: whole-span literal blocks of one archive never touch its
    neighbours' bytes."""
    dev = _dev()
    arcs, inputs = _mixed_archives(24, 11)
    das = [lz.DeviceArchive(a, device=dev) for a in arcs]
    offs, pos = [], 5
    for d in das:
        offs.append(pos)
        pos += max(d.n, 1) + 3
    buf = torch.full((pos + 16,), 0xEE, dtype=torch.uint8, device=dev)
    outs = [buf[o:o + max(d.n, 1)] for o, d in zip(offs, das)]
    print(f"[batch packed] {len(das)} archives, {pos} bytes", flush=True)
    b = lz.Batch(das, outs, None)
    b.launch()
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    for o, d, x in zip(offs, das, inputs):
        assert np.array_equal(host[o:o + d.n], x), (o, d.n)
        assert np.all(host[o + d.n:o + d.n + 3] == 0xEE)
    assert np.all(host[:5] == 0xEE)
    b.destroy()


def test_batch_scratch_alignment_rejected():
    """A batch scratch that is not 256-byte aligned (it holds atomically
    updated words) is refused before anything is recorded or launched."""
    import ctypes
    dev = _dev()
    arcs, _ = _mixed_archives(3, 13)
    das = [lz.DeviceArchive(a, device=dev) for a in arcs]
    outs = [torch.empty(max(d.n, 1), dtype=torch.uint8, device=dev) for d in das]
    hs = (ctypes.c_void_p * len(das))(*[d.h.value for d in das])
    sb = ctypes.c_uint64()
    assert lz.lib().lz_batch_scratch_bytes(len(das), hs, None, ctypes.byref(sb)) == 0
    scratch = torch.empty(sb.value + 512, dtype=torch.uint8, device=dev)
    op = (ctypes.c_void_p * len(das))(*[o.data_ptr() for o in outs])
    caps = np.array([o.numel() for o in outs], dtype=np.uint64)
    b = ctypes.c_void_p()
    rc = lz.lib().lz_batch_create(len(das), hs, op, caps.ctypes.data, None,
                                  ctypes.c_void_p(scratch.data_ptr() + 8), sb.value, None, ctypes.byref(b))
    assert rc == lz.LZ_E_INVAL and not b.value
    for d in das:
        d.close()


def test_autotune_choices_decode_exactly():
    dev = _dev()
    arcs, inputs = _mixed_archives(24, 11)
    das = [lz.DeviceArchive(a, device=dev) for a in arcs]
    outs = [torch.empty(max(d.n, 1), dtype=torch.uint8, device=dev) for d in das]
    cfgs, report = lz.autotune(das, outs, reps=1)
    assert len(report) >= 2 and sum(r["archives"] for r in report) == len(das)
    for r in report:
        assert r["best_ms"] <= r["default_ms"] * 1.0001
    b = lz.Batch(das, outs, cfgs)
    b.launch()
    torch.cuda.synchronize()
    for i, (d, x) in enumerate(zip(das, inputs)):
        assert np.array_equal(outs[i][:d.n].cpu().numpy(), x), i
    b.destroy()


def test_batch_4096_archives():
    """The batched workload's archive count (4096) in one batch graph with the
    default configuration, half Zipf text and half FASTQ-like, the two
    threshold tuples alternating: 4094 archives log-uniform 4 KiB - 256 KiB
    plus two at the distribution's largest size, 16 MiB (the full 7.5 GiB
    mix is checked byte for byte by the batch benchmark).  Every output
    equals its input, and 64 sampled archives equal the oracle's decode."""
    from concurrent.futures import ThreadPoolExecutor
    dev = _dev()
    k = 4096
    sizes = [int(s) for s in synth.loguniform(k - 2, 4096, 256 << 10, 4)] + [16 << 20, 16 << 20]

    def make(i):
        sz = sizes[i]
        x = synth.zipf_text(sz, seed=4000 + i) if i % 2 == 0 else synth.fastq(sz, seed=4000 + i)
        return x, lz.encode(x, 16, (lz.BASE_THR, lz.TUNED_THR)[(i // 2) % 2])

    with ThreadPoolExecutor(8) as pool:  # the encoder's ctypes calls release the GIL
        made = list(pool.map(make, range(k)))
    print("encoded %d archives, %d bytes" % (k, sum(x.size for x, _ in made)), flush=True)
    inputs = [x for x, _ in made]
    arcs = [a for _, a in made]
    das = [lz.DeviceArchive(a, device=dev) for a in arcs]
    outs = [torch.empty(max(d.n, 1), dtype=torch.uint8, device=dev) for d in das]
    b = lz.Batch(das, outs, None)
    b.launch()
    torch.cuda.synchronize()
    print("batch decoded", flush=True)
    for i, (d, x) in enumerate(zip(das, inputs)):
        assert d.n == x.size, i
        assert torch.equal(outs[i][:d.n], torch.from_numpy(x).to(dev)), i
    rng = np.random.default_rng(11)
    for i in list(rng.choice(k - 2, 62, replace=False)) + [k - 2, k - 1]:
        assert np.array_equal(outs[i][:das[i].n].cpu().numpy(), oracle.decode(arcs[i])), int(i)
    b.destroy()
    for d in das:
        d.close()
