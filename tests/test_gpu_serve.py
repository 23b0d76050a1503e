"""Serving loop: requests admitted by slots and memory while others run; every
result is byte-identical to the same range alone (tolerance 0: lossless)."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2607_18541_amd import lz
from test_gpu_range import horizon_by_definition

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("arena_mib,slots", [(256, 64), (40, 3)])
def test_serve_mix_equals_alone(arena_mib, slots):
    dev = _dev()
    x = synth.fastq(24 << 20, seed=5)
    da = lz.DeviceArchive(lz.encode(x, 16, lz.TUNED_THR), device=dev)
    n = da.n
    k = 80
    lens = synth.loguniform(k, 16 << 10, 2 << 20, 17)
    offs = (synth.uniform(k, 18) * (n - lens)).astype(np.uint64)
    srv = lz.Server(da, arena_mib << 20, slots=slots)
    pending = {}
    submitted = 0
    done_order = []
    t_end = time.time() + 120
    # arrivals interleaved with ticks: new requests join while earlier groups run
    while (submitted < k or pending) and time.time() < t_end:
        for _ in range(5):
            if submitted < k:
                rid = srv.submit(int(offs[submitted]), int(lens[submitted]))
                pending[rid] = submitted
                submitted += 1
        srv.tick()
        for rid in list(pending):
            st, _ = srv.status(rid)
            if st == 2:
                i = pending.pop(rid)
                got = srv.result(rid, int(lens[i])).clone()
                done_order.append(i)
                alone = da.decode_range(int(offs[i]), int(lens[i]))
                assert torch.equal(got, alone), i
                assert bytes(got.cpu().numpy()) == bytes(x[int(offs[i]):int(offs[i]) + int(lens[i])])
                srv.release(rid)
        st = srv.stats()
        assert st["arena_used"] <= arena_mib << 20
    assert not pending and len(done_order) == k
    assert srv.stats()["arena_high_water"] <= arena_mib << 20
    srv.destroy()


def test_serve_rejects_oversized_and_out_of_range():
    dev = _dev()
    x = synth.zipf_text(4 << 20, seed=3)
    da = lz.DeviceArchive(lz.encode(x, 14), device=dev)
    srv = lz.Server(da, 1 << 20, slots=2)
    with pytest.raises(lz.LzError):
        srv.submit(da.n - 10, 11)
    with pytest.raises(lz.LzError) as e:
        srv.submit(0, 2 << 20)  # can never fit a 1 MiB arena
    assert e.value.rc == lz.LZ_E_NOMEM
    rid = srv.submit(100, 1000)
    for _ in range(1000):
        srv.tick()
        if srv.status(rid)[0] == 2:
            break
    assert bytes(srv.result(rid, 1000).cpu().numpy()) == bytes(x[100:1100])
    srv.release(rid)
    srv.destroy()


def test_serve_groups_overlap_on_device():
    """Requests arriving one per tick each become a group; with horizon-bounded
    prefix decodes (an archive encoded in 8 MiB segments) the scratch of a
    group is at most a segment, so several groups fit the arena at once and
    a new one is launched while earlier ones still run: at least two groups
    are in flight at some tick.  Every result equals the range decoded alone
    and the input bytes."""
    dev = _dev()
    x = synth.fastq(64 << 20, seed=8)
    da = lz.DeviceArchive(lz.encode(x, 16, lz.TUNED_THR, segment=8 << 20), device=dev)
    n = da.n
    k = 48
    lens = synth.loguniform(k, 2 << 20, 8 << 20, 19).astype(np.int64)
    offs = (synth.uniform(k, 20) * (n - lens)).astype(np.int64)
    srv = lz.Server(da, 512 << 20, slots=64)
    seen_running = 0
    rids = []
    for i in range(k):
        rids.append(srv.submit(int(offs[i]), int(lens[i])))
        srv.tick()
        seen_running = max(seen_running, srv.stats()["running_groups"])
    t_end = time.time() + 60
    while time.time() < t_end and any(srv.status(r)[0] != 2 for r in rids):
        srv.tick()
    st = srv.stats()
    print("max groups in flight: seen %d, server %d; arena high water %d" %
          (seen_running, st["max_running_groups"], st["arena_high_water"]), flush=True)
    assert seen_running >= 2 and st["max_running_groups"] >= 2
    for i, r in enumerate(rids):
        assert srv.status(r)[0] == 2, i
        got = srv.result(r, int(lens[i])).clone()
        assert bytes(got.cpu().numpy()) == bytes(x[int(offs[i]):int(offs[i]) + int(lens[i])]), i
        alone = da.decode_range(int(offs[i]), int(lens[i]))
        assert torch.equal(got, alone), i
        srv.release(r)
    assert srv.stats()["arena_used"] == 0
    srv.destroy()


def test_serve_never_fitting_request_fails_cleanly():
    """A request whose output plus plan scratch exceeds the arena is marked
    failed (state 4) by the tick that meets it, which reports LZ_E_NOMEM; its
    memory is returned at once and its slot on release, and later requests
    are served normally."""
    dev = _dev()
    x = synth.fastq(6 << 20, seed=9)
    da = lz.DeviceArchive(lz.encode(x, 16, lz.TUNED_THR), device=dev)
    n = da.n
    srv = lz.Server(da, 3 << 20, slots=2)
    big = srv.submit(n - (2 << 20), 2 << 20)  # a prefix decode of ~n bytes of scratch cannot fit 3 MiB
    with pytest.raises(lz.LzError) as e:
        for _ in range(10):
            srv.tick()
    assert e.value.rc == lz.LZ_E_NOMEM
    assert srv.status(big)[0] == 4
    assert srv.stats()["arena_used"] == 0
    srv.release(big)
    assert srv.status(big)[0] == 3
    rid = srv.submit(100, 1000)
    for _ in range(1000):
        srv.tick()
        if srv.status(rid)[0] == 2:
            break
    assert bytes(srv.result(rid, 1000).cpu().numpy()) == bytes(x[100:1100])
    srv.release(rid)
    assert srv.stats()["arena_used"] == 0
    srv.destroy()


@pytest.mark.parametrize("arena_mib", [256, 24])
def test_serve_splits_tick_by_horizon(arena_mib):
    """Requests admitted in one tick are split by decode horizon: on an
    archive encoded in 8 MiB segments, requests in different segments become
    different groups launched in the same tick (several groups in flight right
    after it when the arena holds them).  With an arena too small for all of
    them the groups that do not fit go back to the queue and run later.  Every
    result equals the range decoded alone and the input bytes."""
    dev = _dev()
    seg = 8 << 20
    x = synth.fastq(64 << 20, seed=12)
    da = lz.DeviceArchive(lz.encode(x, 16, lz.TUNED_THR, segment=seg), device=dev)
    n = da.n
    k = 24
    lens = synth.loguniform(k, 64 << 10, 1 << 20, 23).astype(np.int64)
    offs = (synth.uniform(k, 24) * (n - lens)).astype(np.int64)
    tk = oracle.tokens(da.arc)
    horizons = {horizon_by_definition(tk, int(o), int(o + L)) for o, L in zip(offs, lens)}
    assert len(horizons) >= 4
    srv = lz.Server(da, arena_mib << 20, slots=64)
    rids = [srv.submit(int(offs[i]), int(lens[i])) for i in range(k)]
    srv.tick()
    first = srv.stats()["running_groups"]
    finished = list(srv.completed())
    t_end = time.time() + 60
    while time.time() < t_end and len(finished) < k:
        srv.tick()
        finished += srv.completed()
    # the completion queue names every request once
    assert sorted(finished) == sorted(rids)
    st = srv.stats()
    print("groups after the first tick %d, horizons %d, max in flight %d, arena high water %d" %
          (first, len(horizons), st["max_running_groups"], st["arena_high_water"]), flush=True)
    if arena_mib == 256:
        assert first == len(horizons)
    else:
        assert 1 <= first < len(horizons)
    assert st["arena_high_water"] <= arena_mib << 20
    for i, r in enumerate(rids):
        assert srv.status(r)[0] == 2, i
        got = srv.result(r, int(lens[i])).clone()
        assert bytes(got.cpu().numpy()) == bytes(x[int(offs[i]):int(offs[i]) + int(lens[i])]), i
        assert torch.equal(got, da.decode_range(int(offs[i]), int(lens[i]))), i
        srv.release(r)
    assert srv.stats()["arena_used"] == 0
    srv.destroy()
