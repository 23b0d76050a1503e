"""ctypes binding of liblz (include/lz.h): argument marshalling only.

Every step of encode, plan and decode runs in the native library; device
memory comes from torch tensors (``.data_ptr()``) and streams from
``torch.cuda.current_stream().cuda_stream``.  If ``liblz.so`` is missing this
module raises on first use -- there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblz.so")
_LIB = None

LZ_OK, LZ_E_INVAL, LZ_E_CORRUPT, LZ_E_RANGE, LZ_E_NOMEM, LZ_E_HIP, LZ_E_BUSY = 0, -1, -2, -3, -4, -5, -6

BOUNDS_CFG = (4096, 65536, 1 << 20)
BASE_THR = (6, 8, 10, 12)
TUNED_THR = (12, 16, 24, 32)

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_p64 = ctypes.POINTER(ctypes.c_uint64)


class LzError(RuntimeError):
    def __init__(self, rc, what):
        msg = lib().lz_last_error().decode(errors="replace")
        super().__init__(f"{what} failed ({rc}): {msg}")
        self.rc = rc


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("log2_bs", _u32), ("thr", _u32 * 4), ("bound", _u64 * 3), ("max_chain", _u32),
                ("n_threads", _u32), ("segment", _u64), ("progress", PROGRESS_FN), ("progress_user", ctypes.c_void_p),
                ("depth_passes", _u32), ("mode", _u32), ("mlp_path", ctypes.c_char_p), ("depth_cap", _u32)]


class Info(ctypes.Structure):
    _fields_ = [("n", _u64), ("n_blocks", _u64), ("n_tok", _u64), ("n_lit", _u64), ("n_match", _u64),
                ("match_bytes", _u64), ("archive_bytes", _u64), ("log2_bs", _u32), ("min_match", _u32),
                ("thr", _u32 * 4), ("bound", _u64 * 3), ("mean_match", ctypes.c_double),
                ("frac_lt32", ctypes.c_double), ("coverage", ctypes.c_double), ("src_bytes", _u64),
                ("hist", (_u64 * 16) * 4)]


class DecodeCfg(ctypes.Structure):
    _fields_ = [("G", _u32), ("unroll", _u32), ("schedule", _u32), ("tail", _u32), ("mapping", _u32),
                ("occupancy", _u32), ("parse_G", _u32), ("parse_unroll", _u32)]


class TuneReport(ctypes.Structure):
    _fields_ = [("min_bytes", _u64), ("max_bytes", _u64), ("bytes", _u64), ("archives", _u32),
                ("best", DecodeCfg), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "lz_params_default": (ctypes.c_int, [ctypes.POINTER(Params)]),
            "lz_encode": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Params), ctypes.POINTER(_vp), _p64]),
            "lz_encode_blockwise": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Params), _vp, _vp,
                                                   ctypes.POINTER(_vp), _p64]),
            "lz_build_archive": (ctypes.c_int, [_u64, _u32, _u32, _u64, _vp, _vp, _vp, _vp, _u64,
                                                ctypes.POINTER(_vp), _p64]),
            "lz_free": (None, [_vp]),
            "lz_archive_info": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Info)]),
            "lz_entropy_size": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(ctypes.c_double), _vp]),
            "lz_plan": (ctypes.c_int, [_vp, _u64, _vp, ctypes.POINTER(_u32)]),
            "lz_fnv1a64": (_u64, [_vp, _u64, _u64]),
            "lz_last_error": (ctypes.c_char_p, []),
            "lz_device_bytes": (ctypes.c_int, [_vp, _u64, _p64]),
            "lz_device_open": (ctypes.c_int, [_vp, _u64, _vp, _u64, _vp, ctypes.POINTER(_vp)]),
            "lz_decode_device": (ctypes.c_int, [_vp, _vp, _u64, ctypes.POINTER(DecodeCfg), _vp]),
            "lz_decode_device_stage": (ctypes.c_int, [_vp, _vp, _u64, ctypes.POINTER(DecodeCfg), ctypes.c_int, _vp]),
            "lz_device_check": (ctypes.c_int, [_vp, _vp]),
            "lz_device_n": (_u64, [_vp]),
            "lz_device_levels": (_u32, [_vp]),
            "lz_device_fused": (_u64, [_vp, _p64]),
            "lz_device_close": (None, [_vp]),
            "lz_range_plan_create": (ctypes.c_int, [_vp, _u64, _vp, _vp, ctypes.POINTER(_vp)]),
            "lz_range_plan_scratch_bytes": (_u64, [_vp]),
            "lz_range_plan_levels": (_u64, [_vp]),
            "lz_range_plan_closure_bytes": (_u64, [_vp]),
            "lz_range_plan_prefix_bytes": (_u64, [_vp]),
            "lz_range_plan_horizon": (_u64, [_vp]),
            "lz_range_plan_free": (None, [_vp]),
            "lz_range_run": (ctypes.c_int, [_vp, _vp, _vp, _u64, _vp, _vp, _u64, ctypes.POINTER(DecodeCfg), _vp]),
            "lz_range_scratch_bytes": (ctypes.c_int, [_vp, _u64, _u64, _p64]),
            "lz_decode_range": (ctypes.c_int, [_vp, _u64, _u64, _vp, _vp, _u64, _vp]),
            "lz_batch_scratch_bytes": (ctypes.c_int, [_u32, _vp, _vp, _p64]),
            "lz_batch_create": (ctypes.c_int, [_u32, _vp, _vp, _vp, _vp, _vp, _u64, _vp, ctypes.POINTER(_vp)]),
            "lz_batch_launch": (ctypes.c_int, [_vp, _vp]),
            "lz_batch_launches": (_u64, [_vp]),
            "lz_batch_destroy": (None, [_vp]),
            "lz_autotune": (ctypes.c_int, [_u32, _vp, _vp, _vp, _vp, _u64, _vp, _u32, _vp, _vp, _u32,
                                           ctypes.POINTER(_u32)]),
            "lz_serve_create": (ctypes.c_int, [_vp, _vp, _u64, _u32, ctypes.POINTER(DecodeCfg), ctypes.POINTER(_vp)]),
            "lz_serve_submit": (ctypes.c_int, [_vp, _u64, _u64, _p64]),
            "lz_serve_tick": (ctypes.c_int, [_vp, _p64, _p64]),
            "lz_serve_status": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp)]),
            "lz_serve_release": (ctypes.c_int, [_vp, _u64]),
            "lz_serve_completed": (_u64, [_vp, _p64, _u64]),
            "lz_serve_stats": (None, [_vp, _p64, _p64, _p64, _p64]),
            "lz_serve_max_running": (_u64, [_vp]),
            "lz_serve_destroy": (ctypes.c_int, [_vp]),
            "lz_block_features": (ctypes.c_int, [_vp, _u64, _vp, _vp]),
            "lz_block_stats": (ctypes.c_int, [_vp, _u64, _vp, _vp, _vp, _vp]),
            "lz_mlp_param_count": (_u64, []),
            "lz_mlp_forward": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _vp, _vp]),
            "lz_mlp_backward": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "lz_mlp_backward_noalloc": (ctypes.c_int, [_vp, _u32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
            "lz_mlp_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _u64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, _u32, _vp]),
            "lz_selector_create": (ctypes.c_int, [_vp, _u32, _u64, ctypes.POINTER(_vp)]),
            "lz_selector_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
            "lz_selector_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
            "lz_selector_free": (None, [_vp]),
            "lz_selector_params": (ctypes.c_int, [_vp, _vp, _vp]),
            "lz_selector_info": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
            "lz_selector_set_norm": (ctypes.c_int, [_vp, _vp, _u64]),
            "lz_learn_labels": (ctypes.c_int, [_u32, _vp, _u32, _vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
            "lz_selector_train_bytes": (ctypes.c_int, [_u64, _u32, _p64]),
            "lz_selector_train": (ctypes.c_int, [_vp, _vp, _vp, _u64, _u32, _u32, ctypes.c_float, _u64, _vp, _u64, _vp,
                                                 _vp]),
            "lz_selector_calibrate": (ctypes.c_int, [_vp, _vp, _vp, _u64, ctypes.c_double]),
            "lz_selector_choose": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp]),
            "lz_encode_learned": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Params), _vp, ctypes.POINTER(_vp), _p64,
                                                 _vp]),
            "lz_read_index_build": (ctypes.c_int, [_vp, _u64, _u32, _u32, ctypes.POINTER(_vp)]),
            "lz_read_index_free": (None, [_vp]),
            "lz_read_index_records": (_u64, [_vp]),
            "lz_read_index_block": (ctypes.c_int, [_vp, _u64, _p64, _p64]),
            "lz_read_index_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
            "lz_read_index_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
            "lz_seek_record_scratch_bytes": (ctypes.c_int, [_vp, _vp, _u64, _p64]),
            "lz_seek_record": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _p64, _vp]),
            "lz_entropy_encode": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(_vp), _p64]),
            "lz_entropy_info": (ctypes.c_int, [_vp, _u64, _p64, _p64, _vp]),
            "lz_coded_device_bytes": (ctypes.c_int, [_vp, _u64, _p64]),
            "lz_device_open_coded": (ctypes.c_int, [_vp, _u64, _vp, _u64, _vp, ctypes.POINTER(_vp)]),
            "lz_entropy_decode_device": (ctypes.c_int, [_vp, _vp]),
            "lz_purecopy_device": (ctypes.c_int, [_u64, _vp, _vp, _vp, _vp, _vp, _u64, _vp, _vp, _u64, _vp,
                                                  _u64, _vp, _u64, ctypes.POINTER(DecodeCfg), _vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _u8(a):
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def _take_archive(pa, size):
    try:
        return np.ctypeslib.as_array(ctypes.cast(pa, ctypes.POINTER(ctypes.c_uint8)), (size,)).copy()
    finally:
        lib().lz_free(pa)


def default_threads():
    """Encoder threads: OMP_NUM_THREADS when set, else up to 16."""
    v = os.environ.get("OMP_NUM_THREADS")
    if v and v.isdigit() and int(v) > 0:
        return int(v)
    return min(os.cpu_count() or 1, 16)


def params(log2_bs=16, thr=BASE_THR, bounds=BOUNDS_CFG, max_chain=32, n_threads=0, segment=0, depth_passes=1,
           depth_cap=0):
    if not n_threads:
        n_threads = default_threads()
    p = Params()
    lib().lz_params_default(ctypes.byref(p))
    p.log2_bs = log2_bs
    for k in range(4):
        p.thr[k] = int(thr[k])
    for k in range(3):
        p.bound[k] = int(bounds[k])
    p.max_chain = max_chain
    p.n_threads = n_threads
    p.segment = segment
    p.depth_passes = depth_passes
    p.depth_cap = depth_cap
    return p


def encode(x, log2_bs=16, thr=BASE_THR, bounds=BOUNDS_CFG, max_chain=32, n_threads=0, segment=0, progress=None,
           depth_passes=1, mlp_path=None, depth_cap=0):
    """Greedy parse with per-distance-class thresholds into a container.
    progress(done, total), if given, is called after each segment;
    depth_passes (default 1) re-parses that many times breaking length ties
    by the lowest resulting dependency depth (0: nearest source); mlp_path,
    if given, selects learned mode: each block's tuple comes from the
    selector saved there (thr is then unused); depth_cap k > 0 turns the
    matches that would lie deeper than k into literals."""
    x = _u8(x)
    p = params(log2_bs, thr, bounds, max_chain, n_threads, segment, depth_passes, depth_cap)
    if mlp_path is not None:
        path = os.fsencode(mlp_path)
        p.mode = 1
        p.mlp_path = path
    if progress is not None:
        cb = PROGRESS_FN(lambda d, t, u: progress(int(d), int(t)))
        p.progress = cb
    pa = _vp()
    sz = _u64()
    rc = lib().lz_encode(x.ctypes.data, x.size, ctypes.byref(p), ctypes.byref(pa), ctypes.byref(sz))
    if rc:
        raise LzError(rc, "lz_encode")
    return _take_archive(pa, sz.value)


def encode_blockwise(x, thr_per_block, tuple_id=None, log2_bs=16, bounds=BOUNDS_CFG, max_chain=32, n_threads=0):
    x = _u8(x)
    tb = np.ascontiguousarray(thr_per_block, dtype=np.uint32).reshape(-1)
    tid = None if tuple_id is None else np.ascontiguousarray(tuple_id, dtype=np.uint8)
    p = params(log2_bs, TUNED_THR, bounds, max_chain, n_threads)  # header thresholds: informational
    pa = _vp()
    sz = _u64()
    rc = lib().lz_encode_blockwise(x.ctypes.data, x.size, ctypes.byref(p), tb.ctypes.data,
                                   None if tid is None else tid.ctypes.data, ctypes.byref(pa), ctypes.byref(sz))
    if rc:
        raise LzError(rc, "lz_encode_blockwise")
    return _take_archive(pa, sz.value)


def build_archive(n, log2_bs, lit_len, mlen, src, lit, min_match=0):
    ll = np.ascontiguousarray(lit_len, dtype=np.uint32)
    ml = np.ascontiguousarray(mlen, dtype=np.uint32)
    sr = np.ascontiguousarray(src, dtype=np.uint64)
    lt = _u8(lit)
    pa = _vp()
    sz = _u64()
    rc = lib().lz_build_archive(n, log2_bs, min_match, ll.size, ll.ctypes.data, ml.ctypes.data, sr.ctypes.data,
                                lt.ctypes.data, lt.size, ctypes.byref(pa), ctypes.byref(sz))
    if rc:
        raise LzError(rc, "lz_build_archive")
    return _take_archive(pa, sz.value)


def archive_info(arc):
    a = _u8(arc)
    inf = Info()
    rc = lib().lz_archive_info(a.ctypes.data, a.size, ctypes.byref(inf))
    if rc:
        raise LzError(rc, "lz_archive_info")
    d = {k: getattr(inf, k) for k, _ in Info._fields_ if k not in ("thr", "bound", "hist")}
    d["thr"] = tuple(inf.thr)
    d["bound"] = tuple(inf.bound)
    d["hist"] = np.array([[inf.hist[a][b] for b in range(16)] for a in range(4)], dtype=np.uint64)
    return d


def entropy_size(arc):
    a = _u8(arc)
    tot = ctypes.c_double()
    parts = np.zeros(7, dtype=np.float64)
    rc = lib().lz_entropy_size(a.ctypes.data, a.size, ctypes.byref(tot), parts.ctypes.data)
    if rc:
        raise LzError(rc, "lz_entropy_size")
    return float(tot.value), parts


def plan(arc):
    a = _u8(arc)
    inf = archive_info(a)
    lv = np.zeros(max(inf["n_tok"], 1), dtype=np.uint32)
    mx = _u32()
    rc = lib().lz_plan(a.ctypes.data, a.size, lv.ctypes.data, ctypes.byref(mx))
    if rc:
        raise LzError(rc, "lz_plan")
    return lv[:inf["n_tok"]], int(mx.value)


def fnv1a64(data, seed=0xcbf29ce484222325):
    a = _u8(data)
    return int(lib().lz_fnv1a64(a.ctypes.data, a.size, seed))


TAIL_OFF = 0xFFFFFFFF


def _cfg(G=64, unroll=2, schedule=1, tail=0, mapping=0, occupancy=0, parse_G=0, parse_unroll=0):
    c = DecodeCfg()
    c.G, c.unroll, c.schedule, c.tail, c.mapping, c.occupancy = G, unroll, schedule, tail, mapping, occupancy
    c.parse_G, c.parse_unroll = parse_G, parse_unroll
    return c


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class DeviceArchive:
    """A validated archive resident in device memory (torch-owned buffer).
    coded=True: `arc` is a tile-rANS coded container (lz_entropy_encode),
    entropy-decoded on the GPU at open and kept resident."""

    def __init__(self, arc, device="cuda", stream=None, coded=False):
        import torch
        self.arc = _u8(arc)
        self.coded = coded
        nb = _u64()
        sizer = lib().lz_coded_device_bytes if coded else lib().lz_device_bytes
        rc = sizer(self.arc.ctypes.data, self.arc.size, ctypes.byref(nb))
        if rc:
            raise LzError(rc, "lz_coded_device_bytes" if coded else "lz_device_bytes")
        self.buf = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = _vp()
        opener = lib().lz_device_open_coded if coded else lib().lz_device_open
        rc = opener(self.arc.ctypes.data, self.arc.size, ctypes.c_void_p(self.buf.data_ptr()), nb.value,
                    _stream(stream), ctypes.byref(h))
        if rc:
            raise LzError(rc, "lz_device_open_coded" if coded else "lz_device_open")
        self.h = h
        self.n = int(lib().lz_device_n(h))
        self.levels = int(lib().lz_device_levels(h))
        fb = _u64()
        self.fused = int(lib().lz_device_fused(h, ctypes.byref(fb)))  # literal-sourced matches the parse copies
        self.fused_bytes = int(fb.value)
        self.device_bytes = nb.value

    def decode(self, out=None, G=64, unroll=2, schedule=1, stream=None, check=True, tail=0, mapping=0, occupancy=0,
               parse_G=0, parse_unroll=0):
        import torch
        if out is None:
            out = torch.empty(max(self.n, 1), dtype=torch.uint8, device=self.buf.device)
        c = _cfg(G, unroll, schedule, tail, mapping, occupancy, parse_G, parse_unroll)
        rc = lib().lz_decode_device(self.h, ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(c),
                                    _stream(stream))
        if rc:
            raise LzError(rc, "lz_decode_device")
        if check:
            self.check(stream)
        return out[:self.n]

    def decode_async(self, out, G=64, unroll=2, schedule=1, stream=None, tail=0, mapping=0, occupancy=0,
                     parse_G=0, parse_unroll=0):
        c = _cfg(G, unroll, schedule, tail, mapping, occupancy, parse_G, parse_unroll)
        rc = lib().lz_decode_device(self.h, ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(c),
                                    _stream(stream))
        if rc:
            raise LzError(rc, "lz_decode_device")

    def decode_stage(self, out, stage, G=64, unroll=2, schedule=1, stream=None, tail=0, mapping=0, parse_G=0,
                     parse_unroll=0):
        """Stage 1 = parse launch, 2 = match passes (after stage 1), 0 = both."""
        c = _cfg(G, unroll, schedule, tail, mapping, 0, parse_G, parse_unroll)
        rc = lib().lz_decode_device_stage(self.h, ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(c),
                                          int(stage), _stream(stream))
        if rc:
            raise LzError(rc, "lz_decode_device_stage")

    def entropy_decode_async(self, stream=None):
        """Re-runs the entropy stage into the archive region (coded only)."""
        rc = lib().lz_entropy_decode_device(self.h, _stream(stream))
        if rc:
            raise LzError(rc, "lz_entropy_decode_device")

    def check(self, stream=None):
        rc = lib().lz_device_check(self.h, _stream(stream))
        if rc:
            raise LzError(rc, "lz_device_check")

    def range_plan(self, offs, lens):
        """Host plan for ranges [offs[i], offs[i]+lens[i])."""
        return RangePlan(self, offs, lens)

    def decode_range(self, off, length, out=None, scratch=None, stream=None):
        """Bytes [off, off+length) as a device tensor (synchronous)."""
        import torch
        sb = _u64()
        rc = lib().lz_range_scratch_bytes(self.h, off, length, ctypes.byref(sb))
        if rc:
            raise LzError(rc, "lz_range_scratch_bytes")
        if out is None:
            out = torch.empty(max(length, 1), dtype=torch.uint8, device=self.buf.device)
        if scratch is None or scratch.numel() < sb.value:
            scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.buf.device)
        rc = lib().lz_decode_range(self.h, off, length, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), _stream(stream))
        if rc:
            raise LzError(rc, "lz_decode_range")
        return out[:length]

    def close(self):
        if getattr(self, "h", None):
            lib().lz_device_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PureCopy:
    """Pre-decoded tokens bound to their device buffers (torch cuda tensors),
    bounds-checked once here on the host; run() only launches."""

    def __init__(self, dst, lit_off, lit_len, src, mlen, unit_start, lit, ref, out):
        import torch
        T = dst.numel()
        for t in (lit_off, lit_len, src, mlen):
            assert t.numel() == T
        if T:
            ends = (dst.to(torch.int64) + lit_len.to(torch.int64) + mlen.to(torch.int64)).max().item()
            lend = (lit_off.to(torch.int64) + lit_len.to(torch.int64)).max().item()
            send = (src.to(torch.int64) + mlen.to(torch.int64)).max().item()
            if ends > out.numel() or lend > lit.numel() or send > ref.numel():
                raise ValueError("pre-decoded tokens index outside their buffers")
            us = unit_start.to("cpu").to(torch.int64)
            if us[0].item() != 0 or us[-1].item() != T or bool((us[1:] < us[:-1]).any()):
                raise ValueError("unit starts must run from 0 to ntok")
        self.args = (dst, lit_off, lit_len, src, mlen, unit_start, lit, ref, out)

    def run(self, G=32, unroll=2, stream=None):
        dst, lit_off, lit_len, src, mlen, unit_start, lit, ref, out = self.args
        c = _cfg(G, unroll, 0)
        rc = lib().lz_purecopy_device(dst.numel(), ctypes.c_void_p(dst.data_ptr()),
                                      ctypes.c_void_p(lit_off.data_ptr()), ctypes.c_void_p(lit_len.data_ptr()),
                                      ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(mlen.data_ptr()),
                                      unit_start.numel() - 1, ctypes.c_void_p(unit_start.data_ptr()),
                                      ctypes.c_void_p(lit.data_ptr()), lit.numel(), ctypes.c_void_p(ref.data_ptr()),
                                      ref.numel(), ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(c),
                                      _stream(stream))
        if rc:
            raise LzError(rc, "lz_purecopy_device")


def purecopy(dst, lit_off, lit_len, src, mlen, unit_start, lit, ref, out, G=32, unroll=2, stream=None):
    """Runs pre-decoded tokens on the device (all arguments torch cuda tensors).
    Bounds are checked here on the host copies before launch."""
    PureCopy(dst, lit_off, lit_len, src, mlen, unit_start, lit, ref, out).run(G, unroll, stream)


class RangePlan:
    """Merged plan of several ranges of one DeviceArchive (host object)."""

    def __init__(self, da, offs, lens):
        self.da = da
        self.offs = np.ascontiguousarray(offs, dtype=np.uint64)
        self.lens = np.ascontiguousarray(lens, dtype=np.uint64)
        p = _vp()
        rc = lib().lz_range_plan_create(da.h, self.offs.size, self.offs.ctypes.data, self.lens.ctypes.data,
                                        ctypes.byref(p))
        if rc:
            raise LzError(rc, "lz_range_plan_create")
        self.p = p
        self.scratch_bytes = int(lib().lz_range_plan_scratch_bytes(p))
        self.levels = int(lib().lz_range_plan_levels(p))
        self.closure_bytes = int(lib().lz_range_plan_closure_bytes(p))
        self.prefix_bytes = int(lib().lz_range_plan_prefix_bytes(p))
        self.horizon = int(lib().lz_range_plan_horizon(p))

    def run(self, out, out_offs, scratch, G=64, unroll=2, stream=None, tail=0):
        """Enqueues the plan; range i lands at out[out_offs[i]:+lens[i]]."""
        oo = np.ascontiguousarray(out_offs, dtype=np.uint64)
        c = _cfg(G, unroll, 0, tail)
        rc = lib().lz_range_run(self.da.h, self.p, ctypes.c_void_p(out.data_ptr()), out.numel(), oo.ctypes.data,
                                ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), ctypes.byref(c),
                                _stream(stream))
        if rc:
            raise LzError(rc, "lz_range_run")

    def free(self):
        if getattr(self, "p", None):
            lib().lz_range_plan_free(self.p)
            self.p = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _ptr_array(vals):
    arr = (ctypes.c_void_p * max(len(vals), 1))()
    for i, v in enumerate(vals):
        arr[i] = v
    return arr


def _cfg_array(cfgs):
    arr = (DecodeCfg * max(len(cfgs), 1))()
    for i, c in enumerate(cfgs):
        if isinstance(c, DecodeCfg):
            arr[i] = c
        else:
            arr[i] = _cfg(*c)
    return arr


class Batch:
    """One replayable launch sequence decoding many DeviceArchives; archive i
    into outs[i] (torch tensors).  cfgs: None, or per archive a DecodeCfg or a
    (G, unroll, schedule[, tail[, mapping]]) tuple."""

    def __init__(self, archives, outs, cfgs=None, stream=None):
        import torch
        self.archives = archives
        self.outs = outs
        hs = _ptr_array([a.h.value for a in archives])
        cf = None if cfgs is None else _cfg_array(cfgs)
        sb = _u64()
        rc = lib().lz_batch_scratch_bytes(len(archives), hs, cf, ctypes.byref(sb))
        if rc:
            raise LzError(rc, "lz_batch_scratch_bytes")
        dev = archives[0].buf.device if archives else torch.device("cuda")
        self.scratch = torch.empty(max(sb.value, 256), dtype=torch.uint8, device=dev)
        op = _ptr_array([o.data_ptr() for o in outs])
        caps = np.array([o.numel() for o in outs], dtype=np.uint64)
        b = _vp()
        rc = lib().lz_batch_create(len(archives), hs, op, caps.ctypes.data, cf, ctypes.c_void_p(self.scratch.data_ptr()),
                                   self.scratch.numel(), _stream(stream), ctypes.byref(b))
        if rc:
            raise LzError(rc, "lz_batch_create")
        self.b = b
        self.launches = int(lib().lz_batch_launches(b))

    def launch(self, stream=None):
        rc = lib().lz_batch_launch(self.b, _stream(stream))
        if rc:
            raise LzError(rc, "lz_batch_launch")

    def destroy(self):
        if getattr(self, "b", None):
            lib().lz_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(archives, outs, reps=3, stream=None):
    """Per-archive configuration chosen per size bucket; returns (cfgs, report)."""
    import torch
    n = len(archives)
    hs = _ptr_array([a.h.value for a in archives])
    sb = _u64()
    rc = lib().lz_batch_scratch_bytes(n, hs, None, ctypes.byref(sb))
    if rc:
        raise LzError(rc, "lz_batch_scratch_bytes")
    # room for the whole batch with several configuration groups (their
    # per-group tables), so the final whole-batch check can run
    scratch = torch.empty(max(sb.value, 256) + (1 << 20), dtype=torch.uint8, device=archives[0].buf.device)
    op = _ptr_array([o.data_ptr() for o in outs])
    caps = np.array([o.numel() for o in outs], dtype=np.uint64)
    chosen = (DecodeCfg * max(n, 1))()
    rep = (TuneReport * 16)()
    nrep = _u32()
    rc = lib().lz_autotune(n, hs, op, caps.ctypes.data, ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                           _stream(stream), reps, chosen, rep, 16, ctypes.byref(nrep))
    if rc:
        raise LzError(rc, "lz_autotune")
    cfgs = [(chosen[i].G, chosen[i].unroll, chosen[i].schedule, chosen[i].tail, chosen[i].mapping) for i in range(n)]
    report = [{"min_bytes": rep[i].min_bytes, "max_bytes": rep[i].max_bytes, "archives": rep[i].archives,
               "bytes": rep[i].bytes,
               "best": (rep[i].best.G, rep[i].best.unroll, rep[i].best.schedule, rep[i].best.mapping),
               "best_ms": rep[i].best_ms, "default_ms": rep[i].default_ms} for i in range(nrep.value)]
    return cfgs, report


class Server:
    """Continuous-batching range server over one DeviceArchive; the arena
    (outputs + scratch) is a torch device buffer of `arena_bytes`."""

    def __init__(self, da, arena_bytes, slots=64, G=64, unroll=2):
        import torch
        self.da = da
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=da.buf.device)
        c = _cfg(G, unroll, 1)
        p = _vp()
        rc = lib().lz_serve_create(da.h, ctypes.c_void_p(self.arena.data_ptr()), arena_bytes, slots, ctypes.byref(c),
                                   ctypes.byref(p))
        if rc:
            raise LzError(rc, "lz_serve_create")
        self.s = p

    def submit(self, off, length):
        i = _u64()
        rc = lib().lz_serve_submit(self.s, off, length, ctypes.byref(i))
        if rc:
            raise LzError(rc, "lz_serve_submit")
        return i.value

    def tick(self):
        d, a = _u64(), _u64()
        rc = lib().lz_serve_tick(self.s, ctypes.byref(d), ctypes.byref(a))
        if rc:
            raise LzError(rc, "lz_serve_tick")
        return d.value, a.value

    def status(self, rid):
        st = ctypes.c_int()
        ptr = _vp()
        rc = lib().lz_serve_status(self.s, rid, ctypes.byref(st), ctypes.byref(ptr))
        if rc:
            raise LzError(rc, "lz_serve_status")
        return st.value, (ptr.value or 0) - self.arena.data_ptr()

    def result(self, rid, length):
        """View of a done request's bytes inside the arena."""
        st, off = self.status(rid)
        assert st == 2, st
        return self.arena[off:off + length]

    def release(self, rid):
        rc = lib().lz_serve_release(self.s, rid)
        if rc:
            raise LzError(rc, "lz_serve_release")

    def completed(self, cap=4096):
        """Ids that finished (done or failed) since the last call."""
        buf = np.zeros(cap, dtype=np.uint64)
        k = int(lib().lz_serve_completed(self.s, buf.ctypes.data_as(_p64), cap))
        return buf[:k].tolist()

    def stats(self):
        w, r, u, hw = _u64(), _u64(), _u64(), _u64()
        lib().lz_serve_stats(self.s, ctypes.byref(w), ctypes.byref(r), ctypes.byref(u), ctypes.byref(hw))
        return {"waiting": w.value, "running_groups": r.value, "arena_used": u.value, "arena_high_water": hw.value,
                "max_running_groups": int(lib().lz_serve_max_running(self.s))}

    def destroy(self):
        if getattr(self, "s", None):
            lib().lz_serve_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def block_features(arc, bounds=BOUNDS_CFG):
    a = _u8(arc)
    nb = archive_info(a)["n_blocks"]
    f = np.zeros((max(nb, 1), 64), dtype=np.float32)
    b = np.asarray(bounds, dtype=np.uint64)
    rc = lib().lz_block_features(a.ctypes.data, a.size, b.ctypes.data, f.ctypes.data)
    if rc:
        raise LzError(rc, "lz_block_features")
    return f[:nb]


def block_stats(arc):
    """Per block: entropy-bound bytes, tokens, matches, match bytes."""
    a = _u8(arc)
    nb = archive_info(a)["n_blocks"]
    ent = np.zeros(max(nb, 1), dtype=np.float64)
    nt, nm, mb = (np.zeros(max(nb, 1), dtype=np.uint64) for _ in range(3))
    rc = lib().lz_block_stats(a.ctypes.data, a.size, ent.ctypes.data, nt.ctypes.data, nm.ctypes.data, mb.ctypes.data)
    if rc:
        raise LzError(rc, "lz_block_stats")
    return ent[:nb], nt[:nb], nm[:nb], mb[:nb]


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def mlp_forward(params, x, h1, h2, logits, stream=None):
    rc = lib().lz_mlp_forward(_p(params), x.shape[0], _p(x), _p(h1), _p(h2), _p(logits), _stream(stream))
    if rc:
        raise LzError(rc, "lz_mlp_forward")


def mlp_backward(params, x, h1, h2, logits, labels, grads, work, loss=None, stream=None):
    rc = lib().lz_mlp_backward(_p(params), x.shape[0], _p(x), _p(h1), _p(h2), _p(logits), _p(labels), _p(grads),
                               _p(work), None if loss is None else _p(loss), _stream(stream))
    if rc:
        raise LzError(rc, "lz_mlp_backward")


def mlp_backward_noalloc(params, x, h1, h2, logits, labels, grads, loss=None, stream=None):
    """mlp_backward with the library's per-GPU work array (batch <= 4096)."""
    rc = lib().lz_mlp_backward_noalloc(_p(params), x.shape[0], _p(x), _p(h1), _p(h2), _p(logits), _p(labels),
                                       _p(grads), None if loss is None else _p(loss), _stream(stream))
    if rc:
        raise LzError(rc, "lz_mlp_backward_noalloc")


def mlp_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    rc = lib().lz_mlp_adam(_p(params), _p(grads), _p(m), _p(v), params.numel(), lr, beta1, beta2, eps, step,
                           _stream(stream))
    if rc:
        raise LzError(rc, "lz_mlp_adam")


# ------------------------------------------------------------ learned thresholds

class Selector:
    """The learned per-block threshold selector (a liblz host object): 16
    candidate tuples, the fixed fallback, feature normalisation, the fallback
    rule's validation table and the network parameters."""

    def __init__(self, tuples=None, fixed=1, seed=1, path=None):
        h = _vp()
        if path is not None:
            rc = lib().lz_selector_load(os.fsencode(path), ctypes.byref(h))
            what = "lz_selector_load"
        else:
            t = np.ascontiguousarray(tuples, dtype=np.uint32).reshape(16, 4)
            rc = lib().lz_selector_create(t.ctypes.data, fixed, seed, ctypes.byref(h))
            what = "lz_selector_create"
        if rc:
            raise LzError(rc, what)
        self.h = h

    def save(self, path):
        rc = lib().lz_selector_save(self.h, os.fsencode(path))
        if rc:
            raise LzError(rc, "lz_selector_save")

    def params(self, new=None):
        """The 26,896 parameters (a copy); with `new`, sets them first."""
        out = np.zeros(26896, dtype=np.float32)
        src = None if new is None else np.ascontiguousarray(new, dtype=np.float32)
        rc = lib().lz_selector_params(self.h, out.ctypes.data, None if src is None else src.ctypes.data)
        if rc:
            raise LzError(rc, "lz_selector_params")
        return out

    def info(self):
        t = np.zeros((16, 4), np.uint32)
        fixed = _u32()
        mu, sd, vj = (np.zeros(n, np.float32) for n in (64, 64, 16))
        rc = lib().lz_selector_info(self.h, t.ctypes.data, ctypes.byref(fixed), mu.ctypes.data, sd.ctypes.data,
                                    vj.ctypes.data)
        if rc:
            raise LzError(rc, "lz_selector_info")
        return {"tuples": t, "fixed": fixed.value, "mu": mu, "sd": sd, "val_J": vj}

    def set_norm(self, feats):
        f = np.ascontiguousarray(feats, dtype=np.float32)
        rc = lib().lz_selector_set_norm(self.h, f.ctypes.data, f.shape[0])
        if rc:
            raise LzError(rc, "lz_selector_set_norm")

    def train(self, feats, labels, epochs=50, batch=256, lr=1e-3, seed=0, stream=None):
        """GPU training with the library's kernels; returns the per-epoch loss."""
        import torch
        f = np.ascontiguousarray(feats, dtype=np.float32)
        y = np.ascontiguousarray(labels, dtype=np.int32)
        nb = _u64()
        rc = lib().lz_selector_train_bytes(f.shape[0], batch, ctypes.byref(nb))
        if rc:
            raise LzError(rc, "lz_selector_train_bytes")
        work = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        hist = np.zeros(max(epochs, 1), dtype=np.float32)
        rc = lib().lz_selector_train(self.h, f.ctypes.data, y.ctypes.data, f.shape[0], epochs, batch, lr, seed,
                                     ctypes.c_void_p(work.data_ptr()), nb.value, hist.ctypes.data, _stream(stream))
        if rc:
            raise LzError(rc, "lz_selector_train")
        return hist[:epochs].tolist()

    def calibrate(self, feats, J, lam=1.0):
        f = np.ascontiguousarray(feats, dtype=np.float32)
        j = np.ascontiguousarray(J, dtype=np.float64)
        rc = lib().lz_selector_calibrate(self.h, f.ctypes.data, j.ctypes.data, f.shape[0], lam)
        if rc:
            raise LzError(rc, "lz_selector_calibrate")

    def choose(self, feats):
        """(tuple index per row with the fallback applied, top probability)."""
        f = np.ascontiguousarray(feats, dtype=np.float32)
        c = np.zeros(max(f.shape[0], 1), np.uint8)
        p = np.zeros(max(f.shape[0], 1), np.float32)
        rc = lib().lz_selector_choose(self.h, f.ctypes.data, f.shape[0], c.ctypes.data, p.ctypes.data)
        if rc:
            raise LzError(rc, "lz_selector_choose")
        return c[:f.shape[0]], p[:f.shape[0]]

    def free(self):
        if getattr(self, "h", None):
            lib().lz_selector_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def learn_labels(file_blocks, size, counts, file_ms, file_depths, lam=1.0, fixed=1):
    """Time-model coefficients, J and labels (lz_learn_labels)."""
    fb = np.ascontiguousarray(file_blocks, dtype=np.uint32)
    sz = np.ascontiguousarray(size, dtype=np.float64)
    ct = np.ascontiguousarray(counts, dtype=np.uint64)
    ms = np.ascontiguousarray(file_ms, dtype=np.float64)
    dp = np.ascontiguousarray(file_depths, dtype=np.uint32)
    K = int(fb.sum())
    assert sz.size == 16 * K and ct.size == 48 * K and ms.size == 16 * fb.size and dp.size == 16 * fb.size
    coef = np.zeros(5, np.float64)
    J = np.zeros((K, 16), np.float64)
    lab = np.zeros(max(K, 1), np.int32)
    rc = lib().lz_learn_labels(fb.size, fb.ctypes.data, fixed, sz.ctypes.data, ct.ctypes.data, ms.ctypes.data,
                               dp.ctypes.data, lam, coef.ctypes.data, J.ctypes.data, lab.ctypes.data)
    if rc:
        raise LzError(rc, "lz_learn_labels")
    return coef, J, lab[:K]


def encode_learned(x, sel, log2_bs=16, bounds=BOUNDS_CFG, max_chain=32, n_threads=0, depth_passes=1):
    """Learned-mode encode: (archive, chosen tuple index per block)."""
    x = _u8(x)
    p = params(log2_bs, TUNED_THR, bounds, max_chain, n_threads, 0, depth_passes)
    nb = (x.size + (1 << log2_bs) - 1) >> log2_bs
    ch = np.zeros(max(nb, 1), np.uint8)
    pa = _vp()
    sz = _u64()
    rc = lib().lz_encode_learned(x.ctypes.data, x.size, ctypes.byref(p), sel.h, ctypes.byref(pa), ctypes.byref(sz),
                                 ch.ctypes.data)
    if rc:
        raise LzError(rc, "lz_encode_learned")
    return _take_archive(pa, sz.value), ch[:nb]


# ------------------------------------------------------------ read seek

class ReadIndex:
    """Record id -> LZ block index of an input (records of `lines` lines)."""

    def __init__(self, x=None, log2_bs=16, lines=4, path=None):
        h = _vp()
        if path is not None:
            rc = lib().lz_read_index_load(os.fsencode(path), ctypes.byref(h))
            what = "lz_read_index_load"
        else:
            a = _u8(x)
            rc = lib().lz_read_index_build(a.ctypes.data, a.size, log2_bs, lines, ctypes.byref(h))
            what = "lz_read_index_build"
        if rc:
            raise LzError(rc, what)
        self.h = h
        self.records = int(lib().lz_read_index_records(h))

    def block(self, b):
        fi, fo = _u64(), _u64()
        rc = lib().lz_read_index_block(self.h, b, ctypes.byref(fi), ctypes.byref(fo))
        if rc:
            raise LzError(rc, "lz_read_index_block")
        return fi.value, fo.value

    def save(self, path):
        rc = lib().lz_read_index_save(self.h, os.fsencode(path))
        if rc:
            raise LzError(rc, "lz_read_index_save")

    def seek(self, da, rid, out=None, scratch=None, stream=None):
        """Record `rid` of DeviceArchive `da` as a device tensor (synchronous)."""
        import torch
        sb = _u64()
        rc = lib().lz_seek_record_scratch_bytes(da.h, self.h, rid, ctypes.byref(sb))
        if rc:
            raise LzError(rc, "lz_seek_record_scratch_bytes")
        if scratch is None or scratch.numel() < sb.value:
            scratch = torch.empty(sb.value, dtype=torch.uint8, device=da.buf.device)
        if out is None:
            out = torch.empty(1 << 16, dtype=torch.uint8, device=da.buf.device)
        n = _u64()
        rc = lib().lz_seek_record(da.h, self.h, rid, ctypes.c_void_p(out.data_ptr()), out.numel(),
                                  ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), ctypes.byref(n),
                                  _stream(stream))
        if rc:
            raise LzError(rc, "lz_seek_record")
        return out[:n.value]

    def free(self):
        if getattr(self, "h", None):
            lib().lz_read_index_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------ entropy stage

def entropy_encode(arc):
    """Tile-rANS coded container of a container (host)."""
    a = _u8(arc)
    pa = _vp()
    sz = _u64()
    rc = lib().lz_entropy_encode(a.ctypes.data, a.size, ctypes.byref(pa), ctypes.byref(sz))
    if rc:
        raise LzError(rc, "lz_entropy_encode")
    return _take_archive(pa, sz.value)


def entropy_info(coded):
    a = _u8(coded)
    ds, nt = _u64(), _u64()
    modes = np.zeros(3, np.uint64)
    rc = lib().lz_entropy_info(a.ctypes.data, a.size, ctypes.byref(ds), ctypes.byref(nt), modes.ctypes.data)
    if rc:
        raise LzError(rc, "lz_entropy_info")
    return {"decoded_size": ds.value, "tiles": nt.value, "raw": int(modes[0]), "rans": int(modes[1]),
            "repeat": int(modes[2])}
