"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Thin ctypes wrapper over ``libsynth.so`` (built from ``synth.c``).  Nothing here
knows the codec: it only makes bytes and token lists with the statistics of the
paper's workloads (Zipf text, FASTQ reads, streams with a controlled mean match
length).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError("synth/libsynth.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        L.synth_zipf_text.restype = ctypes.c_uint64
        L.synth_zipf_text.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_uint32]
        L.synth_fastq.restype = ctypes.c_uint64
        L.synth_fastq.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32]
        L.synth_geo_tokens.restype = ctypes.c_int
        L.synth_geo_tokens.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                       ctypes.POINTER(_u32p), ctypes.POINTER(_u32p), ctypes.POINTER(_u64p),
                                       _u64p, ctypes.POINTER(_u8p)]
        L.synth_free.restype = None
        L.synth_free.argtypes = [ctypes.c_void_p]
        L.synth_random_bytes.restype = None
        L.synth_random_bytes.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
        L.synth_loguniform.restype = None
        L.synth_loguniform.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64]
        L.synth_uniform.restype = None
        L.synth_uniform.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
        L.synth_normal.restype = None
        L.synth_normal.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64]
        _LIB = L
    return _LIB


def zipf_text(n, seed=1, s=1.1, vocab=4096):
    """n bytes of space-separated Zipf(s) words over a `vocab`-word random
    lowercase vocabulary (word length 2..12), newline after every 80 chars."""
    out = np.empty(n, dtype=np.uint8)
    if n:
        lib().synth_zipf_text(out.ctypes.data, n, seed, s, vocab)
    return out


def fastq(cap, seed=3, sub_rate=0.01, n_rate=0.001, ref_len=5_000_000, read_len=150):
    """Whole FASTQ-like records totalling at most `cap` bytes."""
    buf = np.empty(cap, dtype=np.uint8)
    got = lib().synth_fastq(buf.ctypes.data, cap, seed, sub_rate, n_rate, ref_len, read_len)
    return buf[:got].copy() if got < cap // 2 else buf[:got]


def geo_tokens(n, mean, seed=2, lit_prefix=65536, len_cap=65536, min_back=65536):
    """Token stream covering n output bytes with geometric match lengths of the
    given mean.  Returns (lit_len u32[T], mlen u32[T], src u64[T], lit u8[L]);
    token t writes lit_len[t] literal bytes then copies mlen[t] bytes from
    absolute position src[t]."""
    L = lib()
    nt = ctypes.c_uint64()
    nl = ctypes.c_uint64()
    pl = _u32p()
    pm = _u32p()
    ps = _u64p()
    pt = _u8p()
    rc = L.synth_geo_tokens(n, float(mean), seed, lit_prefix, len_cap, min_back, ctypes.byref(nt),
                            ctypes.byref(pl), ctypes.byref(pm), ctypes.byref(ps), ctypes.byref(nl),
                            ctypes.byref(pt))
    if rc != 0:
        raise MemoryError("synth_geo_tokens failed")
    T = nt.value
    try:
        lit_len = np.ctypeslib.as_array(pl, shape=(max(T, 1),))[:T].copy()
        mlen = np.ctypeslib.as_array(pm, shape=(max(T, 1),))[:T].copy()
        src = np.ctypeslib.as_array(ps, shape=(max(T, 1),))[:T].copy()
        lit = np.ctypeslib.as_array(pt, shape=(max(nl.value, 1),))[:nl.value].copy()
    finally:
        for p in (pl, pm, ps, pt):
            L.synth_free(ctypes.cast(p, ctypes.c_void_p))
    return lit_len, mlen, src, lit


def random_bytes(n, seed):
    out = np.empty(n, dtype=np.uint8)
    if n:
        lib().synth_random_bytes(out.ctypes.data, n, seed)
    return out


def loguniform(count, lo, hi, seed):
    out = np.empty(count, dtype=np.uint64)
    if count:
        lib().synth_loguniform(out.ctypes.data, count, lo, hi, seed)
    return out


def uniform(count, seed):
    out = np.empty(count, dtype=np.float64)
    if count:
        lib().synth_uniform(out.ctypes.data, count, seed)
    return out


def normal(count, seed):
    out = np.empty(count, dtype=np.float64)
    if count:
        lib().synth_normal(out.ctypes.data, count, seed)
    return out
