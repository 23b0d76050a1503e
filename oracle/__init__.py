"""CPU oracle for absolute-offset LZ77 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
the oracle shares no code with it: ``lz_oracle.c`` is a plain sequential
implementation written from the paper's definitions (see its header), and
``mlp_ref.py`` is a float64 numpy restatement of the threshold selector.

Wrapped functions (each cites the passage it follows in ``lz_oracle.c`` and
``lz_rans.c``): ``fnv1a64``, ``encode`` (exhaustive greedy parse),
``write_archive``, ``decode``, ``tokens``, ``levels``, ``entropy_size``,
``purecopy``, ``exec_tokens``, and the tile-rANS stage: ``rans_normalise``,
``rans_encode_tile``, ``rans_decode_tile``, ``entropy_encode``,
``entropy_decode``.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_p64 = ctypes.POINTER(ctypes.c_uint64)

OR_OK, OR_E_INVAL, OR_E_CORRUPT, OR_E_NOMEM = 0, -1, -2, -4

# distance classes of the configurations: <4 KiB, <64 KiB, <1 MiB, >=1 MiB
BOUNDS_CFG = (4096, 65536, 1 << 20)
# distance classes named in Sec. 4.2: d<128, d<16384, d<2097152, else
BOUNDS_PAPER = (128, 16384, 2097152)


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"oracle {what} failed with code {rc}")
        self.rc = rc


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        L.or_fnv1a64.restype = _u64
        L.or_fnv1a64.argtypes = [_vp, _u64]
        L.or_free.restype = None
        L.or_free.argtypes = [_vp]
        L.or_encode.restype = ctypes.c_int
        L.or_encode.argtypes = [_vp, _u64, _u32, _vp, _vp, _p64, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                ctypes.POINTER(_vp), ctypes.POINTER(_vp), _p64]
        L.or_write_archive.restype = ctypes.c_int
        L.or_write_archive.argtypes = [_u64, _u32, _u32, _u64, _vp, _vp, _vp, _vp, _u64, _vp, _vp,
                                       ctypes.POINTER(_vp), _p64]
        L.or_decode.restype = ctypes.c_int
        L.or_decode.argtypes = [_vp, _u64, _vp, _u64]
        L.or_info.restype = ctypes.c_int
        L.or_info.argtypes = [_vp, _u64, _p64, _p64, _p64, _p64, _p64]
        L.or_tokens.restype = ctypes.c_int
        L.or_tokens.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp]
        L.or_levels.restype = ctypes.c_int
        L.or_levels.argtypes = [_vp, _u64, _vp, ctypes.POINTER(ctypes.c_uint32)]
        L.or_entropy_size.restype = ctypes.c_int
        L.or_entropy_size.argtypes = [_vp, _u64, ctypes.POINTER(ctypes.c_double), _vp]
        L.or_purecopy.restype = None
        L.or_purecopy.argtypes = [_u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.or_lit_stream.restype = ctypes.c_int
        L.or_lit_stream.argtypes = [_vp, _u64, _p64, _p64]
        L.or_decode_levels_omp.restype = ctypes.c_int
        L.or_decode_levels_omp.argtypes = [_u64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp]
        L.or_exec_tokens.restype = ctypes.c_int
        L.or_exec_tokens.argtypes = [_u64, _u64, _vp, _vp, _vp, _vp, _u64, _vp]
        L.or_rans_normalise.restype = ctypes.c_int
        L.or_rans_normalise.argtypes = [_vp, _u64, _vp]
        L.or_rans_encode_tile.restype = _u64
        L.or_rans_encode_tile.argtypes = [_vp, _u64, _u64, ctypes.POINTER(_vp)]
        L.or_rans_decode_tile.restype = ctypes.c_int
        L.or_rans_decode_tile.argtypes = [_vp, _u64, _u64, _vp, _u64]
        L.or_entropy_encode.restype = ctypes.c_int
        L.or_entropy_encode.argtypes = [_vp, _u64, ctypes.POINTER(_vp), _p64]
        L.or_entropy_decode.restype = ctypes.c_int
        L.or_entropy_decode.argtypes = [_vp, _u64, _vp, _u64, _p64]
        _LIB = L
    return _LIB


def _u8(a):
    if isinstance(a, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(a), dtype=np.uint8)
    return np.ascontiguousarray(a, dtype=np.uint8)


def fnv1a64(data):
    a = _u8(data)
    return int(lib().or_fnv1a64(a.ctypes.data, a.size))


def encode(x, log2_bs=16, thr=(6, 8, 10, 12), bounds=BOUNDS_CFG):
    """Exhaustive greedy parse (Sec. 4.2 thresholds by distance class).
    Returns (lit_len u32[T], mlen u32[T], src u64[T], lit u8[L])."""
    x = _u8(x)
    t = np.asarray(thr, dtype=np.uint32)
    b = np.asarray(bounds, dtype=np.uint64)
    nt = _u64()
    nl = _u64()
    pl, pm, ps, pt = _vp(), _vp(), _vp(), _vp()
    rc = lib().or_encode(x.ctypes.data, x.size, log2_bs, t.ctypes.data, b.ctypes.data, ctypes.byref(nt),
                         ctypes.byref(pl), ctypes.byref(pm), ctypes.byref(ps), ctypes.byref(pt),
                         ctypes.byref(nl))
    if rc:
        raise OracleError(rc, "encode")
    T, NL = nt.value, nl.value
    try:
        lit_len = np.ctypeslib.as_array(ctypes.cast(pl, ctypes.POINTER(ctypes.c_uint32)), (max(T, 1),))[:T].copy()
        mlen = np.ctypeslib.as_array(ctypes.cast(pm, ctypes.POINTER(ctypes.c_uint32)), (max(T, 1),))[:T].copy()
        src = np.ctypeslib.as_array(ctypes.cast(ps, ctypes.POINTER(ctypes.c_uint64)), (max(T, 1),))[:T].copy()
        lit = np.ctypeslib.as_array(ctypes.cast(pt, ctypes.POINTER(ctypes.c_uint8)), (max(NL, 1),))[:NL].copy()
    finally:
        for p in (pl, pm, ps, pt):
            lib().or_free(p)
    return lit_len, mlen, src, lit


def write_archive(n, log2_bs, lit_len, mlen, src, lit, min_match=0, thr=(0, 0, 0, 0), bounds=(0, 0, 0)):
    """Serialises a token list (cut at block ends) into container version 1."""
    ll = np.ascontiguousarray(lit_len, dtype=np.uint32)
    ml = np.ascontiguousarray(mlen, dtype=np.uint32)
    sr = np.ascontiguousarray(src, dtype=np.uint64)
    lt = _u8(lit)
    t = np.asarray(thr, dtype=np.uint32)
    b = np.asarray(bounds, dtype=np.uint64)
    pa = _vp()
    sz = _u64()
    rc = lib().or_write_archive(n, log2_bs, min_match, ll.size, ll.ctypes.data, ml.ctypes.data, sr.ctypes.data,
                                lt.ctypes.data, lt.size, t.ctypes.data, b.ctypes.data, ctypes.byref(pa),
                                ctypes.byref(sz))
    if rc:
        raise OracleError(rc, "write_archive")
    try:
        arc = np.ctypeslib.as_array(ctypes.cast(pa, ctypes.POINTER(ctypes.c_uint8)), (sz.value,)).copy()
    finally:
        lib().or_free(pa)
    return arc


def info(arc):
    a = _u8(arc)
    v = [_u64() for _ in range(5)]
    rc = lib().or_info(a.ctypes.data, a.size, *[ctypes.byref(x) for x in v])
    if rc:
        raise OracleError(rc, "info")
    n, nb, ntok, lb, mm = (x.value for x in v)
    return {"n": n, "n_blocks": nb, "n_tok": ntok, "log2_bs": lb, "min_match": mm}


def decode(arc, cap=None):
    """Validates and decodes a whole archive sequentially."""
    a = _u8(arc)
    n = info(a)["n"]
    out = np.zeros(max(n, 1) if cap is None else max(cap, 1), dtype=np.uint8)
    rc = lib().or_decode(a.ctypes.data, a.size, out.ctypes.data, n if cap is None else cap)
    if rc:
        raise OracleError(rc, "decode")
    return out[:n]


def decode_rc(arc):
    """Return code of a decode attempt (0, or a negative error)."""
    a = _u8(arc)
    if a.size < 128:
        return OR_E_CORRUPT
    try:
        n = info(a)["n"]
    except OracleError as e:
        return e.rc
    out = np.zeros(max(n, 1), dtype=np.uint8)
    return int(lib().or_decode(a.ctypes.data, a.size, out.ctypes.data, n))


def tokens(arc):
    """Per-token arrays: blk, dst (token start), lit_len, lit_off, mlen, src."""
    a = _u8(arc)
    T = info(a)["n_tok"]
    arrs = [np.zeros(max(T, 1), dtype=np.uint64) for _ in range(6)]
    rc = lib().or_tokens(a.ctypes.data, a.size, *[x.ctypes.data for x in arrs])
    if rc:
        raise OracleError(rc, "tokens")
    names = ("blk", "dst", "lit_len", "lit_off", "mlen", "src")
    return {k: v[:T] for k, v in zip(names, arrs)}


def levels(arc):
    """Dependency depth of each token's match (0 for a token without one);
    returns (depths u32[T], max)."""
    a = _u8(arc)
    T = info(a)["n_tok"]
    lv = np.zeros(max(T, 1), dtype=np.uint32)
    mx = ctypes.c_uint32()
    rc = lib().or_levels(a.ctypes.data, a.size, lv.ctypes.data, ctypes.byref(mx))
    if rc:
        raise OracleError(rc, "levels")
    return lv[:T], int(mx.value)


def levels_prepare(arc):
    """Inputs of the level-parallel CPU decode: the tokens, the literal
    stream, and the token indices grouped by dependency depth."""
    a = _u8(arc)
    inf = info(a)
    tk = tokens(a)
    lv, mx = levels(a)
    order = np.argsort(lv, kind="stable").astype(np.uint64)
    start = np.zeros(mx + 2, dtype=np.uint64)
    start[1:] = np.cumsum(np.bincount(lv, minlength=mx + 1))
    off, nl = _u64(), _u64()
    rc = lib().or_lit_stream(a.ctypes.data, a.size, ctypes.byref(off), ctypes.byref(nl))
    if rc:
        raise OracleError(rc, "lit_stream")
    lit = np.zeros(max(nl.value, 1), dtype=np.uint8)
    lit[:nl.value] = a[off.value:off.value + nl.value]
    return {"n": inf["n"], "tok": tk, "lit": lit, "order": order, "start": start, "max_depth": mx}


def decode_levels_omp(prep, out):
    """Level-parallel decode of prepared tokens into out (uint8[n]) on all
    host cores (OMP_NUM_THREADS); returns the number of threads used."""
    tk = prep["tok"]
    T = len(tk["dst"])
    return int(lib().or_decode_levels_omp(T, tk["dst"].ctypes.data, tk["lit_len"].ctypes.data,
                                          tk["lit_off"].ctypes.data, tk["mlen"].ctypes.data, tk["src"].ctypes.data,
                                          prep["lit"].ctypes.data, prep["order"].ctypes.data,
                                          prep["start"].ctypes.data, prep["max_depth"], out.ctypes.data))


def entropy_size(arc):
    """Entropy-bound size (bytes) and its parts: cmd, x16, x32, src planes,
    lit, header+table, src_hi plane."""
    a = _u8(arc)
    tot = ctypes.c_double()
    parts = np.zeros(7, dtype=np.float64)
    rc = lib().or_entropy_size(a.ctypes.data, a.size, ctypes.byref(tot), parts.ctypes.data)
    if rc:
        raise OracleError(rc, "entropy_size")
    return float(tot.value), parts


def purecopy(n, dst, lit_off, lit_len, src, mlen, lit, ref):
    """Executes pre-decoded tokens; matches read from `ref`."""
    out = np.zeros(max(n, 1), dtype=np.uint8)
    d = np.ascontiguousarray(dst, dtype=np.uint64)
    lo = np.ascontiguousarray(lit_off, dtype=np.uint64)
    ll = np.ascontiguousarray(lit_len, dtype=np.uint32)
    s = np.ascontiguousarray(src, dtype=np.uint64)
    ml = np.ascontiguousarray(mlen, dtype=np.uint32)
    lt = _u8(lit)
    rf = _u8(ref)
    lib().or_purecopy(d.size, d.ctypes.data, lo.ctypes.data, ll.ctypes.data, s.ctypes.data, ml.ctypes.data,
                      lt.ctypes.data, rf.ctypes.data, out.ctypes.data)
    return out[:n]


def rans_normalise(counts):
    """Quantised frequencies (total 4096) of a 256-entry count vector."""
    c = np.ascontiguousarray(counts, dtype=np.uint64)
    f = np.zeros(256, np.uint32)
    if not lib().or_rans_normalise(c.ctypes.data, int(c.sum()), f.ctypes.data):
        raise OracleError(OR_E_INVAL, "rans_normalise")
    return f


def rans_encode_tile(sym, stride=1):
    """rANS payload of the symbols sym[0], sym[stride], ... (bytes)."""
    a = _u8(sym)
    N = (a.size + stride - 1) // stride
    out = _vp()
    n = lib().or_rans_encode_tile(a.ctypes.data, stride, N, ctypes.byref(out))
    if n == 0:
        raise OracleError(OR_E_INVAL, "rans_encode_tile")
    res = np.ctypeslib.as_array(ctypes.cast(out, ctypes.POINTER(ctypes.c_uint8)), shape=(n,)).copy()
    lib().or_free(out)
    return res


def rans_decode_tile(payload, N):
    p = _u8(payload)
    out = np.zeros(max(N, 1), np.uint8)
    rc = lib().or_rans_decode_tile(p.ctypes.data, p.size, N, out.ctypes.data, 1)
    if rc:
        raise OracleError(rc, "rans_decode_tile")
    return out[:N]


def entropy_encode(arc):
    """Tile-rANS coded container of a container."""
    a = _u8(arc)
    out = _vp()
    n = _u64()
    rc = lib().or_entropy_encode(a.ctypes.data, a.size, ctypes.byref(out), ctypes.byref(n))
    if rc:
        raise OracleError(rc, "entropy_encode")
    res = np.ctypeslib.as_array(ctypes.cast(out, ctypes.POINTER(ctypes.c_uint8)), shape=(n.value,)).copy()
    lib().or_free(out)
    return res


def entropy_decode(coded):
    """The container a coded container decodes to (every byte written once)."""
    c = _u8(coded)
    if c.size < 16:
        raise OracleError(OR_E_CORRUPT, "entropy_decode")
    total = int(np.frombuffer(c[8:16].tobytes(), np.uint64)[0])
    if total > (1 << 40):
        raise OracleError(OR_E_CORRUPT, "entropy_decode")
    out = np.zeros(max(total, 1), np.uint8)
    n = _u64()
    rc = lib().or_entropy_decode(c.ctypes.data, c.size, out.ctypes.data, out.size, ctypes.byref(n))
    if rc:
        raise OracleError(rc, "entropy_decode")
    return out[:n.value]


def exec_tokens(n, lit_len, mlen, src, lit):
    """Executes an uncut token stream (as generated) into n output bytes."""
    out = np.zeros(max(n, 1), dtype=np.uint8)
    ll = np.ascontiguousarray(lit_len, dtype=np.uint32)
    ml = np.ascontiguousarray(mlen, dtype=np.uint32)
    s = np.ascontiguousarray(src, dtype=np.uint64)
    lt = _u8(lit)
    rc = lib().or_exec_tokens(n, ll.size, ll.ctypes.data, ml.ctypes.data, s.ctypes.data, lt.ctypes.data, lt.size,
                              out.ctypes.data)
    if rc:
        raise OracleError(rc, "exec_tokens")
    return out[:n]
