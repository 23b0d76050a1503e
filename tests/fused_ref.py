"""Which matches the parse may copy from the literal stream, derived from the
oracle's tokens and dependency depths (test infrastructure): a match of depth
1 whose source [src, src + len) lies inside one token's literal run and ends
at or before the match's own output."""
import numpy as np

import oracle


def literal_sourced(arc):
    """Returns (mask over tokens, output start of each match, match lengths)."""
    tk = oracle.tokens(arc)
    depth, _ = oracle.levels(arc)
    dst = tk["dst"].astype(np.int64)
    ll = tk["lit_len"].astype(np.int64)
    ml = tk["mlen"].astype(np.int64)
    src = tk["src"].astype(np.int64)
    md = dst + ll
    t = np.searchsorted(dst, src, side="right") - 1
    t = np.clip(t, 0, len(dst) - 1)
    inside = (src >= dst[t]) & (src + ml <= dst[t] + ll[t])
    mask = (ml > 0) & (depth == 1) & (src + ml <= md) & inside
    return mask, md, ml
