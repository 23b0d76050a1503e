/*
 * lz_oracle.c -- plain, slow, sequential CPU oracle for absolute-offset LZ77.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * bench's CPU-baseline leg load this library.  The product decoder never
 * calls it; it shares no source, header, table or helper with the product.
 *
 * What it computes, and where the paper fixes it:
 *  - The format: every match names an absolute output position as its
 *    source (Abstract; Sec. 1 "Positioning"); the stream is cut into LZ
 *    blocks whose size is an encode-time parameter (Sec. 2, Sec. 5 last
 *    paragraph).  The byte layout is not given in the paper; this file
 *    follows the container layout stated below (version 1), written
 *    independently of the product library.
 *  - Encode: greedy LZ77 with a minimum match length per distance class
 *    (Sec. 4.2: four bands on the distance d = dst - src, "d < b0",
 *    "d < b1", "d < b2", otherwise; thresholds such as 6/8/10/12 or
 *    12/16/24/32).  Every earlier position is a candidate source (whole-prefix
 *    window); a candidate is valid iff its match length reaches the threshold
 *    of its class; the longest valid candidate wins, ties to the nearest.
 *  - Decode: execute tokens in order, copying literals, then copying each
 *    match byte by byte from its absolute source (which realises overlap).
 *  - Integrity: FNV-1a 64 over the output (Sec. 2: FNV on GPU paths).
 *  - Dependency depth of each match for a parallel decode (the paper fixes
 *    no schedule; the reading used here: literal bytes have depth 0, a match
 *    has depth one more than the deepest token that wrote any of its source
 *    bytes, the bytes of the match itself excluded).
 *  - Entropy-bound size: order-0 entropy of each stream over 64 KiB tiles
 *    (Sec. 2: tile-ANS over 64 KB tiles), plus a symbol-table charge.
 *
 * Container, version 1 (all integers little-endian):
 *   [0,128) header: u32 magic 0x314D5A4C, u32 version 1, u64 n,
 *     u32 log2_bs, u32 n_blocks, u32 min_match, u32 flags (bit0: src_hi
 *     plane present, bit1: per-block info bytes present), u64 n_tok,
 *     u64 n_x16, u64 n_x32, u64 n_lit, u8 thr[4], u32 reserved,
 *     u64 bound[3], zero to 128.
 *   [128, 128+32*(n_blocks+1)) block table: per block the cumulative starts
 *     {u64 tok, u64 lit, u64 x16, u64 x32}; entry 0 is zero, the last entry
 *     holds the totals.
 *   then, each at a 16-byte aligned offset in this order: cmd u8[n_tok],
 *     x16 u16[n_x16], x32 u32[n_x32], src_lo u32[n_tok], src_hi u8[n_tok]
 *     (if flag bit0), lit u8[n_lit], info u8[n_blocks] (if flag bit1),
 *     then 16 zero bytes; the archive ends at the next multiple of 16.
 *   Token t of block b (block b covers [b*bs, min(n,(b+1)*bs))):
 *     c = cmd[t]; lit code = c>>4, match code = c&15;
 *     a code of 15 is extended by ext(): v = next x16; if v == 0xFFFF then
 *     v = 0xFFFF + next x32; the value is 15 + v.  Literal extension first.
 *     lit_len = literal value; the last token of a block has match code 0
 *     and match length (block end - position after its literals); any other
 *     token has match length min_match + match value.
 *     src = src_lo[t] | src_hi[t] << 32; a match needs src < its start;
 *     a token without a match has src 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVAL (-1)
#define OR_E_CORRUPT (-2)
#define OR_E_NOMEM (-4)

#define MAGIC 0x314D5A4Cu
#define HDR 128u

/* ---------------------------------------------------------------- FNV-1a 64 */
uint64_t or_fnv1a64(const uint8_t* p, uint64_t n) {
  uint64_t h = 0xcbf29ce484222325ULL;
  for (uint64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

void or_free(void* p) { free(p); }

/* ---------------------------------------------------------------- encode */

static int dist_class(uint64_t d, const uint64_t bound[3]) {
  if (d < bound[0]) return 0;
  if (d < bound[1]) return 1;
  if (d < bound[2]) return 2;
  return 3;
}

/* Greedy parse, straight from the definition: at each position try every
 * earlier source, measure its match length (capped at the block end; the
 * source may run into the bytes being matched), keep the longest valid one,
 * nearest source on ties.  O(n^2) per block; for small inputs only.
 * Output: tokens in order, blocks never straddled; lit = literal bytes. */
int or_encode(const uint8_t* x, uint64_t n, uint32_t log2_bs, const uint32_t thr[4],
              const uint64_t bound[3], uint64_t* ntok_out, uint32_t** lit_len_out,
              uint32_t** mlen_out, uint64_t** src_out, uint8_t** lit_out, uint64_t* nlit_out) {
  if (log2_bs < 4 || log2_bs > 24) return OR_E_INVAL;
  uint64_t bs = 1ULL << log2_bs;
  uint64_t cap = n + 1;
  uint32_t* ll = (uint32_t*)malloc(sizeof(uint32_t) * cap);
  uint32_t* ml = (uint32_t*)malloc(sizeof(uint32_t) * cap);
  uint64_t* sr = (uint64_t*)malloc(sizeof(uint64_t) * cap);
  uint8_t* lt = (uint8_t*)malloc(n + 1);
  if (!ll || !ml || !sr || !lt) { free(ll); free(ml); free(sr); free(lt); return OR_E_NOMEM; }
  uint64_t nt = 0, nl = 0;
  for (uint64_t b0 = 0; b0 < n; b0 += bs) {
    uint64_t end = (b0 + bs < n) ? b0 + bs : n;
    uint64_t pos = b0, run = 0;
    while (pos < end) {
      uint64_t best_len = 0, best_src = 0;
      for (uint64_t s1 = pos; s1 > 0; --s1) {
        uint64_t src = s1 - 1; /* nearest first */
        uint64_t L = 0;
        while (pos + L < end && x[src + L] == x[pos + L]) ++L;
        if (L >= thr[dist_class(pos - src, bound)] && L > best_len) {
          best_len = L;
          best_src = src;
        }
      }
      if (best_len > 0) {
        ll[nt] = (uint32_t)run;
        ml[nt] = (uint32_t)best_len;
        sr[nt] = best_src;
        ++nt;
        run = 0;
        pos += best_len;
      } else {
        lt[nl++] = x[pos];
        ++run;
        ++pos;
      }
    }
    if (run > 0) {
      ll[nt] = (uint32_t)run;
      ml[nt] = 0;
      sr[nt] = 0;
      ++nt;
    }
  }
  *ntok_out = nt;
  *lit_len_out = ll;
  *mlen_out = ml;
  *src_out = sr;
  *lit_out = lt;
  *nlit_out = nl;
  return OR_OK;
}

/* ---------------------------------------------------------------- writer */

typedef struct {
  uint8_t* p;
  uint64_t len, cap;
} obuf;

static int ob_reserve(obuf* b, uint64_t more) {
  if (b->len + more <= b->cap) return 0;
  uint64_t nc = b->cap ? b->cap : 1024;
  while (nc < b->len + more) nc *= 2;
  uint8_t* q = (uint8_t*)realloc(b->p, nc);
  if (!q) return -1;
  b->p = q;
  b->cap = nc;
  return 0;
}

static int ob_put(obuf* b, const void* src, uint64_t k) {
  if (ob_reserve(b, k)) return -1;
  memcpy(b->p + b->len, src, k);
  b->len += k;
  return 0;
}

static void put_le(uint8_t* p, uint64_t v, int k) {
  for (int i = 0; i < k; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get_le(const uint8_t* p, int k) {
  uint64_t v = 0;
  for (int i = 0; i < k; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

/* one block-local token after splitting */
typedef struct {
  uint64_t lit_len, mlen, src;
} btok;

/* Serialises a token list.  Tokens may straddle block ends (generated
 * streams); they are cut at every block boundary first: a literal run is
 * split into two runs, a match into two matches whose second source is
 * shifted by the same amount.  min_match = 0 picks the smallest length of
 * any match that is not the last token of its block. */
int or_write_archive(uint64_t n, uint32_t log2_bs, uint32_t min_match, uint64_t ntok,
                     const uint32_t* lit_len, const uint32_t* mlen, const uint64_t* src,
                     const uint8_t* lit, uint64_t nlit, const uint32_t thr[4],
                     const uint64_t bound[3], uint8_t** arc_out, uint64_t* size_out) {
  if (log2_bs < 4 || log2_bs > 24) return OR_E_INVAL;
  uint64_t bs = 1ULL << log2_bs;
  uint64_t nb = (n + bs - 1) / bs;
  /* pass 1: cut tokens into per-block lists */
  uint64_t cap = ntok + 2 * nb + 2;
  btok* bt = (btok*)malloc(sizeof(btok) * cap);
  uint64_t* bstart = (uint64_t*)calloc(nb + 1, sizeof(uint64_t));
  if (!bt || !bstart) { free(bt); free(bstart); return OR_E_NOMEM; }
  uint64_t nbt = 0, pos = 0, litsum = 0;
  uint64_t cur_block = 0;
  btok open = {0, 0, 0};
  int have_open = 0;
#define FLUSH_OPEN()                                   \
  do {                                                  \
    if (nbt == cap) {                                   \
      cap *= 2;                                         \
      bt = (btok*)realloc(bt, sizeof(btok) * cap);      \
    }                                                   \
    bt[nbt++] = open;                                   \
    open.lit_len = open.mlen = open.src = 0;            \
    have_open = 0;                                      \
  } while (0)
  for (uint64_t t = 0; t < ntok; ++t) {
    uint64_t L = lit_len[t];
    litsum += L;
    while (L > 0) {
      uint64_t bend = (cur_block + 1) * bs;
      uint64_t take = (pos + L <= bend) ? L : bend - pos;
      if (have_open && open.mlen > 0) FLUSH_OPEN();
      open.lit_len += take;
      have_open = 1;
      pos += take;
      L -= take;
      if (pos == bend && pos < n) {
        FLUSH_OPEN();
        ++cur_block;
        bstart[cur_block] = nbt;
      }
    }
    uint64_t M = mlen[t], s = src[t];
    while (M > 0) {
      uint64_t bend = (cur_block + 1) * bs;
      uint64_t take = (pos + M <= bend) ? M : bend - pos;
      if (have_open && open.mlen > 0) FLUSH_OPEN();
      open.mlen = take;
      open.src = s;
      have_open = 1;
      pos += take;
      s += take;
      M -= take;
      if (pos == bend && pos < n) {
        FLUSH_OPEN();
        ++cur_block;
        bstart[cur_block] = nbt;
      }
    }
  }
#undef FLUSH_OPEN
  if (have_open) {
    if (nbt == cap) { cap += 1; bt = (btok*)realloc(bt, sizeof(btok) * cap); }
    bt[nbt++] = open;
  }
  if (pos != n || litsum != nlit) { free(bt); free(bstart); return OR_E_INVAL; }
  bstart[nb] = nbt;
  if (nb == 0) nbt = 0;
  /* min_match: smallest non-final match length */
  if (min_match == 0) {
    uint64_t mm = UINT64_MAX;
    for (uint64_t b = 0; b < nb; ++b)
      for (uint64_t i = bstart[b]; i + 1 < bstart[b + 1]; ++i)
        if (bt[i].mlen < mm) mm = bt[i].mlen;
    min_match = (mm == UINT64_MAX) ? 1 : (uint32_t)mm;
    if (min_match == 0) min_match = 1;
  }
  int hi = n > 0xFFFFFFFFULL;
  /* pass 2: streams */
  obuf cmd = {0}, x16 = {0}, x32 = {0}, slo = {0}, shi = {0};
  uint64_t* tab = (uint64_t*)calloc(4 * (nb + 1), sizeof(uint64_t));
  uint64_t litpos = 0;
  int err = 0;
  for (uint64_t b = 0; b < nb && !err; ++b) {
    tab[4 * b + 0] = bstart[b];
    tab[4 * b + 1] = litpos;
    tab[4 * b + 2] = x16.len / 2;
    tab[4 * b + 3] = x32.len / 4;
    for (uint64_t i = bstart[b]; i < bstart[b + 1]; ++i) {
      int last = (i + 1 == bstart[b + 1]);
      uint64_t lv = bt[i].lit_len;
      uint64_t mv = 0;
      if (!last) {
        if (bt[i].mlen < min_match) { err = 1; break; }
        mv = bt[i].mlen - min_match;
      }
      uint8_t lc = lv < 15 ? (uint8_t)lv : 15, mc = mv < 15 ? (uint8_t)mv : 15;
      uint8_t c = (uint8_t)((lc << 4) | mc);
      ob_put(&cmd, &c, 1);
      uint64_t vals[2] = {lv, mv};
      for (int k = 0; k < 2; ++k) {
        if (vals[k] < 15) continue;
        uint64_t v = vals[k] - 15;
        uint8_t t2[2], t4[4];
        if (v < 0xFFFF) {
          put_le(t2, v, 2);
          ob_put(&x16, t2, 2);
        } else {
          put_le(t2, 0xFFFF, 2);
          ob_put(&x16, t2, 2);
          put_le(t4, v - 0xFFFF, 4);
          ob_put(&x32, t4, 4);
        }
      }
      uint64_t s = bt[i].mlen ? bt[i].src : 0;
      uint8_t t4[4];
      put_le(t4, s & 0xFFFFFFFFULL, 4);
      ob_put(&slo, t4, 4);
      uint8_t h = (uint8_t)(s >> 32);
      ob_put(&shi, &h, 1);
      litpos += lv;
    }
  }
  if (!err) {
    tab[4 * nb + 0] = nbt;
    tab[4 * nb + 1] = litpos;
    tab[4 * nb + 2] = x16.len / 2;
    tab[4 * nb + 3] = x32.len / 4;
  }
  /* pass 3: assemble */
  obuf a = {0};
  uint8_t hdr[HDR];
  memset(hdr, 0, sizeof(hdr));
  put_le(hdr + 0, MAGIC, 4);
  put_le(hdr + 4, 1, 4);
  put_le(hdr + 8, n, 8);
  put_le(hdr + 16, log2_bs, 4);
  put_le(hdr + 20, nb, 4);
  put_le(hdr + 24, min_match, 4);
  put_le(hdr + 28, hi ? 1 : 0, 4);
  put_le(hdr + 32, nbt, 8);
  put_le(hdr + 40, x16.len / 2, 8);
  put_le(hdr + 48, x32.len / 4, 8);
  put_le(hdr + 56, nlit, 8);
  for (int k = 0; k < 4; ++k) hdr[64 + k] = (uint8_t)(thr ? (thr[k] > 255 ? 255 : thr[k]) : 0);
  for (int k = 0; k < 3; ++k) put_le(hdr + 72 + 8 * k, bound ? bound[k] : 0, 8);
  ob_put(&a, hdr, HDR);
  for (uint64_t i = 0; i < 4 * (nb + 1); ++i) {
    uint8_t t8[8];
    put_le(t8, tab[i], 8);
    ob_put(&a, t8, 8);
  }
  static const uint8_t zeros[16] = {0};
#define ALIGN16() ob_put(&a, zeros, (16 - (a.len & 15)) & 15)
  ALIGN16();
  ob_put(&a, cmd.p, cmd.len);
  ALIGN16();
  ob_put(&a, x16.p, x16.len);
  ALIGN16();
  ob_put(&a, x32.p, x32.len);
  ALIGN16();
  ob_put(&a, slo.p, slo.len);
  ALIGN16();
  if (hi) {
    ob_put(&a, shi.p, shi.len);
    ALIGN16();
  }
  ob_put(&a, lit, nlit);
  ALIGN16();
  ob_put(&a, zeros, 16);
#undef ALIGN16
  free(cmd.p); free(x16.p); free(x32.p); free(slo.p); free(shi.p);
  free(tab); free(bt); free(bstart);
  if (err) { free(a.p); return OR_E_INVAL; }
  *arc_out = a.p;
  *size_out = a.len;
  return OR_OK;
}

/* ---------------------------------------------------------------- reader */

typedef struct {
  uint64_t n, bs, nb, min_match, flags, n_tok, n_x16, n_x32, n_lit;
  const uint8_t *tab, *cmd, *x16, *x32, *slo, *shi, *lit, *info;
  uint64_t size_needed;
} view_t;

static uint64_t up16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

static int open_view(const uint8_t* a, uint64_t size, view_t* v) {
  if (size < HDR) return OR_E_CORRUPT;
  if (get_le(a, 4) != MAGIC || get_le(a + 4, 4) != 1) return OR_E_CORRUPT;
  v->n = get_le(a + 8, 8);
  if (v->n > (1ULL << 48)) return OR_E_CORRUPT;
  uint64_t lb = get_le(a + 16, 4);
  if (lb < 4 || lb > 24) return OR_E_CORRUPT;
  v->bs = 1ULL << lb;
  v->nb = get_le(a + 20, 4);
  if (v->nb != (v->n + v->bs - 1) / v->bs) return OR_E_CORRUPT;
  v->min_match = get_le(a + 24, 4);
  if (v->min_match < 1) return OR_E_CORRUPT;
  v->flags = get_le(a + 28, 4);
  if (v->flags & ~3ULL) return OR_E_CORRUPT;
  v->n_tok = get_le(a + 32, 8);
  v->n_x16 = get_le(a + 40, 8);
  v->n_x32 = get_le(a + 48, 8);
  v->n_lit = get_le(a + 56, 8);
  if (v->n_tok > v->n || v->n_lit > v->n || v->n_x16 > 2 * v->n_tok || v->n_x32 > v->n_x16)
    return OR_E_CORRUPT;
  uint64_t off = HDR;
  v->tab = a + off;
  off = up16(off + 32 * (v->nb + 1));
  v->cmd = a + off;
  off = up16(off + v->n_tok);
  v->x16 = a + off;
  off = up16(off + 2 * v->n_x16);
  v->x32 = a + off;
  off = up16(off + 4 * v->n_x32);
  v->slo = a + off;
  off = up16(off + 4 * v->n_tok);
  v->shi = 0;
  if (v->flags & 1) {
    v->shi = a + off;
    off = up16(off + v->n_tok);
  }
  v->lit = a + off;
  off = up16(off + v->n_lit);
  v->info = 0;
  if (v->flags & 2) {
    v->info = a + off;
    off = up16(off + v->nb);
  }
  off += 16;
  v->size_needed = off;
  if (size < off) return OR_E_CORRUPT;
  /* table: monotone, starts at zero, ends at the totals */
  for (int k = 0; k < 4; ++k)
    if (get_le(v->tab + 8 * k, 8) != 0) return OR_E_CORRUPT;
  const uint64_t tot[4] = {v->n_tok, v->n_lit, v->n_x16, v->n_x32};
  for (int k = 0; k < 4; ++k)
    if (get_le(v->tab + 32 * v->nb + 8 * k, 8) != tot[k]) return OR_E_CORRUPT;
  for (uint64_t b = 0; b < v->nb; ++b)
    for (int k = 0; k < 4; ++k)
      if (get_le(v->tab + 32 * (b + 1) + 8 * k, 8) < get_le(v->tab + 32 * b + 8 * k, 8))
        return OR_E_CORRUPT;
  return OR_OK;
}

/* Offset and length of the literal stream inside a valid archive. */
int or_lit_stream(const uint8_t* arc, uint64_t size, uint64_t* off, uint64_t* n_lit) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  *off = (uint64_t)(v.lit - arc);
  *n_lit = v.n_lit;
  return OR_OK;
}

/* Walks every token of every block, checking the container rules; calls
 * `visit` (if given) with the decoded token.  Returns 0 or OR_E_CORRUPT. */
typedef void (*visit_fn)(void* ctx, uint64_t block, uint64_t t, uint64_t dst, uint64_t lit_len,
                         uint64_t lit_off, uint64_t mlen, uint64_t src);

static int walk(const view_t* v, visit_fn visit, void* ctx) {
  for (uint64_t b = 0; b < v->nb; ++b) {
    const uint8_t* e0 = v->tab + 32 * b;
    const uint8_t* e1 = v->tab + 32 * (b + 1);
    uint64_t t0 = get_le(e0, 8), t1 = get_le(e1, 8);
    uint64_t lc = get_le(e0 + 8, 8), lc1 = get_le(e1 + 8, 8);
    uint64_t xc = get_le(e0 + 16, 8), xc1 = get_le(e1 + 16, 8);
    uint64_t yc = get_le(e0 + 24, 8), yc1 = get_le(e1 + 24, 8);
    uint64_t pos = b * v->bs;
    uint64_t end = pos + v->bs < v->n ? pos + v->bs : v->n;
    if (t1 <= t0) return OR_E_CORRUPT; /* a non-empty block has a token */
    for (uint64_t t = t0; t < t1; ++t) {
      uint8_t c = v->cmd[t];
      uint64_t val[2] = {(uint64_t)(c >> 4), (uint64_t)(c & 15)};
      for (int k = 0; k < 2; ++k) {
        if (val[k] < 15) continue;
        if (xc >= xc1) return OR_E_CORRUPT;
        uint64_t e = get_le(v->x16 + 2 * xc, 2);
        ++xc;
        if (e == 0xFFFF) {
          if (yc >= yc1) return OR_E_CORRUPT;
          e += get_le(v->x32 + 4 * yc, 4);
          ++yc;
        }
        val[k] = 15 + e;
      }
      uint64_t lit_len = val[0];
      int last = (t + 1 == t1);
      if (lit_len > end - pos) return OR_E_CORRUPT;
      if (lit_len > lc1 - lc) return OR_E_CORRUPT;
      uint64_t dst = pos + lit_len;
      uint64_t mlen;
      if (last) {
        if ((c & 15) != 0) return OR_E_CORRUPT;
        mlen = end - dst;
      } else {
        mlen = v->min_match + val[1];
        if (mlen > end - dst) return OR_E_CORRUPT;
      }
      uint64_t src = get_le(v->slo + 4 * t, 4);
      if (v->shi) src |= (uint64_t)v->shi[t] << 32;
      if (mlen > 0 && src >= dst) return OR_E_CORRUPT;
      if (mlen == 0 && src != 0) return OR_E_CORRUPT;
      if (visit) visit(ctx, b, t, pos, lit_len, lc, mlen, src);
      lc += lit_len;
      pos = dst + mlen;
    }
    if (pos != end || lc != lc1 || xc != xc1 || yc != yc1) return OR_E_CORRUPT;
  }
  return OR_OK;
}

typedef struct {
  const view_t* v;
  uint8_t* out;
} dec_ctx;

static void dec_visit(void* ctx, uint64_t block, uint64_t t, uint64_t dst, uint64_t lit_len,
                      uint64_t lit_off, uint64_t mlen, uint64_t src) {
  (void)block;
  (void)t;
  dec_ctx* d = (dec_ctx*)ctx;
  for (uint64_t i = 0; i < lit_len; ++i) d->out[dst + i] = d->v->lit[lit_off + i];
  uint64_t m0 = dst + lit_len;
  for (uint64_t i = 0; i < mlen; ++i) d->out[m0 + i] = d->out[src + i];
}

/* Validates and decodes the whole archive into out[0, n). */
int or_decode(const uint8_t* arc, uint64_t size, uint8_t* out, uint64_t cap) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  if (cap < v.n) return OR_E_INVAL;
  rc = walk(&v, 0, 0); /* validate before writing anything */
  if (rc) return rc;
  dec_ctx d = {&v, out};
  return walk(&v, dec_visit, &d);
}

int or_info(const uint8_t* arc, uint64_t size, uint64_t* n, uint64_t* nb, uint64_t* ntok,
            uint64_t* log2_bs, uint64_t* min_match) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  *n = v.n;
  *nb = v.nb;
  *ntok = v.n_tok;
  uint64_t lb = 0;
  while ((1ULL << lb) < v.bs) ++lb;
  *log2_bs = lb;
  *min_match = v.min_match;
  return OR_OK;
}

/* ------------------------------------------------------------- tokens out */

typedef struct {
  uint64_t *blk, *dst, *lit_len, *lit_off, *mlen, *src;
} tok_ctx;

static void tok_visit(void* ctx, uint64_t block, uint64_t t, uint64_t dst, uint64_t lit_len,
                      uint64_t lit_off, uint64_t mlen, uint64_t src) {
  tok_ctx* c = (tok_ctx*)ctx;
  c->blk[t] = block;
  c->dst[t] = dst;
  c->lit_len[t] = lit_len;
  c->lit_off[t] = lit_off;
  c->mlen[t] = mlen;
  c->src[t] = src;
}

/* Per token: block, token start, literal length, literal stream offset,
 * match length, match source.  Arrays sized n_tok by the caller. */
int or_tokens(const uint8_t* arc, uint64_t size, uint64_t* blk, uint64_t* dst, uint64_t* lit_len,
              uint64_t* lit_off, uint64_t* mlen, uint64_t* src) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  tok_ctx c = {blk, dst, lit_len, lit_off, mlen, src};
  return walk(&v, tok_visit, &c);
}

/* ------------------------------------------------------------- levels */

typedef struct {
  uint32_t* byte_depth; /* depth of the token part that wrote each output byte */
  uint32_t* tok_depth;
  uint32_t max_depth;
} lvl_ctx;

static void lvl_visit(void* ctx, uint64_t block, uint64_t t, uint64_t dst, uint64_t lit_len,
                      uint64_t lit_off, uint64_t mlen, uint64_t src) {
  (void)lit_off;
  (void)block;
  lvl_ctx* c = (lvl_ctx*)ctx;
  uint64_t m0 = dst + lit_len;
  for (uint64_t i = 0; i < lit_len; ++i) c->byte_depth[dst + i] = 0;
  uint32_t dep = 0;
  if (mlen > 0) {
    uint32_t deepest = 0;
    uint64_t src_end = src + mlen < m0 ? src + mlen : m0; /* own bytes excluded */
    for (uint64_t q = src; q < src_end; ++q)
      if (c->byte_depth[q] > deepest) deepest = c->byte_depth[q];
    dep = deepest + 1;
  }
  for (uint64_t i = 0; i < mlen; ++i) c->byte_depth[m0 + i] = dep;
  c->tok_depth[t] = dep;
  if (dep > c->max_depth) c->max_depth = dep;
}

/* Depth of every token's match (0 for tokens without a match). */
int or_levels(const uint8_t* arc, uint64_t size, uint32_t* tok_level, uint32_t* max_level) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  rc = walk(&v, 0, 0);
  if (rc) return rc;
  lvl_ctx c;
  c.byte_depth = (uint32_t*)malloc(sizeof(uint32_t) * (v.n + 1));
  c.tok_depth = tok_level;
  c.max_depth = 0;
  if (!c.byte_depth) return OR_E_NOMEM;
  rc = walk(&v, lvl_visit, &c);
  free(c.byte_depth);
  *max_level = c.max_depth;
  return rc;
}

/* ------------------------------------------------------------- entropy */

/* Order-0 entropy size of a byte sequence cut into 64 KiB tiles: per tile
 * ceil(N*H/8) bytes plus a table charge of 1 + 2*(distinct symbols). */
static double tiles_size(const uint8_t* p, uint64_t len) {
  const uint64_t T = 65536;
  double total = 0.0;
  for (uint64_t o = 0; o < len; o += T) {
    uint64_t m = (len - o < T) ? len - o : T;
    uint64_t cnt[256];
    memset(cnt, 0, sizeof(cnt));
    for (uint64_t i = 0; i < m; ++i) cnt[p[o + i]]++;
    double bits = 0.0;
    int distinct = 0;
    for (int s = 0; s < 256; ++s) {
      if (!cnt[s]) continue;
      ++distinct;
      double q = (double)cnt[s] / (double)m;
      bits -= (double)cnt[s] * log2(q);
    }
    total += ceil(bits / 8.0 - 1e-9) + 1.0 + 2.0 * distinct;
  }
  return total;
}

/* Entropy-bound size in bytes: header + block table verbatim, and the
 * streams cmd, x16 (as bytes), x32 (as bytes), each byte plane of the
 * sources, lit at their tile entropy.  parts[7] (optional): cmd, x16, x32,
 * src planes (sum), lit, header+table, src_hi plane. */
int or_entropy_size(const uint8_t* arc, uint64_t size, double* total, double* parts) {
  view_t v;
  int rc = open_view(arc, size, &v);
  if (rc) return rc;
  double p[7] = {0};
  p[0] = tiles_size(v.cmd, v.n_tok);
  p[1] = tiles_size(v.x16, 2 * v.n_x16);
  p[2] = tiles_size(v.x32, 4 * v.n_x32);
  uint8_t* plane = (uint8_t*)malloc(v.n_tok + 1);
  if (!plane) return OR_E_NOMEM;
  for (int k = 0; k < 4; ++k) {
    for (uint64_t t = 0; t < v.n_tok; ++t) plane[t] = v.slo[4 * t + k];
    p[3] += tiles_size(plane, v.n_tok);
  }
  if (v.shi) p[6] = tiles_size(v.shi, v.n_tok);
  free(plane);
  p[4] = tiles_size(v.lit, v.n_lit);
  p[5] = (double)HDR + 32.0 * (double)(v.nb + 1);
  double s = 0;
  for (int k = 0; k < 7; ++k) s += p[k];
  *total = s;
  if (parts)
    for (int k = 0; k < 7; ++k) parts[k] = p[k];
  return OR_OK;
}

/* ------------------------------------------------------------- pure copy */

/* Executes pre-decoded tokens in order: lit_len bytes from lit[lit_off..]
 * to out[dst..], then mlen bytes from ref[src..] to out[dst+lit_len..]. */
void or_purecopy(uint64_t ntok, const uint64_t* dst, const uint64_t* lit_off,
                 const uint32_t* lit_len, const uint64_t* src, const uint32_t* mlen,
                 const uint8_t* lit, const uint8_t* ref, uint8_t* out) {
  for (uint64_t t = 0; t < ntok; ++t) {
    for (uint64_t i = 0; i < lit_len[t]; ++i) out[dst[t] + i] = lit[lit_off[t] + i];
    uint64_t m0 = dst[t] + lit_len[t];
    for (uint64_t i = 0; i < mlen[t]; ++i) out[m0 + i] = ref[src[t] + i];
  }
}

/* Executes an unsplit token stream (as generated) into out[0,n). */
int or_exec_tokens(uint64_t n, uint64_t ntok, const uint32_t* lit_len, const uint32_t* mlen,
                   const uint64_t* src, const uint8_t* lit, uint64_t nlit, uint8_t* out) {
  uint64_t pos = 0, lo = 0;
  for (uint64_t t = 0; t < ntok; ++t) {
    if (pos + lit_len[t] > n || lo + lit_len[t] > nlit) return OR_E_INVAL;
    for (uint64_t i = 0; i < lit_len[t]; ++i) out[pos + i] = lit[lo + i];
    pos += lit_len[t];
    lo += lit_len[t];
    if (mlen[t] && (src[t] >= pos || pos + mlen[t] > n)) return OR_E_INVAL;
    for (uint64_t i = 0; i < mlen[t]; ++i) out[pos + i] = out[src[t] + i];
    pos += mlen[t];
  }
  return pos == n ? OR_OK : OR_E_INVAL;
}
