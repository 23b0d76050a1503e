/*
 * lz_rans.c -- plain sequential CPU oracle of the tile-rANS entropy stage.
 *
 * TEST INFRASTRUCTURE ONLY (see lz_oracle.c): loaded by the test suite and
 * the bench's CPU-baseline leg; shares nothing with the product library.
 *
 * The paper decodes entropy over 64 KB tiles cut across each flat stream
 * independently of the LZ block size, ahead of the match phase (Sec. 2,
 * Experimental Setup), and names the coder tile-ANS without further detail.
 * This file writes out, one symbol at a time, the range variant of
 * asymmetric numeral systems (rANS, Duda) with the parameters this build
 * reads into it (each choice listed):
 *   - alphabet: bytes; tile = at most 65,536 consecutive symbols of a region;
 *   - quantised frequencies, total M = 4096: f[s] = floor(count[s] * M / N),
 *     every present symbol at least 1; the sum is then made exactly M on the
 *     most frequent symbol (lowest byte among equal counts): a shortfall is
 *     added to it, an excess is removed one unit at a time from the symbol
 *     with the largest f above 1 (lowest byte among equals);
 *     c[s] = f[0] + ... + f[s-1];
 *   - 64 interleaved states; symbol i belongs to state i mod 64;
 *   - state x in [L, 2^32), L = 2^16, renormalised by 16-bit words.
 *   Encoding symbol s into x (symbols taken from i = N-1 down to 0): if
 *     x >= f[s] * 2^20, output the word x mod 2^16 and set x = x div 2^16;
 *     then x = (x div f[s]) * M + (x mod f[s]) + c[s].  All states start at L.
 *   Decoding (i = 0 up to N-1, state j = i mod 64): r = x mod M; s is the
 *     symbol with c[s] <= r < c[s] + f[s]; x = f[s] * (x div M) + r - c[s];
 *     if x < L then x = x * 2^16 + the next word.  The decoder reads the
 *     words in the reverse of the order the encoder wrote them.
 *   Payload: 32-byte bitmap of present symbols (bit s of byte s/8), u16 f of
 *   each present symbol (ascending), u32 final encoder state per lane (the
 *   decoder's start), u16 words in decoding order.
 *
 * Coded container (also this build's reading; every integer little-endian):
 *   [0, 64): "LZE1" and 4 zero bytes, u64 decoded size, u32 tile count,
 *   u32 0, u64 192 (directory offset), u64 payload offset (192 + 32 tiles),
 *   u64 total size, 16 zero bytes; [64, 192): the decoded container's first
 *   128 bytes; directory: per tile u64 payload offset (from the payload
 *   start), u64 first output byte, u32 symbols, u32 payload bytes, u32
 *   output stride, u32 mode (0 raw bytes, 1 rANS, 2 one repeated byte).
 *   Regions of the decoded container, in order: bytes [0, src_lo start);
 *   then byte k (k = 0..3) of every 32-bit source as its own region (stride
 *   4) when there are tokens; then the remaining bytes.  Each region is cut
 *   into tiles of 65,536 symbols (the last shorter), and a tile takes the
 *   mode of the smallest payload: repeated if all its bytes are equal, else
 *   rANS when its payload is smaller than the tile, else raw.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RO_OK 0
#define RO_E_INVAL (-1)
#define RO_E_CORRUPT (-2)
#define RO_E_NOMEM (-4)

enum { TILE = 65536, M = 4096, LANES = 64 };
static const uint64_t L_LOW = 1u << 16;

static uint64_t rd(const uint8_t* p, int k) {
  uint64_t v = 0;
  for (int i = 0; i < k; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

static void wr(uint8_t* p, uint64_t v, int k) {
  for (int i = 0; i < k; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

/* Quantised frequencies of N symbols with the given counts; 0 if none. */
int or_rans_normalise(const uint64_t* count, uint64_t N, uint32_t* f) {
  uint64_t sum = 0;
  int top = -1;
  for (int s = 0; s < 256; ++s) {
    f[s] = 0;
    if (count[s] == 0) continue;
    f[s] = (uint32_t)(count[s] * M / N);
    if (f[s] < 1) f[s] = 1;
    sum += f[s];
    if (top < 0 || count[s] > count[top]) top = s;
  }
  if (top < 0) return 0;
  if (sum < M) f[top] += (uint32_t)(M - sum);
  while (sum > M) {
    int big = -1;
    for (int s = 0; s < 256; ++s)
      if (f[s] > 1 && (big < 0 || f[s] > f[big])) big = s;
    if (big < 0) return 0;
    f[big] -= 1;
    sum -= 1;
  }
  return 1;
}

/* rANS payload of N symbols sym[0], sym[stride], ...; returns its size (0 on
 * failure).  *out is malloc'd. */
uint64_t or_rans_encode_tile(const uint8_t* sym, uint64_t stride, uint64_t N, uint8_t** out) {
  uint64_t count[256] = {0};
  for (uint64_t i = 0; i < N; ++i) count[sym[i * stride]] += 1;
  uint32_t f[256], c[256], acc = 0;
  if (!or_rans_normalise(count, N, f)) return 0;
  for (int s = 0; s < 256; ++s) {
    c[s] = acc;
    acc += f[s];
  }
  uint64_t x[LANES];
  for (int j = 0; j < LANES; ++j) x[j] = L_LOW;
  uint16_t* words = (uint16_t*)malloc(sizeof(uint16_t) * (N + 1));
  if (!words) return 0;
  uint64_t nw = 0;
  for (uint64_t k = N; k > 0; --k) {
    const uint64_t i = k - 1;
    const uint32_t s = sym[i * stride];
    const int j = (int)(i % LANES);
    if (x[j] >= ((uint64_t)f[s] << 20)) {
      words[nw++] = (uint16_t)(x[j] & 0xFFFF);
      x[j] >>= 16;
    }
    x[j] = (x[j] / f[s]) * M + (x[j] % f[s]) + c[s];
  }
  int nsym = 0;
  for (int s = 0; s < 256; ++s) nsym += f[s] ? 1 : 0;
  const uint64_t size = 32 + 2 * (uint64_t)nsym + 4 * LANES + 2 * nw;
  uint8_t* p = (uint8_t*)calloc(size, 1);
  if (!p) {
    free(words);
    return 0;
  }
  uint64_t o = 32;
  for (int s = 0; s < 256; ++s)
    if (f[s]) {
      p[s / 8] |= (uint8_t)(1u << (s % 8));
      wr(p + o, f[s], 2);
      o += 2;
    }
  for (int j = 0; j < LANES; ++j, o += 4) wr(p + o, x[j], 4);
  for (uint64_t w = 0; w < nw; ++w, o += 2) wr(p + o, words[nw - 1 - w], 2); /* decoding order */
  free(words);
  *out = p;
  return size;
}

/* Decodes an rANS payload of `size` bytes into N symbols at out[0],
 * out[stride], ...; checks the tables and that every state ends at L. */
int or_rans_decode_tile(const uint8_t* p, uint64_t size, uint64_t N, uint8_t* out, uint64_t stride) {
  if (size < 32) return RO_E_CORRUPT;
  uint32_t f[256], c[256], acc = 0;
  uint64_t o = 32;
  for (int s = 0; s < 256; ++s) {
    f[s] = 0;
    if ((p[s / 8] >> (s % 8)) & 1) {
      if (o + 2 > size) return RO_E_CORRUPT;
      f[s] = (uint32_t)rd(p + o, 2);
      o += 2;
      if (f[s] == 0) return RO_E_CORRUPT;
    }
    c[s] = acc;
    acc += f[s];
  }
  if (acc != M || o + 4 * LANES > size) return RO_E_CORRUPT;
  uint64_t x[LANES];
  for (int j = 0; j < LANES; ++j, o += 4) {
    x[j] = rd(p + o, 4);
    if (x[j] < L_LOW) return RO_E_CORRUPT;
  }
  if ((size - o) % 2) return RO_E_CORRUPT;
  const uint64_t nw = (size - o) / 2;
  uint64_t w = 0;
  for (uint64_t i = 0; i < N; ++i) {
    const int j = (int)(i % LANES);
    const uint32_t r = (uint32_t)(x[j] % M);
    int s = 0;
    while (!(c[s] <= r && r < c[s] + f[s])) ++s;
    out[i * stride] = (uint8_t)s;
    x[j] = f[s] * (x[j] / M) + r - c[s];
    if (x[j] < L_LOW) {
      if (w >= nw) return RO_E_CORRUPT;
      x[j] = (x[j] << 16) | rd(p + o + 2 * w, 2);
      ++w;
    }
  }
  if (w != nw) return RO_E_CORRUPT;
  for (int j = 0; j < LANES; ++j)
    if (x[j] != L_LOW) return RO_E_CORRUPT;
  return RO_OK;
}

typedef struct {
  uint64_t dst, count, stride;
} region_t;

static uint64_t up16(uint64_t v) { return (v + 15) & ~(uint64_t)15; }

/* src_lo offset and total size of a container, from its header. */
static int layout_of(const uint8_t* a, uint64_t size, uint64_t* off_slo, uint64_t* n_tok, uint64_t* total) {
  if (size < 128 || rd(a, 4) != 0x314D5A4Cu) return RO_E_CORRUPT;
  const uint64_t nb = rd(a + 20, 4), flags = rd(a + 28, 4), nt = rd(a + 32, 8), n16 = rd(a + 40, 8),
                 n32 = rd(a + 48, 8), nl = rd(a + 56, 8);
  uint64_t off = up16(128 + 32 * (nb + 1));
  off = up16(off + nt);
  off = up16(off + 2 * n16);
  off = up16(off + 4 * n32);
  *off_slo = off;
  off = up16(off + 4 * nt);
  if (flags & 1) off = up16(off + nt);
  off = up16(off + nl);
  if (flags & 2) off = up16(off + nb);
  *total = off + 16;
  *n_tok = nt;
  return *total <= size ? RO_OK : RO_E_CORRUPT;
}

int or_entropy_encode(const uint8_t* a, uint64_t size, uint8_t** out, uint64_t* out_size) {
  uint64_t slo, nt, total;
  if (layout_of(a, size, &slo, &nt, &total)) return RO_E_CORRUPT;
  region_t R[6];
  int nr = 0;
  if (slo) R[nr++] = (region_t){0, slo, 1};
  uint64_t pos = slo;
  if (nt) {
    for (int k = 0; k < 4; ++k) R[nr++] = (region_t){slo + k, nt, 4};
    pos = slo + 4 * nt;
  }
  if (total > pos) R[nr++] = (region_t){pos, total - pos, 1};
  uint64_t ntiles = 0;
  for (int r = 0; r < nr; ++r) ntiles += (R[r].count + TILE - 1) / TILE;
  uint8_t** pay = (uint8_t**)calloc(ntiles ? ntiles : 1, sizeof(uint8_t*));
  uint64_t* psz = (uint64_t*)calloc(ntiles ? ntiles : 1, sizeof(uint64_t));
  uint64_t* rec = (uint64_t*)calloc(ntiles ? 4 * ntiles : 1, sizeof(uint64_t)); /* dst, count, stride, mode */
  if (!pay || !psz || !rec) return RO_E_NOMEM;
  uint64_t t = 0, paytot = 0;
  for (int r = 0; r < nr; ++r)
    for (uint64_t i0 = 0; i0 < R[r].count; i0 += TILE, ++t) {
      const uint64_t cnt = R[r].count - i0 < TILE ? R[r].count - i0 : TILE, st = R[r].stride;
      const uint8_t* s = a + R[r].dst + i0 * st;
      rec[4 * t] = R[r].dst + i0 * st;
      rec[4 * t + 1] = cnt;
      rec[4 * t + 2] = st;
      int same = 1;
      for (uint64_t i = 1; i < cnt; ++i)
        if (s[i * st] != s[0]) same = 0;
      if (same) {
        rec[4 * t + 3] = 2;
        pay[t] = (uint8_t*)malloc(1);
        pay[t][0] = s[0];
        psz[t] = 1;
      } else {
        uint8_t* q = 0;
        const uint64_t qs = or_rans_encode_tile(s, st, cnt, &q);
        if (qs && qs < cnt) {
          rec[4 * t + 3] = 1;
          pay[t] = q;
          psz[t] = qs;
        } else {
          free(q);
          rec[4 * t + 3] = 0;
          pay[t] = (uint8_t*)malloc(cnt);
          for (uint64_t i = 0; i < cnt; ++i) pay[t][i] = s[i * st];
          psz[t] = cnt;
        }
      }
      paytot += psz[t];
    }
  const uint64_t p0 = 192 + 32 * ntiles, tot = p0 + paytot;
  uint8_t* c = (uint8_t*)calloc(tot, 1);
  if (!c) return RO_E_NOMEM;
  memcpy(c, "LZE1", 4);
  wr(c + 8, total, 8);
  wr(c + 16, ntiles, 4);
  wr(c + 24, 192, 8);
  wr(c + 32, p0, 8);
  wr(c + 40, tot, 8);
  memcpy(c + 64, a, 128);
  uint64_t po = 0;
  for (t = 0; t < ntiles; ++t) {
    uint8_t* d = c + 192 + 32 * t;
    wr(d, po, 8);
    wr(d + 8, rec[4 * t], 8);
    wr(d + 16, rec[4 * t + 1], 4);
    wr(d + 20, psz[t], 4);
    wr(d + 24, rec[4 * t + 2], 4);
    wr(d + 28, rec[4 * t + 3], 4);
    memcpy(c + p0 + po, pay[t], psz[t]);
    po += psz[t];
    free(pay[t]);
  }
  free(pay);
  free(psz);
  free(rec);
  *out = c;
  *out_size = tot;
  return RO_OK;
}

/* Decodes a coded container into out[0, cap); every output byte must be
 * written exactly once. */
int or_entropy_decode(const uint8_t* c, uint64_t size, uint8_t* out, uint64_t cap, uint64_t* out_size) {
  if (size < 192 || memcmp(c, "LZE1\0\0\0\0", 8) != 0) return RO_E_CORRUPT;
  const uint64_t total = rd(c + 8, 8), nt = rd(c + 16, 4), p0 = rd(c + 32, 8);
  if (rd(c + 24, 8) != 192 || p0 != 192 + 32 * nt || rd(c + 40, 8) != size || total > cap) return RO_E_CORRUPT;
  uint8_t* seen = (uint8_t*)calloc(total ? total : 1, 1);
  if (!seen) return RO_E_NOMEM;
  int rc = RO_OK;
  for (uint64_t t = 0; t < nt && rc == RO_OK; ++t) {
    const uint8_t* d = c + 192 + 32 * t;
    const uint64_t po = rd(d, 8), dst = rd(d + 8, 8), cnt = rd(d + 16, 4), pb = rd(d + 20, 4), st = rd(d + 24, 4),
                   mode = rd(d + 28, 4);
    if (cnt == 0 || cnt > TILE || (st != 1 && st != 4) || p0 + po + pb > size || dst + (cnt - 1) * st >= total) {
      rc = RO_E_CORRUPT;
      break;
    }
    for (uint64_t i = 0; i < cnt; ++i) {
      if (seen[dst + i * st]) rc = RO_E_CORRUPT;
      seen[dst + i * st] = 1;
    }
    const uint8_t* p = c + p0 + po;
    if (mode == 0 && pb == cnt) {
      for (uint64_t i = 0; i < cnt; ++i) out[dst + i * st] = p[i];
    } else if (mode == 2 && pb == 1) {
      for (uint64_t i = 0; i < cnt; ++i) out[dst + i * st] = p[0];
    } else if (mode == 1) {
      if (or_rans_decode_tile(p, pb, cnt, out + dst, st) != RO_OK) rc = RO_E_CORRUPT;
    } else {
      rc = RO_E_CORRUPT;
    }
  }
  for (uint64_t i = 0; i < total && rc == RO_OK; ++i)
    if (!seen[i]) rc = RO_E_CORRUPT;
  free(seen);
  if (rc == RO_OK) *out_size = total;
  return rc;
}
