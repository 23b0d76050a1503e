/*
 * synth.c -- seeded synthetic input generators.
 *
 * This module produces inputs only: text, FASTQ-like records, byte streams
 * and token lists whose statistics follow the workloads the paper measures
 * (Zipf-distributed text in place of enwik9/Silesia, FASTQ reads in place of
 * the NA12878 / ERR194147 run, and match-length-controlled token streams in
 * place of the synthetic copy sweep of Table II).  It contains none of the
 * codec's arithmetic: no parsing, no container layout, no decoding.  Both the
 * CPU oracle and the GPU path take their inputs from here.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood) seeds xoshiro256**
 * (Blackman, Vigna); both written from their published definitions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s[4]; int have_spare; double spare; } rng_t;

static uint64_t splitmix64(uint64_t* x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static void rng_seed(rng_t* r, uint64_t seed) {
  uint64_t x = seed;
  for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
  r->have_spare = 0;
  r->spare = 0.0;
}

static inline uint64_t rng_next(rng_t* r) {
  uint64_t* s = r->s;
  const uint64_t result = rotl64(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl64(s[3], 45);
  return result;
}

/* uniform double in [0,1) with 53 random bits */
static inline double rng_unit(rng_t* r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform integer in [0,k) by the multiply-high method (bias < 2^-64*k) */
static inline uint64_t rng_below(rng_t* r, uint64_t k) {
  return (uint64_t)(((__uint128_t)rng_next(r) * (__uint128_t)k) >> 64);
}

/* standard normal, Box-Muller with a cached second variate */
static double rng_normal(rng_t* r) {
  if (r->have_spare) { r->have_spare = 0; return r->spare; }
  double u1 = 1.0 - rng_unit(r); /* (0,1] */
  double u2 = rng_unit(r);
  double rad = sqrt(-2.0 * log(u1));
  double th = 6.283185307179586 * u2;
  r->spare = rad * sin(th);
  r->have_spare = 1;
  return rad * cos(th);
}

/* number of failures before the first success, success probability p */
static uint64_t rng_geom0(rng_t* r, double p) {
  if (p >= 1.0) return 0;
  double u = rng_unit(r);
  double k = floor(log1p(-u) / log1p(-p));
  if (k > 1e15) k = 1e15;
  return (uint64_t)k;
}

/* ------------------------------------------------------------------------ */
/* Zipf text: words of a random vocabulary, ranked in generation order, drawn
 * with P(rank k) proportional to k^-s, separated by spaces, with a newline
 * after every 80 characters of output. */

typedef struct { char w[13]; uint8_t len; } word_t;

static uint64_t hash_word(const char* w, int len) {
  uint64_t h = 1469598103934665603ULL;
  for (int i = 0; i < len; ++i) { h ^= (uint8_t)w[i]; h *= 1099511628211ULL; }
  return h;
}

uint64_t synth_zipf_text(uint8_t* out, uint64_t n, uint64_t seed, double s, uint32_t vocab) {
  if (vocab == 0) vocab = 4096;
  rng_t r;
  rng_seed(&r, seed);
  word_t* words = (word_t*)malloc(sizeof(word_t) * vocab);
  uint32_t hcap = 1;
  while (hcap < 4 * vocab) hcap <<= 1;
  uint32_t* table = (uint32_t*)malloc(sizeof(uint32_t) * hcap); /* index+1, 0 = empty */
  memset(table, 0, sizeof(uint32_t) * hcap);
  uint32_t made = 0;
  while (made < vocab) {
    word_t cand;
    cand.len = (uint8_t)(2 + rng_below(&r, 11)); /* 2..12 */
    for (int i = 0; i < cand.len; ++i) cand.w[i] = (char)('a' + rng_below(&r, 26));
    uint64_t h = hash_word(cand.w, cand.len);
    uint32_t slot = (uint32_t)(h & (hcap - 1));
    int dup = 0;
    while (table[slot]) {
      word_t* o = &words[table[slot] - 1];
      if (o->len == cand.len && memcmp(o->w, cand.w, cand.len) == 0) { dup = 1; break; }
      slot = (slot + 1) & (hcap - 1);
    }
    if (dup) continue;
    words[made] = cand;
    table[slot] = made + 1;
    ++made;
  }
  double* cdf = (double*)malloc(sizeof(double) * vocab);
  double acc = 0.0;
  for (uint32_t k = 0; k < vocab; ++k) { acc += pow((double)(k + 1), -s); cdf[k] = acc; }

  uint64_t o = 0;
  int col = 0;
  int first = 1;
  while (o < n) {
    double u = rng_unit(&r) * acc;
    uint32_t lo = 0, hi = vocab - 1;
    while (lo < hi) { uint32_t mid = (lo + hi) >> 1; if (cdf[mid] > u) hi = mid; else lo = mid + 1; }
    const word_t* w = &words[lo];
    /* separator, then the word, each character subject to the line rule */
    for (int i = first ? 0 : -1; i < (int)w->len && o < n; ++i) {
      char c = (i < 0) ? ' ' : w->w[i];
      if (col == 80) { out[o++] = '\n'; col = 0; if (o >= n) break; }
      out[o++] = (uint8_t)c;
      ++col;
    }
    first = 0;
  }
  free(cdf);
  free(table);
  free(words);
  return n;
}

/* ------------------------------------------------------------------------ */
/* FASTQ-like reads: 4-line records sampled from a random ACGT reference with
 * substitutions and N calls, with Phred+33 qualities from a per-position
 * autoregressive model whose mean decays from Q34 to Q22 along the read
 * (mean about Q30).  Only whole records are written; returns bytes written. */

static int put_u64(char* p, uint64_t v) {
  char tmp[24];
  int k = 0;
  do { tmp[k++] = (char)('0' + v % 10); v /= 10; } while (v);
  for (int i = 0; i < k; ++i) p[i] = tmp[k - 1 - i];
  return k;
}

uint64_t synth_fastq(uint8_t* out, uint64_t cap, uint64_t seed, double sub_rate, double n_rate,
                     uint64_t ref_len, uint32_t read_len) {
  if (read_len == 0) read_len = 150;
  if (ref_len < read_len) ref_len = read_len;
  rng_t r;
  rng_seed(&r, seed);
  static const char B[4] = {'A', 'C', 'G', 'T'};
  char* ref = (char*)malloc(ref_len);
  for (uint64_t i = 0; i < ref_len; ++i) ref[i] = B[rng_next(&r) & 3];
  char* rec = (char*)malloc(2 * (size_t)read_len + 128);
  uint64_t o = 0;
  for (uint64_t id = 1;; ++id) {
    char* p = rec;
    *p++ = '@'; *p++ = 'S'; *p++ = 'Y'; *p++ = 'N'; *p++ = '.';
    p += put_u64(p, id);
    *p++ = ' ';
    p += put_u64(p, id);
    *p++ = '/'; *p++ = '1'; *p++ = '\n';
    char* seq = p;
    uint64_t start = rng_below(&r, ref_len - read_len + 1);
    for (uint32_t i = 0; i < read_len; ++i) {
      char b = ref[start + i];
      if (rng_unit(&r) < sub_rate) {
        int cur = (b == 'A') ? 0 : (b == 'C') ? 1 : (b == 'G') ? 2 : 3;
        int alt = (cur + 1 + (int)rng_below(&r, 3)) & 3;
        b = B[alt];
      }
      if (rng_unit(&r) < n_rate) b = 'N';
      *p++ = b;
    }
    *p++ = '\n';
    *p++ = '+';
    *p++ = '\n';
    double e = 0.0;
    double denom = (read_len > 1) ? (double)(read_len - 1) : 1.0;
    for (uint32_t i = 0; i < read_len; ++i) {
      double x = (double)i / denom;
      double mu = 34.0 - 12.0 * x * x;
      e = 0.8 * e + 3.0 * rng_normal(&r);
      long q = lround(mu + e);
      if (q < 2) q = 2;
      if (q > 41) q = 41;
      if (seq[i] == 'N') q = 2;
      *p++ = (char)(q + 33);
    }
    *p++ = '\n';
    uint64_t len = (uint64_t)(p - rec);
    if (o + len > cap) break;
    memcpy(out + o, rec, len);
    o += len;
  }
  free(rec);
  free(ref);
  return o;
}

/* ------------------------------------------------------------------------ */
/* Token streams with a controlled mean match length, as used by the copy
 * sweep: a literal prefix of `lit_prefix` bytes, then tokens made of a
 * literal run (geometric, mean 0.01*m/0.99, so literals are ~1% of bytes)
 * and a match whose length is 1 + Geom0(1/m) (mean m, capped at len_cap),
 * with its source drawn uniformly from positions at least `min_back` bytes
 * behind the match start.  Literal bytes are uniform.  Arrays are malloc'ed
 * here and released with synth_free. */
int synth_geo_tokens(uint64_t n, double mean, uint64_t seed, uint32_t lit_prefix, uint32_t len_cap,
                     uint32_t min_back, uint64_t* ntok_out, uint32_t** lit_len_out,
                     uint32_t** mlen_out, uint64_t** src_out, uint64_t* nlit_out, uint8_t** lit_out) {
  if (mean < 1.0) mean = 1.0;
  if (lit_prefix > n) lit_prefix = (uint32_t)n;
  if (min_back < 1) min_back = 1;
  if (min_back > lit_prefix && lit_prefix > 0) min_back = lit_prefix;
  rng_t r;
  rng_seed(&r, seed);
  double lit_mean = 0.01 * mean / 0.99;
  double p_lit = 1.0 / (1.0 + lit_mean);
  double p_len = 1.0 / mean;
  uint64_t cap_tok = (uint64_t)((double)n / (mean + lit_mean) * 1.25) + 1024;
  uint32_t* ll = (uint32_t*)malloc(sizeof(uint32_t) * cap_tok);
  uint32_t* ml = (uint32_t*)malloc(sizeof(uint32_t) * cap_tok);
  uint64_t* sr = (uint64_t*)malloc(sizeof(uint64_t) * cap_tok);
  uint64_t cap_lit = (uint64_t)((double)n * 0.02) + lit_prefix + 4096;
  uint8_t* lt = (uint8_t*)malloc(cap_lit);
  if (!ll || !ml || !sr || !lt) { free(ll); free(ml); free(sr); free(lt); return -1; }
  uint64_t pos = 0, nt = 0, nl = 0;
  int firsttok = 1;
  while (pos < n) {
    uint64_t lit = firsttok ? lit_prefix : rng_geom0(&r, p_lit);
    firsttok = 0;
    if (lit > n - pos) lit = n - pos;
    uint64_t mstart = pos + lit;
    uint64_t L = 0, s = 0;
    if (mstart < n && mstart >= min_back) {
      L = 1 + rng_geom0(&r, p_len);
      if (L > len_cap) L = len_cap;
      if (L > n - mstart) L = n - mstart;
      s = rng_below(&r, mstart - min_back + 1);
    } else if (mstart < n) {
      /* not enough history yet: extend the literal run by one byte */
      lit += 1;
      mstart += 1;
    }
    if (nt == cap_tok) {
      cap_tok *= 2;
      ll = (uint32_t*)realloc(ll, sizeof(uint32_t) * cap_tok);
      ml = (uint32_t*)realloc(ml, sizeof(uint32_t) * cap_tok);
      sr = (uint64_t*)realloc(sr, sizeof(uint64_t) * cap_tok);
    }
    if (nl + lit > cap_lit) {
      cap_lit = (nl + lit) * 2;
      lt = (uint8_t*)realloc(lt, cap_lit);
    }
    for (uint64_t i = 0; i < lit; ++i) lt[nl + i] = (uint8_t)(rng_next(&r) >> 56);
    nl += lit;
    ll[nt] = (uint32_t)lit;
    ml[nt] = (uint32_t)L;
    sr[nt] = s;
    ++nt;
    pos = mstart + L;
  }
  *ntok_out = nt;
  *lit_len_out = ll;
  *mlen_out = ml;
  *src_out = sr;
  *nlit_out = nl;
  *lit_out = lt;
  return 0;
}

void synth_free(void* p) { free(p); }

void synth_random_bytes(uint8_t* out, uint64_t n, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  uint64_t i = 0;
  for (; i + 8 <= n; i += 8) { uint64_t v = rng_next(&r); memcpy(out + i, &v, 8); }
  if (i < n) { uint64_t v = rng_next(&r); memcpy(out + i, &v, n - i); }
}

/* `count` sizes drawn log-uniformly from [lo, hi] */
void synth_loguniform(uint64_t* out, uint64_t count, uint64_t lo, uint64_t hi, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  double a = log((double)lo), b = log((double)hi);
  for (uint64_t i = 0; i < count; ++i) {
    double v = exp(a + (b - a) * rng_unit(&r));
    uint64_t x = (uint64_t)llround(v);
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    out[i] = x;
  }
}

/* `count` doubles uniform in [0,1) */
void synth_uniform(double* out, uint64_t count, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  for (uint64_t i = 0; i < count; ++i) out[i] = rng_unit(&r);
}

/* `count` standard normals */
void synth_normal(double* out, uint64_t count, uint64_t seed) {
  rng_t r;
  rng_seed(&r, seed);
  for (uint64_t i = 0; i < count; ++i) out[i] = rng_normal(&r);
}
