// lz_host.cpp -- host side of liblz: greedy encoder with per-distance-class
// thresholds, container writer/reader, validation, statistics, entropy-bound
// size and the dependency-level planner.
//
// Encoder (Sec. 4.2): every earlier position is a candidate source (whole
// prefix, or the caller's segment); a candidate of distance class c is valid
// iff its match reaches thr[c]; the longest valid one wins, nearest on ties.
// Candidates come from two hash-chain indexes built over the whole input
// before parsing: a "near" index keyed on the first min(thr[0],thr[1]) bytes
// walked only inside distance bound[1], and a "far" index keyed on the first
// min(thr[2],thr[3]) bytes walked at every distance.  A valid candidate of
// class c matches at least thr[c] bytes, hence its key, so walking whole
// chains (max_chain = 0) is exhaustive; a finite max_chain trades ratio for
// speed.  Blocks are parsed in parallel since the indexes are read-only.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

#include "lz_internal.h"

namespace lz {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

unsigned hw_threads(uint32_t requested) {
  if (requested) return requested;
  unsigned h = std::thread::hardware_concurrency();
  return h ? std::min(h, 32u) : 1;
}

template <class F>
static void parallel_for(uint64_t count, unsigned threads, F&& f) {
  if (count == 0) return;
  threads = (unsigned)std::min<uint64_t>(threads, count);
  if (threads <= 1) {
    for (uint64_t i = 0; i < count; ++i) f(i, 0u);
    return;
  }
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> pool;
  for (unsigned w = 0; w < threads; ++w)
    pool.emplace_back([&, w] {
      for (;;) {
        uint64_t i = next.fetch_add(1);
        if (i >= count) break;
        f(i, w);
      }
    });
  for (auto& t : pool) t.join();
}

// ------------------------------------------------------------------ reading

int view_header(const uint8_t* arc, ArcView* out) {
  if (!arc) return fail(LZ_E_CORRUPT, "null header");
  if (rd_le(arc, 4) != kMagic || rd_le(arc + 4, 4) != 1) return fail(LZ_E_CORRUPT, "bad magic or version");
  ArcView a;
  a.base = arc;
  a.n = rd_le(arc + 8, 8);
  if (a.n > (1ull << 48)) return fail(LZ_E_CORRUPT, "n out of range");
  a.log2_bs = (uint32_t)rd_le(arc + 16, 4);
  if (a.log2_bs < 4 || a.log2_bs > 24) return fail(LZ_E_CORRUPT, "block size out of range");
  a.bs = 1ull << a.log2_bs;
  a.nb = rd_le(arc + 20, 4);
  if (a.nb != (a.n + a.bs - 1) / a.bs) return fail(LZ_E_CORRUPT, "block count mismatch");
  a.min_match = rd_le(arc + 24, 4);
  if (a.min_match < 1) return fail(LZ_E_CORRUPT, "min_match 0");
  a.flags = rd_le(arc + 28, 4);
  if (a.flags & ~3ull) return fail(LZ_E_CORRUPT, "unknown flags");
  a.n_tok = rd_le(arc + 32, 8);
  a.n_x16 = rd_le(arc + 40, 8);
  a.n_x32 = rd_le(arc + 48, 8);
  a.n_lit = rd_le(arc + 56, 8);
  if (a.n_tok > a.n || a.n_lit > a.n || a.n_x16 > 2 * a.n_tok || a.n_x32 > a.n_x16)
    return fail(LZ_E_CORRUPT, "stream counts out of range");
  for (int k = 0; k < 4; ++k) a.thr[k] = arc[64 + k];
  for (int k = 0; k < 3; ++k) a.bound[k] = rd_le(arc + 72 + 8 * k, 8);
  uint64_t off = kHeader;
  a.off_tab = off;
  off = align16(off + 32 * (a.nb + 1));
  a.off_cmd = off;
  off = align16(off + a.n_tok);
  a.off_x16 = off;
  off = align16(off + 2 * a.n_x16);
  a.off_x32 = off;
  off = align16(off + 4 * a.n_x32);
  a.off_slo = off;
  off = align16(off + 4 * a.n_tok);
  if (a.flags & 1) {
    a.off_shi = off;
    off = align16(off + a.n_tok);
  }
  a.off_lit = off;
  off = align16(off + a.n_lit);
  if (a.flags & 2) {
    a.off_info = off;
    off = align16(off + a.nb);
  }
  off += 16;
  a.total = off;
  *out = a;
  return 0;
}

int view_archive(const uint8_t* arc, uint64_t size, ArcView* v) {
  if (!arc || size < kHeader) return fail(LZ_E_CORRUPT, "archive shorter than its header");
  ArcView a;
  int rc = view_header(arc, &a);
  if (rc) return rc;
  a.size = size;
  const uint64_t off = a.total;
  if (size < off) return fail(LZ_E_CORRUPT, "archive truncated (%llu < %llu)", (unsigned long long)size,
                              (unsigned long long)off);
  const uint64_t* T = a.tab();
  for (int k = 0; k < 4; ++k)
    if (T[k] != 0) return fail(LZ_E_CORRUPT, "block table does not start at zero");
  const uint64_t tot[4] = {a.n_tok, a.n_lit, a.n_x16, a.n_x32};
  for (int k = 0; k < 4; ++k)
    if (T[4 * a.nb + k] != tot[k]) return fail(LZ_E_CORRUPT, "block table totals mismatch");
  for (uint64_t b = 0; b < a.nb; ++b)
    for (int k = 0; k < 4; ++k)
      if (T[4 * (b + 1) + k] < T[4 * b + k]) return fail(LZ_E_CORRUPT, "block table not monotone");
  *v = a;
  return 0;
}

int validate_archive(const ArcView& v, uint32_t n_threads) {
  std::atomic<int> bad{0};
  std::atomic<uint64_t> bad_block{0};
  parallel_for(v.nb, hw_threads(n_threads), [&](uint64_t b, unsigned) {
    if (bad.load(std::memory_order_relaxed)) return;
    int rc = walk_block(v, b, [](uint64_t, const Tok&) {});
    if (rc) {
      bad.store(rc);
      bad_block.store(b);
    }
  });
  if (bad.load()) return fail(LZ_E_CORRUPT, "block %llu fails validation", (unsigned long long)bad_block.load());
  return 0;
}

// ------------------------------------------------------------------ writing

namespace {

struct BTok {
  uint64_t lit_len, mlen, src;
};

// Per-block encoded streams, concatenated afterwards.
struct BlockEnc {
  std::vector<uint8_t> cmd, x16, x32, slo, shi, lit;
};

static void put_len_ext(BlockEnc& e, uint64_t v) {  // v = value - 15
  if (v < 0xFFFF) {
    e.x16.push_back(uint8_t(v));
    e.x16.push_back(uint8_t(v >> 8));
  } else {
    e.x16.push_back(0xFF);
    e.x16.push_back(0xFF);
    uint64_t w = v - 0xFFFF;
    for (int i = 0; i < 4; ++i) e.x32.push_back(uint8_t(w >> (8 * i)));
  }
}

// Encodes one block's token list (lit bytes already in e.lit).
static void encode_block_tokens(const std::vector<BTok>& toks, uint64_t min_match, BlockEnc& e) {
  for (size_t i = 0; i < toks.size(); ++i) {
    const BTok& t = toks[i];
    bool last = (i + 1 == toks.size());
    uint64_t lv = t.lit_len, mv = last ? 0 : t.mlen - min_match;
    uint8_t lc = lv < 15 ? uint8_t(lv) : 15, mc = mv < 15 ? uint8_t(mv) : 15;
    e.cmd.push_back(uint8_t((lc << 4) | mc));
    if (lv >= 15) put_len_ext(e, lv - 15);
    if (mv >= 15) put_len_ext(e, mv - 15);
    uint64_t s = t.mlen ? t.src : 0;
    for (int k = 0; k < 4; ++k) e.slo.push_back(uint8_t(s >> (8 * k)));
    e.shi.push_back(uint8_t(s >> 32));
  }
}

static int assemble(uint64_t n, uint32_t log2_bs, uint64_t min_match, const uint32_t* thr, const uint64_t* bound,
                    std::vector<BlockEnc>& blocks, const uint8_t* info, uint8_t** arc, uint64_t* arc_size) {
  uint64_t nb = blocks.size();
  uint64_t tok = 0, lit = 0, x16 = 0, x32 = 0;
  std::vector<uint64_t> tab(4 * (nb + 1));
  for (uint64_t b = 0; b < nb; ++b) {
    tab[4 * b + 0] = tok;
    tab[4 * b + 1] = lit;
    tab[4 * b + 2] = x16;
    tab[4 * b + 3] = x32;
    tok += blocks[b].cmd.size();
    lit += blocks[b].lit.size();
    x16 += blocks[b].x16.size() / 2;
    x32 += blocks[b].x32.size() / 4;
  }
  tab[4 * nb + 0] = tok;
  tab[4 * nb + 1] = lit;
  tab[4 * nb + 2] = x16;
  tab[4 * nb + 3] = x32;
  bool hi = n > 0xFFFFFFFFull;
  uint64_t flags = (hi ? 1 : 0) | (info ? 2 : 0);
  uint64_t off = kHeader;
  off = align16(off + 32 * (nb + 1));
  uint64_t o_cmd = off;
  off = align16(off + tok);
  uint64_t o_x16 = off;
  off = align16(off + 2 * x16);
  uint64_t o_x32 = off;
  off = align16(off + 4 * x32);
  uint64_t o_slo = off;
  off = align16(off + 4 * tok);
  uint64_t o_shi = off;
  if (hi) off = align16(off + tok);
  uint64_t o_lit = off;
  off = align16(off + lit);
  uint64_t o_info = off;
  if (info) off = align16(off + nb);
  off += 16;
  uint8_t* a = (uint8_t*)calloc(off, 1);
  if (!a) return fail(LZ_E_NOMEM, "archive allocation of %llu bytes failed", (unsigned long long)off);
  auto wr = [&](uint64_t o, uint64_t v, int k) {
    for (int i = 0; i < k; ++i) a[o + i] = uint8_t(v >> (8 * i));
  };
  wr(0, kMagic, 4);
  wr(4, 1, 4);
  wr(8, n, 8);
  wr(16, log2_bs, 4);
  wr(20, nb, 4);
  wr(24, min_match, 4);
  wr(28, flags, 4);
  wr(32, tok, 8);
  wr(40, x16, 8);
  wr(48, x32, 8);
  wr(56, lit, 8);
  for (int k = 0; k < 4; ++k) a[64 + k] = uint8_t(thr ? std::min<uint32_t>(thr[k], 255) : 0);
  for (int k = 0; k < 3; ++k) wr(72 + 8 * k, bound ? bound[k] : 0, 8);
  memcpy(a + kHeader, tab.data(), 8 * tab.size());  // little-endian host
  uint64_t pc = o_cmd, p16 = o_x16, p32 = o_x32, pl = o_slo, ph = o_shi, pt = o_lit;
  for (auto& e : blocks) {
    memcpy(a + pc, e.cmd.data(), e.cmd.size());
    pc += e.cmd.size();
    memcpy(a + p16, e.x16.data(), e.x16.size());
    p16 += e.x16.size();
    memcpy(a + p32, e.x32.data(), e.x32.size());
    p32 += e.x32.size();
    memcpy(a + pl, e.slo.data(), e.slo.size());
    pl += e.slo.size();
    if (hi) {
      memcpy(a + ph, e.shi.data(), e.shi.size());
      ph += e.shi.size();
    }
    memcpy(a + pt, e.lit.data(), e.lit.size());
    pt += e.lit.size();
  }
  if (info) memcpy(a + o_info, info, nb);
  *arc = a;
  *arc_size = off;
  return 0;
}

// ------------------------------------------------------------------ encoder

// Chain entry of position p: low 32 bits = previous position + 1 with the
// same key hash (0 = none), high 32 bits = a fingerprint of p's key, so a walk
// rejects hash collisions from the entry it already loaded.
// Large arrays backed by 2 MiB pages where the kernel allows it: chain walks
// touch entries at random across gigabytes, so small pages miss the TLB.
template <class T>
struct HugeArray {
  T* p = nullptr;
  size_t n = 0;
  HugeArray() = default;
  HugeArray(const HugeArray&) = delete;
  HugeArray& operator=(const HugeArray&) = delete;
  ~HugeArray() { release(); }
  void release() {
    if (p) munmap(p, bytes(n));
    p = nullptr;
    n = 0;
  }
  // Large arrays are rounded to 2 MiB and asked for huge pages; small ones
  // stay on 4 KiB pages, since the first touch of a huge page zeroes all of
  // it (a fixed ~0.3 ms per array that dominated encodes of small inputs).
  static constexpr size_t kHuge = 8u << 20;
  static size_t bytes(size_t k) {
    const size_t b = k * sizeof(T), a = b >= kHuge ? (2u << 20) : 4096;
    return (b + a - 1) & ~(a - 1);
  }
  void assign_zero(size_t k) {
    release();
    void* q = mmap(nullptr, bytes(k), PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (q == MAP_FAILED) throw std::bad_alloc();
    if (bytes(k) >= kHuge) madvise(q, bytes(k), MADV_HUGEPAGE);
    p = (T*)q;  // anonymous mappings start zeroed
    n = k;
  }
  T& operator[](size_t i) { return p[i]; }
  const T& operator[](size_t i) const { return p[i]; }
};

struct HashIndex {
  uint32_t key = 4;  // bytes hashed
  HugeArray<uint64_t> prev;
};

static inline uint64_t load_key(const uint8_t* p, uint32_t k) {
  uint64_t a;
  memcpy(&a, p, 8);
  if (k >= 8) {
    if (k == 8) return a;
    uint64_t b;
    memcpy(&b, p + 8, 8);
    if (k < 16) b &= (~0ull) >> (8 * (16 - k));
    return a ^ (b * 0x9E3779B97F4A7C15ull);
  }
  return a & ((~0ull) >> (8 * (8 - k)));
}

static inline uint32_t hash_key(uint64_t v, int bits) {
  v ^= v >> 29;
  v *= 0xBF58476D1CE4E5B9ull;
  v ^= v >> 32;
  return uint32_t(v >> (64 - bits));
}

static inline uint64_t fingerprint(uint64_t v) {
  v ^= v >> 31;
  v *= 0x94D049BB133111EBull;
  v ^= v >> 29;
  return (v & 0xFFFFFFFF00000000ull);
}

// Builds the chain entries of positions [lo, hi) for p + key <= hi.  The head
// table is split into S hash slices.  Pass 1 counts, per position range and
// slice, the positions whose key hashes into the slice; pass 2 scatters the
// positions into slice-major lists (each list stays in increasing position
// order); pass 3 links every slice's positions in order with its own part of
// the head table, so each chain is written by one thread, nearest-first links
// come out in position order, and the table can be large without per-thread
// copies.
static void build_index(const uint8_t* x, uint64_t lo, uint64_t hi, uint32_t key, unsigned threads,
                        HashIndex& idx, int bits) {
  idx.key = key;
  if (hi - lo < key) return;
  const uint64_t last = hi - key;  // last hashable position (inclusive)
  const uint64_t cnt = last - lo + 1;
  auto key_at = [&](uint64_t p) -> uint64_t {
    if (p + 16 <= hi) return load_key(x + p, key);
    uint8_t tmp[16] = {0};
    memcpy(tmp, x + p, key);
    return load_key(tmp, key);
  };
  const unsigned T = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(threads, cnt >> 16));
  const unsigned S = T;
  const int sbits = bits;
  auto slice_of = [&](uint32_t h) { return (unsigned)(((uint64_t)h * S) >> sbits); };
  std::vector<uint64_t> count((size_t)T * S, 0), off((size_t)T * S, 0);
  auto range = [&](unsigned r, uint64_t& a, uint64_t& b) {
    a = lo + cnt * r / T;
    b = lo + cnt * (r + 1) / T;
  };
  auto run = [&](auto&& body) {
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < T; ++w) pool.emplace_back([&, w] { body(w); });
    for (auto& t : pool) t.join();
  };
  run([&](unsigned r) {
    uint64_t a, b;
    range(r, a, b);
    uint64_t* c = &count[(size_t)r * S];
    for (uint64_t p = a; p < b; ++p) c[slice_of(hash_key(key_at(p), bits))]++;
  });
  uint64_t acc = 0;
  for (unsigned sl = 0; sl < S; ++sl)
    for (unsigned r = 0; r < T; ++r) {
      off[(size_t)r * S + sl] = acc;
      acc += count[(size_t)r * S + sl];
    }
  HugeArray<uint32_t> list;
  list.assign_zero(cnt);
  run([&](unsigned r) {
    uint64_t a, b;
    range(r, a, b);
    uint64_t* o = &off[(size_t)r * S];
    for (uint64_t p = a; p < b; ++p) list[o[slice_of(hash_key(key_at(p), bits))]++] = uint32_t(p - lo);
  });
  HugeArray<uint32_t> head;
  head.assign_zero(1ull << bits);
  run([&](unsigned sl) {
    const uint64_t b0 = (sl == 0) ? 0 : off[(size_t)(T - 1) * S + sl - 1];  // end of previous slice
    const uint64_t b1 = off[(size_t)(T - 1) * S + sl];
    for (uint64_t i = b0; i < b1; ++i) {
      const uint64_t p = lo + list[i];
      const uint64_t kv = key_at(p);
      const uint32_t h = hash_key(kv, bits);
      idx.prev[p] = head[h] | fingerprint(kv);
      head[h] = uint32_t(p - lo + 1);
    }
  });
}

static inline uint64_t match_len(const uint8_t* x, uint64_t src, uint64_t pos, uint64_t end) {
  uint64_t L = 0;
  while (pos + L + 8 <= end) {
    uint64_t a, b;
    memcpy(&a, x + src + L, 8);
    memcpy(&b, x + pos + L, 8);
    uint64_t d = a ^ b;
    if (d) return L + (__builtin_ctzll(d) >> 3);
    L += 8;
  }
  while (pos + L < end && x[src + L] == x[pos + L]) ++L;
  return L;
}

static inline int dclass(uint64_t d, const uint64_t* bound) {
  return d < bound[0] ? 0 : d < bound[1] ? 1 : d < bound[2] ? 2 : 3;
}

struct EncCtx {
  const uint8_t* x;
  uint64_t n;
  uint64_t bs;
  const lz_params* p;
  const uint32_t* thr_block;  // per block tuple or null
  HashIndex near_idx, far_idx;
  uint64_t seg;  // unused: positions are segment-relative
  // Depth-aware ties: dependency depth of every segment position as the
  // previous parse left it (null = ties go to the nearest source).
  const uint16_t* dep = nullptr;
};

constexpr uint32_t kDepthMax = 0xFFFF;

// Greedy parse of one block into tokens + its literal bytes.
static void parse_block(const EncCtx& c, uint64_t b, std::vector<BTok>& toks, std::vector<uint8_t>& lit) {
  const uint8_t* x = c.x;
  uint64_t start = b * c.bs, end = std::min(c.n, start + c.bs);
  const uint64_t seg_lo = 0;  // positions are relative to the segment base c.x
  const uint32_t* thr = c.thr_block ? c.thr_block + 4 * b : c.p->thr;
  const uint64_t* bound = c.p->bound;
  uint32_t maxc = c.p->max_chain;
  // with a chain limit the walk also stops at a match this long (exact mode never does)
  const uint64_t nice = maxc ? 128 : UINT64_MAX;
  uint32_t kn = c.near_idx.key, kf = c.far_idx.key;
  uint64_t pos = start, run = 0;
  toks.clear();
  lit.clear();
  lit.reserve(end - start);
  // Depth-aware ties (reading 4 of the tie-break among equal lengths): the
  // resulting depth of a candidate is 1 + the deepest byte it reads (its own
  // output excluded); bytes of this block take the depths of this parse,
  // earlier bytes those of the previous parse.  Lower depth wins, then the
  // nearer source; lengths are unchanged.
  const bool deep = c.dep != nullptr;
  std::vector<uint16_t> dl;
  if (deep) dl.assign(end - start, 0);
  auto cand_depth = [&](uint64_t src, uint64_t L, uint64_t at) -> uint32_t {
    const uint64_t e = std::min(src + L, at);
    uint32_t m = 0;
    uint64_t q = src;
    for (const uint64_t e1 = std::min(e, start); q < e1; ++q) m = std::max<uint32_t>(m, c.dep[q]);
    for (; q < e; ++q) m = std::max<uint32_t>(m, dl[q - start]);
    return std::min<uint32_t>(m + 1, kDepthMax);
  };
  while (pos < end) {
    uint64_t best_len = 0, best_src = 0;
    uint32_t best_dep = 0;
    // a candidate of cl's class matching L bytes from src: keep the longest,
    // then (depth-aware) the shallowest, then the nearest
    auto consider = [&](uint64_t src, uint64_t L) {
      if (L > best_len) {
        best_len = L;
        best_src = src;
        if (deep) best_dep = cand_depth(src, L, pos);
      } else if (L == best_len && L) {
        if (deep) {
          const uint32_t d = cand_depth(src, L, pos);
          if (d < best_dep || (d == best_dep && src > best_src)) {
            best_src = src;
            best_dep = d;
          }
        } else if (src > best_src) {
          best_src = src;
        }
      }
    };
    // the walk can stop once nothing better is possible: the longest match
    // reaches the block end or is long enough, and (depth-aware) reads only
    // literals
    auto done = [&]() { return (pos + best_len == end || best_len >= nice) && (!deep || best_dep <= 1); };
    if (pos + 4 < end) {
      __builtin_prefetch(&c.near_idx.prev[pos + 4]);
      __builtin_prefetch(&c.far_idx.prev[pos + 4]);
    }
    // near chain: candidates within distance bound[1]
    if (pos + kn <= end) {
      // prev[pos] is the nearest earlier position with the same key hash
      const uint64_t e0 = c.near_idx.prev[pos];
      const uint64_t fp = e0 & 0xFFFFFFFF00000000ull;
      uint32_t link = uint32_t(e0);
      uint32_t steps = 0, walked = 0;
      while (link) {
        uint64_t src = seg_lo + link - 1;
        uint64_t d = pos - src;
        if (d >= bound[1]) break;
        const uint64_t e = c.near_idx.prev[src];
        if ((e & 0xFFFFFFFF00000000ull) != fp) {  // different key, same hash
          if (maxc && ++walked >= 8 * maxc) break;
          link = uint32_t(e);
          continue;
        }
        uint64_t L = match_len(x, src, pos, end);
        int cl = dclass(d, bound);
        if (L >= thr[cl]) {
          consider(src, L);
          if (done()) break;
        }
        if (maxc && ++steps >= maxc) break;
        link = uint32_t(e);
      }
    }
    // far chain: any distance
    if (pos + kf <= end && !done()) {
      const uint64_t e0 = c.far_idx.prev[pos];
      const uint64_t fp = e0 & 0xFFFFFFFF00000000ull;
      uint32_t link = uint32_t(e0);
      uint32_t steps = 0, walked = 0;
      while (link) {
        uint64_t src = seg_lo + link - 1;
        uint64_t d = pos - src;
        const uint64_t e = c.far_idx.prev[src];
        if ((e & 0xFFFFFFFF00000000ull) != fp) {
          if (maxc && ++walked >= 8 * maxc) break;
          link = uint32_t(e);
          continue;
        }
        uint64_t L = match_len(x, src, pos, end);
        int cl = dclass(d, bound);
        if (L >= thr[cl]) {
          consider(src, L);
          if (done()) break;
        }
        if (maxc && ++steps >= maxc) break;
        link = uint32_t(e);
      }
    }
    if (best_len) {
      toks.push_back(BTok{run, best_len, best_src});
      run = 0;
      if (deep) std::fill(dl.begin() + (pos - start), dl.begin() + (pos - start + best_len), (uint16_t)best_dep);
      pos += best_len;
    } else {
      lit.push_back(x[pos]);
      ++run;
      ++pos;
    }
  }
  if (run) toks.push_back(BTok{run, 0, 0});
}

// Depth cap: walks the tokens of blocks [b0, b1) of a segment (input x =
// the segment's first byte, segment-relative positions; token sources are
// absolute, the segment starts at s0) in output order with the dependency
// depth of every byte (literal bytes 0, a match 1 + the deepest byte it reads,
// its own output excluded, as in compute_levels) and turns every match whose
// depth would exceed `cap` into literal bytes, merged into the next token's
// run.  Depths only fall when a match becomes literals, so the walk is exact:
// the archive's deepest match ends at depth <= cap.  Blocks whose tokens
// changed get their literal stream rebuilt from the input.
static void cap_depths(const uint8_t* x, uint64_t s0, uint64_t b0, uint64_t b1, uint64_t bs, uint32_t cap,
                       std::vector<BlockEnc>& blocks, uint16_t* dep) {
  for (uint64_t i = 0; i < b1 - b0; ++i) {
    BlockEnc& e = blocks[b0 + i];
    const BTok* tk = (const BTok*)e.slo.data();
    const size_t nt = e.slo.size() / sizeof(BTok);
    std::vector<BTok> out;
    out.reserve(nt);
    bool changed = false;
    uint64_t q = i * bs, acc = 0;
    for (size_t j = 0; j < nt; ++j) {
      std::fill(dep + q, dep + q + tk[j].lit_len, (uint16_t)0);
      q += tk[j].lit_len;
      acc += tk[j].lit_len;
      if (!tk[j].mlen) continue;
      const uint64_t a = tk[j].src - s0, z = std::min(a + tk[j].mlen, q);
      uint32_t m = 0;
      for (uint64_t r = a; r < z; ++r) m = std::max<uint32_t>(m, dep[r]);
      if (m + 1 > cap) {
        std::fill(dep + q, dep + q + tk[j].mlen, (uint16_t)0);
        acc += tk[j].mlen;
        changed = true;
      } else {
        std::fill(dep + q, dep + q + tk[j].mlen, (uint16_t)(m + 1));
        out.push_back(BTok{acc, tk[j].mlen, tk[j].src});
        acc = 0;
      }
      q += tk[j].mlen;
    }
    if (!changed) continue;
    if (acc) out.push_back(BTok{acc, 0, 0});
    e.lit.clear();
    uint64_t r = i * bs;
    for (const BTok& t : out) {
      e.lit.insert(e.lit.end(), x + r, x + r + t.lit_len);
      r += t.lit_len + t.mlen;
    }
    e.slo.resize(out.size() * sizeof(BTok));
    memcpy(e.slo.data(), out.data(), out.size() * sizeof(BTok));
  }
}

static int check_params(const lz_params* p, uint64_t n) {
  if (!p) return fail(LZ_E_INVAL, "null params");
  if (p->log2_bs < 4 || p->log2_bs > 24) return fail(LZ_E_INVAL, "log2_bs must be in [4,24]");
  for (int k = 0; k < 4; ++k)
    if (p->thr[k] < 1) return fail(LZ_E_INVAL, "thresholds must be >= 1");
  if (!(p->bound[0] <= p->bound[1] && p->bound[1] <= p->bound[2]))
    return fail(LZ_E_INVAL, "class bounds must be non-decreasing");
  uint64_t bs = 1ull << p->log2_bs;
  if (p->segment && (p->segment % bs)) return fail(LZ_E_INVAL, "segment must be a multiple of the block size");
  if (p->segment > 0xFFFFFFFFull - 16) return fail(LZ_E_INVAL, "segment must be below 4 GiB");
  if (!p->segment && n > 0xFFFFFFFFull - 16) return fail(LZ_E_INVAL, "inputs of 4 GiB or more need a segment");
  if (p->depth_passes > 8) return fail(LZ_E_INVAL, "depth_passes must be at most 8");
  if (p->depth_cap >= kDepthMax) return fail(LZ_E_INVAL, "depth_cap must be below 65535");
  return 0;
}

static int encode_impl(const uint8_t* in, uint64_t n, const lz_params* p, const uint32_t* thr_block,
                       const uint8_t* tuple_id, uint8_t** arc, uint64_t* arc_size) {
  int rc = check_params(p, n);
  if (rc) return rc;
  if (!arc || !arc_size || (n && !in)) return fail(LZ_E_INVAL, "null argument");
  uint64_t bs = 1ull << p->log2_bs;
  uint64_t nb = (n + bs - 1) / bs;
  unsigned threads = hw_threads(p->n_threads);
  // key lengths: near serves classes 0-1, far serves classes 2-3; per-block
  // tuples take the minimum over all blocks so every chain stays exhaustive
  uint32_t tmin[4] = {p->thr[0], p->thr[1], p->thr[2], p->thr[3]};
  if (thr_block && nb) {
    for (int k = 0; k < 4; ++k) tmin[k] = UINT32_MAX;
    for (uint64_t b = 0; b < nb; ++b)
      for (int k = 0; k < 4; ++k) tmin[k] = std::min(tmin[k], thr_block[4 * b + k]);
  }
  for (int k = 0; k < 4; ++k)
    if (tmin[k] < 1) return fail(LZ_E_INVAL, "thresholds must be >= 1");
  uint32_t kn = std::min<uint32_t>(std::min(tmin[0], tmin[1]), 8);
  uint32_t kf = std::min<uint32_t>(std::min(tmin[2], tmin[3]), 16);
  std::vector<BlockEnc> blocks(nb);
  uint64_t seg = p->segment ? p->segment : std::max<uint64_t>(n, 1);
  int bits = 10;
  while (bits < 28 && (1ull << bits) < std::min<uint64_t>(seg, n)) ++bits;
  unsigned idx_threads = threads;
  try {
    for (uint64_t s0 = 0; s0 < n; s0 += seg) {
      uint64_t s1 = std::min(n, s0 + seg);
      // indexes of one segment, positions relative to its start
      EncCtx c;
      c.x = in + s0;
      c.n = s1 - s0;
      c.bs = bs;
      c.p = p;
      c.thr_block = thr_block ? thr_block + 4 * (s0 / bs) : nullptr;
      c.seg = 0;
      c.near_idx.prev.assign_zero(s1 - s0 + 16);
      c.far_idx.prev.assign_zero(s1 - s0 + 16);
      build_index(c.x, 0, c.n, kn, idx_threads, c.near_idx, bits);
      build_index(c.x, 0, c.n, kf, idx_threads, c.far_idx, bits);
      uint64_t b0 = s0 / bs, b1 = (s1 + bs - 1) / bs;
      HugeArray<uint16_t> dep;  // byte depths of the previous parse (depth-aware passes)
      for (uint32_t pass = 0; pass <= p->depth_passes; ++pass) {
        if (pass > 0) {
          // dependency depth of every segment byte under the last parse, in
          // output order: literals 0, a match 1 + the deepest byte it reads
          if (!dep.p) dep.assign_zero(s1 - s0);
          for (uint64_t i = 0; i < b1 - b0; ++i) {
            const BlockEnc& e = blocks[b0 + i];
            const BTok* tk = (const BTok*)e.slo.data();
            uint64_t q = i * bs;
            for (size_t j = 0; j < e.slo.size() / sizeof(BTok); ++j) {
              for (uint64_t r = 0; r < tk[j].lit_len; ++r) dep[q + r] = 0;
              q += tk[j].lit_len;
              if (!tk[j].mlen) continue;
              const uint64_t a = tk[j].src - s0, z = std::min(a + tk[j].mlen, q);
              uint32_t m = 0;
              for (uint64_t r = a; r < z; ++r) m = std::max<uint32_t>(m, dep[r]);
              const uint16_t d = (uint16_t)std::min<uint32_t>(m + 1, kDepthMax);
              for (uint64_t r = 0; r < tk[j].mlen; ++r) dep[q + r] = d;
              q += tk[j].mlen;
            }
          }
          c.dep = dep.p;
        }
        parallel_for(b1 - b0, threads, [&](uint64_t i, unsigned) {
          std::vector<BTok> toks;
          BlockEnc& e = blocks[b0 + i];
          parse_block(c, i, toks, e.lit);
          for (auto& t : toks)
            if (t.mlen) t.src += s0;
          // tokens are parked in e.slo until min_match is known
          e.slo.resize(toks.size() * sizeof(BTok));
          memcpy(e.slo.data(), toks.data(), toks.size() * sizeof(BTok));
        });
      }
      if (p->depth_cap) {
        if (!dep.p) dep.assign_zero(s1 - s0);
        cap_depths(c.x, s0, b0, b1, bs, p->depth_cap, blocks, dep.p);
      }
      if (p->progress) p->progress(s1, n, p->progress_user);
    }
  } catch (const std::bad_alloc&) {
    return fail(LZ_E_NOMEM, "encoder allocation failed");
  }
  // min_match: smallest threshold in use (every non-final match reaches it)
  uint64_t mm = std::min(std::min(tmin[0], tmin[1]), std::min(tmin[2], tmin[3]));
  parallel_for(nb, threads, [&](uint64_t b, unsigned) {
    BlockEnc& e = blocks[b];
    std::vector<BTok> toks(e.slo.size() / sizeof(BTok));
    memcpy(toks.data(), e.slo.data(), e.slo.size());
    e.slo.clear();
    encode_block_tokens(toks, mm, e);
  });
  return assemble(n, p->log2_bs, mm, p->thr, p->bound, blocks, tuple_id, arc, arc_size);
}

}  // namespace

}  // namespace lz

using namespace lz;

extern "C" {

int lz_params_default(lz_params* p) {
  if (!p) return fail(LZ_E_INVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->log2_bs = 16;
  p->thr[0] = 6;
  p->thr[1] = 8;
  p->thr[2] = 10;
  p->thr[3] = 12;
  p->bound[0] = 4096;
  p->bound[1] = 65536;
  p->bound[2] = 1 << 20;
  p->max_chain = 32;
  p->n_threads = 0;
  p->segment = 0;
  p->depth_passes = 1;
  return 0;
}

int lz_encode(const uint8_t* in, uint64_t n, const lz_params* p, uint8_t** arc, uint64_t* arc_size) {
  if (p && p->mode > 1) return fail(LZ_E_INVAL, "mode must be 0 (fixed) or 1 (learned)");
  if (p && p->mode == 1) {
    if (!p->mlp_path) return fail(LZ_E_INVAL, "learned mode needs mlp_path");
    lz_selector* sel = nullptr;
    int rc = lz_selector_load(p->mlp_path, &sel);
    if (rc) return rc;
    lz_params q = *p;
    q.mode = 0;
    rc = lz_encode_learned(in, n, &q, sel, arc, arc_size, nullptr);
    lz_selector_free(sel);
    return rc;
  }
  return encode_impl(in, n, p, nullptr, nullptr, arc, arc_size);
}

int lz_encode_blockwise(const uint8_t* in, uint64_t n, const lz_params* p, const uint32_t* thr_per_block,
                        const uint8_t* tuple_id, uint8_t** arc, uint64_t* arc_size) {
  if (!thr_per_block) return fail(LZ_E_INVAL, "null per-block thresholds");
  return encode_impl(in, n, p, thr_per_block, tuple_id, arc, arc_size);
}

int lz_build_archive(uint64_t n, uint32_t log2_bs, uint32_t min_match, uint64_t ntok, const uint32_t* lit_len,
                     const uint32_t* mlen, const uint64_t* src, const uint8_t* lit, uint64_t nlit, uint8_t** arc,
                     uint64_t* arc_size) {
  if (log2_bs < 4 || log2_bs > 24) return fail(LZ_E_INVAL, "log2_bs must be in [4,24]");
  if (!arc || !arc_size || (ntok && (!lit_len || !mlen || !src)) || (nlit && !lit))
    return fail(LZ_E_INVAL, "null argument");
  uint64_t bs = 1ull << log2_bs;
  uint64_t nb = (n + bs - 1) / bs;
  std::vector<std::vector<BTok>> per(nb);
  std::vector<BlockEnc> blocks(nb);
  uint64_t pos = 0, lp = 0;
  // cut tokens at block ends; a match piece keeps its distance
  auto blk_of = [&](uint64_t q) { return q / bs; };
  for (uint64_t t = 0; t < ntok; ++t) {
    uint64_t L = lit_len[t];
    if (pos + L > n || lp + L > nlit) return fail(LZ_E_INVAL, "token %llu overruns", (unsigned long long)t);
    while (L) {
      uint64_t b = blk_of(pos);
      uint64_t take = std::min<uint64_t>(L, (b + 1) * bs - pos);
      auto& v = per[b];
      if (v.empty() || v.back().mlen || pos == b * bs) {
        if (pos == b * bs && !v.empty()) return fail(LZ_E_INVAL, "internal cut error");
        v.push_back(BTok{take, 0, 0});
      } else {
        v.back().lit_len += take;
      }
      blocks[b].lit.insert(blocks[b].lit.end(), lit + lp, lit + lp + take);
      lp += take;
      pos += take;
      L -= take;
    }
    uint64_t M = mlen[t], s = src[t];
    if (M && (s >= pos || pos + M > n)) return fail(LZ_E_INVAL, "token %llu has a bad match", (unsigned long long)t);
    while (M) {
      uint64_t b = blk_of(pos);
      uint64_t take = std::min<uint64_t>(M, (b + 1) * bs - pos);
      auto& v = per[b];
      if (v.empty() || v.back().mlen)
        v.push_back(BTok{0, take, s});
      else {
        v.back().mlen = take;
        v.back().src = s;
      }
      pos += take;
      s += take;
      M -= take;
    }
  }
  if (pos != n || lp != nlit) return fail(LZ_E_INVAL, "tokens cover %llu of %llu bytes", (unsigned long long)pos,
                                          (unsigned long long)n);
  uint64_t mm = min_match;
  if (!mm) {
    mm = UINT64_MAX;
    for (auto& v : per)
      for (size_t i = 0; i + 1 < v.size(); ++i) mm = std::min<uint64_t>(mm, v[i].mlen);
    if (mm == UINT64_MAX || mm == 0) mm = 1;
  }
  for (auto& v : per)
    for (size_t i = 0; i + 1 < v.size(); ++i)
      if (v[i].mlen < mm) return fail(LZ_E_INVAL, "match shorter than min_match");
  for (uint64_t b = 0; b < nb; ++b) encode_block_tokens(per[b], mm, blocks[b]);
  return assemble(n, log2_bs, mm, nullptr, nullptr, blocks, nullptr, arc, arc_size);
}

void lz_free(void* p) { free(p); }

const char* lz_last_error(void) { return g_err.c_str(); }

uint64_t lz_fnv1a64(const uint8_t* p, uint64_t n, uint64_t seed) {
  uint64_t h = seed;
  for (uint64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

static int len_bin(uint64_t L) {
  static const uint64_t edges[16] = {0, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64, 128, 256, 1024, 4096, 16384};
  int b = 0;
  while (b < 15 && L >= edges[b + 1]) ++b;
  return b;
}

int lz_archive_info(const uint8_t* arc, uint64_t arc_size, lz_info* out) {
  if (!out) return fail(LZ_E_INVAL, "null output");
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  memset(out, 0, sizeof(*out));
  out->n = v.n;
  out->n_blocks = v.nb;
  out->n_tok = v.n_tok;
  out->n_lit = v.n_lit;
  out->archive_bytes = v.total;
  out->log2_bs = v.log2_bs;
  out->min_match = (uint32_t)v.min_match;
  for (int k = 0; k < 4; ++k) out->thr[k] = v.thr[k];
  for (int k = 0; k < 3; ++k) out->bound[k] = v.bound[k];
  uint64_t bnd[3] = {v.bound[0] ? v.bound[0] : 4096, v.bound[1] ? v.bound[1] : 65536,
                     v.bound[2] ? v.bound[2] : (1u << 20)};
  unsigned T = hw_threads(0);
  std::vector<lz_info> part(T);
  for (auto& p : part) memset(&p, 0, sizeof(p));
  std::atomic<int> bad{0};
  parallel_for(v.nb, T, [&](uint64_t b, unsigned w) {
    lz_info& P = part[w];
    int r = walk_block(v, b, [&](uint64_t, const Tok& t) {
      if (!t.mlen) return;
      P.n_match++;
      P.match_bytes += t.mlen;
      if (t.mlen < 32) P.frac_lt32 += 1;
      uint64_t d = t.dst + t.lit_len - t.src;
      P.hist[dclass(d, bnd)][len_bin(t.mlen)]++;
    });
    if (r) bad.store(r);
  });
  if (bad.load()) return fail(LZ_E_CORRUPT, "archive fails validation");
  double lt32 = 0;
  for (auto& P : part) {
    out->n_match += P.n_match;
    out->match_bytes += P.match_bytes;
    lt32 += P.frac_lt32;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 16; ++b) out->hist[a][b] += P.hist[a][b];
  }
  out->mean_match = out->n_match ? double(out->match_bytes) / double(out->n_match) : 0.0;
  out->frac_lt32 = out->n_match ? lt32 / double(out->n_match) : 0.0;
  out->coverage = v.n ? double(out->match_bytes) / double(v.n) : 0.0;
  out->src_bytes = v.n_tok * ((v.flags & 1) ? 5 : 4);
  return 0;
}

static double tile_entropy_bytes(const uint8_t* p, uint64_t len, uint64_t stride) {
  const uint64_t T = 65536;
  double total = 0;
  for (uint64_t o = 0; o < len; o += T) {
    uint64_t m = std::min(T, len - o);
    uint64_t cnt[256] = {0};
    for (uint64_t i = 0; i < m; ++i) cnt[p[(o + i) * stride]]++;
    double bits = 0;
    int distinct = 0;
    for (int s = 0; s < 256; ++s)
      if (cnt[s]) {
        ++distinct;
        bits += double(cnt[s]) * (log2(double(m)) - log2(double(cnt[s])));
      }
    total += ceil(bits / 8.0 - 1e-9) + 1.0 + 2.0 * distinct;
  }
  return total;
}

int lz_entropy_size(const uint8_t* arc, uint64_t arc_size, double* total, double* parts) {
  if (!total) return fail(LZ_E_INVAL, "null output");
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  double p[7] = {0, 0, 0, 0, 0, 0, 0};
  p[0] = tile_entropy_bytes(v.base + v.off_cmd, v.n_tok, 1);
  p[1] = tile_entropy_bytes(v.base + v.off_x16, 2 * v.n_x16, 1);
  p[2] = tile_entropy_bytes(v.base + v.off_x32, 4 * v.n_x32, 1);
  for (int k = 0; k < 4; ++k) p[3] += tile_entropy_bytes(v.base + v.off_slo + k, v.n_tok, 4);
  if (v.flags & 1) p[6] = tile_entropy_bytes(v.base + v.off_shi, v.n_tok, 1);
  p[4] = tile_entropy_bytes(v.base + v.off_lit, v.n_lit, 1);
  p[5] = double(kHeader) + 32.0 * double(v.nb + 1);
  double s = 0;
  for (double q : p) s += q;
  *total = s;
  if (parts) memcpy(parts, p, sizeof(p));
  return 0;
}

}  // extern "C"

namespace lz {

// Levels by a sequential sweep in block order.  Each block keeps its runs
// (literal runs at level 0, match pieces at their level) sorted by start, so a
// source interval is resolved by a binary search in the source block's runs
// only; a source interval that spans two blocks is split.
int compute_levels(const ArcView& v, uint32_t* levels, uint32_t* max_level, uint8_t* has_match) {
  // Dependency depth: literal bytes 0, a match 1 + the largest depth among the
  // writers of its source bytes (its own output excluded).  Per block, the
  // output is kept as runs {start, depth} of the tokens' literal and match
  // parts, so a source interval is answered by a binary search and a scan.
  struct Run {
    uint32_t start;  // offset in block
    uint32_t depth;
  };
  std::vector<std::vector<Run>> runs(v.nb);
  uint32_t mx = 0;
  for (uint64_t b = 0; b < v.nb; ++b) {
    std::vector<Run>& mine = runs[b];
    int rc = walk_block(v, b, [&](uint64_t t, const Tok& k) {
      const uint64_t b0 = b << v.log2_bs;
      if (k.lit_len) mine.push_back(Run{uint32_t(k.dst - b0), 0});
      uint32_t dep = 0;
      if (k.mlen) {
        const uint64_t m0 = k.dst + k.lit_len;
        const uint64_t s = k.src, e = std::min(k.src + k.mlen, m0);  // own bytes excluded
        uint32_t deepest = 0;
        for (uint64_t q = s; q < e;) {
          const uint64_t sb = q >> v.log2_bs;
          const uint64_t sb_end = std::min(e, (sb + 1) << v.log2_bs);
          const std::vector<Run>& R = runs[sb];
          const uint32_t lo = uint32_t(q - (sb << v.log2_bs)), hi = uint32_t(sb_end - (sb << v.log2_bs));
          // last run starting at or before lo, then every run starting before hi
          size_t i = std::upper_bound(R.begin(), R.end(), lo, [](uint32_t x, const Run& r) { return x < r.start; }) -
                     R.begin();
          i = i ? i - 1 : 0;
          for (; i < R.size() && R[i].start < hi; ++i) deepest = std::max(deepest, R[i].depth);
          q = sb_end;
        }
        dep = deepest + 1;
        mine.push_back(Run{uint32_t(m0 - b0), dep});
      }
      if (levels) levels[t] = dep;
      if (has_match) has_match[t] = k.mlen ? 1 : 0;
      mx = std::max(mx, dep);
    });
    if (rc) return fail(LZ_E_CORRUPT, "block %llu fails validation", (unsigned long long)b);
  }
  *max_level = mx;
  return 0;
}

}  // namespace lz

extern "C" int lz_plan(const uint8_t* arc, uint64_t arc_size, uint32_t* levels, uint32_t* max_level) {
  if (!max_level) return fail(LZ_E_INVAL, "null output");
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  return compute_levels(v, levels, max_level);
}

// ------------------------------------------------------------------ per-block statistics

namespace lz {
static int len_bin16(uint64_t L) {
  static const uint64_t edges[16] = {0, 6, 8, 10, 12, 16, 20, 24, 32, 48, 64, 128, 256, 1024, 4096, 16384};
  int b = 0;
  while (b < 15 && L >= edges[b + 1]) ++b;
  return b;
}
}  // namespace lz

extern "C" {

// feats[64*b + 16*c + k] = fraction of block b's bytes produced by matches of
// distance class c (bounds as given) and length bin k.
int lz_block_features(const uint8_t* arc, uint64_t arc_size, const uint64_t* bounds, float* feats) {
  if (!feats || !bounds) return fail(LZ_E_INVAL, "null argument");
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  std::atomic<int> bad{0};
  parallel_for(v.nb, hw_threads(0), [&](uint64_t b, unsigned) {
    double acc[64] = {0};
    int r = walk_block(v, b, [&](uint64_t, const Tok& t) {
      if (!t.mlen) return;
      const uint64_t d = t.dst + t.lit_len - t.src;
      acc[16 * dclass(d, bounds) + len_bin16(t.mlen)] += double(t.mlen);
    });
    if (r) bad.store(r);
    const double len = double(std::min(v.bs, v.n - b * v.bs));
    for (int k = 0; k < 64; ++k) feats[64 * b + k] = float(acc[k] / len);
  });
  if (bad.load()) return fail(LZ_E_CORRUPT, "archive fails validation");
  return 0;
}

// Per block: entropy-bound bytes of its streams (each stream of the block one
// tile, same charge as lz_entropy_size), token count, match count, match bytes.
int lz_block_stats(const uint8_t* arc, uint64_t arc_size, double* ent, uint64_t* ntok, uint64_t* nmatch,
                   uint64_t* match_bytes) {
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  std::atomic<int> bad{0};
  const uint64_t* T = v.tab();
  parallel_for(v.nb, hw_threads(0), [&](uint64_t b, unsigned) {
    uint64_t nm = 0, mb = 0;
    int r = walk_block(v, b, [&](uint64_t, const Tok& t) {
      if (t.mlen) {
        ++nm;
        mb += t.mlen;
      }
    });
    if (r) bad.store(r);
    const uint64_t t0 = T[4 * b], t1 = T[4 * b + 4];
    const uint64_t l0 = T[4 * b + 1], l1 = T[4 * b + 5];
    const uint64_t x0 = T[4 * b + 2], x1 = T[4 * b + 6];
    const uint64_t y0 = T[4 * b + 3], y1 = T[4 * b + 7];
    if (ent) {
      double e = tile_entropy_bytes(v.base + v.off_cmd + t0, t1 - t0, 1);
      e += tile_entropy_bytes(v.base + v.off_x16 + 2 * x0, 2 * (x1 - x0), 1);
      e += tile_entropy_bytes(v.base + v.off_x32 + 4 * y0, 4 * (y1 - y0), 1);
      for (int k = 0; k < 4; ++k) e += tile_entropy_bytes(v.base + v.off_slo + 4 * t0 + k, t1 - t0, 4);
      if (v.flags & 1) e += tile_entropy_bytes(v.base + v.off_shi + t0, t1 - t0, 1);
      e += tile_entropy_bytes(v.base + v.off_lit + l0, l1 - l0, 1);
      ent[b] = e;
    }
    if (ntok) ntok[b] = t1 - t0;
    if (nmatch) nmatch[b] = nm;
    if (match_bytes) match_bytes[b] = mb;
  });
  if (bad.load()) return fail(LZ_E_CORRUPT, "archive fails validation");
  return 0;
}

}  // extern "C"
