// lz_entropy.cpp -- host side of the tile-rANS entropy stage.
//
// The paper's pipeline decodes entropy over 64 KB tiles cut across each flat
// stream independently of the LZ block size (Sec. 2, Experimental Setup),
// before the match phase.  Here every byte region of a container (header and
// block table, each stream, and each byte plane of the 32-bit sources) is cut
// into tiles of at most 65,536 symbols; a tile is stored raw, as one repeated
// byte, or order-0 rANS coded (Duda's range variant of asymmetric numeral
// systems) with 64 interleaved states, so one GPU wave decodes one tile.
//
// rANS tile (the coder of this library; the paper names tile-ANS only):
//   probabilities quantised to M = 2^12: f[s] = floor(count[s] M / N), raised
//   to 1 for present symbols, the sum corrected to M on the most frequent
//   symbol (lowest byte value among equals: the remainder added there, or
//   taken 1 at a time from the symbol with the largest f that is above 1);
//   c[s] = sum of f below s.  States are 32-bit in [2^16, 2^32); symbol i of
//   the tile belongs to state i mod 64.  Decoding symbol s from state x:
//   slot = x mod M, s = the symbol with c[s] <= slot < c[s] + f[s],
//   x = f[s] (x >> 12) + slot - c[s], then, if x < 2^16, x = (x << 16) | the
//   next 16-bit word.  Words are consumed in symbol order (i ascending).
//   The encoder runs in reverse and emits a word (the low 16 bits) before a
//   symbol whose state is >= f[s] << 20.
//   Payload: 32-byte presence bitmap, u16 f per present symbol (ascending),
//   u32 initial decoder state per lane (64), u16 words.
//
// Coded container ("LZE1", little-endian): 64-byte header {magic "LZE1" 0 0
// 0 0, u64 size of the decoded container, u32 n_tiles, u32 0, u64 directory
// offset (192), u64 payload offset, u64 total size, 16 zero bytes}, then the
// decoded container's own 128-byte header (so its layout is known before
// decoding); directory
// of 32-byte tile records {u64 payload offset (from the payload start), u64
// first output byte, u32 symbols (1..65536), u32 payload bytes, u32 output
// stride (1 or 4), u32 mode (0 raw, 1 rANS, 2 one repeated byte)}; payloads.
// Every output byte is written by exactly one tile (checked on decode).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "lz_internal.h"

using namespace lz;

namespace lz {

bool rans_normalise(const uint64_t* count, uint64_t N, uint32_t* f) {
  uint32_t sum = 0;
  int top = -1;
  for (int s = 0; s < 256; ++s) {
    f[s] = 0;
    if (!count[s]) continue;
    f[s] = std::max<uint32_t>(1, (uint32_t)(count[s] * kRansM / N));
    sum += f[s];
    if (top < 0 || count[s] > count[top]) top = s;
  }
  if (top < 0) return false;
  if (sum < kRansM) {
    f[top] += kRansM - sum;
  } else {
    while (sum > kRansM) {
      int big = -1;
      for (int s = 0; s < 256; ++s)
        if (f[s] > 1 && (big < 0 || f[s] > f[big])) big = s;
      if (big < 0) return false;
      --f[big];
      --sum;
    }
  }
  return true;
}

uint64_t rans_encode_tile(const uint8_t* sym, uint64_t stride, uint32_t N, std::vector<uint8_t>& out) {
  uint64_t count[256] = {0};
  for (uint32_t i = 0; i < N; ++i) ++count[sym[i * stride]];
  uint32_t f[256], c[256];
  if (!rans_normalise(count, N, f)) return 0;
  uint32_t acc = 0;
  for (int s = 0; s < 256; ++s) {
    c[s] = acc;
    acc += f[s];
  }
  uint32_t x[kRansLanes];
  for (uint32_t j = 0; j < kRansLanes; ++j) x[j] = kRansL;
  std::vector<uint16_t> words;
  words.reserve(N / 2 + 64);
  for (uint32_t i = N; i-- > 0;) {
    const uint32_t s = sym[i * stride], j = i % kRansLanes;
    uint32_t v = x[j];
    if (v >= (f[s] << 20)) {
      words.push_back((uint16_t)(v & 0xFFFF));
      v >>= 16;
    }
    x[j] = ((v / f[s]) << 12) + (v % f[s]) + c[s];
  }
  std::reverse(words.begin(), words.end());
  const size_t o = out.size();
  uint32_t nsym = 0;
  for (int s = 0; s < 256; ++s) nsym += f[s] ? 1 : 0;
  out.resize(o + 32 + 2 * nsym + 4 * kRansLanes + 2 * words.size(), 0);
  uint8_t* p = out.data() + o;
  for (int s = 0; s < 256; ++s)
    if (f[s]) p[s >> 3] |= uint8_t(1u << (s & 7));
  p += 32;
  for (int s = 0; s < 256; ++s)
    if (f[s]) {
      p[0] = uint8_t(f[s]);
      p[1] = uint8_t(f[s] >> 8);
      p += 2;
    }
  for (uint32_t j = 0; j < kRansLanes; ++j, p += 4)
    for (int k = 0; k < 4; ++k) p[k] = uint8_t(x[j] >> (8 * k));
  for (uint16_t w : words) {
    p[0] = uint8_t(w);
    p[1] = uint8_t(w >> 8);
    p += 2;
  }
  return out.size() - o;
}

int parse_coded(const uint8_t* a, uint64_t size, CodedView* v) {
  if (!a || size < 64 || memcmp(a, "LZE1\0\0\0\0", 8) != 0) return fail(LZ_E_CORRUPT, "not a coded container");
  v->base = a;
  v->size = size;
  v->out_size = rd_le(a + 8, 8);
  v->n_tiles = rd_le(a + 16, 4);
  v->dir = rd_le(a + 24, 8);
  v->payload = rd_le(a + 32, 8);
  const uint64_t total = rd_le(a + 40, 8);
  if (total != size || v->dir != kCodedHead || v->payload != kCodedHead + 32 * v->n_tiles || v->payload > size ||
      v->out_size > (1ull << 48) || v->out_size < kHeader)
    return fail(LZ_E_CORRUPT, "coded container header inconsistent");
  ArcView hv;  // the copied header must describe a container of out_size bytes
  if (size < kCodedHead || view_header(a + 64, &hv) != 0 || hv.total != v->out_size)
    return fail(LZ_E_CORRUPT, "coded container's header copy does not describe its decoded size");
  // every tile inside the payload; tiles pairwise disjoint and together as
  // many symbols as output bytes, so every output byte is written exactly once
  std::vector<std::pair<uint64_t, uint64_t>> bytes;            // stride 1: [dst, dst + cnt)
  std::vector<std::pair<uint64_t, uint64_t>> words[4];         // stride 4, per residue: [dst / 4, dst / 4 + cnt)
  uint64_t covered = 0;
  for (uint64_t t = 0; t < v->n_tiles; ++t) {
    const uint8_t* r = a + kCodedHead + 32 * t;
    const uint64_t po = rd_le(r, 8), dst = rd_le(r + 8, 8);
    const uint64_t cnt = rd_le(r + 16, 4), pb = rd_le(r + 20, 4), stride = rd_le(r + 24, 4), mode = rd_le(r + 28, 4);
    if (cnt < 1 || cnt > kRansTile || !(stride == 1 || stride == 4) || mode > 2)
      return fail(LZ_E_CORRUPT, "tile %llu: bad record", (unsigned long long)t);
    if (po > size - v->payload || pb > size - v->payload - po)
      return fail(LZ_E_CORRUPT, "tile %llu: payload outside the container", (unsigned long long)t);
    if (dst >= v->out_size || (v->out_size - 1 - dst) / stride < cnt - 1)
      return fail(LZ_E_CORRUPT, "tile %llu: output outside", (unsigned long long)t);
    const uint8_t* p = a + v->payload + po;
    if (mode == 0 && pb != cnt) return fail(LZ_E_CORRUPT, "tile %llu: raw size", (unsigned long long)t);
    if (mode == 2 && pb != 1) return fail(LZ_E_CORRUPT, "tile %llu: repeat size", (unsigned long long)t);
    if (mode == 1) {
      if (pb < 32) return fail(LZ_E_CORRUPT, "tile %llu: short rANS payload", (unsigned long long)t);
      uint32_t nsym = 0, sum = 0;
      for (int q = 0; q < 256; ++q) nsym += (p[q >> 3] >> (q & 7)) & 1;
      const uint64_t head = 32 + 2ull * nsym + 4ull * kRansLanes;
      if (nsym == 0 || pb < head || ((pb - head) & 1))
        return fail(LZ_E_CORRUPT, "tile %llu: rANS layout", (unsigned long long)t);
      for (uint32_t k = 0; k < nsym; ++k) {
        const uint32_t fk = (uint32_t)rd_le(p + 32 + 2 * k, 2);
        if (fk == 0) return fail(LZ_E_CORRUPT, "tile %llu: zero frequency", (unsigned long long)t);
        sum += fk;
      }
      if (sum != kRansM) return fail(LZ_E_CORRUPT, "tile %llu: frequencies do not sum to 4096", (unsigned long long)t);
      for (uint32_t j = 0; j < kRansLanes; ++j)
        if (rd_le(p + 32 + 2 * nsym + 4 * j, 4) < kRansL)
          return fail(LZ_E_CORRUPT, "tile %llu: state below 2^16", (unsigned long long)t);
    }
    if (stride == 1) bytes.push_back({dst, dst + cnt});
    else words[dst & 3].push_back({dst >> 2, (dst >> 2) + cnt});
    covered += cnt;
  }
  if (covered != v->out_size)
    return fail(LZ_E_CORRUPT, "tiles cover %llu of %llu output bytes", (unsigned long long)covered,
                (unsigned long long)v->out_size);
  auto disjoint = [](std::vector<std::pair<uint64_t, uint64_t>>& iv) {
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i)
      if (iv[i].first < iv[i - 1].second) return false;
    return true;
  };
  if (!disjoint(bytes)) return fail(LZ_E_CORRUPT, "tiles overlap");
  for (int q = 0; q < 4; ++q) {
    if (!disjoint(words[q])) return fail(LZ_E_CORRUPT, "plane tiles overlap");
    // a plane tile's bytes lie in [4 w0, 4 w1): no stride-1 tile may reach there
    for (auto& w : words[q]) {
      const uint64_t b0 = 4 * w.first, b1 = 4 * w.second;
      auto it = std::lower_bound(bytes.begin(), bytes.end(), std::make_pair(b0, uint64_t(0)));
      if ((it != bytes.end() && it->first < b1) || (it != bytes.begin() && std::prev(it)->second > b0))
        return fail(LZ_E_CORRUPT, "plane and byte tiles overlap");
    }
  }
  return 0;
}

}  // namespace lz

namespace {

struct Region {
  uint64_t dst, count, stride;
};

// Regions of a container: every byte exactly once; the 32-bit sources as four
// byte planes (byte k of every source at stride 4).
std::vector<Region> regions_of(const ArcView& v) {
  std::vector<Region> R;
  uint64_t pos = 0;
  auto bytes_to = [&](uint64_t end) {
    if (end > pos) R.push_back({pos, end - pos, 1});
    pos = std::max(pos, end);
  };
  bytes_to(v.off_slo);
  if (v.n_tok) {
    for (uint64_t k = 0; k < 4; ++k) R.push_back({v.off_slo + k, v.n_tok, 4});
    pos = v.off_slo + 4 * v.n_tok;
  }
  bytes_to(v.total);
  return R;
}

}  // namespace

extern "C" {

int lz_entropy_encode(const uint8_t* arc, uint64_t arc_size, uint8_t** out, uint64_t* out_size) {
  if (!out || !out_size) return fail(LZ_E_INVAL, "null argument");
  ArcView v;
  int rc = view_archive(arc, arc_size, &v);
  if (rc) return rc;
  const std::vector<Region> R = regions_of(v);
  struct Tile {
    uint64_t dst, cnt, stride, mode;
    std::vector<uint8_t> pay;
  };
  std::vector<Tile> tiles;
  for (const Region& g : R)
    for (uint64_t i0 = 0; i0 < g.count; i0 += kRansTile) tiles.push_back({g.dst + i0 * g.stride,
                                                                          std::min(kRansTile, g.count - i0), g.stride,
                                                                          0, {}});
  const unsigned W = hw_threads(0);
  std::vector<std::thread> pool;
  std::atomic<uint64_t> next{0};
  for (unsigned w = 0; w < W; ++w)
    pool.emplace_back([&] {
      for (;;) {
        const uint64_t t = next.fetch_add(1);
        if (t >= tiles.size()) break;
        Tile& T = tiles[t];
        const uint8_t* s = arc + T.dst;
        bool same = true;
        for (uint64_t i = 1; i < T.cnt && same; ++i) same = s[i * T.stride] == s[0];
        if (same) {
          T.mode = 2;
          T.pay.assign(1, s[0]);
          continue;
        }
        std::vector<uint8_t> r;
        const uint64_t nb = rans_encode_tile(s, T.stride, (uint32_t)T.cnt, r);
        if (nb && nb < T.cnt) {
          T.mode = 1;
          T.pay.swap(r);
        } else {
          T.mode = 0;
          T.pay.resize(T.cnt);
          for (uint64_t i = 0; i < T.cnt; ++i) T.pay[i] = s[i * T.stride];
        }
      }
    });
  for (auto& t : pool) t.join();
  uint64_t pay = 0;
  for (auto& T : tiles) pay += T.pay.size();
  const uint64_t dir = kCodedHead, p0 = dir + 32 * tiles.size(), total = p0 + pay;
  uint8_t* a = (uint8_t*)calloc(total ? total : 1, 1);
  if (!a) return fail(LZ_E_NOMEM, "coded container allocation failed");
  auto wr = [&](uint64_t o, uint64_t val, int k) {
    for (int i = 0; i < k; ++i) a[o + i] = uint8_t(val >> (8 * i));
  };
  memcpy(a, "LZE1\0\0\0\0", 8);
  wr(8, v.total, 8);
  wr(16, tiles.size(), 4);
  wr(24, dir, 8);
  wr(32, p0, 8);
  wr(40, total, 8);
  memcpy(a + 64, arc, kHeader);
  uint64_t po = 0;
  for (size_t t = 0; t < tiles.size(); ++t) {
    const Tile& T = tiles[t];
    const uint64_t r = dir + 32 * t;
    wr(r, po, 8);
    wr(r + 8, T.dst, 8);
    wr(r + 16, T.cnt, 4);
    wr(r + 20, T.pay.size(), 4);
    wr(r + 24, T.stride, 4);
    wr(r + 28, T.mode, 4);
    memcpy(a + p0 + po, T.pay.data(), T.pay.size());
    po += T.pay.size();
  }
  *out = a;
  *out_size = total;
  return 0;
}

int lz_entropy_info(const uint8_t* coded, uint64_t size, uint64_t* decoded_size, uint64_t* tiles,
                    uint64_t* tiles_by_mode) {
  CodedView v;
  int rc = parse_coded(coded, size, &v);
  if (rc) return rc;
  if (decoded_size) *decoded_size = v.out_size;
  if (tiles) *tiles = v.n_tiles;
  if (tiles_by_mode) {
    tiles_by_mode[0] = tiles_by_mode[1] = tiles_by_mode[2] = 0;
    for (uint64_t t = 0; t < v.n_tiles; ++t) ++tiles_by_mode[rd_le(coded + kCodedHead + 32 * t + 28, 4)];
  }
  return 0;
}

}  // extern "C"
