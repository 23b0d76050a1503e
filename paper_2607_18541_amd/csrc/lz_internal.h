// lz_internal.h -- shared host-side structures of liblz (not part of the ABI).
#pragma once
#include <stdint.h>

#include <array>
#include <atomic>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lz.h"

namespace lz {

constexpr uint32_t kMagic = 0x314D5A4Cu;
constexpr uint64_t kHeader = 128;

void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

inline uint64_t align16(uint64_t v) { return (v + 15) & ~uint64_t(15); }

// Parsed header + stream offsets of a container (version 1).
struct ArcView {
  const uint8_t* base = nullptr;
  uint64_t size = 0;
  uint64_t n = 0, bs = 0, nb = 0, min_match = 0, flags = 0;
  uint64_t n_tok = 0, n_x16 = 0, n_x32 = 0, n_lit = 0;
  uint32_t log2_bs = 0;
  uint32_t thr[4] = {0, 0, 0, 0};
  uint64_t bound[3] = {0, 0, 0};
  uint64_t off_tab = 0, off_cmd = 0, off_x16 = 0, off_x32 = 0, off_slo = 0, off_shi = 0, off_lit = 0,
           off_info = 0, total = 0;
  // block table entry b: {tok, lit, x16, x32}
  const uint64_t* tab() const { return reinterpret_cast<const uint64_t*>(base + off_tab); }
};

// Header and table checks only.
int view_archive(const uint8_t* arc, uint64_t size, ArcView* v);
// The layout a 128-byte header describes (offsets and total; no table checks).
int view_header(const uint8_t* arc, ArcView* v);

// A decoded token, block-local order.
struct Tok {
  uint64_t dst;      // token start (absolute)
  uint64_t lit_len;
  uint64_t lit_off;  // offset in the lit stream
  uint64_t mlen;
  uint64_t src;
  uint64_t x16_off;  // extension cursors before this token
  uint64_t x32_off;
};

// Walks block b's tokens, validating every container rule; calls f(tok_index,
// Tok) for each.  Returns 0 or LZ_E_CORRUPT.
template <class F>
int walk_block(const ArcView& v, uint64_t b, F&& f);

// Full validation (all blocks, multithreaded).
int validate_archive(const ArcView& v, uint32_t n_threads);

// Per-token levels (see lz_plan); returns max level.
int compute_levels(const ArcView& v, uint32_t* levels, uint32_t* max_level, uint8_t* has_match = nullptr);

unsigned hw_threads(uint32_t requested);

// Tile-rANS entropy stage: tiles of at most kRansTile symbols, probabilities
// in units of 1/kRansM, 32-bit states in [kRansL, 2^32), kRansLanes states.
constexpr uint64_t kRansTile = 65536;
constexpr uint64_t kCodedHead = 192;  // 64-byte header + a copy of the 128-byte container header
constexpr uint32_t kRansM = 4096, kRansL = 1u << 16, kRansLanes = 64;
bool rans_normalise(const uint64_t* count, uint64_t N, uint32_t* f);
uint64_t rans_encode_tile(const uint8_t* sym, uint64_t stride, uint32_t N, std::vector<uint8_t>& out);
struct CodedView {
  const uint8_t* base = nullptr;
  uint64_t size = 0, out_size = 0, n_tiles = 0, dir = 0, payload = 0;
};
// Header and directory checks of a coded container (bounds, tables, coverage).
int parse_coded(const uint8_t* a, uint64_t size, CodedView* v);
// Launches the tile decoder: tiles of the coded container at d_coded (device)
// into d_out (the decoded container); d_err bit 0: a word read past a
// payload, bit 1: a tile did not end in the encoder's initial states.
int entropy_launch(const uint8_t* d_coded, uint64_t payload_off, uint64_t n_tiles, uint8_t* d_out, uint32_t* d_err,
                   int cu_count, void* stream);

// Pinned staging that a handle keeps for its synchronous range calls: lends
// the plan its staging (P->staging, not owned by the plan) followed, at a
// 256-byte boundary, by `extra` bytes, whose address it returns.  `lock`
// holds the handle's lock for these calls until the caller has synchronised
// its stream.  nullptr (and no loan) if the pinned allocation fails.
uint8_t* lend_sync_staging(lz_dev* h, lz_range_plan* P, uint64_t extra, std::unique_lock<std::mutex>& lock);

// Learned threshold selector (host object behind lz_selector).
constexpr uint32_t kSelIn = 64, kSelHidden = 128, kSelTuples = 16;
constexpr uint64_t kSelParams = kSelIn * kSelHidden + kSelHidden + kSelHidden * kSelHidden + kSelHidden +
                                kSelHidden * kSelTuples + kSelTuples;  // 26,896

}  // namespace lz

struct lz_selector {
  uint32_t tuples[lz::kSelTuples][4];
  uint32_t fixed = 1;                   // fallback tuple
  float mu[lz::kSelIn], sd[lz::kSelIn];  // feature normalisation
  float val_J[lz::kSelTuples];          // mean validation cost per predicted tuple, relative to the fixed one
  std::vector<float> params;            // kSelParams, row-major W1 b1 W2 b2 W3 b3
};

// ---------------------------------------------------------------- inline impl
namespace lz {

static inline uint64_t rd_le(const uint8_t* p, int k) {
  uint64_t v = 0;
  for (int i = 0; i < k; ++i) v |= uint64_t(p[i]) << (8 * i);
  return v;
}

template <class F>
int walk_block(const ArcView& v, uint64_t b, F&& f) {
  const uint64_t* T = v.tab();
  uint64_t t0 = T[4 * b + 0], t1 = T[4 * b + 4];
  uint64_t lc = T[4 * b + 1], lc1 = T[4 * b + 5];
  uint64_t xc = T[4 * b + 2], xc1 = T[4 * b + 6];
  uint64_t yc = T[4 * b + 3], yc1 = T[4 * b + 7];
  uint64_t pos = b * v.bs;
  uint64_t end = pos + v.bs < v.n ? pos + v.bs : v.n;
  if (t1 <= t0) return LZ_E_CORRUPT;
  const uint8_t* cmd = v.base + v.off_cmd;
  const uint8_t* x16 = v.base + v.off_x16;
  const uint8_t* x32 = v.base + v.off_x32;
  const uint8_t* slo = v.base + v.off_slo;
  const uint8_t* shi = (v.flags & 1) ? v.base + v.off_shi : nullptr;
  for (uint64_t t = t0; t < t1; ++t) {
    const uint64_t xc0 = xc, yc0 = yc;
    uint8_t c = cmd[t];
    uint64_t val[2] = {uint64_t(c >> 4), uint64_t(c & 15)};
    bool last = (t + 1 == t1);
    for (int k = 0; k < 2; ++k) {
      if (val[k] != 15 || (k == 1 && last)) continue;
      if (xc >= xc1) return LZ_E_CORRUPT;
      uint64_t e = rd_le(x16 + 2 * xc, 2);
      ++xc;
      if (e == 0xFFFF) {
        if (yc >= yc1) return LZ_E_CORRUPT;
        e += rd_le(x32 + 4 * yc, 4);
        ++yc;
      }
      val[k] = 15 + e;
    }
    uint64_t lit_len = val[0];
    if (lit_len > end - pos || lit_len > lc1 - lc) return LZ_E_CORRUPT;
    uint64_t mstart = pos + lit_len;
    uint64_t mlen;
    if (last) {
      if ((c & 15) != 0) return LZ_E_CORRUPT;
      mlen = end - mstart;
    } else {
      mlen = v.min_match + val[1];
      if (mlen > end - mstart) return LZ_E_CORRUPT;
    }
    uint64_t src = rd_le(slo + 4 * t, 4);
    if (shi) src |= uint64_t(shi[t]) << 32;
    if (mlen > 0 && src >= mstart) return LZ_E_CORRUPT;
    if (mlen == 0 && src != 0) return LZ_E_CORRUPT;
    f(t, Tok{pos, lit_len, lc, mlen, src, xc0, yc0});
    lc += lit_len;
    pos = mstart + mlen;
  }
  if (pos != end || lc != lc1 || xc != xc1 || yc != yc1) return LZ_E_CORRUPT;
  return 0;
}

}  // namespace lz
