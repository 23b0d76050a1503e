// lz_device.hip -- gfx950 match-phase decoder of absolute-offset LZ77.
//
// Work is done by groups of G lanes of a 64-lane wave (Sec. 2: cooperation
// width G; Sec. 3.1: lanes = G x N_blocks).  A decode is a parse launch
// followed by the match passes:
//
//  parse  One group per segment of 128 tokens of one block: each lane reads
//         one token header (cmd byte, source, plan slot), a group prefix count
//         locates the length extensions, and prefix sums give every token's
//         output position and literal offset, so G tokens are parsed per
//         step.  Each match is stored as a 16-byte record {dst, length, src}
//         at its slot of the match table, which is in plan order (below).
//         The literals of the G tokens are written as the aligned 16-byte
//         blocks of their whole output span when literals are dense (match
//         bytes get arbitrary values there and are rewritten by the match
//         passes), else run by run.
//  match  The plan (computed on the host when the archive is opened) gives
//         each match a dependency depth: literal bytes have depth 0, a match
//         has one more than the deepest token that wrote any of its source
//         bytes (its own bytes excluded), so matches of one depth never read
//         each other's output.  Slots are ordered by (depth, token) and cut
//         into windows of at most 64 matches and 3 KiB inside one output
//         grain of max(2^20, block) bytes (a longer match is split over
//         windows), so a range decode that starts at a grain boundary (its
//         decode horizon) runs whole windows.  Schedule 1 launches each
//         depth's windows separately (kernel boundaries order the depths)
//         with ordinary cached accesses, and runs the deepest, smallest
//         depths in one workgroup with a barrier between them.  Schedule 0 runs every depth in one
//         launch: groups take windows depth by depth from per-depth tickets,
//         wait until the depth below has counted all its windows done, and
//         read and write output bytes with agent-scope (sc1) accesses.
//
// Copy engine: a lane's pending segment (literal run or match piece) is cut
// into 16-byte chunks [16q, 16q + 16), the last one moved back to end at the
// segment end, so every chunk of a segment of 16 bytes or more is one
// unaligned 16-byte load and store inside the segment; shorter segments are
// written with two overlapping power-of-two stores.  Chunks are dealt over the
// group's lanes (`unroll` per lane per step, all loads of a step in flight
// before the first store).  A match whose source overlaps its own output
// (period d = dst - src < length) runs as pieces d, 2d, 4d, ... each reading
// the already final prefix.
//
// Mode 2 executes pre-decoded tokens whose match sources are in a separate
// buffer (the pure-copy control of Sec. 3.3).
//
// Work items are taken in workgroup order, or (mapping 1) so that the
// workgroups one XCD receives -- the hardware deals them to the 8 XCDs in
// turn -- take one contiguous run of items.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lz_internal.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Output, literal and source bytes are addressed as integers; these casts put
// the accesses in the global address space (global_load/global_store, not flat
// instructions, which also count against the LDS wait counter).
#define LZ_G __attribute__((address_space(1)))
typedef unsigned int u32x4_a1 __attribute__((ext_vector_type(4), aligned(1)));
template <typename T>
__device__ __forceinline__ LZ_G T* gptr(uintptr_t a) { return (LZ_G T*)a; }
template <typename T>
__device__ __forceinline__ T gld(const T* p, uint64_t i) { return *(const LZ_G T*)(p + i); }
template <typename T>
__device__ __forceinline__ void gst(T* p, uint64_t i, T v) { *(LZ_G T*)(p + i) = v; }

namespace {

constexpr int kModeFlow = 0;    // every level in one launch, per-level completion counters
constexpr int kModeLevels = 1;  // the windows of one level, no waits
constexpr int kModePure = 2;    // pre-decoded tokens, sources in a reference buffer
constexpr int kModeParse = 3;   // parse blocks, copy literals, fill the match table
constexpr int kModeTail = 4;    // the last, small levels in one workgroup, a barrier between levels
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kSegTok = 128;    // tokens per parse segment
constexpr uint32_t kWinBytes = 3072;  // a match window holds at most this many bytes ...
constexpr uint32_t kWinMatches = 64;  // ... and at most this many matches
constexpr uint32_t kLog2Grain = 20;  // and its matches lie in one aligned grain of max(2^20, block) bytes
constexpr uint64_t kClosureMin = 256ull << 10;  // range closures of up to max(256 KiB, prefix / 4096) bytes;
constexpr uint64_t kClosureRatio = 4096;      // beyond that the prefix is decoded instead
constexpr uint64_t kGatherPiece = 8ull << 10;  // ranges are gathered into the output in pieces of this size,
                                               // one piece per group

constexpr uint64_t kIdleTicks = 500000000ull;  // 5 s of the 100 MHz clock without progress
constexpr int kWG = 256;
constexpr int kWGTail = 1024;           // one workgroup: 16 waves, a group (G = 64) per wave
constexpr uint32_t kTailWindows = 32;   // default: levels of at most this many windows form the tail
constexpr uint32_t kTailOff = 0xFFFFFFFFu;  // no tail launch

// One archive and its output, as the kernels see it.
struct ArcDesc {
  const uint64_t* tab;  // block table
  const uint8_t* cmd;
  const uint16_t* x16;
  const uint32_t* x32;
  const uint32_t* slo;
  const uint8_t* shi;
  const uint8_t* lit;
  uintptr_t lit_lo, lit_hi;  // readable bounds for literal windows
  uint64_t n;
  uint32_t log2_bs, nb, min_match;
  uint32_t n_fused;  // match-table slots below this are copied by the parse from the literal stream
  uint8_t* out;
  const uint8_t* msrc;  // base that match sources index (out, or ref in mode 2)
  uintptr_t msrc_lo, msrc_hi;
  const uint32_t* slot;  // per token: match-table index, or kNone
  u32x4* mtab;           // per match: {dst lo, length, src lo, dst hi | src hi << 16}
  uint64_t out_lo;       // lowest output position a match may read or write (range plans)
};

struct KArgs {
  ArcDesc one;          // the archive of a single decode
  const ArcDesc* arcs;  // batch: archive descriptors (null = single)
  // parse segments: per segment {t_start, t_end, blk_t_end, pos, lit, x16, x32, archive << 32 | blk}
  const uint64_t* seg;
  uint64_t nseg;
  // Match windows, depth-major: {first slot, count | archive << 8, bytes of the
  // first match to skip, end byte of the last match (0 = its length)}
  const u32x4* items;
  const uint32_t* lvl_start;  // per depth: first window; n_levels + 1 entries
  const uint32_t* lvl_hi;     // per depth: end of its windows to run (null = all of them)
  uint32_t* tickets;          // per level: windows taken (schedule 0)
  uint32_t* wdone;            // per level: windows finished (schedule 0)
  uint32_t* err;
  uint32_t n_levels;
  uint64_t lo, hi;  // schedule 1: window range; mode 2: token range (implicit items)
  // mode 2 (pre-decoded tokens)
  const uint64_t* p_dst;
  const uint64_t* p_lit_off;
  const uint32_t* p_lit_len;
  const uint64_t* p_src;
  const uint32_t* p_mlen;
  const uint64_t* p_unit;  // token ranges of the work items; null = windows of G tokens over [lo, hi)
  uint64_t nunits;
  uint32_t per_item;  // mode 2 without p_unit: tokens per work item (0 = G)
  uint32_t xcd_map;  // 1: the workgroups of one XCD take one contiguous run of work items
};

struct Desc {
  uintptr_t a_dst, a_src, b_dst, b_src;
  uint32_t a_len, b_len, base, ca;
};

// U chunks of one lane: loaded window, destination chunk, byte range
template <int U>
struct ChunkSet {
  u32x4 v[U];
  uintptr_t dst[U], win[U];
  int len[U], sh[U];  // bytes stored (16, 1..15, or 0), first byte of them in v
  bool slow[U], from_out[U];
};

template <int G>
__device__ __forceinline__ uint64_t gscan64(uint64_t v, int gl, uint64_t& total) {
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    uint64_t y = __shfl_up(x, d, G);
    if (gl >= d) x += y;
  }
  if constexpr (G == 64) {
    total = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(x >> 32), 63) << 32) |
            __builtin_amdgcn_readlane((uint32_t)x, 63);
  } else {
    total = __shfl(x, G - 1, G);
  }
  return x - v;
}

template <int G>
__device__ __forceinline__ uint32_t gscan32(uint32_t v, int gl, uint32_t& total) {
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    uint32_t y = __shfl_up(x, d, G);
    if (gl >= d) x += y;
  }
  if constexpr (G == 64) total = __builtin_amdgcn_readlane(x, 63);
  else total = __shfl(x, G - 1, G);
  return x - v;
}

// bits of this lane's group in a wave-wide ballot
template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int gw) {
  if constexpr (G == 64) return ballot;
  else return (ballot >> (gw * G)) & ((1ull << G) - 1);
}

// Group-uniform values.  With G = 64 a group is a whole wave, so these live in
// scalar registers (and branches on them are scalar).
template <int G>
__device__ __forceinline__ uint64_t uni(uint64_t x) {
  if constexpr (G == 64) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
  } else {
    return x;
  }
}

template <int G>
__device__ __forceinline__ uint32_t uni32(uint32_t x) {
  if constexpr (G == 64) return __builtin_amdgcn_readfirstlane(x);
  else return x;
}

// 16-byte chunks of a segment: chunk q covers [16q, 16q + 16), the last one is
// moved back to end at the segment's end (it rewrites bytes of the chunk before
// it with the same values); a segment below 16 bytes is one short chunk.
__device__ __forceinline__ uint32_t nchunks(uint32_t len) { return (len + 15u) >> 4; }

// Read target of the lanes whose window is read byte by byte: every lane
// issues its 16-byte load unconditionally, so the loads of a step stay in
// flight together.
__device__ __align__(16) uint8_t g_pad16[16];

// Bytes [lo, hi) of the 16-byte window at w, one byte at a time (windows that
// reach outside the readable range; the other bytes are zero).
__device__ __forceinline__ u32x4 load_bytes(uintptr_t w, int lo, int hi) {
  uint32_t d[4] = {0u, 0u, 0u, 0u};
  for (int i = lo; i < hi; ++i) d[i >> 2] |= uint32_t(*gptr<const uint8_t>(w + i)) << (8 * (i & 3));
  return u32x4{d[0], d[1], d[2], d[3]};
}

typedef unsigned long long u64_a1 __attribute__((aligned(1)));
typedef unsigned int u32_a1 __attribute__((aligned(1)));
typedef unsigned short u16_a1 __attribute__((aligned(1)));

// 8 bytes of v starting at byte o (0..15); bytes past the 16th read as zero
__device__ __forceinline__ uint64_t bytes_at(const u32x4& v, int o) {
  const int dw = o >> 2, b = o & 3;
  const uint32_t a0 = dw == 0 ? v.x : dw == 1 ? v.y : dw == 2 ? v.z : v.w;
  const uint32_t a1 = dw == 0 ? v.y : dw == 1 ? v.z : dw == 2 ? v.w : 0u;
  const uint32_t a2 = dw == 0 ? v.z : dw == 1 ? v.w : 0u;
  const uint32_t lo = __builtin_amdgcn_alignbyte(a1, a0, b);
  const uint32_t hi = __builtin_amdgcn_alignbyte(a2, a1, b);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// A segment of len < 16 bytes whose bytes are v[sh, sh + len): two stores of
// the largest power-of-two width w <= len, at its start and ending at its end.
template <typename ST8, typename ST4, typename ST2, typename ST1>
__device__ __forceinline__ void store_short(const u32x4& v, int sh, int len, ST8 st8, ST4 st4, ST2 st2, ST1 st1) {
  const int w = len >= 8 ? 8 : len >= 4 ? 4 : len >= 2 ? 2 : 1;
  const uint64_t first = bytes_at(v, sh), last = bytes_at(v, sh + len - w);
  if (w == 8) {
    st8(0, first);
    st8(len - 8, last);
  } else if (w == 4) {
    st4(0, (uint32_t)first);
    st4(len - 4, (uint32_t)last);
  } else if (w == 2) {
    st2(0, (uint16_t)first);
    st2(len - 2, (uint16_t)last);
  } else {
    st1(0, (uint8_t)first);
  }
}

__device__ __forceinline__ void store_seg(uintptr_t a, const u32x4& v, int sh, int len) {
  if (len == 16) {
    *gptr<u32x4_a1>(a) = v;
    return;
  }
  store_short(
      v, sh, len, [&](int o, uint64_t x) { *gptr<u64_a1>(a + o) = x; },
      [&](int o, uint32_t x) { *gptr<u32_a1>(a + o) = x; }, [&](int o, uint16_t x) { *gptr<u16_a1>(a + o) = x; },
      [&](int o, uint8_t x) { *gptr<uint8_t>(a + o) = x; });
}

// ---- coherent output path (schedule 0) -------------------------------------
// Output bytes are read and written with agent-scope (sc1) buffer accesses: a
// store is written through to the device-coherent level and a load is served
// from it, so bytes published by a group on one XCD are read correctly by a
// group on another without L2 write-back or invalidation.  Offsets are 32-bit
// (outputs below 4 GiB); the buffer's size also bounds every access.
constexpr int kSC1 = 16;  // cache-policy bit of buffer intrinsics: sc1

__device__ __forceinline__ u32x4 coh_load_bytes(__amdgpu_buffer_rsrc_t r, uint32_t w, int lo, int hi) {
  uint32_t d[4] = {0u, 0u, 0u, 0u};
  for (int i = lo; i < hi; ++i)
    d[i >> 2] |= uint32_t(__builtin_amdgcn_raw_buffer_load_b8(r, (int)(w + i), 0, kSC1)) << (8 * (i & 3));
  return u32x4{d[0], d[1], d[2], d[3]};
}

__device__ __forceinline__ void coh_store_seg(__amdgpu_buffer_rsrc_t r, uint32_t a, const u32x4& v, int sh, int len) {
  if (len == 16) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)a, 0, kSC1);
    return;
  }
  store_short(
      v, sh, len,
      [&](int o, uint64_t x) {
        __builtin_amdgcn_raw_buffer_store_b64(u32x2{(uint32_t)x, (uint32_t)(x >> 32)}, r, (int)(a + o), 0, kSC1);
      },
      [&](int o, uint32_t x) { __builtin_amdgcn_raw_buffer_store_b32(x, r, (int)(a + o), 0, kSC1); },
      [&](int o, uint16_t x) { __builtin_amdgcn_raw_buffer_store_b16(x, r, (int)(a + o), 0, kSC1); },
      [&](int o, uint8_t x) { __builtin_amdgcn_raw_buffer_store_b8(x, r, (int)(a + o), 0, kSC1); });
}

__device__ __forceinline__ void compiler_barrier() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ void mem_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

// v with its bytes moved up by s (0..15) positions (v's byte b lands at b + s)
__device__ __forceinline__ void shift_up(uint64_t lo, uint64_t hi, uint32_t s, uint64_t& rlo, uint64_t& rhi) {
  const uint32_t b = 8u * (s & 7u);
  const uint64_t carry = b ? (lo >> (64u - b)) : 0ull;
  const uint64_t l1 = lo << b, h1 = (hi << b) | carry;
  rlo = (s >= 8u) ? 0ull : l1;
  rhi = (s >= 8u) ? l1 : h1;
}

// Literal bytes of G tokens written as the aligned 16-byte blocks of their
// output span [sp0, sp1).  Every byte of the span is a literal of some run or
// a match byte; match bytes receive arbitrary values here and are rewritten by
// the match passes, so the literal stores are whole aligned blocks (only the two
// end blocks, shared with neighbouring spans, are written byte-exact).
// The literals of the G runs are consecutive in the literal stream, so one
// 16-byte load covers a block: run j's bytes sit at their block position minus
// the match bytes between the block's first run and run j.
// Blocks per lane and pass of the span copy (the U loads of a lane are in
// flight together; measured best at 3 on gfx950 for FASTQ-like literals:
// 2 and 4 are 5 % slower, the latter at occupancy 4).
constexpr int kSpanUnroll = 3;

template <int G, int U>
__device__ __forceinline__ void parse_span(uint64_t sp0, uint64_t sp1, uint64_t l_dst, uint32_t l_len, uintptr_t l_src,
                                           uintptr_t lit_lo, uintptr_t lit_hi, uintptr_t out_b, int gl, int gslot,
                                           uint32_t* s_base, Desc* s_desc) {
  // blocks are aligned in the address space; A0 is the first block's address
  const uintptr_t ab0 = out_b + sp0, ab1 = out_b + sp1;
  const uintptr_t A0 = ab0 & ~(uintptr_t)15;
  const uint32_t C = (uint32_t)(((ab1 + 15u) >> 4) - (ab0 >> 4));
  const uint32_t e0 = (uint32_t)(ab0 - A0), e1 = (uint32_t)(ab1 - A0);  // span, relative to A0
  // run starts relative to A0 (nondecreasing over the group's lanes), lengths,
  // and the literal address of each run's first byte
  s_base[gslot + gl] = (uint32_t)(out_b + l_dst - A0);
  s_desc[gslot + gl].a_len = l_len;
  s_desc[gslot + gl].a_src = l_src;
  compiler_barrier();
  constexpr uint32_t kAny = 1u << 8, kSlow = 1u << 9;
  // The U blocks of a lane advance together, so their LDS reads overlap.
  // Blocks r..r + G * U: per block its first literal run (| kAny, kSlow), and its window loaded.
  auto issue = [&](uint32_t r, uint32_t (&f)[U], u32x4 (&v)[U]) {
    if (r >= C) return;
    uint32_t A[U], k[U], bk[U], lk[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      A[i] = 16u * (r + i * G + gl);
      k[i] = 0;
    }
    // the last run starting at or before the block (run 0 when none does)
#pragma unroll
    for (int step = G / 2; step >= 1; step >>= 1) {
#pragma unroll
      for (int i = 0; i < U; ++i)
        if (s_base[gslot + k[i] + step] <= A[i]) k[i] += step;
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      bk[i] = s_base[gslot + k[i]];
      lk[i] = s_desc[gslot + k[i]].a_len;
    }
    // the block's first literal byte: in run k, or a later run starting inside the block
#pragma unroll
    for (int i = 0; i < U; ++i) {
      while ((lk[i] == 0 || bk[i] + lk[i] <= A[i]) && k[i] + 1 < (uint32_t)G) {
        const uint32_t bn = s_base[gslot + k[i] + 1];
        if (bn >= A[i] + 16u) break;
        ++k[i];
        bk[i] = bn;
        lk[i] = s_desc[gslot + k[i]].a_len;
      }
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const bool any = (r + i * G + gl < C) && lk[i] > 0 && bk[i] < A[i] + 16u && bk[i] + lk[i] > A[i];
      const uintptr_t W = s_desc[gslot + k[i]].a_src + (uintptr_t)((int64_t)A[i] - (int64_t)bk[i]);
      const bool slow = any && (W < lit_lo || W + 16u > lit_hi);
      f[i] = k[i] | (any ? kAny : 0u) | (slow ? kSlow : 0u);
      // lanes without a window read the first 16 bytes of the readable range
      v[i] = *gptr<const u32x4_a1>((any && !slow) ? W : lit_lo);
    }
  };
  auto finish = [&](uint32_t r, const uint32_t (&f)[U], u32x4 (&v)[U]) {
    if (r >= C) return;
    uint32_t bk[U], bn[U];
    uintptr_t sk[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
      const uint32_t k0 = f[i] & 0xFFu;
      bk[i] = s_base[gslot + k0];
      sk[i] = s_desc[gslot + k0].a_src;
      bn[i] = (k0 + 1 < (uint32_t)G) ? s_base[gslot + k0 + 1] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int i = 0; i < U; ++i) {
      if (r + i * G + gl >= C) continue;
      const uint32_t A = 16u * (r + i * G + gl);
      const uint32_t k0 = f[i] & 0xFFu;
      if (f[i] & kSlow) {
        const uintptr_t W = sk[i] + (uintptr_t)((int64_t)A - (int64_t)bk[i]);
        const int lo = W < lit_lo ? (int)(lit_lo - W) : 0;
        const int hi = W + 16u > lit_hi ? (int)(lit_hi - W) : 16;
        v[i] = load_bytes(W, lo, hi);
      }
      uint64_t lo = (uint64_t)v[i].x | ((uint64_t)v[i].y << 32), hi = (uint64_t)v[i].z | ((uint64_t)v[i].w << 32);
      if ((f[i] & kAny) && bn[i] < A + 16u) {
        // later runs starting inside the block: their bytes from v, moved up
        const uint64_t vlo = lo, vhi = hi;
        for (uint32_t j = k0 + 1; j < (uint32_t)G && s_base[gslot + j] < A + 16u; ++j) {
          const uint32_t bj = s_base[gslot + j];
          if (s_desc[gslot + j].a_len == 0) continue;
          const uint32_t st = bj - A;                                                    // first block byte of run j
          const uint32_t sh = (bj - bk[i]) - (uint32_t)(s_desc[gslot + j].a_src - sk[i]);  // match bytes skipped
          uint64_t rlo, rhi;
          shift_up(vlo, vhi, sh, rlo, rhi);
          const uint64_t mlo = st >= 8u ? 0ull : (~0ull << (8u * st));
          const uint64_t mhi = st >= 8u ? (~0ull << (8u * (st - 8u))) : ~0ull;
          lo = (lo & ~mlo) | (rlo & mlo);
          hi = (hi & ~mhi) | (rhi & mhi);
        }
      }
      const u32x4 o = u32x4{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
      // bytes of the span in this block
      const uint32_t b0 = e0 > A ? e0 - A : 0u;
      const uint32_t b1 = min(16u, e1 - A);
      const uintptr_t a = A0 + A;
      if (b1 - b0 == 16u)
        *gptr<u32x4>(a) = o;  // a is 16-byte aligned
      else
        store_seg(a + b0, o, (int)b0, (int)(b1 - b0));
    }
  };
  uint32_t f[U];
  u32x4 v[U];
  for (uint32_t r = 0; r < C; r += G * U) {
    issue(r, f, v);
    finish(r, f, v);
  }
  compiler_barrier();
}

template <int G, int U, int MODE, bool BATCH>
__global__ __launch_bounds__(MODE == kModeTail ? kWGTail : kWG) void k_lz(KArgs A) {
  static_assert(G == 8 || G == 16 || G == 32 || G == 64, "G");
  static_assert(MODE != kModeTail || G == 64, "a tail group is a whole wave (barriers are per wave)");
  constexpr int WG = (MODE == kModeTail) ? kWGTail : kWG;
  if (blockDim.x != (unsigned)WG) {  // the group layout assumes WG threads
    if (threadIdx.x == 0) atomicOr(A.err, 2u);
    return;
  }
  // schedule 0 reads and writes output bytes at device scope
  constexpr bool kCoh = (MODE == kModeFlow);
  constexpr bool kOnlyMatch = (MODE == kModeFlow || MODE == kModeLevels || MODE == kModeTail);
  __shared__ Desc s_desc[WG];
  __shared__ uint32_t s_base[WG];

  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);       // lane in group
  const int gw = lane / G;             // group in wave
  const int gslot = threadIdx.x - gl;  // first LDS slot of this group
  const uint64_t ngroups = (uint64_t)gridDim.x * (WG / G);
  // Workgroup b runs on XCD b mod 8.  XCD-contiguous mapping: XCD x takes
  // the x-th of 8 contiguous runs of logical workgroups (sizes differing by
  // at most one), in the order it receives them.
  uint64_t wg = blockIdx.x;
  if (A.xcd_map) {
    const uint64_t nb = gridDim.x, x = wg & 7u, q = nb >> 3, r = nb & 7u;
    wg = x * q + min(x, r) + (wg >> 3);
  }
  const uint64_t gid = uni<G>(wg * (WG / G) + threadIdx.x / G);
  ArcDesc D = A.one;
  uint64_t bs = 1ull << D.log2_bs;
  uintptr_t out_b = (uintptr_t)D.out;
  uint32_t out_cap32 = (uint32_t)min<uint64_t>(D.msrc_hi - D.msrc_lo, 0xFFFFFFFFull);
  __amdgpu_buffer_rsrc_t out_r = __builtin_amdgcn_make_buffer_rsrc((void*)D.out, 0, (int)out_cap32, 0x00020000);
  // switches the group to archive `aid` of a batch
  auto use_arc = [&](uint32_t aid) {
    if constexpr (!BATCH) return;
    D = A.arcs[uni32<G>(aid)];
    bs = 1ull << D.log2_bs;
    out_b = (uintptr_t)D.out;
    out_cap32 = (uint32_t)min<uint64_t>(D.msrc_hi - D.msrc_lo, 0xFFFFFFFFull);
    out_r = __builtin_amdgcn_make_buffer_rsrc((void*)D.out, 0, (int)out_cap32, 0x00020000);
  };
  // windows of a level (schedule 0)
  // a window holds up to 64 matches; a group of G lanes takes 64 / G parts of it
  constexpr uint32_t kParts = 64 / G;
  auto level_windows = [&](uint32_t p) -> uint32_t {
    return ((A.lvl_hi ? A.lvl_hi[p] : A.lvl_start[p + 1]) - A.lvl_start[p]) * kParts;
  };

  // work item state (replicated on the group's lanes)
  bool finished = false, have_item = false, started = true;
  uint64_t iter = 0;
  uint32_t lvl = 0, cur_lvl = (MODE == kModeTail) ? (uint32_t)A.lo : 0u, ready = 0;  // schedule 0: levels <= ready may start
  if (MODE == kModeParse) {
    for (uint64_t i = (uint64_t)blockIdx.x * kWG + threadIdx.x; i < A.n_levels; i += (uint64_t)gridDim.x * kWG) {
      A.tickets[i] = 0u;
      A.wdone[i] = 0u;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *A.err = 0u;
  }
  uint64_t t_next = 0, t_end = 0, blk_t_end = 0, pos = 0, bend = 0, litc = 0, xc = 0, yc = 0;
  uint64_t sp0 = 0, sp1 = 0;  // parse: output span of the current G tokens
  bool span_mode = false;     // parse: the span is written whole (dense literals)
  bool span_drain = false;    // parse: a span write precedes this pass's match stores
  u32x4 f_rec = u32x4{0u, 0u, 0u, 0u};  // parse: record of this lane's literal-sourced match
  // this lane's buffered token
  uint64_t l_dst = 0, l_src = 0, m_dst = 0, m_src = 0;
  uint32_t l_len = 0, m_len = 0, m_done = 0;
  bool l_pend = false;
  uint32_t idle = 0;
  uint64_t t_last = 0;
  // a window: explicit record, or the w-th run of G slots from `base`
  uint32_t w_skip = 0, w_take = 0;  // the window's first-match skip and last-match end
  uint64_t t_first = 0, t_win_end = 0;
  // part k of the window list starting at window `base`
  auto set_window = [&](uint64_t base, uint64_t k) {
    const u32x4 e = gld(A.items, base + k / kParts);
    use_arc(e.y >> 8);
    t_first = uni<G>(e.x);
    t_win_end = uni<G>((uint64_t)e.x + (e.y & 0xFFu));
    t_next = min(t_first + (k % kParts) * G, t_win_end);
    t_end = min(t_next + G, t_win_end);
    w_skip = uni32<G>(e.z);
    w_take = uni32<G>(e.w);
  };

  for (;;) {
    // ---------------------------------------------------- take a work item
    if (!finished && !have_item) {
      if (MODE == kModeFlow) {
        // windows are taken level by level, so every window waited on was taken earlier
        for (;;) {
          if (cur_lvl >= A.n_levels) {
            finished = true;
            break;
          }
          uint32_t w = 0;
          if (gl == 0) w = atomicAdd(A.tickets + cur_lvl, 1u);
          w = (G == 64) ? __builtin_amdgcn_readfirstlane(w) : __shfl(w, 0, G);
          if (w < level_windows(cur_lvl)) {
            lvl = cur_lvl;
            set_window(A.lvl_start[lvl], w);
            have_item = true;
            started = lvl <= ready;
            break;
          }
          ++cur_lvl;
        }
      } else if (MODE == kModeTail) {
        // one workgroup shares each level's windows; a barrier closes the level
        for (;;) {
          if (cur_lvl >= A.hi) {
            finished = true;
            break;
          }
          const uint64_t k = gid + iter * ngroups;
          if (k < level_windows(cur_lvl)) {
            ++iter;
            lvl = cur_lvl;
            set_window(A.lvl_start[lvl], k);
            have_item = true;
            break;
          }
          // every store of this wave has completed before the barrier (the
          // barrier itself does not wait for them)
          compiler_barrier();
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          ++cur_lvl;
          iter = 0;
        }
      } else if (MODE == kModeLevels) {
        const uint64_t k = gid + iter * ngroups;
        ++iter;
        if (k >= (A.hi - A.lo) * kParts) {
          finished = true;
        } else {
          set_window(A.lo, k);
          have_item = true;
        }
      } else if (MODE == kModePure) {
        const uint64_t k = gid + iter * ngroups;
        ++iter;
        const uint64_t per = A.per_item ? A.per_item : G;
        const uint64_t cnt = A.p_unit ? A.nunits : (A.hi - A.lo + per - 1) / per;
        if (k >= cnt) {
          finished = true;
        } else {
          if (A.p_unit) {
            t_next = A.p_unit[k];
            t_end = A.p_unit[k + 1];
          } else {
            t_next = A.lo + k * per;
            t_end = min(t_next + per, A.hi);
          }
          have_item = true;
        }
      } else {
        const uint64_t k = gid + iter * ngroups;
        ++iter;
        if (k >= A.nseg) {
          finished = true;
        } else {
          const uint64_t* e = A.seg + 8 * k;
          t_next = e[0];
          t_end = e[1];
          blk_t_end = e[2];
          pos = e[3];
          litc = e[4];
          xc = e[5];
          yc = e[6];
          use_arc((uint32_t)(e[7] >> 32));
          const uint64_t blk = e[7] & 0xFFFFFFFFull;
          bend = min(D.n, (blk + 1) * bs);
          have_item = true;
        }
      }
      if (have_item) {
        l_len = m_len = m_done = 0;
        l_pend = false;
      }
    }
    if (__all(finished)) break;

    bool progressed = false;
    if (have_item) {
      const uint32_t m_rem = m_len - m_done;
      const bool lane_pend = l_pend || (m_rem > 0);
      const uint64_t pend_bits = group_bits<G>(__ballot(lane_pend), gw);
      if (pend_bits == 0) {
        if (!started) {
          // ---------------------------------------------- the level below must be complete
          uint32_t c = 0;
          if (gl == 0) c = __hip_atomic_load(A.wdone + (lvl - 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          c = (G == 64) ? __builtin_amdgcn_readfirstlane(c) : __shfl(c, 0, G);
          if (c >= level_windows(lvl - 1)) {
            started = true;
            ready = lvl;
            progressed = true;
            compiler_barrier();  // output loads stay after the counter load
          }
        } else if (t_next >= t_end) {
          // ---------------------------------------------- item complete
          if (MODE == kModeFlow) {
            // every output store of this wave is acknowledged, then publish
            compiler_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            compiler_barrier();
            if (gl == 0) __hip_atomic_fetch_add(A.wdone + lvl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          have_item = false;
          progressed = true;
        } else {
          // ---------------------------------------------- next G tokens
          const uint64_t t = t_next + gl;
          const bool valid = t < t_end;
          uint32_t m_done_init = 0;
          // every lane loads (lanes past the end reread the last token), so the
          // loads of a step are issued together and waited for once
          const uint64_t tc = valid ? t : t_end - 1;
          if (MODE == kModePure) {
            const uint64_t dst = A.p_dst[tc], loff = A.p_lit_off[tc], src = A.p_src[tc];
            const uint32_t ll = A.p_lit_len[tc], ml = A.p_mlen[tc];
            l_dst = valid ? dst : 0;
            l_len = valid ? ll : 0u;
            l_src = valid ? loff : 0;
            m_len = valid ? ml : 0u;
            m_src = valid ? src : 0;
            m_dst = l_dst + l_len;
          } else if (MODE == kModeParse) {
            const uint32_t c_raw = gld(D.cmd, tc);
            const uint32_t s_lo = gld(D.slo, tc);
            const uint32_t s_hi = gld(D.shi ? D.shi : D.cmd, tc);  // without a high plane: ignored
            const uint32_t sl = gld(D.slot, tc);
            const uint64_t src = (uint64_t)s_lo | (D.shi ? (uint64_t)s_hi << 32 : 0ull);
            const uint32_t c = valid ? c_raw : 0u;
            const bool last = (t + 1 == blk_t_end);
            const uint32_t Lc = c >> 4, Mc = c & 15u;
            const uint32_t need_l = (valid && Lc == 15u) ? 1u : 0u;
            const uint32_t need_m = (valid && !last && Mc == 15u) ? 1u : 0u;
            uint32_t e_l = 0u, e_m = 0u, tot16 = 0u, tot32 = 0u;
            if (group_bits<G>(__ballot(need_l + need_m != 0u), gw) != 0) {
              // length extensions: positions from a group prefix count; a lane
              // that needs none reads at the cursor, inside the archive
              const uint64_t i16 = xc + gscan32<G>(need_l + need_m, gl, tot16);
              const uint32_t x_a = gld(D.x16, i16), x_b = gld(D.x16, i16 + need_l);
              e_l = need_l ? x_a : 0u;
              e_m = need_m ? x_b : 0u;
              const uint32_t w_l = (need_l && e_l == 0xFFFFu) ? 1u : 0u;
              const uint32_t w_m = (need_m && e_m == 0xFFFFu) ? 1u : 0u;
              if (group_bits<G>(__ballot(w_l + w_m != 0u), gw) != 0) {
                const uint64_t i32 = yc + gscan32<G>(w_l + w_m, gl, tot32);
                const uint32_t y_a = gld(D.x32, i32), y_b = gld(D.x32, i32 + w_l);
                if (w_l) e_l += y_a;
                if (w_m) e_m += y_b;
              }
            }
            const uint32_t lit_len = (Lc == 15u) ? 15u + e_l : Lc;
            uint32_t mlen = (valid && !last) ? D.min_match + ((Mc == 15u) ? 15u + e_m : Mc) : 0u;
            uint64_t lit_tot;
            const uint64_t loff = litc + gscan64<G>(lit_len, gl, lit_tot);
            uint64_t span_tot;
            const uint64_t tdst = pos + gscan64<G>((uint64_t)lit_len + mlen, gl, span_tot);
            if (valid && last) mlen = (uint32_t)(bend - (tdst + lit_len));
            xc += tot16;
            yc += tot32;
            litc += lit_tot;
            sp0 = pos;
            pos += span_tot;
            // the span ends at the block's end when it holds the block's last token
            sp1 = (min(t_next + G, t_end) == blk_t_end) ? bend : pos;
            // whole-span blocks pay when literals fill a good part of the span;
            // sparse literal runs are copied run by run
            span_mode = 4 * lit_tot >= sp1 - sp0;
            // record the match in plan order; a literal-sourced match (slot
            // below n_fused) is copied here instead, from the literal-stream
            // offset its resident record holds
            m_len = 0;
            if (valid && mlen > 0) {
              const uint64_t md = tdst + lit_len;
              if (sl < D.n_fused) {
                // its record is checked when the copy needs it, so the load
                // completes under the span write
                f_rec = gld((const u32x4*)D.mtab, sl);
                m_dst = md;
                m_len = mlen;
              } else {
                gst(D.mtab, sl, u32x4{(uint32_t)md, mlen, (uint32_t)src,
                                      (uint32_t)((md >> 32) & 0xFFFFu) | (uint32_t)((src >> 32) << 16)});
              }
            }
            l_dst = tdst;
            l_len = lit_len;
            l_src = loff;
          } else {
            // a window's matches from the match table
            const u32x4 rr = gld((const u32x4*)D.mtab, tc);
            const u32x4 r = valid ? rr : u32x4{0u, 0u, 0u, 0u};
            m_dst = (uint64_t)r.x | ((uint64_t)(r.w & 0xFFFFu) << 32);
            m_len = r.y;
            m_src = (uint64_t)r.z | ((uint64_t)(r.w >> 16) << 32);
            l_len = 0;
            if (valid && (m_src >= m_dst || m_dst + m_len > D.n || m_src < D.out_lo)) {  // not a record of this output
              m_len = 0;
              atomicOr(A.err, 4u);
            }
            // a long match is split over windows: this window's byte range of it
            if (valid && t + 1 == t_win_end && w_take) m_len = w_take;
            if (valid && t == t_first) m_done_init = w_skip;
          }
          const uint64_t cnt = min((uint64_t)G, t_end - t_next);
          t_next += cnt;
          m_done = m_done_init;
          l_pend = (MODE == kModeParse && span_mode) ? (sp1 > sp0) : (l_len > 0);
          progressed = true;
        }
      } else if (MODE == kModeParse && span_mode && group_bits<G>(__ballot(l_pend), gw) != 0) {
        // ------------------------------------------------ the span's aligned 16-byte blocks
        parse_span<G, kSpanUnroll>(sp0, sp1, l_dst, l_len, (uintptr_t)D.lit + l_src, D.lit_lo, D.lit_hi, out_b, gl, gslot,
                         s_base, s_desc);
        l_pend = false;
        // literal-sourced matches then rewrite their bytes of that span: the
        // copy's first stores wait until the span's stores have completed
        span_drain = group_bits<G>(__ballot(m_rem > 0), gw) != 0;
        progressed = true;
      } else {
        // ------------------------------------------------ one pass over every pending segment
        // Matches of one level never read each other's output, so every lane
        // copies at once; a self-overlapping match (period d < length) writes
        // pieces d, 2d, 4d, ... each read from the already final prefix.
        // (the parse's matches read the literal stream at their record's
        // offset and are copied whole)
        if (MODE == kModeParse && m_rem) {
          m_src = (uint64_t)f_rec.z | ((uint64_t)(f_rec.w >> 16) << 32);
          if (f_rec.x != (uint32_t)m_dst || f_rec.y != m_len ||
              (f_rec.w & 0xFFFFu) != (uint32_t)((m_dst >> 32) & 0xFFFFu) ||
              (uintptr_t)D.lit + m_src + m_len > D.lit_hi) {
            m_len = m_done;  // not this archive's record: skipped
            atomicOr(A.err, 4u);
          }
        }
        const uint32_t piece = (MODE == kModeParse) ? m_len - m_done
                               : m_rem ? (uint32_t)min<uint64_t>(m_rem, (m_dst - m_src) + m_done) : 0u;
        const bool inc_l = l_pend;
        const bool inc_m = piece > 0;
        const uintptr_t a_dst = out_b + l_dst;
        const uintptr_t b_dst = out_b + m_dst + m_done;
        const uint32_t ca = inc_l ? nchunks(l_len) : 0u;
        const uint32_t cb = inc_m ? nchunks(piece) : 0u;
        uint32_t C;
        const uint32_t base = gscan32<G>(ca + cb, gl, C);
        Desc d;
        d.a_dst = a_dst;
        d.a_src = (uintptr_t)D.lit + l_src;
        d.a_len = inc_l ? l_len : 0u;
        d.b_dst = b_dst;
        // a periodic match copies each piece from the start of its period; any
        // other match (or the part of it this window starts at) from src + done
        d.b_src = (MODE == kModeParse) ? (uintptr_t)D.lit + m_src + m_done
                                       : (uintptr_t)D.msrc + m_src + ((m_dst - m_src < m_len) ? 0u : m_done);
        d.b_len = inc_m ? piece : 0u;
        d.base = base;
        d.ca = ca;
        // a group lives in one wave, whose LDS accesses complete in order
        s_desc[threadIdx.x] = d;
        s_base[threadIdx.x] = base;
        compiler_barrier();
        // Chunks are taken G * U at a time: all U loads of a lane are in
        // flight before its first store.
        auto prep = [&](uint32_t r, ChunkSet<U>& cs) {
          // owner of chunk k: the last lane whose first chunk is <= k
          uint32_t own[U];
#pragma unroll
          for (int i = 0; i < U; ++i) own[i] = 0;
#pragma unroll
          for (int step = G / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (int i = 0; i < U; ++i)
              if (s_base[gslot + own[i] + step] <= r + i * G + gl) own[i] += step;
          }
#pragma unroll
          for (int i = 0; i < U; ++i) {
            const uint32_t k = r + i * G + gl;
            const Desc& e = s_desc[gslot + own[i]];
            const uint32_t q = k - e.base;
            // match passes copy matches only; the parse's match segments read
            // the literal stream
            const bool m = kOnlyMatch ? true : (q >= e.ca);
            const bool m_out = m && MODE != kModeParse;
            const uintptr_t Dd = m ? e.b_dst : e.a_dst;
            const uintptr_t S = m ? e.b_src : e.a_src;
            const uint32_t L = m ? e.b_len : e.a_len;
            const uint32_t qq = m ? q - e.ca : q;
            const bool valid = k < C;
            const uintptr_t lb = m_out ? D.msrc_lo : D.lit_lo, hb = m_out ? D.msrc_hi : D.lit_hi;
            cs.from_out[i] = m_out;
            cs.slow[i] = false;
            cs.sh[i] = 0;
            if (L >= 16) {
              // full chunk (windows of a segment of 16 bytes or more stay inside it)
              const uint32_t off = min(16u * qq, L - 16u);
              cs.dst[i] = Dd + off;
              cs.win[i] = S + off;
              cs.len[i] = valid ? 16 : 0;
            } else {
              // short segment: the window starts at its source, or ends at its
              // end near the top of the readable range.  An empty segment (a
              // lane past the group's last chunk whose owner has nothing to
              // copy) never touches its source, which need not be an address
              // inside the buffer (range plans place the output base below it).
              cs.dst[i] = Dd;
              cs.len[i] = valid ? (int)L : 0;
              if (L == 0) {
                cs.win[i] = S;
                cs.slow[i] = true;
              } else if (S + 16 <= hb) {
                cs.win[i] = S;
              } else if (S + L >= lb + 16) {
                cs.win[i] = S + L - 16;
                cs.sh[i] = 16 - (int)L;
              } else {
                cs.win[i] = S;
                cs.slow[i] = true;
              }
            }
          }
          // every lane loads (a buffer load out of range returns zeros)
#pragma unroll
          for (int i = 0; i < U; ++i) {
            if (kCoh && cs.from_out[i])
              cs.v[i] = __builtin_amdgcn_raw_buffer_load_b128(
                  out_r, cs.slow[i] ? 0 : (int)(uint32_t)(cs.win[i] - out_b), 0, kSC1);
            else
              cs.v[i] = *gptr<const u32x4_a1>(cs.slow[i] ? (uintptr_t)g_pad16 : cs.win[i]);
          }
        };
        auto commit = [&](ChunkSet<U>& cs) {
#pragma unroll
          for (int i = 0; i < U; ++i)
            if (cs.slow[i] && cs.len[i] > 0) {
              if (kCoh && cs.from_out[i])
                cs.v[i] = coh_load_bytes(out_r, (uint32_t)(cs.win[i] - out_b), 0, cs.len[i]);
              else
                cs.v[i] = load_bytes(cs.win[i], 0, cs.len[i]);
            }
#pragma unroll
          for (int i = 0; i < U; ++i)
            if (cs.len[i] > 0) {
              if (kCoh)
                coh_store_seg(out_r, (uint32_t)(cs.dst[i] - out_b), cs.v[i], cs.sh[i], cs.len[i]);
              else
                store_seg(cs.dst[i], cs.v[i], cs.sh[i], cs.len[i]);
            }
        };
        for (uint32_t r = 0; r < C; r += G * U) {
          ChunkSet<U> cs;
          prep(r, cs);
          if (MODE == kModeParse && span_drain) {
            // the span's stores (and these loads) complete before any store of this pass
            compiler_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            compiler_barrier();
            span_drain = false;
          }
          commit(cs);
        }
        span_drain = false;
        compiler_barrier();
        // ---------------------------------------------- retire segments
        if (inc_l) l_pend = false;
        if (inc_m) m_done += piece;
        // a further piece reads what this pass wrote
        if (group_bits<G>(__ballot(m_len > m_done), gw) != 0) mem_order();
        progressed = true;
      }
    }
    // -------------------------------------------------------- idle guard
    if (MODE == kModeFlow) {
      if (__any(progressed)) {
        idle = 0;
      } else {
        // a wave that waits without progress for kIdleTicks gives up
        if ((idle++ & 255u) == 0u) {
          const uint64_t now = __builtin_amdgcn_s_memrealtime();
          if (idle == 1u) t_last = now;
          if (now - t_last > kIdleTicks) {
            if (lane == 0) atomicOr(A.err, 1u);
            break;
          }
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host side

struct lz_dev {
  lz::ArcView v;  // host view of the header (base pointer not kept)
  uint8_t* d_arc = nullptr;
  uint32_t* d_ctrl = nullptr;  // [1] error flag
  uint32_t* d_slot = nullptr;
  uint32_t* d_lvls = nullptr;
  u32x4* d_win = nullptr;
  uint32_t* d_tick = nullptr;
  uint32_t* d_wdone = nullptr;
  uint64_t* d_seg = nullptr;
  uint64_t n_seg = 0;
  u32x4* d_mtab = nullptr;
  uint64_t n_match = 0;
  uint64_t n_fused = 0;  // literal-sourced matches, copied by the parse (slots [0, n_fused))
  uint64_t fused_bytes = 0;
  std::vector<uint64_t> lvl_start;  // first window of each depth, n_levels + 1 entries
  std::vector<uint64_t> h_seg;      // host copies of the parse segments and windows (batch decodes merge them)
  std::vector<uint32_t> h_win;
  std::vector<uint64_t> h_wdst;  // per window: output position of its first byte
  uint32_t log2_grain = 20;      // output grains: see Plan
  std::vector<uint64_t> grain_low;
  // coded archives: the tile-rANS container stays resident; the entropy stage
  // decodes it into the archive region (d_arc) before the match phase
  uint8_t* d_coded = nullptr;
  uint64_t coded_size = 0, coded_payload = 0, coded_tiles = 0;
  int cu_count = 0;
  // replayable launch sequences, one per (output, config)
  struct GraphKey {
    uint8_t* out;
    uint64_t cap;
    uint32_t G, U, sched, tail, stage, map, occ, pG, pU;
    bool operator==(const GraphKey& o) const {
      return out == o.out && cap == o.cap && G == o.G && U == o.U && sched == o.sched && tail == o.tail &&
             stage == o.stage && map == o.map && occ == o.occ && pG == o.pG && pU == o.pU;
    }
  };
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  // host copy of the archive and lazily parsed blocks (range planning)
  std::vector<uint8_t> host_arc;
  struct RTok {
    uint64_t dst, lit_off, src;
    uint32_t ll, ml;
  };
  std::vector<std::vector<RTok>> tok_cache;
  std::vector<uint8_t> tok_cached;
  std::mutex mu;
  // pinned staging lent to the synchronous range calls (lz_decode_range,
  // lz_seek_record) and kept across them, so a seek neither allocates nor
  // frees pinned memory (freeing it waits for the whole device); sync_mu
  // serialises those calls
  uint8_t* sync_pin = nullptr;
  uint64_t sync_pin_bytes = 0;
  std::mutex sync_mu;
  ~lz_dev() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (sync_pin) (void)hipHostFree(sync_pin);
  }
};

namespace {

struct DevLayout {
  uint64_t arc, ctrl, slot, lvls, tick, wdone, seg, win, mtab, total;
};

// Device layout for an archive; level and match counts are bounded by n_tok.
DevLayout layout(const lz::ArcView& v) {
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  const uint64_t T = v.n_tok;
  DevLayout L;
  L.arc = 0;
  L.ctrl = a256(v.total);
  L.slot = a256(L.ctrl + 256);
  L.lvls = a256(L.slot + 4 * (T + 1));
  L.tick = a256(L.lvls + 4 * (T + 2));
  L.wdone = a256(L.tick + 4 * (T + 2));
  L.seg = a256(L.wdone + 4 * (T + 2));
  L.win = a256(L.seg + 64 * (T / kSegTok + v.nb + 2));
  L.mtab = a256(L.win + 16 * (T + v.n / kWinBytes + 2));
  L.total = a256(L.mtab + 16 * (T + 1));
  return L;
}

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return lz::fail(LZ_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// fn(b) for every block b, on up to 16 host threads
template <typename F>
void parallel_blocks(const lz::ArcView& v, F fn) {
  std::vector<std::thread> pool;
  const unsigned W = std::min<unsigned>(lz::hw_threads(0), 16);
  std::atomic<uint64_t> next{0};
  for (unsigned w = 0; w < W; ++w)
    pool.emplace_back([&] {
      for (;;) {
        const uint64_t b = next.fetch_add(1);
        if (b >= v.nb) break;
        fn(b);
      }
    });
  for (auto& t : pool) t.join();
}

// Host plan: dependency depth of every match -> match-table slots ordered by
// (depth, token); parse segments with their stream cursors.
struct Plan {
  std::vector<uint32_t> slot, lvls32;
  std::vector<uint32_t> win;   // windows, 4 words each
  std::vector<uint64_t> wdst;  // per window: output position of its first match
  std::vector<uint64_t> seg;  // parse segments, 8 words each
  std::vector<uint64_t> lvl_start;
  uint64_t n_match = 0;
  // Output grains of 2^log2_grain bytes (aligned; a multiple of the block
  // size): no window holds matches of two grains, and grain_low[g] is the
  // lowest source of a match written in grain g (its start when lower ones
  // do not exist).  A range plan can start decoding at any grain start h whose
  // grains up to the range end read nothing below h.
  uint32_t log2_grain = kLog2Grain;
  std::vector<uint64_t> grain_low;
  // Literal-sourced matches: slots [0, n_fused) hold depth-1 matches whose
  // source is a stretch of one literal run and does not overlap their output.
  // The parse copies them straight from the literal stream, so they take no
  // window; fused_rec holds their records {dst lo, length, literal-stream
  // offset lo, dst hi | offset hi << 16}, resident in the match table.
  uint64_t n_fused = 0, fused_bytes = 0;
  std::vector<uint32_t> fused_rec;
};

int build_plan(const lz::ArcView& v, Plan& P) {
  const uint64_t T = v.n_tok;
  std::vector<uint32_t> depth(T + 1, 0);
  std::vector<uint8_t> hasm(T + 1, 0);
  uint32_t mx = 0;
  int rc = lz::compute_levels(v, depth.data(), &mx, hasm.data());
  if (rc) return rc;
  const uint64_t* tab = v.tab();
  // counting sort of the matches by depth (1..mx), token order inside a depth
  const uint64_t NL = mx;
  std::vector<uint64_t> cnt(NL + 2, 0);
  uint64_t M = 0;
  for (uint64_t t = 0; t < T; ++t)
    if (hasm[t]) {
      cnt[depth[t]]++;
      ++M;
    }
  P.n_match = M;
  if (M > 0xFFFFFFF0ull) return lz::fail(LZ_E_INVAL, "too many matches for 32-bit plan indices");
  // Depth-1 matches read literal bytes only.  Those whose source lies inside
  // one token's literal run, and ends before their own output starts, read
  // that run's bytes from the literal stream at a known offset (flit).
  std::vector<uint64_t> flit(T + 1, UINT64_MAX);
  if (cnt.size() > 1 && cnt[1]) {
    std::vector<uint64_t> tdst(T + 1, 0), tlit(T + 1, 0);
    std::vector<uint32_t> tll(T + 1, 0);
    std::atomic<int> bad{0};
    parallel_blocks(v, [&](uint64_t b) {
      int r = lz::walk_block(v, b, [&](uint64_t t, const lz::Tok& k) {
        tdst[t] = k.dst;
        tlit[t] = k.lit_off;
        tll[t] = (uint32_t)k.lit_len;
      });
      if (r) bad.store(r);
    });
    if (bad.load()) return lz::fail(LZ_E_CORRUPT, "archive fails validation");
    parallel_blocks(v, [&](uint64_t b) {
      (void)lz::walk_block(v, b, [&](uint64_t t, const lz::Tok& k) {
        if (!k.mlen || depth[t] != 1) return;
        const uint64_t md = k.dst + k.lit_len;
        if (k.src + k.mlen > md) return;  // reads its own output
        const uint64_t sb = k.src >> v.log2_bs;
        // the last token of the source block starting at or before the source
        const uint64_t* lo = tdst.data() + tab[4 * sb], * hi = tdst.data() + tab[4 * sb + 4];
        const uint64_t* it = std::upper_bound(lo, hi, k.src);
        if (it == lo) return;
        const uint64_t s = (uint64_t)(it - tdst.data()) - 1;
        if (k.src + k.mlen <= tdst[s] + tll[s]) flit[t] = tlit[s] + (k.src - tdst[s]);
      });
    });
  }
  uint64_t nF = 0;
  for (uint64_t t = 0; t < T; ++t)
    if (hasm[t] && flit[t] != UINT64_MAX) {
      --cnt[depth[t]];
      ++nF;
    }
  P.n_fused = nF;
  std::vector<uint64_t> sstart(NL + 1, 0);  // first slot of each depth (after the fused slots)
  sstart[0] = nF;
  for (uint64_t p = 0; p < NL; ++p) sstart[p + 1] = sstart[p] + cnt[p + 1];
  std::vector<uint64_t> cursor(sstart.begin(), sstart.end());
  P.slot.assign(T + 1, kNone);
  std::vector<uint32_t> tok_of(M + 1, 0), len_of(M + 1, 0);
  std::vector<uint64_t> dst_of(M + 1, 0);
  std::vector<uint8_t> periodic(M + 1, 0);
  std::vector<uint64_t> blk_low(v.nb, UINT64_MAX);  // lowest match source of each block
  uint64_t fc = 0;
  for (uint64_t t = 0; t < T; ++t)
    if (hasm[t]) {
      P.slot[t] = (uint32_t)(flit[t] != UINT64_MAX ? fc++ : cursor[depth[t] - 1]++);
      tok_of[P.slot[t]] = (uint32_t)t;
    }
  // lengths, and whether a match overlaps its own output
  {
    std::atomic<int> bad{0};
    parallel_blocks(v, [&](uint64_t b) {
      int r = lz::walk_block(v, b, [&](uint64_t t, const lz::Tok& k) {
        if (!k.mlen) return;
        const uint32_t sl = P.slot[t];
        len_of[sl] = (uint32_t)k.mlen;
        dst_of[sl] = k.dst + k.lit_len;
        periodic[sl] = (k.dst + k.lit_len - k.src < k.mlen) ? 1 : 0;
        blk_low[b] = std::min(blk_low[b], k.src);
      });
      if (r) bad.store(r);
    });
    if (bad.load()) return lz::fail(LZ_E_CORRUPT, "archive fails validation");
  }
  P.fused_rec.resize(4 * nF);
  for (uint64_t sl = 0; sl < nF; ++sl) {
    const uint64_t md = dst_of[sl], lo = flit[tok_of[sl]];
    uint32_t* r = &P.fused_rec[4 * sl];
    r[0] = (uint32_t)md;
    r[1] = len_of[sl];
    r[2] = (uint32_t)lo;
    r[3] = (uint32_t)((md >> 32) & 0xFFFFu) | (uint32_t)((lo >> 32) << 16);
    P.fused_bytes += len_of[sl];
  }
  P.log2_grain = std::max<uint32_t>(kLog2Grain, v.log2_bs);
  const uint32_t lg = P.log2_grain;
  const uint64_t n_grain = v.n ? ((v.n - 1) >> lg) + 1 : 0;
  P.grain_low.resize(n_grain);
  for (uint64_t g = 0; g < n_grain; ++g) P.grain_low[g] = g << lg;
  for (uint64_t b = 0; b < v.nb; ++b) {
    const uint64_t g = (b << v.log2_bs) >> lg;
    P.grain_low[g] = std::min(P.grain_low[g], blk_low[b]);
  }
  // windows of each depth: at most kWinMatches matches and kWinBytes bytes, all
  // in one grain; a longer match that does not overlap itself is split into
  // kWinBytes pieces
  P.lvl_start.assign(NL + 1, 0);
  for (uint64_t p = 0; p < NL; ++p) {
    P.lvl_start[p] = P.win.size() / 4;
    uint64_t w0 = 0, wc = 0, wb = 0;
    auto flush = [&] {
      if (!wc) return;
      const uint32_t rec[4] = {(uint32_t)w0, (uint32_t)wc, 0u, 0u};
      P.win.insert(P.win.end(), rec, rec + 4);
      P.wdst.push_back(dst_of[w0]);
      wc = wb = 0;
    };
    for (uint64_t sl = sstart[p]; sl < sstart[p + 1]; ++sl) {
      const uint32_t L = len_of[sl];
      if (!periodic[sl] && L > kWinBytes) {
        flush();
        for (uint32_t off = 0; off < L; off += kWinBytes) {
          const uint32_t rec[4] = {(uint32_t)sl, 1u, off, std::min(off + kWinBytes, L)};
          P.win.insert(P.win.end(), rec, rec + 4);
          P.wdst.push_back(dst_of[sl] + off);
        }
        continue;
      }
      if (wc && (wc == kWinMatches || wb + L > kWinBytes || (dst_of[sl] >> lg) != (dst_of[w0] >> lg))) flush();
      if (!wc) w0 = sl;
      ++wc;
      wb += L;
    }
    flush();
  }
  P.lvl_start[NL] = P.win.size() / 4;
  P.lvls32.assign(P.lvl_start.begin(), P.lvl_start.end());
  // parse segments: every kSegTok tokens of a block, with the cursors there
  {
    std::vector<std::vector<uint64_t>> per(v.nb);
    std::vector<std::thread> pool;
    unsigned W = std::min<unsigned>(lz::hw_threads(0), 16);
    std::atomic<uint64_t> next{0};
    for (unsigned w = 0; w < W; ++w)
      pool.emplace_back([&] {
        for (;;) {
          uint64_t b = next.fetch_add(1);
          if (b >= v.nb) break;
          const uint64_t t0 = tab[4 * b], t1 = tab[4 * b + 4];
          auto& o = per[b];
          (void)lz::walk_block(v, b, [&](uint64_t t, const lz::Tok& k) {
            if ((t - t0) % kSegTok == 0) {
              const uint64_t rec[8] = {t, std::min(t + kSegTok, t1), t1, k.dst, k.lit_off, k.x16_off, k.x32_off, b};
              o.insert(o.end(), rec, rec + 8);
            }
          });
        }
      });
    for (auto& t : pool) t.join();
    size_t tot = 0;
    for (auto& o : per) tot += o.size();
    P.seg.reserve(tot);
    for (auto& o : per) P.seg.insert(P.seg.end(), o.begin(), o.end());
  }
  return 0;
}

ArcDesc arc_desc(const lz_dev* h, uint8_t* out, uint64_t out_cap) {
  ArcDesc d;
  memset(&d, 0, sizeof(d));
  const lz::ArcView& v = h->v;
  d.tab = (const uint64_t*)(h->d_arc + v.off_tab);
  d.cmd = h->d_arc + v.off_cmd;
  d.x16 = (const uint16_t*)(h->d_arc + v.off_x16);
  d.x32 = (const uint32_t*)(h->d_arc + v.off_x32);
  d.slo = (const uint32_t*)(h->d_arc + v.off_slo);
  d.shi = (v.flags & 1) ? h->d_arc + v.off_shi : nullptr;
  d.lit = h->d_arc + v.off_lit;
  d.lit_lo = (uintptr_t)h->d_arc;
  d.lit_hi = (uintptr_t)h->d_arc + v.total;
  d.n = v.n;
  d.log2_bs = v.log2_bs;
  d.nb = (uint32_t)v.nb;
  d.min_match = (uint32_t)v.min_match;
  d.n_fused = (uint32_t)h->n_fused;
  d.out = out;
  d.msrc = out;
  d.msrc_lo = (uintptr_t)out;
  d.msrc_hi = (uintptr_t)out + out_cap;
  d.slot = h->d_slot;
  d.mtab = h->d_mtab;
  return d;
}

KArgs base_args(const lz_dev* h) {
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.one = arc_desc(h, nullptr, 0);
  A.lvl_start = h->d_lvls;
  A.items = h->d_win;
  A.tickets = h->d_tick;
  A.wdone = h->d_wdone;
  A.seg = h->d_seg;
  A.nseg = h->n_seg;
  A.err = h->d_ctrl + 1;
  A.n_levels = (uint32_t)(h->lvl_start.size() ? h->lvl_start.size() - 1 : 0);
  return A;
}

typedef void (*kfn_t)(KArgs);

template <int MODE>
kfn_t pick_kernel(uint32_t G, uint32_t U, bool batch = false) {
#define K(g, u) \
  if (G == g && U == u) return batch ? k_lz<g, u, MODE, true> : k_lz<g, u, MODE, false>;
  K(8, 1) K(8, 2) K(8, 4) K(16, 1) K(16, 2) K(16, 4) K(32, 1) K(32, 2) K(32, 4) K(64, 1) K(64, 2) K(64, 4)
#undef K
  return nullptr;
}

kfn_t pick_tail(uint32_t U, bool batch) {
  if (U == 1) return batch ? k_lz<64, 1, kModeTail, true> : k_lz<64, 1, kModeTail, false>;
  if (U == 2) return batch ? k_lz<64, 2, kModeTail, true> : k_lz<64, 2, kModeTail, false>;
  return batch ? k_lz<64, 4, kModeTail, true> : k_lz<64, 4, kModeTail, false>;
}

// First level of the tail: every level from there on has at most `limit`
// windows (returns n_levels when the tail would hold fewer than two levels).
uint64_t tail_start(const std::vector<uint64_t>& windows, uint32_t limit) {
  uint64_t p = windows.size();
  while (p > 0 && windows[p - 1] <= limit) --p;
  return (windows.size() - p >= 2) ? p : windows.size();
}

int resolve_cfg(const lz_decode_cfg* cfg, uint32_t& G, uint32_t& U, uint32_t& sched, uint32_t* tail = nullptr,
                uint32_t* map = nullptr, uint32_t* occ = nullptr, uint32_t* pG = nullptr, uint32_t* pU = nullptr) {
  G = cfg ? cfg->G : 64;
  U = cfg ? cfg->unroll : 2;
  sched = cfg ? cfg->schedule : 1;
  if (tail) *tail = (cfg && cfg->tail) ? cfg->tail : kTailWindows;
  if (map) *map = cfg ? cfg->mapping : 0;
  if (occ) *occ = cfg ? cfg->occupancy : 0;
  const uint32_t parse_G = (cfg && cfg->parse_G) ? cfg->parse_G : 64, parse_U = (cfg && cfg->parse_unroll) ? cfg->parse_unroll : 2;
  if (!(parse_G == 8 || parse_G == 16 || parse_G == 32 || parse_G == 64))
    return lz::fail(LZ_E_INVAL, "parse_G must be 8, 16, 32 or 64");
  if (!(parse_U == 1 || parse_U == 2 || parse_U == 4)) return lz::fail(LZ_E_INVAL, "parse_unroll must be 1, 2 or 4");
  if (pG) *pG = parse_G;
  if (pU) *pU = parse_U;
  if (cfg && cfg->mapping > 1) return lz::fail(LZ_E_INVAL, "mapping must be 0 or 1");
  if (!(G == 8 || G == 16 || G == 32 || G == 64)) return lz::fail(LZ_E_INVAL, "G must be 8, 16, 32 or 64");
  if (!(U == 1 || U == 2 || U == 4)) return lz::fail(LZ_E_INVAL, "unroll must be 1, 2 or 4");
  if (sched > 1) return lz::fail(LZ_E_INVAL, "schedule must be 0 or 1");
  return 0;
}

uint64_t resident_groups(kfn_t k, int cu_count, uint32_t G, size_t smem = 0) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, kWG, smem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return (uint64_t)per_cu * (uint64_t)std::max(cu_count, 1) * (kWG / G);
}

// Dynamic LDS that leaves room for at most `occ` workgroups of k per CU (0:
// no padding); LZ_E_INVAL if that is not a reduction the LDS can make.
int occupancy_pad(kfn_t k, uint32_t occ, size_t* pad) {
  *pad = 0;
  if (occ == 0) return 0;
  constexpr size_t kLdsPerCu = 160 * 1024, kMaxDynamic = 64 * 1024;
  hipFuncAttributes fa;
  int natural = 0;
  if (hipFuncGetAttributes(&fa, (const void*)k) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&natural, (const void*)k, kWG, 0) != hipSuccess)
    return lz::fail(LZ_E_HIP, "occupancy query failed");
  if (occ < 3 || occ > 8 || (int)occ > natural)
    return lz::fail(LZ_E_INVAL, "occupancy %u outside [3, min(8, %d)]", occ, natural);
  const size_t per = (kLdsPerCu / occ) & ~size_t(255);
  if (per <= fa.sharedSizeBytes || per - fa.sharedSizeBytes > kMaxDynamic)
    return lz::fail(LZ_E_INVAL, "occupancy %u cannot be set by LDS padding", occ);
  *pad = (int)occ == natural ? 0 : per - fa.sharedSizeBytes;
  int got = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&got, (const void*)k, kWG, *pad) != hipSuccess || got != (int)occ)
    return lz::fail(LZ_E_INVAL, "occupancy %u not reached by LDS padding (%d)", occ, got);
  return 0;
}

uint64_t grid_for(uint64_t items, uint64_t resident, uint32_t G) {
  uint64_t groups = std::max<uint64_t>(1, std::min(items, resident));
  return (groups + (kWG / G) - 1) / (kWG / G);
}

}  // namespace

extern "C" {

int lz_device_bytes(const uint8_t* arc, uint64_t arc_size, uint64_t* bytes) {
  if (!bytes) return lz::fail(LZ_E_INVAL, "null output");
  lz::ArcView v;
  int rc = lz::view_archive(arc, arc_size, &v);
  if (rc) return rc;
  *bytes = layout(v).total;
  return 0;
}

}  // extern "C"

namespace {

// Opens a validated archive whose device layout starts at d_buf; with
// upload_archive false its bytes are already in the archive region.
int open_impl(const uint8_t* arc, uint64_t arc_size, void* d_buf, uint64_t d_cap, void* stream, lz_dev** out,
              bool upload_archive) {
  lz::ArcView v;
  int rc = lz::view_archive(arc, arc_size, &v);
  if (rc) return rc;
  rc = lz::validate_archive(v, 0);
  if (rc) return rc;
  if (v.nb > 0xFFFFFFF0ull || v.n_tok > 0xFFFFFFF0ull) return lz::fail(LZ_E_INVAL, "archive too large for 32-bit plan");
  DevLayout L = layout(v);
  if (d_cap < L.total)
    return lz::fail(LZ_E_NOMEM, "device buffer %llu < %llu bytes", (unsigned long long)d_cap,
                    (unsigned long long)L.total);
  Plan P;
  try {
    rc = build_plan(v, P);
  } catch (const std::bad_alloc&) {
    return lz::fail(LZ_E_NOMEM, "plan allocation failed");
  }
  if (rc) return rc;
  lz_dev* h = new lz_dev();
  h->v = v;
  try {
    h->host_arc.assign(arc, arc + v.total);
    h->tok_cache.resize(v.nb);
    h->tok_cached.assign(v.nb, 0);
  } catch (const std::bad_alloc&) {
    delete h;
    return lz::fail(LZ_E_NOMEM, "host archive copy failed");
  }
  h->v.base = h->host_arc.data();
  uint8_t* base = (uint8_t*)d_buf;
  h->d_arc = base + L.arc;
  h->d_ctrl = (uint32_t*)(base + L.ctrl);
  h->d_slot = (uint32_t*)(base + L.slot);
  h->d_lvls = (uint32_t*)(base + L.lvls);
  h->d_win = (u32x4*)(base + L.win);
  h->d_tick = (uint32_t*)(base + L.tick);
  h->d_wdone = (uint32_t*)(base + L.wdone);
  h->d_seg = (uint64_t*)(base + L.seg);
  h->n_seg = P.seg.size() / 8;
  h->d_mtab = (u32x4*)(base + L.mtab);
  h->n_match = P.n_match;
  h->n_fused = P.n_fused;
  h->fused_bytes = P.fused_bytes;
  h->lvl_start = P.lvl_start;
  h->h_seg = P.seg;
  h->h_win = P.win;
  h->h_wdst = P.wdst;
  h->log2_grain = P.log2_grain;
  h->grain_low = P.grain_low;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete h;
    return lz::fail(LZ_E_HIP, "device query failed");
  }
  // stage the plan through pinned memory, then the archive
  struct Piece {
    void* dst;
    const void* src;
    uint64_t bytes;
  };
  const Piece pieces[] = {
      {h->d_slot, P.slot.data(), 4 * P.slot.size()},
      {h->d_lvls, P.lvls32.data(), 4 * P.lvls32.size()},
      {h->d_win, P.win.data(), 4 * P.win.size()},
      {h->d_seg, P.seg.data(), 8 * P.seg.size()},
      {h->d_mtab, P.fused_rec.data(), 4 * P.fused_rec.size()},
  };
  uint64_t stage = v.total;
  for (const Piece& q : pieces) stage += (q.bytes + 255) & ~uint64_t(255);
  uint8_t* hp = nullptr;
  if (hipHostMalloc((void**)&hp, stage, 0) != hipSuccess) {
    delete h;
    return lz::fail(LZ_E_NOMEM, "pinned staging allocation of %llu bytes failed", (unsigned long long)stage);
  }
  uint64_t off = 0;
  bool ok = true;
  for (const Piece& q : pieces) {
    if (!q.bytes) continue;
    memcpy(hp + off, q.src, q.bytes);
    ok = ok && hipMemcpyAsync(q.dst, hp + off, q.bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    off += (q.bytes + 255) & ~uint64_t(255);
  }
  if (upload_archive) {
    memcpy(hp + off, arc, v.total);
    ok = ok && hipMemcpyAsync(h->d_arc, hp + off, v.total, hipMemcpyHostToDevice, s) == hipSuccess;
  }
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  ok = (hipHostFree(hp) == hipSuccess) && ok;
  if (!ok) {
    delete h;
    return lz::fail(LZ_E_HIP, "upload failed");
  }
  *out = h;
  return 0;
}

}  // namespace

extern "C" {

int lz_device_open(const uint8_t* arc, uint64_t arc_size, void* d_buf, uint64_t d_cap, void* stream, lz_dev** out) {
  if (!out || !d_buf) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  // the buffer holds words that kernels update atomically (error flags, counters)
  if ((uintptr_t)d_buf & 255u) return lz::fail(LZ_E_INVAL, "d_buf must be 256-byte aligned");
  return open_impl(arc, arc_size, d_buf, d_cap, stream, out, true);
}

int lz_coded_device_bytes(const uint8_t* coded, uint64_t size, uint64_t* bytes) {
  if (!bytes) return lz::fail(LZ_E_INVAL, "null output");
  lz::CodedView cv;
  int rc = lz::parse_coded(coded, size, &cv);
  if (rc) return rc;
  lz::ArcView hv;
  rc = lz::view_header(coded + 64, &hv);
  if (rc) return rc;
  *bytes = ((size + 16 + 255) & ~uint64_t(255)) + layout(hv).total;
  return 0;
}

int lz_device_open_coded(const uint8_t* coded, uint64_t size, void* d_buf, uint64_t d_cap, void* stream,
                         lz_dev** out) {
  if (!out || !d_buf) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  if ((uintptr_t)d_buf & 255u) return lz::fail(LZ_E_INVAL, "d_buf must be 256-byte aligned");
  uint64_t need = 0;
  int rc = lz_coded_device_bytes(coded, size, &need);  // validates the whole coded container
  if (rc) return rc;
  if (d_cap < need)
    return lz::fail(LZ_E_NOMEM, "device buffer %llu < %llu bytes", (unsigned long long)d_cap, (unsigned long long)need);
  lz::CodedView cv;
  (void)lz::parse_coded(coded, size, &cv);
  const uint64_t creg = (size + 16 + 255) & ~uint64_t(255);
  uint8_t* d_coded = (uint8_t*)d_buf;
  uint8_t* base = d_coded + creg;
  const DevLayout L = [&] {
    lz::ArcView hv;
    (void)lz::view_header(coded + 64, &hv);
    return layout(hv);
  }();
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return lz::fail(LZ_E_HIP, "device query failed");
  // resident coded container; entropy stage into the archive region; the
  // decoded container comes back to the host for validation and planning
  uint8_t* hp = nullptr;
  const uint64_t stage = std::max<uint64_t>(size, cv.out_size) + 16;
  if (hipHostMalloc((void**)&hp, stage, 0) != hipSuccess)
    return lz::fail(LZ_E_NOMEM, "pinned staging allocation of %llu bytes failed", (unsigned long long)stage);
  uint32_t* d_err = (uint32_t*)(base + L.ctrl) + 2;
  uint32_t err = 0;
  memcpy(hp, coded, size);
  bool ok = hipMemcpyAsync(d_coded, hp, size, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemsetAsync(d_err, 0, 4, s) == hipSuccess;
  if (ok) ok = lz::entropy_launch(d_coded, cv.payload, cv.n_tiles, base + L.arc, d_err, cu, stream) == 0;
  ok = ok && hipMemcpyAsync(hp, base + L.arc, cv.out_size, hipMemcpyDeviceToHost, s) == hipSuccess &&
       hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, s) == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
  if (!ok || err) {
    (void)hipHostFree(hp);
    return ok ? lz::fail(LZ_E_CORRUPT, "entropy stage failed (err %u)", err) : lz::fail(LZ_E_HIP, "entropy stage failed");
  }
  rc = open_impl(hp, cv.out_size, base, d_cap - creg, stream, out, false);
  (void)hipHostFree(hp);
  if (rc) return rc;
  (*out)->d_coded = d_coded;
  (*out)->coded_size = size;
  (*out)->coded_payload = cv.payload;
  (*out)->coded_tiles = cv.n_tiles;
  return 0;
}

int lz_entropy_decode_device(lz_dev* h, void* stream) {
  if (!h || !h->d_coded) return lz::fail(LZ_E_INVAL, "not a coded archive handle");
  return lz::entropy_launch(h->d_coded, h->coded_payload, h->coded_tiles, h->d_arc, h->d_ctrl + 2, h->cu_count, stream);
}

uint64_t lz_device_n(const lz_dev* h) { return h ? h->v.n : 0; }
uint32_t lz_device_levels(const lz_dev* h) { return h ? (uint32_t)(h->lvl_start.size() ? h->lvl_start.size() - 1 : 0) : 0; }
uint64_t lz_device_fused(const lz_dev* h, uint64_t* bytes) {
  if (bytes) *bytes = h ? h->fused_bytes : 0;
  return h ? h->n_fused : 0;
}
void lz_device_close(lz_dev* h) { delete h; }

}  // extern "C"

namespace {

// stage 0: parse and match passes; 1: parse only; 2: match passes only
int decode_stage(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, int stage, void* stream) {
  if (!h) return lz::fail(LZ_E_INVAL, "null handle");
  if (stage < 0 || stage > 2) return lz::fail(LZ_E_INVAL, "stage must be 0, 1 or 2");
  if (out_cap < h->v.n) return lz::fail(LZ_E_INVAL, "output capacity %llu < n %llu", (unsigned long long)out_cap,
                                        (unsigned long long)h->v.n);
  if (h->v.n && !d_out) return lz::fail(LZ_E_INVAL, "null output");
  uint32_t G, U, sched, tail, map, occ, pG, pU;
  int rc = resolve_cfg(cfg, G, U, sched, &tail, &map, &occ, &pG, &pU);
  if (rc) return rc;
  if (sched == 0 && out_cap > 0xFFFFFFFFull)
    return lz::fail(LZ_E_INVAL, "schedule 0 addresses outputs below 4 GiB; use schedule 1");
  size_t pad = 0;
  if (sched == 1 && (rc = occupancy_pad(pick_kernel<kModeLevels>(G, U), occ, &pad))) return rc;
  if (h->v.nb == 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  lz_dev::GraphKey key{d_out, out_cap, G, U, sched, tail, (uint32_t)stage, map, occ, pG, pU};
  for (auto& g : h->graphs)
    if (g.first == key) {
      HIPCHK(hipGraphLaunch(g.second, s));
      return 0;
    }
  // build the launch sequence once: parse, then the match windows level by level
  KArgs A = base_args(h);
  A.one = arc_desc(h, d_out, out_cap);
  A.xcd_map = map;
  struct Launch {
    kfn_t k;
    uint64_t grid;
    KArgs a;
    unsigned block = kWG;
    size_t smem = 0;
  };
  std::vector<Launch> seq;
  kfn_t kp = pick_kernel<kModeParse>(pG, pU);
  if (stage != 2) seq.push_back({kp, grid_for(h->n_seg, resident_groups(kp, h->cu_count, pG), pG), A});
  if (h->n_match && stage != 1) {
    if (sched == 0) {
      kfn_t k = pick_kernel<kModeFlow>(G, U);
      const uint64_t windows = h->lvl_start.back() * (64 / G);
      seq.push_back({k, grid_for(windows, resident_groups(k, h->cu_count, G), G), A});
    } else {
      kfn_t k = pick_kernel<kModeLevels>(G, U);
      const uint64_t res = resident_groups(k, h->cu_count, G, pad);
      const uint64_t NL = h->lvl_start.size() - 1;
      std::vector<uint64_t> win(NL);
      for (uint64_t p = 0; p < NL; ++p) win[p] = h->lvl_start[p + 1] - h->lvl_start[p];
      const uint64_t pt = (tail == kTailOff) ? NL : tail_start(win, tail);
      for (uint64_t p = 0; p < pt; ++p) {
        KArgs a = A;
        a.lo = h->lvl_start[p];
        a.hi = h->lvl_start[p + 1];
        if (a.hi == a.lo) continue;
        seq.push_back({k, grid_for((a.hi - a.lo) * (64 / G), res, G), a, (unsigned)kWG, pad});
      }
      if (pt < NL) {  // the deepest levels: one workgroup
        KArgs a = A;
        a.lo = pt;
        a.hi = NL;
        seq.push_back({pick_tail(U, false), 1, a, (unsigned)kWGTail});
      }
    }
  }
  hipGraph_t graph = nullptr;
  HIPCHK(hipGraphCreate(&graph, 0));
  hipGraphNode_t prev = nullptr;
  for (Launch& L : seq) {
    hipKernelNodeParams kp2;
    memset(&kp2, 0, sizeof(kp2));
    void* args[] = {&L.a};
    kp2.func = (void*)L.k;
    kp2.gridDim = dim3((unsigned)L.grid);
    kp2.blockDim = dim3(L.block);
    kp2.sharedMemBytes = (unsigned)L.smem;
    kp2.kernelParams = args;
    kp2.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp2);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return lz::fail(LZ_E_HIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
    }
    prev = node;
  }
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return lz::fail(LZ_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  h->graphs.push_back({key, exec});
  HIPCHK(hipGraphLaunch(exec, s));
  return 0;
}

}  // namespace

extern "C" {

int lz_decode_device(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, void* stream) {
  return decode_stage(h, d_out, out_cap, cfg, 0, stream);
}

int lz_decode_device_stage(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, int stage,
                           void* stream) {
  return decode_stage(h, d_out, out_cap, cfg, stage, stream);
}

int lz_device_check(lz_dev* h, void* stream) {
  if (!h) return lz::fail(LZ_E_INVAL, "null handle");
  hipStream_t s = (hipStream_t)stream;
  uint32_t err = 0;
  HIPCHK(hipMemcpyAsync(&err, h->d_ctrl + 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uint32_t eerr = 0;
  if (h->d_coded) {
    HIPCHK(hipMemcpyAsync(&eerr, h->d_ctrl + 2, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  if (eerr) return lz::fail(LZ_E_CORRUPT, "the entropy stage met a corrupt tile (err %u)", eerr);
  if (err & 1u) return lz::fail(LZ_E_BUSY, "a bounded device wait expired (err %u)", err);
  if (err & 4u) return lz::fail(LZ_E_CORRUPT, "a match record outside the output was skipped (err %u)", err);
  if (err) return lz::fail(LZ_E_INVAL, "a kernel was launched with the wrong workgroup size (err %u)", err);
  return 0;
}

int lz_purecopy_device(uint64_t ntok, const uint64_t* d_dst, const uint64_t* d_lit_off, const uint32_t* d_lit_len,
                       const uint64_t* d_src, const uint32_t* d_mlen, uint64_t nunits, const uint64_t* d_unit_start,
                       const uint8_t* d_lit, uint64_t lit_size, const uint8_t* d_ref, uint64_t ref_size,
                       uint8_t* d_out, uint64_t out_size, const lz_decode_cfg* cfg, void* stream) {
  if (ntok && (!d_dst || !d_lit_off || !d_lit_len || !d_src || !d_mlen || !d_unit_start || !d_out))
    return lz::fail(LZ_E_INVAL, "null argument");
  uint32_t G, U, sched, tail, map;
  int rc = resolve_cfg(cfg, G, U, sched, &tail, &map);
  if (rc) return rc;
  if (nunits == 0) return 0;
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.xcd_map = map;
  A.one.lit = d_lit;
  A.one.lit_lo = (uintptr_t)d_lit;
  A.one.lit_hi = (uintptr_t)d_lit + lit_size;
  A.one.out = d_out;
  A.one.msrc = d_ref;
  A.one.msrc_lo = (uintptr_t)d_ref;
  A.one.msrc_hi = (uintptr_t)d_ref + ref_size;
  A.p_dst = d_dst;
  A.p_lit_off = d_lit_off;
  A.p_lit_len = d_lit_len;
  A.p_src = d_src;
  A.p_mlen = d_mlen;
  A.p_unit = d_unit_start;
  A.nunits = nunits;
  (void)out_size;
  kfn_t k = pick_kernel<kModePure>(G, U);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k, dim3((unsigned)grid_for(nunits, resident_groups(k, 256, G), G)), dim3(kWG), 0, s, A);
  HIPCHK(hipGetLastError());
  return 0;
}

}  // extern "C"

// ------------------------------------------------------------------ range decode
//
// Bytes [off, off+len) without a full decode (the region seek of Sec. 1 /
// Sec. 6 on compressed-resident data).  Host: the token closure of the range
// (tokens overlapping it, then, recursively, every token overlapping a source
// interval of a needed token; a self-overlapping match needs its period only)
// is laid out in output order in a scratch region, so any source interval of a
// needed token is contiguous there.  Each needed token becomes a literal piece
// (archive -> scratch) and a match piece (scratch -> scratch) whose depth is
// one more than the deepest piece it reads.  Device: one pure-copy launch for
// all literal pieces, one per match depth, and one gathering every range into
// the caller's output arena.  Several ranges are merged depth by depth.

struct lz_range_plan {
  uint64_t count = 0;
  // prefix mode: every token in [horizon, prefix_end) is decoded into the
  // scratch data, which holds output positions [horizon, data_end) (parse
  // segments [seg_lo, seg_hi), depth p windows [win_lo[p], win_hi[p]))
  bool prefix = false;
  uint64_t prefix_end = 0, horizon = 0, data_end = 0, seg_lo = 0, seg_hi = 0;
  std::vector<uint64_t> win_lo, win_hi;
  std::vector<uint64_t> range_src;   // per range: scratch-data offset of byte off
  std::vector<uint64_t> range_len;
  uint64_t data_bytes = 0;           // scratch-data bytes
  // pieces, level-major: level 0 = literal pieces, then match depths 1..D
  std::vector<uint64_t> p_dst, p_lit_off, p_src;
  std::vector<uint32_t> p_lit_len, p_mlen;
  std::vector<uint64_t> lvl_piece;   // first piece of each level (D+2 entries)
  std::vector<uint64_t> g_range, g_off;  // gather pieces: range and offset inside it
  uint64_t scratch_bytes = 0;        // total device scratch for lz_range_run
  uint8_t* staging = nullptr;        // pinned copy of the piece arrays
  uint64_t staging_bytes = 0;
  bool staging_owned = true;         // false: lent by a server's pinned pool
  ~lz_range_plan() {
    if (staging && staging_owned) (void)hipHostFree(staging);
  }
};

namespace lz {

uint8_t* lend_sync_staging(lz_dev* h, lz_range_plan* P, uint64_t extra, std::unique_lock<std::mutex>& lock) {
  lock = std::unique_lock<std::mutex>(h->sync_mu);
  const uint64_t at = (P->staging_bytes + 255) & ~uint64_t(255);
  const uint64_t need = at + extra;
  if (need > h->sync_pin_bytes) {
    if (h->sync_pin) (void)hipHostFree(h->sync_pin);
    h->sync_pin = nullptr;
    h->sync_pin_bytes = 0;
    const uint64_t nb = std::max<uint64_t>(need, 1ull << 20);
    if (hipHostMalloc((void**)&h->sync_pin, nb, 0) != hipSuccess) {
      h->sync_pin = nullptr;
      return nullptr;  // the plan allocates its own staging
    }
    h->sync_pin_bytes = nb;
  }
  P->staging = h->sync_pin;
  P->staging_owned = false;
  return h->sync_pin + at;
}

}  // namespace lz

namespace {

const std::vector<lz_dev::RTok>& block_tokens(lz_dev* h, uint64_t b) {
  if (!h->tok_cached[b]) {
    auto& o = h->tok_cache[b];
    o.clear();
    (void)lz::walk_block(h->v, b, [&](uint64_t, const lz::Tok& k) {
      o.push_back(lz_dev::RTok{k.dst, k.lit_off, k.src, (uint32_t)k.lit_len, (uint32_t)k.mlen});
    });
    h->tok_cached[b] = 1;
  }
  return h->tok_cache[b];
}

struct NeedTok {
  uint64_t dst, lit_off, src;
  uint32_t ll, ml;
  uint64_t scratch;  // scratch-data offset of dst
  uint32_t level;    // match depth
};

// Token closure of [off, off+len): needed tokens sorted by dst.  Stops and
// returns false once the needed tokens span more than `budget` bytes.
bool closure(lz_dev* h, uint64_t off, uint64_t len, std::vector<NeedTok>& need, uint64_t budget) {
  const uint32_t lb = h->v.log2_bs;
  std::vector<std::pair<uint64_t, uint64_t>> work{{off, off + len}};
  std::unordered_map<uint64_t, std::vector<uint8_t>> seen;  // visited blocks: tokens taken
  uint64_t bytes = 0;
  need.clear();
  while (!work.empty()) {
    auto [a, e] = work.back();
    work.pop_back();
    for (uint64_t b = a >> lb; a < e && b < h->v.nb; ++b) {
      const auto& T = block_tokens(h, b);
      auto& sb = seen[b];
      if (sb.empty()) sb.assign(T.size(), 0);
      // first token with dst + span > a
      size_t i = std::upper_bound(T.begin(), T.end(), a, [](uint64_t x, const lz_dev::RTok& t) { return x < t.dst; }) -
                 T.begin();
      i = i ? i - 1 : 0;
      const uint64_t bend = std::min(e, (b + 1) << lb);
      for (; i < T.size() && T[i].dst < bend; ++i) {
        const auto& t = T[i];
        if (t.dst + t.ll + t.ml <= a || sb[i]) continue;
        sb[i] = 1;
        need.push_back(NeedTok{t.dst, t.lit_off, t.src, t.ll, t.ml, 0, 0});
        bytes += (uint64_t)t.ll + t.ml;
        if (bytes > budget) return false;
        if (t.ml) {
          const uint64_t m0 = t.dst + t.ll;
          work.push_back({t.src, std::min(t.src + t.ml, m0)});
        }
      }
      a = (b + 1) << lb;
    }
  }
  std::sort(need.begin(), need.end(), [](const NeedTok& x, const NeedTok& y) { return x.dst < y.dst; });
  return true;
}

// Index of the needed token containing output position x (it exists).
size_t find_need(const std::vector<NeedTok>& need, uint64_t x) {
  size_t i = std::upper_bound(need.begin(), need.end(), x, [](uint64_t v, const NeedTok& t) { return v < t.dst; }) -
             need.begin();
  return i - 1;
}

// Decode horizon of the output prefix [0, end) as seen from position off: the
// largest grain start h <= off such that no match written in the grains from
// h's through the one holding end - 1 reads below h.  Decoding those grains
// alone (from h) then reproduces every byte of [h, end).  h = 0 always
// qualifies; segment-encoded archives give their segment starts.
uint64_t decode_horizon(const lz_dev* h, uint64_t off, uint64_t end) {
  if (end == 0 || h->grain_low.empty()) return 0;
  const uint32_t lg = h->log2_grain;
  const uint64_t g_last = (end - 1) >> lg;
  uint64_t g = std::min(off >> lg, g_last);
  uint64_t low = UINT64_MAX;
  for (uint64_t q = g; q <= g_last; ++q) low = std::min(low, h->grain_low[q]);
  while (low < (g << lg)) {
    const uint64_t g2 = low >> lg;
    for (uint64_t q = g2; q < g; ++q) low = std::min(low, h->grain_low[q]);
    g = g2;
  }
  return g << lg;
}

}  // namespace

extern "C" {

int lz_range_plan_create(lz_dev* h, uint64_t count, const uint64_t* off, const uint64_t* len, lz_range_plan** out) {
  if (!h || !out || (count && (!off || !len))) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  for (uint64_t r = 0; r < count; ++r)
    if (off[r] > h->v.n || len[r] > h->v.n - off[r])
      return lz::fail(LZ_E_RANGE, "range [%llu, +%llu) outside [0, %llu)", (unsigned long long)off[r],
                      (unsigned long long)len[r], (unsigned long long)h->v.n);
  std::lock_guard<std::mutex> lock(h->mu);
  lz_range_plan* P = new lz_range_plan();
  try {
    P->count = count;
    // per level: pieces, across ranges
    std::vector<std::vector<std::array<uint64_t, 5>>> by_lvl(1);  // dst, lit_off, lit_len, src, mlen
    std::vector<NeedTok> need;
    uint64_t base = 0;
    // A closure costs host work per byte, a prefix decode runs on the device at
    // HBM speed: closures are tried while they stay within a budget that grows
    // with the prefix the ranges would need.
    uint64_t end = 0, first = h->v.n;
    for (uint64_t r = 0; r < count; ++r) {
      end = std::max(end, off[r] + len[r]);
      if (len[r]) first = std::min(first, off[r]);
    }
    const uint64_t horizon = (end > 0 && first < end) ? decode_horizon(h, first, end) : 0;
    uint64_t budget = std::max<uint64_t>(kClosureMin, (end - horizon) / kClosureRatio);
    for (uint64_t r = 0; r < count && !P->prefix; ++r) {
      P->range_len.push_back(len[r]);
      if (len[r] == 0) {
        P->range_src.push_back(base);
        continue;
      }
      if (!closure(h, off[r], len[r], need, budget)) {
        P->prefix = true;
        break;
      }
      uint64_t spent = 0;
      for (auto& t : need) spent += (uint64_t)t.ll + t.ml;
      budget -= std::min(budget, spent);
      uint64_t acc = 0;
      for (auto& t : need) {
        t.scratch = base + acc;
        acc += (uint64_t)t.ll + t.ml;
      }
      // depths in output order: a match reads only earlier needed tokens
      for (size_t k = 0; k < need.size(); ++k) {
        NeedTok& t = need[k];
        if (t.ll) by_lvl[0].push_back({t.scratch, t.lit_off, t.ll, 0, 0});
        if (!t.ml) continue;
        const uint64_t m0 = t.dst + t.ll;
        const uint64_t se = std::min(t.src + t.ml, m0);
        uint32_t d = 0;
        for (size_t j = find_need(need, t.src); j < need.size() && need[j].dst < se; ++j) {
          const NeedTok& u = need[j];
          const uint64_t um0 = u.dst + u.ll;
          if (um0 < se && um0 + u.ml > t.src && u.ml) d = std::max(d, u.level);  // overlaps u's match part
        }
        t.level = d + 1;
        if (by_lvl.size() <= t.level) by_lvl.resize(t.level + 1);
        const size_t j = find_need(need, t.src);
        const uint64_t src_s = need[j].scratch + (t.src - need[j].dst);
        by_lvl[t.level].push_back({t.scratch + t.ll, 0, 0, src_s, t.ml});
      }
      const size_t j = find_need(need, off[r]);
      P->range_src.push_back(need[j].scratch + (off[r] - need[j].dst));
      base += acc;
    }
    if (P->prefix) {
      // decode every token of [horizon, end) into the scratch data, then gather
      by_lvl.assign(1, {});
      P->range_len.assign(len, len + count);
      P->prefix_end = end;
      P->horizon = horizon;
      // windows starting in [horizon, end) have all their matches in the grains
      // up to the one holding end - 1: the parse of those grains' blocks writes
      // their records, and the scratch data covers them
      const uint32_t lg = h->log2_grain;
      P->data_end = end ? std::min(h->v.n, (((end - 1) >> lg) + 1) << lg) : horizon;
      P->range_src.assign(count, 0);  // replaces the entries of ranges served by closures so far
      for (uint64_t r = 0; r < count; ++r) P->range_src[r] = len[r] ? off[r] - horizon : 0;
      base = P->data_end - horizon;
      // parse segments are in block order
      auto seg_bound = [&](uint64_t blk) {  // first segment of a block >= blk
        uint64_t lo = 0, hi = h->h_seg.size() / 8;
        while (lo < hi) {
          const uint64_t mid = (lo + hi) / 2;
          if ((h->h_seg[8 * mid + 7] & 0xFFFFFFFFull) < blk) lo = mid + 1;
          else hi = mid;
        }
        return lo;
      };
      if (P->data_end > horizon) {
        P->seg_lo = seg_bound(horizon >> h->v.log2_bs);
        P->seg_hi = seg_bound(((P->data_end - 1) >> h->v.log2_bs) + 1);
      }
      const size_t NL = h->lvl_start.size() ? h->lvl_start.size() - 1 : 0;
      P->win_lo.assign(NL, 0);
      P->win_hi.assign(NL, 0);
      for (size_t p = 0; p < NL; ++p) {
        // windows of depth p whose first byte lies in [horizon, end)
        auto b0 = h->h_wdst.begin() + h->lvl_start[p], b1 = h->h_wdst.begin() + h->lvl_start[p + 1];
        P->win_lo[p] = (uint64_t)(std::lower_bound(b0, b1, horizon) - h->h_wdst.begin());
        P->win_hi[p] = std::max(P->win_lo[p], (uint64_t)(std::lower_bound(b0, b1, end) - h->h_wdst.begin()));
      }
    }
    P->data_bytes = base;
    P->lvl_piece.push_back(0);
    for (auto& L : by_lvl) {
      for (auto& q : L) {
        P->p_dst.push_back(q[0]);
        P->p_lit_off.push_back(q[1]);
        P->p_lit_len.push_back((uint32_t)q[2]);
        P->p_src.push_back(q[3]);
        P->p_mlen.push_back((uint32_t)q[4]);
      }
      P->lvl_piece.push_back(P->p_dst.size());
    }
    // gather pieces: every range in pieces of kGatherPiece bytes, reading the
    // scratch data as "literals"; output offsets are given at run time
    for (uint64_t r = 0; r < count; ++r)
      for (uint64_t o = 0; o < len[r]; o += kGatherPiece) {
        P->g_range.push_back(r);
        P->g_off.push_back(o);
        P->p_dst.push_back(0);
        P->p_lit_off.push_back(P->range_src[r] + o);
        P->p_lit_len.push_back((uint32_t)std::min<uint64_t>(kGatherPiece, len[r] - o));
        P->p_src.push_back(0);
        P->p_mlen.push_back(0);
      }
    P->lvl_piece.push_back(P->p_dst.size());
  } catch (const std::bad_alloc&) {
    delete P;
    return lz::fail(LZ_E_NOMEM, "range plan allocation failed");
  }
  // staging layout: dst | lit_off | src (u64) | lit_len | mlen (u32) | unit starts (u64, one unit per piece)
  const uint64_t np = P->p_dst.size();
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  P->staging_bytes = a256(8 * np) * 3 + a256(4 * np) * 2 + 2 * a256(4 * P->win_hi.size());
  P->scratch_bytes = P->staging_bytes + a256(P->data_bytes + 16);
  *out = P;
  return 0;
}

uint64_t lz_range_plan_scratch_bytes(const lz_range_plan* P) { return P ? P->scratch_bytes : 0; }
uint64_t lz_range_plan_levels(const lz_range_plan* P) {
  if (!P) return 0;
  if (P->prefix) return P->win_hi.size();
  return P->lvl_piece.size() > 2 ? P->lvl_piece.size() - 3 : 0;
}
uint64_t lz_range_plan_closure_bytes(const lz_range_plan* P) { return P ? (P->prefix ? 0 : P->data_bytes) : 0; }
uint64_t lz_range_plan_prefix_bytes(const lz_range_plan* P) { return P && P->prefix ? P->prefix_end - P->horizon : 0; }
uint64_t lz_range_plan_horizon(const lz_range_plan* P) { return P && P->prefix ? P->horizon : 0; }
void lz_range_plan_free(lz_range_plan* P) { delete P; }

int lz_range_run(lz_dev* h, lz_range_plan* P, uint8_t* d_out, uint64_t out_cap, const uint64_t* out_off,
                 void* d_scratch, uint64_t scratch_cap, const lz_decode_cfg* cfg, void* stream) {
  if (!h || !P || (P->count && (!d_out || !out_off)) || !d_scratch) return lz::fail(LZ_E_INVAL, "null argument");
  if (scratch_cap < P->scratch_bytes)
    return lz::fail(LZ_E_NOMEM, "range scratch %llu < %llu bytes", (unsigned long long)scratch_cap,
                    (unsigned long long)P->scratch_bytes);
  for (uint64_t r = 0; r < P->count; ++r)
    if (out_off[r] > out_cap || P->range_len[r] > out_cap - out_off[r])
      return lz::fail(LZ_E_INVAL, "range %llu does not fit the output arena", (unsigned long long)r);
  uint32_t G, U, sched, tail, map, occ, pG, pU;
  int rc = resolve_cfg(cfg, G, U, sched, &tail, &map, &occ, &pG, &pU);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const uint64_t np = P->p_dst.size();
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  // gather pieces take the caller's output offsets
  const uint64_t g0 = P->lvl_piece[P->lvl_piece.size() - 2];
  for (size_t i = 0; i < P->g_range.size(); ++i) P->p_dst[g0 + i] = out_off[P->g_range[i]] + P->g_off[i];
  if (!P->staging && hipHostMalloc((void**)&P->staging, P->staging_bytes, 0) != hipSuccess) {
    P->staging = nullptr;
    return lz::fail(LZ_E_NOMEM, "pinned staging allocation failed");
  }
  uint8_t* st = P->staging;
  uint64_t o = 0;
  const uint64_t o_dst = o; memcpy(st + o, P->p_dst.data(), 8 * np); o += a256(8 * np);
  const uint64_t o_loff = o; memcpy(st + o, P->p_lit_off.data(), 8 * np); o += a256(8 * np);
  const uint64_t o_src = o; memcpy(st + o, P->p_src.data(), 8 * np); o += a256(8 * np);
  const uint64_t o_llen = o; memcpy(st + o, P->p_lit_len.data(), 4 * np); o += a256(4 * np);
  const uint64_t o_mlen = o; memcpy(st + o, P->p_mlen.data(), 4 * np); o += a256(4 * np);
  const uint64_t o_lo = o;
  for (size_t p = 0; p < P->win_lo.size(); ++p) ((uint32_t*)(st + o))[p] = (uint32_t)P->win_lo[p];
  o += a256(4 * P->win_lo.size());
  const uint64_t o_hi = o;
  for (size_t p = 0; p < P->win_hi.size(); ++p) ((uint32_t*)(st + o))[p] = (uint32_t)P->win_hi[p];
  o += a256(4 * P->win_hi.size());
  uint8_t* D = (uint8_t*)d_scratch;
  HIPCHK(hipMemcpyAsync(D, st, P->staging_bytes, hipMemcpyHostToDevice, s));
  uint8_t* data = D + P->staging_bytes;
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.xcd_map = map;
  A.p_dst = (const uint64_t*)(D + o_dst);
  A.p_lit_off = (const uint64_t*)(D + o_loff);
  A.p_src = (const uint64_t*)(D + o_src);
  A.p_lit_len = (const uint32_t*)(D + o_llen);
  A.p_mlen = (const uint32_t*)(D + o_mlen);
  if (P->prefix) {
    // every token of [horizon, data_end), decoded into the scratch data: the
    // output base is placed `horizon` bytes before it, so absolute positions
    // index it directly, and no match may touch a position below the horizon
    KArgs A = base_args(h);
    A.xcd_map = map;
    A.one = arc_desc(h, data - P->horizon, P->data_end);
    A.one.msrc_lo = (uintptr_t)data;
    A.one.msrc_hi = (uintptr_t)data + P->data_bytes;
    A.one.n = P->data_end;
    A.one.out_lo = P->horizon;
    A.seg = h->d_seg + 8 * P->seg_lo;
    A.nseg = P->seg_hi - P->seg_lo;
    if (A.nseg) {
      kfn_t kp = pick_kernel<kModeParse>(pG, pU);
      hipLaunchKernelGGL(kp, dim3((unsigned)grid_for(A.nseg, resident_groups(kp, h->cu_count, pG), pG)), dim3(kWG),
                         0, s, A);
      HIPCHK(hipGetLastError());
    }
    kfn_t kl = pick_kernel<kModeLevels>(G, U);
    const uint64_t rl = resident_groups(kl, h->cu_count, G);
    const uint64_t NL = P->win_hi.size();
    std::vector<uint64_t> cnt(NL);
    for (uint64_t p = 0; p < NL; ++p) cnt[p] = P->win_hi[p] - P->win_lo[p];
    const uint64_t pt = (tail == kTailOff) ? NL : tail_start(cnt, tail);
    for (uint64_t p = 0; p < pt; ++p) {
      KArgs a = A;
      a.lo = P->win_lo[p];
      a.hi = P->win_hi[p];
      if (a.hi <= a.lo) continue;
      hipLaunchKernelGGL(kl, dim3((unsigned)grid_for((a.hi - a.lo) * (64 / G), rl, G)), dim3(kWG), 0, s, a);
      HIPCHK(hipGetLastError());
    }
    if (pt < NL) {  // the deepest depths of the prefix in one workgroup
      KArgs a = A;
      a.lo = pt;
      a.hi = NL;
      a.lvl_start = (const uint32_t*)(D + o_lo);
      a.lvl_hi = (const uint32_t*)(D + o_hi);
      hipLaunchKernelGGL(pick_tail(U, false), dim3(1), dim3(kWGTail), 0, s, a);
      HIPCHK(hipGetLastError());
    }
  }
  kfn_t k = pick_kernel<kModePure>(G, U);
  const uint64_t res = resident_groups(k, h->cu_count, G);
  const size_t L = P->lvl_piece.size() - 1;  // levels incl. literal and gather
  for (size_t l = 0; l < L; ++l) {
    const uint64_t p0 = P->lvl_piece[l], p1 = P->lvl_piece[l + 1];
    if (p1 == p0) continue;
    KArgs a = A;
    a.lo = p0;  // windows of G pieces (pieces of one depth are independent)
    a.hi = p1;
    const bool gather = (l + 1 == L);
    if (gather) a.per_item = 1;  // a group per gather piece: the copy is spread over the GPU
    if (l == 0) {  // literal pieces: archive literals -> scratch data
      a.one.lit = h->d_arc + h->v.off_lit;
      a.one.lit_lo = (uintptr_t)h->d_arc;
      a.one.lit_hi = (uintptr_t)h->d_arc + h->v.total;
      a.one.out = data;
    } else if (gather) {  // scratch data -> caller's arena
      a.one.lit = data;
      a.one.lit_lo = (uintptr_t)data;
      a.one.lit_hi = (uintptr_t)data + P->data_bytes + 16;
      a.one.out = d_out;
    } else {  // match pieces inside the scratch data
      a.one.out = data;
    }
    a.one.msrc = data;
    a.one.msrc_lo = (uintptr_t)data;
    a.one.msrc_hi = (uintptr_t)data + P->data_bytes + 16;
    const uint64_t items = gather ? (p1 - p0) : (p1 - p0 + G - 1) / G;
    hipLaunchKernelGGL(k, dim3((unsigned)grid_for(items, res, G)), dim3(kWG), 0, s, a);
    HIPCHK(hipGetLastError());
  }
  return 0;
}

int lz_range_scratch_bytes(lz_dev* h, uint64_t off, uint64_t len, uint64_t* bytes) {
  if (!bytes) return lz::fail(LZ_E_INVAL, "null output");
  lz_range_plan* P = nullptr;
  int rc = lz_range_plan_create(h, 1, &off, &len, &P);
  if (rc) return rc;
  *bytes = P->scratch_bytes;
  delete P;
  return 0;
}

int lz_decode_range(lz_dev* h, uint64_t off, uint64_t len, uint8_t* d_out, void* d_scratch, uint64_t scratch_cap,
                    void* stream) {
  lz_range_plan* P = nullptr;
  int rc = lz_range_plan_create(h, 1, &off, &len, &P);
  if (rc) return rc;
  const uint64_t zero = 0;
  std::unique_lock<std::mutex> lock;
  (void)lz::lend_sync_staging(h, P, 0, lock);
  rc = lz_range_run(h, P, d_out, len, &zero, d_scratch, scratch_cap, nullptr, stream);
  // the plan's pinned staging is read by the copy engine: wait before freeing
  // or lending it again
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == 0) rc = lz::fail(LZ_E_HIP, "stream sync failed");
  delete P;
  return rc;
}

}  // extern "C"

// ------------------------------------------------------------------ batch decode
//
// Thousands of archives in one replayable launch sequence: archives that share
// a configuration form a group; a group is one parse launch over the parse
// segments of all its archives and one launch per dependency depth over the
// depth-p windows of all its archives, with the small deepest depths in one
// workgroup (or one launch for schedule 0).  Every
// work item carries its archive index; the kernels read that archive's
// streams, plan and output from a descriptor table.  All groups are recorded
// in one graph.

struct lz_batch {
  hipGraphExec_t exec = nullptr;
  uint64_t scratch_used = 0;
  uint64_t launches = 0;
  ~lz_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

namespace {

struct BatchGroup {
  lz_decode_cfg cfg;
  std::vector<uint32_t> arcs;  // archive indices
};

// windows over every depth of the group's archives
uint64_t group_windows(const std::vector<lz_dev*>& H, const BatchGroup& g, uint64_t* nl_out) {
  uint64_t nw = 0, nl = 0;
  for (uint32_t i : g.arcs) {
    const auto& ls = H[i]->lvl_start;
    nw += ls.empty() ? 0 : ls.back();
    nl = std::max<uint64_t>(nl, ls.size() ? ls.size() - 1 : 0);
  }
  if (nl_out) *nl_out = nl;
  return nw;
}

uint64_t group_scratch(const std::vector<lz_dev*>& H, const BatchGroup& g, uint64_t* nseg_out, uint64_t* nw_out,
                       uint64_t* nl_out) {
  uint64_t nseg = 0, nl = 0;
  for (uint32_t i : g.arcs) nseg += H[i]->h_seg.size() / 8;
  const uint64_t nw = group_windows(H, g, &nl);
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  if (nseg_out) *nseg_out = nseg;
  if (nw_out) *nw_out = nw;
  if (nl_out) *nl_out = nl;
  return a256(sizeof(ArcDesc) * g.arcs.size()) + a256(64 * nseg) + a256(16 * (nw + 1)) + 3 * a256(4 * (nl + 1)) + 256;
}

std::vector<BatchGroup> make_groups(uint32_t count, const lz_decode_cfg* cfgs) {
  std::vector<BatchGroup> groups;
  for (uint32_t i = 0; i < count; ++i) {
    lz_decode_cfg c{64, 2, 1, 0};
    if (cfgs) c = cfgs[i];
    if (!c.G) c.G = 64;
    if (!c.unroll) c.unroll = 2;
    if (!c.parse_G) c.parse_G = 64;
    if (!c.parse_unroll) c.parse_unroll = 2;
    size_t k = 0;
    for (; k < groups.size(); ++k)
      if (groups[k].cfg.G == c.G && groups[k].cfg.unroll == c.unroll && groups[k].cfg.schedule == c.schedule &&
          groups[k].cfg.tail == c.tail && groups[k].cfg.mapping == c.mapping &&
          groups[k].cfg.parse_G == c.parse_G && groups[k].cfg.parse_unroll == c.parse_unroll)
        break;
    if (k == groups.size()) groups.push_back(BatchGroup{c, {}});
    groups[k].arcs.push_back(i);
  }
  return groups;
}

}  // namespace

extern "C" {

int lz_batch_scratch_bytes(uint32_t count, lz_dev* const* handles, const lz_decode_cfg* cfgs, uint64_t* bytes) {
  if (!bytes || (count && !handles)) return lz::fail(LZ_E_INVAL, "null argument");
  std::vector<lz_dev*> H(handles, handles + count);
  uint64_t tot = 0;
  for (auto& g : make_groups(count, cfgs)) tot += group_scratch(H, g, nullptr, nullptr, nullptr);
  *bytes = tot + 256;
  return 0;
}

int lz_batch_create(uint32_t count, lz_dev* const* handles, uint8_t* const* d_out, const uint64_t* out_cap,
                    const lz_decode_cfg* cfgs, void* d_scratch, uint64_t scratch_cap, void* stream, lz_batch** out) {
  if (!out || (count && (!handles || !d_out || !out_cap)) || !d_scratch) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  // the scratch holds words that kernels update atomically (error flag, counters)
  if ((uintptr_t)d_scratch & 255u) return lz::fail(LZ_E_INVAL, "d_scratch must be 256-byte aligned");
  if (count >= (1u << 24)) return lz::fail(LZ_E_INVAL, "at most 2^24 - 1 archives per batch");
  std::vector<lz_dev*> H(handles, handles + count);
  for (uint32_t i = 0; i < count; ++i) {
    if (!H[i]) return lz::fail(LZ_E_INVAL, "null handle %u", i);
    if (out_cap[i] < H[i]->v.n) return lz::fail(LZ_E_INVAL, "output %u too small", i);
    if (H[i]->v.n && !d_out[i]) return lz::fail(LZ_E_INVAL, "null output %u", i);
  }
  auto groups = make_groups(count, cfgs);
  uint64_t need = 256;
  for (auto& g : groups) {
    uint32_t G, U, sched;
    int rc = resolve_cfg(&g.cfg, G, U, sched);
    if (rc) return rc;
    if (sched == 0)
      for (uint32_t i : g.arcs)
        if (out_cap[i] > 0xFFFFFFFFull) return lz::fail(LZ_E_INVAL, "schedule 0 outputs must be below 4 GiB");
    need += group_scratch(H, g, nullptr, nullptr, nullptr);
  }
  if (scratch_cap < need)
    return lz::fail(LZ_E_NOMEM, "batch scratch %llu < %llu bytes", (unsigned long long)scratch_cap,
                    (unsigned long long)need);
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  hipStream_t s = (hipStream_t)stream;
  // host images of every group's tables, uploaded in one copy
  std::vector<uint8_t> img(need, 0);
  uint8_t* D0 = (uint8_t*)d_scratch;
  struct Launch {
    kfn_t k;
    uint64_t grid;
    KArgs a;
    unsigned block = kWG;
  };
  std::vector<Launch> seq;
  uint64_t off = 0;
  int cu = 0;
  for (lz_dev* h : H) cu = std::max(cu, h->cu_count);
  for (auto& g : groups) {
    uint32_t G, U, sched, tail, map, occ, pG, pU;
    (void)resolve_cfg(&g.cfg, G, U, sched, &tail, &map, &occ, &pG, &pU);
    uint64_t nseg, nw, nl;
    group_scratch(H, g, &nseg, &nw, &nl);
    const uint64_t o_desc = off;
    const uint64_t o_seg = o_desc + a256(sizeof(ArcDesc) * g.arcs.size());
    const uint64_t o_items = o_seg + a256(64 * nseg);
    const uint64_t o_lvls = o_items + a256(16 * (nw + 1));
    const uint64_t o_tick = o_lvls + a256(4 * (nl + 1));
    const uint64_t o_wdone = o_tick + a256(4 * (nl + 1));
    const uint64_t o_err = o_wdone + a256(4 * (nl + 1));
    off = o_err + 256;
    ArcDesc* desc = (ArcDesc*)(img.data() + o_desc);
    uint64_t* seg = (uint64_t*)(img.data() + o_seg);
    uint32_t* items = (uint32_t*)(img.data() + o_items);
    uint32_t* lvls = (uint32_t*)(img.data() + o_lvls);
    uint64_t si = 0;
    for (uint32_t j = 0; j < g.arcs.size(); ++j) {
      lz_dev* h = H[g.arcs[j]];
      desc[j] = arc_desc(h, d_out[g.arcs[j]], out_cap[g.arcs[j]]);
      for (size_t r = 0; r + 8 <= h->h_seg.size(); r += 8) {
        for (int w = 0; w < 7; ++w) seg[8 * si + w] = h->h_seg[r + w];
        seg[8 * si + 7] = ((uint64_t)j << 32) | (h->h_seg[r + 7] & 0xFFFFFFFFull);
        ++si;
      }
    }
    // windows of all archives, level-major
    uint64_t wi = 0;
    for (uint64_t p = 0; p < nl; ++p) {
      lvls[p] = (uint32_t)wi;
      for (uint32_t j = 0; j < g.arcs.size(); ++j) {
        const lz_dev* h = H[g.arcs[j]];
        const auto& ls = h->lvl_start;
        if (p + 1 >= ls.size()) continue;
        for (uint64_t q = ls[p]; q < ls[p + 1]; ++q, ++wi) {
          items[4 * wi] = h->h_win[4 * q];
          items[4 * wi + 1] = h->h_win[4 * q + 1] | (j << 8);
          items[4 * wi + 2] = h->h_win[4 * q + 2];
          items[4 * wi + 3] = h->h_win[4 * q + 3];
        }
      }
    }
    lvls[nl] = (uint32_t)wi;
    KArgs A;
    memset(&A, 0, sizeof(A));
    A.xcd_map = map;
    A.arcs = (const ArcDesc*)(D0 + o_desc);
    A.one = desc[0];
    A.seg = (const uint64_t*)(D0 + o_seg);
    A.nseg = nseg;
    A.items = (const u32x4*)(D0 + o_items);
    A.lvl_start = (const uint32_t*)(D0 + o_lvls);
    A.tickets = (uint32_t*)(D0 + o_tick);
    A.wdone = (uint32_t*)(D0 + o_wdone);
    A.err = (uint32_t*)(D0 + o_err);
    A.n_levels = (uint32_t)nl;
    if (nseg) {
      kfn_t kp = pick_kernel<kModeParse>(pG, pU, true);
      seq.push_back({kp, grid_for(nseg, resident_groups(kp, cu, pG), pG), A});
    }
    if (nw) {
      if (sched == 0) {
        kfn_t k = pick_kernel<kModeFlow>(G, U, true);
        seq.push_back({k, grid_for(nw * (64 / G), resident_groups(k, cu, G), G), A});
      } else {
        kfn_t k = pick_kernel<kModeLevels>(G, U, true);
        const uint64_t res = resident_groups(k, cu, G);
        std::vector<uint64_t> win(nl);
        for (uint64_t p = 0; p < nl; ++p) win[p] = lvls[p + 1] - lvls[p];
        const uint64_t pt = (tail == kTailOff) ? nl : tail_start(win, tail);
        for (uint64_t p = 0; p < pt; ++p) {
          KArgs a = A;
          a.lo = lvls[p];
          a.hi = lvls[p + 1];
          if (a.hi == a.lo) continue;
          seq.push_back({k, grid_for((a.hi - a.lo) * (64 / G), res, G), a});
        }
        if (pt < nl) {  // the deepest levels: one workgroup over their windows
          KArgs a = A;
          a.lo = pt;
          a.hi = nl;
          seq.push_back({pick_tail(U, true), 1, a, (unsigned)kWGTail});
        }
      }
    }
  }
  // upload the tables (pinned staging), then record the launches
  uint8_t* hp = nullptr;
  if (hipHostMalloc((void**)&hp, off ? off : 1, 0) != hipSuccess) return lz::fail(LZ_E_NOMEM, "pinned staging failed");
  memcpy(hp, img.data(), off);
  hipError_t e1 = hipMemcpyAsync(D0, hp, off, hipMemcpyHostToDevice, s);
  hipError_t e2 = hipStreamSynchronize(s);
  (void)hipHostFree(hp);
  if (e1 != hipSuccess || e2 != hipSuccess) return lz::fail(LZ_E_HIP, "batch table upload failed");
  hipGraph_t graph = nullptr;
  HIPCHK(hipGraphCreate(&graph, 0));
  hipGraphNode_t prev = nullptr;
  for (Launch& L : seq) {
    hipKernelNodeParams kp2;
    memset(&kp2, 0, sizeof(kp2));
    void* args[] = {&L.a};
    kp2.func = (void*)L.k;
    kp2.gridDim = dim3((unsigned)L.grid);
    kp2.blockDim = dim3(L.block);
    kp2.kernelParams = args;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp2);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return lz::fail(LZ_E_HIP, "hipGraphAddKernelNode: %s", hipGetErrorString(e));
    }
    prev = node;
  }
  lz_batch* B = new lz_batch();
  hipError_t e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    delete B;
    return lz::fail(LZ_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  B->scratch_used = off;
  B->launches = seq.size();
  *out = B;
  return 0;
}

int lz_batch_launch(lz_batch* b, void* stream) {
  if (!b || !b->exec) return lz::fail(LZ_E_INVAL, "null batch");
  HIPCHK(hipGraphLaunch(b->exec, (hipStream_t)stream));
  return 0;
}

uint64_t lz_batch_launches(const lz_batch* b) { return b ? b->launches : 0; }
void lz_batch_destroy(lz_batch* b) { delete b; }

}  // extern "C"

// ------------------------------------------------------------------ autotuner
//
// Archives are bucketed by size (factor-4 buckets from 4 KiB).  For every
// bucket each candidate (G, unroll, schedule) is built as a batch of that
// bucket's archives alone and timed with HIP events over `reps` graph
// launches after one warm-up; the fastest candidate becomes the configuration
// of every archive in the bucket.

extern "C" int lz_autotune(uint32_t count, lz_dev* const* handles, uint8_t* const* d_out, const uint64_t* out_cap,
                           void* d_scratch, uint64_t scratch_cap, void* stream, uint32_t reps, lz_decode_cfg* chosen,
                           lz_tune_report* report, uint32_t report_cap, uint32_t* n_report) {
  if ((count && (!handles || !d_out || !out_cap || !chosen)) || !d_scratch) return lz::fail(LZ_E_INVAL, "null argument");
  if (reps == 0) reps = 3;
  hipStream_t s = (hipStream_t)stream;
  auto bucket_of = [&](uint64_t n) {
    int b = 0;
    uint64_t lim = 16384;
    while (n >= lim && b < 15) {
      lim <<= 2;
      ++b;
    }
    return b;
  };
  std::vector<std::vector<uint32_t>> buckets(16);
  for (uint32_t i = 0; i < count; ++i) buckets[bucket_of(handles[i]->v.n)].push_back(i);
  static const uint32_t Gs[3] = {16, 32, 64}, Us[3] = {1, 2, 4}, Ss[2] = {1, 0}, Ms[2] = {0, 1};
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // mean time of one replay of a batch (one warm-up launch, `reps` timed)
  auto time_batch = [&](uint32_t cnt, lz_dev* const* hs, uint8_t* const* outs, const uint64_t* caps,
                        const lz_decode_cfg* cf, float* ms) -> int {
    lz_batch* B = nullptr;
    int r = lz_batch_create(cnt, hs, outs, caps, cf, d_scratch, scratch_cap, stream, &B);
    if (r) return r;
    *ms = 0;
    r = lz_batch_launch(B, stream);
    if (!r && hipEventRecord(e0, s) != hipSuccess) r = lz::fail(LZ_E_HIP, "event record failed");
    for (uint32_t k = 0; k < reps && !r; ++k) r = lz_batch_launch(B, stream);
    if (!r && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
               hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      r = lz::fail(LZ_E_HIP, "event timing failed");
    lz_batch_destroy(B);
    *ms /= (float)reps;
    return r;
  };
  uint32_t nrep = 0;
  int rc = 0;
  for (int b = 0; b < 16 && rc == 0; ++b) {
    auto& idx = buckets[b];
    if (idx.empty()) continue;
    std::vector<lz_dev*> H;
    std::vector<uint8_t*> O;
    std::vector<uint64_t> C;
    uint64_t bytes = 0;
    for (uint32_t i : idx) {
      H.push_back(handles[i]);
      O.push_back(d_out[i]);
      C.push_back(out_cap[i]);
      bytes += handles[i]->v.n;
    }
    lz_decode_cfg best{64, 2, 1, 0};
    float best_ms = 1e30f, default_ms = -1.f;
    for (uint32_t M : Ms)
    for (uint32_t S : Ss)
      for (uint32_t G : Gs)
        for (uint32_t U : Us) {
          lz_decode_cfg c{G, U, S, 0, M};
          bool too_big = false;
          if (S == 0)
            for (uint64_t cap : C) too_big = too_big || cap > 0xFFFFFFFFull;
          if (too_big) continue;
          std::vector<lz_decode_cfg> cf(idx.size(), c);
          float ms = 0;
          rc = time_batch((uint32_t)idx.size(), H.data(), O.data(), C.data(), cf.data(), &ms);
          if (rc) break;
          if (G == 64 && U == 2 && S == 1 && M == 0) default_ms = ms;
          if (ms < best_ms) {
            best_ms = ms;
            best = c;
          }
        }
    if (rc) break;
    for (uint32_t i : idx) chosen[i] = best;
    if (report && nrep < report_cap) {
      lz_tune_report& R = report[nrep];
      R.min_bytes = (b == 0) ? 0 : (16384ull << (2 * (b - 1)));
      R.max_bytes = 16384ull << (2 * b);
      R.archives = (uint32_t)idx.size();
      R.bytes = bytes;
      R.best = best;
      R.best_ms = best_ms;
      R.default_ms = default_ms;
    }
    ++nrep;
  }
  // Buckets are tuned alone, but a batch with several configurations runs a
  // launch sequence per configuration: keep the choices only if the whole
  // batch is faster with them than with the default (when the scratch holds
  // the batch with the choices)
  if (rc == 0 && nrep > 1) {
    std::vector<lz_decode_cfg> dflt(count, lz_decode_cfg{64, 2, 1, 0, 0, 0, 0, 0});
    uint64_t need = 0;
    if (lz_batch_scratch_bytes(count, handles, chosen, &need) == 0 && need <= scratch_cap) {
      float t_chosen = 0, t_default = 0;
      rc = time_batch(count, handles, d_out, out_cap, chosen, &t_chosen);
      if (!rc) rc = time_batch(count, handles, d_out, out_cap, dflt.data(), &t_default);
      if (!rc && t_default <= t_chosen)
        for (uint32_t i = 0; i < count; ++i) chosen[i] = dflt[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_report) *n_report = nrep;
  return rc;
}

// ------------------------------------------------------------------ serving
//
// Continuous batching of range requests against one device-resident archive.
// Requests wait in a FIFO; a tick first retires every launched group whose
// completion event has fired (their requests become done, their scratch and
// staging are freed), then admits waiting requests in arrival order while a
// request slot is free and the device arena has room for its output, splits
// them by decode horizon and launches one merged range plan per horizon on the
// next of four streams, so groups run beside each other and beside earlier
// ones (a horizon with a group still on the device holds its new requests for
// the next one); a group whose scratch does not fit sends later groups and
// then its newest requests back to the head of the queue.  Outputs stay in the arena until
// released.  A tick allocates and frees no device or pinned memory and creates
// no events: plan staging comes from a pinned pool and completion events from
// a pool, both owned by the server (freeing pinned memory waits for the whole
// device, which would serialise the groups).

namespace {

// First-fit allocator over [0, bytes) in 256-byte units: free extents by offset.
struct Extents {
  std::map<uint64_t, uint64_t> free_ext;
  uint64_t used = 0, high_water = 0;
  static uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }
  void reset(uint64_t bytes) {
    free_ext.clear();
    if (bytes) free_ext[0] = bytes;
    used = 0;
  }
  bool alloc(uint64_t len, uint64_t* at) {
    len = a256(std::max<uint64_t>(len, 1));
    for (auto it = free_ext.begin(); it != free_ext.end(); ++it)
      if (it->second >= len) {
        *at = it->first;
        const uint64_t rest = it->second - len, nxt = it->first + len;
        free_ext.erase(it);
        if (rest) free_ext[nxt] = rest;
        used += len;
        high_water = std::max(high_water, used);
        return true;
      }
    return false;
  }
  void release(uint64_t at, uint64_t len) {
    len = a256(std::max<uint64_t>(len, 1));
    used -= len;
    auto it = free_ext.emplace(at, len).first;
    auto nx = std::next(it);
    if (nx != free_ext.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_ext.erase(nx);
    }
    if (it != free_ext.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_ext.erase(it);
      }
    }
  }
};

constexpr uint64_t kPinPoolMin = 16ull << 20;  // initial pinned staging pool of a server
constexpr int kServeStreams = 4;               // groups launched round-robin on these

}  // namespace

struct lz_server {
  lz_dev* h = nullptr;
  uint8_t* arena = nullptr;
  uint64_t arena_bytes = 0;
  uint32_t slots = 0;
  lz_decode_cfg cfg{64, 2, 1, 0};
  hipStream_t streams[kServeStreams] = {};
  uint32_t next_stream = 0;
  struct Req {
    uint64_t id, off, len;
    uint64_t out_at = 0;          // arena offset of the output
    uint64_t hz = 0;              // decode horizon (set on admission)
    int state = 0;                // 0 waiting, 1 running, 2 done, 3 released, 4 failed
  };
  std::vector<Req> reqs;          // indexed by id (ids increase in arrival order)
  std::deque<uint64_t> queue;     // waiting ids, arrival order
  std::vector<uint64_t> held;     // admitted, waiting for a running group of their horizon
  std::deque<uint64_t> completed; // finished (done or failed), not yet taken by lz_serve_completed
  uint32_t active = 0;            // admitted (or failed), not yet released
  struct Group {
    hipEvent_t ev;
    uint64_t hz;
    lz_range_plan* plan;
    uint64_t scratch_at, scratch_len, pin_at, pin_len;
    std::vector<uint64_t> ids;
  };
  std::vector<Group> running;
  uint64_t max_running = 0;       // most groups in flight after any tick
  Extents mem;                    // device arena
  Extents pin;                    // pinned staging pool
  uint8_t* pin_base = nullptr;
  uint64_t pin_bytes = 0;
  std::vector<hipEvent_t> ev_free;
  ~lz_server() {
    for (hipEvent_t e : ev_free) (void)hipEventDestroy(e);
    if (pin_base) (void)hipHostFree(pin_base);
    for (auto& st : streams)
      if (st) (void)hipStreamDestroy(st);
  }
  void finish_group(Group& G, int state) {
    for (uint64_t id : G.ids) {
      reqs[id].state = state;
      completed.push_back(id);
    }
    mem.release(G.scratch_at, G.scratch_len);
    pin.release(G.pin_at, G.pin_len);
    ev_free.push_back(G.ev);
    lz_range_plan_free(G.plan);
  }
  // admitted requests back to the front of the queue, arrival order kept
  void requeue(std::vector<uint64_t> ids) {
    std::sort(ids.begin(), ids.end());
    for (auto it = ids.rbegin(); it != ids.rend(); ++it) {
      auto& r = reqs[*it];
      mem.release(r.out_at, r.len);
      --active;
      queue.push_front(r.id);
    }
  }
};

extern "C" {

int lz_serve_create(lz_dev* h, void* d_arena, uint64_t arena_bytes, uint32_t slots, const lz_decode_cfg* cfg,
                    lz_server** out) {
  if (!h || !d_arena || !out || slots == 0) return lz::fail(LZ_E_INVAL, "bad argument");
  lz_server* S = new lz_server();
  S->h = h;
  S->arena = (uint8_t*)d_arena;
  S->arena_bytes = arena_bytes & ~uint64_t(255);
  S->slots = slots;
  if (cfg) S->cfg = *cfg;
  S->mem.reset(S->arena_bytes);
  for (auto& st : S->streams)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      st = nullptr;
      delete S;
      return lz::fail(LZ_E_HIP, "stream creation failed");
    }
  if (hipHostMalloc((void**)&S->pin_base, kPinPoolMin, 0) != hipSuccess) {
    S->pin_base = nullptr;
    delete S;
    return lz::fail(LZ_E_NOMEM, "pinned staging pool allocation failed");
  }
  S->pin_bytes = kPinPoolMin;
  S->pin.reset(S->pin_bytes);
  *out = S;
  return 0;
}

int lz_serve_submit(lz_server* S, uint64_t off, uint64_t len, uint64_t* id) {
  if (!S || !id) return lz::fail(LZ_E_INVAL, "null argument");
  if (off > S->h->v.n || len > S->h->v.n - off) return lz::fail(LZ_E_RANGE, "range outside the archive");
  if (Extents::a256(std::max<uint64_t>(len, 1)) > S->arena_bytes)
    return lz::fail(LZ_E_NOMEM, "request of %llu bytes exceeds the arena", (unsigned long long)len);
  lz_server::Req r;
  r.id = S->reqs.size();
  r.off = off;
  r.len = len;
  S->reqs.push_back(r);
  S->queue.push_back(r.id);
  *id = r.id;
  return 0;
}

// One scheduling step; *n_done receives how many requests finished in it.
int lz_serve_tick(lz_server* S, uint64_t* n_done, uint64_t* n_admitted) {
  if (!S) return lz::fail(LZ_E_INVAL, "null server");
  uint64_t done = 0, admitted = 0;
  if (n_done) *n_done = 0;
  if (n_admitted) *n_admitted = 0;
  // 1. retire finished groups
  int rc_retire = 0;
  for (size_t g = 0; g < S->running.size();) {
    hipError_t q = hipEventQuery(S->running[g].ev);
    if (q == hipErrorNotReady) {
      ++g;
      continue;
    }
    auto& G = S->running[g];
    if (q != hipSuccess) rc_retire = lz::fail(LZ_E_HIP, "group failed: %s", hipGetErrorString(q));
    else done += G.ids.size();
    S->finish_group(G, q == hipSuccess ? 2 : 4);
    S->running.erase(S->running.begin() + g);
  }
  if (n_done) *n_done = done;
  if (rc_retire) return rc_retire;
  // 2. admit in arrival order while a slot and room for the output remain
  std::vector<uint64_t> adm;
  while (!S->queue.empty() && S->active < S->slots) {
    auto& r = S->reqs[S->queue.front()];
    uint64_t at;
    if (!S->mem.alloc(r.len, &at)) break;  // the head waits for memory
    r.out_at = at;
    r.hz = r.len ? decode_horizon(S->h, r.off, r.off + r.len) : 0;
    adm.push_back(r.id);
    S->queue.pop_front();
    ++S->active;
  }
  adm.insert(adm.end(), S->held.begin(), S->held.end());
  S->held.clear();
  if (adm.empty()) return 0;
  std::sort(adm.begin(), adm.end());
  // 3. one group per decode horizon: ranges whose prefix decodes start at the
  // same grain share one plan (on a segment-encoded archive, one segment), so
  // no plan decodes the stretch between far-apart ranges.  A horizon that
  // already has a group on the device holds its requests until that group is
  // done, so they merge into one later group instead of decoding the same
  // prefix beside it.
  std::vector<std::pair<uint64_t, std::vector<uint64_t>>> parts;  // horizon, ids in arrival order
  for (uint64_t id : adm) {
    const uint64_t hz = S->reqs[id].hz;
    bool busy = false;
    for (const auto& G : S->running) busy = busy || G.hz == hz;
    if (busy) {
      S->held.push_back(id);
      continue;
    }
    size_t k = 0;
    while (k < parts.size() && parts[k].first != hz) ++k;
    if (k == parts.size()) parts.push_back({hz, {}});
    parts[k].second.push_back(id);
  }
  // 4. launch the groups in order of their oldest request.  A group whose
  // scratch or staging does not fit first sends every later group back to the
  // queue, then its own newest requests, one at a time, and tries again; what
  // still does not fit waits for running groups to finish.
  auto requeue_from = [&](size_t k) {
    std::vector<uint64_t> back;
    for (size_t j = k; j < parts.size(); ++j) back.insert(back.end(), parts[j].second.begin(), parts[j].second.end());
    parts.resize(k);
    S->requeue(back);
  };
  for (size_t k = 0; k < parts.size(); ++k) {
    std::vector<uint64_t>& ids = parts[k].second;
    for (;;) {
      std::vector<uint64_t> offs, lens;
      for (uint64_t id : ids) {
        offs.push_back(S->reqs[id].off);
        lens.push_back(S->reqs[id].len);
      }
      lz_range_plan* P = nullptr;
      int rc = lz_range_plan_create(S->h, ids.size(), offs.data(), lens.data(), &P);
      if (rc) {
        requeue_from(k);
        S->max_running = std::max<uint64_t>(S->max_running, S->running.size());
        if (n_admitted) *n_admitted = admitted;
        return rc;
      }
      uint64_t sat = 0, pat = 0;
      const bool idle = S->running.empty();
      const bool got_mem = S->mem.alloc(P->scratch_bytes, &sat);
      bool got_pin = got_mem && S->pin.alloc(P->staging_bytes, &pat);
      if (got_mem && !got_pin && idle && Extents::a256(P->staging_bytes) > S->pin_bytes) {
        // the pool is too small for this plan and nothing is in flight: grow it
        // (freeing pinned memory waits for the device, which is idle here)
        (void)hipHostFree(S->pin_base);
        S->pin_base = nullptr;
        const uint64_t nb = std::max(2 * S->pin_bytes, Extents::a256(P->staging_bytes));
        if (hipHostMalloc((void**)&S->pin_base, nb, 0) != hipSuccess) {
          S->pin_base = nullptr;
          S->pin_bytes = 0;
          S->pin.reset(0);
        } else {
          S->pin_bytes = nb;
          S->pin.reset(nb);
        }
        got_pin = S->pin.alloc(P->staging_bytes, &pat);
      }
      if (!got_pin) {
        if (got_mem) S->mem.release(sat, P->scratch_bytes);
        const uint64_t need = Extents::a256(std::max<uint64_t>(lens.back(), 1)) + Extents::a256(P->scratch_bytes);
        lz_range_plan_free(P);
        if (k + 1 < parts.size()) {
          requeue_from(k + 1);
          continue;
        }
        if (ids.size() > 1) {
          S->requeue({ids.back()});
          ids.pop_back();
          continue;
        }
        // a lone request that meets an idle server and still does not fit (its
        // output and scratch exceed the whole arena, or its staging the pool
        // could not grow to) can never be served
        if (idle && (need > S->arena_bytes || got_mem)) {
          auto& r = S->reqs[ids[0]];
          S->mem.release(r.out_at, r.len);
          r.state = 4;  // failed; its slot is held until released
          S->completed.push_back(r.id);
          parts.resize(k);
          S->max_running = std::max<uint64_t>(S->max_running, S->running.size());
          if (n_admitted) *n_admitted = admitted;
          return lz::fail(LZ_E_NOMEM, "request %llu needs %llu bytes of arena (or its staging the pinned pool), "
                          "more than there is", (unsigned long long)ids[0], (unsigned long long)need);
        }
        requeue_from(k);  // waits for a running group to finish
        break;
      }
      P->staging = S->pin_base + pat;
      P->staging_owned = false;
      std::vector<uint64_t> oo;
      for (uint64_t id : ids) oo.push_back(S->reqs[id].out_at);
      hipStream_t st = S->streams[S->next_stream];
      S->next_stream = (S->next_stream + 1) % kServeStreams;
      hipEvent_t ev = nullptr;
      if (!S->ev_free.empty()) {
        ev = S->ev_free.back();
        S->ev_free.pop_back();
      } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
      }
      rc = ev ? lz_range_run(S->h, P, S->arena, S->arena_bytes, oo.data(), S->arena + sat, P->scratch_bytes, &S->cfg, st)
              : lz::fail(LZ_E_HIP, "event creation failed");
      if (rc == 0 && hipEventRecord(ev, st) != hipSuccess) {
        // the work is enqueued but cannot be tracked: wait for it here
        rc = (hipStreamSynchronize(st) == hipSuccess) ? 0 : lz::fail(LZ_E_HIP, "event record and stream sync failed");
        lz_server::Group G{ev, parts[k].first, P, sat, P->scratch_bytes, pat, P->staging_bytes, ids};
        for (uint64_t id : ids) S->reqs[id].state = 1;
        S->finish_group(G, rc == 0 ? 2 : 4);
        admitted += ids.size();
        if (rc) {
          requeue_from(k + 1);
          S->max_running = std::max<uint64_t>(S->max_running, S->running.size());
          if (n_admitted) *n_admitted = admitted;
          return rc;
        }
        break;
      }
      if (rc) {
        // nothing of this group reached the device after a failed launch call;
        // wait for what did, then give everything back
        (void)hipStreamSynchronize(st);
        if (ev) S->ev_free.push_back(ev);
        S->mem.release(sat, P->scratch_bytes);
        S->pin.release(pat, P->staging_bytes);
        lz_range_plan_free(P);
        requeue_from(k);
        S->max_running = std::max<uint64_t>(S->max_running, S->running.size());
        if (n_admitted) *n_admitted = admitted;
        return rc;
      }
      lz_server::Group G{ev, parts[k].first, P, sat, P->scratch_bytes, pat, P->staging_bytes, ids};
      for (uint64_t id : ids) S->reqs[id].state = 1;
      S->running.push_back(std::move(G));
      admitted += ids.size();
      break;
    }
  }
  S->max_running = std::max<uint64_t>(S->max_running, S->running.size());
  if (n_admitted) *n_admitted = admitted;
  return 0;
}

// State of a request: 0 waiting, 1 running, 2 done, 3 released, 4 failed;
// *d_ptr its output when done.
int lz_serve_status(lz_server* S, uint64_t id, int* state, uint8_t** d_ptr) {
  if (!S || id >= S->reqs.size() || !state) return lz::fail(LZ_E_INVAL, "bad request id");
  *state = S->reqs[id].state;
  if (d_ptr) *d_ptr = S->arena + S->reqs[id].out_at;
  return 0;
}

// Frees a done request's output (or the slot of a failed one).
int lz_serve_release(lz_server* S, uint64_t id) {
  if (!S || id >= S->reqs.size() || (S->reqs[id].state != 2 && S->reqs[id].state != 4))
    return lz::fail(LZ_E_INVAL, "request not done");
  if (S->reqs[id].state == 2) S->mem.release(S->reqs[id].out_at, S->reqs[id].len);
  S->reqs[id].state = 3;
  --S->active;
  return 0;
}

uint64_t lz_serve_completed(lz_server* S, uint64_t* ids, uint64_t cap) {
  if (!S || !ids) return 0;
  uint64_t k = 0;
  for (; k < cap && !S->completed.empty(); ++k) {
    ids[k] = S->completed.front();
    S->completed.pop_front();
  }
  return k;
}

void lz_serve_stats(const lz_server* S, uint64_t* waiting, uint64_t* running_groups, uint64_t* arena_used,
                    uint64_t* arena_high_water) {
  if (!S) return;
  if (waiting) *waiting = S->queue.size() + S->held.size();
  if (running_groups) *running_groups = S->running.size();
  if (arena_used) *arena_used = S->mem.used;
  if (arena_high_water) *arena_high_water = S->mem.high_water;
}

uint64_t lz_serve_max_running(const lz_server* S) { return S ? S->max_running : 0; }

int lz_serve_destroy(lz_server* S) {
  if (!S) return 0;
  for (auto& G : S->running) {
    (void)hipEventSynchronize(G.ev);
    S->ev_free.push_back(G.ev);
    lz_range_plan_free(G.plan);
  }
  S->running.clear();
  delete S;
  return 0;
}

}  // extern "C"
