// lz_entropy.hip -- gfx950 decoder of the tile-rANS entropy stage.
//
// One wave64 per tile, one tile per workgroup (Sec. 2: entropy decoded over
// 64 KB tiles by many cooperating groups, tiles cut independently of the LZ
// blocks); the tile's 64 interleaved rANS states live one per lane, so a
// step decodes 64 consecutive symbols and stores them with one byte store of
// the wave.  Per wave, LDS holds the slot -> symbol table (4096 bytes), the
// frequencies and cumulative frequencies (256 + 256 u16) and a ring of
// 2 x 512 words of the tile's word stream, refilled a chunk at a time every
// block of 8 steps at most, so a renormalisation reads LDS; 7 KiB a tile
// lets 22 tiles share a CU.  The lanes that need a word in a step take
// consecutive words in lane order (ballot + popcount of the lower lanes).
// Raw tiles are copied and repeated-byte tiles filled.  Every bound was
// checked on the host; a word read past the payload (possible only on a
// corrupt stream that passed those checks) sets an error bit and stops the
// tile.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lz_internal.h"

// Global-memory accesses go through address-space-1 pointers: flat stores
// would also count against the LDS wait counter, so every step's LDS lookups
// would wait for the previous step's output store.
#define LZ_G __attribute__((address_space(1)))

namespace {

template <typename T>
__device__ __forceinline__ T gld(const uint8_t* p) {
  return *(const LZ_G T*)(p);
}
__device__ __forceinline__ void gst8(uint8_t* p, uint8_t v) { *(LZ_G uint8_t*)(p) = v; }

// BLOCK steps run between ring advances and output stores; a block reads
// at most 64 BLOCK words, so the ring holds two chunks of that many words.
template <int BLOCK>
struct alignas(16) WaveLds {
  static constexpr uint32_t kChunk = 64u * BLOCK, kRing = 2u * kChunk;
  uint8_t sym[lz::kRansM];
  uint32_t fc[256];  // f | c << 16
  uint16_t ring[kRing];
};

__device__ __forceinline__ uint32_t ld_u32_unaligned(const uint8_t* p) {
  return (uint32_t)gld<uint8_t>(p) | ((uint32_t)gld<uint8_t>(p + 1) << 8) | ((uint32_t)gld<uint8_t>(p + 2) << 16) |
         ((uint32_t)gld<uint8_t>(p + 3) << 24);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_a1 __attribute__((ext_vector_type(4), aligned(1)));
typedef unsigned int u32x2_a1 __attribute__((ext_vector_type(2), aligned(1)));

// A ring chunk gives each lane BLOCK words (2 BLOCK bytes).
template <int BLOCK> struct Piece;
template <> struct Piece<8> {
  typedef u32x4 chunk_t;
  typedef u32x4_a1 chunk_a1;
};
template <> struct Piece<4> {
  typedef u32x2 chunk_t;
  typedef u32x2_a1 chunk_a1;
};

// Chunk k of the word stream (words [64 BLOCK k, 64 BLOCK (k + 1)), n words
// in all): lane j holds words BLOCK j .. BLOCK j + BLOCK - 1 of it; past the
// end, zeros.  The load is issued a block before its bytes are written to
// the ring.
template <int BLOCK>
__device__ __forceinline__ typename Piece<BLOCK>::chunk_t fetch_chunk(const uint8_t* words, uint64_t n, uint64_t k,
                                                                      int lane) {
  typedef typename Piece<BLOCK>::chunk_t C;
  const uint64_t w0 = k * (64u * BLOCK) + BLOCK * (uint64_t)lane;
  if (w0 + BLOCK <= n) return *(const LZ_G typename Piece<BLOCK>::chunk_a1*)(words + 2 * w0);
  uint32_t d[BLOCK / 2] = {};
  for (uint64_t q = 0; w0 < n && q < 2 * (n - w0); ++q) d[q >> 2] |= (uint32_t)gld<uint8_t>(words + 2 * w0 + q) << (8 * (q & 3));
  C v;
#pragma unroll
  for (int i = 0; i < BLOCK / 2; ++i) v[i] = d[i];
  return v;
}

template <int BLOCK>
__device__ __forceinline__ void put_chunk(WaveLds<BLOCK>& L, uint64_t k, typename Piece<BLOCK>::chunk_t v, int lane) {
  ((typename Piece<BLOCK>::chunk_t*)(L.ring + (k & 1) * WaveLds<BLOCK>::kChunk))[lane] = v;
}

// tiles per workgroup and steps per block of the launched kernel
constexpr int kEntWaves = 1, kEntBlock = 8;

template <int WAVES, int BLOCK>
__global__ __launch_bounds__(64 * WAVES) void k_entropy(const uint8_t* coded, uint64_t payload_off, uint64_t n_tiles,
                                                        uint8_t* out, uint32_t* err) {
  typedef WaveLds<BLOCK> Lds;
  constexpr uint32_t kBlock = BLOCK, kChunk = Lds::kChunk, kRing = Lds::kRing;
  __shared__ Lds lds[WAVES];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Lds& L = lds[wv];
  const uint64_t nwaves = (uint64_t)gridDim.x * WAVES;
  for (uint64_t t = (uint64_t)blockIdx.x * WAVES + wv; t < n_tiles; t += nwaves) {
    const uint8_t* r = coded + lz::kCodedHead + 32 * t;  // directory record
    const uint64_t po = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r)) |
                        ((uint64_t)__builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 4)) << 32);
    const uint64_t dst = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 8)) |
                         ((uint64_t)__builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 12)) << 32);
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 16));
    const uint32_t pb = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 20));
    const uint32_t stride = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 24));
    const uint32_t mode = __builtin_amdgcn_readfirstlane(ld_u32_unaligned(r + 28));
    const uint8_t* p = coded + payload_off + po;
    uint8_t* o = out + dst;
    if (mode == 2) {
      const uint8_t v = gld<uint8_t>(p);
#pragma clang loop vectorize(disable) unroll(disable)
      for (uint32_t i = lane; i < cnt; i += 64) gst8(o + (uint64_t)i * stride, v);
      continue;
    }
    if (mode == 0) {
#pragma clang loop vectorize(disable) unroll(disable)
      for (uint32_t i = lane; i < cnt; i += 64) gst8(o + (uint64_t)i * stride, gld<uint8_t>(p + i));
      continue;
    }
    // frequencies: symbol s present <=> bit s of the bitmap; its f is the
    // (number of present symbols below s)-th u16 after the bitmap
    uint32_t below = 0;  // present symbols below this lane's group of 64
    for (int g = 0; g < 4; ++g) {
      const int s = g * 64 + lane;
      const uint64_t bits = ((uint64_t)ld_u32_unaligned(p + 8 * g + 4) << 32) | ld_u32_unaligned(p + 8 * g);
      const bool present = (bits >> lane) & 1;
      const uint32_t idx = below + __builtin_popcountll(bits & ((1ull << lane) - 1));
      L.fc[s] = present ? (uint32_t)(gld<uint8_t>(p + 32 + 2 * idx) | (gld<uint8_t>(p + 33 + 2 * idx) << 8)) : 0u;
      below += __builtin_popcountll(bits);
    }
    const uint32_t nsym = below;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // cumulative frequencies: 4 groups of 64, each a wave prefix sum
    uint32_t run = 0;
    for (int g = 0; g < 4; ++g) {
      uint32_t v = L.fc[g * 64 + lane], x = v;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      L.fc[g * 64 + lane] = v | ((run + x - v) << 16);
      run += __shfl(x, 63, 64);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // slot -> symbol: mark the first slot of every present symbol above 0
    // with the symbol, then take the running maximum over the slots (symbols
    // start in increasing order, and symbol 0, when present, starts at 0)
    {
      u32x4* row = (u32x4*)L.sym + 4 * lane;  // this lane's 64 slots
      const u32x4 z = {0u, 0u, 0u, 0u};
      row[0] = z;
      row[1] = z;
      row[2] = z;
      row[3] = z;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int g = 0; g < 4; ++g) {
        const int s = g * 64 + lane;
        const uint32_t v = L.fc[s];
        if (s > 0 && (v & 0xFFFFu)) L.sym[v >> 16] = (uint8_t)s;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // the largest symbol starting in each lane's 64 slots, by LDS atomics
      // into a scratch row of the (not yet filled) word ring
      uint32_t* rowmax = (uint32_t*)L.ring;
      rowmax[lane] = 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int g = 0; g < 4; ++g) {
        const int s = g * 64 + lane;
        const uint32_t v = L.fc[s];
        if (s > 0 && (v & 0xFFFFu)) atomicMax(rowmax + (v >> 22), (uint32_t)s);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const uint32_t mx = rowmax[lane];
      // maximum over the lanes below: an exclusive max-scan of the lane maxima
      uint32_t inc = mx;
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc = max(inc, y);
      }
      uint32_t run = __shfl_up(inc, 1, 64);
      if (lane == 0) run = 0;
#pragma unroll 1
      for (int q = 0; q < 4; ++q) {
        u32x4 w = row[q];
        for (int e = 0; e < 4; ++e) {
          uint32_t o = 0;
          for (int b = 0; b < 4; ++b) {
            run = max(run, (w[e] >> (8 * b)) & 0xFFu);
            o |= run << (8 * b);
          }
          w[e] = o;
        }
        row[q] = w;
      }
    }
    // states, and the word stream into the ring
    const uint8_t* st = p + 32 + 2 * nsym;
    uint32_t x = ld_u32_unaligned(st + 4 * lane);
    const uint8_t* words = st + 4 * lz::kRansLanes;
    const uint64_t nwords = (pb - (32 + 2 * nsym + 4 * lz::kRansLanes)) / 2;
    put_chunk(L, 0, fetch_chunk<BLOCK>(words, nwords, 0, lane), lane);
    put_chunk(L, 1, fetch_chunk<BLOCK>(words, nwords, 1, lane), lane);
    auto ahead = fetch_chunk<BLOCK>(words, nwords, 2, lane);  // in flight until the ring next advances
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t wpos = 0, chunk = 0;
    // one step: state `lane` decodes symbol 64 k + lane (when below cnt);
    // the states that fell below 2^16 take the next words in lane order.
    // Branch-free: every lane reads the table and a ring word (in bounds),
    // selects keep what an inactive lane or a lane without renormalisation
    // must not change.
    auto step = [&](bool act) -> uint32_t {
      const uint32_t slot = x & (lz::kRansM - 1);
      const uint32_t sv = L.sym[slot];
      const uint32_t fcv = L.fc[sv];
      uint32_t nx = (fcv & 0xFFFFu) * (x >> 12) + slot - (fcv >> 16);
      nx = act ? nx : x;
      const bool need = act && nx < lz::kRansL;
      const uint64_t m = __ballot(need);
      const uint32_t pos = wpos + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      uint32_t w = L.ring[pos & (kRing - 1)];
      asm volatile("" : "+v"(w));  // keeps the read unconditional (no branch around it)
      x = need ? ((nx << 16) | w) : nx;
      wpos += (uint32_t)__builtin_popcountll(m);
      return sv;
    };
    const uint32_t steps = (cnt + 63) / 64;
    for (uint32_t k0 = 0; k0 < steps; k0 += kBlock) {
      // a block reads at most kChunk words: the ring (chunks `chunk`, +1)
      // covers it after at most one advance; `ahead` was loaded at least a
      // block ago
      if (wpos / kChunk > chunk) {
        __builtin_amdgcn_wave_barrier();
        ++chunk;
        put_chunk(L, chunk + 1, ahead, lane);
        ahead = fetch_chunk<BLOCK>(words, nwords, chunk + 2, lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      // every step stores its 64 symbols, consecutive in the output for
      // stride-1 tiles (one 64-byte store of the wave)
      if (k0 + kBlock < steps) {  // a whole block of full steps (not the last step)
#pragma unroll
        for (int u = 0; u < (int)kBlock; ++u)
          gst8(o + (uint64_t)((k0 + u) * 64 + lane) * stride, (uint8_t)step(true));
      } else {
#pragma unroll
        for (int u = 0; u < (int)kBlock; ++u) {
          if (k0 + u >= steps) break;
          const uint32_t i = (k0 + u) * 64 + lane;
          const uint8_t v = (uint8_t)step(i < cnt);
          if (i < cnt) gst8(o + (uint64_t)i * stride, v);
        }
      }
    }
    // words past the stream read as zero, so a corrupt stream decodes to
    // garbage but stays in bounds; it is caught here: every word consumed,
    // and every state back at the encoder's start (2^16)
    const bool short_words = wpos != nwords;
    const bool off_end = __any(x != lz::kRansL);
    if (lane == 0 && (short_words || off_end)) atomicOr(err, short_words ? 1u : 2u);
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

namespace lz {

int entropy_launch(const uint8_t* d_coded, uint64_t payload_off, uint64_t n_tiles, uint8_t* d_out, uint32_t* d_err,
                   int cu_count, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (n_tiles == 0) return 0;
  constexpr int W = kEntWaves;
  const void* k = (const void*)k_entropy<kEntWaves, kEntBlock>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64 * W, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const uint64_t groups = std::min<uint64_t>((n_tiles + W - 1) / W, (uint64_t)per_cu * std::max(cu_count, 1));
  hipLaunchKernelGGL((k_entropy<kEntWaves, kEntBlock>), dim3((unsigned)groups), dim3(64 * W), 0, s, d_coded,
                     payload_off, n_tiles, d_out, d_err);
  if (hipGetLastError() != hipSuccess) return fail(LZ_E_HIP, "entropy launch failed");
  return 0;
}

}  // namespace lz
