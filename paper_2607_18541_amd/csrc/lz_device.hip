// lz_device.hip -- gfx950 match-phase decoder of absolute-offset LZ77.
//
// One LZ block is decoded by a group of G lanes of a 64-lane wave (Sec. 2:
// cooperation width G; Sec. 3.1: lanes = G x N_blocks).  A group works through
// its block in token order:
//   1. parse: each lane reads one token header (cmd byte, length extensions,
//      absolute source); group prefix sums give every token's output position
//      and literal offset, so G tokens are parsed per step;
//   2. batch: the group's pending segments (literal runs and match pieces) are
//      cut into batches whose sources lie entirely before the batch's first
//      output byte, so a batch has no read-after-write inside it; a match whose
//      source overlaps its own output (period d = dst - src < length) runs as
//      pieces of length d, 2d, 4d, ... each reading the already final prefix;
//   3. copy: a batch's output is covered by 16-byte aligned output chunks,
//      spread over the group's lanes (`unroll` chunks per lane per step).  A
//      lane loads the 16 source bytes of its chunk with one unaligned 16-byte
//      load and writes a full chunk with one aligned 16-byte store; the two
//      chunks at each segment edge are written with exact byte/short/dword/
//      qword stores so neighbouring segments never race on a byte.
// Schedules.  Cross-block sources (absolute offsets reach the whole prefix)
// need the source block final first.  Schedule 0: one launch; groups claim
// blocks in increasing order from an atomic ticket, publish a per-block
// completion flag with an agent-scope release, and wait (bounded) on the flags
// of the blocks a batch reads.  Claims are in order, so the lowest unfinished
// claimed block depends only on finished blocks and always progresses.
// Schedule 1: one launch per dependency level, each group executing only the
// level-p matches of its block (literals in pass 0); kernel boundaries order
// the levels.  Mode 2 runs pre-decoded tokens whose sources are in a separate
// buffer (the pure-copy control of Sec. 3.3).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "lz_internal.h"

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kModeFlags = 0;
constexpr int kModeLevels = 1;
constexpr int kModePure = 2;

constexpr uint64_t kIdleTicks = 500000000ull;  // 5 s of the 100 MHz clock without progress
constexpr int kWG = 256;

struct KArgs {
  // archive streams (device)
  const uint64_t* tab;
  const uint8_t* cmd;
  const uint16_t* x16;
  const uint32_t* x32;
  const uint32_t* slo;
  const uint8_t* shi;
  const uint8_t* lit;
  uintptr_t lit_lo, lit_hi;  // readable bounds for literal windows
  uint64_t n;
  uint32_t log2_bs, nb, min_match;
  // output and match-source bounds
  uint8_t* out;
  const uint8_t* msrc;  // base that match sources index (out, or ref in mode 2)
  uintptr_t msrc_lo, msrc_hi;
  // schedule 0
  uint32_t* flags;
  uint32_t* ticket;
  uint32_t* err;
  // schedule 1
  const uint16_t* lvl;
  const uint16_t* blk_maxlvl;
  uint32_t pass;
  // mode 2 (pre-decoded tokens)
  const uint64_t* p_dst;
  const uint64_t* p_lit_off;
  const uint32_t* p_lit_len;
  const uint64_t* p_src;
  const uint32_t* p_mlen;
  const uint64_t* p_unit;
  uint64_t nunits;
};

struct Desc {
  uintptr_t a_dst, a_src, b_dst, b_src;
  uint32_t a_len, b_len, base, ca;
};

template <int G>
__device__ __forceinline__ uint64_t gscan64(uint64_t v, int gl, uint64_t& total) {
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    uint64_t y = __shfl_up(x, d, G);
    if (gl >= d) x += y;
  }
  total = __shfl(x, G - 1, G);
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
  total = __shfl(x, G - 1, G);
  return x - v;
}

// bits of this lane's group in a wave-wide ballot
template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int gw) {
  if (G == 64) return ballot;
  return (ballot >> (gw * G)) & ((1ull << G) - 1);
}

__device__ __forceinline__ uint32_t nchunks(uintptr_t d, uint32_t len) {
  return len ? (uint32_t)(((d + len + 15) >> 4) - (d >> 4)) : 0u;
}

// 16 source bytes of a window; out-of-range windows fall back to the needed bytes
__device__ __forceinline__ u32x4 load_window(uintptr_t w, uintptr_t lo_b, uintptr_t hi_b, int lo, int hi) {
  u32x4 v;
  if (w >= lo_b && w + 16 <= hi_b) {
    __builtin_memcpy(&v, (const void*)w, 16);
  } else {
    uint32_t d[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i >= lo && i < hi) d[i >> 2] |= uint32_t(*(const uint8_t*)(w + i)) << (8 * (i & 3));
    v = u32x4{d[0], d[1], d[2], d[3]};
  }
  return v;
}

__device__ __forceinline__ uint32_t dword_at(const u32x4& v, int i) {  // i = dword index 0..3
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// Writes bytes [lo, hi) of a 16-byte aligned chunk at a with naturally aligned
// stores only (no read-modify-write of bytes outside the range).
__device__ __forceinline__ void store_chunk(uintptr_t a, const u32x4& v, int lo, int hi) {
  if (lo == 0 && hi == 16) {
    *(u32x4*)a = v;
    return;
  }
  int i = lo;
  if ((i & 1) && i < hi) {
    *(uint8_t*)(a + i) = (uint8_t)(dword_at(v, i >> 2) >> (8 * (i & 3)));
    i += 1;
  }
  if ((i & 2) && i + 2 <= hi) {
    *(uint16_t*)(a + i) = (uint16_t)(dword_at(v, i >> 2) >> (8 * (i & 3)));
    i += 2;
  }
  if ((i & 4) && i + 4 <= hi) {
    *(uint32_t*)(a + i) = dword_at(v, i >> 2);
    i += 4;
  }
  if ((i & 8) && i + 8 <= hi) {
    uint64_t q = (uint64_t)dword_at(v, i >> 2) | ((uint64_t)dword_at(v, (i >> 2) + 1) << 32);
    *(uint64_t*)(a + i) = q;
    i += 8;
  }
  if (i + 8 <= hi) {
    uint64_t q = (uint64_t)dword_at(v, i >> 2) | ((uint64_t)dword_at(v, (i >> 2) + 1) << 32);
    *(uint64_t*)(a + i) = q;
    i += 8;
  }
  if (i + 4 <= hi) {
    *(uint32_t*)(a + i) = dword_at(v, i >> 2);
    i += 4;
  }
  if (i + 2 <= hi) {
    *(uint16_t*)(a + i) = (uint16_t)(dword_at(v, i >> 2) >> (8 * (i & 3)));
    i += 2;
  }
  if (i + 1 <= hi) {
    *(uint8_t*)(a + i) = (uint8_t)(dword_at(v, i >> 2) >> (8 * (i & 3)));
  }
}

__device__ __forceinline__ void lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

template <int G, int U, int MODE>
__global__ __launch_bounds__(kWG) void k_lz(KArgs A) {
  static_assert(G == 8 || G == 16 || G == 32 || G == 64, "G");
  __shared__ Desc s_desc[kWG];
  __shared__ uint32_t s_base[kWG];

  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);     // lane in group
  const int gw = lane / G;           // group in wave
  const int gslot = threadIdx.x - gl;  // first LDS slot of this group
  const uint64_t ngroups = (uint64_t)gridDim.x * (kWG / G);
  const uint64_t gid = (uint64_t)blockIdx.x * (kWG / G) + threadIdx.x / G;
  const uint64_t bs = 1ull << A.log2_bs;

  // group state (replicated on the group's lanes)
  bool finished = false, have_blk = false;
  uint64_t blk = 0, unit_iter = 0;
  uint64_t t_next = 0, t_end = 0, pos = 0, bend = 0, litc = 0, xc = 0, yc = 0;
  uint64_t wm = 0;  // blocks below wm are known complete (schedule 0)
  // this lane's buffered token
  uint64_t l_dst = 0, l_src = 0, m_dst = 0, m_src = 0;
  uint32_t l_len = 0, m_len = 0, m_done = 0;
  bool l_pend = false;
  uint32_t idle = 0;
  uint64_t t_last = 0;

  for (;;) {
    // ---------------------------------------------------- claim a block
    if (!finished && !have_blk) {
      if (MODE == kModeFlags) {
        uint32_t b = 0;
        if (gl == 0) b = atomicAdd(A.ticket, 1u);
        b = __shfl(b, 0, G);
        if (b >= A.nb) {
          finished = true;
        } else {
          blk = b;
          have_blk = true;
        }
      } else if (MODE == kModeLevels) {
        // grid-stride over blocks that have work in this pass
        for (;;) {
          uint64_t b = gid + unit_iter * ngroups;
          if (b >= A.nb) {
            finished = true;
            break;
          }
          ++unit_iter;
          if (A.blk_maxlvl[b] >= A.pass) {
            blk = b;
            have_blk = true;
            break;
          }
        }
      } else {
        uint64_t u = gid + unit_iter * ngroups;
        ++unit_iter;
        if (u >= A.nunits) {
          finished = true;
        } else {
          blk = u;
          have_blk = true;
        }
      }
      if (have_blk) {
        if (MODE == kModePure) {
          t_next = A.p_unit[blk];
          t_end = A.p_unit[blk + 1];
        } else {
          const uint64_t* e = A.tab + 4 * blk;
          t_next = e[0];
          t_end = e[4];
          litc = e[1];
          xc = e[2];
          yc = e[3];
          pos = blk * bs;
          bend = min(A.n, pos + bs);
        }
        l_len = m_len = m_done = 0;
        l_pend = false;
      }
    }
    if (__all(finished)) break;

    bool progressed = false;
    if (have_blk) {
      // ------------------------------------------------ anything pending?
      const uint32_t m_rem = m_len - m_done;
      const bool lane_pend = l_pend || (m_rem > 0);
      const uint64_t pend_bits = group_bits<G>(__ballot(lane_pend), gw);
      if (pend_bits == 0) {
        if (t_next >= t_end) {
          // ---------------------------------------------- block complete
          if (MODE == kModeFlags) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (gl == 0) __hip_atomic_store(A.flags + blk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          have_blk = false;
          progressed = true;
        } else {
          // ---------------------------------------------- parse G tokens
          const uint64_t t = t_next + gl;
          const bool valid = t < t_end;
          if (MODE == kModePure) {
            l_dst = valid ? A.p_dst[t] : 0;
            l_len = valid ? A.p_lit_len[t] : 0u;
            l_src = valid ? A.p_lit_off[t] : 0;
            m_len = valid ? A.p_mlen[t] : 0u;
            m_src = valid ? A.p_src[t] : 0;
            m_dst = l_dst + l_len;
          } else {
            const uint32_t c = valid ? A.cmd[t] : 0u;
            const bool last = (t + 1 == t_end);
            const uint32_t Lc = c >> 4, Mc = c & 15u;
            const uint32_t need_l = (valid && Lc == 15u) ? 1u : 0u;
            const uint32_t need_m = (valid && !last && Mc == 15u) ? 1u : 0u;
            uint32_t tot16;
            const uint64_t i16 = xc + gscan32<G>(need_l + need_m, gl, tot16);
            uint32_t e_l = need_l ? A.x16[i16] : 0u;
            uint32_t e_m = need_m ? A.x16[i16 + need_l] : 0u;
            const uint32_t w_l = (need_l && e_l == 0xFFFFu) ? 1u : 0u;
            const uint32_t w_m = (need_m && e_m == 0xFFFFu) ? 1u : 0u;
            uint32_t tot32;
            const uint64_t i32 = yc + gscan32<G>(w_l + w_m, gl, tot32);
            if (w_l) e_l += A.x32[i32];
            if (w_m) e_m += A.x32[i32 + w_l];
            const uint32_t lit_len = (Lc == 15u) ? 15u + e_l : Lc;
            uint32_t mlen = (valid && !last) ? A.min_match + ((Mc == 15u) ? 15u + e_m : Mc) : 0u;
            uint64_t src = valid ? (uint64_t)A.slo[t] : 0;
            if (A.shi && valid) src |= (uint64_t)A.shi[t] << 32;
            uint64_t lit_tot;
            const uint64_t loff = litc + gscan64<G>(lit_len, gl, lit_tot);
            uint64_t span_tot;
            const uint64_t tdst = pos + gscan64<G>((uint64_t)lit_len + mlen, gl, span_tot);
            if (valid && last) mlen = (uint32_t)(bend - (tdst + lit_len));
            xc += tot16;
            yc += tot32;
            litc += lit_tot;
            pos += span_tot;
            l_dst = tdst;
            l_len = lit_len;
            l_src = loff;
            m_dst = tdst + lit_len;
            m_len = mlen;
            m_src = src;
            if (MODE == kModeLevels) {
              const uint32_t lv = valid ? A.lvl[t] : 0u;
              if (A.pass != 0) l_len = 0;
              if (lv != A.pass) m_len = 0;
            }
          }
          const uint64_t cnt = min((uint64_t)G, t_end - t_next);
          t_next += cnt;
          m_done = 0;
          l_pend = l_len > 0;
          progressed = true;
        }
      } else {
        // ------------------------------------------------ form a batch
        const int first = __builtin_ctzll(pend_bits);
        const uint64_t my_next = l_pend ? l_dst : (m_dst + m_done);
        const uint64_t batch_start = __shfl(my_next, first, G);
        const uint32_t piece = m_rem ? min(m_rem, (uint32_t)(m_dst - m_src) + m_done) : 0u;
        const uint64_t src_end = m_src + piece;
        bool hz = false;
        if (MODE != kModePure) hz = piece > 0 && src_end > batch_start;
        const uint64_t hz_bits = group_bits<G>(__ballot(hz), gw);
        const int h = hz_bits ? __builtin_ctzll(hz_bits) : G;
        const bool inc_l = l_pend && gl <= h;
        const bool inc_m = piece > 0 && gl < h;

        // ------------------------------------------------ cross-block waits
        bool ready = true;
        if (MODE == kModeFlags) {
          const uint64_t sb0 = m_src >> A.log2_bs;
          uint64_t sb1 = inc_m ? ((src_end - 1) >> A.log2_bs) : 0;
          if (sb1 >= blk) sb1 = blk - 1;  // own block's bytes are ordered by the wave
          const bool needs = inc_m && sb0 < blk && sb1 >= wm;
          const uint64_t need_bits = group_bits<G>(__ballot(needs), gw);
          if (need_bits) {
            if (needs) {
              bool ok = true;
              for (uint64_t b = max(sb0, wm); b <= sb1; ++b)
                ok = ok && (__hip_atomic_load(A.flags + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u);
              ready = ok;
            }
            // advance the watermark over the next G blocks
            const uint64_t wb = wm + gl;
            const bool wdone =
                wb < blk && __hip_atomic_load(A.flags + wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
            const uint64_t wbits = group_bits<G>(__ballot(wdone), gw);
            const uint64_t run = (~wbits == 0ull) ? 64ull : (uint64_t)__builtin_ctzll(~wbits);
            wm += min(run, (uint64_t)G);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ready = group_bits<G>(__ballot(!ready), gw) == 0;
          }
        }

        if (ready) {
          // ---------------------------------------------- chunk the batch
          const uintptr_t out_b = (uintptr_t)A.out;
          const uintptr_t a_dst = out_b + l_dst;
          const uintptr_t b_dst = out_b + m_dst + m_done;
          const uint32_t ca = inc_l ? nchunks(a_dst, l_len) : 0u;
          const uint32_t cb = inc_m ? nchunks(b_dst, piece) : 0u;
          uint32_t C;
          const uint32_t base = gscan32<G>(ca + cb, gl, C);
          Desc d;
          d.a_dst = a_dst;
          d.a_src = (uintptr_t)A.lit + l_src;
          d.a_len = inc_l ? l_len : 0u;
          d.b_dst = b_dst;
          d.b_src = (uintptr_t)A.msrc + m_src;
          d.b_len = inc_m ? piece : 0u;
          d.base = base;
          d.ca = ca;
          s_desc[threadIdx.x] = d;
          s_base[threadIdx.x] = base;
          lds_order();
          for (uint32_t r = 0; r < C; r += G * U) {
            u32x4 v[U];
            uintptr_t slot[U];
            int lo[U], hi[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
              const uint32_t k = r + i * G + gl;
              lo[i] = 0;
              hi[i] = 0;
              slot[i] = 0;
              if (k < C) {
                int a = 0, b = G;
                while (b - a > 1) {
                  const int mid = (a + b) >> 1;
                  if (s_base[gslot + mid] <= k) a = mid; else b = mid;
                }
                const Desc& e = s_desc[gslot + a];
                const uint32_t q = k - e.base;
                uintptr_t D, S, lb, hb;
                uint32_t L, qq;
                if (q < e.ca) {
                  D = e.a_dst; S = e.a_src; L = e.a_len; qq = q;
                  lb = A.lit_lo; hb = A.lit_hi;
                } else {
                  D = e.b_dst; S = e.b_src; L = e.b_len; qq = q - e.ca;
                  lb = A.msrc_lo; hb = A.msrc_hi;
                }
                const uintptr_t s0 = (D & ~(uintptr_t)15) + 16 * (uintptr_t)qq;
                const intptr_t l0 = (intptr_t)D - (intptr_t)s0;
                const intptr_t h0 = (intptr_t)(D + L) - (intptr_t)s0;
                lo[i] = l0 > 0 ? (int)l0 : 0;
                hi[i] = h0 < 16 ? (int)h0 : 16;
                slot[i] = s0;
                v[i] = load_window(S + (s0 - D), lb, hb, lo[i], hi[i]);
              }
            }
#pragma unroll
            for (int i = 0; i < U; ++i)
              if (hi[i] > lo[i]) store_chunk(slot[i], v[i], lo[i], hi[i]);
          }
          lds_order();
          // ---------------------------------------------- retire segments
          if (inc_l) l_pend = false;
          if (inc_m) m_done += piece;
          progressed = true;
        }
      }
    }
    // -------------------------------------------------------- idle guard
    if (MODE == kModeFlags) {
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

__global__ void k_fill_u32(uint32_t* p, uint64_t count, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < count; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace

// ------------------------------------------------------------------ host side

struct lz_dev {
  lz::ArcView v;           // host view (base pointer is NOT kept valid)
  uint8_t* d_arc = nullptr;
  uint32_t* d_flags = nullptr;
  uint32_t* d_ctrl = nullptr;  // [0] ticket, [1] err
  uint16_t* d_lvl = nullptr;
  uint16_t* d_bmax = nullptr;
  uint32_t levels = 0;     // max level + 1 when the plan is present
  bool has_plan = false;
  int cu_count = 0;
};

namespace {

struct DevLayout {
  uint64_t arc, flags, ctrl, lvl, bmax, total;
};

DevLayout layout(const lz::ArcView& v, bool plan) {
  auto a256 = [](uint64_t x) { return (x + 255) & ~uint64_t(255); };
  DevLayout L;
  L.arc = 0;
  L.flags = a256(v.total);
  L.ctrl = a256(L.flags + 4 * (v.nb + 1));
  L.lvl = a256(L.ctrl + 256);
  L.bmax = plan ? a256(L.lvl + 2 * v.n_tok) : L.lvl;
  L.total = plan ? a256(L.bmax + 2 * (v.nb + 1)) : L.lvl;
  return L;
}

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) return lz::fail(LZ_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

KArgs base_args(const lz_dev* h) {
  KArgs A;
  memset(&A, 0, sizeof(A));
  const lz::ArcView& v = h->v;
  A.tab = (const uint64_t*)(h->d_arc + v.off_tab);
  A.cmd = h->d_arc + v.off_cmd;
  A.x16 = (const uint16_t*)(h->d_arc + v.off_x16);
  A.x32 = (const uint32_t*)(h->d_arc + v.off_x32);
  A.slo = (const uint32_t*)(h->d_arc + v.off_slo);
  A.shi = (v.flags & 1) ? h->d_arc + v.off_shi : nullptr;
  A.lit = h->d_arc + v.off_lit;
  A.lit_lo = (uintptr_t)h->d_arc;
  A.lit_hi = (uintptr_t)h->d_arc + v.total;
  A.n = v.n;
  A.log2_bs = v.log2_bs;
  A.nb = (uint32_t)v.nb;
  A.min_match = (uint32_t)v.min_match;
  A.flags = h->d_flags;
  A.ticket = h->d_ctrl;
  A.err = h->d_ctrl + 1;
  A.lvl = h->d_lvl;
  A.blk_maxlvl = h->d_bmax;
  return A;
}

typedef void (*kfn_t)(KArgs);

template <int MODE>
kfn_t pick_kernel(uint32_t G, uint32_t U) {
#define K(g, u) \
  if (G == g && U == u) return k_lz<g, u, MODE>;
  K(8, 1) K(8, 2) K(8, 4) K(16, 1) K(16, 2) K(16, 4) K(32, 1) K(32, 2) K(32, 4) K(64, 1) K(64, 2) K(64, 4)
#undef K
  return nullptr;
}

int resolve_cfg(const lz_decode_cfg* cfg, uint32_t& G, uint32_t& U, uint32_t& sched) {
  G = cfg ? cfg->G : 32;
  U = cfg ? cfg->unroll : 2;
  sched = cfg ? cfg->schedule : 0;
  if (cfg && cfg->wg_size && cfg->wg_size != 256) return lz::fail(LZ_E_INVAL, "wg_size must be 0 or 256");
  if (!(G == 8 || G == 16 || G == 32 || G == 64)) return lz::fail(LZ_E_INVAL, "G must be 8, 16, 32 or 64");
  if (!(U == 1 || U == 2 || U == 4)) return lz::fail(LZ_E_INVAL, "unroll must be 1, 2 or 4");
  if (sched > 1) return lz::fail(LZ_E_INVAL, "schedule must be 0 or 1");
  return 0;
}

int resident_groups(kfn_t k, int cu_count, uint32_t G) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k, kWG, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return per_cu * cu_count * (kWG / (int)G);
}

}  // namespace

extern "C" {

int lz_device_bytes(const uint8_t* arc, uint64_t arc_size, uint64_t* bytes) {
  if (!bytes) return lz::fail(LZ_E_INVAL, "null output");
  lz::ArcView v;
  int rc = lz::view_archive(arc, arc_size, &v);
  if (rc) return rc;
  *bytes = layout(v, true).total;
  return 0;
}

int lz_device_open(const uint8_t* arc, uint64_t arc_size, void* d_buf, uint64_t d_cap, void* stream, lz_dev** out) {
  if (!out || !d_buf) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  lz::ArcView v;
  int rc = lz::view_archive(arc, arc_size, &v);
  if (rc) return rc;
  rc = lz::validate_archive(v, 0);
  if (rc) return rc;
  if (v.nb > 0xFFFFFFF0ull) return lz::fail(LZ_E_INVAL, "too many blocks");
  DevLayout L = layout(v, true);
  if (d_cap < L.total)
    return lz::fail(LZ_E_NOMEM, "device buffer %llu < %llu bytes", (unsigned long long)d_cap,
                    (unsigned long long)L.total);
  // dependency levels for schedule 1 (host sweep)
  std::vector<uint32_t> lv(v.n_tok + 1);
  uint32_t mx = 0;
  rc = lz::compute_levels(v, lv.data(), &mx);
  if (rc) return rc;
  lz_dev* h = new lz_dev();
  h->v = v;
  h->v.base = nullptr;
  uint8_t* base = (uint8_t*)d_buf;
  h->d_arc = base + L.arc;
  h->d_flags = (uint32_t*)(base + L.flags);
  h->d_ctrl = (uint32_t*)(base + L.ctrl);
  h->d_lvl = (uint16_t*)(base + L.lvl);
  h->d_bmax = (uint16_t*)(base + L.bmax);
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
  if (mx < 65535) {
    // u16 levels and per-block maxima, staged through pinned memory
    uint64_t nbytes = 2 * (v.n_tok + 1) + 2 * (v.nb + 1);
    uint16_t* hp = nullptr;
    if (hipHostMalloc((void**)&hp, nbytes, 0) != hipSuccess) {
      delete h;
      return lz::fail(LZ_E_NOMEM, "pinned staging allocation failed");
    }
    uint16_t* bm = hp + (v.n_tok + 1);
    for (uint64_t b = 0; b <= v.nb; ++b) bm[b] = 0;
    const uint64_t* T = v.tab();
    for (uint64_t b = 0; b < v.nb; ++b)
      for (uint64_t t = T[4 * b]; t < T[4 * b + 4]; ++t) {
        hp[t] = (uint16_t)lv[t];
        bm[b] = std::max<uint16_t>(bm[b], (uint16_t)lv[t]);
      }
    hipError_t e1 = hipMemcpyAsync(h->d_lvl, hp, 2 * (v.n_tok + 1), hipMemcpyHostToDevice, s);
    hipError_t e2 = hipMemcpyAsync(h->d_bmax, bm, 2 * (v.nb + 1), hipMemcpyHostToDevice, s);
    hipError_t e3 = hipStreamSynchronize(s);
    hipHostFree(hp);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
      delete h;
      return lz::fail(LZ_E_HIP, "plan upload failed");
    }
    h->has_plan = true;
    h->levels = mx + 1;
  }
  if (hipMemcpyAsync(h->d_arc, arc, v.total, hipMemcpyHostToDevice, s) != hipSuccess) {
    delete h;
    return lz::fail(LZ_E_HIP, "archive upload failed");
  }
  if (hipStreamSynchronize(s) != hipSuccess) {
    delete h;
    return lz::fail(LZ_E_HIP, "archive upload failed");
  }
  *out = h;
  return 0;
}

uint64_t lz_device_n(const lz_dev* h) { return h ? h->v.n : 0; }
uint32_t lz_device_levels(const lz_dev* h) { return h ? h->levels : 0; }
void lz_device_close(lz_dev* h) { delete h; }

int lz_decode_device(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, void* stream) {
  if (!h) return lz::fail(LZ_E_INVAL, "null handle");
  if (out_cap < h->v.n) return lz::fail(LZ_E_INVAL, "output capacity %llu < n %llu", (unsigned long long)out_cap,
                                        (unsigned long long)h->v.n);
  if (h->v.n && !d_out) return lz::fail(LZ_E_INVAL, "null output");
  uint32_t G, U, sched;
  int rc = resolve_cfg(cfg, G, U, sched);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  KArgs A = base_args(h);
  A.out = d_out;
  A.msrc = d_out;
  A.msrc_lo = (uintptr_t)d_out;
  A.msrc_hi = (uintptr_t)d_out + out_cap;
  // clear flags, ticket and error word (a fill kernel, also safe under capture)
  uint64_t clear = ((uint64_t)((uint8_t*)h->d_ctrl - (uint8_t*)h->d_flags)) / 4 + 2;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<uint64_t>((clear + 255) / 256, 1024)), dim3(256), 0, s,
                     h->d_flags, clear, 0u);
  HIPCHK(hipGetLastError());
  if (h->v.nb == 0) return 0;
  if (sched == 0) {
    kfn_t k = pick_kernel<kModeFlags>(G, U);
    uint64_t groups = std::min<uint64_t>(h->v.nb, (uint64_t)resident_groups(k, h->cu_count, G));
    uint64_t wgs = (groups + (kWG / G) - 1) / (kWG / G);
    hipLaunchKernelGGL(k, dim3((unsigned)wgs), dim3(kWG), 0, s, A);
    HIPCHK(hipGetLastError());
  } else {
    if (!h->has_plan) return lz::fail(LZ_E_INVAL, "no level plan (more than 65534 levels)");
    kfn_t k = pick_kernel<kModeLevels>(G, U);
    uint64_t wgs = (h->v.nb + (kWG / G) - 1) / (kWG / G);
    for (uint32_t p = 0; p < h->levels; ++p) {
      A.pass = p;
      hipLaunchKernelGGL(k, dim3((unsigned)wgs), dim3(kWG), 0, s, A);
      HIPCHK(hipGetLastError());
    }
  }
  return 0;
}

int lz_device_check(lz_dev* h, void* stream) {
  if (!h) return lz::fail(LZ_E_INVAL, "null handle");
  hipStream_t s = (hipStream_t)stream;
  uint32_t err = 0;
  HIPCHK(hipMemcpyAsync(&err, h->d_ctrl + 1, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (err) return lz::fail(LZ_E_BUSY, "a bounded device wait expired (err %u)", err);
  return 0;
}

int lz_purecopy_device(uint64_t ntok, const uint64_t* d_dst, const uint64_t* d_lit_off, const uint32_t* d_lit_len,
                       const uint64_t* d_src, const uint32_t* d_mlen, uint64_t nunits, const uint64_t* d_unit_start,
                       const uint8_t* d_lit, uint64_t lit_size, const uint8_t* d_ref, uint64_t ref_size,
                       uint8_t* d_out, uint64_t out_size, const lz_decode_cfg* cfg, void* stream) {
  if (ntok && (!d_dst || !d_lit_off || !d_lit_len || !d_src || !d_mlen || !d_unit_start || !d_out))
    return lz::fail(LZ_E_INVAL, "null argument");
  uint32_t G, U, sched;
  int rc = resolve_cfg(cfg, G, U, sched);
  if (rc) return rc;
  if (nunits == 0) return 0;
  KArgs A;
  memset(&A, 0, sizeof(A));
  A.lit = d_lit;
  A.lit_lo = (uintptr_t)d_lit;
  A.lit_hi = (uintptr_t)d_lit + lit_size;
  A.out = d_out;
  A.msrc = d_ref;
  A.msrc_lo = (uintptr_t)d_ref;
  A.msrc_hi = (uintptr_t)d_ref + ref_size;
  A.p_dst = d_dst;
  A.p_lit_off = d_lit_off;
  A.p_lit_len = d_lit_len;
  A.p_src = d_src;
  A.p_mlen = d_mlen;
  A.p_unit = d_unit_start;
  A.nunits = nunits;
  (void)out_size;
  kfn_t k = pick_kernel<kModePure>(G, U);
  uint64_t wgs = (nunits + (kWG / G) - 1) / (kWG / G);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k, dim3((unsigned)wgs), dim3(kWG), 0, s, A);
  HIPCHK(hipGetLastError());
  return 0;
}

}  // extern "C"
