/*
 * lz_levels_omp.c -- level-parallel CPU decode on all host cores (a timing
 * baseline beside the sequential oracle decode).
 *
 * TEST INFRASTRUCTURE ONLY, under the same rules as lz_oracle.c: the tests and
 * the bench's CPU-baseline leg call it; the product never does.
 *
 * Input: the oracle's pre-parsed tokens and each token's dependency depth
 * (lz_oracle.c: literal bytes have depth 0; a match has one more than the
 * deepest token that wrote any of its source bytes, its own bytes excluded),
 * with the tokens listed depth by depth.  Every literal run is copied at once;
 * then for each depth the matches of that depth are copied at once.  Matches
 * of one depth never read each other's bytes, so each depth is a parallel loop
 * with a barrier after it.  A match whose source overlaps its own bytes is
 * copied byte by byte in order, which realises the overlap.
 */
#include <omp.h>
#include <stdint.h>
#include <string.h>

/* order[depth_start[d] .. depth_start[d+1]) = the tokens of depth d, for
 * d = 0..max_depth.  Returns the number of threads used. */
int or_decode_levels_omp(uint64_t ntok, const uint64_t* dst, const uint64_t* lit_len, const uint64_t* lit_off,
                         const uint64_t* mlen, const uint64_t* src, const uint8_t* lit, const uint64_t* order,
                         const uint64_t* depth_start, uint32_t max_depth, uint8_t* out) {
  int threads = 1;
#pragma omp parallel
  {
#pragma omp single
    threads = omp_get_num_threads();
#pragma omp for schedule(static)
    for (int64_t t = 0; t < (int64_t)ntok; ++t)
      if (lit_len[t]) memcpy(out + dst[t], lit + lit_off[t], lit_len[t]);
    for (uint32_t d = 1; d <= max_depth; ++d) {
#pragma omp for schedule(dynamic, 64)
      for (int64_t k = (int64_t)depth_start[d]; k < (int64_t)depth_start[d + 1]; ++k) {
        const uint64_t t = order[k];
        const uint64_t m0 = dst[t] + lit_len[t];
        uint8_t* o = out + m0;
        const uint8_t* s = out + src[t];
        if (src[t] + mlen[t] <= m0) {
          memcpy(o, s, mlen[t]);
        } else {
          for (uint64_t i = 0; i < mlen[t]; ++i) o[i] = s[i];
        }
      }
    }
  }
  return threads;
}
