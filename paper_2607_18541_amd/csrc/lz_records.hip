// lz_records.hip -- read-level seek: record id -> LZ block -> record bytes.
//
// The paper's seek is read/block-level: a read id maps to the block holding
// it (Sec. 6, first limitation; Sec. 1 "Positioning": seek on compressed-
// resident data).  A record is `lines` newline-terminated lines (FASTQ: 4);
// record r starts at 0 (r = 0) or just after the (lines * r)-th newline.  The
// index keeps, per LZ block, the id and offset of the first record starting
// in it or in a later block (16 bytes per block).  Record `id` starts in the
// last block b whose first id is <= id, at or after that block's first
// record start, and ends at or before the start of the first record of the
// next block c > b in which a record starts (or the end of the data).  A seek
// range-decodes exactly [first_off[b], first_off[c]) on the device, then one
// workgroup counts newlines to find the record's ends and copies it out.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "lz_internal.h"

struct lz_read_index {
  uint64_t n = 0, records = 0;
  uint32_t log2_bs = 16, lines = 4;
  std::vector<uint64_t> first_id, first_off;  // per block; first_off = n where no record starts at or after
};

namespace {

constexpr char kIdxMagic[8] = {'L', 'Z', 'R', 'I', 'X', '0', '0', '1'};
constexpr int kFindThreads = 1024;

// Finds, in win[0, W), the position after the k_start-th newline (0 when
// k_start is 0) and after the k_end-th newline (W when there are fewer), and
// copies the bytes between them to out when they fit out_cap.
// res: {start, end, status (0 copied, 1 larger than out_cap)}.
__global__ __launch_bounds__(kFindThreads) void k_find_record(const uint8_t* win, uint64_t W, uint64_t k_start,
                                                               uint64_t k_end, uint8_t* out, uint64_t out_cap,
                                                               uint64_t* res) {
  __shared__ uint64_t s_cnt[kFindThreads];
  __shared__ uint64_t s_pos[2];
  const int t = threadIdx.x;
  const uint64_t chunk = (W + kFindThreads - 1) / kFindThreads;
  const uint64_t a = min(W, (uint64_t)t * chunk), b = min(W, a + chunk);
  uint64_t c = 0;
  for (uint64_t i = a; i < b; ++i) c += (win[i] == '\n');
  s_cnt[t] = c;
  if (t < 2) s_pos[t] = (t == 0 && k_start == 0) ? 0 : W;
  __syncthreads();
  // inclusive prefix over the threads (Hillis-Steele in LDS)
  for (int d = 1; d < kFindThreads; d <<= 1) {
    const uint64_t v = (t >= d) ? s_cnt[t - d] : 0;
    __syncthreads();
    s_cnt[t] += v;
    __syncthreads();
  }
  const uint64_t before = s_cnt[t] - c;  // newlines before this thread's chunk
  const uint64_t ks[2] = {k_start, k_end};
  for (int j = 0; j < 2; ++j) {
    const uint64_t k = ks[j];
    if (k == 0 || k <= before || k > before + c) continue;  // the k-th newline is not in this chunk
    uint64_t seen = before;
    for (uint64_t i = a; i < b; ++i)
      if (win[i] == '\n' && ++seen == k) {
        s_pos[j] = i + 1;
        break;
      }
  }
  __syncthreads();
  const uint64_t st = s_pos[0], en = max(s_pos[0], s_pos[1]);
  const bool fits = en - st <= out_cap;
  if (fits)
    for (uint64_t i = st + t; i < en; i += kFindThreads) out[i - st] = win[i];
  if (t == 0) {
    res[0] = st;
    res[1] = en;
    res[2] = fits ? 0 : 1;
  }
}

// Window [off0, off1) holding record id, and the newlines to skip in it.
int record_window(const lz_read_index* x, uint64_t id, uint64_t* off0, uint64_t* off1, uint64_t* skip) {
  if (id >= x->records)
    return lz::fail(LZ_E_RANGE, "record %llu outside [0, %llu)", (unsigned long long)id,
                    (unsigned long long)x->records);
  const auto& F = x->first_id;
  // last block whose first record id <= id among blocks where a record starts
  size_t b = std::upper_bound(F.begin(), F.end(), id) - F.begin();
  while (b > 0 && x->first_off[b - 1] >= x->n) --b;  // defensive: blocks past the last record start
  if (b == 0) return lz::fail(LZ_E_CORRUPT, "index has no block for record %llu", (unsigned long long)id);
  --b;
  // a block's first record starts in it unless no record starts there; step
  // back to the block that really holds the start of first_id[b]
  *off0 = x->first_off[b];
  *skip = (id - F[b]) * x->lines;
  *off1 = x->n;
  for (size_t c = b + 1; c < F.size(); ++c)
    if (F[c] > id) {
      *off1 = x->first_off[c];
      break;
    }
  return 0;
}

}  // namespace

extern "C" {

int lz_read_index_build(const uint8_t* in, uint64_t n, uint32_t log2_bs, uint32_t lines, lz_read_index** out) {
  if (!out || (n && !in)) return lz::fail(LZ_E_INVAL, "null argument");
  if (log2_bs < 4 || log2_bs > 24 || lines == 0) return lz::fail(LZ_E_INVAL, "bad block size or lines per record");
  *out = nullptr;
  lz_read_index* x = new lz_read_index();
  x->n = n;
  x->log2_bs = log2_bs;
  x->lines = lines;
  const uint64_t bs = 1ull << log2_bs, nb = (n + bs - 1) / bs;
  try {
    x->first_id.assign(nb, 0);
    x->first_off.assign(nb, n);
    // record starts in increasing order: assign each to its block; blocks
    // without a start take the next record's id and offset
    uint64_t r = 0, next_blk = 0;
    auto start_at = [&](uint64_t pos) {
      const uint64_t blk = pos >> log2_bs;
      for (; next_blk <= blk && next_blk < nb; ++next_blk) {
        x->first_id[next_blk] = r;
        x->first_off[next_blk] = pos;
      }
      ++r;
    };
    if (n) start_at(0);
    uint64_t nl = 0;
    const uint8_t* p = in;
    const uint8_t* end = in + n;
    while (p < end) {
      const uint8_t* q = (const uint8_t*)memchr(p, '\n', (size_t)(end - p));
      if (!q) break;
      ++nl;
      const uint64_t pos = (uint64_t)(q - in) + 1;
      if (nl % lines == 0 && pos < n) start_at(pos);
      p = q + 1;
    }
    for (; next_blk < nb; ++next_blk) {
      x->first_id[next_blk] = r;
      x->first_off[next_blk] = n;
    }
    x->records = r;
  } catch (const std::bad_alloc&) {
    delete x;
    return lz::fail(LZ_E_NOMEM, "index allocation failed");
  }
  *out = x;
  return 0;
}

void lz_read_index_free(lz_read_index* x) { delete x; }
uint64_t lz_read_index_records(const lz_read_index* x) { return x ? x->records : 0; }

int lz_read_index_block(const lz_read_index* x, uint64_t block, uint64_t* first_id, uint64_t* first_off) {
  if (!x || block >= x->first_id.size()) return lz::fail(LZ_E_INVAL, "bad index or block");
  if (first_id) *first_id = x->first_id[block];
  if (first_off) *first_off = x->first_off[block];
  return 0;
}

int lz_read_index_save(const lz_read_index* x, const char* path) {
  if (!x || !path) return lz::fail(LZ_E_INVAL, "null argument");
  FILE* f = fopen(path, "wb");
  if (!f) return lz::fail(LZ_E_INVAL, "cannot open %s for writing", path);
  const uint64_t nb = x->first_id.size();
  bool ok = fwrite(kIdxMagic, 1, 8, f) == 8 && fwrite(&x->n, 8, 1, f) == 1 && fwrite(&x->log2_bs, 4, 1, f) == 1 &&
            fwrite(&x->lines, 4, 1, f) == 1 && fwrite(&x->records, 8, 1, f) == 1 && fwrite(&nb, 8, 1, f) == 1 &&
            fwrite(x->first_id.data(), 8, nb, f) == nb && fwrite(x->first_off.data(), 8, nb, f) == nb;
  ok = (fclose(f) == 0) && ok;
  return ok ? 0 : lz::fail(LZ_E_INVAL, "writing %s failed", path);
}

int lz_read_index_load(const char* path, lz_read_index** out) {
  if (!path || !out) return lz::fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return lz::fail(LZ_E_INVAL, "cannot open %s", path);
  lz_read_index* x = new lz_read_index();
  char magic[8];
  uint64_t nb = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kIdxMagic, 8) == 0 && fread(&x->n, 8, 1, f) == 1 &&
            fread(&x->log2_bs, 4, 1, f) == 1 && fread(&x->lines, 4, 1, f) == 1 && fread(&x->records, 8, 1, f) == 1 &&
            fread(&nb, 8, 1, f) == 1 && x->log2_bs >= 4 && x->log2_bs <= 24 && x->lines > 0 &&
            nb == ((x->n + (1ull << x->log2_bs) - 1) >> x->log2_bs);
  if (ok) {
    // the tables must be in the file before they are allocated (a corrupt
    // size field must not ask for an arbitrary allocation)
    const long at = ftell(f);
    ok = at >= 0 && fseek(f, 0, SEEK_END) == 0 && ftell(f) >= at && (uint64_t)(ftell(f) - at) == 16 * nb &&
         fseek(f, at, SEEK_SET) == 0;
  }
  if (ok) {
    try {
      x->first_id.resize(nb);
      x->first_off.resize(nb);
      ok = fread(x->first_id.data(), 8, nb, f) == nb && fread(x->first_off.data(), 8, nb, f) == nb;
    } catch (const std::bad_alloc&) {
      ok = false;
    }
  }
  fclose(f);
  for (uint64_t b = 0; ok && b < nb; ++b)
    ok = x->first_off[b] <= x->n && x->first_id[b] <= x->records &&
         (b == 0 || (x->first_id[b] >= x->first_id[b - 1] && x->first_off[b] >= x->first_off[b - 1]));
  if (!ok) {
    delete x;
    return lz::fail(LZ_E_CORRUPT, "%s is not a read index", path);
  }
  *out = x;
  return 0;
}

int lz_seek_record_scratch_bytes(lz_dev* h, const lz_read_index* x, uint64_t id, uint64_t* bytes) {
  if (!h || !x || !bytes) return lz::fail(LZ_E_INVAL, "null argument");
  if (x->n != lz_device_n(h)) return lz::fail(LZ_E_INVAL, "index and archive sizes differ");
  uint64_t o0, o1, skip;
  int rc = record_window(x, id, &o0, &o1, &skip);
  if (rc) return rc;
  uint64_t len = o1 - o0, plan_bytes = 0;
  rc = lz_range_scratch_bytes(h, o0, len, &plan_bytes);
  if (rc) return rc;
  *bytes = ((len + 255) & ~uint64_t(255)) + 256 + plan_bytes;
  return 0;
}

int lz_seek_record(lz_dev* h, const lz_read_index* x, uint64_t id, uint8_t* d_out, uint64_t out_cap, void* d_scratch,
                   uint64_t scratch_cap, uint64_t* len, void* stream) {
  if (!h || !x || !d_scratch || !len || (out_cap && !d_out)) return lz::fail(LZ_E_INVAL, "null argument");
  if (x->n != lz_device_n(h)) return lz::fail(LZ_E_INVAL, "index and archive sizes differ");
  if ((uintptr_t)d_scratch & 255u) return lz::fail(LZ_E_INVAL, "d_scratch must be 256-byte aligned");
  uint64_t o0, o1, skip;
  int rc = record_window(x, id, &o0, &o1, &skip);
  if (rc) return rc;
  const uint64_t W = o1 - o0, wbytes = (W + 255) & ~uint64_t(255);
  lz_range_plan* P = nullptr;
  rc = lz_range_plan_create(h, 1, &o0, &W, &P);
  if (rc) return rc;
  const uint64_t need = wbytes + 256 + lz_range_plan_scratch_bytes(P);
  if (scratch_cap < need) {
    lz_range_plan_free(P);
    return lz::fail(LZ_E_NOMEM, "seek scratch %llu < %llu bytes", (unsigned long long)scratch_cap,
                    (unsigned long long)need);
  }
  uint8_t* win = (uint8_t*)d_scratch;
  uint64_t* res = (uint64_t*)(win + wbytes);
  const uint64_t zero = 0;
  hipStream_t s = (hipStream_t)stream;
  // the plan's staging and the result words come from the handle's pinned
  // staging (kept across calls), else from a pinned allocation of the plan
  // and a pageable copy
  std::unique_lock<std::mutex> lock;
  uint64_t local[3] = {0, 0, 0};
  uint8_t* pin = lz::lend_sync_staging(h, P, 3 * sizeof(uint64_t), lock);
  uint64_t* hres = pin ? (uint64_t*)pin : local;
  rc = lz_range_run(h, P, win, W, &zero, win + wbytes + 256, scratch_cap - wbytes - 256, nullptr, stream);
  if (!rc) {
    hipLaunchKernelGGL(k_find_record, dim3(1), dim3(kFindThreads), 0, s, (const uint8_t*)win, W, skip, skip + x->lines,
                       d_out, out_cap, res);
    if (hipGetLastError() != hipSuccess) rc = lz::fail(LZ_E_HIP, "record search launch failed");
  }
  if (!rc && (hipMemcpyAsync(hres, res, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = lz::fail(LZ_E_HIP, "record search failed");
  if (rc) (void)hipStreamSynchronize(s);  // the plan's staging may still be read
  lz_range_plan_free(P);
  if (rc) return rc;
  *len = hres[1] - hres[0];
  if (hres[2]) return lz::fail(LZ_E_NOMEM, "record of %llu bytes exceeds the output capacity %llu",
                               (unsigned long long)*len, (unsigned long long)out_cap);
  return 0;
}

}  // extern "C"
