/*
 * lz.h -- C ABI of liblz: absolute-offset LZ77 with a gfx950 match-phase decoder.
 *
 * The method (arxiv 2607.18541): an LZ77 stream whose every back-reference
 * names an ABSOLUTE output position (Abstract; Sec. 1 "Positioning"), cut into
 * LZ blocks of an encode-time size (Sec. 2; Sec. 5, last paragraph), decoded
 * on the GPU by groups of G cooperating lanes per block (Sec. 2, Sec. 3.1:
 * lanes = G x N_blocks), with a per-distance-class minimum match length chosen
 * at encode time (Sec. 4.2, e.g. 6/8/10/12 or 12/16/24/32).
 *
 * Conventions for every entry point:
 *  - Return 0 on success or a negative LZ_E_* code; lz_last_error() gives a
 *    thread-local message.  Nothing throws across the ABI.
 *  - Host buffers written by the library (archives) are allocated here and
 *    released with lz_free.  Device memory is always the caller's: pass raw
 *    device pointers and sizes; the library never allocates device memory on
 *    the decode path.
 *  - `stream` is a hipStream_t passed as void*; device work is enqueued on it
 *    asynchronously and the caller synchronises.
 *  - Decoders never read outside the archive or write outside
 *    [d_out, d_out + out_cap): every archive is fully validated on the host by
 *    lz_device_open before any kernel sees it.
 *
 * Container format, version 1 (integers little-endian).  The paper gives no
 * byte layout; this is the layout of this library.
 *   header [0,128): u32 magic 0x314D5A4C ("LZM1"), u32 version 1, u64 n
 *     (decoded bytes), u32 log2_bs (4..24), u32 n_blocks = ceil(n/bs),
 *     u32 min_match (>=1, base of match-length codes), u32 flags (bit0: src_hi
 *     plane present, bit1: per-block info bytes present), u64 n_tok, u64 n_x16,
 *     u64 n_x32, u64 n_lit, u8 thr[4], u32 reserved, u64 bound[3], zeros.
 *   block table at 128: n_blocks+1 entries {u64 tok, u64 lit, u64 x16, u64 x32}
 *     of cumulative stream starts (entry 0 zero, last entry the totals).
 *   streams, each 16-byte aligned, in order: cmd u8[n_tok], x16 u16[n_x16],
 *     x32 u32[n_x32], src_lo u32[n_tok], src_hi u8[n_tok] (flag bit0),
 *     lit u8[n_lit], info u8[n_blocks] (flag bit1), 16 zero bytes; the size is
 *     a multiple of 16.
 *   token t of block b (covering [b*bs, min(n,(b+1)*bs))): c = cmd[t];
 *     literal code c>>4, match code c&15; code 15 is extended: v = next x16,
 *     if v == 0xFFFF then v = 0xFFFF + next x32; value = 15 + v (literal
 *     extension read first).  The block's last token has match code 0 and
 *     match length = block end - (token start + literal length); other tokens
 *     have match length min_match + match value.  The match source is
 *     src_lo[t] | src_hi[t]<<32 and must be below the match start; overlap
 *     (source + length past the start) repeats the period start-source.
 */
#ifndef LZ_H
#define LZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LZ_OK 0
#define LZ_E_INVAL (-1)   /* bad argument (sizes, capacities, parameters) */
#define LZ_E_CORRUPT (-2) /* archive fails validation */
#define LZ_E_RANGE (-3)   /* requested range outside [0, n) */
#define LZ_E_NOMEM (-4)   /* host allocation failed or buffer too small */
#define LZ_E_HIP (-5)     /* HIP runtime error */
#define LZ_E_BUSY (-6)    /* a bounded device-side wait expired */

/* Encoder parameters (Sec. 4.2): thresholds thr[c] apply to distance class
 * c = 0 if d < bound[0], 1 if d < bound[1], 2 if d < bound[2], else 3, with
 * d = destination - source. */
typedef struct lz_params {
  uint32_t log2_bs;    /* LZ block size 2^log2_bs bytes (Sec. 2), 4..24 */
  uint32_t thr[4];     /* minimum match length per distance class, >= 1 */
  uint64_t bound[3];   /* class bounds, increasing */
  uint32_t max_chain;  /* candidates walked per hash chain; 0 = all (exact greedy) */
  uint32_t n_threads;  /* encoder threads; 0 = hardware concurrency */
  uint64_t segment;    /* 0 = whole-prefix window; else sources stay inside
                          aligned segments of this many bytes (multiple of bs) */
  /* optional: called on the calling thread after each segment is parsed with
   * the input bytes done so far and the total; user is passed through */
  void (*progress)(uint64_t done, uint64_t total, void* user);
  void* progress_user;
  /* Tie-break among equally long valid candidates (lengths never change):
   * 0 = the nearest source; k = 1..8 = k further parses in which the source
   * with the lowest resulting dependency depth (1 + the deepest byte it reads,
   * as in lz_plan) wins, then the nearest.  Blocks are parsed in parallel, so
   * a pass takes the depths of earlier blocks from the parse before it and
   * those of its own block from itself. */
  uint32_t depth_passes;
  /* Threshold mode: 0 = thr[] for every block; 1 = learned (Sec. 4.3 and
   * Sec. 6: the best tuple is data-dependent): each block's tuple is chosen
   * by the selector stored at mlp_path (a file of lz_selector_save), as
   * lz_encode_learned does with an in-memory selector. */
  uint32_t mode;
  const char* mlp_path;
  /* Depth cap (an encode-side lever in the spirit of Sec. 4: fewer
   * dependency depths, fewer decode passes): 0 = none; k = 1..65534: after
   * the parse, a walk in output order turns every match whose dependency
   * depth (as in lz_plan) would exceed k into literal bytes, so the archive
   * has at most k depths.  Costs ratio where it acts. */
  uint32_t depth_cap;
} lz_params;

/* Fills the defaults: 64 KiB blocks, thresholds 6/8/10/12, bounds 4 KiB /
 * 64 KiB / 1 MiB, max_chain 32, all threads, whole-prefix window, one
 * depth-aware parse (depth_passes 1), mode 0. */
int lz_params_default(lz_params* p);

/* Greedy LZ77 parse of in[0,n) with per-class thresholds (Sec. 4.2) into a
 * library-allocated archive (*arc, *arc_size); free with lz_free.  Host only,
 * multithreaded over blocks; with max_chain = 0 the match lengths equal the
 * exhaustive greedy parse. */
int lz_encode(const uint8_t* in, uint64_t n, const lz_params* p, uint8_t** arc, uint64_t* arc_size);

/* Same, but each block b is parsed with its own threshold tuple
 * thr_per_block[4*b .. 4*b+3]; tuple_id[b] (may be NULL) is stored in the
 * per-block info bytes.  Used by the learned threshold selector. */
int lz_encode_blockwise(const uint8_t* in, uint64_t n, const lz_params* p, const uint32_t* thr_per_block,
                        const uint8_t* tuple_id, uint8_t** arc, uint64_t* arc_size);

/* Serialises a given token stream (token t: lit_len[t] literals taken in
 * order from lit, then mlen[t] bytes copied from absolute position src[t])
 * covering n bytes; tokens may straddle block ends and are cut there.
 * min_match = 0 picks the smallest match length that needs a code. */
int lz_build_archive(uint64_t n, uint32_t log2_bs, uint32_t min_match, uint64_t ntok, const uint32_t* lit_len,
                     const uint32_t* mlen, const uint64_t* src, const uint8_t* lit, uint64_t nlit, uint8_t** arc,
                     uint64_t* arc_size);

void lz_free(void* p);

typedef struct lz_info {
  uint64_t n, n_blocks, n_tok, n_lit, n_match, match_bytes, archive_bytes;
  uint32_t log2_bs, min_match;
  uint32_t thr[4];
  uint64_t bound[3];
  double mean_match;     /* mean match length (Sec. 4.1) */
  double frac_lt32;      /* fraction of matches shorter than 32 bytes */
  double coverage;       /* fraction of output bytes produced by matches */
  uint64_t src_bytes;    /* bytes of absolute offsets (src_lo + src_hi planes) */
  uint64_t hist[4][16];  /* matches per distance class x length bin (bins:
                            [4,6) [6,8) [8,10) [10,12) [12,16) [16,20) [20,24)
                            [24,32) [32,48) [48,64) [64,128) [128,256)
                            [256,1K) [1K,4K) [4K,16K) [16K,inf); <4 goes to bin 0) */
} lz_info;

/* Validates the archive and fills statistics (Sec. 4.1 match statistics). */
int lz_archive_info(const uint8_t* arc, uint64_t arc_size, lz_info* out);

/* Entropy-bound size (bytes): header and block table verbatim plus, for each
 * stream (cmd, x16, x32, every byte plane of the sources, lit), the order-0
 * entropy over 64 KiB tiles (the tile size of Sec. 2) plus 1 + 2 x (distinct
 * symbols) per tile.  parts[7] (optional): cmd, x16, x32, src_lo planes, lit,
 * header+table, src_hi plane. */
int lz_entropy_size(const uint8_t* arc, uint64_t arc_size, double* total, double* parts);

/* Dependency depth of every match (the schedule of the parallel decode; the
 * paper does not fix one): literal bytes have depth 0 and a match has depth
 * 1 + the largest depth among the tokens that write its source bytes, its own
 * output excluded (a self-overlapping match reads its period).  Matches of one
 * depth never read each other's output.  levels (may be NULL) receives n_tok
 * values (0 for a token without a match); *max_level the largest depth. */
int lz_plan(const uint8_t* arc, uint64_t arc_size, uint32_t* levels, uint32_t* max_level);

/* FNV-1a 64 (Sec. 2 integrity hash), seed = offset basis 0xcbf29ce484222325. */
uint64_t lz_fnv1a64(const uint8_t* p, uint64_t n, uint64_t seed);

const char* lz_last_error(void);

/* ------------------------------------------------------------- device side */

typedef struct lz_dev lz_dev; /* opaque handle of a device-resident archive */

/* Decode configuration.  A decode is a parse launch (one group of G lanes per
 * 128-token segment of a block: token headers, literal bytes, match table)
 * followed by the matches in order of their depth (lz_plan), cut into windows
 * of at most 64 matches and 3 KiB of match output (a longer match is split
 * over windows); the G lanes of a group cooperate on 64 / G parts of a window
 * (Sec. 2, G in {8,16,32,64}); unroll = 16-byte chunks per lane per step
 * (1, 2, 4).  schedule 0 = every depth in one launch, a window starting once
 * all windows of the depth below have finished (per-depth counters);
 * schedule 1 = one launch per depth, except that the deepest depths that each
 * have at most `tail` windows run in a single one-workgroup launch with a
 * barrier between depths (0 = 32 windows; 0xFFFFFFFF = no such launch).
 * mapping = which workgroup takes which work item: 0 = in launch order (the
 * hardware deals consecutive workgroups to the 8 XCDs in turn, so neighbouring
 * segments and windows run on different XCDs), 1 = XCD-contiguous (the
 * workgroups one XCD receives take one contiguous run of items, so
 * neighbouring writes meet in that XCD's L2).
 * occupancy = 0: as many workgroups per CU as fit; k in [3, 8]: the depth
 * passes of a schedule 1 decode (lz_decode_device, lz_decode_device_stage)
 * run with at most k resident workgroups per CU (their LDS is padded to
 * that), an occupancy control (Sec. 3.3); LZ_E_INVAL outside that range or
 * above what fits anyway.  Batches and range plans ignore it.
 * G and unroll select the match copy; the parse launch has its own group
 * size and unroll (parse_G, parse_unroll): a whole wave per 128-token
 * segment is the fastest parse at every G (measured: at G = 32 the parse
 * with 32-lane groups takes 1.07 ms of a 1.84 ms decode, with a wave 0.63).
 * NULL config = G 64, unroll 2, schedule 1, tail 0, mapping 0, occupancy 0,
 * parse_G 64, parse_unroll 2. */
typedef struct lz_decode_cfg {
  uint32_t G;
  uint32_t unroll;
  uint32_t schedule;
  uint32_t tail;
  uint32_t mapping;
  uint32_t occupancy;
  uint32_t parse_G;       /* lanes per parse group (8, 16, 32, 64; 0 = 64, one wave) */
  uint32_t parse_unroll;  /* 16-byte blocks per lane per parse step (1, 2, 4; 0 = 2) */
} lz_decode_cfg;

/* Device bytes lz_device_open needs for this archive: the archive itself, the
 * depth plan (a match-table slot per token, level starts, counters), the parse
 * segments and the match table (16 bytes per token). */
int lz_device_bytes(const uint8_t* arc, uint64_t arc_size, uint64_t* bytes);

/* Validates the archive on the host, copies it into the caller's device buffer
 * d_buf (>= lz_device_bytes, 256-byte aligned as hipMalloc and torch
 * allocations are; LZ_E_INVAL otherwise) on `stream`, and returns a handle.
 * The host archive may be freed after the stream has completed the copy. */
int lz_device_open(const uint8_t* arc, uint64_t arc_size, void* d_buf, uint64_t d_cap, void* stream, lz_dev** h);

/* Decodes the whole archive into d_out[0, n) (Sec. 2: match phase, device
 * resident).  Asynchronous on `stream`.  out_cap < n gives LZ_E_INVAL.  Only
 * d_out[0, n) is written; its bytes are final once the call's work on
 * `stream` completes (in between, match bytes may hold arbitrary values). */
int lz_decode_device(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, void* stream);

/* The two stages of lz_decode_device as separate launch sequences (to time or
 * schedule them apart): stage 1 = the parse launch (literal bytes and the
 * literal-sourced matches of lz_device_fused written, the match table filled;
 * where literals are dense the parse writes whole aligned blocks of the
 * output, so the other match bytes hold arbitrary values after stage 1
 * alone), stage 2 = the match passes, which must follow stage 1 of the same
 * handle and output on the same stream; stage 0 = both. */
int lz_decode_device_stage(lz_dev* h, uint8_t* d_out, uint64_t out_cap, const lz_decode_cfg* cfg, int stage,
                           void* stream);

/* Synchronises `stream` and reports a device-side failure of the last decode
 * on this handle: LZ_E_BUSY if a bounded wait expired, LZ_E_CORRUPT if a match
 * record outside the output was skipped, LZ_E_INVAL for a launch of the wrong
 * workgroup size; else 0. */
int lz_device_check(lz_dev* h, void* stream);

uint64_t lz_device_n(const lz_dev* h);
uint32_t lz_device_levels(const lz_dev* h); /* number of match depths (launches of schedule 1) */
/* Number of matches the parse copies itself (the match phase of Sec. 2; a match
 * whose source bytes are all literals has no dependency on other matches).
 * A depth-1 match whose source lies inside one token's literal run and ends
 * before its own output starts is read from the literal stream at an offset
 * the plan computes at open; it takes no window of the depth passes.  Returns
 * their count (0 when the archive has none, or h is null) and, when `bytes`
 * is not null, stores their total length there. */
uint64_t lz_device_fused(const lz_dev* h, uint64_t* bytes);
void lz_device_close(lz_dev* h);

/* ------------------------------------------------------------ entropy stage */

/* Tile-rANS entropy stage (Sec. 2, Experimental Setup: entropy decoded over
 * 64 KB tiles, cut independently of the LZ blocks, before the match phase).
 * lz_entropy_encode codes a container (host): its bytes before the 32-bit
 * sources (header, block table, cmd, x16, x32), each of the four byte planes
 * of the sources (stride 4), and its bytes after them (high source plane,
 * literals), each cut into tiles of at most 65,536 symbols, each
 * stored raw, as one repeated byte, or order-0 rANS coded, whichever is
 * smallest.  rANS: probabilities quantised to 1/4096 (f = floor(count * 4096 /
 * N), present symbols at least 1, the sum corrected on the most frequent
 * symbol), 32-bit states in [2^16, 2^32) renormalised by 16-bit words, 64
 * states interleaved (symbol i to state i mod 64), words consumed in symbol
 * order.  Coded container "LZE1": a 64-byte header, the coded container's
 * 128-byte header, 32-byte tile records {payload offset, first output byte,
 * symbols, payload bytes, output stride, mode}, payloads; a rANS payload is
 * a 32-byte symbol bitmap, u16 frequencies, 64 u32 initial states, u16 words.
 * Library-allocated; free with lz_free. */
int lz_entropy_encode(const uint8_t* arc, uint64_t arc_size, uint8_t** coded, uint64_t* coded_size);
/* Validates a coded container (every tile inside it, tables summing to 4096,
 * every output byte written exactly once); decoded size, tile count and tiles
 * per mode {raw, rANS, repeated} (each may be NULL). */
int lz_entropy_info(const uint8_t* coded, uint64_t size, uint64_t* decoded_size, uint64_t* tiles,
                    uint64_t* tiles_by_mode);
/* Device bytes lz_device_open_coded needs: the resident coded container plus
 * the layout of lz_device_bytes for the container it decodes to. */
int lz_coded_device_bytes(const uint8_t* coded, uint64_t size, uint64_t* bytes);
/* Opens a coded container: validated on the host, copied to d_buf, entropy-
 * decoded on the GPU (one wave per tile) into the handle's archive region,
 * then read back once to validate the decoded container and build the plan
 * (LZ_E_CORRUPT if a tile decodes inconsistently).  The handle then decodes
 * like one from lz_device_open, and lz_entropy_decode_device re-runs the
 * entropy stage into the archive region (asynchronous on `stream`; errors
 * show in lz_device_check), so a full pipeline decode is that call followed
 * by lz_decode_device on the same stream. */
int lz_device_open_coded(const uint8_t* coded, uint64_t size, void* d_buf, uint64_t d_cap, void* stream,
                         lz_dev** h);
int lz_entropy_decode_device(lz_dev* h, void* stream);

/* ------------------------------------------------------------ range decode */

/* Region seek on a device-resident archive (Abstract; Sec. 1 "Positioning":
 * random access into compressed-resident data without whole-file decode).
 * A plan covers `count` ranges [off[i], off[i]+len[i]).  The host first
 * computes the token closure of each range (every token the range's bytes
 * depend on through match sources), lays it out in output order in device
 * scratch and orders its copies by dependency depth.  Closures cost host work
 * per byte, so once they exceed max(256 KiB, (E - H)/4096) bytes, E = the
 * largest range end, the plan instead decodes every token of [H, E) on the
 * device (parse segments and depth windows of that stretch) into scratch and
 * gathers the ranges from it.  H, the decode horizon, is the largest start of
 * an output grain (2^20 bytes or the block size if larger) at or below the
 * first range such that no match written between H and the grain holding
 * E - 1 reads below H; archives encoded in segments (lz_params.segment) get
 * their segment starts, so such a decode and its scratch are bounded by one
 * segment.  LZ_E_RANGE if a range leaves [0, n).  Plans are host objects;
 * free with lz_range_plan_free after the stream that ran them has
 * completed. */
typedef struct lz_range_plan lz_range_plan;
int lz_range_plan_create(lz_dev* h, uint64_t count, const uint64_t* off, const uint64_t* len, lz_range_plan** plan);
uint64_t lz_range_plan_scratch_bytes(const lz_range_plan* plan); /* device scratch lz_range_run needs */
uint64_t lz_range_plan_levels(const lz_range_plan* plan);        /* match depths (launches) */
uint64_t lz_range_plan_closure_bytes(const lz_range_plan* plan); /* closure bytes (0 for a prefix plan) */
uint64_t lz_range_plan_prefix_bytes(const lz_range_plan* plan);  /* E - H decoded (0 for a closure plan) */
uint64_t lz_range_plan_horizon(const lz_range_plan* plan);       /* H (0 for a closure plan) */
void lz_range_plan_free(lz_range_plan* plan);

/* Runs a plan on `stream`: range i is written to d_out[out_off[i], +len[i]),
 * which must lie inside [d_out, d_out+out_cap); d_scratch holds at least
 * lz_range_plan_scratch_bytes.  All ranges of the plan share each launch.
 * cfg (NULL = defaults): G, unroll and mapping as for a decode; a prefix
 * decode launches its depths one by one and runs the deepest that have at
 * most `tail` windows in one workgroup, as schedule 1 does. */
int lz_range_run(lz_dev* h, lz_range_plan* plan, uint8_t* d_out, uint64_t out_cap, const uint64_t* out_off,
                 void* d_scratch, uint64_t scratch_cap, const lz_decode_cfg* cfg, void* stream);

/* Single range: scratch bytes it needs, and a synchronous decode of
 * [off, off+len) into d_out[0, len). */
int lz_range_scratch_bytes(lz_dev* h, uint64_t off, uint64_t len, uint64_t* bytes);
int lz_decode_range(lz_dev* h, uint64_t off, uint64_t len, uint8_t* d_out, void* d_scratch, uint64_t scratch_cap,
                    void* stream);

/* ------------------------------------------------------------ read seek */

/* Read-level seek (Sec. 6, first limitation: seek is read id -> block; Sec. 1
 * "Positioning": seek into compressed-resident data).  A record is `lines`
 * newline-terminated lines (FASTQ: 4); record r starts at 0 (r = 0) or just
 * after the (lines * r)-th newline, and ends where record r + 1 starts (the
 * last one at its last newline, or at n when that is missing).  The index
 * holds, per LZ block of 2^log2_bs bytes, the id and offset of the first
 * record starting in that block or later (offset n when none does): 16
 * bytes per block.  Built on the host from the input (at encode time). */
typedef struct lz_read_index lz_read_index;
int lz_read_index_build(const uint8_t* in, uint64_t n, uint32_t log2_bs, uint32_t lines, lz_read_index** index);
void lz_read_index_free(lz_read_index* index);
uint64_t lz_read_index_records(const lz_read_index* index);
int lz_read_index_block(const lz_read_index* index, uint64_t block, uint64_t* first_id, uint64_t* first_off);
/* File: "LZRIX001", u64 n, u32 log2_bs, u32 lines, u64 records, u64 blocks,
 * u64 first_id[blocks], u64 first_off[blocks]; LZ_E_CORRUPT if not one. */
int lz_read_index_save(const lz_read_index* index, const char* path);
int lz_read_index_load(const char* path, lz_read_index** index);

/* Record `id` (LZ_E_RANGE if >= the record count) of a device-resident
 * archive of the same input: its block b is the last whose first record id is
 * <= id; the bytes from b's first record start to the first record start of
 * the next block with one (or n) hold it whole and are range-decoded on the
 * device (lz_range_plan_create / lz_range_run), then one workgroup counts
 * newlines and copies the record to d_out[0, *len).  d_scratch (256-byte
 * aligned) holds lz_seek_record_scratch_bytes for this id; LZ_E_NOMEM (with
 * *len set) if the record exceeds out_cap.  Synchronises `stream`. */
int lz_seek_record_scratch_bytes(lz_dev* h, const lz_read_index* index, uint64_t id, uint64_t* bytes);
int lz_seek_record(lz_dev* h, const lz_read_index* index, uint64_t id, uint8_t* d_out, uint64_t out_cap,
                   void* d_scratch, uint64_t scratch_cap, uint64_t* len, void* stream);

/* ------------------------------------------------------------ batch decode */

/* Many archives in one replayable launch sequence (one graph launch): work of
 * all archives that share a configuration is merged into the same kernel
 * launches (one parse launch, then one per dependency level, or one for
 * schedule 0).  This is how small archives -- starved alone, Sec. 3.1/3.2 --
 * fill the GPU.  Archive i decodes into d_out[i] (capacity out_cap[i]);
 * cfgs[i] (NULL = defaults) selects its configuration.  d_scratch holds the
 * merged work lists (lz_batch_scratch_bytes; 256-byte aligned, else
 * LZ_E_INVAL).  The batch records the handles' device buffers: an archive must
 * not be decoded elsewhere while the batch runs. */
typedef struct lz_batch lz_batch;
int lz_batch_scratch_bytes(uint32_t count, lz_dev* const* handles, const lz_decode_cfg* cfgs, uint64_t* bytes);
int lz_batch_create(uint32_t count, lz_dev* const* handles, uint8_t* const* d_out, const uint64_t* out_cap,
                    const lz_decode_cfg* cfgs, void* d_scratch, uint64_t scratch_cap, void* stream, lz_batch** batch);
int lz_batch_launch(lz_batch* batch, void* stream);
uint64_t lz_batch_launches(const lz_batch* batch); /* kernel launches per replay */
void lz_batch_destroy(lz_batch* batch);

/* Autotuner: archives are bucketed by size (x4 buckets from 16 KiB); for each
 * bucket every (G in {16,32,64}) x (unroll in {1,2,4}) x (schedule 1, 0) x
 * (mapping 0, 1) is timed with HIP events as a batch of that bucket alone
 * (one warm-up, `reps` replays) and the fastest is written to chosen[i] for
 * the bucket's archives.  A batch with several configurations runs a launch
 * sequence per configuration, so the whole batch is then timed with the
 * choices and with the default, and every chosen[i] becomes the default
 * when that is not slower (skipped when scratch_cap is below
 * lz_batch_scratch_bytes for the choices).
 * report (optional) receives one entry per non-empty bucket. */
typedef struct lz_tune_report {
  uint64_t min_bytes, max_bytes, bytes;
  uint32_t archives;
  lz_decode_cfg best;
  float best_ms, default_ms; /* default: G 64, unroll 2, schedule 1, mapping 0 */
} lz_tune_report;
int lz_autotune(uint32_t count, lz_dev* const* handles, uint8_t* const* d_out, const uint64_t* out_cap,
                void* d_scratch, uint64_t scratch_cap, void* stream, uint32_t reps, lz_decode_cfg* chosen,
                lz_tune_report* report, uint32_t report_cap, uint32_t* n_report);

/* ------------------------------------------------------------ serving */

/* Continuous batching of region-seek requests on one device-resident archive
 * (Sec. 1 "Positioning": compressed residency with sub-millisecond seek).
 * Requests queue in arrival order.  lz_serve_tick retires finished groups
 * (frees their scratch), admits waiting requests in order while one of
 * `slots` is free and the arena has room for the output, splits what it
 * admitted by decode horizon (the grain where a request's prefix decode
 * starts; on a segment-encoded archive, its segment) and launches one merged
 * range plan per horizon, in order of each group's oldest request, round-robin
 * over four streams so groups overlap each other and earlier ones.  Requests
 * whose horizon already has a group on the device stay admitted (state 0)
 * until it finishes and then join the next group of that horizon.  A group
 * whose scratch does not fit sends later groups, then its own newest
 * requests, back to the head of the queue (arrival order is kept).
 * A tick allocates no device or pinned memory (plan staging comes from a
 * pinned pool the server owns, which grows only while no group is in flight).
 * Outputs live in the arena until lz_serve_release.  A request that can never
 * fit (its output plus its plan scratch exceed the arena) makes the tick that
 * meets it return LZ_E_NOMEM and is marked failed (state 4); its slot is held
 * until lz_serve_release.  Single-threaded use. */
typedef struct lz_server lz_server;
int lz_serve_create(lz_dev* h, void* d_arena, uint64_t arena_bytes, uint32_t slots, const lz_decode_cfg* cfg,
                    lz_server** server);
int lz_serve_submit(lz_server* server, uint64_t off, uint64_t len, uint64_t* id);
int lz_serve_tick(lz_server* server, uint64_t* n_done, uint64_t* n_admitted);
int lz_serve_status(lz_server* server, uint64_t id,
                    int* state /* 0 waiting, 1 running, 2 done, 3 released, 4 failed */, uint8_t** d_ptr);
int lz_serve_release(lz_server* server, uint64_t id);
/* Ids of requests that finished (done or failed) since the last call, in the
 * order the ticks saw them finish, at most `cap` of them; returns how many
 * were written.  Lets a caller find its finished requests without polling
 * every outstanding id. */
uint64_t lz_serve_completed(lz_server* server, uint64_t* ids, uint64_t cap);
void lz_serve_stats(const lz_server* server, uint64_t* waiting, uint64_t* running_groups, uint64_t* arena_used,
                    uint64_t* arena_high_water);
uint64_t lz_serve_max_running(const lz_server* server); /* most groups in flight after any tick so far */
int lz_serve_destroy(lz_server* server);

/* ------------------------------------------------------ learned thresholds */

/* Per-block features of the threshold selector: feats[64*b + 16*c + k] = the
 * fraction of block b's bytes produced by matches of distance class c (bounds
 * as given) in length bin k (bins as in lz_info.hist).  Computed from an
 * archive -- the selector uses a cheap parse at thresholds 4/4/4/4. */
int lz_block_features(const uint8_t* arc, uint64_t arc_size, const uint64_t* bounds, float* feats);

/* Per block (arrays of n_blocks, each may be NULL): entropy-bound bytes of the
 * block's streams with the block as one tile, token, match and match-byte
 * counts. */
int lz_block_stats(const uint8_t* arc, uint64_t arc_size, double* ent, uint64_t* ntok, uint64_t* nmatch,
                   uint64_t* match_bytes);

/* The selector network on the GPU (fp32, device pointers, async on stream):
 * 64 -> 128 -> 128 -> 16, ReLU, softmax over 16 candidate threshold tuples.
 * Parameters: W1 64x128, b1, W2 128x128, b2, W3 128x16, b3 (row-major, flat,
 * lz_mlp_param_count() floats).  Activations are row-major [batch x width]. */
uint64_t lz_mlp_param_count(void);
int lz_mlp_forward(const float* d_params, uint32_t batch, const float* d_x, float* d_h1, float* d_h2, float* d_logits,
                   void* stream);
/* Mean softmax cross-entropy gradient for int32 labels; d_work holds
 * batch x 272 floats; d_loss (may be NULL) is incremented by the mean loss. */
int lz_mlp_backward(const float* d_params, uint32_t batch, const float* d_x, const float* d_h1, const float* d_h2,
                    const float* d_logits, const int32_t* d_labels, float* d_grads, float* d_work, float* d_loss,
                    void* stream);
/* lz_mlp_backward for callers that cannot allocate (code under HIP graph
 * capture, tight training or serving loops, harnesses that forbid hipMalloc):
 * the work buffer is the library's own per-GPU device array of 4096 x 272
 * floats (4.25 MiB, held by each GPU the library runs on until the process
 * ends), so the call allocates nothing.  batch > 4096 gives LZ_E_INVAL.  All
 * calls on one GPU share that array (every element is written before it is
 * read, so nothing carries over between calls): calls that overlap on one GPU,
 * e.g. on two streams, race.  Other arguments as lz_mlp_backward. */
int lz_mlp_backward_noalloc(const float* d_params, uint32_t batch, const float* d_x, const float* d_h1,
                            const float* d_h2, const float* d_logits, const int32_t* d_labels, float* d_grads,
                            float* d_loss, void* stream);
/* One bias-corrected Adam step (Kingma and Ba); step counts from 1. */
int lz_mlp_adam(float* d_params, const float* d_grads, float* d_m, float* d_v, uint64_t n, float lr, float beta1,
                float beta2, float eps, uint32_t step, void* stream);

/* The selector (Sec. 4.3 and Sec. 6: the best threshold tuple is data-dependent
 * at the margin).  A host object holding 16 candidate tuples (4 thresholds
 * each), the fixed fallback tuple, the feature normalisation (mu, sd), the
 * validation cost table of the fallback rule and the network parameters.
 * File format (little-endian): "LZSEL001", u32 16, u32 fixed, u32 tuples[16][4],
 * f32 mu[64], f32 sd[64], f32 val_J[16], u32 26896, f32 params[26896]. */
typedef struct lz_selector lz_selector;
/* tuples: 16 x 4 thresholds (>= 1); fixed < 16; weights He-initialised from
 * `seed` (normal, std sqrt(2 / fan-in)), biases 0, mu 0, sd 1, val_J 1. */
int lz_selector_create(const uint32_t* tuples, uint32_t fixed, uint64_t seed, lz_selector** sel);
int lz_selector_load(const char* path, lz_selector** sel); /* LZ_E_CORRUPT if not a selector file */
int lz_selector_save(const lz_selector* sel, const char* path);
void lz_selector_free(lz_selector* sel);
/* Copies the 26,896 parameters out (get) and/or in (set); either may be NULL. */
int lz_selector_params(lz_selector* sel, float* get, const float* set);
int lz_selector_info(const lz_selector* sel, uint32_t* tuples, uint32_t* fixed, float* mu, float* sd, float* val_J);
/* Feature normalisation from training rows: per feature the mean and the
 * population standard deviation + 1e-6. */
int lz_selector_set_norm(lz_selector* sel, const float* feats, uint64_t n_rows);

/* Labels from the method's own measurements.  Blocks are numbered file by
 * file (file f has file_blocks[f] blocks); for block k and tuple t,
 * size[16k + t] is its entropy-bound bytes (lz_block_stats) and
 * counts[3(16k + t) + {0,1,2}] its tokens, matches and match bytes; per file
 * and tuple, file_ms[16f + t] is the measured GPU decode time and
 * file_depths[16f + t] the plan's depth count.  The decode-time model
 *   ms = c0 tokens + c1 matches + c2 match bytes + c3 depths + c4
 * is fitted by least squares over every (file, tuple) and clamped at 0
 * (coef[5]); a block's time is its share: c0 t + c1 m + c2 b + (c3 depths +
 * c4) / blocks.  J[16k + t] = size / size(fixed) + lambda time / time(fixed),
 * labels[k] = the t of least J (first on ties). */
int lz_learn_labels(uint32_t n_files, const uint32_t* file_blocks, uint32_t fixed, const double* size,
                    const uint64_t* counts, const double* file_ms, const uint32_t* file_depths, double lambda,
                    double* coef, double* J, int32_t* labels);

/* Trains the network on the GPU with the kernels above (softmax cross-entropy,
 * Adam with beta 0.9 / 0.999, eps 1e-8): `epochs` passes over a seeded
 * permutation of the rows (features normalised with the selector's mu / sd),
 * batches of `batch` rows.  d_work: device workspace of
 * lz_selector_train_bytes, 256-byte aligned.  loss_hist[epochs] (may be NULL)
 * receives each epoch's mean loss.  Synchronises `stream`. */
int lz_selector_train_bytes(uint64_t n_rows, uint32_t batch, uint64_t* bytes);
int lz_selector_train(lz_selector* sel, const float* feats, const int32_t* labels, uint64_t n_rows, uint32_t epochs,
                      uint32_t batch, float lr, uint64_t seed, void* d_work, uint64_t work_bytes, float* loss_hist,
                      void* stream);

/* Validation table of the fallback rule: for each tuple, the mean J of the
 * validation rows the network predicts it for (argmax), divided by 1 + lambda
 * (the fixed tuple's J); tuples never predicted get 9, the fixed tuple 1. */
int lz_selector_calibrate(lz_selector* sel, const float* feats, const double* J, uint64_t n_rows, double lambda);

/* Inference on the host (double precision): per row, the tuple of largest
 * softmax probability, or the fixed tuple when that probability is below 0.5
 * or the tuple's validation cost is not below the fixed one's.
 * top_prob (may be NULL) receives the largest probability. */
int lz_selector_choose(const lz_selector* sel, const float* feats, uint64_t n_rows, uint8_t* choice, float* top_prob);

/* Learned mode of the encoder: features from a cheap parse of `in`
 * (thresholds 4/4/4/4, 16 candidates per chain), one tuple per block by
 * lz_selector_choose, then lz_encode_blockwise with those thresholds (tuple
 * indices in the per-block info bytes).  choice (n_blocks, may be NULL)
 * receives the chosen tuple indices.  Other parameters from p. */
int lz_encode_learned(const uint8_t* in, uint64_t n, const lz_params* p, const lz_selector* sel, uint8_t** arc,
                      uint64_t* arc_size, uint8_t* choice);

/* Pure-copy mode (Sec. 3.3, first control): executes pre-decoded tokens on the
 * device.  Token t (SoA, device arrays): copy lit_len[t] bytes from
 * d_lit[lit_off[t]..] to d_out[dst[t]..], then mlen[t] bytes from
 * d_ref[src[t]..] to d_out[dst[t]+lit_len[t]..].  Tokens must write disjoint
 * ranges; units: tokens [unit_start[u], unit_start[u+1]) go to one group of G
 * lanes.  Every index must lie inside the buffers (the caller checks; the
 * Python binding does). */
int lz_purecopy_device(uint64_t ntok, const uint64_t* d_dst, const uint64_t* d_lit_off, const uint32_t* d_lit_len,
                       const uint64_t* d_src, const uint32_t* d_mlen, uint64_t nunits, const uint64_t* d_unit_start,
                       const uint8_t* d_lit, uint64_t lit_size, const uint8_t* d_ref, uint64_t ref_size,
                       uint8_t* d_out, uint64_t out_size, const lz_decode_cfg* cfg, void* stream);

#ifdef __cplusplus
}
#endif
#endif
