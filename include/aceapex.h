/*
 * aceapex.h — C ABI of the MI355X decoder for the absolute-offset LZ77 block
 * format "AXP1".
 *
 * The operations follow the paper's statement of the problem (Introduction:
 * hold a large archive compressed in device memory and decode on demand;
 * Table 2: full device-resident decode; the random-access section: decode one
 * 16 KB tile or a range of blocks from a resident archive):
 *   aceapex_encode        host encoder (global match search, absolute offsets,
 *                         fixed blocks, four streams per block — Setup);
 *   aceapex_decode_all    device decode of a whole resident archive;
 *   aceapex_decode_range  device decode of one byte range (its source closure);
 *   aceapex_decode_batch  many archives / ranges in one persistent launch.
 *
 * Conventions
 *   - Every function returns int: 0 (AX_OK) or a negative AX_E_* code.  No C++
 *     exception crosses this boundary.  aceapex_last_error() gives a
 *     thread-local detail string for the last failure on the calling thread.
 *   - "h_" pointers are host memory, "d_" pointers are device memory of the
 *     current HIP device.  The caller owns every buffer: archive, output,
 *     workspace.  The library owns only opaque host handles.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Decode calls are asynchronous on that stream: they return after
 *     enqueueing; argument and launch errors are returned synchronously,
 *     format errors found on the device are recorded in a status word in the
 *     workspace (first error wins) and read by aceapex_decoder_status.  After a
 *     decode whose status is nonzero the output contents are unspecified.
 *   - One host thread per decoder handle at a time; concurrent decodes on one
 *     handle need distinct workspaces.  Decodes that share a workspace must be
 *     ordered (same stream).
 *   - Block sizes accepted by the device decoder: 4096, 8192, 16384 bytes.
 */
#ifndef ACEAPEX_H
#define ACEAPEX_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  AX_OK = 0,
  AX_E_ARG = -1,         /* bad argument (null pointer, size too small, ...) */
  AX_E_CORRUPT = -2,     /* the archive violates the format */
  AX_E_UNSUPPORTED = -3, /* valid but outside what this library decodes */
  AX_E_CAPACITY = -4,    /* caller buffer or workspace too small */
  AX_E_HIP = -5,         /* a HIP runtime call failed */
  AX_E_RANGE = -6,       /* byte range outside the archive */
  AX_E_DEVICE = -7,      /* device-side failure other than corruption (e.g. a wait limit) */
  AX_E_NOMEM = -8        /* host allocation failed */
};

const char* aceapex_strerror(int code);
const char* aceapex_last_error(void);

/* ------------------------------------------------------------ encoding --- */

/* Encoder parameters (defaults in parentheses).
 *   block_size             output block size, power of two 4096..65536 (16384)
 *   min_match              shortest match (4)
 *   no_rep                 1 = never emit repeat commands; the paper's
 *                          history-free encoding (0)
 *   depth_cap              0 = none; else re-encode until no match is deeper
 *                          than depth_cap — the forced-literal cap of the
 *                          depth section (0)
 *   hash_bits              hash-chain head table size (22)
 *   chain_depth            candidates walked per position (32)
 *   rans_min_syms_per_lane S of the rANS lane rule (32)
 *   off_cost_q             an explicit-offset match must be at least
 *                          min_match + ceil(off_cost_q * (LEB128 bytes of its
 *                          offset) / 4) long: the offset's cost in quarter
 *                          bytes per LEB128 byte (6)
 *   window_log             0 = candidates anywhere behind; else only within
 *                          2^window_log bytes behind the position (0)
 *   threads                encoder threads, 0 = hardware concurrency (0)
 *   progress, progress_user  optional callback, called on the calling thread
 *                          after each encoded segment (1 GiB with a window,
 *                          else the whole input) with the input bytes done
 *                          and the total; NULL = none (NULL) */
typedef void (*aceapex_progress_fn)(void* user, uint64_t bytes_done, uint64_t bytes_total);
typedef struct {
  uint32_t block_size, min_match, no_rep, depth_cap, hash_bits, chain_depth;
  uint32_t rans_min_syms_per_lane, off_cost_q, window_log, threads;
  aceapex_progress_fn progress;
  void* progress_user;
} aceapex_encode_params;

/* Encoder statistics.  n_src_bytes = sum over matches of min(len, dist): the
 * source bytes a periodic-fill copy reads.  n_off_bytes / n_len_bytes are the
 * decoded sizes of the offset and length streams. */
typedef struct {
  uint64_t n_bytes, n_blocks, comp_bytes, n_commands, n_matches, n_rep, n_match_bytes, n_lit_bytes;
  uint64_t n_src_bytes, n_off_bytes, n_len_bytes;
  uint32_t max_depth, passes;
} aceapex_encode_stats;

void aceapex_encode_params_default(aceapex_encode_params* p);

/* Upper bound on the container size for n input bytes. */
int aceapex_encode_bound(uint64_t n, const aceapex_encode_params* p, uint64_t* bound);

/* Encode h_src[0..n) into h_dst[0..dst_cap); *dst_len receives the size.
 * stats may be NULL.  Deterministic: the bytes do not depend on `threads`. */
int aceapex_encode(const uint8_t* h_src, uint64_t n, const aceapex_encode_params* p, uint8_t* h_dst,
                   uint64_t dst_cap, uint64_t* dst_len, aceapex_encode_stats* stats);

/* ------------------------------------------------------------- reading --- */

typedef struct {
  uint64_t n_bytes;       /* decoded size */
  uint64_t n_blocks;
  uint64_t archive_bytes; /* header + index + payload */
  uint64_t header_bytes;  /* header + index: what aceapex_decoder_create needs on the host */
  uint64_t payload_bytes;
  uint64_t n_matches;     /* MATCH + REP commands in the archive */
  uint64_t xxh3;          /* XXH3-64 of the decoded bytes */
  uint32_t block_size, min_match, flags, depth_cap;
} aceapex_info;

/* Parse the header from at least the first 64 bytes (h_len >= 64). The index
 * is not needed. */
int aceapex_read_info(const uint8_t* h_prefix, uint64_t h_len, aceapex_info* info);

/* ------------------------------------------------------------ decoding --- */

typedef struct aceapex_decoder aceapex_decoder;

/* Create a decoder for an archive resident in device memory.
 *   h_header  host copy of the header and index (info.header_bytes bytes);
 *             read once here, not retained.
 *   d_archive the whole archive in device memory (archive_len bytes); must
 *             stay valid and unchanged for the life of the handle.
 * Errors: AX_E_CORRUPT (bad header/index), AX_E_UNSUPPORTED (block size). */
int aceapex_decoder_create(const uint8_t* h_header, uint64_t h_len, const uint8_t* d_archive,
                           uint64_t archive_len, aceapex_decoder** out);
void aceapex_decoder_destroy(aceapex_decoder* dec);
int aceapex_decoder_info(const aceapex_decoder* dec, aceapex_info* info);

/* Device workspace bytes for aceapex_decode_all (256-byte aligned start). */
int aceapex_decoder_workspace(const aceapex_decoder* dec, uint64_t* bytes);

/* Copy modes for the match layer:
 *   AX_COPY_PERIODIC  self-overlapping matches run as periodic fills
 *                     out[dst+k] = out[src + k mod dist], many lanes per match
 *                     (periodic-fill section);
 *   AX_COPY_SERIAL    the ablation: one lane per match, byte after byte. */
enum { AX_COPY_PERIODIC = 0, AX_COPY_SERIAL = 1 };

/* Decode the whole archive into d_out[0..n_bytes).
 * d_work / work_len: device workspace of at least aceapex_decoder_workspace
 * bytes.  Asynchronous on `stream`. */
int aceapex_decode_all(aceapex_decoder* dec, uint8_t* d_out, uint64_t out_cap, void* d_work, uint64_t work_len,
                       int copy_mode, void* stream);

/* aceapex_decode_all without a caller workspace and without allocating: for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * library-owned device array of AX_STATIC_SCRATCH_BYTES, one per device,
 * held from the first call on that device until the process ends.  The call
 * allocates nothing (no device or pinned memory, no events, streams or
 * graphs): it never captures a graph and records no stage timing, whatever
 * AX_OPT_GRAPH and aceapex_decoder_set_timing say.  All such calls on one
 * device share the array, so calls that overlap on one device (two streams,
 * two threads) race; calls ordered on one stream do not.  Read the device
 * status with aceapex_decoder_status(dec, NULL, ...).
 * Errors (before anything is enqueued): AX_E_CAPACITY when
 * aceapex_decoder_workspace exceeds AX_STATIC_SCRATCH_BYTES or out_cap is
 * below the decoded size; AX_E_ARG for null pointers. */
#define AX_STATIC_SCRATCH_BYTES (128ull << 20)
int aceapex_decode_all_static(aceapex_decoder* dec, uint8_t* d_out, uint64_t out_cap, int copy_mode, void* stream);

/* Stage timing of the last decode on this handle (HIP events on `stream`,
 * recorded around the stages of every window and summed), in milliseconds:
 * entropy (rANS of the four streams), parse (commands, literal placement,
 * token emission), copy (the whole match layer); remainder (nullable) is the
 * part of copy spent on the tokens the bulk rounds left.  Blocks on the
 * events. */
int aceapex_decoder_stage_ms(aceapex_decoder* dec, float* ans_ms, float* parse_ms, float* copy_ms,
                             float* remainder_ms);
/* 1 = record stage events on later decodes (five event records per window). */
int aceapex_decoder_set_timing(aceapex_decoder* dec, int enable);

/* Decoder options (schedule knobs; none changes a decoded byte).
 *   AX_OPT_BULK_ROUNDS  number of level-synchronous match-layer rounds (one
 *     launch each, plain cached accesses) before the launches that finish the
 *     deeper tokens, in [1, 250] (default 4).  Until it is set, a decoder
 *     learns it per window from its first decode: a window whose first round
 *     fills less than a tenth of its matches (a deep archive) runs that round
 *     only. */
enum { AX_OPT_BULK_ROUNDS = 1 };
/*   AX_OPT_FILL_ROUNDS / AX_OPT_FILL_TAIL  how a wave fills its ready tokens
 *     in the rounds after the first / in the persistent launch: 0 short
 *     tokens one lane each and long ones by the whole wave, 1 all ready
 *     tokens laid end to end and split evenly over the lanes (defaults 0 / 0).
 *     AX_OPT_FILL_ROUNDS also applies to the first round when it runs as
 *     waves (AX_OPT_ROUND0_TILE = 0). */
enum { AX_OPT_FILL_ROUNDS = 2, AX_OPT_FILL_TAIL = 3 };
/*   AX_OPT_TAIL_CHUNKS  consecutive 64-token chunks a wave of the persistent
 *     launch takes per ticket, in [1, 64] (default 1): fewer tickets (one
 *     global counter) against less overlap of dependent chunks.
 *   AX_OPT_GRAPH  1 = capture the whole launch sequence (every window, stage
 *     and dependency-level round) as a hipGraph on the first decode and
 *     replay it afterwards (re-captured when the workspace, copy mode or an
 *     option changes); stage timing is not recorded in this mode. */
enum { AX_OPT_TAIL_CHUNKS = 4, AX_OPT_GRAPH = 5 };
/*   AX_OPT_ROUND0_TILE  schedule of the first match-layer round: 1 = one
 *     workgroup per block, filling its tokens in a 16 KiB LDS tile written
 *     back as 16-byte stores (default); 0 = one wave per 64 tokens writing
 *     the fills straight to global memory (fill mode AX_OPT_FILL_ROUNDS). */
enum { AX_OPT_ROUND0_TILE = 6 };
/*   AX_OPT_TAIL_MODE  how the tokens left after the bulk rounds (the deep
 *     remainder) are finished: 0 = pointer jumping over their bytes — every
 *     byte names the byte its value comes from, and each of about
 *     log3(chain length) passes replaces that name by the one two steps
 *     along its chain (default); 1 = one persistent launch that copies each token once the
 *     tokens writing its sources are done (one dependency hop at a time; the
 *     serial copy mode always finishes this way).  Range decodes choose by
 *     their closure: the persistent launch below AX_OPT_RANGE_JUMP_TOKENS
 *     matches (4096 by default), jumping above. */
enum { AX_OPT_TAIL_MODE = 7 };
/*   AX_OPT_JUMP_PASSES  0 = automatic: the first decode runs enough passes
 *     for any chain of the window (log3 of its token count), the next ones the
 *     count the device reported as needed plus one (which reports it again),
 *     and once every window's count is known exactly that count; k in
 *     [1, 32] = at most k passes.  The final gather follows whatever entries the passes left, so
 *     the count changes timing only, never a byte. */
enum { AX_OPT_JUMP_PASSES = 8 };
/*   AX_OPT_RANGE_JUMP_TOKENS  range decodes of this decoder finish closures of
 *     at least this many matches by pointer jumping, smaller ones by the
 *     persistent launch (default 4096; 0 = always jump). */
enum { AX_OPT_RANGE_JUMP_TOKENS = 9 };
int aceapex_decoder_set_option(aceapex_decoder* dec, int option, int64_t value);

/* The entropy stage alone (Setup: per-block rANS of the LIT, LEN, OFF and
 * CMD streams) for archive blocks [first, first + count), count at most
 * 131072: their decoded streams copied to h_out (cap bytes), packed block
 * after block in the order LIT, LEN, OFF, CMD; n_syms (4 * count entries)
 * receives each stream's length in that order.  For checking the entropy
 * stage on its own.  d_work: the decode_all workspace.  Synchronous on
 * `stream`.  Errors: AX_E_RANGE (blocks), AX_E_CAPACITY (workspace or
 * h_out too small), the device status code of a corrupt stream. */
int aceapex_decoder_streams(aceapex_decoder* dec, uint64_t first, uint64_t count, void* d_work, uint64_t work_len,
                            void* stream, uint8_t* h_out, uint64_t cap, uint32_t* n_syms);

/* Read the device status word of a workspace after the work queued on
 * `stream`: synchronises `stream`.  *dev_err is 0 or an AX_E_* code;
 * *bad_block is the first failing block (or ~0).  d_work NULL: the static
 * workspace of aceapex_decode_all_static on the current device. */
int aceapex_decoder_status(aceapex_decoder* dec, void* d_work, void* stream, int32_t* dev_err,
                           uint64_t* bad_block);
/* The same for any workspace (decode, batch or range). */
int aceapex_workspace_status(void* d_work, void* stream, int32_t* dev_err, uint64_t* bad_block);

/* --------------------------------------------------------------- batch --- */

/* Batched decode: many whole archives in one plan.  All blocks of all jobs
 * are cut into windows and every window runs as one sequence of launches
 * (entropy, parse, match layer) over device work lists, so the number of
 * launches does not grow with the number of archives; with AX_OPT_GRAPH the
 * whole sequence is one captured graph.  Each job's bytes go to its d_out
 * (16-byte aligned, out_cap >= its decoded size), fixed at creation. */
typedef struct {
  aceapex_decoder* dec;
  uint8_t* d_out;
  uint64_t out_cap;
} aceapex_job;

typedef struct aceapex_batch aceapex_batch;

int aceapex_batch_create(const aceapex_job* jobs, uint32_t n, aceapex_batch** out);
void aceapex_batch_destroy(aceapex_batch* batch);
int aceapex_batch_workspace(const aceapex_batch* batch, uint64_t* bytes);
int aceapex_batch_set_option(aceapex_batch* batch, int option, int64_t value);
int aceapex_batch_set_timing(aceapex_batch* batch, int enable);
int aceapex_batch_stage_ms(aceapex_batch* batch, float* ans_ms, float* parse_ms, float* copy_ms, float* remainder_ms);
/* Decode every job; asynchronous on `stream`; status via
 * aceapex_workspace_status. */
int aceapex_decode_batch(aceapex_batch* batch, void* d_work, uint64_t work_len, int copy_mode, void* stream);

/* -------------------------------------------------------- random access --- */

/* Build the decoder's token index (every match: src, dst, len) on the host,
 * by a device entropy + parse pass over the archive that writes no output
 * bytes (random-access section: the index is what makes a range's source
 * closure computable without decoding the archive).  d_work: the
 * decode_all workspace.  Synchronous; host memory 16 bytes per match. */
int aceapex_decoder_build_index(aceapex_decoder* dec, void* d_work, uint64_t work_len, void* stream);

/* The device parse's matches, from the token index (build it first):
 * matches [first, first + count) in archive order (block b's matches are
 * the index's entries from the cumulative match count of block b, in
 * output order), each its source, destination and length (Setup: absolute
 * source offsets; REP commands appear with the source their distance
 * history resolved to).  For checking the parse stage on its own.  Errors:
 * AX_E_ARG (index not built), AX_E_RANGE. */
int aceapex_decoder_tokens(const aceapex_decoder* dec, uint64_t first, uint64_t count, uint64_t* src, uint64_t* dst,
                           uint32_t* len);

/* Source-closure size of each of n ranges on its own (blocks and matches),
 * on up to `threads` host threads (0: up to 16): what a request needs from a
 * range plan's limits, for admission by scratch memory before any launch.
 * The sizes of several ranges bound the size of their union.  The closures
 * found here are kept by the decoder (bounded) and reused when a later
 * union closure (aceapex_decode_ranges, aceapex_closure_blocks) meets the
 * same range.  Errors: AX_E_ARG (index not built), AX_E_RANGE. */
int aceapex_closure_sizes(const aceapex_decoder* dec, uint32_t n, const uint64_t* offs, const uint64_t* lens,
                          uint64_t* blocks, uint64_t* tokens, uint32_t threads);

/* Byte-precise source closure of n ranges: the ascending union of the blocks
 * holding any byte the ranges need (their own bytes and, transitively, the
 * bytes their matches copy).  blocks may be NULL to only count; *n_tokens
 * (nullable) receives their match count.  Needs the token index.  Closures
 * run on at most `threads` host threads (0 = up to 16), one per 8 ranges at
 * most (at most 64). */
int aceapex_closure_blocks(aceapex_decoder* dec, uint32_t n, const uint64_t* h_offs, const uint64_t* h_lens,
                           uint64_t* h_blocks, uint64_t cap, uint64_t* n_blocks, uint64_t* n_tokens,
                           uint32_t threads);

/* Device workspace (bytes, 256-byte aligned start) that aceapex_decode_range
 * needs for the range [off, off + len): the decode workspace of its source
 * closure, a compact scratch of (closure blocks + 1) * block_size bytes and
 * a slot table of 4 bytes per archive block — sized by the closure, not by
 * the archive (Introduction: decompressing everything leaves nowhere to put
 * it).  Needs the token index.  AX_E_CAPACITY when the closure exceeds one
 * window (131072 blocks or 2^26 matches). */
int aceapex_range_workspace(const aceapex_decoder* dec, uint64_t off, uint64_t len, uint64_t* bytes);

/* Decode the byte range [off, off + len) into d_out[0..len) (device,
 * out_cap >= len): the range's source closure is decoded into the compact
 * scratch inside d_work (at least aceapex_range_workspace bytes) and the
 * range copied out (random-access section: one tile or a range of blocks
 * from a resident archive).  The closure is computed on the host first;
 * the decode is asynchronous on `stream`.  Errors before any launch:
 * AX_E_RANGE (outside the archive), AX_E_CAPACITY (d_out or d_work too
 * small), AX_E_ARG. */
int aceapex_decode_range(aceapex_decoder* dec, uint64_t off, uint64_t len, uint8_t* d_out, uint64_t out_cap,
                         void* d_work, uint64_t work_len, void* stream);

/* A reusable range-decode plan with capacity limits (blocks and matches of
 * one call's union closure, at most 131072 blocks and 2^26 matches): the
 * batched form for serving.  Its workspace size depends only on the limits:
 * the decode workspace for them, a compact scratch of (max_blocks + 1)
 * blocks and the slot table. */
typedef struct aceapex_range_plan aceapex_range_plan;
int aceapex_range_plan_create(aceapex_decoder* dec, uint64_t max_blocks, uint64_t max_tokens,
                              aceapex_range_plan** out);
void aceapex_range_plan_destroy(aceapex_range_plan* rp);
int aceapex_range_plan_workspace(const aceapex_range_plan* rp, uint64_t* bytes);
/* Blocks and matches of the last call's closure. */
int aceapex_range_plan_last(const aceapex_range_plan* rp, uint64_t* blocks, uint64_t* tokens);

/* Decode n byte ranges [h_offs[i], h_offs[i] + h_lens[i]) of the archive:
 * their union closure is decoded into the compact scratch inside d_work and
 * range i is copied to h_d_outs[i] (a host array of device pointers, each
 * with h_out_caps[i] >= h_lens[i] bytes).  The closure is computed on the
 * host before anything is enqueued; the decode and the copies are
 * asynchronous on `stream`.  Errors before any launch: AX_E_CAPACITY when
 * the closure exceeds the plan's limits or an output or the workspace is too
 * small, AX_E_RANGE for a range outside the archive.  Calls sharing d_work
 * must be ordered (same stream). */
int aceapex_decode_ranges(aceapex_range_plan* rp, uint32_t n, const uint64_t* h_offs, const uint64_t* h_lens,
                          uint8_t* const* h_d_outs, const uint64_t* h_out_caps, void* d_work, uint64_t work_len,
                          int copy_mode, void* stream);

#ifdef __cplusplus
}
#endif
#endif
