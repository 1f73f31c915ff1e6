/*
 * axo — the ORACLE for the absolute-offset LZ77 block format ("AXP1").
 *
 * TEST INFRASTRUCTURE ONLY.  A plain, slow, single-threaded CPU encoder and
 * decoder of the format, written to be checked by eye against the paper.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code with the product library and the product
 * never calls it.
 *
 * What it follows:
 *   - Setup: back-references are absolute output positions; the output is
 *     cut into fixed-size blocks; each block carries four streams (literals,
 *     lengths, absolute offsets, commands); a block decodes once the bytes
 *     its sources name exist.
 *   - Depth section: the two-pass forced-literal depth cap, iterated until no
 *     match is deeper than L.
 *   - Periodic-fill section: out[dst+k] = out[src + (k mod dist)] equals the
 *     byte-serial LZ77 copy.
 *   - Last-sequential-element section: a four-entry distance history behind
 *     repeat matches; varint lengths; the history-free (NO_REP) encoding.
 * Byte layout, entropy-coder constants and greedy tie-breaks are readings of
 * the paper where it is silent; they are listed with the format below.
 *
 * Parity status: every function here is pinned by the CPU tests against
 * something other than itself: round trips, closed forms, brute force over
 * the recursive definitions (depth, block levels, closure), hand-derived
 * golden fixtures (history walk, periodic fill, depth chain, block levels)
 * and the paper's invariants.  The encoder statistics n_lit_cmds and
 * n_escapes are pinned by recounting the decoded command streams.
 */
#ifndef AXO_H
#define AXO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { AXO_OK = 0, AXO_E_ARG = -1, AXO_E_CORRUPT = -2, AXO_E_NOMEM = -3, AXO_E_CHECKSUM = -4 };

typedef struct {
  uint32_t block_size;             /* power of two, 4096..65536 */
  uint32_t min_match;              /* 1..255 */
  uint32_t no_rep;                 /* 1: never emit repeat commands */
  uint32_t depth_cap;              /* 0: none; else max chain depth L */
  uint32_t hash_bits;              /* 10..26 */
  uint32_t chain_depth;            /* candidates walked per position */
  uint32_t rans_min_syms_per_lane; /* S in the lane rule */
  uint32_t off_cost_q;             /* an explicit-offset match must be at least
                                      min_match + ceil(off_cost_q * (LEB128 bytes
                                      of src) / 4) long: quarter bytes per byte */
  uint32_t window_log;             /* 0: candidates anywhere behind; else only
                                      those at most 2^window_log bytes behind */
} axo_params;

void axo_params_default(axo_params* p);

/* Encoder statistics.  n_lit_cmds: literal-run commands; n_escapes:
 * commands whose length continues in the length stream. */
typedef struct {
  uint64_t n_bytes, n_blocks, comp_bytes;
  uint64_t n_commands, n_lit_cmds, n_matches, n_rep, n_escapes, n_match_bytes, n_lit_bytes;
  uint64_t n_forced_bytes;
  uint32_t max_depth, passes;
} axo_stats;

/* Encode in[0..n) into a fresh malloc'd container (*out, *out_len).
 * stats may be NULL. */
int axo_encode(const uint8_t* in, uint64_t n, const axo_params* p, uint8_t** out,
               uint64_t* out_len, axo_stats* stats);

/* As axo_encode, and when forced_out is not NULL it receives one byte per
 * input position: 1 where the depth cap forced the position to literal. */
int axo_encode_ex(const uint8_t* in, uint64_t n, const axo_params* p, uint8_t** out,
                  uint64_t* out_len, axo_stats* stats, uint8_t* forced_out);

/* One command of an explicit command list (assembler / parse dump).
 * kind: 0 LIT, 1 MATCH, 2 REP.  For REP, rep = history index 0..3.
 * dst/src are absolute output positions; lit_pos is the index of the first
 * literal byte in the block's literal stream. */
typedef struct {
  uint64_t dst, src;
  uint32_t len, lit_pos;
  uint8_t kind, rep, pad[6];
} axo_cmd;

/* Build a container from `data` (the intended output) and a command list
 * in output order.  Commands may not cross block boundaries; MATCH takes its
 * src from cmds[i].src, REP its history index from cmds[i].rep.  Used to
 * construct adversarial but valid archives. */
int axo_assemble(const uint8_t* data, uint64_t n, const axo_cmd* cmds, uint64_t n_cmds,
                 const axo_params* p, uint8_t** out, uint64_t* out_len);

void axo_free(void* ptr);

/* Container header fields. */
typedef struct {
  uint64_t n_bytes, n_blocks, xxh3, payload_bytes, n_matches, archive_bytes;
  uint32_t block_size, min_match, flags, depth_cap;
} axo_info;
int axo_read_info(const uint8_t* arc, uint64_t len, axo_info* info);

/* Sequential decode of the whole archive into out[0..n_bytes).
 * copy_mode 0: byte-serial LZ77 copy; 1: periodic form src + (k mod dist).
 * verify_xxh3: compare XXH3-64 of the output with the header. */
int axo_decode(const uint8_t* arc, uint64_t len, uint8_t* out, uint64_t out_cap,
               int copy_mode, int verify_xxh3);

/* Decoded streams of one block (caller buffers of at least block_size bytes
 * for lit and cmd, and of *_cap for off/len). Sizes returned through n_*. */
int axo_block_streams(const uint8_t* arc, uint64_t len, uint64_t block,
                      uint8_t* lit, uint32_t* n_lit, uint8_t* lenb, uint32_t* n_len,
                      uint32_t len_cap, uint8_t* off, uint32_t* n_off, uint32_t off_cap,
                      uint8_t* cmd, uint32_t* n_cmd);

/* Sequential parse of one block: commands with dst, len, lit_pos, src. */
int axo_block_parse(const uint8_t* arc, uint64_t len, uint64_t block, axo_cmd* cmds,
                    uint64_t cap, uint64_t* n_cmds);

/* Every command of the archive in output order (the block parse of each
 * block, concatenated); *cmds is allocated here, release with axo_free. */
int axo_parse_all(const uint8_t* arc, uint64_t len, axo_cmd** cmds, uint64_t* n_cmds);

/* Chain depth of every match (MATCH and REP, archive order) and the maximum.
 * depth = 0 when every source byte was written by a literal command, else
 * 1 + the deepest match that wrote a source byte. Source set of a match:
 * [src, src + min(len, dist)). */
int axo_depths(const uint8_t* arc, uint64_t len, uint32_t* depth, uint64_t cap,
               uint32_t* max_depth);

/* Dependency levels at block granularity:
 *  raw:          blvl(b) = 0 if all sources of b lie in b, else 1 + max blvl
 *                of the other blocks its sources touch;
 *  match-sourced: the same, counting only bytes of other blocks that were
 *                written by matches.
 * Returns the maxima, and when raw_lvl / msrc_lvl are not NULL the level of
 * every block (n_blocks entries each). */
int axo_block_levels(const uint8_t* arc, uint64_t len, uint32_t* raw_max, uint32_t* msrc_max, uint32_t* raw_lvl,
                     uint32_t* msrc_lvl);

/* Byte-precise source closure of the output range [off, off+n): marks in
 * block_mask[] (one byte per block) every block whose bytes are needed to
 * produce the range. Returns the number of marked blocks via *n_marked. */
int axo_closure(const uint8_t* arc, uint64_t len, uint64_t off, uint64_t n, uint8_t* block_mask,
                uint64_t* n_marked);

/* rANS stream codec, exposed for the round-trip pins.
 * Encodes sym[0..n) into a stream record (mode chosen by the mode rule unless
 * force_rans); decode reads one record back.  Both return AXO_* codes. */
int axo_stream_encode(const uint8_t* sym, uint32_t n, uint32_t min_syms_per_lane, int force_rans,
                      int force_lanes_log2, uint8_t** rec, uint32_t* rec_len);
int axo_stream_decode(const uint8_t* rec, uint32_t rec_len, uint8_t* out, uint32_t cap,
                      uint32_t* n_out, uint32_t* used);

/* LEB128 helpers (unsigned, minimal form on encode; at most 10 bytes). */
uint32_t axo_leb_put(uint64_t v, uint8_t* out);
int axo_leb_get(const uint8_t* in, uint32_t avail, uint64_t* v, uint32_t* used);

/* The two copy forms, for the periodic-fill pin. */
void axo_copy_serial(uint8_t* buf, uint64_t dst, uint64_t src, uint64_t len);
void axo_copy_periodic(uint8_t* buf, uint64_t dst, uint64_t src, uint64_t len);

#ifdef __cplusplus
}
#endif
#endif
