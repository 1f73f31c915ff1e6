/*
 * axo.c — ORACLE (test infrastructure only; see axo.h).
 *
 * Plain single-threaded C.  Nothing here is blocked, fused or reordered:
 * every loop walks the data in the order the format defines.
 *
 * FORMAT "AXP1" (little-endian).  The paper fixes absolute offsets, fixed
 * blocks and four streams per block (Setup), a four-entry distance history
 * and varint lengths (last-sequential-element section); the bytes below are
 * this implementation's reading where the paper is silent.
 *
 *   header (64 B)
 *     0 u32 magic "AXP1"   4 u16 version=1   6 u16 flags (1 NO_REP, 2 DEPTH_CAPPED)
 *     8 u32 block_size    12 u16 min_match  14 u16 depth_cap
 *    16 u64 n_bytes       24 u64 n_blocks   32 u64 xxh3_64(original)
 *    40 u64 payload_bytes 48 u64 n_matches  56 u64 0
 *   index: (n_blocks+1) u64 payload offsets (16-aligned, relative to payload)
 *          (n_blocks+1) u64 cumulative match counts (MATCH + REP commands)
 *   payload: per block  u32 rec_size[4]; records LIT, LEN, OFF, CMD; pad to 16
 *   stream record (4-aligned):
 *     u32 n_sym; u8 mode (0 RAW, 1 CONST, 2 RANS); u8 a; u8 b; u8 0
 *     RAW   n_sym bytes, pad 4
 *     CONST a = the symbol
 *     RANS  a = log2 K (K lanes, K <= 64), b = n_present - 1;
 *           u32 n_words; K u32 final states; n_words u16 words; pad 4;
 *           present symbols (ascending list if n_present <= 32, else a 32-B
 *           bitmap); pad 2; n_present u16 frequencies; pad 4
 *   rANS: 12-bit probabilities (sum 4096), 32-bit states, 16-bit
 *     renormalisation words, lower bound 2^16.  Lane j owns symbols i = j
 *     (mod K); words are read in symbol order.  After the last symbol every
 *     state is 2^16 and every word has been read.
 *   command byte c, kind = c & 3:
 *     0 LIT    len = (c>>2)+1, or 64 + LEB(LEN) when c>>2 == 63
 *     1 MATCH  len = (c>>2)+mm, or 63+mm + LEB(LEN) when c>>2 == 63;
 *              src = LEB(OFF), an absolute output position < dst
 *     2 REP    r = (c>>2)&3; len = (c>>4)+mm, or 15+mm + LEB(LEN) when
 *              c>>4 == 15; src = dst - h[r]
 *     3        invalid
 *   history h[4] of distances, (1,2,3,4) at every block start;
 *     MATCH pushes dst-src to the front, REP r moves h[r] to the front.
 */
#include "axo.h"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

extern unsigned long long XXH3_64bits(const void* data, size_t len); /* libxxhash */

#define MAGIC 0x31505841u
#define PROB_BITS 12
#define PROB_SCALE (1u << PROB_BITS)
#define RANS_L (1u << 16)
#define MAX_LANES_LOG2 6

void axo_free(void* p) { free(p); }

void axo_params_default(axo_params* p) {
  p->block_size = 16384;
  p->min_match = 4;
  p->no_rep = 0;
  p->depth_cap = 0;
  p->hash_bits = 22;
  p->chain_depth = 32;
  p->rans_min_syms_per_lane = 32;
  p->off_cost_q = 6;
  p->window_log = 0;
}

/* ------------------------------------------------------------ buffers --- */

typedef struct {
  uint8_t* p;
  uint64_t n, cap;
  int oom;
} buf_t;

static void buf_reserve(buf_t* b, uint64_t extra) {
  if (b->oom) return;
  if (b->n + extra <= b->cap) return;
  uint64_t c = b->cap ? b->cap : 256;
  while (c < b->n + extra) c *= 2;
  uint8_t* q = (uint8_t*)realloc(b->p, c);
  if (!q) { b->oom = 1; return; }
  b->p = q;
  b->cap = c;
}
static void buf_put(buf_t* b, const void* d, uint64_t n) {
  buf_reserve(b, n);
  if (b->oom) return;
  memcpy(b->p + b->n, d, n);
  b->n += n;
}
static void buf_u8(buf_t* b, uint8_t v) { buf_put(b, &v, 1); }
static void buf_u16(buf_t* b, uint16_t v) { uint8_t t[2] = {(uint8_t)v, (uint8_t)(v >> 8)}; buf_put(b, t, 2); }
static void buf_u32(buf_t* b, uint32_t v) {
  uint8_t t[4];
  for (int i = 0; i < 4; i++) t[i] = (uint8_t)(v >> (8 * i));
  buf_put(b, t, 4);
}
static void buf_u64(buf_t* b, uint64_t v) {
  uint8_t t[8];
  for (int i = 0; i < 8; i++) t[i] = (uint8_t)(v >> (8 * i));
  buf_put(b, t, 8);
}
static void buf_pad(buf_t* b, uint64_t a) { while (b->n % a) buf_u8(b, 0); }

static uint16_t rd16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t rd32(const uint8_t* p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24); }
static uint64_t rd64(const uint8_t* p) { return (uint64_t)rd32(p) | ((uint64_t)rd32(p + 4) << 32); }

/* ------------------------------------------------------------- LEB128 --- */

uint32_t axo_leb_put(uint64_t v, uint8_t* out) {
  uint32_t n = 0;
  do {
    uint8_t byte = (uint8_t)(v & 0x7F);
    v >>= 7;
    if (v) byte |= 0x80;
    out[n++] = byte;
  } while (v);
  return n;
}

int axo_leb_get(const uint8_t* in, uint32_t avail, uint64_t* v, uint32_t* used) {
  uint64_t r = 0;
  for (uint32_t i = 0; i < 10; i++) {
    if (i >= avail) return AXO_E_CORRUPT;
    uint8_t byte = in[i];
    if (i == 9 && byte > 1) return AXO_E_CORRUPT; /* would overflow 64 bits */
    r |= (uint64_t)(byte & 0x7F) << (7 * i);
    if (!(byte & 0x80)) { *v = r; *used = i + 1; return AXO_OK; }
  }
  return AXO_E_CORRUPT;
}

static void buf_leb(buf_t* b, uint64_t v) {
  uint8_t t[10];
  buf_put(b, t, axo_leb_put(v, t));
}

/* --------------------------------------------------------------- rANS --- */

/* Scale counts to frequencies summing to 4096 (every present symbol >= 1).
 * Deficit goes to the most frequent symbol (ties: smallest byte); an excess
 * is removed one unit at a time, round robin over the symbols in descending
 * frequency order (ties: smallest byte), never below 1. */
static void normalize(const uint64_t cnt[256], uint64_t n, uint32_t f[256]) {
  uint64_t sum = 0;
  int top = -1;
  for (int s = 0; s < 256; s++) {
    f[s] = 0;
    if (!cnt[s]) continue;
    uint64_t v = cnt[s] * PROB_SCALE / n;
    f[s] = v < 1 ? 1 : (uint32_t)v;
    sum += f[s];
    if (top < 0 || cnt[s] > cnt[top]) top = s;
  }
  if (sum < PROB_SCALE) f[top] += (uint32_t)(PROB_SCALE - sum);
  if (sum > PROB_SCALE) {
    int order[256], m = 0;
    for (int s = 0; s < 256; s++) if (cnt[s]) order[m++] = s;
    for (int i = 1; i < m; i++) { /* insertion sort: f desc, byte asc */
      int x = order[i], j = i - 1;
      while (j >= 0 && (f[order[j]] < f[x] || (f[order[j]] == f[x] && order[j] > x))) { order[j + 1] = order[j]; j--; }
      order[j + 1] = x;
    }
    int k = 0;
    while (sum > PROB_SCALE) {
      int s = order[k];
      if (f[s] > 1) { f[s]--; sum--; }
      k = (k + 1) % m;
    }
  }
}

static uint32_t lanes_log2_for(uint32_t n, uint32_t S) {
  uint32_t lim = n > S ? n : S, lg = 0;
  while (lg < MAX_LANES_LOG2 && ((uint64_t)(1u << (lg + 1)) * S) <= lim) lg++;
  return lg;
}

static uint64_t pad_to(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

int axo_stream_encode(const uint8_t* sym, uint32_t n, uint32_t S, int force_rans, int force_lanes_log2,
                      uint8_t** rec, uint32_t* rec_len) {
  buf_t b = {0};
  uint64_t cnt[256] = {0};
  for (uint32_t i = 0; i < n; i++) cnt[sym[i]]++;
  uint32_t present = 0;
  for (int s = 0; s < 256; s++) present += cnt[s] != 0;
  uint64_t raw_size = pad_to(8 + (uint64_t)n, 4);
  if (n >= 1 && present == 1 && !force_rans) { /* CONST */
    buf_u32(&b, n); buf_u8(&b, 1); buf_u8(&b, sym[0]); buf_u8(&b, 0); buf_u8(&b, 0);
    goto done;
  }
  if (present >= 2) {
    if (S == 0) S = 1;
    uint32_t lg = force_lanes_log2 >= 0 ? (uint32_t)force_lanes_log2 : lanes_log2_for(n, S);
    if (lg > MAX_LANES_LOG2) return AXO_E_ARG;
    uint32_t K = 1u << lg;
    uint32_t f[256], c[256];
    normalize(cnt, n, f);
    uint32_t acc = 0;
    for (int s = 0; s < 256; s++) { c[s] = acc; acc += f[s]; }
    uint32_t x[64];
    for (uint32_t j = 0; j < K; j++) x[j] = RANS_L;
    uint16_t* words = (uint16_t*)malloc(((uint64_t)n + 1) * sizeof(uint16_t));
    if (!words) return AXO_E_NOMEM;
    uint64_t nw = 0;
    for (uint64_t ii = n; ii-- > 0;) { /* encode backwards */
      uint32_t j = (uint32_t)(ii % K), s = sym[ii];
      uint64_t xmax = ((uint64_t)(RANS_L >> PROB_BITS) << 16) * f[s];
      if (x[j] >= xmax) { words[nw++] = (uint16_t)(x[j] & 0xFFFF); x[j] >>= 16; }
      x[j] = ((x[j] / f[s]) << PROB_BITS) + (x[j] % f[s]) + c[s];
    }
    uint64_t set_bytes = present <= 32 ? present : 32;
    uint64_t rans_size = pad_to(pad_to(pad_to(12 + 4ull * K + 2 * nw, 4) + set_bytes, 2) + 2ull * present, 4);
    if (force_rans || rans_size < raw_size) {
      buf_u32(&b, n); buf_u8(&b, 2); buf_u8(&b, (uint8_t)lg); buf_u8(&b, (uint8_t)(present - 1)); buf_u8(&b, 0);
      buf_u32(&b, (uint32_t)nw);
      for (uint32_t j = 0; j < K; j++) buf_u32(&b, x[j]);
      for (uint64_t w = nw; w-- > 0;) buf_u16(&b, words[w]); /* decoder read order */
      buf_pad(&b, 4);
      if (present <= 32) {
        for (int s = 0; s < 256; s++) if (cnt[s]) buf_u8(&b, (uint8_t)s);
      } else {
        uint8_t bm[32] = {0};
        for (int s = 0; s < 256; s++) if (cnt[s]) bm[s >> 3] |= (uint8_t)(1u << (s & 7));
        buf_put(&b, bm, 32);
      }
      buf_pad(&b, 2);
      for (int s = 0; s < 256; s++) if (cnt[s]) buf_u16(&b, (uint16_t)f[s]);
      buf_pad(&b, 4);
      free(words);
      goto done;
    }
    free(words);
  }
  /* RAW */
  buf_u32(&b, n); buf_u8(&b, 0); buf_u8(&b, 0); buf_u8(&b, 0); buf_u8(&b, 0);
  buf_put(&b, sym, n);
  buf_pad(&b, 4);
done:
  if (b.oom) { free(b.p); return AXO_E_NOMEM; }
  *rec = b.p;
  *rec_len = (uint32_t)b.n;
  return AXO_OK;
}

int axo_stream_decode(const uint8_t* rec, uint32_t len, uint8_t* out, uint32_t cap, uint32_t* n_out,
                      uint32_t* used) {
  if (len < 8) return AXO_E_CORRUPT;
  uint32_t n = rd32(rec);
  uint8_t mode = rec[4], a = rec[5], bb = rec[6];
  if (n > cap) return AXO_E_CORRUPT;
  *n_out = n;
  if (mode == 0) {
    uint64_t sz = pad_to(8 + (uint64_t)n, 4);
    if (sz > len) return AXO_E_CORRUPT;
    memcpy(out, rec + 8, n);
    *used = (uint32_t)sz;
    return AXO_OK;
  }
  if (mode == 1) {
    memset(out, a, n);
    *used = 8;
    return AXO_OK;
  }
  if (mode != 2) return AXO_E_CORRUPT;
  if (a > MAX_LANES_LOG2) return AXO_E_CORRUPT;
  uint32_t K = 1u << a, present = (uint32_t)bb + 1;
  if (present < 2 || len < 12) return AXO_E_CORRUPT;
  uint32_t nw = rd32(rec + 8);
  uint64_t p = 12;
  if (p + 4ull * K > len) return AXO_E_CORRUPT;
  uint32_t x[64];
  for (uint32_t j = 0; j < K; j++) { x[j] = rd32(rec + p + 4 * j); if (x[j] < RANS_L) return AXO_E_CORRUPT; }
  p += 4ull * K;
  uint64_t wpos = p;
  p = pad_to(p + 2ull * nw, 4);
  if (p > len) return AXO_E_CORRUPT;
  uint8_t syms[256];
  if (present <= 32) {
    if (p + present > len) return AXO_E_CORRUPT;
    for (uint32_t i = 0; i < present; i++) {
      syms[i] = rec[p + i];
      if (i && syms[i] <= syms[i - 1]) return AXO_E_CORRUPT;
    }
    p += present;
  } else {
    if (p + 32 > len) return AXO_E_CORRUPT;
    uint32_t m = 0;
    for (int s = 0; s < 256; s++) if (rec[p + (s >> 3)] >> (s & 7) & 1) { if (m < 256) syms[m] = (uint8_t)s; m++; }
    if (m != present) return AXO_E_CORRUPT;
    p += 32;
  }
  p = pad_to(p, 2);
  if (p + 2ull * present > len) return AXO_E_CORRUPT;
  uint32_t f[256] = {0}, c[256] = {0}, total = 0;
  uint8_t slot2sym[PROB_SCALE];
  for (uint32_t i = 0; i < present; i++) {
    uint32_t fi = rd16(rec + p + 2 * i);
    if (fi < 1 || fi > PROB_SCALE - 1 || total + fi > PROB_SCALE) return AXO_E_CORRUPT;
    f[syms[i]] = fi;
    c[syms[i]] = total;
    for (uint32_t k = 0; k < fi; k++) slot2sym[total + k] = syms[i];
    total += fi;
  }
  if (total != PROB_SCALE) return AXO_E_CORRUPT;
  p = pad_to(p + 2ull * present, 4);
  if (p > len) return AXO_E_CORRUPT;
  uint32_t ptr = 0;
  for (uint32_t i = 0; i < n; i++) { /* symbol order = (step, lane) order */
    uint32_t j = i % K;
    uint32_t slot = x[j] & (PROB_SCALE - 1);
    uint8_t s = slot2sym[slot];
    uint32_t v = f[s] * (x[j] >> PROB_BITS) + slot - c[s];
    if (v < RANS_L) {
      if (ptr >= nw) return AXO_E_CORRUPT;
      v = (v << 16) | rd16(rec + wpos + 2ull * ptr);
      ptr++;
    }
    x[j] = v;
    out[i] = s;
  }
  if (ptr != nw) return AXO_E_CORRUPT;
  for (uint32_t j = 0; j < K; j++) if (x[j] != RANS_L) return AXO_E_CORRUPT;
  *used = (uint32_t)p;
  return AXO_OK;
}

/* ---------------------------------------------------------- container --- */

typedef struct {
  buf_t lit, len, off, cmd;
  uint64_t n_matches, n_lit_cmds, n_escapes;
} blockstreams_t;

static void bs_reset(blockstreams_t* s) {
  s->lit.n = s->len.n = s->off.n = s->cmd.n = 0;
  s->n_matches = s->n_lit_cmds = s->n_escapes = 0;
}
static void bs_free(blockstreams_t* s) { free(s->lit.p); free(s->len.p); free(s->off.p); free(s->cmd.p); }
static int bs_oom(const blockstreams_t* s) { return s->lit.oom || s->len.oom || s->off.oom || s->cmd.oom; }

/* Append one command to the block's streams. LIT bytes come from lits. */
static void emit_lit(blockstreams_t* s, const uint8_t* lits, uint64_t len) {
  buf_put(&s->lit, lits, len);
  if (len - 1 < 63) buf_u8(&s->cmd, (uint8_t)((len - 1) << 2));
  else { buf_u8(&s->cmd, (uint8_t)(63 << 2)); buf_leb(&s->len, len - 64); s->n_escapes++; }
  s->n_lit_cmds++;
}
static void emit_match(blockstreams_t* s, uint64_t src, uint64_t len, uint32_t mm) {
  if (len - mm < 63) buf_u8(&s->cmd, (uint8_t)(1 | ((len - mm) << 2)));
  else { buf_u8(&s->cmd, (uint8_t)(1 | (63 << 2))); buf_leb(&s->len, len - 63 - mm); s->n_escapes++; }
  buf_leb(&s->off, src);
  s->n_matches++;
}
static void emit_rep(blockstreams_t* s, uint32_t r, uint64_t len, uint32_t mm) {
  if (len - mm < 15) buf_u8(&s->cmd, (uint8_t)(2 | (r << 2) | ((len - mm) << 4)));
  else { buf_u8(&s->cmd, (uint8_t)(2 | (r << 2) | (15 << 4))); buf_leb(&s->len, len - 15 - mm); s->n_escapes++; }
  s->n_matches++;
}

/* Serialise one block's four streams into the payload. */
static int write_block(buf_t* pay, const blockstreams_t* s, uint32_t S) {
  const buf_t* st[4] = {&s->lit, &s->len, &s->off, &s->cmd};
  uint8_t* rec[4] = {0};
  uint32_t rl[4];
  int rc = AXO_OK;
  for (int k = 0; k < 4; k++) {
    rc = axo_stream_encode(st[k]->p, (uint32_t)st[k]->n, S, 0, -1, &rec[k], &rl[k]);
    if (rc) goto out;
  }
  for (int k = 0; k < 4; k++) buf_u32(pay, rl[k]);
  for (int k = 0; k < 4; k++) buf_put(pay, rec[k], rl[k]);
  buf_pad(pay, 16);
out:
  for (int k = 0; k < 4; k++) free(rec[k]);
  return rc;
}

static int finish_container(const uint8_t* in, uint64_t n, const axo_params* p, uint16_t flags,
                            buf_t* pay, const uint64_t* offs, const uint64_t* mpre, uint64_t nb,
                            uint8_t** out, uint64_t* out_len) {
  buf_t c = {0};
  buf_u32(&c, MAGIC); buf_u16(&c, 1); buf_u16(&c, flags);
  buf_u32(&c, p->block_size); buf_u16(&c, (uint16_t)p->min_match); buf_u16(&c, (uint16_t)p->depth_cap);
  buf_u64(&c, n); buf_u64(&c, nb); buf_u64(&c, (uint64_t)XXH3_64bits(in, n));
  buf_u64(&c, pay->n); buf_u64(&c, mpre[nb]); buf_u64(&c, 0);
  for (uint64_t b = 0; b <= nb; b++) buf_u64(&c, offs[b]);
  for (uint64_t b = 0; b <= nb; b++) buf_u64(&c, mpre[b]);
  buf_put(&c, pay->p, pay->n);
  if (c.oom) { free(c.p); return AXO_E_NOMEM; }
  *out = c.p;
  *out_len = c.n;
  return AXO_OK;
}

static int check_params(const axo_params* p) {
  if (p->block_size < 4096 || p->block_size > 65536 || (p->block_size & (p->block_size - 1))) return AXO_E_ARG;
  if (p->min_match < 1 || p->min_match > 255) return AXO_E_ARG;
  if (p->hash_bits < 10 || p->hash_bits > 26) return AXO_E_ARG;
  if (p->window_log > 40) return AXO_E_ARG;
  if (p->off_cost_q > 4096) return AXO_E_ARG;
  return AXO_OK;
}

/* ------------------------------------------------------------ encoder --- */

static uint32_t hash4(const uint8_t* q, uint32_t bits) {
  uint32_t v = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16) | ((uint32_t)q[3] << 24);
  return (uint32_t)(v * 2654435761u) >> (32 - bits);
}

static uint64_t match_len(const uint8_t* in, uint64_t s, uint64_t p, uint64_t maxlen) {
  uint64_t k = 0;
  while (k < maxlen && in[s + k] == in[p + k]) k++;
  return k;
}

/* One greedy pass (C3 reading): forced[] marks positions that must be
 * literal; candidates stop before the first forced position. */
static int encode_pass(const uint8_t* in, uint64_t n, const axo_params* p, const uint8_t* forced,
                       uint8_t** out, uint64_t* out_len, axo_stats* st) {
  uint64_t B = p->block_size, nb = (n + B - 1) / B, mm = p->min_match;
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) << p->hash_bits);
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * (n ? n : 1));
  uint64_t* offs = (uint64_t*)malloc(sizeof(uint64_t) * (nb + 1));
  uint64_t* mpre = (uint64_t*)malloc(sizeof(uint64_t) * (nb + 1));
  blockstreams_t s;
  memset(&s, 0, sizeof(s));
  buf_t pay = {0};
  int rc = AXO_OK;
  if (!head || !prev || !offs || !mpre) { rc = AXO_E_NOMEM; goto out; }
  for (uint64_t i = 0; i < (1ull << p->hash_bits); i++) head[i] = -1;
  uint64_t ins = 0; /* next position to insert into the chains */
  mpre[0] = 0;
  for (uint64_t b = 0; b < nb; b++) {
    uint64_t bs = b * B, be = bs + B < n ? bs + B : n;
    uint64_t h[4] = {1, 2, 3, 4};
    uint64_t pos = bs, lit_start = bs, fcur = bs;
    bs_reset(&s);
    offs[b] = pay.n;
    while (pos < be) {
      uint64_t maxlen = be - pos;
      if (forced) {
        if (fcur < pos) fcur = pos;
        while (fcur < be && !forced[fcur]) fcur++;
        if (fcur - pos < maxlen) maxlen = fcur - pos;
      }
      while (ins < pos && ins + 4 <= n) { /* chain state never depends on the parse */
        uint32_t hv = hash4(in + ins, p->hash_bits);
        prev[ins] = head[hv];
        head[hv] = (int64_t)ins;
        ins++;
      }
      uint64_t lrep = 0, labs = 0, src_abs = 0;
      uint32_t rbest = 0;
      if (!p->no_rep) {
        for (uint32_t r = 0; r < 4; r++) {
          if (h[r] > pos) continue;
          uint64_t l = match_len(in, pos - h[r], pos, maxlen);
          if (l > lrep) { lrep = l; rbest = r; }
        }
      }
      if (pos + 4 <= n && maxlen > 0) {
        int64_t cand = head[hash4(in + pos, p->hash_bits)];
        uint64_t win = p->window_log ? (1ull << p->window_log) : 0;
        for (uint32_t c = 0; c < p->chain_depth && cand >= 0; c++) {
          if (win && (uint64_t)cand + win < pos) break; /* outside the window */
          uint64_t l = match_len(in, (uint64_t)cand, pos, maxlen);
          if (l > labs) { labs = l; src_abs = (uint64_t)cand; }
          if (l == maxlen) break;
          cand = prev[cand];
        }
      }
      /* An explicit match pays for its absolute offset: it must be at least
       * min_match + ceil(off_cost_q * (LEB128 bytes of src) / 4).  A
       * repeat match sends no offset and needs only min_match. */
      uint8_t lb[10];
      uint64_t need_abs = mm + ((uint64_t)p->off_cost_q * axo_leb_put(src_abs, lb) + 3) / 4;
      int take_rep = lrep >= mm && lrep >= labs;
      int take_abs = !take_rep && labs >= need_abs;
      if (!take_rep && !take_abs) { pos++; continue; }
      if (pos > lit_start) emit_lit(&s, in + lit_start, pos - lit_start);
      if (take_rep) {
        emit_rep(&s, rbest, lrep, (uint32_t)mm);
        uint64_t d = h[rbest];
        for (uint32_t k = rbest; k > 0; k--) h[k] = h[k - 1];
        h[0] = d;
        pos += lrep;
        if (st) { st->n_rep++; st->n_match_bytes += lrep; }
      } else {
        emit_match(&s, src_abs, labs, (uint32_t)mm);
        h[3] = h[2]; h[2] = h[1]; h[1] = h[0]; h[0] = pos - src_abs;
        pos += labs;
        if (st) st->n_match_bytes += labs;
      }
      lit_start = pos;
    }
    if (pos > lit_start) emit_lit(&s, in + lit_start, pos - lit_start);
    if (bs_oom(&s)) { rc = AXO_E_NOMEM; goto out; }
    if (st) {
      st->n_commands += s.cmd.n;
      st->n_lit_cmds += s.n_lit_cmds;
      st->n_escapes += s.n_escapes;
      st->n_matches += s.n_matches;
      st->n_lit_bytes += s.lit.n;
    }
    mpre[b + 1] = mpre[b] + s.n_matches;
    rc = write_block(&pay, &s, p->rans_min_syms_per_lane);
    if (rc) goto out;
  }
  offs[nb] = pay.n;
  if (pay.oom) { rc = AXO_E_NOMEM; goto out; }
  {
    uint16_t flags = (uint16_t)((p->no_rep ? 1 : 0) | (p->depth_cap ? 2 : 0));
    rc = finish_container(in, n, p, flags, &pay, offs, mpre, nb, out, out_len);
  }
out:
  free(head); free(prev); free(offs); free(mpre); free(pay.p);
  bs_free(&s);
  return rc;
}

static int walk_all(const uint8_t* arc, uint64_t len, axo_cmd** cmds, uint64_t* n_cmds);
static int depths_of(const uint8_t* arc, uint64_t len, const axo_cmd* cmds, uint64_t nc, uint64_t n,
                     uint32_t* depth_per_cmd, uint32_t* maxd);

int axo_encode(const uint8_t* in, uint64_t n, const axo_params* p, uint8_t** out, uint64_t* out_len,
               axo_stats* st) {
  return axo_encode_ex(in, n, p, out, out_len, st, NULL);
}

int axo_encode_ex(const uint8_t* in, uint64_t n, const axo_params* p, uint8_t** out, uint64_t* out_len,
                  axo_stats* st, uint8_t* forced_out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (st) memset(st, 0, sizeof(*st));
  axo_stats tmp;
  if (forced_out) memset(forced_out, 0, n);
  if (!p->depth_cap) {
    rc = encode_pass(in, n, p, NULL, out, out_len, st ? st : &tmp);
    if (!rc && st) { st->n_bytes = n; st->n_blocks = (n + p->block_size - 1) / p->block_size; st->comp_bytes = *out_len; st->passes = 1; }
    return rc;
  }
  /* depth cap L: encode, derive depths, force the spans of matches deeper
   * than L to literal, re-encode; repeat until no match is deeper than L. */
  uint8_t* forced = (uint8_t*)calloc(n ? n : 1, 1);
  if (!forced) return AXO_E_NOMEM;
  uint32_t passes = 0;
  for (;;) {
    uint8_t* arc = NULL;
    uint64_t alen = 0;
    if (st) memset(st, 0, sizeof(*st));
    rc = encode_pass(in, n, p, forced, &arc, &alen, st ? st : &tmp);
    if (rc) break;
    passes++;
    axo_cmd* cmds = NULL;
    uint64_t nc = 0;
    rc = walk_all(arc, alen, &cmds, &nc);
    uint32_t* dep = rc ? NULL : (uint32_t*)malloc(sizeof(uint32_t) * (nc ? nc : 1));
    uint32_t maxd = 0;
    if (!rc && !dep) rc = AXO_E_NOMEM;
    if (!rc) rc = depths_of(arc, alen, cmds, nc, n, dep, &maxd);
    if (rc) { free(cmds); free(dep); free(arc); break; }
    if (maxd <= p->depth_cap) {
      free(cmds); free(dep);
      *out = arc;
      *out_len = alen;
      if (st) {
        st->max_depth = maxd; st->passes = passes; st->n_bytes = n;
        st->n_blocks = (n + p->block_size - 1) / p->block_size; st->comp_bytes = alen;
        uint64_t fb = 0;
        for (uint64_t i = 0; i < n; i++) fb += forced[i];
        st->n_forced_bytes = fb;
      }
      if (forced_out) memcpy(forced_out, forced, n);
      break;
    }
    for (uint64_t i = 0; i < nc; i++)
      if (cmds[i].kind != 0 && dep[i] > p->depth_cap)
        for (uint64_t k = 0; k < cmds[i].len; k++) forced[cmds[i].dst + k] = 1;
    free(cmds); free(dep); free(arc);
  }
  free(forced);
  return rc;
}

int axo_assemble(const uint8_t* data, uint64_t n, const axo_cmd* cmds, uint64_t n_cmds, const axo_params* p,
                 uint8_t** out, uint64_t* out_len) {
  int rc = check_params(p);
  if (rc) return rc;
  uint64_t B = p->block_size, nb = (n + B - 1) / B, mm = p->min_match;
  uint64_t* offs = (uint64_t*)malloc(sizeof(uint64_t) * (nb + 1));
  uint64_t* mpre = (uint64_t*)malloc(sizeof(uint64_t) * (nb + 1));
  blockstreams_t s;
  memset(&s, 0, sizeof(s));
  buf_t pay = {0};
  if (!offs || !mpre) { rc = AXO_E_NOMEM; goto out; }
  uint64_t ci = 0, pos = 0;
  mpre[0] = 0;
  for (uint64_t b = 0; b < nb; b++) {
    uint64_t be = (b + 1) * B < n ? (b + 1) * B : n;
    bs_reset(&s);
    offs[b] = pay.n;
    while (pos < be) {
      if (ci >= n_cmds) { rc = AXO_E_ARG; goto out; }
      const axo_cmd* c = &cmds[ci++];
      if (c->dst != pos || c->len == 0 || pos + c->len > be) { rc = AXO_E_ARG; goto out; }
      if (c->kind == 0) emit_lit(&s, data + pos, c->len);
      else if (c->kind == 1) {
        if (c->len < mm || c->src >= pos) { rc = AXO_E_ARG; goto out; }
        emit_match(&s, c->src, c->len, (uint32_t)mm);
      } else if (c->kind == 2) {
        if (c->len < mm || c->rep > 3) { rc = AXO_E_ARG; goto out; }
        emit_rep(&s, c->rep, c->len, (uint32_t)mm);
      } else { rc = AXO_E_ARG; goto out; }
      pos += c->len;
    }
    if (bs_oom(&s)) { rc = AXO_E_NOMEM; goto out; }
    mpre[b + 1] = mpre[b] + s.n_matches;
    rc = write_block(&pay, &s, p->rans_min_syms_per_lane);
    if (rc) goto out;
  }
  if (ci != n_cmds) { rc = AXO_E_ARG; goto out; }
  offs[nb] = pay.n;
  if (pay.oom) { rc = AXO_E_NOMEM; goto out; }
  rc = finish_container(data, n, p, (uint16_t)(p->no_rep ? 1 : 0), &pay, offs, mpre, nb, out, out_len);
out:
  free(offs); free(mpre); free(pay.p);
  bs_free(&s);
  return rc;
}

/* ------------------------------------------------------------ decoder --- */

int axo_read_info(const uint8_t* arc, uint64_t len, axo_info* info) {
  if (len < 64 || rd32(arc) != MAGIC || rd16(arc + 4) != 1) return AXO_E_CORRUPT;
  memset(info, 0, sizeof(*info));
  info->flags = rd16(arc + 6);
  info->block_size = rd32(arc + 8);
  info->min_match = rd16(arc + 12);
  info->depth_cap = rd16(arc + 14);
  info->n_bytes = rd64(arc + 16);
  info->n_blocks = rd64(arc + 24);
  info->xxh3 = rd64(arc + 32);
  info->payload_bytes = rd64(arc + 40);
  info->n_matches = rd64(arc + 48);
  uint32_t B = info->block_size;
  if (B < 4096 || B > 65536 || (B & (B - 1)) || info->min_match < 1 || info->min_match > 255) return AXO_E_CORRUPT;
  if (info->n_blocks != (info->n_bytes + B - 1) / B) return AXO_E_CORRUPT;
  if (info->n_blocks > (len - 64) / 16) return AXO_E_CORRUPT;
  uint64_t need = 64 + 16 * (info->n_blocks + 1) + info->payload_bytes;
  if (info->payload_bytes > len || need > len) return AXO_E_CORRUPT;
  info->archive_bytes = need;
  return AXO_OK;
}

typedef struct {
  uint8_t *lit, *len, *off, *cmd;
  uint32_t n_lit, n_len, n_off, n_cmd, len_cap, off_cap;
} streams_t;

static const uint8_t* block_ptr(const uint8_t* arc, const axo_info* in, uint64_t b, uint64_t* blen) {
  const uint8_t* idx = arc + 64;
  uint64_t o0 = rd64(idx + 8 * b), o1 = rd64(idx + 8 * (b + 1));
  if (o0 > o1 || o1 > in->payload_bytes || (o0 & 15)) return NULL;
  *blen = o1 - o0;
  return arc + 64 + 16 * (in->n_blocks + 1) + o0;
}

static int decode_streams(const uint8_t* arc, const axo_info* in, uint64_t b, streams_t* s) {
  uint64_t blen;
  const uint8_t* bp = block_ptr(arc, in, b, &blen);
  if (!bp || blen < 16) return AXO_E_CORRUPT;
  uint64_t p = 16;
  uint8_t* dst[4] = {s->lit, s->len, s->off, s->cmd};
  uint32_t cap[4] = {in->block_size, s->len_cap, s->off_cap, in->block_size};
  uint32_t* nn[4] = {&s->n_lit, &s->n_len, &s->n_off, &s->n_cmd};
  for (int k = 0; k < 4; k++) {
    uint32_t rl = rd32(bp + 4 * k), used = 0;
    if ((rl & 3) || p + rl > blen) return AXO_E_CORRUPT;
    int rc = axo_stream_decode(bp + p, rl, dst[k], cap[k], nn[k], &used);
    if (rc) return rc;
    if (used != rl) return AXO_E_CORRUPT;
    p += rl;
  }
  if (pad_to(p, 16) != blen) return AXO_E_CORRUPT;
  return AXO_OK;
}

static int streams_alloc(streams_t* s, uint32_t B) {
  memset(s, 0, sizeof(*s));
  s->len_cap = 10 * B;
  s->off_cap = 10 * B;
  s->lit = (uint8_t*)malloc(B);
  s->cmd = (uint8_t*)malloc(B);
  s->len = (uint8_t*)malloc(s->len_cap);
  s->off = (uint8_t*)malloc(s->off_cap);
  return (s->lit && s->cmd && s->len && s->off) ? AXO_OK : AXO_E_NOMEM;
}
static void streams_free(streams_t* s) { free(s->lit); free(s->len); free(s->off); free(s->cmd); }

/* Sequential parse of one block's commands (C2 reading), with every check:
 * a valid block tiles [bs, be) exactly and consumes all four streams. */
static int parse_block(const axo_info* in, uint64_t b, const streams_t* s, axo_cmd* out, uint64_t* n_out,
                       uint64_t* n_matches) {
  uint64_t B = in->block_size, bs = b * B, be = bs + B < in->n_bytes ? bs + B : in->n_bytes;
  uint64_t mm = in->min_match, h[4] = {1, 2, 3, 4}, dst = bs;
  uint32_t lp = 0, ep = 0, op = 0;
  uint64_t nm = 0, nc = 0;
  for (uint32_t i = 0; i < s->n_cmd; i++) {
    uint8_t c = s->cmd[i];
    uint32_t kind = c & 3;
    uint64_t len, src = 0, ext;
    uint32_t used;
    axo_cmd* o = &out[nc];
    memset(o, 0, sizeof(*o));
    if (kind == 3) return AXO_E_CORRUPT;
    uint32_t v = kind == 2 ? (uint32_t)(c >> 4) : (uint32_t)(c >> 2);
    uint32_t esc = kind == 2 ? 15 : 63;
    uint64_t base = kind == 0 ? 1 : mm;
    if (v < esc) len = v + base;
    else {
      if (axo_leb_get(s->len + ep, s->n_len - ep, &ext, &used)) return AXO_E_CORRUPT;
      ep += used;
      if (ext > B) return AXO_E_CORRUPT;
      len = esc + base + ext;
    }
    if (dst + len > be) return AXO_E_CORRUPT;
    o->kind = (uint8_t)kind;
    o->dst = dst;
    o->len = (uint32_t)len;
    o->lit_pos = lp;
    if (kind == 0) {
      if (lp + len > s->n_lit) return AXO_E_CORRUPT;
      lp += (uint32_t)len;
    } else if (kind == 1) {
      if (axo_leb_get(s->off + op, s->n_off - op, &src, &used)) return AXO_E_CORRUPT;
      op += used;
      if (src >= dst) return AXO_E_CORRUPT;
      h[3] = h[2]; h[2] = h[1]; h[1] = h[0]; h[0] = dst - src;
      nm++;
    } else {
      uint32_t r = (c >> 2) & 3;
      uint64_t d = h[r];
      if (d > dst) return AXO_E_CORRUPT;
      src = dst - d;
      for (uint32_t k = r; k > 0; k--) h[k] = h[k - 1];
      h[0] = d;
      o->rep = (uint8_t)r;
      nm++;
    }
    o->src = src;
    dst += len;
    nc++;
  }
  if (dst != be || lp != s->n_lit || ep != s->n_len || op != s->n_off) return AXO_E_CORRUPT;
  *n_out = nc;
  *n_matches = nm;
  return AXO_OK;
}

void axo_copy_serial(uint8_t* buf, uint64_t dst, uint64_t src, uint64_t len) {
  for (uint64_t k = 0; k < len; k++) buf[dst + k] = buf[src + k];
}

void axo_copy_periodic(uint8_t* buf, uint64_t dst, uint64_t src, uint64_t len) {
  uint64_t dist = dst - src;
  for (uint64_t k = 0; k < len; k++) buf[dst + k] = buf[src + k % dist];
}

static int check_index(const uint8_t* arc, const axo_info* in) {
  const uint8_t* mp = arc + 64 + 8 * (in->n_blocks + 1);
  if (rd64(mp) != 0 || rd64(mp + 8 * in->n_blocks) != in->n_matches) return AXO_E_CORRUPT;
  if (rd64(arc + 64) != 0 || rd64(arc + 64 + 8 * in->n_blocks) != in->payload_bytes) return AXO_E_CORRUPT;
  return AXO_OK;
}

static uint64_t block_matches(const uint8_t* arc, const axo_info* in, uint64_t b) {
  const uint8_t* mp = arc + 64 + 8 * (in->n_blocks + 1);
  return rd64(mp + 8 * (b + 1)) - rd64(mp + 8 * b);
}

int axo_decode(const uint8_t* arc, uint64_t len, uint8_t* out, uint64_t cap, int copy_mode, int verify) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if (in.n_bytes > cap) return AXO_E_ARG;
  if ((rc = check_index(arc, &in))) return rc;
  streams_t s;
  axo_cmd* cmds = (axo_cmd*)malloc(sizeof(axo_cmd) * in.block_size);
  if (streams_alloc(&s, in.block_size) || !cmds) { streams_free(&s); free(cmds); return AXO_E_NOMEM; }
  for (uint64_t b = 0; b < in.n_blocks && !rc; b++) {
    uint64_t nc = 0, nm = 0;
    rc = decode_streams(arc, &in, b, &s);
    if (!rc) rc = parse_block(&in, b, &s, cmds, &nc, &nm);
    if (!rc && nm != block_matches(arc, &in, b)) rc = AXO_E_CORRUPT;
    for (uint64_t i = 0; i < nc && !rc; i++) {
      const axo_cmd* c = &cmds[i];
      if (c->kind == 0) memcpy(out + c->dst, s.lit + c->lit_pos, c->len);
      else if (copy_mode == 0) axo_copy_serial(out, c->dst, c->src, c->len);
      else axo_copy_periodic(out, c->dst, c->src, c->len);
    }
  }
  streams_free(&s);
  free(cmds);
  if (!rc && verify && (uint64_t)XXH3_64bits(out, in.n_bytes) != in.xxh3) rc = AXO_E_CHECKSUM;
  return rc;
}

int axo_block_streams(const uint8_t* arc, uint64_t len, uint64_t block, uint8_t* lit, uint32_t* n_lit,
                      uint8_t* lenb, uint32_t* n_len, uint32_t len_cap, uint8_t* off, uint32_t* n_off,
                      uint32_t off_cap, uint8_t* cmd, uint32_t* n_cmd) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if (block >= in.n_blocks) return AXO_E_ARG;
  streams_t s = {lit, lenb, off, cmd, 0, 0, 0, 0, len_cap, off_cap};
  rc = decode_streams(arc, &in, block, &s);
  *n_lit = s.n_lit; *n_len = s.n_len; *n_off = s.n_off; *n_cmd = s.n_cmd;
  return rc;
}

int axo_block_parse(const uint8_t* arc, uint64_t len, uint64_t block, axo_cmd* cmds, uint64_t cap,
                    uint64_t* n_cmds) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if (block >= in.n_blocks || cap < in.block_size) return AXO_E_ARG;
  streams_t s;
  if (streams_alloc(&s, in.block_size)) { streams_free(&s); return AXO_E_NOMEM; }
  uint64_t nm;
  rc = decode_streams(arc, &in, block, &s);
  if (!rc) rc = parse_block(&in, block, &s, cmds, n_cmds, &nm);
  streams_free(&s);
  return rc;
}

/* All commands of the archive, in output order. */
int axo_parse_all(const uint8_t* arc, uint64_t len, axo_cmd** cmds, uint64_t* n_cmds) {
  return walk_all(arc, len, cmds, n_cmds);
}

static int walk_all(const uint8_t* arc, uint64_t len, axo_cmd** cmds_out, uint64_t* n_out) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if ((rc = check_index(arc, &in))) return rc;
  streams_t s;
  uint64_t cap = 1024, nc = 0;
  axo_cmd* all = (axo_cmd*)malloc(sizeof(axo_cmd) * cap);
  axo_cmd* tmp = (axo_cmd*)malloc(sizeof(axo_cmd) * in.block_size);
  if (streams_alloc(&s, in.block_size) || !all || !tmp) { streams_free(&s); free(all); free(tmp); return AXO_E_NOMEM; }
  for (uint64_t b = 0; b < in.n_blocks && !rc; b++) {
    uint64_t k = 0, nm = 0;
    rc = decode_streams(arc, &in, b, &s);
    if (!rc) rc = parse_block(&in, b, &s, tmp, &k, &nm);
    if (!rc && nm != block_matches(arc, &in, b)) rc = AXO_E_CORRUPT;
    if (rc) break;
    if (nc + k > cap) {
      while (nc + k > cap) cap *= 2;
      axo_cmd* q = (axo_cmd*)realloc(all, sizeof(axo_cmd) * cap);
      if (!q) { rc = AXO_E_NOMEM; break; }
      all = q;
    }
    memcpy(all + nc, tmp, sizeof(axo_cmd) * k);
    nc += k;
  }
  streams_free(&s);
  free(tmp);
  if (rc) { free(all); return rc; }
  *cmds_out = all;
  *n_out = nc;
  return AXO_OK;
}

/* ---------------------------------------------------------- statistics --- */

/* depth_per_cmd[i] for every command (0 for LIT). Writer depth per output
 * byte: -1 for literal bytes, else the depth of the match that wrote it. */
static int depths_of(const uint8_t* arc, uint64_t len, const axo_cmd* cmds, uint64_t nc, uint64_t n,
                     uint32_t* dep, uint32_t* maxd) {
  (void)arc; (void)len;
  int32_t* wd = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));
  if (!wd) return AXO_E_NOMEM;
  uint32_t mx = 0;
  for (uint64_t i = 0; i < nc; i++) {
    const axo_cmd* c = &cmds[i];
    int32_t d = -1;
    if (c->kind == 0) {
      for (uint64_t k = 0; k < c->len; k++) wd[c->dst + k] = -1;
      dep[i] = 0;
      continue;
    }
    uint64_t dist = c->dst - c->src, sl = c->len < dist ? c->len : dist;
    for (uint64_t k = 0; k < sl; k++) if (wd[c->src + k] > d) d = wd[c->src + k];
    dep[i] = (uint32_t)(d + 1);
    if (dep[i] > mx) mx = dep[i];
    for (uint64_t k = 0; k < c->len; k++) wd[c->dst + k] = d + 1;
  }
  free(wd);
  *maxd = mx;
  return AXO_OK;
}

int axo_depths(const uint8_t* arc, uint64_t len, uint32_t* depth, uint64_t cap, uint32_t* max_depth) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if (cap < in.n_matches) return AXO_E_ARG;
  axo_cmd* cmds = NULL;
  uint64_t nc = 0;
  if ((rc = walk_all(arc, len, &cmds, &nc))) return rc;
  uint32_t* dep = (uint32_t*)malloc(sizeof(uint32_t) * (nc ? nc : 1));
  if (!dep) { free(cmds); return AXO_E_NOMEM; }
  rc = depths_of(arc, len, cmds, nc, in.n_bytes, dep, max_depth);
  uint64_t m = 0;
  for (uint64_t i = 0; i < nc && !rc; i++) if (cmds[i].kind != 0) depth[m++] = dep[i];
  free(cmds); free(dep);
  return rc;
}

int axo_block_levels(const uint8_t* arc, uint64_t len, uint32_t* raw_max, uint32_t* msrc_max, uint32_t* raw_lvl,
                     uint32_t* msrc_lvl) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  axo_cmd* cmds = NULL;
  uint64_t nc = 0;
  if ((rc = walk_all(arc, len, &cmds, &nc))) return rc;
  uint64_t n = in.n_bytes, B = in.block_size;
  uint8_t* bym = (uint8_t*)calloc(n ? n : 1, 1); /* 1: byte written by a match */
  uint32_t* lr = (uint32_t*)calloc(in.n_blocks ? in.n_blocks : 1, sizeof(uint32_t));
  uint32_t* lm = (uint32_t*)calloc(in.n_blocks ? in.n_blocks : 1, sizeof(uint32_t));
  if (!bym || !lr || !lm) { free(cmds); free(bym); free(lr); free(lm); return AXO_E_NOMEM; }
  uint32_t mr = 0, mmx = 0;
  for (uint64_t i = 0; i < nc; i++) {
    const axo_cmd* c = &cmds[i];
    uint64_t b = c->dst / B;
    if (c->kind != 0) {
      uint64_t dist = c->dst - c->src, sl = c->len < dist ? c->len : dist;
      for (uint64_t k = 0; k < sl; k++) {
        uint64_t q = c->src + k, qb = q / B;
        if (qb == b) continue;
        if (lr[qb] + 1 > lr[b]) lr[b] = lr[qb] + 1;
        if (bym[q] && lm[qb] + 1 > lm[b]) lm[b] = lm[qb] + 1;
      }
      for (uint64_t k = 0; k < c->len; k++) bym[c->dst + k] = 1;
    }
    if (lr[b] > mr) mr = lr[b];
    if (lm[b] > mmx) mmx = lm[b];
  }
  *raw_max = mr;
  *msrc_max = mmx;
  for (uint64_t b = 0; b < in.n_blocks; b++) {
    if (raw_lvl) raw_lvl[b] = lr[b];
    if (msrc_lvl) msrc_lvl[b] = lm[b];
  }
  free(cmds); free(bym); free(lr); free(lm);
  return AXO_OK;
}

int axo_closure(const uint8_t* arc, uint64_t len, uint64_t off, uint64_t n, uint8_t* block_mask,
                uint64_t* n_marked) {
  axo_info in;
  int rc = axo_read_info(arc, len, &in);
  if (rc) return rc;
  if (off > in.n_bytes || n > in.n_bytes - off) return AXO_E_ARG;
  axo_cmd* cmds = NULL;
  uint64_t nc = 0;
  if ((rc = walk_all(arc, len, &cmds, &nc))) return rc;
  uint8_t* need = (uint8_t*)calloc(in.n_bytes ? in.n_bytes : 1, 1);
  if (!need) { free(cmds); return AXO_E_NOMEM; }
  for (uint64_t q = off; q < off + n; q++) need[q] = 1;
  /* Sources always lie below their destination, so one backward sweep over
   * the commands propagates every needed byte to the bytes it is copied from. */
  for (uint64_t i = nc; i-- > 0;) {
    const axo_cmd* c = &cmds[i];
    if (c->kind == 0) continue;
    uint64_t dist = c->dst - c->src;
    for (uint64_t k = c->len; k-- > 0;)
      if (need[c->dst + k]) need[c->src + k % dist] = 1;
  }
  uint64_t B = in.block_size, marked = 0;
  for (uint64_t b = 0; b < in.n_blocks; b++) {
    uint64_t bs = b * B, be = bs + B < in.n_bytes ? bs + B : in.n_bytes;
    block_mask[b] = 0;
    for (uint64_t q = bs; q < be; q++) if (need[q]) { block_mask[b] = 1; break; }
    marked += block_mask[b];
  }
  *n_marked = marked;
  free(cmds); free(need);
  return AXO_OK;
}
