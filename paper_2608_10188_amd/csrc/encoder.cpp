// Host encoder of the AXP1 block format (aceapex_encode).
//
// Global greedy match search with absolute offsets over fixed-size blocks,
// four streams per block (Setup), optional history-free encoding and the
// iterated forced-literal depth cap (depth section).  The bytes are a pure
// function of (input, parameters): threads only split independent blocks.
//
// Structure: the hash chains of a segment are built first, independent of the
// parse (every position enters its chain whatever the parse does), after which
// every block of the segment can be encoded on any thread, because a block's
// decisions depend only on the chains, the input and its own history.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "aceapex.h"
#include "ax_common.h"

extern "C" unsigned long long XXH3_64bits(const void* data, size_t len);

namespace {

using ax::BlockStreams;

constexpr uint32_t kNil = 0xFFFFFFFFu;

inline uint32_t hash_at(const uint8_t* p, uint32_t bits) {
  uint32_t v;
  std::memcpy(&v, p, 4);  // little-endian host
  return (v * 2654435761u) >> (32 - bits);
}

inline uint64_t common_prefix(const uint8_t* a, const uint8_t* b, uint64_t limit) {
  uint64_t k = 0;
  while (k + 8 <= limit) {
    uint64_t x, y;
    std::memcpy(&x, a + k, 8);
    std::memcpy(&y, b + k, 8);
    if (x != y) return k + (uint64_t)(__builtin_ctzll(x ^ y) >> 3);
    k += 8;
  }
  while (k < limit && a[k] == b[k]) k++;
  return k;
}

struct Cmd {  // one emitted command, kept for the depth computation
  uint64_t dst, src;
  uint32_t len;
  uint8_t kind;
};

struct Params {
  aceapex_encode_params p;
  uint64_t window;  // 0 = unlimited
};

// Chains for positions [r0, r1): link[q - r0] = previous position with the
// same hash (relative to r0), or kNil.  Built in parallel: each part of the
// range chains its own positions and records, per hash, its first and last
// position; a second pass over disjoint hash ranges links every part's first
// occurrence to the last occurrence in the parts before it.  The links equal
// those of one sequential pass.
struct Chains {
  uint64_t r0 = 0;
  std::vector<uint32_t> link;
  void build(const uint8_t* in, uint64_t n, uint64_t a, uint64_t b, uint32_t bits, unsigned threads) {
    r0 = a;
    link.assign(b - a, kNil);
    const uint64_t end = std::min<uint64_t>(b, n >= 4 ? n - 3 : 0);  // positions with 4 bytes left
    if (end <= a) return;
    const size_t H = size_t(1) << bits;
    const uint64_t span = end - a;
    const unsigned P = unsigned(std::max<uint64_t>(1, std::min<uint64_t>(threads, span >> 22)));
    std::vector<std::vector<uint32_t>> first(P), last(P);
    auto chain_part = [&](unsigned p) {
      const uint64_t lo = a + span * p / P, hi = a + span * (p + 1) / P;
      last[p].assign(H, kNil);
      if (p) first[p].assign(H, kNil);
      uint32_t* L = last[p].data();
      uint32_t* F = p ? first[p].data() : nullptr;
      for (uint64_t q = lo; q < hi; ++q) {
        const uint32_t h = hash_at(in + q, bits), r = uint32_t(q - a);
        link[r] = L[h];
        if (F && L[h] == kNil) F[h] = r;
        L[h] = r;
      }
    };
    auto stitch = [&](unsigned t) {
      const size_t h0 = H * t / P, h1 = H * (t + 1) / P;
      for (size_t h = h0; h < h1; ++h) {
        uint32_t g = last[0][h];
        for (unsigned p = 1; p < P; ++p) {
          if (first[p][h] != kNil) link[first[p][h]] = g;
          if (last[p][h] != kNil) g = last[p][h];
        }
      }
    };
    if (P == 1) {
      chain_part(0);
      return;
    }
    std::vector<std::thread> pool;
    for (unsigned p = 1; p < P; ++p) pool.emplace_back(chain_part, p);
    chain_part(0);
    for (auto& th : pool) th.join();
    pool.clear();
    for (unsigned t = 1; t < P; ++t) pool.emplace_back(stitch, t);
    stitch(0);
    for (auto& th : pool) th.join();
  }
};

// Encode block b into streams; forced (nullable) marks positions that must
// stay literal.  cmds (nullable) receives the commands.
void encode_block(const uint8_t* in, uint64_t n, const Params& P, const Chains& ch, const uint8_t* forced,
                  uint64_t b, BlockStreams& bs, std::vector<Cmd>* cmds, uint64_t* n_rep, uint64_t* n_mbytes,
                  uint64_t* n_srcbytes) {
  const auto& p = P.p;
  const uint64_t B = p.block_size, mm = p.min_match;
  const uint64_t start = b * B, end = std::min(start + B, n);
  uint64_t hist[4] = {1, 2, 3, 4};
  uint64_t pos = start, run = start, next_forced = start;
  bs.clear();
  auto flush_literals = [&](uint64_t upto) {
    if (upto > run) {
      bs.add_literal(in + run, upto - run);
      if (cmds) cmds->push_back({run, 0, uint32_t(upto - run), 0});
    }
  };
  while (pos < end) {
    uint64_t room = end - pos;
    if (forced) {
      if (next_forced < pos) next_forced = pos;
      while (next_forced < end && !forced[next_forced]) ++next_forced;
      room = std::min(room, next_forced - pos);
    }
    uint64_t best_rep = 0, best_abs = 0, abs_src = 0;
    unsigned rep_idx = 0;
    if (!p.no_rep && room) {
      for (unsigned r = 0; r < 4; ++r) {
        if (hist[r] > pos) continue;
        uint64_t l = common_prefix(in + pos - hist[r], in + pos, room);
        if (l > best_rep) best_rep = l, rep_idx = r;
      }
    }
    if (room && pos + 4 <= n) {
      uint32_t c = ch.link[pos - ch.r0];
      for (uint32_t step = 0; step < p.chain_depth && c != kNil; ++step) {
        uint64_t cand = ch.r0 + c;
        if (P.window && cand + P.window < pos) break;
        uint64_t l = common_prefix(in + cand, in + pos, room);
        if (l > best_abs) best_abs = l, abs_src = cand;
        if (l == room) break;
        c = ch.link[cand - ch.r0];
      }
    }
    const uint64_t abs_need = mm + (uint64_t(p.off_cost_q) * ax::leb_size(abs_src) + 3) / 4;
    if (best_rep >= mm && best_rep >= best_abs) {
      flush_literals(pos);
      bs.add_rep(rep_idx, best_rep, mm);
      uint64_t d = hist[rep_idx];
      for (unsigned k = rep_idx; k > 0; --k) hist[k] = hist[k - 1];
      hist[0] = d;
      if (cmds) cmds->push_back({pos, pos - d, uint32_t(best_rep), 2});
      ++*n_rep;
      *n_mbytes += best_rep;
      *n_srcbytes += std::min<uint64_t>(best_rep, d);
      pos += best_rep;
      run = pos;
    } else if (best_abs >= abs_need) {
      flush_literals(pos);
      bs.add_match(abs_src, best_abs, mm);
      hist[3] = hist[2], hist[2] = hist[1], hist[1] = hist[0], hist[0] = pos - abs_src;
      if (cmds) cmds->push_back({pos, abs_src, uint32_t(best_abs), 1});
      *n_mbytes += best_abs;
      *n_srcbytes += std::min<uint64_t>(best_abs, pos - abs_src);
      pos += best_abs;
      run = pos;
    } else {
      ++pos;
    }
  }
  flush_literals(end);
}

struct Encoded {
  std::vector<std::vector<uint8_t>> block_bytes;  // serialised block payloads
  std::vector<uint64_t> block_matches;
  std::vector<std::vector<Cmd>> block_cmds;       // only with a depth cap
  uint64_t n_commands = 0, n_rep = 0, n_mbytes = 0, n_lit = 0, n_src = 0, n_off = 0, n_len = 0;
};

unsigned thread_count(const aceapex_encode_params& p) {
  unsigned t = p.threads ? p.threads : std::thread::hardware_concurrency();
  return std::max(1u, std::min(t, 256u));
}

int encode_pass(const uint8_t* in, uint64_t n, const Params& P, const uint8_t* forced, bool keep_cmds,
                Encoded& E) {
  const auto& p = P.p;
  const uint64_t B = p.block_size, nb = (n + B - 1) / B;
  E.block_bytes.assign(nb, {});
  E.block_matches.assign(nb, 0);
  E.block_cmds.assign(keep_cmds ? nb : 0, {});
  const unsigned T = thread_count(p);
  // Segments bound the chain memory; without a window one segment spans all.
  uint64_t seg = n ? n : 1;
  if (P.window) seg = std::max<uint64_t>(uint64_t(1) << 30, B);
  if (!P.window && n >= kNil) return AX_E_UNSUPPORTED;  // 32-bit chain links need a window
  seg = (seg + B - 1) / B * B;
  std::atomic<uint64_t> tot_cmds{0}, tot_rep{0}, tot_mb{0}, tot_lit{0}, tot_src{0}, tot_off{0}, tot_len{0};
  std::atomic<int> err{0};
  Chains ch;
  for (uint64_t s0 = 0; s0 < n; s0 += seg) {
    uint64_t s1 = std::min(n, s0 + seg);
    uint64_t r0 = (P.window && s0 > P.window) ? s0 - P.window : 0;
    if (s1 - r0 >= kNil) return AX_E_UNSUPPORTED;
    ch.build(in, n, r0, s1, p.hash_bits, T);
    const uint64_t b0 = s0 / B, b1 = (s1 + B - 1) / B;
    std::atomic<uint64_t> next{b0};
    auto worker = [&]() {
      BlockStreams bs;
      uint64_t cmds = 0, reps = 0, mb = 0, lit = 0, srcb = 0, offb = 0, lenb = 0;
      std::vector<uint8_t> rec;
      for (;;) {
        uint64_t b = next.fetch_add(1);
        if (b >= b1) break;
        encode_block(in, n, P, ch, forced, b, bs, keep_cmds ? &E.block_cmds[b] : nullptr, &reps, &mb, &srcb);
        cmds += bs.cmd.size();
        lit += bs.lit.size();
        offb += bs.off.size();
        lenb += bs.len.size();
        E.block_matches[b] = bs.n_matches;
        if (!ax::serialize_block(bs, p.rans_min_syms_per_lane, E.block_bytes[b])) err = AX_E_NOMEM;
      }
      tot_cmds += cmds, tot_rep += reps, tot_mb += mb, tot_lit += lit;
      tot_src += srcb, tot_off += offb, tot_len += lenb;
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < T; ++t) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    if (err) return err;
    if (p.progress) p.progress(p.progress_user, s1, n);
  }
  E.n_commands = tot_cmds, E.n_rep = tot_rep, E.n_mbytes = tot_mb, E.n_lit = tot_lit;
  E.n_src = tot_src, E.n_off = tot_off, E.n_len = tot_len;
  return AX_OK;
}

// Chain depth of every match: 0 when all source bytes are literal bytes,
// else one more than the deepest match that wrote a source byte.
uint32_t match_depths(const Encoded& E, uint64_t n, std::vector<std::vector<uint32_t>>& depth) {
  std::vector<int32_t> wdepth(n, -1);
  uint32_t deepest = 0;
  depth.assign(E.block_cmds.size(), {});
  for (size_t b = 0; b < E.block_cmds.size(); ++b) {
    for (const Cmd& c : E.block_cmds[b]) {
      if (c.kind == 0) {
        std::fill(wdepth.begin() + c.dst, wdepth.begin() + c.dst + c.len, -1);
        depth[b].push_back(0);
        continue;
      }
      uint64_t dist = c.dst - c.src, span = std::min<uint64_t>(c.len, dist);
      int32_t d = -1;
      for (uint64_t k = 0; k < span; ++k) d = std::max(d, wdepth[c.src + k]);
      int32_t mine = d + 1;
      std::fill(wdepth.begin() + c.dst, wdepth.begin() + c.dst + c.len, mine);
      depth[b].push_back(uint32_t(mine));
      deepest = std::max(deepest, uint32_t(mine));
    }
  }
  return deepest;
}

}  // namespace

extern "C" {

void aceapex_encode_params_default(aceapex_encode_params* p) {
  if (!p) return;
  p->block_size = 16384;
  p->min_match = 4;
  p->no_rep = 0;
  p->depth_cap = 0;
  p->hash_bits = 22;
  p->chain_depth = 32;
  p->rans_min_syms_per_lane = 32;
  p->off_cost_q = 6;
  p->window_log = 0;
  p->threads = 0;
  p->progress = nullptr;
  p->progress_user = nullptr;
}

static int check_params(const aceapex_encode_params* p) {
  if (!p) return ax::fail(AX_E_ARG, "null parameters");
  if (p->block_size < 4096 || p->block_size > 65536 || (p->block_size & (p->block_size - 1)))
    return ax::fail(AX_E_ARG, "block_size must be a power of two in [4096, 65536]");
  if (p->min_match < 1 || p->min_match > 255) return ax::fail(AX_E_ARG, "min_match must be in [1, 255]");
  if (p->hash_bits < 10 || p->hash_bits > 26) return ax::fail(AX_E_ARG, "hash_bits must be in [10, 26]");
  if (p->window_log > 40) return ax::fail(AX_E_ARG, "window_log must be <= 40");
  if (p->off_cost_q > 4096) return ax::fail(AX_E_ARG, "off_cost_q must be <= 4096");
  return AX_OK;
}

int aceapex_encode_bound(uint64_t n, const aceapex_encode_params* p, uint64_t* bound) {
  int rc = check_params(p);
  if (rc) return rc;
  if (!bound) return ax::fail(AX_E_ARG, "null bound");
  const uint64_t B = p->block_size, nb = (n + B - 1) / B;
  // per block: 16 B sizes + 4 records of at most 8 + n_sym + 3 bytes (RAW),
  // LIT <= B, CMD <= B, LEN <= 3 bytes per 64-byte command, OFF <= 10 bytes
  // per match of at least min_match bytes; + 15 bytes of padding
  const uint64_t per_block = 16 + 4 * 11 + 2 * B + 3 * (B / 64 + 1) + 10 * (B / p->min_match + 1) + 15;
  *bound = 64 + 16 * (nb + 1) + nb * per_block;
  return AX_OK;
}

int aceapex_encode(const uint8_t* src, uint64_t n, const aceapex_encode_params* pp, uint8_t* dst,
                   uint64_t cap, uint64_t* dst_len, aceapex_encode_stats* stats) {
  int rc = check_params(pp);
  if (rc) return rc;
  if ((!src && n) || !dst || !dst_len) return ax::fail(AX_E_ARG, "null buffer");
  try {
    Params P{*pp, pp->window_log ? (uint64_t(1) << pp->window_log) : 0};
    const uint64_t B = pp->block_size, nb = (n + B - 1) / B;
    Encoded E;
    std::vector<uint8_t> forced;
    uint32_t passes = 0, deepest = 0;
    for (;;) {
      rc = encode_pass(src, n, P, forced.empty() ? nullptr : forced.data(), pp->depth_cap != 0, E);
      if (rc) return ax::fail(rc, "encode pass failed");
      ++passes;
      if (!pp->depth_cap) break;
      std::vector<std::vector<uint32_t>> depth;
      deepest = match_depths(E, n, depth);
      if (deepest <= pp->depth_cap) break;
      if (forced.empty()) forced.assign(n, 0);
      for (uint64_t b = 0; b < nb; ++b)
        for (size_t i = 0; i < E.block_cmds[b].size(); ++i) {
          const Cmd& c = E.block_cmds[b][i];
          if (c.kind != 0 && depth[b][i] > pp->depth_cap) std::memset(forced.data() + c.dst, 1, c.len);
        }
    }
    // container: header, index, payload
    uint64_t payload = 0;
    for (auto& v : E.block_bytes) payload += v.size();
    const uint64_t total = 64 + 16 * (nb + 1) + payload;
    if (total > cap) return ax::fail(AX_E_CAPACITY, "destination too small");
    uint64_t n_matches = 0;
    for (auto m : E.block_matches) n_matches += m;
    uint8_t* h = dst;
    ax::put32(h + 0, ax::kMagic);
    ax::put16(h + 4, 1);
    ax::put16(h + 6, uint16_t((pp->no_rep ? 1 : 0) | (pp->depth_cap ? 2 : 0)));
    ax::put32(h + 8, uint32_t(B));
    ax::put16(h + 12, uint16_t(pp->min_match));
    ax::put16(h + 14, uint16_t(pp->depth_cap));
    ax::put64(h + 16, n);
    ax::put64(h + 24, nb);
    ax::put64(h + 32, (uint64_t)XXH3_64bits(src, n));
    ax::put64(h + 40, payload);
    ax::put64(h + 48, n_matches);
    ax::put64(h + 56, 0);
    uint8_t* off_idx = h + 64;
    uint8_t* cnt_idx = off_idx + 8 * (nb + 1);
    uint8_t* body = cnt_idx + 8 * (nb + 1);
    uint64_t at = 0, mcount = 0;
    for (uint64_t b = 0; b < nb; ++b) {
      ax::put64(off_idx + 8 * b, at);
      ax::put64(cnt_idx + 8 * b, mcount);
      std::memcpy(body + at, E.block_bytes[b].data(), E.block_bytes[b].size());
      at += E.block_bytes[b].size();
      mcount += E.block_matches[b];
    }
    ax::put64(off_idx + 8 * nb, at);
    ax::put64(cnt_idx + 8 * nb, mcount);
    *dst_len = total;
    if (stats) {
      stats->n_bytes = n;
      stats->n_blocks = nb;
      stats->comp_bytes = total;
      stats->n_commands = E.n_commands;
      stats->n_matches = n_matches;
      stats->n_rep = E.n_rep;
      stats->n_match_bytes = E.n_mbytes;
      stats->n_lit_bytes = E.n_lit;
      stats->n_src_bytes = E.n_src;
      stats->n_off_bytes = E.n_off;
      stats->n_len_bytes = E.n_len;
      stats->max_depth = deepest;
      stats->passes = passes;
    }
    return AX_OK;
  } catch (const std::bad_alloc&) {
    return ax::fail(AX_E_NOMEM, "host allocation failed");
  }
}

}  // extern "C"
