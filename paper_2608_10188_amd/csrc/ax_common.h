// Shared host-side pieces of the library: container constants, little-endian
// helpers, per-block stream building and serialisation (rANS encoder), and
// the thread-local error detail behind aceapex_last_error().
//
// Container "AXP1" (little-endian):
//   header 64 B: magic, version, flags (1 NO_REP, 2 DEPTH_CAPPED), block size,
//     min_match, depth cap, decoded size, block count, XXH3-64 of the decoded
//     bytes, payload size, match count;
//   index: (blocks+1) u64 payload offsets, then (blocks+1) u64 cumulative
//     match counts;
//   payload: per block u32 record sizes [4], then the records of the four
//     streams in the paper's order (literals, lengths, offsets, commands),
//     padded to 16 bytes.
// Stream record: u32 n_sym, u8 mode (0 raw, 1 constant, 2 rANS), u8 a, u8 b,
//   u8 0; rANS: a = log2 lanes (<= 6), b = present symbols - 1, u32 word
//   count, lane states (u32), 16-bit words in read order, symbol set (list of
//   <= 32 bytes or a 32-byte bitmap), u16 frequencies (sum 4096).
// Command byte: kind = c & 3 — 0 literal run, 1 match with an absolute
//   offset, 2 repeat match using distance-history slot (c >> 2) & 3, 3 invalid.
#pragma once
#include <cstdint>
#include <cstring>
#include <vector>

namespace ax {

constexpr uint32_t kMagic = 0x31505841u;  // "AXP1"
constexpr uint32_t kProbBits = 12;
constexpr uint32_t kProbScale = 1u << kProbBits;
constexpr uint32_t kRansLow = 1u << 16;
constexpr uint32_t kMaxLanesLog2 = 6;

inline void put16(uint8_t* p, uint16_t v) { std::memcpy(p, &v, 2); }
inline void put32(uint8_t* p, uint32_t v) { std::memcpy(p, &v, 4); }
inline void put64(uint8_t* p, uint64_t v) { std::memcpy(p, &v, 8); }
inline uint16_t get16(const uint8_t* p) { uint16_t v; std::memcpy(&v, p, 2); return v; }
inline uint32_t get32(const uint8_t* p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
inline uint64_t get64(const uint8_t* p) { uint64_t v; std::memcpy(&v, p, 8); return v; }

inline unsigned leb_size(uint64_t v) {
  unsigned n = 1;
  while (v >= 0x80) v >>= 7, ++n;
  return n;
}
inline void leb_append(std::vector<uint8_t>& out, uint64_t v) {
  while (v >= 0x80) { out.push_back(uint8_t(v | 0x80)); v >>= 7; }
  out.push_back(uint8_t(v));
}

// The four streams of one block, filled in command order.
struct BlockStreams {
  std::vector<uint8_t> lit, len, off, cmd;
  uint64_t n_matches = 0;
  void clear() { lit.clear(), len.clear(), off.clear(), cmd.clear(), n_matches = 0; }
  void add_literal(const uint8_t* bytes, uint64_t n) {
    lit.insert(lit.end(), bytes, bytes + n);
    if (n <= 63) cmd.push_back(uint8_t((n - 1) << 2));
    else { cmd.push_back(uint8_t(63 << 2)); leb_append(len, n - 64); }
  }
  void add_match(uint64_t src, uint64_t n, uint64_t mm) {
    if (n - mm < 63) cmd.push_back(uint8_t(1 | ((n - mm) << 2)));
    else { cmd.push_back(uint8_t(1 | (63 << 2))); leb_append(len, n - mm - 63); }
    leb_append(off, src);
    ++n_matches;
  }
  void add_rep(unsigned slot, uint64_t n, uint64_t mm) {
    if (n - mm < 15) cmd.push_back(uint8_t(2 | (slot << 2) | ((n - mm) << 4)));
    else { cmd.push_back(uint8_t(2 | (slot << 2) | (15 << 4))); leb_append(len, n - mm - 15); }
    ++n_matches;
  }
};

// Append one stream record (mode chosen by size) to out.
bool append_stream_record(const uint8_t* sym, uint32_t n, uint32_t min_syms_per_lane, std::vector<uint8_t>& out);

// Serialise a block: u32 record sizes, four records, pad to 16.
bool serialize_block(const BlockStreams& s, uint32_t min_syms_per_lane, std::vector<uint8_t>& out);

// Thread-local error detail; returns code for convenience.
int fail(int code, const char* detail);

}  // namespace ax
