// Host-side stream serialisation: order-0 rANS with 12-bit frequencies,
// 32-bit states and 16-bit renormalisation (Duda, "Asymmetric numeral
// systems", arXiv:1311.2540), K interleaved lanes (Giesen, "Interleaved
// entropy coders", arXiv:1402.3392), plus the raw and constant modes.
#include <algorithm>
#include <array>
#include <string>

#include "aceapex.h"
#include "ax_common.h"

namespace ax {

namespace {

thread_local std::string g_detail;

void pad(std::vector<uint8_t>& v, size_t a) {
  while (v.size() % a) v.push_back(0);
}

// Frequencies summing to 4096 with every present symbol >= 1. Integer
// scaling first; a shortfall goes to the most frequent symbol (smallest
// byte on ties); an excess is taken back one unit at a time walking the
// symbols in descending frequency order (smallest byte first on ties),
// never below 1.
void scale_counts(const std::array<uint64_t, 256>& cnt, uint64_t n, std::array<uint32_t, 256>& f) {
  uint64_t total = 0;
  int top = -1;
  for (int s = 0; s < 256; ++s) {
    f[s] = 0;
    if (!cnt[s]) continue;
    f[s] = uint32_t(std::max<uint64_t>(1, cnt[s] * kProbScale / n));
    total += f[s];
    if (top < 0 || cnt[s] > cnt[top]) top = s;
  }
  if (total < kProbScale) {
    f[top] += uint32_t(kProbScale - total);
  } else if (total > kProbScale) {
    std::vector<int> order;
    for (int s = 0; s < 256; ++s)
      if (cnt[s]) order.push_back(s);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return f[a] > f[b]; });
    for (size_t k = 0; total > kProbScale; k = (k + 1) % order.size())
      if (f[order[k]] > 1) --f[order[k]], --total;
  }
}

uint32_t lanes_log2(uint32_t n, uint32_t per_lane) {
  const uint64_t lim = std::max(n, per_lane);
  uint32_t lg = 0;
  while (lg < kMaxLanesLog2 && (uint64_t(2) << lg) * per_lane <= lim) ++lg;
  return lg;
}

}  // namespace

bool append_stream_record(const uint8_t* sym, uint32_t n, uint32_t per_lane, std::vector<uint8_t>& out) {
  std::array<uint64_t, 256> cnt{};
  for (uint32_t i = 0; i < n; ++i) ++cnt[sym[i]];
  uint32_t present = 0;
  for (auto c : cnt) present += c != 0;
  const size_t base = out.size();
  uint8_t hdr[8];
  put32(hdr, n);
  if (n >= 1 && present == 1) {  // constant
    hdr[4] = 1, hdr[5] = sym[0], hdr[6] = 0, hdr[7] = 0;
    out.insert(out.end(), hdr, hdr + 8);
    return true;
  }
  const uint64_t raw_size = (8 + uint64_t(n) + 3) / 4 * 4;
  if (present >= 2) {
    const uint32_t lg = lanes_log2(n, std::max<uint32_t>(1, per_lane)), K = 1u << lg;
    std::array<uint32_t, 256> f, cum;
    scale_counts(cnt, n, f);
    uint32_t acc = 0;
    for (int s = 0; s < 256; ++s) cum[s] = acc, acc += f[s];
    std::vector<uint32_t> x(K, kRansLow);
    std::vector<uint16_t> pushed;
    pushed.reserve(n / 2 + 16);
    for (uint64_t i = n; i-- > 0;) {
      uint32_t& st = x[i & (K - 1)];
      const uint32_t fs = f[sym[i]];
      if (uint64_t(st) >= (uint64_t(kRansLow >> kProbBits) << 16) * fs) {
        pushed.push_back(uint16_t(st));
        st >>= 16;
      }
      st = ((st / fs) << kProbBits) + (st % fs) + cum[sym[i]];
    }
    const uint64_t nw = pushed.size();
    const uint64_t set_bytes = present <= 32 ? present : 32;
    uint64_t sz = (12 + 4ull * K + 2 * nw + 3) / 4 * 4;
    sz = (sz + set_bytes + 1) / 2 * 2;
    sz = (sz + 2ull * present + 3) / 4 * 4;
    if (sz < raw_size) {
      hdr[4] = 2, hdr[5] = uint8_t(lg), hdr[6] = uint8_t(present - 1), hdr[7] = 0;
      out.insert(out.end(), hdr, hdr + 8);
      uint8_t w4[4];
      put32(w4, uint32_t(nw));
      out.insert(out.end(), w4, w4 + 4);
      for (uint32_t j = 0; j < K; ++j) put32(w4, x[j]), out.insert(out.end(), w4, w4 + 4);
      for (uint64_t k = nw; k-- > 0;) out.push_back(uint8_t(pushed[k])), out.push_back(uint8_t(pushed[k] >> 8));
      pad(out, 4);
      if (present <= 32) {
        for (int s = 0; s < 256; ++s)
          if (cnt[s]) out.push_back(uint8_t(s));
      } else {
        uint8_t bm[32] = {};
        for (int s = 0; s < 256; ++s)
          if (cnt[s]) bm[s >> 3] |= uint8_t(1u << (s & 7));
        out.insert(out.end(), bm, bm + 32);
      }
      pad(out, 2);
      for (int s = 0; s < 256; ++s)
        if (cnt[s]) out.push_back(uint8_t(f[s])), out.push_back(uint8_t(f[s] >> 8));
      pad(out, 4);
      return out.size() - base == sz;
    }
  }
  hdr[4] = 0, hdr[5] = 0, hdr[6] = 0, hdr[7] = 0;  // raw
  out.insert(out.end(), hdr, hdr + 8);
  out.insert(out.end(), sym, sym + n);
  pad(out, 4);
  return true;
}

bool serialize_block(const BlockStreams& s, uint32_t per_lane, std::vector<uint8_t>& out) {
  out.clear();
  out.resize(16);
  const std::vector<uint8_t>* st[4] = {&s.lit, &s.len, &s.off, &s.cmd};
  for (int k = 0; k < 4; ++k) {
    const size_t at = out.size();
    if (!append_stream_record(st[k]->data(), uint32_t(st[k]->size()), per_lane, out)) return false;
    put32(out.data() + 4 * k, uint32_t(out.size() - at));
  }
  pad(out, 16);
  return true;
}

int fail(int code, const char* detail) {
  g_detail = detail ? detail : "";
  return code;
}

}  // namespace ax

extern "C" {

const char* aceapex_strerror(int code) {
  switch (code) {
    case AX_OK: return "ok";
    case AX_E_ARG: return "invalid argument";
    case AX_E_CORRUPT: return "corrupt archive";
    case AX_E_UNSUPPORTED: return "unsupported archive";
    case AX_E_CAPACITY: return "buffer or workspace too small";
    case AX_E_HIP: return "HIP runtime error";
    case AX_E_RANGE: return "range outside the archive";
    case AX_E_DEVICE: return "device-side failure";
    case AX_E_NOMEM: return "out of host memory";
    default: return "unknown error";
  }
}

const char* aceapex_last_error(void) { return ax::g_detail.c_str(); }

}  // extern "C"
