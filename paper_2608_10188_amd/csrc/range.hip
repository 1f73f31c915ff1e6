// Random access: byte-precise source closure of a range and its decode.
//
// A range [off, off+len) needs its own bytes, and for every match that
// writes one of them the source bytes that match copies (periodic form:
// byte k of a match comes from src + k mod dist), transitively.  Because
// offsets are absolute and sources lie below their destinations (Setup), the
// closure is a finite set of byte intervals, and the blocks it touches are
// all a decode of the range needs (random-access section: seek into a
// resident archive).  The token index behind this (the matches of every
// block) is built once by a device parse of the archive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <unordered_map>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

#include "aceapex.h"
#include "ax_common.h"
#include "engine.h"

namespace {

// Byte-precise set of needed output positions: one bitmap per touched block
// (B bits), allocated from a pool.  Inserting a range reports the runs of
// positions that were not needed before, which become new work.
class NeedSet {
 public:
  explicit NeedSet(uint64_t B) : B_(B), words_(B / 64) {}

  // Mark [a, b) needed; append to `fresh` the maximal runs newly marked.
  void insert(uint64_t a, uint64_t b, std::vector<std::pair<uint64_t, uint64_t>>& fresh) {
    uint64_t run0 = 0;
    bool open = false;
    while (a < b) {
      const uint64_t blk = a / B_, base = blk * B_, e = std::min(b, base + B_);
      uint64_t* bm = bitmap(blk);
      for (uint64_t p = a; p < e;) {
        const uint64_t w = (p - base) >> 6, bit = (p - base) & 63;
        const uint64_t n = std::min<uint64_t>(64 - bit, e - p);
        const uint64_t m = (n == 64 ? ~0ull : ((1ull << n) - 1)) << bit;
        uint64_t nw = m & ~bm[w];
        bm[w] |= m;
        // walk the word's bits [bit, bit + n): runs of newly marked positions
        uint64_t q = bit;
        while (q < bit + n) {
          const bool isnew = (nw >> q) & 1;
          const uint64_t rest = isnew ? ~nw : nw;  // first position where the state flips
          uint64_t flip = rest >> q ? q + __builtin_ctzll(rest >> q) : 64;
          flip = std::min<uint64_t>(flip, bit + n);
          const uint64_t pa = base + w * 64 + q;
          if (isnew && !open) run0 = pa, open = true;
          if (!isnew && open) fresh.emplace_back(run0, pa), open = false;
          q = flip;
        }
        p += n;
      }
      a = e;
    }
    if (open) fresh.emplace_back(run0, b);
  }

  // Ascending list of touched blocks (appended to out).
  void blocks(std::vector<uint64_t>& out) const {
    const size_t at = out.size();
    for (const auto& kv : slot_) out.push_back(kv.first);
    std::sort(out.begin() + at, out.end());
  }
  size_t count() const { return slot_.size(); }

 private:
  uint64_t* bitmap(uint64_t blk) {
    if (blk == last_blk_) return pool_.data() + last_at_;  // runs of lookups hit one block
    auto it = slot_.find(blk);
    if (it == slot_.end()) {
      it = slot_.emplace(blk, pool_.size()).first;
      pool_.resize(pool_.size() + words_, 0);
    }
    last_blk_ = blk;
    last_at_ = it->second;
    return pool_.data() + it->second;
  }
  uint64_t B_, words_;
  std::unordered_map<uint64_t, size_t> slot_;
  std::vector<uint64_t> pool_;
  uint64_t last_blk_ = ~0ull;
  size_t last_at_ = 0;
};

// Host threads for the closures of n ranges: one per 8 ranges when they are
// short (a closure takes microseconds, starting a thread tens of them), one
// per range of at least 64 KiB (its closure takes milliseconds), 16 at most
// by default (the process may see more cores than its share).
uint32_t closure_threads(uint32_t n, const uint64_t* lens, uint32_t threads) {
  uint32_t big = 0;
  for (uint32_t i = 0; i < n; ++i) big += lens[i] >= (64u << 10);
  const uint32_t cap = threads ? threads : std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  return std::max(1u, std::min({cap, std::max((n + 7) / 8, big), 64u}));
}

// Closure of one range: every position whose byte the range's bytes depend
// on, found by following each needed match byte to its source.
void closure_of(const aceapex_decoder* d, uint64_t off, uint64_t len, NeedSet& need) {
  const uint64_t B = d->info.block_size;
  const auto& src = d->idx_src;
  const auto& dl = d->idx_dstlen;
  std::vector<std::pair<uint64_t, uint64_t>> work;
  need.insert(off, off + len, work);
  while (!work.empty()) {
    const auto iv = work.back();
    work.pop_back();
    // matches of the blocks under [a, b)
    for (uint64_t blk = iv.first / B; blk <= (iv.second - 1) / B; ++blk) {
      uint64_t lo = d->mpre[blk], hi = d->mpre[blk + 1];
      // first match ending after a
      uint64_t x = lo, y = hi;
      while (x < y) {
        const uint64_t mid = (x + y) / 2;
        const uint64_t e = (dl[mid] & ((1ull << 48) - 1)) + (dl[mid] >> 48) + 1;
        if (e <= iv.first) x = mid + 1; else y = mid;
      }
      for (uint64_t t = x; t < hi; ++t) {
        const uint64_t dst = dl[t] & ((1ull << 48) - 1), n = (dl[t] >> 48) + 1;
        if (dst >= iv.second) break;
        const uint64_t k0 = std::max(iv.first, dst) - dst, k1 = std::min(iv.second, dst + n) - dst;
        const uint64_t dist = dst - src[t];
        if (k1 - k0 >= dist) {
          need.insert(src[t], src[t] + std::min(n, dist), work);
        } else {
          const uint64_t a = k0 % dist, b = a + (k1 - k0);
          if (b <= dist) need.insert(src[t] + a, src[t] + b, work);
          else need.insert(src[t] + a, src[t] + dist, work), need.insert(src[t], src[t] + (b - dist), work);
        }
      }
    }
  }
}

// The closure cache: lookups and bounded inserts (cleared when it holds more
// than 2^22 block entries).
bool cached_closure(const aceapex_decoder* d, uint64_t off, uint64_t len, std::vector<uint64_t>& out) {
  std::lock_guard<std::mutex> lock(d->ccache_mu);
  auto it = d->ccache.find(ax::RangeKey{off, len});
  if (it == d->ccache.end()) return false;
  out.insert(out.end(), it->second.begin(), it->second.end());
  return true;
}
void cache_closure(const aceapex_decoder* d, uint64_t off, uint64_t len, const uint64_t* b, size_t n) {
  std::lock_guard<std::mutex> lock(d->ccache_mu);
  if (d->ccache_blocks + n > (uint64_t(1) << 22)) d->ccache.clear(), d->ccache_blocks = 0;
  auto& v = d->ccache[ax::RangeKey{off, len}];
  if (v.empty()) v.assign(b, b + n), d->ccache_blocks += n;
}

// Closures of many ranges in parallel, merged into one ascending block list.
int union_closure(const aceapex_decoder* d, uint32_t n, const uint64_t* offs, const uint64_t* lens,
                  std::vector<uint64_t>& blocks, uint32_t threads) {
  const uint64_t N = d->info.n_bytes;
  for (uint32_t i = 0; i < n; ++i)
    if (offs[i] > N || lens[i] > N - offs[i]) return ax::fail(AX_E_RANGE, "range outside the archive");
  if (d->idx_dstlen.size() != d->info.n_matches) return ax::fail(AX_E_ARG, "token index not built");
  const uint32_t T = closure_threads(n, lens, threads);
  std::vector<std::vector<uint64_t>> part(T);
  std::atomic<uint32_t> next{0};
  auto worker = [&](uint32_t w) {
    for (;;) {
      const uint32_t i = next.fetch_add(1);
      if (i >= n) break;
      if (!lens[i] || cached_closure(d, offs[i], lens[i], part[w])) continue;
      NeedSet need(d->info.block_size);
      closure_of(d, offs[i], lens[i], need);
      need.blocks(part[w]);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (uint32_t w = 1; w < T; ++w) pool.emplace_back(worker, w);
    worker(0);
    for (auto& t : pool) t.join();
    blocks.clear();
    for (auto& p : part) blocks.insert(blocks.end(), p.begin(), p.end());
    std::sort(blocks.begin(), blocks.end());
    blocks.erase(std::unique(blocks.begin(), blocks.end()), blocks.end());
  } catch (const std::bad_alloc&) {
    return ax::fail(AX_E_NOMEM, "closure");
  }
  return AX_OK;
}

// Copy range bytes from the compact scratch to each caller buffer.  Byte p
// of the archive lives at scratch + slot[p / B] * B + p mod B (the range's
// blocks are all in the plan, so their slots are set).  Every range is cut
// into 4 KiB chunks numbered across the batch (chunk0 is a range's first
// chunk); a workgroup copies one chunk, each thread sixteen bytes with all
// loads issued before the stores, so wide ranges spread over the whole
// device and every byte instruction of a wave covers 64 consecutive bytes.
// Destination alignments are arbitrary.
constexpr uint32_t kGatherThreads = 256;
constexpr uint32_t kGatherChunk = 16 * kGatherThreads;

struct GatherDesc {
  uint64_t off;  // archive position of the range's first byte
  uint8_t* dst;
  uint64_t len;
  uint64_t chunk0;
};

struct ScratchMap {
  const uint8_t* base;
  const uint32_t* slot;
  uint32_t lb, junk;
};

__global__ __launch_bounds__(kGatherThreads) void k_gather(const GatherDesc* desc, uint32_t n, uint64_t chunks,
                                                           ScratchMap m) {
  typedef const __attribute__((address_space(1))) uint8_t* cgbytes;
  const __attribute__((address_space(1))) uint32_t* slot = (const __attribute__((address_space(1))) uint32_t*)m.slot;
  const uint64_t bmask = (1ull << m.lb) - 1;
  for (uint64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
    uint32_t lo = 0, hi = n - 1;  // last range whose first chunk is <= c
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (desc[mid].chunk0 <= c) lo = mid; else hi = mid - 1;
    }
    const GatherDesc g = desc[lo];
    __attribute__((address_space(1))) uint8_t* dst = (__attribute__((address_space(1))) uint8_t*)g.dst;
    const uint64_t base = (c - g.chunk0) * kGatherChunk + threadIdx.x;
    uint8_t v[16];
#pragma unroll
    for (uint32_t q = 0; q < 16; ++q) {
      const uint64_t k = base + q * kGatherThreads;
      if (k < g.len) {
        const uint64_t p = g.off + k;
        uint32_t x = slot[p >> m.lb];
        if (x >= m.junk) x = m.junk;
        v[q] = ((cgbytes)m.base)[(uint64_t(x) << m.lb) + (p & bmask)];
      } else {
        v[q] = 0;
      }
    }
#pragma unroll
    for (uint32_t q = 0; q < 16; ++q) {
      const uint64_t k = base + q * kGatherThreads;
      if (k < g.len) dst[k] = v[q];
    }
  }
}

// Workspace of a range decode whose closure is at most `blocks` blocks and
// `tokens` matches: the plan's workspace, the compact scratch ((blocks + 1)
// blocks: the last is the junk block) and the slot table (one u32 per
// archive block), each 256-byte aligned.
struct RangeLayout {
  uint64_t plan, scratch_at, slot_at, total;
};
RangeLayout range_layout(const aceapex_decoder* d, uint64_t blocks, uint64_t tokens) {
  RangeLayout L;
  const uint64_t B = d->info.block_size;
  L.plan = ax::plan_workspace_for(d, blocks, tokens);
  L.scratch_at = (L.plan + 255) & ~255ull;
  L.slot_at = (L.scratch_at + (blocks + 1) * B + 255) & ~255ull;
  L.total = L.slot_at + 4 * std::max<uint64_t>(1, d->info.n_blocks);
  return L;
}

}  // namespace

// A reusable range-decode plan: the decoder, capacity limits, the plan of
// the current closure and the pinned staging of the gather descriptors.
struct aceapex_range_plan {
  aceapex_decoder* dec = nullptr;
  uint64_t max_blocks = 0, max_tokens = 0;
  ax::Plan* plan = nullptr;          // rebuilt per call
  RangeLayout lay{};                 // for max_blocks / max_tokens
  GatherDesc* d_desc = nullptr;
  GatherDesc* h_desc = nullptr;
  uint32_t desc_cap = 0;
  hipEvent_t upload_done = nullptr;  // the pinned descriptors may be rewritten after this
  uint64_t last_blocks = 0, last_tokens = 0;
  ~aceapex_range_plan() {
    if (upload_done) {
      (void)hipEventSynchronize(upload_done);
      (void)hipEventDestroy(upload_done);
    }
    ax::plan_destroy(plan);
    if (d_desc) (void)hipFree(d_desc);
    if (h_desc) (void)hipHostFree(h_desc);
  }
};

namespace {

// Decode the union closure of n ranges with a range plan into its compact
// scratch and gather each range to its output (everything after the host
// closure is asynchronous on s).
// Closures of fewer matches than the decoder's AX_OPT_RANGE_JUMP_TOKENS
// finish their deep remainder with the persistent chase (few launches; their
// chains are short), larger ones by pointer jumping (a deep closure's chains
// are long).

int run_ranges(aceapex_range_plan* rp, const RangeLayout& lay, uint32_t n, const uint64_t* offs,
               const uint64_t* lens, uint8_t* const* d_outs, const uint64_t* out_caps, void* d_work,
               uint64_t work_len, int copy_mode, hipStream_t s, std::vector<uint64_t>* closure) {
  aceapex_decoder* d = rp->dec;
  if (!d_work) return ax::fail(AX_E_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(d_work) & 255) return ax::fail(AX_E_ARG, "workspace must be 256-byte aligned");
  if (work_len < lay.total) return ax::fail(AX_E_CAPACITY, "workspace too small");
  for (uint32_t i = 0; i < n; ++i) {
    if (lens[i] && !d_outs[i]) return ax::fail(AX_E_ARG, "null output");
    if (out_caps[i] < lens[i]) return ax::fail(AX_E_CAPACITY, "output smaller than its range");
  }
  std::vector<uint64_t> bl;
  int rc = AX_OK;
  if (closure) bl.swap(*closure);  // computed by the caller
  else rc = union_closure(d, n, offs, lens, bl, 0);
  if (rc) return rc;
  uint64_t tok = 0;
  for (uint64_t b : bl) tok += d->mpre[b + 1] - d->mpre[b];
  if (bl.size() > rp->max_blocks || tok > rp->max_tokens)
    return ax::fail(AX_E_CAPACITY, "closure larger than the plan's capacity");
  rp->last_blocks = bl.size();
  rp->last_tokens = tok;
  uint8_t* const w = static_cast<uint8_t*>(d_work);
  uint8_t* const scratch = w + lay.scratch_at;
  uint32_t* const slot = reinterpret_cast<uint32_t*>(w + lay.slot_at);
  // the previous call's uploads must be through before staging is rewritten
  (void)hipEventSynchronize(rp->upload_done);
  if (!bl.empty()) {
    ax::JobSpec js{d, scratch, std::move(bl), slot, uint32_t(rp->max_blocks)};
    if (!rp->plan) {
      rc = ax::plan_create({js}, &rp->plan);
      if (!rc) ax::plan_set_learn(rp->plan, false);
    } else {
      rc = ax::plan_reset(rp->plan, {js}, s);
    }
    if (rc) return rc;
    ax::plan_copy_options(rp->plan, d->plan);
    int64_t jump_from = 0;
    (void)ax::plan_get_option(d->plan, AX_OPT_RANGE_JUMP_TOKENS, &jump_from);
    rc = ax::plan_set_option(rp->plan, AX_OPT_TAIL_MODE, int64_t(tok) >= jump_from ? 0 : 1);
    if (!rc) rc = ax::plan_set_slots(rp->plan, slot, s);
    if (!rc) rc = ax::plan_run(rp->plan, d_work, lay.plan, copy_mode, s);
    if (rc) return rc;
  }
  if (n) {
    if (n > rp->desc_cap) {
      if (rp->d_desc) (void)hipFree(rp->d_desc), rp->d_desc = nullptr;
      if (rp->h_desc) (void)hipHostFree(rp->h_desc), rp->h_desc = nullptr;
      rp->desc_cap = std::max<uint32_t>(n, 2 * rp->desc_cap);
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&rp->d_desc), sizeof(GatherDesc) * rp->desc_cap);
      if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&rp->h_desc), sizeof(GatherDesc) * rp->desc_cap);
      if (e != hipSuccess) return ax::fail(AX_E_HIP, hipGetErrorString(e));
    }
    uint64_t chunks = 0;
    for (uint32_t i = 0; i < n; ++i) {
      rp->h_desc[i] = GatherDesc{offs[i], d_outs[i], lens[i], chunks};
      chunks += (lens[i] + kGatherChunk - 1) / kGatherChunk;
    }
    hipError_t e = hipMemcpyAsync(rp->d_desc, rp->h_desc, sizeof(GatherDesc) * n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return ax::fail(AX_E_HIP, hipGetErrorString(e));
    const ScratchMap m{scratch, slot, uint32_t(__builtin_ctz(d->info.block_size)), uint32_t(rp->max_blocks)};
    if (chunks)
      hipLaunchKernelGGL(k_gather, dim3(uint32_t(std::min<uint64_t>(chunks, 8192))), dim3(kGatherThreads), 0, s,
                         rp->d_desc, n, chunks, m);
    e = hipGetLastError();
    if (e != hipSuccess) return ax::fail(AX_E_HIP, hipGetErrorString(e));
  }
  (void)hipEventRecord(rp->upload_done, s);
  return AX_OK;
}

}  // namespace

extern "C" {

int aceapex_decoder_build_index(aceapex_decoder* d, void* d_work, uint64_t work_len, void* stream) {
  if (!d || !d_work) return ax::fail(AX_E_ARG, "null argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  try {
    d->idx_src.assign(d->info.n_matches, 0);
    d->idx_dstlen.assign(d->info.n_matches, 0);
  } catch (const std::bad_alloc&) {
    return ax::fail(AX_E_NOMEM, "token index");
  }
  return ax::plan_parse_tokens(d->plan, d_work, work_len, s, d->idx_src.data(), d->idx_dstlen.data());
}

int aceapex_decoder_tokens(const aceapex_decoder* d, uint64_t first, uint64_t count, uint64_t* src, uint64_t* dst,
                           uint32_t* len) {
  if (!d || (count && (!src || !dst || !len))) return ax::fail(AX_E_ARG, "null argument");
  if (d->idx_dstlen.size() != d->info.n_matches) return ax::fail(AX_E_ARG, "token index not built");
  if (first > d->info.n_matches || count > d->info.n_matches - first)
    return ax::fail(AX_E_RANGE, "matches outside the archive");
  for (uint64_t i = 0; i < count; ++i) {
    const uint64_t w = d->idx_dstlen[first + i];
    src[i] = d->idx_src[first + i];
    dst[i] = w & ((1ull << 48) - 1);
    len[i] = uint32_t(w >> 48) + 1;
  }
  return AX_OK;
}

int aceapex_closure_sizes(const aceapex_decoder* d, uint32_t n, const uint64_t* offs, const uint64_t* lens,
                          uint64_t* blocks, uint64_t* tokens, uint32_t threads) {
  if (!d || (n && (!offs || !lens || !blocks || !tokens))) return ax::fail(AX_E_ARG, "null argument");
  const uint64_t N = d->info.n_bytes;
  for (uint32_t i = 0; i < n; ++i)
    if (offs[i] > N || lens[i] > N - offs[i]) return ax::fail(AX_E_RANGE, "range outside the archive");
  if (d->idx_dstlen.size() != d->info.n_matches) return ax::fail(AX_E_ARG, "token index not built");
  const uint32_t T = closure_threads(n, lens, threads);
  std::atomic<uint32_t> next{0};
  std::atomic<int> failed{0};
  auto worker = [&]() {
    std::vector<uint64_t> bl;
    for (;;) {
      const uint32_t i = next.fetch_add(1);
      if (i >= n) break;
      bl.clear();
      if (lens[i] && !cached_closure(d, offs[i], lens[i], bl)) {
        try {
          NeedSet need(d->info.block_size);
          closure_of(d, offs[i], lens[i], need);
          need.blocks(bl);
          cache_closure(d, offs[i], lens[i], bl.data(), bl.size());
        } catch (const std::bad_alloc&) {
          failed = 1;
          break;
        }
      }
      uint64_t t = 0;
      for (uint64_t b : bl) t += d->mpre[b + 1] - d->mpre[b];
      blocks[i] = bl.size();
      tokens[i] = t;
    }
  };
  try {
    std::vector<std::thread> pool;
    for (uint32_t w = 1; w < T; ++w) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
  } catch (const std::system_error&) {
    return ax::fail(AX_E_NOMEM, "closure threads");
  }
  return failed ? ax::fail(AX_E_NOMEM, "closure") : AX_OK;
}

int aceapex_closure_blocks(aceapex_decoder* d, uint32_t n, const uint64_t* offs, const uint64_t* lens,
                           uint64_t* blocks, uint64_t cap, uint64_t* n_blocks, uint64_t* n_tokens, uint32_t threads) {
  if (!d || (n && (!offs || !lens)) || !n_blocks) return ax::fail(AX_E_ARG, "null argument");
  std::vector<uint64_t> bl;
  int rc = union_closure(d, n, offs, lens, bl, threads);
  if (rc) return rc;
  *n_blocks = bl.size();
  if (n_tokens) {
    uint64_t t = 0;
    for (uint64_t b : bl) t += d->mpre[b + 1] - d->mpre[b];
    *n_tokens = t;
  }
  if (blocks) {
    if (cap < bl.size()) return ax::fail(AX_E_CAPACITY, "block list capacity");
    std::copy(bl.begin(), bl.end(), blocks);
  }
  return AX_OK;
}

int aceapex_range_plan_create(aceapex_decoder* d, uint64_t max_blocks, uint64_t max_tokens,
                              aceapex_range_plan** out) {
  if (!d || !out || !max_blocks) return ax::fail(AX_E_ARG, "null argument");
  *out = nullptr;
  if (max_blocks > ax::kWindowBlocks || max_tokens > ax::kWindowTokens)
    return ax::fail(AX_E_ARG, "range plans hold one window of blocks");
  aceapex_range_plan* rp = new (std::nothrow) aceapex_range_plan;
  if (!rp) return ax::fail(AX_E_NOMEM, "range plan");
  rp->dec = d;
  rp->max_blocks = max_blocks;
  rp->max_tokens = max_tokens;
  rp->lay = range_layout(d, max_blocks, max_tokens);
  if (hipEventCreateWithFlags(&rp->upload_done, hipEventDisableTiming) != hipSuccess) {
    delete rp;
    return ax::fail(AX_E_HIP, "event");
  }
  *out = rp;
  return AX_OK;
}

void aceapex_range_plan_destroy(aceapex_range_plan* rp) { delete rp; }

int aceapex_range_plan_workspace(const aceapex_range_plan* rp, uint64_t* bytes) {
  if (!rp || !bytes) return ax::fail(AX_E_ARG, "null argument");
  *bytes = rp->lay.total;
  return AX_OK;
}

int aceapex_range_plan_last(const aceapex_range_plan* rp, uint64_t* blocks, uint64_t* tokens) {
  if (!rp || !blocks || !tokens) return ax::fail(AX_E_ARG, "null argument");
  *blocks = rp->last_blocks;
  *tokens = rp->last_tokens;
  return AX_OK;
}

int aceapex_decode_ranges(aceapex_range_plan* rp, uint32_t n, const uint64_t* offs, const uint64_t* lens,
                          uint8_t* const* d_outs, const uint64_t* out_caps, void* d_work, uint64_t work_len,
                          int copy_mode, void* stream) {
  if (!rp || (n && (!offs || !lens || !d_outs || !out_caps))) return ax::fail(AX_E_ARG, "null argument");
  return run_ranges(rp, rp->lay, n, offs, lens, d_outs, out_caps, d_work, work_len, copy_mode,
                    reinterpret_cast<hipStream_t>(stream), nullptr);
}

int aceapex_range_workspace(const aceapex_decoder* d, uint64_t off, uint64_t len, uint64_t* bytes) {
  if (!d || !bytes) return ax::fail(AX_E_ARG, "null argument");
  std::vector<uint64_t> bl;
  int rc = len ? union_closure(d, 1, &off, &len, bl, 1) : AX_OK;
  if (rc) return rc;
  uint64_t tok = 0;
  for (uint64_t b : bl) tok += d->mpre[b + 1] - d->mpre[b];
  if (bl.size() > ax::kWindowBlocks || tok > ax::kWindowTokens)
    return ax::fail(AX_E_CAPACITY, "closure larger than one window");
  *bytes = range_layout(d, std::max<uint64_t>(1, bl.size()), tok).total;
  return AX_OK;
}

int aceapex_decode_range(aceapex_decoder* d, uint64_t off, uint64_t len, uint8_t* d_out, uint64_t out_cap,
                         void* d_work, uint64_t work_len, void* stream) {
  if (!d) return ax::fail(AX_E_ARG, "null decoder");
  if (!d->range) {
    aceapex_range_plan* rp = nullptr;
    int rc = aceapex_range_plan_create(d, ax::kWindowBlocks, ax::kWindowTokens, &rp);
    if (rc) return rc;
    d->range = rp;
  }
  std::vector<uint64_t> bl;
  int rc = len ? union_closure(d, 1, &off, &len, bl, 1) : AX_OK;
  if (rc) return rc;
  uint64_t tok = 0;
  for (uint64_t b : bl) tok += d->mpre[b + 1] - d->mpre[b];
  if (bl.size() > ax::kWindowBlocks || tok > ax::kWindowTokens)
    return ax::fail(AX_E_CAPACITY, "closure larger than one window");
  // the workspace this range needs (aceapex_range_workspace), laid out for its own closure
  const RangeLayout lay = range_layout(d, std::max<uint64_t>(1, bl.size()), tok);
  aceapex_range_plan* rp = d->range;
  rp->max_blocks = std::max<uint64_t>(1, bl.size());
  rp->max_tokens = tok;
  uint8_t* outs[1] = {d_out};
  return run_ranges(rp, lay, 1, &off, &len, outs, &out_cap, d_work, work_len, AX_COPY_PERIODIC,
                    reinterpret_cast<hipStream_t>(stream), &bl);
}

}  // extern "C"
