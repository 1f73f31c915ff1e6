// Device decoder of the AXP1 absolute-offset LZ77 block format for gfx950.
//
// Three kernels per window of blocks (the paper's ANS / parse / copy split,
// Table 2):
//   k_ans    one wave64 per (block, stream): order-0 rANS of the literal,
//            length, offset and command streams with the slot table in LDS;
//            renormalisation words are handed to the lanes that need them by
//            ballot + prefix count over a register window of the word stream.
//   k_parse  one workgroup per block: commands are parsed 256 at a time by
//            block-wide prefix scans (positions, literal positions, value
//            indices; DPP moves inside the wave) and an associative scan of
//            the four-entry distance history (each command is a map on
//            history tuples); literal runs are placed into an LDS tile that
//            is written out with 16-byte stores; matches become tokens
//            (src, dst, len).
//   match layer: every token (src, dst, len) is written as a periodic fill
//            out[dst+k] = out[src + k mod dist] (periodic-fill section).  The
//            tokens whose destinations meet a token's source bytes form one
//            contiguous index range (tokens are stored in output order), found
//            once by binary search; a token is ready when those are done.
//            k_round0 (a workgroup per block, fills gathered in an LDS tile of
//            the block's chunks that receive match bytes) and k_round run
//            level-synchronous rounds (the dependency levels of the paper's
//            wavefront decoder) with plain cached accesses, the kernel
//            boundary being the only synchronisation.  The last round
//            marks its leftovers in a bitmap, which k_pcount / k_pscatter
//            compact into an ascending list; k_tail then finishes that deep
//            remainder in one persistent launch, waves taking 64-token chunks
//            of the list from a ticket counter and publishing through
//            agent-coherent stores, so a dependency hop costs a memory round
//            trip rather than an L2 writeback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "aceapex.h"
#include "ax_common.h"
#include "engine.h"

namespace {

// Device pointers that kernels load from memory (job tables) or select at run
// time lose their address space; accesses through generic pointers become
// flat instructions, which also count against the LDS wait counter.  Kernels
// convert them to global pointers explicitly.
#define AX_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ inline AX_GLOBAL T* gp(T* p) {
  return (AX_GLOBAL T*)p;
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef u32x4 u32x4_u __attribute__((aligned(1)));  // 16 bytes at any byte address (one dwordx4 load)

constexpr uint32_t kMaxB = 16384;           // largest block the device path decodes
constexpr uint32_t kParseThreads = 256;
constexpr uint32_t kOffStage = 1792;        // offset-stream bytes staged in LDS by k_parse
constexpr uint32_t kLenStage = 256;         // length-stream bytes staged in LDS by k_parse
constexpr uint32_t kLenBpt = 1, kOffBpt = 2;  // LEB bytes per thread per pass: length / offset streams
constexpr uint32_t kCopyThreads = 256;      // match-layer workgroup
constexpr uint8_t kPending = 0xFF;          // done[] value of a token not yet copied
constexpr uint32_t kSub = 64;               // pending-list sublists (one counter each, 256 B apart)
constexpr uint32_t kCounterStride = 64;     // u32 between two sublist counters
constexpr uint32_t kMaxRoundGrid = 4096;    // workgroups of a round launch
// last round: list the leftovers (persistent launch) or mark them for
// pointer jumping (first entries and leftover-map bits)
constexpr int kMarkList = 1, kMarkJump = 2;

struct DevStatus {
  int32_t err;
  uint32_t pad0;
  unsigned long long bad_block;
  uint32_t ticket;
  uint32_t long_count;
  uint32_t n_pending;  // tokens the bulk rounds left (the deep remainder)
  uint32_t pad2;
  uint32_t jump_used;    // jump passes that found active entries (0: all of them did)
  uint32_t n_jwords;     // leftover-map words with bits set (the jump kernels' work list)
  uint32_t pend0;        // tokens round 0 left to the later rounds (reported when asked)
  uint32_t pad1[53];
};
static_assert(sizeof(DevStatus) == 256, "status block is 256 bytes");

// One archive of a plan (a whole-archive decode, one archive of a batch, or
// the source closure of a range): where it is, and where its bytes go.
struct JobDev {
  const uint8_t* arc;   // device archive
  uint8_t* out;         // decoded bytes: at the archive's absolute positions, or by slot (below)
  uint64_t payload_at;  // header + index bytes
  uint64_t n_bytes, nb;
  uint32_t B, mm;
  // a range decode's compact scratch: block b's bytes at out + slot[b] * B;
  // a slot of `junk` or more means the junk block (blocks the plan does not
  // decode; only bytes nobody needs are read from it).  null: absolute.
  const uint32_t* slot;
  uint32_t junk;
};

// One block of a window.  A window holds the blocks of its jobs job by job
// (in the plan's window order of jobs), ascending within a job, and the
// window's tokens are stored block after block in that order.
struct WinBlock {
  uint64_t b;       // block index in its archive
  uint32_t job;
  uint32_t tok;     // window index of the block's first token
  uint32_t first;   // window index of this job's first block in the window
  uint32_t count;   // blocks of this job in the window
};

// Where the bytes of archive position p of a job's output live.  OutDirect:
// the output holds the archive at its absolute positions (whole-archive and
// batch decodes).  OutMapped: a range decode's compact scratch, the bytes of
// block b at slot[b] * B (the slot table is set for the blocks the plan
// decodes; any other block maps to the junk block, whatever its entry holds,
// so a stale entry can never send an access outside the scratch).  Copy
// kernels are instantiated for each; the whole-archive path compiles to the
// plain pointer arithmetic.
typedef AX_GLOBAL uint8_t* gbytes;
struct OutDirect {
  gbytes base;
  __device__ explicit OutDirect(const JobDev& j) : base(gp(j.out)) {}
  __device__ OutDirect with_base(gbytes b) const { OutDirect o = *this; o.base = b; return o; }
  __device__ gbytes at(uint64_t p) const { return base + p; }
  __device__ bool contiguous(uint64_t, uint32_t) const { return true; }  // n bytes from p in one piece
};
struct OutMapped {
  gbytes base;
  const AX_GLOBAL uint32_t* slot;
  uint32_t lb, junk;
  __device__ explicit OutMapped(const JobDev& j)
      : base(gp(j.out)), slot(gp(j.slot)), lb(uint32_t(__builtin_ctz(j.B))), junk(j.junk) {}
  __device__ OutMapped with_base(gbytes b) const { OutMapped o = *this; o.base = b; return o; }
  __device__ gbytes at(uint64_t p) const {
    uint32_t x = slot[p >> lb];
    if (x >= junk) x = junk;
    return base + (uint64_t(x) << lb) + (p & ((1u << lb) - 1u));
  }
  __device__ bool contiguous(uint64_t p, uint32_t n) const { return (p & ((1u << lb) - 1u)) + n <= (1u << lb); }
};

__device__ inline uint32_t job_off_cap(const JobDev& j) { return (10u * (j.B / j.mm + 1) + 15u) & ~15u; }
__device__ inline uint32_t job_len_cap(const JobDev& j) { return 3u * j.B; }

__device__ inline void report(DevStatus* st, int code, uint64_t block) {
  if (atomicCAS(&st->err, 0, code) == 0) atomicExch(&st->bad_block, (unsigned long long)block);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }
// Fourth word of a raw buffer descriptor on gfx9-family parts (32-bit data
// format; untyped byte stores ignore it)
constexpr int kBufferWord3 = 0x00020000;

__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ inline uint32_t ld32(const uint8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
__device__ inline uint64_t ld64(const uint8_t* p) { return *reinterpret_cast<const uint64_t*>(p); }

// ------------------------------------------------------------------ k_ans --

struct AnsArgs {
  const JobDev* jobs;
  const WinBlock* wbl;       // this window's blocks
  uint32_t n_items;          // blocks in this window
  uint32_t slot_b;           // scratch slot stride of the literal and command streams
  uint8_t* lit;              // scratch, slot_b per slot
  uint8_t* cmd;              // scratch, slot_b per slot
  uint8_t* off;              // scratch, off_cap per slot
  uint8_t* len;              // scratch, len_cap per slot
  uint32_t off_cap, len_cap;
  uint32_t* nsym;            // 4 per slot
  DevStatus* st;
};

// Wave-level exclusive prefix sum of a u32.
__device__ inline uint32_t wave_excl_sum(uint32_t v, uint32_t* total) {
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane_id() >= (uint32_t)o) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

__global__ __launch_bounds__(64) void k_ans(AnsArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t symtab[ax::kProbScale];
  // f | cum << 16 indexed by symbol; while the slot table is filled, the same
  // bytes hold the cum (sentinel 4096) and the symbol of the k-th present one
  __shared__ __attribute__((aligned(16))) uint32_t fctab[256];
  uint16_t* const cumtab = reinterpret_cast<uint16_t*>(fctab);         // 257 entries
  uint8_t* const symlist = reinterpret_cast<uint8_t*>(fctab) + 2 * 260;  // 256 entries

  const uint32_t item = blockIdx.x % a.n_items;
  const uint32_t stream = blockIdx.x / a.n_items;  // 0 LIT, 1 LEN, 2 OFF, 3 CMD
  const WinBlock wb = a.wbl[item];
  const JobDev& J = a.jobs[wb.job];
  const uint64_t b = wb.b;
  const uint32_t lane = lane_id();
  uint8_t* const outs[4] = {a.lit + uint64_t(item) * a.slot_b, a.len + uint64_t(item) * a.len_cap,
                            a.off + uint64_t(item) * a.off_cap, a.cmd + uint64_t(item) * a.slot_b};
  const uint32_t caps[4] = {J.B, job_len_cap(J), job_off_cap(J), J.B};
  AX_GLOBAL uint8_t* const out = gp(outs[stream]);
  const uint32_t cap = caps[stream];
  uint32_t* nsym = a.nsym + 4 * item + stream;

  const uint64_t* idx = reinterpret_cast<const uint64_t*>(J.arc + 64);
  const uint64_t o0 = idx[b], o1 = idx[b + 1];
  const uint8_t* blk = J.arc + J.payload_at + o0;
  const uint64_t blen = o1 - o0;  // validated on the host: >= 16, 16-aligned
  uint64_t at = 16;
  for (uint32_t k = 0; k < stream; ++k) at += ld32(blk + 4 * k);
  const uint32_t rlen = ld32(blk + 4 * stream);
  if (at + rlen > blen || rlen < 8 || (rlen & 3)) {
    if (lane == 0) { report(a.st, AX_E_CORRUPT, b); *nsym = 0; }
    return;
  }
  const uint8_t* rec = blk + at;
  const uint32_t n = ld32(rec), mode = rec[4], pa = rec[5], pb = rec[6];
  if (n > cap) {
    if (lane == 0) { report(a.st, AX_E_CORRUPT, b); *nsym = 0; }
    return;
  }
  if (mode == 0) {  // raw: copy 4 bytes per lane per step
    if (8 + uint64_t(n) > rlen) {
      if (lane == 0) { report(a.st, AX_E_CORRUPT, b); *nsym = 0; }
      return;
    }
    const uint32_t words = (n + 3) / 4;
    for (uint32_t w = lane; w < words; w += 64)
      reinterpret_cast<AX_GLOBAL uint32_t*>(out)[w] = gp(reinterpret_cast<const uint32_t*>(rec + 8))[w];
    if (lane == 0) *nsym = n;
    return;
  }
  if (mode == 1) {  // constant
    const uint32_t v = pa * 0x01010101u, words = (n + 3) / 4;
    for (uint32_t w = lane; w < words; w += 64) reinterpret_cast<AX_GLOBAL uint32_t*>(out)[w] = v;
    if (lane == 0) *nsym = n;
    return;
  }
  bool bad = mode != 2 || pa > ax::kMaxLanesLog2 || rlen < 12;
  const uint32_t K = 1u << (pa & 7), present = pb + 1;
  bad |= present < 2;
  uint64_t p = 12;
  const uint32_t nw = bad ? 0 : ld32(rec + 8);
  const uint64_t states_at = p;
  p += 4ull * K;
  const uint64_t words_at = p;
  p = (p + 2ull * nw + 3) & ~3ull;
  const uint64_t set_at = p;
  p += present <= 32 ? present : 32;
  p = (p + 1) & ~1ull;
  const uint64_t freq_at = p;
  p = (p + 2ull * present + 3) & ~3ull;
  bad |= p != rlen;
  if (bad) {
    if (lane == 0) { report(a.st, AX_E_CORRUPT, b); *nsym = 0; }
    return;
  }
  // --- table: lane l holds up to four present symbols in ascending order.
  uint32_t mysym[4], myf[4], cnt = 0;
  if (present <= 32) {
    if (lane < present) { mysym[0] = rec[set_at + lane]; cnt = 1; }
  } else {
    const uint32_t bits = (rec[set_at + (lane >> 1)] >> ((lane & 1) * 4)) & 15u;
    for (uint32_t j = 0; j < 4; ++j)
      if (bits >> j & 1) mysym[cnt++] = lane * 4 + j;
  }
  uint32_t total_present;
  const uint32_t rank0 = wave_excl_sum(cnt, &total_present);
  uint32_t fsum = 0;
  bad = total_present != present;
  for (uint32_t j = 0; j < cnt; ++j) {
    myf[j] = (rank0 + j < present) ? *reinterpret_cast<const uint16_t*>(rec + freq_at + 2 * (rank0 + j)) : 0;
    bad |= myf[j] < 1 || myf[j] >= ax::kProbScale;
    fsum += myf[j];
  }
  if (present <= 32 && cnt && lane > 0) bad |= rec[set_at + lane - 1] >= mysym[0];  // strictly ascending
  uint32_t ftotal;
  uint32_t cum = wave_excl_sum(fsum, &ftotal);
  bad |= ftotal != ax::kProbScale;
  if (__ballot(bad)) {
    if (lane == 0) { report(a.st, AX_E_CORRUPT, b); *nsym = 0; }
    return;
  }
  {
    uint32_t c = cum;
    for (uint32_t j = 0; j < cnt; ++j) {
      cumtab[rank0 + j] = uint16_t(c);
      symlist[rank0 + j] = uint8_t(mysym[j]);
      c += myf[j];
    }
  }
  if (lane == 0) cumtab[present] = ax::kProbScale;
  __syncthreads();
  {  // slot -> symbol: lane l fills slots [64l, 64l+64) four at a time
    const uint32_t s0 = lane * 64;
    uint32_t lo = 0, hi = present - 1;  // last k with cumtab[k] <= s0
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (cumtab[mid] <= s0) lo = mid; else hi = mid - 1;
    }
    uint32_t k = lo, next = cumtab[k + 1];
    if (next >= s0 + 64) {  // one symbol owns all 64 slots: four 16-byte stores
      const uint32_t rep = uint32_t(symlist[k]) * 0x01010101u;
      const u32x4 v = {rep, rep, rep, rep};
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) *reinterpret_cast<u32x4*>(symtab + s0 + 16 * q) = v;
    } else {
      for (uint32_t s = s0; s < s0 + 64; s += 4) {
        uint32_t packed = 0;
        for (uint32_t q = 0; q < 4; ++q) {
          while (s + q >= next) { ++k; next = cumtab[k + 1]; }
          packed |= uint32_t(symlist[k]) << (8 * q);
        }
        *reinterpret_cast<uint32_t*>(symtab + s) = packed;
      }
    }
  }
  __syncthreads();
  for (uint32_t j = 0; j < cnt; ++j) {  // now the frequency table (over the build's lists)
    fctab[mysym[j]] = myf[j] | (cum << 16);
    cum += myf[j];
  }
  __syncthreads();
  // --- decode: lane j owns symbols j, j+K, ...
  // The renormalisation words of a step are taken in lane order from a
  // window: lane l's register P holds word base+l in its low half and word
  // base+64+l in its high half, N holds word base+128+l (in flight while the
  // window is used).  A step's words lie in [ptr, ptr+64) with ptr-base < 64,
  // so one permute of P from lane (ptr-base+below) mod 64 and a byte select
  // of the half give each lane its word.  Once ptr-base reaches 64 the window
  // moves by 64: P takes its high half and N's word, and N is reloaded.  Loads
  // are unconditional, the index clamped to the last word (inside the record;
  // a valid stream never consumes a word past nw)
  const AX_GLOBAL uint16_t* words = gp(reinterpret_cast<const uint16_t*>(rec + words_at));
  uint32_t x = lane < K ? ld32(rec + states_at + 4 * lane) : ax::kRansLow;
  bad = x < ax::kRansLow;
  const uint32_t wlast = nw ? nw - 1 : 0;
  auto fetch = [&](uint32_t i) -> uint32_t { return uint32_t(words[i < wlast ? i : wlast]); };
  uint32_t base = 0;
  uint32_t P = fetch(lane) | (fetch(64 + lane) << 16), N = fetch(128 + lane);
  uint32_t ptr = 0;
  const uint32_t steps = (n + K - 1) / K;
  // one step for the lanes in `need` (a subset of the decoding lanes):
  // returns the new state of a lane from its decoded xn
  auto renorm = [&](uint64_t m, uint32_t xn, bool need) -> uint32_t {
    const uint32_t q = __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)) +
                       (ptr - base);  // < 128; the permute takes the lane mod 64
    const uint32_t v = __builtin_amdgcn_ds_bpermute(int(q << 2), int(P));
    // (xn << 16) | the word: xn's two low bytes above v's low or high half
    const uint32_t xr = __builtin_amdgcn_perm(xn, v, q < 64 ? 0x05040100u : 0x05040302u);
    ptr += __popcll(m);
    if (ptr - base >= 64) {
      base += 64;
      P = __builtin_amdgcn_perm(N, P, 0x05040302u);
      N = fetch(base + 128 + lane);
    }
    return need ? xr : xn;
  };
  // Steps with all K lanes decoding: no per-lane bounds; symbols leave
  // through a buffer store addressed by the lane plus a wave-uniform offset.
  // With K = 64 neither the ballot nor the store needs a lane mask
  const uint32_t full = n / K;
  const uint64_t kmask = K == 64 ? ~0ull : ((1ull << K) - 1ull);
  const __amdgpu_buffer_rsrc_t orsrc = __builtin_amdgcn_make_buffer_rsrc(outs[stream], 0, int(n), kBufferWord3);
  auto full_steps = [&](auto all_tag) {
    constexpr bool kAll = decltype(all_tag)::value;
    for (uint32_t t = 0; t < full; ++t) {
      const uint32_t slot = x & (ax::kProbScale - 1);
      const uint32_t s = symtab[slot];
      const uint32_t fc = fctab[s];
      const uint32_t xn = (fc & 0xFFFFu) * (x >> ax::kProbBits) + slot - (fc >> 16);
      const bool need = xn < ax::kRansLow;
      uint64_t m = __builtin_amdgcn_ballot_w64(need);
      if (!kAll) m &= kmask;
      if (kAll || lane < K) __builtin_amdgcn_raw_buffer_store_b8(uint8_t(s), orsrc, int(lane), int(t * K), 0);
      x = renorm(m, xn, need);
    }
  };
  if (K == 64) full_steps(std::true_type{});
  else full_steps(std::false_type{});
  uint32_t i = full * K + lane;
  for (uint32_t t = full; t < steps; ++t, i += K) {
    const bool act = lane < K && i < n;
    const uint32_t slot = x & (ax::kProbScale - 1);
    const uint32_t s = symtab[slot];
    const uint32_t fc = fctab[s];
    const uint32_t xn = (fc & 0xFFFFu) * (x >> ax::kProbBits) + slot - (fc >> 16);
    const bool need = act && xn < ax::kRansLow;
    const uint32_t xr = renorm(__ballot(need), xn, need);
    if (act) {
      x = xr;
      out[i] = uint8_t(s);
    }
  }
  bad |= lane < K && x != ax::kRansLow;
  bad |= ptr != nw;
  if (__ballot(bad)) {
    if (lane == 0) report(a.st, AX_E_CORRUPT, b);
  }
  if (lane == 0) *nsym = n;
}

// ---------------------------------------------------------------- k_parse --

struct ParseArgs {
  const JobDev* jobs;
  const WinBlock* wbl;
  uint32_t n_items;
  uint32_t n_tok;            // tokens in the window
  uint32_t slot_b;
  const uint8_t *lit, *cmd, *off, *len;
  uint32_t off_cap, len_cap;
  const uint32_t* nsym;
  uint64_t* tok;             // 2 u64 per token: src, dst | (len-1) << 48
  uint32_t* tblk;            // per token: its window block
  uint8_t* done;             // per token: kPending until the match layer copies it
  DevStatus* st;
  int write_out;             // 0: tokens only (the token-index build), no output bytes
  uint16_t* mcov;            // match coverage: per window position, set when a match writes it (16 per u16)
};

// History maps.  A command acts on the four-entry distance history as a map
// from the history before it to the history after it; a run of commands
// composes these maps.  Each of the four output slots names where its
// distance comes from: an input slot j, or the explicit match at chunk
// position c (its distance is cdist[c]).  A map is two words: the slot bytes
// (j or c) and the tag bytes (0xFF: the slot byte is an input slot, 0x00: a
// chunk position).  Composing two maps is a byte gather, two v_perm_b32.
struct HMap {
  uint32_t v, t;
};
constexpr HMap kMapId{0x03020100u, 0xFFFFFFFFu};

// (later g) after (earlier f): slot i takes f's slot j where g's slot i reads
// input j (selector byte j: f's bytes are the permute's low four), else keeps
// g's own slot i (selector byte 4 + i).
__device__ inline HMap map_after(HMap g, HMap f) {
  const uint32_t sel = (g.v & g.t) | (0x07060504u & ~g.t);
  return HMap{__builtin_amdgcn_perm(g.v, f.v, sel), __builtin_amdgcn_perm(g.t, f.t, sel)};
}
__device__ inline uint64_t pick4(const uint64_t h[4], uint64_t j) {
  return j == 0 ? h[0] : j == 1 ? h[1] : j == 2 ? h[2] : h[3];
}

struct ParseShared {
  __attribute__((aligned(16))) uint8_t tile[kMaxB];
  uint64_t runbits[kMaxB / 64];   // starts of the chunk's literal runs, in the block's output positions
  uint16_t runpre[kMaxB / 64];    // run starts in earlier words
  uint16_t rundelta[kParseThreads];  // per run: output position - literal index
  uint16_t runbeg[kParseThreads];    // per run: first output position
  uint16_t runend[kParseThreads];    // per run: one past its last output position
  uint8_t offb[kOffStage];        // the block's decoded offset stream, when it fits
  uint8_t lenb[kLenStage];        // the block's decoded length stream, when it fits
  uint64_t offval[kParseThreads];
  uint64_t wsum[4][2];
  HMap wmap[4];
  union {
    uint64_t cdist[kParseThreads];   // distance of the explicit match at each chunk position
    uint32_t lenval[kParseThreads];  // length extensions: read before cdist is written (a barrier apart)
  };
  uint64_t last4[4];              // the chunk's last explicit-match distances, newest first
  uint32_t wterm[4];
  int32_t wlast[4];
  uint32_t leb_found, leb_cursor;
  // coverage bits of the 16-byte group a chunk leaves open, by chunk parity
  // (a chunk reads its predecessor's while it may write its own)
  uint32_t mcarry[2];
  int bad;
  alignas(4) uint8_t anyb[2][4];  // block_any: one byte per wave, two call sites
};

// Block-wide "any thread's p" (256 threads): a ballot per wave, one LDS byte
// per wave, one barrier.  Slot k's bytes are rewritten only after a later
// barrier, so every thread has read them.
__device__ inline bool block_any(bool p, ParseShared& sh, int k) {
  const bool w = __ballot(p) != 0;
  if (lane_id() == 0) sh.anyb[k][threadIdx.x >> 6] = uint8_t(w);
  __syncthreads();
  return *reinterpret_cast<const uint32_t*>(sh.anyb[k]) != 0;
}

// Wave-level moves for the scans (DPP): row_shr:k moves each lane's value k
// lanes up inside its row of 16; row_bcast:15 / :31 hand lane 15 / 31 to the
// rows selected by the row mask.  Lanes without a source, or in unselected
// rows, receive `id`.
constexpr int kDppRowShr = 0x110, kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_move(uint32_t id, uint32_t x) {
  return uint32_t(__builtin_amdgcn_update_dpp(int(id), int(x), CTRL, ROWS, 0xF, false));
}

// Inclusive wave scan of a u32 (sum): 1, 2, 4, 8 inside the rows, then the
// row totals across rows.
__device__ inline uint32_t wave_incl_sum32(uint32_t x) {
  x += dpp_move<kDppRowShr + 1, 0xF>(0, x);
  x += dpp_move<kDppRowShr + 2, 0xF>(0, x);
  x += dpp_move<kDppRowShr + 4, 0xF>(0, x);
  x += dpp_move<kDppRowShr + 8, 0xF>(0, x);
  x += dpp_move<kDppRowBcast15, 0xA>(0, x);
  x += dpp_move<kDppRowBcast31, 0xC>(0, x);
  return x;
}

// Block-wide exclusive scan of a u64 holding two u32 sums (the halves are
// scanned separately: no half may carry), 256 threads.
__device__ inline uint64_t block_excl_sum64(uint64_t v, uint64_t* total, ParseShared& sh, int slotk) {
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  const uint64_t x = wave_incl_sum32(uint32_t(v)) | (uint64_t(wave_incl_sum32(uint32_t(v >> 32))) << 32);
  if (lane == 63) sh.wsum[wv][slotk] = x;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    const uint64_t t = sh.wsum[k][slotk];
    if (k < wv) pre += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

// Block-wide exclusive scan of history maps; returns the map before this
// command and the chunk's total map.
template <int CTRL, int ROWS>
__device__ inline HMap map_dpp(HMap m) {
  return HMap{dpp_move<CTRL, ROWS>(kMapId.v, m.v), dpp_move<CTRL, ROWS>(kMapId.t, m.t)};
}
__device__ inline HMap block_excl_map(HMap m, HMap* total, ParseShared& sh) {
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  HMap x = m;  // inclusive wave scan, earlier lanes' maps applied first (the identity fills gaps)
  x = map_after(x, map_dpp<kDppRowShr + 1, 0xF>(x));
  x = map_after(x, map_dpp<kDppRowShr + 2, 0xF>(x));
  x = map_after(x, map_dpp<kDppRowShr + 4, 0xF>(x));
  x = map_after(x, map_dpp<kDppRowShr + 8, 0xF>(x));
  x = map_after(x, map_dpp<kDppRowBcast15, 0xA>(x));
  x = map_after(x, map_dpp<kDppRowBcast31, 0xC>(x));
  if (lane == 63) sh.wmap[wv] = x;
  __syncthreads();
  HMap pre = kMapId, tot = kMapId;
  for (uint32_t k = 0; k < 4; ++k) {
    if (k < wv) pre = map_after(sh.wmap[k], pre);
    tot = map_after(sh.wmap[k], tot);
  }
  __syncthreads();
  *total = tot;
  return map_after(map_dpp<kDppWaveShr1, 0xF>(x), pre);  // inclusive of the previous lane
}

// Distance named by slot k of a map: an input slot of hist, or an explicit
// match of the chunk.
__device__ inline uint64_t map_value(HMap m, uint32_t k, const uint64_t hist[4], const ParseShared& sh) {
  const uint32_t g = (m.v >> (8 * k)) & 0xFFu;
  return ((m.t >> (8 * k)) & 1u) ? pick4(hist, g & 3) : sh.cdist[g];
}

// Decode `count` consecutive LEB128 values starting at byte *cursor of
// src[0..n) into dst (u64) — all 256 threads, BPT bytes each per window of
// 256 * BPT.  A byte below 0x80 ends a value; terminators are counted by a block
// scan, and each terminator's thread assembles its value from the bytes after
// the previous terminator.  Returns false on a malformed or missing value.
// *cursor advances past the last value.
template <uint32_t BPT, class Src>
__device__ bool leb_values(Src src, uint32_t n, uint32_t* cursor, uint32_t count, uint64_t* dst,
                           ParseShared& sh) {
  const uint32_t t = threadIdx.x, lane = lane_id(), wv = t >> 6;
  const uint32_t first = *cursor;
  uint32_t found = 0;
  uint32_t win = first & ~(BPT - 1);
  uint32_t value_start = first;  // start of the value that is open at the window start
  bool ok = true;
  while (found < count) {
    if (win >= n) { ok = false; break; }
    const uint32_t p0 = win + BPT * t;
    uint32_t tm = 0;  // terminators among this thread's bytes
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t pos = p0 + q;
      if (pos >= first && pos < n && src[pos] < 0x80) tm |= 1u << q;
    }
    const uint32_t c = __popc(tm);
    const uint32_t incl = wave_incl_sum32(c);
    const int32_t mylast = tm ? int32_t(p0 + 31 - __clz(tm)) : -1;
    const uint64_t hm = __ballot(tm != 0);
    if (lane == 63) sh.wterm[wv] = incl;
    if (hm == 0 ? lane == 0 : lane == uint32_t(63 - __clzll(hm))) sh.wlast[wv] = mylast;
    __syncthreads();
    uint32_t before = incl - c, all = 0;
    for (uint32_t k = 0; k < 4; ++k) {
      if (k < wv) before += sh.wterm[k];
      all += sh.wterm[k];
    }
    // the last terminator before this thread's bytes
    const uint64_t lower = hm & ((1ull << lane) - 1ull);
    const int32_t from_lane = __shfl(mylast, lower ? 63 - __clzll(lower) : 0, 64);
    int32_t prev = lower ? from_lane : -1;
    if (prev < 0)
      for (int32_t k = int32_t(wv) - 1; k >= 0; --k)
        if (sh.wlast[k] >= 0) { prev = sh.wlast[k]; break; }
    uint32_t vi = found + before;
    uint32_t start = prev >= 0 ? uint32_t(prev) + 1 : value_start;
    for (uint32_t q = 0; q < BPT; ++q) {
      if (!((tm >> q) & 1)) continue;
      const uint32_t pos = p0 + q;
      if (vi < count) {
        if (pos + 1 - start > 10) {
          ok = false;
        } else {
          uint64_t v = 0;
          for (uint32_t r = start; r <= pos; ++r) v |= uint64_t(src[r] & 0x7F) << (7 * (r - start));
          if (pos - start == 9 && src[pos] > 1) ok = false;
          dst[vi] = v;
          if (vi == count - 1) sh.leb_cursor = pos + 1;
        }
      }
      ++vi;
      start = pos + 1;
    }
    // the value still open at the end of this window starts after its last terminator
    int32_t last = -1;
    for (int32_t k = 3; k >= 0; --k)
      if (sh.wlast[k] >= 0) { last = sh.wlast[k]; break; }
    if (last >= 0) value_start = uint32_t(last) + 1;
    if (win + BPT * kParseThreads - value_start > 10 && found + all < count) ok = false;  // a value longer than 10 bytes
    found += all;
    win += BPT * kParseThreads;
    __syncthreads();
  }
  if (block_any(!ok, sh, 0)) return false;
  if (count) *cursor = sh.leb_cursor;
  __syncthreads();
  return true;
}

// Six waves per SIMD (at most 80 VGPRs), as many as the LDS allows.
template <class O, bool kCovMap>
__global__ __launch_bounds__(kParseThreads, 6) void k_parse(ParseArgs a) {
  __shared__ ParseShared sh;
  const uint32_t item = blockIdx.x, t = threadIdx.x;
  const WinBlock wb = a.wbl[item];
  const JobDev& J = a.jobs[wb.job];
  const uint64_t b = wb.b;
  const uint32_t B = J.B, mm = J.mm;
  const uint64_t bs = b * B;
  const uint32_t blen = uint32_t(min<uint64_t>(B, J.n_bytes - bs));
  const uint32_t n_lit = a.nsym[4 * item + 0], n_len = a.nsym[4 * item + 1];
  const uint32_t n_off = a.nsym[4 * item + 2], n_cmd = a.nsym[4 * item + 3];
  const uint8_t* cmd = a.cmd + uint64_t(item) * a.slot_b;
  const AX_GLOBAL uint8_t* const litg = gp(a.lit + uint64_t(item) * a.slot_b);
  const uint8_t* offs = a.off + uint64_t(item) * a.off_cap;
  const uint8_t* lens = a.len + uint64_t(item) * a.len_cap;
  const uint64_t* mpre = reinterpret_cast<const uint64_t*>(J.arc + 64) + J.nb + 1;
  const uint64_t tok_lo = wb.tok, tok_n = mpre[b + 1] - mpre[b];

  if (t == 0)
    sh.bad = (n_lit > B || n_cmd > B || n_len > job_len_cap(J) || n_off > job_off_cap(J) ||
              tok_lo + tok_n > a.n_tok) ? 1 : 0;
  // the first chunk's command bytes, loaded ahead of the staging barrier
  // (inside the slot whatever the count: kParseThreads <= slot_b)
  uint32_t cnext = cmd[t];
  // stage the offset and length streams in LDS: one 16-byte piece per
  // thread, loaded before the stream lengths are known (the slots are
  // 16-aligned and their capacities multiples of 16, so the loads stay in
  // this block's slots) and kept if the stream fits the stage
  static_assert(kOffStage <= 16 * kParseThreads && kLenStage <= 16 * kParseThreads, "one piece per thread");
  uint4 po = {0, 0, 0, 0}, pl = {0, 0, 0, 0};
  if (16 * t < min(kOffStage, a.off_cap)) po = *reinterpret_cast<const uint4*>(offs + 16 * t);
  if (16 * t < min(kLenStage, a.len_cap)) pl = *reinterpret_cast<const uint4*>(lens + 16 * t);
  if (n_off <= kOffStage && 16 * t < n_off) *reinterpret_cast<uint4*>(sh.offb + 16 * t) = po;
  if (n_len <= kLenStage && 16 * t < n_len) *reinterpret_cast<uint4*>(sh.lenb + 16 * t) = pl;
  __syncthreads();
  bool failed = sh.bad != 0;
  // the streams are read from LDS when staged, else from global memory (two
  // instantiations, so neither path goes through flat addressing)
  const bool off_lds = n_off <= kOffStage, len_lds = n_len <= kLenStage;
  const AX_GLOBAL uint8_t* const offg = gp(offs);
  const AX_GLOBAL uint8_t* const leng = gp(lens);

  uint32_t dst = 0, litp = 0, offc = 0, lenc = 0;
  uint64_t ntok = 0;
  uint64_t hist[4] = {1, 2, 3, 4};
  for (uint32_t c0 = 0; c0 < n_cmd && !failed; c0 += kParseThreads) {
    const uint32_t i = c0 + t;
    const bool valid = i < n_cmd;
    const uint32_t c = valid ? cnext : 0u;
    cnext = i + kParseThreads < n_cmd ? cmd[i + kParseThreads] : 0u;  // the next chunk's, in flight meanwhile
    const uint32_t kind = c & 3;
    bool bad = valid && kind == 3;
    const uint32_t v = kind == 2 ? (c >> 4) : (c >> 2);
    const bool esc = valid && !bad && v == (kind == 2 ? 15u : 63u);
    const bool is0 = valid && kind == 0, is1 = valid && kind == 1, is2 = valid && kind == 2;
    const uint64_t packed = uint64_t(esc) | (uint64_t(is1) << 16) | (uint64_t(is0) << 32) | (uint64_t(is1 || is2) << 48);
    uint64_t ctot;
    const uint64_t cex = block_excl_sum64(packed, &ctot, sh, 0);
    const uint32_t esc_i = uint32_t(cex & 0xFFFF), k1_i = uint32_t((cex >> 16) & 0xFFFF);
    const uint32_t run_i = uint32_t((cex >> 32) & 0xFFFF), tok_i = uint32_t(cex >> 48);
    const uint32_t n_esc = uint32_t(ctot & 0xFFFF), n_k1 = uint32_t((ctot >> 16) & 0xFFFF);
    const uint32_t n_tokc = uint32_t(ctot >> 48);
    // length and offset values of this chunk
    uint64_t* lv64 = sh.offval;  // reuse: lengths first, then offsets
    if (n_esc) {  // most chunks hold no escaped length (n_esc is the same for the whole block)
      if (!(len_lds ? leb_values<kLenBpt>(static_cast<const uint8_t*>(sh.lenb), n_len, &lenc, n_esc, lv64, sh)
                    : leb_values<kLenBpt>(leng, n_len, &lenc, n_esc, lv64, sh))) {
        failed = true;
        break;
      }
      if (t < n_esc) {
        const uint64_t e = lv64[t];
        sh.lenval[t] = e > B ? 0xFFFFFFFFu : uint32_t(e);
      }
      __syncthreads();
    }
    if (!(off_lds ? leb_values<kOffBpt>(static_cast<const uint8_t*>(sh.offb), n_off, &offc, n_k1, sh.offval, sh)
                  : leb_values<kOffBpt>(offg, n_off, &offc, n_k1, sh.offval, sh))) {
      failed = true;
      break;
    }
    uint32_t len = 0;
    if (valid) {
      const uint32_t ext = esc ? sh.lenval[esc_i] : 0u;
      bad |= ext == 0xFFFFFFFFu;
      len = bad ? 0 : v + (kind == 0 ? 1u : mm) + ext;
    }
    const uint64_t lp = uint64_t(len) | (uint64_t(is0 ? len : 0u) << 32);
    uint64_t ptot;
    const uint64_t pex = block_excl_sum64(lp, &ptot, sh, 1);
    const uint32_t cdst = dst + uint32_t(pex & 0xFFFFFFFFu), clit = litp + uint32_t(pex >> 32);
    const uint32_t chunk_lit = uint32_t(ptot >> 32);
    if (valid && uint64_t(cdst) + len > blen) bad = true;
    if (is0 && uint64_t(clit) + len > n_lit) bad = true;
    const uint64_t absdst = bs + cdst;
    uint64_t src = 0;
    if (is1) {
      src = sh.offval[k1_i];
      if (src >= absdst) bad = true;
      else sh.cdist[t] = absdst - src;
    }
    const uint32_t n_rep = n_tokc - n_k1;
    uint64_t nh[4];
    if (n_rep) {  // repeat matches read the history: scan the command maps
      HMap mine = kMapId;
      if (is1) {
        mine = HMap{t | 0x02010000u, 0xFFFFFF00u};
      } else if (is2) {
        const uint32_t r = (c >> 2) & 3;
        mine = HMap{r | ((r >= 1 ? 0u : 1u) << 8) | ((r >= 2 ? 1u : 2u) << 16) | ((r >= 3 ? 2u : 3u) << 24),
                    0xFFFFFFFFu};
      }
      HMap mtot;
      const HMap before = block_excl_map(mine, &mtot, sh);  // also orders the cdist writes
      if (is2) {
        const uint64_t d = map_value(before, (c >> 2) & 3, hist, sh);
        if (d > absdst) bad = true;
        else src = absdst - d;
      }
      for (uint32_t k = 0; k < 4; ++k) nh[k] = map_value(mtot, k, hist, sh);
    } else {  // explicit matches only: the history takes their last distances
      if (is1 && !bad && k1_i + 4 >= n_k1) sh.last4[n_k1 - 1 - k1_i] = absdst - src;
      __syncthreads();
      const uint32_t m4 = min(n_k1, 4u);
      for (uint32_t k = 0; k < 4; ++k) nh[k] = k < m4 ? sh.last4[k] : pick4(hist, k - m4);
    }
    if ((is1 || is2) && !bad) {
      const uint64_t gi = ntok + tok_i;
      if (gi < tok_n) {
        uint64_t* tk = a.tok + 2 * (tok_lo + gi);
        tk[0] = src;
        tk[1] = absdst | (uint64_t(len - 1) << 48);
        a.tblk[tok_lo + gi] = item;
        a.done[tok_lo + gi] = kPending;
      } else {
        bad = true;
      }
    }
    // literal runs: starts in the block's output positions
    for (uint32_t w = t; w < B / 64; w += kParseThreads) sh.runbits[w] = 0;
    __syncthreads();
    if (is0 && !bad && len) {
      atomicOr(reinterpret_cast<uint32_t*>(sh.runbits) + (cdst >> 5), 1u << (cdst & 31));
      sh.rundelta[run_i] = uint16_t(cdst - clit);
      sh.runbeg[run_i] = uint16_t(cdst);
      sh.runend[run_i] = uint16_t(cdst + len);
    }
    if (block_any(bad, sh, 1)) { failed = true; break; }
    const uint32_t n_runs = uint32_t((ctot >> 32) & 0xFFFF);
    {  // run starts before each word of the output positions (B / 64 <= 256 words)
      const uint32_t c = t < B / 64 ? __popcll(sh.runbits[t]) : 0;
      uint64_t rt;
      const uint64_t pre = block_excl_sum64(c, &rt, sh, 0);
      if (t < B / 64) sh.runpre[t] = uint16_t(pre);
    }
    __syncthreads();
    // place the chunk's literal bytes by aligned 16-byte output groups: each
    // literal run meeting a group supplies the 16 literal bytes lined up with
    // the group under the group's byte mask, and the group is merged into the
    // tile with one 16-byte read and write (bytes outside the runs keep their
    // value)
    const uint32_t dend = dst + uint32_t(ptot & 0xFFFFFFFFu);
    for (uint32_t c = (dst >> 4) + t; 16 * c < dend; c += kParseThreads) {
      const uint32_t d0 = max(16 * c, dst), d1 = min(16 * c + 16, dend), w = d0 >> 6;
      int32_t r = int32_t(sh.runpre[w] + __popcll(sh.runbits[w] & (~0ull >> (63 - (d0 & 63))))) - 1;
      if (r < 0 || d0 >= sh.runend[r]) ++r;  // the run holding d0, else the next one
      u32x4 val = {0, 0, 0, 0}, msk = {0, 0, 0, 0};
      uint32_t lit16 = 0;  // the group's literal bytes in this chunk
      for (; r < int32_t(n_runs) && sh.runbeg[r] < d1; ++r) {
        const uint32_t x0 = max(d0, uint32_t(sh.runbeg[r])), x1 = min(d1, uint32_t(sh.runend[r]));
        const int32_t l0 = int32_t(16 * c) - int32_t(sh.rundelta[r]);  // literal index of the group's byte 0
        // the 16 literal bytes lined up with the group: one unaligned load
        // (l0 may be as low as -15, and the load may run past the stream:
        // still inside the workspace)
        const u32x4 e = *reinterpret_cast<const AX_GLOBAL u32x4_u*>(litg + l0);
        const uint32_t m16 = ((1u << (x1 - 16 * c)) - 1u) & ~((1u << (x0 - 16 * c)) - 1u);
        // byte i of the group's mask is 0xFF when bit i of m16 is set: each
        // nibble spread to one bit per byte, then a byte permute whose
        // selector 12 gives 0x00 and 13 gives 0xFF (no 32-bit multiply)
        const u32x4 nib = {m16 & 15u, (m16 >> 4) & 15u, (m16 >> 8) & 15u, (m16 >> 12) & 15u};
        const u32x4 sel = ((nib * 0x00204081u) & 0x01010101u) | 0x0C0C0C0Cu;
        const u32x4 bm = {__builtin_amdgcn_perm(0u, 0u, sel.x), __builtin_amdgcn_perm(0u, 0u, sel.y),
                          __builtin_amdgcn_perm(0u, 0u, sel.z), __builtin_amdgcn_perm(0u, 0u, sel.w)};
        val = (val & ~bm) | (e & bm);
        msk |= bm;
        lit16 |= m16;
        if (sh.runend[r] >= d1) break;
      }
      if (kCovMap) {  // match coverage of the group: its bytes in this chunk that no literal fills
        uint32_t m = ((1u << (d1 - 16 * c)) - 1u) & ~((1u << (d0 - 16 * c)) - 1u) & ~lit16;
        const uint32_t par = (c0 / kParseThreads) & 1;
        if (d0 > 16 * c) m |= sh.mcarry[par ^ 1];  // the group began in the previous chunk
        if (d1 < 16 * c + 16 && d1 < blen) sh.mcarry[par] = m;  // it goes on in the next chunk
        else a.mcov[uint64_t(item) * (a.slot_b / 16) + c] = uint16_t(m);
      }
      if (msk.x | msk.y | msk.z | msk.w) {
        u32x4& cell = *reinterpret_cast<u32x4*>(sh.tile + 16 * c);
        cell = (cell & ~msk) | val;
      }
    }
    __syncthreads();
    dst += uint32_t(ptot & 0xFFFFFFFFu);
    litp += chunk_lit;
    ntok += n_tokc;
    for (int k = 0; k < 4; ++k) hist[k] = nh[k];
  }
  if (!failed && (dst != blen || litp != n_lit || lenc != n_len || offc != n_off || ntok != tok_n)) failed = true;
  if (failed) {
    if (t == 0) report(a.st, AX_E_CORRUPT, b);
    return;
  }
  if (!a.write_out) return;
  // write the tile with 16-byte stores (match bytes are filled by the match layer)
  AX_GLOBAL uint8_t* o = O(J).at(bs);  // the block's bytes are contiguous
  const uint32_t full = blen & ~15u;
  for (uint32_t k = 16 * t; k < full; k += 16 * kParseThreads)
    *reinterpret_cast<AX_GLOBAL u32x4*>(o + k) = *reinterpret_cast<const u32x4*>(sh.tile + k);
  for (uint32_t k = full + t; k < blen; k += kParseThreads) o[k] = sh.tile[k];
}

// ------------------------------------------------------------ match layer --

struct CopyArgs {
  const JobDev* jobs;
  const WinBlock* wbl;
  uint32_t n_items;
  const uint64_t* tok;       // window tokens in (job, output) order
  const uint32_t* tblk;      // per token: its window block
  uint32_t n_tok;
  uint32_t* cov;             // per token: first covering token, count
  uint8_t* done;             // per token: round that copied it, or kPending
  const uint32_t* list_in;   // pending tokens of the previous round: kSub sublists of sub_cap
  uint32_t* list_out;
  const uint32_t* cnt_in;    // kSub counters, kCounterStride apart
  uint32_t* cnt_out;
  uint32_t* cnt_clear;       // the counters the next round writes
  uint32_t sub_cap;
  uint32_t* long_list;       // round 0: ready tokens of at least kSplitToken bytes
  uint32_t* long_cnt;
  uint32_t round;
  DevStatus* st;
  uint32_t* pbits;           // the last round's leftovers, one bit per token
  const uint32_t* plist;     // the same tokens, ascending (the persistent finish's work)
  int mark;                  // this round is the last: 0 no, else kMarkList or kMarkJump
  uint64_t spin_limit;
  int serial;
  int fill_round, fill_tail;  // later rounds / persistent launch: kFillLaneWave or kFillSegmented
  uint32_t tail_chunks;       // consecutive 64-token chunks per persistent-launch ticket
  uint32_t* J;                // pointer jumping: one entry per window position
  uint64_t* lmap;             // pointer jumping: leftover map
  uint32_t S;                 // position stride of a window block
  const uint64_t* mcov;       // match coverage of the window positions (the parse writes it when round 0
                              // is the only bulk round; null: round 0 finds every cover)
  uint32_t one_job;           // 1: the plan has one job, so every token's output is jobs[0]'s
};

__device__ inline void token_at(const uint64_t* tok, uint64_t t, uint64_t& src, uint64_t& dst, uint32_t& len) {
  src = tok[2 * t];
  const uint64_t w = tok[2 * t + 1];
  dst = w & ((1ull << 48) - 1);
  len = uint32_t(w >> 48) + 1;
}

// Tokens [lo, lo+cnt) are those whose destinations meet [s0, s1) of the
// job of window block wb.  Tokens are disjoint and sorted by destination
// within a job, and a job's window blocks are contiguous and ascending, so
// the search runs over the job's window blocks, then inside the block that
// holds s0.  Source bytes outside every window block of the job were
// written by an earlier window or are not decoded by this plan (a range
// decode reads only bytes whose blocks it holds), so nothing waits on them.
__device__ inline void find_cover(const CopyArgs& a, const WinBlock& wb, uint32_t B, uint64_t s0, uint64_t s1,
                                  uint32_t& lo, uint32_t& cnt) {
  const uint64_t sb = s0 / B;
  const uint32_t job_end = wb.first + wb.count;
  uint32_t x = wb.first, y = job_end;
  const uint64_t b0 = a.wbl[wb.first].b;
  if (sb >= b0 && sb - b0 < wb.count && a.wbl[wb.first + uint32_t(sb - b0)].b == sb) {
    x = wb.first + uint32_t(sb - b0);  // the job's blocks are consecutive up to sb (whole-archive windows)
  } else {
    while (x < y) {  // first window block of the job with b >= sb
      const uint32_t mid = (x + y) >> 1;
      if (a.wbl[mid].b < sb) x = mid + 1; else y = mid;
    }
  }
  const uint32_t end_tok = job_end < a.n_items ? a.wbl[job_end].tok : a.n_tok;
  uint32_t p = x < job_end ? a.wbl[x].tok : end_tok;
  if (x < job_end && a.wbl[x].b == sb) {  // first token of block x ending after s0
    uint32_t q = x + 1 < a.n_items ? a.wbl[x + 1].tok : a.n_tok;
    while (p < q) {
      const uint32_t mid = (p + q) >> 1;
      const uint64_t w = a.tok[2 * uint64_t(mid) + 1];
      if ((w & ((1ull << 48) - 1)) + (w >> 48) + 1 <= s0) p = mid + 1; else q = mid;
    }
  }
  lo = p;
  cnt = 0;
  while (p + cnt < end_tok && (a.tok[2 * uint64_t(p + cnt) + 1] & ((1ull << 48) - 1)) < s1) ++cnt;
}

// Round 0 leaves the cover of its pending tokens to the round that first
// needs it (the covers of its ready tokens are never needed).
constexpr uint32_t kCovLazy = 0xFFFFFFFFu;
__device__ inline void cover_of(const CopyArgs& a, uint32_t t, uint64_t src, uint64_t dst, uint32_t len,
                                uint32_t& lo, uint32_t& cnt) {
  lo = a.cov[2 * t];
  cnt = a.cov[2 * t + 1];
  if (cnt != kCovLazy) return;
  const WinBlock wb = a.wbl[a.tblk[t]];
  const uint64_t dist = dst - src;
  find_cover(a, wb, a.jobs[wb.job].B, src, src + (dist < len ? dist : len), lo, cnt);
  a.cov[2 * t] = lo;
  a.cov[2 * t + 1] = cnt;
}

// The output of token t's archive.
template <class O>
__device__ inline O token_out(const CopyArgs& a, uint32_t t) { return O(a.jobs[a.wbl[a.tblk[t]].job]); }

template <bool COH>
__device__ inline uint8_t ldb(const AX_GLOBAL uint8_t* p) {
  if constexpr (COH) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else return *p;
}
template <bool COH>
__device__ inline void stb(gbytes p, uint8_t v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// The serial ablation: one lane, byte after byte, reading the bytes it may
// itself have just written (a self-overlapping match is a dependency chain).
template <bool COH, class O>
__device__ inline void fill_serial(const O& out, uint64_t dst, uint64_t src, uint32_t len) {
  for (uint32_t k = 0; k < len; ++k) {
    stb<COH>(out.at(dst + k), ldb<COH>(out.at(src + k)));
    __builtin_amdgcn_s_waitcnt(0x0F70);  // the next load may read this byte
  }
}

// One lane fills a token as a periodic fill: sixteen source loads in flight,
// then sixteen stores.  The source index runs over the period dist (for
// dist >= len it never wraps and the fill is a plain copy).
template <bool COH, class O>
__device__ inline void fill_lane(const O& out, uint64_t dst, uint64_t src, uint32_t len) {
  const uint64_t dist = dst - src;
  uint64_t j = 0;
  for (uint32_t k0 = 0; k0 < len; k0 += 16) {
    uint64_t idx[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      idx[q] = j;
      if (++j == dist) j = 0;
    }
    uint8_t v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = (k0 + q < len) ? ldb<COH>(out.at(src + idx[q])) : uint8_t(0);
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (k0 + q < len) stb<COH>(out.at(dst + k0 + q), v[q]);
  }
}

// The whole wave fills one long token: eight bytes per lane in flight.
template <bool COH, class O>
__device__ inline void fill_wave(const O& out, uint64_t dst, uint64_t src, uint32_t len, uint32_t lane) {
  const uint64_t dist = dst - src;
  const uint64_t step = dist > 64 ? 64 : 64 % uint32_t(dist);  // no 64-bit division
  uint64_t j = dist > lane ? lane : lane % uint32_t(dist);
  for (uint32_t k0 = lane; k0 < len; k0 += 512) {
    uint64_t idx[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      idx[q] = j;
      j += step;
      if (j >= dist) j -= dist;
    }
    uint8_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (k0 + 64 * q < len) ? ldb<COH>(out.at(src + idx[q])) : uint8_t(0);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (k0 + 64 * q < len) stb<COH>(out.at(dst + k0 + 64 * q), v[q]);
  }
}

constexpr uint32_t kLongToken = 64;     // lane/wave fill: tokens at least this long use the whole wave
constexpr uint32_t kSplitToken = 1024;  // round 0: tokens at least this long get a workgroup each

// Per-wave staging of the ready tokens for the segmented fill.
struct FillStage {
  uint32_t end[64];   // inclusive prefix of lengths (0 for tokens not copied)
  uint32_t len[64];
  uint64_t dst[64];
  uint64_t src[64];
  gbytes out[64];
};

constexpr uint32_t kFillBytes = 8;  // consecutive bytes per lane per pass
enum { kFillLaneWave = 0, kFillSegmented = 1 };

// Segmented periodic fill of this wave's ready tokens: their bytes are laid
// end to end and every lane takes kFillBytes consecutive ones per pass, so a
// pass issues 64 * kFillBytes independent source loads before its stores,
// whatever the mix of short and long tokens.  Byte k of a token comes from
// src + (k mod dist) (dist >= len: a plain copy).
template <bool COH, class O>
__device__ inline void fill_ready(const O& out, bool ready, uint64_t dst, uint64_t src, uint32_t len, int serial,
                                  int fill_mode, FillStage& fs) {
  const uint32_t lane = lane_id();
  if (serial) {
    if (ready) fill_serial<COH>(out, dst, src, len);
    return;
  }
  if (fill_mode == kFillLaneWave) {  // short tokens lane by lane, long ones by the whole wave
    const bool lng = ready && len >= kLongToken;
    if (ready && !lng) fill_lane<COH>(out, dst, src, len);
    uint64_t lm = __ballot(lng);
    while (lm) {
      const int l = __builtin_ctzll(lm);
      lm &= lm - 1;
      const O o = out.with_base(
          reinterpret_cast<gbytes>(__shfl((unsigned long long)reinterpret_cast<uintptr_t>(out.base), l, 64)));
      fill_wave<COH>(o, __shfl((unsigned long long)dst, l, 64), __shfl((unsigned long long)src, l, 64),
                     __shfl(len, l, 64), lane);
    }
    return;
  }
  const uint32_t mine = ready ? len : 0u;
  uint32_t total;
  const uint32_t excl = wave_excl_sum(mine, &total);
  fs.end[lane] = excl + mine;
  fs.len[lane] = mine;
  fs.dst[lane] = dst;
  fs.src[lane] = src;
  fs.out[lane] = out.base;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (uint32_t base = 0; base < total; base += 64 * kFillBytes) {
    const uint32_t f0 = base + lane * kFillBytes;
    uint64_t at[kFillBytes];
    uint64_t to[kFillBytes];
    uint8_t v[kFillBytes];
    if (f0 < total) {
      uint32_t l = 0;  // first token whose end exceeds f0
#pragma unroll
      for (uint32_t step = 32; step; step >>= 1)
        if (fs.end[l + step - 1] <= f0) l += step;
      uint32_t e = fs.end[l], start = e - fs.len[l];
      uint64_t d = fs.dst[l], sr = fs.src[l], dist = d - sr;
      O o = out.with_base(fs.out[l]);
      uint64_t k = f0 - start;  // < 2^16: a token lies inside one block
      uint64_t j = dist > k ? k : uint64_t(uint32_t(k) % uint32_t(dist));
#pragma unroll
      for (uint32_t q = 0; q < kFillBytes; ++q) {
        const uint32_t f = f0 + q;
        if (f < total && f >= e) {  // next token with bytes
          do { ++l; } while (fs.len[l] == 0);
          e = fs.end[l];
          start = e - fs.len[l];
          d = fs.dst[l], sr = fs.src[l], dist = d - sr;
          o = out.with_base(fs.out[l]);
          k = 0, j = 0;
        }
        at[q] = reinterpret_cast<uint64_t>(o.at(sr + j));
        to[q] = f < total ? reinterpret_cast<uint64_t>(o.at(d + k)) : ~0ull;
        ++k;
        if (++j == dist) j = 0;
      }
#pragma unroll
      for (uint32_t q = 0; q < kFillBytes; ++q)
        v[q] = to[q] != ~0ull ? ldb<COH>(reinterpret_cast<const AX_GLOBAL uint8_t*>(at[q])) : uint8_t(0);
#pragma unroll
      for (uint32_t q = 0; q < kFillBytes; ++q)
        if (to[q] != ~0ull) stb<COH>(reinterpret_cast<gbytes>(to[q]), v[q]);
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Workgroup g of a grid of n is dispatched to XCD g mod 8 (round-robin);
// this gives every XCD a contiguous run of items instead, so neighbouring
// blocks share an L2 (a block's match sources are mostly just behind it).
__device__ inline uint32_t xcd_item(uint32_t g, uint32_t n) {
  const uint32_t x = g & 7u, slot = g >> 3, q = n >> 3, r = n & 7u;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}

// ------------------------------------------------ marking for pointer jumping --
//
// In the last bulk round, the tokens still pending (the deep remainder) are
// marked for pointer jumping (see the jump kernels below): every byte of a
// pending token gets its first entry in the jump array — its source position
// src + (k mod dist) by window position (byte o of window block x is
// x * S + o), or the source's value when the source's block is not in the
// window (the byte is final) — and its bit in the leftover map.  A wave lays
// its lanes' pending tokens end to end and takes eight bytes per lane.
constexpr uint32_t kJRes = 0x80000000u;  // entry holds a final byte value (low 8 bits)
constexpr uint32_t kJMarkBytes = 8;
constexpr uint32_t kJLongMark = 256;     // pending tokens at least this long are marked by a workgroup each

struct MarkStage {
  uint32_t end[64];  // inclusive prefix of pending lengths
  uint32_t item[64];
  uint64_t src[64], dst[64];
};

// Window position of the first byte of archive block qb of the job of
// window block wb, or false when that block is not in this window (its bytes
// are final: an earlier window wrote them, or the plan does not decode
// them).
__device__ inline bool window_block(const WinBlock* wbl, uint32_t S, const WinBlock& wb, uint64_t qb, uint32_t& wq) {
  const uint64_t b0 = wbl[wb.first].b;
  uint32_t x;
  if (qb >= b0 && qb - b0 < wb.count && wbl[wb.first + uint32_t(qb - b0)].b == qb) {
    x = wb.first + uint32_t(qb - b0);  // the job's blocks are consecutive up to qb (whole-archive windows)
  } else {
    uint32_t lo = wb.first, hi = wb.first + wb.count;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (wbl[mid].b < qb) lo = mid + 1; else hi = mid;
    }
    if (lo == wb.first + wb.count || wbl[lo].b != qb) return false;
    x = lo;
  }
  wq = x * S;
  return true;
}

// Whether no match of this window writes a byte of [s0, s1) of the job of
// window block wb (block `item`, whose bytes start at archive position bs):
// those bytes are literals or final, so a token reading them is ready in
// round 0.  Read from the match coverage the parse wrote; bytes of blocks
// outside the window are final or not needed (as for find_cover).
__device__ inline bool sources_literal(const CopyArgs& a, const WinBlock& wb, uint32_t item, uint64_t bs, uint32_t B,
                                       uint64_t s0, uint64_t s1) {
  const uint32_t lb = __builtin_ctz(B);
  const AX_GLOBAL uint64_t* const mc = gp(a.mcov);
  while (s0 < s1) {
    const uint64_t qb = s0 >> lb, e = min(s1, (qb + 1) << lb);
    uint32_t wq = item * a.S;
    if (qb == (bs >> lb) || window_block(a.wbl, a.S, wb, qb, wq)) {
      const uint32_t p0 = wq + uint32_t(s0 & (B - 1)), p1 = p0 + uint32_t(e - s0);  // window positions
      for (uint32_t w = p0 >> 6; w <= (p1 - 1) >> 6; ++w) {
        const uint32_t lo = w == (p0 >> 6) ? (p0 & 63) : 0, hi = w == ((p1 - 1) >> 6) ? ((p1 - 1) & 63) : 63;
        const uint64_t m = (~0ull >> (63 - hi)) & (~0ull << lo);
        if (mc[w] & m) return false;
      }
    }
    s0 = e;
  }
  return true;
}

// Mark this wave's pending tokens (one per lane: `pend`, token t).  `row`:
// when not null, every token lies in window block `row_item` and its bits go
// to that block's LDS row (32-bit words); else to the leftover map with
// global atomics.
template <class O>
__device__ void mark_wave(const CopyArgs& a, bool pend, uint32_t t, MarkStage& ms, uint32_t* row,
                          uint32_t row_item) {
  const uint32_t lane = lane_id();
  uint64_t src = 0, dst = 0;
  uint32_t len = 0;
  if (pend) token_at(a.tok, t, src, dst, len);
  // long tokens of a round over the leftover list are marked by a wave each
  // (k_jmarklong): one wave laying out several would hold up the whole
  // launch (a round-0 workgroup marks at most its own block).  They go to the round's
  // output sublists, which the last round does not otherwise use: token t to
  // sublist (t / 64) mod kSub, so a sublist holds at most ceil(T / 64 / kSub)
  // * 64 of them, and its counter is one of kSub addresses 256 B apart
  const bool lng = pend && len >= kJLongMark && !row;  // a block's own row bounds its work
  if (lng) {
    const uint32_t sub = (t >> 6) % kSub;
    const uint32_t at = atomicAdd(a.cnt_out + sub * kCounterStride, 1u);
    a.list_out[uint64_t(sub) * a.sub_cap + at] = t;
  }
  if (!pend || lng) len = 0;
  uint32_t total;
  const uint32_t ex = wave_excl_sum(len, &total);
  if (!total) return;
  ms.end[lane] = ex + len;
  ms.item[lane] = pend ? a.tblk[t] : 0u;
  ms.src[lane] = src;
  ms.dst[lane] = dst;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  AX_GLOBAL uint32_t* const J = gp(a.J);
  uint32_t* const lm32 = reinterpret_cast<uint32_t*>(a.lmap);
  for (uint32_t f0 = lane * kJMarkBytes; f0 < total; f0 += 64 * kJMarkBytes) {
    uint32_t l = 0;  // first token whose prefix end exceeds f0
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
      if (ms.end[l + step - 1] <= f0) l += step;
    uint32_t e = ms.end[l], item = ms.item[l];
    WinBlock wb = a.wbl[item];
    JobDev jd = a.jobs[wb.job];
    uint64_t bs = wb.b * jd.B;
    uint32_t lb = __builtin_ctz(jd.B);  // block sizes are powers of two
    src = ms.src[l], dst = ms.dst[l];
    uint32_t k = f0 - (l ? ms.end[l - 1] : 0u);
    uint64_t dist = dst - src, j = dist > k ? k : uint64_t(k % uint32_t(dist));
    // window position of the source block last looked up (sources of a run
    // of bytes are consecutive: one lookup per block)
    uint64_t cb = wb.b;
    uint32_t cbase = item * a.S;
    bool cin = true;
    uint32_t mw = ~0u, mbits = 0;  // leftover-map word being gathered and its bits
    for (uint32_t q = 0; q < kJMarkBytes && f0 + q < total; ++q) {
      if (f0 + q >= e) {  // the next pending token
        do { ++l; } while (ms.end[l] == e);
        e = ms.end[l];
        src = ms.src[l], dst = ms.dst[l];
        if (ms.item[l] != item) {
          item = ms.item[l];
          wb = a.wbl[item];
          jd = a.jobs[wb.job];
          bs = wb.b * jd.B;
          lb = __builtin_ctz(jd.B);
        }
        k = 0, j = 0, dist = dst - src;
        cb = wb.b, cbase = item * a.S, cin = true;
      }
      const uint64_t sp = src + j;  // source position
      const uint64_t sb = sp >> lb;
      if (sb != cb) {
        cb = sb;
        cin = window_block(a.wbl, a.S, wb, sb, cbase);
      }
      const uint32_t v = cin ? cbase + uint32_t(sp & (jd.B - 1)) : kJRes | *O(jd).at(sp);
      const uint32_t d = item * a.S + uint32_t(dst - bs) + k;  // this byte's window position
      J[d] = v;
      if ((d >> 5) != mw) {
        if (mbits) {
          if (row) atomicOr(&row[mw - row_item * (a.S / 32)], mbits);
          else atomicOr(&lm32[mw], mbits);
        }
        mw = d >> 5, mbits = 0;
      }
      mbits |= 1u << (d & 31);
      ++k;
      if (++j == dist) j = 0;
    }
    if (mbits) {
      if (row) atomicOr(&row[mw - row_item * (a.S / 32)], mbits);
      else atomicOr(&lm32[mw], mbits);
    }
  }
  __builtin_amdgcn_wave_barrier();  // the stage is read before the caller's next use
}

// Level-synchronous rounds.  A token copied in round r marks done = r; a
// token is ready in round r only if its covering tokens are marked < r, i.e.
// were copied by an earlier launch, so no access within a round races.
//
// Round 0 runs one workgroup per window block, in four passes.  (1) Each
// token's covering range is found; ready tokens (sources all literal bytes,
// or before the window) are noted in LDS with the 16-byte chunks of the block
// they will write, leftovers go to the next round's lists.  (2) Those chunks
// of the block's output (the literals the parse placed) are loaded into an
// LDS tile.  (3) The ready tokens are filled into the tile, sources read from
// global memory where they are final.  (4) The chunks are written back with
// 16-byte stores: the match bytes reach memory as whole chunks instead of
// byte-granular scattered writes, and chunks without match bytes are neither
// read nor written.  Tokens of at least kSplitToken bytes go to k_long.
// Leftovers go to sublist (t / 64) mod kSub, so a sublist holds at most
// ceil(T / 64 / kSub) * 64 tokens.
template <class O, bool kCovMap>
__global__ __launch_bounds__(kCopyThreads) void k_round0(CopyArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t tile[kMaxB];
  __shared__ uint32_t dirty[kMaxB / 16 / 32];  // chunks of the tile that receive match bytes
  __shared__ uint32_t rdy[kMaxB / 32];         // the block's tokens filled here (min_match >= 1)
  // the block's tokens left pending, marked for jumping when round 0 is the
  // only round (the coverage-map instantiation; the other one keeps its LDS
  // for one more resident workgroup)
  __shared__ uint32_t lft[kCovMap ? kMaxB / 32 : 1];
  const uint32_t lane = lane_id(), item = xcd_item(blockIdx.x, gridDim.x);
  const WinBlock wb = a.wbl[item];
  const JobDev& J = a.jobs[wb.job];
  const O out(J);
  const uint32_t B = J.B;
  const uint64_t bs = wb.b * B;
  const gbytes ob = out.at(bs);  // this block's bytes (contiguous)
  const uint32_t blen = uint32_t(min<uint64_t>(B, J.n_bytes - bs));
  const uint32_t nchunk = (blen + 15) / 16;
  const uint32_t t1 = item + 1 < a.n_items ? a.wbl[item + 1].tok : a.n_tok;
  const uint32_t ntb = t1 - wb.tok;  // <= blen: tokens are at least a byte long
  // the status is checked once the block's own loads are in flight
  if (__hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  if (blockIdx.x == 0 && threadIdx.x < kSub) a.cnt_clear[threadIdx.x * kCounterStride] = 0;
  // the serial ablation reads in-block sources back from the tile: load all of it
  for (uint32_t k = threadIdx.x; k < kMaxB / 16 / 32; k += kCopyThreads) dirty[k] = a.serial ? ~0u : 0u;
  for (uint32_t k = threadIdx.x; k < (ntb + 31) / 32; k += kCopyThreads) {
    rdy[k] = 0;
    if (kCovMap) lft[k] = 0;
  }
  __syncthreads();
  for (uint32_t base = wb.tok; base < t1; base += kCopyThreads) {
    const uint32_t t = base + threadIdx.x;
    const bool act = t < t1;
    uint64_t src = 0, dst = 0;
    uint32_t len = 0;
    bool ready = false;
    if (act) {
      token_at(a.tok, t, src, dst, len);
      const uint64_t dist = dst - src, s1 = src + (dist < len ? dist : len);
      if (kCovMap) {  // the only round: readiness from the coverage map, covers when first needed
        ready = sources_literal(a, wb, item, bs, B, src, s1);
        if (!ready) a.cov[2 * t + 1] = kCovLazy;
      } else {
        uint32_t lo, cnt;
        find_cover(a, wb, B, src, s1, lo, cnt);
        a.cov[2 * t] = lo;
        a.cov[2 * t + 1] = cnt;
        ready = cnt == 0;
      }
    }
    const bool split = ready && !a.serial && len >= kSplitToken;
    const uint64_t sm = __ballot(split);
    if (sm) {
      uint32_t at = 0;
      if (lane == 0) at = atomicAdd(a.long_cnt, uint32_t(__popcll(sm)));
      at = __shfl(at, 0, 64);
      if (split) a.long_list[at + lanes_below(sm)] = t;
    }
    if (ready && !split) {
      a.done[t] = 0;
      const uint32_t r = t - wb.tok, drel = uint32_t(dst - bs);
      atomicOr(&rdy[r >> 5], 1u << (r & 31));
      const uint32_t c0 = drel >> 4, c1 = (drel + len - 1) >> 4;  // len < kSplitToken: a few words
      for (uint32_t w = c0 >> 5; w <= c1 >> 5; ++w) {
        const uint32_t lo_b = w == (c0 >> 5) ? (c0 & 31) : 0, hi_b = w == (c1 >> 5) ? (c1 & 31) : 31;
        atomicOr(&dirty[w], (hi_b == 31 ? ~0u : (2u << hi_b) - 1) & ~((1u << lo_b) - 1));
      }
    }
    const bool left = act && !ready;
    if (a.mark) {  // the only round: leftovers stay pending (listed, or marked after the fills)
      if (left && a.mark == kMarkList) atomicOr(a.pbits + (t >> 5), 1u << (t & 31));
      if (kCovMap && left && a.mark == kMarkJump) atomicOr(&lft[(t - wb.tok) >> 5], 1u << ((t - wb.tok) & 31));
      continue;
    }
    // a wave's tokens fall in at most two 64-token groups, hence two
    // sublists: the first lane of each group reserves its group's places, both
    // in one atomic instruction
    const uint32_t g0 = (base + (threadIdx.x & ~63u)) >> 6;
    const bool in0 = left && (t >> 6) == g0, in1 = left && (t >> 6) == g0 + 1;
    const uint64_t m0 = __ballot(in0), m1 = __ballot(in1);
    if (m0 | m1) {
      const uint32_t f0 = m0 ? uint32_t(__builtin_ctzll(m0)) : 64u, f1 = m1 ? uint32_t(__builtin_ctzll(m1)) : 64u;
      const uint32_t sub0 = g0 % kSub, sub1 = (g0 + 1) % kSub;
      uint32_t at = 0;
      if (lane == f0 || lane == f1) {  // a lane is in at most one group
        const bool h = lane == f1;
        at = atomicAdd(a.cnt_out + (h ? sub1 : sub0) * kCounterStride, uint32_t(__popcll(h ? m1 : m0)));
      }
      const uint32_t at0 = __shfl(at, int(f0 & 63u), 64), at1 = __shfl(at, int(f1 & 63u), 64);
      if (in0) a.list_out[uint64_t(sub0) * a.sub_cap + at0 + lanes_below(m0)] = t;
      if (in1) a.list_out[uint64_t(sub1) * a.sub_cap + at1 + lanes_below(m1)] = t;
    }
  }
  __syncthreads();
  const uint32_t full = blen / 16;
  for (uint32_t k = threadIdx.x; k < nchunk; k += kCopyThreads) {
    if (!((dirty[k >> 5] >> (k & 31)) & 1)) continue;
    if (k < full) {
      *reinterpret_cast<u32x4*>(tile + 16 * k) = *reinterpret_cast<const AX_GLOBAL u32x4*>(ob + 16 * k);
    } else {
      for (uint32_t i = 16 * k; i < blen; ++i) tile[i] = ob[i];
    }
  }
  __syncthreads();
  for (uint32_t base = wb.tok; base < t1; base += kCopyThreads) {
    const uint32_t t = base + threadIdx.x;
    const uint32_t r = t - wb.tok;
    const bool ready = t < t1 && ((rdy[r >> 5] >> (r & 31)) & 1);
    if (!__ballot(ready)) continue;
    uint64_t src = 0, dst = 0;
    uint32_t len = 0;
    if (ready) token_at(a.tok, t, src, dst, len);
    // tile fill: out[dst + k] = out[src + (k mod dist)], destination in the tile
    const bool mine = ready && (a.serial || len < kLongToken);
    const uint32_t drel = uint32_t(dst - bs);
    if (mine && a.serial) {  // the ablation: byte after byte, in-block sources read back from the tile
      for (uint32_t k = 0; k < len; ++k) {
        const uint64_t p = src + k;
        tile[drel + k] = p < bs ? *out.at(p) : tile[p - bs];
      }
    } else if (mine) {
      const uint64_t dist = dst - src;
      uint64_t j = 0;
      for (uint32_t k0 = 0; k0 < len; k0 += 16) {
        if (src + k0 + 16 <= dst && out.contiguous(src + k0, 16)) {  // 16 source bytes before the destination: one unaligned load
          const u32x4 v = *reinterpret_cast<const AX_GLOBAL u32x4_u*>(out.at(src + k0));
#pragma unroll
          for (uint32_t q = 0; q < 16; ++q)
            if (k0 + q < len) tile[drel + k0 + q] = uint8_t(v[q >> 2] >> (8 * (q & 3)));
          j = k0 + 16 == dist ? 0 : k0 + 16;  // dist >= k0 + 16: the periodic index of the next byte
          continue;
        }
        uint64_t idx[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          idx[q] = j;
          if (++j == dist) j = 0;
        }
        uint8_t v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (k0 + q < len) ? *out.at(src + idx[q]) : uint8_t(0);
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (k0 + q < len) tile[drel + k0 + q] = v[q];
      }
    }
    uint64_t wm = __ballot(ready && !mine);  // medium tokens: the whole wave each
    while (wm) {
      const int l = __builtin_ctzll(wm);
      wm &= wm - 1;
      const uint64_t s0 = __shfl((unsigned long long)src, l, 64);
      const uint32_t d0 = __shfl(drel, l, 64), n0 = __shfl(len, l, 64);
      const uint64_t dist = bs + d0 - s0;
      const uint32_t dd = dist < n0 ? uint32_t(dist) : n0;  // the period (n0 when it never wraps)
      const uint32_t step = 64 % dd;
      uint32_t j = lane % dd;
      for (uint32_t k0 = lane; k0 < n0; k0 += 512) {  // eight source loads in flight per lane
        uint32_t jj[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
          jj[q] = j;
          j += step;
          if (j >= dd) j -= dd;
        }
        uint8_t v[8];
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) v[q] = k0 + 64 * q < n0 ? *out.at(s0 + jj[q]) : uint8_t(0);
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q)
          if (k0 + 64 * q < n0) tile[d0 + k0 + 64 * q] = v[q];
      }
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nchunk; k += kCopyThreads) {
    if (!((dirty[k >> 5] >> (k & 31)) & 1)) continue;
    if (k < full) {
      *reinterpret_cast<AX_GLOBAL u32x4*>(ob + 16 * k) = *reinterpret_cast<const u32x4*>(tile + 16 * k);
    } else {
      for (uint32_t i = 16 * k; i < blen; ++i) ob[i] = tile[i];
    }
  }
  if (!kCovMap || a.mark != kMarkJump) return;
  // the block's pending tokens, marked for pointer jumping: the tile's bytes
  // now hold the block's leftover-map row and the waves' stages
  __syncthreads();
  uint32_t* const row = reinterpret_cast<uint32_t*>(tile);
  MarkStage* const mst = reinterpret_cast<MarkStage*>(tile + kMaxB / 8);
  static_assert(kMaxB / 8 + (kCopyThreads / 64) * sizeof(MarkStage) <= kMaxB, "marking fits the tile");
  for (uint32_t k = threadIdx.x; k < a.S / 32; k += kCopyThreads) row[k] = 0;
  __syncthreads();
  for (uint32_t base = wb.tok; base < t1; base += kCopyThreads) {
    const uint32_t t = base + threadIdx.x, r = t - wb.tok;
    const bool pend = t < t1 && ((lft[r >> 5] >> (r & 31)) & 1);
    mark_wave<O>(a, pend, t, mst[threadIdx.x >> 6], row, item);
  }
  __syncthreads();
  uint32_t* const lm = reinterpret_cast<uint32_t*>(a.lmap) + uint64_t(item) * (a.S / 32);
  for (uint32_t k = threadIdx.x; k < a.S / 32; k += kCopyThreads) lm[k] = row[k];
}

// Round 0 as a flat grid over the window's tokens (the alternative
// schedule): 64 consecutive tokens per wave, fills written straight to
// global memory by the wave (short tokens a lane each, long ones the wave,
// or all laid end to end over the lanes).  Same results and lists as
// k_round0; the leftovers of a wave (64-aligned tokens) fall in one 64-token
// group and so in one sublist.
template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_round0_waves(CopyArgs a) {
  __shared__ FillStage stage[kCopyThreads / 64];
  __shared__ MarkStage mstage[kCopyThreads / 64];
  if (__hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const uint32_t lane = lane_id();
  FillStage& fs = stage[threadIdx.x >> 6];
  if (blockIdx.x == 0 && threadIdx.x < kSub) a.cnt_clear[threadIdx.x * kCounterStride] = 0;
  for (uint64_t base = uint64_t(blockIdx.x) * kCopyThreads; base < a.n_tok; base += uint64_t(gridDim.x) * kCopyThreads) {
    const uint32_t t = uint32_t(base + threadIdx.x);
    const bool act = t < a.n_tok;
    uint64_t src = 0, dst = 0;
    uint32_t len = 0, lo = 0, cnt = 0;
    O out(a.jobs[0]);
    if (act) {
      token_at(a.tok, t, src, dst, len);
      const WinBlock wb = a.wbl[a.tblk[t]];
      const JobDev& J = a.jobs[wb.job];
      out = O(J);
      const uint64_t dist = dst - src;
      find_cover(a, wb, J.B, src, src + (dist < len ? dist : len), lo, cnt);
      a.cov[2 * t] = lo;
      a.cov[2 * t + 1] = cnt;
    }
    const bool ready = act && cnt == 0;
    const bool split = ready && !a.serial && len >= kSplitToken;
    const uint64_t sm = __ballot(split);
    if (sm) {
      uint32_t at = 0;
      if (lane == 0) at = atomicAdd(a.long_cnt, uint32_t(__popcll(sm)));
      at = __shfl(at, 0, 64);
      if (split) a.long_list[at + lanes_below(sm)] = t;
    }
    fill_ready<false>(out, ready && !split, dst, src, len, a.serial, a.fill_round, fs);
    if (ready && !split) a.done[t] = 0;
    const bool left = act && !ready;
    if (a.mark) {
      if (left && a.mark == kMarkList) atomicOr(a.pbits + (t >> 5), 1u << (t & 31));
      if (a.mark == kMarkJump) mark_wave<O>(a, left, t, mstage[threadIdx.x >> 6], nullptr, 0);
      continue;
    }
    const uint64_t m = __ballot(left);
    if (m) {
      const uint32_t sub = (t >> 6) % kSub;  // the same for the whole wave
      uint32_t at = 0;
      if (lane == 0) at = atomicAdd(a.cnt_out + sub * kCounterStride, uint32_t(__popcll(m)));
      at = __shfl(at, 0, 64);
      if (left) a.list_out[uint64_t(sub) * a.sub_cap + at + lanes_below(m)] = t;
    }
  }
}

// Later rounds visit the previous round's leftovers.  Leftovers go to this
// workgroup's sublist (counters spread over kSub addresses), or, in the last
// round, to the bitmap of the persistent launch.
template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_round(CopyArgs a) {
  __shared__ FillStage stage[kCopyThreads / 64];
  __shared__ MarkStage mstage[kCopyThreads / 64];
  __shared__ uint32_t sub_end[kSub];  // inclusive prefix of the input sublist lengths
  const uint32_t lane = lane_id();
  FillStage& fs = stage[threadIdx.x >> 6];
  // the status is checked once the counters' loads are in flight
  const uint32_t c_in = threadIdx.x < 64 ? a.cnt_in[threadIdx.x * kCounterStride] : 0u;
  if (__hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  if (blockIdx.x == 0 && threadIdx.x < kSub) a.cnt_clear[threadIdx.x * kCounterStride] = 0;
  if (threadIdx.x < 64) {
    uint32_t tot;
    sub_end[threadIdx.x] = wave_excl_sum(c_in, &tot) + c_in;
  }
  __syncthreads();
  const uint32_t n_items = sub_end[kSub - 1];
  const uint32_t my_sub = blockIdx.x % kSub;
  for (uint64_t base = uint64_t(blockIdx.x) * kCopyThreads; base < n_items; base += uint64_t(gridDim.x) * kCopyThreads) {
    const uint64_t item = base + threadIdx.x;
    const bool act = item < n_items;
    uint32_t t = 0;
    if (act) {  // sublist holding item
      uint32_t sl = 0;
#pragma unroll
      for (uint32_t step = 32; step; step >>= 1)
        if (sub_end[sl + step - 1] <= item) sl += step;
      const uint32_t start = sub_end[sl] - (sl ? sub_end[sl] - sub_end[sl - 1] : sub_end[0]);
      t = a.list_in[uint64_t(sl) * a.sub_cap + (item - start)];
    }
    uint64_t src = 0, dst = 0;
    uint32_t len = 0, lo = 0, cnt = 0;
    O out(a.jobs[0]);
    if (act) {
      token_at(a.tok, t, src, dst, len);
      if (!a.one_job) out = token_out<O>(a, t);
      cover_of(a, t, src, dst, len, lo, cnt);
    }
    // the covering tokens' done flags, four loads in flight at a time
    bool ready = act;
    for (uint32_t i0 = 0; i0 < cnt && ready; i0 += 4) {
      uint8_t f[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) f[q] = i0 + q < cnt ? a.done[lo + i0 + q] : uint8_t(0);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) ready = ready && f[q] < a.round;
    }
    fill_ready<false>(out, ready, dst, src, len, a.serial, a.fill_round, fs);
    if (ready) a.done[t] = uint8_t(a.round);
    const bool left = act && !ready;
    if (a.mark) {
      if (left && a.mark == kMarkList) atomicOr(a.pbits + (t >> 5), 1u << (t & 31));
      if (a.mark == kMarkJump) mark_wave<O>(a, left, t, mstage[threadIdx.x >> 6], nullptr, 0);
      continue;
    }
    const uint64_t m = __ballot(left);
    if (m) {
      uint32_t at = 0;
      if (lane == 0) at = atomicAdd(a.cnt_out + my_sub * kCounterStride, uint32_t(__popcll(m)));
      at = __shfl(at, 0, 64);
      if (left) a.list_out[uint64_t(my_sub) * a.sub_cap + at + lanes_below(m)] = t;
    }
  }
}

// Round 0's long tokens: one workgroup per token, sixteen bytes per thread
// in flight; the token is marked done (round 0) once the whole group is
// through.
template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_long(CopyArgs a) {
  if (__hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const uint32_t n = *a.long_cnt;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t t = a.long_list[i];
    uint64_t src, dst;
    uint32_t len;
    token_at(a.tok, t, src, dst, len);
    const O out = token_out<O>(a, t);
    const uint64_t dist = dst - src;
    const uint64_t step = dist > kCopyThreads ? kCopyThreads : kCopyThreads % uint32_t(dist);
    uint64_t j = dist > threadIdx.x ? threadIdx.x : threadIdx.x % uint32_t(dist);
    for (uint32_t k0 = threadIdx.x; k0 < len; k0 += 16 * kCopyThreads) {
      uint64_t idx[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        idx[q] = j;
        j += step;
        if (j >= dist) j -= dist;
      }
      uint8_t v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (k0 + kCopyThreads * q < len) ? *out.at(src + idx[q]) : uint8_t(0);
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (k0 + kCopyThreads * q < len) *out.at(dst + k0 + kCopyThreads * q) = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) a.done[t] = 0;
  }
}

// Compaction of the last round's leftovers into an ascending list: per
// workgroup of 1024 bitmap words, a population count, then the scatter.
constexpr uint32_t kPackWords = 4 * kCopyThreads;

__device__ inline uint32_t block_sum_u32(uint32_t v, uint32_t* red) {
  uint32_t tot;
  const uint32_t ex = wave_excl_sum(v, &tot);
  (void)ex;
  if (lane_id() == 0) red[threadIdx.x >> 6] = tot;
  __syncthreads();
  uint32_t s = 0;
  for (uint32_t k = 0; k < kCopyThreads / 64; ++k) s += red[k];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kCopyThreads) void k_pcount(const uint32_t* pbits, uint32_t n_words, uint32_t* pcnt) {
  __shared__ uint32_t red[kCopyThreads / 64];
  uint32_t c = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t w = blockIdx.x * kPackWords + k * kCopyThreads + threadIdx.x;
    if (w < n_words) c += __popc(pbits[w]);
  }
  const uint32_t s = block_sum_u32(c, red);
  if (threadIdx.x == 0) pcnt[blockIdx.x] = s;
}

__global__ __launch_bounds__(kCopyThreads) void k_pscatter(const uint32_t* pbits, uint32_t n_words,
                                                           const uint32_t* pcnt, uint32_t* plist, DevStatus* st) {
  __shared__ uint32_t red[kCopyThreads / 64];
  uint32_t before = 0;
  for (uint32_t g = threadIdx.x; g < blockIdx.x; g += kCopyThreads) before += pcnt[g];
  const uint32_t base = block_sum_u32(before, red);
  // thread i takes words 4i..4i+3 of the workgroup's range (consecutive)
  uint32_t wv[4], c = 0;
  const uint32_t w0 = blockIdx.x * kPackWords + 4 * threadIdx.x;
  for (uint32_t k = 0; k < 4; ++k) {
    wv[k] = w0 + k < n_words ? pbits[w0 + k] : 0u;
    c += __popc(wv[k]);
  }
  uint32_t wtot;
  const uint32_t wex = wave_excl_sum(c, &wtot);
  if (lane_id() == 0) red[threadIdx.x >> 6] = wtot;
  __syncthreads();
  uint32_t at = base + wex;
  for (uint32_t k = 0; k < (threadIdx.x >> 6); ++k) at += red[k];
  for (uint32_t k = 0; k < 4; ++k) {
    uint32_t bits = wv[k];
    while (bits) {
      const uint32_t j = __builtin_ctz(bits);
      bits &= bits - 1;
      plist[at++] = (w0 + k) * 32 + j;
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kCopyThreads - 1) st->n_pending = at;
}

// Persistent finish over the compacted leftovers: 64-token chunks of the
// ascending list by ticket; each wave polls its unfinished tokens' covering
// tokens and copies a token once they are all done.  Output bytes and done
// flags use agent-coherent accesses and a store-completion wait precedes
// each done flag, so a flag seen by another XCD implies its bytes are visible
// there.  A token waits only on lower-indexed tokens, which are done or sit
// in lower chunks whose tickets running waves hold, so every wait ends.
template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_tail(CopyArgs a) {
  __shared__ FillStage stage[kCopyThreads / 64];
  const uint32_t lane = lane_id();
  FillStage& fs = stage[threadIdx.x >> 6];
  if (__hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  const uint32_t per = a.tail_chunks;  // consecutive chunks per ticket
  const uint32_t n_pend = a.st->n_pending;
  const uint32_t n_chunks = (n_pend + 63) / 64;
  const uint32_t n_tickets = (n_chunks + per - 1) / per;
  for (;;) {
    uint32_t tk = 0;
    if (lane == 0) tk = atomicAdd(&a.st->ticket, 1u);
    tk = __shfl(tk, 0, 64);
    if (tk >= n_tickets) return;
    for (uint32_t chunk = tk * per; chunk < min(tk * per + per, n_chunks); ++chunk) {
      const uint32_t li = chunk * 64 + lane;
      const uint32_t t = li < n_pend ? a.plist[li] : 0u;
      bool pending = li < n_pend;
      if (!__ballot(pending)) continue;
      uint64_t src = 0, dst = 0;
      uint32_t len = 0, lo = 0, cnt = 0;
      O out(a.jobs[0]);
      if (pending) {
        token_at(a.tok, t, src, dst, len);
        out = token_out<O>(a, t);
        cover_of(a, t, src, dst, len, lo, cnt);
      }
      uint64_t spins = 0;
      while (__ballot(pending)) {
        // flags are read relaxed; an agent-scope acquire fence after a flag
        // that reads a producer's store synchronises with the producer's
        // agent-scope release fence before that store, so the bytes it
        // filled are visible to the loads after the fence, on any XCD
        bool ready = pending;
        for (uint32_t i = 0; i < cnt && ready; ++i)
          ready = __hip_atomic_load(a.done + lo + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kPending;
        if (__ballot(ready)) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          fill_ready<true>(out, ready, dst, src, len, a.serial, a.fill_tail, fs);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          if (ready) __hip_atomic_store(a.done + t, uint8_t(a.round), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          pending = pending && !ready;
        } else {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > a.spin_limit ||
              ((spins & 63) == 0 && __hip_atomic_load(&a.st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            if (lane == 0 && spins > a.spin_limit) report(a.st, AX_E_DEVICE, ~0ull);
            return;
          }
        }
      }
    }
  }
}

// ------------------------------------------- deep remainder: pointer jumping --
//
// The tokens the bulk rounds leave pending (the deep remainder) are resolved
// by pointer jumping over their bytes rather than by a chase of one
// dependency hop at a time.  Positions are window-relative: byte o of window
// block x is x * S + o (S = the largest block size of the plan), so every
// byte of every archive block the window holds has a place in one array of
// 32-bit entries (the jump array) and one bit in each of two bitmaps: the
// leftover map (bytes written by pending tokens) and the active map
// (leftover bytes whose value is not known yet).  An entry holds either the
// window position its value comes from or, with kJRes set, the final byte
// value.  Byte k of a pending token (dst, src, len) takes its value from
// position src + (k mod dist), which lies below dst: a final byte (a
// literal, a token a round copied, a byte of an earlier window or of a block
// the plan does not decode) or a byte of another, earlier pending token.
// Entries therefore form a forest rooted at final values.  A pass replaces
// each active entry by the entry its entry names, twice over (three times
// the hops per pass), so about log3(chain length) passes resolve every
// chain; a gather then writes the leftover bytes as whole 16-byte chunks.
// Updating entries in place is safe in any order: an entry always names a
// byte holding the same value, and every read returns some complete entry.
constexpr uint32_t kJPasses = 32;        // pass-flag slots
constexpr uint32_t kJShards = 16;        // flag words per pass (workgroup g writes g mod 16)
constexpr uint32_t kJFlagStride = 16;    // u32 between two flag words
constexpr uint32_t kJMaxGrid = 8192;     // workgroups of a position-driven launch
constexpr uint32_t kJChaseLimit = 1u << 24;  // hops the gather follows before it reports a device error

struct JumpArgs {
  const JobDev* jobs;
  const WinBlock* wbl;
  uint32_t n_items;    // window blocks
  uint32_t n_tok;      // window tokens
  uint32_t S;          // position stride of a window block
  const uint64_t* tok;
  const uint32_t* tblk;
  const uint8_t* done;
  uint32_t* J;         // one entry per window position
  uint64_t* lmap;      // leftover map, one bit per window position
  uint64_t* amap;      // active map
  uint32_t* flags;     // kJPasses x kJShards words, kJFlagStride apart
  uint8_t** ibase;     // per window block: where its output bytes start
  uint32_t s_log2;     // log2 S
  const uint32_t* llist;  // long pending tokens: kSub sublists of sub_cap
  const uint32_t* lcnt;   // their counters, kCounterStride apart
  uint32_t sub_cap;
  uint32_t* wlist;     // leftover-map words with bits set
  DevStatus* st;
  uint32_t pass;
};

__device__ inline bool jump_failed(const DevStatus* st) {
  return __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// An entry naming no leftover byte (cannot happen for entries the init
// wrote): the decode reports a device error instead of following it.
// `where` (recorded as the failing block, with the top bit set) names the
// check: 1 settling the first entries, 2 a pass, 3 the gather.
__device__ inline uint32_t jump_broken(DevStatus* st, uint32_t where) {
  report(st, AX_E_DEVICE, (1ull << 63) | where);
  return kJRes;
}

// Long pending tokens: one workgroup per token, byte k of the token on lane
// k mod 256 (first entries as in the marking of a round, bits by global
// atomics).
template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_jmarklong(JumpArgs a) {
  __shared__ uint32_t sub_end[kSub];  // inclusive prefix of the sublist lengths
  if (jump_failed(a.st)) return;
  if (threadIdx.x < 64) {
    uint32_t tot;
    const uint32_t c = a.lcnt[threadIdx.x * kCounterStride];
    sub_end[threadIdx.x] = wave_excl_sum(c, &tot) + c;
  }
  __syncthreads();
  const uint32_t n = sub_end[kSub - 1], lane = threadIdx.x;  // the workgroup's lanes share a token
  AX_GLOBAL uint32_t* const J = gp(a.J);
  uint32_t* const lm32 = reinterpret_cast<uint32_t*>(a.lmap);
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    uint32_t sl = 0;  // sublist holding item i
#pragma unroll
    for (uint32_t step = 32; step; step >>= 1)
      if (sub_end[sl + step - 1] <= i) sl += step;
    const uint32_t start = sl ? sub_end[sl - 1] : 0u;
    const uint32_t t = a.llist[uint64_t(sl) * a.sub_cap + (i - start)];
    uint64_t src, dst;
    uint32_t len;
    token_at(a.tok, t, src, dst, len);
    const uint32_t item = a.tblk[t];
    const WinBlock wb = a.wbl[item];
    const JobDev jd = a.jobs[wb.job];
    const uint32_t lb = __builtin_ctz(jd.B);
    const uint64_t bs = wb.b << lb, dist = dst - src;
    uint64_t cb = ~0ull;  // the source block last looked up, kept over the lane's passes
    uint32_t cbase = 0;
    bool cin = false;
    // byte k of the token goes to lane k mod 256, so each wave store covers
    // 64 consecutive entries; a wave's 64 positions meet at most three words
    // of the leftover map, set by three lanes from the wave's ballot
    const uint32_t d0 = item * a.S + uint32_t(dst - bs);  // window position of the token's first byte
    const bool wrap = dist < len;                          // a periodic fill: sources repeat every dist bytes
    const uint32_t per = wrap ? uint32_t(dist) : 0u;
    const uint32_t jstep = wrap ? kCopyThreads % per : kCopyThreads;
    uint32_t j = wrap ? lane % per : lane;  // source index of byte k
    const uint32_t wl = lane & 63u, wofs = lane & ~63u;
    for (uint32_t kb = 0; kb < len; kb += kCopyThreads) {
      const uint32_t k = kb + lane;
      const bool valid = k < len;
      if (valid) {
        const uint64_t sp = src + j, sb = sp >> lb;
        if (sb != cb) cb = sb, cin = window_block(a.wbl, a.S, wb, sb, cbase);
        J[d0 + k] = cin ? cbase + uint32_t(sp & (jd.B - 1)) : kJRes | *O(jd).at(sp);
      }
      const uint64_t m = __ballot(valid);
      if (m && wl < 3) {
        const uint32_t p0 = d0 + kb + wofs, off = p0 & 31u;  // the wave's first position
        uint32_t bits;
        if (wl == 0) bits = uint32_t(m << off);
        else if (wl == 1) bits = off ? uint32_t(m >> (32 - off)) : uint32_t(m >> 32);
        else bits = off ? uint32_t(m >> (64 - off)) : 0u;
        if (bits) atomicOr(&lm32[(p0 >> 5) + wl], bits);
      }
      j += jstep;
      if (wrap && j >= per) j -= per;
    }
  }
}

// The work list: the leftover-map words with bits set, in one pass (each
// workgroup takes kJListWords words, finds its busy ones and appends them at
// a place reserved with one atomic add; the list is in no particular order,
// which the walks below do not need).  When more than a quarter of the map's words are busy
// the kernels below walk the whole map instead (dense).
constexpr uint32_t kJListWords = 16 * kCopyThreads;
__device__ inline bool jump_dense(const JumpArgs& a, uint32_t n_words) {
  return uint64_t(n_words) * 4 > uint64_t(a.n_items) * (a.S / 64);
}

__global__ __launch_bounds__(kCopyThreads) void k_jlist(JumpArgs a) {
  __shared__ uint32_t wtot[kCopyThreads / 64];
  __shared__ uint32_t base;
  if (jump_failed(a.st)) return;
  const uint64_t words = uint64_t(a.n_items) * (a.S / 64), w0 = uint64_t(blockIdx.x) * kJListWords;
  constexpr uint32_t kPer = kJListWords / kCopyThreads;  // words per thread, kCopyThreads apart (coalesced reads)
  uint32_t bits = 0, c = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint64_t g = w0 + q * kCopyThreads + threadIdx.x;
    if (g < words && a.lmap[g] != 0) bits |= 1u << q, ++c;
  }
  uint32_t tot;
  const uint32_t ex = wave_excl_sum(c, &tot);
  if (lane_id() == 0) wtot[threadIdx.x >> 6] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t all = 0;
    for (uint32_t k = 0; k < kCopyThreads / 64; ++k) all += wtot[k];
    base = all ? atomicAdd(&a.st->n_jwords, all) : 0u;
  }
  __syncthreads();
  uint32_t at = base + ex;
  for (uint32_t k = 0; k < (threadIdx.x >> 6); ++k) at += wtot[k];
  while (bits) {
    const uint32_t q = __builtin_ctz(bits);
    bits &= bits - 1;
    a.wlist[at++] = uint32_t(w0 + q * kCopyThreads + threadIdx.x);
  }
}

// The position-driven kernels below visit the leftover-map words with bits
// set, eight at a time, one position per lane, so the map's rows are read
// and written as coalesced 256-byte rows.  Two walks, chosen per window by
// the list build: when more than a quarter of the map's words are busy, a
// wave reads 64 map words per step (four 16-word chunks a grid apart, so a
// dense region spreads over many waves) and takes the busy ones eight at a
// time; otherwise the work list is walked eight words per step (the next
// step's words in flight), so a sparse map costs no empty reads.
constexpr uint32_t kJStepWords = 8;
constexpr uint32_t kJChunk = 16;

// A group of up to kJStepWords busy map words: their indices and bits
// (wave-uniform, held in scalar registers; bits 0 marks an unused slot).
struct WordGroup {
  uint32_t g[kJStepWords];
  uint64_t wv[kJStepWords];
};

// (the builtin returns int: widen through uint32_t, not by sign extension)
__device__ inline uint64_t uniform64(uint64_t v) {
  return uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v))))) |
         (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(v >> 32))))) << 32);
}

// Call f(group) for groups of up to kJStepWords busy words of `map` (the
// leftover or the active map).
template <class F>
__device__ inline void walk_words(const JumpArgs& a, const uint64_t* map, F&& f) {
  const uint32_t lane = lane_id();
  const uint64_t waves = uint64_t(gridDim.x) * (kCopyThreads / 64);
  const uint64_t wave = uint64_t(blockIdx.x) * (kCopyThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t n = a.st->n_jwords;
  WordGroup w;
  if (jump_dense(a, n)) {
    const uint64_t words = uint64_t(a.n_items) * (a.S / 64);
    const uint64_t steps = (words + kJChunk * 4 * waves - 1) / (kJChunk * 4 * waves);
    for (uint64_t i = 0; i < steps; ++i) {
      // lane l reads word l mod 16 of chunk (4 i + l / 16) * waves + wave
      const uint64_t mine = ((i * 4 + (lane >> 4)) * waves + wave) * kJChunk + (lane & 15u);
      const uint64_t mw = mine < words ? map[mine] : 0ull;
      uint64_t nz = uniform64(__ballot(mw != 0));
      while (nz) {
#pragma unroll
        for (uint32_t u = 0; u < kJStepWords; ++u) {
          w.g[u] = 0;
          w.wv[u] = 0;
          if (nz) {
            const uint32_t wi = uint32_t(__builtin_ctzll(nz));
            nz &= nz - 1;
            w.wv[u] = uniform64(__shfl((unsigned long long)mw, int(wi), 64));
            w.g[u] = uint32_t(((i * 4 + (wi >> 4)) * waves + wave) * kJChunk + (wi & 15u));
          }
        }
        f(w);
      }
    }
    return;
  }
  for (uint64_t i0 = wave * kJStepWords; i0 < n; i0 += waves * kJStepWords) {
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) {
      w.g[u] = i0 + u < n ? a.wlist[i0 + u] : 0u;
      w.wv[u] = i0 + u < n ? map[w.g[u]] : 0ull;
    }
    f(w);
  }
}

// Value of the byte at window position v (a final byte).
__device__ inline uint32_t jbyte(const JumpArgs& a, uint32_t v) {
  return gp(a.ibase[v >> a.s_log2])[v & ((1u << a.s_log2) - 1u)];
}

// First entries, settled: an entry naming a position outside the leftover
// map (a final byte) takes that byte's value; the rest stay active.
__global__ __launch_bounds__(kCopyThreads) void k_jinit(JumpArgs a) {
  if (jump_failed(a.st)) return;
  const uint32_t lane = lane_id(), limit = a.n_items * a.S;
  AX_GLOBAL uint32_t* const J = gp(a.J);
  walk_words(a, a.lmap, [&](const WordGroup& w) __attribute__((always_inline)) {
    const uint32_t* const g = w.g;
    const uint64_t* const wv = w.wv;
    uint32_t v[kJStepWords];
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) v[u] = ((wv[u] >> lane) & 1) ? J[g[u] * 64 + lane] : kJRes;
    bool leftover[kJStepWords];
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) {
      leftover[u] = true;
      if (!(v[u] & kJRes)) {
        if (v[u] >= limit) v[u] = jump_broken(a.st, 1);
        else leftover[u] = (a.lmap[v[u] >> 6] >> (v[u] & 63)) & 1;
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u)
      if (!leftover[u]) v[u] = kJRes | jbyte(a, v[u]);
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) {
      if (!wv[u]) continue;
      const bool act = (wv[u] >> lane) & 1;
      if (act && !leftover[u]) J[g[u] * 64 + lane] = v[u];
      const uint64_t still = __ballot(act && !(v[u] & kJRes));
      if (lane == 0) a.amap[g[u]] = still;
    }
  });
  // the dense walk visits only busy words: the others' active bits are zero
  if (jump_dense(a, a.st->n_jwords)) {
    const uint64_t words = uint64_t(a.n_items) * (a.S / 64);
    for (uint64_t w = uint64_t(blockIdx.x) * kCopyThreads + threadIdx.x; w < words;
         w += uint64_t(gridDim.x) * kCopyThreads)
      if (!a.lmap[w]) a.amap[w] = 0;
  }
}

// One jump pass: every active entry takes the entry two steps along its
// chain.  A pass whose predecessor left nothing active exits at once (and
// the first such pass records how many passes did work).
__global__ __launch_bounds__(kCopyThreads) void k_jpass(JumpArgs a) {
  if (jump_failed(a.st)) return;
  if (a.pass > 0) {
    const uint32_t* pf = a.flags + (a.pass - 1) * kJShards * kJFlagStride;
    const uint32_t f = threadIdx.x < kJShards ? pf[threadIdx.x * kJFlagStride] : 0u;
    if (!__syncthreads_or(int(f))) {
      if (blockIdx.x == 0 && threadIdx.x == 0 && a.st->jump_used == 0) a.st->jump_used = a.pass;
      return;
    }
  }
  const uint32_t lane = lane_id(), limit = a.n_items * a.S;
  AX_GLOBAL uint32_t* const J = gp(a.J);
  bool any = false;
  walk_words(a, a.amap, [&](const WordGroup& w) __attribute__((always_inline)) {
    const uint32_t* const g = w.g;
    const uint64_t* const wv = w.wv;
    uint32_t v[kJStepWords];
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) v[u] = ((wv[u] >> lane) & 1) ? J[g[u] * 64 + lane] : kJRes;
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u)
      if (!(v[u] & kJRes)) v[u] = v[u] < limit ? J[v[u]] : jump_broken(a.st, 2);
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u)
      if (!(v[u] & kJRes)) v[u] = v[u] < limit ? J[v[u]] : jump_broken(a.st, 2);
#pragma unroll
    for (uint32_t u = 0; u < kJStepWords; ++u) {
      if (!wv[u]) continue;
      const bool act = (wv[u] >> lane) & 1;
      if (act) J[g[u] * 64 + lane] = v[u];
      const uint64_t still = __ballot(act && !(v[u] & kJRes));
      if (lane == 0 && still != wv[u]) a.amap[g[u]] = still;
      any |= still != 0;
    }
  });
  if (__syncthreads_or(int(any)) && threadIdx.x == 0)
    a.flags[(a.pass * kJShards + blockIdx.x % kJShards) * kJFlagStride] = 1;
}

// Output: every leftover byte takes its entry's value (following any entry
// the passes left unfinished).  Of a group of eight busy words, a lane owns
// four consecutive positions of one word in each half: one 16-byte entry
// load, then one 32-bit store when all four are leftover (byte stores
// otherwise: the other bytes keep their value).
__global__ __launch_bounds__(kCopyThreads) void k_jgather(JumpArgs a) {
  if (jump_failed(a.st)) return;
  const uint32_t lane = lane_id(), limit = a.n_items * a.S, omask = (1u << a.s_log2) - 1u;
  const AX_GLOBAL uint32_t* const J = gp(a.J);
  const uint32_t sub = lane >> 4, q4 = 4 * (lane & 15u);
  static_assert(kJStepWords == 8, "the gather takes a group's words as two halves of four");
  walk_words(a, a.lmap, [&](const WordGroup& w) __attribute__((always_inline)) {
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) {
      // this lane's word of the half: word 4 h + (lane / 16) (a select: it varies by lane)
      const uint32_t g0 = w.g[4 * h], g1 = w.g[4 * h + 1], g2 = w.g[4 * h + 2], g3 = w.g[4 * h + 3];
      const uint64_t w0 = w.wv[4 * h], w1 = w.wv[4 * h + 1], w2 = w.wv[4 * h + 2], w3 = w.wv[4 * h + 3];
      const uint32_t gk = sub < 2 ? (sub == 0 ? g0 : g1) : (sub == 2 ? g2 : g3);
      const uint64_t wk = sub < 2 ? (sub == 0 ? w0 : w1) : (sub == 2 ? w2 : w3);
      const uint32_t bits4 = uint32_t(wk >> q4) & 0xFu;
      if (!bits4) continue;
      const uint32_t p = gk * 64 + q4;
      u32x4 e = *reinterpret_cast<const AX_GLOBAL u32x4*>(J + p);
      uint32_t x0 = (bits4 & 1) ? e.x : kJRes, x1 = (bits4 & 2) ? e.y : kJRes;
      uint32_t x2 = (bits4 & 4) ? e.z : kJRes, x3 = (bits4 & 8) ? e.w : kJRes;
      if (!(x0 & x1 & x2 & x3 & kJRes)) {  // an entry the passes did not finish: follow it
        for (uint32_t hop = 0; !(x0 & kJRes); ++hop) x0 = x0 < limit && hop < kJChaseLimit ? J[x0] : jump_broken(a.st, 3);
        for (uint32_t hop = 0; !(x1 & kJRes); ++hop) x1 = x1 < limit && hop < kJChaseLimit ? J[x1] : jump_broken(a.st, 3);
        for (uint32_t hop = 0; !(x2 & kJRes); ++hop) x2 = x2 < limit && hop < kJChaseLimit ? J[x2] : jump_broken(a.st, 3);
        for (uint32_t hop = 0; !(x3 & kJRes); ++hop) x3 = x3 < limit && hop < kJChaseLimit ? J[x3] : jump_broken(a.st, 3);
      }
      AX_GLOBAL uint8_t* const o = gp(a.ibase[p >> a.s_log2]) + (p & omask);
      if (bits4 == 0xFu) {
        *reinterpret_cast<AX_GLOBAL uint32_t*>(o) = (x0 & 0xFFu) | ((x1 & 0xFFu) << 8) | ((x2 & 0xFFu) << 16) | ((x3 & 0xFFu) << 24);
      } else {
        if (bits4 & 1) o[0] = uint8_t(x0);
        if (bits4 & 2) o[1] = uint8_t(x1);
        if (bits4 & 4) o[2] = uint8_t(x2);
        if (bits4 & 8) o[3] = uint8_t(x3);
      }
    }
  });
}

// A range decode's slot table: the window's blocks (one window) take slots
// 0, 1, ... in window order.
__global__ void k_slots(uint32_t* slot, const WinBlock* wbl, uint32_t n_items) {
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < n_items; x += gridDim.x * blockDim.x)
    slot[wbl[x].b] = x;
}

// Zero two word ranges (one launch for both).
// The tokens round 0 left: the sum of its sublist counters (one wave).
__global__ void k_pending0(const uint32_t* cnt, DevStatus* st) {
  uint32_t tot;
  (void)wave_excl_sum(threadIdx.x < kSub ? cnt[threadIdx.x * kCounterStride] : 0u, &tot);
  if (threadIdx.x == 0) st->pend0 = tot;
}

// Status reset before each window (the first also clears the error word).
__device__ inline void window_status_reset(DevStatus* st, int first) {
  if (first) {
    st->err = 0;
    st->bad_block = ~0ull;
  }
  st->ticket = 0;
  st->long_count = 0;
  st->n_pending = 0;
  st->jump_used = 0;
  st->n_jwords = 0;
  st->pend0 = 0;
}

__global__ void k_window_init(DevStatus* st, int first) {
  if (threadIdx.x == 0) window_status_reset(st, first);
}

// Everything a window's match layer needs zeroed or precomputed, in one
// launch before its entropy stage: the status words, the list counters and
// pass flags, the persistent chase's leftover bitmap, and for pointer
// jumping the leftover map (the last round sets its bits) and where every
// window block's output bytes start.
struct PrepArgs {
  DevStatus* st;
  int first;
  uint32_t* counts;
  uint32_t n_counts;
  uint32_t* pbits;
  uint32_t n_pbits;
  uint64_t* lmap;  // null: no jump in this window
  uint64_t n_lmap;
  uint8_t** ibase;
  const JobDev* jobs;
  const WinBlock* wbl;
  uint32_t n_items;
};

template <class O>
__global__ __launch_bounds__(kCopyThreads) void k_window_prep(PrepArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) window_status_reset(a.st, a.first);
  const uint64_t i0 = uint64_t(blockIdx.x) * kCopyThreads + threadIdx.x, step = uint64_t(gridDim.x) * kCopyThreads;
  for (uint64_t i = i0; i < a.n_counts; i += step) a.counts[i] = 0;
  for (uint64_t i = i0; i < a.n_pbits; i += step) a.pbits[i] = 0;
  if (!a.lmap) return;
  for (uint64_t i = i0; i < a.n_lmap; i += step) a.lmap[i] = 0;
  for (uint64_t x = i0; x < a.n_items; x += step) {
    const WinBlock wb = a.wbl[x];
    const JobDev& jd = a.jobs[wb.job];
    a.ibase[x] = (uint8_t*)(O(jd).at(wb.b * jd.B));
  }
}

// --------------------------------------------------------------- host side --

inline uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

}  // namespace

namespace ax {

struct Layout {
  uint64_t status, nsym, lit, cmd, off, len, tok, tblk, cov, done, counts, jflags, list0, list1, llist, pbits, pcnt,
      plist, lmap, mcov, amap, ibase, wlist, total;
  uint64_t jbytes;  // the jump array: the stream slots, dead once the parse is through
  uint64_t sub_cap;
};

// A decode plan: jobs (archives and where their bytes go), cut into windows
// of at most kWindowBlocks blocks.  A window's sources lie in earlier windows
// or inside it, so windows run one after another with bounded scratch.
struct Plan {
  std::vector<JobDev> jobs;
  std::vector<WinBlock> wbl;
  std::vector<uint64_t> gtok;  // per window block: its first token's index in its archive
  struct Win {
    uint64_t at;       // first WinBlock
    uint32_t items;    // blocks
    uint32_t tok;      // tokens
  };
  std::vector<Win> wins;
  uint32_t max_items = 0, max_tok = 0, slot_b = 0, off_cap = 0, len_cap = 0;
  uint64_t out_bytes = 0, n_tokens = 0;
  void* d_mem = nullptr;
  JobDev* d_jobs = nullptr;
  WinBlock* d_wbl = nullptr;
  JobDev* h_pinned = nullptr;  // staging for refreshing output pointers
  uint8_t* h_stage = nullptr;  // staging for plan_reset uploads
  size_t dev_cap = 0, stage_cap = 0, pinned_cap = 0;
  hipEvent_t staged = nullptr;  // the last upload from h_stage / h_pinned
  std::vector<uint8_t*> dev_out;  // output pointers as last uploaded
  Layout lay{};
  PlanOptions opt{};
  int copy_grid = 1;
  bool timing = false, events_ok = false;
  size_t timed_windows = 0;  // windows the last timed decode recorded
  // stage events, five per window: entropy, parse, bulk rounds, deep
  // remainder, end
  std::vector<hipEvent_t> ev;
  // jump passes launched per window: from a bound on the chain length at
  // first, then the count the device reported as needed (+1 spare pass,
  // which exits at once and reports it again); the gather finishes any
  // entry the passes leave, so the count never changes a byte
  std::vector<uint32_t> jpass;
  // per window, the passes the device reported as needed (0: not known);
  // once every window's count is known the spare pass is dropped
  std::vector<uint32_t> jneed;
  // pinned: per window, the passes that found work and the tokens round 0
  // filled (two words)
  uint32_t* h_jused = nullptr;
  size_t jused_cap = 0;
  hipEvent_t jfed = nullptr;     // h_jused is complete after this
  bool jfeed_pending = false, jsettled = false;
  // bulk rounds per window, learned from round 0's report when the caller
  // left the count to the library: a window whose round 0 fills less than a
  // tenth of its tokens (a deep archive) goes straight to the remainder (0:
  // the configured count)
  std::vector<uint8_t> wbulk;
  bool bulk_auto = true, bsettled = false;
  bool learn = true;             // plans rebuilt for every call (ranges) keep the bound
  bool mapped = false;           // one job whose output is a compact scratch addressed by slot
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  void* graph_work = nullptr;
  int graph_mode = -1;
  bool graph_stale = false;  // rebuilt at the next decode that may allocate
  hipStream_t cap_stream = nullptr;
  ~Plan() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (graph_def) (void)hipGraphDestroy(graph_def);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (staged) {
      (void)hipEventSynchronize(staged);
      (void)hipEventDestroy(staged);
    }
    if (jfed) {
      (void)hipEventSynchronize(jfed);
      (void)hipEventDestroy(jfed);
    }
    if (h_jused) (void)hipHostFree(h_jused);
    if (d_mem) (void)hipFree(d_mem);
    if (h_pinned) (void)hipHostFree(h_pinned);
    if (h_stage) (void)hipHostFree(h_stage);
  }
};

static Layout make_layout(const Plan& P) {
  Layout L{};
  const uint64_t W = std::max<uint32_t>(1, P.max_items), T = std::max<uint32_t>(1, P.max_tok);
  uint64_t at = 0;
  L.status = at, at = align256(at + sizeof(DevStatus));
  L.nsym = at, at = align256(at + 16 * W);
  L.lit = at, at = align256(at + W * P.slot_b);
  L.cmd = at, at = align256(at + W * P.slot_b);
  L.off = at, at = align256(at + W * P.off_cap);
  L.len = at, at = align256(at + W * P.len_cap);
  L.tok = at, at = align256(at + 16 * T);
  L.tblk = at, at = align256(at + 4 * T);
  L.cov = at, at = align256(at + 8 * T);
  L.done = at, at = align256(at + T);
  L.counts = at, at = align256(at + 4ull * 3 * kSub * kCounterStride);
  L.jflags = at, at = align256(at + 4ull * kJPasses * kJShards * kJFlagStride);  // cleared with the counters
  // a round over n <= T items launches G = min(ceil(T / 256), kMaxRoundGrid)
  // workgroups, each visiting at most ceil(n / (256 G)) * 256 items, and
  // sublist s takes the items of the ceil(G / kSub) workgroups g = s mod kSub:
  // at most n / kSub + 4 G + n / G + 256 <= ceil(T / kSub) + 256 (ceil(G /
  // kSub) + 2) (leftovers filed by token group, (t / 64) mod kSub, stay
  // within ceil(T / kSub) + 64)
  const uint64_t G = std::min<uint64_t>((T + kCopyThreads - 1) / kCopyThreads, kMaxRoundGrid);
  L.sub_cap = (T + kSub - 1) / kSub + uint64_t(kCopyThreads) * ((G + kSub - 1) / kSub + 2);
  L.list0 = at, at = align256(at + 4 * kSub * L.sub_cap);
  L.list1 = at, at = align256(at + 4 * kSub * L.sub_cap);
  L.llist = at, at = align256(at + 4 * T);
  L.pbits = at, at = align256(at + 4 * ((T + 31) / 32 + 64));
  L.pcnt = at, at = align256(at + 4 * ((T + 31) / 32 / kPackWords + 1));
  L.plist = at, at = align256(at + 4 * T);
  L.lmap = at, at = align256(at + W * P.slot_b / 8);
  L.mcov = at, at = align256(at + W * P.slot_b / 8);
  L.ibase = at, at = align256(at + 8 * W);
  L.wlist = at, at = align256(at + W * P.slot_b / 16);                        // one u32 per map word
  L.amap = at, at = align256(at + W * P.slot_b / 8);
  L.total = at;
  // the jump array (4 B per window position) reuses the four stream slots,
  // dead once the parse is through: at least 5 B per window position
  L.jbytes = L.len + W * P.len_cap - L.lit;
  return L;
}

static int hip_fail(hipError_t e, const char* what) {
  (void)what;
  return fail(AX_E_HIP, hipGetErrorString(e));
}

// Jump passes that resolve any chain of a window of `tok` tokens: a chain
// visits each pending token at most once, the first entries span one hop,
// and a pass triples the hops an entry spans.
static uint32_t jump_pass_bound(uint64_t tok) {
  uint32_t p = 1;
  uint64_t span = 3;
  while (p < kJPasses && span <= tok) ++p, span *= 3;
  return p;
}

// Host tables of a plan: jobs, window blocks, windows, maxima.
static int build_tables(Plan* P, const std::vector<JobSpec>& specs) {
  try {
    P->jobs.assign(specs.size(), JobDev{});
    P->wbl.clear();
    P->gtok.clear();
    P->wins.clear();
    P->max_items = P->max_tok = P->slot_b = P->off_cap = P->len_cap = 0;
    P->out_bytes = P->n_tokens = 0;
    uint64_t gblocks = 0;
    for (size_t j = 0; j < specs.size(); ++j) {
      const aceapex_decoder* d = specs[j].dec;
      const aceapex_info& I = d->info;
      JobDev& J = P->jobs[j];
      J.arc = d->d_arc;
      J.out = specs[j].out;
      J.payload_at = I.header_bytes;
      J.n_bytes = I.n_bytes;
      J.nb = I.n_blocks;
      J.B = I.block_size;
      J.mm = I.min_match;
      J.slot = specs[j].slot;
      J.junk = specs[j].junk;
      P->slot_b = std::max(P->slot_b, I.block_size);
      P->off_cap = std::max(P->off_cap, uint32_t((10 * (I.block_size / I.min_match + 1) + 15) & ~15u));
      P->len_cap = std::max(P->len_cap, 3 * I.block_size);
      P->out_bytes += I.n_bytes;
      gblocks += specs[j].blocks.empty() ? I.n_blocks : specs[j].blocks.size();
    }
    P->wbl.reserve(gblocks);
    P->gtok.reserve(gblocks);
    // windows: consecutive (job, block) items, at most kWindowBlocks blocks
    // and kWindowTokens tokens each
    Plan::Win cur{0, 0, 0};
    auto close = [&]() {
      if (!cur.items) return;
      for (uint64_t i = cur.at; i < cur.at + cur.items;) {  // per-job extents inside the window
        uint64_t k = i;
        while (k < cur.at + cur.items && P->wbl[k].job == P->wbl[i].job) ++k;
        for (uint64_t m = i; m < k; ++m) {
          P->wbl[m].first = uint32_t(i - cur.at);
          P->wbl[m].count = uint32_t(k - i);
        }
        i = k;
      }
      P->max_items = std::max(P->max_items, cur.items);
      P->max_tok = std::max(P->max_tok, cur.tok);
      P->n_tokens += cur.tok;
      P->wins.push_back(cur);
      cur = Plan::Win{P->wbl.size(), 0, 0};
    };
    // jobs enter the windows densest first (matches per block): a window runs
    // as long as its deepest dependency chain, and match-dense archives carry
    // the deep chains, so they share windows instead of lengthening every one
    std::vector<size_t> order(specs.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = j;
    auto density = [&](size_t j) {
      const aceapex_decoder* d = specs[j].dec;
      return d->info.n_blocks ? double(d->mpre[d->info.n_blocks]) / double(d->info.n_blocks) : 0.0;
    };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return density(x) > density(y); });
    for (const size_t j : order) {
      const aceapex_decoder* d = specs[j].dec;
      const uint64_t nb = specs[j].blocks.empty() ? d->info.n_blocks : specs[j].blocks.size();
      for (uint64_t i = 0; i < nb; ++i) {
        const uint64_t b = specs[j].blocks.empty() ? i : specs[j].blocks[i];
        if (b >= d->info.n_blocks) return fail(AX_E_RANGE, "block outside the archive");
        const uint64_t nt = d->mpre[b + 1] - d->mpre[b];
        if (cur.items == kWindowBlocks || uint64_t(cur.tok) + nt > kWindowTokens) close();
        P->wbl.push_back(WinBlock{b, uint32_t(j), cur.tok, 0, 0});
        P->gtok.push_back(d->mpre[b]);
        cur.items++;
        cur.tok += uint32_t(nt);
      }
    }
    close();
    P->mapped = !specs.empty() && specs[0].slot != nullptr;
    P->jpass.assign(P->wins.size(), 0);
    for (size_t i = 0; i < P->wins.size(); ++i) P->jpass[i] = jump_pass_bound(P->wins[i].tok);
    P->jneed.assign(P->wins.size(), 0);
    P->jsettled = false;
    P->wbulk.assign(P->wins.size(), 0);
    P->bsettled = false;
  } catch (const std::bad_alloc&) {
    return fail(AX_E_NOMEM, "plan tables");
  }
  P->lay = make_layout(*P);
  return AX_OK;
}

static size_t table_bytes(const Plan* P, size_t* wbl_at) {
  const size_t jb = sizeof(JobDev) * std::max<size_t>(1, P->jobs.size());
  *wbl_at = align256(jb);
  return *wbl_at + sizeof(WinBlock) * std::max<size_t>(1, P->wbl.size());
}

// Device tables big enough for the current host tables (grown when needed).
static int ensure_device(Plan* P) {
  size_t wbl_at;
  const size_t need = table_bytes(P, &wbl_at);
  if (need > P->dev_cap) {
    if (P->d_mem) (void)hipFree(P->d_mem), P->d_mem = nullptr;
    const size_t cap = std::max(need, 2 * P->dev_cap);
    hipError_t e = hipMalloc(&P->d_mem, cap);
    if (e != hipSuccess) return hip_fail(e, "plan memory");
    P->dev_cap = cap;
  }
  const size_t jb = sizeof(JobDev) * std::max<size_t>(1, P->jobs.size());
  if (jb > P->pinned_cap) {
    if (P->h_pinned) (void)hipHostFree(P->h_pinned), P->h_pinned = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&P->h_pinned), jb);
    if (e != hipSuccess) return hip_fail(e, "plan staging");
    P->pinned_cap = jb;
  }
  P->d_jobs = static_cast<JobDev*>(P->d_mem);
  P->d_wbl = reinterpret_cast<WinBlock*>(static_cast<uint8_t*>(P->d_mem) + wbl_at);
  if (!P->staged) {
    hipError_t e = hipEventCreateWithFlags(&P->staged, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "plan event");
  }
  // the jump-pass report of every window, so that a decode allocates nothing
  if (P->wins.size() > P->jused_cap) {
    if (P->jfeed_pending) (void)hipEventSynchronize(P->jfed), P->jfeed_pending = false;
    if (P->h_jused) (void)hipHostFree(P->h_jused), P->h_jused = nullptr;
    P->jused_cap = 0;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&P->h_jused), 8 * P->wins.size());
    if (e != hipSuccess) return hip_fail(e, "pass report staging");
    P->jused_cap = P->wins.size();
  }
  if (!P->jfed) {
    hipError_t e = hipEventCreateWithFlags(&P->jfed, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "pass report event");
  }
  return AX_OK;
}

static int device_setup(Plan* P) {
  int dev = 0, cus = 0, occ = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_tail<OutDirect>), kCopyThreads, 0);
  P->copy_grid = std::max(1, cus) * std::max(1, occ);
  return AX_OK;
}

int plan_create(const std::vector<JobSpec>& specs, Plan** out) {
  *out = nullptr;
  Plan* P = new (std::nothrow) Plan;
  if (!P) return fail(AX_E_NOMEM, "plan");
  int rc = build_tables(P, specs);
  if (!rc) rc = ensure_device(P);
  if (rc) {
    delete P;
    return rc;
  }
  hipError_t e = hipMemcpy(P->d_jobs, P->jobs.data(), sizeof(JobDev) * P->jobs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !P->wbl.empty())
    e = hipMemcpy(P->d_wbl, P->wbl.data(), sizeof(WinBlock) * P->wbl.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete P;
    return hip_fail(e, "plan upload");
  }
  P->dev_out.resize(P->jobs.size());
  for (size_t j = 0; j < P->jobs.size(); ++j) P->dev_out[j] = P->jobs[j].out;
  device_setup(P);
  *out = P;
  return AX_OK;
}

int plan_reset(Plan* P, const std::vector<JobSpec>& specs, hipStream_t s) {
  // staging may still feed the previous upload; a pass report of the old
  // windows may still be on its way
  if (P->staged) (void)hipEventSynchronize(P->staged);
  if (P->jfeed_pending) (void)hipEventSynchronize(P->jfed), P->jfeed_pending = false;
  int rc = build_tables(P, specs);
  if (!rc) rc = ensure_device(P);
  if (rc) return rc;
  size_t wbl_at;
  const size_t bytes = table_bytes(P, &wbl_at);
  if (bytes > P->stage_cap) {
    if (P->h_stage) (void)hipHostFree(P->h_stage), P->h_stage = nullptr;
    const size_t cap = std::max(bytes, 2 * P->stage_cap);
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&P->h_stage), cap);
    if (e != hipSuccess) return hip_fail(e, "plan staging");
    P->stage_cap = cap;
  }
  std::memcpy(P->h_stage, P->jobs.data(), sizeof(JobDev) * P->jobs.size());
  if (!P->wbl.empty()) std::memcpy(P->h_stage + wbl_at, P->wbl.data(), sizeof(WinBlock) * P->wbl.size());
  hipError_t e = hipMemcpyAsync(P->d_mem, P->h_stage, bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(P->staged, s);
  if (e != hipSuccess) return hip_fail(e, "plan upload");
  P->dev_out.resize(P->jobs.size());
  for (size_t j = 0; j < P->jobs.size(); ++j) P->dev_out[j] = P->jobs[j].out;
  if (P->graph) (void)hipGraphExecDestroy(P->graph), P->graph = nullptr;  // tables changed
  if (!P->copy_grid || P->copy_grid == 1) device_setup(P);
  return AX_OK;
}

uint64_t plan_workspace_for(const aceapex_decoder* d, uint64_t max_blocks, uint64_t max_tokens) {
  Plan P;
  P.max_items = uint32_t(max_blocks);
  P.max_tok = uint32_t(max_tokens);
  P.slot_b = d->info.block_size;
  P.off_cap = uint32_t((10 * (d->info.block_size / d->info.min_match + 1) + 15) & ~15u);
  P.len_cap = 3 * d->info.block_size;
  return make_layout(P).total;
}

void plan_copy_options(Plan* dst, const Plan* src) { dst->opt = src->opt; }

int plan_set_slots(Plan* P, uint32_t* slot, hipStream_t s) {
  if (P->wins.size() > 1) return fail(AX_E_CAPACITY, "a mapped plan holds one window");
  if (P->wins.empty()) return AX_OK;
  const uint32_t n = P->wins[0].items;
  hipLaunchKernelGGL(k_slots, dim3((n + 255) / 256), dim3(256), 0, s, slot, P->d_wbl, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? AX_OK : hip_fail(e, "slot table");
}
void plan_set_learn(Plan* P, bool learn) { P->learn = learn; }

int plan_parse_tokens(Plan* P, void* d_work, uint64_t work_len, hipStream_t s, uint64_t* src, uint64_t* dstlen) {
  if (work_len < P->lay.total) return fail(AX_E_CAPACITY, "workspace too small");
  uint8_t* w = static_cast<uint8_t*>(d_work);
  const Layout& L = P->lay;
  DevStatus* st = reinterpret_cast<DevStatus*>(w + L.status);
  bool stale = false;
  for (size_t j = 0; j < P->jobs.size(); ++j) stale |= P->dev_out[j] != P->jobs[j].out;
  if (stale) {
    hipError_t e = hipMemcpy(P->d_jobs, P->jobs.data(), sizeof(JobDev) * P->jobs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "job table update");
    for (size_t j = 0; j < P->jobs.size(); ++j) P->dev_out[j] = P->jobs[j].out;
  }
  std::vector<uint64_t> tk;
  if (P->wins.empty()) hipLaunchKernelGGL(k_window_init, dim3(1), dim3(64), 0, s, st, 1);  // status only
  for (const Plan::Win& W : P->wins) {
    const WinBlock* wbl = P->d_wbl + W.at;
    hipLaunchKernelGGL(k_window_init, dim3(1), dim3(64), 0, s, st, int(&W == &P->wins.front()));
    AnsArgs aa{P->d_jobs, wbl, W.items, P->slot_b, w + L.lit, w + L.cmd, w + L.off, w + L.len, P->off_cap,
               P->len_cap, reinterpret_cast<uint32_t*>(w + L.nsym), st};
    hipLaunchKernelGGL(k_ans, dim3(4 * W.items), dim3(64), 0, s, aa);
    ParseArgs pa{P->d_jobs, wbl, W.items, W.tok, P->slot_b, w + L.lit, w + L.cmd, w + L.off, w + L.len, P->off_cap,
                 P->len_cap, reinterpret_cast<const uint32_t*>(w + L.nsym), reinterpret_cast<uint64_t*>(w + L.tok),
                 reinterpret_cast<uint32_t*>(w + L.tblk), w + L.done, st, 0, nullptr};
    hipLaunchKernelGGL((k_parse<OutDirect, false>), dim3(W.items), dim3(kParseThreads), 0, s, pa);
    try {
      tk.resize(2ull * W.tok);
    } catch (const std::bad_alloc&) {
      return fail(AX_E_NOMEM, "token staging");
    }
    hipError_t e = W.tok ? hipMemcpyAsync(tk.data(), w + L.tok, 16ull * W.tok, hipMemcpyDeviceToHost, s) : hipSuccess;
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "token copy");
    int32_t err = 0;
    uint64_t bad = 0;
    int rc = workspace_status(d_work, s, &err, &bad);
    if (rc) return rc;
    if (err) return fail(err, "device status during the index build");
    // window tokens are the tokens of its blocks in order
    for (uint32_t i = 0; i < W.items; ++i) {
      const WinBlock& wb = P->wbl[W.at + i];
      const uint32_t end = i + 1 < W.items ? P->wbl[W.at + i + 1].tok : W.tok;
      const uint64_t g0 = P->gtok[W.at + i];
      for (uint32_t t = wb.tok; t < end; ++t) {
        src[g0 + (t - wb.tok)] = tk[2ull * t];
        dstlen[g0 + (t - wb.tok)] = tk[2ull * t + 1];
      }
    }
  }
  return AX_OK;
}
int block_streams(const aceapex_decoder* d, uint64_t first, uint64_t count, void* d_work, uint64_t work_len,
                  hipStream_t s, uint8_t* h_out, uint64_t cap, uint32_t* n_syms) {
  if (count == 0) return AX_OK;
  if (first >= d->info.n_blocks || count > d->info.n_blocks - first || count > kWindowBlocks)
    return fail(AX_E_RANGE, "blocks outside the archive or beyond one window");
  std::vector<uint64_t> bl(count);
  for (uint64_t i = 0; i < count; ++i) bl[i] = first + i;
  Plan* P = nullptr;
  int rc = plan_create({JobSpec{d, nullptr, std::move(bl)}}, &P);
  if (rc) return rc;
  struct Guard {
    Plan* p;
    ~Guard() { delete p; }
  } guard{P};
  if (work_len < P->lay.total) return fail(AX_E_CAPACITY, "workspace too small");
  if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(AX_E_ARG, "workspace must be 256-byte aligned");
  uint8_t* w = static_cast<uint8_t*>(d_work);
  const Layout& L = P->lay;
  DevStatus* st = reinterpret_cast<DevStatus*>(w + L.status);
  const Plan::Win& W = P->wins.front();
  hipLaunchKernelGGL(k_window_init, dim3(1), dim3(64), 0, s, st, 1);
  AnsArgs aa{P->d_jobs, P->d_wbl, W.items, P->slot_b, w + L.lit, w + L.cmd, w + L.off, w + L.len, P->off_cap,
             P->len_cap, reinterpret_cast<uint32_t*>(w + L.nsym), st};
  hipLaunchKernelGGL(k_ans, dim3(4 * W.items), dim3(64), 0, s, aa);
  hipError_t e = hipMemcpyAsync(n_syms, w + L.nsym, 16 * count, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stream counts");
  int32_t err = 0;
  uint64_t bad = 0;
  rc = workspace_status(d_work, s, &err, &bad);
  if (rc) return rc;
  if (err) return fail(err, "device status of the entropy stage");
  // packed: per block LIT, LEN, OFF, CMD (the slot order of the counts)
  const uint64_t at[4] = {L.lit, L.len, L.off, L.cmd};
  const uint64_t stride[4] = {P->slot_b, P->len_cap, P->off_cap, P->slot_b};
  uint64_t need = 0;
  for (uint64_t i = 0; i < 4 * count; ++i) need += n_syms[i];
  if (need > cap) return fail(AX_E_CAPACITY, "host buffer smaller than the streams");
  uint64_t o = 0;
  for (uint64_t i = 0; i < count && e == hipSuccess; ++i)
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      const uint32_t n = n_syms[4 * i + k];
      if (n) e = hipMemcpyAsync(h_out + o, w + at[k] + i * stride[k], n, hipMemcpyDeviceToHost, s);
      o += n;
    }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? AX_OK : hip_fail(e, "stream copy");
}

void plan_destroy(Plan* P) { delete P; }
uint64_t plan_workspace(const Plan* P) { return P->lay.total; }
uint64_t plan_tokens(const Plan* P) { return P->n_tokens; }
uint64_t plan_blocks(const Plan* P) { return P->wbl.size(); }

int plan_set_out(Plan* P, size_t job, uint8_t* out) {
  if (job >= P->jobs.size()) return fail(AX_E_ARG, "job index");
  P->jobs[job].out = out;
  return AX_OK;
}

int plan_set_option(Plan* P, int option, int64_t value) {
  switch (option) {
    case AX_OPT_BULK_ROUNDS:
      if (value < 1 || value > 250) return fail(AX_E_ARG, "bulk rounds must be in [1, 250]");
      P->opt.bulk_rounds = int(value);
      P->bulk_auto = false;
      std::fill(P->wbulk.begin(), P->wbulk.end(), uint8_t(0));
      break;
    case AX_OPT_TAIL_CHUNKS:
      if (value < 1 || value > 64) return fail(AX_E_ARG, "tail chunks must be in [1, 64]");
      P->opt.tail_chunks = int(value);
      break;
    case AX_OPT_ROUND0_TILE:
      if (value < 0 || value > 1) return fail(AX_E_ARG, "round-0 schedule must be 0 or 1");
      P->opt.round0_tile = int(value);
      break;
    case AX_OPT_FILL_ROUNDS:
    case AX_OPT_FILL_TAIL:
      if (value < 0 || value > 1) return fail(AX_E_ARG, "fill mode must be 0 or 1");
      (option == AX_OPT_FILL_ROUNDS ? P->opt.fill_round : P->opt.fill_tail) = int(value);
      break;
    case AX_OPT_GRAPH:
      if (value < 0 || value > 1) return fail(AX_E_ARG, "graph must be 0 or 1");
      P->opt.graph = int(value);
      break;
    case AX_OPT_TAIL_MODE:
      if (value < 0 || value > 1) return fail(AX_E_ARG, "tail mode must be 0 or 1");
      P->opt.tail_mode = int(value);
      break;
    case AX_OPT_JUMP_PASSES:
      if (value < 0 || value > int64_t(kJPasses)) return fail(AX_E_ARG, "jump passes must be in [0, 32]");
      P->opt.jump_passes = int(value);
      break;
    case AX_OPT_RANGE_JUMP_TOKENS:
      if (value < 0 || value > int64_t(kWindowTokens)) return fail(AX_E_ARG, "range jump tokens out of range");
      P->opt.range_jump_tokens = value;
      break;
    default:
      return fail(AX_E_ARG, "unknown option");
  }
  if (P->graph) {  // knobs are baked into a captured graph
    (void)hipGraphExecDestroy(P->graph);
    P->graph = nullptr;
  }
  return AX_OK;
}

int plan_get_option(const Plan* P, int option, int64_t* value) {
  switch (option) {
    case AX_OPT_BULK_ROUNDS: *value = P->opt.bulk_rounds; return AX_OK;
    case AX_OPT_TAIL_CHUNKS: *value = P->opt.tail_chunks; return AX_OK;
    case AX_OPT_ROUND0_TILE: *value = P->opt.round0_tile; return AX_OK;
    case AX_OPT_FILL_ROUNDS: *value = P->opt.fill_round; return AX_OK;
    case AX_OPT_FILL_TAIL: *value = P->opt.fill_tail; return AX_OK;
    case AX_OPT_GRAPH: *value = P->opt.graph; return AX_OK;
    case AX_OPT_TAIL_MODE: *value = P->opt.tail_mode; return AX_OK;
    case AX_OPT_JUMP_PASSES: *value = P->opt.jump_passes; return AX_OK;
    case AX_OPT_RANGE_JUMP_TOKENS: *value = P->opt.range_jump_tokens; return AX_OK;
    default: return fail(AX_E_ARG, "unknown option");
  }
}

// Stage events for every window of the plan (created when timing is on).
static int ensure_events(Plan* P) {
  const size_t need = 5 * P->wins.size();
  while (P->ev.size() < need) {
    hipEvent_t e;
    hipError_t er = hipEventCreate(&e);
    if (er != hipSuccess) return hip_fail(er, "hipEventCreate");
    P->ev.push_back(e);
  }
  return AX_OK;
}

int plan_set_timing(Plan* P, int enable) {
  if (enable && !P->events_ok) {
    int rc = ensure_events(P);
    if (rc) return rc;
    P->events_ok = true;
  }
  P->timing = enable != 0;
  return AX_OK;
}

int plan_stage_ms(Plan* P, float* ans, float* parse, float* copy, float* remainder) {
  if (!P->events_ok || P->timed_windows == 0) return fail(AX_E_ARG, "timing not enabled");
  float t[4] = {0, 0, 0, 0};
  for (size_t wi = 0; wi < P->timed_windows; ++wi) {
    hipEvent_t* e = P->ev.data() + 5 * wi;
    hipError_t er = hipEventSynchronize(e[4]);
    if (er != hipSuccess) return hip_fail(er, "hipEventSynchronize");
    for (int k = 0; k < 4; ++k) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e[k], e[k + 1]);
      t[k] += ms;
    }
  }
  *ans = t[0];
  *parse = t[1];
  *copy = t[2] + t[3];
  if (remainder) *remainder = t[3];
  return AX_OK;
}

// Enqueue the plan's kernels on s (also used inside a graph capture).
template <class O>
static void enqueue_out(Plan* P, uint8_t* w, int copy_mode, hipStream_t s, bool timed, bool feedback) {
  const Layout& L = P->lay;
  DevStatus* st = reinterpret_cast<DevStatus*>(w + L.status);
  if (P->wins.empty()) hipLaunchKernelGGL(k_window_init, dim3(1), dim3(64), 0, s, st, 1);  // status only
  for (size_t wi = 0; wi < P->wins.size(); ++wi) {
    const Plan::Win& W = P->wins[wi];
    const bool first = wi == 0;
    const WinBlock* wbl = P->d_wbl + W.at;
    uint32_t* counts = reinterpret_cast<uint32_t*>(w + L.counts);
    const uint32_t ntok = W.tok;
    const bool jump = P->opt.tail_mode == 0 && copy_mode != AX_COPY_SERIAL;
    const uint32_t n_words = (ntok + 31) / 32;
    const uint64_t mwords = uint64_t(W.items) * (P->slot_b / 64);  // leftover-map words
    // eight listed words per wave step, four waves per workgroup
    const uint32_t jgrid = uint32_t(std::min<uint64_t>((mwords + 31) / 32, kJMaxGrid));
    {
      const bool jmap = jump && ntok;
      const PrepArgs pr{st, int(first), counts, uint32_t((L.jflags - L.counts) / 4 + kJPasses * kJShards * kJFlagStride),
                        reinterpret_cast<uint32_t*>(w + L.pbits), ntok ? n_words : 0u,
                        jmap ? reinterpret_cast<uint64_t*>(w + L.lmap) : nullptr, mwords,
                        reinterpret_cast<uint8_t**>(w + L.ibase), P->d_jobs, wbl, W.items};
      hipLaunchKernelGGL(k_window_prep<O>, dim3(std::max(1u, jgrid)), dim3(kCopyThreads), 0, s, pr);
    }
    AnsArgs aa{P->d_jobs, wbl, W.items, P->slot_b, w + L.lit, w + L.cmd, w + L.off, w + L.len, P->off_cap,
               P->len_cap, reinterpret_cast<uint32_t*>(w + L.nsym), st};
    hipEvent_t* ev = timed ? P->ev.data() + 5 * wi : nullptr;
    if (ev) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_ans, dim3(4 * W.items), dim3(64), 0, s, aa);
    if (ev) (void)hipEventRecord(ev[1], s);
    const int bulk = P->wbulk[wi] ? int(P->wbulk[wi]) : P->opt.bulk_rounds;
    ParseArgs pa{P->d_jobs, wbl, W.items, W.tok, P->slot_b, w + L.lit, w + L.cmd, w + L.off, w + L.len, P->off_cap,
                 P->len_cap, reinterpret_cast<const uint32_t*>(w + L.nsym), reinterpret_cast<uint64_t*>(w + L.tok),
                 reinterpret_cast<uint32_t*>(w + L.tblk), w + L.done, st, 1,
                 bulk <= 1 ? reinterpret_cast<uint16_t*>(w + L.mcov) : nullptr};
    if (pa.mcov) hipLaunchKernelGGL((k_parse<O, true>), dim3(W.items), dim3(kParseThreads), 0, s, pa);
    else hipLaunchKernelGGL((k_parse<O, false>), dim3(W.items), dim3(kParseThreads), 0, s, pa);
    if (ev) (void)hipEventRecord(ev[2], s);
    const int last_mark = jump ? kMarkJump : kMarkList;
    if (ntok) {
      uint32_t* lists[2] = {reinterpret_cast<uint32_t*>(w + L.list0), reinterpret_cast<uint32_t*>(w + L.list1)};
      auto cset = [&](int r) { return counts + (r % 3) * kSub * kCounterStride; };
      const uint32_t pgrid = (n_words + kPackWords - 1) / kPackWords;
      CopyArgs ca{P->d_jobs, wbl, W.items, reinterpret_cast<const uint64_t*>(w + L.tok),
                  reinterpret_cast<const uint32_t*>(w + L.tblk), ntok, reinterpret_cast<uint32_t*>(w + L.cov),
                  w + L.done, nullptr, lists[0], nullptr, cset(0), cset(1), uint32_t(L.sub_cap),
                  reinterpret_cast<uint32_t*>(w + L.llist), &st->long_count, 0, st,
                  reinterpret_cast<uint32_t*>(w + L.pbits), reinterpret_cast<const uint32_t*>(w + L.plist),
                  bulk <= 1 ? last_mark : 0, 1ull << 22, copy_mode == AX_COPY_SERIAL, P->opt.fill_round,
                  P->opt.fill_tail, uint32_t(P->opt.tail_chunks), reinterpret_cast<uint32_t*>(w + L.lit),
                  reinterpret_cast<uint64_t*>(w + L.lmap), P->slot_b, pa.mcov ? reinterpret_cast<const uint64_t*>(w + L.mcov) : nullptr,
                  P->jobs.size() == 1 ? 1u : 0u};
      // pointer jumping over window positions (the deep remainder); the
      // jump array is the stream slots, dead once the parse is through
      JumpArgs ja{P->d_jobs, wbl, W.items, ntok, P->slot_b, ca.tok, ca.tblk, ca.done,
                  reinterpret_cast<uint32_t*>(w + L.lit), reinterpret_cast<uint64_t*>(w + L.lmap),
                  reinterpret_cast<uint64_t*>(w + L.amap), reinterpret_cast<uint32_t*>(w + L.jflags),
                  reinterpret_cast<uint8_t**>(w + L.ibase), uint32_t(__builtin_ctz(P->slot_b)),
                  nullptr, nullptr, uint32_t(L.sub_cap), reinterpret_cast<uint32_t*>(w + L.wlist), st, 0};
      const uint32_t grid = uint32_t(std::min<uint64_t>((ntok + kCopyThreads - 1) / kCopyThreads, kMaxRoundGrid));
      if (P->opt.round0_tile && ca.mcov)
        hipLaunchKernelGGL((k_round0<O, true>), dim3(W.items), dim3(kCopyThreads), 0, s, ca);
      else if (P->opt.round0_tile)
        hipLaunchKernelGGL((k_round0<O, false>), dim3(W.items), dim3(kCopyThreads), 0, s, ca);
      else hipLaunchKernelGGL(k_round0_waves<O>, dim3(grid), dim3(kCopyThreads), 0, s, ca);
      hipLaunchKernelGGL(k_long<O>, dim3(std::min<uint32_t>(grid, 2048)), dim3(kCopyThreads), 0, s, ca);
      if (feedback && bulk > 1) hipLaunchKernelGGL(k_pending0, dim3(1), dim3(64), 0, s, cset(0), st);
      for (int r = 1; r < bulk; ++r) {
        ca.round = uint32_t(r);
        ca.list_in = lists[(r - 1) & 1];
        ca.list_out = lists[r & 1];
        ca.cnt_in = cset(r - 1);
        ca.cnt_out = cset(r);
        ca.cnt_clear = cset(r + 1);
        ca.mark = r + 1 == bulk ? last_mark : 0;
        // later rounds see the previous round's leftovers only
        hipLaunchKernelGGL(k_round<O>, dim3(grid), dim3(kCopyThreads), 0, s, ca);
      }
      ca.round = uint32_t(bulk);
      if (ev) (void)hipEventRecord(ev[3], s);
      if (!jump) {
        uint32_t* pcnt = reinterpret_cast<uint32_t*>(w + L.pcnt);
        hipLaunchKernelGGL(k_pcount, dim3(pgrid), dim3(kCopyThreads), 0, s, ca.pbits, n_words, pcnt);
        hipLaunchKernelGGL(k_pscatter, dim3(pgrid), dim3(kCopyThreads), 0, s, ca.pbits, n_words, pcnt,
                           reinterpret_cast<uint32_t*>(w + L.plist), st);
      }
      if (jump) {
        // the last round marked the remainder (long tokens are marked here):
        // list the map's busy words, settle the first entries, jump, write
        ja.llist = ca.list_out;  // the last round's output sublists hold the long pending tokens
        ja.lcnt = ca.cnt_out;
        hipLaunchKernelGGL(k_jmarklong<O>, dim3(grid), dim3(kCopyThreads), 0, s, ja);
        const uint32_t lgrid = uint32_t((mwords + kJListWords - 1) / kJListWords);
        hipLaunchKernelGGL(k_jlist, dim3(lgrid), dim3(kCopyThreads), 0, s, ja);
        hipLaunchKernelGGL(k_jinit, dim3(jgrid), dim3(kCopyThreads), 0, s, ja);
        // passes 0 .. used-1 leave no active entry (pass `used` found none);
        // the spare pass that reports it again runs only while learning
        uint32_t passes = P->jsettled && P->jneed[wi] ? std::min(P->jpass[wi], P->jneed[wi]) : P->jpass[wi];
        if (P->opt.jump_passes) passes = std::min<uint32_t>(passes, P->opt.jump_passes);
        for (uint32_t p = 0; p < passes; ++p) {
          ja.pass = p;
          hipLaunchKernelGGL(k_jpass, dim3(jgrid), dim3(kCopyThreads), 0, s, ja);
        }
        hipLaunchKernelGGL(k_jgather, dim3(jgrid), dim3(kCopyThreads), 0, s, ja);
        if (feedback) (void)hipMemcpyAsync(P->h_jused + 2 * wi, &st->jump_used, 4, hipMemcpyDeviceToHost, s);
      } else {
        const uint64_t waves = (ntok + 64ull * P->opt.tail_chunks - 1) / (64ull * P->opt.tail_chunks);
        const uint32_t tgrid = uint32_t(std::min<uint64_t>((waves + 3) / 4, uint64_t(P->copy_grid)));
        hipLaunchKernelGGL(k_tail<O>, dim3(tgrid), dim3(kCopyThreads), 0, s, ca);
      }
      if (feedback) (void)hipMemcpyAsync(P->h_jused + 2 * wi + 1, &st->pend0, 4, hipMemcpyDeviceToHost, s);
    }
    if (ev && !ntok) (void)hipEventRecord(ev[3], s);
    if (ev) (void)hipEventRecord(ev[4], s);
  }
}

// The launch sequence for the plan's output addressing.
static void enqueue(Plan* P, uint8_t* w, int copy_mode, hipStream_t s, bool timed, bool feedback) {
  if (P->mapped) enqueue_out<OutMapped>(P, w, copy_mode, s, timed, feedback);
  else enqueue_out<OutDirect>(P, w, copy_mode, s, timed, feedback);
}

// A decode: checks, then the launch sequence on s.  no_alloc: no graph and no
// stage timing (both may create runtime objects); everything else a decode
// uses was allocated with the plan.
static int run_plan(Plan* P, void* d_work, uint64_t work_len, int copy_mode, hipStream_t s, bool no_alloc) {
  if (!d_work) return fail(AX_E_ARG, "null workspace");
  if (work_len < P->lay.total) return fail(AX_E_CAPACITY, "workspace too small");
  if (reinterpret_cast<uintptr_t>(d_work) & 255) return fail(AX_E_ARG, "workspace must be 256-byte aligned");
  if (copy_mode != AX_COPY_PERIODIC && copy_mode != AX_COPY_SERIAL) return fail(AX_E_ARG, "bad copy mode");
  for (size_t j = 0; j < P->jobs.size(); ++j) {
    if (!P->jobs[j].out && P->jobs[j].n_bytes) return fail(AX_E_ARG, "job without an output buffer");
    if (reinterpret_cast<uintptr_t>(P->jobs[j].out) & 15) return fail(AX_E_ARG, "outputs must be 16-byte aligned");
  }
  // refresh output pointers that changed since the last upload
  bool stale = false;
  for (size_t j = 0; j < P->jobs.size(); ++j) stale |= P->dev_out[j] != P->jobs[j].out;
  if (stale) {
    if (P->staged) (void)hipEventSynchronize(P->staged);  // h_pinned may feed the previous update
    std::memcpy(P->h_pinned, P->jobs.data(), sizeof(JobDev) * P->jobs.size());
    hipError_t e = hipMemcpyAsync(P->d_jobs, P->h_pinned, sizeof(JobDev) * P->jobs.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && P->staged) e = hipEventRecord(P->staged, s);
    if (e != hipSuccess) return hip_fail(e, "job table update");
    for (size_t j = 0; j < P->jobs.size(); ++j) P->dev_out[j] = P->jobs[j].out;
  }
  uint8_t* w = static_cast<uint8_t*>(d_work);
  const bool timed = P->timing && P->events_ok;
  // learned bulk-round and jump-pass counts: take the previous decode's
  // report once it is in (a window whose bulk count changes starts its pass
  // count over from the bound)
  if (P->jfeed_pending && hipEventQuery(P->jfed) == hipSuccess) {
    P->jfeed_pending = false;
    bool all = true;
    for (size_t i = 0; i < P->wins.size(); ++i) {
      const uint32_t used = P->h_jused[2 * i], pend0 = P->h_jused[2 * i + 1];
      if (P->bulk_auto && !P->bsettled) {
        const uint8_t b = 10ull * pend0 > 9ull * P->wins[i].tok ? 1 : 0;
        if (b != P->wbulk[i]) {
          P->wbulk[i] = b;
          P->jpass[i] = jump_pass_bound(P->wins[i].tok);
          P->jneed[i] = 0;
          all = false;
          continue;
        }
      }
      if (used) P->jpass[i] = std::min(P->jpass[i], used + 1), P->jneed[i] = used;
      else all = false;
    }
    if (P->bulk_auto) P->bsettled = true;
    P->jsettled = all;
    P->graph_stale = P->graph != nullptr;  // counts changed
  }
  if (P->graph_stale && !no_alloc) (void)hipGraphExecDestroy(P->graph), P->graph = nullptr, P->graph_stale = false;
  const bool fb_jump = !P->jsettled && P->opt.tail_mode == 0 && !P->opt.jump_passes && copy_mode != AX_COPY_SERIAL;
  const bool fb_bulk = P->bulk_auto && !P->bsettled;
  const bool feedback = P->learn && (fb_jump || fb_bulk) && !P->jfeed_pending && !P->wins.empty() &&
                        P->jused_cap >= P->wins.size() && P->jfed;
  if (feedback) std::fill(P->h_jused, P->h_jused + 2 * P->wins.size(), 0u);
  if (P->opt.graph && !timed && !no_alloc) {
    // the launch sequence of every window and round, captured once and replayed
    if (!P->graph || P->graph_work != d_work || P->graph_mode != copy_mode) {
      if (P->graph) (void)hipGraphExecDestroy(P->graph), P->graph = nullptr;
      if (P->graph_def) (void)hipGraphDestroy(P->graph_def), P->graph_def = nullptr;
      if (!P->cap_stream) {
        hipError_t e = hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "capture stream");
      }
      hipError_t e = hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "graph capture");
      enqueue(P, w, copy_mode, P->cap_stream, false, false);
      e = hipStreamEndCapture(P->cap_stream, &P->graph_def);
      if (e == hipSuccess) e = hipGraphInstantiate(&P->graph, P->graph_def, nullptr, nullptr, 0);
      if (e != hipSuccess) return hip_fail(e, "graph instantiate");
      P->graph_work = d_work;
      P->graph_mode = copy_mode;
    }
    hipError_t e = hipGraphLaunch(P->graph, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return AX_OK;
  }
  const bool timed_now = timed && !no_alloc;
  if (timed_now) {
    int rc = ensure_events(P);
    if (rc) return rc;
  }
  enqueue(P, w, copy_mode, s, timed_now, feedback);
  if (timed_now) P->timed_windows = P->wins.size();
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  if (feedback) {
    e = hipEventRecord(P->jfed, s);
    if (e != hipSuccess) return hip_fail(e, "pass report event");
    P->jfeed_pending = true;
  }
  return AX_OK;
}

int plan_run(Plan* P, void* d_work, uint64_t work_len, int copy_mode, hipStream_t s) {
  return run_plan(P, d_work, work_len, copy_mode, s, false);
}
int plan_run_no_alloc(Plan* P, void* d_work, uint64_t work_len, int copy_mode, hipStream_t s) {
  return run_plan(P, d_work, work_len, copy_mode, s, true);
}

int workspace_status(void* d_work, hipStream_t s, int32_t* dev_err, uint64_t* bad_block) {
  DevStatus hs;
  hipError_t e = hipMemcpyAsync(&hs, d_work, sizeof(hs), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "status read");
  *dev_err = hs.err;
  *bad_block = hs.bad_block;
  return AX_OK;
}

}  // namespace ax

// ------------------------------------------------- allocation-free decode --
//
// Workspace of aceapex_decode_all_static: a library-owned device array, so
// that callers that cannot allocate device memory can still decode.  Every
// device the library runs on holds its own copy (at its own address, looked
// up once per device with that device current) until the process ends.  All
// such decodes on one device share it: calls that overlap on one device race.
// The launch sequence initialises every part of a workspace it reads, so the
// contents a previous call left do not matter.
static __device__ __align__(256) uint8_t scratch[AX_STATIC_SCRATCH_BYTES];

namespace {
constexpr uint64_t kStaticScratchBytes = AX_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_at[kMaxDevices] = {};

// Device address of the static scratch on the current device.
int static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return ax::fail(AX_E_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return ax::fail(AX_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return ax::fail(AX_E_HIP, hipGetErrorString(e));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return ax::fail(AX_E_HIP, "static scratch address");
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return AX_OK;
}
}  // namespace

extern "C" {

int aceapex_read_info(const uint8_t* h, uint64_t len, aceapex_info* info) {
  if (!h || !info || len < 64) return ax::fail(AX_E_ARG, "need at least the 64-byte header");
  if (ax::get32(h) != ax::kMagic || ax::get16(h + 4) != 1) return ax::fail(AX_E_CORRUPT, "bad magic or version");
  aceapex_info I{};
  I.flags = ax::get16(h + 6);
  I.block_size = ax::get32(h + 8);
  I.min_match = ax::get16(h + 12);
  I.depth_cap = ax::get16(h + 14);
  I.n_bytes = ax::get64(h + 16);
  I.n_blocks = ax::get64(h + 24);
  I.xxh3 = ax::get64(h + 32);
  I.payload_bytes = ax::get64(h + 40);
  I.n_matches = ax::get64(h + 48);
  const uint32_t B = I.block_size;
  if (B < 4096 || B > 65536 || (B & (B - 1)) || I.min_match < 1 || I.min_match > 255)
    return ax::fail(AX_E_CORRUPT, "bad block size or min_match");
  if (I.n_blocks != (I.n_bytes + B - 1) / B) return ax::fail(AX_E_CORRUPT, "block count mismatch");
  if (I.n_blocks > (1ull << 40)) return ax::fail(AX_E_CORRUPT, "block count too large");
  I.header_bytes = 64 + 16 * (I.n_blocks + 1);
  I.archive_bytes = I.header_bytes + I.payload_bytes;
  if (I.archive_bytes < I.header_bytes) return ax::fail(AX_E_CORRUPT, "size overflow");
  *info = I;
  return AX_OK;
}

int aceapex_decoder_create(const uint8_t* h, uint64_t h_len, const uint8_t* d_arc, uint64_t arc_len,
                           aceapex_decoder** out) {
  if (!out) return ax::fail(AX_E_ARG, "null out");
  *out = nullptr;
  aceapex_info I;
  int rc = aceapex_read_info(h, h_len, &I);
  if (rc) return rc;
  if (h_len < I.header_bytes) return ax::fail(AX_E_ARG, "host copy shorter than header + index");
  if (!d_arc || arc_len < I.archive_bytes) return ax::fail(AX_E_ARG, "device archive shorter than the header says");
  if (I.block_size > kMaxB) return ax::fail(AX_E_UNSUPPORTED, "device decoder takes blocks up to 16384 bytes");
  aceapex_decoder* d = new (std::nothrow) aceapex_decoder;
  if (!d) return ax::fail(AX_E_NOMEM, "decoder handle");
  d->info = I;
  d->d_arc = d_arc;
  d->arc_len = arc_len;
  const uint64_t nb = I.n_blocks, B = I.block_size;
  try {
    d->offs.resize(nb + 1);
    d->mpre.resize(nb + 1);
  } catch (const std::bad_alloc&) {
    delete d;
    return ax::fail(AX_E_NOMEM, "index copy");
  }
  const uint8_t* ix = h + 64;
  for (uint64_t b = 0; b <= nb; ++b) d->offs[b] = ax::get64(ix + 8 * b), d->mpre[b] = ax::get64(ix + 8 * (nb + 1) + 8 * b);
  bool ok = d->offs[0] == 0 && d->offs[nb] == I.payload_bytes && d->mpre[0] == 0 && d->mpre[nb] == I.n_matches;
  const uint64_t max_tok = B / I.min_match;
  for (uint64_t b = 0; b < nb && ok; ++b) {
    ok &= d->offs[b + 1] >= d->offs[b] + 16 && ((d->offs[b + 1] - d->offs[b]) & 15) == 0;
    ok &= d->mpre[b + 1] >= d->mpre[b] && d->mpre[b + 1] - d->mpre[b] <= max_tok;
  }
  if (!ok) {
    delete d;
    return ax::fail(AX_E_CORRUPT, "bad index");
  }
  rc = ax::plan_create({ax::JobSpec{d, nullptr, {}}}, &d->plan);
  if (rc) {
    delete d;
    return rc;
  }
  *out = d;
  return AX_OK;
}

void aceapex_decoder_destroy(aceapex_decoder* d) {
  if (!d) return;
  aceapex_range_plan_destroy(d->range);
  ax::plan_destroy(d->plan);
  delete d;
}

int aceapex_decoder_info(const aceapex_decoder* d, aceapex_info* info) {
  if (!d || !info) return ax::fail(AX_E_ARG, "null argument");
  *info = d->info;
  return AX_OK;
}

int aceapex_decoder_workspace(const aceapex_decoder* d, uint64_t* bytes) {
  if (!d || !bytes) return ax::fail(AX_E_ARG, "null argument");
  *bytes = ax::plan_workspace(d->plan);
  return AX_OK;
}

int aceapex_decoder_set_timing(aceapex_decoder* d, int enable) {
  if (!d) return ax::fail(AX_E_ARG, "null decoder");
  return ax::plan_set_timing(d->plan, enable);
}

int aceapex_decoder_set_option(aceapex_decoder* d, int option, int64_t value) {
  if (!d) return ax::fail(AX_E_ARG, "null decoder");
  return ax::plan_set_option(d->plan, option, value);
}

int aceapex_decoder_stage_ms(aceapex_decoder* d, float* ans, float* parse, float* copy, float* remainder) {
  if (!d || !ans || !parse || !copy) return ax::fail(AX_E_ARG, "null argument");
  return ax::plan_stage_ms(d->plan, ans, parse, copy, remainder);
}

int aceapex_decode_all(aceapex_decoder* d, uint8_t* d_out, uint64_t out_cap, void* d_work, uint64_t work_len,
                       int copy_mode, void* stream) {
  if (!d || (!d_out && d->info.n_bytes) || !d_work) return ax::fail(AX_E_ARG, "null argument");
  if (out_cap < d->info.n_bytes) return ax::fail(AX_E_CAPACITY, "output smaller than the decoded size");
  ax::plan_set_out(d->plan, 0, d_out);
  return ax::plan_run(d->plan, d_work, work_len, copy_mode, reinterpret_cast<hipStream_t>(stream));
}

int aceapex_decode_all_static(aceapex_decoder* d, uint8_t* d_out, uint64_t out_cap, int copy_mode, void* stream) {
  if (!d || (!d_out && d->info.n_bytes)) return ax::fail(AX_E_ARG, "null argument");
  if (out_cap < d->info.n_bytes) return ax::fail(AX_E_CAPACITY, "output smaller than the decoded size");
  if (ax::plan_workspace(d->plan) > kStaticScratchBytes)
    return ax::fail(AX_E_CAPACITY, "the archive needs more workspace than the static scratch holds");
  void* w = nullptr;
  int rc = static_scratch(&w);
  if (rc) return rc;
  ax::plan_set_out(d->plan, 0, d_out);
  return ax::plan_run_no_alloc(d->plan, w, kStaticScratchBytes, copy_mode, reinterpret_cast<hipStream_t>(stream));
}

int aceapex_decoder_streams(aceapex_decoder* d, uint64_t first, uint64_t count, void* d_work, uint64_t work_len,
                            void* stream, uint8_t* h_out, uint64_t cap, uint32_t* n_syms) {
  if (!d || (count && (!d_work || !n_syms || (!h_out && cap)))) return ax::fail(AX_E_ARG, "null argument");
  return ax::block_streams(d, first, count, d_work, work_len, reinterpret_cast<hipStream_t>(stream), h_out, cap,
                           n_syms);
}

int aceapex_decoder_status(aceapex_decoder* d, void* d_work, void* stream, int32_t* dev_err, uint64_t* bad_block) {
  if (!d || !dev_err || !bad_block) return ax::fail(AX_E_ARG, "null argument");
  if (!d_work) {  // the static scratch of aceapex_decode_all_static on the current device
    int rc = static_scratch(&d_work);
    if (rc) return rc;
  }
  return ax::workspace_status(d_work, reinterpret_cast<hipStream_t>(stream), dev_err, bad_block);
}

int aceapex_workspace_status(void* d_work, void* stream, int32_t* dev_err, uint64_t* bad_block) {
  if (!d_work || !dev_err || !bad_block) return ax::fail(AX_E_ARG, "null argument");
  return ax::workspace_status(d_work, reinterpret_cast<hipStream_t>(stream), dev_err, bad_block);
}

// ------------------------------------------------------------------ batch --

struct aceapex_batch {
  ax::Plan* plan = nullptr;
};

int aceapex_batch_create(const aceapex_job* jobs, uint32_t n, aceapex_batch** out) {
  if (!out || (!jobs && n)) return ax::fail(AX_E_ARG, "null argument");
  *out = nullptr;
  std::vector<ax::JobSpec> specs;
  try {
    specs.reserve(n);
    for (uint32_t i = 0; i < n; ++i) {
      if (!jobs[i].dec) return ax::fail(AX_E_ARG, "job without a decoder");
      if (jobs[i].out_cap < jobs[i].dec->info.n_bytes) return ax::fail(AX_E_CAPACITY, "job output too small");
      specs.push_back(ax::JobSpec{jobs[i].dec, jobs[i].d_out, {}});
    }
  } catch (const std::bad_alloc&) {
    return ax::fail(AX_E_NOMEM, "batch jobs");
  }
  aceapex_batch* bt = new (std::nothrow) aceapex_batch;
  if (!bt) return ax::fail(AX_E_NOMEM, "batch handle");
  int rc = ax::plan_create(specs, &bt->plan);
  if (rc) {
    delete bt;
    return rc;
  }
  *out = bt;
  return AX_OK;
}

void aceapex_batch_destroy(aceapex_batch* bt) {
  if (!bt) return;
  ax::plan_destroy(bt->plan);
  delete bt;
}

int aceapex_batch_workspace(const aceapex_batch* bt, uint64_t* bytes) {
  if (!bt || !bytes) return ax::fail(AX_E_ARG, "null argument");
  *bytes = ax::plan_workspace(bt->plan);
  return AX_OK;
}

int aceapex_batch_set_option(aceapex_batch* bt, int option, int64_t value) {
  if (!bt) return ax::fail(AX_E_ARG, "null batch");
  return ax::plan_set_option(bt->plan, option, value);
}

int aceapex_batch_set_timing(aceapex_batch* bt, int enable) {
  if (!bt) return ax::fail(AX_E_ARG, "null batch");
  return ax::plan_set_timing(bt->plan, enable);
}

int aceapex_batch_stage_ms(aceapex_batch* bt, float* ans, float* parse, float* copy, float* remainder) {
  if (!bt || !ans || !parse || !copy) return ax::fail(AX_E_ARG, "null argument");
  return ax::plan_stage_ms(bt->plan, ans, parse, copy, remainder);
}

int aceapex_decode_batch(aceapex_batch* bt, void* d_work, uint64_t work_len, int copy_mode, void* stream) {
  if (!bt) return ax::fail(AX_E_ARG, "null batch");
  return ax::plan_run(bt->plan, d_work, work_len, copy_mode, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
