// Internal interface between the decoder engine (decoder.hip) and the host
// pieces built on it (range decode and serving).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "aceapex.h"

namespace ax {

struct Plan;

// Schedule knobs of a plan; none changes a decoded byte.
struct PlanOptions {
  int bulk_rounds = 4;  // level-synchronous match-layer rounds before the persistent launch
  int fill_round = 0;   // rounds after the first: lane/wave fill
  int fill_tail = 0;    // persistent launch: lane/wave fill
  int tail_chunks = 1;  // 64-token chunks per persistent-launch ticket
  int round0_tile = 1;  // round 0: a workgroup per block through an LDS tile (1) or a wave per 64 tokens (0)
  int graph = 0;        // replay the launch sequence from a captured hipGraph
  int tail_mode = 0;    // deep remainder: pointer jumping (0) or the persistent chase (1)
  int jump_passes = 0;  // at most this many jump passes per window (0: automatic)
  int64_t range_jump_tokens = 4096;  // range decodes: closures of at least this many matches jump
};

// One archive to decode: all blocks (blocks empty) or the listed blocks
// (ascending).  Its bytes land in out at their absolute positions, or, when
// slot is set (a plan of one job and one window), block b's bytes at
// out + slot[b] * B with the listed blocks in slots 0, 1, ... (plan_set_slots
// writes those entries) and any slot >= junk meaning the junk block.
struct JobSpec {
  const aceapex_decoder* dec;
  uint8_t* out;
  std::vector<uint64_t> blocks;
  uint32_t* slot = nullptr;
  uint32_t junk = 0;
};

// Window limits: a window's workspace is about 130 KiB per block plus 45 B per
// token (about 18 GiB at these limits, sized to the blocks a plan actually
// holds), so a batch of many archives runs in few windows.
constexpr uint32_t kWindowBlocks = 131072;
constexpr uint64_t kWindowTokens = uint64_t(1) << 26;

int plan_create(const std::vector<JobSpec>& jobs, Plan** out);
// Rebuild an existing plan for new jobs, reusing its device tables (grown
// only when too small); the upload is asynchronous on s.
int plan_reset(Plan* p, const std::vector<JobSpec>& jobs, hipStream_t s);
// Workspace of a one-window plan of decoder d with these maxima.
uint64_t plan_workspace_for(const aceapex_decoder* d, uint64_t max_blocks, uint64_t max_tokens);
void plan_copy_options(Plan* dst, const Plan* src);
// Enqueue the slot-table entries of a mapped plan's blocks on s.
int plan_set_slots(Plan* p, uint32_t* slot, hipStream_t s);
// Whether a plan learns its jump-pass counts from its own decodes (on by
// default; off for plans rebuilt for every call).
void plan_set_learn(Plan* p, bool learn);
// Entropy + parse only, every window, writing no output bytes; the match
// tokens (src; dst | (len-1) << 48) are copied to host arrays in archive
// order.  Synchronous.
int plan_parse_tokens(Plan* p, void* d_work, uint64_t work_len, hipStream_t s, uint64_t* src, uint64_t* dstlen);
// The entropy stage alone for archive blocks [first, first + count) (one
// window): their four decoded streams copied to h_out packed block after
// block (LIT, LEN, OFF, CMD), n_syms[4 i + k] their lengths.  Synchronous.
int block_streams(const aceapex_decoder* d, uint64_t first, uint64_t count, void* d_work, uint64_t work_len,
                  hipStream_t s, uint8_t* h_out, uint64_t cap, uint32_t* n_syms);
void plan_destroy(Plan* p);
uint64_t plan_workspace(const Plan* p);
uint64_t plan_tokens(const Plan* p);
uint64_t plan_blocks(const Plan* p);
int plan_set_out(Plan* p, size_t job, uint8_t* out);
int plan_set_option(Plan* p, int option, int64_t value);
int plan_get_option(const Plan* p, int option, int64_t* value);
int plan_set_timing(Plan* p, int enable);
int plan_stage_ms(Plan* p, float* ans, float* parse, float* copy, float* remainder);
int plan_run(Plan* p, void* d_work, uint64_t work_len, int copy_mode, hipStream_t s);
// the same, creating nothing: no graph, no stage timing
int plan_run_no_alloc(Plan* p, void* d_work, uint64_t work_len, int copy_mode, hipStream_t s);
int workspace_status(void* d_work, hipStream_t s, int32_t* dev_err, uint64_t* bad_block);

}  // namespace ax

namespace ax {
struct RangeKey {
  uint64_t off, len;
  bool operator==(const RangeKey& o) const { return off == o.off && len == o.len; }
};
struct RangeKeyHash {
  size_t operator()(const RangeKey& k) const { return size_t(k.off * 0x9E3779B97F4A7C15ull ^ (k.len + (k.off >> 29))); }
};
}  // namespace ax

// The decoder handle: a host copy of the archive's header and index, the
// device archive, and the plan of a whole-archive decode.
struct aceapex_decoder {
  aceapex_info info{};
  std::vector<uint64_t> offs, mpre;  // payload offsets and cumulative match counts per block
  const uint8_t* d_arc = nullptr;
  uint64_t arc_len = 0;
  ax::Plan* plan = nullptr;
  std::vector<uint64_t> idx_src, idx_dstlen;  // token index (aceapex_decoder_build_index)
  aceapex_range_plan* range = nullptr;        // aceapex_decode_range's plan (created on first use)
  // closures of single ranges already found (ascending blocks), so that a
  // batch's union does not walk again what admission walked; bounded
  mutable std::mutex ccache_mu;
  mutable std::unordered_map<ax::RangeKey, std::vector<uint64_t>, ax::RangeKeyHash> ccache;
  mutable uint64_t ccache_blocks = 0;
};
