// xd_queue.h -- per-tier work queues on the device (library-internal).
//
// All jobs are ordered once by (tier, estimated anti-diagonals descending),
// the latter in logarithmic cost buckets (four per octave), by a counting
// sort.  Tier t works through its segment of that order, then through the
// jobs escalated into it from tier t - 1 (their band outgrew the narrower
// window), those ordered by the anti-diagonals they have left.
#pragma once

#include <hip/hip_runtime.h>

#include "xd_jobs.h"

namespace xd {

constexpr int kLists = kTiers + 1;          // register tiers + global-memory tier

// Device counters (int32): initial jobs per tier, jobs escalated into each
// tier, queue heads, segment offsets in the sorted order.
constexpr int kInit = 0, kEsc = kLists, kHead = 2 * kLists, kOff = 3 * kLists;
// the spill tier's second pass: jobs moved to it and its queue head
constexpr int kHugeCount = 4 * kLists, kHugeHead = 4 * kLists + 1;
constexpr int kCounters = 4 * kLists + 2;
// Device statistics (uint64): jobs finished, cells of those jobs, escalations;
// the bump pointer of the escalation save pool; escalations that found no
// save slot (the job starts over in the next tier) and the cells they had
// computed.
constexpr int kSaveTop = 3 * kLists;
constexpr int kRestart = 3 * kLists + 1;
constexpr int kWasted = 4 * kLists + 1;
constexpr int kStats = 5 * kLists + 1;

// Counting-sort bins: kCostBuckets per tier, longest jobs in the lowest bin.
constexpr int kCostBuckets = 128;
constexpr int kBins = kLists * kCostBuckets;

// Bucket of an estimated cost (anti-diagonals): exact below 8, then four
// buckets per power of two.  At most 4 * 29 + 3 for costs below 2^31.
__device__ __forceinline__ int cost_bucket(uint32_t cost) {
  if (cost < 8u) return (int)cost;
  const int lg = 31 - __builtin_clz(cost);
  return 4 * (lg - 1) + (int)((cost >> (lg - 2)) & 3u);
}


// Job of work item w of a tier: its segment of the sorted order, then the
// jobs escalated into it; -1 past the end.
struct TierQueue {
  const int32_t *order;    // all jobs, sorted by (tier, longest first)
  const int32_t *esc;      // jobs escalated into this tier
  const int32_t *counters;
  int32_t *next_esc;       // escalations out of this tier
  int tier;
};

__device__ __forceinline__ int32_t tier_job(const TierQueue &q, int32_t w, int32_t n_init,
                                            int32_t n_esc) {
  if (w < n_init) return q.order[q.counters[kOff + q.tier] + w];
  if (w < n_init + n_esc) return q.esc[w - n_init];
  return -1;
}

}  // namespace xd
