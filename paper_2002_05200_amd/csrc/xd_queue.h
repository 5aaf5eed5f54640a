// xd_queue.h -- per-tier work queues on the device (library-internal).
//
// All jobs are sorted once by (tier, estimated anti-diagonals descending).
// Tier t works through its segment of that order, then through the jobs
// escalated into it from tier t - 1 (their band outgrew the narrower window).
#pragma once

#include <hip/hip_runtime.h>

#include "xd_jobs.h"

namespace xd {

constexpr int kLists = kTiers + 1;          // register tiers + global-memory tier

// Device counters (int32): initial jobs per tier, jobs escalated into each
// tier, queue heads, segment offsets in the sorted order.
constexpr int kInit = 0, kEsc = kLists, kHead = 2 * kLists, kOff = 3 * kLists;
constexpr int kCounters = 4 * kLists;
// Device statistics (uint64): jobs finished, cells of those jobs, escalations.
constexpr int kStats = 3 * kLists;
constexpr int kKeyBits = 43;   // tier in bits 40..42, inverted cost in 0..39


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
