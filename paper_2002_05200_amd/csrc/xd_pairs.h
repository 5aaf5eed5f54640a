// xd_pairs.h -- per-pair planning and combining (Section IV-B seed split).
//
// A pair with seed A[a_seed, a_seed+k) ~ B[b_seed, b_seed+k) becomes
//   left job : the reversed prefixes, a_i = A[a_seed - i], b_j = B[b_seed - j]
//   right job: the suffixes,          a_i = A[a_seed + k + i - 1], ...
// and its result is left best + seed score + right best, spanning
// A[a_seed - left.bi, a_seed + k + right.bi) and likewise for B.
#pragma once

#include "xdrop.h"
#include "xd_jobs.h"
#include "xd_wave.h"

namespace xd {

// Largest accepted X and score-range guard: every W value of the gap-free
// form stays below 2^30 in magnitude, so int32 arithmetic is exact.
constexpr int64_t kMaxX = int64_t(1) << 29;
constexpr int64_t kGuard = int64_t(1) << 29;

XD_HD inline int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

// Validates one pair and writes its two jobs (left at *left, right at
// *right).  Returns the pair's xd_status; an invalid pair gets two empty jobs.
XD_HD inline int32_t plan_pair(const xd_pair &p, int64_t a_words, int64_t b_words,
                               int32_t match, int32_t mismatch, int32_t gap,
                               Job *left, Job *right) {
  Job empty;
  empty.a_start = 0; empty.b_start = 0; empty.m = 0; empty.n = 0;
  empty.x = 0; empty.dir = 1;
  *left = empty;
  *right = empty;
  const int64_t a_len = p.a_len, b_len = p.b_len, k = p.k;
  if ((int64_t)p.a_seed + k > a_len || (int64_t)p.b_seed + k > b_len) return XD_EINVAL;
  if (p.x < 0 || (int64_t)p.x > kMaxX) return XD_EINVAL;
  if ((int64_t)(p.a_off + p.a_len) > a_words * 16 || (int64_t)(p.b_off + p.b_len) > b_words * 16)
    return XD_EINVAL;
  if (p.a_off > (uint64_t(1) << 60) || p.b_off > (uint64_t(1) << 60)) return XD_EINVAL;
  const int64_t span = iabs64(match) + iabs64(mismatch) + 2 * iabs64(gap);
  if ((a_len + b_len) * span + (int64_t)p.x >= kGuard) return XD_EOVERFLOW;

  left->a_start = (int64_t)p.a_off + (int64_t)p.a_seed - 1;
  left->b_start = (int64_t)p.b_off + (int64_t)p.b_seed - 1;
  left->m = (int32_t)p.a_seed;
  left->n = (int32_t)p.b_seed;
  left->x = p.x;
  left->dir = -1;
  right->a_start = (int64_t)p.a_off + (int64_t)p.a_seed + k;
  right->b_start = (int64_t)p.b_off + (int64_t)p.b_seed + k;
  right->m = (int32_t)(a_len - p.a_seed - k);
  right->n = (int32_t)(b_len - p.b_seed - k);
  right->x = p.x;
  right->dir = 1;
  return XD_OK;
}

XD_HD inline void combine_pair(const xd_pair &p, int32_t status, const JobOut &l,
                               const JobOut &r, int32_t seed_score, xd_result *out) {
  xd_result res;
  res.score = 0; res.left_score = 0; res.right_score = 0; res.seed_score = 0;
  res.a_begin = 0; res.a_end = 0; res.b_begin = 0; res.b_end = 0;
  res.left_cells = 0; res.right_cells = 0; res.reserved = 0;
  res.status = status;
  // a job that no tier could finish reports its own status (XD_ENOMEM when
  // its band is wider than the global-memory tier holds)
  if (status == XD_OK && l.status != kJobOk) res.status = l.status == kJobWider ? XD_EDEVICE : l.status;
  if (res.status == XD_OK && r.status != kJobOk) res.status = r.status == kJobWider ? XD_EDEVICE : r.status;
  if (res.status == XD_OK) {
    res.left_score = l.best;
    res.right_score = r.best;
    res.seed_score = seed_score;
    res.score = l.best + seed_score + r.best;
    res.a_begin = p.a_seed - (uint32_t)l.bi;
    res.a_end = p.a_seed + p.k + (uint32_t)r.bi;
    res.b_begin = p.b_seed - (uint32_t)l.bj;
    res.b_end = p.b_seed + p.k + (uint32_t)r.bj;
    res.left_cells = l.cells;
    res.right_cells = r.cells;
  }
  *out = res;
}

// Initial lane-width tier of a job: the band never exceeds min(m, n) + 1
// cells; X-drop bands with linear gaps are typically about X cells wide.
XD_HD inline int initial_tier(const Job &j) {
  int64_t w = (j.m < j.n ? j.m : j.n) + 1;
  int64_t est = (int64_t)j.x + 4;
  if (est < w) w = est;
  int t = 0;
  while (t < kTiers - 1 && w > (int64_t)kWaveSlots * (1 << t) - 8) ++t;
  return t;
}

}  // namespace xd
