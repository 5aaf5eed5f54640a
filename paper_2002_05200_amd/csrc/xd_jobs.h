// xd_jobs.h -- job descriptors exchanged between the host planner and the
// gfx950 kernels (library-internal; not part of the C ABI).
#pragma once

#include <stdint.h>

namespace xd {

constexpr int32_t kNeg = -(1 << 30);       // -inf of the band (never wins a max)
constexpr int kWaveSlots = 64;             // lanes of a wavefront
constexpr int kTiers = 6;                  // cells per lane 1, 2, 4, 8, 16, 32
constexpr int kSpillTier = kTiers;         // unbounded global-memory band

// One one-directional extension (Section IV-B seed split): a_i = A[a_start +
// dir * (i - 1)], b_j = B[b_start + dir * (j - 1)], 1 <= i <= m, 1 <= j <= n.
struct Job {
  int64_t a_start;
  int64_t b_start;
  int32_t m, n;
  int32_t x;
  int32_t dir;   // +1: right extension (forward), -1: left extension (backward)
};

// Job status values (internal).
enum : int32_t { kJobOk = 0, kJobWider = 100 };

// A finished job's result.  With status kJobWider (the band outgrew the
// window) bi is 1 when the state was saved for the next tier, 0 when the job
// starts over there, and cells holds the cells computed so far.
struct JobOut {
  int32_t best, bi, bj, status;
  uint64_t cells;
};

// Everything one launch needs besides the job list.  With g = gap,
// base = mismatch - 2g and delta = match - mismatch, the diagonal term of the
// gap-free form is W_{d-2} + base + (match ? delta : 0).
struct Params {
  const uint32_t *A;
  const uint32_t *B;
  int64_t a_words, b_words;
  int32_t neg_gap;   // -gap: growth of the W-form thresholds per anti-diagonal
  int32_t base;      // mismatch - 2 gap
  int32_t delta;     // match - mismatch (>= 0)
  int32_t pat;       // delta replicated into every 2-bit field (narrow form)
  int32_t fold;      // +1/-1/-1: base (1) in every field as well (0x55555555), else 0
  int32_t dbase;     // what the diagonal term adds to the field: base, or 0 when folded
  int32_t impl;      // 0: hand-scheduled loops where available, 1: C loops only
  int32_t unit_match;  // match == 1: best grows by exactly 1 when it grows
  // Escalation saves: a job whose band outgrows its window stores its state
  // in a bump-allocated pool so the next tier resumes instead of restarting.
  int32_t *save_pool;              // nullptr: escalated jobs restart
  unsigned long long save_cap;     // pool size in save slots
  unsigned long long *save_top;    // next free slot (cleared per call)
  int32_t *job_save;               // per job: word offset of its slot, or -1
  // Substitution table (xdrop_extend_matrix): lut[4 p + q] scores base p of
  // A against base q of B; has_lut = 0 for match/mismatch scoring.
  int32_t has_lut;
  int32_t lut[16];
  // Persistent tiers: the first prio_jobs jobs a tier hands out (its longest)
  // run at raised wavefront priority; 0 = none.
  int32_t prio_jobs;
};

// Layout of one save: a header, then the W values of the latest even and odd
// anti-diagonals in slot order (S = 64 * C slots each).
enum : int32_t {
  kSvD = 0, kSvLo, kSvHi, kSvH, kSvBest, kSvBi, kSvBj, kSvBw, kSvThr, kSvC, kSvCellsLo,
  kSvCellsHi, kSaveHdr = 16
};
// One save slot holds the widest single-wave band (C = 32); a job keeps its
// slot for all its escalations.
constexpr int32_t kSaveSlotWords = kSaveHdr + 2 * 64 * 32;

}  // namespace xd
