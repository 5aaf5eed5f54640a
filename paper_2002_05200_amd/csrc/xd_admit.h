// xd_admit.h -- the serving loop's admission arithmetic, as plain host code
// with no HIP calls (so it can be built and tested on a machine without a
// GPU): how a slot's share of the device-memory budget is split, which cost
// class a request falls in, and which queued requests a free slot admits.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "xdrop.h"

namespace xd {

// Device memory of one slot, all inside its share of the server's budget:
// the extension context (job lists, band buffers, escalation saves; its own
// budget is half the share), the pair records and results of one batch, and
// the two packed read arenas, which get what remains.
struct SlotPlan {
  uint64_t ctx_budget;   // budget the slot's context is created with
  uint64_t pair_bytes;   // xd_pair + xd_result records of a full batch
  uint64_t cap_words;    // words of each of the two read arenas
};

// ctx_bytes: what the context holds once sized for a full batch (at most
// ctx_budget).  Returns false when nothing is left for the arenas.
inline bool plan_slot(uint64_t share, int32_t max_batch_pairs, uint64_t ctx_bytes,
                      SlotPlan *out) {
  out->ctx_budget = share / 2;
  out->pair_bytes = (uint64_t)max_batch_pairs * (sizeof(xd_pair) + sizeof(xd_result));
  out->cap_words = 0;
  if (ctx_bytes > out->ctx_budget) return false;
  const uint64_t used = ctx_bytes + out->pair_bytes;
  if (share <= used + 64) return false;
  out->cap_words = (share - used) / 8;   // two arenas of 4-byte words
  return true;
}

// Cost class of a request: the tier its X selects (one register for X up to
// 60, wider above) and the octave of its longest pair (a + b bases).  A
// batch runs as long as its longest job's chain of anti-diagonals, about
// a + b of its longest pair, in the tier its X needs; batching requests of
// one class keeps a short request from waiting for a long one.
inline int32_t cost_class(const xd_pair *pairs, uint32_t n) {
  uint64_t longest = 1;
  int32_t x = 0;
  for (uint32_t p = 0; p < n; ++p) {
    const uint64_t l = (uint64_t)pairs[p].a_len + pairs[p].b_len;
    if (l > longest) longest = l;
    if (pairs[p].x > x) x = pairs[p].x;
  }
  int32_t octave = 0;
  while ((longest >> octave) > 1 && octave < 40) ++octave;
  const int32_t wide = x > 60 ? 1 : 0;
  return wide * 64 + octave;
}

// One queued request as admission sees it.
struct AdmitItem {
  uint64_t a_words, b_words;
  uint32_t n_pairs;
  xd_scores scores;
  int32_t cls;
};

inline bool same_scores(const xd_scores &u, const xd_scores &v) {
  return u.match == v.match && u.mismatch == v.mismatch && u.gap == v.gap;
}

// Which queued requests a free slot takes, as indices into `queue` (oldest
// first): the oldest request, then -- scanning at most `scan` requests --
// every later one of the same score set and, with by_class, the same cost
// class, while the batch's reads fit in the arenas and its pairs in the
// batch.  Requests passed over keep their places.  The oldest request always
// fits (submission rejects requests larger than a slot).
inline void admit(const AdmitItem *queue, size_t n, uint64_t cap_words, int64_t cap_pairs,
                  bool by_class, size_t scan, std::vector<size_t> *take) {
  take->clear();
  if (n == 0) return;
  const AdmitItem &head = queue[0];
  uint64_t a = 0, b = 0;
  int64_t np = 0;
  const size_t end = n < scan ? n : scan;
  for (size_t i = 0; i < end; ++i) {
    const AdmitItem &r = queue[i];
    if (!same_scores(r.scores, head.scores)) continue;
    if (by_class && r.cls != head.cls) continue;
    if (a + r.a_words > cap_words || b + r.b_words > cap_words ||
        np + (int64_t)r.n_pairs > cap_pairs) {
      if (i == 0) return;   // cannot happen for a request submission accepted
      continue;             // a smaller later request may still fit
    }
    a += r.a_words;
    b += r.b_words;
    np += r.n_pairs;
    take->push_back(i);
    if (np == cap_pairs) break;
  }
}

}  // namespace xd
