// xd_extend.h -- one X-drop extension per wavefront on gfx950.
//
// What is computed (Section III-A, Algorithms 1 and 2): the anti-diagonal
// dynamic program of the linear-gap recurrence from the origin of an m x n
// matrix, with the running best, pruning of cells below best - X to -inf, the
// next anti-diagonal spanning [first live, last live + 1] clipped to the
// matrix, and the loop ending when nothing survives or d = m + n.
//
// How it is laid out on a wave64 (differs from the paper's one-thread-per-cell
// segments over HBM-resident anti-diagonals):
//
//  * Diagonal-stationary slots.  A cell (i, j) lies on anti-diagonal d = i + j
//    and diagonal k = i - j.  The wave owns S slots; slot s on anti-diagonal
//    d holds the cell with i = s + ceil(d/2) + h (h is the window base, moved
//    only when the band drifts).  Slot s therefore follows one diagonal: its
//    diagonal predecessor (d-2) sits in the same slot, and its up/left
//    predecessors (d-1) sit in slots {s-1, s} for even d and {s, s+1} for odd
//    d.  This file holds the shared pieces and the one-register band (S = 64,
//    lane t = slot t), whose only cross-lane traffic per anti-diagonal is one
//    DPP lane shift; xd_wide.h holds the wider bands.  Nothing of a band
//    lives in LDS or HBM.
//
//  * Gap-free form.  Values are stored as W_d = V_d + d*|gap|.  Then the
//    up/left terms need no add (W_d = max(W_{d-2} + s + 2|gap|, W_{d-1}(nbrs)))
//    and one v_max3_i32 does the whole max; the X-drop threshold and the
//    improvement test move by |gap| per anti-diagonal instead.
//
//  * Score words.  For each slot and parity, 16 consecutive cells of its
//    diagonal get a 2-bit match field precomputed from the 2-bit packed reads
//    with one XOR of two 16-base windows; a cell then costs one v_bfe_u32 +
//    one v_add3_u32 for its diagonal term W_{d-2} + s + 2|gap|.
//
//  * Exact bookkeeping per anti-diagonal in scalar registers: the computed
//    range is a lane mask ANDed with the prune test; the first/last
//    surviving slot give the next range;
//    improvement of best is detected with one compare + ballot, and the best
//    cell (first anti-diagonal reaching the final best, smallest i on it) is
//    taken with one more compare + ballot only when best improves.
#pragma once

#include "xd_jobs.h"
#include "xd_wave.h"

namespace xd {

// The packed reads of one job, addressed relative to its start.
struct SeqView {
  const uint32_t *base;  // words + word_base (never dereferenced out of range)
  int32_t sub;           // start - 16 * word_base
  int32_t lo_rel, hi_rel;  // valid word indices relative to base
};

XD_FN SeqView make_view(const uint32_t *words, int64_t nwords, int64_t start) {
  int64_t wb = (start >> 4) - 2;   // arithmetic shift: floor
  SeqView v;
  v.base = words + wb;
  v.sub = (int32_t)(start - 16 * wb);
  int64_t lo = -wb, hi = nwords - 1 - wb;
  v.lo_rel = (int32_t)(lo < -(1ll << 30) ? -(1ll << 30) : (lo > (1ll << 30) ? (1ll << 30) : lo));
  v.hi_rel = (int32_t)(hi < -(1ll << 30) ? -(1ll << 30) : (hi > (1ll << 30) ? (1ll << 30) : hi));
  return v;
}

// 16 bases starting at (start + off), 2 bits each, base 0 in bits [1:0].
// Positions outside the arena read clamped (garbage) words, never out of
// bounds; such positions only ever feed cells outside the matrix.
XD_FN vint window16(const SeqView &v, vint off) {
  vint g = off + v.sub;
  vint w = shr_s(g, 4);
  vint sh = (g & 15) << 1;
  vint w0 = clamp(w, v.lo_rel, v.hi_rel);
  vint w1 = clamp(w + 1, v.lo_rel, v.hi_rel);
  return funnel_shr(load_word(v.base, w1), load_word(v.base, w0), sh);
}

// XOR of two 2-bit windows -> per-field score word.  Narrow form: each
// 2-bit field holds delta = match - mismatch where the bases agree, else 0.
// Wide form (delta > 3): the field's low bit flags a match.
template <bool NARROW>
XD_FN vint score_word(vint x, int32_t pat, int32_t fold) {
  vint nz = (x | shr_u(x, 1)) & 0x55555555;   // low bit of a field: mismatch
  vint z = nz ^ splat(0x55555555);            // low bit of a field: match
  if (NARROW) return ((z | (z << 1)) & pat) | splat(fold);   // pat = delta in every field
  return z;
}

// Diagonal term of one cell: W_{d-2} + s(a_i, b_j) + 2|gap|.
template <bool NARROW>
XD_FN vint diag_term(vint w2, vint sw, int pos, const Params &P) {
  if (NARROW) return w2 + bfe_u(sw, pos, 2) + P.dbase;           // v_add3_u32
  return mad24(bfe_u(sw, pos, 1), P.delta, w2) + P.dbase;
}

template <int C>
struct Band {
  vint E[C];   // latest even anti-diagonal, W form
  vint O[C];   // latest odd anti-diagonal
  vint SE[C];  // score words for even anti-diagonals
  vint SO[C];  // score words for odd anti-diagonals
};

struct JobView {
  SeqView A, B;
  int64_t a_start, b_start;
  int32_t m, n, x, dir;
  uint32_t *stage;   // the wavefront's LDS words for the wide tiers' score-word build
};

// Score words of the 16 steps e0 .. e0+15 for every slot (both parities),
// slot C*t + r in register r of lane t.
// Slot s at step e: even anti-diagonal 2e holds (i, j) = (s+h+e, e-s-h),
// odd anti-diagonal 2e+1 holds (s+h+e+1, e-s-h).
template <int C, bool NARROW>
XD_FN void build_words(Band<C> &bd, int32_t e0, int32_t h, const JobView &jv, const Params &P) {
  vint s0 = lane_index() * C;
#pragma unroll
  for (int r = 0; r < C; ++r) {
    vint s = s0 + r;
    vint i0 = s + (h + e0);
    vint j0 = splat(e0 - h) - s;
    vint offAe, offAo, offB;
    if (jv.dir > 0) {          // a_i = A[start + i - 1]
      offAe = i0 - 1;
      offAo = i0;
      offB = j0 - 1;
    } else {                   // a_i = A[start - i + 1]: window of the 16 bases below
      offAe = splat(-14) - i0;
      offAo = splat(-15) - i0;
      offB = splat(-14) - j0;
    }
    vint wb = window16(jv.B, offB);
    vint xe = window16(jv.A, offAe) ^ wb;
    vint xo = window16(jv.A, offAo) ^ wb;
    if (jv.dir < 0) {          // backward reads: step q sits in field 15 - q
      xe = bit_reverse(xe);
      xo = bit_reverse(xo);
    }
    bd.SE[r] = score_word<NARROW>(xe, P.pat, P.fold);
    bd.SO[r] = score_word<NARROW>(xo, P.pat, P.fold);
  }
}

// Escalation saves.  A wave whose band outgrows its window stores the state
// of the anti-diagonal it was about to compute -- its number, pending range
// and window base in slot coordinates, best, best cell, both W-form
// thresholds, the cells so far, and the latest even and odd anti-diagonals
// in slot order -- so that the next tier continues from there instead of
// starting over.  When the pool is full the job simply restarts.
XD_FN void save_scalars(int32_t *sv, int32_t d, int32_t lo, int32_t hi, int32_t h, int32_t best,
                        int32_t bi, int32_t bj, int32_t bw, int32_t thr, int32_t C,
                        uint64_t cells) {
  store_first(sv + kSvD, d);
  store_first(sv + kSvLo, lo);
  store_first(sv + kSvHi, hi);
  store_first(sv + kSvH, h);
  store_first(sv + kSvBest, best);
  store_first(sv + kSvBi, bi);
  store_first(sv + kSvBj, bj);
  store_first(sv + kSvBw, bw);
  store_first(sv + kSvThr, thr);
  store_first(sv + kSvC, C);
  store_first(sv + kSvCellsLo, (int32_t)(uint32_t)cells);
  store_first(sv + kSvCellsHi, (int32_t)(uint32_t)(cells >> 32));
}

// The save slot of job j (its own from an earlier escalation, else a new
// one); nullptr when the pool is exhausted.
XD_FN int32_t *save_reserve(const Params &P, int32_t j, int32_t S) {
  if (!P.save_pool || j < 0 || 2 * S + kSaveHdr > kSaveSlotWords) return nullptr;
  const int32_t own = P.job_save[j];
  if (own >= 0) return P.save_pool + own;
  const uint32_t slot = atomic_add_first(P.save_top, 1ull);
  if ((unsigned long long)slot >= P.save_cap) return nullptr;
  return P.save_pool + (int64_t)slot * kSaveSlotWords;
}

XD_FN void save_publish(const Params &P, int32_t j, const int32_t *sv) {
  store_first(P.job_save + j, (int32_t)(sv - P.save_pool));
}

// ---------------------------------------------------------------------------
// One register per lane (64 diagonals).  The computed range, the survivors
// and the window edges of an anti-diagonal are all 64-bit lane masks, so the
// per-anti-diagonal bookkeeping is a handful of scalar instructions:
//   survivors = ballot(v >= threshold) & range            (v_cmp, s_and)
//   first/last survivor a = ff1, 63 - f with f = flbit      (s_ff1, s_flbit)
//   next range = bits [a, 64-f] or [a-1, 63-f]            (s_bfm)
// Matrix clipping is only compiled into the blocks that can reach the end of
// either read; everywhere else the window lies inside the matrix.
enum : int { kStepOn = 0, kStepDone = 1, kStepRecenter = 2 };

struct W1 {
  int32_t e, par;       // next anti-diagonal d = 2e + par
  int32_t h;            // window base: lane s holds i = s + ceil(d/2) + h
  uint64_t range;       // computed range of anti-diagonal d (lanes)
  int32_t width;        // its size
  int32_t lo, hi;       // range ends, valid when a recenter is pending
  int32_t best, bi, bj;
  int32_t bw, thr;      // W-form improvement and prune thresholds of d
  uint32_t cells_blk;
  uint64_t cells;
};

XD_FN uint64_t lane_bits(int lo, int width) {   // bits lo .. lo + width - 1, width < 64
  return ((1ull << width) - 1ull) << lo;
}
XD_FN int clz64(uint64_t m) { return __builtin_clzll(m); }

template <int PAR>
XD_FN void improve_w1(vint cur, W1 &st) {
  int inc = 1;
  while (ballot(cur > st.bw + inc) != 0) ++inc;
  st.bw += inc;
  st.thr += inc;
  st.best += inc;
  const int s = ctz64(ballot(cur == st.bw));
  st.bi = s + st.e + PAR + st.h;         // i = s + ceil(d/2) + h with d = 2e + PAR
  st.bj = 2 * st.e + PAR - st.bi;
}

// Anti-diagonal d = 2 st.e + PAR; cur holds d-2 on entry and d on exit.
template <bool NARROW, bool CLIP, int PAR>
XD_FN int step_w1(vint &cur, vint prv, vint sw, int pos, W1 &st, const JobView &jv,
                  const Params &P) {
  const vint nbr = PAR ? from_next_lane(prv, kNeg) : from_prev_lane(prv, kNeg);
  const vint v = vmax3(diag_term<NARROW>(cur, sw, pos, P), prv, nbr);
  const uint64_t live = ballot(v >= st.thr) & st.range;
  cur = select(lanes(live), v, kNeg);
  st.cells_blk += (uint32_t)st.width;
  if (live == 0) return kStepDone;
  if (ballot(cur > st.bw) != 0) improve_w1<PAR>(cur, st);
  st.bw += P.neg_gap;
  st.thr += P.neg_gap;
  const int a = ctz64(live);
  const int f = clz64(live);             // last survivor is lane 63 - f
  if (PAR) { st.e += 1; st.par = 0; } else { st.par = 1; }
  // next range: [first, last + 1] in i; in lanes [a, 64 - f] after an odd
  // anti-diagonal, [a - 1, 63 - f] after an even one
  if (!CLIP) {
    constexpr uint64_t edge = PAR ? 0xC000000000000001ull : 0x8000000000000003ull;
    if ((live & edge) != 0) {
      st.lo = PAR ? a : a - 1;
      st.hi = PAR ? 64 - f : 63 - f;
      return kStepRecenter;
    }
    st.width = 65 - (a + f);
    st.range = lane_bits(PAR ? a : a - 1, st.width);
    return kStepOn;
  }
  int lo = PAR ? a : a - 1;
  int hi = PAR ? 64 - f : 63 - f;
  const int d1 = 2 * st.e + st.par;        // matrix: d1 - n <= i <= m
  const int smin = (d1 >> 1) - jv.n - st.h;
  const int smax = jv.m - ((d1 + 1) >> 1) - st.h;
  lo = lo > smin ? lo : smin;
  hi = hi < smax ? hi : smax;
  if (lo > hi) return kStepDone;
  if (lo < 1 || hi > kWave - 2) {
    st.lo = lo;
    st.hi = hi;
    return kStepRecenter;
  }
  st.width = hi - lo + 1;
  st.range = lane_bits(lo, st.width);
  return kStepOn;
}

// Steps until anti-diagonal 2 e_end, the end of the extension, or a pending
// recenter.
template <bool NARROW, bool CLIP>
XD_FN int run_w1(Band<1> &bd, W1 &st, int32_t e0, int32_t e_end, const JobView &jv,
                 const Params &P) {
  int rc;
  if (st.par) {
    rc = step_w1<NARROW, CLIP, 1>(bd.O[0], bd.E[0], bd.SO[0], 2 * (st.e - e0), st, jv, P);
    if (rc != kStepOn) return rc;
  }
  while (st.e < e_end) {
    const int pos = 2 * (st.e - e0);
    rc = step_w1<NARROW, CLIP, 0>(bd.E[0], bd.O[0], bd.SE[0], pos, st, jv, P);
    if (rc != kStepOn) return rc;
    rc = step_w1<NARROW, CLIP, 1>(bd.O[0], bd.E[0], bd.SO[0], pos, st, jv, P);
    if (rc != kStepOn) return rc;
  }
  return kStepOn;
}

// Score words of block e0 for the current window base, unless already there.
template <bool NARROW>
XD_FN void ensure_words_w1(Band<1> &bd, const W1 &st, int32_t e0, const JobView &jv,
                           const Params &P, int32_t &words_e0, int32_t &words_h) {
  if (e0 != words_e0 || st.h != words_h) {
    build_words<1, NARROW>(bd, e0, st.h, jv, P);
    words_e0 = e0;
    words_h = st.h;
  }
}

// Runner of extend_job_w1 built from the C steps above.
struct RunC {
  template <bool NARROW, bool CLIP>
  XD_MEMBER static int run(Band<1> &bd, W1 &st, int32_t e0, int32_t e_end,
                           const JobView &jv, const Params &P, int32_t &words_e0,
                           int32_t &words_h) {
    ensure_words_w1<NARROW>(bd, st, e0, jv, P, words_e0, words_h);
    return run_w1<NARROW, CLIP>(bd, st, e0, e_end, jv, P);
  }
};

// Sum over the 64 lanes (log-step exchange through ds_bpermute).
XD_FN uint32_t lane_sum(vint v) {
#pragma unroll
  for (int sh = 1; sh < kWave; sh <<= 1) v = v + from_lane_offset(v, sh, 0);
  return (uint32_t)readlane(v, 0);
}

// Maximum over the 64 lanes (the same exchange).
XD_FN int32_t lane_max(vint v) {
#pragma unroll
  for (int sh = 1; sh < kWave; sh <<= 1) v = vmax(v, from_lane_offset(v, sh, INT32_MIN));
  return readlane(v, 0);
}

template <bool NARROW, class Runner = RunC>
XD_FN JobOut extend_job_w1(const Job &job, const Params &P, int32_t j) {
  JobOut out;
  out.best = 0; out.bi = 0; out.bj = 0; out.status = kJobOk; out.cells = 0;
  if (job.m + job.n == 0) return out;
  JobView jv;
  jv.A = make_view(P.A, P.a_words, job.a_start);
  jv.B = make_view(P.B, P.b_words, job.b_start);
  jv.a_start = job.a_start; jv.b_start = job.b_start;
  jv.m = job.m; jv.n = job.n; jv.x = job.x; jv.dir = job.dir;
  jv.stage = nullptr;

  Band<1> bd;
  bd.O[0] = splat(kNeg);
  bd.E[0] = select(lane_index() == 32, splat(0), kNeg);   // origin, anti-diagonal 0
  W1 st;
  st.h = -32;
  st.e = 0;
  st.par = 1;
  {   // anti-diagonal 1: i in [0, 1], lanes 31 and 32, clipped to the matrix
    int lo = (jv.n >= 1) ? 31 : 32;
    int hi = (jv.m >= 1) ? 32 : 31;
    st.width = hi - lo + 1;
    st.range = lane_bits(lo, st.width);
  }
  st.best = 0; st.bi = 0; st.bj = 0;
  st.bw = P.neg_gap;
  st.thr = P.neg_gap - jv.x;
  st.cells_blk = 0;
  st.cells = 0;

  int32_t words_e0 = -1, words_h = 0;
  for (;;) {
    const int32_t e0 = st.e & ~15;
    const int32_t e_end = e0 + 16;
    // the window stays inside the matrix up to anti-diagonal 2 e_end
    const bool inside = (kWave - 1 + e_end + st.h <= jv.m) && (st.h >= e_end - jv.n);
    const int rc = inside ? Runner::template run<NARROW, false>(bd, st, e0, e_end, jv, P,
                                                                words_e0, words_h)
                          : Runner::template run<NARROW, true>(bd, st, e0, e_end, jv, P,
                                                               words_e0, words_h);
    st.cells += st.cells_blk;
    st.cells_blk = 0;
    if (rc == kStepDone) break;
    if (rc == kStepRecenter) {
      // place the pending range [lo, hi] in the middle of the 64 lanes
      const int width = st.hi - st.lo + 1;
      if (width > kWave - 2) {   // the next tier resumes from here
        int32_t *sv = save_reserve(P, j, kWave);
        const uint64_t cells = st.cells;
        if (sv) {
          save_scalars(sv, 2 * st.e + st.par, st.lo, st.hi, st.h, st.best, st.bi, st.bj, st.bw,
                       st.thr, 1, cells);
          store_vec(sv + kSaveHdr, lane_index(), bd.E[0]);
          store_vec(sv + kSaveHdr + kWave, lane_index(), bd.O[0]);
          save_publish(P, j, sv);
        }
        out.status = kJobWider;
        out.bi = sv ? 1 : 0;
        out.cells = cells;
        return out;
      }
      const int dl = st.lo - (kWave - width) / 2;
      bd.E[0] = from_lane_offset(bd.E[0], dl, kNeg);
      bd.O[0] = from_lane_offset(bd.O[0], dl, kNeg);
      st.h += dl;
      st.width = width;
      st.range = lane_bits(st.lo - dl, width);
    }
  }
  out.best = st.best;
  out.bi = st.bi;
  out.bj = st.bj;
  out.cells = st.cells;
  return out;
}

}  // namespace xd
