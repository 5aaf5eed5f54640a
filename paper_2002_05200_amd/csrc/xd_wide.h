// xd_wide.h -- one X-drop extension per wavefront for bands wider than one
// register: C registers per lane holding the S = 64 C diagonal slots in runs
// of 64 (slot s lives in lane s mod 64 of register s / 64).
//
// Same arithmetic as xd_extend.h (Section III-A recurrence in the gap-free W
// form, pruning against the best of the previous anti-diagonals, next range
// [first live, last live + 1] clipped to the matrix), laid out so that every
// register is a run of 64 consecutive slots:
//   * an anti-diagonal's computed range covers a contiguous span of
//     registers and only that span is updated, so the work follows the
//     band's width rather than the window's;
//   * survivors and the range are 64-bit lane masks per register (compare,
//     ballot, s_ff1 / s_flbit), as in the one-register loop;
//   * the neighbour on the previous anti-diagonal is one whole-wave DPP
//     rotation, with lane 0 (lane 63) taken from the rotated register below
//     (above).
// Registers outside the span last computed on a parity hold -inf, so the
// neighbour lookups at the span's edges read -inf.
#pragma once

#include "xd_extend.h"
#include "xd_wchain_asm.h"

namespace xd {

template <int C>
struct WBand {
  vint E[C];   // latest even anti-diagonal, W form
  vint O[C];   // latest odd anti-diagonal
  vint SE[C];  // score words, even anti-diagonals of the block
  vint SO[C];  // score words, odd anti-diagonals
};

struct WScalars {
  int32_t d;                      // anti-diagonal about to be computed
  int32_t lo, hi;                 // its computed range (slots)
  int32_t h;                      // window base: slot s holds i = s + ceil(d/2) + h
  int32_t best, bi, bj;
  int32_t bw, thr;                // W-form improvement and prune thresholds of d
  int32_t span_lo[2], span_hi[2]; // registers last computed on even / odd d
  int32_t w_lo, w_hi;             // registers whose score words are built
  uint32_t cells_blk;
  uint64_t cells;
};

// Per-wavefront staging of packed words in LDS for the score-word build: A's
// words, then B's, kStageWords each (4 C + 6 consecutive words per sequence
// cover the window; the word after them is a dump slot).
template <int C>
constexpr int kStageWords = 4 * C + 8;

// One sequence's window positions over registers r and lanes l run as
// g = c + 64 r + l (rising) or g = c - 64 r - l (falling).  With r' and l'
// the register and lane counted in the rising sense (r' = C-1-r, l' = 63-l
// for a falling run) and cc = c, resp. c - 64 C + 1, position g lies in word
// (cc >> 4) + 4 r' + q(l') at bit 2 (((cc & 15) + l') & 15), where
// q(l') = ((cc & 15) + l') >> 4 is at most 4.  stage_words copies words
// (cc >> 4) + b, b = 0 .. 4 C + 5, of both sequences, clamped to the arena
// like window16, into the stage: every load is issued before the first store.
template <int C>
XD_FN void stage_words(uint32_t *sa, const SeqView &A, int32_t wa, uint32_t *sb, const SeqView &B,
                       int32_t wb) {
  constexpr int N = 4 * C + 6;
  constexpr int K = (N + kWave - 1) / kWave;
  const int32_t l = lane_id();
  uint32_t ga[K], gb[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int32_t b = l + kWave * k;
    b = b > N - 1 ? N - 1 : b;
    int32_t w = wa + b;
    w = w < A.lo_rel ? A.lo_rel : (w > A.hi_rel ? A.hi_rel : w);
    ga[k] = A.base[w];
    w = wb + b;
    w = w < B.lo_rel ? B.lo_rel : (w > B.hi_rel ? B.hi_rel : w);
    gb[k] = B.base[w];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int32_t b = l + kWave * k;
    b = b > N ? N : b;   // lanes past the words store into the dump slot
    sa[b] = ga[k];
    sb[b] = gb[k];
  }
}

// Score words of every register for the 16 steps e0 .. e0 + 15 (slot s at
// step e: even anti-diagonal 2e holds (s+h+e, e-s-h), odd 2e+1 holds
// (s+h+e+1, e-s-h)).  The words of both sequences are staged in the
// wavefront's LDS buffer first; each register then reads its two-word
// windows at fixed offsets.  A's even- and odd-step windows are one base
// apart and come from the same two words.
template <int C, bool NARROW, int DIR>
XD_FN void wbuild_dir(WBand<C> &bd, int32_t h, int32_t e0, int32_t base, uint32_t *stage,
                      const JobView &jv, const Params &P) {
  uint32_t *sa = stage;
  uint32_t *sb = stage + kStageWords<C>;
  // A's lower window (even step for DIR > 0, odd for DIR < 0) and B's window,
  // for slot s = base + 64 r + l:
  //   DIR > 0: A at (h + e0 - 1) + s rising, B at (e0 - h - 1) - s falling
  //   DIR < 0: A at (-15 - h - e0) - s falling, B at (-14 - e0 + h) + s rising
  const int32_t ca = DIR > 0 ? h + e0 - 1 + base + jv.A.sub
                             : -15 - h - e0 - base + jv.A.sub - 64 * C + 1;
  const int32_t cb = DIR > 0 ? e0 - h - 1 - base + jv.B.sub - 64 * C + 1
                             : -14 - e0 + h + base + jv.B.sub;
  stage_words<C>(sa, jv.A, ca >> 4, sb, jv.B, cb >> 4);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int32_t l = lane_id();
  const int32_t la = DIR > 0 ? l : 63 - l, lb = DIR > 0 ? 63 - l : l;
  const int32_t ta = (ca & 15) + la, tb = (cb & 15) + lb;
  const uint32_t *pa = sa + (ta >> 4);
  const uint32_t *pb = sb + (tb >> 4);
  const uint32_t sha = (uint32_t)(ta & 15) << 1, shb = (uint32_t)(tb & 15) << 1;
#pragma unroll
  for (int r = 0; r < C; ++r) {
    const int ra = DIR > 0 ? r : C - 1 - r, rb = DIR > 0 ? C - 1 - r : r;
    const uint64_t xa = (uint64_t)pa[4 * ra] | ((uint64_t)pa[4 * ra + 1] << 32);
    const uint32_t wb = __builtin_amdgcn_alignbit(pb[4 * rb + 1], pb[4 * rb], shb);
    const uint32_t wlo = (uint32_t)(xa >> sha), whi = (uint32_t)(xa >> (sha + 2));
    vint xe = {(int32_t)((DIR > 0 ? wlo : whi) ^ wb)};
    vint xo = {(int32_t)((DIR > 0 ? whi : wlo) ^ wb)};
    if (DIR < 0) {
      xe = bit_reverse(xe);
      xo = bit_reverse(xo);
    }
    bd.SE[r] = score_word<NARROW>(xe, P.pat, P.fold);
    bd.SO[r] = score_word<NARROW>(xo, P.pat, P.fold);
  }
}

// Builds every register's words (the requested range [r0, r1] is always
// inside), so the next build is due at the block's end or a recentre.
template <int C, bool NARROW>
XD_FN void wbuild(WBand<C> &bd, WScalars &st, int32_t e0, int32_t r0, int32_t r1,
                  const JobView &jv, const Params &P) {
  (void)r0;
  (void)r1;
  if (jv.dir > 0) wbuild_dir<C, NARROW, 1>(bd, st.h, e0, 0, jv.stage, jv, P);
  else wbuild_dir<C, NARROW, -1>(bd, st.h, e0, 0, jv.stage, jv, P);
  st.w_lo = 0;
  st.w_hi = C - 1;
}

// Cell update of register R of the span (no range clipping; see wstep),
// along a chain of registers that carries the rotated neighbour register:
// even anti-diagonals walk the span upwards and odd ones downwards, so each
// register is rotated once.  `carry` holds the rotation of the register
// walked just before; at the chain's start it is -inf (that lane's neighbour
// slot lies outside the previous anti-diagonal's survivors, and every slot
// outside them holds -inf) unless the range was clipped to the matrix there,
// or is the adjacent wave's edge value in the multi-wave tier.  The
// improvement test is deferred: a running lane-wise maximum over the chain
// is compared with bw once afterwards.
template <int C, bool NARROW, int PAR, int R>
XD_FN void wcell_chain(vint *cur, const vint *prv, const vint *sw, int pos, int32_t thr,
                       vint &vmx, vint &carry, const Params &P) {
  vint t;
  if (PAR == 0) {   // slots s-1, s: lane 0 from the rotation of register R-1
    const vint own = rot_prev(prv[R]);
    t = select(lanes(1ull), carry, own);
    carry = own;
  } else {          // slots s, s+1: lane 63 from the rotation of register R+1
    const vint own = rot_next(prv[R]);
    t = select(lanes(1ull << 63), carry, own);
    carry = own;
  }
  const vint v = vmax3(diag_term<NARROW>(cur[R], sw[R], pos, P), prv[R], t);
  cur[R] = select(v >= thr, v, kNeg);
  vmx = vmax(vmx, cur[R]);
}

// Clips register R, an edge of the span, to the range lanes in `mask`;
// returns its surviving lanes.
template <int R>
XD_FN uint64_t wclip(vint *cur, uint64_t mask) {
  cur[R] = select(lanes(mask), cur[R], kNeg);
  return ballot(cur[R] != kNeg);
}

template <int C>
XD_FN uint64_t wclip_at(vint *cur, int r, uint64_t mask) {
  switch (r) {
#define XD_CLIP_CASE(R) \
  case R:               \
    if constexpr (R < C) return wclip<R>(cur, mask); \
    return 0;
    XD_CLIP_CASE(0) XD_CLIP_CASE(1) XD_CLIP_CASE(2) XD_CLIP_CASE(3) XD_CLIP_CASE(4)
    XD_CLIP_CASE(5) XD_CLIP_CASE(6) XD_CLIP_CASE(7) XD_CLIP_CASE(8) XD_CLIP_CASE(9)
    XD_CLIP_CASE(10) XD_CLIP_CASE(11) XD_CLIP_CASE(12) XD_CLIP_CASE(13) XD_CLIP_CASE(14)
    XD_CLIP_CASE(15) XD_CLIP_CASE(16) XD_CLIP_CASE(17) XD_CLIP_CASE(18) XD_CLIP_CASE(19)
    XD_CLIP_CASE(20) XD_CLIP_CASE(21) XD_CLIP_CASE(22) XD_CLIP_CASE(23) XD_CLIP_CASE(24)
    XD_CLIP_CASE(25) XD_CLIP_CASE(26) XD_CLIP_CASE(27) XD_CLIP_CASE(28) XD_CLIP_CASE(29)
    XD_CLIP_CASE(30) XD_CLIP_CASE(31)
#undef XD_CLIP_CASE
    default:
      return 0;
  }
}

template <int C, bool NARROW, int PAR, bool ASM>
XD_FN bool wtail(WBand<C> &bd, WScalars &st, const JobView &jv, const Params &P, int rlo,
                 int rhi, uint64_t live_lo, uint64_t live_hi, vint vmx);

// Anti-diagonal st.d (parity PAR) at step q of the score-word block; then
// prepares st for d + 1.  Returns false once the extension has ended.
//
// The span's registers rlo .. rhi are updated in one fall-through sequence
// entered at its first register (a jump table), each followed by a test for
// its last.  In the C version range clipping is applied afterwards to the
// two edge registers only; lanes outside the range in those registers may
// briefly hold values above best, so an improvement seen during the update
// is confirmed after clipping.  The assembly version (ASM, narrow score
// fields) clips the edge registers inside the chain, so its running maximum
// needs no confirmation, and finds the first best cell with a generated
// scan too.
template <int C, bool NARROW, int PAR, bool ASM>
XD_FN bool wstep(WBand<C> &bd, WScalars &st, int q, const JobView &jv, const Params &P) {
  vint *cur = PAR ? bd.O : bd.E;          // d - 2 on entry, d on exit
  const vint *prv = PAR ? bd.E : bd.O;    // d - 1
  const vint *sw = PAR ? bd.SO : bd.SE;
  const int pos = 2 * q;
  const int rlo = st.lo >> 6, rhi = st.hi >> 6;
  const int plo = st.span_lo[PAR], phi = st.span_hi[PAR];
  if (plo < rlo || phi > rhi) {           // registers leaving the span become -inf
#pragma unroll
    for (int r = 0; r < C; ++r)
      if ((r < rlo || r > rhi) && r >= plo && r <= phi) cur[r] = splat(kNeg);
  }
  const int32_t thr = st.thr;
  vint vmx = splat(kNeg);
  // The chain's outer neighbour slot (below the range on even anti-diagonals,
  // above it on odd ones) holds -inf unless the range was clipped to the
  // matrix at that end; then its register's rotation is fetched.
  vint carry = splat(kNeg);
  {
    const int c = (st.d + 1) >> 1;
    const int i_min = st.d - jv.n > 0 ? st.d - jv.n : 0;
    if (PAR == 0 ? (rlo > 0 && st.lo <= i_min - c - st.h)
                 : (rhi < C - 1 && st.hi >= jv.m - c - st.h)) {
      const int rn = PAR == 0 ? rlo - 1 : rhi + 1;
      switch (rn) {
#define XD_NEIGHBOUR(R)                                                 \
  case R:                                                               \
    if constexpr (R < C) carry = PAR == 0 ? rot_prev(prv[R]) : rot_next(prv[R]); \
    break;
        XD_NEIGHBOUR(0) XD_NEIGHBOUR(1) XD_NEIGHBOUR(2) XD_NEIGHBOUR(3) XD_NEIGHBOUR(4)
        XD_NEIGHBOUR(5) XD_NEIGHBOUR(6) XD_NEIGHBOUR(7) XD_NEIGHBOUR(8) XD_NEIGHBOUR(9)
        XD_NEIGHBOUR(10) XD_NEIGHBOUR(11) XD_NEIGHBOUR(12) XD_NEIGHBOUR(13) XD_NEIGHBOUR(14)
        XD_NEIGHBOUR(15) XD_NEIGHBOUR(16) XD_NEIGHBOUR(17) XD_NEIGHBOUR(18) XD_NEIGHBOUR(19)
        XD_NEIGHBOUR(20) XD_NEIGHBOUR(21) XD_NEIGHBOUR(22) XD_NEIGHBOUR(23) XD_NEIGHBOUR(24)
        XD_NEIGHBOUR(25) XD_NEIGHBOUR(26) XD_NEIGHBOUR(27) XD_NEIGHBOUR(28) XD_NEIGHBOUR(29)
        XD_NEIGHBOUR(30) XD_NEIGHBOUR(31)
#undef XD_NEIGHBOUR
        default:
          break;
      }
    }
  }
  const uint64_t lo_mask = ~0ull << (st.lo & 63);
  const uint64_t hi_mask = ~0ull >> (63 - (st.hi & 63));
  uint64_t live_lo, live_hi;
  if constexpr (ASM && NARROW) {
    // the same chain as generated assembly, with the edge registers clipped
    // to the range inside it (the entry register is rlo going up, rhi going
    // down)
    const uint64_t mf = rlo == rhi ? (lo_mask & hi_mask) : (PAR == 0 ? lo_mask : hi_mask);
    const uint64_t ml = PAR == 0 ? hi_mask : lo_mask;
    uint64_t lf, ll;
    WChain<C, PAR>::run(cur, prv, sw, uniform(pos), uniform(thr), uniform(P.dbase),
                        uniform(rlo), uniform(rhi), carry, vmx, mf, ml, lf, ll);
    live_lo = PAR == 0 ? lf : ll;
    live_hi = PAR == 0 ? ll : lf;
  } else
  {
    if constexpr (PAR == 0) {   // upwards from rlo
      switch (rlo) {
#define XD_SPAN_UP(R)                                                          \
  case R:                                                                      \
    if constexpr (R < C) {                                                     \
      wcell_chain<C, NARROW, 0, R>(cur, prv, sw, pos, thr, vmx, carry, P);     \
      if (rhi == R) break;                                                     \
    }                                                                          \
      [[fallthrough]];
        XD_SPAN_UP(0) XD_SPAN_UP(1) XD_SPAN_UP(2) XD_SPAN_UP(3) XD_SPAN_UP(4)
        XD_SPAN_UP(5) XD_SPAN_UP(6) XD_SPAN_UP(7) XD_SPAN_UP(8) XD_SPAN_UP(9)
        XD_SPAN_UP(10) XD_SPAN_UP(11) XD_SPAN_UP(12) XD_SPAN_UP(13) XD_SPAN_UP(14)
        XD_SPAN_UP(15) XD_SPAN_UP(16) XD_SPAN_UP(17) XD_SPAN_UP(18) XD_SPAN_UP(19)
        XD_SPAN_UP(20) XD_SPAN_UP(21) XD_SPAN_UP(22) XD_SPAN_UP(23) XD_SPAN_UP(24)
        XD_SPAN_UP(25) XD_SPAN_UP(26) XD_SPAN_UP(27) XD_SPAN_UP(28) XD_SPAN_UP(29)
        XD_SPAN_UP(30) XD_SPAN_UP(31)
#undef XD_SPAN_UP
        default:
          break;
      }
    } else {                    // downwards from rhi
      switch (rhi) {
#define XD_SPAN_DOWN(R)                                                               \
  case 31 - R:                                                                        \
    if constexpr (31 - R < C) {                                                       \
      wcell_chain<C, NARROW, 1, (31 - R < C ? 31 - R : 0)>(cur, prv, sw, pos, thr, vmx, \
                                                            carry, P);                \
      if (rlo == 31 - R) break;                                                       \
    }                                                                                 \
      [[fallthrough]];
        XD_SPAN_DOWN(0) XD_SPAN_DOWN(1) XD_SPAN_DOWN(2) XD_SPAN_DOWN(3) XD_SPAN_DOWN(4)
        XD_SPAN_DOWN(5) XD_SPAN_DOWN(6) XD_SPAN_DOWN(7) XD_SPAN_DOWN(8) XD_SPAN_DOWN(9)
        XD_SPAN_DOWN(10) XD_SPAN_DOWN(11) XD_SPAN_DOWN(12) XD_SPAN_DOWN(13) XD_SPAN_DOWN(14)
        XD_SPAN_DOWN(15) XD_SPAN_DOWN(16) XD_SPAN_DOWN(17) XD_SPAN_DOWN(18) XD_SPAN_DOWN(19)
        XD_SPAN_DOWN(20) XD_SPAN_DOWN(21) XD_SPAN_DOWN(22) XD_SPAN_DOWN(23) XD_SPAN_DOWN(24)
        XD_SPAN_DOWN(25) XD_SPAN_DOWN(26) XD_SPAN_DOWN(27) XD_SPAN_DOWN(28) XD_SPAN_DOWN(29)
        XD_SPAN_DOWN(30) XD_SPAN_DOWN(31)
#undef XD_SPAN_DOWN
        default:
          break;
      }
    }
    // clip the edge registers to the computed range
    if (rlo == rhi) {
      live_lo = live_hi = wclip_at<C>(cur, rlo, lo_mask & hi_mask);
    } else {
      live_lo = wclip_at<C>(cur, rlo, lo_mask);
      live_hi = wclip_at<C>(cur, rhi, hi_mask);
    }
  }
  return wtail<C, NARROW, PAR, ASM>(bd, st, jv, P, rlo, rhi, live_lo, live_hi, vmx);
}

// The rest of anti-diagonal st.d (parity PAR) once its span rlo..rhi has
// been updated and clipped: live_lo / live_hi are the survivors of the
// span's lowest and highest register, vmx the running maximum of its cells.
// Span bookkeeping, cells, first and last survivors, the best update and the
// next range.  Returns false once the extension has ended.
template <int C, bool NARROW, int PAR, bool ASM>
XD_FN bool wtail(WBand<C> &bd, WScalars &st, const JobView &jv, const Params &P, int rlo,
                 int rhi, uint64_t live_lo, uint64_t live_hi, vint vmx) {
  vint *cur = PAR ? bd.O : bd.E;
  // (after the assembly chain the maximum saw clipped registers only, so an
  // improvement it shows is already confirmed)
  uint64_t imp = ballot(vmx > st.bw);
  st.span_lo[PAR] = rlo;
  st.span_hi[PAR] = rhi;
  st.cells_blk += (uint32_t)(st.hi - st.lo + 1);

  // first and last survivors: normally in the edge registers, else searched
  int first = -1, last = -1;
  if (live_lo != 0) {
    first = 64 * rlo + ctz64(live_lo);
  } else {
#pragma unroll
    for (int r = 0; r < C; ++r) {
      if (first >= 0 || r <= rlo || r > rhi) continue;
      const uint64_t m = ballot(cur[r] != kNeg);
      if (m != 0) first = 64 * r + ctz64(m);
    }
  }
  if (first < 0) return false;
  if (live_hi != 0) {
    last = 64 * rhi + last_bit64(live_hi);
  } else {
#pragma unroll
    for (int r = C - 1; r >= 0; --r) {
      if (last >= 0 || r < rlo || r >= rhi) continue;
      const uint64_t m = ballot(cur[r] != kNeg);
      if (m != 0) last = 64 * r + last_bit64(m);
    }
  }
  if (imp != 0 && P.unit_match) {
    // match = 1: best rises by exactly 1 and the new best cells are the
    // lanes above bw, so the first register holding one (after clipping)
    // gives both the confirmation and the best cell
    // (for up to 16 registers a fall-through run entered at rlo that stops
    // at the first hit; the 32-register tier measured faster with the
    // unrolled loop, whose code its register allocation handles better)
    int sbest = -1;
    const int32_t bw0 = st.bw;
    if constexpr (ASM && NARROW) {
      sbest = WFirst<C>::run(cur, uniform(bw0), uniform(rlo), uniform(rhi));
    } else
    if constexpr (C >= 32) {
#pragma unroll
      for (int r = 0; r < C; ++r) {
        if (sbest >= 0 || r < rlo || r > rhi) continue;
        const uint64_t m = ballot(cur[r] > bw0);
        if (m != 0) sbest = 64 * r + ctz64(m);
      }
    } else switch (rlo) {
#define XD_FIRST_BEST(R)                                         \
  case R:                                                        \
    if constexpr (R < C) {                                       \
      const uint64_t m = ballot(cur[R] > bw0);                   \
      if (m != 0) {                                              \
        sbest = 64 * R + ctz64(m);                               \
        break;                                                   \
      }                                                          \
      if (rhi == R) break;                                       \
    }                                                            \
    [[fallthrough]];
      XD_FIRST_BEST(0) XD_FIRST_BEST(1) XD_FIRST_BEST(2) XD_FIRST_BEST(3) XD_FIRST_BEST(4)
      XD_FIRST_BEST(5) XD_FIRST_BEST(6) XD_FIRST_BEST(7) XD_FIRST_BEST(8) XD_FIRST_BEST(9)
      XD_FIRST_BEST(10) XD_FIRST_BEST(11) XD_FIRST_BEST(12) XD_FIRST_BEST(13)
      XD_FIRST_BEST(14) XD_FIRST_BEST(15) XD_FIRST_BEST(16) XD_FIRST_BEST(17)
      XD_FIRST_BEST(18) XD_FIRST_BEST(19) XD_FIRST_BEST(20) XD_FIRST_BEST(21)
      XD_FIRST_BEST(22) XD_FIRST_BEST(23) XD_FIRST_BEST(24) XD_FIRST_BEST(25)
      XD_FIRST_BEST(26) XD_FIRST_BEST(27) XD_FIRST_BEST(28) XD_FIRST_BEST(29)
      XD_FIRST_BEST(30) XD_FIRST_BEST(31)
#undef XD_FIRST_BEST
      default:
        break;
    }
    imp = 0;
    if (sbest >= 0) {
      st.bw += 1;
      st.thr += 1;
      st.best += 1;
      st.bi = sbest + ((st.d + 1) >> 1) + st.h;
      st.bj = st.d - st.bi;
    }
  }
  if (!(ASM && NARROW) && imp != 0) {   // confirm on the clipped registers
    imp = 0;
#pragma unroll
    for (int r = 0; r < C; ++r)
      if (r >= rlo && r <= rhi) imp |= ballot(cur[r] > st.bw);
  }

  // best is updated once the whole anti-diagonal is known (Section IV-A)
  if (imp != 0) {
    int inc = 1;
    for (;;) {
      uint64_t more = 0;
#pragma unroll
      for (int r = 0; r < C; ++r)
        if (r >= rlo && r <= rhi) more |= ballot(cur[r] > st.bw + inc);
      if (more == 0) break;
      ++inc;
    }
    st.bw += inc;
    st.thr += inc;
    st.best += inc;
    int sbest = -1;
#pragma unroll
    for (int r = 0; r < C; ++r) {
      if (sbest >= 0 || r < rlo || r > rhi) continue;
      const uint64_t m = ballot(cur[r] == st.bw);
      if (m != 0) sbest = 64 * r + ctz64(m);
    }
    st.bi = sbest + ((st.d + 1) >> 1) + st.h;
    st.bj = st.d - st.bi;
  }

  // next anti-diagonal: [first live, last live + 1] in i, clipped to the matrix
  const int d1 = st.d + 1;
  if (d1 > jv.m + jv.n) return false;
  int lo = PAR ? first : first - 1;
  int hi = PAR ? last + 1 : last;
  const int c1 = (d1 + 1) >> 1;
  const int i_min = d1 - jv.n > 0 ? d1 - jv.n : 0;
  const int smin = i_min - c1 - st.h;
  const int smax = jv.m - c1 - st.h;
  lo = lo > smin ? lo : smin;
  hi = hi < smax ? hi : smax;
  if (lo > hi) return false;
  st.d = d1;
  st.lo = lo;
  st.hi = hi;
  st.bw += P.neg_gap;
  st.thr += P.neg_gap;
  return true;
}

// Lanes [lo, hi] of a 64-lane register, empty when the range misses it.
XD_FN uint64_t lane_span(int lo, int hi) {
  lo = lo < 0 ? 0 : lo;
  hi = hi > 63 ? 63 : hi;
  return lo > hi ? 0ull : ((~0ull >> (63 - hi)) & (~0ull << lo));
}

template <bool NARROW, int PAR>
XD_FN bool wfinish2(WBand<2> &bd, WScalars &st, uint64_t m0, uint64_t m1, const JobView &jv,
                    const Params &P);

// Two registers (128 slots): the same step in straight-line form, both
// registers always updated and clipped by their lane masks.
template <bool NARROW, int PAR>
XD_FN bool wstep2(WBand<2> &bd, WScalars &st, int q, const JobView &jv, const Params &P) {
  vint *cur = PAR ? bd.O : bd.E;
  const vint *prv = PAR ? bd.E : bd.O;
  const vint *sw = PAR ? bd.SO : bd.SE;
  const int pos = 2 * q;
  vint t0, t1;
  if (PAR == 0) {   // slots s-1, s: register 1's lane 0 reads register 0's lane 63
    t0 = rot_prev(prv[0]);
    t1 = select(lanes(1ull), t0, rot_prev(prv[1]));
  } else {          // slots s, s+1: register 0's lane 63 reads register 1's lane 0
    t1 = rot_next(prv[1]);
    t0 = select(lanes(1ull << 63), t1, rot_next(prv[0]));
  }
  const vint v0 = vmax3(diag_term<NARROW>(cur[0], sw[0], pos, P), prv[0], t0);
  const vint v1 = vmax3(diag_term<NARROW>(cur[1], sw[1], pos, P), prv[1], t1);
  const uint64_t m0 = ballot(v0 >= st.thr) & lane_span(st.lo, st.hi);
  const uint64_t m1 = ballot(v1 >= st.thr) & lane_span(st.lo - 64, st.hi - 64);
  cur[0] = select(lanes(m0), v0, kNeg);
  cur[1] = select(lanes(m1), v1, kNeg);
  st.span_lo[PAR] = 0;
  st.span_hi[PAR] = 1;
  st.cells_blk += (uint32_t)(st.hi - st.lo + 1);
  return wfinish2<NARROW, PAR>(bd, st, m0, m1, jv, P);
}

// The rest of a two-register anti-diagonal once its cells are computed and
// pruned (survivor masks m0, m1 of the two registers): end test, best,
// thresholds and the next range.
template <bool NARROW, int PAR>
XD_FN bool wfinish2(WBand<2> &bd, WScalars &st, uint64_t m0, uint64_t m1, const JobView &jv,
                    const Params &P) {
  const vint *cur = PAR ? bd.O : bd.E;
  if ((m0 | m1) == 0) return false;
  const int first = m0 ? ctz64(m0) : 64 + ctz64(m1);
  const int last = m1 ? 64 + last_bit64(m1) : last_bit64(m0);
  if ((ballot(cur[0] > st.bw) | ballot(cur[1] > st.bw)) != 0) {
    int inc = 1;
    while ((ballot(cur[0] > st.bw + inc) | ballot(cur[1] > st.bw + inc)) != 0) ++inc;
    st.bw += inc;
    st.thr += inc;
    st.best += inc;
    const uint64_t e0 = ballot(cur[0] == st.bw);
    const int sbest = e0 ? ctz64(e0) : 64 + ctz64(ballot(cur[1] == st.bw));
    st.bi = sbest + ((st.d + 1) >> 1) + st.h;
    st.bj = st.d - st.bi;
  }
  const int d1 = st.d + 1;
  if (d1 > jv.m + jv.n) return false;
  int lo = PAR ? first : first - 1;
  int hi = PAR ? last + 1 : last;
  const int c1 = (d1 + 1) >> 1;
  const int i_min = d1 - jv.n > 0 ? d1 - jv.n : 0;
  const int smin = i_min - c1 - st.h;
  const int smax = jv.m - c1 - st.h;
  lo = lo > smin ? lo : smin;
  hi = hi < smax ? hi : smax;
  if (lo > hi) return false;
  st.d = d1;
  st.lo = lo;
  st.hi = hi;
  st.bw += P.neg_gap;
  st.thr += P.neg_gap;
  return true;
}

// new slot s <- old slot s + m, 0 < |m| < 64; slots from outside the window
// become -inf.  In place: upward shifts read registers r and r+1, so they run
// in ascending order; downward ones read r and r-1 and run descending.
template <int C>
XD_FN void wshift(vint *a, int m) {
  if (m > 0) {
#pragma unroll
    for (int r = 0; r < C; ++r) {
      const vint here = from_lane_offset(a[r], m, kNeg);
      const vint next = r + 1 < C ? from_lane_offset(a[r + 1], m - 64, kNeg) : splat(kNeg);
      a[r] = vmax(here, next);   // exactly one of the two is a slot; the other is -inf
    }
  } else {
#pragma unroll
    for (int r = C - 1; r >= 0; --r) {
      const vint here = from_lane_offset(a[r], m, kNeg);
      const vint prev = r > 0 ? from_lane_offset(a[r - 1], m + 64, kNeg) : splat(kNeg);
      a[r] = vmax(here, prev);
    }
  }
}

// Where a band of `width` slots starts after a window move: in the middle
// for the two-register tier (its loop wants the band across both
// registers), else low in the window, kLowMargin slots above its bottom
// (WLoop's chains run from the span's top register down to register 0, so
// registers below the span cost work on every anti-diagonal).
constexpr int kLowMargin = 32;
template <int C>
XD_FN int wplace(int width) {
  constexpr int S = kWave * C;
  const int mid = (S - width) / 2;
  return C >= 4 && mid > kLowMargin ? kLowMargin : mid;
}

// Moves the window so the pending range starts at wplace.  Returns false
// when the range is too wide for this tier.
template <int C>
XD_FN bool wrecenter(WBand<C> &bd, WScalars &st) {
  constexpr int S = kWave * C;
  const int width = st.hi - st.lo + 1;
  if (width > S - 2) return false;
  int dl = st.lo - wplace<C>(width);   // new slot = old slot - dl
  while (dl != 0) {
    const int m = dl > 63 ? 63 : (dl < -63 ? -63 : dl);
    wshift<C>(bd.E, m);
    wshift<C>(bd.O, m);
    st.h += m;
    st.lo -= m;
    st.hi -= m;
    dl -= m;
  }
  st.span_lo[0] = st.span_lo[1] = 0;   // any register may now hold values
  st.span_hi[0] = st.span_hi[1] = C - 1;
  st.w_lo = 1;                          // score words belong to the old window
  st.w_hi = 0;
  return true;
}

// Returns false when no save slot was free (the job then starts over).
template <int C>
XD_FN bool wsave(const WBand<C> &bd, const WScalars &st, const Params &P, int32_t j) {
  constexpr int S = kWave * C;
  int32_t *sv = save_reserve(P, j, S);
  if (!sv) return false;
  save_scalars(sv, st.d, st.lo, st.hi, st.h, st.best, st.bi, st.bj, st.bw, st.thr, C,
               st.cells + st.cells_blk);
  const vint l = lane_index();
#pragma unroll
  for (int r = 0; r < C; ++r) {
    store_vec(sv + kSaveHdr, l + 64 * r, bd.E[r]);
    store_vec(sv + kSaveHdr + S, l + 64 * r, bd.O[r]);
  }
  save_publish(P, j, sv);
  return true;
}

// Restores a narrower tier's save (slot order) into the middle of the window.
template <int C>
XD_FN bool wrestore(WBand<C> &bd, WScalars &st, const Params &P, int32_t j) {
  if (!P.save_pool || j < 0) return false;
  const int32_t off = P.job_save[j];
  if (off < 0) return false;
  const int32_t *sv = P.save_pool + off;
  const int32_t cs = uniform(sv[kSvC]);
  if (cs >= C) return false;
  const int32_t ss = kWave * cs;
  const int32_t lo0 = uniform(sv[kSvLo]), hi0 = uniform(sv[kSvHi]);
  const int32_t shift = wplace<C>(hi0 - lo0 + 1) - lo0;   // saved slot + shift = new slot
  st.d = uniform(sv[kSvD]);
  st.lo = lo0 + shift;
  st.hi = hi0 + shift;
  st.h = uniform(sv[kSvH]) - shift;
  st.best = uniform(sv[kSvBest]); st.bi = uniform(sv[kSvBi]); st.bj = uniform(sv[kSvBj]);
  st.bw = uniform(sv[kSvBw]); st.thr = uniform(sv[kSvThr]);
  st.cells = (uint64_t)(uint32_t)uniform(sv[kSvCellsLo]) | ((uint64_t)(uint32_t)uniform(sv[kSvCellsHi]) << 32);
  st.cells_blk = 0;
  const vint l = lane_index();
#pragma unroll
  for (int r = 0; r < C; ++r) {
    const vint old = l + (64 * r - shift);
    const vbool in = le_u(old, (uint32_t)(ss - 1));
    const vint k = select(in, old, 0);
    bd.E[r] = select(in, load_vec(sv + kSaveHdr, k), kNeg);
    bd.O[r] = select(in, load_vec(sv + kSaveHdr + ss, k), kNeg);
  }
  st.span_lo[0] = st.span_lo[1] = 0;
  st.span_hi[0] = st.span_hi[1] = C - 1;
  return true;
}

// ---------------------------------------------------------------------------
// Fast path of the two-register tier: a hand-scheduled loop (xd_w2_asm.h)
// runs anti-diagonals while the band straddles the two registers, stays in
// slots [2, 124] and the window lies inside the matrix.
enum : int { kW2Step = 1, kW2Recenter = 2, kW2Leave = 3 };

// Runs from anti-diagonal st.d (range st.lo .. st.hi, 2 <= lo <= 63 < 64 <=
// hi <= 124; the window inside the matrix for the block of st.d).  Adds the
// cells it computes to st.cells and keeps best, bi, bj, thr, bw current.
// Returns
//   kW2Step      anti-diagonal st.d computed and pruned, survivors m0 / m1
//                with one of them empty; its end test, best, thresholds and
//                next range still to do (wfinish2);
//   kW2Recenter  st.d is the next anti-diagonal, st.lo .. st.hi its range,
//                which reaches slots {0, 1} or {125, 126, 127};
//   kW2Leave     st.d starts a block in which the window would leave the
//                matrix; st.lo .. st.hi its range.
template <bool NARROW, bool FWD, bool FOLD>
XD_FN int w2_loop(WBand<2> &bd, WScalars &st, const JobView &jv, const Params &P, uint64_t &m0,
                  uint64_t &m1);

// Returns 0 to continue with the C steps at st.d, 1 when the extension has
// ended, 2 when the band has outgrown the tier.
template <bool NARROW>
XD_FN int w2_fast(WBand<2> &bd, WScalars &st, const JobView &jv, const Params &P) {
  constexpr int S = 2 * kWave;
  if (!NARROW || !P.unit_match || P.delta != 2) return 0;
  for (;;) {
    const int32_t e_end = ((st.d >> 1) & ~15) + 16;
    if (S - 1 + e_end + st.h > jv.m || st.h < e_end - jv.n) return 0;   // near a read's end
    const int width = st.hi - st.lo + 1;
    if (width < 2 || width > S - 5) return 0;
    if (st.lo < 2 || st.hi > S - 4 || st.lo > kWave - 1 || st.hi < kWave) {
      if (!wrecenter<2>(bd, st)) return 2;
      continue;                          // the window moved: test it again
    }
    uint64_t m0 = 0, m1 = 0;
    const bool fold = P.base == 1;   // = P.fold here (match 1, delta 2 checked above)
    const int rc = jv.dir > 0 ? (fold ? w2_loop<NARROW, true, true>(bd, st, jv, P, m0, m1)
                                      : w2_loop<NARROW, true, false>(bd, st, jv, P, m0, m1))
                              : (fold ? w2_loop<NARROW, false, true>(bd, st, jv, P, m0, m1)
                                      : w2_loop<NARROW, false, false>(bd, st, jv, P, m0, m1));
    st.span_lo[0] = st.span_lo[1] = 0;
    st.span_hi[0] = st.span_hi[1] = 1;
    st.w_lo = 1;                         // score words to be rebuilt by the C steps
    st.w_hi = 0;
    if (rc == kW2Step) {
      const bool go = (st.d & 1) ? wfinish2<NARROW, 1>(bd, st, m0, m1, jv, P)
                                 : wfinish2<NARROW, 0>(bd, st, m0, m1, jv, P);
      if (!go) return 1;
      continue;
    }
    // the pending range may lie in the next block, beyond a read's end: clip
    // it to the matrix as the C step does
    const int c1 = (st.d + 1) >> 1;
    const int i_min = st.d - jv.n > 0 ? st.d - jv.n : 0;
    const int smin = i_min - c1 - st.h, smax = jv.m - c1 - st.h;
    if (st.lo < smin) st.lo = smin;
    if (st.hi > smax) st.hi = smax;
    if (st.d > jv.m + jv.n || st.lo > st.hi) return 1;
    if (rc == kW2Recenter && !wrecenter<2>(bd, st)) return 2;
  }
}

// All anti-diagonals of an extension on C >= 4 registers with the
// generated assembly (match = 1, narrow score fields): block transitions,
// recentres and score words in C, then WLoop for the rest of the block (its
// ranges clipped to the matrix; an anti-diagonal whose survivors left the
// span's edge registers is finished here).  Returns false when the band
// outgrew the window.
template <int C, bool NARROW, bool FOLD>
XD_FN bool wide_fast(WBand<C> &bd, WScalars &st, const JobView &jv, const Params &P) {
  constexpr int S = kWave * C;
  int32_t e0 = (st.d >> 1) & ~15;
  for (;;) {
    const int32_t e = st.d >> 1;
    const bool even = (st.d & 1) == 0;
    bool move = st.lo < 1 || st.hi > S - 2;
    if (even && e - e0 == 16) {
      e0 = e;
      st.cells += st.cells_blk;
      st.cells_blk = 0;
      st.w_lo = 1;
      st.w_hi = 0;
      // a band a register or more above its place moves down (the words are
      // rebuilt for this block anyway)
      if (st.lo - wplace<C>(st.hi - st.lo + 1) >= kWave) move = true;
    }
    if (move) {
      if (!wrecenter<C>(bd, st)) return false;
    }
    if ((st.lo >> 6) < st.w_lo || (st.hi >> 6) > st.w_hi)
      wbuild<C, NARROW>(bd, st, e0, (st.lo >> 6) - 1, (st.hi >> 6) + 1, jv, P);
    WLoopState ws;   // every field a wave-uniform scalar (SGPR operands)
    ws.d = uniform(st.d); ws.lo = uniform(st.lo); ws.hi = uniform(st.hi);
    ws.bw = uniform(st.bw); ws.thr = uniform(st.thr);
    ws.cells = uniform((int32_t)st.cells_blk); ws.bs = 0; ws.bpos = -1;
    ws.spl0 = uniform(st.span_lo[0]); ws.sph0 = uniform(st.span_hi[0]);
    ws.spl1 = uniform(st.span_lo[1]); ws.sph1 = uniform(st.span_hi[1]);
    ws.dstop = uniform(2 * (e0 + 16)); ws.e0x2 = uniform(2 * e0);
    ws.mh = uniform(jv.m - st.h); ws.nh = uniform(jv.n + st.h);
    ws.base = uniform(P.dbase); ws.ng = uniform(P.neg_gap); ws.smax = S - 2;
    ws.rlo = 0; ws.rhi = 0; ws.lf = 0; ws.ll = 0; ws.mx = kNeg;
    const int32_t rc = WLoop<C, FOLD>::run(bd.E, bd.O, bd.SE, bd.SO, ws);
    st.d = uniform(ws.d); st.lo = uniform(ws.lo); st.hi = uniform(ws.hi);
    st.bw = uniform(ws.bw); st.thr = uniform(ws.thr);
    st.cells_blk = (uint32_t)uniform(ws.cells);
    st.span_lo[0] = uniform(ws.spl0); st.span_hi[0] = uniform(ws.sph0);
    st.span_lo[1] = uniform(ws.spl1); st.span_hi[1] = uniform(ws.sph1);
    if (ws.bpos >= 0) {   // the last improvement of best in this run
      st.bi = uniform(ws.bs) + ((uniform(ws.bpos) + 1) >> 1) + st.h;
      st.bj = uniform(ws.bpos) - st.bi;
    }
    st.best = st.bw - st.d * P.neg_gap;   // best = bw - d |gap| between anti-diagonals
    if (rc == 4) return true;             // the next range lies outside the matrix
    if (rc == 2) {   // the chain of st.d is done; finish it here
      vint vmx;
      vmx.x = ws.mx;
      const int rlo = uniform(ws.rlo), rhi = uniform(ws.rhi);
      // (both parities' chains enter at rhi: lf holds its survivors, ll rlo's)
      const bool go = (st.d & 1) == 0
                          ? wtail<C, NARROW, 0, true>(bd, st, jv, P, rlo, rhi, ws.ll, ws.lf, vmx)
                          : wtail<C, NARROW, 1, true>(bd, st, jv, P, rlo, rhi, ws.ll, ws.lf, vmx);
      if (!go) return true;
    }
  }
}

// Whole one-directional extension of job j, resumed from a narrower tier's
// save when there is one.  FAST selects the assembly: the hand-scheduled
// loop for two registers, the generated chain with built-in edge clipping
// for more (narrow score fields only; else FAST changes nothing).
template <int C, bool NARROW, bool FAST = false, bool FOLD = false>
XD_FN JobOut extend_job_wide(const Job &job, const Params &P, int32_t j, uint32_t *stage) {
  constexpr int S = kWave * C;
  JobOut out;
  out.best = 0; out.bi = 0; out.bj = 0; out.status = kJobOk; out.cells = 0;
  if (job.m + job.n == 0) return out;

  JobView jv;
  jv.A = make_view(P.A, P.a_words, job.a_start);
  jv.B = make_view(P.B, P.b_words, job.b_start);
  jv.a_start = job.a_start; jv.b_start = job.b_start;
  jv.m = job.m; jv.n = job.n; jv.x = job.x; jv.dir = job.dir;
  jv.stage = stage;

  WBand<C> bd;
  WScalars st;
  if (!wrestore<C>(bd, st, P, j)) {
    const vbool origin = lane_index() == 0;
#pragma unroll
    for (int r = 0; r < C; ++r) {   // anti-diagonal 0: the origin in slot S/2
      bd.E[r] = (r == C / 2) ? select(origin, splat(0), kNeg) : splat(kNeg);
      bd.O[r] = splat(kNeg);
    }
    st.h = -S / 2;
    st.d = 1;
    {   // range of anti-diagonal 1 from the live origin: i in [0, 1]
      const int smin = (1 - jv.n > 0 ? 1 - jv.n : 0) - 1 - st.h;
      const int smax = jv.m - 1 - st.h;
      st.lo = (S / 2 - 1) > smin ? (S / 2 - 1) : smin;
      st.hi = (S / 2) < smax ? (S / 2) : smax;
    }
    st.best = 0; st.bi = 0; st.bj = 0;
    st.bw = P.neg_gap;            // best + 1*|gap|
    st.thr = P.neg_gap - jv.x;
    st.cells_blk = 0;
    st.cells = 0;
    st.span_lo[0] = st.span_hi[0] = C / 2;   // the origin's register
    st.span_lo[1] = 1;                        // nothing odd yet
    st.span_hi[1] = 0;
  }
  st.w_lo = 1;
  st.w_hi = 0;

  int32_t e = st.d >> 1;
  bool odd = (st.d & 1) != 0;
  int32_t e0 = e & ~15;
  bool ok = true;
  bool fast_loop = false;
  if constexpr (FAST && NARROW && C >= 4) fast_loop = P.unit_match != 0;
  if constexpr (FAST && NARROW && C >= 4) {
    if (fast_loop) ok = wide_fast<C, NARROW, FOLD>(bd, st, jv, P);
  }
  for (; !fast_loop;) {
    if constexpr (FAST && C == 2) {
      const int32_t d_before = st.d;
      const int rc = w2_fast<NARROW>(bd, st, jv, P);
      if (rc == 1) break;
      if (rc == 2) { ok = false; break; }
      if (st.d != d_before) {   // the loop ran (and left the score words to rebuild)
        e = st.d >> 1;
        odd = (st.d & 1) != 0;
        e0 = e & ~15;
      }
    }
    if (!odd) {
      if (st.lo < 1 || st.hi > S - 2) {
        if (!wrecenter<C>(bd, st)) { ok = false; break; }
      }
      if (e - e0 == 16) {
        e0 = e;
        st.cells += st.cells_blk;
        st.cells_blk = 0;
        st.w_lo = 1;
        st.w_hi = 0;
      }
      if ((st.lo >> 6) < st.w_lo || (st.hi >> 6) > st.w_hi)
        wbuild<C, NARROW>(bd, st, e0, (st.lo >> 6) - 1, (st.hi >> 6) + 1, jv, P);
      bool go;
      if constexpr (C == 2) go = wstep2<NARROW, 0>(bd, st, e - e0, jv, P);
      else go = wstep<C, NARROW, 0, FAST>(bd, st, e - e0, jv, P);
      if (!go) break;                                           // d = 2e
    }
    odd = false;
    if (st.lo < 1 || st.hi > S - 2) {
      if (!wrecenter<C>(bd, st)) { ok = false; break; }
    }
    if ((st.lo >> 6) < st.w_lo || (st.hi >> 6) > st.w_hi)
      wbuild<C, NARROW>(bd, st, e0, (st.lo >> 6) - 1, (st.hi >> 6) + 1, jv, P);
    bool go;
    if constexpr (C == 2) go = wstep2<NARROW, 1>(bd, st, e - e0, jv, P);
    else go = wstep<C, NARROW, 1, FAST>(bd, st, e - e0, jv, P);
    if (!go) break;                                             // d = 2e + 1
    ++e;
  }
  if (!ok) {
    out.bi = wsave<C>(bd, st, P, j) ? 1 : 0;
    out.status = kJobWider;
    out.cells = st.cells + st.cells_blk;
    return out;
  }
  out.best = st.best;
  out.bi = st.bi;
  out.bj = st.bj;
  out.cells = st.cells + st.cells_blk;
  return out;
}

}  // namespace xd
