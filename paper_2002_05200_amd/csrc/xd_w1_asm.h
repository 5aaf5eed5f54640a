// xd_w1_asm.h -- hand-scheduled gfx950 loop for one-register bands.
//
// Runs the anti-diagonals of one score-word block while the window stays
// inside the matrix (the caller guarantees it), computing exactly what
// step_w1<.., false, ..> in xd_extend.h computes.  Per anti-diagonal the
// common path is 9 VALU and 7-8 SALU instructions:
//
//   v_addc_co_u32  cnt, 0, cnt, carry=range          cells of this range, per lane
//   v_mov_b32_dpp  t, prev  wave_shr:1 / wave_shl:1  neighbour diagonal (d-1)
//   v_bfe_u32      u, score_word, pos, 2             match field
//   v_add3_u32     cur, cur, base, u                 diagonal term (d-2)
//   v_max3_i32     cur, cur, prev, t                 the recurrence, gap-free form
//   v_cmp_le_i32   vcc, thr, cur                     X-drop test ...
//   s_and_b64      live, vcc, range                  ... within the computed range
//   v_cndmask_b32  cur, -inf, cur, live              pruned cells to -inf
//   v_cmp_lt_i32   vcc, bw, cur                      did best improve?
//   s_add / v_add  thr, bw += -gap                   thresholds of d+1
//   s_ff1 / s_flbit / s_bfm                          trim: next range mask
//
// Window edges: an even anti-diagonal may not use lane 0 (wave_shr leaves it
// without a neighbour) and an odd one may not use lane 63.  Checking after
// every odd anti-diagonal that its survivors avoid lanes 0, 62 and 63 keeps
// the next even range inside [1, 62] and the odd range after it inside
// [0, 62], so even anti-diagonals need no check.  The neighbour-less lane
// keeps a stale t, which the range mask discards.  Integer -inf is -2^30,
// whose bit pattern is the inline constant -2.0.  No memory is accessed.
#pragma once

#include "xd_extend.h"

namespace xd {

#define XD_DIAG_NARROW(CUR, SW)                         \
  "v_bfe_u32 %[u], %[" SW "], %[pos], 2\n\t"            \
  "v_add3_u32 %[" CUR "], %[" CUR "], %[base], %[u]\n\t"
#define XD_DIAG_WIDE(CUR, SW)                           \
  "v_bfe_u32 %[u], %[" SW "], %[pos], 1\n\t"            \
  "v_mad_u32_u24 %[" CUR "], %[u], %[delta], %[" CUR "]\n\t" \
  "v_add_u32 %[" CUR "], %[base], %[" CUR "]\n\t"

// The cell update and prune of one anti-diagonal, then its thresholds and
// survivor ends.
#define XD_CELLS(TAG, DIAG, CUR, PRV, SW, SHIFT)                                  \
  "v_addc_co_u32_e64 %[cnt], vcc, 0, %[cnt], %[range]\n\t"                        \
  "v_mov_b32_dpp %[t], %[" PRV "] " SHIFT " row_mask:0xf bank_mask:0xf\n\t"        \
  DIAG(CUR, SW)                                                                   \
  "v_max3_i32 %[" CUR "], %[" CUR "], %[" PRV "], %[t]\n\t"                        \
  "v_cmp_le_i32 vcc, %[thr], %[" CUR "]\n\t"                                      \
  "s_and_b64 %[live], vcc, %[range]\n\t"                                          \
  "v_cndmask_b32_e64 %[" CUR "], -2.0, %[" CUR "], %[live]\n\t"                   \
  "s_cbranch_scc0 .Ldone%=\n\t"                                                   \
  "v_cmp_lt_i32 vcc, %[bw], %[" CUR "]\n\t"                                       \
  "s_cbranch_vccnz .Limp" TAG "%=\n"                                              \
  ".Lret" TAG "%=:\n\t"                                                           \
  "s_add_i32 %[thr], %[thr], %[ng]\n\t"                                           \
  "v_add_u32 %[bw], %[ng], %[bw]\n\t"                                             \
  "s_ff1_i32_b64 %[a], %[live]\n\t"                                               \
  "s_flbit_i32_b64 %[f], %[live]\n\t"

// Improvement of best on one parity.  The new best W value is bw + inc with
// the smallest inc that no lane exceeds (inc = 1 when match = 1: best grows
// by at most `match` per anti-diagonal).  The best cell is the first lane
// holding it; its lane and position (pos | PAR) are recorded and turned into
// (i, j) after the block.
#define XD_IMPROVE_HEAD_UNIT(TAG, CUR)                                            \
  ".Limp" TAG "%=:\n\t"                                                           \
  "v_add_u32 %[tv], 1, %[bw]\n\t"                                                 \
  "s_mov_b32 %[inc], 1\n\t"
#define XD_IMPROVE_HEAD_LOOP(TAG, CUR)                                            \
  ".Limp" TAG "%=:\n\t"                                                           \
  "s_mov_b32 %[inc], 1\n"                                                         \
  ".Limpl" TAG "%=:\n\t"                                                          \
  "v_add_u32 %[tv], %[inc], %[bw]\n\t"                                            \
  "v_cmp_lt_i32 vcc, %[tv], %[" CUR "]\n\t"                                       \
  "s_cbranch_vccz .Limpd" TAG "%=\n\t"                                            \
  "s_add_i32 %[inc], %[inc], 1\n\t"                                               \
  "s_branch .Limpl" TAG "%=\n"                                                    \
  ".Limpd" TAG "%=:\n\t"
#define XD_IMPROVE(HEAD, TAG, CUR, PARBIT)                                        \
  HEAD(TAG, CUR)                                                                  \
  "v_cmp_eq_u32 vcc, %[tv], %[" CUR "]\n\t"                                       \
  "v_mov_b32 %[bw], %[tv]\n\t"                                                    \
  "s_add_i32 %[thr], %[thr], %[inc]\n\t"                                          \
  "s_add_i32 %[best], %[best], %[inc]\n\t"                                        \
  "s_ff1_i32_b64 %[bs], vcc\n\t"                                                  \
  "s_or_b32 %[bpos], %[pos], " PARBIT "\n\t"                                      \
  "s_branch .Lret" TAG "%=\n"

template <bool NARROW, bool UNIT>
XD_FN int run_w1_fast(Band<1> &bd, W1 &st, vint &cnt, int32_t e0, int32_t e_end,
                      const Params &P) {
  int32_t status = 0;
  int32_t pos = 2 * (st.e - e0);
  const int32_t pos_end = 2 * (e_end - e0);
  int32_t a = 0, f = 0, tmp = 0, inc = 0;
  int32_t bs = 0, bpos = -1;   // lane and position of the last improvement
  uint64_t live = 0;
  const uint64_t edge = 0xC000000000000001ull;   // lanes 0, 62, 63
  int32_t par = st.par;
  int32_t bw = st.bw;
  int32_t u, t, tv;
#define XD_ASM_BODY(DIAG, HEAD)                                                       \
  asm volatile(                                                                       \
      "s_nop 2\n\t"                                                                   \
      "s_cmp_eq_u32 %[par], 0\n\t"                                                    \
      "s_cbranch_scc0 .Lodd%=\n"                                                      \
      ".Leven%=:\n\t"                                                                 \
      XD_CELLS("e", DIAG, "E", "O", "SE", "wave_shr:1")                               \
      "s_add_i32 %[tmp], %[a], %[f]\n\t"                                              \
      "s_sub_i32 %[tmp], 65, %[tmp]\n\t"                                              \
      "s_add_i32 %[a], %[a], -1\n\t"                                                  \
      "s_bfm_b64 %[range], %[tmp], %[a]\n"                                            \
      ".Lodd%=:\n\t"                                                                  \
      XD_CELLS("o", DIAG, "O", "E", "SO", "wave_shl:1")                               \
      "s_and_b64 vcc, %[live], %[edge]\n\t"                                           \
      "s_cbranch_scc1 .Lrec%=\n\t"                                                    \
      "s_add_i32 %[tmp], %[a], %[f]\n\t"                                              \
      "s_sub_i32 %[tmp], 65, %[tmp]\n\t"                                              \
      "s_bfm_b64 %[range], %[tmp], %[a]\n\t"                                          \
      "s_add_i32 %[pos], %[pos], 2\n\t"                                               \
      "s_cmp_lt_i32 %[pos], %[pos_end]\n\t"                                           \
      "s_cbranch_scc1 .Leven%=\n\t"                                                   \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 0\n\t"                                                    \
      "s_branch .Lexit%=\n"                                                           \
      XD_IMPROVE(HEAD, "e", "E", "0")                                                 \
      XD_IMPROVE(HEAD, "o", "O", "1")                                                 \
      ".Ldone%=:\n\t"                                                                 \
      "s_mov_b32 %[status], 1\n\t"                                                    \
      "s_branch .Lexit%=\n"                                                           \
      ".Lrec%=:\n\t"                                                                  \
      "s_add_i32 %[pos], %[pos], 2\n\t"                                               \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 2\n"                                                      \
      ".Lexit%=:\n"                                                                   \
      : [E] "+v"(bd.E[0].x), [O] "+v"(bd.O[0].x), [cnt] "+v"(cnt.x), [bw] "+v"(bw),   \
        [u] "=&v"(u), [t] "=&v"(t), [tv] "=&v"(tv),                                   \
        [thr] "+s"(st.thr), [best] "+s"(st.best), [bs] "+s"(bs), [bpos] "+s"(bpos),   \
        [par] "+s"(par), [pos] "+s"(pos), [range] "+s"(st.range), [live] "+s"(live),  \
        [a] "+s"(a), [f] "+s"(f), [tmp] "+s"(tmp), [inc] "+s"(inc),                   \
        [status] "+s"(status)                                                         \
      : [SE] "v"(bd.SE[0].x), [SO] "v"(bd.SO[0].x), [base] "s"(P.base),               \
        [delta] "s"(P.delta), [ng] "s"(P.neg_gap), [pos_end] "s"(pos_end),            \
        [edge] "s"(edge)                                                              \
      : "vcc", "scc")
  if (NARROW) {
    if (UNIT) { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMPROVE_HEAD_UNIT); }
    else { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMPROVE_HEAD_LOOP); }
  } else {
    if (UNIT) { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMPROVE_HEAD_UNIT); }
    else { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMPROVE_HEAD_LOOP); }
  }
#undef XD_ASM_BODY
  if (bpos >= 0) {   // best cell: i = s + ceil(d/2) + h, j = d - i, d = 2e + par
    const int32_t be = e0 + (bpos >> 1), bp = bpos & 1;
    st.bi = bs + be + bp + st.h;
    st.bj = 2 * be + bp - st.bi;
  }
  st.e = e0 + (pos >> 1);
  st.par = par;
  st.bw = uniform(bw);
  st.width = __builtin_popcountll(st.range);
  if (status == 2) {   // pending even range [a, 64 - f] needs the window moved
    st.lo = a;
    st.hi = 64 - f;
    return kStepRecenter;
  }
  return status == 1 ? kStepDone : kStepOn;
}

// Runner of extend_job_w1: the assembly loop inside the matrix, the C loop
// (with matrix clipping) near the ends of the reads.
struct RunAsm {
  template <bool NARROW, bool CLIP>
  XD_MEMBER static int run(Band<1> &bd, W1 &st, vint &cnt, int32_t e0, int32_t e_end,
                           const JobView &jv, const Params &P) {
    if constexpr (CLIP) {
      return run_w1<NARROW, true>(bd, st, e0, e_end, jv, P);
    } else {
      return P.unit_match ? run_w1_fast<NARROW, true>(bd, st, cnt, e0, e_end, P)
                          : run_w1_fast<NARROW, false>(bd, st, cnt, e0, e_end, P);
    }
  }
};

}  // namespace xd
