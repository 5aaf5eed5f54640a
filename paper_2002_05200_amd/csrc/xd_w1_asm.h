// xd_w1_asm.h -- hand-scheduled gfx950 loop for one-register bands.
//
// Runs the anti-diagonals of one score-word block while the window stays
// inside the matrix (the caller guarantees it), exactly as step_w1<.., false,
// ..> in xd_extend.h does, with the common path of an anti-diagonal reduced
// to 7 VALU and 11 SALU instructions:
//
//   v_mov_b32_dpp  t, prev  wave_shr:1/wave_shl:1   neighbour diagonal (d-1)
//   v_bfe_u32      u, score_word, pos, 2            match field
//   v_add3_u32     cur, cur, base, u                diagonal term (d-2)
//   v_max3_i32     cur, cur, prev, t                the recurrence, gap-free form
//   v_cmp_le_i32   vcc, thr, cur                    X-drop test
//   s_and_b64      live, vcc, range                 ... within the computed range
//   v_cndmask_b32  cur, -inf, cur, live             pruned cells to -inf
//   v_cmp_lt_i32   vcc, bw, cur                     did best improve?
//   s_ff1 / s_flbit / s_bfm                         trim: next range mask
//
// The lane without a neighbour (lane 0 on wave_shr, lane 63 on wave_shl)
// keeps a stale value of t; those lanes are never inside the computed range,
// so the value is discarded by the range mask.  Integer -inf is -2^30, whose bit pattern is
// the inline constant -2.0.  No scalar memory instruction is used.
#pragma once

#include "xd_extend.h"

namespace xd {

// Diagonal term of the narrow (2-bit delta field) and wide (match flag)
// encodings, as assembly text operating on %[cur], %[sw], %[u].
#define XD_DIAG_NARROW(CUR, SW)                         \
  "v_bfe_u32 %[u], %[" SW "], %[pos], 2\n\t"            \
  "v_add3_u32 %[" CUR "], %[" CUR "], %[base], %[u]\n\t"
#define XD_DIAG_WIDE(CUR, SW)                           \
  "v_bfe_u32 %[u], %[" SW "], %[pos], 1\n\t"            \
  "v_mad_u32_u24 %[" CUR "], %[u], %[delta], %[" CUR "]\n\t" \
  "v_add_u32 %[" CUR "], %[base], %[" CUR "]\n\t"

// Steps of one anti-diagonal.  PAR 0 = even (cur E, prev O, shift right),
// PAR 1 = odd (cur O, prev E, shift left).
#define XD_STEP(TAG, DIAG, CUR, PRV, SW, SHIFT, LOADJ, EDGE, PARBIT)              \
  "v_mov_b32_dpp %[t], %[" PRV "] " SHIFT " row_mask:0xf bank_mask:0xf\n\t"          \
  DIAG(CUR, SW)                                                                     \
  "v_max3_i32 %[" CUR "], %[" CUR "], %[" PRV "], %[t]\n\t"                          \
  "s_add_u32 %[cells], %[cells], %[width]\n\t"                                      \
  "v_cmp_le_i32 vcc, %[thr], %[" CUR "]\n\t"                                        \
  "s_and_b64 %[live], vcc, %[range]\n\t"                                            \
  "v_cndmask_b32_e64 %[" CUR "], -2.0, %[" CUR "], %[live]\n\t"                     \
  "s_cbranch_scc0 .Ldone" TAG "%=\n\t"                                              \
  "v_cmp_lt_i32 vcc, %[bw], %[" CUR "]\n\t"                                         \
  "s_cbranch_vccnz .Limp" TAG "%=\n"                                                \
  ".Lret" TAG "%=:\n\t"                                                             \
  "s_add_i32 %[thr], %[thr], %[ng]\n\t"                                             \
  "s_add_i32 %[bw], %[bw], %[ng]\n\t"                                               \
  "s_ff1_i32_b64 %[a], %[live]\n\t"                                                 \
  "s_flbit_i32_b64 %[f], %[live]\n\t"                                               \
  "s_and_b64 vcc, %[live], %[" EDGE "]\n\t"                                         \
  "s_cbranch_scc1 .Lrec" TAG "%=\n\t"                                               \
  "s_add_i32 %[tmp], %[a], %[f]\n\t"                                                \
  "s_sub_i32 %[width], 65, %[tmp]\n\t"                                              \
  LOADJ                                                                             \
  "s_bfm_b64 %[range], %[width], %[a]\n\t"

// Out-of-line tails of one parity: improvement of best (bi = s + e + PAR + h,
// bj = 2e + PAR - bi), end of the extension, pending recenter (the caller
// derives the pending range from a and f).
#define XD_TAILS(TAG, CUR, PARBIT)                                                \
  ".Limp" TAG "%=:\n\t"                                                           \
  "s_mov_b32 %[inc], 1\n"                                                         \
  ".Limpl" TAG "%=:\n\t"                                                          \
  "s_add_i32 %[tmp], %[bw], %[inc]\n\t"                                           \
  "v_cmp_lt_i32 vcc, %[tmp], %[" CUR "]\n\t"                                      \
  "s_cbranch_vccz .Limpd" TAG "%=\n\t"                                            \
  "s_add_i32 %[inc], %[inc], 1\n\t"                                               \
  "s_branch .Limpl" TAG "%=\n"                                                    \
  ".Limpd" TAG "%=:\n\t"                                                          \
  "v_cmp_eq_u32 vcc, %[tmp], %[" CUR "]\n\t"                                      \
  "s_mov_b32 %[bw], %[tmp]\n\t"                                                   \
  "s_add_i32 %[thr], %[thr], %[inc]\n\t"                                          \
  "s_add_i32 %[best], %[best], %[inc]\n\t"                                        \
  "s_ff1_i32_b64 %[tmp], vcc\n\t"                                                 \
  "s_add_i32 %[tmp], %[tmp], %[e]\n\t"                                            \
  "s_add_i32 %[tmp], %[tmp], %[h]\n\t"                                            \
  "s_add_i32 %[bi], %[tmp], " PARBIT "\n\t"                                       \
  "s_lshl_b32 %[tmp], %[e], 1\n\t"                                                \
  "s_add_i32 %[tmp], %[tmp], " PARBIT "\n\t"                                      \
  "s_sub_i32 %[bj], %[tmp], %[bi]\n\t"                                            \
  "s_branch .Lret" TAG "%=\n"                                                     \
  ".Ldone" TAG "%=:\n\t"                                                          \
  "s_mov_b32 %[status], 1\n\t"                                                    \
  "s_branch .Lexit%=\n"                                                           \
  ".Lrec" TAG "%=:\n\t"                                                           \
  "s_mov_b32 %[status], 2\n\t"

template <bool NARROW>
XD_FN int run_w1_fast(Band<1> &bd, W1 &st, int32_t e0, int32_t e_end, const Params &P) {
  int32_t status = 0;
  int32_t pos = 2 * (st.e - e0);
  int32_t a = 0, f = 0, tmp = 0, inc = 0;
  uint64_t live = 0;
  const uint64_t edge_even = 0x8000000000000003ull;   // next odd range [a-1, 63-f] in [1, 62]
  const uint64_t edge_odd = 0xC000000000000001ull;    // next even range [a, 64-f] in [1, 62]
  int32_t e = st.e, par = st.par;
  uint32_t cells = st.cells_blk;
  int32_t u, t;
#define XD_ASM_BODY(DIAG)                                                             \
  asm volatile(                                                                       \
      "s_nop 2\n\t"                                                                   \
      "s_cmp_eq_u32 %[par], 0\n\t"                                                    \
      "s_cbranch_scc0 .Lodd%=\n"                                                      \
      ".Leven%=:\n\t"                                                                 \
      XD_STEP("e", DIAG, "E", "O", "SE", "wave_shr:1", "s_add_i32 %[a], %[a], -1\n\t", \
              "edge_even", "0")                                                       \
      ".Lodd%=:\n\t"                                                                  \
      XD_STEP("o", DIAG, "O", "E", "SO", "wave_shl:1", "", "edge_odd", "1")           \
      "s_add_i32 %[e], %[e], 1\n\t"                                                   \
      "s_add_i32 %[pos], %[pos], 2\n\t"                                               \
      "s_cmp_lt_i32 %[e], %[e_end]\n\t"                                               \
      "s_cbranch_scc1 .Leven%=\n\t"                                                   \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 0\n\t"                                                    \
      "s_branch .Lexit%=\n"                                                           \
      XD_TAILS("e", "E", "0")                                                         \
      "s_mov_b32 %[par], 1\n\t"                                                       \
      "s_branch .Lexit%=\n"                                                           \
      XD_TAILS("o", "O", "1")                                                         \
      "s_add_i32 %[e], %[e], 1\n\t"                                                   \
      "s_mov_b32 %[par], 0\n"                                                         \
      ".Lexit%=:\n"                                                                   \
      : [E] "+v"(bd.E[0].x), [O] "+v"(bd.O[0].x), [u] "=&v"(u), [t] "=&v"(t),        \
        [thr] "+s"(st.thr), [bw] "+s"(st.bw), [best] "+s"(st.best), [bi] "+s"(st.bi), \
        [bj] "+s"(st.bj), [e] "+s"(e), [par] "+s"(par), [pos] "+s"(pos),              \
        [cells] "+s"(cells), [width] "+s"(st.width), [range] "+s"(st.range),          \
        [live] "+s"(live), [a] "+s"(a), [f] "+s"(f), [tmp] "+s"(tmp), [inc] "+s"(inc), \
        [status] "+s"(status)                                                         \
      : [SE] "v"(bd.SE[0].x), [SO] "v"(bd.SO[0].x), [base] "s"(P.base),               \
        [delta] "s"(P.delta), [ng] "s"(P.neg_gap), [e_end] "s"(e_end),                \
        [edge_even] "s"(edge_even), [edge_odd] "s"(edge_odd), [h] "s"(st.h)           \
      : "vcc", "scc", "memory")
  if (NARROW) {
    XD_ASM_BODY(XD_DIAG_NARROW);
  } else {
    XD_ASM_BODY(XD_DIAG_WIDE);
  }
#undef XD_ASM_BODY
  st.e = e;
  st.par = par;
  st.cells_blk = cells;
  if (status == 2) {   // the pending range of the next anti-diagonal, from a and f
    st.lo = par ? a - 1 : a;
    st.hi = par ? 63 - f : 64 - f;
    return kStepRecenter;
  }
  return status == 1 ? kStepDone : kStepOn;
}

// Runner of extend_job_w1: the assembly loop inside the matrix, the C loop
// (with matrix clipping) near the ends of the reads.
struct RunAsm {
  template <bool NARROW, bool CLIP>
  XD_MEMBER static int run(Band<1> &bd, W1 &st, int32_t e0, int32_t e_end, const JobView &jv,
                           const Params &P) {
    if constexpr (CLIP) {
      return run_w1<NARROW, true>(bd, st, e0, e_end, jv, P);
    } else {
      return run_w1_fast<NARROW>(bd, st, e0, e_end, P);
    }
  }
};

}  // namespace xd
