// xd_w2_asm.h -- hand-scheduled gfx950 loop for two-register bands (128
// diagonal slots, slot s in lane s mod 64 of register s / 64).
//
// Computes exactly what wstep2 in xd_wide.h computes, for bands that
// straddle the two registers, while the window lies inside the matrix and the
// scores are +1 for a match with a match/mismatch difference of 2 (the
// narrow two-bit score fields).  Like the one-register loop it runs across
// score-word blocks, prefetching each block's words a block ahead, and
// returns to C code when a register empties (end of the extension, or a band
// that no longer straddles), when the band nears the window's edge, or when
// the window approaches the end of a read.
//
// One anti-diagonal (18 VALU, about 10 SALU, for 128 slots):
//   v_addc x2                      cells of the computed range, per lane
//   v_mov_dpp x2, v_cndmask        neighbour on d-1: a whole-wave rotation of
//                                  each register, the lane crossing between
//                                  the registers taken from the other one
//   v_bfe, v_add3 x2               diagonal term (d-2) from the score field
//                                  (v_add for +1/-1/-1: base 1 in the field)
//   v_max3 x2                      the recurrence, gap-free form
//   v_cmp, s_and, v_cndmask x2     X-drop test within the range, -inf
//   s_cmp + branches               a register without survivors: leave
//   v_cmp x1-2 + branch            improvement of best (out of line)
//   s_add / v_add                  thresholds of d+1
//   s_ff1, s_flbit, 2 shifts       next range: register 0 from its first
//                                  survivor up, register 1 up to its last
// Because the band straddles, the next range always starts in register 0
// and ends in register 1, so each register's range mask is one shift of -1.
//
// Window edges: an even anti-diagonal may not use slot 0 (its rotated
// neighbour is register 1's lane 63) and an odd one may not use slot 127.
// The odd anti-diagonals of odd pairs leave for a recentre when a survivor
// sits in slots {0, 1} or {125, 126, 127}; survivors in [2, 124] there keep
// the next four ranges inside [0, 126] with slot 0 out of even ranges and
// slot 127 out of odd ones, and the loop is entered only with the range
// inside [2, 124].
#pragma once

#include "xd_w1_asm.h"
#include "xd_wide.h"

namespace xd {

#define W2_NBR_EVEN                                                               \
  "v_mov_b32_dpp %[t0], %[O0] wave_ror:1 row_mask:0xf bank_mask:0xf\n\t"         \
  "v_mov_b32_dpp %[t1], %[O1] wave_ror:1 row_mask:0xf bank_mask:0xf\n\t"         \
  "v_cndmask_b32_e64 %[t1], %[t1], %[t0], %[l0]\n\t"
#define W2_NBR_ODD                                                                \
  "v_mov_b32_dpp %[t1], %[E1] wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"         \
  "v_mov_b32_dpp %[t0], %[E0] wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"         \
  "v_cndmask_b32_e64 %[t0], %[t0], %[t1], %[l63]\n\t"

// The diagonal term; W2_DIAG_SEL picks the form where the loop is expanded:
// W2_DIAG_ADD3 adds base, W2_DIAG_FOLD takes words whose fields already hold
// base + delta * match (+1/-1/-1).
#define W2_DIAG_ADD3(CUR, SW, P)                                                  \
  "v_bfe_u32 %[u], %[" SW "], " P ", 2\n\t"                                        \
  "v_add3_u32 %[" CUR "], %[" CUR "], %[base], %[u]\n\t"
#define W2_DIAG_FOLD(CUR, SW, P)                                                  \
  "v_bfe_u32 %[u], %[" SW "], " P ", 2\n\t"                                        \
  "v_add_u32 %[" CUR "], %[u], %[" CUR "]\n\t"
#define W2_DIAG(CUR, SW, P) W2_DIAG_SEL(CUR, SW, P)

// Cells, recurrence, pruning and the improvement test of anti-diagonal
// 2(e0 + K) + PAR, registers C0 / C1 (d-2 in, d out) from P0 / P1 (d-1).
#define W2_CORE(T, K, P, C0, C1, P0, P1, S0, S1, NBR)                            \
  "v_addc_co_u32_e64 %[cnt], vcc, 0, %[cnt], %[r0]\n\t"                           \
  "v_addc_co_u32_e64 %[cnt], vcc, 0, %[cnt], %[r1]\n\t"                           \
  NBR                                                                             \
  W2_DIAG(C0, S0, P)                                                              \
  W2_DIAG(C1, S1, P)                                                              \
  "v_max3_i32 %[" C0 "], %[" C0 "], %[" P0 "], %[t0]\n\t"                         \
  "v_max3_i32 %[" C1 "], %[" C1 "], %[" P1 "], %[t1]\n\t"                         \
  "v_cmp_le_i32 vcc, %[thr], %[" C0 "]\n\t"                                      \
  "s_and_b64 %[v0], vcc, %[r0]\n\t"                                               \
  "v_cmp_le_i32 vcc, %[thr], %[" C1 "]\n\t"                                      \
  "s_and_b64 %[v1], vcc, %[r1]\n\t"                                               \
  "v_cndmask_b32_e64 %[" C0 "], -2.0, %[" C0 "], %[v0]\n\t"                       \
  "v_cndmask_b32_e64 %[" C1 "], -2.0, %[" C1 "], %[v1]\n\t"                       \
  "s_cbranch_scc0 .Lx" T K "_%=\n\t"                                               \
  "s_cmp_eq_u64 %[v0], 0\n\t"                                                     \
  "s_cbranch_scc1 .Lx" T K "_%=\n\t"                                               \
  "v_cmp_lt_i32 vcc, %[bw], %[" C0 "]\n\t"                                       \
  "s_cbranch_vccnz .Li" T K "_%=\n\t"                                              \
  "v_cmp_lt_i32 vcc, %[bw], %[" C1 "]\n\t"                                       \
  "s_cbranch_vccnz .Lj" T K "_%=\n\t"                                              \
  "s_add_i32 %[thr], %[thr], %[ng]\n\t"                                           \
  "v_add_u32 %[bw], %[ng], %[bw]\n"                                               \
  ".Lq" T K "_%=:\n\t"                                                             \
  "s_ff1_i32_b64 %[a], %[v0]\n\t"                                                 \
  "s_flbit_i32_b64 %[f], %[v1]\n\t"

// Even anti-diagonal: next (odd) range is slots [a - 1, 127 - f].
#define W2_EVEN(K, P)                                                             \
  ".Le" K "_%=:\n\t"                                                               \
  W2_CORE("e", K, P, "E0", "E1", "O0", "O1", "SE0", "SE1", W2_NBR_EVEN)           \
  "s_add_i32 %[a], %[a], -1\n\t"                                                  \
  "s_lshl_b64 %[r0], -1, %[a]\n\t"                                                \
  "s_lshr_b64 %[r1], -1, %[f]\n"
// Odd anti-diagonal: next (even) range is slots [a, 128 - f]; on odd K the
// edge test comes first.
#define W2_ODD_RANGE                                                              \
  "s_lshl_b64 %[r0], -1, %[a]\n\t"                                                \
  "s_add_i32 %[f], %[f], -1\n\t"                                                  \
  "s_lshr_b64 %[r1], -1, %[f]\n"
#define W2_ODD(K, P)                                                              \
  ".Lo" K "_%=:\n\t"                                                               \
  W2_CORE("o", K, P, "O0", "O1", "E0", "E1", "SO0", "SO1", W2_NBR_ODD)            \
  W2_ODD_RANGE
#define W2_ODD_EDGE(K, P)                                                         \
  ".Lo" K "_%=:\n\t"                                                               \
  W2_CORE("o", K, P, "O0", "O1", "E0", "E1", "SO0", "SO1", W2_NBR_ODD)            \
  "s_and_b64 %[tq], %[v1], %[e1]\n\t"                                             \
  "s_and_b64 vcc, %[v0], 3\n\t"                                                   \
  "s_or_b64 vcc, vcc, %[tq]\n\t"                                                  \
  "s_cbranch_scc1 .Lc" K "_%=\n\t"                                                 \
  W2_ODD_RANGE
#define W2_PAIR(K, P) W2_EVEN(K, P) W2_ODD(K, P)
#define W2_PAIR_EDGE(K, P) W2_EVEN(K, P) W2_ODD_EDGE(K, P)

// Improvement of best (match = 1: the new best W value is bw + 1 and the
// lanes above bw hold it; register 0's slots come first).  Applies the
// anti-diagonal's threshold drift together with the raise.
#define W2_IMP(TAG, BP, OFF64, RET)                                               \
  ".L" TAG "_%=:\n\t"                                                              \
  "s_ff1_i32_b64 %[bs], vcc\n\t"                                                  \
  OFF64                                                                           \
  "s_add_i32 %[bpos], %[e0x2], " BP "\n\t"                                        \
  "s_add_i32 %[thr], %[thr], %[ng1]\n\t"                                          \
  "v_add_u32 %[bw], %[ng1], %[bw]\n\t"                                            \
  "s_branch .L" RET "_%=\n"
#define W2_REG1 "s_add_i32 %[bs], %[bs], 64\n\t"

#define W2_STUBS(K, P, P1, PN)                                                    \
  W2_IMP("ie" K, P, "", "qe" K)                                                   \
  W2_IMP("je" K, P, W2_REG1, "qe" K)                                              \
  W2_IMP("io" K, P1, "", "qo" K)                                                  \
  W2_IMP("jo" K, P1, W2_REG1, "qo" K)                                             \
  ".Lxe" K "_%=:\n\t"                                                              \
  "s_mov_b32 %[pos], " P "\n\t"                                                   \
  "s_mov_b32 %[par], 0\n\t"                                                       \
  "s_mov_b32 %[status], 1\n\t"                                                    \
  "s_branch .Lexit_%=\n"                                                           \
  ".Lxo" K "_%=:\n\t"                                                              \
  "s_mov_b32 %[pos], " P "\n\t"                                                   \
  "s_mov_b32 %[par], 1\n\t"                                                       \
  "s_mov_b32 %[status], 1\n\t"                                                    \
  "s_branch .Lexit_%=\n"
#define W2_STUBS_EDGE(K, P, P1, PN)                                               \
  W2_STUBS(K, P, P1, PN)                                                          \
  ".Lc" K "_%=:\n\t"                                                               \
  "s_mov_b32 %[pos], " PN "\n\t"                                                  \
  "s_mov_b32 %[par], 0\n\t"                                                       \
  "s_mov_b32 %[status], 2\n\t"                                                    \
  "s_branch .Lexit_%=\n"

#define W2_ALL_PAIRS                                                              \
  W2_PAIR("0", "0") W2_PAIR_EDGE("1", "2") W2_PAIR("2", "4") W2_PAIR_EDGE("3", "6") \
  W2_PAIR("4", "8") W2_PAIR_EDGE("5", "10") W2_PAIR("6", "12")                    \
  W2_PAIR_EDGE("7", "14") W2_PAIR("8", "16") W2_PAIR_EDGE("9", "18")              \
  W2_PAIR("10", "20") W2_PAIR_EDGE("11", "22") W2_PAIR("12", "24")                \
  W2_PAIR_EDGE("13", "26") W2_PAIR("14", "28") W2_PAIR_EDGE("15", "30")
#define W2_ALL_STUBS                                                              \
  W2_STUBS("0", "0", "1", "2") W2_STUBS_EDGE("1", "2", "3", "4")                  \
  W2_STUBS("2", "4", "5", "6") W2_STUBS_EDGE("3", "6", "7", "8")                  \
  W2_STUBS("4", "8", "9", "10") W2_STUBS_EDGE("5", "10", "11", "12")              \
  W2_STUBS("6", "12", "13", "14") W2_STUBS_EDGE("7", "14", "15", "16")            \
  W2_STUBS("8", "16", "17", "18") W2_STUBS_EDGE("9", "18", "19", "20")            \
  W2_STUBS("10", "20", "21", "22") W2_STUBS_EDGE("11", "22", "23", "24")          \
  W2_STUBS("12", "24", "25", "26") W2_STUBS_EDGE("13", "26", "27", "28")          \
  W2_STUBS("14", "28", "29", "30") W2_STUBS_EDGE("15", "30", "31", "32")

// Score words of one register from its windows A (even), A (odd) and B.
#define W2_WORDS(REV, WE, WO, WB, SE, SO)                                         \
  "v_alignbit_b32 %[x0], %[hi" WE "], %[lo" WE "], %[sh" WE "]\n\t"                \
  "v_alignbit_b32 %[x1], %[hi" WO "], %[lo" WO "], %[sh" WO "]\n\t"                \
  "v_alignbit_b32 %[x2], %[hi" WB "], %[lo" WB "], %[sh" WB "]\n\t"                \
  "v_xor_b32 %[x0], %[x0], %[x2]\n\t"                                             \
  "v_xor_b32 %[x1], %[x1], %[x2]\n\t"                                             \
  REV                                                                             \
  W2_SW_SEL(SE, "x0")                                                             \
  W2_SW_SEL(SO, "x1")

template <bool NARROW, bool FWD, bool FOLD>
XD_FN int w2_loop(WBand<2> &bd, WScalars &st, const JobView &jv, const Params &P, uint64_t &m0,
                  uint64_t &m1) {
  // scalar state in SGPRs (the compiler cannot always prove these uniform)
  const int32_t d = uniform(st.d), h = uniform(st.h), lo = uniform(st.lo), hi = uniform(st.hi);
  const int32_t m = uniform(jv.m), n = uniform(jv.n);
  int32_t thr = uniform(st.thr);
  st.h = h;
  const int32_t e = d >> 1;
  const int32_t e0 = e & ~15;
  const int64_t reach = ((int64_t)(jv.m + jv.n) >> 4) + 16;
  const AsmView av_a = make_asm_view(P.A, P.a_words, jv.a_start, reach);
  const AsmView av_b = make_asm_view(P.B, P.b_words, jv.b_start, reach);
  // windows of block e0: A for even and odd anti-diagonals, and B, per register
  const vint l = lane_index();
  const vint i0 = l + (h + e0), i1 = i0 + 64;
  const vint j0 = splat(e0 - h) - l, j1 = j0 - 64;
  Win w0 = make_win<FWD>(av_a, FWD ? i0 - 1 : splat(-14) - i0);
  Win w1 = make_win<FWD>(av_a, FWD ? i0 + 0 : splat(-15) - i0);
  Win w2 = make_win<FWD>(av_b, FWD ? j0 - 1 : splat(-14) - j0);
  Win w3 = make_win<FWD>(av_a, FWD ? i1 - 1 : splat(-14) - i1);
  Win w4 = make_win<FWD>(av_a, FWD ? i1 + 0 : splat(-15) - i1);
  Win w5 = make_win<FWD>(av_b, FWD ? j1 - 1 : splat(-14) - j1);
  {
    const vint b0 = funnel_shr(w2.hi, w2.lo, w2.sh), b1 = funnel_shr(w5.hi, w5.lo, w5.sh);
    vint xe0 = funnel_shr(w0.hi, w0.lo, w0.sh) ^ b0, xo0 = funnel_shr(w1.hi, w1.lo, w1.sh) ^ b0;
    vint xe1 = funnel_shr(w3.hi, w3.lo, w3.sh) ^ b1, xo1 = funnel_shr(w4.hi, w4.lo, w4.sh) ^ b1;
    if (!FWD) {
      xe0 = bit_reverse(xe0); xo0 = bit_reverse(xo0);
      xe1 = bit_reverse(xe1); xo1 = bit_reverse(xo1);
    }
    const int32_t fold = FOLD ? 0x55555555 : 0;   // P.fold, known here
    bd.SE[0] = score_word<true>(xe0, P.pat, fold); bd.SO[0] = score_word<true>(xo0, P.pat, fold);
    bd.SE[1] = score_word<true>(xe1, P.pat, fold); bd.SO[1] = score_word<true>(xo1, P.pat, fold);
  }
  // the window stays inside the matrix for blocks ending at or before e_lim
  int32_t e_lim = m - (2 * kWave - 1) - h;
  if (h + n < e_lim) e_lim = h + n;
  const int32_t lim2 = 2 * (e_lim - 16);
  int32_t e0x2 = 2 * e0, pos = 2 * (e - e0), par = d & 1, status = 0;
  int32_t a = 0, f = 0, bs = 0, bpos = -1;
  uint64_t r0 = ~0ull << lo, r1 = ~0ull >> (2 * kWave - 1 - hi);
  uint64_t v0 = 0, v1 = 0, tq = 0;
  const uint64_t e1 = 0xE000000000000000ull, l0 = 1ull, l63 = 1ull << 63;
  const int32_t hi_a = av_a.hi_rel << 2, hi_b = av_b.hi_rel << 2;   // bytes
  const uint32_t *base_a = av_a.base, *base_b = av_b.base;
  const int32_t ng1 = P.neg_gap + 1;
  int32_t bw = uniform(st.bw);
  vint cnt = splat(0);
  int32_t u, t0, t1, x0, x1, x2, p0, p1, p2, p3, p4, p5;
#define W2_ASM_BODY(SHIFTW, REV)                                                      \
  asm volatile(                                                                       \
      "s_nop 4\n\t"                                                                   \
      XD_PREFETCH("0", "hi_a", "base_a")                                              \
      XD_PREFETCH("1", "hi_a", "base_a")                                              \
      XD_PREFETCH("2", "hi_b", "base_b")                                              \
      XD_PREFETCH("3", "hi_a", "base_a")                                              \
      XD_PREFETCH("4", "hi_a", "base_a")                                              \
      XD_PREFETCH("5", "hi_b", "base_b")                                              \
      "s_add_i32 s42, %[pos], %[par]\n\t"                                             \
      "s_lshl_b32 s42, s42, 2\n\t"                                                    \
      "s_getpc_b64 s[40:41]\n"                                                        \
      ".Lbase_%=:\n\t"                                                                 \
      "s_add_u32 s40, s40, s42\n\t"                                                   \
      "s_addc_u32 s41, s41, 0\n\t"                                                    \
      "s_add_u32 s40, s40, .Ltab_%=-.Lbase_%=\n\t"                                      \
      "s_addc_u32 s41, s41, 0\n\t"                                                    \
      "s_nop 0\n\t"                                                                   \
      "s_setpc_b64 s[40:41]\n"                                                        \
      ".Ltab_%=:\n\t"                                                                  \
      XD_ALL_TABLE                                                                    \
      W2_ALL_PAIRS                                                                    \
      "s_add_i32 %[e0x2], %[e0x2], 32\n\t"                                            \
      "s_cmp_gt_i32 %[e0x2], %[lim2]\n\t"                                             \
      "s_cbranch_scc1 .Lleave_%=\n\t"                                                  \
      "s_waitcnt vmcnt(0)\n\t"                                                        \
      SHIFTW("0") SHIFTW("1") SHIFTW("2") SHIFTW("3") SHIFTW("4") SHIFTW("5")         \
      XD_PREFETCH("0", "hi_a", "base_a")                                              \
      XD_PREFETCH("1", "hi_a", "base_a")                                              \
      XD_PREFETCH("2", "hi_b", "base_b")                                              \
      XD_PREFETCH("3", "hi_a", "base_a")                                              \
      XD_PREFETCH("4", "hi_a", "base_a")                                              \
      XD_PREFETCH("5", "hi_b", "base_b")                                              \
      W2_WORDS(REV, "0", "1", "2", "SE0", "SO0")                                      \
      W2_WORDS(REV, "3", "4", "5", "SE1", "SO1")                                      \
      "s_branch .Le0_%=\n"                                                             \
      W2_ALL_STUBS                                                                    \
      ".Lleave_%=:\n\t"                                                                \
      "s_mov_b32 %[pos], 0\n\t"                                                       \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 3\n"                                                      \
      ".Lexit_%=:\n\t"                                                                 \
      "s_waitcnt vmcnt(0)\n"                                                          \
      : [E0] "+v"(bd.E[0].x), [E1] "+v"(bd.E[1].x), [O0] "+v"(bd.O[0].x),             \
        [O1] "+v"(bd.O[1].x), [SE0] "+v"(bd.SE[0].x), [SE1] "+v"(bd.SE[1].x),         \
        [SO0] "+v"(bd.SO[0].x), [SO1] "+v"(bd.SO[1].x), [cnt] "+v"(cnt.x),            \
        [bw] "+v"(bw),                                                                \
        [lo0] "+v"(w0.lo.x), [hi0] "+v"(w0.hi.x), [nx0] "+v"(w0.nx.x), [idx0] "+v"(w0.idx.x), \
        [lo1] "+v"(w1.lo.x), [hi1] "+v"(w1.hi.x), [nx1] "+v"(w1.nx.x), [idx1] "+v"(w1.idx.x), \
        [lo2] "+v"(w2.lo.x), [hi2] "+v"(w2.hi.x), [nx2] "+v"(w2.nx.x), [idx2] "+v"(w2.idx.x), \
        [lo3] "+v"(w3.lo.x), [hi3] "+v"(w3.hi.x), [nx3] "+v"(w3.nx.x), [idx3] "+v"(w3.idx.x), \
        [lo4] "+v"(w4.lo.x), [hi4] "+v"(w4.hi.x), [nx4] "+v"(w4.nx.x), [idx4] "+v"(w4.idx.x), \
        [lo5] "+v"(w5.lo.x), [hi5] "+v"(w5.hi.x), [nx5] "+v"(w5.nx.x), [idx5] "+v"(w5.idx.x), \
        [u] "=&v"(u), [t0] "=&v"(t0), [t1] "=&v"(t1), [x0] "=&v"(x0), [x1] "=&v"(x1), \
        [x2] "=&v"(x2), [p0] "=&v"(p0), [p1] "=&v"(p1), [p2] "=&v"(p2), [p3] "=&v"(p3), \
        [p4] "=&v"(p4), [p5] "=&v"(p5),                                               \
        [thr] "+s"(thr), [bs] "+s"(bs), [bpos] "+s"(bpos), [par] "+s"(par),        \
        [pos] "+s"(pos), [e0x2] "+s"(e0x2), [r0] "+s"(r0), [r1] "+s"(r1),              \
        [v0] "+s"(v0), [v1] "+s"(v1), [a] "+s"(a), [f] "+s"(f), [tq] "+s"(tq),         \
        [status] "+s"(status)                                                         \
      : [sh0] "v"(w0.sh.x), [sh1] "v"(w1.sh.x), [sh2] "v"(w2.sh.x), [sh3] "v"(w3.sh.x), \
        [sh4] "v"(w4.sh.x), [sh5] "v"(w5.sh.x), [base] "s"(P.dbase), [ng] "s"(P.neg_gap), \
        [ng1] "s"(ng1), [lim2] "s"(lim2), [e1] "s"(e1), [l0] "s"(l0), [l63] "s"(l63),  \
        [pat] "s"(P.pat), [hi_a] "s"(hi_a), [hi_b] "s"(hi_b), [base_a] "s"(base_a),    \
        [base_b] "s"(base_b)                                                          \
      : "vcc", "scc", "memory", "s40", "s41", "s42")
  if (FOLD) {   // +1/-1/-1: base in the score fields
#define W2_DIAG_SEL W2_DIAG_FOLD
#define W2_SW_SEL XD_SW_D2B
    if (FWD) {
      W2_ASM_BODY(XD_SHIFT_FWD, "");
    } else {
      W2_ASM_BODY(XD_SHIFT_BWD, "v_bfrev_b32 %[x0], %[x0]\n\tv_bfrev_b32 %[x1], %[x1]\n\t");
    }
#undef W2_DIAG_SEL
#undef W2_SW_SEL
  } else {
#define W2_DIAG_SEL W2_DIAG_ADD3
#define W2_SW_SEL XD_SW_D2
    if (FWD) {
      W2_ASM_BODY(XD_SHIFT_FWD, "");
    } else {
      W2_ASM_BODY(XD_SHIFT_BWD, "v_bfrev_b32 %[x0], %[x0]\n\tv_bfrev_b32 %[x1], %[x1]\n\t");
    }
#undef W2_DIAG_SEL
#undef W2_SW_SEL
  }
#undef W2_ASM_BODY
  // the anti-diagonal the loop stopped at; W-form thresholds give best there
  const int32_t d_now = e0x2 + pos + par;
  st.d = d_now;
  st.thr = thr;
  st.bw = uniform(bw);
  st.best = st.bw - d_now * P.neg_gap;
  if (bpos >= 0) {   // best cell: i = s + ceil(d/2) + h, j = d - i, d = bpos
    st.bi = bs + ((bpos + 1) >> 1) + h;
    st.bj = bpos - st.bi;
  }
  st.cells += lane_sum(cnt);
  if (status == kW2Step) {
    m0 = v0;
    m1 = v1;
  } else if (status == kW2Recenter) {
    st.lo = a;
    st.hi = 2 * kWave - f;
  } else {
    st.lo = ctz64(r0);
    st.hi = 2 * kWave - 1 - clz64(r1);
  }
  return status;
}

}  // namespace xd
