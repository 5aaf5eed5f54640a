// xd_w1_asm.h -- hand-scheduled gfx950 loop for one-register bands.
//
// Runs anti-diagonals while the 64-lane window stays inside the matrix,
// computing exactly what step_w1<.., false, ..> in xd_extend.h computes, and
// keeps running across score-word blocks: the next block's words are loaded
// a whole block ahead and the score words rebuilt in place, so the loop only
// returns to C code when the extension ends, the band needs recentring, or
// the window approaches the end of a read.
//
// Common path of one anti-diagonal (10 VALU, 6-7 SALU; the 32 anti-diagonals
// of a score-word block are unrolled, so field offsets are immediates):
//   v_mov_b32_dpp  t, prev  wave_shr:1 / wave_shl:1  neighbour diagonal (d-1)
//   v_bfe_u32      u, score_word, 2q, 2              match field
//   v_add3_u32     cur, cur, base, u                 diagonal term (d-2); a VOP2
//                                                    add where base sits in the
//                                                    field (+1/-1/-1)
//   v_max3_i32     cur, cur, prev, t                 the recurrence, gap-free form
//   v_cmp_le_i32   vcc, thr, cur                     X-drop test ...
//   s_and_b64      vcc, vcc, range                   ... within the computed range
//   v_cndmask_b32  cur, -inf, cur, vcc               pruned cells to -inf (VOP2 form:
//                                                    the survivor mask stays in VCC)
//   s_ff1 / s_flbit                                  survivor ends, read before the
//                                                    improvement test takes VCC
//   v_cmp_lt_i32   vcc, bw, cur                      did best improve?
//   v_add / v_add  thr, bw += -gap                   thresholds of d+1
//   s_add / s_sub / s_bfm                            trim: next range mask
//   v_add_u32      cnt, width, cnt                   cells: the next range's width
//                                                    (the s_bfm width, an SGPR)
//                                                    into one VGPR, every lane alike
// The issue slots per anti-diagonal matter less than its dependent chain:
// with one job per wavefront a SIMD runs only a few wavefronts, so the
// kernel is built for the eight resident wavefronts per SIMD that its
// register use allows.
// An improvement of best costs 3 SALU + 1 VALU out of line; best itself is
// not tracked in the loop but recovered from bw afterwards.
// Block transition (every 32 anti-diagonals): 2 window shifts, 2 clamped
// prefetch loads, 3 v_alignbit and a v_cndmask (one A window serves both
// parities), 2 v_xor, 2-4 VALU per score word.
//
// Window edges: an even anti-diagonal may not use lane 0 (wave_shr leaves it
// without a neighbour) and an odd one may not use lane 63.  Checking after
// every odd anti-diagonal that its survivors avoid lanes 0, 62 and 63 keeps
// the next even range inside [1, 62] and the odd range after it inside
// [0, 62], so even anti-diagonals need no check.  The neighbour-less lane
// keeps a stale t, which the range mask discards.  Integer -inf is -2^30,
// whose bit pattern is the inline constant -2.0.  Loads are vector loads of
// clamped, in-bounds word indices; nothing is stored.
#pragma once

#include "xd_extend.h"

namespace xd {

// Packed read addressed for the assembly loop: word indices relative to
// `base` are non-negative and at most hi_rel.
struct AsmView {
  const uint32_t *base;
  int32_t sub;       // start - 16 * (base - words)
  int32_t hi_rel;
};

XD_FN AsmView make_asm_view(const uint32_t *words, int64_t nwords, int64_t start,
                            int64_t reach_words) {
  int64_t wb = (start >> 4) - reach_words;
  if (wb > nwords - 1) wb = nwords - 1;
  if (wb < 0) wb = 0;
  AsmView v;
  v.base = words + wb;
  v.sub = (int32_t)(start - 16 * wb);
  const int64_t hi = nwords - 1 - wb;
  v.hi_rel = (int32_t)(hi > (1 << 28) ? (1 << 28) : hi);
  return v;
}

// One 16-base window of a read, followed from block to block: the words
// (lo, hi) holding it now, the word prefetched for the next block, the index
// of the word to prefetch after that, and the window's bit offset.
struct Win {
  vint lo, hi, nx, idx, sh;   // idx: byte offset of the next word to fetch
};

XD_FN vint load_clamped(const AsmView &v, vint w) { return load_word(v.base, clamp(w, 0, v.hi_rel)); }

// Window state of block e0 for base offset `off` (relative to the read start).
template <bool FWD>
XD_FN Win make_win(const AsmView &v, vint off) {
  Win w;
  const vint g = off + v.sub;
  const vint wi = shr_s(g, 4);
  w.sh = (g & 15) << 1;
  w.lo = load_clamped(v, wi);
  w.hi = load_clamped(v, wi + 1);
  w.idx = (FWD ? wi + 2 : wi - 1) << 2;   // next block's word, as a byte offset
  w.nx = splat(0);
  return w;
}

#define XD_DIAG_NARROW(CUR, SW, P)                      \
  "v_bfe_u32 %[u], %[" SW "], " P ", 2\n\t"             \
  "v_add3_u32 %[" CUR "], %[" CUR "], %[base], %[u]\n\t"
#define XD_DIAG_WIDE(CUR, SW, P)                        \
  "v_bfe_u32 %[u], %[" SW "], " P ", 1\n\t"             \
  "v_mad_u32_u24 %[" CUR "], %[u], %[delta], %[" CUR "]\n\t" \
  "v_add_u32 %[" CUR "], %[base], %[" CUR "]\n\t"

// base + delta * match held in the field itself (+1/-1/-1: 1 or 3), so the
// diagonal term is one VOP2 add after the extract.
#define XD_DIAG_FOLD(CUR, SW, P)                        \
  "v_bfe_u32 %[u], %[" SW "], " P ", 2\n\t"             \
  "v_add_u32 %[" CUR "], %[u], %[" CUR "]\n\t"

// Score word from an XOR of two windows: match bits z = ~(x | x >> 1) & 0x5555..;
// narrow form: delta in every matching 2-bit field; wide form: z itself.
#define XD_SW_NARROW(S, X)                                          \
  "v_lshrrev_b32 %[u], 1, %[" X "]\n\t"                             \
  "v_bitop3_b32 %[u], %[u], %[k55], %[" X "] bitop3:4\n\t"          \
  "v_lshl_add_u32 %[u], %[u], 1, %[u]\n\t"                          \
  "v_and_b32 %[" S "], %[pat], %[u]\n\t"
// delta = 2: ~(x | x << 1) keeps a match flag in the high bit of each field,
// which is the value 2 itself.
#define XD_SW_D2(S, X)                                              \
  "v_lshlrev_b32 %[u], 1, %[" X "]\n\t"                             \
  "v_bitop3_b32 %[" S "], %[u], %[pat], %[" X "] bitop3:4\n\t"
// delta = 2 and base = 1: the high bit of each field as in XD_SW_D2, the low
// bit set, ~(pat & (x | x << 1)), so a field holds base + delta * match.
#define XD_SW_D2B(S, X)                                             \
  "v_lshlrev_b32 %[u], 1, %[" X "]\n\t"                             \
  "v_bitop3_b32 %[" S "], %[u], %[pat], %[" X "] bitop3:0x37\n\t"
#define XD_SW_WIDE(S, X)                                            \
  "v_lshrrev_b32 %[u], 1, %[" X "]\n\t"                             \
  "v_bitop3_b32 %[" S "], %[u], %[k55], %[" X "] bitop3:4\n\t"

// Prefetch of window K's next word (byte offset clamped into the read's view).
#define XD_PREFETCH(K, HI, BASE)                                    \
  "v_med3_i32 %[p" K "], %[idx" K "], 0, %[" HI "]\n\t"             \
  "global_load_dword %[nx" K "], %[p" K "], %[" BASE "]\n\t"

// Window K moves one word along the read.
#define XD_SHIFT_FWD(K)                                             \
  "v_mov_b32 %[lo" K "], %[hi" K "]\n\t"                            \
  "v_mov_b32 %[hi" K "], %[nx" K "]\n\t"                            \
  "v_add_u32 %[idx" K "], 4, %[idx" K "]\n\t"
#define XD_SHIFT_BWD(K)                                             \
  "v_mov_b32 %[hi" K "], %[lo" K "]\n\t"                            \
  "v_mov_b32 %[lo" K "], %[nx" K "]\n\t"                            \
  "v_add_u32 %[idx" K "], -4, %[idx" K "]\n\t"

// Score words of the next block.  One window of A serves both parities: the
// other parity's bases start one base (two bits) further along the same two
// words, which v_alignbit reaches for every lane except those whose window
// starts at bit 30 (mask m30), where the shifted window is exactly `hi`.
// XK is the word of the window kept in registers, XD the derived one.
#define XD_WORDS1(SW, REV, XK, XD)                                  \
  "v_alignbit_b32 %[" XK "], %[hi0], %[lo0], %[sh0]\n\t"            \
  "v_alignbit_b32 %[" XD "], %[hi0], %[lo0], %[shd]\n\t"            \
  "v_cndmask_b32_e64 %[" XD "], %[" XD "], %[hi0], %[m30]\n\t"       \
  "v_alignbit_b32 %[x2], %[hi2], %[lo2], %[sh2]\n\t"                \
  "v_xor_b32 %[x0], %[x0], %[x2]\n\t"                               \
  "v_xor_b32 %[x1], %[x1], %[x2]\n\t"                               \
  REV                                                               \
  SW("SE", "x0")                                                    \
  SW("SO", "x1")
#define XD_WORDS_FWD(SW, REV) XD_WORDS1(SW, REV, "x0", "x1")
#define XD_WORDS_BWD(SW, REV) XD_WORDS1(SW, REV, "x1", "x0")

// Cell update and prune of one anti-diagonal (field P of the score word),
// then its thresholds and survivor ends.  TAG names the step's exits:
// .Ld (nothing survived), .Li (best improved; returns to .Lr, or past the drift
// to .Lq).
#define XD_CORE(TAG, DIAG, CUR, PRV, SW, SHIFT, P, EDGE)                          \
  "v_mov_b32_dpp %[t], %[" PRV "] " SHIFT " row_mask:0xf bank_mask:0xf\n\t"        \
  DIAG(CUR, SW, P)                                                                \
  "v_max3_i32 %[" CUR "], %[" CUR "], %[" PRV "], %[t]\n\t"                        \
  "v_cmp_le_i32 vcc, %[thr], %[" CUR "]\n\t"                                      \
  "s_and_b64 vcc, vcc, %[range]\n\t"                                             \
  "s_cbranch_scc0 .Ld" TAG "_%=\n\t"                                               \
  "v_cndmask_b32_e32 %[" CUR "], -2.0, %[" CUR "], vcc\n\t"                         \
  "s_ff1_i32_b64 %[a], vcc\n\t"                                                  \
  "s_flbit_i32_b64 %[f], vcc\n\t"                                                \
  EDGE                                                                            \
  "v_cmp_lt_i32 vcc, %[bw], %[" CUR "]\n\t"                                       \
  "s_cbranch_vccnz .Li" TAG "_%=\n"                                                \
  ".Lr" TAG "_%=:\n\t"                                                             \
  "v_add_u32 %[thr], %[ng], %[thr]\n\t"                                           \
  "v_add_u32 %[bw], %[ng], %[bw]\n"                                               \
  ".Lq" TAG "_%=:\n\t"

// Even anti-diagonal 2(e0 + K): next (odd) range is lanes [a - 1, 63 - f].
#define XD_EVEN(K, P, DIAG)                                                       \
  ".Le" K "_%=:\n\t"                                                               \
  XD_CORE("e" K, DIAG, "E", "O", "SE", "wave_shr:1", P, "")                       \
  "s_add_i32 %[tmp], %[a], %[f]\n\t"                                              \
  "s_sub_i32 %[tmp], 65, %[tmp]\n\t"                                              \
  "s_add_i32 %[a], %[a], -1\n\t"                                                  \
  "s_bfm_b64 %[range], %[tmp], %[a]\n\t"                                           \
  "v_add_u32 %[cnt], %[tmp], %[cnt]\n"
// Odd anti-diagonal 2(e0 + K) + 1: the next (even) range is [a, 64 - f].  On
// odd K the step first leaves for a recentre (.Lc) when a survivor sits in
// lanes 0-1 or 61-63.  Survivors in lanes [2, 60] there keep the ranges of
// the next four anti-diagonals inside lanes [0, 62], 63 lanes at most, with
// lane 0 out of even ranges and lane 63 out of odd ones (the lanes whose
// shifted neighbour does not exist); the loop is entered only with the
// range inside lanes [2, 60], which bounds the steps before the first check
// the same way.
#define XD_ODD_RANGE                                                              \
  "s_add_i32 %[tmp], %[a], %[f]\n\t"                                              \
  "s_sub_i32 %[tmp], 65, %[tmp]\n\t"                                              \
  "s_bfm_b64 %[range], %[tmp], %[a]\n\t"                                           \
  "v_add_u32 %[cnt], %[tmp], %[cnt]\n"
#define XD_ODD(K, P, DIAG)                                                        \
  ".Lo" K "_%=:\n\t"                                                               \
  XD_CORE("o" K, DIAG, "O", "E", "SO", "wave_shl:1", P, "")                       \
  XD_ODD_RANGE
#define XD_ODD_EDGE(K, P, DIAG)                                                   \
  ".Lo" K "_%=:\n\t"                                                               \
  XD_CORE("o" K, DIAG, "O", "E", "SO", "wave_shl:1", P,                           \
          "s_and_b64 %[live], vcc, %[edge]\n\t")                                   \
  "s_cbranch_scc1 .Lco" K "_%=\n\t"                                                \
  XD_ODD_RANGE
#define XD_PAIR(K, P, DIAG) XD_EVEN(K, P, DIAG) XD_ODD(K, P, DIAG)
#define XD_PAIR_EDGE(K, P, DIAG) XD_EVEN(K, P, DIAG) XD_ODD_EDGE(K, P, DIAG)

// Improvement of best on anti-diagonal e0x2 + BP.  The new best W value is
// bw + inc with the smallest inc that no lane exceeds; with match = 1 it is
// always bw + 1 (best grows by at most `match` per anti-diagonal), so the
// lanes above bw are exactly the lanes holding the new best.  The first of
// them and the anti-diagonal are recorded; (i, j) and best itself are
// derived after the loop.  The unit form applies the anti-diagonal's drift of
// both thresholds together with the raise and rejoins the step after it; it
// records the anti-diagonal in a per-lane register instead (bl: its offset in
// the block for the lanes that raised best, turned into -2 - d at the block's
// end), which leaves the scalar unit and SCC alone, and the lanes holding the
// largest d give the first best cell after the loop.
#define XD_IMP_UNIT(TAG, CUR, BP, TAIL)                                           \
  ".Li" TAG "_%=:\n\t"                                                             \
  "v_cndmask_b32_e64 %[bl], %[bl], " BP ", vcc\n\t"                                \
  "v_add_u32 %[thr], %[ng1], %[thr]\n\t"                                          \
  "v_add_u32 %[bw], %[ng1], %[bw]\n\t"                                            \
  "s_branch .Lq" TAG "_%=\n"
#define XD_IMP_LOOP(TAG, CUR, BP, TAIL)                                           \
  ".Li" TAG "_%=:\n\t"                                                             \
  "s_mov_b32 %[inc], 1\n"                                                         \
  ".Lil" TAG "_%=:\n\t"                                                            \
  "v_add_u32 %[tv], %[inc], %[bw]\n\t"                                            \
  "v_cmp_lt_i32 vcc, %[tv], %[" CUR "]\n\t"                                       \
  "s_cbranch_vccz .Lid" TAG "_%=\n\t"                                              \
  "s_add_i32 %[inc], %[inc], 1\n\t"                                               \
  "s_branch .Lil" TAG "_%=\n"                                                      \
  ".Lid" TAG "_%=:\n\t"                                                            \
  "v_cmp_eq_u32 vcc, %[tv], %[" CUR "]\n\t"                                       \
  "v_mov_b32 %[bw], %[tv]\n\t"                                                    \
  "v_add_u32 %[thr], %[inc], %[thr]\n\t"                                          \
  "s_ff1_i32_b64 %[bs], vcc\n\t"                                                  \
  "s_add_i32 %[bpos], %[e0x2], " BP "\n\t"                                        \
  TAIL                                                                            \
  "s_branch .Lr" TAG "_%=\n"

// Out-of-line exits of the pair K: improvements, end of the extension, and
// the recentre exit of the odd anti-diagonal (which resumes at pair K + 1).
#define XD_STUBS(K, P, P1, PN, IMP)                                               \
  IMP("e" K, "E", P, "")                                                          \
  IMP("o" K, "O", P1, "s_cmp_lg_u64 %[live], 0\n\t")                             \
  ".Lde" K "_%=:\n\t"                                                              \
  "s_mov_b32 %[pos], " P "\n\t"                                                   \
  "s_mov_b32 %[par], 0\n\t"                                                       \
  "s_branch .Ldone_%=\n"                                                           \
  ".Ldo" K "_%=:\n\t"                                                              \
  "s_mov_b32 %[pos], " P "\n\t"                                                   \
  "s_mov_b32 %[par], 1\n\t"                                                       \
  "s_branch .Ldone_%=\n"                                                           \
  ".Lco" K "_%=:\n\t"                                                              \
  "s_mov_b32 %[pos], " PN "\n\t"                                                  \
  "s_branch .Lrec_%=\n"

#define XD_TABLE(K) "s_branch .Le" K "_%=\n\ts_branch .Lo" K "_%=\n\t"

#define XD_ALL_PAIRS(DIAG)                                                        \
  XD_PAIR("0", "0", DIAG) XD_PAIR_EDGE("1", "2", DIAG) XD_PAIR("2", "4", DIAG)    \
  XD_PAIR_EDGE("3", "6", DIAG) XD_PAIR("4", "8", DIAG)                            \
  XD_PAIR_EDGE("5", "10", DIAG) XD_PAIR("6", "12", DIAG)                          \
  XD_PAIR_EDGE("7", "14", DIAG) XD_PAIR("8", "16", DIAG)                          \
  XD_PAIR_EDGE("9", "18", DIAG) XD_PAIR("10", "20", DIAG)                         \
  XD_PAIR_EDGE("11", "22", DIAG) XD_PAIR("12", "24", DIAG)                        \
  XD_PAIR_EDGE("13", "26", DIAG) XD_PAIR("14", "28", DIAG)                        \
  XD_PAIR_EDGE("15", "30", DIAG)
#define XD_ALL_STUBS(IMP)                                                         \
  XD_STUBS("0", "0", "1", "2", IMP) XD_STUBS("1", "2", "3", "4", IMP)             \
  XD_STUBS("2", "4", "5", "6", IMP) XD_STUBS("3", "6", "7", "8", IMP)             \
  XD_STUBS("4", "8", "9", "10", IMP) XD_STUBS("5", "10", "11", "12", IMP)         \
  XD_STUBS("6", "12", "13", "14", IMP) XD_STUBS("7", "14", "15", "16", IMP)       \
  XD_STUBS("8", "16", "17", "18", IMP) XD_STUBS("9", "18", "19", "20", IMP)       \
  XD_STUBS("10", "20", "21", "22", IMP) XD_STUBS("11", "22", "23", "24", IMP)     \
  XD_STUBS("12", "24", "25", "26", IMP) XD_STUBS("13", "26", "27", "28", IMP)     \
  XD_STUBS("14", "28", "29", "30", IMP) XD_STUBS("15", "30", "31", "32", IMP)
#define XD_ALL_TABLE                                                              \
  XD_TABLE("0") XD_TABLE("1") XD_TABLE("2") XD_TABLE("3") XD_TABLE("4")           \
  XD_TABLE("5") XD_TABLE("6") XD_TABLE("7") XD_TABLE("8") XD_TABLE("9")           \
  XD_TABLE("10") XD_TABLE("11") XD_TABLE("12") XD_TABLE("13") XD_TABLE("14")      \
  XD_TABLE("15")

enum : int { kStepLeave = 3 };
// Lanes [2, 60]: the assembly loop starts only with the computed range inside
// them (its edge checks come every fourth anti-diagonal).
constexpr uint64_t kAsmEntryLanes = ((1ull << 59) - 1ull) << 2;

template <bool NARROW, bool UNIT, bool FWD, bool D2, bool FOLD = false>
XD_FN int run_w1_asm(Band<1> &bd, W1 &st, int32_t e0, const JobView &jv,
                     const AsmView &av_a, const AsmView &av_b, const Params &P,
                     int32_t &words_e0) {
  // windows of block e0: A (the parity whose bases start lower in memory:
  // even forwards, odd backwards; the other parity is derived) and B
  const vint s = lane_index();
  const vint i0 = s + (st.h + e0);
  const vint j0 = splat(e0 - st.h) - s;
  Win w0 = make_win<FWD>(av_a, FWD ? i0 - 1 : splat(-15) - i0);
  Win w2 = make_win<FWD>(av_b, FWD ? j0 - 1 : splat(-14) - j0);
  const vint shd = (w0.sh + 2) & 31;
  const uint64_t m30 = ballot(w0.sh == 30);
  int32_t e0x2 = 2 * e0;
  // the window stays inside the matrix for blocks ending at or before e_lim
  int32_t e_lim = jv.m - (kWave - 1) - st.h;
  if (st.h + jv.n < e_lim) e_lim = st.h + jv.n;
  // at most 2^24 anti-diagonals per call: the cell count stays below 2^32
  if (e_lim > e0 + (1 << 23)) e_lim = e0 + (1 << 23);
  const int32_t lim2 = uniform(2 * (e_lim - 16));
  int32_t status = 0;
  int32_t pos = 2 * (st.e - e0);
  int32_t a = 0, f = 0, tmp = 0, inc = 0;
  int32_t bs = 0, bpos = -1;   // lane and anti-diagonal of the last improvement
  vint bl = splat(-1);          // the same, per lane, in the unit form (none: -1)
  // cells: each range's width (its s_bfm width) added when it is computed, the
  // entry range's here; the same in every lane
  int32_t cntv = __builtin_popcountll(st.range);
  uint64_t live = 0;
  const uint64_t edge = 0xE000000000000003ull;   // lanes 0, 1, 61, 62, 63
  const int32_t k55 = 0x55555555;
  const int32_t ng1 = P.neg_gap + 1;   // drift of an anti-diagonal that raised best by 1
  const int32_t hi_a = av_a.hi_rel << 2, hi_b = av_b.hi_rel << 2;   // bytes
  const uint32_t *base_a = av_a.base, *base_b = av_b.base;
  int32_t par = st.par;
  int32_t bw = st.bw;
  int32_t thrv = st.thr;   // the prune threshold in a VGPR: its drift is a VOP2 add, off the scalar unit
  int32_t u, t, tv, x0, x1, x2, p0, p2;
  // score words of block e0 (the loop rebuilds them at each later block)
  {
    const vint xk = funnel_shr(w0.hi, w0.lo, w0.sh);
    const vint xd = select(lanes(m30), w0.hi, funnel_shr(w0.hi, w0.lo, shd));
    const vint xb = funnel_shr(w2.hi, w2.lo, w2.sh);
    vint xe = (FWD ? xk : xd) ^ xb;
    vint xo = (FWD ? xd : xk) ^ xb;
    if (!FWD) { xe = bit_reverse(xe); xo = bit_reverse(xo); }
    const int32_t fold = FOLD ? 0x55555555 : 0;   // P.fold, known here
    bd.SE[0] = score_word<NARROW>(xe, P.pat, fold);
    bd.SO[0] = score_word<NARROW>(xo, P.pat, fold);
  }
  // The 32 anti-diagonals of a block are unrolled, so field offsets and
  // anti-diagonal numbers are immediates; entry jumps through a table of
  // branches indexed by the step within the block (pos + par).
#define XD_ASM_BODY(DIAG, IMP, SW, SHIFTW, REV, WORDS)                                \
  asm volatile(                                                                       \
      "s_nop 4\n\t"                                                                   \
      XD_PREFETCH("0", "hi_a", "base_a")                                              \
      XD_PREFETCH("2", "hi_b", "base_b")                                              \
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
      XD_ALL_PAIRS(DIAG)                                                              \
      "v_cmp_le_i32 vcc, 0, %[bl]\n\t"                                                \
      "s_sub_i32 %[tmp], -2, %[e0x2]\n\t"                                             \
      "v_sub_u32_e32 %[tv], %[tmp], %[bl]\n\t"                                        \
      "v_cndmask_b32_e32 %[bl], %[bl], %[tv], vcc\n\t"                                \
      "s_add_i32 %[e0x2], %[e0x2], 32\n\t"                                            \
      "s_cmp_gt_i32 %[e0x2], %[lim2]\n\t"                                             \
      "s_cbranch_scc1 .Lleave_%=\n\t"                                                  \
      "s_waitcnt vmcnt(0)\n\t"                                                        \
      SHIFTW("0") SHIFTW("2")                                                         \
      XD_PREFETCH("0", "hi_a", "base_a")                                              \
      XD_PREFETCH("2", "hi_b", "base_b")                                              \
      WORDS(SW, REV)                                                                  \
      "s_branch .Le0_%=\n"                                                             \
      XD_ALL_STUBS(IMP)                                                               \
      ".Ldone_%=:\n\t"                                                                 \
      "s_mov_b32 %[status], 1\n\t"                                                    \
      "s_branch .Lexit_%=\n"                                                           \
      ".Lrec_%=:\n\t"                                                                  \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 2\n\t"                                                    \
      "s_branch .Lexit_%=\n"                                                           \
      ".Lleave_%=:\n\t"                                                                \
      "s_mov_b32 %[pos], 0\n\t"                                                       \
      "s_mov_b32 %[par], 0\n\t"                                                       \
      "s_mov_b32 %[status], 3\n"                                                      \
      ".Lexit_%=:\n\t"                                                                 \
      "s_waitcnt vmcnt(0)\n"                                                          \
      : [E] "+v"(bd.E[0].x), [O] "+v"(bd.O[0].x), [cnt] "+v"(cntv), [bw] "+v"(bw),   \
        [SE] "+v"(bd.SE[0].x), [SO] "+v"(bd.SO[0].x),                                 \
        [lo0] "+v"(w0.lo.x), [hi0] "+v"(w0.hi.x), [nx0] "+v"(w0.nx.x), [idx0] "+v"(w0.idx.x), \
        [lo2] "+v"(w2.lo.x), [hi2] "+v"(w2.hi.x), [nx2] "+v"(w2.nx.x), [idx2] "+v"(w2.idx.x), \
        [u] "=&v"(u), [t] "=&v"(t), [tv] "=&v"(tv), [x0] "=&v"(x0), [x1] "=&v"(x1),   \
        [x2] "=&v"(x2), [p0] "=&v"(p0), [p2] "=&v"(p2),               \
        [thr] "+v"(thrv), [bl] "+v"(bl.x), [bs] "+s"(bs), [bpos] "+s"(bpos),       \
        [par] "+s"(par), [pos] "+s"(pos), [e0x2] "+s"(e0x2), [range] "+s"(st.range),  \
        [live] "+s"(live), [a] "+s"(a), [f] "+s"(f), [tmp] "+s"(tmp), [inc] "+s"(inc), \
        [status] "+s"(status)                                                         \
      : [sh0] "v"(w0.sh.x), [shd] "v"(shd.x), [m30] "s"(m30), [sh2] "v"(w2.sh.x),     \
        [base] "s"(P.dbase),                                                           \
        [delta] "s"(P.delta), [ng] "s"(P.neg_gap), [ng1] "s"(ng1), [lim2] "s"(lim2),   \
        [edge] "s"(edge),                                                             \
        [k55] "s"(k55), [pat] "s"(P.pat), [hi_a] "s"(hi_a), [hi_b] "s"(hi_b),          \
        [base_a] "s"(base_a), [base_b] "s"(base_b)                                    \
      : "vcc", "scc", "memory", "s40", "s41", "s42")
#define XD_REV_NONE ""
#define XD_REV_BOTH "v_bfrev_b32 %[x0], %[x0]\n\tv_bfrev_b32 %[x1], %[x1]\n\t"
  if (FOLD) {   // +1/-1/-1: base 1 folded into the fields
    if (FWD) { XD_ASM_BODY(XD_DIAG_FOLD, XD_IMP_UNIT, XD_SW_D2B, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
    else { XD_ASM_BODY(XD_DIAG_FOLD, XD_IMP_UNIT, XD_SW_D2B, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
  } else if (D2) {   // match = 1 and match - mismatch = 2
    if (FWD) { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_UNIT, XD_SW_D2, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
    else { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_UNIT, XD_SW_D2, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
  } else if (FWD) {
    if (NARROW) {
      if (UNIT) { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_UNIT, XD_SW_NARROW, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
      else { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_LOOP, XD_SW_NARROW, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
    } else {
      if (UNIT) { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMP_UNIT, XD_SW_WIDE, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
      else { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMP_LOOP, XD_SW_WIDE, XD_SHIFT_FWD, XD_REV_NONE, XD_WORDS_FWD); }
    }
  } else {
    if (NARROW) {
      if (UNIT) { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_UNIT, XD_SW_NARROW, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
      else { XD_ASM_BODY(XD_DIAG_NARROW, XD_IMP_LOOP, XD_SW_NARROW, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
    } else {
      if (UNIT) { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMP_UNIT, XD_SW_WIDE, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
      else { XD_ASM_BODY(XD_DIAG_WIDE, XD_IMP_LOOP, XD_SW_WIDE, XD_SHIFT_BWD, XD_REV_BOTH, XD_WORDS_BWD); }
    }
  }
#undef XD_REV_NONE
#undef XD_REV_BOTH
#undef XD_ASM_BODY
  // the anti-diagonal the loop stopped at: d = e0x2 + pos + par; W-form
  // thresholds satisfy bw = best + d |gap| there, which gives best
  const int32_t d_now = e0x2 + pos + par;
  // a leave at a block boundary has computed, and counted, the range of an
  // anti-diagonal the C steps will compute
  st.cells += (uint32_t)uniform(cntv) -
              (status == kStepLeave ? (uint64_t)__builtin_popcountll(st.range) : 0ull);
  st.bw = uniform(bw);
  st.thr = uniform(thrv);
  st.best = st.bw - d_now * P.neg_gap;
  if (UNIT) {   // records: block offsets of block e0x2 (>= 0), or -2 - d
    const vint dl = select(bl >= 0, bl + splat(e0x2), splat(-2) - bl);
    bpos = lane_max(dl);
    if (bpos >= 0) bs = __builtin_ctzll(ballot(dl == bpos));
  }
  if (bpos >= 0) {   // best cell: i = s + ceil(d/2) + h, j = d - i, d = bpos
    st.bi = bs + ((bpos + 1) >> 1) + st.h;
    st.bj = bpos - st.bi;
  }
  const int32_t e0_now = e0x2 >> 1;
  st.e = e0_now + (pos >> 1);
  st.par = par;
  st.width = __builtin_popcountll(st.range);
  // the score words in SE/SO belong to block e0_now unless the loop left at a
  // block boundary before rebuilding them
  words_e0 = (status == kStepLeave) ? -1 : e0_now;
  if (status == 2) {   // pending even range [a, 64 - f] needs the window moved
    st.lo = a;
    st.hi = 64 - f;
    return kStepRecenter;
  }
  if (status == 1) return kStepDone;
  return kStepOn;
}
// Runner of extend_job_w1: the assembly loop inside the matrix, the C loop
// (with matrix clipping) near the ends of the reads.
struct RunAsm {
  template <bool NARROW, bool CLIP>
  XD_MEMBER static int run(Band<1> &bd, W1 &st, int32_t e0, int32_t e_end,
                           const JobView &jv, const Params &P, int32_t &words_e0,
                           int32_t &words_h) {
    if constexpr (CLIP) {
      ensure_words_w1<NARROW>(bd, st, e0, jv, P, words_e0, words_h);
      return run_w1<NARROW, true>(bd, st, e0, e_end, jv, P);
    } else {
      if (st.range & ~kAsmEntryLanes) {   // too near the edges: C steps for this block
        ensure_words_w1<NARROW>(bd, st, e0, jv, P, words_e0, words_h);
        return run_w1<NARROW, false>(bd, st, e0, e_end, jv, P);
      }
      const int64_t reach = ((int64_t)(jv.m + jv.n) >> 4) + 16;
      const AsmView av_a = make_asm_view(P.A, P.a_words, jv.a_start, reach);
      const AsmView av_b = make_asm_view(P.B, P.b_words, jv.b_start, reach);
      // the loop leaves score words of block words_e0 built for this window base
      words_h = st.h;
      if (NARROW && P.fold) {   // +1/-1/-1
        return jv.dir > 0
                   ? run_w1_asm<NARROW, true, true, true, true>(bd, st, e0, jv, av_a, av_b, P, words_e0)
                   : run_w1_asm<NARROW, true, false, true, true>(bd, st, e0, jv, av_a, av_b, P, words_e0);
      }
      if (NARROW && P.unit_match && P.delta == 2) {
        return jv.dir > 0
                   ? run_w1_asm<NARROW, true, true, true>(bd, st, e0, jv, av_a, av_b, P, words_e0)
                   : run_w1_asm<NARROW, true, false, true>(bd, st, e0, jv, av_a, av_b, P, words_e0);
      }
      if (jv.dir > 0) {
        return P.unit_match
                   ? run_w1_asm<NARROW, true, true, false>(bd, st, e0, jv, av_a, av_b, P, words_e0)
                   : run_w1_asm<NARROW, false, true, false>(bd, st, e0, jv, av_a, av_b, P, words_e0);
      }
      return P.unit_match
                 ? run_w1_asm<NARROW, true, false, false>(bd, st, e0, jv, av_a, av_b, P, words_e0)
                 : run_w1_asm<NARROW, false, false, false>(bd, st, e0, jv, av_a, av_b, P, words_e0);
    }
  }
};

}  // namespace xd
