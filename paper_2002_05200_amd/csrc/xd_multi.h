// xd_multi.h -- X-drop extension of one job by a whole workgroup, for bands
// wider than one wavefront's registers hold (more than 2,046 cells).
//
// NW wavefronts each own a chunk of C registers (64 C slots, in runs of 64
// consecutive slots per register as in xd_wide.h), so the window is 64 C NW
// diagonal slots.  Per anti-diagonal
// every wave updates the part of the computed range that falls in its chunk
// with the single-wave step, clips its edge registers, and posts to LDS
//   * its chunk's first and last slot values (the neighbours the adjacent
//     waves need on the next anti-diagonal), and
//   * its first and last survivor and its best value with the first slot
//     holding it;
// after one barrier every wave reduces the posts identically (first live =
// min, last live = max, best = max with the lowest slot), so all waves carry
// the same scalar state and take the same branches.  Posts alternate between
// two LDS buffers by parity, so one barrier per anti-diagonal suffices.  This
// is the paper's many-threads-per-alignment layout (Section IV-A) with the
// band in registers instead of global memory.
#pragma once

#include "xd_wide.h"
#include "xd_queue.h"

namespace xd {

// Shapes: NW wavefronts per job, C registers per wavefront.  4 x 16 (4,096
// slots, two workgroups per CU) takes the bands no single wavefront holds;
// the multi_wave option's shapes (2 or 4 wavefronts sharing a tier's
// registers) shorten each anti-diagonal of very long jobs by spreading a
// band one wavefront could hold over several.
template <int NW, int C>
struct MwShape {
  static constexpr int kChunk = 64 * C;
  static constexpr int kSlots = kChunk * NW;
  static constexpr int kThreads = 64 * NW;
};

template <int NW, int C>
struct MwShared {
  int32_t job;
  int32_t edge[2][NW][2];   // by parity: chunk's first and last slot value
  int32_t red[2][NW][4];    // by parity: first, last, best value, its slot
  int32_t stage[64 * C * NW];   // window moves: one anti-diagonal by slot
  int32_t save_off;             // escalation save slot of the current job
  uint32_t words[NW][2 * kStageWords<C>];   // each wave's packed words for its score words
};

// Block-wide scalar state (every wave keeps an identical copy).
struct MwScalars {
  int32_t d, lo, hi, h;           // global slots
  int32_t best, bi, bj, bw, thr;
  int32_t span_lo[2], span_hi[2]; // this wave's registers last computed per parity
  int32_t w_lo, w_hi;             // this wave's registers with score words
  uint32_t cells_blk;
  uint64_t cells;
};

// Score words of every register of this wave's chunk (starting at slot
// base), staged through the wave's own LDS words as in wbuild; the
// requested range [r0, r1] is always inside.
template <int C, bool NARROW>
XD_FN void mw_build(WBand<C> &bd, MwScalars &st, int32_t base, int32_t e0, int32_t r0,
                    int32_t r1, const JobView &jv, const Params &P, uint32_t *words) {
  (void)r0;
  (void)r1;
  if (jv.dir > 0) wbuild_dir<C, NARROW, 1>(bd, st.h, e0, base, words, jv, P);
  else wbuild_dir<C, NARROW, -1>(bd, st.h, e0, base, words, jv, P);
  st.w_lo = 0;
  st.w_hi = C - 1;
}

// Posts both parities' chunk-edge values (after the band was (re)loaded).
template <int NW, int C>
XD_FN void mw_post_edges(const WBand<C> &bd, MwShared<NW, C> &sh, int w) {
  if (lane_id() == 0) {
    sh.edge[0][w][0] = readlane(bd.E[0], 0);
    sh.edge[0][w][1] = readlane(bd.E[C - 1], 63);
    sh.edge[1][w][0] = readlane(bd.O[0], 0);
    sh.edge[1][w][1] = readlane(bd.O[C - 1], 63);
  }
}

// Anti-diagonal st.d (parity PAR).  Returns false once the extension ended.
template <int NW, int C, bool NARROW, int PAR, bool ASM>
XD_FN bool mw_step(WBand<C> &bd, MwScalars &st, MwShared<NW, C> &sh, int w, int q,
                   const JobView &jv, const Params &P) {
  vint *cur = PAR ? bd.O : bd.E;
  const vint *prv = PAR ? bd.E : bd.O;
  const vint *sw = PAR ? bd.SO : bd.SE;
  const int pos = 2 * q;
  const int base = w * (64 * C);
  // this chunk's part of the range
  const int cl = st.lo - base > 0 ? st.lo - base : 0;
  const int ch = st.hi - base < (64 * C) - 1 ? st.hi - base : (64 * C) - 1;
  const bool active = cl <= ch;
  const int rlo = active ? cl >> 6 : 1, rhi = active ? ch >> 6 : 0;
  const int plo = st.span_lo[PAR], phi = st.span_hi[PAR];
  if (plo < rlo || phi > rhi) {
#pragma unroll
    for (int r = 0; r < C; ++r)
      if ((r < rlo || r > rhi) && r >= plo && r <= phi) cur[r] = splat(kNeg);
  }
  int first = 0x7fffffff, last = -1, bestv = kNeg, bests = 0x7fffffff;
  if (active) {
    if (rlo < st.w_lo || rhi > st.w_hi)
      mw_build<C, NARROW>(bd, st, base, (st.d >> 1) - q, rlo - 1, rhi + 1, jv, P, sh.words[w]);
    // neighbours in the adjacent chunks, posted on the previous anti-diagonal
    const int32_t nb_below = w > 0 ? sh.edge[1 - PAR][w - 1][1] : kNeg;
    const int32_t nb_above = w < NW - 1 ? sh.edge[1 - PAR][w + 1][0] : kNeg;
    const int32_t thr = st.thr, bw = st.bw;
    // the chunk's registers as one chain (see wcell_chain): upwards on even
    // anti-diagonals, downwards on odd ones; the chain's outer neighbour is
    // the adjacent wave's posted edge when the chain starts at the chunk's
    // edge, else -inf unless the range was clipped to the matrix there
    vint carry = splat(kNeg);
    {
      const int c = (st.d + 1) >> 1;
      const int i_min = st.d - jv.n > 0 ? st.d - jv.n : 0;
      if (PAR == 0 && rlo == 0) {
        carry = splat(nb_below);
      } else if (PAR == 1 && rhi == C - 1) {
        carry = splat(nb_above);
      } else if (PAR == 0 ? st.lo <= i_min - c - st.h : st.hi >= jv.m - c - st.h) {
        const int rn = PAR == 0 ? rlo - 1 : rhi + 1;
        switch (rn) {
#define XD_MW_NEIGHBOUR(R)                                                                  \
  case R:                                                                                   \
    if constexpr (R < C) carry = PAR == 0 ? rot_prev(prv[R]) : rot_next(prv[R]);           \
    break;
          XD_MW_NEIGHBOUR(0) XD_MW_NEIGHBOUR(1) XD_MW_NEIGHBOUR(2) XD_MW_NEIGHBOUR(3)
          XD_MW_NEIGHBOUR(4) XD_MW_NEIGHBOUR(5) XD_MW_NEIGHBOUR(6) XD_MW_NEIGHBOUR(7)
          XD_MW_NEIGHBOUR(8) XD_MW_NEIGHBOUR(9) XD_MW_NEIGHBOUR(10) XD_MW_NEIGHBOUR(11)
          XD_MW_NEIGHBOUR(12) XD_MW_NEIGHBOUR(13) XD_MW_NEIGHBOUR(14) XD_MW_NEIGHBOUR(15)
#undef XD_MW_NEIGHBOUR
          default:
            break;
        }
      }
    }
    vint vmx = splat(kNeg);
    uint64_t live_lo, live_hi;
    if constexpr (ASM && NARROW) {
      // the same chain as generated assembly, with the chunk's edge
      // registers clipped inside it
      const int ucl = uniform(cl), uch = uniform(ch);
      const int urlo = uniform(rlo), urhi = uniform(rhi);
      const uint64_t lo_mask = ~0ull << (ucl & 63);
      const uint64_t hi_mask = ~0ull >> (63 - (uch & 63));
      const uint64_t mf =
          urlo == urhi ? (lo_mask & hi_mask) : (PAR == 0 ? lo_mask : hi_mask);
      const uint64_t ml = PAR == 0 ? hi_mask : lo_mask;
      uint64_t lf, ll;
      WChainRun<C, PAR>::run(cur, prv, sw, uniform(pos), uniform(thr), uniform(P.dbase), urlo,
                             urhi, carry, vmx, mf, ml, lf, ll);
      live_lo = PAR == 0 ? lf : ll;
      live_hi = PAR == 0 ? ll : lf;
    } else
    {
      if constexpr (PAR == 0) {
        switch (rlo) {
#define XD_MW_UP(R)                                                                          \
  case R:                                                                                    \
    if constexpr (R < C) {                                                                   \
      wcell_chain<C, NARROW, 0, R>(cur, prv, sw, pos, thr, vmx, carry, P);                  \
      if (rhi == R) break;                                                                   \
    }                                                                                        \
    [[fallthrough]];
          XD_MW_UP(0) XD_MW_UP(1) XD_MW_UP(2) XD_MW_UP(3) XD_MW_UP(4) XD_MW_UP(5) XD_MW_UP(6)
          XD_MW_UP(7) XD_MW_UP(8) XD_MW_UP(9) XD_MW_UP(10) XD_MW_UP(11) XD_MW_UP(12)
          XD_MW_UP(13) XD_MW_UP(14) XD_MW_UP(15)
#undef XD_MW_UP
          default:
            break;
        }
      } else {
        switch (rhi) {
#define XD_MW_DOWN(R)                                                                         \
  case 15 - R:                                                                                \
    if constexpr (15 - R < C) {                                                               \
      wcell_chain<C, NARROW, 1, (15 - R < C ? 15 - R : 0)>(cur, prv, sw, pos, thr, vmx,      \
                                                            carry, P);                       \
      if (rlo == 15 - R) break;                                                               \
    }                                                                                         \
    [[fallthrough]];
          XD_MW_DOWN(0) XD_MW_DOWN(1) XD_MW_DOWN(2) XD_MW_DOWN(3) XD_MW_DOWN(4) XD_MW_DOWN(5)
          XD_MW_DOWN(6) XD_MW_DOWN(7) XD_MW_DOWN(8) XD_MW_DOWN(9) XD_MW_DOWN(10) XD_MW_DOWN(11)
          XD_MW_DOWN(12) XD_MW_DOWN(13) XD_MW_DOWN(14) XD_MW_DOWN(15)
#undef XD_MW_DOWN
          default:
            break;
        }
      }
      const uint64_t lo_mask = ~0ull << (cl & 63);
      const uint64_t hi_mask = ~0ull >> (63 - (ch & 63));
      if (rlo == rhi) {
        live_lo = live_hi = wclip_at<C>(cur, rlo, lo_mask & hi_mask);
      } else {
        live_lo = wclip_at<C>(cur, rlo, lo_mask);
        live_hi = wclip_at<C>(cur, rhi, hi_mask);
      }
    }
    const uint64_t imp = ballot(vmx > bw);
    if (live_lo != 0) {
      first = base + 64 * rlo + ctz64(live_lo);
    } else {
#pragma unroll
      for (int r = 0; r < C; ++r) {
        if (first != 0x7fffffff || r <= rlo || r > rhi) continue;
        const uint64_t m = ballot(cur[r] != kNeg);
        if (m != 0) first = base + 64 * r + ctz64(m);
      }
    }
    if (live_hi != 0) {
      last = base + 64 * rhi + last_bit64(live_hi);
    } else {
#pragma unroll
      for (int r = C - 1; r >= 0; --r) {
        if (last >= 0 || r < rlo || r >= rhi) continue;
        const uint64_t m = ballot(cur[r] != kNeg);
        if (m != 0) last = base + 64 * r + last_bit64(m);
      }
    }
    if (imp != 0 && P.unit_match) {   // best can rise by 1 only: one pass
      if constexpr (ASM && NARROW) {
        const int32_t sb = WFirst<C>::run(cur, uniform(bw), uniform(rlo), uniform(rhi));
        if (sb >= 0) {
          bestv = bw + 1;
          bests = base + sb;
        }
      } else
      {
#pragma unroll
        for (int r = 0; r < C; ++r) {
          if (bests != 0x7fffffff || r < rlo || r > rhi) continue;
          const uint64_t m = ballot(cur[r] > bw);
          if (m != 0) {
            bestv = bw + 1;
            bests = base + 64 * r + ctz64(m);
          }
        }
      }
    } else if (imp != 0) {   // this chunk's best value above bw and its first slot
      int inc = 0;
      for (;;) {
        uint64_t more = 0;
#pragma unroll
        for (int r = 0; r < C; ++r)
          if (r >= rlo && r <= rhi) more |= ballot(cur[r] > bw + inc);
        if (more == 0) break;
        ++inc;
      }
      if (inc > 0) {
        bestv = bw + inc;
#pragma unroll
        for (int r = 0; r < C; ++r) {
          if (bests != 0x7fffffff || r < rlo || r > rhi) continue;
          const uint64_t m = ballot(cur[r] == bestv);
          if (m != 0) bests = base + 64 * r + ctz64(m);
        }
      }
    }
  }
  st.span_lo[PAR] = rlo;
  st.span_hi[PAR] = rhi;
  if (lane_id() == 0) {
    sh.edge[PAR][w][0] = readlane(cur[0], 0);
    sh.edge[PAR][w][1] = readlane(cur[C - 1], 63);
    sh.red[PAR][w][0] = first;
    sh.red[PAR][w][1] = last;
    sh.red[PAR][w][2] = bestv;
    sh.red[PAR][w][3] = bests;
  }
  __syncthreads();
  int gfirst = 0x7fffffff, glast = -1, gbest = kNeg, gslot = 0x7fffffff;
#pragma unroll
  for (int v = 0; v < NW; ++v) {
    const int f = sh.red[PAR][v][0], l = sh.red[PAR][v][1], b = sh.red[PAR][v][2];
    gfirst = f < gfirst ? f : gfirst;
    glast = l > glast ? l : glast;
    if (b > gbest) {   // waves are in slot order: the first wave with the max
      gbest = b;
      gslot = sh.red[PAR][v][3];
    }
  }
  st.cells_blk += (uint32_t)(st.hi - st.lo + 1);
  if (glast < 0) return false;
  if (gbest > st.bw) {
    const int inc = gbest - st.bw;
    st.bw += inc;
    st.thr += inc;
    st.best += inc;
    st.bi = gslot + ((st.d + 1) >> 1) + st.h;
    st.bj = st.d - st.bi;
  }
  const int d1 = st.d + 1;
  if (d1 > jv.m + jv.n) return false;
  int lo = PAR ? gfirst : gfirst - 1;
  int hi = PAR ? glast + 1 : glast;
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

// Window move through the LDS stage, one anti-diagonal at a time: new slot
// s <- old slot s + dl (-inf from outside the window).
template <int NW, int C>
XD_FN void mw_move(vint *a, MwShared<NW, C> &sh, int base, int dl) {
  const vint l = lane_index();
  __syncthreads();                       // the stage is free
#pragma unroll
  for (int r = 0; r < C; ++r) store_vec(sh.stage + base + 64 * r, l, a[r]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < C; ++r) {
    const vint src = l + (base + 64 * r + dl);
    const vbool in = le_u(src, (uint32_t)((64 * C * NW) - 1));
    a[r] = select(in, load_vec(sh.stage, select(in, src, 0)), kNeg);
  }
}

template <int C>
XD_FN void mw_full_spans(MwScalars &st) {
  st.span_lo[0] = st.span_lo[1] = 0;
  st.span_hi[0] = st.span_hi[1] = C - 1;
  st.w_lo = 1;
  st.w_hi = 0;
}

// Moves the whole window so the pending range sits in its middle (through
// the LDS stage).  Returns false when the range is wider than the window.
template <int NW, int C>
XD_FN bool mw_recenter(WBand<C> &bd, MwScalars &st, MwShared<NW, C> &sh, int w) {
  const int width = st.hi - st.lo + 1;
  if (width > (64 * C * NW) - 2) return false;
  const int dl = st.lo - ((64 * C * NW) - width) / 2;
  mw_move<NW, C>(bd.E, sh, w * (64 * C), dl);
  mw_move<NW, C>(bd.O, sh, w * (64 * C), dl);
  st.h += dl;
  st.lo -= dl;
  st.hi -= dl;
  mw_full_spans<C>(st);
  mw_post_edges<NW, C>(bd, sh, w);
  __syncthreads();
  return true;
}

// Restores a single-wave tier's save into the middle of the window.
template <int NW, int C>
XD_FN bool mw_restore(WBand<C> &bd, MwScalars &st, MwShared<NW, C> &sh, int w, const Params &P,
                      int32_t j) {
  if (!P.save_pool || j < 0) return false;
  const int32_t off = P.job_save[j];
  if (off < 0) return false;
  const int32_t *sv = P.save_pool + off;
  const int32_t ss = kWave * sv[kSvC];
  if (ss >= 64 * C * NW) return false;
  const int32_t shift = ((64 * C * NW) - ss) / 2;
  st.d = sv[kSvD];
  st.lo = sv[kSvLo] + shift;
  st.hi = sv[kSvHi] + shift;
  st.h = sv[kSvH] - shift;
  st.best = sv[kSvBest]; st.bi = sv[kSvBi]; st.bj = sv[kSvBj];
  st.bw = sv[kSvBw]; st.thr = sv[kSvThr];
  st.cells = (uint64_t)(uint32_t)sv[kSvCellsLo] | ((uint64_t)(uint32_t)sv[kSvCellsHi] << 32);
  st.cells_blk = 0;
  const vint l = lane_index();
  const int base = w * (64 * C);
#pragma unroll
  for (int r = 0; r < C; ++r) {
    const vint old = l + (base + 64 * r - shift);
    const vbool in = le_u(old, (uint32_t)(ss - 1));
    const vint k = select(in, old, 0);
    bd.E[r] = select(in, load_vec(sv + kSaveHdr, k), kNeg);
    bd.O[r] = select(in, load_vec(sv + kSaveHdr + ss, k), kNeg);
  }
  mw_full_spans<C>(st);
  return true;
}

// Stores the workgroup's state in the job's save slot (slot order, C field =
// slots / 64) for the next, wider tier; nothing when the window is wider than
// a save slot holds or the pool is full.  Returns whether it saved.
template <int NW, int C>
XD_FN bool mw_save(const WBand<C> &bd, const MwScalars &st, MwShared<NW, C> &sh, int w,
                   const Params &P, int32_t j) {
  constexpr int S = 64 * C * NW;
  if (w == 0) {
    int32_t *sv = save_reserve(P, j, S);
    if (lane_id() == 0) sh.save_off = sv ? (int32_t)(sv - P.save_pool) : -1;
    if (sv)
      save_scalars(sv, st.d, st.lo, st.hi, st.h, st.best, st.bi, st.bj, st.bw, st.thr, C * NW,
                   st.cells + st.cells_blk);
  }
  __syncthreads();
  const int32_t off = sh.save_off;
  if (off >= 0) {
    int32_t *sv = P.save_pool + off;
    const vint l = lane_index();
#pragma unroll
    for (int r = 0; r < C; ++r) {
      store_vec(sv + kSaveHdr, l + (w * 64 * C + 64 * r), bd.E[r]);
      store_vec(sv + kSaveHdr + S, l + (w * 64 * C + 64 * r), bd.O[r]);
    }
  }
  __syncthreads();
  if (w == 0 && off >= 0) save_publish(P, j, P.save_pool + off);
  return off >= 0;
}

// Whole extension of job j by the workgroup.  kJobWider when the band
// outgrows the window.
template <int NW, int C, bool NARROW, bool ASM>
XD_FN JobOut mw_extend(const Job &job, const Params &P, int32_t j, MwShared<NW, C> &sh, int w) {
  JobOut out;
  out.best = 0; out.bi = 0; out.bj = 0; out.status = kJobOk; out.cells = 0;
  if (job.m + job.n == 0) return out;
  JobView jv;
  jv.A = make_view(P.A, P.a_words, job.a_start);
  jv.B = make_view(P.B, P.b_words, job.b_start);
  jv.a_start = job.a_start; jv.b_start = job.b_start;
  jv.m = job.m; jv.n = job.n; jv.x = job.x; jv.dir = job.dir;
  jv.stage = nullptr;

  WBand<C> bd;
  MwScalars st;
  if (!mw_restore<NW, C>(bd, st, sh, w, P, j)) {
    // anti-diagonal 0: the origin in slot (64 * C * NW) / 2 (register 0, lane 0 of
    // wave NW / 2)
    const vbool origin = lane_index() == 0;
#pragma unroll
    for (int r = 0; r < C; ++r) {
      bd.E[r] = (r == 0 && w == NW / 2) ? select(origin, splat(0), kNeg) : splat(kNeg);
      bd.O[r] = splat(kNeg);
    }
    st.h = -(64 * C * NW) / 2;
    st.d = 1;
    {
      const int smin = (1 - jv.n > 0 ? 1 - jv.n : 0) - 1 - st.h;
      const int smax = jv.m - 1 - st.h;
      st.lo = ((64 * C * NW) / 2 - 1) > smin ? ((64 * C * NW) / 2 - 1) : smin;
      st.hi = ((64 * C * NW) / 2) < smax ? ((64 * C * NW) / 2) : smax;
    }
    st.best = 0; st.bi = 0; st.bj = 0;
    st.bw = P.neg_gap;
    st.thr = P.neg_gap - jv.x;
    st.cells_blk = 0;
    st.cells = 0;
    mw_full_spans<C>(st);
  }
  mw_post_edges<NW, C>(bd, sh, w);
  __syncthreads();

  int32_t e = st.d >> 1;
  bool odd = (st.d & 1) != 0;
  int32_t e0 = e & ~15;
  bool ok = true;
  for (;;) {
    if (!odd) {
      if (st.lo < 1 || st.hi > (64 * C * NW) - 2) {
        if (!mw_recenter<NW, C>(bd, st, sh, w)) { ok = false; break; }
      }
      if (e - e0 == 16) {
        e0 = e;
        st.cells += st.cells_blk;
        st.cells_blk = 0;
        st.w_lo = 1;
        st.w_hi = 0;
      }
      if (!mw_step<NW, C, NARROW, 0, ASM>(bd, st, sh, w, e - e0, jv, P)) break;   // d = 2e
    }
    odd = false;
    if (st.lo < 1 || st.hi > (64 * C * NW) - 2) {
      if (!mw_recenter<NW, C>(bd, st, sh, w)) { ok = false; break; }
    }
    if (!mw_step<NW, C, NARROW, 1, ASM>(bd, st, sh, w, e - e0, jv, P)) break;     // d = 2e + 1
    ++e;
  }
  if (!ok) {
    out.bi = mw_save<NW, C>(bd, st, sh, w, P, j) ? 1 : 0;
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

// One job per workgroup.  Plain (head == nullptr): workgroup b takes work item
// b.  Persistent: workgroups pop work items.  A job whose band outgrows the
// window is appended to `overflow` (the next tier's escalation list, with its
// state saved, or the global-memory pass's list).
template <int NW, int C, bool NARROW>
__global__ __launch_bounds__(64 * NW) void k_extend_mw(const Job *__restrict__ jobs, TierQueue q,
                                                       int32_t *head, JobOut *__restrict__ outs,
                                                       unsigned long long *stats, Params P,
                                                       int32_t *overflow,
                                                       int32_t *overflow_count) {
  __shared__ MwShared<NW, C> sh;
  const int32_t n_init = q.counters[kInit + q.tier];
  const int32_t n_esc = q.counters[kEsc + q.tier];
  const int32_t count = n_init + n_esc;
  int32_t widx = (int32_t)blockIdx.x;
  for (;;) {
    if (head != nullptr) {
      if (threadIdx.x == 0) sh.job = atomicAdd(head, 1);
      __syncthreads();
      widx = sh.job;
      __syncthreads();
    }
    if (widx >= count) break;
    const int32_t j = tier_job(q, widx, n_init, n_esc);
    const Job job = jobs[j];
    const int w = (int)(threadIdx.x >> 6);
    const JobOut o = NARROW && P.impl == 0 ? mw_extend<NW, C, NARROW, true>(job, P, j, sh, w)
                                           : mw_extend<NW, C, NARROW, false>(job, P, j, sh, w);
    if (threadIdx.x == 0) {
      if (o.status == kJobWider) {
        overflow[atomicAdd(overflow_count, 1)] = j;
        atomicAdd(&stats[2 * kLists + q.tier], 1ull);
        if (o.bi == 0) {
          atomicAdd(&stats[kRestart + q.tier], 1ull);
          atomicAdd(&stats[kWasted + q.tier], (unsigned long long)o.cells);
        }
      } else {
        outs[j] = o;
        atomicAdd(&stats[q.tier], 1ull);
        atomicAdd(&stats[kLists + q.tier], (unsigned long long)o.cells);
      }
    }
    __syncthreads();
    if (head == nullptr) break;
  }
}

}  // namespace xd
