// xd_matrix.h -- X-drop extension under a 4 x 4 substitution table.
//
// Same computation as the match/mismatch tiers (Section III-A recurrence,
// Algorithms 1 and 2), with the diagonal step scored by a table: aligning
// base p of A with base q of B adds table[4 p + q] (Section VIII names other
// scoring schemes as future work).  One wavefront per job, the band in a
// 64-slot one-register window laid out as in xd_extend.h (lane t holds
// i = t + ceil(d/2) + h; gap-free W form).  The match/mismatch tiers fold the
// score into 2-bit fields of one XOR word; a table needs both bases, so each
// lane keeps 16-base windows of A (one per parity) and of B, extracts both
// codes per cell and reads the score from a 16-entry copy of the table in
// LDS.  A job whose band outgrows 62 slots leaves for the global-memory tier
// (k_spill, which also reads the table) and starts over there.
#pragma once

#include "xd_extend.h"
#include "xd_queue.h"

namespace xd {

// The 16-base windows of one block of 16 steps: A for even and odd
// anti-diagonals, B (the same for both parities).
struct MWin {
  vint ae, ao, b;
};

// Windows of steps e0 .. e0+15 for the window base h.  Step q of a forward
// job sits in field q, of a backward one in field 15 - q.
XD_FN void build_mwin(MWin &w, int32_t e0, int32_t h, const JobView &jv) {
  const vint s = lane_index();
  const vint i0 = s + (h + e0);
  const vint j0 = splat(e0 - h) - s;
  if (jv.dir > 0) {
    w.ae = window16(jv.A, i0 - 1);
    w.ao = window16(jv.A, i0);
    w.b = window16(jv.B, j0 - 1);
  } else {
    w.ae = window16(jv.A, splat(-14) - i0);
    w.ao = window16(jv.A, splat(-15) - i0);
    w.b = window16(jv.B, splat(-14) - j0);
  }
}

// Largest value over the wavefront.
XD_FN int32_t wave_max(vint v) {
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) v = vmax(v, {__shfl_xor(v.x, sh)});
  return uniform(v.x);
}

// Anti-diagonal d = 2 st.e + PAR under the table in LDS (entries hold the
// table plus 2|gap|, the diagonal term of the W form); cur holds d-2 on entry
// and d on exit.  The range is clipped to the matrix on every step.
template <int PAR>
XD_FN int step_m(vint &cur, vint prv, const MWin &w, int pos, W1 &st, const JobView &jv,
                 const int32_t *lut, const Params &P) {
  const vint nbr = PAR ? from_next_lane(prv, kNeg) : from_prev_lane(prv, kNeg);
  const vint ca = bfe_u(PAR ? w.ao : w.ae, pos, 2);
  const vint cb = bfe_u(w.b, pos, 2);
  const vint s = {lut[(ca.x << 2) | cb.x]};
  const vint v = vmax3(cur + s, prv, nbr);
  const uint64_t live = ballot(v >= st.thr) & st.range;
  cur = select(lanes(live), v, kNeg);
  st.cells_blk += (uint32_t)st.width;
  if (live == 0) return kStepDone;
  if (ballot(cur > st.bw) != 0) {   // best rises, by any amount under a table
    const int32_t mx = wave_max(cur);
    const int32_t inc = mx - st.bw;
    st.bw = mx;
    st.thr += inc;
    st.best += inc;
    const int sl = ctz64(ballot(cur == mx));
    st.bi = sl + st.e + PAR + st.h;
    st.bj = 2 * st.e + PAR - st.bi;
  }
  st.bw += P.neg_gap;
  st.thr += P.neg_gap;
  const int a = ctz64(live);
  const int f = clz64(live);
  if (PAR) { st.e += 1; st.par = 0; } else { st.par = 1; }
  int lo = PAR ? a : a - 1;
  int hi = PAR ? 64 - f : 63 - f;
  const int d1 = 2 * st.e + st.par;
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

// Whole extension of one job; kJobWider (with the cells computed so far)
// when the band needs more than 62 slots.
XD_FN JobOut extend_job_matrix(const Job &job, const Params &P, const int32_t *lut) {
  JobOut out;
  out.best = 0; out.bi = 0; out.bj = 0; out.status = kJobOk; out.cells = 0;
  if (job.m + job.n == 0) return out;
  JobView jv;
  jv.A = make_view(P.A, P.a_words, job.a_start);
  jv.B = make_view(P.B, P.b_words, job.b_start);
  jv.a_start = job.a_start; jv.b_start = job.b_start;
  jv.m = job.m; jv.n = job.n; jv.x = job.x; jv.dir = job.dir;
  jv.stage = nullptr;

  vint E = select(lane_index() == 32, splat(0), kNeg);   // anti-diagonal 0: the origin
  vint O = splat(kNeg);
  W1 st;
  st.h = -32;
  st.e = 0;
  st.par = 1;
  {
    const int lo = (jv.n >= 1) ? 31 : 32;
    const int hi = (jv.m >= 1) ? 32 : 31;
    st.width = hi - lo + 1;
    st.range = lane_bits(lo, st.width);
  }
  st.best = 0; st.bi = 0; st.bj = 0;
  st.bw = P.neg_gap;
  st.thr = P.neg_gap - jv.x;
  st.cells_blk = 0;
  st.cells = 0;
  MWin w;
  int32_t w_e0 = -1, w_h = 0;
  for (;;) {
    const int32_t e0 = st.e & ~15;
    if (e0 != w_e0 || st.h != w_h) {
      build_mwin(w, e0, st.h, jv);
      w_e0 = e0;
      w_h = st.h;
    }
    int rc = kStepOn;
    if (st.par) {
      const int q = st.e - e0;
      rc = step_m<1>(O, E, w, jv.dir > 0 ? 2 * q : 30 - 2 * q, st, jv, lut, P);
    }
    while (rc == kStepOn && st.e < e0 + 16) {
      const int q = st.e - e0;
      const int pos = jv.dir > 0 ? 2 * q : 30 - 2 * q;
      rc = step_m<0>(E, O, w, pos, st, jv, lut, P);
      if (rc != kStepOn) break;
      rc = step_m<1>(O, E, w, pos, st, jv, lut, P);
    }
    st.cells += st.cells_blk;
    st.cells_blk = 0;
    if (rc == kStepDone) break;
    if (rc == kStepRecenter) {
      const int width = st.hi - st.lo + 1;
      if (width > kWave - 2) {
        out.status = kJobWider;
        out.cells = st.cells;
        return out;
      }
      const int dl = st.lo - (kWave - width) / 2;
      E = from_lane_offset(E, dl, kNeg);
      O = from_lane_offset(O, dl, kNeg);
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

// One job per wavefront, persistent over the planned order (every job of a
// table call is planned into the first tier).  Jobs whose band outgrows the
// window go to `wider` for the global-memory tier; they start over there.
__global__ __launch_bounds__(256) void k_extend_matrix(const Job *__restrict__ jobs, TierQueue q,
                                                       int32_t *head, JobOut *__restrict__ outs,
                                                       unsigned long long *stats, Params P,
                                                       int32_t *wider, int32_t *wider_count) {
  __shared__ int32_t lut[16];
  if (threadIdx.x < 16) lut[threadIdx.x] = P.lut[threadIdx.x] + 2 * P.neg_gap;
  __syncthreads();
  const int32_t n_init = q.counters[kInit + q.tier];
  int32_t got = 0;
  if (lane_id() == 0) got = atomicAdd(head, 1);
  int32_t w = uniform(got);
  while (w < n_init) {
    const int32_t j = tier_job(q, w, n_init, 0);
    const JobOut o = extend_job_matrix(jobs[j], P, lut);
    if (lane_id() == 0) {
      if (o.status == kJobWider) {
        wider[atomicAdd(wider_count, 1)] = j;
        atomicAdd(&stats[2 * kLists + q.tier], 1ull);
        atomicAdd(&stats[kRestart + q.tier], 1ull);
        atomicAdd(&stats[kWasted + q.tier], (unsigned long long)o.cells);
      } else {
        outs[j] = o;
        atomicAdd(&stats[q.tier], 1ull);
        atomicAdd(&stats[kLists + q.tier], (unsigned long long)o.cells);
      }
    }
    got = 0;
    if (lane_id() == 0) got = atomicAdd(head, 1);
    w = uniform(got);
  }
}

}  // namespace xd
