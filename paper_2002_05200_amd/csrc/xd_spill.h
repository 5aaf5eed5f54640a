// xd_spill.h -- unbounded tier: X-drop extension with the band in global
// memory, for jobs whose band outgrows the widest register window.
//
// One 256-thread workgroup per job, persistent over the spill list.  Each
// anti-diagonal is stored compactly over its computed i-range in one of three
// rotating global buffers (Algorithm 1's three anti-diagonals, kept in HBM as
// in Section IV-B); the threads stride over the range (Algorithm 2's
// segments), and block-wide reductions through LDS give the anti-diagonal's
// maximum, its first maximising i and the first/last surviving cell.
#pragma once

#include <hip/hip_runtime.h>

#include "xdrop.h"
#include "xd_jobs.h"
#include "xd_queue.h"

namespace xd {

constexpr int kSpillThreads = 256;
// Jobs whose band outgrows the multi-wave tier's window start over here:
// kHugeSlots workgroups with room for `cap` cells per anti-diagonal (kHugeCap
// unless a memory budget asks for less); a job whose band is wider still
// fails with XD_ENOMEM.
constexpr int kHugeSlots = 8;
constexpr int64_t kHugeCap = (1 << 20) + 4;
constexpr int64_t kHugeCapMin = (1 << 14) + 4;

struct SpillScratch {
  int32_t *huge = nullptr;   // kHugeSlots * 3 * cap
  int64_t cap = 0;
};

constexpr uint64_t spill_bytes(int64_t cap) { return sizeof(int32_t) * 3 * (uint64_t)cap * kHugeSlots; }

// Where a spill pass takes its jobs from: a tier queue, or a plain list.
struct SpillSource {
  TierQueue q;
  const int32_t *list;        // nullptr: the tier queue
  const int32_t *list_count;
  int32_t *overflow;          // jobs too wide for this pass (nullptr: fail them)
  int32_t *overflow_count;
  int64_t cap;                // cells per stored anti-diagonal
};

__device__ __forceinline__ uint32_t base_at(const uint32_t *W, int64_t g) {
  return (W[g >> 4] >> (2 * (g & 15))) & 3u;
}

__global__ __launch_bounds__(kSpillThreads) void k_spill(const Job *__restrict__ jobs,
                                                         SpillSource src,
                                                         int32_t *head, JobOut *__restrict__ outs,
                                                         unsigned long long *stats, Params P,
                                                         int32_t *__restrict__ band) {
  __shared__ int32_t s_job;
  __shared__ int32_t s_first, s_last, s_max, s_imax;
  __shared__ int32_t s_lut[16];
  const int tid = threadIdx.x;
  if (tid < 16) s_lut[tid] = P.lut[tid];
  const TierQueue &q = src.q;
  const int32_t n_init = src.list ? 0 : q.counters[kInit + q.tier];
  const int32_t n_esc = src.list ? *src.list_count : q.counters[kEsc + q.tier];
  const int32_t count = n_init + n_esc;
  const int64_t cap = src.cap;
  int32_t *bufs[3];
  for (int t = 0; t < 3; ++t) bufs[t] = band + ((int64_t)blockIdx.x * 3 + t) * cap;
  const int32_t gap = -P.neg_gap;
  const int32_t mismatch = P.base + 2 * gap;
  const int32_t match = mismatch + P.delta;

  for (;;) {
    if (tid == 0) s_job = atomicAdd(head, 1);
    __syncthreads();
    const int32_t w = s_job;
    __syncthreads();
    if (w >= count) break;
    const int32_t j = src.list ? src.list[w] : tier_job(q, w, n_init, n_esc);
    const Job job = jobs[j];
    JobOut out;
    out.best = 0; out.bi = 0; out.bj = 0; out.status = kJobOk; out.cells = 0;
    const int32_t m = job.m, n = job.n;
    bool moved = false;
    // rotating anti-diagonals: [2] = d-2, [1] = d-1, [0] = d
    int32_t *vb[3] = {bufs[0], bufs[1], bufs[2]};
    int32_t lo2 = 1, hi2 = 0;          // d-2 empty
    int32_t lo1 = 0, hi1 = 0;          // d-1 = origin
    if (tid == 0) vb[1][0] = 0;
    int32_t live_lo = 0, live_hi = 0;
    int32_t best = 0, bi = 0, bj = 0;
    uint64_t cells = 0;
    __syncthreads();
    for (int32_t d = 1; d <= m + n; ++d) {
      int32_t lo = live_lo > d - n ? live_lo : d - n;
      int32_t hi = live_hi + 1 < m ? live_hi + 1 : m;
      if (lo > hi) break;
      if ((int64_t)(hi - lo + 1) > cap) {   // band wider than this pass holds
        moved = true;
        break;
      }
      const int32_t thr = best - job.x;
      int32_t my_first = 0x7fffffff, my_last = -1, my_max = kNeg, my_imax = 0x7fffffff;
      for (int32_t i = lo + tid; i <= hi; i += kSpillThreads) {
        const int32_t jj = d - i;
        int32_t v = kNeg;
        if (i >= 1 && jj >= 1 && i - 1 >= lo2 && i - 1 <= hi2) {
          const int32_t p = vb[2][i - 1 - lo2];
          if (p != kNeg) {
            const uint32_t ca = base_at(P.A, job.a_start + (int64_t)job.dir * (i - 1));
            const uint32_t cb = base_at(P.B, job.b_start + (int64_t)job.dir * (jj - 1));
            const int32_t sub =
                P.has_lut ? s_lut[(ca << 2) | cb] : (ca == cb ? match : mismatch);
            const int32_t s = p + sub;
            v = s > v ? s : v;
          }
        }
        if (i >= 1 && i - 1 >= lo1 && i - 1 <= hi1) {
          const int32_t p = vb[1][i - 1 - lo1];
          if (p != kNeg && p + gap > v) v = p + gap;
        }
        if (jj >= 1 && i >= lo1 && i <= hi1) {
          const int32_t p = vb[1][i - lo1];
          if (p != kNeg && p + gap > v) v = p + gap;
        }
        if (v != kNeg && v < thr) v = kNeg;
        vb[0][i - lo] = v;
        if (v != kNeg) {
          if (i < my_first) my_first = i;
          my_last = i;
          if (v > my_max) { my_max = v; my_imax = i; }
        }
      }
      if (tid == 0) { s_first = 0x7fffffff; s_last = -1; s_max = kNeg; s_imax = 0x7fffffff; }
      __syncthreads();
      if (my_last >= 0) {
        atomicMin(&s_first, my_first);
        atomicMax(&s_last, my_last);
        atomicMax(&s_max, my_max);
      }
      __syncthreads();
      if (my_last >= 0 && my_max == s_max) atomicMin(&s_imax, my_imax);
      __syncthreads();
      cells += (uint64_t)(hi - lo + 1);
      const int32_t first = s_first, last = s_last, vmax = s_max, imax = s_imax;
      __syncthreads();
      if (last < 0) break;
      if (vmax > best) { best = vmax; bi = imax; bj = d - imax; }
      live_lo = first;
      live_hi = last;
      int32_t *t = vb[2]; vb[2] = vb[1]; vb[1] = vb[0]; vb[0] = t;
      lo2 = lo1; hi2 = hi1; lo1 = lo; hi1 = hi;
    }
    out.best = best; out.bi = bi; out.bj = bj; out.cells = cells;
    if (tid == 0) {
      if (moved && src.overflow) {
        src.overflow[atomicAdd(src.overflow_count, 1)] = j;
        atomicAdd(&stats[2 * kLists + q.tier], 1ull);
        atomicAdd(&stats[kRestart + q.tier], 1ull);
        atomicAdd(&stats[kWasted + q.tier], (unsigned long long)cells);
      } else {
        if (moved) out.status = XD_ENOMEM;
        outs[j] = out;
        atomicAdd(&stats[q.tier], 1ull);
        atomicAdd(&stats[kLists + q.tier], (unsigned long long)cells);
      }
    }
    __syncthreads();
  }
}

inline xd_status spill_alloc(SpillScratch *sp, int64_t cap) {
  if (!sp->huge) {
    void *p = nullptr;
    if (hipMalloc(&p, spill_bytes(cap)) != hipSuccess) return XD_ENOMEM;
    sp->huge = (int32_t *)p;
    sp->cap = cap;
  }
  return XD_OK;
}

// A global-memory pass over `list` with `groups` workgroups sharing the band
// buffers (each holds cells per anti-diagonal = the buffers / (3 groups)).
// Jobs wider than that go to `overflow` (nullptr: they fail with XD_ENOMEM).
inline xd_status spill_launch(const SpillScratch *sp, hipStream_t s, const Job *jobs,
                              const TierQueue &q, int32_t *head, const int32_t *list,
                              const int32_t *list_count, JobOut *outs,
                              unsigned long long *stats, const Params &P, int groups = kHugeSlots,
                              int32_t *overflow = nullptr, int32_t *overflow_count = nullptr) {
  if (!sp->huge || groups < 1) return XD_ENOMEM;
  SpillSource b;
  b.q = q;
  b.list = list;
  b.list_count = list_count;
  b.overflow = overflow;
  b.overflow_count = overflow_count;
  b.cap = sp->cap * kHugeSlots / groups;
  hipLaunchKernelGGL(k_spill, dim3(groups), dim3(kSpillThreads), 0, s, jobs, b, head, outs,
                     stats, P, sp->huge);
  return hipGetLastError() == hipSuccess ? XD_OK : XD_EDEVICE;
}

inline void spill_free(SpillScratch *sp) {
  if (sp->huge) (void)hipFree(sp->huge);
  sp->huge = nullptr;
  sp->cap = 0;
}

}  // namespace xd
