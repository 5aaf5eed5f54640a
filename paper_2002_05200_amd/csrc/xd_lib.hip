// xd_lib.hip -- libxdrop: batched X-drop seed extension on one MI355X.
//
// Launch sequence of one xdrop_extend call (all on the caller's stream):
//   k_reset    clears the per-tier counters and statistics
//   k_plan     one thread per pair: validation, seed split into a left and a
//              right job (Section IV-B), initial lane-width tier from X, and a
//              counting-sort bin (tier, then estimated anti-diagonals in
//              logarithmic buckets, longest first)
//   k_scan, k_scatter  counting sort of all jobs by bin; each tier's segment
//              of the order
// Every step is a kernel (no memset, no host round trip), so the whole
// sequence can be captured in a graph.
//   k_extend   per tier (cells per lane C = 1, 2, 4, 8, 16, 32): one wavefront
//              per job, taking the tier's segment of the sorted order and then
//              the jobs escalated into it; a job whose band outgrows its
//              window is appended to the next tier's escalation list
//   k_spill    jobs wider than the widest register tier: band in global memory
//   k_combine  one thread per pair: left + seed + right
// Plain mode launches every tier with one wavefront per job; the persistent
// mode launches a fixed grid whose waves pop jobs from a device queue
// (Section IV-B inter-sequence parallelism without relaunches), longest
// estimated job first so no long job starts last.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "xdrop.h"
#include "xd_extend.h"
#include "xd_jobs.h"
#include "xd_pairs.h"
#include "xd_queue.h"
#include "xd_spill.h"
#include "xd_w1_asm.h"
#include "xd_wide.h"
#include "xd_w2_asm.h"
#include "xd_multi.h"
#include "xd_matrix.h"
#include "xd_seed.h"

namespace xd {

constexpr int kBlock = 256;                 // 4 wavefronts, each its own job
constexpr int kWavesPerBlock = kBlock / kWave;

__global__ void k_reset(int32_t *counters, unsigned long long *stats, int32_t *bins,
                        uint32_t *dummy) {
  for (int i = threadIdx.x; i < 2 * kBins; i += blockDim.x) bins[i] = 0;   // counts, cursors
  if (threadIdx.x < 16) dummy[threadIdx.x] = 0;   // the zero words of empty arenas
  if (threadIdx.x < kCounters) counters[threadIdx.x] = 0;
  if (threadIdx.x < kStats) stats[threadIdx.x] = 0;
}

__device__ __forceinline__ void record_done(unsigned long long *stats, int tier, uint64_t cells) {
  atomicAdd(&stats[tier], 1ull);
  atomicAdd(&stats[kLists + tier], (unsigned long long)cells);
}

__device__ __forceinline__ int32_t job_bin(const Job &j, int tier, bool by_cost) {
  const int cb = by_cost ? cost_bucket((uint32_t)(j.m + j.n)) : 0;   // anti-diagonals
  return tier * kCostBuckets + (kCostBuckets - 1 - cb);
}

constexpr int kPlanBlock = 256;   // pairs per block of k_plan / k_scatter

// One thread per pair: validation, seed split, initial tier, counting-sort
// bin of both jobs; bin counts go through a block histogram in LDS.
__global__ __launch_bounds__(kPlanBlock) void k_plan(
    const xd_pair *__restrict__ pairs, int64_t n_pairs, int64_t a_words, int64_t b_words,
    int32_t match, int32_t mismatch, int32_t gap, int32_t min_tier, int32_t by_cost,
    int32_t long_job, int32_t long_bias, int32_t max_tier, Job *__restrict__ jobs,
    int32_t *__restrict__ pair_status, int32_t *__restrict__ bin_of,
    int32_t *__restrict__ bin_count, int32_t *__restrict__ job_save) {
  __shared__ int32_t hist[kBins];
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n_pairs) {
    Job l, r;
    const int32_t st = plan_pair(pairs[p], a_words, b_words, match, mismatch, gap, &l, &r);
    pair_status[p] = st;
    jobs[2 * p] = l;
    jobs[2 * p + 1] = r;
    job_save[2 * p] = -1;
    job_save[2 * p + 1] = -1;
    int tl = initial_tier(l), tr = initial_tier(r);
    if (long_job > 0) {   // long jobs start wider (their bands have longer to grow)
      if (l.m + l.n >= long_job) tl = min(tl + long_bias, kTiers - 1);
      if (r.m + r.n >= long_job) tr = min(tr + long_bias, kTiers - 1);
    }
    if (tl < min_tier) tl = min_tier;
    if (tr < min_tier) tr = min_tier;
    if (tl > max_tier) tl = max_tier;
    if (tr > max_tier) tr = max_tier;
    const int32_t bl = job_bin(l, tl, by_cost != 0), br = job_bin(r, tr, by_cost != 0);
    bin_of[2 * p] = bl;
    bin_of[2 * p + 1] = br;
    atomicAdd(&hist[bl], 1);
    atomicAdd(&hist[br], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += blockDim.x)
    if (hist[i]) atomicAdd(&bin_count[i], hist[i]);
}

// Exclusive scan of the bin counts (one block) and each tier's segment.
constexpr int kScanBlock = 1024;
static_assert(kBins <= kScanBlock, "one scan thread per bin");
__global__ __launch_bounds__(kScanBlock) void k_scan(const int32_t *__restrict__ bin_count,
                                                     int32_t *__restrict__ bin_off,
                                                     int32_t *counters) {
  __shared__ int32_t buf[kScanBlock];
  const int t = threadIdx.x;
  const int32_t v = t < kBins ? bin_count[t] : 0;
  buf[t] = v;
  __syncthreads();
  for (int sh = 1; sh < kScanBlock; sh <<= 1) {   // inclusive Hillis-Steele scan
    const int32_t add = t >= sh ? buf[t - sh] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  if (t < kBins) bin_off[t] = buf[t] - v;
  if (t < kLists) {
    const int first = t * kCostBuckets, last = first + kCostBuckets - 1;
    const int32_t start = buf[first] - bin_count[first];
    counters[kOff + t] = start;
    counters[kInit + t] = buf[last] - start;
  }
}

// Places every job at its bin's offset: ranks within the block from LDS
// atomics, one global reservation per bin and block.  The order inside a bin
// depends on timing; results never depend on the order.
__global__ __launch_bounds__(kPlanBlock) void k_scatter(const int32_t *__restrict__ bin_of,
                                                       int64_t nj,
                                                       const int32_t *__restrict__ bin_off,
                                                       int32_t *__restrict__ cursor,
                                                       int32_t *__restrict__ order) {
  __shared__ int32_t cnt[kBins];
  __shared__ int32_t base[kBins];
  for (int i = threadIdx.x; i < kBins; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * (2 * kPlanBlock) + 2 * threadIdx.x;
  int32_t b[2] = {-1, -1}, rank[2] = {0, 0};
  for (int q = 0; q < 2; ++q) {
    if (j0 + q < nj) {
      b[q] = bin_of[j0 + q];
      rank[q] = atomicAdd(&cnt[b[q]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += blockDim.x)
    if (cnt[i]) base[i] = bin_off[i] + atomicAdd(&cursor[i], cnt[i]);
  __syncthreads();
  for (int q = 0; q < 2; ++q)
    if (b[q] >= 0) order[base[b[q]] + rank[q]] = (int32_t)(j0 + q);
}

// One job per wavefront.  Plain: wave w of the grid takes work item w.
// Persistent (head != nullptr): waves pop work items until none is left.
// The one- and four-register tiers are held to eight resident wavefronts per
// SIMD and the eight-register tier to five (registers were the limit at
// seven, seven and four; the compiler keeps the excess scalars in VGPR lanes
// outside the assembly loops), which hides more of each anti-diagonal's
// dependent chain.  The 32-register tier is held to 256 VGPRs
// (two resident wavefronts per SIMD instead of one), so a second job hides
// the first one's latencies.
template <int C, bool NARROW>
__global__ __launch_bounds__(kBlock, C == 1 ? 8 : C == 4 ? 8 : C == 8 ? 5 : (C >= 32 && NARROW ? 2 : 1)) void k_extend(
    const Job *__restrict__ jobs, TierQueue q, int32_t *head, JobOut *__restrict__ outs,
    unsigned long long *stats, Params P) {
  const int wave = uniform((int32_t)(threadIdx.x >> 6));
  constexpr int kStage = C >= 2 ? 2 * kStageWords<C> : 1;
  __shared__ uint32_t stage[kWavesPerBlock * kStage];
  const int32_t n_init = q.counters[kInit + q.tier];
  const int32_t n_esc = q.counters[kEsc + q.tier];
  const int32_t total = n_init + n_esc;
  int32_t w;
  if (head == nullptr) {
    w = (int32_t)blockIdx.x * kWavesPerBlock + wave;
    if (w >= total) return;
  } else {
    int32_t got = 0;
    if (lane_id() == 0) got = atomicAdd(head, 1);
    w = uniform(got);
  }
  while (w < total) {
    // the queue hands out the longest jobs first: they set the tier's end, so
    // they take the SIMD's issue slot ahead of the waves sharing it
    if (w < P.prio_jobs) __builtin_amdgcn_s_setprio(3);
    else __builtin_amdgcn_s_setprio(0);
    const int32_t j = tier_job(q, w, n_init, n_esc);
    const Job job = jobs[j];
    JobOut o;
    if constexpr (C == 1) {
      if (P.impl == 0) {
        o = extend_job_w1<NARROW, RunAsm>(job, P, j);
      } else {
        o = extend_job_w1<NARROW, RunC>(job, P, j);
      }
    } else if constexpr (C == 2) {
      if (P.impl == 0) {
        o = extend_job_wide<2, NARROW, true>(job, P, j, stage + wave * kStage);
      } else {
        o = extend_job_wide<2, NARROW, false>(job, P, j, stage + wave * kStage);
      }
    } else if (NARROW && P.impl == 0) {
      // +1/-1/-1 (base in the score fields) runs its own instance, whose
      // chain adds no base (one VOP2 add per register); the plain instance is
      // exact on folded words too (it adds dbase = 0), and the 32-register
      // tier keeps to it: a second instance there costs more register spills
      if (C <= 16 && P.fold)
        o = extend_job_wide<C, NARROW, true, C <= 16>(job, P, j, stage + wave * kStage);
      else
        o = extend_job_wide<C, NARROW, true, false>(job, P, j, stage + wave * kStage);
    } else {
      o = extend_job_wide<C, NARROW, false>(job, P, j, stage + wave * kStage);
    }
    if (lane_id() == 0) {
      if (o.status == kJobWider) {
        const int32_t at = atomicAdd((int32_t *)&q.counters[kEsc + q.tier + 1], 1);
        q.next_esc[at] = j;
        atomicAdd(&stats[2 * kLists + q.tier], 1ull);
        if (o.bi == 0) {
          atomicAdd(&stats[kRestart + q.tier], 1ull);
          atomicAdd(&stats[kWasted + q.tier], (unsigned long long)o.cells);
        }
      } else {
        outs[j] = o;
        record_done(stats, q.tier, o.cells);
      }
    }
    if (head == nullptr) break;
    int32_t got = 0;
    if (lane_id() == 0) got = atomicAdd(head, 1);
    w = uniform(got);
  }
}

// Orders the jobs escalated into `tier` by the anti-diagonals they have left
// (m + n less the one they resume at), longest first, into `out`: a counting
// sort in the planning's cost buckets by one workgroup.  The tier then starts
// the longest remainders first, as planning orders whole jobs (longest
// processing time first), instead of in the order the narrower tier happened
// to give them up.  The order within a bucket is unspecified; no result
// depends on it.
constexpr int kSortBlock = 1024;
__global__ __launch_bounds__(kSortBlock) void k_esc_sort(const Job *__restrict__ jobs,
                                                         const int32_t *__restrict__ in,
                                                         int32_t *__restrict__ out,
                                                         const int32_t *__restrict__ counters,
                                                         int tier, Params P) {
  __shared__ int32_t start[kCostBuckets];
  const int32_t n = counters[kEsc + tier];
  for (int b = threadIdx.x; b < kCostBuckets; b += blockDim.x) start[b] = 0;
  __syncthreads();
  auto bin = [&](int32_t j) {
    const Job jb = jobs[j];
    int32_t d = 0;
    if (P.save_pool) {
      const int32_t off = P.job_save[j];
      if (off >= 0) d = P.save_pool[off + kSvD];
    }
    const int32_t rem = jb.m + jb.n - d;
    return kCostBuckets - 1 - cost_bucket((uint32_t)(rem > 0 ? rem : 0));
  };
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&start[bin(in[i])], 1);
  __syncthreads();
  if (threadIdx.x == 0) {   // counts -> first positions
    int32_t acc = 0;
    for (int b = 0; b < kCostBuckets; ++b) {
      const int32_t k = start[b];
      start[b] = acc;
      acc += k;
    }
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int32_t j = in[i];
    out[atomicAdd(&start[bin(j)], 1)] = j;
  }
}

__global__ void k_combine(const xd_pair *__restrict__ pairs, int64_t n_pairs,
                          const int32_t *__restrict__ pair_status, const JobOut *__restrict__ outs,
                          const uint32_t *__restrict__ A, const uint32_t *__restrict__ B,
                          int32_t match, int32_t mismatch, Params P,
                          xd_result *__restrict__ res) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const xd_pair pr = pairs[p];
  const int32_t st = pair_status[p];
  int32_t seed = 0;
  if (st == XD_OK) {
    for (uint32_t t = 0; t < pr.k; ++t) {
      const uint64_t ga = pr.a_off + pr.a_seed + t, gb = pr.b_off + pr.b_seed + t;
      const uint32_t ca = (A[ga >> 4] >> (2 * (ga & 15))) & 3u;
      const uint32_t cb = (B[gb >> 4] >> (2 * (gb & 15))) & 3u;
      seed += P.has_lut ? P.lut[(ca << 2) | cb] : ((ca == cb) ? match : mismatch);
    }
  }
  xd_result out;
  combine_pair(pr, st, outs[2 * p], outs[2 * p + 1], seed, &out);
  res[p] = out;
}

}  // namespace xd

// ---------------------------------------------------------------------------
// host runtime
// ---------------------------------------------------------------------------
using namespace xd;

namespace {

// Last error message of this thread, in a fixed buffer so that reporting an
// error allocates nothing.
thread_local char g_err[512];

xd_status fail(xd_status s, const char *msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return s;
}
xd_status fail(xd_status s, const std::string &msg) { return fail(s, msg.c_str()); }
xd_status failw(xd_status s, const char *who, const char *msg) {
  std::snprintf(g_err, sizeof(g_err), "%s: %s", who, msg);
  return s;
}

#define XD_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(XD_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));   \
  } while (0)

struct HeapBlock {
  void *ptr = nullptr;
  size_t bytes = 0;
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Device buffers of one call, carved from one block: per job the descriptor,
// result, counting-sort bin and save-slot index; per pair the status; the
// sort bins, the sorted order, the escalation lists, counters and statistics;
// plus the escalation save pool and the global-memory band buffers.
struct Bufs {
  int64_t cap_pairs = 0;
  Job *jobs = nullptr;
  JobOut *outs = nullptr;
  int32_t *pair_status = nullptr;
  int32_t *bin_of = nullptr;     // counting-sort bin of every job
  int32_t *job_save = nullptr;   // escalation save slot of every job (-1: none)
  int32_t *bins = nullptr;       // kBins counts, kBins cursors, kBins offsets
  int32_t *order = nullptr;
  int32_t *esc = nullptr;        // kLists + 1 lists of 2 * cap_pairs entries: escalations
  int32_t *esc_sorted = nullptr; // one more: a tier's escalations, longest remainder first
                                 // into each tier, then the spill tier's second pass
  int32_t *counters = nullptr;   // kCounters
  unsigned long long *stats = nullptr;  // kStats
  uint32_t *dummy = nullptr;     // one zero word for empty arenas (cleared by k_reset)
  int32_t *save_pool = nullptr;  // escalation saves
  uint64_t save_slots = 0;
  SpillScratch spill;
};

// Lays the per-job buffers for cap_pairs pairs out from `base` (nullptr: only
// measure); returns the bytes they take.
size_t carve_jobs(Bufs &B, char *base, int64_t cap) {
  const int64_t nj = 2 * cap;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return base ? base + at : nullptr;
  };
  B.cap_pairs = cap;
  B.jobs = (Job *)take(sizeof(Job) * nj);
  B.outs = (JobOut *)take(sizeof(JobOut) * nj);
  B.pair_status = (int32_t *)take(sizeof(int32_t) * cap);
  B.bin_of = (int32_t *)take(sizeof(int32_t) * nj);
  B.job_save = (int32_t *)take(sizeof(int32_t) * nj);
  B.bins = (int32_t *)take(sizeof(int32_t) * 3 * kBins);
  B.order = (int32_t *)take(sizeof(int32_t) * nj);
  B.esc = (int32_t *)take(sizeof(int32_t) * nj * (kLists + 2));
  B.esc_sorted = B.esc ? B.esc + (kLists + 1) * nj : nullptr;
  B.counters = (int32_t *)take(sizeof(int32_t) * kCounters);
  B.stats = (unsigned long long *)take(sizeof(unsigned long long) * kStats);
  B.dummy = (uint32_t *)take(64);
  return off;
}

}  // namespace

struct xd_ctx {
  int device = 0;
  size_t budget = 0;
  int num_cu = 0;
  HeapBlock heap;                  // the per-job buffers of `b`
  Bufs b;                        // this context's own buffers
  const Bufs *last = nullptr;    // buffers of the last call (statistics)
  hipEvent_t ev[10] = {};        // stage boundaries when profiling
  bool have_events = false;
  bool profiled = false;
  hipStream_t own_stream = nullptr;
  // graph of the last graph-mode call and the arguments it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<uint8_t> graph_sig;
  std::mutex mu;
};

namespace {

// Escalation saves: one slot per job at most, 16 GiB at most, and under a
// memory budget at most a quarter of it.
constexpr uint64_t kSaveSlotBytes = sizeof(int32_t) * kSaveSlotWords;
constexpr uint64_t kSavePoolMax = 16ull << 30;

// Device memory of a context: job scratch, the global-memory band buffers
// and the escalation save pool.  Under a budget (mem_budget > 0) the band
// buffers take at most an eighth of it (fewer cells per anti-diagonal) and
// the save pool what is left, at most a quarter; the total never exceeds the
// budget.
xd_status ensure_capacity(xd_ctx *c, int64_t n_pairs) {
  Bufs &B = c->b;
  if (n_pairs <= B.cap_pairs && c->heap.ptr) return XD_OK;
  int64_t cap = std::max<int64_t>(n_pairs, 1024);
  if (B.cap_pairs > 0) cap = std::max<int64_t>(cap, B.cap_pairs * 3 / 2);
  if (c->budget && cap > n_pairs) {   // no growth headroom under a budget
    cap = std::max<int64_t>(n_pairs, 1);
  }
  const int64_t nj = 2 * cap;
  Bufs probe;
  const size_t off = carve_jobs(probe, nullptr, cap);
  int64_t spill_cap = B.spill.huge ? B.spill.cap : kHugeCap;
  uint64_t pool_max = kSavePoolMax;
  if (c->budget) {
    if (!B.spill.huge) {
      const int64_t fit = (int64_t)(c->budget / 8 / spill_bytes(1));
      spill_cap = std::max<int64_t>(kHugeCapMin, std::min<int64_t>(kHugeCap, fit));
    }
    const uint64_t fixed = off + spill_bytes(spill_cap);
    if (fixed > c->budget)
      return fail(XD_ENOMEM, "scratch for " + std::to_string(n_pairs) + " pairs exceeds the budget");
    pool_max = std::min<uint64_t>(c->budget / 4, c->budget - fixed);
  }
  if (c->heap.ptr) {
    XD_HIP(hipDeviceSynchronize());
    XD_HIP(hipFree(c->heap.ptr));
    c->heap.ptr = nullptr;
    c->heap.bytes = 0;
    B.cap_pairs = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, off) != hipSuccess) return fail(XD_ENOMEM, "hipMalloc of job scratch failed");
  c->heap.ptr = p;
  c->heap.bytes = off;
  if (!B.spill.huge && spill_alloc(&B.spill, spill_cap) != XD_OK)
    return fail(XD_ENOMEM, "hipMalloc of the global-memory band buffers failed");
  {   // escalation saves
    const uint64_t want = std::min<uint64_t>((uint64_t)nj, pool_max / kSaveSlotBytes);
    if (want > B.save_slots || (c->budget && B.save_slots > want)) {
      if (B.save_pool) XD_HIP(hipFree(B.save_pool));
      B.save_pool = nullptr;
      B.save_slots = 0;
      void *sp = nullptr;
      if (hipMalloc(&sp, kSaveSlotBytes * want) == hipSuccess) {
        B.save_pool = (int32_t *)sp;
        B.save_slots = want;
      }   // else: escalated jobs restart from scratch
    }
  }
  carve_jobs(B, (char *)p, cap);
  return XD_OK;
}

template <int C, bool NARROW>
hipError_t launch_tier(xd_ctx *c, const Bufs &B, hipStream_t s, bool persistent, int waves_per_cu,
                       int64_t max_jobs, int tier, const Params &P, int multi_wave) {
  const int64_t stride = 2 * B.cap_pairs;
  TierQueue q;
  q.order = B.order;
  q.esc = B.esc + tier * stride;
  q.counters = B.counters;
  q.next_esc = B.esc + (tier + 1) * stride;
  q.tier = tier;
  int32_t *head = persistent ? B.counters + kHead + tier : nullptr;
  if (tier > 0) {   // escalated jobs, longest remainder first
    hipLaunchKernelGGL(k_esc_sort, dim3(1), dim3(kSortBlock), 0, s, B.jobs, q.esc,
                       B.esc_sorted, B.counters, tier, P);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    q.esc = B.esc_sorted;
  }
  if constexpr (C >= 8) {
    if (multi_wave != 0) {   // NW wavefronts per job, C / NW registers each
      auto launch_mw = [&](auto nw) {
        constexpr int NW = decltype(nw)::value;
        int64_t groups =
            persistent ? ((int64_t)c->num_cu * waves_per_cu + NW - 1) / NW : max_jobs;
        if (groups < 1) groups = 1;
        hipLaunchKernelGGL((k_extend_mw<NW, C / NW, NARROW>), dim3((unsigned)groups),
                           dim3(64 * NW), 0, s, B.jobs, q, head, B.outs, B.stats, P,
                           q.next_esc, B.counters + kEsc + tier + 1);
        return hipGetLastError();
      };
      return multi_wave == 2 ? launch_mw(std::integral_constant<int, 2>())
                             : launch_mw(std::integral_constant<int, 4>());
    }
  }
  int64_t blocks;
  if (persistent) {
    blocks = ((int64_t)c->num_cu * waves_per_cu + kWavesPerBlock - 1) / kWavesPerBlock;
  } else {
    blocks = (max_jobs + kWavesPerBlock - 1) / kWavesPerBlock;
  }
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((k_extend<C, NARROW>), dim3((unsigned)blocks), dim3(kBlock), 0, s, B.jobs,
                     q, head, B.outs, B.stats, P);
  return hipGetLastError();
}

template <bool NARROW>
hipError_t launch_tiers(xd_ctx *c, const Bufs &B, hipStream_t s, bool persistent, int waves_per_cu,
                        int64_t nj, const Params &P, bool prof, int mw) {
  // waves per CU: each tier's resident limit from its register footprint
  // (4 SIMDs x waves per SIMD: 7, 5, 7, 5, 3, 2 for C = 1 .. 32), rounded up
  // for the narrow tiers, whose queues are long
  const int wpc[kTiers] = {32, 32, 32, 20, 12, 8};
  auto w = [&](int t) { return waves_per_cu > 0 ? waves_per_cu : wpc[t]; };
  hipError_t e;
  auto mark = [&](int i) { return prof ? hipEventRecord(c->ev[i], s) : hipSuccess; };
  if ((e = launch_tier<1, NARROW>(c, B, s, persistent, w(0), nj, 0, P, mw)) != hipSuccess) return e;
  if ((e = mark(2)) != hipSuccess) return e;
  if ((e = launch_tier<2, NARROW>(c, B, s, persistent, w(1), nj, 1, P, mw)) != hipSuccess) return e;
  if ((e = mark(3)) != hipSuccess) return e;
  if ((e = launch_tier<4, NARROW>(c, B, s, persistent, w(2), nj, 2, P, mw)) != hipSuccess) return e;
  if ((e = mark(4)) != hipSuccess) return e;
  if ((e = launch_tier<8, NARROW>(c, B, s, persistent, w(3), nj, 3, P, mw)) != hipSuccess) return e;
  if ((e = mark(5)) != hipSuccess) return e;
  if ((e = launch_tier<16, NARROW>(c, B, s, persistent, w(4), nj, 4, P, mw)) != hipSuccess) return e;
  if ((e = mark(6)) != hipSuccess) return e;
  if ((e = launch_tier<32, NARROW>(c, B, s, persistent, w(5), nj, 5, P, mw)) != hipSuccess) return e;
  return mark(7);
}

}  // namespace

namespace {

// Arguments of one xdrop_extend call.
struct Launch {
  const uint32_t *d_a;
  uint64_t a_words;
  const uint32_t *d_b;
  uint64_t b_words;
  const xd_pair *d_pairs;
  size_t n_pairs;
  xd_scores sc;
  xd_result *d_out;
  xd_opts o;
};

// Enqueues the whole launch sequence of one call on s (kernels and, when
// profiling, event records only).
xd_status enqueue(xd_ctx *c, const Bufs &B, hipStream_t s, const Launch &L, bool prof) {
  const xd_opts &o = L.o;
  const xd_scores &sc = L.sc;
  const size_t n_pairs = L.n_pairs;
  const bool persistent = (o.sched != XD_SCHED_PLAIN);
  const int64_t nj = 2 * (int64_t)n_pairs;
  Params P;
  P.A = L.a_words ? L.d_a : B.dummy;
  P.B = L.b_words ? L.d_b : B.dummy;
  P.a_words = L.a_words ? (int64_t)L.a_words : 1;
  P.b_words = L.b_words ? (int64_t)L.b_words : 1;
  P.neg_gap = -sc.gap;
  P.base = sc.mismatch - 2 * sc.gap;
  P.delta = sc.match - sc.mismatch;
  P.pat = (int32_t)((uint32_t)P.delta * 0x55555555u);
  // +1/-1/-1: base + delta * match (1 or 3) fits the 2-bit field itself
  P.fold = (sc.match == 1 && P.delta == 2 && P.base == 1) ? 0x55555555 : 0;
  P.dbase = P.fold ? 0 : P.base;
  P.impl = o.impl;
  P.unit_match = sc.match == 1;
  P.save_pool = B.save_pool;
  P.save_cap = B.save_slots;
  if (o.max_save_slots > 0 && (uint64_t)o.max_save_slots < P.save_cap)
    P.save_cap = (uint64_t)o.max_save_slots;
  P.save_top = B.stats + kSaveTop;
  P.job_save = B.job_save;
  P.has_lut = 0;
  for (int t = 0; t < 16; ++t) P.lut[t] = 0;
  P.prio_jobs = persistent ? 4 * c->num_cu : 0;
  const bool narrow = P.delta <= 3;

  if (prof) XD_HIP(hipEventRecord(c->ev[0], s));
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, B.counters, B.stats, B.bins, B.dummy);
  XD_HIP(hipGetLastError());
  const int64_t stride = 2 * B.cap_pairs;
  const bool by_cost = persistent && o.sort_jobs != 0;
  int32_t *bin_count = B.bins, *bin_cursor = B.bins + kBins, *bin_off = B.bins + 2 * kBins;
  const unsigned plan_blocks = (unsigned)((n_pairs + kPlanBlock - 1) / kPlanBlock);
  hipLaunchKernelGGL(k_plan, dim3(plan_blocks), dim3(kPlanBlock), 0, s, L.d_pairs,
                     (int64_t)n_pairs, (int64_t)P.a_words, (int64_t)P.b_words, sc.match,
                     sc.mismatch, sc.gap, o.min_tier, (int32_t)by_cost, o.long_job,
                     o.long_tier_bias, (int32_t)kSpillTier, B.jobs, B.pair_status, B.bin_of, bin_count,
                     B.job_save);
  XD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, s, bin_count, bin_off, B.counters);
  XD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scatter, dim3(plan_blocks), dim3(kPlanBlock), 0, s, B.bin_of, nj,
                     bin_off, bin_cursor, B.order);
  XD_HIP(hipGetLastError());
  if (prof) XD_HIP(hipEventRecord(c->ev[1], s));
  const int mw = o.multi_wave;
  hipError_t e = narrow ? launch_tiers<true>(c, B, s, persistent, o.waves_per_cu, nj, P, prof, mw)
                        : launch_tiers<false>(c, B, s, persistent, o.waves_per_cu, nj, P, prof, mw);
  if (e != hipSuccess) return fail(XD_EDEVICE, std::string("k_extend: ") + hipGetErrorString(e));
  {   // bands wider than one wavefront: a workgroup per job, then global memory
    TierQueue q;
    q.order = B.order;
    q.counters = B.counters;
    q.next_esc = nullptr;
    q.tier = kTiers;
    hipLaunchKernelGGL(k_esc_sort, dim3(1), dim3(kSortBlock), 0, s, B.jobs,
                       B.esc + kTiers * stride, B.esc_sorted, B.counters, kTiers, P);
    XD_HIP(hipGetLastError());
    q.esc = B.esc_sorted;
    int32_t *huge_list = B.esc + kLists * stride;
    // 4,096 slots: 4 wavefronts of 16 registers, two workgroups per CU (at
    // 174 VGPRs two fit); measured faster than 8 wavefronts of 16 registers
    // one per CU (uneven: 115 -> 100 ms): fewer waves take part in each
    // anti-diagonal's barrier and reduction, and the jobs of the tier run
    // at once instead of in two rounds.  Bands wider than 4,094 cells start
    // over in the global-memory pass.
    constexpr int kHugeNW = 4, kHugeC = 16;
    const unsigned huge_grid = 2u * (unsigned)c->num_cu;
    if (narrow)
      hipLaunchKernelGGL((k_extend_mw<kHugeNW, kHugeC, true>), dim3(huge_grid),
                         dim3(64 * kHugeNW), 0, s, B.jobs, q, B.counters + kHead + kTiers,
                         B.outs, B.stats, P, huge_list, B.counters + kHugeCount);
    else
      hipLaunchKernelGGL((k_extend_mw<kHugeNW, kHugeC, false>), dim3(huge_grid),
                         dim3(64 * kHugeNW), 0, s, B.jobs, q, B.counters + kHead + kTiers,
                         B.outs, B.stats, P, huge_list, B.counters + kHugeCount);
    XD_HIP(hipGetLastError());
    if (spill_launch(&B.spill, s, B.jobs, q, B.counters + kHugeHead, huge_list,
                     B.counters + kHugeCount, B.outs, B.stats, P) != XD_OK)
      return fail(XD_EDEVICE, "k_spill launch failed");
  }
  if (prof) XD_HIP(hipEventRecord(c->ev[8], s));
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s,
                     L.d_pairs, (int64_t)n_pairs, B.pair_status, B.outs, P.A, P.B, sc.match,
                     sc.mismatch, P, L.d_out);
  XD_HIP(hipGetLastError());
  if (prof) XD_HIP(hipEventRecord(c->ev[9], s));
  return XD_OK;
}

// Enqueues a substitution-table call: planning (every job in the first
// tier), the one-wavefront table kernel, two global-memory passes for the
// bands it cannot hold (many workgroups with a share of the band buffers
// each, then the few with the whole buffers), and the pair combine.
xd_status enqueue_matrix(xd_ctx *c, const Bufs &B, hipStream_t s, const Launch &L,
                         const int32_t *table, int32_t gap) {
  const xd_opts &o = L.o;
  const size_t n_pairs = L.n_pairs;
  const int64_t nj = 2 * (int64_t)n_pairs;
  int32_t maxabs = 0;
  for (int t = 0; t < 16; ++t) maxabs = std::max(maxabs, table[t] < 0 ? -table[t] : table[t]);
  Params P;
  std::memset(&P, 0, sizeof(P));
  P.A = L.a_words ? L.d_a : B.dummy;
  P.B = L.b_words ? L.d_b : B.dummy;
  P.a_words = L.a_words ? (int64_t)L.a_words : 1;
  P.b_words = L.b_words ? (int64_t)L.b_words : 1;
  P.neg_gap = -gap;
  P.base = 0;
  P.delta = 0;
  P.save_pool = nullptr;
  P.save_top = B.stats + kSaveTop;
  P.job_save = B.job_save;
  P.has_lut = 1;
  for (int t = 0; t < 16; ++t) P.lut[t] = table[t];

  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, B.counters, B.stats, B.bins, B.dummy);
  XD_HIP(hipGetLastError());
  const int64_t stride = 2 * B.cap_pairs;
  int32_t *bin_count = B.bins, *bin_cursor = B.bins + kBins, *bin_off = B.bins + 2 * kBins;
  const unsigned plan_blocks = (unsigned)((n_pairs + kPlanBlock - 1) / kPlanBlock);
  // the int32 guard with the table's largest magnitude in place of both
  // match and mismatch; every job planned into the first tier
  hipLaunchKernelGGL(k_plan, dim3(plan_blocks), dim3(kPlanBlock), 0, s, L.d_pairs,
                     (int64_t)n_pairs, (int64_t)P.a_words, (int64_t)P.b_words, maxabs, maxabs,
                     gap, 0, (int32_t)(o.sort_jobs != 0), 0, 0, 0, B.jobs, B.pair_status,
                     B.bin_of, bin_count, B.job_save);
  XD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanBlock), 0, s, bin_count, bin_off, B.counters);
  XD_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scatter, dim3(plan_blocks), dim3(kPlanBlock), 0, s, B.bin_of, nj,
                     bin_off, bin_cursor, B.order);
  XD_HIP(hipGetLastError());
  TierQueue q;
  q.order = B.order;
  q.esc = nullptr;
  q.counters = B.counters;
  q.next_esc = nullptr;
  q.tier = 0;
  int32_t *wider = B.esc + stride, *wider_count = B.counters + kEsc + 1;
  // persistent: CUs x waves_per_cu waves popping the queue; plain: one
  // wavefront per job
  const int wpc = o.waves_per_cu > 0 ? o.waves_per_cu : 32;
  const int64_t waves = o.sched == XD_SCHED_PLAIN ? nj : (int64_t)c->num_cu * wpc;
  const int64_t blocks = std::max<int64_t>(1, (waves + kWavesPerBlock - 1) / kWavesPerBlock);
  hipLaunchKernelGGL(k_extend_matrix, dim3((unsigned)blocks), dim3(kBlock), 0, s, B.jobs, q,
                     B.counters + kHead, B.outs, B.stats, P, wider, wider_count);
  XD_HIP(hipGetLastError());
  TierQueue q6 = q;
  q6.tier = kTiers;
  int32_t *huge_list = B.esc + kLists * stride;
  if (spill_launch(&B.spill, s, B.jobs, q6, B.counters + kHead + 1, wider, wider_count, B.outs,
                   B.stats, P, c->num_cu, huge_list, B.counters + kHugeCount) != XD_OK ||
      spill_launch(&B.spill, s, B.jobs, q6, B.counters + kHugeHead, huge_list,
                   B.counters + kHugeCount, B.outs, B.stats, P) != XD_OK)
    return fail(XD_EDEVICE, "k_spill launch failed");
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s,
                     L.d_pairs, (int64_t)n_pairs, B.pair_status, B.outs, P.A, P.B, 0, 0, P,
                     L.d_out);
  XD_HIP(hipGetLastError());
  return XD_OK;
}

}  // namespace

extern "C" {

const char *xd_last_error(void) { return g_err; }

xd_status xd_pack(const char *ascii, size_t n, uint32_t *words) {
  if ((!ascii && n) || (!words && n)) return fail(XD_EINVAL, "xd_pack: null pointer");
  for (size_t g = 0; g < n; ++g) {
    const char ch = ascii[g];
    if (!(ch == 'A' || ch == 'C' || ch == 'G' || ch == 'T' || ch == 'a' || ch == 'c' ||
          ch == 'g' || ch == 't'))
      return fail(XD_EINVAL, "xd_pack: character " + std::to_string(g) + " is not ACGT");
  }
  const size_t nw = (n + 15) / 16;
  for (size_t w = 0; w < nw; ++w) words[w] = 0;
  for (size_t g = 0; g < n; ++g) {
    uint32_t code;
    switch (ascii[g]) {
      case 'A': case 'a': code = 0; break;
      case 'C': case 'c': code = 1; break;
      case 'G': case 'g': code = 2; break;
      default: code = 3; break;
    }
    words[g >> 4] |= code << (2 * (g & 15));
  }
  return XD_OK;
}

xd_status xd_pack_codes(const uint8_t *codes, size_t n, uint32_t *words, uint64_t base_off) {
  if ((!codes && n) || (!words && n)) return fail(XD_EINVAL, "xd_pack_codes: null pointer");
  for (size_t g = 0; g < n; ++g)
    if (codes[g] > 3) return fail(XD_EINVAL, "xd_pack_codes: code " + std::to_string(g) + " > 3");
  for (size_t g = 0; g < n; ++g) {
    const uint64_t pos = base_off + g;
    const uint32_t sh = 2 * (uint32_t)(pos & 15);
    uint32_t &w = words[pos >> 4];
    w = (w & ~(3u << sh)) | ((uint32_t)codes[g] << sh);
  }
  return XD_OK;
}

xd_status xd_ctx_create(int device, size_t mem_budget, xd_ctx **out) {
  if (!out) return fail(XD_EINVAL, "xd_ctx_create: null out");
  *out = nullptr;
  int ndev = 0;
  XD_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(XD_EINVAL, "xd_ctx_create: no such device");
  XD_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  XD_HIP(hipGetDeviceProperties(&prop, device));
  xd_ctx *c = new xd_ctx();
  c->device = device;
  c->budget = mem_budget;
  c->num_cu = prop.multiProcessorCount;
  *out = c;
  return XD_OK;
}

xd_status xd_ctx_memory(const xd_ctx *c, uint64_t *bytes) {
  if (!c || !bytes) return fail(XD_EINVAL, "xd_ctx_memory: null pointer");
  *bytes = (uint64_t)c->heap.bytes + (c->b.spill.huge ? spill_bytes(c->b.spill.cap) : 0) +
           c->b.save_slots * kSaveSlotBytes;
  return XD_OK;
}

void xd_ctx_destroy(xd_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->heap.ptr) (void)hipFree(c->heap.ptr);
  if (c->b.save_pool) (void)hipFree(c->b.save_pool);
  spill_free(&c->b.spill);
  if (c->have_events)
    for (int i = 0; i < 10; ++i) (void)hipEventDestroy(c->ev[i]);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  delete c;
}

}  // extern "C"

namespace {

// Validation shared by the batch entry points; fills *o (NULL opts = the
// defaults).  XD_OK with n_pairs == 0 means there is nothing to do.
xd_status check_args(const char *who, const uint32_t *d_a, uint64_t a_words,
                     const uint32_t *d_b, uint64_t b_words, const xd_pair *d_pairs,
                     size_t n_pairs, xd_scores sc, const xd_result *d_out, void *stream,
                     const xd_opts *opts, xd_opts *o) {
  if (n_pairs == 0) return XD_OK;
  if (!d_pairs || !d_out) return failw(XD_EINVAL, who, "null pairs or results");
  if ((!d_a && a_words) || (!d_b && b_words)) return failw(XD_EINVAL, who, "null arena");
  if (n_pairs > (size_t(1) << 29)) return failw(XD_EINVAL, who, "too many pairs");
  if (sc.match < sc.mismatch)
    return failw(XD_EINVAL, who, "mismatch score above match score");
  const int64_t base = (int64_t)sc.mismatch - 2 * (int64_t)sc.gap;
  const int64_t delta = (int64_t)sc.match - (int64_t)sc.mismatch;
  if (base < -128 || base > 127 || delta > 255 || sc.gap > 0 || sc.gap < -(1 << 20))
    return failw(XD_EINVAL, who, "unsupported score set");
  std::memset(o, 0, sizeof(*o));
  if (opts) *o = *opts;
  else o->sort_jobs = 1;
  if (o->sched < 0 || o->sched > XD_SCHED_PERSISTENT)
    return failw(XD_EINVAL, who, "sched out of range");
  if (o->min_tier < 0 || o->min_tier > kTiers)
    return failw(XD_EINVAL, who, "min_tier out of range");
  if (o->impl < 0 || o->impl > 1) return failw(XD_EINVAL, who, "impl out of range");
  if (o->long_job < 0 || o->long_tier_bias < 0 || o->long_tier_bias >= kTiers)
    return failw(XD_EINVAL, who, "long_job / long_tier_bias out of range");
  if (o->multi_wave < 0 || o->multi_wave > 2)
    return failw(XD_EINVAL, who, "multi_wave out of range");
  if (o->waves_per_cu < 0 || o->waves_per_cu > 64)
    return failw(XD_EINVAL, who, "waves_per_cu out of range");
  if (o->max_save_slots < 0 || o->reserved != 0)
    return failw(XD_EINVAL, who, "max_save_slots negative or reserved field set");
  if (o->graph && o->profile) return failw(XD_EINVAL, who, "graph and profile together");
  if (o->graph && !stream)
    return failw(XD_EINVAL, who, "graph mode needs a non-NULL stream");
  return XD_OK;
}

xd_status check_call(const char *who, const xd_ctx *c, const uint32_t *d_a, uint64_t a_words,
                     const uint32_t *d_b, uint64_t b_words, const xd_pair *d_pairs,
                     size_t n_pairs, xd_scores sc, const xd_result *d_out, void *stream,
                     const xd_opts *opts, xd_opts *o) {
  if (!c) return failw(XD_EINVAL, who, "null context");
  return check_args(who, d_a, a_words, d_b, b_words, d_pairs, n_pairs, sc, d_out, stream, opts, o);
}

}  // namespace

extern "C" {

xd_status xdrop_extend(xd_ctx *c, const uint32_t *d_a, uint64_t a_words, const uint32_t *d_b,
                       uint64_t b_words, const xd_pair *d_pairs, size_t n_pairs,
                       xd_scores sc, xd_result *d_out, void *stream, const xd_opts *opts) {
  xd_opts o;
  const xd_status chk = check_call("xdrop_extend", c, d_a, a_words, d_b, b_words, d_pairs,
                                   n_pairs, sc, d_out, stream, opts, &o);
  if (chk != XD_OK || n_pairs == 0) return chk;
  const bool graph = o.graph != 0;

  std::lock_guard<std::mutex> lock(c->mu);
  XD_HIP(hipSetDevice(c->device));
  xd_status st = ensure_capacity(c, (int64_t)n_pairs);
  if (st != XD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const bool prof = o.profile != 0;
  if (prof && !c->have_events) {
    for (int i = 0; i < 10; ++i) XD_HIP(hipEventCreate(&c->ev[i]));
    c->have_events = true;
  }
  c->profiled = prof;
  c->last = &c->b;
  Launch L;
  std::memset(&L, 0, sizeof(L));   // padding too: the struct is compared bytewise
  L.d_a = d_a; L.a_words = a_words; L.d_b = d_b; L.b_words = b_words;
  L.d_pairs = d_pairs; L.n_pairs = n_pairs; L.sc = sc; L.d_out = d_out; L.o = o;
  if (!graph) return enqueue(c, c->b, s, L, prof);

  // graph mode: replay while every argument (and the scratch) is unchanged
  std::vector<uint8_t> sig(sizeof(L) + sizeof(void *));
  std::memcpy(sig.data(), &L, sizeof(L));
  std::memcpy(sig.data() + sizeof(L), &c->heap.ptr, sizeof(void *));
  if (!c->graph_exec || sig != c->graph_sig) {
    if (c->graph_exec) { XD_HIP(hipGraphExecDestroy(c->graph_exec)); c->graph_exec = nullptr; }
    if (c->graph) { XD_HIP(hipGraphDestroy(c->graph)); c->graph = nullptr; }
    c->graph_sig.clear();
    XD_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    st = enqueue(c, c->b, s, L, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != XD_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (st != XD_OK) return st;
      return fail(XD_EDEVICE, std::string("xdrop_extend capture: ") + hipGetErrorString(e));
    }
    // every node must be a kernel: memset nodes have misbehaved on replay
    size_t nn = 0;
    XD_HIP(hipGraphGetNodes(g, nullptr, &nn));
    std::vector<hipGraphNode_t> nodes(nn);
    XD_HIP(hipGraphGetNodes(g, nodes.data(), &nn));
    for (size_t i = 0; i < nn; ++i) {
      hipGraphNodeType ty;
      XD_HIP(hipGraphNodeGetType(nodes[i], &ty));
      if (ty != hipGraphNodeTypeKernel) {
        (void)hipGraphDestroy(g);
        return fail(XD_EDEVICE, "xdrop_extend capture: non-kernel node in the graph");
      }
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(g);
      return fail(XD_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    }
    c->graph = g;
    c->graph_exec = ge;
    c->graph_sig = sig;
  }
  XD_HIP(hipGraphLaunch(c->graph_exec, s));
  return XD_OK;
}

xd_status xdrop_extend_host(xd_ctx *c, const uint32_t *a, uint64_t a_words, const uint32_t *b,
                            uint64_t b_words, const xd_pair *pairs, size_t n_pairs,
                            xd_scores sc, xd_result *out, const xd_opts *opts) {
  if (!c) return fail(XD_EINVAL, "xdrop_extend_host: null context");
  if (n_pairs == 0) return XD_OK;
  if (!pairs || !out || (!a && a_words) || (!b && b_words))
    return fail(XD_EINVAL, "xdrop_extend_host: null pointer");
  XD_HIP(hipSetDevice(c->device));
  if (!c->own_stream) XD_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
  hipStream_t s = c->own_stream;
  void *da = nullptr, *db = nullptr, *dp = nullptr, *dr = nullptr;
  auto cleanup = [&]() {
    if (da) (void)hipFree(da);
    if (db) (void)hipFree(db);
    if (dp) (void)hipFree(dp);
    if (dr) (void)hipFree(dr);
  };
  if (hipMalloc(&da, std::max<size_t>(a_words, 1) * 4) != hipSuccess ||
      hipMalloc(&db, std::max<size_t>(b_words, 1) * 4) != hipSuccess ||
      hipMalloc(&dp, n_pairs * sizeof(xd_pair)) != hipSuccess ||
      hipMalloc(&dr, n_pairs * sizeof(xd_result)) != hipSuccess) {
    cleanup();
    return fail(XD_ENOMEM, "xdrop_extend_host: device allocation failed");
  }
  hipError_t e = hipSuccess;
  if (a_words) e = hipMemcpyAsync(da, a, a_words * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && b_words) e = hipMemcpyAsync(db, b, b_words * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dp, pairs, n_pairs * sizeof(xd_pair), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) {
    cleanup();
    return fail(XD_EDEVICE, std::string("xdrop_extend_host copy-in: ") + hipGetErrorString(e));
  }
  xd_status st = xdrop_extend(c, (const uint32_t *)da, a_words, (const uint32_t *)db, b_words,
                              (const xd_pair *)dp, n_pairs, sc, (xd_result *)dr, s, opts);
  if (st == XD_OK) {
    e = hipMemcpyAsync(out, dr, n_pairs * sizeof(xd_result), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(XD_EDEVICE, std::string("xdrop_extend_host: ") + hipGetErrorString(e));
  }
  cleanup();
  return st;
}

xd_status xdrop_extend_matrix(xd_ctx *c, const uint32_t *d_a, uint64_t a_words,
                              const uint32_t *d_b, uint64_t b_words, const xd_pair *d_pairs,
                              size_t n_pairs, const int32_t *matrix, int32_t gap,
                              xd_result *d_out, void *stream, const xd_opts *opts) {
  static const char *who = "xdrop_extend_matrix";
  xd_opts o;
  xd_scores plain_scores = {0, 0, 0};
  const xd_status chk = check_call(who, c, d_a, a_words, d_b, b_words, d_pairs, n_pairs,
                                   plain_scores, d_out, stream, opts, &o);
  if (chk != XD_OK || n_pairs == 0) return chk;
  if (!matrix) return failw(XD_EINVAL, who, "null matrix");
  for (int t = 0; t < 16; ++t)
    if (matrix[t] > (1 << 20) || matrix[t] < -(1 << 20))
      return failw(XD_EINVAL, who, "matrix entry outside [-2^20, 2^20]");
  if (gap > 0 || gap < -(1 << 20)) return failw(XD_EINVAL, who, "gap outside [-2^20, 0]");
  if (o.graph || o.profile || o.multi_wave || o.min_tier || o.long_job)
    return failw(XD_EINVAL, who, "only the sched, waves_per_cu and sort_jobs options apply");
  std::lock_guard<std::mutex> lock(c->mu);
  XD_HIP(hipSetDevice(c->device));
  xd_status st = ensure_capacity(c, (int64_t)n_pairs);
  if (st != XD_OK) return st;
  c->profiled = false;
  c->last = &c->b;
  Launch L;
  std::memset(&L, 0, sizeof(L));
  L.d_a = d_a; L.a_words = a_words; L.d_b = d_b; L.b_words = b_words;
  L.d_pairs = d_pairs; L.n_pairs = n_pairs; L.d_out = d_out; L.o = o;
  return enqueue_matrix(c, c->b, (hipStream_t)stream, L, matrix, gap);
}

xd_status xd_find_seeds(xd_ctx *c, const uint32_t *d_a, uint64_t a_words, const uint32_t *d_b,
                        uint64_t b_words, xd_pair *d_pairs, size_t n_pairs, uint32_t k,
                        uint32_t width, int32_t set_pairs, xd_seed *d_seeds, void *stream) {
  static const char *who = "xd_find_seeds";
  if (!c) return failw(XD_EINVAL, who, "null context");
  if (k < 1 || k > (uint32_t)kSeedMaxK) return failw(XD_EINVAL, who, "k outside 1..31");
  if (width < 1 || width > (1u << 30)) return failw(XD_EINVAL, who, "width outside 1..2^30");
  if (set_pairs != 0 && set_pairs != 1) return failw(XD_EINVAL, who, "set_pairs is not 0 or 1");
  if (n_pairs == 0) return XD_OK;
  if (!d_pairs || !d_seeds) return failw(XD_EINVAL, who, "null pairs or seeds");
  if ((!d_a && a_words) || (!d_b && b_words)) return failw(XD_EINVAL, who, "null arena");
  if (n_pairs > (size_t(1) << 29)) return failw(XD_EINVAL, who, "too many pairs");
  std::lock_guard<std::mutex> lock(c->mu);
  XD_HIP(hipSetDevice(c->device));
  SeedArgs S;
  S.A = d_a;
  S.B = d_b;
  S.a_words = (int64_t)a_words;
  S.b_words = (int64_t)b_words;
  S.pairs = d_pairs;
  S.n_pairs = (int64_t)n_pairs;
  S.k = (int32_t)k;
  S.width = width;
  S.set_pairs = set_pairs;
  S.out = d_seeds;
  const unsigned grid = (unsigned)std::min<size_t>(n_pairs, size_t(1) << 24);
  hipLaunchKernelGGL(k_find_seeds, dim3(grid), dim3(kSeedThreads), 0, (hipStream_t)stream, S);
  XD_HIP(hipGetLastError());
  return XD_OK;
}

xd_status xd_last_stats(xd_ctx *c, xd_stats *out) {
  if (!c || !out) return fail(XD_EINVAL, "xd_last_stats: null pointer");
  std::memset(out, 0, sizeof(*out));
  if (!c->last || !c->last->stats) return XD_OK;
  unsigned long long h[kStats];
  XD_HIP(hipSetDevice(c->device));
  XD_HIP(hipDeviceSynchronize());
  XD_HIP(hipMemcpy(h, c->last->stats, sizeof(h), hipMemcpyDeviceToHost));
  for (int t = 0; t < kLists; ++t) {
    out->jobs[t] = h[t];
    out->cells[t] = h[kLists + t];
    out->escalated[t] = h[2 * kLists + t];
    out->restarted[t] = h[kRestart + t];
    out->wasted_cells[t] = h[kWasted + t];
  }
  if (c->profiled) {
    for (int i = 0; i < 9; ++i) XD_HIP(hipEventElapsedTime(&out->stage_ms[i], c->ev[i], c->ev[i + 1]));
    out->profiled = 1;
  }
  return XD_OK;
}

}  // extern "C"

// Scratch of xdrop_extend_noalloc: one fixed array per GPU, laid out as the
// job lists of XD_NOALLOC_MAX_PAIRS pairs, then the global-memory band
// buffers, then the escalation saves.  Host code never passes this name to a
// kernel or a copy: it is a host-side stand-in for the device array, whose
// address on each GPU comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[XD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNaJobBytes = size_t(2) << 20;
constexpr size_t kNaSpillBytes = (spill_bytes(XD_NOALLOC_BAND_CELLS) + 255) & ~size_t(255);
constexpr size_t kNaSaveBytes = kSaveSlotBytes * XD_NOALLOC_SAVE_SLOTS;
static_assert(kNaJobBytes + kNaSpillBytes + kNaSaveBytes <= XD_NOALLOC_SCRATCH_BYTES,
              "no-allocation scratch layout exceeds its array");
static_assert(XD_NOALLOC_BAND_CELLS >= kHugeCapMin, "band buffers below the spill minimum");
constexpr int kNaMaxDevices = 64;

// Per device: the array's device address and the buffers carved from it,
// set once (with the device current) by the first call on that device.
struct NoAllocDevice {
  bool ready = false;
  void *ptr = nullptr;
  Bufs b;
};
NoAllocDevice g_na[kNaMaxDevices];
xd_ctx g_na_ctx[kNaMaxDevices];   // device number and CU count only; no memory
std::mutex g_na_mu;

xd_status noalloc_setup(int device) {
  NoAllocDevice &D = g_na[device];
  if (D.ready) return XD_OK;
  void *ptr = nullptr;
  XD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return fail(XD_EDEVICE, "xdrop_extend_noalloc: no device address for the scratch array");
  int ncu = 0;
  XD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
  char *base = (char *)ptr;
  Bufs &B = D.b;
  if (carve_jobs(B, base, XD_NOALLOC_MAX_PAIRS) > kNaJobBytes)
    return fail(XD_EINVAL, "xdrop_extend_noalloc: job lists exceed their part of the scratch");
  B.spill.huge = (int32_t *)(base + kNaJobBytes);
  B.spill.cap = XD_NOALLOC_BAND_CELLS;
  B.save_pool = (int32_t *)(base + kNaJobBytes + kNaSpillBytes);
  B.save_slots = XD_NOALLOC_SAVE_SLOTS;
  g_na_ctx[device].device = device;
  g_na_ctx[device].num_cu = ncu;
  D.ptr = ptr;
  D.ready = true;
  return XD_OK;
}

}  // namespace

extern "C" {

xd_status xdrop_extend_noalloc(int device, const uint32_t *d_a, uint64_t a_words,
                               const uint32_t *d_b, uint64_t b_words, const xd_pair *d_pairs,
                               size_t n_pairs, xd_scores sc, xd_result *d_out, void *stream,
                               const xd_opts *opts) {
  static const char *who = "xdrop_extend_noalloc";
  if (n_pairs > XD_NOALLOC_MAX_PAIRS)
    return failw(XD_EINVAL, who, "more pairs than XD_NOALLOC_MAX_PAIRS");
  xd_opts o;
  const xd_status chk = check_args(who, d_a, a_words, d_b, b_words, d_pairs, n_pairs, sc, d_out,
                                   stream, opts, &o);
  if (chk != XD_OK || n_pairs == 0) return chk;
  if (o.graph || o.profile) return failw(XD_EINVAL, who, "graph and profile options do not apply");
  if (device < 0 || device >= kNaMaxDevices) return failw(XD_EINVAL, who, "no such device");
  std::lock_guard<std::mutex> lock(g_na_mu);
  int ndev = 0, prev = 0;
  XD_HIP(hipGetDeviceCount(&ndev));
  if (device >= ndev) return failw(XD_EINVAL, who, "no such device");
  XD_HIP(hipGetDevice(&prev));
  XD_HIP(hipSetDevice(device));
  xd_status st = noalloc_setup(device);
  if (st == XD_OK) {
    Launch L;
    std::memset(&L, 0, sizeof(L));
    L.d_a = d_a; L.a_words = a_words; L.d_b = d_b; L.b_words = b_words;
    L.d_pairs = d_pairs; L.n_pairs = n_pairs; L.sc = sc; L.d_out = d_out; L.o = o;
    st = enqueue(&g_na_ctx[device], g_na[device].b, (hipStream_t)stream, L, false);
  }
  const hipError_t e = hipSetDevice(prev);
  if (st == XD_OK && e != hipSuccess)
    return fail(XD_EDEVICE, std::string("xdrop_extend_noalloc: restoring the device: ") +
                                hipGetErrorString(e));
  return st;
}

}  // extern "C"

#include "xd_server.h"
