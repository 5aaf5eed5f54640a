// xd_server.h -- serving loop of libxdrop (host code; included once by
// xd_lib.hip after the batch entry points).
//
// A scheduler thread owns `slots` execution slots.  Each slot has its own
// stream, its own xd_ctx (job scratch, band buffers and escalation saves,
// sized for a full batch under half the slot's share of the memory budget),
// a device arena for the packed reads and pair records of one batch, pinned
// host staging of the same size, and a completion event.  Requests wait in
// one FIFO; whenever a slot is free and the FIFO is not empty, the scheduler
// admits the oldest request and later ones of its score set and cost class
// while they fit in the slot's memory (xd_admit.h), copies them to the
// device, launches xdrop_extend on the slot's stream and records the event.
// Requests arriving meanwhile go to the next free slot, whose kernels then
// run beside the batches already on the device.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "xd_admit.h"

namespace {

uint64_t steady_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

xd_status check_scores(const xd_scores &sc) {
  const int64_t base = (int64_t)sc.mismatch - 2 * (int64_t)sc.gap;
  const int64_t delta = (int64_t)sc.match - (int64_t)sc.mismatch;
  if (sc.match < sc.mismatch || base < -128 || base > 127 || delta > 255 || sc.gap > 0 ||
      sc.gap < -(1 << 20))
    return XD_EINVAL;
  return XD_OK;
}

struct Request {
  uint64_t ticket = 0;
  std::vector<uint32_t> a, b;
  std::vector<xd_pair> pairs;
  xd_scores scores{};
  std::vector<xd_result> out;
  int32_t cls = 0;          // cost class (xd_admit.h)
  int state = 0;            // 0 queued, 1 on the device, 2 done, 3 failed, 4 canceled,
                            // 5 timed out (watchdog)
  uint64_t done_ns = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  xd_ctx *ctx = nullptr;
  uint32_t *d_a = nullptr, *d_b = nullptr;
  xd_pair *d_pairs = nullptr;
  xd_result *d_out = nullptr;
  uint32_t *h_a = nullptr, *h_b = nullptr;
  xd_pair *h_pairs = nullptr;
  xd_result *h_out = nullptr;
  uint64_t cap_words = 0;   // per arena
  int32_t cap_pairs = 0;
  uint64_t device_bytes = 0;   // arenas, pair records, results and the context
  bool busy = false;
  bool draining = false;       // the watchdog failed this batch; its kernels still run
  uint64_t launched_ns = 0;
  int32_t n_pairs = 0;
  std::vector<std::shared_ptr<Request>> reqs;
  std::vector<int32_t> first;   // first pair of each request in the batch
};

}  // namespace

struct xd_server {
  xd_server_opts o{};
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new request or stop
  std::condition_variable cv_done;   // pollers: a request finished
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread thread;
  xd_server_stats st{};
  std::string thread_error;
  int pollers = 0;                   // xd_server_poll calls inside the server now
  std::condition_variable cv_pollers;
  std::vector<AdmitItem> items;      // admission scratch (scheduler thread only)
  std::vector<size_t> take;
};

namespace {

void free_slot(Slot &s) {
  if (s.ctx) xd_ctx_destroy(s.ctx);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  if (s.d_a) (void)hipFree(s.d_a);
  if (s.d_b) (void)hipFree(s.d_b);
  if (s.d_pairs) (void)hipFree(s.d_pairs);
  if (s.d_out) (void)hipFree(s.d_out);
  if (s.h_a) (void)hipHostFree(s.h_a);
  if (s.h_b) (void)hipHostFree(s.h_b);
  if (s.h_pairs) (void)hipHostFree(s.h_pairs);
  if (s.h_out) (void)hipHostFree(s.h_out);
  s = Slot();
}

// A slot's context is created under half the slot's share and sized for a
// full batch first; the arenas get what the share has left (xd_admit.h).
xd_status alloc_slot(const xd_server_opts &o, uint64_t share, Slot &s) {
  s.cap_pairs = o.max_batch_pairs;
  SlotPlan plan;
  plan_slot(share, s.cap_pairs, 0, &plan);
  xd_status st = xd_ctx_create(o.device, plan.ctx_budget, &s.ctx);
  if (st != XD_OK) return st;
  st = ensure_capacity(s.ctx, s.cap_pairs);
  if (st != XD_OK) return st == XD_ENOMEM ? XD_EINVAL : st;
  uint64_t ctx_bytes = 0;
  xd_ctx_memory(s.ctx, &ctx_bytes);
  if (!plan_slot(share, s.cap_pairs, ctx_bytes, &plan)) return XD_EINVAL;
  s.cap_words = plan.cap_words;
  s.device_bytes = ctx_bytes + plan.pair_bytes + 2 * 4 * s.cap_words;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess)
    return XD_EDEVICE;
  if (hipMalloc(&s.d_a, s.cap_words * 4) != hipSuccess ||
      hipMalloc(&s.d_b, s.cap_words * 4) != hipSuccess ||
      hipMalloc(&s.d_pairs, sizeof(xd_pair) * s.cap_pairs) != hipSuccess ||
      hipMalloc(&s.d_out, sizeof(xd_result) * s.cap_pairs) != hipSuccess ||
      hipHostMalloc(&s.h_a, s.cap_words * 4) != hipSuccess ||
      hipHostMalloc(&s.h_b, s.cap_words * 4) != hipSuccess ||
      hipHostMalloc(&s.h_pairs, sizeof(xd_pair) * s.cap_pairs) != hipSuccess ||
      hipHostMalloc(&s.h_out, sizeof(xd_result) * s.cap_pairs) != hipSuccess)
    return XD_ENOMEM;
  return XD_OK;
}

// Packs the admitted requests of a slot into its staging buffers and
// launches the batch.  Called by the scheduler thread without the lock (the
// requests are owned by the slot while on the device).
xd_status launch_batch(xd_server *srv, Slot &s) {
  uint64_t a_used = 0, b_used = 0;
  int32_t np = 0;
  s.first.clear();
  for (auto &r : s.reqs) {
    std::memcpy(s.h_a + a_used, r->a.data(), r->a.size() * 4);
    std::memcpy(s.h_b + b_used, r->b.data(), r->b.size() * 4);
    s.first.push_back(np);
    for (const xd_pair &p : r->pairs) {
      xd_pair q = p;
      q.a_off += a_used * 16;   // request-local base offsets -> batch arena
      q.b_off += b_used * 16;
      s.h_pairs[np++] = q;
    }
    a_used += r->a.size();
    b_used += r->b.size();
  }
  s.n_pairs = np;
  const bool graph = srv->o.graph != 0;
  int32_t launch_pairs = np;
  uint64_t a_words = a_used, b_words = b_used;
  if (graph) {   // fixed arguments: whole capacity, padding pairs are empty
    std::memset(s.h_pairs + np, 0, sizeof(xd_pair) * (s.cap_pairs - np));
    launch_pairs = s.cap_pairs;
    a_words = b_words = s.cap_words;
  }
  if (a_used && hipMemcpyAsync(s.d_a, s.h_a, a_used * 4, hipMemcpyHostToDevice, s.stream) != hipSuccess)
    return XD_EDEVICE;
  if (b_used && hipMemcpyAsync(s.d_b, s.h_b, b_used * 4, hipMemcpyHostToDevice, s.stream) != hipSuccess)
    return XD_EDEVICE;
  if (hipMemcpyAsync(s.d_pairs, s.h_pairs, sizeof(xd_pair) * launch_pairs, hipMemcpyHostToDevice,
                     s.stream) != hipSuccess)
    return XD_EDEVICE;
  xd_opts eo = srv->o.extend_opts;
  eo.graph = graph ? 1 : 0;
  eo.profile = 0;
  const xd_status st = xdrop_extend(s.ctx, s.d_a, a_words ? a_words : 1, s.d_b,
                                    b_words ? b_words : 1, s.d_pairs, (size_t)launch_pairs,
                                    s.reqs[0]->scores, s.d_out, s.stream, &eo);
  if (st != XD_OK) return st;
  if (hipMemcpyAsync(s.h_out, s.d_out, sizeof(xd_result) * np, hipMemcpyDeviceToHost, s.stream) !=
          hipSuccess ||
      hipEventRecord(s.done, s.stream) != hipSuccess)
    return XD_EDEVICE;
  return XD_OK;
}

void finish_batch(xd_server *srv, Slot &s, bool ok) {
  const uint64_t now = steady_ns();
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    for (size_t q = 0; q < s.reqs.size(); ++q) {
      Request &r = *s.reqs[q];
      if (ok) {
        r.out.assign(s.h_out + s.first[q], s.h_out + s.first[q] + r.pairs.size());
        for (const xd_result &x : r.out) srv->st.cells += x.left_cells + x.right_cells;
        r.state = 2;
        srv->st.pairs += r.pairs.size();
      } else {
        r.state = 3;
      }
      r.done_ns = now;
      srv->st.requests += 1;
    }
    if (ok) srv->st.batches += 1;
  }
  s.reqs.clear();
  s.busy = false;
  srv->cv_done.notify_all();
}

// The watchdog: the requests of a batch that has run too long fail now; the
// slot keeps draining until its kernels are done.
void expire_batch(xd_server *srv, Slot &s) {
  const uint64_t now = steady_ns();
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    for (auto &r : s.reqs) {
      r->state = 5;
      r->done_ns = now;
      srv->st.timed_out += 1;
    }
  }
  s.reqs.clear();
  s.draining = true;
  srv->cv_done.notify_all();
}

void scheduler(xd_server *srv) {
  (void)hipSetDevice(srv->o.device);
  for (;;) {
    bool progress = false;
    int inflight = 0;
    const uint64_t wd_ns = (uint64_t)srv->o.watchdog_ms * 1000000ull;
    for (Slot &s : srv->slots) {   // completions
      if (!s.busy) continue;
      const hipError_t e = hipEventQuery(s.done);
      if (e != hipErrorNotReady && s.draining) {   // a timed-out batch has drained
        s.busy = false;
        s.draining = false;
        progress = true;
      } else if (e == hipSuccess) {
        finish_batch(srv, s, true);
        progress = true;
      } else if (e != hipErrorNotReady) {
        finish_batch(srv, s, false);
        progress = true;
      } else {
        if (wd_ns && !s.draining && steady_ns() - s.launched_ns > wd_ns) {
          expire_batch(srv, s);
          progress = true;
        }
        ++inflight;
      }
    }
    for (Slot &s : srv->slots) {   // admission into free slots
      if (s.busy) continue;
      {
        std::unique_lock<std::mutex> lock(srv->mu);
        if (srv->queue.empty()) break;
        // admission (xd_admit.h): the oldest request, then later ones of its
        // score set and cost class while the batch fits the slot
        constexpr size_t kScan = 4096;
        const size_t nq = std::min(srv->queue.size(), kScan);
        srv->items.resize(nq);
        for (size_t i = 0; i < nq; ++i) {
          const Request &r = *srv->queue[i];
          srv->items[i] = {r.a.size(), r.b.size(), (uint32_t)r.pairs.size(), r.scores, r.cls};
        }
        admit(srv->items.data(), nq, s.cap_words, s.cap_pairs, srv->o.group_by_class != 0,
              kScan, &srv->take);
        for (size_t i : srv->take) {
          srv->queue[i]->state = 1;
          s.reqs.push_back(srv->queue[i]);
        }
        for (size_t t = srv->take.size(); t-- > 0;)
          srv->queue.erase(srv->queue.begin() + (ptrdiff_t)srv->take[t]);
        srv->st.queued = srv->queue.size();
      }
      if (s.reqs.empty()) break;
      s.busy = true;
      s.launched_ns = steady_ns();
      ++inflight;
      if (launch_batch(srv, s) != XD_OK) {
        (void)hipStreamSynchronize(s.stream);
        finish_batch(srv, s, false);
        --inflight;
      }
      progress = true;
    }
    {
      std::unique_lock<std::mutex> lock(srv->mu);
      if ((uint64_t)inflight > srv->st.max_inflight) srv->st.max_inflight = inflight;
      if (srv->stop && inflight == 0) break;
      if (!progress) {
        if (inflight == 0 && srv->queue.empty() && !srv->stop)
          srv->cv_work.wait(lock);                    // idle: until a request arrives
        else
          srv->cv_work.wait_for(lock, std::chrono::microseconds(20));   // batches running
      }
    }
  }
}

}  // namespace

extern "C" {

xd_status xd_server_create(const xd_server_opts *opts, xd_server **out) {
  if (!opts || !out) return fail(XD_EINVAL, "xd_server_create: null pointer");
  *out = nullptr;
  xd_server_opts o = *opts;
  if (o.slots == 0) o.slots = 4;
  if (o.max_batch_pairs == 0) o.max_batch_pairs = 2048;
  if (o.mem_budget == 0) o.mem_budget = 1ull << 30;
  if (o.slots < 1 || o.slots > 16 || o.max_batch_pairs < 1 || o.max_batch_pairs > (1 << 24))
    return fail(XD_EINVAL, "xd_server_create: slots or max_batch_pairs out of range");
  if (o.group_by_class < 0 || o.group_by_class > 1 || o.watchdog_ms < 0)
    return fail(XD_EINVAL, "xd_server_create: group_by_class not 0/1 or negative watchdog");
  int ndev = 0;
  XD_HIP(hipGetDeviceCount(&ndev));
  if (o.device < 0 || o.device >= ndev) return fail(XD_EINVAL, "xd_server_create: no such device");
  XD_HIP(hipSetDevice(o.device));
  xd_server *srv = new xd_server();
  srv->o = o;
  srv->slots.resize(o.slots);
  const uint64_t share = o.mem_budget / (uint64_t)o.slots;
  for (Slot &s : srv->slots) {
    const xd_status st = alloc_slot(o, share, s);
    if (st != XD_OK) {
      for (Slot &t : srv->slots) free_slot(t);
      delete srv;
      return fail(st, st == XD_EINVAL ? "xd_server_create: mem_budget too small for the slots"
                                      : "xd_server_create: slot allocation failed");
    }
    srv->st.device_bytes += s.device_bytes;
    srv->st.arena_words = s.cap_words;
  }
  srv->thread = std::thread(scheduler, srv);
  *out = srv;
  return XD_OK;
}

xd_status xd_server_submit(xd_server *srv, const xd_request *req, uint64_t *ticket) {
  if (!srv || !req || !ticket) return fail(XD_EINVAL, "xd_server_submit: null pointer");
  if (req->n_pairs == 0 || !req->pairs) return fail(XD_EINVAL, "xd_server_submit: no pairs");
  if ((req->a_words && !req->a) || (req->b_words && !req->b))
    return fail(XD_EINVAL, "xd_server_submit: null reads");
  if (check_scores(req->scores) != XD_OK)
    return fail(XD_EINVAL, "xd_server_submit: unsupported score set");
  const Slot &s0 = srv->slots[0];
  if ((int64_t)req->n_pairs > s0.cap_pairs || req->a_words > s0.cap_words ||
      req->b_words > s0.cap_words)
    return fail(XD_EINVAL, "xd_server_submit: request larger than a slot");
  for (uint32_t p = 0; p < req->n_pairs; ++p) {   // reads must lie in this request's arenas
    const xd_pair &q = req->pairs[p];
    if (q.a_off + q.a_len > req->a_words * 16 || q.b_off + q.b_len > req->b_words * 16)
      return fail(XD_EINVAL, "xd_server_submit: pair " + std::to_string(p) +
                                 " reaches outside the request's reads");
  }
  auto r = std::make_shared<Request>();
  r->a.assign(req->a, req->a + req->a_words);
  r->b.assign(req->b, req->b + req->b_words);
  r->pairs.assign(req->pairs, req->pairs + req->n_pairs);
  r->scores = req->scores;
  r->cls = cost_class(req->pairs, req->n_pairs);
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->stop) return fail(XD_ECANCELED, "xd_server_submit: server is stopping");
    r->ticket = srv->next_ticket++;
    srv->table[r->ticket] = r;
    srv->queue.push_back(r);
    srv->st.queued = srv->queue.size();
    *ticket = r->ticket;
  }
  srv->cv_work.notify_one();
  return XD_OK;
}

xd_status xd_server_poll(xd_server *srv, uint64_t ticket, xd_result *out, int32_t wait_ms,
                         uint64_t *done_ns) {
  if (!srv || !out) return fail(XD_EINVAL, "xd_server_poll: null pointer");
  std::unique_lock<std::mutex> lock(srv->mu);
  auto it = srv->table.find(ticket);
  if (it == srv->table.end()) return fail(XD_EINVAL, "xd_server_poll: unknown ticket");
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->state >= 2; };
  if (!ready()) {
    ++srv->pollers;   // xd_server_destroy waits until no poll is inside
    if (wait_ms < 0) srv->cv_done.wait(lock, ready);
    else if (wait_ms > 0) srv->cv_done.wait_for(lock, std::chrono::milliseconds(wait_ms), ready);
    if (--srv->pollers == 0) srv->cv_pollers.notify_all();
  }
  if (!ready()) return XD_ENOTREADY;
  srv->table.erase(r->ticket);
  if (done_ns) *done_ns = r->done_ns;
  if (r->state == 4) return fail(XD_ECANCELED, "xd_server_poll: the request was canceled");
  if (r->state == 5)
    return fail(XD_ETIMEDOUT, "xd_server_poll: the request's batch outran the watchdog");
  if (r->state == 3) return fail(XD_EDEVICE, "xd_server_poll: the request's batch failed");
  std::memcpy(out, r->out.data(), sizeof(xd_result) * r->out.size());
  return XD_OK;
}

xd_status xd_server_cancel(xd_server *srv, uint64_t ticket) {
  if (!srv) return fail(XD_EINVAL, "xd_server_cancel: null server");
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->table.find(ticket);
    if (it == srv->table.end()) return fail(XD_EINVAL, "xd_server_cancel: unknown ticket");
    Request &r = *it->second;
    if (r.state != 0)
      return fail(XD_EBUSY, "xd_server_cancel: the request is already on the device or done");
    for (auto q = srv->queue.begin(); q != srv->queue.end(); ++q)
      if ((*q)->ticket == ticket) {
        srv->queue.erase(q);
        break;
      }
    r.state = 4;
    r.done_ns = steady_ns();
    srv->st.canceled += 1;
    srv->st.queued = srv->queue.size();
  }
  srv->cv_done.notify_all();
  return XD_OK;
}

xd_status xd_server_get_stats(xd_server *srv, xd_server_stats *out) {
  if (!srv || !out) return fail(XD_EINVAL, "xd_server_get_stats: null pointer");
  std::lock_guard<std::mutex> lock(srv->mu);
  *out = srv->st;
  out->waiting_polls = (uint64_t)srv->pollers;
  return XD_OK;
}

void xd_server_destroy(xd_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stop = true;
    const uint64_t now = steady_ns();
    for (auto &r : srv->queue) {   // never admitted: canceled
      r->state = 4;
      r->done_ns = now;
      srv->st.canceled += 1;
    }
    srv->queue.clear();
  }
  srv->cv_work.notify_all();
  srv->cv_done.notify_all();
  if (srv->thread.joinable()) srv->thread.join();
  {   // pollers woken by the last completions or cancellations leave first
    std::unique_lock<std::mutex> lock(srv->mu);
    srv->cv_done.notify_all();
    srv->cv_pollers.wait(lock, [&] { return srv->pollers == 0; });
  }
  (void)hipSetDevice(srv->o.device);
  for (Slot &s : srv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  delete srv;
}

}  // extern "C"
