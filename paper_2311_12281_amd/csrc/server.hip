// Serving: graphs stay resident with the exact closed count of every edge,
// and (graph, eps, mu) queries are answered by re-thresholding those counts
// (no intersection), which needs only streaming passes over the edges.
//
// Continuous batching: a dispatcher thread admits queued requests onto free
// slots as soon as slots free up; each slot owns a HIP stream and per-query
// scratch, so requests that arrive while others are running overlap on the
// device.  A query's result goes to a pinned host buffer taken from a pool;
// on completion (detected with an event) the buffer is handed to the request
// and the slot is reused at once, and the waiting caller's thread copies the
// result out and gives the buffer back.  The pool is bounded: when every
// buffer holds a result not yet collected, admissions wait for one.
//
// Memory admission: a graph is made resident only if its footprint (the
// in-memory layout as scan_graph_create builds it, degree-ranked rows
// included, plus the cached counts and closed-size products, plus what the
// slots' scratch would grow by) fits the budget; otherwise it is kept in host
// memory and its queries run on a fallback worker thread with its own stream,
// through a partitioned scan_graph_create with the remaining budget (kept for
// the next query of the same graph) and scan_run, while the dispatcher keeps
// admitting and completing resident queries.
#include "graph.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

struct ServedGraph {
  int32_t n = 0;
  int64_t nnz = 0, m = 0;
  bool resident = false;
  scan_graph* g = nullptr;       // resident: device layout
  int32_t* d_ecount = nullptr;   // resident: closed count per oriented edge
  uint64_t* d_ab = nullptr;      // resident: |N[u]| |N[v]| per oriented edge
  uint64_t bytes = 0;            // device bytes held while resident
  std::vector<int64_t> h_rp;     // non-resident: host copy
  std::vector<int32_t> h_ci;
  int inflight = 0;
  bool removing = false;
};

// Pinned host buffer for one query's labels and roles.
struct OutBuf {
  int32_t* labels = nullptr;
  uint8_t* roles = nullptr;
  int32_t cap = 0;
};

void free_out(OutBuf& b) {
  if (b.labels) (void)hipHostFree(b.labels);
  if (b.roles) (void)hipHostFree(b.roles);
  b = OutBuf();
}

struct Request {
  int64_t id = 0;
  int32_t gid = 0;
  int64_t p = 1, q = 1;
  int32_t mu = 2;
  Clock::time_point t_submit, t_done;
  int status = 1;  // 1 pending/running, 0 ok, < 0 error
  std::string error;
  std::vector<int32_t> labels;   // fallback path
  std::vector<uint8_t> roles;
  OutBuf out;                    // resident path: the result, until collected
  int32_t n = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t cap_n = 0;
  int64_t cap_m = 0;
  int32_t *d_lower = nullptr, *d_parent = nullptr, *d_label = nullptr, *d_out_labels = nullptr;
  uint8_t *d_role = nullptr, *d_state = nullptr, *d_out_roles = nullptr;
  OutBuf out;                    // the running request's result buffer
  std::shared_ptr<Request> req;  // running request, or null
};

uint64_t slot_bytes(int32_t n, int64_t m) { return 18ull * (uint64_t)n + (uint64_t)m; }

// Peak device bytes of adding a graph: the in-memory layout as
// scan_graph_create builds it (with the degree-ranked copy of the rows where
// the options ask for it), the cached closed counts (4 bytes per edge) and
// closed-size products (8 bytes per edge).
uint64_t graph_bytes(int32_t n, int64_t nnz, const scan_opts& o) {
  const uint64_t m = (uint64_t)nnz / 2;
  return inmemory_footprint(n, nnz, o.hub_ranked != 0) + 12ull * m;
}

void release_resident(ServedGraph* G) {
  if (G->d_ecount) (void)hipFree(G->d_ecount);
  if (G->d_ab) (void)hipFree(G->d_ab);
  G->d_ecount = nullptr;
  G->d_ab = nullptr;
  if (G->g) scan_graph_destroy(G->g);
  G->g = nullptr;
}

void free_slot_buffers(Slot& s) {
  void* d[] = {s.d_lower, s.d_parent, s.d_label, s.d_out_labels, s.d_role, s.d_state, s.d_out_roles};
  for (void* p : d)
    if (p) (void)hipFree(p);
  s.d_lower = s.d_parent = s.d_label = s.d_out_labels = nullptr;
  s.d_role = s.d_state = s.d_out_roles = nullptr;
  s.cap_n = 0;
  s.cap_m = 0;
}

hipError_t alloc_slot_buffers(Slot& s, int32_t n, int64_t m) {
  free_slot_buffers(s);
  const size_t N = (size_t)(n > 0 ? n : 1), M = (size_t)(m > 0 ? m : 1);
  hipError_t e;
  if ((e = hipMalloc((void**)&s.d_lower, 4 * N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_parent, 4 * N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_label, 4 * N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_out_labels, 4 * N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_role, N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_out_roles, N)) != hipSuccess) return e;
  if ((e = hipMalloc((void**)&s.d_state, M)) != hipSuccess) return e;
  s.cap_n = n;
  s.cap_m = m;
  return hipSuccess;
}

}  // namespace

// The partitioned graph the fallback worker built last, kept for the next
// query of the same non-resident graph; its budget counts as resident bytes.
struct FallbackGraph {
  int32_t gid = -1;
  scan_graph* g = nullptr;
  uint64_t bytes = 0;
  bool busy = false;  // a query is running on it (outside the server lock)
};

struct scan_server {
  scan_opts opts{};
  uint64_t budget = 0;  // 0 = no cap
  uint64_t resident_bytes = 0;
  std::mutex mu;
  std::condition_variable cv_work;  // dispatcher wake-up
  std::condition_variable cv_done;  // waiters
  std::condition_variable cv_fb;    // fallback worker wake-up
  std::map<int32_t, std::unique_ptr<ServedGraph>> graphs;
  int32_t next_gid = 0;
  int64_t next_req = 1;
  std::deque<std::shared_ptr<Request>> pending;
  std::deque<std::shared_ptr<Request>> fb_pending;  // queries of non-resident graphs
  FallbackGraph fb;
  std::map<int64_t, std::shared_ptr<Request>> requests;
  std::vector<Slot> slots;
  std::vector<OutBuf> out_free;  // result buffers not in use
  int32_t out_total = 0;         // result buffers allocated
  int32_t out_max = 0;           // bound on them
  int32_t slot_n = 0;  // slot scratch capacity
  int64_t slot_m = 0;
  int64_t completed = 0;
  bool stop = false;
  bool pause_dispatch = false;  // set while slot buffers are being resized
  bool dispatch_done = false;   // the dispatcher has stopped (no more fallback queries)
  std::thread worker;
  std::thread fb_worker;
};

namespace {

void finish(scan_server* S, const std::shared_ptr<Request>& r) {
  r->t_done = Clock::now();
  S->completed++;
  S->cv_done.notify_all();
}

// Drops the cached partitioned graph (server lock held; not busy).
void fallback_evict(scan_server* S) {
  if (S->fb.g) scan_graph_destroy(S->fb.g);
  S->resident_bytes -= S->fb.bytes;
  S->fb = FallbackGraph();
}

// Fallback worker: queries of graphs kept outside the device, one at a time,
// each through a partitioned graph (built with the budget left over, on its
// own library stream) that is kept for the next query of the same graph.  Runs
// beside the dispatcher, which keeps admitting and completing resident queries.
void fallback_loop(scan_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_fb.wait(lk, [&] { return S->dispatch_done || !S->fb_pending.empty(); });
    if (S->fb_pending.empty()) break;  // the dispatcher has stopped and nothing is left
    auto r = S->fb_pending.front();
    S->fb_pending.pop_front();
    ServedGraph* G = S->graphs[r->gid].get();
    int rc = SCAN_OK;
    std::string error;
    if (S->fb.gid != r->gid) {
      fallback_evict(S);
      const uint64_t budget = S->budget > S->resident_bytes ? S->budget - S->resident_bytes : 1;
      S->resident_bytes += budget;
      S->fb.gid = r->gid;
      S->fb.bytes = budget;
      S->fb.busy = true;
      scan_opts o = S->opts;
      o.hip_stream = nullptr;
      o.device_budget_bytes = budget;
      scan_graph* g = nullptr;
      lk.unlock();
      // the host CSR stays valid: the graph is not removed while a query on it is in flight
      rc = scan_graph_create(G->n, G->nnz, G->h_rp.data(), G->h_ci.data(), &o, &g);
      if (rc != SCAN_OK) error = scan_last_error();
      lk.lock();
      S->fb.g = g;
      S->fb.busy = false;
      if (rc != SCAN_OK) fallback_evict(S);
    }
    if (rc == SCAN_OK) {
      scan_graph* g = S->fb.g;
      S->fb.busy = true;
      std::vector<int32_t> labels((size_t)G->n);
      std::vector<uint8_t> roles((size_t)G->n);
      const int64_t p = r->p, q = r->q;
      const int32_t mu = r->mu;
      lk.unlock();
      rc = scan_run(g, p, q, mu, labels.data(), roles.data());
      if (rc != SCAN_OK) error = scan_last_error();
      lk.lock();
      S->fb.busy = false;
      r->labels.swap(labels);
      r->roles.swap(roles);
    }
    r->error = error;
    r->status = rc;
    G->inflight--;
    finish(S, r);
  }
}

// Starts one request on a free slot (server lock held).  Returns false if
// the request finished at once (with an error).
bool launch_on_slot(scan_server* S, Slot& slot, const std::shared_ptr<Request>& r, ServedGraph* G) {
  int64_t p = r->p, q = r->q;
  int64_t a = p, b = q;
  while (b) { int64_t t = a % b; a = b; b = t; }
  p /= a;
  q /= a;
  scan_graph* g = G->g;
  if (G->n > slot.cap_n || G->m > slot.cap_m) {
    r->status = SCAN_E_NOMEM;
    r->error = "slot scratch smaller than the graph";
    return false;
  }
  if (!slot.out.labels || slot.out.cap < G->n) {
    r->status = SCAN_E_NOMEM;
    r->error = "no result buffer";
    return false;
  }
  launch_rethreshold(slot.stream, G->n, G->m, g->d_edges, G->d_ecount, G->d_ab, (uint64_t)p, (uint64_t)q,
                     r->mu, slot.d_lower, slot.d_role, slot.d_parent, slot.d_label, slot.d_state,
                     slot.d_out_labels, slot.d_out_roles, S->opts.hub_outlier ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && G->n > 0)
    e = hipMemcpyAsync(slot.out.labels, slot.d_out_labels, 4 * (size_t)G->n, hipMemcpyDeviceToHost, slot.stream);
  if (e == hipSuccess && G->n > 0)
    e = hipMemcpyAsync(slot.out.roles, slot.d_out_roles, (size_t)G->n, hipMemcpyDeviceToHost, slot.stream);
  if (e == hipSuccess) e = hipEventRecord(slot.done, slot.stream);
  if (e != hipSuccess) {
    r->status = SCAN_E_DEVICE;
    r->error = hipGetErrorString(e);
    return false;
  }
  G->inflight++;
  slot.req = r;
  return true;
}

// A result buffer can be had (server lock held).
bool out_available(const scan_server* S) { return !S->out_free.empty() || S->out_total < S->out_max; }

// Gives the slot a result buffer of the current capacity if it has none
// (server lock held); false when the pool is exhausted.
bool acquire_out(scan_server* S, Slot& slot) {
  if (slot.out.labels && slot.out.cap >= S->slot_n) return true;
  if (slot.out.labels) {  // too small since the capacity grew
    free_out(slot.out);
    --S->out_total;
  }
  while (!S->out_free.empty()) {
    OutBuf b = S->out_free.back();
    S->out_free.pop_back();
    if (b.cap >= S->slot_n) {
      slot.out = b;
      return true;
    }
    free_out(b);
    --S->out_total;
  }
  if (S->out_total >= S->out_max) return false;
  const size_t N = (size_t)(S->slot_n > 0 ? S->slot_n : 1);
  OutBuf b;
  if (hipHostMalloc((void**)&b.labels, 4 * N, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b.roles, N, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    free_out(b);
    return false;
  }
  b.cap = S->slot_n;
  slot.out = b;
  ++S->out_total;
  return true;
}

void worker_loop(scan_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progress = false;
    // completions
    for (auto& slot : S->slots) {
      if (!slot.req) continue;
      const hipError_t q = hipEventQuery(slot.done);
      if (q == hipErrorNotReady) continue;
      auto r = slot.req;
      slot.req.reset();
      ServedGraph* G = S->graphs[r->gid].get();
      G->inflight--;
      if (q == hipSuccess) {
        // the buffer goes to the request; the slot takes another at its next admission
        r->out = slot.out;
        r->n = G->n;
        slot.out = OutBuf();
        r->status = SCAN_OK;
      } else {
        r->status = SCAN_E_DEVICE;
        r->error = hipGetErrorString(q);
      }
      finish(S, r);
      progress = true;
    }
    // admissions: queries of non-resident graphs go to the fallback worker;
    // resident ones, in order of arrival, onto free slots
    for (auto it = S->pending.begin(); it != S->pending.end() && !S->pause_dispatch;) {
      auto r = *it;
      auto git = S->graphs.find(r->gid);
      ServedGraph* G = git == S->graphs.end() ? nullptr : git->second.get();
      if (!G) {
        r->status = SCAN_E_INVAL;
        r->error = "unknown graph id";
        finish(S, r);
      } else if (!G->resident) {
        G->inflight++;
        S->fb_pending.push_back(r);
        S->cv_fb.notify_one();
      } else {
        Slot* free_slot = nullptr;
        for (auto& slot : S->slots)
          if (!slot.req) {
            free_slot = &slot;
            break;
          }
        if (!free_slot) {
          ++it;
          continue;
        }
        if (!acquire_out(S, *free_slot)) break;  // every result buffer awaits collection
        if (!launch_on_slot(S, *free_slot, r, G)) finish(S, r);
      }
      it = S->pending.erase(it);
      progress = true;
    }
    bool busy = false;
    for (auto& slot : S->slots) busy = busy || (bool)slot.req;
    if (S->stop && !busy && S->pending.empty()) {
      // every request is on its way: the fallback worker may finish its queue and stop
      S->dispatch_done = true;
      S->cv_fb.notify_all();
      break;
    }
    if (!progress) {
      if (busy) {
        // poll the running slots without holding the lock
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        // woken by a submit, a returned result buffer, a resumed dispatch or a stop
        S->cv_work.wait(lk, [&] {
          return S->stop || (!S->pending.empty() && !S->pause_dispatch && out_available(S));
        });
      }
    }
  }
}

// Stop admissions and wait (lock held) until no slot is running, so that
// slot buffers can be replaced; the caller clears pause_dispatch afterwards.
void drain(scan_server* S, std::unique_lock<std::mutex>& lk) {
  S->pause_dispatch = true;
  S->cv_done.wait(lk, [&] {
    for (auto& s : S->slots)
      if (s.req) return false;
    return true;
  });
}

}  // namespace

extern "C" {

int scan_server_create(const scan_opts* opts, int32_t num_slots, scan_server** out) {
  if (!out) return fail(SCAN_E_INVAL, "out is NULL");
  *out = nullptr;
  if (num_slots < 1 || num_slots > 64) return fail(SCAN_E_INVAL, "num_slots must be in 1..64");
  auto* S = new (std::nothrow) scan_server();
  if (!S) return fail(SCAN_E_NOMEM, "host allocation failed");
  if (opts) S->opts = *opts;
  else scan_opts_default(&S->opts);
  S->opts.hip_stream = nullptr;
  S->budget = S->opts.device_budget_bytes;
  S->slots.resize((size_t)num_slots);
  S->out_max = 4 * num_slots + 16;
  for (auto& s : S->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      for (auto& t : S->slots) {
        if (t.stream) (void)hipStreamDestroy(t.stream);
        if (t.done) (void)hipEventDestroy(t.done);
      }
      delete S;
      return fail(SCAN_E_DEVICE, "cannot create slot streams");
    }
  }
  S->worker = std::thread(worker_loop, S);
  S->fb_worker = std::thread(fallback_loop, S);
  *out = S;
  return SCAN_OK;
}

int scan_server_add_graph(scan_server* S, int32_t n, int64_t nnz, const int64_t* row_ptr,
                          const int32_t* col_idx, int32_t* gid_out) {
  if (!S || !gid_out) return fail(SCAN_E_INVAL, "NULL argument");
  if (n < 0 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx)) return fail(SCAN_E_INVAL, "bad CSR arguments");
  auto G = std::make_unique<ServedGraph>();
  G->n = n;
  G->nnz = nnz;
  G->m = nnz / 2;
  const uint64_t gbytes = graph_bytes(n, nnz, S->opts);
  bool resident;
  {
    // admission: reserve the graph's peak bytes and what the slots would grow
    // by; an idle cached fallback graph gives its budget back first if needed
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t new_n = n > S->slot_n ? n : S->slot_n;
    const int64_t new_m = G->m > S->slot_m ? G->m : S->slot_m;
    const uint64_t grow = S->slots.size() * (slot_bytes(new_n, new_m) - slot_bytes(S->slot_n, S->slot_m));
    auto fits = [&] { return S->budget == 0 || S->resident_bytes + gbytes + grow <= S->budget; };
    resident = fits();
    if (!resident && S->fb.g && !S->fb.busy) {
      fallback_evict(S);
      resident = fits();
    }
    if (resident) S->resident_bytes += gbytes;
  }
  uint64_t held = gbytes;  // bytes reserved for this graph so far
  if (resident) {
    scan_opts o = S->opts;
    o.device_budget_bytes = 0;
    scan_graph* g = nullptr;
    int rc = scan_graph_create(n, nnz, row_ptr, col_idx, &o, &g);
    G->g = g;
    if (rc == SCAN_OK && g->m > 0) {
      hipError_t e = hipMalloc((void**)&G->d_ecount, sizeof(int32_t) * (size_t)g->m);
      if (e == hipSuccess) e = hipMalloc((void**)&G->d_ab, sizeof(uint64_t) * (size_t)g->m);
      if (e != hipSuccess) {
        rc = fail_hip(e, "hipMalloc counts");
      } else {
        std::lock_guard<std::mutex> glk(g->lock);
        rc = run_counts(g, nullptr, G->d_ecount, g->stream);
        if (rc == SCAN_OK) {
          launch_closed_products(g->stream, g->m, g->d_rp, g->d_edges, G->d_ab);
          e = hipGetLastError();
          if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
          if (e != hipSuccess) rc = fail_hip(e, "closed-size products");
        }
      }
    }
    if (rc == SCAN_OK) {
      // queries never intersect again: the rows renamed by degree rank and
      // the other inputs of the intersections, used only by the counting run,
      // are released
      if (g->d_hci) {
        (void)hipFree(g->d_hci);
        g->d_hci = nullptr;
      }
      if (g->d_hsamp) {  // samples of the rows the counting run read
        (void)hipFree(g->d_hsamp);
        g->d_hsamp = nullptr;
      }
      if (g->d_edeg) {  // degree pairs (the closed-size products replace them)
        (void)hipFree(g->d_edeg);
        g->d_edeg = nullptr;
      }
      const uint64_t now = graph_device_bytes(g) + 12ull * (uint64_t)g->m;
      std::lock_guard<std::mutex> lk(S->mu);
      S->resident_bytes -= held;
      S->resident_bytes += now;
      held = now;
    }
    if (rc != SCAN_OK) {
      release_resident(G.get());
      std::lock_guard<std::mutex> lk(S->mu);
      S->resident_bytes -= held;
      return rc;
    }
    G->resident = true;
    G->bytes = held;
  } else {
    G->h_rp.assign(row_ptr, row_ptr + n + 1);
    if (nnz > 0) G->h_ci.assign(col_idx, col_idx + nnz);
  }
  std::unique_lock<std::mutex> lk(S->mu);
  if (resident && (n > S->slot_n || G->m > S->slot_m)) {
    const int32_t new_n = n > S->slot_n ? n : S->slot_n;
    const int64_t new_m = G->m > S->slot_m ? G->m : S->slot_m;
    drain(S, lk);
    hipError_t e = hipSuccess;
    for (auto& s : S->slots)
      if (e == hipSuccess) e = alloc_slot_buffers(s, new_n, new_m);
    if (e != hipSuccess) {
      for (auto& s : S->slots) (void)alloc_slot_buffers(s, S->slot_n, S->slot_m);
      S->pause_dispatch = false;
      S->cv_work.notify_one();
      S->resident_bytes -= held;
      lk.unlock();
      release_resident(G.get());
      return fail_hip(e, "slot scratch");
    }
    S->resident_bytes += S->slots.size() * (slot_bytes(new_n, new_m) - slot_bytes(S->slot_n, S->slot_m));
    S->slot_n = new_n;
    S->slot_m = new_m;
    S->pause_dispatch = false;
    S->cv_work.notify_one();
  }
  const int32_t gid = S->next_gid++;
  S->graphs[gid] = std::move(G);
  *gid_out = gid;
  return SCAN_OK;
}

int scan_server_set_budget(scan_server* S, uint64_t device_budget_bytes) {
  if (!S) return fail(SCAN_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  S->budget = device_budget_bytes;
  return SCAN_OK;
}

int scan_server_remove_graph(scan_server* S, int32_t gid) {
  if (!S) return fail(SCAN_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->graphs.find(gid);
  if (it == S->graphs.end()) return fail(SCAN_E_INVAL, "unknown graph id %d", gid);
  ServedGraph* G = it->second.get();
  G->removing = true;
  S->cv_done.wait(lk, [&] {
    if (G->inflight > 0) return false;
    for (auto& r : S->pending)
      if (r->gid == gid) return false;
    return true;
  });
  if (S->fb.gid == gid) fallback_evict(S);  // idle: its queries are done
  if (G->resident) {
    release_resident(G);
    S->resident_bytes -= G->bytes;
  }
  S->graphs.erase(it);
  return SCAN_OK;
}

int scan_server_submit(scan_server* S, int32_t gid, int64_t eps_num, int64_t eps_den, int32_t mu,
                       int64_t* req_out) {
  if (!S || !req_out) return fail(SCAN_E_INVAL, "NULL argument");
  if (eps_num < 1 || eps_den < eps_num) return fail(SCAN_E_INVAL, "eps must satisfy 1 <= eps_num <= eps_den");
  if (mu < 2) return fail(SCAN_E_INVAL, "mu must be >= 2");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->graphs.find(gid);
  if (it == S->graphs.end() || it->second->removing) return fail(SCAN_E_INVAL, "unknown graph id %d", gid);
  const ServedGraph* G = it->second.get();
  if (G->resident) {
    int64_t a = eps_num, b = eps_den;
    while (b) { int64_t t = a % b; a = b; b = t; }
    const unsigned __int128 q = (unsigned __int128)(eps_den / a);
    if (q * (unsigned __int128)((uint64_t)G->g->max_degree + 1) >= ((unsigned __int128)1 << 32))
      return fail(SCAN_E_RANGE, "eps denominator too large for this graph's maximum degree");
  }
  auto r = std::make_shared<Request>();
  r->id = S->next_req++;
  r->gid = gid;
  r->p = eps_num;
  r->q = eps_den;
  r->mu = mu;
  r->t_submit = Clock::now();
  S->requests[r->id] = r;
  S->pending.push_back(r);
  *req_out = r->id;
  S->cv_work.notify_one();
  return SCAN_OK;
}

int scan_server_wait(scan_server* S, int64_t req, int32_t* labels, uint8_t* roles, double* latency_ms) {
  if (!S) return fail(SCAN_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->requests.find(req);
  if (it == S->requests.end()) return fail(SCAN_E_INVAL, "unknown request %lld", (long long)req);
  auto r = it->second;
  S->cv_done.wait(lk, [&] { return r->status != 1; });
  S->requests.erase(req);
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  if (r->status != SCAN_OK) return fail(r->status, "%s", r->error.c_str());
  if (r->out.labels) {
    // copy out of the pinned buffer without the lock, then give it back
    const OutBuf b = r->out;
    r->out = OutBuf();
    lk.unlock();
    if (labels) memcpy(labels, b.labels, 4 * (size_t)r->n);
    if (roles) memcpy(roles, b.roles, (size_t)r->n);
    lk.lock();
    S->out_free.push_back(b);
    S->cv_work.notify_one();
    return SCAN_OK;
  }
  if (labels && !r->labels.empty()) memcpy(labels, r->labels.data(), 4 * r->labels.size());
  if (roles && !r->roles.empty()) memcpy(roles, r->roles.data(), r->roles.size());
  return SCAN_OK;
}

int scan_server_info(scan_server* S, uint64_t* resident_bytes, int32_t* graphs, int32_t* resident_graphs,
                     int64_t* completed) {
  if (!S) return fail(SCAN_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  int32_t res = 0;
  for (auto& kv : S->graphs) res += kv.second->resident ? 1 : 0;
  if (resident_bytes) *resident_bytes = S->resident_bytes;
  if (graphs) *graphs = (int32_t)S->graphs.size();
  if (resident_graphs) *resident_graphs = res;
  if (completed) *completed = S->completed;
  return SCAN_OK;
}

int scan_server_destroy(scan_server* S) {
  if (!S) return SCAN_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  if (S->fb_worker.joinable()) S->fb_worker.join();
  fallback_evict(S);
  for (auto& kv : S->graphs) {
    ServedGraph* G = kv.second.get();
    if (G->resident) release_resident(G);
  }
  for (auto& s : S->slots) {
    free_slot_buffers(s);
    free_out(s.out);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  for (auto& b : S->out_free) free_out(b);
  for (auto& kv : S->requests) free_out(kv.second->out);  // results never collected
  delete S;
  return SCAN_OK;
}

}  // extern "C"
