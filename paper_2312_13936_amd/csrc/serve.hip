// Batched and served Leiden: many independent graphs on one GPU.
//
// Both run the single-graph path (gvl_leiden) on a pool of "lanes".  A lane
// is a HIP stream (default priority) with its own context (pinned read-back
// buffers) and a device workspace, driven by one host worker thread; lanes
// overlap on the device, so small graphs that cannot fill the GPU alone share
// it.  Every graph runs exactly the code path it runs alone, so results are
// identical alone and in a batch or a served mix (bit-exact in deterministic
// mode).
//
// Serving adds continuous admission: requests queue in arrival order; a free
// lane takes the oldest waiting request whose workspace fits into the free
// part of the caller's device arena, so requests that arrive while others
// run are admitted as lanes and memory free up.  Results go to the caller's
// own output buffers, so the arena only ever holds the workspaces of running
// requests: once nothing runs it is one free block again, and every request
// that passed the size check at submission is eventually admitted.  A request may be overtaken by later, smaller ones at most
// kMaxBypass times; after that admission waits until it fits, so a large
// request cannot starve.  Latency is measured from submission to completion
// on the host steady clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "gvl.h"

hipStream_t gvl_context_stream(gvl_ctx_t ctx);  // driver.hip

namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kMaxBypass = 64;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Lane {
  hipStream_t stream = nullptr;
  gvl_ctx_t ctx = nullptr;
};

gvl_status make_lanes(int device, int32_t lanes, std::vector<Lane>& out) {
  if (hipSetDevice(device) != hipSuccess) return GVL_E_HIP;
  out.assign(lanes, Lane());
  for (int32_t k = 0; k < lanes; ++k) {
    if (hipStreamCreateWithFlags(&out[k].stream, hipStreamNonBlocking) != hipSuccess) return GVL_E_HIP;
    gvl_status s = gvl_create(&out[k].ctx, device, out[k].stream);
    if (s != GVL_OK) return s;
  }
  return GVL_OK;
}

void free_lanes(std::vector<Lane>& lanes) {
  for (Lane& l : lanes) {
    if (l.stream) (void)hipStreamSynchronize(l.stream);
    if (l.ctx) gvl_destroy(l.ctx);
    if (l.stream) (void)hipStreamDestroy(l.stream);
  }
  lanes.clear();
}

size_t graph_ws_bytes(const gvl_graph_desc& g, const gvl_options* opt) {
  size_t b = 0;
  gvl_workspace_bytes(g.n, g.m, opt, &b);
  return align_up(b);
}

// First-fit allocator over a device arena (offsets only).
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
    total_ = bytes;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t total() const { return total_; }
  size_t largest() const {
    size_t mx = 0;
    for (const auto& kv : free_) mx = std::max(mx, kv.second);
    return mx;
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;
  size_t total_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace

extern "C" {

// ------------------------------------------------------------------ batch ---

gvl_status gvl_batch_workspace_bytes(int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                                     int32_t lanes, size_t* bytes) {
  if (!bytes || num_graphs < 0 || (num_graphs > 0 && !graphs) || lanes < 1 || !opt) return GVL_E_INVALID_ARG;
  size_t mx = kAlign;
  for (int32_t g = 0; g < num_graphs; ++g) {
    if (graphs[g].n < 0 || graphs[g].m < 0) return GVL_E_INVALID_ARG;
    mx = std::max(mx, graph_ws_bytes(graphs[g], opt));
  }
  *bytes = mx * (size_t)lanes;
  return GVL_OK;
}

gvl_status gvl_leiden_batch(gvl_ctx_t ctx, int32_t num_graphs, const gvl_graph_desc* graphs, const gvl_options* opt,
                            int32_t lanes, void* d_workspace, size_t workspace_bytes, double* modularities,
                            gvl_status* statuses) {
  if (!ctx || num_graphs < 0 || (num_graphs > 0 && (!graphs || !modularities)) || lanes < 1 || lanes > 64 || !opt)
    return GVL_E_INVALID_ARG;
  size_t need = 0;
  gvl_status s = gvl_batch_workspace_bytes(num_graphs, graphs, opt, lanes, &need);
  if (s != GVL_OK) return s;
  if (!d_workspace || workspace_bytes < need) return GVL_E_WORKSPACE;
  if (num_graphs == 0) return GVL_OK;
  const size_t slice = need / (size_t)lanes;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return GVL_E_HIP;
  std::vector<Lane> pool;
  s = make_lanes(device, lanes, pool);
  if (s != GVL_OK) { free_lanes(pool); return s; }
  // inputs produced on the caller's stream are visible to every lane
  hipStream_t caller = gvl_context_stream(ctx);
  hipEvent_t ready;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) { free_lanes(pool); return GVL_E_HIP; }
  (void)hipEventRecord(ready, caller);
  for (Lane& l : pool) (void)hipStreamWaitEvent(l.stream, ready, 0);
  std::atomic<int32_t> next{0};
  std::atomic<int32_t> failures{0};
  auto work = [&](int32_t k) {
    (void)hipSetDevice(device);
    char* ws = (char*)d_workspace + slice * (size_t)k;
    for (int32_t g = next++; g < num_graphs; g = next++) {
      const gvl_graph_desc& d = graphs[g];
      double q = 0.0;
      gvl_status st = gvl_leiden(pool[k].ctx, d.n, d.m, d.d_offsets, d.d_indices, d.d_weights, d.resolution, opt, ws,
                                 slice, d.d_membership, &q, nullptr);
      modularities[g] = q;
      if (statuses) statuses[g] = st;
      if (st != GVL_OK) ++failures;
    }
  };
  std::vector<std::thread> th;
  for (int32_t k = 1; k < lanes; ++k) th.emplace_back(work, k);
  work(0);
  for (auto& t : th) t.join();
  free_lanes(pool);
  (void)hipEventDestroy(ready);
  return failures.load() ? GVL_E_BATCH : GVL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- serving ---

struct gvl_server {
  struct Request {
    gvl_graph_desc g;
    size_t ws_bytes = 0, off = 0;
    int32_t state = GVL_REQ_PENDING;
    int32_t bypassed = 0;  // times a later request was admitted first
    double q = 0.0;
    gvl_status result = GVL_OK;
    std::chrono::steady_clock::time_point t_submit, t_start, t_done;
  };
  int device = 0;
  gvl_options opt;
  char* arena = nullptr;
  Arena alloc;
  std::vector<Lane> lanes;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;
  std::map<uint64_t, Request> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  int64_t completed = 0, running = 0, max_running = 0;
  // micro-batching: a lane that admits a request of at most batch_vertices
  // vertices fuses up to batch_max waiting requests of that size into one
  // gvl_leiden_fused run (results identical to solo runs)
  int32_t batch_max = 32;
  int64_t batch_vertices = 262144;

  // With the lock held: the waiting requests fused with the admitted `head`
  // (its own workspace at head.off), their workspace allocated in the arena.
  // Returns the group (head first); group size 1 keeps the solo workspace.
  std::vector<uint64_t> fuse_group(uint64_t head, size_t* off, size_t* bytes) {
    std::vector<uint64_t> group{head};
    Request& h = reqs[head];
    *off = h.off;
    *bytes = h.ws_bytes;
    if (batch_max < 2 || h.g.n > batch_vertices) return group;
    std::vector<gvl_graph_desc> descs{h.g};
    alloc.release(h.off, h.ws_bytes);
    const size_t room = alloc.largest();
    size_t fb = 0;
    for (auto it = pending.begin(); it != pending.end() && (int32_t)group.size() < batch_max; ++it) {
      const Request& q = reqs[*it];
      if (q.g.n > batch_vertices) continue;
      descs.push_back(q.g);
      size_t b = 0;
      if (gvl_fused_workspace_bytes((int32_t)descs.size(), descs.data(), &opt, &b) != GVL_OK || b > room) {
        descs.pop_back();
        break;
      }
      group.push_back(*it);
      fb = b;
    }
    size_t o = 0;
    if (group.size() > 1 && alloc.alloc(fb, &o)) {
      for (size_t j = 1; j < group.size(); ++j) {
        pending.erase(std::find(pending.begin(), pending.end(), group[j]));
        if (!pending.empty() && pending.front() != group[j]) ++reqs[pending.front()].bypassed;
      }
      *off = o;
      *bytes = fb;
      return group;
    }
    (void)alloc.alloc(h.ws_bytes, &h.off);  // the block just freed: always fits again
    *off = h.off;
    return std::vector<uint64_t>{head};
  }

  void worker(int k) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      uint64_t id = 0;
      Request* r = nullptr;
      while (!stop) {
        for (auto it = pending.begin(); it != pending.end(); ++it) {
          Request& q = reqs[*it];
          size_t off = 0;
          if (alloc.alloc(q.ws_bytes, &off)) {
            q.off = off;
            id = *it;
            r = &q;
            if (it != pending.begin()) ++reqs[pending.front()].bypassed;
            pending.erase(it);
            break;
          }
          if (q.bypassed >= kMaxBypass) break;  // the oldest request goes next
        }
        if (r) break;
        cv.wait(lk);
      }
      if (!r) return;  // stopping
      size_t goff = 0, gbytes = 0;
      const std::vector<uint64_t> group = fuse_group(id, &goff, &gbytes);
      const auto t_start = std::chrono::steady_clock::now();
      std::vector<gvl_graph_desc> descs;
      for (uint64_t gid : group) {
        Request& q = reqs[gid];
        q.state = GVL_REQ_RUNNING;
        q.t_start = t_start;
        descs.push_back(q.g);
      }
      running += (int64_t)group.size();
      max_running = std::max(max_running, running);
      char* ws = arena + goff;
      lk.unlock();
      std::vector<double> qs(group.size(), 0.0);
      std::vector<gvl_status> sts(group.size(), GVL_OK);
      if (group.size() == 1) {
        const gvl_graph_desc& g = descs[0];
        sts[0] = gvl_leiden(lanes[k].ctx, g.n, g.m, g.d_offsets, g.d_indices, g.d_weights, g.resolution, &opt, ws,
                            gbytes, g.d_membership, &qs[0], nullptr);
      } else {
        const gvl_status all = gvl_leiden_fused(lanes[k].ctx, (int32_t)group.size(), descs.data(), &opt, ws, gbytes,
                                                qs.data(), sts.data());
        if (all != GVL_OK && all != GVL_E_BATCH)
          for (auto& x : sts) x = all;
      }
      lk.lock();
      const auto t_done = std::chrono::steady_clock::now();
      for (size_t j = 0; j < group.size(); ++j) {
        Request& rr = reqs[group[j]];
        rr.q = qs[j];
        rr.result = sts[j];
        rr.t_done = t_done;
        rr.state = GVL_REQ_DONE;
      }
      alloc.release(goff, gbytes);
      running -= (int64_t)group.size();
      completed += (int64_t)group.size();
      cv.notify_all();
    }
  }
};

extern "C" {

gvl_status gvl_server_create(gvl_server_t* out, int device, int32_t lanes, const gvl_options* opt, void* d_arena,
                             size_t arena_bytes) {
  if (!out || !opt || lanes < 1 || lanes > 64 || !d_arena || arena_bytes < kAlign) return GVL_E_INVALID_ARG;
  *out = nullptr;
  gvl_server* s = new gvl_server();
  s->device = device;
  s->opt = *opt;
  s->arena = (char*)d_arena;
  s->alloc.reset(arena_bytes & ~(kAlign - 1));
  gvl_status st = make_lanes(device, lanes, s->lanes);
  if (st != GVL_OK) {
    free_lanes(s->lanes);
    delete s;
    return st;
  }
  for (int k = 0; k < lanes; ++k) s->workers.emplace_back(&gvl_server::worker, s, k);
  *out = s;
  return GVL_OK;
}

gvl_status gvl_server_submit(gvl_server_t s, const gvl_graph_desc* g, uint64_t* ticket) {
  if (!s || !g || !ticket || g->n < 0 || g->m < 0 || (g->n > 0 && !g->d_membership)) return GVL_E_INVALID_ARG;
  gvl_server::Request r;
  r.g = *g;
  r.ws_bytes = graph_ws_bytes(*g, &s->opt);
  r.t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  if (r.ws_bytes > s->alloc.total()) return GVL_E_WORKSPACE;
  const uint64_t id = s->next_id++;
  s->reqs[id] = r;
  s->pending.push_back(id);
  *ticket = id;
  s->cv.notify_all();
  return GVL_OK;
}

static void fill_result(gvl_server_t s, const gvl_server::Request& r, gvl_request_info* info) {
  info->state = r.state;
  info->result = r.result;
  info->modularity = r.q;
  using ms = std::chrono::duration<double, std::milli>;
  info->latency_ms = r.state == GVL_REQ_DONE ? ms(r.t_done - r.t_submit).count() : 0.0;
  info->queue_ms = r.state != GVL_REQ_PENDING ? ms(r.t_start - r.t_submit).count() : 0.0;
}

gvl_status gvl_server_poll(gvl_server_t s, uint64_t ticket, gvl_request_info* info) {
  if (!s || !info) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GVL_E_INVALID_ARG;
  fill_result(s, it->second, info);
  return GVL_OK;
}

gvl_status gvl_server_wait(gvl_server_t s, uint64_t ticket, int64_t timeout_ms, gvl_request_info* info) {
  if (!s || !info) return GVL_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  // look the ticket up again after every wake-up: another thread may release it
  auto it = s->reqs.find(ticket);
  auto finished = [&] {
    it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.state == GVL_REQ_DONE || it->second.state == GVL_REQ_CANCELLED;
  };
  if (timeout_ms < 0) {
    s->cv.wait(lk, finished);
  } else if (!s->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished)) {
    fill_result(s, it->second, info);
    return GVL_E_BUSY;
  }
  if (it == s->reqs.end()) return GVL_E_INVALID_ARG;
  fill_result(s, it->second, info);
  return GVL_OK;
}

gvl_status gvl_server_cancel(gvl_server_t s, uint64_t ticket) {
  if (!s) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GVL_E_INVALID_ARG;
  if (it->second.state != GVL_REQ_PENDING) return GVL_E_BUSY;
  s->pending.erase(std::find(s->pending.begin(), s->pending.end(), ticket));
  it->second.state = GVL_REQ_CANCELLED;
  s->cv.notify_all();
  return GVL_OK;
}

gvl_status gvl_server_release(gvl_server_t s, uint64_t ticket) {
  if (!s) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return GVL_E_INVALID_ARG;
  gvl_server::Request& r = it->second;
  if (r.state == GVL_REQ_PENDING || r.state == GVL_REQ_RUNNING) return GVL_E_BUSY;
  s->reqs.erase(it);
  s->cv.notify_all();
  return GVL_OK;
}

gvl_status gvl_server_set_batching(gvl_server_t s, int32_t max_batch, int64_t max_vertices) {
  if (!s || max_batch < 1 || max_vertices < 0) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->batch_max = max_batch;
  s->batch_vertices = max_vertices;
  return GVL_OK;
}

gvl_status gvl_server_stats(gvl_server_t s, gvl_server_info* info) {
  if (!s || !info) return GVL_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  info->completed = s->completed;
  info->pending = (int64_t)s->pending.size();
  info->running = s->running;
  info->max_running = s->max_running;
  info->arena_bytes = s->alloc.total();
  info->arena_used = s->alloc.used();
  info->arena_peak = s->alloc.peak();
  return GVL_OK;
}

gvl_status gvl_server_destroy(gvl_server_t s) {
  if (!s) return GVL_E_INVALID_ARG;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // finish admitted work; requests still waiting are cancelled
    for (uint64_t id : s->pending) s->reqs[id].state = GVL_REQ_CANCELLED;
    s->pending.clear();
    s->cv.wait(lk, [&] { return s->running == 0; });
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  free_lanes(s->lanes);
  delete s;
  return GVL_OK;
}

}  // extern "C"
