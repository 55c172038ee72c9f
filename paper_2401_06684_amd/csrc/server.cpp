// Serving runtime: a request loop over fa_apply with continuous admission.
//
// Requests (one f(A)b solve each, any operator, kind, tolerance) are queued
// in arrival order.  A request is admitted when a worker is idle and the
// device pool has room for its workspace (the Krylov basis, m_max + 1
// vectors of n entries, plus scratch: the figure of fa_workspace_bytes), so
// the basis memory m_max * n bounds how many solves are in flight.  Each
// worker owns a HIP stream; admitted solves run concurrently on the device,
// their kernels interleaving as the hardware queues allow, and a finished
// solve frees its memory and its worker for the next admission at once
// (requests join and leave the running set at any Krylov step of the
// others, not in rounds).  The kernels are deterministic and do not depend
// on what else runs, so a solve gives the same bits alone and in the mix.
//
// Pool allocator: first fit over a free list kept sorted by offset, blocks
// 256-byte aligned, neighbours coalesced on free.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fa.h"

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Pool {
  size_t size = 0;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, bytes), sorted by offset

  void init(size_t bytes) {
    size = bytes;
    free_list.assign(1, {0, bytes});
  }
  // first fit; returns false when no free block is large enough
  bool take(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (size_t i = 0; i < free_list.size(); ++i) {
      if (free_list[i].second >= bytes) {
        *off = free_list[i].first;
        free_list[i].first += bytes;
        free_list[i].second -= bytes;
        if (free_list[i].second == 0) free_list.erase(free_list.begin() + (long)i);
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, size_t(0)));
    it = free_list.insert(it, {off, bytes});
    // merge with the next, then with the previous block
    auto nx = it + 1;
    if (nx != free_list.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_list.erase(nx);
    }
    if (it != free_list.begin()) {
      auto pv = it - 1;
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_list.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (const auto& f : free_list) m = std::max(m, f.second);
    return m;
  }
};

struct Request {
  fa_op op;
  int kind;
  const void* b;
  void* x;
  int m_max;
  double tol;
  int check_every;
  uint32_t flags;
  size_t ws_bytes;
  size_t ws_off = 0;
  bool done = false;
  fa_request_info info;
};

}  // namespace

struct fa_server_s {
  int device = 0;
  char* pool_base = nullptr;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Request> reqs;
  uint64_t next_id = 1;
  int inflight = 0;
  size_t bytes_inflight = 0, peak_bytes = 0;
  int peak_inflight = 0;
  uint64_t completed = 0;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;

  void worker(int w) {
    const bool dev_ok = hipSetDevice(device) == hipSuccess;
    hipStream_t s = streams[w];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      // admission: the oldest request, when the pool has room for it
      size_t off = 0;
      cv_work.wait(lk, [&] {
        if (stopping && pending.empty()) return true;
        return !pending.empty() && pool.take(reqs.at(pending.front()).ws_bytes, &off);
      });
      if (pending.empty()) return;  // stopping
      const uint64_t id = pending.front();
      pending.pop_front();
      Request& r = reqs.at(id);
      r.ws_off = off;
      ++inflight;
      bytes_inflight += r.ws_bytes;
      peak_inflight = std::max(peak_inflight, inflight);
      peak_bytes = std::max(peak_bytes, bytes_inflight);
      r.info.t_start_ms = now_ms();
      r.info.worker = w;
      const fa_op op = r.op;
      const int kind = r.kind;
      const void* b = r.b;
      void* x = r.x;
      const int m_max = r.m_max, ce = r.check_every;
      const double tol = r.tol;
      const uint32_t fl = r.flags;
      const size_t wsb = r.ws_bytes;
      lk.unlock();
      cv_work.notify_all();  // another idle worker may admit the next request
      fa_stats st;
      std::memset(&st, 0, sizeof(st));
      const int status =
          dev_ok ? fa_apply(op, kind, b, x, m_max, tol, ce, pool_base + off, wsb, fl, s, &st)
                 : FA_ERR_HIP;
      lk.lock();
      Request& rr = reqs.at(id);
      rr.info.status = status;
      rr.info.stats = st;
      rr.info.t_done_ms = now_ms();
      rr.done = true;
      pool.give(off, wsb);
      --inflight;
      bytes_inflight -= wsb;
      ++completed;
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int fa_server_create(fa_server* out, void* d_pool, size_t pool_bytes, int n_workers,
                     void* const* hip_streams) {
  if (!out || !d_pool || ((uintptr_t)d_pool & 255) || pool_bytes < 256 || n_workers < 1 ||
      n_workers > 64 || !hip_streams)
    return FA_ERR_ARG;
  fa_server_s* srv = new (std::nothrow) fa_server_s;
  if (!srv) return FA_ERR_ARG;
  if (hipGetDevice(&srv->device) != hipSuccess) {
    delete srv;
    return FA_ERR_HIP;
  }
  srv->pool_base = (char*)d_pool;
  srv->pool.init(pool_bytes & ~size_t(255));
  for (int w = 0; w < n_workers; ++w) srv->streams.push_back((hipStream_t)hip_streams[w]);
  try {
    for (int w = 0; w < n_workers; ++w) srv->workers.emplace_back([srv, w] { srv->worker(w); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> g(srv->mu);
      srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto& t : srv->workers) t.join();
    delete srv;
    return FA_ERR_ARG;
  }
  *out = srv;
  return FA_OK;
}

int fa_server_submit(fa_server srv, fa_op op, int kind, const void* d_b, void* d_x, int m_max,
                     double tol, int check_every, uint32_t flags, uint64_t* ticket) {
  if (!srv || !op || !d_b || !d_x || d_b == d_x || m_max < 1 || !ticket ||
      (kind != FA_INVSQRT && kind != FA_SQRT) || check_every < 0 || (flags & FA_PROFILE))
    return FA_ERR_ARG;
  const size_t wsb = fa_workspace_bytes(op, m_max, flags);
  if (wsb == 0) return FA_ERR_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->stopping) return FA_ERR_ARG;
  if (((wsb + 255) & ~size_t(255)) > srv->pool.size) return FA_ERR_WORKSPACE;  // can never fit
  const uint64_t id = srv->next_id++;
  Request r;
  r.op = op;
  r.kind = kind;
  r.b = d_b;
  r.x = d_x;
  r.m_max = m_max;
  r.tol = tol;
  r.check_every = check_every;
  r.flags = flags;
  r.ws_bytes = wsb;
  std::memset(&r.info, 0, sizeof(r.info));
  r.info.t_submit_ms = now_ms();
  r.info.ws_bytes = wsb;
  r.info.worker = -1;
  srv->reqs.emplace(id, r);
  srv->pending.push_back(id);
  *ticket = id;
  srv->cv_work.notify_one();
  return FA_OK;
}

int fa_server_poll(fa_server srv, uint64_t ticket, int* done) {
  if (!srv || !done) return FA_ERR_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FA_ERR_ARG;
  *done = it->second.done ? 1 : 0;
  return FA_OK;
}

int fa_server_wait(fa_server srv, uint64_t ticket, fa_request_info* info) {
  if (!srv) return FA_ERR_ARG;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FA_ERR_ARG;
  srv->cv_done.wait(lk, [&] {
    auto jt = srv->reqs.find(ticket);
    return jt == srv->reqs.end() || jt->second.done;
  });
  it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return FA_ERR_ARG;  // collected by another waiter
  Request& r = it->second;
  if (info) *info = r.info;
  const int st = r.info.status;
  srv->reqs.erase(ticket);
  return st;
}

int fa_server_status(fa_server srv, fa_server_info* info) {
  if (!srv || !info) return FA_ERR_ARG;
  std::lock_guard<std::mutex> g(srv->mu);
  info->pending = (int32_t)srv->pending.size();
  info->inflight = srv->inflight;
  info->peak_inflight = srv->peak_inflight;
  info->completed = srv->completed;
  info->pool_bytes = srv->pool.size;
  info->bytes_inflight = srv->bytes_inflight;
  info->peak_bytes_inflight = srv->peak_bytes;
  info->largest_free = srv->pool.largest();
  return FA_OK;
}

int fa_server_destroy(fa_server srv) {
  if (!srv) return FA_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();  // the queue drains first
  delete srv;
  return FA_OK;
}

}  // extern "C"
