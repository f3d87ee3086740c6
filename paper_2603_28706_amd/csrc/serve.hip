// Request server for independent slab solves: a queue with admission by slot
// and arena room, host worker threads each driving one HIP stream, first-fit
// sub-allocation of the caller's device arena.  Each request runs the
// Newton-Krylov solve of solve.hip (Sec. 6-6.2) on its own context.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ctx.h"

using namespace pns;

namespace {

constexpr int kMaxSlots = 16;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// first-fit allocator over [0, size) of the arena, blocks 256-byte aligned
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length

  void init(char* b, size_t n) {
    base = b;
    size = n / kAlign * kAlign;
    free_.clear();
    if (size) free_[0] = size;
  }
  char* take(size_t bytes) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      return base + off;
    }
    return nullptr;
  }
  void give(char* p, size_t bytes) {
    bytes = round_up(bytes);
    size_t off = (size_t)(p - base);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
};

struct Sizes {
  size_t ws = 0, solve = 0, nst = 0, nv = 0;
};

// host-side sizes of a request (a context is created on the host only)
int request_sizes(const pns_request* q, Sizes* out) {
  if (!q || !q->v_prev_host || !q->U_host) return PNS_EINVAL;
  pns_mesh m{};
  m.dim = 2;
  m.n_cells[0] = q->n_cells[0];
  m.n_cells[1] = q->n_cells[1];
  m.n_cells[2] = 1;
  m.lo[0] = q->lo[0];
  m.lo[1] = q->lo[1];
  m.hi[0] = q->hi[0];
  m.hi[1] = q->hi[1];
  m.hi[2] = 1.0;
  pns_discretization d{2, 1, 0.0, q->tau};
  pns_ctx* c = nullptr;
  int rc = pns_ctx_create(&m, &d, q->n_levels, q->precision, nullptr, &c);
  if (rc != PNS_OK) return rc;
  Model md;
  std::string err;
  rc = make_model(&q->model, &md, &err);
  if (rc == PNS_OK && !c->has_coarse) rc = PNS_EUNSUPPORTED;
  if (rc == PNS_OK && q->patch_kind != PNS_PATCH_SURROGATE && q->patch_kind != PNS_PATCH_EXACT)
    rc = PNS_EINVAL;
  if (rc == PNS_OK && q->vcycle_graph != 0 && q->vcycle_graph != 1) rc = PNS_EINVAL;
  if (rc == PNS_OK) {
    out->ws = pns_workspace_bytes(c);
    out->solve = pns_solve_workspace_bytes(c, q->params.restart);
    out->nst = (size_t)c->lev[0].g.nst;
    out->nv = (size_t)c->lev[0].g.nv;
    if (out->solve == 0) rc = PNS_EINVAL;
  }
  pns_ctx_destroy(c);
  return rc;
}

size_t footprint_of(const Sizes& z) {
  return round_up(z.ws) + round_up(z.solve) + round_up(z.nst * 8) + round_up(z.nv * 8);
}

struct Req {
  uint64_t ticket = 0;
  pns_request q{};
  std::vector<double> vprev;
  Sizes sz;
  size_t footprint = 0;
  char* mem = nullptr;
  pns_result res{};
};

}  // namespace

struct pns_server {
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, std::unique_ptr<Req>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
};

namespace {

// one request on one stream: context, workspace and vectors carved from mem
int run_request(Req* r, hipStream_t s, pns_solve_info* info) {
  const pns_request& q = r->q;
  pns_mesh m{};
  m.dim = 2;
  m.n_cells[0] = q.n_cells[0];
  m.n_cells[1] = q.n_cells[1];
  m.n_cells[2] = 1;
  m.lo[0] = q.lo[0];
  m.lo[1] = q.lo[1];
  m.hi[0] = q.hi[0];
  m.hi[1] = q.hi[1];
  m.hi[2] = 1.0;
  pns_discretization d{2, 1, 0.0, q.tau};
  pns_ctx* c = nullptr;
  int rc = pns_ctx_create(&m, &d, q.n_levels, q.precision, s, &c);
  if (rc != PNS_OK) return rc;
  char* p = r->mem;
  char* ws = p;
  p += round_up(r->sz.ws);
  char* work = p;
  p += round_up(r->sz.solve);
  double* U = (double*)p;
  p += round_up(r->sz.nst * 8);
  double* vp = (double*)p;
  const int64_t ns = c->lev[0].g.ns, nv = c->lev[0].g.nv;
  if ((rc = pns_bind_workspace(c, ws, r->sz.ws)) == PNS_OK &&
      (rc = pns_set_patch_kind(c, q.patch_kind)) == PNS_OK &&
      (rc = pns_set_vcycle_graph(c, q.vcycle_graph ? 1 : 0)) == PNS_OK) {
    // the host copy of the left trace is released once it is on the device
    bool ok = hipMemcpyAsync(vp, r->vprev.data(), nv * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipStreamSynchronize(s) == hipSuccess;
    std::vector<double>().swap(r->vprev);
    r->q.v_prev_host = nullptr;
    // first attempt from U = 0 (the first linearisation then has a uniform
    // viscosity); if it stops with PNS_ENOTCONV, a second attempt starts from
    // the left trace at both Radau nodes with zero pressure
    ok = ok && hipMemsetAsync(U, 0, r->sz.nst * 8, s) == hipSuccess;
    if (!ok) {
      rc = PNS_EHIP;
    } else {
      rc = pns_solve(c, &q.model, vp, U, &q.params, work, r->sz.solve, info);
      if (rc == PNS_ENOTCONV) {
        pns_solve_info first = *info;
        if (hipMemsetAsync(U, 0, r->sz.nst * 8, s) != hipSuccess ||
            hipMemcpyAsync(U, vp, nv * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(U + ns, vp, nv * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
          rc = PNS_EHIP;
        } else {
          rc = pns_solve(c, &q.model, vp, U, &q.params, work, r->sz.solve, info);
          info->newton_iterations += first.newton_iterations;
          info->krylov_iterations += first.krylov_iterations;
          info->smoother_setups += first.smoother_setups;
          info->backtracks += first.backtracks;
        }
      }
      if (rc == PNS_OK || rc == PNS_ENOTCONV || rc == PNS_ENONFINITE) {
        if (hipMemcpyAsync(q.U_host, U, r->sz.nst * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          rc = PNS_EHIP;
      }
    }
  }
  (void)hipStreamSynchronize(s);
  pns_ctx_destroy(c);
  return rc;
}

void worker_main(pns_server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t s = S->streams[slot];
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    Req* r = nullptr;
    // admission: the first queued request (arrival order) that fits the arena
    for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
      char* mem = S->arena.take((*it)->footprint);
      if (mem) {
        r = *it;
        r->mem = mem;
        S->queue.erase(it);
        break;
      }
    }
    if (!r) {
      if (S->stop && S->queue.empty()) return;
      S->cv_work.wait(lk);
      continue;
    }
    r->res.state = PNS_REQ_RUNNING;
    r->res.t_start = now_s();
    lk.unlock();
    // the request's result is written only under the lock (pns_poll reads it)
    pns_solve_info info{};
    const int rc = run_request(r, s, &info);
    lk.lock();
    r->res.info = info;
    S->arena.give(r->mem, r->footprint);
    r->mem = nullptr;
    r->res.status = rc;
    r->res.t_done = now_s();
    r->res.state = PNS_REQ_DONE;
    S->cv_done.notify_all();
    S->cv_work.notify_all();  // arena room may admit waiting requests
  }
}

}  // namespace

extern "C" {

size_t pns_request_footprint(const pns_request* req) {
  Sizes z;
  if (request_sizes(req, &z) != PNS_OK) return 0;
  return footprint_of(z);
}

int pns_server_create(int slots, void* arena, size_t bytes, pns_server** out) {
  if (!out) return PNS_EINVAL;
  *out = nullptr;
  if (slots < 1 || slots > kMaxSlots || !arena || ((uintptr_t)arena % kAlign) != 0 || bytes < kAlign)
    return PNS_EINVAL;
  pns_server* S = new pns_server();
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return PNS_EHIP;
  }
  S->arena.init((char*)arena, bytes);
  for (int i = 0; i < slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
      delete S;
      return PNS_EHIP;
    }
    S->streams.push_back(st);
  }
  for (int i = 0; i < slots; ++i) S->workers.emplace_back(worker_main, S, i);
  *out = S;
  return PNS_OK;
}

int pns_solve_request(pns_server* S, const pns_request* req, uint64_t* ticket) {
  if (!S || !req || !ticket) return PNS_EINVAL;
  auto r = std::make_unique<Req>();
  int rc = request_sizes(req, &r->sz);
  if (rc != PNS_OK) return rc;
  r->q = *req;
  r->vprev.assign(req->v_prev_host, req->v_prev_host + r->sz.nv);
  r->q.v_prev_host = r->vprev.data();
  r->footprint = footprint_of(r->sz);
  if (r->footprint > S->arena.size) return PNS_EWORKSPACE;
  std::lock_guard<std::mutex> lk(S->mu);
  r->ticket = S->next_ticket++;
  r->res.state = PNS_REQ_QUEUED;
  r->res.t_submit = now_s();
  r->res.footprint = r->footprint;
  *ticket = r->ticket;
  S->queue.push_back(r.get());
  S->all[r->ticket] = std::move(r);
  S->cv_work.notify_one();
  return PNS_OK;
}

int pns_poll(pns_server* S, uint64_t ticket, pns_result* out) {
  if (!S || !out) return PNS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PNS_EINVAL;
  *out = it->second->res;
  return PNS_OK;
}

int pns_wait(pns_server* S, uint64_t ticket, pns_result* out) {
  if (!S || !out) return PNS_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PNS_EINVAL;
  Req* r = it->second.get();
  S->cv_done.wait(lk, [r] { return r->res.state == PNS_REQ_DONE; });
  *out = r->res;
  return PNS_OK;
}

int pns_release(pns_server* S, uint64_t ticket) {
  if (!S) return PNS_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return PNS_EINVAL;
  if (it->second->res.state != PNS_REQ_DONE) return PNS_ESTATE;
  S->all.erase(it);
  return PNS_OK;
}

void pns_server_destroy(pns_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
