// Continuous-batching engine for steady-state solves, built on the public
// C ABI (m1_init, m1_step, m1_residual, m1_residuals, m1_batch_*).
//
// Device memory: one caller-owned arena.  The front of it holds the batch
// descriptor tables for max_resident grids; the rest is handed out first-fit
// in 256-byte units, one block of exactly m1_workspace_bytes per request.
//
// Schedule: a round admits queued requests that fit, advances every
// resident request by its share of steps (min(check_every, steps left)),
// then evaluates each resident's residual.  Requests whose share is a full
// check_every advance together through one batch; the others step alone.
// Because the per-request sequence of steps and residual checks is the one
// m1_solve_steady follows, and batched steps are bitwise equal to solo
// steps, every request's result is independent of what else is resident.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <deque>
#include <iterator>
#include <map>
#include <unordered_map>
#include <vector>

#include "m1_internal.h"
#include "m1lya.h"

namespace {

constexpr size_t kUnit = 256;
size_t round_unit(size_t x) { return (x + kUnit - 1) & ~(kUnit - 1); }

int err(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return m1::record_error(code, buf);
}

// First-fit allocator over byte offsets [0, size) with coalescing frees.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    size_ = size;
    used_ = 0;
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_unit(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_unit(bytes);
    size_t start = off, len = bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
    used_ -= bytes;
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t size_ = 0, used_ = 0;
};

struct Request {
  int64_t id = 0;
  m1_config cfg{};
  int64_t ncls = 0;
  double tol = 0;
  int64_t max_steps = 0;
  size_t ws = 0, off = 0;
  m1_handle* h = nullptr;
  int64_t steps = 0;
  double resid = INFINITY;
  int state = M1_REQ_QUEUED;
  int error = M1_OK;
  int64_t admit_round = -1, finish_round = -1;
  int bypassed = 0;
};

}  // namespace

struct m1_server {
  m1_server_config c{};
  char* arena = nullptr;
  size_t batch_ws = 0;          // bytes reserved at the arena front for batch tables
  hipStream_t stream = nullptr;
  m1_fields_cb cb = nullptr;
  void* user = nullptr;
  Arena blocks;                 // offsets relative to arena + batch_ws
  std::deque<Request*> queue;
  std::vector<Request*> resident;
  std::unordered_map<int64_t, Request*> all;
  std::vector<m1_request_info> unpolled;
  m1_batch* batch = nullptr;
  std::vector<m1_handle*> batch_members;
  int tile = 0;                 // tuned bins per block, 0 until known
  int64_t rounds = 0, next_id = 0, finished = 0;
};

namespace {

m1_request_info info_of(const Request* r) {
  m1_request_info i{};
  i.id = r->id;
  i.state = r->state;
  i.error = r->error;
  i.steps = r->steps;
  i.residual = r->resid;
  i.admit_round = r->admit_round;
  i.finish_round = r->finish_round;
  i.ws_bytes = r->ws;
  return i;
}

void finish(m1_server* s, Request* r, int state, int error) {
  r->state = state;
  r->error = error;
  r->finish_round = s->rounds;
  s->unpolled.push_back(info_of(r));
  ++s->finished;
}

void drop_batch(m1_server* s) {
  if (s->batch) {
    int bk = 0;
    if (m1_batch_info(s->batch, &bk, nullptr, 0) == M1_OK && bk > 0) s->tile = bk;
    m1_batch_free(s->batch);
  }
  s->batch = nullptr;
  s->batch_members.clear();
}

// Tries to admit r into a free block; returns false when no block fits.
bool try_admit(m1_server* s, Request* r) {
  size_t off = 0;
  if (!s->blocks.alloc(r->ws, &off)) return false;
  r->off = off;
  m1_fields f{};
  int st = s->cb ? s->cb(s->user, r->id, &f) : M1_EINVAL;
  if (st == M1_OK) {
    m1_config cfg = r->cfg;
    cfg.prec = s->c.prec;
    st = m1_init(&cfg, &f, s->arena + s->batch_ws + off, r->ws, (void*)s->stream, &r->h);
  }
  r->admit_round = s->rounds;
  if (st != M1_OK) {
    s->blocks.release(off, r->ws);
    r->h = nullptr;
    finish(s, r, M1_REQ_FAILED, st);
  } else {
    r->state = M1_REQ_RESIDENT;
    s->resident.push_back(r);
  }
  return true;
}

void admit(m1_server* s) {
  if (s->queue.empty()) return;
  Request* head = s->queue.front();
  bool head_blocked = false;
  std::deque<Request*> keep;
  while (!s->queue.empty()) {
    Request* r = s->queue.front();
    const bool full = (int)s->resident.size() >= s->c.max_resident;
    const bool head_waits = head_blocked && head->bypassed >= s->c.max_bypass;
    if (full || head_waits) break;
    s->queue.pop_front();
    if (try_admit(s, r)) {
      if (head_blocked && r != head) ++head->bypassed;
    } else {
      keep.push_back(r);
      if (r == head) head_blocked = true;
    }
  }
  // requests passed over keep their arrival order ahead of the rest
  while (!keep.empty()) {
    s->queue.push_front(keep.back());
    keep.pop_back();
  }
}

int advance(m1_server* s) {
  std::vector<Request*> together;
  std::vector<int32_t> share(s->resident.size());
  for (size_t q = 0; q < s->resident.size(); ++q) {
    Request* r = s->resident[q];
    share[q] = (int32_t)std::min<int64_t>(s->c.check_every, r->max_steps - r->steps);
    if (s->c.batched && share[q] == s->c.check_every) together.push_back(r);
  }
  if (!together.empty()) {
    std::vector<m1_handle*> hs;
    for (Request* r : together) hs.push_back(r->h);
    if (!s->batch || hs != s->batch_members) {
      drop_batch(s);
      size_t need = 0;
      int st = m1_batch_workspace_bytes(hs.data(), (int32_t)hs.size(), &need);
      if (st) return st;
      if (need > s->batch_ws) return err(M1_ENOMEM, "batch tables need %zu > %zu bytes", need, s->batch_ws);
      st = m1_batch_init(hs.data(), (int32_t)hs.size(), s->arena, s->batch_ws, s->c.use_graph, &s->batch);
      if (st) return st;
      if (s->tile > 0) {
        st = m1_batch_set_tile(s->batch, s->tile);
        if (st) return st;
      }
      s->batch_members = hs;
    }
    int st = m1_batch_step(s->batch, s->c.check_every);
    if (st) return st;
    for (Request* r : together) r->steps += s->c.check_every;
  }
  for (size_t q = 0; q < s->resident.size(); ++q) {
    Request* r = s->resident[q];
    if (s->c.batched && share[q] == s->c.check_every) continue;
    int st = m1_step(r->h, share[q], nullptr);
    if (st) return st;
    r->steps += share[q];
  }
  return M1_OK;
}

void check_residuals(m1_server* s) {
  std::vector<Request*> still;
  // every resident's residual with one wait; on an error, one by one, so
  // that the request that failed is the one marked
  std::vector<m1_handle*> hs;
  for (Request* r : s->resident) hs.push_back(r->h);
  std::vector<double> all(hs.size(), INFINITY);
  const bool together = !hs.empty() && m1_residuals(hs.data(), (int32_t)hs.size(), all.data()) == M1_OK;
  size_t q = 0;
  for (Request* r : s->resident) {
    double res = all[q++];
    int st = together ? M1_OK : m1_residual(r->h, &res);
    r->resid = res;
    if (st != M1_OK) finish(s, r, M1_REQ_FAILED, st);
    else if (res < r->tol) finish(s, r, M1_REQ_CONVERGED, M1_OK);
    else if (r->steps >= r->max_steps) finish(s, r, M1_REQ_NOT_CONVERGED, M1_ENOTCONV);
    else still.push_back(r);
  }
  if (still.size() != s->resident.size()) s->resident.swap(still);
}

}  // namespace

extern "C" {

int32_t m1_server_create(const m1_server_config* c, void* d_arena, size_t arena_bytes, void* stream,
                         m1_fields_cb cb, void* user, m1_server** out) {
  if (!c || !out || !cb) return err(M1_EINVAL, "config, callback and out must be given");
  *out = nullptr;
  if (c->prec != M1_FP32 && c->prec != M1_FP64) return err(M1_EINVAL, "bad precision");
  if (c->max_resident < 1 || c->check_every < 1 || c->max_bypass < 0)
    return err(M1_EINVAL, "need max_resident >= 1, check_every >= 1, max_bypass >= 0");
  if (!d_arena || ((uintptr_t)d_arena & (kUnit - 1))) return err(M1_EINVAL, "arena NULL or not 256-byte aligned");
  size_t bw = 0;
  int st = m1_batch_workspace_bound(c->max_resident, c->prec, &bw);
  if (st) return st;
  bw = round_unit(bw);
  if (arena_bytes <= bw) return err(M1_ENOMEM, "arena of %zu bytes holds no request", arena_bytes);
  m1_server* s = new m1_server();
  s->c = *c;
  s->arena = (char*)d_arena;
  s->batch_ws = bw;
  s->stream = (hipStream_t)stream;
  s->cb = cb;
  s->user = user;
  s->blocks.reset((arena_bytes - bw) & ~(kUnit - 1));
  *out = s;
  return M1_OK;
}

int32_t m1_server_submit(m1_server* s, const m1_config* cfg, int64_t n_temp_classes, double rel_tol,
                         int64_t max_steps, int64_t* id) {
  if (!s || !cfg || !id) return err(M1_EINVAL, "bad arguments");
  if (!(rel_tol > 0) || max_steps < 1) return err(M1_EINVAL, "need rel_tol > 0 and max_steps >= 1");
  m1_config c = *cfg;
  c.prec = s->c.prec;
  if (s->c.batched && c.substep_rule)
    return err(M1_EUNSUPPORTED, "the substep rule needs single-grid stepping (batched server)");
  if (s->c.batched && c.flux != M1_FLUX_GLF)
    return err(M1_EUNSUPPORTED, "the eigenvalue HLL flux needs single-grid stepping (batched server)");
  size_t ws = 0;
  int st = m1_workspace_bytes(&c, n_temp_classes, &ws);
  if (st) return st;
  Request* r = new Request();
  r->id = s->next_id++;
  r->cfg = c;
  r->ncls = n_temp_classes;
  r->tol = rel_tol;
  r->max_steps = max_steps;
  r->ws = ws;
  s->all[r->id] = r;
  *id = r->id;
  if (round_unit(ws) > s->blocks.size()) finish(s, r, M1_REQ_REJECTED, M1_ENOMEM);
  else s->queue.push_back(r);
  return M1_OK;
}

int32_t m1_server_run(m1_server* s, int32_t rounds, int32_t* n_busy) {
  if (!s || rounds < 0) return err(M1_EINVAL, "bad arguments");
  int st = M1_OK;
  for (int k = 0; k < rounds; ++k) {
    admit(s);
    if (s->resident.empty()) break;
    st = advance(s);
    if (st) break;
    check_residuals(s);
    ++s->rounds;
  }
  if (n_busy) *n_busy = (int32_t)(s->queue.size() + s->resident.size());
  return st;
}

int32_t m1_server_poll(m1_server* s, m1_request_info* out, int32_t cap, int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !out)) return err(M1_EINVAL, "bad arguments");
  const int32_t k = (int32_t)std::min<size_t>((size_t)cap, s->unpolled.size());
  std::copy(s->unpolled.begin(), s->unpolled.begin() + k, out);
  s->unpolled.erase(s->unpolled.begin(), s->unpolled.begin() + k);
  *n = k;
  return M1_OK;
}

int32_t m1_server_handle(m1_server* s, int64_t id, m1_handle** h) {
  if (!s || !h) return err(M1_EINVAL, "bad arguments");
  auto it = s->all.find(id);
  if (it == s->all.end() || !it->second->h) return err(M1_EINVAL, "request %lld holds no handle", (long long)id);
  *h = it->second->h;
  return M1_OK;
}

int32_t m1_server_release(m1_server* s, int64_t id) {
  if (!s) return err(M1_EINVAL, "server is NULL");
  auto it = s->all.find(id);
  if (it == s->all.end()) return err(M1_EINVAL, "unknown request %lld", (long long)id);
  Request* r = it->second;
  if (r->state == M1_REQ_QUEUED || r->state == M1_REQ_RESIDENT)
    return err(M1_ESTATE, "request %lld has not finished", (long long)id);
  if (r->h) {
    for (m1_handle* m : s->batch_members)
      if (m == r->h) drop_batch(s);
    (void)hipStreamSynchronize(s->stream);
    m1_free(r->h);
    s->blocks.release(r->off, r->ws);
  }
  s->all.erase(it);
  delete r;
  return M1_OK;
}

int32_t m1_server_stats(const m1_server* s, int64_t* queued, int64_t* resident, int64_t* finished,
                        int64_t* rounds, size_t* arena_used, size_t* largest_free) {
  if (!s) return err(M1_EINVAL, "server is NULL");
  int64_t held = 0;
  for (auto& kv : s->all)
    if (kv.second->state >= M1_REQ_CONVERGED) ++held;
  if (queued) *queued = (int64_t)s->queue.size();
  if (resident) *resident = (int64_t)s->resident.size();
  if (finished) *finished = held;
  if (rounds) *rounds = s->rounds;
  if (arena_used) *arena_used = s->blocks.used() + s->batch_ws;
  if (largest_free) *largest_free = s->blocks.largest();
  return M1_OK;
}

int32_t m1_server_free(m1_server* s) {
  if (!s) return M1_OK;
  drop_batch(s);
  bool any = false;                        // nothing was enqueued without a handle
  for (auto& kv : s->all) any = any || kv.second->h;
  if (any) (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->all) {
    if (kv.second->h) m1_free(kv.second->h);
    delete kv.second;
  }
  delete s;
  return M1_OK;
}

}  // extern "C"
