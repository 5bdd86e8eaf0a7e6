// Request loop for many concurrent ADMM solves: sessions with device-resident
// warm-start blocks (paper §6: each PSD variable is projected once per ADMM
// iteration from its previous Ritz block), admission by device-memory
// footprint, and continuous batching.
//
// Execution resources:
//   slots        worker threads, each with its own library handle and HIP
//                stream, running the single-cone path (psdp_project) for
//                one request at a time; requests on different slots overlap
//                on the GPU.
//   batch lane   one worker that, whenever it is free, takes every waiting
//                small request (order <= small_n, positive side, block <= 32)
//                and projects them in one persistent batched launch; those
//                that arrive meanwhile join the next launch.
// A session never has two requests in flight (its warm start is the
// previous result); requests of different sessions are admitted in
// submission order as resources free up, skipping over sessions that are
// busy.  Admission keeps the sum of the workspace estimates of all running
// work within hbm_budget; idle workers give their workspace back when a
// request needs the room.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/psdp.h"
#include "batched.h"
#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;
using psdp::kBatchMaxM;
using psdp::kBatchMaxN;
constexpr int kSlotMaxM = 48;
constexpr int kLaneMaxIter = 60;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Session {
  int id = 0, n = 0, m_cap = 0;
  int pos_hint = -1;
  int m = 0;            // warm-start columns in V
  int block_side = 0;   // side of the block in V (PSDP_SIDE_POS / _NEG), 0 = none
  double* V = nullptr;  // n x m_cap, leading dim n
  double* lam = nullptr;
  bool busy = false;
  long long seq = 0;
  int inflight = 0;     // submitted, not completed
  bool closing = false;
  // adaptive path: after a block solve had to fall back to the exact path,
  // the next `full_left` requests go straight to it (back-off doubles, 16 max)
  int full_left = 0, backoff = 0;
};

struct Request {
  long long ticket = 0;
  Session* s = nullptr;
  const double* X = nullptr;
  double* Pi = nullptr;
  hipEvent_t ready = nullptr;
  Clock::time_point t_submit, t_start, t_done;
  int side = 0;
  size_t need = 0;
  int lane = 0, batch_size = 1;
  long long seq = 0;
  bool done = false;
  bool force_full = false;  // lane result not converged: exact path next
  psdp_info info{};
};

struct Worker {
  int k = 0;
  psdp_handle h = nullptr;
  hipStream_t stream = nullptr;
  size_t held = 0;     // workspace estimate the handle keeps
  bool busy = false;
  bool is_lane = false;
  std::thread th;
};

size_t ws_estimate(int n, int m_cap, int prec, int side) {
  size_t b = 0;
  if (psdp_workspace_bytes(n, std::max(1, std::min(m_cap, kSlotMaxM)), prec, &b) != PSDP_OK)
    b = 0;
  if (side == PSDP_SIDE_FULL) {
    const size_t L = (size_t)((n + 63) / 64 * 64);
    b += 24 * L * L;  // eigenvector matrix + solver workspace
  }
  return b;
}

}  // namespace

struct psdp_server_s {
  int device = 0;
  psdp_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv;      // work available / resources freed
  std::condition_variable cv_done; // a request completed
  bool stopping = false;
  std::vector<Worker*> workers;    // slots, then the lane (if any)
  std::map<int, Session*> sessions;
  int next_session = 1;
  std::list<Request*> pending;
  std::map<long long, Request*> tickets;
  long long next_ticket = 1;
  std::vector<hipEvent_t> event_pool;
  // statistics
  long long submitted = 0, completed = 0, rejected = 0;
  long long batched_launches = 0, batched_requests = 0, lane_fallbacks = 0;
  std::vector<double> lat;
  bool have_first = false;
  Clock::time_point t_first, t_last;
  size_t held_peak = 0;
  int active = 0, max_active = 0;

  size_t held_total() const {
    size_t t = 0;
    for (auto* w : workers) t += w->held;
    return t;
  }
  bool lane_enabled() const { return cfg.batch_lane && workers.size() > (size_t)cfg.slots; }

  // side and block for the next request of s (same rule as psdp_project,
  // plus the session's back-off after failed block solves)
  int resolve_side(const Session& s) const {
    int side = cfg.opt.side;
    if (side == PSDP_SIDE_AUTO) {
      if (s.full_left > 0) return PSDP_SIDE_FULL;
      side = psdp::auto_side(s.n, s.pos_hint, s.m_cap, cfg.opt);
    }
    return side;
  }
  static size_t lane_extra(const Session& s) {
    return 8 * ((size_t)s.n * s.n + (size_t)s.n * s.m_cap + s.m_cap);  // tuning outputs
  }
  static size_t lane_full_bytes(const Session& s) {
    const size_t nb = (size_t)((s.n + 31) / 32 * 32);
    return 24 * nb * nb + 64 * nb;  // padded matrix + solver workspace estimate
  }
  // small requests: the block solver on the positive side, or the exact path
  bool lane_eligible(const Session& s, int side) const {
    if (!lane_enabled() || s.n > cfg.small_n) return false;
    if (side == PSDP_SIDE_FULL) return lane_full_bytes(s) <= cfg.hbm_budget;
    if (side != PSDP_SIDE_POS || s.pos_hint < 0) return false;
    const int mm = std::min(s.m_cap, kBatchMaxM);
    if (psdp::block_need(s.pos_hint, cfg.opt) > mm) return false;
    // a batch of this request alone must fit the budget
    return psdp::batched_scratch_bytes(s.n, mm) + lane_extra(s) <= cfg.hbm_budget;
  }

  // Make room for `need` more bytes on worker w (lock held): the worker's
  // own holding is replaced; idle workers release theirs if necessary.
  bool reserve(Worker* w, size_t need) {
    const size_t budget = cfg.hbm_budget;
    auto total_with = [&]() { return held_total() - w->held + std::max(w->held, need); };
    if (total_with() <= budget) {
      w->held = std::max(w->held, need);
      held_peak = std::max(held_peak, held_total());
      return true;
    }
    for (auto* o : workers) {
      if (o == w || o->busy || o->held == 0) continue;
      if (o->h) {
        (void)psdp_destroy(o->h);  // frees its workspace; recreated on use
        o->h = nullptr;
      }
      o->held = 0;
      if (total_with() <= budget) break;
    }
    if (total_with() > budget) return false;
    w->held = std::max(w->held, need);
    held_peak = std::max(held_peak, held_total());
    return true;
  }

  // next request for a slot worker (lock held), or nullptr
  Request* pick_slot(Worker* w) {
    std::vector<int> blocked;
    auto is_blocked = [&](int id) { return std::find(blocked.begin(), blocked.end(), id) != blocked.end(); };
    for (auto it = pending.begin(); it != pending.end(); ++it) {
      Request* r = *it;
      Session& s = *r->s;
      if (s.busy || is_blocked(s.id)) continue;
      const int side = r->force_full ? (int)PSDP_SIDE_FULL : resolve_side(s);
      if (lane_eligible(s, side)) { blocked.push_back(s.id); continue; }
      const size_t need = ws_estimate(s.n, s.m_cap, cfg.opt.prec, side);
      if (!reserve(w, need)) { blocked.push_back(s.id); continue; }
      if (side == PSDP_SIDE_FULL && s.full_left > 0 && !r->force_full) s.full_left -= 1;
      r->side = side;
      r->need = need;
      s.busy = true;
      pending.erase(it);
      return r;
    }
    return nullptr;
  }

  // every waiting lane-eligible request (lock held)
  std::vector<Request*> pick_batch(Worker* w) {
    std::vector<Request*> out;
    std::vector<int> blocked;
    auto is_blocked = [&](int id) { return std::find(blocked.begin(), blocked.end(), id) != blocked.end(); };
    int nmax = 1, mmax = 1;
    size_t extra = 0, full = 0;
    bool any_lob = false;
    for (auto it = pending.begin(); it != pending.end() && (int)out.size() < cfg.max_batch;) {
      Request* r = *it;
      Session& s = *r->s;
      if (s.busy || is_blocked(s.id)) { ++it; continue; }
      const int side = r->force_full ? (int)PSDP_SIDE_FULL : resolve_side(s);
      if (!lane_eligible(s, side)) { blocked.push_back(s.id); ++it; continue; }
      size_t need;
      int nm = nmax, mm = mmax;
      if (side == PSDP_SIDE_FULL) {
        need = (any_lob ? psdp::batched_scratch_bytes(nmax, mmax) * std::min<size_t>(out.size(), 512) : 0) +
               extra + full + lane_full_bytes(s);
      } else {
        nm = std::max(nmax, s.n);
        mm = std::max(mmax, std::min(s.m_cap, kBatchMaxM));
        need = psdp::batched_scratch_bytes(nm, mm) * std::min<size_t>(out.size() + 1, 512) + extra +
               lane_extra(s) + full;
      }
      if (!reserve(w, need)) { blocked.push_back(s.id); ++it; continue; }
      if (side == PSDP_SIDE_FULL) {
        full += lane_full_bytes(s);
        if (s.full_left > 0 && !r->force_full) s.full_left -= 1;
      } else {
        nmax = nm;
        mmax = mm;
        extra += lane_extra(s);
        any_lob = true;
      }
      r->side = side;
      r->need = need;
      s.busy = true;
      out.push_back(r);
      it = pending.erase(it);
    }
    return out;
  }

  void finish(Request* r, const Clock::time_point& t_done) {
    // lock held
    Session& s = *r->s;
    r->t_done = t_done;
    r->done = true;
    const psdp_info& f = r->info;
    if (f.status == PSDP_FELL_BACK_FULL_EIG && r->side != PSDP_SIDE_FULL) {
      // the block solver did not converge: exact path for a while
      s.backoff = s.backoff ? std::min(2 * s.backoff, 16) : 2;
      s.full_left = s.backoff;
    } else if (f.status == PSDP_OK && r->side != PSDP_SIDE_FULL) {
      s.backoff = 0;
    }
    if (f.status >= 0) {
      if (f.side_used == PSDP_SIDE_FULL) {
        s.pos_hint = f.n_pos_full;
        s.m = f.m_out;  // positive eigenpairs: a positive-side warm start
        s.block_side = PSDP_SIDE_POS;
      } else {
        s.m = f.m_out;
        s.block_side = f.side_used;
        s.pos_hint = (f.side_used == PSDP_SIDE_POS) ? f.n_pos : s.n - f.n_pos;
      }
    }
    s.busy = false;
    s.inflight -= 1;
    completed += 1;
    lat.push_back(ms_between(r->t_submit, t_done));
    t_last = t_done;
    active -= 1;
    if (r->ready) event_pool.push_back(r->ready);
    r->ready = nullptr;
  }

  psdp_options request_opt(const Request* r) const {
    psdp_options o = cfg.opt;
    o.side = r->side;
    o.pos_hint = r->s->pos_hint;
    o.fallback_full = 1;
    // random columns depend on the session and its request count only
    o.seed = cfg.opt.seed ^ (0x9E3779B97F4A7C15ull * (unsigned long long)(r->s->id + 1)) ^
             ((unsigned long long)r->seq << 20);
    return o;
  }

  bool ensure_handle(Worker* w) {
    if (w->h) return true;
    return psdp_create(&w->h, device, (void*)w->stream) == PSDP_OK;
  }

  void run_slot(Worker* w, Request* r) {
    Session& s = *r->s;
    r->info = psdp_info{};
    r->lane = 0;
    r->batch_size = 1;
    if (!ensure_handle(w)) { r->info.status = PSDP_ERR_HIP; return; }
    if (r->ready) (void)hipStreamWaitEvent(w->stream, r->ready, 0);
    psdp_options o = request_opt(r);
    int m = (r->side != PSDP_SIDE_FULL && s.block_side == r->side) ? std::min(s.m, s.m_cap) : 0;
    psdp_status rc = psdp_project(w->h, s.n, r->X, s.n, s.V, s.n, s.m_cap, &m, s.lam, r->Pi, s.n,
                                  &o, &r->info);
    r->info.status = rc;
    if (rc >= 0) r->info.m_out = m;
  }

  void run_batch(Worker* w, std::vector<Request*>& rs) {
    if (!ensure_handle(w)) {
      for (auto* r : rs) { r->info = psdp_info{}; r->info.status = PSDP_ERR_HIP; }
      return;
    }
    for (auto* r : rs)
      if (r->ready) (void)hipStreamWaitEvent(w->stream, r->ready, 0);
    std::vector<Request*> lob, full;
    for (auto* r : rs) (r->side == PSDP_SIDE_FULL ? full : lob).push_back(r);
    auto run = [&](std::vector<Request*>& grp, bool exact) {
      const int c = (int)grp.size();
      if (c == 0) return;
      std::vector<int> n(c), mcap(c), mio(c);
      std::vector<const double*> X(c);
      std::vector<double*> V(c), L(c), P(c);
      std::vector<psdp_info> info(c);
      for (int i = 0; i < c; ++i) {
        Session& s = *grp[i]->s;
        n[i] = s.n;
        X[i] = grp[i]->X;
        V[i] = s.V;
        L[i] = s.lam;
        P[i] = grp[i]->Pi;
        if (exact) {
          mcap[i] = s.m_cap;
          mio[i] = 0;
        } else {
          mcap[i] = std::min(s.m_cap, kBatchMaxM);
          mio[i] = (s.block_side == PSDP_SIDE_POS) ? std::min(s.m, mcap[i]) : 0;
          // a cold start uses m_cap columns: size the block from the hint
          if (mio[i] == 0) mcap[i] = std::min(mcap[i], std::max(1, psdp::block_need(s.pos_hint, cfg.opt)));
        }
      }
      psdp_status rc;
      if (exact) {
        rc = psdp_full_eig_project_batched(w->h, c, n.data(), X.data(), V.data(), mcap.data(),
                                           mio.data(), L.data(), P.data(), info.data());
      } else {
        psdp_options o = cfg.opt;
        o.side = PSDP_SIDE_POS;
        o.fallback_full = 1;
        o.seed = cfg.opt.seed ^ 0x5851F42D4C957F2Dull;
        // a launch lasts as long as its slowest cone: cones that have not
        // converged within kLaneMaxIter iterations take the exact path, and
        // the launch shape is fixed (batches change composition every time,
        // so tuning each one would cost more than it saves)
        o.max_iter = std::min(o.max_iter, kLaneMaxIter);
        if (o.batch_variant < 0) o.batch_variant = 0;
        rc = psdp_project_batched(w->h, c, n.data(), X.data(), V.data(), mcap.data(), mio.data(),
                                  L.data(), P.data(), &o, info.data());
      }
      for (int i = 0; i < c; ++i) {
        Request* r = grp[i];
        r->lane = 1;
        r->batch_size = (int)rs.size();
        if (rc == PSDP_ERR_INVALID_ARG || rc == PSDP_ERR_HIP || rc == PSDP_ERR_OUT_OF_MEMORY) {
          r->info = psdp_info{};
          r->info.status = rc;
        } else {
          r->info = info[i];
          if (r->info.status >= 0) r->info.m_out = mio[i];
        }
      }
    };
    run(lob, false);
    run(full, true);
  }

  void worker_main(Worker* w) {
    (void)hipSetDevice(device);
    for (;;) {
      Request* one = nullptr;
      std::vector<Request*> many;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          if (w->is_lane) many = pick_batch(w);
          else one = pick_slot(w);
          if (one || !many.empty()) break;
          if (stopping && pending.empty()) return;
          cv.wait(lk);
        }
        w->busy = true;
        const auto now = Clock::now();
        const int got = one ? 1 : (int)many.size();
        active += got;
        max_active = std::max(max_active, active);
        if (one) one->t_start = now;
        for (auto* r : many) r->t_start = now;
        if (!many.empty()) {
          batched_launches += 1;
          batched_requests += (long long)many.size();
        }
      }
      if (one) run_slot(w, one);
      else run_batch(w, many);
      {
        std::lock_guard<std::mutex> lk(mu);
        const auto now = Clock::now();
        if (one) finish(one, now);
        // a lane result that did not converge goes back to the front of the
        // queue for the exact path on a worker (the batched engine has no
        // full-eig fallback); its session stays in order
        for (auto it = many.rbegin(); it != many.rend(); ++it) {
          Request* r = *it;
          if (r->info.status == PSDP_NOT_CONVERGED) {
            r->force_full = true;
            r->s->busy = false;
            active -= 1;
            lane_fallbacks += 1;
            pending.push_front(r);
          } else {
            finish(r, now);
          }
        }
        w->busy = false;
      }
      cv.notify_all();
      cv_done.notify_all();
    }
  }
};

extern "C" {

void psdp_server_default_config(psdp_server_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->slots = 4;
  c->hbm_budget = 0;
  c->batch_lane = 1;
  c->small_n = kBatchMaxN;
  c->max_batch = 512;
  psdp_default_options(&c->opt);
}

psdp_status psdp_server_create(psdp_server* out, int device, const psdp_server_config* cfg_in) {
  if (!out) return PSDP_ERR_INVALID_ARG;
  *out = nullptr;
  psdp_server_config cfg;
  if (cfg_in) cfg = *cfg_in; else psdp_server_default_config(&cfg);
  if (cfg.slots < 1 || cfg.slots > 16 || cfg.max_batch < 1 || cfg.small_n < 1 ||
      cfg.small_n > kBatchMaxN || cfg.opt.prec < 0 || cfg.opt.prec > 2 || cfg.opt.side < 0 ||
      cfg.opt.side > 3 || cfg.opt.max_iter < 1)
    return PSDP_ERR_INVALID_ARG;
  if (cfg.hbm_budget == 0) cfg.hbm_budget = (size_t)16 << 30;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return PSDP_ERR_HIP;
  if (device < 0 || device >= count) return PSDP_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return PSDP_ERR_HIP;
  psdp_server S = new psdp_server_s();
  S->device = device;
  S->cfg = cfg;
  const int nw = cfg.slots + (cfg.batch_lane ? 1 : 0);
  for (int k = 0; k < nw; ++k) {
    Worker* w = new Worker();
    w->k = k;
    w->is_lane = (k >= cfg.slots);
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      for (auto* o : S->workers) { (void)hipStreamDestroy(o->stream); delete o; }
      delete S;
      return PSDP_ERR_HIP;
    }
    S->workers.push_back(w);
  }
  for (auto* w : S->workers) w->th = std::thread([S, w]() { S->worker_main(w); });
  *out = S;
  return PSDP_OK;
}

psdp_status psdp_server_drain(psdp_server S) {
  if (!S) return PSDP_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&]() { return S->completed >= S->submitted; });
  return PSDP_OK;
}

psdp_status psdp_server_destroy(psdp_server S) {
  if (!S) return PSDP_ERR_INVALID_ARG;
  (void)psdp_server_drain(S);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv.notify_all();
  for (auto* w : S->workers) if (w->th.joinable()) w->th.join();
  (void)hipSetDevice(S->device);
  for (auto* w : S->workers) {
    if (w->h) (void)psdp_destroy(w->h);
    if (w->stream) (void)hipStreamDestroy(w->stream);
    delete w;
  }
  for (auto& kv : S->sessions) {
    if (kv.second->V) (void)hipFree(kv.second->V);
    if (kv.second->lam) (void)hipFree(kv.second->lam);
    delete kv.second;
  }
  for (auto& kv : S->tickets) {
    if (kv.second->ready) S->event_pool.push_back(kv.second->ready);
    delete kv.second;
  }
  for (auto e : S->event_pool) (void)hipEventDestroy(e);
  delete S;
  return PSDP_OK;
}

psdp_status psdp_server_open_session(psdp_server S, int n, int m_cap, int pos_hint, int* id) {
  if (!S || !id || n < 1 || m_cap < 1 || m_cap > kSlotMaxM || pos_hint < -1 || pos_hint > n)
    return PSDP_ERR_INVALID_ARG;
  Session* s = new Session();
  s->n = n;
  s->m_cap = std::min(m_cap, n);
  s->pos_hint = pos_hint;
  if (hipSetDevice(S->device) != hipSuccess) { delete s; return PSDP_ERR_HIP; }
  if (hipMalloc(&s->V, sizeof(double) * (size_t)n * s->m_cap) != hipSuccess ||
      hipMalloc(&s->lam, sizeof(double) * (size_t)s->m_cap) != hipSuccess) {
    if (s->V) (void)hipFree(s->V);
    delete s;
    return PSDP_ERR_OUT_OF_MEMORY;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  s->id = S->next_session++;
  S->sessions[s->id] = s;
  *id = s->id;
  return PSDP_OK;
}

psdp_status psdp_server_close_session(psdp_server S, int id) {
  if (!S) return PSDP_ERR_INVALID_ARG;
  Session* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(id);
    if (it == S->sessions.end()) return PSDP_ERR_INVALID_ARG;
    if (it->second->inflight > 0) return PSDP_PENDING;
    s = it->second;
    S->sessions.erase(it);
  }
  (void)hipSetDevice(S->device);
  (void)hipFree(s->V);
  (void)hipFree(s->lam);
  delete s;
  return PSDP_OK;
}

psdp_status psdp_server_submit(psdp_server S, int id, const double* X, double* Pi,
                               void* producer_stream, long long* ticket) {
  if (!S || !X || !Pi || !ticket || (const void*)X == (const void*)Pi) return PSDP_ERR_INVALID_ARG;
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->event_pool.empty()) { ev = S->event_pool.back(); S->event_pool.pop_back(); }
  }
  (void)hipSetDevice(S->device);
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return PSDP_ERR_HIP;
  if (hipEventRecord(ev, (hipStream_t)producer_stream) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return PSDP_ERR_HIP;
  }
  Request* r = new Request();
  r->X = X;
  r->Pi = Pi;
  r->ready = ev;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(id);
    if (it == S->sessions.end() || it->second->closing) {
      S->event_pool.push_back(ev);
      delete r;
      return PSDP_ERR_INVALID_ARG;
    }
    Session* s = it->second;
    // a request larger than the whole budget can never be admitted
    const size_t worst = std::max(ws_estimate(s->n, s->m_cap, S->cfg.opt.prec, PSDP_SIDE_FULL),
                                  ws_estimate(s->n, s->m_cap, S->cfg.opt.prec, PSDP_SIDE_POS));
    if (worst > S->cfg.hbm_budget) {
      S->event_pool.push_back(ev);
      delete r;
      S->rejected += 1;
      return PSDP_ERR_CAPACITY;
    }
    r->s = s;
    r->ticket = S->next_ticket++;
    r->seq = s->seq++;
    r->t_submit = Clock::now();
    if (!S->have_first) { S->have_first = true; S->t_first = r->t_submit; }
    s->inflight += 1;
    S->submitted += 1;
    S->pending.push_back(r);
    S->tickets[r->ticket] = r;
    *ticket = r->ticket;
  }
  S->cv.notify_all();
  return PSDP_OK;
}

psdp_status psdp_server_wait(psdp_server S, long long ticket, double timeout_ms, psdp_result* out) {
  if (!S) return PSDP_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return PSDP_ERR_INVALID_ARG;
  Request* r = it->second;
  auto done = [&]() { return r->done; };
  if (timeout_ms < 0) S->cv_done.wait(lk, done);
  else if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done))
    return PSDP_PENDING;
  if (out) {
    out->info = r->info;
    out->ticket = r->ticket;
    out->session = r->s->id;
    out->lane = r->lane;
    out->batch_size = r->batch_size;
    out->queue_ms = ms_between(r->t_submit, r->t_start);
    out->latency_ms = ms_between(r->t_submit, r->t_done);
  }
  S->tickets.erase(it);
  delete r;
  return PSDP_OK;
}

psdp_status psdp_server_session_block(psdp_server S, int id, double* V, int ldv, double* lambda,
                                      int* m) {
  if (!S || !m) return PSDP_ERR_INVALID_ARG;
  Session* s = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(id);
    if (it == S->sessions.end()) return PSDP_ERR_INVALID_ARG;
    s = it->second;
    if (s->busy) return PSDP_PENDING;
    *m = s->m;
  }
  if (!V && !lambda) return PSDP_OK;
  if (V && ldv < s->n) return PSDP_ERR_INVALID_ARG;
  (void)hipSetDevice(S->device);
  if (V && s->m > 0 &&
      hipMemcpy2D(V, sizeof(double) * ldv, s->V, sizeof(double) * s->n, sizeof(double) * s->n, s->m,
                  hipMemcpyDeviceToDevice) != hipSuccess)
    return PSDP_ERR_HIP;
  if (lambda && s->m > 0 &&
      hipMemcpy(lambda, s->lam, sizeof(double) * s->m, hipMemcpyDeviceToDevice) != hipSuccess)
    return PSDP_ERR_HIP;
  return PSDP_OK;
}

psdp_status psdp_server_stats_get(psdp_server S, psdp_server_stats* st) {
  if (!S || !st) return PSDP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(st, 0, sizeof(*st));
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->rejected = S->rejected;
  if (!S->lat.empty()) {
    std::vector<double> v = S->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) {
      const double pos = q * (v.size() - 1);
      const size_t i = (size_t)pos;
      const double f = pos - i;
      return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
    };
    st->p50_ms = pct(0.50);
    st->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_ms = sum / v.size();
    st->max_ms = v.back();
    const double span = ms_between(S->t_first, S->t_last);
    st->throughput = span > 0 ? 1e3 * S->completed / span : 0.0;
  }
  st->hbm_held = S->held_total();
  st->hbm_peak = S->held_peak;
  st->active = S->active;
  st->queued = (int)S->pending.size();
  st->max_active = S->max_active;
  st->batched_launches = S->batched_launches;
  st->batched_requests = S->batched_requests;
  st->lane_fallbacks = S->lane_fallbacks;
  return PSDP_OK;
}

psdp_status psdp_server_stats_reset(psdp_server S) {
  if (!S) return PSDP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  S->submitted -= S->completed;
  S->completed = 0;
  S->rejected = 0;
  S->lat.clear();
  S->have_first = false;
  S->batched_launches = 0;
  S->batched_requests = 0;
  S->lane_fallbacks = 0;
  S->held_peak = S->held_total();
  S->max_active = S->active;
  return PSDP_OK;
}

}  // extern "C"
