// Request loop with continuous batching.
//
// Submitted games (or FAMGpi hierarchies) wait in a FIFO queue.  A scheduling
// step admits queued requests while their estimated device footprint fits the
// HBM budget, then advances every active request by one policy-iteration step
// in one lock-step engine (one merged launch per kernel for all of them).
// Requests leave as they converge and free their budget; an FAMGpi request
// that finishes a grid moves to the next finer grid in place (its state is
// transferred by I and U) without leaving the batch.  Requests that arrive
// while others run join at the next step boundary.
#include "internal.hpp"

#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>

namespace shp {

static double wall_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  Game* handle = nullptr;   // plain game or hierarchy
  shapley_solve_opts opts{};
  std::vector<int32_t> alpha0, beta0;
  std::vector<double> v0;
  size_t footprint = 0;
  int level = 0;            // current FAMGpi grid (index into levels)
  bool famg = false;
  bool done = false;
  int status = SHAPLEY_OK;
  SlotState slot;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int outer = 0, inner = 0, cycles = 0;
  double setup_s = 0, cycle_s = 0, improve_s = 0;
  shapley_stats stats{};

  Game* current() { return famg ? handle->levels[level] : handle->finest(); }
};

}  // namespace shp

struct shapley_server_s {
  std::mutex mu;        // queue, tickets, results
  std::mutex step_mu;   // one scheduler at a time
  size_t budget = 0, used = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint64_t next_ticket = 1;
  std::deque<shp::Request*> queue;
  std::vector<shp::Request*> active;
  std::map<uint64_t, shp::Request*> all;
  std::unique_ptr<shp::Engine> eng;
};

namespace shp {

// Device memory a request needs while active: its game data plus the merged
// level-0 system, the AMG hierarchy and the cycle vectors (about 24 doubles
// and 10 ints per unknown at operator complexity 2).
static size_t estimate_footprint(Game* h) {
  Game* f = h->finest();
  size_t b = h->device_bytes();
  b += (size_t)f->n * (24 * sizeof(double) + 10 * sizeof(int)) + (size_t)f->unnz * 3 * (sizeof(double) + 4);
  return b;
}

static void init_slot(Request* r, hipStream_t s) {
  Game* g = r->current();
  r->slot = SlotState();
  r->slot.g = g;
  r->slot.opt = engine_opts_from(r->opts, g->dim);
  const bool last = !r->famg || r->level == (int)r->handle->levels.size() - 1;
  if (r->famg && !last) {
    double h = 1.0 / (g->s + 1);
    r->slot.opt.eps = r->opts.c_fmg * h * h;
  }
  if (r->level > 0) {
    r->slot.init_alpha = r->slot.init_beta = true;  // v, alpha, beta transferred from the coarser grid
    return;
  }
  const int n = g->n;
  if (!r->v0.empty()) h2d(g->v.p, r->v0.data(), n, s);
  else SHP_HIP(hipMemsetAsync(g->v.p, 0, sizeof(double) * n, s));
  if (!r->alpha0.empty()) {
    h2d(g->alpha.p, r->alpha0.data(), n, s);
    r->slot.init_alpha = true;
  } else {
    SHP_HIP(hipMemsetAsync(g->alpha.p, 0xFF, sizeof(int) * n, s));
  }
  if (!r->alpha0.empty() && !r->beta0.empty()) {
    h2d(g->beta.p, r->beta0.data(), n, s);
    r->slot.init_beta = true;
  } else {
    SHP_HIP(hipMemsetAsync(g->beta.p, 0xFF, sizeof(int) * n, s));
  }
  SHP_HIP(hipStreamSynchronize(s));
}

static void finish(shapley_server_s* srv, Request* r) {
  r->done = true;
  r->t_done = wall_s();
  std::memset(&r->stats, 0, sizeof(r->stats));
  r->stats.outer = r->outer;
  r->stats.inner_total = r->inner;
  r->stats.cycles_total = r->cycles;
  r->stats.levels = r->slot.levels;
  r->stats.converged = r->slot.converged ? 1 : 0;
  r->stats.fmg_levels = r->famg ? r->level + 1 : 1;
  r->stats.residual = r->slot.res;
  r->stats.residual_l2 = r->slot.res_l2;
  r->stats.seconds = r->t_done - r->t_submit;  // latency: completion - submission
  r->stats.setup_seconds = r->setup_s;
  r->stats.cycle_seconds = r->cycle_s;
  r->stats.improve_seconds = r->improve_s;
  r->stats.op_complexity = r->slot.opc;
  r->stats.grid_complexity = r->slot.gc;
  std::memcpy(r->stats.inner_per_outer, r->slot.inner_per_outer, sizeof(r->stats.inner_per_outer));
  r->handle->finest()->solved = true;
  srv->used -= r->footprint;
}

// One scheduling step; returns the number of requests still active.
static int server_step(shapley_server_s* srv) {
  std::lock_guard<std::mutex> sl(srv->step_mu);
  bool changed = false;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    while (!srv->queue.empty()) {
      Request* r = srv->queue.front();
      if (!srv->active.empty() && srv->used + r->footprint > srv->budget) break;
      srv->queue.pop_front();
      srv->used += r->footprint;
      r->t_admit = wall_s();
      srv->active.push_back(r);
      init_slot(r, srv->stream);
      changed = true;
    }
  }
  if (srv->active.empty()) return 0;
  if (!srv->eng) srv->eng.reset(new Engine(srv->stream));
  Engine& eng = *srv->eng;
  if (changed || eng.slots.size() != srv->active.size()) {
    eng.slots.clear();
    for (Request* r : srv->active) eng.slots.push_back(&r->slot);
    eng.invalidate_layout();
  }
  eng.step();
  SHP_HIP(hipStreamSynchronize(srv->stream));
  std::vector<Request*> keep;
  bool moved = false;
  for (Request* r : srv->active) {
    SlotState& S = r->slot;
    if (!S.done) { keep.push_back(r); continue; }
    r->outer += S.k;
    r->inner += S.inner_total;
    r->cycles += S.cycles_total;
    r->setup_s += S.setup_s;
    r->cycle_s += S.cycle_s;
    r->improve_s += S.improve_s;
    const bool more = r->famg && r->level + 1 < (int)r->handle->levels.size() &&
                      (S.status == SHAPLEY_OK || S.status == SHAPLEY_ENOCONV);
    if (more) {
      fmg_transfer(r->handle->levels[r->level], r->handle->levels[r->level + 1], srv->stream);
      SHP_HIP(hipStreamSynchronize(srv->stream));
      r->level += 1;
      init_slot(r, srv->stream);
      keep.push_back(r);
      moved = true;
      continue;
    }
    r->status = S.status;
    std::lock_guard<std::mutex> lk(srv->mu);
    finish(srv, r);
    moved = true;
  }
  srv->active.swap(keep);
  if (moved) {
    eng.slots.clear();
    for (Request* r : srv->active) eng.slots.push_back(&r->slot);
    eng.invalidate_layout();
  }
  return (int)srv->active.size();
}

}  // namespace shp

using namespace shp;

template <class F>
static int sguard(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SHAPLEY_EDEVICE;
  }
}

extern "C" {

int shapley_server_create(shapley_server_t* out, size_t hbm_budget, void* stream) {
  return sguard([&] {
    if (!out || hbm_budget == 0) throw Error(SHAPLEY_EINVAL, "server: out and a positive budget required");
    auto* s = new shapley_server_s();
    s->budget = hbm_budget;
    if (stream) {
      s->stream = (hipStream_t)stream;
    } else {
      hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete s;
        throw Error(SHAPLEY_EDEVICE, "server: stream creation failed");
      }
      s->own_stream = true;
    }
    *out = s;
    return SHAPLEY_OK;
  });
}

int shapley_server_submit(shapley_server_t srv, shapley_game_t g, const shapley_solve_opts* o,
                          uint64_t* ticket) {
  return sguard([&] {
    if (!srv || !g || !g->g || !ticket) throw Error(SHAPLEY_EINVAL, "server: null argument");
    shapley_solve_opts opts;
    if (o) opts = *o; else shapley_default_opts(&opts);
    if (opts.nu1 < 1 || opts.max_outer < 1 || opts.max_inner < 1 || opts.max_cycles < 1 ||
        opts.coarse_max < 1 || opts.coarse_max > kDenseMax || opts.max_levels < 1 || opts.max_levels > 64 ||
        !(opts.omega > 0.0 && opts.omega < 2.0) || !(opts.eps >= 0.0) || !(opts.c_fmg > 0.0) ||
        !(opts.forcing >= 0.0 && opts.forcing < 1.0) || !(opts.reuse_frac >= 0.0 && opts.reuse_frac <= 1.0))
      throw Error(SHAPLEY_EINVAL, "server: invalid options");
    auto* r = new Request();
    r->handle = g->g;
    r->famg = g->g->is_hierarchy() && opts.method == SHAPLEY_FAMGPI;
    Game* first = r->famg ? g->g->levels[0] : g->g->finest();
    const int n = first->n;
    if (opts.alpha0) {
      r->alpha0.assign(opts.alpha0, opts.alpha0 + n);
      for (int32_t a : r->alpha0)
        if (a < 0 || a >= first->m1) { delete r; throw Error(SHAPLEY_EINVAL, "alpha0 out of range"); }
      if (opts.beta0) {
        r->beta0.assign(opts.beta0, opts.beta0 + n);
        for (int32_t b : r->beta0)
          if (b < 0 || b >= first->m2) { delete r; throw Error(SHAPLEY_EINVAL, "beta0 out of range"); }
      }
    }
    if (opts.v0) r->v0.assign(opts.v0, opts.v0 + n);
    opts.alpha0 = opts.beta0 = nullptr;
    opts.v0 = nullptr;
    r->opts = opts;
    r->footprint = estimate_footprint(g->g);
    if (r->footprint > srv->budget) {
      delete r;
      throw Error(SHAPLEY_ENOMEM, "server: request larger than the HBM budget");
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    r->t_submit = wall_s();
    srv->queue.push_back(r);
    srv->all[r->ticket] = r;
    *ticket = r->ticket;
    return SHAPLEY_OK;
  });
}

int shapley_server_poll(shapley_server_t srv, uint64_t ticket, shapley_stats* st) {
  return sguard([&] {
    if (!srv) throw Error(SHAPLEY_EINVAL, "server: null");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) throw Error(SHAPLEY_EINVAL, "server: unknown ticket");
    Request* r = it->second;
    if (!r->done) return SHAPLEY_EAGAIN;
    if (st) *st = r->stats;
    return r->status;
  });
}

int shapley_server_step(shapley_server_t srv, int32_t* active) {
  return sguard([&] {
    if (!srv) throw Error(SHAPLEY_EINVAL, "server: null");
    int a = server_step(srv);
    if (active) {
      std::lock_guard<std::mutex> lk(srv->mu);
      *active = a + (int)srv->queue.size();
    }
    return SHAPLEY_OK;
  });
}

int shapley_server_wait(shapley_server_t srv, uint64_t ticket, int32_t max_steps, shapley_stats* st) {
  return sguard([&] {
    if (!srv) throw Error(SHAPLEY_EINVAL, "server: null");
    for (int k = 0; max_steps <= 0 || k < max_steps; ++k) {
      {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->all.find(ticket);
        if (it == srv->all.end()) throw Error(SHAPLEY_EINVAL, "server: unknown ticket");
        if (it->second->done) {
          if (st) *st = it->second->stats;
          return it->second->status;
        }
      }
      server_step(srv);
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    Request* r = srv->all[ticket];
    if (r->done) {
      if (st) *st = r->stats;
      return r->status;
    }
    return SHAPLEY_EAGAIN;
  });
}

void shapley_server_destroy(shapley_server_t srv) {
  if (!srv) return;
  srv->eng.reset();
  for (auto& kv : srv->all) delete kv.second;
  if (srv->own_stream && srv->stream) (void)hipStreamDestroy(srv->stream);
  delete srv;
}

}  // extern "C"
