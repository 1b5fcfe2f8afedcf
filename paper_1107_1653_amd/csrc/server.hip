// Request loop with continuous batching.
//
// Submitted games (or FAMGpi hierarchies) wait in a FIFO queue.  A scheduling
// step admits queued requests while their estimated device footprint fits the
// HBM budget and advances every active request by one policy-iteration step.
// Requests admitted together with the same engine options form a cohort: one
// lock-step engine on a stream of its own, whose merged launches serve all of
// them and whose AMG hierarchy stays on the device until its last member
// leaves (a member that converges leaves without a rebuild: the hierarchy
// serves any subset of the games it was built for).  Cohorts run concurrently,
// each stepped by its own host thread on its own stream, so that the work of
// requests admitted at different times overlaps on the device.  An FAMGpi
// request that finishes a grid moves to the next finer grid (its state is
// transferred by I and U) and joins a new cohort there.  When the cohort
// count reaches its limit, newly admitted requests join the compatible cohort
// with the fewest running unknowns (that cohort rebuilds its hierarchy).
#include "internal.hpp"
#include "probe.hpp"

#include <chrono>
#include <cstring>
#include <deque>
#include <future>
#include <map>
#include <mutex>

namespace shp {

static double wall_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxCohorts = 16;
// a cohort's games hold at most this many states together (a bigger request
// runs alone): merged levels stay far from the 32-bit limits of one hierarchy
// and the setup scratch of one engine stays a few GB
constexpr int64_t kCohortMaxStates = int64_t(1) << 23;
constexpr size_t kPoolEngines = 4;  // idle engines kept with their workspace

struct Cohort;

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
  std::string msg;          // error message of a failed request
  SlotState* slot = nullptr;  // inside the current cohort
  Cohort* cohort = nullptr;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int outer = 0, inner = 0, cycles = 0;
  int sfull = 0, sref = 0, vsteps = 0;
  double setup_s = 0, cycle_s = 0, improve_s = 0;
  shapley_stats stats{};

  Game* current() { return famg ? handle->levels[level] : handle->finest(); }
};

// Engine options that act on the whole merged hierarchy or sweep: requests
// share a cohort only when all of them agree.
struct CohortKey {
  int precision, nu1, nu2, coarse_max, max_levels, smoother, gamma;
  double theta, omega, reuse_frac, tie_rtol;
  bool operator==(const CohortKey& o) const {
    return precision == o.precision && nu1 == o.nu1 && nu2 == o.nu2 && coarse_max == o.coarse_max &&
           max_levels == o.max_levels && smoother == o.smoother && gamma == o.gamma && theta == o.theta &&
           omega == o.omega && reuse_frac == o.reuse_frac && tie_rtol == o.tie_rtol;
  }
};
static CohortKey key_of(const shapley_solve_opts& o) {
  return CohortKey{o.precision, o.nu1,   o.nu2,   o.coarse_max, o.max_levels, o.smoother,
                   o.gamma,     o.theta, o.omega, o.reuse_frac, o.tie_rtol};
}

struct Cohort {
  CohortKey key{};
  hipStream_t stream = nullptr;
  std::unique_ptr<Engine> eng;
  std::vector<std::unique_ptr<SlotState>> slots;  // one per membership
  std::vector<Request*> members;                  // members[i] runs in slots[i]
  int error = SHAPLEY_OK;
  std::string msg;
  int64_t running_unknowns() const {
    int64_t u = 0;
    for (const auto& s : slots)
      if (!s->done) u += s->g->n;
    return u;
  }
  bool running() const {
    for (const auto& s : slots)
      if (!s->done) return true;
    return false;
  }
};

}  // namespace shp

struct shapley_server_s {
  std::mutex mu;        // queue, tickets, results
  std::mutex step_mu;   // one scheduler at a time
  size_t budget = 0, used = 0;
  int device = 0;
  hipStream_t stream = nullptr;  // the caller's stream (all cohorts on it), or null
  uint64_t next_ticket = 1;
  std::deque<shp::Request*> queue;
  std::vector<shp::Request*> active;
  std::map<uint64_t, shp::Request*> all;
  std::vector<std::unique_ptr<shp::Cohort>> cohorts;
  // idle engines with their streams, reused by new cohorts (their device
  // buffers are kept: a cohort no larger than an earlier one allocates nothing)
  std::vector<std::pair<hipStream_t, std::unique_ptr<shp::Engine>>> pool;
  std::vector<hipStream_t> own_streams;
  std::vector<hipStream_t> free_streams;  // owned, not held by a cohort or the pool
};

namespace shp {

// Device memory a request needs while active: its game data plus the merged
// level-0 system, the AMG hierarchy and the cycle vectors (about 24 doubles
// and 10 ints per unknown at operator complexity 2) and its share of the
// setup scratch of the Galerkin product (up to 16 products of 12 bytes per
// level-0 entry).
static size_t estimate_footprint(Game* h) {
  Game* f = h->finest();
  size_t b = h->device_bytes();
  b += (size_t)f->n * (25 * sizeof(double) + 11 * sizeof(int)) + (size_t)f->unnz * 3 * (sizeof(double) + 4);
  b += (size_t)f->unnz * PW * PW * (sizeof(double) + sizeof(int));
  // the stencil form of level 0 (grid games): slot values in both precisions and a code word
  if (!f->st_off.empty()) b += (size_t)f->n * ((size_t)f->st_w * (sizeof(double) + sizeof(float)) + 4);
  return b;
}

// A fresh slot for the request's current grid, its start (v, alpha, beta)
// written on stream s: the warm start on the first grid, the state
// transferred from the coarser grid on the others.
static std::unique_ptr<SlotState> make_slot(Request* r, hipStream_t s) {
  Game* g = r->current();
  std::unique_ptr<SlotState> S(new SlotState());
  S->g = g;
  S->opt = engine_opts_from(r->opts, g->dim);
  const bool last = !r->famg || r->level == (int)r->handle->levels.size() - 1;
  if (r->famg && !last) {
    double h = 1.0 / (g->s + 1);
    S->opt.eps = r->opts.c_fmg * h * h;
  }
  if (r->level > 0) {
    S->init_alpha = S->init_beta = true;  // v, alpha, beta transferred from the coarser grid
    return S;
  }
  const int n = g->n;
  if (!r->v0.empty()) h2d(g->v.p, r->v0.data(), n, s);
  else fill_async(g->v.p, 0.0, n, s);
  if (!r->alpha0.empty()) {
    h2d(g->alpha.p, r->alpha0.data(), n, s);
    S->init_alpha = true;
  } else {
    fill_async(g->alpha.p, -1, n, s);
  }
  if (!r->alpha0.empty() && !r->beta0.empty()) {
    h2d(g->beta.p, r->beta0.data(), n, s);
    S->init_beta = true;
  } else {
    fill_async(g->beta.p, -1, n, s);
  }
  SHP_HIP(hipStreamSynchronize(s));
  return S;
}

static void finish(shapley_server_s* srv, Request* r, int status, const std::string& msg) {
  SlotState* S = r->slot;
  r->done = true;
  r->status = status;
  r->msg = msg;
  r->t_done = wall_s();
  std::memset(&r->stats, 0, sizeof(r->stats));
  r->stats.outer = r->outer;
  r->stats.inner_total = r->inner;
  r->stats.cycles_total = r->cycles;
  r->stats.fmg_levels = r->famg ? r->level + 1 : 1;
  r->stats.seconds = r->t_done - r->t_submit;  // latency: completion - submission
  r->stats.setup_seconds = r->setup_s;
  r->stats.cycle_seconds = r->cycle_s;
  r->stats.improve_seconds = r->improve_s;
  r->stats.setups_full = r->sfull;
  r->stats.setups_refresh = r->sref;
  r->stats.value_steps = r->vsteps;
  if (S) {
    r->stats.levels = S->levels;
    r->stats.converged = S->converged && status == SHAPLEY_OK ? 1 : 0;
    r->stats.residual = S->res;
    r->stats.residual_l2 = S->res_l2;
    r->stats.op_complexity = S->opc;
    r->stats.grid_complexity = S->gc;
    std::memcpy(r->stats.inner_per_outer, S->inner_per_outer, sizeof(r->stats.inner_per_outer));
  }
  r->handle->finest()->solved = true;
  r->cohort = nullptr;
  r->slot = nullptr;  // owned by the cohort, which may retire now
  srv->used -= r->footprint;
}

static void account(Request* r) {
  const SlotState& S = *r->slot;
  r->outer += S.k;
  r->inner += S.inner_total;
  r->cycles += S.cycles_total;
  r->sfull += S.setups_full;
  r->sref += S.setups_refresh;
  r->vsteps += S.solves;
  r->setup_s += S.setup_s;
  r->cycle_s += S.cycle_s;
  r->improve_s += S.improve_s;
}

static Cohort* new_cohort(shapley_server_s* srv, const CohortKey& key) {
  std::unique_ptr<Cohort> c(new Cohort());
  c->key = key;
  if (srv->stream) {
    c->stream = srv->stream;
    c->eng.reset(new Engine(srv->stream));
  } else if (!srv->pool.empty()) {
    c->stream = srv->pool.back().first;
    c->eng = std::move(srv->pool.back().second);
    srv->pool.pop_back();
  } else {
    hipStream_t s;
    if (!srv->free_streams.empty()) {
      s = srv->free_streams.back();
      srv->free_streams.pop_back();
    } else {
      SHP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      srv->own_streams.push_back(s);
    }
    c->stream = s;
    c->eng.reset(new Engine(s));
  }
  c->eng->reset();
  srv->cohorts.emplace_back(std::move(c));
  return srv->cohorts.back().get();
}

// Puts requests (already counted in the budget) into cohorts: a new cohort
// per group of equal engine options, or, with the cohort count at its limit,
// the compatible cohort with the fewest running unknowns.
static void place(shapley_server_s* srv, const std::vector<Request*>& rs) {
  std::vector<std::pair<CohortKey, std::vector<Request*>>> groups;
  for (Request* r : rs) {
    const CohortKey k = key_of(r->opts);
    bool found = false;
    for (auto& gr : groups)
      if (gr.first == k) { gr.second.push_back(r); found = true; break; }
    if (!found) groups.push_back({k, {r}});
  }
  // each group in chunks of at most kCohortMaxStates states (in FIFO order)
  std::vector<std::pair<CohortKey, std::vector<Request*>>> chunks;
  for (auto& gr : groups) {
    int64_t states = 0;
    chunks.push_back({gr.first, {}});
    for (Request* r : gr.second) {
      const int64_t n = r->current()->n;
      if (!chunks.back().second.empty() && states + n > kCohortMaxStates) {
        chunks.push_back({gr.first, {}});
        states = 0;
      }
      chunks.back().second.push_back(r);
      states += n;
    }
  }
  for (auto& gr : chunks) {
    int64_t add = 0;
    for (Request* r : gr.second) add += r->current()->n;
    Cohort* c = nullptr;
    bool joining = false;
    if ((int)srv->cohorts.size() >= kMaxCohorts) {
      int64_t best = INT64_MAX;
      for (auto& q : srv->cohorts) {
        const int64_t u = q->running_unknowns();
        if (q->key == gr.first && q->error == SHAPLEY_OK && u + add <= kCohortMaxStates && u < best) {
          best = u;
          c = q.get();
        }
      }
      joining = c != nullptr;
    }
    if (!c) c = new_cohort(srv, gr.first);
    if (joining) {
      // finished memberships leave the merged layout at this rebuild
      std::vector<std::unique_ptr<SlotState>> keep_s;
      std::vector<Request*> keep_m;
      for (size_t i = 0; i < c->slots.size(); ++i)
        if (!c->slots[i]->done) {
          keep_s.push_back(std::move(c->slots[i]));
          keep_m.push_back(c->members[i]);
        }
      c->slots.swap(keep_s);
      c->members.swap(keep_m);
    }
    for (Request* r : gr.second) {
      c->slots.push_back(make_slot(r, c->stream));
      c->members.push_back(r);
      r->slot = c->slots.back().get();
      r->cohort = c;
    }
    c->eng->slots.clear();
    for (auto& s : c->slots) c->eng->slots.push_back(s.get());
    c->eng->invalidate_layout();
  }
}

static void step_cohort(Cohort* c, int device) {
  try {
    SHP_HIP(hipSetDevice(device));
    c->eng->step();
    SHP_HIP(hipStreamSynchronize(c->stream));
  } catch (const Error& e) {
    c->error = e.code;
    c->msg = e.what();
  } catch (const std::bad_alloc&) {
    c->error = SHAPLEY_ENOMEM;
    c->msg = "host allocation failed";
  } catch (const std::exception& e) {
    c->error = SHAPLEY_EDEVICE;
    c->msg = e.what();
  }
}

// One scheduling step; returns the number of requests still active.
static int server_step(shapley_server_s* srv) {
  std::lock_guard<std::mutex> sl(srv->step_mu);
  SHP_HIP(hipSetDevice(srv->device));
  std::vector<Request*> admitted;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    while (!srv->queue.empty()) {
      Request* r = srv->queue.front();
      if (!srv->active.empty() && srv->used + r->footprint > srv->budget) break;
      srv->queue.pop_front();
      srv->used += r->footprint;
      r->t_admit = wall_s();
      srv->active.push_back(r);
      admitted.push_back(r);
    }
  }
  if (!admitted.empty()) place(srv, admitted);
  if (srv->active.empty()) return 0;
  // one policy-iteration step of every cohort with running members; cohorts on
  // streams of their own step concurrently (the timing probe's event pairs are
  // process-wide, so with a probe on they step one after the other)
  std::vector<Cohort*> run;
  for (auto& c : srv->cohorts)
    if (c->error == SHAPLEY_OK && c->running()) run.push_back(c.get());
  bool probing = false;
  for (int f = 0; f < kProbeFamilies; ++f) probing |= probe_on(f);
  if (run.size() == 1 || srv->stream || probing) {
    for (Cohort* c : run) step_cohort(c, srv->device);
  } else {
    std::vector<std::future<void>> fut;
    for (size_t i = 1; i < run.size(); ++i)
      fut.push_back(std::async(std::launch::async, step_cohort, run[i], srv->device));
    step_cohort(run[0], srv->device);
    for (auto& f : fut) f.get();
  }
  // leave, finish or move to the next grid
  std::vector<Request*> moving;
  std::vector<Request*> keep;
  for (Request* r : srv->active) {
    Cohort* c = r->cohort;
    SlotState& S = *r->slot;
    if (c->error != SHAPLEY_OK) {
      account(r);
      std::lock_guard<std::mutex> lk(srv->mu);
      finish(srv, r, c->error, c->msg);
      continue;
    }
    if (!S.done) { keep.push_back(r); continue; }
    account(r);
    const bool more = r->famg && r->level + 1 < (int)r->handle->levels.size() &&
                      (S.status == SHAPLEY_OK || S.status == SHAPLEY_ENOCONV);
    if (more) {
      fmg_transfer(r->handle->levels[r->level], r->handle->levels[r->level + 1], c->stream);
      SHP_HIP(hipStreamSynchronize(c->stream));
      r->level += 1;
      r->cohort = nullptr;
      r->slot = nullptr;
      moving.push_back(r);
      keep.push_back(r);
      continue;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    finish(srv, r, S.status, S.status == SHAPLEY_OK ? std::string() : (S.why.empty() ? "policy iteration stopped "
                                                                                     "with an error" : S.why));
  }
  srv->active.swap(keep);
  // retire cohorts with no running member: their engines return to the pool
  // (or are dropped after an error)
  std::vector<std::unique_ptr<Cohort>> live;
  for (auto& c : srv->cohorts) {
    if (c->error == SHAPLEY_OK && c->running()) {
      live.push_back(std::move(c));
      continue;
    }
    if (c->error == SHAPLEY_OK && !srv->stream && srv->pool.size() < kPoolEngines) {
      c->eng->reset();
      srv->pool.emplace_back(c->stream, std::move(c->eng));
    } else if (!srv->stream) {
      // the engine and its workspace are released with the cohort; the stream
      // serves a later cohort
      c->eng.reset();
      srv->free_streams.push_back(c->stream);
    }
  }
  srv->cohorts.swap(live);
  if (!moving.empty()) place(srv, moving);
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
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return SHAPLEY_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return SHAPLEY_EDEVICE;
  }
}

static int result_of(shp::Request* r, shapley_stats* st) {
  if (st) *st = r->stats;
  if (r->status != SHAPLEY_OK) set_last_error(r->msg);
  return r->status;
}

extern "C" {

int shapley_server_create(shapley_server_t* out, size_t hbm_budget, void* stream) {
  return sguard([&] {
    if (!out || hbm_budget == 0) throw Error(SHAPLEY_EINVAL, "server: out and a positive budget required");
    int dev = 0;
    SHP_HIP(hipGetDevice(&dev));
    auto* s = new shapley_server_s();
    s->budget = hbm_budget;
    s->device = dev;
    s->stream = (hipStream_t)stream;
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
    check_solve_opts(opts);
    std::unique_ptr<Request> r(new Request());
    r->handle = g->g;
    r->famg = g->g->is_hierarchy() && opts.method == SHAPLEY_FAMGPI;
    Game* first = r->famg ? g->g->levels[0] : g->g->finest();
    const int n = first->n;
    // warm start checked against the first grid now (the game is not in use
    // by the server before its admission)
    check_warm_start(first, opts.alpha0, opts.alpha0 ? opts.beta0 : nullptr, first->stream);
    if (opts.alpha0) {
      r->alpha0.assign(opts.alpha0, opts.alpha0 + n);
      if (opts.beta0) r->beta0.assign(opts.beta0, opts.beta0 + n);
    }
    if (opts.v0) r->v0.assign(opts.v0, opts.v0 + n);
    opts.alpha0 = opts.beta0 = nullptr;
    opts.v0 = nullptr;
    r->opts = opts;
    r->footprint = estimate_footprint(g->g);
    if (r->footprint > srv->budget)
      throw Error(SHAPLEY_ENOMEM, "server: request larger than the HBM budget");
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    r->t_submit = wall_s();
    *ticket = r->ticket;
    srv->all[r->ticket] = r.get();
    srv->queue.push_back(r.release());
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
    return result_of(r, st);
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
        if (it->second->done) return result_of(it->second, st);
      }
      server_step(srv);
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) throw Error(SHAPLEY_EINVAL, "server: unknown ticket");
    if (it->second->done) return result_of(it->second, st);
    return SHAPLEY_EAGAIN;
  });
}

int shapley_server_info(shapley_server_t srv, shapley_server_stats* st) {
  return sguard([&] {
    if (!srv || !st) throw Error(SHAPLEY_EINVAL, "server: null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::memset(st, 0, sizeof(*st));
    st->queued = (int32_t)srv->queue.size();
    st->active = (int32_t)srv->active.size();
    st->cohorts = (int32_t)srv->cohorts.size();
    st->budget_used = srv->used;
    st->budget = srv->budget;
    return SHAPLEY_OK;
  });
}

void shapley_server_destroy(shapley_server_t srv) {
  if (!srv) return;
  srv->cohorts.clear();
  srv->pool.clear();
  for (auto& kv : srv->all) delete kv.second;
  for (hipStream_t s : srv->own_streams) (void)hipStreamDestroy(s);
  delete srv;
}

}  // extern "C"
