// Lock-step policy-iteration engine (AMGpi, Sec. 5.1) over one or many games.
//
// Every step performs, for each running game: the value step -- assemble the
// policy system (LSPI) and solve it by AMG (setup + FP64 iterative
// refinement around FP32 or FP64 V-cycles, Algorithm MGcycle) -- then one
// improvement sweep giving MIN's improvement (algo-MDP step 2), MAX's
// improvement (PIalgo step 2) and the residual ||F(v) - v||_inf, after which
// each game decides on its own whether it continues the inner loop, moves to
// the next outer iteration or stops.  Games are merged block-diagonally into
// every AMG level so that one launch per kernel serves all of them.
#include "amg_kernels.hpp"
#include "probe.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <climits>
#include <exception>
#include <map>
#include <mutex>
#include <chrono>
#include <cmath>

namespace shp {

namespace {
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class T>
struct LV;
template <>
struct LV<float> {
  static float* a(Level& L) { return L.a32.p; }
  static float* d(Level& L) { return L.dinv32.p; }
  static float* pv(Level& L) { return L.pv32.p; }
  static float* rv(Level& L) { return L.rv32.p; }
  static float* dm(Level& L) { return L.dmat32.p; }
  static float* x(Level& L) { return L.x32.p; }
  static float* y(Level& L) { return L.y32.p; }
  static float* b(Level& L) { return L.b32.p; }
  static float* r(Level& L) { return L.r32.p; }
  static float* st(Level& L) { return L.st32.p; }
};
template <>
struct LV<double> {
  static double* a(Level& L) { return L.a64.p; }
  static double* d(Level& L) { return L.dinv64.p; }
  static double* pv(Level& L) { return L.pv64.p; }
  static double* rv(Level& L) { return L.rv64.p; }
  static double* dm(Level& L) { return L.dmat64.p; }
  static double* x(Level& L) { return L.x64.p; }
  static double* y(Level& L) { return L.y64.p; }
  static double* b(Level& L) { return L.b64.p; }
  static double* r(Level& L) { return L.r64.p; }
  static double* st(Level& L) { return L.st64.p; }
};
}  // namespace

std::vector<Tile> make_tiles(const std::vector<int>& off, const std::vector<char>& keep, int rows) {
  std::vector<Tile> t;
  int G = (int)off.size() - 1;
  for (int g = 0; g < G; ++g) {
    if (!keep[g]) continue;
    for (int r = off[g]; r < off[g + 1]; r += rows) t.push_back({r, std::min(r + rows, off[g + 1]), g});
  }
  return t;
}

// Optional phase profile (environment SHAPLEY_PROFILE=1): wall time per
// setup/solve phase with a stream synchronisation at each phase boundary,
// printed to stderr when the engine is destroyed.
static bool profiling() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("SHAPLEY_PROFILE");
    on = (e && e[0] == '1') ? 1 : 0;
  }
  return on == 1;
}

// First kernel of a row-wise Galerkin product whose rows are expected to
// average `cols` distinct columns (the level's previous product, else an
// estimate).  Products through P's four slots take four lanes per row (up
// to 32 or 64 columns); products through an identity P (one slot) take a
// thread per row (up to 16 or 32).  Rows beyond the kernel's columns go to
// the wavefront kernel.  shapley_tune_galerkin forces the family; the
// product is the same bit for bit whichever kernel computes a row.
static std::atomic<int> g_gal_mode{-1};
void set_forced_rap_cols(int mode) { g_gal_mode.store(mode); }
// interpolation of coarse levels: 0 the wavefront kernel alone, 4 four lanes
// per row first, -1 four lanes on large levels (the same weights either way)
static std::atomic<int> g_interp_mode{-1};
constexpr int kInterpQuadRows = 1 << 16;  // automatic choice: levels of at least this many rows
void set_interp_mode(int mode) { g_interp_mode.store(mode); }
// compact matrix forms for the cycle kernels: -1 (default) level 0 in the
// stencil form when every game is a stencil game, 16-bit column offsets on
// the other levels where they fit; 0 CSR with 32-bit columns (the same results)
static std::atomic<int> g_stencil_mode{-1};
void set_stencil_mode(int mode) { g_stencil_mode.store(mode); }
static int gal_kernel(double cols, bool one_slot) {
  const int mode = g_gal_mode.load();
  if (mode == 0) return kGalWave;
  const bool thread = mode == 1 || (mode == -1 && one_slot);
  if (thread) {
    if (mode == -1 && cols > 20.0) return kGalWave;
    return cols <= 9.0 ? kGalThread16 : kGalThread32;
  }
  if (mode == -1 && cols > 44.0) return kGalWave;
  return cols <= 24.0 ? kGalQuad32 : kGalQuad64;
}

struct PhaseTimer {
  Engine* eng;
  std::vector<std::pair<std::string, double>>& acc;
  double t;
  PhaseTimer(Engine* e, std::vector<std::pair<std::string, double>>& a) : eng(e), acc(a), t(0) {
    if (profiling()) { SHP_HIP(hipStreamSynchronize(e->stream)); t = now_s(); }
  }
  void mark(const char* name) {
    if (!profiling()) return;
    SHP_HIP(hipStreamSynchronize(eng->stream));
    double t1 = now_s();
    for (auto& p : acc)
      if (p.first == name) { p.second += t1 - t; t = t1; return; }
    acc.emplace_back(name, t1 - t);
    t = t1;
  }
};

Engine::Engine(hipStream_t s) : stream(s) {}

void* Engine::pin_take(size_t bytes) {
  bytes = (bytes + 63) & ~(size_t)63;
  if (pin_used + bytes > pin_cap) {
    // a fresh, larger arena; the full one may still be the source or the
    // target of queued copies and is released at the next synchronisation
    if (pin) pin_old.push_back(pin);
    pin = nullptr;
    pin_cap = std::max<size_t>(bytes, std::max<size_t>(2 * pin_cap, 1 << 16));
    SHP_HIP(hipHostMalloc((void**)&pin, pin_cap, hipHostMallocDefault));
    pin_used = 0;
  }
  void* p = pin + pin_used;
  pin_used += bytes;
  return p;
}

void Engine::sync() {
  SHP_HIP(hipStreamSynchronize(stream));
  pin_used = 0;
  for (char* q : pin_old) SHP_HIP(hipHostFree(q));
  pin_old.clear();
}

void Engine::reset() {
  slots.clear();
  layout_dirty = true;
  asm_stale = true;
  have_hier = false;
  ++hier_gen;
  run_at_setup.clear();
  changes_since_setup = 0;
  changes_since_refresh = 0;
  last_cycles = 0;
  cycles_after_full = -1;
  stagnated = false;
  full_setups = refreshes = 0;
}

namespace {
// idle engines per stream; never destroyed at process exit (the runtime may
// already be gone then), emptied when the last game handle is destroyed.
// While less than a quarter of the device memory is free (or more than
// kIdleEngines are idle), the least recently used are destroyed: games solved
// one after another on streams of their own keep their workspaces only as
// long as memory allows.
std::mutex g_cache_mu;
auto& g_cache = *new std::map<hipStream_t, std::unique_ptr<Engine>>();
auto& g_cache_use = *new std::map<hipStream_t, uint64_t>();
uint64_t g_cache_clock = 0;
int g_games_alive = 0;
constexpr size_t kIdleEngines = 1024;
}  // namespace

void games_alive_add(int delta) {
  std::map<hipStream_t, std::unique_ptr<Engine>> drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_games_alive += delta;
    if (g_games_alive <= 0) {
      g_games_alive = 0;
      drop.swap(g_cache);  // last game gone: release the workspace
      g_cache_use.clear();
    }
  }
}

void engine_cache_drop(hipStream_t s) {
  std::unique_ptr<Engine> drop;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(s);
  if (it == g_cache.end()) return;
  drop = std::move(it->second);
  g_cache.erase(it);
  g_cache_use.erase(s);
}

Engine* engine_cached(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  auto it = g_cache.find(s);
  return it == g_cache.end() ? nullptr : it->second.get();
}

void Engine::level_export(int l, int* levels, int64_t* n, int64_t* nnz, int64_t* nc, int32_t* rp, int32_t* ci,
                          double* a, int32_t* pc, double* pv) {
  if (l < 0 || l >= nlev) throw Error(SHAPLEY_EINVAL, "level out of range");
  const Level& L = lv[l];
  const int cn = l + 1 < nlev ? L.nc : 0;
  if (levels) *levels = nlev;
  if (n) *n = L.n;
  if (nnz) *nnz = L.nnz;
  if (nc) *nc = cn;
  SHP_HIP(hipStreamSynchronize(stream));
  if (rp) SHP_HIP(hipMemcpy(rp, L.rp.p, sizeof(int) * ((size_t)L.n + 1), hipMemcpyDeviceToHost));
  if (ci && L.nnz) SHP_HIP(hipMemcpy(ci, L.ci.p, sizeof(int) * (size_t)L.nnz, hipMemcpyDeviceToHost));
  // level 0: the operator the coarse levels were formed from (the last setup
  // or refresh; later policy steps may have assembled newer values since)
  const double* av = (l == 0 && L.a_prev.p) ? L.a_prev.p : L.a64.p;
  if (a && L.nnz) SHP_HIP(hipMemcpy(a, av, sizeof(double) * (size_t)L.nnz, hipMemcpyDeviceToHost));
  if (cn && pc) SHP_HIP(hipMemcpy(pc, L.pc.p, sizeof(int) * (size_t)L.n * PW, hipMemcpyDeviceToHost));
  if (cn && pv) SHP_HIP(hipMemcpy(pv, L.pv64.p, sizeof(double) * (size_t)L.n * PW, hipMemcpyDeviceToHost));
}

EngineLease::EngineLease(hipStream_t s, bool keep)
    : s_(s), keep_(keep), uncaught_(std::uncaught_exceptions()) {
  if (keep) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(s);
    if (it != g_cache.end()) {
      e_ = std::move(it->second);
      g_cache.erase(it);
      g_cache_use.erase(s);
    }
  }
  if (!e_) e_.reset(new Engine(s));
  e_->reset();
}

EngineLease::~EngineLease() {
  if (!keep_ || std::uncaught_exceptions() > uncaught_) return;  // not kept: destroyed here
  e_->reset();
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_games_alive > 0 && !g_cache.count(s_)) {
      g_cache[s_] = std::move(e_);
      g_cache_use[s_] = ++g_cache_clock;
    }
  }
  // one engine at a time, each destroyed (its memory freed) before the next check
  for (;;) {
    std::unique_ptr<Engine> victim;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      if (g_cache.empty()) break;
      size_t fr = 0, tot = 0;
      const bool low = hipMemGetInfo(&fr, &tot) == hipSuccess && fr < tot / 4;
      if (!low && g_cache.size() <= kIdleEngines) break;
      auto lru = g_cache_use.begin();
      for (auto u = g_cache_use.begin(); u != g_cache_use.end(); ++u)
        if (u->second < lru->second) lru = u;
      victim = std::move(g_cache[lru->first]);
      g_cache.erase(lru->first);
      g_cache_use.erase(lru);
    }
  }
}
void Engine::drop_graph() {
  if (cyc_exec) (void)hipGraphExecDestroy(cyc_exec);
  cyc_exec = nullptr;
}

Engine::~Engine() {
  drop_graph();
  if (profiling() && !prof.empty()) {
    fprintf(stderr, "[shapley profile]");
    for (auto& p : prof) fprintf(stderr, " %s=%.2fms", p.first.c_str(), 1e3 * p.second);
    fprintf(stderr, "\n");
  }
  if (pin || !pin_old.empty()) {
    (void)hipStreamSynchronize(stream);
    if (pin) (void)hipHostFree(pin);
    for (char* q : pin_old) (void)hipHostFree(q);
  }
}

std::vector<int> Engine::running_slots() const {
  std::vector<int> r;
  for (int g = 0; g < (int)slots.size(); ++g)
    if (!slots[g]->done) r.push_back(g);
  return r;
}

void Engine::build_layout() {
  G = (int)slots.size();
  x_off.assign(G + 1, 0);
  a_off.assign(G + 1, 0);
  for (int g = 0; g < G; ++g) {
    Game* gm = slots[g]->g;
    x_off[g + 1] = x_off[g] + gm->n;
    int64_t an = (int64_t)a_off[g] + gm->unnz;
    if (an > INT32_MAX) throw Error(SHAPLEY_EINVAL, "merged level-0 pattern exceeds 2^31 entries");
    a_off[g + 1] = (int)an;
  }
  N0 = x_off[G];
  NNZ0 = a_off[G];
  // kernels with a wavefront per row index 64 N threads in 32 bits
  if (N0 > kMaxMergedRows)
    throw Error(SHAPLEY_ENOMEM, "the games solved together hold " + std::to_string(N0) +
                                    " states, more than one merged hierarchy takes (" +
                                    std::to_string(kMaxMergedRows) + "): solve fewer games together");
  hdesc.resize(G);
  h_gtiles_all.clear();
  h_gtiles_imp.clear();
  {
    int max_rows = 1;
    for (int g = 0; g < G; ++g) max_rows = std::max(max_rows, slots[g]->g->m1 * slots[g]->g->m2);
    // 128-thread workgroups where a state's rows fit (measured on the 256-game
    // batch: 10.0-10.1 ms of improvement sweeps per solve against 10.4 with
    // 256 threads and 10.3 with 64)
    imp_threads = improve_threads(max_rows, 128);
  }
  for (int g = 0; g < G; ++g) {
    Game* gm = slots[g]->g;
    GameDesc d{};
    d.rp = gm->rp.p; d.ci = gm->ci.p; d.w = gm->w.p; d.r = gm->r.p; d.valid = gm->valid.p;
    d.urp = gm->urp.p; d.uci = gm->uci.p;
    d.v = gm->v.p; d.alpha = gm->alpha.p; d.beta = gm->beta.p;
    d.beta_in = gm->beta_in.p; d.alpha_c = gm->alpha_c.p; d.beta_c = gm->beta_c.p;
    d.F = keep_F ? gm->F.p : nullptr;  // policy-iteration sweeps need only its residual
    d.bvals = gm->has_bvals ? gm->bvals.p : nullptr;
    d.n = gm->n; d.m1 = gm->m1; d.m2 = gm->m2; d.slot = g; d.mu = gm->mu;
    d.x_off = x_off[g]; d.a_off = a_off[g];
    hdesc[g] = d;
    for (int x = 0; x < gm->n; x += kBlock) h_gtiles_all.push_back({g, x, std::min(x + kBlock, gm->n)});
    const int spb = improve_states_per_tile(gm->m1, gm->m2, imp_threads);
    for (int x = 0; x < gm->n; x += spb) h_gtiles_imp.push_back({g, x, std::min(x + spb, gm->n)});
  }
  ddesc.ensure(std::max(G, 1));
  up(ddesc.p, hdesc.data(), G);
  gtiles_all.ensure(std::max<size_t>(h_gtiles_all.size(), 1));
  up(gtiles_all.p, h_gtiles_all.data(), h_gtiles_all.size());
  gtiles_imp.ensure(std::max<size_t>(h_gtiles_imp.size(), 1));
  up(gtiles_imp.p, h_gtiles_imp.data(), h_gtiles_imp.size());
  launch_tile_entries(ddesc.p, gtiles_imp.p, (int)h_gtiles_imp.size(), stream);

  int maxlev = 2;
  for (auto* s : slots) maxlev = std::max(maxlev, s->opt.max_levels + 1);
  if ((int)lv.size() < maxlev) lv.resize(maxlev);
  Level& L0 = lv[0];
  L0.n = N0;
  L0.nnz = NNZ0;
  L0.rp.ensure(N0 + 1);
  L0.ci.ensure(std::max(NNZ0, 1));
  launch_layout(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), L0.rp.p, L0.ci.p, N0, NNZ0, stream);
  L0.goff = x_off;
  // the stencil form of level 0: every game a stencil game, relaxation by
  // whole sweeps (the C/F half sweeps keep the CSR kernels)
  L0.stencil = g_stencil_mode.load() != 0 && G > 0 && slots[0]->opt.smoother != SHAPLEY_SMOOTH_CF;
  L0.st_w = 0;
  for (int g = 0; g < G && L0.stencil; ++g) {
    const Game* gm = slots[g]->g;
    L0.stencil = !gm->st_off.empty();
    L0.st_w = std::max(L0.st_w, gm->st_w);
  }
  if (L0.stencil) {
    std::vector<int> off((size_t)kStencilMax * G, 0);
    for (int g = 0; g < G; ++g) {
      const std::vector<int>& o = slots[g]->g->st_off;
      std::copy(o.begin(), o.end(), off.begin() + (size_t)kStencilMax * g);
    }
    d_st_off.ensure(off.size());
    up(d_st_off.p, off.data(), off.size());
    L0.st_code.ensure(std::max(N0, 1));
    launch_stencil_codes(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_st_off.p, L0.st_code.p, stream);
  }

  d_active.ensure(std::max(G, 1));
  h_active_dev.clear();
  d_norm.ensure(4 * std::max(G, 1));
  d_shap.ensure(4 * std::max(G, 1));
  d_cnt = reinterpret_cast<int*>(d_shap.p + 2 * std::max(G, 1));
  d_lin.ensure(2 * std::max(G, 1));  // LinCtl is larger than an int
  d_lin_active = reinterpret_cast<int*>(d_lin.p + std::max(G, 1));
  d_decision.ensure(std::max(G, 1));
  {
    const int gp = stripe_games(G);
    const size_t m = (size_t)kStripes * gp * 4;
    fold_d.ensure(m);
    fold_i.ensure(m);
    fill_async(fold_d.p, 0.0, m, stream);
    fill_async(fold_i.p, 0, m, stream);
    fold = Stripes{fold_d.p, fold_i.p, gp};
  }
  h_active.assign(G, 0);
  h_lin_active.assign(G, 0);
  asm_stale = true;
  layout_dirty = false;
}

void Engine::build_tiles(Level& L, const std::vector<char>& keep, bool cont_only) {
  std::vector<Tile>& t = cont_only ? L.h_ctiles : L.h_tiles;
  t = make_tiles(L.goff, keep, kTileRows);
  int rows = 0;
  for (const Tile& x : t) rows += x.r1 - x.r0;
  if (cont_only) {
    L.nctiles = (int)t.size();
    L.rows_ctiles = rows;
    L.ctiles.ensure(std::max<size_t>(t.size(), 1));
    up(L.ctiles.p, t.data(), t.size());
  } else {
    L.ntiles = (int)t.size();
    L.rows_tiles = rows;
    L.tiles.ensure(std::max<size_t>(t.size(), 1));
    up(L.tiles.p, t.data(), t.size());
  }
}

void Engine::assemble(const std::vector<int>& run, bool mixed) {
  Level& L0 = lv[0];
  L0.a64.ensure(std::max(NNZ0, 1));
  L0.dinv64.ensure(std::max(N0, 1));
  if (mixed) {
    L0.a32.ensure(std::max(NNZ0, 1));
    L0.dinv32.ensure(std::max(N0, 1));
  }
  L0.b64.ensure(std::max(N0, 1));   // cycle vectors (FP64 mode) and refinement storage below
  L0.r64.ensure(std::max(N0, 1));
  L0.x64.ensure(std::max(N0, 1));
  L0.y64.ensure(std::max(N0, 1));
  d_norm.ensure(4 * std::max(G, 1));
  // refinement storage: solution in sol (L0.tmp is int; use dedicated buffers)
  asm_pol.ensure(std::max(N0, 1));
  asm_dinv.ensure(std::max(N0, 1));
  if (L0.stencil) {
    L0.st64.ensure((size_t)L0.st_w * std::max(N0, 1));
    if (mixed) L0.st32.ensure((size_t)L0.st_w * std::max(N0, 1));
  }
  double* st64 = L0.stencil ? L0.st64.p : nullptr;
  float* st32 = L0.stencil && mixed ? L0.st32.p : nullptr;
  // rows are kept only in the buffers they were built in
  const std::array<const void*, 9> bufs{L0.a64.p, mixed ? L0.a32.p : nullptr, L0.dinv64.p,
                                        mixed ? L0.dinv32.p : nullptr, rhs.p, asm_pol.p, asm_dinv.p, st64, st32};
  if (asm_stale || asm_mixed != mixed || bufs != asm_bufs) {
    asm_stale = true;
    fill_async(asm_pol.p, -1, (size_t)std::max(N0, 1), stream);
  }
  asm_mixed = mixed;
  asm_bufs = bufs;
  launch_gather_v(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_active.p, sol.p, stream);
  launch_assemble(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_active.p, L0.a64.p,
                  mixed ? L0.a32.p : nullptr, rhs.p, L0.dinv64.p, mixed ? L0.dinv32.p : nullptr, asm_pol.p,
                  asm_dinv.p, st64, st32, L0.st_w, N0, fold, stream);
  asm_stale = false;
  launch_fold_finish(fold, G, 1, 0u, 0, d_bnorm.p, 1, nullptr, 0, stream);
  (void)run;
}

// ---- lanes per sparse row (a speed choice only: the cycle kernels' row sums
// are the same bit for bit for every lane count)
namespace {
std::mutex g_tune_mu;
std::map<std::array<int, 3>, int> g_tuned;  // (value bytes, log2 rows, 4 log2 entries per row) -> lanes
int g_forced = 0;
constexpr int64_t kTuneMinNnz = 1 << 18;    // smaller levels take the rule (timing noise)
// the timed sweeps start from cold caches, as in a V-cycle where the other
// levels pass through between two sweeps of a level: a buffer larger than the
// last-level cache is written before each (one per device, kept for the
// process)
constexpr size_t kFlushDoubles = size_t(36) << 20;  // 288 MiB
std::map<int, double*> g_flush;
double* flush_buffer() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  auto it = g_flush.find(dev);
  if (it != g_flush.end()) return it->second;
  double* p = nullptr;
  if (hipMalloc(&p, kFlushDoubles * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  g_flush[dev] = p;
  return p;
}
}  // namespace

void set_forced_lanes(int lanes) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_forced = lanes;
}
int forced_lanes() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_forced;
}

int Engine::tune_lanes(Level& L, bool mixed) {
  const int n = L.n;
  const double avg = (double)L.nnz / std::max(n, 1);
  const int forced = forced_lanes();
  if (forced) return forced;
  const int rule = row_group(avg);
  if ((int64_t)L.nnz < kTuneMinNnz || L.ntiles == 0) return rule;
  const std::array<int, 3> key{mixed ? 4 : 8, (int)std::floor(std::log2((double)n)),
                               (int)std::floor(4.0 * std::log2(std::max(avg, 1.0)))};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return it->second;
  }
  // per candidate, the level's kernels of one V-cycle visit: the fused first
  // two sweeps, a plain sweep and the residual (inputs: any finite vectors of
  // the level; outputs to scratch), best of three after a first run
  s_tune.ensure(2 * (size_t)std::max(n, 1));
  s_ones.ensure(std::max(G, 1));
  fill_async(s_ones.p, 1, (size_t)std::max(G, 1), stream);
  double* flush;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    flush = flush_buffer();
  }
  hipEvent_t e0, e1;  // timing only: no system-scope fence
  SHP_HIP(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  SHP_HIP(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  int best = rule;
  float best_ms = INFINITY;
  for (int g : {1, 2, 4}) {
    float ms_min = INFINITY;
    for (int rep = 0; rep < 4; ++rep) {
      if (flush) fill_async(flush, 0.0, kFlushDoubles, stream);
      SHP_HIP(hipEventRecord(e0, stream));
      if (mixed) {
        float* o1 = reinterpret_cast<float*>(s_tune.p);
        float* o2 = o1 + std::max(n, 1);
        cyc_smooth<float>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a32.p, L.dinv32.p, L.dinv32.p, nullptr,
                          o1, 0.8f, 2, g, stream, nullptr);
        cyc_smooth<float>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a32.p, L.dinv32.p, L.dinv32.p, o1, o2,
                          0.8f, 0, g, stream, nullptr);
        cyc_resid<float>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a32.p, L.dinv32.p, o2, o1, g, stream);
      } else {
        double* o1 = s_tune.p;
        double* o2 = o1 + std::max(n, 1);
        cyc_smooth<double>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a64.p, L.dinv64.p, L.dinv64.p, nullptr,
                           o1, 0.8, 2, g, stream, nullptr);
        cyc_smooth<double>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a64.p, L.dinv64.p, L.dinv64.p, o1, o2,
                           0.8, 0, g, stream, nullptr);
        cyc_resid<double>(L.tiles.p, L.ntiles, s_ones.p, L.rp.p, L.ci.p, L.a64.p, L.dinv64.p, o2, o1, g, stream);
      }
      SHP_HIP(hipEventRecord(e1, stream));
      SHP_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SHP_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ms_min = std::min(ms_min, ms);  // the first run also loads the code
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = g;
    }
  }
  SHP_HIP(hipEventDestroy(e0));
  SHP_HIP(hipEventDestroy(e1));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[key] = best;
  return best;
}

// The Galerkin product's scratch rows are addressed by 32-bit offsets (an
// exclusive scan of per-row bounds): a level whose bound total could pass
// 2^31 is refused before any launch instead of wrapping around.
static void check_offsets(size_t total_bound) {
  if (total_bound > (size_t)INT32_MAX)
    throw Error(SHAPLEY_ENOMEM, "a merged AMG level is too large for one Galerkin product (bound " +
                                    std::to_string(total_bound) + " entries > 2^31): solve fewer games together");
}

constexpr int kRelLevels = 72;  // > the most levels a hierarchy takes

void Engine::setup(const std::vector<int>& run, const EngineOpts& o) {
  const bool mixed = o.precision == SHAPLEY_MIXED;
  std::vector<char> present(G, 0);
  for (int g : run) present[g] = 1;
  double theta = o.theta;
  if (theta <= 0) {
    int dim = 0;
    for (int g : run) dim = std::max(dim, slots[g]->g->dim);
    theta = dim >= 3 ? 0.3 : 0.25;
  }
  s_err.ensure(4);
  s_left.ensure(3);
  fill_async(s_err.p, 0, 4, stream);
  s_rel.ensure(kRelLevels);
  fill_async(s_rel.p, 0, (size_t)kRelLevels, stream);
  PhaseTimer pt(this, prof);
  nlev = 0;
  int l = 0;
  double growth = 2.6;  // entries per coarse row / per fine row of the last product
  lv[0].goff = x_off;
  lv[0].present = present;
  while (true) {
    Level& L = lv[l];
    const int n = L.n;
    L.gA = row_group((double)L.nnz / std::max(n, 1));  // tuned below once the level is complete
    L.gR = 1;
    L.apf = false;
    L.drap = false;
    L.cont.assign(G, 0);
    bool any_cont = false;
    for (int g = 0; g < G; ++g) {
      if (!L.present[g]) continue;
      int ng = L.goff[g + 1] - L.goff[g];
      if (ng > o.coarse_max && l + 1 < (int)lv.size() && l + 1 < o.max_levels) {
        L.cont[g] = 1;
        any_cont = true;
      }
    }
    if (l > 0) {
      L.dinv64.ensure(std::max(n, 1));
      if (mixed) L.dinv32.ensure(std::max(n, 1));
      if (mixed) {
        L.a32.ensure(std::max(L.nnz, 1));
        amg_cast(L.a64.p, L.a32.p, L.nnz, stream);
      }
    }
    build_tiles(L, L.present, false);
    // the cycle kernels' columns as 16-bit offsets from the row where they fit
    L.rel16 = false;
    L.rel16_built = !L.stencil && L.ntiles && g_stencil_mode.load() != 0;
    if (L.rel16_built) {
      L.ci16.ensure(std::max(L.nnz, 1));
      amg_rel16(L.tiles.p, L.ntiles, L.rp.p, L.ci.p, L.ci16.p, s_rel.p + l, stream);
    }
    L.dir.ensure(std::max(n, 1));
    if (any_cont) {
      build_tiles(L, L.cont, true);
      L.strong.ensure(std::max(L.nnz, 1));
      L.lam.ensure(n + 1);
      L.cf.ensure(std::max(n, 1));
      L.key.ensure(std::max(n, 1));
      L.cidx.ensure(n + 1);
      L.tmp.ensure(n + 1);
      // cf = -2 on rows of terminal games, which no tile covers
      amg_level_init(n, L.nnz, L.lam.p, L.cf.p, L.dir.p, L.strong.p, stream);
    }
    // 1/a_ii (level 0: the assembly's), Dirichlet flags, and Dirichlet rows
    // relaxed exactly (unit weight), in one pass
    amg_diag_dir(L.tiles.p, L.ntiles, L.rp.p, L.ci.p, L.a64.p, l == 0, 1.0 / o.omega, L.dir.p, L.dinv64.p,
                 mixed ? L.dinv32.p : nullptr, L.gA, stream);
    L.gA = tune_lanes(L, mixed);
    pt.mark("diag+tiles");
    if (any_cont) {
      // ---- strength of connection: a thread, four lanes or a wavefront per row
      const bool wide_rows = (long long)L.nnz > (long long)kApRowLen * n;
      const int slanes = wide_rows ? 64 : row_group((double)L.nnz / std::max(n, 1));
      amg_strength(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.a64.p, L.dir.p, theta, L.strong.p, L.lam.p, slanes,
                   stream);
      // transpose of the strength pattern
      L.st_rp.ensure(n + 1);
      scan_exclusive(L.lam.p, L.st_rp.p, n + 1, stream, s_scan);
      L.st_ci.ensure(std::max(L.nnz, 1));  // strong entries never exceed the entries of A
      s_cursor.ensure(n + 1);
      fill_async(s_cursor.p, 0, (size_t)n + 1, stream);
      amg_strength_t(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.strong.p, L.st_rp.p, s_cursor.p, L.st_ci.p, slanes,
                     stream);
      pt.mark("strength");
      // ---- PMIS
      s_goff.ensure(G + 1);
      up(s_goff.p, L.goff.data(), G + 1);
      uint32_t salt = mix32(0x9E3779B9u * (uint32_t)(l + 1) + 12345u);
      amg_pmis_init(L.ctiles.p, L.nctiles, s_goff.p, L.dir.p, L.lam.p, salt, L.cf.p, L.key.p, stream);
      s_newc.ensure(std::max(n, 1));
      // rounds are queued in bursts; the undecided count is checked with the
      // coarse numbering below (rounds after the last undecided row do nothing)
      int round = 0;
      // PMIS rounds take a wavefront per row only where one thread per row
      // would leave the chip mostly idle (long rows, few of them)
      const bool wide_pmis = wide_rows && n < (1 << 17);
      auto pmis_rounds = [&](int k) {
        for (int rr = 0; rr < k; ++rr, ++round) {
          amg_pmis_select(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.strong.p, L.st_rp.p, L.st_ci.p, L.cf.p,
                          L.key.p, s_newc.p, s_left.p, round, wide_pmis, stream);
          amg_pmis_update(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.strong.p, L.cf.p, s_newc.p, s_left.p, round,
                          wide_pmis, stream);
        }
      };
      // as many rounds as this level needed last time, plus one; a small
      // level runs all its rounds in one workgroup (counted as one round:
      // left[0] then holds the points still undecided)
      if ((int)pmis_need.size() <= l) pmis_need.resize(l + 1, 5);
      fill_async(s_left.p + 2, INT_MAX, 1, stream);
      if (L.nctiles * kTileRows <= kPmisSmallRows) {
        amg_pmis_small(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.strong.p, L.st_rp.p, L.st_ci.p, L.cf.p, L.key.p,
                       s_newc.p, s_left.p, 64, stream);
        round = 1;
      } else {
        pmis_rounds(std::max(2, std::min(pmis_need[l] + 1, 12)));
      }
      pt.mark("pmis");
      // ---- coarse numbering and per-game coarse sizes
      auto number = [&](std::vector<int>& ncg) {
        while (true) {
          amg_is_c(L.cf.p, L.tmp.p, n, stream);
          scan_exclusive(L.tmp.p, L.cidx.p, n + 1, stream, s_scan);
          s_gout.ensure(G + 1);
          amg_gather_int(L.cidx.p, s_goff.p, G + 1, s_gout.p, stream);
          std::vector<int> cpre(G + 1);
          const int* cp = down(s_gout.p, G + 1);
          const int* left = down(s_left.p, 3);
          sync();
          if (left[(round - 1) & 1] != 0) {  // PMIS not finished: more rounds, then number again
            if (round >= 1000) throw Error(SHAPLEY_EDEVICE, "PMIS did not terminate");
            pmis_rounds(4);
            continue;
          }
          // rounds that did work: up to the first idle one, or all of them
          pmis_need[l] = left[2] < round ? left[2] : round;
          cpre.assign(cp, cp + G + 1);
          ncg.assign(G, 0);
          for (int g = 0; g < G; ++g) ncg[g] = cpre[g + 1] - cpre[g];
          return cpre;
        }
      };
      std::vector<int> ncg;
      std::vector<int> cpre = number(ncg);
      bool changed = false;
      for (int g = 0; g < G; ++g) {
        if (!L.cont[g]) continue;
        int ng = L.goff[g + 1] - L.goff[g];
        // coarsening stalled: small blocks end here with a dense solve.
        // A block without any coarse point (only Dirichlet or weakly coupled
        // rows, e.g. the identity of "stop everywhere") stays on this level
        // and is handled by the smoother alone, which solves such rows.
        if (ncg[g] > 0 && ncg[g] > 0.9 * ng && ng <= kDenseMax) {
          L.cont[g] = 0;
          changed = true;
        }
      }
      if (changed) {
        std::vector<char> term(G, 0);
        for (int g = 0; g < G; ++g) term[g] = L.present[g] && !L.cont[g];
        std::vector<Tile> tt = make_tiles(L.goff, term, kTileRows);
        s_tiles.ensure(std::max<size_t>(tt.size(), 1));
        up(s_tiles.p, tt.data(), tt.size());
        amg_fill_cf(s_tiles.p, (int)tt.size(), L.cf.p, (int8_t)-2, stream);
        any_cont = false;
        for (int g = 0; g < G; ++g) any_cont |= (bool)L.cont[g];
        build_tiles(L, L.cont, true);
        cpre = number(ncg);
      }
      if (any_cont) {
        const int nc = cpre[G];
        L.nc = nc;
        // ---- interpolation
        L.pc.ensure((size_t)std::max(n, 1) * PW);
        L.pv64.ensure((size_t)std::max(n, 1) * PW);
        // s_err[0]: interpolatory sets truncated, [1]: Galerkin product flags, [2]: singular block
        probe_begin(kProbeInterp, stream);
        // level 0 (grid stencils, short rows): one thread per row; coarse
        // levels (long rows): one wavefront per row, with the larger LDS sets
        // where rows average more than 32 entries
        // (four lanes per row take a row through a longer chain than a
        // wavefront does: only levels with rows enough to fill the chip, and
        // rows averaging at most 24 entries -- measured: the 129^3 game's
        // coarse levels, longer, 42.5 -> 40.7 ms per solve with the wavefront
        // kernel; the 256-game batch unchanged)
        const int imode = g_interp_mode.load();
        const bool quad =
            imode == 4 || (imode == -1 && n >= kInterpQuadRows && (double)L.nnz <= 24.0 * std::max(n, 1));
        const int iw = l == 0 ? 0 : ((double)L.nnz > 32.0 * std::max(n, 1) ? 2 : (quad ? 3 : 1));
        s_defer.ensure(2 * ((size_t)L.rows_ctiles + 1));  // two hand-over lists
        amg_interp(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.a64.p, L.dinv64.p, L.strong.p, L.cf.p,
                   L.cidx.p, L.dir.p, L.pc.p, L.pv64.p, s_err.p, iw, s_defer.p, L.rows_ctiles, stream);
        probe_end(kProbeInterp, stream, (double)L.rows_ctiles * (PW * 12) + (double)L.nnz * 13);
        pt.mark("interp");
        // ---- next level rows
        Level& Ln = lv[l + 1];
        Ln.n = nc;
        Ln.goff.assign(G + 1, 0);
        Ln.present.assign(G, 0);
        for (int g = 0; g <= G; ++g) Ln.goff[g] = cpre[g];
        for (int g = 0; g < G; ++g) Ln.present[g] = L.cont[g] && ncg[g] > 0;
        // ---- R = P^T
        s_cnt.ensure(nc + 1);
        fill_async(s_cnt.p, 0, (size_t)nc + 1, stream);
        amg_pt_count(L.ctiles.p, L.nctiles, L.pc.p, s_cnt.p, stream);
        L.rrp.ensure(nc + 1);
        scan_exclusive(s_cnt.p, L.rrp.p, nc + 1, stream, s_scan);
        const int rnnz = n * PW;  // upper bound of the entries of P^T
        L.rci.ensure(std::max(rnnz, 1));
        L.rv64.ensure(std::max(rnnz, 1));
        s_cursor.ensure(nc + 1);
        fill_async(s_cursor.p, 0, (size_t)nc + 1, stream);
        amg_pt_fill(L.ctiles.p, L.nctiles, L.pc.p, L.pv64.p, L.rrp.p, s_cursor.p, L.rci.p, L.rv64.p, stream);
        amg_sort_rows(L.rrp.p, L.rci.p, L.rv64.p, nc, stream);
        pt.mark("transpose");
        // ---- Galerkin product.  Small next levels: dense per-game blocks.
        // Otherwise row-wise: bounds, one fused pass into scratch rows, row
        // pointers, compaction.
        Ln.rp.ensure(nc + 1);
        s_cnt.ensure(nc + 1);
        s_toff.ensure(nc + 1);
        {
          long long ap = 0, ac = 0;
          int maxc = 0;
          for (int g = 0; g < G; ++g) {
            const long long ncg = cpre[g + 1] - cpre[g];
            maxc = std::max(maxc, (int)ncg);
            ap += ncg * (L.goff[g + 1] - L.goff[g]);
            ac += ncg * ncg;
          }
          const bool small = maxc <= kDrapSmallCols && ap <= kDrapSmallEntries && ac <= kDrapSmallEntries;
          const bool dense = (long long)L.nnz >= kDrapRowLen * (long long)n &&
                             ap <= kDrapDensity * PW * (long long)L.nnz;
          L.drap = maxc <= kDrapMaxCols && ap <= kDrapMaxEntries && ac <= kDrapMaxEntries && (small || dense);
          L.drap_ap = ap;
          L.drap_maxc = maxc;
          L.drap_ac = ac;
          if (L.drap) {
            std::vector<long long>& t = L.h_drap_tab;  // kept alive for the asynchronous upload
            t.assign(4 * (size_t)(G + 1), 0);
            for (int g = 0; g <= G; ++g) {
              t[g] = L.goff[g];
              t[(G + 1) + g] = cpre[g];
            }
            for (int g = 0; g < G; ++g) {
              const long long ncg = cpre[g + 1] - cpre[g];
              t[2 * (G + 1) + g + 1] = t[2 * (G + 1) + g] + ncg * (L.goff[g + 1] - L.goff[g]);
              t[3 * (G + 1) + g + 1] = t[3 * (G + 1) + g] + ncg * ncg;
            }
            L.drap_tab.ensure(t.size());
            up(L.drap_tab.p, t.data(), t.size());
          }
        }
        // probed launches: the dense product, the single pass R A P, or each
        // pass of R (A P) (the product kernels only: bounds, scans and the
        // synchronisation between the passes left out)
        const double rap_bytes = (double)L.nnz * 12 + (double)n * PW * 12 + (double)nc * 8;
        if (L.drap) {
          probe_begin(kProbeRap, stream);
          L.dap.ensure(std::max<long long>(L.drap_ap, 1));
          s_dapt.ensure(std::max<long long>(L.drap_ap, 1));
          s_dac.ensure(std::max<long long>(L.drap_ac, 1));
          s_dacf.ensure(std::max<long long>(L.drap_ac, 1));
          amg_drap_full(n, nc, L.drap_maxc, L.drap_tab.p, G, L.drap_ac, L.rp.p, L.ci.p, L.a64.p, L.pc.p,
                        L.pv64.p, L.rrp.p, L.rci.p, L.rv64.p, L.dap.p, s_dapt.p, s_dac.p, s_dacf.p, s_cnt.p,
                        stream);
          probe_end(kProbeRap, stream, rap_bytes);
        } else {
          // the single pass R A P, or for long rows A P first and R (AP) after
          const int* Arp = L.rp.p;
          const int* Aci = L.ci.p;
          const double* Aa = L.a64.p;
          const int* Ppc = L.pc.p;
          const double* Ppv = L.pv64.p;
          int pwf = PW;                 // filled slots per row of the right operand
          size_t opnnz = (size_t)std::max(L.nnz, 1);
          L.apf = (long long)L.nnz >= (long long)kApRowLen * n;
          if (L.apf) {
            L.id_rp.ensure((size_t)n + 1);
            L.id_ci.ensure(std::max(n, 1));
            L.id_rv.ensure(std::max(n, 1));
            L.id_pc.ensure((size_t)std::max(n, 1) * PW);
            L.id_pv.ensure((size_t)std::max(n, 1) * PW);
            amg_identity_ops(n, L.id_rp.p, L.id_ci.p, L.id_rv.p, L.id_pc.p, L.id_pv.p, stream);
            s_cnt.ensure((size_t)n + 1);
            s_toff.ensure((size_t)n + 1);
            s_big.ensure(2 * ((size_t)n + 1));
            const size_t tcap1 = std::max<size_t>(
                1, std::min((size_t)PW * (size_t)std::max(L.nnz, 1), (size_t)n * (size_t)kRapMaxCols));
            check_offsets(tcap1);
            s_tcol.ensure(tcap1);
            s_tval.ensure(tcap1);
            amg_rap_bound(n, L.id_rp.p, L.id_ci.p, L.rp.p, s_cnt.p, PW, stream);
            scan_exclusive(s_cnt.p, s_toff.p, n + 1, stream, s_scan);
            probe_begin(kProbeRap, stream);
            // A P rows: the previous product's average, else about A's
            const double ap_cols = L.ap_nnz > 0 ? (double)L.ap_nnz / n : (double)L.nnz / n;
            amg_rap_fused(n, L.id_rp.p, L.id_ci.p, L.id_rv.p, L.rp.p, L.ci.p, L.a64.p, L.pc.p, L.pv64.p,
                          s_toff.p, s_cnt.p, s_tcol.p, s_tval.p, s_err.p + 1, s_big.p, stream,
                          gal_kernel(ap_cols, false));
            probe_end(kProbeRap, stream, (double)L.nnz * 12 + (double)n * PW * 12);
            L.ap_rp.ensure((size_t)n + 1);
            scan_exclusive(s_cnt.p, L.ap_rp.p, n + 1, stream, s_scan);
            const int* pap = down(L.ap_rp.p + n, 1);
            sync();
            L.ap_nnz = *pap;
            probe_add_bytes(kProbeRap, (double)L.ap_nnz * 12);  // A P written by that pass
            L.ap_ci.ensure(std::max(L.ap_nnz, 1));
            L.ap_v.ensure(std::max(L.ap_nnz, 1));
            amg_rap_compact(n, s_toff.p, s_tcol.p, s_tval.p, L.ap_rp.p, L.ap_ci.p, L.ap_v.p, stream);
            Arp = L.ap_rp.p;
            Aci = L.ap_ci.p;
            Aa = L.ap_v.p;
            Ppc = L.id_pc.p;
            Ppv = L.id_pv.p;
            pwf = 1;
            opnnz = (size_t)std::max(L.ap_nnz, 1);
          }
          // sum of the bounds <= pwf * (pairs) <= pwf * PW * nnz(operand)
          const size_t tcap = std::max<size_t>(
              1, std::min((size_t)pwf * PW * opnnz, (size_t)nc * (size_t)kRapMaxCols));
          check_offsets(tcap);
          s_tcol.ensure(tcap);
          s_tval.ensure(tcap);
          s_big.ensure(2 * ((size_t)std::max(n, nc) + 1));
          amg_rap_bound(nc, L.rrp.p, L.rci.p, Arp, s_cnt.p, pwf, stream);
          // coarse rows: the level's previous product, else the fine rows'
          // entries times the growth of the level above (2.6 on level 0: grid
          // stencils)
          const double c_cols =
              (Ln.nnz > 0 && Ln.n == nc) ? (double)Ln.nnz / nc : growth * L.nnz / std::max(n, 1);
          scan_exclusive(s_cnt.p, s_toff.p, nc + 1, stream, s_scan);
          probe_begin(kProbeRap, stream);
          amg_rap_fused(nc, L.rrp.p, L.rci.p, L.rv64.p, Arp, Aci, Aa, Ppc, Ppv, s_toff.p, s_cnt.p, s_tcol.p,
                        s_tval.p, s_err.p + 1, s_big.p, stream, gal_kernel(c_cols, L.apf));
          probe_end(kProbeRap, stream, L.apf ? (double)L.ap_nnz * 12 + (double)nc * 8 : rap_bytes);
        }
        scan_exclusive(s_cnt.p, Ln.rp.p, nc + 1, stream, s_scan);
        int cnnz = 0, rnnz_used = 0;
        const int* pc_nnz = down(Ln.rp.p + nc, 1);
        const int* pr_nnz = down(L.rrp.p + nc, 1);
        sync();
        cnnz = *pc_nnz;
        rnnz_used = *pr_nnz;
        Ln.nnz = cnnz;
        if (L.nnz > 0 && nc > 0) growth = ((double)cnnz / nc) / ((double)L.nnz / std::max(n, 1));
        L.gR = forced_lanes() ? forced_lanes() : row_group((double)rnnz_used / std::max(nc, 1));
        Ln.ci.ensure(std::max(cnnz, 1));
        Ln.a64.ensure(std::max(cnnz, 1));
        if (L.drap)
          amg_drap_compact(nc, L.drap_tab.p, G, s_dac.p, s_dacf.p, Ln.rp.p, Ln.ci.p, Ln.a64.p, stream);
        else
          amg_rap_compact(nc, s_toff.p, s_tcol.p, s_tval.p, Ln.rp.p, Ln.ci.p, Ln.a64.p, stream);
        if (mixed) {
          L.pv32.ensure((size_t)std::max(n, 1) * PW);
          amg_cast(L.pv64.p, L.pv32.p, (size_t)n * PW, stream);
          L.rv32.ensure(std::max(rnnz, 1));
          amg_cast(L.rv64.p, L.rv32.p, rnnz, stream);
        }
        pt.mark("rap");
      }
    }
    // ---- dense inverses of the games that end at this level
    std::vector<int>& hblk = L.h_blk;  // kept alive for the asynchronous upload
    hblk.clear();
    size_t doff = 0;
    L.max_blk = 0;
    for (int g = 0; g < G; ++g) {
      if (!L.present[g] || L.cont[g]) continue;
      int nb = L.goff[g + 1] - L.goff[g];
      if (nb == 0) continue;
      if (nb > kDenseMax) throw Error(SHAPLEY_ENOCONV, "coarsest block exceeds the dense-solve limit");
      hblk.insert(hblk.end(), {L.goff[g], nb, (int)doff, g});
      doff += (size_t)nb * nb;
      L.max_blk = std::max(L.max_blk, nb);
    }
    L.nblk = (int)hblk.size() / 4;
    if (L.nblk) {
      L.blk.ensure(hblk.size());
      up(L.blk.p, hblk.data(), hblk.size());
      L.dmat64.ensure(doff);
      if (mixed) L.dmat32.ensure(doff);
      const bool large = L.max_blk > kDenseWave;
      if (large) s_dense.ensure(2 * doff);
      amg_dense_inv(L.blk.p, L.nblk, L.rp.p, L.ci.p, L.a64.p, s_dense.p, L.dmat64.p,
                    mixed ? L.dmat32.p : nullptr, s_err.p + 2, L.max_blk, stream);
      pt.mark("dense");
    }
    // cycle vectors
    if (mixed) {
      L.x32.ensure(std::max(n, 1)); L.y32.ensure(std::max(n, 1));
      L.b32.ensure(std::max(n, 1)); L.r32.ensure(std::max(n, 1));
    } else {
      L.x64.ensure(std::max(n, 1)); L.y64.ensure(std::max(n, 1));
      L.b64.ensure(std::max(n, 1)); L.r64.ensure(std::max(n, 1));
    }
    pt.mark("vectors");
    if (o.verbose >= 2) {
      int ncont = 0, nterm = 0;
      for (int g = 0; g < G; ++g) { ncont += L.cont[g]; nterm += L.present[g] && !L.cont[g]; }
      fprintf(stderr, "[shapley amg] level %d n %d nnz %d nc %d cont %d term %d blocks %d max_blk %d\n", l, n,
              L.nnz, any_cont ? L.nc : 0, ncont, nterm, L.nblk, L.max_blk);
    }
    if (!any_cont) {
      L.nctiles = 0;
      nlev = l + 1;
      break;
    }
    ++l;
  }
  {
    int herr[4] = {0, 0, 0, 0};
    const int* pe = down(s_err.p, 4);
    const int* pr = down(s_rel.p, (size_t)kRelLevels);
    sync();
    std::memcpy(herr, pe, sizeof(herr));
    for (int k = 0; k < nlev; ++k) lv[k].rel16 = lv[k].rel16_built && pr[k] == 0;
    if (herr[1] != 0)
      throw Error(SHAPLEY_EDEVICE, "Galerkin product: coarse row too long (code " + std::to_string(herr[1]) + ")");
    if (herr[2] != 0) throw Error(SHAPLEY_EDEVICE, "singular coarsest block");
  }
  // the tail kernel runs V-cycles with (weighted or l1) Jacobi sweeps; W-cycles
  // and C/F relaxation take every level level by level
  build_tail(mixed, o.gamma == 1 && o.smoother != SHAPLEY_SMOOTH_CF);
  hier_game = G == 1 ? slots[0]->g : nullptr;
  // statistics
  double nnz_sum = 0, n_sum = 0;
  for (int k = 0; k < nlev; ++k) { nnz_sum += lv[k].nnz; n_sum += lv[k].n; }
  for (int g : run) {
    slots[g]->levels = nlev;
    slots[g]->opc = lv[0].nnz ? nnz_sum / lv[0].nnz : 1.0;
    slots[g]->gc = lv[0].n ? n_sum / lv[0].n : 1.0;
  }
}

// Splits every level between the level-by-level cycle and the per-game tails
// (a game's tail starts on its first level with at most kTailRows rows) and
// uploads the tail tables.  Pointers stay valid through numeric refreshes.
void Engine::build_tail(bool mixed, bool allow) {
  const int cap = kTailLdsBytes / (2 * (mixed ? (int)sizeof(float) : (int)sizeof(double)));
  h_lt.assign(G, nlev);
  std::vector<int> lds_rows(std::max(nlev, 1), 0);
  for (int g = 0; g < G && allow; ++g) {
    int last = -1;  // the game's last level
    for (int l = 0; l < nlev && lv[l].present[g]; ++l) {
      last = l;
      if (!lv[l].cont[g]) break;
    }
    // rows of the game summed over levels l..last, and their largest level
    std::vector<long> cum(last + 2, 0), big(last + 2, 0);
    for (int l = last; l >= 0; --l) {
      const long rows = lv[l].goff[g + 1] - lv[l].goff[g];
      cum[l] = cum[l + 1] + rows;
      big[l] = std::max(big[l + 1], rows);
    }
    for (int l = 0; l <= last; ++l) {
      // the tail start level's entries (estimated from the level's average row)
      const double est_nnz = lv[l].n ? (double)lv[l].nnz * (lv[l].goff[g + 1] - lv[l].goff[g]) / lv[l].n : 0.0;
      if (big[l] <= kTailRows && cum[l] <= cap && est_nnz <= kTailNnz && last - l < kTailMaxLevels) {
        h_lt[g] = l;
        lds_rows[l] = std::max(lds_rows[l], (int)cum[l]);
        break;
      }
    }
  }
  // host image of the tables, each at a 256-byte aligned offset
  std::vector<char>& hpack = h_tailpack;
  hpack.clear();
  auto pack = [&](const auto* data, size_t n) -> size_t {
    const size_t o = (hpack.size() + 255) & ~(size_t)255;
    const size_t bytes = sizeof(*data) * n;
    hpack.resize(o + std::max<size_t>(bytes, 1), 0);
    if (bytes) std::memcpy(hpack.data() + o, data, bytes);
    return o;
  };
  std::vector<std::array<size_t, 4>> off(std::max(nlev, 1));
  std::vector<TailGL> gl((size_t)std::max(nlev, 1) * std::max(G, 1), TailGL{0, 0, 0, 0});
  std::vector<TailLev<double>> t64(std::max(nlev, 1));
  std::vector<TailLev<float>> t32(std::max(nlev, 1));
  for (int l = 0; l < nlev; ++l) {
    Level& L = lv[l];
    std::vector<int> doff(G, -1);
    for (size_t k = 0; k + 3 < L.h_blk.size(); k += 4) doff[L.h_blk[k + 3]] = L.h_blk[k + 2];
    std::vector<char> keepv(G, 0), keepr(G, 0);
    L.h_vblk.clear();
    L.h_tailg.clear();
    for (int g = 0; g < G; ++g) {
      if (!L.present[g]) continue;
      TailGL& q = gl[(size_t)l * G + g];
      q.r0 = L.goff[g];
      q.r1 = L.goff[g + 1];
      q.flags = kTailPresent | (L.cont[g] ? kTailCont : 0);
      if (doff[g] >= 0) {
        q.flags |= kTailDense;
        q.doff = doff[g];
      }
      if (l + 1 < nlev && lv[l + 1].present[g]) q.flags |= kTailNext;
      keepv[g] = L.cont[g] && h_lt[g] > l;
      keepr[g] = l > 0 && h_lt[g] > l - 1;
      if (h_lt[g] == l) L.h_tailg.push_back(g);
    }
    for (size_t k = 0; k + 3 < L.h_blk.size(); k += 4)
      if (h_lt[L.h_blk[k + 3]] > l) L.h_vblk.insert(L.h_vblk.end(), L.h_blk.begin() + k, L.h_blk.begin() + k + 4);
    auto tiles_of = [&](std::vector<Tile>& h, int& nt, int& rows, const std::vector<char>& keep) {
      h = make_tiles(L.goff, keep, kTileRows);
      nt = (int)h.size();
      rows = 0;
      for (const Tile& x : h) rows += x.r1 - x.r0;
    };
    tiles_of(L.h_vctiles, L.nvctiles, L.rows_vctiles, keepv);
    tiles_of(L.h_rtiles, L.nrtiles, L.rows_rtiles, keepr);
    off[l][0] = pack(L.h_vctiles.data(), L.h_vctiles.size());
    off[l][1] = pack(L.h_rtiles.data(), L.h_rtiles.size());
    off[l][2] = pack(L.h_vblk.data(), L.h_vblk.size());
    off[l][3] = pack(L.h_tailg.data(), L.h_tailg.size());
    L.nvblk = (int)L.h_vblk.size() / 4;
    L.ntailg = (int)L.h_tailg.size();
    L.tail_lds_rows = lds_rows[l];
    L.upper = L.nvctiles > 0 || L.nvblk > 0;
    if (mixed)
      t32[l] = TailLev<float>{L.rp.p, L.ci.p, L.a32.p, L.dinv32.p, L.x32.p, L.y32.p, L.b32.p, L.r32.p,
                              L.rrp.p, L.rci.p, L.rv32.p, L.pc.p, L.pv32.p, L.dmat32.p};
    else
      t64[l] = TailLev<double>{L.rp.p, L.ci.p, L.a64.p, L.dinv64.p, L.x64.p, L.y64.p, L.b64.p, L.r64.p,
                               L.rrp.p, L.rci.p, L.rv64.p, L.pc.p, L.pv64.p, L.dmat64.p};
  }
  const size_t o_gl = pack(gl.data(), gl.size());
  const size_t o_t = mixed ? pack(t32.data(), t32.size()) : pack(t64.data(), t64.size());
  // one upload of all tables
  d_tailpack.ensure(std::max<size_t>(hpack.size(), 1));
  up(d_tailpack.p, hpack.data(), hpack.size());
  char* base = d_tailpack.p;
  for (int l = 0; l < nlev; ++l) {
    Level& L = lv[l];
    L.vctiles.p = reinterpret_cast<Tile*>(base + off[l][0]);
    L.rtiles.p = reinterpret_cast<Tile*>(base + off[l][1]);
    L.vblk.p = reinterpret_cast<int*>(base + off[l][2]);
    L.tailg.p = reinterpret_cast<int*>(base + off[l][3]);
  }
  d_tailgl.p = reinterpret_cast<TailGL*>(base + o_gl);
  d_tail32.p = mixed ? reinterpret_cast<TailLev<float>*>(base + o_t) : nullptr;
  d_tail64.p = mixed ? nullptr : reinterpret_cast<TailLev<double>*>(base + o_t);
}

// Numeric refresh of the last hierarchy: the C/F splitting, P and R = P^T
// are kept and only the Galerkin products A_{l+1} = R A_l P, the diagonals,
// the FP32 copies and the dense coarsest inverses are recomputed from the
// freshly assembled level-0 matrix (whose sparsity pattern does not depend on
// the policies).
void Engine::refresh(const EngineOpts& o) {
  const bool mixed = o.precision == SHAPLEY_MIXED;
  PhaseTimer pt(this, prof);
  fill_async(s_err.p, 0, 4, stream);
  {
    Level& L0 = lv[0];
    L0.chg.ensure(std::max(L0.n, 1));
    amg_row_changed(L0.tiles.p, L0.ntiles, L0.rp.p, L0.a64.p, L0.a_prev.p, L0.chg.p, stream);
  }
  for (int l = 0; l < nlev; ++l) {
    Level& L = lv[l];
    const int n = L.n;
    if (l > 0 && mixed) amg_cast(L.a64.p, L.a32.p, L.nnz, stream);
    if (L.nctiles) {
      // relaxation data of the smoothed rows (level 0 keeps the assembled
      // diagonal); rows of games that end here use the dense inverse instead
      // level 0's diagonals were rewritten by the assembly; a coarse level's
      // change only in the rows its Galerkin product recomputes
      amg_diag_dir(L.ctiles.p, L.nctiles, L.rp.p, L.ci.p, L.a64.p, l == 0, 1.0 / o.omega, L.dir.p, L.dinv64.p,
                   mixed ? L.dinv32.p : nullptr, L.gA, stream, l == 0 ? nullptr : L.chg.p);
      Level& Ln = lv[l + 1];
      Ln.chg.ensure(std::max(L.nc, 1));
      fill_async(Ln.chg.p, (uint8_t)0, (size_t)std::max(L.nc, 1), stream);
      amg_mark_coarse(L.ctiles.p, L.nctiles, L.pc.p, L.chg.p, Ln.chg.p, stream);
      if (L.drap) {
        probe_begin(kProbeRap, stream);
        // the A P rows of the changed fine rows, then the coarse rows they reach
        amg_drap_known(L.n, L.nc, L.drap_maxc, L.drap_tab.p, G, L.rp.p, L.ci.p, L.a64.p, L.pc.p, L.pv64.p,
                       L.rrp.p, L.rci.p, L.rv64.p, L.dap.p, Ln.rp.p, Ln.ci.p, Ln.a64.p, stream, Ln.chg.p, L.chg.p);
        probe_end(kProbeRap, stream, 0.0);  // a refresh recomputes the changed rows only: no bytes claimed
      } else if (L.apf) {
        // A P rows of the changed fine rows, then the coarse rows they reach
        s_big.ensure(2 * ((size_t)std::max(n, L.nc) + 1));
        probe_begin(kProbeRap, stream);
        s_list.ensure((size_t)n + 1);
        amg_rap_known(n, L.id_rp.p, L.id_ci.p, L.id_rv.p, L.rp.p, L.ci.p, L.a64.p, L.pc.p, L.pv64.p, L.ap_rp.p,
                      L.ap_ci.p, L.ap_v.p, s_err.p + 1, s_big.p, stream, L.chg.p, s_list.p,
                      gal_kernel((double)L.ap_nnz / std::max(n, 1), false));
        probe_end(kProbeRap, stream, 0.0);  // a refresh recomputes the changed rows only: no bytes claimed
        probe_begin(kProbeRap, stream);
        s_list.ensure((size_t)L.nc + 1);
        amg_rap_known(L.nc, L.rrp.p, L.rci.p, L.rv64.p, L.ap_rp.p, L.ap_ci.p, L.ap_v.p, L.id_pc.p, L.id_pv.p,
                      Ln.rp.p, Ln.ci.p, Ln.a64.p, s_err.p + 1, s_big.p, stream, Ln.chg.p, s_list.p,
                      gal_kernel((double)Ln.nnz / std::max(L.nc, 1), true));
        probe_end(kProbeRap, stream, 0.0);  // a refresh recomputes the changed rows only: no bytes claimed
      } else {
        s_big.ensure(2 * ((size_t)L.nc + 1));
        s_list.ensure((size_t)L.nc + 1);
        probe_begin(kProbeRap, stream);
        amg_rap_known(L.nc, L.rrp.p, L.rci.p, L.rv64.p, L.rp.p, L.ci.p, L.a64.p, L.pc.p, L.pv64.p, Ln.rp.p,
                      Ln.ci.p, Ln.a64.p, s_err.p + 1, s_big.p, stream, Ln.chg.p, s_list.p,
                      gal_kernel((double)Ln.nnz / std::max(L.nc, 1), false));
        probe_end(kProbeRap, stream, 0.0);  // a refresh recomputes the changed rows only: no bytes claimed
      }
    }
    if (L.nblk)
      amg_dense_inv(L.blk.p, L.nblk, L.rp.p, L.ci.p, L.a64.p, s_dense.p, L.dmat64.p, mixed ? L.dmat32.p : nullptr,
                    s_err.p + 2, L.max_blk, stream, L.chg.p);
  }
  // the error flags are read with the linear solve's first synchronisation
  // (no synchronisation of its own)
  err_pending = true;
  pt.mark("refresh");
}

// Error flags of a refresh, downloaded with a transfer of the caller's and
// checked after its synchronisation.
const int* Engine::refresh_errors_down() { return err_pending ? down(s_err.p, 4) : nullptr; }
void Engine::refresh_errors_check(const int* pe) {
  if (!pe) return;
  err_pending = false;
  if (pe[1] != 0) throw Error(SHAPLEY_EDEVICE, "Galerkin product failed during refresh");
  if (pe[2] != 0) throw Error(SHAPLEY_EDEVICE, "singular coarsest block");
}

// algorithmic bytes of the cycle kernels (each value read or written once)
// (the stencil form: per row a code word and st_w slot values, no columns)
template <class T>
static double bytes_smooth(const Level& L, bool first) {
  const double sv = sizeof(T), rows = L.rows_vctiles;
  if (first) return rows * 3 * sv;
  const double nnz = L.n ? (double)L.nnz * rows / L.n : 0.0;
  return rows * (4 + 4 * sv) + (L.stencil ? rows * L.st_w * sv : nnz * ((L.rel16 ? 2 : 4) + sv));
}
template <class T>
static double bytes_resid(const Level& L) {
  const double sv = sizeof(T), rows = L.rows_vctiles;
  const double nnz = L.n ? (double)L.nnz * rows / L.n : 0.0;
  return rows * (4 + 3 * sv) + (L.stencil ? rows * L.st_w * sv : nnz * ((L.rel16 ? 2 : 4) + sv));
}

template <class T>
static T* vcycle_level(Engine* e, std::vector<Level>& lv, int l, const EngineOpts& o, const int* act,
                       hipStream_t s, double* sol, const TailRefine* rf = nullptr, T* start = nullptr);

// weight of the relaxation: l1-Jacobi takes none
static double relax_weight(const EngineOpts& o) { return o.smoother == SHAPLEY_SMOOTH_L1 ? 1.0 : o.omega; }

// One relaxation sweep cur -> nxt of the level-by-level rows (a C/F sweep is
// two half sweeps through the free buffer, ending in nxt).
static const int16_t* ci16_of(const Level& L) { return L.rel16 ? L.ci16.p : nullptr; }

static StencilView stencil_view(const Level& L, const int* st_off) {
  return StencilView{L.st_code.p, st_off, L.st_w, L.n};
}

template <class T>
static void relax_sweep(Level& L, const EngineOpts& o, const int* act, const T* b, T* cur, T* nxt, T* tmp,
                        hipStream_t s, double* sol, const int* st_off) {
  const T om = (T)relax_weight(o);
  if (o.smoother == SHAPLEY_SMOOTH_CF) {
    probe_begin(kProbeSmooth, s);
    cyc_smooth<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, LV<T>::a(L), LV<T>::d(L), b, cur, tmp, om, 0, L.gA,
                  s, nullptr, L.cf.p, 1, ci16_of(L));
    cyc_smooth<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, LV<T>::a(L), LV<T>::d(L), b, tmp, nxt, om, 0, L.gA,
                  s, nullptr, L.cf.p, -1, ci16_of(L));
    probe_end(kProbeSmooth, s, 2 * bytes_smooth<T>(L, false));
    return;
  }
  probe_begin(kProbeSmooth, s);
  if (L.stencil)
    cyc_smooth_st<T>(L.vctiles.p, L.nvctiles, act, stencil_view(L, st_off), LV<T>::st(L), LV<T>::d(L), b, cur, nxt,
                     om, 0, s, sol);
  else
    cyc_smooth<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, LV<T>::a(L), LV<T>::d(L), b, cur, nxt, om, 0, L.gA,
                  s, sol, nullptr, 0, ci16_of(L));
  probe_end(kProbeSmooth, s, bytes_smooth<T>(L, false));
}

// Level-by-level part of the multigrid cycle on level l (Algorithm MGcycle):
// the games whose tail starts deeper.  The iterate starts from zero, or from
// `start` (one of the level's x and y buffers: a W-cycle's second visit);
// the coarse problem is visited gamma times.  Returns the buffer (x or y)
// holding the level's result.
template <class T>
static T* vcycle_impl(Engine* e, std::vector<Level>& lv, int l, const EngineOpts& o, const int* act,
                      hipStream_t s, double* sol, T* start) {
  Level& L = lv[l];
  T* cur = start ? start : LV<T>::x(L);
  T* nxt = cur == LV<T>::x(L) ? LV<T>::y(L) : LV<T>::x(L);
  T* b = LV<T>::b(L);
  const T om = (T)relax_weight(o);
  const int* st_off = e->stencil_offsets();
  const bool cf = o.smoother == SHAPLEY_SMOOTH_CF;
  if (L.nvctiles) {
    const T* A = LV<T>::a(L);
    const T* D = LV<T>::d(L);
    T* tmp = LV<T>::r(L);  // free until the residual
    int k = 0;
    if (!start && cf) {
      fill_async(cur, (T)0, (size_t)L.n, s);
    } else if (!start && o.nu1 >= 2) {  // the first two sweeps in one pass
      probe_begin(kProbeSmooth, s);
      if (L.stencil)
        cyc_smooth_st<T>(L.vctiles.p, L.nvctiles, act, stencil_view(L, st_off), LV<T>::st(L), D, b, nullptr, nxt,
                         om, 2, s);
      else
        cyc_smooth<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, A, D, b, nullptr, nxt, om, 2, L.gA, s, nullptr,
                      nullptr, 0, ci16_of(L));
      probe_end(kProbeSmooth, s, bytes_smooth<T>(L, false) - (double)L.rows_vctiles * sizeof(T));
      std::swap(cur, nxt);
      k = 2;
    } else if (!start) {
      probe_begin(kProbeSmooth, s);
      cyc_smooth<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, A, D, b, nullptr, cur, om, 1, 1, s);
      probe_end(kProbeSmooth, s, bytes_smooth<T>(L, true));
      k = 1;
    }
    for (; k < o.nu1; ++k) {
      relax_sweep<T>(L, o, act, b, cur, nxt, tmp, s, nullptr, st_off);
      std::swap(cur, nxt);
    }
    T* r = LV<T>::r(L);
    probe_begin(kProbeResid, s);
    if (L.stencil)
      cyc_resid_st<T>(L.vctiles.p, L.nvctiles, act, stencil_view(L, st_off), LV<T>::st(L), b, cur, r, s);
    else
      cyc_resid<T>(L.vctiles.p, L.nvctiles, act, L.rp.p, L.ci.p, A, b, cur, r, L.gA, s, ci16_of(L));
    probe_end(kProbeResid, s, bytes_resid<T>(L));
    Level& Ln = lv[l + 1];
    probe_begin(kProbeRestrict, s);
    cyc_restrict<T>(Ln.rtiles.p, Ln.nrtiles, act, L.rrp.p, L.rci.p, LV<T>::rv(L), r, LV<T>::b(Ln), L.gR, s);
    probe_end(kProbeRestrict, s,
              (double)Ln.rows_rtiles * (4 + sizeof(T)) + (double)L.rows_vctiles * (4 + 2 * sizeof(T)));
    T* xc = vcycle_level<T>(e, lv, l + 1, o, act, s, nullptr);
    for (int v = 1; v < o.gamma; ++v) xc = vcycle_level<T>(e, lv, l + 1, o, act, s, nullptr, nullptr, xc);
    probe_begin(kProbeProlong, s);
    cyc_prolong<T>(L.vctiles.p, L.nvctiles, act, L.pc.p, LV<T>::pv(L), xc, cur, s);
    probe_end(kProbeProlong, s,
              (double)L.rows_vctiles * (PW * (4 + sizeof(T)) + 2 * sizeof(T)) + (double)Ln.rows_rtiles * sizeof(T));
    for (int k = 0; k < o.nu2; ++k) {
      relax_sweep<T>(L, o, act, b, cur, nxt, tmp, s, k + 1 == o.nu2 ? sol : nullptr, st_off);
      std::swap(cur, nxt);
    }
  }
  if (L.nvblk) cyc_dense<T>(L.vblk.p, L.nvblk, act, LV<T>::dm(L), b, cur, s);
  return cur;
}

// Cycle on level l: the level-by-level part, then one launch for the games
// whose tail starts here, writing into the same buffer.
template <class T>
static T* vcycle_level(Engine* e, std::vector<Level>& lv, int l, const EngineOpts& o, const int* act,
                       hipStream_t s, double* sol, const TailRefine* rf, T* start) {
  Level& L = lv[l];
  T* res = L.upper ? vcycle_impl<T>(e, lv, l, o, act, s, sol, start) : (start ? start : LV<T>::x(L));
  if (L.ntailg) {
    double bytes = 0.0;
    if (probe_on(kProbeTail))
      for (int k = l; k < e->num_levels(); ++k) {
        const Level& Lk = lv[k];
        const double rows = Lk.n ? (double)Lk.n : 0.0, sv = sizeof(T);
        // tail games' share of the level, (nu1 + nu2 + 1) sweeps of matrix and vectors
        double share = 0.0;
        for (int g : L.h_tailg) share += Lk.goff[g + 1] - Lk.goff[g];
        const double nnz = rows > 0 ? (double)Lk.nnz * share / rows : 0.0;
        bytes += (o.nu1 + o.nu2 + 1) * (share * (4 + 3 * sv) + nnz * (4 + sv));
      }
    probe_begin(kProbeTail, s);
    cyc_tail<T>(L.tailg.p, L.ntailg, l, e->num_levels(), e->num_slots(), e->tail_levels((T*)nullptr),
                e->tail_games(), act, (T)relax_weight(o), o.nu1, o.nu2, res == LV<T>::y(L) ? 1 : 0,
                L.tail_lds_rows, s, sol, rf);
    probe_end(kProbeTail, s, rf ? 0.0 : bytes);  // refinement: bytes once the cycles are known
    if (rf) e->tail_cycle_bytes = bytes;
  }
  return res;
}

void Engine::solve_linear(const std::vector<int>& run, const EngineOpts& o) {
  const bool mixed = o.precision == SHAPLEY_MIXED;
  Level& L0 = lv[0];
  h_lin_active.assign(G, 0);
  h_lin.assign(G, LinCtl{});
  for (int g : run) {
    const SlotState* S = slots[g];
    h_lin_active[g] = 1;
    LinCtl& c = h_lin[g];
    c.rtol = S->opt.lin_rtol;
    c.atol = S->opt.lin_atol;
    c.forcing = S->exact ? 0.0 : S->opt.forcing;  // exact solves once cycling was seen
    c.res_prev = S->res_prev;
    c.max_cycles = S->opt.max_cycles;
  }
  // controls and active flags in one transfer
  const int Gm = std::max(G, 1);
  h_linbuf.assign(2 * (size_t)Gm, LinCtl{});
  std::copy(h_lin.begin(), h_lin.end(), h_linbuf.begin());
  std::memcpy(h_linbuf.data() + Gm, h_lin_active.data(), sizeof(int) * G);
  up(d_lin.p, h_linbuf.data(), 2 * (size_t)Gm);
  // The stop test runs on the device after every FP64 residual; cycles are
  // queued in chunks ending with a residual and its test, the first chunk as
  // long as the previous solve (cycles of games that stopped return at once).
  auto resid_check = [&]() {
    probe_begin(kProbeResid64, stream);
    if (L0.stencil) {
      const StencilView sv = stencil_view(L0, d_st_off.p);
      if (mixed)
        cyc_resid64_st<float>(L0.tiles.p, L0.ntiles, d_lin_active, sv, L0.st64.p, rhs.p, sol.p, L0.b32.p, fold,
                              stream);
      else
        cyc_resid64_st<double>(L0.tiles.p, L0.ntiles, d_lin_active, sv, L0.st64.p, rhs.p, sol.p, L0.b64.p, fold,
                               stream);
    } else if (mixed) {
      cyc_resid64<float>(L0.tiles.p, L0.ntiles, d_lin_active, L0.rp.p, L0.ci.p, L0.a64.p, rhs.p, sol.p,
                         L0.b32.p, fold, L0.gA, stream);
    } else {
      cyc_resid64<double>(L0.tiles.p, L0.ntiles, d_lin_active, L0.rp.p, L0.ci.p, L0.a64.p, rhs.p, sol.p,
                          L0.b64.p, fold, L0.gA, stream);
    }
    {
      // per row: row pointer or code word, b, x, the residual; per entry (or
      // stencil slot): column and value, or the value alone
      const double rows = L0.rows_tiles;
      const double nnz = L0.n ? (double)L0.nnz * rows / L0.n : 0.0;
      probe_end(kProbeResid64, stream,
                rows * (4 + 8 + 8 + (mixed ? 4 : 8)) + (L0.stencil ? rows * L0.st_w * 8 : nnz * 12));
    }
    launch_lin_check(fold, G, d_bnorm.p, d_lin.p, d_lin_active, d_norm.p, stream);
  };
  // every level-0 row ends its cycle in a post-smoothing sweep or in a tail
  const bool fuse_update = o.nu2 >= 1 && L0.nvblk == 0 && o.smoother != SHAPLEY_SMOOTH_CF;
  resid_check();
  if (fuse_update && !L0.upper && L0.ntailg > 0) {
    // every game's tail starts on level 0: all its cycles, FP64 residuals and
    // stop tests in one launch of the tail kernel
    int maxc = 1;
    for (int g : run) maxc = std::max(maxc, slots[g]->opt.max_cycles);
    TailRefine rf{L0.a64.p, rhs.p, d_bnorm.p, d_lin.p, d_lin_active, d_norm.p, maxc + 1};
    tail_cycle_bytes = 0.0;
    if (mixed)
      vcycle_level<float>(this, lv, 0, o, d_lin_active, stream, sol.p, &rf);
    else
      vcycle_level<double>(this, lv, 0, o, d_lin_active, stream, sol.p, &rf);
    const LinCtl* pl = down(d_lin.p, 2 * (size_t)Gm);
    const int* pe = refresh_errors_down();
    sync();
    refresh_errors_check(pe);
    h_lin.assign(pl, pl + G);
    if (probe_on(kProbeTail)) {
      double cyc = 0.0;
      for (int g : run) cyc = std::max(cyc, (double)h_lin[g].cyc);
      probe_add_bytes(kProbeTail, tail_cycle_bytes * cyc);
    }
  } else {
  // one refinement cycle: the V- or W-cycle, the FP64 update and the FP64
  // residual with its stop test
  auto cycle = [&]() {
    // the last post-smoothing sweep of level 0 (or the tail that ends on
    // it) adds the correction to the FP64 iterate; otherwise a separate pass
    double* fused = fuse_update ? sol.p : nullptr;
    if (mixed) {
      float* e = vcycle_level<float>(this, lv, 0, o, d_lin_active, stream, fused);
      if (!fused) cyc_update64<float>(L0.tiles.p, L0.ntiles, d_lin_active, e, sol.p, stream);
    } else {
      double* e = vcycle_level<double>(this, lv, 0, o, d_lin_active, stream, fused);
      if (!fused) cyc_update64<double>(L0.tiles.p, L0.ntiles, d_lin_active, e, sol.p, stream);
    }
    resid_check();
  };
  // The cycle's launches are captured once per hierarchy into a HIP graph and
  // replayed (the hierarchy's buffers, tiles and lane counts stay fixed
  // through refreshes; the per-game flags are read from device memory).  A
  // probed run launches one by one so that its events bracket each kernel.
  bool probing = false;
  for (int f = 0; f < kProbeFamilies; ++f) probing |= probe_on(f);
  const bool use_graph = o.graph && !probing;
  if (use_graph) {
    const GraphKey key{hier_gen, mixed, o.nu1, o.nu2, o.omega, o.smoother, o.gamma, fuse_update, sol.p};
    if (!cyc_exec || !(key == cyc_key)) {
      drop_graph();
      hipGraph_t gr = nullptr;
      SHP_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
      try {
        cycle();
      } catch (...) {
        (void)hipStreamEndCapture(stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      SHP_HIP(hipStreamEndCapture(stream, &gr));
      const hipError_t ie = hipGraphInstantiate(&cyc_exec, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (ie != hipSuccess) {
        cyc_exec = nullptr;
        throw Error(SHAPLEY_EDEVICE, std::string("HIP graph instantiation failed: ") + hipGetErrorString(ie));
      }
      cyc_key = key;
    }
  }
  int chunk = std::max(1, std::min(last_cycles, 16));
  while (true) {
    for (int c = 0; c < chunk; ++c) {
      if (use_graph) SHP_HIP(hipGraphLaunch(cyc_exec, stream));
      else cycle();
    }
    const LinCtl* pl = down(d_lin.p, 2 * (size_t)Gm);
    const int* pe = refresh_errors_down();
    sync();
    refresh_errors_check(pe);
    const int* pa = reinterpret_cast<const int*>(pl + Gm);
    h_lin_active.assign(pa, pa + G);
    bool any = false;
    for (int g : run) any |= h_lin_active[g] != 0;
    if (!any) {
      h_lin.assign(pl, pl + G);
      break;
    }
    chunk = 1;
  }
  }
  for (int g : run) {
    SlotState* S = slots[g];
    const LinCtl& c = h_lin[g];
    S->cycles_total += c.cyc;
    S->loose = (c.flags & 1) != 0;
    if (c.flags & 4) {
      S->status = SHAPLEY_EDEVICE;
      S->why = "non-finite values in the linear solve";
    } else if (c.flags & 16) {
      S->status = SHAPLEY_ENOCONV;
      S->why = "the multigrid cycles diverge on this game's policy system (its AMG hierarchy does not fit it)";
      S->diverged = true;
    }
    if (c.flags & 2) stagnated = true;
  }
}

void Engine::improve(const std::vector<int>& run, double tie_rtol) {
  double bytes = 0.0;
  if (probe_on(kProbeImprove))
    for (int g : run) {
      const Game* gm = slots[g]->g;
      // per row: row pointer, reward, validity; per entry: column, weight;
      // per state: value, the five policy arrays and F when it is stored
      bytes += (double)gm->nrows * (4 + 8 + (gm->valid.p ? 1 : 0)) + (double)gm->nnz * 12 +
               (double)gm->n * (8 + 5 * 4 + (keep_F ? 8 : 0));
    }
  probe_begin(kProbeImprove, stream);
  launch_improve(ddesc.p, gtiles_imp.p, (int)h_gtiles_imp.size(), d_active.p, tie_rtol, fold, imp_threads, stream);
  probe_end(kProbeImprove, stream, bytes);
  launch_fold_finish(fold, G, 2, 2u, 3, d_shap.p, 2, d_cnt, 3, stream);
}

// The decisions are applied asynchronously (the host copy stays alive in a
// member until the next step); callers synchronise the stream before
// reading results.
void Engine::apply_decisions(const std::vector<int>& code) {
  h_decision = code;
  up(d_decision.p, h_decision.data(), G);
  launch_apply(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_decision.p, stream);
}

void Engine::run_init(const std::vector<int>& run) {
  std::vector<int> fresh;
  for (int g : run)
    if (slots[g]->need_init) fresh.push_back(g);
  if (fresh.empty()) return;
  asm_stale = true;  // a slot's game starts: its level-0 rows were never built for it
  std::vector<int> act(G, 0);
  for (int g : fresh) act[g] = 1;
  up(d_active.p, act.data(), G);
  h_active_dev = act;
  improve(fresh, slots[fresh[0]]->opt.tie_rtol);
  std::vector<double> hs(2 * G);
  const double* ps = down(d_shap.p, 2 * G);
  sync();
  hs.assign(ps, ps + 2 * G);
  std::vector<int> code(G, 0);
  for (int g : fresh) {
    SlotState* S = slots[g];
    code[g] = !S->init_alpha ? 2 : (!S->init_beta ? 1 : 0);
    S->need_init = false;
    S->res_prev = hs[2 * g];
  }
  apply_decisions(code);
}

void Engine::improve_only() {
  if (!keep_F) {
    keep_F = true;
    layout_dirty = true;
  }
  if (layout_dirty) build_layout();
  std::vector<int> all;
  for (int g = 0; g < G; ++g) all.push_back(g);
  std::vector<int> act(G, 1);
  up(d_active.p, act.data(), G);
  h_active_dev = act;
  improve(all, slots.empty() ? 1e-12 : slots[0]->opt.tie_rtol);
  sync();
}

// whether MAX's improved strategy (hash h) is one of an earlier outer step
// whose Shapley residual was no larger than the current one
static bool revisits(const SlotState* S, uint32_t h) {
  for (const auto& e : S->outer_hist)
    if (e.first == h && e.second <= S->res) return true;
  return false;
}

// a refresh is skipped while fewer than this fraction of the states changed
// policy since the coarse operators were last formed
constexpr double kLazyRefresh = 0.20;

int Engine::step() {
  if (layout_dirty) build_layout();
  std::vector<int> run = running_slots();
  if (run.empty()) return 0;
  run_init(run);
  const EngineOpts& o = slots[run[0]]->opt;
  const bool mixed = o.precision == SHAPLEY_MIXED;
  sol.ensure(std::max(N0, 1));
  rhs.ensure(std::max(N0, 1));
  d_bnorm.ensure(std::max(G, 1));
  h_active.assign(G, 0);
  for (int g : run) h_active[g] = 1;
  if (h_active != h_active_dev) {
    up(d_active.p, h_active.data(), G);
    h_active_dev = h_active;
  }

  double t0 = now_s();
  PhaseTimer pt(this, prof);
  assemble(run, mixed);
  pt.mark("assemble");
  // the hierarchy serves any subset of the games it was built for (the
  // levels are block diagonal over games; finished games are skipped)
  std::vector<int> rs = run, hs_ = run_at_setup;
  std::sort(rs.begin(), rs.end());
  std::sort(hs_.begin(), hs_.end());
  const bool subset = std::includes(hs_.begin(), hs_.end(), rs.begin(), rs.end());
  bool full = !have_hier || stagnated || !subset || o.reuse_frac <= 0.0 ||
              (double)changes_since_setup > o.reuse_frac * std::max(1, N0) ||
              last_cycles > std::max(2 * cycles_after_full, cycles_after_full + 6);
  stagnated = false;
  double t1 = 0.0;
  // a linear solve that diverges on a kept or refreshed hierarchy is done
  // again, once, on a new one (from the same start)
  for (int attempt = 0;; ++attempt) {
  for (int g : run) {
    if (full) ++slots[g]->setups_full; else ++slots[g]->setups_refresh;
  }
  if (full) {
    ++hier_gen;  // a new hierarchy: captured cycles are stale
    setup(run, o);
    lv[0].a_prev.ensure(std::max(NNZ0, 1));
    d2d(lv[0].a_prev.p, lv[0].a64.p, NNZ0, stream);
    have_hier = true;
    run_at_setup = run;
    changes_since_setup = 0;
    changes_since_refresh = 0;
    cycles_after_full = -1;
    ++full_setups;
  } else if ((double)changes_since_refresh < kLazyRefresh * std::max(1, N0) &&
             last_cycles <= cycles_after_full + 2) {
    // Few states changed policy since the coarse operators were last formed:
    // they are kept.  Level 0 (the assembled operator, its diagonal) is
    // always current, and the FP64 refinement measures the true residual, so
    // a slightly stale coarse correction only costs cycles -- a refresh is
    // taken again once the cycle count grows.
  } else {
    refresh(o);
    ++refreshes;
    changes_since_refresh = 0;
  }
  if (o.smoother == SHAPLEY_SMOOTH_L1) {
    // l1-Jacobi: the relaxation diagonals replace 1/a_ii once setup or refresh
    // (whose interpolation and Dirichlet scaling read 1/a_ii) is done
    for (int l = 0; l < nlev; ++l)
      amg_l1_diag(lv[l].tiles.p, lv[l].ntiles, lv[l].rp.p, lv[l].a64.p, lv[l].dinv64.p,
                  mixed ? lv[l].dinv32.p : nullptr, stream);
  }
  pt.mark("setup");
  t1 = now_s();  // a full setup ends with a synchronisation; a refresh does not
  {
    std::vector<int> before(G);
    for (int g : run) before[g] = slots[g]->cycles_total;
    solve_linear(run, o);
    int mx = 0;
    for (int g : run) mx = std::max(mx, slots[g]->cycles_total - before[g]);
    last_cycles = mx;
    if (cycles_after_full < 0) cycles_after_full = mx;
  }
  bool again = false;
  if (!full && attempt == 0)
    for (int g : run) again |= slots[g]->diverged;
  if (!again) break;
  for (int g : run) {
    SlotState* S = slots[g];
    if (!S->diverged) continue;
    S->diverged = false;
    S->status = SHAPLEY_OK;
    S->why.clear();
  }
  launch_gather_v(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_active.p, sol.p, stream);
  full = true;
  }
  pt.mark("solve");
  double t2 = now_s();  // solve_linear ends with a synchronisation
  launch_scatter_v(ddesc.p, gtiles_all.p, (int)h_gtiles_all.size(), d_active.p, sol.p, stream);
  improve(run, o.tie_rtol);
  std::vector<double> hs(2 * G);
  std::vector<int> hc(3 * G);
  const double* ps = down(d_shap.p, 4 * (size_t)std::max(G, 1));  // residuals, then the counts and hashes
  const int* pcn = reinterpret_cast<const int*>(ps + 2 * std::max(G, 1));
  sync();
  hs.assign(ps, ps + 2 * G);
  hc.assign(pcn, pcn + 3 * G);
  double t3 = now_s();
  pt.mark("improve");

  std::vector<int> code(G, 0);
  int still = 0;
  for (int g : run) {
    SlotState* S = slots[g];
    S->setup_s += t1 - t0;
    S->cycle_s += t2 - t1;
    S->improve_s += t3 - t2;
    const Game* gm = S->g;
    S->res = hs[2 * g];
    S->res_prev = S->res;
    ++S->solves;
    S->res_l2 = gm->n ? std::sqrt(hs[2 * g + 1] / gm->n) : 0.0;
    int nin = hc[3 * g], nout = hc[3 * g + 1];
    const uint32_t hout = (uint32_t)hc[3 * g + 2];
    S->nk += 1;
    S->inner_total += 1;
    if (S->status != SHAPLEY_OK) {
      S->done = true;
      continue;
    }
    if (!std::isfinite(S->res)) {
      S->status = SHAPLEY_EDEVICE;
      S->why = "non-finite Shapley residual";
      S->done = true;
      continue;
    }
    if (S->opt.verbose)
      fprintf(stderr, "[shapley] slot %d k %d nk %d res %.3e in %d out %d levels %d cycles %d %s\n", g, S->k,
              S->nk, S->res, nin, nout, S->levels, S->cycles_total, full ? "full" : "refresh");
    if (S->res <= S->opt.eps) {
      if (S->k <= 64) S->inner_per_outer[S->k - 1] = S->nk;
      code[g] = 2;
      S->converged = true;
      S->done = true;
    } else if (nin > 0 && S->nk < S->opt.max_inner) {
      code[g] = 1;
      changes_since_setup += nin;
      changes_since_refresh += nin;
      S->resolves = 0;
    } else if (nout == 0 && S->loose && S->resolves < 2) {
      // both policies look stable after an inexact solve: solve the same
      // system again, to forcing * eps (or to full accuracy when eps = 0),
      // before stopping (at most twice in a row)
      S->res_prev = S->opt.eps;
      S->nk -= 1;
      S->inner_total -= 1;
      S->resolves += 1;
    } else {
      if (S->k <= 64) S->inner_per_outer[S->k - 1] = S->nk;
      if (nout == 0 && nin > 0) {
        // MIN still improves but its loop was cut by max_inner, and MAX has
        // nothing to improve against an inexact inner solution: the stop of
        // Algorithm PIalgo assumes an exact inner loop, so this is no fixed
        // point (the residual is above eps, tested above)
        S->status = SHAPLEY_ENOCONV;
        S->why = "MIN's policy iteration was cut by max_inner while MAX had nothing left to improve";
        S->done = true;
      } else if (nout == 0) {
        S->converged = true;
        S->done = true;
      } else if (S->k >= S->opt.max_outer) {
        S->status = SHAPLEY_ENOCONV;
        S->why = "policy iteration hit an iteration limit (max_outer)";
        S->done = true;
      } else if (revisits(S, hout)) {
        // MAX's improved strategy is one taken at an earlier outer step whose
        // residual was no larger: policy iteration cycles (exact evaluations
        // improve strictly, Sec. 4.1).  After inexact solves the game goes on
        // with exact ones; with exact ones it stops.
        if (S->loose && !S->exact) {
          S->exact = true;
          S->outer_hist.clear();
          code[g] = 2;
          S->k += 1;
          S->nk = 0;
          changes_since_setup += nout;
          changes_since_refresh += nout;
          S->resolves = 0;
        } else {
          S->status = SHAPLEY_ENOCONV;
          S->why = "policy iteration cycles: MAX's strategy of an earlier outer step came back without a lower "
                   "Shapley residual";
          S->done = true;
        }
      } else {
        S->outer_hist.emplace_back(hout, S->res);
        if (S->outer_hist.size() > 32) S->outer_hist.erase(S->outer_hist.begin());
        code[g] = 2;
        S->k += 1;
        S->nk = 0;
        changes_since_setup += nout;
        changes_since_refresh += nout;
        S->resolves = 0;
      }
    }
    if (!S->done) ++still;
  }
  apply_decisions(code);
  return still;
}

EngineOpts engine_opts_from(const shapley_solve_opts& o, int dim) {
  (void)dim;
  EngineOpts e;
  e.eps = o.eps;
  e.precision = o.precision;
  e.max_outer = o.max_outer;
  e.max_inner = o.max_inner;
  e.max_cycles = o.max_cycles;
  e.lin_rtol = o.lin_rtol;
  e.lin_atol = o.lin_atol;
  e.tie_rtol = o.tie_rtol;
  e.theta = o.theta;
  e.nu1 = o.nu1;
  e.nu2 = o.nu2;
  e.omega = o.omega;
  e.coarse_max = o.coarse_max;
  e.max_levels = o.max_levels;
  e.verbose = o.verbose;
  e.reuse_frac = o.reuse_frac;
  e.forcing = o.forcing;
  e.smoother = o.smoother;
  e.gamma = o.gamma;
  e.graph = o.graph;
  return e;
}

}  // namespace shp
