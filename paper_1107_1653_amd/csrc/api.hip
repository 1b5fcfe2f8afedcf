// C ABI of libshapley: argument checking, game creation, solve drivers
// (AMGpi, FAMGpi, batch), result getters.
#include "internal.hpp"
#include "amg_kernels.hpp"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <numeric>

namespace shp {

static thread_local std::string g_last_error;

void set_last_error(const std::string& msg) { g_last_error = msg; }

Game::~Game() {
  for (Game* l : levels) delete l;
  levels.clear();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

size_t Game::device_bytes() const {
  size_t b = rp.bytes() + ci.bytes() + w.bytes() + r.bytes() + valid.bytes() + urp.bytes() + uci.bytes() +
             v.bytes() + F.bytes() + alpha.bytes() + beta.bytes() + beta_in.bytes() + alpha_c.bytes() +
             beta_c.bytes() + bvals.bytes();
  for (const Game* l : levels) b += l->device_bytes();
  return b;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

#define SHP_REQUIRE(cond, msg) \
  do {                         \
    if (!(cond)) throw Error(SHAPLEY_EINVAL, msg); \
  } while (0)

// Level-0 pattern, state and policy arrays and the grid description of a game
// whose transition arrays are on the device (shared by both create paths).
static void finish_game(Game* g, const shapley_grid* grid, bool device_ptrs) {
  hipStream_t s = g->stream;
  const int n = g->n;
  // level-0 pattern: union of the columns of a state's rows plus the diagonal
  g->urp.alloc(n + 1);
  DBuf<int> cnt(n + 1), scr;
  fill_async(cnt.p + n, 0, 1, s);
  launch_union_count(g->rp.p, g->ci.p, n, g->m1, g->m2, cnt.p, nullptr, s);
  scan_exclusive(cnt.p, g->urp.p, n + 1, s, scr);
  int unnz = 0;
  d2h(&unnz, g->urp.p + n, 1, s);
  SHP_HIP(hipStreamSynchronize(s));
  g->unnz = unnz;
  g->uci.alloc(std::max(unnz, 1));
  launch_union_fill(g->rp.p, g->ci.p, n, g->m1, g->m2, g->urp.p, g->uci.p, s);
  // the pattern's offsets col - x: a stencil when few (grid games)
  DBuf<int> st(2 + kStencilHash);
  launch_stencil_scan(g->urp.p, g->uci.p, n, st.p, s);
  int sth[2 + kStencilHash];
  d2h(sth, st.p, 2 + kStencilHash, s);
  g->v.alloc(n); g->F.alloc(n);
  g->alpha.alloc(n); g->beta.alloc(n); g->beta_in.alloc(n); g->alpha_c.alloc(n); g->beta_c.alloc(n);
  fill_async(g->v.p, 0.0, n, s);
  fill_async(g->alpha.p, 0, n, s);
  fill_async(g->beta.p, 0, n, s);
  if (grid) {
    g->dim = grid->dim;
    g->s = grid->s;
    if (grid->bvals) {
      int64_t ne = 1;
      for (int k = 0; k < grid->dim; ++k) ne *= (grid->s + 2);
      g->bvals.alloc(ne);
      if (device_ptrs) d2d(g->bvals.p, grid->bvals, ne, s);
      else h2d(g->bvals.p, grid->bvals, ne, s);
      g->has_bvals = true;
    }
  }
  SHP_HIP(hipStreamSynchronize(s));
  g->st_off.clear();
  g->st_w = 0;
  if (sth[0] == 0 && sth[1] <= kStencilMax) {
    std::vector<int> off;
    for (int k = 0; k < kStencilHash; ++k)
      if (sth[2 + k] != INT_MIN) off.push_back(sth[2 + k]);
    if (!off.empty() && (int)off.size() <= kStencilMax) {
      std::sort(off.begin(), off.end());
      g->st_off = off;
      g->st_w = sth[1];
    }
  }
}

static void check_grid(const shapley_grid* grid, int64_t n64) {
  if (!grid) return;
  SHP_REQUIRE(grid->dim >= 1 && grid->dim <= 3 && grid->s >= 1, "grid: dim in 1..3 and s >= 1");
  int64_t p = 1;
  for (int k = 0; k < grid->dim; ++k) p *= grid->s;
  SHP_REQUIRE(p == n64, "grid: s^dim must equal n");
}

static void make_stream(Game* g, void* stream) {
  if (stream) {
    g->stream = (hipStream_t)stream;
  } else {
    SHP_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    g->own_stream = true;
  }
}

// Arrays in device memory: the same conditions as for host arrays, checked by
// a kernel (one synchronisation), then device-to-device copies; rows whose
// columns are not ascending are sorted on the device (stable, as on the host).
static Game* create_game_device(int n, int m1, int m2, const int64_t* row_ptr, const int32_t* col,
                                const double* w, const double* r, double mu, const uint8_t* valid,
                                const shapley_grid* grid, void* stream) {
  const int nrows = n * m1 * m2;
  std::unique_ptr<Game> g(new Game());
  g->n = n; g->m1 = m1; g->m2 = m2; g->nrows = nrows; g->mu = mu;
  make_stream(g.get(), stream);
  hipStream_t s = g->stream;
  int64_t nnz = 0;
  d2h(&nnz, row_ptr + nrows, 1, s);
  SHP_HIP(hipStreamSynchronize(s));
  SHP_REQUIRE(nnz >= 0 && nnz < INT32_MAX, "number of transitions must be below 2^31");
  SHP_REQUIRE(nnz == 0 || (col && w), "null input array");
  DBuf<int> err(1);
  const int bits = check_game_device(row_ptr, col, w, r, valid, n, m1 * m2, nnz, err.p, s);
  SHP_REQUIRE(!(bits & kChkRp0), "row_ptr[0] must be 0");
  SHP_REQUIRE(!(bits & kChkRp), "row_ptr must be non-decreasing");
  SHP_REQUIRE(!(bits & kChkCol), "column index out of range");
  SHP_REQUIRE(!(bits & kChkW), "transition weights must be finite and >= 0");
  SHP_REQUIRE(!(bits & kChkSum), "row sum of transition weights exceeds 1");
  SHP_REQUIRE(!(bits & kChkR), "rewards must be finite");
  SHP_REQUIRE(!(bits & kChkEmpty), "empty action set at a state");
  g->nnz = nnz;
  g->rp.alloc(nrows + 1);
  g->ci.alloc(std::max<int64_t>(nnz, 1));
  g->w.alloc(std::max<int64_t>(nnz, 1));
  g->r.alloc(nrows);
  launch_rp_narrow(row_ptr, g->rp.p, nrows + 1, s);
  d2d(g->ci.p, col, nnz, s);
  d2d(g->w.p, w, nnz, s);
  if (bits & kChkUnsorted) launch_sort_pairs(g->rp.p, g->ci.p, g->w.p, nrows, s);
  d2d(g->r.p, r, nrows, s);
  if (valid) {
    g->valid.alloc(nrows);
    d2d(g->valid.p, valid, nrows, s);
  }
  finish_game(g.get(), grid, true);
  return g.release();
}

static Game* create_game(int64_t n64, int m1, int m2, const int64_t* row_ptr, const int32_t* col,
                         const double* w, const double* r, double mu, const uint8_t* valid,
                         const shapley_grid* grid, uint32_t flags, void* stream) {
  SHP_REQUIRE(flags == SHAPLEY_HOST_PTRS || flags == SHAPLEY_DEVICE_PTRS, "unsupported flags");
  SHP_REQUIRE(n64 >= 1 && m1 >= 1 && m2 >= 1, "n, m1 and m2 must be positive");
  SHP_REQUIRE((int64_t)m1 * m2 <= 256, "m1 * m2 must not exceed 256");
  const int64_t nrows64 = n64 * m1 * m2;
  SHP_REQUIRE(nrows64 < INT32_MAX, "n * m1 * m2 must be below 2^31");
  SHP_REQUIRE(row_ptr && r, "null input array");
  SHP_REQUIRE(std::isfinite(mu) && mu > 0.0 && mu <= 1.0, "mu must lie in (0, 1]");
  check_grid(grid, n64);
  if (flags == SHAPLEY_DEVICE_PTRS)
    return create_game_device((int)n64, m1, m2, row_ptr, col, w, r, mu, valid, grid, stream);
  SHP_REQUIRE(row_ptr[nrows64] == 0 || (col && w), "null input array");
  SHP_REQUIRE(row_ptr[0] == 0, "row_ptr[0] must be 0");
  const int n = (int)n64, nrows = (int)nrows64;
  const int64_t nnz = row_ptr[nrows];
  SHP_REQUIRE(nnz >= 0 && nnz < INT32_MAX, "number of transitions must be below 2^31");
  std::vector<int> rp32(nrows + 1);
  std::vector<int> ci_sorted;
  std::vector<double> w_sorted;
  bool need_sort = false;
  for (int i = 0; i < nrows; ++i) {
    SHP_REQUIRE(row_ptr[i + 1] >= row_ptr[i] && row_ptr[i + 1] <= nnz, "row_ptr must be non-decreasing");
    rp32[i] = (int)row_ptr[i];
    double sum = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      SHP_REQUIRE(col[e] >= 0 && col[e] < n, "column index out of range");
      SHP_REQUIRE(std::isfinite(w[e]) && w[e] >= 0.0, "transition weights must be finite and >= 0");
      if (e > row_ptr[i] && col[e] < col[e - 1]) need_sort = true;
      sum += w[e];
    }
    SHP_REQUIRE(sum <= 1.0 + 1e-12, "row sum of transition weights exceeds 1");
    SHP_REQUIRE(std::isfinite(r[i]), "rewards must be finite");
  }
  rp32[nrows] = (int)nnz;
  if (valid) {
    for (int x = 0; x < n; ++x) {
      bool any = false;
      for (int q = 0; q < m1 * m2; ++q) any |= valid[(int64_t)x * m1 * m2 + q] != 0;
      SHP_REQUIRE(any, "empty action set at a state");
    }
  }
  const int32_t* colp = col;
  const double* wp = w;
  if (need_sort) {
    ci_sorted.assign(col, col + nnz);
    w_sorted.assign(w, w + nnz);
    std::vector<int> idx;
    for (int i = 0; i < nrows; ++i) {
      int e0 = rp32[i], e1 = rp32[i + 1];
      idx.resize(e1 - e0);
      std::iota(idx.begin(), idx.end(), e0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return col[a] < col[b]; });
      for (int k = 0; k < e1 - e0; ++k) { ci_sorted[e0 + k] = col[idx[k]]; w_sorted[e0 + k] = w[idx[k]]; }
    }
    colp = ci_sorted.data();
    wp = w_sorted.data();
  }
  std::unique_ptr<Game> g(new Game());
  g->n = n; g->m1 = m1; g->m2 = m2; g->nrows = nrows; g->nnz = nnz; g->mu = mu;
  make_stream(g.get(), stream);
  hipStream_t s = g->stream;
  g->rp.alloc(nrows + 1);
  g->ci.alloc(std::max<int64_t>(nnz, 1));
  g->w.alloc(std::max<int64_t>(nnz, 1));
  g->r.alloc(nrows);
  h2d(g->rp.p, rp32.data(), nrows + 1, s);
  h2d(g->ci.p, colp, nnz, s);
  h2d(g->w.p, wp, nnz, s);
  h2d(g->r.p, r, nrows, s);
  if (valid) {
    g->valid.alloc(nrows);
    h2d(g->valid.p, valid, nrows, s);
  }
  finish_game(g.get(), grid, false);
  return g.release();
}

void check_solve_opts(const shapley_solve_opts& o) {
  SHP_REQUIRE(std::isfinite(o.eps) && o.eps >= 0.0, "eps must be >= 0");
  SHP_REQUIRE(o.precision == SHAPLEY_FP64 || o.precision == SHAPLEY_MIXED, "bad precision");
  SHP_REQUIRE(o.method == SHAPLEY_AMGPI || o.method == SHAPLEY_FAMGPI, "bad method");
  SHP_REQUIRE(o.max_outer >= 1 && o.max_inner >= 1 && o.max_cycles >= 1, "iteration limits must be >= 1");
  SHP_REQUIRE(o.nu1 >= 1 && o.nu2 >= 0, "nu1 >= 1 and nu2 >= 0 required");
  SHP_REQUIRE(o.omega > 0.0 && o.omega < 2.0, "omega must lie in (0, 2)");
  SHP_REQUIRE(o.coarse_max >= 1 && o.coarse_max <= kDenseMax, "coarse_max must lie in [1, 1024]");
  SHP_REQUIRE(o.max_levels >= 1 && o.max_levels <= 64, "max_levels must lie in [1, 64]");
  SHP_REQUIRE(o.lin_rtol >= 0.0 && o.lin_atol >= 0.0 && o.tie_rtol >= 0.0, "tolerances must be >= 0");
  SHP_REQUIRE(o.c_fmg > 0.0, "c_fmg must be > 0");
  SHP_REQUIRE(o.reuse_frac >= 0.0 && o.reuse_frac <= 1.0, "reuse_frac must lie in [0, 1]");
  SHP_REQUIRE(std::isfinite(o.forcing) && o.forcing >= 0.0 && o.forcing < 1.0, "forcing must lie in [0, 1)");
  SHP_REQUIRE(o.smoother == SHAPLEY_SMOOTH_JACOBI || o.smoother == SHAPLEY_SMOOTH_L1 ||
                  o.smoother == SHAPLEY_SMOOTH_CF,
              "bad smoother");
  SHP_REQUIRE(o.gamma == 1 || o.gamma == 2, "gamma must be 1 (V-cycle) or 2 (W-cycle)");
  SHP_REQUIRE(o.graph == 0 || o.graph == 1, "graph must be 0 or 1");
  SHP_REQUIRE(std::isfinite(o.theta) && std::isfinite(o.omega) && std::isfinite(o.c_fmg) &&
                  std::isfinite(o.lin_rtol) && std::isfinite(o.lin_atol) && std::isfinite(o.tie_rtol) &&
                  std::isfinite(o.reuse_frac),
              "options must be finite");
}

}  // namespace shp

// Warm-start strategies of a solve (host arrays, n entries; beta0 optional):
// alpha0(x) must be an available action (one with a valid b) and (alpha0,
// beta0) a valid pair at every state.  Checked on the device against the
// game's validity mask before anything is modified; EINVAL otherwise.
void shp::check_warm_start(Game* g, const int32_t* alpha0, const int32_t* beta0, hipStream_t s) {
  if (!alpha0) return;
  const int n = g->n;
  for (int x = 0; x < n; ++x) SHP_REQUIRE(alpha0[x] >= 0 && alpha0[x] < g->m1, "alpha0 out of range");
  if (beta0)
    for (int x = 0; x < n; ++x) SHP_REQUIRE(beta0[x] >= 0 && beta0[x] < g->m2, "beta0 out of range");
  if (!g->valid.p) return;
  DBuf<int> tmp(2 * (size_t)n + 1);
  h2d(tmp.p, alpha0, n, s);
  if (beta0) h2d(tmp.p + n, beta0, n, s);
  const int bits = check_policy_device(tmp.p, beta0 ? tmp.p + n : nullptr, g->valid.p, n, g->m1, g->m2,
                                       tmp.p + 2 * n, s);
  SHP_REQUIRE(!(bits & 1), "alpha0 names an action with no valid b at some state");
  SHP_REQUIRE(!(bits & 2), "(alpha0, beta0) is not a valid pair at some state");
}

namespace shp {

// The default start of a solve (v = 0, no incumbent strategies) of several
// games in one launch: blockIdx.y is the game; null arrays are left as they are.
struct StartDesc {
  double* v;
  int* alpha;
  int* beta;
  int n;
};
__global__ void k_reset_start(const StartDesc* __restrict__ d, StartDesc one) {
  const StartDesc g = d ? d[blockIdx.y] : one;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < g.n; x += gridDim.x * blockDim.x) {
    if (g.v) g.v[x] = 0.0;
    if (g.alpha) g.alpha[x] = -1;
    if (g.beta) g.beta[x] = -1;
  }
}
static unsigned reset_blocks(int n) { return (unsigned)std::max(1, std::min((n + kBlock - 1) / kBlock, 256)); }

static void load_warm_start(Game* g, const shapley_solve_opts& o, SlotState& S, hipStream_t s,
                            std::vector<StartDesc>* defer = nullptr) {
  const int n = g->n;
  check_warm_start(g, o.alpha0, o.beta0, s);
  bool copied = false;
  if (o.v0) {
    h2d(g->v.p, o.v0, n, s);
    copied = true;
  }
  if (o.alpha0) {
    h2d(g->alpha.p, o.alpha0, n, s);
    S.init_alpha = true;
    copied = true;
  }
  if (o.alpha0 && o.beta0) {
    h2d(g->beta.p, o.beta0, n, s);
    S.init_beta = true;
    copied = true;
  }
  const StartDesc d{o.v0 ? nullptr : g->v.p, o.alpha0 ? nullptr : g->alpha.p,
                    (o.alpha0 && o.beta0) ? nullptr : g->beta.p, n};
  if (d.v || d.alpha || d.beta) {
    if (defer) {
      defer->push_back(d);  // one launch for the games of a batch
    } else {
      hipLaunchKernelGGL(k_reset_start, dim3(reset_blocks(n)), dim3(kBlock), 0, s, (const StartDesc*)nullptr, d);
      SHP_LAUNCH_CHECK();
    }
  }
  // the caller's host arrays are no longer read once this returns
  if (copied) SHP_HIP(hipStreamSynchronize(s));
}

static void fill_stats(const SlotState& S, shapley_stats* st, double seconds) {
  if (!st) return;
  std::memset(st, 0, sizeof(*st));
  st->outer = S.k;
  st->inner_total = S.inner_total;
  st->cycles_total = S.cycles_total;
  st->levels = S.levels;
  st->converged = S.converged ? 1 : 0;
  st->fmg_levels = 1;
  st->residual = S.res;
  st->residual_l2 = S.res_l2;
  st->seconds = seconds;
  st->setup_seconds = S.setup_s;
  st->cycle_seconds = S.cycle_s;
  st->improve_seconds = S.improve_s;
  st->op_complexity = S.opc;
  st->grid_complexity = S.gc;
  std::memcpy(st->inner_per_outer, S.inner_per_outer, sizeof(st->inner_per_outer));
  st->setups_full = S.setups_full;
  st->setups_refresh = S.setups_refresh;
  st->value_steps = S.solves;
}

// AMGpi on one game (the value step and improvement of every iteration run
// in the engine); returns the slot's status.
static int run_amgpi(Game* g, const shapley_solve_opts& o, double eps, bool warm_from_opts,
                     hipStream_t s, SlotState& S) {
  const bool keep = o.stream == nullptr;  // the game's own stream
  S = SlotState();
  S.g = g;
  S.opt = engine_opts_from(o, g->dim);
  S.opt.eps = eps;
  if (warm_from_opts) {
    load_warm_start(g, o, S, s);
  } else {
    S.init_alpha = S.init_beta = true;  // v, alpha, beta already on the device
  }
  EngineLease eng(s, keep);
  eng->slots.push_back(&S);
  while (eng->step() > 0) {
  }
  SHP_HIP(hipStreamSynchronize(s));
  g->solved = true;
  return S.status;
}

}  // namespace shp

using namespace shp;

template <class F>
static int guarded(F&& f) {
  try {
    f();
    return SHAPLEY_OK;
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

namespace shp {
std::atomic<long long> g_alloc_fault{0};  // armed by shapley_debug_fail_alloc
}

extern "C" {

const char* shapley_last_error(void) { return g_last_error.c_str(); }

void shapley_default_opts(shapley_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->eps = 0.0;
  o->precision = SHAPLEY_FP64;
  o->method = SHAPLEY_AMGPI;
  o->c_fmg = 1e-2;
  o->max_outer = 100000;
  o->max_inner = 100000;
  o->max_cycles = 200;
  o->lin_rtol = 1e-14;
  o->lin_atol = 0.0;
  o->tie_rtol = 1e-12;
  o->theta = -1.0;
  o->nu1 = 2;
  o->nu2 = 2;
  o->omega = 0.8;
  o->coarse_max = 64;
  o->max_levels = 25;
  o->verbose = 0;
  o->stream = nullptr;
  o->reuse_frac = 0.5;
  o->forcing = 0.0;
  o->smoother = SHAPLEY_SMOOTH_JACOBI;
  o->gamma = 1;
  o->graph = 1;
}

int shapley_game_create(shapley_game_t* out, int64_t n, int32_t m1, int32_t m2, const int64_t* row_ptr,
                        const int32_t* col, const double* w, const double* r, double mu,
                        const uint8_t* valid, const shapley_grid* grid, uint32_t flags, void* stream) {
  return guarded([&] {
    SHP_REQUIRE(out != nullptr, "out must not be null");
    Game* g = create_game(n, m1, m2, row_ptr, col, w, r, mu, valid, grid, flags, stream);
    *out = new shapley_game_s{g};
    games_alive_add(1);
  });
}

int shapley_game_create_hierarchy(shapley_game_t* out, int32_t nlev, shapley_game_t* levels) {
  return guarded([&] {
    SHP_REQUIRE(out && levels && nlev >= 1, "bad hierarchy arguments");
    int dim = -1;
    for (int l = 0; l < nlev; ++l) {
      SHP_REQUIRE(levels[l] && levels[l]->g, "null level handle");
      Game* g = levels[l]->g;
      SHP_REQUIRE(!g->is_hierarchy(), "levels must be plain games");
      SHP_REQUIRE(g->dim >= 1, "every level needs a grid description");
      if (dim < 0) dim = g->dim;
      SHP_REQUIRE(g->dim == dim, "levels must share the grid dimension");
      if (l > 0) {
        SHP_REQUIRE(g->s > levels[l - 1]->g->s, "levels must be ordered coarse -> fine");
        SHP_REQUIRE(g->m1 == levels[l - 1]->g->m1 && g->m2 == levels[l - 1]->g->m2,
                    "levels must have the same numbers of actions");
      }
    }
    Game* h = new Game();
    for (int l = 0; l < nlev; ++l) {
      h->levels.push_back(levels[l]->g);
      delete levels[l];
      levels[l] = nullptr;
    }
    Game* f = h->levels.back();
    h->n = f->n; h->m1 = f->m1; h->m2 = f->m2; h->dim = f->dim; h->s = f->s;
    h->stream = f->stream;
    *out = new shapley_game_s{h};
    games_alive_add(1 - nlev);  // the level handles were absorbed
  });
}

int shapley_solve(shapley_game_t gh, const shapley_solve_opts* op, shapley_stats* st) {
  int status = SHAPLEY_OK;
  int rc = guarded([&] {
    shapley_solve_opts o;
    if (op) o = *op; else shapley_default_opts(&o);
    check_solve_opts(o);  // before the handle: no device state is needed to reject options
    SHP_REQUIRE(gh && gh->g, "null game");
    Game* g = gh->g;
    hipStream_t s = o.stream ? (hipStream_t)o.stream : g->finest()->stream;
    double t0 = now_s();
    SlotState S;
    if (g->is_hierarchy() && o.method == SHAPLEY_FAMGPI) {
      // FAMGpi (Algorithm algo-FAMGPI): coarse -> fine with eps_l = c h_l^2,
      // transfers of (v, alpha, beta) by I and U between consecutive levels.
      const int L = (int)g->levels.size();
      int outer = 0, inner = 0, cycles = 0, sfull = 0, sref = 0, vsteps = 0;
      double su = 0, cy = 0, im = 0;
      for (int l = 0; l < L; ++l) {
        Game* lg = g->levels[l];
        bool last = l == L - 1;
        double h = 1.0 / (lg->s + 1);
        double eps = last ? o.eps : o.c_fmg * h * h;
        if (l > 0) {
          fmg_transfer(g->levels[l - 1], lg, s);
          SHP_HIP(hipStreamSynchronize(s));
        }
        int stt = run_amgpi(lg, o, eps, l == 0, s, S);
        outer += S.k; inner += S.inner_total; cycles += S.cycles_total;
        sfull += S.setups_full; sref += S.setups_refresh; vsteps += S.solves;
        su += S.setup_s; cy += S.cycle_s; im += S.improve_s;
        if (stt != SHAPLEY_OK && stt != SHAPLEY_ENOCONV) { status = stt; break; }
        if (last) status = stt;
      }
      double t1 = now_s();
      fill_stats(S, st, t1 - t0);
      if (st) {
        st->fmg_levels = L;
        st->outer = outer; st->inner_total = inner; st->cycles_total = cycles;
        st->setup_seconds = su; st->cycle_seconds = cy; st->improve_seconds = im;
        st->setups_full = sfull; st->setups_refresh = sref; st->value_steps = vsteps;
      }
    } else {
      status = run_amgpi(g->finest(), o, o.eps, true, s, S);
      fill_stats(S, st, now_s() - t0);
    }
    if (status == SHAPLEY_ENOCONV)
      set_last_error(S.why.empty() ? "policy iteration hit an iteration limit" : S.why);
    if (status == SHAPLEY_EDEVICE) set_last_error(S.why.empty() ? "non-finite values during the solve" : S.why);
  });
  return rc != SHAPLEY_OK ? rc : status;
}

int shapley_solve_batch(shapley_game_t* games, int32_t count, const shapley_solve_opts* op,
                        shapley_stats* stats) {
  int status = SHAPLEY_OK;
  int rc = guarded([&] {
    shapley_solve_opts o;
    if (op) o = *op; else shapley_default_opts(&o);
    check_solve_opts(o);
    SHP_REQUIRE(games && count >= 1, "bad batch arguments");
    SHP_REQUIRE(o.alpha0 == nullptr && o.beta0 == nullptr && o.v0 == nullptr,
                "warm starts are not accepted in batch mode");
    std::vector<SlotState> S(count);
    for (int i = 0; i < count; ++i) {
      SHP_REQUIRE(games[i] && games[i]->g && !games[i]->g->is_hierarchy(), "batch members must be games");
    }
    hipStream_t s = o.stream ? (hipStream_t)o.stream : games[0]->g->stream;
    double t0 = now_s();
    EngineLease eng(s, o.stream == nullptr);
    std::vector<StartDesc> starts;
    int nmax = 1;
    for (int i = 0; i < count; ++i) {
      Game* g = games[i]->g;
      S[i].g = g;
      S[i].opt = engine_opts_from(o, g->dim);
      load_warm_start(g, o, S[i], s, &starts);
      nmax = std::max(nmax, g->n);
      eng->slots.push_back(&S[i]);
    }
    DBuf<StartDesc> dstarts(std::max<size_t>(starts.size(), 1));
    for (size_t k0 = 0; k0 < starts.size(); k0 += 65535) {  // grid y limit
      const size_t k1 = std::min(starts.size(), k0 + 65535);
      h2d(dstarts.p + k0, starts.data() + k0, k1 - k0, s);
      hipLaunchKernelGGL(k_reset_start, dim3(reset_blocks(nmax), (unsigned)(k1 - k0)), dim3(kBlock), 0, s,
                         (const StartDesc*)(dstarts.p + k0), StartDesc{});
      SHP_LAUNCH_CHECK();
    }
    while (eng->step() > 0) {
    }
    SHP_HIP(hipStreamSynchronize(s));
    double t1 = now_s();
    for (int i = 0; i < count; ++i) {
      games[i]->g->solved = true;
      if (stats) fill_stats(S[i], &stats[i], t1 - t0);
      if (S[i].status != SHAPLEY_OK && status == SHAPLEY_OK) {
        status = S[i].status;
        set_last_error("game " + std::to_string(i) + ": " +
                       (S[i].why.empty() ? std::string("policy iteration stopped with an error") : S[i].why));
      }
    }
  });
  return rc != SHAPLEY_OK ? rc : status;
}

int shapley_get_value(shapley_game_t gh, double* v, int32_t on_device) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g && v, "null argument");
    Game* g = gh->g->finest();
    SHP_HIP(hipMemcpyAsync(v, g->v.p, sizeof(double) * g->n,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, g->stream));
    SHP_HIP(hipStreamSynchronize(g->stream));
  });
}

int shapley_get_policy(shapley_game_t gh, int32_t* alpha, int32_t* beta, int32_t* beta_all) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g, "null game");
    Game* g = gh->g->finest();
    hipStream_t s = g->stream;
    if (alpha) d2h(alpha, g->alpha.p, g->n, s);
    if (beta) d2h(beta, g->beta.p, g->n, s);
    SHP_HIP(hipStreamSynchronize(s));
    if (beta_all) {
      // MIN's lowest-index argmin at every a: run the improvement sweep with
      // alpha = a fixed and no incumbent, for each a
      std::vector<int> keep_a(g->n), keep_b(g->n);
      d2h(keep_a.data(), g->alpha.p, g->n, s);
      d2h(keep_b.data(), g->beta.p, g->n, s);
      SHP_HIP(hipStreamSynchronize(s));
      SlotState S;
      S.g = g;
      Engine eng(s);
      eng.slots.push_back(&S);
      std::vector<int> col(g->n);
      for (int a = 0; a < g->m1; ++a) {
        std::vector<int> av(g->n, a);
        h2d(g->alpha.p, av.data(), g->n, s);
        fill_async(g->beta.p, -1, g->n, s);
        eng.improve_only();
        d2h(col.data(), g->beta_in.p, g->n, s);
        SHP_HIP(hipStreamSynchronize(s));
        for (int x = 0; x < g->n; ++x) beta_all[(int64_t)x * g->m1 + a] = col[x];
      }
      h2d(g->alpha.p, keep_a.data(), g->n, s);
      h2d(g->beta.p, keep_b.data(), g->n, s);
      SHP_HIP(hipStreamSynchronize(s));
    }
  });
}

int shapley_apply_operator(shapley_game_t gh, const double* v, double* F, int32_t* alpha, int32_t* beta) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g && v, "null argument");
    Game* g = gh->g->finest();
    hipStream_t s = g->stream;
    const int n = g->n;
    std::vector<double> keep_v(n);
    std::vector<int> keep_a(n), keep_b(n);
    d2h(keep_v.data(), g->v.p, n, s);
    d2h(keep_a.data(), g->alpha.p, n, s);
    d2h(keep_b.data(), g->beta.p, n, s);
    SHP_HIP(hipStreamSynchronize(s));
    h2d(g->v.p, v, n, s);
    fill_async(g->alpha.p, -1, n, s);
    fill_async(g->beta.p, -1, n, s);
    SlotState S;
    S.g = g;
    Engine eng(s);
    eng.slots.push_back(&S);
    eng.improve_only();
    if (F) d2h(F, g->F.p, n, s);
    if (alpha) d2h(alpha, g->alpha_c.p, n, s);
    if (beta) d2h(beta, g->beta_c.p, n, s);
    SHP_HIP(hipStreamSynchronize(s));
    h2d(g->v.p, keep_v.data(), n, s);
    h2d(g->alpha.p, keep_a.data(), n, s);
    h2d(g->beta.p, keep_b.data(), n, s);
    SHP_HIP(hipStreamSynchronize(s));
  });
}

int shapley_game_info(shapley_game_t gh, int64_t* n, int32_t* m1, int32_t* m2) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g, "null game");
    Game* g = gh->g->finest();
    if (n) *n = g->n;
    if (m1) *m1 = g->m1;
    if (m2) *m2 = g->m2;
  });
}

int shapley_hierarchy_level(shapley_game_t gh, int32_t level, shapley_level_info* info, int32_t* rp, int32_t* ci,
                            double* a, int32_t* pc, double* pv) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g, "null game");
    Game* g = gh->g->finest();
    Engine* e = engine_cached(g->stream);
    SHP_REQUIRE(e && e->hier_game == g, "no AMG hierarchy of this game (solve it alone on its own stream first)");
    int levels = 0;
    int64_t n = 0, nnz = 0, nc = 0;
    e->level_export(level, &levels, &n, &nnz, &nc, rp, ci, a, pc, pv);
    if (info) {
      info->levels = levels;
      info->pw = PW;
      info->n = n;
      info->nnz = nnz;
      info->nc = nc;
    }
  });
}

int shapley_debug_fail_alloc(int64_t after) {
  if (after < 0) {
    shp::set_last_error("after must be >= 0");
    return SHAPLEY_EINVAL;
  }
  shp::g_alloc_fault.store(after);
  return SHAPLEY_OK;
}

int shapley_tune_lanes(int32_t lanes) {
  if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4) {
    shp::set_last_error("lanes must be 0, 1, 2 or 4");
    return SHAPLEY_EINVAL;
  }
  shp::set_forced_lanes(lanes);
  return SHAPLEY_OK;
}

int shapley_tune_galerkin(int32_t kernel) {
  if (kernel != -1 && kernel != 0 && kernel != 1 && kernel != 4) {
    shp::set_last_error("kernel must be -1, 0, 1 or 4");
    return SHAPLEY_EINVAL;
  }
  shp::set_forced_rap_cols(kernel);
  return SHAPLEY_OK;
}

int shapley_tune_interp(int32_t kernel) {
  if (kernel != -1 && kernel != 0 && kernel != 4) {
    shp::set_last_error("kernel must be -1, 0 or 4");
    return SHAPLEY_EINVAL;
  }
  shp::set_interp_mode(kernel);
  return SHAPLEY_OK;
}

int shapley_tune_dense(int32_t kernel) {
  if (kernel != -1 && kernel != 0) {
    shp::set_last_error("kernel must be -1 or 0");
    return SHAPLEY_EINVAL;
  }
  shp::set_dense_mode(kernel);
  return SHAPLEY_OK;
}

int shapley_coarse_inverse(const double* a, const int32_t* sizes, int32_t count, double* inv) {
  return guarded([&] {
    SHP_REQUIRE(count >= 0, "count must be >= 0");
    if (count == 0) return;
    SHP_REQUIRE(a && sizes && inv, "null argument");
    std::vector<int> hblk, hrp(1, 0), hci;
    std::vector<double> ha;
    size_t doff = 0;
    int row0 = 0, max_nb = 0;
    for (int g = 0; g < count; ++g) {
      const int nb = sizes[g];
      SHP_REQUIRE(nb >= 1 && nb <= kDenseMax, "block sizes must lie in 1 .. 1024");
      SHP_REQUIRE(doff + (size_t)nb * nb < (size_t)INT_MAX, "blocks exceed 2^31 entries together");
      hblk.insert(hblk.end(), {row0, nb, (int)doff, g});
      for (int i = 0; i < nb; ++i) {
        for (int j = 0; j < nb; ++j) {
          const double v = a[doff + (size_t)i * nb + j];
          SHP_REQUIRE(std::isfinite(v), "entries must be finite");
          hci.push_back(row0 + j);
          ha.push_back(v);
        }
        hrp.push_back((int)hci.size());
      }
      row0 += nb;
      doff += (size_t)nb * nb;
      max_nb = std::max(max_nb, nb);
    }
    hipStream_t s = nullptr;
    DBuf<int> dblk(hblk.size()), drp(hrp.size()), dci(hci.size()), derr(1);
    DBuf<double> da(ha.size()), dinv(doff), dwork(max_nb > kDenseWave ? 2 * doff : 0);
    const int zero = 0;
    h2d(dblk.p, hblk.data(), hblk.size(), s);
    h2d(drp.p, hrp.data(), hrp.size(), s);
    h2d(dci.p, hci.data(), hci.size(), s);
    h2d(da.p, ha.data(), ha.size(), s);
    h2d(derr.p, &zero, 1, s);
    amg_dense_inv(dblk.p, count, drp.p, dci.p, da.p, dwork.p, dinv.p, nullptr, derr.p, max_nb, s);
    std::vector<double> hinv(doff);
    int herr = 0;
    d2h(hinv.data(), dinv.p, doff, s);
    d2h(&herr, derr.p, 1, s);
    SHP_HIP(hipStreamSynchronize(s));
    if (herr & 4) throw Error(SHAPLEY_EDEVICE, "singular block");
    doff = 0;
    for (int g = 0; g < count; ++g) {  // column-major on the device, row-major for the caller
      const int nb = sizes[g];
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) inv[doff + (size_t)i * nb + j] = hinv[doff + (size_t)j * nb + i];
      doff += (size_t)nb * nb;
    }
  });
}

int shapley_tune_stencil(int32_t mode) {
  if (mode != -1 && mode != 0) {
    shp::set_last_error("mode must be -1 or 0");
    return SHAPLEY_EINVAL;
  }
  shp::set_stencil_mode(mode);
  return SHAPLEY_OK;
}

int shapley_game_bytes(shapley_game_t gh, size_t* bytes) {
  return guarded([&] {
    SHP_REQUIRE(gh && gh->g && bytes, "null argument");
    *bytes = gh->g->device_bytes();
  });
}

void shapley_game_destroy(shapley_game_t gh) {
  if (!gh) return;
  try {
    if (gh->g) {
      engine_cache_drop(gh->g->stream);
      for (Game* l : gh->g->levels) engine_cache_drop(l->stream);
    }
  } catch (...) {
  }
  delete gh->g;
  delete gh;
  try {
    games_alive_add(-1);
  } catch (...) {
  }
}

}  // extern "C"
