// Internal data structures of libshapley: games, merged AMG levels, engine.
#pragma once

#include "../../include/shapley.h"
#include "common.hpp"

#include <array>
#include <cstring>
#include <memory>

namespace shp {

constexpr int PW = 4;            // max interpolation entries per fine row (ELL width)
constexpr int kTileRows = 256;   // rows per level tile
constexpr int kMaxUnion = 128;   // max entries of one state's level-0 pattern row
constexpr int kDenseMax = 1024;  // largest dense coarse block
constexpr int kDenseWave = 96;   // blocks up to this size: one thread per row, rows in registers
constexpr int kMaxMergedRows = 1 << 25;  // states of the games solved together (64 lanes per row fit 2^31)
constexpr int kStencilMax = 8;   // offsets and row length of a stencil pattern (3-bit slot codes)
constexpr int kStencilHash = 32;

// POD view of one game for work-list kernels.
struct GameDesc {
  const int* rp;          // game CSR row pointer [nrows+1]
  const int* ci;          // columns
  const double* w;        // weights
  const double* r;        // rewards [nrows]
  const uint8_t* valid;   // [nrows] or null
  const int* urp;         // level-0 pattern of the game: row pointer [n+1] (local)
  const int* uci;         // level-0 pattern columns (local, sorted, incl. diagonal)
  double* v;              // value [n]
  int* alpha;             // MAX policy [n]
  int* beta;              // MIN policy at alpha [n]
  int* beta_in;           // improvement outputs [n]
  int* alpha_c;
  int* beta_c;
  double* F;              // F(v) [n], or null: not stored
  const double* bvals;    // Dirichlet values on the extended grid or null
  int n, m1, m2, slot;
  double mu;
  int x_off;              // first row of this game in the merged level 0
  int a_off;              // first nnz of this game in the merged level 0
};

// State range of one game for work-list kernels.
struct GTile {
  int game, s0, s1;
  int e0 = 0, e1 = 0;  // improvement tiles: the entry range of the tile's rows
};

// Device-resident game (the payload of a shapley_game_t).
struct Game {
  int n = 0, m1 = 0, m2 = 0, nrows = 0;
  int64_t nnz = 0;
  double mu = 1.0;
  DBuf<int> rp, ci;
  DBuf<double> w, r;
  DBuf<uint8_t> valid;
  DBuf<int> urp, uci;
  int unnz = 0;
  // the level-0 pattern as a stencil: the distinct offsets col - x of its
  // entries, ascending (empty: more than kStencilMax of them or rows longer
  // than kStencilMax), and its longest row
  std::vector<int> st_off;
  int st_w = 0;
  DBuf<double> v, F;
  DBuf<int> alpha, beta, beta_in, alpha_c, beta_c;
  int dim = 0, s = 0;
  DBuf<double> bvals;
  bool has_bvals = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool solved = false;
  // hierarchy handles own their levels (coarse -> fine)
  std::vector<Game*> levels;
  bool is_hierarchy() const { return !levels.empty(); }
  Game* finest() { return levels.empty() ? this : levels.back(); }
  size_t device_bytes() const;
  ~Game();
};

// A device pointer into a buffer owned elsewhere.
template <class T>
struct DPtr {
  T* p = nullptr;
};

// One merged (block-diagonal over games) AMG level.
// ---------------------------------------------------------------------------
// V-cycle tail: once a game's rows on a level are few (kTailRows), the rest of
// its V-cycle (that level and all coarser ones, down to its dense solve) runs
// in one workgroup of one launch, one workgroup per game, instead of a launch
// per kernel and level.
// ---------------------------------------------------------------------------
constexpr int kTailRows = 2048;
constexpr int kTailNnz = 16384;  // entries of the tail's first level (one CU streams them per sweep)
constexpr int kTailThreads = 1024;
// the tail keeps two iterate vectors per level in LDS: a game's rows summed
// over its tail levels are at most kTailLdsBytes / (2 * sizeof(T))
constexpr int kTailLdsBytes = 60 * 1024;
constexpr int kTailMaxLevels = 32;  // levels in one game's tail
enum { kTailPresent = 1, kTailCont = 2, kTailDense = 4, kTailNext = 8 };
template <class T>
struct TailLev {  // one level's matrices and cycle vectors
  const int* rp;
  const int* ci;
  const T* a;
  const T* d;
  T* x;
  T* y;
  T* b;
  T* r;
  const int* rrp;  // R = P^T to the next level
  const int* rci;
  const T* rv;
  const int* pc;   // P from the next level
  const T* pv;
  const T* dm;     // dense inverses (column-major blocks)
};
struct TailGL {  // one game on one level
  int r0, r1;    // its rows
  int flags;     // kTail*
  int doff;      // offset of its dense inverse (kTailDense)
};

struct Level {
  int n = 0, nnz = 0;
  int gA = 1, gR = 1;             // lanes per row of A and of R in the cycle kernels
  DBuf<int> rp, ci;
  DBuf<double> a64, dinv64;
  DBuf<float> a32, dinv32;
  // level 0 of stencil games, for the cycle kernels: slot t of row i at
  // [t * n + i] (st_w slots, zero past the row's end), its column
  // i + offset[code_t] from the row's code word (3 bits per slot, the row
  // length in bits 24..27); the slots follow the CSR order of the row
  bool stencil = false;
  int st_w = 0;
  // columns as 16-bit offsets from the row for the cycle kernels (when all fit)
  bool rel16 = false;
  bool rel16_built = false;  // ci16 written by this setup (usable once no offset overflowed)
  DBuf<int16_t> ci16;
  DBuf<uint32_t> st_code;
  DBuf<double> st64;
  DBuf<float> st32;
  std::vector<int> goff;          // per slot offsets, size G+1
  std::vector<char> present;      // slot has rows here
  std::vector<char> cont;         // slot continues to the next level
  DBuf<Tile> tiles;               // tiles of all present slots
  int ntiles = 0;
  DBuf<Tile> ctiles;              // tiles of continuing slots
  int nctiles = 0;
  int rows_tiles = 0, rows_ctiles = 0;  // rows covered by tiles / ctiles
  std::vector<Tile> h_tiles, h_ctiles;  // host copies (kept alive for async uploads)
  std::vector<int> h_blk;
  // split for the V-cycle tail: rows handled level by level (games whose tail
  // starts deeper), rows receiving their restriction that way, and the games
  // whose tail starts on this level
  DPtr<Tile> vctiles, rtiles;     // inside the engine's packed tail tables
  int nvctiles = 0, nrtiles = 0, rows_vctiles = 0, rows_rtiles = 0;
  std::vector<Tile> h_vctiles, h_rtiles;
  DPtr<int> vblk, tailg;
  int nvblk = 0, ntailg = 0;
  int tail_lds_rows = 0;  // largest sum of rows over the tail levels of a game whose tail starts here
  std::vector<int> h_vblk, h_tailg;
  bool upper = false;             // level-by-level work on this level
  // transfer to the next level (continuing slots)
  int nc = 0;
  DBuf<int> pc;                   // [n*PW], -1 = empty
  DBuf<double> pv64;
  DBuf<float> pv32;
  DBuf<int> rrp, rci;             // R = P^T, CSR over the next level's rows
  DBuf<double> rv64;
  DBuf<float> rv32;
  // Galerkin product as R (A P) (long rows): A P kept for refreshes, with
  // the identity operators it is formed with
  bool apf = false;
  int ap_nnz = 0;
  DBuf<int> ap_rp, ap_ci;
  DBuf<double> ap_v;
  DBuf<int> id_rp, id_ci, id_pc;
  DBuf<double> id_rv, id_pv;
  // Galerkin product through dense per-game blocks (small next levels)
  bool drap = false;
  long long drap_ap = 0, drap_ac = 0;  // dense entries of AP and of R A P
  int drap_maxc = 0;                    // rows of the largest game's next level
  DBuf<long long> drap_tab;       // offset tables (fine rows, coarse rows, AP, R A P), 4 x (G+1)
  DBuf<double> dap;               // the dense A P blocks, kept for refreshes
  std::vector<long long> h_drap_tab;
  // dense inverses of terminal slots: blocks (row0, size, offset into dmat)
  int nblk = 0, max_blk = 0;
  DBuf<int> blk;                  // [3*nblk]
  DBuf<double> dmat64;
  DBuf<float> dmat32;
  // cycle vectors
  DBuf<double> x64, y64, b64, r64;
  DBuf<float> x32, y32, b32, r32;
  // setup scratch
  DBuf<uint8_t> strong;           // [nnz]
  DBuf<int> st_rp, st_ci;         // transpose of the strength pattern
  DBuf<int8_t> cf;                // C/F/U state
  DBuf<uint8_t> dir;              // Dirichlet (no off-diagonal) rows
  DBuf<int> lam, cidx, tmp;
  DBuf<uint64_t> key;
  DBuf<uint8_t> chg;              // rows changed since the last setup (incremental refresh)
  DBuf<double> a_prev;            // level 0: values the hierarchy was last built from
};

struct EngineOpts {
  double eps = 0.0;
  int precision = SHAPLEY_FP64;
  int max_outer = 100000, max_inner = 100000, max_cycles = 200;
  double lin_rtol = 1e-14, lin_atol = 0.0, tie_rtol = 1e-12;
  double theta = -1.0;
  int nu1 = 2, nu2 = 2;
  double omega = 0.8;
  int coarse_max = 64, max_levels = 25;
  int verbose = 0;
  double reuse_frac = 0.05;
  double forcing = 0.0;
  int smoother = SHAPLEY_SMOOTH_JACOBI;
  int gamma = 1;
  int graph = 1;
};

// What a captured refinement cycle depends on besides device memory contents.
struct GraphKey {
  long long gen = -1;  // hierarchy generation (a full setup or a new layout starts a new one)
  bool mixed = false;
  int nu1 = 0, nu2 = 0;
  double omega = 0.0;
  int smoother = 0, gamma = 0;
  bool fused = false;
  const double* sol = nullptr;
  bool operator==(const GraphKey& o) const {
    return gen == o.gen && mixed == o.mixed && nu1 == o.nu1 && nu2 == o.nu2 && omega == o.omega &&
           smoother == o.smoother && gamma == o.gamma && fused == o.fused && sol == o.sol;
  }
};

EngineOpts engine_opts_from(const shapley_solve_opts& o, int dim);

// Per-game policy-iteration progress inside the engine.
struct SlotState {
  Game* g = nullptr;
  EngineOpts opt;
  bool need_init = true;
  bool init_alpha = false, init_beta = false;  // warm-start policies were given
  bool done = false;
  int k = 1, nk = 0;
  int inner_total = 0, cycles_total = 0;
  int status = SHAPLEY_OK;
  std::string why;  // reason of a non-OK status
  bool converged = false;
  double res = 0.0, res_l2 = 0.0;
  double res_prev = INFINITY;   // Shapley residual after the previous value step
  bool loose = false;           // the last linear solve used the forcing tolerance
  bool diverged = false;        // the last linear solve diverged
  bool exact = false;           // forcing off: cycling was seen after inexact solves
  std::vector<std::pair<uint32_t, double>> outer_hist;  // (strategy hash, residual) of outer steps
  int resolves = 0;             // consecutive accuracy re-solves at stable policies
  int solves = 0;               // value steps performed (including accuracy re-solves)
  int setups_full = 0, setups_refresh = 0;
  double setup_s = 0, cycle_s = 0, improve_s = 0;
  int levels = 0;
  double opc = 0, gc = 0;
  int inner_per_outer[64] = {0};
  double bnorm = 0.0;
};

// Per-game control of the refinement loop (FP64 residual, stop test, cycle
// count), kept on the device so that several cycles can be queued between
// two host checks.  flags: 1 forcing tolerance used, 2 stagnated (no halving
// over six cycles), 4 non-finite residual, 8 cycle limit reached, 16
// diverged (the residual grew 10^4 times past the solve's first one).
struct LinCtl {
  double rtol, atol, forcing, res_prev;
  double hist[8];  // last residual norms, entry i at hist[i % 8]
  double r0;       // the first residual norm of the solve
  int max_cycles, cyc, nh, flags;
};

// The stop test of game g after an FP64 residual: folds the residual and
// iterate maxima out of the stripes (and clears them), records them in
// norm[4g], norm[4g+1], and for an active game decides whether its solve
// stops (act[g] = 0) or takes another cycle.
__device__ inline bool lin_decide(int g, double rn, double xn, const double* __restrict__ bnorm,
                                  LinCtl* __restrict__ ctl, int* __restrict__ act, double* __restrict__ norm);
__device__ inline void lin_check_game(const Stripes& st, int g, const double* __restrict__ bnorm,
                                      LinCtl* __restrict__ ctl, int* __restrict__ act, double* __restrict__ norm) {
  double rn = 0.0, xn = 0.0;
#pragma unroll 16
  for (int k = 0; k < kStripes; ++k) {
    double* a0 = st.d + stripe_at(st, k, g, 0);
    double* a1 = st.d + stripe_at(st, k, g, 1);
    rn = fmax(rn, *a0);
    xn = fmax(xn, *a1);
    *a0 = 0.0;
    *a1 = 0.0;
  }
  lin_decide(g, rn, xn, bnorm, ctl, act, norm);
}
// The decision part of the stop test from max |r| and max |x| of game g;
// returns whether the game's solve goes on.
__device__ inline bool lin_decide(int g, double rn, double xn, const double* __restrict__ bnorm,
                                  LinCtl* __restrict__ ctl, int* __restrict__ act, double* __restrict__ norm) {
  norm[4 * g] = rn;
  norm[4 * g + 1] = xn;
  if (!act[g]) return false;
  LinCtl c = ctl[g];
  double tol = fmax(c.rtol * fmax(bnorm[g], xn), c.atol);
  int flags = c.flags & ~1;
  if (c.forcing > 0.0 && isfinite(c.res_prev) && c.res_prev > 0.0 && c.forcing * c.res_prev > tol) {
    tol = c.forcing * c.res_prev;
    flags |= 1;
  }
  const int n = c.nh;
  c.hist[n & 7] = rn;
  c.nh = n + 1;
  if (n == 0) c.r0 = rn;
  bool stop = false;
  if (!isfinite(rn)) {
    stop = true;
    flags |= 4;
  } else if (n > 0 && rn > 1e4 * c.r0 && rn > tol) {
    stop = true;  // the cycles amplify the error: no point in going on
    flags |= 16;
  } else if (rn <= tol) {
    stop = true;
  } else if (c.cyc >= c.max_cycles) {
    stop = true;
    flags |= 8;
  } else if (n + 1 >= 8 && rn > 0.5 * c.hist[(n - 6) & 7]) {
    stop = true;  // no halving over six cycles
    flags |= 2;
  }
  if (stop) act[g] = 0; else c.cyc += 1;
  c.flags = flags;
  ctl[g] = c;
  return !stop;
}

// Refinement inside the tail kernel (games whose tail starts on level 0):
// after each cycle the correction is added to sol, the FP64 residual of the
// game's rows becomes level 0's right-hand side and the stop test decides;
// up to `cycles` cycles in one launch.
struct TailRefine {
  const double* a64;   // level-0 matrix values (FP64), pattern of level 0
  const double* rhs;   // b of A v = b (FP64)
  const double* bnorm;
  LinCtl* ctl;
  int* act;            // the same flags the kernel reads, written by the stop test
  double* norm;
  int cycles;          // 0: one cycle, no refinement
};

// Lock-step policy-iteration engine over a set of games (one slot per game).
class Engine {
 public:
  explicit Engine(hipStream_t s);
  ~Engine();
  hipStream_t stream;
  std::vector<SlotState*> slots;   // not owned
  // Runs one PI step (solve + improve + decide) for every slot not done.
  // Returns the number of slots still running.
  int step();
  void invalidate_layout() { layout_dirty = true; have_hier = false; ++hier_gen; }
  int num_levels() const { return nlev; }
  int num_slots() const { return G; }
  const TailGL* tail_games() const { return d_tailgl.p; }
  const int* stencil_offsets() const { return d_st_off.p; }
  const TailLev<double>* tail_levels(double*) const { return d_tail64.p; }
  const TailLev<float>* tail_levels(float*) const { return d_tail32.p; }
  // Small host <-> device transfers go through a pinned bump arena (pageable
  // copies are staged and can wait for the whole queue); the arena is reset
  // at every synchronisation of the engine's stream.
  void sync();
  template <class T>
  void up(T* dst, const T* src, size_t n) {
    if (n == 0) return;
    void* st = pin_take(sizeof(T) * n);
    std::memcpy(st, src, sizeof(T) * n);
    SHP_HIP(hipMemcpyAsync(dst, st, sizeof(T) * n, hipMemcpyHostToDevice, stream));
  }
  // device -> pinned arena; the returned pointer is valid after sync() until
  // the next transfer
  template <class T>
  const T* down(const T* src, size_t n) {
    T* st = static_cast<T*>(pin_take(sizeof(T) * std::max<size_t>(n, 1)));
    if (n) SHP_HIP(hipMemcpyAsync(st, src, sizeof(T) * n, hipMemcpyDeviceToHost, stream));
    return st;
  }
  // Forgets the slots and the hierarchy; keeps the device buffers, so that
  // a reused engine allocates nothing for games no larger than before.
  void reset();
  // Evaluates the improvement sweep at the slots' current v (no decisions),
  // storing F(v) in the games' F arrays.
  void improve_only();
  bool keep_F = false;  // store F(v) in the sweeps (improve_only sets it)
  std::vector<int> pmis_need;        // PMIS rounds each level needed at its last setup
  double tail_cycle_bytes = 0.0;     // algorithmic bytes of one tail cycle (probe)
  bool err_pending = false;          // a refresh's error flags not read yet
  const int* refresh_errors_down();
  void refresh_errors_check(const int* pe);
  const Game* hier_game = nullptr;  // the game of a one-game hierarchy (inspection)
  // Copies level l of a one-game hierarchy to the host (synchronous): sizes,
  // A_l (CSR) and, when a coarser level exists, P_l (PW slots per row).
  void level_export(int l, int* levels, int64_t* n, int64_t* nnz, int64_t* nc, int32_t* rp, int32_t* ci,
                    double* a, int32_t* pc, double* pv);

 private:
  bool layout_dirty = true;
  char* pin = nullptr;
  std::vector<char*> pin_old;  // full arenas, released at the next sync()
  size_t pin_cap = 0, pin_used = 0;
  void* pin_take(size_t bytes);
  int G = 0, N0 = 0, NNZ0 = 0;
  std::vector<int> x_off, a_off;
  std::vector<GameDesc> hdesc;
  DBuf<GameDesc> ddesc;
  DBuf<GTile> gtiles_all, gtiles_imp;  // state tiles (assembly / improvement)
  std::vector<GTile> h_gtiles_all, h_gtiles_imp;
  int imp_threads = 256;  // workgroup size of the improvement sweep (tiles of at most this many rows)
  std::vector<Level> lv;
  int nlev = 0;
  // per-slot device scalars
  DBuf<int> d_active;
  std::vector<int> h_active_dev;              // what d_active holds
  DBuf<double> d_norm;                        // [4*G] res max, x max, b max, spare
  DBuf<double> d_shap;                        // [2*G] shapley residual max, sum sq, then cnt
  int* d_cnt = nullptr;                       // [2*G] inner/outer change counts (inside d_shap)
  DBuf<int> d_decision;
  // V-cycle tail tables (built at setup)
  DBuf<char> d_tailpack;          // all tables built by build_tail, one upload
  std::vector<char> h_tailpack;
  DPtr<TailGL> d_tailgl;
  DPtr<TailLev<double>> d_tail64;
  DPtr<TailLev<float>> d_tail32;
  std::vector<int> h_lt;  // first tail level of each game (nlev: none)
  void build_tail(bool mixed, bool allow);  // allow = false: no game takes the tail kernel
  DBuf<LinCtl> d_lin;                         // [G] controls, then the active flags
  int* d_lin_active = nullptr;                // [G] (inside d_lin)
  std::vector<LinCtl> h_linbuf;
  std::vector<LinCtl> h_lin;
  std::vector<int> h_decision;
  // striped reduction copies (kept cleared between uses)
  DBuf<double> fold_d;
  DBuf<int> fold_i;
  Stripes fold{nullptr, nullptr, 0};
  std::vector<int> h_active, h_lin_active;
  // refinement storage on the merged level 0
  DBuf<double> sol, rhs, d_bnorm;
  DBuf<int> d_st_off;  // stencil offsets of each slot's game, kStencilMax per slot
  // assembled level 0: the pair each row was built for and its 1/a_ii;
  // asm_stale forces a rebuild of every row (new layout, new games, other
  // precision)
  DBuf<int> asm_pol;
  DBuf<double> asm_dinv;
  bool asm_stale = true;
  bool asm_mixed = false;
  std::array<const void*, 9> asm_bufs{};  // level-0 buffers the rows were built in
  // setup scratch
  DBuf<int> s_cnt, s_cursor, s_scan, s_err, s_left, s_newc, s_gidx, s_gout, s_goff;
  DBuf<int> s_toff, s_tcol;   // Galerkin product scratch rows (offsets, columns)
  DBuf<int> s_big;            // Galerkin product: rows left to the workgroup kernel
  DBuf<int> s_list;           // refresh: count, then the changed coarse rows
  DBuf<int> s_defer;          // interpolation: rows left to the larger instance
  DBuf<int> s_rel;            // per level: a column offset does not fit 16 bits
  DBuf<double> s_tval;        // and values
  DBuf<double> s_dac;         // dense Galerkin product scratch: R A P
  DBuf<uint8_t> s_dapt, s_dacf;  // and their structural flags
  DBuf<Tile> s_tiles;
  DBuf<double> s_dense;
  DBuf<double> s_tune;  // lane-count tuning: output of the timed sweeps
  DBuf<int> s_ones;     // lane-count tuning: every game active
 public:
  std::vector<std::pair<std::string, double>> prof;  // phase profile (SHAPLEY_PROFILE=1)
 private:

  void build_layout();
  std::vector<int> running_slots() const;
  void run_init(const std::vector<int>& run);
  void assemble(const std::vector<int>& run, bool mixed);
  void setup(const std::vector<int>& run, const EngineOpts& o);
  void refresh(const EngineOpts& o);
  // hierarchy reuse across policy-iteration steps
  bool have_hier = false;
  std::vector<int> run_at_setup;
  int64_t changes_since_setup = 0, changes_since_refresh = 0;
  int last_cycles = 0, cycles_after_full = -1;
  bool stagnated = false;  // a linear solve stalled: rebuild the hierarchy
  // the refinement cycle captured as a HIP graph for the current hierarchy
  long long hier_gen = 0;
  hipGraphExec_t cyc_exec = nullptr;
  GraphKey cyc_key;
  void drop_graph();
 public:
  int full_setups = 0, refreshes = 0;
 private:
  void solve_linear(const std::vector<int>& run, const EngineOpts& o);
  void improve(const std::vector<int>& run, double tie_rtol);
  void apply_decisions(const std::vector<int>& code);
  void build_tiles(Level& L, const std::vector<char>& keep, bool cont_only);
  // lanes per row of level L's relaxation and residual sweeps (row sums do
  // not depend on it): timed on large levels, cached per size class
  int tune_lanes(Level& L, bool mixed);
};

// Forced lanes per sparse row in the cycle kernels (0: tuned per level).
void set_forced_lanes(int lanes);
int forced_lanes();
void set_forced_rap_cols(int mode);  // Galerkin kernel family, -1: automatic
void set_interp_mode(int mode);      // coarse-level interpolation kernels, -1: automatic
void set_stencil_mode(int mode);     // level 0 in the stencil form: -1 where it applies, 0 never

// Engines (with their device workspace) are kept per game stream between
// solves; a lease takes the idle engine of a stream or makes one, and gives
// it back unless the solve failed or `keep` is false (a caller's stream,
// whose lifetime the library does not know).  Destroying a game drops the
// engine of its stream first.
class EngineLease {
 public:
  EngineLease(hipStream_t s, bool keep);
  ~EngineLease();
  Engine& operator*() { return *e_; }
  Engine* operator->() { return e_.get(); }
 private:
  std::unique_ptr<Engine> e_;
  hipStream_t s_;
  bool keep_;
  int uncaught_;
};
void games_alive_add(int delta);      // game handles created (+1) / destroyed (-1)
void engine_cache_drop(hipStream_t s);  // before a stream is destroyed
Engine* engine_cached(hipStream_t s);   // the idle engine cached for s, or null

// FAMGpi transfers between two grid levels of the same game family.
void fmg_transfer(Game* coarse, Game* fine, hipStream_t s);

// kernels launched by the engine (defined in the .hip files)
void launch_layout(const GameDesc* d, const GTile* t, int nt, int* rp0, int* ci0, int N0, int NNZ0,
                   hipStream_t s);
void launch_gather_v(const GameDesc* d, const GTile* t, int nt, const int* active, double* x0,
                     hipStream_t s);
void launch_scatter_v(const GameDesc* d, const GTile* t, int nt, const int* active, const double* x0,
                      hipStream_t s);
// Rows whose (alpha, beta) equals pol[X] are kept (pol = -1: rebuild); the
// rebuilt rows record their pair in pol and 1/a_ii in dbuilt.  st64/st32
// (may be null): the rows also in the stencil form (st_w slots of stride N).
void launch_assemble(const GameDesc* d, const GTile* t, int nt, const int* active, double* a64, float* a32,
                     double* b0, double* dinv64, float* dinv32, int* pol, double* dbuilt, double* st64,
                     float* st32, int st_w, int N, Stripes bnorm, hipStream_t s);
// Offsets of a level-0 pattern (out: [0] overflow flag, [1] longest row,
// [2 ..] a kStencilHash-slot table of the distinct offsets, INT_MIN = empty;
// cleared here).
void launch_stencil_scan(const int* urp, const int* uci, int n, int* out, hipStream_t s);
// Code words of the merged level-0 rows (offsets of each slot's game in
// off[kStencilMax * slot]).
void launch_stencil_codes(const GameDesc* d, const GTile* t, int nt, const int* off, uint32_t* code,
                          hipStream_t s);
void launch_improve(const GameDesc* d, const GTile* t, int nt, const int* active, double tie_rtol,
                    Stripes red, int threads, hipStream_t s);
int improve_threads(int max_rows_per_state, int want);
// The same sweep over one game passed by value, tiles computed from the block
// index (no work list in memory); alpha/beta/beta_in/F may be null (no
// incumbents, outputs not stored); its reductions fold into red as game 0.
void launch_improve_flat(const GameDesc& d, double tie_rtol, Stripes red, hipStream_t s);
int improve_states_per_tile(int m1, int m2, int threads);
// the entry range [e0, e1) of each improvement tile's rows, from the games' row pointers
void launch_tile_entries(const GameDesc* d, GTile* t, int nt, hipStream_t s);
void launch_fold_finish(Stripes st, int G, int nd, unsigned sum_mask, int ni, double* out_d, int sd, int* out_i,
                        int si, hipStream_t s);
// combines the FP64-residual stripes (max |r|, max |x|) and takes the stop
// decision of each game whose lin_active flag is set
void launch_lin_check(Stripes st, int G, const double* bnorm, LinCtl* ctl, int* lin_active, double* norm,
                      hipStream_t s);
void launch_apply(const GameDesc* d, const GTile* t, int nt, const int* decision, hipStream_t s);
void launch_union_count(const int* rp, const int* ci, int n, int m1, int m2, int* cnt, int* err,
                        hipStream_t s);
void launch_union_fill(const int* rp, const int* ci, int n, int m1, int m2, const int* urp, int* uci,
                       hipStream_t s);
void launch_fmg(const Game* c, const Game* f, hipStream_t s);

// Checks of a game given in device memory (error bits kChk*; synchronises s).
enum {
  kChkRp0 = 1, kChkRp = 2, kChkCol = 4, kChkW = 8, kChkSum = 16, kChkR = 32, kChkEmpty = 64,
  kChkUnsorted = 128
};
int check_game_device(const int64_t* rp, const int32_t* ci, const double* w, const double* r,
                      const uint8_t* valid, int n, int K, int64_t nnz, int* err_dev, hipStream_t s);
void launch_rp_narrow(const int64_t* in, int* out, int m, hipStream_t s);
void launch_sort_pairs(const int* rp, int* ci, double* w, int nrows, hipStream_t s);
// Warm-start strategies (device arrays; beta may be null) against the game:
// bit 1 alpha unavailable or out of range, bit 2 beta or the pair invalid.
// Checks solve options (EINVAL).
void check_solve_opts(const shapley_solve_opts& o);
// Checks warm-start strategies (host arrays) of game g; throws EINVAL.
void check_warm_start(Game* g, const int32_t* alpha0, const int32_t* beta0, hipStream_t s);
int check_policy_device(const int* alpha, const int* beta, const uint8_t* valid, int n, int m1, int m2,
                        int* err_dev, hipStream_t s);

// device scan (exclusive) of n ints into out (out may alias in):
// out[i] = in[0] + ... + in[i-1] for i < n.  in[n-1] reaches no output, so a
// count array scanned over n = rows + 1 entries (out[rows] = the total) needs
// no zero in its last slot
void scan_exclusive(const int* in, int* out, int n, hipStream_t s, DBuf<int>& scratch);

}  // namespace shp

// payload of the opaque game handle of the C ABI
struct shapley_game_s {
  shp::Game* g;
};
