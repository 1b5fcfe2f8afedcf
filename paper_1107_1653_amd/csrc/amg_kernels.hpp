// Launchers of the AMG setup and cycle kernels.
#pragma once

#include "internal.hpp"

namespace shp {

// lam[0..n] = 0, cf[0..n) = -2, dir[0..n) = 1, strong[0..nnz) = 0
void amg_level_init(int n, int nnz, int* lam, int8_t* cf, uint8_t* dir, uint8_t* strong, hipStream_t s);
// Relaxation data of the tiles' rows in one pass, g lanes per row: Dirichlet
// flag (no nonzero off-diagonal entry), 1/a_ii (kept from d64 when
// keep_diag), divided by omega on Dirichlet rows.
// only: rows with a nonzero flag (others keep their data), or null for all
void amg_diag_dir(const Tile* t, int nt, const int* rp, const int* ci, const double* a, bool keep_diag,
                  double inv_omega, uint8_t* dir, double* d64, float* d32, int g, hipStream_t s,
                  const uint8_t* only = nullptr);
// lanes per row: 1, 4, or 64 (one wavefront per row, levels whose rows are long)
void amg_strength(const Tile* t, int nt, const int* rp, const int* ci, const double* a,
                  const uint8_t* dir, double theta, uint8_t* strong, int* lam, int lanes, hipStream_t s);
void amg_strength_t(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                    const int* st_rp, int* cursor, int* st_ci, int lanes, hipStream_t s);
void amg_pmis_init(const Tile* t, int nt, const int* goff, const uint8_t* dir, const int* lam,
                   uint32_t salt, int8_t* cf, uint64_t* key, hipStream_t s);
void amg_pmis_select(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                     const int* st_rp, const int* st_ci, const int8_t* cf, const uint64_t* key,
                     int* newc, int* left, int round, bool wide, hipStream_t s);
void amg_pmis_update(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                     int8_t* cf, const int* newc, int* left, int round, bool wide, hipStream_t s);
// all PMIS rounds of a small level (tiles covering at most kPmisSmallRows rows,
// one row per thread) in one workgroup; left[0] = points still undecided (0:
// done), left[2] = rounds run
constexpr int kPmisSmallRows = 1024;
void amg_pmis_small(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong, const int* st_rp,
                    const int* st_ci, int8_t* cf, const uint64_t* key, int* newc, int* left, int max_rounds,
                    hipStream_t s);
// PMIS round `round` (0, 1, ...): left[0..1] hold the undecided counts of the
// last two rounds; a round after one that left nothing undecided does nothing
// and lowers left[2] (set to a large value before round 0) to its number
void amg_fill_cf(const Tile* t, int nt, int8_t* cf, int8_t val, hipStream_t s);
void amg_is_c(const int8_t* cf, int* out, int n, hipStream_t s);
void amg_gather_int(const int* src, const int* idx, int m, int* dst, hipStream_t s);
void amg_interp(const Tile* t, int nt, const int* rp, const int* ci, const double* a, const double* dinv,
                const uint8_t* strong, const int8_t* cf, const int* cidx, const uint8_t* dir, int* pc,
                double* pv, int* capped, int wave, int* defer, int rows, hipStream_t s);
// wave: 0 thread per row (level 0), 1 or 2 wavefront per row (small and
// large LDS sets), 3 four lanes per row first and the wavefront kernels for
// the rows it hands on (the same weights as 1); defer: scratch of
// 2 (rows + 1) ints, rows: rows covered by the tiles
void amg_pt_count(const Tile* t, int nt, const int* pc, int* cnt, hipStream_t s);
void amg_pt_fill(const Tile* t, int nt, const int* pc, const double* pv, const int* rrp, int* cursor,
                 int* rci, double* rv, hipStream_t s);
void amg_sort_rows(const int* rp, int* ci, double* v, int n, hipStream_t s);
constexpr int kRapMaxCols = 1024;  // distinct columns of one coarse row
// Galerkin product (`big`: scratch of nc + 1 ints).  Full setup: bounds -> exclusive scan into toff ->
// fused (row lengths into tcnt, rows into the scratch tcol/tval) -> scan of
// tcnt into the coarse row pointers -> compaction.  Refresh: values of the
// rows flagged in `only` (all when null) into the existing pattern.
void amg_rap_bound(int nc, const int* rrp, const int* rci, const int* rp, int* ub, int pw, hipStream_t s);
// R = I (CSR, n rows) and P = I (ELL width PW) over n rows: the Galerkin
// kernels with these operands compute A P (R = I) and R (AP) (P = I) exactly
// (every product is multiplied by 1.0)
void amg_identity_ops(int n, int* rrp, int* rci, double* rv, int* pc, double* pv, hipStream_t s);
// levels averaging at least this many entries per row form A P first (the
// rows of P are then read once per fine row, not once per coarse row reaching
// it) and R (AP) after
constexpr int kApRowLen = 16;
// The row-wise Galerkin product.  big: scratch of 2 (nc + 1) ints.  kern:
// the kernel that takes the rows that fit it first (the wavefront kernel
// alone, a thread per row with up to 16 or 32 columns, four lanes per row
// with up to 32 or 64); the result is the same bit for bit either way.
enum { kGalWave = 0, kGalThread16 = 1, kGalThread32 = 2, kGalQuad32 = 3, kGalQuad64 = 4 };
void amg_rap_fused(int nc, const int* rrp, const int* rci, const double* rv, const int* rp, const int* ci,
                   const double* a, const int* pc, const double* pv, const int* toff, int* tcnt, int* tcol,
                   double* tval, int* err, int* big, hipStream_t s, int kern = kGalWave);
void amg_rap_compact(int nc, const int* toff, const int* tcol, const double* tval, const int* crp, int* cci,
                     double* cval, hipStream_t s);
// list: scratch of nc + 1 ints; with `only`, large levels run the flagged rows
// from a list on a fixed grid
void amg_rap_known(int nc, const int* rrp, const int* rci, const double* rv, const int* rp, const int* ci,
                   const double* a, const int* pc, const double* pv, const int* crp, const int* cci, double* cval,
                   int* err, int* big, hipStream_t s, const uint8_t* only, int* list = nullptr, int kern = kGalWave);
// Galerkin product of a small level through dense per-game blocks.  tab
// holds four tables of G + 1 offsets: fine rows, coarse rows, AP entries
// (sum of n_f * n_c over the games before) and coarse dense entries (sum of
// n_c^2).  nf, nc: rows of the level and of the next one; maxc: the largest
// n_c of a game (<= kDrapMaxCols).  ap/apt: [ap_total] scratch, ac/acf: [ac_total] scratch.  Full
// setup: amg_drap_full (row lengths into cnt), scan of cnt into the coarse
// row pointers, amg_drap_compact.  Refresh: amg_drap_known.
constexpr int kDrapMaxCols = 2048;             // coarse rows of one game (LDS row of the AP kernel)
constexpr long long kDrapMaxEntries = 1 << 25;  // sum over games of n_f * n_c, and of n_c^2
// A level takes the dense blocks when its games' next levels are small
// (<= 1024 rows, <= 2^21 dense entries) or when its rows are long (>=
// kDrapRowLen entries on average) and the dense AP is at most kDrapDensity
// times the products of the row-wise path (dense coarse operators, e.g. 3-D
// coarse levels)
constexpr int kDrapSmallCols = 1024;
constexpr long long kDrapSmallEntries = 1 << 21;
constexpr long long kDrapRowLen = 32;
constexpr long long kDrapDensity = 16;
void amg_drap_full(int nf, int nc, int maxc, const long long* tab, int G, long long ac_total, const int* rp,
                   const int* ci, const double* a, const int* pc, const double* pv, const int* rrp, const int* rci,
                   const double* rv, double* ap, uint8_t* apt, double* ac, uint8_t* acf, int* cnt, hipStream_t s);
void amg_drap_compact(int nc, const long long* tab, int G, const double* ac, const uint8_t* acf, const int* crp,
                      int* cci, double* cval, hipStream_t s);
void amg_drap_known(int nf, int nc, int maxc, const long long* tab, int G, const int* rp, const int* ci,
                    const double* a, const int* pc, const double* pv, const int* rrp, const int* rci,
                    const double* rv, double* ap, const int* crp, const int* cci, double* cval, hipStream_t s,
                    const uint8_t* only, const uint8_t* only_f);
void amg_cast(const double* in, float* out, size_t n, hipStream_t s);
void set_dense_mode(int mode);  // -1: matrix-core sweep for blocks <= 64, 0: register Gauss-Jordan
void amg_dense_inv(const int* blk, int nblk, const int* rp, const int* ci, const double* a, double* work,
                   double* inv64, float* inv32, int* err, int max_nb, hipStream_t s,
                   const uint8_t* only = nullptr);
void amg_row_changed(const Tile* t, int nt, const int* rp, const double* a, double* prev, uint8_t* chg,
                     hipStream_t s);
void amg_mark_coarse(const Tile* t, int nt, const int* pc, const uint8_t* chg, uint8_t* cmark, hipStream_t s);

// games[k] (k < ngames) start their tail on level `l0`; the result on level l0
// is left in y when out_y, else in x; lds_rows: the largest sum over the tail
// levels of a game's rows (two LDS vectors per level)
template <class T>
void cyc_tail(const int* games, int ngames, int l0, int nlev, int G, const TailLev<T>* lv, const TailGL* gl,
              const int* act, T omega, int nu1, int nu2, int out_y, int lds_rows, hipStream_t s,
              double* sol = nullptr,  // sol: also sol += result on level l0 (FP64)
              const TailRefine* rf = nullptr);  // l0 == 0: refinement cycles in the launch

// lanes per sparse row (1 or 4) for a level with this average row length
int row_group(double avg_len);
template <class T>
void cyc_smooth(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const T* a,
                const T* dinv, const T* b, const T* xin, T* xout, T omega, int first, int g, hipStream_t s,
                double* sol = nullptr,  // sol: also sol += xout (FP64), sweeps with first == 0
                const int8_t* cf = nullptr, int cfphase = 0,  // cf: C/F half sweep (first == 0, no sol)
                const int16_t* ci16 = nullptr);  // columns as 16-bit offsets from the row (instead of ci)
// l1-Jacobi diagonal 1 / sum_j |a_ij| of the tiles' rows
void amg_l1_diag(const Tile* t, int nt, const int* rp, const double* a, double* d64, float* d32, hipStream_t s);
template <class T>
void cyc_resid(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const T* a, const T* b,
               const T* x, T* r, int g, hipStream_t s, const int16_t* ci16 = nullptr);
// columns of the tiles' rows as 16-bit offsets from the row; *over = 1 when
// one does not fit (ci16 then unusable)
void amg_rel16(const Tile* t, int nt, const int* rp, const int* ci, int16_t* ci16, int* over, hipStream_t s);
template <class T>
void cyc_restrict(const Tile* t, int nt, const int* act, const int* rrp, const int* rci, const T* rv,
                  const T* rf, T* bc, int g, hipStream_t s);
template <class T>
void cyc_prolong(const Tile* t, int nt, const int* act, const int* pc, const T* pv, const T* xc, T* x,
                 hipStream_t s);
template <class T>
void cyc_dense(const int* blk, int nblk, const int* act, const T* inv, const T* b, T* x, hipStream_t s);
template <class T>
void cyc_resid64(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const double* a,
                 const double* b, const double* x, T* rc, Stripes norm, int g, hipStream_t s);
template <class T>
void cyc_update64(const Tile* t, int nt, const int* act, const T* e, double* x, hipStream_t s);
// the same sweeps and residuals on the stencil form of level 0 (the same sums
// bit for bit); sv.off: kStencilMax offsets per game slot
struct StencilView {
  const uint32_t* code;
  const int* off;
  int w, n;
};
template <class T>
void cyc_smooth_st(const Tile* t, int nt, const int* act, const StencilView& sv, const T* a, const T* dinv,
                   const T* b, const T* xin, T* xout, T omega, int first, hipStream_t s, double* sol = nullptr);
template <class T>
void cyc_resid_st(const Tile* t, int nt, const int* act, const StencilView& sv, const T* a, const T* b, const T* x,
                  T* r, hipStream_t s);
template <class T>
void cyc_resid64_st(const Tile* t, int nt, const int* act, const StencilView& sv, const double* a, const double* b,
                    const double* x, T* rc, Stripes norm, hipStream_t s);

}  // namespace shp
