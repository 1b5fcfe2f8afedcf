// AMG kernels (Sec. 4.3): setup -- strength of connection, PMIS C/F split,
// extended+i interpolation, R = P^T, Galerkin A_{l+1} = R A_l P, dense
// inverse of the coarsest blocks -- and the cycle -- weighted Jacobi
// relaxation u <- u + omega D^{-1}(f - A u), residual, restriction,
// prolongation + correction, dense coarse solve, FP64 residual of the
// iterative refinement.  Every row kernel takes a tile list (row ranges of
// one game each) so one launch covers all games of a merged level.
#include <utility>
#include <atomic>
#include "amg_kernels.hpp"

#include <climits>

namespace shp {

// ---------------------------------------------------------------------------
// setup: Dirichlet rows (no non-zero off-diagonal) and strength
// ---------------------------------------------------------------------------
// j strongly influences i when -a_ij >= theta max_{k != i} (-a_ik) (classical
// strength for M-matrix rows); Dirichlet columns are never strong.
// lam[j] counts the rows that depend strongly on j.
__global__ void k_strength(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                           const int* __restrict__ ci, const double* __restrict__ a,
                           const uint8_t* __restrict__ dir, double theta,
                           uint8_t* __restrict__ strong, int* __restrict__ lam) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  int e0 = rp[i], e1 = rp[i + 1];
  double m = 0.0;
  if (!dir[i])
    for (int e = e0; e < e1; ++e) {
      int j = ci[e];
      if (j != i && !dir[j]) m = fmax(m, -a[e]);
    }
  for (int e = e0; e < e1; ++e) {
    int j = ci[e];
    bool s = !dir[i] && j != i && !dir[j] && m > 0.0 && -a[e] >= theta * m;
    strong[e] = s ? 1 : 0;
    if (s) atomicAdd(&lam[j], 1);
  }
}

// transpose of the strength pattern: st_ci[st_rp[j] + slot] = i for strong (i, j)
__global__ void k_strength_t(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                             const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                             const int* __restrict__ st_rp, int* __restrict__ cursor,
                             int* __restrict__ st_ci) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (strong[e]) {
      int j = ci[e];
      int pos = atomicAdd(&cursor[j], 1);
      st_ci[st_rp[j] + pos] = i;
    }
}

// the same two passes with one wavefront per row (levels with long rows):
// the row maximum by a wavefront reduction (the maximum does not depend on
// the order), the flags and counts by the lanes over the entries
__global__ __launch_bounds__(256) void k_strength_w(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ a,
                                                    const uint8_t* __restrict__ dir, double theta,
                                                    uint8_t* __restrict__ strong, int* __restrict__ lam) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / (kTileRows / 4)];
  const int i = t.r0 + (int)(bid % (kTileRows / 4)) * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= t.r1) return;  // per wavefront
  const int e0 = rp[i], e1 = rp[i + 1];
  const bool di = dir[i] != 0;
  double m = 0.0;
  if (!di)
    for (int e = e0 + lane; e < e1; e += 64) {
      const int j = ci[e];
      if (j != i && !dir[j]) m = fmax(m, -a[e]);
    }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  for (int e = e0 + lane; e < e1; e += 64) {
    const int j = ci[e];
    const bool st = !di && j != i && !dir[j] && m > 0.0 && -a[e] >= theta * m;
    strong[e] = st ? 1 : 0;
    if (st) atomicAdd(&lam[j], 1);
  }
}

// transpose with one wavefront per row (the order within a transposed row
// follows the atomics, as above; PMIS does not depend on it)
__global__ __launch_bounds__(256) void k_strength_t_w(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                      const int* __restrict__ st_rp, int* __restrict__ cursor,
                                                      int* __restrict__ st_ci) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / (kTileRows / 4)];
  const int i = t.r0 + (int)(bid % (kTileRows / 4)) * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= t.r1) return;
  for (int e = rp[i] + lane; e < rp[i + 1]; e += 64)
    if (strong[e]) {
      const int j = ci[e];
      const int pos = atomicAdd(&cursor[j], 1);
      st_ci[st_rp[j] + pos] = i;
    }
}

// ---------------------------------------------------------------------------
// PMIS (parallel maximal independent set) C/F splitting
// ---------------------------------------------------------------------------
constexpr int8_t CF_U = 0, CF_C = 1, CF_F = -1;  // -2: rows of games that end on this level

__global__ void k_pmis_init(const Tile* __restrict__ tiles, const int* __restrict__ goff,
                            const uint8_t* __restrict__ dir, const int* __restrict__ lam,
                            uint32_t salt, int8_t* __restrict__ cf, uint64_t* __restrict__ key) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  int local = i - goff[t.game];
  key[i] = ((uint64_t)(uint32_t)lam[i] << 32) | mix32((uint32_t)local ^ salt);
  cf[i] = (dir[i] || lam[i] == 0) ? CF_F : CF_U;
}

// A point joins C when its weight beats every undecided strong neighbour
// (both directions of the strength graph).
__device__ __forceinline__ int pmis_select_row(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                               const uint8_t* __restrict__ strong, const int* __restrict__ st_rp,
                                               const int* __restrict__ st_ci, const int8_t* __restrict__ cf,
                                               const uint64_t* __restrict__ key) {
  if (cf[i] != CF_U) return 0;
  const uint64_t ki = key[i];
  bool best = true;
  for (int e = rp[i]; e < rp[i + 1] && best; ++e)
    if (strong[e]) {
      const int j = ci[e];
      if (cf[j] == CF_U && key[j] >= ki) best = false;
    }
  for (int e = st_rp[i]; e < st_rp[i + 1] && best; ++e) {
    const int j = st_ci[e];
    if (cf[j] == CF_U && key[j] >= ki) best = false;
  }
  return best ? 1 : 0;
}

// New C points are fixed; an undecided point depending strongly on a C point
// becomes F.  Returns 1 when row i stays undecided.  (A neighbour being set
// concurrently is read either way with the same outcome: a new C point is
// also flagged in newc, and an F point is not C.)
__device__ __forceinline__ int pmis_update_row(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                               const uint8_t* __restrict__ strong, int8_t* __restrict__ cf,
                                               const int* __restrict__ newc) {
  if (newc[i]) {
    cf[i] = CF_C;
    return 0;
  }
  if (cf[i] != CF_U) return 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (strong[e]) {
      const int j = ci[e];
      if (cf[j] == CF_C || newc[j]) {
        cf[i] = CF_F;
        return 0;
      }
    }
  return 1;
}

__global__ void k_pmis_select(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                              const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                              const int* __restrict__ st_rp, const int* __restrict__ st_ci,
                              const int8_t* __restrict__ cf, const uint64_t* __restrict__ key,
                              int* __restrict__ newc, int* __restrict__ left, int round) {
  // the following update kernel flags undecided rows in left[round & 1];
  // once a round has left none undecided, later rounds do nothing
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    left[round & 1] = 0;
    if (round > 0 && left[(round - 1) & 1] == 0) atomicMin(&left[2], round);  // first round with nothing to do
  }
  if (round > 0 && left[(round - 1) & 1] == 0) return;
  Tile t = tiles[xcd_block()];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  newc[i] = pmis_select_row(i, rp, ci, strong, st_rp, st_ci, cf, key);
}

// `left[round & 1]` becomes nonzero when a point is still undecided (only
// zero or nonzero is read).  One write per workgroup at most, and none once
// another workgroup has set it: a count by atomics on one address serialised
// over a level's workgroups.
__device__ __forceinline__ void flag_undecided(int* left, bool mine) {
  if (mine && __hip_atomic_load(left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    __hip_atomic_store(left, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kTileRows) void k_pmis_update(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const uint8_t* __restrict__ strong,
                                                          int8_t* __restrict__ cf, const int* __restrict__ newc,
                                                          int* __restrict__ left, int round) {
  if (round > 0 && left[(round - 1) & 1] == 0) return;
  Tile t = tiles[xcd_block()];
  int i = t.r0 + threadIdx.x;
  int und = 0;
  if (i < t.r1) und = pmis_update_row(i, rp, ci, strong, cf, newc);
  const bool any = __syncthreads_or(und);
  if (threadIdx.x == 0) flag_undecided(&left[round & 1], any);
}

// The same two kernels with one wavefront per row (levels with long rows):
// the lanes test the entries, a ballot decides the row; the outcome is the
// one the kernels above give.
__global__ __launch_bounds__(256) void k_pmis_select_w(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                       const int* __restrict__ st_rp, const int* __restrict__ st_ci,
                                                       const int8_t* __restrict__ cf, const uint64_t* __restrict__ key,
                                                       int* __restrict__ newc, int* __restrict__ left, int round) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    left[round & 1] = 0;
    if (round > 0 && left[(round - 1) & 1] == 0) atomicMin(&left[2], round);
  }
  if (round > 0 && left[(round - 1) & 1] == 0) return;
  const unsigned bid = xcd_block();
  const Tile t = tiles[bid / (kTileRows / 4)];
  const int i = t.r0 + (int)(bid % (kTileRows / 4)) * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= t.r1) return;  // per wavefront
  if (cf[i] != CF_U) {
    if (lane == 0) newc[i] = 0;
    return;
  }
  const uint64_t ki = key[i];
  bool beaten = false;
  for (int e = rp[i] + lane; e < rp[i + 1] && !beaten; e += 64)
    if (strong[e]) {
      const int j = ci[e];
      beaten = cf[j] == CF_U && key[j] >= ki;
    }
  for (int e = st_rp[i] + lane; e < st_rp[i + 1] && !beaten; e += 64) {
    const int j = st_ci[e];
    beaten = cf[j] == CF_U && key[j] >= ki;
  }
  const bool any = __ballot(beaten) != 0;
  if (lane == 0) newc[i] = any ? 0 : 1;
}

__global__ __launch_bounds__(256) void k_pmis_update_w(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                       const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                       int8_t* __restrict__ cf, const int* __restrict__ newc,
                                                       int* __restrict__ left, int round) {
  if (round > 0 && left[(round - 1) & 1] == 0) return;
  const unsigned bid = xcd_block();
  const Tile t = tiles[bid / (kTileRows / 4)];
  const int i = t.r0 + (int)(bid % (kTileRows / 4)) * 4 + (int)(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= t.r1) return;
  if (newc[i]) {
    if (lane == 0) cf[i] = CF_C;
    return;
  }
  if (cf[i] != CF_U) return;
  bool hit = false;
  for (int e = rp[i] + lane; e < rp[i + 1] && !hit; e += 64)
    if (strong[e]) {
      const int j = ci[e];
      hit = cf[j] == CF_C || newc[j];
    }
  const bool any = __ballot(hit) != 0;
  if (lane == 0) {
    if (any) cf[i] = CF_F;
    else flag_undecided(&left[round & 1], true);
  }
}

// All rounds of a small level in one workgroup (rounds separated by
// workgroup barriers instead of launches; the same rounds as the two kernels
// above).  Stops after the first round that leaves no point undecided, or
// after max_rounds.  left[0] = left[1] = points still undecided, left[2] =
// rounds run.
constexpr int kPmisSmallThreads = 1024;
__global__ __launch_bounds__(kPmisSmallThreads) void k_pmis_small(
    const Tile* __restrict__ tiles, int nt, const int* __restrict__ rp, const int* __restrict__ ci,
    const uint8_t* __restrict__ strong, const int* __restrict__ st_rp, const int* __restrict__ st_ci,
    int8_t* __restrict__ cf, const uint64_t* __restrict__ key, int* __restrict__ newc, int* __restrict__ left,
    int max_rounds) {
  __shared__ int s_und[kPmisSmallThreads / 64];
  __shared__ int s_tot;
  const int tid = threadIdx.x;
  const int total = nt * kTileRows;
  int rounds = 0, und_all = 0;
  while (rounds < max_rounds) {
    for (int t = tid; t < total; t += kPmisSmallThreads) {
      const Tile tl = tiles[t / kTileRows];
      const int i = tl.r0 + t % kTileRows;
      if (i < tl.r1) newc[i] = pmis_select_row(i, rp, ci, strong, st_rp, st_ci, cf, key);
    }
    __syncthreads();
    int und = 0;
    for (int t = tid; t < total; t += kPmisSmallThreads) {
      const Tile tl = tiles[t / kTileRows];
      const int i = tl.r0 + t % kTileRows;
      if (i < tl.r1) und += pmis_update_row(i, rp, ci, strong, cf, newc);
    }
    for (int o = 32; o > 0; o >>= 1) und += __shfl_xor(und, o);
    if ((tid & 63) == 0) s_und[tid >> 6] = und;
    __syncthreads();
    if (tid == 0) {
      int sum = 0;
      for (int w = 0; w < kPmisSmallThreads / 64; ++w) sum += s_und[w];
      s_tot = sum;
    }
    __syncthreads();
    und_all = s_tot;
    ++rounds;
    if (und_all == 0) break;
  }
  if (tid == 0) {
    left[0] = und_all;
    left[1] = und_all;
    left[2] = rounds;
  }
}

__global__ void k_fill_cf(const Tile* __restrict__ tiles, int8_t* __restrict__ cf, int8_t val) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i < t.r1) cf[i] = val;
}

__global__ void k_is_c(const int8_t* __restrict__ cf, int* __restrict__ out, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cf[i] == CF_C ? 1 : 0;
}

__global__ void k_gather_int(const int* __restrict__ src, const int* __restrict__ idx, int m,
                             int* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = src[idx[i]];
}

// ---------------------------------------------------------------------------
// extended+i interpolation.  Each thread builds the interpolatory set of its
// row (the strong C neighbours, then the strong C neighbours of its strong F
// neighbours) in its own column of an LDS array -- no dynamic indexing of
// registers, no scratch, no synchronisation between threads.  When the set
// is full, later candidates are left out in that enumeration order; the
// denominators and weights then only range over the kept set, so the
// formula stays consistent.  Rows that hit the cap are counted in `capped`.
// The PW largest weights are kept and rescaled to preserve the row sum.
// ---------------------------------------------------------------------------
constexpr int kIThreads = 64;
constexpr int kIChat = 32;       // set cap of the interpolation formula
constexpr int kIChatSmall = 8;   // first pass (most rows of grid stencils fit)

// Row i.  The set lives in this thread's column of the block's LDS arrays (C,
// Wt: entry p at [p * kIThreads]).  DEFER: a row whose set would exceed CAP
// is appended to defer[1 ..] for the kIChat instance instead of being capped;
// any other row is computed exactly as by that instance.
template <int CAP, bool DEFER>
__device__ __forceinline__ void interp_lds_row(int i, int* C, double* Wt, const int* __restrict__ rp,
                                               const int* __restrict__ ci, const double* __restrict__ a,
                                               const double* __restrict__ dinv, const uint8_t* __restrict__ strong,
                                               const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                               const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                               double* __restrict__ pv, int* __restrict__ capped,
                                               int* __restrict__ defer) {
  {
    int* pci = pc + (size_t)i * PW;
    double* pvi = pv + (size_t)i * PW;
    for (int q = 0; q < PW; ++q) { pci[q] = -1; pvi[q] = 0.0; }
    if (cf[i] == CF_C) { pci[0] = cidx[i]; pvi[0] = 1.0; return; }
    if (dir[i]) return;
    int n = 0;
    bool full = false;
    auto find = [&](int v) -> int {
      for (int p = 0; p < n; ++p)
        if (C[p * kIThreads] == v) return p;
      return -1;
    };
    auto add = [&](int v) {
      if (find(v) >= 0) return;
      if (n >= CAP) { full = true; return; }
      C[n * kIThreads] = v;
      Wt[n * kIThreads] = 0.0;
      ++n;
    };
    const int e0 = rp[i], e1 = rp[i + 1];
    double aii = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int j = ci[e];
      if (j == i) { aii = a[e]; continue; }
      if (strong[e] && cf[j] == CF_C) add(j);
    }
    for (int e = e0; e < e1; ++e) {
      const int k = ci[e];
      if (k == i || !strong[e] || cf[k] != CF_F) continue;
      for (int e2 = rp[k]; e2 < rp[k + 1]; ++e2) {
        const int l = ci[e2];
        if (strong[e2] && cf[l] == CF_C) add(l);
      }
    }
    if (full) {
      if (DEFER) {
        defer[1 + atomicAdd(defer, 1)] = i;
        return;
      }
      atomicAdd(capped, 1);
    }
    if (n == 0) return;
    double dd = aii;
    for (int e = e0; e < e1; ++e) {
      const int j = ci[e];
      if (j == i) continue;
      const double aij = a[e];
      if (aij == 0.0) continue;
      const int p = find(j);
      if (p >= 0) { Wt[p * kIThreads] += aij; continue; }
      if (strong[e] && cf[j] == CF_F) {
        // distribute a_ij over the kept set through row k = j
        const int k = j;
        const bool kpos = dinv[k] >= 0.0;
        double den = 0.0;
        for (int e2 = rp[k]; e2 < rp[k + 1]; ++e2) {
          const int l = ci[e2];
          if (l == k) continue;
          const double akl = a[e2];
          const double abar = kpos ? (akl < 0.0 ? akl : 0.0) : (akl > 0.0 ? akl : 0.0);
          if (abar != 0.0 && (l == i || find(l) >= 0)) den += abar;
        }
        if (den == 0.0) { dd += aij; continue; }
        for (int e2 = rp[k]; e2 < rp[k + 1]; ++e2) {
          const int l = ci[e2];
          if (l == k) continue;
          const double akl = a[e2];
          const double abar = kpos ? (akl < 0.0 ? akl : 0.0) : (akl > 0.0 ? akl : 0.0);
          if (abar == 0.0) continue;
          if (l == i) { dd += aij * abar / den; continue; }
          const int p2 = find(l);
          if (p2 >= 0) Wt[p2 * kIThreads] += aij * abar / den;
        }
        continue;
      }
      if (dir[j]) continue;  // Dirichlet neighbour: its error vanishes after relaxation
      dd += aij;             // weak connection: lumped into the diagonal
    }
    if (dd == 0.0) return;
    double total = 0.0;
    for (int p = 0; p < n; ++p) {
      const double w = -Wt[p * kIThreads] / dd;
      Wt[p * kIThreads] = w;
      total += w;
    }
    // the PW largest |w| (lowest position first on ties)
    int kc[PW];
    double kw[PW];
    int nk = 0;
    uint32_t used = 0u;
    for (int q = 0; q < PW; ++q) {
      int best = -1;
      double bw = 0.0;
      for (int p = 0; p < n; ++p) {
        const double aw = fabs(Wt[p * kIThreads]);
        if (!((used >> p) & 1u) && aw > bw) { best = p; bw = aw; }
      }
      if (best < 0) break;
      used |= 1u << best;
      kc[q] = cidx[C[best * kIThreads]];
      kw[q] = Wt[best * kIThreads];
      ++nk;
    }
    double kept = 0.0;
    for (int q = 0; q < nk; ++q) kept += kw[q];
    const double sc = (kept != 0.0) ? total / kept : 1.0;
    // insertion sort of the kept entries by coarse column
    for (int u = 1; u < nk; ++u) {
      const int c0 = kc[u];
      const double w0 = kw[u];
      int v = u - 1;
      while (v >= 0 && kc[v] > c0) { kc[v + 1] = kc[v]; kw[v + 1] = kw[v]; --v; }
      kc[v + 1] = c0;
      kw[v + 1] = w0;
    }
    for (int q = 0; q < nk; ++q) { pci[q] = kc[q]; pvi[q] = kw[q] * sc; }
  }
}

// one thread per row of the tiles (kTileRows / kIThreads blocks per tile)
template <int CAP, bool DEFER>
__global__ __launch_bounds__(kIThreads) void k_interp_lds(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                          const int* __restrict__ ci, const double* __restrict__ a,
                                                          const double* __restrict__ dinv,
                                                          const uint8_t* __restrict__ strong,
                                                          const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                                          const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                          double* __restrict__ pv, int* __restrict__ capped,
                                                          int* __restrict__ defer) {
  __shared__ int lc[CAP * kIThreads];
  __shared__ double lw[CAP * kIThreads];
  const unsigned bid = xcd_block();
  const Tile t = tiles[bid / (kTileRows / kIThreads)];
  const int sub = bid % (kTileRows / kIThreads);
  const int i = t.r0 + sub * kIThreads + (int)threadIdx.x;
  if (i >= t.r1) return;
  interp_lds_row<CAP, DEFER>(i, lc + threadIdx.x, lw + threadIdx.x, rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv,
                             capped, defer);
}

// the rows deferred by the small-set instance, one thread each
__global__ __launch_bounds__(kIThreads) void k_interp_lds_list(const int* __restrict__ list,
                                                               const int* __restrict__ rp, const int* __restrict__ ci,
                                                               const double* __restrict__ a,
                                                               const double* __restrict__ dinv,
                                                               const uint8_t* __restrict__ strong,
                                                               const int8_t* __restrict__ cf,
                                                               const int* __restrict__ cidx,
                                                               const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                               double* __restrict__ pv, int* __restrict__ capped) {
  __shared__ int lc[kIChat * kIThreads];
  __shared__ double lw[kIChat * kIThreads];
  const int cnt = list[0];
  for (int k = blockIdx.x * kIThreads + (int)threadIdx.x; k < cnt; k += gridDim.x * kIThreads)
    interp_lds_row<kIChat, false>(list[1 + k], lc + threadIdx.x, lw + threadIdx.x, rp, ci, a, dinv, strong, cf, cidx,
                                  dir, pc, pv, capped, nullptr);
}

// ---------------------------------------------------------------------------
// extended+i interpolation, one wavefront per row (coarse levels, whose rows
// are long).  Same formula as above without the set cap: the interpolatory
// set (strong C neighbours and strong C neighbours of strong F neighbours)
// is collected in an LDS hash and sorted; the sums run in fixed orders:
//   * den_k (row k's same-sign entries towards the set and i): per k in row
//     order, from pair terms staged in LDS;
//   * the weight of a set member: direct entry first, then the distributed
//     entries in the order of the F neighbours k in row i;
//   * the lumped diagonal and the total: per lane, then a fixed tree.
// A row with more than kIwK strong F neighbours or more than the hash holds
// falls back to direct interpolation (its strong C neighbours only, strong F
// neighbours lumped) and is counted in `capped`.
// ---------------------------------------------------------------------------
// HASH: slots for the interpolatory set of one row; KCAP: strong F
// neighbours of one row; STAGE: (k, entry) pairs staged at a time (the sums
// take their terms in the same order for any STAGE).

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// DEFER: a row that does not fit is appended to defer[1 ..] (count in
// defer[0]) and left to a larger instance, instead of falling back to direct
// interpolation; the larger instance then computes exactly what it computes
// for any row.
template <int kIwHash, int kIwK, int STAGE, bool DEFER>
__device__ __forceinline__ void interp_row(int i, const int* __restrict__ rp, const int* __restrict__ ci,
                                           const double* __restrict__ a, const double* __restrict__ dinv,
                                           const uint8_t* __restrict__ strong, const int8_t* __restrict__ cf,
                                           const int* __restrict__ cidx, const uint8_t* __restrict__ dir,
                                           int* __restrict__ pc, double* __restrict__ pv, int* __restrict__ capped,
                                           int* __restrict__ defer) {
  __shared__ int hkey[kIwHash];
  __shared__ int hpos[kIwHash];
  __shared__ int mem[kIwHash];
  __shared__ double W[kIwHash];
  __shared__ int kcol[kIwK], kbeg[kIwK], koff[kIwK + 1];
  __shared__ double kaik[kIwK], kden[kIwK], kabi[kIwK];
  __shared__ uint8_t kneg[kIwK];
  __shared__ int sq[STAGE];
  __shared__ double sc[STAGE];
  __shared__ int full_sh;

  const int lane = threadIdx.x;
  if (lane < PW) {
    pc[(size_t)i * PW + lane] = -1;
    pv[(size_t)i * PW + lane] = 0.0;
  }
  const int8_t cfi = cf[i];
  if (cfi == CF_C) {
    if (lane == 0) { pc[(size_t)i * PW] = cidx[i]; pv[(size_t)i * PW] = 1.0; }
    return;
  }
  if (dir[i]) return;
  const int e0 = rp[i], len = rp[i + 1] - e0;
  const unsigned hmask = kIwHash - 1;

  auto insert = [&](int v) -> bool {
    unsigned h = mix32((uint32_t)v) & hmask;
    for (int pr = 0; pr < kIwHash; ++pr) {
      const int old = atomicCAS(&hkey[h], -1, v);
      if (old == -1 || old == v) return true;
      h = (h + 1) & hmask;
    }
    return false;
  };
  auto lookup = [&](int v) -> int {
    unsigned h = mix32((uint32_t)v) & hmask;
    for (int pr = 0; pr < kIwHash; ++pr) {
      const int k = hkey[h];
      if (k == v) return hpos[h];
      if (k == -1) return -1;
      h = (h + 1) & hmask;
    }
    return -1;
  };

  bool direct = false;  // fallback: strong C neighbours only
  for (int attempt = 0; attempt < 2; ++attempt) {
    for (int h = lane; h < kIwHash; h += 64) hkey[h] = -1;
    if (lane == 0) full_sh = 0;
    __syncthreads();
    // ---- row i: strong C neighbours into the set, strong F neighbours listed in row order
    int nK = 0;
    bool bad = false;
    for (int base = 0; base < len; base += 64) {
      const bool in = base + lane < len;
      const int e = e0 + base + lane;
      int j = -1;
      bool st = false;
      double aij = 0.0;
      if (in) { j = ci[e]; st = strong[e] != 0; aij = a[e]; }
      const bool off = in && st && j != i;
      const int8_t cj = off ? cf[j] : (int8_t)0;
      if (off && cj == CF_C && !insert(j)) bad = true;
      const bool isF = !direct && off && cj == CF_F;
      const unsigned long long m = __ballot(isF);
      const int pos = nK + __popcll(m & ((1ull << lane) - 1ull));
      if (isF && pos < kIwK) { kcol[pos] = j; kaik[pos] = aij; }
      nK += __popcll(m);
    }
    if (bad) atomicOr(&full_sh, 1);
    if (nK > kIwK) atomicOr(&full_sh, 1);
    __syncthreads();
    if (full_sh) {
      if (DEFER) {
        if (lane == 0) defer[1 + atomicAdd(defer, 1)] = i;
        return;
      }
      if (lane == 0) atomicAdd(capped, 1);
      if (direct) return;  // even the direct set does not fit: no interpolation
      direct = true;
      __syncthreads();
      continue;
    }
    // ---- rows of the strong F neighbours: offsets of their entries
    int T = 0;
    for (int base = 0; base < nK; base += 64) {
      const int p = base + lane;
      int ln = 0;
      if (p < nK) {
        const int k = kcol[p];
        const int b = rp[k];
        ln = rp[k + 1] - b;
        kbeg[p] = b;
        kneg[p] = dinv[k] < 0.0 ? 1 : 0;
        kden[p] = 0.0;
        kabi[p] = 0.0;
      }
      int v = ln;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
      }
      if (p < nK) koff[p + 1] = T + v;
      T += __shfl(v, 63);
    }
    if (lane == 0) koff[0] = 0;
    __syncthreads();
    auto seg = [&](int f) {  // largest p with koff[p] <= f
      int lo = 0, hi = nK - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (koff[mid] <= f) lo = mid; else hi = mid - 1;
      }
      return lo;
    };
    // ---- distance-two candidates
    bad = false;
    for (int f = lane; f < T; f += 64) {
      const int p = seg(f);
      const int e2 = kbeg[p] + (f - koff[p]);
      const int l = ci[e2];
      if (strong[e2] && l != kcol[p] && cf[l] == CF_C && !insert(l)) bad = true;
    }
    if (bad) atomicOr(&full_sh, 1);
    __syncthreads();
    if (full_sh) {
      if (DEFER) {
        if (lane == 0) defer[1 + atomicAdd(defer, 1)] = i;
        return;
      }
      if (lane == 0) atomicAdd(capped, 1);
      if (direct) return;
      direct = true;
      __syncthreads();
      continue;
    }
    // ---- members: compact and sort by fine index
    int m = 0;
    for (int base = 0; base < kIwHash; base += 64) {
      const int key = hkey[base + lane];
      const unsigned long long bm = __ballot(key >= 0);
      if (key >= 0) mem[m + __popcll(bm & ((1ull << lane) - 1ull))] = key;
      m += __popcll(bm);
    }
    int P2 = 1;
    while (P2 < m) P2 <<= 1;
    for (int h = m + lane; h < P2; h += 64) mem[h] = INT_MAX;
    __syncthreads();
    for (int k2 = 2; k2 <= P2; k2 <<= 1) {
      for (int jj = k2 >> 1; jj > 0; jj >>= 1) {
        for (int idx = lane; idx < P2; idx += 64) {
          const int ixj = idx ^ jj;
          if (ixj > idx) {
            const int x = mem[idx], y = mem[ixj];
            const bool up = (idx & k2) == 0;
            if ((x > y) == up) { mem[idx] = y; mem[ixj] = x; }
          }
        }
        __syncthreads();
      }
    }
    // position of each member in the sorted list, reachable through the hash
    for (int q = lane; q < m; q += 64) {
      const int v = mem[q];
      unsigned h = mix32((uint32_t)v) & hmask;
      while (hkey[h] != v) h = (h + 1) & hmask;
      hpos[h] = q;
      W[q] = 0.0;
    }
    __syncthreads();
    // ---- den_k and abar_ki: terms of each pair staged, summed per k in row order
    for (int c0 = 0; c0 < T; c0 += STAGE) {
      const int c1 = (T < c0 + STAGE) ? T : c0 + STAGE;
      for (int f = c0 + lane; f < c1; f += 64) {
        const int p = seg(f);
        const int e2 = kbeg[p] + (f - koff[p]);
        const int l = ci[e2];
        const double akl = a[e2];
        const double abar = kneg[p] ? (akl > 0.0 ? akl : 0.0) : (akl < 0.0 ? akl : 0.0);
        double term = 0.0;
        int q = -1;
        if (l != kcol[p] && abar != 0.0) {
          if (l == i) {
            term = abar;
            kabi[p] = abar;
          } else {
            q = lookup(l);
            if (q >= 0) term = abar;
          }
        }
        sc[f - c0] = term;
        sq[f - c0] = q;
      }
      __syncthreads();
      for (int p = lane; p < nK; p += 64) {
        const int lo = koff[p] > c0 ? koff[p] : c0;
        const int hi = koff[p + 1] < c1 ? koff[p + 1] : c1;
        double d = kden[p];
        for (int f = lo; f < hi; ++f) d += sc[f - c0];
        kden[p] = d;
      }
      __syncthreads();
    }
    // ---- diagonal: a_ii, weak entries, parts of F neighbours sent back to i;
    //      direct entries towards set members
    double ddl = 0.0;
    int rank = 0;
    for (int base = 0; base < len; base += 64) {
      const bool in = base + lane < len;
      const int e = e0 + base + lane;
      int j = -1;
      bool st = false;
      double aij = 0.0;
      if (in) { j = ci[e]; st = strong[e] != 0; aij = a[e]; }
      const bool off = in && j != i;
      const int8_t cj = off ? cf[j] : (int8_t)0;
      const bool isF = !direct && off && st && cj == CF_F;
      const unsigned long long bm = __ballot(isF);
      const int p = rank + __popcll(bm & ((1ull << lane) - 1ull));
      rank += __popcll(bm);
      if (in && j == i) ddl += aij;
      if (!off || aij == 0.0) continue;
      const int q = lookup(j);
      if (q >= 0) { W[q] += aij; continue; }  // one entry per column: no conflicts
      if (isF) {
        const double den = kden[p];
        ddl += den == 0.0 ? aij : aij * kabi[p] / den;
        continue;
      }
      if (dir[j]) continue;
      ddl += aij;
    }
    __syncthreads();
    // ---- distributed entries: F neighbours in row order; each row k holds a
    //      column at most once, so the lanes of one k never collide
    for (int c0 = 0; c0 < T; c0 += STAGE) {
      const int c1 = (T < c0 + STAGE) ? T : c0 + STAGE;
      for (int f = c0 + lane; f < c1; f += 64) {
        const int p = seg(f);
        const int e2 = kbeg[p] + (f - koff[p]);
        const int l = ci[e2];
        const double akl = a[e2];
        const double abar = kneg[p] ? (akl > 0.0 ? akl : 0.0) : (akl < 0.0 ? akl : 0.0);
        int q = -1;
        double c = 0.0;
        if (l != kcol[p] && l != i && abar != 0.0 && kden[p] != 0.0) {
          q = lookup(l);
          c = kaik[p] * abar / kden[p];
        }
        sq[f - c0] = q;
        sc[f - c0] = c;
      }
      __syncthreads();
      const int pa = seg(c0), pb = seg(c1 - 1);
      for (int p = pa; p <= pb; ++p) {
        const int lo = koff[p] > c0 ? koff[p] : c0;
        const int hi = koff[p + 1] < c1 ? koff[p + 1] : c1;
        for (int f = lo + lane; f < hi; f += 64) {
          const int q = sq[f - c0];
          if (q >= 0) W[q] += sc[f - c0];
        }
        __syncthreads();
      }
    }
    const double dd = wave_sum(ddl);
    if (dd == 0.0 || m == 0) return;
    // ---- weights, their total, the PW largest (lowest column on ties)
    double tl = 0.0;
    for (int q = lane; q < m; q += 64) {
      const double w = -W[q] / dd;
      W[q] = w;
      tl += w;
    }
    const double total = wave_sum(tl);
    int kq[PW];
    double kw[PW];
    int nk = 0;
#pragma unroll
    for (int r = 0; r < PW; ++r) {
      kq[r] = INT_MAX;
      kw[r] = 0.0;
    }
#pragma unroll
    for (int r = 0; r < PW; ++r) {
      if (nk == r) {
        double bw = 0.0;
        int bq = INT_MAX;
        for (int q = lane; q < m; q += 64) {
          bool used = false;
#pragma unroll
          for (int u = 0; u < r; ++u) used |= kq[u] == q;
          const double aw = fabs(W[q]);
          if (!used && (aw > bw || (aw == bw && aw > 0.0 && q < bq))) { bw = aw; bq = q; }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ow = __shfl_xor(bw, o);
          const int oq = __shfl_xor(bq, o);
          if (ow > bw || (ow == bw && oq < bq)) { bw = ow; bq = oq; }
        }
        if (bq != INT_MAX && bw != 0.0) {
          kq[r] = bq;
          kw[r] = W[bq];
          nk = r + 1;
        }
      }
    }
    if (lane == 0 && nk > 0) {
      double kept = 0.0;
#pragma unroll
      for (int u = 0; u < PW; ++u)
        if (u < nk) kept += kw[u];
      const double scl = kept != 0.0 ? total / kept : 1.0;
      // output sorted by column: the members are sorted by fine index and the
      // coarse numbering is increasing in the fine index
#pragma unroll
      for (int u = 0; u < PW; ++u) {
        if (u >= nk) continue;
        int r = 0;
#pragma unroll
        for (int v = 0; v < PW; ++v) r += (v < nk && kq[v] < kq[u]) ? 1 : 0;
        pc[(size_t)i * PW + r] = cidx[mem[kq[u]]];
        pv[(size_t)i * PW + r] = kw[u] * scl;
      }
    }
    return;
  }
}

// one wavefront per row of the tiles
template <int kIwHash, int kIwK, int STAGE, bool DEFER>
__global__ __launch_bounds__(64) void k_interp_wave(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ a,
                                                    const double* __restrict__ dinv,
                                                    const uint8_t* __restrict__ strong,
                                                    const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                                    const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                    double* __restrict__ pv, int* __restrict__ capped,
                                                    int* __restrict__ defer) {
  const unsigned bid = xcd_block();
  const Tile t = tiles[bid / kTileRows];
  const int i = t.r0 + (int)(bid % kTileRows);
  if (i >= t.r1) return;
  interp_row<kIwHash, kIwK, STAGE, DEFER>(i, rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv, capped, defer);
}

// the rows of a list (rows deferred by a smaller kernel), one wavefront each
// in turn; with DEFER, rows this instance cannot hold go on to defer[1 ..]
template <int kIwHash, int kIwK, bool DEFER>
__global__ __launch_bounds__(64) void k_interp_wave_list(const int* __restrict__ list, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ a,
                                                         const double* __restrict__ dinv,
                                                         const uint8_t* __restrict__ strong,
                                                         const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                                         const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                         double* __restrict__ pv, int* __restrict__ capped,
                                                         int* __restrict__ defer) {
  const int cnt = list[0];
  for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
    interp_row<kIwHash, kIwK, 256, DEFER>(list[1 + k], rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv, capped,
                                          defer);
    __syncthreads();  // the next row reuses the LDS
  }
}

// ---------------------------------------------------------------------------
// R = P^T as CSR over coarse rows (entries sorted by fine row)
// ---------------------------------------------------------------------------
__global__ void k_pt_count(const Tile* __restrict__ tiles, const int* __restrict__ pc,
                           int* __restrict__ cnt) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  for (int q = 0; q < PW; ++q) {
    int c = pc[(size_t)i * PW + q];
    if (c >= 0) atomicAdd(&cnt[c], 1);
  }
}

__global__ void k_pt_fill(const Tile* __restrict__ tiles, const int* __restrict__ pc,
                          const double* __restrict__ pv, const int* __restrict__ rrp,
                          int* __restrict__ cursor, int* __restrict__ rci, double* __restrict__ rv) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  for (int q = 0; q < PW; ++q) {
    int c = pc[(size_t)i * PW + q];
    if (c >= 0) {
      int pos = rrp[c] + atomicAdd(&cursor[c], 1);
      rci[pos] = i;
      rv[pos] = pv[(size_t)i * PW + q];
    }
  }
}


// ---------------------------------------------------------------------------
// Galerkin product A_c = R A P, one workgroup of NT threads per coarse row.
// The row's (R entry, A entry) pairs are flattened over the lanes so that
// their loads issue in parallel.  The distinct coarse columns of the row are
// either collected in an LDS hash set and sorted (full setup), or read from
// the existing coarse matrix (numeric refresh: same pattern).  The products
// of a chunk of pairs are written to LDS at fixed slots of the enumeration
// order (R entry, A entry, P slot); the lane owning an output column (column
// position mod NT) adds its products slot by slot, so the sums are
// bit-reproducible whatever the batch, the launch shape and the mode.
// Full setup: each row goes to a scratch area at an upper-bound offset with
// its length; a compaction then copies the rows into the final CSR.
// err bits: 1 hash full, 2 R row too long, 4 too many distinct columns.
// ---------------------------------------------------------------------------
constexpr int kRapRCap = 256;      // max entries of one R row
constexpr int kRapHash = 2048;     // hash slots (>= 2 x products when possible)
constexpr int kRapND = kRapMaxCols;  // max distinct columns of one coarse row
enum { kRapFused = 0, kRapKnown = 1 };

// LDS ordering between the lanes of one wavefront
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ascending bitonic sort of one value per lane across a wavefront (64 lanes)
__device__ inline void wave_sort64(int& key, double& val) {
  const int lane = threadIdx.x & 63;
  for (int k2 = 2; k2 <= 64; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      const int ok = __shfl_xor(key, j);
      const double ov = __shfl_xor(val, j);
      const bool up = (lane & k2) == 0;
      const bool low = (lane & j) == 0;
      if ((up == low) ? (ok < key) : (ok > key)) {
        key = ok;
        val = ov;
      }
    }
  }
}
__device__ inline void wave_sort64(int& key) {
  const int lane = threadIdx.x & 63;
  for (int k2 = 2; k2 <= 64; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      const int ok = __shfl_xor(key, j);
      const bool up = (lane & k2) == 0;
      const bool low = (lane & j) == 0;
      if ((up == low) ? (ok < key) : (ok > key)) key = ok;
    }
  }
}

// rows of R = P^T sorted by column, 16 lanes per row: a row of up to 64
// entries is staged in LDS and each entry written at its rank (the columns
// of a row are distinct); longer rows, rare, by one lane
__global__ __launch_bounds__(256) void k_sort_rows_seg(const int* __restrict__ rp, int* __restrict__ ci,
                                                       double* __restrict__ v, int n) {
  __shared__ int sk[16][64];
  __shared__ double sv[16][64];
  const int seg = threadIdx.x >> 4, l = threadIdx.x & 15;
  const int I = blockIdx.x * 16 + seg;
  if (I >= n) return;  // nothing below synchronises the workgroup
  const int e0 = rp[I], len = rp[I + 1] - e0;
  if (len <= 64) {
    for (int j = l; j < len; j += 16) {
      sk[seg][j] = ci[e0 + j];
      sv[seg][j] = v[e0 + j];
    }
    wave_lds_sync();
    for (int j = l; j < len; j += 16) {
      const int key = sk[seg][j];
      int r = 0;
      for (int t = 0; t < len; ++t) r += sk[seg][t] < key ? 1 : 0;
      ci[e0 + r] = key;
      v[e0 + r] = sv[seg][j];
    }
    return;
  }
  if (l != 0) return;
  for (int e = e0 + 1; e < e0 + len; ++e) {
    const int c = ci[e];
    const double x = v[e];
    int f = e - 1;
    while (f >= e0 && ci[f] > c) { ci[f + 1] = ci[f]; v[f + 1] = v[f]; --f; }
    ci[f + 1] = c;
    v[f + 1] = x;
  }
}

// ascending bitonic sort of 128 keys, elements `lane` (k0) and `lane + 64`
// (k1) of each lane
__device__ inline void wave_sort128(int& k0, int& k1) {
  const int lane = threadIdx.x & 63;
  for (int k2 = 2; k2 <= 128; k2 <<= 1) {
    for (int j = k2 >> 1; j > 0; j >>= 1) {
      if (j == 64) {  // partners in the same lane; k2 = 128: ascending
        const int lo = k0 < k1 ? k0 : k1, hi = k0 < k1 ? k1 : k0;
        k0 = lo;
        k1 = hi;
        continue;
      }
      const int o0 = __shfl_xor(k0, j), o1 = __shfl_xor(k1, j);
      const bool low = (lane & j) == 0;
      const bool up0 = (lane & k2) == 0, up1 = ((lane + 64) & k2) == 0;
      if ((up0 == low) ? (o0 < k0) : (o0 > k0)) k0 = o0;
      if ((up1 == low) ? (o1 < k1) : (o1 > k1)) k1 = o1;
    }
  }
}

__device__ inline int rap_locate(const int* rO, int P, int f) {
  int lo = 0, hi = P - 1;  // largest p with rO[p] <= f
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (rO[mid] <= f) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The cnt (1..64) queued products at queue counter head (positions qpos,
// values qval, ring of mask + 1 entries) into the sums acc[position]: the run
// is sorted by (position, queue order) on keys alone, and the first product
// of each position adds the position's products of the run to its sum one
// after the other, so each sum takes its products in queue order.  Positions
// of one run are owned by this wavefront alone.
__device__ __forceinline__ void rap_run(int cnt, int head, const int* __restrict__ qpos,
                                        const double* __restrict__ qval, int mask, double* __restrict__ acc) {
  const int lane = threadIdx.x & 63;
  const int idx = (head + lane) & mask;
  const bool live = lane < cnt;
  const double v = live ? qval[idx] : 0.0;
  int key = live ? (qpos[idx] << 6) | lane : INT_MAX;
  wave_sort64(key);
  const double x = __shfl(v, key & 63);  // the product now at this lane
  const int pos = key >> 6;
  const int prev = __shfl_up(pos, 1);
  const bool first = lane == 0 || prev != pos;
  const bool edge = key != INT_MAX && first;  // first product of a position
  const unsigned long long bounds = __ballot(first);
  const unsigned long long above = lane == 63 ? 0ull : (bounds >> (lane + 1));
  const int len = above ? __ffsll((long long)above) : 64 - lane;
  int most = edge ? len : 0;
  for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
  double sum = edge ? acc[pos] : 0.0;
  for (int j = 0; j < most; ++j) {
    const double y = __shfl(x, lane + j);
    if (edge && j < len) sum += y;
  }
  if (edge) acc[pos] = sum;
  wave_lds_sync();
}

// upper bound of the distinct columns of each coarse row: min(pw x pairs,
// kRapND), pw = the filled slots per row of P (PW, or 1 for the identity)
__global__ void k_rap_bound(int nc, const int* __restrict__ rrp, const int* __restrict__ rci,
                            const int* __restrict__ rp, int* __restrict__ ub, int pw) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  const int p0 = rrp[I], p1 = rrp[I + 1];
  if (p1 - p0 > kRapRCap) { ub[I] = 0; return; }
  long long E = 0;
  for (int p = p0; p < p1; ++p) {
    const int i = rci[p];
    E += rp[i + 1] - rp[i];
  }
  const long long b = E * pw;
  ub[I] = (int)(b < kRapND ? b : kRapND);
}

// One coarse row I of R A P by a workgroup of NT lanes (rows too long for
// one wavefront).  The (R, A) pairs are taken NT at a time, one per lane; the
// lanes' nonzero products r_Ii a_ik p_kJ are stored in generation order (R's
// row, A's row, P's slots) by a workgroup scan; wavefront w then queues, in
// that order, the products of its own range of output positions and adds
// them to their sums run by run (rap_run).  Every sum takes its products in
// generation order, as in k_rap_small: the two kernels agree bit for bit.
constexpr int kRapRing = 128;  // per-wavefront queue: < 64 left over + <= 64 new

template <int NT, int MODE>
__device__ __forceinline__ void rap_row(int I, const int* __restrict__ rrp, const int* __restrict__ rci,
                                        const double* __restrict__ rv, const int* __restrict__ rp,
                                        const int* __restrict__ ci, const double* __restrict__ a,
                                        const int* __restrict__ pc, const double* __restrict__ pv,
                                        const int* __restrict__ toff, int* __restrict__ tcnt,
                                        int* __restrict__ tcol, double* __restrict__ tval,
                                        const int* __restrict__ crp, const int* __restrict__ cci,
                                        double* __restrict__ cval, int* __restrict__ err) {
  constexpr int W = NT / 64;
  constexpr int CP = NT * PW;  // products of one chunk at most
  constexpr int UB = (kRapHash / 2 > CP) ? kRapHash / 2 : CP;
  static_assert(kRapRing >= 127 && (kRapRing & (kRapRing - 1)) == 0, "queue too small");
  __shared__ int rS[kRapRCap];
  __shared__ int rO[kRapRCap + 1];
  __shared__ double rV[kRapRCap];
  __shared__ double ubuf[UB];  // hash table, later the chunk's product values
  __shared__ int cpos[CP];     // output position of each product of the chunk
  __shared__ int lst[kRapND];
  __shared__ double acc[kRapND];
  __shared__ int qpos[W][kRapRing];
  __shared__ double qval[W][kRapRing];
  __shared__ int wsum[W];
  __shared__ int nd_sh;
  int* tab = reinterpret_cast<int*>(ubuf);
  double* cv = ubuf;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int p0 = rrp[I], P = rrp[I + 1] - p0;
  if (P > kRapRCap) {
    if (tid == 0) {
      atomicOr(err, 2);
      if (MODE == kRapFused) tcnt[I] = 0;
    }
    return;
  }
  for (int t = tid; t < P; t += NT) {
    const int i = rci[p0 + t];
    const int b = rp[i];
    rS[t] = b;
    rO[t + 1] = rp[i + 1] - b;
    rV[t] = rv[p0 + t];
  }
  __syncthreads();
  if (tid < 64) {  // offsets of the pairs of each R entry (one wavefront scan)
    int carry = 0;
    for (int base = 0; base < P; base += 64) {
      const int t = base + lane;
      int v = t < P ? rO[t + 1] : 0;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
      }
      if (t < P) rO[t + 1] = carry + v;
      carry += __shfl(v, 63);
    }
    if (lane == 0) {
      rO[0] = 0;
      nd_sh = 0;
    }
  }
  __syncthreads();
  const int E = rO[P];
  int nd;
  if (MODE == kRapFused) {
    int hs = 64;
    while (hs < 2 * PW * E && hs < kRapHash) hs <<= 1;
    for (int h = tid; h < hs; h += NT) tab[h] = -1;
    __syncthreads();
    bool full = false;
    for (int f = tid; f < E; f += NT) {
      const int p = rap_locate(rO, P, f);
      const int k = ci[rS[p] + (f - rO[p])];
      for (int q = 0; q < PW; ++q) {
        const int J = pc[(size_t)k * PW + q];
        if (J < 0) continue;
        unsigned h = mix32((uint32_t)J) & (hs - 1);
        int probes = 0;
        while (true) {
          const int old = atomicCAS(&tab[h], -1, J);
          if (old == -1 || old == J) break;
          h = (h + 1) & (hs - 1);
          if (++probes >= hs) { full = true; break; }
        }
      }
    }
    if (full) atomicOr(err, 1);
    __syncthreads();
    bool over = false;
    for (int h = tid; h < hs; h += NT) {
      const int J = tab[h];
      if (J >= 0) {
        const int pos = atomicAdd(&nd_sh, 1);
        if (pos < kRapND) lst[pos] = J; else over = true;
      }
    }
    if (over) atomicOr(err, 4);
    __syncthreads();
    nd = nd_sh < kRapND ? nd_sh : kRapND;
    int P2 = 1;
    while (P2 < nd) P2 <<= 1;
    if (P2 <= 64) {  // one wavefront sorts in registers
      if (tid < 64) {
        int key = lane < nd ? lst[lane] : INT_MAX;
        wave_sort64(key);
        if (lane < nd) lst[lane] = key;
      }
      __syncthreads();
      P2 = 1;  // nothing left for the workgroup network below
    }
    for (int h = nd + tid; h < P2; h += NT) lst[h] = INT_MAX;
    __syncthreads();
    for (int k2 = 2; k2 <= P2; k2 <<= 1) {
      for (int j = k2 >> 1; j > 0; j >>= 1) {
        for (int idx = tid; idx < P2; idx += NT) {
          const int ixj = idx ^ j;
          if (ixj > idx) {
            const int x = lst[idx], y = lst[ixj];
            const bool up = (idx & k2) == 0;
            if ((x > y) == up) { lst[idx] = y; lst[ixj] = x; }
          }
        }
        __syncthreads();
      }
    }
  } else {
    const int base = crp[I];
    nd = crp[I + 1] - base;
    if (nd > kRapND) {
      if (tid == 0) atomicOr(err, 4);
      return;
    }
    for (int h = tid; h < nd; h += NT) lst[h] = cci[base + h];
  }
  for (int h = tid; h < nd; h += NT) acc[h] = 0.0;
  __syncthreads();  // the hash table is dead: its space holds chunk products
  const int own0 = (int)((long long)nd * w / W), own1 = (int)((long long)nd * (w + 1) / W);
  int* myq = qpos[w];
  double* myv = qval[w];
  int head = 0, tail = 0;  // this wavefront's queue counters
  for (int f0 = 0; f0 < E; f0 += NT) {
    const int f = f0 + tid;
    int np[PW];
    double nv[PW];
    unsigned valid = 0;  // bit q: slot q has a product
    if (f < E && nd > 0) {
      const int p = rap_locate(rO, P, f);
      const int e = rS[p] + (f - rO[p]);
      const int k = ci[e];
      const double ra = rV[p] * a[e];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        np[q] = 0;
        nv[q] = 0.0;
        const int J = pc[(size_t)k * PW + q];
        if (J < 0) continue;
        int lo = 0, hi = nd - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (lst[mid] < J) lo = mid + 1; else hi = mid;
        }
        if (lst[lo] == J) {
          np[q] = lo;
          nv[q] = ra * pv[(size_t)k * PW + q];
          valid |= 1u << q;
        }
      }
    }
    const int n_new = __popc(valid);
    int incl = n_new;  // chunk offsets in (pair, slot) order: workgroup scan
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int at = incl - n_new, total = 0;
#pragma unroll
    for (int u = 0; u < W; ++u) {
      if (u < w) at += wsum[u];
      total += wsum[u];
    }
#pragma unroll
    for (int q = 0; q < PW; ++q)
      if (valid >> q & 1u) {
        const int o = at + __popc(valid & ((1u << q) - 1u));
        cpos[o] = np[q];
        cv[o] = nv[q];
      }
    __syncthreads();
    for (int base = 0; base < total; base += 64) {  // this wavefront's products, in order
      const int t = base + lane;
      const int pp = t < total ? cpos[t] : -1;
      const bool mine = pp >= own0 && pp < own1;
      const unsigned long long m = __ballot(mine);
      if (mine) {
        const int idx = (tail + __popcll(m & ((1ull << lane) - 1ull))) & (kRapRing - 1);
        myq[idx] = pp;
        myv[idx] = cv[t];
      }
      tail += __popcll(m);
      wave_lds_sync();
      if (tail - head >= 64) {
        rap_run(64, head, myq, myv, kRapRing - 1, acc);
        head += 64;
      }
    }
    __syncthreads();  // the next chunk overwrites the products and wsum
  }
  if (tail > head) rap_run(tail - head, head, myq, myv, kRapRing - 1, acc);
  __syncthreads();
  if (MODE == kRapFused) {
    const int o = toff[I];
    const int cap = toff[I + 1] - o;
    if (nd > cap) {  // cannot happen: nd <= min(PW x pairs, kRapND)
      if (tid == 0) { atomicOr(err, 4); tcnt[I] = 0; }
      return;
    }
    for (int h = tid; h < nd; h += NT) {
      tcol[o + h] = lst[h];
      tval[o + h] = acc[h];
    }
    if (tid == 0) tcnt[I] = nd;
  } else {
    const int base = crp[I];
    for (int h = tid; h < nd; h += NT) cval[base + h] = acc[h];
  }
}

// one workgroup per coarse row
template <int NT, int MODE>
__global__ __launch_bounds__(NT) void k_rap(int nc, const int* __restrict__ rrp, const int* __restrict__ rci,
                                            const double* __restrict__ rv, const int* __restrict__ rp,
                                            const int* __restrict__ ci, const double* __restrict__ a,
                                            const int* __restrict__ pc, const double* __restrict__ pv,
                                            const int* __restrict__ toff, int* __restrict__ tcnt,
                                            int* __restrict__ tcol, double* __restrict__ tval,
                                            const int* __restrict__ crp, const int* __restrict__ cci,
                                            double* __restrict__ cval, int* __restrict__ err,
                                            const uint8_t* __restrict__ only) {
  const int I = blockIdx.x;
  if (I >= nc) return;
  if (only && !only[I]) return;  // incremental refresh: row unchanged
  rap_row<NT, MODE>(I, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, err);
}

// the rows listed in big[1 .. big[0]] (too large for the wavefront kernel)
template <int NT, int MODE>
__global__ __launch_bounds__(NT) void k_rap_list(const int* __restrict__ big, const int* __restrict__ rrp,
                                                 const int* __restrict__ rci, const double* __restrict__ rv,
                                                 const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ a, const int* __restrict__ pc,
                                                 const double* __restrict__ pv, const int* __restrict__ toff,
                                                 int* __restrict__ tcnt, int* __restrict__ tcol,
                                                 double* __restrict__ tval, const int* __restrict__ crp,
                                                 const int* __restrict__ cci, double* __restrict__ cval,
                                                 int* __restrict__ err) {
  const int cnt = big[0];
  for (int k = blockIdx.x; k < cnt; k += gridDim.x) {
    rap_row<NT, MODE>(big[1 + k], rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, err);
    __syncthreads();  // the next row reuses the LDS
  }
}


// ---------------------------------------------------------------------------
// Galerkin product of small levels through dense per-game blocks.  The coarse
// levels of a hierarchy have few rows, each collecting many fine rows, so the
// row-wise product has little parallelism and long rows to merge; here every
// entry of AP = A P (per game: fine rows x coarse columns) and then of
// R (AP) is computed by its own thread, each a sum in a fixed order (A row in
// CSR order and the P slots in order; R row in order), so the result does not
// depend on the launch shape.  An entry of R A P belongs to the pattern when
// some product reaches it (the same structural pattern as the row-wise
// product).
// ---------------------------------------------------------------------------
// the game g < G with off[g] <= t < off[g + 1] (the last one with off[g] <= t)
__device__ __forceinline__ int drap_game(const long long* __restrict__ off, int G, long long t) {
  int lo = 0, hi = G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// one wavefront per fine row i: the products a_ij p_jJ (A row in CSR order,
// P slots in order) go through LDS in chunks of 64; a chunk is sorted by
// (J, position), each run of equal J summed by a segmented scan and added to
// the row's dense accumulator, chunk after chunk
template <bool TOUCH, int MAXC>
__global__ __launch_bounds__(kBlock) void k_drap_ap(int nf, const long long* __restrict__ tab, int G,
                                                    const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const double* __restrict__ a, const int* __restrict__ pc,
                                                    const double* __restrict__ pv, double* __restrict__ ap,
                                                    uint8_t* __restrict__ apt, const uint8_t* __restrict__ only) {
  constexpr int W = kBlock / 64;
  __shared__ double acc_s[W][MAXC];
  __shared__ uint8_t hit_s[W][MAXC];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * W + wid;
  if (i >= nf) return;
  if (only && !only[i]) return;  // refresh: row i of A, hence of A P, unchanged
  const long long* fo = tab;
  const long long* co = tab + (G + 1);
  const long long* ao = tab + 2 * (G + 1);
  const int g = drap_game(fo, G, i);
  const int ncg = (int)(co[g + 1] - co[g]);
  if (ncg == 0) return;  // the game ends on this level
  const int c0 = (int)co[g];
  double* acc = acc_s[wid];
  uint8_t* hit = hit_s[wid];
  for (int J = lane; J < ncg; J += 64) {
    acc[J] = 0.0;
    hit[J] = 0;
  }
  wave_lds_sync();
  const int e0 = rp[i], slots = (rp[i + 1] - e0) * PW;
  for (int s0 = 0; s0 < slots; s0 += 64) {
    const int sl = s0 + lane;
    int key = INT_MAX;
    double val = 0.0;
    if (sl < slots) {
      const int e = e0 + sl / PW, q = sl % PW;
      const int j = ci[e];
      const int J = pc[(size_t)j * PW + q];
      if (J >= 0) {
        key = ((J - c0) << 6) | lane;
        val = a[e] * pv[(size_t)j * PW + q];
      }
    }
    wave_sort64(key, val);
    const int Jk = key == INT_MAX ? -1 : key >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {  // segmented inclusive scan over runs of equal J
      const double y = __shfl_up(val, o);
      const int Jy = __shfl_up(Jk, o);
      if (lane >= o && Jy == Jk) val += y;
    }
    const int Jn = __shfl_down(Jk, 1);
    if (Jk >= 0 && (lane == 63 || Jn != Jk)) {  // last of its run: the run's sum
      acc[Jk] += val;
      hit[Jk] = 1;
    }
    wave_lds_sync();
  }
  const long long base = ao[g] + (long long)(i - fo[g]) * ncg;
  for (int J = lane; J < ncg; J += 64) {
    ap[base + J] = acc[J];
    if (TOUCH) apt[base + J] = hit[J];
  }
}

// coarse entry (I, J) of game g: sum over the R row of I, in order
__device__ __forceinline__ double drap_entry(int p0, int p1, const int* __restrict__ rci,
                                             const double* __restrict__ rv, const double* __restrict__ ap,
                                             long long base, long long ncg) {
  double acc = 0.0;
  for (int p = p0; p < p1; ++p) acc += rv[p] * ap[base + (long long)rci[p] * ncg];
  return acc;
}

__global__ __launch_bounds__(kBlock) void k_drap_ac(long long total, const long long* __restrict__ tab, int G,
                                                    const int* __restrict__ rrp, const int* __restrict__ rci,
                                                    const double* __restrict__ rv, const double* __restrict__ ap,
                                                    const uint8_t* __restrict__ apt, double* __restrict__ ac,
                                                    uint8_t* __restrict__ acf) {
  const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= total) return;
  const long long* fo = tab;
  const long long* co = tab + (G + 1);
  const long long* ao = tab + 2 * (G + 1);
  const long long* qo = tab + 3 * (G + 1);
  const int g = drap_game(qo, G, t);
  const long long ncg = co[g + 1] - co[g];
  const long long loc = t - qo[g];
  const int I = (int)(co[g] + loc / ncg);
  const long long base = ao[g] - fo[g] * ncg + loc % ncg;  // AP entry (i, J) at base + i * ncg
  const int p0 = rrp[I], p1 = rrp[I + 1];
  int hit = 0;
  for (int p = p0; p < p1; ++p) hit |= apt[base + (long long)rci[p] * ncg];
  ac[t] = drap_entry(p0, p1, rci, rv, ap, base, ncg);
  acf[t] = (uint8_t)(hit != 0);
}

// one wavefront per coarse row: entries of the pattern
__global__ __launch_bounds__(kBlock) void k_drap_count(int nc, const long long* __restrict__ tab, int G,
                                                       const uint8_t* __restrict__ acf, int* __restrict__ cnt) {
  const int I = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (I >= nc) return;
  const long long* co = tab + (G + 1);
  const long long* qo = tab + 3 * (G + 1);
  const int g = drap_game(co, G, I);
  const long long ncg = co[g + 1] - co[g];
  const long long base = qo[g] + (I - co[g]) * ncg;
  int c = 0;
  for (long long J = lane; J < ncg; J += 64) c += acf[base + J] ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (lane == 0) cnt[I] = c;
}

// one wavefront per coarse row: the pattern's entries in column order
__global__ __launch_bounds__(kBlock) void k_drap_compact(int nc, const long long* __restrict__ tab, int G,
                                                         const double* __restrict__ ac,
                                                         const uint8_t* __restrict__ acf,
                                                         const int* __restrict__ crp, int* __restrict__ cci,
                                                         double* __restrict__ cval) {
  const int I = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (I >= nc) return;
  const long long* co = tab + (G + 1);
  const long long* qo = tab + 3 * (G + 1);
  const int g = drap_game(co, G, I);
  const long long ncg = co[g + 1] - co[g];
  const long long base = qo[g] + (I - co[g]) * ncg;
  int o = crp[I];
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (long long J0 = 0; J0 < ncg; J0 += 64) {
    const long long J = J0 + lane;
    const bool f = J < ncg && acf[base + J];
    const unsigned long long m = __ballot(f);
    if (f) {
      const int pos = o + __popcll(m & below);
      cci[pos] = (int)(co[g] + J);
      cval[pos] = ac[base + J];
    }
    o += __popcll(m);
  }
}

// refresh: values of the known pattern, one wavefront per coarse row, the
// same sums as k_drap_ac
__global__ __launch_bounds__(kBlock) void k_drap_known(int nc, const long long* __restrict__ tab, int G,
                                                       const int* __restrict__ rrp, const int* __restrict__ rci,
                                                       const double* __restrict__ rv, const double* __restrict__ ap,
                                                       const int* __restrict__ crp, const int* __restrict__ cci,
                                                       double* __restrict__ cval, const uint8_t* __restrict__ only) {
  const int I = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (I >= nc) return;
  if (only && !only[I]) return;
  const long long* fo = tab;
  const long long* co = tab + (G + 1);
  const long long* ao = tab + 2 * (G + 1);
  const int g = drap_game(co, G, I);
  const long long ncg = co[g + 1] - co[g];
  const long long base0 = ao[g] - fo[g] * ncg - co[g];
  const int p0 = rrp[I], p1 = rrp[I + 1];
  for (int e = crp[I] + lane; e < crp[I + 1]; e += 64) cval[e] = drap_entry(p0, p1, rci, rv, ap, base0 + cci[e], ncg);
}


// Coarse rows with at most kSmR entries of R and kSmN distinct columns, one
// wavefront per row and four rows per workgroup (the large levels, whose rows
// are short); a row that does not fit is appended to big[1 ..] for
// k_rap_list.  The nonzero products r_Ii a_ik p_kJ are generated in the order
// of R's row, A's row and P's slots (32 (R, A) pairs at a time, two lanes per
// pair) and queued in LDS; each run of 64 queued products is sorted by
// (output column, queue order) on keys alone, and the first product of each
// column adds the column's products of the run to the column's sum, one after
// the other.  Every column is thus the sequential sum of its products in
// generation order, as in rap_row: the two kernels agree bit for bit.
constexpr int kSmR = 64, kSmN = 128, kSmHash = 512;
constexpr int kSmRing = 256;  // queued products: < 64 left over + <= 128 new

// One coarse row I by one wavefront (the body of k_rap_small); the LDS
// areas are the wavefront's own.  A row it cannot take goes to `big`.
template <int MODE>
__device__ __forceinline__ void rap_small_row(int I, int lane, const int* __restrict__ rrp, const int* __restrict__ rci,
                                              const double* __restrict__ rv, const int* __restrict__ rp,
                                              const int* __restrict__ ci, const double* __restrict__ a,
                                              const int* __restrict__ pc, const double* __restrict__ pv,
                                              const int* __restrict__ toff, int* __restrict__ tcnt,
                                              int* __restrict__ tcol, double* __restrict__ tval,
                                              const int* __restrict__ crp, const int* __restrict__ cci,
                                              double* __restrict__ cval, int* __restrict__ big, int* rS, int* rO,
                                              double* rV, int* lst, int* qpos, double* qval, double* acc) {
  int* tab = reinterpret_cast<int*>(qval);
  auto to_big = [&]() {
    if (lane == 0) big[1 + atomicAdd(big, 1)] = I;
  };
  const int p0 = rrp[I], P = rrp[I + 1] - p0;
  if (P > kSmR) { to_big(); return; }
  int E = 0;  // R entries 64 at a time, offsets by a wavefront scan
  for (int base = 0; base < P; base += 64) {
    const int t = base + lane;
    int b = 0, ln = 0;
    double rvv = 0.0;
    if (t < P) {
      const int i = rci[p0 + t];
      b = rp[i];
      ln = rp[i + 1] - b;
      rvv = rv[p0 + t];
    }
    int v = ln;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(v, o);
      if (lane >= o) v += y;
    }
    if (t < P) {
      rS[t] = b;
      rO[t + 1] = E + v;
      rV[t] = rvv;
    }
    E += __shfl(v, 63);
  }
  if (lane == 0) rO[0] = 0;
  wave_lds_sync();
  int nd;
  if (MODE == kRapFused) {
    for (int h = lane; h < kSmHash; h += 64) tab[h] = -1;
    wave_lds_sync();
    // a key left out of a full table only happens beyond kSmN keys, where
    // the row goes to the workgroup kernel anyway
    for (int f = lane; f < E; f += 64) {
      const int p = rap_locate(rO, P, f);
      const int k = ci[rS[p] + (f - rO[p])];
      for (int q = 0; q < PW; ++q) {
        const int J = pc[(size_t)k * PW + q];
        if (J < 0) continue;
        unsigned h = mix32((uint32_t)J) & (kSmHash - 1);
        for (int pr = 0; pr < kSmHash; ++pr) {
          const int old = atomicCAS(&tab[h], -1, J);
          if (old == -1 || old == J) break;
          h = (h + 1) & (kSmHash - 1);
        }
      }
    }
    wave_lds_sync();
    nd = 0;
    for (int base = 0; base < kSmHash; base += 64) {
      const int key = tab[base + lane];
      const unsigned long long m = __ballot(key >= 0);
      const int pos = nd + __popcll(m & ((1ull << lane) - 1ull));
      if (key >= 0 && pos < kSmN) lst[pos] = key;
      nd += __popcll(m);
    }
    if (nd > kSmN) { to_big(); return; }
    wave_lds_sync();
    int key0 = lane < nd ? lst[lane] : INT_MAX;
    int key1 = lane + 64 < nd ? lst[lane + 64] : INT_MAX;
    wave_sort128(key0, key1);
    if (lane < nd) lst[lane] = key0;
    if (lane + 64 < nd) lst[lane + 64] = key1;
  } else {
    const int base = crp[I];
    nd = crp[I + 1] - base;
    if (nd > kSmN) { to_big(); return; }
    for (int h = lane; h < nd; h += 64) lst[h] = cci[base + h];
  }
  for (int h = lane; h < nd; h += 64) acc[h] = 0.0;
  wave_lds_sync();  // the hash table is dead: its space queues products
  int head = 0, tail = 0;  // queue counters (indices modulo kSmRing)
  for (int g0 = 0; g0 < E; g0 += 32) {
    const int f = g0 + (lane >> 1);
    int np[2] = {0, 0};
    double nv[2] = {0.0, 0.0};
    unsigned valid = 0;  // bit u: slot 2 (lane & 1) + u has a product
    if (f < E && nd > 0) {
      const int p = rap_locate(rO, P, f);
      const int e = rS[p] + (f - rO[p]);
      const int k = ci[e];
      const double ra = rV[p] * a[e];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int q = 2 * (lane & 1) + u;
        const int J = pc[(size_t)k * PW + q];
        if (J < 0) continue;
        int lo = 0, hi = nd - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (lst[mid] < J) lo = mid + 1; else hi = mid;
        }
        if (lst[lo] == J) {
          np[u] = lo;
          nv[u] = ra * pv[(size_t)k * PW + q];
          valid |= 1u << u;
        }
      }
    }
    const int n_new = __popc(valid);
    int incl = n_new;  // queue offsets in (pair, slot) order
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const int at = tail + incl - n_new;
    if (valid & 1u) {
      qpos[at & (kSmRing - 1)] = np[0];
      qval[at & (kSmRing - 1)] = nv[0];
    }
    if (valid & 2u) {
      const int o = (at + (valid & 1u)) & (kSmRing - 1);
      qpos[o] = np[1];
      qval[o] = nv[1];
    }
    tail += __shfl(incl, 63);
    wave_lds_sync();
    for (; tail - head >= 64; head += 64) rap_run(64, head, qpos, qval, kSmRing - 1, acc);
  }
  if (tail > head) rap_run(tail - head, head, qpos, qval, kSmRing - 1, acc);
  if (MODE == kRapFused) {
    const int o = toff[I];
    for (int h = lane; h < nd; h += 64) {
      tcol[o + h] = lst[h];
      tval[o + h] = acc[h];
    }
    if (lane == 0) tcnt[I] = nd;
  } else {
    const int base = crp[I];
    for (int h = lane; h < nd; h += 64) cval[base + h] = acc[h];
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_rap_small(int nc, const int* __restrict__ rrp, const int* __restrict__ rci,
                                                   const double* __restrict__ rv, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const double* __restrict__ a,
                                                   const int* __restrict__ pc, const double* __restrict__ pv,
                                                   const int* __restrict__ toff, int* __restrict__ tcnt,
                                                   int* __restrict__ tcol, double* __restrict__ tval,
                                                   const int* __restrict__ crp, const int* __restrict__ cci,
                                                   double* __restrict__ cval, const uint8_t* __restrict__ only,
                                                   int* __restrict__ big, const int* __restrict__ list,
                                                   const int* __restrict__ count) {
  static_assert(kSmHash * sizeof(int) <= kSmRing * sizeof(double), "hash must fit in the product queue");
  static_assert((kSmRing & (kSmRing - 1)) == 0 && kSmRing >= 63 + 32 * PW, "queue too small");
  __shared__ int s_rS[4][kSmR];
  __shared__ int s_rO[4][kSmR + 1];
  __shared__ double s_rV[4][kSmR];
  __shared__ double s_buf[4][kSmRing];  // hash table, later the queued product values
  __shared__ int s_lst[4][kSmN];
  __shared__ int s_qpos[4][kSmRing];    // output position of each queued product
  __shared__ double s_acc[4][kSmN];     // the row's sums by output position
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // nothing below synchronises the workgroup: each wavefront runs its rows
  if (list) {
    // the rows listed (a refresh's changed rows), a fixed grid looping over them
    const int cnt = *count;
    for (int q = blockIdx.x * 4 + w; q < cnt; q += gridDim.x * 4) {
      rap_small_row<MODE>(list[q], lane, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval,
                          big, s_rS[w], s_rO[w], s_rV[w], s_lst[w], s_qpos[w], s_buf[w], s_acc[w]);
      wave_lds_sync();
    }
    return;
  }
  const int I = (int)xcd_block() * 4 + w;
  if (I >= nc) return;
  if (only && !only[I]) return;
  rap_small_row<MODE>(I, lane, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, big,
                      s_rS[w], s_rO[w], s_rV[w], s_lst[w], s_qpos[w], s_buf[w], s_acc[w]);
}

// Short coarse rows by one thread each (levels of grid stencils): the row's
// sorted columns and sums live in the thread's column of two LDS arrays
// (entry h at h * 64 + lane, so the lanes of a wavefront never share a bank).
// The products r_Ii a_ik p_kJ are generated in the same order as in the
// wavefront and workgroup kernels (R's row, A's row, P's slots) and each is
// added to its column's sum when generated: every sum takes its products in
// generation order, starting from zero, so the three kernels agree bit for
// bit.  A row the thread cannot take (more than NC columns, or an R row
// beyond the workgroup kernel's cap) is handed to the wavefront kernel.
template <int MODE, int NC>
__device__ __forceinline__ bool rap_thread_row(int I, const int* __restrict__ rrp, const int* __restrict__ rci,
                                               const double* __restrict__ rv, const int* __restrict__ rp,
                                               const int* __restrict__ ci, const double* __restrict__ a,
                                               const int* __restrict__ pc, const double* __restrict__ pv,
                                               const int* __restrict__ toff, int* __restrict__ tcnt,
                                               int* __restrict__ tcol, double* __restrict__ tval,
                                               const int* __restrict__ crp, const int* __restrict__ cci,
                                               double* __restrict__ cval, int* col, double* acc) {
#pragma clang fp contract(off)
  const int p0 = rrp[I], p1 = rrp[I + 1];
  if (p1 - p0 > kRapRCap) return false;
  int nd = 0;
  if (MODE == kRapKnown) {
    const int base = crp[I];
    nd = crp[I + 1] - base;
    if (nd > NC) return false;
    for (int h = 0; h < nd; ++h) {
      col[h * 64] = cci[base + h];
      acc[h * 64] = 0.0;
    }
  }
  for (int p = p0; p < p1; ++p) {
    const int i = rci[p];
    const double r = rv[p];
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) {
      const int k = ci[e];
      const double ra = r * a[e];
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int J = pc[(size_t)k * PW + q];
        if (J < 0) continue;
        const double x = ra * pv[(size_t)k * PW + q];
        int lo = 0, hi = nd;  // first position with col >= J
        while (lo < hi) {
          const int m = (lo + hi) >> 1;
          if (col[m * 64] < J) lo = m + 1; else hi = m;
        }
        if (lo < nd && col[lo * 64] == J) {
          acc[lo * 64] = acc[lo * 64] + x;
          continue;
        }
        if (MODE == kRapKnown) continue;  // outside the known pattern: skipped, as in the other kernels
        if (nd == NC) return false;
        for (int h = nd; h > lo; --h) {
          col[h * 64] = col[(h - 1) * 64];
          acc[h * 64] = acc[(h - 1) * 64];
        }
        col[lo * 64] = J;
        acc[lo * 64] = 0.0 + x;
        ++nd;
      }
    }
  }
  if (MODE == kRapFused) {
    const int o = toff[I];
    for (int h = 0; h < nd; ++h) {
      tcol[o + h] = col[h * 64];
      tval[o + h] = acc[h * 64];
    }
    tcnt[I] = nd;
  } else {
    const int base = crp[I];
    for (int h = 0; h < nd; ++h) cval[base + h] = acc[h * 64];
  }
  return true;
}

// rows with f set appended to lst[1 ..] (count in lst[0]; order free), one
// atomic per wavefront
__device__ __forceinline__ void append_rows(bool f, int I, int* __restrict__ lst) {
  const unsigned long long m = __ballot(f);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(lst, __popcll(m));
  base = __shfl(base, leader);
  if (f) lst[1 + base + __popcll(m & ((1ull << lane) - 1ull))] = I;
}

template <int MODE, int NC>
__global__ __launch_bounds__(64) void k_rap_thr(int nc, const int* __restrict__ rrp, const int* __restrict__ rci,
                                                const double* __restrict__ rv, const int* __restrict__ rp,
                                                const int* __restrict__ ci, const double* __restrict__ a,
                                                const int* __restrict__ pc, const double* __restrict__ pv,
                                                const int* __restrict__ toff, int* __restrict__ tcnt,
                                                int* __restrict__ tcol, double* __restrict__ tval,
                                                const int* __restrict__ crp, const int* __restrict__ cci,
                                                double* __restrict__ cval, const uint8_t* __restrict__ only,
                                                int* __restrict__ mid, const int* __restrict__ list,
                                                const int* __restrict__ count) {
  __shared__ int s_col[NC * 64];
  __shared__ double s_acc[NC * 64];
  const int lane = threadIdx.x;
  int* col = s_col + lane;
  double* acc = s_acc + lane;
  // nothing below synchronises the workgroup: each thread runs its own rows
  if (list) {
    const int cnt = *count;
    for (int q = blockIdx.x * 64 + lane; q < cnt; q += gridDim.x * 64) {
      const int I = list[q];
      const bool ok = rap_thread_row<MODE, NC>(I, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp,
                                               cci, cval, col, acc);
      append_rows(!ok, I, mid);
    }
    return;
  }
  const int I = (int)xcd_block() * 64 + lane;
  if (I >= nc) return;
  bool ok = true;
  if (!only || only[I])
    ok = rap_thread_row<MODE, NC>(I, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, col,
                                  acc);
  append_rows(!ok, I, mid);
}

// Coarse rows by four lanes each (16 rows per wavefront): lane q of a row's
// group takes slot q of P's row in every (R entry, A entry) pair, so the four
// products of a pair, which go to distinct columns, are formed at once and
// each column still takes its products in generation order.  The group keeps
// the row's sorted columns and sums in LDS (NC of each).  A full product
// first finds the columns (inserted into a hash table in the sums' space,
// then ranked), then forms the sums; a refresh reads the known columns.  The
// pairs of an A row are taken four at a time, their loads issued together.
// Rows that do not fit are handed to the wavefront kernel, as in the
// thread-per-row kernel.
template <int NC>
__device__ __forceinline__ int quad_lower_bound(const int* col, int nd, int J) {
  int pos = 0;  // number of columns < J (nd <= NC)
#pragma unroll
  for (int step = NC; step > 0; step >>= 1)
    if (pos + step <= nd && col[pos + step - 1] < J) pos += step;
  return pos;
}

template <int MODE, int NC>
__device__ __forceinline__ bool rap_quad_row(int I, int q, const int* __restrict__ rrp, const int* __restrict__ rci,
                                             const double* __restrict__ rv, const int* __restrict__ rp,
                                             const int* __restrict__ ci, const double* __restrict__ a,
                                             const int* __restrict__ pc, const double* __restrict__ pv,
                                             const int* __restrict__ toff, int* __restrict__ tcnt,
                                             int* __restrict__ tcol, double* __restrict__ tval,
                                             const int* __restrict__ crp, const int* __restrict__ cci,
                                             double* __restrict__ cval, int* col, double* acc) {
#pragma clang fp contract(off)
  constexpr int kU = 8;        // pairs whose loads are issued together
  constexpr int kH = 2 * NC;   // hash slots (in the space of the sums)
  constexpr int kR = NC / 4;   // columns ranked per lane
  const int lane = threadIdx.x & 63;
  const int gbase = lane & ~3;  // first lane of the group
  const int p0 = rrp[I], p1 = rrp[I + 1];
  if (p1 - p0 > kRapRCap) return false;
  int nd = 0;
  if (MODE == kRapKnown) {
    const int base = crp[I];
    nd = crp[I + 1] - base;
    if (nd > NC) return false;
    for (int h = q; h < nd; h += 4) col[h] = cci[base + h];
  } else {
    int* tab = reinterpret_cast<int*>(acc);
    for (int h = q; h < kH; h += 4) tab[h] = -1;
    wave_lds_sync();
    bool full = false;  // a column found no free slot: more than kH columns
    for (int p = p0; p < p1; ++p) {
      const int i = rci[p];
      const int e1 = rp[i + 1];
      for (int e = rp[i]; e < e1; e += kU) {
        int k[kU], J[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) k[u] = e + u < e1 ? ci[e + u] : -1;
#pragma unroll
        for (int u = 0; u < kU; ++u) J[u] = k[u] >= 0 ? pc[(size_t)k[u] * PW + q] : -1;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (J[u] < 0) continue;
          unsigned h = mix32((uint32_t)J[u]) & (kH - 1);
          bool done = false;
          for (int t = 0; t < kH && !done; ++t) {
            const int old = atomicCAS(&tab[h], -1, J[u]);
            done = old == -1 || old == J[u];
            h = (h + 1) & (kH - 1);
          }
          full |= !done;
        }
      }
    }
    wave_lds_sync();
    // the occupied slots into col (in slot order), then each column to its rank
    for (int h0 = 0; h0 < kH; h0 += 4) {
      const int key = tab[h0 + q];
      const unsigned m = (unsigned)(__ballot(key >= 0) >> gbase) & 0xFu;
      const int at = nd + __popc(m & ((1u << q) - 1u));
      if (key >= 0 && at < NC) col[at] = key;
      nd += __popc(m);
    }
    const bool over = (((unsigned)(__ballot(full) >> gbase) & 0xFu) != 0u) || nd > NC;
    if (over) return false;
    wave_lds_sync();
    int key[kR], rank[kR];
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const int j = q + 4 * u;
      key[u] = j < nd ? col[j] : INT_MAX;
      rank[u] = 0;
    }
    for (int t = 0; t < nd; ++t) {
      const int c = col[t];
#pragma unroll
      for (int u = 0; u < kR; ++u) rank[u] += c < key[u] ? 1 : 0;
    }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < kR; ++u)
      if (q + 4 * u < nd) col[rank[u]] = key[u];
  }
  for (int h = q; h < nd; h += 4) acc[h] = 0.0;
  wave_lds_sync();
  // the sums: the pairs in order, the four slots of a pair at once
  for (int p = p0; p < p1; ++p) {
    const int i = rci[p];
    const double r = rv[p];
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; e += kU) {
      int k[kU], J[kU];
      double av[kU], pw[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        k[u] = -1;
        av[u] = 0.0;
        if (e + u < e1) {
          k[u] = ci[e + u];
          av[u] = a[e + u];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        J[u] = -1;
        pw[u] = 0.0;
        if (k[u] >= 0) {
          J[u] = pc[(size_t)k[u] * PW + q];
          pw[u] = pv[(size_t)k[u] * PW + q];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (J[u] < 0) continue;
        const double ra = r * av[u];
        const double x = ra * pw[u];
        const int pos = quad_lower_bound<NC>(col, nd, J[u]);
        // outside a known pattern: skipped, as in the other kernels
        if (pos < nd && col[pos] == J[u]) acc[pos] = acc[pos] + x;
      }
    }
  }
  if (MODE == kRapFused) {
    const int o = toff[I];
    for (int h = q; h < nd; h += 4) {
      tcol[o + h] = col[h];
      tval[o + h] = acc[h];
    }
    if (q == 0) tcnt[I] = nd;
  } else {
    const int base = crp[I];
    for (int h = q; h < nd; h += 4) cval[base + h] = acc[h];
  }
  return true;
}

template <int MODE, int NC>
__global__ __launch_bounds__(256) void k_rap_quad(int nc, const int* __restrict__ rrp, const int* __restrict__ rci,
                                                  const double* __restrict__ rv, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const double* __restrict__ a,
                                                  const int* __restrict__ pc, const double* __restrict__ pv,
                                                  const int* __restrict__ toff, int* __restrict__ tcnt,
                                                  int* __restrict__ tcol, double* __restrict__ tval,
                                                  const int* __restrict__ crp, const int* __restrict__ cci,
                                                  double* __restrict__ cval, const uint8_t* __restrict__ only,
                                                  int* __restrict__ mid, const int* __restrict__ list,
                                                  const int* __restrict__ count) {
  __shared__ int s_col[64][NC];
  __shared__ double s_acc[64][NC];
  const int grp = threadIdx.x >> 2, q = threadIdx.x & 3;
  int* col = s_col[grp];
  double* acc = s_acc[grp];
  // nothing below synchronises the workgroup: each group of four lanes runs
  // its own rows (the groups of a wavefront may diverge)
  if (list) {
    const int cnt = *count;
    for (int t = blockIdx.x * 64 + grp; t < cnt; t += gridDim.x * 64) {
      const int I = list[t];
      const bool ok = rap_quad_row<MODE, NC>(I, q, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci,
                                             cval, col, acc);
      append_rows(!ok && q == 0, I, mid);
      wave_lds_sync();
    }
    return;
  }
  const int I = (int)xcd_block() * 64 + grp;
  if (I >= nc) return;
  bool ok = true;
  if (!only || only[I])
    ok = rap_quad_row<MODE, NC>(I, q, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, col,
                                acc);
  append_rows(!ok && q == 0, I, mid);
}

// ---------------------------------------------------------------------------
// extended+i interpolation of coarse levels, four lanes per row (16 rows per
// wavefront): the formula and every sum of the wavefront kernel above, in the
// same orders, so a row gives the same weights bit for bit whichever of the
// two computes it.  The set is collected in a per-row LDS hash, ranked by
// fine index and searched by bisection; den_k takes its terms in row k's
// entry order; a member's weight takes its direct entry, then the distributed
// entries in the order of the F neighbours; the lumped diagonal and the
// total are the wavefront's butterfly over 64 lane slots (slot s of the
// butterfly held by lane s mod 4 of the group: its steps 32 ... 4 inside a
// lane, 2 and 1 across the group).  Rows longer than 64 entries, with more
// than 16 strong F neighbours or 32 set members, go to the wavefront kernel.
// ---------------------------------------------------------------------------
constexpr int kIqMem = 32, kIqHash = 64, kIqK = 8, kIqLen = 64;
struct IqGroup {
  int hs[kIqHash];  // the set's hash, later the members' weights (kIqMem doubles)
  int mem[kIqMem];
  int kcol[kIqK], kbeg[kIqK], kend[kIqK], kneg[kIqK];
  double kaik[kIqK], kden[kIqK], kabi[kIqK];
};
static_assert(kIqHash * sizeof(int) >= kIqMem * sizeof(double), "weights must fit in the hash space");

__device__ __forceinline__ unsigned group_ballot(bool b, int gbase) {
  return (unsigned)(__ballot(b) >> gbase) & 0xFu;
}

__device__ __forceinline__ bool iq_insert(int* hs, int v) {
  unsigned h = mix32((uint32_t)v) & (kIqHash - 1);
  for (int pr = 0; pr < kIqHash; ++pr) {
    const int old = atomicCAS(&hs[h], -1, v);
    if (old == -1 || old == v) return true;
    h = (h + 1) & (kIqHash - 1);
  }
  return false;
}

// position of v among the m sorted members, or -1
__device__ __forceinline__ int iq_find(const int* mem, int m, int v) {
  int pos = 0;
#pragma unroll
  for (int step = kIqMem; step > 0; step >>= 1)
    if (pos + step <= m && mem[pos + step - 1] < v) pos += step;
  return (pos < m && mem[pos] == v) ? pos : -1;
}

// the wavefront butterfly sum (xor 32, 16, ..., 1) of 64 slot values; lane q
// of the group holds slots q + 4u in v[u].  Every pair of the butterfly adds
// the same two values, so all lanes end with one result.
__device__ __forceinline__ double iq_tree(double (&v)[16], int q, int gbase) {
#pragma unroll
  for (int b = 8; b >= 1; b >>= 1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (u & b) continue;
      const double t = v[u] + v[u | b];
      v[u] = t;
      v[u | b] = t;
    }
  }
  double x = v[0];
  x = x + __shfl(x, gbase | (q ^ 2));
  x = x + __shfl(x, gbase | (q ^ 1));
  return x;
}

__device__ __forceinline__ bool interp_quad_row(int i, int q, int gbase, IqGroup& G, const int* __restrict__ rp,
                                                const int* __restrict__ ci, const double* __restrict__ a,
                                                const double* __restrict__ dinv, const uint8_t* __restrict__ strong,
                                                const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                                const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                double* __restrict__ pv) {
#pragma clang fp contract(off)
  const unsigned below = (1u << q) - 1u;
  if (q < PW) {
    pc[(size_t)i * PW + q] = -1;
    pv[(size_t)i * PW + q] = 0.0;
  }
  if (cf[i] == CF_C) {
    if (q == 0) {
      pc[(size_t)i * PW] = cidx[i];
      pv[(size_t)i * PW] = 1.0;
    }
    return true;
  }
  if (dir[i]) return true;
  const int e0 = rp[i], len = rp[i + 1] - e0;
  if (len > kIqLen) return false;
  // ---- row i: strong C neighbours into the set, strong F neighbours listed in row order
  for (int h = q; h < kIqHash; h += 4) G.hs[h] = -1;
  wave_lds_sync();
  int nK = 0;
  bool full = false;
  for (int b16 = 0; b16 < len; b16 += 16) {  // four chunks of four entries, loads first
    int jj[4];
    bool offs[4];
    double aa[4];
    int8_t cc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = b16 + 4 * u + q;
      jj[u] = -1;
      offs[u] = false;
      aa[u] = 0.0;
      if (t < len) {
        jj[u] = ci[e0 + t];
        offs[u] = strong[e0 + t] != 0;
        aa[u] = a[e0 + t];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      offs[u] = offs[u] && jj[u] != i;
      cc[u] = offs[u] ? cf[jj[u]] : (int8_t)0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (b16 + 4 * u >= len) break;  // the same for the whole group
      if (offs[u] && cc[u] == CF_C && !iq_insert(G.hs, jj[u])) full = true;
      const bool isF = offs[u] && cc[u] == CF_F;
      const unsigned m4 = group_ballot(isF, gbase);
      const int pos = nK + __popc(m4 & below);
      if (isF && pos < kIqK) {
        G.kcol[pos] = jj[u];
        G.kaik[pos] = aa[u];
      }
      nK += __popc(m4);
    }
  }
  if (group_ballot(full, gbase) || nK > kIqK) return false;
  wave_lds_sync();
  for (int p = q; p < nK; p += 4) {
    const int k = G.kcol[p];
    G.kbeg[p] = rp[k];
    G.kend[p] = rp[k + 1];
    G.kneg[p] = dinv[k] < 0.0 ? 1 : 0;
  }
  wave_lds_sync();
  // ---- distance-two candidates: strong C neighbours of the strong F neighbours
  for (int p = 0; p < nK; ++p) {
    const int k = G.kcol[p], en = G.kend[p];
    for (int c0 = G.kbeg[p]; c0 < en; c0 += 16) {  // loads of four chunks first
      int ll[4];
      int8_t cl[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e2 = c0 + 4 * u + q;
        ll[u] = (e2 < en && strong[e2]) ? ci[e2] : -1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) cl[u] = (ll[u] >= 0 && ll[u] != k) ? cf[ll[u]] : (int8_t)0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (cl[u] == CF_C && !iq_insert(G.hs, ll[u])) full = true;
    }
  }
  if (group_ballot(full, gbase)) return false;
  wave_lds_sync();
  // ---- members: the occupied slots compacted, then each to its rank
  int m = 0;
  for (int h0 = 0; h0 < kIqHash; h0 += 4) {
    const int key = G.hs[h0 + q];
    const unsigned m4 = group_ballot(key >= 0, gbase);
    const int at = m + __popc(m4 & below);
    if (key >= 0 && at < kIqMem) G.mem[at] = key;
    m += __popc(m4);
  }
  if (m > kIqMem) return false;
  wave_lds_sync();
  {
    int key[kIqMem / 4], rank[kIqMem / 4];
#pragma unroll
    for (int u = 0; u < kIqMem / 4; ++u) {
      const int j = q + 4 * u;
      key[u] = j < m ? G.mem[j] : INT_MAX;
      rank[u] = 0;
    }
    for (int t = 0; t < m; ++t) {
      const int c = G.mem[t];
#pragma unroll
      for (int u = 0; u < kIqMem / 4; ++u) rank[u] += c < key[u] ? 1 : 0;
    }
    wave_lds_sync();
#pragma unroll
    for (int u = 0; u < kIqMem / 4; ++u)
      if (q + 4 * u < m) G.mem[rank[u]] = key[u];
  }
  double* W = reinterpret_cast<double*>(G.hs);  // the hash is dead
  wave_lds_sync();
  for (int h = q; h < m; h += 4) W[h] = 0.0;
  // ---- den_k and abar_ki: row k's terms in entry order (every lane forms the same sum)
  for (int p = 0; p < nK; ++p) {
    const int k = G.kcol[p], en = G.kend[p];
    const bool neg = G.kneg[p] != 0;
    double d = 0.0, abi = 0.0;
    bool has_i = false;
    for (int c16 = G.kbeg[p]; c16 < en; c16 += 16) {  // loads of four chunks first
      int ll[4];
      double ak[4], term[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e2 = c16 + 4 * u + q;
        ll[u] = -1;
        ak[u] = 0.0;
        if (e2 < en) {
          ll[u] = ci[e2];
          ak[u] = a[e2];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        term[u] = 0.0;
        const double abar = neg ? (ak[u] > 0.0 ? ak[u] : 0.0) : (ak[u] < 0.0 ? ak[u] : 0.0);
        if (ll[u] >= 0 && ll[u] != k && abar != 0.0) {
          if (ll[u] == i) {
            term[u] = abar;
            abi = abar;
            has_i = true;
          } else if (iq_find(G.mem, m, ll[u]) >= 0) {
            term[u] = abar;
          }
        }
      }
      // the terms in entry order: chunk by chunk, lane by lane
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) d = d + __shfl(term[u], gbase | w);
    }
    const unsigned hi = group_ballot(has_i, gbase);
    abi = hi ? __shfl(abi, gbase | (__ffs(hi) - 1)) : 0.0;
    if (q == 0) {
      G.kden[p] = d;
      G.kabi[p] = abi;
    }
  }
  wave_lds_sync();
  // ---- diagonal: a_ii, weak entries, parts of F neighbours sent back to i;
  //      direct entries towards set members (slot t of the butterfly = entry t)
  double v[16];
  int rankF = 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    v[u] = 0.0;
    const int t = 4 * u + q;
    if (4 * u >= len) continue;  // the same for the whole group
    const bool in = t < len;
    int j = -1;
    bool st = false;
    double aij = 0.0;
    if (in) {
      j = ci[e0 + t];
      st = strong[e0 + t] != 0;
      aij = a[e0 + t];
    }
    const bool off = in && j != i;
    const int8_t cj = off ? cf[j] : (int8_t)0;
    const bool isF = off && st && cj == CF_F;
    const unsigned m4 = group_ballot(isF, gbase);
    const int p = rankF + __popc(m4 & below);
    rankF += __popc(m4);
    double c = 0.0;
    if (in && j == i) {
      c = aij;
    } else if (off && aij != 0.0) {
      const int qq = iq_find(G.mem, m, j);
      if (qq >= 0) {
        W[qq] = W[qq] + aij;  // one entry per column: no conflicts
      } else if (isF) {
        const double den = G.kden[p];
        c = den == 0.0 ? aij : aij * G.kabi[p] / den;
      } else if (!dir[j]) {
        c = aij;
      }
    }
    v[u] = 0.0 + c;
  }
  wave_lds_sync();
  // ---- distributed entries: F neighbours in row order; each row k holds a
  //      column at most once, so the lanes of one k never collide
  for (int p = 0; p < nK; ++p) {
    const int k = G.kcol[p], en = G.kend[p];
    const bool neg = G.kneg[p] != 0;
    const double den = G.kden[p], aik = G.kaik[p];
    if (den != 0.0) {
      for (int c16 = G.kbeg[p]; c16 < en; c16 += 16) {  // loads of four chunks first
        int ll[4];
        double ak[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e2 = c16 + 4 * u + q;
          ll[u] = -1;
          ak[u] = 0.0;
          if (e2 < en) {
            ll[u] = ci[e2];
            ak[u] = a[e2];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double abar = neg ? (ak[u] > 0.0 ? ak[u] : 0.0) : (ak[u] < 0.0 ? ak[u] : 0.0);
          if (ll[u] < 0 || ll[u] == k || ll[u] == i || abar == 0.0) continue;
          const int qq = iq_find(G.mem, m, ll[u]);
          if (qq >= 0) W[qq] = W[qq] + aik * abar / den;
        }
      }
    }
    wave_lds_sync();
  }
  const double dd = iq_tree(v, q, gbase);
  if (dd == 0.0 || m == 0) return true;
  // ---- weights, their total, the PW largest (lowest member on ties)
  double vt[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int s = 4 * u + q;
    double w = 0.0;
    if (s < m) {
      w = -W[s] / dd;
      W[s] = w;
    }
    vt[u] = 0.0 + w;
  }
  const double total = iq_tree(vt, q, gbase);
  wave_lds_sync();
  int kq[PW];
  double kw[PW];
  int nk = 0;
#pragma unroll
  for (int r = 0; r < PW; ++r) {
    kq[r] = INT_MAX;
    kw[r] = 0.0;
  }
#pragma unroll
  for (int r = 0; r < PW; ++r) {
    if (nk == r) {
      double bw = 0.0;
      int bq = INT_MAX;
      for (int s = q; s < m; s += 4) {
        bool used = false;
#pragma unroll
        for (int u = 0; u < r; ++u) used |= kq[u] == s;
        const double aw = fabs(W[s]);
        if (!used && (aw > bw || (aw == bw && aw > 0.0 && s < bq))) {
          bw = aw;
          bq = s;
        }
      }
#pragma unroll
      for (int o = 2; o >= 1; o >>= 1) {
        const double ow = __shfl(bw, gbase | (q ^ o));
        const int oq = __shfl(bq, gbase | (q ^ o));
        if (ow > bw || (ow == bw && oq < bq)) {
          bw = ow;
          bq = oq;
        }
      }
      if (bq != INT_MAX && bw != 0.0) {
        kq[r] = bq;
        kw[r] = W[bq];
        nk = r + 1;
      }
    }
  }
  if (q == 0 && nk > 0) {
    double kept = 0.0;
#pragma unroll
    for (int u = 0; u < PW; ++u)
      if (u < nk) kept += kw[u];
    const double scl = kept != 0.0 ? total / kept : 1.0;
#pragma unroll
    for (int u = 0; u < PW; ++u) {
      if (u >= nk) continue;
      int r = 0;
#pragma unroll
      for (int w2 = 0; w2 < PW; ++w2) r += (w2 < nk && kq[w2] < kq[u]) ? 1 : 0;
      pc[(size_t)i * PW + r] = cidx[G.mem[kq[u]]];
      pv[(size_t)i * PW + r] = kw[u] * scl;
    }
  }
  return true;
}

// 16 rows of a tile per workgroup of one wavefront; rows that do not fit are
// appended to defer[1 ..] for the wavefront kernel
__global__ __launch_bounds__(64) void k_interp_quad(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ a,
                                                    const double* __restrict__ dinv,
                                                    const uint8_t* __restrict__ strong,
                                                    const int8_t* __restrict__ cf, const int* __restrict__ cidx,
                                                    const uint8_t* __restrict__ dir, int* __restrict__ pc,
                                                    double* __restrict__ pv, int* __restrict__ defer) {
  __shared__ IqGroup s_g[16];
  const int grp = threadIdx.x >> 2, q = threadIdx.x & 3, gbase = threadIdx.x & ~3;
  const unsigned bid = xcd_block();
  const Tile t = tiles[bid / (kTileRows / 16)];
  const int i = t.r0 + (int)(bid % (kTileRows / 16)) * 16 + grp;
  if (i >= t.r1) return;  // nothing below synchronises the workgroup
  const bool ok = interp_quad_row(i, q, gbase, s_g[grp], rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv);
  append_rows(!ok && q == 0, i, defer);
}

// rows of the scratch area into the final CSR (eight lanes per row)
__global__ __launch_bounds__(256) void k_rap_compact(int nc, const int* __restrict__ toff,
                                                     const int* __restrict__ tcol, const double* __restrict__ tval,
                                                     const int* __restrict__ crp, int* __restrict__ cci,
                                                     double* __restrict__ cval) {
  const int I = blockIdx.x * 32 + (int)(threadIdx.x >> 3);
  if (I >= nc) return;
  const int o = toff[I], base = crp[I], nd = crp[I + 1] - base;
  for (int h = threadIdx.x & 7; h < nd; h += 8) {
    cci[base + h] = tcol[o + h];
    cval[base + h] = tval[o + h];
  }
}

// ---------------------------------------------------------------------------
// incremental refresh: rows of level 0 whose values changed since the last
// setup (the copy is updated in place), and the coarse rows they reach
// through P (A_c row I depends on fine row i only when P[i, I] != 0).
// ---------------------------------------------------------------------------
__global__ void k_row_changed(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                              const double* __restrict__ a, double* __restrict__ prev,
                              uint8_t* __restrict__ chg) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  uint8_t c = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const double v = a[e];
    if (v != prev[e]) { c = 1; prev[e] = v; }
  }
  chg[i] = c;
}

__global__ void k_mark_coarse(const Tile* __restrict__ tiles, const int* __restrict__ pc,
                              const uint8_t* __restrict__ chg, uint8_t* __restrict__ cmark) {
  Tile t = tiles[blockIdx.x];
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1 || !chg[i]) return;
  for (int q = 0; q < PW; ++q) {
    const int c = pc[(size_t)i * PW + q];
    if (c >= 0) cmark[c] = 1;
  }
}

void amg_row_changed(const Tile* t, int nt, const int* rp, const double* a, double* prev, uint8_t* chg,
                     hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_row_changed, dim3(nt), dim3(kTileRows), 0, s, t, rp, a, prev, chg);
  SHP_LAUNCH_CHECK();
}

void amg_mark_coarse(const Tile* t, int nt, const int* pc, const uint8_t* chg, uint8_t* cmark, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_mark_coarse, dim3(nt), dim3(kTileRows), 0, s, t, pc, chg, cmark);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// level helpers
// ---------------------------------------------------------------------------
__global__ void k_cast(const double* __restrict__ in, float* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

// ---------------------------------------------------------------------------
// dense inverse of the coarsest blocks: Gauss-Jordan with partial pivoting on
// [A | I], one workgroup per block.  blk = (row0, size, dense offset, slot).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dense_inv(const int* __restrict__ blk, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const double* __restrict__ a,
                                                   double* __restrict__ work, double* __restrict__ inv64,
                                                   float* __restrict__ inv32, int* __restrict__ err) {
  __shared__ double fac[kDenseMax];
  __shared__ double redv[256];
  __shared__ int redi[256];
  const int row0 = blk[4 * blockIdx.x], nb = blk[4 * blockIdx.x + 1];
  const size_t doff = (size_t)blk[4 * blockIdx.x + 2];
  if (nb <= kDenseWave) return;  // handled by the single-wave kernel
  double* M = work + 2 * doff;  // nb x 2nb, row-major
  const int W = 2 * nb;
  const int tid = threadIdx.x;
  for (size_t idx = tid; idx < (size_t)nb * W; idx += blockDim.x) M[idx] = 0.0;
  __syncthreads();
  for (int i = tid; i < nb; i += blockDim.x) {
    int r = row0 + i;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      int c = ci[e] - row0;
      if (c >= 0 && c < nb) M[(size_t)i * W + c] += a[e];
    }
    M[(size_t)i * W + nb + i] = 1.0;
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    double bv = -1.0;
    int bi = k;
    for (int i = k + tid; i < nb; i += blockDim.x) {
      double v = fabs(M[(size_t)i * W + k]);
      if (v > bv) { bv = v; bi = i; }
    }
    redv[tid] = bv;
    redi[tid] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (tid < o) {
        double v2 = redv[tid + o];
        int i2 = redi[tid + o];
        if (v2 > redv[tid] || (v2 == redv[tid] && i2 < redi[tid])) { redv[tid] = v2; redi[tid] = i2; }
      }
      __syncthreads();
    }
    const int p = redi[0];
    const double pmag = redv[0];
    __syncthreads();
    if (!(pmag > 0.0)) {
      if (tid == 0) atomicOr(err, 4);
      return;
    }
    if (p != k)
      for (int j = tid; j < W; j += blockDim.x) {
        double t0 = M[(size_t)k * W + j];
        M[(size_t)k * W + j] = M[(size_t)p * W + j];
        M[(size_t)p * W + j] = t0;
      }
    __syncthreads();
    const double piv = M[(size_t)k * W + k];
    __syncthreads();
    for (int j = tid; j < W; j += blockDim.x) M[(size_t)k * W + j] /= piv;
    for (int i = tid; i < nb; i += blockDim.x) fac[i] = M[(size_t)i * W + k];
    __syncthreads();
    for (int j = tid; j < W; j += blockDim.x) {
      const double mkj = M[(size_t)k * W + j];
      if (mkj == 0.0) continue;
      for (int i = 0; i < nb; ++i)
        if (i != k) M[(size_t)i * W + j] -= fac[i] * mkj;
    }
    __syncthreads();
  }
  for (size_t idx = tid; idx < (size_t)nb * nb; idx += blockDim.x) {
    int j = (int)(idx / nb), i = (int)(idx % nb);  // column-major output
    double v = M[(size_t)i * W + nb + j];
    inv64[doff + idx] = v;
    if (inv32) inv32[doff + idx] = (float)v;
  }
}

// maximum over the lanes of a wavefront (ROCm device library)
extern "C" __device__ unsigned long long __ockl_wfred_max_u64(unsigned long long);

// In-place Gauss-Jordan inversion with partial pivoting for blocks of at
// most 64 unknowns, four wavefronts: lane i of wavefront w holds row i's
// entries in columns 16w .. 16w+15 in registers.  Step k: the wavefront that
// owns column k picks the pivot (the unused row with the largest |M[i][k]|,
// compared on the leading 56 bits, the lowest row first) and publishes the
// column; every wavefront then reads the pivot row's entries of its columns
// from the pivot lane and eliminates.  Rows are not swapped; with p_k the
// pivot row of step k the in-place result M holds inv[k][p_j] = M[p_k][j].
__device__ __forceinline__ double lane_read(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ __launch_bounds__(256) void k_dense_inv_cols(const int* __restrict__ blk, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const double* __restrict__ a,
                                                        double* __restrict__ inv64, float* __restrict__ inv32,
                                                        int* __restrict__ err, const uint8_t* __restrict__ only) {
  constexpr int CB = 16, LD = 65;
  __shared__ double S[64 * LD];
  __shared__ double colk[2][64];
  __shared__ int pk[2];
  __shared__ int perm[64];
  const int row0 = blk[4 * blockIdx.x], nb = blk[4 * blockIdx.x + 1];
  const size_t doff = (size_t)blk[4 * blockIdx.x + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (nb > 64) return;  // a larger block: another kernel
  if (only) {           // incremental refresh: skip blocks none of whose rows changed
    int any = 0;
    for (int r = threadIdx.x; r < nb; r += 256) any |= only[row0 + r];
    if (!__syncthreads_or(any)) return;
  }
  for (int idx = threadIdx.x; idx < 64 * LD; idx += 256) S[idx] = 0.0;
  __syncthreads();
  if (w == 0 && lane < nb) {  // row `lane` into column-major staging
    const int r = row0 + lane;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int c = ci[e] - row0;
      if (c >= 0 && c < nb) S[c * LD + lane] += a[e];
    }
  }
  __syncthreads();
  double v[CB];
#pragma unroll
  for (int jj = 0; jj < CB; ++jj) v[jj] = S[(CB * w + jj) * LD + lane];
  bool used = lane >= nb;
  int myk = 0;
  for (int kb = 0; kb * CB < nb; ++kb) {
#pragma unroll
    for (int kk = 0; kk < CB; ++kk) {
      const int k = kb * CB + kk;
      if (k < nb) {  // uniform over the workgroup
        const int buf = k & 1;
        if (w == kb) {
          unsigned long long key = 0;
          if (!used) {
            const double m = fabs(v[kk]);
            if (m == m)
              key = ((unsigned long long)__double_as_longlong(m) & ~0xFFull) | (unsigned long long)(255 - lane);
          }
          key = __ockl_wfred_max_u64(key);
          colk[buf][lane] = v[kk];
          if (lane == 0) pk[buf] = (key >> 8) == 0 ? -1 : 255 - (int)(key & 0xFF);
        }
        __syncthreads();
        const int p = pk[buf];
        if (p < 0) {  // no nonzero pivot left (uniform): singular block
          if (threadIdx.x == 0) atomicOr(err, 4);
          return;
        }
        const double inv = 1.0 / colk[buf][p];
        const double f = colk[buf][lane] * inv;  // M[i][k] / pivot
        const bool piv = lane == p;
#pragma unroll
        for (int jj = 0; jj < CB; ++jj) {
          const double pr = lane_read(v[jj], p);
          v[jj] = piv ? pr * inv : v[jj] - f * pr;
        }
        if (w == kb) v[kk] = piv ? inv : -f;
        if (piv) {
          used = true;
          myk = k;
          if (w == 0) perm[k] = p;
        }
      }
    }
  }
  __syncthreads();
  if (lane < nb) {
#pragma unroll
    for (int jj = 0; jj < CB; ++jj) {
      const int j = CB * w + jj;
      if (j < nb) {
        const size_t o = doff + (size_t)perm[j] * nb + myk;
        inv64[o] = v[jj];
        if (inv32) inv32[o] = (float)v[jj];
      }
    }
  }
}

// Dense inverse of blocks of at most 64 unknowns on the FP64 matrix cores: a
// blocked Gauss-Jordan sweep in LDS over panels of 16 columns, the block padded
// to a multiple of 16 with identity rows and columns.  For the panel at
// columns K = k0 .. k0+15:
//   1. wavefront 0 holds the panel's columns of every row (lane = row) and
//      sweeps its 16 pivots by Gauss-Jordan with partial pivoting: each column
//      takes, among the rows at positions k0 .. not yet chosen, the one with
//      the largest |entry| (magnitudes compared on their leading 56 bits, the
//      lowest row first) and eliminates it from every other row.  This leaves
//      T = A_KK^-1 in the pivot rows and -A_RK T in the others R;
//   2. the rows at positions k0 .. are regrouped, the pivots first in the
//      order chosen, the others after them in their order;
//   3. the columns C outside the panel, as 16x16x4 FP64 MFMA tiles, one
//      wavefront per row tile:  A_RC <- A_RC + (-A_RK T) A_KC,  A_KC <- T A_KC.
// After the last panel the matrix holds X = (Pi A)^-1 for the accumulated row
// regrouping Pi, and column j of A^-1 is column q(j) of X, q(j) the final
// position of row j (written column-major, like the other kernels).
// The accumulator layout of the MFMA is read at run time from two products
// whose entries are their own row and column indices, so the kernel assumes
// only the operand layout: lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
typedef double shp_dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_dense_inv_mfma(const int* __restrict__ blk, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const double* __restrict__ a,
                                                        double* __restrict__ inv64, float* __restrict__ inv32,
                                                        int* __restrict__ err, const uint8_t* __restrict__ only) {
  constexpr int NP = 64, LD = NP + 1, B = 16, NT = NP / B;
  __shared__ double M[NP * LD];
  __shared__ int npos[NP];  // this panel: new position of the row at position l
  __shared__ int orig[NP];  // original row now at position l
  __shared__ int q[NP];     // final position of original row j
  __shared__ int srp[NP + 1];
  __shared__ int bad;
  const int row0 = blk[4 * blockIdx.x], nb = blk[4 * blockIdx.x + 1];
  const size_t doff = (size_t)blk[4 * blockIdx.x + 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  if (nb > NP) return;  // a larger block: another kernel
  if (only) {           // incremental refresh: skip blocks none of whose rows changed
    int any = 0;
    for (int r = tid; r < nb; r += 256) any |= only[row0 + r];
    if (!__syncthreads_or(any)) return;
  }
  const int np = (nb + B - 1) / B * B, nt = np / B;
  for (int idx = tid; idx < np * np; idx += 256) {
    const int i = idx / np, j = idx - i * np;
    M[i * LD + j] = (i == j && i >= nb) ? 1.0 : 0.0;
  }
  if (tid < NP) orig[tid] = tid;
  if (tid <= nb) srp[tid] = rp[row0 + tid];
  if (tid == 0) bad = 0;
  __syncthreads();
  // the block's rows are contiguous in the CSR: a thread per entry, its row by
  // bisection of the row pointers (entries outside the block are dropped)
  for (int e = srp[0] + tid; e < srp[nb]; e += 256) {
    int lo = 0, hi = nb;  // srp[lo] <= e < srp[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (srp[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int c = ci[e] - row0;
    if (c >= 0 && c < nb) atomicAdd(&M[lo * LD + c], a[e]);
  }
  // accumulator layout: register r of this lane holds entry (crow[r], ccol[r])
  int crow[4], ccol[4];
  {
    const shp_dbl4 z = {0.0, 0.0, 0.0, 0.0};
    const double lead = lk == 0 ? 1.0 : 0.0, idx = lk == 0 ? (double)li : 0.0;
    const shp_dbl4 ri = __builtin_amdgcn_mfma_f64_16x16x4f64(idx, lead, z, 0, 0, 0);
    const shp_dbl4 cj = __builtin_amdgcn_mfma_f64_16x16x4f64(lead, idx, z, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      crow[r] = (int)ri[r];
      ccol[r] = (int)cj[r];
    }
  }
  __syncthreads();
  for (int kb = 0; kb < nt; ++kb) {
    const int k0 = kb * B;
    // 1. Gauss-Jordan sweep of the panel's pivots on its columns (wavefront 0)
    double pv[B];
    if (w == 0) {
      const bool live = lane < np;
#pragma unroll
      for (int c = 0; c < B; ++c) pv[c] = live ? M[lane * LD + k0 + c] : 0.0;
      bool used = !live || lane < k0;
      int myk = -1;
      bool sing = false;
#pragma unroll
      for (int jj = 0; jj < B; ++jj) {
        if (!sing) {
          unsigned long long key = 0;
          if (!used) {
            const double m = fabs(pv[jj]);
            if (m == m)
              key = ((unsigned long long)__double_as_longlong(m) & ~0xFFull) | (unsigned long long)(255 - lane);
          }
          key = __ockl_wfred_max_u64(key);
          if ((key >> 8) == 0) {  // no nonzero pivot left (uniform): singular block
            sing = true;
          } else {
            const int p = 255 - (int)(key & 0xFF);
            const double inv = 1.0 / lane_read(pv[jj], p);
            const double f = pv[jj];
            const bool isp = lane == p;
#pragma unroll
            for (int c = 0; c < B; ++c) {
              const double pr = lane_read(pv[c], p);
              if (c == jj) pv[c] = isp ? inv : -f * inv;
              else pv[c] = isp ? pr * inv : pv[c] - f * (pr * inv);
            }
            if (isp) {
              used = true;
              myk = jj;
            }
          }
        }
      }
      // 2. new positions: pivots in the order chosen, then the other rows
      const unsigned long long rest = __ballot(live && lane >= k0 && myk < 0);
      int to = lane;
      if (lane >= k0) to = myk >= 0 ? k0 + myk : k0 + B + __popcll(rest & ((1ull << lane) - 1ull));
      if (live) npos[lane] = to;
      if (sing && lane == 0) bad = 1;
    }
    __syncthreads();
    if (bad) {  // uniform
      if (tid == 0) atomicOr(err, 4);
      return;
    }
    {  // regroup rows k0 .. np-1 (columns outside the panel); wavefront 0 writes the panel
      const int cnt = (np - k0) * np;
      double tmp[NP * NP / 256];
#pragma unroll
      for (int t = 0; t < NP * NP / 256; ++t) {
        const int idx = tid + 256 * t;
        if (idx < cnt) tmp[t] = M[(k0 + idx / np) * LD + idx % np];
      }
      const int o_l = tid >= k0 && tid < np ? orig[tid] : 0;
      __syncthreads();
#pragma unroll
      for (int t = 0; t < NP * NP / 256; ++t) {
        const int idx = tid + 256 * t;
        const int l = k0 + idx / np, c = idx % np;
        if (idx < cnt && (c < k0 || c >= k0 + B)) M[npos[l] * LD + c] = tmp[t];
      }
      if (tid >= k0 && tid < np) orig[npos[tid]] = o_l;
      if (w == 0 && lane < np) {
        const int to = npos[lane];
#pragma unroll
        for (int c = 0; c < B; ++c) M[to * LD + k0 + c] = pv[c];
      }
    }
    __syncthreads();
    // 3. columns outside the panel: row tiles R first (they read the old A_KC),
    // the pivot tile's T A_KC kept in registers until they are done
    shp_dbl4 keep[NT];
    if (w < nt && w == kb) {
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        keep[ct] = shp_dbl4{0.0, 0.0, 0.0, 0.0};
        if (ct < nt && ct != kb) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            keep[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(k0 + li) * LD + k0 + 4 * s + lk],
                                                             M[(k0 + 4 * s + lk) * LD + ct * B + li], keep[ct], 0,
                                                             0, 0);
        }
      }
    } else if (w < nt) {
      const int r0 = w * B;
      double ar[4];  // -A_RK T of this row tile
#pragma unroll
      for (int s = 0; s < 4; ++s) ar[s] = M[(r0 + li) * LD + k0 + 4 * s + lk];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        if (ct < nt && ct != kb) {
          shp_dbl4 acc;
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[r] = M[(r0 + crow[r]) * LD + ct * B + ccol[r]];
#pragma unroll
          for (int s = 0; s < 4; ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[s], M[(k0 + 4 * s + lk) * LD + ct * B + li], acc, 0, 0,
                                                       0);
#pragma unroll
          for (int r = 0; r < 4; ++r) M[(r0 + crow[r]) * LD + ct * B + ccol[r]] = acc[r];
        }
      }
    }
    __syncthreads();
    if (w < nt && w == kb) {
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        if (ct < nt && ct != kb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) M[(k0 + crow[r]) * LD + ct * B + ccol[r]] = keep[ct][r];
        }
    }
    __syncthreads();
  }
  if (tid < np) q[orig[tid]] = tid;
  __syncthreads();
  for (int idx = tid; idx < nb * nb; idx += 256) {
    const int j = idx / nb, i = idx - j * nb;
    const double v = M[i * LD + q[j]];
    inv64[doff + idx] = v;
    if (inv32) inv32[doff + idx] = (float)v;
  }
}

// In-place Gauss-Jordan inversion with partial pivoting for blocks of at
// most NB <= kDenseWave unknowns: one thread per row of the block, the row in
// registers.  Pivot rows are not swapped: step k takes the row p not yet used
// as a pivot with the largest |M[p][k]| (magnitudes compared on their leading
// 56 bits, the lowest row first among equal ones), scales it and eliminates
// column k from every other row.  Each step shifts the rows one register to
// the left and appends the new column of the inverse on the right, so that
// column k is always in v[0] and every register index is a constant: after
// nb steps v[NB - nb + j] holds column j of the in-place result M, and with
// p_k the pivot row of step k, inv[k][p_j] = M[p_k][j].
template <int NB, int NT>
__global__ __launch_bounds__(NT) void k_dense_inv_reg(const int* __restrict__ blk, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const double* __restrict__ a,
                                                      double* __restrict__ inv64, float* __restrict__ inv32,
                                                      int* __restrict__ err, const uint8_t* __restrict__ only) {
  static_assert(NT % 64 == 0 && NB <= NT && NT <= 256, "one thread per row, at most four wavefronts");
  constexpr int CW = NB <= 64 ? NB : (NB + 1) / 2;  // columns staged through LDS at a time
  constexpr int LD = NT + 1;
  __shared__ double S[CW * LD];
  __shared__ double piv[2][NB];
  __shared__ unsigned long long best[2][NT / 64];
  __shared__ int perm[NB];
  const int row0 = blk[4 * blockIdx.x], nb = blk[4 * blockIdx.x + 1];
  const size_t doff = (size_t)blk[4 * blockIdx.x + 2];
  const int i = threadIdx.x, lane = i & 63, w = i >> 6;
  if (nb > NB) return;  // a larger block: the workgroup kernel
  if (only) {           // incremental refresh: skip blocks none of whose rows changed
    int any = 0;
    for (int r = i; r < nb; r += NT) any |= only[row0 + r];
    if (!__syncthreads_or(any)) return;
  }
  double v[NB];
#pragma unroll
  for (int c0 = 0; c0 < NB; c0 += CW) {
    for (int idx = i; idx < CW * LD; idx += NT) S[idx] = 0.0;
    __syncthreads();
    if (i < nb) {
      const int r = row0 + i;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int c = ci[e] - row0 - c0;
        if (c >= 0 && c < CW && c0 + c < nb) S[c * LD + i] += a[e];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CW; ++j)
      if (c0 + j < NB) v[c0 + j] = S[j * LD + i];
    __syncthreads();
  }
  bool used = i >= nb;
  int myk = 0;
  for (int k = 0; k < nb; ++k) {
    const int buf = k & 1;
    unsigned long long key = 0;
    if (!used) {
      const double m = fabs(v[0]);
      if (m == m) key = ((unsigned long long)__double_as_longlong(m) & ~0xFFull) | (unsigned long long)(255 - i);
    }
    key = __ockl_wfred_max_u64(key);
    if (NT > 64) {
      if (lane == 0) best[buf][w] = key;
      __syncthreads();
      key = best[buf][0];
#pragma unroll
      for (int u = 1; u < NT / 64; ++u) key = best[buf][u] > key ? best[buf][u] : key;
    }
    if ((key >> 8) == 0) {  // no nonzero pivot left (uniform): singular block
      if (i == 0) atomicOr(err, 4);
      return;
    }
    const int p = 255 - (int)(key & 0xFF);
    double* pv = piv[buf];
    if (i == p) {
      const double inv = 1.0 / v[0];
#pragma unroll
      for (int j = 0; j + 1 < NB; ++j) pv[j] = v[j + 1] * inv;
      pv[NB - 1] = inv;
      perm[k] = p;
      used = true;
      myk = k;
    }
    __syncthreads();
    if (i == p) {
#pragma unroll
      for (int j = 0; j < NB; ++j) v[j] = pv[j];
    } else {
      const double f = v[0];
#pragma unroll
      for (int j = 0; j + 1 < NB; ++j) v[j] = v[j + 1] - f * pv[j];
      v[NB - 1] = -f * pv[NB - 1];
    }
  }
  __syncthreads();
  if (i < nb) {
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      const int j = r - (NB - nb);
      if (j >= 0) {
        const size_t o = doff + (size_t)perm[j] * nb + myk;
        inv64[o] = v[r];
        if (inv32) inv32[o] = (float)v[r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// cycle kernels (T = float for mixed precision, double for FP64 cycles)
// ---------------------------------------------------------------------------
// Sparse rows in the cycle kernels: G lanes per row, G in {1, 2, 4}.
// A row's sum does not depend on G: entry t of the row (t = 0, 1, ...) goes
// to partial sum t mod kAcc, each partial sum adds its entries in order, and
// the kAcc partial sums are combined by a fixed butterfly (v_u += v_{u+o} for
// u < o, o = kAcc/2, ..., 1).  Lane gl holds the partial sums u = gl + G j; the
// butterfly steps with o >= G run inside the lane, the others across lanes by
// xor shuffles, with the same operands in the same order.  The lane count is
// therefore a pure speed choice (tuned per level) and every row sum is the
// same bit for bit whatever the batch.
constexpr int kAcc = 4;

// row r of a tile-based launch: G blocks share one tile of kTileRows rows
template <int G>
__device__ inline int tile_row(const Tile& t, int& gl, unsigned bid) {
  gl = threadIdx.x % G;
  return t.r0 + (int)(bid % G) * (kTileRows / G) + (int)threadIdx.x / G;
}

// sum of a[e] f(ci[e]) over the row's entries [e0, e1); all G lanes of the
// row call it (the shuffles need them)
template <class T, int G, class F, class CI = int>
__device__ inline T row_sum(const CI* __restrict__ ci, const T* __restrict__ a, F f, int e0, int e1, int gl,
                            int cbase = 0) {
  static_assert(G >= 1 && G <= kAcc && (kAcc % G) == 0, "lane count must divide kAcc");
  constexpr int J = kAcc / G;  // partial sums per lane
  T acc[J];
#pragma unroll
  for (int j = 0; j < J; ++j) acc[j] = 0;
  int base = e0;
  constexpr int UN = J >= 4 ? 1 : 4 / J;  // chunks in flight: four entries' loads per lane
#pragma unroll UN
  for (; base + kAcc <= e1; base += kAcc) {  // whole chunks: loads first, all in flight
    int c[J];
    T v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      c[j] = cbase + (int)ci[base + gl + G * j];
      v[j] = a[base + gl + G * j];
    }
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] += v[j] * f(c[j]);
  }
  if (base < e1) {  // the last, partial chunk
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int e = base + gl + G * j;
      if (e < e1) acc[j] += a[e] * f(cbase + (int)ci[e]);
    }
  }
#pragma unroll
  for (int o = kAcc / 2; o >= G; o >>= 1) {
#pragma unroll
    for (int j = 0; j < o / G; ++j) acc[j] = acc[j] + acc[j + o / G];
  }
  T s = acc[0];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s = s + __shfl_xor(s, o);
  return s;
}

// CI = int: absolute columns; CI = int16_t: columns relative to the row (cbase = the row)
template <class T, class TX, int G, class CI = int>
__device__ inline T row_dot(const CI* __restrict__ ci, const T* __restrict__ a, const TX* __restrict__ x, int e0,
                            int e1, int gl, int cbase = 0) {
  return row_sum<T, G>(ci, a, [&](int j) -> T { return (T)x[j]; }, e0, e1, gl, cbase);
}

template <class T, int G, class F, class CI = int>
__device__ inline T row_dot_fn(const CI* __restrict__ ci, const T* __restrict__ a, F f, int e0, int e1, int gl,
                               int cbase = 0) {
  return row_sum<T, G>(ci, a, f, e0, e1, gl, cbase);
}

// first = 1: the first sweep from zero, x = omega D^-1 b; first = 2: the first
// two sweeps from zero in one pass (the first sweep's values recomputed where
// the second reads them, the same operations as the two passes)
template <class T, int G, class CI = int>
__global__ __launch_bounds__(256) void k_smooth(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                const int* __restrict__ rp, const CI* __restrict__ ci,
                                                const T* __restrict__ a, const T* __restrict__ dinv,
                                                const T* __restrict__ b, const T* __restrict__ xin,
                                                T* __restrict__ xout, T omega, int first,
                                                double* __restrict__ sol, const int8_t* __restrict__ cfm,
                                                int cfphase) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  if (!act[t.game]) return;
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  const bool in = i < t.r1;
  const int cb = sizeof(CI) < sizeof(int) ? i : 0;  // relative columns: offsets from the row
  if (cfm) {
    // C/F relaxation: this half sweep relaxes the coarse points (cfphase 1)
    // or the others (cfphase -1) and carries the rest over unchanged
    const int e0 = in ? rp[i] : 0, e1 = in ? rp[i + 1] : 0;
    const T ax = row_dot<T, T, G>(ci, a, xin, e0, e1, gl, cb);
    if (in && gl == 0) {
      const bool mine = (cfm[i] == CF_C) == (cfphase == 1);
      xout[i] = mine ? xin[i] + omega * dinv[i] * (b[i] - ax) : xin[i];
    }
    return;
  }
  if (first == 1) {
    if (in && gl == 0) xout[i] = omega * dinv[i] * b[i];
    return;
  }
  const int e0 = in ? rp[i] : 0, e1 = in ? rp[i + 1] : 0;
  if (first == 2) {
    const T ax = row_dot_fn<T, G>(ci, a, [&](int j) -> T { return omega * dinv[j] * b[j]; }, e0, e1, gl, cb);
    if (in && gl == 0) {
      const T x1 = omega * dinv[i] * b[i];
      xout[i] = x1 + omega * dinv[i] * (b[i] - ax);
    }
    return;
  }
  const T ax = row_dot<T, T, G>(ci, a, xin, e0, e1, gl, cb);  // all lanes: the shuffles need them
  if (in && gl == 0) {
    const T xi = xin[i] + omega * dinv[i] * (b[i] - ax);
    xout[i] = xi;
    if (sol) sol[i] += (double)xi;  // level 0's last sweep: the FP64 update of the refinement
  }
}

template <class T, int G, class CI = int>
__global__ __launch_bounds__(256) void k_resid(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                               const int* __restrict__ rp, const CI* __restrict__ ci,
                                               const T* __restrict__ a, const T* __restrict__ b,
                                               const T* __restrict__ x, T* __restrict__ r) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  if (!act[t.game]) return;
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  const bool in = i < t.r1;
  const int e0 = in ? rp[i] : 0, e1 = in ? rp[i + 1] : 0;
  const T ax = row_dot<T, T, G>(ci, a, x, e0, e1, gl, sizeof(CI) < sizeof(int) ? i : 0);
  if (in && gl == 0) r[i] = b[i] - ax;
}

// numeric refresh of the relaxation data of a level's rows in one pass, G
// lanes per row: Dirichlet flag (no nonzero off-diagonal entry), 1/a_ii
// (recomputed, or kept when `keep_diag`, e.g. from the assembly), divided by
// omega on Dirichlet rows so that the weighted relaxation solves them exactly
template <int G>
__global__ __launch_bounds__(256) void k_diag_dir(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                  const int* __restrict__ ci, const double* __restrict__ a,
                                                  int keep_diag, double inv_omega, uint8_t* __restrict__ dir,
                                                  double* __restrict__ d64, float* __restrict__ d32,
                                                  const uint8_t* __restrict__ only) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  // rows not flagged keep their data (the lanes of a row leave together)
  const bool in = i < t.r1 && (!only || only[i]);
  int any = 0;
  double d = 0.0;  // one diagonal entry per row: the sum over lanes is exact
  if (in) {
    for (int e = rp[i] + gl; e < rp[i + 1]; e += G) {
      const int c = ci[e];
      const double x = a[e];
      if (c == i) d += x; else if (x != 0.0) any = 1;
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    d += __shfl_xor(d, o);
    any |= __shfl_xor(any, o);
  }
  if (!in || gl != 0) return;
  double di = keep_diag ? d64[i] : (d != 0.0 ? 1.0 / d : 0.0);
  if (!any) di *= inv_omega;
  dir[i] = any ? 0 : 1;
  d64[i] = di;
  if (d32) d32[i] = (float)di;
}

// Strength of connection and its transpose with G lanes per row (levels of
// medium rows): the lanes take the row's entries in turn; the row maximum
// (order-independent) by shuffles within the row's lanes.  Same flags and
// counts as the thread-per-row and wavefront-per-row kernels.
template <int G>
__global__ __launch_bounds__(256) void k_strength_g(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                    const int* __restrict__ ci, const double* __restrict__ a,
                                                    const uint8_t* __restrict__ dir, double theta,
                                                    uint8_t* __restrict__ strong, int* __restrict__ lam) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  const bool in = i < t.r1;
  const int e0 = in ? rp[i] : 0, e1 = in ? rp[i + 1] : 0;
  const bool di = !in || dir[i] != 0;
  double m = 0.0;
  if (!di)
    for (int e = e0 + gl; e < e1; e += G) {
      const int j = ci[e];
      if (j != i && !dir[j]) m = fmax(m, -a[e]);
    }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  for (int e = e0 + gl; e < e1; e += G) {
    const int j = ci[e];
    const bool st = !di && j != i && !dir[j] && m > 0.0 && -a[e] >= theta * m;
    strong[e] = st ? 1 : 0;
    if (st) atomicAdd(&lam[j], 1);
  }
}

template <int G>
__global__ __launch_bounds__(256) void k_strength_t_g(const Tile* __restrict__ tiles, const int* __restrict__ rp,
                                                      const int* __restrict__ ci, const uint8_t* __restrict__ strong,
                                                      const int* __restrict__ st_rp, int* __restrict__ cursor,
                                                      int* __restrict__ st_ci) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  if (i >= t.r1) return;
  for (int e = rp[i] + gl; e < rp[i + 1]; e += G)
    if (strong[e]) {
      const int j = ci[e];
      const int pos = atomicAdd(&cursor[j], 1);
      st_ci[st_rp[j] + pos] = i;
    }
}

template <class T, int G>
__global__ __launch_bounds__(256) void k_restrict(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                  const int* __restrict__ rrp, const int* __restrict__ rci,
                                                  const T* __restrict__ rv, const T* __restrict__ rf,
                                                  T* __restrict__ bc) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  if (!act[t.game]) return;
  int gl;
  const int I = tile_row<G>(t, gl, bid);
  const bool in = I < t.r1;
  const int e0 = in ? rrp[I] : 0, e1 = in ? rrp[I + 1] : 0;
  const T s = row_dot<T, T, G>(rci, rv, rf, e0, e1, gl);
  if (in && gl == 0) bc[I] = s;
}

template <class T>
__global__ __launch_bounds__(256) void k_prolong(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                 const int* __restrict__ pc, const T* __restrict__ pv,
                                                 const T* __restrict__ xc, T* __restrict__ x) {
  Tile t = tiles[blockIdx.x];
  if (!act[t.game]) return;
  int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  T s = x[i];
  for (int q = 0; q < PW; ++q) {
    int c = pc[(size_t)i * PW + q];
    if (c >= 0) s += pv[(size_t)i * PW + q] * xc[c];
  }
  x[i] = s;
}

// row_dot<T, T, 1> with the vector entries produced by f(column): the same
// products in the same order, hence the same result as on an array
// one lane per row (the V-cycle tail, whose levels belong to one game: its
// sums need not match the level kernels'), four partial sums
template <class T, class F>
__device__ inline T row_dot1_f(const int* __restrict__ ci, const T* __restrict__ a, F f, int e0, int e1) {
  constexpr int U = 4;
  T acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = 0;
  int e = e0;
  for (; e + (U - 1) < e1; e += U) {
    int c[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = ci[e + u];
      v[u] = a[e + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] += v[u] * f(c[u]);
  }
  for (; e < e1; ++e) acc[0] += a[e] * f(ci[e]);
  T s = acc[0];
#pragma unroll
  for (int u = 1; u < U; ++u) s += acc[u];
  return s;
}

// V-cycle tail of one game per workgroup (see internal.hpp).  Same steps as
// the level-by-level cycle: nu1 weighted-Jacobi sweeps from zero, residual,
// restriction, the coarser levels, prolongation and correction, nu2 sweeps;
// the dense inverse on the game's last level.  The iterates of every tail
// level live in LDS (two vectors per level, dynamic LDS sized by the host);
// matrices, right-hand sides and the level-l0 result are in global memory.
template <class T>
__global__ __launch_bounds__(kTailThreads) void k_tail(const int* __restrict__ games, int l0, int nlev, int G,
                                                       const TailLev<T>* __restrict__ lvs,
                                                       const TailGL* __restrict__ gls, const int* __restrict__ act,
                                                       T omega, int nu1, int nu2, int out_y,
                                                       double* __restrict__ sol, TailRefine rf) {
  extern __shared__ unsigned char tail_lds[];
  __shared__ int off[kTailMaxLevels];  // by level - l0
  T* lds = reinterpret_cast<T*>(tail_lds);
  const int g = games[blockIdx.x];
  if (!act[g]) return;
  const int tid = threadIdx.x;
  if (tid == 0) {  // the level-l vectors: x at off[l - l0], y at off[l - l0] + rows
    int o = 0;
    for (int l = l0; l < nlev && l - l0 < kTailMaxLevels; ++l) {
      const TailGL q = gls[(size_t)l * G + g];
      if (!(q.flags & kTailPresent)) break;
      off[l - l0] = o;
      o += 2 * (q.r1 - q.r0);
    }
  }
  __syncthreads();
  __shared__ double s_rm[kTailThreads / 64], s_xm[kTailThreads / 64];
  __shared__ int s_go;
  const int ncyc = rf.cycles > 0 ? rf.cycles : 1;
  for (int cyc = 0; cyc < ncyc; ++cyc) {
    unsigned parity = 0;  // bit l - l0: the level-l iterate is in y
    int deep = l0;
    // ---- down
    for (int l = l0; l < nlev; ++l) {
      const TailGL q = gls[(size_t)l * G + g];
      const TailLev<T> L = lvs[l];
      const int r0 = q.r0, n = q.r1 - q.r0;
      T* xv = lds + off[l - l0];
      T* yv = xv + n;
      deep = l;
      if (q.flags & kTailDense) {  // x = inv b: one wavefront per row, lanes over columns
        const int lane = tid & 63;
        for (int i = tid >> 6; i < n; i += kTailThreads / 64) {
          T acc = 0;
          for (int j = lane; j < n; j += 64) acc += L.dm[(size_t)q.doff + (size_t)j * n + i] * L.b[r0 + j];
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
          if (lane == 0) xv[i] = acc;
        }
        __syncthreads();
        break;
      }
      if (!(q.flags & kTailCont)) break;
      T* cur = xv;
      T* nxt = yv;
      for (int i = tid; i < n; i += kTailThreads) cur[i] = omega * L.d[r0 + i] * L.b[r0 + i];
      __syncthreads();
      for (int k = 1; k < nu1; ++k) {
        const T* c0 = cur;
        for (int i = tid; i < n; i += kTailThreads) {
          const int r = r0 + i;
          nxt[i] = cur[i] + omega * L.d[r] *
                                (L.b[r] - row_dot1_f<T>(L.ci, L.a, [&](int j) -> T { return c0[j - r0]; }, L.rp[r],
                                                        L.rp[r + 1]));
        }
        __syncthreads();
        T* t = cur; cur = nxt; nxt = t;
      }
      if (cur == yv) parity |= 1u << (l - l0);
      if (!(q.flags & kTailNext)) break;  // no coarse rows: smoothing only
      T* rr = nxt;                         // the free vector holds the residual
      {
        const T* c0 = cur;
        for (int i = tid; i < n; i += kTailThreads) {
          const int r = r0 + i;
          rr[i] = L.b[r] - row_dot1_f<T>(L.ci, L.a, [&](int j) -> T { return c0[j - r0]; }, L.rp[r], L.rp[r + 1]);
        }
      }
      __syncthreads();
      const TailGL qn = gls[(size_t)(l + 1) * G + g];
      const TailLev<T> Ln = lvs[l + 1];
      for (int I = qn.r0 + tid; I < qn.r1; I += kTailThreads)
        Ln.b[I] = row_dot1_f<T>(L.rci, L.rv, [&](int i) -> T { return rr[i - r0]; }, L.rrp[I], L.rrp[I + 1]);
      __syncthreads();
    }
    // ---- up
    for (int l = deep; l >= l0; --l) {
      const TailGL q = gls[(size_t)l * G + g];
      if (!(q.flags & kTailCont) || (q.flags & kTailDense)) continue;  // the dense result is in x
      const TailLev<T> L = lvs[l];
      const int r0 = q.r0, n = q.r1 - q.r0;
      T* xv = lds + off[l - l0];
      T* yv = xv + n;
      T* cur = ((parity >> (l - l0)) & 1u) ? yv : xv;
      T* nxt = ((parity >> (l - l0)) & 1u) ? xv : yv;
      if (l < deep) {
        const TailGL qn = gls[(size_t)(l + 1) * G + g];
        const int n1 = qn.r1 - qn.r0;
        const T* xc = lds + off[l + 1 - l0] + (((parity >> (l + 1 - l0)) & 1u) ? n1 : 0);
        for (int i = tid; i < n; i += kTailThreads) {
          const int r = r0 + i;
          T acc = cur[i];
#pragma unroll
          for (int k = 0; k < PW; ++k) {
            const int c = L.pc[(size_t)r * PW + k];
            if (c >= 0) acc += L.pv[(size_t)r * PW + k] * xc[c - qn.r0];
          }
          cur[i] = acc;
        }
        __syncthreads();
      }
      for (int k = 0; k < nu2; ++k) {
        const T* c0 = cur;
        for (int i = tid; i < n; i += kTailThreads) {
          const int r = r0 + i;
          nxt[i] = cur[i] + omega * L.d[r] *
                                (L.b[r] - row_dot1_f<T>(L.ci, L.a, [&](int j) -> T { return c0[j - r0]; }, L.rp[r],
                                                        L.rp[r + 1]));
        }
        __syncthreads();
        T* t = cur; cur = nxt; nxt = t;
      }
      if (cur == yv) parity |= 1u << (l - l0); else parity &= ~(1u << (l - l0));
    }
    // ---- the level-l0 result where the caller expects it
    const TailGL q = gls[(size_t)l0 * G + g];
    const TailLev<T> L = lvs[l0];
    const int n = q.r1 - q.r0;
    const T* src = lds + off[0] + ((parity & 1u) ? n : 0);
    T* dst = out_y ? L.y : L.x;
    for (int i = tid; i < n; i += kTailThreads) {
      dst[q.r0 + i] = src[i];
      if (sol) sol[q.r0 + i] += (double)src[i];  // level 0: the FP64 update of the refinement
    }
    if (rf.cycles == 0) break;
    // ---- refinement (l0 == 0): FP64 residual of the game's rows into level 0's
    //      right-hand side, then the stop test
    __syncthreads();
    double rm = 0.0, xm = 0.0;
    for (int i = q.r0 + tid; i < q.r1; i += kTailThreads) {
      const double ax = row_dot1_f<double>(L.ci, rf.a64, [&](int j) -> double { return sol[j]; }, L.rp[i],
                                           L.rp[i + 1]);
      const double r = rf.rhs[i] - ax;
      L.b[i] = (T)r;
      const double xi = sol[i];
      rm = fmax(rm, r == r ? fabs(r) : INFINITY);  // NaN must survive the maximum
      xm = fmax(xm, xi == xi ? fabs(xi) : INFINITY);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      rm = fmax(rm, __shfl_xor(rm, o));
      xm = fmax(xm, __shfl_xor(xm, o));
    }
    if ((tid & 63) == 0) {
      s_rm[tid >> 6] = rm;
      s_xm[tid >> 6] = xm;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < kTailThreads / 64; ++w) {
        rm = fmax(rm, s_rm[w]);
        xm = fmax(xm, s_xm[w]);
      }
      s_go = lin_decide(g, rm, xm, rf.bnorm, rf.ctl, rf.act, rf.norm) ? 1 : 0;
    }
    __syncthreads();
    if (!s_go) break;
  }
}

// x_blk = inv_blk b_blk, one workgroup per block; inv is column-major
template <class T>
__global__ __launch_bounds__(256) void k_dense_solve(const int* __restrict__ blk, const int* __restrict__ act,
                                                     const T* __restrict__ inv, const T* __restrict__ b,
                                                     T* __restrict__ x) {
  __shared__ T bs[kDenseMax];
  const int row0 = blk[4 * blockIdx.x], nb = blk[4 * blockIdx.x + 1];
  const size_t doff = (size_t)blk[4 * blockIdx.x + 2];
  const int slot = blk[4 * blockIdx.x + 3];
  if (!act[slot]) return;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) bs[j] = b[row0 + j];
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    T s = 0;
    for (int j = 0; j < nb; ++j) s += inv[doff + (size_t)j * nb + i] * bs[j];
    x[row0 + i] = s;
  }
}

// FP64 residual of the refinement: r = b - A x, its copy in the cycle type,
// and per-game max |r|, max |x|.
template <class T, int G>
__device__ inline void resid64_block(const Tile& t, unsigned bid, const int* __restrict__ rp, const int* __restrict__ ci,
                                     const double* __restrict__ a, const double* __restrict__ b,
                                     const double* __restrict__ x, T* __restrict__ rc, const Stripes& norm) {
  int gl;
  const int i = tile_row<G>(t, gl, bid);
  const bool in = i < t.r1;
  double rm = 0.0, xm = 0.0;
  const int e0 = in ? rp[i] : 0, e1 = in ? rp[i + 1] : 0;
  const double ax = row_dot<double, double, G>(ci, a, x, e0, e1, gl);
  if (in && gl == 0) {
    const double s = b[i] - ax;
    rc[i] = (T)s;
    const double xi = x[i];
    rm = s == s ? fabs(s) : INFINITY;   // NaN must survive the maximum
    xm = xi == xi ? fabs(xi) : INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1) {
    rm = fmax(rm, __shfl_xor(rm, o));
    xm = fmax(xm, __shfl_xor(xm, o));
  }
  const double v[2] = {rm, xm};
  block_fold<2, 0>(norm, t.game, v, 0u, nullptr);
}

// FP64 residual r = b - A x (copied to rc in the cycle type) and per-game
// maxima of |r| and |x| folded into the stripes
template <class T, int G>
__global__ __launch_bounds__(256) void k_resid64(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                 const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ x, T* __restrict__ rc,
                                                 Stripes norm) {
  const unsigned bid = blockIdx.x;
  const Tile t = tiles[bid / G];
  if (!act[t.game]) return;
  resid64_block<T, G>(t, bid, rp, ci, a, b, x, rc, norm);
}

// ---------------------------------------------------------------------------
// Cycle kernels on the stencil form of level 0, one thread per row: slot t of
// the row is loaded from its own array (coalesced over rows), its column is
// the row plus the offset its code names.  Entry t goes into partial sum
// t mod kAcc and the partial sums meet in row_sum's butterfly, so a row sum is
// the same bit for bit as the CSR kernels'.
// ---------------------------------------------------------------------------
template <class T, class F>
__device__ inline T st_row_sum(const StencilView& sv, const T* __restrict__ a, int i, const int* __restrict__ off,
                               F f) {
  // the game's offsets (the same for the whole tile) in registers
  int o[kStencilMax];
#pragma unroll
  for (int q = 0; q < kStencilMax; ++q) o[q] = off[q];
  const uint32_t c = sv.code[i];
  const int len = (int)(c >> 24);
  T v[kStencilMax];
#pragma unroll
  for (int t = 0; t < kStencilMax; ++t) v[t] = t < sv.w ? a[(size_t)t * sv.n + i] : (T)0;
  T acc[kAcc];
#pragma unroll
  for (int j = 0; j < kAcc; ++j) acc[j] = 0;
#pragma unroll
  for (int t = 0; t < kStencilMax; ++t) {
    const uint32_t ct = (c >> (3 * t)) & 7u;
    int d = o[0];
#pragma unroll
    for (int q = 1; q < kStencilMax; ++q) d = ct == (uint32_t)q ? o[q] : d;
    if (t < len) acc[t % kAcc] += v[t] * f(i + d);
  }
#pragma unroll
  for (int o = kAcc / 2; o >= 1; o >>= 1) {
#pragma unroll
    for (int j = 0; j < o; ++j) acc[j] = acc[j] + acc[j + o];
  }
  return acc[0];
}

template <class T>
__global__ __launch_bounds__(256) void k_smooth_st(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                   StencilView sv, const T* __restrict__ a,
                                                   const T* __restrict__ dinv, const T* __restrict__ b,
                                                   const T* __restrict__ xin, T* __restrict__ xout, T omega,
                                                   int first, double* __restrict__ sol) {
  const Tile t = tiles[blockIdx.x];
  if (!act[t.game]) return;
  const int i = t.r0 + (int)threadIdx.x;
  if (i >= t.r1) return;
  const int* off = sv.off + kStencilMax * t.game;
  if (first == 1) {
    xout[i] = omega * dinv[i] * b[i];
    return;
  }
  if (first == 2) {
    const T ax = st_row_sum<T>(sv, a, i, off, [&](int j) -> T { return omega * dinv[j] * b[j]; });
    const T x1 = omega * dinv[i] * b[i];
    xout[i] = x1 + omega * dinv[i] * (b[i] - ax);
    return;
  }
  const T ax = st_row_sum<T>(sv, a, i, off, [&](int j) -> T { return (T)xin[j]; });
  const T xi = xin[i] + omega * dinv[i] * (b[i] - ax);
  xout[i] = xi;
  if (sol) sol[i] += (double)xi;
}

template <class T>
__global__ __launch_bounds__(256) void k_resid_st(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                  StencilView sv, const T* __restrict__ a,
                                                  const T* __restrict__ b, const T* __restrict__ x,
                                                  T* __restrict__ r) {
  const Tile t = tiles[blockIdx.x];
  if (!act[t.game]) return;
  const int i = t.r0 + (int)threadIdx.x;
  if (i >= t.r1) return;
  const T ax = st_row_sum<T>(sv, a, i, sv.off + kStencilMax * t.game, [&](int j) -> T { return (T)x[j]; });
  r[i] = b[i] - ax;
}

template <class T>
__global__ __launch_bounds__(256) void k_resid64_st(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                    StencilView sv, const double* __restrict__ a,
                                                    const double* __restrict__ b, const double* __restrict__ x,
                                                    T* __restrict__ rc, Stripes norm) {
  const Tile t = tiles[blockIdx.x];
  if (!act[t.game]) return;
  const int i = t.r0 + (int)threadIdx.x;
  double rm = 0.0, xm = 0.0;
  if (i < t.r1) {
    const double ax =
        st_row_sum<double>(sv, a, i, sv.off + kStencilMax * t.game, [&](int j) -> double { return x[j]; });
    const double s = b[i] - ax;
    rc[i] = (T)s;
    const double xi = x[i];
    rm = s == s ? fabs(s) : INFINITY;  // NaN must survive the maximum
    xm = xi == xi ? fabs(xi) : INFINITY;
  }
  for (int o = 32; o > 0; o >>= 1) {
    rm = fmax(rm, __shfl_xor(rm, o));
    xm = fmax(xm, __shfl_xor(xm, o));
  }
  const double v[2] = {rm, xm};
  block_fold<2, 0>(norm, t.game, v, 0u, nullptr);
}

template <class T>
__global__ __launch_bounds__(256) void k_update64(const Tile* __restrict__ tiles, const int* __restrict__ act,
                                                  const T* __restrict__ e, double* __restrict__ x) {
  Tile t = tiles[blockIdx.x];
  if (!act[t.game]) return;
  int i = t.r0 + threadIdx.x;
  if (i < t.r1) x[i] += (double)e[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// the per-level flags before strength and PMIS, in one launch: lam = 0
// (n + 1 entries), cf = -2 (rows of games that end on this level) and dir = 1 (n), strong = 0 (nnz)
__global__ void k_level_init(int n, int nnz, int* __restrict__ lam, int8_t* __restrict__ cf,
                             uint8_t* __restrict__ dir, uint8_t* __restrict__ strong) {
  const int m = max(n + 1, nnz);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    if (i <= n) lam[i] = 0;
    if (i < n) {
      cf[i] = -2;
      dir[i] = 1;
    }
    if (i < nnz) strong[i] = 0;
  }
}
void amg_level_init(int n, int nnz, int* lam, int8_t* cf, uint8_t* dir, uint8_t* strong, hipStream_t s) {
  const int m = std::max(n + 1, nnz);
  hipLaunchKernelGGL(k_level_init, dim3(grid_for(m)), dim3(kBlock), 0, s, n, nnz, lam, cf, dir, strong);
  SHP_LAUNCH_CHECK();
}
void amg_diag_dir(const Tile* t, int nt, const int* rp, const int* ci, const double* a, bool keep_diag,
                  double inv_omega, uint8_t* dir, double* d64, float* d32, int g, hipStream_t s,
                  const uint8_t* only) {
  if (!nt) return;
  const int kd = keep_diag ? 1 : 0;
  if (g == 16)
    hipLaunchKernelGGL(k_diag_dir<16>, dim3(nt * 16), dim3(kTileRows), 0, s, t, rp, ci, a, kd, inv_omega, dir, d64, d32,
                       only);
  else if (g == 4)
    hipLaunchKernelGGL(k_diag_dir<4>, dim3(nt * 4), dim3(kTileRows), 0, s, t, rp, ci, a, kd, inv_omega, dir, d64, d32,
                       only);
  else
    hipLaunchKernelGGL(k_diag_dir<1>, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, a, kd, inv_omega, dir, d64, d32,
                       only);
  SHP_LAUNCH_CHECK();
}
void amg_strength(const Tile* t, int nt, const int* rp, const int* ci, const double* a,
                  const uint8_t* dir, double theta, uint8_t* strong, int* lam, int lanes, hipStream_t s) {
  if (!nt) return;
  if (lanes == 64)
    hipLaunchKernelGGL(k_strength_w, dim3(nt * (kTileRows / 4)), dim3(256), 0, s, t, rp, ci, a, dir, theta, strong,
                       lam);
  else if (lanes == 4)
    hipLaunchKernelGGL(k_strength_g<4>, dim3(nt * 4), dim3(kTileRows), 0, s, t, rp, ci, a, dir, theta, strong,
                       lam);
  else
    hipLaunchKernelGGL(k_strength, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, a, dir, theta, strong, lam);
  SHP_LAUNCH_CHECK();
}
void amg_strength_t(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                    const int* st_rp, int* cursor, int* st_ci, int lanes, hipStream_t s) {
  if (!nt) return;
  if (lanes == 64)
    hipLaunchKernelGGL(k_strength_t_w, dim3(nt * (kTileRows / 4)), dim3(256), 0, s, t, rp, ci, strong, st_rp,
                       cursor, st_ci);
  else if (lanes == 4)
    hipLaunchKernelGGL(k_strength_t_g<4>, dim3(nt * 4), dim3(kTileRows), 0, s, t, rp, ci, strong, st_rp, cursor,
                       st_ci);
  else
    hipLaunchKernelGGL(k_strength_t, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, strong, st_rp, cursor,
                       st_ci);
  SHP_LAUNCH_CHECK();
}
void amg_pmis_init(const Tile* t, int nt, const int* goff, const uint8_t* dir, const int* lam,
                   uint32_t salt, int8_t* cf, uint64_t* key, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_pmis_init, dim3(nt), dim3(kTileRows), 0, s, t, goff, dir, lam, salt, cf, key);
  SHP_LAUNCH_CHECK();
}
void amg_pmis_select(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                     const int* st_rp, const int* st_ci, const int8_t* cf, const uint64_t* key,
                     int* newc, int* left, int round, bool wide, hipStream_t s) {
  if (!nt) return;
  if (wide)
    hipLaunchKernelGGL(k_pmis_select_w, dim3(nt * (kTileRows / 4)), dim3(256), 0, s, t, rp, ci, strong, st_rp,
                       st_ci, cf, key, newc, left, round);
  else
    hipLaunchKernelGGL(k_pmis_select, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, strong, st_rp, st_ci,
                       cf, key, newc, left, round);
  SHP_LAUNCH_CHECK();
}
void amg_pmis_update(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong,
                     int8_t* cf, const int* newc, int* left, int round, bool wide, hipStream_t s) {
  if (!nt) return;
  if (wide)
    hipLaunchKernelGGL(k_pmis_update_w, dim3(nt * (kTileRows / 4)), dim3(256), 0, s, t, rp, ci, strong, cf, newc,
                       left, round);
  else
    hipLaunchKernelGGL(k_pmis_update, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, strong, cf, newc, left, round);
  SHP_LAUNCH_CHECK();
}
void amg_pmis_small(const Tile* t, int nt, const int* rp, const int* ci, const uint8_t* strong, const int* st_rp,
                    const int* st_ci, int8_t* cf, const uint64_t* key, int* newc, int* left, int max_rounds,
                    hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_pmis_small, dim3(1), dim3(kPmisSmallThreads), 0, s, t, nt, rp, ci, strong, st_rp, st_ci, cf,
                     key, newc, left, max_rounds);
  SHP_LAUNCH_CHECK();
}
void amg_fill_cf(const Tile* t, int nt, int8_t* cf, int8_t val, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_fill_cf, dim3(nt), dim3(kTileRows), 0, s, t, cf, val);
  SHP_LAUNCH_CHECK();
}
void amg_is_c(const int8_t* cf, int* out, int n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_is_c, dim3(grid_for(n)), dim3(kBlock), 0, s, cf, out, n);
  SHP_LAUNCH_CHECK();
}
void amg_gather_int(const int* src, const int* idx, int m, int* dst, hipStream_t s) {
  if (!m) return;
  hipLaunchKernelGGL(k_gather_int, dim3(grid_for(m)), dim3(kBlock), 0, s, src, idx, m, dst);
  SHP_LAUNCH_CHECK();
}
void amg_interp(const Tile* t, int nt, const int* rp, const int* ci, const double* a, const double* dinv,
                const uint8_t* strong, const int8_t* cf, const int* cidx, const uint8_t* dir, int* pc,
                double* pv, int* capped, int wave, int* defer, int rows, hipStream_t s) {
  if (!nt) return;
  const unsigned lb = (unsigned)std::max(1, std::min(rows, 32768));  // wavefronts of the list kernels
  if (wave == 2) {
    // long rows: the 512-slot instance (18 KB of LDS per row) for all rows,
    // then the rows it could not hold with the largest one (33 KB)
    zero_counters_async(s, defer);
    hipLaunchKernelGGL((k_interp_wave<512, 128, 256, true>), dim3(nt * kTileRows), dim3(64), 0, s, t, rp, ci, a, dinv,
                       strong, cf, cidx, dir, pc, pv, capped, defer);
    SHP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_interp_wave_list<1024, 256, false>), dim3(lb), dim3(64), 0, s, defer, rp, ci, a, dinv,
                       strong, cf, cidx, dir, pc, pv, capped, (int*)nullptr);
  } else if (wave == 1) {
    // a small instance (about 5 KB of LDS per row: twice the rows per CU of
    // the next size) for all rows, then the rows it could not hold
    zero_counters_async(s, defer);
    hipLaunchKernelGGL((k_interp_wave<128, 32, 128, true>), dim3(nt * kTileRows), dim3(64), 0, s, t, rp, ci, a, dinv,
                       strong, cf, cidx, dir, pc, pv, capped, defer);
    SHP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_interp_wave_list<512, 128, false>), dim3(lb), dim3(64), 0, s, defer, rp, ci, a, dinv,
                       strong, cf, cidx, dir, pc, pv, capped, (int*)nullptr);
  } else if (wave == 3) {
    // four lanes per row for the rows that fit, then the small wavefront
    // instance over the others, then the larger over what that one could
    // not hold (the same weights as wave == 1)
    int* defer2 = defer + rows + 1;
    zero_counters_async(s, defer, defer2);
    hipLaunchKernelGGL(k_interp_quad, dim3(nt * (kTileRows / 16)), dim3(64), 0, s, t, rp, ci, a, dinv, strong, cf,
                       cidx, dir, pc, pv, defer);
    SHP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_interp_wave_list<128, 32, true>), dim3(lb), dim3(64), 0, s, defer, rp, ci, a, dinv, strong,
                       cf, cidx, dir, pc, pv, capped, defer2);
    SHP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_interp_wave_list<512, 128, false>), dim3(lb), dim3(64), 0, s, defer2, rp, ci, a, dinv,
                       strong, cf, cidx, dir, pc, pv, capped, (int*)nullptr);
  } else {
    // the small set first (twice the wavefronts per CU), then the rows it
    // could not hold
    zero_counters_async(s, defer);
    hipLaunchKernelGGL((k_interp_lds<kIChatSmall, true>), dim3(nt * (kTileRows / kIThreads)), dim3(kIThreads), 0, s,
                       t, rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv, capped, defer);
    SHP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_interp_lds_list, dim3(std::max(1, std::min((rows + kIThreads - 1) / kIThreads, 1024))),
                       dim3(kIThreads), 0, s, defer, rp, ci, a, dinv, strong, cf, cidx, dir, pc, pv, capped);
  }
  SHP_LAUNCH_CHECK();
}
void amg_pt_count(const Tile* t, int nt, const int* pc, int* cnt, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_pt_count, dim3(nt), dim3(kTileRows), 0, s, t, pc, cnt);
  SHP_LAUNCH_CHECK();
}
void amg_pt_fill(const Tile* t, int nt, const int* pc, const double* pv, const int* rrp, int* cursor,
                 int* rci, double* rv, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_pt_fill, dim3(nt), dim3(kTileRows), 0, s, t, pc, pv, rrp, cursor, rci, rv);
  SHP_LAUNCH_CHECK();
}
void amg_sort_rows(const int* rp, int* ci, double* v, int n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_sort_rows_seg, dim3((n + 15) / 16), dim3(256), 0, s, rp, ci, v, n);
  SHP_LAUNCH_CHECK();
}
void amg_rap_bound(int nc, const int* rrp, const int* rci, const int* rp, int* ub, int pw, hipStream_t s) {
  if (!nc) return;
  hipLaunchKernelGGL(k_rap_bound, dim3(grid_for(nc)), dim3(kBlock), 0, s, nc, rrp, rci, rp, ub, pw);
  SHP_LAUNCH_CHECK();
}
// identity operators over n rows: R = I in CSR (rrp, rci, rv) and P = I in
// the ELL layout (pc, pv; one filled slot per row)
__global__ void k_identity_ops(int n, int* __restrict__ rrp, int* __restrict__ rci, double* __restrict__ rv,
                               int* __restrict__ pc, double* __restrict__ pv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  rrp[i] = i;
  if (i == n) return;
  rci[i] = i;
  rv[i] = 1.0;
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    pc[(size_t)i * PW + q] = q == 0 ? i : -1;
    pv[(size_t)i * PW + q] = q == 0 ? 1.0 : 0.0;
  }
}
void amg_identity_ops(int n, int* rrp, int* rci, double* rv, int* pc, double* pv, hipStream_t s) {
  hipLaunchKernelGGL(k_identity_ops, dim3(grid_for(n + 1)), dim3(kBlock), 0, s, n, rrp, rci, rv, pc, pv);
  SHP_LAUNCH_CHECK();
}
// rows whose flag is set, appended to list (order free: each row's result
// does not depend on it); *count = their number (zero before the launch).
// Each thread looks at kFlagPer rows; one atomic per workgroup.
constexpr int kFlagPer = 4;
__global__ __launch_bounds__(kBlock) void k_flag_list(const uint8_t* __restrict__ flags, int n, int* __restrict__ list,
                                                      int* __restrict__ count) {
  __shared__ int s_w[kBlock / 64];
  __shared__ int s_base;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i0 = (blockIdx.x * kBlock + threadIdx.x) * kFlagPer;
  int mine = 0;
#pragma unroll
  for (int u = 0; u < kFlagPer; ++u) mine += (i0 + u < n && flags[i0 + u] != 0) ? 1 : 0;
  int incl = mine;  // wavefront scan of the counts
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_w[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 0; k < kBlock / 64; ++k) {
      const int c = s_w[k];
      s_w[k] = tot;
      tot += c;
    }
    s_base = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  int at = s_base + s_w[w] + incl - mine;
#pragma unroll
  for (int u = 0; u < kFlagPer; ++u)
    if (i0 + u < n && flags[i0 + u] != 0) list[at++] = i0 + u;
}
static unsigned flag_blocks(int n) { return (unsigned)((n + kBlock * kFlagPer - 1) / (kBlock * kFlagPer)); }
constexpr int kRapListBlocks = 2048;  // grid of a refresh over a list of rows

// Levels with few coarse rows (long rows): one workgroup of 256 lanes per
// row.  Larger levels: with a first kernel (kern: thread per row with 16 or
// 32 columns, or four lanes per row with 32 or 64) taking the rows that fit,
// then the wavefront kernel over the rows it handed on, then the workgroup
// kernel over the rows the wavefront kernel could not take; without, the
// wavefront kernel over every row.  big holds 2 (nc + 1) ints: the two
// hand-over lists.  The results do not depend on the path.
template <int MODE, typename K>
static void first_pass(K kern, unsigned blocks, unsigned threads, hipStream_t s, int nc, const int* rrp,
                       const int* rci, const double* rv, const int* rp, const int* ci, const double* a, const int* pc,
                       const double* pv, const int* toff, int* tcnt, int* tcol, double* tval, const int* crp,
                       const int* cci, double* cval, const uint8_t* only, int* mid, const int* tl, const int* tn) {
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), 0, s, nc, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol,
                     tval, crp, cci, cval, only, mid, tl, tn);
  SHP_LAUNCH_CHECK();
}

template <int MODE>
static void rap_launch(int nc, const int* rrp, const int* rci, const double* rv, const int* rp, const int* ci,
                       const double* a, const int* pc, const double* pv, const int* toff, int* tcnt, int* tcol,
                       double* tval, const int* crp, const int* cci, double* cval, int* err, const uint8_t* only,
                       int* big, hipStream_t s, int* list, int kern) {
  if (nc < 8192) {
    hipLaunchKernelGGL((k_rap<256, MODE>), dim3(nc), dim3(256), 0, s, nc, rrp, rci, rv, rp, ci, a, pc, pv, toff,
                       tcnt, tcol, tval, crp, cci, cval, err, only);
    SHP_LAUNCH_CHECK();
    return;
  }
  int* mid = big + nc + 1;  // rows handed from the first kernel to the wavefront kernel
  const bool refresh = only && list;
  zero_counters_async(s, big, kern != kGalWave ? mid : nullptr, refresh ? list : nullptr);
  if (refresh) {
    // a refresh: the flagged rows into a list, then a fixed grid over it (a
    // grid over every coarse row costs as much as the work when few changed)
    hipLaunchKernelGGL(k_flag_list, dim3(flag_blocks(nc)), dim3(kBlock), 0, s, only, nc, list + 1, list);
    SHP_LAUNCH_CHECK();
  }
  const unsigned wblocks = (unsigned)std::min<int>((nc + 3) / 4, kRapListBlocks);
  if (kern != kGalWave) {
    const int* tl = refresh ? (const int*)(list + 1) : nullptr;
    const int* tn = refresh ? (const int*)list : nullptr;
    const bool quad = kern == kGalQuad32 || kern == kGalQuad64;
    const int per = quad ? 64 : 64;  // rows per workgroup
    const unsigned blocks = refresh ? (unsigned)std::min<int>((nc + per - 1) / per, kRapListBlocks)
                                    : (unsigned)((nc + per - 1) / per);
#define SHP_FIRST(K, T) first_pass<MODE>(K, blocks, T, s, nc, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, \
                                         crp, cci, cval, only, mid, tl, tn)
    switch (kern) {
      case kGalThread16: SHP_FIRST((k_rap_thr<MODE, 16>), 64); break;
      case kGalThread32: SHP_FIRST((k_rap_thr<MODE, 32>), 64); break;
      case kGalQuad32: SHP_FIRST((k_rap_quad<MODE, 32>), 256); break;
      default: SHP_FIRST((k_rap_quad<MODE, 64>), 256); break;
    }
#undef SHP_FIRST
    hipLaunchKernelGGL((k_rap_small<MODE>), dim3(wblocks), dim3(256), 0, s, nc, rrp, rci, rv, rp, ci, a, pc, pv,
                       toff, tcnt, tcol, tval, crp, cci, cval, only, big, (const int*)(mid + 1), (const int*)mid);
  } else if (refresh) {
    hipLaunchKernelGGL((k_rap_small<MODE>), dim3(wblocks), dim3(256), 0, s, nc, rrp, rci, rv, rp, ci, a, pc, pv,
                       toff, tcnt, tcol, tval, crp, cci, cval, only, big, (const int*)(list + 1), (const int*)list);
  } else {
    hipLaunchKernelGGL((k_rap_small<MODE>), dim3((nc + 3) / 4), dim3(256), 0, s, nc, rrp, rci, rv, rp, ci, a, pc,
                       pv, toff, tcnt, tcol, tval, crp, cci, cval, only, big, (const int*)nullptr, (const int*)nullptr);
  }
  SHP_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_rap_list<128, MODE>), dim3(std::min(nc, 2048)), dim3(128), 0, s, big, rrp, rci, rv, rp, ci,
                     a, pc, pv, toff, tcnt, tcol, tval, crp, cci, cval, err);
  SHP_LAUNCH_CHECK();
}
void amg_rap_fused(int nc, const int* rrp, const int* rci, const double* rv, const int* rp, const int* ci,
                   const double* a, const int* pc, const double* pv, const int* toff, int* tcnt, int* tcol,
                   double* tval, int* err, int* big, hipStream_t s, int kern) {
  if (!nc) return;
  rap_launch<kRapFused>(nc, rrp, rci, rv, rp, ci, a, pc, pv, toff, tcnt, tcol, tval, nullptr, nullptr, nullptr, err,
                        nullptr, big, s, nullptr, kern);
}
void amg_rap_compact(int nc, const int* toff, const int* tcol, const double* tval, const int* crp, int* cci,
                     double* cval, hipStream_t s) {
  if (!nc) return;
  hipLaunchKernelGGL(k_rap_compact, dim3((nc + 31) / 32), dim3(256), 0, s, nc, toff, tcol, tval, crp, cci, cval);
  SHP_LAUNCH_CHECK();
}
void amg_rap_known(int nc, const int* rrp, const int* rci, const double* rv, const int* rp, const int* ci,
                   const double* a, const int* pc, const double* pv, const int* crp, const int* cci, double* cval,
                   int* err, int* big, hipStream_t s, const uint8_t* only, int* list, int kern) {
  if (!nc) return;
  rap_launch<kRapKnown>(nc, rrp, rci, rv, rp, ci, a, pc, pv, nullptr, nullptr, nullptr, nullptr, crp, cci, cval, err,
                        only, big, s, list, kern);
}
static unsigned drap_blocks(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }
void amg_drap_full(int nf, int nc, int maxc, const long long* tab, int G, long long ac_total, const int* rp,
                   const int* ci, const double* a, const int* pc, const double* pv, const int* rrp, const int* rci,
                   const double* rv, double* ap, uint8_t* apt, double* ac, uint8_t* acf, int* cnt, hipStream_t s) {
  if (nc <= 0) return;
  if (maxc <= kDrapSmallCols)
    hipLaunchKernelGGL((k_drap_ap<true, kDrapSmallCols>), dim3(drap_blocks(64LL * nf)), dim3(kBlock), 0, s, nf, tab, G,
                       rp, ci, a, pc, pv, ap, apt, (const uint8_t*)nullptr);
  else
    hipLaunchKernelGGL((k_drap_ap<true, kDrapMaxCols>), dim3(drap_blocks(64LL * nf)), dim3(kBlock), 0, s, nf, tab, G,
                       rp, ci, a, pc, pv, ap, apt, (const uint8_t*)nullptr);
  SHP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_drap_ac, dim3(drap_blocks(ac_total)), dim3(kBlock), 0, s, ac_total, tab, G, rrp, rci, rv, ap,
                     apt, ac, acf);
  SHP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_drap_count, dim3(drap_blocks(64LL * nc)), dim3(kBlock), 0, s, nc, tab, G, acf, cnt);
  SHP_LAUNCH_CHECK();
}
void amg_drap_compact(int nc, const long long* tab, int G, const double* ac, const uint8_t* acf, const int* crp,
                      int* cci, double* cval, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_drap_compact, dim3(drap_blocks(64LL * nc)), dim3(kBlock), 0, s, nc, tab, G, ac, acf, crp, cci,
                     cval);
  SHP_LAUNCH_CHECK();
}
void amg_drap_known(int nf, int nc, int maxc, const long long* tab, int G, const int* rp, const int* ci,
                    const double* a, const int* pc, const double* pv, const int* rrp, const int* rci,
                    const double* rv, double* ap, const int* crp, const int* cci, double* cval, hipStream_t s,
                    const uint8_t* only, const uint8_t* only_f) {
  if (nc <= 0) return;
  if (maxc <= kDrapSmallCols)
    hipLaunchKernelGGL((k_drap_ap<false, kDrapSmallCols>), dim3(drap_blocks(64LL * nf)), dim3(kBlock), 0, s, nf, tab,
                       G, rp, ci, a, pc, pv, ap, (uint8_t*)nullptr, only_f);
  else
    hipLaunchKernelGGL((k_drap_ap<false, kDrapMaxCols>), dim3(drap_blocks(64LL * nf)), dim3(kBlock), 0, s, nf, tab,
                       G, rp, ci, a, pc, pv, ap, (uint8_t*)nullptr, only_f);
  SHP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_drap_known, dim3(drap_blocks(64LL * nc)), dim3(kBlock), 0, s, nc, tab, G, rrp, rci, rv, ap,
                     crp, cci, cval, only);
  SHP_LAUNCH_CHECK();
}
void amg_cast(const double* in, float* out, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_cast, dim3(grid_for((int64_t)n)), dim3(kBlock), 0, s, in, out, n);
  SHP_LAUNCH_CHECK();
}
// kernel of the dense coarsest inverses of blocks up to 64 unknowns:
// -1 the FP64 matrix-core sweep, 0 the register Gauss-Jordan kernel
static std::atomic<int> g_dense_mode{-1};
void set_dense_mode(int mode) { g_dense_mode.store(mode); }

void amg_dense_inv(const int* blk, int nblk, const int* rp, const int* ci, const double* a, double* work,
                   double* inv64, float* inv32, int* err, int max_nb, hipStream_t s, const uint8_t* only) {
  if (!nblk) return;
  static_assert(kDenseWave == 96, "register kernel sizes");
  if (max_nb <= 64 && g_dense_mode.load(std::memory_order_relaxed) != 0)
    hipLaunchKernelGGL(k_dense_inv_mfma, dim3(nblk), dim3(256), 0, s, blk, rp, ci, a, inv64, inv32, err, only);
  else if (max_nb <= 64)
    hipLaunchKernelGGL(k_dense_inv_cols, dim3(nblk), dim3(256), 0, s, blk, rp, ci, a, inv64, inv32, err, only);
  else
    hipLaunchKernelGGL((k_dense_inv_reg<96, 128>), dim3(nblk), dim3(128), 0, s, blk, rp, ci, a, inv64, inv32, err,
                       only);
  SHP_LAUNCH_CHECK();
  if (max_nb > kDenseWave) {
    hipLaunchKernelGGL(k_dense_inv, dim3(nblk), dim3(256), 0, s, blk, rp, ci, a, work, inv64, inv32, err);
    SHP_LAUNCH_CHECK();
  }
}

// lanes per row from the average row length of a level
int row_group(double avg_len) { return avg_len <= 10.0 ? 1 : 4; }

#define SHP_GROUP_LAUNCH(K, g, nt, s, ...)                                                              \
  do {                                                                                                 \
    if ((g) == 4) hipLaunchKernelGGL((K<T, 4>), dim3((nt) * 4), dim3(kTileRows), 0, s, __VA_ARGS__);    \
    else if ((g) == 2) hipLaunchKernelGGL((K<T, 2>), dim3((nt) * 2), dim3(kTileRows), 0, s, __VA_ARGS__);    \
    else hipLaunchKernelGGL((K<T, 1>), dim3(nt), dim3(kTileRows), 0, s, __VA_ARGS__);                  \
  } while (0)

#define SHP_GROUP_LAUNCH16(K, g, nt, s, ...)                                                               \
  do {                                                                                                     \
    if ((g) == 4) hipLaunchKernelGGL((K<T, 4, int16_t>), dim3((nt) * 4), dim3(kTileRows), 0, s, __VA_ARGS__); \
    else if ((g) == 2) hipLaunchKernelGGL((K<T, 2, int16_t>), dim3((nt) * 2), dim3(kTileRows), 0, s, __VA_ARGS__); \
    else hipLaunchKernelGGL((K<T, 1, int16_t>), dim3(nt), dim3(kTileRows), 0, s, __VA_ARGS__);            \
  } while (0)

template <class T>
void cyc_smooth(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const T* a,
                const T* dinv, const T* b, const T* xin, T* xout, T omega, int first, int g, hipStream_t s,
                double* sol, const int8_t* cf, int cfphase, const int16_t* ci16) {
  if (!nt) return;
  if (ci16 && !(first == 1 && !cf))
    SHP_GROUP_LAUNCH16(k_smooth, g, nt, s, t, act, rp, ci16, a, dinv, b, xin, xout, omega, first, sol, cf, cfphase);
  else
    SHP_GROUP_LAUNCH(k_smooth, first == 1 && !cf ? 1 : g, nt, s, t, act, rp, ci, a, dinv, b, xin, xout, omega,
                     first, sol, cf, cfphase);
  SHP_LAUNCH_CHECK();
}

// columns as 16-bit offsets from their row (thread per row)
__global__ void k_rel16(const Tile* __restrict__ tiles, const int* __restrict__ rp, const int* __restrict__ ci,
                        int16_t* __restrict__ ci16, int* __restrict__ over) {
  const Tile t = tiles[blockIdx.x];
  const int i = t.r0 + (int)threadIdx.x;
  if (i >= t.r1) return;
  bool bad = false;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int d = ci[e] - i;
    bad |= d < -32768 || d > 32767;
    ci16[e] = (int16_t)d;
  }
  if (bad) *over = 1;
}
void amg_rel16(const Tile* t, int nt, const int* rp, const int* ci, int16_t* ci16, int* over, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_rel16, dim3(nt), dim3(kTileRows), 0, s, t, rp, ci, ci16, over);
  SHP_LAUNCH_CHECK();
}

// l1-Jacobi diagonal: d_i = 1 / sum_j |a_ij| over the rows of the tiles
__global__ void k_l1_diag(const Tile* __restrict__ tiles, const int* __restrict__ rp, const double* __restrict__ a,
                          double* __restrict__ d64, float* __restrict__ d32) {
  const Tile t = tiles[blockIdx.x];
  const int i = t.r0 + threadIdx.x;
  if (i >= t.r1) return;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) s += fabs(a[e]);
  const double di = s != 0.0 ? 1.0 / s : 0.0;
  d64[i] = di;
  if (d32) d32[i] = (float)di;
}
void amg_l1_diag(const Tile* t, int nt, const int* rp, const double* a, double* d64, float* d32, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_l1_diag, dim3(nt), dim3(kTileRows), 0, s, t, rp, a, d64, d32);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_resid(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const T* a, const T* b,
               const T* x, T* r, int g, hipStream_t s, const int16_t* ci16) {
  if (!nt) return;
  if (ci16)
    SHP_GROUP_LAUNCH16(k_resid, g, nt, s, t, act, rp, ci16, a, b, x, r);
  else
    SHP_GROUP_LAUNCH(k_resid, g, nt, s, t, act, rp, ci, a, b, x, r);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_restrict(const Tile* t, int nt, const int* act, const int* rrp, const int* rci, const T* rv,
                  const T* rf, T* bc, int g, hipStream_t s) {
  if (!nt) return;
  SHP_GROUP_LAUNCH(k_restrict, g, nt, s, t, act, rrp, rci, rv, rf, bc);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_prolong(const Tile* t, int nt, const int* act, const int* pc, const T* pv, const T* xc, T* x,
                 hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_prolong<T>, dim3(nt), dim3(kTileRows), 0, s, t, act, pc, pv, xc, x);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_dense(const int* blk, int nblk, const int* act, const T* inv, const T* b, T* x, hipStream_t s) {
  if (!nblk) return;
  hipLaunchKernelGGL(k_dense_solve<T>, dim3(nblk), dim3(256), 0, s, blk, act, inv, b, x);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_resid64(const Tile* t, int nt, const int* act, const int* rp, const int* ci, const double* a,
                 const double* b, const double* x, T* rc, Stripes norm, int g, hipStream_t s) {
  if (!nt) return;
  SHP_GROUP_LAUNCH(k_resid64, g, nt, s, t, act, rp, ci, a, b, x, rc, norm);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_smooth_st(const Tile* t, int nt, const int* act, const StencilView& sv, const T* a, const T* dinv,
                   const T* b, const T* xin, T* xout, T omega, int first, hipStream_t s, double* sol) {
  if (!nt) return;
  hipLaunchKernelGGL(k_smooth_st<T>, dim3(nt), dim3(kTileRows), 0, s, t, act, sv, a, dinv, b, xin, xout, omega,
                     first, sol);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_resid_st(const Tile* t, int nt, const int* act, const StencilView& sv, const T* a, const T* b, const T* x,
                  T* r, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_resid_st<T>, dim3(nt), dim3(kTileRows), 0, s, t, act, sv, a, b, x, r);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_resid64_st(const Tile* t, int nt, const int* act, const StencilView& sv, const double* a, const double* b,
                    const double* x, T* rc, Stripes norm, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_resid64_st<T>, dim3(nt), dim3(kTileRows), 0, s, t, act, sv, a, b, x, rc, norm);
  SHP_LAUNCH_CHECK();
}
template <class T>
void cyc_update64(const Tile* t, int nt, const int* act, const T* e, double* x, hipStream_t s) {
  if (!nt) return;
  hipLaunchKernelGGL(k_update64<T>, dim3(nt), dim3(kTileRows), 0, s, t, act, e, x);
  SHP_LAUNCH_CHECK();
}

template <class T>
void cyc_tail(const int* games, int ngames, int l0, int nlev, int G, const TailLev<T>* lv, const TailGL* gl,
              const int* act, T omega, int nu1, int nu2, int out_y, int lds_rows, hipStream_t s,
              double* sol, const TailRefine* rf) {
  if (ngames <= 0) return;
  const size_t lds = 2 * sizeof(T) * (size_t)std::max(lds_rows, 1);
  TailRefine r{};
  if (rf) r = *rf;
  hipLaunchKernelGGL(k_tail<T>, dim3(ngames), dim3(kTailThreads), lds, s, games, l0, nlev, G, lv, gl, act, omega,
                     nu1, nu2, out_y, sol, r);
  SHP_LAUNCH_CHECK();
}

#define SHP_INST(T)                                                                                  \
  template void cyc_smooth<T>(const Tile*, int, const int*, const int*, const int*, const T*, const T*, \
                              const T*, const T*, T*, T, int, int, hipStream_t, double*,             \
                              const int8_t*, int, const int16_t*);                                   \
  template void cyc_resid<T>(const Tile*, int, const int*, const int*, const int*, const T*, const T*,  \
                             const T*, T*, int, hipStream_t, const int16_t*);                        \
  template void cyc_restrict<T>(const Tile*, int, const int*, const int*, const int*, const T*,        \
                                const T*, T*, int, hipStream_t);                                     \
  template void cyc_prolong<T>(const Tile*, int, const int*, const int*, const T*, const T*, T*,       \
                               hipStream_t);                                                         \
  template void cyc_dense<T>(const int*, int, const int*, const T*, const T*, T*, hipStream_t);        \
  template void cyc_resid64<T>(const Tile*, int, const int*, const int*, const int*, const double*,    \
                               const double*, const double*, T*, Stripes, int, hipStream_t);         \
  template void cyc_update64<T>(const Tile*, int, const int*, const T*, double*, hipStream_t);          \
  template void cyc_smooth_st<T>(const Tile*, int, const int*, const StencilView&, const T*, const T*,  \
                                 const T*, const T*, T*, T, int, hipStream_t, double*);              \
  template void cyc_resid_st<T>(const Tile*, int, const int*, const StencilView&, const T*, const T*,   \
                                const T*, T*, hipStream_t);                                          \
  template void cyc_resid64_st<T>(const Tile*, int, const int*, const StencilView&, const double*,     \
                                  const double*, const double*, T*, Stripes, hipStream_t);           \
  template void cyc_tail<T>(const int*, int, int, int, int, const TailLev<T>*, const TailGL*, const int*, T, int, \
                            int, int, int, hipStream_t, double*, const TailRefine*);
SHP_INST(float)
SHP_INST(double)
#undef SHP_INST

}  // namespace shp
