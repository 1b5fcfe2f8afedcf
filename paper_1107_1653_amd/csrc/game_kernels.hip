// Game-level kernels: level-0 pattern, policy-system assembly, policy
// improvement with the Shapley residual, policy updates and FAMGpi transfers.
// All of them walk a work-list of (game, state range) tiles so that one launch
// serves every game of a batch.
#include "internal.hpp"

#include <algorithm>
#include <climits>

namespace shp {

// ---------------------------------------------------------------------------
// level-0 pattern of a game: per state the union of the columns of its
// m1*m2 rows plus the diagonal, sorted.  The rows of state x are contiguous,
// so the union is found by repeated selection of the next larger column.
// ---------------------------------------------------------------------------
__global__ void k_union(const int* __restrict__ rp, const int* __restrict__ ci, int n, int K,
                        const int* __restrict__ urp, int* __restrict__ uci, int* __restrict__ cnt) {
  int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  int e0 = rp[(int64_t)x * K], e1 = rp[(int64_t)(x + 1) * K];
  int last = -1, c = 0;
  int base = uci ? urp[x] : 0;
  while (true) {
    int nxt = INT_MAX;
    if (x > last) nxt = x;
    for (int e = e0; e < e1; ++e) {
      int col = ci[e];
      if (col > last && col < nxt) nxt = col;
    }
    if (nxt == INT_MAX) break;
    if (uci) uci[base + c] = nxt;
    ++c;
    last = nxt;
  }
  if (!uci) cnt[x] = c;
}

void launch_union_count(const int* rp, const int* ci, int n, int m1, int m2, int* cnt, int* err,
                        hipStream_t s) {
  (void)err;
  if (n == 0) return;
  hipLaunchKernelGGL(k_union, dim3(grid_for(n)), dim3(kBlock), 0, s, rp, ci, n, m1 * m2,
                     (const int*)nullptr, (int*)nullptr, cnt);
  SHP_LAUNCH_CHECK();
}

void launch_union_fill(const int* rp, const int* ci, int n, int m1, int m2, const int* urp, int* uci,
                       hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_union, dim3(grid_for(n)), dim3(kBlock), 0, s, rp, ci, n, m1 * m2, urp, uci,
                     (int*)nullptr);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// merged level-0 layout: row pointer and columns of the block-diagonal matrix
// ---------------------------------------------------------------------------
__global__ void k_layout(const GameDesc* __restrict__ gd, const GTile* __restrict__ tiles,
                         int* __restrict__ rp0, int* __restrict__ ci0, int N0, int NNZ0) {
  GTile t = tiles[blockIdx.x];
  const GameDesc d = gd[t.game];
  for (int x = t.s0 + threadIdx.x; x < t.s1; x += blockDim.x) {
    int u0 = d.urp[x], u1 = d.urp[x + 1];
    rp0[d.x_off + x] = d.a_off + u0;
    for (int j = u0; j < u1; ++j) ci0[d.a_off + j] = d.x_off + d.uci[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rp0[N0] = NNZ0;
}

void launch_layout(const GameDesc* d, const GTile* t, int nt, int* rp0, int* ci0, int N0, int NNZ0,
                   hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_layout, dim3(nt), dim3(kBlock), 0, s, d, t, rp0, ci0, N0, NNZ0);
  SHP_LAUNCH_CHECK();
}

__global__ void k_gather_v(const GameDesc* __restrict__ gd, const GTile* __restrict__ tiles,
                           const int* __restrict__ active, double* __restrict__ x0) {
  GTile t = tiles[blockIdx.x];
  if (active && !active[t.game]) return;
  const GameDesc d = gd[t.game];
  for (int x = t.s0 + threadIdx.x; x < t.s1; x += blockDim.x) x0[d.x_off + x] = d.v[x];
}

__global__ void k_scatter_v(const GameDesc* __restrict__ gd, const GTile* __restrict__ tiles,
                            const int* __restrict__ active, const double* __restrict__ x0) {
  GTile t = tiles[blockIdx.x];
  if (active && !active[t.game]) return;
  const GameDesc d = gd[t.game];
  for (int x = t.s0 + threadIdx.x; x < t.s1; x += blockDim.x) d.v[x] = x0[d.x_off + x];
}

void launch_gather_v(const GameDesc* d, const GTile* t, int nt, const int* active, double* x0,
                     hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_gather_v, dim3(nt), dim3(kBlock), 0, s, d, t, active, x0);
  SHP_LAUNCH_CHECK();
}

void launch_scatter_v(const GameDesc* d, const GTile* t, int nt, const int* active, const double* x0,
                      hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_scatter_v, dim3(nt), dim3(kBlock), 0, s, d, t, active, x0);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Policy-system assembly.  Row x of A = I - mu M^{alpha beta} and
// b = r^{alpha beta} (Sec. 4.2, eq. (LSPI)), written into the fixed level-0
// pattern of the game (explicit zeros where the chosen row has no entry).
// A row is rebuilt only when its pair (alpha(x), beta(x)) differs from the
// one it was last built for (`pol`, -1: never built); 1/a_ii of the built
// row is kept in `dbuilt` and copied to the relaxation diagonal of every row,
// which the AMG setup rescales on Dirichlet rows.
// ---------------------------------------------------------------------------
__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline int warp_sum_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

constexpr int kAsmRow = 8;  // pattern rows built in registers

__global__ __launch_bounds__(256) void k_assemble(const GameDesc* __restrict__ gd,
                                                  const GTile* __restrict__ tiles,
                                                  const int* __restrict__ active,
                                                  double* __restrict__ a64, float* __restrict__ a32,
                                                  double* __restrict__ b0, double* __restrict__ dinv64,
                                                  float* __restrict__ dinv32, int* __restrict__ pol,
                                                  double* __restrict__ dbuilt, double* __restrict__ st64,
                                                  float* __restrict__ st32, int st_w, int N, Stripes bnorm) {
  GTile t = tiles[blockIdx.x];
  if (!active[t.game]) return;
  const GameDesc d = gd[t.game];
  double bmax = 0.0;
  int x = t.s0 + threadIdx.x;
  const int X = d.x_off + x;
  const int q = x < t.s1 ? d.alpha[x] * d.m2 + d.beta[x] : -1;
  if (x < t.s1 && q >= 0 && pol[X] == q) {
    // the row already holds this pair's coefficients
    const double rb = b0[X];
    const double di = dbuilt[X];
    dinv64[X] = di;
    if (dinv32) dinv32[X] = (float)di;
    bmax = rb == rb ? fabs(rb) : INFINITY;
  } else if (x < t.s1) {
    const int s = x * d.m1 * d.m2 + q;
    const int e0 = d.rp[s], e1 = d.rp[s + 1];
    const int j0 = d.urp[x], j1 = d.urp[x + 1];
    // the identity row on the level-0 pattern, then each entry of the chosen
    // row subtracted at its column, in row order (the pattern row is sorted
    // and holds every column of the state's rows)
    double diag = 0.0;
    if (j1 - j0 <= kAsmRow) {
      // short pattern rows (grid stencils): the row is built in registers
      // and written once
      int col[kAsmRow];
      double val[kAsmRow];
#pragma unroll
      for (int k = 0; k < kAsmRow; ++k) {
        col[k] = j0 + k < j1 ? d.uci[j0 + k] : -1;
        val[k] = col[k] == x ? 1.0 : 0.0;
      }
      for (int e = e0; e < e1; ++e) {
        const int c = d.ci[e];
        const double mw = d.mu * d.w[e];
#pragma unroll
        for (int k = 0; k < kAsmRow; ++k)
          if (col[k] == c) val[k] -= mw;
      }
#pragma unroll
      for (int k = 0; k < kAsmRow; ++k) {
        if (j0 + k >= j1) break;
        a64[d.a_off + j0 + k] = val[k];
        if (a32) a32[d.a_off + j0 + k] = (float)val[k];
        if (col[k] == x) diag = val[k];
      }
      if (st64) {
        // the stencil form: slot k = entry k of the row, zero past its end
#pragma unroll
        for (int k = 0; k < kAsmRow; ++k) {
          if (k >= st_w) break;
          const double vk = j0 + k < j1 ? val[k] : 0.0;
          st64[(size_t)k * N + X] = vk;
          if (st32) st32[(size_t)k * N + X] = (float)vk;
        }
      }
    } else {
      int jd = j0;
      for (int j = j0; j < j1; ++j) {
        const int c = d.uci[j];
        a64[d.a_off + j] = c == x ? 1.0 : 0.0;
        if (c == x) jd = j;
      }
      for (int e = e0; e < e1; ++e) {  // column by bisection
        const int c = d.ci[e];
        int lo = j0, hi = j1 - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (d.uci[mid] < c) lo = mid + 1; else hi = mid;
        }
        a64[d.a_off + lo] -= d.mu * d.w[e];
      }
      diag = a64[d.a_off + jd];
      if (a32)
        for (int j = j0; j < j1; ++j) a32[d.a_off + j] = (float)a64[d.a_off + j];
    }
    const double rb = d.r[s];
    b0[X] = rb;
    const double di = diag != 0.0 ? 1.0 / diag : 0.0;
    dinv64[X] = di;
    if (dinv32) dinv32[X] = (float)di;
    dbuilt[X] = di;
    pol[X] = q;
    bmax = rb == rb ? fabs(rb) : INFINITY;
  }
  bmax = warp_max(bmax);
  block_fold<1, 0>(bnorm, t.game, &bmax, 0u, nullptr);
}

void launch_assemble(const GameDesc* d, const GTile* t, int nt, const int* active, double* a64, float* a32,
                     double* b0, double* dinv64, float* dinv32, int* pol, double* dbuilt, double* st64,
                     float* st32, int st_w, int N, Stripes bnorm, hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_assemble, dim3(nt), dim3(kBlock), 0, s, d, t, active, a64, a32, b0, dinv64,
                     dinv32, pol, dbuilt, st64, st32, st_w, N, bnorm);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Level-0 patterns as stencils.  A pattern whose entries take at most
// kStencilMax distinct offsets col - x, in rows of at most kStencilMax
// entries (grid games), is stored for the cycle kernels by slot: entry t of
// every row in one array (coalesced over rows), its column from a 3-bit code.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stencil_scan(const int* __restrict__ urp, const int* __restrict__ uci,
                                                      int n, int* __restrict__ out) {
  // the workgroup's distinct offsets in LDS, merged into the global table at the end
  __shared__ int tab[kStencilHash];
  __shared__ int s_over, s_len;
  if (threadIdx.x < kStencilHash) tab[threadIdx.x] = INT_MIN;
  if (threadIdx.x == 0) { s_over = 0; s_len = 0; }
  __syncthreads();
  int len = 0;
  bool over = false;
  for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
    const int j0 = urp[x], j1 = urp[x + 1];
    len = max(len, j1 - j0);
    for (int j = j0; j < j1; ++j) {
      const int o = uci[j] - x;
      unsigned h = mix32((uint32_t)o) & (kStencilHash - 1);
      bool done = false;
      for (int p = 0; p < kStencilHash && !done; ++p) {
        const int old = atomicCAS(&tab[h], INT_MIN, o);
        done = old == INT_MIN || old == o;
        h = (h + 1) & (kStencilHash - 1);
      }
      over |= !done;
    }
  }
  if (over) s_over = 1;
  atomicMax(&s_len, len);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_over) out[0] = 1;
    atomicMax(&out[1], s_len);
  }
  if (threadIdx.x < kStencilHash) {
    const int o = tab[threadIdx.x];
    if (o != INT_MIN) {
      int* g = out + 2;
      unsigned h = mix32((uint32_t)o) & (kStencilHash - 1);
      bool done = false;
      for (int p = 0; p < kStencilHash && !done; ++p) {
        const int old = atomicCAS(&g[h], INT_MIN, o);
        done = old == INT_MIN || old == o;
        h = (h + 1) & (kStencilHash - 1);
      }
      if (!done) out[0] = 1;
    }
  }
}

__global__ void k_stencil_clear(int* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < 2) out[i] = 0;
  if (i < kStencilHash) out[2 + i] = INT_MIN;
}

void launch_stencil_scan(const int* urp, const int* uci, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stencil_clear, dim3(1), dim3(64), 0, s, out);
  SHP_LAUNCH_CHECK();
  if (n == 0) return;
  hipLaunchKernelGGL(k_stencil_scan, dim3(std::min<unsigned>(grid_for(n), 1024u)), dim3(kBlock), 0, s, urp, uci, n, out);
  SHP_LAUNCH_CHECK();
}

__global__ void k_stencil_codes(const GameDesc* __restrict__ gd, const GTile* __restrict__ tiles,
                                const int* __restrict__ off, uint32_t* __restrict__ code) {
  const GTile t = tiles[blockIdx.x];
  const GameDesc d = gd[t.game];
  const int x = t.s0 + (int)threadIdx.x;
  if (x >= t.s1) return;
  const int* o = off + kStencilMax * t.game;
  int zero = 0;  // the code of offset 0 (the diagonal), for the slots past the row's end
  for (int c = 0; c < kStencilMax; ++c)
    if (o[c] == 0) zero = c;
  const int j0 = d.urp[x], j1 = d.urp[x + 1];
  uint32_t w = (uint32_t)(j1 - j0) << 24;
  for (int k = 0; k < kStencilMax; ++k) {
    int c = zero;
    if (j0 + k < j1) {
      const int dlt = d.uci[j0 + k] - x;
      for (int q = 0; q < kStencilMax; ++q)
        if (o[q] == dlt) c = q;
    }
    w |= (uint32_t)c << (3 * k);
  }
  code[d.x_off + x] = w;
}

void launch_stencil_codes(const GameDesc* d, const GTile* t, int nt, const int* off, uint32_t* code,
                          hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_stencil_codes, dim3(nt), dim3(kBlock), 0, s, d, t, off, code);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Policy improvement and Shapley residual in one sweep.
//   Q(x,a,b) = r(x,a,b) + mu sum_y w(y|x,a,b) v(y)   (the bracket of eq. (eq1))
//   beta_in(x)  : MIN's improvement at alpha(x)       (Algorithm algo-MDP, step 2)
//   F(x)        : max_a min_b Q                        (eq. (eq1))
//   alpha_c(x)  : MAX's improvement                    (Algorithm PIalgo, step 2)
//   beta_c(x)   : MIN's answer at alpha_c(x)
// Ties: the incumbent is kept unless another action is better by more than
// tie_rtol times the rounding scale |r| + mu sum |w v| of the compared rows;
// otherwise the lowest index attaining the extremum is taken.
// The products w v of the tile's entries (contiguous in the CSR) are formed
// with coalesced loads, kImpStage at a time, into LDS; one thread per row then
// adds its row's products in entry order into Q; one thread per (state, a)
// takes MIN over b, one thread per state MAX over a and the decisions.
// ---------------------------------------------------------------------------
constexpr int kImpUnroll = 5;  // entries staged per thread and stage: a tile of 2-D grid states (9 rows of 5
                               // entries each) in one stage

// One tile of states (at most NT rows, a thread per row): either taken from
// the work list (FLAT = false: the tile's game descriptor is read from gd),
// or, for a single game passed by value, the states
// [blockIdx.x * spb, (blockIdx.x + 1) * spb).
template <bool FLAT, int NT>
__global__ __launch_bounds__(NT) void k_improve(const GameDesc* __restrict__ gd,
                                                const GTile* __restrict__ tiles,
                                                const int* __restrict__ active, double tie_rtol,
                                                Stripes red, GameDesc d1, int spb) {
  constexpr int kImpStage = NT * kImpUnroll;
  __shared__ double sq[NT];
  __shared__ double ss[NT];
  __shared__ unsigned char sv[NT];
  __shared__ double s_mn[NT], s_sc[NT];  // per (state, a): MIN's minimum over b and its scale
  __shared__ int s_lb[NT];               // and its lowest b
  __shared__ double sp[kImpStage];
  GTile t;
  GameDesc d;
  if (FLAT) {
    d = d1;
    t.game = 0;
    t.s0 = blockIdx.x * spb;
    t.s1 = t.s0 + spb < d1.n ? t.s0 + spb : d1.n;
  } else {
    t = tiles[blockIdx.x];
    if (active && !active[t.game]) return;
    d = gd[t.game];
  }
  const int K = d.m1 * d.m2;
  const int ns = t.s1 - t.s0;
  const int tid = threadIdx.x;
  const int row0 = t.s0 * K;  // the tile's rows: row0 + [0, ns K)
  const bool mine = tid < ns * K;
  const int row = row0 + tid;
  const int e0 = mine ? d.rp[row] : 0, e1 = mine ? d.rp[row + 1] : 0;
  // the tile's entry range: stored in the tile (one dependent load less)
  const int eb = FLAT ? d.rp[row0] : t.e0, ee = FLAT ? d.rp[row0 + ns * K] : t.e1;
  // loads that do not depend on the products, issued before the stages
  const double rr = mine ? d.r[row] : 0.0;
  const bool ok = mine && (d.valid ? (d.valid[row] != 0) : true);
  const bool owner = tid < ns;
  const int al = owner && d.alpha ? d.alpha[t.s0 + tid] : -1;  // no incumbents: the greedy choice
  const int be = owner && d.beta ? d.beta[t.s0 + tid] : -1;
  const double vx = owner ? d.v[t.s0 + tid] : 0.0;
  double acc = 0.0, sacc = 0.0;
  for (int c0 = eb; c0 < ee; c0 += kImpStage) {
    const int c1 = ee < c0 + kImpStage ? ee : c0 + kImpStage;
    // the stage's columns and weights first (all loads in flight), then the
    // values they gather, then the products into LDS
    int cc[kImpUnroll];
    double ww[kImpUnroll], vv[kImpUnroll];
#pragma unroll
    for (int u = 0; u < kImpUnroll; ++u) {
      const int e = c0 + tid + NT * u;
      cc[u] = e < c1 ? d.ci[e] : 0;
      ww[u] = e < c1 ? d.w[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kImpUnroll; ++u) vv[u] = c0 + tid + NT * u < c1 ? d.v[cc[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < kImpUnroll; ++u)
      if (c0 + tid + NT * u < c1) sp[tid + NT * u] = ww[u] * vv[u];
    __syncthreads();
    const int lo = e0 > c0 ? e0 : c0, hi = e1 < c1 ? e1 : c1;
    for (int e = lo; e < hi; ++e) {
      const double p = sp[e - c0];
      acc += p;
      sacc += fabs(p);
    }
    __syncthreads();
  }
  if (mine) {
    sq[tid] = rr + d.mu * acc;
    ss[tid] = fabs(rr) + d.mu * sacc;
    sv[tid] = ok ? 1 : 0;
  }
  __syncthreads();
  // MIN over b for every (state, a) in parallel: the minimum, its lowest b
  // and the rounding scale of the rows compared (one thread per pair)
  if (tid < ns * d.m1) {
    const int qb = tid * d.m2;  // rows of the pair: state tid / m1, action tid % m1
    double mn = INFINITY, sc = 0.0;
    int low = -1;
    for (int b = 0; b < d.m2; ++b) {
      if (!sv[qb + b]) continue;
      if (sq[qb + b] < mn) { mn = sq[qb + b]; low = b; }
      sc = fmax(sc, ss[qb + b]);
    }
    s_mn[tid] = mn;
    s_sc[tid] = sc;
    s_lb[tid] = low;
  }
  __syncthreads();
  double res = 0.0, res2 = 0.0;
  int chg_in = 0, chg_out = 0, hash_out = 0;
  if (owner) {
    const int x = t.s0 + tid;
    const int base = tid * K;
    const int pb = tid * d.m1;  // the state's pairs
    // MIN at the incumbent alpha
    int bin = -1;
    if (al >= 0) {
      const double mn = s_mn[pb + al], sc = s_sc[pb + al];
      bin = s_lb[pb + al];
      if (be >= 0 && be < d.m2 && sv[base + al * d.m2 + be] &&
          sq[base + al * d.m2 + be] <= mn + tie_rtol * sc)
        bin = be;
    }
    // MAX over a of min over b
    double F = -INFINITY, scall = 0.0;
    int lowa = -1;
    double inner_al = -INFINITY;
    for (int a = 0; a < d.m1; ++a) {
      const double mn = s_mn[pb + a];
      scall = fmax(scall, s_sc[pb + a]);
      if (mn == INFINITY) continue;  // no valid b: action a not available
      if (a == al) inner_al = mn;
      if (mn > F) { F = mn; lowa = a; }
    }
    int ac = lowa;
    if (al >= 0 && inner_al >= F - tie_rtol * scall) ac = al;
    // an incumbent alpha with no valid b (never produced by the library: warm
    // starts and transfers are checked) is not kept
    const bool al_ok = al >= 0 && inner_al > -INFINITY;
    // MIN's answer at the new alpha (keep the incumbent if alpha is unchanged)
    int bc = -1;
    if (ac >= 0) {
      const double mn = s_mn[pb + ac], sc = s_sc[pb + ac];
      bc = s_lb[pb + ac];
      if (ac == al && be >= 0 && be < d.m2 && sv[base + ac * d.m2 + be] &&
          sq[base + ac * d.m2 + be] <= mn + tie_rtol * sc)
        bc = be;
    }
    if (!al_ok) bin = bc;  // never -1: MIN's answer at MAX's improvement
    if (d.beta_in) d.beta_in[x] = bin;
    d.alpha_c[x] = ac;
    d.beta_c[x] = bc;
    if (d.F) d.F[x] = F;  // stored only when asked for
    double dv = F - vx;
    res = dv == dv ? fabs(dv) : INFINITY;
    res2 = dv * dv;
    chg_in = (bin != be) ? 1 : 0;
    chg_out = (ac != al || (al >= 0 && !al_ok)) ? 1 : 0;
    // a hash of MAX's improved strategy: the wrapping sum over states of a
    // mix of (state, action), independent of the summation order
    hash_out = (int)mix32((uint32_t)x * 0x9E3779B9u ^ (uint32_t)(ac + 1));
  }
  // per-game max |F(v) - v|, sum (F(v) - v)^2, change counts, strategy hash
  const double vd[2] = {warp_max(res), warp_sum(res2)};
  const int vi[3] = {warp_sum_i(chg_in), warp_sum_i(chg_out), warp_sum_i(hash_out)};
  block_fold<2, 3>(red, t.game, vd, 2u, vi);
}

void launch_improve(const GameDesc* d, const GTile* t, int nt, const int* active, double tie_rtol,
                    Stripes red, int threads, hipStream_t s) {
  if (nt == 0) return;
  if (threads == 64)
    hipLaunchKernelGGL((k_improve<false, 64>), dim3(nt), dim3(64), 0, s, d, t, active, tie_rtol, red, GameDesc{}, 0);
  else if (threads == 128)
    hipLaunchKernelGGL((k_improve<false, 128>), dim3(nt), dim3(128), 0, s, d, t, active, tie_rtol, red, GameDesc{},
                       0);
  else
    hipLaunchKernelGGL((k_improve<false, 256>), dim3(nt), dim3(256), 0, s, d, t, active, tie_rtol, red, GameDesc{},
                       0);
  SHP_LAUNCH_CHECK();
}

// threads of the improvement workgroups: the smallest of 64, 128, 256 that
// holds a state's rows and is at least `want`
int improve_threads(int max_rows_per_state, int want) {
  int t = want == 64 || want == 128 ? want : 256;
  while (t < 256 && t < max_rows_per_state) t *= 2;
  return t;
}

__global__ void k_tile_entries(const GameDesc* __restrict__ gd, GTile* __restrict__ tiles, int nt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  GTile t = tiles[k];
  const GameDesc& d = gd[t.game];
  const int K = d.m1 * d.m2;
  t.e0 = d.rp[(size_t)t.s0 * K];
  t.e1 = d.rp[(size_t)t.s1 * K];
  tiles[k] = t;
}

void launch_tile_entries(const GameDesc* d, GTile* t, int nt, hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_tile_entries, dim3(grid_for(nt)), dim3(kBlock), 0, s, d, t, nt);
  SHP_LAUNCH_CHECK();
}

// states per improvement tile: whole states, at most `threads` rows
int improve_states_per_tile(int m1, int m2, int threads) { return std::max(1, threads / (m1 * m2)); }

void launch_improve_flat(const GameDesc& d, double tie_rtol, Stripes red, hipStream_t s) {
  if (d.n == 0) return;
  const int spb = improve_states_per_tile(d.m1, d.m2, kBlock);
  hipLaunchKernelGGL((k_improve<true, 256>), dim3((d.n + spb - 1) / spb), dim3(kBlock), 0, s,
                     (const GameDesc*)nullptr, (const GTile*)nullptr, (const int*)nullptr, tie_rtol, red, d, spb);
  SHP_LAUNCH_CHECK();
}

// Combines the stripes of every game (nd double quantities, bit q of
// sum_mask = sum else max; ni int sums), writes out_d[g * sd + q] and
// out_i[g * si + q], and clears the stripes.
__global__ void k_fold_finish(Stripes st, int G, int nd, unsigned sum_mask, int ni, double* __restrict__ out_d,
                              int sd, int* __restrict__ out_i, int si) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = t >> 2, q = t & 3;
  if (g >= G) return;
  if (q < nd) {
    const bool sum = (sum_mask >> q) & 1u;
    double v = 0.0;
#pragma unroll 16
    for (int k = 0; k < kStripes; ++k) {
      double* a = st.d + stripe_at(st, k, g, q);
      const double x = *a;
      *a = 0.0;
      v = sum ? v + x : fmax(v, x);
    }
    out_d[(size_t)g * sd + q] = v;
  }
  if (q < ni) {
    int v = 0;
#pragma unroll 16
    for (int k = 0; k < kStripes; ++k) {
      int* a = st.i + stripe_at(st, k, g, q);
      v += *a;
      *a = 0;
    }
    out_i[(size_t)g * si + q] = v;
  }
}

// stop test of the refinement loop, one thread per game (same rule as a host
// check after every cycle: ||r||_inf <= max(rtol max(||b||, ||x||), atol),
// loosened to forcing x previous Shapley residual; stagnation; cycle limit)
__global__ void k_lin_check(Stripes st, int G, const double* __restrict__ bnorm, LinCtl* __restrict__ ctl,
                            int* __restrict__ act, double* __restrict__ norm) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) lin_check_game(st, g, bnorm, ctl, act, norm);
}

void launch_lin_check(Stripes st, int G, const double* bnorm, LinCtl* ctl, int* lin_active, double* norm,
                      hipStream_t s) {
  if (G <= 0) return;
  hipLaunchKernelGGL(k_lin_check, dim3(grid_for(G)), dim3(kBlock), 0, s, st, G, bnorm, ctl, lin_active, norm);
  SHP_LAUNCH_CHECK();
}

void launch_fold_finish(Stripes st, int G, int nd, unsigned sum_mask, int ni, double* out_d, int sd, int* out_i,
                        int si, hipStream_t s) {
  if (G <= 0) return;
  hipLaunchKernelGGL(k_fold_finish, dim3(grid_for(4 * (int64_t)G)), dim3(kBlock), 0, s, st, G, nd, sum_mask, ni,
                     out_d, sd, out_i, si);
  SHP_LAUNCH_CHECK();
}

// decision codes: 1 = take beta_in (inner step), 2 = take (alpha_c, beta_c) (outer step)
__global__ void k_apply(const GameDesc* __restrict__ gd, const GTile* __restrict__ tiles,
                        const int* __restrict__ decision) {
  GTile t = tiles[blockIdx.x];
  int code = decision[t.game];
  if (code == 0) return;
  const GameDesc d = gd[t.game];
  for (int x = t.s0 + threadIdx.x; x < t.s1; x += blockDim.x) {
    if (code == 1) {
      d.beta[x] = d.beta_in[x];
    } else {
      d.alpha[x] = d.alpha_c[x];
      d.beta[x] = d.beta_c[x];
    }
  }
}

void launch_apply(const GameDesc* d, const GTile* t, int nt, const int* decision, hipStream_t s) {
  if (nt == 0) return;
  hipLaunchKernelGGL(k_apply, dim3(nt), dim3(kBlock), 0, s, d, t, decision);
  SHP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// FAMGpi transfers (Sec. 5.2).  Value interpolation I: multilinear on the
// coarse grid extended by its Dirichlet nodes (on nested dyadic grids this is
// the paper's average of the coarse neighbours within distance h_l).
// Strategy interpolation U: copy the coarse node at floor(i (s_c+1)/(s_f+1))
// clamped to [1, s_c] on every axis.
// ---------------------------------------------------------------------------
__global__ void k_fmg(int dim, int sc, int sf, const double* __restrict__ vc,
                      const int* __restrict__ ac, const int* __restrict__ bc,
                      const double* __restrict__ bvals, double* __restrict__ vf,
                      int* __restrict__ af, int* __restrict__ bf, int nf,
                      const uint8_t* __restrict__ valid_f, int m1, int m2) {
  int xf = blockIdx.x * blockDim.x + threadIdx.x;
  if (xf >= nf) return;
  int kk[3] = {0, 0, 0};
  double tt[3] = {0.0, 0.0, 0.0};
  int rem = xf;
  const int64_t den = sf + 1;
  for (int ax = 0; ax < dim; ++ax) {
    int i = rem % sf + 1;
    rem /= sf;
    int64_t num = (int64_t)i * (sc + 1);
    int64_t k = num / den;
    kk[ax] = (int)k;
    tt[ax] = (double)(num - k * den) / (double)den;
  }
  const int se = sc + 2;
  double acc = 0.0;
  for (int corner = 0; corner < (1 << dim); ++corner) {
    double wgt = 1.0;
    int ext = 0, lin = 0, stride_e = 1, stride_i = 1;
    bool inner = true;
    for (int ax = 0; ax < dim; ++ax) {
      int hi = (corner >> ax) & 1;
      int c = kk[ax] + hi;
      if (c > sc + 1) c = sc + 1;
      wgt *= hi ? tt[ax] : (1.0 - tt[ax]);
      ext += c * stride_e;
      stride_e *= se;
      if (c < 1 || c > sc) inner = false;
      lin += (c - 1) * stride_i;
      stride_i *= sc;
    }
    if (wgt == 0.0) continue;
    double val = inner ? vc[lin] : (bvals ? bvals[ext] : 0.0);
    acc += wgt * val;
  }
  vf[xf] = acc;
  int lin = 0, stride = 1;
  for (int ax = 0; ax < dim; ++ax) {
    int c = kk[ax];
    if (c < 1) c = 1;
    if (c > sc) c = sc;
    lin += (c - 1) * stride;
    stride *= sc;
  }
  int a = ac[lin], b = bc[lin];
  if (valid_f) {
    // the fine game may mask the copied pair: take MIN's lowest valid action
    // at the copied a, else the lowest valid pair (every state has one)
    const uint8_t* vx = valid_f + (int64_t)xf * m1 * m2;
    if (a < 0 || a >= m1 || b < 0 || b >= m2 || !vx[a * m2 + b]) {
      int nb = -1;
      if (a >= 0 && a < m1)
        for (int q = 0; q < m2 && nb < 0; ++q)
          if (vx[a * m2 + q]) nb = q;
      if (nb >= 0) {
        b = nb;
      } else {
        for (int q = 0; q < m1 * m2; ++q)
          if (vx[q]) { a = q / m2; b = q % m2; break; }
      }
    }
  }
  af[xf] = a;
  bf[xf] = b;
}

void launch_fmg(const Game* c, const Game* f, hipStream_t s) {
  if (f->n == 0) return;
  hipLaunchKernelGGL(k_fmg, dim3(grid_for(f->n)), dim3(kBlock), 0, s, c->dim, c->s, f->s, c->v.p,
                     c->alpha.p, c->beta.p, c->has_bvals ? c->bvals.p : (const double*)nullptr,
                     f->v.p, f->alpha.p, f->beta.p, f->n, f->valid.p, f->m1, f->m2);
  SHP_LAUNCH_CHECK();
}

void fmg_transfer(Game* coarse, Game* fine, hipStream_t s) { launch_fmg(coarse, fine, s); }

// ---------------------------------------------------------------------------
// Checks of a game handed over in device memory: the conditions the create
// call states for host arrays, evaluated per row (row pointer monotone and
// within the entries, columns in [0, n), weights finite and >= 0, row sum
// <= 1 + 1e-12 summed in entry order, finite reward), per state (a valid
// pair), and a flag for rows whose columns are not ascending.
// ---------------------------------------------------------------------------
__global__ void k_check_game(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                             const double* __restrict__ w, const double* __restrict__ r, int nrows, int n,
                             int64_t nnz, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  int bits = 0;
  const int64_t e0 = rp[i], e1 = rp[i + 1];
  if (i == 0 && e0 != 0) bits |= kChkRp0;
  if (e0 < 0 || e1 < e0 || e1 > nnz) {
    bits |= kChkRp;
  } else {
    double sum = 0.0;
    int last = INT_MIN;
    for (int64_t e = e0; e < e1; ++e) {
      const int c = ci[e];
      const double x = w[e];
      if (c < 0 || c >= n) bits |= kChkCol;
      if (!(x >= 0.0 && x <= 1.7976931348623157e308)) bits |= kChkW;
      if (c < last) bits |= kChkUnsorted;
      last = c;
      sum += x;
    }
    if (!(sum <= 1.0 + 1e-12) && !(bits & kChkW)) bits |= kChkSum;
  }
  const double ri = r[i];
  if (!(ri - ri == 0.0)) bits |= kChkR;
  if (bits) atomicOr(err, bits);
}

__global__ void k_check_valid(const uint8_t* __restrict__ valid, int n, int K, int* __restrict__ err) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  bool any = false;
  for (int q = 0; q < K; ++q) any |= valid[(int64_t)x * K + q] != 0;
  if (!any) atomicOr(err, kChkEmpty);
}

__global__ void k_rp_narrow(const int64_t* __restrict__ in, int* __restrict__ out, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = (int)in[i];
}

// stable insertion sort of each row's (column, weight) pairs, one thread per row
__global__ void k_sort_pairs(const int* __restrict__ rp, int* __restrict__ ci, double* __restrict__ w,
                             int nrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int e0 = rp[i], e1 = rp[i + 1];
  for (int e = e0 + 1; e < e1; ++e) {
    const int c = ci[e];
    const double x = w[e];
    int f = e - 1;
    while (f >= e0 && ci[f] > c) {
      ci[f + 1] = ci[f];
      w[f + 1] = w[f];
      --f;
    }
    ci[f + 1] = c;
    w[f + 1] = x;
  }
}

// warm-start strategies against the game: bit 1 = alpha out of range or with
// no valid b (the action is not available), bit 2 = beta out of range or the
// pair (alpha, beta) not valid
__global__ void k_check_policy(const int* __restrict__ alpha, const int* __restrict__ beta,
                               const uint8_t* __restrict__ valid, int n, int m1, int m2, int* __restrict__ err) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int a = alpha[x];
  int bits = 0;
  if (a < 0 || a >= m1) {
    bits |= 1;
  } else if (valid) {
    bool any = false;
    for (int b = 0; b < m2; ++b) any |= valid[((int64_t)x * m1 + a) * m2 + b] != 0;
    if (!any) bits |= 1;
  }
  if (beta && !(bits & 1)) {
    const int b = beta[x];
    if (b < 0 || b >= m2 || (valid && !valid[((int64_t)x * m1 + a) * m2 + b])) bits |= 2;
  }
  if (bits) atomicOr(err, bits);
}

int check_game_device(const int64_t* rp, const int32_t* ci, const double* w, const double* r,
                      const uint8_t* valid, int n, int K, int64_t nnz, int* err_dev, hipStream_t s) {
  const int nrows = n * K;
  fill_async(err_dev, 0, 1, s);
  hipLaunchKernelGGL(k_check_game, dim3(grid_for(nrows)), dim3(kBlock), 0, s, rp, ci, w, r, nrows, n, nnz,
                     err_dev);
  SHP_LAUNCH_CHECK();
  if (valid) {
    hipLaunchKernelGGL(k_check_valid, dim3(grid_for(n)), dim3(kBlock), 0, s, valid, n, K, err_dev);
    SHP_LAUNCH_CHECK();
  }
  int bits = 0;
  d2h(&bits, err_dev, 1, s);
  SHP_HIP(hipStreamSynchronize(s));
  return bits;
}

void launch_rp_narrow(const int64_t* in, int* out, int m, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_rp_narrow, dim3(grid_for(m)), dim3(kBlock), 0, s, in, out, m);
  SHP_LAUNCH_CHECK();
}

void launch_sort_pairs(const int* rp, int* ci, double* w, int nrows, hipStream_t s) {
  if (nrows <= 0) return;
  hipLaunchKernelGGL(k_sort_pairs, dim3(grid_for(nrows)), dim3(kBlock), 0, s, rp, ci, w, nrows);
  SHP_LAUNCH_CHECK();
}

int check_policy_device(const int* alpha, const int* beta, const uint8_t* valid, int n, int m1, int m2,
                        int* err_dev, hipStream_t s) {
  fill_async(err_dev, 0, 1, s);
  hipLaunchKernelGGL(k_check_policy, dim3(grid_for(n)), dim3(kBlock), 0, s, alpha, beta, valid, n, m1, m2,
                     err_dev);
  SHP_LAUNCH_CHECK();
  int bits = 0;
  d2h(&bits, err_dev, 1, s);
  SHP_HIP(hipStreamSynchronize(s));
  return bits;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (block scan + recursive scan of block sums)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(256) void k_scan_block(const int* __restrict__ in, int* __restrict__ out,
                                                    int* __restrict__ sums, int n) {
  __shared__ int sh[kBlock];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int tot = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    tot += v[i];
  }
  sh[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    int add = (threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tot;  // exclusive prefix of this thread
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == kBlock - 1) sums[blockIdx.x] = sh[kBlock - 1];
}

__global__ void k_scan_add(int* __restrict__ out, const int* __restrict__ sums, int n) {
  int i = blockIdx.x * kScanTile + threadIdx.x;
  int add = sums[blockIdx.x];
  for (int j = 0; j < kScanItems; ++j, i += kBlock)
    if (i < n) out[i] += add;
}

static void scan_rec(const int* in, int* out, int n, hipStream_t s, int* scratch, size_t cap) {
  int nb = (n + kScanTile - 1) / kScanTile;
  if ((size_t)nb > cap) throw Error(SHAPLEY_EDEVICE, "scan scratch too small");
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kBlock), 0, s, in, out, scratch, n);
  SHP_LAUNCH_CHECK();
  if (nb > 1) {
    scan_rec(scratch, scratch, nb, s, scratch + nb, cap - nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kBlock), 0, s, out, scratch, n);
    SHP_LAUNCH_CHECK();
  }
}

void scan_exclusive(const int* in, int* out, int n, hipStream_t s, DBuf<int>& scratch) {
  if (n <= 0) return;
  size_t need = 0;
  for (int m = n; m > 1; m = (m + kScanTile - 1) / kScanTile) need += (m + kScanTile - 1) / kScanTile;
  need += 4;
  scratch.ensure(need);
  scan_rec(in, out, n, s, scratch.p, scratch.n);
}

}  // namespace shp
