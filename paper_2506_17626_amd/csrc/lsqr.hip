// Right-preconditioned LSQR on the block-sparse system (Algorithm 2, Proposition 3.1)
// on gfx950, and the back-substitution a = S^{-1} y.
//
// Operator A = sum_j V_j^T Q_hat_j W_hat_j (Q form).  Vectors over columns use the
// padded per-feature layout (entry (j,k) at feat_off[j] + k, k < r_j; the rest stay 0).
//
// One LSQR iteration of the Q form = five launches on the caller's stream:
//   fwd_local   t_(j,i) = sum_k Q_hat_j[i,k] v_j[k]       lane <-> row, coalesced column reads
//   fwd_gather  p_r = sum_{j covering r} t_(j,r) - alpha u_r, summed in ascending j (no
//               atomics, so the result does not depend on scheduling); ||p||^2 partials
//   reduce_step beta
//   adj_local   z_j = Q_hat_j^T (p / beta) over column tiles of I_j x r_j (the block's rows
//               of p, copied contiguously by fwd_gather, staged in LDS once per
//               workgroup), q = z - beta v; ||q||^2 partials
//   yw_update   alpha = sqrt(sum of the adjoint partials) and the Givens-rotation scalar step
//               of Paige-Saunders, y += (phi/rho) w, w = v - (theta/rho) w; ||y||^2 partials
//   reduce_step ||y|| and the stopping rule (raises the done flag)
// Every grid-wide sum is a fixed-order sum of per-workgroup partials, so results are bitwise
// reproducible.  A one-workgroup reduce_step finishes a sum and is the only writer of the
// scalar state, except in yw_update, where every workgroup recomputes alpha from the
// adjoint partials (identical instructions on identical data, so every workgroup holds the
// same value) and one workgroup stores the scalars, in fields no workgroup of the same launch
// reads.  The R form (transposed solves around the products) finishes alpha in a reduce_step
// too.  After the done flag is up every kernel returns at once, so the host launches
// iterations in batches (optionally one captured HIP graph per batch) and only reads the
// scalar state between batches.
#include <cmath>
#include <cstdint>
#include <vector>

#include <hip/hip_ext.h>

#include "common.hpp"

namespace rfm {
namespace {

struct State {
  double alpha, beta;      // alpha_i, beta_i of u_i = p/beta_i, v_i = q/alpha_i
  double beta_next;        // beta_{i+1} from the forward gather
  double rhobar, phibar;
  double rhobar_n, phibar_n;  // the rotation's new values, promoted by the step that follows
  double phi_rho, theta_rho;
  double rnorm, artnorm, ynorm, hnorm, anorm;
  double atol, btol;
  int64_t iter, maxit;
  int32_t done, stop;
  double *history;         // nullable device [2 * maxit]: (rnorm, artnorm) estimates
  double *bidiag;          // nullable device [2 * maxit + 2]: (alpha_i, beta_i), i = 1..
};

enum Mode : int { ITER = 0, INIT = 1, RESID = 2, COPYH = 3 };
enum Flags : int { F_CHECK_DONE = 1, F_DIV_ALPHA = 2, F_DIV_BETA = 4, F_COMBINE = 8 };
enum Reduce : int { R_BETA = 0, R_BETA_INIT = 1, R_ALPHA = 2, R_ALPHA_INIT = 3, R_Y = 4, R_Y_INIT = 5,
                    R_CHK_R = 6, R_CHK_AT = 7, R_YF = 8 };

constexpr int kRowTile = 256;
constexpr int kAdjThreads = 256;
constexpr int kAdjCols = 4;    // adjoint products: columns per wave ...
constexpr int kAdjChunks = 2;  // ... and rows chunks of 64 per step (kAdjCols x kAdjChunks loads in flight)
constexpr int kVecThreads = 256;
constexpr int kRedThreads = 1024;
constexpr int kStages = 5;   // timed stages of one iteration (see rfm_kernel_times)

// Givens rotation eliminating beta_{i+1} (Paige-Saunders recurrences), from rhobar_i,
// phibar_i, alpha_{i+1} and beta_{i+1}.
struct Rotation {
  double rhobar, phibar, phi_rho, theta_rho, artnorm;
};
__device__ __forceinline__ Rotation givens(double rhobar, double phibar, double an, double bn) {
  const double rho = hypot(rhobar, bn);
  const double c = rhobar / rho;
  const double sn = bn / rho;
  const double theta = sn * an;
  const double phi = c * phibar;
  Rotation g;
  g.rhobar = -c * an;
  g.phibar = sn * phibar;
  g.phi_rho = phi / rho;
  g.theta_rho = theta / rho;
  g.artnorm = g.phibar * an * fabs(c);
  return g;
}

// Fixed-order sum of part[0..n) by one workgroup (four strided accumulators per thread, then
// the workgroup sum); the result is in every thread.
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int64_t n, double *red) {
  const int64_t s = blockDim.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 3 * s < n; i += 4 * s) {
    a0 += part[i];
    a1 += part[i + s];
    a2 += part[i + 2 * s];
    a3 += part[i + 3 * s];
  }
  for (; i < n; i += s) a0 += part[i];
  return block_sum((a0 + a1) + (a2 + a3), red);
}

// Per-block operands of the block products, gathered once per solve so that a workgroup
// reads them with one scalar load issued together with the state's: the block's first row
// and first feature, its offset in the operand storage, its rows m_j and kept columns r_j.
struct alignas(32) BlockDesc {
  int64_t r0, f0, base;
  int32_t m, r;
};
static_assert(sizeof(BlockDesc) == 32, "one 32-byte scalar load per block");

__global__ void block_desc(rfm_layout L, const int32_t *__restrict__ rank, BlockDesc *__restrict__ d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L.J) return;
  BlockDesc b;
  b.r0 = L.row_off[j];
  b.f0 = L.feat_off[j];
  b.base = L.blk_off[j];
  b.m = (int32_t)(L.row_off[j + 1] - L.row_off[j]);
  b.r = rank[j];
  d[j] = b;
}

// ||M_hat_j||_F^2 over the kept columns of block j, one workgroup per block, fixed order.
__global__ __launch_bounds__(256) void kept_fro2(const double *__restrict__ M, const int32_t *__restrict__ kept,
                                                 const BlockDesc *__restrict__ desc, double *out) {
  __shared__ double red[256 / kWave];
  const BlockDesc d = desc[blockIdx.x];
  double s = 0.0;
  for (int k = 0; k < d.r; ++k) {
    const double *__restrict__ c = M + d.base + (int64_t)kept[d.f0 + k] * d.m;
    for (int i = threadIdx.x; i < d.m; i += 256) s = fma(c[i], c[i], s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void fill_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// y <- y0 on kept coordinates (or 0), 0 elsewhere.
__global__ void init_y(rfm_layout L, const int32_t *rank, const double *y0, double *y) {
  const int j = blockIdx.y;
  const int64_t f0 = L.feat_off[j];
  const int K = (int)(L.feat_off[j + 1] - f0);
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  y[f0 + k] = (y0 && k < rank[j]) ? y0[f0 + k] : 0.0;
}

// Operand element types of the block products: binary64, binary32, and bfloat16 stored as
// its upper 16 bits (products of the narrow types accumulate in binary32).
struct bf16_t {
  uint16_t bits;
};
template <typename T> struct Acc { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<bf16_t> { using type = float; };
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ float widen(bf16_t v) { return __uint_as_float(((uint32_t)v.bits) << 16); }

// Column k of block j's operand: Q_hat_j[:, k] (Q form, k < r_j), or the kept column
// M_j[:, kept_k] (R form, KEPT = true).
template <typename T, bool KEPT>
__device__ __forceinline__ const T *operand_col(const T *Op, int64_t base, const int *kept_lds, int k, int m) {
  return Op + base + (int64_t)(KEPT ? kept_lds[k] : k) * m;
}

// t_(j,i) = sum_k Op_j[i,k] * v_j[k] with v = vin / alpha (F_DIV_ALPHA) or vin.
template <typename T, bool KEPT>
__global__ __launch_bounds__(kRowTile) void fwd_local(rfm_layout L, const T *__restrict__ Op,
                                                      const int32_t *__restrict__ kept,
                                                      const BlockDesc *__restrict__ desc,
                                                      const double *__restrict__ vin,
                                                      double *__restrict__ t, const State *st,
                                                      int flags) {
  using A = typename Acc<T>::type;
  extern __shared__ double smem[];
  const int j = blockIdx.y;
  // the descriptor and the state are loaded before the first branch: one round trip
  const BlockDesc d = desc[j];
  const int dn = st->done;
  const double alpha = (flags & F_DIV_ALPHA) ? st->alpha : 1.0;
  if (((flags & F_CHECK_DONE) && dn) || (int)blockIdx.x * kRowTile >= d.m) return;
  const int64_t r0 = d.r0, f0 = d.f0;
  const int m = d.m, r = d.r;
  A *vs = (A *)smem;
  int *ks = (int *)(smem + L.max_cols);
  for (int k = threadIdx.x; k < r; k += kRowTile) {
    vs[k] = (A)((flags & F_DIV_ALPHA) ? vin[f0 + k] / alpha : vin[f0 + k]);
    if (KEPT) ks[k] = kept[f0 + k];
  }
  __syncthreads();
  const int i = blockIdx.x * kRowTile + threadIdx.x;
  if (i >= m) return;
  const int64_t base = d.base + i;
  // eight independent accumulators: eight loads in flight per thread
  A acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int k = 0;
  for (; k + 8 <= r; k += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += (A)widen(*operand_col<T, KEPT>(Op, base, ks, k + u, m)) * vs[k + u];
  }
  for (; k < r; ++k) acc[0] += (A)widen(*operand_col<T, KEPT>(Op, base, ks, k, m)) * vs[k];
  t[r0 + i] = (double)(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
}

// p_r = sum_j t_(j,r) - alpha * (pcur_r / beta)     (ITER)
// p_r = h_r - sum_j t_(j,r)                         (RESID)
// p_r = h_r                                         (COPYH)
// p goes to pnew (row order) and to ub in the block-row layout of t (ub[e] = p_rows[e]), so
// the adjoint products read their rows contiguously.  Per-workgroup partial sums of p^2 (and
// of h^2 outside ITER) go to part[] / part2[].
__global__ __launch_bounds__(kVecThreads) void fwd_gather(rfm_layout L, const double *__restrict__ t,
                                                          const double *__restrict__ h,
                                                          const double *__restrict__ pcur,
                                                          double *__restrict__ pnew, double *__restrict__ ub,
                                                          double *part, double *part2, const State *st,
                                                          int mode) {
  __shared__ double red[kVecThreads / kWave];
  if (mode == ITER && st->done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0, hh = 0.0;
  if (r < L.N) {
    double s = 0.0;
    const int64_t q0 = L.rinc_off[r], q1 = L.rinc_off[r + 1];
    if (mode != COPYH)
      for (int64_t q = q0; q < q1; ++q) s += t[L.rinc[q]];
    if (mode == ITER) {
      val = s - st->alpha * (pcur[r] / st->beta);
    } else {
      const double hr = h[r];
      val = (mode == RESID) ? hr - s : hr;
      hh = hr * hr;
    }
    pnew[r] = val;
    for (int64_t q = q0; q < q1; ++q) ub[L.rinc[q]] = val;
  }
  const double bs = block_sum(val * val, red);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
  if (mode != ITER) {
    const double bh = block_sum(hh, red);
    if (threadIdx.x == 0) part2[blockIdx.x] = bh;
  }
}

// z_j = Op_j^T u_{I_j} over a tile of ct columns of block j, u = p / beta_next (F_DIV_BETA)
// or p, with p in the block-row layout (ub, written by fwd_gather); with F_COMBINE
// q = z - beta_next * (qcur / alpha), else q = z.  Each wave takes kAdjCols columns at a time and
// reads u with the columns (no LDS staging; the R form stages its kept indices).  One
// partial of sum q^2 per workgroup.
template <typename T, bool KEPT>
__global__ __launch_bounds__(kAdjThreads) void adj_local(rfm_layout L, const T *__restrict__ Op,
                                                         const int32_t *__restrict__ kept,
                                                         const BlockDesc *__restrict__ desc,
                                                         const double *__restrict__ ub,
                                                         const double *__restrict__ qcur,
                                                         double *__restrict__ qnew, double *part,
                                                         int ct, const State *st, int flags) {
  using A = typename Acc<T>::type;
  extern __shared__ double smem[];
  __shared__ double colsum[kAdjThreads / kWave];
  constexpr int NW = kAdjThreads / kWave;
  const int j = blockIdx.y;
  const int k0 = blockIdx.x * ct;
  const int64_t pidx = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  // the descriptor and the state are loaded before the first branch: one round trip
  const BlockDesc d = desc[j];
  const int dn = st->done;
  const double bn = st->beta_next, alpha = st->alpha;
  const bool stop = (flags & F_CHECK_DONE) && dn;
  if (stop || k0 >= d.r) {
    if (!stop && threadIdx.x == 0) part[pidx] = 0.0;
    return;
  }
  const int r = d.r, m = d.m;
  const int k1 = min(r, k0 + ct);
  const int64_t r0 = d.r0, f0 = d.f0;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  int *ks = (int *)smem;
  if (KEPT) {
    for (int k = k0 + threadIdx.x; k < k1; k += kAdjThreads) ks[k - k0] = kept[f0 + k];
    __syncthreads();
  }
  // u_i read where it is used (the block's rows of p are contiguous in ub and shared by the
  // block's workgroups through the caches), so the column loads start without a barrier
  const double *__restrict__ pu = ub + r0;
  const bool divb = (flags & F_DIV_BETA) != 0;
  auto uval = [&](int i) -> A {
    const double p = pu[i];
    return (A)(divb ? (bn > 0.0 ? p / bn : 0.0) : p);
  };
  const int64_t base = d.base;
  double ssq = 0.0;
  for (int k = k0 + kAdjCols * wid; k < k1; k += kAdjCols * NW) {
    // column k + c of the tile: Q_hat_j[:, k + c], or M_j[:, kept] with the kept index staged
    // at ks[k + c - k0]; past the tile's end the last column is read again (and not stored)
    const T *__restrict__ cp[kAdjCols];
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c) {
      const int kk = min(k + c, k1 - 1);
      cp[c] = Op + base + (int64_t)(KEPT ? ks[kk - k0] : kk) * m;
    }
    A acc[kAdjCols][kAdjChunks];
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c)
#pragma unroll
      for (int h = 0; h < kAdjChunks; ++h) acc[c][h] = 0;
    int i = lane;
    for (; i + (kAdjChunks - 1) * kWave < m; i += kAdjChunks * kWave) {
#pragma unroll
      for (int h = 0; h < kAdjChunks; ++h) {
        const A u = uval(i + h * kWave);
#pragma unroll
        for (int c = 0; c < kAdjCols; ++c) acc[c][h] += (A)widen(cp[c][i + h * kWave]) * u;
      }
    }
    for (; i < m; i += kWave) {
      const A u = uval(i);
#pragma unroll
      for (int c = 0; c < kAdjCols; ++c) acc[c][0] += (A)widen(cp[c][i]) * u;
    }
    double z = 0.0;  // lane c < kAdjCols keeps the sum of column k + c
#pragma unroll
    for (int c = 0; c < kAdjCols; ++c) {
      A t = acc[c][0];
#pragma unroll
      for (int h = 1; h < kAdjChunks; ++h) t += acc[c][h];
      const double zc = wave_sum_dpp((double)t);
      if (lane == c) z = zc;
    }
    if (lane < kAdjCols && k + lane < k1) {
      const int kk = k + lane;
      const double q = (flags & F_COMBINE) ? z - bn * (qcur[f0 + kk] / alpha) : z;
      qnew[f0 + kk] = q;
      ssq += q * q;
    }
  }
  // lanes 0..kAdjCols-1 hold the squares of their columns; sum them in lane order
  ssq = wave_sum(ssq);
  if (lane == 0) colsum[wid] = ssq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += colsum[w];
    part[pidx] = s;
  }
}

// Blocked triangular solves with R_hat_j (upper, column-major in its K_j x K_j slot), one
// workgroup per block.  Tiles of 64 unknowns: the diagonal tile is staged in LDS and solved
// by one wave with shuffles (no barriers), the rest of the right-hand side is updated by the
// whole workgroup with coalesced reads of R.
constexpr int kTri = 64;
constexpr int kTriThreads = 256;

// x = R^{-1} b, b = vin / alpha (F_DIV_ALPHA) or vin; writes xout (entries k < r_j).
__global__ __launch_bounds__(kTriThreads) void trsv_upper(rfm_layout L, const int32_t *__restrict__ rank,
                                                          const double *__restrict__ R,
                                                          const double *__restrict__ vin,
                                                          double *__restrict__ xout, const State *st,
                                                          int flags) {
  extern __shared__ double smem[];
  if ((flags & F_CHECK_DONE) && st->done) return;
  const int j = blockIdx.x;
  const int64_t f0 = L.feat_off[j];
  const int n = (int)(L.feat_off[j + 1] - f0);
  const int r = rank[j];
  if (r == 0) return;
  const double *__restrict__ Rj = R + L.rsq_off[j];
  double *x = smem;
  double *D = smem + L.max_cols;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const double alpha = (flags & F_DIV_ALPHA) ? st->alpha : 1.0;
  for (int k = threadIdx.x; k < r; k += kTriThreads)
    x[k] = (flags & F_DIV_ALPHA) ? vin[f0 + k] / alpha : vin[f0 + k];
  for (int t = (r - 1) / kTri; t >= 0; --t) {
    const int k0 = t * kTri, w = min(kTri, r - k0);
    for (int e = threadIdx.x; e < kTri * kTri; e += kTriThreads) {
      const int c = e / kTri, rr = e % kTri;
      D[e] = (c < w && rr <= c) ? Rj[(int64_t)(k0 + c) * n + k0 + rr] : 0.0;
    }
    __syncthreads();
    if (wid == 0) {
      double xi = (lane < w) ? x[k0 + lane] : 0.0;
      for (int c = w - 1; c >= 0; --c) {
        if (lane == c) xi = xi / D[c * kTri + c];
        const double xc = __shfl(xi, c, kWave);
        if (lane < c) xi -= D[c * kTri + lane] * xc;
      }
      if (lane < w) x[k0 + lane] = xi;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k0; i += kTriThreads) {
      double acc = 0.0;
      for (int c = 0; c < w; ++c) acc += Rj[(int64_t)(k0 + c) * n + i] * x[k0 + c];
      x[i] -= acc;
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < r; k += kTriThreads) xout[f0 + k] = x[k];
}

// w = R^{-T} z; with F_COMBINE q = w - beta_next * (qcur / alpha), else q = w; one partial
// of sum q^2 per block.
__global__ __launch_bounds__(kTriThreads) void trsv_upper_t(rfm_layout L, const int32_t *__restrict__ rank,
                                                            const double *__restrict__ R,
                                                            const double *__restrict__ z,
                                                            const double *__restrict__ qcur,
                                                            double *__restrict__ qnew, double *part,
                                                            const State *st, int flags) {
  extern __shared__ double smem[];
  __shared__ double red[kTriThreads / kWave];
  if ((flags & F_CHECK_DONE) && st->done) return;
  const int j = blockIdx.x;
  const int64_t f0 = L.feat_off[j];
  const int n = (int)(L.feat_off[j + 1] - f0);
  const int r = rank[j];
  if (r == 0) {
    if (threadIdx.x == 0) part[j] = 0.0;
    return;
  }
  const double *__restrict__ Rj = R + L.rsq_off[j];
  double *x = smem;
  double *D = smem + L.max_cols;
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  constexpr int NW = kTriThreads / kWave;
  for (int k = threadIdx.x; k < r; k += kTriThreads) x[k] = z[f0 + k];
  for (int t = 0; t * kTri < r; ++t) {
    const int k0 = t * kTri, w = min(kTri, r - k0), k1 = k0 + w;
    for (int e = threadIdx.x; e < kTri * kTri; e += kTriThreads) {
      const int c = e / kTri, rr = e % kTri;
      D[e] = (c < w && rr <= c) ? Rj[(int64_t)(k0 + c) * n + k0 + rr] : 0.0;
    }
    __syncthreads();
    if (wid == 0) {
      double xi = (lane < w) ? x[k0 + lane] : 0.0;
      for (int c = 0; c < w; ++c) {
        if (lane == c) xi = xi / D[c * kTri + c];
        const double xc = __shfl(xi, c, kWave);
        if (lane > c && lane < w) xi -= D[lane * kTri + c] * xc;
      }
      if (lane < w) x[k0 + lane] = xi;
    }
    __syncthreads();
    // rows k1..r-1: x_i -= sum_{c in tile} R[k0+c, i] x_{k0+c}; column i of R is contiguous
    for (int i = k1 + wid; i < r; i += NW) {
      const double v = (lane < w) ? Rj[(int64_t)i * n + k0 + lane] * x[k0 + lane] : 0.0;
      const double s = wave_sum(v);
      if (lane == 0) x[i] -= s;
    }
    __syncthreads();
  }
  const double bn = st->beta_next, alpha = st->alpha;
  double ssq = 0.0;
  for (int k = threadIdx.x; k < r; k += kTriThreads) {
    const double q = (flags & F_COMBINE) ? x[k] - bn * (qcur[f0 + k] / alpha) : x[k];
    qnew[f0 + k] = q;
    ssq += q * q;
  }
  ssq = block_sum(ssq, red);
  if (threadIdx.x == 0) part[j] = ssq;
}

// ITER: y += (phi/rho) w ; w = v - (theta/rho) w with v = q / alpha.   INIT: w = q / alpha.
// With apart (ITER, Q form) every workgroup forms alpha from the napart adjoint partials and
// performs the rotation itself; the first workgroup stores the scalars (the rotation's
// rhobar / phibar in the _n fields, promoted by the R_YF step).  Per-workgroup partials of
// ||y||^2.
__global__ __launch_bounds__(kVecThreads) void yw_update(int64_t n, const double *__restrict__ qnew,
                                                         double *__restrict__ w,
                                                         double *__restrict__ y, double *part,
                                                         State *st, int mode,
                                                         const double *__restrict__ apart, int64_t napart) {
  __shared__ double red[kVecThreads / kWave];
  if (st->done && mode == ITER) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double a, phr, thr;
  if (mode == ITER && apart) {
    const double an = sqrt(sum_partials(apart, napart, red));
    const double bn = st->beta_next;
    const Rotation g = givens(st->rhobar, st->phibar, an, bn);
    a = an;
    phr = g.phi_rho;
    thr = g.theta_rho;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->alpha = an;
      st->beta = bn;
      st->rhobar_n = g.rhobar;
      st->phibar_n = g.phibar;
      st->phi_rho = g.phi_rho;
      st->theta_rho = g.theta_rho;
      st->rnorm = g.phibar;
      st->artnorm = g.artnorm;
    }
  } else {
    a = st->alpha;
    phr = st->phi_rho;
    thr = st->theta_rho;
  }
  double yy = 0.0;
  if (k < n) {
    const double v = (a > 0.0) ? qnew[k] / a : 0.0;
    if (mode == ITER) {
      const double wk = w[k];
      const double yk = y[k] + phr * wk;
      y[k] = yk;
      w[k] = v - thr * wk;
      yy = yk * yk;
    } else {
      w[k] = v;
      yy = y[k] * y[k];
    }
  }
  const double bs = block_sum(yy, red);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

// One workgroup: finishes a grid-wide sum of partials in a fixed order and performs the
// scalar step that needs it (the only writer of the state, so no other workgroup can
// observe a half-updated state).
__global__ __launch_bounds__(kRedThreads) void reduce_step(const double *part, int64_t n,
                                                           const double *part2, State *st, int what) {
  __shared__ double red[kRedThreads / kWave];
  if ((what == R_BETA || what == R_ALPHA || what == R_Y || what == R_YF) && st->done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kRedThreads) s += part[i];
  s = block_sum(s, red);
  double s2 = 0.0;
  if (what == R_BETA_INIT || what == R_CHK_R) {
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kRedThreads) t += part2[i];
    s2 = block_sum(t, red);
  }
  if (threadIdx.x != 0) return;
  switch (what) {
    case R_BETA:
      st->beta_next = sqrt(s);
      break;
    case R_BETA_INIT:
      st->beta_next = sqrt(s);
      st->hnorm = sqrt(s2);
      break;
    case R_ALPHA_INIT: {
      const double an = sqrt(s), bn = st->beta_next;
      st->alpha = an;
      st->beta = bn;
      st->rhobar = an;
      st->phibar = bn;
      if (st->bidiag) {
        st->bidiag[0] = an;
        st->bidiag[1] = bn;
      }
      st->rnorm = bn;
      st->artnorm = an * bn;
      st->iter = 0;
      st->stop = 0;
      st->done = (an == 0.0 || bn == 0.0) ? 1 : 0;
      if (st->done) st->stop = 4;
      break;
    }
    case R_ALPHA: {
      const double an = sqrt(s), bn = st->beta_next;
      const Rotation g = givens(st->rhobar, st->phibar, an, bn);
      st->rhobar = g.rhobar;
      st->phibar = g.phibar;
      st->phi_rho = g.phi_rho;
      st->theta_rho = g.theta_rho;
      st->rnorm = g.phibar;
      st->artnorm = g.artnorm;
      st->alpha = an;
      st->beta = bn;
      break;
    }
    case R_Y_INIT:
      st->ynorm = sqrt(s);
      break;
    case R_YF:  // the rotation of the fused update becomes the current one
      st->rhobar = st->rhobar_n;
      st->phibar = st->phibar_n;
      [[fallthrough]];
    case R_Y: {
      st->ynorm = sqrt(s);
      st->iter += 1;
      if (st->history && st->iter <= st->maxit) {
        st->history[2 * (st->iter - 1)] = st->rnorm;
        st->history[2 * (st->iter - 1) + 1] = st->artnorm;
      }
      if (st->bidiag && st->iter <= st->maxit) {  // alpha_{i+1}, beta_{i+1} of iteration i
        st->bidiag[2 * st->iter] = st->alpha;
        st->bidiag[2 * st->iter + 1] = st->beta;
      }
      int stop = 0;
      if (st->beta == 0.0 || st->alpha == 0.0) stop = 4;
      else if (st->rnorm <= st->btol * st->hnorm + st->atol * st->anorm * st->ynorm) stop = 1;
      else if (st->artnorm <= st->atol * st->anorm * st->rnorm) stop = 2;
      else if (st->iter >= st->maxit) stop = 3;
      if (stop) {
        st->stop = stop;
        st->done = 1;
      }
      break;
    }
    case R_CHK_R:
      st->rnorm = sqrt(s);
      st->hnorm = sqrt(s2);
      break;
    case R_CHK_AT:
      st->artnorm = sqrt(s);
      break;
  }
}

// a_hat_j = R_hat_j^{-1} y_j (column-oriented back-substitution in LDS) scattered to
// a[f0 + kept[k]]; every other coefficient of the block is 0.
__global__ __launch_bounds__(256) void back_substitute(rfm_layout L, const int32_t *rank,
                                                       const int32_t *kept, const double *R,
                                                       const double *y, double *a) {
  extern __shared__ double x[];
  const int j = blockIdx.x;
  const int64_t f0 = L.feat_off[j];
  const int n = (int)(L.feat_off[j + 1] - f0);
  const int r = rank[j];
  const double *Rj = R + L.rsq_off[j];
  for (int k = threadIdx.x; k < r; k += blockDim.x) x[k] = y[f0 + k];
  for (int k = threadIdx.x; k < n; k += blockDim.x) a[f0 + k] = 0.0;
  __syncthreads();
  for (int k = r - 1; k >= 0; --k) {
    if (threadIdx.x == 0) x[k] = x[k] / Rj[(int64_t)k * n + k];
    __syncthreads();
    const double xk = x[k];
    for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] -= Rj[(int64_t)k * n + i] * xk;
    __syncthreads();
  }
  for (int k = threadIdx.x; k < r; k += blockDim.x) a[f0 + kept[f0 + k]] = x[k];
}

// Round the kept columns of Q_hat to binary32 (round to nearest even) or to bfloat16 (the
// binary32 value rounded to nearest even on its upper 16 bits).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename T> __device__ __forceinline__ T narrow(double v);
template <> __device__ __forceinline__ float narrow<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16_t narrow<bf16_t>(double v) { return bf16_t{bf16_bits((float)v)}; }

template <typename T>
__global__ __launch_bounds__(kRowTile) void pack_q(rfm_layout L, const int32_t *__restrict__ rank,
                                                   const double *__restrict__ Q, T *__restrict__ out) {
  const int j = blockIdx.y;
  const int m = (int)(L.row_off[j + 1] - L.row_off[j]);
  const int i = blockIdx.x * kRowTile + threadIdx.x;
  if (i >= m) return;
  const int r = rank[j];
  const int64_t base = L.blk_off[j] + i;
  for (int k = 0; k < r; ++k) out[base + (int64_t)k * m] = narrow<T>(Q[base + (int64_t)k * m]);
}

__global__ void axpy_inplace(int64_t n, const double *__restrict__ x, double *__restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] += x[k];
}

__global__ __launch_bounds__(kVecThreads) void sq_partials(int64_t n, const double *__restrict__ x, double *part) {
  __shared__ double red[kVecThreads / kWave];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double v = (k < n) ? x[k] : 0.0;
  const double bs = block_sum(v * v, red);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
}

struct Work {
  double *t, *ub, *p[2], *res, *q[2], *w, *z, *xs, *zs, *dy, *part, *part2, *part3;
  BlockDesc *desc;
  State *st, *st2;
  int64_t npart;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Column tile of the adjoint products: about 4096 workgroups in total, tiles a multiple
// of kAdjQuantum columns (every wave of the workgroup takes kAdjCols columns).
constexpr int kAdjQuantum = kAdjCols * (kAdjThreads / kWave);
int adj_tile(const rfm_layout *L) {
  const int64_t mc = L->max_cols > 0 ? L->max_cols : 1;
  int64_t tiles = (4096 + L->J - 1) / L->J;
  const int64_t max_tiles = (mc + kAdjQuantum - 1) / kAdjQuantum;
  if (tiles > max_tiles) tiles = max_tiles;
  if (tiles < 1) tiles = 1;
  const int64_t per = (mc + tiles - 1) / tiles;
  return (int)(((per + kAdjQuantum - 1) / kAdjQuantum) * kAdjQuantum);
}

size_t carve(const rfm_layout *L, char *base, Work *W) {
  const int64_t N = L->N, nc = L->ncols;
  const int64_t g_rows = (N + kVecThreads - 1) / kVecThreads;
  const int64_t g_cols = (nc + kVecThreads - 1) / kVecThreads;
  const int ct = kAdjQuantum;  // smallest allowed adjoint tile: the most partials
  const int64_t g_adj = (int64_t)L->J * (((L->max_cols > 0 ? L->max_cols : 1) + ct - 1) / ct);
  int64_t npart = g_rows;
  if (g_cols > npart) npart = g_cols;
  if (g_adj > npart) npart = g_adj;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  Work w{};
  w.desc = (BlockDesc *)take(sizeof(BlockDesc) * (size_t)L->J);
  w.t = (double *)take(sizeof(double) * (size_t)L->nnz_rows);
  w.ub = (double *)take(sizeof(double) * (size_t)L->nnz_rows);
  w.p[0] = (double *)take(sizeof(double) * N);
  w.p[1] = (double *)take(sizeof(double) * N);
  w.res = (double *)take(sizeof(double) * N);
  w.q[0] = (double *)take(sizeof(double) * nc);
  w.q[1] = (double *)take(sizeof(double) * nc);
  w.w = (double *)take(sizeof(double) * nc);
  w.z = (double *)take(sizeof(double) * nc);
  w.xs = (double *)take(sizeof(double) * nc);
  w.zs = (double *)take(sizeof(double) * nc);
  w.dy = (double *)take(sizeof(double) * nc);
  w.part = (double *)take(sizeof(double) * npart);
  w.part2 = (double *)take(sizeof(double) * npart);
  w.part3 = (double *)take(sizeof(double) * npart);
  w.st = (State *)take(sizeof(State));
  w.st2 = (State *)take(sizeof(State));
  w.npart = npart;
  if (W) *W = w;
  return off;
}

// Kernel launch that, when given events, has the runtime stamp them with the kernel's own
// start and end (the dispatch's timestamps, as a profiler sees them), not the time at which
// the stream reached the event.
template <typename F, typename... Args>
void launch(F kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
            Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, s, e0, e1, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

struct Launcher {
  const rfm_layout *L;
  const rfm_operator *A;
  const double *h;
  Work W;
  int ct;
  bool rform;
  bool mform = false;          // the kept columns of M without the preconditioner
  int dtype = RFM_F64;         // operand of the Q form: RFM_F64 (A->Q) or a narrow copy
  const void *Qlow = nullptr;  // RFM_F32 / RFM_BF16 copy of Q_hat in the block layout

  size_t fwd_lds() const { return (size_t)(L->max_cols > 0 ? L->max_cols : 1) * (sizeof(double) + sizeof(int)); }
  size_t adj_lds() const {
    return (rform || mform) ? sizeof(int) * (size_t)(L->max_cols > 0 ? L->max_cols : 1) : 0;
  }
  size_t tri_lds() const { return sizeof(double) * ((size_t)(L->max_cols > 0 ? L->max_cols : 1) + kTri * kTri); }
  unsigned g_rows() const { return ceil_div(L->N, kVecThreads); }
  unsigned g_cols() const { return ceil_div(L->ncols, kVecThreads); }
  unsigned g_adj_x() const { return ceil_div(L->max_cols > 0 ? L->max_cols : 1, ct); }
  int64_t n_adj_part() const { return rform ? (int64_t)L->J : (int64_t)g_adj_x() * L->J; }
  // Q form iterations take alpha and the rotation inside yw_update (see the file comment)
  bool fused() const { return !rform; }

  // Each stage below takes optional events: e0 is stamped at the start of its first kernel,
  // e1 at the end of its last.

  // t = A_local v (per-incidence block products); v = vin / alpha in ITER mode
  void fwd(hipStream_t s, const double *vin, State *st, int mode, hipEvent_t e0 = nullptr,
           hipEvent_t e1 = nullptr) {
    if (L->max_rows <= 0) return;
    const int flags = (mode == ITER) ? (F_CHECK_DONE | F_DIV_ALPHA) : 0;
    const dim3 grid(ceil_div(L->max_rows, kRowTile), L->J);
    const int32_t *nk = nullptr;
    if (mform) {
      launch(fwd_local<double, true>, grid, dim3(kRowTile), fwd_lds(), s, e0, e1, *L, (const double *)A->M, A->kept,
             (const BlockDesc *)W.desc, vin, W.t, (const State *)st, flags);
    } else if (!rform && dtype == RFM_F32) {
      launch(fwd_local<float, false>, grid, dim3(kRowTile), fwd_lds(), s, e0, e1, *L, (const float *)Qlow, nk,
             (const BlockDesc *)W.desc, vin, W.t, (const State *)st, flags);
    } else if (!rform && dtype == RFM_BF16) {
      launch(fwd_local<bf16_t, false>, grid, dim3(kRowTile), fwd_lds(), s, e0, e1, *L, (const bf16_t *)Qlow, nk,
             (const BlockDesc *)W.desc, vin, W.t, (const State *)st, flags);
    } else if (!rform) {
      launch(fwd_local<double, false>, grid, dim3(kRowTile), fwd_lds(), s, e0, e1, *L, (const double *)A->Q, nk,
             (const BlockDesc *)W.desc, vin, W.t, (const State *)st, flags);
    } else {
      launch(trsv_upper, dim3(L->J), dim3(kTriThreads), tri_lds(), s, e0, (hipEvent_t) nullptr, *L, A->rank,
             (const double *)A->R, vin, W.xs, (const State *)st, flags);
      launch(fwd_local<double, true>, grid, dim3(kRowTile), fwd_lds(), s, (hipEvent_t) nullptr, e1, *L,
             (const double *)A->M, A->kept, (const BlockDesc *)W.desc, (const double *)W.xs, W.t, (const State *)st,
             flags & F_CHECK_DONE);
    }
  }
  void gather(hipStream_t s, const double *pcur, double *pnew, State *st, int mode, hipEvent_t e0 = nullptr,
              hipEvent_t e1 = nullptr) {
    launch(fwd_gather, dim3(g_rows()), dim3(kVecThreads), 0, s, e0, e1, *L, (const double *)W.t, h, pcur, pnew,
           W.ub, W.part, W.part2, (const State *)st, mode);
  }
  // q = A^T u (- beta v in ITER mode), u = p / beta outside RESID mode; partials of ||q||^2.
  // p is the vector of the last gather (read from its block-row copy W.ub).
  void adj(hipStream_t s, const double *qcur, double *qnew, State *st, int mode, hipEvent_t e0 = nullptr,
           hipEvent_t e1 = nullptr) {
    const double *ubk = W.ub;
    int flags = 0;
    if (mode == ITER) flags = F_CHECK_DONE | F_DIV_BETA | F_COMBINE;
    if (mode == INIT) flags = F_DIV_BETA;
    // fused: the adjoint partials go to W.part3, where yw_update sums them
    double *pout = (mode == ITER && fused()) ? W.part3 : W.part;
    const dim3 grid(g_adj_x(), L->J);
    const int32_t *nk = nullptr;
    const BlockDesc *dsc = W.desc;
    const State *cst = st;
    if (mform) {
      launch(adj_local<double, true>, grid, dim3(kAdjThreads), adj_lds(), s, e0, e1, *L, (const double *)A->M,
             A->kept, dsc, ubk, qcur, qnew, pout, ct, cst, flags);
    } else if (!rform && dtype == RFM_F32) {
      launch(adj_local<float, false>, grid, dim3(kAdjThreads), adj_lds(), s, e0, e1, *L, (const float *)Qlow, nk,
             dsc, ubk, qcur, qnew, pout, ct, cst, flags);
    } else if (!rform && dtype == RFM_BF16) {
      launch(adj_local<bf16_t, false>, grid, dim3(kAdjThreads), adj_lds(), s, e0, e1, *L, (const bf16_t *)Qlow,
             nk, dsc, ubk, qcur, qnew, pout, ct, cst, flags);
    } else if (!rform) {
      launch(adj_local<double, false>, grid, dim3(kAdjThreads), adj_lds(), s, e0, e1, *L, (const double *)A->Q,
             nk, dsc, ubk, qcur, qnew, pout, ct, cst, flags);
    } else {
      launch(adj_local<double, true>, grid, dim3(kAdjThreads), adj_lds(), s, e0, (hipEvent_t) nullptr, *L,
             (const double *)A->M, A->kept, dsc, ubk, qcur, W.zs, W.part, ct, cst, flags & ~F_COMBINE);
      launch(trsv_upper_t, dim3(L->J), dim3(kTriThreads), tri_lds(), s, (hipEvent_t) nullptr, e1, *L, A->rank,
             (const double *)A->R, (const double *)W.zs, qcur, qnew, W.part, cst, flags & (F_CHECK_DONE | F_COMBINE));
    }
  }
  void yw(hipStream_t s, const double *qnew, double *y, State *st, int mode, hipEvent_t e0 = nullptr,
          hipEvent_t e1 = nullptr) {
    // fused: alpha and the rotation from the adjoint partials (W.part3)
    const bool fz = (mode == ITER && fused());
    launch(yw_update, dim3(g_cols()), dim3(kVecThreads), 0, s, e0, e1, (int64_t)L->ncols, qnew, W.w, y, W.part,
           st, mode, fz ? (const double *)W.part3 : (const double *)nullptr, fz ? n_adj_part() : (int64_t)0);
  }
  void reduce(hipStream_t s, int64_t n, State *st, int what, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    launch(reduce_step, dim3(1), dim3(kRedThreads), 0, s, e0, e1, (const double *)W.part, n,
           (const double *)W.part2, st, what);
  }
  // ev (nullable): 2 * kStages events, a start and an end per stage of one iteration, stamped
  // by the stage's kernels (the fused Q form has no separate alpha / rotation stage)
  void iteration(hipStream_t s, int64_t i, double *y, hipEvent_t *ev) {
    const int a = (int)((i - 1) & 1), b = (int)(i & 1);
    const bool fz = fused();
    auto E = [&](int k) { return ev ? ev[k] : (hipEvent_t) nullptr; };
    fwd(s, W.q[a], W.st, ITER, E(0), E(1));
    gather(s, W.p[a], W.p[b], W.st, ITER, E(2), nullptr);
    reduce(s, g_rows(), W.st, R_BETA, nullptr, E(3));
    adj(s, W.q[a], W.q[b], W.st, ITER, E(4), E(5));
    if (!fz) reduce(s, n_adj_part(), W.st, R_ALPHA, E(6), E(7));
    yw(s, W.q[b], y, W.st, ITER, E(8), nullptr);
    reduce(s, g_cols(), W.st, fz ? R_YF : R_Y, nullptr, E(9));
  }
};

struct EventPool {
  std::vector<hipEvent_t> ev;
  ~EventPool() {
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
  }
  hipError_t init(size_t n) {
    ev.resize(n, nullptr);
    for (size_t k = 0; k < n; ++k) {
      hipError_t e = hipEventCreate(&ev[k]);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
};

// A batch of iterations captured once on a private stream and replayed on the caller's.
struct Graph {
  hipStream_t cap = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  ~Graph() {
    if (ge) hipGraphExecDestroy(ge);
    if (g) hipGraphDestroy(g);
    if (cap) hipStreamDestroy(cap);
  }
};

// LSQR with the launcher's operator on the right-hand side X.h, from y0 (nullable) into y.
// Fills *out with the final scalar state (iterations, stop reason, estimates).
// A warm start whose residual ||h - A y0|| exceeds ||h|| is discarded for the cold start
// (the cold start stays the fallback); *rejected (nullable) reports it.
rfm_status run_lsqr(Launcher &X, double anorm, const double *y0, double *y, double atol, double btol,
                    int64_t maxit, int check_every, bool use_graph, rfm_kernel_times *times,
                    double *history, hipStream_t st, State *out, int32_t *rejected = nullptr,
                    double *bidiag = nullptr) {
  const rfm_layout *L = X.L;
  State hs{};
  hs.anorm = anorm;
  hs.atol = atol;
  hs.btol = btol;
  hs.maxit = maxit;
  hs.history = history;
  hs.bidiag = bidiag;
  RFM_HIP_TRY(hipMemcpyAsync(X.W.st, &hs, sizeof(State), hipMemcpyHostToDevice, st));
  for (double *b : {X.W.q[0], X.W.q[1], X.W.w})
    hipLaunchKernelGGL(fill_zero, dim3(ceil_div(L->ncols, 256)), dim3(256), 0, st, b, L->ncols);
  if (L->max_cols > 0)
    hipLaunchKernelGGL(init_y, dim3(ceil_div(L->max_cols, 256), L->J), dim3(256), 0, st, *L, X.A->rank, y0, y);
  RFM_LAUNCH_CHECK();

  // r0 = h - A y0, beta_1 u_1 = r0, alpha_1 v_1 = A^T u_1, w_1 = v_1
  bool cold = (y0 == nullptr);
  if (rejected) *rejected = 0;
  if (!cold) {
    X.fwd(st, y, X.W.st, RESID);
    X.gather(st, nullptr, X.W.p[0], X.W.st, RESID);
    X.reduce(st, X.g_rows(), X.W.st, R_BETA_INIT);
    RFM_LAUNCH_CHECK();
    RFM_HIP_TRY(hipMemcpyAsync(&hs, X.W.st, sizeof(State), hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    if (hs.beta_next > hs.hnorm) {
      cold = true;
      if (rejected) *rejected = 1;
      hipLaunchKernelGGL(init_y, dim3(ceil_div(L->max_cols > 0 ? L->max_cols : 1, 256), L->J), dim3(256), 0, st, *L,
                         X.A->rank, (const double *)nullptr, y);
    }
  }
  if (cold) {
    X.gather(st, nullptr, X.W.p[0], X.W.st, COPYH);
    X.reduce(st, X.g_rows(), X.W.st, R_BETA_INIT);
  }
  X.adj(st, nullptr, X.W.q[0], X.W.st, INIT);
  X.reduce(st, X.n_adj_part(), X.W.st, R_ALPHA_INIT);
  X.yw(st, X.W.q[0], y, X.W.st, INIT);
  X.reduce(st, X.g_cols(), X.W.st, R_Y_INIT);
  RFM_LAUNCH_CHECK();
  RFM_HIP_TRY(hipMemcpyAsync(&hs, X.W.st, sizeof(State), hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));

  int64_t i = 0;
  // batches of an even number of iterations, so the ping-pong buffers return to their start;
  // with timing requested the first two iterations of every batch are launched eagerly with
  // events around each stage (a sample of the kernels' durations inside the same solve)
  const int64_t batch = 2 * (((int64_t)check_every + 1) / 2);
  const int64_t sampled = times ? 2 : 0;
  const bool graph = use_graph && batch > sampled;
  EventPool pool;
  Graph G;
  if (times) RFM_HIP_TRY(pool.init((size_t)(2 * kStages) * sampled));
  if (graph && !hs.done) {
    RFM_HIP_TRY(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    RFM_HIP_TRY(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    for (int64_t b = sampled + 1; b <= batch; ++b) X.iteration(G.cap, b, y, nullptr);
    hipError_t le = hipGetLastError();
    hipError_t ce = hipStreamEndCapture(G.cap, &G.g);
    if (le != hipSuccess) return fail(RFM_EHIP, std::string("capture launch: ") + hipGetErrorString(le));
    if (ce != hipSuccess) return fail(RFM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    RFM_HIP_TRY(hipGraphInstantiate(&G.ge, G.g, nullptr, nullptr, 0));
  }
  while (!hs.done && i < maxit) {
    const int64_t first = i + 1;
    for (int64_t b = 0; b < sampled; ++b) X.iteration(st, ++i, y, pool.ev.data() + 2 * kStages * b);
    if (graph) {
      RFM_HIP_TRY(hipGraphLaunch(G.ge, st));
      i += batch - sampled;
    } else {
      for (int64_t b = sampled; b < batch; ++b) X.iteration(st, ++i, y, nullptr);
    }
    RFM_LAUNCH_CHECK();
    RFM_HIP_TRY(hipMemcpyAsync(&hs, X.W.st, sizeof(State), hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    // sampled iterations that did work (later launches return at once after the stop)
    for (int64_t b = 0; b < sampled && first + b <= hs.iter; ++b)
      for (int k = 0; k < kStages; ++k) {
        if (k == 3 && X.fused()) continue;  // no separate alpha / rotation launch
        float ms = 0.f;
        const size_t e0 = (size_t)(2 * kStages) * b + 2 * k;
        RFM_HIP_TRY(hipEventElapsedTime(&ms, pool.ev[e0], pool.ev[e0 + 1]));
        times->ms[k] += ms;
        times->launches[k] += 1;
      }
  }
  *out = hs;
  return RFM_OK;
}

// Explicit residuals of y with the launcher's operator and right-hand side X.h:
// out->rnorm = ||h - A y||, out->hnorm = ||h||, out->artnorm = ||A^T r||, out->ynorm = ||y||.
// The residual is left in X.W.res.
rfm_status explicit_check(Launcher &X, const double *y, hipStream_t st, State *out) {
  X.fwd(st, y, X.W.st2, RESID);
  X.gather(st, nullptr, X.W.res, X.W.st2, RESID);
  X.reduce(st, X.g_rows(), X.W.st2, R_CHK_R);
  X.adj(st, nullptr, X.W.z, X.W.st2, RESID);
  X.reduce(st, X.n_adj_part(), X.W.st2, R_CHK_AT);
  hipLaunchKernelGGL(sq_partials, dim3(X.g_cols()), dim3(kVecThreads), 0, st, X.L->ncols, y, X.W.part);
  X.reduce(st, X.g_cols(), X.W.st2, R_Y_INIT);
  RFM_LAUNCH_CHECK();
  RFM_HIP_TRY(hipMemcpyAsync(out, X.W.st2, sizeof(State), hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));
  return RFM_OK;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_lsqr_ws_bytes(const rfm_layout *L) {
  if (!L) return 0;
  return rfm::carve(L, nullptr, nullptr);
}

extern "C" rfm_status rfm_pack_q(const rfm_layout *L, const int32_t *rank, const double *Q, int32_t dtype,
                                 void *Qlow, void *stream) {
  using namespace rfm;
  rfm_status s0 = check_layout(L, "rfm_pack_q");
  if (s0 != RFM_OK) return s0;
  if (dtype != RFM_F32 && dtype != RFM_BF16) return fail(RFM_EINVAL, "rfm_pack_q: dtype must be RFM_F32 or RFM_BF16");
  if (!rank || (L->nnz > 0 && (!Q || !Qlow))) return fail(RFM_EINVAL, "rfm_pack_q: null pointer");
  if (L->max_rows <= 0) return RFM_OK;
  const dim3 grid(ceil_div(L->max_rows, kRowTile), L->J);
  if (dtype == RFM_F32)
    hipLaunchKernelGGL(pack_q<float>, grid, dim3(kRowTile), 0, (hipStream_t)stream, *L, rank, Q, (float *)Qlow);
  else
    hipLaunchKernelGGL(pack_q<bf16_t>, grid, dim3(kRowTile), 0, (hipStream_t)stream, *L, rank, Q, (bf16_t *)Qlow);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_lsqr_solve(const rfm_layout *L, const rfm_operator *A, const double *h,
                                     const double *y0, const rfm_lsqr_opts *opts, double *y,
                                     rfm_lsqr_info *info, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s0 = check_layout(L, "rfm_lsqr_solve");
  if (s0 != RFM_OK) return s0;
  if (!A || !A->rank || !opts || !h || !y || !info) return fail(RFM_EINVAL, "rfm_lsqr_solve: null pointer");
  if (A->form != RFM_FORM_Q && A->form != RFM_FORM_R && A->form != RFM_FORM_M)
    return fail(RFM_EINVAL, "rfm_lsqr_solve: bad form");
  if (A->form == RFM_FORM_M && ((L->nnz > 0 && !A->M) || !A->kept))
    return fail(RFM_EINVAL, "rfm_lsqr_solve: M form needs M and kept");
  if (A->form == RFM_FORM_Q && L->nnz > 0 && !A->Q) return fail(RFM_EINVAL, "rfm_lsqr_solve: null Q");
  if (A->form == RFM_FORM_R && ((L->nnz > 0 && !A->M) || !A->kept || (L->nrsq > 0 && !A->R)))
    return fail(RFM_EINVAL, "rfm_lsqr_solve: R form needs M, kept and R");
  if (opts->maxit < 1 || opts->check_every < 1 || !(opts->atol >= 0) || !(opts->btol >= 0))
    return fail(RFM_EINVAL, "rfm_lsqr_solve: bad options");
  const bool mixed = opts->inner_dtype != RFM_F64;
  if (mixed && A->form != RFM_FORM_Q) return fail(RFM_EINVAL, "rfm_lsqr_solve: the precision form needs the Q form");
  if (mixed) {
    if (opts->inner_dtype != RFM_F32 && opts->inner_dtype != RFM_BF16)
      return fail(RFM_EINVAL, "rfm_lsqr_solve: inner_dtype must be RFM_F64, RFM_F32 or RFM_BF16");
    if (!A->Qlow || A->low_dtype != opts->inner_dtype)
      return fail(RFM_EINVAL, "rfm_lsqr_solve: the operator needs Qlow packed in inner_dtype");
    if (opts->max_outer < 1 || opts->max_inner < 1 || !(opts->inner_tol > 0 && opts->inner_tol < 1))
      return fail(RFM_EINVAL, "rfm_lsqr_solve: bad refinement options");
  }
  if (ws_bytes < rfm_lsqr_ws_bytes(L) || !ws) return fail(RFM_EINVAL, "rfm_lsqr_solve: workspace too small");
  if ((size_t)L->max_cols * (sizeof(double) + sizeof(int)) > 120 * 1024 ||
      ((size_t)L->max_cols + kTri * kTri) * sizeof(double) > 120 * 1024)
    return fail(RFM_EUNSUPPORTED, "rfm_lsqr_solve: block too large for LDS staging");
  hipStream_t st = (hipStream_t)stream;

  Launcher X;
  X.L = L;
  X.A = A;
  X.h = h;
  X.ct = opts->adj_tile > 0 ? ((opts->adj_tile + kAdjQuantum - 1) / kAdjQuantum) * kAdjQuantum : adj_tile(L);
  X.rform = (A->form == RFM_FORM_R);
  X.mform = (A->form == RFM_FORM_M);
  carve(L, (char *)ws, &X.W);
  hipLaunchKernelGGL(block_desc, dim3(ceil_div(L->J, 256)), dim3(256), 0, st, *L, A->rank, X.W.desc);
  RFM_LAUNCH_CHECK();

  // ||A||_F: sqrt(sum_j r_j) for the Q and R forms (unit-norm columns); for the M form the
  // kept columns' Frobenius norm, per block on the device, summed here in block order
  double anorm;
  if (X.mform) {
    std::vector<double> hf(L->J);
    hipLaunchKernelGGL(kept_fro2, dim3(L->J), dim3(256), 0, st, A->M, A->kept, (const BlockDesc *)X.W.desc,
                       X.W.part);
    RFM_LAUNCH_CHECK();
    RFM_HIP_TRY(hipMemcpyAsync(hf.data(), X.W.part, sizeof(double) * L->J, hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    double f2 = 0.0;
    for (int32_t j = 0; j < L->J; ++j) f2 += hf[j];
    anorm = std::sqrt(f2);
  } else {
    std::vector<int32_t> hrank(L->J);
    RFM_HIP_TRY(hipMemcpyAsync(hrank.data(), A->rank, sizeof(int32_t) * L->J, hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    double nr = 0.0;
    for (int32_t j = 0; j < L->J; ++j) nr += hrank[j];
    anorm = std::sqrt(nr);
  }
  if (opts->times) *opts->times = rfm_kernel_times{};

  State hs{}, hc{};
  int64_t outer = 0;
  info->polish = 0;
  info->warm_rejected = 0;
  if (!mixed) {
    rfm_status s = run_lsqr(X, anorm, y0, y, opts->atol, opts->btol, opts->maxit, opts->check_every,
                            opts->use_graph != 0, opts->times, opts->history, st, &hs, &info->warm_rejected,
                            opts->bidiag);
    if (s != RFM_OK) return s;
    s = explicit_check(X, y, st, &hc);
    if (s != RFM_OK) return s;
  } else {
    // Refinement: the residual and the stopping test in binary64 with the full operator,
    // corrections from LSQR on the narrow copy of Q_hat (products accumulated in binary32).
    Launcher Xl = X;
    Xl.dtype = opts->inner_dtype;
    Xl.Qlow = A->Qlow;
    Xl.h = X.W.res;
    hipLaunchKernelGGL(init_y, dim3(ceil_div(L->max_cols > 0 ? L->max_cols : 1, 256), L->J), dim3(256), 0, st,
                       *L, A->rank, y0, y);
    RFM_LAUNCH_CHECK();
    if (y0) {  // the warm-start guard of the plain path, on the binary64 residual
      rfm_status s = explicit_check(X, y, st, &hc);
      if (s != RFM_OK) return s;
      if (hc.rnorm > hc.hnorm) {
        info->warm_rejected = 1;
        hipLaunchKernelGGL(init_y, dim3(ceil_div(L->max_cols > 0 ? L->max_cols : 1, 256), L->J), dim3(256), 0, st,
                           *L, A->rank, (const double *)nullptr, y);
        RFM_LAUNCH_CHECK();
      }
    }
    int64_t inner_total = 0, budget = opts->maxit;
    double prev_at = INFINITY;
    bool polish = false;
    hs.stop = 3;
    for (;; ++outer) {
      rfm_status s = explicit_check(X, y, st, &hc);
      if (s != RFM_OK) return s;
      const double rn = hc.rnorm, hn = hc.hnorm;
      if (rn == 0.0 || hc.artnorm == 0.0) { hs.stop = 4; break; }
      if (rn <= opts->btol * hn + opts->atol * anorm * hc.ynorm) { hs.stop = 1; break; }
      if (hc.artnorm <= opts->atol * anorm * rn) { hs.stop = 2; break; }
      if (budget <= 0) { hs.stop = 3; break; }
      // refinement through the narrow operator converges to A_low^T (h - A y) = 0, so once the
      // binary64 gradient stops falling the solve is finished by binary64 LSQR from y
      if (outer >= opts->max_outer || hc.artnorm > 0.5 * prev_at) { polish = true; break; }
      prev_at = hc.artnorm;
      State hi{};
      const int64_t cap = opts->max_inner < budget ? opts->max_inner : budget;
      if (outer == 0) {
        // first step: the narrow LSQR on h itself from the current y (in place), so its rule is
        // relative to ||h|| and ||y||; from y = 0 this is the correction solve on r = h
        Launcher Xh = Xl;
        Xh.h = h;
        s = run_lsqr(Xh, anorm, y, y, opts->inner_tol, opts->inner_tol, cap, opts->check_every,
                     opts->use_graph != 0, opts->times, nullptr, st, &hi);
      } else {
        s = run_lsqr(Xl, anorm, nullptr, X.W.dy, opts->inner_tol, opts->inner_tol, cap, opts->check_every,
                     opts->use_graph != 0, opts->times, nullptr, st, &hi);
        if (s == RFM_OK) {
          hipLaunchKernelGGL(axpy_inplace, dim3(ceil_div(L->ncols, 256)), dim3(256), 0, st, L->ncols, X.W.dy, y);
          RFM_LAUNCH_CHECK();
        }
      }
      if (s != RFM_OK) return s;
      inner_total += hi.iter;
      budget -= hi.iter;
    }
    int64_t polish_iters = 0;
    if (polish) {
      State hp{};
      rfm_status s = run_lsqr(X, anorm, y, y, opts->atol, opts->btol, budget, opts->check_every,
                              opts->use_graph != 0, nullptr, nullptr, st, &hp);
      if (s != RFM_OK) return s;
      s = explicit_check(X, y, st, &hc);
      if (s != RFM_OK) return s;
      polish_iters = hp.iter;
      hs.stop = hp.stop;
    }
    hs.iter = inner_total + polish_iters;
    info->polish = polish_iters;
    hs.rnorm = hc.rnorm;
    hs.artnorm = hc.artnorm;
    hs.hnorm = hc.hnorm;
    hs.ynorm = hc.ynorm;
    hs.anorm = anorm;
  }

  info->iters = hs.iter;
  info->stop = hs.stop;
  info->outer = outer;
  info->rnorm_est = hs.rnorm;
  info->artnorm_est = hs.artnorm;
  info->anorm = anorm;
  info->hnorm = hc.hnorm;
  info->ynorm = hc.ynorm;
  info->relres = hc.hnorm > 0 ? hc.rnorm / hc.hnorm : 0.0;
  info->eta = (hc.rnorm > 0 && anorm > 0) ? hc.artnorm / (anorm * hc.rnorm) : 0.0;
  return hs.stop == 3 ? RFM_ENOTCONV : RFM_OK;
}

extern "C" rfm_status rfm_coefficients(const rfm_layout *L, const int32_t *rank, const int32_t *kept,
                                       const double *R, const double *y, double *a, void *stream) {
  using namespace rfm;
  rfm_status s0 = check_layout(L, "rfm_coefficients");
  if (s0 != RFM_OK) return s0;
  if (!rank || !kept || !y || !a || (L->nrsq > 0 && !R)) return fail(RFM_EINVAL, "rfm_coefficients: null pointer");
  if (L->max_cols > 16384) return fail(RFM_EUNSUPPORTED, "rfm_coefficients: max_cols too large");
  hipLaunchKernelGGL(back_substitute, dim3(L->J), dim3(256), sizeof(double) * (L->max_cols > 0 ? L->max_cols : 1),
                     (hipStream_t)stream, *L, rank, kept, R, y, a);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}
