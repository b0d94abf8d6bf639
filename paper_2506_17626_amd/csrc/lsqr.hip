// Right-preconditioned LSQR on the block-sparse system (Algorithm 2, Proposition 3.1)
// on gfx950, and the back-substitution a = S^{-1} y.
//
// Operator A = sum_j V_j^T Q_hat_j W_hat_j (Q form).  Vectors over columns use the
// padded per-feature layout (entry (j,k) at feat_off[j] + k, k < r_j; the rest stay 0).
//
// One LSQR iteration = four launches on the caller's stream:
//   fwd_local   t_(j,i) = sum_k Q_hat_j[i,k] v_j[k]       lane <-> row, coalesced column reads
//   fwd_gather  p_r = sum_{j covering r} t_(j,r) - alpha u_r, summed in ascending j (no
//               atomics, so the result does not depend on scheduling); ||p||^2 partials
//   adj_local   z_j = Q_hat_j^T (p / beta) restricted to I_j (rows gathered to LDS once per
//               block), q = z - beta v; ||q||^2 partials; the last workgroup finishes the
//               norm and does the Givens-rotation scalar step of Paige and Saunders
//   yw_update   y += (phi/rho) w, w = v - (theta/rho) w; ||y||^2; the last workgroup
//               applies the stopping rule and raises the done flag
// Grid-wide norms are finished by the last workgroup to arrive (threadfence + counter),
// summing the per-workgroup partials in a fixed order.  After the done flag is up every
// kernel returns at once, so the host may launch iterations in batches and only reads
// the scalar state between batches.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace rfm {
namespace {

struct State {
  double alpha, beta;      // alpha_i, beta_i of u_i = p/beta_i, v_i = q/alpha_i
  double beta_next;        // beta_{i+1} from the forward gather
  double rhobar, phibar;
  double phi_rho, theta_rho;
  double rnorm, artnorm, ynorm, hnorm, anorm;
  double atol, btol;
  int64_t iter, maxit;
  int32_t done, stop;
};

enum Mode : int { ITER = 0, INIT = 1, RESID = 2, COPYH = 3 };

constexpr int kRowTile = 256;
constexpr int kAdjThreads = 512;
constexpr int kVecThreads = 256;

__global__ void fill_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void fill_zero_u32(unsigned *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
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

// t_(j,i) = sum_k Q_hat_j[i,k] * v_j[k], v = vin / alpha (ITER) or vin (otherwise).
__global__ __launch_bounds__(kRowTile) void fwd_local(rfm_layout L, const double *__restrict__ Q,
                                                      const int32_t *__restrict__ rank,
                                                      const double *__restrict__ vin,
                                                      double *__restrict__ t, const State *st,
                                                      int mode) {
  extern __shared__ double vs[];
  if (mode == ITER && st->done) return;
  const int j = blockIdx.y;
  const int64_t r0 = L.row_off[j];
  const int m = (int)(L.row_off[j + 1] - r0);
  if ((int)blockIdx.x * kRowTile >= m) return;
  const int64_t f0 = L.feat_off[j];
  const int r = rank[j];
  const double alpha = (mode == ITER) ? st->alpha : 1.0;
  for (int k = threadIdx.x; k < r; k += kRowTile) vs[k] = (mode == ITER) ? vin[f0 + k] / alpha : vin[f0 + k];
  __syncthreads();
  const int i = blockIdx.x * kRowTile + threadIdx.x;
  if (i >= m) return;
  const double *__restrict__ q = Q + L.blk_off[j] + i;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  int k = 0;
  for (; k + 4 <= r; k += 4) {
    acc0 += q[(int64_t)k * m] * vs[k];
    acc1 += q[(int64_t)(k + 1) * m] * vs[k + 1];
    acc2 += q[(int64_t)(k + 2) * m] * vs[k + 2];
    acc3 += q[(int64_t)(k + 3) * m] * vs[k + 3];
  }
  for (; k < r; ++k) acc0 += q[(int64_t)k * m] * vs[k];
  t[r0 + i] = (acc0 + acc1) + (acc2 + acc3);
}

// p_r = sum_j t_(j,r) - alpha * (pcur_r / beta)     (ITER)
// p_r = h_r - sum_j t_(j,r)                         (RESID)
// p_r = h_r                                         (COPYH)
__global__ __launch_bounds__(kVecThreads) void fwd_gather(rfm_layout L, const double *__restrict__ t,
                                                          const double *__restrict__ h,
                                                          const double *__restrict__ pcur,
                                                          double *__restrict__ pnew, double *part,
                                                          unsigned *counter, State *st, int mode) {
  __shared__ double red[kVecThreads / kWave];
  __shared__ int last_flag;
  if (mode == ITER && st->done) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double val = 0.0, hh = 0.0;
  if (r < L.N) {
    double s = 0.0;
    if (mode != COPYH) {
      const int64_t q1 = L.rinc_off[r + 1];
      for (int64_t q = L.rinc_off[r]; q < q1; ++q) s += t[L.rinc[q]];
    }
    if (mode == ITER) {
      val = s - st->alpha * (pcur[r] / st->beta);
    } else {
      const double hr = h[r];
      val = (mode == RESID) ? hr - s : hr;
      hh = hr * hr;
    }
    pnew[r] = val;
  }
  const double bs = block_sum(val * val, red);
  const double bh = (mode == ITER) ? 0.0 : block_sum(hh, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bs;
    if (mode != ITER) part[gridDim.x + blockIdx.x] = bh;
  }
  if (!arrive_last(counter, gridDim.x, &last_flag)) return;
  const double tot = sum_partials(part, gridDim.x, red);
  const double toth = (mode == ITER) ? 0.0 : sum_partials(part + gridDim.x, gridDim.x, red);
  if (threadIdx.x == 0) {
    st->beta_next = sqrt(tot);
    if (mode != ITER) st->hnorm = sqrt(toth);
  }
}

// z_j = Q_hat_j^T u_{I_j} with u = pnew / beta_next (ITER, INIT) or pnew (RESID);
// q = z - beta_next * (qcur / alpha) (ITER), q = z (otherwise).  One workgroup per block.
__global__ __launch_bounds__(kAdjThreads) void adj_local(rfm_layout L, const double *__restrict__ Q,
                                                         const int32_t *__restrict__ rank,
                                                         const double *__restrict__ pnew,
                                                         const double *__restrict__ qcur,
                                                         double *__restrict__ qnew, double *part,
                                                         unsigned *counter, State *st, int mode) {
  extern __shared__ double us[];
  __shared__ double red[kAdjThreads / kWave];
  __shared__ double colsum[kAdjThreads / kWave];
  __shared__ int last_flag;
  if (mode == ITER && st->done) return;
  const int j = blockIdx.x;
  const int64_t r0 = L.row_off[j];
  const int m = (int)(L.row_off[j + 1] - r0);
  const int64_t f0 = L.feat_off[j];
  const int r = rank[j];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  constexpr int NW = kAdjThreads / kWave;
  const double bn = st->beta_next;
  const double alpha = st->alpha;
  double ssq = 0.0;
  if (r > 0) {
    for (int i = threadIdx.x; i < m; i += kAdjThreads) {
      const double p = pnew[L.rows[r0 + i]];
      us[i] = (mode == RESID) ? p : (bn > 0.0 ? p / bn : 0.0);
    }
    __syncthreads();
    const double *__restrict__ Qj = Q + L.blk_off[j];
    for (int k = 2 * wid; k < r; k += 2 * NW) {
      const bool two = (k + 1 < r);
      const double *__restrict__ c0 = Qj + (int64_t)k * m;
      const double *__restrict__ c1 = Qj + (int64_t)(two ? k + 1 : k) * m;
      double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
      int i = lane;
      for (; i + kWave < m; i += 2 * kWave) {
        const double u0 = us[i], u1 = us[i + kWave];
        a0 += c0[i] * u0;
        b0 += c1[i] * u0;
        a1 += c0[i + kWave] * u1;
        b1 += c1[i + kWave] * u1;
      }
      if (i < m) {
        a0 += c0[i] * us[i];
        b0 += c1[i] * us[i];
      }
      const double z0 = wave_sum(a0 + a1);
      const double z1 = wave_sum(b0 + b1);
      if (lane == 0) {
        double q0 = z0, q1 = z1;
        if (mode == ITER) {
          q0 = z0 - bn * (qcur[f0 + k] / alpha);
          if (two) q1 = z1 - bn * (qcur[f0 + k + 1] / alpha);
        }
        qnew[f0 + k] = q0;
        ssq += q0 * q0;
        if (two) {
          qnew[f0 + k + 1] = q1;
          ssq += q1 * q1;
        }
      }
    }
  }
  // per-workgroup partial (lane 0 of each wave holds its columns' sum of squares)
  if (lane == 0) colsum[wid] = ssq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += colsum[w];
    part[blockIdx.x] = s;
  }
  if (!arrive_last(counter, gridDim.x, &last_flag)) return;
  const double tot = sum_partials(part, gridDim.x, red);
  if (threadIdx.x != 0) return;
  const double an = sqrt(tot);
  if (mode == RESID) {
    st->artnorm = an;
    st->rnorm = st->beta_next;
    return;
  }
  if (mode == INIT) {
    st->alpha = an;
    st->beta = bn;
    st->rhobar = an;
    st->phibar = bn;
    st->rnorm = bn;
    st->artnorm = an * bn;
    st->iter = 0;
    st->stop = 0;
    st->done = (an == 0.0 || bn == 0.0) ? 1 : 0;
    if (st->done) st->stop = 4;
    return;
  }
  // Givens rotation eliminating beta_{i+1} (Paige-Saunders recurrences)
  const double rho = hypot(st->rhobar, bn);
  const double c = st->rhobar / rho;
  const double s = bn / rho;
  const double theta = s * an;
  const double phi = c * st->phibar;
  st->rhobar = -c * an;
  st->phibar = s * st->phibar;
  st->phi_rho = phi / rho;
  st->theta_rho = theta / rho;
  st->rnorm = st->phibar;
  st->artnorm = st->phibar * an * fabs(c);
  st->alpha = an;
  st->beta = bn;
}

// ITER: y += (phi/rho) w ; w = v - (theta/rho) w with v = q / alpha; stop test.
// INIT: w = q / alpha ; ||y||.
__global__ __launch_bounds__(kVecThreads) void yw_update(int64_t n, const double *__restrict__ qnew,
                                                         double *__restrict__ w,
                                                         double *__restrict__ y, double *part,
                                                         unsigned *counter, State *st, int mode) {
  __shared__ double red[kVecThreads / kWave];
  __shared__ int last_flag;
  if (st->done && mode == ITER) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = st->alpha;
  double yy = 0.0;
  if (k < n) {
    const double v = (a > 0.0) ? qnew[k] / a : 0.0;
    if (mode == ITER) {
      const double wk = w[k];
      const double yk = y[k] + st->phi_rho * wk;
      y[k] = yk;
      w[k] = v - st->theta_rho * wk;
      yy = yk * yk;
    } else {
      w[k] = v;
      yy = y[k] * y[k];
    }
  }
  const double bs = block_sum(yy, red);
  if (threadIdx.x == 0) part[blockIdx.x] = bs;
  if (!arrive_last(counter, gridDim.x, &last_flag)) return;
  const double tot = sum_partials(part, gridDim.x, red);
  if (threadIdx.x != 0) return;
  st->ynorm = sqrt(tot);
  if (mode != ITER) return;
  st->iter += 1;
  int stop = 0;
  if (st->beta == 0.0 || st->alpha == 0.0) stop = 4;
  else if (st->rnorm <= st->btol * st->hnorm + st->atol * st->anorm * st->ynorm) stop = 1;
  else if (st->artnorm <= st->atol * st->anorm * st->rnorm) stop = 2;
  else if (st->iter >= st->maxit) stop = 3;
  if (stop) {
    st->stop = stop;
    st->done = 1;
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

struct Work {
  double *t, *p[2], *res, *q[2], *w, *z, *part;
  State *st, *st2;
  unsigned *counter;
  int64_t npart;
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t carve(const rfm_layout *L, char *base, Work *W) {
  const int64_t N = L->N, nc = L->ncols;
  const int64_t g_rows = (N + kVecThreads - 1) / kVecThreads;
  const int64_t g_cols = (nc + kVecThreads - 1) / kVecThreads;
  int64_t npart = 2 * g_rows;
  if (g_cols > npart) npart = g_cols;
  if (L->J > npart) npart = L->J;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  Work w{};
  w.t = (double *)take(sizeof(double) * (size_t)L->nnz_rows);
  w.p[0] = (double *)take(sizeof(double) * N);
  w.p[1] = (double *)take(sizeof(double) * N);
  w.res = (double *)take(sizeof(double) * N);
  w.q[0] = (double *)take(sizeof(double) * nc);
  w.q[1] = (double *)take(sizeof(double) * nc);
  w.w = (double *)take(sizeof(double) * nc);
  w.z = (double *)take(sizeof(double) * nc);
  w.part = (double *)take(sizeof(double) * npart);
  w.st = (State *)take(sizeof(State));
  w.st2 = (State *)take(sizeof(State));
  w.counter = (unsigned *)take(sizeof(unsigned) * 64);
  w.npart = npart;
  if (W) *W = w;
  return off;
}

struct Launcher {
  const rfm_layout *L;
  const rfm_operator *A;
  const double *h;
  Work W;
  hipStream_t st;

  size_t adj_lds() const { return sizeof(double) * (size_t)(L->max_rows > 0 ? L->max_rows : 1); }
  size_t fwd_lds() const { return sizeof(double) * (size_t)(L->max_cols > 0 ? L->max_cols : 1); }

  void fwd(const double *vin, State *s, int mode) {
    if (L->max_rows > 0)
      hipLaunchKernelGGL(fwd_local, dim3(ceil_div(L->max_rows, kRowTile), L->J), dim3(kRowTile),
                         fwd_lds(), st, *L, A->Q, A->rank, vin, W.t, s, mode);
  }
  void gather(const double *pcur, double *pnew, State *s, int mode) {
    hipLaunchKernelGGL(fwd_gather, dim3(ceil_div(L->N, kVecThreads)), dim3(kVecThreads), 0, st, *L,
                       W.t, h, pcur, pnew, W.part, W.counter, s, mode);
  }
  void adj(const double *pnew, const double *qcur, double *qnew, State *s, int mode) {
    hipLaunchKernelGGL(adj_local, dim3(L->J), dim3(kAdjThreads), adj_lds(), st, *L, A->Q, A->rank,
                       pnew, qcur, qnew, W.part, W.counter, s, mode);
  }
  void yw(const double *qnew, double *y, State *s, int mode) {
    hipLaunchKernelGGL(yw_update, dim3(ceil_div(L->ncols, kVecThreads)), dim3(kVecThreads), 0, st,
                       L->ncols, qnew, W.w, y, W.part, W.counter, s, mode);
  }
  // ev (nullable): 5 events recorded around the four launches
  void iteration(int64_t i, double *y, hipEvent_t *ev) {
    const int a = (int)((i - 1) & 1), b = (int)(i & 1);
    if (ev) hipEventRecord(ev[0], st);
    fwd(W.q[a], W.st, ITER);
    if (ev) hipEventRecord(ev[1], st);
    gather(W.p[a], W.p[b], W.st, ITER);
    if (ev) hipEventRecord(ev[2], st);
    adj(W.p[b], W.q[a], W.q[b], W.st, ITER);
    if (ev) hipEventRecord(ev[3], st);
    yw(W.q[b], y, W.st, ITER);
    if (ev) hipEventRecord(ev[4], st);
  }
};

struct EventPool {
  std::vector<hipEvent_t> ev;
  ~EventPool() {
    for (hipEvent_t e : ev) hipEventDestroy(e);
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

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_lsqr_ws_bytes(const rfm_layout *L) {
  if (!L) return 0;
  return rfm::carve(L, nullptr, nullptr);
}

extern "C" rfm_status rfm_lsqr_solve(const rfm_layout *L, const rfm_operator *A, const double *h,
                                     const double *y0, const rfm_lsqr_opts *opts, double *y,
                                     rfm_lsqr_info *info, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s0 = check_layout(L, "rfm_lsqr_solve");
  if (s0 != RFM_OK) return s0;
  if (!A || !A->rank || !opts || !h || !y || !info) return fail(RFM_EINVAL, "rfm_lsqr_solve: null pointer");
  if (A->form != RFM_FORM_Q) return fail(RFM_EUNSUPPORTED, "rfm_lsqr_solve: only the Q form is built");
  if (L->nnz > 0 && !A->Q) return fail(RFM_EINVAL, "rfm_lsqr_solve: null Q");
  if (opts->maxit < 1 || opts->check_every < 1 || !(opts->atol >= 0) || !(opts->btol >= 0))
    return fail(RFM_EINVAL, "rfm_lsqr_solve: bad options");
  if (ws_bytes < rfm_lsqr_ws_bytes(L) || !ws) return fail(RFM_EINVAL, "rfm_lsqr_solve: workspace too small");
  if ((size_t)L->max_rows * sizeof(double) > 120 * 1024)
    return fail(RFM_EUNSUPPORTED, "rfm_lsqr_solve: max_rows too large for LDS staging");
  hipStream_t st = (hipStream_t)stream;

  Launcher X;
  X.L = L;
  X.A = A;
  X.h = h;
  X.st = st;
  carve(L, (char *)ws, &X.W);

  // ||A||_F = sqrt(sum_j r_j): the Q form has unit-norm columns
  std::vector<int32_t> hrank(L->J);
  RFM_HIP_TRY(hipMemcpyAsync(hrank.data(), A->rank, sizeof(int32_t) * L->J, hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));
  double nr = 0.0;
  for (int32_t j = 0; j < L->J; ++j) nr += hrank[j];

  State hs{};
  hs.anorm = std::sqrt(nr);
  hs.atol = opts->atol;
  hs.btol = opts->btol;
  hs.maxit = opts->maxit;
  RFM_HIP_TRY(hipMemcpyAsync(X.W.st, &hs, sizeof(State), hipMemcpyHostToDevice, st));
  RFM_HIP_TRY(hipMemcpyAsync(X.W.st2, &hs, sizeof(State), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(fill_zero_u32, dim3(1), dim3(64), 0, st, X.W.counter, 64);
  for (double *b : {X.W.q[0], X.W.q[1], X.W.w, X.W.z})
    hipLaunchKernelGGL(fill_zero, dim3(ceil_div(L->ncols, 256)), dim3(256), 0, st, b, L->ncols);
  if (L->max_cols > 0)
    hipLaunchKernelGGL(init_y, dim3(ceil_div(L->max_cols, 256), L->J), dim3(256), 0, st, *L, A->rank, y0, y);
  RFM_LAUNCH_CHECK();

  // r0 = h - A y0, beta_1 u_1 = r0, alpha_1 v_1 = A^T u_1, w_1 = v_1
  if (y0) {
    X.fwd(y, X.W.st, RESID);
    X.gather(nullptr, X.W.p[0], X.W.st, RESID);
  } else {
    X.gather(nullptr, X.W.p[0], X.W.st, COPYH);
  }
  X.adj(X.W.p[0], nullptr, X.W.q[0], X.W.st, INIT);
  X.yw(X.W.q[0], y, X.W.st, INIT);
  RFM_LAUNCH_CHECK();
  RFM_HIP_TRY(hipMemcpyAsync(&hs, X.W.st, sizeof(State), hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));

  int64_t i = 0;
  const int64_t batch = opts->check_every;
  EventPool pool;
  if (opts->times) {
    *opts->times = rfm_kernel_times{};
    RFM_HIP_TRY(pool.init((size_t)(5 * batch)));
  }
  while (!hs.done && i < opts->maxit) {
    const int64_t first = i + 1;
    for (int64_t b = 0; b < batch; ++b)
      X.iteration(++i, y, opts->times ? pool.ev.data() + 5 * b : nullptr);
    RFM_LAUNCH_CHECK();
    RFM_HIP_TRY(hipMemcpyAsync(&hs, X.W.st, sizeof(State), hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    if (opts->times) {
      // iterations first..hs.iter did work; later launches of the batch returned at once
      for (int64_t b = 0; b < batch && first + b <= hs.iter; ++b)
        for (int k = 0; k < 4; ++k) {
          float ms = 0.f;
          RFM_HIP_TRY(hipEventElapsedTime(&ms, pool.ev[5 * b + k], pool.ev[5 * b + k + 1]));
          opts->times->ms[k] += ms;
          opts->times->launches[k] += 1;
        }
    }
  }

  // explicit residuals: r = h - A y, A^T r
  X.fwd(y, X.W.st2, RESID);
  X.gather(nullptr, X.W.res, X.W.st2, RESID);
  X.adj(X.W.res, nullptr, X.W.z, X.W.st2, RESID);
  RFM_LAUNCH_CHECK();
  State hc{};
  RFM_HIP_TRY(hipMemcpyAsync(&hc, X.W.st2, sizeof(State), hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));

  info->iters = hs.iter;
  info->stop = hs.stop;
  info->rnorm_est = hs.rnorm;
  info->artnorm_est = hs.artnorm;
  info->anorm = hs.anorm;
  info->hnorm = hs.hnorm;
  info->ynorm = hs.ynorm;
  info->relres = hc.hnorm > 0 ? hc.rnorm / hc.hnorm : 0.0;
  info->eta = (hc.rnorm > 0 && hs.anorm > 0) ? hc.artnorm / (hs.anorm * hc.rnorm) : 0.0;
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
