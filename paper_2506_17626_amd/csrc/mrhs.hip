// LSQR for up to 64 right-hand sides at once on the same preconditioned operator
// A = sum_j V_j^T Q_hat_j W_hat_j (Q form, binary64): independent Paige-Saunders recurrences,
// one per right-hand side, whose block products share every pass over Q_hat, so the
// products become small dense matrix-matrix products per block (64 rows or columns x 64
// right-hand sides per workgroup, 16-deep slices staged in LDS, 4x4 register tiles).
//
// Vectors are stored right-hand-side-minor: entry (index, b) at index * B + b.  Every
// right-hand side has its own scalars and stopping test (the rule of rfm_lsqr_solve); a
// finished one is frozen (its y no longer changes) while the others go on.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace rfm {
namespace {

constexpr int TR = 64;     // rows (or columns) per tile
constexpr int TB = 64;     // right-hand sides per tile
constexpr int TK = 16;     // depth of the staged slice

struct MState {
  double alpha, beta, beta_next, rhobar, phibar, phi_rho, theta_rho;
  double rnorm, artnorm, ynorm, hnorm;
  int64_t iter;
  int32_t done, stop;
};

struct MGlobal {
  double anorm, atol, btol;
  int64_t maxit;
};

enum MMode : int { M_ITER = 0, M_INIT = 1, M_RESID = 2, M_COPYH = 3 };
enum MRed : int { MR_BETA = 0, MR_BETA_INIT = 1, MR_ALPHA = 2, MR_ALPHA_INIT = 3, MR_Y = 4, MR_Y_INIT = 5 };

// T[(r0+i), b] = sum_k Q_hat_j[i,k] V[(f0+k), b] * s_b with s_b = 1/alpha_b (ITER, 0 when
// frozen) or 1.
__global__ __launch_bounds__(256) void mr_fwd(rfm_layout L, const double *__restrict__ Q,
                                              const int32_t *__restrict__ rank, const double *__restrict__ V,
                                              double *__restrict__ T, int B, const MState *st, int mode) {
  __shared__ double Qs[TK][TR + 1];
  __shared__ double Vs[TK][TB + 1];
  __shared__ double sv[TB];
  const int j = blockIdx.y;
  const int64_t r0 = L.row_off[j];
  const int m = (int)(L.row_off[j + 1] - r0);
  const int i0 = blockIdx.x * TR;
  if (i0 >= m) return;
  const int64_t f0 = L.feat_off[j];
  const int r = rank[j];
  if (threadIdx.x < TB) {
    const int b = threadIdx.x;
    double s = 0.0;
    if (b < B) s = (mode == M_ITER) ? (st[b].done ? 0.0 : 1.0 / st[b].alpha) : 1.0;
    sv[b] = s;
  }
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  const double *Qj = Q + L.blk_off[j];
  for (int k0 = 0; k0 < r; k0 += TK) {
    __syncthreads();
    for (int e = threadIdx.x; e < TK * TR; e += 256) {
      const int kk = e / TR, ii = e % TR;
      const int k = k0 + kk, i = i0 + ii;
      Qs[kk][ii] = (k < r && i < m) ? Qj[(int64_t)k * m + i] : 0.0;
    }
    for (int e = threadIdx.x; e < TK * TB; e += 256) {
      const int kk = e / TB, b = e % TB;
      const int k = k0 + kk;
      Vs[kk][b] = (k < r && b < B) ? V[(f0 + k) * B + b] * sv[b] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      double a[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = Qs[kk][ty * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = Vs[kk][tx * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], v[w], acc[q][w]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ty * 4 + q;
    if (i >= m) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int b = tx * 4 + w;
      if (b < B) T[(r0 + i) * B + b] = acc[q][w];
    }
  }
}

// P[r, b] = sum_j T[(j,r), b] - alpha_b P_cur[r, b] / beta_b (ITER), H - sum (RESID), H (COPYH);
// per-workgroup partials of sum_r P^2 (and of H^2 outside ITER) for each b.
// Workgroup: 64 rows x 64 right-hand sides, thread = (b, 16-row group).
__global__ __launch_bounds__(256) void mr_gather(rfm_layout L, const double *__restrict__ T,
                                                 const double *__restrict__ Hm, const double *__restrict__ Pcur,
                                                 double *__restrict__ Pnew, int B, double *part, double *part2,
                                                 const MState *st, int mode) {
  __shared__ double red[4][TB];
  __shared__ double red2[4][TB];
  const int b = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t rbase = (int64_t)blockIdx.x * 64 + g * 16;
  double ss = 0.0, hh = 0.0;
  if (b < B) {
    const bool frozen = (mode == M_ITER) && st[b].done;
    const double a = (mode == M_ITER) ? st[b].alpha : 0.0;
    const double be = (mode == M_ITER) ? st[b].beta : 1.0;
    for (int q = 0; q < 16; ++q) {
      const int64_t r = rbase + q;
      if (r >= L.N) break;
      double s = 0.0;
      if (mode != M_COPYH) {
        const int64_t q1 = L.rinc_off[r + 1];
        for (int64_t t = L.rinc_off[r]; t < q1; ++t) s += T[L.rinc[t] * B + b];
      }
      double val;
      if (mode == M_ITER) {
        val = frozen ? 0.0 : s - a * (Pcur[r * B + b] / be);
      } else {
        const double hv = Hm[r * B + b];
        val = (mode == M_RESID) ? hv - s : hv;
        hh += hv * hv;
      }
      Pnew[r * B + b] = val;
      ss += val * val;
    }
  }
  red[g][b] = ss;
  red2[g][b] = hh;
  __syncthreads();
  if (threadIdx.x < TB && threadIdx.x < B) {
    part[(int64_t)blockIdx.x * B + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    if (mode != M_ITER)
      part2[(int64_t)blockIdx.x * B + threadIdx.x] =
          ((red2[0][threadIdx.x] + red2[1][threadIdx.x]) + red2[2][threadIdx.x]) + red2[3][threadIdx.x];
  }
}

// Z[(f0+k), b] = sum_i Q_hat_j[i,k] U[rows_i, b], U = P / beta_next_b (ITER, INIT) or P;
// Qn = Z - beta_next_b Qcur / alpha_b (ITER) or Z; per-workgroup partials of sum Qn^2 per b.
__global__ __launch_bounds__(256) void mr_adj(rfm_layout L, const double *__restrict__ Q,
                                              const int32_t *__restrict__ rank, const double *__restrict__ P,
                                              const double *__restrict__ Qcur, double *__restrict__ Qn, int B,
                                              double *part, const MState *st, int mode) {
  __shared__ double Qs[TK][TR + 1];
  __shared__ double Us[TK][TB + 1];
  __shared__ double su[TB];
  __shared__ double red[16][TB];
  const int j = blockIdx.y;
  const int r = rank[j];
  const int k0 = blockIdx.x * TR;
  const int64_t pidx = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (k0 >= r) {
    if (threadIdx.x < B) part[pidx * B + threadIdx.x] = 0.0;
    return;
  }
  const int64_t r0 = L.row_off[j];
  const int m = (int)(L.row_off[j + 1] - r0);
  const int64_t f0 = L.feat_off[j];
  if (threadIdx.x < TB) {
    const int b = threadIdx.x;
    double s = 0.0;
    if (b < B) {
      const double bn = st[b].beta_next;
      s = (mode == M_RESID) ? 1.0 : ((mode == M_ITER && st[b].done) || !(bn > 0.0) ? 0.0 : 1.0 / bn);
    }
    su[b] = s;
  }
  double acc[4][4] = {};
  const double *Qj = Q + L.blk_off[j];
  for (int i0 = 0; i0 < m; i0 += TK) {
    __syncthreads();
    for (int e = threadIdx.x; e < TK * TR; e += 256) {
      const int c = e / TK, ii = e % TK;
      const int k = k0 + c, i = i0 + ii;
      Qs[ii][c] = (k < r && i < m) ? Qj[(int64_t)k * m + i] : 0.0;
    }
    for (int e = threadIdx.x; e < TK * TB; e += 256) {
      const int ii = e / TB, b = e % TB;
      const int i = i0 + ii;
      Us[ii][b] = (i < m && b < B) ? P[(int64_t)L.rows[r0 + i] * B + b] * su[b] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < TK; ++ii) {
      double a[4], u[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = Qs[ii][ty * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q) u[q] = Us[ii][tx * 4 + q];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = fma(a[q], u[w], acc[q][w]);
    }
  }
  double ssq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = k0 + ty * 4 + q;
    if (k >= r) continue;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int b = tx * 4 + w;
      if (b >= B) continue;
      double z = acc[q][w];
      if (mode == M_ITER) {
        const bool frozen = st[b].done;
        z = frozen ? 0.0 : z - st[b].beta_next * (Qcur[(f0 + k) * B + b] / st[b].alpha);
      }
      Qn[(f0 + k) * B + b] = z;
      ssq[w] += z * z;
    }
  }
  // per-b sum over the 16 row groups (ty) in a fixed order
#pragma unroll
  for (int w = 0; w < 4; ++w) red[ty][tx * 4 + w] = ssq[w];
  __syncthreads();
  if (threadIdx.x < B) {
    double s = 0.0;
    for (int g = 0; g < 16; ++g) s += red[g][threadIdx.x];
    part[pidx * B + threadIdx.x] = s;
  }
}

// y += phi_rho w, w = v - theta_rho w with v = Qn / alpha (ITER, skipping frozen right-hand
// sides); w = Qn / alpha (INIT).  Workgroup: 64 coordinates x 64 right-hand sides.
__global__ __launch_bounds__(256) void mr_yw(int64_t n, const double *__restrict__ Qn, double *__restrict__ W,
                                             double *__restrict__ Y, int B, double *part, const MState *st,
                                             int mode) {
  __shared__ double red[4][TB];
  const int b = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t kbase = (int64_t)blockIdx.x * 64 + g * 16;
  double yy = 0.0;
  if (b < B) {
    const MState s = st[b];
    const bool frozen = (mode == M_ITER) && s.done;
    for (int q = 0; q < 16; ++q) {
      const int64_t k = kbase + q;
      if (k >= n) break;
      const int64_t e = k * B + b;
      double yk = Y[e];
      if (!frozen) {
        const double v = (s.alpha > 0.0) ? Qn[e] / s.alpha : 0.0;
        if (mode == M_ITER) {
          const double wk = W[e];
          yk = yk + s.phi_rho * wk;
          Y[e] = yk;
          W[e] = v - s.theta_rho * wk;
        } else {
          W[e] = v;
        }
      }
      yy += yk * yk;
    }
  }
  red[g][b] = yy;
  __syncthreads();
  if (threadIdx.x < B)
    part[(int64_t)blockIdx.x * B + threadIdx.x] =
        ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

// One workgroup per right-hand side: fixed-order sum of its partials and its scalar step.
__global__ __launch_bounds__(256) void mr_reduce(const double *part, const double *part2, int64_t n, int B,
                                                 MState *st, MGlobal gl, int what) {
  __shared__ double red[256 / kWave];
  const int b = blockIdx.x;
  MState &s = st[b];
  if ((what == MR_BETA || what == MR_ALPHA || what == MR_Y) && s.done) return;
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) t += part[i * B + b];
  t = block_sum(t, red);
  double t2 = 0.0;
  if (what == MR_BETA_INIT) {
    double u = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) u += part2[i * B + b];
    t2 = block_sum(u, red);
  }
  if (threadIdx.x != 0) return;
  switch (what) {
    case MR_BETA: s.beta_next = sqrt(t); break;
    case MR_BETA_INIT:
      s.beta_next = sqrt(t);
      s.hnorm = sqrt(t2);
      break;
    case MR_ALPHA_INIT: {
      const double an = sqrt(t), bn = s.beta_next;
      s.alpha = an;
      s.beta = bn;
      s.rhobar = an;
      s.phibar = bn;
      s.rnorm = bn;
      s.artnorm = an * bn;
      s.iter = 0;
      s.stop = (an == 0.0 || bn == 0.0) ? 4 : 0;
      s.done = s.stop != 0;
      break;
    }
    case MR_ALPHA: {
      const double an = sqrt(t), bn = s.beta_next;
      const double rho = hypot(s.rhobar, bn);
      const double c = s.rhobar / rho, sn = bn / rho;
      const double phi = c * s.phibar;
      s.rhobar = -c * an;
      s.phibar = sn * s.phibar;
      s.phi_rho = phi / rho;
      s.theta_rho = (sn * an) / rho;
      s.rnorm = s.phibar;
      s.artnorm = s.phibar * an * fabs(c);
      s.alpha = an;
      s.beta = bn;
      break;
    }
    case MR_Y_INIT: s.ynorm = sqrt(t); break;
    case MR_Y: {
      s.ynorm = sqrt(t);
      s.iter += 1;
      int stop = 0;
      if (s.beta == 0.0 || s.alpha == 0.0) stop = 4;
      else if (s.rnorm <= gl.btol * s.hnorm + gl.atol * gl.anorm * s.ynorm) stop = 1;
      else if (s.artnorm <= gl.atol * gl.anorm * s.rnorm) stop = 2;
      else if (s.iter >= gl.maxit) stop = 3;
      if (stop) {
        s.stop = stop;
        s.done = 1;
      }
      break;
    }
  }
}

__global__ void mr_init_y(rfm_layout L, const int32_t *rank, const double *Y0, double *Y, int B) {
  const int j = blockIdx.y;
  const int64_t f0 = L.feat_off[j];
  const int K = (int)(L.feat_off[j + 1] - f0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = e / B, b = e % B;
  if (k >= K) return;
  Y[(f0 + k) * B + b] = (Y0 && k < rank[j]) ? Y0[(f0 + k) * B + b] : 0.0;
}

// zero the columns b of Y whose bit is set in mask (starts discarded by the warm-start guard)
__global__ void mr_drop_start(int64_t ncols, int B, uint64_t mask, double *Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ncols * B && ((mask >> (e % B)) & 1ull)) Y[e] = 0.0;
}

__global__ void mr_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

struct MWork {
  double *t, *p[2], *q[2], *w, *part, *part2;
  MState *st;
  int64_t npart;
};

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

size_t mcarve(const rfm_layout *L, int B, char *base, MWork *W) {
  const int64_t g_rows = (L->N + 63) / 64, g_cols = (L->ncols + 63) / 64;
  const int64_t g_adj = (int64_t)L->J * ((L->max_cols > 0 ? L->max_cols : 1) + TR - 1) / TR;
  int64_t np = g_rows;
  if (g_cols > np) np = g_cols;
  if (g_adj > np) np = g_adj;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += al(bytes);
    return p;
  };
  MWork w{};
  w.t = (double *)take(sizeof(double) * (size_t)L->nnz_rows * B);
  w.p[0] = (double *)take(sizeof(double) * (size_t)L->N * B);
  w.p[1] = (double *)take(sizeof(double) * (size_t)L->N * B);
  w.q[0] = (double *)take(sizeof(double) * (size_t)L->ncols * B);
  w.q[1] = (double *)take(sizeof(double) * (size_t)L->ncols * B);
  w.w = (double *)take(sizeof(double) * (size_t)L->ncols * B);
  w.part = (double *)take(sizeof(double) * (size_t)np * B);
  w.part2 = (double *)take(sizeof(double) * (size_t)np * B);
  w.st = (MState *)take(sizeof(MState) * 64);
  w.npart = np;
  if (W) *W = w;
  return off;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_lsqr_multi_ws_bytes(const rfm_layout *L, int32_t nrhs) {
  if (!L || nrhs < 1 || nrhs > 64) return 0;
  return rfm::mcarve(L, nrhs, nullptr, nullptr);
}

extern "C" rfm_status rfm_lsqr_multi(const rfm_layout *L, const rfm_operator *A, const double *H, int32_t nrhs,
                                     const double *Y0, const rfm_lsqr_opts *opts, double *Y, int64_t *iters,
                                     int32_t *stops, int32_t *rejected, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s0 = check_layout(L, "rfm_lsqr_multi");
  if (s0 != RFM_OK) return s0;
  if (!A || A->form != RFM_FORM_Q || !A->rank || (L->nnz > 0 && !A->Q))
    return fail(RFM_EINVAL, "rfm_lsqr_multi: needs the Q form operator");
  if (!H || !Y || !opts || nrhs < 1 || nrhs > 64) return fail(RFM_EINVAL, "rfm_lsqr_multi: bad arguments");
  if (opts->maxit < 1 || opts->check_every < 1) return fail(RFM_EINVAL, "rfm_lsqr_multi: bad options");
  if (!ws || ws_bytes < rfm_lsqr_multi_ws_bytes(L, nrhs)) return fail(RFM_EINVAL, "rfm_lsqr_multi: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const int B = nrhs;
  MWork W;
  mcarve(L, B, (char *)ws, &W);
  std::vector<int32_t> hrank(L->J);
  RFM_HIP_TRY(hipMemcpyAsync(hrank.data(), A->rank, sizeof(int32_t) * L->J, hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));
  double nr = 0.0;
  for (int32_t j = 0; j < L->J; ++j) nr += hrank[j];
  MGlobal gl{std::sqrt(nr), opts->atol, opts->btol, opts->maxit};

  const unsigned g_rows = ceil_div(L->N, 64), g_cols = ceil_div(L->ncols, 64);
  const dim3 g_fwd(ceil_div(L->max_rows > 0 ? L->max_rows : 1, TR), L->J);
  const dim3 g_adj(ceil_div(L->max_cols > 0 ? L->max_cols : 1, TR), L->J);
  const int64_t n_adj = (int64_t)g_adj.x * L->J;
  const int64_t nvec = L->ncols * (int64_t)B;
  for (double *b : {W.q[0], W.q[1], W.w})
    hipLaunchKernelGGL(mr_zero, dim3(ceil_div(nvec, 256)), dim3(256), 0, st, b, nvec);
  hipLaunchKernelGGL(mr_zero, dim3(1), dim3(256), 0, st, (double *)W.st, (int64_t)(sizeof(MState) * 64 / sizeof(double)));
  hipLaunchKernelGGL(mr_init_y, dim3(ceil_div((int64_t)(L->max_cols > 0 ? L->max_cols : 1) * B, 256), L->J), dim3(256),
                     0, st, *L, A->rank, Y0, Y, B);
  // r0 = H - A Y0 (or H), beta u = r0, alpha v = A^T u, w = v
  auto residual = [&]() {
    hipLaunchKernelGGL(mr_fwd, g_fwd, dim3(256), 0, st, *L, A->Q, A->rank, Y, W.t, B, W.st, (int)M_RESID);
    hipLaunchKernelGGL(mr_gather, dim3(g_rows), dim3(256), 0, st, *L, W.t, H, (const double *)nullptr, W.p[0], B,
                       W.part, W.part2, W.st, (int)M_RESID);
    hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, (int64_t)g_rows, B, W.st, gl,
                       (int)MR_BETA_INIT);
  };
  std::vector<MState> hs(B);
  if (rejected)
    for (int b = 0; b < B; ++b) rejected[b] = 0;
  if (Y0) {
    // warm-start guard, per right-hand side: a start whose residual exceeds ||h_b|| is replaced
    // by the zero start (the rule of rfm_lsqr_solve)
    residual();
    RFM_LAUNCH_CHECK();
    RFM_HIP_TRY(hipMemcpyAsync(hs.data(), W.st, sizeof(MState) * B, hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    uint64_t mask = 0;
    for (int b = 0; b < B; ++b)
      if (hs[b].beta_next > hs[b].hnorm) {
        mask |= 1ull << b;
        if (rejected) rejected[b] = 1;
      }
    if (mask) {
      hipLaunchKernelGGL(mr_drop_start, dim3(ceil_div(nvec, 256)), dim3(256), 0, st, L->ncols, B, mask, Y);
      residual();
    }
  } else {
    hipLaunchKernelGGL(mr_gather, dim3(g_rows), dim3(256), 0, st, *L, W.t, H, (const double *)nullptr, W.p[0], B,
                       W.part, W.part2, W.st, (int)M_COPYH);
    hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, (int64_t)g_rows, B, W.st, gl,
                       (int)MR_BETA_INIT);
  }
  hipLaunchKernelGGL(mr_adj, g_adj, dim3(256), 0, st, *L, A->Q, A->rank, W.p[0], (const double *)nullptr, W.q[0], B,
                     W.part, W.st, (int)M_INIT);
  hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, n_adj, B, W.st, gl, (int)MR_ALPHA_INIT);
  hipLaunchKernelGGL(mr_yw, dim3(g_cols), dim3(256), 0, st, L->ncols, W.q[0], W.w, Y, B, W.part, W.st, (int)M_INIT);
  hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, (int64_t)g_cols, B, W.st, gl,
                     (int)MR_Y_INIT);
  RFM_LAUNCH_CHECK();
  int64_t i = 0;
  for (;;) {
    RFM_HIP_TRY(hipMemcpyAsync(hs.data(), W.st, sizeof(MState) * B, hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    bool all = true;
    for (int b = 0; b < B; ++b) all = all && hs[b].done;
    if (all || i >= opts->maxit) break;
    for (int c = 0; c < opts->check_every && i < opts->maxit; ++c) {
      ++i;
      const int a = (int)((i - 1) & 1), b = (int)(i & 1);
      hipLaunchKernelGGL(mr_fwd, g_fwd, dim3(256), 0, st, *L, A->Q, A->rank, W.q[a], W.t, B, W.st, (int)M_ITER);
      hipLaunchKernelGGL(mr_gather, dim3(g_rows), dim3(256), 0, st, *L, W.t, (const double *)nullptr, W.p[a], W.p[b],
                         B, W.part, W.part2, W.st, (int)M_ITER);
      hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, (int64_t)g_rows, B, W.st, gl,
                         (int)MR_BETA);
      hipLaunchKernelGGL(mr_adj, g_adj, dim3(256), 0, st, *L, A->Q, A->rank, W.p[b], W.q[a], W.q[b], B, W.part, W.st,
                         (int)M_ITER);
      hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, n_adj, B, W.st, gl, (int)MR_ALPHA);
      hipLaunchKernelGGL(mr_yw, dim3(g_cols), dim3(256), 0, st, L->ncols, W.q[b], W.w, Y, B, W.part, W.st,
                         (int)M_ITER);
      hipLaunchKernelGGL(mr_reduce, dim3(B), dim3(256), 0, st, W.part, W.part2, (int64_t)g_cols, B, W.st, gl,
                         (int)MR_Y);
    }
    RFM_LAUNCH_CHECK();
  }
  for (int b = 0; b < B; ++b) {
    if (iters) iters[b] = hs[b].iter;
    if (stops) stops[b] = hs[b].done ? hs[b].stop : 3;
  }
  bool all = true;
  for (int b = 0; b < B; ++b) all = all && hs[b].done && hs[b].stop != 3;
  return all ? RFM_OK : RFM_ENOTCONV;
}
