// Evaluation of the solution at test points and its L1 error (Sec. 4.2 performance
// evaluation): u_hat(x) = sum over the subdomains j covering x of w_j(x) phi_j(x)^T a_j
// (eq. elm_solution with the partition-of-unity windows of eq. used_window_function_nd),
// times a hard-constraint ansatz factor g(x) when the problem has one (Section 5.1), with the
// features of a depth-h network acting on its last hidden layer when depth > 1, and
// e_L1 = mean |u_hat - u| / std(u).
//
// eval_points: one thread per test point; the covering subdomains in ascending j (the
//   transpose incidence of the test-point layout), the normaliser first, then the window-
//   weighted feature sums, so u_hat does not depend on scheduling.  Per-workgroup partial
//   sums of |u_hat - u| and u.
// eval_spread: per-workgroup partial sums of (u - mean u)^2 (two-pass variance).
// eval_reduce: one workgroup, fixed-order sums of the partials.
#include <cmath>

#include "common.hpp"

namespace rfm {
namespace {

constexpr int kEvalThreads = 256;

template <int D>
__device__ __forceinline__ double window_hat(const double *xr, const double *mu, const double *hw) {
  const double pi = 3.141592653589793;
  double W = 1.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double c = 1.0 + cos(pi * ((xr[i] - mu[i]) / hw[i]));
    W *= c * c;
  }
  return W;
}

// Last hidden layer of a depth-h subdomain network at xn (values only; entries u >= H are 0).
template <int D, int ACT>
__device__ __forceinline__ void hidden_value(const rfm_problem &P, int j, const double *xn, double (&z)[kHMax]) {
  const int H = P.hidden;
  const double *net = P.net + (int64_t)j * net_stride(P, D);
#pragma unroll
  for (int u = 0; u < kHMax; ++u) {
    z[u] = 0.0;
    if (u < H) {
      double s = net[H * D + u];
#pragma unroll
      for (int a = 0; a < D; ++a) s += net[u * D + a] * xn[a];
      z[u] = activation1c<ACT, double>(s);
    }
  }
  net += H * D + H;
  for (int l = 2; l < P.depth; ++l, net += H * H + H) {
    double nz[kHMax];
#pragma unroll
    for (int u = 0; u < kHMax; ++u) {
      nz[u] = 0.0;
      if (u < H) {
        double s = net[H * H + u];
#pragma unroll
        for (int v = 0; v < kHMax; ++v)
          if (v < H) s += net[u * H + v] * z[v];
        nz[u] = activation1c<ACT, double>(s);
      }
    }
#pragma unroll
    for (int u = 0; u < kHMax; ++u) z[u] = nz[u];
  }
}

template <int D, bool DEEP, int ACT>
__global__ __launch_bounds__(kEvalThreads) void eval_points(rfm_layout L, rfm_problem P, const double *__restrict__ a,
                                                            double *__restrict__ uhat,
                                                            const double *__restrict__ ue, double *part) {
  __shared__ double red[kEvalThreads / kWave];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double err = 0.0, uv = 0.0;
  if (r < L.N) {
    double xr[D];
#pragma unroll
    for (int i = 0; i < D; ++i) xr[i] = P.x[r * D + i];
    const int64_t q0 = L.rinc_off[r], q1 = L.rinc_off[r + 1];
    double S = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t j = L.inc_blk[L.rinc[q]];
      S += window_hat<D>(xr, P.mu + (int64_t)j * D, P.hw + (int64_t)j * D);
    }
    double u = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t j = L.inc_blk[L.rinc[q]];
      const double *mu = P.mu + (int64_t)j * D, *hw = P.hw + (int64_t)j * D;
      const double w = window_hat<D>(xr, mu, hw) / S;
      double xn[D];
#pragma unroll
      for (int i = 0; i < D; ++i) xn[i] = (xr[i] - mu[i]) / hw[i];
      const int64_t f0 = L.feat_off[j], f1 = L.feat_off[j + 1];
      double acc = 0.0;
      if constexpr (DEEP) {
        double z[kHMax];
        hidden_value<D, ACT>(P, j, xn, z);
        const int H = P.hidden;
        for (int64_t k = f0; k < f1; ++k) {
          double s = P.b[k];
#pragma unroll
          for (int u = 0; u < kHMax; ++u)
            if (u < H) s += P.w[k * H + u] * z[u];
          acc += a[k] * activation1c<ACT, double>(s);
        }
      } else {
        for (int64_t k = f0; k < f1; ++k) {
          double s = P.b[k];
#pragma unroll
          for (int i = 0; i < D; ++i) s += xn[i] * P.w[k * D + i];
          acc += a[k] * activation1c<ACT, double>(s);
        }
      }
      u += w * acc;
    }
    if (P.ansatz) u *= P.ansatz[r * (1 + 2 * D)];
    uhat[r] = u;
    if (ue) {
      uv = ue[r];
      err = fabs(u - uv);
    }
  }
  if (!ue) return;
  const double se = block_sum(err, red);
  const double su = block_sum(uv, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = se;
    part[gridDim.x + blockIdx.x] = su;
  }
}

__global__ __launch_bounds__(kEvalThreads) void eval_spread(int64_t T, const double *__restrict__ ue,
                                                            const double *sums, double *part) {
  __shared__ double red[kEvalThreads / kWave];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double mean = sums[1] / (double)T;
  const double dv = (r < T) ? ue[r] - mean : 0.0;
  const double s = block_sum(dv * dv, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// sums[k] = sum_b part[k * n + b] for k < nk, fixed order (one workgroup)
__global__ __launch_bounds__(1024) void eval_reduce(const double *part, int64_t n, int nk, double *sums) {
  __shared__ double red[1024 / kWave];
  for (int k = 0; k < nk; ++k) {
    double t = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) t += part[k * n + i];
    t = block_sum(t, red);
    if (threadIdx.x == 0) sums[k] = t;
    __syncthreads();
  }
}

template <int D>
rfm_status launch_eval(const rfm_layout *L, const rfm_problem *P, const double *a, double *uhat, const double *ue,
                       double *part, double *sums, hipStream_t st) {
  const unsigned g = ceil_div(L->N, kEvalThreads);
  const bool deep = P->depth > 1;
#define RFM_EVAL(DP, ACT) \
  hipLaunchKernelGGL((eval_points<D, DP, ACT>), dim3(g), dim3(kEvalThreads), 0, st, *L, *P, a, uhat, ue, part)
  if (P->activation == RFM_ACT_SIN) {
    if (deep) RFM_EVAL(true, RFM_ACT_SIN); else RFM_EVAL(false, RFM_ACT_SIN);
  } else if (P->activation == RFM_ACT_SIGMOID) {
    if (deep) RFM_EVAL(true, RFM_ACT_SIGMOID); else RFM_EVAL(false, RFM_ACT_SIGMOID);
  } else {
    if (deep) RFM_EVAL(true, RFM_ACT_TANH); else RFM_EVAL(false, RFM_ACT_TANH);
  }
#undef RFM_EVAL
  RFM_LAUNCH_CHECK();
  if (ue) {
    hipLaunchKernelGGL(eval_reduce, dim3(1), dim3(1024), 0, st, part, (int64_t)g, 2, sums);
    hipLaunchKernelGGL(eval_spread, dim3(g), dim3(kEvalThreads), 0, st, L->N, ue, sums, part);
    hipLaunchKernelGGL(eval_reduce, dim3(1), dim3(1024), 0, st, part, (int64_t)g, 1, sums + 2);
    RFM_LAUNCH_CHECK();
  }
  return RFM_OK;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_evaluate_ws_bytes(const rfm_layout *L) {
  if (!L) return 0;
  return (4 + 2 * (size_t)rfm::ceil_div(L->N, rfm::kEvalThreads)) * sizeof(double);
}

extern "C" rfm_status rfm_evaluate(const rfm_layout *L, const rfm_problem *P, const double *a, double *uhat,
                                   const double *u_exact, double *e_l1, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s = check_layout(L, "rfm_evaluate");
  if (s != RFM_OK) return s;
  if (!P || !P->x || !P->mu || !P->hw || !P->w || !P->b || !a || !uhat)
    return fail(RFM_EINVAL, "rfm_evaluate: null pointer");
  if ((u_exact || e_l1) && (!u_exact || !e_l1)) return fail(RFM_EINVAL, "rfm_evaluate: u_exact and e_l1 go together");
  if (P->activation < RFM_ACT_TANH || P->activation > RFM_ACT_SIN)
    return fail(RFM_EINVAL, "rfm_evaluate: unknown activation");
  s = check_network(P, "rfm_evaluate");
  if (s != RFM_OK) return s;
  if (!ws || ws_bytes < rfm_evaluate_ws_bytes(L)) return fail(RFM_EINVAL, "rfm_evaluate: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  double *sums = (double *)ws, *part = sums + 4;
  switch (L->d) {
    case 1: s = launch_eval<1>(L, P, a, uhat, u_exact, part, sums, st); break;
    case 2: s = launch_eval<2>(L, P, a, uhat, u_exact, part, sums, st); break;
    default: s = launch_eval<3>(L, P, a, uhat, u_exact, part, sums, st); break;
  }
  if (s != RFM_OK || !u_exact) return s;
  double h[3];
  RFM_HIP_TRY(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, st));
  RFM_HIP_TRY(hipStreamSynchronize(st));
  const double T = (double)L->N;
  const double sd = std::sqrt(h[2] / T);
  *e_l1 = (sd > 0.0) ? (h[0] / T) / sd : INFINITY;
  return RFM_OK;
}
