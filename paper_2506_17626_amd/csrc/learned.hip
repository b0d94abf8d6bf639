// Learned warm start, data path and training loop: right-hand sides of a parametric family,
// targets from LSQR solutions (per-coordinate standardised), mini-batch Adam training of the
// perceptron, and decoding of its prediction into LSQR starting coordinates.
#include <cmath>
#include <utility>
#include <vector>

#include "common.hpp"

namespace rfm {
namespace {

unsigned cdv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// H[r, b] = weight[r] * rhs[r, b]  (eq. ELMFBPINN_ls row scaling, right-hand-side-minor)
__global__ void weighted_rhs(int64_t N, int B, const double *__restrict__ w, const double *__restrict__ rhs,
                             double *__restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N * B) H[e] = w[e / B] * rhs[e];
}

// out[row0 + b, k] = (float) Y[k, b]  (solutions [ncols x B] to sample rows [* x ncols])
__global__ void solutions_to_rows(int64_t ncols, int B, const double *__restrict__ Y, int64_t row0,
                                  float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ncols * B) return;
  const int64_t k = e / B;
  const int b = (int)(e % B);
  out[(row0 + b) * ncols + k] = (float)Y[e];
}

// per-column mean and standard deviation over n rows (fixed row order, binary64 sums), then
// T <- (T - mean) / sd with sd = 1 for constant columns
__global__ void col_standardize(int64_t n, int64_t cols, float *__restrict__ T, float *__restrict__ mean,
                                float *__restrict__ sd) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0, s2 = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    const double v = T[r * cols + c];
    s += v;
    s2 += v * v;
  }
  const double mu = s / (double)n;
  double var = s2 / (double)n - mu * mu;
  double d = var > 0.0 ? sqrt(var) : 0.0;
  if (!(d > 1e-30 * (fabs(mu) + 1e-300))) d = 1.0;
  mean[c] = (float)mu;
  sd[c] = (float)d;
  const float fm = (float)mu, inv = (float)(1.0 / d);
  for (int64_t r = 0; r < n; ++r) T[r * cols + c] = (T[r * cols + c] - fm) * inv;
}

// y0[k, b] = pred[b, k] * sd[k] + mean[k] on the kept coordinates, 0 elsewhere (binary64,
// right-hand-side-minor; B = 1 gives a plain vector)
__global__ void decode_start(rfm_layout L, const int32_t *__restrict__ rank, int B, const float *__restrict__ pred,
                             const float *__restrict__ mean, const float *__restrict__ sd, double *__restrict__ y0) {
  const int j = blockIdx.y;
  const int64_t f0 = L.feat_off[j];
  const int K = (int)(L.feat_off[j + 1] - f0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = e / B, b = e % B;
  if (k >= K) return;
  const int64_t col = f0 + k;
  y0[col * B + b] = (k < rank[j]) ? (double)pred[(int64_t)b * L.ncols + col] * (double)sd[col] + (double)mean[col] : 0.0;
}

}  // namespace
}  // namespace rfm

extern "C" rfm_status rfm_weighted_rhs(int64_t N, int32_t nrhs, const double *weight, const double *rhs, double *H,
                                       void *stream) {
  using namespace rfm;
  if (N < 1 || nrhs < 1 || !weight || !rhs || !H) return fail(RFM_EINVAL, "rfm_weighted_rhs: bad arguments");
  hipLaunchKernelGGL(weighted_rhs, dim3(cdv(N * nrhs, 256)), dim3(256), 0, (hipStream_t)stream, N, nrhs, weight, rhs,
                     H);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_solutions_to_rows(int64_t ncols, int32_t nrhs, const double *Y, int64_t row0, float *out,
                                            void *stream) {
  using namespace rfm;
  if (ncols < 1 || nrhs < 1 || !Y || !out || row0 < 0) return fail(RFM_EINVAL, "rfm_solutions_to_rows: bad arguments");
  hipLaunchKernelGGL(solutions_to_rows, dim3(cdv(ncols * nrhs, 256)), dim3(256), 0, (hipStream_t)stream, ncols, nrhs,
                     Y, row0, out);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_standardize_columns(int64_t n, int64_t cols, float *T, float *mean, float *sd,
                                              void *stream) {
  using namespace rfm;
  if (n < 1 || cols < 1 || !T || !mean || !sd) return fail(RFM_EINVAL, "rfm_standardize_columns: bad arguments");
  hipLaunchKernelGGL(col_standardize, dim3(cdv(cols, 256)), dim3(256), 0, (hipStream_t)stream, n, cols, T, mean, sd);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_decode_start(const rfm_layout *L, const int32_t *rank, int32_t nrhs, const float *pred,
                                       const float *mean, const float *sd, double *y0, void *stream) {
  using namespace rfm;
  rfm_status s = check_layout(L, "rfm_decode_start");
  if (s != RFM_OK) return s;
  if (nrhs < 1 || !rank || !pred || !mean || !sd || !y0) return fail(RFM_EINVAL, "rfm_decode_start: bad arguments");
  const int mc = L->max_cols > 0 ? L->max_cols : 1;
  hipLaunchKernelGGL(decode_start, dim3(cdv((int64_t)mc * nrhs, 256), L->J), dim3(256), 0, (hipStream_t)stream, *L,
                     rank, nrhs, pred, mean, sd, y0);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_mlp_train(const rfm_mlp *P, const rfm_mlp *G, const rfm_mlp *Mom, const rfm_mlp *Var,
                                    const float *X, const float *T, int64_t n, int32_t batch, int32_t epochs, float lr,
                                    uint64_t seed, int32_t *idx, float *scratch, size_t scratch_floats, void *ws,
                                    size_t ws_bytes, float *loss_history, void *stream) {
  using namespace rfm;
  if (!P || !G || !Mom || !Var || !X || !T || n < 1 || batch < 1 || batch > n || epochs < 1 || !scratch || !idx)
    return fail(RFM_EINVAL, "rfm_mlp_train: bad arguments");
  const int64_t I = P->n_in, H = P->n_hidden, O = P->n_out;
  const int64_t need = batch * (I + O + 4 * H + 2 * O) + 1 + 64;
  if ((int64_t)scratch_floats < need) return fail(RFM_EINVAL, "rfm_mlp_train: scratch too small");
  hipStream_t st = (hipStream_t)stream;
  float *Xb = scratch, *Tb = Xb + batch * I, *H1 = Tb + batch * O, *H2 = H1 + batch * H, *Y = H2 + batch * H;
  float *dY = Y + batch * O, *dH1 = dY + batch * O, *dH2 = dH1 + batch * H, *loss = dH2 + batch * H;
  int32_t *dev_idx = idx;
  std::vector<int32_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  uint64_t state = seed * 0x9E3779B97F4A7C15ull + 1;
  auto next = [&]() {  // splitmix64
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int64_t sizes[6] = {I * H, H, H * H, H, H * O, O};
  float *pp[6] = {P->W1, P->b1, P->W2, P->b2, P->W3, P->b3};
  float *gg[6] = {G->W1, G->b1, G->W2, G->b2, G->W3, G->b3};
  float *mm[6] = {Mom->W1, Mom->b1, Mom->W2, Mom->b2, Mom->W3, Mom->b3};
  float *vv[6] = {Var->W1, Var->b1, Var->W2, Var->b2, Var->W3, Var->b3};
  int32_t step = 0;
  rfm_status s = RFM_OK;
  std::vector<float> hl;
  for (int32_t ep = 0; ep < epochs && s == RFM_OK; ++ep) {
    for (int64_t i = n - 1; i > 0; --i) {  // Fisher-Yates shuffle of the sample order
      const int64_t k = (int64_t)(next() % (uint64_t)(i + 1));
      std::swap(perm[i], perm[k]);
    }
    RFM_HIP_TRY(hipMemcpyAsync(dev_idx, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    double ep_loss = 0.0;
    int64_t nb = 0;
    for (int64_t b0 = 0; b0 + batch <= n && s == RFM_OK; b0 += batch) {
      if ((s = rfm_gather_rows(batch, (int32_t)I, dev_idx + b0, X, Xb, stream)) != RFM_OK) break;
      if ((s = rfm_gather_rows(batch, (int32_t)O, dev_idx + b0, T, Tb, stream)) != RFM_OK) break;
      if ((s = rfm_mlp_forward(P, Xb, batch, H1, H2, Y, stream)) != RFM_OK) break;
      if ((s = rfm_mlp_backward(P, G, Xb, H1, H2, Y, Tb, batch, dY, dH1, dH2, loss, ws, ws_bytes, stream)) != RFM_OK)
        break;
      ++step;
      for (int q = 0; q < 6 && s == RFM_OK; ++q)
        s = rfm_adam_step(sizes[q], pp[q], gg[q], mm[q], vv[q], lr, 0.9f, 0.999f, 1e-8f, step, stream);
      float hlv = 0.f;
      if (loss_history && hipMemcpyAsync(&hlv, loss, sizeof(float), hipMemcpyDeviceToHost, st) == hipSuccess &&
          hipStreamSynchronize(st) == hipSuccess) {
        ep_loss += hlv;
        ++nb;
      }
    }
    if (loss_history) loss_history[ep] = nb ? (float)(ep_loss / nb) : NAN;
  }
  return s;
}
