// Learned warm start: a 3-layer MLP (n_in -> H -> H -> n_out, tanh hidden layers, linear
// output) trained with MSE loss and Adam, binary32, hand-written kernels for gfx950.
//
// gemm_f32: C = op(A) op(B) over row-major matrices, 64x64 output tiles, 256 threads with
// 4x4 register micro-tiles, 16-deep k slices staged in LDS; fused epilogue (bias, tanh) or
// split-K partials (summed afterwards in a fixed order, so results do not depend on
// scheduling).  The other kernels are elementwise or column reductions.
#include <cmath>
#include <vector>

#include "common.hpp"

namespace rfm {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

enum Epi : int { E_STORE = 0, E_BIAS = 1, E_BIAS_TANH = 2 };

// C[M x N] (+)= op(A)[M x K] op(B)[K x N]; op(A)[m,k] = ta ? A[k*lda+m] : A[m*lda+k],
// op(B)[k,n] = tb ? B[n*ldb+k] : B[k*ldb+n].  With split-K (gridDim.z > 1) slice z covers
// k in [z*kchunk, (z+1)*kchunk) and writes C + z*M*N (no epilogue).
__global__ __launch_bounds__(256) void gemm_f32(int M, int N, int K, const float *__restrict__ A, int lda, int ta,
                                                const float *__restrict__ B, int ldb, int tb, float *__restrict__ C,
                                                int ldc, const float *__restrict__ bias, int epi, int kchunk) {
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  float acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // stage op(A)[m0:m0+64, k0:k0+16] and op(B)[k0:k0+16, n0:n0+64]: 1024 values each
    for (int e = threadIdx.x; e < BM * BK; e += 256) {
      int mm, kk;
      if (ta) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
      const int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < kend) v = ta ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk];
      As[kk][mm] = v;
    }
    for (int e = threadIdx.x; e < BK * BN; e += 256) {
      int kk, nn;
      if (tb) { kk = e % BK; nn = e / BK; } else { nn = e % BN; kk = e / BN; }
      const int gk = k0 + kk, gn = n0 + nn;
      float v = 0.f;
      if (gn < N && gk < kend) v = tb ? B[(int64_t)gn * ldb + gk] : B[(int64_t)gk * ldb + gn];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] = Bs[kk][tx * 4 + i];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = fmaf(a[i], b[jj], acc[i][jj]);
    }
    __syncthreads();
  }
  float *Cz = C + (int64_t)blockIdx.z * M * ldc;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int gn = n0 + tx * 4 + jj;
      if (gn >= N) continue;
      float v = acc[i][jj];
      if (gridDim.z == 1) {
        if (epi >= E_BIAS) v += bias[gn];
        if (epi == E_BIAS_TANH) v = tanhf(v);
      }
      Cz[(int64_t)gm * ldc + gn] = v;
    }
  }
}

// C = sum over z of the split-K partials, in z order.
__global__ void sum_splits(int64_t n, int splits, const float *__restrict__ part, float *__restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * n + e];
  C[e] = s;
}

// dY = 2 (Y - T) / (batch * n_out); per-block partial sums of (Y - T)^2.
__global__ __launch_bounds__(256) void mse_grad(int64_t n, float scale, const float *__restrict__ Y,
                                                const float *__restrict__ T, float *__restrict__ dY,
                                                double *part) {
  __shared__ double red[256 / kWave];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (e < n) {
    const float d = Y[e] - T[e];
    dY[e] = 2.f * d * scale;
    sq = (double)d * (double)d;
  }
  const double s = block_sum(sq, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void finish_loss(const double *part, int64_t n, double scale, float *loss) {
  __shared__ double red[1024 / kWave];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *loss = (float)(s * scale);
}

// dZ = dH * (1 - H^2) (tanh derivative through the stored activation)
__global__ void tanh_back(int64_t n, const float *__restrict__ H, float *__restrict__ dH) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dH[e] = dH[e] * (1.f - H[e] * H[e]);
}

// db[n] = sum over rows of dZ[:, n] (fixed row order)
__global__ void col_sum(int rows, int cols, const float *__restrict__ dZ, float *__restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += dZ[(int64_t)r * cols + c];
  db[c] = s;
}

__global__ void adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                     float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// rows of a sample matrix in a given order: out[i, :] = in[idx[i], :]
__global__ void gather_rows(int rows, int cols, const int32_t *__restrict__ idx, const float *__restrict__ in,
                            float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e / cols), c = (int)(e % cols);
  out[e] = in[(int64_t)idx[r] * cols + c];
}

unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

struct Gemm {
  hipStream_t st;
  float *split_buf;      // >= splits * M * N floats when split-K is used
  int64_t split_cap;
  rfm_status run(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb, float *C,
                 int ldc, const float *bias, int epi) {
    // split K when the output tiles alone cannot fill the chip
    const int64_t tiles = (int64_t)cdiv(M, BM) * cdiv(N, BN);
    int splits = 1;
    if (tiles < 256 && K >= 1024 && split_buf) {
      splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, 1024 / tiles));
      while (splits > 1 && (int64_t)splits * M * N > split_cap) --splits;
    }
    const int kchunk = splits > 1 ? (int)(((int64_t)cdiv(K, splits) + BK - 1) / BK * BK) : K;
    if (splits > 1) splits = (int)cdiv(K, kchunk);
    if (splits > 1 && (epi != E_STORE || ldc != N)) return fail(RFM_EINVAL, "gemm: split-K needs a plain store");
    dim3 grid(cdiv(N, BN), cdiv(M, BM), splits);
    hipLaunchKernelGGL(gemm_f32, grid, dim3(256), 0, st, M, N, K, A, lda, ta, B, ldb, tb,
                       splits > 1 ? split_buf : C, splits > 1 ? N : ldc, bias, epi, kchunk);
    if (splits > 1)
      hipLaunchKernelGGL(sum_splits, dim3(cdiv((int64_t)M * N, 256)), dim3(256), 0, st, (int64_t)M * N, splits,
                         split_buf, C);
    RFM_LAUNCH_CHECK();
    return RFM_OK;
  }
};

rfm_status check_mlp(const rfm_mlp *P, const char *who) {
  if (!P || P->n_in < 1 || P->n_hidden < 1 || P->n_out < 1)
    return fail(RFM_EINVAL, std::string(who) + ": bad network sizes");
  if (!P->W1 || !P->b1 || !P->W2 || !P->b2 || !P->W3 || !P->b3)
    return fail(RFM_EINVAL, std::string(who) + ": null parameter");
  return RFM_OK;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_mlp_ws_bytes(const rfm_mlp *P, int32_t batch) {
  if (!P || batch < 1) return 0;
  const int64_t H = P->n_hidden, O = P->n_out;
  // split-K partials of dH2 = dY W3^T (batch x H, up to 64 slices) and loss partials
  return sizeof(float) * (size_t)(64 * batch * H) + sizeof(double) * (size_t)((batch * O + 255) / 256 + 1) + 256;
}

extern "C" rfm_status rfm_mlp_forward(const rfm_mlp *P, const float *X, int32_t batch, float *H1, float *H2,
                                      float *Y, void *stream) {
  using namespace rfm;
  rfm_status s = check_mlp(P, "rfm_mlp_forward");
  if (s != RFM_OK) return s;
  if (batch < 1 || !X || !H1 || !H2 || !Y) return fail(RFM_EINVAL, "rfm_mlp_forward: bad arguments");
  Gemm g{(hipStream_t)stream, nullptr, 0};
  const int H = P->n_hidden, O = P->n_out, I = P->n_in;
  if ((s = g.run(batch, H, I, X, I, 0, P->W1, H, 0, H1, H, P->b1, E_BIAS_TANH)) != RFM_OK) return s;
  if ((s = g.run(batch, H, H, H1, H, 0, P->W2, H, 0, H2, H, P->b2, E_BIAS_TANH)) != RFM_OK) return s;
  return g.run(batch, O, H, H2, H, 0, P->W3, O, 0, Y, O, P->b3, E_BIAS);
}

extern "C" rfm_status rfm_mlp_backward(const rfm_mlp *P, const rfm_mlp *G, const float *X, const float *H1,
                                       const float *H2, const float *Y, const float *T, int32_t batch, float *dY,
                                       float *dH1, float *dH2, float *loss, void *ws, size_t ws_bytes,
                                       void *stream) {
  using namespace rfm;
  rfm_status s = check_mlp(P, "rfm_mlp_backward");
  if (s != RFM_OK) return s;
  if ((s = check_mlp(G, "rfm_mlp_backward")) != RFM_OK) return s;
  if (G->n_in != P->n_in || G->n_hidden != P->n_hidden || G->n_out != P->n_out)
    return fail(RFM_EINVAL, "rfm_mlp_backward: gradient sizes differ");
  if (batch < 1 || !X || !H1 || !H2 || !Y || !T || !dY || !dH1 || !dH2 || !loss)
    return fail(RFM_EINVAL, "rfm_mlp_backward: bad arguments");
  if (!ws || ws_bytes < rfm_mlp_ws_bytes(P, batch)) return fail(RFM_EINVAL, "rfm_mlp_backward: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const int H = P->n_hidden, O = P->n_out, I = P->n_in;
  const int64_t nY = (int64_t)batch * O;
  float *split = (float *)ws;
  double *lpart = (double *)(split + (size_t)64 * batch * H);
  Gemm g{st, split, (int64_t)64 * batch * H};
  // loss and dY = 2 (Y - T) / (batch n_out)
  hipLaunchKernelGGL(mse_grad, dim3(cdiv(nY, 256)), dim3(256), 0, st, nY, 1.f / (float)nY, Y, T, dY, lpart);
  hipLaunchKernelGGL(finish_loss, dim3(1), dim3(1024), 0, st, lpart, (int64_t)cdiv(nY, 256), 1.0 / (double)nY, loss);
  // layer 3: dW3 = H2^T dY, db3 = colsum(dY), dH2 = dY W3^T
  if ((s = g.run(H, O, batch, H2, H, 1, dY, O, 0, G->W3, O, nullptr, E_STORE)) != RFM_OK) return s;
  hipLaunchKernelGGL(col_sum, dim3(cdiv(O, 256)), dim3(256), 0, st, batch, O, dY, G->b3);
  if ((s = g.run(batch, H, O, dY, O, 0, P->W3, O, 1, dH2, H, nullptr, E_STORE)) != RFM_OK) return s;
  hipLaunchKernelGGL(tanh_back, dim3(cdiv((int64_t)batch * H, 256)), dim3(256), 0, st, (int64_t)batch * H, H2, dH2);
  // layer 2
  if ((s = g.run(H, H, batch, H1, H, 1, dH2, H, 0, G->W2, H, nullptr, E_STORE)) != RFM_OK) return s;
  hipLaunchKernelGGL(col_sum, dim3(cdiv(H, 256)), dim3(256), 0, st, batch, H, dH2, G->b2);
  if ((s = g.run(batch, H, H, dH2, H, 0, P->W2, H, 1, dH1, H, nullptr, E_STORE)) != RFM_OK) return s;
  hipLaunchKernelGGL(tanh_back, dim3(cdiv((int64_t)batch * H, 256)), dim3(256), 0, st, (int64_t)batch * H, H1, dH1);
  // layer 1
  if ((s = g.run(I, H, batch, X, I, 1, dH1, H, 0, G->W1, H, nullptr, E_STORE)) != RFM_OK) return s;
  hipLaunchKernelGGL(col_sum, dim3(cdiv(H, 256)), dim3(256), 0, st, batch, H, dH1, G->b1);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_adam_step(int64_t n, float *p, const float *g, float *m, float *v, float lr, float beta1,
                                    float beta2, float eps, int32_t step, void *stream) {
  using namespace rfm;
  if (n < 1 || !p || !g || !m || !v || step < 1) return fail(RFM_EINVAL, "rfm_adam_step: bad arguments");
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam, dim3(cdiv(n, 256)), dim3(256), 0, (hipStream_t)stream, n, p, g, m, v, lr, beta1, beta2,
                     eps, c1, c2);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

extern "C" rfm_status rfm_gather_rows(int32_t rows, int32_t cols, const int32_t *idx, const float *in, float *out,
                                      void *stream) {
  using namespace rfm;
  if (rows < 1 || cols < 1 || !idx || !in || !out) return fail(RFM_EINVAL, "rfm_gather_rows: bad arguments");
  hipLaunchKernelGGL(gather_rows, dim3(cdiv((int64_t)rows * cols, 256)), dim3(256), 0, (hipStream_t)stream, rows,
                     cols, idx, in, out);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}
