// sigma-RRQR filter of every block (Algorithm 1) on gfx950: one workgroup per block.
//
// Column-pivoted Householder QR of the block, copied into its Q slot and factored in
// place:
//   * the pivot is the trailing column of largest norm (bit-equal norms: smallest local
//     feature id); the norms are recomputed exactly from the updated column at every
//     step, fused into the trailing update, so no downdating error enters the choice;
//   * the factorisation stops at the first step s with |R_ss| <= tau |R_00| (threshold
//     relative to the leading diagonal of R);
//   * the trailing update is done one column per wave: the column (rows s..m-1) is held
//     in registers, lane <-> row, so every element is read and written once per step;
//     the dot product with the reflector (kept in LDS) and the new norm are butterfly
//     reductions across the wave;
//   * afterwards R_hat is copied out, the first r columns of Q are formed in place from
//     the stored reflectors (backward accumulation), and the signs are normalised so
//     diag(R_hat) > 0.
// Householder reflector of x = A[s:m, s]: beta = -sign(alpha) ||x||, v = [1, x_2:/(alpha -
// beta)], tau_h = (beta - alpha)/beta, sign(0) = +.
#include <climits>

#include "common.hpp"

namespace rfm {
namespace {

struct Lds {
  double *c;       // [n] current trailing column norms
  double *taus;    // [n] reflector scalars
  double *dsgn;    // [n] sign of diag(R)
  int *perm;       // [n] local feature id of each column position
  double *v;       // [64*T] reflector (relative row index)
  double *red;     // [32] cross-wave reduction scratch
  int *ired;       // [64]
};

// Wave argmax with tie-break on the smaller id; all lanes get the winner.
__device__ __forceinline__ void wave_argmax(double &best, int &bid, int &bk) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, kWave);
    const int oid = __shfl_xor(bid, off, kWave);
    const int ok = __shfl_xor(bk, off, kWave);
    if (ob > best || (ob == best && oid < bid)) {
      best = ob;
      bid = oid;
      bk = ok;
    }
  }
}

template <int T, int NT>
__global__ __launch_bounds__(NT) void rrqr_block(rfm_layout L, const double *__restrict__ M,
                                                 double tau, int32_t *__restrict__ rank_out,
                                                 int32_t *__restrict__ kept,
                                                 double *__restrict__ Rout, double *__restrict__ Q,
                                                 double *__restrict__ ratios) {
  constexpr int NW = NT / kWave;
  extern __shared__ double lds_raw[];
  const int j = blockIdx.x;
  const int64_t m64 = L.row_off[j + 1] - L.row_off[j];
  const int m = (int)m64;
  const int64_t f0 = L.feat_off[j];
  const int n = (int)(L.feat_off[j + 1] - f0);
  const int64_t base = L.blk_off[j];
  double *__restrict__ A = Q + base;
  const double *__restrict__ Mj = M + base;
  double *__restrict__ R = Rout + L.rsq_off[j];

  Lds s_;
  s_.c = lds_raw;
  s_.taus = s_.c + n;
  s_.dsgn = s_.taus + n;
  s_.v = s_.dsgn + n;
  s_.red = s_.v + kWave * T;
  s_.perm = (int *)(s_.red + 32);
  s_.ired = s_.perm + n;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;

  // copy the block into its Q slot and take the initial column norms
  for (int k = wid; k < n; k += NW) {
    double ss = 0.0;
    for (int i = lane; i < m; i += kWave) {
      const double a = Mj[(int64_t)k * m + i];
      A[(int64_t)k * m + i] = a;
      ss += a * a;
    }
    ss = wave_sum(ss);
    if (lane == 0) {
      s_.c[k] = sqrt(ss);
      s_.perm[k] = k;
      if (ratios) ratios[f0 + k] = 0.0;
    }
  }
  __syncthreads();

  const int steps = min(m, n);
  int r = steps;
  double ref = 0.0;
  for (int s = 0; s < steps; ++s) {
    // ---- pivot: largest trailing norm, ties to the smallest feature id
    double best = -1.0;
    int bid = INT_MAX, bk = -1;
    for (int k = s + tid; k < n; k += NT) {
      const double cv = s_.c[k];
      const int id = s_.perm[k];
      if (cv > best || (cv == best && id < bid)) {
        best = cv;
        bid = id;
        bk = k;
      }
    }
    wave_argmax(best, bid, bk);
    if (lane == 0) {
      s_.red[wid] = best;
      s_.ired[wid] = bid;
      s_.ired[32 + wid] = bk;
    }
    __syncthreads();
    best = s_.red[0];
    bid = s_.ired[0];
    bk = s_.ired[32];
    for (int w = 1; w < NW; ++w) {
      const double ob = s_.red[w];
      const int oid = s_.ired[w];
      if (ob > best || (ob == best && oid < bid)) {
        best = ob;
        bid = oid;
        bk = s_.ired[32 + w];
      }
    }
    if (s == 0) ref = best;
    if (ref == 0.0) {  // zero block: nothing is kept
      r = 0;
      break;
    }
    if (tid == 0 && ratios) ratios[f0 + s] = best / ref;
    if (best <= tau * ref) {
      r = s;
      break;
    }
    const int p = bk;
    __syncthreads();  // everyone has read red/ired and c before they change
    if (p != s) {
      for (int i = tid; i < m; i += NT) {
        const double a = A[(int64_t)s * m + i];
        A[(int64_t)s * m + i] = A[(int64_t)p * m + i];
        A[(int64_t)p * m + i] = a;
      }
      if (tid == 0) {
        const double cc = s_.c[s];
        s_.c[s] = s_.c[p];
        s_.c[p] = cc;
        const int pp = s_.perm[s];
        s_.perm[s] = s_.perm[p];
        s_.perm[p] = pp;
      }
    }
    __syncthreads();

    // ---- Householder reflector of column s (wave 0)
    if (wid == 0) {
      double *col = A + (int64_t)s * m;
      const double alpha = col[s];
      double sig2 = 0.0;
      for (int i = s + 1 + lane; i < m; i += kWave) sig2 += col[i] * col[i];
      sig2 = wave_sum(sig2);
      double th = 0.0;
      if (sig2 == 0.0) {
        for (int i = lane; i < m - s; i += kWave) s_.v[i] = (i == 0) ? 1.0 : 0.0;
      } else {
        const double nrm = sqrt(alpha * alpha + sig2);
        const double beta = (alpha >= 0.0) ? -nrm : nrm;
        const double den = alpha - beta;
        th = (beta - alpha) / beta;
        for (int i = s + 1 + lane; i < m; i += kWave) {
          const double vi = col[i] / den;
          col[i] = vi;
          s_.v[i - s] = vi;
        }
        if (lane == 0) {
          col[s] = beta;
          s_.v[0] = 1.0;
        }
      }
      if (lane == 0) s_.taus[s] = th;
    }
    __syncthreads();

    // ---- trailing update with fused exact norm recomputation, one column per wave
    const double th = s_.taus[s];
    const int mrel = m - s;
    double vr[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = lane + kWave * t;
      vr[t] = (i < mrel) ? s_.v[i] : 0.0;
    }
    for (int k = s + 1 + wid; k < n; k += NW) {
      double *col = A + (int64_t)k * m + s;
      double x[T];
      double f = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = lane + kWave * t;
        x[t] = (i < mrel) ? col[i] : 0.0;
        f += vr[t] * x[t];
      }
      f = wave_sum(f);
      double ss = 0.0;
      if (th != 0.0) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int i = lane + kWave * t;
          x[t] -= th * (vr[t] * f);
          if (i < mrel) col[i] = x[t];
        }
      }
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = lane + kWave * t;
        if (i >= 1 && i < mrel) ss += x[t] * x[t];
      }
      ss = wave_sum(ss);
      if (lane == 0) s_.c[k] = sqrt(ss);
    }
    __syncthreads();
  }

  // ---- outputs: rank, kept ids, R_hat (sign-normalised)
  if (tid == 0) rank_out[j] = r;
  for (int k = tid; k < n; k += NT) kept[f0 + k] = (k < r) ? s_.perm[k] : -1;
  for (int k = tid; k < r; k += NT) s_.dsgn[k] = (A[(int64_t)k * m + k] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  for (int k = wid; k < r; k += NW)
    for (int i = lane; i < r; i += kWave)
      R[(int64_t)k * n + i] = (i <= k) ? s_.dsgn[i] * A[(int64_t)k * m + i] : 0.0;
  __syncthreads();

  // ---- explicit Q_hat: apply H_{r-1} ... H_0 to [I_r; 0] in place (backward)
  for (int s = r - 1; s >= 0; --s) {
    const double th = s_.taus[s];
    const int mrel = m - s;
    for (int i = tid; i < mrel; i += NT) s_.v[i] = (i == 0) ? 1.0 : A[(int64_t)s * m + s + i];
    __syncthreads();
    double vr[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = lane + kWave * t;
      vr[t] = (i < mrel) ? s_.v[i] : 0.0;
    }
    if (th != 0.0) {
      for (int k = s + 1 + wid; k < r; k += NW) {
        double *col = A + (int64_t)k * m + s;
        double x[T];
        double f = 0.0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int i = lane + kWave * t;
          x[t] = (i < mrel) ? col[i] : 0.0;
          f += vr[t] * x[t];
        }
        f = wave_sum(f);
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int i = lane + kWave * t;
          if (i < mrel) col[i] = x[t] - th * (vr[t] * f);
        }
      }
    }
    __syncthreads();
    // column s of Q: -tau v below the diagonal, 1 - tau on it, zeros above
    for (int i = tid; i < m; i += NT) {
      double q;
      if (i < s) q = 0.0;
      else if (i == s) q = 1.0 - th;
      else q = -th * s_.v[i - s];
      A[(int64_t)s * m + i] = q;
    }
    __syncthreads();
  }
  // sign normalisation of the columns of Q_hat
  for (int k = wid; k < r; k += NW) {
    const double sg = s_.dsgn[k];
    if (sg < 0.0)
      for (int i = lane; i < m; i += kWave) A[(int64_t)k * m + i] = -A[(int64_t)k * m + i];
  }
}

template <int T, int NT>
rfm_status launch_rrqr(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                       int32_t *kept, double *R, double *Q, double *ratios, hipStream_t st) {
  const size_t n = (size_t)L->max_cols;
  const size_t lds = n * 3 * sizeof(double) + (size_t)kWave * T * sizeof(double) +
                     32 * sizeof(double) + n * sizeof(int) + 64 * sizeof(int);
  if (lds > 150 * 1024) return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: block too large for LDS");
  auto kern = rrqr_block<T, NT>;
  RFM_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(L->J), dim3(NT), lds, st, *L, M, tau, rank, kept, R, Q, ratios);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_rrqr_ws_bytes(const rfm_layout *L) {
  (void)L;
  return 0;
}

extern "C" rfm_status rfm_rrqr_filter(const rfm_layout *L, const double *M, double tau,
                                      int32_t *rank, int32_t *kept, double *R, double *Q,
                                      double *ratios, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  (void)ws;
  (void)ws_bytes;
  rfm_status s = check_layout(L, "rfm_rrqr_filter");
  if (s != RFM_OK) return s;
  if (!(tau >= 0.0 && tau < 1.0)) return fail(RFM_EINVAL, "rfm_rrqr_filter: tau must be in [0,1)");
  if (!rank || !kept || (L->nnz > 0 && (!M || !Q)) || (L->nrsq > 0 && !R))
    return fail(RFM_EINVAL, "rfm_rrqr_filter: null pointer");
  if (L->max_cols > 2048) return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: max_cols > 2048");
  hipStream_t st = (hipStream_t)stream;
  const int mr = L->max_rows;
  if (mr <= 64) return launch_rrqr<1, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 128) return launch_rrqr<2, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 256) return launch_rrqr<4, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 512) return launch_rrqr<8, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 768) return launch_rrqr<12, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 1024) return launch_rrqr<16, 1024>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 1536) return launch_rrqr<24, 512>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 2048) return launch_rrqr<32, 512>(L, M, tau, rank, kept, R, Q, ratios, st);
  if (mr <= 3072) return launch_rrqr<48, 512>(L, M, tau, rank, kept, R, Q, ratios, st);
  return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: max_rows > 3072");
}
