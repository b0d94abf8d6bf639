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
#include <algorithm>
#include <climits>
#include <utility>
#include <vector>

#include "common.hpp"
#include "rrqr_rfirst.hpp"

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

// The strong variant's additions (all null for the plain filter): the full pivot order out,
// a forced pivot order in (with the number of steps to take), see rfm_rrqr_strong.
struct StrongIO {
  int32_t *perm_out;          // [ncols] position k of block j -> local feature id
  const int32_t *force;       // [ncols] pivot order to follow instead of the norm rule
  const int32_t *force_rank;  // [J] steps to take under force
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

// The whole filter of block j by one workgroup of NT threads (m_j <= 64 T rows).
template <int T, int NT>
__device__ void rrqr_one(const rfm_layout &L, const double *__restrict__ M, double tau,
                         int32_t *__restrict__ rank_out, int32_t *__restrict__ kept,
                         double *__restrict__ Rout, double *__restrict__ Q,
                         double *__restrict__ ratios, const int j, const StrongIO sio) {
  constexpr int NW = NT / kWave;
  extern __shared__ double lds_raw[];
  __syncthreads();  // a persistent workgroup reuses the LDS of its previous block
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
  const int frank = sio.force ? sio.force_rank[j] : steps;
  int r = steps;
  double ref = 0.0;
  for (int s = 0; s < steps; ++s) {
    if (s >= frank) {  // forced order: the given number of steps
      r = s;
      break;
    }
    // ---- pivot: largest trailing norm, ties to the smallest feature id (or, under a forced
    // order, the position holding the given feature)
    const int want = sio.force ? sio.force[f0 + s] : -1;
    double best = -1.0;
    int bid = INT_MAX, bk = -1;
    for (int k = s + tid; k < n; k += NT) {
      const double cv = s_.c[k];
      const int id = s_.perm[k];
      if (want >= 0 ? id == want : (cv > best || (cv == best && id < bid))) {
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
    if (bk < 0) {  // a forced feature not among the remaining positions: stop here
      r = s;
      break;
    }
    if (tid == 0 && ratios) ratios[f0 + s] = best / ref;
    if (!sio.force && best <= tau * ref) {
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
  if (sio.perm_out) {
    // the strong variant reads the trailing columns [B; C] left in the slot: their first r
    // rows take the sign normalisation of R_hat's rows, so B stays consistent with R_hat
    for (int k = tid; k < n; k += NT) sio.perm_out[f0 + k] = s_.perm[k];
    for (int k = r + wid; k < n; k += NW)
      for (int i = lane; i < r; i += kWave) A[(int64_t)k * m + i] *= s_.dsgn[i];
  }
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

// One workgroup per block, block b of the launch taking order[b] (or b).
template <int T, int NT>
__global__ __launch_bounds__(NT) void rrqr_block(rfm_layout L, const double *__restrict__ M, double tau,
                                                 int32_t *__restrict__ rank_out, int32_t *__restrict__ kept,
                                                 double *__restrict__ Rout, double *__restrict__ Q,
                                                 double *__restrict__ ratios, const int32_t *__restrict__ order,
                                                 const StrongIO sio) {
  const int b = blockIdx.x;
  rrqr_one<T, NT>(L, M, tau, rank_out, kept, Rout, Q, ratios, order ? order[b] : b, sio);
}

// Persistent form: a fixed grid whose workgroups take blocks from a shared counter in the
// order given (largest first), so uneven blocks are balanced over the CUs; every
// workgroup leaves once the counter passes J.
template <int T, int NT>
__global__ __launch_bounds__(NT) void rrqr_persistent(rfm_layout L, const double *__restrict__ M, double tau,
                                                      int32_t *__restrict__ rank_out, int32_t *__restrict__ kept,
                                                      double *__restrict__ Rout, double *__restrict__ Q,
                                                      double *__restrict__ ratios,
                                                      const int32_t *__restrict__ order, unsigned *queue) {
  __shared__ int next;
  for (;;) {
    if (threadIdx.x == 0) next = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int b = next;
    __syncthreads();  // every thread has read `next` before thread 0 takes the next block
    if (b >= L.J) return;
    rrqr_one<T, NT>(L, M, tau, rank_out, kept, Rout, Q, ratios, order ? order[b] : b, StrongIO{});
  }
}

__global__ void reset_queue(unsigned *q) { *q = 0u; }

struct Launch {
  const rfm_layout *L;
  const double *M;
  double tau;
  int32_t *rank, *kept;
  double *R, *Q, *ratios;
  const int32_t *order;
  unsigned *queue;
  int persistent, wgs_per_cu;
  hipStream_t st;
  StrongIO sio;
};

template <int T, int NT>
rfm_status launch_rrqr(const Launch &a) {
  const rfm_layout *L = a.L;
  const size_t n = (size_t)L->max_cols;
  const size_t lds = n * 3 * sizeof(double) + (size_t)kWave * T * sizeof(double) +
                     32 * sizeof(double) + n * sizeof(int) + 64 * sizeof(int);
  if (lds > 150 * 1024) return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: block too large for LDS");
  if (!a.persistent) {
    auto kern = rrqr_block<T, NT>;
    RFM_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(L->J), dim3(NT), lds, a.st, *L, a.M, a.tau, a.rank, a.kept, a.R, a.Q,
                       a.ratios, a.order, a.sio);
  } else {
    int dev = 0, cus = 0;
    RFM_HIP_TRY(hipGetDevice(&dev));
    RFM_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t grid = (int64_t)cus * (a.wgs_per_cu > 0 ? a.wgs_per_cu : 1);
    if (grid > L->J) grid = L->J;
    auto kern = rrqr_persistent<T, NT>;
    RFM_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(reset_queue, dim3(1), dim3(1), 0, a.st, a.queue);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NT), lds, a.st, *L, a.M, a.tau, a.rank, a.kept, a.R,
                       a.Q, a.ratios, a.order, a.queue);
  }
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

// Rows per lane T from the tallest block; workgroup size NT from the tuning (the register
// array of T doubles per lane limits NT = 1024 to T <= 16).
template <int T>
rfm_status pick_threads(const Launch &a, int threads) {
  if (threads == 256) return launch_rrqr<T, 256>(a);
  if (threads == 1024 && T <= 16) return launch_rrqr<T, (T <= 16 ? 1024 : 512)>(a);
  return launch_rrqr<T, 512>(a);
}

rfm_status dispatch(const Launch &a, int threads) {
  const int mr = a.L->max_rows;
  if (threads == 0) threads = (mr <= 1024) ? 1024 : 512;
  if (mr <= 64) return pick_threads<1>(a, threads);
  if (mr <= 128) return pick_threads<2>(a, threads);
  if (mr <= 256) return pick_threads<4>(a, threads);
  if (mr <= 512) return pick_threads<8>(a, threads);
  if (mr <= 768) return pick_threads<12>(a, threads);
  if (mr <= 1024) return pick_threads<16>(a, threads);
  if (mr <= 1536) return pick_threads<24>(a, threads);
  if (mr <= 2048) return pick_threads<32>(a, threads);
  if (mr <= 3072) return pick_threads<48>(a, threads);
  return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: max_rows > 3072");
}

// ---------------------------------------------------------------- strong RRQR swap test
// For block j with 0 < r < n after a factorisation that left R_hat (r x r, positive diagonal)
// in the R slot and the trailing columns [B; C] (sign-consistent with R_hat) in the Q slot,
// in position order perm:
//   X = R_hat^-1, upper triangular, row-major in the block's R-sized slot of the workspace,
//   formed a row at a time from the last (row i of R_hat staged in LDS; the entries of row i
//   of X are independent given rows > i, one thread per column, coalesced reads of X);
//   1/omega_i^2 = ||row i of X||^2 (a wave per row), gamma_q^2 = ||C e_q||^2 (a wave per
//   trailing column), and rho_iq = (X B)_iq^2 + gamma_q^2 / omega_i^2 over all (i, q) pairs.
// The largest rho (ties: smaller i, then smaller q) is the candidate swap of Gu and
// Eisenstat's strong RRQR; if it exceeds f^2 the block's next pivot order is perm with
// positions i and r + q exchanged (and the swap counter is raised), else perm itself.
constexpr int kStrongThreads = 256;

__global__ __launch_bounds__(kStrongThreads) void strong_check(rfm_layout L, const int32_t *__restrict__ rank,
                                                               const double *__restrict__ Rout,
                                                               const double *__restrict__ Q,
                                                               const int32_t *__restrict__ perm, double f2,
                                                               int32_t *__restrict__ force, double *__restrict__ rho_out,
                                                               double *__restrict__ Xws, unsigned *nswap) {
  constexpr int NW = kStrongThreads / kWave;
  __shared__ double red[NW];
  __shared__ int ired[2 * NW];
  extern __shared__ double sm[];  // arow [n], om2 [n], g2 [n]
  const int j = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int64_t f0 = L.feat_off[j];
  const int n = (int)(L.feat_off[j + 1] - f0);
  const int m = (int)(L.row_off[j + 1] - L.row_off[j]);
  const int r = rank[j];
  for (int k = tid; k < n; k += kStrongThreads) force[f0 + k] = perm[f0 + k];
  if (tid == 0) rho_out[j] = 0.0;
  if (r == 0 || r >= n) return;
  double *arow = sm, *om2 = sm + n, *g2 = sm + 2 * n;
  const int nt = n - r;
  const double *__restrict__ R = Rout + L.rsq_off[j];  // R_hat(i, c) = R[c * n + i]
  const double *__restrict__ Bq = Q + L.blk_off[j];    // slot column k, row i: Bq[k * m + i]
  double *__restrict__ X = Xws + L.rsq_off[j];         // X(i, c) = X[i * r + c]
  for (int i = r - 1; i >= 0; --i) {
    for (int k = i + tid; k < r; k += kStrongThreads) arow[k] = R[(int64_t)k * n + i];
    __syncthreads();
    const double inv = 1.0 / arow[i];
    for (int c = tid; c < r; c += kStrongThreads) {
      double t = 0.0;
      if (c >= i) {
        t = (c == i) ? 1.0 : 0.0;
        for (int k = i + 1; k <= c; ++k) t -= arow[k] * X[(int64_t)k * r + c];
        t *= inv;
      }
      X[(int64_t)i * r + c] = t;
    }
    __syncthreads();
  }
  for (int i = wid; i < r; i += NW) {
    double t = 0.0;
    for (int c = i + lane; c < r; c += kWave) t += X[(int64_t)i * r + c] * X[(int64_t)i * r + c];
    t = wave_sum(t);
    if (lane == 0) om2[i] = t;
  }
  for (int q = wid; q < nt; q += NW) {
    const double *col = Bq + (int64_t)(r + q) * m;
    double t = 0.0;
    for (int i = r + lane; i < m; i += kWave) t += col[i] * col[i];
    t = wave_sum(t);
    if (lane == 0) g2[q] = t;
  }
  __syncthreads();
  double best = -1.0;
  int bi = INT_MAX, bq = INT_MAX;
  for (int64_t e = tid; e < (int64_t)r * nt; e += kStrongThreads) {
    const int i = (int)(e / nt), q = (int)(e % nt);
    const double *col = Bq + (int64_t)(r + q) * m;
    double w = 0.0;
    for (int c = i; c < r; ++c) w += X[(int64_t)i * r + c] * col[c];
    const double rho = w * w + g2[q] * om2[i];
    if (rho > best || (rho == best && (i < bi || (i == bi && q < bq)))) {
      best = rho;
      bi = i;
      bq = q;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, kWave);
    const int oi = __shfl_xor(bi, off, kWave), oq = __shfl_xor(bq, off, kWave);
    if (ob > best || (ob == best && (oi < bi || (oi == bi && oq < bq)))) {
      best = ob;
      bi = oi;
      bq = oq;
    }
  }
  if (lane == 0) {
    red[wid] = best;
    ired[2 * wid] = bi;
    ired[2 * wid + 1] = bq;
  }
  __syncthreads();
  if (tid == 0) {
    best = red[0];
    bi = ired[0];
    bq = ired[1];
    for (int w = 1; w < NW; ++w) {
      const double ob = red[w];
      const int oi = ired[2 * w], oq = ired[2 * w + 1];
      if (ob > best || (ob == best && (oi < bi || (oi == bi && oq < bq)))) {
        best = ob;
        bi = oi;
        bq = oq;
      }
    }
    rho_out[j] = best;
    if (best > f2 && bi < r && bq < nt) {
      force[f0 + bi] = perm[f0 + r + bq];
      force[f0 + r + bq] = perm[f0 + bi];
      atomicAdd(nswap, 1u);
    }
  }
}

rfm_status validate(const rfm_layout *L, const double *M, double tau, int32_t *rank, int32_t *kept, double *R,
                    double *Q, const char *who) {
  rfm_status s = check_layout(L, who);
  if (s != RFM_OK) return s;
  if (!(tau >= 0.0 && tau < 1.0)) return fail(RFM_EINVAL, std::string(who) + ": tau must be in [0,1)");
  if (!rank || !kept || (L->nnz > 0 && (!M || !Q)) || (L->nrsq > 0 && !R))
    return fail(RFM_EINVAL, std::string(who) + ": null pointer");
  if (L->max_cols > 2048) return fail(RFM_EUNSUPPORTED, std::string(who) + ": max_cols > 2048");
  if (L->max_rows > 3072) return fail(RFM_EUNSUPPORTED, std::string(who) + ": max_rows > 3072");
  return RFM_OK;
}

}  // namespace
}  // namespace rfm

extern "C" size_t rfm_rrqr_ws_bytes(const rfm_layout *L) {
  // the work-queue counter of the direct form's persistent launch, or the R-first workspace
  if (!L) return 0;
  const size_t rf = rfm::rfirst_supported(L) ? rfm::rfirst_ws_bytes(L) : 0;
  return rf > 256 ? rf : 256;
}

extern "C" rfm_status rfm_rrqr_filter(const rfm_layout *L, const double *M, double tau,
                                      int32_t *rank, int32_t *kept, double *R, double *Q,
                                      double *ratios, void *ws, size_t ws_bytes, void *stream) {
  return rfm_rrqr_filter_tuned(L, M, tau, rank, kept, R, Q, ratios, nullptr, nullptr, ws, ws_bytes, stream);
}

extern "C" rfm_status rfm_rrqr_filter_tuned(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                                            int32_t *kept, double *R, double *Q, double *ratios,
                                            const int32_t *order, const rfm_tuning *tune, void *ws,
                                            size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s = validate(L, M, tau, rank, kept, R, Q, "rfm_rrqr_filter");
  if (s != RFM_OK) return s;
  const int persistent = tune ? tune->rrqr_persistent : 0;
  const int algo = tune ? tune->rrqr_algo : RFM_RRQR_AUTO;
  if (algo != RFM_RRQR_AUTO && algo != RFM_RRQR_DIRECT && algo != RFM_RRQR_RFIRST)
    return fail(RFM_EINVAL, "rfm_rrqr_filter: rrqr_algo must be RFM_RRQR_AUTO, _DIRECT or _RFIRST");
  if (algo == RFM_RRQR_RFIRST && persistent)
    return fail(RFM_EINVAL, "rfm_rrqr_filter: the persistent launch belongs to the direct form");
  // by default the R-first form, except for narrow blocks (at most 64 features), where the
  // direct form's single launch is faster than five
  if (algo == RFM_RRQR_RFIRST || (algo == RFM_RRQR_AUTO && !persistent && L->max_cols > 64 && rfirst_supported(L))) {
    RfirstArgs ra{L, M, tau, rank, kept, R, Q, ratios, order, ws, ws_bytes, (hipStream_t)stream};
    return rrqr_rfirst(ra);
  }
  if (persistent && (!ws || ws_bytes < 256))
    return fail(RFM_EINVAL, "rfm_rrqr_filter: the persistent launch needs the workspace");
  const int threads = tune ? tune->rrqr_threads : 0;
  if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
    return fail(RFM_EINVAL, "rfm_rrqr_filter: rrqr_threads must be 0, 256, 512 or 1024");
  Launch a{L, M, tau, rank, kept, R, Q, ratios, order, (unsigned *)ws, persistent,
           tune ? tune->rrqr_wgs_per_cu : 1, (hipStream_t)stream, StrongIO{}};
  return dispatch(a, threads);
}

extern "C" size_t rfm_rrqr_strong_ws_bytes(const rfm_layout *L) {
  if (!L) return 0;
  // swap counter, two pivot orders, the R_hat inverses (64-byte aligned)
  return 256 + 2 * (size_t)L->ncols * sizeof(int32_t) + 64 + (size_t)L->nrsq * sizeof(double);
}

extern "C" rfm_status rfm_rrqr_strong(const rfm_layout *L, const double *M, double tau, double f,
                                      int32_t max_rounds, int32_t *rank, int32_t *kept, double *R, double *Q,
                                      double *rho, int32_t *stats, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s = validate(L, M, tau, rank, kept, R, Q, "rfm_rrqr_strong");
  if (s != RFM_OK) return s;
  if (!(f > 1.0)) return fail(RFM_EINVAL, "rfm_rrqr_strong: f must exceed 1");
  if (max_rounds < 0) return fail(RFM_EINVAL, "rfm_rrqr_strong: max_rounds must be >= 0");
  if (!rho || !stats) return fail(RFM_EINVAL, "rfm_rrqr_strong: null pointer");
  if (!ws || ws_bytes < rfm_rrqr_strong_ws_bytes(L)) return fail(RFM_EINVAL, "rfm_rrqr_strong: workspace too small");
  if (3 * (size_t)L->max_cols * sizeof(double) > 64 * 1024)
    return fail(RFM_EUNSUPPORTED, "rfm_rrqr_strong: max_cols too large");
  hipStream_t st = (hipStream_t)stream;
  char *p = (char *)ws;
  unsigned *nswap = (unsigned *)p;
  int32_t *perm = (int32_t *)(p + 256);
  int32_t *force = perm + L->ncols;
  double *X = (double *)(((uintptr_t)(force + L->ncols) + 63) & ~(uintptr_t)63);
  // the plain filter (direct factorisation, norm-rule pivots) with the full pivot order out
  Launch a{L, M, tau, rank, kept, R, Q, nullptr, nullptr, nullptr, 0, 1, st, StrongIO{perm, nullptr, nullptr}};
  s = dispatch(a, 0);
  if (s != RFM_OK) return s;
  int32_t swaps = 0, rounds = 0, pending = 0;
  const size_t lds = 3 * (size_t)L->max_cols * sizeof(double);
  for (;;) {
    RFM_HIP_TRY(hipMemsetAsync(nswap, 0, sizeof(unsigned), st));
    hipLaunchKernelGGL(strong_check, dim3(L->J), dim3(kStrongThreads), lds, st, *L, (const int32_t *)rank,
                       (const double *)R, (const double *)Q, (const int32_t *)perm, f * f, force, rho, X, nswap);
    RFM_LAUNCH_CHECK();
    unsigned h = 0;
    RFM_HIP_TRY(hipMemcpyAsync(&h, nswap, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    RFM_HIP_TRY(hipStreamSynchronize(st));
    if (h == 0 || rounds == max_rounds) {
      pending = (int32_t)h;  // blocks whose last test still exceeded f^2
      break;
    }
    swaps += (int32_t)h;
    ++rounds;
    // refactor every block in its new order, keeping its rank
    Launch b{L, M, tau, rank, kept, R, Q, nullptr, nullptr, nullptr, 0, 1, st, StrongIO{perm, force, rank}};
    s = dispatch(b, 0);
    if (s != RFM_OK) return s;
  }
  stats[0] = swaps;
  stats[1] = rounds;
  stats[2] = pending;
  return RFM_OK;
}

extern "C" rfm_status rfm_plan_order(int32_t J, const int64_t *row_off, const int64_t *feat_off,
                                     int32_t *order) {
  using namespace rfm;
  if (J < 1 || !row_off || !feat_off || !order) return fail(RFM_EINVAL, "rfm_plan_order: bad arguments");
  std::vector<std::pair<double, int32_t>> cost(J);
  for (int32_t j = 0; j < J; ++j) {
    const double m = (double)(row_off[j + 1] - row_off[j]);
    const double n = (double)(feat_off[j + 1] - feat_off[j]);
    const double k = m < n ? m : n;
    // Householder QR flops of the full factorisation: the work of the block up to its rank
    cost[j] = {4.0 * m * n * k - 2.0 * (m + n) * k * k + (4.0 / 3.0) * k * k * k, j};
  }
  std::stable_sort(cost.begin(), cost.end(),
                   [](const std::pair<double, int32_t> &x, const std::pair<double, int32_t> &y) {
                     return x.first > y.first;
                   });
  for (int32_t j = 0; j < J; ++j) order[j] = cost[j].second;
  return RFM_OK;
}
