// sigma-RRQR filter of every block (Algorithm 1), R-first form.
//
// The column-pivoted QR of a tall block M_j (m x n) has the same pivots, the same R and the
// same Q (up to rounding) as the pivoted QR of the triangular factor R0 of its unpivoted QR
// M_j = Q0 R0, because the column norms and every later step only see M_j through Q0^T M_j.
// Working on R0 (n x n, at most 512 x 512) instead of M_j keeps the whole pivoted
// factorisation on chip, and the two passes over the tall block need no pivoting, so
// their updates can be deferred over panels of reflectors.  Five kernels, one workgroup
// per block (or a persistent grid taking blocks from a counter, largest first):
//   rf_qr     copy M_j into its Q slot; unpivoted Householder QR in panels of nb columns:
//             the panel is factored with its columns in registers, then every trailing
//             column is loaded once, takes the panel's nb reflectors in order, and is
//             stored once (HBM traffic ~ 2 m n^2 / nb instead of ~ m n^2);
//   rf_qrcp   Businger-Golub pivoting on R0 with exact norm recomputation at every step:
//             columns live in three tiers (registers of the eight waves, LDS, then a global
//             slot), every active column takes the step's reflector and has its norm
//             recomputed from its updated entries; stops at the first |R_ss| <= tau |R_00|;
//             writes R_hat (signs normalised so diag > 0) and the reflectors below it;
//   rf_formq1 Q1 = H'_0 ... H'_{r-1} [I_r; 0] (n x r) backward, in panels;
//   rf_formq0 Q0 = H_0 ... H_{n-1} [I_n; 0] (m x n) backward in place, in panels;
//   rf_gemm   Q_hat = Q0 Q1 D (D the sign normalisation) in place, by row tiles in LDS.
// Householder reflector of x (pivot row s): beta = -sign(alpha) ||x||, v = [1, x_2:/(alpha -
// beta)], tau_h = (beta - alpha)/beta, sign(0) = +; nothing to zero gives tau_h = 0.
#include <algorithm>

#include "rrqr_rfirst.hpp"

namespace rfm {
namespace {

constexpr int NT = 512;
constexpr int NW = NT / kWave;
constexpr size_t kLdsCap = 158 * 1024;

struct Blk {
  int m, n, nr;
  int64_t f0, base, rsq;
};

__device__ __forceinline__ Blk blk(const rfm_layout &L, int j) {
  Blk b;
  b.m = (int)(L.row_off[j + 1] - L.row_off[j]);
  b.f0 = L.feat_off[j];
  b.n = (int)(L.feat_off[j + 1] - b.f0);
  b.nr = b.m < b.n ? b.m : b.n;
  b.base = L.blk_off[j];
  b.rsq = L.rsq_off[j];
  return b;
}

// Reflector of a column held by one wave: row r0 + lane + 64 t in x[t], rows [s, hi) live.
// Writes v (v[0] = 1) to vdst[row - s] for rows s..hi-1 and overwrites x with beta at row s
// and v below it (x is left as it is when there is nothing to zero).  Returns tau_h.
template <int TT>
__device__ __forceinline__ double reflect(double (&x)[TT], int r0, int s, int hi, double *vdst) {
  const int lane = threadIdx.x & (kWave - 1);
  double alpha = 0.0, sig2 = 0.0;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int row = r0 + lane + kWave * t;
    if (row == s) alpha = x[t];
    else if (row > s && row < hi) sig2 += x[t] * x[t];
  }
  wave_sum2_dpp(alpha, sig2);  // alpha: one non-zero term
  if (sig2 == 0.0) {
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const int row = r0 + lane + kWave * t;
      if (row >= s && row < hi) vdst[row - s] = (row == s) ? 1.0 : 0.0;
    }
    return 0.0;
  }
  const double nrm = sqrt(alpha * alpha + sig2);
  const double beta = (alpha >= 0.0) ? -nrm : nrm;
  const double rden = 1.0 / (alpha - beta);
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int row = r0 + lane + kWave * t;
    if (row == s) {
      x[t] = beta;
      vdst[0] = 1.0;
    } else if (row > s && row < hi) {
      const double vi = x[t] * rden;
      x[t] = vi;
      vdst[row - s] = vi;
    }
  }
  return (beta - alpha) / beta;
}

// As reflect, branch-free, for a column held as rows r0 + lane + 64 t (t < TT) whose
// reflector row vrow has room for all 64 TT of them: every lane stores all TT entries of
// v by row - r0 (zero above the pivot row s and from hi on), so no conditional stores.
template <int TT>
__device__ __forceinline__ double reflect_rows(double (&x)[TT], int r0, int s, int hi, double *vrow,
                                               double *diag = nullptr) {
  const int lane = threadIdx.x & (kWave - 1);
  double alpha = 0.0, sig2 = 0.0;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int row = r0 + lane + kWave * t;
    alpha += (row == s) ? x[t] : 0.0;
    const double xb = (row > s && row < hi) ? x[t] : 0.0;
    sig2 = fma(xb, xb, sig2);
  }
  wave_sum2_dpp(alpha, sig2);  // alpha: one non-zero term
  if (sig2 == 0.0) {
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      const int row = r0 + lane + kWave * t;
      vrow[lane + kWave * t] = (row == s) ? 1.0 : 0.0;
    }
    if (diag) *diag = alpha;
    return 0.0;
  }
  const double nrm = sqrt(alpha * alpha + sig2);
  const double beta = (alpha >= 0.0) ? -nrm : nrm;
  if (diag) *diag = beta;
  const double rden = 1.0 / (alpha - beta);
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int row = r0 + lane + kWave * t;
    const bool below = row > s && row < hi;
    const double vi = below ? x[t] * rden : 0.0;
    vrow[lane + kWave * t] = (row == s) ? 1.0 : vi;
    x[t] = (row == s) ? beta : (below ? vi : x[t]);
  }
  return (beta - alpha) / beta;
}

// x_g <- (I - th v v^T) x_g for G columns held by one wave (v in vr, same row layout).
template <int TT, int G>
__device__ __forceinline__ void apply_refl(double (&x)[G][TT], const double (&vr)[TT], double th) {
  double f[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    f[g] = 0.0;
#pragma unroll
    for (int t = 0; t < TT; ++t) f[g] += vr[t] * x[g][t];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) f[g] = wave_sum_dpp(f[g]);
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < TT; ++t) x[g][t] -= th * (vr[t] * f[g]);
}

template <int TT>
__device__ __forceinline__ void apply_refl1(double (&x)[TT], const double (&vr)[TT], double th) {
  double f = 0.0;
#pragma unroll
  for (int t = 0; t < TT; ++t) f += vr[t] * x[t];
  f = wave_sum_dpp(f);
#pragma unroll
  for (int t = 0; t < TT; ++t) x[t] -= th * (vr[t] * f);
}

// apply_refl1 on two columns of one wave with one interleaved reduction; a column whose
// flag is off is left as it is.
template <int TT>
__device__ __forceinline__ void apply_refl1x2(double (&x)[TT], double (&y)[TT], const double (&vr)[TT], double th,
                                              bool onx, bool ony) {
  double f = 0.0, g = 0.0;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    f += vr[t] * x[t];
    g += vr[t] * y[t];
  }
  wave_sum2_dpp(f, g);
  if (onx) {
#pragma unroll
    for (int t = 0; t < TT; ++t) x[t] -= th * (vr[t] * f);
  }
  if (ony) {
#pragma unroll
    for (int t = 0; t < TT; ++t) y[t] -= th * (vr[t] * g);
  }
}

// As apply_refl, with v read from LDS (row lane + 64 t at v[lane + 64 t], rows >= nv zero)
// twice instead of being held in registers: for tall blocks.
template <int TT, int G>
__device__ __forceinline__ void apply_refl_lds(double (&x)[G][TT], const double *v, int nv, double th) {
  const int lane = threadIdx.x & (kWave - 1);
  double f[G];
#pragma unroll
  for (int g = 0; g < G; ++g) f[g] = 0.0;
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int rr = lane + kWave * t;
    const double vv = (rr < nv) ? v[rr] : 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) f[g] += vv * x[g][t];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) f[g] = wave_sum_dpp(f[g]);
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    const int rr = lane + kWave * t;
    const double vv = (rr < nv) ? v[rr] : 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) x[g][t] -= th * (vv * f[g]);
  }
}

// Sum over each group of 16 lanes (a DPP row) by a rotate butterfly: every lane of the row
// receives the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_row<0x128>(v);  // row_ror:8
  v += dpp_row<0x124>(v);  // row_ror:4
  v += dpp_row<0x122>(v);  // row_ror:2
  v += dpp_row<0x121>(v);  // row_ror:1
  return v;
}


// One column per group of 16 lanes (lane i of group g holds rows r0 + i + 16 t, t < R16):
// x <- H x for the reflector v at V (rows relative to r0, zero-padded to 16 R16) with scalar
// th; a 16-lane reduction per reflector serves the four columns of a wave at once.
template <int R16>
__device__ __forceinline__ void apply_refl16(double (&x)[R16], const double *v, double th) {
  static_assert(R16 % 4 == 0, "four interleaved partial dot products");
  const int li = threadIdx.x & 15;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
#pragma unroll
  for (int t = 0; t < R16; t += 4) {
    f0 = fma(v[li + 16 * t], x[t], f0);
    f1 = fma(v[li + 16 * (t + 1)], x[t + 1], f1);
    f2 = fma(v[li + 16 * (t + 2)], x[t + 2], f2);
    f3 = fma(v[li + 16 * (t + 3)], x[t + 3], f3);
  }
  double f = (f0 + f1) + (f2 + f3);
  f = row16_sum(f);
  const double g = -th * f;
#pragma unroll
  for (int t = 0; t < R16; ++t) x[t] = fma(g, v[li + 16 * t], x[t]);
}

// ---------------------------------------------------------------- unpivoted QR of the block
// Reflector i of the current panel: Vp[i * ldv + (row - p)] for rows p..m-1 (zero above its
// pivot row, 1 on it).  taus: [max_cols] in LDS.
template <int T, int G, int NPC>
__global__ __launch_bounds__(NT) void rf_qr(rfm_layout L, const double *__restrict__ M, double *__restrict__ Q,
                                            double *__restrict__ tau0, int nb, const int32_t *__restrict__ order) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  {
    const int j = order ? order[blockIdx.x] : blockIdx.x;
    const Blk B = blk(L, j);
    const int m = B.m, n = B.n, nr = B.nr;
    double *__restrict__ A = Q + B.base;
    const double *__restrict__ Mj = M + B.base;
    double *taus = lds;
    double *Vp = lds + L.max_cols;
    constexpr bool Q16 = T <= 12;     // trailing update with one column per 16 lanes
    const int ldv = Q16 ? 64 * T : m;  // reflector rows zero-padded to 64 T in that case
    // the first panel reads M_j itself and every column of the slot is stored in it, so M_j
    // is not copied separately (m = 0 or n = 0: nothing to store)
    for (int p = 0; p < nr; p += nb) {
      const int b = min(nb, nr - p);
      const double *__restrict__ src = (p == 0) ? Mj : A;
      // the panel's columns in registers: column p + w + NW u
      double pc[NPC][T];
#pragma unroll
      for (int u = 0; u < NPC; ++u) {
        const int k = p + w + NW * u;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const int row = p + lane + kWave * t;
          pc[u][t] = (k < p + b && row < m) ? src[(int64_t)k * m + row] : 0.0;
        }
      }
      for (int i = 0; i < b; ++i) {
        const int s = p + i;
        if (w == i % NW) {
          double *vrow = Vp + (int64_t)i * ldv;
          double th;
          if constexpr (Q16) {
            // the padded row (64 T entries from row p) is written whole
            if (NPC == 1 || i < NW) th = reflect_rows<T>(pc[0], p, s, m, vrow);
            else th = reflect_rows<T>(pc[NPC - 1], p, s, m, vrow);
          } else {
            for (int rr = lane; rr < i; rr += kWave) vrow[rr] = 0.0;
            for (int rr = m - p + lane; rr < ldv; rr += kWave) vrow[rr] = 0.0;
            if (NPC == 1 || i < NW) th = reflect<T>(pc[0], p, s, m, vrow + i);
            else th = reflect<T>(pc[NPC - 1], p, s, m, vrow + i);
          }
          if (lane == 0) taus[s] = th;
        }
        __syncthreads();
        const double th = taus[s];
        if constexpr (T >= 24) {
          if (p + w > s && p + w < p + b)
            apply_refl_lds<T, 1>(reinterpret_cast<double(&)[1][T]>(pc[0]), Vp + (int64_t)i * ldv, m - p, th);
        } else {
          double vr[T];
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int rr = lane + kWave * t;
            // Q16: rows of the padded reflector are zero from m - p on
            vr[t] = (Q16 || p + rr < m) ? Vp[(int64_t)i * ldv + rr] : 0.0;
          }
          const bool on0 = p + w > s && p + w < p + b;
          if constexpr (NPC > 1) {
            const bool on1 = p + w + NW > s && p + w + NW < p + b;
            if (on0 && on1) apply_refl1x2<T>(pc[0], pc[NPC - 1], vr, th, true, true);
            else if (on0) apply_refl1<T>(pc[0], vr, th);
            else if (on1) apply_refl1<T>(pc[NPC - 1], vr, th);
          } else if (on0) {
            apply_refl1<T>(pc[0], vr, th);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < NPC; ++u) {
        const int k = p + w + NW * u;
        if (k < p + b) {
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int row = p + lane + kWave * t;
            if (row < m) A[(int64_t)k * m + row] = pc[u][t];
          }
        }
      }
      // trailing columns: loaded once, the panel's reflectors in order, stored once
      if constexpr (Q16) {
        constexpr int R16 = 4 * T;
        const int li = lane & 15, qd = lane >> 4;
        for (int c0 = p + b + 4 * w; c0 < n; c0 += 4 * NW) {
          const int k = c0 + qd;
          double x[R16];
#pragma unroll
          for (int t = 0; t < R16; ++t) {
            const int row = p + li + 16 * t;
            x[t] = (k < n && row < m) ? src[(int64_t)k * m + row] : 0.0;
          }
          for (int i = 0; i < b; ++i) apply_refl16<R16>(x, Vp + (int64_t)i * ldv, taus[p + i]);
          if (k < n) {
#pragma unroll
            for (int t = 0; t < R16; ++t) {
              const int row = p + li + 16 * t;
              if (row < m) A[(int64_t)k * m + row] = x[t];
            }
          }
        }
      } else
      for (int c0 = p + b + w * G; c0 < n; c0 += NW * G) {
        double x[G][T];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int k = c0 + g;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int row = p + lane + kWave * t;
            x[g][t] = (k < n && row < m) ? src[(int64_t)k * m + row] : 0.0;
          }
        }
        for (int i = 0; i < b; ++i) {
          if constexpr (T >= 24) {
            apply_refl_lds<T, G>(x, Vp + (int64_t)i * ldv, m - p, taus[p + i]);
          } else {
            double vr[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
              const int rr = lane + kWave * t;
              vr[t] = (p + rr < m) ? Vp[(int64_t)i * ldv + rr] : 0.0;
            }
            apply_refl<T, G>(x, vr, taus[p + i]);
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int k = c0 + g;
          if (k < n) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
              const int row = p + lane + kWave * t;
              if (row < m) A[(int64_t)k * m + row] = x[g][t];
            }
          }
        }
      }
      __syncthreads();
    }
    for (int k = tid; k < nr; k += NT) tau0[B.f0 + k] = taus[k];
  }
}

// ---------------------------------------------------------------- pivoted QR of R0
// One column per group of 16 lanes: lane i of a group holds rows i + 16 t (t < R16) of its
// column, so the four groups of a wave work on four columns at once and each dot product is
// a 16-lane reduction.  Columns of R0 (rows 0..nr-1) live in slots: slot u < NREG is a
// register slot (group u % 4, index (u / 4) % S4, wave u / (4 S4)), NREG <= u < NREG + nl an
// LDS column, u >= NREG + nl column u - NREG - nl of the block's part of W1 (K_j columns of
// stride ld = 16 R16 from 16 R16 feat_off[j]; rows >= nr zero).  Column c starts in slot c.  When the pivot comes from a
// register or LDS slot, an active column of the global tier moves into the freed slot, so
// the global tier drains as the factorisation proceeds.
// At step s every active column takes the reflector, gives up its row s (final: R entry
// (s, column), kept in Rrow[column * n + s] of the block's slot W3) and has that row
// cleared, so its norm below the pivot row is the norm of the whole stored column.
// LDS: sn, scol [nslot] (norm, -1 once retired or empty; column id, -1 empty), t1, ds, perm
// [nmax], glist, gpos (global slots still active, and where each sits in glist), vabs [32 R16]
// (the reflector by absolute row, zero outside [s, nr) and in its upper half), pcol [16 R16],
// red/ired, regact [NW] (active register slots of each wave), then the LDS tier.
// Register slots are kept aligned to the current window of 16 rows: entry t of lane i holds
// row 16 (s / 16) + i + 16 t, the arrays shifting down by one entry every 16 steps, so row s
// is always entry 0 of lane s % 16 and no row test is needed in the inner loops.
__host__ __device__ constexpr size_t qrcp_small_bytes(int nmax, int nreg, int r16) {
  return (size_t)(2 * nmax + (nmax + nreg) + 3 * 16 * r16 + 32) * sizeof(double) +
         (size_t)(2 * (nmax + nreg) + 2 * nmax + 64 + NW + 2) * sizeof(int) + 8;
}

template <int R16, int S4>
__global__ __launch_bounds__(NT) void rf_qrcp(rfm_layout L, const double *__restrict__ Q, double tau,
                                              int32_t *__restrict__ rank_out, int32_t *__restrict__ kept,
                                              double *__restrict__ Rout, double *__restrict__ ratios,
                                              double *__restrict__ tau1, double *__restrict__ dsgn,
                                              double *__restrict__ W1, double *__restrict__ W3,
                                              int64_t tier_doubles, const int32_t *__restrict__ order) {
  extern __shared__ double lds[];
  constexpr int TR = R16 / 4;       // rows per lane in the 64-lane layout of the reflector
  constexpr int NREG = NW * S4 * 4;
  constexpr int LD = 16 * R16;      // stride of LDS and global tier columns
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int li = lane & 15, qd = lane >> 4;
  const int nmax = L.max_cols, nsl = nmax + NREG;
  double *sn = lds;                  // [nsl]
  double *t1 = sn + nsl;             // [nmax]
  double *ds = t1 + nmax;            // [nmax]
  double *vabs = ds + nmax;          // [2 * 16 R16] reflector by absolute row, zero elsewhere
  double *pcol = vabs + 2 * LD;      // [16 R16]
  double *red = pcol + LD;           // [32]
  int *scol = (int *)(red + 32);     // [nsl]
  int *gpos = scol + nsl;            // [nsl]
  int *perm = gpos + nsl;            // [nmax]
  int *glist = perm + nmax;          // [nmax]
  int *ired = glist + nmax;          // [64]
  unsigned *regact = (unsigned *)(ired + 64);  // [NW]
  int *gcnt = (int *)(regact + NW);             // [2]
  // the LDS tier starts at the next 8-byte boundary (an element offset from lds, without an
  // integer round trip, so the compiler keeps it an LDS pointer)
  double *tier = lds + (((char *)(gcnt + 2) - (char *)lds) + 7) / 8;

  const int j = order ? order[blockIdx.x] : blockIdx.x;
  const Blk B = blk(L, j);
  const int m = B.m, n = B.n, nr = B.nr;
  const double *__restrict__ A = Q + B.base;
  double *__restrict__ R = Rout + B.rsq;
  double *__restrict__ Wg = W1 + B.f0 * LD;
  double *__restrict__ Rrow = W3 + B.rsq;
  const int nl = (nr > 0) ? (int)min((int64_t)max(n - NREG, 0), tier_doubles / LD) : 0;
  const int gbase = NREG + nl;
  const int nslot = max(n, NREG);
  auto colptr = [&](int u) -> double * {
    return (u < gbase) ? tier + (int64_t)(u - NREG) * LD : Wg + (int64_t)(u - gbase) * LD;
  };

  // Every lane tracks the best (norm, column, slot) among the columns its group of 16 lanes
  // (or its wave, in the 64-lane loops) has just normed; a wave's best goes to red/ired.
  double bn = -0.5;
  int bc = 0x7fffffff, bs = -1;
  auto track = [&](double v, int c, int u) {
    if (v > bn || (v == bn && c < bc)) {
      bn = v;
      bc = c;
      bs = u;
    }
  };
  auto publish = [&]() {  // combine the four groups of the wave; lane 0 writes
#pragma unroll
    for (int off = 16; off < kWave; off <<= 1) {
      const double ob = __shfl_xor(bn, off, kWave);
      const int oc = __shfl_xor(bc, off, kWave);
      const int ou = __shfl_xor(bs, off, kWave);
      if (ob > bn || (ob == bn && oc < bc)) {
        bn = ob;
        bc = oc;
        bs = ou;
      }
    }
    if (lane == 0) {
      red[w] = bn;
      ired[w] = bc;
      ired[32 + w] = bs;
    }
    bn = -0.5;
    bc = 0x7fffffff;
    bs = -1;
  };

  // ---- R0 into the tiers (rows >= nr zero), initial norms
  double xs[S4][R16];
#pragma unroll
  for (int q = 0; q < S4; ++q) {
    const int c = (w * S4 + q) * 4 + qd;
    double ss = 0.0;
#pragma unroll
    for (int t = 0; t < R16; ++t) {
      const int row = li + 16 * t;
      const bool ok = c < n && row < nr && row <= c;
      xs[q][t] = ok ? A[(int64_t)c * m + row] : 0.0;
      ss += xs[q][t] * xs[q][t];
    }
    ss = row16_sum(ss);
    if (c < n) track(sqrt(ss), c, c);
    if (li == 0) {
      sn[c] = (c < n) ? sqrt(ss) : -1.0;
      scol[c] = (c < n) ? c : -1;
    }
  }
  for (int c = NREG + w; c < n; c += NW) {
    double ss = 0.0;
    double *dst = colptr(c);
    for (int row = lane; row < LD; row += kWave) {
      const double a = (row <= c && row < nr) ? A[(int64_t)c * m + row] : 0.0;
      dst[row] = a;
      ss += a * a;
    }
    ss = wave_sum_dpp(ss);
    track(sqrt(ss), c, c);
    if (lane == 0) {
      sn[c] = sqrt(ss);
      scol[c] = c;
    }
  }
  publish();
  for (int u = gbase + tid; u < n; u += NT) {
    glist[u - gbase] = u;
    gpos[u] = u - gbase;
  }
  if (tid < NW) {
    unsigned bits = 0;
    for (int b = 0; b < 4 * S4; ++b)
      if ((tid * S4 + b / 4) * 4 + b % 4 < n) bits |= 1u << b;
    regact[tid] = bits;
  }
  if (tid == 0) gcnt[0] = max(n - gbase, 0);
  if (ratios)
    for (int c = tid; c < n; c += NT) ratios[B.f0 + c] = 0.0;
  for (int row = tid; row < 2 * LD; row += NT) vabs[row] = 0.0;
  __syncthreads();

  int r = nr;
  double ref = 0.0;
  for (int s = 0; s < nr; ++s) {
    const int ts = s >> 4, ls = s & 15;
    if (s > 0 && ls == 0) {  // the register window moves down 16 rows
#pragma unroll
      for (int q = 0; q < S4; ++q)
#pragma unroll
        for (int t = 0; t < R16; ++t) xs[q][t] = (t + 1 < R16) ? xs[q][t + 1] : 0.0;
    }
    // ---- pivot: the best of the waves' bests (largest norm, ties to the smallest column)
    double best = red[0];
    int bid = ired[0], bu = ired[32];
    for (int ww = 1; ww < NW; ++ww) {
      const double ob = red[ww];
      const int oid = ired[ww];
      if (ob > best || (ob == best && oid < bid)) {
        best = ob;
        bid = oid;
        bu = ired[32 + ww];
      }
    }
    if (s == 0) ref = best;
    if (ref == 0.0) {  // zero block: nothing is kept
      r = 0;
      break;
    }
    if (tid == 0 && ratios) ratios[B.f0 + s] = best / ref;
    if (best <= tau * ref) {
      r = s;
      break;
    }
    const int P = bid, U = bu;

    // ---- the pivot column to LDS (absolute rows) by the wave that holds it; a global
    // column refills the slot
    const int owner = (U < NREG) ? U / (4 * S4) : 0;
    if (w == owner) {
      const int gc = gcnt[0];
      const int g = (U < gbase && gc > 0) ? glist[gc - 1] : -1;
      const double *gsrc = (g >= 0) ? colptr(g) : nullptr;
      if (U < NREG) {
        const int qp = (U / 4) % S4, qq = U % 4;
        if (qd == qq) {
#pragma unroll
          for (int q = 0; q < S4; ++q)
            if (q == qp) {
#pragma unroll
              for (int t = 0; t < R16; ++t) {
                if (t + ts < R16) {
                  const int row = 16 * ts + li + 16 * t;
                  pcol[row] = xs[q][t];
                  if (gsrc) xs[q][t] = gsrc[row];
                }
              }
            }
        }
      } else {
        double *src = colptr(U);
        for (int row = lane; row < LD; row += kWave) {
          pcol[row] = src[row];
          if (gsrc) src[row] = gsrc[row];
        }
      }
      if (lane == 0) {
        perm[s] = P;
        if (g >= 0) {  // slot U takes column scol[g]; g (the last of glist) leaves the global tier
          scol[U] = scol[g];
          sn[U] = sn[g];
          scol[g] = -1;
          sn[g] = -1.0;
          gcnt[0] = gc - 1;
        } else {
          sn[U] = -1.0;
          scol[U] = -1;
          if (U < NREG) regact[owner] &= ~(1u << (U - owner * 4 * S4));
          if (U >= gbase) {  // swap-remove U from glist
            const int k = gpos[U], last = glist[gc - 1];
            glist[k] = last;
            gpos[last] = k;
            gcnt[0] = gc - 1;
          }
        }
      }
    }
    __syncthreads();

    // ---- reflector (wave 0, 64-lane layout) into vabs
    if (w == 0) {
      double x[TR];
#pragma unroll
      for (int t = 0; t < TR; ++t) x[t] = pcol[lane + kWave * t];
      // the whole row range 0..64 TR - 1 of vabs is written (zero outside [s, nr)); dg is
      // the new diagonal entry
      double dg;
      const double th = reflect_rows<TR>(x, 0, s, nr, vabs, &dg);
      if (lane == 0) {
        t1[s] = th;
        ds[s] = (dg < 0.0) ? -1.0 : 1.0;
        red[16] = dg;
      }
    }
    __syncthreads();

    // ---- column s of the R slot (last wave): the pivot column's R entries from Rrow and its
    // diagonal with normalised signs, the reflector below
    if (w == NW - 1) {
      const double dg = red[16];
      for (int row = lane; row < nr; row += kWave)
        R[(int64_t)s * n + row] = (row < s) ? ds[row] * Rrow[(int64_t)P * n + row]
                                            : (row == s) ? ds[s] * dg : vabs[row];
    }

    // ---- every active column takes the reflector, gives up row s (entry 0 of lane s % 16),
    // and has its norm recomputed from its entries below the pivot row
    const double th = t1[s];
    double vr[R16];
#pragma unroll
    for (int t = 0; t < R16; ++t) vr[t] = vabs[16 * ts + li + 16 * t];
    {
      const unsigned act = regact[w];
      double f[S4];
#pragma unroll
      for (int q = 0; q < S4; ++q) {
        f[q] = 0.0;
#pragma unroll
        for (int t = 0; t < R16; ++t) f[q] = fma(vr[t], xs[q][t], f[q]);
      }
#pragma unroll
      for (int q = 0; q < S4; ++q) f[q] = row16_sum(f[q]);
#pragma unroll
      for (int q = 0; q < S4; ++q) {
        const bool on = (act >> (4 * q + qd)) & 1u;
        const double g = on ? -th * f[q] : 0.0;
#pragma unroll
        for (int t = 0; t < R16; ++t) xs[q][t] = fma(g, vr[t], xs[q][t]);
        const double ext = xs[q][0];
        if (li == ls) xs[q][0] = 0.0;
        double ss = 0.0;
#pragma unroll
        for (int t = 0; t < R16; ++t) ss = fma(xs[q][t], xs[q][t], ss);
        f[q] = ss;
        if (on && li == ls) Rrow[(int64_t)scol[(w * S4 + q) * 4 + qd] * n + s] = ext;
      }
#pragma unroll
      for (int q = 0; q < S4; ++q) f[q] = row16_sum(f[q]);
#pragma unroll
      for (int q = 0; q < S4; ++q) {
        if ((act >> (4 * q + qd)) & 1u) {
          const int u = (w * S4 + q) * 4 + qd;
          const double nv = sqrt(f[q]);
          track(nv, scol[u], u);
          if (li == 0) sn[u] = nv;
        }
      }
    }
    // LDS tier, then the global tier (by glist): one column per group of 16 lanes, loaded
    // into the same window layout; rows below the window are zero in storage and are
    // neither read nor written
    for (int k0 = 4 * w; k0 < nl + gcnt[0]; k0 += 4 * NW) {
      const int kk = k0 + qd;
      const int gcv = gcnt[0];
      int u = -1;
      if (kk < nl) u = NREG + kk;
      else if (kk < nl + gcv) u = glist[kk - nl];
      const bool live = u >= 0 && sn[u] >= 0.0;
      double *col = live ? colptr(u) : pcol;  // a dead group reads pcol and writes nothing
      double x[R16];
      double f = 0.0;
#pragma unroll
      for (int t = 0; t < R16; ++t) {
        x[t] = (t + ts < R16) ? col[16 * ts + li + 16 * t] : 0.0;
        f = fma(vr[t], x[t], f);
      }
      f = row16_sum(f);
      const double g = live ? -th * f : 0.0;
#pragma unroll
      for (int t = 0; t < R16; ++t) x[t] = fma(g, vr[t], x[t]);
      const double ext = x[0];
      if (li == ls) x[0] = 0.0;
      double ss = 0.0;
#pragma unroll
      for (int t = 0; t < R16; ++t) ss = fma(x[t], x[t], ss);
      ss = row16_sum(ss);
      if (live) {
#pragma unroll
        for (int t = 0; t < R16; ++t)
          if (t + ts < R16) col[16 * ts + li + 16 * t] = x[t];
        const int c = scol[u];
        const double nv = sqrt(ss);
        track(nv, c, u);
        if (li == ls) Rrow[(int64_t)c * n + s] = ext;
        if (li == 0) sn[u] = nv;
      }
    }
    publish();
    __syncthreads();
  }

  // ---- outputs: the rest of the R slot cleared, kept ids, scalars
  for (int64_t e = tid; e < (int64_t)n * n; e += NT) {
    const int q = (int)(e / n), row = (int)(e % n);
    if (q >= r || row >= nr) R[e] = 0.0;
  }
  if (tid == 0) rank_out[j] = r;
  for (int q = tid; q < n; q += NT) {
    kept[B.f0 + q] = (q < r) ? perm[q] : -1;
    if (q < r) {
      tau1[B.f0 + q] = t1[q];
      dsgn[B.f0 + q] = ds[q];
    }
  }
}

// ---------------------------------------------------------------- Q1 = H'_0..H'_{r-1} [I_r; 0]
// Backward over panels of nb reflectors (read from below the diagonal of the R slot, which
// is cleared as it is consumed); the result Z (nr x r, ld nr) in the block's slot W2.
template <int R16>
__global__ __launch_bounds__(NT) void rf_formq1(rfm_layout L, const int32_t *__restrict__ rank,
                                                double *__restrict__ Rout, const double *__restrict__ tau1,
                                                double *__restrict__ W2, int nb,
                                                const int32_t *__restrict__ order) {
  extern __shared__ double lds[];
  constexpr int LD = 16 * R16;  // reflector rows, zero-padded
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int li = lane & 15, qd = lane >> 4;
  const int j = order ? order[blockIdx.x] : blockIdx.x;
  const Blk B = blk(L, j);
  const int n = B.n, nr = B.nr, r = rank[j];
  if (r == 0) return;
  double *__restrict__ R = Rout + B.rsq;
  double *__restrict__ Z = W2 + B.rsq;
  double *tl = lds;       // [nb]
  double *Vp = lds + 16;  // [nb][LD]
  for (int p = ((r - 1) / nb) * nb; p >= 0; p -= nb) {
    const int b = min(nb, r - p);
    for (int e = tid; e < b * LD; e += NT) {
      const int i = e / LD, rr = e % LD;
      const int q = p + i, row = p + rr;
      Vp[e] = (row >= nr || rr < i) ? 0.0 : (rr == i) ? 1.0 : R[(int64_t)q * n + row];
    }
    for (int i = tid; i < b; i += NT) tl[i] = tau1[B.f0 + p + i];
    __syncthreads();
    for (int e = tid; e < b * (nr - p); e += NT) {
      const int i = e / (nr - p), rr = e % (nr - p);
      if (rr > i) R[(int64_t)(p + i) * n + p + rr] = 0.0;
    }
    // one column per group of 16 lanes: columns >= p + b are already formed, the panel's
    // own columns start as unit vectors
    for (int c0 = p + 4 * w; c0 < r; c0 += 4 * NW) {
      const int k = c0 + qd;
      double x[R16];
#pragma unroll
      for (int t = 0; t < R16; ++t) {
        const int row = p + li + 16 * t;
        double v = 0.0;
        if (k < r && row < nr) v = (k < p + b) ? (row == k ? 1.0 : 0.0) : Z[(int64_t)k * nr + row];
        x[t] = v;
      }
      for (int i = b - 1; i >= 0; --i) apply_refl16<R16>(x, Vp + i * LD, tl[i]);
      if (k < r) {
#pragma unroll
        for (int t = 0; t < R16; ++t) {
          const int row = p + li + 16 * t;
          if (row < nr) Z[(int64_t)k * nr + row] = x[t];
        }
        if (k < p + b)
          for (int row = li; row < p; row += 16) Z[(int64_t)k * nr + row] = 0.0;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- Q0 = H_0..H_{nr-1} [I; 0]
// Every panel re-reads and rewrites the formed columns right of it, so the panel is as wide as
// the LDS holds (not limited by registers, unlike the factorisation's panels).
constexpr int kFormq0MaxNb = 32;
// In place in the Q slot, backward over panels: the panel's reflectors go to LDS first, so
// its columns can be overwritten; columns left of the panel still hold their reflectors.
template <int T, int G>
__global__ __launch_bounds__(NT) void rf_formq0(rfm_layout L, const int32_t *__restrict__ rank,
                                                double *__restrict__ Q, const double *__restrict__ tau0, int nb,
                                                const int32_t *__restrict__ order) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  {
    const int j = order ? order[blockIdx.x] : blockIdx.x;
    const Blk B = blk(L, j);
    const int m = B.m, nr = B.nr;
    if (rank[j] == 0) return;
    double *__restrict__ A = Q + B.base;
    double *tl = lds;                 // [nb], nb <= kFormq0MaxNb
    double *Vp = lds + kFormq0MaxNb;  // [nb][ldv]
    constexpr bool Q16 = T <= 12;     // one column per 16 lanes
    const int ldv = Q16 ? 64 * T : m;  // reflector rows zero-padded to 64 T in that case
    for (int p = ((nr - 1) / nb) * nb; p >= 0; p -= nb) {
      const int b = min(nb, nr - p);
      for (int e = tid; e < b * ldv; e += NT) {
        const int i = e / ldv, rr = e % ldv;
        const int k = p + i, row = p + rr;
        Vp[e] = (row >= m || rr < i) ? 0.0 : (rr == i) ? 1.0 : A[(int64_t)k * m + row];
      }
      for (int i = tid; i < b; i += NT) tl[i] = tau0[B.f0 + p + i];
      __syncthreads();
      if constexpr (Q16) {
        constexpr int R16 = 4 * T;
        const int li = lane & 15, qd = lane >> 4;
        for (int c0 = p + 4 * w; c0 < nr; c0 += 4 * NW) {
          const int k = c0 + qd;
          double x[R16];
#pragma unroll
          for (int t = 0; t < R16; ++t) {
            const int row = p + li + 16 * t;
            double v = 0.0;
            if (k < nr && row < m) v = (k < p + b) ? (row == k ? 1.0 : 0.0) : A[(int64_t)k * m + row];
            x[t] = v;
          }
          for (int i = b - 1; i >= 0; --i) apply_refl16<R16>(x, Vp + (int64_t)i * ldv, tl[i]);
          if (k < nr) {
#pragma unroll
            for (int t = 0; t < R16; ++t) {
              const int row = p + li + 16 * t;
              if (row < m) A[(int64_t)k * m + row] = x[t];
            }
            if (k < p + b)
              for (int row = li; row < p; row += 16) A[(int64_t)k * m + row] = 0.0;
          }
        }
      } else
      for (int c0 = p + w * G; c0 < nr; c0 += NW * G) {
        double x[G][T];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int k = c0 + g;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int row = p + lane + kWave * t;
            double v = 0.0;
            if (k < nr && row < m) v = (k < p + b) ? (row == k ? 1.0 : 0.0) : A[(int64_t)k * m + row];
            x[g][t] = v;
          }
        }
        for (int i = b - 1; i >= 0; --i) {
          if constexpr (T >= 24) {
            apply_refl_lds<T, G>(x, Vp + (int64_t)i * ldv, m - p, tl[i]);
          } else {
            double vr[T];
#pragma unroll
            for (int t = 0; t < T; ++t) {
              const int rr = lane + kWave * t;
              vr[t] = (p + rr < m) ? Vp[(int64_t)i * ldv + rr] : 0.0;
            }
            apply_refl<T, G>(x, vr, tl[i]);
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int k = c0 + g;
          if (k < nr) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
              const int row = p + lane + kWave * t;
              if (row < m) A[(int64_t)k * m + row] = x[g][t];
            }
            if (k < p + b)
              for (int row = lane; row < p; row += kWave) A[(int64_t)k * m + row] = 0.0;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- Q_hat = Q0 Q1 D in place
// Row tiles of RT = 16384 / CP rows of the RT x CP output (CP >= r), computed with FP64
// matrix cores: each wave owns 2 x 4 tiles of 16 x 16 and accumulates them with
// v_mfma_f64_16x16x4f64 over slices of 16 of the nr inner indices staged in LDS (Q0 rows
// As[k][row], Q1 rows Zs[k][q]; the next slice's loads are in flight while one is
// multiplied).  Operand layout of the instruction: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16x4 by 4x16 product and holds D[l / 16 + 4 v][l % 16] in element v
// of its accumulator.  The tile is written (times the sign normalisation) only after its last
// slice, so the rows it overwrites have been read.
typedef double d4_t __attribute__((ext_vector_type(4)));

template <int CP, int RA>
__global__ __launch_bounds__(NT) void rf_gemm(rfm_layout L, const int32_t *__restrict__ rank,
                                              double *__restrict__ Q, const double *__restrict__ W2,
                                              const double *__restrict__ dsgn, const int32_t *__restrict__ order) {
  // row tiles of RT rows; each wave holds RA x 4 output tiles of 16 x 16, the waves laid out
  // WR x (NW / WR); Z (Q1 D) is read once per row tile, so taller tiles read it fewer times
  constexpr int WR = NW * 64 / CP, RT = 16 * RA * WR, KC = 16;
  __shared__ double As[KC][RT];
  __shared__ double Zs[KC][CP];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int wr = w % WR, wc = w / WR;
  const int li = lane & 15, lk = lane >> 4;
  const int j = order ? order[blockIdx.x] : blockIdx.x;
  const Blk B = blk(L, j);
  const int m = B.m, nr = B.nr, r = rank[j];
  if (r == 0) return;
  double *__restrict__ A = Q + B.base;
  const double *__restrict__ Z = W2 + B.rsq;
  constexpr int NA = KC * RT / NT, NZ = KC * CP / NT;
  for (int i0 = 0; i0 < m; i0 += RT) {
    d4_t acc[RA][4];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
    double pa[NA], pz[NZ];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        const int e = tid + u * NT, kk = e / RT, rr = e % RT;
        pa[u] = (k0 + kk < nr && i0 + rr < m) ? A[(int64_t)(k0 + kk) * m + i0 + rr] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NZ; ++u) {
        const int e = tid + u * NT, q = e / KC, kk = e % KC;
        pz[u] = (k0 + kk < nr && q < r) ? Z[(int64_t)q * nr + k0 + kk] : 0.0;
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < nr; k0 += KC) {
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        const int e = tid + u * NT;
        As[e / RT][e % RT] = pa[u];
      }
#pragma unroll
      for (int u = 0; u < NZ; ++u) {
        const int e = tid + u * NT;
        Zs[e % KC][e / KC] = pz[u];
      }
      __syncthreads();
      if (k0 + KC < nr) fetch(k0 + KC);
#pragma unroll
      for (int kq = 0; kq < KC; kq += 4) {
        double av[RA], bv[4];
#pragma unroll
        for (int a = 0; a < RA; ++a) av[a] = As[kq + lk][(RA * wr + a) * 16 + li];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Zs[kq + lk][(4 * wc + b) * 16 + li];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int q = (4 * wc + b) * 16 + li;
      if (q < r) {
        const double sg = dsgn[B.f0 + q];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = i0 + (RA * wr + a) * 16 + lk + 4 * v;
            if (row < m) A[(int64_t)q * m + row] = sg * acc[a][b][v];
          }
      }
    }
  }
}

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Ws {
  double *tau0, *tau1, *dsgn, *W1, *W2, *W3;
};

// Rows per lane of the pivoted QR's 16-lane layout for blocks of up to nr_max rows of R0.
int r16_of(int nr_max) { return nr_max <= 64 ? 4 : nr_max <= 128 ? 8 : nr_max <= 256 ? 16 : nr_max <= 320 ? 20 : 32; }

int nr_max_of(const rfm_layout *L) { return std::max(1, std::min(L->max_rows, L->max_cols)); }

size_t carve(const rfm_layout *L, char *base, Ws *W) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base ? base + off : nullptr;
    off += al256(bytes);
    return p;
  };
  const size_t nc = (size_t)(L->ncols > 0 ? L->ncols : 1), nq = (size_t)(L->nrsq > 0 ? L->nrsq : 1);
  Ws w;
  w.tau0 = (double *)take(nc * sizeof(double));
  w.tau1 = (double *)take(nc * sizeof(double));
  w.dsgn = (double *)take(nc * sizeof(double));
  w.W1 = (double *)take(nc * 16 * (size_t)r16_of(nr_max_of(L)) * sizeof(double));
  w.W2 = (double *)take(nq * sizeof(double));
  w.W3 = (double *)take(nq * sizeof(double));
  if (W) *W = w;
  return off;
}

constexpr int g_of(int T) { return T <= 4 ? 8 : T <= 12 ? 4 : T <= 16 ? 2 : 1; }
constexpr int npc_of(int T) { return T <= 16 ? 2 : 1; }

template <class K>
rfm_status prep(K kern, size_t lds) {
  RFM_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return RFM_OK;
}

template <int T>
rfm_status launch_tall(const RfirstArgs &a, const Ws &W, bool first) {
  const rfm_layout *L = a.L;
  constexpr int GG = g_of(T);
  const dim3 grid((unsigned)L->J);
  // reflector rows in LDS: zero-padded to 64 T for the 16-lane layout (T <= 12), else
  // max_rows; panel width nb from the LDS budget, at most the panel columns the waves hold in
  // registers (the tall blocks of the 3D workload, 2,744 rows, fit 7 reflectors)
  const size_t ldv = (T <= 12) ? (size_t)64 * T : (size_t)std::max(1, L->max_rows);
  // dynamic LDS for the reflector panels: all but 2 KB of the 160 KB a workgroup may take
  constexpr size_t tall_lds = 158 * 1024;
  int nb = (int)((tall_lds - (size_t)L->max_cols * sizeof(double)) / (ldv * sizeof(double)));
  nb = std::max(1, std::min(npc_of(T) * NW, nb));
  if (first) {
    const size_t lds = ((size_t)L->max_cols + (size_t)nb * ldv) * sizeof(double);
    auto kern = rf_qr<T, GG, npc_of(T)>;
    rfm_status s = prep(kern, lds);
    if (s != RFM_OK) return s;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, a.st, *L, a.M, a.Q, W.tau0, nb, a.order);
  } else {
    int nbq = (int)((tall_lds - kFormq0MaxNb * sizeof(double)) / (ldv * sizeof(double)));
    nbq = std::max(1, std::min(kFormq0MaxNb, nbq));
    nb = nbq;
    const size_t lds = (kFormq0MaxNb + (size_t)nb * ldv) * sizeof(double);
    auto kern = rf_formq0<T, GG>;
    rfm_status s = prep(kern, lds);
    if (s != RFM_OK) return s;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, a.st, *L, a.rank, a.Q, W.tau0, nb, a.order);
  }
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

rfm_status dispatch_tall(const RfirstArgs &a, const Ws &W, bool first) {
  const int mr = a.L->max_rows;
  if (mr <= 64) return launch_tall<1>(a, W, first);
  if (mr <= 128) return launch_tall<2>(a, W, first);
  if (mr <= 256) return launch_tall<4>(a, W, first);
  if (mr <= 512) return launch_tall<8>(a, W, first);
  if (mr <= 768) return launch_tall<12>(a, W, first);
  if (mr <= 1024) return launch_tall<16>(a, W, first);
  if (mr <= 1536) return launch_tall<24>(a, W, first);
  if (mr <= 2048) return launch_tall<32>(a, W, first);
  return launch_tall<48>(a, W, first);
}

template <int R16, int S4>
rfm_status launch_small(const RfirstArgs &a, const Ws &W, int nr_max) {
  constexpr int TR = R16 / 4;
  const rfm_layout *L = a.L;
  const dim3 grid((unsigned)L->J);
  const int nmax = L->max_cols;
  const int nreg = NW * S4 * 4;
  const size_t small = qrcp_small_bytes(nmax, nreg, R16);
  const int64_t want = (int64_t)std::max(0, nmax - nreg) * 16 * R16;
  int64_t tier = (int64_t)((kLdsCap - small) / sizeof(double));
  if (tier > want) tier = want;
  if (tier < 0) tier = 0;
  const size_t lds = small + (size_t)tier * sizeof(double);
  {
    auto kern = rf_qrcp<R16, S4>;
    rfm_status s = prep(kern, lds);
    if (s != RFM_OK) return s;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, a.st, *L, (const double *)a.Q, a.tau, a.rank, a.kept, a.R,
                       a.ratios, W.tau1, W.dsgn, W.W1, W.W3, tier, a.order);
    RFM_LAUNCH_CHECK();
  }
  {
    const int nb = 16;
    const size_t lds1 = (16 + (size_t)nb * 16 * R16) * sizeof(double);
    auto kern = rf_formq1<R16>;
    rfm_status s = prep(kern, lds1);
    if (s != RFM_OK) return s;
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds1, a.st, *L, a.rank, a.R, W.tau1, W.W2, nb, a.order);
    RFM_LAUNCH_CHECK();
  }
  return RFM_OK;
}

rfm_status dispatch_small(const RfirstArgs &a, const Ws &W, int nr_max) {
  switch (r16_of(nr_max)) {
    case 4: return launch_small<4, 8>(a, W, nr_max);
    case 8: return launch_small<8, 8>(a, W, nr_max);
    case 16: return launch_small<16, 4>(a, W, nr_max);
    case 20: return launch_small<20, 3>(a, W, nr_max);
    default: return launch_small<32, 1>(a, W, nr_max);
  }
}

}  // namespace

bool rfirst_supported(const rfm_layout *L) { return L && L->max_cols <= 512 && L->max_rows <= 3072; }

size_t rfirst_ws_bytes(const rfm_layout *L) { return carve(L, nullptr, nullptr); }

rfm_status rrqr_rfirst(const RfirstArgs &a) {
  const rfm_layout *L = a.L;
  if (!rfirst_supported(L)) return fail(RFM_EUNSUPPORTED, "rfm_rrqr_filter: the R-first form needs max_cols <= 512");
  if (!a.ws || a.ws_bytes < rfirst_ws_bytes(L))
    return fail(RFM_EINVAL, "rfm_rrqr_filter: workspace too small (rfm_rrqr_ws_bytes)");
  if (L->J < 1) return RFM_OK;
  Ws W;
  carve(L, (char *)a.ws, &W);
  const int nr_max = nr_max_of(L);
  rfm_status s = dispatch_tall(a, W, true);
  if (s != RFM_OK) return s;
  s = dispatch_small(a, W, nr_max);
  if (s != RFM_OK) return s;
  s = dispatch_tall(a, W, false);
  if (s != RFM_OK) return s;
  const dim3 grid((unsigned)L->J);
  if (nr_max <= 256)
    hipLaunchKernelGGL((rf_gemm<256, 3>), grid, dim3(NT), 0, a.st, *L, a.rank, a.Q, W.W2, W.dsgn, a.order);
  else
    hipLaunchKernelGGL((rf_gemm<512, 2>), grid, dim3(NT), 0, a.st, *L, a.rank, a.Q, W.W2, W.dsgn, a.order);
  RFM_LAUNCH_CHECK();
  return RFM_OK;
}

}  // namespace rfm
