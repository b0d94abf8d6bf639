// Assembly of the weighted ELM-FBPINN least-squares system on gfx950.
//
// window_table: one thread per global row r.  Walks the subdomains covering r in
//   ascending j, accumulates the unnormalised windows what_j and their first and pure
//   second derivatives, then writes the normalised window w_j = what_j / sum_i what_i
//   and its derivatives (quotient rule) for every incidence (j, r) -- the partition of
//   unity of eq. used_window_function_nd -- and h_r = s_r rhs_r (eq. ELMFBPINN_ls).  A
//   hard-constraint ansatz factor g is folded in here: the table holds g w_j and its
//   derivatives, so the entries below see the product g w_j phi_jk unchanged.
// assemble_entries: lane <-> row of one block, so the column-major block is written
//   with coalesced 64-wide stores; each thread produces a run of features for its row,
//   reusing the row's point and window data.  Entry = s_r Op_r[w_j phi_jk](x_r) by the
//   product rule with phi = Xi(w . xn + b), xn = (x - mu_j)/hw_j (eq. fcn_depth_h), Xi the
//   problem's activation (tanh, sigmoid or sin); with a depth-h network the features act on the
//   last hidden layer, evaluated per row with forward-mode derivatives (hidden_forward).
// Both run in binary64, or in binary32 for the precision form (rfm_assemble_low), whose
// entries are stored as binary32 or bfloat16.
#include "common.hpp"

namespace rfm {
namespace {

constexpr int kRowsPerBlock = 256;
constexpr int kFeatPerThread = 32;

// Tc: the arithmetic (double, or float for the precision form); inputs are read as double
// and rounded to Tc once.
template <int D, typename Tc>
__device__ __forceinline__ void window_factors(const Tc *xr, const double *mu,
                                               const double *hw, Tc &W, Tc *dW,
                                               Tc *ddW) {
  const Tc pi = (Tc)3.141592653589793;
  Tc f[D], f1[D], f2[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const Tc h = (Tc)hw[i];
    const Tc t = (xr[i] - (Tc)mu[i]) / h;
    const Tc cs = cos(pi * t);
    const Tc c = (Tc)1 + cs;
    const Tc s = sin(pi * t);
    f[i] = c * c;
    f1[i] = -((Tc)2 * pi / h) * s * c;
    f2[i] = ((Tc)2 * pi * pi / (h * h)) * (s * s - cs * c);
  }
  W = (Tc)1;
#pragma unroll
  for (int i = 0; i < D; ++i) W *= f[i];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Tc others = (Tc)1;
#pragma unroll
    for (int l = 0; l < D; ++l)
      if (l != i) others *= f[l];
    dW[i] = f1[i] * others;
    ddW[i] = f2[i] * others;
  }
}

template <int D, typename Tc>
__global__ __launch_bounds__(256) void window_table(rfm_layout L, rfm_problem P, Tc *win,
                                                    double *h) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= L.N) return;
  h[r] = P.weight[r] * P.rhs[r];
  Tc xr[D];
#pragma unroll
  for (int i = 0; i < D; ++i) xr[i] = (Tc)P.x[r * D + i];
  Tc S = 0, dS[D], ddS[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dS[i] = ddS[i] = 0;
  const int64_t q0 = L.rinc_off[r], q1 = L.rinc_off[r + 1];
  for (int64_t q = q0; q < q1; ++q) {
    const int64_t p = L.rinc[q];
    const int32_t j = L.inc_blk[p];
    Tc W, dW[D], ddW[D];
    window_factors<D, Tc>(xr, P.mu + (int64_t)j * D, P.hw + (int64_t)j * D, W, dW, ddW);
    S += W;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      dS[i] += dW[i];
      ddS[i] += ddW[i];
    }
  }
  // ansatz factor: g, d_i g, d_ii g (g = 1 without one)
  Tc g = (Tc)1, dg[D], ddg[D];
#pragma unroll
  for (int i = 0; i < D; ++i) dg[i] = ddg[i] = 0;
  if (P.ansatz) {
    const double *ar = P.ansatz + r * (1 + 2 * D);
    g = (Tc)ar[0];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      dg[i] = (Tc)ar[1 + i];
      ddg[i] = (Tc)ar[1 + D + i];
    }
  }
  for (int64_t q = q0; q < q1; ++q) {
    const int64_t p = L.rinc[q];
    const int32_t j = L.inc_blk[p];
    Tc W, dW[D], ddW[D];
    window_factors<D, Tc>(xr, P.mu + (int64_t)j * D, P.hw + (int64_t)j * D, W, dW, ddW);
    const Tc w = W / S;
    Tc *out = win + p * (1 + 2 * D);
    if (!P.ansatz) {
      out[0] = w;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const Tc dw = (dW[i] - w * dS[i]) / S;
        out[1 + i] = dw;
        out[1 + D + i] = (ddW[i] - (Tc)2 * dw * dS[i] - w * ddS[i]) / S;
      }
    } else {
      out[0] = g * w;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        const Tc dw = (dW[i] - w * dS[i]) / S;
        const Tc ddw = (ddW[i] - (Tc)2 * dw * dS[i] - w * ddS[i]) / S;
        out[1 + i] = dg[i] * w + g * dw;
        out[1 + D + i] = ddg[i] * w + (Tc)2 * dg[i] * dw + g * ddw;
      }
    }
  }
}

// Output element: binary64, binary32, or bfloat16 (round to nearest even on the binary32
// value, kept as its upper 16 bits).
template <typename To> struct Out;
template <> struct Out<double> { static __device__ double put(double v) { return v; } };
template <> struct Out<float> { static __device__ float put(float v) { return v; } };
template <> struct Out<uint16_t> {
  static __device__ uint16_t put(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  }
};

// Hidden layers of a depth-h subdomain network (eq. fcn_depth_h) with forward-mode first and
// pure second derivatives in x: z, d_a z, d_aa z of the last hidden layer, width H <= kHMax
// (entries u >= H stay 0).  z0 = xn has d_a z0 = e_a / hw_a and no second derivative.
template <int D, typename Tc>
__device__ __forceinline__ void hidden_forward(const rfm_problem &P, int j, const Tc *xn, const Tc *hwj,
                                               Tc (&z)[kHMax], Tc (&dz)[D][kHMax], Tc (&ddz)[D][kHMax]) {
  const int H = P.hidden;
  const double *net = P.net + (int64_t)j * net_stride(P, D);
  // layer 1 on the normalised input
#pragma unroll
  for (int u = 0; u < kHMax; ++u) {
    z[u] = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) dz[a][u] = ddz[a][u] = 0;
    if (u < H) {
      Tc s = (Tc)net[H * D + u];
#pragma unroll
      for (int a = 0; a < D; ++a) s += (Tc)net[u * D + a] * xn[a];
      Tc t, g, gg;
      activation3<Tc>(P.activation, s, t, g, gg);
      z[u] = t;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const Tc sc = (Tc)net[u * D + a] / hwj[a];
        dz[a][u] = g * sc;
        ddz[a][u] = gg * (sc * sc);
      }
    }
  }
  net += H * D + H;
  // layers 2 .. h-1
  for (int l = 2; l < P.depth; ++l, net += H * H + H) {
    Tc nz[kHMax], ndz[D][kHMax], nddz[D][kHMax];
#pragma unroll
    for (int u = 0; u < kHMax; ++u) {
      nz[u] = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) ndz[a][u] = nddz[a][u] = 0;
      if (u < H) {
        Tc s = (Tc)net[H * H + u], ds[D], dds[D];
#pragma unroll
        for (int a = 0; a < D; ++a) ds[a] = dds[a] = 0;
#pragma unroll
        for (int v = 0; v < kHMax; ++v) {
          if (v < H) {
            const Tc wv = (Tc)net[u * H + v];
            s += wv * z[v];
#pragma unroll
            for (int a = 0; a < D; ++a) {
              ds[a] += wv * dz[a][v];
              dds[a] += wv * ddz[a][v];
            }
          }
        }
        Tc t, g, gg;
        activation3<Tc>(P.activation, s, t, g, gg);
        nz[u] = t;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          ndz[a][u] = g * ds[a];
          nddz[a][u] = gg * ds[a] * ds[a] + g * dds[a];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < kHMax; ++u) {
      z[u] = nz[u];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        dz[a][u] = ndz[a][u];
        ddz[a][u] = nddz[a][u];
      }
    }
  }
}

// DEEP: features on the last hidden layer of a depth-h network (P.depth > 1).
template <int D, typename Tc, typename To, bool DEEP>
__global__ __launch_bounds__(kRowsPerBlock) void assemble_entries(rfm_layout L, rfm_problem P,
                                                                  const Tc *win, To *M) {
  const int j = blockIdx.z;
  const int64_t r0 = L.row_off[j];
  const int m = (int)(L.row_off[j + 1] - r0);
  const int i = blockIdx.x * kRowsPerBlock + threadIdx.x;
  const int64_t f0 = L.feat_off[j];
  const int K = (int)(L.feat_off[j + 1] - f0);
  const int k0 = blockIdx.y * kFeatPerThread;
  if (i >= m || k0 >= K) return;
  const int64_t p = r0 + i;
  const int32_t r = L.rows[p];
  Tc xn[D], hwj[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const Tc h = (Tc)P.hw[(int64_t)j * D + a];
    xn[a] = ((Tc)P.x[(int64_t)r * D + a] - (Tc)P.mu[(int64_t)j * D + a]) / h;
    hwj[a] = h;
  }
  const Tc *wp = win + p * (1 + 2 * D);
  const Tc w = wp[0];
  Tc dw[D], ddw[D];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    dw[a] = wp[1 + a];
    ddw[a] = wp[1 + D + a];
  }
  int op = P.rowop[r];
  const Tc sr = (Tc)P.weight[r];
  const Tc kappa = (Tc)P.kappa, ksq = (Tc)P.ksq;
  // constant-coefficient operator of the table: c0 u + sum_a (c1_a d_a u + c2_a d_aa u)
  Tc c0 = 0, c1[D], c2[D];
#pragma unroll
  for (int a = 0; a < D; ++a) c1[a] = c2[a] = 0;
  if (op >= RFM_OP_COEF) {
    const int t = op - RFM_OP_COEF;
    if (t < P.nopcoef) {
      const double *cr = P.opcoef + (int64_t)t * (1 + 2 * D);
      c0 = (Tc)cr[0];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        c1[a] = (Tc)cr[1 + a];
        c2[a] = (Tc)cr[1 + D + a];
      }
    } else {
      op = RFM_OP_VALUE;
    }
  }
  constexpr int HM = DEEP ? kHMax : 1;
  Tc z[HM], dz[D][HM], ddz[D][HM];
  if constexpr (DEEP) hidden_forward<D, Tc>(P, j, xn, hwj, z, dz, ddz);
  To *out = M + L.blk_off[j] + (int64_t)i;
  const int k1 = min(K, k0 + kFeatPerThread);
  for (int k = k0; k < k1; ++k) {
    Tc t, dphi[D], ddphi[D];  // phi and its derivatives in x
    if constexpr (DEEP) {
      const int H = P.hidden;
      const double *wk = P.w + (f0 + k) * H;
      Tc s = (Tc)P.b[f0 + k], ds[D], dds[D];
#pragma unroll
      for (int a = 0; a < D; ++a) ds[a] = dds[a] = 0;
#pragma unroll
      for (int u = 0; u < kHMax; ++u) {
        if (u < H) {
          const Tc wu = (Tc)wk[u];
          s += wu * z[u];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            ds[a] += wu * dz[a][u];
            dds[a] += wu * ddz[a][u];
          }
        }
      }
      Tc g, gg;
      activation3<Tc>(P.activation, s, t, g, gg);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        dphi[a] = g * ds[a];
        ddphi[a] = gg * ds[a] * ds[a] + g * dds[a];
      }
    } else {
      const double *wk = P.w + (f0 + k) * D;
      Tc s = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) s += xn[a] * (Tc)wk[a];
      s += (Tc)P.b[f0 + k];
      Tc g, gg;  // phi, phi', phi'' of the activation at s
      activation3<Tc>(P.activation, s, t, g, gg);
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const Tc sc = (Tc)wk[a] / hwj[a];
        dphi[a] = g * sc;
        ddphi[a] = gg * (sc * sc);
      }
    }
    const Tc psi = w * t;
    Tc lap = 0, spatial = 0, dlast = 0, gen = c0 * psi;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const Tc dpsi = dw[a] * t + w * dphi[a];
      const Tc ddpsi = ddw[a] * t + (Tc)2 * dw[a] * dphi[a] + w * ddphi[a];
      lap += ddpsi;
      if (a < D - 1) spatial += ddpsi;
      if (a == D - 1) dlast = dpsi;
      gen += c1[a] * dpsi + c2[a] * ddpsi;
    }
    Tc v;
    switch (op) {
      case RFM_OP_NEG_LAPLACE: v = -lap; break;
      case RFM_OP_HEAT: v = dlast - kappa * (D > 1 ? spatial : (Tc)0); break;
      case RFM_OP_HELMHOLTZ: v = lap + ksq * psi; break;
      default: v = (op >= RFM_OP_COEF) ? gen : psi; break;
    }
    out[(int64_t)k * m] = Out<To>::put(sr * v);
  }
}

template <int D, typename Tc, typename To>
rfm_status launch(const rfm_layout *L, const rfm_problem *P, To *M, double *h, Tc *win, hipStream_t st) {
  hipLaunchKernelGGL((window_table<D, Tc>), dim3(ceil_div(L->N, 256)), dim3(256), 0, st, *L, *P, win, h);
  RFM_LAUNCH_CHECK();
  if (L->max_rows > 0 && L->max_cols > 0) {
    dim3 grid(ceil_div(L->max_rows, kRowsPerBlock), ceil_div(L->max_cols, kFeatPerThread), L->J);
    if (P->depth > 1)
      hipLaunchKernelGGL((assemble_entries<D, Tc, To, true>), grid, dim3(kRowsPerBlock), 0, st, *L, *P, win, M);
    else
      hipLaunchKernelGGL((assemble_entries<D, Tc, To, false>), grid, dim3(kRowsPerBlock), 0, st, *L, *P, win, M);
    RFM_LAUNCH_CHECK();
  }
  return RFM_OK;
}

template <typename Tc, typename To>
rfm_status launch_d(const rfm_layout *L, const rfm_problem *P, To *M, double *h, void *ws, hipStream_t st) {
  Tc *win = (Tc *)ws;
  switch (L->d) {
    case 1: return launch<1, Tc, To>(L, P, M, h, win, st);
    case 2: return launch<2, Tc, To>(L, P, M, h, win, st);
    default: return launch<3, Tc, To>(L, P, M, h, win, st);
  }
}

rfm_status check_problem(const rfm_layout *L, const rfm_problem *P, const void *M, const double *h,
                         const void *ws, size_t ws_bytes, const char *who) {
  rfm_status s = check_layout(L, who);
  if (s != RFM_OK) return s;
  if (!P || !P->x || !P->rowop || !P->weight || !P->rhs || !P->mu || !P->hw || !P->w || !P->b)
    return fail(RFM_EINVAL, std::string(who) + ": null problem array");
  if (P->nopcoef < 0 || (P->nopcoef > 0 && !P->opcoef))
    return fail(RFM_EINVAL, std::string(who) + ": operator table size or pointer");
  if (P->activation < RFM_ACT_TANH || P->activation > RFM_ACT_SIN)
    return fail(RFM_EINVAL, std::string(who) + ": unknown activation");
  s = check_network(P, who);
  if (s != RFM_OK) return s;
  if (!h || (L->nnz > 0 && !M)) return fail(RFM_EINVAL, std::string(who) + ": null output");
  if (ws_bytes < rfm_assemble_ws_bytes(L) || (rfm_assemble_ws_bytes(L) > 0 && !ws))
    return fail(RFM_EINVAL, std::string(who) + ": workspace too small");
  return RFM_OK;
}

}  // namespace

rfm_status check_layout(const rfm_layout *L, const char *who) {
  if (!L) return fail(RFM_EINVAL, std::string(who) + ": null layout");
  if (L->d < 1 || L->d > 3) return fail(RFM_EINVAL, std::string(who) + ": d must be 1..3");
  if (L->J < 1 || L->N < 1) return fail(RFM_EINVAL, std::string(who) + ": empty layout");
  if (L->J > 65535) return fail(RFM_EUNSUPPORTED, std::string(who) + ": J > 65535");
  if (!L->row_off || !L->rows || !L->inc_blk || !L->rinc_off || !L->rinc || !L->feat_off ||
      !L->blk_off || !L->rsq_off)
    return fail(RFM_EINVAL, std::string(who) + ": null layout array");
  if (L->max_rows < 0 || L->max_cols < 0 || L->nnz < 0 || L->ncols < 0)
    return fail(RFM_EINVAL, std::string(who) + ": negative size");
  return RFM_OK;
}

}  // namespace rfm

extern "C" size_t rfm_assemble_ws_bytes(const rfm_layout *L) {
  if (!L) return 0;
  return (size_t)L->nnz_rows * (1 + 2 * (size_t)L->d) * sizeof(double);
}

extern "C" rfm_status rfm_assemble(const rfm_layout *L, const rfm_problem *P, double *M, double *h,
                                   void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s = check_problem(L, P, M, h, ws, ws_bytes, "rfm_assemble");
  if (s != RFM_OK) return s;
  return launch_d<double, double>(L, P, M, h, ws, (hipStream_t)stream);
}

extern "C" rfm_status rfm_assemble_low(const rfm_layout *L, const rfm_problem *P, int32_t dtype, void *M,
                                       double *h, void *ws, size_t ws_bytes, void *stream) {
  using namespace rfm;
  rfm_status s = check_problem(L, P, M, h, ws, ws_bytes, "rfm_assemble_low");
  if (s != RFM_OK) return s;
  if (dtype == RFM_F32) return launch_d<float, float>(L, P, (float *)M, h, ws, (hipStream_t)stream);
  if (dtype == RFM_BF16) return launch_d<float, uint16_t>(L, P, (uint16_t *)M, h, ws, (hipStream_t)stream);
  return fail(RFM_EINVAL, "rfm_assemble_low: dtype must be RFM_F32 or RFM_BF16");
}
