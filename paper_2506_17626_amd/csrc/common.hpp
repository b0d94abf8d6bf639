// Shared helpers of the HIP library: error plumbing, launch checks and wave64
// reductions for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "rfm.h"

namespace rfm {

void set_error(const std::string &msg);
rfm_status fail(rfm_status st, const std::string &msg);
rfm_status check_layout(const rfm_layout *L, const char *who);

#define RFM_HIP_TRY(expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::rfm::fail(RFM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define RFM_LAUNCH_CHECK()                                                         \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess)                                                          \
      return ::rfm::fail(RFM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

constexpr int kWave = 64;

// Butterfly sum over the 64 lanes of a wave; every lane receives the same value
// (each step adds the same two operands in both partner lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Sum over the 64 lanes of a wave through DPP row shifts and lane reads (no LDS traffic):
// an inclusive scan within each row of 16 lanes (shifts by 1, 2, 4, 8; lanes without a
// source add zero), then ((row0 + row1) + row2) + row3 from the rows' last lanes.  Every
// lane receives the same value; the order of the additions is fixed.
template <int CTRL>
__device__ __forceinline__ double dpp_row_shr(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_read(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_row_shr<0x111>(v);  // row_shr:1
  v += dpp_row_shr<0x112>(v);  // row_shr:2
  v += dpp_row_shr<0x114>(v);  // row_shr:4
  v += dpp_row_shr<0x118>(v);  // row_shr:8
  return ((lane_read(v, 15) + lane_read(v, 31)) + lane_read(v, 47)) + lane_read(v, 63);
}

// Two wave sums at once (the same fixed order as wave_sum_dpp for each), interleaved so
// that the two chains hide each other's latency.
__device__ __forceinline__ void wave_sum2_dpp(double &a, double &b) {
  a += dpp_row_shr<0x111>(a);
  b += dpp_row_shr<0x111>(b);
  a += dpp_row_shr<0x112>(a);
  b += dpp_row_shr<0x112>(b);
  a += dpp_row_shr<0x114>(a);
  b += dpp_row_shr<0x114>(b);
  a += dpp_row_shr<0x118>(a);
  b += dpp_row_shr<0x118>(b);
  const double a0 = lane_read(a, 15), b0 = lane_read(b, 15), a1 = lane_read(a, 31), b1 = lane_read(b, 31);
  const double a2 = lane_read(a, 47), b2 = lane_read(b, 47), a3 = lane_read(a, 63), b3 = lane_read(b, 63);
  a = ((a0 + a1) + a2) + a3;
  b = ((b0 + b1) + b2) + b3;
}

// Sum over a workgroup of nthreads (multiple of 64) in a fixed order; result valid
// in every thread.  scratch holds at least nthreads/64 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double *scratch) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += scratch[i];
  return t;
}

// Feature activation and its first two derivatives at s (rfm_activation): phi, phi', phi''.
template <typename T>
__device__ __forceinline__ void activation3(int act, T s, T &t, T &g, T &gg) {
  if (act == RFM_ACT_SIN) {
    t = sin(s);
    g = cos(s);
    gg = -t;
  } else if (act == RFM_ACT_SIGMOID) {
    t = (T)1 / ((T)1 + exp(-s));
    g = t * ((T)1 - t);
    gg = g * ((T)1 - (T)2 * t);
  } else {
    t = tanh(s);
    g = (T)1 - t * t;
    gg = (T)-2 * t * g;
  }
}

template <typename T>
__device__ __forceinline__ T activation1(int act, T s) {
  if (act == RFM_ACT_SIN) return sin(s);
  if (act == RFM_ACT_SIGMOID) return (T)1 / ((T)1 + exp(-s));
  return tanh(s);
}

// The same with the activation fixed at compile time (kernels instantiated per activation).
template <int ACT, typename T>
__device__ __forceinline__ T activation1c(T s) {
  if constexpr (ACT == RFM_ACT_SIN) return sin(s);
  else if constexpr (ACT == RFM_ACT_SIGMOID) return (T)1 / ((T)1 + exp(-s));
  else return tanh(s);
}

// Widest hidden layer of a depth-h feature network (held in registers per row).
constexpr int kHMax = 16;
constexpr int kMaxDepth = 8;

// Doubles per subdomain in rfm_problem::net.
__host__ __device__ inline int64_t net_stride(const rfm_problem &P, int d) {
  const int64_t H = P.hidden;
  return H * d + H + (int64_t)(P.depth - 2) * (H * H + H);
}

inline rfm_status check_network(const rfm_problem *P, const char *who) {
  if (P->depth < 0 || P->depth > kMaxDepth) return fail(RFM_EINVAL, std::string(who) + ": depth out of range");
  if (P->depth > 1 && (P->hidden < 1 || P->hidden > kHMax || !P->net))
    return fail(RFM_EINVAL, std::string(who) + ": hidden width (1..16) or network pointer");
  return RFM_OK;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace rfm
