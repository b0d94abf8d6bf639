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

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace rfm
