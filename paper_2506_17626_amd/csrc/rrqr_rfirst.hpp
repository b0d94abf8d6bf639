// R-first form of the sigma-RRQR filter (the default path of rfm_rrqr_filter).
#pragma once

#include "common.hpp"

namespace rfm {

struct RfirstArgs {
  const rfm_layout *L;
  const double *M;
  double tau;
  int32_t *rank, *kept;
  double *R, *Q, *ratios;
  const int32_t *order;  // nullable: 0..J-1 (launch order of the blocks)
  void *ws;
  size_t ws_bytes;
  hipStream_t st;
};

// Blocks the R-first kernels take: max_cols <= 512 and max_rows <= 3072.
bool rfirst_supported(const rfm_layout *L);
// Device workspace of the R-first form (reflector scalars, signs, two K_j x K_j slots).
size_t rfirst_ws_bytes(const rfm_layout *L);
rfm_status rrqr_rfirst(const RfirstArgs &a);

}  // namespace rfm
