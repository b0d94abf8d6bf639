// Host planner: supports I_j of every subdomain (eq. DomainDecomp), their transpose
// (row -> covering blocks in ascending j) and the offsets of the block layout.
//
// Points are binned on a regular grid whose cells are at least as wide as the widest
// support, so each support touches at most two bins per dimension and each point
// only tests the blocks registered in its own bin.  Membership is the strict test
// |x_i - mu_ji| < hw_ji in binary64 for every dimension.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rfm.h"

namespace rfm {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

rfm_status fail(rfm_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

namespace {

struct Bins {
  int d = 0;
  double lo[3] = {0, 0, 0}, width[3] = {1, 1, 1};
  int64_t nb[3] = {1, 1, 1};
  std::vector<int64_t> off;   // CSR over bins
  std::vector<int32_t> blk;   // blocks per bin, ascending

  int64_t coord(int i, double v) const {
    int64_t c = (int64_t)std::floor((v - lo[i]) / width[i]);
    return std::min<int64_t>(std::max<int64_t>(c, 0), nb[i] - 1);
  }
  int64_t flat(const int64_t *c) const {
    int64_t f = 0;
    for (int i = d - 1; i >= 0; --i) f = f * nb[i] + c[i];
    return f;
  }
};

bool build_bins(int d, int32_t J, int64_t N, const double *x, const double *mu, const double *hw,
                Bins &B) {
  B.d = d;
  for (int i = 0; i < d; ++i) {
    double lo = INFINITY, hi = -INFINITY, wmax = 0.0;
    for (int64_t r = 0; r < N; ++r) {
      lo = std::min(lo, x[r * d + i]);
      hi = std::max(hi, x[r * d + i]);
    }
    for (int32_t j = 0; j < J; ++j) wmax = std::max(wmax, 2.0 * hw[(int64_t)j * d + i]);
    if (!(wmax > 0.0) || !std::isfinite(lo) || !std::isfinite(hi)) return false;
    B.lo[i] = lo;
    B.width[i] = wmax;
    B.nb[i] = std::max<int64_t>(1, std::min<int64_t>(4096, (int64_t)std::ceil((hi - lo) / wmax) + 1));
  }
  int64_t nbins = 1;
  for (int i = 0; i < d; ++i) nbins *= B.nb[i];
  std::vector<int64_t> cnt(nbins + 1, 0);
  // each block registers in every bin its support interval touches
  auto for_each_bin = [&](int32_t j, auto &&fn) {
    int64_t c0[3], c1[3], c[3];
    for (int i = 0; i < d; ++i) {
      c0[i] = B.coord(i, mu[(int64_t)j * d + i] - hw[(int64_t)j * d + i]);
      c1[i] = B.coord(i, mu[(int64_t)j * d + i] + hw[(int64_t)j * d + i]);
    }
    for (c[2] = (d > 2 ? c0[2] : 0); c[2] <= (d > 2 ? c1[2] : 0); ++c[2])
      for (c[1] = (d > 1 ? c0[1] : 0); c[1] <= (d > 1 ? c1[1] : 0); ++c[1])
        for (c[0] = c0[0]; c[0] <= c1[0]; ++c[0]) fn(B.flat(c));
  };
  for (int32_t j = 0; j < J; ++j) for_each_bin(j, [&](int64_t f) { cnt[f + 1]++; });
  for (int64_t f = 0; f < nbins; ++f) cnt[f + 1] += cnt[f];
  B.off = cnt;
  B.blk.assign(cnt[nbins], 0);
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  for (int32_t j = 0; j < J; ++j) for_each_bin(j, [&](int64_t f) { B.blk[pos[f]++] = j; });
  return true;
}

inline bool inside(int d, const double *xr, const double *muj, const double *hwj) {
  for (int i = 0; i < d; ++i)
    if (!(std::fabs(xr[i] - muj[i]) < hwj[i])) return false;
  return true;
}

}  // namespace
}  // namespace rfm

extern "C" const char *rfm_last_error(void) { return rfm::g_last_error.c_str(); }

extern "C" rfm_status rfm_plan(int32_t d, int32_t J, int64_t N, const double *x, const double *mu,
                               const double *hw, const int32_t *K, int64_t *sizes_out,
                               int64_t *row_off, int32_t *rows, int32_t *inc_blk,
                               int64_t *rinc_off, int64_t *rinc, int64_t *feat_off,
                               int64_t *blk_off, int64_t *rsq_off) {
  using namespace rfm;
  if (d < 1 || d > 3) return fail(RFM_EINVAL, "rfm_plan: d must be 1..3");
  if (J < 1 || N < 1) return fail(RFM_EINVAL, "rfm_plan: J and N must be positive");
  if (N > INT32_MAX) return fail(RFM_EUNSUPPORTED, "rfm_plan: N must fit in int32");
  if (!x || !mu || !hw || !K || !sizes_out) return fail(RFM_EINVAL, "rfm_plan: null input");
  for (int32_t j = 0; j < J; ++j) {
    if (K[j] < 0) return fail(RFM_EINVAL, "rfm_plan: negative feature count");
    for (int i = 0; i < d; ++i)
      if (!(hw[(int64_t)j * d + i] > 0.0)) return fail(RFM_EINVAL, "rfm_plan: half-widths must be > 0");
  }
  Bins B;
  if (!build_bins(d, J, N, x, mu, hw, B)) return fail(RFM_EINVAL, "rfm_plan: non-finite points");

  std::vector<int64_t> cnt(J, 0), cover(N, 0);
  for (int64_t r = 0; r < N; ++r) {
    int64_t c[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) c[i] = B.coord(i, x[r * d + i]);
    const int64_t f = B.flat(c);
    for (int64_t q = B.off[f]; q < B.off[f + 1]; ++q) {
      const int32_t j = B.blk[q];
      if (inside(d, x + r * d, mu + (int64_t)j * d, hw + (int64_t)j * d)) {
        cnt[j]++;
        cover[r]++;
      }
    }
  }
  int64_t nnz_rows = 0, nnz = 0, ncols = 0, nrsq = 0, max_rows = 0, max_cols = 0;
  for (int32_t j = 0; j < J; ++j) {
    nnz_rows += cnt[j];
    nnz += cnt[j] * (int64_t)K[j];
    ncols += K[j];
    nrsq += (int64_t)K[j] * K[j];
    max_rows = std::max(max_rows, cnt[j]);
    max_cols = std::max<int64_t>(max_cols, K[j]);
  }
  sizes_out[0] = nnz_rows;
  sizes_out[1] = nnz;
  sizes_out[2] = ncols;
  sizes_out[3] = nrsq;
  sizes_out[4] = max_rows;
  sizes_out[5] = max_cols;
  const bool any = row_off || rows || inc_blk || rinc_off || rinc || feat_off || blk_off || rsq_off;
  if (!any) return RFM_OK;
  if (!(row_off && rows && inc_blk && rinc_off && rinc && feat_off && blk_off && rsq_off))
    return fail(RFM_EINVAL, "rfm_plan: either all or none of the output arrays must be given");

  row_off[0] = feat_off[0] = blk_off[0] = rsq_off[0] = 0;
  for (int32_t j = 0; j < J; ++j) {
    row_off[j + 1] = row_off[j] + cnt[j];
    feat_off[j + 1] = feat_off[j] + K[j];
    blk_off[j + 1] = blk_off[j] + cnt[j] * (int64_t)K[j];
    rsq_off[j + 1] = rsq_off[j] + (int64_t)K[j] * K[j];
  }
  rinc_off[0] = 0;
  for (int64_t r = 0; r < N; ++r) rinc_off[r + 1] = rinc_off[r] + cover[r];
  std::vector<int64_t> fill(J, 0);
  for (int64_t r = 0; r < N; ++r) {
    int64_t c[3] = {0, 0, 0};
    for (int i = 0; i < d; ++i) c[i] = B.coord(i, x[r * d + i]);
    const int64_t f = B.flat(c);
    int64_t k = rinc_off[r];
    for (int64_t q = B.off[f]; q < B.off[f + 1]; ++q) {
      const int32_t j = B.blk[q];
      if (inside(d, x + r * d, mu + (int64_t)j * d, hw + (int64_t)j * d)) {
        const int64_t p = row_off[j] + fill[j]++;
        rows[p] = (int32_t)r;
        inc_blk[p] = j;
        rinc[k++] = p;
      }
    }
  }
  return RFM_OK;
}
