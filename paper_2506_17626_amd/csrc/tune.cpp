// Autotuner of the batching form: times candidate launch shapes of the filter and of the
// LSQR adjoint products on the caller's data with HIP events and keeps the fastest.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "rfm.h"

namespace rfm {
rfm_status fail(rfm_status st, const std::string &msg);
}

namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
  }
};

}  // namespace

extern "C" rfm_status rfm_autotune(const rfm_layout *L, const double *M, double tau, int32_t *rank,
                                   int32_t *kept, double *R, double *Q, double *ratios,
                                   const int32_t *order, const double *h, int64_t lsqr_iters,
                                   double *y_scratch, void *ws, size_t ws_bytes, rfm_tuning *best,
                                   double *ms_out, rfm_tuning *cand_out, int32_t *ncand, void *stream) {
  using rfm::fail;
  if (!L || !best || !ncand || !h || !y_scratch) return fail(RFM_EINVAL, "rfm_autotune: null pointer");
  if (lsqr_iters < 2) return fail(RFM_EINVAL, "rfm_autotune: lsqr_iters must be >= 2");
  const size_t need = rfm_rrqr_ws_bytes(L) > rfm_lsqr_ws_bytes(L) ? rfm_rrqr_ws_bytes(L) : rfm_lsqr_ws_bytes(L);
  if (!ws || ws_bytes < need) return fail(RFM_EINVAL, "rfm_autotune: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  Events ev;
  if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess)
    return fail(RFM_EHIP, "rfm_autotune: hipEventCreate");

  std::vector<rfm_tuning> cands;
  if (L->max_cols <= 512)  // R-first form: one block per workgroup in the given order
    cands.push_back(rfm_tuning{0, 0, 1, 0, RFM_RRQR_RFIRST});
  const int threads[3] = {256, 512, 1024};
  for (int t : threads) {
    if (t == 1024 && L->max_rows > 1024) continue;
    cands.push_back(rfm_tuning{t, 0, 1, 0, RFM_RRQR_DIRECT});
    cands.push_back(rfm_tuning{t, 1, 1, 0, RFM_RRQR_DIRECT});
    cands.push_back(rfm_tuning{t, 1, 2, 0, RFM_RRQR_DIRECT});
  }
  int32_t n = 0;
  double best_ms = 1e300;
  rfm_tuning win = cands[0];
  // one untimed run first (code objects loaded, caches warm)
  rfm_status s = rfm_rrqr_filter_tuned(L, M, tau, rank, kept, R, Q, ratios, order, &cands[0], ws, ws_bytes, stream);
  if (s != RFM_OK) return s;
  for (const rfm_tuning &c : cands) {
    if (hipEventRecord(ev.a, st) != hipSuccess) return fail(RFM_EHIP, "rfm_autotune: hipEventRecord");
    s = rfm_rrqr_filter_tuned(L, M, tau, rank, kept, R, Q, ratios, order, &c, ws, ws_bytes, stream);
    if (s != RFM_OK) return s;
    if (hipEventRecord(ev.b, st) != hipSuccess || hipEventSynchronize(ev.b) != hipSuccess)
      return fail(RFM_EHIP, "rfm_autotune: event");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return fail(RFM_EHIP, "rfm_autotune: elapsed");
    if (n < 32 && ms_out) ms_out[n] = ms;
    if (n < 32 && cand_out) cand_out[n] = c;
    ++n;
    if (ms < best_ms) {
      best_ms = ms;
      win = c;
    }
  }

  // the outputs are those of the winning filter shape
  s = rfm_rrqr_filter_tuned(L, M, tau, rank, kept, R, Q, ratios, order, &win, ws, ws_bytes, stream);
  if (s != RFM_OK) return s;

  // adjoint tile of LSQR: sampled stage times of a short solve per candidate
  rfm_operator A{};
  A.form = RFM_FORM_Q;
  A.rank = rank;
  A.Q = Q;
  const int tiles[5] = {16, 32, 64, 128, 256};
  double best_adj = 1e300;
  int best_tile = 0;
  for (int tile : tiles) {
    if (tile > 16 && tile - 16 >= L->max_cols) break;
    rfm_kernel_times times{};
    rfm_lsqr_opts o{};
    o.atol = 0.0;
    o.btol = 0.0;
    o.maxit = lsqr_iters;
    o.check_every = (int32_t)lsqr_iters;
    o.use_graph = 0;
    o.times = &times;
    o.inner_dtype = RFM_F64;
    o.adj_tile = tile;
    rfm_lsqr_info info{};
    s = rfm_lsqr_solve(L, &A, h, nullptr, &o, y_scratch, &info, ws, ws_bytes, stream);
    if (s != RFM_OK && s != RFM_ENOTCONV) return s;
    const double avg = times.launches[2] > 0 ? times.ms[2] / (double)times.launches[2] : 1e300;
    rfm_tuning c = win;
    c.adj_tile = tile;
    if (n < 32 && ms_out) ms_out[n] = avg;
    if (n < 32 && cand_out) cand_out[n] = c;
    ++n;
    if (avg < best_adj) {
      best_adj = avg;
      best_tile = tile;
    }
  }
  win.adj_tile = best_tile;
  *best = win;
  *ncand = n;
  return RFM_OK;
}
