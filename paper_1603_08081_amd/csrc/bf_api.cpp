// C ABI of libbf: argument checking, coefficient fit, spatial weights and the
// single-image entry point.  The batched entry points and plans live in
// bf_batch.cpp.  See include/bf.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <sstream>
#include <string>
#include <vector>

#include "bf_internal.h"

namespace bf {

namespace {
thread_local std::string g_error;
}

void set_error(const std::string& msg) { g_error = msg; }

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

int check_fit_args(bf_range_kind kind, double sigma_r, const double* table, int T, double eps,
                   int K_max) {
  if (kind != BF_RANGE_GAUSSIAN && kind != BF_RANGE_EXPONENTIAL && kind != BF_RANGE_TABLE)
    return fail(BF_E_INVALID, "unknown range kernel kind");
  if (T < 1 || T > BF_MAX_T) return fail(BF_E_INVALID, "T must satisfy 1 <= T <= BF_MAX_T");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(BF_E_INVALID, "eps must be finite and >= 0");
  if (K_max < 0 || K_max > T) return fail(BF_E_INVALID, "K_max must satisfy 0 <= K_max <= T");
  if (kind == BF_RANGE_TABLE) {
    if (!table) return fail(BF_E_INVALID, "phi_table is required for BF_RANGE_TABLE");
    for (int t = 0; t <= T; ++t)
      if (!std::isfinite(table[t])) return fail(BF_E_INVALID, "phi_table holds a non-finite value");
  } else if (!(sigma_r > 0.0) || !std::isfinite(sigma_r)) {
    return fail(BF_E_INVALID, "sigma_r must be finite and > 0");
  }
  return BF_OK;
}

int resolve_job(const bf_job* j, Resolved* out) {
  if (!j) return fail(BF_E_INVALID, "job is NULL");
  if (!j->src || !j->dst) return fail(BF_E_INVALID, "src and dst must be device pointers");
  if (j->height < 1 || j->width < 1) return fail(BF_E_INVALID, "height and width must be >= 1");
  if (j->src_pitch < j->width || j->dst_pitch < j->width)
    return fail(BF_E_INVALID, "pitch must be >= width");
  if (j->spatial != BF_SPATIAL_GAUSSIAN && j->spatial != BF_SPATIAL_BOX)
    return fail(BF_E_INVALID, "unknown spatial kernel kind");
  if (j->flags & ~(BF_FLAG_INTEGER_INPUT | BF_FLAG_OFFSETS16)) return fail(BF_E_INVALID, "unknown bits in flags");
  int W = j->W;
  if (j->spatial == BF_SPATIAL_GAUSSIAN) {
    if (!(j->sigma_s > 0.0) || !std::isfinite(j->sigma_s))
      return fail(BF_E_INVALID, "sigma_s must be finite and > 0 for the Gaussian spatial kernel");
    if (W < 0) {
      const double w3 = std::ceil(3.0 * j->sigma_s);
      if (w3 > BF_MAX_W) return fail(BF_E_UNSUPPORTED, "ceil(3 sigma_s) exceeds BF_MAX_W");
      W = static_cast<int>(w3);
    }
  } else if (W < 0) {
    return fail(BF_E_INVALID, "the box kernel needs W >= 0");
  }
  if (W > BF_MAX_W) return fail(BF_E_UNSUPPORTED, "W exceeds BF_MAX_W");
  if (W >= j->height || W >= j->width)
    return fail(BF_E_INVALID, "W must be smaller than both image sides (symmetric border)");
  if (j->T < 1 || j->T > BF_MAX_T) return fail(BF_E_INVALID, "T must satisfy 1 <= T <= BF_MAX_T");
  if (j->f_max < 0 || j->f_max > BF_MAX_T) return fail(BF_E_INVALID, "f_max must satisfy 0 <= f_max <= BF_MAX_T");
  // src and dst ranges must not overlap
  const uintptr_t s0 = reinterpret_cast<uintptr_t>(j->src);
  const uintptr_t s1 = s0 + sizeof(float) * ((size_t)(j->height - 1) * j->src_pitch + j->width);
  const uintptr_t d0 = reinterpret_cast<uintptr_t>(j->dst);
  const uintptr_t d1 = d0 + sizeof(float) * ((size_t)(j->height - 1) * j->dst_pitch + j->width);
  if (s0 < d1 && d0 < s1) return fail(BF_E_INVALID, "src and dst overlap");

  std::vector<double> d;
  int status = BF_OK;
  if (j->d) {
    if (j->K < 0) return fail(BF_E_INVALID, "K must be >= 0 when d is given");
    if (j->K > BF_MAX_K) return fail(BF_E_UNSUPPORTED, "K exceeds BF_MAX_K");
    d.assign(j->d, j->d + j->K + 1);
    for (double v : d)
      if (!std::isfinite(v)) return fail(BF_E_INVALID, "d holds a non-finite value");
  } else {
    int rc = check_fit_args(j->range, j->sigma_r, j->phi_table, j->T, j->eps, j->K_max);
    if (rc != BF_OK) return rc;
    if (j->K_max > BF_MAX_K) return fail(BF_E_UNSUPPORTED, "K_max exceeds BF_MAX_K");
    std::vector<double> b;
    sample_range_kernel(j->range, j->sigma_r, j->phi_table, j->T, b);
    FitOutcome fo = fit_cosine_series(b, j->T, j->eps, j->K_max);
    d = fo.d;
    if (!fo.converged) status = BF_FIT_NOT_CONVERGED;
  }
  JobDesc& jd = out->desc;
  std::memset(&jd, 0, sizeof(jd));
  jd.src = j->src;
  jd.dst = j->dst;
  jd.height = j->height;
  jd.width = j->width;
  jd.src_pitch = j->src_pitch;
  jd.dst_pitch = j->dst_pitch;
  jd.W = W;
  jd.K = static_cast<int>(d.size()) - 1;
  jd.T = j->T;
  jd.F = j->f_max > 0 ? j->f_max : j->T;
  jd.flags = j->flags | (j->spatial == BF_SPATIAL_BOX ? kJobBox : 0);
  // centre of the gray-level range: |f - c0| <= F / 2 before 16-bit rounding
  jd.c0 = 0.5f * static_cast<float>(jd.F);
  // unit-sum 1-D profile (eq. (2) is separable: w(x, y) = w1(x) w1(y))
  double sum = 0.0;
  std::vector<double> w1(2 * W + 1);
  for (int t = -W; t <= W; ++t) {
    const double v = (j->spatial == BF_SPATIAL_BOX)
                         ? 1.0
                         : std::exp(-static_cast<double>(t) * t / (2.0 * j->sigma_s * j->sigma_s));
    w1[t + W] = v;
    sum += v;
  }
  for (int t = 0; t <= 2 * W; ++t) jd.w1[t] = static_cast<float>(w1[t] / sum);
  for (size_t k = 0; k < d.size(); ++k) jd.d[k] = d[k];
  out->status = status;
  return BF_OK;
}

int pick_tile_rows(const JobDesc& jd, bf_planes prec) {
  // fp32 planes with windows wider than 6 row tiles (W > 40) spill registers
  // at taller tiles
  if (prec == BF_PLANES_FP32 && window_tiles(jd.W) >= 7) return 32;
  // the tallest tile that still gives every CU about one workgroup
  // (choose_tile falls back to a shorter one where a height does not exist)
  const long col_blocks = (jd.width + tile_cols(prec) - 1) / tile_cols(prec);
  if (col_blocks * ((jd.height + 127) / 128) >= 240) return 128;
  return col_blocks * ((jd.height + 63) / 64) >= 240 ? 64 : 32;
}

}  // namespace bf

using namespace bf;

extern "C" const char* bf_last_error(void) { return g_error.c_str(); }

extern "C" int bf_fit_coeffs(bf_range_kind kind, double sigma_r, const double* phi_table, int T,
                             double eps, int K_max, double* d, int* K, double* err_l2,
                             double* err_max) {
  int rc = check_fit_args(kind, sigma_r, phi_table, T, eps, K_max);
  if (rc != BF_OK) return rc;
  if (!d || !K) return fail(BF_E_INVALID, "d and K must be non-NULL");
  std::vector<double> b;
  sample_range_kernel(kind, sigma_r, phi_table, T, b);
  FitOutcome fo = fit_cosine_series(b, T, eps, K_max);
  for (int k = 0; k <= fo.K; ++k) d[k] = fo.d[k];
  *K = fo.K;
  if (err_l2) *err_l2 = fo.err_l2;
  if (err_max) *err_max = fo.err_max;
  if (!fo.converged) {
    set_error("fit stopped at K_max with ||b - A d|| > eps");
    return BF_FIT_NOT_CONVERGED;
  }
  return BF_OK;
}

extern "C" int bf_filter(const bf_job* job, bf_planes prec, void* workspace, size_t ws_bytes,
                         void* hip_stream) {
  (void)workspace;
  (void)ws_bytes;
  if (prec != BF_PLANES_FP32 && prec != BF_PLANES_FP16 && prec != BF_PLANES_BF16)
    return fail(BF_E_INVALID, "unknown plane precision");
  Resolved r;
  int rc = resolve_job(job, &r);
  if (rc < 0) return rc;
  hipError_t e = launch_fused(r.desc, prec, pick_tile_rows(r.desc, prec), static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  if (r.status != BF_OK) set_error("fit stopped at K_max with ||b - A d|| > eps");
  return r.status;
}
