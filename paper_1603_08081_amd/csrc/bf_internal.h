// Internal declarations shared by the host side of libbf (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/bf.h"

namespace bf {

// ---- host fit -------------------------------------------------------------
struct FitOutcome {
  int K = 0;
  std::vector<double> d;
  double err_l2 = 0.0;
  double err_max = 0.0;
  bool converged = false;
};

int sample_range_kernel(bf_range_kind kind, double sigma_r, const double* table, int T,
                        std::vector<double>& b);
FitOutcome fit_cosine_series(const std::vector<double>& b, int T, double eps, int K_max);

// ---- device-side job description -------------------------------------------
// Everything one image needs on the device.  Passed by value as a kernel
// argument for bf_filter; stored in the workspace table for bf_filter_batched.
struct JobDesc {
  const float* src;
  float* dst;
  int height, width, src_pitch, dst_pitch;
  int W;            // window half-width
  int K;            // highest harmonic
  int T;            // half-period
  int F;            // gray-level tables cover f = 0..F (integer-input path); F >= 1
  int flags;
  float c0;         // range centring constant (T / 2)
  float w1[2 * BF_MAX_W + 1];   // unit-sum 1-D spatial profile on [-W, W]
  double d[BF_MAX_K + 1];       // coefficients d_0..d_K
};

// internal JobDesc.flags bits (above the public BF_FLAG_* bits)
constexpr int kJobBox = 0x100;  // box spatial kernel (w = 1 on the window)

// Geometry of the fused kernel: a workgroup owns a tile_cols(prec)-column by
// `th`-row output tile; one wave owns a 16-column strip of it.
inline int tile_cols(bf_planes prec) { return prec == BF_PLANES_FP32 ? 64 : 128; }

// number of 16-row tiles spanned by 16 output rows plus a W-row halo on each side
inline int window_tiles(int W) {
  int nt = (16 + 2 * W + 15) / 16;
  return nt < 2 ? 2 : nt;
}

// running-sum box kernel (bf_box.hip): float32 planes on integer images with
// the box spatial kernel, W <= 24
bool box_supported(const JobDesc& job);
hipError_t launch_box(const JobDesc& job, hipStream_t stream);
hipError_t launch_box_batched(const JobDesc* jobs, const int4* items, int n_items, int t_max, int f_max, int grid,
                              hipStream_t stream);

// launchers (bf_fused_inst.hip instantiations); return the hipError_t of the launch
hipError_t launch_fused(const JobDesc& job, bf_planes prec, int th, hipStream_t stream);

// Tile geometry and kernel family chosen for one job: family 1 = barrier-free
// wave kernel, 2 = shared-plane kernel with staged tile, 3 = running-sum box
// kernel, 0 = general path.
struct TileChoice {
  int cols, th, family;
  bool offsets16;  // wave kernel: stage 16-bit table offsets (BF_FLAG_OFFSETS16 on a job of the class)
};
TileChoice choose_tile(const JobDesc& job, bf_planes prec, int th_pref);
// one persistent launch over n_items work items (int4: job, x0, y0, -) that
// share window class, plane format and TileChoice; grid = workgroups
hipError_t launch_batched(const JobDesc* jobs_dev, const int4* items_dev, int n_items, int t_max, int f_max,
                          bf_planes prec, int window_tiles, TileChoice tc, int grid, hipStream_t stream);

// bf_filter_batched with the job table and tiles copied straight from
// ordinary host memory into device memory of table_cap bytes (256-byte
// aligned; table_of(stream, &ptr) returns its address on the stream's device
// and is called only after every argument and the table size have been
// checked): no pinned staging and no allocation of device or pinned memory.
// BF_E_UNSUPPORTED (naming cap_name) when the table does not fit.
int filter_batched_pageable(const bf_job* jobs, int n_jobs, bf_planes prec, size_t table_cap, const char* cap_name,
                            int (*table_of)(hipStream_t, void**), hipStream_t stream);

// thread-local error text
void set_error(const std::string& msg);
// set_error(msg) and return code
int fail(int code, const std::string& msg);

// argument checks of Algorithm 2's inputs; BF_OK or a negative status
int check_fit_args(bf_range_kind kind, double sigma_r, const double* table, int T, double eps, int K_max);

// Everything the kernels need, resolved from a bf_job (validation, W, fit).
struct Resolved {
  JobDesc desc;
  int status = BF_OK;  // BF_OK or BF_FIT_NOT_CONVERGED
};
int resolve_job(const bf_job* j, Resolved* out);

// output-tile height for bf_filter (32 or 64 rows)
int pick_tile_rows(const JobDesc& jd, bf_planes prec);

}  // namespace bf
