// Selects the fused-kernel instantiation for a job's precision and window.
#include "bf_fused.h"

namespace bf {

namespace {
template <int PREC>
hipError_t launch_prec(const JobDesc& job, int th, hipStream_t stream) {
  switch (window_tiles(job.W)) {
    case 2: return launch_fused_nt<PREC, 2>(job, th, stream);
    case 3: return launch_fused_nt<PREC, 3>(job, th, stream);
    case 4: return launch_fused_nt<PREC, 4>(job, th, stream);
    case 5: return launch_fused_nt<PREC, 5>(job, th, stream);
    case 6: return launch_fused_nt<PREC, 6>(job, th, stream);
    case 7: return launch_fused_nt<PREC, 7>(job, th, stream);
    case 8: return launch_fused_nt<PREC, 8>(job, th, stream);
    case 9: return launch_fused_nt<PREC, 9>(job, th, stream);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

hipError_t launch_fused(const JobDesc& job, bf_planes prec, int th, hipStream_t stream) {
  if (prec == BF_PLANES_FP32 && box_supported(job)) return launch_box(job, stream);
  switch (prec) {
    case BF_PLANES_FP32: return launch_prec<BF_PLANES_FP32>(job, th, stream);
    case BF_PLANES_FP16: return launch_prec<BF_PLANES_FP16>(job, th, stream);
    case BF_PLANES_BF16: return launch_prec<BF_PLANES_BF16>(job, th, stream);
    default: return hipErrorInvalidValue;
  }
}

namespace {
template <int PREC>
TileChoice choose_prec(const JobDesc& job, int th_pref) {
  switch (window_tiles(job.W)) {
    case 2: return fused_detail::choose_tile<PREC, 2>(job, th_pref);
    case 3: return fused_detail::choose_tile<PREC, 3>(job, th_pref);
    case 4: return fused_detail::choose_tile<PREC, 4>(job, th_pref);
    case 5: return fused_detail::choose_tile<PREC, 5>(job, th_pref);
    case 6: return fused_detail::choose_tile<PREC, 6>(job, th_pref);
    case 7: return fused_detail::choose_tile<PREC, 7>(job, th_pref);
    case 8: return fused_detail::choose_tile<PREC, 8>(job, th_pref);
    default: return fused_detail::choose_tile<PREC, 9>(job, th_pref);
  }
}
template <int PREC>
hipError_t batched_prec(const JobDesc* jobs, const int4* items, int n, int t_max, int f_max, int nt, TileChoice tc, int grid,
                        hipStream_t st) {
  switch (nt) {
    case 2: return fused_detail::launch_batched_class<PREC, 2>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 3: return fused_detail::launch_batched_class<PREC, 3>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 4: return fused_detail::launch_batched_class<PREC, 4>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 5: return fused_detail::launch_batched_class<PREC, 5>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 6: return fused_detail::launch_batched_class<PREC, 6>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 7: return fused_detail::launch_batched_class<PREC, 7>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 8: return fused_detail::launch_batched_class<PREC, 8>(jobs, items, n, t_max, f_max, tc, grid, st);
    case 9: return fused_detail::launch_batched_class<PREC, 9>(jobs, items, n, t_max, f_max, tc, grid, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

TileChoice choose_tile(const JobDesc& job, bf_planes prec, int th_pref) {
  if (prec == BF_PLANES_FP32 && box_supported(job)) return TileChoice{64, 64, 3, false};
  switch (prec) {
    case BF_PLANES_FP32: return choose_prec<BF_PLANES_FP32>(job, th_pref);
    case BF_PLANES_FP16: return choose_prec<BF_PLANES_FP16>(job, th_pref);
    default: return choose_prec<BF_PLANES_BF16>(job, th_pref);
  }
}

hipError_t launch_batched(const JobDesc* jobs_dev, const int4* items_dev, int n_items, int t_max, int f_max,
                          bf_planes prec, int nt, TileChoice tc, int grid, hipStream_t stream) {
  if (tc.family == 3) return launch_box_batched(jobs_dev, items_dev, n_items, t_max, f_max, grid, stream);
  switch (prec) {
    case BF_PLANES_FP32: return batched_prec<BF_PLANES_FP32>(jobs_dev, items_dev, n_items, t_max, f_max, nt, tc, grid, stream);
    case BF_PLANES_FP16: return batched_prec<BF_PLANES_FP16>(jobs_dev, items_dev, n_items, t_max, f_max, nt, tc, grid, stream);
    case BF_PLANES_BF16: return batched_prec<BF_PLANES_BF16>(jobs_dev, items_dev, n_items, t_max, f_max, nt, tc, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bf
