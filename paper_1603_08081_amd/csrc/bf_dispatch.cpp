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
  switch (prec) {
    case BF_PLANES_FP32: return launch_prec<BF_PLANES_FP32>(job, th, stream);
    case BF_PLANES_FP16: return launch_prec<BF_PLANES_FP16>(job, th, stream);
    case BF_PLANES_BF16: return launch_prec<BF_PLANES_BF16>(job, th, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bf
