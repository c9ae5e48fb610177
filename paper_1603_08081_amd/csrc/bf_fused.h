// Declarations of the fused-kernel launchers; each (precision, window-tile
// count) pair is instantiated in its own object file (bf_fused_inst.hip
// compiled with -DBF_INST_PREC and -DBF_INST_NT).
#pragma once

#include "bf_internal.h"

namespace bf {

template <int PREC, int NT>
hipError_t launch_fused_nt(const JobDesc& job, int th, hipStream_t stream);

namespace fused_detail {
template <int PREC, int NT>
TileChoice choose_tile(const JobDesc& job, int th_pref);
template <int PREC, int NT>
hipError_t launch_batched_class(const JobDesc* jobs, const int4* items, int n_items, int t_max, int f_max,
                                TileChoice tc, int grid, hipStream_t stream);
}  // namespace fused_detail

}  // namespace bf
