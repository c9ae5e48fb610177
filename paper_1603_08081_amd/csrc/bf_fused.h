// Declarations of the fused-kernel launchers; each (precision, window-tile
// count) pair is instantiated in its own object file (bf_fused_inst.hip
// compiled with -DBF_INST_PREC and -DBF_INST_NT).
#pragma once

#include "bf_internal.h"

namespace bf {

template <int PREC, int NT>
hipError_t launch_fused_nt(const JobDesc& job, int th, hipStream_t stream);

}  // namespace bf
