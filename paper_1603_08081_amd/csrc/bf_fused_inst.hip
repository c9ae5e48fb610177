// One explicit instantiation of the fused kernel launcher, selected at build
// time by BF_INST_PREC (a bf_planes value) and BF_INST_NT (window tiles).
#include "bf_wave_impl.h"

#if !defined(BF_INST_PREC) || !defined(BF_INST_NT)
#error "compile with -DBF_INST_PREC=<0|1|2> -DBF_INST_NT=<2..9>"
#endif

namespace bf {
template hipError_t launch_fused_nt<BF_INST_PREC, BF_INST_NT>(const JobDesc&, int, hipStream_t);
namespace fused_detail {
template TileChoice choose_tile<BF_INST_PREC, BF_INST_NT>(const JobDesc&, int);
template hipError_t launch_batched_class<BF_INST_PREC, BF_INST_NT>(const JobDesc*, const int4*, int, int, int,
                                                                   TileChoice, int, hipStream_t);
}  // namespace fused_detail
}  // namespace bf
