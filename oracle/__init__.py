"""FP64 reference ("oracle") for the Fourier-kernel bilateral filter.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call,
link or run anything in this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the GPU path: its
inputs come from the seeded generator in ``synth`` and its arithmetic is
written here from the paper.

Parts:
  fit.progressive_fit       Algorithm 2 (Sec. 3), FP64
  filters.direct            eq. (1), FP64, C + OpenMP
  filters.fourier           eq. (9), FP64, C + OpenMP (the GPU's parity target)
  filters.shiftable_alg1    Algorithm 1 in complex FP64 (numpy)
  filters.brute_direct      eq. (1) in pure Python, tiny images
  dynamic_range.local_dynamic_range   the dynamic range T of Sec. 3 measured on an image
  recursive.fourier_recursive  eq. (9) with Deriche's recursive Gaussian as the
                               spatial smoothing (Sec. 2), FP64 numpy
"""
from .fit import (  # noqa: F401
    FitResult, accuracy_bound, back_substitute, fit_kernel, progressive_fit, sample_kernel, series,
)
from .filters import (  # noqa: F401
    brute_direct, build, center_weight, direct, fourier, num_threads, set_threads, shiftable_alg1,
    spatial_profile,
)
from .dynamic_range import brute_local_dynamic_range, local_dynamic_range  # noqa: F401,E402
