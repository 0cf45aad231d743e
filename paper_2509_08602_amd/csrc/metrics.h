// Clinical metrics of a batch's plans on a dose grid (coverage, selectivity,
// gradient index; Sec. 2.A).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ladmm {

// counts[3 j + 0]: target voxels v with d_j(v) >= presc[tgt[v]];
// counts[3 j + 1]: voxels with d_j(v) >= d_ref; counts[3 j + 2]: voxels with
// d_j(v) >= d_ref / 2.  d: n_vox rows of ldd plan columns (FP64).  counts must
// be zero on entry.
hipError_t plan_metric_counts(hipStream_t s, const double *d, int ldd, int n_vox, int k,
                              const int32_t *tgt, const double *presc, double d_ref,
                              unsigned long long *counts);

}  // namespace ladmm
