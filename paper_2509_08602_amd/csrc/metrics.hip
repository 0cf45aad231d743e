// Voxel counts behind the clinical metrics (see metrics.h).
#include "metrics.h"

#include <algorithm>

namespace ladmm {

namespace {

// Thread = plan (consecutive plans read consecutive doses of a voxel row);
// blocks stride over the voxel rows; one integer atomic per counter and block.
__global__ void k_metric_counts(const double *__restrict__ d, int ldd, int n_vox, int k,
                                const int32_t *__restrict__ tgt, const double *__restrict__ presc,
                                double d_ref, unsigned long long *__restrict__ counts) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double half = 0.5 * d_ref;
  unsigned long long cov = 0, piv = 0, piv2 = 0;
  for (int v = blockIdx.x; v < n_vox; v += gridDim.x) {
    const double x = d[(size_t)v * ldd + j];
    const int t = tgt[v];
    cov += (t >= 0 && x >= presc[t]) ? 1ull : 0ull;
    piv += x >= d_ref ? 1ull : 0ull;
    piv2 += x >= half ? 1ull : 0ull;
  }
  atomicAdd(&counts[3 * (size_t)j + 0], cov);
  atomicAdd(&counts[3 * (size_t)j + 1], piv);
  atomicAdd(&counts[3 * (size_t)j + 2], piv2);
}

}  // namespace

hipError_t plan_metric_counts(hipStream_t s, const double *d, int ldd, int n_vox, int k,
                              const int32_t *tgt, const double *presc, double d_ref,
                              unsigned long long *counts) {
  if (n_vox < 1 || k < 1) return hipSuccess;
  const dim3 grid((unsigned)std::min(n_vox, 1024), (unsigned)((k + 63) / 64));
  hipLaunchKernelGGL(k_metric_counts, grid, dim3(64), 0, s, d, ldd, n_vox, k, tgt, presc, d_ref,
                     counts);
  return hipGetLastError();
}

}  // namespace ladmm
