// FP32 instantiations of the dose-matrix products (templates in gemm_impl.h).
#include "gemm_impl.h"

namespace ladmm {
template hipError_t gemm_tn<float>(hipStream_t, const float *, int, const float *, int, float *,
                                   int, int, int, int, int, const PointTable<float> *, int);
template hipError_t gemm_nn<float>(hipStream_t, int, const float *, int, const float *, int, int,
                                   int, int, const EpiArgs<float> &, int);
template hipError_t rescale_points<float>(hipStream_t, float *, int, int, const PointTable<float> &,
                                          const double *);
template hipError_t w_from_q<float>(hipStream_t, const float *, float *, int, int,
                                    const PointTable<float> &);
}  // namespace ladmm
