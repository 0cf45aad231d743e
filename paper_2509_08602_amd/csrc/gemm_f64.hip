// FP64 instantiations of the dose-matrix and setup products (templates in gemm_impl.h).
#include "gemm_impl.h"

namespace ladmm {

bool gemm_tn_cfg_ok(int cfg, int M, int N) {
  if (cfg < 0 || cfg >= kGemmCfgs) return false;
  const TnCfg c = kTnCfgs[cfg];
  const int BN = pick_bn(N);
  return M % c.bm == 0 && c.bm % (16 * c.wm) == 0 && BN % (16 * c.wn) == 0;
}

bool gemm_nn_cfg_ok(int cfg, int M, int N) {
  if (cfg < 0 || cfg >= kGemmCfgs) return false;
  const NnCfg c = kNnCfgs[cfg];
  const int BN = nn_bn(c, N);
  const bool inst = BN == 16 || BN == 32 || BN == 48 || BN == 64 || BN == 96 || BN == 128;
  return inst && N % BN == 0 && M % c.bm == 0 && c.bm % (16 * c.wm) == 0 &&
         BN % (16 * c.wn) == 0 && (c.wn == 1 || BN % 32 == 0);
}

template hipError_t gemm_tn<double>(hipStream_t, const double *, int, const double *, int,
                                    double *, int, int, int, int, int, const PointTable<double> *,
                                    int);
template hipError_t gemm_nn<double>(hipStream_t, int, const double *, int, const double *, int,
                                    int, int, int, const EpiArgs<double> &, int);
template hipError_t rescale_points<double>(hipStream_t, double *, int, int, const PointTable<double> &,
                                          const double *);
template hipError_t w_from_q<double>(hipStream_t, const double *, double *, int, int,
                                     const PointTable<double> &);
}  // namespace ladmm
