// Column moves between a batch and its warm-start store (see warm.h).
#include "warm.h"

#include <algorithm>

#include "gemm_impl.h"

namespace ladmm {

namespace {

// One block row of 256 rows of each array for column pair blockIdx.y.
template <typename T, bool SAVE>
__global__ void k_warm_move(WarmCols w, T *__restrict__ q, double *__restrict__ q2,
                            double *__restrict__ qs, int Np, int mAp, int n_sec, int kp,
                            T *__restrict__ wq, double *__restrict__ wq2, double *__restrict__ wqs) {
  const int i = blockIdx.y;
  if (i >= w.n) return;
  const int col = w.col[i];
  const size_t ent = (size_t)w.ent[i];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < Np) {
    if (SAVE) wq[ent * Np + r] = q[(size_t)r * kp + col];
    else q[(size_t)r * kp + col] = wq[ent * Np + r];
  }
  if (r < mAp) {
    if (SAVE) wq2[ent * mAp + r] = q2[(size_t)r * kp + col];
    else q2[(size_t)r * kp + col] = wq2[ent * mAp + r];
  }
  if (r < n_sec) {
    if (SAVE) wqs[ent * n_sec + r] = qs[(size_t)r * kp + col];
    else qs[(size_t)r * kp + col] = wqs[ent * n_sec + r];
  }
}

template <typename T>
__global__ void k_warm_w(WarmCols w, const T *__restrict__ q, T *__restrict__ W, int Np, int kp,
                         PointTable<T> pt) {
  const int i = blockIdx.y;
  if (i >= w.n) return;
  const int j = w.col[i];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Np) return;
  const size_t e = (size_t)p * kp + j;
  const T qv = q[e];
  W[e] = T(2) * clip0u(qv, upper_of(pt, pt.grp[p], p, j)) - qv;
}

dim3 move_grid(const WarmCols &w, int rows) { return dim3((unsigned)((rows + 255) / 256), (unsigned)w.n); }

}  // namespace

template <typename T>
hipError_t warm_save(hipStream_t s, const WarmCols &w, const T *q, const double *q2, const double *qs,
                     int Np, int mAp, int n_sec, int kp, T *wq, double *wq2, double *wqs) {
  if (w.n <= 0) return hipSuccess;
  if (w.n > kWarmCols) return hipErrorInvalidValue;
  const int rows = std::max(Np, std::max(mAp, n_sec));
  hipLaunchKernelGGL((k_warm_move<T, true>), move_grid(w, rows), dim3(256), 0, s, w,
                     const_cast<T *>(q), const_cast<double *>(q2), const_cast<double *>(qs), Np, mAp,
                     n_sec, kp, wq, wq2, wqs);
  return hipGetLastError();
}

template <typename T>
hipError_t warm_load(hipStream_t s, const WarmCols &w, const T *wq, const double *wq2,
                     const double *wqs, int Np, int mAp, int n_sec, int kp, T *q, double *q2,
                     double *qs) {
  if (w.n <= 0) return hipSuccess;
  if (w.n > kWarmCols) return hipErrorInvalidValue;
  const int rows = std::max(Np, std::max(mAp, n_sec));
  hipLaunchKernelGGL((k_warm_move<T, false>), move_grid(w, rows), dim3(256), 0, s, w, q, q2, qs, Np,
                     mAp, n_sec, kp, const_cast<T *>(wq), const_cast<double *>(wq2),
                     const_cast<double *>(wqs));
  return hipGetLastError();
}

template <typename T>
hipError_t warm_w(hipStream_t s, const WarmCols &w, const T *q, T *W, int Np, int kp,
                  const PointTable<T> &pt) {
  if (w.n <= 0) return hipSuccess;
  if (w.n > kWarmCols) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_warm_w<T>), move_grid(w, Np), dim3(256), 0, s, w, q, W, Np, kp, pt);
  return hipGetLastError();
}

template hipError_t warm_save<float>(hipStream_t, const WarmCols &, const float *, const double *,
                                     const double *, int, int, int, int, float *, double *, double *);
template hipError_t warm_save<double>(hipStream_t, const WarmCols &, const double *, const double *,
                                      const double *, int, int, int, int, double *, double *, double *);
template hipError_t warm_load<float>(hipStream_t, const WarmCols &, const float *, const double *,
                                     const double *, int, int, int, int, float *, double *, double *);
template hipError_t warm_load<double>(hipStream_t, const WarmCols &, const double *, const double *,
                                      const double *, int, int, int, int, double *, double *, double *);
template hipError_t warm_w<float>(hipStream_t, const WarmCols &, const float *, float *, int, int,
                                  const PointTable<float> &);
template hipError_t warm_w<double>(hipStream_t, const WarmCols &, const double *, double *, int, int,
                                   const PointTable<double> &);

}  // namespace ladmm
