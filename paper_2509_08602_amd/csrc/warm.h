// Warm starts of served plans: solved plans' iterates kept per case in HBM and
// copied into the columns of newly admitted plans.
#pragma once
#include "kernels.h"

namespace ladmm {

constexpr int kWarmCols = 32;   // columns moved per launch
// Pairs (batch column, store entry) of one launch.
struct WarmCols {
  int n;
  int col[kWarmCols];
  int ent[kWarmCols];
};

// Store entries <- batch columns: q (Np x kp, T) -> wq (entries x Np), q2
// (mAp x kp) -> wq2 (entries x mAp), qs (n_sec x kp) -> wqs (entries x n_sec).
template <typename T>
hipError_t warm_save(hipStream_t s, const WarmCols &w, const T *q, const double *q2, const double *qs,
                     int Np, int mAp, int n_sec, int kp, T *wq, double *wq2, double *wqs);
// Batch columns <- store entries (the inverse copy).
template <typename T>
hipError_t warm_load(hipStream_t s, const WarmCols &w, const T *wq, const double *wq2,
                     const double *wqs, int Np, int mAp, int n_sec, int kp, T *q, double *q2,
                     double *qs);
// W' = 2 Pi(q) - q of the loaded columns under their plans' bounds (point-major T).
template <typename T>
hipError_t warm_w(hipStream_t s, const WarmCols &w, const T *q, T *W, int Np, int kp,
                  const PointTable<T> &pt);
// The same for W' held as plan-major BF16 pairs (rows j: hi, rows kp + j: lo);
// with wref and dw (LADMM_BF16) also dW = bf16(W' - W_ref) of those columns.
hipError_t warm_w_bf(hipStream_t s, const WarmCols &w, const float *q, uint16_t *wh, uint16_t *wl,
                     int Np, int kp, const PointTable<float> &pt, const float *wref = nullptr,
                     uint16_t *dw = nullptr);

}  // namespace ladmm
