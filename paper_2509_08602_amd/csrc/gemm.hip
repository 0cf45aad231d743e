// MFMA GEMM kernels for gfx950: the two dose-matrix products of every ADMM
// iteration (Sec. 2.B: A W in Eq. partial_elimination and A' v in the closed
// form that follows it), with the elementwise steps of Eq. (admm) fused into
// their prologue and epilogue, plus the FP64 products of the case setup.
//
// Both kernels stage BK-deep slices of the operands through LDS and feed
// v_mfma_*_16x16x4 instructions (f32 or f64).  A 256-thread workgroup holds a
// BM x BN output tile as 2 x 2 wavefronts; each wavefront owns
// (BM/32) x (BN/32) 16x16 accumulator tiles.
//
// MFMA 16x16x4 operand layout (gfx950, checked by a lane probe): lane l supplies
// A[i][k] with i = l % 16, k = l / 16 and B[k][j] with j = l % 16, k = l / 16.
// It receives D[i][j] for j = l % 16 and, in accumulator register r = 0..3,
// i = 4 (l / 16) + r for the f32 instruction but i = l / 16 + 4 r for f64.
#include "kernels.h"

#include <math.h>

namespace ladmm {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T> struct MV;
template <> struct MV<float> { typedef f4v V; };
template <> struct MV<double> { typedef d4v V; };

__device__ __forceinline__ f4v mfma16(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Upper bound u of dose point p in plan j (App. A: w/N per group, +inf for OAR;
// 0 for a low-dose point outside the plan's second-pass subset).
template <typename T>
__device__ __forceinline__ T upper_of(const PointTable<T> &pt, int g, int p, int j) {
  T u = pt.utab[(size_t)g * pt.ldu + j];
  if (pt.mask != nullptr && pt.is_ld[g]) {
    uint64_t w = pt.mask[(size_t)j * pt.mask_words + (p >> 6)];
    if (!((w >> (p & 63)) & 1ull)) u = T(0);
  }
  return u;
}

template <typename T>
__device__ __forceinline__ T clip0u(T q, T u) { return fmin(fmax(q, T(0)), u); }

// Row of the 16x16 output tile held by `lane` in accumulator register r.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// ---------------------------------------------------------------------------
// P[z][m][n] = sum_{k in chunk z} A[k][m] * B'[k][n]
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, bool PRO>
__global__ __launch_bounds__(256) void k_gemm_tn(const T *__restrict__ A, int lda,
                                                 const T *__restrict__ B, int ldb,
                                                 T *__restrict__ P, int ldp, size_t pstride,
                                                 int K, int kchunk, PointTable<T> pt) {
  constexpr int TM = BM / 32, TN = BN / 32;
  __shared__ T sA[BK][BM + 1];
  __shared__ T sB[BK][BN + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  typename MV<T>::V acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename MV<T>::V{0, 0, 0, 0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    for (int e = tid; e < BK * BM; e += 256) {
      const int kk = e / BM, mm = e % BM, k = k0 + kk;
      sA[kk][mm] = (k < kend) ? A[(size_t)k * lda + m0 + mm] : T(0);
    }
    for (int e = tid; e < BK * BN; e += 256) {
      const int kk = e / BN, nn = e % BN, k = k0 + kk;
      T val = T(0);
      if (k < kend) {
        const T qv = B[(size_t)k * ldb + n0 + nn];
        if (PRO) {
          const int g = pt.grp[k];
          const T z = clip0u(qv, upper_of(pt, g, k, n0 + nn));
          val = T(2) * z - qv;               // z1 - y1 with y1 = q - z1
        } else {
          val = qv;
        }
      }
      sB[kk][nn] = val;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) a[tm] = sA[kk + (lane >> 4)][wm * TM * 16 + tm * 16 + (lane & 15)];
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) b[tn] = sB[kk + (lane >> 4)][wn * TN * 16 + tn * 16 + (lane & 15)];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma16(a[tm], b[tn], acc[tm][tn]);
    }
    __syncthreads();
  }
  T *Pz = P + (size_t)blockIdx.z * pstride;
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < TN; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * TM * 16 + tm * 16 + acc_row<T>(lane, r);
        const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
        Pz[(size_t)m * ldp + n] = acc[tm][tn][r];
      }
}

template <typename T>
hipError_t gemm_tn(hipStream_t s, const T *A, int lda, const T *B, int ldb, T *P, int ldp,
                   int M, int N, int K, int nchunk, const PointTable<T> *pro) {
  constexpr int BM = 64, BK = 16;
  if (M % BM != 0 || N % 32 != 0 || nchunk < 1) return hipErrorInvalidValue;
  int kchunk = (K + nchunk - 1) / nchunk;
  kchunk = (kchunk + BK - 1) / BK * BK;
  const size_t pstride = (size_t)M * ldp;
  PointTable<T> pt{};
  if (pro) pt = *pro;
  if (N % 64 == 0) {
    dim3 grid(M / BM, N / 64, nchunk);
    if (pro)
      hipLaunchKernelGGL((k_gemm_tn<T, BM, 64, BK, true>), grid, dim3(256), 0, s, A, lda, B, ldb,
                         P, ldp, pstride, K, kchunk, pt);
    else
      hipLaunchKernelGGL((k_gemm_tn<T, BM, 64, BK, false>), grid, dim3(256), 0, s, A, lda, B, ldb,
                         P, ldp, pstride, K, kchunk, pt);
  } else {
    dim3 grid(M / BM, N / 32, nchunk);
    if (pro)
      hipLaunchKernelGGL((k_gemm_tn<T, BM, 32, BK, true>), grid, dim3(256), 0, s, A, lda, B, ldb,
                         P, ldp, pstride, K, kchunk, pt);
    else
      hipLaunchKernelGGL((k_gemm_tn<T, BM, 32, BK, false>), grid, dim3(256), 0, s, A, lda, B, ldb,
                         P, ldp, pstride, K, kchunk, pt);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// C = A B with fused epilogues (A: M x K row-major, B: K x N row-major)
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, int EPI>
__global__ __launch_bounds__(256) void k_gemm_nn(const T *__restrict__ A, int lda,
                                                 const T *__restrict__ B, int ldb, int K,
                                                 EpiArgs<T> ea) {
  constexpr int TM = BM / 32, TN = BN / 32;
  __shared__ T sA[BM][BK + 1];
  __shared__ T sB[BK][BN + 1];
  constexpr int NST = (EPI == EPI_OBJ) ? kObjStats : kAdmmStats;
  __shared__ double sred[2][NST][BN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  typename MV<T>::V acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename MV<T>::V{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      const int mm = e / BK, kk = e % BK;
      sA[mm][kk] = A[(size_t)(m0 + mm) * lda + k0 + kk];
    }
    for (int e = tid; e < BK * BN; e += 256) {
      const int kk = e / BN, nn = e % BN;
      sB[kk][nn] = B[(size_t)(k0 + kk) * ldb + n0 + nn];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) a[tm] = sA[wm * TM * 16 + tm * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) b[tn] = sB[kk + (lane >> 4)][wn * TN * 16 + tn * 16 + (lane & 15)];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma16(a[tm], b[tn], acc[tm][tn]);
    }
    __syncthreads();
  }

  if (EPI == EPI_STORE) {
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int tn = 0; tn < TN; ++tn)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * TM * 16 + tm * 16 + acc_row<T>(lane, r);
          const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
          ea.C[(size_t)m * ea.ldc + n] = acc[tm][tn][r];
        }
    return;
  }

  // per-column partial statistics of this lane
  double st[TN][NST];
#pragma unroll
  for (int tn = 0; tn < TN; ++tn)
#pragma unroll
    for (int q = 0; q < NST; ++q) st[tn][q] = 0.0;

#pragma unroll
  for (int tn = 0; tn < TN; ++tn) {
    const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
    const double invrho = ea.invrho[n];
    const bool act = ea.active[n] != 0;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * TM * 16 + tm * 16 + acc_row<T>(lane, r);
        const int g = ea.pt.grp[m];
        const T sg = ea.pt.sig[m];
        const T u = upper_of(ea.pt, g, m, n);
        const T s = acc[tm][tn][r];
        if (EPI == EPI_OBJ) {
          // s = sign * dose / threshold at this point for shot times t / E
          if (ea.pt.is_oar[g]) {
            st[tn][1] = fmax(st[tn][1], (double)(-s));
          } else {
            const double h = fmax(0.0, (double)sg - (double)s);
            st[tn][0] += (double)u * h;
          }
        } else {
          T *qp = ea.q + (size_t)m * ea.ldq + n;
          const T qv = *qp;
          const T z = clip0u(qv, u);
          // q' = x1 + y1 = z1 - c/rho - A_s' v, with c_p = -sign_p
          const T qn = z + sg * (T)invrho - s;
          if (act) *qp = qn;
          if (EPI == EPI_ADMM_STATS) {
            const double yo = (double)qv - (double)z;
            const double zn = (double)clip0u(qn, u);
            const double yn = (double)qn - zn;
            const double x = (double)qn - yo;
            st[tn][0] += (yn - yo) * (yn - yo);     // (x - z')^2
            st[tn][1] += x * x;
            st[tn][2] += zn * zn;
            st[tn][3] += (zn - (double)z) * (zn - (double)z);
            st[tn][4] += yn * yn;
            st[tn][5] += -(double)sg * zn;           // c' z1
          }
        }
      }
  }
  if (EPI == EPI_ADMM) return;

  // reduce over lanes with the same column (l, l+16, l+32, l+48), then waves
#pragma unroll
  for (int tn = 0; tn < TN; ++tn)
#pragma unroll
    for (int q = 0; q < NST; ++q) {
      double v = st[tn][q];
      if (EPI == EPI_OBJ && q == 1) {
        v = fmax(v, __shfl_xor(v, 16));
        v = fmax(v, __shfl_xor(v, 32));
      } else {
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
      }
      if (lane < 16) sred[wm][q][wn * TN * 16 + tn * 16 + lane] = v;
    }
  __syncthreads();
  for (int e = tid; e < NST * BN; e += 256) {
    const int q = e / BN, c = e % BN;
    const double a = sred[0][q][c], b = sred[1][q][c];
    const double v = (EPI == EPI_OBJ && q == 1) ? fmax(a, b) : a + b;
    ea.stats[((size_t)blockIdx.x * NST + q) * ea.nstat_cols + n0 + c] = v;
  }
}

template <typename T>
hipError_t gemm_nn(hipStream_t s, int epi, const T *A, int lda, const T *B, int ldb, int M,
                   int N, int K, const EpiArgs<T> &ea) {
  constexpr int BM = 64, BK = 16;
  if (M % BM != 0 || N % 32 != 0 || K % BK != 0) return hipErrorInvalidValue;
#define LAUNCH_NN(BN, E)                                                                  \
  hipLaunchKernelGGL((k_gemm_nn<T, BM, BN, BK, E>), dim3(M / BM, N / BN), dim3(256), 0, s, A, \
                     lda, B, ldb, K, ea)
#define LAUNCH_NN_E(BN)                                   \
  switch (epi) {                                          \
    case EPI_STORE: LAUNCH_NN(BN, EPI_STORE); break;      \
    case EPI_ADMM: LAUNCH_NN(BN, EPI_ADMM); break;        \
    case EPI_ADMM_STATS: LAUNCH_NN(BN, EPI_ADMM_STATS); break; \
    case EPI_OBJ: LAUNCH_NN(BN, EPI_OBJ); break;          \
    default: return hipErrorInvalidValue;                 \
  }
  if (N % 64 == 0) {
    LAUNCH_NN_E(64)
  } else {
    LAUNCH_NN_E(32)
  }
#undef LAUNCH_NN_E
#undef LAUNCH_NN
  return hipGetLastError();
}

template hipError_t gemm_tn<float>(hipStream_t, const float *, int, const float *, int, float *,
                                   int, int, int, int, int, const PointTable<float> *);
template hipError_t gemm_tn<double>(hipStream_t, const double *, int, const double *, int,
                                    double *, int, int, int, int, int, const PointTable<double> *);
template hipError_t gemm_nn<float>(hipStream_t, int, const float *, int, const float *, int, int,
                                   int, int, const EpiArgs<float> &);
template hipError_t gemm_nn<double>(hipStream_t, int, const double *, int, const double *, int,
                                    int, int, int, const EpiArgs<double> &);

}  // namespace ladmm
