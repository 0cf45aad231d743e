// MFMA GEMM kernels for gfx950: the two dose-matrix products of every ADMM
// iteration (Sec. 2.B: A W in Eq. partial_elimination and A' v in the closed
// form that follows it), with the elementwise steps of Eq. (admm) fused into
// their prologue and epilogue, plus the FP64 products of the case setup.
//
// Shapes.  The dose block D^ is tall (N points x n_t shots, N up to 2e5) and
// the plan dimension is short (k <= a few hundred), so a workgroup takes a slab
// of D^ and multiplies it by a whole block of plan columns (BN up to 128): D^ is
// streamed from HBM once per product.  BK-deep slices of both operands are
// staged through double-buffered LDS with 16-byte global loads; the next slice
// is fetched into registers while the current one feeds the MFMA pipes.
// Four wavefronts per workgroup, arranged WM x WN over the output tile, each
// own TM x TN tiles of 16 x 16.
//
// MFMA 16x16x4 operand layout (gfx950, checked by a lane probe): lane l supplies
// A[i][k] with i = l % 16, k = l / 16 and B[k][j] with j = l % 16, k = l / 16.
// It receives D[i][j] for j = l % 16 and, in accumulator register r = 0..3,
// i = 4 (l / 16) + r for the f32 instruction but i = l / 16 + 4 r for f64.
//
// LDS padding: a half-wavefront (32 lanes) reads 16 consecutive words from
// two rows; a row stride congruent to 16 (mod 32) words keeps the 32 banks
// distinct (rows of k-contiguous tiles use a stride congruent to 2 instead).
#pragma once
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

// Row of the 16x16 output tile held by `lane` in accumulator register r.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return (lane >> 4) + 4 * r; }

// 16-byte vector of T.
template <typename T> struct V16;
template <> struct V16<float> { typedef float4 V; static constexpr int n = 4; };
template <> struct V16<double> { typedef double2 V; static constexpr int n = 2; };

template <typename T>
__device__ __forceinline__ T vget(const typename V16<T>::V &v, int i);
template <> __device__ __forceinline__ float vget<float>(const float4 &v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}
template <> __device__ __forceinline__ double vget<double>(const double2 &v, int i) {
  return i == 0 ? v.x : v.y;
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

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber them so that consecutive tile indices run on the same XCD: tiles
// that share an operand slab (the column blocks of a row slab, the row tiles
// of a split-K chunk) then share one L2.  A bijection on [0, total).
__device__ __forceinline__ int xcd_tile(int id, int total) {
  constexpr int X = 8;
  const int per = (total + X - 1) / X;
  const int tall = total % X == 0 ? X : total % X;   // XCDs that take `per` tiles
  const int xcd = id % X, local = id / X;
  return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

// Padding (in elements) that makes a row of W + pad elements of T span 16 (mod
// 32) LDS banks, so two half-wavefronts reading consecutive rows never collide.
template <typename T, int W>
constexpr int row_pad() {
  return sizeof(T) == 4 ? ((16 - W) % 32 + 32) % 32 : ((8 - W) % 16 + 16) % 16;
}

// ---------------------------------------------------------------------------
// P[z][m][n] = sum_{k in chunk z} A[k][m] * B'[k][n],  A: K x M, B: K x N
// B' = B, or with the ADMM prologue B' = 2 clip(q, 0, u) - q  (z1 - y1).
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, int WM, int WN, bool PRO>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_tn(const T *__restrict__ A, int lda,
                                                          const T *__restrict__ B, int ldb,
                                                          T *__restrict__ P, int ldp, size_t pstride,
                                                          int K, int kchunk, int mtiles, int ntiles,
                                                          PointTable<T> pt) {
  constexpr int NT = 64 * WM * WN;
  constexpr int VN = V16<T>::n;
  constexpr int TM = BM / (16 * WM), TN = BN / (16 * WN);
  static_assert(TM >= 1 && TN >= 1 && TM * 16 * WM == BM && TN * 16 * WN == BN, "tile shape");
  constexpr int PADA = row_pad<T, BM>(), PADB = row_pad<T, BN>();
  constexpr int AV = BK * BM / VN, BV = BK * BN / VN;           // vectors per slice
  constexpr int AVT = (AV + NT - 1) / NT, BVT = (BV + NT - 1) / NT;  // per thread
  typedef typename V16<T>::V VT;
  __shared__ T sA[2][BK][BM + PADA];
  __shared__ T sB[2][BK][BN + PADB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // tile order: column blocks fastest (they share the row slab of A), then
  // row tiles (which share a split-K chunk of B), then chunks
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int nt = tile % ntiles, mt = (tile / ntiles) % mtiles, zc = tile / (mtiles * ntiles);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = zc * kchunk;
  const int kend = min(K, kbeg + kchunk);
  typename MV<T>::V acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename MV<T>::V{0, 0, 0, 0};

  VT ra[AVT], rb[BVT];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int kk = e / (BM / VN), mm = (e % (BM / VN)) * VN, k = k0 + kk;
        ra[i] = (k < kend) ? *reinterpret_cast<const VT *>(A + (size_t)k * lda + m0 + mm) : VT{};
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int kk = e / (BN / VN), nn = (e % (BN / VN)) * VN, k = k0 + kk;
        VT v = VT{};
        if (k < kend) {
          v = *reinterpret_cast<const VT *>(B + (size_t)k * ldb + n0 + nn);
          if (PRO) {
            const int g = pt.grp[k];
            T *pv = reinterpret_cast<T *>(&v);
#pragma unroll
            for (int c = 0; c < VN; ++c) {
              const T z = clip0u(pv[c], upper_of(pt, g, k, n0 + nn + c));
              pv[c] = T(2) * z - pv[c];
            }
          }
        }
        rb[i] = v;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int kk = e / (BM / VN), mm = (e % (BM / VN)) * VN;
        *reinterpret_cast<VT *>(&sA[buf][kk][mm]) = ra[i];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int kk = e / (BN / VN), nn = (e % (BN / VN)) * VN;
        *reinterpret_cast<VT *>(&sB[buf][kk][nn]) = rb[i];
      }
    }
  };

  if (kbeg < kend) {
    load(kbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) load(k0 + BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T a[TM], b[TN];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
          a[tm] = sA[buf][kk + (lane >> 4)][wm * TM * 16 + tm * 16 + (lane & 15)];
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
          b[tn] = sB[buf][kk + (lane >> 4)][wn * TN * 16 + tn * 16 + (lane & 15)];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma16(a[tm], b[tn], acc[tm][tn]);
      }
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  T *Pz = P + (size_t)zc * pstride;
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

// Column block of the plan dimension: the whole of N when it is at most 128.
static int pick_bn(int N) {
  if (N <= 128 && N % 32 == 0) return N;
  if (N % 128 == 0) return 128;
  if (N % 64 == 0) return 64;
  return 32;
}

// Tile configurations of the split-K product: row tile BM, slice depth BK,
// wavefront grid WM x WN; the column block is pick_bn(N).
struct TnCfg { int bm, bk, wm, wn; };
static const TnCfg kTnCfgs[kGemmCfgs] = {{64, 16, 2, 2}, {32, 16, 2, 2}, {64, 32, 4, 2}, {64, 16, 4, 2}};


template <typename T>
hipError_t gemm_tn(hipStream_t s, const T *A, int lda, const T *B, int ldb, T *P, int ldp,
                   int M, int N, int K, int nchunk, const PointTable<T> *pro, int cfg) {
  if (!gemm_tn_cfg_ok(cfg, M, N)) cfg = 0;
  if (!gemm_tn_cfg_ok(cfg, M, N) || N % 32 != 0 || nchunk < 1) return hipErrorInvalidValue;
  if (lda % V16<T>::n || ldb % V16<T>::n) return hipErrorInvalidValue;
  // chunk boundaries are multiples of 32 rows whatever the slice depth, so the
  // order of every sum is the same in every configuration
  int kchunk = (K + nchunk - 1) / nchunk;
  kchunk = (kchunk + 31) / 32 * 32;
  const size_t pstride = (size_t)M * ldp;
  PointTable<T> pt{};
  if (pro) pt = *pro;
  const int BN = pick_bn(N);
  const TnCfg c = kTnCfgs[cfg];
  const int mtiles = M / c.bm, ntiles = N / BN;
  const dim3 grid(mtiles * ntiles * nchunk);
#define TN_ONE(BMv, BNv, BKv, WMv, WNv)                                                       \
  do {                                                                                       \
    if (pro)                                                                                 \
      hipLaunchKernelGGL((k_gemm_tn<T, BMv, BNv, BKv, WMv, WNv, true>), grid, dim3(64 * WMv * WNv), \
                         0, s, A, lda, B, ldb, P, ldp, pstride, K, kchunk, mtiles, ntiles, pt); \
    else                                                                                     \
      hipLaunchKernelGGL((k_gemm_tn<T, BMv, BNv, BKv, WMv, WNv, false>), grid, dim3(64 * WMv * WNv), \
                         0, s, A, lda, B, ldb, P, ldp, pstride, K, kchunk, mtiles, ntiles, pt); \
  } while (0)
#define TN_BN(BMv, BKv, WMv, WNv)                                  \
  switch (BN) {                                               \
    case 32: if (32 % (16 * WNv) == 0) TN_ONE(BMv, 32, BKv, WMv, WNv); break; \
    case 64: TN_ONE(BMv, 64, BKv, WMv, WNv); break;                \
    case 96: if (96 % (16 * WNv) == 0) TN_ONE(BMv, 96, BKv, WMv, WNv); break; \
    case 128: TN_ONE(BMv, 128, BKv, WMv, WNv); break;              \
    default: return hipErrorInvalidValue;                     \
  }
  switch (cfg) {
    case 0: TN_BN(64, 16, 2, 2) break;
    case 1: TN_BN(32, 16, 2, 2) break;
    case 2: TN_BN(64, 32, 4, 2) break;
    case 3: TN_BN(64, 16, 4, 2) break;
  }
#undef TN_BN
#undef TN_ONE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// C = A B with fused epilogues (A: M x K row-major, B: K x N row-major)
// ---------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, int WM, int WN, int EPI>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nn(const T *__restrict__ A, int lda,
                                                          const T *__restrict__ B, int ldb, int K,
                                                          int ntiles, EpiArgs<T> ea) {
  constexpr int NT = 64 * WM * WN;
  constexpr int VN = V16<T>::n;
  constexpr int TM = BM / (16 * WM), TN = BN / (16 * WN);
  static_assert(TM >= 1 && TN >= 1 && TM * 16 * WM == BM && TN * 16 * WN == BN, "tile shape");
  constexpr int PADA = (sizeof(T) == 4) ? 2 : 1;       // k-contiguous rows: stride = 2 mod 32 words
  constexpr int PADB = row_pad<T, BN>();
  constexpr int AV = BM * BK / VN, BV = BK * BN / VN;
  constexpr int AVT = (AV + NT - 1) / NT, BVT = (BV + NT - 1) / NT;
  constexpr int NST = (EPI == EPI_OBJ) ? kObjStats : kAdmmStats;
  typedef typename V16<T>::V VT;
  // operand tiles; the statistics reduction reuses the same LDS after the K loop
  constexpr size_t kBytesA = sizeof(T) * 2 * BM * (BK + PADA);
  constexpr size_t kBytesB = sizeof(T) * 2 * BK * (BN + PADB);
  static_assert(BM % 32 == 0, "statistics partials are per 32-row block");
  constexpr int T16 = BM / 16;   // 16-row tiles of the workgroup
  constexpr bool kStats = EPI == EPI_ADMM_STATS || EPI == EPI_OBJ;
  constexpr size_t kBytesR = kStats ? sizeof(double) * T16 * NST * BN : 0;
  constexpr size_t kBytes = (kBytesA + kBytesB > kBytesR) ? kBytesA + kBytesB : kBytesR;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  auto sA = reinterpret_cast<T (*)[BM][BK + PADA]>(smem);
  auto sB = reinterpret_cast<T (*)[BK][BN + PADB]>(smem + kBytesA);
  auto sred = reinterpret_cast<double (*)[NST][BN]>(smem);   // [16-row tile][stat][column]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // tile order: the column blocks of a row slab are consecutive
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int mt = tile / ntiles, nt = tile % ntiles;
  const int m0 = mt * BM, n0 = nt * BN;
  typename MV<T>::V acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = typename MV<T>::V{0, 0, 0, 0};

  VT ra[AVT], rb[BVT];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int mm = e / (BK / VN), kk = (e % (BK / VN)) * VN;
        ra[i] = *reinterpret_cast<const VT *>(A + (size_t)(m0 + mm) * lda + k0 + kk);
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int kk = e / (BN / VN), nn = (e % (BN / VN)) * VN;
        rb[i] = *reinterpret_cast<const VT *>(B + (size_t)(k0 + kk) * ldb + n0 + nn);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int mm = e / (BK / VN), kk = (e % (BK / VN)) * VN;
        const T *pv = reinterpret_cast<const T *>(&ra[i]);
#pragma unroll
        for (int c = 0; c < VN; ++c) sA[buf][mm][kk + c] = pv[c];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int kk = e / (BN / VN), nn = (e % (BN / VN)) * VN;
        *reinterpret_cast<VT *>(&sB[buf][kk][nn]) = rb[i];
      }
    }
  };

  load(0);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T a[TM], b[TN];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
        a[tm] = sA[buf][wm * TM * 16 + tm * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int tn = 0; tn < TN; ++tn)
        b[tn] = sB[buf][kk + (lane >> 4)][wn * TN * 16 + tn * 16 + (lane & 15)];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma16(a[tm], b[tn], acc[tm][tn]);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
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

  // Statistics: every lane sums its 4 rows of a 16-row tile, the 4 lanes of a
  // column are combined by two shuffles, and the two 16-row tiles of each
  // 32-row block are added.  The partial of a 32-row block is therefore the
  // same for every tile configuration.
  double st[TM][TN][NST];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < TN; ++tn)
#pragma unroll
      for (int q = 0; q < NST; ++q) st[tm][tn][q] = 0.0;

  // per-column step sizes and activity, loaded once
  T irc[TN];
  bool act[TN];
#pragma unroll
  for (int tn = 0; tn < TN; ++tn) {
    const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
    irc[tn] = EPI == EPI_OBJ ? T(0) : (T)ea.invrho[n];
    act[tn] = EPI == EPI_OBJ ? false : ea.active[n] != 0;
  }
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * TM * 16 + tm * 16 + acc_row<T>(lane, r);
      const int g = ea.pt.grp[m];
      const T sg = ea.pt.sig[m];
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
        const T u = upper_of(ea.pt, g, m, n);
        const T s = acc[tm][tn][r];
        if (EPI == EPI_OBJ) {
          // s = sign * dose / threshold at this point for shot times t / E
          if (ea.pt.is_oar[g]) {
            st[tm][tn][1] = fmax(st[tm][tn][1], (double)(-s));
          } else {
            const double h = fmax(0.0, (double)sg - (double)s);
            st[tm][tn][0] = fma((double)u, h, st[tm][tn][0]);
            if (sg > T(0)) st[tm][tn][2] = fma((double)u, (double)s, st[tm][tn][2]);
          }
        } else {
          T *qp = ea.q + (size_t)m * ea.ldq + n;
          const T qv = *qp;
          const T z = clip0u(qv, u);
          // q' = x1 + y1 = z1 - c/rho - A_s' v, with c_p = -sign_p; the next
          // right-hand-side product needs W' = z1' - y1' = 2 clip(q') - q'
          const T qx = z + sg * irc[tn] - s;     // x + y of the closed-form x-step
          // over-relaxed: x_hat + y = alpha (x + y) + (1 - alpha) (z + y)
          const T qn = ea.alpha == 1.0 ? qx : qv + (T)ea.alpha * (qx - qv);
          if (act[tn]) {
            *qp = qn;
            ea.w[(size_t)m * ea.ldq + n] = T(2) * clip0u(qn, u) - qn;
          }
          if (EPI == EPI_ADMM_STATS) {
            const double yo = (double)qv - (double)z;
            const double zn = (double)clip0u(qn, u);
            const double yn = (double)qn - zn;
            const double x = (double)qx - yo;
            // x - z' (the unrelaxed x); without relaxation y' - y is the same value
            const double dxz = ea.alpha == 1.0 ? yn - yo : x - zn, dz = zn - (double)z;
            // explicit fused multiply-adds: the compiler's contraction choices
            // may differ between configurations, these may not
            st[tm][tn][0] = fma(dxz, dxz, st[tm][tn][0]);   // (x - z')^2
            st[tm][tn][1] = fma(x, x, st[tm][tn][1]);
            st[tm][tn][2] = fma(zn, zn, st[tm][tn][2]);
            st[tm][tn][3] = fma(dz, dz, st[tm][tn][3]);
            st[tm][tn][4] = fma(yn, yn, st[tm][tn][4]);
            st[tm][tn][5] = fma(-(double)sg, zn, st[tm][tn][5]);   // c' z1
          }
        }
      }
    }
  if (EPI == EPI_ADMM) return;

  // per 16-row tile: combine the lanes of a column (l, l+16, l+32, l+48)
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < TN; ++tn)
#pragma unroll
      for (int q = 0; q < NST; ++q) {
        double v = st[tm][tn][q];
        if (EPI == EPI_OBJ && q == 1) {
          v = fmax(v, __shfl_xor(v, 16));
          v = fmax(v, __shfl_xor(v, 32));
        } else {
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
        }
        if (lane < 16) sred[wm * TM + tm][q][wn * TN * 16 + tn * 16 + lane] = v;
      }
  __syncthreads();
  for (int e = tid; e < (BM / 32) * NST * BN; e += NT) {
    const int b = e / (NST * BN), q = (e / BN) % NST, c = e % BN;
    const double t0 = sred[2 * b][q][c], t1 = sred[2 * b + 1][q][c];
    const double v = (EPI == EPI_OBJ && q == 1) ? fmax(t0, t1) : t0 + t1;
    ea.stats[((size_t)(mt * (BM / 32) + b) * NST + q) * ea.nstat_cols + n0 + c] = v;
  }
}

// Tile configurations of the point-row product: BM rows, a column block of
// pick_bn(N) / bn_div columns (bn_div = 0: 32 columns), wavefront grid WM x WN.
// Narrower column blocks give more workgroups (better balance over the CUs)
// at the price of reading the row slab once per column block.
struct NnCfg { int bm, bn_div, wm, wn; };
static const NnCfg kNnCfgs[kGemmCfgs] = {{128, 1, 4, 1}, {64, 2, 4, 1}, {128, 0, 4, 1}, {64, 1, 4, 2}};

static int nn_bn(const NnCfg &c, int N) { return c.bn_div == 0 ? 32 : pick_bn(N) / c.bn_div; }



template <typename T>
hipError_t gemm_nn(hipStream_t s, int epi, const T *A, int lda, const T *B, int ldb, int M,
                   int N, int K, const EpiArgs<T> &ea, int cfg) {
  constexpr int BK = 16;
  if (!gemm_nn_cfg_ok(cfg, M, N)) cfg = 0;
  if (!gemm_nn_cfg_ok(cfg, M, N) || N % 32 != 0 || K % BK != 0) return hipErrorInvalidValue;
  if (lda % V16<T>::n || ldb % V16<T>::n) return hipErrorInvalidValue;
  const NnCfg c = kNnCfgs[cfg];
  const int BN = nn_bn(c, N);
  const int ntiles = N / BN;
  const dim3 grid((M / c.bm) * ntiles);
#define NN_ONE(BMv, BNv, WMv, WNv, E)                                                          \
  hipLaunchKernelGGL((k_gemm_nn<T, BMv, BNv, BK, WMv, WNv, E>), grid, dim3(64 * WMv * WNv), 0, s, \
                     A, lda, B, ldb, K, ntiles, ea)
#define NN_E(BMv, BNv, WMv, WNv)                                          \
  switch (epi) {                                                         \
    case EPI_STORE: NN_ONE(BMv, BNv, WMv, WNv, EPI_STORE); break;        \
    case EPI_ADMM: NN_ONE(BMv, BNv, WMv, WNv, EPI_ADMM); break;          \
    case EPI_ADMM_STATS: NN_ONE(BMv, BNv, WMv, WNv, EPI_ADMM_STATS); break; \
    case EPI_OBJ: NN_ONE(BMv, BNv, WMv, WNv, EPI_OBJ); break;            \
    default: return hipErrorInvalidValue;                                \
  }
#define NN_BN(BMv, WMv, WNv)                                              \
  switch (BN) {                                                          \
    case 16: if (WNv == 1) { NN_E(BMv, 16, WMv, 1) } break;               \
    case 32: if (32 % (16 * WNv) == 0) { NN_E(BMv, 32, WMv, WNv) } break; \
    case 48: if (WNv == 1) { NN_E(BMv, 48, WMv, 1) } break;               \
    case 64: { NN_E(BMv, 64, WMv, WNv) } break;                          \
    case 96: if (96 % (16 * WNv) == 0) { NN_E(BMv, 96, WMv, WNv) } break; \
    case 128: { NN_E(BMv, 128, WMv, WNv) } break;                        \
    default: return hipErrorInvalidValue;                                \
  }
  switch (cfg) {
    case 0: NN_BN(128, 4, 1) break;
    case 1: NN_BN(64, 4, 1) break;
    case 2: NN_BN(128, 4, 1) break;
    case 3: NN_BN(64, 4, 2) break;
  }
#undef NN_BN
#undef NN_E
#undef NN_ONE
  return hipGetLastError();
}

}  // namespace ladmm

namespace ladmm {

template <typename T>
__global__ void k_w_from_q(const T *__restrict__ q, T *__restrict__ w, int Np, int kp,
                           PointTable<T> pt) {
  const size_t total = (size_t)Np * kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / kp), j = (int)(e % kp);
    const T qv = q[e];
    w[e] = T(2) * clip0u(qv, upper_of(pt, pt.grp[p], p, j)) - qv;
  }
}

template <typename T>
__global__ void k_rescale_points(T *__restrict__ q, int Np, int kp, PointTable<T> pt,
                                 const double *__restrict__ fac) {
  const size_t total = (size_t)Np * kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / kp), j = (int)(e % kp);
    const double f = fac[j];
    if (f == 1.0) continue;
    const T qv = q[e];
    const T z = clip0u(qv, upper_of(pt, pt.grp[p], p, j));
    q[e] = (T)((double)z + ((double)qv - (double)z) * f);
  }
}

template <typename T>
hipError_t rescale_points(hipStream_t s, T *q, int Np, int kp, const PointTable<T> &pt,
                          const double *fac) {
  hipLaunchKernelGGL((k_rescale_points<T>), dim3(2048), dim3(256), 0, s, q, Np, kp, pt, fac);
  return hipGetLastError();
}

template <typename T>
hipError_t w_from_q(hipStream_t s, const T *q, T *w, int Np, int kp, const PointTable<T> &pt) {
  hipLaunchKernelGGL((k_w_from_q<T>), dim3(2048), dim3(256), 0, s, q, w, Np, kp, pt);
  return hipGetLastError();
}

}  // namespace ladmm
