// BF16-pair MFMA products for the large case (precision mode LADMM_BF16X3).
//
// The dose block D^ and the plan-side operands (W = z1 - y1, v_top, the scaled
// shot times) are carried as pairs hi = bf16(x), lo = bf16(x - hi), which keep
// 16 significant bits.  A product sums A_hi B_hi + A_hi B_lo + A_lo B_hi on the
// v_mfma_f32_16x16x32_bf16 instruction (FP32 accumulation); the dropped A_lo B_lo
// term is below 2^-16 relative.  This is the split-BF16 product that carries the
// x-update of Eq. (partial_elimination) at close to FP32 accuracy on the BF16
// matrix cores; the Schur complement solve and the small side stay FP64.
//
// Layout: both operands row-major with the reduction index contiguous, so a
// lane's fragment (8 consecutive k of one row) is one 16-byte LDS read.
// MFMA 16x16x32 bf16 operand layout (gfx950, checked by a lane probe): lane l
// supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7, and
// receives D[4 (l / 16) + r][l % 16] in accumulator register r.
#include "kernels.h"

#include <math.h>

#include <algorithm>

namespace ladmm {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4v mfma_bf(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t bf_bits(__bf16 x) { return __builtin_bit_cast(uint16_t, x); }

// hi = bf16(x), lo = bf16(x - hi), both round-to-nearest-even.
__device__ __forceinline__ void split_pair(double x, uint16_t &h, uint16_t &l) {
  const __bf16 bh = (__bf16)(float)x;
  const double r = x - (double)(float)bh;
  h = bf_bits(bh);
  l = bf_bits((__bf16)(float)r);
}

__device__ __forceinline__ float clip0u_f(float q, float u) { return fminf(fmaxf(q, 0.f), u); }

// Consecutive tile indices on one XCD (workgroups go round-robin over the 8
// XCDs); a bijection on [0, total).
__device__ __forceinline__ int xcd_tile_bf(int id, int total) {
  constexpr int X = 8;
  const int per = (total + X - 1) / X;
  const int tall = total % X == 0 ? X : total % X;
  const int xcd = id % X, local = id / X;
  return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

__device__ __forceinline__ float upper_bf(const PointTable<float> &pt, int g, int p, int j) {
  float u = pt.utab[(size_t)g * pt.ldu + j];
  if (pt.mask != nullptr && pt.is_ld[g]) {
    uint64_t w = pt.mask[(size_t)j * pt.mask_words + (p >> 6)];
    if (!((w >> (p & 63)) & 1ull)) u = 0.f;
  }
  return u;
}

constexpr int kBfBK = 32;              // one MFMA k-step per stage
constexpr int kBfLd = kBfBK + 8;       // LDS row: 80 bytes, 8 rows cover all banks

// MODE 0: split-K partial store; otherwise the NN epilogue EPI_ADMM / _STATS / _OBJ.
// NBUF: 2 = double-buffered LDS stages; 1 = one stage (half the LDS, so more
// workgroups per CU), the next stage waiting in registers behind a barrier.
template <int BM, int BN, int WM, int WN, int TERMS, int MODE, int NBUF>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_bf(BfPair A, BfPair B, int K, int kchunk,
                                                         int mtiles, int ntiles,
                                                         float *__restrict__ P, int ldp,
                                                         size_t pstride, EpiArgs<float> ea) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / (16 * WM), TN = BN / (16 * WN);
  static_assert(TM >= 1 && TN >= 1 && TM * 16 * WM == BM && TN * 16 * WN == BN, "tile shape");
  static_assert(MODE == 0 || BM % 32 == 0, "statistics partials are per 32-row block");
  constexpr int KV = kBfBK / 8;                        // 16-byte vectors per row slice
  constexpr int AV = BM * KV, BV = BN * KV;
  constexpr int AVT = (AV + NT - 1) / NT, BVT = (BV + NT - 1) / NT;
  constexpr bool ALO = TERMS == 3;
  constexpr int NST = (MODE == EPI_OBJ) ? kObjStats : kAdmmStats;
  constexpr bool kStats = MODE == EPI_ADMM_STATS || MODE == EPI_OBJ;
  constexpr int T16 = BM / 16;
  constexpr size_t kTileA = sizeof(uint16_t) * NBUF * BM * kBfLd;
  constexpr size_t kTileB = sizeof(uint16_t) * NBUF * BN * kBfLd;
  constexpr size_t kBytesT = kTileA * (ALO ? 2 : 1) + kTileB * 2;
  constexpr size_t kBytesR = kStats ? sizeof(double) * T16 * NST * BN : 0;
  constexpr size_t kBytes = kBytesT > kBytesR ? kBytesT : kBytesR;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  auto sAh = reinterpret_cast<uint16_t (*)[BM][kBfLd]>(smem);
  auto sBh = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem + kTileA);
  auto sBl = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem + kTileA + kTileB);
  auto sAl = reinterpret_cast<uint16_t (*)[BM][kBfLd]>(smem + kTileA + 2 * kTileB);
  auto sred = reinterpret_cast<double (*)[NST][BN]>(smem);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // tile order: column blocks fastest (they share the row slab of A), then
  // row tiles (which share a split-K chunk of B), then chunks
  const int tile = xcd_tile_bf(blockIdx.x, gridDim.x);
  const int nt = tile % ntiles, mt = (tile / ntiles) % mtiles, zc = tile / (mtiles * ntiles);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = MODE == 0 ? zc * kchunk : 0;
  const int kend = MODE == 0 ? min(K, kbeg + kchunk) : K;

  f4v acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};

  uint4 rah[AVT], ral[ALO ? AVT : 1], rbh[BVT], rbl[BVT];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int row = e / KV, k = k0 + (e % KV) * 8;
        const size_t off = (size_t)(m0 + row) * A.ld + k;
        rah[i] = k < kend ? *reinterpret_cast<const uint4 *>(A.hi + off) : uint4{0, 0, 0, 0};
        if (ALO) ral[i] = k < kend ? *reinterpret_cast<const uint4 *>(A.lo + off) : uint4{0, 0, 0, 0};
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int row = e / KV, k = k0 + (e % KV) * 8;
        const size_t off = (size_t)(n0 + row) * B.ld + k;
        rbh[i] = k < kend ? *reinterpret_cast<const uint4 *>(B.hi + off) : uint4{0, 0, 0, 0};
        rbl[i] = k < kend ? *reinterpret_cast<const uint4 *>(B.lo + off) : uint4{0, 0, 0, 0};
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int row = e / KV, kv = (e % KV) * 8;
        *reinterpret_cast<uint4 *>(&sAh[buf][row][kv]) = rah[i];
        if (ALO) *reinterpret_cast<uint4 *>(&sAl[buf][row][kv]) = ral[i];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int row = e / KV, kv = (e % KV) * 8;
        *reinterpret_cast<uint4 *>(&sBh[buf][row][kv]) = rbh[i];
        *reinterpret_cast<uint4 *>(&sBl[buf][row][kv]) = rbl[i];
      }
    }
  };

  if (kbeg < kend) {
    load(kbeg);
    store(0);
    __syncthreads();
    int buf = 0;
    const int g8 = 8 * (lane >> 4), r16 = lane & 15;
    for (int k0 = kbeg; k0 < kend; k0 += kBfBK) {
      const bool more = k0 + kBfBK < kend;
      if (more) load(k0 + kBfBK);
      bf8v ah[TM], al[ALO ? TM : 1], bh[TN], bl[TN];
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const int row = wm * TM * 16 + tm * 16 + r16;
        ah[tm] = *reinterpret_cast<const bf8v *>(&sAh[buf][row][g8]);
        if (ALO) al[tm] = *reinterpret_cast<const bf8v *>(&sAl[buf][row][g8]);
      }
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const int row = wn * TN * 16 + tn * 16 + r16;
        bh[tn] = *reinterpret_cast<const bf8v *>(&sBh[buf][row][g8]);
        bl[tn] = *reinterpret_cast<const bf8v *>(&sBl[buf][row][g8]);
      }
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          acc[tm][tn] = mfma_bf(ah[tm], bh[tn], acc[tm][tn]);
          acc[tm][tn] = mfma_bf(ah[tm], bl[tn], acc[tm][tn]);
          if (ALO) acc[tm][tn] = mfma_bf(al[tm], bh[tn], acc[tm][tn]);
        }
      if (NBUF == 2) {
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      } else {
        __syncthreads();          // every wave has read the stage
        if (more) store(0);
        __syncthreads();
      }
    }
  }

  if (MODE == 0) {
    float *Pz = P + (size_t)zc * pstride;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int tn = 0; tn < TN; ++tn)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * TM * 16 + tm * 16 + 4 * (lane >> 4) + r;
          const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
          Pz[(size_t)m * ldp + n] = acc[tm][tn][r];
        }
    return;
  }

  // Epilogue on the point-row product: the same arithmetic as the FP32 path,
  // with W' written plan-major as pairs.  Statistics: per 16-row tile, every
  // lane sums its 4 rows, two shuffles combine the 4 lanes of a column, and the
  // two tiles of each 32-row block are added (one partial per 32-row block).
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
      const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
      const int mb = m0 + wm * TM * 16 + tm * 16 + 4 * (lane >> 4);
      double st[NST];
#pragma unroll
      for (int q = 0; q < NST; ++q) st[q] = 0.0;
      uint16_t wh[4] = {0, 0, 0, 0}, wl[4] = {0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = mb + r;
        const int g = ea.pt.grp[m];
        const float sg = ea.pt.sig[m];
        const float u = upper_bf(ea.pt, g, m, n);
        const float s = acc[tm][tn][r];
        if (MODE == EPI_OBJ) {
          if (ea.pt.is_oar[g]) {
            st[1] = fmax(st[1], (double)(-s));
          } else {
            const double h = fmax(0.0, (double)sg - (double)s);
            st[0] = fma((double)u, h, st[0]);
          }
        } else {
          float *qp = ea.q + (size_t)m * ea.ldq + n;
          const float qv = *qp;
          const float z = clip0u_f(qv, u);
          const float qn = z + sg * (float)ea.invrho[n] - s;
          const float wv = 2.f * clip0u_f(qn, u) - qn;
          split_pair((double)wv, wh[r], wl[r]);
          if (ea.active[n]) *qp = qn;
          if (MODE == EPI_ADMM_STATS) {
            const double yo = (double)qv - (double)z;
            const double zn = (double)clip0u_f(qn, u);
            const double yn = (double)qn - zn;
            const double x = (double)qn - yo;
            const double dxz = yn - yo, dz = zn - (double)z;
            st[0] = fma(dxz, dxz, st[0]);
            st[1] = fma(x, x, st[1]);
            st[2] = fma(zn, zn, st[2]);
            st[3] = fma(dz, dz, st[3]);
            st[4] = fma(yn, yn, st[4]);
            st[5] = fma(-(double)sg, zn, st[5]);
          }
        }
      }
      if (MODE != EPI_OBJ && ea.active[n]) {
        const size_t o = (size_t)n * ea.ldwt + mb;
        *reinterpret_cast<uint2 *>(ea.wt_hi + o) =
            uint2{(uint32_t)wh[0] | ((uint32_t)wh[1] << 16), (uint32_t)wh[2] | ((uint32_t)wh[3] << 16)};
        *reinterpret_cast<uint2 *>(ea.wt_lo + o) =
            uint2{(uint32_t)wl[0] | ((uint32_t)wl[1] << 16), (uint32_t)wl[2] | ((uint32_t)wl[3] << 16)};
      }
      if (kStats) {
        // the operand tiles are no longer read: every wave passed the last barrier
#pragma unroll
        for (int q = 0; q < NST; ++q) {
          double v = st[q];
          if (MODE == EPI_OBJ && q == 1) {
            v = fmax(v, __shfl_xor(v, 16));
            v = fmax(v, __shfl_xor(v, 32));
          } else {
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
          }
          if (lane < 16) sred[wm * TM + tm][q][wn * TN * 16 + tn * 16 + lane] = v;
        }
      }
    }
  if (!kStats) return;
  __syncthreads();
  for (int e = tid; e < (BM / 32) * NST * BN; e += NT) {
    const int b = e / (NST * BN), q = (e / BN) % NST, c = e % BN;
    const double t0 = sred[2 * b][q][c], t1 = sred[2 * b + 1][q][c];
    const double v = (MODE == EPI_OBJ && q == 1) ? fmax(t0, t1) : t0 + t1;
    ea.stats[((size_t)(mt * (BM / 32) + b) * NST + q) * ea.nstat_cols + n0 + c] = v;
  }
}

// Tile configurations (rows BM, columns BN, wavefront grid WM x WN, LDS
// stages) of the split-K product (which = 0) and the point-row product (1).
struct BfCfg { int bm, bn, wm, wn, nbuf; };
static const BfCfg kBfCfgs[2][kGemmCfgs] = {
    {{64, 32, 2, 1, 2}, {64, 64, 2, 1, 1}, {64, 64, 4, 1, 1}, {128, 64, 4, 1, 1}},
    {{64, 32, 2, 1, 2}, {128, 32, 4, 1, 1}, {128, 64, 4, 1, 1}, {256, 64, 4, 1, 1}}};

bool gemm_bf_cfg_ok(int which, int cfg, int M, int N) {
  if (cfg < 0 || cfg >= kGemmCfgs) return false;
  const BfCfg c = kBfCfgs[which][cfg];
  return M % c.bm == 0 && N % c.bn == 0;
}

template <int MODE, int TERMS>
static hipError_t launch_bf(int cfg, int M, int N, int nchunk, hipStream_t s, BfPair A, BfPair B,
                            int K, int kchunk, float *P, int ldp, size_t pstride,
                            const EpiArgs<float> &ea) {
  const BfCfg c = kBfCfgs[MODE == 0 ? 0 : 1][cfg];
  const int mtiles = M / c.bm, ntiles = N / c.bn;
  const dim3 grid(mtiles * ntiles * nchunk);
#define BF_ONE(BMv, BNv, WMv, WNv, NB)                                                             \
  hipLaunchKernelGGL((k_gemm_bf<BMv, BNv, WMv, WNv, TERMS, MODE, NB>), grid, dim3(64 * WMv * WNv), 0, \
                     s, A, B, K, kchunk, mtiles, ntiles, P, ldp, pstride, ea)
  if (MODE == 0) {
    switch (cfg) {
      case 0: BF_ONE(64, 32, 2, 1, 2); break;
      case 1: BF_ONE(64, 64, 2, 1, 1); break;
      case 2: BF_ONE(64, 64, 4, 1, 1); break;
      case 3: BF_ONE(128, 64, 4, 1, 1); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (cfg) {
      case 0: BF_ONE(64, 32, 2, 1, 2); break;
      case 1: BF_ONE(128, 32, 4, 1, 1); break;
      case 2: BF_ONE(128, 64, 4, 1, 1); break;
      case 3: BF_ONE(256, 64, 4, 1, 1); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef BF_ONE
  return hipGetLastError();
}

hipError_t gemm_bf_tn(hipStream_t s, BfPair A, BfPair B, float *P, int ldp, int M, int N, int K,
                      int nchunk, int terms, int cfg) {
  if (!gemm_bf_cfg_ok(0, cfg, M, N)) cfg = 0;
  if (!gemm_bf_cfg_ok(0, cfg, M, N) || nchunk < 1 || K % 8 || A.ld % 8 || B.ld % 8)
    return hipErrorInvalidValue;
  int kchunk = (K + nchunk - 1) / nchunk;
  kchunk = (kchunk + 31) / 32 * 32;
  const EpiArgs<float> ea{};
  const size_t pstride = (size_t)M * ldp;
  return terms == 3 ? launch_bf<0, 3>(cfg, M, N, nchunk, s, A, B, K, kchunk, P, ldp, pstride, ea)
                    : launch_bf<0, 2>(cfg, M, N, nchunk, s, A, B, K, kchunk, P, ldp, pstride, ea);
}

hipError_t gemm_bf_nn(hipStream_t s, int epi, BfPair A, BfPair B, int M, int N, int K,
                      const EpiArgs<float> &ea, int terms, int cfg) {
  if (!gemm_bf_cfg_ok(1, cfg, M, N)) cfg = 0;
  if (!gemm_bf_cfg_ok(1, cfg, M, N) || K % kBfBK || A.ld % 8 || B.ld % 8) return hipErrorInvalidValue;
#define BF_EPI(E)                                                                               \
  return terms == 3 ? launch_bf<E, 3>(cfg, M, N, 1, s, A, B, K, K, nullptr, 0, 0, ea)           \
                    : launch_bf<E, 2>(cfg, M, N, 1, s, A, B, K, K, nullptr, 0, 0, ea)
  switch (epi) {
    case EPI_ADMM: BF_EPI(EPI_ADMM);
    case EPI_ADMM_STATS: BF_EPI(EPI_ADMM_STATS);
    case EPI_OBJ: BF_EPI(EPI_OBJ);
    default: return hipErrorInvalidValue;
  }
#undef BF_EPI
}

// ---------------------------------------------------------------------------
// operand preparation
// ---------------------------------------------------------------------------
// Point-major pairs: one thread per element, coalesced along shots.
__global__ void k_split_dose(const double *__restrict__ Dt, const double *__restrict__ E, int Np,
                             int ntp, uint16_t *__restrict__ Dh, uint16_t *__restrict__ Dl) {
  const size_t total = (size_t)Np * ntp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int t = (int)(e % ntp);
    uint16_t h, l;
    split_pair(Dt[e] * E[t], h, l);
    Dh[e] = h;
    Dl[e] = l;
  }
}

// Shot-major copy through a 64 x 64 LDS tile.
__global__ void k_transpose_u16(const uint16_t *__restrict__ in, int rows, int cols,
                                uint16_t *__restrict__ out) {
  __shared__ uint16_t tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  for (int i = threadIdx.y; i < 64; i += blockDim.y) {
    const int r = r0 + i, c = c0 + threadIdx.x;
    tile[i][threadIdx.x] = (r < rows && c < cols) ? in[(size_t)r * cols + c] : 0;
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 64; i += blockDim.y) {
    const int c = c0 + i, r = r0 + threadIdx.x;
    if (c < cols && r < rows) out[(size_t)c * rows + r] = tile[threadIdx.x][i];
  }
}

hipError_t split_dose_bf16(hipStream_t s, const double *Dt, const double *E, int Np, int ntp,
                           uint16_t *Dh, uint16_t *Dl, uint16_t *DTh, uint16_t *DTl) {
  hipLaunchKernelGGL(k_split_dose, dim3(4096), dim3(256), 0, s, Dt, E, Np, ntp, Dh, Dl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid((ntp + 63) / 64, (Np + 63) / 64);
  hipLaunchKernelGGL(k_transpose_u16, grid, dim3(64, 4), 0, s, Dh, Np, ntp, DTh);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_transpose_u16, grid, dim3(64, 4), 0, s, Dl, Np, ntp, DTl);
  return hipGetLastError();
}

// v = sum of the S^-1 r partials; v_top as plan-major pairs (kp x ntp).
__global__ void k_vreduce_bf(SmallArgs a, const double *__restrict__ P2, size_t zstride, int nchunk,
                             double *__restrict__ v, uint16_t *__restrict__ vh,
                             uint16_t *__restrict__ vl) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.mAp || j >= a.kp) return;
  const size_t idx = (size_t)m * a.kp + j;
  double acc = 0.0;
#pragma unroll 8
  for (int z = 0; z < nchunk; ++z) acc += P2[z * zstride + idx];
  v[idx] = acc;
  if (m < a.L.ntp) {
    uint16_t h, l;
    split_pair(acc, h, l);
    vh[(size_t)j * a.L.ntp + m] = h;
    vl[(size_t)j * a.L.ntp + m] = l;
  }
}

hipError_t vreduce_bf(hipStream_t s, const SmallArgs &a, const double *P2, size_t zstride, int nchunk,
                      double *v, uint16_t *vh, uint16_t *vl) {
  hipLaunchKernelGGL(k_vreduce_bf, dim3((a.L.mAp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s, a,
                     P2, zstride, nchunk, v, vh, vl);
  return hipGetLastError();
}

// that = rho max(q2_top, 0) (the shot times over E) as plan-major pairs.
__global__ void k_shot_scaled_bf(SmallArgs a, const double *__restrict__ q2, uint16_t *__restrict__ th,
                                 uint16_t *__restrict__ tl) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.ntp || j >= a.kp) return;
  const double ir = a.invrho[j];
  const double t = (m < a.L.n_t && ir > 0.0) ? fmax(q2[(size_t)m * a.kp + j], 0.0) / ir : 0.0;
  uint16_t h, l;
  split_pair(t, h, l);
  th[(size_t)j * a.L.ntp + m] = h;
  tl[(size_t)j * a.L.ntp + m] = l;
}

hipError_t shot_scaled_bf(hipStream_t s, const SmallArgs &a, const double *q2, uint16_t *th,
                          uint16_t *tl) {
  hipLaunchKernelGGL(k_shot_scaled_bf, dim3((a.L.ntp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s,
                     a, q2, th, tl);
  return hipGetLastError();
}

__global__ void k_w_from_q_bf(const float *__restrict__ q, int Np, int kp, PointTable<float> pt,
                              uint16_t *__restrict__ wh, uint16_t *__restrict__ wl) {
  const size_t total = (size_t)Np * kp;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(e / kp), j = (int)(e % kp);
    const float qv = q[e];
    const float w = 2.f * clip0u_f(qv, upper_bf(pt, pt.grp[p], p, j)) - qv;
    uint16_t h, l;
    split_pair((double)w, h, l);
    wh[(size_t)j * Np + p] = h;
    wl[(size_t)j * Np + p] = l;
  }
}

hipError_t w_from_q_bf(hipStream_t s, const float *q, int Np, int kp, const PointTable<float> &pt,
                       uint16_t *wh, uint16_t *wl) {
  hipLaunchKernelGGL(k_w_from_q_bf, dim3(2048), dim3(256), 0, s, q, Np, kp, pt, wh, wl);
  return hipGetLastError();
}

// Zero the rows j (hi and lo) of plan-major pairs (2 kp rows of len) whose
// flag[j] is nonzero: a fresh plan in a reused column.
__global__ void k_zero_plan_rows(uint16_t *__restrict__ a, int kp, int len, const int32_t *__restrict__ flag) {
  const size_t total = (size_t)2 * kp * len;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    if (flag[(e / len) % kp]) a[e] = 0;
}

hipError_t zero_plan_rows_bf(hipStream_t s, uint16_t *a, int kp, int len, const int32_t *flag) {
  hipLaunchKernelGGL(k_zero_plan_rows, dim3(2048), dim3(256), 0, s, a, kp, len, flag);
  return hipGetLastError();
}

}  // namespace ladmm
