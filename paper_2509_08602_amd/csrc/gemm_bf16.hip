// BF16 MFMA products for the large case (precision modes LADMM_BF16X3 and
// LADMM_BF16).
//
// The dose block D^ and the plan-side operands (W = z1 - y1, v_top, the scaled
// shot times) are carried as pairs hi = bf16(x), lo = bf16(x - hi), which keep
// 16 significant bits.  A product sums A_hi B_hi + A_hi B_lo + A_lo B_hi on the
// v_mfma_f32_16x16x32_bf16 instruction (FP32 accumulation); the dropped A_lo B_lo
// term is below 2^-16 relative.  This is the split-BF16 product that carries the
// x-update of Eq. (partial_elimination) at close to FP32 accuracy on the BF16
// matrix cores; the Schur complement solve and the small side stay FP64.
//
// LADMM_BF16 reads the dose block as a single BF16 operand (the hi half) in
// every hot iteration and multiplies it by the change of the plan-side operand
// since the last refresh, dW = bf16(W - W_ref) and dv = bf16(v - v_ref):
//   A_s W = G_ref + D_hi' dW,   A_s' v = X_ref + D_hi dv,
// where G_ref = D^' W_ref and X_ref = D^ v_ref are three-term (near FP32)
// products taken at the last refresh.  The BF16 rounding of the dose block and
// of the operand then acts only on the change, which shrinks as the iterates
// converge, so the fixed point is that of the exact products: this is the
// iterative refinement of the x-update of Eq. (partial_elimination).  The
// refresh is the last iteration of every check chunk, so the statistics and
// the objective of every check come from the three-term products.
//
// MFMA 16x16x32 bf16 operand layout (gfx950, checked by a lane probe): lane l
// supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7, and
// receives D[4 (l / 16) + r][l % 16] in accumulator register r.
//
// Layouts.  The dose block (operand A of both products) is stored in fragment
// order: for every 16-row tile and every 32-wide k step, the 64 lanes' 16-byte
// pieces (lane l: row l % 16, k 8 (l / 16) .. + 8) are consecutive, so a
// fragment is 1 KiB of contiguous HBM and a wavefront loads it with one fully
// coalesced 16-byte-per-lane instruction (frag_off gives the offsets).
// The plan-side operand B (W, v_top, the scaled shot times) is plan-major with
// the reduction index contiguous; both are staged through LDS as rows with the
// k index contiguous, so a lane's fragment is one 16-byte LDS read.
#include "kernels.h"
#include "warm.h"

#include <math.h>

#include <algorithm>

namespace ladmm {

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
// 16 bytes of operand as a plain vector (register rings of loads stay in VGPRs)
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

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

__device__ __forceinline__ float bf_val(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// The value a pair carries: hi + lo is exact in FP32 (17 significant bits at most).
__device__ __forceinline__ float pair_val(uint16_t h, uint16_t l) { return bf_val(h) + bf_val(l); }

__device__ __forceinline__ uint16_t bf_round(float x) { return bf_bits((__bf16)x); }

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

// Element offset of the 16-byte piece (row, k .. k + 7), k % 8 == 0, of an
// M x K operand in fragment order (K % 32 == 0).
__host__ __device__ __forceinline__ size_t frag_off(int row, int k, int K) {
  return ((size_t)(row >> 4) * (size_t)(K >> 5) + (size_t)(k >> 5)) * 512 +
         (size_t)((((k & 31) >> 3) << 4) | (row & 15)) * 8;
}

__device__ __forceinline__ float upper_bf(const PointTable<float> &pt, int g, int p, int j) {
  float u = pt.utab[(size_t)g * pt.ldu + j];
  if (pt.mask != nullptr && pt.is_ld[g]) {
    uint64_t w = pt.mask[(size_t)j * pt.mask_words + (p >> 6)];
    if (!((w >> (p & 63)) & 1ull)) u = 0.f;
  }
  return u;
}

constexpr int kBfBK = 32;              // one MFMA k-step
constexpr int kBfLd = kBfBK + 8;       // LDS row: 80 bytes, 8 rows cover all banks

template <int MODE>
constexpr int bf_nstat() { return MODE == EPI_OBJ ? kObjStats : kAdmmStats; }
template <int MODE>
constexpr bool bf_has_stats() { return MODE == EPI_ADMM_STATS || MODE == EPI_OBJ; }
// LDS of the epilogue: the statistics partials (one per 16-row tile, statistic
// and column); in the plain ADMM epilogue, W' hi and lo halves (or dW alone in
// the BF_DELTA variant) staged as BN columns of BM rows (padded by 8 elements,
// 16-byte aligned columns) so that each plan's rows leave as contiguous
// 16-byte pieces.  The statistics variant (one launch per convergence check)
// stores its plan-major outputs directly instead: staging on top of its
// partials would halve its occupancy.
template <int BM, int BN, int MODE>
constexpr size_t bf_stat_bytes() { return bf_has_stats<MODE>() ? sizeof(double) * (BM / 16) * bf_nstat<MODE>() * BN : 0; }
template <int BM>
constexpr int bf_wstage_ld() { return BM + 8; }
template <int DL>
constexpr int bf_wstage_halves() { return DL == BF_DELTA ? 1 : 2; }
// Staged only where the staging fits beside the operand tiles' LDS (the widest
// tiles write W' pairs directly).
template <int BM, int BN, int MODE, int DL>
constexpr bool bf_wstaged() {
  return MODE == EPI_ADMM && bf_wstage_halves<DL>() * sizeof(uint16_t) * BN * bf_wstage_ld<BM>() <= 128 * 1024;
}
template <int BM, int BN, int MODE, int DL>
constexpr size_t bf_red_bytes() {
  return bf_stat_bytes<BM, BN, MODE>() +
         (bf_wstaged<BM, BN, MODE, DL>() ? bf_wstage_halves<DL>() * sizeof(uint16_t) * BN * bf_wstage_ld<BM>() : 0);
}

__device__ __forceinline__ bf8v as_bf8(uint4 u) { return __builtin_bit_cast(bf8v, u); }
__device__ __forceinline__ bf8v as_bf8(u4v u) { return __builtin_bit_cast(bf8v, u); }

__device__ __forceinline__ uint2 pack4(const uint16_t (&v)[4]) {
  return uint2{(uint32_t)v[0] | ((uint32_t)v[1] << 16), (uint32_t)v[2] | ((uint32_t)v[3] << 16)};
}

// After the k loop, shared by both kernels.  MODE 0: the split-K partial
// store; otherwise the point-row epilogue EPI_ADMM / _STATS / _OBJ with the
// same arithmetic as the FP32 path and W' written plan-major.  DL selects the
// variant of the BF16 refinement mode (BF_PLAIN for the pair mode and the
// objective product).
// Statistics: per 16-row tile, every lane sums its 4 rows, two shuffles combine
// the 4 lanes of a column, and the two tiles of each 32-row block are added
// (one partial per 32-row block).  `smem` must hold bf_red_bytes and no wave
// may still read operand tiles from it.
// Waves per SIMD the registers of a pair-product kernel must allow: two up to
// 16 accumulator tiles per wave (the batched epilogue would otherwise take
// enough registers to halve the occupancy), else one.
constexpr int bf_min_waves(int tm, int tn) { return tm * tn <= 16 ? 2 : 1; }

// Tiles per batch of the point-row epilogue (the last batch may be shorter):
// fewer where the accumulators already take most of the registers.
constexpr int bf_epi_batch(int tm, int tn) { return tm * tn >= 28 ? 2 : tn < 4 ? tn : 4; }

template <int BM, int BN, int WM, int WN, int MODE, int DL>
__device__ __forceinline__ void bf_epilogue(f4v (&acc)[BM / (16 * WM)][BN / (16 * WN)],
                                            unsigned char *smem, int tid, int mt, int m0, int n0,
                                            int zc, float *__restrict__ P, int ldp, size_t pstride,
                                            const EpiArgs<float> &ea) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / (16 * WM), TN = BN / (16 * WN);
  constexpr int NST = bf_nstat<MODE>();
  constexpr bool kStats = bf_has_stats<MODE>();
  constexpr bool kDeltaIn = DL == BF_DELTA || DL == BF_DELTA_PAIR;   // product = X_ref + D_hi dv
  constexpr bool kPairsOut = DL != BF_DELTA;                          // W' as pairs
  constexpr bool kDwOut = DL == BF_DELTA || DL == BF_REFRESH;         // dW = bf16(W' - W_ref)
  static_assert(MODE != EPI_OBJ || DL == BF_PLAIN, "the objective product has no refinement variant");
  static_assert(DL != BF_REFRESH || !bf_wstaged<BM, BN, MODE, DL>(), "the refresh stores its outputs directly");
  static_assert(MODE != EPI_ADMM_STATS || DL == BF_PLAIN || DL == BF_REFRESH,
                "statistics come from the pair products");
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
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
  auto sred = reinterpret_cast<double (*)[NST][BN]>(smem);
  constexpr int LDW = bf_wstage_ld<BM>();
  auto swh = reinterpret_cast<uint16_t (*)[LDW]>(smem + bf_stat_bytes<BM, BN, MODE>());
  auto swl = reinterpret_cast<uint16_t (*)[LDW]>(smem + bf_stat_bytes<BM, BN, MODE>() +
                                                  sizeof(uint16_t) * BN * LDW);
  // per-row (group, sign, whether its bound follows the low-dose mask) and
  // per-column (1/rho, active) values, loaded once
  int grow[TM][4];
  float srow[TM][4];
  bool lrow[TM][4];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm * TM * 16 + tm * 16 + 4 * (lane >> 4) + r;
      grow[tm][r] = ea.pt.grp[m];
      srow[tm][r] = ea.pt.sig[m];
      lrow[tm][r] = ea.pt.mask != nullptr && ea.pt.is_ld[grow[tm][r]] != 0;
    }
  float irc[TN];
  bool act[TN];
#pragma unroll
  for (int tn = 0; tn < TN; ++tn) {
    const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
    irc[tn] = MODE == EPI_OBJ ? 0.f : (float)ea.invrho[n];
    act[tn] = MODE == EPI_OBJ ? false : ea.active[n] != 0;
  }
  // Tiles go in batches of NB: every load of a batch (q, the references and the
  // bounds u) is issued before any of its stores.  Loads and stores share one
  // counter, and once both are in flight a wait is a wait for all of them, so
  // interleaving them per tile would cost a memory round trip per tile.
  constexpr int NB = bf_epi_batch(TM, TN);
  float qv4[NB][4], xr4[NB][4], wr4[NB][4], uu4[NB][4];
  uint64_t mw[NB];
#pragma unroll
  for (int tm = 0; tm < TM; ++tm)
#pragma unroll
    for (int tb = 0; tb < TN; tb += NB) {
      if (MODE != EPI_OBJ) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (tb + b >= TN) break;
          const int n = n0 + wn * TN * 16 + (tb + b) * 16 + (lane & 15);
          const int mb = m0 + wm * TM * 16 + tm * 16 + 4 * (lane >> 4);
          // the low-dose mask word of rows mb .. mb + 3 (one 64-row block)
          mw[b] = ea.pt.mask != nullptr ? ea.pt.mask[(size_t)n * ea.pt.mask_words + (mb >> 6)] : ~0ull;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t o = (size_t)(mb + r) * ea.ldq + n;
            uu4[b][r] = ea.pt.utab[(size_t)grow[tm][r] * ea.pt.ldu + n];
            qv4[b][r] = ea.q[o];
            if (kDeltaIn) xr4[b][r] = ea.xref[o];
            if (DL == BF_DELTA) wr4[b][r] = ea.wref[o];
          }
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int tn = tb + b;
        if (tn >= TN) break;
        const int n = n0 + wn * TN * 16 + tn * 16 + (lane & 15);
        const int mb = m0 + wm * TM * 16 + tm * 16 + 4 * (lane >> 4);
        double st[NST];
#pragma unroll
        for (int q = 0; q < NST; ++q) st[q] = 0.0;
        uint16_t wh[4] = {0, 0, 0, 0}, wl[4] = {0, 0, 0, 0}, dw[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + r;
          const int g = grow[tm][r];
          const float sg = srow[tm][r];
          // upper_bf from the values of the load phase
          const float u = MODE == EPI_OBJ                                ? upper_bf(ea.pt, g, m, n)
                          : lrow[tm][r] && !((mw[b] >> (m & 63)) & 1ull) ? 0.f
                                                                         : uu4[b][r];
          float s = acc[tm][tn][r];
          if (kDeltaIn) s = xr4[b][r] + s;
          if (MODE == EPI_OBJ) {
            if (ea.pt.is_oar[g]) {
              st[1] = fmax(st[1], (double)(-s));
            } else {
              const double h = fmax(0.0, (double)sg - (double)s);
              st[0] = fma((double)u, h, st[0]);
              if (sg > 0.f) st[2] = fma((double)u, (double)s, st[2]);
            }
          } else {
            const float qv = qv4[b][r];
            const float z = clip0u_f(qv, u);
            float wref = 0.f;
            if (DL == BF_DELTA) wref = wr4[b][r];
            if (DL == BF_REFRESH) {
              // the references of the running plans (a frozen plan keeps those
              // of its last refresh, consistent with its G_ref and v_ref, which
              // are recorded for running plans only too)
              uint16_t h, l;
              split_pair((double)(2.f * z - qv), h, l);   // the pairs the refresh's GEMM1 read
              wref = pair_val(h, l);
              if (act[tn]) {
                const size_t o = (size_t)m * ea.ldq + n;
                ea.xref[o] = s;
                ea.wref[o] = wref;
              }
            }
            const float qx = z + sg * irc[tn] - s;   // x + y of the closed-form x-step
            // over-relaxed: x_hat + y = alpha (x + y) + (1 - alpha) (z + y)
            const float qn = ea.alpha == 1.0 ? qx : qv + (float)ea.alpha * (qx - qv);
            const float wv = 2.f * clip0u_f(qn, u) - qn;
            if (kPairsOut) split_pair((double)wv, wh[r], wl[r]);
            if (kDwOut) dw[r] = bf_round(wv - wref);
            if (act[tn]) ea.q[(size_t)m * ea.ldq + n] = qn;
            if (MODE == EPI_ADMM_STATS) {
              const double yo = (double)qv - (double)z;
              const double zn = (double)clip0u_f(qn, u);
              const double yn = (double)qn - zn;
              const double x = (double)qx - yo;
              // x - z' (the unrelaxed x); without relaxation y' - y is the same value
              const double dxz = ea.alpha == 1.0 ? yn - yo : x - zn, dz = zn - (double)z;
              st[0] = fma(dxz, dxz, st[0]);
              st[1] = fma(x, x, st[1]);
              st[2] = fma(zn, zn, st[2]);
              st[3] = fma(dz, dz, st[3]);
              st[4] = fma(yn, yn, st[4]);
              st[5] = fma(-(double)sg, zn, st[5]);
            }
          }
        }
        if (bf_wstaged<BM, BN, MODE, DL>()) {
          // staged: column n - n0, rows mb - m0 .. + 3
          const int cl = n - n0, rl = mb - m0;
          if (DL == BF_DELTA) {
            *reinterpret_cast<uint2 *>(&swh[cl][rl]) = pack4(dw);
          } else {
            *reinterpret_cast<uint2 *>(&swh[cl][rl]) = pack4(wh);
            *reinterpret_cast<uint2 *>(&swl[cl][rl]) = pack4(wl);
          }
        } else if (MODE != EPI_OBJ && act[tn]) {
          const size_t o = (size_t)n * ea.ldwt + mb;
          if (kPairsOut) {
            *reinterpret_cast<uint2 *>(ea.wt_hi + o) = pack4(wh);
            *reinterpret_cast<uint2 *>(ea.wt_lo + o) = pack4(wl);
          }
          if (kDwOut) *reinterpret_cast<uint2 *>(ea.dw + o) = pack4(dw);
        }
        if (kStats) {
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
    }
  if (MODE == EPI_OBJ && !kStats) return;
  __syncthreads();
  if (bf_wstaged<BM, BN, MODE, DL>()) {
    // W' (or dW) of the active plans: each column's BM rows as 16-byte pieces,
    // in order (the column flags are read before the first store)
    constexpr int NW = (BN * (BM / 8) + NT - 1) / NT;
    static_assert(NW <= 32, "one flag bit per piece");
    uint32_t wact = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int e = tid + i * NT;
      if (e < BN * (BM / 8) && ea.active[n0 + e / (BM / 8)] != 0) wact |= 1u << i;
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int e = tid + i * NT;
      if (!((wact >> i) & 1u)) continue;
      const int cl = e / (BM / 8), ch = (e % (BM / 8)) * 8;
      const int n = n0 + cl;
      const size_t o = (size_t)n * ea.ldwt + m0 + ch;
      if (DL == BF_DELTA) {
        *reinterpret_cast<uint4 *>(ea.dw + o) = *reinterpret_cast<const uint4 *>(&swh[cl][ch]);
      } else {
        *reinterpret_cast<uint4 *>(ea.wt_hi + o) = *reinterpret_cast<const uint4 *>(&swh[cl][ch]);
        *reinterpret_cast<uint4 *>(ea.wt_lo + o) = *reinterpret_cast<const uint4 *>(&swl[cl][ch]);
      }
    }
  }
  if (!kStats) return;
  for (int e = tid; e < (BM / 32) * NST * BN; e += NT) {
    const int b = e / (NST * BN), q = (e / BN) % NST, c = e % BN;
    const double t0 = sred[2 * b][q][c], t1 = sred[2 * b + 1][q][c];
    const double v = (MODE == EPI_OBJ && q == 1) ? fmax(t0, t1) : t0 + t1;
    ea.stats[((size_t)(mt * (BM / 32) + b) * NST + q) * ea.nstat_cols + n0 + c] = v;
  }
}

// Both operands staged through LDS.  MODE 0: split-K partial store; otherwise
// the NN epilogue.  NBUF: 2 = double-buffered LDS stages; 1 = one stage (half
// the LDS, so more workgroups per CU), the next stage waiting in registers
// behind a barrier.
template <int BM, int BN, int WM, int WN, int TERMS, int MODE, int NBUF, int DL>
__global__ __launch_bounds__(64 * WM * WN, bf_min_waves(BM / (16 * WM), BN / (16 * WN))) void k_gemm_bf(
    BfPair A, BfPair B, int K, int kchunk,
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
  static_assert(TERMS == 1 || TERMS == 3, "one or three products per k step");
  constexpr bool ALO = TERMS == 3;   // A_lo B_hi and A_hi B_lo terms
  constexpr size_t kTileA = sizeof(uint16_t) * NBUF * BM * kBfLd;
  constexpr size_t kTileB = sizeof(uint16_t) * NBUF * BN * kBfLd;
  constexpr size_t kBytesT = kTileA * (ALO ? 2 : 1) + kTileB * (ALO ? 2 : 1);
  constexpr size_t kBytesR = bf_red_bytes<BM, BN, MODE, DL>();
  constexpr size_t kBytes = kBytesT > kBytesR ? kBytesT : kBytesR;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  auto sAh = reinterpret_cast<uint16_t (*)[BM][kBfLd]>(smem);
  auto sBh = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem + kTileA);
  auto sBl = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem + kTileA + kTileB);
  auto sAl = reinterpret_cast<uint16_t (*)[BM][kBfLd]>(smem + kTileA + 2 * kTileB);

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

  // A pieces: 64 consecutive threads take one fragment (1 KiB contiguous)
  static_assert(KV == 4, "one fragment per 16 rows and k step");
  auto a_row = [](int e) { return (e >> 6) * 16 + (e & 15); };
  auto a_kv = [](int e) { return ((e & 63) >> 4) * 8; };
  uint4 rah[AVT], ral[ALO ? AVT : 1], rbh[BVT], rbl[ALO ? BVT : 1];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        const int k = k0 + a_kv(e);
        const size_t off = frag_off(m0 + a_row(e), k, A.ld);
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
        if (ALO) rbl[i] = k < kend ? *reinterpret_cast<const uint4 *>(B.lo + off) : uint4{0, 0, 0, 0};
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < AVT; ++i) {
      const int e = tid + i * NT;
      if (e < AV) {
        *reinterpret_cast<uint4 *>(&sAh[buf][a_row(e)][a_kv(e)]) = rah[i];
        if (ALO) *reinterpret_cast<uint4 *>(&sAl[buf][a_row(e)][a_kv(e)]) = ral[i];
      }
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int row = e / KV, kv = (e % KV) * 8;
        *reinterpret_cast<uint4 *>(&sBh[buf][row][kv]) = rbh[i];
        if (ALO) *reinterpret_cast<uint4 *>(&sBl[buf][row][kv]) = rbl[i];
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
      bf8v ah[TM], al[ALO ? TM : 1], bh[TN], bl[ALO ? TN : 1];
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
        if (ALO) bl[tn] = *reinterpret_cast<const bf8v *>(&sBl[buf][row][g8]);
      }
      // term-major: TM TN independent products between two on one accumulator
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma_bf(ah[tm], bh[tn], acc[tm][tn]);
      if (ALO) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma_bf(ah[tm], bl[tn], acc[tm][tn]);
      }
      if (ALO) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma_bf(al[tm], bh[tn], acc[tm][tn]);
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
  bf_epilogue<BM, BN, WM, WN, MODE, DL>(acc, smem, tid, mt, m0, n0, zc, P, ldp, pstride, ea);
}

// Direct-A variant.  The waves split the rows only, so the rows of A a wave
// multiplies are its own: each lane loads its A fragments straight from global
// memory into registers in the MFMA operand layout; only B, which every wave
// reads, is staged through LDS (two stages).  Global loads of both operands are
// issued PD stages ahead into a register ring, so PD k-steps of MFMA work cover
// the latency of a load.  Per k-step and tile: the same three products in the
// same order as k_gemm_bf, so both kernels give the same bits.  LDS traffic per
// k-step and wave: 2 TN fragment reads for 3 TM TN MFMAs, against 2 (TM + TN)
// with A staged too.
//
// WN > 1: the waves form a WM x WN grid and also split the columns; a
// workgroup then spans up to all plan columns of a batch (the dose block is read
// once per product), the waves of a row share its A fragments (the second load
// of a fragment hits the cache) and each wave reads only its own TN column
// tiles of B from LDS.
template <int TM, int TN, int WM, int WN, int PD, int TERMS, int MODE, int DL>
__global__ __launch_bounds__(64 * WM * WN, bf_min_waves(TM, TN)) void k_gemm_bfd(
    BfPair A, BfPair B, int K, int kchunk,
                                                           int mtiles, int ntiles,
                                                           float *__restrict__ P, int ldp,
                                                           size_t pstride, EpiArgs<float> ea) {
  constexpr int BM = TM * 16 * WM, BN = TN * 16 * WN, NT = 64 * WM * WN;
  constexpr int KV = kBfBK / 8;
  constexpr int BV = BN * KV, BVT = (BV + NT - 1) / NT;
  static_assert(TERMS == 1 || TERMS == 3, "one or three products per k step");
  constexpr bool ALO = TERMS == 3;   // A_lo B_hi and A_hi B_lo terms
  constexpr int TA = ALO ? TM : 1;
  constexpr int BVL = ALO ? BVT : 1;
  static_assert(PD >= 1, "prefetch distance");
  static_assert(MODE == 0 || (TM * 16) % 32 == 0, "statistics partials are per 32-row block");
  constexpr size_t kTileB = sizeof(uint16_t) * 2 * BN * kBfLd;
  constexpr size_t kBytesT = (ALO ? 2 : 1) * kTileB;
  constexpr size_t kBytesR = bf_red_bytes<BM, BN, MODE, DL>();
  constexpr size_t kBytes = kBytesT > kBytesR ? kBytesT : kBytesR;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  auto sBh = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem);
  auto sBl = reinterpret_cast<uint16_t (*)[BN][kBfLd]>(smem + kTileB);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int tile = xcd_tile_bf(blockIdx.x, gridDim.x);
  const int nt = tile % ntiles, mt = (tile / ntiles) % mtiles, zc = tile / (mtiles * ntiles);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = MODE == 0 ? zc * kchunk : 0;
  const int kend = MODE == 0 ? min(K, kbeg + kchunk) : K;
  const int g8 = 8 * (lane >> 4), r16 = lane & 15;
  const int bcol = wn * TN * 16;   // this wave's first column in the workgroup's B tile

  f4v acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};

  // register ring: slot 0 holds the stage being multiplied, slot p the stage p
  // ahead.  A fragment of 16-row tile t at k step k0 / 32: 1 KiB at
  // frag_off(16 t, k0, K); this lane's piece is 8 lane elements further.
  const size_t arow = frag_off(m0 + wm * TM * 16, 0, A.ld) + (size_t)lane * 8;
  const size_t astep = (size_t)(A.ld >> 5) * 512;   // next 16-row tile
  uint4 ah[PD + 1][TM], al[PD + 1][TA], rbh[PD + 1][BVT], rbl[PD + 1][BVL];
  auto load = [&](int k0, int slot) {
    const bool in = k0 + g8 < kend;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm) {
      const size_t off = arow + tm * astep + (size_t)(k0 >> 5) * 512;
      ah[slot][tm] = in ? *reinterpret_cast<const uint4 *>(A.hi + off) : uint4{0, 0, 0, 0};
      if (ALO) al[slot][tm] = in ? *reinterpret_cast<const uint4 *>(A.lo + off) : uint4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int row = e / KV, k = k0 + (e % KV) * 8;
        const size_t off = (size_t)(n0 + row) * B.ld + k;
        rbh[slot][i] = k < kend ? *reinterpret_cast<const uint4 *>(B.hi + off) : uint4{0, 0, 0, 0};
        if (ALO) rbl[slot][i] = k < kend ? *reinterpret_cast<const uint4 *>(B.lo + off) : uint4{0, 0, 0, 0};
      }
    }
  };
  auto store_b = [&](int slot, int buf) {
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int e = tid + i * NT;
      if (e < BV) {
        const int row = e / KV, kv = (e % KV) * 8;
        *reinterpret_cast<uint4 *>(&sBh[buf][row][kv]) = rbh[slot][i];
        if (ALO) *reinterpret_cast<uint4 *>(&sBl[buf][row][kv]) = rbl[slot][i];
      }
    }
  };

  if (kbeg < kend) {
#pragma unroll
    for (int p = 0; p < PD; ++p)
      if (kbeg + p * kBfBK < kend) load(kbeg + p * kBfBK, p);
    store_b(0, 0);
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += kBfBK) {
      if (k0 + PD * kBfBK < kend) load(k0 + PD * kBfBK, PD);
      bf8v bh[TN], bl[ALO ? TN : 1];
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        bh[tn] = *reinterpret_cast<const bf8v *>(&sBh[buf][bcol + tn * 16 + r16][g8]);
        if (ALO) bl[tn] = *reinterpret_cast<const bf8v *>(&sBl[buf][bcol + tn * 16 + r16][g8]);
      }
      // term-major: TM TN independent products between two on one accumulator
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma_bf(as_bf8(ah[0][tm]), bh[tn], acc[tm][tn]);
      if (ALO) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = mfma_bf(as_bf8(ah[0][tm]), bl[ALO ? tn : 0], acc[tm][tn]);
      }
      if (ALO) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn)
            acc[tm][tn] = mfma_bf(as_bf8(al[0][ALO ? tm : 0]), bh[tn], acc[tm][tn]);
      }
      const bool more = k0 + kBfBK < kend;
      if (more) store_b(1, buf ^ 1);
      __syncthreads();
      buf ^= 1;
#pragma unroll
      for (int p = 0; p < PD; ++p) {
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) ah[p][tm] = ah[p + 1][tm];
#pragma unroll
        for (int tm = 0; tm < TA; ++tm) al[p][tm] = al[p + 1][tm];
#pragma unroll
        for (int i = 0; i < BVT; ++i) rbh[p][i] = rbh[p + 1][i];
#pragma unroll
        for (int i = 0; i < BVL; ++i) rbl[p][i] = rbl[p + 1][i];
      }
    }
  }
  bf_epilogue<BM, BN, WM, WN, MODE, DL>(acc, smem, tid, mt, m0, n0, zc, P, ldp, pstride, ea);
}

// Single-operand products (terms = 1, LADMM_BF16's hot iterations).  With one
// MFMA per accumulator and k step, a step's MFMA work (TM TN per wave) is a
// third of the pair products', far too short to hide a fetch from HBM behind
// one step of prefetch.  Here both operands run RING stages ahead in register
// rings: the A fragments (the dose block, read once per product) straight from
// global memory, and B (the small plan-side operand, served by L2) on its way
// to one of two LDS stages.  A stage is KS MFMA k steps (one barrier per
// stage).  Vector loads retire in issue order, so a wait for one load is a
// wait for every older one: the rings are indexed by stage modulo RING with the
// loop unrolled RING times (no register copies that would wait for a load in
// flight), and every load in the unrolled body is issued unconditionally
// (addresses past the last k step are clamped to it and the data is never
// used), so that the compiler's waits name exact counts and about RING - 1
// stages of loads stay in flight.  The last stage may hold fewer than KS k
// steps; its MFMAs past the end are skipped.  Per stage: the B load of stage
// t + RING goes out first, then the MFMAs of stage t, then the A load of stage
// t + RING into the slot just used, and the LDS store of B for stage t + 1.
// The waves form a WM x WN grid (a workgroup spans up to all plan columns).
// Every accumulator takes one MFMA per k step in k order, as in the other
// kernels, so the results are the same bits.  OCC: waves per SIMD the
// registers must allow.  (kend - kbeg) % 32 == 0.
template <int TM, int TN, int WM, int WN, int OCC, int RING, int KS, int MODE, int DL>
__global__ __launch_bounds__(64 * WM * WN, OCC) void k_gemm_b1(BfPair A, BfPair B, int K, int kchunk,
                                                               int mtiles, int ntiles,
                                                               float *__restrict__ P, int ldp,
                                                               size_t pstride, EpiArgs<float> ea) {
  constexpr int BM = TM * 16 * WM, BN = TN * 16 * WN, NT = 64 * WM * WN;
  constexpr int KV = kBfBK / 8;              // 16-byte pieces per row of one k step
  constexpr int BV = BN * KV * KS, BVT = (BV + NT - 1) / NT;
  static_assert(RING >= 2 && RING % 2 == 0, "the LDS stage of stage t is t % 2 = (t % RING) % 2");
  static_assert(MODE == 0 || (TM * 16) % 32 == 0, "statistics partials are per 32-row block");
  constexpr int kSub = BN * kBfLd;           // uint16 per k step of a stage
  constexpr int kStage = KS * kSub;
  constexpr size_t kTileB = sizeof(uint16_t) * 2 * kStage;
  constexpr size_t kBytesR = bf_red_bytes<BM, BN, MODE, DL>();
  constexpr size_t kBytes = kTileB > kBytesR ? kTileB : kBytesR;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kBytes];
  uint16_t *const sB = reinterpret_cast<uint16_t *>(smem);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int tile = xcd_tile_bf(blockIdx.x, gridDim.x);
  const int nt = tile % ntiles, mt = (tile / ntiles) % mtiles, zc = tile / (mtiles * ntiles);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = MODE == 0 ? zc * kchunk : 0;
  const int kend = MODE == 0 ? min(K, kbeg + kchunk) : K;
  const int nsub = kend > kbeg ? (kend - kbeg) / kBfBK : 0;   // k steps
  const int nfull = nsub / KS, nst = (nsub + KS - 1) / KS;     // full and all stages
  const int g8 = 8 * (lane >> 4), r16 = lane & 15;
  const int bread = (wn * TN * 16 + r16) * kBfLd + g8;   // this wave's B fragments in a k step

  f4v acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};

  // this lane's piece of the first A fragment of the chunk; per B slot (slots
  // past BV load slot BV - 1 again and are not stored) its global address at
  // the chunk's first stage and its place in a stage
  const uint16_t *abase = A.hi + frag_off(m0 + wm * TM * 16, kbeg, A.ld) + (size_t)lane * 8;
  const size_t astep = (size_t)(A.ld >> 5) * 512;   // next 16-row tile
  const uint16_t *bbase[BVT];
  int bput[BVT], bks[BVT];
#pragma unroll
  for (int i = 0; i < BVT; ++i) {
    const int e = min(tid + i * NT, BV - 1);
    const int ks = e / (BN * KV), r = e % (BN * KV);
    const int n = r / KV, c = r % KV;
    bbase[i] = B.hi + (size_t)(n0 + n) * B.ld + kbeg + ks * kBfBK + c * 8;
    bput[i] = ks * kSub + n * kBfLd + c * 8;
    bks[i] = ks;
  }
  u4v ah[RING][KS][TM], rb[RING][BVT];
  auto load_a = [&](int t, u4v (&dst)[KS][TM]) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const size_t ko = (size_t)min(t * KS + ks, nsub - 1) * 512;
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) dst[ks][tm] = *reinterpret_cast<const u4v *>(abase + tm * astep + ko);
    }
  };
  // B slot i belongs to k step bks[i] of a stage (bbase[i] includes its offset)
  auto load_b = [&](int t, u4v (&dst)[BVT]) {
#pragma unroll
    for (int i = 0; i < BVT; ++i) {
      const int ko = (min(t * KS + bks[i], nsub - 1) - bks[i]) * kBfBK;
      dst[i] = *reinterpret_cast<const u4v *>(bbase[i] + ko);
    }
  };
  auto store_b = [&](const u4v (&src)[BVT], int stage) {
#pragma unroll
    for (int i = 0; i < BVT; ++i)
      if (BV % NT == 0 || tid + i * NT < BV)
        *reinterpret_cast<u4v *>(sB + stage * kStage + bput[i]) = src[i];
  };
  // nk: k steps of the stage to multiply (KS, or fewer in a last partial stage)
  auto mma = [&](const u4v (&a)[KS][TM], int stage, int nk) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks >= nk) break;
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const bf8v b = *reinterpret_cast<const bf8v *>(sB + stage * kStage + ks * kSub + bread +
                                                       tn * 16 * kBfLd);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) acc[tm][tn] = mfma_bf(as_bf8(a[ks][tm]), b, acc[tm][tn]);
      }
    }
  };

  if (nsub > 0) {
#pragma unroll
    for (int p = 0; p < RING; ++p) {
      load_b(p, rb[p]);
      load_a(p, ah[p]);
    }
    store_b(rb[0], 0);
    __syncthreads();
    int t0 = 0;
    for (; t0 + RING <= nfull; t0 += RING) {
#pragma unroll
      for (int i = 0; i < RING; ++i) {
        const int t = t0 + i;
        load_b(t + RING, rb[i]);            // B of stage t left rb[i] for LDS at stage t - 1
        mma(ah[i], i & 1, KS);
        load_a(t + RING, ah[i]);
        store_b(rb[(i + 1) % RING], (i + 1) & 1);   // past the last stage: never read
        __syncthreads();
      }
    }
    // the last stages (fewer than RING full ones, then a partial one): their
    // operands are already loaded
#pragma unroll
    for (int i = 0; i < RING; ++i) {
      if (t0 + i < nst) {
        mma(ah[i], i & 1, min(KS, nsub - (t0 + i) * KS));
        store_b(rb[(i + 1) % RING], (i + 1) & 1);
        __syncthreads();
      }
    }
  }
  bf_epilogue<BM, BN, WM, WN, MODE, DL>(acc, smem, tid, mt, m0, n0, zc, P, ldp, pstride, ea);
}

// Tile configurations of the split-K product (which = 0) and the point-row
// product (1): rows BM x columns BN of a workgroup, staged (both operands
// through LDS, k_gemm_bf) or direct (A from global memory, k_gemm_bfd).
// Configuration 0 is valid for every padded shape (M % 64, N % 32).
// Configurations 6 to 9 are for single-operand products only (terms = 1,
// K % 32 == 0), on k_gemm_b1: 4 waves of 48 (split-K) or 32 (point-row) rows
// by 64, 112 and 96 columns, so that every launch width of a compacted run (a
// multiple of 64, 96 or 224) has one, and 8 waves of 32 x 112 (split-K) or
// 32 x 224 (point-row) that cover all 448 plan columns of a 441-plan batch.
// Ring depth and k steps per stage (BF_DW's last two arguments) as measured
// fastest on the large case: two stages of two k steps, four k steps in the
// 64-column point-row tile, and four stages of one in the 448-column tiles.
constexpr int kBfCfgCount = 10;
struct BfCfg { int bm, bn; bool single_only; };
static const BfCfg kBfCfgs[2][kBfCfgCount] = {
    {{64, 32, false}, {64, 64, false}, {192, 112, false}, {160, 112, false}, {64, 96, false},
     {192, 64, false}, {192, 64, true}, {192, 112, true}, {192, 96, true}, {64, 448, true}},
    {{64, 32, false}, {256, 64, false}, {128, 112, false}, {128, 112, false}, {128, 96, false},
     {128, 64, false}, {128, 64, true}, {128, 112, true}, {128, 96, true}, {128, 448, true}}};

bool gemm_bf_cfg_ok(int which, int cfg, int M, int N, int terms) {
  if (cfg < 0 || cfg >= kBfCfgCount) return false;
  const BfCfg c = kBfCfgs[which][cfg];
  if (c.single_only && terms != 1) return false;
  return M % c.bm == 0 && N % c.bn == 0;
}

template <int MODE, int TERMS, int DL>
static hipError_t launch_bf(int cfg, int M, int N, int nchunk, hipStream_t s, BfPair A, BfPair B,
                            int K, int kchunk, float *P, int ldp, size_t pstride,
                            const EpiArgs<float> &ea) {
  const BfCfg c = kBfCfgs[MODE == 0 ? 0 : 1][cfg];
  const int mtiles = M / c.bm, ntiles = N / c.bn;
  const dim3 grid(mtiles * ntiles * nchunk);
#define BF_ST(BMv, BNv, WMv, WNv, NB)                                                              \
  hipLaunchKernelGGL((k_gemm_bf<BMv, BNv, WMv, WNv, TERMS, MODE, NB, DL>), grid, dim3(64 * WMv * WNv), 0, \
                     s, A, B, K, kchunk, mtiles, ntiles, P, ldp, pstride, ea)
#define BF_DI(TMv, TNv, WMv)                                                                       \
  hipLaunchKernelGGL((k_gemm_bfd<TMv, TNv, WMv, 1, 1, TERMS, MODE, DL>), grid, dim3(64 * WMv), 0, s, A, B, \
                     K, kchunk, mtiles, ntiles, P, ldp, pstride, ea)
#define BF_DW(TMv, TNv, WMv, WNv, OCCv, RINGv, KSv)                                                \
  hipLaunchKernelGGL((k_gemm_b1<TMv, TNv, WMv, WNv, OCCv, RINGv, KSv, MODE, DL>), grid,                  \
                     dim3(64 * WMv * WNv), 0, s, A, B, K, kchunk, mtiles, ntiles, P, ldp, pstride, ea)
  if constexpr (MODE == 0) {
    switch (cfg) {
      case 0: BF_ST(64, 32, 2, 1, 2); break;
      case 1: BF_ST(64, 64, 2, 1, 1); break;
      case 2: BF_DI(3, 7, 4); break;
      case 3: BF_DI(5, 7, 2); break;
      case 4: BF_DI(1, 6, 4); break;
      case 5: BF_DI(3, 4, 4); break;
      case 6:
        if constexpr (TERMS == 1) { BF_DW(3, 4, 4, 1, 3, 2, 2); } else { return hipErrorInvalidValue; }
        break;
      case 7:
        if constexpr (TERMS == 1) { BF_DW(3, 7, 4, 1, 2, 2, 2); } else { return hipErrorInvalidValue; }
        break;
      case 8:
        if constexpr (TERMS == 1) { BF_DW(3, 6, 4, 1, 2, 2, 2); } else { return hipErrorInvalidValue; }
        break;
      case 9:
        if constexpr (TERMS == 1) { BF_DW(2, 7, 2, 4, 2, 4, 1); } else { return hipErrorInvalidValue; }
        break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (cfg) {
      case 0: BF_ST(64, 32, 2, 1, 2); break;
      case 1: BF_ST(256, 64, 4, 1, 1); break;
      case 2: BF_DI(2, 7, 4); break;
      case 3: BF_DI(4, 7, 2); break;
      case 4: BF_DI(2, 6, 4); break;
      case 5: BF_DI(2, 4, 4); break;
      case 6:
        if constexpr (TERMS == 1) { BF_DW(2, 4, 4, 1, 3, 2, 4); } else { return hipErrorInvalidValue; }
        break;
      case 7:
        if constexpr (TERMS == 1) { BF_DW(2, 7, 4, 1, 2, 2, 2); } else { return hipErrorInvalidValue; }
        break;
      case 8:
        if constexpr (TERMS == 1) { BF_DW(2, 6, 4, 1, 2, 2, 2); } else { return hipErrorInvalidValue; }
        break;
      case 9:
        if constexpr (TERMS == 1) { BF_DW(2, 14, 4, 2, 2, 4, 1); } else { return hipErrorInvalidValue; }
        break;
      default: return hipErrorInvalidValue;
    }
  }
#undef BF_ST
#undef BF_DI
#undef BF_DW
  return hipGetLastError();
}

hipError_t gemm_bf_tn(hipStream_t s, BfPair A, BfPair B, float *P, int ldp, int M, int N, int K,
                      int nchunk, int terms, int cfg) {
  if (!gemm_bf_cfg_ok(0, cfg, M, N, terms) || (kBfCfgs[0][cfg].single_only && K % kBfBK)) cfg = 0;
  if (!gemm_bf_cfg_ok(0, cfg, M, N, terms) || nchunk < 1 || K % 8 || A.ld % 8 || B.ld % 8)
    return hipErrorInvalidValue;
  int kchunk = (K + nchunk - 1) / nchunk;
  kchunk = (kchunk + 31) / 32 * 32;
  const EpiArgs<float> ea{};
  const size_t pstride = (size_t)M * ldp;
  if (terms == 3) return launch_bf<0, 3, BF_PLAIN>(cfg, M, N, nchunk, s, A, B, K, kchunk, P, ldp, pstride, ea);
  if (terms == 1) return launch_bf<0, 1, BF_PLAIN>(cfg, M, N, nchunk, s, A, B, K, kchunk, P, ldp, pstride, ea);
  return hipErrorInvalidValue;
}

hipError_t gemm_bf_nn(hipStream_t s, int epi, BfPair A, BfPair B, int M, int N, int K,
                      const EpiArgs<float> &ea, int terms, int cfg, int delta) {
  if (!gemm_bf_cfg_ok(1, cfg, M, N, terms)) cfg = 0;
  if (!gemm_bf_cfg_ok(1, cfg, M, N, terms) || K % kBfBK || A.ld % 8 || B.ld % 8) return hipErrorInvalidValue;
  // the combinations the iteration uses: pairs (three terms) for BF16X3, the
  // objective and the refresh; single operands for the hot iterations
#define BF_EPI(E, T, D) return launch_bf<E, T, D>(cfg, M, N, 1, s, A, B, K, K, nullptr, 0, 0, ea)
  if (terms == 3 && delta == BF_PLAIN) {
    if (epi == EPI_ADMM) BF_EPI(EPI_ADMM, 3, BF_PLAIN);
    if (epi == EPI_ADMM_STATS) BF_EPI(EPI_ADMM_STATS, 3, BF_PLAIN);
    if (epi == EPI_OBJ) BF_EPI(EPI_OBJ, 3, BF_PLAIN);
  }
  if (terms == 3 && delta == BF_REFRESH && epi == EPI_ADMM_STATS) BF_EPI(EPI_ADMM_STATS, 3, BF_REFRESH);
  if (terms == 1 && delta == BF_DELTA && epi == EPI_ADMM) BF_EPI(EPI_ADMM, 1, BF_DELTA);
  if (terms == 1 && delta == BF_DELTA_PAIR && epi == EPI_ADMM) BF_EPI(EPI_ADMM, 1, BF_DELTA_PAIR);
#undef BF_EPI
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// operand preparation
// ---------------------------------------------------------------------------
// D^ = Dt diag(E) as pairs in fragment order, for both products at once: a
// workgroup converts a 64-point x 64-shot tile in LDS and writes the 8
// fragments it holds of the point-major block (16-point tiles x 32-shot steps,
// the point-row product's operand) and the 8 of the shot-major block (16-shot
// tiles x 32-point steps, the split-K product's operand), 1 KiB each,
// coalesced.  Np % 64 == 0 and ntp % 64 == 0.
__global__ __launch_bounds__(256) void k_split_dose_frag(const double *__restrict__ Dt,
                                                         const double *__restrict__ E, int Np,
                                                         int ntp, uint16_t *__restrict__ Dh,
                                                         uint16_t *__restrict__ Dl,
                                                         uint16_t *__restrict__ DTh,
                                                         uint16_t *__restrict__ DTl) {
  __shared__ uint16_t sh[64][66], sl[64][66];   // [point][shot]
  const int t0 = blockIdx.x * 64, p0 = blockIdx.y * 64, tid = threadIdx.x;
  for (int i = tid; i < 64 * 64; i += 256) {
    const int pp = i >> 6, tt = i & 63;
    uint16_t h, l;
    split_pair(Dt[(size_t)(p0 + pp) * ntp + t0 + tt] * E[t0 + tt], h, l);
    sh[pp][tt] = h;
    sl[pp][tt] = l;
  }
  __syncthreads();
  // 8 fragments x 64 lanes per block; lane L of a fragment: row L % 16, k 8 (L / 16) + e
  for (int piece = tid; piece < 8 * 64; piece += 256) {
    const int f = piece >> 6, L = piece & 63, r = L & 15, k8 = (L >> 4) * 8;
    {  // point-major: rows = points, k = shots
      const int pt = f >> 1, ts = f & 1;
      const int pp = pt * 16 + r, tt = ts * 32 + k8;
      uint16_t vh[8], vl[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        vh[e] = sh[pp][tt + e];
        vl[e] = sl[pp][tt + e];
      }
      const size_t o = frag_off(p0 + pp, t0 + tt, ntp);
      *reinterpret_cast<uint4 *>(Dh + o) = *reinterpret_cast<const uint4 *>(vh);
      *reinterpret_cast<uint4 *>(Dl + o) = *reinterpret_cast<const uint4 *>(vl);
    }
    {  // shot-major: rows = shots, k = points
      const int tt0 = f >> 1, ps = f & 1;
      const int tt = tt0 * 16 + r, pp = ps * 32 + k8;
      uint16_t vh[8], vl[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        vh[e] = sh[pp + e][tt];
        vl[e] = sl[pp + e][tt];
      }
      const size_t o = frag_off(t0 + tt, p0 + pp, Np);
      *reinterpret_cast<uint4 *>(DTh + o) = *reinterpret_cast<const uint4 *>(vh);
      *reinterpret_cast<uint4 *>(DTl + o) = *reinterpret_cast<const uint4 *>(vl);
    }
  }
}

hipError_t split_dose_bf16(hipStream_t s, const double *Dt, const double *E, int Np, int ntp,
                           uint16_t *Dh, uint16_t *Dl, uint16_t *DTh, uint16_t *DTl) {
  if (Np % 64 || ntp % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_split_dose_frag, dim3(ntp / 64, Np / 64), dim3(256), 0, s, Dt, E, Np, ntp, Dh,
                     Dl, DTh, DTl);
  return hipGetLastError();
}

// v = sum of the S^-1 r partials; v_top as plan-major pairs (kp x ntp), and
// with vref (a refresh of LADMM_BF16) the value the pairs carry.
__global__ void k_vreduce_bf(SmallArgs a, const double *__restrict__ P2, size_t zstride, int nchunk,
                             double *__restrict__ v, uint16_t *__restrict__ vh,
                             uint16_t *__restrict__ vl, double *__restrict__ vref,
                             double *__restrict__ vout) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.mAp || j >= a.kp) return;
  const size_t idx = (size_t)m * a.kp + j;
  double acc = 0.0;
#pragma unroll 8
  for (int z = 0; z < nchunk; ++z) acc += P2[z * zstride + idx];
  v[idx] = acc;
  if (vout != nullptr && a.active[j]) vout[idx] = acc;
  if (m < a.L.ntp) {
    uint16_t h, l;
    split_pair(acc, h, l);
    vh[(size_t)j * a.L.ntp + m] = h;
    vl[(size_t)j * a.L.ntp + m] = l;
    if (vref != nullptr && a.active[j]) vref[idx] = (double)pair_val(h, l);
  }
}

hipError_t vreduce_bf(hipStream_t s, const SmallArgs &a, const double *P2, size_t zstride, int nchunk,
                      double *v, uint16_t *vh, uint16_t *vl, double *vref, double *vout) {
  hipLaunchKernelGGL(k_vreduce_bf, dim3((a.L.mAp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0, s, a,
                     P2, zstride, nchunk, v, vh, vl, vref, vout);
  return hipGetLastError();
}

// v = vbase + the sum of the FP32 partials of S^-1 (r - r_ref); dv = bf16(v_top -
// vref) plan-major (kp x ntp).
__global__ void k_vreduce_delta_bf(SmallArgs a, const float *__restrict__ P2, size_t zstride,
                                   int nchunk, const double *__restrict__ vbase,
                                   double *__restrict__ v, const double *__restrict__ vref,
                                   uint16_t *__restrict__ dv) {
  const int j = blockIdx.y * 64 + threadIdx.x;
  const int m = blockIdx.x * 4 + threadIdx.y;
  if (m >= a.L.mAp || j >= a.kp) return;
  const size_t idx = (size_t)m * a.kp + j;
  double acc = 0.0;
#pragma unroll 8
  for (int z = 0; z < nchunk; ++z) acc += (double)P2[z * zstride + idx];
  acc += vbase[idx];
  v[idx] = acc;
  if (m < a.L.ntp) dv[(size_t)j * a.L.ntp + m] = bf_round((float)(acc - vref[idx]));
}

hipError_t vreduce_delta_bf(hipStream_t s, const SmallArgs &a, const float *P2, size_t zstride,
                            int nchunk, const double *vbase, double *v, const double *vref,
                            uint16_t *dv) {
  hipLaunchKernelGGL(k_vreduce_delta_bf, dim3((a.L.mAp + 3) / 4, (a.kp + 63) / 64), dim3(64, 4), 0,
                     s, a, P2, zstride, nchunk, vbase, v, vref, dv);
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

// Point-major FP32 values of q -> plan-major BF16 rows, through a 64 x 64 LDS
// tile so that both the reads (plans contiguous) and the writes (points
// contiguous) are coalesced.  KIND 0: z1 = clip(q, 0, u) as pairs; KIND 1:
// W = 2 clip(q, 0, u) - q as pairs and, with dw, dW = bf16(W - W_ref).
template <int KIND>
__global__ __launch_bounds__(256) void k_plan_major_bf(const float *__restrict__ q, int Np, int kp,
                                                       PointTable<float> pt,
                                                       uint16_t *__restrict__ hi,
                                                       uint16_t *__restrict__ lo,
                                                       const float *__restrict__ wref,
                                                       uint16_t *__restrict__ dw) {
  __shared__ uint16_t sh[64][66], sl[64][66], sd[64][66];   // [plan][point]
  const int p0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int pp = i >> 6, jj = i & 63;
    const int p = p0 + pp, j = j0 + jj;
    uint16_t h = 0, l = 0, d = 0;
    if (p < Np && j < kp) {
      const size_t e = (size_t)p * kp + j;
      const float qv = q[e];
      const float z = clip0u_f(qv, upper_bf(pt, pt.grp[p], p, j));
      const float v = KIND == 0 ? z : 2.f * z - qv;
      split_pair((double)v, h, l);
      if (KIND == 1 && dw != nullptr) d = bf_round(v - wref[e]);
    }
    sh[jj][pp] = h;
    sl[jj][pp] = l;
    sd[jj][pp] = d;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int jj = i >> 6, pp = i & 63;
    const int p = p0 + pp, j = j0 + jj;
    if (p < Np && j < kp) {
      const size_t o = (size_t)j * Np + p;
      hi[o] = sh[jj][pp];
      lo[o] = sl[jj][pp];
      if (KIND == 1 && dw != nullptr) dw[o] = sd[jj][pp];
    }
  }
}

hipError_t w_from_q_bf(hipStream_t s, const float *q, int Np, int kp, const PointTable<float> &pt,
                       uint16_t *wh, uint16_t *wl, const float *wref, uint16_t *dw) {
  hipLaunchKernelGGL(k_plan_major_bf<1>, dim3((Np + 63) / 64, (kp + 63) / 64), dim3(256), 0, s, q, Np,
                     kp, pt, wh, wl, wref, dw);
  return hipGetLastError();
}

// z1 = clip(q, 0, u) as plan-major pairs: the certificate's product operand.
hipError_t z_from_q_bf(hipStream_t s, const float *q, int Np, int kp, const PointTable<float> &pt,
                       uint16_t *zh, uint16_t *zl) {
  hipLaunchKernelGGL(k_plan_major_bf<0>, dim3((Np + 63) / 64, (kp + 63) / 64), dim3(256), 0, s, q, Np,
                     kp, pt, zh, zl, nullptr, nullptr);
  return hipGetLastError();
}

// W' rows of warm-started plans as pairs, from their loaded q columns (and
// dW = bf16(W' - W_ref) with wref, dw: LADMM_BF16).
__global__ void k_warm_w_bf(WarmCols w, const float *__restrict__ q, int Np, int kp,
                            PointTable<float> pt, uint16_t *__restrict__ wh,
                            uint16_t *__restrict__ wl, const float *__restrict__ wref,
                            uint16_t *__restrict__ dw) {
  const int i = blockIdx.y;
  if (i >= w.n) return;
  const int j = w.col[i];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Np) return;
  const float qv = q[(size_t)p * kp + j];
  const float wv = 2.f * clip0u_f(qv, upper_bf(pt, pt.grp[p], p, j)) - qv;
  uint16_t h, l;
  split_pair((double)wv, h, l);
  wh[(size_t)j * Np + p] = h;
  wl[(size_t)j * Np + p] = l;
  if (dw != nullptr) dw[(size_t)j * Np + p] = bf_round(wv - wref[(size_t)p * kp + j]);
}

hipError_t warm_w_bf(hipStream_t s, const WarmCols &w, const float *q, uint16_t *wh, uint16_t *wl,
                     int Np, int kp, const PointTable<float> &pt, const float *wref, uint16_t *dw) {
  if (w.n <= 0) return hipSuccess;
  if (w.n > kWarmCols) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_warm_w_bf, dim3((unsigned)((Np + 255) / 256), (unsigned)w.n), dim3(256), 0, s,
                     w, q, Np, kp, pt, wh, wl, wref, dw);
  return hipGetLastError();
}

// Zero the rows j of plan-major BF16 arrays (halves x kp rows of len: hi then
// lo rows of pairs, or one single array) whose flag[j] is nonzero: a fresh
// plan in a reused column.
__global__ void k_zero_plan_rows(uint16_t *__restrict__ a, int kp, int len, int halves,
                                 const int32_t *__restrict__ flag) {
  const size_t total = (size_t)halves * kp * len;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    if (flag[(e / len) % kp]) a[e] = 0;
}

hipError_t zero_plan_rows_bf(hipStream_t s, uint16_t *a, int kp, int len, const int32_t *flag,
                             int halves) {
  hipLaunchKernelGGL(k_zero_plan_rows, dim3(2048), dim3(256), 0, s, a, kp, len, halves, flag);
  return hipGetLastError();
}

}  // namespace ladmm
