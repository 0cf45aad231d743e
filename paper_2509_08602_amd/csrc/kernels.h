// Internal launchers of the HIP kernels (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace ladmm {

// Tile sizes shared by the launchers and the host-side padding rules.
constexpr int kTileRows = 256;    // dose-point padding: a multiple of every row tile
constexpr int kSmallAlign = 64;   // padding of the shot / small-row dimension

// Layout of the small (m_A) vectors: shot rows t in [0, ntp) (t < n_t real),
// BOT rows at ntp + i (i < n_iso), zero padding up to mAp.
struct SmallLayout {
  int n_t, ntp, n_iso, mAp, n_sec, S, C;
};

// Per-point description used by the prologue / epilogues.
template <typename T>
struct PointTable {
  const int32_t *grp;     // Np: group id (G = padding group)
  const T *sig;           // Np: +1 target, -1 other, 0 padding
  const int32_t *is_ld;   // per group: 1 if low-dose group
  const int32_t *is_oar;  // per group: 1 if OAR group
  const T *utab;          // (G+1) x ldu: u of (group, plan); +inf for OAR
  int ldu;
  const uint64_t *mask;   // NULL or kp rows x mask_words: low-dose membership
  int mask_words;
};

// ---- generic products -----------------------------------------------------
// P[z][m][n] = sum over rows k of chunk z of A[k][m] * B[k][n]   (A: K x M, B: K x N)
// With the ADMM prologue, B is replaced by W = 2 clip(q, 0, u) - q.
// Tile configuration cfg in [0, kGemmCfgs) (0 is valid for every padded shape;
// an invalid cfg falls back to 0).  The configurations do not change the
// order of the floating-point sums, only the work split.
constexpr int kGemmCfgs = 4;
bool gemm_tn_cfg_ok(int cfg, int M, int N);
bool gemm_nn_cfg_ok(int cfg, int M, int N);
// The statistics epilogues of the point-row product write one partial per
// 32-row block (M / 32 of them) whatever the configuration, summed in a fixed
// order, so the statistics do not depend on the configuration either.
constexpr int kNnStatRows = 32;
template <typename T>
hipError_t gemm_tn(hipStream_t s, const T *A, int lda, const T *B, int ldb, T *P, int ldp,
                   int M, int N, int K, int nchunk, const PointTable<T> *pro, int cfg = 0);
// P[z][m][n] for FP64 accumulation of FP64 operands is the T = double case.

// Epilogues of C = A B (A: M x K row-major, B: K x N row-major).
enum { EPI_STORE = 0, EPI_ADMM = 1, EPI_ADMM_STATS = 2, EPI_OBJ = 3 };
constexpr int kAdmmStats = 6;   // (x-z)^2, x^2, z^2, (z-zprev)^2, y^2, c'z
constexpr int kObjStats = 3;    // hinge sum, OAR dose ratio max, sum of u d / D over targets
template <typename T>
struct EpiArgs {
  T *C; int ldc;                   // EPI_STORE output
  T *q; int ldq;                   // EPI_ADMM: iterate q (in place)
  T *w;                            // EPI_ADMM: W = z1 - y1 of the new iterate (ld = ldq)
  const double *invrho;            // per plan 1/rho
  const int32_t *active;           // per plan
  double *stats; int nstat_cols;   // partial stats [blockIdx.x][stat][nstat_cols]
  PointTable<T> pt;
  uint16_t *wt_hi, *wt_lo; int ldwt;   // BF16-pair products: W' = z1' - y1' as plans x points
  double alpha;                    // over-relaxation of the z- and y-steps (1: none)
  // BF16 refinement (LADMM_BF16): the exact products at the last refresh,
  // X_ref = D^ v_ref and W_ref (points x plans, ld = ldq), and the change
  // dW = bf16(W' - W_ref) written plan-major (ld = ldwt) for the next GEMM1.
  float *xref, *wref;
  uint16_t *dw;
};
template <typename T>
hipError_t gemm_nn(hipStream_t s, int epi, const T *A, int lda, const T *B, int ldb,
                   int M, int N, int K, const EpiArgs<T> &ea, int cfg = 0);

// ---- setup ------------------------------------------------------------------
// Dt[p][t] = sig[p] * phi[p][t] / thr[p]; zero padding rows/cols (FP64).
// The smallest index of a negative or non-finite dose entry into *first (set
// to UINT64_MAX by the caller).
hipError_t check_dose(hipStream_t s, const double *phi, size_t n, unsigned long long *first);
hipError_t scale_dose(hipStream_t s, const double *phi, int N, int n_t, const double *sig,
                      const double *inv_thr, double *Dt, int Np, int ntp);
// out[p][t] = (T)(Dt[p][t] * E[t])
template <typename T>
hipError_t scale_columns(hipStream_t s, const double *Dt, const double *E, T *out, int Np, int ntp);
// sum of nchunk partials [z][rows][cols] (ld) -> out (double)
template <typename T>
hipError_t reduce_partials(hipStream_t s, const T *P, size_t zstride, int nchunk, int rows, int cols,
                           int ld, double *out, int ldo);
// E and S from K = Dt' Dt (ntp x ntp); S is mAp x mAp.
hipError_t assemble_schur(hipStream_t s, const double *K, int ldk, const SmallLayout &L,
                          double cs, double beta, double e_bot, int row_normalize,
                          double *E, double *S);
// Blocked Cholesky S = L L' in place (lower), n x n, ld; info set to 1 on failure.
hipError_t cholesky(hipStream_t s, double *S, int n, int ld, int *dinfo);
// X = L^-1 (lower triangular), n x n.
hipError_t tri_inverse(hipStream_t s, const double *L, double *X, int n, int ld);

// ---- per iteration ----------------------------------------------------------
struct SmallArgs {
  SmallLayout L;
  const double *E;      // mAp
  const double *gvec;   // ntp
  double beta, cs;
  const double *invrho; // kp
  const double *bbot;   // n_iso x kp: scaled BOT bound E_bot * w_BOT
  const int32_t *active;
  int kp;
  double alpha;         // over-relaxation of the z- and y-steps (1: none)
};
// r = A_s W + g / rho - (2 clip(q2) - q2), from the GEMM1 partials.  The
// dose-point part G = sum of the partials; with gref (the BF16 refinement's hot
// iterations) G = gref + partials (the product of the change since the last
// refresh), and with gout (its refresh) G is also stored there for the
// running plans.  The refinement of S^-1 r: with rout (a refresh) r is also
// stored there for the running plans; with r32 (a hot iteration) r32 = r - rsub
// in FP32.
template <typename T>
hipError_t rhs(hipStream_t s, const SmallArgs &a, const T *P1, size_t zstride, int nchunk,
               const double *qs, const double *q2, double *r, const double *gref = nullptr,
               double *gout = nullptr, double *rout = nullptr, const double *rsub = nullptr,
               float *r32 = nullptr);
// y = (float) x, n values.
hipError_t to_f32(hipStream_t s, const double *x, float *y, size_t n);
// v = sum of the Sinv r partials (mAp x kp) and vT = (T) v_top (ntp x kp).
template <typename T>
hipError_t vreduce(hipStream_t s, const SmallArgs &a, const double *P2, size_t zstride, int nchunk,
                   double *v, T *vT);
// q2 <- v + Pi(q2); qs <- max(qs,0) - (A_sec' v); optional stats partials
// [block][kAdmmStats][kp].
hipError_t post(hipStream_t s, const SmallArgs &a, const double *v, double *qs, double *q2,
                double *stats, int *nblocks_out);
int post_blocks(const SmallLayout &L);
// that = rho * max(q2_top, 0) (shot times over E), as T.
template <typename T>
hipError_t shot_scaled(hipStream_t s, const SmallArgs &a, const double *q2, T *that);
// Per plan: F, c'z1, gap, r_pri, r_dual, oar ratio, from the partial stats.
struct FinalArgs {
  const double *admm_stats; int admm_blocks;
  const double *post_stats; int post_blocks;
  const double *obj_stats; int obj_blocks;
  const double *q2; const double *E; const double *invrho; const double *wbot;
  SmallLayout L; double cs; int kp;
  // certificate (NULL: none): per shot column and plan, the smallest sector
  // value that column's shot row allows for the dual point x = clip(z1)
  const double *need;   // ntp x kp
  double *out;   // kp x kFinal
};
// F, c'z, gap, r_pri, r_dual, oar_ratio, bot_sum, hinge, lower bound L, certified gap
constexpr int kFinal = 10;
hipError_t finalize(hipStream_t s, const FinalArgs &a);
// Certified bounds of a check (App. A duality): z1 = clip(q, 0, u) of the dose
// points as the operand of a split-K product with the dose block, then
// need[t][j] = max(0, (D~' z1)_t) D_T / phi_cal from its partials (E_t scales
// them back from the scaled block).  z_from_q writes z1 point-major (Np x kp, T).
template <typename T>
hipError_t z_from_q(hipStream_t s, const T *q, T *z, int Np, int kp, const PointTable<T> &pt);
template <typename T>
hipError_t cert_need(hipStream_t s, const SmallArgs &a, const T *P, size_t zstride, int nchunk,
                     double *need);
// t[j][t] = E_t rho_j max(q2_t, 0) (k x n_t, double)
hipError_t extract_t(hipStream_t s, const SmallArgs &a, const double *q2, double *t, int k);

// t as a shot-major matrix for products with dose rates: out[t][j] = E_t rho_j max(q2_t, 0)
// (ntp x kp, zero padding).
hipError_t shot_times_matrix(hipStream_t s, const SmallArgs &a, const double *q2, double *out);

// ---- Algorithm 1 and the low-dose band -----------------------------------------
struct Alg1Work {
  uint64_t *Vu, *pu, *pt, *nw, *po, *tmp, *uni;   // W words each
  uint64_t *keys;                                  // W * 64
  uint64_t *pj;                                    // k * W
  int64_t *vsize;                                  // k
  int32_t *order;                                  // k
  int64_t *offs;                                   // W
};
// vols: k x W words (device); P: n_vox capacity; masks: k rows of ldm >= W words.
hipError_t alg1_select(hipStream_t s, int k, int64_t n_vox, const uint64_t *vols, const int32_t *n_ld,
                       uint64_t seed, Alg1Work &wk, int64_t *P, int64_t *nP, uint64_t *masks, int ldm);
// Scratch of the allocation-free Algorithm 1: a file-scope device array of
// alg1_scratch_bytes() per device; alg1_scratch gives its device address on
// `device` (current), to be used under alg1_scratch_lock(device).
size_t alg1_scratch_bytes();
hipError_t alg1_scratch(int device, unsigned char **ptr);
std::mutex *alg1_scratch_lock(int device);
// bits[j][v / 64] bit v % 64 = (lo <= d[v][j] < hi), d: n_vox rows of ldd.
hipError_t band_bits(hipStream_t s, const double *d, int ldd, int n_vox, int k, double lo, double hi,
                     uint64_t *bits);

// W = 2 clip(q, 0, u) - q for every point and plan (Np x kp), after a state import.
template <typename T>
hipError_t w_from_q(hipStream_t s, const T *q, T *w, int Np, int kp, const PointTable<T> &pt);

// ---- step-size switch ------------------------------------------------------------
// For every plan j with fac[j] != 1: y <- fac[j] y at fixed z (q = z + y) on
// the dose points, the sector variables and the small rows, and 1/rho_j <-
// fac[j] / rho_j (fac = rho_old / rho_new).
template <typename T>
hipError_t rescale_points(hipStream_t s, T *q, int Np, int kp, const PointTable<T> &pt, const double *fac);
hipError_t rescale_small(hipStream_t s, const SmallArgs &a, double *q2, double *qs, double *invrho,
                         const double *fac);

// ---- state conversion ---------------------------------------------------------
template <typename T>
hipError_t export_points(hipStream_t s, const T *q, int ldq, const PointTable<T> &pt, int N, int k,
                         double *z, double *y);
template <typename T>
hipError_t import_points(hipStream_t s, T *q, int ldq, int N, int k, const double *z, const double *y);

// ---- BF16-pair products --------------------------------------------------------
// An FP32/FP64 operand x is carried as the pair hi = bf16(x), lo = bf16(x - hi)
// (16 significant bits); both operands are stored row-major with the
// reduction index contiguous (A: M x K rows, B: N x K rows).  A product sums
// A_hi B_hi + A_hi B_lo + A_lo B_hi (terms = 3) or A_hi B_hi alone (terms = 1,
// a single BF16 operand on each side) on the BF16 MFMA with FP32
// accumulation, in the same order for every tile configuration.
struct BfPair { const uint16_t *hi, *lo; int ld; };
// which: 0 split-K, 1 point-row; some configurations serve terms = 1 only
bool gemm_bf_cfg_ok(int which, int cfg, int M, int N, int terms);
// P[z][m][n] = sum over rows k of chunk z of A[m][k] B[n][k]  (split-K partials, FP32)
hipError_t gemm_bf_tn(hipStream_t s, BfPair A, BfPair B, float *P, int ldp, int M, int N, int K,
                      int nchunk, int terms, int cfg);
// Epilogue variants of the point-row product for the BF16 refinement mode
// (LADMM_BF16).  The hot iterations multiply single BF16 operands by the
// change since the last refresh; a refresh iteration runs the three-term
// products and records the references.
enum {
  BF_PLAIN = 0,     // pairs in and out (LADMM_BF16X3; also the objective product)
  BF_DELTA = 1,     // product = X_ref + D_hi dv; writes dW = bf16(W' - W_ref)
  BF_DELTA_PAIR = 2,// product = X_ref + D_hi dv; writes W' as pairs (a refresh follows)
  BF_REFRESH = 3    // three-term product; X_ref := product, W_ref := W (pairs' value);
                    // writes W' as pairs and dW
};
// C = A B' with the ADMM / statistics / objective epilogues
hipError_t gemm_bf_nn(hipStream_t s, int epi, BfPair A, BfPair B, int M, int N, int K,
                      const EpiArgs<float> &ea, int terms, int cfg, int delta = BF_PLAIN);
// D^ = Dt diag(E) as pairs in fragment order (16-row tiles x 32-wide k steps,
// 1 KiB per fragment), point-major (Np x ntp) and shot-major (ntp x Np).
hipError_t split_dose_bf16(hipStream_t s, const double *Dt, const double *E, int Np, int ntp,
                           uint16_t *Dh, uint16_t *Dl, uint16_t *DTh, uint16_t *DTl);
// v_top and the scaled shot times as plan-major pairs (kp x ntp) for the products.
// With vref != NULL (a refresh): also vref := hi + lo (the value the pairs
// carry) for the running plans, and with vout, v itself (all mAp rows).
hipError_t vreduce_bf(hipStream_t s, const SmallArgs &a, const double *P2, size_t zstride, int nchunk,
                      double *v, uint16_t *vh, uint16_t *vl, double *vref = nullptr,
                      double *vout = nullptr);
// The hot iterations of LADMM_BF16: v = vbase + the FP32 partials of
// S^-1 (r - r_ref) (summed in FP64), and dv = bf16(v_top - vref) plan-major
// (kp x ntp).
hipError_t vreduce_delta_bf(hipStream_t s, const SmallArgs &a, const float *P2, size_t zstride,
                            int nchunk, const double *vbase, double *v, const double *vref,
                            uint16_t *dv);
hipError_t shot_scaled_bf(hipStream_t s, const SmallArgs &a, const double *q2, uint16_t *th,
                          uint16_t *tl);
// z1 = clip(q, 0, u) as plan-major pairs (kp x Np), the certificate's operand.
hipError_t z_from_q_bf(hipStream_t s, const float *q, int Np, int kp, const PointTable<float> &pt,
                       uint16_t *zh, uint16_t *zl);
// Zero rows j of plan-major BF16 arrays (halves x kp rows of len: 2 for pairs,
// hi rows then lo rows; 1 for a single array) with flag[j] != 0.
hipError_t zero_plan_rows_bf(hipStream_t s, uint16_t *a, int kp, int len, const int32_t *flag,
                             int halves = 2);
// W' pairs (kp x Np) from q after a state import; with wref and dw (LADMM_BF16)
// also dw = bf16(W' - W_ref).
hipError_t w_from_q_bf(hipStream_t s, const float *q, int Np, int kp, const PointTable<float> &pt,
                       uint16_t *wh, uint16_t *wl, const float *wref = nullptr,
                       uint16_t *dw = nullptr);

// Permutations of plan columns (bytes = element size: 2, 4 or 8).
// gather_cols: out[r][c] = in[r][src[c]] for a row-major rows x ld array;
// gather_rows: out[r][:] = in[src[r]][:] for nrows rows of len elements.
hipError_t gather_cols(hipStream_t s, const void *in, void *out, size_t rows, int ld, int bytes,
                       const int *src);
hipError_t gather_rows(hipStream_t s, const void *in, void *out, int nrows, size_t len, int bytes,
                       const int *src);

// Zero the columns j of a (rows x ld, row-major) whose flag[j] is nonzero:
// the start of a fresh plan in a reused column.
template <typename T>
hipError_t zero_columns(hipStream_t s, T *a, size_t rows, int ld, const int32_t *flag);

}  // namespace ladmm
