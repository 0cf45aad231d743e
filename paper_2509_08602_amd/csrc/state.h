// Internal state of the library's handles (not part of the C ABI).
//
// A context owns a device and an HBM budget; a case owns the resident dose
// block, the Schur complement inverse and the point tables; a batch owns k plan
// columns (padded to kp) of iterates and per-plan tables.  The serving engine
// keeps one batch per resident case whose columns are reused as slots.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ladmm.h"
#include "kernels.h"

namespace ladmm {

// Tile configurations per dose-matrix product in the largest table (the
// BF16-pair kernels; the FP32 / FP64 tables have kGemmCfgs and reject the rest).
constexpr int kMaxGemmCfgs = 10;

// Message of the last error on the calling thread (ladmm_last_error).
extern thread_local std::string g_err;
int fail(int code, const std::string &msg);

#define HIPC(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::ladmm::fail(LADMM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Precision modes whose dose block is held as BF16 pairs (products on the BF16 MFMA).
inline bool bf16_block(int precision) { return precision == LADMM_BF16X3 || precision == LADMM_BF16; }

// Stopping rule of one plan column: converged at a check where rel_gap,
// r_pri and r_dual are within their tolerances (tol_gap <= 0: never), and
// stopped at max_iter iterations of its own.
struct StopRule {
  int32_t max_iter;
  double tol_gap, tol_pri, tol_dual, tol_cert;
  // step-size balancing (adapt = 0: the fixed rule); rho kept in [rho_lo, rho_hi]
  int32_t adapt;
  double mu, tau, rho_lo, rho_hi;
};

// The stopping and step-size rule of a plan that starts with step size rho.
inline StopRule make_rule(const ladmm_opts &o, int32_t max_iter, double rho) {
  return StopRule{max_iter, o.tol_gap, o.tol_pri, o.tol_dual, o.tol_cert, o.adapt_rho, o.adapt_mu,
                  o.adapt_tau, rho * 1e-3, rho * 1e3};
}

// Whether a plan's statistics at a check (kFinal values: F, c'z, gap, r_pri,
// r_dual, oar, bot, hinge, L, cert gap) meet its stopping rule: every
// tolerance in use holds, and at least one of tol_gap, tol_cert is in use.
inline bool rule_met(const StopRule &r, const double *f) {
  if (!(r.tol_gap > 0) && !(r.tol_cert > 0)) return false;
  if (r.tol_gap > 0 && !(f[2] <= r.tol_gap)) return false;
  if (r.tol_cert > 0 && !(f[9] <= r.tol_cert)) return false;
  if (r.tol_pri > 0 && !(f[3] <= r.tol_pri)) return false;
  if (r.tol_dual > 0 && !(f[4] <= r.tol_dual)) return false;
  return true;
}

}  // namespace ladmm

struct ladmm_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  int refs = 0;              // live cases
  bool destroyed = false;    // destroy requested while cases were alive
  std::mutex mu;
};

struct ladmm_case {
  ladmm_ctx *ctx = nullptr;
  int precision = LADMM_F64;
  int N = 0, Np = 0, n_iso = 0, S = 8, C = 3, n_t = 0, ntp = 0, n_sec = 0, mAp = 0, G = 0;
  double beta = 1.0, cs = 0.0;
  int row_normalize = 1;
  ladmm::SmallLayout L{};
  void *D = nullptr;         // Np x ntp, scaled point block of A' (precision T)
  // LADMM_BF16X3 and LADMM_BF16: the same block as BF16 pairs, point-major and shot-major
  const uint16_t *Dh = nullptr, *Dl = nullptr, *DTh = nullptr, *DTl = nullptr;
  void *sig = nullptr;       // Np (T)
  int32_t *grp = nullptr;    // Np
  int32_t *is_ld = nullptr;  // G + 1
  int32_t *is_oar = nullptr; // G + 1
  double *E = nullptr;       // mAp
  double *gvec = nullptr;    // ntp
  double *Smat = nullptr;    // mAp x mAp
  double *Sinv = nullptr;    // mAp x mAp
  float *Sinv32 = nullptr;   // LADMM_BF16: Sinv in FP32 for the hot iterations
  std::vector<ladmm_group> groups;
  std::vector<int32_t> hgrp;
  std::vector<int64_t> counts;
  std::vector<double> hE;
  std::vector<void *> allocs;
  size_t bytes = 0;
  float setup_ms = 0.f;
  int nchunk1 = 1, nchunk2 = 1;
  int refs = 0;              // live batches
  bool destroyed = false;    // destroy requested while batches were alive
  // per padded plan count: tiles of GEMM1, GEMM2 and the S^-1 product
  struct Tuned { int kp, cfg1, cfg2, cfg_s, cfg1r, cfg2r; };
  std::vector<Tuned> tuned;
};

struct ladmm_batch {
  ladmm_case *c = nullptr;
  int k = 0, kp = 0, mask_words = 0;
  // Launched plan columns of the dose-matrix products: kp, or (while
  // ladmm_batch_run compacts the running plans into a dense prefix) fewer.
  int kact = 0;
  // Compaction state: plan held by each column (identity outside a run), and
  // device scratch for the column permutation.
  std::vector<int> plan_at;
  int *perm_d = nullptr;
  void *perm_tmp = nullptr;
  size_t perm_tmp_bytes = 0;
  bool compact = true;
  hipStream_t stream = nullptr;
  void *q = nullptr;          // Np x kp (T): q = z1 + y1 of the dose points
  void *W = nullptr;          // Np x kp (T): W = z1 - y1, input of the next GEMM1
  double *qs = nullptr;       // n_sec x kp
  double *q2 = nullptr;       // mAp x kp
  void *utab = nullptr;       // (G + 1) x kp (T)
  uint64_t *mask = nullptr;   // kp x mask_words
  double *invrho = nullptr, *bbot = nullptr, *wbot = nullptr;
  double *fac = nullptr;      // kp: scaled-dual factor rho_old / rho_new of a switch
  double *h_fac = nullptr;    // pinned kp
  int32_t *active = nullptr;
  void *P1 = nullptr;
  double *r = nullptr, *P2 = nullptr, *v = nullptr;
  void *vT = nullptr, *that = nullptr;
  // LADMM_BF16 (refinement): references of the last refresh and the change of
  // W since it (plan-major, kp x Np)
  float *xref = nullptr, *wref = nullptr;   // Np x kp
  // and of S^-1 r: r and v of the last refresh (mAp x kp), and the change of r
  // since it in FP32
  double *rref = nullptr, *vfull = nullptr;
  float *r32 = nullptr;
  double *gref = nullptr, *vref = nullptr;  // ntp x kp
  uint16_t *dW = nullptr;
  // certificate of a check: z1 of the dose points (point-major T, or plan-major
  // pairs for the BF16 blocks) and the smallest sector values of the dual point
  void *zc = nullptr;
  double *need = nullptr;     // ntp x kp
  double *admm_stats = nullptr, *post_stats = nullptr, *obj_stats = nullptr, *fin = nullptr;
  int admm_blocks = 0, post_blocks = 0, obj_blocks = 0;
  std::vector<void *> allocs;
  size_t bytes = 0;
  std::vector<ladmm_weights> w;
  std::vector<double> rho;
  std::vector<int32_t> h_active, status, iters;
  std::vector<int32_t> start;   // per plan: iters_run when the plan (re)started
  std::vector<ladmm::StopRule> rule;   // per plan stopping rule
  std::vector<double> rec;    // k x kFinal, per-plan statistics at the last check
  double *h_fin = nullptr;    // pinned kp x kFinal
  ladmm_opts opts{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double iterate_ms = 0.0;
  int64_t plan_iters = 0;
  int iters_run = 0;
  int chunk_active = 0;       // active plans of the chunk in flight
  // tile configurations of the two dose-matrix products (autotuned)
  int cfg1 = 0, cfg2 = 0;
  // LADMM_BF16: configurations of the refresh's three-term products (the
  // widest single-operand tiles do not fit their LDS)
  int cfg1r = 0, cfg2r = 0;
  int cfg_s = 1;              // the FP64 S^-1 r product (autotuned too)
  double alpha = 1.0;         // over-relaxation of the z- and y-steps
  bool tuned = false;
  // captured iteration chunks, replayed while profiling is off
  struct Graph { int n, kact, cfg1, cfg2, cfg_s, cfg1r, cfg2r; hipGraphExec_t exec; };
  bool graphs = true;
  std::vector<Graph> graph_cache;
  // captures run on a stream of their own that does not synchronize with the
  // legacy stream, so other threads' synchronous copies never meet a capture
  hipStream_t cap_stream = nullptr;
  // per-kernel event timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;      // kind of each recorded pair
  size_t ev_used = 0;            // events handed out in the current chunk
  double kms[LADMM_N_KERNEL_CLASSES] = {};
  int64_t kcount[LADMM_N_KERNEL_CLASSES] = {};
};

namespace ladmm {

int ctx_alloc(ladmm_ctx *ctx, void **p, size_t bytes, size_t *charged);
void ctx_release(ladmm_ctx *ctx, size_t bytes);
// Case references held by batches and queued requests; the last one frees a
// destroyed case.
int case_ref(ladmm_case *c);
void case_unref(ladmm_case *c);
int batch_alloc(ladmm_batch *b, void **p, size_t bytes);
// slots = true: every column starts inactive, with a device LD mask, and the
// per-plan tables are left for the caller to fill (the weights are ignored).
int create_batch_impl(ladmm_case *c, int32_t k, const ladmm_weights *w, const uint64_t *ld_mask,
                      const double *rho, const ladmm_opts *opts, ladmm_batch **out,
                      bool slots = false);
int destroy_batch_impl(ladmm_batch *b);
SmallArgs small_args(const ladmm_batch *b);
// Point tables of a batch (group, sign, bounds, LD mask) for the kernels.
template <typename T>
PointTable<T> point_table(const ladmm_batch *b) {
  const ladmm_case *c = b->c;
  PointTable<T> pt;
  pt.grp = c->grp;
  pt.sig = (const T *)c->sig;
  pt.is_ld = c->is_ld;
  pt.is_oar = c->is_oar;
  pt.utab = (const T *)b->utab;
  pt.ldu = b->kp;
  pt.mask = b->mask;
  pt.mask_words = b->mask_words;
  return pt;
}
// Tile configurations of the two dose-matrix products (autotuned or default).
int prepare_batch(ladmm_batch *b);
// Enqueue n iterations (the last with statistics) and the read-back of the
// statistics on the batch's stream; returns without waiting.
int chunk_launch(ladmm_batch *b, int n);
// Wait for the chunk, update per-plan records, and with `decide` apply each
// plan's stopping rule.  Frozen plans get h_active = 0; *changed reports any.
int chunk_complete(ladmm_batch *b, int n, bool decide, bool *changed);
// Step-size balancing after a full check chunk (decide): new rho of the
// running plans that ask for it, and the rescale of their scaled duals on the
// batch's stream.  *switched reports any change.
int adapt_rho(ladmm_batch *b, bool *switched);
// tau_i = (phi_cal/D_T) max_s sum_c t_isc for one plan's shot times.
void bot_from_t(const ladmm_case *c, const double *t, double *bot);

}  // namespace ladmm
