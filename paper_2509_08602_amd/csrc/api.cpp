// C ABI of the batched ADMM library: contexts, resident cases, plan batches.
//
// The host code here validates descriptors, owns device memory, and orders
// the kernel launches of one ADMM iteration (Sec. 2.B) on the batch's stream:
//
//   GEMM1   P1 = D^' W,   W = z1 - y1 of the dose points     (A_s x1 part of
//           Eq. partial_elimination; split over point chunks)
//   rhs     r = A_s (z1 - y1 - c/rho) - (z2 - y2)
//   solve   v = S^-1 r                                      (cached FP64 inverse)
//   post    x2/z2/y2 update and the sector variables
//   GEMM2   q <- clip(q, 0, u) - c/rho - D^ v  for the dose points (closed form
//           of the x-step with the z- and y-steps of Eq. (admm) fused)
//
// and, every check_every iterations, the planning objective F(t) of the
// current shot times with the stopping statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "state.h"
#include "metrics.h"

namespace ladmm {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// Device allocation charged to a context's HBM budget.
int ctx_alloc(ladmm_ctx *ctx, void **p, size_t bytes, size_t *charged) {
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->budget && ctx->used + bytes > ctx->budget)
      return fail(LADMM_E_NOMEM, "HBM budget exceeded: need " + std::to_string(bytes) +
                                     " more bytes, " + std::to_string(ctx->budget - ctx->used) +
                                     " left");
    ctx->used += bytes;
  }
  hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->used -= bytes;
    *p = nullptr;
    return fail(LADMM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  *charged += bytes;
  return LADMM_OK;
}

void ctx_release(ladmm_ctx *ctx, size_t bytes) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->used -= std::min(bytes, ctx->used);
}

}  // namespace ladmm

using namespace ladmm;

namespace ladmm {

void ctx_ref(ladmm_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->refs++;
}

// Drop a case's reference; frees a context whose destroy call came first.
void ctx_unref(ladmm_ctx *ctx) {
  bool last;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->refs--;
    last = ctx->destroyed && ctx->refs == 0;
  }
  if (last) delete ctx;
}

}  // namespace ladmm

namespace ladmm {

int case_alloc(ladmm_case *c, void **p, size_t bytes) {
  int rc = ctx_alloc(c->ctx, p, bytes, &c->bytes);
  if (rc == LADMM_OK) c->allocs.push_back(*p);
  return rc;
}

int batch_alloc(ladmm_batch *b, void **p, size_t bytes) {
  int rc = ctx_alloc(b->c->ctx, p, bytes, &b->bytes);
  if (rc == LADMM_OK) b->allocs.push_back(*p);
  return rc;
}


SmallArgs small_args(const ladmm_batch *b) {
  const ladmm_case *c = b->c;
  SmallArgs a;
  a.L = c->L;
  a.E = c->E;
  a.gvec = c->gvec;
  a.beta = c->beta;
  a.cs = c->cs;
  a.invrho = b->invrho;
  a.bbot = b->bbot;
  a.active = b->active;
  a.kp = b->kp;
  a.alpha = b->alpha;
  return a;
}

// ---------------------------------------------------------------------------
// case setup
// ---------------------------------------------------------------------------
template <typename T>
int setup_precision(ladmm_case *c, const double *Dt, hipStream_t s) {
  void *p = nullptr;
  int rc = case_alloc(c, &p, (size_t)c->Np * c->ntp * sizeof(T));
  if (rc) return rc;
  c->D = p;
  HIPC(scale_columns<T>(s, Dt, c->E, (T *)c->D, c->Np, c->ntp));
  return LADMM_OK;
}

// D^ = Dt diag(E) as BF16 pairs in both layouts: point-major (for the
// point-row products) and shot-major (for the split-K product).
int setup_bf16(ladmm_case *c, const double *Dt, hipStream_t s) {
  void *p = nullptr;
  const size_t n = (size_t)c->Np * c->ntp;
  int rc = case_alloc(c, &p, 4 * n * sizeof(uint16_t));
  if (rc) return rc;
  uint16_t *base = (uint16_t *)p;
  c->Dh = base;
  c->Dl = base + n;
  c->DTh = base + 2 * n;
  c->DTl = base + 3 * n;
  HIPC(split_dose_bf16(s, Dt, c->E, c->Np, c->ntp, base, base + n, base + 2 * n, base + 3 * n));
  return LADMM_OK;
}

// Number of row chunks of a split-K product over K rows whose output has
// `tiles` tiles: the fewest chunks (of at least min_rows rows, boundaries on
// 32-row multiples as the product places them) that give `rounds` or more
// rounds of workgroups over the CUs with the last round nearly full.
int balanced_chunks(int K, int tiles, int min_rows, int rounds_min) {
  constexpr int kCUs = 256;
  const int maxc = std::max(1, K / min_rows);
  int best = maxc;
  double best_eff = -1.0;
  for (int n = 1; n <= maxc; ++n) {
    const int kchunk = round_up((K + n - 1) / n, 32);
    const int neff = (K + kchunk - 1) / kchunk;
    const long W = (long)tiles * neff;
    const long rounds = (W + kCUs - 1) / kCUs;
    const double eff = (double)W / (double)(kCUs * rounds);
    if (W >= rounds_min * kCUs - kCUs / 16 && eff >= 0.95) return neff;
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = neff;
    }
  }
  return best;
}

// dose_dev: the N x n_t dose rates already on the device (caller-owned; d->dose
// is then not read).  keep_dose: receives the device copy of the dose rates
// made from d->dose, which the caller then owns (hipFree), for later passes.
int create_case_impl(ladmm_ctx *ctx, const ladmm_case_desc *d, ladmm_case **out,
                     const double *dose_dev = nullptr, double **keep_dose = nullptr) {
  if (!ctx || !d || !out) return fail(LADMM_E_INVALID, "null argument");
  if (d->n_points < 1 || d->n_iso < 1 || d->n_sectors < 1 || d->n_collimators < 1)
    return fail(LADMM_E_INVALID, "sizes must be positive");
  if ((!d->dose && !dose_dev) || !d->point_group || !d->groups || d->n_groups < 1)
    return fail(LADMM_E_INVALID, "dose, point_group and groups are required");
  if (!(d->prescription_mean > 0) || !(d->phi_cal > 0))
    return fail(LADMM_E_INVALID, "prescription_mean and phi_cal must be > 0");
  if (d->precision != LADMM_F64 && d->precision != LADMM_F32 && !bf16_block(d->precision))
    return fail(LADMM_E_INVALID, "unknown precision");
  const int n_t = d->n_iso * d->n_sectors * d->n_collimators;
  for (int g = 0; g < d->n_groups; ++g) {
    const ladmm_group &gr = d->groups[g];
    if (gr.type < LADMM_PT_TS || gr.type > LADMM_PT_OAR)
      return fail(LADMM_E_INVALID, "group " + std::to_string(g) + ": bad type");
    if (!(gr.threshold > 0) || !std::isfinite(gr.threshold))
      return fail(LADMM_E_INVALID, "group " + std::to_string(g) + ": threshold must be > 0");
    if (!(gr.share >= 0) || !std::isfinite(gr.share))
      return fail(LADMM_E_INVALID, "group " + std::to_string(g) + ": share must be >= 0");
  }
  std::vector<int64_t> counts(d->n_groups, 0);
  for (int p = 0; p < d->n_points; ++p) {
    const int g = d->point_group[p];
    if (g < 0 || g >= d->n_groups)
      return fail(LADMM_E_INVALID, "point " + std::to_string(p) + ": group out of range");
    counts[g]++;
  }
  const size_t nd = (size_t)d->n_points * n_t;   // dose entries: checked on the device

  ladmm_case *c = new ladmm_case();
  c->ctx = ctx;
  c->precision = d->precision;
  c->N = d->n_points;
  c->Np = round_up(c->N, kTileRows);
  c->n_iso = d->n_iso;
  c->S = d->n_sectors;
  c->C = d->n_collimators;
  c->n_t = n_t;
  c->ntp = round_up(n_t, kSmallAlign);
  c->n_sec = d->n_iso * d->n_sectors;
  c->mAp = round_up(c->ntp + c->n_iso, kSmallAlign);
  c->G = d->n_groups;
  c->cs = d->phi_cal / d->prescription_mean;
  c->row_normalize = d->row_normalize ? 1 : 0;
  c->groups.assign(d->groups, d->groups + d->n_groups);
  c->hgrp.assign(d->point_group, d->point_group + d->n_points);
  c->counts = counts;
  if (d->beta > 0) {
    c->beta = d->beta;
  } else {
    const double den = d->beta_denominator > 0 ? d->beta_denominator : 2000.0;
    int64_t non_oar = 0;
    for (int g = 0; g < d->n_groups; ++g)
      if (d->groups[g].type != LADMM_PT_OAR) non_oar += counts[g];
    c->beta = (double)non_oar / den;
    if (!(c->beta > 0)) c->beta = 1.0;
  }
  c->L = SmallLayout{c->n_t, c->ntp, c->n_iso, c->mAp, c->n_sec, c->S, c->C};
  // GEMM split factors depend on the case only, so a plan's arithmetic does
  // not depend on how many other plans share its batch.
  c->nchunk1 = balanced_chunks(c->Np, c->ntp / 64, 256, 4);
  c->nchunk2 = balanced_chunks(c->mAp, c->mAp / 32, 64, 2);

  auto cleanup = [&](int rc) {
    for (void *p : c->allocs) hipFree(p);
    ctx_release(ctx, c->bytes);
    delete c;
    return rc;
  };
  int rc;
  HIPC(hipSetDevice(ctx->device));
  hipStream_t s;
  HIPC(hipStreamCreate(&s));
  hipEvent_t e0, e1;
  HIPC(hipEventCreate(&e0));
  HIPC(hipEventCreate(&e1));
  HIPC(hipEventRecord(e0, s));

  // point tables
  std::vector<double> hsig(c->Np, 0.0), hinv(c->Np, 0.0);
  std::vector<int32_t> hgrp(c->Np, c->G);
  for (int p = 0; p < c->N; ++p) {
    const ladmm_group &gr = d->groups[d->point_group[p]];
    hsig[p] = (gr.type == LADMM_PT_TS || gr.type == LADMM_PT_TI) ? 1.0 : -1.0;
    hinv[p] = 1.0 / gr.threshold;
    hgrp[p] = d->point_group[p];
  }
  std::vector<int32_t> hld(c->G + 1, 0), hoar(c->G + 1, 0);
  for (int g = 0; g < c->G; ++g) {
    hld[g] = d->groups[g].type == LADMM_PT_LD;
    hoar[g] = d->groups[g].type == LADMM_PT_OAR;
  }
  void *p = nullptr;
  double *dphi = nullptr, *dsig64 = nullptr, *dinv = nullptr, *Dt = nullptr, *K = nullptr;
  double *Pk = nullptr, *Sw = nullptr, *X = nullptr, *Pg = nullptr, *sigmat = nullptr;
  int *dinfo = nullptr;
  std::vector<void *> temps;
  auto talloc = [&](void **pp, size_t bytes) -> int {
    hipError_t e = hipMalloc(pp, bytes ? bytes : 1);
    if (e != hipSuccess) return fail(LADMM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    temps.push_back(*pp);
    return LADMM_OK;
  };
  auto tclean = [&](int code) {
    hipStreamSynchronize(s);
    for (void *t : temps) hipFree(t);
    hipStreamDestroy(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return cleanup(code);
  };
#define SETUP_HIP(call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      fail(LADMM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));               \
      return tclean(LADMM_E_DEVICE);                                                         \
    }                                                                                        \
  } while (0)
#define SETUP_RC(expr)            \
  do {                            \
    int rc_ = (expr);             \
    if (rc_) return tclean(rc_);  \
  } while (0)

  const size_t Tsz = c->precision == LADMM_F64 ? sizeof(double) : sizeof(float);
  SETUP_RC(case_alloc(c, &p, (size_t)c->Np * sizeof(int32_t)));
  c->grp = (int32_t *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)c->Np * Tsz));
  c->sig = p;
  SETUP_RC(case_alloc(c, &p, (size_t)(c->G + 1) * sizeof(int32_t)));
  c->is_ld = (int32_t *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)(c->G + 1) * sizeof(int32_t)));
  c->is_oar = (int32_t *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)c->mAp * sizeof(double)));
  c->E = (double *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)c->ntp * sizeof(double)));
  c->gvec = (double *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)c->mAp * c->mAp * sizeof(double)));
  c->Smat = (double *)p;
  SETUP_RC(case_alloc(c, &p, (size_t)c->mAp * c->mAp * sizeof(double)));
  c->Sinv = (double *)p;
  if (c->precision == LADMM_BF16) {
    SETUP_RC(case_alloc(c, &p, (size_t)c->mAp * c->mAp * sizeof(float)));
    c->Sinv32 = (float *)p;
  }

  SETUP_HIP(hipMemcpyAsync(c->grp, hgrp.data(), c->Np * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SETUP_HIP(hipMemcpyAsync(c->is_ld, hld.data(), (c->G + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  SETUP_HIP(hipMemcpyAsync(c->is_oar, hoar.data(), (c->G + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (c->precision == LADMM_F64) {
    SETUP_HIP(hipMemcpyAsync(c->sig, hsig.data(), c->Np * sizeof(double), hipMemcpyHostToDevice, s));
  } else {
    std::vector<float> fs(hsig.begin(), hsig.end());
    SETUP_HIP(hipMemcpyAsync(c->sig, fs.data(), c->Np * sizeof(float), hipMemcpyHostToDevice, s));
    SETUP_HIP(hipStreamSynchronize(s));
  }

  // dose matrix -> D~ = sign * phi / D_alpha (FP64, padded)
  if (dose_dev != nullptr) {
    dphi = const_cast<double *>(dose_dev);   // read only
  } else {
    SETUP_RC(talloc((void **)&dphi, nd * sizeof(double)));
    SETUP_HIP(hipMemcpyAsync(dphi, d->dose, nd * sizeof(double), hipMemcpyHostToDevice, s));
  }
  SETUP_RC(talloc((void **)&dsig64, c->Np * sizeof(double)));
  SETUP_RC(talloc((void **)&dinv, c->Np * sizeof(double)));
  SETUP_RC(talloc((void **)&Dt, (size_t)c->Np * c->ntp * sizeof(double)));
  // every dose entry >= 0 and finite, checked where the entries now are
  unsigned long long *dbad = nullptr, hbad = ~0ull;
  SETUP_RC(talloc((void **)&dbad, sizeof(unsigned long long)));
  SETUP_HIP(hipMemcpyAsync(dbad, &hbad, sizeof(hbad), hipMemcpyHostToDevice, s));
  SETUP_HIP(check_dose(s, dphi, nd, dbad));
  SETUP_HIP(hipMemcpyAsync(&hbad, dbad, sizeof(hbad), hipMemcpyDeviceToHost, s));
  SETUP_HIP(hipStreamSynchronize(s));
  if (hbad != ~0ull) {
    fail(LADMM_E_INVALID, "dose entry " + std::to_string(hbad) + " is negative or not finite");
    return tclean(LADMM_E_INVALID);
  }
  SETUP_HIP(hipMemcpyAsync(dsig64, hsig.data(), c->Np * sizeof(double), hipMemcpyHostToDevice, s));
  SETUP_HIP(hipMemcpyAsync(dinv, hinv.data(), c->Np * sizeof(double), hipMemcpyHostToDevice, s));
  SETUP_HIP(scale_dose(s, dphi, c->N, n_t, dsig64, dinv, Dt, c->Np, c->ntp));

  // K = D~' D~ (FP64 SYRK through the split-K product), then E and S
  const int nck = std::max(1, std::min(64, c->Np / 256));
  SETUP_RC(talloc((void **)&Pk, (size_t)nck * c->ntp * c->ntp * sizeof(double)));
  SETUP_RC(talloc((void **)&K, (size_t)c->ntp * c->ntp * sizeof(double)));
  SETUP_HIP(gemm_tn<double>(s, Dt, c->ntp, Dt, c->ntp, Pk, c->ntp, c->ntp, c->ntp, c->Np, nck, nullptr));
  SETUP_HIP(reduce_partials<double>(s, Pk, (size_t)c->ntp * c->ntp, nck, c->ntp, c->ntp, c->ntp, K, c->ntp));
  SETUP_HIP(assemble_schur(s, K, c->ntp, c->L, c->cs, c->beta, 0.0, c->row_normalize, c->E, c->Smat));

  // g = A_s (-c) on the shot rows: E_t sum_p sign_p D~[p][t]
  SETUP_RC(talloc((void **)&sigmat, (size_t)c->Np * 32 * sizeof(double)));
  {
    std::vector<double> hs(c->Np * 32, 0.0);
    for (int q = 0; q < c->Np; ++q) hs[(size_t)q * 32] = hsig[q];
    SETUP_HIP(hipMemcpyAsync(sigmat, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    SETUP_RC(talloc((void **)&Pg, (size_t)nck * c->ntp * 32 * sizeof(double)));
    SETUP_HIP(gemm_tn<double>(s, Dt, c->ntp, sigmat, 32, Pg, 32, c->ntp, 32, c->Np, nck, nullptr));
    double *gt = nullptr;
    SETUP_RC(talloc((void **)&gt, (size_t)c->ntp * 32 * sizeof(double)));
    SETUP_HIP(reduce_partials<double>(s, Pg, (size_t)c->ntp * 32, nck, c->ntp, 32, 32, gt, 32));
    std::vector<double> hgt((size_t)c->ntp * 32), hE(c->mAp);
    SETUP_HIP(hipMemcpyAsync(hgt.data(), gt, hgt.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipMemcpyAsync(hE.data(), c->E, c->mAp * sizeof(double), hipMemcpyDeviceToHost, s));
    SETUP_HIP(hipStreamSynchronize(s));
    std::vector<double> hg(c->ntp, 0.0);
    for (int t = 0; t < c->n_t; ++t) hg[t] = hE[t] * hgt[(size_t)t * 32];
    SETUP_HIP(hipMemcpyAsync(c->gvec, hg.data(), c->ntp * sizeof(double), hipMemcpyHostToDevice, s));
    SETUP_HIP(hipStreamSynchronize(s));
    c->hE = hE;
  }

  // Cholesky of S (FP64), then S^-1 = X' X with X = L^-1
  SETUP_RC(talloc((void **)&Sw, (size_t)c->mAp * c->mAp * sizeof(double)));
  SETUP_RC(talloc((void **)&X, (size_t)c->mAp * c->mAp * sizeof(double)));
  SETUP_RC(talloc((void **)&dinfo, sizeof(int)));
  SETUP_HIP(hipMemsetAsync(dinfo, 0, sizeof(int), s));
  SETUP_HIP(hipMemcpyAsync(Sw, c->Smat, (size_t)c->mAp * c->mAp * sizeof(double), hipMemcpyDeviceToDevice, s));
  SETUP_HIP(cholesky(s, Sw, c->mAp, c->mAp, dinfo));
  SETUP_HIP(tri_inverse(s, Sw, X, c->mAp, c->mAp));
  {
    const int nci = std::max(1, std::min(16, c->mAp / 64));
    double *Pi = nullptr;
    SETUP_RC(talloc((void **)&Pi, (size_t)nci * c->mAp * c->mAp * sizeof(double)));
    SETUP_HIP(gemm_tn<double>(s, X, c->mAp, X, c->mAp, Pi, c->mAp, c->mAp, c->mAp, c->mAp, nci, nullptr));
    SETUP_HIP(reduce_partials<double>(s, Pi, (size_t)c->mAp * c->mAp, nci, c->mAp, c->mAp, c->mAp, c->Sinv, c->mAp));
    if (c->Sinv32 != nullptr) SETUP_HIP(to_f32(s, c->Sinv, c->Sinv32, (size_t)c->mAp * c->mAp));
  }
  int hinfo = 0;
  SETUP_HIP(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s));

  // scaled dose block in the iteration precision: D^ = D~ diag(E)
  if (c->precision == LADMM_F64) {
    SETUP_RC(setup_precision<double>(c, Dt, s));
  } else if (c->precision == LADMM_F32) {
    SETUP_RC(setup_precision<float>(c, Dt, s));
  } else {
    SETUP_RC(setup_bf16(c, Dt, s));
  }
  SETUP_HIP(hipEventRecord(e1, s));
  SETUP_HIP(hipStreamSynchronize(s));
  if (hinfo != 0) {
    fail(LADMM_E_NUMERIC, "Schur complement is not positive definite");
    return tclean(LADMM_E_NUMERIC);
  }
  SETUP_HIP(hipEventElapsedTime(&c->setup_ms, e0, e1));
  if (keep_dose != nullptr) {
    *keep_dose = nullptr;
    if (dose_dev == nullptr) {   // hand the device copy of the dose rates to the caller
      temps.erase(std::find(temps.begin(), temps.end(), (void *)dphi));
      *keep_dose = dphi;
    }
  }
  for (void *t : temps) hipFree(t);
  hipStreamDestroy(s);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
#undef SETUP_HIP
#undef SETUP_RC
  (void)rc;
  ctx_ref(ctx);
  *out = c;
  return LADMM_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
void case_free(ladmm_case *c) {
  hipSetDevice(c->ctx->device);
  for (void *p : c->allocs) hipFree(p);
  ctx_release(c->ctx, c->bytes);
  ladmm_ctx *ctx = c->ctx;
  delete c;
  ctx_unref(ctx);
}

// Take a reference on a live case (LADMM_E_STATE once destroy was called).
int case_ref(ladmm_case *c) {
  std::lock_guard<std::mutex> lk(c->ctx->mu);
  if (c->destroyed) return fail(LADMM_E_STATE, "case has been destroyed");
  c->refs++;
  return LADMM_OK;
}

// Drop a reference; frees a case whose destroy call came first.
void case_unref(ladmm_case *c) {
  bool last;
  {
    std::lock_guard<std::mutex> lk(c->ctx->mu);
    c->refs--;
    last = c->destroyed && c->refs == 0;
  }
  if (last) case_free(c);
}

int destroy_batch_impl(ladmm_batch *b) {
  if (!b) return LADMM_OK;
  if (b->stream) hipStreamSynchronize(b->stream);
  for (auto &g : b->graph_cache) hipGraphExecDestroy(g.exec);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  for (hipEvent_t e : b->ev_pool) hipEventDestroy(e);
  for (void *p : b->allocs) hipFree(p);
  ctx_release(b->c->ctx, b->bytes);
  if (b->h_fin) hipHostFree(b->h_fin);
  if (b->h_fac) hipHostFree(b->h_fac);
  if (b->ev0) hipEventDestroy(b->ev0);
  if (b->ev1) hipEventDestroy(b->ev1);
  if (b->stream) hipStreamDestroy(b->stream);
  ladmm_case *c = b->c;
  delete b;
  case_unref(c);
  return LADMM_OK;
}

int upload_tables(ladmm_batch *b, const uint64_t *ld_mask) {
  ladmm_case *c = b->c;
  const int G = c->G, kp = b->kp, k = b->k;
  // per-plan LD point counts under the mask
  std::vector<int64_t> cnt((size_t)(G + 1) * kp, 0);
  for (int g = 0; g < G; ++g)
    for (int j = 0; j < k; ++j) cnt[(size_t)g * kp + j] = c->counts[g];
  if (ld_mask) {
    for (int g = 0; g < G; ++g) {
      if (c->groups[g].type != LADMM_PT_LD) continue;
      for (int j = 0; j < k; ++j) cnt[(size_t)g * kp + j] = 0;
    }
    const int cw = (c->N + 63) / 64;   // caller's words per plan row
    for (int pnt = 0; pnt < c->N; ++pnt) {
      const int g = c->hgrp[pnt];
      if (c->groups[g].type != LADMM_PT_LD) continue;
      for (int j = 0; j < k; ++j) {
        const uint64_t wd = ld_mask[(size_t)j * cw + (pnt >> 6)];
        if ((wd >> (pnt & 63)) & 1ull) cnt[(size_t)g * kp + j]++;
      }
    }
  }
  std::vector<double> u((size_t)(G + 1) * kp, 0.0);
  for (int g = 0; g < G; ++g) {
    const ladmm_group &gr = c->groups[g];
    for (int j = 0; j < k; ++j) {
      double wt = 0.0;
      switch (gr.type) {
        case LADMM_PT_TS:
        case LADMM_PT_TI: wt = b->w[j].w_t; break;
        case LADMM_PT_RING: wt = b->w[j].w_r; break;
        case LADMM_PT_LD: wt = b->w[j].w_ld; break;
        default: wt = INFINITY;
      }
      double val;
      if (gr.type == LADMM_PT_OAR) {
        val = INFINITY;
      } else {
        const int64_t n = cnt[(size_t)g * kp + j];
        val = n > 0 ? gr.share * wt / (double)n : 0.0;
      }
      u[(size_t)g * kp + j] = val;
    }
  }
  if (c->precision == LADMM_F64) {
    HIPC(hipMemcpy(b->utab, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    std::vector<float> uf(u.begin(), u.end());
    HIPC(hipMemcpy(b->utab, uf.data(), uf.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  std::vector<double> invrho(kp, 0.0), wbot(kp, 0.0), bbot((size_t)c->n_iso * kp, 0.0);
  for (int j = 0; j < k; ++j) {
    invrho[j] = 1.0 / b->rho[j];
    wbot[j] = b->w[j].w_bot;
    for (int i = 0; i < c->n_iso; ++i) bbot[(size_t)i * kp + j] = c->hE[c->ntp + i] * b->w[j].w_bot;
  }
  HIPC(hipMemcpy(b->invrho, invrho.data(), kp * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(b->wbot, wbot.data(), kp * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(b->bbot, bbot.data(), bbot.size() * sizeof(double), hipMemcpyHostToDevice));
  if (ld_mask) {
    // device rows are padded to the padded point count; padding bits are zero
    const int cw = (c->N + 63) / 64;
    std::vector<uint64_t> m((size_t)kp * b->mask_words, 0);
    for (int j = 0; j < k; ++j) {
      std::memcpy(&m[(size_t)j * b->mask_words], ld_mask + (size_t)j * cw, cw * sizeof(uint64_t));
      if (c->N % 64) m[(size_t)j * b->mask_words + cw - 1] &= (1ull << (c->N % 64)) - 1;
    }
    HIPC(hipMemcpy(b->mask, m.data(), m.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
  }
  HIPC(hipMemcpy(b->active, b->h_active.data(), kp * sizeof(int32_t), hipMemcpyHostToDevice));
  return LADMM_OK;
}

int create_batch_impl(ladmm_case *c, int32_t k, const ladmm_weights *w, const uint64_t *ld_mask,
                      const double *rho, const ladmm_opts *opts, ladmm_batch **out, bool slots) {
  if (!c || (!w && !slots) || !opts || !out) return fail(LADMM_E_INVALID, "null argument");
  if (k < 1) return fail(LADMM_E_INVALID, "k must be >= 1");
  if (opts->max_iter < 0 || opts->check_every < 1)
    return fail(LADMM_E_INVALID, "max_iter must be >= 0 and check_every >= 1");
  for (int j = 0; j < k && !slots; ++j) {
    const ladmm_weights &x = w[j];
    if (!(x.w_bot > 0) || !std::isfinite(x.w_bot))
      return fail(LADMM_E_INVALID, "plan " + std::to_string(j) + ": w_bot must be > 0");
    if (!(x.w_t >= 0) || !(x.w_r >= 0) || !(x.w_ld >= 0) || !std::isfinite(x.w_t) ||
        !std::isfinite(x.w_r) || !std::isfinite(x.w_ld))
      return fail(LADMM_E_INVALID, "plan " + std::to_string(j) + ": weights must be finite and >= 0");
    if (rho && (!(rho[j] > 0) || !std::isfinite(rho[j])))
      return fail(LADMM_E_INVALID, "plan " + std::to_string(j) + ": rho must be > 0");
  }
  if (!slots && !rho && (!(opts->rho0 > 0) || !(opts->w0_bot > 0)))
    return fail(LADMM_E_INVALID, "rho0 and w0_bot must be > 0");
  if (opts->adapt_rho && (!(opts->adapt_mu > 1) || !(opts->adapt_tau > 1) ||
                          !std::isfinite(opts->adapt_mu) || !std::isfinite(opts->adapt_tau)))
    return fail(LADMM_E_INVALID, "adapt_mu and adapt_tau must be finite and > 1");
  if (opts->alpha != 0.0 && !(opts->alpha > 0.0 && opts->alpha < 2.0))
    return fail(LADMM_E_INVALID, "alpha must be in (0, 2) (0 selects 1)");

  {
    int rc = case_ref(c);
    if (rc) return rc;
  }
  ladmm_batch *b = new ladmm_batch();
  b->c = c;
  b->kp = round_up(k, 32);
  b->kact = b->kp;
  b->k = slots ? b->kp : k;
  k = b->k;
  b->plan_at.resize(k);
  for (int j = 0; j < k; ++j) b->plan_at[j] = j;
  b->opts = *opts;
  b->alpha = opts->alpha == 0.0 ? 1.0 : opts->alpha;
  if (slots)
    b->w.assign(k, ladmm_weights{0.0, 0.0, 0.0, 1.0});
  else
    b->w.assign(w, w + k);
  b->rho.resize(k);
  for (int j = 0; j < k; ++j)
    b->rho[j] = slots ? 1.0 : rho ? rho[j] : opts->rho0 * std::sqrt(opts->w0_bot / w[j].w_bot);
  b->h_active.assign(b->kp, 0);
  for (int j = 0; j < k && !slots; ++j) b->h_active[j] = 1;
  b->status.assign(k, slots ? LADMM_PLAN_CONVERGED : LADMM_PLAN_RUNNING);
  b->iters.assign(k, 0);
  b->start.assign(k, 0);
  b->rule.resize(k);
  for (int j = 0; j < k; ++j) b->rule[j] = make_rule(*opts, opts->max_iter, b->rho[j]);
  b->rec.assign((size_t)k * kFinal, NAN);
  b->mask_words = (c->Np + 63) / 64;

  auto bad = [&](int rc) {
    destroy_batch_impl(b);
    return rc;
  };
#define B_RC(expr)           \
  do {                       \
    int rc_ = (expr);        \
    if (rc_) return bad(rc_); \
  } while (0)
#define B_HIP(call)                                                                    \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      fail(LADMM_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));         \
      return bad(LADMM_E_DEVICE);                                                      \
    }                                                                                  \
  } while (0)
  B_HIP(hipSetDevice(c->ctx->device));
  B_HIP(hipStreamCreate(&b->stream));
  B_HIP(hipEventCreate(&b->ev0));
  B_HIP(hipEventCreate(&b->ev1));
  const size_t Tsz = c->precision == LADMM_F64 ? sizeof(double) : sizeof(float);
  const int kp = b->kp;
  void *p;
  B_RC(batch_alloc(b, &p, (size_t)c->Np * kp * Tsz)); b->q = p;
  B_RC(batch_alloc(b, &p, (size_t)c->Np * kp * Tsz)); b->W = p;
  B_RC(batch_alloc(b, &p, (size_t)c->n_sec * kp * sizeof(double))); b->qs = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(double))); b->q2 = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)(c->G + 1) * kp * Tsz)); b->utab = p;
  if (ld_mask || slots) {
    B_RC(batch_alloc(b, &p, (size_t)kp * b->mask_words * sizeof(uint64_t)));
    b->mask = (uint64_t *)p;
  }
  B_RC(batch_alloc(b, &p, kp * sizeof(double))); b->invrho = (double *)p;
  B_RC(batch_alloc(b, &p, kp * sizeof(double))); b->wbot = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->n_iso * kp * sizeof(double))); b->bbot = (double *)p;
  B_RC(batch_alloc(b, &p, kp * sizeof(int32_t))); b->active = (int32_t *)p;
  B_RC(batch_alloc(b, &p, kp * sizeof(double))); b->fac = (double *)p;
  B_RC(batch_alloc(b, &p, kp * sizeof(int32_t))); b->perm_d = (int *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->nchunk1 * c->ntp * kp * Tsz)); b->P1 = p;
  B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(double))); b->r = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->nchunk2 * c->mAp * kp * sizeof(double))); b->P2 = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(double))); b->v = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)c->ntp * kp * Tsz)); b->vT = p;
  B_RC(batch_alloc(b, &p, (size_t)c->ntp * kp * Tsz)); b->that = p;
  if (c->precision == LADMM_BF16) {
    // references of the refinement (zero: the first products are of the full operands)
    B_RC(batch_alloc(b, &p, (size_t)c->Np * kp * sizeof(float))); b->xref = (float *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->Np * kp * sizeof(float))); b->wref = (float *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->ntp * kp * sizeof(double))); b->gref = (double *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->ntp * kp * sizeof(double))); b->vref = (double *)p;
    B_RC(batch_alloc(b, &p, (size_t)kp * c->Np * sizeof(uint16_t))); b->dW = (uint16_t *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(double))); b->rref = (double *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(double))); b->vfull = (double *)p;
    B_RC(batch_alloc(b, &p, (size_t)c->mAp * kp * sizeof(float))); b->r32 = (float *)p;
    B_HIP(hipMemsetAsync(b->rref, 0, (size_t)c->mAp * kp * sizeof(double), b->stream));
    B_HIP(hipMemsetAsync(b->vfull, 0, (size_t)c->mAp * kp * sizeof(double), b->stream));
    B_HIP(hipMemsetAsync(b->r32, 0, (size_t)c->mAp * kp * sizeof(float), b->stream));
    B_HIP(hipMemsetAsync(b->xref, 0, (size_t)c->Np * kp * sizeof(float), b->stream));
    B_HIP(hipMemsetAsync(b->wref, 0, (size_t)c->Np * kp * sizeof(float), b->stream));
    B_HIP(hipMemsetAsync(b->gref, 0, (size_t)c->ntp * kp * sizeof(double), b->stream));
    B_HIP(hipMemsetAsync(b->vref, 0, (size_t)c->ntp * kp * sizeof(double), b->stream));
    B_HIP(hipMemsetAsync(b->dW, 0, (size_t)kp * c->Np * sizeof(uint16_t), b->stream));
  }
  // certificate operand (z1 of the points) and sector values
  B_RC(batch_alloc(b, &p, (size_t)c->Np * kp * Tsz)); b->zc = p;
  B_RC(batch_alloc(b, &p, (size_t)c->ntp * kp * sizeof(double))); b->need = (double *)p;
  // statistics partials: one per row block of GEMM2, sized for the smallest
  // row block of any tile configuration (the autotuner may pick it)
  const int max_row_blocks = c->Np / kNnStatRows;
  b->admm_blocks = b->obj_blocks = c->Np / kNnStatRows;
  b->post_blocks = post_blocks(c->L);
  B_RC(batch_alloc(b, &p, (size_t)max_row_blocks * kAdmmStats * kp * sizeof(double))); b->admm_stats = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)b->post_blocks * kAdmmStats * kp * sizeof(double))); b->post_stats = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)max_row_blocks * kObjStats * kp * sizeof(double))); b->obj_stats = (double *)p;
  B_RC(batch_alloc(b, &p, (size_t)kp * kFinal * sizeof(double))); b->fin = (double *)p;
  B_HIP(hipHostMalloc((void **)&b->h_fin, (size_t)kp * kFinal * sizeof(double), hipHostMallocDefault));
  B_HIP(hipHostMalloc((void **)&b->h_fac, (size_t)kp * sizeof(double), hipHostMallocDefault));
  B_HIP(hipMemsetAsync(b->q, 0, (size_t)c->Np * kp * Tsz, b->stream));
  B_HIP(hipMemsetAsync(b->W, 0, (size_t)c->Np * kp * Tsz, b->stream));
  B_HIP(hipMemsetAsync(b->qs, 0, (size_t)c->n_sec * kp * sizeof(double), b->stream));
  B_HIP(hipMemsetAsync(b->q2, 0, (size_t)c->mAp * kp * sizeof(double), b->stream));
  B_HIP(hipStreamSynchronize(b->stream));
  if (!slots) B_RC(upload_tables(b, ld_mask));
#undef B_RC
#undef B_HIP
  *out = b;
  return LADMM_OK;
}

// Event pair around one launch when profiling (start if begin, else end).
int prof_mark(ladmm_batch *b, int kind, bool begin) {
  if (!b->profiling) return LADMM_OK;
  if (b->ev_used == b->ev_pool.size()) {
    hipEvent_t e;
    HIPC(hipEventCreate(&e));
    b->ev_pool.push_back(e);
  }
  if (begin) b->ev_kind.push_back(kind);
  HIPC(hipEventRecord(b->ev_pool[b->ev_used++], b->stream));
  return LADMM_OK;
}

// After the stream has completed: accumulate the recorded pairs.
int prof_collect(ladmm_batch *b) {
  for (size_t i = 0; i < b->ev_kind.size(); ++i) {
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, b->ev_pool[2 * i], b->ev_pool[2 * i + 1]));
    b->kms[b->ev_kind[i]] += ms;
    b->kcount[b->ev_kind[i]] += 1;
  }
  b->ev_kind.clear();
  b->ev_used = 0;
  return LADMM_OK;
}

#define PROF(kind, launch)                      \
  do {                                          \
    int rc_ = prof_mark(b, kind, true);         \
    if (rc_) return rc_;                        \
    HIPC(launch);                               \
    rc_ = prof_mark(b, kind, false);            \
    if (rc_) return rc_;                        \
  } while (0)

// One ADMM iteration; with `stats`, also the per-plan statistics after it.
template <typename T>
int iterate_once(ladmm_batch *b, bool stats) {
  ladmm_case *c = b->c;
  hipStream_t s = b->stream;
  const int kp = b->kp, kw = b->kact;   // leading dimension, launched columns
  PointTable<T> pt = point_table<T>(b);
  SmallArgs sa = small_args(b);
  PROF(0, (gemm_tn<T>(s, (const T *)c->D, c->ntp, (const T *)b->W, kp, (T *)b->P1, kp, c->ntp,
                      kw, c->Np, c->nchunk1, nullptr, b->cfg1)));
  PROF(1, (rhs<T>(s, sa, (const T *)b->P1, (size_t)c->ntp * kp, c->nchunk1, b->qs, b->q2, b->r)));
  PROF(2, (gemm_tn<double>(s, c->Sinv, c->mAp, b->r, kp, b->P2, kp, c->mAp, kw, c->mAp,
                           c->nchunk2, nullptr, b->cfg_s)));
  PROF(3, (vreduce<T>(s, sa, b->P2, (size_t)c->mAp * kp, c->nchunk2, b->v, (T *)b->vT)));
  PROF(3, (post(s, sa, b->v, b->qs, b->q2, stats ? b->post_stats : nullptr, &b->post_blocks)));
  EpiArgs<T> ea{};
  ea.q = (T *)b->q;
  ea.w = (T *)b->W;
  ea.ldq = kp;
  ea.invrho = b->invrho;
  ea.active = b->active;
  ea.stats = b->admm_stats;
  ea.nstat_cols = kp;
  ea.pt = pt;
  ea.alpha = b->alpha;
  PROF(4, (gemm_nn<T>(s, stats ? EPI_ADMM_STATS : EPI_ADMM, (const T *)c->D, c->ntp,
                      (const T *)b->vT, kp, c->Np, kw, c->ntp, ea, b->cfg2)));
  if (stats) {
    PROF(6, (shot_scaled<T>(s, sa, b->q2, (T *)b->that)));
    EpiArgs<T> eo = ea;
    eo.stats = b->obj_stats;
    PROF(5, (gemm_nn<T>(s, EPI_OBJ, (const T *)c->D, c->ntp, (const T *)b->that, kp, c->Np, kw,
                        c->ntp, eo, b->cfg2)));
    // certificate: z1 of the new iterate times the dose block (the GEMM1
    // partials are free until the next iteration)
    PROF(8, (z_from_q<T>(s, (const T *)b->q, (T *)b->zc, c->Np, kp, pt)));
    PROF(8, (gemm_tn<T>(s, (const T *)c->D, c->ntp, (const T *)b->zc, kp, (T *)b->P1, kp, c->ntp,
                        kw, c->Np, c->nchunk1, nullptr, b->cfg1)));
    PROF(8, (cert_need<T>(s, sa, (const T *)b->P1, (size_t)c->ntp * kp, c->nchunk1, b->need)));
    FinalArgs fa;
    fa.admm_stats = b->admm_stats;
    fa.admm_blocks = b->admm_blocks;
    fa.post_stats = b->post_stats;
    fa.post_blocks = b->post_blocks;
    fa.obj_stats = b->obj_stats;
    fa.obj_blocks = b->obj_blocks;
    fa.q2 = b->q2;
    fa.E = c->E;
    fa.invrho = b->invrho;
    fa.wbot = b->wbot;
    fa.L = c->L;
    fa.cs = c->cs;
    fa.kp = kp;
    fa.need = b->need;
    fa.out = b->fin;
    PROF(7, (finalize(s, fa)));
  }
  return LADMM_OK;
}

// Plan-major BF16 pairs stored in the space of a Np x kp (or ntp x kp) FP32
// buffer: hi rows first, then lo rows.
BfPair plan_pairs(void *buf, int kp, int len) {
  const uint16_t *h = (const uint16_t *)buf;
  return BfPair{h, h + (size_t)kp * len, len};
}

// Tile configuration of a three-term pair product (which: 0 split-K, 1
// point-row): LADMM_BF16 keeps its own for the refresh and the checks.
int cfg_pairs(const ladmm_batch *b, int which) {
  if (b->c->precision == LADMM_BF16) return which == 0 ? b->cfg1r : b->cfg2r;
  return which == 0 ? b->cfg1 : b->cfg2;
}

// The check after a pair-product iteration: the objective product of the
// current shot times (pairs) and the per-plan statistics.
int check_stats_bf(ladmm_batch *b, const EpiArgs<float> &ea) {
  ladmm_case *c = b->c;
  hipStream_t s = b->stream;
  const int kp = b->kp;
  const BfPair Dp{c->Dh, c->Dl, c->ntp};
  SmallArgs sa = small_args(b);
  const BfPair Tt = plan_pairs(b->that, kp, c->ntp);
  PROF(6, (shot_scaled_bf(s, sa, b->q2, (uint16_t *)Tt.hi, (uint16_t *)Tt.lo)));
  EpiArgs<float> eo = ea;
  eo.stats = b->obj_stats;
  PROF(5, (gemm_bf_nn(s, EPI_OBJ, Dp, Tt, c->Np, b->kact, c->ntp, eo, 3, cfg_pairs(b, 1))));
  // certificate: z1 of the new iterate (pairs) times the dose block
  const BfPair DT{c->DTh, c->DTl, c->Np};
  const BfPair Z = plan_pairs(b->zc, kp, c->Np);
  PROF(8, (z_from_q_bf(s, (const float *)b->q, c->Np, kp, ea.pt, (uint16_t *)Z.hi, (uint16_t *)Z.lo)));
  PROF(8, (gemm_bf_tn(s, DT, Z, (float *)b->P1, kp, c->ntp, b->kact, c->Np, c->nchunk1, 3,
                      cfg_pairs(b, 0))));
  PROF(8, (cert_need<float>(s, sa, (const float *)b->P1, (size_t)c->ntp * kp, c->nchunk1, b->need)));
  FinalArgs fa;
  fa.admm_stats = b->admm_stats;
  fa.admm_blocks = b->admm_blocks;
  fa.post_stats = b->post_stats;
  fa.post_blocks = b->post_blocks;
  fa.obj_stats = b->obj_stats;
  fa.obj_blocks = b->obj_blocks;
  fa.q2 = b->q2;
  fa.E = c->E;
  fa.invrho = b->invrho;
  fa.wbot = b->wbot;
  fa.L = c->L;
  fa.cs = c->cs;
  fa.kp = kp;
  fa.need = b->need;
  fa.out = b->fin;
  PROF(7, (finalize(s, fa)));
  return LADMM_OK;
}

// One iteration with the BF16-pair products (same steps as iterate_once).
int iterate_bf(ladmm_batch *b, bool stats) {
  ladmm_case *c = b->c;
  hipStream_t s = b->stream;
  const int kp = b->kp;
  const BfPair Dp{c->Dh, c->Dl, c->ntp}, DT{c->DTh, c->DTl, c->Np};
  const BfPair W = plan_pairs(b->W, kp, c->Np), V = plan_pairs(b->vT, kp, c->ntp);
  SmallArgs sa = small_args(b);
  const int kw = b->kact;
  PROF(0, (gemm_bf_tn(s, DT, W, (float *)b->P1, kp, c->ntp, kw, c->Np, c->nchunk1, 3, b->cfg1)));
  PROF(1, (rhs<float>(s, sa, (const float *)b->P1, (size_t)c->ntp * kp, c->nchunk1, b->qs, b->q2, b->r)));
  PROF(2, (gemm_tn<double>(s, c->Sinv, c->mAp, b->r, kp, b->P2, kp, c->mAp, kw, c->mAp,
                           c->nchunk2, nullptr, b->cfg_s)));
  PROF(3, (vreduce_bf(s, sa, b->P2, (size_t)c->mAp * kp, c->nchunk2, b->v, (uint16_t *)V.hi,
                      (uint16_t *)V.lo)));
  PROF(3, (post(s, sa, b->v, b->qs, b->q2, stats ? b->post_stats : nullptr, &b->post_blocks)));
  EpiArgs<float> ea{};
  ea.q = (float *)b->q;
  ea.ldq = kp;
  ea.invrho = b->invrho;
  ea.active = b->active;
  ea.stats = b->admm_stats;
  ea.nstat_cols = kp;
  ea.pt = point_table<float>(b);
  ea.wt_hi = (uint16_t *)W.hi;
  ea.wt_lo = (uint16_t *)W.lo;
  ea.ldwt = c->Np;
  ea.alpha = b->alpha;
  PROF(4, (gemm_bf_nn(s, stats ? EPI_ADMM_STATS : EPI_ADMM, Dp, V, c->Np, kw, c->ntp, ea, 3, b->cfg2)));
  if (stats) return check_stats_bf(b, ea);
  return LADMM_OK;
}

// One iteration of the refinement mode (LADMM_BF16).  phase BF_DELTA: single
int iterate_bfr(ladmm_batch *b, int phase) {
  ladmm_case *c = b->c;
  if (phase == BF_PLAIN) return iterate_bf(b, false);
  hipStream_t s = b->stream;
  const int kp = b->kp;
  const bool refresh = phase == BF_REFRESH;
  const BfPair Dp{c->Dh, c->Dl, c->ntp}, DT{c->DTh, c->DTl, c->Np};
  const BfPair W = plan_pairs(b->W, kp, c->Np), V = plan_pairs(b->vT, kp, c->ntp);
  const BfPair dW{b->dW, nullptr, c->Np}, dV{V.hi, nullptr, c->ntp};
  SmallArgs sa = small_args(b);
  const int kw = b->kact;
  if (refresh)
    PROF(9, (gemm_bf_tn(s, DT, W, (float *)b->P1, kp, c->ntp, kw, c->Np, c->nchunk1, 3, b->cfg1r)));
  else
    PROF(0, (gemm_bf_tn(s, DT, dW, (float *)b->P1, kp, c->ntp, kw, c->Np, c->nchunk1, 1, b->cfg1)));
  // S^-1 r refined like the dose products: the refresh multiplies r by the FP64
  // inverse and records (r, v) for the running plans; a hot iteration adds the
  // FP32 product of the FP32 inverse with r - r_ref to that v (S^-1 is linear,
  // so any recorded pair gives S^-1 r; FP32 rounds only the change)
  PROF(1, (rhs<float>(s, sa, (const float *)b->P1, (size_t)c->ntp * kp, c->nchunk1, b->qs, b->q2, b->r,
                      refresh ? nullptr : b->gref, refresh ? b->gref : nullptr,
                      refresh ? b->rref : nullptr, refresh ? nullptr : b->rref,
                      refresh ? nullptr : b->r32)));
  if (refresh) {
    PROF(2, (gemm_tn<double>(s, c->Sinv, c->mAp, b->r, kp, b->P2, kp, c->mAp, kw, c->mAp,
                             c->nchunk2, nullptr, b->cfg_s)));
    PROF(3, (vreduce_bf(s, sa, b->P2, (size_t)c->mAp * kp, c->nchunk2, b->v, (uint16_t *)V.hi,
                        (uint16_t *)V.lo, b->vref, b->vfull)));
  } else {
    PROF(2, (gemm_tn<float>(s, c->Sinv32, c->mAp, b->r32, kp, (float *)b->P2, kp, c->mAp, kw, c->mAp,
                            c->nchunk2, nullptr, b->cfg_s)));
    PROF(3, (vreduce_delta_bf(s, sa, (const float *)b->P2, (size_t)c->mAp * kp, c->nchunk2, b->vfull,
                              b->v, b->vref, (uint16_t *)V.hi)));
  }
  PROF(3, (post(s, sa, b->v, b->qs, b->q2, refresh ? b->post_stats : nullptr, &b->post_blocks)));
  EpiArgs<float> ea{};
  ea.q = (float *)b->q;
  ea.ldq = kp;
  ea.invrho = b->invrho;
  ea.active = b->active;
  ea.stats = b->admm_stats;
  ea.nstat_cols = kp;
  ea.pt = point_table<float>(b);
  ea.wt_hi = (uint16_t *)W.hi;
  ea.wt_lo = (uint16_t *)W.lo;
  ea.ldwt = c->Np;
  ea.alpha = b->alpha;
  ea.xref = b->xref;
  ea.wref = b->wref;
  ea.dw = b->dW;
  if (refresh)
    PROF(10, (gemm_bf_nn(s, EPI_ADMM_STATS, Dp, V, c->Np, kw, c->ntp, ea, 3, b->cfg2r, BF_REFRESH)));
  else
    PROF(4, (gemm_bf_nn(s, EPI_ADMM, Dp, dV, c->Np, kw, c->ntp, ea, 1, b->cfg2, phase)));
  if (refresh) return check_stats_bf(b, ea);
  return LADMM_OK;
}

// Iteration i of a chunk of n (the last one with statistics).
int iterate_any(ladmm_batch *b, int i, int n) {
  const bool stats = i == n - 1;
  switch (b->c->precision) {
    case LADMM_F64: return iterate_once<double>(b, stats);
    case LADMM_F32: return iterate_once<float>(b, stats);
    case LADMM_BF16:
      return iterate_bfr(b, stats ? BF_REFRESH : i == n - 2 ? BF_DELTA_PAIR : BF_DELTA);
    default: return iterate_bf(b, stats);
  }
}

// Number of GEMM2 statistics partials (one per 32-row block, every configuration).
void set_row_blocks(ladmm_batch *b) { b->admm_blocks = b->obj_blocks = b->c->Np / kNnStatRows; }

// Pick the fastest tile configuration of each dose-matrix product for this
// case and plan count: a few timed launches of every valid configuration on the
// live batch (GEMM2 runs with its writes masked off).  Results are cached per
// case and padded plan count.  The configurations change only the work split,
// never the order of the sums, so the choice does not affect the iterates.
// Whether tile configuration cfg suits the split-K (which = 0) or the
// point-row (which = 1) product of this batch's shapes.
bool cfg_ok(const ladmm_batch *b, int which, int cfg, int terms) {
  const ladmm_case *c = b->c;
  if (bf16_block(c->precision))
    return which == 0 ? gemm_bf_cfg_ok(0, cfg, c->ntp, b->kact, terms)
                      : gemm_bf_cfg_ok(1, cfg, c->Np, b->kact, terms);
  return which == 0 ? gemm_tn_cfg_ok(cfg, c->ntp, b->kact) : gemm_nn_cfg_ok(cfg, c->Np, b->kact);
}

// One launch of a dose-matrix product in configuration cfg (the point-row
// product with its writes masked off by `noact`).
template <typename T>
// Pick the fastest tile configuration of each dose-matrix product for this
// case and plan count: a few timed launches of every valid configuration on the
// live batch (GEMM2 runs with its writes masked off).  Results are cached per
// case and padded plan count.  The configurations change only the work split,
// never the order of the sums, so the choice does not affect the iterates.
// Whether tile configuration cfg suits the split-K (which = 0) or the
// point-row (which = 1) product of this batch's shapes.
bool cfg_ok(const ladmm_batch *b, int which, int cfg, int terms) {
  const ladmm_case *c = b->c;
  if (bf16_block(c->precision))
    return which == 0 ? gemm_bf_cfg_ok(0, cfg, c->ntp, b->kact, terms)
                      : gemm_bf_cfg_ok(1, cfg, c->Np, b->kact, terms);
  return which == 0 ? gemm_tn_cfg_ok(cfg, c->ntp, b->kact) : gemm_nn_cfg_ok(cfg, c->Np, b->kact);
}

// One launch of a dose-matrix product in configuration cfg (the point-row
// product with its writes masked off by `noact`).
template <typename T>
hipError_t tune_launch(ladmm_batch *b, int which, int cfg, const int32_t *noact, int terms) {
  ladmm_case *c = b->c;
  hipStream_t s = b->stream;
  const int kp = b->kp;
  if (bf16_block(c->precision)) {
    // LADMM_BF16's hot iterations: single-operand products; its refresh and
    // LADMM_BF16X3: pair products
    const bool one = terms == 1;
    const BfPair Dp{c->Dh, c->Dl, c->ntp}, DT{c->DTh, c->DTl, c->Np};
    if (which == 0)
      return gemm_bf_tn(s, DT, one ? BfPair{b->dW, nullptr, c->Np} : plan_pairs(b->W, kp, c->Np),
                        (float *)b->P1, kp, c->ntp, kp, c->Np, c->nchunk1, one ? 1 : 3, cfg);
    EpiArgs<float> ea{};
    ea.q = (float *)b->q;
    ea.ldq = kp;
    ea.invrho = b->invrho;
    ea.active = noact;
    ea.pt = point_table<float>(b);
    ea.wt_hi = (uint16_t *)b->W;
    ea.wt_lo = (uint16_t *)b->W + (size_t)kp * c->Np;
    ea.ldwt = c->Np;
    ea.alpha = b->alpha;
    ea.xref = b->xref;
    ea.wref = b->wref;
    ea.dw = b->dW;
    const BfPair V = plan_pairs(b->vT, kp, c->ntp);
    return gemm_bf_nn(s, EPI_ADMM, Dp, one ? BfPair{V.hi, nullptr, c->ntp} : V, c->Np, kp, c->ntp, ea,
                      one ? 1 : 3, cfg, one ? BF_DELTA : BF_PLAIN);
  }
  if (which == 0)
    return gemm_tn<T>(s, (const T *)c->D, c->ntp, (const T *)b->W, kp, (T *)b->P1, kp, c->ntp, kp,
                      c->Np, c->nchunk1, nullptr, cfg);
  EpiArgs<T> ea{};
  ea.q = (T *)b->q;
  ea.w = (T *)b->W;
  ea.ldq = kp;
  ea.invrho = b->invrho;
  ea.active = noact;
  ea.pt = point_table<T>(b);
  ea.alpha = b->alpha;
  return gemm_nn<T>(s, EPI_ADMM, (const T *)c->D, c->ntp, (const T *)b->vT, kp, c->Np, kp, c->ntp,
                    ea, cfg);
}

// Pick the fastest tile configuration of each dose-matrix product for this
// case and launched width: a few timed launches of every valid configuration on
// the live batch (the point-row product runs with its writes masked off).
// Results are cached per case and launched width (the padded plan count, or a
// compacted width).  The configurations change only the work split, never the
// order of the sums, so the choice does not affect the iterates.
template <typename T>
int autotune(ladmm_batch *b) {
  ladmm_case *c = b->c;
  for (auto &e : c->tuned)
    if (e.kp == b->kact) {
      b->cfg1 = e.cfg1;
      b->cfg2 = e.cfg2;
      b->cfg_s = e.cfg_s;
      b->cfg1r = e.cfg1r;
      b->cfg2r = e.cfg2r;
      b->tuned = true;
      set_row_blocks(b);
      return LADMM_OK;
    }
  hipStream_t s = b->stream;
  const int kp = b->kp;
  int32_t *noact = nullptr;
  HIPC(hipMalloc((void **)&noact, kp * sizeof(int32_t)));
  hipError_t e = hipMemsetAsync(noact, 0, kp * sizeof(int32_t), s);
  // the hot products; LADMM_BF16 also times its refresh's pair products
  const int hot_terms = c->precision == LADMM_BF16 ? 1 : 3;
  for (int pass = 0; pass < (c->precision == LADMM_BF16 ? 2 : 1) && e == hipSuccess; ++pass) {
    const int terms = pass == 0 ? hot_terms : 3;
    float best1 = 1e30f, best2 = 1e30f;
    int *c1 = pass == 0 ? &b->cfg1 : &b->cfg1r, *c2 = pass == 0 ? &b->cfg2 : &b->cfg2r;
    for (int cfg = 0; cfg < kMaxGemmCfgs && e == hipSuccess; ++cfg) {
      for (int which = 0; which < 2 && e == hipSuccess; ++which) {
        if (!cfg_ok(b, which, cfg, terms)) continue;
        float tot = 0.f;
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
          e = hipEventRecord(b->ev0, s);
          if (e == hipSuccess) e = tune_launch<T>(b, which, cfg, noact, terms);
          if (e == hipSuccess) e = hipEventRecord(b->ev1, s);
          if (e == hipSuccess) e = hipEventSynchronize(b->ev1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev0, b->ev1);
          if (rep > 0) tot += ms;     // the first launch warms caches
        }
        if (which == 0 && tot < best1) { best1 = tot; *c1 = cfg; }
        if (which == 1 && tot < best2) { best2 = tot; *c2 = cfg; }
      }
    }
  }
  hipFree(noact);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  // the S^-1 r product (it writes only its split partials; LADMM_BF16 tunes its
  // hot iterations' FP32 product, the FP64 one runs once per chunk)
  float best_s = 1e30f;
  for (int cfg = 0; cfg < kGemmCfgs && e == hipSuccess; ++cfg) {
    if (!gemm_tn_cfg_ok(cfg, c->mAp, b->kact)) continue;
    float tot = 0.f;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      e = hipEventRecord(b->ev0, s);
      if (e == hipSuccess && c->Sinv32 != nullptr)
        e = gemm_tn<float>(s, c->Sinv32, c->mAp, b->r32, kp, (float *)b->P2, kp, c->mAp, b->kact,
                           c->mAp, c->nchunk2, nullptr, cfg);
      else if (e == hipSuccess)
        e = gemm_tn<double>(s, c->Sinv, c->mAp, b->r, kp, b->P2, kp, c->mAp, b->kact, c->mAp,
                            c->nchunk2, nullptr, cfg);
      if (e == hipSuccess) e = hipEventRecord(b->ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(b->ev1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, b->ev0, b->ev1);
      if (rep > 0) tot += ms;
    }
    if (tot < best_s) { best_s = tot; b->cfg_s = cfg; }
  }
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
  c->tuned.push_back({b->kact, b->cfg1, b->cfg2, b->cfg_s, b->cfg1r, b->cfg2r});
  b->tuned = true;
  set_row_blocks(b);
  return LADMM_OK;
}

int prepare_batch(ladmm_batch *b) {
  if (b->tuned) return LADMM_OK;
  if (b->opts.autotune) return b->c->precision == LADMM_F64 ? autotune<double>(b) : autotune<float>(b);
  b->tuned = true;
  set_row_blocks(b);
  return LADMM_OK;
}

// Enqueue n iterations (the last with statistics).  Outside profiling the
// launches are captured once into a HIP graph and replayed: every kernel
// argument is a pointer or a size fixed for the batch's life except the tile
// configurations, which key the graph together with n.  Frozen plans, new
// step sizes and new slots change only device memory the kernels read.
int enqueue_iterations(ladmm_batch *b, int n) {
  if (b->profiling || !b->graphs) {
    for (int i = 0; i < n; ++i) {
      int rc = iterate_any(b, i, n);
      if (rc) return rc;
    }
    return LADMM_OK;
  }
  hipGraphExec_t exec = nullptr;
  for (const auto &g : b->graph_cache)
    if (g.n == n && g.kact == b->kact && g.cfg1 == b->cfg1 && g.cfg2 == b->cfg2 &&
        g.cfg_s == b->cfg_s && g.cfg1r == b->cfg1r && g.cfg2r == b->cfg2r)
      exec = g.exec;
  if (!exec) {
    if (!b->cap_stream) HIPC(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    // the launches below go to the capture stream; the graph runs on b->stream
    const hipStream_t run_stream = b->stream;
    b->stream = b->cap_stream;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      b->stream = run_stream;
      return fail(LADMM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    }
    int rc = LADMM_OK;
    for (int i = 0; i < n && rc == LADMM_OK; ++i) rc = iterate_any(b, i, n);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(b->stream, &graph);
    b->stream = run_stream;
    if (rc == LADMM_OK && e != hipSuccess)
      rc = fail(LADMM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    if (rc == LADMM_OK) {
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) rc = fail(LADMM_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    if (graph) hipGraphDestroy(graph);
    if (rc) return rc;
    // a handful of chunk lengths and compacted widths per batch; keep the
    // eight most recent
    if (b->graph_cache.size() == 8) {
      hipGraphExecDestroy(b->graph_cache.front().exec);
      b->graph_cache.erase(b->graph_cache.begin());
    }
    b->graph_cache.push_back({n, b->kact, b->cfg1, b->cfg2, b->cfg_s, b->cfg1r, b->cfg2r, exec});
  }
  HIPC(hipGraphLaunch(exec, b->stream));
  return LADMM_OK;
}

int chunk_launch(ladmm_batch *b, int n) {
  b->chunk_active = 0;
  for (int j = 0; j < b->k; ++j) b->chunk_active += b->h_active[j] != 0;
  HIPC(hipEventRecord(b->ev0, b->stream));
  int rc = enqueue_iterations(b, n);
  if (rc) return rc;
  HIPC(hipEventRecord(b->ev1, b->stream));
  HIPC(hipMemcpyAsync(b->h_fin, b->fin, (size_t)b->kp * kFinal * sizeof(double),
                      hipMemcpyDeviceToHost, b->stream));
  return LADMM_OK;
}

int chunk_complete(ladmm_batch *b, int n, bool decide, bool *changed_out) {
  HIPC(hipStreamSynchronize(b->stream));
  {
    int rc = prof_collect(b);
    if (rc) return rc;
  }
  float ms = 0.f;
  HIPC(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->iterate_ms += ms;
  b->plan_iters += (int64_t)n * b->chunk_active;
  b->iters_run += n;
  bool changed = false;
  for (int j = 0; j < b->k; ++j) {
    if (!b->h_active[j]) continue;
    const double *f = b->h_fin + (size_t)j * kFinal;
    std::memcpy(&b->rec[(size_t)j * kFinal], f, kFinal * sizeof(double));
    b->iters[j] = b->iters_run - b->start[j];
    bool bad = false;
    for (int q = 0; q < 8; ++q) bad |= !std::isfinite(f[q]);   // the certificate may be undefined
    if (bad) {
      b->status[j] = LADMM_PLAN_NUMERIC;
      b->h_active[j] = 0;
      changed = true;
      continue;
    }
    if (!decide) continue;
    const StopRule &r = b->rule[j];
    if (rule_met(r, f)) {
      b->status[j] = LADMM_PLAN_CONVERGED;
      b->h_active[j] = 0;
      changed = true;
    } else if (b->iters[j] >= r.max_iter) {
      b->status[j] = LADMM_PLAN_MAX_ITER;
      b->h_active[j] = 0;
      changed = true;
    }
  }
  if (changed_out) *changed_out = changed;
  return LADMM_OK;
}

int adapt_rho(ladmm_batch *b, bool *switched) {
  ladmm_case *c = b->c;
  bool any = false;
  for (int j = 0; j < b->kp; ++j) b->h_fac[j] = 1.0;
  for (int j = 0; j < b->k; ++j) {
    const StopRule &r = b->rule[j];
    if (!b->h_active[j] || !r.adapt) continue;
    const double rp = b->rec[(size_t)j * kFinal + 3], rd = b->rec[(size_t)j * kFinal + 4];
    double nr = b->rho[j];
    if (rp > r.mu * rd) nr *= r.tau;
    else if (rd > r.mu * rp) nr /= r.tau;
    nr = std::min(std::max(nr, r.rho_lo), r.rho_hi);
    if (nr == b->rho[j]) continue;
    b->h_fac[j] = b->rho[j] / nr;
    b->rho[j] = nr;
    any = true;
  }
  if (switched) *switched = any;
  if (!any) return LADMM_OK;
  hipStream_t s = b->stream;
  HIPC(hipMemcpyAsync(b->fac, b->h_fac, b->kp * sizeof(double), hipMemcpyHostToDevice, s));
  SmallArgs sa = small_args(b);
  HIPC(rescale_small(s, sa, b->q2, b->qs, b->invrho, b->fac));
  if (c->precision == LADMM_F64) {
    HIPC(rescale_points<double>(s, (double *)b->q, c->Np, b->kp, point_table<double>(b), b->fac));
    HIPC(w_from_q<double>(s, (const double *)b->q, (double *)b->W, c->Np, b->kp, point_table<double>(b)));
  } else {
    HIPC(rescale_points<float>(s, (float *)b->q, c->Np, b->kp, point_table<float>(b), b->fac));
    if (c->precision == LADMM_F32)
      HIPC(w_from_q<float>(s, (const float *)b->q, (float *)b->W, c->Np, b->kp, point_table<float>(b)));
    else
      HIPC(w_from_q_bf(s, (const float *)b->q, c->Np, b->kp, point_table<float>(b), (uint16_t *)b->W,
                       (uint16_t *)b->W + (size_t)b->kp * c->Np, b->wref, b->dW));
  }
  return LADMM_OK;
}

// Permute the plan columns of a batch: column c takes the plan held in column
// src[c] (src is a permutation of [0, k); padding columns stay), with all of
// its device state (iterates, references of the refinement, bounds, step
// sizes, masks) and host records.  Every kernel computes a plan's column from
// that column's data only, in an order that does not depend on the column, so
// a plan's arithmetic is the same in any column.
int permute_columns(ladmm_batch *b, const std::vector<int> &src_k) {
  ladmm_case *c = b->c;
  hipStream_t s = b->stream;
  const int kp = b->kp, k = b->k;
  std::vector<int> src(kp);
  for (int j = 0; j < kp; ++j) src[j] = j < k ? src_k[j] : j;
  const size_t Tsz = c->precision == LADMM_F64 ? sizeof(double) : sizeof(float);
  // arrays: (pointer, rows, element bytes, plan-major rows?)
  struct Arr { void *p; size_t rows; int bytes; bool plan_rows; };
  std::vector<Arr> arrs = {
      {b->q, (size_t)c->Np, (int)Tsz, false},
      {b->qs, (size_t)c->n_sec, 8, false},
      {b->q2, (size_t)c->mAp, 8, false},
      {b->utab, (size_t)(c->G + 1), (int)Tsz, false},
      {b->invrho, 1, 8, false},
      {b->wbot, 1, 8, false},
      {b->bbot, (size_t)c->n_iso, 8, false},
      {b->active, 1, 4, false}};
  if (bf16_block(c->precision)) {
    // W' pairs: kp hi rows, then kp lo rows, of Np values each
    arrs.push_back({b->W, (size_t)c->Np, 2, true});
    arrs.push_back({(uint16_t *)b->W + (size_t)kp * c->Np, (size_t)c->Np, 2, true});
  } else {
    arrs.push_back({b->W, (size_t)c->Np, (int)Tsz, false});
  }
  if (c->precision == LADMM_BF16) {
    arrs.push_back({b->xref, (size_t)c->Np, 4, false});
    arrs.push_back({b->wref, (size_t)c->Np, 4, false});
    arrs.push_back({b->gref, (size_t)c->ntp, 8, false});
    arrs.push_back({b->vref, (size_t)c->ntp, 8, false});
    arrs.push_back({b->rref, (size_t)c->mAp, 8, false});
    arrs.push_back({b->vfull, (size_t)c->mAp, 8, false});
    arrs.push_back({b->dW, (size_t)c->Np, 2, true});
  }
  if (b->mask) arrs.push_back({b->mask, (size_t)b->mask_words, 8, true});
  size_t need = 0;
  for (const Arr &a : arrs) need = std::max(need, a.rows * (size_t)kp * a.bytes);
  if (need > b->perm_tmp_bytes) {
    void *p = nullptr;
    int rc = batch_alloc(b, &p, need);
    if (rc) return rc;
    b->perm_tmp = p;
    b->perm_tmp_bytes = need;
  }
  HIPC(hipMemcpyAsync(b->perm_d, src.data(), kp * sizeof(int), hipMemcpyHostToDevice, s));
  for (const Arr &a : arrs) {
    const size_t bytes = a.rows * (size_t)kp * a.bytes;
    if (a.plan_rows)
      HIPC(gather_rows(s, a.p, b->perm_tmp, kp, a.rows, a.bytes, b->perm_d));
    else
      HIPC(gather_cols(s, a.p, b->perm_tmp, a.rows, kp, a.bytes, b->perm_d));
    HIPC(hipMemcpyAsync(a.p, b->perm_tmp, bytes, hipMemcpyDeviceToDevice, s));
  }
  HIPC(hipStreamSynchronize(s));
  // host records of the columns
  auto perm = [&](auto &v) {
    auto old = v;
    for (int j = 0; j < k; ++j) v[j] = old[src[j]];
  };
  perm(b->w);
  perm(b->rho);
  perm(b->status);
  perm(b->iters);
  perm(b->start);
  perm(b->rule);
  perm(b->plan_at);
  {
    std::vector<int32_t> old(b->h_active.begin(), b->h_active.begin() + k);
    for (int j = 0; j < k; ++j) b->h_active[j] = old[src[j]];
  }
  {
    std::vector<double> old = b->rec;
    for (int j = 0; j < k; ++j)
      std::memcpy(&b->rec[(size_t)j * kFinal], &old[(size_t)src[j] * kFinal], kFinal * sizeof(double));
  }
  return LADMM_OK;
}

// Launched width for n running plans: the smallest multiple of 32 (every
// product's column granule) that holds them and, for the BF16 blocks, also
// admits one of their wider column tiles (64, 96 or 224 columns; widths with
// only the 32-column tile are skipped), never above kp.
int launch_width(const ladmm_batch *b, int n) {
  const bool bf = bf16_block(b->c->precision);
  for (int w = round_up(std::max(n, 1), 32); w < b->kp; w += 32)
    if (!bf || w % 64 == 0 || w % 96 == 0 || w % 224 == 0) return w;
  return b->kp;
}

// Between check chunks of a run: move the running plans to the lowest columns
// when that lets the dose-matrix products launch fewer columns.
int compact(ladmm_batch *b) {
  const int k = b->k;
  int n = 0;
  for (int j = 0; j < k; ++j) n += b->h_active[j] != 0;
  if (n == 0) return LADMM_OK;
  const int w = launch_width(b, n);
  if (w >= b->kact) return LADMM_OK;
  std::vector<int> src;
  src.reserve(k);
  for (int j = 0; j < k; ++j)
    if (b->h_active[j]) src.push_back(j);
  for (int j = 0; j < k; ++j)
    if (!b->h_active[j]) src.push_back(j);
  int rc = permute_columns(b, src);
  if (rc) return rc;
  b->kact = w;
  if (b->opts.autotune) b->tuned = false;   // tile configurations for the new width (cached)
  return LADMM_OK;
}

// After a run: every plan back in its own column, all columns launched.
int uncompact(ladmm_batch *b) {
  const int k = b->k;
  bool ident = true;
  for (int j = 0; j < k; ++j) ident &= b->plan_at[j] == j;
  if (!ident) {
    std::vector<int> src(k);
    for (int j = 0; j < k; ++j) src[b->plan_at[j]] = j;
    int rc = permute_columns(b, src);
    if (rc) return rc;
  }
  if (b->kact != b->kp) {
    b->kact = b->kp;
    if (b->opts.autotune) b->tuned = false;
  }
  return LADMM_OK;
}

// Run n iterations (the last one with statistics), update the host records and,
// if `decide`, freeze plans that meet their stopping rule and, after a full
// check chunk, balance the step sizes of the plans that ask for it.
int run_chunk(ladmm_batch *b, int n, bool decide) {
  if (n <= 0) return LADMM_OK;
  int rc = prepare_batch(b);
  if (rc) return rc;
  rc = chunk_launch(b, n);
  if (rc) return rc;
  bool changed = false;
  rc = chunk_complete(b, n, decide, &changed);
  if (rc) return rc;
  if (decide && n == b->opts.check_every) {
    rc = adapt_rho(b, nullptr);
    if (rc) return rc;
  }
  if (changed)
    HIPC(hipMemcpy(b->active, b->h_active.data(), b->kp * sizeof(int32_t), hipMemcpyHostToDevice));
  return LADMM_OK;
}

// Run check chunks until every plan has stopped or max_iter is reached, or
// until max_checks chunks have run (max_checks <= 0: no limit).  The running
// plans are compacted between chunks and return to their own columns before
// this returns.  *running (optional): plans still running.
int run_impl(ladmm_batch *b, int max_checks = 0, int32_t *running = nullptr) {
  HIPC(hipSetDevice(b->c->ctx->device));
  const int every = b->opts.check_every;
  int checks = 0;
  auto count_running = [&]() {
    int n = 0;
    for (int j = 0; j < b->k; ++j) n += b->h_active[j] != 0;
    return n;
  };
  while (b->iters_run < b->opts.max_iter && count_running() > 0 &&
         (max_checks <= 0 || checks < max_checks)) {
    const int n = std::min(every, b->opts.max_iter - b->iters_run);
    int rc = run_chunk(b, n, true);
    if (rc) return rc;
    ++checks;
    if (b->compact) {
      rc = compact(b);
      if (rc) return rc;
    }
  }
  int rc = uncompact(b);
  if (rc) return rc;
  const bool done = b->iters_run >= b->opts.max_iter || count_running() == 0;
  if (done) {
    for (int j = 0; j < b->k; ++j)
      if (b->status[j] == LADMM_PLAN_RUNNING) {
        b->status[j] = LADMM_PLAN_MAX_ITER;
        b->h_active[j] = 0;
      }
  }
  if (running) *running = done ? 0 : count_running();
  return LADMM_OK;
}

void bot_from_t(const ladmm_case *c, const double *t, double *bot) {
  for (int i = 0; i < c->n_iso; ++i) {
    double best = 0.0;
    for (int s = 0; s < c->S; ++s) {
      double sec = 0.0;
      for (int cc = 0; cc < c->C; ++cc) sec += t[(i * c->S + s) * c->C + cc];
      best = std::max(best, sec);
    }
    bot[i] = c->cs * best;
  }
}

int results_impl(ladmm_batch *b, ladmm_result *out) {
  if (!out) return fail(LADMM_E_INVALID, "null result");
  ladmm_case *c = b->c;
  const int k = b->k;
  if (out->t || out->bot) {
    double *dt = nullptr;
    HIPC(hipMalloc((void **)&dt, (size_t)k * c->n_t * sizeof(double)));
    SmallArgs sa = small_args(b);
    hipError_t e = extract_t(b->stream, sa, b->q2, dt, k);
    std::vector<double> ht((size_t)k * c->n_t);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ht.data(), dt, ht.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    hipFree(dt);
    if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("extract: ") + hipGetErrorString(e));
    if (out->t) std::memcpy(out->t, ht.data(), ht.size() * sizeof(double));
    if (out->bot)
      for (int j = 0; j < k; ++j) bot_from_t(c, &ht[(size_t)j * c->n_t], out->bot + (size_t)j * c->n_iso);
  }
  for (int j = 0; j < k; ++j) {
    const double *f = &b->rec[(size_t)j * kFinal];
    if (out->objective) out->objective[j] = f[0];
    if (out->dual_obj) out->dual_obj[j] = f[1];
    if (out->rel_gap) out->rel_gap[j] = f[2];
    if (out->r_pri) out->r_pri[j] = f[3];
    if (out->r_dual) out->r_dual[j] = f[4];
    if (out->iters) out->iters[j] = b->iters[j];
    if (out->plan_status) out->plan_status[j] = b->status[j];
    if (out->lower_bound) out->lower_bound[j] = f[8];
    if (out->cert_gap) out->cert_gap[j] = f[9];
  }
  return LADMM_OK;
}

}  // namespace ladmm

// ---------------------------------------------------------------------------
// exported entry points
// ---------------------------------------------------------------------------
extern "C" {

const char *ladmm_last_error(void) { return g_err.c_str(); }
const char *ladmm_version(void) { return "ladmm 0.1 gfx950"; }

int ladmm_ctx_create(int device, size_t hbm_budget_bytes, ladmm_ctx **out) {
  if (!out) return fail(LADMM_E_INVALID, "null out");
  int n = 0;
  HIPC(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(LADMM_E_INVALID, "no such device");
  HIPC(hipSetDevice(device));
  ladmm_ctx *c = new ladmm_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return LADMM_OK;
}

int ladmm_ctx_destroy(ladmm_ctx *ctx) {
  if (!ctx) return LADMM_OK;
  bool now;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->destroyed = true;
    now = ctx->refs == 0;
  }
  if (now) delete ctx;   // otherwise freed with its last case
  return LADMM_OK;
}

size_t ladmm_ctx_used_bytes(const ladmm_ctx *ctx) { return ctx ? ctx->used : 0; }

int ladmm_create_case(ladmm_ctx *ctx, const ladmm_case_desc *desc, ladmm_case **out) {
  try {
    return create_case_impl(ctx, desc, out);
  } catch (const std::exception &e) {
    return fail(LADMM_E_NOMEM, e.what());
  }
}

int ladmm_destroy_case(ladmm_case *c) {
  if (!c) return LADMM_OK;
  bool now;
  {
    std::lock_guard<std::mutex> lk(c->ctx->mu);
    c->destroyed = true;
    now = c->refs == 0;
  }
  if (now) case_free(c);   // otherwise freed with its last batch
  return LADMM_OK;
}

int ladmm_case_scaling(const ladmm_case *c, double *E, double *beta) {
  if (!c) return fail(LADMM_E_STATE, "null case");
  if (E) {
    for (int t = 0; t < c->n_t; ++t) E[t] = c->hE[t];
    for (int i = 0; i < c->n_iso; ++i) E[c->n_t + i] = c->hE[c->ntp + i];
  }
  if (beta) *beta = c->beta;
  return LADMM_OK;
}

int ladmm_case_schur(const ladmm_case *c, double *S, double *S_inv) {
  if (!c) return fail(LADMM_E_STATE, "null case");
  HIPC(hipSetDevice(c->ctx->device));
  const int mA = c->n_t + c->n_iso;
  std::vector<double> h((size_t)c->mAp * c->mAp);
  auto idx = [&](int a) { return a < c->n_t ? a : c->ntp + (a - c->n_t); };
  for (int w = 0; w < 2; ++w) {
    double *dst = w == 0 ? S : S_inv;
    if (!dst) continue;
    HIPC(hipMemcpy(h.data(), w == 0 ? c->Smat : c->Sinv, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int a = 0; a < mA; ++a)
      for (int bb = 0; bb < mA; ++bb) dst[(size_t)a * mA + bb] = h[(size_t)idx(a) * c->mAp + idx(bb)];
  }
  return LADMM_OK;
}

double ladmm_case_setup_ms(const ladmm_case *c) { return c ? c->setup_ms : 0.0; }

int ladmm_batch_create(ladmm_case *c, int32_t k, const ladmm_weights *w, const uint64_t *ld_mask,
                       const double *rho, const ladmm_opts *opts, ladmm_batch **out) {
  try {
    return create_batch_impl(c, k, w, ld_mask, rho, opts, out);
  } catch (const std::exception &e) {
    return fail(LADMM_E_NOMEM, e.what());
  }
}

int ladmm_batch_destroy(ladmm_batch *b) { return destroy_batch_impl(b); }

int ladmm_batch_iterate(ladmm_batch *b, int32_t iters) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (iters < 0) return fail(LADMM_E_INVALID, "iters must be >= 0");
  HIPC(hipSetDevice(b->c->ctx->device));
  return run_chunk(b, iters, false);
}

int ladmm_batch_run(ladmm_batch *b) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  return run_impl(b);
}

int ladmm_batch_run_checks(ladmm_batch *b, int32_t max_checks, int32_t *running) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (max_checks < 1) return fail(LADMM_E_INVALID, "max_checks must be >= 1");
  return run_impl(b, max_checks, running);
}

int ladmm_batch_results(ladmm_batch *b, ladmm_result *out) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  HIPC(hipSetDevice(b->c->ctx->device));
  return results_impl(b, out);
}

int ladmm_batch_export(ladmm_batch *b, double *z1, double *y1, double *z2, double *y2) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  ladmm_case *c = b->c;
  HIPC(hipSetDevice(c->ctx->device));
  const int k = b->k, kp = b->kp, N = c->N, nA = N + c->n_sec, mA = c->n_t + c->n_iso;
  std::vector<double> hz((size_t)N * k), hy((size_t)N * k);
  double *dz = nullptr, *dy = nullptr;
  HIPC(hipMalloc((void **)&dz, hz.size() * sizeof(double)));
  hipError_t e = hipMalloc((void **)&dy, hy.size() * sizeof(double));
  if (e == hipSuccess) {
    if (c->precision == LADMM_F64)
      e = export_points<double>(b->stream, (const double *)b->q, kp, point_table<double>(b), N, k, dz, dy);
    else
      e = export_points<float>(b->stream, (const float *)b->q, kp, point_table<float>(b), N, k, dz, dy);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hz.data(), dz, hz.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), dy, hy.size() * sizeof(double), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  hipFree(dz);
  if (dy) hipFree(dy);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("export: ") + hipGetErrorString(e));
  std::vector<double> qs((size_t)c->n_sec * kp), q2((size_t)c->mAp * kp), bb((size_t)c->n_iso * kp);
  HIPC(hipMemcpy(qs.data(), b->qs, qs.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(q2.data(), b->q2, q2.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPC(hipMemcpy(bb.data(), b->bbot, bb.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int p = 0; p < N; ++p)
    for (int j = 0; j < k; ++j) {
      if (z1) z1[(size_t)p * k + j] = hz[(size_t)p * k + j];
      if (y1) y1[(size_t)p * k + j] = hy[(size_t)p * k + j];
    }
  for (int sct = 0; sct < c->n_sec; ++sct)
    for (int j = 0; j < k; ++j) {
      const double q = qs[(size_t)sct * kp + j], z = std::max(q, 0.0);
      if (z1) z1[(size_t)(N + sct) * k + j] = z;
      if (y1) y1[(size_t)(N + sct) * k + j] = q - z;
    }
  for (int a = 0; a < mA; ++a) {
    const int row = a < c->n_t ? a : c->ntp + (a - c->n_t);
    for (int j = 0; j < k; ++j) {
      const double bnd = a < c->n_t ? 0.0 : bb[(size_t)(a - c->n_t) * kp + j];
      const double q = q2[(size_t)row * kp + j], z = std::min(q, bnd);
      if (z2) z2[(size_t)a * k + j] = z;
      if (y2) y2[(size_t)a * k + j] = q - z;
    }
  }
  (void)nA;
  return LADMM_OK;
}

int ladmm_batch_import(ladmm_batch *b, const double *z1, const double *y1, const double *z2,
                       const double *y2) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (!z1 || !y1 || !z2 || !y2) return fail(LADMM_E_INVALID, "import needs z1, y1, z2, y2");
  ladmm_case *c = b->c;
  HIPC(hipSetDevice(c->ctx->device));
  const int k = b->k, kp = b->kp, N = c->N, mA = c->n_t + c->n_iso;
  double *dz = nullptr, *dy = nullptr;
  HIPC(hipMalloc((void **)&dz, (size_t)N * k * sizeof(double)));
  hipError_t e = hipMalloc((void **)&dy, (size_t)N * k * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(dz, z1, (size_t)N * k * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dy, y1, (size_t)N * k * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    if (c->precision == LADMM_F64) {
      e = import_points<double>(b->stream, (double *)b->q, kp, N, k, dz, dy);
      if (e == hipSuccess)
        e = w_from_q<double>(b->stream, (const double *)b->q, (double *)b->W, c->Np, kp,
                             point_table<double>(b));
    } else {
      e = import_points<float>(b->stream, (float *)b->q, kp, N, k, dz, dy);
      if (e == hipSuccess && c->precision == LADMM_F32)
        e = w_from_q<float>(b->stream, (const float *)b->q, (float *)b->W, c->Np, kp,
                            point_table<float>(b));
      else if (e == hipSuccess)
        e = w_from_q_bf(b->stream, (const float *)b->q, c->Np, kp, point_table<float>(b),
                        (uint16_t *)b->W, (uint16_t *)b->W + (size_t)kp * c->Np, b->wref, b->dW);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  hipFree(dz);
  if (dy) hipFree(dy);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("import: ") + hipGetErrorString(e));
  std::vector<double> qs((size_t)c->n_sec * kp, 0.0), q2((size_t)c->mAp * kp, 0.0);
  for (int sct = 0; sct < c->n_sec; ++sct)
    for (int j = 0; j < k; ++j)
      qs[(size_t)sct * kp + j] = z1[(size_t)(N + sct) * k + j] + y1[(size_t)(N + sct) * k + j];
  for (int a = 0; a < mA; ++a) {
    const int row = a < c->n_t ? a : c->ntp + (a - c->n_t);
    for (int j = 0; j < k; ++j) q2[(size_t)row * kp + j] = z2[(size_t)a * k + j] + y2[(size_t)a * k + j];
  }
  HIPC(hipMemcpy(b->qs, qs.data(), qs.size() * sizeof(double), hipMemcpyHostToDevice));
  HIPC(hipMemcpy(b->q2, q2.data(), q2.size() * sizeof(double), hipMemcpyHostToDevice));
  return LADMM_OK;
}

int ladmm_batch_set_graphs(ladmm_batch *b, int32_t on) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  b->graphs = on != 0;
  return LADMM_OK;
}

int ladmm_batch_set_compaction(ladmm_batch *b, int32_t on) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  b->compact = on != 0;
  return LADMM_OK;
}

int ladmm_batch_set_profiling(ladmm_batch *b, int32_t on) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  b->profiling = on != 0;
  for (int i = 0; i < LADMM_N_KERNEL_CLASSES; ++i) {
    b->kms[i] = 0.0;
    b->kcount[i] = 0;
  }
  return LADMM_OK;
}

int ladmm_batch_kernel_times(const ladmm_batch *b, double *ms_total, int64_t *launches) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  for (int i = 0; i < LADMM_N_KERNEL_CLASSES; ++i) {
    if (ms_total) ms_total[i] = b->kms[i];
    if (launches) launches[i] = b->kcount[i];
  }
  return LADMM_OK;
}

int ladmm_batch_step_sizes(const ladmm_batch *b, double *rho) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (!rho) return fail(LADMM_E_INVALID, "null rho");
  for (int j = 0; j < b->k; ++j) rho[j] = b->rho[j];
  return LADMM_OK;
}

int ladmm_batch_tiles(const ladmm_batch *b, int32_t *gemm1, int32_t *gemm2) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (gemm1) *gemm1 = b->cfg1;
  if (gemm2) *gemm2 = b->cfg2;
  return LADMM_OK;
}

int ladmm_batch_set_tiles(ladmm_batch *b, int32_t gemm1, int32_t gemm2) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (gemm1 < 0 || gemm1 >= kMaxGemmCfgs || gemm2 < 0 || gemm2 >= kMaxGemmCfgs)
    return fail(LADMM_E_INVALID, "tile configuration out of range");
  // the refresh's pair products take the same configurations where they serve
  // three terms, else configuration 0
  b->cfg1r = cfg_ok(b, 0, gemm1, 3) ? gemm1 : 0;
  b->cfg2r = cfg_ok(b, 1, gemm2, 3) ? gemm2 : 0;
  const int terms = b->c->precision == LADMM_BF16 ? 1 : 3;
  b->cfg1 = cfg_ok(b, 0, gemm1, terms) ? gemm1 : 0;
  b->cfg2 = cfg_ok(b, 1, gemm2, terms) ? gemm2 : 0;
  b->tuned = true;
  set_row_blocks(b);
  return LADMM_OK;
}

int ladmm_batch_timing(const ladmm_batch *b, double *iterate_ms, int64_t *plan_iterations) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (iterate_ms) *iterate_ms = b->iterate_ms;
  if (plan_iterations) *plan_iterations = b->plan_iters;
  return LADMM_OK;
}

}  // extern "C"

namespace {

// FP64 dose of every plan of batch b at n_vox voxels, from its current shot
// times: *dd (n_vox rows padded to the tile, kp columns) and, if dt_host is not
// NULL, the shot times themselves (ntp x kp) on the host.  The caller frees *dd.
int grid_dose(ladmm_batch *b, int64_t n_vox, const double *phi_vox, double **dd,
              std::vector<double> *dt_host, const char *who) {
  if (n_vox < 1 || !phi_vox) return fail(LADMM_E_INVALID, std::string(who) + ": bad arguments");
  if (n_vox > (int64_t)1 << 30) return fail(LADMM_E_INVALID, std::string(who) + ": too many voxels");
  ladmm_case *c = b->c;
  HIPC(hipSetDevice(c->ctx->device));
  const int nv = (int)n_vox, nvp = round_up(nv, kTileRows);
  const size_t nd = (size_t)nv * c->n_t;
  for (size_t e = 0; e < nd; ++e)
    if (!(phi_vox[e] >= 0.0) || !std::isfinite(phi_vox[e]))
      return fail(LADMM_E_INVALID, std::string(who) + ": dose rates must be finite and >= 0");
  std::vector<double> hp((size_t)nvp * c->ntp, 0.0);
  for (int v = 0; v < nv; ++v)
    std::memcpy(&hp[(size_t)v * c->ntp], phi_vox + (size_t)v * c->n_t, c->n_t * sizeof(double));
  double *dphi = nullptr, *dt = nullptr;
  *dd = nullptr;
  hipError_t e = hipMalloc((void **)&dphi, hp.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&dt, (size_t)c->ntp * b->kp * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)dd, (size_t)nvp * b->kp * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(dphi, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, b->stream);
  SmallArgs sa = small_args(b);
  if (e == hipSuccess) e = shot_times_matrix(b->stream, sa, b->q2, dt);
  if (e == hipSuccess) {
    EpiArgs<double> ea{};
    ea.C = *dd;
    ea.ldc = b->kp;
    e = gemm_nn<double>(b->stream, EPI_STORE, dphi, c->ntp, dt, b->kp, nvp, b->kp, c->ntp, ea);
  }
  if (e == hipSuccess && dt_host) {
    dt_host->assign((size_t)c->ntp * b->kp, 0.0);
    e = hipMemcpyAsync(dt_host->data(), dt, dt_host->size() * sizeof(double), hipMemcpyDeviceToHost,
                       b->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (dphi) hipFree(dphi);
  if (dt) hipFree(dt);
  if (e != hipSuccess) {
    if (*dd) hipFree(*dd);
    *dd = nullptr;
    return fail(LADMM_E_DEVICE, std::string(who) + ": " + hipGetErrorString(e));
  }
  return LADMM_OK;
}

}  // namespace

extern "C" {

int ladmm_batch_ld_band(ladmm_batch *b, int64_t n_vox, const double *phi_vox, double d_ld,
                        double delta, uint64_t *vol_bits) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (!vol_bits || !(delta > 0) || !std::isfinite(d_ld))
    return fail(LADMM_E_INVALID, "ld_band: bad arguments");
  double *dd = nullptr;
  int rc = grid_dose(b, n_vox, phi_vox, &dd, nullptr, "ld_band");
  if (rc) return rc;
  const int nv = (int)n_vox, W = (nv + 63) / 64;
  uint64_t *dbits = nullptr;
  hipError_t e = hipMalloc((void **)&dbits, (size_t)b->k * W * sizeof(uint64_t));
  if (e == hipSuccess) e = band_bits(b->stream, dd, b->kp, nv, b->k, d_ld, d_ld + delta, dbits);
  if (e == hipSuccess)
    e = hipMemcpyAsync(vol_bits, dbits, (size_t)b->k * W * sizeof(uint64_t), hipMemcpyDeviceToHost,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  hipFree(dd);
  if (dbits) hipFree(dbits);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("ld_band: ") + hipGetErrorString(e));
  return LADMM_OK;
}

int ladmm_batch_metrics(ladmm_batch *b, int64_t n_vox, const double *phi_vox,
                        const int32_t *vox_target, int32_t n_targets, const double *presc,
                        double d_ref, double *out) {
  if (!b) return fail(LADMM_E_STATE, "null batch");
  if (!vox_target || !presc || !out || n_targets < 1 || !(d_ref > 0) || !std::isfinite(d_ref))
    return fail(LADMM_E_INVALID, "metrics: bad arguments");
  int64_t n_target_vox = 0;
  for (int64_t v = 0; v < n_vox; ++v) {
    if (vox_target[v] < -1 || vox_target[v] >= n_targets)
      return fail(LADMM_E_INVALID, "metrics: voxel target index out of range");
    n_target_vox += vox_target[v] >= 0;
  }
  for (int i = 0; i < n_targets; ++i)
    if (!(presc[i] > 0) || !std::isfinite(presc[i]))
      return fail(LADMM_E_INVALID, "metrics: prescriptions must be > 0");
  ladmm_case *c = b->c;
  double *dd = nullptr;
  std::vector<double> t;
  int rc = grid_dose(b, n_vox, phi_vox, &dd, &t, "metrics");
  if (rc) return rc;
  const int nv = (int)n_vox, k = b->k;
  int32_t *dtgt = nullptr;
  double *dpresc = nullptr;
  unsigned long long *dcnt = nullptr;
  std::vector<unsigned long long> cnt((size_t)3 * k, 0);
  hipError_t e = hipMalloc((void **)&dtgt, (size_t)nv * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc((void **)&dpresc, (size_t)n_targets * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&dcnt, cnt.size() * sizeof(unsigned long long));
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtgt, vox_target, (size_t)nv * sizeof(int32_t), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dpresc, presc, (size_t)n_targets * sizeof(double), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dcnt, cnt.data(), cnt.size() * sizeof(unsigned long long),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = plan_metric_counts(b->stream, dd, b->kp, nv, k, dtgt, dpresc, d_ref, dcnt);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cnt.data(), dcnt, cnt.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  hipFree(dd);
  if (dtgt) hipFree(dtgt);
  if (dpresc) hipFree(dpresc);
  if (dcnt) hipFree(dcnt);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("metrics: ") + hipGetErrorString(e));
  const double nan = std::numeric_limits<double>::quiet_NaN();
  for (int j = 0; j < k; ++j) {
    const double cov = (double)cnt[3 * j], piv = (double)cnt[3 * j + 1], piv2 = (double)cnt[3 * j + 2];
    double bot = 0.0;
    for (int i = 0; i < c->n_iso; ++i) {
      double best = 0.0;
      for (int s = 0; s < c->S; ++s) {
        double sec = 0.0;
        for (int cc = 0; cc < c->C; ++cc) sec += t[(size_t)((i * c->S + s) * c->C + cc) * b->kp + j];
        best = std::max(best, sec);
      }
      bot += best;
    }
    out[4 * j + 0] = n_target_vox > 0 ? cov / (double)n_target_vox : nan;
    out[4 * j + 1] = piv > 0 ? cov / piv : nan;
    out[4 * j + 2] = piv > 0 ? piv2 / piv : nan;
    out[4 * j + 3] = bot;
  }
  return LADMM_OK;
}

int ladmm_select_ld_points(ladmm_ctx *ctx, int32_t k, int64_t n_vox, const uint64_t *vol_bits,
                           const int32_t *n_ld, uint64_t seed, int64_t *P, int64_t *nP,
                           uint64_t *masks) {
  if (!ctx) return fail(LADMM_E_STATE, "null context");
  if (k < 0 || n_vox < 1 || !nP || (k > 0 && (!vol_bits || !n_ld || !P || !masks)))
    return fail(LADMM_E_INVALID, "select_ld_points: bad arguments");
  if (n_vox > (int64_t)1 << 31) return fail(LADMM_E_INVALID, "select_ld_points: too many voxels");
  const int W = (int)((n_vox + 63) / 64);
  if (k == 0) {
    *nP = 0;
    return LADMM_OK;
  }
  // bits past n_vox must be clear
  if (n_vox % 64)
    for (int j = 0; j < k; ++j)
      if (vol_bits[(size_t)j * W + W - 1] >> (n_vox % 64))
        return fail(LADMM_E_INVALID, "select_ld_points: bits set past n_vox");
  HIPC(hipSetDevice(ctx->device));
  Alg1Work wk{};
  std::vector<void *> mem;
  hipError_t e = hipSuccess;
  auto get = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 8);
    if (e == hipSuccess) mem.push_back(*p);
  };
  const size_t wb = (size_t)W * sizeof(uint64_t);
  get((void **)&wk.Vu, wb); get((void **)&wk.pu, wb); get((void **)&wk.pt, wb);
  get((void **)&wk.nw, wb); get((void **)&wk.po, wb); get((void **)&wk.tmp, wb);
  get((void **)&wk.uni, wb); get((void **)&wk.keys, wb * 64); get((void **)&wk.pj, wb * k);
  get((void **)&wk.vsize, (size_t)k * sizeof(int64_t)); get((void **)&wk.order, (size_t)k * sizeof(int32_t));
  get((void **)&wk.offs, (size_t)W * sizeof(int64_t));
  uint64_t *dvols = nullptr, *dmasks = nullptr;
  int32_t *dn = nullptr;
  int64_t *dP = nullptr, *dnP = nullptr;
  get((void **)&dvols, wb * k); get((void **)&dmasks, wb * k); get((void **)&dn, (size_t)k * sizeof(int32_t));
  get((void **)&dP, (size_t)n_vox * sizeof(int64_t)); get((void **)&dnP, sizeof(int64_t));
  hipStream_t s = nullptr;
  if (e == hipSuccess) e = hipStreamCreate(&s);
  if (e == hipSuccess) e = hipMemcpyAsync(dvols, vol_bits, wb * k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dn, n_ld, (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = alg1_select(s, k, n_vox, dvols, dn, seed, wk, dP, dnP, dmasks, W);
  int64_t hn = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hn, dnP, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && hn > 0)
    e = hipMemcpyAsync(P, dP, (size_t)hn * sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(masks, dmasks, wb * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (void *p : mem) hipFree(p);
  if (s) hipStreamDestroy(s);
  if (e != hipSuccess) return fail(LADMM_E_DEVICE, std::string("select_ld_points: ") + hipGetErrorString(e));
  *nP = hn;
  return LADMM_OK;
}

int ladmm_select_ld_points_static(ladmm_ctx *ctx, int32_t k, int64_t n_vox,
                                  const uint64_t *vol_bits, const int32_t *n_ld, uint64_t seed,
                                  int64_t *P, int64_t *nP, uint64_t *masks) {
  if (!ctx) return fail(LADMM_E_STATE, "null context");
  if (k < 0 || n_vox < 1 || !nP || (k > 0 && (!vol_bits || !n_ld || !P || !masks)))
    return fail(LADMM_E_INVALID, "select_ld_points_static: bad arguments");
  if (n_vox > (int64_t)1 << 31) return fail(LADMM_E_INVALID, "select_ld_points_static: too many voxels");
  const int W = (int)((n_vox + 63) / 64);
  if (k == 0) {
    *nP = 0;
    return LADMM_OK;
  }
  if (n_vox % 64)
    for (int j = 0; j < k; ++j)
      if (vol_bits[(size_t)j * W + W - 1] >> (n_vox % 64))
        return fail(LADMM_E_INVALID, "select_ld_points_static: bits set past n_vox");
  // layout in the scratch array: the same buffers as ladmm_select_ld_points
  // allocates, each 256-byte aligned
  const size_t wb = (size_t)W * sizeof(uint64_t);
  const size_t sizes[] = {wb, wb, wb, wb, wb, wb, wb, wb * 64, wb * (size_t)k,
                          (size_t)k * sizeof(int64_t), (size_t)k * sizeof(int32_t),
                          (size_t)W * sizeof(int64_t), wb * (size_t)k, wb * (size_t)k,
                          (size_t)k * sizeof(int32_t), (size_t)n_vox * sizeof(int64_t),
                          sizeof(int64_t)};
  constexpr int kBufs = sizeof(sizes) / sizeof(sizes[0]);
  size_t off[kBufs], need = 0;
  for (int i = 0; i < kBufs; ++i) {
    off[i] = need;
    need += (sizes[i] + 255) / 256 * 256;
  }
  if (need > alg1_scratch_bytes())
    return fail(LADMM_E_INVALID, "select_ld_points_static: needs " + std::to_string(need) +
                                     " bytes of scratch, more than its " +
                                     std::to_string(alg1_scratch_bytes()) +
                                     " (use ladmm_select_ld_points)");
  std::mutex *mu = alg1_scratch_lock(ctx->device);
  if (!mu) return fail(LADMM_E_INVALID, "select_ld_points_static: device index out of range");
  std::lock_guard<std::mutex> lk(*mu);
  HIPC(hipSetDevice(ctx->device));
  unsigned char *base = nullptr;
  HIPC(alg1_scratch(ctx->device, &base));
  auto at = [&](int i) { return (void *)(base + off[i]); };
  Alg1Work wk{};
  wk.Vu = (uint64_t *)at(0); wk.pu = (uint64_t *)at(1); wk.pt = (uint64_t *)at(2);
  wk.nw = (uint64_t *)at(3); wk.po = (uint64_t *)at(4); wk.tmp = (uint64_t *)at(5);
  wk.uni = (uint64_t *)at(6); wk.keys = (uint64_t *)at(7); wk.pj = (uint64_t *)at(8);
  wk.vsize = (int64_t *)at(9); wk.order = (int32_t *)at(10); wk.offs = (int64_t *)at(11);
  uint64_t *dvols = (uint64_t *)at(12), *dmasks = (uint64_t *)at(13);
  int32_t *dn = (int32_t *)at(14);
  int64_t *dP = (int64_t *)at(15), *dnP = (int64_t *)at(16);
  // the null stream: nothing is created; every array the kernels read is
  // written by this call first (inputs copied, work arrays set by the kernels)
  hipStream_t s = nullptr;
  HIPC(hipMemcpyAsync(dvols, vol_bits, wb * k, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(dn, n_ld, (size_t)k * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPC(alg1_select(s, k, n_vox, dvols, dn, seed, wk, dP, dnP, dmasks, W));
  int64_t hn = 0;
  HIPC(hipMemcpyAsync(&hn, dnP, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (hn > 0) HIPC(hipMemcpyAsync(P, dP, (size_t)hn * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIPC(hipMemcpyAsync(masks, dmasks, wb * k, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  *nP = hn;
  return LADMM_OK;
}

int ladmm_passes(ladmm_ctx *ctx, const ladmm_case_desc *d1, int32_t k, const ladmm_weights *w,
                 const ladmm_opts *opts, int32_t n_sets, const ladmm_pass2_desc *sets,
                 int32_t n_passes, ladmm_result *pass_out, int64_t *P_out, int64_t *n_points,
                 double *times_ms) {
  if (!ctx || !d1 || !w || !opts || !sets) return fail(LADMM_E_INVALID, "passes: null argument");
  if (k < 1 || n_sets < 1 || n_passes < 2 || n_passes > 64)
    return fail(LADMM_E_INVALID, "passes: k >= 1, n_sets >= 1, n_passes in [2, 64]");
  for (int i = 0; i < n_sets; ++i) {
    const ladmm_pass2_desc &p2 = sets[i];
    if (p2.n_vox < 1 || !p2.phi_vox || !p2.n_ld)
      return fail(LADMM_E_INVALID, "passes: bad second-pass description");
    if (p2.ld_group < 0 || p2.ld_group >= d1->n_groups || d1->groups[p2.ld_group].type != LADMM_PT_LD)
      return fail(LADMM_E_INVALID, "passes: ld_group must name a low-dose group");
    for (int j = 0; j < i; ++j)
      if (sets[j].ld_group == p2.ld_group)
        return fail(LADMM_E_INVALID, "passes: each set replaces a different low-dose group");
  }
  using clk = std::chrono::steady_clock;
  auto ms = [](clk::time_point a, clk::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  std::vector<double> tm;
  const int n_t = d1->n_iso * d1->n_sectors * d1->n_collimators;
  // points kept in every later pass: those outside the replaced groups
  std::vector<int32_t> keep;
  for (int p = 0; p < d1->n_points; ++p) {
    bool replaced = false;
    for (int i = 0; i < n_sets; ++i) replaced |= d1->point_group[p] == sets[i].ld_group;
    if (!replaced) keep.push_back(p);
  }
  // pass 1
  auto t0 = clk::now();
  ladmm_case *cur_c = nullptr;
  ladmm_batch *cur_b = nullptr;
  // pass 1's dose rates stay on the device: every later pass gathers its kept
  // rows there and uploads only its new low-dose rows
  double *dose1 = nullptr;
  int32_t *keep_d = nullptr;
  int rc = create_case_impl(ctx, d1, &cur_c, nullptr, n_passes > 1 ? &dose1 : nullptr);
  if (rc) return rc;
  auto free_dev = [&]() {
    if (dose1) hipFree(dose1);
    if (keep_d) hipFree(keep_d);
    dose1 = nullptr;
    keep_d = nullptr;
  };
  if (n_passes > 1 && !keep.empty()) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc((void **)&keep_d, keep.size() * sizeof(int32_t));
    if (e == hipSuccess)
      e = hipMemcpy(keep_d, keep.data(), keep.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      ladmm_destroy_case(cur_c);
      free_dev();
      return fail(LADMM_E_DEVICE, std::string("passes: ") + hipGetErrorString(e));
    }
  }
  auto t1 = clk::now();
  rc = ladmm_batch_create(cur_c, k, w, nullptr, nullptr, opts, &cur_b);
  if (rc == LADMM_OK) rc = ladmm_batch_run(cur_b);
  if (rc == LADMM_OK && pass_out) rc = ladmm_batch_results(cur_b, &pass_out[0]);
  auto t2 = clk::now();
  tm.push_back(ms(t0, t1));
  tm.push_back(ms(t1, t2));
  std::vector<std::vector<int64_t>> P(n_sets);
  std::vector<int64_t> nP(n_sets, 0);
  int64_t N2 = 0;
  for (int pass = 1; pass < n_passes && rc == LADMM_OK; ++pass) {
    // per set: low-dose band of the previous pass's dose at its threshold, then Algorithm 1
    auto ta = clk::now();
    std::vector<std::vector<uint64_t>> masks(n_sets);
    for (int i = 0; i < n_sets && rc == LADMM_OK; ++i) {
      const ladmm_pass2_desc &p2 = sets[i];
      const int64_t nv = p2.n_vox;
      const size_t Wv = (size_t)((nv + 63) / 64);
      std::vector<uint64_t> vol((size_t)k * Wv);
      masks[i].assign((size_t)k * Wv, 0);
      P[i].assign(nv, 0);
      rc = ladmm_batch_ld_band(cur_b, nv, p2.phi_vox, p2.d_ld, p2.delta, vol.data());
      if (rc == LADMM_OK)
        rc = ladmm_select_ld_points(ctx, k, nv, vol.data(), p2.n_ld, p2.seed, P[i].data(), &nP[i],
                                    masks[i].data());
    }
    ladmm_batch_destroy(cur_b);
    ladmm_destroy_case(cur_c);
    cur_b = nullptr;
    cur_c = nullptr;
    if (rc) break;
    auto tb = clk::now();
    // this pass's case: the kept points, then the points of each set's P in its group
    N2 = (int64_t)keep.size();
    for (int i = 0; i < n_sets; ++i) N2 += nP[i];
    if (N2 < 1 || N2 > INT32_MAX) {
      rc = fail(LADMM_E_INVALID, "passes: empty or too large pass");
      break;
    }
    // this pass's dose rates on the device: the kept rows gathered from pass 1's
    // copy, then the new low-dose rows of each set uploaded behind them
    std::vector<int32_t> grp2(N2);
    for (size_t i = 0; i < keep.size(); ++i) grp2[i] = d1->point_group[keep[i]];
    double *dose2 = nullptr;
    {
      const size_t nk = keep.size();
      size_t n_new = (size_t)(N2 - (int64_t)nk);
      std::vector<double> rows_new(n_new * n_t);
      size_t r = 0;
      for (int st = 0; st < n_sets; ++st)
        for (int64_t i = 0; i < nP[st]; ++i, ++r)
          std::memcpy(&rows_new[r * n_t], sets[st].phi_vox + (size_t)P[st][i] * n_t, n_t * sizeof(double));
      hipError_t e = hipSetDevice(ctx->device);
      if (e == hipSuccess) e = hipMalloc((void **)&dose2, (size_t)N2 * n_t * sizeof(double));
      if (e == hipSuccess && nk > 0) e = gather_rows(nullptr, dose1, dose2, (int)nk, (size_t)n_t, 8, keep_d);
      if (e == hipSuccess && n_new > 0)
        e = hipMemcpy(dose2 + nk * n_t, rows_new.data(), n_new * n_t * sizeof(double), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess) {
        if (dose2) hipFree(dose2);
        rc = fail(LADMM_E_DEVICE, std::string("passes: ") + hipGetErrorString(e));
        break;
      }
    }
    const int W2 = (int)((N2 + 63) / 64);
    std::vector<uint64_t> mask2((size_t)k * W2, 0);
    int64_t at = (int64_t)keep.size();
    for (int st = 0; st < n_sets; ++st) {
      const ladmm_pass2_desc &p2 = sets[st];
      const size_t Wv = (size_t)((p2.n_vox + 63) / 64);
      for (int64_t i = 0; i < nP[st]; ++i) grp2[at + i] = p2.ld_group;
      for (int j = 0; j < k; ++j)
        for (int64_t i = 0; i < nP[st]; ++i)
          if ((masks[st][(size_t)j * Wv + (i >> 6)] >> (i & 63)) & 1ull) {
            const int64_t pt = at + i;
            mask2[(size_t)j * W2 + (pt >> 6)] |= 1ull << (pt & 63);
          }
      at += nP[st];
    }
    ladmm_case_desc d2 = *d1;
    d2.n_points = (int32_t)N2;
    d2.dose = nullptr;
    d2.point_group = grp2.data();
    rc = create_case_impl(ctx, &d2, &cur_c, dose2, nullptr);
    hipFree(dose2);
    if (rc) break;
    auto tc = clk::now();
    rc = ladmm_batch_create(cur_c, k, w, mask2.data(), nullptr, opts, &cur_b);
    if (rc == LADMM_OK) rc = ladmm_batch_run(cur_b);
    if (rc == LADMM_OK && pass_out) rc = ladmm_batch_results(cur_b, &pass_out[pass]);
    auto td = clk::now();
    tm.push_back(ms(ta, tb));
    tm.push_back(ms(tb, tc));
    tm.push_back(ms(tc, td));
  }
  if (cur_b) ladmm_batch_destroy(cur_b);
  if (cur_c) ladmm_destroy_case(cur_c);
  free_dev();
  if (rc) return rc;
  if (times_ms) std::memcpy(times_ms, tm.data(), tm.size() * sizeof(double));
  if (P_out) {
    int64_t o = 0;
    for (int st = 0; st < n_sets; ++st) {
      std::memcpy(P_out + o, P[st].data(), (size_t)nP[st] * sizeof(int64_t));
      o += nP[st];
    }
  }
  if (n_points) {
    for (int st = 0; st < n_sets; ++st) n_points[st] = nP[st];
    n_points[n_sets] = N2;
  }
  return LADMM_OK;
}

int ladmm_two_pass_sets(ladmm_ctx *ctx, const ladmm_case_desc *d1, int32_t k,
                        const ladmm_weights *w, const ladmm_opts *opts, int32_t n_sets,
                        const ladmm_pass2_desc *sets, ladmm_result *pass1_out, ladmm_result *out,
                        int64_t *P_out, int64_t *n_points2, double *times_ms) {
  if (!out) return fail(LADMM_E_INVALID, "two_pass: null argument");
  ladmm_result res[2];
  std::memset(&res[0], 0, sizeof(res[0]));
  if (pass1_out) res[0] = *pass1_out;
  res[1] = *out;
  return ladmm_passes(ctx, d1, k, w, opts, n_sets, sets, 2, res, P_out, n_points2, times_ms);
}

int ladmm_two_pass(ladmm_ctx *ctx, const ladmm_case_desc *d1, int32_t k, const ladmm_weights *w,
                   const ladmm_opts *opts, const ladmm_pass2_desc *p2, ladmm_result *pass1_out,
                   ladmm_result *out, int64_t *P_out, int64_t *n_points2, double *times_ms) {
  return ladmm_two_pass_sets(ctx, d1, k, w, opts, 1, p2, pass1_out, out, P_out, n_points2, times_ms);
}

int ladmm_solve_batch(ladmm_case *c, int32_t k, const ladmm_weights *w, const uint64_t *ld_mask,
                      const ladmm_opts *opts, ladmm_result *out) {
  ladmm_batch *b = nullptr;
  int rc = ladmm_batch_create(c, k, w, ld_mask, nullptr, opts, &b);
  if (rc) return rc;
  rc = ladmm_batch_run(b);
  if (rc == LADMM_OK) rc = ladmm_batch_results(b, out);
  destroy_batch_impl(b);
  return rc;
}

}  // extern "C"
