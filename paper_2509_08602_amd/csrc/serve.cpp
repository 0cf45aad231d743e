// Serving engine: continuous batching of plan requests over resident cases.
//
// Plans are the columns of the batched iteration (end of Sec. 2.B): all plans
// of a case share its dose block and Schur complement inverse and differ only
// in b, u and their step size (Eq. rho_rule, Sec. 3.C).  A server keeps, for
// each case with work, one batch whose columns are slots (a lane).  One worker
// thread drives every lane in rounds:
//
//   1. take new requests and cancellations from the callers;
//   2. admit queued plans, oldest request first, into free slots: the slot's
//      columns of the iterates are zeroed and its table entries written (u, b,
//      1/rho, LD mask), so the plan starts cold exactly as in a batch of its
//      own; with a warm store, the columns are instead loaded from the stored
//      solved plan of the nearest weighting;
//   3. launch check_every iterations on every lane with work, each lane on its
//      own stream so that lanes of different cases overlap on the device;
//   4. wait for the lanes, apply each plan's stopping rule at the check, and
//      retire finished plans: shot times and statistics go to the request's
//      result buffers and the slot becomes free for the next round.
//
// A plan's arithmetic never depends on the other columns, on its slot index or
// on the tile configuration, and its checks fall every check_every iterations
// of its own, so its result is bitwise the one of a batch holding it alone.
// Lane memory is charged to the context's HBM budget; when a new lane does not
// fit, idle lanes are released, least recently used first, and requests wait
// while busy lanes hold the memory.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "state.h"
#include "warm.h"

using namespace ladmm;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket = 0;
  ladmm_case *c = nullptr;
  int k = 0;
  std::vector<ladmm_weights> w;
  std::vector<uint64_t> mask;   // k x ceil(N/64) words; empty = every LD point
  ladmm_opts opts{};
  int32_t max_iter = 0;   // rounded up to a multiple of the server's check_every
  ladmm_result out{};
  // worker-owned
  int next = 0;        // plans admitted so far
  int in_slots = 0;    // plans occupying slots
  // guarded by the server mutex
  int done = 0;                 // plans retired
  int status = LADMM_PENDING;   // final status once not PENDING
  bool cancel = false;
  std::string err;
  Clock::time_point t_submit, t_done;
};

struct Lane {
  ladmm_case *c = nullptr;
  ladmm_batch *b = nullptr;
  std::vector<Request *> owner;   // per slot
  std::vector<int> plan;          // per slot: plan index in the owner
  // pinned host mirrors of the per-plan tables (uploaded on the lane's stream)
  void *h_utab = nullptr;
  double *h_invrho = nullptr, *h_wbot = nullptr, *h_bbot = nullptr, *h_t = nullptr;
  uint64_t *h_mask = nullptr;
  int32_t *h_active = nullptr, *h_reset = nullptr;
  int32_t *d_reset = nullptr;
  double *d_t = nullptr;
  bool dirty = false, any_reset = false, launched = false;
  Clock::time_point last_used;
  std::vector<int> ld_points;     // indices of the case's LD points
  // warm-start store: final iterates of up to wcap converged plans
  int wcap = 0, wcount = 0, wnext = 0;
  void *wq = nullptr;             // wcap x Np (the iterate type)
  double *wq2 = nullptr, *wqs = nullptr;   // wcap x mAp, wcap x n_sec
  std::vector<ladmm_weights> ww;  // weighting of each entry
  std::vector<double> wrho;       // final step size of each entry
  std::vector<int> warm_src;      // per slot: entry to load at the next upload, -1 none

  int busy() const {
    int n = 0;
    for (Request *r : owner) n += r != nullptr;
    return n;
  }
};

}  // namespace

struct ladmm_server {
  ladmm_ctx *ctx = nullptr;
  ladmm_server_opts opts{};
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::map<uint64_t, Request *> tickets;   // guarded
  std::vector<Request *> incoming;         // guarded
  bool cancel_pending = false;             // guarded
  // statistics (guarded)
  int64_t submitted = 0, completed = 0, cancelled = 0, failed = 0, plans_retired = 0;
  int64_t plan_iterations = 0;
  double busy_ms = 0.0;
  std::vector<double> latency_ms;
  int32_t n_lanes = 0, busy_slots = 0;
  int64_t warm_starts = 0;
  // worker-owned
  int64_t warm_round = 0;   // warm starts of the current round
  std::vector<std::unique_ptr<Lane>> lanes;
  std::deque<Request *> pending;   // requests with plans not yet admitted
  std::vector<Request *> live;     // requests not yet final
};

namespace {

template <typename T>
void set_u_column(Lane &L, int s, const ladmm_weights &w, const std::vector<int64_t> &cnt) {
  const ladmm_case *c = L.c;
  const int kp = L.b->kp;
  T *u = (T *)L.h_utab;
  for (int g = 0; g < c->G; ++g) {
    const ladmm_group &gr = c->groups[g];
    double wt = 0.0;
    switch (gr.type) {
      case LADMM_PT_TS:
      case LADMM_PT_TI: wt = w.w_t; break;
      case LADMM_PT_RING: wt = w.w_r; break;
      case LADMM_PT_LD: wt = w.w_ld; break;
      default: break;
    }
    double val = INFINITY;
    if (gr.type != LADMM_PT_OAR) val = cnt[g] > 0 ? gr.share * wt / (double)cnt[g] : 0.0;
    u[(size_t)g * kp + s] = (T)val;
  }
  u[(size_t)c->G * kp + s] = T(0);
}

// Start plan p of request r in slot s: table entries and a zeroed column.
void admit(Lane &L, int s, Request *r, int p) {
  ladmm_case *c = L.c;
  ladmm_batch *b = L.b;
  const int kp = b->kp, mw = b->mask_words, cw = (c->N + 63) / 64;
  const ladmm_weights &w = r->w[p];
  // LD membership bits of the slot and the per-group point counts under them
  uint64_t *row = L.h_mask + (size_t)s * mw;
  std::memset(row, 0, (size_t)mw * sizeof(uint64_t));
  std::vector<int64_t> cnt(c->counts.begin(), c->counts.end());
  if (r->mask.empty()) {
    for (int q = 0; q < c->N; ++q) row[q >> 6] |= 1ull << (q & 63);
  } else {
    const uint64_t *src = &r->mask[(size_t)p * cw];
    std::memcpy(row, src, (size_t)cw * sizeof(uint64_t));
    if (c->N % 64) row[cw - 1] &= (1ull << (c->N % 64)) - 1;
    for (int g = 0; g < c->G; ++g)
      if (c->groups[g].type == LADMM_PT_LD) cnt[g] = 0;
    for (int q : L.ld_points)
      if ((row[q >> 6] >> (q & 63)) & 1ull) cnt[c->hgrp[q]]++;
  }
  if (c->precision == LADMM_F64)
    set_u_column<double>(L, s, w, cnt);
  else
    set_u_column<float>(L, s, w, cnt);
  double rho = r->opts.rho0 * std::sqrt(r->opts.w0_bot / w.w_bot);
  L.warm_src[s] = -1;
  if (L.wcount > 0) {
    // nearest stored weighting in slider coordinates
    int best = -1;
    double bd = 0.0;
    for (int e = 0; e < L.wcount; ++e) {
      const ladmm_weights &v = L.ww[e];
      const double dt = v.w_t - w.w_t, dr = v.w_r - w.w_r, dl = v.w_ld - w.w_ld;
      const double db = (std::log10(v.w_bot) - std::log10(w.w_bot)) / 3.0;
      const double d = dt * dt + dr * dr + dl * dl + db * db;
      if (best < 0 || d < bd) {
        best = e;
        bd = d;
      }
    }
    L.warm_src[s] = best;
    rho = L.wrho[best];
  }
  L.h_invrho[s] = 1.0 / rho;
  L.h_wbot[s] = w.w_bot;
  for (int i = 0; i < c->n_iso; ++i) L.h_bbot[(size_t)i * kp + s] = c->hE[c->ntp + i] * w.w_bot;
  L.h_reset[s] = 1;
  b->h_active[s] = 1;
  b->w[s] = w;
  b->rho[s] = rho;
  b->start[s] = b->iters_run;
  b->rule[s] = make_rule(r->opts, r->max_iter, rho);
  b->status[s] = LADMM_PLAN_RUNNING;
  b->iters[s] = 0;
  std::fill(b->rec.begin() + (size_t)s * kFinal, b->rec.begin() + (size_t)(s + 1) * kFinal, NAN);
  L.owner[s] = r;
  L.plan[s] = p;
  L.dirty = L.any_reset = true;
  r->next++;
  r->in_slots++;
}

// Upload the tables of a lane whose slots changed, and zero the admitted columns.
int upload(Lane &L) {
  ladmm_case *c = L.c;
  ladmm_batch *b = L.b;
  hipStream_t s = b->stream;
  const int kp = b->kp;
  const size_t Tsz = c->precision == LADMM_F64 ? sizeof(double) : sizeof(float);
  for (int j = 0; j < kp; ++j) L.h_active[j] = b->h_active[j];
  HIPC(hipMemcpyAsync(b->utab, L.h_utab, (size_t)(c->G + 1) * kp * Tsz, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(b->invrho, L.h_invrho, kp * sizeof(double), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(b->wbot, L.h_wbot, kp * sizeof(double), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(b->bbot, L.h_bbot, (size_t)c->n_iso * kp * sizeof(double), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(b->mask, L.h_mask, (size_t)kp * b->mask_words * sizeof(uint64_t),
                      hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(b->active, L.h_active, kp * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (L.any_reset) {
    HIPC(hipMemcpyAsync(L.d_reset, L.h_reset, kp * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (c->precision == LADMM_F64) {
      HIPC(zero_columns<double>(s, (double *)b->q, c->Np, kp, L.d_reset));
      HIPC(zero_columns<double>(s, (double *)b->W, c->Np, kp, L.d_reset));
    } else if (c->precision == LADMM_F32) {
      HIPC(zero_columns<float>(s, (float *)b->q, c->Np, kp, L.d_reset));
      HIPC(zero_columns<float>(s, (float *)b->W, c->Np, kp, L.d_reset));
    } else {   // W' is held as plan-major BF16 pairs
      HIPC(zero_columns<float>(s, (float *)b->q, c->Np, kp, L.d_reset));
      HIPC(zero_plan_rows_bf(s, (uint16_t *)b->W, kp, c->Np, L.d_reset));
      if (c->precision == LADMM_BF16) {   // a fresh plan's references are zero too
        HIPC(zero_columns<float>(s, b->xref, c->Np, kp, L.d_reset));
        HIPC(zero_columns<float>(s, b->wref, c->Np, kp, L.d_reset));
        HIPC(zero_columns<double>(s, b->gref, c->ntp, kp, L.d_reset));
        HIPC(zero_columns<double>(s, b->vref, c->ntp, kp, L.d_reset));
        HIPC(zero_columns<double>(s, b->rref, c->mAp, kp, L.d_reset));
        HIPC(zero_columns<double>(s, b->vfull, c->mAp, kp, L.d_reset));
        HIPC(zero_plan_rows_bf(s, b->dW, kp, c->Np, L.d_reset, 1));
      }
    }
    HIPC(zero_columns<double>(s, b->qs, c->n_sec, kp, L.d_reset));
    HIPC(zero_columns<double>(s, b->q2, c->mAp, kp, L.d_reset));
    // warm-started slots: columns from the store, then their W' columns
    WarmCols wc{};
    auto flush = [&]() -> int {
      if (wc.n == 0) return LADMM_OK;
      if (c->precision == LADMM_F64) {
        HIPC(warm_load<double>(s, wc, (const double *)L.wq, L.wq2, L.wqs, c->Np, c->mAp, c->n_sec,
                               kp, (double *)b->q, b->q2, b->qs));
        HIPC(warm_w<double>(s, wc, (const double *)b->q, (double *)b->W, c->Np, kp,
                            point_table<double>(b)));
      } else {
        HIPC(warm_load<float>(s, wc, (const float *)L.wq, L.wq2, L.wqs, c->Np, c->mAp, c->n_sec, kp,
                              (float *)b->q, b->q2, b->qs));
        if (c->precision == LADMM_F32) {
          HIPC(warm_w<float>(s, wc, (const float *)b->q, (float *)b->W, c->Np, kp,
                             point_table<float>(b)));
        } else {
          uint16_t *wh = (uint16_t *)b->W;
          HIPC(warm_w_bf(s, wc, (const float *)b->q, wh, wh + (size_t)kp * c->Np, c->Np, kp,
                         point_table<float>(b), b->wref, b->dW));
        }
      }
      wc.n = 0;
      return LADMM_OK;
    };
    for (int j = 0; j < kp; ++j) {
      if (L.warm_src[j] < 0) continue;
      wc.col[wc.n] = j;
      wc.ent[wc.n] = L.warm_src[j];
      L.warm_src[j] = -1;
      if (++wc.n == kWarmCols) {
        int rc = flush();
        if (rc) return rc;
      }
    }
    int rc = flush();
    if (rc) return rc;
  }
  L.dirty = false;
  return LADMM_OK;
}

void free_lane(Lane *L) {
  if (L->b) destroy_batch_impl(L->b);   // synchronizes the lane's stream first
  if (L->h_utab) hipHostFree(L->h_utab);
  if (L->h_invrho) hipHostFree(L->h_invrho);
  if (L->h_wbot) hipHostFree(L->h_wbot);
  if (L->h_bbot) hipHostFree(L->h_bbot);
  if (L->h_t) hipHostFree(L->h_t);
  if (L->h_mask) hipHostFree(L->h_mask);
  if (L->h_active) hipHostFree(L->h_active);
  if (L->h_reset) hipHostFree(L->h_reset);
}

int make_lane(ladmm_server *sv, ladmm_case *c, std::unique_ptr<Lane> *out) {
  std::unique_ptr<Lane> L(new Lane());
  L->c = c;
  ladmm_opts o{};
  o.max_iter = 1;
  o.check_every = sv->opts.check_every;
  o.autotune = sv->opts.autotune;
  int rc = create_batch_impl(c, sv->opts.slots, nullptr, nullptr, nullptr, &o, &L->b, true);
  if (rc) return rc;
  ladmm_batch *b = L->b;
  b->graphs = sv->opts.eager == 0;
  const int kp = b->kp;
  const size_t Tsz = c->precision == LADMM_F64 ? sizeof(double) : sizeof(float);
  L->owner.assign(kp, nullptr);
  L->plan.assign(kp, -1);
  for (int q = 0; q < c->N; ++q)
    if (c->groups[c->hgrp[q]].type == LADMM_PT_LD) L->ld_points.push_back(q);
  hipError_t e = hipSuccess;
  auto pin = [&](void **p, size_t bytes) {
    if (e == hipSuccess) e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) std::memset(*p, 0, bytes);
  };
  pin(&L->h_utab, (size_t)(c->G + 1) * kp * Tsz);
  pin((void **)&L->h_invrho, kp * sizeof(double));
  pin((void **)&L->h_wbot, kp * sizeof(double));
  pin((void **)&L->h_bbot, (size_t)c->n_iso * kp * sizeof(double));
  pin((void **)&L->h_t, (size_t)kp * c->n_t * sizeof(double));
  pin((void **)&L->h_mask, (size_t)kp * b->mask_words * sizeof(uint64_t));
  pin((void **)&L->h_active, kp * sizeof(int32_t));
  pin((void **)&L->h_reset, kp * sizeof(int32_t));
  if (e != hipSuccess) {
    free_lane(L.get());
    return fail(LADMM_E_NOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  void *p = nullptr;
  rc = batch_alloc(b, &p, kp * sizeof(int32_t));
  if (rc == LADMM_OK) L->d_reset = (int32_t *)p;
  if (rc == LADMM_OK) rc = batch_alloc(b, &p, (size_t)kp * c->n_t * sizeof(double));
  if (rc == LADMM_OK) L->d_t = (double *)p;
  L->warm_src.assign(kp, -1);
  if (rc == LADMM_OK && sv->opts.warm_store > 0) {
    L->wcap = sv->opts.warm_store;
    rc = batch_alloc(b, &L->wq, (size_t)L->wcap * c->Np * Tsz);
    if (rc == LADMM_OK) rc = batch_alloc(b, &p, (size_t)L->wcap * c->mAp * sizeof(double));
    if (rc == LADMM_OK) L->wq2 = (double *)p;
    if (rc == LADMM_OK) rc = batch_alloc(b, &p, (size_t)L->wcap * c->n_sec * sizeof(double));
    if (rc == LADMM_OK) L->wqs = (double *)p;
    L->ww.assign(L->wcap, ladmm_weights{});
    L->wrho.assign(L->wcap, 0.0);
  }
  if (rc == LADMM_OK) rc = prepare_batch(b);
  if (rc) {
    free_lane(L.get());
    return rc;
  }
  // padding slots: zero u and rho, inactive; the first upload writes every table
  L->dirty = true;
  L->last_used = Clock::now();
  *out = std::move(L);
  return LADMM_OK;
}

Lane *find_lane(ladmm_server *sv, const ladmm_case *c) {
  for (auto &L : sv->lanes)
    if (L->c == c) return L.get();
  return nullptr;
}

// Lane for case c, creating it if memory allows (idle lanes are released,
// least recently used first).  Returns LADMM_PENDING when the memory is held
// by busy lanes.
int lane_for(ladmm_server *sv, ladmm_case *c, Lane **out) {
  if (Lane *L = find_lane(sv, c)) {
    *out = L;
    return LADMM_OK;
  }
  auto evict_one = [&]() {
    int best = -1;
    for (size_t i = 0; i < sv->lanes.size(); ++i)
      if (sv->lanes[i]->busy() == 0 &&
          (best < 0 || sv->lanes[i]->last_used < sv->lanes[best]->last_used))
        best = (int)i;
    if (best < 0) return false;
    free_lane(sv->lanes[best].get());
    sv->lanes.erase(sv->lanes.begin() + best);
    return true;
  };
  while (sv->opts.max_lanes > 0 && (int)sv->lanes.size() >= sv->opts.max_lanes)
    if (!evict_one()) return LADMM_PENDING;
  for (;;) {
    std::unique_ptr<Lane> L;
    int rc = make_lane(sv, c, &L);
    if (rc == LADMM_OK) {
      sv->lanes.push_back(std::move(L));
      *out = sv->lanes.back().get();
      return LADMM_OK;
    }
    if (rc != LADMM_E_NOMEM) return rc;
    if (!evict_one()) {
      bool busy = false;
      for (auto &x : sv->lanes) busy |= x->busy() > 0;
      return busy ? LADMM_PENDING : rc;
    }
  }
}

// Final status of a request (worker, with the server mutex held).
void finish_locked(ladmm_server *sv, Request *r, int status, const std::string &err) {
  r->status = status;
  r->err = err;
  r->t_done = Clock::now();
  if (status == LADMM_OK) {
    sv->completed++;
    sv->latency_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
  } else if (status == LADMM_E_CANCELLED) {
    sv->cancelled++;
  } else {
    sv->failed++;
  }
}

// Remove a request from the worker's queues and free its slots.
void drop(ladmm_server *sv, Request *r) {
  for (auto &L : sv->lanes)
    for (size_t s = 0; s < L->owner.size(); ++s)
      if (L->owner[s] == r) {
        L->owner[s] = nullptr;
        L->b->h_active[s] = 0;
        L->dirty = true;
      }
  r->in_slots = 0;
  sv->pending.erase(std::remove(sv->pending.begin(), sv->pending.end(), r), sv->pending.end());
  sv->live.erase(std::remove(sv->live.begin(), sv->live.end(), r), sv->live.end());
}

// Fail every request holding a slot of lane L and release the lane.
void fail_lane(ladmm_server *sv, Lane *L, int rc, const std::string &msg,
               std::vector<std::pair<Request *, int>> *finals) {
  std::vector<Request *> rs;
  for (Request *r : L->owner)
    if (r && std::find(rs.begin(), rs.end(), r) == rs.end()) rs.push_back(r);
  for (Request *r : rs) {
    drop(sv, r);
    finals->push_back({r, rc});
    r->err = msg;
  }
  for (size_t i = 0; i < sv->lanes.size(); ++i)
    if (sv->lanes[i].get() == L) {
      free_lane(L);
      sv->lanes.erase(sv->lanes.begin() + i);
      break;
    }
}

// Copy the results of the finished slots of a lane into their requests.
int retire(ladmm_server *sv, Lane &L, std::vector<Request *> *touched) {
  ladmm_case *c = L.c;
  ladmm_batch *b = L.b;
  bool any = false;
  for (int s = 0; s < b->kp; ++s) any |= L.owner[s] && !b->h_active[s];
  if (!any) return LADMM_OK;
  HIPC(extract_t(b->stream, small_args(b), b->q2, L.d_t, b->kp));
  HIPC(hipMemcpyAsync(L.h_t, L.d_t, (size_t)b->kp * c->n_t * sizeof(double), hipMemcpyDeviceToHost,
                      b->stream));
  HIPC(hipStreamSynchronize(b->stream));
  // converged plans enter the warm store (oldest entry replaced)
  WarmCols wc{};
  auto flush = [&]() -> int {
    if (wc.n == 0) return LADMM_OK;
    if (c->precision == LADMM_F64) {
      HIPC(warm_save<double>(b->stream, wc, (const double *)b->q, b->q2, b->qs, c->Np, c->mAp,
                             c->n_sec, b->kp, (double *)L.wq, L.wq2, L.wqs));
    } else {
      HIPC(warm_save<float>(b->stream, wc, (const float *)b->q, b->q2, b->qs, c->Np, c->mAp,
                            c->n_sec, b->kp, (float *)L.wq, L.wq2, L.wqs));
    }
    wc.n = 0;
    return LADMM_OK;
  };
  for (int s = 0; s < b->kp; ++s) {
    Request *r = L.owner[s];
    if (!r || b->h_active[s]) continue;
    if (L.wcap > 0 && b->status[s] == LADMM_PLAN_CONVERGED) {
      const int e = L.wnext;
      L.wnext = (L.wnext + 1) % L.wcap;
      L.wcount = std::min(L.wcount + 1, L.wcap);
      L.ww[e] = b->w[s];
      L.wrho[e] = b->rho[s];
      wc.col[wc.n] = s;
      wc.ent[wc.n] = e;
      if (++wc.n == kWarmCols) {
        int rc = flush();
        if (rc) return rc;
      }
    }
    const int p = L.plan[s];
    const double *t = L.h_t + (size_t)s * c->n_t;
    const double *f = &b->rec[(size_t)s * kFinal];
    ladmm_result &o = r->out;
    if (o.t) std::memcpy(o.t + (size_t)p * c->n_t, t, c->n_t * sizeof(double));
    if (o.bot) bot_from_t(c, t, o.bot + (size_t)p * c->n_iso);
    if (o.objective) o.objective[p] = f[0];
    if (o.dual_obj) o.dual_obj[p] = f[1];
    if (o.rel_gap) o.rel_gap[p] = f[2];
    if (o.r_pri) o.r_pri[p] = f[3];
    if (o.r_dual) o.r_dual[p] = f[4];
    if (o.iters) o.iters[p] = b->iters[s];
    if (o.plan_status) o.plan_status[p] = b->status[s];
    if (o.lower_bound) o.lower_bound[p] = f[8];
    if (o.cert_gap) o.cert_gap[p] = f[9];
    L.owner[s] = nullptr;
    L.plan[s] = -1;
    L.dirty = true;
    r->in_slots--;
    touched->push_back(r);
  }
  return flush();
}

void worker_main(ladmm_server *sv) {
  hipSetDevice(sv->ctx->device);
  for (;;) {
    // 1. intake
    std::vector<Request *> cancelled;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      auto has_work = [&]() {
        if (sv->stop || !sv->incoming.empty() || sv->cancel_pending) return true;
        for (auto &L : sv->lanes)
          if (L->busy()) return true;
        return !sv->pending.empty();
      };
      sv->cv_work.wait(lk, has_work);
      if (sv->stop) break;
      for (Request *r : sv->incoming) {
        sv->pending.push_back(r);
        sv->live.push_back(r);
      }
      sv->incoming.clear();
      if (sv->cancel_pending) {
        for (Request *r : sv->live)
          if (r->cancel) cancelled.push_back(r);
        sv->cancel_pending = false;
      }
    }
    std::vector<std::pair<Request *, int>> finals;   // requests reaching a final status
    for (Request *r : cancelled) {
      drop(sv, r);
      finals.push_back({r, LADMM_E_CANCELLED});
    }
    // 2. admission, oldest request first
    for (size_t i = 0; i < sv->pending.size();) {
      Request *r = sv->pending[i];
      Lane *L = nullptr;
      int rc = lane_for(sv, r->c, &L);
      if (rc == LADMM_PENDING) {
        ++i;
        continue;
      }
      if (rc != LADMM_OK) {
        r->err = g_err;
        drop(sv, r);   // removes it from pending
        finals.push_back({r, rc});
        continue;
      }
      for (int s = 0; s < L->b->kp && r->next < r->k; ++s)
        if (!L->owner[s]) {
          admit(*L, s, r, r->next);
          sv->warm_round += L->warm_src[s] >= 0;
        }
      if (r->next == r->k)
        sv->pending.erase(sv->pending.begin() + i);
      else
        ++i;
    }
    // 3. launch every lane with work
    const int K = sv->opts.check_every;
    auto t0 = Clock::now();
    int64_t pit = 0;
    std::vector<Lane *> run;
    for (auto &L : sv->lanes) {
      int rc = LADMM_OK;
      if (L->dirty) rc = upload(*L);
      if (rc == LADMM_OK && L->busy()) {
        rc = chunk_launch(L->b, K);
        if (rc == LADMM_OK) run.push_back(L.get());
      } else if (rc == LADMM_OK) {
        // the host mirrors may change next round: let the copies finish
        if (hipStreamSynchronize(L->b->stream) != hipSuccess)
          rc = fail(LADMM_E_DEVICE, "lane stream synchronization failed");
        std::fill(L->h_reset, L->h_reset + L->b->kp, 0);
        L->any_reset = false;
      }
      if (rc) {
        // the lane's stream is synchronized by its release
        Lane *bad = L.get();
        fail_lane(sv, bad, rc, g_err, &finals);
        break;   // lanes changed; the remaining lanes launch next round
      }
    }
    // 4. completion, stopping rules, retirement
    std::vector<Request *> touched;
    int busy_slots = 0;
    for (Lane *L : run) {
      bool changed = false;
      const int active = L->b->chunk_active;
      int rc = chunk_complete(L->b, K, true, &changed);
      if (rc == LADMM_OK) rc = retire(sv, *L, &touched);
      if (rc == LADMM_OK) {
        // step-size balancing of the running plans; keep the table mirror in step
        bool switched = false;
        rc = adapt_rho(L->b, &switched);
        if (rc == LADMM_OK && switched)
          for (int s = 0; s < L->b->kp; ++s)
            if (L->owner[s]) L->h_invrho[s] = 1.0 / L->b->rho[s];
      }
      if (rc) {
        fail_lane(sv, L, rc, g_err, &finals);
        continue;
      }
      pit += (int64_t)K * active;
      std::fill(L->h_reset, L->h_reset + L->b->kp, 0);
      L->any_reset = false;
      L->last_used = Clock::now();
    }
    // lanes of destroyed cases with no work are released
    for (size_t i = 0; i < sv->lanes.size();) {
      Lane *L = sv->lanes[i].get();
      if (L->busy() == 0 && L->c->destroyed) {
        free_lane(L);
        sv->lanes.erase(sv->lanes.begin() + i);
      } else {
        ++i;
      }
    }
    for (auto &L : sv->lanes) busy_slots += L->busy();
    const double round_ms = std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    std::vector<ladmm_case *> unrefs;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (!run.empty()) sv->busy_ms += round_ms;
      sv->plan_iterations += pit;
      sv->warm_starts += sv->warm_round;
      sv->warm_round = 0;
      for (Request *r : touched) {
        r->done++;
        sv->plans_retired++;
      }
        // a request is handed to the callers by its final status; after that the
      // worker no longer touches it (a caller may release it at once)
      for (Request *r : touched)
        if (r->status == LADMM_PENDING && r->done == r->k) {
          sv->live.erase(std::remove(sv->live.begin(), sv->live.end(), r), sv->live.end());
          unrefs.push_back(r->c);
          r->c = nullptr;
          finish_locked(sv, r, LADMM_OK, "");
        }
      for (auto &f : finals)
        if (f.first->status == LADMM_PENDING) {
          unrefs.push_back(f.first->c);
          f.first->c = nullptr;
          finish_locked(sv, f.first, f.second, f.first->err);
        }
      sv->n_lanes = (int32_t)sv->lanes.size();
      sv->busy_slots = busy_slots;
    }
    for (ladmm_case *c : unrefs)
      if (c) case_unref(c);
    sv->cv_done.notify_all();
  }
  // shutdown: every request not final is cancelled; lanes are released
  for (auto &L : sv->lanes) free_lane(L.get());
  sv->lanes.clear();
  std::lock_guard<std::mutex> lk(sv->mu);
  for (Request *r : sv->incoming) sv->live.push_back(r);
  sv->incoming.clear();
  for (Request *r : sv->live)
    if (r->status == LADMM_PENDING) {
      finish_locked(sv, r, LADMM_E_CANCELLED, "server destroyed");
      if (r->c) case_unref(r->c);
      r->c = nullptr;
    }
  sv->live.clear();
  sv->pending.clear();
  sv->cv_done.notify_all();
}

// Report a final status to the caller and release the ticket.
int report_locked(ladmm_server *sv, std::map<uint64_t, Request *>::iterator it) {
  Request *r = it->second;
  const int st = r->status;
  if (st < 0 && !r->err.empty()) g_err = r->err;
  sv->tickets.erase(it);
  delete r;
  return st;
}

int validate_weights(int32_t k, const ladmm_weights *w) {
  for (int j = 0; j < k; ++j) {
    const ladmm_weights &x = w[j];
    if (!(x.w_bot > 0) || !std::isfinite(x.w_bot))
      return fail(LADMM_E_INVALID, "plan " + std::to_string(j) + ": w_bot must be > 0");
    if (!(x.w_t >= 0) || !(x.w_r >= 0) || !(x.w_ld >= 0) || !std::isfinite(x.w_t) ||
        !std::isfinite(x.w_r) || !std::isfinite(x.w_ld))
      return fail(LADMM_E_INVALID, "plan " + std::to_string(j) + ": weights must be finite and >= 0");
  }
  return LADMM_OK;
}

}  // namespace

extern "C" {

int ladmm_server_create(ladmm_ctx *ctx, const ladmm_server_opts *opts, ladmm_server **out) {
  if (!ctx || !opts || !out) return fail(LADMM_E_INVALID, "server_create: null argument");
  if (opts->slots < 1 || opts->slots > 4096 || opts->check_every < 1 || opts->max_lanes < 0 ||
      opts->warm_store < 0 || opts->warm_store > 65536)
    return fail(LADMM_E_INVALID, "server_create: slots in [1, 4096], check_every >= 1, "
                                 "max_lanes >= 0, warm_store in [0, 65536]");
  ladmm_server *sv = new ladmm_server();
  sv->ctx = ctx;
  sv->opts = *opts;
  try {
    sv->worker = std::thread(worker_main, sv);
  } catch (const std::exception &e) {
    delete sv;
    return fail(LADMM_E_STATE, std::string("server_create: ") + e.what());
  }
  *out = sv;
  return LADMM_OK;
}

int ladmm_server_destroy(ladmm_server *sv) {
  if (!sv) return LADMM_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (auto &t : sv->tickets) delete t.second;
  delete sv;
  return LADMM_OK;
}

int ladmm_submit(ladmm_server *sv, ladmm_case *c, int32_t k, const ladmm_weights *w,
                 const uint64_t *ld_mask, const ladmm_opts *opts, ladmm_result *out,
                 uint64_t *ticket) {
  if (!sv || !c || !w || !opts || !out || !ticket) return fail(LADMM_E_INVALID, "submit: null argument");
  if (c->ctx != sv->ctx) return fail(LADMM_E_INVALID, "submit: case belongs to another context");
  if (k < 1) return fail(LADMM_E_INVALID, "submit: k must be >= 1");
  if (opts->max_iter < 1) return fail(LADMM_E_INVALID, "submit: max_iter must be >= 1");
  if (opts->check_every != 0 && opts->check_every != sv->opts.check_every)
    return fail(LADMM_E_INVALID, "submit: check_every must be 0 or the server's");
  if (!(opts->rho0 > 0) || !(opts->w0_bot > 0)) return fail(LADMM_E_INVALID, "submit: rho0 and w0_bot must be > 0");
  if (opts->alpha != 0.0 && opts->alpha != 1.0)
    return fail(LADMM_E_INVALID, "submit: served plans run without over-relaxation (alpha 0 or 1)");
  if (opts->adapt_rho && (!(opts->adapt_mu > 1) || !(opts->adapt_tau > 1) ||
                          !std::isfinite(opts->adapt_mu) || !std::isfinite(opts->adapt_tau)))
    return fail(LADMM_E_INVALID, "submit: adapt_mu and adapt_tau must be finite and > 1");
  int rc = validate_weights(k, w);
  if (rc) return rc;
  Request *r = new Request();
  r->k = k;
  r->w.assign(w, w + k);
  if (ld_mask) r->mask.assign(ld_mask, ld_mask + (size_t)k * ((c->N + 63) / 64));
  const int K = sv->opts.check_every;
  r->opts = *opts;
  r->max_iter = (opts->max_iter + K - 1) / K * K;
  r->out = *out;
  rc = case_ref(c);
  if (rc) {
    delete r;
    return rc;
  }
  r->c = c;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      case_unref(c);
      delete r;
      return fail(LADMM_E_STATE, "submit: server is shutting down");
    }
    r->ticket = sv->next_ticket++;
    sv->tickets[r->ticket] = r;
    sv->incoming.push_back(r);
    sv->submitted++;
    *ticket = r->ticket;
  }
  sv->cv_work.notify_all();
  return LADMM_OK;
}

int ladmm_poll(ladmm_server *sv, uint64_t ticket, int32_t *plans_done) {
  if (!sv) return fail(LADMM_E_INVALID, "poll: null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(LADMM_E_STATE, "poll: unknown or released ticket");
  if (plans_done) *plans_done = it->second->done;
  if (it->second->status == LADMM_PENDING) return LADMM_PENDING;
  return report_locked(sv, it);
}

int ladmm_wait(ladmm_server *sv, uint64_t ticket, int64_t timeout_us) {
  if (!sv) return fail(LADMM_E_INVALID, "wait: null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(LADMM_E_STATE, "wait: unknown or released ticket");
  // the ticket is looked up on every wake-up: another caller may release it
  auto ready = [&]() {
    auto i = sv->tickets.find(ticket);
    return i == sv->tickets.end() || i->second->status != LADMM_PENDING;
  };
  if (timeout_us < 0)
    sv->cv_done.wait(lk, ready);
  else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return LADMM_PENDING;
  it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(LADMM_E_STATE, "wait: ticket released by another caller");
  return report_locked(sv, it);
}

int ladmm_cancel(ladmm_server *sv, uint64_t ticket) {
  if (!sv) return fail(LADMM_E_INVALID, "cancel: null server");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(LADMM_E_STATE, "cancel: unknown or released ticket");
    if (it->second->status != LADMM_PENDING) return LADMM_OK;   // already final
    it->second->cancel = true;
    sv->cancel_pending = true;
  }
  sv->cv_work.notify_all();
  return LADMM_OK;
}

int ladmm_server_reset_stats(ladmm_server *sv) {
  if (!sv) return fail(LADMM_E_INVALID, "server_reset_stats: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->submitted = sv->completed = sv->cancelled = sv->failed = sv->plans_retired = 0;
  sv->plan_iterations = sv->warm_starts = 0;
  sv->busy_ms = 0.0;
  sv->latency_ms.clear();
  return LADMM_OK;
}

int ladmm_server_get_stats(ladmm_server *sv, ladmm_server_stats *out) {
  if (!sv || !out) return fail(LADMM_E_INVALID, "server_get_stats: null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  ladmm_server_stats s{};
  s.submitted = sv->submitted;
  s.completed = sv->completed;
  s.cancelled = sv->cancelled;
  s.failed = sv->failed;
  s.plans_completed = sv->plans_retired;
  s.plan_iterations = sv->plan_iterations;
  s.warm_starts = sv->warm_starts;
  s.busy_ms = sv->busy_ms;
  s.lanes = sv->n_lanes;
  s.busy_slots = sv->busy_slots;
  std::vector<double> lat = sv->latency_ms;
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto rank = [&](double q) {   // nearest-rank percentile
      size_t i = (size_t)std::ceil(q * (double)lat.size());
      return lat[std::min(lat.size(), std::max<size_t>(i, 1)) - 1];
    };
    s.p50_ms = rank(0.50);
    s.p99_ms = rank(0.99);
    s.max_ms = lat.back();
    double sum = 0.0;
    for (double x : lat) sum += x;
    s.mean_ms = sum / (double)lat.size();
  }
  *out = s;
  return LADMM_OK;
}

}  // extern "C"
