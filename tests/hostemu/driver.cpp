#include <algorithm>
// Drives libladmm's C ABI, built for the host emulation, on inputs written by
// the Python test (tests/test_hostemu.py), and writes what it computed.
//   driver <dir>   reads  <dir>/meta.txt, dose.f64, group.i32, groups.txt,
//                          weights.f64 [, mask.u64] [, vols.u64, nld.i32] [, vox.f64]
//                  writes <dir>/S.f64, Sinv.f64, E.f64, z1.f64, y1.f64, z2.f64,
//                          y2.f64, res.f64 [, P.i64, masks.u64] [, band.u64]
#include <cstdio>
#include <fstream>
#include <string>
#include <vector>

#include "ladmm.h"

template <typename T>
static std::vector<T> load(const std::string &path, size_t n) {
  std::vector<T> v(n);
  FILE *f = fopen(path.c_str(), "rb");
  if (!f) return {};
  size_t got = fread(v.data(), sizeof(T), n, f);
  fclose(f);
  if (got != n) { fprintf(stderr, "short read %s\n", path.c_str()); exit(2); }
  return v;
}

template <typename T>
static void save(const std::string &path, const T *p, size_t n) {
  FILE *f = fopen(path.c_str(), "wb");
  fwrite(p, sizeof(T), n, f);
  fclose(f);
}

#define CHECK(x)                                                           \
  do {                                                                     \
    int rc_ = (x);                                                         \
    if (rc_ < 0) {                                                         \
      fprintf(stderr, "%s failed: %d %s\n", #x, rc_, ladmm_last_error());  \
      return 3;                                                            \
    }                                                                      \
  } while (0)

int main(int argc, char **argv) {
  if (argc < 2) return 1;
  const std::string dir = argv[1];
  std::ifstream meta(dir + "/meta.txt");
  int N, n_iso, S, C, G, precision, k, iters, use_mask, n_vols, n_vox, band_vox, solve_iters;
  int tile1 = -1, tile2 = -1, run_two_pass = 0, serve = 0, compact_iters = 0;
  double rho0, w0, D_T, phi_cal, d_ld, delta;
  unsigned long long seed;
  meta >> N >> n_iso >> S >> C >> G >> precision >> k >> iters >> rho0 >> w0 >> D_T >> phi_cal >>
      use_mask >> n_vols >> n_vox >> seed >> band_vox >> d_ld >> delta >> solve_iters >> tile1 >> tile2 >> run_two_pass >> serve >> compact_iters;
  const int n_t = n_iso * S * C, m_A = n_t + n_iso, n_A = N + n_iso * S;
  auto dose = load<double>(dir + "/dose.f64", (size_t)N * n_t);
  auto grp = load<int32_t>(dir + "/group.i32", N);
  std::vector<ladmm_group> groups(G);
  std::ifstream gf(dir + "/groups.txt");
  for (auto &g : groups) gf >> g.type >> g.structure >> g.threshold >> g.share;
  auto wv = load<double>(dir + "/weights.f64", (size_t)k * 4);
  std::vector<ladmm_weights> w(k);
  for (int j = 0; j < k; ++j) w[j] = {wv[4 * j], wv[4 * j + 1], wv[4 * j + 2], wv[4 * j + 3]};

  ladmm_ctx *ctx = nullptr;
  CHECK(ladmm_ctx_create(0, 0, &ctx));
  ladmm_case_desc d{};
  d.n_points = N; d.n_iso = n_iso; d.n_sectors = S; d.n_collimators = C;
  d.dose = dose.data(); d.point_group = grp.data(); d.n_groups = G; d.groups = groups.data();
  d.prescription_mean = D_T; d.phi_cal = phi_cal; d.precision = precision; d.row_normalize = 1;
  d.beta = 0.0; d.beta_denominator = 2000.0;
  ladmm_case *cs = nullptr;
  CHECK(ladmm_create_case(ctx, &d, &cs));
  std::vector<double> Sm((size_t)m_A * m_A), Si((size_t)m_A * m_A), E(m_A);
  double beta = 0;
  CHECK(ladmm_case_schur(cs, Sm.data(), Si.data()));
  CHECK(ladmm_case_scaling(cs, E.data(), &beta));
  save(dir + "/S.f64", Sm.data(), Sm.size());
  save(dir + "/Sinv.f64", Si.data(), Si.size());
  save(dir + "/E.f64", E.data(), E.size());

  const int W = (N + 63) / 64;
  std::vector<uint64_t> mask;
  if (use_mask) mask = load<uint64_t>(dir + "/mask.u64", (size_t)k * W);
  ladmm_opts o{};
  o.max_iter = 1000; o.check_every = 7; o.tol_gap = 0.0; o.tol_pri = 1; o.tol_dual = 1;
  o.rho0 = rho0; o.w0_bot = w0; o.autotune = 1;
  if (!serve) {
  ladmm_batch *b = nullptr;
  CHECK(ladmm_batch_create(cs, k, w.data(), use_mask ? mask.data() : nullptr, nullptr, &o, &b));
  if (tile1 >= 0) CHECK(ladmm_batch_set_tiles(b, tile1, tile2));
  CHECK(ladmm_batch_iterate(b, iters));
  {
    int32_t used[2] = {-1, -1};
    CHECK(ladmm_batch_tiles(b, &used[0], &used[1]));
    save(dir + "/tiles.i32", used, 2);
  }
  std::vector<double> z1((size_t)n_A * k), y1((size_t)n_A * k), z2((size_t)m_A * k), y2((size_t)m_A * k);
  CHECK(ladmm_batch_export(b, z1.data(), y1.data(), z2.data(), y2.data()));
  save(dir + "/z1.f64", z1.data(), z1.size());
  save(dir + "/y1.f64", y1.data(), y1.size());
  save(dir + "/z2.f64", z2.data(), z2.size());
  save(dir + "/y2.f64", y2.data(), y2.size());
  std::vector<double> res((size_t)k * 7), t((size_t)k * n_t), bot((size_t)k * n_iso);
  std::vector<int32_t> it(k), st(k);
  ladmm_result r{t.data(), bot.data(), &res[0], &res[k], &res[2 * k], &res[3 * k], &res[4 * k],
                 it.data(), st.data(), &res[5 * k], &res[6 * k]};
  CHECK(ladmm_batch_results(b, &r));
  save(dir + "/res.f64", res.data(), res.size());
  save(dir + "/t.f64", t.data(), t.size());
  if (band_vox > 0 && !run_two_pass) {
    auto vox = load<double>(dir + "/vox.f64", (size_t)band_vox * n_t);
    std::vector<uint64_t> bits((size_t)k * ((band_vox + 63) / 64));
    CHECK(ladmm_batch_ld_band(b, band_vox, vox.data(), d_ld, delta, bits.data()));
    save(dir + "/band.u64", bits.data(), bits.size());
  }
  // re-import the exported state and continue (exercises import and W rebuild)
  CHECK(ladmm_batch_import(b, z1.data(), y1.data(), z2.data(), y2.data()));
  CHECK(ladmm_batch_iterate(b, 1));
  CHECK(ladmm_batch_export(b, z1.data(), y1.data(), z2.data(), y2.data()));
  save(dir + "/z1b.f64", z1.data(), z1.size());
  CHECK(ladmm_batch_destroy(b));
  if (solve_iters > 0) {
    ladmm_opts so = o;
    so.max_iter = solve_iters; so.check_every = 5; so.tol_gap = 1e-6; so.tol_pri = 1e-6; so.tol_dual = 1e-6;
    so.adapt_rho = 1; so.adapt_mu = 1.5; so.adapt_tau = 2.0;   // step-size switches at every check
    CHECK(ladmm_solve_batch(cs, k, w.data(), use_mask ? mask.data() : nullptr, &so, &r));
  }
  if (compact_iters > 0) {
    // plans that stop at different checks, run with compaction on and off
    ladmm_opts co = o;
    co.max_iter = compact_iters; co.check_every = 2; co.tol_gap = 0.2; co.tol_pri = 0; co.tol_dual = 0;
    co.autotune = 1;
    for (int on = 1; on >= 0; --on) {
      ladmm_batch *cb = nullptr;
      CHECK(ladmm_batch_create(cs, k, w.data(), use_mask ? mask.data() : nullptr, nullptr, &co, &cb));
      CHECK(ladmm_batch_set_compaction(cb, on));
      CHECK(ladmm_batch_run(cb));
      CHECK(ladmm_batch_results(cb, &r));
      const std::string tag = on ? "on" : "off";
      save(dir + "/compact_t_" + tag + ".f64", t.data(), t.size());
      save(dir + "/compact_res_" + tag + ".f64", res.data(), res.size());
      save(dir + "/compact_it_" + tag + ".i32", it.data(), it.size());
      CHECK(ladmm_batch_export(cb, z1.data(), y1.data(), z2.data(), y2.data()));
      save(dir + "/compact_z1_" + tag + ".f64", z1.data(), z1.size());
      CHECK(ladmm_batch_destroy(cb));
    }
  }
  }
  if (n_vols > 0) {
    const int Wv = (n_vox + 63) / 64;
    auto vols = load<uint64_t>(dir + "/vols.u64", (size_t)n_vols * Wv);
    auto nld = load<int32_t>(dir + "/nld.i32", n_vols);
    std::vector<int64_t> P(n_vox);
    std::vector<uint64_t> masks((size_t)n_vols * Wv);
    int64_t nP = 0;
    CHECK(ladmm_select_ld_points(ctx, n_vols, n_vox, vols.data(), nld.data(), seed, P.data(), &nP, masks.data()));
    save(dir + "/P.i64", P.data(), (size_t)nP);
    save(dir + "/masks.u64", masks.data(), masks.size());
    // the allocation-free variant (static scratch), twice: the second call on
    // the first plans only (a smaller input into the used scratch)
    for (int rep = 0; rep < 2; ++rep) {
      const int kk = rep == 0 ? n_vols : std::max(1, n_vols / 2);
      std::fill(P.begin(), P.end(), -1);
      std::fill(masks.begin(), masks.end(), 0);
      CHECK(ladmm_select_ld_points_static(ctx, kk, n_vox, vols.data(), nld.data(), seed, P.data(), &nP,
                                          masks.data()));
      save(dir + "/P_static" + std::to_string(rep) + ".i64", P.data(), (size_t)nP);
      save(dir + "/masks_static" + std::to_string(rep) + ".u64", masks.data(), (size_t)kk * Wv);
    }
  }
  if (band_vox > 0 && run_two_pass) {
    // both passes, a few fixed iterations each
    // one second-pass set per low-dose group: threshold d_ld / (i + 1), seed + 1 + i
    auto vox = load<double>(dir + "/vox.f64", (size_t)band_vox * n_t);
    std::vector<int> ldg;
    for (int g = 0; g < G; ++g)
      if (groups[g].type == LADMM_PT_LD) ldg.push_back(g);
    const int ns = (int)ldg.size();
    std::vector<int32_t> nld(k, 25);
    std::vector<ladmm_pass2_desc> sets(ns);
    for (int i = 0; i < ns; ++i)
      sets[i] = ladmm_pass2_desc{band_vox, vox.data(), d_ld / (i + 1), delta, nld.data(),
                                 seed + 1 + (uint64_t)i, ldg[i]};
    ladmm_opts to = o;
    to.max_iter = 6; to.check_every = 3; to.tol_gap = 0.0; to.autotune = 0;
    std::vector<double> t1((size_t)k * n_t), t2((size_t)k * n_t), f2(k);
    std::vector<int32_t> it1(k), st1(k), it2(k), st2(k);
    ladmm_result r1{t1.data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, it1.data(), st1.data()};
    ladmm_result r2{t2.data(), nullptr, f2.data(), nullptr, nullptr, nullptr, nullptr, it2.data(), st2.data()};
    std::vector<int64_t> P((size_t)band_vox * ns);
    std::vector<int64_t> n2(ns + 1, 0);
    const int n_passes = run_two_pass == 1 ? 2 : run_two_pass;
    std::vector<double> times(2 + 3 * (n_passes - 1));
    std::vector<std::vector<double>> tmid(n_passes);
    if (n_passes > 2) {
      // every pass's shot times (the middle ones let the test redo each selection)
      std::vector<ladmm_result> rs(n_passes);
      for (int q = 0; q < n_passes; ++q) {
        tmid[q].resize((size_t)k * n_t);
        rs[q] = ladmm_result{tmid[q].data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr};
      }
      rs[0] = r1;
      rs[n_passes - 1] = r2;
      CHECK(ladmm_passes(ctx, &d, k, w.data(), &to, ns, sets.data(), n_passes, rs.data(), P.data(),
                         n2.data(), times.data()));
      for (int q = 1; q + 1 < n_passes; ++q)
        save(dir + "/tp_tmid" + std::to_string(q + 1) + ".f64", tmid[q].data(), tmid[q].size());
    } else if (ns == 1) {
      CHECK(ladmm_two_pass(ctx, &d, k, w.data(), &to, &sets[0], &r1, &r2, P.data(), n2.data(),
                           times.data()));
    } else {
      CHECK(ladmm_two_pass_sets(ctx, &d, k, w.data(), &to, ns, sets.data(), &r1, &r2, P.data(),
                                n2.data(), times.data()));
    }
    int64_t total = 0;
    for (int i = 0; i < ns; ++i) total += n2[i];
    save(dir + "/tp_t1.f64", t1.data(), t1.size());
    save(dir + "/tp_t2.f64", t2.data(), t2.size());
    save(dir + "/tp_f2.f64", f2.data(), f2.size());
    save(dir + "/tp_P.i64", P.data(), (size_t)total);
    save(dir + "/tp_n.i64", n2.data(), n2.size());
  }
  if (serve) {
    // Continuous batching on 32 slots: a long request cancelled at once, then
    // request A (k - 6 plans, 2K iterations) and B (6 plans, K iterations), so
    // B's later plans start in slots freed by its earlier ones.  The same plans
    // are also solved alone with ladmm_solve_batch for a bitwise comparison.
    const int K = 2, kA = k - 6, kB = 6;
    ladmm_server_opts sopt{32, K, 0, 0};
    ladmm_server *sv = nullptr;
    CHECK(ladmm_server_create(ctx, &sopt, &sv));
    ladmm_opts ro = o;
    ro.check_every = 0; ro.tol_gap = 0.0; ro.autotune = 0;
    ladmm_opts oc = ro, oa = ro, ob = ro;
    oc.max_iter = 1000; oa.max_iter = 2 * K; ob.max_iter = K;
    std::vector<double> tc(n_t);
    ladmm_result rc{tc.data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    uint64_t tkc = 0, tka = 0, tkb = 0;
    CHECK(ladmm_submit(sv, cs, 1, &w[0], nullptr, &oc, &rc, &tkc));
    CHECK(ladmm_cancel(sv, tkc));
    const int nreq = 2;
    const int kk[nreq] = {kA, kB}, off[nreq] = {0, kA};
    std::vector<double> tt[nreq], ff[nreq], rt[nreq], rf[nreq];
    std::vector<int32_t> ii[nreq], ss[nreq], ri[nreq], rs[nreq];
    ladmm_result rr[nreq], ref[nreq];
    for (int q = 0; q < nreq; ++q) {
      tt[q].resize((size_t)kk[q] * n_t); ff[q].resize(kk[q]); ii[q].resize(kk[q]); ss[q].resize(kk[q]);
      rt[q].resize((size_t)kk[q] * n_t); rf[q].resize(kk[q]); ri[q].resize(kk[q]); rs[q].resize(kk[q]);
      rr[q] = ladmm_result{tt[q].data(), nullptr, ff[q].data(), nullptr, nullptr, nullptr, nullptr,
                           ii[q].data(), ss[q].data()};
      ref[q] = ladmm_result{rt[q].data(), nullptr, rf[q].data(), nullptr, nullptr, nullptr, nullptr,
                            ri[q].data(), rs[q].data()};
    }
    const uint64_t *ma = use_mask ? mask.data() : nullptr;
    const uint64_t *mb = use_mask ? mask.data() + (size_t)kA * W : nullptr;
    CHECK(ladmm_submit(sv, cs, kA, &w[0], ma, &oa, &rr[0], &tka));
    CHECK(ladmm_submit(sv, cs, kB, &w[kA], mb, &ob, &rr[1], &tkb));
    if (ladmm_wait(sv, tkc, -1) != LADMM_E_CANCELLED) { fprintf(stderr, "cancel failed\n"); return 4; }
    CHECK(ladmm_wait(sv, tka, -1));
    CHECK(ladmm_wait(sv, tkb, -1));
    if (ladmm_poll(sv, tka, nullptr) != LADMM_E_STATE) { fprintf(stderr, "ticket not released\n"); return 4; }
    ladmm_server_stats st{};
    CHECK(ladmm_server_get_stats(sv, &st));
    if (st.completed != 2 || st.cancelled != 1 || st.plans_completed != k) {
      fprintf(stderr, "stats %lld %lld %lld\n", (long long)st.completed, (long long)st.cancelled,
              (long long)st.plans_completed);
      return 4;
    }
    CHECK(ladmm_server_destroy(sv));
    ladmm_opts sa = oa, sb = ob;
    sa.check_every = K; sb.check_every = K;
    CHECK(ladmm_solve_batch(cs, kA, &w[0], ma, &sa, &ref[0]));
    CHECK(ladmm_solve_batch(cs, kB, &w[kA], mb, &sb, &ref[1]));
    for (int q = 0; q < nreq; ++q) {
      const std::string tag = q == 0 ? "A" : "B";
      save(dir + "/serve_t" + tag + ".f64", tt[q].data(), tt[q].size());
      save(dir + "/serve_f" + tag + ".f64", ff[q].data(), ff[q].size());
      save(dir + "/serve_i" + tag + ".i32", ii[q].data(), ii[q].size());
      save(dir + "/alone_t" + tag + ".f64", rt[q].data(), rt[q].size());
      save(dir + "/alone_f" + tag + ".f64", rf[q].data(), rf[q].size());
      save(dir + "/alone_i" + tag + ".i32", ri[q].data(), ri[q].size());
    }
    (void)off;
    // Warm starts: the last 6 plans twice on a server with a store.  Loose
    // tolerances let every plan converge at its first check and enter the
    // store; the second request starts from it (nearest weighting = itself), so
    // its K iterations continue the first request's: the result is that of 2K
    // iterations from cold (same step sizes; the balancing is off here).
    {
      ladmm_server_opts wopt{32, K, 0, 0, 0, 16};
      ladmm_server *ws = nullptr;
      CHECK(ladmm_server_create(ctx, &wopt, &ws));
      ladmm_opts ow = ro;
      ow.max_iter = 1000; ow.tol_gap = 1e30; ow.tol_pri = 1e30; ow.tol_dual = 1e30;
      std::vector<double> f1(kB), f2(kB), t2((size_t)kB * n_t), f3(kB), t3((size_t)kB * n_t);
      std::vector<int32_t> i1(kB), i2(kB), s1(kB), s2(kB), i3(kB), s3(kB);
      ladmm_result r1{nullptr, nullptr, f1.data(), nullptr, nullptr, nullptr, nullptr, i1.data(), s1.data()};
      ladmm_result r2{t2.data(), nullptr, f2.data(), nullptr, nullptr, nullptr, nullptr, i2.data(), s2.data()};
      ladmm_result r3{t3.data(), nullptr, f3.data(), nullptr, nullptr, nullptr, nullptr, i3.data(), s3.data()};
      uint64_t t1 = 0, tw = 0;
      CHECK(ladmm_submit(ws, cs, kB, &w[kA], mb, &ow, &r1, &t1));
      CHECK(ladmm_wait(ws, t1, -1));
      CHECK(ladmm_submit(ws, cs, kB, &w[kA], mb, &ow, &r2, &tw));
      CHECK(ladmm_wait(ws, tw, -1));
      ladmm_server_stats wst{};
      CHECK(ladmm_server_get_stats(ws, &wst));
      if (wst.warm_starts != kB) {
        fprintf(stderr, "warm starts %lld\n", (long long)wst.warm_starts);
        return 4;
      }
      CHECK(ladmm_server_destroy(ws));
      ladmm_opts o2 = ro;
      o2.max_iter = 2 * K; o2.check_every = K;
      CHECK(ladmm_solve_batch(cs, kB, &w[kA], mb, &o2, &r3));
      save(dir + "/warm_t.f64", t2.data(), t2.size());
      save(dir + "/warm_f.f64", f2.data(), f2.size());
      save(dir + "/warm_i.i32", i2.data(), i2.size());
      save(dir + "/cold2_t.f64", t3.data(), t3.size());
      save(dir + "/cold2_f.f64", f3.data(), f3.size());
    }
  }
  CHECK(ladmm_destroy_case(cs));
  CHECK(ladmm_ctx_destroy(ctx));
  return 0;
}
