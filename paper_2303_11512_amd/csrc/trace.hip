// Trace estimators on the GPU: plain Hutchinson (Alg. 1), Hutch++ (Sec. 2.4),
// MG-MLMC (Sec. 3.1) and MG-MLMC++ (Alg. 2).
//
// Every vector operation runs in the library's kernels: noise, multigrid
// solves, restriction/prolongation, CholQR, projections and sample dot
// products.  The host only keeps Alg. 2's scalars.  Samples are evaluated
// `batch` at a time for every active level difference (their noise is
// counter-based, so sample s of level l is the same vector whatever the
// batching), and the stopping rule is then replayed sample by sample in index
// order; samples past a level's stopping point are discarded.  The result
// therefore equals the sequential algorithm's on the same seeds.
#include <cmath>
#include <complex>

#include "internal.h"

namespace mgm {

int solve_chunked(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* b, cd* x,
                  const mgm_solve_params& sp, int* iters, double* relres);

namespace {

using zc = std::complex<double>;

struct StochLevel {
  int level = 0;       // operator level of the finer side
  int64_t n = 0;       // noise length
  int d = 0;           // Hutch++ vectors
  double cost = 0;
  zc tau_lr = 0;
  std::vector<zc> samples;
  bool active = true;
  DevBuf* Q = nullptr; // [d][n], owned by the field's estimator workspace
  int s() const { return (int)samples.size(); }
  zc mean() const {
    if (samples.empty()) return 0.0;
    zc acc = 0;
    for (const zc& v : samples) acc += v;
    return acc / (double)samples.size();
  }
  double var() const {
    if (samples.size() < 2) return std::nan("");
    const zc mu = mean();
    double acc = 0;
    for (const zc& v : samples) acc += std::norm(v - mu);
    return acc / (double)(samples.size() - 1);
  }
};

struct Estimator {
  mgm_ctx* c;
  Gauge& g;
  const mgm_trace_params& p;
  mgm_trace_result& res;
  int L;                 // number of levels of the hierarchy
  bool full;             // full (hatted) form
  bool hutch;            // single-level variants on D^{-1}
  // workspaces of the field (scratch vectors; noise, A*noise, projection
  // coefficients, sketch, sketch images)
  DevBuf &t1, &t2, &t3, &t4, &dots, &part, &zb, &xb, &cb, &sb, &yb;

  Estimator(mgm_ctx* c_, Gauge& g_, const mgm_trace_params& p_, mgm_trace_result& r_)
      : c(c_), g(g_), p(p_), res(r_), t1(g_.est.t1), t2(g_.est.t2), t3(g_.est.t3), t4(g_.est.t4),
        dots(g_.est.dots), part(g_.est.part), zb(g_.est.zb), xb(g_.est.xb), cb(g_.est.cb), sb(g_.est.sb),
        yb(g_.est.yb) {
    L = g.mlmc_levels;
    full = p.form == MGM_FORM_FULL;
    hutch = p.variant == MGM_VARIANT_HUTCH || p.variant == MGM_VARIANT_HUTCHPP;
  }

  void solve(int l, int k, const cd* b, cd* x) {
    std::vector<int> its(k);
    const int st = solve_chunked(c, g, l, k, b, x, p.solve, its.data(), nullptr);
    if (st != MGM_OK) throw Error(st, "solve on level " + std::to_string(l) + " did not converge");
    res.lvl_solves[l] += k;
    for (int v : its) res.lvl_iters[l] += v;
  }

  // lift(j, X) = Ph_j D_j^{-1} Ph_j^H X for fine vectors X (full form)
  void lift(int j, int k, const cd* X, cd* out) {
    hipStream_t s = c->stream;
    if (j == 0) {
      solve(0, k, X, out);
      return;
    }
    // restrict down to level j, ping-ponging between t3 and t4
    std::vector<int64_t> nn(L);
    for (int q = 0; q < L; ++q) nn[q] = g.levels[q]->n;
    size_t maxn = 0;
    for (int q = 0; q <= j; ++q) maxn = std::max<size_t>(maxn, nn[q]);
    t3.ensure(sizeof(cd) * (size_t)k * maxn);
    t4.ensure(sizeof(cd) * (size_t)k * maxn);
    const cd* src = X;
    cd* bufs[2] = {t3.as<cd>(), t4.as<cd>()};
    int cur = 0;
    for (int q = 0; q < j; ++q) {
      Level& Lq = *g.levels[q];
      launch_restrict<double>(s, Lq.d.P.as<cd>(), Lq.Nx, Lq.Nt, Lq.M, Lq.bx, Lq.bt, Lq.ntv, k, src,
                              bufs[cur], nullptr);
      src = bufs[cur];
      cur ^= 1;
    }
    solve(j, k, src, bufs[cur]);
    src = bufs[cur];
    cur ^= 1;
    for (int q = j - 1; q >= 0; --q) {
      Level& Lq = *g.levels[q];
      cd* dst = (q == 0) ? out : bufs[cur];
      launch_prolong<double>(s, Lq.d.P.as<cd>(), Lq.Nx, Lq.Nt, Lq.M, Lq.bx, Lq.bt, Lq.ntv, k, src, dst, 0,
                             nullptr);
      src = dst;
      cur ^= 1;
    }
  }

  // Y = A_l X  for k vectors of the level difference sl
  void applyA(const StochLevel& sl, int k, const cd* X, cd* Y) {
    hipStream_t s = c->stream;
    const int l = sl.level;
    if (hutch) {
      solve(0, k, X, Y);
      return;
    }
    if (!full) {
      Level& F = *g.levels[l];
      Level& C = *g.levels[l + 1];
      solve(l, k, X, Y);
      t1.ensure(sizeof(cd) * (size_t)k * C.n);
      t2.ensure(sizeof(cd) * (size_t)k * C.n);
      t3.ensure(sizeof(cd) * (size_t)k * F.n);
      launch_restrict<double>(s, F.d.P.as<cd>(), F.Nx, F.Nt, F.M, F.bx, F.bt, F.ntv, k, X, t1.as<cd>(),
                              nullptr);
      solve(l + 1, k, t1.as<cd>(), t2.as<cd>());
      launch_prolong<double>(s, F.d.P.as<cd>(), F.Nx, F.Nt, F.M, F.bx, F.bt, F.ntv, k, t2.as<cd>(),
                             t3.as<cd>(), 0, nullptr);
      launch_axpby<double>(s, 1.0, Y, -1.0, t3.as<cd>(), Y, F.n, k, nullptr);
      return;
    }
    const int64_t n0 = g.levels[0]->n;
    t1.ensure(sizeof(cd) * (size_t)k * n0);
    lift(l, k, X, Y);
    lift(l + 1, k, X, t1.as<cd>());
    launch_axpby<double>(s, 1.0, Y, -1.0, t1.as<cd>(), Y, n0, k, nullptr);
  }

  // out[r] = x_r^H y_r  (HOST, k values)
  void dots_host(const cd* x, const cd* y, int64_t n, int k, std::vector<zc>& out) {
    hipStream_t s = c->stream;
    dots.ensure(sizeof(cd) * k);
    part.ensure(sizeof(cd) * (size_t)k * reduce_chunks(n) * 64);
    launch_dot_multi_ld<double>(s, x, 0, n, 1, y, n, k, dots.as<cd>(), 1, 0, nullptr, part.as<cd>());
    std::vector<cd> h(k);
    HIPCHK(hipMemcpyAsync(h.data(), dots.p, sizeof(cd) * k, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    out.resize(k);
    for (int r = 0; r < k; ++r) out[r] = zc(h[r].re, h[r].im);
  }

  // Hutch++ low-rank part: k sweeps of Y = A S, Q = qr(Y), S = Q; then
  // tau_lr = sum_i q_i^H A q_i.
  void low_rank(int idx, StochLevel& sl) {
    const int d = sl.d;
    const int64_t n = sl.n;
    DevBuf& S = sb;
    DevBuf& Y = yb;
    S.ensure(sizeof(cd) * (size_t)d * n);
    Y.ensure(sizeof(cd) * (size_t)d * n);
    sl.Q->ensure(sizeof(cd) * (size_t)d * n);
    launch_noise<double>(c->stream, S.as<cd>(), n, d, p.noise, p.seed, MGM_PURPOSE_SKETCH, idx, 0);
    const cd* src = S.as<cd>();
    for (int it = 0; it < std::max(1, p.k_power); ++it) {
      applyA(sl, d, src, Y.as<cd>());
      orthonormalize(c, n, d, Y.as<cd>(), sl.Q->as<cd>());
      src = sl.Q->as<cd>();
    }
    applyA(sl, d, sl.Q->as<cd>(), Y.as<cd>());
    std::vector<zc> v;
    dots_host(sl.Q->as<cd>(), Y.as<cd>(), n, d, v);
    zc acc = 0;
    for (const zc& x : v) acc += x;
    sl.tau_lr = acc;
  }

  // b samples tau_{s,l} = z^H (A zeta), z = zeta - Q (Q^H zeta), indices s0..s0+b-1
  void sample_batch(int idx, StochLevel& sl, int s0, int b, std::vector<zc>& out) {
    hipStream_t s = c->stream;
    const int64_t n = sl.n;
    DevBuf& Z = zb;
    DevBuf& X = xb;
    DevBuf& C = cb;
    Z.ensure(sizeof(cd) * (size_t)b * n);
    X.ensure(sizeof(cd) * (size_t)b * n);
    launch_noise<double>(s, Z.as<cd>(), n, b, p.noise, p.seed, MGM_PURPOSE_SAMPLE, idx, s0);
    applyA(sl, b, Z.as<cd>(), X.as<cd>());
    if (sl.d > 0) {
      C.ensure(sizeof(cd) * (size_t)b * sl.d);
      part.ensure(sizeof(cd) * (size_t)b * sl.d * reduce_chunks(n) + 64);
      launch_dot_multi_ld<double>(s, sl.Q->as<cd>(), n, 0, sl.d, Z.as<cd>(), n, b, C.as<cd>(), sl.d, 0,
                                  nullptr, part.as<cd>());
      launch_update_multi<double>(s, sl.Q->as<cd>(), n, 0, sl.d, C.as<cd>(), sl.d, -1.0, Z.as<cd>(), n, b,
                                  nullptr, nullptr, nullptr);
    }
    dots_host(Z.as<cd>(), X.as<cd>(), n, b, out);
  }

  std::vector<double> weights(const std::vector<StochLevel>& lv) {
    const int nl = (int)lv.size();
    std::vector<double> w(nl, 1.0 / nl);
    if (p.targets == MGM_TARGETS_UNIFORM) return w;
    std::vector<double> cv(nl);
    double tot = 0;
    for (int i = 0; i < nl; ++i) {
      cv[i] = lv[i].s() >= 2 ? std::sqrt(lv[i].cost * lv[i].var()) : 0.0;
      tot += cv[i];
    }
    if (!std::isfinite(tot) || tot == 0.0) return w;
    for (int i = 0; i < nl; ++i) w[i] = cv[i] / tot;
    return w;
  }

  double nnz_model(int j) const {
    const Level& Lj = *g.levels[j];
    return j == 0 ? 9.0 * Lj.n : 5.0 * Lj.M * Lj.n;
  }

  int run() {
    require(g.mg_ready, "trace_estimate needs setup_mg first", MGM_ESTATE);
    require(p.eps > 0 || p.fixed_samples, "eps must be positive");
    require(p.batch >= 1, "batch must be >= 1");
    const int nst = hutch ? 1 : L - 1;
    require(nst >= 1, "MLMC variants need at least two levels");
    const bool lr = p.variant == MGM_VARIANT_HUTCHPP || p.variant == MGM_VARIANT_MLMCPP;
    std::vector<StochLevel> lv(nst);
    for (int i = 0; i < nst; ++i) {
      StochLevel& sl = lv[i];
      sl.Q = &g.est.Q[i];
      sl.level = hutch ? 0 : i;
      sl.n = (hutch || full) ? g.levels[0]->n : g.levels[i]->n;
      sl.d = lr ? p.d[i] : 0;
      require(sl.d >= 0 && sl.d <= 64, "d must be in [0, 64]");
      if (p.use_fixed_cost) {
        sl.cost = p.fixed_cost[i];
      } else {
        sl.cost = nnz_model(i) + 2.0 * sl.n * sl.d;
        if (i + 1 < L) sl.cost += nnz_model(i + 1);
      }
    }
    const zc tau_exact = hutch ? zc(0) : zc(g.trL[0], g.trL[1]);
    for (int i = 0; i < nst; ++i)
      if (lv[i].d > 0) low_rank(i, lv[i]);

    const int minS = std::max(2, p.min_samples);
    const int maxS = p.max_samples > 0 ? p.max_samples : (1 << 30);
    zc tau = 0;
    int s = 0;
    while (true) {
      bool any = false;
      for (auto& sl : lv) any = any || sl.active;
      if (!any) break;
      // speculative batch for every active level.  The batch length only
      // decides how much work may be discarded, never the result: in
      // adaptive mode it is the number of samples the current variances and
      // targets predict are still missing (all active levels advance
      // together, as in Alg. 2), between 4 and p.batch.
      int common = p.batch;
      if (!p.fixed_samples) {
        if (s < 2) {
          common = std::max(minS, p.batch / 2);
        } else {
          const std::vector<double> w = weights(lv);
          double need = 0;
          for (int i = 0; i < nst; ++i) {
            if (!lv[i].active) continue;
            const double rho2 = w[i] * (p.eps * std::abs(tau)) * (p.eps * std::abs(tau));
            const double want = rho2 > 0 ? lv[i].var() / rho2 : 1e30;
            need = std::max(need, std::isfinite(want) ? want - lv[i].s() : 1e30);
          }
          common = (int)std::min<double>(p.batch, std::max(4.0, std::ceil(1.15 * need) + 2));
        }
      }
      std::vector<std::vector<zc>> vals(nst);
      for (int i = 0; i < nst; ++i) {
        if (!lv[i].active) continue;
        int b = common;
        if (p.fixed_samples) b = std::min(b, p.fixed_samples[i] - lv[i].s());
        b = std::min(b, maxS - lv[i].s());
        if (b > 0) sample_batch(i, lv[i], lv[i].s(), b, vals[i]);
      }
      // replay Alg. 2 sample by sample; stop where an active level has no
      // evaluated sample left (levels advance in lockstep)
      for (int t = 0; t < p.batch; ++t) {
        bool any_active = false, missing = false;
        for (int i = 0; i < nst; ++i) {
          any_active = any_active || lv[i].active;
          if (lv[i].active && t >= (int)vals[i].size()) missing = true;
        }
        if (!any_active || missing) break;
        for (int i = 0; i < nst; ++i)
          if (lv[i].active) lv[i].samples.push_back(vals[i][t]);
        ++s;
        tau = tau_exact;
        for (auto& sl : lv) tau += sl.mean() + sl.tau_lr;
        if (p.fixed_samples) {
          for (int i = 0; i < nst; ++i)
            if (lv[i].s() >= p.fixed_samples[i]) lv[i].active = false;
          continue;
        }
        const std::vector<double> w = weights(lv);
        for (int i = 0; i < nst; ++i) {
          StochLevel& sl = lv[i];
          if (!sl.active) continue;
          if (sl.s() >= maxS) {
            sl.active = false;
            continue;
          }
          if (sl.s() < minS) continue;
          const double rho2 = w[i] * (p.eps * std::abs(tau)) * (p.eps * std::abs(tau));
          if (sl.var() / sl.s() <= rho2) sl.active = false;
        }
      }
      if (p.fixed_samples) {
        for (int i = 0; i < nst; ++i)
          if (lv[i].s() >= p.fixed_samples[i]) lv[i].active = false;
      }
    }
    res.tau[0] = tau.real();
    res.tau[1] = tau.imag();
    res.tau_exact[0] = tau_exact.real();
    res.tau_exact[1] = tau_exact.imag();
    res.nstoch = nst;
    for (int i = 0; i < nst; ++i) {
      const zc mu = lv[i].mean();
      res.lvl_mean[i][0] = mu.real();
      res.lvl_mean[i][1] = mu.imag();
      res.lvl_lr[i][0] = lv[i].tau_lr.real();
      res.lvl_lr[i][1] = lv[i].tau_lr.imag();
      res.lvl_var[i] = lv[i].var();
      res.lvl_cost[i] = lv[i].cost;
      res.lvl_samples[i] = lv[i].s();
      if (res.sample_dump && res.max_dump > 0) {
        for (int k = 0; k < std::min(res.max_dump, lv[i].s()); ++k) {
          res.sample_dump[((int64_t)i * res.max_dump + k) * 2] = lv[i].samples[k].real();
          res.sample_dump[((int64_t)i * res.max_dump + k) * 2 + 1] = lv[i].samples[k].imag();
        }
      }
    }
    return MGM_OK;
  }
};

}  // namespace

int trace_estimate(mgm_ctx* c, Gauge& g, const mgm_trace_params& p, mgm_trace_result& r) {
  for (int i = 0; i < MGM_MAX_LEVELS; ++i) {
    r.lvl_solves[i] = 0;
    r.lvl_iters[i] = 0;
    r.lvl_samples[i] = 0;
  }
  Estimator e(c, g, p, r);
  return e.run();
}

}  // namespace mgm
