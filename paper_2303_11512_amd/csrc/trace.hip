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
//
// In the reduced form, difference l needs solves with D_l (its fine part) and
// with D_{l+1} (its coarse part, on P_l^H of the same vectors), so every
// inner level is solved for two differences.  Both sets of right-hand sides
// go into one solve per level: a coarse level is small enough that its
// kernels cost nearly the same for 32 or 64 right-hand sides, and each
// right-hand side still has its own Krylov space and stopping test.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <thread>

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
  std::vector<double> costs;                // C_{s,l} of each sample (cost model)
  std::vector<std::array<int, 2>> its;      // FGMRES iterations of its two solves
  double cost_sum = 0;
  double lr_cost = 0;                       // cost model work of the Hutch++ phase
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

// Evaluated samples of one level difference in one batch, in index order.
struct Batch {
  std::vector<zc> vals;
  std::vector<double> cost;
  std::vector<std::array<int, 2>> its;
};
using Its = std::vector<std::array<int, 2>>;  // per vector: iterations on D_l and D_{l+1}

struct Estimator {
  mgm_ctx* c;
  Gauge& g;
  const mgm_trace_params& p;
  mgm_trace_result& res;
  int L;                 // number of levels of the hierarchy
  bool full;             // full (hatted) form
  bool hutch;            // single-level variants on D^{-1}
  bool deflated;         // deflated Hutchinson (subspace-iteration basis)
  bool two_sided;        // samples z^H A z instead of z^H A zeta
  int kmax = 1;          // most vectors one difference hands to a solve
  // workspaces of the field (scratch vectors, dot products)
  DevBuf &t1, &t3, &t4, &dots, &part;

  Estimator(mgm_ctx* c_, Gauge& g_, const mgm_trace_params& p_, mgm_trace_result& r_)
      : c(c_), g(g_), p(p_), res(r_), t1(g_.est.t1), t3(g_.est.t3), t4(g_.est.t4),
        dots(g_.est.dots), part(g_.est.part) {
    L = g.mlmc_levels;
    full = p.form == MGM_FORM_FULL;
    hutch = p.variant == MGM_VARIANT_HUTCH || p.variant == MGM_VARIANT_HUTCHPP ||
            p.variant == MGM_VARIANT_DEFLATED;
    deflated = p.variant == MGM_VARIANT_DEFLATED;
    two_sided = p.projection == MGM_PROJ_TWO_SIDED;
    cost_init();
  }

  // ---- the cost model of Sec. 4: complex multiply-adds of every
  // matrix-vector product a sample performs.  Operators count their
  // structural non-zeros (9 per fine row, 5 M^2 per coarse site), R and P
  // n_j ntv_j each, a SAP cycle the residual rows of both colours plus one
  // K x K block-inverse product per block, a dense inverse n^2; an FGMRES
  // iteration one preconditioner and one operator product, a restart cycle
  // two residuals; the projection 2 n d.  Vector work (Gram-Schmidt, dot
  // products) is not counted.  Solves on a level with a dense inverse are
  // one dense product and the residual check.
  std::vector<double> c_nnzD, c_nnzP, c_prec;
  void cost_init() {
    const int Ls = (int)g.levels.size();
    c_nnzD.assign(Ls, 0.0);
    c_nnzP.assign(Ls, 0.0);
    c_prec.assign(Ls, 0.0);
    for (int j = 0; j < Ls; ++j) {
      const Level& Lj = *g.levels[j];
      c_nnzD[j] = j == 0 ? 9.0 * Lj.n : 5.0 * Lj.M * Lj.M * (double)Lj.sites;
      c_nnzP[j] = Lj.has_coarse ? (double)Lj.n * Lj.ntv : 0.0;
    }
    for (int j = Ls - 1; j >= 0; --j) {
      const Level& Lj = *g.levels[j];
      if (Lj.is_coarsest || !Lj.has_coarse) {
        c_prec[j] = (double)Lj.n * Lj.n;
        continue;
      }
      const Level& C = *g.levels[j + 1];
      const double coarse = C.is_coarsest ? (double)C.n * C.n
                            : C.inner_iters <= 0 ? c_prec[j + 1]
                                                 : C.inner_iters * (c_prec[j + 1] + c_nnzD[j + 1]);
      const double sap = c_nnzD[j] + (double)Lj.nblk * Lj.K * Lj.K;
      c_prec[j] = 2.0 * c_nnzP[j] + coarse + Lj.sap_cycles * sap;
    }
  }
  double solve_cost(int j, int its) const {
    const Level& Lj = *g.levels[j];
    if (Lj.has_dense) return (double)Lj.n * Lj.n + c_nnzD[j];
    const int m = std::max(1, p.solve.restart);
    const int cycles = std::max(1, (its + m - 1) / m);
    return its * (c_nnzD[j] + c_prec[j]) + 2.0 * cycles * c_nnzD[j];
  }
  // A_l applied to one vector whose solves took (its[0], its[1]) iterations
  double apply_cost(int l, const std::array<int, 2>& its) const {
    if (hutch) return solve_cost(0, its[0]);
    if (!full) return 2.0 * c_nnzP[l] + solve_cost(l, its[0]) + solve_cost(l + 1, its[1]);
    auto walk = [&](int j) {
      double w = 0;
      for (int q = 0; q < j; ++q) w += 2.0 * c_nnzP[q];
      return w;
    };
    return walk(l) + solve_cost(l, its[0]) + walk(l + 1) + solve_cost(l + 1, its[1]);
  }

  // solve on level l through the view cv (this thread's, or the worker's on
  // the field's second stream); solve and iteration counts go to cnt[l], the
  // iterations of each right-hand side to its_out
  void solve_on(mgm_ctx* cv, int l, int k, const cd* b, cd* x, std::vector<std::array<int64_t, 2>>& cnt,
                std::vector<int>& its_out) {
    its_out.assign(k, 0);
    const int st = solve_chunked(cv, g, l, k, b, x, p.solve, its_out.data(), nullptr);
    if (st != MGM_OK) throw Error(st, "solve on level " + std::to_string(l) + " did not converge");
    cnt[l][0] += k;
    for (int v : its_out) cnt[l][1] += v;
  }
  std::vector<int> solve(int l, int k, const cd* b, cd* x) {
    std::vector<std::array<int64_t, 2>> cnt(MGM_MAX_LEVELS, {0, 0});
    std::vector<int> its;
    solve_on(c, l, k, b, x, cnt, its);
    res.lvl_solves[l] += (int)cnt[l][0];
    res.lvl_iters[l] += (int)cnt[l][1];
    return its;
  }

  // lift(j, X) = Ph_j D_j^{-1} Ph_j^H X for fine vectors X (full form);
  // returns the iterations of its solve per vector
  std::vector<int> lift(int j, int k, const cd* X, cd* out) {
    hipStream_t s = c->stream;
    if (j == 0) return solve(0, k, X, out);
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
    std::vector<int> its = solve(j, k, src, bufs[cur]);
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
    return its;
  }

  // Y = A_l X for k vectors of the level difference sl: Hutchinson variants
  // (A = D^{-1}) and the full form on fine vectors
  Its applyA(const StochLevel& sl, int k, const cd* X, cd* Y) {
    hipStream_t s = c->stream;
    const int l = sl.level;
    Its its(k, {0, 0});
    if (hutch) {
      const std::vector<int> a = solve(0, k, X, Y);
      for (int v = 0; v < k; ++v) its[v][0] = a[v];
      return its;
    }
    const int64_t n0 = g.levels[0]->n;
    t1.ensure(sizeof(cd) * (size_t)k * n0);
    const std::vector<int> a = lift(l, k, X, Y);
    const std::vector<int> b = lift(l + 1, k, X, t1.as<cd>());
    launch_axpby<double>(s, 1.0, Y, -1.0, t1.as<cd>(), Y, n0, k, nullptr);
    for (int v = 0; v < k; ++v) its[v] = {a[v], b[v]};
    return its;
  }

  // Y = A_i X for several blocks of vectors, each of one level difference i
  // (a difference may bring several blocks).  Reduced form: the right-hand
  // sides of each operator level j -- P_{j-1}^H X of the blocks of difference
  // j-1, then the X of the blocks of difference j -- are solved together; then
  // Y = (D_i^{-1} X) - P_i (D_{i+1}^{-1} P_i^H X) per block.  Other forms
  // apply the blocks one after the other.
  struct Item {
    int i, k;
    const cd* X;
    cd* Y;
  };
  static constexpr int kSegs = 4;  // most blocks one level's solve gathers
  // its[q]: per vector of block q, the iterations of its two solves
  void applyA_levels(const std::vector<StochLevel>& lv, const std::vector<Item>& items, std::vector<Its>& its) {
    its.assign(items.size(), Its());
    if (hutch || full) {
      for (size_t q = 0; q < items.size(); ++q) its[q] = applyA(lv[items[q].i], items[q].k, items[q].X, items[q].Y);
      return;
    }
    hipStream_t s = c->stream;
    const int ni = (int)items.size();
    // segments of level j: (block, coarse part?) -- coarse parts first
    std::vector<std::vector<std::pair<int, bool>>> segs(L);
    for (int q = 0; q < ni; ++q) {
      const int l = lv[items[q].i].level;
      require(l + 1 < L, "applyA_levels: bad level difference");
      require(items[q].k >= 1 && items[q].k <= kmax, "applyA_levels: too many vectors");
      segs[l + 1].push_back({q, true});
    }
    for (int q = 0; q < ni; ++q) segs[lv[items[q].i].level].push_back({q, false});
    std::vector<int> own_off(ni, 0), crs_off(ni, 0), total(L, 0);
    std::vector<const cd*> src(L, nullptr);
    for (int j = 0; j < L; ++j) {
      if (segs[j].empty()) continue;
      require((int)segs[j].size() <= kSegs, "applyA_levels: too many blocks on one level");
      for (const auto& sg : segs[j]) {
        (sg.second ? crs_off : own_off)[sg.first] = total[j];
        total[j] += items[sg.first].k;
      }
      Level& Lj = *g.levels[j];
      const int64_t n = Lj.n;
      // sized for the most vectors any call can bring, so that later
      // estimates reuse the buffers (captured graphs stay valid)
      const size_t cap = sizeof(cd) * (size_t)n * kSegs * kmax;
      g.est.lout[j].ensure(cap);
      if (segs[j].size() == 1 && !segs[j][0].second) {
        src[j] = items[segs[j][0].first].X;  // one fine-part block: solved in place
        continue;
      }
      DevBuf& in = g.est.lin[j];
      in.ensure(cap);
      for (const auto& sg : segs[j]) {
        const Item& it = items[sg.first];
        cd* dst = in.as<cd>() + (int64_t)total_before(segs[j], items, sg) * n;
        if (sg.second) {
          Level& F = *g.levels[j - 1];
          launch_restrict<double>(s, F.d.P.as<cd>(), F.Nx, F.Nt, F.M, F.bx, F.bt, F.ntv, it.k, it.X, dst, nullptr);
        } else {
          HIPCHK(hipMemcpyAsync(dst, it.X, sizeof(cd) * (size_t)it.k * n, hipMemcpyDeviceToDevice, s));
        }
      }
      src[j] = in.as<cd>();
    }
    std::vector<std::vector<int>> lits(L);
    solve_levels(total, src, lits);
    t3.ensure(sizeof(cd) * (size_t)kmax * g.levels[0]->n);
    for (int q = 0; q < ni; ++q) {
      const Item& it = items[q];
      const int l = lv[it.i].level;
      its[q].resize(it.k);
      for (int v = 0; v < it.k; ++v) its[q][v] = {lits[l][own_off[q] + v], lits[l + 1][crs_off[q] + v]};
      Level& F = *g.levels[l];
      Level& C = *g.levels[l + 1];
      const cd* fine = g.est.lout[l].as<cd>() + (int64_t)own_off[q] * F.n;
      const cd* coarse = g.est.lout[l + 1].as<cd>() + (int64_t)crs_off[q] * C.n;
      launch_prolong<double>(s, F.d.P.as<cd>(), F.Nx, F.Nt, F.M, F.bx, F.bt, F.ntv, it.k, coarse, t3.as<cd>(),
                             0, nullptr);
      launch_axpby<double>(s, 1.0, fine, -1.0, t3.as<cd>(), it.Y, F.n, it.k, nullptr);
    }
  }
  // vectors ahead of segment sg in its level's gathered block
  static int total_before(const std::vector<std::pair<int, bool>>& segs, const std::vector<Item>& items,
                          const std::pair<int, bool>& sg) {
    int off = 0;
    for (const auto& x : segs) {
      if (x == sg) break;
      off += items[x.first].k;
    }
    return off;
  }

  // Solve level j's total[j] right-hand sides src[j] into g.est.lout[j] for
  // every j.  The solves are independent: the finest runs on this thread and
  // the field's stream; the other iterative ones one after the other on the
  // field's second stream from a worker thread with its own workspace set, so
  // the latency-bound coarse-level kernels overlap the fine level's; the
  // exact (dense-inverse) solves from a third thread on the third stream.
  void solve_levels(const std::vector<int>& total, const std::vector<const cd*>& src,
                    std::vector<std::vector<int>>& lits) {
    std::vector<int> todo;
    for (int j = 0; j < L; ++j)
      if (total[j] > 0) todo.push_back(j);
    using Counts = std::vector<std::array<int64_t, 2>>;
    Counts cnt(MGM_MAX_LEVELS, {0, 0});
    std::vector<Counts> wcnt(2, Counts(MGM_MAX_LEVELS, {0, 0}));
    auto out = [&](int j) { return g.est.lout[j].as<cd>(); };
    if (todo.size() < 2 || !p.concurrent) {
      for (int j : todo) solve_on(c, j, total[j], src[j], out(j), cnt, lits[j]);
    } else {
      // worker 0: iterative levels on stream 2; worker 1: exact levels on
      // stream 3, then the second half of an iterative level with more than
      // 64 right-hand sides (its solves are independent per RHS)
      struct Job {
        int j, off, k;
        std::vector<int> its;
      };
      std::vector<Job> part[2];
      for (size_t q = 1; q < todo.size(); ++q) {
        const int j = todo[q];
        if (g.levels[j]->has_dense) part[1].push_back({j, 0, total[j], {}});
      }
      for (size_t q = 1; q < todo.size(); ++q) {
        const int j = todo[q];
        if (g.levels[j]->has_dense) continue;
        if (total[j] > 64) {
          const int k0 = (total[j] / 2 + 15) / 16 * 16;
          part[0].push_back({j, 0, k0, {}});
          part[1].push_back({j, k0, total[j] - k0, {}});
        } else {
          part[0].push_back({j, 0, total[j], {}});
        }
      }
      if (part[0].empty()) part[0].swap(part[1]);
      ensure_stream2();
      HIPCHK(hipEventRecord(g.ev_fork, c->stream));
      HIPCHK(hipStreamWaitEvent(g.stream2, g.ev_fork, 0));
      if (!part[1].empty()) HIPCHK(hipStreamWaitEvent(g.stream3, g.ev_fork, 0));
      int wst[2] = {MGM_OK, MGM_OK};
      std::string wmsg[2];
      std::vector<std::thread> workers;
      for (int k = 0; k < 2; ++k) {
        if (part[k].empty()) continue;
        workers.emplace_back([&, k] {
          mgm_ctx w;  // worker view: its stream, its workspace set, private scratch
          w.device = c->device;
          w.stream = k == 0 ? g.stream2 : g.stream3;
          w.cnn = c->cnn;
          w.wslot = 1 + k;
          try {
            HIPCHK(hipSetDevice(c->device));
            for (Job& jb : part[k]) {
              const int64_t n = g.levels[jb.j]->n;
              solve_on(&w, jb.j, jb.k, src[jb.j] + (int64_t)jb.off * n, out(jb.j) + (int64_t)jb.off * n, wcnt[k],
                       jb.its);
            }
          } catch (const Error& e) {
            wst[k] = e.code;
            wmsg[k] = e.what();
          } catch (const std::exception& e) {
            wst[k] = MGM_EHIP;
            wmsg[k] = e.what();
          }
        });
      }
      int st = MGM_OK;
      std::string msg;
      try {
        solve_on(c, todo[0], total[todo[0]], src[todo[0]], out(todo[0]), cnt, lits[todo[0]]);
      } catch (const Error& e) {
        st = e.code;
        msg = e.what();
      } catch (const std::exception& e) {
        st = MGM_EHIP;
        msg = e.what();
      }
      for (auto& t : workers) t.join();
      HIPCHK(hipEventRecord(g.ev_join, g.stream2));
      HIPCHK(hipStreamWaitEvent(c->stream, g.ev_join, 0));
      if (!part[1].empty()) {
        HIPCHK(hipEventRecord(g.ev_join3, g.stream3));
        HIPCHK(hipStreamWaitEvent(c->stream, g.ev_join3, 0));
      }
      if (st != MGM_OK) throw Error(st, msg);
      for (int k = 0; k < 2; ++k)
        if (wst[k] != MGM_OK) throw Error(wst[k], wmsg[k]);
      for (int k = 0; k < 2; ++k)
        for (const Job& jb : part[k]) {
          lits[jb.j].resize(total[jb.j]);
          std::copy(jb.its.begin(), jb.its.end(), lits[jb.j].begin() + jb.off);
        }
    }
    for (int j = 0; j < L; ++j) {
      res.lvl_solves[j] += (int)(cnt[j][0] + wcnt[0][j][0] + wcnt[1][j][0]);
      res.lvl_iters[j] += (int)(cnt[j][1] + wcnt[0][j][1] + wcnt[1][j][1]);
    }
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

  // Several blocks of x_r^H y_r with one read-back: dots_add launches one
  // block's dots into its own slice of `dots` (sized for the largest batch up
  // front in run(), so no slice moves while launches are queued) and returns
  // the slice index; dots_fetch copies every slice with one synchronisation.
  std::vector<std::array<int, 2>> dslices;
  int dtot = 0;
  int dots_add(const cd* x, const cd* y, int64_t n, int k) {
    require((size_t)(dtot + k) * sizeof(cd) <= dots.bytes, "trace: dot batch exceeds its workspace");
    part.ensure(sizeof(cd) * (size_t)k * reduce_chunks(n) * 64);
    launch_dot_multi_ld<double>(c->stream, x, 0, n, 1, y, n, k, dots.as<cd>() + dtot, 1, 0, nullptr,
                                part.as<cd>());
    dslices.push_back({dtot, k});
    dtot += k;
    return (int)dslices.size() - 1;
  }
  std::vector<std::vector<zc>> dots_fetch() {
    std::vector<cd> h(std::max(1, dtot));
    if (dtot > 0) HIPCHK(hipMemcpyAsync(h.data(), dots.p, sizeof(cd) * dtot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<std::vector<zc>> out;
    for (const auto& sl : dslices) {
      std::vector<zc> v(sl[1]);
      for (int r = 0; r < sl[1]; ++r) v[r] = zc(h[sl[0] + r].re, h[sl[0] + r].im);
      out.push_back(std::move(v));
    }
    dslices.clear();
    dtot = 0;
    return out;
  }

  // The field's second stream and its fork / join events (created on first use)
  void ensure_stream2() {
    if (g.stream2) return;
    HIPCHK(hipStreamCreateWithFlags(&g.stream2, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&g.stream3, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&g.ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&g.ev_join, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&g.ev_join3, hipEventDisableTiming));
  }

  // Q = qr+(Y) of every item's block: the differences' QRs are independent,
  // so they run two at a time (the field's stream and its second stream, each
  // difference with a workspace of its own), and one read-back checks every
  // failure flag
  void orthonormalize_items(const std::vector<StochLevel>& lv, const std::vector<Item>& items,
                            const std::vector<cd*>& dst) {
    ensure_stream2();
    HIPCHK(hipEventRecord(g.ev_fork, c->stream));
    HIPCHK(hipStreamWaitEvent(g.stream2, g.ev_fork, 0));
    for (size_t q = 0; q < items.size(); ++q) {
      const Item& x = items[q];
      const int64_t n = lv[x.i].n;
      const int d = x.k;
      EstWork& E = g.est;
      E.qtmp[x.i].ensure(sizeof(cd) * (size_t)d * n);
      E.qG[x.i].ensure(sizeof(cd) * (size_t)d * d);
      E.qpart[x.i].ensure(sizeof(cd) * (size_t)d * d * gram_partials(n));
      E.qfail[x.i].ensure(sizeof(int));
      orthonormalize_launch(q % 2 ? g.stream2 : c->stream, n, d, x.Y, dst[q], E.qtmp[x.i].as<cd>(),
                            E.qG[x.i].as<cd>(), E.qpart[x.i].as<cd>(), E.qfail[x.i].as<int>());
    }
    HIPCHK(hipEventRecord(g.ev_join, g.stream2));
    HIPCHK(hipStreamWaitEvent(c->stream, g.ev_join, 0));
    std::vector<int> hf(items.size(), 0);
    for (size_t q = 0; q < items.size(); ++q)
      HIPCHK(hipMemcpyAsync(&hf[q], g.est.qfail[items[q].i].p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int f : hf)
      if (f) throw Error(MGM_ENONFINITE, "CholQR: Gram matrix not positive definite (rank-deficient block)");
  }

  // Hutch++ low-rank parts of all differences (d_i > 0), sweep by sweep:
  // k sweeps of Y = A S, Q = qr(Y), S = Q; then tau_lr = sum_i q_i^H A q_i.
  // The solves of the last round (A Q) go together with those of the first
  // stochastic batch (A zeta does not depend on Q; only the projection of
  // zeta, applied afterwards, does): first[i] samples of difference i,
  // returned in first_vals.
  void add_lr_cost(std::vector<StochLevel>& lv, const std::vector<Item>& items, const std::vector<Its>& its,
                   size_t nitems) {
    for (size_t q = 0; q < nitems; ++q)
      for (const auto& v : its[q]) lv[items[q].i].lr_cost += apply_cost(lv[items[q].i].level, v);
  }
  void low_rank_all(std::vector<StochLevel>& lv, const std::vector<int>& first, std::vector<Batch>& first_vals) {
    std::vector<Item> items;
    for (int i = 0; i < (int)lv.size(); ++i) {
      StochLevel& sl = lv[i];
      if (sl.d <= 0) continue;
      const size_t bytes = sizeof(cd) * (size_t)sl.d * sl.n;
      g.est.S[i].ensure(bytes);
      g.est.Y[i].ensure(bytes);
      sl.Q->ensure(bytes);
      launch_noise<double>(c->stream, g.est.S[i].as<cd>(), sl.n, sl.d, p.noise, p.seed, MGM_PURPOSE_SKETCH, i, 0);
      items.push_back({i, sl.d, g.est.S[i].as<cd>(), g.est.Y[i].as<cd>()});
    }
    if (items.empty()) {
      sample_batches(lv, first, first_vals);
      return;
    }
    std::vector<Its> its;
    if (deflated) {
      deflation_basis(lv[0]);
      items[0].X = lv[0].Q->as<cd>();
    } else {
    for (int it = 0; it < std::max(1, p.k_power); ++it) {
      applyA_levels(lv, items, its);
      add_lr_cost(lv, items, its, items.size());
      std::vector<cd*> dst;
      for (const Item& x : items) dst.push_back(lv[x.i].Q->as<cd>());
      orthonormalize_items(lv, items, dst);
      for (Item& x : items) x.X = lv[x.i].Q->as<cd>();
    }
    }
    const size_t nlr = items.size();
    const std::vector<int> first_b = equal_work_batch(lv, first);
    // A zeta does not depend on Q, so the first batch of one-sided samples
    // rides with the last round; two-sided samples need the final Q first
    if (!two_sided) sample_start(lv, first_b, items);
    applyA_levels(lv, items, its);
    add_lr_cost(lv, items, its, nlr);
    // tau_lr of every difference and the first samples' dots: one read-back
    std::vector<int> lr_req(nlr);
    for (size_t q = 0; q < nlr; ++q) lr_req[q] = dots_add(items[q].X, items[q].Y, lv[items[q].i].n, items[q].k);
    const std::vector<Item> sitems(items.begin() + nlr, items.end());
    const std::vector<Its> sits(its.begin() + nlr, its.end());
    std::vector<int> s_req;
    if (!two_sided) s_req = sample_finish_launch(lv, sitems);
    const std::vector<std::vector<zc>> got = dots_fetch();
    for (size_t q = 0; q < nlr; ++q) {
      zc acc = 0;
      for (const zc& y : got[lr_req[q]]) acc += y;
      lv[items[q].i].tau_lr = acc;
    }
    if (two_sided) {
      sample_batches(lv, first_b, first_vals);
    } else {
      sample_finish_collect(lv, sitems, sits, got, s_req, first_vals);
    }
    if (deflated) ritz_triplets(lv[0]);
  }

  // The first stochastic batch, speculative like every batch (the replay
  // takes the same samples whatever it holds): each difference is given
  // about the cost-model work of the costliest one, so the cheaper
  // differences evaluate proportionally more samples in the same phase.
  // Per-vector costs are those of the power rounds so far; rounded up to the
  // 16-RHS tile, at most `batch`.
  std::vector<int> equal_work_batch(const std::vector<StochLevel>& lv, const std::vector<int>& b) const {
    if (p.fixed_samples || p.k_power < 1) return b;
    std::vector<double> cv(lv.size(), 0.0);
    double cmax = 0;
    for (size_t i = 0; i < lv.size(); ++i) {
      if (b[i] <= 0 || lv[i].d <= 0) continue;
      cv[i] = lv[i].lr_cost / ((double)p.k_power * lv[i].d);
      if (!(cv[i] > 0) || !std::isfinite(cv[i])) return b;
      cmax = std::max(cmax, cv[i]);
    }
    const int maxS = p.max_samples > 0 ? p.max_samples : (1 << 30);
    std::vector<int> out = b;
    for (size_t i = 0; i < lv.size(); ++i) {
      if (cv[i] <= 0) continue;
      const double want = std::ceil(std::ceil(b[i] * cmax / cv[i]) / 16.0) * 16.0;
      const int v = std::max(b[i], (int)std::min<double>(p.batch, want));
      out[i] = std::min(v, maxS - lv[i].s());
    }
    return out;
  }

  // ---- adaptive number of Hutch++ vectors per level difference (the
  // choice of d is left open by the paper, Sec. 5).  Candidates d, 2d, ...
  // <= d_max; for each: the block power iteration's basis (into the level's
  // spare basis buffer), tau_lr, and `pilot` samples of the projected
  // remainder (noise purpose PILOT, the same vectors for every candidate,
  // discarded afterwards) give the variance V(d) and per-sample cost C(d);
  // the level's predicted cost is T(d) = W_lr(d) + V(d) C(d) / rho^2 with
  // rho^2 = (eps |tau0|)^2 / (levels), tau0 from the first candidates.  The
  // doubling stops at the first candidate that does not lower T.  W_lr and
  // C come from the cost model in use (static/fixed: (k+1) d C_A and C_A +
  // 2 n d; flops: as counted).
  struct Cand {
    int d = 0;
    int buf = 0;  // 0: est.Q[i], 1: est.Q2[i]
    zc tau_lr = 0, mean = 0;
    double V = 0, C = 0, W = 0;
  };
  // C_A of the static or fixed model: one application of A_l (as the static
  // per-sample cost, without the projection)
  double apply_static(int i, const StochLevel&) const {
    if (p.cost == MGM_COST_FIXED) return p.fixed_cost[i];
    return c_nnzD[i] + (i + 1 < L ? c_nnzD[i + 1] : 0.0);
  }
  void candidates(std::vector<StochLevel>& lv, const std::vector<int>& which, const std::vector<int>& dd,
                  const std::vector<int>& buf, std::vector<Cand>& out) {
    std::vector<Item> items;
    std::vector<double> w0(lv.size(), 0.0);
    for (int i : which) {
      StochLevel& sl = lv[i];
      DevBuf& Qb = buf[i] ? g.est.Q2[i] : g.est.Q[i];
      const size_t bytes = sizeof(cd) * (size_t)dd[i] * sl.n;
      g.est.S[i].ensure(sizeof(cd) * (size_t)p.d_max * sl.n);
      g.est.Y[i].ensure(sizeof(cd) * (size_t)p.d_max * sl.n);
      Qb.ensure(bytes);
      launch_noise<double>(c->stream, g.est.S[i].as<cd>(), sl.n, dd[i], p.noise, p.seed, MGM_PURPOSE_SKETCH, i, 0);
      items.push_back({i, dd[i], g.est.S[i].as<cd>(), g.est.Y[i].as<cd>()});
      w0[i] = sl.lr_cost;
    }
    std::vector<Its> its;
    for (int it = 0; it < std::max(1, p.k_power); ++it) {
      applyA_levels(lv, items, its);
      add_lr_cost(lv, items, its, items.size());
      for (Item& x : items) {
        DevBuf& Qb = buf[x.i] ? g.est.Q2[x.i] : g.est.Q[x.i];
        orthonormalize(c, lv[x.i].n, x.k, x.Y, Qb.as<cd>());
        x.X = Qb.as<cd>();
      }
    }
    applyA_levels(lv, items, its);
    add_lr_cost(lv, items, its, items.size());
    for (const Item& x : items) {
      std::vector<zc> v;
      dots_host(x.X, x.Y, lv[x.i].n, x.k, v);
      Cand& cd_ = out[x.i];
      cd_ = Cand();
      cd_.d = x.k;
      cd_.buf = buf[x.i];
      for (const zc& y : v) cd_.tau_lr += y;
    }
    // pilot samples with each level's trial basis
    std::vector<int> nb(lv.size(), 0);
    std::vector<DevBuf*> saveQ(lv.size());
    std::vector<int> saved(lv.size());
    for (int i : which) {
      nb[i] = p.pilot;
      saveQ[i] = lv[i].Q;
      saved[i] = lv[i].d;
      lv[i].Q = buf[i] ? &g.est.Q2[i] : &g.est.Q[i];
      lv[i].d = dd[i];
    }
    std::vector<Item> pit;
    sample_start(lv, nb, pit, true);
    applyA_levels(lv, pit, its);
    std::vector<Batch> pv(lv.size());
    sample_finish(lv, pit, its, pv);
    for (int i : which) {
      StochLevel& sl = lv[i];
      Cand& cd_ = out[i];
      const std::vector<zc>& t = pv[i].vals;
      zc mu = 0;
      for (const zc& y : t) mu += y;
      mu /= (double)t.size();
      double V = 0;
      for (const zc& y : t) V += std::norm(y - mu);
      cd_.V = V / (double)(t.size() - 1);
      cd_.mean = mu;
      double cs = 0;
      for (double x : pv[i].cost) cs += x;
      sl.lr_cost += cs;  // the pilot work is planning overhead of the Hutch++ phase
      if (p.cost == MGM_COST_FLOPS) {
        cd_.C = cs / (double)t.size();
        cd_.W = sl.lr_cost - cs - w0[i];
      } else {
        const double ca = apply_static(i, sl);
        cd_.C = p.cost == MGM_COST_FIXED ? ca : ca + 2.0 * (double)sl.n * dd[i];
        cd_.W = (std::max(1, p.k_power) + 1.0) * dd[i] * ca;
      }
      sl.Q = saveQ[i];
      sl.d = saved[i];
    }
  }
  void low_rank_adaptive(std::vector<StochLevel>& lv) {
    const int nl = (int)lv.size();
    require(p.pilot >= 2, "adaptive d: pilot must be >= 2");
    require(p.d_max <= 64, "adaptive d: d_max must be <= 64");
    std::vector<int> which, dd(nl), buf(nl, 0);
    std::vector<Cand> best(nl), trial(nl);
    for (int i = 0; i < nl; ++i) {
      require(lv[i].d >= 1 && lv[i].d <= p.d_max, "adaptive d: need 1 <= d[l] <= d_max");
      which.push_back(i);
      dd[i] = lv[i].d;
    }
    candidates(lv, which, dd, buf, best);
    zc tau0 = hutch ? zc(0) : zc(g.trL[0], g.trL[1]);
    for (int i = 0; i < nl; ++i) tau0 += best[i].mean + best[i].tau_lr;
    const double rho2 = (p.eps * std::abs(tau0)) * (p.eps * std::abs(tau0)) / nl;
    auto T = [&](const Cand& x) { return x.W + x.V * x.C / rho2; };
    std::vector<char> growing(nl);
    for (int i = 0; i < nl; ++i) growing[i] = 2 * best[i].d <= p.d_max;
    while (true) {
      which.clear();
      for (int i = 0; i < nl; ++i)
        if (growing[i]) {
          which.push_back(i);
          dd[i] = 2 * best[i].d;
          buf[i] = 1 - best[i].buf;  // the trial goes into the other buffer
        }
      if (which.empty()) break;
      candidates(lv, which, dd, buf, trial);
      for (int i : which) {
        if (T(trial[i]) < T(best[i])) {
          best[i] = trial[i];
          growing[i] = 2 * best[i].d <= p.d_max;
        } else {
          growing[i] = 0;
        }
      }
    }
    for (int i = 0; i < nl; ++i) {
      StochLevel& sl = lv[i];
      sl.d = best[i].d;
      sl.Q = best[i].buf ? &g.est.Q2[i] : &g.est.Q[i];
      sl.tau_lr = best[i].tau_lr;
      if (p.cost == MGM_COST_STATIC) sl.cost = apply_static(i, sl) + 2.0 * (double)sl.n * sl.d;
    }
  }

  // Deflation basis (Sec. 2.2): k_power sweeps of block subspace iteration
  // Q <- qr(D^{-1} gamma5 D^{-1} gamma5 Q) from noise of purpose DEFLATE; it
  // converges to the right singular vectors of D of the smallest singular
  // values, since D^{-1} D^{-H} = D^{-1} gamma5 D^{-1} gamma5 here.
  void deflation_basis(StochLevel& sl) {
    hipStream_t s = c->stream;
    const int d = sl.d;
    const int64_t n = sl.n;
    cd* S = g.est.S[0].as<cd>();
    cd* Y = g.est.Y[0].as<cd>();
    t1.ensure(sizeof(cd) * (size_t)d * n);
    cd* T = t1.as<cd>();
    launch_noise<double>(s, S, n, d, p.noise, p.seed, MGM_PURPOSE_DEFLATE, 0, 0);
    const cd* X = S;
    for (int it = 0; it < std::max(1, p.k_power); ++it) {
      launch_gamma5(s, X, Y, (int64_t)d * n);
      for (int v : solve(0, d, Y, T)) sl.lr_cost += solve_cost(0, v);
      launch_gamma5(s, T, Y, (int64_t)d * n);
      for (int v : solve(0, d, Y, T)) sl.lr_cost += solve_cost(0, v);
      orthonormalize(c, n, d, T, sl.Q->as<cd>());
      X = sl.Q->as<cd>();
    }
  }

  // Ritz singular triplets of D on span(Q): W = D Q, G = W^H W, C = W^H Q;
  // sum_i u_i^H v_i / sigma_i = tr(G^{-1} C) (with G = Y diag(sigma^2) Y^H,
  // v_i = Q y_i, u_i = W y_i / sigma_i) and sigma = sqrt(eig(G)).
  void ritz_triplets(StochLevel& sl) {
    hipStream_t s = c->stream;
    const int d = sl.d;
    const int64_t n = sl.n;
    cd* W = g.est.S[0].as<cd>();  // free after the subspace iteration
    apply_level(c, g, 0, d, sl.Q->as<cd>(), W);
    dots.ensure(sizeof(cd) * 2 * (size_t)d * d);
    cd* Gd = dots.as<cd>();
    cd* Cd = Gd + (int64_t)d * d;
    launch_dot_multi_ld<double>(s, W, n, 0, d, W, n, d, Gd, d, 0, nullptr, part.as<cd>());
    launch_dot_multi_ld<double>(s, W, n, 0, d, sl.Q->as<cd>(), n, d, Cd, d, 0, nullptr, part.as<cd>());
    std::vector<cd> h(2 * (size_t)d * d);
    HIPCHK(hipMemcpyAsync(h.data(), Gd, sizeof(cd) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    // out[r * d + i] = (W_i)^H X_r, i.e. G[i][r] and C[i][r]
    std::vector<zc> G((size_t)d * d), Cm((size_t)d * d);
    for (int r = 0; r < d; ++r)
      for (int i = 0; i < d; ++i) {
        G[(size_t)i * d + r] = zc(h[(size_t)r * d + i].re, h[(size_t)r * d + i].im);
        Cm[(size_t)i * d + r] = zc(h[(size_t)d * d + (size_t)r * d + i].re, h[(size_t)d * d + (size_t)r * d + i].im);
      }
    // Cholesky G = L L^H, then tr(G^{-1} C) = sum_j (L^{-H} L^{-1} C)_jj
    std::vector<zc> Lc = G;
    for (int j = 0; j < d; ++j) {
      double dj = Lc[(size_t)j * d + j].real();
      for (int k = 0; k < j; ++k) dj -= std::norm(Lc[(size_t)j * d + k]);
      require(dj > 0, "deflation: D Q is rank-deficient", MGM_ENONFINITE);
      dj = std::sqrt(dj);
      Lc[(size_t)j * d + j] = dj;
      for (int i = j + 1; i < d; ++i) {
        zc v = Lc[(size_t)i * d + j];
        for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * d + k] * std::conj(Lc[(size_t)j * d + k]);
        Lc[(size_t)i * d + j] = v / dj;
      }
    }
    zc tr = 0;
    std::vector<zc> col(d);
    for (int r = 0; r < d; ++r) {
      for (int i = 0; i < d; ++i) col[i] = Cm[(size_t)i * d + r];
      for (int i = 0; i < d; ++i) {  // L y = c
        zc v = col[i];
        for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * d + k] * col[k];
        col[i] = v / Lc[(size_t)i * d + i];
      }
      for (int i = d - 1; i >= 0; --i) {  // L^H x = y
        zc v = col[i];
        for (int k = i + 1; k < d; ++k) v -= std::conj(Lc[(size_t)k * d + i]) * col[k];
        col[i] = v / Lc[(size_t)i * d + i];
      }
      tr += col[r];
    }
    res.defl_ritz[0] = tr.real();
    res.defl_ritz[1] = tr.imag();
    if (res.sigma_dump) {
      const std::vector<double> lam = hermitian_eigenvalues(G, d);
      for (int i = 0; i < d; ++i) res.sigma_dump[i] = std::sqrt(std::max(0.0, lam[i]));
    }
  }

  // eigenvalues (ascending) of the Hermitian d x d matrix A by cyclic Jacobi
  // on its real symmetric embedding [[Re A, -Im A], [Im A, Re A]], whose
  // eigenvalues are those of A, each twice
  static std::vector<double> hermitian_eigenvalues(const std::vector<zc>& A, int d) {
    const int m = 2 * d;
    std::vector<double> B((size_t)m * m);
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const zc a = A[(size_t)i * d + j];
        B[(size_t)i * m + j] = a.real();
        B[(size_t)(i + d) * m + j + d] = a.real();
        B[(size_t)i * m + j + d] = -a.imag();
        B[(size_t)(i + d) * m + j] = a.imag();
      }
    for (int sweep = 0; sweep < 100; ++sweep) {
      double off = 0, tot = 0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          tot += B[(size_t)i * m + j] * B[(size_t)i * m + j];
          if (i != j) off += B[(size_t)i * m + j] * B[(size_t)i * m + j];
        }
      if (off <= 1e-30 * tot) break;
      for (int pp = 0; pp < m; ++pp)
        for (int q = pp + 1; q < m; ++q) {
          const double apq = B[(size_t)pp * m + q];
          if (apq == 0.0) continue;
          const double th = (B[(size_t)q * m + q] - B[(size_t)pp * m + pp]) / (2.0 * apq);
          const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
          const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
          for (int k = 0; k < m; ++k) {  // columns pp, q
            const double bkp = B[(size_t)k * m + pp], bkq = B[(size_t)k * m + q];
            B[(size_t)k * m + pp] = cs * bkp - sn * bkq;
            B[(size_t)k * m + q] = sn * bkp + cs * bkq;
          }
          for (int k = 0; k < m; ++k) {  // rows pp, q
            const double bpk = B[(size_t)pp * m + k], bqk = B[(size_t)q * m + k];
            B[(size_t)pp * m + k] = cs * bpk - sn * bqk;
            B[(size_t)q * m + k] = sn * bpk + cs * bqk;
          }
        }
    }
    std::vector<double> ev(m);
    for (int i = 0; i < m; ++i) ev[i] = B[(size_t)i * m + i];
    std::sort(ev.begin(), ev.end());
    std::vector<double> out(d);
    for (int i = 0; i < d; ++i) out[i] = 0.5 * (ev[2 * i] + ev[2 * i + 1]);
    return out;
  }

  // noise zeta for samples s .. s+b[i]-1 of every difference i with b[i] > 0
  // (s = samples taken so far); appends the blocks Y = A zeta to `items`
  void sample_start(std::vector<StochLevel>& lv, const std::vector<int>& b, std::vector<Item>& items,
                    bool pilot = false) {
    for (int i = 0; i < (int)lv.size(); ++i) {
      if (b[i] <= 0) continue;
      StochLevel& sl = lv[i];
      g.est.Z[i].ensure(sizeof(cd) * (size_t)kmax * sl.n);
      g.est.X[i].ensure(sizeof(cd) * (size_t)kmax * sl.n);
      // stochastic samples continue their stream; pilot samples are the
      // same PILOT vectors 0 .. b-1 for every candidate
      launch_noise<double>(c->stream, g.est.Z[i].as<cd>(), sl.n, b[i], p.noise, p.seed,
                           pilot ? MGM_PURPOSE_PILOT : MGM_PURPOSE_SAMPLE, i, pilot ? 0 : sl.s());
      if (two_sided) project(sl, i, b[i]);
      items.push_back({i, b[i], g.est.Z[i].as<cd>(), g.est.X[i].as<cd>()});
    }
  }

  // tau_{s,l} = z^H (A zeta) with z = zeta - Q (Q^H zeta), for the blocks
  // sample_start made (X = zeta, Y = A zeta)
  void sample_finish(std::vector<StochLevel>& lv, const std::vector<Item>& items, const std::vector<Its>& its,
                     std::vector<Batch>& out) {
    const std::vector<int> req = sample_finish_launch(lv, items);
    sample_finish_collect(lv, items, its, dots_fetch(), req, out);
  }
  // the projections and the dots of the blocks (slice indices of dots_add)
  std::vector<int> sample_finish_launch(std::vector<StochLevel>& lv, const std::vector<Item>& items) {
    std::vector<int> req;
    for (const Item& it : items) {
      StochLevel& sl = lv[it.i];
      if (!two_sided) project(sl, it.i, it.k);  // (two-sided: done before the solve)
      req.push_back(dots_add(g.est.Z[it.i].as<cd>(), it.Y, sl.n, it.k));
    }
    return req;
  }
  void sample_finish_collect(std::vector<StochLevel>& lv, const std::vector<Item>& items,
                             const std::vector<Its>& its, const std::vector<std::vector<zc>>& got,
                             const std::vector<int>& req, std::vector<Batch>& out) {
    for (size_t q = 0; q < items.size(); ++q) {
      const Item& it = items[q];
      StochLevel& sl = lv[it.i];
      Batch& bt = out[it.i];
      bt.vals = got[req[q]];
      bt.its = its[q];
      bt.cost.resize(it.k);
      for (int v = 0; v < it.k; ++v) bt.cost[v] = apply_cost(sl.level, its[q][v]) + 2.0 * (double)sl.n * sl.d;
    }
  }

  // z = zeta - Q (Q^H zeta) in place for the k noise vectors of difference i
  void project(StochLevel& sl, int i, int k) {
    if (sl.d <= 0) return;
    hipStream_t s = c->stream;
    const int64_t n = sl.n;
    cd* Z = g.est.Z[i].as<cd>();
    DevBuf& C = g.est.C[i];
    C.ensure(sizeof(cd) * (size_t)kmax * sl.d);
    DevBuf& pp = g.est.ppart[i];
    pp.ensure(sizeof(cd) * (size_t)proj_partials(n) * sl.d * std::min(kmax, 64));
    // blocks of at most 64 vectors (the matrix-core tiles of one launch)
    for (int r0 = 0; r0 < k; r0 += 64)
      launch_project(s, sl.Q->as<cd>(), sl.d, Z + (int64_t)r0 * n, std::min(64, k - r0), n, C.as<cd>(),
                     pp.as<cd>());
  }

  void sample_batches(std::vector<StochLevel>& lv, const std::vector<int>& b, std::vector<Batch>& out) {
    std::vector<Item> items;
    std::vector<Its> its;
    sample_start(lv, b, items);
    applyA_levels(lv, items, its);
    sample_finish(lv, items, its, out);
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

  // samples of the next speculative batch for every active level.  The
  // batch length only decides how much work may be discarded, never the
  // result: in adaptive mode it is the number of samples the current
  // variances and targets predict are still missing (all active levels
  // advance together, as in Alg. 2), between 4 and p.batch; s is the number
  // of samples taken per level so far and tau the current estimate.
  std::vector<int> batch_sizes(const std::vector<StochLevel>& lv, int s, zc tau, int maxS) {
    const int nst = (int)lv.size();
    const int minS = std::max(2, p.min_samples);
    int common = p.batch;
    if (!p.fixed_samples) {
      if (s < 2) {
        common = std::min(p.batch, std::max(minS, p.batch / 2));
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
      // up to the 16-RHS tile of the matrix-core kernels: no slower, the
      // replay below takes the same samples whatever the batch holds, and
      // the level solves see few distinct RHS counts (their captured graphs
      // are replayed instead of captured again)
      common = std::min(p.batch, (common + 15) / 16 * 16);
    }
    std::vector<int> nb(nst, 0);
    for (int i = 0; i < nst; ++i) {
      if (!lv[i].active) continue;
      int b = common;
      if (p.fixed_samples) b = std::min(b, p.fixed_samples[i] - lv[i].s());
      nb[i] = std::min(b, maxS - lv[i].s());
    }
    return nb;
  }

  int run() {
    require(g.mg_ready, "trace_estimate needs setup_mg first", MGM_ESTATE);
    require(p.eps > 0 || p.fixed_samples, "eps must be positive");
    require(p.batch >= 1, "batch must be >= 1");
    require(p.cost == MGM_COST_STATIC || p.cost == MGM_COST_FIXED || p.cost == MGM_COST_FLOPS,
            "unknown cost model");
    require(p.projection == MGM_PROJ_ONE_SIDED || p.projection == MGM_PROJ_TWO_SIDED, "unknown projection");
    const int nst = hutch ? 1 : L - 1;
    require(nst >= 1, "MLMC variants need at least two levels");
    const bool lr = p.variant == MGM_VARIANT_HUTCHPP || p.variant == MGM_VARIANT_MLMCPP || deflated;
    const bool adaptive = p.d_max > 0 && (p.variant == MGM_VARIANT_HUTCHPP || p.variant == MGM_VARIANT_MLMCPP);
    require(!deflated || (p.d[0] >= 1 && p.d[0] <= 64), "deflated variant: d[0] must be in [1, 64]");
    std::vector<StochLevel> lv(nst);
    for (int i = 0; i < nst; ++i) {
      StochLevel& sl = lv[i];
      sl.Q = &g.est.Q[i];
      sl.level = hutch ? 0 : i;
      sl.n = (hutch || full) ? g.levels[0]->n : g.levels[i]->n;
      sl.d = lr ? p.d[i] : 0;
      require(sl.d >= 0 && sl.d <= 64, "d must be in [0, 64]");
      if (p.cost == MGM_COST_FIXED) {
        sl.cost = p.fixed_cost[i];
      } else if (p.cost == MGM_COST_STATIC) {
        sl.cost = c_nnzD[i] + 2.0 * sl.n * sl.d;
        if (i + 1 < L) sl.cost += c_nnzD[i + 1];
      } else {
        sl.cost = std::nan("");  // C_l: the mean cost of the samples taken
      }
    }
    const zc tau_exact = hutch ? zc(0) : zc(g.trL[0], g.trL[1]);
    const int minS = std::max(2, p.min_samples);
    // a batch never exceeds p.batch samples per level (batch_sizes)
    kmax = std::max(1, p.batch);
    for (int i = 0; i < nst; ++i) kmax = std::max(kmax, lv[i].d);
    if (adaptive) kmax = std::max(kmax, std::max(p.d_max, p.pilot));
    // every reduction workspace at its largest size up front (no reallocation later)
    part.ensure(sizeof(cd) * (size_t)kmax * 64 * reduce_chunks(g.levels[0]->n) + 64);
    // one dot batch holds at most two blocks per difference (tau_lr and samples)
    dots.ensure(sizeof(cd) * (size_t)2 * nst * kmax);
    const int maxS = p.max_samples > 0 ? p.max_samples : (1 << 30);
    zc tau = 0;
    int s = 0;
    // the first stochastic batch rides with the last low-rank round
    std::vector<Batch> pre(nst);
    bool have_pre = false;
    if (lr && adaptive) {
      low_rank_adaptive(lv);
    } else if (lr) {
      const std::vector<int> nb = batch_sizes(lv, s, tau, maxS);
      low_rank_all(lv, nb, pre);
      have_pre = true;
    }
    while (true) {
      bool any = false;
      for (auto& sl : lv) any = any || sl.active;
      if (!any) break;
      std::vector<Batch> vals(nst);
      if (have_pre) {
        vals.swap(pre);
        have_pre = false;
      } else {
        sample_batches(lv, batch_sizes(lv, s, tau, maxS), vals);
      }
      // replay Alg. 2 sample by sample; stop where an active level has no
      // evaluated sample left (levels advance in lockstep)
      for (int t = 0;; ++t) {
        bool any_active = false, missing = false;
        for (int i = 0; i < nst; ++i) {
          any_active = any_active || lv[i].active;
          if (lv[i].active && t >= (int)vals[i].vals.size()) missing = true;
        }
        if (!any_active || missing) break;
        for (int i = 0; i < nst; ++i) {
          StochLevel& sl = lv[i];
          if (!sl.active) continue;
          sl.samples.push_back(vals[i].vals[t]);
          sl.costs.push_back(vals[i].cost[t]);
          sl.its.push_back(vals[i].its[t]);
          sl.cost_sum += vals[i].cost[t];
          if (p.cost == MGM_COST_FLOPS) sl.cost = sl.cost_sum / sl.s();
        }
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
      res.lvl_d[i] = lv[i].d;
      res.lvl_lr_work[i] = lv[i].lr_cost;
      res.lvl_work[i] = lv[i].lr_cost + lv[i].cost_sum;
      const int nd = res.max_dump > 0 ? std::min(res.max_dump, lv[i].s()) : 0;
      for (int k = 0; k < nd; ++k) {
        const int64_t at = (int64_t)i * res.max_dump + k;
        if (res.sample_dump) {
          res.sample_dump[at * 2] = lv[i].samples[k].real();
          res.sample_dump[at * 2 + 1] = lv[i].samples[k].imag();
        }
        if (res.cost_dump) res.cost_dump[at] = lv[i].costs[k];
        if (res.iter_dump) {
          res.iter_dump[at * 2] = lv[i].its[k][0];
          res.iter_dump[at * 2 + 1] = lv[i].its[k][1];
        }
      }
    }
    return MGM_OK;
  }
};

}  // namespace

int trace_estimate(mgm_ctx* c, Gauge& g, const mgm_trace_params& p, mgm_trace_result& r) {
  r.defl_ritz[0] = r.defl_ritz[1] = 0;
  for (int i = 0; i < MGM_MAX_LEVELS; ++i) {
    r.lvl_solves[i] = 0;
    r.lvl_iters[i] = 0;
    r.lvl_samples[i] = 0;
    r.lvl_lr_work[i] = 0;
    r.lvl_work[i] = 0;
    r.lvl_d[i] = 0;
  }
  Estimator e(c, g, p, r);
  return e.run();
}

}  // namespace mgm
