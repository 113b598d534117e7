// Solvers on top of the level kernels: the multigrid preconditioner (coarse
// correction by a fixed-length inner FGMRES -- a K-cycle -- or the dense
// coarsest inverse, then red/black SAP post-smoothing), the outer FP64
// right-preconditioned FGMRES with per-RHS stopping on the true residual, the
// CholQR orthonormalisation, and the deterministic bootstrap setup of the
// aggregation hierarchy.
#include <algorithm>
#include <cmath>

#include <type_traits>

#include "internal.h"

namespace mgm {

namespace {

template <class T>
LevelData<T>& ldata(Level& L);
template <>
LevelData<double>& ldata<double>(Level& L) { return L.d; }
template <>
LevelData<float>& ldata<float>(Level& L) { return L.f; }

template <class T>
Work<T>& work(Level& L, int slot);
template <>
Work<double>& work<double>(Level& L, int slot) { return L.wd[slot]; }
template <>
Work<float>& work<float>(Level& L, int slot) { return L.wf[slot]; }

template <class T>
const cx<T>* links_of(Gauge& g);
template <>
const cd* links_of<double>(Gauge& g) { return g.links.as<cd>(); }
template <>
const cf* links_of<float>(Gauge& g) { return g.links32.as<cf>(); }

template <class T>
void ensure_work(Level& L, int slot, int nrhs, int m) {
  Work<T>& W = work<T>(L, slot);
  const int64_t n = L.n;
  const size_t c = sizeof(cx<T>);
  W.V.ensure(c * (size_t)(m + 1) * nrhs * n);
  W.Z.ensure(c * (size_t)m * nrhs * n);
  W.w.ensure(c * (size_t)nrhs * n);
  W.H.ensure(c * (size_t)nrhs * m * (m + 1));
  W.cs.ensure(sizeof(T) * (size_t)nrhs * m);
  W.sn.ensure(c * (size_t)nrhs * m);
  W.g.ensure(c * (size_t)nrhs * (m + 1));
  W.y.ensure(c * (size_t)nrhs * m);
  W.beta.ensure(sizeof(T) * nrhs);
  W.thr.ensure(sizeof(T) * nrhs);
  W.bnorm.ensure(sizeof(T) * nrhs);
  W.act.ensure(sizeof(int) * 2 * nrhs);  // active flags, then "done" flags
  W.nit.ensure(sizeof(int) * nrhs);
  W.part.ensure(2 * c * (size_t)nrhs * (m + 1) * reduce_chunks(n));  // two Gram-Schmidt passes' partials
  W.npart.ensure(sizeof(T) * (size_t)nrhs * reduce_chunks(n));
  W.coef.ensure(c * (size_t)nrhs * (m + 1));
  W.coef2.ensure(c * (size_t)nrhs * (m + 1));
  W.gram.ensure(c * (size_t)nrhs * (m + 1) * (m + 1));
}

// FP16 mode: coarse levels with 16 dofs per site apply their blocks in FP16
bool half_blocks(const Gauge& g, const Level& L) {
  return g.prm.precision == MGM_PREC_FP16 && L.M == 16 && L.f.hblocks.p != nullptr;
}

template <class T>
void apply_op(mgm_ctx* c, Gauge& g, int l, int nrhs, const cx<T>* x, cx<T>* y, const cx<T>* b,
              const int* act) {
  Level& L = *g.levels[l];
  if (l == 0) {
    launch_wilson<T>(c->stream, links_of<T>(g), (T)(g.m0 + 2.0), g.Lx, g.Lt, nrhs, x, y, b, act);
  } else if constexpr (std::is_same<T, float>::value) {
    if (half_blocks(g, L))
      launch_stencil_h(c->stream, L.f.hblocks.as<chalf>(), L.Nx, L.Nt, nrhs, x, y, b, act);
    else
      launch_stencil<T>(c->stream, ldata<T>(L).B(), L.Nx, L.Nt, L.M, nrhs, x, y, b, act);
  } else {
    launch_stencil<T>(c->stream, ldata<T>(L).B(), L.Nx, L.Nt, L.M, nrhs, x, y, b, act);
  }
}

template <class T>
void fgmres_inner(mgm_ctx* c, Gauge& g, int l, int nrhs, const cx<T>* b, cx<T>* x, int m, T tol,
                  const int* parent);

// whether precond<float> on level l can hand its result over in FP64 itself
// (last SAP cycle on 4x4-site blocks of 2 dofs)
bool precond_writes_fp64(const Gauge& g, const Level& L) {
  return L.M == 2 && L.sbx == 4 && L.sbt == 4 && L.sap_cycles > 0 && !L.is_coarsest &&
         !(half_blocks(g, L) && L.sbt == 1);
}

// whether the FP32 cycle on level l keeps its vectors in the block-major
// layout (SAP blocks = aggregates = 4x4 sites of 2 dofs, 8 test vectors; its
// input is rounded into that layout and its FP64 result written back in the
// lattice layout by the last SAP sweeps)
bool fine_blocked(const Gauge& g, const Level& L) {
  return precond_writes_fp64(g, L) && L.has_coarse && L.bx == 4 && L.bt == 4 && L.ntv == 8;
}

// x = D^{-1} r on the coarsest level from its dense inverse (in the FP16
// mode the FP16 copy, when the inverse fits FP16's range)
template <class T>
void coarse_solve(mgm_ctx* c, Gauge& g, Level& L, int nrhs, const cx<T>* r, cx<T>* x, const int* act) {
  if constexpr (std::is_same<T, float>::value) {
    if (g.prm.precision == MGM_PREC_FP16 && L.f.hdinv.p) {
      launch_dense_apply_h(c->stream, L.f.hdinv.as<chalf>(), L.n, nrhs, r, x, act);
      return;
    }
  }
  launch_dense_apply<T>(c->stream, ldata<T>(L).dinv.template as<cx<T>>(), L.n, nrhs, r, x, act,
                        &g.scratch[c->wslot]);
}

// M_l r -> x.  Coarsest: x = D^{-1} r.  Else x = P_l C_{l+1}(P_l^H r) (or 0
// while the hierarchy below l is not built), then SAP cycles on D x = r.
template <class T>
void precond(mgm_ctx* c, Gauge& g, int l, int nrhs, const cx<T>* r, cx<T>* x, const int* act,
             cd* x64 = nullptr) {
  hipStream_t s = c->stream;
  Level& L = *g.levels[l];
  LevelData<T>& D = ldata<T>(L);
  if (L.is_coarsest) {
    coarse_solve<T>(c, g, L, nrhs, r, x, act);
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (x64 && fine_blocked(g, L)) {  // r and x block-major, the result also into x64
      Level& C = *g.levels[l + 1];
      Work<float>& W = work<float>(L, c->wslot);
      W.rc.ensure(sizeof(cf) * (size_t)nrhs * C.n);
      W.ec.ensure(sizeof(cf) * (size_t)nrhs * C.n);
      cf* rc = W.rc.as<cf>();
      cf* ec = W.ec.as<cf>();
      launch_restrict_blk(s, D.P.template as<cf>(), L.Nx, L.Nt, nrhs, r, rc, act);
      if (C.is_coarsest) {
        coarse_solve<float>(c, g, C, nrhs, rc, ec, act);
      } else if (C.inner_iters <= 0) {
        precond<float>(c, g, l + 1, nrhs, rc, ec, act);
      } else {
        fgmres_inner<float>(c, g, l + 1, nrhs, rc, ec, C.inner_iters, (float)g.prm.inner_tol, act);
      }
      launch_prolong_blk(s, D.P.template as<cf>(), L.Nx, L.Nt, nrhs, ec, x, act);
      for (int cyc = 0; cyc < L.sap_cycles; ++cyc)
        for (int col = 0; col < 2; ++col)
          launch_sap0_blk(s, D.B(), D.sapinv.template as<cf>(), L.Nx, L.Nt, L.color_list[col].as<int>(),
                          L.ncolor[col], nrhs, r, x, act, cyc + 1 == L.sap_cycles ? x64 : nullptr);
      return;
    }
  }
  // FP16 2x2 or single-site sweeps after a 2x2-aggregate coarse correction:
  // the first colour's first sweep forms its halo from the coarse correction
  // itself, so the prolongation is not stored (it is read nowhere else)
  const cf* ec_halo = nullptr;
  if (L.has_coarse) {
    Level& C = *g.levels[l + 1];
    Work<T>& W = work<T>(L, c->wslot);
    W.rc.ensure(sizeof(cx<T>) * (size_t)nrhs * C.n);
    W.ec.ensure(sizeof(cx<T>) * (size_t)nrhs * C.n);
    cx<T>* rc = W.rc.template as<cx<T>>();
    cx<T>* ec = W.ec.template as<cx<T>>();
    launch_restrict<T>(s, D.P.template as<cx<T>>(), L.Nx, L.Nt, L.M, L.bx, L.bt, L.ntv, nrhs, r, rc, act);
    if (C.is_coarsest) {
      coarse_solve<T>(c, g, C, nrhs, rc, ec, act);
    } else if (C.inner_iters <= 0) {
      precond<T>(c, g, l + 1, nrhs, rc, ec, act);  // plain V-cycle on the coarse level
    } else {
      fgmres_inner<T>(c, g, l + 1, nrhs, rc, ec, C.inner_iters, (T)g.prm.inner_tol, act);
    }
    bool fused = false;
    if constexpr (std::is_same<T, float>::value)
      fused = half_blocks(g, L) && L.sap_cycles > 0 && L.f.hP.p &&
              ((L.sbx == 2 && L.sbt == 2 && L.f.hsapM.p) || (L.sbx == 1 && L.sbt == 1));
    if (fused)
      ec_halo = reinterpret_cast<const cf*>(ec);
    else
      launch_prolong<T>(s, D.P.template as<cx<T>>(), L.Nx, L.Nt, L.M, L.bx, L.bt, L.ntv, nrhs, ec, x, 0, act);
  } else {
    launch_axpby<T>(s, (T)0, r, (T)0, nullptr, x, L.n, nrhs, act);
  }
  if (L.M == 16 && L.sbx == 2 && L.sbt == 2 && L.sap_cycles > 0) {
    // premultiplied 2x2-site sweeps x_B = rho_B - M_B x_H; the first cycle
    // forms rho_B = inv_B r_B and keeps it for the others
    require(D.sapM.p && D.sapinv.p, "2x2 SAP blocks: premultiplied operator missing", MGM_ESTATE);
    Work<T>& W = work<T>(L, c->wslot);
    W.rho.ensure(sizeof(cx<T>) * (size_t)nrhs * L.n);
    for (int cyc = 0; cyc < L.sap_cycles; ++cyc)
      for (int col = 0; col < 2; ++col) {
        const int* bl = L.color_list[col].as<int>();
        if constexpr (std::is_same<T, float>::value) {
          if (half_blocks(g, L)) {
            const bool from_coarse = ec_halo && cyc == 0 && col == 0;
            launch_sap4p_h(s, L.f.hsapM.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, bl, L.ncolor[col], nrhs,
                           cyc == 0, r, W.rho.template as<cf>(), x, act, from_coarse ? L.f.hP.as<chalf>() : nullptr,
                           from_coarse ? ec_halo : nullptr);
            continue;
          }
        }
        launch_sap4p<T>(s, D.sapM.template as<cx<T>>(), D.sapinv.template as<cx<T>>(), L.Nx, L.Nt, bl,
                        L.ncolor[col], nrhs, cyc == 0, r, W.rho.template as<cx<T>>(), x, act);
      }
    return;
  }
  bool half = false;
  if constexpr (std::is_same<T, float>::value) {
    half = half_blocks(g, L) && L.sbt == 1 && (L.sbx == 1 || L.sbx == 2);
    if (half && L.sbx == 2 && L.f.hsapM.p && L.sap_cycles > 0) {
      // premultiplied two-site sweeps x_B = rho_B - M_B x_H; the first cycle
      // forms rho_B = inv_B r_B and keeps it for the others
      Work<float>& W = work<float>(L, c->wslot);
      W.rho.ensure(sizeof(cf) * (size_t)nrhs * L.n);
      for (int cyc = 0; cyc < L.sap_cycles; ++cyc)
        for (int col = 0; col < 2; ++col)
          launch_sap2p_h(s, L.f.hsapM.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, L.color_list[col].as<int>(),
                         L.ncolor[col], nrhs, cyc == 0, r, W.rho.as<cf>(), x, act);
      return;
    }
  }
  for (int cyc = 0; cyc < L.sap_cycles; ++cyc)
    for (int col = 0; col < 2; ++col) {
      if constexpr (std::is_same<T, float>::value) {
        if (half) {
          const bool from_coarse = ec_halo && cyc == 0 && col == 0;
          launch_sap_h(s, L.f.hblocks.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, L.sbx, L.sbt,
                       L.color_list[col].as<int>(), L.ncolor[col], nrhs, r, x, act,
                       from_coarse ? L.f.hP.as<chalf>() : nullptr, from_coarse ? ec_halo : nullptr);
          continue;
        }
      }
      // the last cycle's two colours leave every block final: they also
      // store the FP64 result when the caller asked for it
      launch_sap_sweep<T>(s, D.B(), D.sapinv.template as<cx<T>>(), L.Nx, L.Nt, L.M, L.sbx, L.sbt,
                          L.color_list[col].as<int>(), L.ncolor[col], nrhs, r, x, act,
                          cyc + 1 == L.sap_cycles ? x64 : nullptr);
    }
}

// One Arnoldi step j of FGMRES: z_j = M v_j, w = D z_j, CGS2 against v_0..v_j,
// Hessenberg column, v_{j+1} = w/||w||, Givens update.
// fused (FP64 steps whose preconditioner rounds its input to FP32): step
// j's last launch forms the Hessenberg column and Givens update together
// with v_{j+1} = w / |w| and its FP32 rounding (into W.cvt_in), and the next
// step calls prec with v = null.
// cvt0 (with fused, step 0): the cycle start has rounded v_0 into W.cvt_in.
template <class T, class PrecFn>
void arnoldi_step(mgm_ctx* c, Gauge& g, int l, int nrhs, int j, int m, Work<T>& W, PrecFn&& prec,
                  int* host_flags = nullptr, bool fused = false, bool cvt0 = false) {
  hipStream_t s = c->stream;
  Level& L = *g.levels[l];
  const int64_t n = L.n;
  const int64_t vs = (int64_t)nrhs * n;
  cx<T>* V = W.V.template as<cx<T>>();
  cx<T>* Z = W.Z.template as<cx<T>>();
  cx<T>* w = W.w.template as<cx<T>>();
  int* act = W.act.template as<int>();
  cx<T>* part = W.part.template as<cx<T>>();
  cx<T>* c1 = W.coef.template as<cx<T>>();
  cx<T>* c2 = W.coef2.template as<cx<T>>();
  T* hn = W.beta.template as<T>() ;  // beta is free after the cycle start: reuse for ||w||
  T* np = W.npart.template as<T>();
  if (fused && (j > 0 || cvt0)) {
    // v_j was rounded into W.cvt_in by the previous step's last launch (or,
    // for step 0, by the cycle start)
    prec(nullptr, Z + j * vs, (const int*)act);
  } else {
    prec(V + j * vs, Z + j * vs, (const int*)act);
  }
  apply_op<T>(c, g, l, nrhs, Z + j * vs, w, nullptr, act);
  // Classical Gram-Schmidt applied twice, the second pass in its Gram form:
  // one read of the basis gives h1 = V^H w and the Gram column V^H v_j, and
  // one update applies h1 + (I - G) h1 (= h1 + V^H (w - V h1) with G = V^H V);
  // each reduction over chunks is done by the kernel that consumes it
  const int nch = launch_dot_partial2<T>(s, V, vs, n, j + 1, w, V + j * vs, n, nrhs, act, part);
  launch_update_gram<T>(s, V, vs, n, j + 1, part, nch, W.gram.template as<cx<T>>(), m + 1, c1, m + 1, w, n, nrhs,
                        act, np);
  c2 = nullptr;
  if (fused) {
    // Hessenberg column, Givens update, host flags, and v_{j+1} = w / |w|
    // with its FP32 rounding for the next step, in one launch
    if constexpr (std::is_same<T, double>::value) {
      W.cvt_in.ensure(sizeof(cf) * (size_t)vs);
      launch_hcol_scale<T>(s, j, m, nrhs, c1, np, W.H.template as<cx<T>>(), W.cs.template as<T>(),
                           W.sn.template as<cx<T>>(), W.g.template as<cx<T>>(), W.thr.template as<T>(), act,
                           W.nit.template as<int>(), host_flags, w, n, V + (j + 1) * vs, W.cvt_in.template as<cf>(),
                           fine_blocked(g, L) ? L.Nx : 0);
    }
    return;
  }
  launch_scale_r<T>(s, w, np, n, nrhs, V + (j + 1) * vs, hn, act);
  launch_hcol_givens<T>(s, j, m, nrhs, c1, c2, hn, W.H.template as<cx<T>>(), W.cs.template as<T>(),
                        W.sn.template as<cx<T>>(), W.g.template as<cx<T>>(), W.thr.template as<T>(), act,
                        W.nit.template as<int>(), host_flags);
}

// x = m steps of FGMRES from x0 = 0 on D_l x = b (no restart), a RHS stops
// early when its residual estimate reaches tol * ||b||.  No host sync.
template <class T>
void fgmres_inner(mgm_ctx* c, Gauge& g, int l, int nrhs, const cx<T>* b, cx<T>* x, int m, T tol,
                  const int* parent) {
  hipStream_t s = c->stream;
  Level& L = *g.levels[l];
  require(m >= 1 && m <= 63, "inner FGMRES length must be in [1, 63]");
  ensure_work<T>(L, c->wslot, nrhs, m);
  Work<T>& W = work<T>(L, c->wslot);
  const int64_t n = L.n;
  cx<T>* V = W.V.template as<cx<T>>();
  cx<T>* Z = W.Z.template as<cx<T>>();
  int* act = W.act.template as<int>();
  T* beta = W.beta.template as<T>();
  launch_norm<T>(s, b, n, nrhs, beta, parent, (T*)W.part.p);
  launch_fgmres_init<T>(s, nrhs, beta, parent, nullptr, tol, nullptr, m, act, W.nit.template as<int>(),
                        W.g.template as<cx<T>>(), W.thr.template as<T>());
  launch_scale<T>(s, b, beta, n, nrhs, V, act);
  for (int j = 0; j < m; ++j)
    arnoldi_step<T>(c, g, l, nrhs, j, m, W, [&](const cx<T>* v, cx<T>* z, const int* a) {
      precond<T>(c, g, l, nrhs, v, z, a);
    });
  launch_backsolve<T>(s, m, nrhs, W.H.template as<cx<T>>(), W.g.template as<cx<T>>(),
                      W.nit.template as<int>(), W.y.template as<cx<T>>());
  launch_axpby<T>(s, (T)0, b, (T)0, nullptr, x, n, nrhs, parent);
  launch_update_multi<T>(s, Z, (int64_t)nrhs * n, n, m, W.y.template as<cx<T>>(), m, (T)1, x, n, nrhs,
                         parent, nullptr, nullptr, W.nit.template as<int>());
}

}  // namespace

// ------------------------------------------------------------------ public solver pieces
void apply_level(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* x, cd* y) {
  apply_op<double>(c, g, l, nrhs, x, y, nullptr, nullptr);
}

// FP64 preconditioner entry; in FP32 mode the residual is rounded to FP32, the
// whole multigrid cycle runs in FP32, and the correction is widened again.
bool precondition_in_fp32(const Gauge& g) { return g.prm.precision != MGM_PREC_FP64 && g.mg_ready; }

// the FP32 cycle on the residual already rounded into W.cvt_in; x in FP64
void precondition_f32in(mgm_ctx* c, Gauge& g, int l, int nrhs, cd* x, const int* act) {
  Level& L = *g.levels[l];
  Work<double>& W = L.wd[c->wslot];
  const int64_t cnt = (int64_t)nrhs * L.n;
  W.cvt_out.ensure(sizeof(cf) * cnt);
  if (precond_writes_fp64(g, L)) {
    precond<float>(c, g, l, nrhs, W.cvt_in.as<cf>(), W.cvt_out.as<cf>(), act, x);
  } else {
    precond<float>(c, g, l, nrhs, W.cvt_in.as<cf>(), W.cvt_out.as<cf>(), act);
    launch_convert<double, float>(c->stream, W.cvt_out.as<cf>(), x, cnt);
  }
}

void precondition_d(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* r, cd* x, const int* act) {
  Level& L = *g.levels[l];
  if (precondition_in_fp32(g)) {
    Work<double>& W = L.wd[c->wslot];
    const int64_t cnt = (int64_t)nrhs * L.n;
    W.cvt_in.ensure(sizeof(cf) * cnt);
    if (fine_blocked(g, L))
      launch_convert_blk(c->stream, r, W.cvt_in.as<cf>(), L.Nx, L.Nt, nrhs);
    else
      launch_convert<float, double>(c->stream, r, W.cvt_in.as<cf>(), cnt);
    precondition_f32in(c, g, l, nrhs, x, act);
  } else {
    precond<double>(c, g, l, nrhs, r, x, act);
  }
}

// A fixed sequence of launches with no host synchronisation (a preconditioner
// application, an Arnoldi step) is replayed as a HIP graph.  A key is first
// run directly, which performs any buffer allocation; the second time, if no
// allocation happened since (same epoch), it is captured, instantiated and
// launched; later calls launch the graph.  Any reallocation anywhere
// invalidates the graph (its kernel arguments hold buffer addresses).
template <class F>
void run_graph(mgm_ctx* c, Gauge& g, const GraphKey& key, F&& body) {
  hipStream_t s = c->stream;
  if (!g.prm.graphs || !s) {
    body();
    return;
  }
  auto& graphs = g.graphs[c->wslot];
  auto it = graphs.find(key);
  const uint64_t ep = g_alloc_epoch.load();
  if (it != graphs.end() && it->second.exec && it->second.epoch == ep) {
    HIPCHK(hipGraphLaunch(it->second.exec, s));
    return;
  }
  if (it == graphs.end() || it->second.failed || it->second.epoch != ep) {
    if (it != graphs.end() && it->second.exec) {
      (void)hipGraphExecDestroy(it->second.exec);
      it->second.exec = nullptr;
    }
    const bool failed = it != graphs.end() && it->second.failed;
    body();
    GraphEntry& e = graphs[key];
    e.epoch = g_alloc_epoch.load();
    e.failed = failed;
    return;
  }
  // second run at an unchanged epoch: capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    it->second.failed = true;
    body();
    return;
  }
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIPCHK(hipStreamEndCapture(s, &graph));
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess || g_alloc_epoch.load() != ep) {
    // a failed instantiation is final; a buffer reallocated meanwhile (by
    // another host thread) only means the next call runs directly again
    (void)hipGetLastError();
    if (exec) (void)hipGraphExecDestroy(exec);
    it->second.failed = ie != hipSuccess;
    it->second.epoch = ~0ull;
    body();
    return;
  }
  it->second.exec = exec;
  HIPCHK(hipGraphLaunch(exec, s));
}

void precondition_graph(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* r, cd* x, const int* act) {
  const GraphKey key{l, nrhs, (const void*)r, (void*)x, act, g.prm.precision};
  run_graph(c, g, key, [&] { precondition_d(c, g, l, nrhs, r, x, act); });
}

// Outer FGMRES(m) in FP64.  Per RHS: stop on ||b - D x|| <= tol ||b|| (true
// residual, checked at the end of every cycle).  Inside a cycle the host reads
// the active flags of step j - 1 (written to pinned memory by that step's last
// kernel) while step j is already queued, and ends the cycle once every RHS
// has converged (the extra step is a no-op: every kernel of a step skips
// inactive RHS).
int solve_level(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* b, cd* x,
                const mgm_solve_params& sp, int* iters_out, double* relres_out) {
  hipStream_t s = c->stream;
  Level& L = *g.levels[l];
  const int64_t n = L.n;
  const int m = sp.restart;
  require(m >= 1 && m <= 63, "restart length must be in [1, 63]");
  require(sp.tol > 0, "tolerance must be positive");
  ensure_work<double>(L, c->wslot, nrhs, m);
  Work<double>& W = L.wd[c->wslot];
  W.flags.ensure(nrhs);
  cd* V = W.V.as<cd>();
  cd* Z = W.Z.as<cd>();
  cd* w = W.w.as<cd>();
  int* act = W.act.as<int>();
  int* done = act + nrhs;
  double* bnorm = W.bnorm.as<double>();
  double* beta = W.beta.as<double>();
  std::vector<int> hdone(nrhs, 0), hnit(nrhs), its(nrhs, 0);
  std::vector<double> hb(nrhs), hr(nrhs);
  bool have_hb = false;
  auto read_hb = [&] {  // ||b|| per RHS, fetched with the first residual read-back
    if (have_hb) return;
    have_hb = true;
    for (int r = 0; r < nrhs; ++r) {
      if (!std::isfinite(hb[r])) throw Error(MGM_ENONFINITE, "non-finite right-hand side");
      hdone[r] = hb[r] == 0.0;
    }
  };

  W.rb.ensure(nrhs);
  require(sp.use_cnn >= 0 && sp.use_cnn <= (MGM_CNN_GUESS | MGM_CNN_STAGE), "use_cnn: unknown flags");
  const bool learned = l == 0 && !L.has_dense;
  const bool stage = learned && (sp.use_cnn & MGM_CNN_STAGE);
  if (stage) require(c->cnn && c->cnn->ready, "no network parameters set (mgm_cnn_set_params)", MGM_ESTATE);
  const bool guess = learned && (sp.use_cnn & MGM_CNN_GUESS);
  // from x = 0 the first cycle starts from r0 = b and ||r0|| = ||b||
  // exactly: ||b|| and that start come from one launch in the loop below
  const bool zero_start = !L.has_dense && !guess && sp.max_restarts >= 0;
  // ||b||; zero right-hand sides are solved
  if (!zero_start) launch_norm<double>(s, b, n, nrhs, bnorm, nullptr, (double*)W.part.p, done);
  if (guess)
    cnn_initial_guess(c, g, nrhs, b, x, w);
  else if (!L.has_dense && sp.max_restarts < 0)
    launch_axpby<double>(s, 0.0, b, 0.0, nullptr, x, n, nrhs, nullptr);
  // otherwise x = 0 is never stored: the dense apply or the first cycle's
  // update writes x without reading it
  // read the residual norms, ||b|| and the iteration counts the reduce kernel
  // stored in pinned memory (the stream is synchronised)
  auto take_rb = [&] {
    const double* h = W.rb.h;
    for (int r = 0; r < nrhs; ++r) {
      hr[r] = h[r];
      hb[r] = h[nrhs + r];
      hnit[r] = W.rb.nit()[r];
    }
  };

  bool final_known = false;  // hr holds the residuals of the returned x
  // steps whose preconditioner takes an FP32 input: each step's last launch
  // also scales and rounds v_{j+1} for the next one
  const bool fused = !stage && precondition_in_fp32(g);
  if (L.has_dense) {
    launch_dense_apply<double>(s, L.d.dinv.as<cd>(), n, nrhs, b, x, nullptr, &g.scratch[c->wslot]);
  } else {
    for (int cycle = 0; cycle <= sp.max_restarts; ++cycle) {
      // r0 = b - D x ; v0 = r0 / ||r0||
      // from x = 0 with an FP32-input preconditioner the start also rounds v_0
      // for it, and step 0 hands the preconditioner that copy
      const bool cvt0 = cycle == 0 && zero_start && fused;
      if (cycle == 0 && zero_start) {
        if (cvt0) W.cvt_in.ensure(sizeof(cf) * (size_t)nrhs * n);
        launch_fgmres_start(s, b, n, nrhs, (double*)W.part.p, m, sp.tol, bnorm, done, act, W.nit.as<int>(),
                            W.g.as<cd>(), W.thr.as<double>(), V, cvt0 ? W.cvt_in.as<cf>() : nullptr,
                            fine_blocked(g, L) ? L.Nx : 0);
      } else {
        apply_op<double>(c, g, l, nrhs, x, w, b, nullptr);
        launch_norm<double>(s, w, n, nrhs, beta, nullptr, (double*)W.part.p);
        launch_fgmres_init<double>(s, nrhs, beta, nullptr, done, sp.tol, bnorm, m, act,
                                   W.nit.as<int>(), W.g.as<cd>(), W.thr.as<double>());
        launch_scale<double>(s, w, beta, n, nrhs, V, act);
      }
      for (int j = 0; j < m; ++j) {
        // the whole step is one graph: key level field (m + 1) * 1000 + l
        // (+ 500 with the learned stage) tells it from the preconditioner's
        // own graphs, from other restart lengths and from the plain step;
        // the step index is in the V / Z addresses
        const int64_t vs = (int64_t)nrhs * n;
        const GraphKey key{(m + 1) * 1000 + l + (stage ? 500 : 0) + (cvt0 && j == 0 ? 250 : 0), nrhs,
                           (const void*)(V + j * vs),
                           (void*)(Z + j * vs), act, g.prm.precision};
        // the step's last kernel writes the active flags into pinned host
        // slot j % kDepth (no copy); the event marks the step's end
        const int slot = j % PinnedFlags::kDepth;
        run_graph(c, g, key, [&] {
          arnoldi_step<double>(
              c, g, l, nrhs, j, m, W,
              [&](const cd* v, cd* z, const int* a) {
                if (stage) cnn_precondition(c, g, nrhs, v, z, a);
                else if (v) precondition_d(c, g, l, nrhs, v, z, a);
                else precondition_f32in(c, g, l, nrhs, z, a);
              },
              W.flags.h + slot * nrhs, fused, cvt0 && j == 0);
        });
        HIPCHK(hipEventRecord(W.flags.ev[slot], s));
        if (j + 1 < PinnedFlags::kDepth) continue;
        const int prev = (j + 1) % PinnedFlags::kDepth;  // step j - (kDepth - 1)
        HIPCHK(hipEventSynchronize(W.flags.ev[prev]));
        const int* f = W.flags.h + prev * nrhs;
        if (std::all_of(f, f + nrhs, [](int a) { return a == 0; })) break;
        // every RHS still running is within reach of its threshold: wait for
        // step j itself rather than queue a step that would likely be a no-op
        if (std::all_of(f, f + nrhs, [](int a) { return a != 1; })) {
          HIPCHK(hipEventSynchronize(W.flags.ev[slot]));
          const int* fj = W.flags.h + slot * nrhs;
          if (std::all_of(fj, fj + nrhs, [](int a) { return a == 0; })) break;
        }
      }
      // x += Z y (from x = 0: x = Z y), y = R^{-1} g solved by the update's workgroups
      launch_update_backsolve<double>(s, Z, (int64_t)nrhs * n, n, m, W.H.as<cd>(), W.g.as<cd>(), W.nit.as<int>(),
                                      x, nrhs, cycle == 0 && zero_start);
      // true residual
      apply_op<double>(c, g, l, nrhs, x, w, b, nullptr);
      launch_norm_readback(s, w, n, nrhs, beta, (double*)W.part.p, bnorm, W.nit.as<int>(), W.rb.h,
                           W.rb.nit());
      HIPCHK(hipStreamSynchronize(s));
      take_rb();
      read_hb();
      bool all = true;
      for (int r = 0; r < nrhs; ++r) {
        if (hdone[r]) continue;
        its[r] += hnit[r];
        if (!std::isfinite(hr[r])) throw Error(MGM_ENONFINITE, "non-finite residual in FGMRES");
        if (hr[r] <= sp.tol * hb[r]) hdone[r] = 1;
        else all = false;
      }
      if (all) {
        final_known = true;
        break;
      }
      HIPCHK(hipMemcpyAsync(done, hdone.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
    }
  }
  if (!final_known) {
    apply_op<double>(c, g, l, nrhs, x, w, b, nullptr);
    launch_norm_readback(s, w, n, nrhs, beta, (double*)W.part.p, bnorm, W.nit.as<int>(), W.rb.h, W.rb.nit());
    HIPCHK(hipStreamSynchronize(s));
    take_rb();
    read_hb();
  }
  bool ok = true;
  for (int r = 0; r < nrhs; ++r) {
    const double rel = hb[r] > 0 ? hr[r] / hb[r] : 0.0;
    if (!std::isfinite(rel)) throw Error(MGM_ENONFINITE, "non-finite residual");
    if (rel > sp.tol) ok = false;
    if (iters_out) iters_out[r] = its[r];
    if (relres_out) relres_out[r] = rel;
  }
  return ok ? MGM_OK : MGM_ENOTCONV;
}

// Q = qr+(Y): shifted CholQR followed by two plain CholQR passes.  The
// product of the three triangular factors has a positive diagonal, so Q is
// the unique thin-QR factor with positive real diag(R).  Workspace: tmp
// [d][n], G [d][d], part [gram_partials(n)][d][d], fail (one int).
void orthonormalize_launch(hipStream_t s, int64_t n, int d, const cd* Y, cd* Q, cd* tmp, cd* G, cd* part,
                           int* fail) {
  require(d >= 1 && d <= 64 && n >= d, "orthonormalize: need 1 <= d <= 64 and n >= d");
  require(Y != Q, "orthonormalize: Y and Q must not overlap");
  launch_fill_int(s, fail, 1, 0);
  // pass 0: Y -> Q (shifted Gram), pass 1: Q -> tmp, pass 2: tmp -> Q
  const double shifts[3] = {1e-14, 0.0, 0.0};
  const cd* srcs[3] = {Y, Q, tmp};
  cd* dsts[3] = {Q, tmp, Q};
  for (int pass = 0; pass < 3; ++pass) {
    const cd* src = srcs[pass];
    cd* dst = dsts[pass];
    launch_gram(s, src, n, d, G, part);
    launch_cholesky_rinv(s, G, d, shifts[pass], fail);
    launch_right_tri(s, src, G, n, d, dst);
  }
}

void orthonormalize_ws(hipStream_t s, int64_t n, int d, const cd* Y, cd* Q, cd* tmp, cd* G, cd* part,
                       int* fail) {
  orthonormalize_launch(s, n, d, Y, Q, tmp, G, part, fail);
  int hfail = 0;
  HIPCHK(hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hfail) throw Error(MGM_ENONFINITE, "CholQR: Gram matrix not positive definite (rank-deficient block)");
}

void orthonormalize(mgm_ctx* c, int64_t n, int d, const cd* Y, cd* Q) {
  require(d >= 1 && d <= 64 && n >= d, "orthonormalize: need 1 <= d <= 64 and n >= d");
  c->qr_tmp.ensure(sizeof(cd) * (size_t)d * n);
  c->qr_G.ensure(sizeof(cd) * d * d);
  c->qr_part.ensure(sizeof(cd) * (size_t)d * d * gram_partials(n));
  c->qr_fail.ensure(sizeof(int));
  orthonormalize_ws(c->stream, n, d, Y, Q, c->qr_tmp.as<cd>(), c->qr_G.as<cd>(), c->qr_part.as<cd>(),
                    c->qr_fail.as<int>());
}

// ------------------------------------------------------------------ setup
namespace {

void build_sap(mgm_ctx* c, Level& L, int sbx, int sbt) {
  hipStream_t s = c->stream;
  require(sbx >= 1 && sbt >= 1 && L.Nx % sbx == 0 && L.Nt % sbt == 0,
          "SAP block must divide the level's lattice");
  const int NBx = L.Nx / sbx, NBt = L.Nt / sbt;
  require((NBx == 1 || NBx % 2 == 0) && (NBt == 1 || NBt % 2 == 0),
          "SAP needs an even number of blocks (or one) per direction");
  L.sbx = sbx;
  L.sbt = sbt;
  L.K = sbx * sbt * L.M;
  // 2x2 sites of 16 dofs (K = 64) run in premultiplied form, whose eight
  // outward hops must leave the block: at least two blocks per direction
  const bool quad = L.M == 16 && sbx == 2 && sbt == 2;
  require(L.K <= 32 || quad, "SAP block too large: sbx*sbt*dofs must be <= 32 (or 2x2 sites of 16 dofs)");
  require(!quad || (NBx >= 2 && NBt >= 2), "2x2 SAP blocks need at least two blocks per direction");
  L.nblk = NBx * NBt;
  L.d.sapinv.ensure(sizeof(cd) * (size_t)L.nblk * L.K * L.K);
  launch_sap_extract(s, L.d.B(), L.Nx, L.Nt, L.M, sbx, sbt, L.d.sapinv.as<cd>());
  DevBuf fail;
  fail.ensure(sizeof(int));
  HIPCHK(hipMemsetAsync(fail.p, 0, sizeof(int), s));
  launch_small_inverse(s, L.d.sapinv.as<cd>(), L.K, L.nblk, fail.as<int>());
  int hf = 0;
  HIPCHK(hipMemcpyAsync(&hf, fail.p, sizeof(int), hipMemcpyDeviceToHost, s));
  std::vector<int> lists[2];
  for (int b = 0; b < L.nblk; ++b) lists[((b % NBx) + (b / NBx)) % 2].push_back(b);
  for (int col = 0; col < 2; ++col) {
    L.ncolor[col] = (int)lists[col].size();
    L.color_list[col].ensure(sizeof(int) * std::max<size_t>(1, lists[col].size()));
    if (!lists[col].empty())
      HIPCHK(hipMemcpyAsync(L.color_list[col].p, lists[col].data(), sizeof(int) * lists[col].size(),
                            hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  require(!hf, "singular SAP block", MGM_ENONFINITE);
  if (quad) {  // M_B = inv_B D_BH of the premultiplied sweeps (the setup's own solves use it)
    L.d.sapM.ensure(sizeof(cd) * (size_t)L.nblk * 8 * 64 * 16);
    launch_sap4_premul(s, L.d.blocks.as<cd>(), L.d.sapinv.as<cd>(), L.Nx, L.nblk, L.d.sapM.as<cd>());
    HIPCHK(hipStreamSynchronize(s));
  }
}

template <class TO>
void copy_convert(mgm_ctx* c, const DevBuf& src, DevBuf& dst) {
  if (!src.p) return;
  const int64_t cnt = (int64_t)(src.bytes / sizeof(cd));
  dst.ensure(sizeof(cx<TO>) * cnt);
  launch_convert<TO, double>(c->stream, src.as<cd>(), dst.as<cx<TO>>(), cnt);
}

}  // namespace

void setup_hierarchy(mgm_ctx* c, Gauge& g, const mgm_mg_params& p) {
  hipStream_t s = c->stream;
  const int Lv = p.nlevels;
  require(Lv >= 1 && Lv <= MGM_MAX_LEVELS, "nlevels out of range");
  require(p.precision == MGM_PREC_FP64 || p.precision == MGM_PREC_FP32 || p.precision == MGM_PREC_FP16,
          "unknown precision");
  g.prm = p;
  g.mg_ready = false;
  g.levels.clear();
  auto L0 = std::make_unique<Level>();
  L0->Nx = g.Lx;
  L0->Nt = g.Lt;
  L0->M = 2;
  L0->sites = (int64_t)g.Lx * g.Lt;
  L0->n = 2 * L0->sites;
  L0->d.blocks.ensure(sizeof(cd) * (size_t)L0->sites * 20);
  launch_fine_blocks(s, g.links.as<cd>(), g.m0 + 2.0, g.Lx, g.Lt, L0->d.blocks.as<cd>());
  g.levels.push_back(std::move(L0));

  const int T = p.mlmc_levels > 0 ? p.mlmc_levels - 1 : Lv - 1;
  require(T >= 0 && T < Lv, "mlmc_levels must be in [0, nlevels]");
  g.mlmc_levels = T + 1;
  // dense inverse of level l; its trace closes the MLMC sum when l == T
  auto densify = [&](Level& L, int l) {
    require(L.n <= 20000, "level too large for the dense inverse (n > 20000)");
    DevBuf work;
    work.ensure(sizeof(cd) * (size_t)L.n * L.n);
    L.d.dinv.ensure(sizeof(cd) * (size_t)L.n * L.n);
    launch_dense_from_stencil(s, L.d.B(), L.Nx, L.Nt, L.M, work.as<cd>());
    if (dense_inverse(s, work.as<cd>(), L.n, L.d.dinv.as<cd>()))
      throw Error(MGM_ENONFINITE, "operator of level " + std::to_string(l) + " is singular");
    L.has_dense = true;
    if (l == T) {
      DevBuf tr;
      tr.ensure(sizeof(cd));
      launch_diag_sum(s, L.d.dinv.as<cd>(), L.n, tr.as<cd>());
      cd h;
      HIPCHK(hipMemcpyAsync(&h, tr.p, sizeof(cd), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      g.trL[0] = h.re;
      g.trL[1] = h.im;
    }
  };

  for (int l = 0; l < Lv; ++l) {
    Level& L = *g.levels[l];
    L.is_coarsest = (l == Lv - 1);
    if (L.is_coarsest) {
      densify(L, l);
      break;
    }
    if (l == T) densify(L, l);
    const int bx = p.block[l][0], bt = p.block[l][1], ntv = p.ntv[l];
    require(bx >= 1 && bt >= 1 && L.Nx % bx == 0 && L.Nt % bt == 0,
            "aggregate block must divide the level's lattice");
    require(ntv >= 1 && ntv <= 16, "ntv must be in [1, 16]");
    const int Mc = 2 * ntv;
    require(Mc == 2 || Mc == 4 || Mc == 8 || Mc == 16 || Mc == 32, "2*ntv must be 2, 4, 8, 16 or 32");
    L.sap_cycles = std::max(1, p.sap_cycles[l]);
    L.inner_iters = p.inner_iters[l];
    build_sap(c, L, std::max(1, p.sap_block[l][0]), std::max(1, p.sap_block[l][1]));

    // test vectors: block inverse iteration from Z2xZ2 noise
    DevBuf Vb, Wb;
    Vb.ensure(sizeof(cd) * (size_t)ntv * L.n);
    Wb.ensure(sizeof(cd) * (size_t)ntv * L.n);
    launch_noise<double>(s, Vb.as<cd>(), L.n, ntv, MGM_NOISE_Z2Z2, p.seed, MGM_PURPOSE_SETUP, l, 0);
    mgm_solve_params sp{p.setup_tol, p.setup_restart, p.setup_max_restarts, 0};
    for (int it = 0; it < p.setup_iters; ++it) {
      const int st = solve_level(c, g, l, ntv, Vb.as<cd>(), Wb.as<cd>(), sp, nullptr, nullptr);
      if (st != MGM_OK) throw Error(st, "setup solve did not converge on level " + std::to_string(l));
      orthonormalize(c, L.n, ntv, Wb.as<cd>(), Vb.as<cd>());
    }
    L.bx = bx;
    L.bt = bt;
    L.ntv = ntv;
    L.d.P.ensure(sizeof(cd) * (size_t)L.nagg() * 2 * L.nrow() * ntv);
    launch_local_qr(s, Vb.as<cd>(), L.n, L.Nx, L.Nt, L.M, bx, bt, ntv, L.d.P.as<cd>());

    auto C = std::make_unique<Level>();
    C->Nx = L.Nx / bx;
    C->Nt = L.Nt / bt;
    C->M = Mc;
    C->sites = (int64_t)C->Nx * C->Nt;
    C->n = C->sites * Mc;
    C->d.blocks.ensure(sizeof(cd) * (size_t)C->sites * 5 * Mc * Mc);
    launch_galerkin(s, L.d.B(), L.Nx, L.Nt, L.M, L.d.P.as<cd>(), bx, bt, ntv, C->d.blocks.as<cd>());
    HIPCHK(hipStreamSynchronize(s));
    L.has_coarse = true;
    g.levels.push_back(std::move(C));
  }
  // FP32 copies for the mixed-precision preconditioner
  for (auto& Lp : g.levels) {
    Level& L = *Lp;
    copy_convert<float>(c, L.d.blocks, L.f.blocks);
    copy_convert<float>(c, L.d.P, L.f.P);
    copy_convert<float>(c, L.d.sapinv, L.f.sapinv);
    copy_convert<float>(c, L.d.dinv, L.f.dinv);
    if (L.is_coarsest && L.d.dinv.p && L.n % 256 == 0) {
      // FP16 copy of the coarsest inverse: the FP16 cycle's coarse solve (kept
      // only if every entry is in range)
      const int64_t cnt = L.n * L.n;
      DevBuf ovf;
      ovf.ensure(sizeof(int));
      launch_fill_int(s, ovf.as<int>(), 1, 0);
      L.f.hdinv.ensure(sizeof(chalf) * cnt);
      launch_to_half_checked(s, L.d.dinv.as<cd>(), L.f.hdinv.as<chalf>(), cnt, ovf.as<int>());
      int h = 0;
      HIPCHK(hipMemcpyAsync(&h, ovf.p, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (h) L.f.hdinv.release();
    }
    copy_convert<float>(c, L.d.sapM, L.f.sapM);
    if (L.M == 16 && L.d.sapinv.p) {  // FP16 blocks for the FP16 mode
      const int64_t nbk = (int64_t)(L.d.blocks.bytes / sizeof(cd));
      const int64_t nin = (int64_t)(L.d.sapinv.bytes / sizeof(cd));
      L.f.hblocks.ensure(sizeof(chalf) * nbk);
      L.f.hsapinv.ensure(sizeof(chalf) * nin);
      launch_to_half(s, L.d.blocks.as<cd>(), L.f.hblocks.as<chalf>(), nbk);
      launch_to_half(s, L.d.sapinv.as<cd>(), L.f.hsapinv.as<chalf>(), nin);
      if (L.sbx == 2 && L.sbt == 1 && L.nblk > 0) {
        L.f.hsapM.ensure(sizeof(chalf) * (size_t)L.nblk * 6 * 32 * 16);  // 16 dofs per site
        launch_sap2_premul(s, L.d.blocks.as<cd>(), L.d.sapinv.as<cd>(), L.Nx, L.nblk, L.f.hsapM.as<chalf>());
      }
      if (L.sbx == 2 && L.sbt == 2 && L.d.sapM.p) {
        const int64_t nm = (int64_t)(L.d.sapM.bytes / sizeof(cd));
        L.f.hsapM.ensure(sizeof(chalf) * nm);
        launch_to_half(s, L.d.sapM.as<cd>(), L.f.hsapM.as<chalf>(), nm);
      }
      if (L.has_coarse && L.bx == 2 && L.bt == 2 && L.ntv == 8 && L.d.P.p) {
        const int64_t np = (int64_t)(L.d.P.bytes / sizeof(cd));  // [nagg][2][32][8]
        L.f.hP.ensure(sizeof(chalf) * np);
        launch_to_half(s, L.d.P.as<cd>(), L.f.hP.as<chalf>(), np);
      }
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  g.mg_ready = true;
}

}  // namespace mgm
