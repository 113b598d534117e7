// C ABI of the library (declared in include/mgmlmc.h).  Each entry point
// validates its arguments, runs on the context's stream and converts internal
// errors into status codes; nothing here aborts the process.
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>

#include "internal.h"

using namespace mgm;

namespace mgm {

std::atomic<uint64_t> g_alloc_epoch{0};

// Solve in chunks of sp.rhs_block right-hand sides (all at once when 0; the
// autotuned width of the level when -1).
int solve_chunked(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* b, cd* x,
                  const mgm_solve_params& sp, int* iters, double* relres) {
  int want = sp.rhs_block;
  if (want < 0) want = g.tuned_block[l];
  const int blk = (want > 0 && want < nrhs) ? want : nrhs;
  const int64_t n = g.levels[l]->n;
  int status = MGM_OK;
  for (int r0 = 0; r0 < nrhs; r0 += blk) {
    const int k = std::min(blk, nrhs - r0);
    const int st = solve_level(c, g, l, k, b + (int64_t)r0 * n, x + (int64_t)r0 * n, sp,
                               iters ? iters + r0 : nullptr, relres ? relres + r0 : nullptr);
    if (st != MGM_OK) status = st;
  }
  return status;
}

}  // namespace mgm

namespace {

// ---------------------------------------------------------------- no-allocation workspace
// Device memory of mgm_orthonormalize_noalloc: the CholQR workspace of a
// d x n block with n d <= kNoAllocND -- the temporary Q (n d), the Gram
// partials (ceil(n / 128) d^2 <= n d 64 / 128 + 64^2 for d <= 64), the Gram
// matrix / R^{-1} (64^2) and the failure flag -- in one static array
// that every device holds from the library's load until the process ends.
// Host code never uses the array's name as an address: its per-device
// address comes from hipGetSymbolAddress (resolved by mgm_create with the
// device current) and only that address reaches kernels.
constexpr int64_t kNoAllocND = int64_t(1) << 20;                  // complex elements of Q
constexpr int64_t kNoAllocPart = kNoAllocND / 128 * 64 + 64 * 64;  // Gram partials
constexpr int64_t kNoAllocG = 64 * 64;
constexpr int64_t kNoAllocCx = kNoAllocND + kNoAllocPart + kNoAllocG + 16;  // + the flag
__device__ __align__(256) cd scratch[kNoAllocCx];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
cd* g_scratch_ptr[kMaxDevices] = {nullptr};

// the array's address on `device` (must be the current device); once per device
cd* resolve_scratch(int device) {
  require(device >= 0 && device < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, "no device address for the no-allocation workspace", MGM_EHIP);
    g_scratch_ptr[device] = static_cast<cd*>(ptr);
  }
  return g_scratch_ptr[device];
}

cd* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  require(device >= 0 && device < kMaxDevices && g_scratch_ptr[device],
          "no-allocation workspace not resolved on this device", MGM_ESTATE);
  return g_scratch_ptr[device];
}

template <class F>
int guarded(mgm_ctx* c, F&& f) {
  if (!c) return MGM_EINVAL;
  try {
    HIPCHK(hipSetDevice(c->device));
    const int st = f();
    if (st == MGM_OK) c->err.clear();
    return st;
  } catch (const Error& e) {
    c->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return MGM_EHIP;
  }
}

Gauge& gauge_of(mgm_ctx* c, int id) {
  require(id >= 0 && id < (int)c->gauges.size() && c->gauges[id], "unknown gauge id");
  return *c->gauges[id];
}

Cnn& cnn_of(mgm_ctx* c) {
  require(c->cnn && c->cnn->ready, "no network parameters set (mgm_cnn_set_params)", MGM_ESTATE);
  return *c->cnn;
}

// Distinct sites outside the colour-0 SAP blocks that neighbour one of them:
// the x values one colour sweep must read (each once).
int64_t sap_halo_sites(const Level& L) {
  const int NBx = L.Nx / L.sbx;
  std::vector<int> blocks(L.ncolor[0]);
  HIPCHK(hipMemcpy(blocks.data(), L.color_list[0].p, sizeof(int) * blocks.size(), hipMemcpyDeviceToHost));
  std::vector<char> in(L.sites, 0), mark(L.sites, 0);
  auto site = [&](int x, int t) { return (int64_t)((t + L.Nt) % L.Nt) * L.Nx + (x + L.Nx) % L.Nx; };
  for (int b : blocks)
    for (int st = 0; st < L.sbt; ++st)
      for (int sx = 0; sx < L.sbx; ++sx) in[site((b % NBx) * L.sbx + sx, (b / NBx) * L.sbt + st)] = 1;
  int64_t cnt = 0;
  for (int b : blocks)
    for (int st = 0; st < L.sbt; ++st)
      for (int sx = 0; sx < L.sbx; ++sx) {
        const int x = (b % NBx) * L.sbx + sx, t = (b / NBx) * L.sbt + st;
        const int64_t nb[4] = {site(x + 1, t), site(x - 1, t), site(x, t + 1), site(x, t - 1)};
        for (int64_t v : nb)
          if (!in[v] && !mark[v]) {
            mark[v] = 1;
            ++cnt;
          }
      }
  return cnt;
}

Level& level_of(Gauge& g, int level) {
  require(level >= 0 && level < (int)g.levels.size(),
          "level out of range (call setup_mg for coarse levels)");
  return *g.levels[level];
}

// Runs a call's work on the field's stream, ordered after everything already
// enqueued on the caller's stream and before anything enqueued there later.
struct OnGauge {
  mgm_ctx* c;
  Gauge& g;
  hipStream_t saved;
  OnGauge(mgm_ctx* c_, Gauge& g_) : c(c_), g(g_), saved(c_->stream) {
    HIPCHK(hipEventRecord(g.ev_in, saved));
    HIPCHK(hipStreamWaitEvent(g.stream, g.ev_in, 0));
    c->stream = g.stream;
  }
  ~OnGauge() {
    c->stream = saved;
    (void)hipEventRecord(g.ev_out, g.stream);
    (void)hipStreamWaitEvent(saved, g.ev_out, 0);
  }
};

}  // namespace

extern "C" {

int mgm_create(mgm_ctx** out, int device, void* stream) {
  if (!out) return MGM_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MGM_EHIP;
  if (hipSetDevice(device) != hipSuccess) return MGM_EHIP;
  try {
    resolve_scratch(device);
  } catch (const Error& e) {
    return e.code;
  }
  mgm_ctx* c = new mgm_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  *out = c;
  return MGM_OK;
}

void mgm_destroy(mgm_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* mgm_last_error(const mgm_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mgm_set_gauge(mgm_ctx* c, int Lx, int Lt, const void* links, double m0, int bc_t_anti,
                  int* gauge_id) {
  return guarded(c, [&] {
    require(links && gauge_id, "null pointer");
    require(Lx >= 2 && Lt >= 2 && Lx % 2 == 0 && Lt % 2 == 0, "Lx and Lt must be even and >= 2");
    require((int64_t)Lx * Lt <= (int64_t)1 << 30, "lattice too large (more than 2^30 sites)");
    auto g = std::make_unique<Gauge>();
    g->Lx = Lx;
    g->Lt = Lt;
    g->m0 = m0;
    g->anti = bc_t_anti ? 1 : 0;
    const int64_t cnt = 2 * (int64_t)Lx * Lt;
    g->links.ensure(sizeof(cd) * cnt);
    HIPCHK(hipMemcpyAsync(g->links.p, links, sizeof(cd) * cnt, hipMemcpyDeviceToDevice, c->stream));
    if (g->anti) launch_fold_anti(c->stream, g->links.as<cd>(), Lx, Lt);
    g->links32.ensure(sizeof(cf) * cnt);
    launch_convert<float, double>(c->stream, g->links.as<cd>(), g->links32.as<cf>(), cnt);
    // level 0 exists before any multigrid setup
    auto L0 = std::make_unique<Level>();
    L0->Nx = Lx;
    L0->Nt = Lt;
    L0->M = 2;
    L0->sites = (int64_t)Lx * Lt;
    L0->n = 2 * L0->sites;
    g->levels.push_back(std::move(L0));
    HIPCHK(hipStreamSynchronize(c->stream));
    // the field's own stream (default priority) and its ordering events
    HIPCHK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming));
    c->gauges.push_back(std::move(g));
    *gauge_id = (int)c->gauges.size() - 1;
    return MGM_OK;
  });
}

int mgm_free_gauge(mgm_ctx* c, int gauge_id) {
  return guarded(c, [&] {
    (void)gauge_of(c, gauge_id);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->gauges[gauge_id].reset();  // waits for the field's stream, frees its memory
    return MGM_OK;
  });
}

int mgm_setup_mg(mgm_ctx* c, int gauge_id, const mgm_mg_params* prm) {
  return guarded(c, [&] {
    require(prm != nullptr, "null params");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    g.clear_graphs();
    setup_hierarchy(c, g, *prm);
    return MGM_OK;
  });
}

int mgm_set_precision(mgm_ctx* c, int gauge_id, int precision) {
  return guarded(c, [&] {
    require(precision == MGM_PREC_FP64 || precision == MGM_PREC_FP32 || precision == MGM_PREC_FP16,
            "unknown precision");
    Gauge& g = gauge_of(c, gauge_id);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    OnGauge og(c, g);
    HIPCHK(hipStreamSynchronize(c->stream));
    g.clear_graphs();
    g.prm.precision = precision;
    return MGM_OK;
  });
}

int mgm_level_info(mgm_ctx* c, int gauge_id, int level, int* info) {
  return guarded(c, [&] {
    require(info != nullptr, "null pointer");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    Level& L = level_of(g, level);
    info[0] = L.Nx;
    info[1] = L.Nt;
    info[2] = L.M;
    info[3] = (int)L.n;
    return MGM_OK;
  });
}

int mgm_apply_D(mgm_ctx* c, int gauge_id, int level, int nrhs, const void* x, void* y) {
  return guarded(c, [&] {
    require(x && y && nrhs > 0 && x != y, "bad vectors");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    level_of(g, level);
    require(level == 0 || g.mg_ready, "coarse operators need setup_mg", MGM_ESTATE);
    apply_level(c, g, level, nrhs, static_cast<const cd*>(x), static_cast<cd*>(y));
    return MGM_OK;
  });
}

int mgm_apply_P(mgm_ctx* c, int gauge_id, int level, int nrhs, const void* x, void* y) {
  return guarded(c, [&] {
    require(x && y && nrhs > 0, "bad vectors");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    Level& L = level_of(g, level);
    require(L.has_coarse, "level has no coarser level");
    launch_prolong<double>(c->stream, L.d.P.as<cd>(), L.Nx, L.Nt, L.M, L.bx, L.bt, L.ntv, nrhs,
                           static_cast<const cd*>(x), static_cast<cd*>(y), 0, nullptr);
    return MGM_OK;
  });
}

int mgm_apply_R(mgm_ctx* c, int gauge_id, int level, int nrhs, const void* x, void* y) {
  return guarded(c, [&] {
    require(x && y && nrhs > 0, "bad vectors");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    Level& L = level_of(g, level);
    require(L.has_coarse, "level has no coarser level");
    launch_restrict<double>(c->stream, L.d.P.as<cd>(), L.Nx, L.Nt, L.M, L.bx, L.bt, L.ntv, nrhs,
                            static_cast<const cd*>(x), static_cast<cd*>(y), nullptr);
    return MGM_OK;
  });
}

int mgm_precondition(mgm_ctx* c, int gauge_id, int level, int nrhs, const void* r, void* x) {
  return guarded(c, [&] {
    require(r && x && nrhs > 0 && r != x, "bad vectors");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    level_of(g, level);
    precondition_d(c, g, level, nrhs, static_cast<const cd*>(r), static_cast<cd*>(x), nullptr);
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

int mgm_get_prolongator(mgm_ctx* c, int gauge_id, int level, void* out) {
  return guarded(c, [&] {
    require(out != nullptr, "null pointer");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    Level& L = level_of(g, level);
    require(L.has_coarse, "level has no coarser level");
    HIPCHK(hipMemcpyAsync(out, L.d.P.p, sizeof(cd) * (size_t)L.nagg() * 2 * L.nrow() * L.ntv,
                          hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

int mgm_coarsest_trace(mgm_ctx* c, int gauge_id, double* out) {
  return guarded(c, [&] {
    require(out != nullptr, "null pointer");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    out[0] = g.trL[0];
    out[1] = g.trL[1];
    return MGM_OK;
  });
}

int mgm_solve_batch(mgm_ctx* c, int gauge_id, int level, int nrhs, const void* b, void* x,
                    const mgm_solve_params* prm, mgm_solve_stats* stats) {
  return guarded(c, [&] {
    require(b && x && prm && nrhs > 0 && b != x, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    level_of(g, level);
    return solve_chunked(c, g, level, nrhs, static_cast<const cd*>(b), static_cast<cd*>(x), *prm,
                         stats ? stats->iters : nullptr, stats ? stats->relres : nullptr);
  });
}

int mgm_noise(mgm_ctx* c, int kind, uint64_t seed, int purpose, int level, int64_t index0, int64_t n,
              int nrhs, void* out) {
  return guarded(c, [&] {
    require(out && n > 0 && nrhs > 0, "bad arguments");
    require(kind == MGM_NOISE_RADEMACHER || kind == MGM_NOISE_Z2Z2, "unknown noise kind");
    require(purpose >= 0 && purpose < 256 && level >= 0 && level < 256, "key field out of range");
    require(index0 >= 0 && index0 + nrhs <= (int64_t(1) << 48), "index out of range");
    launch_noise<double>(c->stream, static_cast<cd*>(out), n, nrhs, kind, seed, purpose, level, index0);
    return MGM_OK;
  });
}

int mgm_orthonormalize(mgm_ctx* c, int64_t n, int d, const void* Y, void* Q) {
  return guarded(c, [&] {
    require(Y && Q && Y != Q, "bad arguments");
    orthonormalize(c, n, d, static_cast<const cd*>(Y), static_cast<cd*>(Q));
    return MGM_OK;
  });
}

int mgm_orthonormalize_noalloc(mgm_ctx* c, int64_t n, int d, const void* Y, void* Q) {
  return guarded(c, [&] {
    require(Y && Q && Y != Q, "bad arguments");
    require(d >= 1 && d <= 64 && n >= d, "orthonormalize: need 1 <= d <= 64 and n >= d");
    require(n <= kNoAllocND / d, "orthonormalize_noalloc: n * d exceeds 2^20 complex elements");
    const int64_t np = gram_partials(n) * d * d;
    require(np <= kNoAllocPart, "orthonormalize_noalloc: Gram partials exceed the workspace");
    cd* base = scratch_of(c->device);
    cd* tmp = base;
    cd* part = base + kNoAllocND;
    cd* G = part + kNoAllocPart;
    int* fail = reinterpret_cast<int*>(G + kNoAllocG);
    orthonormalize_ws(c->stream, n, d, static_cast<const cd*>(Y), static_cast<cd*>(Q), tmp, G, part, fail);
    return MGM_OK;
  });
}

int mgm_time_kernel(mgm_ctx* c, int gauge_id, int kind, int level, int nrhs, int reps,
                    double* us_out, double* bytes_out, double* flops_out) {
  return guarded(c, [&] {
    require(us_out && bytes_out && flops_out && nrhs > 0 && reps > 0, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    Level& L = level_of(g, level);
    hipStream_t s = c->stream;
    const int64_t n = L.n;
    const double b = nrhs;
    c->scratch2.ensure(sizeof(cd) * (size_t)nrhs * n * 3);
    cd* x = c->scratch2.as<cd>();
    cd* y = x + (int64_t)nrhs * n;
    cd* r = y + (int64_t)nrhs * n;
    launch_noise<double>(s, x, n, nrhs, MGM_NOISE_Z2Z2, 11, 0, 0, 0);
    launch_noise<double>(s, r, n, nrhs, MGM_NOISE_Z2Z2, 12, 0, 0, 0);
    HIPCHK(hipMemcpyAsync(y, x, sizeof(cd) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, s));
    std::function<void()> launch;
    double bytes = 0, flops = 0;
    DevBuf lowbuf;  // FP32 copies of the vectors for the low-precision kinds
    switch (kind) {
      case MGM_KERNEL_STENCIL:
        // every lambda captures pointers and sizes by value: some of them
        // are block-scoped and gone by the time launch() runs
        launch = [=, &g] { apply_level(c, g, level, nrhs, x, y); };
        if (level == 0) {
          bytes = (double)L.sites * (64.0 * b + 32.0);
          flops = (double)L.sites * b * 8.0 * 2.0 * 9.0;
        } else {
          bytes = 32.0 * n * b + 16.0 * L.sites * 5.0 * L.M * L.M;
          flops = 8.0 * L.sites * 5.0 * L.M * L.M * b;
        }
        break;
      case MGM_KERNEL_SAP: {
        require(g.mg_ready && L.ncolor[0] > 0, "SAP needs setup_mg on this level", MGM_ESTATE);
        const bool quad = L.d.sapM.p != nullptr;  // premultiplied 2x2 blocks (r stands in for rho)
        if (quad) {
          launch = [=, &L] {
            launch_sap4p<double>(s, L.d.sapM.as<cd>(), L.d.sapinv.as<cd>(), L.Nx, L.Nt, L.color_list[0].as<int>(),
                                 L.ncolor[0], nrhs, false, nullptr, const_cast<cd*>(r), y, nullptr);
          };
        } else {
          launch = [=, &L] {
            launch_sap_sweep<double>(s, L.d.B(), L.d.sapinv.as<cd>(), L.Nx, L.Nt, L.M, L.sbx, L.sbt,
                                     L.color_list[0].as<int>(), L.ncolor[0], nrhs, r, y, nullptr);
          };
        }
        // with the exact block inverse a sweep is x_B = inv_B (r_B - D_BH x_H):
        // r_B and the distinct halo values read, x_B written, inv_B and the
        // outward hops read (each once); premultiplied: rho_B, the halo and
        // M_B read, x_B written
        const double nb = L.ncolor[0];
        const double halo = 2.0 * (L.sbx + L.sbt) * L.M;  // outward hop dofs per block
        const double hx = (double)sap_halo_sites(L) * L.M;
        const double ment = quad ? (double)L.K * halo : (double)L.K * L.K + halo * L.M;
        bytes = 16.0 * b * (2.0 * nb * L.K + hx) + 16.0 * nb * ment;
        flops = 8.0 * b * nb * ment;
        break;
      }
      case MGM_KERNEL_DENSE_LOW: {
        require(g.mg_ready && L.is_coarsest && L.f.dinv.p, "level is not the coarsest of a built hierarchy",
                MGM_ESTATE);
        require(g.prm.precision != MGM_PREC_FP64, "the preconditioner runs in FP64 (mgm_set_precision)",
                MGM_ESTATE);
        lowbuf.ensure(sizeof(cf) * 2 * (size_t)nrhs * n);
        cf* xf = lowbuf.as<cf>();
        cf* yf = xf + (int64_t)nrhs * n;
        launch_convert<float, double>(s, x, xf, (int64_t)nrhs * n);
        const bool half = g.prm.precision == MGM_PREC_FP16 && L.f.hdinv.p != nullptr;
        if (half) {
          launch = [=, &L] { launch_dense_apply_h(s, L.f.hdinv.as<chalf>(), n, nrhs, xf, yf, nullptr); };
        } else {
          launch = [=, &L, &g] {
            launch_dense_apply<float>(s, L.f.dinv.as<cf>(), n, nrhs, xf, yf, nullptr, &g.scratch[c->wslot]);
          };
        }
        bytes = (half ? 4.0 : 8.0) * n * n + 16.0 * n * b;
        flops = 8.0 * n * n * b;
        break;
      }
      case MGM_KERNEL_SAP_LOW: {
        require(g.mg_ready && L.ncolor[0] > 0, "SAP needs setup_mg on this level", MGM_ESTATE);
        require(g.prm.precision != MGM_PREC_FP64, "the preconditioner runs in FP64 (mgm_set_precision)",
                MGM_ESTATE);
        lowbuf.ensure(sizeof(cf) * 2 * (size_t)nrhs * n);
        cf* xf = lowbuf.as<cf>();
        cf* rf = xf + (int64_t)nrhs * n;
        launch_convert<float, double>(s, x, xf, (int64_t)nrhs * n);
        launch_convert<float, double>(s, r, rf, (int64_t)nrhs * n);
        const bool quad = L.f.sapM.p != nullptr;  // premultiplied 2x2 blocks
        const bool half = g.prm.precision == MGM_PREC_FP16 && L.M == 16 &&
                          ((L.sbt == 1 && (L.sbx == 1 || L.sbx == 2)) || quad) && L.f.hblocks.p != nullptr;
        // the premultiplied two-site sweep x_B = rho_B - M_B x_H of the later
        // cycles (rf stands in for rho)
        const bool premul = half && L.sbx == 2 && L.f.hsapM.p != nullptr;
        // the fine level's FP32 cycle runs its sweeps in the block-major layout
        const bool fblk = L.M == 2 && L.sbx == 4 && L.sbt == 4 && L.has_coarse && L.bx == 4 && L.bt == 4 &&
                          L.ntv == 8;
        if (fblk) {
          launch = [=, &L] {
            launch_sap0_blk(s, L.f.B(), L.f.sapinv.as<cf>(), L.Nx, L.Nt, L.color_list[0].as<int>(), L.ncolor[0],
                            nrhs, rf, xf, nullptr, nullptr);
          };
        } else if (quad && half) {
          launch = [=, &L] {
            launch_sap4p_h(s, L.f.hsapM.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, L.color_list[0].as<int>(),
                           L.ncolor[0], nrhs, false, nullptr, rf, xf, nullptr);
          };
        } else if (quad) {
          launch = [=, &L] {
            launch_sap4p<float>(s, L.f.sapM.as<cf>(), L.f.sapinv.as<cf>(), L.Nx, L.Nt, L.color_list[0].as<int>(),
                                L.ncolor[0], nrhs, false, nullptr, rf, xf, nullptr);
          };
        } else if (premul) {
          launch = [=, &L] {
            launch_sap2p_h(s, L.f.hsapM.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, L.color_list[0].as<int>(),
                           L.ncolor[0], nrhs, false, nullptr, rf, xf, nullptr);
          };
        } else if (half) {
          launch = [=, &L] {
            launch_sap_h(s, L.f.hblocks.as<chalf>(), L.f.hsapinv.as<chalf>(), L.Nx, L.Nt, L.sbx, L.sbt,
                         L.color_list[0].as<int>(), L.ncolor[0], nrhs, rf, xf, nullptr);
          };
        } else {
          launch = [=, &L] {
            launch_sap_sweep<float>(s, L.f.B(), L.f.sapinv.as<cf>(), L.Nx, L.Nt, L.M, L.sbx, L.sbt,
                                    L.color_list[0].as<int>(), L.ncolor[0], nrhs, rf, xf, nullptr);
          };
        }
        const double nb = L.ncolor[0];
        const double halo = 2.0 * (L.sbx + L.sbt) * L.M;
        const double hx = (double)sap_halo_sites(L) * L.M;
        const double mb = half ? 4.0 : 8.0;  // bytes per complex matrix entry
        // matrix entries per block: inv_B (K^2) and the outward hops (halo M),
        // or M_B (K x halo) in the premultiplied form
        const double ment = premul || quad ? (double)L.K * halo : (double)L.K * L.K + halo * L.M;
        bytes = 8.0 * b * (2.0 * nb * L.K + hx) + mb * nb * ment;
        flops = 8.0 * b * nb * ment;
        break;
      }
      case MGM_KERNEL_DENSE:
        require(L.has_dense, "level has no dense inverse", MGM_ESTATE);
        launch = [=, &L, &g] {
          launch_dense_apply<double>(s, L.d.dinv.as<cd>(), n, nrhs, x, y, nullptr, &g.scratch[c->wslot]);
        };
        bytes = 16.0 * n * n + 32.0 * n * b;
        flops = 8.0 * n * n * b;
        break;
      case MGM_KERNEL_CGS: {
        // the projection coefficients of one Gram-Schmidt pass in FGMRES
        // step 15: 16 distinct basis vectors per RHS in the solver's layout
        // V[i][r][n] against w = y
        const int nv = 16;
        const int64_t vs = (int64_t)nrhs * n;
        c->scratch3.ensure(sizeof(cd) * ((size_t)nv * vs + (size_t)nrhs * (nv + 1) * reduce_chunks(n) +
                                         (size_t)nrhs * nv));
        cd* V = c->scratch3.as<cd>();
        cd* out = V + nv * vs;
        cd* part = out + (int64_t)nrhs * nv;
        launch_noise<double>(s, V, n, nrhs * nv, MGM_NOISE_Z2Z2, 13, 0, 0, 0);
        launch = [=] { launch_dot_multi_ld<double>(s, V, vs, n, nv, y, n, nrhs, out, nv, 0, nullptr, part); };
        bytes = 16.0 * (nv + 1) * n * b;
        flops = 8.0 * nv * n * b;
        break;
      }
      case MGM_KERNEL_COPY:
        launch = [=] { launch_axpby<double>(s, 1.0, x, 0.0, nullptr, y, n, nrhs, nullptr); };
        bytes = 32.0 * n * b;
        break;
      case MGM_KERNEL_CONV: {
        require(level == 0, "the network runs on level 0");
        cnn_check_lattice(g);
        const Cnn* net = &cnn_of(c);
        const int64_t V = (int64_t)g.Lx * g.Lt;
        g.cnn.a[0].ensure(sizeof(float) * V * 32 * nrhs);
        g.cnn.a[1].ensure(sizeof(float) * V * 32 * nrhs);
        const float* in = g.cnn.a[0].as<float>();
        float* out = g.cnn.a[1].as<float>();
        HIPCHK(hipMemsetAsync(g.cnn.a[0].p, 0, sizeof(float) * V * 32 * nrhs, s));
        launch = [=, &g] { cnn_time_conv(s, *net, g, nrhs, in, out); };
        bytes = 4.0 * V * b * 64 + 4.0 * 32 * 289;
        flops = 2.0 * V * b * 32 * 288;
        break;
      }
      case MGM_KERNEL_CONV_H: {
        require(level == 0, "the network runs on level 0");
        cnn_check_lattice(g);
        const Cnn* net = &cnn_of(c);
        const int64_t V = (int64_t)g.Lx * g.Lt;
        g.cnn.h[0].ensure(sizeof(_Float16) * V * 32 * nrhs);
        g.cnn.h[1].ensure(sizeof(_Float16) * V * 32 * nrhs);
        const _Float16* in = g.cnn.h[0].as<_Float16>();
        _Float16* out = g.cnn.h[1].as<_Float16>();
        HIPCHK(hipMemsetAsync(g.cnn.h[0].p, 0, sizeof(_Float16) * V * 32 * nrhs, s));
        launch = [=, &g] { cnn_time_conv_h(s, *net, g, nrhs, in, out); };
        bytes = 2.0 * V * b * 64 + 2.0 * 32 * 288 + 4.0 * 32;
        flops = 2.0 * V * b * 32 * 288;
        break;
      }
      default:
        throw Error(MGM_EINVAL, "unknown kernel kind");
    }
    launch();  // warm up
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) launch();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *us_out = 1e3 * ms / reps;
    *bytes_out = bytes;
    *flops_out = flops;
    return MGM_OK;
  });
}

int mgm_solve_jobs(mgm_ctx* c, int njobs, const mgm_job* jobs, const mgm_solve_params* prm,
                   int* iters) {
  return guarded(c, [&] {
    require(njobs >= 0 && (njobs == 0 || jobs) && prm, "bad arguments");
    // group the jobs by gauge field, keeping their order inside a group
    std::map<int, std::vector<int>> groups;
    std::vector<int64_t> it_off(njobs + 1, 0);
    for (int j = 0; j < njobs; ++j) {
      const mgm_job& jb = jobs[j];
      require(jb.b && jb.x && jb.nrhs > 0 && jb.b != jb.x, "bad job vectors");
      Gauge& g = gauge_of(c, jb.gauge_id);
      require(g.mg_ready, "setup_mg first", MGM_ESTATE);
      level_of(g, jb.level);
      groups[jb.gauge_id].push_back(j);
      it_off[j + 1] = it_off[j] + jb.nrhs;
    }
    for (auto& kv : groups) {
      Gauge& g = *c->gauges[kv.first];
      HIPCHK(hipEventRecord(g.ev_in, c->stream));
      HIPCHK(hipStreamWaitEvent(g.stream, g.ev_in, 0));
    }
    std::vector<int> status(groups.size(), MGM_OK);
    std::vector<std::string> msg(groups.size());
    std::vector<std::thread> workers;
    int gi = 0;
    for (auto& kv : groups) {
      const int slot = gi++;
      workers.emplace_back([&, slot, gid = kv.first, idx = kv.second] {
        mgm_ctx w;  // per-thread view: the field's stream, private scratch
        w.device = c->device;
        Gauge& g = *c->gauges[gid];
        w.stream = g.stream;
        w.cnn = c->cnn;
        try {
          HIPCHK(hipSetDevice(c->device));
          for (int j : idx) {
            const mgm_job& jb = jobs[j];
            const int st = solve_chunked(&w, g, jb.level, jb.nrhs, static_cast<const cd*>(jb.b),
                                         static_cast<cd*>(jb.x), *prm,
                                         iters ? iters + it_off[j] : nullptr, nullptr);
            if (st != MGM_OK && status[slot] == MGM_OK) status[slot] = st;
          }
          HIPCHK(hipStreamSynchronize(g.stream));
        } catch (const Error& e) {
          status[slot] = e.code;
          msg[slot] = e.what();
        } catch (const std::exception& e) {
          status[slot] = MGM_EHIP;
          msg[slot] = e.what();
        }
      });
    }
    for (auto& t : workers) t.join();
    for (auto& kv : groups) {
      Gauge& g = *c->gauges[kv.first];
      HIPCHK(hipEventRecord(g.ev_out, g.stream));
      HIPCHK(hipStreamWaitEvent(c->stream, g.ev_out, 0));
    }
    for (size_t k = 0; k < status.size(); ++k)
      if (status[k] != MGM_OK) {
        if (!msg[k].empty()) throw Error(status[k], msg[k]);
        c->err = "a job did not converge";
        return status[k];
      }
    return MGM_OK;
  });
}

int mgm_autotune_rhs_block(mgm_ctx* c, int gauge_id, int level, int nrhs,
                           const mgm_solve_params* prm, int* best) {
  return guarded(c, [&] {
    require(prm && best && nrhs > 0, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    Level& L = level_of(g, level);
    hipStream_t s = c->stream;
    c->scratch2.ensure(sizeof(cd) * (size_t)2 * nrhs * L.n);
    cd* b = c->scratch2.as<cd>();
    cd* x = b + (int64_t)nrhs * L.n;
    launch_noise<double>(s, b, L.n, nrhs, MGM_NOISE_Z2Z2, 97, 0, level, 0);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 0;
    int best_w = nrhs;
    for (int w : {8, 16, 32, 64}) {
      if (w > nrhs && w != 8) break;
      mgm_solve_params sp = *prm;
      sp.rhs_block = std::min(w, nrhs);
      // once untimed (allocations, graph capture), then timed
      solve_chunked(c, g, level, nrhs, b, x, sp, nullptr, nullptr);
      HIPCHK(hipEventRecord(e0, s));
      solve_chunked(c, g, level, nrhs, b, x, sp, nullptr, nullptr);
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (best_ms == 0 || ms < best_ms) {
        best_ms = ms;
        best_w = sp.rhs_block;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g.tuned_block[level] = best_w;
    *best = best_w;
    return MGM_OK;
  });
}

// ---------------------------------------------------------------- learned initial guess

int mgm_cnn_set_params(mgm_ctx* c, const float* theta) {
  return guarded(c, [&] {
    require(theta != nullptr, "null pointer");
    if (!c->cnn) {
      c->cnn = std::make_shared<Cnn>();
      c->cnn->init();
    }
    Cnn& net = *c->cnn;
    hipStream_t s = c->stream;
    HIPCHK(hipMemcpyAsync(net.theta.p, theta, sizeof(float) * MGM_CNN_NPARAMS, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(net.m.p, 0, sizeof(float) * MGM_CNN_NPARAMS, s));
    HIPCHK(hipMemsetAsync(net.v.p, 0, sizeof(float) * MGM_CNN_NPARAMS, s));
    net.t = 0;
    net.pack(s);
    HIPCHK(hipStreamSynchronize(s));
    net.ready = true;
    return MGM_OK;
  });
}

int mgm_cnn_set_precision(mgm_ctx* c, int precision) {
  return guarded(c, [&] {
    require(precision == MGM_PREC_FP32 || precision == MGM_PREC_FP16, "network precision must be FP32 or FP16");
    Cnn& net = cnn_of(c);
    const bool half = precision == MGM_PREC_FP16;
    if (net.half != half) {
      net.half = half;
      // captured solver steps with the learned stage hold the other
      // precision's kernels: retire every captured graph
      g_alloc_epoch.fetch_add(1);
    }
    return MGM_OK;
  });
}

int mgm_cnn_get_params(mgm_ctx* c, float* theta) {
  return guarded(c, [&] {
    require(theta != nullptr, "null pointer");
    Cnn& net = cnn_of(c);
    HIPCHK(hipMemcpyAsync(theta, net.theta.p, sizeof(float) * MGM_CNN_NPARAMS, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

int mgm_cnn_apply(mgm_ctx* c, int gauge_id, int nb, const void* b, void* y) {
  return guarded(c, [&] {
    require(b && y && nb > 0, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    cnn_apply(c->stream, cnn_of(c), g, nb, static_cast<const cd*>(b), static_cast<cd*>(y), g.cnn);
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

namespace {
// channel-last FP32 copy of b and the loss/gradient of the pairs (b, x)
const double* loss_grad_pairs(mgm_ctx* c, Gauge& g, int nb, const void* b, const void* x) {
  cnn_check_lattice(g);
  Cnn& net = cnn_of(c);
  const int64_t n = g.levels[0]->n;
  g.cnn.x0.ensure(sizeof(float) * nb * n * 2);
  cnn_to_channels(c->stream, static_cast<const cd*>(b), nb * n, g.cnn.x0.as<float>());
  return cnn_loss_grad<double>(c->stream, net, g, nb, g.cnn.x0.as<float>(),
                               static_cast<const double*>(x), g.cnn);
}
}  // namespace

int mgm_cnn_loss_grad(mgm_ctx* c, int gauge_id, int nb, const void* b, const void* x, double* loss,
                      float* grad) {
  return guarded(c, [&] {
    require(b && x && loss && nb > 0, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    const double* ld = loss_grad_pairs(c, g, nb, b, x);
    HIPCHK(hipMemcpyAsync(loss, ld, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (grad)
      HIPCHK(hipMemcpyAsync(grad, c->cnn->grad.p, sizeof(float) * MGM_CNN_NPARAMS, hipMemcpyDeviceToHost,
                            c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

int mgm_cnn_train_step(mgm_ctx* c, int gauge_id, int nb, const void* b, const void* x,
                       const mgm_adam_params* adam, double* loss) {
  return guarded(c, [&] {
    require(b && x && loss && adam && nb > 0, "bad arguments");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    const double* ld = loss_grad_pairs(c, g, nb, b, x);
    HIPCHK(hipMemcpyAsync(loss, ld, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    cnn_adam(c->stream, *c->cnn, *adam);
    HIPCHK(hipStreamSynchronize(c->stream));
    return MGM_OK;
  });
}

int mgm_cnn_train(mgm_ctx* c, int nfields, const int* gauge_ids, const mgm_cnn_train_params* prm,
                  double* epoch_loss) {
  return guarded(c, [&] {
    require(gauge_ids && prm && nfields > 0, "bad arguments");
    require(prm->pairs_per_field > 0 && prm->batch > 0 && prm->epochs >= 0, "bad training sizes");
    Cnn& net = cnn_of(c);
    Gauge& g0 = gauge_of(c, gauge_ids[0]);
    cnn_check_lattice(g0);
    for (int f = 0; f < nfields; ++f) {
      Gauge& g = gauge_of(c, gauge_ids[f]);
      require(g.Lx == g0.Lx && g.Lt == g0.Lt && g.anti == g0.anti,
              "training fields must share lattice size and boundary condition");
      require(g.mg_ready, "setup_mg first", MGM_ESTATE);
    }
    const int64_t n = g0.levels[0]->n;
    const int P = prm->pairs_per_field;
    const int64_t npairs = (int64_t)nfields * P;
    CnnWork& w = g0.cnn;
    w.pairs_b.ensure(sizeof(float) * npairs * n * 2);
    w.pairs_x.ensure(sizeof(float) * npairs * n * 2);
    // targets: multigrid solves on each field's own stream, in chunks
    const int chunk = std::min(P, 64);
    int status = MGM_OK;
    for (int f = 0; f < nfields; ++f) {
      Gauge& g = gauge_of(c, gauge_ids[f]);
      OnGauge og(c, g);
      hipStream_t s = c->stream;
      c->scratch2.ensure(sizeof(cd) * (size_t)2 * chunk * n);
      cd* bb = c->scratch2.as<cd>();
      cd* xx = bb + (int64_t)chunk * n;
      for (int p0 = 0; p0 < P; p0 += chunk) {
        const int k = std::min(chunk, P - p0);
        launch_noise<double>(s, bb, n, k, MGM_NOISE_Z2Z2, prm->seed, MGM_PURPOSE_TRAIN, 0, p0);
        mgm_solve_params sp = prm->solve;
        sp.use_cnn = 0;
        const int st = solve_chunked(c, g, 0, k, bb, xx, sp, nullptr, nullptr);
        if (st != MGM_OK) status = st;
        const int64_t at = ((int64_t)f * P + p0) * n * 2;
        cnn_to_channels(s, bb, (int64_t)k * n, w.pairs_b.as<float>() + at);
        cnn_to_channels(s, xx, (int64_t)k * n, w.pairs_x.as<float>() + at);
      }
      HIPCHK(hipStreamSynchronize(s));
    }
    if (status != MGM_OK) throw Error(status, "a training target solve did not converge");
    // epochs over the pairs in a seeded order (Fisher-Yates on SplitMix64)
    OnGauge og(c, g0);
    hipStream_t s = c->stream;
    const int B = (int)std::min<int64_t>(prm->batch, npairs);
    w.batch_b.ensure(sizeof(float) * B * n * 2);
    w.batch_x.ensure(sizeof(float) * B * n * 2);
    std::vector<int64_t> order(npairs);
    for (int e = 0; e < prm->epochs; ++e) {
      for (int64_t i = 0; i < npairs; ++i) order[i] = i;
      const uint64_t key = mix64(prm->seed + kGolden) ^ ((uint64_t)MGM_PURPOSE_TRAIN << 56) ^ (uint64_t)e;
      for (int64_t i = npairs - 1; i > 0; --i) {
        const uint64_t z = mix64(key + (uint64_t)i * kGolden);
        std::swap(order[i], order[(int64_t)(z % (uint64_t)(i + 1))]);
      }
      double sum = 0.0;
      int nsteps = 0;
      for (int64_t p0 = 0; p0 + B <= npairs; p0 += B) {
        for (int j = 0; j < B; ++j) {
          const int64_t src = order[p0 + j] * n * 2;
          HIPCHK(hipMemcpyAsync(w.batch_b.as<float>() + (int64_t)j * n * 2, w.pairs_b.as<float>() + src,
                                sizeof(float) * n * 2, hipMemcpyDeviceToDevice, s));
          HIPCHK(hipMemcpyAsync(w.batch_x.as<float>() + (int64_t)j * n * 2, w.pairs_x.as<float>() + src,
                                sizeof(float) * n * 2, hipMemcpyDeviceToDevice, s));
        }
        const double* ld = cnn_loss_grad<float>(s, net, g0, B, w.batch_b.as<float>(),
                                                w.batch_x.as<float>(), w);
        double l = 0;
        HIPCHK(hipMemcpyAsync(&l, ld, sizeof(double), hipMemcpyDeviceToHost, s));
        cnn_adam(s, net, prm->adam);
        HIPCHK(hipStreamSynchronize(s));
        sum += l;
        ++nsteps;
      }
      if (epoch_loss) epoch_loss[e] = nsteps ? sum / nsteps : 0.0;
    }
    return MGM_OK;
  });
}

int mgm_trace_estimate(mgm_ctx* c, int gauge_id, const mgm_trace_params* prm,
                       mgm_trace_result* res) {
  return guarded(c, [&] {
    require(prm && res, "null pointer");
    Gauge& g = gauge_of(c, gauge_id);
    OnGauge og(c, g);
    return trace_estimate(c, g, *prm, *res);
  });
}

int mgm_trace_jobs(mgm_ctx* c, int njobs, const int* gauge_ids, const mgm_trace_params* prm,
                   mgm_trace_result* res) {
  return guarded(c, [&] {
    require(njobs >= 0 && (njobs == 0 || (gauge_ids && prm && res)), "bad arguments");
    std::vector<Gauge*> gs(njobs);
    for (int j = 0; j < njobs; ++j) {
      gs[j] = &gauge_of(c, gauge_ids[j]);
      for (int q = 0; q < j; ++q) require(gs[q] != gs[j], "trace_jobs: every job needs a field of its own");
    }
    for (Gauge* g : gs) {
      HIPCHK(hipEventRecord(g->ev_in, c->stream));
      HIPCHK(hipStreamWaitEvent(g->stream, g->ev_in, 0));
      if (!g->view) g->view = std::make_shared<mgm_ctx>();
      mgm_ctx& w = *g->view;  // the field's worker context: its stream, its workspaces
      w.device = c->device;
      w.stream = g->stream;
      w.cnn = c->cnn;
      w.wslot = 0;
    }
    std::vector<int> status(njobs, MGM_OK);
    std::vector<std::string> msg(njobs);
    std::vector<std::thread> workers;
    for (int j = 0; j < njobs; ++j) {
      workers.emplace_back([&, j] {
        Gauge& g = *gs[j];
        try {
          HIPCHK(hipSetDevice(c->device));
          status[j] = trace_estimate(g.view.get(), g, prm[j], res[j]);
          HIPCHK(hipStreamSynchronize(g.stream));
        } catch (const Error& e) {
          status[j] = e.code;
          msg[j] = e.what();
        } catch (const std::exception& e) {
          status[j] = MGM_EHIP;
          msg[j] = e.what();
        }
      });
    }
    for (auto& t : workers) t.join();
    for (Gauge* g : gs) {
      HIPCHK(hipEventRecord(g->ev_out, g->stream));
      HIPCHK(hipStreamWaitEvent(c->stream, g->ev_out, 0));
    }
    for (int j = 0; j < njobs; ++j)
      if (status[j] != MGM_OK) {
        if (!msg[j].empty()) throw Error(status[j], "job " + std::to_string(j) + ": " + msg[j]);
        c->err = "job " + std::to_string(j) + " did not reach its target";
        return status[j];
      }
    return MGM_OK;
  });
}

}  // extern "C"
