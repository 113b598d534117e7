// Internal types and kernel launchers of the MG-MLMC++ library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mgmlmc.h"

namespace mgm {

// ---------------------------------------------------------------- complex
template <class T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};
using cd = cx<double>;
using cf = cx<float>;
// complex FP16 storage (coarse stencil blocks and inverses of the FP16 mode)
struct alignas(4) chalf {
  _Float16 re, im;
};

template <class T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  return cx<T>{a, b};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return {s * a.re, s * a.im};
}
template <class T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) {
  return {a.re, -a.im};
}
// conj(a) * b
template <class T>
__host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc += a * b
// ok ? *p : 0 with the load issued unconditionally; p must be a valid address
// either way (callers clamp their indices).  Written as a conditional load,
// the compiler branches around the load and waits for memory right after
// it, which serialises all such loads of a thread; a select after an
// unconditional load lets them all be in flight together.
template <class T>
__device__ __forceinline__ cx<T> ld_or0(const cx<T>* p, bool ok) {
  const cx<T> v = *p;
  return ok ? v : mk<T>(0, 0);
}

// The chip hands workgroups to its eight XCDs round-robin by linear
// workgroup id, and each XCD has its own L2.  xcd_tile(b, G) renumbers b in
// [0, G) so that the ids one XCD receives cover one contiguous range of tiles;
// neighbouring tiles, and the halo values they share, then meet in the same
// L2 instead of being fetched from HBM once per XCD.  It is a bijection on
// [0, G) for every G; the ranges line up with the XCDs exactly when the
// grid's x extent is a multiple of eight.
__host__ __device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) {
  constexpr int64_t NXCD = 8;
  const int64_t q = G / NXCD, rem = G % NXCD;
  const int64_t x = b % NXCD, loc = b / NXCD;
  return x * q + (x < rem ? x : rem) + loc;
}

template <class T>
__host__ __device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += conj(a) * b
template <class T>
__host__ __device__ __forceinline__ void cjfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}
template <class T>
__host__ __device__ __forceinline__ T abs2(cx<T> a) {
  return a.re * a.re + a.im * a.im;
}
// a / b
template <class T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
  T d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// ---------------------------------------------------------------- matrix cores
// 16x16x4 matrix-core step in the precision of the cycle.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; element v of its result is
// D[out_row(l, v)][l%16]: rows l/16 + 4v for FP64, 4(l/16) + v for FP32
// (both measured on gfx950 with an in-bounds probe).
template <class T>
struct MF;
template <>
struct MF<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct MF<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <class T>
struct CAcc {
  typename MF<T>::v4 re, im;
};

template <class T>
__device__ __forceinline__ void cmma(cx<T> a, cx<T> b, CAcc<T>& acc) {
  acc.re = MF<T>::mma(a.re, b.re, acc.re);
  acc.re = MF<T>::mma(-a.im, b.im, acc.re);
  acc.im = MF<T>::mma(a.re, b.im, acc.im);
  acc.im = MF<T>::mma(a.im, b.re, acc.im);
}

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      throw ::mgm::Error(e_ == hipErrorOutOfMemory ? MGM_ENOMEM : MGM_EHIP,          \
                         std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define KCHK() HIPCHK(hipGetLastError())

inline void require(bool ok, const std::string& msg, int code = MGM_EINVAL) {
  if (!ok) throw Error(code, msg);
}

// ---------------------------------------------------------------- memory
// Bumped on every device (re)allocation: a captured HIP graph is only valid
// while the buffers it references keep their addresses.
extern std::atomic<uint64_t> g_alloc_epoch;

// Owning device buffer (freed with hipFree; never used for host memory).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t b) {
    if (b <= bytes) return;
    release();
    g_alloc_epoch.fetch_add(1);
    HIPCHK(hipMalloc(&p, b));
    bytes = b;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// ---------------------------------------------------------------- noise
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

template <class T>
void launch_noise(hipStream_t s, cx<T>* out, int64_t n, int nrhs, int kind, uint64_t seed,
                  int purpose, int level, int64_t index0);

// ---------------------------------------------------------------- level operators
// Direction order of the block stencil: 0 self, 1 +x, 2 -x, 3 +t, 4 -t.
template <class T>
void launch_wilson(hipStream_t s, const cx<T>* links, T diag, int Lx, int Lt, int nrhs,
                   const cx<T>* x, cx<T>* y, const cx<T>* b, const int* active);
void launch_fine_blocks(hipStream_t s, const cd* links, double diag, int Lx, int Lt, cd* blocks);
void launch_fold_anti(hipStream_t s, cd* links, int Lx, int Lt);
template <class T>
void launch_stencil(hipStream_t s, const cx<T>* blocks, int Nx, int Nt, int M, int nrhs,
                    const cx<T>* x, cx<T>* y, const cx<T>* b, const int* active);
template <class T>
void launch_restrict(hipStream_t s, const cx<T>* P, int Nx, int Nt, int M, int bx, int bt, int ntv,
                     int nrhs, const cx<T>* xf, cx<T>* xc, const int* active);
template <class T>
void launch_prolong(hipStream_t s, const cx<T>* P, int Nx, int Nt, int M, int bx, int bt, int ntv,
                    int nrhs, const cx<T>* xc, cx<T>* yf, int accumulate, const int* active);
void launch_galerkin(hipStream_t s, const cd* Bf, int Nx, int Nt, int Mf, const cd* P, int bx,
                     int bt, int ntv, cd* Bc);
void launch_sap_extract(hipStream_t s, const cd* B, int Nx, int Nt, int M, int sbx, int sbt,
                        cd* blocks_out);
void launch_small_inverse(hipStream_t s, cd* mats, int K, int count, int* fail);
template <class T>
// x64 (or null, 4x4-site blocks of 2 dofs only): also store the swept
// blocks' new values widened to FP64 there
void launch_sap_sweep(hipStream_t s, const cx<T>* B, const cx<T>* inv, int Nx, int Nt, int M,
                      int sbx, int sbt, const int* blist, int nb, int nrhs, const cx<T>* r,
                      cx<T>* x, const int* active, cd* x64 = nullptr);
void launch_dense_from_stencil(hipStream_t s, const cd* B, int Nx, int Nt, int M, cd* A);
// FP16-block variants for coarse levels with 16 dofs per site (FP32 vectors,
// FP16 matrix-core products, FP32 accumulation)
void launch_to_half(hipStream_t s, const cd* in, chalf* out, int64_t count);
// The fine level's FP32 cycle in the block-major layout (4x4-site blocks =
// 4x4 aggregates, 2 dofs, 8 test vectors: a block's 32 dofs contiguous, sites
// t-major): restriction from it, prolongation into it (overwriting), one SAP
// colour sweep in it (x64: the result also widened to FP64 in the lattice
// layout, or null), and the FP64 lattice -> FP32 block-major rounding
void launch_restrict_blk(hipStream_t s, const cf* P, int Nx, int Nt, int nrhs, const cf* xf, cf* xc,
                         const int* active);
void launch_prolong_blk(hipStream_t s, const cf* P, int Nx, int Nt, int nrhs, const cf* xc, cf* yf,
                        const int* active);
void launch_sap0_blk(hipStream_t s, const cf* B, const cf* inv, int Nx, int Nt, const int* blist, int nb,
                     int nrhs, const cf* r, cf* x, const int* active, cd* x64);
void launch_convert_blk(hipStream_t s, const cd* in, cf* out, int Nx, int Nt, int nrhs);
// the same, setting *overflow (device) when a component is not finite in FP16
void launch_to_half_checked(hipStream_t s, const cd* in, chalf* out, int64_t count, int* overflow);
// y[r] = A x[r], A n x n in FP16 (x rounded to FP16, FP32 accumulation), n % 256 == 0
void launch_dense_apply_h(hipStream_t s, const chalf* A, int64_t n, int nrhs, const cf* x, cf* y,
                          const int* active);
void launch_stencil_h(hipStream_t s, const chalf* blocks, int Nx, int Nt, int nrhs, const cf* x, cf* y,
                      const cf* b, const int* active);
// ec (single-site blocks): the first colour's first sweep after the coarse
// correction, the neighbours' x formed from ec through hP (FP16 prolongation
// of 2x2 aggregates with 8 test vectors) instead of read from x
void launch_sap_h(hipStream_t s, const chalf* blocks, const chalf* inv, int Nx, int Nt, int sbx, int sbt,
                  const int* blist, int nb, int nrhs, const cf* r, cf* x, const int* active, const chalf* hP = nullptr,
                  const cf* ec = nullptr);
// Two-site (2x1) FP16 SAP in premultiplied form: M_B = inv_B D_BH at setup
// ([nblk][6 hops][32][16] FP16) and a colour sweep x_B = rho_B - M_B x_H; the
// first sweep of each colour in a visit (`first`) forms rho_B = inv_B r_B
// from r and stores it in rho ([nrhs][n]) for the later ones
void launch_sap2_premul(hipStream_t s, const cd* blocks, const cd* inv, int Nx, int nblk, chalf* M);
// 2x2-site blocks of 16-dof levels: M_B = inv_B D_BH ([nblk][8 hops][64][16], FP64)
// and one colour of the premultiplied sweep x_B = rho_B - M_B x_H (first:
// rho_B = inv_B r_B formed and stored); FP16 operands, or FP32 / FP64
void launch_sap4_premul(hipStream_t s, const cd* blocks, const cd* inv, int Nx, int nblk, cd* M);
// ec (with first): the colour's first sweep after the coarse correction,
// whose halo comes from ec (coarse vector) through hP (FP16 prolongation of
// 2x2 aggregates with 8 test vectors) instead of from x
void launch_sap4p_h(hipStream_t s, const chalf* M, const chalf* inv, int Nx, int Nt, const int* blist, int nb,
                    int nrhs, bool first, const cf* r, cf* rho, cf* x, const int* active, const chalf* hP = nullptr,
                    const cf* ec = nullptr);
template <class T>
void launch_sap4p(hipStream_t s, const cx<T>* M, const cx<T>* inv, int Nx, int Nt, const int* blist, int nb,
                  int nrhs, bool first, const cx<T>* r, cx<T>* rho, cx<T>* x, const int* active);
void launch_sap2p_h(hipStream_t s, const chalf* M, const chalf* inv, int Nx, int Nt, const int* blist, int nb,
                    int nrhs, bool first, const cf* r, cf* rho, cf* x, const int* active);
// In-place Gauss-Jordan inverse with partial pivoting of the n x n matrix A.
int dense_inverse(hipStream_t s, cd* A, int64_t n, cd* scratch_out);
void launch_diag_sum(hipStream_t s, const cd* A, int64_t n, cd* out);
template <class T>
void launch_dense_apply(hipStream_t s, const cx<T>* A, int64_t n, int nrhs, const cx<T>* x,
                        cx<T>* y, const int* active, DevBuf* scratch);

// ---------------------------------------------------------------- batched BLAS
// V_i of RHS r sits at V + i*sI + r*sR (complex elements).
template <class T>
void launch_dot_multi_ld(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv,
                         const cx<T>* w, int64_t n, int nrhs, cx<T>* out, int ldo, int accumulate,
                         const int* active, cx<T>* partial);
// done[r] = (bnorm[r] == 0)
// number of chunk partials a reduction over n elements produces
// (upper bound: the shortest chunk is 256 elements)
inline int64_t reduce_chunks(int64_t n) { return (n + 255) / 256; }
// w[r] += sign * sum_{i < min(nv, nlim[r])} V_i[r] coef[r*ldc + i]; optional ||w||
template <class T>
void launch_update_multi(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv,
                         const cx<T>* coef, int ldc, T sign, cx<T>* w, int64_t n, int nrhs,
                         const int* active, T* norm_out, T* partial, const int* nlim = nullptr);
// zero_done (optional): zero_done[r] = 1 where the norm is 0, else 0
template <class T>
void launch_norm(hipStream_t s, const cx<T>* w, int64_t n, int nrhs, T* out, const int* active,
                 T* partial, int* zero_done = nullptr);
// FGMRES from x = 0: ||b|| (with the zero-RHS flags), the first cycle's
// state (launch_fgmres_init with beta = ||b||) and v_0 = b / ||b|| in one
// norm-partial launch and one more (same bits as launch_norm, launch_fgmres_init
// and launch_scale); vf (or null): v_0 rounded to FP32 as launch_hcol_scale
// stores v_{j+1} (block-major when blk_nx > 0)
void launch_fgmres_start(hipStream_t s, const cd* b, int64_t n, int nrhs, double* partial, int m, double tol,
                         double* bnorm, int* done, int* active, int* nit, cd* g, double* thr, cd* v, cf* vf,
                         int blk_nx);
// launch_norm (same bits) whose reduce kernel also hands the host what it
// reads with the norms, in pinned host memory: host[r] = ||w_r||,
// host[nrhs + r] = bnorm[r], hnit[r] = nit[r] (no copies)
void launch_norm_readback(hipStream_t s, const cd* w, int64_t n, int nrhs, double* out, double* partial,
                          const double* bnorm, const int* nit, double* host, int* hnit);
template <class T>
void launch_scale(hipStream_t s, const cx<T>* w, const T* den, int64_t n, int nrhs, cx<T>* v,
                  const int* active);
template <class T>
void launch_axpby(hipStream_t s, T a, const cx<T>* x, T b, const cx<T>* y, cx<T>* z, int64_t n,
                  int nrhs, const int* active);
template <class TO, class TI>
void launch_convert(hipStream_t s, const cx<TI>* in, cx<TO>* out, int64_t count);
template <class T>
void launch_givens(hipStream_t s, int j, int m, int nrhs, cx<T>* H, T* cs, cx<T>* sn, cx<T>* g,
                   const T* thr, int* active, int* nit);
// The Gram-Schmidt pieces of an Arnoldi step with the chunk reductions moved
// into the consumers: V_i^H w and V_i^H u (i < nv) with one read of the
// basis, partials [r][2 nv][nch] (w's first; returns nch); the update that
// reduces them itself; v = w / ||w|| that reduces the norm partials itself
// (||w|| also to den_out).
template <class T>
int launch_dot_partial2(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv, const cx<T>* w,
                        const cx<T>* u, int64_t n, int nrhs, const int* active, cx<T>* partial);
// w -= V (h1 + (I - G) h1) from those partials (h1 = V^H w, new Gram column
// g = V^H v_{nv-1}; gram: per RHS ldg x ldg column-major, earlier columns
// kept from the previous steps, column nv-1 stored here); coefficients to
// coef_out; optional |w|^2 chunk partials
template <class T>
void launch_update_gram(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv, const cx<T>* dpart,
                        int nchd, cx<T>* gram, int ldg, cx<T>* coef_out, int ldc, cx<T>* w, int64_t n, int nrhs,
                        const int* active, T* norm_partial);
// the end of a fused Arnoldi step j: |w| from the chunk partials of |w|^2,
// launch_hcol_givens (no c2), and v = v_{j+1} = w / |w| with its FP32
// rounding vf (block-major when blk_nx > 0), in one launch
template <class T>
void launch_hcol_scale(hipStream_t s, int j, int m, int nrhs, const cx<T>* c1, const T* npart, cx<T>* H, T* cs,
                       cx<T>* sn, cx<T>* g, const T* thr, int* active, int* nit, int* host_flags, const cx<T>* w,
                       int64_t n, cx<T>* v, cf* vf, int blk_nx);
template <class T>
void launch_scale_r(hipStream_t s, const cx<T>* w, const T* npart, int64_t n, int nrhs, cx<T>* v, T* den_out,
                    const int* active);
// the Hessenberg column of step j and its Givens update in one launch;
// host_flags (pinned, or null) receives the active flags after the step
template <class T>
void launch_hcol_givens(hipStream_t s, int j, int m, int nrhs, const cx<T>* c1, const cx<T>* c2, const T* hn,
                        cx<T>* H, T* cs, cx<T>* sn, cx<T>* g, const T* thr, int* active, int* nit,
                        int* host_flags);
template <class T>
void launch_backsolve(hipStream_t s, int m, int nrhs, const cx<T>* H, const cx<T>* g,
                      const int* nit, cx<T>* y);
// x += Z y (overwrite: x = Z y, x not read) with y = R^{-1} g solved inside
// the update (k_backsolve's arithmetic, same bits): Z [r] at stride sI per
// basis vector, H/g/nit as launch_backsolve takes them
template <class T>
void launch_update_backsolve(hipStream_t s, const cx<T>* Z, int64_t sI, int64_t n, int m, const cx<T>* H,
                             const cx<T>* g, const int* nit, cx<T>* x, int nrhs, bool overwrite);
template <class T>
void launch_fgmres_init(hipStream_t s, int nrhs, const T* beta, const int* parent, const int* done,
                        T tol, const T* bnorm, int m, int* active, int* nit, cx<T>* g, T* thr);
void launch_gram(hipStream_t s, const cd* Y, int64_t n, int d, cd* G, cd* partial);
// out = gamma5 in for `count` complex numbers of fine-level vectors (even
// length n, so the dof parity is the spin)
void launch_gamma5(hipStream_t s, const cd* in, cd* out, int64_t count);
// p[0..count) = v (a kernel, so that captured graphs hold no memset node)
void launch_fill_int(hipStream_t s, int* p, int count, int v);
// G + shift tr(G) I = R^H R; G <- R^{-1}; *fail_dev |= 1 if not positive definite
void launch_cholesky_rinv(hipStream_t s, cd* G, int d, double shift, int* fail_dev);
// number of Gram partials launch_gram writes (each d x d)
int64_t gram_partials(int64_t n);
void launch_local_qr(hipStream_t s, const cd* V, int64_t n, int Nx, int Nt, int M, int bx, int bt,
                     int ntv, cd* P);
void launch_right_tri(hipStream_t s, const cd* Y, const cd* Rinv, int64_t n, int d, cd* Q);
// Z -= Q (Q^H Z) for k <= 64 vectors Z [k][n] and d <= 64 basis vectors
// Q [d][n] on the FP64 matrix cores; C receives Q^H Z ([d][k]); partial
// holds proj_partials(n) * d * k values.
void launch_project(hipStream_t s, const cd* Q, int d, cd* Z, int k, int64_t n, cd* C, cd* partial);
int64_t proj_partials(int64_t n);

// ---------------------------------------------------------------- context
template <class T>
struct LevelData {
  DevBuf blocks;   // [sites][5][M][M]
  DevBuf P;        // [nagg][2][nrow][ntv]   (level -> level+1)
  DevBuf sapinv;   // [nblk][K][K]
  DevBuf dinv;     // coarsest: [n][n]
  DevBuf hblocks, hsapinv;  // FP16 copies of blocks / sapinv (16-dof coarse levels)
  DevBuf hsapM;             // FP16 inv_B D_BH of 2x1 SAP blocks (16-dof coarse levels)
  DevBuf hdinv;             // FP16 dense inverse of the coarsest level (empty if out of range)
  DevBuf sapM;              // inv_B D_BH of 2x2 SAP blocks (16-dof levels; FP16 copy in hsapM)
  DevBuf hP;                // FP16 copy of P (16-dof levels with 2x2 aggregates, 8 test vectors)
  const cx<T>* B() const { return blocks.as<cx<T>>(); }
};

// Pinned host slots for per-RHS flags, written by the device, with kDepth
// completion events, so the host can read step j's flags while the following
// step is already queued.
struct PinnedFlags {
  static constexpr int kDepth = 2;
  int* h = nullptr;
  int cap = 0;
  hipEvent_t ev[kDepth] = {};
  PinnedFlags() = default;
  PinnedFlags(const PinnedFlags&) = delete;
  PinnedFlags& operator=(const PinnedFlags&) = delete;
  void ensure(int n) {
    if (!ev[0])
      for (hipEvent_t& e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (n <= cap) return;
    if (h) (void)hipHostFree(h);
    h = nullptr;
    cap = 0;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h), sizeof(int) * kDepth * (size_t)n, hipHostMallocDefault));
    cap = n;
    g_alloc_epoch.fetch_add(1);  // captured steps hold the old address
  }
  ~PinnedFlags() {
    if (h) (void)hipHostFree(h);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Pinned host copies of a cycle's end residuals, RHS norms and iteration
// counts, written by the norm's reduce kernel (launch_norm_readback).
struct PinnedReadback {
  double* h = nullptr;  // [2][cap]: ||r||, ||b||; then cap ints of iterations
  int cap = 0;
  PinnedReadback() = default;
  PinnedReadback(const PinnedReadback&) = delete;
  PinnedReadback& operator=(const PinnedReadback&) = delete;
  void ensure(int n) {
    if (n <= cap) return;
    if (h) (void)hipHostFree(h);
    h = nullptr;
    cap = 0;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h), (2 * sizeof(double) + sizeof(int)) * (size_t)n,
                         hipHostMallocDefault));
    cap = n;
  }
  int* nit() const { return reinterpret_cast<int*>(h + 2 * (size_t)cap); }
  ~PinnedReadback() {
    if (h) (void)hipHostFree(h);
  }
};

template <class T>
struct Work {  // FGMRES + multigrid workspace of one level in one precision
  int cap = 0, mcap = 0;
  int64_t n = 0;
  DevBuf V, Z, w, H, cs, sn, g, y, beta, thr, bnorm, act, nit, part, npart, coef, coef2, gram;
  DevBuf rc, ec, cvt_in, cvt_out;  // coarse rhs/solution, precision conversions
  DevBuf rho;                        // inv_B r_B of the premultiplied SAP
  PinnedFlags flags;                 // active flags read back during FGMRES
  PinnedReadback rb;                 // residuals read back at a cycle's end
};

struct Level {
  int Nx = 0, Nt = 0, M = 0;
  int64_t sites = 0, n = 0;
  int bx = 0, bt = 0, ntv = 0;  // aggregation to level+1 (0 on the coarsest)
  int sbx = 0, sbt = 0, K = 0, nblk = 0, sap_cycles = 0, inner_iters = 0;
  bool has_coarse = false, is_coarsest = false;
  bool has_dense = false;  // dense inverse available (coarsest or MLMC-closing level)
  DevBuf color_list[2];
  int ncolor[2] = {0, 0};
  LevelData<double> d;
  LevelData<float> f;
  // two workspace sets: set 1 serves a solve that runs concurrently with
  // one on set 0 (the estimator's coarse-level solves)
  Work<double> wd[3];
  Work<float> wf[3];
  int64_t nrow() const { return (int64_t)bx * bt * (M / 2); }
  int64_t nagg() const { return bx ? (int64_t)(Nx / bx) * (Nt / bt) : 0; }
};

// A captured preconditioner application: (level, nrhs, input, output, active
// flags, precision) -> instantiated graph.
using GraphKey = std::tuple<int, int, const void*, void*, const int*, int>;
struct GraphEntry {
  uint64_t epoch = 0;             // allocation epoch when first run / captured
  hipGraphExec_t exec = nullptr;  // null until captured
  bool failed = false;            // capture not possible: always run directly
};

// Learned initial guess: parameters (FP32 master copy, Adam moments, last
// gradient) and the per-layer packed weights the convolution kernels read.
struct Cnn {
  DevBuf theta, m, v, grad;
  DevBuf wf[4], wb[4], wh[4];  // FP32 forward / transposed, FP16 forward copies
  int64_t t = 0;  // Adam steps taken
  bool ready = false;
  bool half = false;  // inference (mgm_cnn_apply, initial guess) in FP16
  void init();
  void pack(hipStream_t s);
  const float* bias(int l) const;
};

// Per-field network workspaces (activations of the RHS chunk in flight).
struct CnnWork {
  DevBuf x0, y, gy, a[3], g[2], part, lpart, mr;
  DevBuf hx0, hy, h[2];  // FP16 inference buffers
  DevBuf pairs_b, pairs_x, batch_b, batch_x, idx;
  DevBuf st_x, st_u;  // learned preconditioner stage: x1 and D x1 / residual
};

// Trace-estimator workspaces, kept with the field so that repeated estimates
// reuse them (no reallocation, so captured graphs stay valid).
struct EstWork {
  DevBuf t1, t3, t4, dots, part;
  // per level difference: Hutch++ sketch S, its image Y and basis Q; sample
  // noise Z, its image X and projection coefficients C
  DevBuf S[MGM_MAX_LEVELS], Y[MGM_MAX_LEVELS], Q[MGM_MAX_LEVELS];
  DevBuf Q2[MGM_MAX_LEVELS];  // second basis: the trial of the adaptive choice of d
  DevBuf Z[MGM_MAX_LEVELS], X[MGM_MAX_LEVELS], C[MGM_MAX_LEVELS];
  DevBuf ppart[MGM_MAX_LEVELS];  // partial coefficients of the projection
  // per-difference CholQR workspaces (the differences' QRs run concurrently)
  DevBuf qtmp[MGM_MAX_LEVELS], qG[MGM_MAX_LEVELS], qpart[MGM_MAX_LEVELS], qfail[MGM_MAX_LEVELS];
  // per operator level: the merged right-hand sides of one solve and its solutions
  DevBuf lin[MGM_MAX_LEVELS], lout[MGM_MAX_LEVELS];
};

struct Gauge {
  int Lx = 0, Lt = 0, anti = 1;
  double m0 = 0;
  DevBuf links;    // complex128 [2][Lt][Lx], t-boundary sign folded in
  DevBuf links32;  // complex64 copy
  std::vector<std::unique_ptr<Level>> levels;
  bool mg_ready = false;
  mgm_mg_params prm{};
  int mlmc_levels = 0;      // levels of the MLMC telescoping sum
  double trL[2] = {0, 0};   // tr(D^{-1}) of level mlmc_levels-1
  int tuned_block[MGM_MAX_LEVELS] = {0};  // autotuned RHS block per level
  // all work on this field runs on its own stream, ordered against the
  // caller's stream with ev_in / ev_out at every entry point
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // second and third streams of the field (default priority) for the
  // concurrent solves, with their fork / join events; created on first use
  hipStream_t stream2 = nullptr, stream3 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_join3 = nullptr;
  DevBuf scratch[3];  // split-k partials of the dense applies, per workspace set
  CnnWork cnn;
  EstWork est;
  std::map<GraphKey, GraphEntry> graphs[3];  // per workspace set (one host thread each)
  // the field's own worker context of mgm_trace_jobs, kept so that its
  // workspaces (and the graphs that hold their addresses) are reused
  std::shared_ptr<mgm_ctx> view;
  void clear_graphs() {
    for (auto& m : graphs) {
      for (auto& kv : m)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
      m.clear();
    }
  }
  ~Gauge() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (stream2) (void)hipStreamSynchronize(stream2);
    if (stream3) (void)hipStreamSynchronize(stream3);
    clear_graphs();
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_join3) (void)hipEventDestroy(ev_join3);
    if (stream) (void)hipStreamDestroy(stream);
    if (stream2) (void)hipStreamDestroy(stream2);
    if (stream3) (void)hipStreamDestroy(stream3);
  }
};

}  // namespace mgm

struct mgm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int wslot = 0;  // workspace set of the levels this view solves with (0, 1 or 2)
  std::string err;
  std::vector<std::unique_ptr<mgm::Gauge>> gauges;
  mgm::DevBuf scratch, scratch2, scratch3, ibuf;
  mgm::DevBuf qr_tmp, qr_G, qr_part, qr_fail;  // orthonormalize workspace
  std::shared_ptr<mgm::Cnn> cnn;  // shared with the per-field worker views
};

namespace mgm {
// host-side solver entry points (solver.hip)
void precondition_d(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* r, cd* x, const int* act);
int solve_level(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* b, cd* x,
                const mgm_solve_params& sp, int* iters_out, double* relres_out);
void apply_level(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* x, cd* y);
void precondition_graph(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* r, cd* x, const int* act);
int solve_chunked(mgm_ctx* c, Gauge& g, int l, int nrhs, const cd* b, cd* x,
                  const mgm_solve_params& sp, int* iters, double* relres);
void setup_hierarchy(mgm_ctx* c, Gauge& g, const mgm_mg_params& p);
void orthonormalize(mgm_ctx* c, int64_t n, int d, const cd* Y, cd* Q);
void orthonormalize_ws(hipStream_t s, int64_t n, int d, const cd* Y, cd* Q, cd* tmp, cd* G, cd* part,
                       int* fail);
// the same passes without the read-back: *fail (device) is set when the
// Gram matrix is not positive definite
void orthonormalize_launch(hipStream_t s, int64_t n, int d, const cd* Y, cd* Q, cd* tmp, cd* G, cd* part,
                           int* fail);
int trace_estimate(mgm_ctx* c, Gauge& g, const mgm_trace_params& p, mgm_trace_result& r);
// learned initial guess (cnn.hip)
void cnn_check_lattice(const Gauge& g);
void cnn_forward(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const float* x0, CnnWork& w,
                 float* y);
template <class TT>
const double* cnn_loss_grad(hipStream_t s, Cnn& net, const Gauge& g, int nb, const float* x0,
                            const TT* target, CnnWork& w);
void cnn_adam(hipStream_t s, Cnn& net, const mgm_adam_params& ap);
void cnn_to_channels(hipStream_t s, const cd* in, int64_t ndof, float* out);
void cnn_from_channels(hipStream_t s, const float* in, int64_t ndof, cd* out);
void cnn_apply(hipStream_t s, const Cnn& net, const Gauge& g, int nrhs, const cd* b, cd* y, CnnWork& w);
void cnn_initial_guess(mgm_ctx* c, Gauge& g, int nrhs, const cd* b, cd* x, cd* u);
void cnn_precondition(mgm_ctx* c, Gauge& g, int nrhs, const cd* v, cd* z, const int* act);
void cnn_time_conv(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const float* in, float* out);
void cnn_time_conv_h(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const _Float16* in,
                     _Float16* out);
}  // namespace mgm
