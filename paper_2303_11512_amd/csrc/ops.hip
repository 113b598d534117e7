// Level operators of the multigrid hierarchy on gfx950: the fine Schwinger
// (2D Wilson-Dirac, U(1)) stencil, the Galerkin block stencil of the coarse
// levels, restriction/prolongation, the SAP smoother, the coarsest dense
// inverse, and the counter-based noise.
//
// Vectors are complex [nrhs][n] with n = sites * M (M dofs per site, site
// index t * Nx + x).  The block stencil stores, per site u, five M x M blocks
// B[u][d] (d = 0 self, 1 +x, 2 -x, 3 +t, 4 -t) with
//     (D x)_u = sum_d B[u][d] x_{nb(u, d)},   periodic neighbours.
#include <algorithm>
#include <atomic>

#include "internal.h"

namespace mgm {

namespace {

constexpr int NT = 256;

// Site indices fit in 32 bits (the host limits lattices to 2^30 sites), so
// the division is done in 32-bit arithmetic: 64-bit division by a runtime
// value expands into a long branchy sequence.
__device__ __forceinline__ int64_t nb_site(int64_t u, int d, int Nx, int Nt) {
  const int ui = (int)u;
  int x = ui % Nx, t = ui / Nx;
  switch (d) {
    case 1: x = (x + 1 == Nx) ? 0 : x + 1; break;
    case 2: x = (x == 0) ? Nx - 1 : x - 1; break;
    case 3: t = (t + 1 == Nt) ? 0 : t + 1; break;
    case 4: t = (t == 0) ? Nt - 1 : t - 1; break;
    default: break;
  }
  return (int64_t)t * Nx + x;
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// ------------------------------------------------------------------ noise
// SplitMix64 counter stream: key = mix64(seed + golden) ^ purpose<<56 ^
// level<<48 ^ index; word_i = mix64(mix64(key) + (i+1) golden).  Bit 63 is the
// sign of the real part, bit 62 of the imaginary part.
template <class T>
__global__ void __launch_bounds__(NT) k_noise(cx<T>* out, int64_t n, int kind, uint64_t base,
                                              int purpose, int level, int64_t index0) {
  const int r = blockIdx.y;
  const uint64_t key = base ^ ((uint64_t)purpose << 56) ^ ((uint64_t)level << 48) ^
                       (uint64_t)(index0 + r);
  const uint64_t s0 = mix64(key);
  const T h = (T)0.70710678118654752440;  // sqrt(1/2)
  cx<T>* o = out + (int64_t)r * n;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    const uint64_t w = mix64(s0 + (uint64_t)(i + 1) * kGolden);
    const bool re_neg = (w >> 63) & 1ull;
    if (kind == MGM_NOISE_RADEMACHER) {
      o[i] = mk<T>(re_neg ? (T)-1 : (T)1, (T)0);
    } else {
      const bool im_neg = (w >> 62) & 1ull;
      o[i] = mk<T>(re_neg ? -h : h, im_neg ? -h : h);
    }
  }
}

// ------------------------------------------------------------------ fine Wilson
// (D psi)(x) = (m0+2) psi(x) - 1/2 sum_mu [(1 - sigma_mu) U_mu(x) psi(x+mu)
//              + (1 + sigma_mu) U_mu(x-mu)^* psi(x-mu)],
// sigma_0 = Pauli x, sigma_1 = Pauli y.  Each (1 -+ sigma_mu) has rank one, so
// every hop moves one complex number h (spin projection):
//   +x: h = c0 - c1, contributes (-h/2, +h/2) * U
//   -x: h = c0 + c1, contributes (-h/2, -h/2) * U^*
//   +t: h = c0 + i c1, contributes (-h/2, +i h/2) * U
//   -t: h = c0 - i c1, contributes (-h/2, -i h/2) * U^*
// The antiperiodic t boundary is folded into the links.  y = D x, or
// y = b - D x when b is given.
// One site: o = own spinor, e/w = +x/-x neighbours with the links ue (own)
// and uw (the -x neighbour's, conjugated inside), n/s = +t/-t neighbours with
// un (own) and us (the -t neighbour's).
template <class T>
__device__ __forceinline__ void wilson_site(T diag, cx<T> o0, cx<T> o1, cx<T> e0, cx<T> e1, cx<T> ue,
                                            cx<T> w0, cx<T> w1, cx<T> uw, cx<T> n0, cx<T> n1, cx<T> un,
                                            cx<T> s0, cx<T> s1, cx<T> us, cx<T>& a0, cx<T>& a1) {
  const T half = (T)0.5;
  a0 = diag * o0;
  a1 = diag * o1;
  {
    const cx<T> h = ue * (e0 - e1);
    a0 = a0 - half * h;
    a1 = a1 + half * h;
  }
  {
    const cx<T> h = cjmul(uw, w0 + w1);
    a0 = a0 - half * h;
    a1 = a1 - half * h;
  }
  {
    const cx<T> h = un * mk<T>(n0.re - n1.im, n0.im + n1.re);
    a0 = a0 - half * h;
    a1 = a1 + half * mk<T>(-h.im, h.re);
  }
  {
    const cx<T> h = cjmul(us, mk<T>(s0.re + s1.im, s0.im - s1.re));
    a0 = a0 - half * h;
    a1 = a1 - half * mk<T>(-h.im, h.re);
  }
}

// The output is written once and not read again by this kernel: streaming
// stores keep it from displacing the input's halo rows in L2.
template <class T>
__device__ __forceinline__ void store_stream(cx<T>* p, cx<T> v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.re;
  w.y = v.im;
  __builtin_nontemporal_store(w, reinterpret_cast<v2*>(p));
}

// Thread per site, for any lattice.  The (tile, RHS) grid is renumbered as a
// whole, so an XCD takes whole right-hand sides and their halos stay in its L2.
template <class T>
__global__ void __launch_bounds__(NT) k_wilson(const cx<T>* __restrict__ U, T diag, int Lx, int Lt,
                                               const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                               const cx<T>* __restrict__ b,
                                               const int* __restrict__ active) {
  const int64_t G = gridDim.x;
  const int64_t Lg = xcd_tile(blockIdx.x + G * blockIdx.y, G * gridDim.y);
  const int r = (int)(Lg / G);
  if (active && !active[r]) return;
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t site = (Lg % G) * NT + threadIdx.x;
  if (site >= V) return;
  const int xx = (int)(site % Lx), tt = (int)(site / Lx);
  const cx<T>* __restrict__ xr = x + (int64_t)r * 2 * V;
  const int64_t sxp = (int64_t)tt * Lx + (xx + 1 == Lx ? 0 : xx + 1);
  const int64_t sxm = (int64_t)tt * Lx + (xx == 0 ? Lx - 1 : xx - 1);
  const int64_t stp = (int64_t)(tt + 1 == Lt ? 0 : tt + 1) * Lx + xx;
  const int64_t stm = (int64_t)(tt == 0 ? Lt - 1 : tt - 1) * Lx + xx;
  cx<T> a0, a1;
  wilson_site<T>(diag, xr[2 * site], xr[2 * site + 1], xr[2 * sxp], xr[2 * sxp + 1], U[site],
                 xr[2 * sxm], xr[2 * sxm + 1], U[sxm], xr[2 * stp], xr[2 * stp + 1], U[V + site],
                 xr[2 * stm], xr[2 * stm + 1], U[V + stm], a0, a1);
  cx<T>* yr = y + (int64_t)r * 2 * V;
  if (b) {
    const cx<T>* br = b + (int64_t)r * 2 * V;
    a0 = br[2 * site] - a0;
    a1 = br[2 * site + 1] - a1;
  }
  store_stream(yr + 2 * site, a0);
  store_stream(yr + 2 * site + 1, a1);
}

// Row strips for lattices whose rows split into 64-multiple pieces of at most
// 256 sites: a workgroup of Lx / SPT threads (thread = SPT columns, blockDim
// apart, so each column slice of a row is one coalesced segment) walks TR
// consecutive time slices of one RHS.
// Each spinor is loaded from global memory once per strip (plus the two rows
// bordering it): the rows behind, at and ahead of the current one roll
// through registers, and the +-x neighbours of the current row come from a
// double-buffered LDS row, so one barrier per row suffices (a buffer is
// rewritten two rows later, after every thread has passed the barrier in
// between).  Even strips walk up in t and odd strips down, so the two rows on
// each strip boundary are read by both neighbouring strips at the same phase
// (both at the start or both at the end) and the second read hits L2.
template <class T, int TR, int SPT>
__global__ void __launch_bounds__(NT) k_wilson_strip(const cx<T>* __restrict__ U, T diag, int Lx, int Lt,
                                                     const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                     const cx<T>* __restrict__ b,
                                                     const int* __restrict__ active) {
  __shared__ cx<T> sx[2][2][NT * SPT];
  __shared__ cx<T> su[2][NT * SPT];
  const int64_t G = gridDim.x;
  const int64_t NR = gridDim.y;
  const int64_t Lg = xcd_tile(blockIdx.x + G * blockIdx.y, G * NR);
  // RHS fastest: the strips an XCD holds at once share rows of the links
  const int r = (int)(Lg % NR);
  const int strip = (int)(Lg / NR);
  if (active && !active[r]) return;
  const int64_t V = (int64_t)Lx * Lt;
  const int BD = blockDim.x;
  int xs[SPT], xp[SPT], xm[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    xs[j] = threadIdx.x + j * BD;
    xp[j] = xs[j] + 1 == Lx ? 0 : xs[j] + 1;
    xm[j] = xs[j] == 0 ? Lx - 1 : xs[j] - 1;
  }
  const cx<T>* __restrict__ xr = x + (int64_t)r * 2 * V;
  const cx<T>* __restrict__ U1 = U + V;
  cx<T>* __restrict__ yr = y + (int64_t)r * 2 * V;
  const bool up = (strip & 1) == 0;
  const int dir = up ? 1 : -1;
  auto wrap = [Lt](int t) { return t < 0 ? t + Lt : (t >= Lt ? t - Lt : t); };
  const int tf = up ? strip * TR : strip * TR + TR - 1;  // first row walked
  const int tb = wrap(tf - dir);
  // rows behind (t - dir) and at t; ur is U1 of the row below the current
  // one when walking up, of the current row when walking down
  cx<T> h0[SPT], h1[SPT], c0[SPT], c1[SPT], ur[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    h0[j] = xr[2 * ((int64_t)tb * Lx + xs[j])];
    h1[j] = xr[2 * ((int64_t)tb * Lx + xs[j]) + 1];
    c0[j] = xr[2 * ((int64_t)tf * Lx + xs[j])];
    c1[j] = xr[2 * ((int64_t)tf * Lx + xs[j]) + 1];
    ur[j] = U1[(int64_t)(up ? tb : tf) * Lx + xs[j]];
  }
#pragma unroll 2
  for (int i = 0; i < TR; ++i) {
    const int t = tf + dir * i;
    const int ta = wrap(t + dir);
    const int bs = i & 1;
    cx<T> a0x[SPT], a1x[SPT], ul[SPT], u0[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      a0x[j] = xr[2 * ((int64_t)ta * Lx + xs[j])];
      a1x[j] = xr[2 * ((int64_t)ta * Lx + xs[j]) + 1];
      ul[j] = U1[(int64_t)(up ? t : ta) * Lx + xs[j]];
      u0[j] = U[(int64_t)t * Lx + xs[j]];
      sx[bs][0][xs[j]] = c0[j];
      sx[bs][1][xs[j]] = c1[j];
      su[bs][xs[j]] = u0[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int64_t site = (int64_t)t * Lx + xs[j];
      cx<T> a0, a1;
      wilson_site<T>(diag, c0[j], c1[j], sx[bs][0][xp[j]], sx[bs][1][xp[j]], u0[j], sx[bs][0][xm[j]],
                     sx[bs][1][xm[j]], su[bs][xm[j]], up ? a0x[j] : h0[j], up ? a1x[j] : h1[j],
                     up ? ul[j] : ur[j], up ? h0[j] : a0x[j], up ? h1[j] : a1x[j], up ? ur[j] : ul[j], a0, a1);
      if (b) {
        const cx<T>* br = b + (int64_t)r * 2 * V;
        a0 = br[2 * site] - a0;
        a1 = br[2 * site + 1] - a1;
      }
      store_stream(yr + 2 * site, a0);
      store_stream(yr + 2 * site + 1, a1);
      h0[j] = c0[j];
      h1[j] = c1[j];
      c0[j] = a0x[j];
      c1[j] = a1x[j];
      ur[j] = ul[j];
    }
  }
}

// The fine operator written as a block stencil (2x2 blocks), for the setup.
__global__ void __launch_bounds__(NT) k_fine_blocks(const cd* __restrict__ U, double diag, int Lx,
                                                    int Lt, cd* __restrict__ B) {
  const int64_t V = (int64_t)Lx * Lt;
  const int64_t u = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (u >= V) return;
  const cd* U0 = U;
  const cd* U1 = U + V;
  cd* o = B + u * 20;  // [5][2][2]
  const cd z = mk(0.0, 0.0);
  // self
  o[0] = mk(diag, 0.0); o[1] = z; o[2] = z; o[3] = mk(diag, 0.0);
  // +x: -1/2 U [[1,-1],[-1,1]]
  {
    const cd h = -0.5 * U0[u];
    o[4] = h; o[5] = -1.0 * h; o[6] = -1.0 * h; o[7] = h;
  }
  // -x: -1/2 U(u-x)^* [[1,1],[1,1]]
  {
    const cd h = -0.5 * conj(U0[nb_site(u, 2, Lx, Lt)]);
    o[8] = h; o[9] = h; o[10] = h; o[11] = h;
  }
  // +t: -1/2 U [[1, i],[-i, 1]]
  {
    const cd h = -0.5 * U1[u];
    o[12] = h; o[13] = mk(-h.im, h.re); o[14] = mk(h.im, -h.re); o[15] = h;
  }
  // -t: -1/2 U(u-t)^* [[1, -i],[i, 1]]
  {
    const cd h = -0.5 * conj(U1[nb_site(u, 4, Lx, Lt)]);
    o[16] = h; o[17] = mk(h.im, -h.re); o[18] = mk(-h.im, h.re); o[19] = h;
  }
}

// ------------------------------------------------------------------ block stencil
// One thread per (site, row i); blockIdx.y = RHS.
template <class T, int M>
__global__ void __launch_bounds__(NT) k_stencil(const cx<T>* __restrict__ B, int Nx, int Nt,
                                                const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                const cx<T>* __restrict__ b,
                                                const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t sites = (int64_t)Nx * Nt;
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= sites * M) return;
  const int64_t u = idx / M;
  const int i = (int)(idx % M);
  const int64_t n = sites * M;
  const cx<T>* __restrict__ xr = x + (int64_t)r * n;
  cx<T> acc = mk<T>(0, 0);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    const cx<T>* __restrict__ row = B + ((u * 5 + d) * M + i) * M;
    const cx<T>* __restrict__ xv = xr + nb_site(u, d, Nx, Nt) * M;
#pragma unroll
    for (int j = 0; j < M; ++j) cfma(acc, row[j], xv[j]);
  }
  if (b) acc = b[(int64_t)r * n + idx] - acc;
  y[(int64_t)r * n + idx] = acc;
}

// Coarse levels: one workgroup per site and up to `rpc` RHS.  The site's five
// M x M blocks are staged once in LDS, transposed ([d][j][i]) so that the M
// lanes computing rows i of one RHS read consecutive words; x is read with a
// broadcast across those lanes.  256/M RHS per round.
template <class T, int M>
__global__ void __launch_bounds__(NT) k_stencil_lds(const cx<T>* __restrict__ B, int Nx, int Nt,
                                                    int nrhs, int rpc, const cx<T>* __restrict__ x,
                                                    cx<T>* __restrict__ y, const cx<T>* __restrict__ b,
                                                    const int* __restrict__ active) {
  constexpr int RPW = NT / M;
  __shared__ cx<T> BT[5 * M * M];
  __shared__ cx<T> XS[RPW * 5 * M];  // the five neighbour sites' dofs of RPW RHS
  const int tid = threadIdx.x;
  const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
  for (int e = tid; e < 5 * M * M; e += NT) {
    const int j = e % M, i = (e / M) % M, d = e / (M * M);
    BT[(d * M + j) * M + i] = B[u * 5 * M * M + e];
  }
  const int i = tid % M, rl = tid / M;
  const int64_t n = (int64_t)Nx * Nt * M;
  int64_t nbs[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) nbs[d] = nb_site(u, d, Nx, Nt) * M;
  const int rbeg = blockIdx.y * rpc;
  const int rend = min(nrhs, rbeg + rpc);
  for (int r0 = rbeg; r0 < rend; r0 += RPW) {
    // cooperative, row-contiguous load of the neighbour dofs of this round's RHS
    for (int e = tid; e < RPW * 5 * M; e += NT) {
      const int j = e % M, d = (e / M) % 5, rr = e / (5 * M);
      const int r = r0 + rr;
      XS[e] = x[(int64_t)(r < rend ? r : rbeg) * n + nbs[d] + j];  // rows past rend are never used
    }
    __syncthreads();
    const int r = r0 + rl;
    if (r < rend && (!active || active[r])) {
      const cx<T>* xs = XS + rl * 5 * M;
      cx<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        const cx<T>* bt = BT + d * M * M + i;
#pragma unroll
        for (int j = 0; j < M; ++j) cfma(acc, bt[j * M], xs[d * M + j]);
      }
      const int64_t o = (int64_t)r * n + u * M + i;
      if (b) acc = b[o] - acc;
      y[o] = acc;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ restriction / prolongation
// P[A][c][s][k]: row s of aggregate A, chirality c -- site sl = s / Mh of the
// aggregate (t-major), dof c*Mh + s % Mh of that site; column k.
__device__ __forceinline__ int64_t agg_row(int64_t A, int c, int s, int Nx, int M, int bx, int bt,
                                           int NAx) {
  const int Mh = M / 2;
  const int sl = s / Mh, a = s % Mh;
  const int dx = sl % bx, dt = sl / bx;
  const int Ax = (int)(A % NAx), At = (int)(A / NAx);
  const int64_t site = (int64_t)(At * bt + dt) * Nx + (Ax * bx + dx);
  return site * M + c * Mh + a;
}

template <class T>
__global__ void __launch_bounds__(NT) k_restrict(const cx<T>* __restrict__ P, int Nx, int Nt, int M,
                                                 int bx, int bt, int ntv, const cx<T>* __restrict__ xf,
                                                 cx<T>* __restrict__ xc,
                                                 const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int NAx = Nx / bx;
  const int64_t nagg = (int64_t)NAx * (Nt / bt);
  const int64_t nc = nagg * 2 * ntv;
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= nc) return;
  const int64_t A = idx / (2 * ntv);
  const int c = (int)((idx / ntv) % 2);
  const int k = (int)(idx % ntv);
  const int nrow = bx * bt * (M / 2);
  const cx<T>* __restrict__ xr = xf + (int64_t)r * Nx * Nt * M;
  const cx<T>* __restrict__ Pc = P + ((A * 2 + c) * nrow) * ntv + k;
  cx<T> acc = mk<T>(0, 0);
  for (int s = 0; s < nrow; ++s) cjfma(acc, Pc[(int64_t)s * ntv], xr[agg_row(A, c, s, Nx, M, bx, bt, NAx)]);
  xc[(int64_t)r * nc + idx] = acc;
}

template <class T>
__global__ void __launch_bounds__(NT) k_prolong(const cx<T>* __restrict__ P, int Nx, int Nt, int M,
                                                int bx, int bt, int ntv, const cx<T>* __restrict__ xc,
                                                cx<T>* __restrict__ yf, int accumulate,
                                                const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t n = (int64_t)Nx * Nt * M;
  const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  const int NAx = Nx / bx;
  const int64_t nc = (int64_t)NAx * (Nt / bt) * 2 * ntv;
  const int Mh = M / 2;
  const int64_t site = row / M;
  const int alpha = (int)(row % M);
  const int c = alpha / Mh, a = alpha % Mh;
  const int sx = (int)(site % Nx), st = (int)(site / Nx);
  const int64_t A = (int64_t)(st / bt) * NAx + sx / bx;
  const int sl = (st % bt) * bx + (sx % bx);
  const int s = sl * Mh + a;
  const int nrow = bx * bt * Mh;
  const cx<T>* __restrict__ Pr = P + ((A * 2 + c) * nrow + s) * ntv;
  const cx<T>* __restrict__ xv = xc + (int64_t)r * nc + (A * 2 + c) * ntv;
  cx<T> acc = mk<T>(0, 0);
  for (int k = 0; k < ntv; ++k) cfma(acc, Pr[k], xv[k]);
  cx<T>* o = yf + (int64_t)r * n + row;
  *o = accumulate ? (*o + acc) : acc;
}

// right-hand sides per restriction thread (measured: 4 / 2 beat 2 / 1 and 8 / 2)
constexpr int RT_RESTRICT_FINE = 4;    // 2-dof sites in 4x4 aggregates
constexpr int RT_RESTRICT_COARSE = 2;  // 16-dof sites in 2x2 aggregates

// The same two maps for a hierarchy shape fixed at compile time (M dofs per
// site, BX x BT aggregates, NTV test vectors per chirality).  Every index is a
// shift or a multiply and the row loop is unrolled, so a thread issues all of
// its loads at once instead of one dependent round trip per aggregate row;
// the generic kernels above are latency bound for exactly that reason.
// BLK: xf in the block-major layout of the fine FP32 cycle (the BX x BT
// aggregate's sites t-major, then dofs, contiguous per aggregate).
// RT right-hand sides per thread (blockIdx.y: RHS r0 = RT blockIdx.y ..):
// the thread's P column is loaded once for all of them.
template <class T, int M, int BX, int BT, int NTV, bool BLK = false, int RT = 1>
__global__ void __launch_bounds__(NT) k_restrict_t(const cx<T>* __restrict__ P, int Nx, int Nt,
                                                   const cx<T>* __restrict__ xf, cx<T>* __restrict__ xc,
                                                   const int* __restrict__ active, int nrhs) {
  constexpr int Mh = M / 2, NROW = BX * BT * Mh;
  const int r0 = blockIdx.y * RT;
  const int NAx = Nx / BX;
  const int64_t nc = (int64_t)NAx * (Nt / BT) * 2 * NTV;
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= nc) return;
  const int64_t Ac = idx / NTV;  // aggregate * 2 + chirality
  const int k = (int)(idx % NTV);
  const int64_t A = Ac / 2;
  const int c = (int)(Ac % 2);
  const int Ax = (int)(A % NAx), At = (int)(A / NAx);
  const int64_t nf = (int64_t)Nx * Nt * M;
  const cx<T>* __restrict__ xa = BLK ? xf + A * (BX * BT * M) + c * Mh
                                     : xf + ((int64_t)At * BT * Nx + (int64_t)Ax * BX) * M + c * Mh;
  const cx<T>* __restrict__ Pc = P + Ac * NROW * NTV + k;
  cx<T> pv[NROW], xv[RT][NROW];
  bool on[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int r = r0 + rt;
    on[rt] = r < nrhs && (!active || active[r]);
    const cx<T>* __restrict__ xr = xa + (int64_t)(r < nrhs ? r : r0) * nf;  // lanes past nrhs: never stored
#pragma unroll
    for (int s = 0; s < NROW; ++s) {
      const int sl = s / Mh, a = s % Mh;
      xv[rt][s] = BLK ? xr[sl * M + a] : xr[((int64_t)(sl / BX) * Nx + sl % BX) * M + a];
    }
  }
#pragma unroll
  for (int s = 0; s < NROW; ++s) pv[s] = Pc[s * NTV];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    cx<T> acc = mk<T>(0, 0);
#pragma unroll
    for (int s = 0; s < NROW; ++s) cjfma(acc, pv[s], xv[rt][s]);
    if (on[rt]) xc[(int64_t)(r0 + rt) * nc + idx] = acc;
  }
}

template <class T, int M, int BX, int BT, int NTV, bool BLK = false>
__global__ void __launch_bounds__(NT) k_prolong_t(const cx<T>* __restrict__ P, int Nx, int Nt,
                                                  const cx<T>* __restrict__ xc, cx<T>* __restrict__ yf,
                                                  int accumulate, const int* __restrict__ active) {
  constexpr int Mh = M / 2, NROW = BX * BT * Mh;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t n = (int64_t)Nx * Nt * M;
  const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  const int NAx = Nx / BX;
  const int64_t nc = (int64_t)NAx * (Nt / BT) * 2 * NTV;
  int64_t Ac;
  int s;
  if (BLK) {  // row = aggregate * BX BT M + sl M + alpha
    const int64_t A = row / (BX * BT * M);
    const int q = (int)(row % (BX * BT * M)), alpha = q % M;
    Ac = A * 2 + alpha / Mh;
    s = (q / M) * Mh + alpha % Mh;
  } else {
    const int64_t site = row / M;
    const int alpha = (int)(row % M);
    const int c = alpha / Mh, a = alpha % Mh;
    const int sx = (int)(site % Nx), st = (int)(site / Nx);
    Ac = ((int64_t)(st / BT) * NAx + sx / BX) * 2 + c;
    s = ((st % BT) * BX + (sx % BX)) * Mh + a;
  }
  const cx<T>* __restrict__ Pr = P + (Ac * NROW + s) * NTV;
  const cx<T>* __restrict__ xv = xc + (int64_t)r * nc + Ac * NTV;
  cx<T> pv[NTV], cv[NTV];
#pragma unroll
  for (int k = 0; k < NTV; ++k) {
    pv[k] = Pr[k];
    cv[k] = xv[k];
  }
  cx<T>* o = yf + (int64_t)r * n + row;
  cx<T> acc = accumulate ? *o : mk<T>(0, 0);
#pragma unroll
  for (int k = 0; k < NTV; ++k) cfma(acc, pv[k], cv[k]);
  *o = acc;
}

// ------------------------------------------------------------------ Galerkin
// Bc[A][D][I][J] = sum over hops (u, d) of aggregate A that land in the
// aggregate nbA(A, D) (D = 0: hops that stay inside A, including the self
// block) of conj(P_A[u, I]) Bf[u][d] P_{nbA}[v, J],  v = nb(u, d).
__global__ void __launch_bounds__(NT) k_galerkin(const cd* __restrict__ Bf, int Nx, int Nt, int Mf,
                                                 const cd* __restrict__ P, int bx, int bt, int ntv,
                                                 cd* __restrict__ Bc) {
  const int Mc = 2 * ntv;
  const int NAx = Nx / bx, NAt = Nt / bt;
  const int64_t nagg = (int64_t)NAx * NAt;
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= nagg * 5 * Mc * Mc) return;
  const int J = (int)(idx % Mc);
  const int I = (int)((idx / Mc) % Mc);
  const int D = (int)((idx / (Mc * Mc)) % 5);
  const int64_t A = idx / (5 * Mc * Mc);
  const int c = I / ntv, k = I % ntv, c2 = J / ntv, k2 = J % ntv;
  const int Ax = (int)(A % NAx), At = (int)(A / NAx);
  int Bx = Ax, Bt = At;
  if (D == 1) Bx = (Ax + 1 == NAx) ? 0 : Ax + 1;
  if (D == 2) Bx = (Ax == 0) ? NAx - 1 : Ax - 1;
  if (D == 3) Bt = (At + 1 == NAt) ? 0 : At + 1;
  if (D == 4) Bt = (At == 0) ? NAt - 1 : At - 1;
  const int64_t An = (int64_t)Bt * NAx + Bx;
  const int Mh = Mf / 2;
  const int nrow = bx * bt * Mh;
  const cd* __restrict__ PA = P + (A * 2 + c) * nrow * ntv;
  const cd* __restrict__ PB = P + (An * 2 + c2) * nrow * ntv;
  cd acc = mk(0.0, 0.0);
  for (int dt = 0; dt < bt; ++dt) {
    for (int dx = 0; dx < bx; ++dx) {
      const int64_t u = (int64_t)(At * bt + dt) * Nx + (Ax * bx + dx);
      const int sl = dt * bx + dx;
      for (int d = 0; d < 5; ++d) {
        int route = 0;
        if (d == 1 && dx == bx - 1) route = 1;
        if (d == 2 && dx == 0) route = 2;
        if (d == 3 && dt == bt - 1) route = 3;
        if (d == 4 && dt == 0) route = 4;
        if (route != D) continue;
        const int64_t v = nb_site(u, d, Nx, Nt);
        const int vsl = (int)((v / Nx) % bt) * bx + (int)((v % Nx) % bx);
        const cd* __restrict__ Bud = Bf + (u * 5 + d) * Mf * Mf;
        for (int a = 0; a < Mh; ++a) {
          const cd pu = PA[(int64_t)(sl * Mh + a) * ntv + k];
          cd t = mk(0.0, 0.0);
          for (int bb = 0; bb < Mh; ++bb) {
            const cd pv = PB[(int64_t)(vsl * Mh + bb) * ntv + k2];
            cfma(t, Bud[(int64_t)(c * Mh + a) * Mf + c2 * Mh + bb], pv);
          }
          cjfma(acc, pu, t);
        }
      }
    }
  }
  Bc[idx] = acc;
}

// ------------------------------------------------------------------ SAP blocks
// D restricted to each sbx x sbt block of sites (local dof q = sl * M + alpha,
// sl = dt * sbx + dx): out[blk][q][q'] = sum_{d : nb(u_q, d) = u_q'} B[u_q][d].
__global__ void __launch_bounds__(NT) k_sap_extract(const cd* __restrict__ B, int Nx, int Nt, int M,
                                                    int sbx, int sbt, cd* __restrict__ out) {
  const int K = sbx * sbt * M;
  const int NBx = Nx / sbx;
  const int64_t nblk = (int64_t)NBx * (Nt / sbt);
  const int64_t idx = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (idx >= nblk * K * K) return;
  const int q2 = (int)(idx % K);
  const int q = (int)((idx / K) % K);
  const int64_t blk = idx / ((int64_t)K * K);
  const int ibx = (int)(blk % NBx), ibt = (int)(blk / NBx);
  const int sl = q / M, al = q % M, sl2 = q2 / M, be = q2 % M;
  const int64_t u = (int64_t)(ibt * sbt + sl / sbx) * Nx + ibx * sbx + sl % sbx;
  const int64_t u2 = (int64_t)(ibt * sbt + sl2 / sbx) * Nx + ibx * sbx + sl2 % sbx;
  cd acc = mk(0.0, 0.0);
  for (int d = 0; d < 5; ++d)
    if (nb_site(u, d, Nx, Nt) == u2) acc = acc + B[((u * 5 + d) * M + al) * M + be];
  out[idx] = acc;
}

// Gauss-Jordan inverse with partial pivoting of `count` K x K matrices in LDS
// (one workgroup per matrix, K <= KMAX).  Sets *fail on a zero pivot.
template <int KMAX>
__global__ void __launch_bounds__(NT) k_small_inverse(cd* __restrict__ mats, int K,
                                                      int* __restrict__ fail) {
  __shared__ cd A[KMAX * KMAX];
  __shared__ cd fcol[KMAX];
  __shared__ int perm[KMAX];
  __shared__ cd pivinv;
  __shared__ int prow;
  const int tid = threadIdx.x;
  cd* g = mats + (int64_t)blockIdx.x * K * K;
  for (int e = tid; e < K * K; e += NT) A[e] = g[e];
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    if (tid == 0) {
      int p = k;
      double best = abs2(A[k * K + k]);
      for (int i = k + 1; i < K; ++i) {
        const double v = abs2(A[i * K + k]);
        if (v > best) { best = v; p = i; }
      }
      perm[k] = p;
      prow = p;
      if (best == 0.0) {
        *fail = 1;
        pivinv = mk(0.0, 0.0);
      } else {
        pivinv = cdiv(mk(1.0, 0.0), A[p * K + k]);
      }
    }
    __syncthreads();
    const int p = prow;
    for (int j = tid; j < K; j += NT) {
      const cd vk = A[k * K + j], vp = A[p * K + j];
      if (p != k) A[p * K + j] = vk;
      A[k * K + j] = ((j == k) ? mk(1.0, 0.0) : vp) * pivinv;
    }
    __syncthreads();
    for (int i = tid; i < K; i += NT) fcol[i] = (i == k) ? mk(0.0, 0.0) : A[i * K + k];
    __syncthreads();
    for (int e = tid; e < K * K; e += NT) {
      const int i = e / K, j = e % K;
      if (i == k) continue;
      const cd base = (j == k) ? mk(0.0, 0.0) : A[e];
      A[e] = base - fcol[i] * A[k * K + j];
    }
    __syncthreads();
  }
  for (int k = K - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {
      for (int i = tid; i < K; i += NT) {
        const cd t = A[i * K + k];
        A[i * K + k] = A[i * K + p];
        A[i * K + p] = t;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < K * K; e += NT) g[e] = A[e];
}

// One colour of the red/black Schwarz sweep with exact block solves:
//   res_B = r_B - (D x)_B ;  x_B += inv_B res_B
// for every listed block B.  K = sbx*sbt*M dofs per block.  A workgroup owns
// one block and `rpc` RHS: it stages the block inverse and the block's rows
// of the stencil in LDS once (transposed, so that lanes of a wave read
// consecutive words) and then sweeps its RHS 256/K at a time.
constexpr int SAP_INV_MAX = 1024;   // K <= 32
constexpr int SAP_B_MAX = 1280;     // sites_in_block * 5 * M * M staged in LDS
template <class T>
__global__ void __launch_bounds__(NT) k_sap_sweep(const cx<T>* __restrict__ B,
                                                  const cx<T>* __restrict__ inv, int Nx, int Nt, int M,
                                                  int sbx, int sbt, const int* __restrict__ blist,
                                                  int nrhs, int rpc, const cx<T>* __restrict__ rr,
                                                  cx<T>* __restrict__ x,
                                                  const int* __restrict__ active) {
  __shared__ cx<T> invT[SAP_INV_MAX];
  __shared__ cx<T> BT[SAP_B_MAX];
  __shared__ cx<T> res[NT];
  const int nsb = sbx * sbt;
  const int K = nsb * M;
  const int rpw = NT / K;
  const int tid = threadIdx.x;
  const int q = tid % K, rl = tid / K;
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int NBx = Nx / sbx;
  const int ibx = blk % NBx, ibt = blk / NBx;
  // stage inv^T and the block's stencil rows (B^T per direction)
  for (int e = tid; e < K * K; e += NT) {
    const int q1 = e / K, q2 = e % K;
    invT[q2 * K + q1] = inv[((int64_t)blk * K + q1) * K + q2];
  }
  const int nbe = nsb * 5 * M * M;
  const bool staged = nbe <= SAP_B_MAX;
  if (staged) {
    for (int e = tid; e < nbe; e += NT) {
      const int b = e % M, a = (e / M) % M, d = (e / (M * M)) % 5, s = e / (5 * M * M);
      const int64_t us = (int64_t)(ibt * sbt + s / sbx) * Nx + ibx * sbx + s % sbx;
      BT[((s * 5 + d) * M + b) * M + a] = B[((us * 5 + d) * M + a) * M + b];
    }
  }
  __syncthreads();
  const int sl = q / M, al = q % M;
  const int64_t u = (int64_t)(ibt * sbt + sl / sbx) * Nx + ibx * sbx + sl % sbx;
  const int64_t n = (int64_t)Nx * Nt * M;
  int64_t nbs[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) nbs[d] = nb_site(u, d, Nx, Nt) * M;
  const int rbeg = blockIdx.y * rpc;
  const int rend = min(nrhs, rbeg + rpc);
  for (int r0 = rbeg; r0 < rend; r0 += rpw) {
    const int r = r0 + rl;
    const bool valid = rl < rpw && r < rend && (!active || active[r]);
    if (valid) {
      const cx<T>* __restrict__ xr = x + (int64_t)r * n;
      cx<T> acc = rr[(int64_t)r * n + u * M + al];
      for (int d = 0; d < 5; ++d) {
        const cx<T>* __restrict__ xv = xr + nbs[d];
        cx<T> t = mk<T>(0, 0);
        if (staged) {
          const cx<T>* bt = BT + (sl * 5 + d) * M * M + al;
          for (int j = 0; j < M; ++j) cfma(t, bt[j * M], xv[j]);
        } else {
          const cx<T>* __restrict__ row = B + ((u * 5 + d) * M + al) * M;
          for (int j = 0; j < M; ++j) cfma(t, row[j], xv[j]);
        }
        acc = acc - t;
      }
      res[tid] = acc;
    }
    __syncthreads();
    if (valid) {
      const cx<T>* rs = res + rl * K;
      cx<T> acc = mk<T>(0, 0);
      for (int j = 0; j < K; ++j) cfma(acc, invT[j * K + q], rs[j]);
      cx<T>* o = x + (int64_t)r * n + u * M + al;
      *o = *o + acc;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ coarse levels on the matrix cores
// Levels with 16 dofs per site (8 test vectors x 2 chiralities).  A wave owns
// a 16 (dofs) x 16 (RHS) complex tile; a complex product is four real MFMAs.
// In K-chunk c, lane l takes the K index kc(l, c) = out_row(l, c), so that the
// result tile of one product (element c of a lane = row kc(l, c)) is already
// the B operand of the next one, with no shuffle.
constexpr int CM = 16;

// acc += B_d x_{nb(u, d)} for one direction d and the RHS column of this lane
// (zero operand for lanes past the last RHS); the block is read straight from
// the stencil B [site][5][16][16] (row-major) as the MFMA A operand.
template <class T>
__device__ __forceinline__ void coarse_hop(const cx<T>* __restrict__ B, const cx<T>* __restrict__ x,
                                           int64_t n, int64_t u, int d, int Nx, int Nt, int64_t rrow,
                                           bool ok, int lane, CAcc<T>& acc) {
  const int i = lane & 15;
  const cx<T>* xv = x + rrow * n + nb_site(u, d, Nx, Nt) * CM;
  const cx<T>* Bd = B + ((u * 5 + d) * CM + i) * CM;
  cx<T> a[4], xb[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int k = MF<T>::out_row(lane, c);
    a[c] = Bd[k];
    xb[c] = xv[k];  // lanes past the last RHS read row rrow; their column is never stored
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) cmma(a[c], xb[c], acc);
}

// Sum the partial tiles of waves 1..3 into wave 0 (LDS); returns false on
// the waves that are done.
template <class T>
__device__ __forceinline__ bool reduce_waves(CAcc<T>& acc, T (*red)[8][64], int wave, int lane) {
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[wave - 1][v][lane] = acc.re[v];
      red[wave - 1][4 + v][lane] = acc.im[v];
    }
  }
  __syncthreads();
  if (wave > 0) return false;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc.re[v] += red[w][v][lane];
      acc.im[v] += red[w][4 + v][lane];
    }
  return true;
}

// y = D x or y = b - D x on a coarse level (16 dofs per site).  One workgroup
// per (site, 16 RHS).  The product is 5 blocks x 4 K-chunks = 20 chunk
// products; wave w takes chunks 5w .. 5w+4 (in (direction, chunk) order), so
// the four waves carry equal matrix-core work, and the partial tiles are
// summed in LDS.
template <class T>
__global__ void __launch_bounds__(NT) k_stencil_mfma(const cx<T>* __restrict__ B, int Nx, int Nt, int nrhs,
                                                     const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
                                                     const cx<T>* __restrict__ b,
                                                     const int* __restrict__ active) {
  constexpr int QW = 5;  // chunk products per wave
  __shared__ T red[3][8][64];
  const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  cx<T> a[QW], xq[QW];
#pragma unroll
  for (int q = 0; q < QW; ++q) {
    const int g = wave * QW + q, d = g >> 2;
    const int k = MF<T>::out_row(lane, g & 3);
    a[q] = B[((u * 5 + d) * CM + i) * CM + k];
    xq[q] = x[rrow * n + nb_site(u, d, Nx, Nt) * CM + k];
  }
  CAcc<T> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int q = 0; q < QW; ++q) cmma(a[q], xq[q], acc);
  if (!reduce_waves(acc, red, wave, lane)) return;
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t o = (int64_t)r * n + u * CM + MF<T>::out_row(lane, v);
    const cx<T> val = mk<T>(acc.re[v], acc.im[v]);
    y[o] = b ? b[o] - val : val;
  }
}

// One colour of the coarse SAP sweep with one-site blocks: for each site u of
// the colour and each RHS, x_u = inv_u (r_u - sum_{d > 0} B_d x_{nb(u, d)}),
// which equals x_u + inv_u (r - D x)_u for the exact inverse of the self block.
// One workgroup per (site, 16 RHS): wave w takes the hop in direction w + 1,
// wave 0 sums them (LDS) and applies inv_u.
template <class T>
__global__ void __launch_bounds__(NT) k_sap_mfma(const cx<T>* __restrict__ B, const cx<T>* __restrict__ inv,
                                                 int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                 const cx<T>* __restrict__ rr, cx<T>* __restrict__ x,
                                                 const int* __restrict__ active) {
  __shared__ T red[3][8][64];
  const int64_t u = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<T> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  coarse_hop(B, x, n, u, wave + 1, Nx, Nt, rrow, ok, lane, acc);
  // the block solve's operands, loaded after the hops
  cx<T> rv[4], a[4];
  if (wave == 0) {
    const cx<T>* Iu = inv + (u * CM + i) * CM;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = MF<T>::out_row(lane, c);
      rv[c] = rr[rrow * n + u * CM + k];
      a[c] = Iu[k];
    }
  }
  if (!reduce_waves(acc, red, wave, lane)) return;
  // t = r_u - (hops) in the result layout: element c = row out_row(lane, c)
  cx<T> t[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) t[c] = mk<T>(rv[c].re - acc.re[c], rv[c].im - acc.im[c]);
  CAcc<T> cor{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int c = 0; c < 4; ++c) cmma(a[c], t[c], cor);
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    x[(int64_t)r * n + u * CM + MF<T>::out_row(lane, v)] = mk<T>(cor.re[v], cor.im[v]);
}

// ---- FP16 blocks: one 16x16x16 FP16 MFMA covers a whole 16 x 16 block.
// Lane l supplies A[l%16][4(l/16) + j] and B[4(l/16) + j][l%16] (j = 0..3);
// element v of its FP32 result is D[4(l/16) + v][l%16] (measured on gfx950).
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

// Sixteen complex zeros: the x operand of an unused hop slot.
__device__ const cf zero_cf[16] = {};

__device__ __forceinline__ void hmma(h4 ar, h4 ai, h4 br, h4 bi, CAcc<float>& acc) {
  acc.re = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, br, acc.re, 0, 0, 0);
  acc.re = __builtin_amdgcn_mfma_f32_16x16x16f16(-ai, bi, acc.re, 0, 0, 0);
  acc.im = __builtin_amdgcn_mfma_f32_16x16x16f16(ar, bi, acc.im, 0, 0, 0);
  acc.im = __builtin_amdgcn_mfma_f32_16x16x16f16(ai, br, acc.im, 0, 0, 0);
}

// acc += B_d x_{nb(u, d)} with the block in FP16 and x rounded to FP16
__device__ __forceinline__ void coarse_hop_h(const chalf* __restrict__ B, const cf* __restrict__ x, int64_t n,
                                             int64_t u, int d, int Nx, int Nt, int64_t rrow, bool ok, int lane,
                                             CAcc<float>& acc) {
  const int i = lane & 15, q = lane >> 4;
  const chalf* row = B + ((u * 5 + d) * CM + i) * CM + 4 * q;
  const cf* xv = x + rrow * n + nb_site(u, d, Nx, Nt) * CM + 4 * q;
  h4 ar, ai, br, bi;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const chalf a = row[j];
    const cf v = xv[j];
    ar[j] = a.re;
    ai[j] = a.im;
    br[j] = (_Float16)v.re;
    bi[j] = (_Float16)v.im;
  }
  hmma(ar, ai, br, bi, acc);
}

__global__ void __launch_bounds__(NT) k_stencil_h(const chalf* __restrict__ B, int Nx, int Nt, int nrhs,
                                                  const cf* __restrict__ x, cf* __restrict__ y,
                                                  const cf* __restrict__ b, const int* __restrict__ active) {
  __shared__ float red[3][8][64];
  const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + (lane & 15);
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<float> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  coarse_hop_h(B, x, n, u, wave + 1, Nx, Nt, rrow, ok, lane, acc);
  if (wave == 0) coarse_hop_h(B, x, n, u, 0, Nx, Nt, rrow, ok, lane, acc);
  if (!reduce_waves(acc, red, wave, lane)) return;
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t o = (int64_t)r * n + u * CM + 4 * (lane >> 4) + v;
    const cf val = mk<float>(acc.re[v], acc.im[v]);
    y[o] = b ? b[o] - val : val;
  }
}

// coarse_hop_h with x at the neighbour taken from the coarse correction: x_nb
// = P e for the 2x2 aggregate of the neighbour (hP: FP16 copy of P, [agg][2]
// [32][8]; ec: coarse vector, ncoarse per RHS), formed on the matrix cores in
// the B layout of the hop product
__device__ __forceinline__ void coarse_hop_hc(const chalf* __restrict__ B, const chalf* __restrict__ hP,
                                              const cf* __restrict__ ec, int64_t ncoarse, int64_t u, int d, int Nx,
                                              int Nt, int64_t rrow, int lane, CAcc<float>& acc) {
  const int i = lane & 15, q = lane >> 4;
  const int v = (int)nb_site(u, d, Nx, Nt);
  const int vx = v % Nx, vt = v / Nx;
  const int64_t A = (int64_t)(vt >> 1) * (Nx >> 1) + (vx >> 1);
  const int sl = ((vt & 1) << 1) + (vx & 1);
  const int c = i >> 3, cq = q >> 1;
  const chalf* pa = hP + (((A * 2 + c) * 32 + sl * 8 + (i & 7)) * 8) + 4 * (q & 1);
  const cf* ev = ec + rrow * ncoarse + A * CM + 4 * q;
  const chalf* row = B + ((u * 5 + d) * CM + i) * CM + 4 * q;
  h4 pr, pi, er, ei, ar, ai;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const chalf pv = pa[j];
    pr[j] = cq == c ? pv.re : (_Float16)0;
    pi[j] = cq == c ? pv.im : (_Float16)0;
    const cf e = ev[j];
    er[j] = (_Float16)e.re;
    ei[j] = (_Float16)e.im;
    const chalf a = row[j];
    ar[j] = a.re;
    ai[j] = a.im;
  }
  CAcc<float> xh{{0, 0, 0, 0}, {0, 0, 0, 0}};
  hmma(pr, pi, er, ei, xh);
  h4 br, bi;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    br[j] = (_Float16)xh.re[j];
    bi[j] = (_Float16)xh.im[j];
  }
  hmma(ar, ai, br, bi, acc);
}

__global__ void __launch_bounds__(NT) k_sap_h(const chalf* __restrict__ B, const chalf* __restrict__ inv,
                                              int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                              const cf* __restrict__ rr, cf* __restrict__ x,
                                              const int* __restrict__ active) {
  __shared__ float red[3][8][64];
  const int64_t u = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<float> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  coarse_hop_h(B, x, n, u, wave + 1, Nx, Nt, rrow, ok, lane, acc);
  // the block solve's operands are loaded after the hops (measured faster
  // than loading them first)
  cf rv[4];
  chalf iv[4];
  if (wave == 0) {
    const chalf* Iu = inv + (u * CM + i) * CM + 4 * q;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rv[j] = rr[rrow * n + u * CM + 4 * q + j];
      iv[j] = Iu[j];
    }
  }
  if (!reduce_waves(acc, red, wave, lane)) return;
  // t = r_u - hops: element j of this lane is row 4q + j, which is also the
  // B operand layout of the next product
  h4 tr, ti, ar, ai;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    tr[j] = (_Float16)(rv[j].re - acc.re[j]);
    ti[j] = (_Float16)(rv[j].im - acc.im[j]);
    ar[j] = iv[j].re;
    ai[j] = iv[j].im;
  }
  CAcc<float> cor{{0, 0, 0, 0}, {0, 0, 0, 0}};
  hmma(ar, ai, tr, ti, cor);
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) x[(int64_t)r * n + u * CM + 4 * q + v] = mk<float>(cor.re[v], cor.im[v]);
}

// k_sap_h for the first colour's first sweep after the coarse correction:
// the neighbours' x come from the coarse correction (coarse_hop_hc), so the
// prolongation is never stored
__global__ void __launch_bounds__(NT) k_sap_hc(const chalf* __restrict__ B, const chalf* __restrict__ inv,
                                              int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                               const cf* __restrict__ rr, cf* __restrict__ x,
                                               const int* __restrict__ active, const chalf* __restrict__ hP,
                                               const cf* __restrict__ ec) {
  __shared__ float red[3][8][64];
  const int64_t u = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<float> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  const int64_t ncoarse = (int64_t)(Nx / 2) * (Nt / 2) * CM;
  coarse_hop_hc(B, hP, ec, ncoarse, u, wave + 1, Nx, Nt, rrow, lane, acc);
  // the block solve's operands are loaded after the hops (measured faster
  // than loading them first)
  cf rv[4];
  chalf iv[4];
  if (wave == 0) {
    const chalf* Iu = inv + (u * CM + i) * CM + 4 * q;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      rv[j] = rr[rrow * n + u * CM + 4 * q + j];
      iv[j] = Iu[j];
    }
  }
  if (!reduce_waves(acc, red, wave, lane)) return;
  // t = r_u - hops: element j of this lane is row 4q + j, which is also the
  // B operand layout of the next product
  h4 tr, ti, ar, ai;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    tr[j] = (_Float16)(rv[j].re - acc.re[j]);
    ti[j] = (_Float16)(rv[j].im - acc.im[j]);
    ar[j] = iv[j].re;
    ai[j] = iv[j].im;
  }
  CAcc<float> cor{{0, 0, 0, 0}, {0, 0, 0, 0}};
  hmma(ar, ai, tr, ti, cor);
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) x[(int64_t)r * n + u * CM + 4 * q + v] = mk<float>(cor.re[v], cor.im[v]);
}

// ---- Two-site FP16 SAP in premultiplied form.  With the exact block
// inverse, x_B = inv_B (r_B - D_BH x_H) = rho_B - M_B x_H, where
// M_B = inv_B D_BH (32 x 96: the six outward hops of the 2x1 block, 16 dofs
// each) is formed once at setup and rho_B = inv_B r_B by the first sweep of
// each colour in a smoothing visit (r does not change during the cycles).  A colour sweep is then one
// dependent stage: each wave owns a 16 x 16 tile of x_B (16 block rows x 16
// RHS) and sums its six hop products itself, so there is no reduction
// between waves, no LDS and no barrier.
// Outward hops h = 0..5: site 0 (-x, +t, -t), site 1 (+x, +t, -t).
__device__ __forceinline__ int sap2_hop_site(int h) { return h < 3 ? 0 : 1; }
__device__ __forceinline__ int sap2_hop_dir(int h) { return h == 0 ? 2 : (h == 3 ? 1 : (h % 3 == 1 ? 3 : 4)); }

// M[blk][h][row][col] = sum_k inv[blk][row][16 s(h) + k] B[u_s(h)][dir(h)][k][col], in FP64, stored FP16
__global__ void __launch_bounds__(NT) k_sap2_premul(const cd* __restrict__ B, const cd* __restrict__ inv,
                                                    int Nx, int nblk, chalf* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)nblk * 6 * 32 * CM) return;
  const int col = (int)(e % CM), row = (int)((e / CM) % 32), h = (int)((e / (CM * 32)) % 6);
  const int blk = (int)(e / (CM * 32 * 6));
  const int NBx = Nx / 2;
  const int64_t us = (int64_t)(blk / NBx) * Nx + (blk % NBx) * 2 + sap2_hop_site(h);
  const cd* ir = inv + ((int64_t)blk * 32 + row) * 32 + 16 * sap2_hop_site(h);
  const cd* bc = B + ((us * 5 + sap2_hop_dir(h)) * CM) * CM + col;
  cd acc = mk(0.0, 0.0);
  for (int k = 0; k < CM; ++k) cfma(acc, ir[k], bc[(int64_t)k * CM]);
  M[e] = chalf{(_Float16)acc.re, (_Float16)acc.im};
}

// One colour: x_B = rho_B - M_B x_H; wave w owns all 32 block rows of RHS
// tile 4 blockIdx.y + w, so each halo value is loaded once per RHS tile.
// FIRST (the colour's first sweep of a smoothing visit): rho_B = inv_B r_B
// is formed here from r and kept in rho for the later cycles.
template <bool FIRST>
__global__ void __launch_bounds__(NT) k_sap2p_h(const chalf* __restrict__ M, const chalf* __restrict__ inv,
                                                int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                const cf* __restrict__ rr, cf* __restrict__ rho,
                                                cf* __restrict__ x, const int* __restrict__ active) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int r0 = (blockIdx.y * 4 + wave) * 16;
  if (r0 >= nrhs) return;
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int NBx = Nx / 2;
  const int64_t u0 = (int64_t)(blk / NBx) * Nx + (blk % NBx) * 2;
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  // every load of the wave is issued before the first product
  h4 br[6], bi[6];
#pragma unroll
  for (int h = 0; h < 6; ++h) {
    const cf* xv = x + rrow * n + nb_site(u0 + sap2_hop_site(h), sap2_hop_dir(h), Nx, Nt) * CM + 4 * q;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const cf v = xv[j];
      br[h][j] = (_Float16)v.re;
      bi[h][j] = (_Float16)v.im;
    }
  }
  h4 ar[2][6], ai[2][6];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int h = 0; h < 6; ++h) {
      const chalf* a = M + (((int64_t)blk * 6 + h) * 32 + rt * 16 + i) * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const chalf av = a[j];
        ar[rt][h][j] = av.re;
        ai[rt][h][j] = av.im;
      }
    }
  CAcc<float> rv[2];
  if constexpr (FIRST) {
    // rho rows rt: sum over the two sites kt of inv_B[rt][kt] r_kt
    h4 ir[2][2], ii[2][2], sr[2], si[2];
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
      const cf* rv_ = rr + rrow * n + (u0 + kt) * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const cf v = rv_[j];
        sr[kt][j] = (_Float16)v.re;
        si[kt][j] = (_Float16)v.im;
      }
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const chalf* a = inv + ((int64_t)blk * 32 + rt * 16 + i) * 32 + kt * 16 + 4 * q;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const chalf av = a[j];
          ir[rt][kt][j] = av.re;
          ii[rt][kt][j] = av.im;
        }
      }
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      rv[rt] = CAcc<float>{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
      for (int kt = 0; kt < 2; ++kt) hmma(ir[rt][kt], ii[rt][kt], sr[kt], si[kt], rv[rt]);
      if (ok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) rho[rrow * n + (u0 + rt) * CM + 4 * q + v] = mk<float>(rv[rt].re[v], rv[rt].im[v]);
      }
    }
  } else {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const cf t = rho[rrow * n + (u0 + rt) * CM + 4 * q + v];
        rv[rt].re[v] = t.re;
        rv[rt].im[v] = t.im;
      }
  }
  const bool on = ok && (!active || active[rrow] != 0);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    CAcc<float> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int h = 0; h < 6; ++h) hmma(ar[rt][h], ai[rt][h], br[h], bi[h], acc);
    if (on) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        x[rrow * n + (u0 + rt) * CM + 4 * q + v] = mk<float>(rv[rt].re[v] - acc.re[v], rv[rt].im[v] - acc.im[v]);
    }
  }
}

// ---- 2x2-site SAP blocks (K = 64) in premultiplied form, every precision:
// x_B = rho_B - M_B x_H with M_B = inv_B D_BH (64 x 128: the eight outward
// hops, 16 dofs each) formed at setup and rho_B = inv_B r_B formed by each
// colour's first sweep of a smoothing visit.  Sites s = 2 dt + dx of the
// block (t-major, the order of the block extraction); hop h = 2 s + e leaves
// site s along x (e = 0: -x for dx = 0, +x for dx = 1) or t (e = 1: -t for
// dt = 0, +t for dt = 1).  A wave owns the 32 rows of sites 2 hh, 2 hh + 1
// (hh its row half) for 16 RHS and sums its 16 hop products itself: no LDS,
// no barrier.
__device__ __forceinline__ int sap4_hop_dir(int h) {
  const int s = h >> 1;
  return (h & 1) ? ((s >> 1) ? 3 : 4) : ((s & 1) ? 1 : 2);
}
__device__ __forceinline__ int64_t sap4_site(int blk, int s, int Nx) {
  const int NBx = Nx / 2;
  return (int64_t)((blk / NBx) * 2 + (s >> 1)) * Nx + (blk % NBx) * 2 + (s & 1);
}

// M[blk][h][row][col] = sum_k inv[blk][row][16 s(h) + k] B[u_s(h)][dir(h)][k][col], in FP64
__global__ void __launch_bounds__(NT) k_sap4_premul(const cd* __restrict__ B, const cd* __restrict__ inv,
                                                    int Nx, int nblk, cd* __restrict__ M) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)nblk * 8 * 64 * CM) return;
  const int col = (int)(e % CM), row = (int)((e / CM) % 64), h = (int)((e / (CM * 64)) % 8);
  const int blk = (int)(e / (CM * 64 * 8));
  const int64_t us = sap4_site(blk, h >> 1, Nx);
  const cd* ir = inv + ((int64_t)blk * 64 + row) * 64 + 16 * (h >> 1);
  const cd* bc = B + ((us * 5 + sap4_hop_dir(h)) * CM) * CM + col;
  cd acc = mk(0.0, 0.0);
  for (int k = 0; k < CM; ++k) cfma(acc, ir[k], bc[(int64_t)k * CM]);
  M[e] = acc;
}

// FP16 operands (FP32 vectors, FP32 accumulation) on the 16x16x16 matrix cores.
// FROMC (with FIRST: the first colour's first sweep after the coarse
// correction): the halo values x_H = P e come from the coarse correction e
// itself (hP: FP16 copy of the 2x2-aggregate prolongation, [agg][2][32][8]),
// one 16x16x16 product per hop whose result layout is the B layout of the
// sweep's own product, so the prolongated x is never stored; x is then only
// written.
template <bool FIRST, bool FROMC>
__device__ __forceinline__ void sap4p_h_body(const chalf* __restrict__ M, const chalf* __restrict__ inv, int Nx,
                                             int Nt, const int* __restrict__ blist, int nrhs,
                                             const cf* __restrict__ rr, cf* __restrict__ rho, cf* __restrict__ x,
                                             const int* __restrict__ active, const chalf* __restrict__ hP,
                                             const cf* __restrict__ ec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int hh = wave & 1;
  const int r0 = (blockIdx.y * (int)(blockDim.x >> 7) + (wave >> 1)) * 16;  // 2 waves per 16-RHS tile
  if (r0 >= nrhs) return;
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;  // lanes past the last RHS read row r0; never stored
  // every load of the wave is issued before the first product
  h4 br[8], bi[8];
  // FROMC operands: P and e of every hop, loaded with everything else below
  chalf pvs[FROMC ? 8 : 1][4];
  cf evs[FROMC ? 8 : 1][4];
  const int c = i >> 3, cq = q >> 1;
  if constexpr (FROMC) {
    // x_H at hop site v: rows = v's 16 dofs (chirality i / 8, row sl' 8 + i % 8
    // of its 2x2 aggregate A'), K = the 16 coarse dofs of A' (c' 8 + k; zero
    // unless c' = chirality), columns = RHS
    const int64_t ncoarse = (int64_t)(Nx / 2) * (Nt / 2) * CM;
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int v = (int)nb_site(sap4_site(blk, h >> 1, Nx), sap4_hop_dir(h), Nx, Nt);
      const int vx = v % Nx, vt = v / Nx;
      const int64_t A = (int64_t)(vt >> 1) * (Nx >> 1) + (vx >> 1);
      const int sl = ((vt & 1) << 1) + (vx & 1);
      const chalf* pa = hP + (((A * 2 + c) * 32 + sl * 8 + (i & 7)) * 8) + 4 * (q & 1);
      const cf* ev = ec + rrow * ncoarse + A * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        pvs[h][j] = pa[j];
        evs[h][j] = ev[j];
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const cf* xv = x + rrow * n + nb_site(sap4_site(blk, h >> 1, Nx), sap4_hop_dir(h), Nx, Nt) * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const cf v = xv[j];
        br[h][j] = (_Float16)v.re;
        bi[h][j] = (_Float16)v.im;
      }
    }
  }
  h4 ar[2][8], ai[2][8];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const chalf* a = M + (((int64_t)blk * 8 + h) * 64 + (2 * hh + rt) * 16 + i) * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const chalf av = a[j];
        ar[rt][h][j] = av.re;
        ai[rt][h][j] = av.im;
      }
    }
  CAcc<float> rv[2];
  // FIRST operands: the block's r and the rows of inv_B, loaded here too
  cf rs[FIRST ? 4 : 1][4];
  chalf ivs[FIRST ? 2 : 1][FIRST ? 4 : 1][4];
  if constexpr (FIRST) {
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      const cf* rv_ = rr + rrow * n + sap4_site(blk, kt, Nx) * CM + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j) rs[kt][j] = rv_[j];
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        const chalf* a = inv + ((int64_t)blk * 64 + (2 * hh + rt) * 16 + i) * 64 + kt * 16 + 4 * q;
#pragma unroll
        for (int j = 0; j < 4; ++j) ivs[rt][kt][j] = a[j];
      }
  }
  // later cycles: rho_B of the first sweep
  cf rhos[FIRST ? 1 : 2][4];
  if constexpr (!FIRST) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
      for (int v = 0; v < 4; ++v) rhos[rt][v] = rho[rrow * n + u * CM + 4 * q + v];
    }
  }
  // every load above is issued before the first product below
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (FROMC) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      h4 pr, pi, er, ei;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const chalf pv = pvs[h][j];
        pr[j] = cq == c ? pv.re : (_Float16)0;
        pi[j] = cq == c ? pv.im : (_Float16)0;
        const cf e = evs[h][j];
        er[j] = (_Float16)e.re;
        ei[j] = (_Float16)e.im;
      }
      CAcc<float> xh{{0, 0, 0, 0}, {0, 0, 0, 0}};
      hmma(pr, pi, er, ei, xh);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        br[h][j] = (_Float16)xh.re[j];
        bi[h][j] = (_Float16)xh.im[j];
      }
    }
  }
  if constexpr (FIRST) {
    // rho rows of site 2 hh + rt: sum over the block's sites kt of inv_B[.][kt] r_kt
    h4 sr[4], si[4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sr[kt][j] = (_Float16)rs[kt][j].re;
        si[kt][j] = (_Float16)rs[kt][j].im;
      }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      rv[rt] = CAcc<float>{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) {
        h4 ir, ii;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ir[j] = ivs[rt][kt][j].re;
          ii[j] = ivs[rt][kt][j].im;
        }
        hmma(ir, ii, sr[kt], si[kt], rv[rt]);
      }
      if (ok) {
        const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
        for (int v = 0; v < 4; ++v) rho[rrow * n + u * CM + 4 * q + v] = mk<float>(rv[rt].re[v], rv[rt].im[v]);
      }
    }
  } else {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rv[rt].re[v] = rhos[rt][v].re;
        rv[rt].im[v] = rhos[rt][v].im;
      }
  }
  const bool on = ok && (!active || active[rrow] != 0);
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    CAcc<float> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int h = 0; h < 8; ++h) hmma(ar[rt][h], ai[rt][h], br[h], bi[h], acc);
    if (on) {
      const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        x[rrow * n + u * CM + 4 * q + v] = mk<float>(rv[rt].re[v] - acc.re[v], rv[rt].im[v] - acc.im[v]);
    }
  }
}

template <bool FIRST>
__global__ void __launch_bounds__(NT) k_sap4p_h(const chalf* __restrict__ M, const chalf* __restrict__ inv,
                                                int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                const cf* __restrict__ rr, cf* __restrict__ rho,
                                                cf* __restrict__ x, const int* __restrict__ active) {
  sap4p_h_body<FIRST, false>(M, inv, Nx, Nt, blist, nrhs, rr, rho, x, active, nullptr, nullptr);
}
__global__ void __launch_bounds__(NT) k_sap4p_hc(const chalf* __restrict__ M, const chalf* __restrict__ inv,
                                                 int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                 const cf* __restrict__ rr, cf* __restrict__ rho,
                                                 cf* __restrict__ x, const int* __restrict__ active,
                                                 const chalf* __restrict__ hP, const cf* __restrict__ ec) {
  sap4p_h_body<true, true>(M, inv, Nx, Nt, blist, nrhs, rr, rho, x, active, hP, ec);
}

// FP32 / FP64 operands on the 16x16x4 matrix cores (K chunks of 4 per hop;
// in chunk c lane l takes the K index out_row(l, c), so a product's result
// layout is the next one's B layout, as for the coarse stencil)
template <class T, bool FIRST>
__global__ void __launch_bounds__(NT) k_sap4p(const cx<T>* __restrict__ M, const cx<T>* __restrict__ inv,
                                              int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                              const cx<T>* __restrict__ rr, cx<T>* __restrict__ rho,
                                              cx<T>* __restrict__ x, const int* __restrict__ active) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15;
  const int hh = wave & 1;
  const int r0 = (blockIdx.y * (int)(blockDim.x >> 7) + (wave >> 1)) * 16;  // 2 waves per 16-RHS tile
  if (r0 >= nrhs) return;
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<T> rv[2];
  if constexpr (FIRST) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      rv[rt] = CAcc<T>{{0, 0, 0, 0}, {0, 0, 0, 0}};
      const cx<T>* ir = inv + ((int64_t)blk * 64 + (2 * hh + rt) * 16 + i) * 64;
      for (int kt = 0; kt < 4; ++kt) {
        const cx<T>* rv_ = rr + rrow * n + sap4_site(blk, kt, Nx) * CM;
        cx<T> a[4], b[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int k = MF<T>::out_row(lane, c);
          a[c] = ir[kt * 16 + k];
          b[c] = rv_[k];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) cmma(a[c], b[c], rv[rt]);
      }
      if (ok) {
        const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          rho[rrow * n + u * CM + MF<T>::out_row(lane, v)] = mk<T>(rv[rt].re[v], rv[rt].im[v]);
      }
    }
  } else {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const cx<T> t = rho[rrow * n + u * CM + MF<T>::out_row(lane, v)];
        rv[rt].re[v] = t.re;
        rv[rt].im[v] = t.im;
      }
    }
  }
  CAcc<T> acc[2] = {CAcc<T>{{0, 0, 0, 0}, {0, 0, 0, 0}}, CAcc<T>{{0, 0, 0, 0}, {0, 0, 0, 0}}};
#pragma unroll 2
  for (int h = 0; h < 8; ++h) {
    const cx<T>* xv = x + rrow * n + nb_site(sap4_site(blk, h >> 1, Nx), sap4_hop_dir(h), Nx, Nt) * CM;
    cx<T> b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) b[c] = xv[MF<T>::out_row(lane, c)];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const cx<T>* a = M + (((int64_t)blk * 8 + h) * 64 + (2 * hh + rt) * 16 + i) * CM;
#pragma unroll
      for (int c = 0; c < 4; ++c) cmma(a[MF<T>::out_row(lane, c)], b[c], acc[rt]);
    }
  }
  if (!ok || (active && !active[rrow])) return;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt) {
    const int64_t u = sap4_site(blk, 2 * hh + rt, Nx);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      x[rrow * n + u * CM + MF<T>::out_row(lane, v)] =
          mk<T>(rv[rt].re[v] - acc[rt].re[v], rv[rt].im[v] - acc[rt].im[v]);
  }
}

__global__ void __launch_bounds__(NT) k_to_half(const cd* __restrict__ in, chalf* __restrict__ out,
                                                int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= count) return;
  out[e] = chalf{(_Float16)in[e].re, (_Float16)in[e].im};
}

// One colour of the coarse SAP sweep with two-site blocks along x (sites u0,
// u1 = u0 + x^, K = 32): x_B = inv_B (r_B - outward hops).  One workgroup per
// (block, 16 RHS); the six outward hops are spread over the four waves
// (u0: -x, +t | -t; u1: +x, +t | -t), summed per site in LDS, and waves 0 and
// 1 apply the two row halves of inv_B.
template <class T>
__global__ void __launch_bounds__(NT) k_sap2_mfma(const cx<T>* __restrict__ B, const cx<T>* __restrict__ inv,
                                                  int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                  const cx<T>* __restrict__ rr, cx<T>* __restrict__ x,
                                                  const int* __restrict__ active) {
  __shared__ T red[4][8][64];
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int NBx = Nx / 2;
  const int64_t u0 = (int64_t)(blk / NBx) * Nx + (blk % NBx) * 2, u1 = u0 + 1;
  const int64_t n = (int64_t)Nx * Nt * CM;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15;
  const int r0 = blockIdx.y * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  CAcc<T> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  const int64_t us = wave < 2 ? u0 : u1;
  if (wave == 0 || wave == 2) {
    coarse_hop(B, x, n, us, wave == 0 ? 2 : 1, Nx, Nt, rrow, ok, lane, acc);
    coarse_hop(B, x, n, us, 3, Nx, Nt, rrow, ok, lane, acc);
  } else {
    coarse_hop(B, x, n, us, 4, Nx, Nt, rrow, ok, lane, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    red[wave][v][lane] = acc.re[v];
    red[wave][4 + v][lane] = acc.im[v];
  }
  // operands of the block solve, loaded after the hops (waves 0 and 1: row
  // half = wave)
  cx<T> rv[2][4], a[2][4];
  if (wave < 2) {
    const cx<T>* Ih = inv + ((int64_t)blk * 32 + wave * 16 + i) * 32;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = MF<T>::out_row(lane, c);
      rv[0][c] = rr[rrow * n + u0 * CM + k];
      rv[1][c] = rr[rrow * n + u1 * CM + k];
      a[0][c] = Ih[k];
      a[1][c] = Ih[16 + k];
    }
  }
  __syncthreads();
  if (wave >= 2) return;
  cx<T> t[2][4];
#pragma unroll
  for (int sidx = 0; sidx < 2; ++sidx)
#pragma unroll
    for (int c = 0; c < 4; ++c)
      t[sidx][c] = mk<T>(rv[sidx][c].re - red[2 * sidx][c][lane] - red[2 * sidx + 1][c][lane],
                         rv[sidx][c].im - red[2 * sidx][4 + c][lane] - red[2 * sidx + 1][4 + c][lane]);
  CAcc<T> cor{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
  for (int sidx = 0; sidx < 2; ++sidx)
#pragma unroll
    for (int c = 0; c < 4; ++c) cmma(a[sidx][c], t[sidx][c], cor);
  if (!ok || (active && !active[r])) return;
  const int64_t uo = wave == 0 ? u0 : u1;
#pragma unroll
  for (int v = 0; v < 4; ++v)
    x[(int64_t)r * n + uo * CM + MF<T>::out_row(lane, v)] = mk<T>(cor.re[v], cor.im[v]);
}

// One colour of the fine-level SAP sweep with 4x4-site blocks (K = 32 dofs).
// With the exact block inverse, x_B + inv_B (r - D x)_B = inv_B (r_B - D_BH x_H):
// only the hops that leave the block (x of the other colour) enter, and the
// old x_B is not read.  One workgroup per block and 64 RHS (a wave per 16):
// the halo term on the vector units, the 32 x 32 solve as two 16-row tiles
// of complex MFMAs over 8 K-chunks.
// x64 (or null): the block's new values are also stored widened to FP64
// there, in the lattice layout (the last sweeps of an FP32 cycle write its
// FP64 result directly).  BLK: r and x in the block-major layout (a block's
// 32 dofs contiguous, sites t-major), so that a colour's sweep fetches only
// its own r and the other colour's x; unused hop slots then read the row's
// +x neighbour outside the block, which that row's last site loads anyway.
template <class T, bool BLK = false>
__global__ void __launch_bounds__(NT) k_sap0_mfma(const cx<T>* __restrict__ B, const cx<T>* __restrict__ inv,
                                                  int Nx, int Nt, const int* __restrict__ blist, int nrhs,
                                                  const cx<T>* __restrict__ rr, cx<T>* __restrict__ x,
                                                  const int* __restrict__ active, cd* __restrict__ x64) {
  constexpr int SB = 4, NS = SB * SB, K = 2 * NS;
  __shared__ cx<T> Is[K * K];
  __shared__ cx<T> Bs[NS * 5 * 4];
  __shared__ cx<T> Hs[4][16][K + 1];  // per wave: 16 RHS x the block's 32 dofs
  const int blk = blist[xcd_tile(blockIdx.x, gridDim.x)];
  const int NBx = Nx / SB;
  const int bx = (blk % NBx) * SB, bt = (blk / NBx) * SB;
  const int nthr = blockDim.x;  // 64 per 16-RHS tile, at most NT
  for (int e = threadIdx.x; e < K * K; e += nthr) Is[e] = inv[(int64_t)blk * K * K + e];
  for (int e = threadIdx.x; e < NS * 20; e += nthr) {
    const int s = e / 20;
    const int64_t us = (int64_t)(bt + s / SB) * Nx + bx + s % SB;
    Bs[e] = B[us * 20 + e % 20];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = (blockIdx.y * (nthr >> 6) + wave) * 16;
  const int64_t n = (int64_t)Nx * Nt * 2;
  // Halo term h = r_B - D_BH x_H on the vector units, lanes along the block's
  // dofs (k = lane % 32: a time row of the block is 8 consecutive dofs) and
  // two RHS per pass, so a load instruction covers 8 segments of 64 bytes.
  // A wave whose RHS are all past nrhs still runs (clamped loads, no stores)
  // so that every wave reaches the barriers.
  const int k = lane & 31;
  const int s = k >> 1, a = k & 1, sx = s & 3, st = s >> 2;
  const int gx = bx + sx, gt = bt + st;
  const int own = gt * Nx + gx;
  // at most two outward hops per site of a 4x4 block; unused slots point at
  // the site itself (BLK: at the row's +x neighbour) so that every load is
  // unconditional
  const int fill = BLK ? gt * Nx + (bx + SB == Nx ? 0 : bx + SB) : own;
  int nbs[2] = {fill, fill}, dirs[2] = {0, 0}, nh = 0;
  if (sx == SB - 1) { dirs[nh] = 1; nbs[nh++] = gt * Nx + (gx + 1 == Nx ? 0 : gx + 1); }
  if (sx == 0) { dirs[nh] = 2; nbs[nh++] = gt * Nx + (gx == 0 ? Nx - 1 : gx - 1); }
  if (st == SB - 1) { dirs[nh] = 3; nbs[nh++] = (gt + 1 == Nt ? 0 : gt + 1) * Nx + gx; }
  if (st == 0) { dirs[nh] = 4; nbs[nh++] = (gt == 0 ? Nt - 1 : gt - 1) * Nx + gx; }
  // offsets of the two dofs of a site in r / x (lattice or block-major)
  auto vofs = [&](int v) -> int64_t {
    if (!BLK) return (int64_t)v * 2;
    const int vx = v % Nx, vt = v / Nx;
    return (int64_t)((vt / SB) * NBx + vx / SB) * K + ((vt % SB) * SB + vx % SB) * 2;
  };
  const int64_t own_o = BLK ? (int64_t)blk * K + k : (int64_t)own * 2 + a;
  const int64_t nbo[2] = {vofs(nbs[0]), vofs(nbs[1])};
  // the r and halo x of all eight passes are loaded before the barrier that
  // ends the staging of inv_B and the links, so both sets of loads are in
  // flight together (one memory round trip, not two)
  cx<T> rv[8], xh[8][2][2];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int r = r0 + 2 * p + (lane >> 5);
    const int64_t rc = r < nrhs ? r : 0;
    const cx<T>* xr = x + rc * n;
    rv[p] = rr[rc * n + own_o];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      xh[p][j][0] = xr[nbo[j]];
      xh[p][j][1] = xr[nbo[j] + 1];
    }
  }
  __syncthreads();
  cx<T> bb[2][2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const cx<T>* bp = Bs + (s * 5 + dirs[j]) * 4 + a * 2;
    const bool use = j < nh;
    bb[j][0] = use ? bp[0] : mk<T>(0, 0);
    bb[j][1] = use ? bp[1] : mk<T>(0, 0);
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int ri = 2 * p + (lane >> 5);
    cx<T> acc = rv[p];
#pragma unroll
    for (int j = 0; j < 2; ++j) acc = acc - bb[j][0] * xh[p][j][0] - bb[j][1] * xh[p][j][1];
    Hs[wave][ri][k] = acc;
  }
  __syncthreads();
  // x_B = inv_B h: the 32 x 32 solve as two 16-row tiles of complex MFMAs
  // over 8 K-chunks (B operand: K index x 16 RHS, read back from LDS)
  const int i = lane & 15;
  cx<T> h[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) h[c] = Hs[wave][i][16 * (c >> 2) + MF<T>::out_row(lane, c & 3)];
  CAcc<T> acc[2];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    acc[half] = CAcc<T>{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int kcol = 16 * (c >> 2) + MF<T>::out_row(lane, c & 3);
      cmma(Is[(half * 16 + i) * K + kcol], h[c], acc[half]);
    }
  }
  __syncthreads();  // every lane has read its h before Hs is overwritten
#pragma unroll
  for (int half = 0; half < 2; ++half)
#pragma unroll
    for (int v = 0; v < 4; ++v) Hs[wave][i][half * 16 + MF<T>::out_row(lane, v)] = mk<T>(acc[half].re[v], acc[half].im[v]);
  __syncthreads();
  // coalesced stores, lanes along the block's dofs as for the loads
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int ri = 2 * p + (lane >> 5);
    const int r = r0 + ri;
    if (r < nrhs && !(active && !active[r])) {
      const cx<T> v = Hs[wave][ri][k];
      x[(int64_t)r * n + own_o] = v;
      if (x64) x64[(int64_t)r * n + (int64_t)own * 2 + a] = mk((double)v.re, (double)v.im);
    }
  }
}

// y[r] = A x[r] for a dense n x n A held in FP16 (x rounded to FP16, FP32
// accumulation) on the 16x16x32 matrix cores: the coarse solve of the FP16
// cycle.  A workgroup owns 16 TR rows x 16 RHS; each of its eight waves takes
// an eighth of the k range with TR 16 x 16 result tiles (one per 16 rows),
// loading the next 32-wide k step while the matrix cores work on the current
// one, and the eighths are summed in LDS in wave order.  The RHS tiles of a
// row group are consecutive in the XCD-ordered workgroup index, so the rows
// of A they share are fetched into one L2.  Lane l supplies the K slots
// 8 (l/16) .. 8 (l/16) + 7 of row l%16 of A and of RHS column l%16 (32 bytes
// of A per row tile, 64 bytes of x); n is a multiple of 256.
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h16 __attribute__((ext_vector_type(16)));
typedef float f16v __attribute__((ext_vector_type(16)));
constexpr int DH_W = 8;  // waves per workgroup (k split)

template <int TR>
__device__ __forceinline__ void dense_h_step(const h16 (&a)[TR], const f16v& xv, CAcc<float> (&acc)[TR]) {
  h8 xr, xi;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    xr[j] = (_Float16)xv[2 * j];
    xi[j] = (_Float16)xv[2 * j + 1];
  }
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const h8 ar = __builtin_shufflevector(a[t], a[t], 0, 2, 4, 6, 8, 10, 12, 14);
    const h8 ai = __builtin_shufflevector(a[t], a[t], 1, 3, 5, 7, 9, 11, 13, 15);
    acc[t].re = __builtin_amdgcn_mfma_f32_16x16x32_f16(ar, xr, acc[t].re, 0, 0, 0);
    acc[t].re = __builtin_amdgcn_mfma_f32_16x16x32_f16(-ai, xi, acc[t].re, 0, 0, 0);
    acc[t].im = __builtin_amdgcn_mfma_f32_16x16x32_f16(ar, xi, acc[t].im, 0, 0, 0);
    acc[t].im = __builtin_amdgcn_mfma_f32_16x16x32_f16(ai, xr, acc[t].im, 0, 0, 0);
  }
}

template <int TR>
__global__ void __launch_bounds__(64 * DH_W) k_dense_h(const chalf* __restrict__ A, int64_t n, int nrhs,
                                                      const cf* __restrict__ x, cf* __restrict__ y,
                                                      const int* __restrict__ active) {
  __shared__ float red[DH_W - 1][TR][8][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int ntile = gridDim.y;
  const int64_t Lg = xcd_tile(blockIdx.x + (int64_t)gridDim.x * blockIdx.y, (int64_t)gridDim.x * ntile);
  const int64_t i0 = (Lg / ntile) * 16 * TR;
  const int r0 = (int)(Lg % ntile) * 16;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;  // lanes past the last RHS read row r0; never stored
  const int64_t kw = n / DH_W, kb = kw * wave;
  CAcc<float> acc[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) acc[t] = CAcc<float>{{0, 0, 0, 0}, {0, 0, 0, 0}};
  const chalf* Ab = A + (i0 + i) * n + kb + 8 * q;
  const cf* xb = x + rrow * n + kb + 8 * q;
  h16 a0[TR], a1[TR];
  f16v x0, x1;
  auto load = [&](h16 (&a)[TR], f16v& xv, int64_t k0) {
    xv = *reinterpret_cast<const f16v*>(xb + k0);
#pragma unroll
    for (int t = 0; t < TR; ++t) a[t] = *reinterpret_cast<const h16*>(Ab + 16 * t * n + k0);
  };
  load(a0, x0, 0);
  for (int64_t k0 = 0; k0 < kw; k0 += 64) {
    const bool second = k0 + 32 < kw;
    if (second) load(a1, x1, k0 + 32);
    dense_h_step<TR>(a0, x0, acc);
    if (second) {
      if (k0 + 64 < kw) load(a0, x0, k0 + 64);
      dense_h_step<TR>(a1, x1, acc);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        red[wave - 1][t][v][lane] = acc[t].re[v];
        red[wave - 1][t][4 + v][lane] = acc[t].im[v];
      }
  }
  __syncthreads();
  if (wave != 0 || !ok || (active && !active[r])) return;
#pragma unroll
  for (int t = 0; t < TR; ++t) {
#pragma unroll
    for (int w = 0; w < DH_W - 1; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[t].re[v] += red[w][t][v][lane];
        acc[t].im[v] += red[w][t][4 + v][lane];
      }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      y[(int64_t)r * n + i0 + 16 * t + 4 * q + v] = mk<float>(acc[t].re[v], acc[t].im[v]);
  }
}

// FP16 copy of a matrix; *overflow is set when a component does not fit
// (|v| above the largest finite FP16 value after rounding)
__global__ void __launch_bounds__(NT) k_to_half_checked(const cd* __restrict__ in, chalf* __restrict__ out,
                                                        int64_t count, int* __restrict__ overflow) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= count) return;
  const _Float16 re = (_Float16)in[e].re, im = (_Float16)in[e].im;
  out[e] = chalf{re, im};
  if (!__builtin_isfinite((float)re) || !__builtin_isfinite((float)im)) *overflow = 1;
}

// y[r] = A x[r] for a dense n x n A (n a multiple of 16): a wave owns 16 rows
// x 16 RHS over a quarter of the workgroup's k range; the quarters are summed
// in LDS, and k ranges split over gridDim.z go to part[z] (k_dense_reduce).
template <class T>
__global__ void __launch_bounds__(NT) k_dense_mfma(const cx<T>* __restrict__ A, int64_t n, int nrhs,
                                                   int64_t klen, const cx<T>* __restrict__ x,
                                                   cx<T>* __restrict__ y, cx<T>* __restrict__ part,
                                                   const int* __restrict__ active) {
  __shared__ T red[2][3][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 16;
  const int r0 = blockIdx.y * 16;
  const int i = lane & 15;
  const int r = r0 + i;
  const bool ok = r < nrhs;
  const int64_t rrow = ok ? r : r0;
  const int64_t kb = (int64_t)blockIdx.z * klen;
  const int64_t ke = min(n, kb + klen);
  // the workgroup's k range in 16-wide steps, split over the 4 waves
  const int64_t steps = (ke - kb + 15) / 16, per = (steps + 3) / 4;
  const int64_t kw0 = min(ke, kb + per * 16 * wave);
  const int64_t kw1 = min(ke, kw0 + per * 16);
  CAcc<T> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
  const cx<T>* Ar = A + (i0 + i) * n;
  const cx<T>* xr = x + rrow * n;
  for (int64_t k0 = kw0; k0 < kw1; k0 += 16) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t k = k0 + MF<T>::out_row(lane, c);
      // kw0, kw1 are multiples of 16 (n, klen and so every range bound are),
      // so k < kw1 here; lanes past the last RHS read row rrow
      const cx<T> a = Ar[k];
      const cx<T> xb = xr[k];
      cmma(a, xb, acc);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      red[0][wave - 1][v][lane] = acc.re[v];
      red[1][wave - 1][v][lane] = acc.im[v];
    }
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      acc.re[v] += red[0][w][v][lane];
      acc.im[v] += red[1][w][v][lane];
    }
  if (!ok || (active && !active[r])) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t row = i0 + MF<T>::out_row(lane, v);
    const cx<T> val = mk<T>(acc.re[v], acc.im[v]);
    if (gridDim.z == 1) y[(int64_t)r * n + row] = val;
    else part[((int64_t)blockIdx.z * nrhs + r) * n + row] = val;
  }
}

// ------------------------------------------------------------------ dense coarsest level
__global__ void __launch_bounds__(NT) k_dense_from_stencil(const cd* __restrict__ B, int Nx, int Nt,
                                                           int M, cd* __restrict__ A) {
  const int64_t sites = (int64_t)Nx * Nt;
  const int64_t n = sites * M;
  const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (row >= n) return;
  const int64_t u = row / M;
  const int al = (int)(row % M);
  for (int d = 0; d < 5; ++d) {
    const int64_t v = nb_site(u, d, Nx, Nt);
    for (int be = 0; be < M; ++be) {
      cd* o = A + row * n + v * M + be;
      *o = *o + B[((u * 5 + d) * M + al) * M + be];
    }
  }
}

// pivot search in column k below the diagonal (largest |a|, first on ties)
__global__ void __launch_bounds__(NT) k_gj_pivot(const cd* __restrict__ A, int64_t n, int64_t k,
                                                 int* __restrict__ perm, cd* __restrict__ pivinv,
                                                 int* __restrict__ fail) {
  __shared__ double bv[NT];
  __shared__ int64_t bi[NT];
  const int tid = threadIdx.x;
  double best = -1.0;
  int64_t bidx = k;
  for (int64_t i = k + tid; i < n; i += NT) {
    const double v = abs2(A[i * n + k]);
    if (v > best) { best = v; bidx = i; }
  }
  bv[tid] = best;
  bi[tid] = bidx;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double v2 = bv[tid + s];
      const int64_t i2 = bi[tid + s];
      if (v2 > bv[tid] || (v2 == bv[tid] && i2 < bi[tid])) { bv[tid] = v2; bi[tid] = i2; }
    }
    __syncthreads();
  }
  if (tid == 0) {
    perm[k] = (int)bi[0];
    if (bv[0] <= 0.0) {
      *fail = 1;
      *pivinv = mk(0.0, 0.0);
    } else {
      *pivinv = cdiv(mk(1.0, 0.0), A[bi[0] * n + k]);
    }
  }
}

__global__ void __launch_bounds__(NT) k_gj_swap_scale(cd* __restrict__ A, int64_t n, int64_t k,
                                                      const int* __restrict__ perm,
                                                      const cd* __restrict__ pivinv) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const int64_t p = perm[k];
  const cd vk = A[k * n + j], vp = A[p * n + j];
  if (p != k) A[p * n + j] = vk;
  A[k * n + j] = ((j == k) ? mk(1.0, 0.0) : vp) * (*pivinv);
}

__global__ void __launch_bounds__(NT) k_gj_col(const cd* __restrict__ A, int64_t n, int64_t k,
                                               cd* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  f[i] = (i == k) ? mk(0.0, 0.0) : A[i * n + k];
}

__global__ void __launch_bounds__(NT) k_gj_eliminate(cd* __restrict__ A, int64_t n, int64_t k,
                                                     const cd* __restrict__ f) {
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i == k || j >= n) return;
  const cd fi = f[i];
  if (fi.re == 0.0 && fi.im == 0.0) return;
  cd* o = A + i * n + j;
  const cd base = (j == k) ? mk(0.0, 0.0) : *o;
  *o = base - fi * A[k * n + j];
}

// ---- blocked Gauss-Jordan: the steps of a 64-column panel run on the panel
// only; the rest of the matrix then takes the panel's row swaps and one
// rank-64 update on the FP64 matrix cores.
constexpr int GJ_NB = 64;

// swap rows k and perm[k], then scale row k, on the columns [c0, c0 + GJ_NB)
__global__ void __launch_bounds__(NT) k_gj_swap_scale_panel(cd* __restrict__ A, int64_t n, int64_t k,
                                                            int64_t c0, const int* __restrict__ perm,
                                                            const cd* __restrict__ pivinv) {
  const int t = threadIdx.x;
  if (t >= GJ_NB) return;
  const int64_t j = c0 + t;
  const int64_t p = perm[k];
  const cd vk = A[k * n + j], vp = A[p * n + j];
  if (p != k) A[p * n + j] = vk;
  A[k * n + j] = ((j == k) ? mk(1.0, 0.0) : vp) * (*pivinv);
}

// elimination of column k on the panel columns: thread e -> (row e / 64, column c0 + e % 64)
__global__ void __launch_bounds__(NT) k_gj_eliminate_panel(cd* __restrict__ A, int64_t n, int64_t k,
                                                           int64_t c0, const cd* __restrict__ f) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int64_t i = e / GJ_NB, j = c0 + e % GJ_NB;
  if (i >= n || i == k) return;
  const cd fi = f[i];
  if (fi.re == 0.0 && fi.im == 0.0) return;
  cd* o = A + i * n + j;
  const cd base = (j == k) ? mk(0.0, 0.0) : *o;
  *o = base - fi * A[k * n + j];
}

// the panel's row swaps on the other columns, in step order; T = the panel
// rows of those columns (zero on the panel columns)
__global__ void __launch_bounds__(NT) k_gj_swaps_rest(cd* __restrict__ A, int64_t n, int64_t c0,
                                                      const int* __restrict__ perm, cd* __restrict__ T) {
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  const bool panel = j >= c0 && j < c0 + GJ_NB;
  if (!panel) {
    for (int q = 0; q < GJ_NB; ++q) {
      const int64_t k = c0 + q, p = perm[k];
      if (p != k) {
        const cd a = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = a;
      }
    }
  }
  for (int q = 0; q < GJ_NB; ++q) T[(int64_t)q * n + j] = panel ? mk(0.0, 0.0) : A[(c0 + q) * n + j];
}

// A[i][j] = (i in panel rows ? 0 : A[i][j]) + sum_q A[i][c0 + q] T[q][j] for
// the columns j outside the panel.  64 x 64 output tiles, each wave a 32 x 32
// quarter as 2 x 2 blocks of 16 x 16; complex products as four real FP64 MFMAs.
__global__ void __launch_bounds__(NT) k_gj_update(cd* __restrict__ A, int64_t n, int64_t c0,
                                                  const cd* __restrict__ T) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * 64 + (wave >> 1) * 32;
  const int64_t j0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  if (j0 + 32 > c0 && j0 < c0 + GJ_NB) return;  // panel columns (uniform per wave)
  typedef MF<double>::v4 v4;
  v4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = v4{0, 0, 0, 0};
      ci[a][b] = v4{0, 0, 0, 0};
    }
  const int r = lane & 15, q4 = lane >> 4;
  for (int kk = 0; kk < GJ_NB; kk += 4) {
    const int q = kk + q4;
    cd av[2], bv[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) av[a] = A[(i0 + a * 16 + r) * n + c0 + q];
#pragma unroll
    for (int b = 0; b < 2; ++b) bv[b] = T[(int64_t)q * n + j0 + b * 16 + r];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        cr[a][b] = MF<double>::mma(av[a].re, bv[b].re, cr[a][b]);
        cr[a][b] = MF<double>::mma(-av[a].im, bv[b].im, cr[a][b]);
        ci[a][b] = MF<double>::mma(av[a].re, bv[b].im, ci[a][b]);
        ci[a][b] = MF<double>::mma(av[a].im, bv[b].re, ci[a][b]);
      }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + a * 16 + MF<double>::out_row(lane, v);
        const int64_t j = j0 + b * 16 + r;
        cd* o = A + i * n + j;
        const cd base = (i >= c0 && i < c0 + GJ_NB) ? mk(0.0, 0.0) : *o;
        *o = mk(base.re + cr[a][b][v], base.im + ci[a][b][v]);
      }
}

__global__ void __launch_bounds__(NT) k_gather_cols(const cd* __restrict__ W, int64_t n,
                                                    const int* __restrict__ pi, cd* __restrict__ out) {
  const int64_t i = blockIdx.y;
  const int64_t j = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (j >= n) return;
  out[i * n + j] = W[i * n + pi[j]];
}

__global__ void __launch_bounds__(NT) k_diag_sum(const cd* __restrict__ A, int64_t n,
                                                 cd* __restrict__ out) {
  __shared__ cd part[NT];
  const int tid = threadIdx.x;
  cd acc = mk(0.0, 0.0);
  for (int64_t i = tid; i < n; i += NT) acc = acc + A[i * n + i];
  part[tid] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) part[tid] = part[tid] + part[tid + s];
    __syncthreads();
  }
  if (tid == 0) *out = part[0];
}

// y[r][i] = sum_j A[i][j] x[r][j]: tiles of 64 rows x 16 RHS, 32-wide k steps,
// the k range split over gridDim.z workgroups.  With a split, every
// workgroup writes its partial sums to part[z][r][i] and k_dense_reduce adds
// them in z order (deterministic); without, the tile is written to y.
template <class T>
__global__ void __launch_bounds__(NT) k_dense_apply(const cx<T>* __restrict__ A, int64_t n, int nrhs,
                                                    int64_t klen, const cx<T>* __restrict__ x,
                                                    cx<T>* __restrict__ y, cx<T>* __restrict__ part,
                                                    const int* __restrict__ active) {
  constexpr int TI = 64, TR = 16, TJ = 32;
  __shared__ cx<T> As[TJ][TI + 1];
  __shared__ cx<T> Xs[TR][TJ + 1];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * TI;
  const int r0 = blockIdx.y * TR;
  const int il = tid % TI, rg = tid / TI;  // 4 groups of 4 RHS
  if (active) {  // skip tiles whose RHS are all converged (uniform per workgroup)
    bool any = false;
    for (int q = 0; q < TR; ++q) any = any || (r0 + q < nrhs && active[r0 + q]);
    if (!any) return;
  }
  const int64_t kb = (int64_t)blockIdx.z * klen;
  const int64_t ke = min(n, kb + klen);
  cx<T> acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = mk<T>(0, 0);
  for (int64_t j0 = kb; j0 < ke; j0 += TJ) {
    for (int e = tid; e < TI * TJ; e += NT) {
      const int ii = e / TJ, jj = e % TJ;
      const int64_t gi = i0 + ii, gj = j0 + jj;
      As[jj][ii] = ld_or0(A + (gi < n ? gi : 0) * n + (gj < ke ? gj : kb), gi < n && gj < ke);
    }
    for (int e = tid; e < TR * TJ; e += NT) {
      const int rr = e / TJ, jj = e % TJ;
      const int gr = r0 + rr;
      const int64_t gj = j0 + jj;
      Xs[rr][jj] = ld_or0(x + (int64_t)(gr < nrhs ? gr : 0) * n + (gj < ke ? gj : kb), gr < nrhs && gj < ke);
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < TJ; ++jj) {
      const cx<T> a = As[jj][il];
#pragma unroll
      for (int q = 0; q < 4; ++q) cfma(acc[q], a, Xs[rg * 4 + q][jj]);
    }
    __syncthreads();
  }
  const int64_t gi = i0 + il;
  if (gi < n) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gr = r0 + rg * 4 + q;
      if (gr >= nrhs || (active && !active[gr])) continue;
      if (gridDim.z == 1) y[(int64_t)gr * n + gi] = acc[q];
      else part[((int64_t)blockIdx.z * nrhs + gr) * n + gi] = acc[q];
    }
  }
}

template <class T>
__global__ void __launch_bounds__(NT) k_dense_reduce(const cx<T>* __restrict__ part, int ks, int64_t n,
                                                     int nrhs, cx<T>* __restrict__ y,
                                                     const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  cx<T> acc = mk<T>(0, 0);
  for (int z = 0; z < ks; ++z) acc = acc + part[((int64_t)z * nrhs + r) * n + i];
  y[(int64_t)r * n + i] = acc;
}

// qr+ of the rows of V (columns = test vectors, V[k][n]) belonging to each
// aggregate A and chirality c: classical Gram-Schmidt applied twice per column,
// positive real norms.  One workgroup per (A, c), one thread per row.
constexpr int QR_MAXTV = 16;
__global__ void __launch_bounds__(NT) k_local_qr(const cd* __restrict__ V, int64_t n, int Nx, int M,
                                                 int bx, int bt, int ntv, cd* __restrict__ P) {
  __shared__ cd red[4][QR_MAXTV];
  const int64_t A = blockIdx.x / 2;
  const int c = blockIdx.x % 2;
  const int s = threadIdx.x;
  const int nrow = bx * bt * (M / 2);
  const int NAx = Nx / bx;
  const int lane = s & 63, wv = s >> 6;
  cd v[QR_MAXTV];
  const bool has = s < nrow;
  const int64_t row = has ? agg_row(A, c, s, Nx, M, bx, bt, NAx) : 0;
#pragma unroll
  for (int k = 0; k < QR_MAXTV; ++k) v[k] = (has && k < ntv) ? V[(int64_t)k * n + row] : mk(0.0, 0.0);
  for (int k = 0; k < ntv; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
      cd coef[QR_MAXTV];
#pragma unroll
      for (int i = 0; i < QR_MAXTV; ++i) {
        coef[i] = mk(0.0, 0.0);
        if (i < k) {
          cd t = cjmul(v[i], v[k]);
          for (int o = 32; o > 0; o >>= 1) {
            t.re += __shfl_xor(t.re, o, 64);
            t.im += __shfl_xor(t.im, o, 64);
          }
          if (lane == 0) red[wv][i] = t;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < QR_MAXTV; ++i)
        if (i < k) coef[i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < QR_MAXTV; ++i)
        if (i < k) v[k] = v[k] - v[i] * coef[i];
    }
    double t = abs2(v[k]);
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) red[wv][0] = mk(t, 0.0);
    __syncthreads();
    const double nrm = sqrt((red[0][0].re + red[1][0].re) + (red[2][0].re + red[3][0].re));
    __syncthreads();
    v[k] = (1.0 / nrm) * v[k];
  }
  if (has) {
    cd* o = P + ((A * 2 + c) * nrow + s) * ntv;
#pragma unroll
    for (int k = 0; k < QR_MAXTV; ++k)
      if (k < ntv) o[k] = v[k];
  }
}

// antiperiodic t boundary: the t-links leaving the last time slice get -1
__global__ void __launch_bounds__(NT) k_fold_anti(cd* __restrict__ links, int Lx, int Lt) {
  const int x = blockIdx.x * NT + threadIdx.x;
  if (x >= Lx) return;
  cd* u = links + (int64_t)Lx * Lt + (int64_t)(Lt - 1) * Lx + x;
  *u = -1.0 * (*u);
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_fold_anti(hipStream_t s, cd* links, int Lx, int Lt) {
  hipLaunchKernelGGL(k_fold_anti, dim3(grid1(Lx)), dim3(NT), 0, s, links, Lx, Lt);
  KCHK();
}
void launch_local_qr(hipStream_t s, const cd* V, int64_t n, int Nx, int Nt, int M, int bx, int bt,
                     int ntv, cd* P) {
  require(ntv >= 1 && ntv <= QR_MAXTV, "at most 16 test vectors per chirality");
  require(bx * bt * (M / 2) <= NT, "aggregate has more than 256 rows per chirality");
  require(bx * bt * (M / 2) >= ntv, "aggregate has fewer rows than test vectors");
  const int64_t nagg = (int64_t)(Nx / bx) * (Nt / bt);
  hipLaunchKernelGGL(k_local_qr, dim3((unsigned)(nagg * 2)), dim3(NT), 0, s, V, n, Nx, M, bx, bt, ntv, P);
  KCHK();
}
template <class T>
void launch_noise(hipStream_t s, cx<T>* out, int64_t n, int nrhs, int kind, uint64_t seed,
                  int purpose, int level, int64_t index0) {
  if (n <= 0 || nrhs <= 0) return;
  const uint64_t base = mix64(seed + kGolden);
  unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 4096);
  hipLaunchKernelGGL(k_noise<T>, dim3(gx, nrhs), dim3(NT), 0, s, out, n, kind, base, purpose, level,
                     index0);
  KCHK();
}
template void launch_noise<double>(hipStream_t, cd*, int64_t, int, int, uint64_t, int, int, int64_t);
template void launch_noise<float>(hipStream_t, cf*, int64_t, int, int, uint64_t, int, int, int64_t);

// Workgroups of k_wilson_strip<T, *, SPT> with `threads` threads the whole
// device holds at once, from the runtime's occupancy calculator (per device,
// cached).
template <class T, int SPT>
int64_t strip_capacity(int threads) {
  static std::atomic<int64_t> cap[64][5];
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  require(dev >= 0 && dev < 64, "device index out of range");
  const int slot = threads / 64;  // 1 .. 4
  int64_t c = cap[dev][slot].load(std::memory_order_relaxed);
  if (c == 0) {
    int per_cu = 0, cus = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_wilson_strip<T, 8, SPT>, threads,
                                                        0));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    c = (int64_t)std::max(per_cu, 1) * std::max(cus, 1);
    cap[dev][slot].store(c, std::memory_order_relaxed);
  }
  return c;
}

template <class T, int SPT>
void launch_wilson_strip(hipStream_t s, const cx<T>* links, T diag, int Lx, int Lt, int nrhs, const cx<T>* x,
                         cx<T>* y, const cx<T>* b, const int* active) {
  // strip height: the smallest that keeps every workgroup resident at once
  // (more, shorter strips hide more latency; a second round of workgroups
  // costs more than it hides)
  const int threads = Lx / SPT;
  const int64_t cap = strip_capacity<T, SPT>(threads);
  int tr = 0;
  for (int c : {1, 2, 4, 8, 16, 32, 64})
    if (Lt % c == 0) {
      tr = c;
      if ((int64_t)(Lt / c) * nrhs <= cap) break;
    }
  const dim3 g(Lt / tr, nrhs), blk(threads);
  switch (tr) {
    case 32: hipLaunchKernelGGL((k_wilson_strip<T, 32, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    case 64: hipLaunchKernelGGL((k_wilson_strip<T, 64, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    case 1: hipLaunchKernelGGL((k_wilson_strip<T, 1, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    case 2: hipLaunchKernelGGL((k_wilson_strip<T, 2, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    case 4: hipLaunchKernelGGL((k_wilson_strip<T, 4, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    case 8: hipLaunchKernelGGL((k_wilson_strip<T, 8, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
    default: hipLaunchKernelGGL((k_wilson_strip<T, 16, SPT>), g, blk, 0, s, links, diag, Lx, Lt, x, y, b, active); break;
  }
}

template <class T>
void launch_wilson(hipStream_t s, const cx<T>* links, T diag, int Lx, int Lt, int nrhs,
                   const cx<T>* x, cx<T>* y, const cx<T>* b, const int* active) {
  const int64_t V = (int64_t)Lx * Lt;
  // row strips when a row splits into 1, 2 or 4 slices of a 64-multiple of
  // at most NT sites; the thread-per-site kernel otherwise
  if (Lx % 64 == 0 && Lx <= NT) {
    launch_wilson_strip<T, 1>(s, links, diag, Lx, Lt, nrhs, x, y, b, active);
  } else if (Lx % 128 == 0 && Lx <= 2 * NT) {
    launch_wilson_strip<T, 2>(s, links, diag, Lx, Lt, nrhs, x, y, b, active);
  } else if (Lx % 256 == 0 && Lx <= 4 * NT) {
    launch_wilson_strip<T, 4>(s, links, diag, Lx, Lt, nrhs, x, y, b, active);
  } else {
    hipLaunchKernelGGL(k_wilson<T>, dim3(grid1(V), nrhs), dim3(NT), 0, s, links, diag, Lx, Lt, x, y, b,
                       active);
  }
  KCHK();
}
template void launch_wilson<double>(hipStream_t, const cd*, double, int, int, int, const cd*, cd*,
                                    const cd*, const int*);
template void launch_wilson<float>(hipStream_t, const cf*, float, int, int, int, const cf*, cf*,
                                   const cf*, const int*);

void launch_fine_blocks(hipStream_t s, const cd* links, double diag, int Lx, int Lt, cd* blocks) {
  hipLaunchKernelGGL(k_fine_blocks, dim3(grid1((int64_t)Lx * Lt)), dim3(NT), 0, s, links, diag, Lx,
                     Lt, blocks);
  KCHK();
}

template <class T>
void launch_stencil(hipStream_t s, const cx<T>* blocks, int Nx, int Nt, int M, int nrhs,
                    const cx<T>* x, cx<T>* y, const cx<T>* b, const int* active) {
  const int64_t n = (int64_t)Nx * Nt * M;
  const int64_t sites = (int64_t)Nx * Nt;
  dim3 g(grid1(n), nrhs);
  // LDS-staged variant: RHS per workgroup chosen to give ~2048 workgroups
  int rpc = (int)std::min<int64_t>(std::min(nrhs, 64), std::max<int64_t>(1, (int64_t)nrhs * sites / 2048));
  const int rpw = M > 0 ? NT / M : 1;
  rpc = std::min(((rpc + rpw - 1) / rpw) * rpw, std::max(nrhs, 1));
  dim3 gl((unsigned)sites, (nrhs + rpc - 1) / rpc);
  switch (M) {
    case 2: hipLaunchKernelGGL((k_stencil<T, 2>), g, dim3(NT), 0, s, blocks, Nx, Nt, x, y, b, active); break;
    case 4: hipLaunchKernelGGL((k_stencil_lds<T, 4>), gl, dim3(NT), 0, s, blocks, Nx, Nt, nrhs, rpc, x, y, b, active); break;
    case 8: hipLaunchKernelGGL((k_stencil_lds<T, 8>), gl, dim3(NT), 0, s, blocks, Nx, Nt, nrhs, rpc, x, y, b, active); break;
    case 16:
      hipLaunchKernelGGL(k_stencil_mfma<T>, dim3((unsigned)sites, (nrhs + 15) / 16), dim3(NT), 0, s, blocks,
                         Nx, Nt, nrhs, x, y, b, active);
      break;
    case 32: hipLaunchKernelGGL((k_stencil<T, 32>), g, dim3(NT), 0, s, blocks, Nx, Nt, x, y, b, active); break;
    default: throw Error(MGM_EINVAL, "block stencil: dofs per site must be 2, 4, 8, 16 or 32");
  }
  KCHK();
}
template void launch_stencil<double>(hipStream_t, const cd*, int, int, int, int, const cd*, cd*,
                                     const cd*, const int*);
template void launch_stencil<float>(hipStream_t, const cf*, int, int, int, int, const cf*, cf*,
                                    const cf*, const int*);

void launch_dense_apply_h(hipStream_t s, const chalf* A, int64_t n, int nrhs, const cf* x, cf* y,
                          const int* active) {
  require(n % (32 * DH_W) == 0, "FP16 dense apply: n must be a multiple of 256");
  if (nrhs <= 0) return;
  // four row tiles per workgroup while that still gives 256 workgroups
  const unsigned nt = (unsigned)((nrhs + 15) / 16);
  if ((n / 64) * nt >= 256)
    hipLaunchKernelGGL(k_dense_h<4>, dim3((unsigned)(n / 64), nt), dim3(64 * DH_W), 0, s, A, n, nrhs, x, y,
                       active);
  else
    hipLaunchKernelGGL(k_dense_h<1>, dim3((unsigned)(n / 16), nt), dim3(64 * DH_W), 0, s, A, n, nrhs, x, y,
                       active);
  KCHK();
}

void launch_to_half_checked(hipStream_t s, const cd* in, chalf* out, int64_t count, int* overflow) {
  hipLaunchKernelGGL(k_to_half_checked, dim3(grid1(count)), dim3(NT), 0, s, in, out, count, overflow);
  KCHK();
}

void launch_to_half(hipStream_t s, const cd* in, chalf* out, int64_t count) {
  hipLaunchKernelGGL(k_to_half, dim3(grid1(count)), dim3(NT), 0, s, in, out, count);
  KCHK();
}

void launch_stencil_h(hipStream_t s, const chalf* blocks, int Nx, int Nt, int nrhs, const cf* x, cf* y,
                      const cf* b, const int* active) {
  hipLaunchKernelGGL(k_stencil_h, dim3((unsigned)((int64_t)Nx * Nt), (nrhs + 15) / 16), dim3(NT), 0, s,
                     blocks, Nx, Nt, nrhs, x, y, b, active);
  KCHK();
}

void launch_sap2_premul(hipStream_t s, const cd* blocks, const cd* inv, int Nx, int nblk, chalf* M) {
  const int64_t cnt = (int64_t)nblk * 6 * 32 * CM;
  hipLaunchKernelGGL(k_sap2_premul, dim3((unsigned)((cnt + NT - 1) / NT)), dim3(NT), 0, s, blocks, inv, Nx, nblk, M);
  KCHK();
}

void launch_sap4_premul(hipStream_t s, const cd* blocks, const cd* inv, int Nx, int nblk, cd* M) {
  const int64_t cnt = (int64_t)nblk * 8 * 64 * CM;
  hipLaunchKernelGGL(k_sap4_premul, dim3((unsigned)((cnt + NT - 1) / NT)), dim3(NT), 0, s, blocks, inv, Nx, nblk, M);
  KCHK();
}

// 16-RHS tiles per workgroup of the FP16 2x2 sweep: one (two waves) spreads
// a 32-RHS sweep over 256 workgroups instead of 128; measured inside the
// step against two: 94.0 vs 93.5 estimates/s (back to back at 64 RHS 5.9 vs
// 5.8 us)
constexpr int SAP4_TILES_PER_WG = 1;
void launch_sap4p_h(hipStream_t s, const chalf* M, const chalf* inv, int Nx, int Nt, const int* blist, int nb,
                    int nrhs, bool first, const cf* r, cf* rho, cf* x, const int* active, const chalf* hP,
                    const cf* ec) {
  if (nb <= 0 || nrhs <= 0) return;
  constexpr int TPW = SAP4_TILES_PER_WG;  // 16-RHS tiles per workgroup (two waves each)
  const dim3 g(nb, ((nrhs + 15) / 16 + TPW - 1) / TPW);
  require(!ec || (first && hP), "FP16 2x2 SAP: the halo from the coarse correction needs the first sweep and P");
  if (ec)
    hipLaunchKernelGGL(k_sap4p_hc, g, dim3(128 * TPW), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active, hP,
                       ec);
  else if (first)
    hipLaunchKernelGGL(k_sap4p_h<true>, g, dim3(128 * TPW), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  else
    hipLaunchKernelGGL(k_sap4p_h<false>, g, dim3(128 * TPW), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  KCHK();
}

template <class T>
void launch_sap4p(hipStream_t s, const cx<T>* M, const cx<T>* inv, int Nx, int Nt, const int* blist, int nb,
                  int nrhs, bool first, const cx<T>* r, cx<T>* rho, cx<T>* x, const int* active) {
  if (nb <= 0 || nrhs <= 0) return;
  const dim3 g(nb, ((nrhs + 15) / 16 + 1) / 2);
  if (first)
    hipLaunchKernelGGL((k_sap4p<T, true>), g, dim3(NT), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  else
    hipLaunchKernelGGL((k_sap4p<T, false>), g, dim3(NT), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  KCHK();
}
template void launch_sap4p<double>(hipStream_t, const cd*, const cd*, int, int, const int*, int, int, bool,
                                   const cd*, cd*, cd*, const int*);
template void launch_sap4p<float>(hipStream_t, const cf*, const cf*, int, int, const int*, int, int, bool,
                                  const cf*, cf*, cf*, const int*);

void launch_sap2p_h(hipStream_t s, const chalf* M, const chalf* inv, int Nx, int Nt, const int* blist, int nb,
                    int nrhs, bool first, const cf* r, cf* rho, cf* x, const int* active) {
  if (nb <= 0) return;
  const dim3 g(nb, ((nrhs + 15) / 16 + 3) / 4);
  if (first)
    hipLaunchKernelGGL(k_sap2p_h<true>, g, dim3(NT), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  else
    hipLaunchKernelGGL(k_sap2p_h<false>, g, dim3(NT), 0, s, M, inv, Nx, Nt, blist, nrhs, r, rho, x, active);
  KCHK();
}

void launch_sap_h(hipStream_t s, const chalf* blocks, const chalf* inv, int Nx, int Nt, int sbx, int sbt,
                  const int* blist, int nb, int nrhs, const cf* r, cf* x, const int* active, const chalf* hP,
                  const cf* ec) {
  if (nb <= 0) return;
  if (ec) {
    require(hP && sbx == 1 && sbt == 1, "FP16 SAP: the halo from the coarse correction needs single sites and P");
    hipLaunchKernelGGL(k_sap_hc, dim3(nb, (nrhs + 15) / 16), dim3(NT), 0, s, blocks, inv, Nx, Nt, blist, nrhs, r, x,
                       active, hP, ec);
    KCHK();
    return;
  }
  // (2x1 blocks take the premultiplied sweep, launch_sap2p_h)
  if (sbx == 1 && sbt == 1)
    hipLaunchKernelGGL(k_sap_h, dim3(nb, (nrhs + 15) / 16), dim3(NT), 0, s, blocks, inv, Nx, Nt, blist, nrhs,
                       r, x, active);
  else
    throw Error(MGM_EINVAL, "FP16 SAP: single-site blocks only (2x1 blocks use the premultiplied sweep)");
  KCHK();
}

template <class T>
void launch_restrict(hipStream_t s, const cx<T>* P, int Nx, int Nt, int M, int bx, int bt, int ntv,
                     int nrhs, const cx<T>* xf, cx<T>* xc, const int* active) {
  const int64_t nc = (int64_t)(Nx / bx) * (Nt / bt) * 2 * ntv;
  const dim3 g(grid1(nc), nrhs);
  if (M == 2 && bx == 4 && bt == 4 && ntv == 8)
    hipLaunchKernelGGL((k_restrict_t<T, 2, 4, 4, 8, false, RT_RESTRICT_FINE>),
                       dim3(grid1(nc), (nrhs + RT_RESTRICT_FINE - 1) / RT_RESTRICT_FINE), dim3(NT), 0, s, P, Nx,
                       Nt, xf, xc, active, nrhs);
  else if (M == 16 && bx == 2 && bt == 2 && ntv == 8)
    hipLaunchKernelGGL((k_restrict_t<T, 16, 2, 2, 8, false, RT_RESTRICT_COARSE>),
                       dim3(grid1(nc), (nrhs + RT_RESTRICT_COARSE - 1) / RT_RESTRICT_COARSE), dim3(NT), 0, s, P,
                       Nx, Nt, xf, xc, active, nrhs);
  else
    hipLaunchKernelGGL(k_restrict<T>, g, dim3(NT), 0, s, P, Nx, Nt, M, bx, bt, ntv, xf, xc, active);
  KCHK();
}
template void launch_restrict<double>(hipStream_t, const cd*, int, int, int, int, int, int, int,
                                      const cd*, cd*, const int*);
template void launch_restrict<float>(hipStream_t, const cf*, int, int, int, int, int, int, int,
                                     const cf*, cf*, const int*);

template <class T>
void launch_prolong(hipStream_t s, const cx<T>* P, int Nx, int Nt, int M, int bx, int bt, int ntv,
                    int nrhs, const cx<T>* xc, cx<T>* yf, int accumulate, const int* active) {
  const int64_t n = (int64_t)Nx * Nt * M;
  const dim3 g(grid1(n), nrhs);
  if (M == 2 && bx == 4 && bt == 4 && ntv == 8)
    hipLaunchKernelGGL((k_prolong_t<T, 2, 4, 4, 8>), g, dim3(NT), 0, s, P, Nx, Nt, xc, yf, accumulate,
                       active);
  else if (M == 16 && bx == 2 && bt == 2 && ntv == 8)
    hipLaunchKernelGGL((k_prolong_t<T, 16, 2, 2, 8>), g, dim3(NT), 0, s, P, Nx, Nt, xc, yf, accumulate,
                       active);
  else
    hipLaunchKernelGGL(k_prolong<T>, g, dim3(NT), 0, s, P, Nx, Nt, M, bx, bt, ntv, xc, yf, accumulate,
                       active);
  KCHK();
}
template void launch_prolong<double>(hipStream_t, const cd*, int, int, int, int, int, int, int,
                                     const cd*, cd*, int, const int*);
template void launch_prolong<float>(hipStream_t, const cf*, int, int, int, int, int, int, int,
                                    const cf*, cf*, int, const int*);

void launch_sap0_blk(hipStream_t s, const cf* B, const cf* inv, int Nx, int Nt, const int* blist, int nb,
                     int nrhs, const cf* r, cf* x, const int* active, cd* x64) {
  if (nb <= 0) return;
  // one wave per 16-RHS tile, at most four per workgroup: no idle waves below 64 RHS
  const int nt = (nrhs + 15) / 16, w = std::min(4, nt);
  hipLaunchKernelGGL((k_sap0_mfma<float, true>), dim3(nb, (nt + w - 1) / w), dim3(64 * w), 0, s, B, inv, Nx, Nt,
                     blist, nrhs, r, x, active, x64);
  KCHK();
}

void launch_restrict_blk(hipStream_t s, const cf* P, int Nx, int Nt, int nrhs, const cf* xf, cf* xc,
                         const int* active) {
  const int64_t nc = (int64_t)(Nx / 4) * (Nt / 4) * 2 * 8;
  hipLaunchKernelGGL((k_restrict_t<float, 2, 4, 4, 8, true, RT_RESTRICT_FINE>),
                     dim3(grid1(nc), (nrhs + RT_RESTRICT_FINE - 1) / RT_RESTRICT_FINE), dim3(NT), 0, s, P, Nx, Nt,
                     xf, xc, active, nrhs);
  KCHK();
}

void launch_prolong_blk(hipStream_t s, const cf* P, int Nx, int Nt, int nrhs, const cf* xc, cf* yf,
                        const int* active) {
  const int64_t n = (int64_t)Nx * Nt * 2;
  hipLaunchKernelGGL((k_prolong_t<float, 2, 4, 4, 8, true>), dim3(grid1(n), nrhs), dim3(NT), 0, s, P, Nx, Nt, xc,
                     yf, 0, active);
  KCHK();
}

void launch_galerkin(hipStream_t s, const cd* Bf, int Nx, int Nt, int Mf, const cd* P, int bx,
                     int bt, int ntv, cd* Bc) {
  const int64_t tot = (int64_t)(Nx / bx) * (Nt / bt) * 5 * (2 * ntv) * (2 * ntv);
  hipLaunchKernelGGL(k_galerkin, dim3(grid1(tot)), dim3(NT), 0, s, Bf, Nx, Nt, Mf, P, bx, bt, ntv, Bc);
  KCHK();
}

void launch_sap_extract(hipStream_t s, const cd* B, int Nx, int Nt, int M, int sbx, int sbt,
                        cd* out) {
  const int64_t K = (int64_t)sbx * sbt * M;
  const int64_t tot = (int64_t)(Nx / sbx) * (Nt / sbt) * K * K;
  hipLaunchKernelGGL(k_sap_extract, dim3(grid1(tot)), dim3(NT), 0, s, B, Nx, Nt, M, sbx, sbt, out);
  KCHK();
}

void launch_small_inverse(hipStream_t s, cd* mats, int K, int count, int* fail) {
  require(K >= 1 && K <= 64, "SAP block too large: sbx*sbt*M must be <= 64");
  if (K <= 32)
    hipLaunchKernelGGL(k_small_inverse<32>, dim3(count), dim3(NT), 0, s, mats, K, fail);
  else
    hipLaunchKernelGGL(k_small_inverse<64>, dim3(count), dim3(NT), 0, s, mats, K, fail);
  KCHK();
}

template <class T>
void launch_sap_sweep(hipStream_t s, const cx<T>* B, const cx<T>* inv, int Nx, int Nt, int M,
                      int sbx, int sbt, const int* blist, int nb, int nrhs, const cx<T>* r,
                      cx<T>* x, const int* active, cd* x64) {
  if (nb <= 0) return;
  require(!x64 || (M == 2 && sbx == 4 && sbt == 4), "SAP: an FP64 copy of the result only with 4x4 blocks");
  const int K = sbx * sbt * M;
  require(K <= 32, "SAP block too large");
  if (M == CM && sbx == 1 && sbt == 1) {
    hipLaunchKernelGGL(k_sap_mfma<T>, dim3(nb, (nrhs + 15) / 16), dim3(NT), 0, s, B, inv, Nx, Nt, blist,
                       nrhs, r, x, active);
    KCHK();
    return;
  }
  if (M == CM && sbx == 2 && sbt == 1) {
    hipLaunchKernelGGL(k_sap2_mfma<T>, dim3(nb, (nrhs + 15) / 16), dim3(NT), 0, s, B, inv, Nx, Nt, blist,
                       nrhs, r, x, active);
    KCHK();
    return;
  }
  if (M == 2 && sbx == 4 && sbt == 4) {
    hipLaunchKernelGGL(k_sap0_mfma<T>, dim3(nb, (nrhs + 63) / 64), dim3(NT), 0, s, B, inv, Nx, Nt, blist,
                       nrhs, r, x, active, x64);
    KCHK();
    return;
  }
  const int rpw = NT / K;
  // RHS per workgroup: enough workgroups (~2048, 8 per CU) to hide the
  // memory latency of each round, at the price of re-reading the block's
  // matrices from L2 once per workgroup
  int rpc = (int)std::min<int64_t>(std::min(nrhs, 64), std::max<int64_t>(1, (int64_t)nrhs * nb / 2048));
  rpc = std::max(rpc, rpw);
  rpc = ((rpc + rpw - 1) / rpw) * rpw;
  hipLaunchKernelGGL(k_sap_sweep<T>, dim3(nb, (nrhs + rpc - 1) / rpc), dim3(NT), 0, s, B, inv, Nx, Nt,
                     M, sbx, sbt, blist, nrhs, rpc, r, x, active);
  KCHK();
}
template void launch_sap_sweep<double>(hipStream_t, const cd*, const cd*, int, int, int, int, int,
                                       const int*, int, int, const cd*, cd*, const int*, cd*);
template void launch_sap_sweep<float>(hipStream_t, const cf*, const cf*, int, int, int, int, int,
                                      const int*, int, int, const cf*, cf*, const int*, cd*);

void launch_dense_from_stencil(hipStream_t s, const cd* B, int Nx, int Nt, int M, cd* A) {
  const int64_t n = (int64_t)Nx * Nt * M;
  HIPCHK(hipMemsetAsync(A, 0, sizeof(cd) * n * n, s));
  hipLaunchKernelGGL(k_dense_from_stencil, dim3(grid1(n)), dim3(NT), 0, s, B, Nx, Nt, M, A);
  KCHK();
}

// In-place Gauss-Jordan with partial pivoting (blocked for n a multiple of 64,
// n >= 512); the column unscrambling is a gather into `out`.  Returns 0, or 1
// on a zero pivot.
int dense_inverse(hipStream_t s, cd* A, int64_t n, cd* out) {
  DevBuf perm, piv, fcol, fail, pi;
  perm.ensure(sizeof(int) * n);
  piv.ensure(sizeof(cd));
  fcol.ensure(sizeof(cd) * n);
  fail.ensure(sizeof(int));
  pi.ensure(sizeof(int) * n);
  HIPCHK(hipMemsetAsync(fail.p, 0, sizeof(int), s));
  if (n % GJ_NB == 0 && n >= 8 * GJ_NB) {
    // blocked: panel steps on 64 columns, then swaps and a rank-64 update
    DevBuf T;
    T.ensure(sizeof(cd) * GJ_NB * n);
    const unsigned tiles = (unsigned)(n / 64);
    for (int64_t c0 = 0; c0 < n; c0 += GJ_NB) {
      for (int64_t k = c0; k < c0 + GJ_NB; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(NT), 0, s, A, n, k, perm.as<int>(), piv.as<cd>(),
                           fail.as<int>());
        hipLaunchKernelGGL(k_gj_swap_scale_panel, dim3(1), dim3(NT), 0, s, A, n, k, c0, perm.as<int>(),
                           piv.as<cd>());
        hipLaunchKernelGGL(k_gj_col, dim3(grid1(n)), dim3(NT), 0, s, A, n, k, fcol.as<cd>());
        hipLaunchKernelGGL(k_gj_eliminate_panel, dim3(grid1(n * GJ_NB)), dim3(NT), 0, s, A, n, k, c0,
                           fcol.as<cd>());
      }
      hipLaunchKernelGGL(k_gj_swaps_rest, dim3(grid1(n)), dim3(NT), 0, s, A, n, c0, perm.as<int>(),
                         T.as<cd>());
      hipLaunchKernelGGL(k_gj_update, dim3(tiles, tiles), dim3(NT), 0, s, A, n, c0, T.as<cd>());
      KCHK();
    }
  } else {
    for (int64_t k = 0; k < n; ++k) {
      hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(NT), 0, s, A, n, k, perm.as<int>(), piv.as<cd>(),
                         fail.as<int>());
      hipLaunchKernelGGL(k_gj_swap_scale, dim3(grid1(n)), dim3(NT), 0, s, A, n, k, perm.as<int>(),
                         piv.as<cd>());
      hipLaunchKernelGGL(k_gj_col, dim3(grid1(n)), dim3(NT), 0, s, A, n, k, fcol.as<cd>());
      hipLaunchKernelGGL(k_gj_eliminate, dim3(grid1(n), (unsigned)n), dim3(NT), 0, s, A, n, k,
                         fcol.as<cd>());
      KCHK();
    }
  }
  std::vector<int> hperm(n), hpi(n);
  int hfail = 0;
  HIPCHK(hipMemcpyAsync(hperm.data(), perm.p, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&hfail, fail.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hfail) return 1;
  for (int64_t j = 0; j < n; ++j) hpi[j] = (int)j;
  for (int64_t k = n - 1; k >= 0; --k)
    if (hperm[k] != k) std::swap(hpi[k], hpi[hperm[k]]);
  HIPCHK(hipMemcpyAsync(pi.p, hpi.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gather_cols, dim3(grid1(n), (unsigned)n), dim3(NT), 0, s, A, n, pi.as<int>(),
                     out);
  KCHK();
  HIPCHK(hipStreamSynchronize(s));
  return 0;
}

void launch_diag_sum(hipStream_t s, const cd* A, int64_t n, cd* out) {
  hipLaunchKernelGGL(k_diag_sum, dim3(1), dim3(NT), 0, s, A, n, out);
  KCHK();
}

template <class T>
void launch_dense_apply(hipStream_t s, const cx<T>* A, int64_t n, int nrhs, const cx<T>* x,
                        cx<T>* y, const int* active, DevBuf* scratch) {
  if (n % 16 == 0 && scratch) {
    // matrix cores: 16 x 16 tiles, k split over 4 waves and then over
    // workgroups until ~1024 workgroups (k ranges of at least 256)
    const unsigned ti = (unsigned)(n / 16), tr = (unsigned)((nrhs + 15) / 16);
    int ks = 1;
    while (ks < 32 && (int64_t)ti * tr * ks < 1024 && n / (2 * ks) >= 256) ks *= 2;
    const int64_t klen = ((n + ks - 1) / ks + 15) / 16 * 16;
    ks = (int)((n + klen - 1) / klen);
    cx<T>* part = nullptr;
    if (ks > 1) {
      scratch->ensure(sizeof(cx<T>) * (size_t)ks * nrhs * n);
      part = scratch->as<cx<T>>();
    }
    hipLaunchKernelGGL(k_dense_mfma<T>, dim3(ti, tr, ks), dim3(NT), 0, s, A, n, nrhs, klen, x, y, part,
                       active);
    KCHK();
    if (ks > 1) {
      hipLaunchKernelGGL(k_dense_reduce<T>, dim3(grid1(n), nrhs), dim3(NT), 0, s, part, ks, n, nrhs, y,
                         active);
      KCHK();
    }
    return;
  }
  const unsigned tiles_i = (unsigned)((n + 63) / 64), tiles_r = (unsigned)((nrhs + 15) / 16);
  // split k until ~1024 workgroups, keeping k ranges of at least 128
  int ks = 1;
  while (ks < 16 && (int64_t)tiles_i * tiles_r * ks < 1024 && n / (2 * ks) >= 128) ks *= 2;
  if (!scratch) ks = 1;
  const int64_t klen = ((n + ks - 1) / ks + 31) / 32 * 32;
  ks = (int)((n + klen - 1) / klen);
  cx<T>* part = nullptr;
  if (ks > 1) {
    scratch->ensure(sizeof(cx<T>) * (size_t)ks * nrhs * n);
    part = scratch->as<cx<T>>();
  }
  hipLaunchKernelGGL(k_dense_apply<T>, dim3(tiles_i, tiles_r, ks), dim3(NT), 0, s, A, n, nrhs, klen, x, y,
                     part, active);
  KCHK();
  if (ks > 1) {
    hipLaunchKernelGGL(k_dense_reduce<T>, dim3(grid1(n), nrhs), dim3(NT), 0, s, part, ks, n, nrhs, y, active);
    KCHK();
  }
}
template void launch_dense_apply<double>(hipStream_t, const cd*, int64_t, int, const cd*, cd*,
                                         const int*, DevBuf*);
template void launch_dense_apply<float>(hipStream_t, const cf*, int64_t, int, const cf*, cf*,
                                        const int*, DevBuf*);

}  // namespace mgm
