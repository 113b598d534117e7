// Learned initial guess: a 4-layer 3x3 convolutional network on the fine
// lattice (4 -> 32 -> 32 -> 32 -> 4 channels, tanh after the first three),
// trained on pairs (b, D^{-1} b) with its own forward, backward and Adam
// kernels.  It only changes where a solve starts; every solve still runs to
// its FP64 tolerance.
//
// Layouts.  Activations are channel-last FP32 [nb][Lt][Lx][C]; for C = 4 this
// is the memory order of a complex128 vector (site, spin, re/im), so the
// network's input and output are element-wise conversions of solver vectors.
// Parameters are kept in the packing W1 b1 .. W4 b4, W[co][ci][dt][dx]; each
// layer also has two packed copies: forward [co][tap*cin + ci] and, for the
// gradient with respect to the input (the transposed convolution, taps
// mirrored), [ci][tap'*cout + co] with tap' = 8 - tap.
//
// Convolutions are implicit GEMMs on the FP32 matrix cores: M = 16 sites
// along x, N = 16 output channels, K = 4 (tap, channel) pairs per step.  A
// workgroup stages a 16x16-site tile with a one-site halo (the lattice
// boundary conditions applied while loading) and the layer's weights in LDS;
// each of its 4 waves owns 4 rows of 16 sites.
#include <cmath>

#include "internal.h"

namespace mgm {
namespace {

constexpr int TE = 16;      // tile edge (sites)
constexpr int HE = TE + 2;  // tile edge with halo
constexpr int CNT = 256;    // threads per workgroup

typedef float f4 __attribute__((ext_vector_type(4)));

// 16x16x4 FP32 matrix-core step: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element v of its result is D[4(l/16) + v][l%16].
__device__ __forceinline__ f4 mma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

enum { EPI_NONE = 0, EPI_TANH = 1, EPI_DTANH = 2 };

// Stage the (TE+2)^2 halo tile of a C-channel field into LDS (site stride
// C + 1): x periodic; t periodic, or antiperiodic (a value fetched across the
// t boundary changes sign).
template <int C>
__device__ __forceinline__ void load_tile(const float* __restrict__ in, int Lx, int Lt, int anti,
                                          int b, int t0, int x0, float* xs) {
  constexpr int S = C + 1;
  const float* base = in + (int64_t)b * Lx * Lt * C;
  for (int e = threadIdx.x; e < HE * HE * C; e += CNT) {
    const int site = e / C, ch = e - site * C;
    const int r = site / HE, cc = site - r * HE;
    int t = t0 + r - 1, x = x0 + cc - 1;
    float sg = 1.f;
    if (t < 0) {
      t += Lt;
      sg = anti ? -1.f : 1.f;
    } else if (t >= Lt) {
      t -= Lt;
      sg = anti ? -1.f : 1.f;
    }
    if (x < 0)
      x += Lx;
    else if (x >= Lx)
      x -= Lx;
    xs[site * S + ch] = sg * base[((int64_t)t * Lx + x) * C + ch];
  }
}

// out[site][n] = epi( sum_{tap, c} in[site + off(tap)][c] wp[n][tap*CIN + c] + bias[n] )
// off(tap) = (tap/3 - 1, tap%3 - 1) in (t, x).  EPI_DTANH multiplies by
// 1 - h[site][n]^2 instead of adding a bias (backward through tanh).
template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(CNT) k_conv(const float* __restrict__ in, int Lx, int Lt, int anti,
                                              const float* __restrict__ wp,
                                              const float* __restrict__ bias,
                                              const float* __restrict__ h, float* __restrict__ out) {
  constexpr int K = 9 * CIN;
  constexpr int KS = K + 1;
  constexpr int S = CIN + 1;
  constexpr int NB = (COUT + 15) / 16;
  __shared__ float xs[HE * HE * S];
  __shared__ float ws[COUT * KS];
  const int x0 = blockIdx.x * TE, t0 = blockIdx.y * TE, b = blockIdx.z;
  load_tile<CIN>(in, Lx, Lt, anti, b, t0, x0, xs);
  for (int e = threadIdx.x; e < COUT * K; e += CNT) {
    const int n = e / K;
    ws[n * KS + (e - n * K)] = wp[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  f4 acc[4][NB];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + q;
    const int tap = k / CIN, ch = k - tap * CIN;
    const int dt = tap / 3, dx = tap - 3 * dt;
    float bw[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 16 + i;
      bw[nb] = n < COUT ? ws[n * KS + k] : 0.f;
    }
    const float* xr = xs + ((wave * 4 + dt) * HE + i + dx) * S + ch;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const float a = xr[rr * HE * S];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = mma4(a, bw[nb], acc[rr][nb]);
    }
  }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int n = nb * 16 + i;
    if (n >= COUT) continue;
    const float bn = bias ? bias[n] : 0.f;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int64_t row = ((int64_t)b * Lt + t0 + wave * 4 + rr) * Lx + x0 + 4 * q;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t o = (row + v) * COUT + n;
        float z = acc[rr][nb][v] + bn;
        if (EPI == EPI_TANH) z = tanhf(z);
        if (EPI == EPI_DTANH) {
          const float hv = h[o];
          z *= 1.f - hv * hv;
        }
        out[o] = z;
      }
    }
  }
}

// The same convolution with FP16 activations and weights on the FP16 matrix
// cores (FP32 accumulation; bias, tanh and the output rounding in FP32 ->
// FP16).  K index k = tap * CIN + ch in chunks of 16 or 32 (padded with zeros
// past 9 * CIN).
typedef _Float16 hv4 __attribute__((ext_vector_type(4)));

typedef _Float16 hv8 __attribute__((ext_vector_type(8)));

// words of W halves (4: 8 bytes, 8: 16 bytes)
template <int W> struct HWord;
template <> struct HWord<4> { typedef hv4 T; };
template <> struct HWord<8> { typedef hv8 T; };

// Halo tile into LDS with site stride S (halves), in words of W channels.
template <int C, int S, int W>
__device__ __forceinline__ void load_tile_h(const _Float16* __restrict__ in, int Lx, int Lt, int anti, int b,
                                            int t0, int x0, _Float16* xs) {
  typedef typename HWord<W>::T word;
  constexpr int CQ = C / W;  // words per site
  static_assert(C % W == 0 && S % W == 0, "channels in whole words");
  const _Float16* base = in + (int64_t)b * Lx * Lt * C;
  for (int e = threadIdx.x; e < HE * HE * CQ; e += CNT) {
    const int site = e / CQ, w = e - site * CQ;
    const int r = site / HE, cc = site - r * HE;
    int t = t0 + r - 1, x = x0 + cc - 1;
    bool neg = false;
    if (t < 0) {
      t += Lt;
      neg = anti;
    } else if (t >= Lt) {
      t -= Lt;
      neg = anti;
    }
    if (x < 0)
      x += Lx;
    else if (x >= Lx)
      x -= Lx;
    word v = *reinterpret_cast<const word*>(base + ((int64_t)t * Lx + x) * C + W * w);
    if (neg) v = -v;
    *reinterpret_cast<word*>(xs + site * S + W * w) = v;
  }
}

// FP16 matrix-core step on words of W halves: 16x16x16 (W = 4) or the
// 16x16x32 shape of gfx950 (W = 8).  Lane l supplies the K slots
// W (l/16) .. W (l/16) + W - 1 of row l%16 of A and of column l%16 of B; the
// hardware pairs equal slots of A and B, so the product sums over all K
// whatever order it takes them in.  Result element v: D[4(l/16) + v][l%16].
template <int W>
__device__ __forceinline__ f4 hmma_w(typename HWord<W>::T a, typename HWord<W>::T b, f4 c) {
  if constexpr (W == 8)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// Global traffic in words: the halo tile and the weights are loaded as words
// of W halves (W = 8 when CIN is a multiple of 8: then the 16x16x32 shape),
// and the 16 x 16 x COUT output tile is transposed through LDS (reusing the
// tile's space) so that it is stored as contiguous 8-byte words.
template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(CNT) k_conv_h(const _Float16* __restrict__ in, int Lx, int Lt, int anti,
                                                const _Float16* __restrict__ wp, const float* __restrict__ bias,
                                                _Float16* __restrict__ out) {
  constexpr int W = CIN % 8 == 0 ? 8 : 4;  // K slots per lane
  typedef typename HWord<W>::T word;
  constexpr int KW = 4 * W;                // K per matrix-core step
  constexpr int K = 9 * CIN;
  constexpr int KC = (K + KW - 1) / KW;    // K chunks (zero-padded past K)
  constexpr int KS = KC * KW + W;          // LDS row stride of the weights (halves)
  constexpr int S = CIN + W;               // LDS site stride of the tile
  constexpr int NB = (COUT + 15) / 16;
  constexpr int OS = COUT + 4;             // LDS site stride of the output tile
  constexpr int XN = HE * HE * S, WN = COUT * KS, ON = TE * TE * OS;
  constexpr int SM = XN + WN > ON ? XN + WN : ON;
  static_assert(CIN % 4 == 0 && COUT % 4 == 0 && K % W == 0 && KS % W == 0 && S % W == 0 && XN % W == 0,
                "whole LDS words");
  __shared__ __attribute__((aligned(16))) _Float16 smem[SM];
  _Float16* xs = smem;
  _Float16* ws = smem + XN;
  const int x0 = blockIdx.x * TE, t0 = blockIdx.y * TE, b = blockIdx.z;
  load_tile_h<CIN, S, W>(in, Lx, Lt, anti, b, t0, x0, xs);
  word zero;
#pragma unroll
  for (int j = 0; j < W; ++j) zero[j] = (_Float16)0;
  constexpr int RW = KC * KW / W;  // words per weight row
  for (int e = threadIdx.x; e < COUT * RW; e += CNT) {
    const int n = e / RW, k = W * (e - n * RW);
    // K is a multiple of W: a word is wholly inside or wholly past K
    *reinterpret_cast<word*>(ws + n * KS + k) = k < K ? *reinterpret_cast<const word*>(wp + n * K + k) : zero;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  f4 acc[4][NB];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = f4{0.f, 0.f, 0.f, 0.f};
  for (int kc = 0; kc < KC; ++kc) {
    const int k = kc * KW + W * q;  // this lane's W consecutive K indices
    // W consecutive K indices share one tap (CIN is a multiple of W), so the
    // lane's A and B fragments are single LDS words
    word bw[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int n = nb * 16 + i;
      bw[nb] = n < COUT ? *reinterpret_cast<const word*>(ws + n * KS + k) : zero;
    }
    const bool inK = k < K;
    const int tap = inK ? k / CIN : 0, ch = inK ? k - tap * CIN : 0;
    const int dt = tap / 3, dx = tap - 3 * dt;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const _Float16* xr = xs + ((wave * 4 + rr + dt) * HE + i + dx) * S + ch;
      const word a = inK ? *reinterpret_cast<const word*>(xr) : zero;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) acc[rr][nb] = hmma_w<W>(a, bw[nb], acc[rr][nb]);
    }
  }
  __syncthreads();  // every wave is done with the tile and weights: reuse smem
  _Float16* os = smem;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    const int n = nb * 16 + i;
    if (n >= COUT) continue;
    const float bn = bias[n];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float z = acc[rr][nb][v] + bn;
        if (EPI == EPI_TANH) z = tanhf(z);
        os[((wave * 4 + rr) * TE + 4 * q + v) * OS + n] = (_Float16)z;
      }
    }
  }
  __syncthreads();
  constexpr int OQ = COUT / 4;
  for (int e = threadIdx.x; e < TE * TE * OQ; e += CNT) {
    const int site = e / OQ, w4 = e - site * OQ;
    const int row = site / TE, col = site - row * TE;
    const int64_t o = (((int64_t)b * Lt + t0 + row) * Lx + x0 + col) * COUT + 4 * w4;
    *reinterpret_cast<hv4*>(out + o) = *reinterpret_cast<const hv4*>(os + site * OS + 4 * w4);
  }
}

// Partial weight and bias gradients of one layer over the tiles a workgroup
// visits: part[wg][co][k] = sum_sites G[site][co] X[site + off(tap)][c] for
// k = tap*CIN + c < 9*CIN, and sum_sites G[site][co] for k = 9*CIN.  The
// matrix-core step runs M = 16 output channels x N = 16 (tap, channel)
// columns x K = 4 sites; the 4 waves share the output tiles.
template <int CIN, int COUT>
__global__ void __launch_bounds__(CNT) k_wgrad(const float* __restrict__ X, const float* __restrict__ G,
                                               int Lx, int Lt, int anti, int nb,
                                               float* __restrict__ part) {
  constexpr int K = 9 * CIN, KB = K + 1;
  constexpr int S = CIN + 1, GS = COUT + 1;
  constexpr int MB = (COUT + 15) / 16, NK = (KB + 15) / 16, T = MB * NK, TPW = (T + 3) / 4;
  __shared__ float xs[HE * HE * S];
  __shared__ float gs[TE * TE * GS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  // per output tile of this wave: LDS offset of column (kb*16 + i) relative
  // to the site, or -1 for the bias column and -2 beyond it
  int xoff[TPW], goff[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = wave + 4 * j;
    const int mb = tile / NK, kb = tile - mb * NK;
    const int k = kb * 16 + i;
    if (tile >= T || k > K) {
      xoff[j] = -2;
    } else if (k == K) {
      xoff[j] = -1;
    } else {
      const int tap = k / CIN, ch = k - tap * CIN;
      xoff[j] = ((tap / 3) * HE + tap % 3) * S + ch;
    }
    const int co = mb * 16 + i;
    goff[j] = (tile < T && co < COUT) ? co : -1;
  }
  f4 acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
  const int tx = Lx / TE, tt = Lt / TE;
  const int64_t ntile = (int64_t)nb * tx * tt;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int b = (int)(tile / (tx * tt));
    const int rem = (int)(tile - (int64_t)b * tx * tt);
    const int t0 = (rem / tx) * TE, x0 = (rem % tx) * TE;
    __syncthreads();
    load_tile<CIN>(X, Lx, Lt, anti, b, t0, x0, xs);
    for (int e = threadIdx.x; e < TE * TE * COUT; e += CNT) {
      const int site = e / COUT, ch = e - site * COUT;
      const int r = site / TE, c = site - r * TE;
      gs[site * GS + ch] = G[(((int64_t)b * Lt + t0 + r) * Lx + x0 + c) * COUT + ch];
    }
    __syncthreads();
    for (int s0 = 0; s0 < TE * TE; s0 += 4) {
      const int s = s0 + q;
      const int xb = ((s / TE) * HE + (s % TE)) * S;
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        if (wave + 4 * j >= T) break;
        const float a = goff[j] >= 0 ? gs[s * GS + goff[j]] : 0.f;
        const float bv = xoff[j] >= 0 ? xs[xb + xoff[j]] : (xoff[j] == -1 ? 1.f : 0.f);
        acc[j] = mma4(a, bv, acc[j]);
      }
    }
  }
  float* P = part + (int64_t)blockIdx.x * COUT * KB;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    const int tile = wave + 4 * j;
    if (tile >= T) break;
    const int mb = tile / NK, kb = tile - mb * NK;
    const int k = kb * 16 + i;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int co = mb * 16 + 4 * q + v;
      if (co < COUT && k < KB) P[co * KB + k] = acc[j][v];
    }
  }
}

// Sum the workgroup partials (fixed order, FP64) into the parameter packing.
template <int CIN, int COUT>
__global__ void __launch_bounds__(CNT) k_wgrad_reduce(const float* __restrict__ part, int nparts,
                                                      float* __restrict__ grad) {
  constexpr int K = 9 * CIN, KB = K + 1;
  const int e = blockIdx.x * CNT + threadIdx.x;
  if (e >= COUT * KB) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * COUT * KB + e];
  const int co = e / KB, k = e - co * KB;
  if (k < K) {
    const int tap = k / CIN, ci = k - tap * CIN;
    grad[(co * CIN + ci) * 9 + tap] = (float)s;
  } else {
    grad[COUT * CIN * 9 + co] = (float)s;
  }
}

// Packed forward and transposed copies of one layer's weights.
__global__ void __launch_bounds__(CNT) k_pack(const float* __restrict__ W, int cin, int cout,
                                              float* __restrict__ wf, float* __restrict__ wb) {
  const int e = blockIdx.x * CNT + threadIdx.x;
  if (e >= cout * cin * 9) return;
  const int co = e / (cin * 9), r = e - co * cin * 9;
  const int ci = r / 9, tap = r - ci * 9;
  const float w = W[e];
  wf[co * 9 * cin + tap * cin + ci] = w;
  wb[ci * 9 * cout + (8 - tap) * cout + co] = w;
}

__global__ void __launch_bounds__(CNT) k_pack_half(const float* __restrict__ wf, int cnt,
                                                   _Float16* __restrict__ wh) {
  const int e = blockIdx.x * CNT + threadIdx.x;
  if (e < cnt) wh[e] = (_Float16)wf[e];
}

__global__ void __launch_bounds__(CNT) k_adam(float* __restrict__ th, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int e = blockIdx.x * CNT + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  th[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

template <class TI, class TO>
__global__ void __launch_bounds__(CNT) k_cast(const TI* __restrict__ in, TO* __restrict__ out, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x;
  if (e < n) out[e] = (TO)in[e];
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// Per-(RHS, chunk) sums of (y - t)^2 and t^2.
template <class TT>
__global__ void __launch_bounds__(CNT) k_loss_partial(const float* __restrict__ y, const TT* __restrict__ tg,
                                                      int64_t per, double* __restrict__ part) {
  __shared__ double red[4];
  const int b = blockIdx.y, nch = gridDim.x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < per; e += (int64_t)nch * CNT) {
    const double t = (double)tg[b * per + e];
    const double d = (double)y[b * per + e] - t;
    s1 += d * d;
    s2 += t * t;
  }
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0) {
    part[((int64_t)b * nch + blockIdx.x) * 2] = s1;
    part[((int64_t)b * nch + blockIdx.x) * 2 + 1] = s2;
  }
}

// loss = mean_b num_b / den_b; scale_b = 2 / (den_b nb) for the gradient.
__global__ void __launch_bounds__(CNT) k_loss_final(const double* __restrict__ part, int nch, int nb,
                                                    double* __restrict__ loss, float* __restrict__ scale,
                                                    double* __restrict__ ratio) {
  for (int b = threadIdx.x; b < nb; b += CNT) {
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nch; ++c) {
      num += part[((int64_t)b * nch + c) * 2];
      den += part[((int64_t)b * nch + c) * 2 + 1];
    }
    ratio[b] = num / den;
    scale[b] = (float)(2.0 / (den * nb));
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += ratio[b];
    *loss = s / nb;
  }
}

template <class TT>
__global__ void __launch_bounds__(CNT) k_loss_grad(const float* __restrict__ y, const TT* __restrict__ tg,
                                                   const float* __restrict__ scale, int64_t per, int64_t n,
                                                   float* __restrict__ g) {
  const int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x;
  if (e >= n) return;
  g[e] = scale[e / per] * (float)((double)y[e] - (double)tg[e]);
}

// Minimal-residual factor along y per RHS: sums of conj(u) b and |u|^2, u = D y.
__global__ void __launch_bounds__(CNT) k_mr_partial(const cd* __restrict__ u, const cd* __restrict__ b,
                                                    int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int r = blockIdx.y, nch = gridDim.x;
  double sr = 0.0, si = 0.0, sd = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < n; e += (int64_t)nch * CNT) {
    const cd ue = u[r * n + e], be = b[r * n + e];
    sr += ue.re * be.re + ue.im * be.im;
    si += ue.re * be.im - ue.im * be.re;
    sd += ue.re * ue.re + ue.im * ue.im;
  }
  sr = block_sum(sr, red);
  si = block_sum(si, red);
  sd = block_sum(sd, red);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)r * nch + blockIdx.x) * 3;
    o[0] = sr;
    o[1] = si;
    o[2] = sd;
  }
}

// x = alpha_r y with alpha_r = <u, b> / |u|^2, or x = 0 when alpha_r is not a
// finite non-zero number (an unusable guess falls back to x0 = 0).
__global__ void __launch_bounds__(CNT) k_mr_apply(const double* __restrict__ part, int nch, int64_t n,
                                                  cd* __restrict__ x) {
  const int r = blockIdx.y;
  double sr = 0.0, si = 0.0, sd = 0.0;
  for (int c = 0; c < nch; ++c) {
    const double* p = part + ((int64_t)r * nch + c) * 3;
    sr += p[0];
    si += p[1];
    sd += p[2];
  }
  double ar = sr / sd, ai = si / sd;
  const bool ok = sd > 0.0 && isfinite(ar) && isfinite(ai) && (ar != 0.0 || ai != 0.0);
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * CNT) {
    const cd y = x[r * n + e];
    x[r * n + e] = ok ? cd{ar * y.re - ai * y.im, ar * y.im + ai * y.re} : cd{0.0, 0.0};
  }
}

// Learned stage: x = alpha_r y and res = b - alpha_r u per RHS, alpha_r as in
// k_mr_apply; an unusable alpha_r gives x = 0 and res = b (multigrid alone).
// res may alias u (element-wise read before write).
__global__ void __launch_bounds__(CNT) k_mr_apply_res(const double* __restrict__ part, int nch, int64_t n,
                                                      cd* __restrict__ x, const cd* u, const cd* __restrict__ b,
                                                      cd* res) {
  const int r = blockIdx.y;
  double sr = 0.0, si = 0.0, sd = 0.0;
  for (int c = 0; c < nch; ++c) {
    const double* p = part + ((int64_t)r * nch + c) * 3;
    sr += p[0];
    si += p[1];
    sd += p[2];
  }
  const double ar = sr / sd, ai = si / sd;
  const bool ok = sd > 0.0 && isfinite(ar) && isfinite(ai) && (ar != 0.0 || ai != 0.0);
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * CNT) {
    const int64_t o = r * n + e;
    const cd y = x[o], ue = u[o], be = b[o];
    // the fallback never multiplies: y and u may hold NaN
    x[o] = ok ? cd{ar * y.re - ai * y.im, ar * y.im + ai * y.re} : cd{0.0, 0.0};
    res[o] = ok ? cd{be.re - (ar * ue.re - ai * ue.im), be.im - (ar * ue.im + ai * ue.re)} : be;
  }
}

// z += x for the active RHS
__global__ void __launch_bounds__(CNT) k_stage_add(cd* __restrict__ z, const cd* __restrict__ x, int64_t n,
                                                   const int* __restrict__ act) {
  const int r = blockIdx.y;
  if (act && !act[r]) return;
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < n; e += (int64_t)gridDim.x * CNT) {
    const cd a = z[r * n + e], v = x[r * n + e];
    z[r * n + e] = cd{a.re + v.re, a.im + v.im};
  }
}

// in * s
__global__ void __launch_bounds__(CNT) k_scale_copy(const cd* __restrict__ in, double s, int64_t cnt,
                                                    cd* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * CNT + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * CNT) {
    const cd v = in[e];
    out[e] = cd{s * v.re, s * v.im};
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + CNT - 1) / CNT); }

constexpr int WIDTH[5] = {4, 32, 32, 32, 4};

int param_offset(int l) {
  int o = 0;
  for (int j = 0; j < l; ++j) o += WIDTH[j + 1] * WIDTH[j] * 9 + WIDTH[j + 1];
  return o;
}

constexpr int WGRAD_PARTS = 512;

}  // namespace

void Cnn::init() {
  theta.ensure(sizeof(float) * MGM_CNN_NPARAMS);
  m.ensure(sizeof(float) * MGM_CNN_NPARAMS);
  v.ensure(sizeof(float) * MGM_CNN_NPARAMS);
  grad.ensure(sizeof(float) * MGM_CNN_NPARAMS);
  for (int l = 0; l < 4; ++l) {
    const size_t w = sizeof(float) * 9 * WIDTH[l] * WIDTH[l + 1];
    wf[l].ensure(w);
    wb[l].ensure(w);
    wh[l].ensure(w / 2);
  }
}

void Cnn::pack(hipStream_t s) {
  for (int l = 0; l < 4; ++l) {
    const int cin = WIDTH[l], cout = WIDTH[l + 1];
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(9 * cin * cout)), dim3(CNT), 0, s,
                       theta.as<float>() + param_offset(l), cin, cout, wf[l].as<float>(),
                       wb[l].as<float>());
    hipLaunchKernelGGL(k_pack_half, dim3(blocks_for(9 * cin * cout)), dim3(CNT), 0, s, wf[l].as<float>(),
                       9 * cin * cout, wh[l].as<_Float16>());
    KCHK();
  }
}

const float* Cnn::bias(int l) const {
  return theta.as<float>() + param_offset(l) + 9 * WIDTH[l] * WIDTH[l + 1];
}

void cnn_check_lattice(const Gauge& g) {
  require(g.Lx % TE == 0 && g.Lt % TE == 0, "the network needs Lx and Lt divisible by 16");
}

// Forward pass on nb channel-last inputs x0 [nb][V][4]; keeps the three
// hidden activations in w.a[0..2] and writes y [nb][V][4].
void cnn_forward(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const float* x0,
                 CnnWork& w, float* y) {
  const int64_t V = (int64_t)g.Lx * g.Lt;
  for (int l = 0; l < 3; ++l) w.a[l].ensure(sizeof(float) * nb * V * 32);
  const dim3 grid(g.Lx / TE, g.Lt / TE, nb);
  hipLaunchKernelGGL((k_conv<4, 32, EPI_TANH>), grid, dim3(CNT), 0, s, x0, g.Lx, g.Lt, g.anti,
                     net.wf[0].as<float>(), net.bias(0), nullptr, w.a[0].as<float>());
  hipLaunchKernelGGL((k_conv<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, w.a[0].as<float>(), g.Lx, g.Lt,
                     g.anti, net.wf[1].as<float>(), net.bias(1), nullptr, w.a[1].as<float>());
  hipLaunchKernelGGL((k_conv<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, w.a[1].as<float>(), g.Lx, g.Lt,
                     g.anti, net.wf[2].as<float>(), net.bias(2), nullptr, w.a[2].as<float>());
  hipLaunchKernelGGL((k_conv<32, 4, EPI_NONE>), grid, dim3(CNT), 0, s, w.a[2].as<float>(), g.Lx, g.Lt,
                     g.anti, net.wf[3].as<float>(), net.bias(3), nullptr, y);
  KCHK();
}

// One hidden 32 -> 32 convolution with tanh (the network's dominant kernel),
// for timing.
void cnn_time_conv(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const float* in, float* out) {
  const dim3 grid(g.Lx / TE, g.Lt / TE, nb);
  hipLaunchKernelGGL((k_conv<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, in, g.Lx, g.Lt, g.anti,
                     net.wf[1].as<float>(), net.bias(1), nullptr, out);
  KCHK();
}

void cnn_time_conv_h(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const _Float16* in,
                     _Float16* out) {
  const dim3 grid(g.Lx / TE, g.Lt / TE, nb);
  hipLaunchKernelGGL((k_conv_h<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, in, g.Lx, g.Lt, g.anti,
                     net.wh[1].as<_Float16>(), net.bias(1), out);
  KCHK();
}

namespace {
template <int CIN, int COUT>
void wgrad(hipStream_t s, const Gauge& g, int nb, const float* X, const float* G, CnnWork& w,
           float* grad) {
  const int64_t ntile = (int64_t)nb * (g.Lx / TE) * (g.Lt / TE);
  const int parts = (int)std::min<int64_t>(ntile, WGRAD_PARTS);
  constexpr int KB = 9 * CIN + 1;
  w.part.ensure(sizeof(float) * (size_t)parts * COUT * KB);
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(parts), dim3(CNT), 0, s, X, G, g.Lx, g.Lt, g.anti, nb,
                     w.part.as<float>());
  hipLaunchKernelGGL((k_wgrad_reduce<CIN, COUT>), dim3(blocks_for(COUT * KB)), dim3(CNT), 0, s,
                     w.part.as<float>(), parts, grad);
  KCHK();
}

// loss and dL/dy for targets of type TT ([nb][V][4] in the vector order)
template <class TT>
const double* loss_grad_y(hipStream_t s, int nb, int64_t per, const float* y, const TT* tg, CnnWork& w,
                          float* gy) {
  const int nch = (int)std::min<int64_t>(64, (per + CNT - 1) / CNT);
  w.lpart.ensure(sizeof(double) * (size_t)nb * nch * 2 + sizeof(double) * (nb + 1) +
                 sizeof(float) * nb);
  double* part = w.lpart.as<double>();
  double* loss = part + (size_t)nb * nch * 2;
  double* ratio = loss + 1;
  float* scale = reinterpret_cast<float*>(ratio + nb);
  hipLaunchKernelGGL(k_loss_partial<TT>, dim3(nch, nb), dim3(CNT), 0, s, y, tg, per, part);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(CNT), 0, s, part, nch, nb, loss, scale, ratio);
  hipLaunchKernelGGL(k_loss_grad<TT>, dim3(blocks_for(nb * per)), dim3(CNT), 0, s, y, tg, scale, per,
                     nb * per, gy);
  KCHK();
  return loss;
}
}  // namespace

// Forward + backward on nb pairs (x0 channel-last float, target of type TT in
// the same order); gradients into net.grad, the loss into *loss_dev.
template <class TT>
const double* cnn_loss_grad(hipStream_t s, Cnn& net, const Gauge& g, int nb, const float* x0,
                            const TT* target, CnnWork& w) {
  const int64_t V = (int64_t)g.Lx * g.Lt;
  w.y.ensure(sizeof(float) * nb * V * 4);
  w.gy.ensure(sizeof(float) * nb * V * 4);
  w.g[0].ensure(sizeof(float) * nb * V * 32);
  w.g[1].ensure(sizeof(float) * nb * V * 32);
  cnn_forward(s, net, g, nb, x0, w, w.y.as<float>());
  const double* loss = loss_grad_y<TT>(s, nb, V * 4, w.y.as<float>(), target, w, w.gy.as<float>());
  float* grad = net.grad.as<float>();
  const dim3 grid(g.Lx / TE, g.Lt / TE, nb);
  float* gA = w.g[0].as<float>();
  float* gB = w.g[1].as<float>();
  const float* a1 = w.a[0].as<float>();
  const float* a2 = w.a[1].as<float>();
  const float* a3 = w.a[2].as<float>();
  wgrad<32, 4>(s, g, nb, a3, w.gy.as<float>(), w, grad + param_offset(3));
  hipLaunchKernelGGL((k_conv<4, 32, EPI_DTANH>), grid, dim3(CNT), 0, s, w.gy.as<float>(), g.Lx, g.Lt,
                     g.anti, net.wb[3].as<float>(), nullptr, a3, gA);
  wgrad<32, 32>(s, g, nb, a2, gA, w, grad + param_offset(2));
  hipLaunchKernelGGL((k_conv<32, 32, EPI_DTANH>), grid, dim3(CNT), 0, s, gA, g.Lx, g.Lt, g.anti,
                     net.wb[2].as<float>(), nullptr, a2, gB);
  wgrad<32, 32>(s, g, nb, a1, gB, w, grad + param_offset(1));
  hipLaunchKernelGGL((k_conv<32, 32, EPI_DTANH>), grid, dim3(CNT), 0, s, gB, g.Lx, g.Lt, g.anti,
                     net.wb[1].as<float>(), nullptr, a1, gA);
  wgrad<4, 32>(s, g, nb, x0, gA, w, grad + param_offset(0));
  KCHK();
  return loss;
}
template const double* cnn_loss_grad<double>(hipStream_t, Cnn&, const Gauge&, int, const float*,
                                             const double*, CnnWork&);
template const double* cnn_loss_grad<float>(hipStream_t, Cnn&, const Gauge&, int, const float*,
                                            const float*, CnnWork&);

void cnn_adam(hipStream_t s, Cnn& net, const mgm_adam_params& ap) {
  net.t += 1;
  const double c1 = 1.0 - std::pow(ap.beta1, (double)net.t);
  const double c2 = 1.0 - std::pow(ap.beta2, (double)net.t);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(MGM_CNN_NPARAMS)), dim3(CNT), 0, s, net.theta.as<float>(),
                     net.m.as<float>(), net.v.as<float>(), net.grad.as<float>(), MGM_CNN_NPARAMS,
                     (float)ap.lr, (float)ap.beta1, (float)ap.beta2, (float)ap.eps, (float)c1, (float)c2);
  KCHK();
  net.pack(s);
}

void cnn_to_channels(hipStream_t s, const cd* in, int64_t ndof, float* out) {
  hipLaunchKernelGGL((k_cast<double, float>), dim3(blocks_for(2 * ndof)), dim3(CNT), 0, s,
                     reinterpret_cast<const double*>(in), out, 2 * ndof);
  KCHK();
}

void cnn_from_channels(hipStream_t s, const float* in, int64_t ndof, cd* out) {
  hipLaunchKernelGGL((k_cast<float, double>), dim3(blocks_for(2 * ndof)), dim3(CNT), 0, s, in,
                     reinterpret_cast<double*>(out), 2 * ndof);
  KCHK();
}

// FP16 forward pass: x0 and y are FP16 channel-last [nb][V][4]; the hidden
// activations go to w.h[0..1] (ping-pong).
void cnn_forward_h(hipStream_t s, const Cnn& net, const Gauge& g, int nb, const _Float16* x0, CnnWork& w,
                   _Float16* y) {
  const int64_t V = (int64_t)g.Lx * g.Lt;
  for (int l = 0; l < 2; ++l) w.h[l].ensure(sizeof(_Float16) * nb * V * 32);
  _Float16* h0 = w.h[0].as<_Float16>();
  _Float16* h1 = w.h[1].as<_Float16>();
  const dim3 grid(g.Lx / TE, g.Lt / TE, nb);
  hipLaunchKernelGGL((k_conv_h<4, 32, EPI_TANH>), grid, dim3(CNT), 0, s, x0, g.Lx, g.Lt, g.anti,
                     net.wh[0].as<_Float16>(), net.bias(0), h0);
  hipLaunchKernelGGL((k_conv_h<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, h0, g.Lx, g.Lt, g.anti,
                     net.wh[1].as<_Float16>(), net.bias(1), h1);
  hipLaunchKernelGGL((k_conv_h<32, 32, EPI_TANH>), grid, dim3(CNT), 0, s, h1, g.Lx, g.Lt, g.anti,
                     net.wh[2].as<_Float16>(), net.bias(2), h0);
  hipLaunchKernelGGL((k_conv_h<32, 4, EPI_NONE>), grid, dim3(CNT), 0, s, h0, g.Lx, g.Lt, g.anti,
                     net.wh[3].as<_Float16>(), net.bias(3), y);
  KCHK();
}

// y = f(b) for complex128 vectors, in RHS chunks that keep the hidden
// activations under ~512 MB; FP32 or FP16 network (net.half).
void cnn_apply(hipStream_t s, const Cnn& net, const Gauge& g, int nrhs, const cd* b, cd* y,
               CnnWork& w) {
  cnn_check_lattice(g);
  const int64_t V = (int64_t)g.Lx * g.Lt, n = 2 * V;
  const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nrhs, (int64_t(512) << 20) / (V * 32 * 4)));
  if (net.half) {
    w.hx0.ensure(sizeof(_Float16) * chunk * V * 4);
    w.hy.ensure(sizeof(_Float16) * chunk * V * 4);
    for (int r0 = 0; r0 < nrhs; r0 += chunk) {
      const int k = std::min(chunk, nrhs - r0);
      hipLaunchKernelGGL((k_cast<double, _Float16>), dim3(blocks_for(2 * (int64_t)k * n)), dim3(CNT), 0, s,
                         reinterpret_cast<const double*>(b + (int64_t)r0 * n), w.hx0.as<_Float16>(),
                         2 * (int64_t)k * n);
      cnn_forward_h(s, net, g, k, w.hx0.as<_Float16>(), w, w.hy.as<_Float16>());
      hipLaunchKernelGGL((k_cast<_Float16, double>), dim3(blocks_for(2 * (int64_t)k * n)), dim3(CNT), 0, s,
                         w.hy.as<_Float16>(), reinterpret_cast<double*>(y + (int64_t)r0 * n), 2 * (int64_t)k * n);
      KCHK();
    }
    return;
  }
  w.x0.ensure(sizeof(float) * chunk * V * 4);
  w.y.ensure(sizeof(float) * chunk * V * 4);
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int k = std::min(chunk, nrhs - r0);
    cnn_to_channels(s, b + (int64_t)r0 * n, (int64_t)k * n, w.x0.as<float>());
    cnn_forward(s, net, g, k, w.x0.as<float>(), w, w.y.as<float>());
    cnn_from_channels(s, w.y.as<float>(), (int64_t)k * n, y + (int64_t)r0 * n);
  }
}

// x = alpha f(b) per RHS with alpha minimising ||b - alpha D f(b)|| (u is a
// work vector of the same shape).
void cnn_initial_guess(mgm_ctx* c, Gauge& g, int nrhs, const cd* b, cd* x, cd* u) {
  hipStream_t s = c->stream;
  require(c->cnn && c->cnn->ready, "no network parameters set (mgm_cnn_set_params)");
  cnn_apply(s, *c->cnn, g, nrhs, b, x, g.cnn);
  apply_level(c, g, 0, nrhs, x, u);
  const int64_t n = g.levels[0]->n;
  const int nch = (int)std::min<int64_t>(64, (n + CNT - 1) / CNT);
  g.cnn.mr.ensure(sizeof(double) * 3 * nrhs * nch);
  hipLaunchKernelGGL(k_mr_partial, dim3(nch, nrhs), dim3(CNT), 0, s, u, b, n, g.cnn.mr.as<double>());
  hipLaunchKernelGGL(k_mr_apply, dim3(nch, nrhs), dim3(CNT), 0, s, g.cnn.mr.as<double>(), nch, n, x);
  KCHK();
}

// Learned first stage of the level-0 preconditioner of the flexible outer
// FGMRES: z = x1 + M(v - D x1) with M the multigrid cycle and
// x1 = alpha_r f(sqrt(n) v_r), alpha_r minimising ||v_r - alpha D f(.)|| (the
// Arnoldi vectors have unit norm; the factor sqrt(n) gives the network inputs
// of the size of its Z2 x Z2 training right-hand sides).  A zero or
// non-finite alpha_r leaves z = M v (multigrid fallback).  The error of z is
// (I - M D) applied to the error of x1.  No host synchronisation.
void cnn_precondition(mgm_ctx* c, Gauge& g, int nrhs, const cd* v, cd* z, const int* act) {
  hipStream_t s = c->stream;
  require(c->cnn && c->cnn->ready, "no network parameters set (mgm_cnn_set_params)");
  const int64_t n = g.levels[0]->n, cnt = (int64_t)nrhs * n;
  CnnWork& w = g.cnn;
  w.st_x.ensure(sizeof(cd) * cnt);
  w.st_u.ensure(sizeof(cd) * cnt);
  cd* x1 = w.st_x.as<cd>();
  cd* u = w.st_u.as<cd>();
  const unsigned gb = (unsigned)std::min<int64_t>(blocks_for(cnt), 8192);
  hipLaunchKernelGGL(k_scale_copy, dim3(gb), dim3(CNT), 0, s, v, std::sqrt((double)n), cnt, u);
  cnn_apply(s, *c->cnn, g, nrhs, u, x1, w);
  apply_level(c, g, 0, nrhs, x1, u);
  const int nch = (int)std::min<int64_t>(64, (n + CNT - 1) / CNT);
  w.mr.ensure(sizeof(double) * 3 * nrhs * nch);
  hipLaunchKernelGGL(k_mr_partial, dim3(nch, nrhs), dim3(CNT), 0, s, u, v, n, w.mr.as<double>());
  hipLaunchKernelGGL(k_mr_apply_res, dim3(nch, nrhs), dim3(CNT), 0, s, w.mr.as<double>(), nch, n, x1, u, v, u);
  KCHK();
  precondition_d(c, g, 0, nrhs, u, z, act);
  const unsigned ga = (unsigned)std::min<int64_t>(blocks_for(n), 1024);
  hipLaunchKernelGGL(k_stage_add, dim3(ga, nrhs), dim3(CNT), 0, s, z, x1, n, act);
  KCHK();
}

}  // namespace mgm
