// Batched vector kernels for FGMRES (classical Gram-Schmidt applied twice,
// Givens least squares) and for the CholQR2 orthonormalisation of tall-skinny
// blocks.  Reductions are deterministic: every workgroup sums a fixed chunk in
// a fixed order (wave64 butterfly, then the four waves), and a second kernel
// adds the chunk partials in chunk order.  No atomics.
#include "internal.h"

namespace mgm {

namespace {

constexpr int NT = 256;

// Elements per thread of the chunked reductions: the largest of 8, 4, 2, 1
// that still gives ~1024 workgroups over all RHS (short vectors and few RHS
// otherwise leave most of the 256 CUs idle).  Chunk length = 256 * EPT.
inline int pick_ept(int64_t n, int nrhs) {
  int e = 8;
  while (e > 1 && ((n + NT * e - 1) / (NT * e)) * (int64_t)nrhs < 1024) e /= 2;
  return e;
}
inline unsigned nchunks(int64_t n, int ept) { return (unsigned)((n + NT * ept - 1) / (NT * ept)); }

#define EPT_DISPATCH(ept, KERNEL, ...)                           \
  switch (ept) {                                                 \
    case 8: { constexpr int E = 8; KERNEL; } break;              \
    case 4: { constexpr int E = 4; KERNEL; } break;              \
    case 2: { constexpr int E = 2; KERNEL; } break;              \
    default: { constexpr int E = 1; KERNEL; } break;             \
  }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of v over the 256 threads, valid in thread 0.  `sh` holds 2*4 values.
template <class T>
__device__ __forceinline__ cx<T> block_sum(cx<T> v, T* sh) {
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[2 * w] = v.re;
    sh[2 * w + 1] = v.im;
  }
  __syncthreads();
  cx<T> r = mk<T>(0, 0);
  if (threadIdx.x == 0) {
    r.re = (sh[0] + sh[2]) + (sh[4] + sh[6]);
    r.im = (sh[1] + sh[3]) + (sh[5] + sh[7]);
  }
  return r;
}

template <class T>
__device__ __forceinline__ T block_sum_real(T v, T* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

// partial[(r*nv + i)*nch + chunk] = sum_{k in chunk} conj(V_i[r][k]) w[r][k].
// Vectors go in groups of DG so that DG * EPT loads are in flight at once; each
// wave reduces its share with shuffles only and the four wave sums meet in LDS
// once per 64 vectors (one barrier pair instead of one per vector).  Past the
// end of the vectors w is zero, and the V loads there read element n - 1
// instead (the index is clamped, the load is not conditional): a conditional
// load compiles to a branch and a wait for memory per element.
constexpr int DG = 4;

template <class T, int EPT>
__global__ void __launch_bounds__(NT) k_dot_multi(const cx<T>* __restrict__ V, int64_t sI, int64_t sR,
                                                  int nv, const cx<T>* __restrict__ w, int64_t n,
                                                  cx<T>* __restrict__ partial,
                                                  const int* __restrict__ active) {
  constexpr int CH = NT * EPT;
  __shared__ cx<T> sh[4][64];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int nch = gridDim.x;
  const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  const cx<T>* __restrict__ wr = w + (int64_t)r * n;
  const cx<T>* __restrict__ Vr = V + (int64_t)r * sR;
  cx<T> wv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    wv[e] = ld_or0(wr + (k < n ? k : 0), k < n);
  }
  auto put = [&](int slot, cx<T> acc) {
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) sh[wv_id][slot] = acc;
  };
  for (int i0 = 0; i0 < nv; i0 += 64) {
    const int nb = min(64, nv - i0);
    int j = 0;
    for (; j + DG <= nb; j += DG) {
      cx<T> acc[DG];
#pragma unroll
      for (int g = 0; g < DG; ++g) {
        const cx<T>* __restrict__ vi = Vr + (int64_t)(i0 + j + g) * sI;
        acc[g] = mk<T>(0, 0);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const int64_t k = base + (int64_t)e * NT;
          cjfma(acc[g], vi[k < n ? k : n - 1], wv[e]);
        }
      }
#pragma unroll
      for (int g = 0; g < DG; ++g) put(j + g, acc[g]);
    }
    for (; j < nb; ++j) {
      const cx<T>* __restrict__ vi = Vr + (int64_t)(i0 + j) * sI;
      cx<T> acc = mk<T>(0, 0);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int64_t k = base + (int64_t)e * NT;
        cjfma(acc, vi[k < n ? k : n - 1], wv[e]);
      }
      put(j, acc);
    }
    __syncthreads();
    if (threadIdx.x < nb) {
      const int t = threadIdx.x;
      partial[((int64_t)r * nv + i0 + t) * nch + blockIdx.x] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    }
    __syncthreads();
  }
}

// k_dot_multi against two vectors: partial[(r * 2 nv + i) * nch + chunk] =
// V_i^H w (i < nv) and V_{i - nv}^H u (i >= nv), one read of the basis for
// both (u is the newest basis vector in the Gram-corrected Arnoldi step).
template <class T, int EPT>
__global__ void __launch_bounds__(NT) k_dot_multi2(const cx<T>* __restrict__ V, int64_t sI, int64_t sR,
                                                   int nv, const cx<T>* __restrict__ w, const cx<T>* __restrict__ u,
                                                   int64_t n, cx<T>* __restrict__ partial,
                                                   const int* __restrict__ active) {
  constexpr int CH = NT * EPT;
  __shared__ cx<T> sh[4][128];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int nch = gridDim.x;
  const int lane = threadIdx.x & 63, wv_id = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  const cx<T>* __restrict__ wr = w + (int64_t)r * n;
  const cx<T>* __restrict__ ur = u + (int64_t)r * sR;
  const cx<T>* __restrict__ Vr = V + (int64_t)r * sR;
  cx<T> wv[EPT], uv[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    wv[e] = ld_or0(wr + (k < n ? k : 0), k < n);
    uv[e] = ld_or0(ur + (k < n ? k : 0), k < n);
  }
  auto put = [&](int slot, cx<T> acc) {
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) sh[wv_id][slot] = acc;
  };
  for (int i0 = 0; i0 < nv; i0 += 64) {
    const int nb = min(64, nv - i0);
    for (int j = 0; j < nb; j += 2) {
      const int g2 = min(2, nb - j);
      cx<T> aw[2], au[2];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        aw[g] = mk<T>(0, 0);
        au[g] = mk<T>(0, 0);
        if (g < g2) {
          const cx<T>* __restrict__ vi = Vr + (int64_t)(i0 + j + g) * sI;
#pragma unroll
          for (int e = 0; e < EPT; ++e) {
            const int64_t k = base + (int64_t)e * NT;
            const cx<T> x = vi[k < n ? k : n - 1];
            cjfma(aw[g], x, wv[e]);
            cjfma(au[g], x, uv[e]);
          }
        }
      }
#pragma unroll
      for (int g = 0; g < 2; ++g)
        if (g < g2) {
          put(2 * (j + g), aw[g]);
          put(2 * (j + g) + 1, au[g]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nb) {
      const int t = threadIdx.x, i = i0 + (t >> 1);
      const cx<T> v = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
      partial[((int64_t)r * 2 * nv + (t & 1) * nv + i) * nch + blockIdx.x] = v;
    }
    __syncthreads();
  }
}

// The Arnoldi step's Gram-Schmidt in one update: from the partials of
// k_dot_multi2, h1 = V^H w and the newest Gram column g = V^H v_j; with the
// earlier columns of G = V^H V (gram, [r][ldg][ldg], column-major: G[i][k] at
// k ldg + i), coef = h1 + (I - G) h1 -- the second classical Gram-Schmidt pass
// with V^H (w - V h1) = h1 - G h1 -- and w -= V coef.  The workgroups of
// chunk 0 store g into G and coef to coef_out; every workgroup adds the
// partials in the order of k_reduce_chunks.  Optional |w|^2 chunk partials.
template <class T, int EPT>
__global__ void __launch_bounds__(NT) k_update_gram(const cx<T>* __restrict__ V, int64_t sI, int64_t sR, int nv,
                                                    const cx<T>* __restrict__ dpart, int nchd,
                                                    cx<T>* __restrict__ gram, int ldg,
                                                    cx<T>* __restrict__ coef_out, int ldc,
                                                    cx<T>* __restrict__ w, int64_t n, T* __restrict__ partial,
                                                    const int* __restrict__ active) {
  constexpr int CH = NT * EPT;
  __shared__ cx<T> h1[64], gc[64], cs[64];
  __shared__ T sh[8];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < 2 * nv; q += NT / 64) {
    const cx<T>* p = dpart + ((int64_t)r * 2 * nv + q) * nchd;
    cx<T> acc = mk<T>(0, 0);
    for (int c = lane; c < nchd; c += 64) acc = acc + p[c];
    acc.re = wave_sum(acc.re);
    acc.im = wave_sum(acc.im);
    if (lane == 0) {
      if (q < nv) h1[q] = acc;
      else gc[q - nv] = acc;
    }
  }
  __syncthreads();
  cx<T>* G = gram + (int64_t)r * ldg * ldg;
  const int j = nv - 1;  // the new column
  for (int i = threadIdx.x; i < nv; i += NT) {
    // (G h1)_i = sum_{k < j} G[i][k] h1[k] + G[i][j] h1[j], G[i][j] = g_i, G[j][k] = conj(g_k)
    cx<T> gh = mk<T>(0, 0);
    if (i < j) {
      for (int k = 0; k < j; ++k) cfma(gh, G[(int64_t)k * ldg + i], h1[k]);
    } else {
      for (int k = 0; k < j; ++k) cfma(gh, conj(gc[k]), h1[k]);
    }
    cfma(gh, gc[i], h1[j]);
    const cx<T> c = h1[i] + (h1[i] - gh);
    cs[i] = (T)-1 * c;
    if (blockIdx.x == 0) {
      coef_out[(int64_t)r * ldc + i] = c;
      G[(int64_t)j * ldg + i] = gc[i];
      if (i < j) G[(int64_t)i * ldg + j] = conj(gc[i]);
    }
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  cx<T>* __restrict__ wr = w + (int64_t)r * n;
  const cx<T>* __restrict__ Vr = V + (int64_t)r * sR;
  cx<T> acc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    acc[e] = wr[k < n ? k : n - 1];  // past n: computed, never stored
  }
  constexpr int G2 = EPT >= 8 ? 2 : DG;
  int i = 0;
  for (; i + G2 <= nv; i += G2) {
    cx<T> vv[G2][EPT];
#pragma unroll
    for (int g = 0; g < G2; ++g) {
      const cx<T>* __restrict__ vi = Vr + (int64_t)(i + g) * sI;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int64_t k = base + (int64_t)e * NT;
        vv[g][e] = vi[k < n ? k : n - 1];
      }
    }
#pragma unroll
    for (int g = 0; g < G2; ++g) {
      const cx<T> c = cs[i + g];
#pragma unroll
      for (int e = 0; e < EPT; ++e) cfma(acc[e], vv[g][e], c);
    }
  }
  for (; i < nv; ++i) {
    const cx<T>* __restrict__ vi = Vr + (int64_t)i * sI;
    const cx<T> c = cs[i];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int64_t k = base + (int64_t)e * NT;
      cfma(acc[e], vi[k < n ? k : n - 1], c);
    }
  }
  T nrm = 0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    if (k < n) {
      wr[k] = acc[e];
      nrm += abs2(acc[e]);
    }
  }
  if (partial) {
    nrm = block_sum_real(nrm, sh);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = nrm;
  }
}

// out[r*ldo + i] (=|+=) sum_chunks partial: one wave per output, lane l adds
// chunks l, l+64, ... in order, then a fixed shuffle tree.
template <class T>
__global__ void __launch_bounds__(NT) k_reduce_chunks(const cx<T>* __restrict__ partial, int nv, int nch,
                                                      int nrhs, cx<T>* __restrict__ out, int ldo,
                                                      int accumulate, const int* __restrict__ active) {
  const int64_t t = ((int64_t)blockIdx.x * NT + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (t >= (int64_t)nv * nrhs) return;
  const int r = (int)(t / nv), i = (int)(t % nv);
  if (active && !active[r]) return;
  const cx<T>* p = partial + ((int64_t)r * nv + i) * nch;
  cx<T> acc = mk<T>(0, 0);
  for (int c = lane; c < nch; c += 64) acc = acc + p[c];
  acc.re = wave_sum(acc.re);
  acc.im = wave_sum(acc.im);
  if (lane == 0) {
    cx<T>* o = out + (int64_t)r * ldo + i;
    *o = accumulate ? (*o + acc) : acc;
  }
}

// w[r] += sign * sum_i V_i[r] coef[r*ldc + i]; optional partial |w|^2 per chunk.
// Vectors are added in index order, a few of them loaded together.
// BS: the coefficients are y = R^{-1} g of an FGMRES cycle (R: the rotated
// Hessenberg Hb, [r][m][m + 1] with m = ldc; g: gb, [r][m + 1]; nlim[r]
// steps), solved by every workgroup for its RHS with k_backsolve's
// operations in its order: the triangle and g staged in LDS by the whole
// workgroup, the substitution by one thread.  overwrite: w = sum (w not read).
template <class T, int EPT, bool BS>
__global__ void __launch_bounds__(NT) k_update_multi(const cx<T>* __restrict__ V, int64_t sI, int64_t sR,
                                                     int nv, const cx<T>* __restrict__ coef, int ldc,
                                                     T sign, cx<T>* __restrict__ w, int64_t n,
                                                     T* __restrict__ partial,
                                                     const int* __restrict__ active,
                                                     const int* __restrict__ nlim, const cx<T>* __restrict__ Hb,
                                                     const cx<T>* __restrict__ gb, int overwrite) {
  constexpr int CH = NT * EPT;
  __shared__ cx<T> cs[64];
  __shared__ T sh[8];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  if (nlim) nv = min(nv, nlim[r]);
  if constexpr (BS) {
    constexpr int KT = 32;  // largest step count staged in LDS
    __shared__ cx<T> ht[KT * (KT + 1) / 2];
    __shared__ cx<T> gs[KT];
    const int m = ldc;
    const cx<T>* __restrict__ Hr = Hb + (int64_t)r * m * (m + 1);
    const cx<T>* __restrict__ gr = gb + (int64_t)r * (m + 1);
    const bool lds = nv <= KT;
    if (lds) {
      // ht[l (l + 1) / 2 + i] = R(i, l) = Hr[l (m + 1) + i], i <= l < nv
      for (int e = threadIdx.x; e < nv * KT; e += NT) {
        const int l = e / KT, i = e % KT;
        if (i <= l) ht[l * (l + 1) / 2 + i] = Hr[(int64_t)l * (m + 1) + i];
      }
      for (int i = threadIdx.x; i < nv; i += NT) gs[i] = gr[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = nv - 1; i >= 0; --i) {
        cx<T> acc = lds ? gs[i] : gr[i];
        for (int l = i + 1; l < nv; ++l)
          acc = acc - (lds ? ht[l * (l + 1) / 2 + i] : Hr[(int64_t)l * (m + 1) + i]) * cs[l];
        cs[i] = cdiv(acc, lds ? ht[i * (i + 1) / 2 + i] : Hr[(int64_t)i * (m + 1) + i]);
      }
      for (int i = 0; i < nv; ++i) cs[i] = sign * cs[i];
    }
  } else {
    for (int i = threadIdx.x; i < nv; i += NT) cs[i] = sign * coef[(int64_t)r * ldc + i];
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  cx<T>* __restrict__ wr = w + (int64_t)r * n;
  const cx<T>* __restrict__ Vr = V + (int64_t)r * sR;
  cx<T> acc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    acc[e] = overwrite ? cx<T>{0, 0} : wr[k < n ? k : n - 1];  // past n: computed, never stored
  }
  constexpr int G = EPT >= 8 ? 2 : DG;  // G * EPT loads in flight, within the register budget
  int i = 0;
  for (; i + G <= nv; i += G) {
    cx<T> vv[G][EPT];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const cx<T>* __restrict__ vi = Vr + (int64_t)(i + g) * sI;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int64_t k = base + (int64_t)e * NT;
        vv[g][e] = vi[k < n ? k : n - 1];
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const cx<T> c = cs[i + g];
#pragma unroll
      for (int e = 0; e < EPT; ++e) cfma(acc[e], vv[g][e], c);
    }
  }
  for (; i < nv; ++i) {
    const cx<T>* __restrict__ vi = Vr + (int64_t)i * sI;
    const cx<T> c = cs[i];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int64_t k = base + (int64_t)e * NT;
      cfma(acc[e], vi[k < n ? k : n - 1], c);
    }
  }
  T nrm = 0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    if (k < n) {
      wr[k] = acc[e];
      nrm += abs2(acc[e]);
    }
  }
  if (partial) {
    nrm = block_sum_real(nrm, sh);
    if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = nrm;
  }
}

template <class T, int EPT>
__global__ void __launch_bounds__(NT) k_norm_partial(const cx<T>* __restrict__ w, int64_t n,
                                                     T* __restrict__ partial,
                                                     const int* __restrict__ active) {
  constexpr int CH = NT * EPT;
  __shared__ T sh[8];
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const int64_t base = (int64_t)blockIdx.x * CH + threadIdx.x;
  const cx<T>* __restrict__ wr = w + (int64_t)r * n;
  T acc = 0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int64_t k = base + (int64_t)e * NT;
    acc += abs2(wr[k < n ? k : n - 1]) * (T)(k < n);
  }
  acc = block_sum_real(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)r * gridDim.x + blockIdx.x] = acc;
}

// out[r] = sqrt(sum_chunks partial): one wave per RHS, as k_reduce_chunks.
// zero_done (optional): 1 where the norm is 0, else 0.
template <class T>
__global__ void __launch_bounds__(NT) k_norm_reduce(const T* __restrict__ partial, int nch, int nrhs,
                                                    T* __restrict__ out, const int* __restrict__ active,
                                                    int* __restrict__ zero_done) {
  const int r = (int)(((int64_t)blockIdx.x * NT + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrhs) return;
  if (active && !active[r]) return;
  T acc = 0;
  for (int c = lane; c < nch; c += 64) acc += partial[(int64_t)r * nch + c];
  acc = wave_sum(acc);
  if (lane == 0) {
    const T v = sqrt(acc);
    out[r] = v;
    if (zero_done) zero_done[r] = v == (T)0 ? 1 : 0;
  }
}

// k_norm_reduce (same sum, same bits) for norms the host reads: lane 0 also
// stores them, the RHS norms and the iteration counts into pinned host
// memory (host[r], host[nrhs + r], hnit[r]), so no copies follow.
__global__ void __launch_bounds__(NT) k_norm_reduce_rb(const double* __restrict__ partial, int nch, int nrhs,
                                                       double* __restrict__ out, const double* __restrict__ bnorm,
                                                       const int* __restrict__ nit, double* __restrict__ host,
                                                       int* __restrict__ hnit) {
  const int r = (int)(((int64_t)blockIdx.x * NT + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= nrhs) return;
  double acc = 0;
  for (int c = lane; c < nch; c += 64) acc += partial[(int64_t)r * nch + c];
  acc = wave_sum(acc);
  if (lane == 0) {
    const double v = sqrt(acc);
    out[r] = v;
    host[r] = v;
    host[nrhs + r] = bnorm[r];
    hnit[r] = nit[r];
  }
}

// v = w / ||w|| with ||w|| = sqrt(sum over chunks of the norm partials),
// added as k_norm_reduce adds them (same bits); the workgroup with
// blockIdx.x == 0 also stores ||w|| to den_out[r].
template <class T>
__global__ void __launch_bounds__(NT) k_scale_r(const cx<T>* __restrict__ w, const T* __restrict__ npart,
                                                int nch, int64_t n, cx<T>* __restrict__ v,
                                                T* __restrict__ den_out, const int* __restrict__ active) {
  __shared__ T dsh;
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    T acc = 0;
    for (int c = lane; c < nch; c += 64) acc += npart[(int64_t)r * nch + c];
    acc = wave_sum(acc);
    if (lane == 0) {
      const T d = sqrt(acc);
      dsh = d;
      if (blockIdx.x == 0) den_out[r] = d;
    }
  }
  __syncthreads();
  const T d = dsh;
  const T s = (d > 0) ? (T)1 / d : (T)0;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT)
    v[(int64_t)r * n + k] = s * w[(int64_t)r * n + k];
}

// Position of fine-level dof k (lattice layout: site-major, 2 dofs) in the
// block-major layout of the fine FP32 cycle (4x4-site blocks of 32 dofs,
// sites t-major within a block); Nx = 0: the lattice layout itself
__device__ __forceinline__ int64_t blk_pos(int64_t k, int Nx) {
  if (Nx == 0) return k;
  const int64_t site = k >> 1;
  const int x = (int)(site % Nx), t = (int)(site / Nx);
  return ((int64_t)(t >> 2) * (Nx >> 2) + (x >> 2)) * 32 + (((t & 3) << 2) + (x & 3)) * 2 + (k & 1);
}

// The first cycle of FGMRES from x = 0, started in one launch per RHS r:
// ||b_r|| from the norm partials (k_norm_reduce's sum, same bits); the cycle
// state as k_fgmres_init sets it with beta = ||b_r|| (no parent), a zero
// right-hand side marked solved; v_0 = b_r / ||b_r|| (k_scale's arithmetic),
// and, with vf, its FP32 rounding for the preconditioner (block-major when
// blk_nx > 0, as k_hcol_scale stores it).  Workgroup 0 of each RHS stores
// ||b_r||, the flags and the state.
__global__ void __launch_bounds__(NT) k_fgmres_start(const cd* __restrict__ b, const double* __restrict__ npart,
                                                     int nch, int64_t n, int m, double tol,
                                                     double* __restrict__ bnorm, int* __restrict__ done,
                                                     int* __restrict__ active, int* __restrict__ nit,
                                                     cd* __restrict__ g, double* __restrict__ thr,
                                                     cd* __restrict__ v, cf* __restrict__ vf, int blk_nx) {
  __shared__ double dsh;
  const int r = blockIdx.y;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double acc = 0;
    for (int c = lane; c < nch; c += 64) acc += npart[(int64_t)r * nch + c];
    acc = wave_sum(acc);
    if (lane == 0) dsh = sqrt(acc);
  }
  __syncthreads();
  const double d = dsh;
  const bool on = d > 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bnorm[r] = d;
    done[r] = d == 0.0 ? 1 : 0;
    active[r] = on ? 1 : 0;
    nit[r] = 0;
    g[(int64_t)r * (m + 1)] = mk<double>(on ? d : 0.0, 0);
    thr[r] = tol * d;
  }
  if (!on) return;
  const double sc = 1.0 / d;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
    const cd vv = sc * b[(int64_t)r * n + k];
    v[(int64_t)r * n + k] = vv;
    if (vf) vf[(int64_t)r * n + blk_pos(k, blk_nx)] = mk<float>((float)vv.re, (float)vv.im);
  }
}



// FP32 rounding of a fine-level FP64 block [nrhs][n] into the block-major layout
__global__ void __launch_bounds__(NT) k_convert_blk(const cd* __restrict__ in, cf* __restrict__ out, int Nx,
                                                    int64_t n, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < count; e += (int64_t)gridDim.x * NT) {
    const int64_t r = e / n, k = e % n;
    out[r * n + blk_pos(k, Nx)] = mk<float>((float)in[e].re, (float)in[e].im);
  }
}

template <class T>
__global__ void __launch_bounds__(NT) k_scale(const cx<T>* __restrict__ w, const T* __restrict__ den,
                                              int64_t n, cx<T>* __restrict__ v,
                                              const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const T d = den[r];
  const T s = (d > 0) ? (T)1 / d : (T)0;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT)
    v[(int64_t)r * n + k] = s * w[(int64_t)r * n + k];
}

template <class T>
__global__ void __launch_bounds__(NT) k_axpby(T a, const cx<T>* __restrict__ x, T b,
                                              const cx<T>* __restrict__ y, cx<T>* __restrict__ z,
                                              int64_t n, const int* __restrict__ active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
    const int64_t o = (int64_t)r * n + k;
    const cx<T> yv = y ? y[o] : mk<T>(0, 0);
    z[o] = a * x[o] + b * yv;
  }
}

template <class TO, class TI>
__global__ void __launch_bounds__(NT) k_convert(const cx<TI>* __restrict__ in, cx<TO>* __restrict__ out,
                                                int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < count; k += (int64_t)gridDim.x * NT)
    out[k] = mk<TO>((TO)in[k].re, (TO)in[k].im);
}

// Arnoldi step j of RHS r: rotate column j of H (H[(r*m + j)*(m+1) + i]) by
// the previous Givens rotations, form the new one, update g and the residual
// estimate |g_{j+1}|; stop the RHS when it falls to thr[r], on breakdown, or
// at the last step.
template <class T>
__global__ void __launch_bounds__(NT) k_givens(int j, int m, int nrhs, cx<T>* __restrict__ H,
                                               T* __restrict__ cs, cx<T>* __restrict__ sn,
                                               cx<T>* __restrict__ g, const T* __restrict__ thr,
                                               int* __restrict__ active, int* __restrict__ nit) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  cx<T>* h = H + ((int64_t)r * m + j) * (m + 1);
  T* c = cs + (int64_t)r * m;
  cx<T>* s = sn + (int64_t)r * m;
  cx<T>* gr = g + (int64_t)r * (m + 1);
  for (int i = 0; i < j; ++i) {
    const cx<T> a = h[i], b = h[i + 1];
    h[i] = c[i] * a + s[i] * b;
    h[i + 1] = c[i] * b - conj(s[i]) * a;
  }
  const cx<T> a = h[j], b = h[j + 1];
  const T na = sqrt(abs2(a)), nb = sqrt(abs2(b));
  const T rho = sqrt(na * na + nb * nb);
  T cj;
  cx<T> sj;
  if (na == (T)0) {
    cj = 0;
    sj = mk<T>(1, 0);
    h[j] = b;
  } else {
    cj = na / rho;
    const cx<T> ph = mk<T>(a.re / na, a.im / na);
    sj = ph * conj(b);
    sj = mk<T>(sj.re / rho, sj.im / rho);
    h[j] = rho * ph;
  }
  h[j + 1] = mk<T>(0, 0);
  c[j] = cj;
  s[j] = sj;
  const cx<T> gj = gr[j];
  gr[j] = cj * gj;
  gr[j + 1] = (T)-1 * (conj(sj) * gj);
  nit[r] = j + 1;
  const T res = sqrt(abs2(gr[j + 1]));
  if (res <= thr[r] || nb == (T)0 || j + 1 == m) active[r] = 0;
}


// Hessenberg column j (as k_hcol) followed by the Givens update (as
// k_givens) in one launch; host_flags (pinned host memory, or null) receives
// every RHS's state after the step, so the host can poll it without a copy:
// 0 converged (inactive), 2 active with the residual estimate within a factor
// NEAR of its threshold (the next step will most likely end it), 1 active.
constexpr double NEAR = 32.0;
template <class T>
__device__ __forceinline__ void hcol_givens_rhs(int r, int j, int m, const cx<T>* __restrict__ c1,
                                                const cx<T>* __restrict__ c2, T hnr, cx<T>* __restrict__ H,
                                                T* __restrict__ cs, cx<T>* __restrict__ sn,
                                                cx<T>* __restrict__ g, const T* __restrict__ thr,
                                                int* __restrict__ active, int* __restrict__ nit,
                                                int* __restrict__ host_flags) {
  int code = 0;
  if (active[r]) {
    cx<T>* h = H + ((int64_t)r * m + j) * (m + 1);
    for (int i = 0; i <= j; ++i)
      h[i] = c2 ? c1[(int64_t)r * (m + 1) + i] + c2[(int64_t)r * (m + 1) + i] : c1[(int64_t)r * (m + 1) + i];
    h[j + 1] = mk<T>(hnr, 0);
    T* c = cs + (int64_t)r * m;
    cx<T>* s = sn + (int64_t)r * m;
    cx<T>* gr = g + (int64_t)r * (m + 1);
    for (int i = 0; i < j; ++i) {
      const cx<T> a = h[i], b = h[i + 1];
      h[i] = c[i] * a + s[i] * b;
      h[i + 1] = c[i] * b - conj(s[i]) * a;
    }
    const cx<T> a = h[j], b = h[j + 1];
    const T na = sqrt(abs2(a)), nb = sqrt(abs2(b));
    const T rho = sqrt(na * na + nb * nb);
    T cj;
    cx<T> sj;
    if (na == (T)0) {
      cj = 0;
      sj = mk<T>(1, 0);
      h[j] = b;
    } else {
      cj = na / rho;
      const cx<T> ph = mk<T>(a.re / na, a.im / na);
      sj = ph * conj(b);
      sj = mk<T>(sj.re / rho, sj.im / rho);
      h[j] = rho * ph;
    }
    h[j + 1] = mk<T>(0, 0);
    c[j] = cj;
    s[j] = sj;
    const cx<T> gj = gr[j];
    gr[j] = cj * gj;
    gr[j + 1] = (T)-1 * (conj(sj) * gj);
    nit[r] = j + 1;
    const T res = sqrt(abs2(gr[j + 1]));
    if (res <= thr[r] || nb == (T)0 || j + 1 == m) active[r] = 0;
    code = active[r] ? (res <= (T)NEAR * thr[r] ? 2 : 1) : 0;
  }
  if (host_flags) host_flags[r] = code;
}

template <class T>
__global__ void __launch_bounds__(NT) k_hcol_givens(int j, int m, int nrhs, const cx<T>* __restrict__ c1,
                                                    const cx<T>* __restrict__ c2, const T* __restrict__ hn,
                                                    cx<T>* __restrict__ H, T* __restrict__ cs,
                                                    cx<T>* __restrict__ sn, cx<T>* __restrict__ g,
                                                    const T* __restrict__ thr, int* __restrict__ active,
                                                    int* __restrict__ nit, int* __restrict__ host_flags) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= nrhs) return;
  hcol_givens_rhs<T>(r, j, m, c1, c2, hn[r], H, cs, sn, g, thr, active, nit, host_flags);
}


// The end of a fused Arnoldi step j in one launch: every workgroup sums |w|
// from the chunk partials of |w|^2 (k_norm_reduce's order, same bits);
// workgroup 0 of each RHS forms the Hessenberg column with its Givens update
// as k_hcol_givens does (it may end the RHS and writes the host flag);
// every workgroup forms v_{j+1} = w / |w| and its FP32 rounding for the next
// step's preconditioner (block-major when blk_nx > 0).  The active flag is
// read once when a workgroup starts: for a RHS that this step ends, v_{j+1}
// may or may not be written, and it is never read.
template <class T>
__global__ void __launch_bounds__(NT) k_hcol_scale(int j, int m, const cx<T>* __restrict__ c1,
                                                   const T* __restrict__ npart, int nch, cx<T>* __restrict__ H,
                                                   T* __restrict__ cs, cx<T>* __restrict__ sn,
                                                   cx<T>* __restrict__ g, const T* __restrict__ thr,
                                                   int* __restrict__ active, int* __restrict__ nit,
                                                   int* __restrict__ host_flags, const cx<T>* __restrict__ w,
                                                   int64_t n, cx<T>* __restrict__ v, cf* __restrict__ vf,
                                                   int blk_nx) {
  __shared__ T dsh;
  const int r = blockIdx.y;
  const bool was = active[r] != 0;
  if (!was && blockIdx.x != 0) return;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    T acc = 0;
    if (was)
      for (int c = lane; c < nch; c += 64) acc += npart[(int64_t)r * nch + c];
    acc = wave_sum(acc);
    if (lane == 0) {
      const T d = sqrt(acc);
      dsh = d;
      if (blockIdx.x == 0)
        hcol_givens_rhs<T>(r, j, m, c1, (const cx<T>*)nullptr, d, H, cs, sn, g, thr, active, nit, host_flags);
    }
  }
  __syncthreads();
  if (!was) return;
  const T d = dsh;
  const T sc = (d > 0) ? (T)1 / d : (T)0;
  for (int64_t k = (int64_t)blockIdx.x * NT + threadIdx.x; k < n; k += (int64_t)gridDim.x * NT) {
    const cx<T> vv = sc * w[(int64_t)r * n + k];
    v[(int64_t)r * n + k] = vv;
    vf[(int64_t)r * n + blk_pos(k, blk_nx)] = mk<float>((float)vv.re, (float)vv.im);
  }
}

// y = R^{-1} g with R the rotated (upper triangular) H of nit[r] steps
template <class T>
__global__ void __launch_bounds__(NT) k_backsolve(int m, int nrhs, const cx<T>* __restrict__ H,
                                                  const cx<T>* __restrict__ g,
                                                  const int* __restrict__ nit, cx<T>* __restrict__ y) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= nrhs) return;
  const int k = nit[r];
  cx<T>* yr = y + (int64_t)r * m;
  const cx<T>* Hr = H + (int64_t)r * m * (m + 1);
  const cx<T>* gr = g + (int64_t)r * (m + 1);
  for (int i = k; i < m; ++i) yr[i] = mk<T>(0, 0);
  for (int i = k - 1; i >= 0; --i) {
    cx<T> acc = gr[i];
    for (int l = i + 1; l < k; ++l) acc = acc - Hr[(int64_t)l * (m + 1) + i] * yr[l];
    yr[i] = cdiv(acc, Hr[(int64_t)i * (m + 1) + i]);
  }
}

template <class T>
__global__ void __launch_bounds__(NT) k_fgmres_init(int nrhs, const T* __restrict__ beta,
                                                    const int* __restrict__ parent,
                                                    const int* __restrict__ done, T tol,
                                                    const T* __restrict__ bnorm, int m,
                                                    int* __restrict__ active, int* __restrict__ nit,
                                                    cx<T>* __restrict__ g, T* __restrict__ thr) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= nrhs) return;
  const bool on = (!parent || parent[r]) && (!done || !done[r]) && beta[r] > (T)0;
  active[r] = on ? 1 : 0;
  nit[r] = 0;
  g[(int64_t)r * (m + 1)] = mk<T>(on ? beta[r] : (T)0, 0);
  thr[r] = tol * (bnorm ? bnorm[r] : beta[r]);
}


// ------------------------------------------------------------------ CholQR2 pieces
// Gram partials on the FP64 matrix cores: partial[chunk][i][j] = sum over the
// chunk's k of conj(Y_i[k]) Y_j[k], d <= 64.  A workgroup owns GCH elements
// of k; its waves take the 16 x 16 output tiles (i-tile, j-tile) in turn.
// The k loop has a fixed trip count and clamped loads, so a wave keeps
// several k steps of loads in flight.
constexpr int GCH = 128;
__global__ void __launch_bounds__(NT) k_gram_partial(const cd* __restrict__ Y, int64_t n, int d,
                                                     cd* __restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15;
  const int nt = (d + 15) / 16;
  const int64_t k0 = (int64_t)blockIdx.x * GCH;
  for (int tile = wave; tile < nt * nt; tile += 4) {
    const int i0 = (tile / nt) * 16, j0 = (tile % nt) * 16;
    const int i = i0 + r, j = j0 + r;
    const cd* Yi = Y + (int64_t)(i < d ? i : 0) * n;
    const cd* Yj = Y + (int64_t)(j < d ? j : 0) * n;
    CAcc<double> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll 16
    for (int kk = 0; kk < GCH; kk += 4) {
      const int64_t k = k0 + kk + (lane >> 4);
      const bool in = k < n;
      const int64_t kc = in ? k : 0;
      const cd a = ld_or0(Yi + kc, in && i < d);
      const cd b = ld_or0(Yj + kc, in && j < d);
      cmma(conj(a), b, acc);
    }
    // element v: row i0 + out_row(lane, v), column j0 + lane % 16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = i0 + MF<double>::out_row(lane, v);
      if (ii < d && j < d) partial[((int64_t)blockIdx.x * d + ii) * d + j] = mk(acc.re[v], acc.im[v]);
    }
  }
}

// G[e] = sum over chunks of partial[chunk][e]: a workgroup owns 8 consecutive
// elements (one 128-byte row of every chunk), 32 threads per element stride
// over the chunks, then the 32 sums are added in a fixed order.
__global__ void __launch_bounds__(NT) k_gram_reduce(const cd* __restrict__ partial, int nch, int dd,
                                                    cd* __restrict__ G) {
  __shared__ cd sh[32][8];
  const int t = threadIdx.x, e8 = t & 7, c0 = t >> 3;
  const int e = blockIdx.x * 8 + e8;
  const int ec = e < dd ? e : 0;
  cd acc = mk(0.0, 0.0);
#pragma unroll 4
  for (int c = c0; c < nch; c += 32) acc = acc + partial[(int64_t)c * dd + ec];
  sh[c0][e8] = acc;
  __syncthreads();
  if (t < 8 && blockIdx.x * 8 + t < dd) {
    cd sum = mk(0.0, 0.0);
    for (int q = 0; q < 32; ++q) sum = sum + sh[q][t];
    G[blockIdx.x * 8 + t] = sum;
  }
}

// G + shift * tr(G) * I = R^H R (R upper, positive real diagonal); on exit G
// holds R^{-1} (upper).  One workgroup, the matrix in LDS.  The elimination
// keeps the unscaled upper factor A (row j of A = sqrt(a_jj) times row j of
// R), so a step needs no square root: A_k. -= conj(a_jk) (a_j. / a_jj) for
// k > j.  Then A^{-1} by backward Gauss-Jordan on [A | I] with each row's
// division by its pivot deferred to the end, and R^{-1} = A^{-1} diag(sqrt
// a_jj).  One barrier per step; square roots and divisions by the pivots
// are taken for all rows at once outside the dependent chains.  *fail is
// set on a non-positive pivot.
__global__ void __launch_bounds__(NT) k_cholesky_rinv(cd* __restrict__ G, int d, double shift,
                                                      int* __restrict__ fail) {
  __shared__ cd A[64][65];
  __shared__ cd X[64][65];
  __shared__ double inva[64], sqa[64];
  __shared__ double trs;
  const int t = threadIdx.x;
  // thread (row slot, column) = (t / 64, t % 64): rows stride 4, so no loop
  // divides by the runtime size d
  const int tr = t >> 6, tc = t & 63;
  const bool col_ok = tc < d;
  // all loads of G issued together (a loop of dependent global loads here
  // would cost a memory round trip per element)
#pragma unroll 4
  for (int a = tr; a < d; a += 4) {
    const cd v = G[(col_ok ? a * d + tc : 0)];
    if (col_ok) A[a][tc] = tc >= a ? v : mk(0.0, 0.0);
  }
  __syncthreads();
  if (t < 64) {  // shift * tr(G), summed by wave 0
    const double tr_sum = wave_sum(t < d ? A[t][t].re : 0.0);
    if (t == 0) trs = shift * tr_sum;
  }
  __syncthreads();
  if (t < d) A[t][t].re += trs;
  __syncthreads();
  bool failed = false;
  for (int j = 0; j < d; ++j) {
    const double s = A[j][j].re;  // final since the last barrier; same for every thread
    if (!(s > 0.0)) {
      failed = true;
      break;
    }
    const double inv = 1.0 / s;
    if (tc > j && col_ok) {
      const cd u = inv * A[j][tc];
      for (int k = j + 1 + tr; k <= tc; k += 4) A[k][tc] = A[k][tc] - cjmul(A[j][k], u);
    }
    __syncthreads();
  }
  if (failed) {
    if (t == 0) atomicOr(fail, 1);
    return;
  }
  if (t < d) {
    inva[t] = 1.0 / A[t][t].re;
    sqa[t] = sqrt(A[t][t].re);
  }
  for (int a = tr; a < d; a += 4)
    if (col_ok) X[a][tc] = mk(a == tc ? 1.0 : 0.0, 0.0);
  __syncthreads();
  // Y = unscaled rows of A^{-1}: for j = d-1 .. 0, row j of Y is final (its
  // true value is Y_j / a_jj) and is eliminated from every row i < j
  for (int j = d - 1; j > 0; --j) {
    if (tc >= j && col_ok) {
      const cd u = inva[j] * X[j][tc];
      for (int i = tr; i < j; i += 4) X[i][tc] = X[i][tc] - A[i][j] * u;
    }
    __syncthreads();
  }
  for (int a = tr; a < d; a += 4)
    if (col_ok) G[a * d + tc] = tc >= a ? (inva[a] * sqa[tc]) * X[a][tc] : mk(0.0, 0.0);
}

// Q_j[k] = sum_{i <= j} Y_i[k] Rinv[i][j] on the FP64 matrix cores: a wave
// owns 16 values of k x 16 columns j; K runs over i in chunks of 4.
__global__ void __launch_bounds__(NT) k_right_tri(const cd* __restrict__ Y, const cd* __restrict__ Rinv,
                                                  int64_t n, int d, cd* __restrict__ Q) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int64_t k0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (k0 >= n) return;
  const int64_t k = k0 + r;
  const int nt = (d + 15) / 16;
  for (int jt = 0; jt < nt; ++jt) {
    const int j = jt * 16 + r;
    CAcc<double> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
    const int iend = min(d, jt * 16 + 16);  // Rinv is upper: rows i <= j only
    for (int ic = 0; ic < iend; ic += 4) {
      const int ia = ic + q;  // A[k][i] = Y_i[k], B[i][j] = Rinv[i][j]
      const cd a = ld_or0(Y + (int64_t)(ia < d ? ia : 0) * n + (k < n ? k : 0), ia < d && k < n);
      const cd b = ld_or0(Rinv + (ia < d ? ia : 0) * d + (j < d ? j : 0), ia < d && j < d);
      cmma(a, b, acc);
    }
    // element v: row k0 + out_row(lane, v), column j
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t kk = k0 + MF<double>::out_row(lane, v);
      if (kk < n && j < d) Q[(int64_t)j * n + kk] = mk(acc.re[v], acc.im[v]);
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
// out[r*ldo + i] (=|+=) V_i[r]^H w[r]
template <class T>
void launch_dot_multi_ld(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv,
                         const cx<T>* w, int64_t n, int nrhs, cx<T>* out, int ldo, int accumulate,
                         const int* active, cx<T>* partial) {
  if (nv <= 0) return;
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_dot_multi<T, E>), dim3(nch, nrhs), dim3(NT), 0, s, V, sI, sR,
                                       nv, w, n, partial, active));
  KCHK();
  const int64_t tot = (int64_t)nv * nrhs;
  hipLaunchKernelGGL(k_reduce_chunks<T>, dim3((unsigned)((tot + 3) / 4)), dim3(NT), 0, s, partial,
                     nv, (int)nch, nrhs, out, ldo, accumulate, active);
  KCHK();
}

template <class T>
void launch_update_multi(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv,
                         const cx<T>* coef, int ldc, T sign, cx<T>* w, int64_t n, int nrhs,
                         const int* active, T* norm_out, T* partial, const int* nlim) {
  require(nv <= 64, "update_multi: at most 64 vectors");
  if (nv <= 0) return;
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_update_multi<T, E, false>), dim3(nch, nrhs), dim3(NT), 0, s, V, sI,
                                       sR, nv, coef, ldc, sign, w, n, norm_out ? partial : (T*)nullptr,
                                       active, nlim, (const cx<T>*)nullptr, (const cx<T>*)nullptr, 0));
  KCHK();
  if (norm_out) {
    hipLaunchKernelGGL(k_norm_reduce<T>, dim3((nrhs + 3) / 4), dim3(NT), 0, s, partial, (int)nch,
                       nrhs, norm_out, active, (int*)nullptr);
    KCHK();
  }
}

template <class T>
void launch_update_backsolve(hipStream_t s, const cx<T>* Z, int64_t sI, int64_t n, int m, const cx<T>* H,
                             const cx<T>* g, const int* nit, cx<T>* x, int nrhs, bool overwrite) {
  require(m >= 1 && m <= 64, "update_backsolve: 1 <= m <= 64");
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_update_multi<T, E, true>), dim3(nch, nrhs), dim3(NT), 0, s, Z, sI,
                                       n, m, (const cx<T>*)nullptr, m, (T)1, x, n, (T*)nullptr,
                                       (const int*)nullptr, nit, H, g, overwrite ? 1 : 0));
  KCHK();
}

template <class T>
int launch_dot_partial2(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv, const cx<T>* w,
                        const cx<T>* u, int64_t n, int nrhs, const int* active, cx<T>* partial) {
  require(nv >= 1 && nv <= 64, "dot_partial2: 1 to 64 vectors");
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_dot_multi2<T, E>), dim3(nch, nrhs), dim3(NT), 0, s, V, sI, sR, nv, w, u,
                                       n, partial, active));
  KCHK();
  return (int)nch;
}

template <class T>
void launch_update_gram(hipStream_t s, const cx<T>* V, int64_t sI, int64_t sR, int nv, const cx<T>* dpart,
                        int nchd, cx<T>* gram, int ldg, cx<T>* coef_out, int ldc, cx<T>* w, int64_t n, int nrhs,
                        const int* active, T* norm_partial) {
  require(nv >= 1 && nv <= 64 && nv <= ldg, "update_gram: 1 to 64 vectors");
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  require((int)nch == nchd, "update_gram: chunking differs from the dot partials'");
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_update_gram<T, E>), dim3(nch, nrhs), dim3(NT), 0, s, V, sI, sR, nv,
                                       dpart, nchd, gram, ldg, coef_out, ldc, w, n, norm_partial, active));
  KCHK();
}


template <class T>
void launch_hcol_scale(hipStream_t s, int j, int m, int nrhs, const cx<T>* c1, const T* npart, cx<T>* H, T* cs,
                       cx<T>* sn, cx<T>* g, const T* thr, int* active, int* nit, int* host_flags, const cx<T>* w,
                       int64_t n, cx<T>* v, cf* vf, int blk_nx) {
  const unsigned nch = nchunks(n, pick_ept(n, nrhs));  // the chunks of k_update_gram
  const unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_hcol_scale<T>, dim3(gx, nrhs), dim3(NT), 0, s, j, m, c1, npart, (int)nch, H, cs, sn, g, thr,
                     active, nit, host_flags, w, n, v, vf, blk_nx);
  KCHK();
}

void launch_convert_blk(hipStream_t s, const cd* in, cf* out, int Nx, int Nt, int nrhs) {
  const int64_t n = (int64_t)Nx * Nt * 2, cnt = n * nrhs;
  const unsigned gx = (unsigned)std::min<int64_t>((cnt + NT - 1) / NT, 4096);
  hipLaunchKernelGGL(k_convert_blk, dim3(gx), dim3(NT), 0, s, in, out, Nx, n, cnt);
  KCHK();
}


template <class T>
void launch_scale_r(hipStream_t s, const cx<T>* w, const T* npart, int64_t n, int nrhs, cx<T>* v, T* den_out,
                    const int* active) {
  const unsigned nch = nchunks(n, pick_ept(n, nrhs));  // the chunks of k_update_gram
  unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_scale_r<T>, dim3(gx, nrhs), dim3(NT), 0, s, w, npart, (int)nch, n, v, den_out, active);
  KCHK();
}

void launch_fgmres_start(hipStream_t s, const cd* b, int64_t n, int nrhs, double* partial, int m, double tol,
                         double* bnorm, int* done, int* active, int* nit, cd* g, double* thr, cd* v, cf* vf,
                         int blk_nx) {
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_norm_partial<double, E>), dim3(nch, nrhs), dim3(NT), 0, s, b, n,
                                       partial, (const int*)nullptr));
  KCHK();
  const unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_fgmres_start, dim3(gx, nrhs), dim3(NT), 0, s, b, partial, (int)nch, n, m, tol, bnorm,
                     done, active, nit, g, thr, v, vf, blk_nx);
  KCHK();
}

template <class T>
void launch_norm(hipStream_t s, const cx<T>* w, int64_t n, int nrhs, T* out, const int* active,
                 T* partial, int* zero_done) {
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_norm_partial<T, E>), dim3(nch, nrhs), dim3(NT), 0, s, w, n,
                                       partial, active));
  KCHK();
  hipLaunchKernelGGL(k_norm_reduce<T>, dim3((nrhs + 3) / 4), dim3(NT), 0, s, partial, (int)nch,
                     nrhs, out, active, zero_done);
  KCHK();
}

void launch_norm_readback(hipStream_t s, const cd* w, int64_t n, int nrhs, double* out, double* partial,
                          const double* bnorm, const int* nit, double* host, int* hnit) {
  const int ept = pick_ept(n, nrhs);
  const unsigned nch = nchunks(n, ept);
  EPT_DISPATCH(ept, hipLaunchKernelGGL((k_norm_partial<double, E>), dim3(nch, nrhs), dim3(NT), 0, s, w, n,
                                       partial, (const int*)nullptr));
  KCHK();
  hipLaunchKernelGGL(k_norm_reduce_rb, dim3((nrhs + 3) / 4), dim3(NT), 0, s, partial, (int)nch, nrhs, out, bnorm,
                     nit, host, hnit);
  KCHK();
}

template <class T>
void launch_scale(hipStream_t s, const cx<T>* w, const T* den, int64_t n, int nrhs, cx<T>* v,
                  const int* active) {
  unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_scale<T>, dim3(gx, nrhs), dim3(NT), 0, s, w, den, n, v, active);
  KCHK();
}

template <class T>
void launch_axpby(hipStream_t s, T a, const cx<T>* x, T b, const cx<T>* y, cx<T>* z, int64_t n,
                  int nrhs, const int* active) {
  unsigned gx = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 1024);
  hipLaunchKernelGGL(k_axpby<T>, dim3(gx, nrhs), dim3(NT), 0, s, a, x, b, y, z, n, active);
  KCHK();
}

template <class TO, class TI>
void launch_convert(hipStream_t s, const cx<TI>* in, cx<TO>* out, int64_t count) {
  unsigned gx = (unsigned)std::min<int64_t>((count + NT - 1) / NT, 65535);
  hipLaunchKernelGGL((k_convert<TO, TI>), dim3(gx), dim3(NT), 0, s, in, out, count);
  KCHK();
}

template <class T>
void launch_givens(hipStream_t s, int j, int m, int nrhs, cx<T>* H, T* cs, cx<T>* sn, cx<T>* g,
                   const T* thr, int* active, int* nit) {
  hipLaunchKernelGGL(k_givens<T>, dim3((nrhs + NT - 1) / NT), dim3(NT), 0, s, j, m, nrhs, H, cs, sn, g,
                     thr, active, nit);
  KCHK();
}

template <class T>
void launch_hcol_givens(hipStream_t s, int j, int m, int nrhs, const cx<T>* c1, const cx<T>* c2, const T* hn,
                        cx<T>* H, T* cs, cx<T>* sn, cx<T>* g, const T* thr, int* active, int* nit,
                        int* host_flags) {
  hipLaunchKernelGGL(k_hcol_givens<T>, dim3((nrhs + NT - 1) / NT), dim3(NT), 0, s, j, m, nrhs, c1, c2, hn, H,
                     cs, sn, g, thr, active, nit, host_flags);
  KCHK();
}


template <class T>
void launch_backsolve(hipStream_t s, int m, int nrhs, const cx<T>* H, const cx<T>* g, const int* nit,
                      cx<T>* y) {
  hipLaunchKernelGGL(k_backsolve<T>, dim3((nrhs + NT - 1) / NT), dim3(NT), 0, s, m, nrhs, H, g, nit, y);
  KCHK();
}

template <class T>
void launch_fgmres_init(hipStream_t s, int nrhs, const T* beta, const int* parent, const int* done,
                        T tol, const T* bnorm, int m, int* active, int* nit, cx<T>* g, T* thr) {
  hipLaunchKernelGGL(k_fgmres_init<T>, dim3((nrhs + NT - 1) / NT), dim3(NT), 0, s, nrhs, beta, parent,
                     done, tol, bnorm, m, active, nit, g, thr);
  KCHK();
}


void launch_gram(hipStream_t s, const cd* Y, int64_t n, int d, cd* G, cd* partial) {
  require(d >= 1 && d <= 64, "orthonormalize: 1 <= d <= 64");
  const unsigned nch = (unsigned)((n + GCH - 1) / GCH);
  hipLaunchKernelGGL(k_gram_partial, dim3(nch), dim3(NT), 0, s, Y, n, d, partial);
  KCHK();
  hipLaunchKernelGGL(k_gram_reduce, dim3((d * d + 7) / 8), dim3(NT), 0, s, partial, (int)nch, d * d, G);
  KCHK();
}

int64_t gram_partials(int64_t n) { return (n + GCH - 1) / GCH; }


// ------------------------------------------------------------------ Hutch++ projection
// z = zeta - Q (Q^H zeta) for a block of k vectors as two FP64 matrix-core
// products.  Q: d basis vectors [d][n]; Z: k vectors [k][n]; C: d x k
// coefficients, C[i][r] = Q_i^H Z_r, stored at C[i * k + r].
//
// Coefficient partials: a workgroup owns PCH values of the element index e;
// its waves take the 16 x 16 tiles (i-tile, r-tile) of C in turn and sum
// conj(Q_i[e]) Z_r[e] over the chunk (M = i, N = r, K = e in steps of 4).
constexpr int PCH = 256;
__global__ void __launch_bounds__(NT) k_proj_partial(const cd* __restrict__ Q, int d, const cd* __restrict__ Z,
                                                     int k, int64_t n, cd* __restrict__ partial) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int nti = (d + 15) / 16, ntr = (k + 15) / 16;
  const int64_t e0 = (int64_t)blockIdx.x * PCH;
  for (int tile = wave; tile < nti * ntr; tile += 4) {
    const int i0 = (tile / ntr) * 16, r0 = (tile % ntr) * 16;
    const int i = i0 + l16, r = r0 + l16;
    const cd* Qi = Q + (int64_t)(i < d ? i : 0) * n;
    const cd* Zr = Z + (int64_t)(r < k ? r : 0) * n;
    CAcc<double> acc{{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll 16
    for (int kk = 0; kk < PCH; kk += 4) {
      const int64_t e = e0 + kk + (lane >> 4);
      const bool in = e < n;
      const int64_t ec = in ? e : 0;
      const cd a = ld_or0(Qi + ec, in && i < d);
      const cd b = ld_or0(Zr + ec, in && r < k);
      cmma(conj(a), b, acc);
    }
    // element v: row i0 + out_row(lane, v) of C, column r
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = i0 + MF<double>::out_row(lane, v);
      if (ii < d && r < k) partial[((int64_t)blockIdx.x * d + ii) * k + r] = mk(acc.re[v], acc.im[v]);
    }
  }
}

// Z_r[e] -= sum_i Q_i[e] C[i][r]: a wave owns 16 values of e and every
// r-tile (at most 4, k <= 64); M = r, N = e, K = i in steps of 4, so each Q
// value is loaded once and serves all k vectors, and each Z value is read and
// written once.
__global__ void __launch_bounds__(NT) k_proj_update(const cd* __restrict__ Q, int d, const cd* __restrict__ C,
                                                    int k, int64_t n, cd* __restrict__ Z) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int64_t e0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (e0 >= n) return;
  const int64_t e = e0 + l16;
  const bool ein = e < n;
  const int ntr = (k + 15) / 16;
  CAcc<double> acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = CAcc<double>{{0, 0, 0, 0}, {0, 0, 0, 0}};
  for (int i0 = 0; i0 < d; i0 += 4) {
    const int i = i0 + q;  // B[i][e] = Q_i[e]; A[r][i] = C[i][r]
    const cd b = ld_or0(Q + (int64_t)(i < d ? i : 0) * n + (ein ? e : 0), i < d && ein);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ntr) {
        const int r = t * 16 + l16;
        const cd a = ld_or0(C + (int64_t)(i < d ? i : 0) * k + (r < k ? r : 0), i < d && r < k);
        cmma(a, b, acc[t]);
      }
    }
  }
  // element v of tile t: vector r = 16 t + out_row(lane, v), element e
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= ntr) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = t * 16 + MF<double>::out_row(lane, v);
      if (r < k && ein) {
        cd* zp = Z + (int64_t)r * n + e;
        const cd z = *zp;
        *zp = mk(z.re - acc[t].re[v], z.im - acc[t].im[v]);
      }
    }
  }
}

int64_t proj_partials(int64_t n) { return (n + PCH - 1) / PCH; }

void launch_project(hipStream_t s, const cd* Q, int d, cd* Z, int k, int64_t n, cd* C, cd* partial) {
  require(d >= 1 && d <= 64 && k >= 1 && k <= 64, "projection: 1 <= d, k <= 64");
  const unsigned nch = (unsigned)proj_partials(n);
  hipLaunchKernelGGL(k_proj_partial, dim3(nch), dim3(NT), 0, s, Q, d, Z, k, n, partial);
  KCHK();
  hipLaunchKernelGGL(k_gram_reduce, dim3((d * k + 7) / 8), dim3(NT), 0, s, partial, (int)nch, d * k, C);
  KCHK();
  hipLaunchKernelGGL(k_proj_update, dim3((unsigned)((n + 63) / 64)), dim3(NT), 0, s, Q, d, C, k, n, Z);
  KCHK();
}

// out = gamma5 in on the fine level: the spin-1 component (odd dof) negated
__global__ void __launch_bounds__(NT) k_gamma5(const cd* __restrict__ in, cd* __restrict__ out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= count) return;
  const cd v = in[i];
  out[i] = (i & 1) ? mk(-v.re, -v.im) : v;
}

void launch_gamma5(hipStream_t s, const cd* in, cd* out, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_gamma5, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, s, in, out, count);
  KCHK();
}

__global__ void k_fill_int(int* __restrict__ p, int count, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

void launch_fill_int(hipStream_t s, int* p, int count, int v) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3((count + NT - 1) / NT), dim3(NT), 0, s, p, count, v);
  KCHK();
}

void launch_cholesky_rinv(hipStream_t s, cd* G, int d, double shift, int* fail_dev) {
  require(d >= 1 && d <= 64, "orthonormalize: 1 <= d <= 64");
  hipLaunchKernelGGL(k_cholesky_rinv, dim3(1), dim3(NT), 0, s, G, d, shift, fail_dev);
  KCHK();
}

void launch_right_tri(hipStream_t s, const cd* Y, const cd* Rinv, int64_t n, int d, cd* Q) {
  hipLaunchKernelGGL(k_right_tri, dim3((unsigned)((n + 63) / 64)), dim3(NT), 0, s, Y, Rinv, n, d, Q);
  KCHK();
}

#define INST(T)                                                                                   \
  template void launch_dot_multi_ld<T>(hipStream_t, const cx<T>*, int64_t, int64_t, int,          \
                                       const cx<T>*, int64_t, int, cx<T>*, int, int, const int*,  \
                                       cx<T>*);                                                   \
  template void launch_update_multi<T>(hipStream_t, const cx<T>*, int64_t, int64_t, int,          \
                                       const cx<T>*, int, T, cx<T>*, int64_t, int, const int*, T*, \
                                       T*, const int*);                                           \
  template void launch_norm<T>(hipStream_t, const cx<T>*, int64_t, int, T*, const int*, T*, int*);       \
  template void launch_scale<T>(hipStream_t, const cx<T>*, const T*, int64_t, int, cx<T>*,         \
                                const int*);                                                      \
  template void launch_axpby<T>(hipStream_t, T, const cx<T>*, T, const cx<T>*, cx<T>*, int64_t, int, \
                                const int*);                                                      \
  template void launch_givens<T>(hipStream_t, int, int, int, cx<T>*, T*, cx<T>*, cx<T>*, const T*, \
                                 int*, int*);                                                     \
  template int launch_dot_partial2<T>(hipStream_t, const cx<T>*, int64_t, int64_t, int, const cx<T>*, \
                                      const cx<T>*, int64_t, int, const int*, cx<T>*);              \
  template void launch_update_gram<T>(hipStream_t, const cx<T>*, int64_t, int64_t, int, const cx<T>*, \
                                      int, cx<T>*, int, cx<T>*, int, cx<T>*, int64_t, int,          \
                                      const int*, T*);                                             \
  template void launch_hcol_scale<T>(hipStream_t, int, int, int, const cx<T>*, const T*, cx<T>*, T*, \
                                     cx<T>*, cx<T>*, const T*, int*, int*, int*, const cx<T>*,       \
                                     int64_t, cx<T>*, cf*, int);                                    \
  template void launch_scale_r<T>(hipStream_t, const cx<T>*, const T*, int64_t, int, cx<T>*, T*,    \
                                  const int*);                                                   \
  template void launch_hcol_givens<T>(hipStream_t, int, int, int, const cx<T>*, const cx<T>*,       \
                                      const T*, cx<T>*, T*, cx<T>*, cx<T>*, const T*, int*, int*,    \
                                      int*);                                                       \
  template void launch_backsolve<T>(hipStream_t, int, int, const cx<T>*, const cx<T>*, const int*, \
                                    cx<T>*);                                                      \
  template void launch_update_backsolve<T>(hipStream_t, const cx<T>*, int64_t, int64_t, int,         \
                                           const cx<T>*, const cx<T>*, const int*, cx<T>*, int, bool); \
  template void launch_fgmres_init<T>(hipStream_t, int, const T*, const int*, const int*, T,       \
                                      const T*, int, int*, int*, cx<T>*, T*);
INST(double)
INST(float)
#undef INST
template void launch_convert<float, double>(hipStream_t, const cd*, cf*, int64_t);
template void launch_convert<double, float>(hipStream_t, const cf*, cd*, int64_t);

}  // namespace mgm
