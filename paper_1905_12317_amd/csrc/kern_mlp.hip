// Kernels of the template-proposal network: a tiled GEMM on MFMA (bf16 or
// FP32 operands, FP32 accumulation) with bias / ReLU / ReLU-mask epilogues,
// two-head softmax cross-entropy, column sums, AdamW, feature extraction,
// standardised row gathers, per-row top-k and the small bookkeeping kernels
// of the proposal search.
#include <hip/hip_runtime.h>

#include "mlp_kernels.h"

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// block-wide reductions over 256 threads (4 waves); red holds 4 floats
__device__ float block_max(float v, float* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__device__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename T>
__device__ __forceinline__ T from_float(float x) {
  return static_cast<T>(x);
}

// ---------------------------------------------------------------- GEMM

// 64 x 64 output tile per workgroup, 4 waves of 32 x 32 (one MFMA
// accumulator each), K staged through LDS in chunks of 32.  Both operands
// sit in LDS with k contiguous per row (A: [i][k], B: [j][k]).
template <typename T>
__global__ void __launch_bounds__(kThreads) gemm_kernel(GemmArgs g) {
  constexpr bool BF = sizeof(T) == 2;
  constexpr int TM = 64, TN = 64, KC = 32;
  constexpr int LS = BF ? KC + 8 : KC + 1;  // row stride in elements
  __shared__ __attribute__((aligned(16))) T As[TM * LS];
  __shared__ __attribute__((aligned(16))) T Bs[TN * LS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);
  const T zero = from_float<T>(0.f);
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  for (int k0 = 0; k0 < g.K; k0 += KC) {
    if (g.sak == 1) {
      const int i = tid >> 2, kk = (tid & 3) * 8;
      const long long gi = i0 + i;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + kk + e;
        As[i * LS + kk + e] = (gi < g.M && gk < g.K) ? A[gi * g.sai + gk] : zero;
      }
    } else {
      const int kk = tid >> 3, ii = (tid & 7) * 8;
      const long long gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gi = i0 + ii + e;
        As[(ii + e) * LS + kk] = (gi < g.M && gk < g.K) ? A[gi + gk * g.sak] : zero;
      }
    }
    if (g.sbk == 1) {
      const int j = tid >> 2, kk = (tid & 3) * 8;
      const long long gj = j0 + j;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + kk + e;
        Bs[j * LS + kk + e] = (gj < g.N && gk < g.K) ? B[gk + gj * g.sbj] : zero;
      }
    } else {
      const int kk = tid >> 3, jj = (tid & 7) * 8;
      const long long gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gj = j0 + jj + e;
        Bs[(jj + e) * LS + kk] = (gj < g.N && gk < g.K) ? B[gk * g.sbk + gj] : zero;
      }
    }
    __syncthreads();
    const int r = lane & 31, h = lane >> 5;
    if constexpr (BF) {
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(wi + r) * LS + 16 * s + 8 * h]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[(wj + r) * LS + 16 * s + 8 * h]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < KC / 2; ++s) {
        const float a = As[(wi + r) * LS + 2 * s + h];
        const float b = Bs[(wj + r) * LS + 2 * s + h];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int j = j0 + wj + (lane & 31);
  if (j >= g.N) return;
  const float bj = g.bias ? g.bias[j] : 0.f;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const long long i = i0 + wi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (i >= g.M) continue;
    float z = acc[v] + bj;
    if (g.mask && !(g.mask[i * g.ldm + j] > 0.f)) z = 0.f;
    if (g.C) g.C[i * g.ldc + j] = z;
    if (g.Cb) static_cast<T*>(g.Cb)[i * g.ldcb + j] = from_float<T>(g.relu ? fmaxf(z, 0.f) : z);
  }
}

// bf16 GEMM, tiled for the wide layers: a (64 MI) x (64 NI) output tile per
// workgroup of 4 waves (2 x 2), each wave (32 MI) x (32 NI) in MI x NI
// accumulators of v_mfma_f32_32x32x16_bf16.  K runs in chunks of KC through
// two LDS buffers ([row][k], KC + 8 bf16 per row; KC = 32 for the large
// tile, 64 for the small one): the next chunk is loaded into
// registers (16-byte loads where the operand's rows are 16-byte aligned,
// else element loads) while the current one feeds the MFMAs.  Split K
// (kparts > 1): workgroup z of the grid sums its K range into
// part[z][M][N] and gemm_reduce_kernel adds the parts and applies the
// epilogue; otherwise the epilogue (bias, ReLU mask, FP32 and bf16 outputs)
// is applied here, as in gemm_kernel.
template <int R, int KC>
struct TileLoad {
  // R rows x KC k of bf16 as 16-byte vectors of 8: V per thread
  static constexpr int V = R * KC / (8 * 256);
  uint4 v[V];
};

// vector u of this thread: k-contiguous operands take 8 consecutive k of one
// row, row-contiguous ones 8 consecutive rows at one k
template <int R, int KC>
__device__ __forceinline__ void tile_coords(int u, bool kc, int& row, int& k) {
  const int vi = threadIdx.x + 256 * u;
  if (kc) {
    row = vi / (KC / 8);
    k = (vi % (KC / 8)) * 8;
  } else {
    k = vi / (R / 8);
    row = (vi % (R / 8)) * 8;
  }
}

// rows r0.. of an operand with element (row, k) at P[row * sr + k * sk]; kc:
// k-contiguous (sk == 1), else row-contiguous (sr == 1); vec: 16-byte loads
template <int R, int KC>
__device__ __forceinline__ void tile_load(TileLoad<R, KC>& t, const __bf16* __restrict__ P, long long sr,
                                          long long sk, int r0, int nrows, int k0, int K, bool kc, bool vec) {
#pragma unroll
  for (int u = 0; u < TileLoad<R, KC>::V; ++u) {
    int row, k;
    tile_coords<R, KC>(u, kc, row, k);
    const int gr = r0 + row, gk = k0 + k;
    __bf16 e[8];
    if (kc) {
      if (vec && gr < nrows && gk + 8 <= K) {
        t.v[u] = *reinterpret_cast<const uint4*>(P + gr * sr + gk);
        continue;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) e[q] = (gr < nrows && gk + q < K) ? P[gr * sr + gk + q] : static_cast<__bf16>(0.f);
    } else {
      if (vec && gk < K && gr + 8 <= nrows) {
        t.v[u] = *reinterpret_cast<const uint4*>(P + gk * sk + gr);
        continue;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) e[q] = (gr + q < nrows && gk < K) ? P[(gr + q) + gk * sk] : static_cast<__bf16>(0.f);
    }
    t.v[u] = *reinterpret_cast<const uint4*>(e);
  }
}

template <int R, int KC>
__device__ __forceinline__ void tile_store(const TileLoad<R, KC>& t, __bf16* __restrict__ S, bool kc) {
  constexpr int TS = KC + 8;  // LDS row stride (bf16)
#pragma unroll
  for (int u = 0; u < TileLoad<R, KC>::V; ++u) {
    int row, k;
    tile_coords<R, KC>(u, kc, row, k);
    if (kc) {
      *reinterpret_cast<uint4*>(S + row * TS + k) = t.v[u];
    } else {
      const __bf16* e = reinterpret_cast<const __bf16*>(&t.v[u]);
#pragma unroll
      for (int q = 0; q < 8; ++q) S[(row + q) * TS + k] = e[q];
    }
  }
}

template <int MI, int NI, int KC>
__global__ void __launch_bounds__(kThreads) gemm_bf16_tiled(GemmArgs g, int kparts, float* __restrict__ part) {
  constexpr int TM = 64 * MI, TN = 64 * NI, TS = KC + 8;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][TM * TS];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TN * TS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int wm = wave >> 1, wn = wave & 1;
  const __bf16* A = static_cast<const __bf16*>(g.A);
  const __bf16* B = static_cast<const __bf16*>(g.B);
  const bool akc = g.sak == 1, bkc = g.sbk == 1;
  // A rows are i (stride sai, k stride sak); B "rows" are j (stride sbj, k stride sbk)
  const bool avec = (akc ? g.sai : g.sak) % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool bvec = (bkc ? g.sbj : g.sbk) % 8 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  // K range of this workgroup
  const int nch = (g.K + KC - 1) / KC;
  const int per = (nch + kparts - 1) / kparts;
  const int c0 = blockIdx.z * per, c1 = min(nch, c0 + per);
  f32x16 acc[MI][NI];
#pragma unroll
  for (int a = 0; a < MI; ++a)
#pragma unroll
    for (int b = 0; b < NI; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;
  TileLoad<TM, KC> ta;
  TileLoad<TN, KC> tb;
  if (c0 < c1) {
    tile_load<TM, KC>(ta, A, g.sai, g.sak, i0, g.M, c0 * KC, g.K, akc, avec);
    tile_load<TN, KC>(tb, B, g.sbj, g.sbk, j0, g.N, c0 * KC, g.K, bkc, bvec);
    tile_store<TM, KC>(ta, As[0], akc);
    tile_store<TN, KC>(tb, Bs[0], bkc);
  }
  __syncthreads();
  const int r = lane & 31, h = lane >> 5;
  for (int c = c0; c < c1; ++c) {
    const int cur = (c - c0) & 1;
    const bool more = c + 1 < c1;
    if (more) {
      tile_load<TM, KC>(ta, A, g.sai, g.sak, i0, g.M, (c + 1) * KC, g.K, akc, avec);
      tile_load<TN, KC>(tb, B, g.sbj, g.sbk, j0, g.N, (c + 1) * KC, g.K, bkc, bvec);
    }
#pragma unroll
    for (int st = 0; st < KC / 16; ++st) {
      bf16x8 av[MI], bv[NI];
#pragma unroll
      for (int a = 0; a < MI; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(&As[cur][(wm * 32 * MI + 32 * a + r) * TS + 16 * st + 8 * h]);
#pragma unroll
      for (int b = 0; b < NI; ++b)
        bv[b] = *reinterpret_cast<const bf16x8*>(&Bs[cur][(wn * 32 * NI + 32 * b + r) * TS + 16 * st + 8 * h]);
#pragma unroll
      for (int a = 0; a < MI; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) {
      tile_store<TM, KC>(ta, As[cur ^ 1], akc);
      tile_store<TN, KC>(tb, Bs[cur ^ 1], bkc);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NI; ++b) {
    const int j = j0 + wn * 32 * NI + 32 * b + r;
    if (j >= g.N) continue;
    const float bj = (kparts == 1 && g.bias) ? g.bias[j] : 0.f;
#pragma unroll
    for (int a = 0; a < MI; ++a)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const long long i = i0 + wm * 32 * MI + 32 * a + 8 * (v >> 2) + 4 * h + (v & 3);
        if (i >= g.M) continue;
        if (kparts > 1) {
          part[(static_cast<size_t>(blockIdx.z) * g.M + i) * g.N + j] = acc[a][b][v];
          continue;
        }
        float z = acc[a][b][v] + bj;
        if (g.mask && !(g.mask[i * g.ldm + j] > 0.f)) z = 0.f;
        if (g.C) g.C[i * g.ldc + j] = z;
        if (g.Cb) static_cast<__bf16*>(g.Cb)[i * g.ldcb + j] = static_cast<__bf16>(g.relu ? fmaxf(z, 0.f) : z);
      }
  }
}

// sum of the K parts in a fixed order, then the epilogue of gemm_kernel
__global__ void gemm_reduce_kernel(GemmArgs g, int kparts, const float* __restrict__ part) {
  const size_t total = static_cast<size_t>(g.M) * g.N;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const long long i = static_cast<long long>(t / g.N), j = static_cast<long long>(t - i * g.N);
    float z = 0.f;
    for (int p = 0; p < kparts; ++p) z += part[p * total + t];
    if (g.bias) z += g.bias[j];
    if (g.mask && !(g.mask[i * g.ldm + j] > 0.f)) z = 0.f;
    if (g.C) g.C[i * g.ldc + j] = z;
    if (g.Cb) static_cast<__bf16*>(g.Cb)[i * g.ldcb + j] = static_cast<__bf16>(g.relu ? fmaxf(z, 0.f) : z);
  }
}

// ---------------------------------------------------------------- rows

template <typename T>
__global__ void standardise_kernel(const float* __restrict__ x, const int32_t* __restrict__ idx, int B, int D,
                                   const float* __restrict__ mu, const float* __restrict__ is, T* __restrict__ X) {
  const size_t total = static_cast<size_t>(B) * D;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int b = static_cast<int>(t / D);
    const int f = static_cast<int>(t - static_cast<size_t>(b) * D);
    const size_t row = idx ? static_cast<size_t>(idx[b]) : static_cast<size_t>(b);
    X[t] = from_float<T>((x[row * D + f] - mu[f]) * is[f]);
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) softmax_ce_kernel(const float* __restrict__ logits, int B, int D, int ldz,
                                                              int n_t, int n_s, const int32_t* __restrict__ lab_t,
                                                              const int32_t* __restrict__ lab_s,
                                                              const int32_t* __restrict__ idx, float* __restrict__ dZ,
                                                              T* __restrict__ dZb, float* __restrict__ row_loss) {
  __shared__ float red[4];
  const int b = blockIdx.x;
  const float* z = logits + static_cast<size_t>(b) * D;
  const int r = idx ? idx[b] : b;
  const float invB = 1.f / static_cast<float>(B);
  float loss = 0.f;
  for (int head = 0; head < 2; ++head) {
    const int lo = head == 0 ? 0 : n_t;
    const int width = head == 0 ? n_t : n_s;
    if (width == 0) continue;
    const int lab = lo + (head == 0 ? lab_t[r] : lab_s[r]);
    float mx = -__builtin_inff();
    for (int j = lo + threadIdx.x; j < lo + width; j += kThreads) mx = fmaxf(mx, z[j]);
    mx = block_max(mx, red);
    float se = 0.f;
    for (int j = lo + threadIdx.x; j < lo + width; j += kThreads) se += __expf(z[j] - mx);
    se = block_sum(se, red);
    const float inv = 1.f / se;
    for (int j = lo + threadIdx.x; j < lo + width; j += kThreads) {
      const float d = (__expf(z[j] - mx) * inv - (j == lab ? 1.f : 0.f)) * invB;
      dZ[static_cast<size_t>(b) * ldz + j] = d;
      if (dZb) dZb[static_cast<size_t>(b) * ldz + j] = from_float<T>(d);
    }
    loss += __logf(se) + mx - z[lab];
  }
  // padding columns of the gradient rows
  for (int j = D + threadIdx.x; j < ldz; j += kThreads) {
    dZ[static_cast<size_t>(b) * ldz + j] = 0.f;
    if (dZb) dZb[static_cast<size_t>(b) * ldz + j] = from_float<T>(0.f);
  }
  if (threadIdx.x == 0) row_loss[b] = loss;
}

__global__ void __launch_bounds__(kThreads) mean_kernel(const float* __restrict__ v, int n, float* __restrict__ out) {
  __shared__ float red[4];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += kThreads) s += v[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s / static_cast<float>(n);
}

// db[j] = sum_b dZ[b][j]: a workgroup per 64 columns, its 4 waves summing a
// quarter of the rows each (coalesced across the columns), then the four
// partial sums added in a fixed order.
__global__ void colsum_kernel(const float* __restrict__ dZ, int B, int N, int ld, float* __restrict__ db) {
  __shared__ float part[4][64];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  float s = 0.f;
  if (j < N) {
    const int b0 = g * ((B + 3) / 4), b1 = min(B, b0 + (B + 3) / 4);
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += dZ[static_cast<size_t>(b) * ld + j];
  }
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && j < N) db[j] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

template <typename T>
__global__ void adamw_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps, float wd,
                             float bc1, float bc2, T* __restrict__ wc) {
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    const float mh = mt / bc1;
    const float vh = vt / bc2;
    const float wt = w[t];
    const float wn = wt - lr * (mh / (sqrtf(vh) + eps) + wd * wt);
    w[t] = wn;
    if (wc) wc[t] = from_float<T>(wn);
  }
}

template <typename T>
__global__ void convert_kernel(const float* __restrict__ w, size_t n, T* __restrict__ wc) {
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
       t += static_cast<size_t>(gridDim.x) * blockDim.x)
    wc[t] = from_float<T>(w[t]);
}

// kind 0: F[m n_q + q] = |a(k_m; q)|^2.
// kind 1: per mode q a block of n_r^2 values s(Re c) for k1 <= k2, then
// s(Im c) for k1 < k2 (row-major pairs), c = a(k1; q) conj a(k2; q),
// s(x) = sign(x) sqrt|x|.
__global__ void features_kernel(const float2* __restrict__ c, int nA, int Qa, int M, int kind, int n_r, int n_q,
                                float* __restrict__ F) {
  const size_t D = kind == 1 ? static_cast<size_t>(n_r) * n_r * n_q : static_cast<size_t>(n_r) * n_q;
  const size_t total = static_cast<size_t>(nA) * D;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t a = t / D;
    const int f = static_cast<int>(t - a * D);
    if (kind == 0) {
      const int m = f / n_q;
      const int q = f - m * n_q;
      const float2 v = c[(a * Qa + q) * M + m];
      F[t] = v.x * v.x + v.y * v.y;
      continue;
    }
    if (kind == 2) {
      // sqrt|P(k_m; 2 j)|, P(k; s) = sum_q a(k; q) conj a(k; q - s) (indices
      // mod Qa): the ring power's angular Fourier coefficient, unchanged by
      // shifts (a phase on Ahat) and, in modulus, by rotations
      const int m = f / n_q;
      const int s2 = 2 * (f - m * n_q);
      const float2* col = c + a * Qa * M + m;
      float re = 0.f, im = 0.f;
      for (int q = 0; q < Qa; ++q) {
        int q2 = q - s2;
        q2 += q2 < 0 ? Qa : 0;
        const float2 u = col[static_cast<size_t>(q) * M], w = col[static_cast<size_t>(q2) * M];
        re += u.x * w.x + u.y * w.y;
        im += u.y * w.x - u.x * w.y;
      }
      F[t] = sqrtf(hypotf(re, im));
      continue;
    }
    const int blk = n_r * n_r;
    const int q = f / blk;
    int u = f - q * blk;
    const int P = n_r * (n_r + 1) / 2;
    const bool imag = u >= P;
    if (imag) u -= P;
    int k1 = 0;
    int len = imag ? n_r - 1 : n_r;  // pairs in row k1
    while (u >= len) {
      u -= len;
      ++k1;
      --len;
    }
    const int k2 = k1 + u + (imag ? 1 : 0);
    const float2 v1 = c[(a * Qa + q) * M + k1];
    const float2 v2 = c[(a * Qa + q) * M + k2];
    const float x = imag ? (v1.y * v2.x - v1.x * v2.y) : (v1.x * v2.x + v1.y * v2.y);
    F[t] = copysignf(sqrtf(fabsf(x)), x);
  }
}

// (value, index) order used by the proposal: larger value first, then the
// lower index; NaN logits rank below every number
__device__ __forceinline__ bool ranks_before(float v, int i, float w, int j) {
  return v > w || (v == w && i < j);
}

__device__ __forceinline__ float clean(float x) { return (x == x) ? x : -__builtin_inff(); }

__global__ void __launch_bounds__(kThreads) topk_kernel(const float* __restrict__ logits, int D, int n_t, int n_s,
                                                        int k, int32_t* __restrict__ top, float* __restrict__ mass,
                                                        int32_t* __restrict__ sbin) {
  __shared__ float rv[4];
  __shared__ int ri[4];
  __shared__ float sel_v[64];
  __shared__ int sel_i[64];
  const int row = blockIdx.x;
  const float* z = logits + static_cast<size_t>(row) * D;
  float pv = __builtin_inff();
  int pi = -1;
  for (int r = 0; r < k; ++r) {
    // the first element, in (value desc, index asc) order, after (pv, pi)
    float bv = -__builtin_inff();
    int bi = 0x7fffffff;
    for (int j = threadIdx.x; j < n_t; j += kThreads) {
      const float v = clean(z[j]);
      if (ranks_before(pv, pi, v, j) && ranks_before(v, j, bv, bi)) {
        bv = v;
        bi = j;
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float ov = __shfl_xor(bv, o);
      const int oi = __shfl_xor(bi, o);
      if (ranks_before(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      rv[threadIdx.x >> 6] = bv;
      ri[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    bv = rv[0];
    bi = ri[0];
    for (int w = 1; w < 4; ++w)
      if (ranks_before(rv[w], ri[w], bv, bi)) {
        bv = rv[w];
        bi = ri[w];
      }
    if (threadIdx.x == 0) {
      sel_v[r] = bv;
      sel_i[r] = bi;
    }
    pv = bv;
    pi = bi;
  }
  __syncthreads();
  const float mx = sel_v[0];
  float se = 0.f;
  for (int j = threadIdx.x; j < n_t; j += kThreads) se += __expf(clean(z[j]) - mx);
  __shared__ float red[4];
  se = block_sum(se, red);
  if (threadIdx.x == 0) {
    float ms = 0.f;
    for (int r = 0; r < k; ++r) {
      top[static_cast<size_t>(row) * k + r] = sel_i[r];
      ms += __expf(sel_v[r] - mx);
    }
    mass[row] = ms / se;
    int sb = 0;
    float sv = -__builtin_inff();
    for (int j = 0; j < n_s; ++j) {
      const float v = clean(z[n_t + j]);
      if (v > sv) {
        sv = v;
        sb = j;
      }
    }
    sbin[row] = sb;
  }
}

struct Pose {
  float value;
  int32_t shift;
  int32_t rot;
};

__global__ void best_template_kernel(const Pose* __restrict__ poses, const int32_t* __restrict__ lists, int nA, int K,
                                     int32_t* __restrict__ best_t, Pose* __restrict__ best_pose) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nA) return;
  float bv = -__builtin_inff();
  int bt = -1, bj = -1;
  for (int j = 0; j < K; ++j) {
    const Pose p = poses[static_cast<size_t>(a) * K + j];
    const int t = lists ? lists[static_cast<size_t>(a) * K + j] : j;
    if (!(p.value == p.value)) continue;
    if (p.value > bv || (p.value == bv && t < bt)) {
      bv = p.value;
      bt = t;
      bj = j;
    }
  }
  best_t[a] = bt;
  Pose o;
  if (bj >= 0) {
    o = poses[static_cast<size_t>(a) * K + bj];
  } else {
    o.value = __builtin_nanf("");
    o.shift = -1;
    o.rot = -1;
  }
  best_pose[a] = o;
}

// one workgroup: rows with mass < tau in increasing order (block scan)
__global__ void __launch_bounds__(kThreads) select_below_kernel(const float* __restrict__ mass, int nA, float tau,
                                                                int32_t* __restrict__ list,
                                                                int32_t* __restrict__ count,
                                                                int32_t* __restrict__ flag) {
  __shared__ int wsum[4];
  __shared__ int base_s;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nA; c0 += kThreads) {
    const int i = c0 + threadIdx.x;
    const int f = (i < nA && !(mass[i] >= tau)) ? 1 : 0;
    if (i < nA && flag) flag[i] = f;
    // inclusive scan within the wave
    int x = f;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[threadIdx.x >> 6] = x;
    __syncthreads();
    int before = base_s;
    for (int w = 0; w < static_cast<int>(threadIdx.x >> 6); ++w) before += wsum[w];
    if (f) list[before + x - 1] = i;
    __syncthreads();
    if (threadIdx.x == 0) base_s += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = base_s;
}

__global__ void gather_rows_kernel(const uint2* __restrict__ src, const int32_t* __restrict__ list, int count,
                                   size_t words, uint2* __restrict__ dst) {
  const size_t total = static_cast<size_t>(count) * words;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t r = t / words;
    const size_t w = t - r * words;
    dst[t] = src[static_cast<size_t>(list[r]) * words + w];
  }
}

__global__ void gather_words_kernel(const uint32_t* __restrict__ src, const int32_t* __restrict__ list, int count,
                                    size_t words, uint32_t* __restrict__ dst) {
  const size_t total = static_cast<size_t>(count) * words;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t r = t / words;
    dst[t] = src[static_cast<size_t>(list[r]) * words + (t - r * words)];
  }
}

// dst[list[r]][j] = src[r][j] with the shift index mapped through map
// (window index -> plan index); poses without a result (shift < 0) kept
__global__ void scatter_poses_kernel(const Pose* __restrict__ src, const int32_t* __restrict__ list, int count, int K,
                                     const int32_t* __restrict__ map, Pose* __restrict__ dst) {
  const size_t total = static_cast<size_t>(count) * K;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const size_t r = t / K;
    Pose p = src[t];
    if (map && p.shift >= 0) p.shift = map[p.shift];
    dst[static_cast<size_t>(list[r]) * K + (t - r * K)] = p;
  }
}

__global__ void scatter_results_kernel(const int32_t* __restrict__ bt, const Pose* __restrict__ bp,
                                       const int32_t* __restrict__ list, int count, int32_t* __restrict__ dt,
                                       Pose* __restrict__ dp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int a = list[i];
  dt[a] = bt[i];
  dp[a] = bp[i];
}

unsigned grid_for(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return static_cast<unsigned>(b);
}

}  // namespace

GemmPlan gemm_plan(int M, int N, int K) {
  GemmPlan p;
  const long long t128 = static_cast<long long>((M + 127) / 128) * ((N + 127) / 128);
  p.big = t128 >= 256;
  const long long tiles = p.big ? t128 : static_cast<long long>((M + 63) / 64) * ((N + 63) / 64);
  // split K until about 256 workgroups, keeping >= 8 chunks of 32 per part
  p.kparts = 1;
  while (tiles * p.kparts * 2 <= 512 && K / (p.kparts * 2) >= 256 && p.kparts < 16) p.kparts *= 2;
  return p;
}

size_t gemm_part_floats(int M, int N, int K) {
  const GemmPlan p = gemm_plan(M, N, K);
  return p.kparts > 1 ? static_cast<size_t>(p.kparts) * M * N : 0;
}

hipError_t launch_gemm(const GemmArgs& g, int bf16, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (!((g.sak == 1) || (g.sai == 1)) || !((g.sbk == 1) || (g.sbj == 1))) return hipErrorInvalidValue;
  if (!bf16) {
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
    if (grid.y > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(kThreads), 0, s, g);
    return hipGetLastError();
  }
  GemmPlan pl = gemm_plan(g.M, g.N, g.K);
  if (pl.kparts > 1 && (!g.part || g.part_floats < static_cast<size_t>(pl.kparts) * g.M * g.N)) pl.kparts = 1;
  const int T = pl.big ? 128 : 64;
  dim3 grid((g.N + T - 1) / T, (g.M + T - 1) / T, pl.kparts);
  if (grid.y > 65535) return hipErrorInvalidValue;
  if (pl.big)
    hipLaunchKernelGGL((gemm_bf16_tiled<2, 2, 32>), grid, dim3(kThreads), 0, s, g, pl.kparts, g.part);
  else
    hipLaunchKernelGGL((gemm_bf16_tiled<1, 1, 64>), grid, dim3(kThreads), 0, s, g, pl.kparts, g.part);
  if (pl.kparts > 1)
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3(grid_for(static_cast<size_t>(g.M) * g.N)), dim3(kThreads), 0, s, g,
                       pl.kparts, static_cast<const float*>(g.part));
  return hipGetLastError();
}

hipError_t launch_standardise(const float* x, const int32_t* idx, int B, int D, const float* mu,
                              const float* inv_sigma, void* X, int bf16, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  const unsigned grid = grid_for(static_cast<size_t>(B) * D);
  if (bf16)
    hipLaunchKernelGGL(standardise_kernel<__bf16>, dim3(grid), dim3(kThreads), 0, s, x, idx, B, D, mu, inv_sigma,
                       static_cast<__bf16*>(X));
  else
    hipLaunchKernelGGL(standardise_kernel<float>, dim3(grid), dim3(kThreads), 0, s, x, idx, B, D, mu, inv_sigma,
                       static_cast<float*>(X));
  return hipGetLastError();
}

hipError_t launch_softmax_ce(const float* logits, int B, int D, int ldz, int n_t, int n_s, const int32_t* lab_t,
                             const int32_t* lab_s, const int32_t* idx, float* dZ, void* dZb, int bf16,
                             float* row_loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (bf16)
    hipLaunchKernelGGL(softmax_ce_kernel<__bf16>, dim3(B), dim3(kThreads), 0, s, logits, B, D, ldz, n_t, n_s, lab_t,
                       lab_s, idx, dZ, static_cast<__bf16*>(dZb), row_loss);
  else
    hipLaunchKernelGGL(softmax_ce_kernel<float>, dim3(B), dim3(kThreads), 0, s, logits, B, D, ldz, n_t, n_s, lab_t, lab_s,
                       idx, dZ, static_cast<float*>(dZb), row_loss);
  return hipGetLastError();
}

hipError_t launch_mean(const float* row_loss, int B, float* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(kThreads), 0, s, row_loss, B, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, int B, int N, int ld, float* db, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 63) / 64), dim3(kThreads), 0, s, dZ, B, N, ld, db);
  return hipGetLastError();
}

hipError_t launch_adamw(float* w, const float* g, float* m, float* v, size_t n, float lr, float beta1, float beta2,
                        float eps, float wd, float bc1, float bc2, void* wc, int bf16, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (bf16)
    hipLaunchKernelGGL(adamw_kernel<__bf16>, dim3(grid_for(n)), dim3(kThreads), 0, s, w, g, m, v, n, lr, beta1,
                       beta2, eps, wd, bc1, bc2, static_cast<__bf16*>(wc));
  else
    hipLaunchKernelGGL(adamw_kernel<float>, dim3(grid_for(n)), dim3(kThreads), 0, s, w, g, m, v, n, lr, beta1,
                       beta2, eps, wd, bc1, bc2, static_cast<float*>(wc));
  return hipGetLastError();
}

hipError_t launch_convert(const float* w, size_t n, void* wc, int bf16, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (bf16)
    hipLaunchKernelGGL(convert_kernel<__bf16>, dim3(grid_for(n)), dim3(kThreads), 0, s, w, n,
                       static_cast<__bf16*>(wc));
  else
    hipLaunchKernelGGL(convert_kernel<float>, dim3(grid_for(n)), dim3(kThreads), 0, s, w, n, static_cast<float*>(wc));
  return hipGetLastError();
}

hipError_t launch_features(const float2* coeffs, int nA, int Qa, int M, int kind, int n_r, int n_q, float* F,
                           hipStream_t s) {
  if (nA <= 0) return hipSuccess;
  const size_t D = kind == 1 ? static_cast<size_t>(n_r) * n_r * n_q : static_cast<size_t>(n_r) * n_q;
  hipLaunchKernelGGL(features_kernel, dim3(grid_for(static_cast<size_t>(nA) * D)), dim3(kThreads), 0, s, coeffs, nA,
                     Qa, M, kind, n_r, n_q, F);
  return hipGetLastError();
}

hipError_t launch_topk(const float* logits, int rows, int D, int n_t, int n_s, int k, int32_t* top, float* mass,
                       int32_t* sbin, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (k < 1 || k > 64 || k > n_t) return hipErrorInvalidValue;
  hipLaunchKernelGGL(topk_kernel, dim3(rows), dim3(kThreads), 0, s, logits, D, n_t, n_s, k, top, mass, sbin);
  return hipGetLastError();
}

hipError_t launch_best_template(const void* poses, const int32_t* lists, int nA, int K, int32_t* best_t,
                                void* best_pose, hipStream_t s) {
  if (nA <= 0) return hipSuccess;
  hipLaunchKernelGGL(best_template_kernel, dim3((nA + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     static_cast<const Pose*>(poses), lists, nA, K, best_t, static_cast<Pose*>(best_pose));
  return hipGetLastError();
}

hipError_t launch_select_below(const float* mass, int nA, float tau, int32_t* list, int32_t* count, int32_t* flag,
                               hipStream_t s) {
  hipLaunchKernelGGL(select_below_kernel, dim3(1), dim3(kThreads), 0, s, mass, nA, tau, list, count, flag);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const void* src, const int32_t* list, int count, size_t row_bytes, void* dst,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (row_bytes % 8) return hipErrorInvalidValue;
  const size_t words = row_bytes / 8;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(static_cast<size_t>(count) * words)), dim3(kThreads), 0, s,
                     static_cast<const uint2*>(src), list, count, words, static_cast<uint2*>(dst));
  return hipGetLastError();
}

hipError_t launch_gather_words(const void* src, const int32_t* list, int count, size_t row_words, void* dst,
                               hipStream_t s) {
  if (count <= 0 || row_words == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_words_kernel, dim3(grid_for(static_cast<size_t>(count) * row_words)), dim3(kThreads), 0, s,
                     static_cast<const uint32_t*>(src), list, count, row_words, static_cast<uint32_t*>(dst));
  return hipGetLastError();
}

hipError_t launch_scatter_poses(const void* src, const int32_t* list, int count, int K, const int32_t* map, void* dst,
                                hipStream_t s) {
  if (count <= 0 || K <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_poses_kernel, dim3(grid_for(static_cast<size_t>(count) * K)), dim3(kThreads), 0, s,
                     static_cast<const Pose*>(src), list, count, K, map, static_cast<Pose*>(dst));
  return hipGetLastError();
}

hipError_t launch_scatter_results(const int32_t* bt, const void* bp, const int32_t* list, int count, int32_t* dst_t,
                                  void* dst_p, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_results_kernel, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, s, bt,
                     static_cast<const Pose*>(bp), list, count, dst_t, static_cast<Pose*>(dst_p));
  return hipGetLastError();
}
