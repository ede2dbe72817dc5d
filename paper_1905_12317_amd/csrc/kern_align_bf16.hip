// Step 3 of the FTK in split form on gfx950 MFMA: split bf16 (FTK_BF16X3) and
// split fp16 (FTK_FP16X3).
//
// Every operand x of the two contractions is written as x = hi + lo with
// hi = T(x) and lo = T(x - hi) (round to nearest even, T = bf16 or fp16),
// and each product uses three MFMAs with FP32 accumulation:
//     A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi.
// With bf16 (8 significant bits) this keeps about 16 bits per product; with
// fp16 (11 bits) about 22, but fp16 has a narrow exponent range, so the fp16
// form runs on operands scaled by powers of two (per call for the data, per
// SVD term for the tables, as the FP16 form: Zhat / (s_a s_b sg_zeta) is
// bounded by 2M, the scaled shift panel by 1) and multiplies X back when it
// is stored.  The quadrature weights and the operator SVD stay FP64 on the
// host; only their FP32 products enter.
//
// Data flow is that of the FP32 form (kern_align.hip): Step 1
// (kern_step1.hip) writes Zhat, already split into hi + lo and in chunks of
// 32 k' laid out as Step 3 stages them, Step 3 copies the chunks into LDS
// and ends with the same rotation FFT and argmax.
// MFMA: v_mfma_f32_32x32x16_bf16 / _f16; lane l holds rows/cols l % 32 and
// the 8 consecutive k = 8 (l / 32) .. +7 of each 16-wide K step.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"
#include "step3_epilogue.h"

using namespace ftkdev;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// element type of a split form: its 8-wide MFMA operand and the 32x32x16 MFMA
template <class T>
struct Split;
template <>
struct Split<__bf16> {
  typedef bf16x8 v8;
  static __device__ __forceinline__ f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Split<_Float16> {
  typedef f16x8 v8;
  static __device__ __forceinline__ f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <class T, class V>
__device__ __forceinline__ f32x16 mfma3(V ahi, V alo, V bhi, V blo, f32x16 c) {
  c = Split<T>::mma(ahi, bhi, c);
  c = Split<T>::mma(ahi, blo, c);
  c = Split<T>::mma(alo, bhi, c);
  return c;
}

// ---------------------------------------------------------------- Step 3

// The K loop for one pair and one shift block: Zhat chunks staged through
// LDS (two buffers of QH rows at `region`), three bf16 MFMAs per term.  The
// first chunk is in buffer 0 and visible to the block on entry; ends after the
// last chunk's MFMAs (no barrier).  With next_pair >= 0 (PREF only), the last
// chunk's prefetch fetches the first chunk of next_pair instead and stores it
// into buffer 0 after its MFMAs: visible after the caller's next barrier.
// PREF: the block has enough threads to prefetch a whole chunk in MAXF4
// float4 per thread (double buffering through registers); otherwise each
// chunk is fetched after the MFMAs of the previous one.
template <class T, int CTQ, bool PREF>
__device__ __forceinline__ void split_kloop(const Step3Args& p, float* region, int pair, int d0, bool active,
                                           f32x16 (&acc)[CTQ], int next_pair) {
  constexpr int QH = 32 * CTQ;
  constexpr int KC = 32;     // k' per staged chunk (2 MFMA K steps)
  constexpr int ROWW = 36;   // LDS words per q row: 16 hi, 16 lo, 4 pad
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nk = 2 * p.H_pad;
  const int nks = nk / 16;
  // this pair's chunks of Zhat, already split: chunk c is QH rows of 128
  // bytes (16 words hi, 16 words lo), 8 float4 per row, contiguous
  const float4* zsp = static_cast<const float4*>(p.zs) + static_cast<size_t>(pair) * QH * (nk / 4);
  const float4* znext =
      static_cast<const float4*>(p.zs) + static_cast<size_t>(next_pair < 0 ? pair : next_pair) * QH * (nk / 4);
  const int buf_words = QH * ROWW;
  const int nthr = blockDim.x;
  typedef typename Split<T>::v8 V;
  constexpr int MAXF4 = 2;
  const int nf4 = QH * (KC / 4);
  auto fetch = [&](int kc, int t) { return load_stream(zsp + static_cast<size_t>(kc / KC) * nf4 + t); };
  // unit t = 8 q + u of a chunk goes to words 4 u .. 4 u + 3 of LDS row q
  auto put = [&](int buf, int t, float4 v) {
    *reinterpret_cast<float4*>(region + buf * buf_words + (t >> 3) * ROWW + (t & 7) * 4) = v;
  };
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) acc[ct] = zero16();
  // shift panel in MFMA lane order: [row tile][K step][lane][8] for hi and lo
  const size_t tile = static_cast<size_t>(min(d0, p.N_pad - 16) / 16) * nks;
  const V* yhi = reinterpret_cast<const V*>(p.yt_hi) + tile * 64 + lane;
  const V* ylo = reinterpret_cast<const V*>(p.yt_lo) + tile * 64 + lane;
  // shift-panel operands of the chunk at kc (past the end: the last chunk
  // again, so the loads need no condition)
  auto load_y = [&](int kc, V (&yh)[KC / 16], V (&yl)[KC / 16]) {
    const int kk = min(kc, nk - KC);
#pragma unroll
    for (int s = 0; s < KC / 16; ++s) {
      yh[s] = yhi[(kk / 16 + s) * 64];
      yl[s] = ylo[(kk / 16 + s) * 64];
    }
  };
  // One chunk: the MFMAs on LDS buffer (kc / KC) % 2 with the panel operands
  // loaded one chunk earlier, then the next chunk is stored into the other
  // buffer.  Loads retire in order, so each chunk issues its loads in the
  // order they are consumed (next chunk's Zhat, then the panel operands of the
  // chunk after it) and the waits before the MFMAs cover no load issued in
  // this chunk.  Every wave issues the same unconditional loads (clamped to
  // valid addresses), so the wait counts are exact.
  auto chunk = [&](int kc, const V (&ah)[KC / 16], const V (&al)[KC / 16], V (&nh)[KC / 16],
                   V (&nl)[KC / 16]) {
    const int cur = (kc / KC) & 1;
    const bool more = kc + KC < nk;
    float4 nreg[MAXF4];
    if (PREF) {
      if (more || next_pair < 0) {
        const int kn = more ? kc + KC : kc;  // the last chunk re-reads itself
#pragma unroll
        for (int k = 0; k < MAXF4; ++k) nreg[k] = fetch(kn, min(tid + k * nthr, nf4 - 1));
      } else {
#pragma unroll
        for (int k = 0; k < MAXF4; ++k) nreg[k] = load_stream(znext + min(tid + k * nthr, nf4 - 1));
      }
    }
    load_y(kc + KC, nh, nl);
    __builtin_amdgcn_sched_barrier(0);
    if (active) {
      const float* Zb = region + cur * buf_words + c32 * ROWW + 4 * r;
#pragma unroll
      for (int s = 0; s < KC / 16; ++s) {
#pragma unroll
        for (int ct = 0; ct < CTQ; ++ct) {
          const float* row = Zb + ct * 32 * ROWW + 8 * s;
          const V bhi = *reinterpret_cast<const V*>(row);
          const V blo = *reinterpret_cast<const V*>(row + 16);
          acc[ct] = mfma3<T>(ah[s], al[s], bhi, blo, acc[ct]);
        }
      }
    }
    if (more) {
      if (PREF) {
#pragma unroll
        for (int k = 0; k < MAXF4; ++k) {
          const int t = tid + k * nthr;
          if (t < nf4) put(cur ^ 1, t, nreg[k]);
        }
      } else {
        for (int t = tid; t < nf4; t += nthr) put(cur ^ 1, t, fetch(kc + KC, t));
      }
      __syncthreads();
    } else if (PREF && next_pair >= 0) {
      // the last chunk is in buffer 1 (an even number of chunks): buffer 0 is free
#pragma unroll
      for (int k = 0; k < MAXF4; ++k) {
        const int t = tid + k * nthr;
        if (t < nf4) put(0, t, nreg[k]);
      }
    }
  };
  V yah[KC / 16], yal[KC / 16], ybh[KC / 16], ybl[KC / 16];
  load_y(0, yah, yal);
  // nk / KC is even (H_pad is a multiple of 64)
  for (int kc = 0; kc < nk; kc += 2 * KC) {
    chunk(kc, yah, yal, ybh, ybl);
    chunk(kc + KC, ybh, ybl, yah, yal);
  }
}

// The first Zhat chunk of `pair` into LDS buffer 0.
template <int CTQ>
__device__ __forceinline__ void split_first_chunk(const Step3Args& p, float* region, int pair) {
  constexpr int QH = 32 * CTQ;
  const int nf4 = QH * 8;
  const float4* zsp = static_cast<const float4*>(p.zs) + static_cast<size_t>(pair) * QH * (2 * p.H_pad / 4);
  for (int t = threadIdx.x; t < nf4; t += blockDim.x)
    *reinterpret_cast<float4*>(region + (t >> 3) * 36 + (t & 7) * 4) = load_stream(zsp + t);
}

template <class T, int CTQ, int MAXT, bool PREF, int EPI>
__global__ void __launch_bounds__(MAXT) step3_split(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int pair, yb;
  step3_block(blockIdx.x, p.nblk, p.pairs, pair, yb);
  const int d0 = (yb * p.nwaves + wave) * 16;
  float2* twl = reinterpret_cast<float2*>(smem);
  float* region = smem + 4 * QH;
  for (int i = tid; i < 2 * QH; i += blockDim.x) twl[i] = p.tw_qa[i];
  const bool active = d0 < p.N;
  split_first_chunk<CTQ>(p, region, pair);
  __syncthreads();
  f32x16 acc[CTQ];
  split_kloop<T, CTQ, PREF>(p, region, pair, d0, active, acc, -1);
  __syncthreads();
  if (!active) return;
  float2* rows = reinterpret_cast<float2*>(region) + wave * (epilogue_lds_bytes_per_wave() / sizeof(float2));
  step3_epilogue_reg<CTQ, EPI>(p, acc, pair, d0, rows, twl, lane);
}

// Persistent form (one workgroup per CU, looping over its shift blocks) where
// the FFT rows fit LDS beside the Zhat buffers: the next pair's first chunk is
// stored during the last chunk of the current one, and a wave goes on to the
// next pair's K loop as soon as its own FFT epilogue is done.
template <class T, int CTQ, bool PREF>
__global__ void __launch_bounds__(1024) step3_split_p(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  float2* twl = reinterpret_cast<float2*>(smem);
  float* region = smem + 4 * QH;  // Zhat buffers
  float2* rows = reinterpret_cast<float2*>(region + 2 * QH * 36) +
                 wave * (epilogue_lds_bytes_per_wave() / sizeof(float2));
  for (int i = tid; i < 2 * QH; i += blockDim.x) twl[i] = p.tw_qa[i];
  const int total = p.pairs * p.nblk;
  int b = blockIdx.x;
  if (b >= total) return;
  int pair, yb;
  step3_block(b, p.nblk, p.pairs, pair, yb);
  split_first_chunk<CTQ>(p, region, pair);
  __syncthreads();
  for (;;) {
    const int d0 = (yb * p.nwaves + wave) * 16;
    const bool active = d0 < p.N;
    const int bn = b + gridDim.x;
    int pn = 0, ybn = 0;
    if (bn < total) step3_block(bn, p.nblk, p.pairs, pn, ybn);
    f32x16 acc[CTQ];
    split_kloop<T, CTQ, PREF>(p, region, pair, d0, active, acc, (PREF && bn < total) ? pn : -1);
    __syncthreads();  // every wave is past the Zhat buffers; the next first chunk is visible
    if (active) step3_epilogue_reg<CTQ>(p, acc, pair, d0, rows, twl, lane);
    if (bn >= total) break;
    if (!PREF) {
      __syncthreads();
      split_first_chunk<CTQ>(p, region, pn);
      __syncthreads();
    }
    b = bn;
    pair = pn;
    yb = ybn;
  }
}

}  // namespace

size_t step3_bf16_lds_bytes(int Qa, int nwaves) {
  const size_t QH = Qa / 2;
  const size_t k = sizeof(float) * 2 * QH * 36;
  const size_t e = static_cast<size_t>(nwaves) * epilogue_lds_bytes_per_wave();
  return sizeof(float2) * Qa + (k > e ? k : e);
}

// LDS of the persistent form: twiddles, Zhat buffers and FFT rows side by side
static size_t bf16_persistent_lds(int Qa, int nwaves) {
  const size_t QH = Qa / 2;
  return sizeof(float2) * Qa + sizeof(float) * 2 * QH * 36 + static_cast<size_t>(nwaves) * epilogue_lds_bytes_per_wave();
}

static int bf16_device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] <= 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <class T, int CTQ, int MAXT>
static hipError_t launch_step3_split_t(const Step3Args& a0, hipStream_t s) {
  Step3Args a = a0;
  const int per_blk = 16 * a.nwaves;
  a.nblk = (a.N + per_blk - 1) / per_blk;
  const size_t nwg = static_cast<size_t>(a.pairs) * a.nblk;
  if (nwg * 64 * a.nwaves > 0xffffffffull) return hipErrorInvalidConfiguration;
  const int nf4 = 32 * CTQ * 8, nthr = 64 * a.nwaves;
  const bool pref = (nf4 + nthr - 1) / nthr <= 2;
  if constexpr (MAXT == 1024) {
    const size_t plds = bf16_persistent_lds(a.Qa, a.nwaves);
    if (pref && plds <= 160 * 1024 && !a.xhat) {
      auto kern = step3_split_p<T, CTQ, true>;
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(plds));
      if (e != hipSuccess) return e;
      const unsigned grid = static_cast<unsigned>(std::min<size_t>(nwg, static_cast<size_t>(bf16_device_cus())));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(nthr), plds, s, a);
      return hipGetLastError();
    }
  }
  const dim3 grid(static_cast<unsigned>(nwg));
  size_t lds = step3_bf16_lds_bytes(a.Qa, a.nwaves);
  // Xhat out (rotation upsampling): the plain form with the storing epilogue
  auto kern = a.xhat ? (pref ? step3_split<T, CTQ, MAXT, true, kEpiStore> : step3_split<T, CTQ, MAXT, false, kEpiStore>)
                     : (pref ? step3_split<T, CTQ, MAXT, true, kEpiRotate>
                             : step3_split<T, CTQ, MAXT, false, kEpiRotate>);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(64 * a.nwaves), lds, s, a);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_step3_split_q(const Step3Args& a, hipStream_t s) {
  switch (a.Qa / 64) {
    case 1: return launch_step3_split_t<T, 1, 1024>(a, s);
    case 2: return launch_step3_split_t<T, 2, 1024>(a, s);
    case 3: return launch_step3_split_t<T, 3, 1024>(a, s);
    case 4: return launch_step3_split_t<T, 4, 1024>(a, s);
    case 6: return launch_step3_split_t<T, 6, 512>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step3_bf16(const Step3Args& a, bool fp16, hipStream_t s) {
  if (a.pairs <= 0) return hipSuccess;
  if (fp16 && !a.xscale) return hipErrorInvalidValue;
  return fp16 ? launch_step3_split_q<_Float16>(a, s) : launch_step3_split_q<__bf16>(a, s);
}
