// Step 3 of the FTK in FP16 form on gfx950 MFMA, and the data scales of that
// form.
//
// Both contractions take one FP16 product per term with FP32 accumulation.
// FP16 keeps 11 significant bits, so every operand is scaled by a power of
// two to sit near the top of the FP16 range:
//   * per call, s_a and s_b: the powers of two at or above max |a| over the
//     images and max |b| over the templates (computed here on the device);
//   * per zeta, sg_zeta: the power of two at or above max_m 2 pi w_m G_zeta
//     (planned on the host; the 2 pi w G table of an FP16 plan is stored
//     divided by it, and the shift panel multiplied by it);
//   * s_y: the power of two at or above the largest entry of the scaled
//     shift panel (host).
// Step 1 then forms Zhat / (s_a s_b sg_zeta), bounded by M in magnitude, and
// Step 3 X / (s_a s_b s_y); the stored X values and the pose values are
// multiplied back by s_a s_b s_y, and the argmax does not depend on it.
//
// Staging: Step 1 (kern_step1.hip) writes Zhat rounded to fp16 in chunks of
// 64 k' whose rows have the layout of the split form's (128 bytes per q), so
// the K loop stages them the same way, 64 k' (four MFMA K steps) per chunk.
#include <algorithm>

#include "device_common.h"
#include "kernels.h"
#include "step3_epilogue.h"

using namespace ftkdev;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// PREF: the block has enough threads to hold a whole chunk in MAXF4 float4
// per thread, and the next chunk is prefetched through registers while the
// current one is multiplied; otherwise each chunk is fetched after the MFMAs
// of the previous one.
template <int CTQ, int MAXT, bool PREF>
__global__ void __launch_bounds__(MAXT) step3_fp16(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  constexpr int KC = 64;     // k' per staged chunk (4 MFMA K steps)
  constexpr int KS = KC / 16;
  constexpr int ROWW = 36;   // LDS words per q row: 32 data, 4 pad
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int pair, yb;
  step3_block(blockIdx.x, p.nblk, p.pairs, pair, yb);
  const int d0 = (yb * p.nwaves + wave) * 16;
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nk = 2 * p.H_pad;
  const int nks = nk / 16;
  // this pair's chunks of Zhat: chunk c is QH rows of 128 bytes, 8 float4 per
  // row, contiguous
  const float4* zsp = static_cast<const float4*>(p.zs) + static_cast<size_t>(pair) * QH * (nk / 8);
  float2* twl = reinterpret_cast<float2*>(smem);
  float* region = smem + 4 * QH;
  const int buf_words = QH * ROWW;
  const int nthr = blockDim.x;
  for (int i = tid; i < 2 * QH; i += nthr) twl[i] = p.tw_qa[i];
  constexpr int MAXF4 = 2;
  const int nf4 = QH * 8;
  auto fetch = [&](int kc, int t) { return load_stream(zsp + static_cast<size_t>(kc / KC) * nf4 + t); };
  // unit t = 8 q + u of a chunk goes to words 4 u .. 4 u + 3 of LDS row q
  auto put = [&](int buf, int t, float4 v) {
    *reinterpret_cast<float4*>(region + buf * buf_words + (t >> 3) * ROWW + (t & 7) * 4) = v;
  };
  for (int t = tid; t < nf4; t += nthr) put(0, t, fetch(0, t));
  __syncthreads();
  f32x16 acc[CTQ];
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) acc[ct] = zero16();
  const bool active = d0 < p.N;
  // shift panel in MFMA lane order: [row tile][K step][lane][8] fp16
  const size_t tile = static_cast<size_t>(min(d0, p.N_pad - 16) / 16) * nks;
  const f16x8* yp = reinterpret_cast<const f16x8*>(p.yt_hi) + tile * 64 + lane;
  // shift-panel operands of the chunk at kc (past the end: the last chunk
  // again, so the loads need no condition)
  auto load_y = [&](int kc, f16x8 (&y)[KS]) {
    const int kk = min(kc, nk - KC);
#pragma unroll
    for (int s = 0; s < KS; ++s) y[s] = yp[(kk / 16 + s) * 64];
  };
  // One chunk: the MFMAs on LDS buffer (kc / KC) % 2 with the panel operands
  // loaded one chunk earlier, then the next chunk is stored into the other
  // buffer.  The loads are issued in the order they are consumed (next
  // chunk's Zhat, then the panel operands of the chunk after it), so the
  // waits before the MFMAs cover no load issued in this chunk.
  auto chunk = [&](int kc, const f16x8 (&ay)[KS], f16x8 (&ny)[KS]) {
    const int cur = (kc / KC) & 1;
    const bool more = kc + KC < nk;
    float4 nreg[MAXF4];
    if (PREF) {
      const int kn = more ? kc + KC : kc;  // the last chunk re-reads itself
#pragma unroll
      for (int k = 0; k < MAXF4; ++k) nreg[k] = fetch(kn, min(tid + k * nthr, nf4 - 1));
    }
    load_y(kc + KC, ny);
    __builtin_amdgcn_sched_barrier(0);
    if (active) {
      const float* Zb = region + cur * buf_words + c32 * ROWW + 4 * r;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int ct = 0; ct < CTQ; ++ct) {
          const f16x8 b = *reinterpret_cast<const f16x8*>(Zb + ct * 32 * ROWW + 8 * s);
          acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ay[s], b, acc[ct], 0, 0, 0);
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
    }
  };
  f16x8 y0[KS], y1[KS];
  load_y(0, y0);
  // nk / KC is even (H_pad is a multiple of 64)
  for (int kc = 0; kc < nk; kc += 2 * KC) {
    chunk(kc, y0, y1);
    chunk(kc + KC, y1, y0);
  }
  __syncthreads();
  if (!active) return;
  float2* T = reinterpret_cast<float2*>(region) + wave * (epilogue_lds_bytes_per_wave() / sizeof(float2));
  step3_epilogue_reg<CTQ>(p, acc, pair, d0, T, twl, lane);
}

// ---- data scales ----------------------------------------------------------

__global__ void scales_init(unsigned* s) {
  if (threadIdx.x < 2) s[threadIdx.x] = 0u;
}

// max |v| over count floats into *out (non-negative floats order as their
// bit patterns)
__global__ void absmax_kernel(const float* __restrict__ v, size_t count, unsigned* out) {
  float m = 0.f;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    m = fmaxf(m, fabsf(v[i]));
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__device__ __forceinline__ float pow2_at_or_above(float m) {
  if (!(m > 0.f) || !(m < 3.0e38f)) return 1.f;  // zero, NaN or not finite: no scaling
  int e;
  const float f = frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, f == 0.5f ? e - 1 : e);
}

__global__ void scales_finalize(float* s, float s_y) {
  if (threadIdx.x != 0) return;
  const float sa = pow2_at_or_above(__uint_as_float(reinterpret_cast<unsigned*>(s)[0]));
  const float sb = pow2_at_or_above(__uint_as_float(reinterpret_cast<unsigned*>(s)[1]));
  s[2] = 1.f / sa;
  s[3] = 1.f / sb;
  s[4] = sa * sb * s_y;
}

}  // namespace

size_t step3_fp16_lds_bytes(int Qa, int nwaves) {
  const size_t QH = Qa / 2;
  const size_t k = sizeof(float) * 2 * QH * 36;
  const size_t e = static_cast<size_t>(nwaves) * epilogue_lds_bytes_per_wave();
  return sizeof(float2) * Qa + (k > e ? k : e);
}

template <int CTQ, int MAXT>
static hipError_t launch_step3_fp16_t(const Step3Args& a0, hipStream_t s) {
  Step3Args a = a0;
  const int per_blk = 16 * a.nwaves;
  a.nblk = (a.N + per_blk - 1) / per_blk;
  const size_t nwg = static_cast<size_t>(a.pairs) * a.nblk;
  if (nwg * 64 * a.nwaves > 0xffffffffull) return hipErrorInvalidConfiguration;
  const dim3 grid(static_cast<unsigned>(nwg));
  size_t lds = step3_fp16_lds_bytes(a.Qa, a.nwaves);
  const int nf4 = 32 * CTQ * 8, nthr = 64 * a.nwaves;
  auto kern = (nf4 + nthr - 1) / nthr <= 2 ? step3_fp16<CTQ, MAXT, true> : step3_fp16<CTQ, MAXT, false>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(64 * a.nwaves), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_step3_fp16(const Step3Args& a, hipStream_t s) {
  if (a.pairs <= 0) return hipSuccess;
  switch (a.Qa / 64) {
    case 1: return launch_step3_fp16_t<1, 1024>(a, s);
    case 2: return launch_step3_fp16_t<2, 1024>(a, s);
    case 3: return launch_step3_fp16_t<3, 1024>(a, s);
    case 4: return launch_step3_fp16_t<4, 1024>(a, s);
    case 6: return launch_step3_fp16_t<6, 512>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fp16_scales(const float* a, size_t a_count, const float* b, size_t b_count, float s_y,
                              float* scales, hipStream_t s) {
  unsigned* u = reinterpret_cast<unsigned*>(scales);
  hipLaunchKernelGGL(scales_init, dim3(1), dim3(64), 0, s, u);
  const int ga = static_cast<int>(std::min<size_t>((a_count + 255) / 256, 2048));
  const int gb = static_cast<int>(std::min<size_t>((b_count + 255) / 256, 2048));
  if (a_count) hipLaunchKernelGGL(absmax_kernel, dim3(ga), dim3(256), 0, s, a, a_count, u);
  if (b_count) hipLaunchKernelGGL(absmax_kernel, dim3(gb), dim3(256), 0, s, b, b_count, u + 1);
  hipLaunchKernelGGL(scales_finalize, dim3(1), dim3(64), 0, s, scales, s_y);
  return hipGetLastError();
}
