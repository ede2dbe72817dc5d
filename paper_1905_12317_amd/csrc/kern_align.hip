// Step 3 + Step 2 of the FTK (eq. fbk3), FP32 form.  Per pair,
//     Xhat[delta][q] = sum_zeta Y[delta][zeta] Zhat[zeta][q]
// as a real GEMM (rows = (delta, re|im), K = (zeta, re|im), columns = q)
// with the shift panel read from L2 and Zhat staged in LDS; then for every
// shift the real rotation sum X[delta][r] = sum_q Xhat e^{-2 pi i q r / Qa}
// as a half-length complex FFT (real-output packing), and the argmax over
// (delta, r) reduced with wave shuffles and a 64-bit atomicMax per pair.
#include "device_common.h"
#include "kernels.h"
#include "step3_epilogue.h"

using namespace ftkdev;

typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// ---------------------------------------------------------------- Step 3

// PREF: enough threads to prefetch a whole chunk in MAXF4 float4 per thread
// (double buffering through registers); otherwise each chunk is fetched after
// the MFMAs of the previous one.
template <int CTQ, int MAXT, bool PREF, int EPI>
__global__ void __launch_bounds__(MAXT) step3_fp32(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  constexpr int ZS = (QH % 64 == 0) ? QH + 32 : QH;  // row stride: ZS % 64 == 32
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  int pair, yb;
  step3_block(blockIdx.x, p.nblk, p.pairs, pair, yb);
  const int d0 = (yb * p.nwaves + wave) * 16;
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nk = 2 * p.H_pad;
  const int ystride = 2 * p.N_pad;
  const float* zsp = static_cast<const float*>(p.zs) + static_cast<size_t>(pair) * QH * nk;
  // LDS: twiddles [Qa] (complex), then two staging buffers [32][ZS] for the
  // K-chunks of Zhat, reused by the FFT epilogue once the K loop is done
  float2* twl = reinterpret_cast<float2*>(smem);
  float* region = smem + 2 * (2 * QH);
  // staging buffer b is region + b * 32 * ZS (formed from the shared base)
  const int nthr = blockDim.x;
  for (int i = tid; i < 2 * QH; i += nthr) twl[i] = p.tw_qa[i];
  constexpr int MAXF4 = 2;
  const int nf4 = QH * 8;  // float4 per K-chunk
  // Zhat rows are [q][k'] (k' = c H_pad + zeta), row 0 already holding the
  // Nyquist fold; a chunk of 32 k' is stored transposed, [k'][q]
  auto load_v = [&](int kc, int t) {
    return load_stream(reinterpret_cast<const float4*>(zsp + static_cast<size_t>(t >> 3) * nk + kc + (t & 7) * 4));
  };
  auto put = [&](float* dst, int t, float4 v) {
    const int qq = t >> 3;
    const int k4 = (t & 7) * 4;
    dst[(k4 + 0) * ZS + qq] = v.x;
    dst[(k4 + 1) * ZS + qq] = v.y;
    dst[(k4 + 2) * ZS + qq] = v.z;
    dst[(k4 + 3) * ZS + qq] = v.w;
  };
  for (int t = tid; t < nf4; t += nthr) put(region, t, load_v(0, t));
  __syncthreads();
  f32x16 acc[CTQ];
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) acc[ct] = zero16();
  const bool active = d0 < p.N;
  // waves past the last shift tile load a valid column and never use it
  const int dcol = 2 * min(d0, p.N_pad - 16) + c32;
  int cur = 0;
  for (int kc = 0; kc < nk; kc += 32) {
    const bool more = kc + 32 < nk;
    // this chunk's shift-panel operands first: loads retire in order, so
    // waiting for them does not wait for the prefetch issued after them
    float av[16];
#pragma unroll
    for (int z = 0; z < 16; ++z) av[z] = p.yt[static_cast<size_t>(kc + 2 * z + r) * ystride + dcol];
    __builtin_amdgcn_sched_barrier(0);
    float4 nreg[MAXF4];
    if (PREF) {
      const int kn = more ? kc + 32 : kc;  // the last chunk re-reads itself
#pragma unroll
      for (int k = 0; k < MAXF4; ++k) nreg[k] = load_v(kn, min(tid + k * nthr, nf4 - 1));
    }
    __builtin_amdgcn_sched_barrier(0);
    if (active) {
      const float* Z = region + cur * (32 * ZS) + r * ZS + c32;
#pragma unroll
      for (int z = 0; z < 16; ++z)
#pragma unroll
        for (int ct = 0; ct < CTQ; ++ct) {
          const float b = Z[(2 * z) * ZS + ct * 32];
          acc[ct] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[z], b, acc[ct], 0, 0, 0);
        }
    }
    if (more) {
      if (PREF) {
#pragma unroll
        for (int k = 0; k < MAXF4; ++k) {
          const int t = tid + k * nthr;
          if (t < nf4) put(region + (cur ^ 1) * (32 * ZS), t, nreg[k]);
        }
      } else {
        for (int t = tid; t < nf4; t += nthr) put(region + (cur ^ 1) * (32 * ZS), t, load_v(kc + 32, t));
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  __syncthreads();
  if (!active) return;
  float2* T = reinterpret_cast<float2*>(region) + wave * (epilogue_lds_bytes_per_wave() / sizeof(float2));
  step3_epilogue_reg<CTQ, EPI>(p, acc, pair, d0, T, twl, lane);
}

__global__ void keys_init_kernel(unsigned long long* keys, size_t count) {
  size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) keys[i] = 0ull;
}

struct PoseOut {
  float value;
  int32_t shift;
  int32_t rot;
};

__global__ void keys_to_poses_kernel(const unsigned long long* keys, PoseOut* poses, size_t count, int Qa,
                                     const float* vscale) {
  size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const unsigned long long k = keys[i];
  PoseOut o;
  if (k == 0ull) {
    o.value = __builtin_nanf("");
    o.shift = -1;
    o.rot = -1;
  } else {
    const uint32_t idx = key_index(k);
    o.value = key_value(k) * (vscale ? *vscale : 1.f);
    o.shift = static_cast<int32_t>(idx / Qa);
    o.rot = static_cast<int32_t>(idx % Qa);
  }
  poses[i] = o;
}

}  // namespace

size_t step3_lds_bytes(int Qa, int nwaves) {
  const int QH = Qa / 2;
  const int ZS = (QH % 64 == 0) ? QH + 32 : QH;
  size_t k = sizeof(float) * 2 * 32 * ZS;
  size_t e = static_cast<size_t>(nwaves) * epilogue_lds_bytes_per_wave();
  return sizeof(float2) * Qa + (k > e ? k : e);
}

template <int CTQ, int MAXT>
static hipError_t launch_step3_t(const Step3Args& a0, hipStream_t s) {
  Step3Args a = a0;
  const int per_blk = 16 * a.nwaves;
  a.nblk = (a.N + per_blk - 1) / per_blk;
  const size_t nwg = static_cast<size_t>(a.pairs) * a.nblk;
  if (nwg * 64 * a.nwaves > 0xffffffffull) return hipErrorInvalidConfiguration;
  const dim3 grid(static_cast<unsigned>(nwg));
  size_t lds = step3_lds_bytes(a.Qa, a.nwaves);
  const int nf4 = 32 * CTQ * 8, nthr = 64 * a.nwaves;
  const bool pref = (nf4 + nthr - 1) / nthr <= 2;
  auto kern = a.xhat ? (pref ? step3_fp32<CTQ, MAXT, true, kEpiStore> : step3_fp32<CTQ, MAXT, false, kEpiStore>)
                     : (pref ? step3_fp32<CTQ, MAXT, true, kEpiRotate> : step3_fp32<CTQ, MAXT, false, kEpiRotate>);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(64 * a.nwaves), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_step3(const Step3Args& a, int precision, hipStream_t s) {
  (void)precision;
  if (a.pairs <= 0) return hipSuccess;
  switch (a.Qa / 64) {
    case 1: return launch_step3_t<1, 1024>(a, s);
    case 2: return launch_step3_t<2, 1024>(a, s);
    case 3: return launch_step3_t<3, 1024>(a, s);
    case 4: return launch_step3_t<4, 1024>(a, s);
    case 6: return launch_step3_t<6, 512>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_keys_init(unsigned long long* keys, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_init_kernel, dim3((count + 255) / 256), dim3(256), 0, s, keys, count);
  return hipGetLastError();
}

hipError_t launch_keys_to_poses(const unsigned long long* keys, void* poses, size_t count, int Qa,
                                const float* vscale, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(keys_to_poses_kernel, dim3((count + 255) / 256), dim3(256), 0, s, keys,
                     static_cast<PoseOut*>(poses), count, Qa, vscale);
  return hipGetLastError();
}
