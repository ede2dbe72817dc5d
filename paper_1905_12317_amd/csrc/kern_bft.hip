// Brute-force translations (Section 6.2 of the paper) on gfx950: the
// comparison method that steps through the shifts one by one and handles the
// rotations with the angular FFT, in FP32.
//
//   1. bft_translate: for every image A, shift delta and ring m, the ring
//      samples Ahat(k_m, psi_p) / Qa (kept by the transform) are multiplied
//      by the translation phase exp(-i k_m . delta) (eq. Fdk) and
//      transformed along the ring (eq. aqkcalc), giving the translated
//      coefficients T_delta a(k_m; q), q = 0 .. Qa/2.  One wave per ring, a
//      Stockham FFT in LDS; the outputs go out through an LDS tile so that
//      every store is a 128-byte run of m.
//   2. Step 1 with zeta = delta and no mode offset (launch_step1_bft,
//      kern_step1.hip): the sum of eq. fbk3 with l_max = 0,
//      Xhat(delta, q) = 2 pi sum_m w_m T_delta a(k_m; q) conj b(k_m; q),
//      as the same MFMA GEMM over the templates, staged as Zhat would be.
//   3. xhat_rotate: each wave reads the Xhat of 16 shifts of a pair into the
//      register layout of the Step 3 epilogue (rotation FFT of eq. 1dfft and
//      the argmax) and runs it, U times over for U-fold rotation upsampling.
//      FTK's Step 3 hands its Xhat to the same kernel when upsampling.
#include "device_common.h"
#include "kernels.h"
#include "step3_epilogue.h"

using namespace ftkdev;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr float kPiF = 3.14159265358979f;
constexpr int kBftDB = 8;       // shifts per translate workgroup
constexpr int kBftWaves = 16;   // waves per translate workgroup

template <int QA>
__global__ void __launch_bounds__(64 * kBftWaves) bft_translate_kernel(BftTranslateArgs p) {
  extern __shared__ float2 lds[];
  constexpr bool CT = QA > 0;
  const int Qa = CT ? QA : p.Qa;
  const int QH = Qa / 2;
  const int M = p.M;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int NW = kBftWaves;
  const int dblocks = (p.N_pad + kBftDB - 1) / kBftDB;
  const int A = blockIdx.x / dblocks;
  const int db = blockIdx.x - A * dblocks;
  // LDS: twiddles [Qa], output tile [QH + 1][NW], per-wave FFT buffers [2][Qa]
  float2* tw = lds;
  float2* tile = tw + Qa;
  float2* ring = tile + (QH + 1) * NW + wave * 2 * Qa;
  for (int i = tid; i < Qa; i += blockDim.x) tw[i] = p.tw_qa[i];
  __syncthreads();
  const float2* pol = p.polar + static_cast<size_t>(A) * M * Qa;
  for (int dd = 0; dd < kBftDB; ++dd) {
    const int d = db * kBftDB + dd;
    if (d >= p.N_pad) break;  // the same for the whole workgroup
    float2* out = p.ta + (static_cast<size_t>(A) * (QH + 1) * p.N_pad + d) * M;
    for (int m0 = 0; m0 < M; m0 += NW) {
      const int m = m0 + wave;
      if (m < M) {
        if (d < p.N) {
          const float2 kd = p.kd[static_cast<size_t>(d) * M + m];
          const float2* src = pol + static_cast<size_t>(m) * Qa;
          float2* ba = ring;
          float2* bb = ring + Qa;
          for (int pp = lane; pp < Qa; pp += 64) {
            // k . delta at psi_p: tw[p] = (cos psi_p, -sin psi_p)
            const float2 c = tw[pp];
            const float th = kd.x * c.x - kd.y * c.y;
            float sn, cn;
            sincosf(th, &sn, &cn);
            const float2 v = src[pp];
            ba[pp] = make_float2(v.x * cn + v.y * sn, v.y * cn - v.x * sn);  // v e^{-i th}
          }
          wave_sync();
          float2* r;
          if constexpr (CT)
            r = ct_fft<QA, 1, 1, false, 64, 1>(ba, bb, tw, lane, WaveSync());
          else
            r = fft_batched<false>(ba, bb, Qa, 1, tw, 1, lane, 64, WaveSync());
          for (int q = lane; q <= QH; q += 64) tile[q * NW + wave] = r[q];
        } else {
          for (int q = lane; q <= QH; q += 64) tile[q * NW + wave] = make_float2(0.f, 0.f);
        }
      }
      __syncthreads();
      const int mc = min(NW, M - m0);
      for (int t = tid; t < (QH + 1) * mc; t += blockDim.x) {
        const int q = t / mc;
        const int mm = t - q * mc;
        out[static_cast<size_t>(q) * p.N_pad * M + m0 + mm] = tile[q * NW + mm];
      }
      __syncthreads();
    }
  }
}

// One wave per (pair, 16 shifts).  The Xhat row of mode q holds
// [c][delta] (c = 0 real, 1 imaginary part; H_pad = the padded shift count),
// so the wave's Xhat is 2 QH runs of 16 floats (64 bytes).  They are read
// with 16-byte loads, four lanes per run, into LDS rows [c][q][16] (stride
// kRotRow), then into the epilogue's register layout: lane (h, j), register
// v = 4 g + r of tile ct holds mode 32 ct + j, shift d0 + 4 g + 2 h + r / 2,
// part r % 2 (one LDS float2 read gives two neighbouring shifts of a part).
// Without upsampling the epilogue's transpose rows reuse the same LDS once
// the registers hold Xhat.  With U > 1 (UP) the rows stay, and pass u reads
// them multiplied by e^{-i q phi_u}, phi_u = 2 pi u / (U Qa): the Qa-point
// transform of that sequence is X at the rotations gamma_r + phi_u (the
// zero-padded sum of the remark after eq. 1dfft, sampled U times finer).
// The Nyquist mode (imaginary part of the q = 0 column) contributes
// Xhat_N cos(Qa gamma / 2), i.e. Xhat_N (-1)^r cos(pi u / U) on pass u.
constexpr int kRotRow = 18;  // floats per LDS row: 16 shifts + 2 (row starts spread over the banks)

__host__ __device__ constexpr size_t rot_rows_floats(int QH) { return static_cast<size_t>(2) * QH * kRotRow; }
__host__ __device__ constexpr size_t rot_wave_floats(int QH, bool up) {
  return up ? rot_rows_floats(QH) + epilogue_lds_bytes_per_wave() / sizeof(float)
            : (rot_rows_floats(QH) > epilogue_lds_bytes_per_wave() / sizeof(float)
                   ? rot_rows_floats(QH)
                   : epilogue_lds_bytes_per_wave() / sizeof(float));
}

template <int CTQ, bool UP>
__global__ void __launch_bounds__(256) xhat_rotate_kernel(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  constexpr int Qa = 2 * QH;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  float2* twl = reinterpret_cast<float2*>(smem);
  for (int i = tid; i < Qa; i += blockDim.x) twl[i] = p.tw_qa[i];
  __syncthreads();
  const int tiles = (p.N + 15) / 16;
  const size_t unit = static_cast<size_t>(blockIdx.x) * p.nwaves + wave;
  if (unit >= static_cast<size_t>(p.pairs) * tiles) return;
  const int pair = static_cast<int>(unit / tiles);
  const int d0 = static_cast<int>(unit - static_cast<size_t>(pair) * tiles) * 16;
  const int h = lane >> 5;
  const int j = lane & 31;
  float* S = smem + 2 * Qa + wave * rot_wave_floats(QH, UP);
  {
    // run s = 16 k + lane / 4 is (q, c) = (s / 2, s % 2); quarter lane % 4
    const float* zp = static_cast<const float*>(p.zs) + static_cast<size_t>(pair) * QH * 2 * p.H_pad + d0 +
                      4 * (lane & 3);
    constexpr int NK = 2 * QH / 16;
    f32x4 v[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int s = 16 * k + (lane >> 2);
      v[k] = __builtin_nontemporal_load(
          reinterpret_cast<const f32x4*>(zp + static_cast<size_t>(s >> 1) * 2 * p.H_pad + (s & 1) * p.H_pad));
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int s = 16 * k + (lane >> 2);
      float* d = S + ((s & 1) * QH + (s >> 1)) * kRotRow + 4 * (lane & 3);
      d[0] = v[k][0];
      d[1] = v[k][1];
      d[2] = v[k][2];
      d[3] = v[k][3];
    }
  }
  wave_sync();
  f32x16 acc[CTQ];
  if constexpr (!UP) {
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const float2 x = *reinterpret_cast<const float2*>(S + (c * QH + 32 * ct + j) * kRotRow + 4 * g + 2 * h);
          acc[ct][4 * g + c] = x.x;
          acc[ct][4 * g + 2 + c] = x.y;
        }
    wave_sync();
    step3_epilogue_reg<CTQ>(p, acc, pair, d0, reinterpret_cast<float2*>(S), twl, lane);
  } else {
    const int U = p.up;
    const int Qr = U * Qa;
    float2* T = reinterpret_cast<float2*>(S + rot_rows_floats(QH));
    for (int u = 0; u < U; ++u) {
      const float nyq = cosf(static_cast<float>(kPiF * u) / static_cast<float>(U));
#pragma unroll
      for (int ct = 0; ct < CTQ; ++ct) {
        const int q = 32 * ct + j;
        // e^{-i q phi_u} from the exact angle index (q u mod U Qa)
        float sn, cn;
        sincosf(2.f * kPiF * static_cast<float>((q * u) % Qr) / static_cast<float>(Qr), &sn, &cn);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float2 re = *reinterpret_cast<const float2*>(S + (32 * ct + j) * kRotRow + 4 * g + 2 * h);
          const float2 im = *reinterpret_cast<const float2*>(S + (QH + 32 * ct + j) * kRotRow + 4 * g + 2 * h);
          if (q == 0) {
            acc[ct][4 * g + 0] = re.x;
            acc[ct][4 * g + 1] = im.x * nyq;
            acc[ct][4 * g + 2] = re.y;
            acc[ct][4 * g + 3] = im.y * nyq;
          } else {
            acc[ct][4 * g + 0] = re.x * cn + im.x * sn;
            acc[ct][4 * g + 1] = im.x * cn - re.x * sn;
            acc[ct][4 * g + 2] = re.y * cn + im.y * sn;
            acc[ct][4 * g + 3] = im.y * cn - re.y * sn;
          }
        }
      }
      step3_epilogue_reg<CTQ, kEpiUpsample>(p, acc, pair, d0, T, twl, lane, U, u);
    }
  }
}

template <class K>
hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(lds));
}

}  // namespace

size_t bft_translate_lds_bytes(int Qa) {
  return sizeof(float2) * (static_cast<size_t>(Qa) + static_cast<size_t>(Qa / 2 + 1) * kBftWaves +
                           static_cast<size_t>(kBftWaves) * 2 * Qa);
}

hipError_t launch_bft_translate(const BftTranslateArgs& a, hipStream_t s) {
  if (a.nA <= 0 || a.N_pad <= 0) return hipSuccess;
  const size_t nwg = static_cast<size_t>(a.nA) * ((a.N_pad + kBftDB - 1) / kBftDB);
  if (nwg > 0x7fffffffull) return hipErrorInvalidConfiguration;
  const size_t lds = bft_translate_lds_bytes(a.Qa);
  auto kern = bft_translate_kernel<0>;
  switch (a.Qa) {
    case 64: kern = bft_translate_kernel<64>; break;
    case 128: kern = bft_translate_kernel<128>; break;
    case 192: kern = bft_translate_kernel<192>; break;
    case 256: kern = bft_translate_kernel<256>; break;
    case 384: kern = bft_translate_kernel<384>; break;
    default: break;
  }
  hipError_t e = set_lds(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(nwg)), dim3(64 * kBftWaves), lds, s, a);
  return hipGetLastError();
}

size_t xhat_rotate_lds_bytes(int Qa, int nwaves, int up) {
  return sizeof(float2) * static_cast<size_t>(Qa) +
         sizeof(float) * static_cast<size_t>(nwaves) * rot_wave_floats(Qa / 2, up > 1);
}

hipError_t launch_xhat_rotate(const Step3Args& a, hipStream_t s) {
  if (a.pairs <= 0) return hipSuccess;
  if (a.nwaves < 1 || a.nwaves > 4 || a.up < 1) return hipErrorInvalidValue;
  const size_t units = static_cast<size_t>(a.pairs) * ((a.N + 15) / 16);
  const size_t nwg = (units + a.nwaves - 1) / a.nwaves;
  if (nwg > 0x7fffffffull) return hipErrorInvalidConfiguration;
  const size_t lds = xhat_rotate_lds_bytes(a.Qa, a.nwaves, a.up);
  hipError_t e;
#define FTK_BR(ct)                                                                                  \
  case ct: {                                                                                         \
    auto k = a.up > 1 ? xhat_rotate_kernel<ct, true> : xhat_rotate_kernel<ct, false>;                \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;                                               \
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nwg)), dim3(64 * a.nwaves), lds, s, a);          \
    break;                                                                                           \
  }
  switch (a.Qa / 64) {
    FTK_BR(1)
    FTK_BR(2)
    FTK_BR(3)
    FTK_BR(4)
    FTK_BR(6)
    default: return hipErrorInvalidValue;
  }
#undef FTK_BR
  return hipGetLastError();
}
