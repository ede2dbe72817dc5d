// Pixels -> Fourier-Bessel coefficients (Section 3.2 of the paper).
//
// Per image:
//   1. deapodise and zero-pad the n x n pixels onto an nf x nf grid and take
//      its 2D DFT (rows, then columns; Stockham FFTs in LDS), giving the
//      spreading-kernel-deconvolved spectrum G(l1, l2) on a grid of spacing
//      h = 2 pi / nf in t = k dx;
//   2. interpolate G with the w x w separable spreading kernel to the polar
//      points (k_m cos psi_p, k_m sin psi_p) for p < Qa/2 (type-2 NUFFT);
//      the other half follows from Ahat(k, psi + pi) = conj Ahat(k, psi)
//      for real images;
//   3. a length-Qa DFT on each ring gives a(k_m; q) (eq. aqkcalc).
// All scale factors (dx^2 h^2 / Qa and the kernel deconvolution) are folded
// into the per-dimension deapodisation table.
#include <cstdlib>

#include "device_common.h"
#include "kernels.h"

using namespace ftkdev;

namespace {

// NF, QA > 0: the grid and ring lengths known at compile time (unrolled
// passes, twiddles copied to LDS); 0: read from the arguments.
template <int NF, int QA>
__global__ void __launch_bounds__(1024) transform_kernel(TransformArgs p) {
  extern __shared__ float2 lds_all[];
  constexpr bool CT = NF > 0 && QA > 0;
  const int img = blockIdx.x;
  const int n = p.n, nf = CT ? NF : p.nf, Qa = CT ? QA : p.Qa, M = p.M, w = p.w;
  // compile-time form: twiddles of both lengths at the front of LDS
  float2* lds = lds_all + (CT ? NF + QA : 0);
  const float2* tw_nf = p.tw_nf;
  const float2* tw_qa = p.tw_qa;
  if constexpr (CT) {
    for (int i = threadIdx.x; i < NF; i += blockDim.x) lds_all[i] = p.tw_nf[i];
    for (int i = threadIdx.x; i < QA; i += blockDim.x) lds_all[NF + i] = p.tw_qa[i];
    __syncthreads();
    tw_nf = lds_all;
    tw_qa = lds_all + NF;
  }
  auto fft_nf = [&](float2* a, float2* b, int lane) -> float2* {
    if constexpr (CT)
      return ct_fft<NF, 1, 1, false, 64, 1>(a, b, tw_nf, lane, WaveSync());
    else
      return fft_batched<false>(a, b, nf, 1, tw_nf, 1, lane, 64, WaveSync());
  };
  auto fft_qa = [&](float2* a, float2* b, int lane) -> float2* {
    if constexpr (CT)
      return ct_fft<QA, 1, 1, false, 64, 1>(a, b, tw_qa, lane, WaveSync());
    else
      return fft_batched<false>(a, b, Qa, 1, tw_qa, 1, lane, 64, WaveSync());
  };
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const float* A = p.imgs + static_cast<size_t>(img) * n * n;
  float2* H = p.scratchH + static_cast<size_t>(img) * n * nf;   // [i][l2]
  float2* Gt = p.scratchG + static_cast<size_t>(img) * nf * nf; // [l2][l1]
  float2* out = p.coeffs + static_cast<size_t>(img) * Qa * M;   // [q][m]

  if constexpr (CT) {
    // compile-time form: the next row / column is loaded while the current
    // one is transformed (n <= NF / 2, so NPL values per lane)
    constexpr int NPL = (NF / 2 + 63) / 64;
    float2* ba = lds + wave * 2 * NF;
    float2* bb = ba + NF;
    // ---- 1a. rows: H[i][l2] = sum_j D[i] D[j] A[i][j] e^{-2 pi i s2 l2 / nf}
    {
      float dj[NPL], cur[NPL], nxt[NPL];
#pragma unroll
      for (int k = 0; k < NPL; ++k) {
        const int j = lane + 64 * k;
        dj[k] = j < n ? p.deapod[j] : 0.f;
      }
      auto load_row = [&](int i, float (&v)[NPL]) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const int j = lane + 64 * k;
          v[k] = (i < n && j < n) ? A[i * n + j] : 0.f;
        }
      };
      load_row(wave, cur);
      for (int i = wave; i < n; i += nwaves) {
        load_row(i + nwaves, nxt);
#pragma unroll
        for (int k = 0; k < NF / 64; ++k) ba[lane + 64 * k] = make_float2(0.f, 0.f);
        wave_sync();
        const float di = p.deapod[i];
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const int j = lane + 64 * k;
          if (j < n) {
            int pos = j - n / 2;
            pos += (pos < 0) ? NF : 0;
            ba[pos] = make_float2(di * dj[k] * cur[k], 0.f);
          }
        }
        wave_sync();
        float2* r = fft_nf(ba, bb, lane);
#pragma unroll
        for (int k = 0; k < NF / 64; ++k) H[static_cast<size_t>(i) * NF + lane + 64 * k] = r[lane + 64 * k];
        wave_sync();
#pragma unroll
        for (int k = 0; k < NPL; ++k) cur[k] = nxt[k];
      }
    }
    __syncthreads();
    // ---- 1b. columns: Gt[l2][l1] = sum_i H[i][l2] e^{-2 pi i s1 l1 / nf}
    {
      float2 cur[NPL], nxt[NPL];
      auto load_col = [&](int l2, float2 (&v)[NPL]) {
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const int i = lane + 64 * k;
          v[k] = (i < n && l2 < NF) ? H[static_cast<size_t>(i) * NF + l2] : make_float2(0.f, 0.f);
        }
      };
      load_col(wave, cur);
      for (int l2 = wave; l2 < NF; l2 += nwaves) {
        load_col(l2 + nwaves, nxt);
#pragma unroll
        for (int k = 0; k < NF / 64; ++k) ba[lane + 64 * k] = make_float2(0.f, 0.f);
        wave_sync();
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
          const int i = lane + 64 * k;
          if (i < n) {
            int pos = i - n / 2;
            pos += (pos < 0) ? NF : 0;
            ba[pos] = cur[k];
          }
        }
        wave_sync();
        float2* r = fft_nf(ba, bb, lane);
#pragma unroll
        for (int k = 0; k < NF / 64; ++k) Gt[static_cast<size_t>(l2) * NF + lane + 64 * k] = r[lane + 64 * k];
        wave_sync();
#pragma unroll
        for (int k = 0; k < NPL; ++k) cur[k] = nxt[k];
      }
    }
    __syncthreads();  // Gt complete, and the LDS rows free for the rings
  } else {
    // ---- 1a. rows: H[i][l2] = sum_j D[i] D[j] A[i][j] e^{-2 pi i s2 l2 / nf}
    {
      float2* ba = lds + wave * 2 * nf;
      float2* bb = ba + nf;
      for (int i = wave; i < n; i += nwaves) {
        for (int t = lane; t < nf; t += 64) ba[t] = make_float2(0.f, 0.f);
        wave_sync();
        const float di = p.deapod[i];
        for (int j = lane; j < n; j += 64) {
          int pos = j - n / 2;
          pos += (pos < 0) ? nf : 0;
          ba[pos] = make_float2(di * p.deapod[j] * A[i * n + j], 0.f);
        }
        wave_sync();
        float2* r = fft_nf(ba, bb, lane);
        for (int t = lane; t < nf; t += 64) H[static_cast<size_t>(i) * nf + t] = r[t];
        wave_sync();
      }
    }
    __syncthreads();
    // ---- 1b. columns: Gt[l2][l1] = sum_i H[i][l2] e^{-2 pi i s1 l1 / nf}
    {
      float2* ba = lds + wave * 2 * nf;
      float2* bb = ba + nf;
      for (int l2 = wave; l2 < nf; l2 += nwaves) {
        for (int t = lane; t < nf; t += 64) ba[t] = make_float2(0.f, 0.f);
        wave_sync();
        for (int i = lane; i < n; i += 64) {
          int pos = i - n / 2;
          pos += (pos < 0) ? nf : 0;
          ba[pos] = H[static_cast<size_t>(i) * nf + l2];
        }
        wave_sync();
        float2* r = fft_nf(ba, bb, lane);
        for (int t = lane; t < nf; t += 64) Gt[static_cast<size_t>(l2) * nf + t] = r[t];
        wave_sync();
      }
    }
    __syncthreads();
  }
  if (!p.coeffs) return;  // the fine grid only (uniform over the launch)
  // ---- 2+3. per ring: interpolate half the angles, fill by symmetry, ring DFT
  const int half = Qa / 2;
  float2* ring = lds + wave * 2 * Qa;
  float2* tile = lds + nwaves * 2 * Qa;  // [Qa][nwaves] transposed output tile
  for (int m0 = 0; m0 < M; m0 += nwaves) {
    const int m = m0 + wave;
    if (m < M) {
      float2* ba = ring;
      float2* bb = ring + Qa;
      // compile-time form: width 8, every tap load of a point issued at once
      const int wk = CT ? 8 : w;
#pragma unroll
      for (int pp = lane; pp < half; pp += 64) {
        const int pt = m * half + pp;
        const int b1 = p.pt_base[2 * pt + 0];
        const int b2 = p.pt_base[2 * pt + 1];
        const float* k1 = p.pt_ker + static_cast<size_t>(pt) * 2 * wk;
        const float* k2 = k1 + wk;
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int bi = 0; bi < wk; ++bi) {
          int l2 = b2 + bi;
          l2 -= (l2 >= nf) ? nf : 0;
          const float2* col = Gt + static_cast<size_t>(l2) * nf;
          float2 s = make_float2(0.f, 0.f);
#pragma unroll
          for (int ai = 0; ai < wk; ++ai) {
            int l1 = b1 + ai;
            l1 -= (l1 >= nf) ? nf : 0;
            float2 g = col[l1];
            s.x += k1[ai] * g.x;
            s.y += k1[ai] * g.y;
          }
          acc.x += k2[bi] * s.x;
          acc.y += k2[bi] * s.y;
        }
        ba[pp] = acc;
        ba[pp + half] = cconj(acc);
        if (p.polar) {
          float2* pr = p.polar + (static_cast<size_t>(img) * M + m) * Qa;
          pr[pp] = acc;
          pr[pp + half] = cconj(acc);
        }
      }
      wave_sync();
      float2* r = fft_qa(ba, bb, lane);
      for (int q = lane; q < Qa; q += 64) tile[q * nwaves + wave] = r[q];
    }
    __syncthreads();
    const int mcount = min(nwaves, M - m0);
    for (int t = tid; t < Qa * mcount; t += blockDim.x) {
      const int q = t / mcount;
      const int mm = t - q * mcount;
      out[static_cast<size_t>(q) * M + m0 + mm] = tile[q * nwaves + mm];
    }
    __syncthreads();
  }
}

}  // namespace

size_t transform_lds_bytes(int nf, int Qa, int nwaves) {
  size_t a = static_cast<size_t>(nwaves) * 2 * nf * sizeof(float2);
  size_t c = static_cast<size_t>(nwaves) * 2 * Qa * sizeof(float2) +
             static_cast<size_t>(Qa) * nwaves * sizeof(float2);
  // plus the twiddles of the compile-time form
  return (a > c ? a : c) + static_cast<size_t>(nf + Qa) * sizeof(float2);
}

int transform_waves(int nf, int Qa) {
  static int w = 0;
  if (w == 0) {
    const char* v = std::getenv("FTK_TRANSFORM_WAVES");
    const int x = v ? std::atoi(v) : 0;
    w = (x >= 1 && x <= 16) ? x : 16;
  }
  int k = w;
  while (k > 1 && transform_lds_bytes(nf, Qa, k) > 160 * 1024) --k;
  return k;
}

hipError_t launch_transform(const TransformArgs& args, int cnt, hipStream_t stream) {
  if (cnt <= 0) return hipSuccess;
  const int nwaves = transform_waves(args.nf, args.Qa);
  const size_t lds = transform_lds_bytes(args.nf, args.Qa, nwaves);
  auto kern = transform_kernel<0, 0>;
  if (args.nf == args.Qa && args.w == 8) {
    switch (args.nf) {
      case 128: kern = transform_kernel<128, 128>; break;
      case 192: kern = transform_kernel<192, 192>; break;
      case 256: kern = transform_kernel<256, 256>; break;
      case 384: kern = transform_kernel<384, 384>; break;
      default: break;
    }
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(cnt), dim3(64 * nwaves), lds, stream, args);
  return hipGetLastError();
}
