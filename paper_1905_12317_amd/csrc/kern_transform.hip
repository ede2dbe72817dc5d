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

__global__ void __launch_bounds__(1024) transform_kernel(TransformArgs p) {
  extern __shared__ float2 lds[];
  const int img = blockIdx.x;
  const int n = p.n, nf = p.nf, Qa = p.Qa, M = p.M, w = p.w;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  const float* A = p.imgs + static_cast<size_t>(img) * n * n;
  float2* H = p.scratchH + static_cast<size_t>(img) * n * nf;   // [i][l2]
  float2* Gt = p.scratchG + static_cast<size_t>(img) * nf * nf; // [l2][l1]
  float2* out = p.coeffs + static_cast<size_t>(img) * Qa * M;   // [q][m]

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
      float2* r = fft_batched<false>(ba, bb, nf, 1, p.tw_nf, 1, lane, 64, WaveSync());
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
      float2* r = fft_batched<false>(ba, bb, nf, 1, p.tw_nf, 1, lane, 64, WaveSync());
      for (int t = lane; t < nf; t += 64) Gt[static_cast<size_t>(l2) * nf + t] = r[t];
      wave_sync();
    }
  }
  __syncthreads();
  // ---- 2+3. per ring: interpolate half the angles, fill by symmetry, ring DFT
  const int half = Qa / 2;
  float2* ring = lds + wave * 2 * Qa;
  float2* tile = lds + nwaves * 2 * Qa;  // [Qa][nwaves] transposed output tile
  for (int m0 = 0; m0 < M; m0 += nwaves) {
    const int m = m0 + wave;
    if (m < M) {
      float2* ba = ring;
      float2* bb = ring + Qa;
      for (int pp = lane; pp < half; pp += 64) {
        const int pt = m * half + pp;
        const int b1 = p.pt_base[2 * pt + 0];
        const int b2 = p.pt_base[2 * pt + 1];
        const float* k1 = p.pt_ker + static_cast<size_t>(pt) * 2 * w;
        const float* k2 = k1 + w;
        float2 acc = make_float2(0.f, 0.f);
        for (int bi = 0; bi < w; ++bi) {
          int l2 = b2 + bi;
          l2 -= (l2 >= nf) ? nf : 0;
          const float2* col = Gt + static_cast<size_t>(l2) * nf;
          float2 s = make_float2(0.f, 0.f);
          for (int ai = 0; ai < w; ++ai) {
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
      }
      wave_sync();
      float2* r = fft_batched<false>(ba, bb, Qa, 1, p.tw_qa, 1, lane, 64, WaveSync());
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
  return a > c ? a : c;
}

int transform_waves() {
  static int w = 0;
  if (w == 0) {
    const char* v = std::getenv("FTK_TRANSFORM_WAVES");
    const int x = v ? std::atoi(v) : 0;
    w = (x >= 1 && x <= 16) ? x : 16;
  }
  return w;
}

hipError_t launch_transform(const TransformArgs& args, int cnt, hipStream_t stream) {
  if (cnt <= 0) return hipSuccess;
  const int nwaves = transform_waves();
  size_t lds = transform_lds_bytes(args.nf, args.Qa, nwaves);
  hipLaunchKernelGGL(transform_kernel, dim3(cnt), dim3(64 * nwaves), lds, stream, args);
  return hipGetLastError();
}
