// Device helpers shared by the FTK kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftkdev {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Make LDS writes of this wave visible to all of its lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct WaveSync {
  __device__ __forceinline__ void operator()() const { wave_sync(); }
};
struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

// Small DFTs in registers.  Forward sign exp(-2 pi i / R); INV flips it.
template <bool INV>
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <bool INV>
__device__ __forceinline__ void dft3(float2* v) {
  const float s3 = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 t1 = cadd(v[1], v[2]);
  float2 t2 = csub(v[1], v[2]);
  float2 m = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  // forward: V1 = m - i s3 t2, V2 = m + i s3 t2
  float2 it2 = make_float2(-s3 * t2.y, s3 * t2.x);  // i s3 t2
  v[0] = cadd(v[0], t1);
  if (!INV) {
    v[1] = csub(m, it2);
    v[2] = cadd(m, it2);
  } else {
    v[1] = cadd(m, it2);
    v[2] = csub(m, it2);
  }
}
template <bool INV>
__device__ __forceinline__ void dft4(float2* v) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
  // -i t3 = (t3.y, -t3.x)
  float2 mit3 = make_float2(t3.y, -t3.x);
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  if (!INV) {
    v[1] = cadd(t1, mit3);
    v[3] = csub(t1, mit3);
  } else {
    v[1] = csub(t1, mit3);
    v[3] = cadd(t1, mit3);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void stockham_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                              int L, int Ns, int batch, const float2* __restrict__ tw,
                                              int tw_stride, int tid, int nth) {
  const int LR = L / R;
  const int stride = L / (Ns * R);
  const int total = LR * batch;
  for (int t = tid; t < total; t += nth) {
    const int b = t / LR;
    const int j = t - b * LR;
    const float2* s = src + b * L;
    float2* d = dst + b * L;
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float2 x = s[j + r * LR];
      if (r > 0) {
        float2 w = tw[(k * r * stride) * tw_stride];
        if (INV) w.y = -w.y;
        x = cmul(x, w);
      }
      v[r] = x;
    }
    if (R == 2) dft2<INV>(v);
    if (R == 3) dft3<INV>(v);
    if (R == 4) dft4<INV>(v);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[base + r * Ns] = v[r];
  }
}

// Batched Stockham FFT of `batch` contiguous sequences of length L
// (L = 2^a 3^b) held in LDS.  Twiddles: tw[k * tw_stride] = exp(-2 pi i k / L)
// for k < L.  Radix order: 4s, then 2, then 3s.  Returns the buffer that
// holds the result (a or b).  Sync is called after every pass.
template <bool INV, class Sync>
__device__ float2* fft_batched(float2* a, float2* b, int L, int batch, const float2* __restrict__ tw,
                               int tw_stride, int tid, int nth, Sync sync) {
  int Ns = 1, rem = L;
  float2* src = a;
  float2* dst = b;
  while (rem > 1) {
    if (rem % 4 == 0) {
      stockham_pass<4, INV>(src, dst, L, Ns, batch, tw, tw_stride, tid, nth);
      Ns *= 4; rem /= 4;
    } else if (rem % 2 == 0) {
      stockham_pass<2, INV>(src, dst, L, Ns, batch, tw, tw_stride, tid, nth);
      Ns *= 2; rem /= 2;
    } else {
      stockham_pass<3, INV>(src, dst, L, Ns, batch, tw, tw_stride, tid, nth);
      Ns *= 3; rem /= 3;
    }
    sync();
    float2* t = src; src = dst; dst = t;
  }
  return src;
}

// The same Stockham FFT with the length, batch, thread count and twiddle
// stride known at compile time: every index division becomes a shift or a
// multiply and every pass unrolls.  Radix order as above.
template <int L, int R, int NS, int BATCH, bool INV, int NTH, int TWS>
__device__ __forceinline__ void ct_pass(const float2* __restrict__ src, float2* __restrict__ dst,
                                        const float2* __restrict__ tw, int tid) {
  constexpr int LR = L / R;
  constexpr int STRIDE = L / (NS * R);
  constexpr int TOTAL = LR * BATCH;
#pragma unroll
  for (int t0 = 0; t0 < TOTAL; t0 += NTH) {
    const int t = t0 + tid;
    if ((TOTAL % NTH) == 0 || t < TOTAL) {
      const int b = t / LR;
      const int j = t - b * LR;
      const int k = j % NS;
      const float2* s = src + b * L;
      float2* d = dst + b * L;
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        float2 x = s[j + r * LR];
        if (r > 0) {
          float2 w = tw[(k * r * STRIDE) * TWS];
          if (INV) w.y = -w.y;
          x = cmul(x, w);
        }
        v[r] = x;
      }
      if (R == 2) dft2<INV>(v);
      if (R == 3) dft3<INV>(v);
      if (R == 4) dft4<INV>(v);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) d[base + r * NS] = v[r];
    }
  }
}

template <int L, int NS, int BATCH, bool INV, int NTH, int TWS, class Sync>
__device__ __forceinline__ float2* ct_fft(float2* a, float2* b, const float2* __restrict__ tw, int tid, Sync sync) {
  if constexpr (NS >= L) {
    return a;
  } else {
    constexpr int REM = L / NS;
    constexpr int R = (REM % 4 == 0) ? 4 : ((REM % 2 == 0) ? 2 : 3);
    ct_pass<L, R, NS, BATCH, INV, NTH, TWS>(a, b, tw, tid);
    sync();
    return ct_fft<L, NS * R, BATCH, INV, NTH, TWS>(b, a, tw, tid, sync);
  }
}

// Order-preserving key of (value, index): a larger key is a larger value,
// and for equal values the smaller index.  Used with 64-bit atomicMax.
__device__ __forceinline__ unsigned long long pose_key(float v, uint32_t idx) {
  uint32_t u = __float_as_uint(v);
  uint32_t hi = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return (static_cast<unsigned long long>(hi) << 32) | static_cast<unsigned long long>(~idx);
}
__device__ __forceinline__ float key_value(unsigned long long key) {
  uint32_t hi = static_cast<uint32_t>(key >> 32);
  uint32_t u = (hi & 0x80000000u) ? (hi & 0x7fffffffu) : ~hi;
  return __uint_as_float(u);
}
__device__ __forceinline__ uint32_t key_index(unsigned long long key) {
  return ~static_cast<uint32_t>(key & 0xffffffffull);
}

}  // namespace ftkdev
