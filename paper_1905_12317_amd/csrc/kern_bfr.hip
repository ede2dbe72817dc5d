// Brute-force rotations (Section 6.1 of the paper, eq. 2dconv), the
// comparison method: for every rotation gamma_r the correlation of the image
// with the rotated template over a Cartesian grid of shifts, through the 2D
// convolution theorem on the Cartesian Fourier grid of the pixel DFT,
// k = pi (u, v) with u^2 + v^2 <= (n / 2)^2:
//
//   X(delta, r) = pi^2 sum_k exp(-i k . delta) Ahat(k) conj(Bhat(R_{gamma_r} k)).
//
// For real images the terms at k and -k are conjugates, so the sum is the
// real part of the row v = 0 plus twice the real part of the rows v > 0.
// The phase factorises, exp(-2 pi i u x / n) exp(-2 pi i v y / n) for a shift
// (x, y) in pixels, so over the product grid of the requested shifts' x and
// y offsets the sum is a pruned 2D inverse DFT in two stages:
//
//   T_v(x) = sum_u Ex(x, u) Ahat(u, v) conj(Bhat_r(u, v))      matrix cores
//   X(x, y) = Re sum_v c_v Ey(y, v) T_v(x)                    registers
//
// The paper takes one zero-padded inverse 2D FFT per rotation; on the shift
// grids of alignment (hundreds of shifts) the pruned sums do fewer
// operations than the padded FFT and the first stage is a dense contraction:
// rows are images, columns (template, rotation, x offset), K the u of one
// Fourier row.
#include <cmath>

#include "device_common.h"
#include "kernels.h"

using namespace ftkdev;

namespace {

using f32x4 = float __attribute__((ext_vector_type(4)));

// ---- spectra: the transform's fine grid interpolated at (rotated) grid points
//
// One workgroup per tile of 16 x 16 source points (a, b) of rotation r and
// one image; the tile's rotated points span a patch of the fine grid at most
// 15 s (|cos| + |sin|) + 8 taps wide (s = fine-grid units per unit of u),
// which is staged in LDS once and read by every point's 8 x 8 taps.  With
// quarter set, the rotations r < R / 4 are interpolated over the full disk
// and each value is written for the four quarter turns: the disk maps onto
// itself, Bhat_{r + R/4}(u, v) = Bhat_r(-v, u), so the value at (a, b) of
// rotation r is the value at (b, -a) of rotation r + R / 4.  Only rows
// v >= 0 are stored.  The points' fine-grid coordinates are formed in double
// precision (a float coordinate near nf / 2 would move the point by 1e-5 grid
// units); the tap weights then need only its fractional part, in float, and
// are evaluated as exp(-beta z^2 / (1 + sqrt(1 - z^2))), which equals
// exp(beta (sqrt(1 - z^2) - 1)) without its cancellation at small z.
constexpr int kW = 8;
constexpr int kTile = 16;

__global__ void __launch_bounds__(256) bfr_spectra_kernel(BfrSpectraArgs p) {
  extern __shared__ float2 patch[];  // [ps][ps]
  const int img = blockIdx.y;
  const int V = p.V, ps = p.patch, nf = p.nf;
  const int bmin = p.quarter ? -V : 0;
  const int TA = (2 * V + kTile) / kTile, TB = (V - bmin + kTile) / kTile;
  int t = static_cast<int>(blockIdx.x);
  const int r = t / (TA * TB);
  t -= r * TA * TB;
  const int tb = t / TA, ta = t - tb * TA;
  const int a0 = -V + kTile * ta, b0 = bmin + kTile * tb;
  const int a = a0 + (threadIdx.x & (kTile - 1)), b = b0 + static_cast<int>(threadIdx.x / kTile);
  double c = 1.0, sn = 0.0;
  if (p.quarter) {
    c = p.cs[2 * r];
    sn = p.cs[2 * r + 1];
  }
  // patch origin: the tile's smallest rotated coordinates (a corner) minus
  // the taps below a point
  double mx = 1e300, my = 1e300;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double ca = a0 + (k & 1) * (kTile - 1), cb = b0 + (k >> 1) * (kTile - 1);
    mx = fmin(mx, (c * ca - sn * cb) * p.s_per_u);
    my = fmin(my, (sn * ca + c * cb) * p.s_per_u);
  }
  const int ox = static_cast<int>(floor(mx)) - kW / 2 + 1, oy = static_cast<int>(floor(my)) - kW / 2 + 1;
  // the tile's point nearest the origin decides whether any point is in the disk
  const int na = a0 > 0 ? a0 : (a0 + kTile - 1 < 0 ? a0 + kTile - 1 : 0);
  const int nb = b0 > 0 ? b0 : (b0 + kTile - 1 < 0 ? b0 + kTile - 1 : 0);
  const bool any = na * na + nb * nb <= V * V;  // uniform over the workgroup
  if (any) {
    const float2* G = p.grid + static_cast<size_t>(img) * nf * nf;
    for (int i = threadIdx.x; i < ps * ps; i += blockDim.x) {
      const int ly = i / ps, lx = i - ly * ps;
      int gy = (oy + ly) % nf, gx = (ox + lx) % nf;
      gy += gy < 0 ? nf : 0;
      gx += gx < 0 ? nf : 0;
      patch[i] = G[static_cast<size_t>(gy) * nf + gx];
    }
    __syncthreads();
  }
  float2 val = make_float2(0.f, 0.f);
  if (any && a <= V && b <= V && a * a + b * b <= V * V) {
    const double sx = (c * a - sn * b) * p.s_per_u;  // fine-grid coordinates of R_gamma k
    const double sy = (sn * a + c * b) * p.s_per_u;
    const double fx = floor(sx), fy = floor(sy);
    const float rx = static_cast<float>(sx - fx), ry = static_cast<float>(sy - fy);
    const int bx = static_cast<int>(fx) - kW / 2 + 1 - ox, by = static_cast<int>(fy) - kW / 2 + 1 - oy;
    float wx[kW], wy[kW];
#pragma unroll
    for (int k = 0; k < kW; ++k) {
      // z = (s - (floor(s) - kW/2 + 1 + k)) / (kW / 2)
      const float zx = (rx + static_cast<float>(kW / 2 - 1 - k)) * (2.f / kW);
      const float zy = (ry + static_cast<float>(kW / 2 - 1 - k)) * (2.f / kW);
      const float qx = zx * zx, qy = zy * zy;
      wx[k] = qx < 1.f ? __expf(-p.beta * qx / (1.f + sqrtf(1.f - qx))) : 0.f;
      wy[k] = qy < 1.f ? __expf(-p.beta * qy / (1.f + sqrtf(1.f - qy))) : 0.f;
    }
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int bi = 0; bi < kW; ++bi) {
      const float2* row = patch + (by + bi) * ps + bx;
      float2 s2 = make_float2(0.f, 0.f);
#pragma unroll
      for (int ai = 0; ai < kW; ++ai) {
        const float2 g = row[ai];
        s2.x += wx[ai] * g.x;
        s2.y += wx[ai] * g.y;
      }
      acc.x += wy[bi] * s2.x;
      acc.y += wy[bi] * s2.y;
    }
    val = make_float2(acc.x * p.scale, acc.y * p.scale);
  }
  if (a > V || b > V) return;
  const size_t V1 = static_cast<size_t>(V + 1);
  if (!p.quarter) {
    p.out[(static_cast<size_t>(img) * V1 + b) * p.Up + a + V] = val;
    return;
  }
  int u = a, v = b;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (v >= 0) {
      const size_t rr = static_cast<size_t>(img) * p.R + r + j * (p.R / 4);
      p.out[(rr * V1 + v) * p.Up + u + V] = val;
    }
    const int tmp = u;  // (u, v) -> (v, -u): the same value one quarter turn on
    u = v;
    v = -tmp;
  }
}

// ---- the correlation
//
// Workgroup: 64 images x 32 columns (template, rotation, x offset), four
// waves of 32 x 16 (two 16 x 16 MFMA tiles each, v_mfma_f32_16x16x4_f32,
// complex products as four real ones).  Per chunk of 32 values of u of one
// Fourier row v the image spectra (64 x 32) and the column operand
// Ex(x, u) conj(Bhat_r(u, v)) (32 x 32) are staged in LDS, the next chunk's
// loads in flight during the MFMAs.  At the end of each row the wave folds
// T_v into the 17 y offsets of the pass it keeps per element (136
// accumulators per lane).  Column tiles of 16 never straddle a template
// (R Dx is a multiple of 16), so the 16 lanes holding one image's row of a
// tile reduce their pose keys by shuffles before one atomicMax.
constexpr int kRows = 64, kCols = 32, kKc = 32;
constexpr int kLs = kRows + 2;  // float2 per u of the image tile
constexpr int kRs = kCols + 2;  // float2 per u of the column tile

__global__ void __launch_bounds__(256) bfr_corr_kernel(BfrCorrArgs p) {
  extern __shared__ float2 lds[];
  float2* Ls = lds;
  float2* Rs = Ls + kKc * kLs;
  float2* Es = Rs + kKc * kRs;  // [kBfrDy][V + 1] y phases of the pass
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int nRT = (p.nA + kRows - 1) / kRows;
  const int rt = static_cast<int>(blockIdx.x % nRT), ct = static_cast<int>(blockIdx.x / nRT);
  const int A0 = rt * kRows, c0 = ct * kCols;
  const int V1 = p.V + 1, Up = p.Up, RD = p.R * p.Dx;
  for (int i = tid; i < kBfrDy * V1; i += 256) {
    const int iy = p.iy0 + i / V1;
    Es[i] = iy < p.Dy ? p.ey[static_cast<size_t>(iy) * V1 + i % V1] : make_float2(0.f, 0.f);
  }
  // staging roles: image rows (row = lane: a wave stores 64 consecutive rows of
  // one u into the transposed tile, free of bank conflicts; 8 u from jp),
  // columns (col, 4 u from 4 jq)
  const int lrow = tid & 63, jp = (tid >> 6) * 8;
  const bool lvalid = A0 + lrow < p.nA;
  const float2* lsrc = p.sa + static_cast<size_t>(lvalid ? A0 + lrow : 0) * V1 * Up;
  const int scol = tid & 31, jq = tid >> 5;
  const float2* bsrc;
  const float2* xsrc;
  {
    const int c = c0 + scol;
    const int Bl = c / RD, rem = c - Bl * RD, r = rem / p.Dx, ix = rem - r * p.Dx;
    bsrc = p.sb + (static_cast<size_t>(Bl) * p.R + r) * V1 * Up;
    xsrc = p.ex + static_cast<size_t>(ix) * Up;
  }
  f32x4 lreg[4], breg[2], ereg[2];
  auto load = [&](int4 ch) {
    const int v = ch.x, kc = ch.y;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int j = kc + jp + 2 * m;
      lreg[m] = (lvalid && j < Up) ? *reinterpret_cast<const f32x4*>(lsrc + static_cast<size_t>(v) * Up + j)
                                   : f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const int j = kc + 4 * jq;
    const bool ok = j < Up;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      breg[m] = ok ? *reinterpret_cast<const f32x4*>(bsrc + static_cast<size_t>(v) * Up + j + 2 * m)
                   : f32x4{0.f, 0.f, 0.f, 0.f};
      ereg[m] = ok ? *reinterpret_cast<const f32x4*>(xsrc + j + 2 * m) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      Ls[(jp + 2 * m) * kLs + lrow] = make_float2(lreg[m][0], lreg[m][1]);
      Ls[(jp + 2 * m + 1) * kLs + lrow] = make_float2(lreg[m][2], lreg[m][3]);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float bx = breg[m][2 * h], by = breg[m][2 * h + 1];
        const float ex = ereg[m][2 * h], ey = ereg[m][2 * h + 1];
        // Ex conj(Bhat)
        Rs[(4 * jq + 2 * m + h) * kRs + scol] = make_float2(ex * bx + ey * by, ey * bx - ex * by);
      }
    }
  };
  f32x4 Tr[2], Ti[2];
  float acc[2][4][kBfrDy];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    Tr[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    Ti[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int y = 0; y < kBfrDy; ++y) acc[t][i][y] = 0.f;
  }
  const int k16 = lane >> 4, r16 = lane & 15;
  int4 ch = p.chunks[0];
  load(ch);
  for (int ci = 0; ci < p.nch; ++ci) {
    __syncthreads();  // the previous chunk's reads are done
    store();
    __syncthreads();
    const int4 cur = ch;
    if (ci + 1 < p.nch) {
      ch = p.chunks[ci + 1];
      load(ch);
    }
    for (int ks = 0; ks < cur.z; ++ks) {
      const int k = 4 * ks + k16;
      const float2 b = Rs[k * kRs + 16 * wc + r16];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float2 a = Ls[k * kLs + 32 * wr + 16 * t + r16];
        Tr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, Tr[t], 0, 0, 0);
        Tr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.y, b.y, Tr[t], 0, 0, 0);
        Ti[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.y, Ti[t], 0, 0, 0);
        Ti[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.x, Ti[t], 0, 0, 0);
      }
    }
    if (cur.w) {  // the row v is complete: fold T_v into the y offsets
      const float2* e = Es + cur.x;
#pragma unroll
      for (int y = 0; y < kBfrDy; ++y) {
        const float2 ey = e[y * V1];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[t][i][y] += ey.x * Tr[t][i] - ey.y * Ti[t][i];
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        Tr[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        Ti[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  // outputs: lane holds rows 32 wr + 16 t + 4 k16 + i of column 16 wc + r16
  const int c = c0 + 16 * wc + r16;
  const int Bl = c / RD, rem = c - Bl * RD, r = rem / p.Dx, ix = rem - r * p.Dx;
  const size_t Bg = static_cast<size_t>(p.B0) + Bl;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int A = A0 + 32 * wr + 16 * t + 4 * k16 + i;
      unsigned long long key = 0ull;
      if (A < p.nA) {
#pragma unroll
        for (int y = 0; y < kBfrDy; ++y) {
          const int iy = p.iy0 + y;
          if (iy >= p.Dy) break;
          const int s = p.head[ix * p.Dy + iy];
          if (s < 0) continue;
          const float val = acc[t][i][y];
          const unsigned long long k = pose_key(val, static_cast<uint32_t>(s) * p.R + r);
          key = k > key ? k : key;
          if (p.X) {
            float* xrow = p.X + (static_cast<size_t>(A) * p.nB + Bg) * p.N * p.R + r;
            for (int ss = s; ss >= 0; ss = p.nxt[ss]) xrow[static_cast<size_t>(ss) * p.R] = val;
          }
        }
      }
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const unsigned long long o = __shfl_xor(key, off, 64);
        key = o > key ? o : key;
      }
      if (r16 == 0 && A < p.nA && key != 0ull) atomicMax(p.keys + static_cast<size_t>(A) * p.nB + Bg, key);
    }
}

}  // namespace

int bfr_spectra_patch(double s_per_u) {
  // the rotated tile's extent (at most (kTile - 1) s sqrt 2) plus the taps and rounding
  return static_cast<int>(std::ceil((kTile - 1) * s_per_u * 1.4142135623730951)) + kW + 2;
}

hipError_t launch_bfr_spectra(const BfrSpectraArgs& a, hipStream_t s) {
  if (a.cnt <= 0) return hipSuccess;
  if (a.w != kW || a.patch < bfr_spectra_patch(a.s_per_u)) return hipErrorInvalidValue;
  const long long TA = (2LL * a.V + kTile) / kTile, TB = ((a.quarter ? 2LL * a.V : a.V) + kTile) / kTile;
  const long long nblk = TA * TB * (a.quarter ? a.R / 4 : 1);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const size_t lds = sizeof(float2) * a.patch * a.patch;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(bfr_spectra_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bfr_spectra_kernel, dim3(static_cast<unsigned>(nblk), a.cnt), dim3(kTile * kTile), lds, s, a);
  return hipGetLastError();
}

size_t bfr_corr_lds_bytes(int V) {
  return sizeof(float2) * (static_cast<size_t>(kKc) * kLs + static_cast<size_t>(kKc) * kRs +
                           static_cast<size_t>(kBfrDy) * (V + 1));
}

hipError_t launch_bfr_corr(const BfrCorrArgs& a, hipStream_t s) {
  if (a.nA <= 0 || a.nBc <= 0) return hipSuccess;
  const size_t cols = static_cast<size_t>(a.nBc) * a.R * a.Dx;
  if (cols % kCols != 0 || a.nch < 1) return hipErrorInvalidValue;
  const size_t nRT = (a.nA + kRows - 1) / kRows;
  const size_t grid = nRT * (cols / kCols);
  if (grid > 0x7fffffffu) return hipErrorInvalidValue;
  const size_t lds = bfr_corr_lds_bytes(a.V);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(bfr_corr_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bfr_corr_kernel, dim3(static_cast<unsigned>(grid)), dim3(256), lds, s, a);
  return hipGetLastError();
}
