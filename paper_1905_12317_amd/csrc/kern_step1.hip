// Step 1 of the FTK (eq. fbk3) on gfx950 MFMA: FP32, split (bf16 or fp16,
// three products) and FP16 forms.
//
//     Zhat_B[zeta](q) = sum_m conj b_B(k_m; q) P_zeta(m; q),
//     P_zeta(m; q)   = 2 pi w_m G_zeta(k_m) a(k_m; q - l_zeta mod Qa),
//
// for one image, one mode q and every template B, written as a real GEMM:
//   rows    (B, c)      c = 0 real part, c = 1 imaginary part of Zhat
//   K       (m, c')     c' = 0 real part, c' = 1 imaginary part of P
//   columns zeta
// with the template operand R'[(B,c)][(m,c')] = [[br, bi], [-bi, br]] and the
// image operand P[(m,c')][zeta] = (Re P, Im P).  The template operand is
// embedded once per call by tmpl_prep_* in MFMA lane order (and, for the
// split form, split into bf16 hi + lo); a workgroup owns one image, one q
// and a block of zeta, forms P for that q once in LDS, and its waves sweep
// all template blocks.  Modes q = 0 .. Qa/2 are computed (Hermitian
// symmetry of a real inner product); the result is staged as
// zs[pair][q][c][zeta] with Qa/2 + 1 rows of q.
#include <type_traits>

#include "device_common.h"
#include "kernels.h"

using namespace ftkdev;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

namespace {

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// R'[(B,c)][(m,c')] from the template's complex coefficient b = (br, bi)
__device__ __forceinline__ float embed(float2 b, int c, int cp) {
  return c == 0 ? (cp == 0 ? b.x : b.y) : (cp == 0 ? -b.y : b.x);
}

// ---- template operand preparation -------------------------------------

// Template of row tile rt, slot s (0..15).  Plain mode: template rt 16 + s.
// List mode (lists != null): tiles come in groups of nRTk per image of the
// chunk; slot j = (rt % nRTk) 16 + s of image a0 + rt / nRTk is template
// lists[image][j] (j < K), else none (-1).
__device__ __forceinline__ int tile_template(int rt, int s, int nB, const int* __restrict__ lists, int K, int nRTk,
                                             int a0) {
  if (!lists) {
    const int B = rt * 16 + s;
    return B < nB ? B : -1;
  }
  const int img = rt / nRTk;
  const int j = (rt - img * nRTk) * 16 + s;
  if (j >= K) return -1;
  const int B = lists[static_cast<size_t>(a0 + img) * K + j];
  return (B >= 0 && B < nB) ? B : -1;
}

// FP32 form, 32x32x2 MFMA: one K step is one m (k' = 2m + c').
// Layout [q][row tile][m][lane] floats; lane l: row l % 32 -> (B, c), c' = l / 32.
__global__ void tmpl_prep_fp32(const float2* __restrict__ b, float* __restrict__ out, int nB, int nRT, int M,
                               int Qa, int NQ, const int* __restrict__ lists, int K, int nRTk, int a0) {
  const size_t total = static_cast<size_t>(NQ) * nRT * M * 64;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int lane = static_cast<int>(t & 63);
    size_t u = t >> 6;
    const int m = static_cast<int>(u % M);
    u /= M;
    const int rt = static_cast<int>(u % nRT);
    const int q = static_cast<int>(u / nRT);
    const int row = lane & 31;
    const int B = tile_template(rt, row >> 1, nB, lists, K, nRTk, a0);
    float v = 0.f;
    if (B >= 0) v = embed(b[(static_cast<size_t>(B) * Qa + q) * M + m], row & 1, lane >> 5);
    out[t] = v;
  }
}

// Split forms, 32x32x16 MFMA: one K step is 8 m (k' = 16 ks + 8 (l/32) + e).
// Layout [q][row tile][ks][lane][8 hi, 8 lo] of T (bf16, or fp16 with b
// scaled by dscale[1] = 2^e / s_b).
template <class T>
__global__ void tmpl_prep_split(const float2* __restrict__ b, T* __restrict__ out, int nB, int nRT, int M, int Qa,
                                int NQ, const int* __restrict__ lists, int K, int nRTk, int a0,
                                const float* __restrict__ dscale) {
  typedef T v8 __attribute__((ext_vector_type(8)));
  const float sb = dscale ? dscale[1] : 1.f;
  const int nks = M / 8;
  const size_t total = static_cast<size_t>(NQ) * nRT * nks * 64;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int lane = static_cast<int>(t & 63);
    size_t u = t >> 6;
    const int ks = static_cast<int>(u % nks);
    u /= nks;
    const int rt = static_cast<int>(u % nRT);
    const int q = static_cast<int>(u / nRT);
    const int row = lane & 31;
    const int B = tile_template(rt, row >> 1, nB, lists, K, nRTk, a0);
    const int c = row & 1;
    v8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kp = ks * 16 + 8 * (lane >> 5) + e;
      float v = 0.f;
      if (B >= 0) v = embed(b[(static_cast<size_t>(B) * Qa + q) * M + (kp >> 1)], c, kp & 1) * sb;
      const T h = static_cast<T>(v);
      hi[e] = h;
      lo[e] = static_cast<T>(v - static_cast<float>(h));
    }
    v8* o = reinterpret_cast<v8*>(out) + t * 2;
    o[0] = hi;
    o[1] = lo;
  }
}

// FP16 form, 32x32x16 MFMA: one K step is 8 m (k' = 16 ks + 8 (l/32) + e),
// b scaled by 1/s_b.  Layout [q][row tile][ks][lane][8] fp16.
__global__ void tmpl_prep_fp16(const float2* __restrict__ b, _Float16* __restrict__ out, int nB, int nRT, int M,
                               int Qa, int NQ, const int* __restrict__ lists, int K, int nRTk, int a0,
                               const float* __restrict__ dscale) {
  const float sb = dscale[1];
  const int nks = M / 8;
  const size_t total = static_cast<size_t>(NQ) * nRT * nks * 64;
  for (size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int lane = static_cast<int>(t & 63);
    size_t u = t >> 6;
    const int ks = static_cast<int>(u % nks);
    u /= nks;
    const int rt = static_cast<int>(u % nRT);
    const int q = static_cast<int>(u / nRT);
    const int row = lane & 31;
    const int B = tile_template(rt, row >> 1, nB, lists, K, nRTk, a0);
    const int c = row & 1;
    f16x8 h;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kp = ks * 16 + 8 * (lane >> 5) + e;
      float v = 0.f;
      if (B >= 0) v = embed(b[(static_cast<size_t>(B) * Qa + q) * M + (kp >> 1)], c, kp & 1) * sb;
      h[e] = static_cast<_Float16>(v);
    }
    reinterpret_cast<f16x8*>(out)[t] = h;
  }
}

// Fill of the image operand in LDS, U items per thread at a time: the index
// loads (ell) of all U items, then their data loads, then the LDS stores, so
// a batch costs two memory round trips instead of two per item.  Items past
// `total` load a valid item (the last) and store nothing.
template <int U, class FI, class FD, class FS>
__device__ __forceinline__ void batched_fill(int total, FI load_index, FD load_data, FS store) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i0 = tid; i0 < total; i0 += U * nthr) {
    decltype(load_index(0)) ix[U];
#pragma unroll
    for (int u = 0; u < U; ++u) ix[u] = load_index(min(i0 + u * nthr, total - 1));
    decltype(load_data(ix[0], 0)) dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) dv[u] = load_data(ix[u], min(i0 + u * nthr, total - 1));
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * nthr < total) store(dv[u], i0 + u * nthr);
  }
}

// Items of two m (split and FP16 forms): (Pr, Pi) of m and m + 1, the 4
// consecutive k' of one zeta row (M is even, so both m lie in the same half).
struct FillData {
  float4 av;  // a(k_m; row), a(k_{m+1}; row)
  float2 cm;  // the 2 pi w G entries of m, m + 1
};
__device__ __forceinline__ FillData fill_load(const Step1Args& p, const float2* arow, int ell, int i, int MK, int M,
                                              int q, int QH, int Qa, int z0, bool fold) {
  const int z = i / (MK / 2);
  const int m2 = i - z * (MK / 2);
  const bool ny = fold && 2 * m2 >= M;
  const int ml = ny ? m2 - M / 2 : m2;
  int row = (ny ? QH : q) - ell;
  row %= Qa;
  row += (row < 0) ? Qa : 0;
  return FillData{reinterpret_cast<const float4*>(arow + static_cast<size_t>(row) * M)[ml],
                  reinterpret_cast<const float2*>(p.cz + static_cast<size_t>(z0 + z) * M)[ml]};
}
// the 4 values (times scale), multiplied by i in the Nyquist half:
// i (x + i y) = -y + i x
// The products are rounded to FP32 here, in every kernel that inlines this:
// left visible, a conversion of a product to fp16 may be selected as one
// mixed-precision fused instruction (a single rounding of the exact product)
// in one kernel and as a multiply and a conversion (two roundings) in
// another, and the fp16 forms' Step 1 would then depend on the launch shape.
__device__ __forceinline__ void fill_value(const FillData& d, bool ny, float scale, float (&x)[4]) {
  const float c0 = d.cm.x * scale, c1 = d.cm.y * scale;
  x[0] = c0 * d.av.x;
  x[1] = c0 * d.av.y;
  x[2] = c1 * d.av.z;
  x[3] = c1 * d.av.w;
#pragma unroll
  for (int e = 0; e < 4; ++e) asm volatile("" : "+v"(x[e]));
  if (ny) {
    const float t0 = x[0], t2 = x[2];
    x[0] = -x[1];
    x[1] = t0;
    x[2] = -x[3];
    x[3] = t2;
  }
}

// ---- Step 1, FP32 form --------------------------------------------------

// Workgroup b of the 1-D grid.  A group is one (mode slot y, zeta block x
// template part zp); its nA images run on one XCD one after another
// (workgroups are dealt to the 8 XCDs round-robin, so b and b + 8 share an
// XCD), and the group's template operand comes from HBM once and from that
// XCD's L2 for the other images.  Group g = 8 gl + x goes to XCD x; the grid
// holds whole rounds of 8 groups and the padding workgroups exit.
__device__ __forceinline__ int step1_groups(const Step1Args& p, int CT) {
  return (p.Qa / 2 - 1 + CT) * (p.H_pad / p.zblk) * p.tparts;
}
__device__ __forceinline__ bool step1_block(int b, const Step1Args& p, int CT, int& A, int& y, int& zp) {
  const int S = p.Qa / 2 - 1 + CT;
  const int x = b & 7;
  const int s = b >> 3;
  const int gl = s / p.nA;
  A = s - gl * p.nA;
  const int g = 8 * gl + x;
  if (g >= step1_groups(p, CT)) return false;
  y = g % S;
  zp = g / S;
  return true;
}


// Grid: x = image in chunk, y = mode slot, z = zeta block x template part.
// Slots y < CT are the Nyquist fold: slot y covers the 32 zeta of column tile
// y of the block for mode 0 and accumulates Zhat(0) + i Zhat(Qa/2) as one
// GEMM with K = 2 x 2M (the image operand of the second half is i P(Qa/2),
// the template operand that of mode Qa/2).  Slots y >= CT are the modes
// q = y - CT + 1 .. Qa/2 - 1 over the whole block.
// LDS: image operand P[k'][zeta] (k' = 2m + c', zeta contiguous, stride PS).
// BFT: the brute-force-translation contraction instead (zeta is a shift
// delta, H_pad the padded shift count): P_delta(m; q) = 2 pi w_m Ta(k_m; q)
// from the translated coefficients p.ta [image][q = 0 .. Qa/2][delta][m],
// with p.cz[m] = 2 pi w_m and no mode offset.
template <int RT, int CT, bool FOLD, bool BFT>
__device__ __forceinline__ void step1_fp32_tile(const Step1Args& p, float* smem, int A, int q, int z0, int part) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int M = p.M, Qa = p.Qa, QH = Qa / 2;
  constexpr int ZB = 32 * CT;
  constexpr int PS = (ZB % 64 == 0) ? ZB + 32 : ZB;  // row stride == 32 mod 64 words
  constexpr int NP = FOLD ? 2 : 1;
  const int MK = NP * M;
  struct D {
    float2 av;
    float cm;
  };
  auto store = [&](const D& d, int i) {
    const int z = i / MK;
    const int mm = i - z * MK;
    const bool ny = FOLD && mm >= M;
    // i (x + i y) = -y + i x for the Nyquist half
    smem[(2 * mm) * PS + z] = ny ? -d.cm * d.av.y : d.cm * d.av.x;
    smem[(2 * mm + 1) * PS + z] = ny ? d.cm * d.av.x : d.cm * d.av.y;
  };
  if constexpr (BFT) {
    const float2* tq = p.ta + static_cast<size_t>(A) * (QH + 1) * p.H_pad * M;
    batched_fill<8>(
        ZB * MK, [&](int) { return 0; },
        [&](int, int i) {
          const int z = i / MK;
          const int mm = i - z * MK;
          const bool ny = FOLD && mm >= M;
          const int m = ny ? mm - M : mm;
          return D{tq[(static_cast<size_t>(ny ? QH : q) * p.H_pad + z0 + z) * M + m], p.cz[m]};
        },
        store);
  } else {
    const float2* arow = p.a + static_cast<size_t>(A) * Qa * M;
    batched_fill<8>(
        ZB * MK, [&](int i) { return p.ell[z0 + i / MK]; },
        [&](int ell, int i) {
          const int z = i / MK;
          const int mm = i - z * MK;
          const bool ny = FOLD && mm >= M;
          const int m = ny ? mm - M : mm;
          int row = (ny ? QH : q) - ell;
          row %= Qa;
          row += (row < 0) ? Qa : 0;
          return D{arow[static_cast<size_t>(row) * M + m], p.cz[static_cast<size_t>(z0 + z) * M + m]};
        },
        store);
  }
  __syncthreads();
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nRT = (p.nB + 15) / 16;
  const int twoH = 2 * p.H_pad;
  const float* Pb = smem + r * PS + c32;
  float* zbase = static_cast<float*>(p.zs) + static_cast<size_t>(A) * p.nB * QH * twoH + static_cast<size_t>(q) * twoH;
  const size_t img_off = static_cast<size_t>(A) * p.img_tiles;
  const int nw = static_cast<int>(blockDim.x) >> 6;
  for (int rt0 = (part * nw + wave) * RT; rt0 < nRT; rt0 += nw * RT * p.tparts) {
    f32x16 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[i][j] = zero16();
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int qt = pass ? QH : q;  // mode of the template operand
      const float* rq = p.r32 + (static_cast<size_t>(qt) * p.tiles_per_q + img_off) * M * 64 + lane;
      const float* ra[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) ra[i] = rq + static_cast<size_t>(min(rt0 + i, nRT - 1)) * M * 64;
      float an[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) an[i] = ra[i][0];
      const float* Pp = Pb + pass * (2 * M) * PS;
      for (int m = 0; m < M; ++m) {
        float av[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) av[i] = an[i];
        if (m + 1 < M) {
#pragma unroll
          for (int i = 0; i < RT; ++i) an[i] = ra[i][(m + 1) * 64];
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          const float bv = Pp[(2 * m) * PS + j * 32];
#pragma unroll
          for (int i = 0; i < RT; ++i)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv, acc[i][j], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      if (rt0 + i >= nRT) continue;
#pragma unroll
      for (int j = 0; j < CT; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = 8 * (v >> 2) + 4 * r + (v & 3);
          const int B = (rt0 + i) * 16 + (row >> 1);
          if (B < p.nB)
            __builtin_nontemporal_store(acc[i][j][v], zbase + static_cast<size_t>(B) * QH * twoH + (row & 1) * p.H_pad + z0 + j * 32 + c32);
        }
    }
  }
}

template <int RT, int CT, bool BFT>
__global__ void __launch_bounds__(256) step1_fp32_v2(Step1Args p) {
  extern __shared__ float smem[];
  int A, y, zp;
  if (!step1_block(blockIdx.x, p, CT, A, y, zp)) return;
  const int zb = (zp / p.tparts) * (32 * CT);
  const int part = zp % p.tparts;
  if (y < CT)
    step1_fp32_tile<RT, 1, true, BFT>(p, smem, A, 0, zb + 32 * y, part);
  else
    step1_fp32_tile<RT, CT, false, BFT>(p, smem, A, y - CT + 1, zb, part);
}

// ---- Step 1, split forms (bf16 or fp16, three products) -----------------

__device__ __forceinline__ f32x16 mma16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mma16(f16x8 a, f16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
template <class V>
__device__ __forceinline__ f32x16 mfma3(V ahi, V alo, V bhi, V blo, f32x16 c) {
  c = mma16(ahi, bhi, c);
  c = mma16(ahi, blo, c);
  c = mma16(alo, bhi, c);
  return c;
}

// Same work split and Nyquist fold as the FP32 form.  LDS: image operand per
// zeta row: [2 MK hi][2 MK lo] of T + 4 words pad (MK = M, or 2M when
// folding).  The result is split into hi + lo and written in Step 3's chunk
// layout [pair][k' / 32][q][32 hi][32 lo]: lanes j and j + 1 (adjacent zeta)
// trade halves so that the even lane stores the hi pair and the odd lane the
// lo pair as 32-bit words.  T = fp16: the image operand is 2^e P / (s_a
// sg_zeta) (dscale[0] = 2^e / s_a; the 2 pi w G table of the plan is stored
// divided by sg_zeta), the template operand 2^e b / s_b, and the FP32 result
// is multiplied by dscale[3] = 2^e_z before the split (the exponents keep
// every hi and lo a normal fp16 number over the useful range; the scales are
// powers of two, so no rounding is added).
template <class T, int RT, int CT, bool FOLD>
__device__ __forceinline__ void step1_split_tile(const Step1Args& p, float* smem, int A, int q, int z0, int part) {
  typedef T v8 __attribute__((ext_vector_type(8)));
  typedef T v4 __attribute__((ext_vector_type(4)));
  typedef T v2 __attribute__((ext_vector_type(2)));
  constexpr bool kScaled = std::is_same<T, _Float16>::value;
  const float sa = kScaled ? p.dscale[0] : 1.f;
  const float zsc = kScaled ? p.dscale[3] : 1.f;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int M = p.M, Qa = p.Qa, QH = Qa / 2;
  constexpr int ZB = 32 * CT;
  constexpr int NP = FOLD ? 2 : 1;
  const int MK = NP * M;
  const int RW = 2 * MK + 4;  // words per zeta row
  const float2* arow = p.a + static_cast<size_t>(A) * Qa * M;
  // two m per item: (Pr, Pi) of m and m+1 -> 4 consecutive k' (M is even,
  // so both lie in the same half)
  batched_fill<8>(
      ZB * (MK / 2), [&](int i) { return p.ell[z0 + i / (MK / 2)]; },
      [&](int ell, int i) { return fill_load(p, arow, ell, i, MK, M, q, QH, Qa, z0, FOLD); },
      [&](const FillData& d, int i) {
        const int z = i / (MK / 2);
        const int m2 = i - z * (MK / 2);
        float x[4];
        fill_value(d, FOLD && 2 * m2 >= M, sa, x);
        v4 hi, lo;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const T h = static_cast<T>(x[e]);
          hi[e] = h;
          lo[e] = static_cast<T>(x[e] - static_cast<float>(h));
        }
        float* dst = smem + z * RW + 2 * m2;
        *reinterpret_cast<v4*>(dst) = hi;
        *reinterpret_cast<v4*>(dst + MK) = lo;
      });
  __syncthreads();
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nRT = (p.nB + 15) / 16;
  const int nks = M / 8;
  const size_t pair_words = static_cast<size_t>(QH) * 2 * p.H_pad;
  const float* Pb = smem + c32 * RW + 4 * r;
  // word of this lane in a 128-byte (32-word) row: even lanes hi, odd lanes lo
  const int odd = c32 & 1;
  const int wsel = odd ? 16 + (c32 >> 1) : (c32 >> 1);
  uint32_t* zw = static_cast<uint32_t*>(p.zs) + static_cast<size_t>(A) * p.nB * pair_words +
                 static_cast<size_t>(q) * 32 + wsel;
  const size_t img_off = static_cast<size_t>(A) * p.img_tiles;
  const int nw = static_cast<int>(blockDim.x) >> 6;
  for (int rt0 = (part * nw + wave) * RT; rt0 < nRT; rt0 += nw * RT * p.tparts) {
    f32x16 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[i][j] = zero16();
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int qt = pass ? QH : q;
      const v8* rq = reinterpret_cast<const v8*>(p.r16) +
                         ((static_cast<size_t>(qt) * p.tiles_per_q + img_off) * nks * 64 + lane) * 2;
      const v8* ra[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) ra[i] = rq + static_cast<size_t>(min(rt0 + i, nRT - 1)) * nks * 128;
      v8 nhi[RT], nlo[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        nhi[i] = ra[i][0];
        nlo[i] = ra[i][1];
      }
      const float* Pp = Pb + pass * M;  // the Nyquist half starts at k' = 2M (M words)
      for (int ks = 0; ks < nks; ++ks) {
        v8 ahi[RT], alo[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          ahi[i] = nhi[i];
          alo[i] = nlo[i];
        }
        if (ks + 1 < nks) {
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            nhi[i] = ra[i][(ks + 1) * 128];
            nlo[i] = ra[i][(ks + 1) * 128 + 1];
          }
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          const float* prow = Pp + j * 32 * RW + 8 * ks;
          const v8 bhi = *reinterpret_cast<const v8*>(prow);
          const v8 blo = *reinterpret_cast<const v8*>(prow + MK);
#pragma unroll
          for (int i = 0; i < RT; ++i) acc[i][j] = mfma3(ahi[i], alo[i], bhi, blo, acc[i][j]);
        }
      }
    }
    // tiles whose 16 templates all exist store without a per-row test
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int rt = rt0 + i;
      if (rt >= nRT) break;
      // the lane's base address once per tile; each store adds scalar
      // offsets (template row and chunk).  Tiles whose 16 templates all exist
      // store without a row test.
      const int nrows = p.nB - rt * 16 - 2 * r;
      uint32_t* tb = zw + (static_cast<size_t>(rt) * 16 + 2 * r) * pair_words;
      auto store_tile = [&](auto guarded) {
#pragma unroll
        for (int j = 0; j < CT; ++j) {
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const float x = kScaled ? acc[i][j][v] * zsc : acc[i][j][v];
            // hi = T(x), lo = T(x - hi), packed (hi, lo) in one word
            const float xh = static_cast<float>(static_cast<T>(x));
            const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{x, x - xh}, v2));
            // even lane sends its lo half, odd lane its hi half; the even lane
            // stores (hi, hi of the odd lane), the odd lane (lo of the even, lo)
            const uint32_t got = static_cast<uint32_t>(
                __builtin_amdgcn_mov_dpp(static_cast<int>(odd ? w : (w >> 16)), 0xB1, 0xF, 0xF, false));
            const uint32_t word = odd ? ((got & 0xffffu) | (w & 0xffff0000u)) : ((w & 0xffffu) | (got << 16));
            // accumulator row 8 (v / 4) + 4 r + v % 4: template rt 16 + kv + 2 r,
            // part c = v % 2; k' = c H_pad + z0 + 32 j + c32 lies in chunk
            // (c H_pad + z0) / 32 + j
            const int kv = 4 * (v >> 2) + ((v & 3) >> 1);
            const int chunk = ((v & 1) * p.H_pad + z0) / 32 + j;
            // streaming store: the staging is read back once, by Step 3
            if (!decltype(guarded)::value || kv < nrows)
              __builtin_nontemporal_store(word, tb + static_cast<size_t>(kv) * pair_words +
                                                    static_cast<size_t>(chunk) * QH * 32);
          }
        }
      };
      if ((rt + 1) * 16 <= p.nB)
        store_tile(std::false_type{});
      else
        store_tile(std::true_type{});
    }
  }
}

// At least 2 waves per SIMD: left free, the compiler keeps the accumulators
// in AGPRs and copies them all to VGPRs for the split at the end (about 300
// registers, 1 wave per SIMD).
template <class T, int RT, int CT, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 2))) step1_split_v2(Step1Args p) {
  extern __shared__ float smem[];
  int A, y, zp;
  if (!step1_block(blockIdx.x, p, CT, A, y, zp)) return;
  const int zb = (zp / p.tparts) * (32 * CT);
  const int part = zp % p.tparts;
  if (y < CT)
    step1_split_tile<T, RT, 1, true>(p, smem, A, 0, zb + 32 * y, part);
  else
    step1_split_tile<T, RT, CT, false>(p, smem, A, y - CT + 1, zb, part);
}

// ---- Step 1, FP16 form --------------------------------------------------

// Same work split and Nyquist fold as the other forms, one FP16 product per
// term.  The image operand is P / (s_a sg_zeta) (the 2 pi w G table of an
// FP16 plan is stored divided by its per-zeta power of two sg_zeta), the
// template operand b / s_b, both rounded to fp16; accumulation in FP32.
// LDS: per zeta row [2 MK fp16] + 4 words pad.  The result is rounded to
// fp16 and written in Step 3's chunk layout [pair][k' / 64][q][64 fp16]:
// accumulator rows v (real part) and v + 1 (imaginary part) of one template
// are traded between adjacent lanes (adjacent zeta), so that the even lane
// stores the real-part pair and the odd lane the imaginary-part pair, each as
// one 32-bit word.
// Store rows of one wave (FP16 form, plain slots): one template tile's
// values as [template t][part c][zeta] fp16, rows of ZB / 2 words padded to
// ZB / 2 + 4 (the two halves of a wave's rows then fall in different banks).
__host__ __device__ constexpr int fp16_store_row_words(int zb) { return zb / 2 + 4; }
__host__ __device__ constexpr int fp16_store_words(int zb) { return 32 * fp16_store_row_words(zb); }

// Plain slots of the FP16 form: each (template, part) holds ZB consecutive
// k' = c H_pad + z0 + zeta, whole 128-byte staging rows.  The wave's RT
// template tiles from rt0 go through its LDS rows so that 8 lanes store one
// row with 16-byte stores.  zw: the image's staging at mode q.
template <int RT, int CT>
__device__ __forceinline__ void fp16_store_plain(const Step1Args& p, float* smem, const f32x16 (&acc)[RT][CT],
                                                 int rt0, int z0, uint32_t* zw) {
  constexpr int ZB = 32 * CT;
  constexpr int SRW = fp16_store_row_words(ZB);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int odd = c32 & 1;
  const int nRT = (p.nB + 15) / 16;
  const int QH = p.Qa / 2;
  const size_t pair_words = static_cast<size_t>(QH) * p.H_pad;
  // after the image operand (the larger of a plain and a fold slot)
  const int opw = max(p.zblk * (p.M + 4), 32 * (2 * p.M + 4));
  uint32_t* st = reinterpret_cast<uint32_t*>(smem + opw) + wave * fp16_store_words(ZB);
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int rt = rt0 + i;
    if (rt >= nRT) break;
#pragma unroll
    for (int j = 0; j < CT; ++j)
#pragma unroll
      for (int v = 0; v < 16; v += 2) {
        const float xr = acc[i][j][v], xi = acc[i][j][v + 1];
        // even lane: (re of zeta, re of zeta + 1); odd lane: (im of zeta - 1, im of zeta)
        const float got = __builtin_bit_cast(
            float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, odd ? xr : xi), 0xB1, 0xF, 0xF, false));
        f16x2 w;
        w[0] = static_cast<_Float16>(odd ? got : xr);
        w[1] = static_cast<_Float16>(odd ? xi : got);
        const int t = 4 * (v >> 2) + 2 * r + ((v & 3) >> 1);
        st[(2 * t + odd) * SRW + 16 * j + (c32 >> 1)] = __builtin_bit_cast(uint32_t, w);
      }
    wave_sync();
    // 16-byte units u: row (t, c) = u / (ZB / 8), segment u % (ZB / 8)
    constexpr int SEGS = ZB / 8;
#pragma unroll
    for (int k = 0; k < (32 * SEGS) / 64; ++k) {
      const int u = lane + 64 * k;
      const int row = u / SEGS, seg = u - row * SEGS;
      const int t = row >> 1, c = row & 1;
      const int B = rt * 16 + t;
      if (B < p.nB) {
        const int kp = c * p.H_pad + z0 + 8 * seg;
        const float4 val = *reinterpret_cast<const float4*>(st + row * SRW + 4 * seg);
        typedef float v4f __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(v4f{val.x, val.y, val.z, val.w},
                                    reinterpret_cast<v4f*>(zw + static_cast<size_t>(B) * pair_words +
                                                           static_cast<size_t>(kp >> 6) * QH * 32 + ((kp & 63) >> 1)));
      }
    }
    wave_sync();
  }
}

template <int RT, int CT, bool FOLD, int NKS>
__device__ __forceinline__ void step1_fp16_tile(const Step1Args& p, float* smem, int A, int q, int z0, int part) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int M = p.M, Qa = p.Qa, QH = Qa / 2;
  constexpr int ZB = 32 * CT;
  constexpr int NP = FOLD ? 2 : 1;
  const int MK = NP * M;
  const int RW = MK + 4;  // words per zeta row
  const float sa = p.dscale[0];
  const float2* arow = p.a + static_cast<size_t>(A) * Qa * M;
  batched_fill<8>(
      ZB * (MK / 2), [&](int i) { return p.ell[z0 + i / (MK / 2)]; },
      [&](int ell, int i) { return fill_load(p, arow, ell, i, MK, M, q, QH, Qa, z0, FOLD); },
      [&](const FillData& d, int i) {
        const int z = i / (MK / 2);
        const int m2 = i - z * (MK / 2);
        float x[4];
        fill_value(d, FOLD && 2 * m2 >= M, sa, x);
        f16x4 h;
#pragma unroll
        for (int e = 0; e < 4; ++e) h[e] = static_cast<_Float16>(x[e]);
        *reinterpret_cast<f16x4*>(smem + z * RW + 2 * m2) = h;
      });
  __syncthreads();
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nRT = (p.nB + 15) / 16;
  const int nks = M / 8;
  const size_t pair_words = static_cast<size_t>(QH) * p.H_pad;
  const float* Pb = smem + c32 * RW + 4 * r;
  const int odd = c32 & 1;
  uint32_t* zw = static_cast<uint32_t*>(p.zs) + static_cast<size_t>(A) * p.nB * pair_words + static_cast<size_t>(q) * 32;
  const size_t img_off = static_cast<size_t>(A) * p.img_tiles;
  const int nw = static_cast<int>(blockDim.x) >> 6;
  if constexpr (!FOLD && NKS > 0) {
    // Plain slots with nks = NKS: the template operand of the wave's next
    // tiles is loaded during the K loop of the current ones (each K step's
    // registers refilled once its MFMAs have read them) and has landed
    // before the current tiles' stores are issued.  Loads and stores share
    // one completion count per wave, so a load issued after a tile's stores
    // can only be waited for together with them: loading the next operand at
    // the head of its K loop, as the general loop does, holds the matrix
    // cores until the previous stores have reached memory, whereas here the
    // next K loop runs while they drain (n = 128, 64 images x 2048
    // templates: 2.0 -> 1.6 ms per launch).  Past the last tile the loads
    // repeat the last tile (unused).
    const f16x8* rq = reinterpret_cast<const f16x8*>(p.r16) +
                      (static_cast<size_t>(q) * p.tiles_per_q + img_off) * NKS * 64 + lane;
    const int stride = nw * RT * p.tparts;
    int rt0 = (part * nw + wave) * RT;
    if (rt0 >= nRT) return;
    f16x8 ah[RT][NKS];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const f16x8* ra = rq + static_cast<size_t>(min(rt0 + i, nRT - 1)) * NKS * 64;
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) ah[i][ks] = ra[ks * 64];
    }
    // landed before the loop as well: the loop head then has no operand load
    // in flight on either path into it, and waits for none of the stores
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) asm volatile("" ::"v"(ah[i][ks]));
    for (; rt0 < nRT; rt0 += stride) {
      const f16x8* rb[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) rb[i] = rq + static_cast<size_t>(min(rt0 + stride + i, nRT - 1)) * NKS * 64;
      f32x16 acc[RT][CT];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = zero16();
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          const f16x8 bv = *reinterpret_cast<const f16x8*>(Pb + j * 32 * RW + 8 * ks);
#pragma unroll
          for (int i = 0; i < RT; ++i)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[i][ks], bv, acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < RT; ++i) ah[i][ks] = rb[i][ks * 64];
      }
      // the next tiles' operands have landed before this tile's stores
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) asm volatile("" ::"v"(ah[i][ks]));
      fp16_store_plain<RT, CT>(p, smem, acc, rt0, z0, zw);
    }
    return;
  }
  for (int rt0 = (part * nw + wave) * RT; rt0 < nRT; rt0 += nw * RT * p.tparts) {
    f32x16 acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[i][j] = zero16();
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int qt = pass ? QH : q;
      const f16x8* rq = reinterpret_cast<const f16x8*>(p.r16) +
                        (static_cast<size_t>(qt) * p.tiles_per_q + img_off) * nks * 64 + lane;
      const f16x8* ra[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) ra[i] = rq + static_cast<size_t>(min(rt0 + i, nRT - 1)) * nks * 64;
      f16x8 nh[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) nh[i] = ra[i][0];
      const float* Pp = Pb + pass * M;  // the Nyquist half starts at k' = 2M (M words)
      for (int ks = 0; ks < nks; ++ks) {
        f16x8 ah[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) ah[i] = nh[i];
        if (ks + 1 < nks) {
#pragma unroll
          for (int i = 0; i < RT; ++i) nh[i] = ra[i][(ks + 1) * 64];
        }
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          const f16x8 bv = *reinterpret_cast<const f16x8*>(Pp + j * 32 * RW + 8 * ks);
#pragma unroll
          for (int i = 0; i < RT; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[i], bv, acc[i][j], 0, 0, 0);
        }
      }
    }
    // Accumulator row 8 (v / 4) + 4 r + v % 4 is template rt 16 + 4 (v / 4)
    // + 2 r + (v % 4) / 2 (re|im in adjacent rows).
    if constexpr (!FOLD) {
      fp16_store_plain<RT, CT>(p, smem, acc, rt0, z0, zw);
      continue;
    }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int rt = rt0 + i;
      if (rt >= nRT) break;
      const int nrows = p.nB - rt * 16 - 2 * r;  // rows of this lane's template pair that exist
      uint32_t* tb = zw + (static_cast<size_t>(rt) * 16 + 2 * r) * pair_words;
      auto store_tile = [&](auto guarded) {
#pragma unroll
        for (int j = 0; j < CT; ++j) {
          // k' = c H_pad + z0 + 32 j + (c32 & ~1) for the pair this lane stores
          const int kp = odd * p.H_pad + z0 + 32 * j + (c32 & ~1);
          uint32_t* tj = tb + static_cast<size_t>(kp >> 6) * QH * 32 + ((kp & 63) >> 1);
#pragma unroll
          for (int v = 0; v < 16; v += 2) {
            const float xr = acc[i][j][v], xi = acc[i][j][v + 1];
            // even lane sends its imaginary part, odd lane its real part
            const float got = __builtin_bit_cast(
                float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, odd ? xr : xi), 0xB1, 0xF, 0xF, false));
            f16x2 w;
            w[0] = static_cast<_Float16>(odd ? got : xr);
            w[1] = static_cast<_Float16>(odd ? xi : got);
            const int brow = 4 * (v >> 2) + ((v & 3) >> 1);
            if (!decltype(guarded)::value || brow < nrows)
              __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, w), tj + static_cast<size_t>(brow) * pair_words);
          }
        }
      };
      if ((rt + 1) * 16 <= p.nB)
        store_tile(std::false_type{});
      else
        store_tile(std::true_type{});
    }
  }
}

// NKS > 0: the plain slots of plans with M = 8 NKS take the prefetching loop
// (M = 48, 64, 96; at M = 32 it measured no faster, and NKS = 12 needs one
// column tile per workgroup to fit the registers).
template <int RT, int CT, int NKS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) step1_fp16_v2(Step1Args p) {
  extern __shared__ float smem[];
  int A, y, zp;
  if (!step1_block(blockIdx.x, p, CT, A, y, zp)) return;
  const int zb = (zp / p.tparts) * (32 * CT);
  const int part = zp % p.tparts;
  if (y < CT)
    step1_fp16_tile<RT, 1, true, 0>(p, smem, A, 0, zb + 32 * y, part);
  else
    step1_fp16_tile<RT, CT, false, NKS>(p, smem, A, y - CT + 1, zb, part);
}

template <class K>
hipError_t set_lds(K kern, size_t lds) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(lds));
}

}  // namespace

size_t tmpl_prep_tile_bytes(size_t tiles, int M, int Qa, int precision) {
  const size_t NQ = Qa / 2 + 1;
  if (precision == 0) return NQ * tiles * M * 64 * sizeof(float);
  if (precision == 2) return NQ * tiles * (M / 8) * 64 * 16;
  return NQ * tiles * (M / 8) * 64 * 32;
}

size_t tmpl_prep_bytes(int nB, int M, int Qa, int precision) {
  return tmpl_prep_tile_bytes((nB + 15) / 16, M, Qa, precision);
}

hipError_t launch_tmpl_prep(const float2* b, void* out, int nB, int M, int Qa, int precision, const float* dscale,
                            hipStream_t s) {
  return launch_tmpl_prep_lists(b, out, nB, M, Qa, precision, dscale, nullptr, 0, 0, 0, s);
}

hipError_t launch_tmpl_prep_lists(const float2* b, void* out, int nB, int M, int Qa, int precision,
                                  const float* dscale, const int* lists, int K, int na, int a0, hipStream_t s) {
  if (nB <= 0 || (lists && (K <= 0 || na <= 0))) return hipSuccess;
  if ((precision == 2 || precision == 3) && !dscale) return hipErrorInvalidValue;
  const int nRTk = lists ? (K + 15) / 16 : 0;
  const int nRT = lists ? na * nRTk : (nB + 15) / 16;
  const int NQ = Qa / 2 + 1;
  const size_t total = static_cast<size_t>(NQ) * nRT * (precision == 0 ? M : M / 8) * 64;
  const int blocks = static_cast<int>(std::min<size_t>((total + 255) / 256, 65536));
  if (precision == 0)
    hipLaunchKernelGGL(tmpl_prep_fp32, dim3(blocks), dim3(256), 0, s, b, static_cast<float*>(out), nB, nRT, M, Qa,
                       NQ, lists, K, nRTk, a0);
  else if (precision == 2)
    hipLaunchKernelGGL(tmpl_prep_fp16, dim3(blocks), dim3(256), 0, s, b, static_cast<_Float16*>(out), nB, nRT, M,
                       Qa, NQ, lists, K, nRTk, a0, dscale);
  else if (precision == 3)
    hipLaunchKernelGGL(tmpl_prep_split<_Float16>, dim3(blocks), dim3(256), 0, s, b, static_cast<_Float16*>(out), nB,
                       nRT, M, Qa, NQ, lists, K, nRTk, a0, dscale);
  else
    hipLaunchKernelGGL(tmpl_prep_split<__bf16>, dim3(blocks), dim3(256), 0, s, b, static_cast<__bf16*>(out), nB,
                       nRT, M, Qa, NQ, lists, K, nRTk, a0, nullptr);
  return hipGetLastError();
}

size_t step1_v2_lds_bytes(int M, int zb, int precision) {
  // the larger of a plain slot (zb zeta, K = 2M) and a fold slot (32 zeta, K = 4M)
  size_t plain, fold;
  if (precision == 0) {
    const int PS = (zb % 64 == 0) ? zb + 32 : zb;
    plain = sizeof(float) * 2 * M * PS;
    fold = sizeof(float) * 4 * M * 32;
  } else if (precision == 2) {
    plain = sizeof(float) * zb * (M + 4);
    fold = sizeof(float) * 32 * (2 * M + 4);
    // plus the store rows of the 4 waves (fp16_store_words each)
    return (plain > fold ? plain : fold) + sizeof(float) * 4 * fp16_store_words(zb);
  } else {
    plain = sizeof(float) * zb * (2 * M + 4);
    fold = sizeof(float) * 32 * (4 * M + 4);
  }
  return plain > fold ? plain : fold;
}

// split form: template row tiles per wave and waves per workgroup (per-image
// lists of at most 16 templates have one tile per image: one per wave)
constexpr int kBf16RT = 2, kBf16NW = 4;

hipError_t launch_step1_v2(const Step1Args& a, int precision, hipStream_t s) {
  if (a.nA <= 0 || a.nB <= 0) return hipSuccess;
  const int CT = a.zblk / 32;
  const int QH = a.Qa / 2;
  // QH - 1 plain modes and CT slots of the Nyquist fold per zeta block and
  // template part; nA workgroups per group, whole rounds of 8 groups
  const size_t groups = static_cast<size_t>(QH - 1 + CT) * (a.H_pad / a.zblk) * a.tparts;
  const size_t nwg = 8 * static_cast<size_t>(a.nA) * ((groups + 7) / 8);
  if (nwg > 0x7fffffffull) return hipErrorInvalidConfiguration;
  const dim3 grid(static_cast<unsigned>(nwg));
  const size_t lds = step1_v2_lds_bytes(a.M, a.zblk, precision);
  hipError_t e;
  if (precision == 0) {
#define FTK_S1(ct)                                              \
  case ct: {                                                     \
    auto k = step1_fp32_v2<2, ct, false>;                       \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;          \
    hipLaunchKernelGGL(k, grid, dim3(256), lds, s, a);          \
    break;                                                       \
  }
    switch (CT) {
      FTK_S1(2)
      FTK_S1(4)
      default: return hipErrorInvalidValue;
    }
#undef FTK_S1
  } else if (precision == 2) {
    if (!a.dscale) return hipErrorInvalidValue;
#define FTK_S1(ct)                                              \
  case ct: {                                                     \
    auto k = a.M == 64   ? step1_fp16_v2<2, ct, 8>                                      \
             : a.M == 48 ? step1_fp16_v2<2, ct, 6>                                      \
             : a.M == 96 ? step1_fp16_v2<2, ct, (ct == 2 ? 12 : 0)>                     \
                         : step1_fp16_v2<2, ct, 0>;                                     \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;          \
    hipLaunchKernelGGL(k, grid, dim3(256), lds, s, a);          \
    break;                                                       \
  }
    switch (CT) {
      FTK_S1(2)
      FTK_S1(4)
      default: return hipErrorInvalidValue;
    }
#undef FTK_S1
  } else if (precision == 3) {
    if (!a.dscale) return hipErrorInvalidValue;
#define FTK_S1(ct)                                                        \
  case ct: {                                                               \
    auto k = a.img_tiles == 1 ? step1_split_v2<_Float16, 1, ct, kBf16NW>                 \
                              : step1_split_v2<_Float16, kBf16RT, ct, kBf16NW>;          \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;                    \
    hipLaunchKernelGGL(k, grid, dim3(64 * kBf16NW), lds, s, a);           \
    break;                                                                 \
  }
    switch (CT) {
      FTK_S1(2)
      FTK_S1(4)
      default: return hipErrorInvalidValue;
    }
#undef FTK_S1
  } else {
#define FTK_S1(ct)                                                        \
  case ct: {                                                               \
    auto k = a.img_tiles == 1 ? step1_split_v2<__bf16, 1, ct, kBf16NW>                 \
                              : step1_split_v2<__bf16, kBf16RT, ct, kBf16NW>;          \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;                    \
    hipLaunchKernelGGL(k, grid, dim3(64 * kBf16NW), lds, s, a);           \
    break;                                                                 \
  }
    switch (CT) {
      FTK_S1(2)
      FTK_S1(4)
      default: return hipErrorInvalidValue;
    }
#undef FTK_S1
  }
  return hipGetLastError();
}

hipError_t launch_step1_bft(const Step1Args& a, hipStream_t s) {
  if (a.nA <= 0 || a.nB <= 0) return hipSuccess;
  if (!a.ta) return hipErrorInvalidValue;
  const int CT = a.zblk / 32;
  const int QH = a.Qa / 2;
  const size_t groups = static_cast<size_t>(QH - 1 + CT) * (a.H_pad / a.zblk) * a.tparts;
  const size_t nwg = 8 * static_cast<size_t>(a.nA) * ((groups + 7) / 8);
  if (nwg > 0x7fffffffull) return hipErrorInvalidConfiguration;
  const dim3 grid(static_cast<unsigned>(nwg));
  const size_t lds = step1_v2_lds_bytes(a.M, a.zblk, 0);
  hipError_t e;
#define FTK_S1(ct)                                              \
  case ct: {                                                     \
    auto k = step1_fp32_v2<2, ct, true>;                        \
    if ((e = set_lds(k, lds)) != hipSuccess) return e;          \
    hipLaunchKernelGGL(k, grid, dim3(256), lds, s, a);          \
    break;                                                       \
  }
  switch (CT) {
    FTK_S1(1)
    FTK_S1(2)
    FTK_S1(4)
    default: return hipErrorInvalidValue;
  }
#undef FTK_S1
  return hipGetLastError();
}
