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
typedef float float2_v __attribute__((ext_vector_type(2)));

namespace {

__device__ __forceinline__ f32x16 zero16() {
  f32x16 z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

// The K loop of Step 3 for one pair and one shift block: Zhat chunks staged
// through LDS (two buffers of QH rows at `region`), one FP16 MFMA per term,
// accumulators acc[ct] of the 32 x 32 tile (rows 2 dl + c of the wave's 16
// shifts, columns q = 32 ct + lane % 32).  The first chunk is in buffer 0
// and visible to the block on entry (fp16_first_chunk); ends after the last
// chunk's MFMAs (no barrier).  With next_pair >= 0 (PREF only), the last
// chunk's prefetch fetches the first chunk of next_pair instead and stores
// it into buffer 0 after its MFMAs: visible after the caller's next barrier.
// PREF: the block has enough threads to hold a whole chunk in MAXF4 float4
// per thread, and the next chunk is prefetched through registers while the
// current one is multiplied; otherwise each chunk is fetched after the MFMAs
// of the previous one.
// The first Zhat chunk of `pair` (QH rows of 128 bytes) into LDS buffer 0.
template <int CTQ>
__device__ __forceinline__ void fp16_first_chunk(const Step3Args& p, float* region, int pair) {
  constexpr int QH = 32 * CTQ;
  const int nf4 = QH * 8;
  const float4* zsp = static_cast<const float4*>(p.zs) + static_cast<size_t>(pair) * QH * (p.H_pad / 4);
  for (int t = threadIdx.x; t < nf4; t += blockDim.x)
    *reinterpret_cast<float4*>(region + (t >> 3) * 36 + (t & 7) * 4) = load_stream(zsp + t);
}

template <int CTQ, bool PREF>
__device__ __forceinline__ void fp16_kloop(const Step3Args& p, float* region, int pair, int d0, bool active,
                                           f32x16 (&acc)[CTQ], int next_pair) {
  constexpr int QH = 32 * CTQ;
  constexpr int KC = 64;     // k' per staged chunk (4 MFMA K steps)
  constexpr int KS = KC / 16;
  constexpr int ROWW = 36;   // LDS words per q row: 32 data, 4 pad
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int r = lane >> 5;
  const int c32 = lane & 31;
  const int nk = 2 * p.H_pad;
  const int nks = nk / 16;
  // this pair's chunks of Zhat: chunk c is QH rows of 128 bytes, 8 float4 per
  // row, contiguous
  const float4* zsp = static_cast<const float4*>(p.zs) + static_cast<size_t>(pair) * QH * (nk / 8);
  const int buf_words = QH * ROWW;
  const int nthr = blockDim.x;
  constexpr int MAXF4 = 2;
  const int nf4 = QH * 8;
  auto fetch = [&](int kc, int t) { return load_stream(zsp + static_cast<size_t>(kc / KC) * nf4 + t); };
  const float4* znext =
      static_cast<const float4*>(p.zs) + static_cast<size_t>(next_pair < 0 ? pair : next_pair) * QH * (nk / 8);
  // unit t = 8 q + u of a chunk goes to words 4 u .. 4 u + 3 of LDS row q
  auto put = [&](int buf, int t, float4 v) {
    *reinterpret_cast<float4*>(region + buf * buf_words + (t >> 3) * ROWW + (t & 7) * 4) = v;
  };
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) acc[ct] = zero16();
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
  // One chunk: the MFMAs on LDS buffer (kc / KC) % 2, then the panel
  // operands of the next chunk are loaded (one set of registers: the freed
  // registers let all CTQ Zhat fragments of a K step be read before its
  // MFMAs) and the next chunk is stored into the other buffer.
  auto chunk = [&](int kc, f16x8 (&y)[KS]) {
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
    __builtin_amdgcn_sched_barrier(0);
    if (active) {
      const float* Zb = region + cur * buf_words + c32 * ROWW + 4 * r;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        f16x8 b[CTQ];
#pragma unroll
        for (int ct = 0; ct < CTQ; ++ct) b[ct] = *reinterpret_cast<const f16x8*>(Zb + ct * 32 * ROWW + 8 * s);
#pragma unroll
        for (int ct = 0; ct < CTQ; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(y[s], b[ct], acc[ct], 0, 0, 0);
      }
    }
    load_y(kc + KC, y);
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
  f16x8 y[KS];
  load_y(0, y);
  // nk / KC is even (H_pad is a multiple of 64): the last chunk is in buffer 1
  for (int kc = 0; kc < nk; kc += KC) chunk(kc, y);
}

template <int CTQ, int MAXT, bool PREF>
__global__ void __launch_bounds__(MAXT) step3_fp16(Step3Args p) {
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
  fp16_first_chunk<CTQ>(p, region, pair);
  __syncthreads();
  f32x16 acc[CTQ];
  fp16_kloop<CTQ, PREF>(p, region, pair, d0, active, acc, -1);
  __syncthreads();
  if (!active) return;
  float2* T = reinterpret_cast<float2*>(region) + wave * (epilogue_lds_bytes_per_wave() / sizeof(float2));
  step3_epilogue_reg<CTQ>(p, acc, pair, d0, T, twl, lane);
}

// ---- rotation transform on MFMA (Qa <= 256) --------------------------------
//
// The Qa real outputs of a shift are a real linear map of the packed modes
// P(q) = Xhat(q), q = 0 .. QH - 1 (P(0) = Xhat(0) + i Xhat(QH)):
//   X(r) = Re P(0) + (-1)^r Im P(0)
//          + sum_{q >= 1} 2 (Re P(q) cos(2 pi q r / Qa) + Im P(q) sin(2 pi q r / Qa)).
// Split by the parity of q, X(r) = E(r) + O(r) and X(r + QH) = E(r) - O(r)
// for r < QH (the odd-q terms change sign under r -> r + QH, the even ones
// and the Nyquist term do not).  E and O are two real products
//   E[r][dl] = sum_k T_E[r][k] V_E[k][dl],  O likewise,
// with k = 2 m + c over the modes q = 2 m (E) or 2 m + 1 (O), c = 0 real and
// 1 imaginary part: each is a (QH x QH) by (QH x 16 shifts) product, done
// with v_mfma_f32_16x16x32_f16 (fp16 operands, FP32 accumulation).  The
// tables T_E and T_O (fp16, built on the host, laid out as the MFMA's
// A-operand fragments: [E/O][row tile t][K step s][lane][8]) stay in LDS for
// the whole kernel, which loops over its pairs (one workgroup per CU).
//
// 16x16x32 operand layouts: A lane l holds A[l % 16][8 (l / 16) + e],
// B lane l holds B[8 (l / 16) + e][l % 16], e = 0 .. 7; the result lane l
// holds D[4 (l / 16) + v][l % 16], v = 0 .. 3.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int rot_row_words(int QH) { return QH / 2 + 4; }  // transpose row: QH/2 words + pad

template <int CTQ>
__device__ __forceinline__ void rot_epilogue(const Step3Args& p, f32x16 (&acc)[CTQ], int pair, int d0,
                                             const float4* __restrict__ tbl, uint32_t* sc, int lane) {
  constexpr int QH = 32 * CTQ;
  constexpr int Qa = 2 * QH;
  constexpr int NT = QH / 16;  // row tiles (16 rotations each)
  constexpr int NS = QH / 32;  // K steps of 32
  constexpr int RS = rot_row_words(QH);
  const int jj = lane & 31;
  const int hh = lane >> 5;
  // (1) fp16 (re, im) pairs: acc rows 2 dl + c, register v = 2 g + c holds
  // shift dl = 4 (g / 2) + 2 hh + g % 2 of column q = 32 ct + jj
  uint32_t h2[CTQ][8];
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct)
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
      const f16x2 v = __builtin_convertvector((float2_v{acc[ct][2 * g], acc[ct][2 * g + 1]}), f16x2);
      h2[ct][g] = __builtin_bit_cast(uint32_t, v);
    }
  // (2) transpose through this wave's LDS rows: row dl holds words m =
  // 0 .. QH/2 - 1, the (re, im) of mode 2 m + parity; even columns first
  f16x8 BE[NS], BO[NS];
  uint32_t* const wbase = sc + 2 * hh * RS + (jj >> 1);            // + compile-time offsets
  const uint32_t* const rbase = sc + (lane & 15) * RS + 4 * (lane >> 4);
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    if ((jj & 1) == par) {
#pragma unroll
      for (int ct = 0; ct < CTQ; ++ct)
#pragma unroll
        for (int g = 0; g < 8; ++g) wbase[(4 * (g >> 1) + (g & 1)) * RS + 16 * ct] = h2[ct][g];
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const f16x8 v = *reinterpret_cast<const f16x8*>(rbase + 16 * s);
      if (par == 0)
        BE[s] = v;
      else
        BO[s] = v;
    }
    wave_sync();
  }
  // (3) 16 rotations per tile: E and O products, X(r) = E + O and
  // X(r + QH) = E - O; per lane one shift, rotations r = 16 t + 4 (l / 16) + v
  const int dl = lane & 15;
  const int delta = d0 + dl;
  const bool valid = delta < p.N;
  const int r4 = 4 * (lane >> 4);
  float* xr = (p.X && valid) ? p.X + (static_cast<size_t>(pair) * p.N + delta) * Qa + r4 : nullptr;
  const float xs = (xr && p.xscale) ? *p.xscale : 1.f;
  const f16x8* tb = reinterpret_cast<const f16x8*>(tbl) + lane;
  float bv0 = -__builtin_inff(), bv1 = -__builtin_inff();
  int bs0 = -1, bs1 = -1;  // step 4 t + v of the best in each half
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    f32x4 dE = {0.f, 0.f, 0.f, 0.f}, dO = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      dE = __builtin_amdgcn_mfma_f32_16x16x32_f16(tb[64 * (t * NS + s)], BE[s], dE, 0, 0, 0);
      dO = __builtin_amdgcn_mfma_f32_16x16x32_f16(tb[64 * ((NT + t) * NS + s)], BO[s], dO, 0, 0, 0);
    }
    f32x4 x0, x1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      x0[v] = dE[v] + dO[v];
      x1[v] = dE[v] - dO[v];
      // increasing r within each half: a later equal value never replaces
      // (the lowest index wins ties); NaN never compares greater
      if (x0[v] > bv0) {
        bv0 = x0[v];
        bs0 = 4 * t + v;
      }
      if (x1[v] > bv1) {
        bv1 = x1[v];
        bs1 = 4 * t + v;
      }
    }
    if (xr) {
      *reinterpret_cast<float4*>(xr + 16 * t) = make_float4(x0[0] * xs, x0[1] * xs, x0[2] * xs, x0[3] * xs);
      *reinterpret_cast<float4*>(xr + QH + 16 * t) = make_float4(x1[0] * xs, x1[1] * xs, x1[2] * xs, x1[3] * xs);
    }
  }
  // the lane's best: the first half wins ties (lower index)
  const bool take1 = bs1 >= 0 && (bs0 < 0 || bv1 > bv0);
  const int bs = take1 ? bs1 : bs0;
  float bv = take1 ? bv1 : bv0;
  uint32_t bi = 0xffffffffu;
  if (valid && bs >= 0)
    bi = static_cast<uint32_t>(delta) * Qa + (take1 ? QH : 0) + 16 * (bs >> 2) + r4 + (bs & 3);
  else
    bv = -__builtin_inff();
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const uint32_t oi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(bi), off));
    ep_better(bv, bi, ov, oi);
  }
  if (lane == 0 && bi != 0xffffffffu) atomicMax(p.keys + pair, pose_key(bv, bi));
}

// SEP: the transpose rows have LDS of their own after the Zhat buffers (the
// next pair's first chunk is then stored during the last chunk of the
// current one); otherwise they reuse the Zhat buffers.
template <int CTQ, bool PREF, bool SEP>
__global__ void __launch_bounds__(1024) step3_fp16_rot(Step3Args p) {
  extern __shared__ float smem[];
  constexpr int QH = 32 * CTQ;
  constexpr int NFRAG = 2 * (QH / 16) * (QH / 32);  // 1 KB each
  constexpr int RS = rot_row_words(QH);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  float4* tbl = reinterpret_cast<float4*>(smem);
  const float4* tsrc = static_cast<const float4*>(p.rot16);
  for (int i = tid; i < NFRAG * 64; i += blockDim.x) tbl[i] = tsrc[i];
  float* region = smem + NFRAG * 256;
  uint32_t* sc = reinterpret_cast<uint32_t*>(region + (SEP ? 2 * QH * 36 : 0)) + wave * 16 * RS;
  const int total = p.pairs * p.nblk;
  int b = blockIdx.x;
  if (b >= total) return;
  int pair, yb;
  step3_block(b, p.nblk, p.pairs, pair, yb);
  fp16_first_chunk<CTQ>(p, region, pair);
  __syncthreads();
  for (;;) {
    const int d0 = (yb * p.nwaves + wave) * 16;
    const bool active = d0 < p.N;
    const int bn = b + gridDim.x;
    int pn = 0, ybn = 0;
    if (bn < total) step3_block(bn, p.nblk, p.pairs, pn, ybn);
    constexpr bool early = SEP && PREF;  // next first chunk stored inside the K loop
    f32x16 acc[CTQ];
    fp16_kloop<CTQ, PREF>(p, region, pair, d0, active, acc, (early && bn < total) ? pn : -1);
    // every wave is past the Zhat buffers (the transposes may reuse them),
    // and the next pair's first chunk is visible
    __syncthreads();
    if (active) rot_epilogue<CTQ>(p, acc, pair, d0, tbl, sc, tid & 63);
    if (bn >= total) break;
    if (!early) {
      __syncthreads();  // transposes done before buffer 0 is written again
      fp16_first_chunk<CTQ>(p, region, pn);
      __syncthreads();
    }
    b = bn;
    pair = pn;
    yb = ybn;
  }
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

// s[2], s[3] = 2^e_data / s_a, 2^e_data / s_b; s[4] = s_a s_b s_y 2^e_x;
// s[5] = 2^e_z (all exact powers of two)
__global__ void scales_finalize(float* s, float s_y, int e_data, int e_x, int e_z) {
  if (threadIdx.x != 0) return;
  const float sa = pow2_at_or_above(__uint_as_float(reinterpret_cast<unsigned*>(s)[0]));
  const float sb = pow2_at_or_above(__uint_as_float(reinterpret_cast<unsigned*>(s)[1]));
  s[2] = ldexpf(1.f / sa, e_data);
  s[3] = ldexpf(1.f / sb, e_data);
  s[4] = ldexpf(sa * sb * s_y, e_x);
  s[5] = ldexpf(1.f, e_z);
}

}  // namespace

size_t step3_fp16_lds_bytes(int Qa, int nwaves) {
  const size_t QH = Qa / 2;
  const size_t k = sizeof(float) * 2 * QH * 36;
  const size_t e = static_cast<size_t>(nwaves) * epilogue_lds_bytes_per_wave();
  return sizeof(float2) * Qa + (k > e ? k : e);
}

size_t rot16_table_bytes(int Qa) {
  const size_t QH = Qa / 2;
  return (Qa % 64 == 0 && Qa <= 256) ? 2 * (QH / 16) * (QH / 32) * 1024 : 0;
}

// LDS of the MFMA-transform kernel: the tables, then the Zhat buffers and the
// transpose rows, side by side where they fit (sep), else overlapping
static size_t rot_lds(int Qa, int nwaves, bool sep) {
  const size_t QH = Qa / 2;
  const size_t k = sizeof(float) * 2 * QH * 36;
  const size_t e = sizeof(uint32_t) * static_cast<size_t>(nwaves) * 16 * rot_row_words(static_cast<int>(QH));
  return rot16_table_bytes(Qa) + (sep ? k + e : (k > e ? k : e));
}
constexpr size_t kRotLdsLimit = 160 * 1024;

size_t step3_fp16_rot_lds_bytes(int Qa, int nwaves) {
  const size_t sep = rot_lds(Qa, nwaves, true);
  return sep <= kRotLdsLimit ? sep : rot_lds(Qa, nwaves, false);
}

namespace {

int device_cus() {
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

}  // namespace

template <int CTQ, int MAXT>
static hipError_t launch_step3_fp16_t(const Step3Args& a0, hipStream_t s) {
  Step3Args a = a0;
  const int per_blk = 16 * a.nwaves;
  a.nblk = (a.N + per_blk - 1) / per_blk;
  const size_t nwg = static_cast<size_t>(a.pairs) * a.nblk;
  if (nwg * 64 * a.nwaves > 0xffffffffull) return hipErrorInvalidConfiguration;
  const int nf4 = 32 * CTQ * 8, nthr = 64 * a.nwaves;
  const bool pref = (nf4 + nthr - 1) / nthr <= 2;
  if constexpr (CTQ <= 4) {
    if (a.rot16) {
      // one workgroup per CU, looping over its pairs' shift blocks
      const bool sep = rot_lds(a.Qa, a.nwaves, true) <= kRotLdsLimit;
      const size_t lds = rot_lds(a.Qa, a.nwaves, sep);
      auto kern = pref ? (sep ? step3_fp16_rot<CTQ, true, true> : step3_fp16_rot<CTQ, true, false>)
                       : (sep ? step3_fp16_rot<CTQ, false, true> : step3_fp16_rot<CTQ, false, false>);
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
      if (e != hipSuccess) return e;
      const unsigned grid = static_cast<unsigned>(std::min<size_t>(nwg, static_cast<size_t>(device_cus())));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(nthr), lds, s, a);
      return hipGetLastError();
    }
  }
  const dim3 grid(static_cast<unsigned>(nwg));
  size_t lds = step3_fp16_lds_bytes(a.Qa, a.nwaves);
  auto kern = pref ? step3_fp16<CTQ, MAXT, true> : step3_fp16<CTQ, MAXT, false>;
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
                              float* scales, int e_data, int e_x, int e_z, hipStream_t s) {
  unsigned* u = reinterpret_cast<unsigned*>(scales);
  hipLaunchKernelGGL(scales_init, dim3(1), dim3(64), 0, s, u);
  const int ga = static_cast<int>(std::min<size_t>((a_count + 255) / 256, 2048));
  const int gb = static_cast<int>(std::min<size_t>((b_count + 255) / 256, 2048));
  if (a_count) hipLaunchKernelGGL(absmax_kernel, dim3(ga), dim3(256), 0, s, a, a_count, u);
  if (b_count) hipLaunchKernelGGL(absmax_kernel, dim3(gb), dim3(256), 0, s, b, b_count, u + 1);
  hipLaunchKernelGGL(scales_finalize, dim3(1), dim3(64), 0, s, scales, s_y, e_data, e_x, e_z);
  return hipGetLastError();
}
