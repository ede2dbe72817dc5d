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

// ---- shift contraction and rotation transform on MFMA (Qa <= 256) -------
//
// The Qa real outputs of a shift are a real linear map of the packed modes
// P(q) = Xhat(q), q = 0 .. QH - 1 (P(0) = Xhat(0) + i Xhat(QH)):
//   X(r) = Re P(0) + (-1)^r Im P(0)
//          + sum_{q >= 1} 2 (Re P(q) cos(2 pi q r / Qa) + Im P(q) sin(2 pi q r / Qa)).
// Split by the parity of q, X(r) = E(r) + O(r) and X(r + QH) = E(r) - O(r)
// for r < QH (the odd-q terms change sign under r -> r + QH, the even ones
// and the Nyquist term do not).  E and O are two real products with the
// fp16 tables T_E, T_O (QH rotations by QH (mode, re|im) entries each),
// v_mfma_f32_16x16x32_f16, FP32 accumulation.
//
// The shift contraction runs transposed, D[q][j] = sum_k' Zhat[q][k'] Y[k'][j]
// (v_mfma_f32_32x32x16_f16, the staged Zhat fragment as A, the shift panel
// as B), with column j = 16 c + dl of a tile of 16 shifts (c = 0 real, 1
// imaginary part).  Lane l then holds column l % 32 and, in register v of
// column tile ct, the mode q = 32 ct + 8 (v / 4) + 4 (l / 32) + v % 4.  That
// is the B operand of the 16x16x32 MFMA (lane l holds column n = l % 16 =
// dl and k = 8 (l / 16) + e, e = 0 .. 7) once the rotation's K index of lane
// group g = l / 16 is read as c = g % 2 and q = 32 ct + 8 (e / 2) +
// 4 (g / 2) + 2 (e % 2) + parity, i.e. register v = 2 e + parity: the
// tables are built in that K order (host), and the contraction's results
// feed the rotation MFMAs with no lane exchange and no LDS transpose.
//
// Each wave owns two tiles of 16 shifts: every Zhat fragment read from LDS
// feeds two contraction MFMAs and every table fragment two rotation MFMAs.
// One workgroup of 8 waves per CU loops over its (pair, shift block) units;
// the tables stay in LDS for the whole kernel, and the next pair's first
// Zhat chunk is stored during the last chunk of the current one.
//
// 16x16x32 operand layouts: A lane l holds A[l % 16][8 (l / 16) + e],
// B lane l holds B[8 (l / 16) + e][l % 16]; the result lane l holds
// D[4 (l / 16) + v][l % 16], v = 0 .. 3.
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMtWaves = 8;        // waves per workgroup of the two-tile kernel
constexpr int kMtCompute = 7;      // waves 0..6 compute; wave 7 stages Zhat
constexpr int kMtTiles = 2;        // shift tiles (16 shifts each) per compute wave
constexpr int kMtBlockShifts = 16 * kMtCompute * kMtTiles;  // shifts of one shift block

// Zhat staging of the two-tile kernel.  The workgroup walks a stream of
// chunks: for each of its (pair, shift block) units in turn, the pair's Zhat
// in chunks of 64 k' (QH rows of 128 bytes, 4 MFMA K steps).  Wave 7 (the
// stager) loads the stream from HBM into registers three chunks ahead and
// stores chunk g into LDS buffer g % kMtRing as soon as every compute wave
// has finished chunk g - kMtRing; it then publishes ready[g % kMtRing] =
// g + 1.  A compute wave waits for that value before it reads chunk g and
// publishes prog[wave] = g + 1 once its reads of chunk g are done.  There is
// no workgroup barrier in the loop: the stager runs ahead of the compute
// waves by up to kMtRing chunks, the compute waves drift freely (one wave's
// rotation epilogue overlaps another's contraction on the same SIMD), and the
// compute waves issue no Zhat loads, so their shift-panel loads never wait
// behind an HBM load.
constexpr int kMtRing = 5;

template <int CTQ>
struct MtStage {
  static constexpr int QH = 32 * CTQ;
  static constexpr int ROWW = 36;       // LDS words per q row: 32 data, 4 pad
  static constexpr int BUF = QH * ROWW;  // words of one buffer
  static constexpr int NF4 = QH * 8;     // float4 of one chunk
  static constexpr int PER = NF4 / 64;   // float4 per stager lane
  static __device__ __forceinline__ float* at(float* region, int buf, int t) {
    return region + buf * BUF + (t >> 3) * ROWW + (t & 7) * 4;
  }
  // flags after the ring: ready[kMtRing], prog[kMtCompute], abort
  static __device__ __forceinline__ int* flags(float* region) {
    return reinterpret_cast<int*>(region + kMtRing * BUF);
  }
};
constexpr int kMtFlagWords = kMtRing + kMtCompute + 1;

// Wait (workgroup-scope acquire) until *addr >= want.  Bounded: after about
// 2^20 polls the wait gives up and sets *abort, which ends every later wait
// at once (the results are then wrong, but no wave can hang).
__device__ __forceinline__ void mt_wait_ge(int* addr, int want, int* abort) {
  for (int it = 0; it < (1 << 20); ++it) {
    if (__hip_atomic_load(addr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= want) return;
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0) return;
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Workgroup-scope release store of v (one lane), after this wave's LDS
// accesses so far.
__device__ __forceinline__ void mt_publish(int* addr, int v) {
  if ((threadIdx.x & 63) == 0) __hip_atomic_store(addr, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Stream position g -> the Zhat chunk it stages (float4 pointer).
__device__ __forceinline__ const float4* mt_chunk_src(const Step3Args& p, int g, int nch, int QH) {
  const int unit = blockIdx.x + (g / nch) * gridDim.x;
  int pair, yb;
  step3_block(unit, p.nblk, p.pairs, pair, yb);
  return static_cast<const float4*>(p.zs) + (static_cast<size_t>(pair) * (2 * p.H_pad / 64) + g % nch) * QH * 8;
}

// The stager: T chunks in the stream, three register sets of PER float4.
template <int CTQ>
__device__ __forceinline__ void mt_stager(const Step3Args& p, float* region, int T, int nch) {
  using S = MtStage<CTQ>;
  const int lane = threadIdx.x & 63;
  int* ready = S::flags(region);
  int* prog = ready + kMtRing;
  int* abort = prog + kMtCompute;
  float4 r0[S::PER], r1[S::PER], r2[S::PER];
  auto issue = [&](float4 (&r)[S::PER], int g) {
    const float4* src = mt_chunk_src(p, min(g, T - 1), nch, S::QH) + lane;  // past the end: reloads the last
#pragma unroll
    for (int k = 0; k < S::PER; ++k) r[k] = load_stream(src + 64 * k);
  };
  auto step = [&](float4 (&r)[S::PER], int g) {
    // buffer g % kMtRing is free once every compute wave has finished chunk g - kMtRing
    if (g >= kMtRing) {
      for (int w = 0; w < kMtCompute; ++w) mt_wait_ge(prog + w, g - kMtRing + 1, abort);
    }
    const int buf = g % kMtRing;
#pragma unroll
    for (int k = 0; k < S::PER; ++k) *reinterpret_cast<float4*>(S::at(region, buf, lane + 64 * k)) = r[k];
    mt_publish(ready + buf, g + 1);
    issue(r, g + 3);
  };
  issue(r0, 0);
  issue(r1, 1);
  issue(r2, 2);
  for (int g = 0; g < T; g += 3) {
    step(r0, g);
    if (g + 1 >= T) break;
    step(r1, g + 1);
    if (g + 2 >= T) break;
    step(r2, g + 2);
  }
}

// One chunk of the transposed contraction for a compute wave: K steps
// 4 c .. 4 c + 3 from LDS buffer `buf`, both tiles (only the first if !two);
// the shift panel operands come from a ring of four register slots, each
// refilled after use with the K step four ahead (wrapping into the next
// unit's tiles at the end of the pair: yn0, yn1).
template <int CTQ>
__device__ __forceinline__ void mt_chunk(const float* region, int buf, int c, int nks, f32x16 (&acc)[kMtTiles][CTQ],
                                         f16x8 (&y0)[4], f16x8 (&y1)[4], const f16x8* y0p, const f16x8* y1p,
                                         const f16x8* yn0, const f16x8* yn1, bool two, int lane) {
  using S = MtStage<CTQ>;
  const float* Zb = region + buf * S::BUF + (lane & 31) * S::ROWW + 4 * (lane >> 5);
  // Zhat fragments double-buffered: those of K step s + 1 are read while the
  // MFMAs of step s issue
  f16x8 a2[2][CTQ];
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) a2[0][ct] = *reinterpret_cast<const f16x8*>(Zb + ct * 32 * S::ROWW);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s + 1 < 4) {
#pragma unroll
      for (int ct = 0; ct < CTQ; ++ct)
        a2[(s + 1) & 1][ct] = *reinterpret_cast<const f16x8*>(Zb + ct * 32 * S::ROWW + 8 * (s + 1));
    }
    const f16x8 (&a)[CTQ] = a2[s & 1];
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct)
      acc[0][ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[ct], y0[s], acc[0][ct], 0, 0, 0);
    // a slot with one tile skips the second (wave-uniform branch; its panel
    // registers still cycle, loaded from the last tile)
    if (two) {
#pragma unroll
      for (int ct = 0; ct < CTQ; ++ct)
        acc[1][ct] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[ct], y1[s], acc[1][ct], 0, 0, 0);
    }
    const int kn = 4 * c + s + 4;
    const bool wrap = kn >= nks;
    const int ko = (wrap ? kn - nks : kn) * 64;
    y0[s] = (wrap ? yn0 : y0p)[ko];
    y1[s] = (wrap ? yn1 : y1p)[ko];
  }
}

// Rotation transform, argmax and (WX) X stores of the wave's two tiles
// (shifts past N, e.g. of a missing second tile, take no part in the argmax
// and are not stored).  Software-pipelined over the row tiles t of 16
// rotations: the table fragments of t + 1 are read, the MFMAs of t issued
// and the vector work of t - 1 done, so both overlap the matrix cores.
//
// Argmax.  Lane l holds, per tile and half of the rotations, the quads
// r = 16 t + 4 (l / 16) + v, v = 0..3 (and r + QH).  With X stored (WX) every
// element is compared and stored.  Without, a lane keeps per tile and half
// only the largest quad maximum and the first t that reached it (5 vector
// operations per quad instead of 12); the wave then takes the best
// (value, quad index) over its lanes, which is the best (value, index) over
// the wave at quad granularity: quads of different lanes are disjoint index
// ranges, and within a lane the first t and the first half win ties.  The
// winning lane's quad is recomputed (one row tile of products, the same
// inputs and order, so bitwise the same values) and its lowest element equal
// to the maximum completes the index.
template <int CTQ, bool WX>
__device__ __forceinline__ void mt_epilogue(const Step3Args& p, f32x16 (&acc)[kMtTiles][CTQ], int pair, int t0,
                                            const float4* __restrict__ tbl, int lane) {
  constexpr int QH = 32 * CTQ;
  constexpr int Qa = 2 * QH;
  constexpr int NT = QH / 16;  // row tiles of 16 rotations
  constexpr int NTL = kMtTiles;
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  // B operands: the even-q (E) and odd-q (O) registers of each column tile
  f16x8 BE[NTL][CTQ], BO[NTL][CTQ];
#pragma unroll
  for (int st = 0; st < NTL; ++st)
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) {
      u32x4 e4, o4;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        e4[w] = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                                                  (float2_v{acc[st][ct][4 * w], acc[st][ct][4 * w + 2]}), f16x2));
        o4[w] = __builtin_bit_cast(uint32_t, __builtin_convertvector(
                                                  (float2_v{acc[st][ct][4 * w + 1], acc[st][ct][4 * w + 3]}), f16x2));
      }
      BE[st][ct] = __builtin_bit_cast(f16x8, e4);
      BO[st][ct] = __builtin_bit_cast(f16x8, o4);
    }
  const int dl = lane & 15;
  const int r4 = 4 * (lane >> 4);
  float xs = 1.f;
  float* xr[NTL];
  bool valid[NTL];
  float bv0[NTL], bv1[NTL];
  int bs0[NTL], bs1[NTL];  // WX: step 4 t + v of the best in each half; else the first t of the best quad
#pragma unroll
  for (int st = 0; st < NTL; ++st) {
    const int delta = 16 * (t0 + st) + dl;
    valid[st] = delta < p.N;
    xr[st] = WX ? p.X + (static_cast<size_t>(pair) * p.N + (valid[st] ? delta : 0)) * Qa + r4 : nullptr;
    bv0[st] = bv1[st] = -__builtin_inff();
    bs0[st] = bs1[st] = -1;
  }
  if (WX && p.xscale) xs = *p.xscale;
  const f16x8* tb = reinterpret_cast<const f16x8*>(tbl) + lane;
  f16x8 tE[2][CTQ], tO[2][CTQ];  // table fragments of t (slot t % 2)
  f32x4 dE[2][NTL], dO[2][NTL];  // products of t (slot t % 2)
  auto load_tables = [&](int t, int slot) {
#pragma unroll
    for (int s = 0; s < CTQ; ++s) {
      tE[slot][s] = tb[64 * (t * CTQ + s)];
      tO[slot][s] = tb[64 * ((NT + t) * CTQ + s)];
    }
  };
  auto products = [&](int slot) {
#pragma unroll
    for (int st = 0; st < NTL; ++st) {
      dE[slot][st] = f32x4{0.f, 0.f, 0.f, 0.f};
      dO[slot][st] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    // a missing second tile's products are formed too (its shifts take no
    // part: valid[1] is false); a branch here costs more registers than the
    // kernel has
#pragma unroll
    for (int s = 0; s < CTQ; ++s)
#pragma unroll
      for (int st = 0; st < NTL; ++st) {
        dE[slot][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tE[slot][s], BE[st][s], dE[slot][st], 0, 0, 0);
        dO[slot][st] = __builtin_amdgcn_mfma_f32_16x16x32_f16(tO[slot][s], BO[st][s], dO[slot][st], 0, 0, 0);
      }
  };
  // sums and compares (increasing r within each half: a later equal value
  // never replaces, so the lowest index wins ties; NaN never compares
  // greater) and (WX) stores of the rotations of row tile t
  auto finish = [&](int t, int slot) {
#pragma unroll
    for (int st = 0; st < NTL; ++st) {
      f32x4 x0, x1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        x0[v] = dE[slot][st][v] + dO[slot][st][v];
        x1[v] = dE[slot][st][v] - dO[slot][st][v];
      }
      if (WX) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool g0 = x0[v] > bv0[st], g1 = x1[v] > bv1[st];
          bv0[st] = g0 ? x0[v] : bv0[st];
          bs0[st] = g0 ? 4 * t + v : bs0[st];
          bv1[st] = g1 ? x1[v] : bv1[st];
          bs1[st] = g1 ? 4 * t + v : bs1[st];
        }
        if (valid[st]) {
          *reinterpret_cast<float4*>(xr[st] + 16 * t) = make_float4(x0[0] * xs, x0[1] * xs, x0[2] * xs, x0[3] * xs);
          *reinterpret_cast<float4*>(xr[st] + QH + 16 * t) =
              make_float4(x1[0] * xs, x1[1] * xs, x1[2] * xs, x1[3] * xs);
        }
      } else {
        // quad maxima (fmaxf skips NaN), then the first t of the largest
        const float m0 = fmaxf(fmaxf(fmaxf(x0[0], x0[1]), x0[2]), x0[3]);
        const float m1 = fmaxf(fmaxf(fmaxf(x1[0], x1[1]), x1[2]), x1[3]);
        const bool g0 = m0 > bv0[st], g1 = m1 > bv1[st];
        bv0[st] = g0 ? m0 : bv0[st];
        bs0[st] = g0 ? t : bs0[st];
        bv1[st] = g1 ? m1 : bv1[st];
        bs1[st] = g1 ? t : bs1[st];
      }
    }
  };
  load_tables(0, 0);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t + 1 < NT) load_tables(t + 1, (t + 1) & 1);
    products(t & 1);
    if (t > 0) finish(t - 1, (t - 1) & 1);
  }
  finish(NT - 1, (NT - 1) & 1);
  // the lane's best over its shifts (the first half of the rotations wins
  // ties: lower index), then over the wave; without X the index is that of
  // the quad (its element v = 0)
  float bv = -__builtin_inff();
  uint32_t bi = 0xffffffffu;
#pragma unroll
  for (int st = 0; st < NTL; ++st) {
    const bool take1 = bs1[st] >= 0 && (bs0[st] < 0 || bv1[st] > bv0[st]);
    const int bs = take1 ? bs1[st] : bs0[st];
    const bool ok = valid[st] && bs >= 0;
    const uint32_t r = WX ? 16 * (bs >> 2) + r4 + (bs & 3) : 16 * bs + r4;
    const uint32_t i = static_cast<uint32_t>(16 * (t0 + st) + dl) * Qa + (take1 ? QH : 0) + r;
    ep_better(bv, bi, ok ? (take1 ? bv1[st] : bv0[st]) : -__builtin_inff(), ok ? i : 0xffffffffu);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const uint32_t oi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(bi), off));
    ep_better(bv, bi, ov, oi);
  }
  if (bi == 0xffffffffu) return;  // no valid shift (wave-uniform)
  if (!WX) {
    // the winning quad: shift delta = bi / Qa (tile st, lane dl + 16 (r4 / 4)),
    // rotation r = bi % Qa = half QH + 16 t + r4
    const uint32_t delta = bi / Qa, rr = bi - delta * Qa;
    const int half = rr >= static_cast<uint32_t>(QH);
    const int rq = static_cast<int>(rr) - (half ? QH : 0);
    const int t = __builtin_amdgcn_readfirstlane(rq >> 4);
    const int st = __builtin_amdgcn_readfirstlane(static_cast<int>(delta >> 4) - t0);
    const int win = static_cast<int>(delta & 15) + 4 * (rq & 15);
    load_tables(t, 0);
    f32x4 e = {0.f, 0.f, 0.f, 0.f}, o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < CTQ; ++s) {
      e = __builtin_amdgcn_mfma_f32_16x16x32_f16(tE[0][s], st ? BE[1][s] : BE[0][s], e, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_16x16x32_f16(tO[0][s], st ? BO[1][s] : BO[0][s], o, 0, 0, 0);
    }
    int v = 3;
#pragma unroll
    for (int k = 3; k >= 0; --k) v = ((half ? e[k] - o[k] : e[k] + o[k]) == bv) ? k : v;
    bi += static_cast<uint32_t>(__shfl(v, win));
  }
  if (lane == 0) atomicMax(p.keys + pair, pose_key(bv, bi));
}

// One workgroup of kMtWaves waves per CU, looping over (pair, shift block)
// units; a shift block is kMtCompute * kMtTiles tiles of 16 shifts.
template <int CTQ, bool WX>
__global__ void __launch_bounds__(64 * kMtWaves) step3_fp16_mt(Step3Args p) {
  extern __shared__ float smem[];
  using S = MtStage<CTQ>;
  constexpr int QH = 32 * CTQ;
  constexpr int NFRAG = 2 * (QH / 16) * CTQ;  // 1 KB each
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  float4* tbl = reinterpret_cast<float4*>(smem);
  const float4* tsrc = static_cast<const float4*>(p.rot16);
  for (int i = tid; i < NFRAG * 64; i += blockDim.x) tbl[i] = tsrc[i];
  float* region = smem + NFRAG * 256;
  int* ready = S::flags(region);
  int* prog = ready + kMtRing;
  int* abort = prog + kMtCompute;
  if (tid < kMtFlagWords) ready[tid] = 0;
  const int total = p.pairs * p.nblk;
  if (static_cast<int>(blockIdx.x) >= total) return;
  __syncthreads();  // tables and flags set (the only workgroup barrier)
  const int units = (total - 1 - static_cast<int>(blockIdx.x)) / static_cast<int>(gridDim.x) + 1;
  const int nks = p.H_pad / 8;   // K steps of 16 k' (2 H_pad k')
  const int nch = p.H_pad / 32;  // chunks of 64 k'
  if (wave == kMtCompute) {
    mt_stager<CTQ>(p, region, units * nch, nch);
    return;
  }
  const int lane = tid & 63;
  const int ntiles = (p.N + 15) / 16;
  const int ntile_pad = p.N_pad / 16;
  // shift panel fragments [tile][K step][lane][8] fp16 (column j = 16 c + dl)
  // of the two tiles of slot ws in shift block yb (a missing tile reads the
  // last).  A shift block is kMtCompute slots of two tiles; the wave takes
  // slot (wave + k) mod kMtCompute in the k-th unit of its workgroup, so a
  // short last slot (N = 197: 13 tiles in 7 slots) falls on each wave, hence
  // each SIMD, in turn instead of always on the same one.
  auto panel = [&](int yb, int ws, int st) {
    const int t = min((yb * kMtCompute + ws) * kMtTiles + st, ntile_pad - 1);
    return reinterpret_cast<const f16x8*>(p.yt_hi) + static_cast<size_t>(t) * nks * 64 + lane;
  };
  int b = blockIdx.x;
  int pair, yb;
  step3_block(b, p.nblk, p.pairs, pair, yb);
  int ws = wave;
  const f16x8* y0p = panel(yb, ws, 0);
  const f16x8* y1p = panel(yb, ws, 1);
  f16x8 y0[4], y1[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    y0[s] = y0p[min(s, nks - 1) * 64];
    y1[s] = y1p[min(s, nks - 1) * 64];
  }
  int g = 0;  // stream position
  for (;;) {
    const int t0 = (yb * kMtCompute + ws) * kMtTiles;
    const int nt = max(0, min(kMtTiles, ntiles - t0));
    const int bn = b + gridDim.x;
    int pn = pair, ybn = yb;
    if (bn < total) step3_block(bn, p.nblk, p.pairs, pn, ybn);
    const int wsn = ws + 1 == kMtCompute ? 0 : ws + 1;
    const f16x8* yn0 = panel(ybn, wsn, 0);
    const f16x8* yn1 = panel(ybn, wsn, 1);
    f32x16 acc[kMtTiles][CTQ];
#pragma unroll
    for (int st = 0; st < kMtTiles; ++st)
#pragma unroll
      for (int ct = 0; ct < CTQ; ++ct) acc[st][ct] = zero16();
    for (int c = 0; c < nch; ++c, ++g) {
      const int buf = g % kMtRing;
      mt_wait_ge(ready + buf, g + 1, abort);  // chunk g is in buffer g % kMtRing
      if (nt > 0) mt_chunk<CTQ>(region, buf, c, nks, acc, y0, y1, y0p, y1p, yn0, yn1, nt > 1, lane);
      mt_publish(prog + wave, g + 1);  // done reading chunk g
    }
    if (nt > 0) {
      mt_epilogue<CTQ, WX>(p, acc, pair, t0, tbl, lane);
    } else {
      // an idle unit did not run the K loop, whose last chunk loads the next
      // unit's first four K steps into the panel ring: load them here
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        y0[s] = yn0[s * 64];
        y1[s] = yn1[s * 64];
      }
    }
    if (bn >= total) break;
    b = bn;
    pair = pn;
    yb = ybn;
    ws = wsn;
    y0p = yn0;
    y1p = yn1;
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

// LDS of the two-tile kernel: the tables, the ring of Zhat buffers of 64 k',
// the flags
size_t step3_fp16_rot_lds_bytes(int Qa, int) {
  const size_t QH = Qa / 2;
  return rot16_table_bytes(Qa) + sizeof(float) * kMtRing * QH * 36 + sizeof(int) * kMtFlagWords;
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
      // one workgroup of kMtWaves waves per CU; a shift block is
      // kMtCompute * kMtTiles tiles of 16 shifts
      Step3Args m = a0;
      m.nwaves = kMtWaves;
      m.nblk = (m.N + kMtBlockShifts - 1) / kMtBlockShifts;
      const size_t units = static_cast<size_t>(m.pairs) * m.nblk;
      if (units > 0x7fffffffull) return hipErrorInvalidConfiguration;
      const size_t lds = step3_fp16_rot_lds_bytes(m.Qa, kMtWaves);
      auto kern = m.X ? step3_fp16_mt<CTQ, true> : step3_fp16_mt<CTQ, false>;
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
      if (e != hipSuccess) return e;
      const unsigned grid = static_cast<unsigned>(std::min<size_t>(units, static_cast<size_t>(device_cus())));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * kMtWaves), lds, s, m);
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
