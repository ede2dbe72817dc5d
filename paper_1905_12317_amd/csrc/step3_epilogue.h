// Rotation FFT + argmax of Step 3 (Step 2 of eq. fbk3, eq. 1dfft), shared by
// the FP32, split-bf16 and FP16 forms, working mostly in registers.
//
// Input: the wave's MFMA accumulators acc[ct][v] of the shift contraction:
// lane l (h = l / 32, j = l % 32) holds column q = 32 ct + j (mode) for rows
// 8 (v / 4) + 4 h + (v % 4); row 2 dl + c is shift d0 + dl, c = 0 real and
// c = 1 imaginary part of Xhat(delta, q), q = 0 .. QH - 1 (QH = Qa / 2; the
// Nyquist mode was folded into q = 0 as Xhat(0) + i Xhat(QH)).
//
// For each shift the Qa real outputs X(delta, r) = Re sum_q ... come from a
// length-QH complex FFT of the packed sequence
//     Z[k] = (P[k] + conj P[QH - k]) + i W^k (P[k] - conj P[QH - k]),
//     Z[0] = (Re P0 + Im P0) + i (Re P0 - Im P0),  W = exp(-2 pi i / Qa),
// with X(2s) = Re z[s], X(2s + 1) = Im z[s].  The FFT splits k = 32 ct + j and
// s = s1 + CTQ m:
//   (1) a CTQ-point DFT over ct in registers, then the twiddle w^{j s1}
//       (w = exp(-2 pi i / QH));
//   (2) per s1 a 32-point DFT over the lanes j of each half-wave: one LDS
//       transpose gives each quad of lanes one sequence (lane a of the quad
//       holds elements 4 b + a), an 8-point FFT runs in each lane, and a
//       radix-4 step across the quad uses DPP lane permutes.
// The argmax over (shift, rotation) is kept per lane and reduced with wave
// shuffles; one 64-bit atomicMax per wave publishes it.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace ftkdev {

typedef float f32x16_e __attribute__((ext_vector_type(16)));

constexpr int kEpiRowStride = 36;  // float2 per transpose row (32 + 4: conflict-free)
constexpr int kEpiRounds = 2;      // FFT rounds staged in LDS at a time

// LDS bytes of the epilogue per wave: kEpiRounds x two half-waves x 8 rows
__host__ __device__ constexpr size_t epilogue_lds_bytes_per_wave() {
  return sizeof(float2) * kEpiRounds * 2 * 8 * kEpiRowStride;
}

__device__ __forceinline__ void ep_better(float& bv, uint32_t& bi, float v, uint32_t i) {
  const bool g = v > bv || (v == bv && i < bi);
  bv = g ? v : bv;
  bi = g ? i : bi;
}

// value of the lane `lane ^ x` of the same quad (x = 1 or 2)
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
// exp(-i pi k / 12), k = 0 .. 23 (every CTQ in {1, 2, 3, 4, 6} divides 12)
__device__ __forceinline__ float2 ep_unit12(int k) {
  const float sg = k < 12 ? 1.f : -1.f;
  k = k < 12 ? k : k - 12;
  constexpr float cs[12] = {1.f, 0.96592582628906829f, 0.86602540378443865f, 0.70710678118654752f, 0.5f,
                            0.25881904510252076f, 0.f, -0.25881904510252076f, -0.5f, -0.70710678118654752f,
                            -0.86602540378443865f, -0.96592582628906829f};
  constexpr float sn[12] = {0.f, 0.25881904510252076f, 0.5f, 0.70710678118654752f, 0.86602540378443865f,
                            0.96592582628906829f, 1.f, 0.96592582628906829f, 0.86602540378443865f,
                            0.70710678118654752f, 0.5f, 0.25881904510252076f};
  return make_float2(sg * cs[k], -sg * sn[k]);
}
// Pair and shift block of workgroup b in the 1-D grid of pairs * nblk.
// Workgroups are dealt to the 8 XCDs round-robin, so blocks b and b + 8 share
// an XCD: in each full group of 8 nblk workgroups, the nblk shift blocks of a
// pair sit 8 apart and the later ones find the pair's Zhat in that XCD's L2.
// A last, partial group takes its pairs' blocks consecutively.
__device__ __forceinline__ void step3_block(int b, int nblk, int pairs, int& pair, int& yb) {
  const int gs = 8 * nblk;
  const int g = b / gs;
  const int i = b - g * gs;
  if (8 * (g + 1) <= pairs) {
    pair = 8 * g + (i & 7);
    yb = i >> 3;
  } else {
    pair = 8 * g + i / nblk;
    yb = i - (i / nblk) * nblk;
  }
}

// streaming 16-byte load of the staging (read once, by one workgroup: not
// kept in the caches, which then keep Step 1's template operand)
__device__ __forceinline__ float4 load_stream(const float4* p) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const v4f x = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(x[0], x[1], x[2], x[3]);
}
// value of lane addr / 4 (ds_bpermute with a precomputed byte address)
__device__ __forceinline__ float ep_bperm(float v, int addr) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]

// Modes of the epilogue (compile time, so the plain form keeps its registers):
//   kEpiRotate:  the rotation sum and argmax as described above;
//   kEpiStore:   no rotation sum; the wave stores its Xhat into p.xhat, rows
//                [pair][q][c][delta] (c = 0 real, 1 imaginary part, N_pad
//                shifts), for the upsampled rotation kernel;
//   kEpiUpsample: pass u of U of the rotation upsampling: acc holds
//                Xhat(q) e^{-i q 2 pi u / (U Qa)} and output r of this pass is
//                rotation U r + u of the U Qa-point grid (X rows of U Qa
//                values, pose index delta U Qa + U r + u).
constexpr int kEpiRotate = 0, kEpiStore = 1, kEpiUpsample = 2;

template <int CTQ, int MODE = kEpiRotate, class Acc>
__device__ __forceinline__ void step3_epilogue_reg(const Step3Args& p, Acc (&acc)[CTQ], int pair, int d0, float2* T,
                                                   const float2* __restrict__ tw, int lane, int Ur = 1, int ur = 0) {
  constexpr int QH = 32 * CTQ;
  constexpr int Qa = 2 * QH;
  constexpr bool UP = MODE == kEpiUpsample;
  const int h = lane >> 5;
  const int j = lane & 31;
  const int U = UP ? Ur : 1;
  const int u = UP ? ur : 0;
  if constexpr (MODE == kEpiStore) {
    float* xb = p.xhat + static_cast<size_t>(pair) * QH * 2 * p.N_pad + d0 + 2 * h;
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) {
      float* row = xb + static_cast<size_t>(32 * ct + j) * 2 * p.N_pad;
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          *reinterpret_cast<float2*>(row + c * p.N_pad + 4 * g) = make_float2(acc[ct][4 * g + c], acc[ct][4 * g + 2 + c]);
    }
    return;
  } else {
  const int src4 = ((h << 5) | ((32 - j) & 31)) << 2;  // byte address of the lane of column QH - k (j > 0)
  // W^{32 ct + j}, and the powers w^{j s1} (w = exp(-2 pi i / QH)), from the
  // table: the same for every shift of the lane
  float2 wk[CTQ], wjs[CTQ];
#pragma unroll
  for (int ct = 0; ct < CTQ; ++ct) {
    wk[ct] = tw[32 * ct + j];
    wjs[ct] = tw[(2 * j * ct) % Qa];
  }

  // ---- (0) real-output packing, in place: acc[ct][(u)] <- Z_u[32 ct + j]
  // u = 2 v4 + d is the shift 4 v4 + 2 h + d of this lane; its (re, im) sit
  // in registers 4 v4 + 2 d and 4 v4 + 2 d + 1.
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int vr = 4 * (u >> 1) + 2 * (u & 1);
    float2 P[CTQ], Pp[CTQ];
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) P[ct] = make_float2(acc[ct][vr], acc[ct][vr + 1]);
    // partner of column k = 32 ct + j: lane 32 - j at tile CTQ - 1 - ct (j > 0),
    // this lane at tile CTQ - ct (j = 0)
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) {
      const float2 o = P[CTQ - 1 - ct];
      Pp[ct] = make_float2(ep_bperm(o.x, src4), ep_bperm(o.y, src4));
      if (j == 0) Pp[ct] = P[(CTQ - ct) % CTQ];
    }
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) {
      float2 Z;
      if (ct == 0 && j == 0) {
        Z = make_float2(P[0].x + P[0].y, P[0].x - P[0].y);
      } else {
        const float2 Qc = cconj(Pp[ct]);
        const float2 s = cadd(P[ct], Qc);
        const float2 uu = cmul(csub(P[ct], Qc), wk[ct]);
        Z = make_float2(s.x - uu.y, s.y + uu.x);
      }
      acc[ct][vr] = Z.x;
      acc[ct][vr + 1] = Z.y;
    }
    // keep each shift's lane exchanges next to their use (register pressure)
    __builtin_amdgcn_sched_barrier(0);
  }

  // ---- (1) CTQ-point DFT over ct and the twiddle w^{j s1}, in place
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int vr = 4 * (u >> 1) + 2 * (u & 1);
    float2 v[CTQ];
#pragma unroll
    for (int ct = 0; ct < CTQ; ++ct) v[ct] = make_float2(acc[ct][vr], acc[ct][vr + 1]);
    if constexpr (CTQ == 2) {
      dft2<false>(v);
    } else if constexpr (CTQ == 3) {
      dft3<false>(v);
    } else if constexpr (CTQ == 4) {
      dft4<false>(v);
    } else if constexpr (CTQ == 6) {
      // 6 = 3 x 2: n = 3 n1 + n2, k = k1 + 2 k2
      float2 A0[2] = {v[0], v[3]}, A1[2] = {v[1], v[4]}, A2[2] = {v[2], v[5]};
      dft2<false>(A0);
      dft2<false>(A1);
      dft2<false>(A2);
      A1[1] = cmul(A1[1], ep_unit12(4));  // W6^1
      A2[1] = cmul(A2[1], ep_unit12(8));  // W6^2
      float2 B0[3] = {A0[0], A1[0], A2[0]}, B1[3] = {A0[1], A1[1], A2[1]};
      dft3<false>(B0);
      dft3<false>(B1);
      v[0] = B0[0];
      v[2] = B0[1];
      v[4] = B0[2];
      v[1] = B1[0];
      v[3] = B1[1];
      v[5] = B1[2];
    } else if constexpr (CTQ > 4) {
      float2 y[CTQ];
#pragma unroll
      for (int s1 = 0; s1 < CTQ; ++s1) {
        y[s1] = v[0];
#pragma unroll
        for (int ct = 1; ct < CTQ; ++ct) y[s1] = cadd(y[s1], cmul(v[ct], ep_unit12(24 * ((ct * s1) % CTQ) / CTQ)));
      }
#pragma unroll
      for (int s1 = 0; s1 < CTQ; ++s1) v[s1] = y[s1];
    }
#pragma unroll
    for (int s1 = 0; s1 < CTQ; ++s1) {
      const float2 y = s1 > 0 ? cmul(v[s1], wjs[s1]) : v[s1];
      acc[s1][vr] = y.x;
      acc[s1][vr + 1] = y.y;
    }
  }

  // ---- (2) per s1: 32-point DFT over j through an LDS transpose.  The
  // rounds are staged kEpiRounds at a time, so that the accumulators of
  // those rounds are dead before the FFT temporaries are needed.
  float bv = -__builtin_inff();
  uint32_t bi = 0xffffffffu;
  const int Qo = U * Qa;  // X row length and pose index stride
  float* Xp = p.X ? p.X + static_cast<size_t>(pair) * p.N * Qo : nullptr;
  // scale of the stored X values (the FP16 form computes X / (s_a s_b s_y));
  // the argmax does not depend on it
  const float xs = (Xp && p.xscale) ? *p.xscale : 1.f;
  const int Q = j >> 2;  // the sequence (shift u = Q) this lane's quad transforms
  const int a = j & 3;
  const int a0 = a & 1, a1 = a >> 1;
  const int dl = 4 * (Q >> 1) + 2 * h + (Q & 1);
  const int delta = d0 + dl;
  const bool valid = delta < p.N;
  const float sg1 = a1 ? -1.f : 1.f;  // first radix-2 stage: y + x or x' - x
  const float sg0 = a0 ? -1.f : 1.f;  // second stage
  const bool rot = a0 && a1;
  constexpr float c8 = 0.70710678118654752440f;
  constexpr int RP = CTQ < kEpiRounds ? CTQ : kEpiRounds;
#pragma unroll
  for (int s0 = 0; s0 < CTQ; s0 += RP) {
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) {
      const int s1 = s0 + rr;
      if (s1 >= CTQ) break;
      float2* Th = T + (2 * rr + h) * 8 * kEpiRowStride;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int vr = 4 * (u >> 1) + 2 * (u & 1);
        Th[u * kEpiRowStride + j] = make_float2(acc[s1][vr], acc[s1][vr + 1]);
      }
    }
    wave_sync();
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) {
      const int s1 = s0 + rr;
      if (s1 >= CTQ) break;
      const float2* Th = T + (2 * rr + h) * 8 * kEpiRowStride;
      float2 x[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) x[b] = Th[Q * kEpiRowStride + 4 * b + a];
      // 8-point DFT of x[b] (elements 4 b + a of the sequence) in registers
      float2 e[4] = {x[0], x[2], x[4], x[6]};
      float2 o[4] = {x[1], x[3], x[5], x[7]};
      dft4<false>(e);
      dft4<false>(o);
      const float2 w8[4] = {make_float2(1.f, 0.f), make_float2(c8, -c8), make_float2(0.f, -1.f),
                            make_float2(-c8, -c8)};
      float2 Y[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const float2 t = cmul(o[k], w8[k]);
        Y[k] = cadd(e[k], t);
        Y[k + 4] = csub(e[k], t);
      }
      // twiddle exp(-2 pi i a s' / 32) (from the table), then the radix-4
      // DFT over the quad
#pragma unroll
      for (int sp = 1; sp < 8; ++sp) Y[sp] = cmul(Y[sp], tw[a * sp * (Qa / 32)]);
      // butterflies as sign FMAs (x * (+-1) + y is exact: same values as
      // y +- x); lane 3 of the quad also rotates its difference by -i
#pragma unroll
      for (int sp = 0; sp < 8; ++sp) {
        const float2 oy = make_float2(quad_swap<kQuadXor2>(Y[sp].x), quad_swap<kQuadXor2>(Y[sp].y));
        float2 U = make_float2(__builtin_fmaf(sg1, Y[sp].x, oy.x), __builtin_fmaf(sg1, Y[sp].y, oy.y));
        if (rot) U = make_float2(U.y, -U.x);
        const float2 ou = make_float2(quad_swap<kQuadXor1>(U.x), quad_swap<kQuadXor1>(U.y));
        Y[sp] = make_float2(__builtin_fmaf(sg0, U.x, ou.x), __builtin_fmaf(sg0, U.y, ou.y));
      }
      // lane a holds z[s1 + CTQ (s' + 8 (a1 + 2 a0))]: its 16 outputs have
      // flat indices delta Qa + 2 s (+1) that grow with s'.  Their maximum
      // (fmaxf skips NaN, as ep_better does), then the lowest output equal
      // to it; the compares are independent, so no select waits on another.
      float rv = Y[0].x;
#pragma unroll
      for (int k = 1; k < 16; ++k) rv = fmaxf(rv, (k & 1) ? Y[k >> 1].y : Y[k >> 1].x);
      int rk = -1;
#pragma unroll
      for (int k = 15; k >= 0; --k) rk = (((k & 1) ? Y[k >> 1].y : Y[k >> 1].x) == rv) ? k : rk;
      const bool ok = valid && rk >= 0;
      const uint32_t ridx = static_cast<uint32_t>(delta) * Qo +
                            U * (2 * (s1 + CTQ * (8 * (a1 + 2 * a0) + (rk >> 1))) + (rk & 1)) + u;
      ep_better(bv, bi, ok ? rv : -__builtin_inff(), ok ? ridx : 0xffffffffu);
      if (Xp && valid) {
        if (!UP) {
          float2* xr = reinterpret_cast<float2*>(Xp + static_cast<size_t>(delta) * Qa);
#pragma unroll
          for (int sp = 0; sp < 8; ++sp)
            xr[s1 + CTQ * (sp + 8 * (a1 + 2 * a0))] = make_float2(Y[sp].x * xs, Y[sp].y * xs);
        } else {
          float* xr = Xp + static_cast<size_t>(delta) * Qo + u;
#pragma unroll
          for (int sp = 0; sp < 8; ++sp) {
            const int t2 = 2 * (s1 + CTQ * (sp + 8 * (a1 + 2 * a0)));
            xr[U * t2] = Y[sp].x * xs;
            xr[U * (t2 + 1)] = Y[sp].y * xs;
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    wave_sync();
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const uint32_t oi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(bi), off));
    ep_better(bv, bi, ov, oi);
  }
  if (lane == 0 && bi != 0xffffffffu) atomicMax(p.keys + pair, pose_key(bv, bi));
  }
}

}  // namespace ftkdev
