// ftk_bft_align: brute-force translations (Section 6.2 of the paper), the
// comparison method, on the plan's grids: transform, translated
// coefficients per shift, the l_max = 0 contraction and the rotation FFT
// with the argmax.  FP32 throughout, whatever the plan's precision form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "plan_internal.h"

using namespace ftkint;

namespace {

// Shifts per contraction workgroup (32, 64 or 128; the padded shift count
// is a multiple of it): wider blocks reuse each template operand load over
// more MFMAs but pad more.  Contraction time per padded shift (relative,
// measured on the 197-shift, 512 x 2048 workload: 246, 226 and 202 ms per
// step for 224, 256 and 256 padded shifts) times the padded count, smallest
// wins.
int bft_zblk(int N) {
  const char* v = std::getenv("FTK_BFT_ZBLK");
  const int x = v ? std::atoi(v) : 0;
  if (x == 32 || x == 64 || x == 128) return x;
  const int zb[3] = {32, 64, 128};
  const double cost[3] = {1.098, 0.881, 0.790};
  int best = 32;
  double bc = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double c = round_up(N, zb[i]) * cost[i];
    if (i == 0 || c < bc) {
      bc = c;
      best = zb[i];
    }
  }
  return best;
}

}  // namespace

extern "C" {

int ftk_bft_align(ftk_plan* p, const float* images, int nA, const float* templates, int nB, float* X,
                  ftk_pose* best, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_bft_align: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_bft_align: negative count");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_bft_align: call ftk_set_shifts first");
  if (p->has_ctf) return fail(FTK_EUNSUPPORTED, "ftk_bft_align: plans with a CTF are not supported");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (!X && !best) return fail(FTK_EINVAL, "ftk_bft_align: X and best are both NULL");
  if (!images || !templates) return fail(FTK_EINVAL, "ftk_bft_align: NULL images");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int M = p->M, Qa = p->Qa, QH = Qa / 2, N = p->N;
  const int zblk = bft_zblk(N);
  const int Np = round_up(N, zblk);
  if (step1_v2_lds_bytes(M, zblk, 0) > kLdsLimit || bft_translate_lds_bytes(Qa) > kLdsLimit)
    return fail(FTK_EUNSUPPORTED, "ftk_bft_align: tiles exceed LDS");
  // images per chunk: the staging of Xhat (QH rows of 2 Np floats per pair)
  const size_t per_pair = static_cast<size_t>(QH) * 2 * Np * sizeof(float);
  const size_t budget = static_cast<size_t>(p->tune.stage_mib) << 20;
  const int chunk = static_cast<int>(std::min<size_t>(nA, std::max<size_t>(1, budget / (per_pair * nB))));
  const size_t coef = static_cast<size_t>(Qa) * M * sizeof(float2);
  Workspace& ws = *p->ws;
  if (ws.stage.ensure(static_cast<size_t>(chunk) * nB * per_pair) != hipSuccess ||
      ws.keys.ensure(static_cast<size_t>(nA) * nB * sizeof(unsigned long long)) != hipSuccess ||
      ws.tmpl.ensure(tmpl_prep_bytes(nB, M, Qa, 0)) != hipSuccess ||
      ws.coef_a.ensure(static_cast<size_t>(chunk) * coef) != hipSuccess ||
      ws.coef_b.ensure(static_cast<size_t>(nB) * coef) != hipSuccess ||
      ws.polar.ensure(static_cast<size_t>(chunk) * coef) != hipSuccess ||
      ws.ta.ensure(static_cast<size_t>(chunk) * (QH + 1) * Np * M * sizeof(float2)) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_bft_align: workspace");
  hipError_t e;
  int rc = transform_run(p, templates, nB, ws.coef_b.as<float2>(), nullptr, stream);
  if (rc != FTK_OK) return rc;
  StageTimer& tm = p->timer;
  unsigned long long* keys = ws.keys.as<unsigned long long>();
  const size_t pairs = static_cast<size_t>(nA) * nB;
  hipEvent_t ev = tm.begin(s);
  if ((e = launch_keys_init(keys, pairs, s)) != hipSuccess) return hip_fail(e, "ftk_bft_align: keys init");
  tm.end(ev, s, 3);
  ev = tm.begin(s);
  if ((e = launch_tmpl_prep(ws.coef_b.as<float2>(), ws.tmpl.ptr, nB, M, Qa, 0, nullptr, s)) != hipSuccess)
    return hip_fail(e, "ftk_bft_align: template operand");
  tm.end(ev, s, 4);

  BftTranslateArgs at{};
  at.polar = ws.polar.as<float2>();
  at.ta = ws.ta.as<float2>();
  at.kd = p->bft_kd.as<float2>();
  at.tw_qa = p->tw_qa.as<float2>();
  at.M = M;
  at.Qa = Qa;
  at.N = N;
  at.N_pad = Np;
  Step1Args a1{};
  a1.ta = ws.ta.as<float2>();
  a1.cz = p->bft_cz.as<float>();
  a1.zs = ws.stage.ptr;
  a1.b = ws.coef_b.as<float2>();
  a1.r32 = ws.tmpl.as<float>();
  a1.nB = nB;
  a1.tiles_per_q = (nB + 15) / 16;
  a1.M = M;
  a1.Qa = Qa;
  a1.H_pad = Np;
  a1.zblk = zblk;
  Step3Args a3{};
  a3.zs = ws.stage.ptr;
  a3.tw_qa = p->tw_qa.as<float2>();
  a3.Qa = Qa;
  a3.H_pad = Np;
  a3.N = N;
  a3.N_pad = Np;
  a3.nwaves = 4;
  a3.up = p->up;
  for (int A0 = 0; A0 < nA; A0 += chunk) {
    const int na = std::min(chunk, nA - A0);
    rc = transform_run(p, images + static_cast<size_t>(A0) * p->n * p->n, na, ws.coef_a.as<float2>(),
                       ws.polar.as<float2>(), stream);
    if (rc != FTK_OK) return rc;
    at.nA = na;
    ev = tm.begin(s);
    if ((e = launch_bft_translate(at, s)) != hipSuccess) return hip_fail(e, "ftk_bft_align: translate");
    tm.end(ev, s, 5);
    a1.nA = na;
    {
      const int base = na * (QH - 1 + zblk / 32) * (Np / zblk);
      const int max_parts = std::max(1, ((nB + 15) / 16 + 7) / 8);
      a1.tparts = std::min(max_parts, std::max(1, (p->tune.step1_wgs + base - 1) / base));
    }
    ev = tm.begin(s);
    if ((e = launch_step1_bft(a1, s)) != hipSuccess) return hip_fail(e, "ftk_bft_align: contraction");
    tm.end(ev, s, 1);
    a3.pairs = na * nB;
    a3.keys = keys + static_cast<size_t>(A0) * nB;
    a3.X = X ? X + static_cast<size_t>(A0) * nB * N * Qa * p->up : nullptr;
    ev = tm.begin(s);
    if ((e = launch_xhat_rotate(a3, s)) != hipSuccess) return hip_fail(e, "ftk_bft_align: rotation");
    tm.end(ev, s, 2);
  }
  if (best) {
    ev = tm.begin(s);
    if ((e = launch_keys_to_poses(keys, best, pairs, Qa * p->up, nullptr, s)) != hipSuccess)
      return hip_fail(e, "ftk_bft_align: poses");
    tm.end(ev, s, 3);
  }
  return FTK_OK;
}

}  // extern "C"
