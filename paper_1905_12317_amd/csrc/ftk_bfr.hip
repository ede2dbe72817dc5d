// ftk_bfr_align: brute-force rotations (Section 6.1 of the paper), the
// comparison method that correlates over a grid of shifts by the 2D
// convolution theorem once per rotation (eq. 2dconv).  FP32 whatever the
// plan's precision form; shifts from ftk_set_shifts; R = Qa U rotations
// gamma_r = 2 pi r / R (U the plan's rotation upsampling factor).
//
// Per call: the image spectra on the half-disk rows of the Cartesian grid
// (the transform's fine grid, interpolated at k = pi (u, v)); then per chunk
// of templates their spectra at the R rotated grids (a quarter of them
// interpolated, the rest by quarter turns) and the correlation kernel, once
// per pass of 17 y offsets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "plan_internal.h"

using namespace ftkint;

namespace {

constexpr double kPiD = 3.14159265358979323846;

// Host tables of one call: the x and y offsets of the shift list, their
// phases, the shift index of every grid point and the chunks of the u sums.
struct BfrTables {
  std::vector<float2> ex, ey;
  std::vector<int> head, nxt;
  std::vector<int4> chunks;
  int Dx = 0, Dy = 0, Dy_pad = 0;
};

std::vector<double> distinct(std::vector<double> v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

BfrTables bfr_tables(const ftk_plan* p, int V, int Up) {
  BfrTables t;
  const int N = p->N, n = p->n;
  std::vector<double> xs(N), ys(N);
  for (int i = 0; i < N; ++i) {
    xs[i] = p->shifts[2 * i];
    ys[i] = p->shifts[2 * i + 1];
  }
  const std::vector<double> ux = distinct(xs), uy = distinct(ys);
  t.Dx = static_cast<int>(ux.size());
  t.Dy = static_cast<int>(uy.size());
  t.Dy_pad = round_up(t.Dy, kBfrDy);
  t.ex.assign(static_cast<size_t>(t.Dx) * Up, make_float2(0.f, 0.f));
  for (int ix = 0; ix < t.Dx; ++ix)
    for (int j = 0; j <= 2 * V; ++j) {
      const double ph = -2.0 * kPiD * (j - V) * ux[ix] / n;
      t.ex[static_cast<size_t>(ix) * Up + j] = make_float2(static_cast<float>(std::cos(ph)), static_cast<float>(std::sin(ph)));
    }
  t.ey.assign(static_cast<size_t>(t.Dy_pad) * (V + 1), make_float2(0.f, 0.f));
  for (int iy = 0; iy < t.Dy; ++iy)
    for (int v = 0; v <= V; ++v) {
      const double ph = -2.0 * kPiD * v * uy[iy] / n;
      const double c = kPiD * kPiD * (v == 0 ? 1.0 : 2.0);
      t.ey[static_cast<size_t>(iy) * (V + 1) + v] =
          make_float2(static_cast<float>(c * std::cos(ph)), static_cast<float>(c * std::sin(ph)));
    }
  t.head.assign(static_cast<size_t>(t.Dx) * t.Dy, -1);
  t.nxt.assign(N, -1);
  for (int s = N - 1; s >= 0; --s) {  // ascending chains, the lowest index first
    const int ix = static_cast<int>(std::lower_bound(ux.begin(), ux.end(), xs[s]) - ux.begin());
    const int iy = static_cast<int>(std::lower_bound(uy.begin(), uy.end(), ys[s]) - uy.begin());
    int& h = t.head[static_cast<size_t>(ix) * t.Dy + iy];
    t.nxt[s] = h;
    h = s;
  }
  for (int v = 0; v <= V; ++v) {
    int umax = static_cast<int>(std::floor(std::sqrt(static_cast<double>(V) * V - static_cast<double>(v) * v)));
    while (umax * umax + v * v > V * V) --umax;
    while ((umax + 1) * (umax + 1) + v * v <= V * V) ++umax;
    const int k0 = (V - umax) & ~3;
    const int k1 = std::min(Up, round_up(V + umax + 1, 4));
    for (int kc = k0; kc < k1; kc += 32) {
      const int nk = std::min(8, (k1 - kc) / 4);
      t.chunks.push_back(make_int4(v, kc, nk, kc + 32 >= k1 ? 1 : 0));
    }
  }
  return t;
}

template <class T>
size_t put(std::vector<unsigned char>& blob, const std::vector<T>& v) {
  const size_t off = round_up(static_cast<int>(blob.size()), 256);
  blob.resize(off + v.size() * sizeof(T));
  std::copy(reinterpret_cast<const unsigned char*>(v.data()),
            reinterpret_cast<const unsigned char*>(v.data()) + v.size() * sizeof(T), blob.begin() + off);
  return off;
}

}  // namespace

extern "C" {

int ftk_bfr_align(ftk_plan* p, const float* images, int nA, const float* templates, int nB, float* X,
                  ftk_pose* best, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_bfr_align: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_bfr_align: negative count");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_bfr_align: call ftk_set_shifts first");
  if (p->has_ctf) return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: plans with a CTF are not supported");
  if (p->sk.w != 8) return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: spreading kernel width other than 8");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (!X && !best) return fail(FTK_EINVAL, "ftk_bfr_align: X and best are both NULL");
  if (!images || !templates) return fail(FTK_EINVAL, "ftk_bfr_align: NULL images");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = p->n, V = n / 2, V1 = V + 1, Up = round_up(n + 1, 4), R = p->Qa * p->up;
  if (R % 64 != 0) return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: rotation count not a multiple of 64");
  if (bfr_corr_lds_bytes(V) > kLdsLimit) return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: tiles exceed LDS");
  const BfrTables t = bfr_tables(p, V, Up);
  // templates per chunk: their spectra at every rotation within the staging budget
  const size_t per_tmpl = static_cast<size_t>(R) * V1 * Up * sizeof(float2);
  const size_t budget = static_cast<size_t>(p->tune.stage_mib) << 20;
  const int chunk = static_cast<int>(std::min<size_t>(nB, std::max<size_t>(1, budget / per_tmpl)));
  const Needs nd = plan_needs(p, std::max(nA, chunk), 0, true);
  const int tchunk = nd.transform_chunk;
  std::vector<unsigned char> blob;
  std::vector<double> cs(2 * (R / 4));
  for (int r = 0; r < R / 4; ++r) {
    cs[2 * r] = std::cos(2.0 * kPiD * r / R);
    cs[2 * r + 1] = std::sin(2.0 * kPiD * r / R);
  }
  const size_t o_ex = put(blob, t.ex), o_ey = put(blob, t.ey), o_head = put(blob, t.head),
               o_nxt = put(blob, t.nxt), o_ch = put(blob, t.chunks), o_cs = put(blob, cs);
  Workspace& ws = *p->ws;
  const size_t sa_bytes = static_cast<size_t>(nA) * V1 * Up * sizeof(float2);
  const size_t sb_bytes = static_cast<size_t>(chunk) * per_tmpl;
  if (ws.bfr_a.ensure(sa_bytes) != hipSuccess || ws.bfr_b.ensure(sb_bytes) != hipSuccess ||
      ws.bfr_tab.ensure(blob.size()) != hipSuccess ||
      ws.keys.ensure(static_cast<size_t>(nA) * nB * sizeof(unsigned long long)) != hipSuccess ||
      ws.tr_h.ensure(nd.tr_h) != hipSuccess || ws.tr_g.ensure(nd.tr_g) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_bfr_align: workspace");
  hipError_t e;
  unsigned char* tab = ws.bfr_tab.as<unsigned char>();
  // on the caller's stream after its earlier work (which may still read the
  // previous call's tables), and complete before the host vector goes away
  if ((e = hipMemcpyAsync(tab, blob.data(), blob.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "ftk_bfr_align: tables");
  // the padding columns j > 2V are never written by the spectra kernel
  if ((e = hipMemsetAsync(ws.bfr_a.ptr, 0, sa_bytes, s)) != hipSuccess ||
      (e = hipMemsetAsync(ws.bfr_b.ptr, 0, sb_bytes, s)) != hipSuccess)
    return hip_fail(e, "ftk_bfr_align: clear");
  StageTimer& tm = p->timer;
  unsigned long long* keys = ws.keys.as<unsigned long long>();
  const size_t pairs = static_cast<size_t>(nA) * nB;
  hipEvent_t ev = tm.begin(s);
  if ((e = launch_keys_init(keys, pairs, s)) != hipSuccess) return hip_fail(e, "ftk_bfr_align: keys init");
  tm.end(ev, s, 3);

  TransformArgs ta{};
  ta.coeffs = nullptr;  // the fine grid only
  ta.scratchH = ws.tr_h.as<float2>();
  ta.scratchG = ws.tr_g.as<float2>();
  ta.deapod = p->deapod.as<float>();
  ta.tw_nf = p->tw_nf.as<float2>();
  ta.tw_qa = p->tw_qa.as<float2>();
  ta.pt_base = p->ptbase.as<int>();
  ta.pt_ker = p->ptker.as<float>();
  ta.n = n;
  ta.nf = p->sk.nf;
  ta.M = p->M;
  ta.Qa = p->Qa;
  ta.w = p->sk.w;
  BfrSpectraArgs sp{};
  sp.grid = ws.tr_g.as<float2>();
  sp.cs = reinterpret_cast<const double*>(tab + o_cs);
  sp.nf = p->sk.nf;
  sp.w = p->sk.w;
  sp.V = V;
  sp.Up = Up;
  sp.R = R;
  sp.s_per_u = kPiD * (2.0 / n) / p->sk.h;
  sp.beta = static_cast<float>(p->sk.beta);
  sp.scale = static_cast<float>(p->Qa);
  sp.patch = bfr_spectra_patch(sp.s_per_u);
  if (sizeof(float2) * sp.patch * sp.patch > 64 * 1024) return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: spectra patch");
  // spectra of cnt images from imgs into out (quarter: all R rotations)
  auto spectra = [&](const float* imgs, int cnt, float2* out, int quarter) -> int {
    const size_t per = static_cast<size_t>(quarter ? R : 1) * V1 * Up;
    for (int c0 = 0; c0 < cnt; c0 += tchunk) {
      const int c = std::min(tchunk, cnt - c0);
      ta.imgs = imgs + static_cast<size_t>(c0) * n * n;
      hipEvent_t e0 = tm.begin(s);
      if ((e = launch_transform(ta, c, s)) != hipSuccess) return hip_fail(e, "ftk_bfr_align: fine grid");
      tm.end(e0, s, 0);
      sp.cnt = c;
      sp.out = out + static_cast<size_t>(c0) * per;
      sp.quarter = quarter;
      e0 = tm.begin(s);
      if ((e = launch_bfr_spectra(sp, s)) != hipSuccess) return hip_fail(e, "ftk_bfr_align: spectra");
      tm.end(e0, s, 6);
    }
    return FTK_OK;
  };
  if (transform_lds_bytes(p->sk.nf, p->Qa, transform_waves(p->sk.nf, p->Qa)) > kLdsLimit)
    return fail(FTK_EUNSUPPORTED, "ftk_bfr_align: transform LDS");
  int rc = spectra(images, nA, ws.bfr_a.as<float2>(), 0);
  if (rc != FTK_OK) return rc;
  BfrCorrArgs a{};
  a.sa = ws.bfr_a.as<float2>();
  a.sb = ws.bfr_b.as<float2>();
  a.ex = reinterpret_cast<const float2*>(tab + o_ex);
  a.ey = reinterpret_cast<const float2*>(tab + o_ey);
  a.chunks = reinterpret_cast<const int4*>(tab + o_ch);
  a.head = reinterpret_cast<const int*>(tab + o_head);
  a.nxt = reinterpret_cast<const int*>(tab + o_nxt);
  a.keys = keys;
  a.X = X;
  a.nA = nA;
  a.nB = nB;
  a.R = R;
  a.Dx = t.Dx;
  a.Dy = t.Dy;
  a.N = p->N;
  a.V = V;
  a.Up = Up;
  a.nch = static_cast<int>(t.chunks.size());
  for (int B0 = 0; B0 < nB; B0 += chunk) {
    const int nb = std::min(chunk, nB - B0);
    rc = spectra(templates + static_cast<size_t>(B0) * n * n, nb, ws.bfr_b.as<float2>(), 1);
    if (rc != FTK_OK) return rc;
    a.B0 = B0;
    a.nBc = nb;
    for (int iy0 = 0; iy0 < t.Dy; iy0 += kBfrDy) {
      a.iy0 = iy0;
      ev = tm.begin(s);
      if ((e = launch_bfr_corr(a, s)) != hipSuccess) return hip_fail(e, "ftk_bfr_align: correlation");
      tm.end(ev, s, 7);
    }
  }
  if (best) {
    ev = tm.begin(s);
    if ((e = launch_keys_to_poses(keys, best, pairs, R, nullptr, s)) != hipSuccess)
      return hip_fail(e, "ftk_bfr_align: poses");
    tm.end(ev, s, 3);
  }
  return FTK_OK;
}

}  // extern "C"
