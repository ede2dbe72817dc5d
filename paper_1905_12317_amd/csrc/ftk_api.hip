// C-ABI of the FTK library: plans, shift tables, transform and alignment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "plan_internal.h"

namespace ftkint {

namespace {
thread_local std::string g_last_error;
}  // namespace

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(FTK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

size_t env_mib(const char* name, size_t dflt_mib) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt_mib;
  char* end = nullptr;
  unsigned long long x = std::strtoull(v, &end, 10);
  if (end == v || x == 0) return dflt_mib;
  return static_cast<size_t>(x);
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

hipError_t DevBuf::ensure(size_t want) {
  if (want <= bytes) return hipSuccess;
  release();
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    ptr = nullptr;
    return e;
  }
  bytes = want;
  return hipSuccess;
}

hipEvent_t StageTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t StageTimer::begin(hipStream_t s) {
  if (!on) return nullptr;
  hipEvent_t e = get();
  if (e) (void)hipEventRecord(e, s);
  return e;
}

void StageTimer::end(hipEvent_t a, hipStream_t s, int stage) {
  if (!on || !a) return;
  hipEvent_t b = get();
  if (!b) return;
  (void)hipEventRecord(b, s);
  recs.push_back({a, b, stage});
}

void StageTimer::clear() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}

void StageTimer::destroy() {
  clear();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

}  // namespace ftkint

using namespace ftkint;

namespace {

// bf16 bits of a float, round to nearest even (NaN kept quiet)
uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// IEEE binary16 bits of x, round to nearest even (overflow to infinity,
// subnormals kept)
uint16_t f16_rne(double x) {
  if (std::isnan(x)) return 0x7e00;
  const uint16_t sign = std::signbit(x) ? 0x8000 : 0;
  const double a = std::fabs(x);
  if (a >= 65520.0) return sign | 0x7c00;
  if (a < std::ldexp(1.0, -14))  // subnormal: units of 2^-24 (1024 units is the smallest normal)
    return sign | static_cast<uint16_t>(std::nearbyint(a * std::ldexp(1.0, 24)));
  int e;
  const double f = std::frexp(a, &e);  // a = f 2^e, f in [0.5, 1): a = (2f) 2^(e-1)
  uint32_t m = static_cast<uint32_t>(std::nearbyint((2.0 * f - 1.0) * 1024.0));
  int ef = e - 1 + 15;
  if (m == 1024) {
    m = 0;
    ++ef;
  }
  if (ef >= 31) return sign | 0x7c00;
  return sign | static_cast<uint16_t>((ef << 10) | m);
}

// value of finite IEEE binary16 bits: (1024 + m) 2^(e - 25), or m 2^-24 for e = 0
double f16_value(uint16_t h) {
  const int e = (h >> 10) & 31, m = h & 1023;
  const double v = e == 0 ? std::ldexp(static_cast<double>(m), -24) : std::ldexp(static_cast<double>(1024 + m), e - 25);
  return (h & 0x8000) ? -v : v;
}

double bf16_value(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int build_tables(int n, int M, double W, double eps, HostTables& t, const ftkplan::Weight& weight,
                 const ftkplan::Ctf& ctf) {
  const double kmax = 0.5 * kPi * n;
  ftkplan::radial_rule(M, kmax, t.k, t.w);
  t.tr = ftkplan::truncate(kPi * W, eps, weight, ctf);
  t.L = t.tr.L;
  t.sigma_next = t.tr.sigma_next;
  t.H = static_cast<int>(t.tr.terms.size());
  for (const auto& term : t.tr.terms) {
    t.ell.push_back(term.ell);
    t.eta.push_back(term.eta);
    t.sigma.push_back(term.sigma);
  }
  // G[zeta][m] = Sigma v(y_m) = sum_{i,t} sqrt(xw_i tw_t) J_l(x_i y_m) C(y_m; tau_t) U[(i, t)][eta]
  // (one tau node and C = 1 without a CTF); every mode shares the nodes
  t.G.assign(static_cast<size_t>(t.H) * M, 0.0);
  const ftkplan::ModalSVD& s0 = t.tr.svds[0];
  const int P = s0.P, Pt = s0.Pt, Py = s0.Py;
  std::vector<double> J(static_cast<size_t>(t.L + 1) * P);
  std::vector<double> tmp(t.L + 1), c(Pt, 1.0);
  for (int m = 0; m < M; ++m) {
    const double y = t.k[m] / kmax;
    for (int i = 0; i < P; ++i) {
      ftkplan::bessel_orders(t.L, s0.xn[i] * y, tmp.data());
      for (int l = 0; l <= t.L; ++l) J[static_cast<size_t>(l) * P + i] = tmp[l];
    }
    if (s0.ctf.on)
      for (int q = 0; q < Pt; ++q) c[q] = s0.ctf(y, s0.tn[q]) * std::sqrt(s0.tw[q]);
    for (int z = 0; z < t.H; ++z) {
      const int la = std::abs(t.ell[z]);
      const ftkplan::ModalSVD& s = t.tr.svds[la];
      double acc = 0.0;
      for (int i = 0; i < P; ++i)
        for (int q = 0; q < Pt; ++q)
          acc += std::sqrt(s.xw[i]) * c[q] * J[static_cast<size_t>(la) * P + i] *
                 s.U[static_cast<size_t>(i * Pt + q) * Py + t.eta[z]];
      if (t.ell[z] < 0 && (la & 1)) acc = -acc;
      t.G[static_cast<size_t>(z) * M + m] = acc;
    }
  }
  return FTK_OK;
}

// Y[delta][zeta] = u_zeta(pi |d|, tau) exp(-i l (omega + pi/2)), d in
// pixels, tau the pose's defocus (defocus NULL: plans without a CTF).
int build_Y(const HostTables& t, const double* shifts, const double* defocus, int N, double W,
            std::vector<std::complex<double>>& Y) {
  const ftkplan::ModalSVD& s0 = t.tr.svds[0];
  const int Py = s0.Py;
  if (s0.ctf.on && !defocus) return fail(FTK_ESTATE, "ftk_set_poses: a plan with a CTF needs a defocus per pose");
  if (!s0.ctf.on && defocus) return fail(FTK_EINVAL, "ftk_set_poses: defocus given to a plan without a CTF");
  Y.assign(static_cast<size_t>(N) * t.H, 0.0);
  std::vector<double> J(static_cast<size_t>(t.L + 1) * Py), tmp(t.L + 1), cy(Py, 1.0);
  for (int d = 0; d < N; ++d) {
    const double dx = shifts[2 * d], dy = shifts[2 * d + 1];
    if (!std::isfinite(dx) || !std::isfinite(dy)) return fail(FTK_EINVAL, "ftk_set_shifts: non-finite shift");
    const double rad = std::hypot(dx, dy);
    if (rad > W * (1.0 + 1e-9)) return fail(FTK_ERANGE, "ftk_set_shifts: shift outside the planned disk");
    if (defocus) {
      const double tau = defocus[d];
      const double span = s0.ctf.tmax - s0.ctf.tmin;
      if (!std::isfinite(tau) || tau < s0.ctf.tmin - 1e-9 * span || tau > s0.ctf.tmax + 1e-9 * span)
        return fail(FTK_ERANGE, "ftk_set_poses: defocus outside the planned range");
      for (int j = 0; j < Py; ++j) cy[j] = s0.ctf(s0.yn[j], tau);
    }
    const double om = std::atan2(dy, dx);
    const double x = kPi * rad;
    for (int j = 0; j < Py; ++j) {
      ftkplan::bessel_orders(t.L, x * s0.yn[j], tmp.data());
      for (int l = 0; l <= t.L; ++l) J[static_cast<size_t>(l) * Py + j] = tmp[l];
    }
    for (int z = 0; z < t.H; ++z) {
      const int la = std::abs(t.ell[z]);
      const ftkplan::ModalSVD& s = t.tr.svds[la];
      double acc = 0.0;
      for (int j = 0; j < Py; ++j)
        acc += std::sqrt(s.yw[j]) * J[static_cast<size_t>(la) * Py + j] * cy[j] * s.V[static_cast<size_t>(j) * Py + t.eta[z]];
      const double u = acc / s.sigma[t.eta[z]];
      const double ph = -t.ell[z] * (om + 0.5 * kPi);
      Y[static_cast<size_t>(d) * t.H + z] = std::complex<double>(u * std::cos(ph), u * std::sin(ph));
    }
  }
  return FTK_OK;
}

template <class T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
  hipError_t e = b.ensure(v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

std::vector<float> twiddles(int L) {
  std::vector<float> t(2 * L);
  for (int k = 0; k < L; ++k) {
    const double a = -2.0 * kPi * k / L;
    t[2 * k] = static_cast<float>(std::cos(a));
    t[2 * k + 1] = static_cast<float>(std::sin(a));
  }
  return t;
}

// power of two at or above x > 0 (1 for x = 0)
double pow2_at_or_above(double x) {
  if (!(x > 0.0)) return 1.0;
  int e;
  const double f = std::frexp(x, &e);  // x = f 2^e, f in [0.5, 1)
  return std::ldexp(1.0, f == 0.5 ? e - 1 : e);
}

// The FP16 form's rotation transform tables T_E, T_O (the real map from the
// packed modes to the rotations r < Qa/2, split by the parity of the mode),
// fp16, as the A-operand fragments of the 16x16x32 MFMA in the K order of the
// two-tile Step 3 (kernels.h): fragment (parity, row tile t, K step s), lane
// l, element e holds the entry of rotation r = 16 t + l % 16 and mode q =
// 32 s + 8 (e / 2) + 4 (g / 2) + 2 (e % 2) + parity, part c = g % 2
// (g = l / 16).
std::vector<uint16_t> rotation_tables_f16(int Qa) {
  const int QH = Qa / 2, NT = QH / 16, NS = QH / 32;
  std::vector<uint16_t> out(static_cast<size_t>(2) * NT * NS * 64 * 8);
  for (int par = 0; par < 2; ++par)
    for (int t = 0; t < NT; ++t)
      for (int s = 0; s < NS; ++s)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int r = 16 * t + l % 16;
            const int g = l / 16, c = g % 2;
            const int q = 32 * s + 8 * (e / 2) + 4 * (g / 2) + 2 * (e % 2) + par;
            double v;
            if (q == 0) {
              v = c == 0 ? 1.0 : ((r & 1) ? -1.0 : 1.0);
            } else {
              // angle 2 pi q r / Qa, reduced exactly in integers first
              const double th = 2.0 * kPi * static_cast<double>((static_cast<long>(q) * r) % Qa) / Qa;
              v = 2.0 * (c == 0 ? std::cos(th) : std::sin(th));
            }
            out[((static_cast<size_t>(par * NT + t) * NS + s) * 64 + l) * 8 + e] = f16_rne(v);
          }
  return out;
}

int upload_plan_tables(ftk_plan* p) {
  const int M = p->M, H = p->t.H, Hp = p->H_pad;
  std::vector<float> cz(static_cast<size_t>(Hp) * M, 0.f);
  std::vector<int> ell(Hp, 0);
  p->zeta_scale.assign(Hp, 1.f);
  for (int z = 0; z < H; ++z) {
    ell[z] = p->t.ell[z];
    double sg = 1.0;
    if (p->precision == FTK_FP16 || p->precision == FTK_FP16X3) {
      // the fp16 forms store the row divided by the power of two at or above
      // its largest entry; the shift panel carries that factor
      double mx = 0.0;
      for (int m = 0; m < M; ++m)
        mx = std::max(mx, std::fabs(2.0 * kPi * p->t.w[m] * p->t.G[static_cast<size_t>(z) * M + m]));
      sg = pow2_at_or_above(mx);
      p->zeta_scale[z] = static_cast<float>(sg);
    }
    for (int m = 0; m < M; ++m)
      cz[static_cast<size_t>(z) * M + m] =
          static_cast<float>(2.0 * kPi * p->t.w[m] * p->t.G[static_cast<size_t>(z) * M + m] / sg);
  }
  // NUFFT: deapodisation with all scale factors, and per-point kernel weights
  const int n = p->n, nf = p->sk.nf, w = p->sk.w, Qa = p->Qa, half = Qa / 2;
  const double dx = 2.0 / n;
  std::vector<float> dea(n);
  const double scale = dx * p->sk.h / std::sqrt(static_cast<double>(Qa));
  for (int i = 0; i < n; ++i) dea[i] = static_cast<float>(scale / p->sk.ft(i - n / 2));
  std::vector<int> pb(static_cast<size_t>(M) * half * 2);
  std::vector<float> pk(static_cast<size_t>(M) * half * 2 * w);
  for (int m = 0; m < M; ++m)
    for (int q = 0; q < half; ++q) {
      const double psi = 2.0 * kPi * q / Qa;
      const double t[2] = {p->t.k[m] * std::cos(psi) * dx, p->t.k[m] * std::sin(psi) * dx};
      const size_t pt = static_cast<size_t>(m) * half + q;
      for (int d = 0; d < 2; ++d) {
        const double u = t[d] / p->sk.h;
        const long base = static_cast<long>(std::floor(u)) - w / 2 + 1;
        long bm = base % nf;
        if (bm < 0) bm += nf;
        pb[2 * pt + d] = static_cast<int>(bm);
        for (int a = 0; a < w; ++a) {
          const double z = (u - static_cast<double>(base + a)) / (0.5 * w);
          double v = 0.0;
          if (std::fabs(z) < 1.0) v = std::exp(p->sk.beta * (std::sqrt(1.0 - z * z) - 1.0));
          pk[(pt * 2 + d) * w + a] = static_cast<float>(v);
        }
      }
    }
  hipError_t e;
  if ((e = upload(p->cz, cz)) != hipSuccess) return hip_fail(e, "upload cz");
  if ((e = upload(p->ell, ell)) != hipSuccess) return hip_fail(e, "upload ell");
  {
    // brute-force translations: 2 pi w_m
    std::vector<float> bcz(M);
    for (int m = 0; m < M; ++m) bcz[m] = static_cast<float>(2.0 * kPi * p->t.w[m]);
    if ((e = upload(p->bft_cz, bcz)) != hipSuccess) return hip_fail(e, "upload bft_cz");
  }
  if ((e = upload(p->tw_nf, twiddles(nf))) != hipSuccess) return hip_fail(e, "upload tw_nf");
  if ((e = upload(p->tw_qa, twiddles(Qa))) != hipSuccess) return hip_fail(e, "upload tw_qa");
  if ((e = upload(p->deapod, dea)) != hipSuccess) return hip_fail(e, "upload deapod");
  if ((e = upload(p->ptbase, pb)) != hipSuccess) return hip_fail(e, "upload ptbase");
  if ((e = upload(p->ptker, pk)) != hipSuccess) return hip_fail(e, "upload ptker");
  if (p->precision == FTK_FP16 && rot16_table_bytes(Qa) > 0) {
    if ((e = upload(p->rot16, rotation_tables_f16(Qa))) != hipSuccess) return hip_fail(e, "upload rot16");
  }
  return FTK_OK;
}

int check_plan_args(int n, int K, int Q, double W, double eps, int precision) {
  if (n < 4 || n > 1024 || (n & 1)) return fail(FTK_EINVAL, "n must be even and in [4, 1024]");
  if (K < 1 || K > 512) return fail(FTK_EINVAL, "K (radial nodes) must be in [1, 512]");
  if (Q < 8 || Q > 4096 || (Q & 1)) return fail(FTK_EINVAL, "Q must be even and in [8, 4096]");
  if (!(W > 0.0) || W > n / 4.0) return fail(FTK_EINVAL, "W (shift radius, px) must be in (0, n/4]");
  if (!(eps > 0.0) || !(eps < 1.0)) return fail(FTK_EINVAL, "eps must be in (0, 1)");
  if (precision != FTK_FP32 && precision != FTK_BF16X3 && precision != FTK_FP16 && precision != FTK_FP16X3)
    return fail(FTK_EINVAL, "unknown precision");
  if (precision != FTK_FP32 && K % 8 != 0)
    return fail(FTK_EUNSUPPORTED, "the bf16x3 and fp16 forms need K (radial nodes) to be a multiple of 8");
  if (!ftkplan::fft_supported(Q) || Q % 64 != 0 || Q > 384)
    return fail(FTK_EUNSUPPORTED, "Q must be a multiple of 64 of the form 2^a 3^b, at most 384");
  const int nf = ftkplan::fft_size(2 * n);
  if (nf <= 0 || nf > 4096) return fail(FTK_EUNSUPPORTED, "image too large for the transform");
  return FTK_OK;
}

}  // namespace

namespace ftkint {

ftk_tuning_t default_tuning(int precision) {
  ftk_tuning_t t;
  t.step3_waves = static_cast<int>(std::min<size_t>(16, env_mib("FTK_STEP3_WAVES", 16)));
  // the FP16 form's Step 1 is faster with 64 SVD terms per workgroup
  t.step1_zblk = env_mib("FTK_STEP1_ZBLK", precision == FTK_FP16 ? 64 : 128) == 64 ? 64 : 128;
  t.step1_wgs = static_cast<int>(std::min<size_t>(65536, std::max<size_t>(64, env_mib("FTK_STEP1_WGS", 4096))));
  t.stage_mib = static_cast<int>(std::min<size_t>(65536, std::max<size_t>(16, env_mib("FTK_STAGE_MB", 8192))));
  return t;
}

int step3_waves(const ftk_plan* p) {
  const int units = (p->N + 15) / 16;
  // each wave owns 16 shifts; more than 8 waves only below Qa = 320, where
  // the staging and FFT buffers of 16 waves still fit LDS
  int maxw = std::max(1, std::min(p->tune.step3_waves, (p->Qa / 64 > 4) ? 8 : 16));
  const int prec = prec_code(p);
  auto lds = [&](int w) {
    return (prec == 1 || prec == 3) ? step3_bf16_lds_bytes(p->Qa, w)
                     : (prec == 2 ? (p->rot16.ptr ? step3_fp16_rot_lds_bytes(p->Qa, w) : step3_fp16_lds_bytes(p->Qa, w))
                                  : step3_lds_bytes(p->Qa, w));
  };
  while (maxw > 1 && lds(maxw) > kLdsLimit) --maxw;
  const int nblk = (units + maxw - 1) / maxw;
  return (units + nblk - 1) / nblk;
}

int step1_zblk(const ftk_plan* p) {
  const int prec = prec_code(p);
  int z = p->tune.step1_zblk;
  if (p->H_pad % z != 0 || step1_v2_lds_bytes(p->M, z, prec) > kLdsLimit) z = 64;
  return z;
}

Needs plan_needs(const ftk_plan* p, int nA, int nB, bool from_pixels) {
  Needs d;
  const size_t n = p->n, nf = p->sk.nf;
  const size_t cb = static_cast<size_t>(8) * p->M * p->Qa;
  if (from_pixels) {
    const int cnt = std::max(nA, nB);
    const size_t per_img = (n * nf + nf * nf) * sizeof(float2);
    const size_t budget = env_mib("FTK_TRANSFORM_SCRATCH_MB", 4096) << 20;
    d.transform_chunk = static_cast<int>(std::min<size_t>(std::max<size_t>(1, budget / per_img), std::max(cnt, 1)));
    d.tr_h = static_cast<size_t>(d.transform_chunk) * n * nf * sizeof(float2);
    d.tr_g = static_cast<size_t>(d.transform_chunk) * nf * nf * sizeof(float2);
    d.coef_a = cb * nA;
    d.coef_b = cb * nB;
  }
  if (nA > 0 && nB > 0) {
    const size_t per_pair = stage_bytes_per_pair(p) + xhat_bytes_per_pair(p);
    const size_t budget = static_cast<size_t>(p->tune.stage_mib) << 20;
    d.chunk_images = static_cast<int>(std::min<size_t>(nA, std::max<size_t>(1, budget / (per_pair * nB))));
    d.stage = static_cast<size_t>(d.chunk_images) * nB * stage_bytes_per_pair(p);
    d.xhat = static_cast<size_t>(d.chunk_images) * nB * xhat_bytes_per_pair(p);
    d.keys = static_cast<size_t>(nA) * nB * sizeof(unsigned long long);
    d.tmpl = tmpl_prep_bytes(nB, p->M, p->Qa, prec_code(p));
    d.scales = (prec_code(p) == 2 || prec_code(p) == 3) ? 64 : 0;
  }
  return d;
}

Needs plan_needs_lists(const ftk_plan* p, int nA, int K) {
  Needs d;
  if (nA <= 0 || K <= 0) return d;
  const size_t per_pair = stage_bytes_per_pair(p) + xhat_bytes_per_pair(p);
  const size_t budget = static_cast<size_t>(p->tune.stage_mib) << 20;
  d.chunk_images = static_cast<int>(std::min<size_t>(nA, std::max<size_t>(1, budget / (per_pair * K))));
  d.stage = static_cast<size_t>(d.chunk_images) * K * stage_bytes_per_pair(p);
  d.xhat = static_cast<size_t>(d.chunk_images) * K * xhat_bytes_per_pair(p);
  d.keys = static_cast<size_t>(nA) * K * sizeof(unsigned long long);
  d.tmpl = tmpl_prep_tile_bytes(static_cast<size_t>(d.chunk_images) * ((K + 15) / 16), p->M, p->Qa, prec_code(p));
  d.scales = (prec_code(p) == 2 || prec_code(p) == 3) ? 64 : 0;
  return d;
}

}  // namespace ftkint

extern "C" {

const char* ftk_strerror(int status) {
  switch (status) {
    case FTK_OK: return "FTK_OK";
    case FTK_EINVAL: return "FTK_EINVAL: invalid argument";
    case FTK_ENOMEM: return "FTK_ENOMEM: out of memory";
    case FTK_EDEVICE: return "FTK_EDEVICE: HIP runtime error";
    case FTK_ERANGE: return "FTK_ERANGE: shift outside the planned disk";
    case FTK_ESTATE: return "FTK_ESTATE: call order violated";
    case FTK_EUNSUPPORTED: return "FTK_EUNSUPPORTED: size not supported";
    default: return "unknown ftk status";
  }
}

const char* ftk_last_error_message(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

ftkplan::Ctf ctf_of(const ftk_ctf_t* c) {
  if (!c) return ftkplan::Ctf();
  return ftkplan::make_ctf(c->wavelength_A, c->cs_mm, c->amplitude_contrast, c->pixel_A, c->defocus_min_A,
                           c->defocus_max_A);
}

int plan_tables_impl(int n, int K, double W, double eps, const double* alpha, const double* beta, int nterms,
                     const ftk_ctf_t* ctf, const double* shifts_px, const double* defocus, int N, int* H_out,
                     int32_t* ell, double* sigma, double* G, double* k, double* w, double* Y, double* sigma_next) {
  if (n < 4 || K < 1 || K > 512 || !(W > 0) || !(eps > 0) || !(eps < 1) || N < 0 || (N > 0 && !shifts_px) ||
      nterms < 0 || nterms > 4096 || (ctf && nterms > 0))
    return fail(FTK_EINVAL, "ftk_plan_tables: invalid argument");
  try {
    HostTables t;
    build_tables(n, K, W, eps, t, ftkplan::make_weight(alpha, beta, nterms), ctf_of(ctf));
    if (H_out) *H_out = t.H;
    if (sigma_next) *sigma_next = t.sigma_next;
    for (int z = 0; z < t.H; ++z) {
      if (ell) ell[z] = t.ell[z];
      if (sigma) sigma[z] = t.sigma[z];
    }
    if (G) std::memcpy(G, t.G.data(), t.G.size() * sizeof(double));
    if (k) std::memcpy(k, t.k.data(), K * sizeof(double));
    if (w) std::memcpy(w, t.w.data(), K * sizeof(double));
    if (Y && N > 0) {
      std::vector<std::complex<double>> Yc;
      int rc = build_Y(t, shifts_px, defocus, N, W, Yc);
      if (rc != FTK_OK) return rc;
      std::memcpy(Y, Yc.data(), Yc.size() * sizeof(std::complex<double>));
    }
  } catch (const std::bad_alloc&) {
    return fail(FTK_ENOMEM, "ftk_plan_tables: host allocation failed");
  } catch (const std::exception& ex) {
    return fail(FTK_EINVAL, std::string("ftk_plan_tables: ") + ex.what());
  }
  return FTK_OK;
}

int plan_create_impl(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision, const double* alpha,
                     const double* beta, int nterms, const ftk_ctf_t* ctf) {
  if (!out) return fail(FTK_EINVAL, "ftk_plan_create: out is NULL");
  *out = nullptr;
  int rc = check_plan_args(n, K, Q, W, eps, precision);
  if (rc != FTK_OK) return rc;
  if (nterms < 0 || nterms > 4096 || (nterms > 0 && (!alpha || !beta)))
    return fail(FTK_EINVAL, "ftk_plan_create_weighted: nterms must be in [0, 4096] with alpha and beta given");
  if (ctf && nterms > 0) return fail(FTK_EINVAL, "ftk_plan_create: a k-side weight and a CTF together");
  ftk_plan* p = nullptr;
  try {
    p = new ftk_plan();
    p->n = n;
    p->M = K;
    p->Qa = Q;
    p->W = W;
    p->eps = eps;
    p->precision = precision;
    p->kmax = 0.5 * kPi * n;
    p->tune = default_tuning(precision);
    p->weighted = nterms > 0;
    p->has_ctf = ctf != nullptr;
    build_tables(n, K, W, eps, p->t, ftkplan::make_weight(alpha, beta, nterms), ctf_of(ctf));
    p->H_pad = round_up(std::max(p->t.H, 1), 64);
    p->sk = ftkplan::spread_kernel(n, kNufftWidth);
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(FTK_ENOMEM, "ftk_plan_create: host allocation failed");
  } catch (const std::exception& ex) {
    delete p;
    return fail(FTK_EINVAL, std::string("ftk_plan_create: ") + ex.what());
  }
  rc = upload_plan_tables(p);
  if (rc != FTK_OK) {
    p->release_all();
    delete p;
    return rc;
  }
  *out = p;
  return FTK_OK;
}

int set_poses_impl(ftk_plan* p, const double* shifts_px, const double* defocus, int N);

}  // namespace

extern "C" {

int ftk_plan_tables_weighted(int n, int K, double W, double eps, const double* alpha, const double* beta,
                             int nterms, const double* shifts_px, int N, int* H_out, int32_t* ell, double* sigma,
                             double* G, double* k, double* w, double* Y, double* sigma_next) {
  return plan_tables_impl(n, K, W, eps, alpha, beta, nterms, nullptr, shifts_px, nullptr, N, H_out, ell, sigma, G,
                          k, w, Y, sigma_next);
}

int ftk_plan_tables_ctf(int n, int K, double W, double eps, const ftk_ctf_t* ctf, const double* shifts_px,
                        const double* defocus_A, int N, int* H_out, int32_t* ell, double* sigma, double* G, double* k,
                        double* w, double* Y, double* sigma_next) {
  if (!ctf) return fail(FTK_EINVAL, "ftk_plan_tables_ctf: NULL ctf");
  if (N > 0 && !defocus_A) return fail(FTK_EINVAL, "ftk_plan_tables_ctf: NULL defocus");
  return plan_tables_impl(n, K, W, eps, nullptr, nullptr, 0, ctf, shifts_px, defocus_A, N, H_out, ell, sigma, G, k,
                          w, Y, sigma_next);
}

int ftk_plan_tables(int n, int K, double W, double eps, const double* shifts_px, int N, int* H_out, int32_t* ell,
                    double* sigma, double* G, double* k, double* w, double* Y, double* sigma_next) {
  return ftk_plan_tables_weighted(n, K, W, eps, nullptr, nullptr, 0, shifts_px, N, H_out, ell, sigma, G, k, w, Y,
                                  sigma_next);
}

int ftk_plan_create(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision) {
  return ftk_plan_create_weighted(out, n, K, Q, W, eps, precision, nullptr, nullptr, 0);
}

int ftk_plan_create_weighted(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision,
                             const double* alpha, const double* beta, int nterms) {
  return plan_create_impl(out, n, K, Q, W, eps, precision, alpha, beta, nterms, nullptr);
}

int ftk_plan_create_ctf(ftk_plan** out, int n, int K, int Q, double W, double eps, int precision,
                        const ftk_ctf_t* ctf) {
  if (!ctf) return fail(FTK_EINVAL, "ftk_plan_create_ctf: NULL ctf");
  return plan_create_impl(out, n, K, Q, W, eps, precision, nullptr, nullptr, 0, ctf);
}

void ftk_plan_destroy(ftk_plan* p) {
  if (!p) return;
  p->timer.destroy();
  p->release_all();
  delete p;
}

int ftk_plan_info(const ftk_plan* p, ftk_plan_info_t* o) {
  if (!p || !o) return fail(FTK_EINVAL, "ftk_plan_info: NULL argument");
  o->n = p->n;
  o->M = p->M;
  o->Qa = p->Qa;
  o->H = p->t.H;
  o->L = p->t.L;
  o->N = p->N;
  o->precision = p->precision;
  o->nufft_width = p->sk.w;
  o->nufft_grid = p->sk.nf;
  o->shift_radius_px = p->W;
  o->eps = p->eps;
  o->sigma_next = p->t.sigma_next;
  o->kmax = p->kmax;
  o->coeff_bytes_per_image = static_cast<size_t>(8) * p->M * p->Qa;
  o->device_bytes = p->device_bytes();
  o->weighted = p->weighted ? 1 : 0;
  o->rotations = p->Qa * p->up;
  o->ctf = p->has_ctf ? 1 : 0;
  return FTK_OK;
}

int ftk_plan_set_rotations(ftk_plan* p, int upsample) {
  if (!p) return fail(FTK_EINVAL, "ftk_plan_set_rotations: NULL plan");
  if (upsample < 1 || upsample > 16) return fail(FTK_EINVAL, "ftk_plan_set_rotations: upsample must be in [1, 16]");
  p->up = upsample;
  return FTK_OK;
}

int ftk_set_shifts(ftk_plan* p, const double* shifts_px, int N) {
  if (!p || !shifts_px) return fail(FTK_EINVAL, "ftk_set_shifts: NULL argument");
  if (p->has_ctf) return fail(FTK_ESTATE, "ftk_set_shifts: the plan has a CTF; use ftk_set_poses");
  return set_poses_impl(p, shifts_px, nullptr, N);
}

int ftk_plan_set_shift_windows(ftk_plan* p, const double* centers_px, int nw, double half_width_px) {
  if (!p) return fail(FTK_EINVAL, "ftk_plan_set_shift_windows: NULL plan");
  if (p->N <= 0 || p->shifts.empty()) return fail(FTK_ESTATE, "ftk_plan_set_shift_windows: call ftk_set_shifts first");
  if (p->has_ctf) return fail(FTK_EUNSUPPORTED, "ftk_plan_set_shift_windows: plans with a CTF are not supported");
  if (nw < 0 || nw > 1024 || (nw > 0 && !centers_px))
    return fail(FTK_EINVAL, "ftk_plan_set_shift_windows: nw must be in [0, 1024] with centres given");
  if (nw > 0 && !(half_width_px > 0.0 && std::isfinite(half_width_px)))
    return fail(FTK_EINVAL, "ftk_plan_set_shift_windows: half_width must be positive");
  for (auto& w : p->windows) w.release();
  p->windows.clear();
  std::vector<ShiftWindow> ws(nw);
  auto undo = [&](int rc) {
    for (auto& w : ws) w.release();
    return rc;
  };
  for (int b = 0; b < nw; ++b) {
    const double c = centers_px[b];
    if (!std::isfinite(c) || c < 0.0) return undo(fail(FTK_EINVAL, "ftk_plan_set_shift_windows: bad centre"));
    std::vector<double> sub;
    for (int i = 0; i < p->N; ++i) {
      const double r = std::hypot(p->shifts[2 * i], p->shifts[2 * i + 1]);
      if (std::fabs(r - c) <= half_width_px * (1.0 + 1e-12)) {
        ws[b].idx.push_back(i);
        sub.push_back(p->shifts[2 * i]);
        sub.push_back(p->shifts[2 * i + 1]);
      }
    }
    if (ws[b].idx.empty())
      return undo(fail(FTK_EINVAL, "ftk_plan_set_shift_windows: window " + std::to_string(b) + " holds no shift"));
    int rc = build_panels(p, sub.data(), nullptr, static_cast<int>(ws[b].idx.size()), ws[b].pan);
    if (rc != FTK_OK) return undo(rc);
    hipError_t e = upload(ws[b].didx, ws[b].idx);
    if (e != hipSuccess) return undo(hip_fail(e, "ftk_plan_set_shift_windows: upload"));
  }
  p->windows = std::move(ws);
  return FTK_OK;
}

int ftk_set_poses(ftk_plan* p, const double* shifts_px, const double* defocus_A, int N) {
  if (!p || !shifts_px) return fail(FTK_EINVAL, "ftk_set_poses: NULL argument");
  if (p->has_ctf != (defocus_A != nullptr))
    return fail(FTK_EINVAL, p->has_ctf ? "ftk_set_poses: a plan with a CTF needs a defocus per pose"
                           : "ftk_set_poses: defocus given to a plan without a CTF");
  return set_poses_impl(p, shifts_px, defocus_A, N);
}

}  // extern "C"

namespace ftkint {

// The shift-side device panels of a pose list (Y embedded for Step 3 in the
// plan's precision form, the brute-force (k dx, k dy) table), into out.
int build_panels(const ftk_plan* p, const double* shifts_px, const double* defocus, int N, ShiftPanels& out) {
  if (N < 1 || N > 65536) return fail(FTK_EINVAL, "ftk_set_shifts: N must be in [1, 65536]");
  std::vector<std::complex<double>> Y;
  try {
    int rc = build_Y(p->t, shifts_px, defocus, N, p->W, Y);
    if (rc != FTK_OK) return rc;
  } catch (const std::bad_alloc&) {
    return fail(FTK_ENOMEM, "ftk_set_shifts: host allocation failed");
  }
  const int H = p->t.H, Hp = p->H_pad;
  const int Np = round_up(N, 16);
  // real embedding of Y, transposed: yt[k'][2 delta + c] with the K index
  // k' = c' H_pad + zeta matching the staged Zhat rows [q][c'][zeta]
  std::vector<float> yt(static_cast<size_t>(2 * Hp) * 2 * Np, 0.f);
  const size_t rs = static_cast<size_t>(2 * Np);
  for (int d = 0; d < N; ++d)
    for (int z = 0; z < H; ++z) {
      const std::complex<double> y = Y[static_cast<size_t>(d) * H + z];
      const float yr = static_cast<float>(y.real()), yi = static_cast<float>(y.imag());
      yt[static_cast<size_t>(z) * rs + 2 * d + 0] = yr;
      yt[static_cast<size_t>(Hp + z) * rs + 2 * d + 0] = -yi;
      yt[static_cast<size_t>(z) * rs + 2 * d + 1] = yi;
      yt[static_cast<size_t>(Hp + z) * rs + 2 * d + 1] = yr;
    }
  hipError_t e = upload(out.yt, yt);
  if (e != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
  // reduced-precision copies in MFMA lane order: [row tile][K step][lane][8],
  // row tile = 32 embedded rows (16 shifts), K step = 16 embedded terms; lane
  // l holds row l % 32 and k = 8 (l / 32) .. +7 of the step
  const int nrt = 2 * Np / 32, nks = 2 * Hp / 16;
  // the FP64 value of an embedded entry, times sg_zeta in the fp16 forms
  auto entry = [&](int row, int k) {
    const int d = row >> 1, z = k % Hp;
    if (d >= N || z >= H) return 0.0;
    const std::complex<double> y = Y[static_cast<size_t>(d) * H + z];
    const int c = row & 1, cp = k / Hp;
    return ((c == cp) ? y.real() : (c == 0 ? -y.imag() : y.imag())) * p->zeta_scale[z];
  };
  auto at = [&](int rt, int ks, int l, int e8) { return ((static_cast<size_t>(rt) * nks + ks) * 64 + l) * 8 + e8; };
  if (p->precision == FTK_BF16X3) {
    // split hi/lo bf16 copies
    std::vector<uint16_t> hi(static_cast<size_t>(nrt) * nks * 512), lo(hi.size());
    for (int rt = 0; rt < nrt; ++rt)
      for (int ks = 0; ks < nks; ++ks)
        for (int l = 0; l < 64; ++l)
          for (int e8 = 0; e8 < 8; ++e8) {
            const double v = entry(rt * 32 + (l & 31), ks * 16 + 8 * (l >> 5) + e8);
            const size_t i = at(rt, ks, l, e8);
            hi[i] = bf16_rne(static_cast<float>(v));
            lo[i] = bf16_rne(static_cast<float>(v - bf16_value(hi[i])));
          }
    if ((e = upload(out.yt_hi, hi)) != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
    if ((e = upload(out.yt_lo, lo)) != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
  }
  if (p->precision == FTK_FP16 || p->precision == FTK_FP16X3) {
    // fp16 panel, column zeta multiplied by sg_zeta and the whole panel
    // divided by the power of two s_y at or above its largest entry; the
    // split fp16 form also keeps lo = fp16(v - hi), rounded from FP64
    double mx = 0.0;
    for (int row = 0; row < 2 * N; ++row)
      for (int k = 0; k < 2 * Hp; ++k) mx = std::max(mx, std::fabs(entry(row, k)));
    const double sy = pow2_at_or_above(mx);
    const bool split = p->precision == FTK_FP16X3;
    // the FP16 form's two-tile Step 3 (Qa <= 256) takes the panel as the B
    // operand of its transposed contraction: column rho = 16 c + dl of a
    // shift tile instead of row 2 dl + c
    const bool jcol = !split && rot16_table_bytes(p->Qa) > 0;
    // the split form lifts the panel to the top of the fp16 range (its lo
    // parts then stay normal numbers down to 2^-18 of the largest entry)
    const double ysc = split ? std::ldexp(1.0, split_f16_exps(p->M).data) : 1.0;
    std::vector<uint16_t> h16(static_cast<size_t>(nrt) * nks * 512), l16(split ? h16.size() : 0);
    for (int rt = 0; rt < nrt; ++rt)
      for (int ks = 0; ks < nks; ++ks)
        for (int l = 0; l < 64; ++l)
          for (int e8 = 0; e8 < 8; ++e8) {
            const int rho = l & 31;
            const int row = jcol ? 2 * (rt * 16 + (rho & 15)) + (rho >> 4) : rt * 32 + rho;
            const double v = entry(row, ks * 16 + 8 * (l >> 5) + e8) / sy * ysc;
            const size_t i = at(rt, ks, l, e8);
            h16[i] = f16_rne(v);
            if (split) l16[i] = f16_rne(v - f16_value(h16[i]));
          }
    if ((e = upload(out.yt_hi, h16)) != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
    if (split && (e = upload(out.yt_lo, l16)) != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
    out.y_scale = static_cast<float>(sy);
  }
  {
    // brute-force translations: (k_m dx, k_m dy), the shift in image units
    const int M = p->M;
    const double px = 2.0 / p->n;
    std::vector<float> kd(static_cast<size_t>(2) * N * M);
    for (int d = 0; d < N; ++d)
      for (int m = 0; m < M; ++m) {
        kd[2 * (static_cast<size_t>(d) * M + m) + 0] = static_cast<float>(p->t.k[m] * shifts_px[2 * d] * px);
        kd[2 * (static_cast<size_t>(d) * M + m) + 1] = static_cast<float>(p->t.k[m] * shifts_px[2 * d + 1] * px);
      }
    if ((e = upload(out.kd, kd)) != hipSuccess) return hip_fail(e, "ftk_set_shifts: upload");
  }
  out.N = N;
  out.N_pad = Np;
  return FTK_OK;
}

// swap the plan's shift-side panels with a set
void swap_panels(ftk_plan* p, ShiftPanels& w) {
  std::swap(p->yt, w.yt);
  std::swap(p->yt_hi, w.yt_hi);
  std::swap(p->yt_lo, w.yt_lo);
  std::swap(p->bft_kd, w.kd);
  std::swap(p->N, w.N);
  std::swap(p->N_pad, w.N_pad);
  std::swap(p->y_scale, w.y_scale);
}

}  // namespace ftkint

namespace {

int set_poses_impl(ftk_plan* p, const double* shifts_px, const double* defocus, int N) {
  ShiftPanels sp;
  int rc = build_panels(p, shifts_px, defocus, N, sp);
  if (rc != FTK_OK) {
    sp.release();
    return rc;
  }
  swap_panels(p, sp);
  sp.release();  // the previous panels
  p->shifts.assign(shifts_px, shifts_px + 2 * static_cast<size_t>(N));
  for (auto& w : p->windows) w.release();  // windows refer to the previous shift list
  p->windows.clear();
  return FTK_OK;
}

}  // namespace

extern "C" {

int ftk_transform(ftk_plan* p, const float* imgs, int cnt, void* coeffs, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_transform: NULL plan");
  if (cnt < 0) return fail(FTK_EINVAL, "ftk_transform: cnt < 0");
  if (cnt == 0) return FTK_OK;
  if (!imgs || !coeffs) return fail(FTK_EINVAL, "ftk_transform: NULL buffer");
  return transform_run(p, imgs, cnt, static_cast<float2*>(coeffs), nullptr, stream);
}

}  // extern "C"

namespace ftkint {

int transform_run(ftk_plan* p, const float* imgs, int cnt, float2* coeffs, float2* polar, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = p->n, nf = p->sk.nf;
  const Needs nd = plan_needs(p, cnt, 0, true);
  const int chunk = nd.transform_chunk;
  Workspace& ws = *p->ws;
  if (ws.tr_h.ensure(nd.tr_h) != hipSuccess || ws.tr_g.ensure(nd.tr_g) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_transform: scratch");
  if (transform_lds_bytes(nf, p->Qa, transform_waves(nf, p->Qa)) > kLdsLimit) return fail(FTK_EUNSUPPORTED, "ftk_transform: LDS");
  hipError_t e;
  for (int c0 = 0; c0 < cnt; c0 += chunk) {
    const int c = std::min(chunk, cnt - c0);
    TransformArgs a;
    a.imgs = imgs + static_cast<size_t>(c0) * n * n;
    a.coeffs = coeffs + static_cast<size_t>(c0) * p->Qa * p->M;
    a.polar = polar ? polar + static_cast<size_t>(c0) * p->Qa * p->M : nullptr;
    a.scratchH = ws.tr_h.as<float2>();
    a.scratchG = ws.tr_g.as<float2>();
    a.deapod = p->deapod.as<float>();
    a.tw_nf = p->tw_nf.as<float2>();
    a.tw_qa = p->tw_qa.as<float2>();
    a.pt_base = p->ptbase.as<int>();
    a.pt_ker = p->ptker.as<float>();
    a.n = n;
    a.nf = nf;
    a.M = p->M;
    a.Qa = p->Qa;
    a.w = p->sk.w;
    hipEvent_t ev = p->timer.begin(s);
    if ((e = launch_transform(a, c, s)) != hipSuccess) return hip_fail(e, "ftk_transform: launch");
    p->timer.end(ev, s, 0);
  }
  return FTK_OK;
}

// Steps 1-3 + argmax for nA images against nB templates (lists == NULL) or
// against K templates of their own (lists [nA][K]); results per pair
// (image, template or list slot) in X [.][N][Qa] and best.  The buffers
// are the caller's (sized by plan_needs / plan_needs_lists, or carved from
// the no-allocation scratch); tm (null: no timing) records the launches.
int align_run(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB, const int32_t* lists,
              int K, float* X, ftk_pose* best, const AlignBufs& buf, StageTimer* tm, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int QH = p->Qa / 2;
  const int nBe = lists ? K : nB;  // templates per image
  const size_t pairs = static_cast<size_t>(nA) * nBe;
  const int prec = prec_code(p);
  const int chunkA = buf.chunk_images;
  if (chunkA < 1) return fail(FTK_EINVAL, "ftk_align: no staging for one image");
  const int U = p->up;
  if (U > 1 && prec == 2)
    return fail(FTK_EUNSUPPORTED, "ftk_align: rotation upsampling is not available in the FP16 form");
  if (U > 1 && !buf.xhat) return fail(FTK_EUNSUPPORTED, "ftk_align: rotation upsampling needs an Xhat buffer");
  struct NoTimer {
    StageTimer* t;
    hipEvent_t begin(hipStream_t st) { return t ? t->begin(st) : nullptr; }
    void end(hipEvent_t a, hipStream_t st, int stage) {
      if (t) t->end(a, st, stage);
    }
  } timer{tm};
  // short per-image lists fill one template tile per workgroup: the smaller
  // SVD block gives twice the workgroups for the same operand work
  const int zblk = (lists && K <= 16) ? 64 : step1_zblk(p);
  if (step1_v2_lds_bytes(p->M, zblk, prec) > kLdsLimit) return fail(FTK_EUNSUPPORTED, "ftk_align: step 1 tiles exceed LDS");
  unsigned long long* keys = buf.keys;
  hipError_t e;
  hipEvent_t ev = timer.begin(s);
  if ((e = launch_keys_init(keys, pairs, s)) != hipSuccess) return hip_fail(e, "ftk_align: keys init");
  timer.end(ev, s, 3);
  const float2* bco = static_cast<const float2*>(tmpl_coeffs);
  // fp16 forms: the per-call data scales, [max|a|, max|b|, 2^e/s_a, 2^e/s_b,
  // s_a s_b s_y 2^e_x, 2^e_z] (exponents 0 in the FP16 form, split_f16_exps
  // in the split-fp16 form)
  float* scales = (prec == 2 || prec == 3) ? buf.scales : nullptr;
  if (scales) {
    ev = timer.begin(s);
    const size_t per = static_cast<size_t>(2) * p->Qa * p->M;
    const SplitF16Exps x = prec == 3 ? split_f16_exps(p->M) : SplitF16Exps{0, 0, 0};
    if ((e = launch_fp16_scales(static_cast<const float*>(img_coeffs), per * nA, reinterpret_cast<const float*>(bco),
                                per * nB, p->y_scale, scales, x.data, x.x, x.z, s)) != hipSuccess)
      return hip_fail(e, "ftk_align: fp16 scales");
    timer.end(ev, s, 4);
  }
  if (!lists) {
    // template operand of Step 1: embedded (and split or scaled) once per call
    ev = timer.begin(s);
    if ((e = launch_tmpl_prep(bco, buf.tmpl, nB, p->M, p->Qa, prec, scales ? scales + 2 : nullptr, s)) !=
        hipSuccess)
      return hip_fail(e, "ftk_align: template operand");
    timer.end(ev, s, 4);
  }

  Step1Args a1{};
  a1.cz = p->cz.as<float>();
  a1.ell = p->ell.as<int>();
  a1.zs = buf.stage;
  a1.b = bco;
  a1.r32 = static_cast<float*>(buf.tmpl);
  a1.r16 = buf.tmpl;
  a1.dscale = scales ? scales + 2 : nullptr;
  a1.nB = nBe;
  a1.img_tiles = lists ? (K + 15) / 16 : 0;
  a1.tiles_per_q = (nBe + 15) / 16;
  a1.M = p->M;
  a1.Qa = p->Qa;
  a1.H_pad = p->H_pad;
  a1.L = p->t.L;
  a1.zblk = zblk;
  Step3Args a3{};
  a3.yt = p->yt.as<float>();
  a3.yt_hi = p->yt_hi.as<uint16_t>();
  a3.yt_lo = p->yt_lo.as<uint16_t>();
  a3.xscale = scales ? scales + 4 : nullptr;
  a3.tw_qa = p->tw_qa.as<float2>();
  a3.rot16 = prec == 2 ? p->rot16.ptr : nullptr;
  a3.Qa = p->Qa;
  a3.H_pad = p->H_pad;
  a3.N = p->N;
  a3.N_pad = p->N_pad;
  a3.nwaves = step3_waves(p);
  for (int A0 = 0; A0 < nA; A0 += chunkA) {
    const int na = std::min(chunkA, nA - A0);
    a1.a = static_cast<const float2*>(img_coeffs) + static_cast<size_t>(A0) * p->Qa * p->M;
    a1.nA = na;
    if (lists) {
      // this chunk's own template operand, gathered through the lists
      a1.tiles_per_q = na * a1.img_tiles;
      ev = timer.begin(s);
      if ((e = launch_tmpl_prep_lists(bco, buf.tmpl, nB, p->M, p->Qa, prec, scales ? scales + 2 : nullptr, lists,
                                      K, na, A0, s)) != hipSuccess)
        return hip_fail(e, "ftk_align_lists: template operand");
      timer.end(ev, s, 4);
    }
    {
      // split the template sweep until the grid holds about step1_wgs workgroups
      const int base = na * (QH - 1 + a1.zblk / 32) * (p->H_pad / a1.zblk);
      const int max_parts = std::max(1, ((nBe + 15) / 16 + 7) / 8);
      a1.tparts = std::min(max_parts, std::max(1, (p->tune.step1_wgs + base - 1) / base));
    }
    ev = timer.begin(s);
    e = launch_step1_v2(a1, prec, s);
    if (e != hipSuccess) return hip_fail(e, "ftk_align: step 1");
    timer.end(ev, s, 1);
    a3.zs = buf.stage;
    a3.pairs = na * nBe;
    a3.keys = keys + static_cast<size_t>(A0) * nBe;
    a3.X = X ? X + static_cast<size_t>(A0) * nBe * p->N * p->Qa * U : nullptr;
    a3.xhat = U > 1 ? buf.xhat : nullptr;
    ev = timer.begin(s);
    e = (prec == 1 || prec == 3) ? launch_step3_bf16(a3, prec == 3, s)
                                 : (prec == 2 ? launch_step3_fp16(a3, s) : launch_step3(a3, p->precision, s));
    if (e != hipSuccess) return hip_fail(e, "ftk_align: step 3");
    if (U > 1) {
      // the rotation sum on the U-fold grid, from the Xhat Step 3 stored
      Step3Args ar = a3;
      ar.zs = buf.xhat;
      ar.xhat = nullptr;
      ar.H_pad = p->N_pad;
      ar.nwaves = 4;
      ar.up = U;
      if ((e = launch_xhat_rotate(ar, s)) != hipSuccess) return hip_fail(e, "ftk_align: upsampled rotation");
    }
    timer.end(ev, s, 2);
  }
  if (best) {
    ev = timer.begin(s);
    if ((e = launch_keys_to_poses(keys, best, pairs, p->Qa * U, scales ? scales + 4 : nullptr, s)) != hipSuccess)
      return hip_fail(e, "ftk_align: poses");
    timer.end(ev, s, 3);
  }
  return FTK_OK;
}

}  // namespace ftkint

namespace {

int align_impl(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB, const int32_t* lists,
               int K, float* X, ftk_pose* best, void* stream) {
  const Needs nd = lists ? plan_needs_lists(p, nA, K) : plan_needs(p, nA, nB, false);
  Workspace& ws = *p->ws;
  if (ws.stage.ensure(nd.stage) != hipSuccess) return fail(FTK_ENOMEM, "ftk_align: staging buffer");
  if (ws.keys.ensure(nd.keys) != hipSuccess) return fail(FTK_ENOMEM, "ftk_align: key buffer");
  if (ws.tmpl.ensure(nd.tmpl) != hipSuccess) return fail(FTK_ENOMEM, "ftk_align: template operand buffer");
  if (ws.scales.ensure(nd.scales) != hipSuccess) return fail(FTK_ENOMEM, "ftk_align: scale buffer");
  if (ws.xhat.ensure(nd.xhat) != hipSuccess) return fail(FTK_ENOMEM, "ftk_align: Xhat buffer");
  const AlignBufs buf{ws.stage.ptr, ws.keys.as<unsigned long long>(), ws.tmpl.ptr, ws.scales.as<float>(),
                      nd.chunk_images, ws.xhat.as<float>()};
  return align_run(p, img_coeffs, nA, tmpl_coeffs, nB, lists, K, X, best, buf, &p->timer, stream);
}

}  // namespace

extern "C" {

int ftk_align_coeffs(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB, float* X,
                     ftk_pose* best, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_align_coeffs: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_align_coeffs: negative count");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_align_coeffs: call ftk_set_shifts first");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (!X && !best) return fail(FTK_EINVAL, "ftk_align_coeffs: X and best are both NULL");
  if (!img_coeffs || !tmpl_coeffs) return fail(FTK_EINVAL, "ftk_align_coeffs: NULL coefficients");
  return align_impl(p, img_coeffs, nA, tmpl_coeffs, nB, nullptr, 0, X, best, stream);
}

int ftk_align_lists(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB,
                    const int32_t* lists, int K, ftk_pose* best, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_align_lists: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_align_lists: negative count");
  if (K < 1 || K > 4096) return fail(FTK_EINVAL, "ftk_align_lists: K must be in [1, 4096]");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_align_lists: call ftk_set_shifts first");
  if (nA == 0) return FTK_OK;
  if (nB == 0) return fail(FTK_EINVAL, "ftk_align_lists: lists need templates (nB = 0)");
  if (!img_coeffs || !tmpl_coeffs || !lists || !best) return fail(FTK_EINVAL, "ftk_align_lists: NULL argument");
  return align_impl(p, img_coeffs, nA, tmpl_coeffs, nB, lists, K, nullptr, best, stream);
}

int ftk_align(ftk_plan* p, const float* images, int nA, const float* templates, int nB, float* X, ftk_pose* best,
              void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_align: NULL plan");
  if (nA < 0 || nB < 0) return fail(FTK_EINVAL, "ftk_align: negative count");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_align: call ftk_set_shifts first");
  if (nA == 0 || nB == 0) return FTK_OK;
  if (!X && !best) return fail(FTK_EINVAL, "ftk_align: X and best are both NULL");
  if (!images || !templates) return fail(FTK_EINVAL, "ftk_align: NULL images");
  const Needs nd = plan_needs(p, nA, nB, true);
  Workspace& ws = *p->ws;
  if (ws.coef_a.ensure(nd.coef_a) != hipSuccess || ws.coef_b.ensure(nd.coef_b) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_align: coefficients");
  int rc = ftk_transform(p, images, nA, ws.coef_a.ptr, stream);
  if (rc != FTK_OK) return rc;
  rc = ftk_transform(p, templates, nB, ws.coef_b.ptr, stream);
  if (rc != FTK_OK) return rc;
  return ftk_align_coeffs(p, ws.coef_a.ptr, nA, ws.coef_b.ptr, nB, X, best, stream);
}

int ftk_plan_set_tuning(ftk_plan* p, const ftk_tuning_t* t) {
  if (!p || !t) return fail(FTK_EINVAL, "ftk_plan_set_tuning: NULL argument");
  if (t->step3_waves < 0 || t->step3_waves > 16) return fail(FTK_EINVAL, "step3_waves must be in [0, 16]");
  if (t->step1_zblk != 0 && t->step1_zblk != 64 && t->step1_zblk != 128)
    return fail(FTK_EINVAL, "step1_zblk must be 0, 64 or 128");
  if (t->step1_wgs != 0 && (t->step1_wgs < 64 || t->step1_wgs > 65536))
    return fail(FTK_EINVAL, "step1_wgs must be 0 or in [64, 65536]");
  if (t->stage_mib != 0 && (t->stage_mib < 16 || t->stage_mib > 65536))
    return fail(FTK_EINVAL, "stage_mib must be 0 or in [16, 65536]");
  const ftk_tuning_t d = default_tuning(p->precision);
  p->tune.step3_waves = t->step3_waves ? t->step3_waves : d.step3_waves;
  p->tune.step1_zblk = t->step1_zblk ? t->step1_zblk : d.step1_zblk;
  p->tune.step1_wgs = t->step1_wgs ? t->step1_wgs : d.step1_wgs;
  p->tune.stage_mib = t->stage_mib ? t->stage_mib : d.stage_mib;
  return FTK_OK;
}

int ftk_plan_get_tuning(const ftk_plan* p, ftk_tuning_t* out) {
  if (!p || !out) return fail(FTK_EINVAL, "ftk_plan_get_tuning: NULL argument");
  *out = p->tune;
  return FTK_OK;
}

int ftk_plan_profile(ftk_plan* p, int enable) {
  if (!p) return fail(FTK_EINVAL, "ftk_plan_profile: NULL plan");
  p->timer.clear();
  p->timer.on = enable != 0;
  return FTK_OK;
}

int ftk_plan_stage_times(ftk_plan* p, double* ms, int64_t* launches, int nstages) {
  if (!p || nstages < 0) return fail(FTK_EINVAL, "ftk_plan_stage_times: invalid argument");
  for (int i = 0; i < nstages; ++i) {
    if (ms) ms[i] = 0.0;
    if (launches) launches[i] = 0;
  }
  int rc = FTK_OK;
  for (const auto& r : p->timer.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) {
      rc = hip_fail(e, "ftk_plan_stage_times");
      break;
    }
    if (r.stage < nstages) {
      if (ms) ms[r.stage] += t;
      if (launches) launches[r.stage] += 1;
    }
  }
  p->timer.clear();
  return rc;
}

}  // extern "C"
