// Internal definition of the FTK plan object, shared by the C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "ftk.h"
#include "kernels.h"
#include "planner.h"

namespace ftkint {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kNufftWidth = 8;
constexpr size_t kLdsLimit = 160 * 1024;

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* where);
size_t env_mib(const char* name, size_t dflt_mib);
inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// A device allocation that only grows.  ensure() never allocates when the
// buffer is already large enough, so work issued during graph capture does
// not allocate once the buffers are sized.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  void release();
  hipError_t ensure(size_t want);
  template <class T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// Events around kernel launches, per stage (see ftk_plan_profile).
struct StageTimer {
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    int stage;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  hipEvent_t begin(hipStream_t s);
  void end(hipEvent_t a, hipStream_t s, int stage);
  void clear();
  void destroy();
};

// Per-mode factor tables, FP64 (Section 4.5 of the paper).
struct HostTables {
  int H = 0, L = 0;
  double sigma_next = 0;
  std::vector<int> ell, eta;
  std::vector<double> sigma;
  std::vector<double> k, w;  // radial rule
  std::vector<double> G;     // [H][M] Sigma v(k_m / kmax), sign (-1)^l for l < 0
  ftkplan::Truncation tr;
};

// Scratch of the transform and the alignment.  A plan owns one; a batch
// lends a shared one to each of its plans while it runs them.
struct Workspace {
  DevBuf tr_h, tr_g, coef_a, coef_b, stage, keys, tmpl, scales;
  DevBuf refine;     // lists and poses of the two-pass alignment
  DevBuf polar, ta;  // brute-force translations: ring samples, translated coefficients
  DevBuf xhat;       // rotation upsampling: Xhat of a chunk of pairs
  DevBuf bfr_a, bfr_b, bfr_tab;  // brute-force rotations: Cartesian spectra of images, of templates, tables
  size_t bytes() const {
    return tr_h.bytes + tr_g.bytes + coef_a.bytes + coef_b.bytes + stage.bytes + keys.bytes + tmpl.bytes +
           scales.bytes + refine.bytes + polar.bytes + ta.bytes + xhat.bytes + bfr_a.bytes + bfr_b.bytes +
           bfr_tab.bytes;
  }
  void release() {
    for (DevBuf* b : {&tr_h, &tr_g, &coef_a, &coef_b, &stage, &keys, &tmpl, &scales, &refine, &polar, &ta, &xhat,
                      &bfr_a, &bfr_b, &bfr_tab})
      b->release();
  }
};

// Workspace sizes a call needs (the same formulas size and use the buffers).
struct Needs {
  size_t tr_h = 0, tr_g = 0, coef_a = 0, coef_b = 0, stage = 0, keys = 0, tmpl = 0;
  size_t scales = 0;        // FP16 form: the per-call data scales
  size_t xhat = 0;          // rotation upsampling: Xhat of a chunk
  int chunk_images = 0;     // images per Step 1 / Step 3 chunk
  int transform_chunk = 0;  // images per transform launch
};

// Shift-side device panels of one pose list (see ftk_set_shifts): Y
// embedded for Step 3, the brute-force table, the counts and the FP16
// panel scale.
struct ShiftPanels {
  DevBuf yt, yt_hi, yt_lo, kd;
  int N = 0, N_pad = 0;
  float y_scale = 1.f;
  void release() {
    for (DevBuf* b : {&yt, &yt_hi, &yt_lo, &kd}) b->release();
  }
  size_t bytes() const { return yt.bytes + yt_hi.bytes + yt_lo.bytes + kd.bytes; }
};

// A shift window (ftk_plan_set_shift_windows): the shifts of the plan whose
// radius lies within half_width of the window's centre, their panels, and
// the map from window index to plan index (host and device int32).
struct ShiftWindow {
  ShiftPanels pan;
  std::vector<int32_t> idx;
  DevBuf didx;
  void release() {
    pan.release();
    didx.release();
  }
};

}  // namespace ftkint

struct ftk_plan {
  ftkint::StageTimer timer;
  int n = 0, M = 0, Qa = 0, precision = 0;
  int up = 1;  // rotation upsampling: U Qa rotations (remark after eq. 1dfft)
  bool weighted = false;  // operator SVD with a k-side weight (Section 4.5 remark)
  bool has_ctf = false;   // joint translation-CTF factorisation (Section 7.1); poses carry a defocus
  double W = 0, eps = 0, kmax = 0;
  ftkint::HostTables t;
  int H_pad = 0, N = 0, N_pad = 0;
  // FP16 form: per-zeta powers of two sg_zeta dividing the 2 pi w G table and
  // multiplying the shift panel, and the power of two s_y of that panel
  std::vector<float> zeta_scale;
  float y_scale = 1.f;
  ftkplan::SpreadKernel sk;
  ftk_tuning_t tune{};
  // plan-owned device tables
  ftkint::DevBuf cz, ell, yt, yt_hi, yt_lo, tw_nf, tw_qa, deapod, ptbase, ptker;
  ftkint::DevBuf rot16;  // FP16 form, Qa <= 256: rotation transform tables
  // brute-force translations: [M] 2 pi w_m, and [N][M] (k_m dx, k_m dy) of
  // each shift in image units
  ftkint::DevBuf bft_cz, bft_kd;
  ftkint::Workspace own_ws;
  ftkint::Workspace* ws = &own_ws;
  std::vector<double> shifts;  // the current shift list (px), [N][2]
  std::vector<ftkint::ShiftWindow> windows;
  ~ftk_plan() {
    for (auto& w : windows) w.release();
  }
  size_t device_bytes() const {
    return cz.bytes + ell.bytes + yt.bytes + yt_hi.bytes + yt_lo.bytes + tw_nf.bytes + tw_qa.bytes +
           deapod.bytes + ptbase.bytes + ptker.bytes + rot16.bytes + bft_cz.bytes + bft_kd.bytes + own_ws.bytes() +
           windows_bytes();
  }
  size_t windows_bytes() const {
    size_t s = 0;
    for (const auto& w : windows) s += w.pan.bytes() + w.didx.bytes;
    return s;
  }
  void release_all() {
    for (ftkint::DevBuf* b :
         {&cz, &ell, &yt, &yt_hi, &yt_lo, &tw_nf, &tw_qa, &deapod, &ptbase, &ptker, &rot16, &bft_cz, &bft_kd})
      b->release();
    own_ws.release();
    for (auto& w : windows) w.release();
    windows.clear();
  }
};

namespace ftkint {
// Built-in launch shapes (environment overrides applied).
ftk_tuning_t default_tuning(int precision);
Needs plan_needs(const ftk_plan* p, int nA, int nB, bool from_pixels);
// alignment of nA images against K listed templates each
Needs plan_needs_lists(const ftk_plan* p, int nA, int K);
// kernel precision code of a plan: 0 FP32, 1 split-bf16, 2 FP16, 3 split-fp16
inline int prec_code(const ftk_plan* p) {
  switch (p->precision) {
    case FTK_BF16X3: return 1;
    case FTK_FP16: return 2;
    case FTK_FP16X3: return 3;
    default: return 0;
  }
}
// Buffers of one alignment call: Zhat staging for chunk_images images, the
// pose keys of every pair, the Step 1 template operand and the data scales
// of the fp16 forms.
struct AlignBufs {
  void* stage;
  unsigned long long* keys;
  void* tmpl;
  float* scales;
  int chunk_images;
  float* xhat;  // rotation upsampling (plan up > 1): Xhat of chunk_images images
};
// Steps 1-3 and the argmax on caller-provided buffers (ftk_api.hip); tm may
// be null (no stage timing).
int align_run(ftk_plan* p, const void* img_coeffs, int nA, const void* tmpl_coeffs, int nB, const int32_t* lists,
              int K, float* X, ftk_pose* best, const AlignBufs& buf, StageTimer* tm, void* stream);
// Zhat staging bytes of one image-template pair: Qa/2 rows of 2 H_pad values,
// 2 bytes each in the FP16 form, 4 otherwise (FP32, or hi + lo).
inline size_t stage_bytes_per_pair(const ftk_plan* p) {
  return static_cast<size_t>(p->Qa / 2) * 2 * p->H_pad * (prec_code(p) == 2 ? 2 : 4);
}
// Xhat bytes of one pair when the plan upsamples the rotations (else 0):
// Qa/2 rows of 2 N_pad floats.
inline size_t xhat_bytes_per_pair(const ftk_plan* p) {
  return p->up > 1 ? static_cast<size_t>(p->Qa / 2) * 2 * p->N_pad * sizeof(float) : 0;
}
// Power-of-two exponents of the split-fp16 form.  Its lo parts lose
// precision where they fall below the smallest normal fp16 (2^-14), so every
// operand is lifted to the top of the fp16 range: a / s_a, b / s_b and the
// scaled shift panel (all at most 1) are multiplied by 2^data; Step 1's FP32
// result, at most 4M 2^(2 data) in magnitude (K = 4M terms in the Nyquist
// fold), is multiplied by 2^z = 2^-(data + ceil(log2 4M)) before it is split,
// which leaves it at most 2^data; X is multiplied back by s_a s_b s_y 2^x
// with x = ceil(log2 4M) - 2 data.
struct SplitF16Exps {
  int data, x, z;
};
inline SplitF16Exps split_f16_exps(int M) {
  constexpr int kData = 15;  // fp16 holds values up to 65504 < 2^16
  int c = 0;
  while ((1 << c) < 4 * M) ++c;
  return SplitF16Exps{kData, c - 2 * kData, -(kData + c)};
}
int build_panels(const ftk_plan* p, const double* shifts_px, const double* defocus, int N, ShiftPanels& out);
void swap_panels(ftk_plan* p, ShiftPanels& w);
// ftk_transform's body; polar (optional) receives the ring samples
// [cnt][M][Qa] that the ring DFT transforms (TransformArgs::polar).
int transform_run(ftk_plan* p, const float* imgs, int cnt, float2* coeffs, float2* polar, void* stream);
// Step 3 waves per workgroup and Step 1 zeta block actually used by a plan.
int step3_waves(const ftk_plan* p);
int step1_zblk(const ftk_plan* p);
}  // namespace ftkint
