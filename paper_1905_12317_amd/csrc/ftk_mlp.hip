// C-ABI of the learned template proposal: the network object (parameters,
// AdamW state, activations for max_batch rows), features, training steps,
// proposals, and the proposal search with its full-FTK fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "ftk_mlp.h"
#include "mlp_kernels.h"
#include "plan_internal.h"

using namespace ftkint;

struct ftk_mlp {
  int L = 0;
  int dims[FTK_MLP_MAX_LAYERS + 1] = {};
  int n_t = 0, n_s = 0, prec = 0, maxB = 0;
  int64_t step = 0;
  std::vector<DevBuf> W, b, Wc, mW, vW, mb, vb, dW, db;
  DevBuf mu, is;
  DevBuf X0;                 // standardised input, operand type [maxB][d0]
  std::vector<DevBuf> Z;     // pre-activations / logits, FP32 [maxB][d_{l+1}]
  std::vector<DevBuf> H;     // H[l] = input of layer l (l >= 1), operand type
  DevBuf dZf[2], dZb[2];     // gradients w.r.t. pre-activations, ping-pong
  DevBuf row_loss;
  DevBuf part;               // K-split partial sums of the bf16 GEMMs (kGemmPartFloats)
  // proposal search workspace (grown on demand)
  DevBuf feat, top, mass, sbin, pair_poses, flist, fcount, fcoef, fposes, fbt, fbp, coef;
  DevBuf wlist, wcoef, wtop, wposes;  // shift-window search
  size_t esize() const { return prec == FTK_MLP_BF16 ? 2 : 4; }
  size_t device_bytes() const {
    size_t s = mu.bytes + is.bytes + X0.bytes + row_loss.bytes + part.bytes;
    for (const auto* v : {&W, &b, &Wc, &mW, &vW, &mb, &vb, &dW, &db, &Z, &H})
      for (const auto& x : *v) s += x.bytes;
    for (int i = 0; i < 2; ++i) s += dZf[i].bytes + dZb[i].bytes;
    for (const DevBuf* x : {&feat, &top, &mass, &sbin, &pair_poses, &flist, &fcount, &fcoef, &fposes, &fbt, &fbp, &coef,
                            &wlist, &wcoef, &wtop, &wposes})
      s += x->bytes;
    return s;
  }
  void release() {
    for (auto* v : {&W, &b, &Wc, &mW, &vW, &mb, &vb, &dW, &db, &Z, &H})
      for (auto& x : *v) x.release();
    for (DevBuf* x : {&mu, &is, &X0, &row_loss, &part, &dZf[0], &dZf[1], &dZb[0], &dZb[1], &feat, &top, &mass, &sbin,
                      &pair_poses, &flist, &fcount, &fcoef, &fposes, &fbt, &fbp, &coef, &wlist, &wcoef, &wtop, &wposes})
      x->release();
  }
};

namespace {

// Bound of the K-split workspace: a bf16 GEMM splits only while its tiles
// times parts stay within 512, so kparts M N <= 512 x 128 x 128 floats.
constexpr size_t kGemmPartFloats = static_cast<size_t>(512) * 128 * 128;

hipError_t zero_fill(DevBuf& d) { return hipMemset(d.ptr, 0, d.bytes); }

template <class T>
hipError_t upload_vec(DevBuf& d, const T* h, size_t n) {
  return hipMemcpy(d.ptr, h, n * sizeof(T), hipMemcpyHostToDevice);
}

// Forward over rows already standardised in X0; FP32 pre-activations into
// Z[l] (the last one: logits, or `logits` when given).
int forward_rows(ftk_mlp* m, int B, float* logits, hipStream_t s) {
  for (int l = 0; l < m->L; ++l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    GemmArgs g{};
    g.A = l == 0 ? m->X0.ptr : m->H[l].ptr;
    g.sai = din;
    g.sak = 1;
    g.B = m->Wc[l].ptr;
    g.sbk = 1;
    g.sbj = din;
    g.M = B;
    g.N = dout;
    g.K = din;
    const bool last = l == m->L - 1;
    g.C = (last && logits) ? logits : m->Z[l].as<float>();
    g.ldc = dout;
    g.Cb = last ? nullptr : m->H[l + 1].ptr;
    g.ldcb = dout;
    g.bias = m->b[l].as<float>();
    g.part = m->part.as<float>();
    g.part_floats = m->part.bytes / sizeof(float);
    g.relu = last ? 0 : 1;
    hipError_t e = launch_gemm(g, m->prec, s);
    if (e != hipSuccess) return hip_fail(e, "ftk_mlp: forward GEMM");
  }
  return FTK_OK;
}

int check_rows(const ftk_mlp* m, int B, const char* who) {
  if (B < 1 || B > m->maxB) return fail(FTK_EINVAL, std::string(who) + ": B must be in [1, max_batch]");
  return FTK_OK;
}

// The proposed images grouped by the window of their predicted shift bin:
// per window, the images' coefficients and template lists gathered, the
// list alignment run with the window's shift panels in place of the plan's,
// and the poses (window shift index mapped to the plan's) scattered back.
// Images below tau are left to the full search.  One host sync (the
// proposal's mass and bins).
int align_windows(ftk_plan* p, ftk_mlp* m, int nA, const void* tmpl_coeffs, int nB, int topk, float tau,
                  hipStream_t s) {
  std::vector<float> mass(nA);
  std::vector<int32_t> bin(nA);
  hipError_t e;
  if ((e = hipMemcpyAsync(mass.data(), m->mass.ptr, 4ull * nA, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(bin.data(), m->sbin.ptr, 4ull * nA, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "ftk_align_proposed: proposal to host");
  const int nw = static_cast<int>(p->windows.size());
  std::vector<std::vector<int32_t>> groups(nw);
  for (int i = 0; i < nA; ++i)
    if (!(mass[i] < tau)) groups[std::min(std::max(bin[i], 0), nw - 1)].push_back(i);
  size_t most = 0;
  for (const auto& g : groups) most = std::max(most, g.size());
  if (most == 0) return FTK_OK;
  const size_t cb = static_cast<size_t>(8) * p->M * p->Qa;
  if (m->wlist.ensure(4 * most) != hipSuccess || m->wcoef.ensure(cb * most) != hipSuccess ||
      m->wtop.ensure(4 * most * topk) != hipSuccess || m->wposes.ensure(12 * most * topk) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_align_proposed: window workspace");
  for (int b = 0; b < nw; ++b) {
    const int cnt = static_cast<int>(groups[b].size());
    if (cnt == 0) continue;
    // the list stays alive until the stream has used it (synchronous copy)
    if ((e = hipMemcpy(m->wlist.ptr, groups[b].data(), 4ull * cnt, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "ftk_align_proposed: window list");
    if ((e = launch_gather_words(m->coef.ptr, m->wlist.as<int32_t>(), cnt, cb / 4, m->wcoef.ptr, s)) != hipSuccess ||
        (e = launch_gather_words(m->top.ptr, m->wlist.as<int32_t>(), cnt, topk, m->wtop.ptr, s)) != hipSuccess)
      return hip_fail(e, "ftk_align_proposed: window gather");
    ShiftWindow& w = p->windows[b];
    swap_panels(p, w.pan);
    int rc = ftk_align_lists(p, m->wcoef.ptr, cnt, tmpl_coeffs, nB, m->wtop.as<int32_t>(), topk,
                             m->wposes.as<ftk_pose>(), s);
    swap_panels(p, w.pan);
    if (rc != FTK_OK) return rc;
    if ((e = launch_scatter_poses(m->wposes.ptr, m->wlist.as<int32_t>(), cnt, topk, w.didx.as<int32_t>(),
                                  m->pair_poses.ptr, s)) != hipSuccess)
      return hip_fail(e, "ftk_align_proposed: window scatter");
    // the next window's list overwrites wlist: wait for this one's kernels
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "ftk_align_proposed: window sync");
  }
  return FTK_OK;
}

}  // namespace

extern "C" {

int ftk_mlp_create(ftk_mlp** out, const int* dims, int nlayers, int n_template, int n_shift, int precision,
                   int max_batch) {
  if (!out || !dims) return fail(FTK_EINVAL, "ftk_mlp_create: NULL argument");
  *out = nullptr;
  if (nlayers < 1 || nlayers > FTK_MLP_MAX_LAYERS) return fail(FTK_EINVAL, "ftk_mlp_create: nlayers out of range");
  for (int l = 0; l <= nlayers; ++l)
    if (dims[l] < 1 || dims[l] > 65536) return fail(FTK_EINVAL, "ftk_mlp_create: width out of range");
  if (n_template < 1 || n_shift < 0 || dims[nlayers] != n_template + n_shift)
    return fail(FTK_EINVAL, "ftk_mlp_create: dims[nlayers] must equal n_template + n_shift");
  if (precision != FTK_MLP_FP32 && precision != FTK_MLP_BF16) return fail(FTK_EINVAL, "ftk_mlp_create: precision");
  if (max_batch < 1 || max_batch > 65536) return fail(FTK_EINVAL, "ftk_mlp_create: max_batch out of range");
  ftk_mlp* m = nullptr;
  try {
    m = new ftk_mlp();
    m->L = nlayers;
    for (int l = 0; l <= nlayers; ++l) m->dims[l] = dims[l];
    m->n_t = n_template;
    m->n_s = n_shift;
    m->prec = precision;
    m->maxB = max_batch;
    for (auto* v : {&m->W, &m->b, &m->Wc, &m->mW, &m->vW, &m->mb, &m->vb, &m->dW, &m->db, &m->Z, &m->H})
      v->resize(nlayers);
  } catch (const std::bad_alloc&) {
    delete m;
    return fail(FTK_ENOMEM, "ftk_mlp_create: host allocation failed");
  }
  const size_t es = m->esize();
  int maxd = 0;
  for (int l = 0; l <= nlayers; ++l) maxd = std::max(maxd, dims[l]);
  hipError_t e = hipSuccess;
  auto grab = [&](DevBuf& d, size_t bytes) {
    if (e == hipSuccess) e = d.ensure(std::max<size_t>(bytes, 16));
    if (e == hipSuccess) e = zero_fill(d);
  };
  for (int l = 0; l < nlayers; ++l) {
    const size_t nw = static_cast<size_t>(dims[l + 1]) * dims[l], nb = dims[l + 1];
    grab(m->W[l], nw * 4);
    grab(m->Wc[l], nw * es);
    grab(m->mW[l], nw * 4);
    grab(m->vW[l], nw * 4);
    grab(m->dW[l], nw * 4);
    grab(m->b[l], nb * 4);
    grab(m->mb[l], nb * 4);
    grab(m->vb[l], nb * 4);
    grab(m->db[l], nb * 4);
    grab(m->Z[l], static_cast<size_t>(max_batch) * dims[l + 1] * 4);
    if (l >= 1) grab(m->H[l], static_cast<size_t>(max_batch) * dims[l] * es);
  }
  grab(m->X0, static_cast<size_t>(max_batch) * dims[0] * es);
  for (int i = 0; i < 2; ++i) {  // rows of up to maxd columns, padded to 8
    grab(m->dZf[i], static_cast<size_t>(max_batch) * ((maxd + 7) / 8 * 8) * 4);
    grab(m->dZb[i], static_cast<size_t>(max_batch) * ((maxd + 7) / 8 * 8) * es);
  }
  grab(m->row_loss, static_cast<size_t>(max_batch) * 4);
  if (m->prec == FTK_MLP_BF16) grab(m->part, kGemmPartFloats * 4);
  grab(m->mu, static_cast<size_t>(dims[0]) * 4);
  grab(m->is, static_cast<size_t>(dims[0]) * 4);
  if (e == hipSuccess) {
    std::vector<float> ones(dims[0], 1.f);
    e = upload_vec(m->is, ones.data(), ones.size());
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    m->release();
    delete m;
    return fail(FTK_ENOMEM, std::string("ftk_mlp_create: ") + hipGetErrorString(e));
  }
  *out = m;
  return FTK_OK;
}

void ftk_mlp_destroy(ftk_mlp* m) {
  if (!m) return;
  m->release();
  delete m;
}

int ftk_mlp_info(const ftk_mlp* m, ftk_mlp_info_t* o) {
  if (!m || !o) return fail(FTK_EINVAL, "ftk_mlp_info: NULL argument");
  *o = ftk_mlp_info_t{};
  o->nlayers = m->L;
  for (int l = 0; l <= m->L; ++l) o->dims[l] = m->dims[l];
  o->n_template = m->n_t;
  o->n_shift = m->n_s;
  o->precision = m->prec;
  o->max_batch = m->maxB;
  o->step = m->step;
  size_t pc = 0;
  for (int l = 0; l < m->L; ++l) pc += static_cast<size_t>(m->dims[l + 1]) * (m->dims[l] + 1);
  o->param_count = pc;
  o->device_bytes = m->device_bytes();
  return FTK_OK;
}

int ftk_mlp_set_layer(ftk_mlp* m, int layer, const float* W, const float* b) {
  if (!m || !W || !b) return fail(FTK_EINVAL, "ftk_mlp_set_layer: NULL argument");
  if (layer < 0 || layer >= m->L) return fail(FTK_EINVAL, "ftk_mlp_set_layer: layer out of range");
  const size_t nw = static_cast<size_t>(m->dims[layer + 1]) * m->dims[layer], nb = m->dims[layer + 1];
  hipError_t e;
  if ((e = upload_vec(m->W[layer], W, nw)) != hipSuccess || (e = upload_vec(m->b[layer], b, nb)) != hipSuccess ||
      (e = launch_convert(m->W[layer].as<float>(), nw, m->Wc[layer].ptr, m->prec, nullptr)) != hipSuccess ||
      (e = zero_fill(m->mW[layer])) != hipSuccess || (e = zero_fill(m->vW[layer])) != hipSuccess ||
      (e = zero_fill(m->mb[layer])) != hipSuccess || (e = zero_fill(m->vb[layer])) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return hip_fail(e, "ftk_mlp_set_layer");
  return FTK_OK;
}

int ftk_mlp_get_layer(const ftk_mlp* m, int layer, float* W, float* b) {
  if (!m) return fail(FTK_EINVAL, "ftk_mlp_get_layer: NULL network");
  if (layer < 0 || layer >= m->L) return fail(FTK_EINVAL, "ftk_mlp_get_layer: layer out of range");
  const size_t nw = static_cast<size_t>(m->dims[layer + 1]) * m->dims[layer], nb = m->dims[layer + 1];
  hipError_t e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "ftk_mlp_get_layer");
  if (W && (e = hipMemcpy(W, m->W[layer].ptr, nw * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "ftk_mlp_get_layer");
  if (b && (e = hipMemcpy(b, m->b[layer].ptr, nb * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "ftk_mlp_get_layer");
  return FTK_OK;
}

int ftk_mlp_get_grad(const ftk_mlp* m, int layer, float* dW, float* db) {
  if (!m) return fail(FTK_EINVAL, "ftk_mlp_get_grad: NULL network");
  if (layer < 0 || layer >= m->L) return fail(FTK_EINVAL, "ftk_mlp_get_grad: layer out of range");
  const size_t nw = static_cast<size_t>(m->dims[layer + 1]) * m->dims[layer], nb = m->dims[layer + 1];
  hipError_t e;
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "ftk_mlp_get_grad");
  if (dW && (e = hipMemcpy(dW, m->dW[layer].ptr, nw * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "ftk_mlp_get_grad");
  if (db && (e = hipMemcpy(db, m->db[layer].ptr, nb * 4, hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "ftk_mlp_get_grad");
  return FTK_OK;
}

int ftk_mlp_set_input_norm(ftk_mlp* m, const float* mu, const float* inv_sigma) {
  if (!m || !mu || !inv_sigma) return fail(FTK_EINVAL, "ftk_mlp_set_input_norm: NULL argument");
  hipError_t e;
  if ((e = upload_vec(m->mu, mu, m->dims[0])) != hipSuccess || (e = upload_vec(m->is, inv_sigma, m->dims[0])) != hipSuccess)
    return hip_fail(e, "ftk_mlp_set_input_norm");
  return FTK_OK;
}

int ftk_features(const ftk_plan* p, const void* coeffs, int nA, int kind, int n_r, int n_q, float* F, void* stream) {
  if (!p) return fail(FTK_EINVAL, "ftk_features: NULL plan");
  if (kind != FTK_FEATURES_POWER && kind != FTK_FEATURES_CROSS && kind != FTK_FEATURES_INVARIANT)
    return fail(FTK_EINVAL, "ftk_features: unknown kind");
  if (nA < 0 || n_r < 1 || n_r > p->M || n_q < 1 || n_q > p->Qa / 2)
    return fail(FTK_EINVAL, "ftk_features: sizes out of range");
  if (nA == 0) return FTK_OK;
  if (!coeffs || !F) return fail(FTK_EINVAL, "ftk_features: NULL buffer");
  hipError_t e = launch_features(static_cast<const float2*>(coeffs), nA, p->Qa, p->M, kind, n_r, n_q, F,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "ftk_features");
  return FTK_OK;
}

int ftk_mlp_forward(ftk_mlp* m, const float* x, int B, float* logits, void* stream) {
  if (!m || !x || !logits) return fail(FTK_EINVAL, "ftk_mlp_forward: NULL argument");
  int rc = check_rows(m, B, "ftk_mlp_forward");
  if (rc != FTK_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_standardise(x, nullptr, B, m->dims[0], m->mu.as<float>(), m->is.as<float>(), m->X0.ptr,
                                    m->prec, s);
  if (e != hipSuccess) return hip_fail(e, "ftk_mlp_forward: input");
  return forward_rows(m, B, logits, s);
}

int ftk_mlp_gradients(ftk_mlp* m, const float* x_all, const int32_t* lab_t, const int32_t* lab_s,
                      const int32_t* idx, int B, float* loss, void* stream) {
  if (!m || !x_all || !lab_t || !idx || !loss || (m->n_s > 0 && !lab_s))
    return fail(FTK_EINVAL, "ftk_mlp_gradients: NULL argument");
  int rc = check_rows(m, B, "ftk_mlp_gradients");
  if (rc != FTK_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_standardise(x_all, idx, B, m->dims[0], m->mu.as<float>(), m->is.as<float>(), m->X0.ptr,
                                    m->prec, s);
  if (e != hipSuccess) return hip_fail(e, "ftk_mlp_gradients: input");
  if ((rc = forward_rows(m, B, nullptr, s)) != FTK_OK) return rc;
  const int L = m->L, D = m->dims[L];
  // the output gradient rows are padded to a multiple of 8 columns, so the
  // GEMMs that read them as bf16 get 16-byte aligned rows
  const int ldz = (D + 7) / 8 * 8;
  int cur = 0;
  if ((e = launch_softmax_ce(m->Z[L - 1].as<float>(), B, D, ldz, m->n_t, m->n_s, lab_t, lab_s, idx, m->dZf[cur].as<float>(),
                             m->dZb[cur].ptr, m->prec, m->row_loss.as<float>(), s)) != hipSuccess)
    return hip_fail(e, "ftk_mlp_gradients: loss");
  if ((e = launch_mean(m->row_loss.as<float>(), B, loss, s)) != hipSuccess) return hip_fail(e, "ftk_mlp_gradients");
  for (int l = L - 1; l >= 0; --l) {
    const int din = m->dims[l], dout = m->dims[l + 1];
    const int ld = l == L - 1 ? ldz : dout;  // row stride of this layer's dZ
    // dW[o][j] = sum_b dZ[b][o] H_l[b][j]
    GemmArgs g{};
    g.A = m->dZb[cur].ptr;
    g.sai = 1;
    g.sak = ld;
    g.B = l == 0 ? m->X0.ptr : m->H[l].ptr;
    g.sbk = din;
    g.sbj = 1;
    g.M = dout;
    g.N = din;
    g.K = B;
    g.C = m->dW[l].as<float>();
    g.ldc = din;
    g.part = m->part.as<float>();
    g.part_floats = m->part.bytes / sizeof(float);
    if ((e = launch_gemm(g, m->prec, s)) != hipSuccess) return hip_fail(e, "ftk_mlp_gradients: dW");
    if ((e = launch_colsum(m->dZf[cur].as<float>(), B, dout, ld, m->db[l].as<float>(), s)) != hipSuccess)
      return hip_fail(e, "ftk_mlp_gradients: db");
    if (l == 0) break;
    // dZ_{l-1}[b][j] = (sum_o dZ[b][o] W[o][j]) (Z_{l-1}[b][j] > 0)
    GemmArgs h{};
    h.A = m->dZb[cur].ptr;
    h.sai = ld;
    h.sak = 1;
    h.B = m->Wc[l].ptr;
    h.sbk = din;
    h.sbj = 1;
    h.M = B;
    h.N = din;
    h.K = dout;
    h.mask = m->Z[l - 1].as<float>();
    h.ldm = din;
    h.C = m->dZf[cur ^ 1].as<float>();
    h.ldc = din;
    h.Cb = m->dZb[cur ^ 1].ptr;
    h.ldcb = din;
    h.part = m->part.as<float>();
    h.part_floats = m->part.bytes / sizeof(float);
    if ((e = launch_gemm(h, m->prec, s)) != hipSuccess) return hip_fail(e, "ftk_mlp_gradients: dX");
    cur ^= 1;
  }
  return FTK_OK;
}

int ftk_mlp_train_step(ftk_mlp* m, const float* x_all, const int32_t* lab_t, const int32_t* lab_s,
                       const int32_t* idx, int B, float lr, float beta1, float beta2, float eps, float wd,
                       float* loss, void* stream) {
  if (!m) return fail(FTK_EINVAL, "ftk_mlp_train_step: NULL network");
  if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f) ||
      !(wd >= 0.f))
    return fail(FTK_EINVAL, "ftk_mlp_train_step: hyper-parameter out of range");
  int rc = ftk_mlp_gradients(m, x_all, lab_t, lab_s, idx, B, loss, stream);
  if (rc != FTK_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  m->step += 1;
  const float bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta1), static_cast<double>(m->step)));
  const float bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(beta2), static_cast<double>(m->step)));
  for (int l = 0; l < m->L; ++l) {
    const size_t nw = static_cast<size_t>(m->dims[l + 1]) * m->dims[l], nb = m->dims[l + 1];
    hipError_t e = launch_adamw(m->W[l].as<float>(), m->dW[l].as<float>(), m->mW[l].as<float>(), m->vW[l].as<float>(),
                                nw, lr, beta1, beta2, eps, wd, bc1, bc2, m->Wc[l].ptr, m->prec, s);
    if (e == hipSuccess)
      e = launch_adamw(m->b[l].as<float>(), m->db[l].as<float>(), m->mb[l].as<float>(), m->vb[l].as<float>(), nb, lr,
                       beta1, beta2, eps, 0.f, bc1, bc2, nullptr, m->prec, s);
    if (e != hipSuccess) return hip_fail(e, "ftk_mlp_train_step: AdamW");
  }
  return FTK_OK;
}

int ftk_propose(ftk_mlp* m, const float* x, int nA, int topk, int32_t* top, float* mass, int32_t* shift_bin,
                void* stream) {
  if (!m) return fail(FTK_EINVAL, "ftk_propose: NULL network");
  if (nA < 0) return fail(FTK_EINVAL, "ftk_propose: nA < 0");
  if (topk < 1 || topk > 64 || topk > m->n_t) return fail(FTK_EINVAL, "ftk_propose: topk out of range");
  if (nA == 0) return FTK_OK;
  if (!x || !top || !mass || !shift_bin) return fail(FTK_EINVAL, "ftk_propose: NULL buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int D0 = m->dims[0], D = m->dims[m->L];
  for (int r0 = 0; r0 < nA; r0 += m->maxB) {
    const int nb = std::min(m->maxB, nA - r0);
    hipError_t e = launch_standardise(x + static_cast<size_t>(r0) * D0, nullptr, nb, D0, m->mu.as<float>(),
                                      m->is.as<float>(), m->X0.ptr, m->prec, s);
    if (e != hipSuccess) return hip_fail(e, "ftk_propose: input");
    int rc = forward_rows(m, nb, nullptr, s);
    if (rc != FTK_OK) return rc;
    e = launch_topk(m->Z[m->L - 1].as<float>(), nb, D, m->n_t, m->n_s, topk, top + static_cast<size_t>(r0) * topk,
                    mass + r0, shift_bin + r0, s);
    if (e != hipSuccess) return hip_fail(e, "ftk_propose: top-k");
  }
  return FTK_OK;
}

int ftk_best_template(const ftk_pose* poses, const int32_t* lists, int nA, int K, int32_t* best_t,
                      ftk_pose* best_pose, void* stream) {
  if (nA < 0 || K < 1) return fail(FTK_EINVAL, "ftk_best_template: sizes out of range");
  if (nA == 0) return FTK_OK;
  if (!poses || !best_t || !best_pose) return fail(FTK_EINVAL, "ftk_best_template: NULL buffer");
  hipError_t e = launch_best_template(poses, lists, nA, K, best_t, best_pose, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "ftk_best_template");
  return FTK_OK;
}

int ftk_align_proposed(ftk_plan* p, ftk_mlp* m, const float* images, int nA, const void* tmpl_coeffs, int nB,
                       int kind, int n_r, int n_q, int topk, float tau, int32_t* best_t, ftk_pose* best_pose,
                       int32_t* fallback, int* n_fallback, void* stream) {
  if (!p || !m) return fail(FTK_EINVAL, "ftk_align_proposed: NULL plan or network");
  if (n_fallback) *n_fallback = 0;
  if (nA < 0) return fail(FTK_EINVAL, "ftk_align_proposed: nA < 0");
  if (nB != m->n_t) return fail(FTK_EINVAL, "ftk_align_proposed: nB must equal the network's n_template");
  const long long nfeat = kind == FTK_FEATURES_CROSS ? 1LL * n_r * n_r * n_q : 1LL * n_r * n_q;
  if (nfeat != m->dims[0]) return fail(FTK_EINVAL, "ftk_align_proposed: the feature count must equal dims[0]");
  if (topk < 1 || topk > 64 || topk > nB) return fail(FTK_EINVAL, "ftk_align_proposed: topk out of range");
  if (p->N <= 0) return fail(FTK_ESTATE, "ftk_align_proposed: call ftk_set_shifts first");
  if (nA == 0) return FTK_OK;
  if (!images || !tmpl_coeffs || !best_t || !best_pose) return fail(FTK_EINVAL, "ftk_align_proposed: NULL buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t cb = static_cast<size_t>(8) * p->M * p->Qa;
  const size_t D0 = m->dims[0];
  if (m->coef.ensure(cb * nA) != hipSuccess || m->feat.ensure(D0 * nA * 4) != hipSuccess ||
      m->top.ensure(static_cast<size_t>(nA) * topk * 4) != hipSuccess || m->mass.ensure(nA * 4ull) != hipSuccess ||
      m->sbin.ensure(nA * 4ull) != hipSuccess || m->pair_poses.ensure(static_cast<size_t>(nA) * topk * 12) != hipSuccess ||
      m->flist.ensure(nA * 4ull) != hipSuccess || m->fcount.ensure(16) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_align_proposed: workspace");
  const bool win = !p->windows.empty();
  if (win && static_cast<int>(p->windows.size()) != m->n_s)
    return fail(FTK_EINVAL, "ftk_align_proposed: the plan's shift windows must match the network's shift bins");
  int rc = ftk_transform(p, images, nA, m->coef.ptr, stream);
  if (rc == FTK_OK) rc = ftk_features(p, m->coef.ptr, nA, kind, n_r, n_q, m->feat.as<float>(), stream);
  if (rc == FTK_OK)
    rc = ftk_propose(m, m->feat.as<float>(), nA, topk, m->top.as<int32_t>(), m->mass.as<float>(),
                     m->sbin.as<int32_t>(), stream);
  if (rc == FTK_OK && !win)
    rc = ftk_align_lists(p, m->coef.ptr, nA, tmpl_coeffs, nB, m->top.as<int32_t>(), topk,
                         m->pair_poses.as<ftk_pose>(), stream);
  if (rc == FTK_OK && win) rc = align_windows(p, m, nA, tmpl_coeffs, nB, topk, tau, s);
  if (rc == FTK_OK)
    rc = ftk_best_template(m->pair_poses.as<ftk_pose>(), m->top.as<int32_t>(), nA, topk, best_t, best_pose, stream);
  if (rc != FTK_OK) return rc;
  hipError_t e = launch_select_below(m->mass.as<float>(), nA, tau, m->flist.as<int32_t>(), m->fcount.as<int32_t>(),
                                     fallback, s);
  if (e != hipSuccess) return hip_fail(e, "ftk_align_proposed: select");
  int32_t cnt = 0;
  if ((e = hipMemcpyAsync(&cnt, m->fcount.ptr, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "ftk_align_proposed: count");
  if (n_fallback) *n_fallback = cnt;
  if (cnt == 0) return FTK_OK;
  if (m->fcoef.ensure(cb * cnt) != hipSuccess || m->fposes.ensure(static_cast<size_t>(cnt) * nB * 12) != hipSuccess ||
      m->fbt.ensure(cnt * 4ull) != hipSuccess || m->fbp.ensure(cnt * 12ull) != hipSuccess)
    return fail(FTK_ENOMEM, "ftk_align_proposed: fallback workspace");
  if ((e = launch_gather_rows(m->coef.ptr, m->flist.as<int32_t>(), cnt, cb, m->fcoef.ptr, s)) != hipSuccess)
    return hip_fail(e, "ftk_align_proposed: gather");
  rc = ftk_align_coeffs(p, m->fcoef.ptr, cnt, tmpl_coeffs, nB, nullptr, m->fposes.as<ftk_pose>(), stream);
  if (rc == FTK_OK)
    rc = ftk_best_template(m->fposes.as<ftk_pose>(), nullptr, cnt, nB, m->fbt.as<int32_t>(), m->fbp.as<ftk_pose>(),
                           stream);
  if (rc != FTK_OK) return rc;
  if ((e = launch_scatter_results(m->fbt.as<int32_t>(), m->fbp.ptr, m->flist.as<int32_t>(), cnt, best_t, best_pose,
                                  s)) != hipSuccess)
    return hip_fail(e, "ftk_align_proposed: scatter");
  return FTK_OK;
}

}  // extern "C"
